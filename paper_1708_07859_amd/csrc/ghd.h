// Generalized hypertree decompositions: planning and bottom-up execution
// (sections 2.3 and 3.2).
#pragma once

#include <vector>

#include "lh_internal.h"

namespace lh {

struct GhdNode {
  uint32_t edges = 0;   // hyperedges evaluated in this node
  uint32_t attrs = 0;   // chi: union of the edges' attributes
  int32_t parent = -1;
  bool pushed = false;  // a selection node: one filtered edge of its parent
  double fhw = 0.0;     // fractional edge cover number of attrs by edges
};

struct Ghd {
  std::vector<GhdNode> nodes;  // node 0 is the root; parent[t] < t
  double fhw = 0.0;
  uint32_t depth = 0, shared = 0, sel_depth = 0;
};

// Least fractional edge cover of the attributes of the edges in `bag`, by
// those edges (edge_attrs: attribute mask per edge).
double fractional_cover(const std::vector<uint32_t>& edge_attrs, uint32_t bag);

// The decomposition of least width, broken by the tie-breaks of section
// 3.2, compressed to one node at width 1, selections pushed down.  The root
// holds every edge in root_edges and every attribute in out_mask.
Ghd choose_ghd(const std::vector<uint32_t>& edge_attrs, uint32_t sel_edges, uint32_t root_edges,
               uint32_t out_mask);

// Validate a caller's decomposition of the same hypergraph and fill in its
// derived quantities (attrs, widths, depth, shared, sel_depth).
void check_ghd(const std::vector<uint32_t>& edge_attrs, uint32_t sel_edges, uint32_t root_edges, uint32_t out_mask,
               Ghd& g);

// Run a query under a checked decomposition; returns a tracked result.
lh_result* run_ghd(const lh_query* q, const Ghd& g, hipStream_t s);

}  // namespace lh
