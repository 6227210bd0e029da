// The cost estimate of section 4 ("Cost-Based Optimizer"): for an attribute
// order [v_0, ..., v_{n-1}], cost = SUM_i icost(v_i) * weight(v_i).
#pragma once

#include <stdint.h>

#include <vector>

namespace lh {

struct Edge {
  std::vector<uint32_t> attrs;  // attributes of the relation
  uint64_t card = 0;            // relation cardinality (before filters)
  bool eq = false;              // an equality selection applies to the relation
  bool dense = false;           // completely dense: contributes no intersection
  // per attribute (aligned with attrs): log2 of the mean and the largest
  // number of rows sharing one value of that attribute's column
  std::vector<float> lf_mean, lf_max;
};

struct Hypergraph {
  uint32_t n_attrs = 0;
  std::vector<Edge> edges;
};

// Cost of one order; optionally the per-position icost and weight.
double order_cost(const Hypergraph& h, const std::vector<uint32_t>& order, uint32_t* icost, uint32_t* weight);

// Sum of icosts of an order (the quantity the relaxation rule compares).
uint32_t order_icost(const Hypergraph& h, const std::vector<uint32_t>& order);

// Cheapest order among those with the materialized attributes first, plus
// the one-swap relaxation of section 4.1.2; ties go to the lexicographically
// smallest order.  Returns its cost.
double choose_order(const Hypergraph& h, const std::vector<uint32_t>& out_attrs, std::vector<uint32_t>& order);

// Cardinality score of each edge: ceil(|r| / |r_heavy| * 100).
std::vector<uint32_t> edge_scores(const Hypergraph& h);

}  // namespace lh
