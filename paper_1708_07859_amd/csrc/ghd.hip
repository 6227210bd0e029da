// Multi-node query plans: generalized hypertree decompositions (section
// 2.3, "Generalized Hypertree Decompositions"; section 3.2).
//
// Planning (host only):
//  - the fractional hypertree width of a node is the fractional edge cover
//    number of its attributes by its own hyperedges, found through the dual
//    LP (a fractional vertex packing) by a small simplex;
//  - decompositions assign every hyperedge to exactly one node, the node's
//    attributes being the union of its edges' attributes; all of them are
//    enumerated by choosing a root bag and decomposing each component of the
//    remaining edges (connected through attributes outside the bag) under a
//    child whose bag holds the component's interface with the root, which
//    keeps the running-intersection property;
//  - among the decompositions of least width, section 3.2's tie-breaks
//    pick: fewest nodes, least depth, fewest vertices shared between
//    adjacent nodes, deepest selections; a last tie-break of this library
//    puts wide nodes nearer the root (least sum of width x depth); a chosen
//    decomposition of width 1 is compressed into one node (section 2.3);
//  - selections are pushed down (section 3.2): a filtered edge in a node of
//    several edges gets a child node holding it alone.
//
// Execution runs the nodes bottom-up through the public entry points.  A
// node joins its edges and its children's results, grouped by the
// attributes it shares with its parent (the root: by the query's outputs),
// and hands up two weights per group (the semiring view of section 2.3):
// the number of full-join tuples below it and, for SUM, the sum of their
// annotation products.  A selection node is the filtered copy of its edge,
// which the node's plan makes (the selection pre-pass).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "engine.h"
#include "exact.h"
#include "ghd.h"

namespace lh {

namespace {

constexpr double FHW_EPS = 1e-9;

inline uint32_t popcount(uint32_t x) { return (uint32_t)__builtin_popcount(x); }

}  // namespace

double fractional_cover(const std::vector<uint32_t>& edge_attrs, uint32_t bag) {
  // max sum_v y_v  s.t.  sum_{v in e} y_v <= 1 for e in bag, y >= 0.  Its
  // optimum equals the least fractional edge cover of the bag's attributes
  // by the bag's edges (LP duality).  Primal simplex from the slack basis,
  // Bland's rule against cycling.
  std::vector<uint32_t> E, V;
  uint32_t chi = 0;
  for (uint32_t e = 0; e < edge_attrs.size(); e++)
    if (bag >> e & 1u) {
      E.push_back(e);
      chi |= edge_attrs[e];
    }
  for (uint32_t v = 0; v < 32; v++)
    if (chi >> v & 1u) V.push_back(v);
  const int m = (int)E.size(), nv = (int)V.size(), n = nv + m;
  if (m == 0 || nv == 0) return 0.0;
  std::vector<double> T((size_t)m * (n + 1), 0.0), r(n, 0.0);
  std::vector<int> basis(m);
  auto at = [&](int i, int j) -> double& { return T[(size_t)i * (n + 1) + j]; };
  for (int i = 0; i < m; i++) {
    for (int j = 0; j < nv; j++) at(i, j) = (edge_attrs[E[i]] >> V[j] & 1u) ? 1.0 : 0.0;
    at(i, nv + i) = 1.0;
    at(i, n) = 1.0;
    basis[i] = nv + i;
  }
  for (int j = 0; j < nv; j++) r[j] = 1.0;
  double z = 0.0;
  for (int it = 0; it < 1000; it++) {
    int enter = -1;
    for (int j = 0; j < n; j++)
      if (r[j] > FHW_EPS) {
        enter = j;
        break;
      }
    if (enter < 0) break;
    int leave = -1;
    double best = 0.0;
    for (int i = 0; i < m; i++) {
      const double a = at(i, enter);
      if (a <= FHW_EPS) continue;
      const double q = at(i, n) / a;
      if (leave < 0 || q < best - FHW_EPS || (q <= best + FHW_EPS && basis[i] < basis[leave])) {
        leave = i;
        best = q;
      }
    }
    if (leave < 0) fail(LH_ERR_DEVICE, "ghd: unbounded vertex packing");  // every attribute lies in an edge
    const double piv = at(leave, enter);
    for (int j = 0; j <= n; j++) at(leave, j) /= piv;
    for (int i = 0; i < m; i++) {
      if (i == leave) continue;
      const double f = at(i, enter);
      if (f == 0.0) continue;
      for (int j = 0; j <= n; j++) at(i, j) -= f * at(leave, j);
    }
    const double f = r[enter];
    for (int j = 0; j < n; j++) r[j] -= f * at(leave, j);
    z += f * at(leave, n);
    basis[leave] = enter;
  }
  return z;
}

namespace {

struct Sub {                       // a decomposition of one subproblem, rooted
  double fhw = 0.0;
  uint32_t nodes = 0, depth = 0, shared = 0, sel = 0;
  double wsum = 0.0, wdepth = 0.0;  // sum of node widths; sum of width x depth
  std::vector<uint32_t> bag;       // node edge masks, node 0 = this root
  std::vector<int32_t> parent;     // local parent index, -1 for node 0
};

// a is at least as good as b in every tie-break quantity
bool covers(const Sub& a, const Sub& b) {
  return a.fhw <= b.fhw + FHW_EPS && a.nodes <= b.nodes && a.depth <= b.depth && a.shared <= b.shared &&
         a.sel >= b.sel && a.wsum <= b.wsum + FHW_EPS && a.wdepth <= b.wdepth + FHW_EPS;
}

// Lexicographic order of section 3.2: width, nodes, depth, shared vertices,
// the deeper selections; then wide nodes nearer the root (least sum of
// width x depth): nodes run bottom-up, so a child's result restricts its
// parent's join, and a narrow node below a wide one filters the expensive
// join instead of the reverse.
bool better(const Sub& a, const Sub& b) {
  if (a.fhw < b.fhw - FHW_EPS) return true;
  if (a.fhw > b.fhw + FHW_EPS) return false;
  if (a.nodes != b.nodes) return a.nodes < b.nodes;
  if (a.depth != b.depth) return a.depth < b.depth;
  if (a.shared != b.shared) return a.shared < b.shared;
  if (a.sel != b.sel) return a.sel > b.sel;
  return a.wdepth < b.wdepth - FHW_EPS;
}

struct Enumerator {
  const std::vector<uint32_t>& ea;  // attribute mask per edge
  uint32_t sel_edges, root_edges, out_mask;
  std::map<uint32_t, double> fhw_memo;
  std::map<uint64_t, std::vector<Sub>> memo;

  Enumerator(const std::vector<uint32_t>& e, uint32_t s, uint32_t r, uint32_t o)
      : ea(e), sel_edges(s), root_edges(r), out_mask(o) {}

  uint32_t chi(uint32_t edges) const {
    uint32_t c = 0;
    for (uint32_t e = 0; e < ea.size(); e++)
      if (edges >> e & 1u) c |= ea[e];
    return c;
  }

  double fhw(uint32_t bag) {
    auto it = fhw_memo.find(bag);
    if (it != fhw_memo.end()) return it->second;
    const double f = fractional_cover(ea, bag);
    fhw_memo[bag] = f;
    return f;
  }

  // Components of `rest` connected through attributes outside `sep`.
  std::vector<uint32_t> components(uint32_t rest, uint32_t sep) const {
    std::vector<uint32_t> out;
    while (rest) {
      uint32_t comp = rest & (~rest + 1u);
      for (bool grew = true; grew;) {
        grew = false;
        const uint32_t reach = chi(comp) & ~sep;
        for (uint32_t e = 0; e < ea.size(); e++)
          if ((rest >> e & 1u) && !(comp >> e & 1u) && (ea[e] & reach)) {
            comp |= 1u << e;
            grew = true;
          }
      }
      out.push_back(comp);
      rest &= ~comp;
    }
    return out;
  }

  static void add_pareto(std::vector<Sub>& set, Sub&& c) {
    for (const Sub& s : set)
      if (covers(s, c)) return;
    set.erase(std::remove_if(set.begin(), set.end(), [&](const Sub& s) { return covers(c, s); }), set.end());
    set.push_back(std::move(c));
  }

  // Pareto-optimal decompositions of `edges` whose root bag holds `need`.
  const std::vector<Sub>& solve(uint32_t edges, uint32_t need, bool top) {
    const uint64_t key = (uint64_t)edges << 32 | need | (top ? 1ull << 31 : 0ull);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    std::vector<Sub> best;
    // every non-empty bag B of the edges, largest mask first
    for (uint32_t B = edges; B; B = (B - 1) & edges) {
      const uint32_t cb = chi(B);
      if ((cb & need) != need) continue;
      if (top && ((B & root_edges) != root_edges || (cb & out_mask) != out_mask)) continue;
      const std::vector<uint32_t> comps = components(edges & ~B, cb);
      const double fb = fhw(B);
      // Each child subtree holds one or more whole components (an attribute
      // outside B cannot span two subtrees): every grouping of the
      // components, as a restricted growth string.
      const size_t nc = comps.size();
      std::vector<uint32_t> grp(nc, 0);
      for (;;) {
        uint32_t ng = 0;
        for (size_t c = 0; c < nc; c++) ng = std::max(ng, grp[c] + 1);
        std::vector<uint32_t> gm(ng, 0), iface(ng, 0);
        for (size_t c = 0; c < nc; c++) gm[grp[c]] |= comps[c];
        bool ok = true;
        for (uint32_t k = 0; k < ng; k++) {
          iface[k] = chi(gm[k]) & cb;
          if (!iface[k]) ok = false;  // a disconnected part has nothing to hand up
        }
        if (ok) {
          std::vector<const std::vector<Sub>*> kids(ng);
          for (uint32_t k = 0; k < ng; k++) kids[k] = &solve(gm[k], iface[k], false);
          // cartesian product of the children's Pareto sets
          std::vector<size_t> pick(ng, 0);
          for (;;) {
            Sub sb;
            sb.fhw = fb;
            sb.wsum = fb;
            sb.nodes = 1;
            sb.bag.push_back(B);
            sb.parent.push_back(-1);
            for (uint32_t k = 0; k < ng; k++) {
              const Sub& kd = (*kids[k])[pick[k]];
              sb.fhw = std::max(sb.fhw, kd.fhw);
              sb.nodes += kd.nodes;
              sb.depth = std::max(sb.depth, kd.depth + 1);
              sb.shared += kd.shared + popcount(iface[k]);
              sb.sel += kd.sel + popcount(gm[k] & sel_edges);
              sb.wsum += kd.wsum;
              sb.wdepth += kd.wdepth + kd.wsum;
              const int32_t base = (int32_t)sb.bag.size();
              for (size_t j = 0; j < kd.bag.size(); j++) {
                sb.bag.push_back(kd.bag[j]);
                sb.parent.push_back(kd.parent[j] < 0 ? 0 : kd.parent[j] + base);
              }
            }
            add_pareto(best, std::move(sb));
            uint32_t k = 0;
            for (; k < ng; k++) {
              if (++pick[k] < kids[k]->size()) break;
              pick[k] = 0;
            }
            if (k == ng) break;
          }
        }
        // next restricted growth string: grp[c] <= 1 + max(grp[0..c-1])
        size_t c = nc;
        while (c-- > 1) {
          uint32_t mx = 0;
          for (size_t j = 0; j < c; j++) mx = std::max(mx, grp[j]);
          if (grp[c] <= mx) {
            grp[c]++;
            for (size_t j = c + 1; j < nc; j++) grp[j] = 0;
            break;
          }
        }
        if (c == 0 || c == (size_t)-1 || nc <= 1) break;
      }
    }
    return memo[key] = std::move(best);
  }
};

}  // namespace

Ghd choose_ghd(const std::vector<uint32_t>& edge_attrs, uint32_t sel_edges, uint32_t root_edges,
               uint32_t out_mask) {
  const uint32_t ne = (uint32_t)edge_attrs.size();
  if (ne == 0 || ne > 8) fail(LH_ERR_INVALID, "ghd: 1..8 hyperedges");
  const uint32_t all = (ne == 32) ? ~0u : ((1u << ne) - 1u);
  Enumerator en(edge_attrs, sel_edges, root_edges, out_mask);
  const std::vector<Sub>& cands = en.solve(all, 0, true);
  if (cands.empty()) fail(LH_ERR_DEVICE, "ghd: no decomposition");
  const Sub* pick = &cands[0];
  for (const Sub& c : cands)
    if (better(c, *pick)) pick = &c;
  Sub chosen = *pick;
  if (chosen.fhw <= 1.0 + FHW_EPS && chosen.nodes > 1) {
    // width 1: one generic-join node is as good (section 2.3)
    Sub one;
    one.fhw = en.fhw(all);
    one.nodes = 1;
    one.bag.push_back(all);
    one.parent.push_back(-1);
    chosen = one;
  }
  // breadth-first numbering: parents before children
  Ghd g;
  std::vector<int32_t> newid(chosen.bag.size(), -1);
  std::vector<uint32_t> queue{0};
  newid[0] = 0;
  for (size_t h = 0; h < queue.size(); h++) {
    const uint32_t u = queue[h];
    for (uint32_t v = 0; v < chosen.bag.size(); v++)
      if (chosen.parent[v] == (int32_t)u) {
        newid[v] = (int32_t)queue.size();
        queue.push_back(v);
      }
  }
  for (uint32_t u : queue) {
    GhdNode n;
    n.edges = chosen.bag[u];
    n.attrs = en.chi(n.edges);
    n.parent = chosen.parent[u] < 0 ? -1 : newid[chosen.parent[u]];
    n.fhw = en.fhw(n.edges);
    g.nodes.push_back(n);
  }
  // depth of every node, selection depth, shared vertices
  std::vector<uint32_t> dep(g.nodes.size(), 0);
  for (size_t t = 1; t < g.nodes.size(); t++) dep[t] = dep[g.nodes[t].parent] + 1;
  g.fhw = 0.0;
  for (const GhdNode& n : g.nodes) g.fhw = std::max(g.fhw, n.fhw);
  for (size_t t = 0; t < g.nodes.size(); t++) {
    g.depth = std::max(g.depth, dep[t]);
    if (t) g.shared += popcount(g.nodes[t].attrs & g.nodes[g.nodes[t].parent].attrs);
    g.sel_depth += dep[t] * popcount(g.nodes[t].edges & sel_edges);
  }
  // selection push-down (section 3.2)
  const size_t base_nodes = g.nodes.size();
  for (size_t t = 0; t < base_nodes; t++) {
    if (popcount(g.nodes[t].edges) < 2) continue;
    for (uint32_t e = 0; e < ne; e++)
      if ((g.nodes[t].edges >> e & 1u) && (sel_edges >> e & 1u)) {
        GhdNode n;
        n.edges = 1u << e;
        n.attrs = edge_attrs[e];
        n.parent = (int32_t)t;
        n.pushed = true;
        n.fhw = 1.0;
        g.nodes.push_back(n);
      }
  }
  if (g.nodes.size() > LH_GHD_MAX_NODES) fail(LH_ERR_UNSUPPORTED, "ghd: more than 16 nodes");
  return g;
}

void check_ghd(const std::vector<uint32_t>& edge_attrs, uint32_t sel_edges, uint32_t root_edges, uint32_t out_mask,
               Ghd& g) {
  const uint32_t ne = (uint32_t)edge_attrs.size();
  const size_t nn = g.nodes.size();
  if (nn == 0 || nn > LH_GHD_MAX_NODES) fail(LH_ERR_INVALID, "ghd: 1..16 nodes");
  if (g.nodes[0].parent != -1 || g.nodes[0].pushed) fail(LH_ERR_INVALID, "ghd: node 0 must be the root");
  uint32_t seen = 0;
  auto chi = [&](uint32_t edges) {
    uint32_t c = 0;
    for (uint32_t e = 0; e < ne; e++)
      if (edges >> e & 1u) c |= edge_attrs[e];
    return c;
  };
  for (size_t t = 0; t < nn; t++) {
    GhdNode& n = g.nodes[t];
    if (t && (n.parent < 0 || n.parent >= (int32_t)t)) fail(LH_ERR_INVALID, "ghd: parent[t] must be below t");
    if (!n.edges || (ne < 32 && (n.edges >> ne))) fail(LH_ERR_INVALID, "ghd: node edge set empty or out of range");
    n.attrs = chi(n.edges);
    if (n.pushed) {
      const GhdNode& p = g.nodes[n.parent];
      if (popcount(n.edges) != 1 || !(n.edges & sel_edges) || !(p.edges & n.edges) || p.pushed)
        fail(LH_ERR_INVALID, "ghd: a selection node holds one filtered edge of its parent");
      continue;
    }
    if (t && g.nodes[n.parent].pushed) fail(LH_ERR_INVALID, "ghd: a selection node has no children");
    if (seen & n.edges) fail(LH_ERR_INVALID, "ghd: an edge in two nodes");
    seen |= n.edges;
    if (t && !(n.attrs & g.nodes[n.parent].attrs)) fail(LH_ERR_INVALID, "ghd: a node shares nothing with its parent");
  }
  if (seen != ((1u << ne) - 1u)) fail(LH_ERR_INVALID, "ghd: an edge in no node");
  if ((g.nodes[0].edges & root_edges) != root_edges || (g.nodes[0].attrs & out_mask) != out_mask)
    fail(LH_ERR_INVALID, "ghd: the root must hold the output attributes and the GROUP BY relations");
  // running intersection: the nodes holding an attribute form a subtree,
  // i.e. exactly one of them has a parent without it
  for (uint32_t v = 0; v < 32; v++) {
    uint32_t tops = 0, holders = 0;
    for (size_t t = 0; t < nn; t++) {
      const GhdNode& n = g.nodes[t];
      if (n.pushed || !(n.attrs >> v & 1u)) continue;
      holders++;
      if (t == 0 || !(g.nodes[n.parent].attrs >> v & 1u)) tops++;
    }
    if (holders && tops != 1) fail(LH_ERR_INVALID, "ghd: running intersection property violated");
  }
  // derived quantities
  std::vector<uint32_t> dep(nn, 0);
  g.fhw = 0.0;
  g.depth = g.shared = g.sel_depth = 0;
  for (size_t t = 0; t < nn; t++) {
    GhdNode& n = g.nodes[t];
    if (t) dep[t] = dep[n.parent] + (n.pushed ? 0 : 1);
    n.fhw = fractional_cover(edge_attrs, n.edges);
    if (n.pushed) continue;
    g.fhw = std::max(g.fhw, n.fhw);
    g.depth = std::max(g.depth, dep[t]);
    if (t) g.shared += popcount(n.attrs & g.nodes[n.parent].attrs);
    g.sel_depth += dep[t] * popcount(n.edges & sel_edges);
  }
}

// ---------------------------------------------------------------------------
// execution
// ---------------------------------------------------------------------------

namespace {

__global__ void k_u64_to_f64(const uint64_t* in, double* out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

// Weighted counts come back as exactly rounded sums of integers; below 2^53
// they are the exact integers.
__global__ void k_f64_to_u64(const double* in, uint64_t* out, uint64_t n, uint32_t* err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = in[i];
  if (!(v >= 0.0 && v < 9007199254740992.0)) {
    atomicOr(err, 1u);
    out[i] = 0;
    return;
  }
  out[i] = (uint64_t)v;
}

unsigned grid1(uint64_t n) { return (unsigned)((n + 255) / 256); }

// Non-zero exact parts of each group's sum (at least one per group, so the
// group stays present with its count weight).
__global__ void k_count_parts(const double* parts, uint64_t n, uint32_t* cnt) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c = 1;
  for (int k = 1; k < EXACT_PARTS; k++) c += parts[i * EXACT_PARTS + k] != 0.0 ? 1u : 0u;
  cnt[i] = c;
}

struct ExpandArgs {
  uint32_t n_cols;
  const uint32_t* key_in[MAXV];
  uint32_t* key_out[MAXV];
  const double* wc;       // count weight of each group
  const double* parts;    // EXACT_PARTS per group
  const uint64_t* off;    // first output row of each group
  double* wc_out;
  double* part_out;
};

// One row per non-zero part: the group's keys, its count weight on the
// first row (0 on the others), and the part.  The parts are non-zero in
// order, so a group's rows are its first parts.
__global__ void k_expand_parts(ExpandArgs a, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t o = a.off[i], m = a.off[i + 1] - o;
  for (uint64_t k = 0; k < m; k++) {
    for (uint32_t c = 0; c < a.n_cols; c++) a.key_out[c][o + k] = a.key_in[c][i];
    a.wc_out[o + k] = k == 0 ? a.wc[i] : 0.0;
    a.part_out[o + k] = a.parts[i * EXACT_PARTS + k];
  }
}

void check(lh_status st) {
  if (st != LH_OK) fail(st, std::string("ghd node: ") + lh_last_error());
}

// One node's outcome: the group keys with the two weights.
struct NodeOut {
  lh_result* a = nullptr;      // counts run
  lh_result* b = nullptr;      // SUM run (nullptr: weights equal the counts)
  DBuf<double> wcount;         // count weight per row (when a holds plain counts)
  lh_trie* trie = nullptr;     // the intermediate relation handed to the parent
  std::vector<uint32_t> keys;  // its key attributes (global ids, ascending)
  bool has_anno = false;       // an annotated atom lies in this subtree
  // the relation's rows when each sum is handed up as its exact parts
  std::vector<DBuf<uint32_t>> ekeys;
  DBuf<double> ewc, epart;
};

struct Owned {  // frees everything made on the way, also on errors
  std::vector<void*> h;
  ~Owned() {
    for (void* p : h) lh_free(p);
  }
};

}  // namespace

lh_result* run_ghd(const lh_query* q, const Ghd& g, hipStream_t s) {
  const size_t nn = g.nodes.size();
  std::vector<NodeOut> out(nn);
  Owned own;
  const bool is_sum = q->agg == LH_AGG_SUM;
  for (size_t ti = nn; ti-- > 0;) {
    const GhdNode& node = g.nodes[ti];
    if (node.pushed) continue;  // realised as the filtered copy in its parent's plan
    const bool root = ti == 0;
    std::vector<uint32_t> kids;
    for (size_t c = ti + 1; c < nn; c++)
      if (g.nodes[c].parent == (int32_t)ti && !g.nodes[c].pushed) kids.push_back((uint32_t)c);
    // local attribute ids: the node's attributes in ascending global order
    uint32_t loc[32];
    uint32_t nl = 0;
    for (uint32_t v = 0; v < 32; v++) loc[v] = (node.attrs >> v & 1u) ? nl++ : UINT32_MAX;
    bool has_anno = false;
    for (uint32_t e = 0; e < q->n_atoms; e++)
      if ((node.edges >> e & 1u) && q->atoms[e].anno >= 0) has_anno = true;
    for (uint32_t c : kids) has_anno = has_anno || out[c].has_anno;
    out[ti].has_anno = has_anno;

    std::vector<std::vector<uint32_t>> amaps;
    std::vector<lh_atom> atoms;
    std::vector<uint32_t> atom_of_edge(q->n_atoms, UINT32_MAX);
    for (uint32_t e = 0; e < q->n_atoms; e++) {
      if (!(node.edges >> e & 1u)) continue;
      const lh_atom& A = q->atoms[e];
      std::vector<uint32_t> m;
      for (uint32_t k = 0; k < A.trie->n_levels; k++) m.push_back(loc[A.attr_of_key[k]]);
      amaps.push_back(m);
      atom_of_edge[e] = (uint32_t)atoms.size();
      atoms.push_back(lh_atom{A.trie, nullptr, A.anno});
    }
    const size_t n_edge_atoms = atoms.size();
    for (uint32_t c : kids) {
      std::vector<uint32_t> m;
      for (uint32_t v : out[c].keys) m.push_back(loc[v]);
      amaps.push_back(m);
      atoms.push_back(lh_atom{out[c].trie, nullptr, 0});
    }
    for (size_t i = 0; i < atoms.size(); i++) atoms[i].attr_of_key = amaps[i].data();
    std::vector<lh_filter> filters;
    for (uint32_t f = 0; f < q->n_filters; f++)
      if (atom_of_edge[q->filters[f].atom] != UINT32_MAX) {
        lh_filter F = q->filters[f];
        F.atom = atom_of_edge[F.atom];
        filters.push_back(F);
      }
    std::vector<uint32_t> outs;
    std::vector<lh_group_col> groups;
    if (root) {
      for (uint32_t i = 0; i < q->n_out; i++) outs.push_back(loc[q->out_attrs[i]]);
      for (uint32_t i = 0; i < q->n_group; i++) {
        lh_group_col G = q->group_cols[i];
        G.atom = atom_of_edge[G.atom];
        groups.push_back(G);
      }
    } else {
      const uint32_t iface = node.attrs & g.nodes[node.parent].attrs;
      for (uint32_t v = 0; v < 32; v++)
        if (iface >> v & 1u) {
          outs.push_back(loc[v]);
          out[ti].keys.push_back(v);
        }
    }
    std::vector<uint32_t> order;
    if (q->attr_order)
      for (uint32_t i = 0; i < q->n_attrs; i++)
        if (loc[q->attr_order[i]] != UINT32_MAX) order.push_back(loc[q->attr_order[i]]);

    auto run = [&](bool sum_run) -> lh_result* {
      std::vector<lh_atom> at = atoms;
      for (size_t i = 0; i < at.size(); i++) {
        if (i < n_edge_atoms) {
          if (!sum_run) at[i].anno = -1;
        } else {
          const NodeOut& k = out[kids[i - n_edge_atoms]];
          at[i].anno = (sum_run && k.has_anno) ? 1 : 0;
        }
      }
      lh_query nq{};
      nq.n_attrs = nl;
      nq.n_atoms = (uint32_t)at.size();
      nq.atoms = at.data();
      nq.n_out = (uint32_t)outs.size();
      nq.out_attrs = outs.data();
      nq.n_group = (uint32_t)groups.size();
      nq.group_cols = groups.data();
      nq.agg = (sum_run || !kids.empty()) ? LH_AGG_SUM : LH_AGG_COUNT;
      nq.n_filters = (uint32_t)filters.size();
      nq.filters = filters.data();
      nq.attr_order = q->attr_order ? order.data() : nullptr;
      nq.policy = q->policy;
      lh_plan_t* p = nullptr;
      check(lh_plan(&nq, s, &p));
      own.h.push_back(p);
      // a child's sums go up as exact parts, so the parent sums exactly
      if (sum_run && !root) p->want_parts = true;
      lh_result* r = nullptr;
      check(lh_join_aggregate(&p, 1, s, &r));
      own.h.push_back(r);
      return r;
    };
    NodeOut& o = out[ti];
    const bool sum_needed = is_sum && has_anno;
    if (kids.empty()) {
      // one run gives both: its counts are the tuples, its sums the products
      o.a = run(sum_needed);
      o.b = sum_needed ? o.a : nullptr;
    } else {
      o.a = run(false);
      o.b = sum_needed ? run(true) : nullptr;
    }
    const uint64_t nr = o.a->n_rows;
    if (o.b && o.b->n_rows != nr) fail(LH_ERR_DEVICE, "ghd: the two runs of a node disagree on its groups");
    const double* wc = o.a->sums;
    if (kids.empty()) {
      o.wcount.alloc(nr, s);
      if (nr) k_u64_to_f64<<<grid1(nr), 256, 0, s>>>(o.a->counts, o.wcount.p, nr);
      LH_HIP(hipGetLastError());
      wc = o.wcount.p;
    }
    if (!root) {
      const double* annos[2] = {wc, o.b ? o.b->sums : wc};
      lh_relation_desc rel{};
      rel.n_rows = nr;
      rel.n_keys = o.a->n_cols;
      rel.keys = o.a->out_keys;
      rel.n_annos = 2;
      rel.annos = annos;
      rel.flags = LH_BAG | LH_LAYOUT_PLAIN;
      std::vector<const uint32_t*> ekp;
      const lh_result_impl* rb = o.b ? reinterpret_cast<const lh_result_impl*>(o.b) : nullptr;
      if (rb && rb->parts.p && nr) {
        // one bag row per non-zero exact part of each group's sum
        if (o.a->n_cols > MAXV) fail(LH_ERR_UNSUPPORTED, "ghd: too many interface attributes");
        DBuf<uint32_t> cnt(nr, s);
        DBuf<uint64_t> off(nr + 1, s);
        k_count_parts<<<grid1(nr), 256, 0, s>>>(rb->parts.p, nr, cnt.p);
        LH_HIP(hipGetLastError());
        const uint64_t m = scan_u32_to_u64(cnt.p, off.p, nr, s);
        ExpandArgs ea{};
        ea.n_cols = o.a->n_cols;
        o.ekeys.resize(ea.n_cols);
        for (uint32_t c = 0; c < ea.n_cols; c++) {
          o.ekeys[c].alloc(m, s);
          ea.key_in[c] = o.a->out_keys[c];
          ea.key_out[c] = o.ekeys[c].p;
          ekp.push_back(o.ekeys[c].p);
        }
        o.ewc.alloc(m, s);
        o.epart.alloc(m, s);
        ea.wc = wc;
        ea.parts = rb->parts.p;
        ea.off = off.p;
        ea.wc_out = o.ewc.p;
        ea.part_out = o.epart.p;
        k_expand_parts<<<grid1(nr), 256, 0, s>>>(ea, nr);
        LH_HIP(hipGetLastError());
        annos[0] = o.ewc.p;
        annos[1] = o.epart.p;
        rel.n_rows = m;
        rel.keys = ekp.data();
      }
      check(lh_trie_build(&rel, s, &o.trie));
      own.h.push_back(o.trie);
    }
  }
  // the root's outcome becomes the result: its keys, the weighted counts and
  // the SUM run's sums
  NodeOut& R = out[0];
  lh_result_impl* res = reinterpret_cast<lh_result_impl*>(R.a);
  const uint64_t nr = R.a->n_rows;
  bool has_kids = false;
  for (size_t c = 1; c < nn; c++) has_kids = has_kids || (g.nodes[c].parent == 0 && !g.nodes[c].pushed);
  if (has_kids) {
    DBuf<uint64_t> cnt(nr, s);
    DBuf<uint32_t> err(1, s);
    fill_u32(err.p, 0, 1, s);
    if (nr) k_f64_to_u64<<<grid1(nr), 256, 0, s>>>(R.a->sums, cnt.p, nr, err.p);
    LH_HIP(hipGetLastError());
    if (read_scalar(err.p, s)) fail(LH_ERR_OVERFLOW, "ghd: a group's count reaches 2^53");
    res->counts = std::move(cnt);
  }
  if (R.b != R.a) {
    res->sums.reset();
    if (R.b) res->sums = std::move(reinterpret_cast<lh_result_impl*>(R.b)->sums);
  }
  res->pub.counts = res->counts.p;
  res->pub.sums = is_sum ? res->sums.p : nullptr;
  // Children hand their sums up as exact parts, and a term of two factors
  // is an exact product: with at most two annotated atoms in the query
  // every node's terms are those of the single plan, so the root's sums are
  // its correctly rounded exact sums.  More factors are rounded per node.
  uint32_t n_annotated = 0;
  for (uint32_t e = 0; e < q->n_atoms; e++) n_annotated += q->atoms[e].anno >= 0 ? 1u : 0u;
  bool all_exact = R.b && R.b->exact;
  for (size_t c = 1; c < nn; c++)
    if (out[c].b) all_exact = all_exact && out[c].b->exact;
  res->pub.exact = (is_sum && all_exact && (!has_kids || n_annotated <= 2)) ? 1u : 0u;
  uint64_t nj = 0;
  if (nr) {
    std::vector<uint64_t> h(nr);
    LH_HIP(hipMemcpyAsync(h.data(), res->counts.p, nr * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
    for (uint64_t v : h) nj += v;
  }
  res->pub.n_join_tuples = nj;
  // hand the root's result out; everything else is freed
  own.h.erase(std::find(own.h.begin(), own.h.end(), (void*)R.a));
  LH_HIP(hipStreamSynchronize(s));
  return R.a;
}

}  // namespace lh
