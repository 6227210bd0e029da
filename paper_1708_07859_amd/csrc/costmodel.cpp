// Section 4 cost estimate and order search (host code).
#include "costmodel.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace lh {

namespace {

enum Layout { BS = 0, UINT = 1 };

// icost of intersecting two sets of the given layouts (section 4.1.1):
// bs & bs = 1, bs & uint = 10, uint & uint = 50.
uint32_t pair_icost(Layout a, Layout b) {
  if (a == BS && b == BS) return 1;
  if (a == UINT && b == UINT) return 50;
  return 10;
}

// Layout of an intersection's result: only bs & bs stays a bitset.
Layout pair_layout(Layout a, Layout b) { return (a == BS && b == BS) ? BS : UINT; }

bool contains(const Edge& e, uint32_t v) { return std::find(e.attrs.begin(), e.attrs.end(), v) != e.attrs.end(); }

void per_vertex(const Hypergraph& h, const std::vector<uint32_t>& order, uint32_t* icost, uint32_t* weight) {
  const std::vector<uint32_t> score = edge_scores(h);
  std::vector<bool> seen(h.edges.size(), false);
  for (size_t i = 0; i < order.size(); i++) {
    const uint32_t v = order[i];
    // Crucial Observation 1: a relation's first trie level is guessed a
    // bitset, any later level a uint array.
    std::vector<Layout> ls;
    bool any_eq = false;
    uint32_t wmin = std::numeric_limits<uint32_t>::max(), wmax = 0;
    for (size_t e = 0; e < h.edges.size(); e++) {
      if (!contains(h.edges[e], v)) continue;
      if (!h.edges[e].dense) ls.push_back(seen[e] ? UINT : BS);
      any_eq = any_eq || h.edges[e].eq;
      wmin = std::min(wmin, score[e]);
      wmax = std::max(wmax, score[e]);
    }
    for (size_t e = 0; e < h.edges.size(); e++)
      if (contains(h.edges[e], v)) seen[e] = true;
    // N-way: sum of pairwise icosts, bitsets first
    std::sort(ls.begin(), ls.end());
    uint32_t c = 0;
    if (ls.size() >= 2) {
      Layout cur = ls[0];
      for (size_t j = 1; j < ls.size(); j++) {
        c += pair_icost(cur, ls[j]);
        cur = pair_layout(cur, ls[j]);
      }
    }
    if (icost) icost[i] = c;
    // Crucial Observation 2: heaviest edge under an equality selection,
    // otherwise the lightest edge.
    if (weight) weight[i] = (wmax == 0 && wmin == std::numeric_limits<uint32_t>::max()) ? 0 : (any_eq ? wmax : wmin);
  }
}

}  // namespace

std::vector<uint32_t> edge_scores(const Hypergraph& h) {
  uint64_t heavy = 0;
  for (auto& e : h.edges) heavy = std::max(heavy, e.card);
  std::vector<uint32_t> s(h.edges.size(), 0);
  for (size_t e = 0; e < h.edges.size(); e++) {
    if (heavy == 0) continue;
    // ceil(card * 100 / heavy) in integers
    s[e] = (uint32_t)((h.edges[e].card * 100 + heavy - 1) / heavy);
  }
  return s;
}

double order_cost(const Hypergraph& h, const std::vector<uint32_t>& order, uint32_t* icost, uint32_t* weight) {
  std::vector<uint32_t> ic(order.size()), w(order.size());
  per_vertex(h, order, ic.data(), w.data());
  double c = 0;
  for (size_t i = 0; i < order.size(); i++) c += (double)ic[i] * (double)w[i];
  if (icost) std::copy(ic.begin(), ic.end(), icost);
  if (weight) std::copy(w.begin(), w.end(), weight);
  return c;
}

uint32_t order_icost(const Hypergraph& h, const std::vector<uint32_t>& order) {
  std::vector<uint32_t> ic(order.size());
  per_vertex(h, order, ic.data(), nullptr);
  return std::accumulate(ic.begin(), ic.end(), 0u);
}

double choose_order(const Hypergraph& h, const std::vector<uint32_t>& out_attrs, std::vector<uint32_t>& order) {
  const uint32_t n = h.n_attrs;
  std::vector<bool> mat(n, false);
  for (uint32_t v : out_attrs) mat[v] = true;
  std::vector<uint32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0u);
  double best = std::numeric_limits<double>::infinity();
  std::vector<uint32_t> best_order = perm;
  auto consider = [&](const std::vector<uint32_t>& o) {
    double c = order_cost(h, o, nullptr, nullptr);
    if (c < best || (c == best && o < best_order)) {
      best = c;
      best_order = o;
    }
  };
  if (n > 9) {
    // too many orders to enumerate: materialized attributes first, each
    // group by descending edge count (a fixed, cheap fallback)
    std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) { return mat[a] > mat[b]; });
    order = perm;
    return order_cost(h, order, nullptr, nullptr);
  }
  do {
    // materialized attributes before projected-away ones
    bool ok = true;
    bool seen_proj = false;
    for (uint32_t v : perm) {
      if (!mat[v]) seen_proj = true;
      else if (seen_proj) { ok = false; break; }
    }
    if (!ok) continue;
    consider(perm);
    // relaxation (section 4.1.2): last projected, second-to-last
    // materialized, and the swap lowers the icost
    if (n >= 2 && !mat[perm[n - 1]] && mat[perm[n - 2]]) {
      std::vector<uint32_t> sw = perm;
      std::swap(sw[n - 1], sw[n - 2]);
      if (order_icost(h, sw) < order_icost(h, perm)) consider(sw);
    }
  } while (std::next_permutation(perm.begin(), perm.end()));
  order = best_order;
  return best;
}

}  // namespace lh
