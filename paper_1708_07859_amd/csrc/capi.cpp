// The C ABI: validation of descriptors, handle bookkeeping and the mapping
// of internal errors to lh_status.  No exception crosses this boundary.
#include <cstring>
#include <mutex>
#include <set>

#include "costmodel.h"
#include "engine.h"
#include "ghd.h"

namespace lh {

namespace {

thread_local std::string g_last_error;

std::mutex g_mu;
std::set<const void*> g_tries, g_plans, g_results;

void track(std::set<const void*>& s, const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  s.insert(p);
}

bool untrack(std::set<const void*>& s, const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return s.erase(p) != 0;
}

bool tracked(const std::set<const void*>& s, const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return s.count(p) != 0;
}

template <class F>
lh_status guard(F&& f) {
  try {
    f();
    g_last_error.clear();
    return LH_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LH_ERR_OOM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return LH_ERR_DEVICE;
  }
}

Hypergraph hypergraph_from(const lh_hypergraph* h) {
  if (!h || !h->edge_attr_count || !h->edge_attrs || !h->edge_card) fail(LH_ERR_INVALID, "hypergraph is incomplete");
  if (h->n_attrs == 0 || h->n_attrs > MAXV) fail(LH_ERR_INVALID, "n_attrs must be 1..16");
  Hypergraph g;
  g.n_attrs = h->n_attrs;
  uint32_t k = 0;
  for (uint32_t e = 0; e < h->n_edges; e++) {
    Edge E;
    for (uint32_t i = 0; i < h->edge_attr_count[e]; i++) {
      uint32_t v = h->edge_attrs[k++];
      if (v >= h->n_attrs) fail(LH_ERR_INVALID, "edge attribute out of range");
      E.attrs.push_back(v);
    }
    E.card = h->edge_card[e];
    E.eq = h->edge_eq && h->edge_eq[e];
    E.dense = h->edge_dense && h->edge_dense[e];
    g.edges.push_back(E);
  }
  return g;
}

std::vector<uint32_t> edge_masks(const lh_hypergraph* h) {
  if (!h || !h->edge_attr_count || !h->edge_attrs) fail(LH_ERR_INVALID, "hypergraph is incomplete");
  if (h->n_attrs == 0 || h->n_attrs > MAXV) fail(LH_ERR_INVALID, "n_attrs must be 1..16");
  if (h->n_edges == 0 || h->n_edges > MAXA) fail(LH_ERR_INVALID, "n_edges must be 1..8");
  std::vector<uint32_t> m(h->n_edges, 0);
  uint32_t k = 0;
  for (uint32_t e = 0; e < h->n_edges; e++)
    for (uint32_t i = 0; i < h->edge_attr_count[e]; i++) {
      const uint32_t v = h->edge_attrs[k++];
      if (v >= h->n_attrs) fail(LH_ERR_INVALID, "edge attribute out of range");
      m[e] |= 1u << v;
    }
  return m;
}

void ghd_to_public(const Ghd& g, lh_ghd* out) {
  memset(out, 0, sizeof(*out));
  out->n_nodes = (uint32_t)g.nodes.size();
  for (size_t t = 0; t < g.nodes.size(); t++) {
    out->parent[t] = g.nodes[t].parent;
    out->edges[t] = g.nodes[t].edges;
    out->attrs[t] = g.nodes[t].attrs;
    out->pushed[t] = g.nodes[t].pushed ? 1u : 0u;
    out->node_fhw[t] = g.nodes[t].fhw;
  }
  out->fhw = g.fhw;
  out->depth = g.depth;
  out->shared = g.shared;
  out->sel_depth = g.sel_depth;
}

// The hypergraph of a query: edge attribute masks, filtered edges, GROUP BY
// edges and the output attribute mask.
void query_hypergraph(const lh_query* q, std::vector<uint32_t>& masks, uint32_t& sel, uint32_t& root,
                      uint32_t& outm) {
  if (!q || !q->atoms) fail(LH_ERR_INVALID, "NULL argument");
  if (q->n_attrs == 0 || q->n_attrs > MAXV) fail(LH_ERR_INVALID, "n_attrs must be 1..16");
  if (q->n_atoms == 0 || q->n_atoms > MAXA) fail(LH_ERR_INVALID, "n_atoms must be 1..8");
  masks.assign(q->n_atoms, 0);
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    const lh_atom& A = q->atoms[e];
    if (!tracked(g_tries, A.trie)) fail(LH_ERR_INVALID, "atom trie is not a live lh_trie");
    if (!A.attr_of_key) fail(LH_ERR_INVALID, "attr_of_key is NULL");
    for (uint32_t k = 0; k < A.trie->n_levels; k++) {
      if (A.attr_of_key[k] >= q->n_attrs) fail(LH_ERR_INVALID, "attribute out of range");
      masks[e] |= 1u << A.attr_of_key[k];
    }
  }
  sel = root = outm = 0;
  if (q->n_filters && !q->filters) fail(LH_ERR_INVALID, "filters is NULL");
  for (uint32_t f = 0; f < q->n_filters; f++) {
    if (q->filters[f].atom >= q->n_atoms) fail(LH_ERR_INVALID, "filter atom out of range");
    sel |= 1u << q->filters[f].atom;
  }
  if (q->n_group && !q->group_cols) fail(LH_ERR_INVALID, "group_cols is NULL");
  for (uint32_t g = 0; g < q->n_group; g++) {
    if (q->group_cols[g].atom >= q->n_atoms) fail(LH_ERR_INVALID, "group column out of range");
    root |= 1u << q->group_cols[g].atom;
  }
  if (q->n_out && !q->out_attrs) fail(LH_ERR_INVALID, "out_attrs is NULL");
  for (uint32_t i = 0; i < q->n_out; i++) {
    if (q->out_attrs[i] >= q->n_attrs) fail(LH_ERR_INVALID, "output attribute out of range");
    outm |= 1u << q->out_attrs[i];
  }
}

}  // namespace

void free_trie(lh_trie* t) { delete t; }

}  // namespace lh

using namespace lh;

extern "C" {

lh_status lh_trie_build(const lh_relation_desc* rel, void* hip_stream, lh_trie** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!rel || !out) fail(LH_ERR_INVALID, "NULL argument");
    if (rel->n_keys == 0 || rel->n_keys > LH_MAX_KEYS) fail(LH_ERR_INVALID, "n_keys must be 1..8");
    if (!rel->keys) fail(LH_ERR_INVALID, "keys is NULL");
    if (rel->n_rows >= (1ull << 32) - 1) fail(LH_ERR_OVERFLOW, "n_rows must be below 2^32 - 1");
    for (uint32_t c = 0; c < rel->n_keys; c++)
      if (!rel->keys[c] && rel->n_rows) fail(LH_ERR_INVALID, "a key column is NULL");
    if (rel->n_annos && !rel->annos) fail(LH_ERR_INVALID, "annos is NULL");
    if (rel->n_meta && !rel->meta) fail(LH_ERR_INVALID, "meta is NULL");
    for (uint32_t a = 0; a < rel->n_annos; a++)
      if (!rel->annos[a] && rel->n_rows) fail(LH_ERR_INVALID, "an annotation column is NULL");
    for (uint32_t m = 0; m < rel->n_meta; m++)
      if (!rel->meta[m] && rel->n_rows) fail(LH_ERR_INVALID, "a meta column is NULL");
    if (!(rel->flags & LH_BAG) && (rel->n_annos || rel->n_meta))
      fail(LH_ERR_INVALID, "a set relation carries no annotation or meta columns");
    if (rel->flags & ~(LH_BAG | LH_LAYOUT_MASK)) fail(LH_ERR_INVALID, "unknown flag bits");
    uint32_t lo[LH_MAX_KEYS];
    uint32_t seen = 0;
    for (uint32_t l = 0; l < rel->n_keys; l++) {
      lo[l] = rel->level_order ? rel->level_order[l] : l;
      if (lo[l] >= rel->n_keys || (seen >> lo[l] & 1u)) fail(LH_ERR_INVALID, "level_order is not a permutation");
      seen |= 1u << lo[l];
    }
    hipStream_t s = (hipStream_t)hip_stream;
    lh_trie* t = build_trie(rel->n_rows, rel->n_keys, rel->keys, rel->n_annos, rel->annos, rel->n_meta, rel->meta, lo,
                            rel->flags, nullptr, 0, s, 0, true);
    track(g_tries, t);
    *out = t;
  });
}

lh_status lh_plan(const lh_query* q, void* hip_stream, lh_plan_t** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!q || !out) fail(LH_ERR_INVALID, "NULL argument");
    for (uint32_t e = 0; q->atoms && e < q->n_atoms; e++)
      if (!tracked(g_tries, q->atoms[e].trie)) fail(LH_ERR_INVALID, "atom trie is not a live lh_trie");
    hipStream_t s = (hipStream_t)hip_stream;
    lh_plan_t* p = make_plan(q, s);
    LH_HIP(hipStreamSynchronize(s));
    track(g_plans, p);
    *out = p;
  });
}

lh_status lh_join_aggregate(lh_plan_t* const* plans, uint32_t n_plans, void* hip_stream, lh_result** out) {
  if (out)
    for (uint32_t i = 0; i < n_plans; i++) out[i] = nullptr;
  std::vector<lh_result_impl*> made;
  lh_status st = guard([&] {
    if (!plans || !out || n_plans == 0) fail(LH_ERR_INVALID, "NULL argument or no plans");
    for (uint32_t i = 0; i < n_plans; i++)
      if (!tracked(g_plans, plans[i])) fail(LH_ERR_INVALID, "not a live lh_plan");
    hipStream_t s = (hipStream_t)hip_stream;
    made.assign(n_plans, nullptr);
    if (n_plans > 1) {
      // the plans of the row-union shape run as one batch; the others
      // one by one
      std::vector<uint32_t> idx;
      std::vector<lh_plan_t*> sub;
      for (uint32_t i = 0; i < n_plans; i++)
        if (row_union_kind(plans[i]) >= 0) {
          idx.push_back(i);
          sub.push_back(plans[i]);
        }
      std::vector<lh_result_impl*> got;
      if (sub.size() > 1 && run_batch(sub.data(), (uint32_t)sub.size(), s, got))
        for (size_t k = 0; k < idx.size(); k++) made[idx[k]] = got[k];
    }
    for (uint32_t i = 0; i < n_plans; i++)
      if (!made[i]) made[i] = run_plan(plans[i], s);
  });
  if (st != LH_OK) {
    for (auto* r : made) delete r;
    return st;
  }
  for (uint32_t i = 0; i < n_plans; i++) {
    out[i] = &made[i]->pub;
    track(g_results, made[i]);
  }
  return LH_OK;
}

lh_status lh_join_aggregate_noalloc(const lh_plan_t* plan, void* hip_stream, uint64_t max_rows,
                                    uint32_t* const* out_keys, uint64_t* counts, double* sums, uint64_t* n_rows) {
  if (n_rows) *n_rows = 0;
  return guard([&] {
    if (!plan || !counts || !n_rows) fail(LH_ERR_INVALID, "NULL argument");
    if (!tracked(g_plans, plan)) fail(LH_ERR_INVALID, "not a live lh_plan");
    const uint32_t n_cols = (uint32_t)(plan->out_attrs.size() + plan->groups.size());
    if (n_cols && !out_keys) fail(LH_ERR_INVALID, "NULL out_keys for a result with key columns");
    for (uint32_t c = 0; c < n_cols; c++)
      if (!out_keys[c]) fail(LH_ERR_INVALID, "NULL output key column");
    if (plan->agg == LH_AGG_SUM && !sums) fail(LH_ERR_INVALID, "NULL sums for a SUM plan");
    *n_rows = run_plan_noalloc(plan, (hipStream_t)hip_stream, max_rows, out_keys, counts, sums, nullptr);
  });
}

void lh_free(void* h) {
  if (!h) return;
  if (untrack(g_tries, h)) {
    delete static_cast<lh_trie*>(h);
  } else if (untrack(g_plans, h)) {
    batch_forget_plan(static_cast<lh_plan_t*>(h));
    delete static_cast<lh_plan_t*>(h);
  } else if (untrack(g_results, h)) {
    delete reinterpret_cast<lh_result_impl*>(h);
  }
  // anything else (already freed, foreign pointer) is ignored
}

const char* lh_last_error(void) { return g_last_error.c_str(); }

lh_status lh_trie_get_info(const lh_trie* t, lh_trie_info* info) {
  return guard([&] {
    if (!t || !info || !tracked(g_tries, t)) fail(LH_ERR_INVALID, "not a live lh_trie");
    lh::ensure_column_stats(const_cast<lh_trie*>(t), nullptr);
    LH_HIP(hipStreamSynchronize(nullptr));
    memset(info, 0, sizeof *info);
    info->n_levels = t->n_levels;
    info->n_rows = t->n_rows;
    for (uint32_t l = 0; l < t->n_levels; l++) {
      info->level_size[l] = t->lv[l].n;
      info->level_sets[l] = t->lv[l].n_sets;
      info->level_words[l] = t->lv[l].pool_words;
      info->level_order[l] = t->level_order[l];
      info->col_distinct[l] = t->col_distinct[l];
      info->col_freq_max[l] = t->col_freq_max[l];
      info->level_bitsets[l] = count_bitsets(t, l, nullptr);
    }
  });
}

lh_status lh_trie_read_level(const lh_trie* t, uint32_t level, uint32_t* keys, uint32_t* offs) {
  return guard([&] {
    if (!t || !tracked(g_tries, t)) fail(LH_ERR_INVALID, "not a live lh_trie");
    if (level >= t->n_levels) fail(LH_ERR_INVALID, "level out of range");
    const Level& L = t->lv[level];
    if (keys && L.n) LH_HIP(hipMemcpy(keys, L.keys.p, L.n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (offs) {
      if (L.offs.p) {
        LH_HIP(hipMemcpy(offs, L.offs.p, (L.n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost));
      } else {
        for (uint64_t i = 0; i <= L.n; i++) offs[i] = (uint32_t)i;
      }
    }
  });
}

lh_status lh_result_read(const lh_result* r, uint32_t* const* keys, uint64_t* counts, double* sums) {
  return guard([&] {
    if (!r || !tracked(g_results, r)) fail(LH_ERR_INVALID, "not a live lh_result");
    if (!r->n_rows) return;
    if (keys)
      for (uint32_t c = 0; c < r->n_cols; c++)
        if (keys[c]) LH_HIP(hipMemcpy(keys[c], r->out_keys[c], r->n_rows * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (counts) LH_HIP(hipMemcpy(counts, r->counts, r->n_rows * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (sums && r->sums) LH_HIP(hipMemcpy(sums, r->sums, r->n_rows * sizeof(double), hipMemcpyDeviceToHost));
  });
}

lh_status lh_plan_get_info(const lh_plan_t* p, lh_plan_info* info) {
  return guard([&] {
    if (!p || !info || !tracked(g_plans, p)) fail(LH_ERR_INVALID, "not a live lh_plan");
    memset(info, 0, sizeof *info);
    info->n_attrs = p->n_attrs;
    for (uint32_t i = 0; i < p->n_attrs; i++) {
      info->attr_order[i] = p->order[i];
      info->level_alg[i] = p->level_alg[i];
    }
    info->cost = p->cost;
    info->case_prefix = p->case_prefix ? 1u : 0u;
    info->exact_digits = p->exact_digits;
    info->exact_lsb = p->exact_lsb;
    info->blas = p->blas;
  });
}

lh_status lh_order_cost(const lh_hypergraph* h, const uint32_t* order, uint32_t* icost, uint32_t* weight,
                        double* cost) {
  return guard([&] {
    Hypergraph g = hypergraph_from(h);
    if (!order) fail(LH_ERR_INVALID, "order is NULL");
    std::vector<uint32_t> o(order, order + g.n_attrs);
    uint32_t seen = 0;
    for (uint32_t v : o) {
      if (v >= g.n_attrs || (seen >> v & 1u)) fail(LH_ERR_INVALID, "order is not a permutation");
      seen |= 1u << v;
    }
    double c = order_cost(g, o, icost, weight);
    if (cost) *cost = c;
  });
}

lh_status lh_choose_order(const lh_hypergraph* h, uint32_t n_out, const uint32_t* out_attrs, uint32_t* order,
                          double* cost) {
  return guard([&] {
    Hypergraph g = hypergraph_from(h);
    if (!order || (n_out && !out_attrs)) fail(LH_ERR_INVALID, "NULL argument");
    std::vector<uint32_t> out(out_attrs, out_attrs + n_out);
    for (uint32_t v : out)
      if (v >= g.n_attrs) fail(LH_ERR_INVALID, "output attribute out of range");
    std::vector<uint32_t> o;
    double c = choose_order(g, out, o);
    std::copy(o.begin(), o.end(), order);
    if (cost) *cost = c;
  });
}

lh_status lh_ghd_fhw(const lh_hypergraph* h, uint32_t edge_mask, double* fhw) {
  return guard([&] {
    std::vector<uint32_t> m = edge_masks(h);
    if (!fhw) fail(LH_ERR_INVALID, "NULL argument");
    if (edge_mask >> m.size()) fail(LH_ERR_INVALID, "edge mask out of range");
    *fhw = fractional_cover(m, edge_mask);
  });
}

lh_status lh_ghd_choose(const lh_hypergraph* h, const uint32_t* edge_sel, const uint32_t* edge_root,
                        uint32_t n_out, const uint32_t* out_attrs, lh_ghd* out) {
  return guard([&] {
    std::vector<uint32_t> m = edge_masks(h);
    if (!out || (n_out && !out_attrs)) fail(LH_ERR_INVALID, "NULL argument");
    uint32_t sel = 0, root = 0, outm = 0;
    for (uint32_t e = 0; e < m.size(); e++) {
      if (edge_sel && edge_sel[e]) sel |= 1u << e;
      if (edge_root && edge_root[e]) root |= 1u << e;
    }
    for (uint32_t i = 0; i < n_out; i++) {
      if (out_attrs[i] >= h->n_attrs) fail(LH_ERR_INVALID, "output attribute out of range");
      outm |= 1u << out_attrs[i];
    }
    ghd_to_public(choose_ghd(m, sel, root, outm), out);
  });
}

lh_status lh_ghd_for_query(const lh_query* q, lh_ghd* out) {
  return guard([&] {
    if (!out) fail(LH_ERR_INVALID, "NULL argument");
    std::vector<uint32_t> m;
    uint32_t sel, root, outm;
    query_hypergraph(q, m, sel, root, outm);
    ghd_to_public(choose_ghd(m, sel, root, outm), out);
  });
}

lh_status lh_ghd_join_aggregate(const lh_query* q, const lh_ghd* g, void* hip_stream, lh_result** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!out) fail(LH_ERR_INVALID, "NULL argument");
    std::vector<uint32_t> m;
    uint32_t sel, root, outm;
    query_hypergraph(q, m, sel, root, outm);
    Ghd d;
    if (g) {
      if (g->n_nodes == 0 || g->n_nodes > LH_GHD_MAX_NODES) fail(LH_ERR_INVALID, "ghd: 1..16 nodes");
      for (uint32_t t = 0; t < g->n_nodes; t++) {
        GhdNode n;
        n.edges = g->edges[t];
        n.parent = g->parent[t];
        n.pushed = g->pushed[t] != 0;
        d.nodes.push_back(n);
      }
      check_ghd(m, sel, root, outm, d);
    } else {
      d = choose_ghd(m, sel, root, outm);
    }
    *out = run_ghd(q, d, (hipStream_t)hip_stream);
  });
}

long lh_live_allocations(void) { return live_allocations(); }

lh_status lh_encode(uint64_t n, uint32_t n_id_cols, const uint32_t* const* ids, uint32_t row_col, uint32_t n_cols,
                    const lh_feature_col* cols, uint32_t bias, uint32_t* out_row, uint32_t* out_feat,
                    double* out_val, uint32_t* n_feat, void* hip_stream) {
  return guard([&] {
    if (!ids || !n_feat || (n_cols && !cols)) fail(LH_ERR_INVALID, "NULL argument");
    *n_feat = encode_features(n, n_id_cols, ids, row_col, n_cols, cols, bias, out_row, out_feat, out_val,
                              (hipStream_t)hip_stream);
  });
}

lh_status lh_logreg_fit(const lh_trie* x_rows, const lh_trie* x_cols, uint32_t anno, const double* y, uint64_t n_y,
                        uint32_t n_feat, uint32_t iters, double step, double* w, double* loss, void* hip_stream) {
  return guard([&] {
    if (!tracked(g_tries, x_rows) || !tracked(g_tries, x_cols)) fail(LH_ERR_INVALID, "X is not a live lh_trie");
    logreg_fit(x_rows, x_cols, anno, y, n_y, n_feat, iters, step, w, loss, (hipStream_t)hip_stream);
  });
}

}  // extern "C"
