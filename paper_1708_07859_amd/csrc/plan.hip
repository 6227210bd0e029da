// Query planning: validation, selection push-down, the cost-based choice of
// the attribute order (section 4) and the exact-summation window.
#include <algorithm>
#include <cmath>
#include <climits>
#include <cstring>
#include <numeric>

#include "costmodel.h"
#include "engine.h"

namespace lh {

bool learned_order(const Hypergraph& h, const std::vector<uint32_t>& out_attrs, const std::vector<uint32_t>& plain,
                   std::vector<uint32_t>& order, hipStream_t s);

namespace {

// One selection over a trie's rows (trie order): equality on a key or meta
// column, or a half-open range [lo, hi) on an annotation or meta column.
struct FilterDev {
  uint32_t kind, eq;
  double lo, hi;
  const uint32_t* ucol;
  const double* dcol;
};

constexpr int MAXF = 16;
struct FilterSet {
  uint32_t nf;
  FilterDev f[MAXF];
};

__global__ void k_eval_filters(FilterSet fs, uint64_t n, uint32_t* flags) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t ok = 1;
    for (uint32_t j = 0; j < fs.nf && ok; j++) {
      const FilterDev& f = fs.f[j];
      switch (f.kind) {
        case LH_EQ_KEY:
        case LH_EQ_META:
          ok = f.ucol[i] == f.eq;
          break;
        case LH_RANGE_META: {
          double v = (double)f.ucol[i];
          ok = (v >= f.lo && v < f.hi);
          break;
        }
        default: {
          double v = f.dcol[i];
          ok = (v >= f.lo && v < f.hi);
        }
      }
    }
    flags[i] = ok;
  }
}

void eval_filters(const FilterDev* f, uint32_t nf, uint64_t n, uint32_t* flags, hipStream_t s) {
  if (nf > MAXF) fail(LH_ERR_UNSUPPORTED, "more than 16 filters on one relation");
  FilterSet fs{};
  fs.nf = nf;
  for (uint32_t i = 0; i < nf; i++) fs.f[i] = f[i];
  if (!n) return;
  uint64_t b = std::min<uint64_t>((n + 255) / 256, 16384);
  k_eval_filters<<<(unsigned)b, 256, 0, s>>>(fs, n, flags);
  LH_HIP(hipGetLastError());
}

lh_trie* filtered_or_reordered(const lh_trie* t, const uint32_t* level_order, const std::vector<FilterDev>& filt,
                               hipStream_t s) {
  // columns of the trie's rows in the relation's own column order
  const uint32_t* keys[LH_MAX_KEYS];
  for (uint32_t l = 0; l < t->n_levels; l++) keys[t->level_order[l]] = row_keys(t, l);
  // the swapped order of a two-level trie whose rows were already sorted
  // that way (by the column statistics): no sort at all
  if (filt.empty() && t->n_levels == 2 && t->tsorted[0].p && level_order[0] == t->level_order[1] &&
      level_order[1] == t->level_order[0]) {
    keys[t->level_order[1]] = t->tsorted[0].p;
    keys[t->level_order[0]] = t->tsorted[1].p;
    return build_trie(t->n_rows, 2, keys, 0, nullptr, 0, nullptr, level_order, t->flags, nullptr, 0, s, 2);
  }
  std::vector<const double*> annos;
  for (auto& a : t->annos) annos.push_back(a.p);
  std::vector<const uint32_t*> meta;
  for (auto& m : t->meta) meta.push_back(m.p);
  const uint64_t n = t->n_rows;
  DBuf<uint32_t> sel;
  uint64_t n_sel = n;
  if (!filt.empty()) {
    DBuf<uint32_t> flags(n, s);
    eval_filters(filt.data(), (uint32_t)filt.size(), n, flags.p, s);
    sel.alloc(n, s);
    n_sel = select_flagged(flags.p, n, sel.p, s);
  }
  // The rows are in the trie's order: if the new order ends with a prefix
  // of the old one, those levels are already sorted (a filtered copy in the
  // same order needs no sort at all).
  const uint32_t k = t->n_levels;
  uint32_t tail = 0;
  for (uint32_t m = k; m > 0 && !tail; m--) {
    bool ok = true;
    for (uint32_t i = 0; i < m && ok; i++) ok = level_order[k - m + i] == t->level_order[i];
    if (ok) tail = m;
  }
  // a set relation keeps its set semantics; its rows are already distinct
  return build_trie(n, t->n_levels, keys, (uint32_t)annos.size(), annos.data(), (uint32_t)meta.size(), meta.data(),
                    level_order, t->flags, filt.empty() ? nullptr : sel.p, n_sel, s, tail);
}

bool same_order(const lh_trie* t, const uint32_t* lo) {
  for (uint32_t l = 0; l < t->n_levels; l++)
    if (t->level_order[l] != lo[l]) return false;
  return true;
}

}  // namespace

// The learned order model sees each filtered relation at its size after the
// selection (the relation its GHD node joins), where the plain rule of
// section 4 scores the base cardinality.
Hypergraph learned_view(const lh_query* q, const Hypergraph& h, const std::vector<std::vector<FilterDev>>& filt,
                        hipStream_t s) {
  Hypergraph hl = h;
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    if (filt[e].empty()) continue;
    const uint64_t n = q->atoms[e].trie->n_rows;
    DBuf<uint32_t> flags(n, s);
    DBuf<uint64_t> off(n + 1, s);
    eval_filters(filt[e].data(), (uint32_t)filt[e].size(), n, flags.p, s);
    hl.edges[e].card = n ? scan_u32_to_u64(flags.p, off.p, n, s) : 0;
  }
  return hl;
}

lh_plan_t* make_plan(const lh_query* q, hipStream_t s) {
  if (!q) fail(LH_ERR_INVALID, "query is NULL");
  if (q->agg != LH_AGG_COUNT && q->agg != LH_AGG_SUM) fail(LH_ERR_UNSUPPORTED, "aggregate must be COUNT or SUM");
  if (q->n_attrs == 0 || q->n_attrs > MAXV) fail(LH_ERR_INVALID, "n_attrs must be 1..16");
  if (q->n_atoms == 0 || q->n_atoms > MAXA || !q->atoms) fail(LH_ERR_INVALID, "n_atoms must be 1..8");
  if (q->n_out && !q->out_attrs) fail(LH_ERR_INVALID, "out_attrs is NULL");
  if (q->n_group && !q->group_cols) fail(LH_ERR_INVALID, "group_cols is NULL");
  if (q->n_filters && !q->filters) fail(LH_ERR_INVALID, "filters is NULL");
  std::unique_ptr<lh_plan_t> p(new lh_plan_t());
  p->n_attrs = q->n_attrs;
  p->agg = q->agg;
  p->policy = q->policy & LH_POLICY_MASK;
  p->group_impl = (q->policy & LH_GROUP_MASK) >> 4;
  uint32_t covered = 0;
  int annotated = 0;
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    const lh_atom& A = q->atoms[e];
    if (!A.trie || A.trie->magic != TRIE_MAGIC) fail(LH_ERR_INVALID, "atom has no valid trie");
    if (!A.attr_of_key) fail(LH_ERR_INVALID, "atom attr_of_key is NULL");
    uint32_t mine = 0;
    for (uint32_t c = 0; c < A.trie->n_levels; c++) {
      uint32_t v = A.attr_of_key[c];
      if (v >= q->n_attrs) fail(LH_ERR_INVALID, "attribute id out of range");
      if (mine >> v & 1u) fail(LH_ERR_INVALID, "an atom maps two key columns to one attribute");
      mine |= 1u << v;
    }
    covered |= mine;
    if (A.anno >= 0 && (uint32_t)A.anno >= A.trie->annos.size()) fail(LH_ERR_INVALID, "annotation column out of range");
    if (q->agg == LH_AGG_SUM && A.anno >= 0) annotated++;
  }
  if (covered != ((q->n_attrs == 32 ? 0u : (1u << q->n_attrs)) - 1u)) fail(LH_ERR_INVALID, "an attribute is in no atom");
  if (q->agg == LH_AGG_SUM && annotated == 0) fail(LH_ERR_INVALID, "SUM needs an annotated atom");
  uint32_t outs = 0;
  for (uint32_t i = 0; i < q->n_out; i++) {
    uint32_t v = q->out_attrs[i];
    if (v >= q->n_attrs || (outs >> v & 1u)) fail(LH_ERR_INVALID, "bad output attribute");
    outs |= 1u << v;
    p->out_attrs.push_back(v);
  }
  for (uint32_t g = 0; g < q->n_group; g++) {
    const lh_group_col& G = q->group_cols[g];
    if (G.atom >= q->n_atoms || G.meta_col >= q->atoms[G.atom].trie->meta.size())
      fail(LH_ERR_INVALID, "group column out of range");
    p->groups.push_back(G);
  }
  std::vector<std::vector<FilterDev>> filt(q->n_atoms);
  std::vector<bool> eqsel(q->n_atoms, false);
  for (uint32_t i = 0; i < q->n_filters; i++) {
    const lh_filter& f = q->filters[i];
    if (f.atom >= q->n_atoms) fail(LH_ERR_INVALID, "filter atom out of range");
    const lh_trie* t = q->atoms[f.atom].trie;
    FilterDev d{};
    d.kind = f.kind;
    d.eq = f.eq;
    d.lo = f.lo;
    d.hi = f.hi;
    switch (f.kind) {
      case LH_EQ_KEY: {
        if (f.col >= t->n_levels) fail(LH_ERR_INVALID, "filter key column out of range");
        for (uint32_t l = 0; l < t->n_levels; l++)
          if (t->level_order[l] == f.col) d.ucol = row_keys(t, l);
        eqsel[f.atom] = true;
        break;
      }
      case LH_EQ_META:
      case LH_RANGE_META:
        if (f.col >= t->meta.size()) fail(LH_ERR_INVALID, "filter meta column out of range");
        d.ucol = t->meta[f.col].p;
        if (f.kind == LH_EQ_META) eqsel[f.atom] = true;
        break;
      case LH_RANGE_ANNO:
        if (f.col >= t->annos.size()) fail(LH_ERR_INVALID, "filter annotation column out of range");
        d.dcol = t->annos[f.col].p;
        break;
      default:
        fail(LH_ERR_INVALID, "unknown filter kind");
    }
    filt[f.atom].push_back(d);
  }

  // ---- attribute order --------------------------------------------------------
  Hypergraph h;
  h.n_attrs = q->n_attrs;
  const bool learned_policy = !q->attr_order && (q->policy & LH_POLICY_MASK) == LH_POLICY_LEARNED;
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    const lh_atom& A = q->atoms[e];
    if (learned_policy) ensure_column_stats(const_cast<lh_trie*>(A.trie), s);
    Edge E;
    // attributes in the trie's level order (an order that breaks it re-sorts the relation)
    for (uint32_t l = 0; l < A.trie->n_levels; l++) {
      E.attrs.push_back(A.attr_of_key[A.trie->level_order[l]]);
      const double d = (double)std::max<uint64_t>(1, A.trie->col_distinct[l]);
      E.lf_mean.push_back((float)std::log2(1.0 + (double)A.trie->n_rows / d));
      E.lf_max.push_back((float)std::log2(1.0 + (double)A.trie->col_freq_max[l]));
    }
    E.card = A.trie->n_input;
    E.eq = eqsel[e];
    E.dense = (A.trie->n_levels == 1 && A.trie->lv[0].n > 0 && A.trie->lv[0].n == (uint64_t)A.trie->key_max[0] + 1 &&
               filt[e].empty());
    h.edges.push_back(E);
  }
  std::vector<uint32_t> order(q->n_attrs);
  if (q->attr_order) {
    uint32_t seen = 0;
    for (uint32_t i = 0; i < q->n_attrs; i++) {
      uint32_t v = q->attr_order[i];
      if (v >= q->n_attrs || (seen >> v & 1u)) fail(LH_ERR_INVALID, "attr_order is not a permutation");
      seen |= 1u << v;
      order[i] = v;
    }
    p->cost = order_cost(h, order, nullptr, nullptr);
  } else {
    p->cost = choose_order(h, p->out_attrs, order);
    std::vector<uint32_t> learned;
    if ((q->policy & LH_POLICY_MASK) == LH_POLICY_LEARNED &&
        learned_order(learned_view(q, h, filt, s), p->out_attrs, order, learned, s) && learned != order) {
      order = learned;
      p->cost = order_cost(h, order, nullptr, nullptr);
    }
  }
  for (uint32_t i = 0; i < q->n_attrs; i++) {
    p->order[i] = order[i];
    p->depth_of[order[i]] = i;
    p->level_alg[i] = ALG_PROBE;
  }

  // ---- atoms: filtered / re-ordered tries ---------------------------------------
  p->parts.assign(q->n_attrs, {});
  std::vector<const lh_trie*> reorder_src;
  std::vector<std::vector<uint32_t>> reorder_cols;
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    const lh_atom& A = q->atoms[e];
    const lh_trie* t = A.trie;
    PlanAtom pa;
    pa.n_levels = t->n_levels;
    pa.anno = q->agg == LH_AGG_SUM ? A.anno : -1;
    pa.bag = (t->flags & LH_BAG) != 0;
    pa.card = t->n_input;
    pa.has_eq_filter = eqsel[e];
    // key columns by depth of their attribute
    std::vector<uint32_t> cols(t->n_levels);
    std::iota(cols.begin(), cols.end(), 0u);
    std::sort(cols.begin(), cols.end(),
              [&](uint32_t a, uint32_t b) { return p->depth_of[A.attr_of_key[a]] < p->depth_of[A.attr_of_key[b]]; });
    if (!filt[e].empty()) {
      pa.owned = filtered_or_reordered(t, cols.data(), filt[e], s);
      pa.trie = pa.owned;
    } else if (!same_order(t, cols.data())) {
      // one re-sorted copy per (relation, level order), shared by its atoms
      lh_trie* shared = nullptr;
      for (size_t i = 0; i < reorder_src.size() && !shared; i++)
        if (reorder_src[i] == t && reorder_cols[i] == cols) shared = p->reordered[i];
      if (!shared) {
        shared = filtered_or_reordered(t, cols.data(), filt[e], s);
        p->reordered.push_back(shared);
        reorder_src.push_back(t);
        reorder_cols.push_back(cols);
      }
      pa.trie = shared;
    } else {
      pa.trie = t;
    }
    for (uint32_t l = 0; l < pa.n_levels; l++) {
      pa.attr_of_level[l] = A.attr_of_key[cols[l]];
      p->parts[p->depth_of[pa.attr_of_level[l]]].push_back(Participant{e, l});
    }
    p->atoms.push_back(pa);
  }
  for (auto& g : p->groups) (void)g;

  // streamed groups when the output is a proper prefix of the order
  p->case_full = p->groups.empty() && p->agg == LH_AGG_COUNT && p->n_attrs > 0 && p->out_attrs.size() == p->n_attrs;
  p->case_prefix = p->groups.empty() && p->out_attrs.size() < p->n_attrs;
  for (uint32_t j = 0; j < p->out_attrs.size() && p->case_prefix; j++)
    if (p->out_attrs[j] != p->order[j]) p->case_prefix = false;

  // ---- exact summation window ------------------------------------------------------
  if (q->agg == LH_AGG_SUM) {
    int32_t lsb = 0;
    double maxprod = 1.0;
    bool allzero = false;
    for (auto& pa : p->atoms) {
      if (pa.anno < 0) continue;
      const AnnoStats& st = pa.trie->astats[pa.anno];
      if (st.nonfinite) fail(LH_ERR_UNSUPPORTED, "annotation column holds a non-finite value");
      if (st.qmin == INT_MAX) allzero = true;
      else lsb += st.qmin;
      maxprod *= st.maxabs;
    }
    if (allzero) {
      lsb = 0;
      maxprod = 0.0;
    }
    // headroom for every join tuple: their number is at most the product
    // of the relations' row counts (and a count beyond 2^64 is an error of
    // its own), each tuple adding |hi| + |lo| <= 2 * maxprod
    int tuple_bits = 0;
    for (auto& pa : p->atoms) {
      const uint64_t n = std::max<uint64_t>(1, pa.trie->n_rows);
      tuple_bits += 64 - __builtin_clzll(n);   // n < 2^bits
    }
    tuple_bits = std::min(tuple_bits, 64);
    int top = maxprod > 0 ? (int)std::ceil(std::log2(maxprod)) + 1 : 0;
    top += tuple_bits + 1;
    int bits = top - lsb + 2;
    uint32_t D = (uint32_t)std::max(1, (bits + 31) / 32);
    if (D > 8) fail(LH_ERR_UNSUPPORTED, "annotation values span too many binades for exact summation");
    p->exact_lsb = lsb;
    p->exact_digits = D;
  }
  plan_dense(q, p.get(), s);
  return p.release();
}

}  // namespace lh
