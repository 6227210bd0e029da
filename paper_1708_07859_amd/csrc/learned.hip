// The learned cost model in the planner and the trie builder, plus the C ABI
// of the network.  The plain rules of section 4 stay the fallback: without a
// registered model every decision is the plain rule's.
//
// Decisions:
//  * layout of each set at trie build (LH_LAYOUT_LEARNED): the network
//    predicts log2 of the time of one probe into a set of a given
//    cardinality and span stored as a uint array or as a bitset (features
//    below); a set becomes a bitset when that is predicted cheaper (and its
//    bitset stays within 4096 words per 64 elements);
//  * attribute order at plan time (LH_POLICY_LEARNED): the network predicts
//    log2 of the plan's run time from per-depth features of a candidate
//    order; the cheapest candidate wins.
// The engine's results do not depend on these choices (exact aggregation).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "costmodel.h"
#include "device_common.h"
#include "engine.h"
#include "mlp.h"

struct lh_mlp {
  uint32_t magic;
  lh::Mlp m;
};

namespace lh {

namespace {

constexpr uint32_t MLP_MAGIC = 0x4d4c5031u;
std::mutex g_model_mu;
const Mlp* g_models[2] = {nullptr, nullptr};
constexpr uint32_t LEARNED_MIN_CARD = 32;  // smaller sets keep the plain rule

struct SetRangeL {
  const uint32_t* offs;
  uint64_t root_n;
};

__device__ __forceinline__ void range_of(const SetRangeL& sr, uint64_t s, uint32_t& b, uint32_t& e) {
  if (!sr.offs) {
    b = 0;
    e = (uint32_t)sr.root_n;
  } else {
    b = sr.offs[s];
    e = sr.offs[s + 1];
  }
}

__device__ __forceinline__ void layout_features(float card, float span, float choice, float* x) {
  x[0] = log2f(card);
  x[1] = log2f(span);
  x[2] = log2f(card / span);
  x[3] = choice;
}

// Candidates: sets with at least LEARNED_MIN_CARD elements.
__global__ void k_cand_flags(SetRangeL sr, uint64_t n_sets, uint32_t* flags) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sets; s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    range_of(sr, s, b, e);
    flags[s] = (e - b) >= LEARNED_MIN_CARD ? 1u : 0u;
  }
}

__global__ void k_cand_features(SetRangeL sr, const uint32_t* keys, const uint32_t* cand, uint64_t nc, float* X) {
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    range_of(sr, cand[c], b, e);
    const float card = (float)(e - b);
    const float span = (float)(keys[e - 1] - keys[b]) + 1.0f;
    layout_features(card, span, 0.0f, X + (2 * c) * LAYOUT_FEATURES);
    layout_features(card, span, 1.0f, X + (2 * c + 1) * LAYOUT_FEATURES);
  }
}

// choice[s]: 0 plain rule, 1 uint, 2 bitset
__global__ void k_cand_decide(SetRangeL sr, const uint32_t* keys, const uint32_t* cand, uint64_t nc, const float* y,
                              uint8_t* choice) {
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    const uint64_t s = cand[c];
    range_of(sr, s, b, e);
    const uint64_t card = e - b;
    const uint64_t span = (uint64_t)keys[e - 1] - keys[b] + 1;
    const bool bs = y[2 * c + 1] < y[2 * c] && span <= 4096ull * card;
    choice[s] = bs ? 2 : 1;
  }
}

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 256 * 64));
}

}  // namespace

const Mlp* registered_model(uint32_t slot) {
  std::lock_guard<std::mutex> lk(g_model_mu);
  return slot < 2 ? g_models[slot] : nullptr;
}

// Per-set layout choices of one trie level from the registered layout
// model; empty when no model is registered (the plain rule applies).
bool learned_layout_choices(const lh_trie* t, uint32_t l, hipStream_t s, DBuf<uint8_t>& choice) {
  const Mlp* m = registered_model(MODEL_LAYOUT);
  if (!m) return false;
  const Level& L = t->lv[l];
  SetRangeL sr{l == 0 ? nullptr : t->lv[l - 1].offs.p, t->lv[0].n};
  choice.alloc(L.n_sets, s);
  if (!L.n_sets) return true;
  LH_HIP(hipMemsetAsync(choice.p, 0, L.n_sets, s));
  DBuf<uint32_t> flags(L.n_sets, s), cand(L.n_sets, s);
  k_cand_flags<<<grid_for(L.n_sets), 256, 0, s>>>(sr, L.n_sets, flags.p);
  LH_HIP(hipGetLastError());
  const uint64_t nc = select_flagged(flags.p, L.n_sets, cand.p, s);
  if (!nc) return true;
  DBuf<float> X(2 * nc * LAYOUT_FEATURES, s), y(2 * nc, s);
  {
    ProfScope ps("learned_layout_features", s, nc, 0);
    k_cand_features<<<grid_for(nc), 256, 0, s>>>(sr, L.keys.p, cand.p, nc, X.p);
  }
  {
    ProfScope ps("learned_layout_infer_bf16", s, 2 * nc, 0);
    m->predict_dev(X.p, y.p, 2 * nc, true, s);
  }
  k_cand_decide<<<grid_for(nc), 256, 0, s>>>(sr, L.keys.p, cand.p, nc, y.p, choice.p);
  LH_HIP(hipGetLastError());
  return true;
}

// Features of one candidate order (ORDER_FEATURES floats): for each of
// the first 4 positions, the section 4 icost / 50, log2(1 + weight), and
// over the relations holding the attribute the smallest and the largest
// log2 expected size and the largest log2 maximum size of the set each
// offers there (zeros past the last attribute); then log2(1 + the rows of
// relations whose trie levels the order breaks, which a plan must
// re-sort), log2(1 + all rows), the attribute count and log2(1 + the
// section 4 cost).  Edge attributes are listed in trie level order.
void order_features(const Hypergraph& h, const std::vector<uint32_t>& order, float* f) {
  std::vector<uint32_t> ic(order.size()), w(order.size());
  const double cost = order_cost(h, order, ic.data(), w.data());
  std::fill(f, f + ORDER_FEATURES, 0.0f);
  std::vector<uint32_t> depth(h.n_attrs, 0);
  for (size_t i = 0; i < order.size(); i++) depth[order[i]] = (uint32_t)i;
  double resort = 0, all = 0;
  for (auto& e : h.edges) {
    all += (double)e.card;
    for (size_t l = 1; l < e.attrs.size(); l++)
      if (depth[e.attrs[l]] < depth[e.attrs[l - 1]]) {
        resort += (double)e.card;
        break;
      }
  }
  f[20] = (float)std::log2(1.0 + resort);
  f[21] = (float)std::log2(1.0 + all);
  f[22] = (float)h.n_attrs;
  f[23] = (float)std::log2(1.0 + cost);
  for (size_t i = 0; i < order.size() && i < 4; i++) {
    // per participating relation, the expected / largest size of the set it
    // offers at this position: its root set (distinct values) when the
    // attribute is its first bound one, else the children of the attribute
    // bound just before (rows per value of that column)
    float mean_lo = 0.0f, mean_hi = 0.0f, max_hi = 0.0f;
    bool first = true;
    for (auto& e : h.edges) {
      int self = -1, parent = -1;
      uint32_t pd = 0;
      for (size_t k = 0; k < e.attrs.size(); k++) {
        const uint32_t dk = depth[e.attrs[k]];
        if (e.attrs[k] == order[i]) self = (int)k;
        else if (dk < i && (parent < 0 || dk > pd)) {
          parent = (int)k;
          pd = dk;
        }
      }
      if (self < 0 || e.dense) continue;
      float mn, mx;
      if (parent < 0) {
        const float d = e.lf_mean.empty() ? 0.0f : (float)std::log2(1.0 + (double)e.card) - e.lf_mean[self];
        mn = mx = std::max(0.0f, d);
      } else {
        mn = e.lf_mean.empty() ? 0.0f : e.lf_mean[parent];
        mx = e.lf_max.empty() ? 0.0f : e.lf_max[parent];
      }
      mean_lo = first ? mn : std::min(mean_lo, mn);
      mean_hi = first ? mn : std::max(mean_hi, mn);
      max_hi = first ? mx : std::max(max_hi, mx);
      first = false;
    }
    f[5 * i + 0] = (float)ic[i] / 50.0f;
    f[5 * i + 1] = std::log2(1.0f + (float)w[i]);
    f[5 * i + 2] = mean_lo;
    f[5 * i + 3] = mean_hi;
    f[5 * i + 4] = max_hi;
  }
}

// The model overrides the plain rule's order only when it predicts the
// override to be faster by at least this much (log2 of a time ratio, so
// 2^0.5 = 1.41x): about its root-mean-square error on its training set.
// Below that the predicted gain is within the model's own noise.
constexpr float LEARNED_ORDER_MARGIN = 0.5f;

// The learned order: every candidate the plain search considers, scored
// by the registered order model; the plain rule's order (plain) stays
// unless the model's best beats it by LEARNED_ORDER_MARGIN.  False when no
// model is registered.
bool learned_order(const Hypergraph& h, const std::vector<uint32_t>& out_attrs, const std::vector<uint32_t>& plain,
                   std::vector<uint32_t>& order, hipStream_t s) {
  const Mlp* m = registered_model(MODEL_ORDER);
  if (!m || h.n_attrs > 8) return false;
  const uint32_t n = h.n_attrs;
  std::vector<bool> mat(n, false);
  for (uint32_t v : out_attrs) mat[v] = true;
  std::vector<std::vector<uint32_t>> cands;
  std::vector<uint32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0u);
  do {
    bool ok = true, seen_proj = false;
    for (uint32_t v : perm) {
      if (!mat[v]) seen_proj = true;
      else if (seen_proj) ok = false;
    }
    if (!ok) continue;
    cands.push_back(perm);
    if (n >= 2 && !mat[perm[n - 1]] && mat[perm[n - 2]]) {
      std::vector<uint32_t> sw = perm;
      std::swap(sw[n - 1], sw[n - 2]);
      cands.push_back(sw);
    }
  } while (std::next_permutation(perm.begin(), perm.end()));
  size_t ip = 0;
  while (ip < cands.size() && cands[ip] != plain) ip++;
  if (ip == cands.size()) cands.push_back(plain);
  std::vector<float> X(cands.size() * ORDER_FEATURES), y(cands.size());
  for (size_t c = 0; c < cands.size(); c++) order_features(h, cands[c], X.data() + c * ORDER_FEATURES);
  m->predict(X.data(), y.data(), cands.size(), true, s);
  size_t best = 0;
  for (size_t c = 1; c < cands.size(); c++)
    if (y[c] < y[best] || (y[c] == y[best] && cands[c] < cands[best])) best = c;
  order = (y[ip] - y[best] >= LEARNED_ORDER_MARGIN) ? cands[best] : plain;
  return true;
}

}  // namespace lh

using namespace lh;

namespace {
thread_local std::string g_mlp_err;

template <class F>
lh_status mguard(F&& f) {
  try {
    f();
    return LH_OK;
  } catch (const Error& e) {
    g_mlp_err = e.msg;
    return e.status;
  } catch (...) {
    return LH_ERR_DEVICE;
  }
}

bool live(const lh_mlp* m) { return m && m->magic == MLP_MAGIC; }
}  // namespace

extern "C" {

lh_status lh_mlp_create(uint32_t d_in, uint32_t width, uint64_t seed, lh_mlp** out) {
  if (out) *out = nullptr;
  return mguard([&] {
    if (!out) fail(LH_ERR_INVALID, "out is NULL");
    *out = new lh_mlp{MLP_MAGIC, Mlp(d_in, width, seed)};
  });
}

void lh_mlp_free(lh_mlp* m) {
  if (!live(m)) return;
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    for (auto& slot : g_models)
      if (slot == &m->m) slot = nullptr;
  }
  m->magic = 0;
  delete m;
}

uint64_t lh_mlp_num_params(const lh_mlp* m) { return live(m) ? m->m.num_params() : 0; }

lh_status lh_mlp_get_params(const lh_mlp* m, float* params) {
  return mguard([&] {
    if (!live(m) || !params) fail(LH_ERR_INVALID, "bad arguments");
    memcpy(params, m->m.host.data(), m->m.num_params() * sizeof(float));
  });
}

lh_status lh_mlp_set_params(lh_mlp* m, const float* params) {
  return mguard([&] {
    if (!live(m) || !params) fail(LH_ERR_INVALID, "bad arguments");
    memcpy(m->m.host.data(), params, m->m.num_params() * sizeof(float));
  });
}

lh_status lh_mlp_loss_grad(const lh_mlp* m, const float* X, const float* y, uint32_t n, void* hip_stream,
                           float* loss, float* grad) {
  return mguard([&] {
    if (!live(m) || !X || !y || n == 0) fail(LH_ERR_INVALID, "bad arguments");
    float l = m->m.loss_grad(X, y, n, grad, (hipStream_t)hip_stream);
    if (loss) *loss = l;
  });
}

lh_status lh_mlp_train(lh_mlp* m, const float* X, const float* y, uint32_t n, uint32_t epochs, uint32_t batch,
                       float lr, uint64_t seed, void* hip_stream, float* final_loss) {
  return mguard([&] {
    if (!live(m) || !X || !y || n == 0) fail(LH_ERR_INVALID, "bad arguments");
    float l = m->m.train(X, y, n, epochs, batch, lr, seed, (hipStream_t)hip_stream);
    if (final_loss) *final_loss = l;
  });
}

lh_status lh_mlp_predict(const lh_mlp* m, const float* X, uint64_t n, uint32_t bf16, void* hip_stream, float* y) {
  return mguard([&] {
    if (!live(m) || (n && (!X || !y))) fail(LH_ERR_INVALID, "bad arguments");
    m->m.predict(X, y, n, bf16 != 0, (hipStream_t)hip_stream);
  });
}

lh_status lh_use_model(uint32_t slot, const lh_mlp* m) {
  return mguard([&] {
    if (slot > 1) fail(LH_ERR_INVALID, "slot must be LH_MODEL_LAYOUT or LH_MODEL_ORDER");
    if (m && !live(m)) fail(LH_ERR_INVALID, "not a live lh_mlp");
    const uint32_t want = slot == 0 ? LAYOUT_FEATURES : ORDER_FEATURES;
    if (m && m->m.din != want) fail(LH_ERR_INVALID, "model input width does not match the decision's features");
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_models[slot] = m ? &m->m : nullptr;
  });
}

lh_status lh_order_features(const lh_hypergraph* h, const uint32_t* order, float* features) {
  return mguard([&] {
    if (!h || !order || !features) fail(LH_ERR_INVALID, "bad arguments");
    Hypergraph g;
    g.n_attrs = h->n_attrs;
    uint32_t k = 0;
    for (uint32_t e = 0; e < h->n_edges; e++) {
      Edge E;
      for (uint32_t i = 0; i < h->edge_attr_count[e]; i++) E.attrs.push_back(h->edge_attrs[k++]);
      E.card = h->edge_card[e];
      E.eq = h->edge_eq && h->edge_eq[e];
      E.dense = h->edge_dense && h->edge_dense[e];
      for (size_t a = 0; a < E.attrs.size(); a++) {
        const size_t at = k - E.attrs.size() + a;
        if (h->edge_attr_lf_mean) E.lf_mean.push_back(h->edge_attr_lf_mean[at]);
        if (h->edge_attr_lf_max) E.lf_max.push_back(h->edge_attr_lf_max[at]);
      }
      g.edges.push_back(E);
    }
    std::vector<uint32_t> o(order, order + h->n_attrs);
    order_features(g, o, features);
  });
}

}  // extern "C"
