// The machine-learning phase of a mixed SQL + ML pipeline (section 7):
// categorical feature encoding of a join result and logistic regression
// trained by full-batch gradient descent directly on tries.
//
// The design matrix X is a two-level bag relation (row, feature) with the
// entry value as its annotation.  Its trie in (row, feature) order is a
// row-compressed sparse matrix and its trie in (feature, row) order the
// column-compressed one, so the training loop reads the two tries as they
// are: no conversion into a sparse-BLAS format (section 7, Table 4's point).
//
// One iteration is z = X w, p = 1 / (1 + exp(-z)), g = X^T (p - y) / n and
// w -= step * g.  Both products sum in a fixed order (ascending positions
// within a row; fixed chunks and a fixed tree within a feature), so results
// do not change from run to run.
#include <algorithm>

#include "engine.h"

namespace lh {

namespace {

constexpr int LR_NT = 256;          // threads per workgroup
constexpr uint32_t LR_CAP = 4096;   // staged products per row workgroup (32 KB of LDS)
constexpr uint32_t LR_CHUNK = 2048; // entries of one feature per column workgroup

// ---- encoding ----------------------------------------------------------------

struct EncArgs {
  const uint32_t* ids[LH_ENC_MAX_IDS];
  const uint32_t* codes[LH_ENC_MAX_COLS];
  const double* vals[LH_ENC_MAX_COLS];
  uint64_t n_ids[LH_ENC_MAX_COLS];
  uint32_t by[LH_ENC_MAX_COLS];
  uint32_t base[LH_ENC_MAX_COLS];
  uint32_t card[LH_ENC_MAX_COLS];
  uint32_t row_col, slots, bias;
  uint32_t* out_row;
  uint32_t* out_feat;
  double* out_val;
  uint32_t* err;  // bit 0: an id out of range, bit 1: a code out of range
};

// One thread per output triple (row r, slot k): consecutive threads write
// consecutive triples.
template <class I>
__global__ void k_encode(EncArgs a, uint64_t n) {
  // I: the index type, 32-bit when n * slots fits (a cheaper division)
  const I total = (I)(n * a.slots);
  for (I e = (I)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (I)gridDim.x * blockDim.x) {
    const I r = e / a.slots;
    const uint32_t k = (uint32_t)(e - r * a.slots);
    uint32_t feat = 0;
    double val = 1.0;  // the bias slot and indicators carry 1
    if (k >= a.bias) {
      const uint32_t c = k - a.bias;
      const uint64_t id = a.ids[a.by[c]][r];
      if (id >= a.n_ids[c]) {
        atomicOr(a.err, 1u);
        val = 0.0;
      } else if (a.codes[c]) {
        const uint32_t code = a.codes[c][id];
        if (code >= a.card[c]) {
          atomicOr(a.err, 2u);
          val = 0.0;
        } else {
          feat = a.base[c] + code;
        }
      } else {
        feat = a.base[c];
        val = a.vals[c][id];
      }
    }
    a.out_row[e] = a.ids[a.row_col][r];
    a.out_feat[e] = feat;
    a.out_val[e] = val;
  }
}

// ---- logistic regression --------------------------------------------------------

// Value of X at level-1 node j: its annotation, or the sum over its run
// when the bag holds the same (row, feature) more than once.
__device__ __forceinline__ double entry_value(const uint32_t* runs, const double* val, uint64_t j) {
  if (!runs) return val[j];
  double v = 0.0;
  for (uint32_t k = runs[j], e = runs[j + 1]; k < e; k++) v = __dadd_rn(v, val[k]);
  return v;
}

// Sum of one value per thread in a fixed tree order; thread 0 gets it.
__device__ __forceinline__ double block_sum(double v, double* s_red) {
  const int tid = threadIdx.x;
  s_red[tid] = v;
  __syncthreads();
  for (int h = LR_NT / 2; h > 0; h >>= 1) {
    if (tid < h) s_red[tid] = __dadd_rn(s_red[tid], s_red[tid + h]);
    __syncthreads();
  }
  return s_red[0];
}

struct LrRows {
  const uint32_t* rkeys;  // level 0 of the (row, feature) trie: row ids
  const uint32_t* roffs;  // its child offsets (n0 + 1)
  const uint32_t* fkeys;  // level 1: feature ids
  const uint32_t* runs;   // level-1 run offsets, or null (one value per node)
  const double* val;      // annotation column in trie order
  const double* y;        // label of row id r at y[r]
  const double* w;
  double* res;            // p - y at the row id
  double* lpart;          // per workgroup: sum of log-loss terms, or null
  uint64_t n0;
};

// z, p and the residual of LR_NT consecutive training rows.  The rows'
// level-1 entries are contiguous: their products are formed with coalesced
// loads into LDS when they fit, then every thread sums its own row in
// position order (the unstaged path sums in the same order).
__global__ __launch_bounds__(LR_NT) void k_lr_rows(LrRows a) {
  __shared__ double s_prod[LR_CAP];
  __shared__ uint32_t s_off[LR_NT + 1];
  __shared__ double s_red[LR_NT];
  const int tid = threadIdx.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * LR_NT;
  const uint32_t nr = (uint32_t)min<uint64_t>(LR_NT, a.n0 - i0);
  for (uint32_t t = tid; t <= nr; t += LR_NT) s_off[t] = a.roffs[i0 + t];
  __syncthreads();
  const uint32_t base = s_off[0], tot = s_off[nr] - base;
  const bool staged = tot <= LR_CAP;  // uniform over the workgroup
  if (staged) {
    for (uint32_t j = tid; j < tot; j += LR_NT)
      s_prod[j] = __dmul_rn(entry_value(a.runs, a.val, base + j), a.w[a.fkeys[base + j]]);
    __syncthreads();
  }
  double lterm = 0.0;
  if ((uint32_t)tid < nr) {
    const uint32_t b = s_off[tid], e = s_off[tid + 1];
    double z = 0.0;
    if (staged) {
      for (uint32_t j = b; j < e; j++) z = __dadd_rn(z, s_prod[j - base]);
    } else {
      for (uint32_t j = b; j < e; j++) z = __dadd_rn(z, __dmul_rn(entry_value(a.runs, a.val, j), a.w[a.fkeys[j]]));
    }
    const uint32_t r = a.rkeys[i0 + tid];
    const double yv = a.y[r];
    const double p = 1.0 / (1.0 + exp(-z));
    a.res[r] = p - yv;
    // log(1 + e^z) - y z, with log(1 + e^z) = max(z, 0) + log1p(e^-|z|)
    lterm = fmax(z, 0.0) + log1p(exp(-fabs(z))) - yv * z;
  }
  if (a.lpart) {
    const double sum = block_sum(lterm, s_red);
    if (tid == 0) a.lpart[blockIdx.x] = sum;
  }
}

struct LrCols {
  const uint32_t* foffs;   // level 0 of the (feature, row) trie: child offsets (n0 + 1)
  const uint32_t* rkeys;   // level 1: row ids
  const uint32_t* runs;    // level-1 run offsets, or null
  const double* val;       // annotation column in trie order
  const double* res;       // p - y at the row id
  const uint32_t* cfeat;   // chunk -> level-0 position of its feature
  const uint32_t* cstart;  // level-0 position -> its first chunk (n0 + 1)
  double* part;            // per chunk: sum of value x residual
};

// One workgroup per chunk of LR_CHUNK entries of one feature.  Thread t
// takes entries t, t + LR_NT, ... of the chunk: all of its loads are
// issued before the sum, which adds them in that order.
__global__ __launch_bounds__(LR_NT) void k_lr_cols(LrCols a) {
  constexpr uint32_t PER = LR_CHUNK / LR_NT;
  __shared__ double s_red[LR_NT];
  const uint32_t c = blockIdx.x;
  const uint32_t f = a.cfeat[c];
  const uint32_t b = a.foffs[f] + (c - a.cstart[f]) * LR_CHUNK;
  const uint32_t e = (uint32_t)min<uint64_t>(a.foffs[f + 1], (uint64_t)b + LR_CHUNK);
  uint32_t r[PER];
  double v[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t j = b + threadIdx.x + k * LR_NT;
    const bool in = j < e;
    r[k] = in ? a.rkeys[j] : 0u;
    v[k] = in ? entry_value(a.runs, a.val, j) : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t j = b + threadIdx.x + k * LR_NT;
    if (j < e) acc = __dadd_rn(acc, __dmul_rn(v[k], a.res[r[k]]));
  }
  const double sum = block_sum(acc, s_red);
  if (threadIdx.x == 0) a.part[c] = sum;
}

// ---- the blocked column pass ------------------------------------------------
// Row ids are cut into blocks of 2^RB_SHIFT.  A feature's rows are sorted,
// so its entries of one block are a contiguous segment.  One workgroup per
// block stages the block's residuals in LDS and its waves take the
// features in turn: each wave sums a feature's segment (lanes strided,
// then a fixed shuffle tree) with every residual read from LDS.
constexpr uint32_t RB_SHIFT = 12;
constexpr uint32_t RB = 1u << RB_SHIFT;
constexpr int RB_NT = 512;  // 8 waves share the block's features (32 KB of LDS per workgroup)

// seg[f * (nb + 1) + b]: first entry of feature f (level-0 position) at a
// row id >= b * RB; seg[f * (nb + 1) + nb] = the end of f's list.
__global__ void k_lr_segments(const uint32_t* foffs, const uint32_t* rkeys, uint64_t f0, uint32_t nb, uint32_t* seg) {
  const uint64_t total = f0 * (nb + 1);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t f = i / (nb + 1);
    const uint32_t b = (uint32_t)(i - f * (nb + 1));
    uint32_t lo = foffs[f], hi = foffs[f + 1];
    if (b < nb) {
      const uint64_t key = (uint64_t)b << RB_SHIFT;
      while (lo < hi) {  // first row id >= key
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)rkeys[mid] < key) lo = mid + 1;
        else hi = mid;
      }
    } else {
      lo = hi;
    }
    seg[i] = lo;
  }
}

struct LrBlocked {
  const uint32_t* seg;    // (f0, nb + 1) segment starts
  const uint32_t* rkeys;  // level 1 of the (feature, row) trie: row ids
  const uint32_t* runs;   // level-1 run offsets, or null
  const double* val;      // annotation column in trie order
  const double* res;      // p - y at the row id (n_res entries)
  uint64_t n_res;
  uint64_t f0;
  uint32_t nb;
  double* part;           // (f0, nb): per feature and block
};

__global__ __launch_bounds__(RB_NT) void k_lr_cols_blocked(LrBlocked a) {
  __shared__ double s_res[RB];
  const uint32_t b = blockIdx.x;
  const uint64_t r0 = (uint64_t)b << RB_SHIFT;
  const uint32_t nr = (uint32_t)min<uint64_t>(RB, a.n_res - r0);
  for (uint32_t i = threadIdx.x; i < nr; i += RB_NT) s_res[i] = a.res[r0 + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (uint64_t f = w; f < a.f0; f += RB_NT / 64) {
    const uint32_t s = a.seg[f * (a.nb + 1) + b], e = a.seg[f * (a.nb + 1) + b + 1];
    double acc = 0.0;
    for (uint32_t j = s + lane; j < e; j += 64)
      acc = __dadd_rn(acc, __dmul_rn(entry_value(a.runs, a.val, j), s_res[a.rkeys[j] - (uint32_t)r0]));
    for (int o = 32; o > 0; o >>= 1) acc = __dadd_rn(acc, __shfl_xor(acc, o, 64));
    if (lane == 0) a.part[f * a.nb + b] = acc;
  }
}

__global__ void k_stride_starts(uint64_t f0, uint32_t nb, uint32_t* cstart) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f <= f0; f += (uint64_t)gridDim.x * blockDim.x)
    cstart[f] = (uint32_t)(f * nb);
}

__global__ void k_chunk_counts(const uint32_t* foffs, uint64_t n0, uint32_t* cnt) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n0; f += (uint64_t)gridDim.x * blockDim.x)
    cnt[f] = (uint32_t)(((uint64_t)foffs[f + 1] - foffs[f] + LR_CHUNK - 1) / LR_CHUNK);
}

__global__ void k_chunk_fill(const uint32_t* cstart, uint64_t n0, uint32_t* cfeat) {
  for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n0; f += (uint64_t)gridDim.x * blockDim.x)
    for (uint32_t c = cstart[f], e = cstart[f + 1]; c < e; c++) cfeat[c] = (uint32_t)f;
}

// One workgroup per feature: g = (its chunk sums, thread t adding chunks
// t, t + LR_NT, ..., then a fixed tree) / n; w -= step * g.
__global__ __launch_bounds__(LR_NT) void k_lr_update(const uint32_t* fkeys, const uint32_t* cstart,
                                                     const double* part, double n, double step, double* w) {
  __shared__ double s_red[LR_NT];
  const uint32_t f = blockIdx.x;
  double acc = 0.0;
  for (uint32_t c = cstart[f] + threadIdx.x, e = cstart[f + 1]; c < e; c += LR_NT) acc = __dadd_rn(acc, part[c]);
  const double sum = block_sum(acc, s_red);
  if (threadIdx.x == 0) {
    const uint32_t fid = fkeys[f];
    w[fid] = __dsub_rn(w[fid], __dmul_rn(step, __ddiv_rn(sum, n)));
  }
}

// Mean of the per-workgroup loss sums, in a fixed order.
__global__ __launch_bounds__(LR_NT) void k_lr_loss(const double* lpart, uint64_t nb, double n, double* out) {
  __shared__ double s_red[LR_NT];
  double acc = 0.0;
  for (uint64_t i = threadIdx.x; i < nb; i += LR_NT) acc = __dadd_rn(acc, lpart[i]);
  const double sum = block_sum(acc, s_red);
  if (threadIdx.x == 0) *out = __ddiv_rn(sum, n);
}

unsigned grid_of(uint64_t n, uint64_t cap = 1u << 16) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, cap));
}

}  // namespace

uint32_t encode_features(uint64_t n, uint32_t n_id_cols, const uint32_t* const* ids, uint32_t row_col,
                         uint32_t n_cols, const lh_feature_col* cols, uint32_t bias, uint32_t* out_row,
                         uint32_t* out_feat, double* out_val, hipStream_t s) {
  if (n_id_cols == 0 || n_id_cols > LH_ENC_MAX_IDS) fail(LH_ERR_INVALID, "encode: n_id_cols must be 1..8");
  if (n_cols > LH_ENC_MAX_COLS) fail(LH_ERR_INVALID, "encode: at most 32 feature columns");
  if (row_col >= n_id_cols) fail(LH_ERR_INVALID, "encode: row_col out of range");
  if (bias > 1) fail(LH_ERR_INVALID, "encode: bias must be 0 or 1");
  if (n_cols + bias == 0) fail(LH_ERR_INVALID, "encode: no feature");
  EncArgs a{};
  for (uint32_t i = 0; i < n_id_cols; i++) {
    if (!ids[i] && n) fail(LH_ERR_INVALID, "encode: an id column is NULL");
    a.ids[i] = ids[i];
  }
  uint64_t nf = bias;
  for (uint32_t c = 0; c < n_cols; c++) {
    const lh_feature_col& fc = cols[c];
    if (fc.by >= n_id_cols) fail(LH_ERR_INVALID, "encode: a column's id column is out of range");
    if ((fc.codes != nullptr) == (fc.values != nullptr))
      fail(LH_ERR_INVALID, "encode: a column needs exactly one of codes and values");
    if (fc.codes && fc.card == 0) fail(LH_ERR_INVALID, "encode: a categorical column with card 0");
    a.codes[c] = fc.codes;
    a.vals[c] = fc.values;
    a.n_ids[c] = fc.n_ids;
    a.by[c] = fc.by;
    a.card[c] = fc.codes ? fc.card : 1;
    a.base[c] = (uint32_t)nf;
    nf += a.card[c];
    if (nf >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "encode: 2^32 features or more");
  }
  a.row_col = row_col;
  a.slots = n_cols + bias;
  a.bias = bias;
  a.out_row = out_row;
  a.out_feat = out_feat;
  a.out_val = out_val;
  if (n) {
    if (!out_row || !out_feat || !out_val) fail(LH_ERR_INVALID, "encode: an output buffer is NULL");
    DBuf<uint32_t> err(1, s);
    fill_u32(err.p, 0, 1, s);
    a.err = err.p;
    {
      ProfScope ps("encode", s, n, n * a.slots);
      if (n * a.slots < (1ull << 32) - (1ull << 26))
        k_encode<uint32_t><<<grid_of(n * a.slots), 256, 0, s>>>(a, n);
      else
        k_encode<uint64_t><<<grid_of(n * a.slots), 256, 0, s>>>(a, n);
      LH_HIP(hipGetLastError());
    }
    const uint32_t e = read_scalar(err.p, s);
    if (e & 1u) fail(LH_ERR_INVALID, "encode: an id is not below its column's n_ids");
    if (e & 2u) fail(LH_ERR_INVALID, "encode: a categorical code is not below its card");
  }
  return (uint32_t)nf;
}

void logreg_fit(const lh_trie* xr, const lh_trie* xc, uint32_t anno, const double* y, uint64_t n_y, uint32_t n_feat,
                uint32_t iters, double step, double* w, double* loss, hipStream_t s) {
  for (const lh_trie* t : {xr, xc}) {
    if (t->n_levels != 2 || !(t->flags & LH_BAG)) fail(LH_ERR_INVALID, "logreg: X must be two-level bag tries");
    if (anno >= t->annos.size()) fail(LH_ERR_INVALID, "logreg: annotation column out of range");
  }
  if (xr->level_order[0] != xc->level_order[1] || xr->level_order[1] != xc->level_order[0])
    fail(LH_ERR_INVALID, "logreg: the two tries' level orders are not transposes");
  if (xr->n_rows != xc->n_rows) fail(LH_ERR_INVALID, "logreg: the two tries hold different relations");
  const uint64_t n0 = xr->lv[0].n, f0 = xc->lv[0].n;
  if (f0 >= (1ull << 31)) fail(LH_ERR_OVERFLOW, "logreg: 2^31 features or more");
  if (n0 && (xr->key_max[0] >= n_y || xc->key_max[1] >= n_y))
    fail(LH_ERR_INVALID, "logreg: a row id is not below n_y");
  if (n0 && (xr->key_max[1] >= n_feat || xc->key_max[0] >= n_feat))
    fail(LH_ERR_INVALID, "logreg: a feature id is not below n_feat");
  if (n0 && (!y || !w)) fail(LH_ERR_INVALID, "logreg: y or w is NULL");
  if (iters && n0 == 0) {
    // no training rows: the weights stay, the mean loss is taken as 0
    if (loss) fill_u64(reinterpret_cast<uint64_t*>(loss), 0, iters, s);
    LH_HIP(hipStreamSynchronize(s));
    return;
  }
  if (!iters) return;
  const double n = (double)n0;

  LrRows ra{};
  ra.rkeys = xr->lv[0].keys.p;
  ra.roffs = xr->lv[0].offs.p;
  ra.fkeys = xr->lv[1].keys.p;
  ra.runs = xr->n_rows == xr->lv[1].n ? nullptr : xr->lv[1].offs.p;
  ra.val = xr->annos[anno].p;
  ra.y = y;
  ra.w = w;
  ra.n0 = n0;
  // residuals by row id, covering the row ids of both tries (zero where a
  // caller's two tries disagree, rather than undefined)
  const uint64_t n_res = (uint64_t)std::max(xr->key_max[0], xc->key_max[1]) + 1;
  DBuf<double> res(n_res, s);
  fill_u64(reinterpret_cast<uint64_t*>(res.p), 0, n_res, s);
  ra.res = res.p;
  const uint64_t nb = (n0 + LR_NT - 1) / LR_NT;
  DBuf<double> lpart(loss ? nb : 0, s);
  ra.lpart = loss ? lpart.p : nullptr;

  // The column pass: blocked by row id when the (feature, block) partial
  // sums stay few next to the entries, else chunks of each feature's list.
  // Either way cstart[f] .. cstart[f + 1] are feature f's partial sums.
  const uint64_t nnz = xr->lv[1].n;
  const uint64_t nblk = (n_res + RB - 1) / RB;
  const bool blocked = nblk < (1u << 24) && f0 * nblk <= std::max<uint64_t>(nnz / 4, 1u << 16);
  DBuf<uint32_t> cnt, cstart(f0 + 1, s), cfeat, seg;
  DBuf<double> part;
  uint32_t nchunks = 0;
  if (blocked) {
    seg.alloc(f0 * (nblk + 1), s);
    k_lr_segments<<<grid_of(f0 * (nblk + 1)), 256, 0, s>>>(xc->lv[0].offs.p, xc->lv[1].keys.p, f0, (uint32_t)nblk,
                                                          seg.p);
    LH_HIP(hipGetLastError());
    k_stride_starts<<<grid_of(f0 + 1), 256, 0, s>>>(f0, (uint32_t)nblk, cstart.p);
    LH_HIP(hipGetLastError());
    part.alloc(f0 * nblk, s);
  } else {
    cnt.alloc(f0, s);
    k_chunk_counts<<<grid_of(f0), 256, 0, s>>>(xc->lv[0].offs.p, f0, cnt.p);
    LH_HIP(hipGetLastError());
    nchunks = scan_u32(cnt.p, cstart.p, f0, s);
    cfeat.alloc(nchunks, s);
    part.alloc(nchunks, s);
    k_chunk_fill<<<grid_of(f0), 256, 0, s>>>(cstart.p, f0, cfeat.p);
    LH_HIP(hipGetLastError());
  }
  LrBlocked ba{};
  ba.seg = seg.p;
  ba.rkeys = xc->lv[1].keys.p;
  ba.runs = xc->n_rows == xc->lv[1].n ? nullptr : xc->lv[1].offs.p;
  ba.val = xc->annos[anno].p;
  ba.res = res.p;
  ba.n_res = n_res;
  ba.f0 = f0;
  ba.nb = (uint32_t)nblk;
  ba.part = part.p;
  LrCols ca{};
  ca.foffs = xc->lv[0].offs.p;
  ca.rkeys = xc->lv[1].keys.p;
  ca.runs = xc->n_rows == xc->lv[1].n ? nullptr : xc->lv[1].offs.p;
  ca.val = xc->annos[anno].p;
  ca.res = res.p;
  ca.cfeat = cfeat.p;
  ca.cstart = cstart.p;
  ca.part = part.p;

  for (uint32_t it = 0; it < iters; it++) {
    {
      ProfScope ps("lr_rows", s, n0, nnz);
      k_lr_rows<<<(unsigned)nb, LR_NT, 0, s>>>(ra);
      LH_HIP(hipGetLastError());
    }
    if (loss) {
      k_lr_loss<<<1, LR_NT, 0, s>>>(lpart.p, nb, n, loss + it);
      LH_HIP(hipGetLastError());
    }
    if (blocked) {
      ProfScope ps("lr_cols_blocked", s, f0, nnz);
      k_lr_cols_blocked<<<(unsigned)nblk, RB_NT, 0, s>>>(ba);
      LH_HIP(hipGetLastError());
    } else if (nchunks) {
      ProfScope ps("lr_cols", s, f0, nnz);
      k_lr_cols<<<nchunks, LR_NT, 0, s>>>(ca);
      LH_HIP(hipGetLastError());
    }
    k_lr_update<<<(unsigned)f0, LR_NT, 0, s>>>(xc->lv[0].keys.p, cstart.p, part.p, n, step, w);
    LH_HIP(hipGetLastError());
  }
  LH_HIP(hipStreamSynchronize(s));
}

}  // namespace lh
