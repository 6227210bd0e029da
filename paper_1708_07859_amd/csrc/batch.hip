// Batched execution of many join-aggregate instances of uneven size in one
// persistent, graph-captured launch.
//
// Handled shape ("row union"): two annotated relations A(i, j) and E(j)
// or E(j, k) under the order i, j[, k] with output [i] or [i, k] -- the
// sparse matrix-vector and matrix-matrix products the paper expresses as
// join-aggregate queries (the order i, j, k is the relaxed order of section
// 4.1.2, whose last attribute is materialized by a GROUP BY on a key,
// section 5).  Every row i of every instance is a work item:
//  * light rows (few products) are taken by one wave, which sums exactly
//    into a private LDS hash keyed by k;
//  * heavy rows are taken by a whole block: a symbolic pass marks the k the
//    row produces in an LDS bitmap, whose popcount prefixes rank them; the
//    products are then summed exactly in LDS accumulators indexed by rank,
//    512 ranks at a time, each window's products cut out of the B rows by
//    binary search and spread evenly over the block, and emitted in k order;
//  * rows with many products relative to the size of E are taken by a
//    block in inner-product form: A's row becomes an LDS bitmap over j and
//    the entries of E transposed (built once per batch) are streamed
//    through it, matches adding to per-column LDS accumulators.
// Workers pull items from two device queues (heavy rows first, longest
// first), so one launch balances thousands of instances.  The launch and
// its queue resets are captured once in a hipGraph and replayed.  Sums are
// exact (the same accumulator as the single-plan path), so every instance's
// result is bit-identical to running its plan alone.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>

#include "device_common.h"
#include "engine.h"
#include "exact.h"

namespace lh {

namespace {

constexpr int B_NT = 256;
constexpr int B_NW = B_NT / WAVE;
constexpr uint32_t KW_MAX = 64 * 4 * B_NT;   // k values per heavy window (4 bitmap words per thread)
constexpr uint32_t EMPTY_KEY = 0xffffffffu;

struct BInst {
  uint32_t kind;             // 0: E(j) (vector), 1: E(j, k) (matrix)
  uint32_t n_rows;           // nodes of A's first level (the rows i)
  const uint32_t* a_i;       // A level 0 keys
  const uint32_t* a_off;     // A level 0 child offsets
  const uint32_t* a_j;       // A level 1 keys
  const uint32_t* a_run;     // A bag runs of level 1 (null: one row per node)
  const double* a_val;       // A annotation in trie order (null for COUNT)
  const uint32_t* e_j;       // E level 0 keys
  uint32_t e_n0;
  uint32_t e_dense;          // E's first-level keys are exactly 0 .. e_n0 - 1
  uint64_t e_bsw;            // E root set bitset word (UINT64_MAX: uint layout)
  uint32_t e_bsb;
  const uint64_t* e_pool;
  const uint32_t* e_off;     // matrix: E level 0 child offsets
  const uint32_t* e_k;       // matrix: E level 1 keys
  const uint32_t* e_run;     // bag runs of E's last level (null: one row per node)
  const double* e_val;
  int32_t lsb;
  uint32_t D;
  uint32_t sum;
  uint32_t n_k;              // matrix: largest k + 1
  uint64_t row_base;         // first batch row of this instance
  // matrix, inner-product rows: E transposed (levels k, j) and A's j range
  uint32_t n_j;              // largest j of A + 1
  uint32_t bt_n0;            // k nodes of E transposed
  const uint32_t* bt_k;      // their k values
  const uint32_t* bt_off;    // child offsets into bt_j
  const uint32_t* bt_j;      // j of each (k, j)
  const uint32_t* bt_run;    // bag runs of (k, j) into bt_val rows (null: one row each)
  const double* bt_val;      // E's annotation in transposed row order
  uint64_t nnz_e;            // (k, j) pairs of E
};

__device__ __forceinline__ bool find_j(const BInst& I, uint32_t j, uint32_t& pos) {
  if (I.e_dense) {  // E's first level holds every key 0 .. e_n0 - 1: j is its own position
    pos = j;
    return j < I.e_n0;
  }
  if (I.e_n0 == 0) return false;
  if (I.e_bsw != UINT64_MAX) {
    if (j < I.e_bsb || j > I.e_j[I.e_n0 - 1]) return false;
    const uint32_t d = j - I.e_bsb;
    if (!((I.e_pool[I.e_bsw + (d >> 6)] >> (d & 63u)) & 1ull)) return false;
  }
  const uint32_t q = lower_bound_u32(I.e_j, 0, I.e_n0, j);
  if (q < I.e_n0 && I.e_j[q] == j) {
    pos = q;
    return true;
  }
  return false;
}

__device__ __forceinline__ void rows_of(const uint32_t* run, uint32_t node, uint32_t& b, uint32_t& e) {
  if (run) {
    b = run[node];
    e = run[node + 1];
  } else {
    b = node;
    e = node + 1;
  }
}

// ---- setup: per-row product bounds and classes ----------------------------

__global__ void k_row_setup(const BInst* inst, const uint64_t* inst_row0, uint32_t n_inst, uint64_t R,
                            uint32_t light_max, uint32_t inner_ratio, uint32_t* row_inst, uint64_t* prod, uint32_t* ub,
                            uint32_t* is_heavy, uint32_t* is_light, uint32_t* is_inner) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < R; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t ii = (uint32_t)upper_bound_minus1<uint64_t>(inst_row0, 0, n_inst, t);
    const BInst& I = inst[ii];
    const uint32_t p = (uint32_t)(t - inst_row0[ii]);
    row_inst[t] = ii;
    uint64_t u = 0;
    for (uint32_t q = I.a_off[p]; q < I.a_off[p + 1]; q++) {
      uint32_t pe;
      if (!find_j(I, I.a_j[q], pe)) continue;
      uint32_t ab, ae, eb, ee;
      rows_of(I.a_run, q, ab, ae);
      if (I.kind == 0) {
        rows_of(I.e_run, pe, eb, ee);
        u += (uint64_t)(ae - ab) * (ee - eb);
      } else {
        u += (uint64_t)(ae - ab) * (I.e_off[pe + 1] - I.e_off[pe]);
      }
    }
    prod[t] = u;
    const bool heavy = I.kind == 1 && u > light_max;
    // inner-product form when walking all of E costs less than inner_ratio
    // scattered updates per product
    const bool inner = heavy && I.bt_k && I.n_j <= KW_MAX && u * inner_ratio >= I.nnz_e;
    ub[t] = I.kind == 0 ? 1u : (uint32_t)min<uint64_t>(u, I.n_k);
    is_heavy[t] = heavy && !inner ? 1u : 0u;
    is_light[t] = heavy ? 0u : 1u;
    is_inner[t] = inner ? 1u : 0u;
  }
}

__global__ void k_fill_u32_dev(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---- the persistent kernel -------------------------------------------------------

struct BatchArgs {
  const BInst* inst;
  const uint32_t* row_inst;
  const uint64_t* inst_row0;
  const uint64_t* ub_off;    // per batch row: first upper-bound output slot
  const uint32_t* heavy;     // heavy rows, longest first
  uint64_t n_heavy;
  const uint32_t* light;     // light rows
  uint64_t n_light;
  const uint32_t* inner;     // inner-product rows, grouped by instance
  uint64_t n_inner;
  uint32_t* qhead;           // [0] heavy queue, [1] light queue, [2] inner queue
  uint32_t* row_nnz;         // outputs per row
  uint32_t* ub_k;
  uint64_t* ub_cnt;
  double* ub_sum;
  uint32_t* err;
  const uint64_t* prod;      // per batch row: its number of products
  uint32_t kw;                      // k values per heavy window (multiple of 64, <= KW_MAX)
};

// LDS accumulators of the heavy and inner kernels sit DSTRIDE 8-byte slots
// apart: with 9 (72 bytes), the same digit of different accumulators falls
// in different LDS banks (at 8, 64 bytes apart, every accumulator's digit k
// shared two banks and the atomics of a wave serialized on them).
constexpr int DSTRIDE = EXACT_MAXD + 1;

// A row with fewer products than this keeps its LDS accumulators in signed
// slots: a product adds two terms, each at most one word below 2^32 to any
// slot, so no slot can leave int64 (2 * 2^30 * 2^32 = 2^63).
constexpr uint64_t BOUNDED_PRODUCTS = 1ull << 30;

// Exact sum held in the LDS slots (digits) of one accumulator: add v.
// bounded (the row has fewer than BOUNDED_PRODUCTS products): signed slots,
// plain atomic adds whose returned values nobody waits for.  Otherwise the
// shared slot form, which carries every wrap, so any number of terms is
// exact.  A row uses one form for all of its accumulators.
__device__ __forceinline__ bool lds_add_term(long long* slots, double v, int32_t lsb, uint32_t D, bool bounded) {
  if (!bounded) return atomic_add_term((int64_t*)slots, v, lsb, D, 1);
  if (v == 0.0) return true;
  int32_t k0;
  uint32_t p[5];
  bool neg;
  if (!term_words(v, lsb, 1, k0, p, neg)) return false;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 5; j++) {
    if (!p[j]) continue;
    if (k0 + j >= (int32_t)D) {
      ok = false;
      continue;
    }
    const int64_t w = neg ? -(int64_t)p[j] : (int64_t)p[j];
    atomicAdd((unsigned long long*)&slots[k0 + j], (unsigned long long)w);
  }
  return ok;
}

// The correctly rounded value of an LDS accumulator in the form lds_add_term
// used: signed slots are carried into digits first (a normalized value is
// also a shared-form value).
__device__ __forceinline__ double lds_round(const long long* slots, uint32_t D, int32_t lsb, bool bounded,
                                            uint32_t* err) {
  if (!bounded) return exact_round((const int64_t*)slots, D, lsb, err);
  RegAcc r;
#pragma unroll
  for (int i = 0; i < EXACT_MAXD; i++) r.s[i] = i < (int)D ? (int64_t)slots[i] : 0;
  r.normalize(D);
  return exact_round(r.s, D, lsb, err);
}

// Heavy rows: one block per row.  A symbolic pass marks every k the row
// produces in an LDS bitmap (per window of kw values of k); per-word
// popcount prefixes give each k its rank, which is also its place in the
// row's sorted output.  The ranks are then taken HC at a time: the k range
// of the rank window is found from the bitmap, every B row is cut to that
// range by two binary searches, and the products in it add their exact
// digits to LDS accumulators indexed by rank - r0, which are emitted in
// order and cleared.  No global atomics.  In both passes the products of
// B_NT entries of A's row at a time are numbered by a block scan and dealt
// out evenly to the threads.  A row of at most CUR_MAX entries whose
// outputs take several rank windows keeps, per entry of A, a cursor into
// its E row in LDS: windows are taken in increasing k, so each window's
// products of an entry start at its cursor and end where a short gallop
// finds the window's upper k; neither j's lookup nor the two binary
// searches are repeated per window.
constexpr uint32_t HC = 512;
constexpr uint32_t CUR_MAX = 2048;

// First position in [b, e) of the sorted a holding a value >= x, found by
// galloping from b (most windows take few products of one entry).
__device__ __forceinline__ uint32_t gallop_lower_bound(const uint32_t* a, uint32_t b, uint32_t e, uint32_t x) {
  if (b >= e || a[b] >= x) return b;
  uint32_t lo = b, step = 1;   // a[lo] < x
  while (lo + step < e && a[lo + step] < x) {
    lo += step;
    step <<= 1;
  }
  return lower_bound_u32(a, lo + 1, min(lo + step, e), x);
}

__device__ __forceinline__ uint32_t rank_select(const unsigned long long* bm, const uint32_t* pre, uint32_t nwords,
                                                uint32_t r) {
  // the k whose rank is r: the word holding the r-th set bit, then the bit
  uint32_t w = 0, n = nwords;
  while (n > 1) {
    const uint32_t half = n >> 1;
    w = (pre[w + half] <= r) ? w + half : w;
    n -= half;
  }
  uint64_t word = bm[w];
  for (uint32_t i = pre[w]; i < r; i++) word &= word - 1;
  return w * 64 + (uint32_t)__builtin_ctzll(word);
}

__global__ __launch_bounds__(B_NT) void k_batch_heavy(BatchArgs a) {
  __shared__ unsigned long long bm[KW_MAX / 64];   // k the row touches in the window
  __shared__ uint32_t pre[KW_MAX / 64];            // set bits before each word
  __shared__ uint32_t sk[HC];
  __shared__ unsigned long long scnt[HC];
  __shared__ long long sdig[HC * DSTRIDE];
  __shared__ uint32_t s_item, s_klo, s_khi;
  __shared__ uint32_t s_wsum[B_NW];
  // products of a batch of B_NT entries of A's row, numbered by a block
  // scan so that every thread takes an equal share (E's rows have skewed
  // lengths, and one thread per entry would wait on the longest)
  __shared__ uint32_t s_off[B_NT], s_kb[B_NT], s_ab[B_NT], s_ae[B_NT];
  __shared__ uint32_t s_cur[CUR_MAX], s_cend[CUR_MAX];   // per entry of A: its E row, from the next window on
  const int tid = threadIdx.x;
  uint32_t bad = 0;
  // owner of product idx: the last entry whose first product is <= idx
  auto owner = [&](uint32_t idx) {
    uint32_t lo = 0, n = B_NT;
    while (n > 1) {
      const uint32_t half = n >> 1;
      lo = (s_off[lo + half] <= idx) ? lo + half : lo;
      n -= half;
    }
    return lo;
  };
  for (uint32_t sl = tid; sl < HC; sl += B_NT) {
    scnt[sl] = 0;
#pragma unroll
    for (int d = 0; d < EXACT_MAXD; d++) sdig[sl * DSTRIDE + d] = 0;
  }
  for (;;) {
    if (tid == 0) s_item = atomicAdd(&a.qhead[0], 1u);
    __syncthreads();
    // uniform across the block: the row's descriptor goes to scalar registers
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= a.n_heavy) break;
    const uint32_t t = __builtin_amdgcn_readfirstlane(a.heavy[item]);
    const BInst I = a.inst[a.row_inst[t]];
    const uint32_t p = t - (uint32_t)a.inst_row0[a.row_inst[t]];
    const uint32_t qb = I.a_off[p], qe = I.a_off[p + 1];
    const uint64_t out = a.ub_off[t];
    const bool bounded = a.prod[t] < BOUNDED_PRODUCTS;
    uint32_t nnz = 0;
    for (uint32_t w0 = 0; w0 < I.n_k; w0 += a.kw) {
      const uint32_t wend = min(w0 + a.kw, I.n_k);
      const uint32_t nwords = (wend - w0 + 63) / 64;
      for (uint32_t sl = tid; sl < nwords; sl += B_NT) bm[sl] = 0;
      __syncthreads();
      for (uint32_t qs = qb; qs < qe; qs += B_NT) {
        const uint32_t q = qs + tid;
        uint32_t cnt = 0, kb = 0;
        uint32_t pe;
        if (q < qe && find_j(I, I.a_j[q], pe)) {
          kb = I.e_off[pe];
          uint32_t kend = I.e_off[pe + 1];
          if (I.n_k > a.kw) {
            kb = lower_bound_u32(I.e_k, kb, kend, w0);
            kend = lower_bound_u32(I.e_k, kb, kend, wend);
          }
          cnt = kend - kb;
        }
        uint32_t tot;
        const uint32_t off = block_excl_scan<uint32_t, B_NT>(cnt, s_wsum, tot);
        s_off[tid] = off;
        s_kb[tid] = kb;
        __syncthreads();
        for (uint32_t idx = tid; idx < tot; idx += B_NT) {
          const uint32_t o = owner(idx);
          const uint32_t k = I.e_k[s_kb[o] + (idx - s_off[o])] - w0;
          atomicOr(&bm[k >> 6], 1ull << (k & 63u));
        }
        __syncthreads();
      }
      uint32_t m;
      {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const uint32_t wi = 4 * tid + i;
          c += wi < nwords ? (uint32_t)__popcll(bm[wi]) : 0u;
        }
        uint32_t r = block_excl_scan<uint32_t, B_NT>(c, s_wsum, m);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const uint32_t wi = 4 * tid + i;
          if (wi < nwords) {
            pre[wi] = r;
            r += (uint32_t)__popcll(bm[wi]);
          }
        }
      }
      // cursors: several rank windows over one k window, few enough entries
      const bool cursors = m > HC && I.n_k <= a.kw && qe - qb <= CUR_MAX;
      if (cursors) {
        for (uint32_t q = qb + tid; q < qe; q += B_NT) {
          uint32_t pe, b = 0, e = 0;
          if (find_j(I, I.a_j[q], pe)) {
            b = I.e_off[pe];
            e = I.e_off[pe + 1];
          }
          s_cur[q - qb] = b;
          s_cend[q - qb] = e;
        }
      }
      __syncthreads();
      for (uint32_t r0 = 0; r0 < m; r0 += HC) {
        if (tid == 0) {
          s_klo = rank_select(bm, pre, nwords, r0);
          s_khi = r0 + HC < m ? rank_select(bm, pre, nwords, r0 + HC) : wend - w0;
        }
        __syncthreads();
        const uint32_t klo = s_klo + w0, khi = s_khi + w0;
        for (uint32_t qs = qb; qs < qe; qs += B_NT) {
          const uint32_t q = qs + tid;
          uint32_t cnt = 0, kb = 0, ab = 0, ae = 0;
          uint32_t pe;
          if (cursors) {
            if (q < qe) {
              // this thread alone reads and advances entry q's cursor
              kb = s_cur[q - qb];
              const uint32_t kend = gallop_lower_bound(I.e_k, kb, s_cend[q - qb], khi);
              s_cur[q - qb] = kend;
              cnt = kend - kb;
              if (cnt) rows_of(I.a_run, q, ab, ae);
            }
          } else if (q < qe && find_j(I, I.a_j[q], pe)) {
            rows_of(I.a_run, q, ab, ae);
            kb = I.e_off[pe];
            uint32_t kend = I.e_off[pe + 1];
            if (m > HC || I.n_k > a.kw) {
              kb = lower_bound_u32(I.e_k, kb, kend, klo);
              kend = lower_bound_u32(I.e_k, kb, kend, khi);
            }
            cnt = kend - kb;
          }
          uint32_t tot;
          const uint32_t off = block_excl_scan<uint32_t, B_NT>(cnt, s_wsum, tot);
          s_off[tid] = off;
          s_kb[tid] = kb;
          s_ab[tid] = ab;
          s_ae[tid] = ae;
          __syncthreads();
          for (uint32_t idx = tid; idx < tot; idx += B_NT) {
            const uint32_t own = owner(idx);
            const uint32_t kp = s_kb[own] + (idx - s_off[own]);
            const uint32_t ab = s_ab[own], ae = s_ae[own];
            const uint32_t k = I.e_k[kp] - w0;
            const uint64_t word = bm[k >> 6];
            const uint32_t sl = pre[k >> 6] + (uint32_t)__popcll(word & ((1ull << (k & 63u)) - 1ull)) - r0;
            sk[sl] = k + w0;
            uint32_t eb, ee;
            rows_of(I.e_run, kp, eb, ee);
            atomicAdd(&scnt[sl], (unsigned long long)(ae - ab) * (ee - eb));
            if (I.sum)
              for (uint32_t ra = ab; ra < ae; ra++)
                for (uint32_t re = eb; re < ee; re++) {
                  double hi, lo;
                  two_prod(I.a_val[ra], I.e_val[re], hi, lo);
                  bool ok = lds_add_term(sdig + sl * DSTRIDE, hi, I.lsb, I.D, bounded);
                  ok = lds_add_term(sdig + sl * DSTRIDE, lo, I.lsb, I.D, bounded) && ok;
                  if (!ok) bad = 1;
                }
          }
          __syncthreads();
        }
        __syncthreads();
        const uint32_t nw = min(HC, m - r0);
        for (uint32_t sl = tid; sl < nw; sl += B_NT) {
          const uint64_t o = out + nnz + r0 + sl;
          a.ub_k[o] = sk[sl];
          a.ub_cnt[o] = scnt[sl];
          if (I.sum) a.ub_sum[o] = lds_round(sdig + sl * DSTRIDE, I.D, I.lsb, bounded, a.err);
          scnt[sl] = 0;
#pragma unroll
          for (int d = 0; d < EXACT_MAXD; d++) sdig[sl * DSTRIDE + d] = 0;
        }
        __syncthreads();
      }
      nnz += m;
    }
    if (tid == 0) a.row_nnz[t] = nnz;
  }
  if (bad) atomicOr(a.err, 1u);
}

// Inner-product rows: one block per row.  A's row is marked in an LDS
// bitmap over j with per-word rank prefixes (the position of j in the row).
// E transposed is then streamed chunk by chunk (256 columns k at a time):
// the block's threads take the chunk's (k, j) entries in order, coalesced
// and independent, probe j in the bitmap, and add each matching product's
// exact digits to its column's LDS accumulator (the column found by
// bisecting the chunk's offsets); the columns are then emitted in k order
// and their accumulators cleared.
__global__ __launch_bounds__(B_NT) void k_batch_inner(BatchArgs a) {
  __shared__ unsigned long long bm[KW_MAX / 64];
  __shared__ uint32_t pre[KW_MAX / 64];
  __shared__ uint32_t soff[B_NT + 1];                 // the chunk's column offsets
  __shared__ unsigned long long ccnt[B_NT];           // per column of the chunk
  __shared__ long long cdig[B_NT * DSTRIDE];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_wsum[B_NW];
  const int tid = threadIdx.x;
  uint32_t bad = 0;
  ccnt[tid] = 0;
#pragma unroll
  for (int d = 0; d < EXACT_MAXD; d++) cdig[tid * DSTRIDE + d] = 0;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(&a.qhead[2], 1u);
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= a.n_inner) break;
    const uint32_t t = __builtin_amdgcn_readfirstlane(a.inner[item]);
    const BInst I = a.inst[a.row_inst[t]];
    const uint32_t p = t - (uint32_t)a.inst_row0[a.row_inst[t]];
    const uint32_t qb = I.a_off[p], qe = I.a_off[p + 1];
    const bool bounded = a.prod[t] < BOUNDED_PRODUCTS;
    const uint32_t nwords = (I.n_j + 63) / 64;
    for (uint32_t s = tid; s < nwords; s += B_NT) bm[s] = 0;
    __syncthreads();
    for (uint32_t q = qb + tid; q < qe; q += B_NT) {
      const uint32_t j = I.a_j[q];
      atomicOr(&bm[j >> 6], 1ull << (j & 63u));
    }
    __syncthreads();
    {
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint32_t wi = 4 * tid + i;
        c += wi < nwords ? (uint32_t)__popcll(bm[wi]) : 0u;
      }
      uint32_t tot;
      uint32_t r = block_excl_scan<uint32_t, B_NT>(c, s_wsum, tot);
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint32_t wi = 4 * tid + i;
        if (wi < nwords) {
          pre[wi] = r;
          r += (uint32_t)__popcll(bm[wi]);
        }
      }
    }
    const uint64_t out = a.ub_off[t];
    uint32_t nnz = 0;
    for (uint32_t kb0 = 0; kb0 < I.bt_n0; kb0 += B_NT) {
      const uint32_t nk = min((uint32_t)B_NT, I.bt_n0 - kb0);
      soff[tid] = I.bt_off[kb0 + min((uint32_t)tid, nk)];
      if (tid == 0) soff[B_NT] = I.bt_off[kb0 + nk];
      __syncthreads();
      const uint32_t e0 = soff[0], e1 = soff[nk];
      // four entries per thread per round: their loads are independent and
      // in flight together (few entries match, so the loop is load latency)
      constexpr uint32_t UNR = 4;
      for (uint32_t eb = e0 + tid; eb < e1; eb += UNR * B_NT) {
        uint32_t jv[UNR];
#pragma unroll
        for (uint32_t u = 0; u < UNR; u++) {
          const uint32_t e = eb + u * B_NT;
          jv[u] = e < e1 ? I.bt_j[e] : UINT32_MAX;
        }
#pragma unroll
        for (uint32_t u = 0; u < UNR; u++) {
        const uint32_t e = eb + u * B_NT;
        const uint32_t j = jv[u];
        if (j >= I.n_j) continue;
        const uint64_t word = bm[j >> 6];
        if (!((word >> (j & 63u)) & 1ull)) continue;
        // column of entry e: the last c with soff[c] <= e
        uint32_t c = 0, n = nk;
        while (n > 1) {
          const uint32_t half = n >> 1;
          c = (soff[c + half] <= e) ? c + half : c;
          n -= half;
        }
        const uint32_t q = qb + pre[j >> 6] + (uint32_t)__popcll(word & ((1ull << (j & 63u)) - 1ull));
        uint32_t ab, ae, eb, ee;
        rows_of(I.a_run, q, ab, ae);
        rows_of(I.bt_run, e, eb, ee);
        atomicAdd(&ccnt[c], (unsigned long long)(ae - ab) * (ee - eb));
        if (I.sum)
          for (uint32_t ra = ab; ra < ae; ra++)
            for (uint32_t re = eb; re < ee; re++) {
              double hi, lo;
              two_prod(I.a_val[ra], I.bt_val[re], hi, lo);
              bool ok = lds_add_term(cdig + c * DSTRIDE, hi, I.lsb, I.D, bounded);
              ok = lds_add_term(cdig + c * DSTRIDE, lo, I.lsb, I.D, bounded) && ok;
              if (!ok) bad = 1;
            }
        }
      }
      __syncthreads();
      const uint64_t cnt = (uint32_t)tid < nk ? ccnt[tid] : 0ull;
      uint32_t tot;
      const uint32_t r = block_excl_scan<uint32_t, B_NT>(cnt ? 1u : 0u, s_wsum, tot);
      if (cnt) {
        const uint64_t o = out + nnz + r;
        a.ub_k[o] = I.bt_k[kb0 + tid];
        a.ub_cnt[o] = cnt;
        if (I.sum) a.ub_sum[o] = lds_round(cdig + tid * DSTRIDE, I.D, I.lsb, bounded, a.err);
      }
      ccnt[tid] = 0;
#pragma unroll
      for (int d = 0; d < EXACT_MAXD; d++) cdig[tid * DSTRIDE + d] = 0;
      nnz += tot;
      __syncthreads();
    }
    if (tid == 0) a.row_nnz[t] = nnz;
    __syncthreads();
  }
  if (bad) atomicOr(a.err, 1u);
}

constexpr uint32_t LIGHT_GRAB = 32;

// Light rows: one wave per row, private LDS hash of HS slots.
template <int HS>
__global__ __launch_bounds__(B_NT) void k_batch_light(BatchArgs a) {
  constexpr int SLOT_BYTES = 4 + 8 + 8 * EXACT_MAXD + 2;
  constexpr uint32_t HS_SHIFT = HS == 128 ? 25 : 24;  // top bits of the multiplicative hash
  static_assert(HS == 128 || HS == 256, "hash size");
  __shared__ __align__(16) unsigned char lds[B_NW * HS * SLOT_BYTES];
  const int tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
  uint32_t bad = 0;
  uint32_t* hk = (uint32_t*)(lds + w * HS * SLOT_BYTES);
  unsigned long long* hc = (unsigned long long*)(hk + HS);
  long long* hd = (long long*)(hc + HS);
  uint16_t* hl = (uint16_t*)(hd + HS * EXACT_MAXD);
  // Light rows are claimed LIGHT_GRAB at a time: one atomic on the queue
  // head per claim (a head taken once per row serializes millions of rows).
  uint32_t item = 0, item_end = 0;
  for (;;) {
    if (item == item_end) {
      uint32_t g = 0;
      if (lane == 0) g = atomicAdd(&a.qhead[1], LIGHT_GRAB);
      item = __builtin_amdgcn_readfirstlane(__shfl(g, 0, WAVE));
      item_end = (uint32_t)min<uint64_t>((uint64_t)item + LIGHT_GRAB, a.n_light);
    }
    if (item >= a.n_light) break;
    const uint32_t t = __builtin_amdgcn_readfirstlane(a.light[item]);
    item++;
    const BInst I = a.inst[a.row_inst[t]];
    const uint32_t p = t - (uint32_t)a.inst_row0[a.row_inst[t]];
    const uint32_t qb = I.a_off[p], qe = I.a_off[p + 1];
    const uint64_t out = a.ub_off[t];
    if (I.kind == 0) {
      // vector: one output per row, reduced across the wave
      RegAcc acc;
      acc.clear();
      uint64_t cnt = 0;
      for (uint32_t q = qb + lane; q < qe; q += WAVE) {
        uint32_t pe;
        if (!find_j(I, I.a_j[q], pe)) continue;
        uint32_t ab, ae, eb, ee;
        rows_of(I.a_run, q, ab, ae);
        rows_of(I.e_run, pe, eb, ee);
        cnt += (uint64_t)(ae - ab) * (ee - eb);
        if (I.sum)
          for (uint32_t ra = ab; ra < ae; ra++)
            for (uint32_t re = eb; re < ee; re++) {
              double hi, lo;
              two_prod(I.a_val[ra], I.e_val[re], hi, lo);
              bool ok = acc.add(hi, I.lsb, I.D, 1);
              ok = acc.add(lo, I.lsb, I.D, 1) && ok;
              if (!ok) bad = 1;
            }
      }
      if (I.sum) acc.normalize(I.D);
      cnt = wave_sum(cnt);
      int64_t tot[EXACT_MAXD];
#pragma unroll
      for (int s = 0; s < EXACT_MAXD; s++) tot[s] = wave_sum(acc.s[s]);
      if (lane == 0) {
        if (cnt) {
          a.ub_k[out] = 0;
          a.ub_cnt[out] = cnt;
          if (I.sum) a.ub_sum[out] = exact_round(tot, I.D, I.lsb, a.err);
        }
        a.row_nnz[t] = cnt ? 1u : 0u;
      }
      continue;
    }
    // matrix: hash the row's products by k
    const bool bounded = a.prod[t] < BOUNDED_PRODUCTS;
    for (int s = lane; s < HS; s += WAVE) {
      hk[s] = EMPTY_KEY;
      hc[s] = 0;
#pragma unroll
      for (int d = 0; d < EXACT_MAXD; d++) hd[s * EXACT_MAXD + d] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // The row's products are spread over the lanes: per chunk of 64 A
    // entries, a scan of their B-row lengths numbers the products, and
    // each lane takes products f, f + 64, ... (finding its A entry by
    // bisecting the scan across lanes), so all loads are independent.
    for (uint32_t c0 = qb; c0 < qe; c0 += WAVE) {
      const uint32_t q = c0 + lane;
      uint32_t pe = 0, len = 0, kb = 0;
      if (q < qe && find_j(I, I.a_j[q], pe)) {
        kb = I.e_off[pe];
        len = I.e_off[pe + 1] - kb;
      }
      const uint32_t incl = wave_incl_scan(len);
      const uint32_t start = incl - len;
      const uint32_t total = (uint32_t)__shfl((int)incl, WAVE - 1, WAVE);
      for (uint32_t f0 = 0; f0 < total; f0 += WAVE) {   // uniform: every lane takes part in the shuffles
        const uint32_t f = f0 + lane;
        // owner: the last lane whose start <= f (lanes with len 0 share a start)
        uint32_t src = 0, n = WAVE;
#pragma unroll
        for (int step = 0; step < 6; step++) {
          const uint32_t half = n >> 1;
          const uint32_t st = (uint32_t)__shfl((int)start, (int)(src + half), WAVE);
          src = st <= f ? src + half : src;
          n -= half;
        }
        const uint32_t kbs = (uint32_t)__shfl((int)kb, (int)src, WAVE);
        const uint32_t sts = (uint32_t)__shfl((int)start, (int)src, WAVE);
        if (f >= total) continue;
        const uint32_t qq = c0 + src;
        const uint32_t kp = kbs + (f - sts);
        uint32_t ab, ae;
        rows_of(I.a_run, qq, ab, ae);
        const uint32_t k = I.e_k[kp];
        uint32_t slot = (k * 2654435761u) >> HS_SHIFT;
        for (;;) {
          const uint32_t prev = atomicCAS(&hk[slot], EMPTY_KEY, k);
          if (prev == EMPTY_KEY || prev == k) break;
          slot = (slot + 1) & (HS - 1);
        }
        uint32_t eb, ee;
        rows_of(I.e_run, kp, eb, ee);
        atomicAdd(&hc[slot], (unsigned long long)(ae - ab) * (ee - eb));
        if (I.sum)
          for (uint32_t ra = ab; ra < ae; ra++)
            for (uint32_t re = eb; re < ee; re++) {
              double hi, lo;
              two_prod(I.a_val[ra], I.e_val[re], hi, lo);
              bool ok = lds_add_term(hd + slot * EXACT_MAXD, hi, I.lsb, I.D, bounded);
              ok = lds_add_term(hd + slot * EXACT_MAXD, lo, I.lsb, I.D, bounded) && ok;
              if (!ok) bad = 1;
            }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // list the occupied slots, then place each by its rank in k order
    uint32_t m = 0;
    for (int s0 = 0; s0 < HS; s0 += WAVE) {
      const bool occ = hk[s0 + lane] != EMPTY_KEY;
      const uint64_t bal = ballot(occ);
      if (occ) hl[m + lanes_below(bal)] = (uint16_t)(s0 + lane);
      m += (uint32_t)__popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // rank of each listed key among the listed keys: lane holds entries
    // lane + 64 c in registers; every key is broadcast once by a shuffle
    constexpr int NC = HS / WAVE;
    uint32_t kk[NC], ss[NC], rk[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      const uint32_t f = c * WAVE + lane;
      ss[c] = f < m ? hl[f] : 0u;
      kk[c] = f < m ? hk[ss[c]] : EMPTY_KEY;
      rk[c] = 0;
    }
#pragma unroll
    for (int c2 = 0; c2 < NC; c2++) {
      if ((uint32_t)c2 * WAVE >= m) break;
      const uint32_t n2 = min((uint32_t)WAVE, m - (uint32_t)c2 * WAVE);
      for (uint32_t j = 0; j < n2; j++) {
        const uint32_t kf = (uint32_t)__shfl((int)kk[c2], (int)j, WAVE);
#pragma unroll
        for (int c = 0; c < NC; c++) rk[c] += kf < kk[c] ? 1u : 0u;
      }
    }
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if ((uint32_t)c * WAVE + lane >= m) continue;
      const uint32_t s = ss[c];
      const uint64_t o = out + rk[c];
      a.ub_k[o] = kk[c];
      a.ub_cnt[o] = hc[s];
      if (I.sum) a.ub_sum[o] = lds_round(hd + s * EXACT_MAXD, I.D, I.lsb, bounded, a.err);
    }
    if (lane == 0) a.row_nnz[t] = m;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (bad) atomicOr(a.err, 1u);
}

// Copy each row's outputs from its upper-bound slots to the packed result.
struct PackArgs2 {
  const BInst* inst;
  const uint32_t* row_inst;
  const uint64_t* inst_row0;
  const uint64_t* ub_off;
  const uint64_t* out_off;   // exclusive scan of row_nnz
  const uint32_t* ub_k;
  const uint64_t* ub_cnt;
  const double* ub_sum;
  uint32_t* out_i;
  uint32_t* out_k;
  uint64_t* out_cnt;
  double* out_sum;
  uint64_t R;
};

// A wave takes 64 consecutive rows: lane l loads row t0 + l's offsets, its
// instance and its i, then the wave copies the rows' outputs as one flat
// range (the rows' packed outputs are contiguous), each lane finding the
// row of its output by bisecting the rows' output offsets across the
// lanes.  Every lane does useful copies whatever the rows' lengths.
__global__ void k_pack_rows(PackArgs2 a) {
  const int lane = lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / WAVE);
  for (uint64_t t0 = ((uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * WAVE; t0 < a.R;
       t0 += nw * WAVE) {
    const uint64_t t = t0 + lane;
    const bool row = t < a.R;
    // lanes past the last row start where the group ends
    const uint64_t oo = a.out_off[row ? t : a.R];
    const uint64_t base = a.out_off[t0], end = a.out_off[min<uint64_t>(t0 + WAVE, a.R)];
    uint32_t iv = 0, flags = 0;
    uint64_t uo = 0;
    if (row) {
      const uint32_t ii = a.row_inst[t];
      const BInst& I = a.inst[ii];
      iv = I.a_i[t - a.inst_row0[ii]];
      flags = (I.kind == 1 ? 1u : 0u) | (I.sum ? 2u : 0u);
      uo = a.ub_off[t];
    }
    if (end - base >= (1ull << 32)) {
      // more than 2^32 outputs in the group: row by row
      for (int l = 0; l < WAVE; l++) {
        const uint64_t o0 = (uint64_t)__shfl((long long)oo, l, WAVE);
        const uint64_t o1 = l + 1 < WAVE ? (uint64_t)__shfl((long long)oo, l + 1, WAVE) : end;
        const uint64_t u0 = (uint64_t)__shfl((long long)uo, l, WAVE);
        const uint32_t il = (uint32_t)__shfl((int)iv, l, WAVE), fl = (uint32_t)__shfl((int)flags, l, WAVE);
        for (uint64_t e = o0 + lane; e < o1; e += WAVE) {
          a.out_i[e] = il;
          if (fl & 1u) a.out_k[e] = a.ub_k[u0 + (e - o0)];
          a.out_cnt[e] = a.ub_cnt[u0 + (e - o0)];
          if (fl & 2u) a.out_sum[e] = a.ub_sum[u0 + (e - o0)];
        }
      }
      continue;
    }
    const uint32_t rel = (uint32_t)(oo - base);
    const uint32_t uo_lo = (uint32_t)uo, uo_hi = (uint32_t)(uo >> 32);
    for (uint64_t e0 = base; e0 < end; e0 += WAVE) {   // uniform: every lane takes part in the shuffles
      const uint64_t e = e0 + (uint64_t)lane;
      const uint32_t re = (uint32_t)(e - base);
      // the row of output e: the last lane whose first output is <= e
      uint32_t src = 0;
#pragma unroll
      for (int step = WAVE / 2; step > 0; step >>= 1) {
        const uint32_t r = (uint32_t)__shfl((int)rel, (int)(src + step), WAVE);
        src = r <= re ? src + step : src;
      }
      const uint32_t rs = (uint32_t)__shfl((int)rel, (int)src, WAVE);
      const uint32_t is = (uint32_t)__shfl((int)iv, (int)src, WAVE);
      const uint32_t fs = (uint32_t)__shfl((int)flags, (int)src, WAVE);
      const uint64_t us = (uint64_t)(uint32_t)__shfl((int)uo_lo, (int)src, WAVE) |
                          ((uint64_t)(uint32_t)__shfl((int)uo_hi, (int)src, WAVE) << 32);
      if (e >= end) continue;
      const uint64_t u = us + (re - rs);
      a.out_i[e] = is;
      if (fs & 1u) a.out_k[e] = a.ub_k[u];
      a.out_cnt[e] = a.ub_cnt[u];
      if (fs & 2u) a.out_sum[e] = a.ub_sum[u];
    }
  }
}

// Join tuples of each instance (one block per instance): the sum of its
// rows' product counts, which is the sum of its output counts.
__global__ void k_inst_sums(const uint64_t* prod, const uint64_t* row0, uint64_t* out) {
  __shared__ uint64_t red[B_NW];
  uint64_t s = 0;
  for (uint64_t t = row0[blockIdx.x] + threadIdx.x; t < row0[blockIdx.x + 1]; t += blockDim.x) s += prod[t];
  s = block_sum<uint64_t, B_NT>(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Packed output offsets at the instances' first rows (n + 1 of them).
__global__ void k_inst_offsets(const uint64_t* out_off, const uint64_t* row0, uint32_t n, uint64_t* dst) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
    dst[i] = out_off[row0[i]];
}

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 256 * 64));
}

// ---- host side ----------------------------------------------------------------

struct Tuning {
  uint32_t light_max = 128;   // products above which a matrix row is heavy (light hash: 2x slots)
  uint32_t blocks_per_cu = 2; // persistent grid
  uint32_t inner_ratio = 16;  // heavy row in inner-product form when products * ratio >= nnz(E)
};

// E transposed (levels k, j) of every matrix instance, built once per batch
// and shared by the autotuner's candidate setups; keyed by E's trie and
// annotation column.
struct Transposes {
  std::map<std::pair<const lh_trie*, int32_t>, lh_trie*> by_e;
  ~Transposes() {
    for (auto& kv : by_e) free_trie(kv.second);
  }
};
constexpr uint32_t MAX_BLOCKS_PER_CU = 4;

// Everything one batch needs; kept across calls with the same plans so the
// graph is replayed rather than rebuilt.
struct BatchState {
  std::vector<const lh_plan_t*> plans;
  Tuning tune;
  uint64_t R = 0, UB = 0;
  hipStream_t s = nullptr;
  DBuf<BInst> inst;
  DBuf<uint64_t> inst_row0, prod, ub_off;
  std::vector<uint64_t> h_nj;   // join tuples per instance (fixed by the plans)
  DBuf<uint32_t> row_inst, ub, heavy_f, light_f, inner_f, heavy, light, inner, qhead, row_nnz, ub_k, err;
  std::shared_ptr<Transposes> tr;
  DBuf<uint64_t> ub_cnt;
  DBuf<double> ub_sum;
  uint32_t kw = 64;
  uint64_t n_heavy = 0, n_light = 0, n_inner = 0;
  std::vector<uint64_t> h_inst_row0;
  std::vector<BInst> h_inst;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  ~BatchState() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

std::mutex g_batch_mu;
std::unique_ptr<BatchState> g_batch;

BInst describe(const lh_plan_t* p) {
  const PlanAtom& A = p->atoms[0];
  const PlanAtom& E = p->atoms[1];
  const lh_trie* ta = A.trie;
  const lh_trie* te = E.trie;
  BInst b{};
  b.kind = E.n_levels == 1 ? 0u : 1u;
  b.n_rows = (uint32_t)ta->lv[0].n;
  b.a_i = ta->lv[0].keys.p;
  b.a_off = ta->lv[0].offs.p;
  b.a_j = ta->lv[1].keys.p;
  b.a_run = A.bag ? ta->lv[1].offs.p : nullptr;
  b.sum = p->agg == LH_AGG_SUM ? 1u : 0u;
  b.a_val = (b.sum && A.anno >= 0) ? ta->annos[A.anno].p : nullptr;
  b.e_j = te->lv[0].keys.p;
  b.e_n0 = (uint32_t)te->lv[0].n;
  // distinct sorted keys, as many as the largest key + 1: exactly 0 .. n - 1
  b.e_dense = (b.e_n0 > 0 && (uint64_t)te->key_max[0] + 1 == te->lv[0].n) ? 1u : 0u;
  b.e_pool = te->lv[0].pool.p;
  b.e_bsw = UINT64_MAX;
  b.e_bsb = 0;
  if (b.e_n0) {
    LH_HIP(hipMemcpy(&b.e_bsw, te->lv[0].bs_word.p, sizeof(uint64_t), hipMemcpyDeviceToHost));
    LH_HIP(hipMemcpy(&b.e_bsb, te->lv[0].bs_base.p, sizeof(uint32_t), hipMemcpyDeviceToHost));
  }
  if (b.kind == 1) {
    b.e_off = te->lv[0].offs.p;
    b.e_k = te->lv[1].keys.p;
    b.n_k = te->key_max[1] + 1;
  }
  b.e_run = E.bag ? te->lv[E.n_levels - 1].offs.p : nullptr;
  b.e_val = (b.sum && E.anno >= 0) ? te->annos[E.anno].p : nullptr;
  b.lsb = p->exact_lsb;
  b.D = p->exact_digits;
  b.n_j = ta->key_max[1] + 1;
  return b;
}

// E transposed: the same rows keyed (k, j), bag semantics, sorted arrays.
lh_trie* transpose_e(const lh_trie* te, int32_t anno, hipStream_t s) {
  const uint32_t* keys[2] = {row_keys(te, 0), row_keys(te, 1)};
  const double* annos[1] = {anno >= 0 ? te->annos[anno].p : nullptr};
  const uint32_t level_order[2] = {1, 0};
  return build_trie(te->n_rows, 2, keys, anno >= 0 ? 1u : 0u, annos, 0, nullptr, level_order,
                    LH_BAG | LH_LAYOUT_UINT, nullptr, 0, s);
}

void attach_transpose(BInst& b, const lh_plan_t* p, Transposes& tr, hipStream_t s) {
  const PlanAtom& E = p->atoms[1];
  const int32_t anno = b.sum ? E.anno : -1;
  auto key = std::make_pair(E.trie, anno);
  auto it = tr.by_e.find(key);
  if (it == tr.by_e.end()) it = tr.by_e.emplace(key, transpose_e(E.trie, anno, s)).first;
  const lh_trie* t = it->second;
  b.bt_n0 = (uint32_t)t->lv[0].n;
  b.bt_k = t->lv[0].keys.p;
  b.bt_off = t->lv[0].offs.p;
  b.bt_j = t->lv[1].keys.p;
  b.bt_run = t->lv[1].offs.p;
  b.bt_val = anno >= 0 ? t->annos[0].p : nullptr;
  b.nnz_e = t->lv[1].n;
}

std::string cache_path() {
  const char* e = std::getenv("LH_AUTOTUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/lh_autotune.txt";
}

std::string signature(const BatchState& b) {
  hipDeviceProp_t prop;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  std::ostringstream os;
  uint64_t rows_log = 0, ub_log = 0;
  while ((1ull << rows_log) < b.R) rows_log++;
  while ((1ull << ub_log) < b.UB) ub_log++;
  os << "v4_" << prop.gcnArchName << "_cu" << prop.multiProcessorCount << "_inst" << b.plans.size() << "_r" << rows_log
     << "_u" << ub_log;
  return os.str();
}

bool load_tuning(const std::string& sig, Tuning& t) {
  std::ifstream f(cache_path());
  std::string key;
  Tuning x;
  while (f >> key >> x.light_max >> x.blocks_per_cu >> x.inner_ratio) {
    if (key == sig) {
      t = x;
      return true;
    }
  }
  return false;
}

void save_tuning(const std::string& sig, const Tuning& t) {
  std::string path = cache_path();
  std::error_code ec;  // an unwritable cache only costs the next run a re-tune
  std::filesystem::create_directories(std::filesystem::path(path).parent_path(), ec);
  std::ofstream f(path, std::ios::app);
  f << sig << " " << t.light_max << " " << t.blocks_per_cu << " " << t.inner_ratio << "\n";
}

void setup(BatchState& b, hipStream_t s) {
  const uint32_t n = (uint32_t)b.plans.size();
  b.s = s;
  b.h_inst.resize(n);
  b.h_inst_row0.assign(n + 1, 0);
  if (!b.tr) b.tr = std::make_shared<Transposes>();
  for (uint32_t i = 0; i < n; i++) {
    b.h_inst[i] = describe(b.plans[i]);
    if (b.h_inst[i].kind == 1) attach_transpose(b.h_inst[i], b.plans[i], *b.tr, s);
    b.h_inst[i].row_base = b.h_inst_row0[i];
    b.h_inst_row0[i + 1] = b.h_inst_row0[i] + b.h_inst[i].n_rows;
  }
  b.R = b.h_inst_row0[n];
  if (b.R >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "batch: more than 2^32 rows");
  b.inst.alloc(n, s);
  LH_HIP(hipMemcpyAsync(b.inst.p, b.h_inst.data(), n * sizeof(BInst), hipMemcpyHostToDevice, s));
  b.inst_row0.alloc(n + 1, s);
  LH_HIP(hipMemcpyAsync(b.inst_row0.p, b.h_inst_row0.data(), (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  b.row_inst.alloc(b.R, s);
  b.prod.alloc(b.R, s);
  b.ub.alloc(b.R, s);
  b.heavy_f.alloc(b.R, s);
  b.light_f.alloc(b.R, s);
  b.inner_f.alloc(b.R, s);
  if (b.R) {
    k_row_setup<<<grid_for(b.R), 256, 0, s>>>(b.inst.p, b.inst_row0.p, n, b.R, b.tune.light_max, b.tune.inner_ratio,
                                              b.row_inst.p, b.prod.p, b.ub.p, b.heavy_f.p, b.light_f.p, b.inner_f.p);
    LH_HIP(hipGetLastError());
  }
  b.ub_off.alloc(b.R + 1, s);
  b.UB = scan_u32_to_u64(b.ub.p, b.ub_off.p, b.R, s);
  b.h_nj.assign(n, 0);
  if (n) {
    DBuf<uint64_t> dnj(n, s);
    k_inst_sums<<<n, B_NT, 0, s>>>(b.prod.p, b.inst_row0.p, dnj.p);
    LH_HIP(hipGetLastError());
    LH_HIP(hipMemcpyAsync(b.h_nj.data(), dnj.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
  }
  b.heavy.alloc(b.R, s);
  b.light.alloc(b.R, s);
  b.n_heavy = select_flagged(b.heavy_f.p, b.R, b.heavy.p, s);
  b.n_light = select_flagged(b.light_f.p, b.R, b.light.p, s);
  b.inner.alloc(b.R, s);
  b.n_inner = select_flagged(b.inner_f.p, b.R, b.inner.p, s);   // in row order: grouped by instance
  // heavy rows longest first (LPT): sort their ids by descending product count
  if (b.n_heavy > 1) {
    DBuf<uint64_t> key(b.n_heavy, s), tk(b.n_heavy, s);
    DBuf<uint32_t> tv(b.n_heavy, s);
    std::vector<uint32_t> hrows(b.n_heavy);
    std::vector<uint64_t> hp(b.R);
    LH_HIP(hipMemcpyAsync(hrows.data(), b.heavy.p, b.n_heavy * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    LH_HIP(hipMemcpyAsync(hp.data(), b.prod.p, b.R * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
    std::stable_sort(hrows.begin(), hrows.end(), [&](uint32_t x, uint32_t y) { return hp[x] > hp[y]; });
    LH_HIP(hipMemcpyAsync(b.heavy.p, hrows.data(), b.n_heavy * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  }
  b.qhead.alloc(3, s);
  b.row_nnz.alloc(b.R, s);
  b.ub_k.alloc(b.UB, s);
  b.ub_cnt.alloc(b.UB, s);
  b.ub_sum.alloc(b.UB, s);
  b.err.alloc(1, s);
  // heavy rows: the window of k values their bitmap covers
  {
    uint32_t nk = 0;
    for (const BInst& I : b.h_inst)
      if (I.kind == 1) nk = std::max(nk, I.n_k);
    b.kw = std::max<uint32_t>(64, std::min<uint32_t>(KW_MAX, (nk + 63) / 64 * 64));
  }
  LH_HIP(hipStreamSynchronize(s));
}

void launch_compute(BatchState& b, hipStream_t s) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  k_fill_u32_dev<<<1, 64, 0, s>>>(b.qhead.p, 0u, 3);
  k_fill_u32_dev<<<1, 64, 0, s>>>(b.err.p, 0u, 1);
  BatchArgs a{};
  a.inst = b.inst.p;
  a.row_inst = b.row_inst.p;
  a.inst_row0 = b.inst_row0.p;
  a.ub_off = b.ub_off.p;
  a.heavy = b.heavy.p;
  a.n_heavy = b.n_heavy;
  a.light = b.light.p;
  a.n_light = b.n_light;
  a.inner = b.inner.p;
  a.n_inner = b.n_inner;
  a.qhead = b.qhead.p;
  a.row_nnz = b.row_nnz.p;
  a.ub_k = b.ub_k.p;
  a.ub_cnt = b.ub_cnt.p;
  a.ub_sum = b.ub_sum.p;
  a.err = b.err.p;
  a.prod = b.prod.p;
  a.kw = b.kw;
  const unsigned grid = (unsigned)(cus * std::min(b.tune.blocks_per_cu, MAX_BLOCKS_PER_CU));
  if (b.n_inner) k_batch_inner<<<grid, B_NT, 0, s>>>(a);
  if (b.n_heavy) k_batch_heavy<<<grid, B_NT, 0, s>>>(a);
  if (b.tune.light_max <= 64) k_batch_light<128><<<grid, B_NT, 0, s>>>(a);
  else k_batch_light<256><<<grid, B_NT, 0, s>>>(a);
}

void build_graph(BatchState& b) {
  if (!b.cap) LH_HIP(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
  LH_HIP(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
  launch_compute(b, b.cap);
  hipError_t e = hipStreamEndCapture(b.cap, &b.graph);
  if (e != hipSuccess) hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
  LH_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
}

float time_replay(BatchState& b, hipStream_t s) {
  hipEvent_t e0, e1;
  LH_HIP(hipEventCreate(&e0));
  LH_HIP(hipEventCreate(&e1));
  LH_HIP(hipEventRecord(e0, s));
  LH_HIP(hipGraphLaunch(b.exec, s));
  LH_HIP(hipEventRecord(e1, s));
  LH_HIP(hipEventSynchronize(e1));
  float ms = 0;
  LH_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// The project's autotuner: time each candidate's graph, keep the fastest,
// remember it per device and batch signature.  The light/heavy split and
// the inner-product ratio change the setup (row classes and queues); the
// grid only changes the captured launch, so it is tried on each setup.
// Only the best setup so far is kept alive (each holds the output bounds).
void autotune(std::unique_ptr<BatchState>& cur, lh_plan_t* const* plans, uint32_t n, hipStream_t s) {
  const std::string sig = signature(*cur);
  Tuning t;
  if (load_tuning(sig, t)) {
    if (t.light_max != cur->tune.light_max || t.blocks_per_cu != cur->tune.blocks_per_cu ||
        t.inner_ratio != cur->tune.inner_ratio) {
      auto nb = std::make_unique<BatchState>();
      nb->plans = cur->plans;
      nb->tr = cur->tr;
      nb->tune = t;
      cur.reset();
      setup(*nb, s);
      build_graph(*nb);
      cur = std::move(nb);
    }
    return;
  }
  const uint32_t lights[] = {64, 128};
  const uint32_t ratios[] = {4, 16, 64};
  const uint32_t bpcs[] = {1, 2, 4};
  const std::vector<const lh_plan_t*> pv(plans, plans + n);
  std::shared_ptr<Transposes> tr = cur->tr;
  float best = 3.0e38f;
  std::unique_ptr<BatchState> winner;
  for (uint32_t lm : lights)
    for (uint32_t ir : ratios) {
      std::unique_ptr<BatchState> cand;
      if (cur && lm == cur->tune.light_max && ir == cur->tune.inner_ratio) {
        cand = std::move(cur);
      } else {
        cand = std::make_unique<BatchState>();
        cand->plans = pv;
        cand->tr = tr;
        cand->tune.light_max = lm;
        cand->tune.inner_ratio = ir;
        setup(*cand, s);
      }
      float cand_best = 3.0e38f;
      uint32_t cand_bp = cand->tune.blocks_per_cu;
      for (uint32_t bp : bpcs) {
        if (cand->exec) (void)hipGraphExecDestroy(cand->exec);
        if (cand->graph) (void)hipGraphDestroy(cand->graph);
        cand->exec = nullptr;
        cand->graph = nullptr;
        cand->tune.blocks_per_cu = bp;
        build_graph(*cand);
        const float ms = time_replay(*cand, s);
        if (ms < cand_best) {
          cand_best = ms;
          cand_bp = bp;
        }
      }
      if (cand->tune.blocks_per_cu != cand_bp) {
        (void)hipGraphExecDestroy(cand->exec);
        (void)hipGraphDestroy(cand->graph);
        cand->exec = nullptr;
        cand->graph = nullptr;
        cand->tune.blocks_per_cu = cand_bp;
        build_graph(*cand);
      }
      if (cand_best < best) {
        best = cand_best;
        winner = std::move(cand);
      }
    }
  save_tuning(sig, winner->tune);
  cur = std::move(winner);
}

struct SharedOut {
  DBuf<uint32_t> out_i, out_k;
  DBuf<uint64_t> out_cnt;
  DBuf<double> out_sum;
};

}  // namespace

int row_union_kind(const lh_plan_t* p) {
  if (p->atoms.size() != 2 || !p->groups.empty()) return -1;
  const PlanAtom& A = p->atoms[0];
  const PlanAtom& E = p->atoms[1];
  if (A.n_levels != 2) return -1;
  // attribute roles: i = A's first level, j = A's second level
  const uint32_t i = A.attr_of_level[0], j = A.attr_of_level[1];
  if (p->order[0] != i || p->order[1] != j) return -1;
  if (E.n_levels == 1) {
    if (p->n_attrs != 2 || E.attr_of_level[0] != j) return -1;
    if (p->out_attrs.size() != 1 || p->out_attrs[0] != i) return -1;
    return 0;
  }
  if (E.n_levels == 2) {
    if (p->n_attrs != 3 || E.attr_of_level[0] != j) return -1;
    const uint32_t k = E.attr_of_level[1];
    if (p->order[2] != k) return -1;
    if (p->out_attrs.size() != 2 || p->out_attrs[0] != i || p->out_attrs[1] != k) return -1;
    return 1;
  }
  return -1;
}

bool run_batch(lh_plan_t* const* plans, uint32_t n, hipStream_t s, std::vector<lh_result_impl*>& out) {
  for (uint32_t i = 0; i < n; i++)
    if (row_union_kind(plans[i]) < 0) return false;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  std::vector<const lh_plan_t*> pv(plans, plans + n);
  if (!g_batch || g_batch->plans != pv) {
    g_batch.reset();
    auto b = std::make_unique<BatchState>();
    b->plans = pv;
    setup(*b, s);
    build_graph(*b);
    autotune(b, plans, n, s);
    g_batch = std::move(b);
  }
  BatchState& b = *g_batch;
  {
    ProfScope ps("batch_graph", s, b.R, b.UB);
    LH_HIP(hipGraphLaunch(b.exec, s));
  }
  // pack: scan the per-row output counts, one shared output block
  DBuf<uint64_t> out_off(b.R + 1, s);
  const uint64_t total = scan_u32_to_u64(b.row_nnz.p, out_off.p, b.R, s);
  if (read_scalar(b.err.p, s)) fail(LH_ERR_UNSUPPORTED, "an annotation product did not fit the exact accumulator");
  auto sh = std::make_shared<SharedOut>();
  sh->out_i.alloc(total, s);
  sh->out_k.alloc(total, s);
  sh->out_cnt.alloc(total, s);
  sh->out_sum.alloc(total, s);
  PackArgs2 pa{};
  pa.inst = b.inst.p;
  pa.row_inst = b.row_inst.p;
  pa.inst_row0 = b.inst_row0.p;
  pa.ub_off = b.ub_off.p;
  pa.out_off = out_off.p;
  pa.ub_k = b.ub_k.p;
  pa.ub_cnt = b.ub_cnt.p;
  pa.ub_sum = b.ub_sum.p;
  pa.out_i = sh->out_i.p;
  pa.out_k = sh->out_k.p;
  pa.out_cnt = sh->out_cnt.p;
  pa.out_sum = sh->out_sum.p;
  pa.R = b.R;
  if (b.R) {
    ProfScope ps("batch_pack", s, b.R, total);
    k_pack_rows<<<grid_for(b.R), 256, 0, s>>>(pa);
    LH_HIP(hipGetLastError());
  }
  // each instance's rows are contiguous: its outputs are [offs[i], offs[i + 1])
  std::vector<uint64_t> offs(n + 1);
  {
    DBuf<uint64_t> d(n + 1, s);
    k_inst_offsets<<<(n + 256) / 256, 256, 0, s>>>(out_off.p, b.inst_row0.p, n, d.p);
    LH_HIP(hipGetLastError());
    LH_HIP(hipMemcpyAsync(offs.data(), d.p, (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
  }
  for (uint32_t i = 0; i < n; i++) {
    const BInst& I = b.h_inst[i];
    const uint64_t o0 = offs[i], o1 = offs[i + 1];
    auto* r = new lh_result_impl();
    memset(&r->pub, 0, sizeof(r->pub));
    r->shared = sh;
    r->colptr.push_back(sh->out_i.p ? sh->out_i.p + o0 : nullptr);
    if (I.kind == 1) r->colptr.push_back(sh->out_k.p ? sh->out_k.p + o0 : nullptr);
    r->pub.n_rows = o1 - o0;
    r->pub.n_cols = (uint32_t)r->colptr.size();
    r->pub.out_keys = r->colptr.data();
    r->pub.counts = sh->out_cnt.p ? sh->out_cnt.p + o0 : nullptr;
    r->pub.sums = I.sum ? (sh->out_sum.p ? sh->out_sum.p + o0 : nullptr) : nullptr;
    r->pub.exact = I.sum;
    r->pub.n_join_tuples = b.h_nj[i];
    out.push_back(r);
  }
  return true;
}

void batch_forget_plan(const lh_plan_t* p) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (g_batch && std::find(g_batch->plans.begin(), g_batch->plans.end(), p) != g_batch->plans.end()) g_batch.reset();
}

}  // namespace lh
