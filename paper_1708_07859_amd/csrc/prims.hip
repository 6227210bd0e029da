// Device-wide primitives: scans, reductions, fills, gathers, LSD radix sort.
#include <algorithm>
#include <climits>
#include <cstring>

#include "device_common.h"
#include "lh_internal.h"

namespace lh {

namespace {

constexpr int SC_NT = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_NT * SC_ITEMS;

inline unsigned blocks_for(uint64_t n, uint64_t per) { return (unsigned)((n + per - 1) / per); }

// Per-tile sums of the input.
template <class TI, class TO>
__global__ __launch_bounds__(SC_NT) void k_tile_sums(const TI* in, uint64_t n, TO* sums) {
  __shared__ TO lds[SC_NT / WAVE];
  uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
  TO s = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; i++) {
    uint64_t idx = base + (uint64_t)i * SC_NT + threadIdx.x;
    if (idx < n) s += (TO)in[idx];
  }
  TO tot = block_sum<TO, SC_NT>(s, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of each tile plus its tile offset; thread t owns
// SC_ITEMS consecutive elements.
template <class TI, class TO>
__global__ __launch_bounds__(SC_NT) void k_tile_scan(const TI* in, uint64_t n, const TO* tile_off, TO* out) {
  __shared__ TO lds[SC_NT / WAVE];
  __shared__ TI stage[SC_TILE];
  uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
  // coalesced load into LDS
#pragma unroll
  for (int i = 0; i < SC_ITEMS; i++) {
    uint64_t idx = base + (uint64_t)i * SC_NT + threadIdx.x;
    stage[i * SC_NT + threadIdx.x] = idx < n ? in[idx] : (TI)0;
  }
  __syncthreads();
  TO v[SC_ITEMS];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; i++) {
    v[i] = (TO)stage[threadIdx.x * SC_ITEMS + i];
    s += v[i];
  }
  TO tot;
  TO run = block_excl_scan<TO, SC_NT>(s, lds, tot) + tile_off[blockIdx.x];
  __syncthreads();
  // write back through LDS as TO (reuse needs a separate buffer for 64-bit)
  __shared__ TO ostage[SC_TILE];
#pragma unroll
  for (int i = 0; i < SC_ITEMS; i++) {
    ostage[threadIdx.x * SC_ITEMS + i] = run;
    run += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SC_ITEMS; i++) {
    uint64_t idx = base + (uint64_t)i * SC_NT + threadIdx.x;
    if (idx < n) out[idx] = ostage[i * SC_NT + threadIdx.x];
  }
}

template <class TO>
__global__ void k_set_total(TO* out, uint64_t n, const TO* tile_off, const TO* tile_sums, uint64_t ntiles) {
  out[n] = tile_off[ntiles - 1] + tile_sums[ntiles - 1];
}

// Exclusive scan of in[0, n) into out[0, n) and the total into out[n], all
// on the device (the tile sums' own scan included): no host round trip.
template <class TI, class TO>
void scan_dev(const TI* in, TO* out, uint64_t n, hipStream_t s) {
  if (n == 0) {
    LH_HIP(hipMemsetAsync(out, 0, sizeof(TO), s));
    return;
  }
  uint64_t ntiles = (n + SC_TILE - 1) / SC_TILE;
  DBuf<TO> sums(ntiles, s), offs(ntiles + 1, s);
  k_tile_sums<TI, TO><<<(unsigned)ntiles, SC_NT, 0, s>>>(in, n, sums.p);
  LH_HIP(hipGetLastError());
  if (ntiles == 1) {
    LH_HIP(hipMemsetAsync(offs.p, 0, sizeof(TO), s));
  } else {
    scan_dev<TO, TO>(sums.p, offs.p, ntiles, s);
  }
  k_tile_scan<TI, TO><<<(unsigned)ntiles, SC_NT, 0, s>>>(in, n, offs.p, out);
  LH_HIP(hipGetLastError());
  k_set_total<TO><<<1, 1, 0, s>>>(out, n, offs.p, sums.p, ntiles);
  LH_HIP(hipGetLastError());
}

// The same, and the total read back to the host.
template <class TI, class TO>
TO scan_impl(const TI* in, TO* out, uint64_t n, hipStream_t s) {
  scan_dev<TI, TO>(in, out, n, s);
  return read_scalar(out + n, s);
}

// Largest of in[0, n).  The body is read as 16-byte vectors, four rounds
// in flight per thread; the elements before the first 16-byte boundary and
// after the last whole vector are read singly.
__global__ __launch_bounds__(256) void k_reduce_max_u32(const uint32_t* in, uint64_t n, uint32_t* out) {
  __shared__ uint32_t s_m[256 / WAVE];
  const uint64_t head = min<uint64_t>(n, (4u - (((uintptr_t)in >> 2) & 3u)) & 3u);
  const uint4* body = reinterpret_cast<const uint4*>(in + head);
  const uint64_t nv = (n - head) / 4, tail = head + nv * 4;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t m = 0;
  if (gid < head) m = in[gid];
  if (gid < n - tail) m = max(m, in[tail + gid]);
  uint64_t i = gid;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    const uint4 a = body[i], b = body[i + stride], c = body[i + 2 * stride], d = body[i + 3 * stride];
    m = max(m, max(max(max(a.x, a.y), max(a.z, a.w)), max(max(b.x, b.y), max(b.z, b.w))));
    m = max(m, max(max(max(c.x, c.y), max(c.z, c.w)), max(max(d.x, d.y), max(d.z, d.w))));
  }
  for (; i < nv; i += stride) {
    const uint4 a = body[i];
    m = max(m, max(max(a.x, a.y), max(a.z, a.w)));
  }
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, WAVE));
  if (lane_id() == 0) s_m[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int w = 0; w < 256 / WAVE; w++) b = max(b, s_m[w]);
    atomicMax(out, b);
  }
}

__global__ void k_iota(uint32_t* out, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)i;
}

template <class T>
__global__ void k_fill(T* out, T v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = v;
}

template <class T>
__global__ void k_gather(const T* src, const uint32_t* idx, T* dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}

__global__ void k_scatter_flagged(const uint32_t* flags, const uint64_t* off, uint64_t n, uint32_t* out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    if (flags[i]) out[off[i]] = (uint32_t)i;
}

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 256 * 64));
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  Per pass: tile histograms (digit-major, so
// an exclusive scan yields every tile's first slot per digit), then a
// stable scatter that ranks equal digits inside a wave with eight ballots
// and across the block's waves through LDS.  A sort of key columns reads
// the columns in its first pass (packing each row's key on the fly) and
// writes the sorted columns in its last (unpacking them), so no pass of
// its own packs or unpacks.
// ---------------------------------------------------------------------------
constexpr int RS_NT = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_NT * RS_ITEMS;
constexpr int RS_NW = RS_NT / WAVE;

// Key columns packed into one word: column c at bit shift[c].
struct PackArgs {
  const uint32_t* col[LH_MAX_KEYS];
  uint32_t shift[LH_MAX_KEYS];
  uint32_t ncols;
};

// One word unpacked into key columns: bits[c] bits at shift[c].
struct UnpackCols {
  uint32_t* col[LH_MAX_KEYS];
  uint32_t shift[LH_MAX_KEYS];
  uint32_t bits[LH_MAX_KEYS];
  uint32_t ncols;
};

__device__ __forceinline__ uint64_t pack_row(const PackArgs& a, uint64_t r) {
  uint64_t k = 0;
#pragma unroll
  for (uint32_t c = 0; c < LH_MAX_KEYS; c++)
    if (c < a.ncols) k |= (uint64_t)a.col[c][r] << a.shift[c];
  return k;
}

__device__ __forceinline__ void unpack_row(const UnpackCols& a, uint64_t r, uint64_t k) {
#pragma unroll
  for (uint32_t c = 0; c < LH_MAX_KEYS; c++)
    if (c < a.ncols) a.col[c][r] = a.bits[c] ? (uint32_t)((k >> a.shift[c]) & ((1ull << a.bits[c]) - 1)) : 0u;
}

// FROM_COLS: the keys are packed from the columns of `pa` (else read from
// `keys`).
template <bool FROM_COLS>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t* keys, PackArgs pa, uint64_t n, uint32_t shift,
                                                   uint32_t* hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  if (!FROM_COLS && !((uintptr_t)keys & 15u)) {
    // packed keys, two per 16-byte load (the order of a histogram's keys
    // does not matter)
    const uint64_t ntile = min<uint64_t>(RS_TILE, n - base);
    const ulonglong2* k2 = reinterpret_cast<const ulonglong2*>(keys + base);
#pragma unroll
    for (int i = 0; i < RS_ITEMS / 2; i++) {
      const uint64_t j = (uint64_t)i * RS_NT + threadIdx.x;  // pair index in the tile
      if (2 * j + 1 < ntile) {
        const ulonglong2 v = k2[j];
        atomicAdd(&h[(uint32_t)(v.x >> shift) & 255u], 1u);
        atomicAdd(&h[(uint32_t)(v.y >> shift) & 255u], 1u);
      } else if (2 * j < ntile) {
        atomicAdd(&h[(uint32_t)(keys[base + 2 * j] >> shift) & 255u], 1u);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
      uint64_t idx = base + (uint64_t)i * RS_NT + threadIdx.x;
      if (idx < n) {
        const uint64_t k = FROM_COLS ? pack_row(pa, idx) : keys[idx];
        atomicAdd(&h[(uint32_t)(k >> shift) & 255u], 1u);
      }
    }
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile.  Wave w holds the tile's elements
// [w * RS_ITEMS * 64, (w + 1) * RS_ITEMS * 64), item i of lane l at offset
// i * 64 + l, so a wave's items in order are the input order.  A wave ranks
// its items one after another against digit counters of its own (eight
// ballots find a lane's equal-digit peers; no barrier between items, the
// wave's LDS operations run in order), then one prefix over the waves per
// digit places every element in LDS in digit order, and the tile is written
// out in that order, so each digit's run of the tile goes to consecutive
// global slots (coalesced writes).
// HAS_V: a 32-bit value travels with each key (else keys only); a null
// `vin` gives every element its input position as value.
// FROM_COLS: keys packed from the columns of `pa` (else read from `kin`).
// TO_COLS: sorted keys unpacked into the columns of `ua` (else to `kout`).
template <bool HAS_V, bool FROM_COLS, bool TO_COLS>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t* kin, PackArgs pa, const uint32_t* vin,
                                                      uint64_t* kout, UnpackCols ua, uint32_t* vout, uint64_t n,
                                                      uint32_t shift, const uint32_t* offs, const uint32_t* hist,
                                                      uint32_t ntiles) {
  __shared__ uint64_t sk[RS_TILE];
  __shared__ uint32_t sv[HAS_V ? RS_TILE : 1];
  __shared__ uint32_t lstart[256];       // first slot of each digit in the tile
  __shared__ uint32_t wcnt[RS_NW][256];  // each wave's digit counts, then its first slot per digit
  __shared__ uint32_t s_red[RS_NW];
  const int tid = threadIdx.x, w = tid / WAVE, lane = tid & (WAVE - 1);
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  const uint32_t ntile = (uint32_t)min<uint64_t>(RS_TILE, n - base);
  const uint32_t wbase = (uint32_t)w * RS_ITEMS * WAVE;
  // all of the wave's loads are issued first
  uint64_t kk[RS_ITEMS];
  uint32_t vv[RS_ITEMS];
#pragma unroll
  for (int i = 0; i < RS_ITEMS; i++) {
    const uint32_t li = wbase + (uint32_t)i * WAVE + lane;
    if constexpr (FROM_COLS) kk[i] = li < ntile ? pack_row(pa, base + li) : 0;
    else kk[i] = li < ntile ? kin[base + li] : 0;
    vv[i] = 0;
    if constexpr (HAS_V) vv[i] = li < ntile ? (vin ? vin[base + li] : (uint32_t)(base + li)) : 0u;
  }
  {
    const uint32_t c = hist[(uint64_t)tid * ntiles + blockIdx.x];
    uint32_t tot;
    lstart[tid] = block_excl_scan<uint32_t, RS_NT>(c, s_red, tot);
  }
#pragma unroll
  for (int j = 0; j < RS_NW; j++) wcnt[j][tid] = 0;
  __syncthreads();
  uint32_t rank[RS_ITEMS];
#pragma unroll
  for (int i = 0; i < RS_ITEMS; i++) {
    const bool valid = wbase + (uint32_t)i * WAVE + lane < ntile;
    const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = lanes_below(peers);
    const uint32_t pre = valid ? wcnt[w][d] : 0u;
    rank[i] = pre + below;
    // the lowest peer moves the wave's count on, after every peer has read it
    if (valid && below == 0) wcnt[w][d] = pre + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    // digit tid: the first slot of each wave's run of it
    uint32_t slot = lstart[tid];
#pragma unroll
    for (int j = 0; j < RS_NW; j++) {
      const uint32_t c = wcnt[j][tid];
      wcnt[j][tid] = slot;
      slot += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; i++) {
    if (wbase + (uint32_t)i * WAVE + lane < ntile) {
      const uint32_t lp = wcnt[w][(uint32_t)(kk[i] >> shift) & 255u] + rank[i];
      sk[lp] = kk[i];
      if constexpr (HAS_V) sv[lp] = vv[i];
    }
  }
  __syncthreads();
  for (uint32_t t = tid; t < ntile; t += RS_NT) {
    const uint64_t k = sk[t];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t pos = offs[(uint64_t)d * ntiles + blockIdx.x] + (t - lstart[d]);
    if constexpr (TO_COLS) unpack_row(ua, pos, k);
    else kout[pos] = k;
    if constexpr (HAS_V) vout[pos] = sv[t];
  }
}

template <bool HAS_V>
void launch_rs_scatter(bool from_cols, bool to_cols, unsigned grid, hipStream_t s, const uint64_t* kin,
                       const PackArgs& pa, const uint32_t* vin, uint64_t* kout, const UnpackCols& ua, uint32_t* vout,
                       uint64_t n, uint32_t shift, const uint32_t* offs, const uint32_t* hist, uint32_t ntiles) {
  if (from_cols && to_cols)
    k_rs_scatter<HAS_V, true, true><<<grid, RS_NT, 0, s>>>(kin, pa, vin, kout, ua, vout, n, shift, offs, hist, ntiles);
  else if (from_cols)
    k_rs_scatter<HAS_V, true, false><<<grid, RS_NT, 0, s>>>(kin, pa, vin, kout, ua, vout, n, shift, offs, hist, ntiles);
  else if (to_cols)
    k_rs_scatter<HAS_V, false, true><<<grid, RS_NT, 0, s>>>(kin, pa, vin, kout, ua, vout, n, shift, offs, hist, ntiles);
  else
    k_rs_scatter<HAS_V, false, false><<<grid, RS_NT, 0, s>>>(kin, pa, vin, kout, ua, vout, n, shift, offs, hist,
                                                             ntiles);
  LH_HIP(hipGetLastError());
}

__global__ void k_pack(PackArgs a, const uint32_t* perm, uint64_t* out, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = pack_row(a, perm ? perm[i] : (uint32_t)i);
}

__device__ __forceinline__ int32_t lowest_bit_exp(double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  uint32_t ex = (uint32_t)(b >> 52) & 0x7ffu;
  uint64_t mant = b & ((1ull << 52) - 1);
  if (ex == 0) return -1074 + (int32_t)__builtin_ctzll(mant);
  mant |= 1ull << 52;
  return (int32_t)ex - 1075 + (int32_t)__builtin_ctzll(mant);
}

__global__ void k_anno_stats(const double* v, uint64_t n, int32_t* qmin, unsigned long long* maxabs, uint32_t* nonfinite) {
  int32_t q = INT_MAX;
  uint64_t m = 0;
  uint32_t bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    double x = v[i];
    if (!isfinite(x)) { bad = 1; continue; }
    if (x == 0.0) continue;
    q = min(q, lowest_bit_exp(x));
    uint64_t ab = (uint64_t)__double_as_longlong(fabs(x));
    m = max(m, ab);
  }
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    q = min(q, __shfl_xor(q, d, WAVE));
    m = max(m, (uint64_t)__shfl_xor((unsigned long long)m, d, WAVE));
    bad |= (uint32_t)__shfl_xor((int)bad, d, WAVE);
  }
  // one update per workgroup, and only when it changes the result (the
  // same three words are the target of every workgroup)
  __shared__ int32_t s_q[8];
  __shared__ unsigned long long s_m[8];
  __shared__ uint32_t s_b[8];
  const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  if (lane_id() == 0) {
    s_q[w] = q;
    s_m[w] = m;
    s_b[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < nw; j++) {
      q = min(q, s_q[j]);
      m = max(m, (uint64_t)s_m[j]);
      bad |= s_b[j];
    }
    if (q < __hip_atomic_load(qmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(qmin, q);
    if (m > __hip_atomic_load(maxabs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(maxabs, (unsigned long long)m);
    if (bad && !__hip_atomic_load(nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicOr(nonfinite, 1u);
  }
}

}  // namespace

uint64_t scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  return scan_impl<uint32_t, uint64_t>(in, out, n, s);
}
uint64_t scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  return scan_impl<uint64_t, uint64_t>(in, out, n, s);
}
uint32_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s) {
  return scan_impl<uint32_t, uint32_t>(in, out, n, s);
}
void scan_u32_dev(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s) {
  scan_dev<uint32_t, uint32_t>(in, out, n, s);
}

void max_u32_into(const uint32_t* in, uint64_t n, uint32_t* out, hipStream_t s) {
  if (!n) return;
  k_reduce_max_u32<<<std::min(grid_for((n + 3) / 4), 2048u), 256, 0, s>>>(in, n, out);
  LH_HIP(hipGetLastError());
}

uint32_t reduce_max_u32(const uint32_t* in, uint64_t n, hipStream_t s) {
  DBuf<uint32_t> r(1, s);
  LH_HIP(hipMemsetAsync(r.p, 0, sizeof(uint32_t), s));
  max_u32_into(in, n, r.p, s);
  return read_scalar(r.p, s);
}

uint64_t select_flagged(const uint32_t* flags, uint64_t n, uint32_t* out, hipStream_t s) {
  DBuf<uint64_t> off(n + 1, s);
  uint64_t m = scan_u32_to_u64(flags, off.p, n, s);
  if (m) {
    k_scatter_flagged<<<grid_for(n), 256, 0, s>>>(flags, off.p, n, out);
    LH_HIP(hipGetLastError());
  }
  return m;
}

// Runs of a sorted column: their number and the longest.  A wave takes
// RS_GROUPS groups of 64 consecutive values, all loads issued together; a
// ballot of each group's run heads gives every run that ends inside the
// group its length, and a run still going at a group's end is carried into
// the next group.  One still going at the wave's last value is followed
// into the next 64 values with one more load and a ballot; only a run
// longer than that gallops to its end (probes 1, 2, 4, ... past them, then
// bisects the last step).  Each block writes its count and longest run
// (atomics of every block on one address would serialize).
constexpr int RS_GROUPS = 8;

struct RunStats {
  unsigned long long distinct;
  unsigned int longest;
  unsigned int pad;
};

__global__ __launch_bounds__(256) void k_run_stats(const uint32_t* v, uint64_t n, RunStats* part) {
  __shared__ uint32_t s_red[256 / WAVE];
  const int lane = lane_id();
  uint32_t heads = 0, longest = 0;
  constexpr uint64_t span = (uint64_t)RS_GROUPS * WAVE;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / WAVE;
  for (uint64_t c0 = wave * span; c0 < n; c0 += nwaves * span) {
    uint32_t xs[RS_GROUPS];
#pragma unroll
    for (int g = 0; g < RS_GROUPS; g++) {
      const uint64_t i = c0 + (uint64_t)g * WAVE + lane;
      xs[g] = i < n ? v[i] : 0u;
    }
    const uint32_t before = c0 > 0 ? v[c0 - 1] : 0u;
    bool open = false;      // a run started at os (value xo) is still going (uniform over the wave)
    uint64_t os = 0;
    uint32_t xo = 0;
#pragma unroll
    for (int g = 0; g < RS_GROUPS; g++) {
      const uint64_t g0 = c0 + (uint64_t)g * WAVE, i = g0 + lane;
      const uint32_t x = xs[g];
      const uint32_t last_before = g ? (uint32_t)__shfl((int)xs[g > 0 ? g - 1 : 0], WAVE - 1, WAVE) : before;
      uint32_t p = (uint32_t)__shfl_up((int)x, 1, WAVE);
      if (lane == 0) p = last_before;
      const bool head = i < n && (i == 0 || p != x);
      const uint64_t Hh = ballot(head);
      // lanes past the end count as heads: a run ends at the next set bit
      const uint64_t H = Hh | ballot(i >= n);
      if (open && H) {
        if (lane == 0) longest = max(longest, (uint32_t)(g0 + (uint64_t)__builtin_ctzll(H) - os));
        open = false;
      }
      if (head) heads++;
      const uint64_t above = lane < WAVE - 1 ? H >> (lane + 1) : 0ull;
      if (head && above) longest = max(longest, (uint32_t)__builtin_ctzll(above) + 1u);
      // the last head's run reaches the group's last lane (every lane in range)
      if (Hh && !((H >> (63 - __builtin_clzll(Hh))) >> 1)) {
        open = true;
        os = g0 + (uint64_t)(63 - __builtin_clzll(Hh));
        xo = (uint32_t)__shfl((int)x, WAVE - 1, WAVE);
      }
    }
    if (open) {  // it reaches c0 + span - 1 < n
      const uint64_t e0 = c0 + span, k = e0 + lane;
      const uint64_t D = ballot(k >= n || v[k] != xo);
      uint64_t end = e0 + (D ? (uint64_t)__builtin_ctzll(D) : 0u);
      if (!D && lane == 0) {
        uint64_t lo = e0 + WAVE - 1, step = 1;  // v[lo] == xo
        while (lo + step < n && v[lo + step] == xo) {
          lo += step;
          step <<= 1;
        }
        uint64_t hi = min<uint64_t>(lo + step, n);  // v[hi] != xo, or hi == n
        while (hi - lo > 1) {
          const uint64_t mid = lo + (hi - lo) / 2;
          if (v[mid] == xo) lo = mid;
          else hi = mid;
        }
        end = hi;
      }
      if (lane == 0) longest = max(longest, (uint32_t)(end - os));
    }
  }
  const uint32_t h = block_sum<uint32_t, 256>(heads, s_red);  // ends with a barrier: s_red is free
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) longest = max(longest, (uint32_t)__shfl_xor((int)longest, d, WAVE));
  if (lane == 0) s_red[threadIdx.x / WAVE] = longest;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int w = 0; w < 256 / WAVE; w++) m = max(m, s_red[w]);
    part[blockIdx.x] = RunStats{h, m, 0u};
  }
}

// The blocks' partial run statistics summed and maximized by one block.
__global__ __launch_bounds__(256) void k_run_stats_total(const RunStats* part, uint32_t nb, RunStats* out) {
  __shared__ unsigned long long s_d[256 / WAVE];
  __shared__ uint32_t s_m[256 / WAVE];
  unsigned long long d = 0;
  uint32_t m = 0;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    d += part[b].distinct;
    m = max(m, part[b].longest);
  }
  d = wave_sum(d);
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, WAVE));
  if (lane_id() == 0) {
    s_d[threadIdx.x / WAVE] = d;
    s_m[threadIdx.x / WAVE] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    RunStats r{0ull, 0u, 0u};
    for (int w = 0; w < 256 / WAVE; w++) {
      r.distinct += s_d[w];
      r.longest = max(r.longest, s_m[w]);
    }
    *out = r;
  }
}

void column_freq(const uint32_t* col, uint64_t n, uint32_t range, uint64_t& distinct, uint64_t& freq_max,
                 hipStream_t s) {
  // sort the values (no atomics: hub values would serialize them), then
  // the distinct values are the runs and the largest frequency the longest
  // run
  distinct = 0;
  freq_max = 0;
  if (!n) return;
  const uint32_t bits = range ? 32 - __builtin_clz(range) : 0;
  DBuf<uint32_t> sorted(n, s);
  uint32_t* out = sorted.p;
  if (!sort_packed(&col, &bits, 1, n, nullptr, &out, s)) fail(LH_ERR_DEVICE, "column statistics: sort failed");
  sorted_run_stats(sorted.p, n, distinct, freq_max, s);
}

void sorted_run_stats(const uint32_t* sorted, uint64_t n, uint64_t& distinct, uint64_t& freq_max, hipStream_t s) {
  distinct = 0;
  freq_max = 0;
  if (!n) return;
  const unsigned nb = grid_for((n + RS_GROUPS - 1) / RS_GROUPS);
  DBuf<RunStats> part(nb, s), r(1, s);
  k_run_stats<<<nb, 256, 0, s>>>(sorted, n, part.p);
  LH_HIP(hipGetLastError());
  k_run_stats_total<<<1, 256, 0, s>>>(part.p, nb, r.p);
  LH_HIP(hipGetLastError());
  const RunStats h = read_scalar(r.p, s);
  distinct = h.distinct;
  freq_max = h.longest;
}

void iota_u32(uint32_t* out, uint64_t n, hipStream_t s) {
  if (!n) return;
  k_iota<<<grid_for(n), 256, 0, s>>>(out, n);
  LH_HIP(hipGetLastError());
}
void fill_u32(uint32_t* out, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  k_fill<uint32_t><<<grid_for(n), 256, 0, s>>>(out, v, n);
  LH_HIP(hipGetLastError());
}
void fill_u64(uint64_t* out, uint64_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  k_fill<uint64_t><<<grid_for(n), 256, 0, s>>>(out, v, n);
  LH_HIP(hipGetLastError());
}
void gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, uint64_t n, hipStream_t s) {
  if (!n) return;
  k_gather<uint32_t><<<grid_for(n), 256, 0, s>>>(src, idx, dst, n);
  LH_HIP(hipGetLastError());
}
void gather_f64(const double* src, const uint32_t* idx, double* dst, uint64_t n, hipStream_t s) {
  if (!n) return;
  k_gather<double><<<grid_for(n), 256, 0, s>>>(src, idx, dst, n);
  LH_HIP(hipGetLastError());
}

namespace {

// The passes of one radix sort over bits [lo_bit, lo_bit + 8 * passes) of
// the keys.  The first pass reads `pa`'s columns when from_cols (else
// kin) and, when vals are wanted, `vin` (null: input positions).  Pass p
// writes kbuf[(p + phase) & 1] and vbuf[(p + phase) & 1], except that
// the last writes `ua`'s columns instead of keys when to_cols.
void radix_passes(const uint64_t* kin, const PackArgs& pa, bool from_cols, const uint32_t* vin, bool vals,
                  uint64_t* const kbuf[2], const UnpackCols& ua, bool to_cols, uint32_t* const vbuf[2],
                  uint32_t phase, uint64_t n, uint32_t lo_bit, uint32_t passes, hipStream_t s) {
  const uint32_t ntiles = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
  const uint64_t hn = (uint64_t)ntiles * 256;
  DBuf<uint32_t> hist(hn, s), offs(hn + 1, s);
  const uint64_t in_bytes = from_cols ? 4ull * pa.ncols : 8ull, out_bytes = to_cols ? 4ull * ua.ncols : 8ull;
  const uint64_t* ki = kin;
  const uint32_t* vi = vin;
  for (uint32_t p = 0; p < passes; p++) {
    const uint32_t shift = lo_bit + p * 8;
    const bool first = p == 0, last = p + 1 == passes;
    const bool fc = first && from_cols, tc = last && to_cols;
    {
      // elements: the pass's algorithmic bytes (its keys read)
      ProfScope ps("sort_hist", s, n, (fc ? in_bytes : 8) * n);
      if (fc) k_rs_hist<true><<<ntiles, RS_NT, 0, s>>>(nullptr, pa, n, shift, hist.p, ntiles);
      else k_rs_hist<false><<<ntiles, RS_NT, 0, s>>>(ki, pa, n, shift, hist.p, ntiles);
    }
    LH_HIP(hipGetLastError());
    scan_u32_dev(hist.p, offs.p, hn, s);
    uint64_t* ko = tc ? nullptr : kbuf[(p + phase) & 1];
    uint32_t* vo = vals ? vbuf[(p + phase) & 1] : nullptr;
    {
      // elements: the pass's algorithmic bytes (keys, and values when they
      // travel, read once and written once; values made from positions
      // are written only)
      const uint64_t vb = vals ? (vi ? 8 : 4) : 0;
      ProfScope ps("sort_scatter", s, n, ((fc ? in_bytes : 8) + (tc ? out_bytes : 8) + vb) * n);
      if (vals) launch_rs_scatter<true>(fc, tc, ntiles, s, ki, pa, vi, ko, ua, vo, n, shift, offs.p, hist.p, ntiles);
      else launch_rs_scatter<false>(fc, tc, ntiles, s, ki, pa, nullptr, ko, ua, nullptr, n, shift, offs.p, hist.p,
                                    ntiles);
    }
    ki = ko;
    vi = vo;
  }
}

}  // namespace

void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tkeys, uint32_t* tvals, uint64_t n,
                      uint32_t bits, hipStream_t s, uint32_t lo_bit) {
  // vals == nullptr: keys only
  if (n <= 1 || bits <= lo_bit) return;
  if (n >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "radix sort: more than 2^32 - 1 keys");
  const uint32_t passes = (bits - lo_bit + 7) / 8;
  // pass p writes buffer (p + 1) & 1: the first writes the temporaries,
  // the last the caller's buffers when the count is even
  uint64_t* const kbuf[2] = {keys, tkeys};
  uint32_t* const vbuf[2] = {vals, tvals};
  radix_passes(keys, PackArgs{}, false, vals, vals != nullptr, kbuf, UnpackCols{}, false, vbuf, 1, n, lo_bit, passes,
               s);
  if (passes & 1) {
    LH_HIP(hipMemcpyAsync(keys, tkeys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    if (vals) LH_HIP(hipMemcpyAsync(vals, tvals, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
}

void lex_sort_perm(const uint32_t* const* cols, const uint32_t* bits, uint32_t ncols, uint64_t n, uint32_t* perm,
                   hipStream_t s) {
  iota_u32(perm, n, s);
  if (n <= 1) return;
  DBuf<uint64_t> k(n, s), tk(n, s);
  DBuf<uint32_t> tv(n, s);
  int end = (int)ncols;
  while (end > 0) {
    int start = end - 1;
    uint32_t tot = bits[start];
    while (start > 0 && tot + bits[start - 1] <= 64) {
      start--;
      tot += bits[start];
    }
    if (tot > 0) {
      PackArgs a{};
      a.ncols = (uint32_t)(end - start);
      uint32_t sh = 0;
      for (int c = end - 1; c >= start; c--) {  // least significant column at the bottom
        a.col[c - start] = cols[c];
        a.shift[c - start] = sh;
        sh += bits[c];
      }
      k_pack<<<grid_for(n), 256, 0, s>>>(a, perm, k.p, n);
      LH_HIP(hipGetLastError());
      radix_sort_pairs(k.p, perm, tk.p, tv.p, n, tot, s);
    }
    end = start;
  }
}

bool sort_packed(const uint32_t* const* cols, const uint32_t* bits, uint32_t ncols, uint64_t n, uint32_t* perm,
                 uint32_t* const* sorted, hipStream_t s, uint32_t sorted_tail) {
  uint32_t tot = 0;
  for (uint32_t c = 0; c < ncols; c++) tot += bits[c];
  if (tot > 64 || ncols > LH_MAX_KEYS) return false;
  if (!n) return true;
  if (n >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "radix sort: more than 2^32 - 1 keys");
  PackArgs a{};
  UnpackCols u{};
  a.ncols = u.ncols = ncols;
  uint32_t sh = 0;
  for (int c = (int)ncols - 1; c >= 0; c--) {  // the last column lowest
    a.col[c] = cols[c];
    a.shift[c] = u.shift[c] = sh;
    u.bits[c] = bits[c];
    u.col[c] = sorted[c];
    sh += bits[c];
  }
  uint32_t tail_bits = 0;
  for (uint32_t c = ncols - std::min(sorted_tail, ncols); c < ncols; c++) tail_bits += bits[c];
  const uint32_t passes = tot > tail_bits ? (tot - tail_bits + 7) / 8 : 0;
  if (!passes) {
    // in order already: every value fits its column's bits, so the sorted
    // columns are copies
    for (uint32_t c = 0; c < ncols; c++)
      LH_HIP(hipMemcpyAsync(sorted[c], cols[c], n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (perm) iota_u32(perm, n, s);
    return true;
  }
  // the first pass packs the columns, the last unpacks into `sorted`; the
  // permutation starts as the input positions and ends in perm
  DBuf<uint64_t> k(passes > 1 ? n : 0, s), tk(passes > 2 ? n : 0, s);
  DBuf<uint32_t> tv(perm && passes > 1 ? n : 0, s);
  uint64_t* const kbuf[2] = {k.p, tk.p};
  uint32_t* const vbuf[2] = {perm, tv.p};
  // pass p writes buffer (p + phase) & 1: the last writes vbuf[0] = perm,
  // the first writes kbuf[0] = k
  const uint32_t phase = (passes - 1) & 1;
  uint64_t* const kb[2] = {kbuf[phase], kbuf[phase ^ 1]};
  radix_passes(nullptr, a, true, nullptr, perm != nullptr, kb, u, true, vbuf, phase, n, tail_bits, passes, s);
  return true;
}

AnnoStats anno_stats(const double* v, uint64_t n, hipStream_t s) {
  DBuf<int32_t> q(1, s);
  DBuf<unsigned long long> m(1, s);
  DBuf<uint32_t> bad(1, s);
  k_fill<int32_t><<<1, 64, 0, s>>>(q.p, INT_MAX, 1);
  LH_HIP(hipGetLastError());
  LH_HIP(hipMemsetAsync(m.p, 0, sizeof(unsigned long long), s));
  LH_HIP(hipMemsetAsync(bad.p, 0, sizeof(uint32_t), s));
  if (n) {
    k_anno_stats<<<grid_for(n), 256, 0, s>>>(v, n, q.p, m.p, bad.p);
    LH_HIP(hipGetLastError());
  }
  AnnoStats st;
  st.qmin = read_scalar(q.p, s);
  unsigned long long mb = read_scalar(m.p, s);
  double md;
  memcpy(&md, &mb, sizeof md);
  st.maxabs = md;
  st.nonfinite = read_scalar(bad.p, s);
  return st;
}

}  // namespace lh
