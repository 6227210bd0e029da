// Generic worst-case optimal join with fused aggregation (Algorithm 1,
// section 2.4), executed level-synchronously on the GPU.
//
// The recursion of Algorithm 1 is unrolled breadth-first: the frontier at
// depth d holds one row per binding of the first d+1 attributes of the
// order, each row recording, for every relation that has a bound
// attribute, its node position in that relation's trie.  Binding attribute
// v_d intersects, for each frontier row, the sets of every relation that
// contains v_d (its children under the row's node, or its root set).  The
// work of a depth is flattened over the elements of each row's smallest
// set, so rows of any size are spread evenly over the GPU: a count pass,
// a scan and a fill pass that compacts hits with wave ballots.  The last
// attribute is never materialized: each hit is aggregated directly
// (annotations multiplied, the commutative-semiring sum of section 2.3).
#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "engine.h"
#include "exact.h"
#include "search.h"

namespace lh {

namespace {

constexpr int J_NT = 256;          // 4 waves per block, one work unit per wave
constexpr int J_NW = J_NT / WAVE;
constexpr int U_IT = 4;            // elements per lane per unit
constexpr int U_EL = WAVE * U_IT;  // driver elements per unit
// Two-set leaves: rows whose two sets hold TOP_MIN elements or more
// together form the top bucket, the largest intersections.  They run as a
// launch of their own.  Units of TOP_IT elements per lane (twice the loads
// in flight per wave) are used where a unit's probes stay cheap: word-AND
// rows, rows probing a bitset, and rows whose probed set is at most
// TOP_BALANCE times the driver (its range for a unit still fits the LDS
// stage).  Other top rows keep units of U_IT: a larger unit's probed range
// would overflow the stage and fall to the line-sample search (units of 512
// there measured 3 ms slower per plain-order triangle step).
constexpr uint32_t TOP_MIN = 1u << 14;
constexpr int TOP_IT = 2 * U_IT;
constexpr int TOP_EL = WAVE * TOP_IT;
constexpr uint32_t TOP_BALANCE = 2;

// Driver elements (or words) per unit of a two-set leaf row whose sets hold
// c0 and c1 elements; wide: a word-AND row, or one probing a bitset.
__device__ __forceinline__ uint32_t leaf2_chunk(uint32_t c0, uint32_t c1, bool wide) {
  const bool top = (uint64_t)c0 + c1 >= TOP_MIN;
  const bool big = wide || (uint64_t)TOP_BALANCE * min(c0, c1) >= max(c0, c1);
  return top && big ? (uint32_t)TOP_EL : (uint32_t)U_EL;
}
// Rows of two sorted (uint) sets of MERGE_MIN elements or more each, the
// larger at most MERGE_RATIO times the smaller, are co-iterated instead of
// probed (section 4.1.1's balanced case): the merged sequence is cut into
// tiles of MERGE_TILE elements along its diagonal (merge path), and one
// block streams a tile's two runs and intersects them in LDS.  Both sets
// are read once, in order.
constexpr int M_NT = 256;
constexpr int M_PER = 16;                       // merged elements per thread
constexpr uint32_t MERGE_TILE = M_NT * M_PER;
constexpr uint32_t MERGE_MIN = 1u << 12;
constexpr uint32_t MERGE_RATIO = 4;
// A tile is intersected through an LDS bitmap of MERGE_TILE words of 32
// bits when its value span fits, and the span is at most MERGE_BM_SPREAD
// values per key of the tile (clearing the bitmap then costs at most one
// word per four keys); sparser tiles are merged.  Rows are taken by the
// merge tiles only when their value span is that dense overall: sparser
// pairs intersect faster by the staged probes.
constexpr uint64_t MERGE_BM_SPAN = 32ull * MERGE_TILE;
constexpr uint64_t MERGE_BM_SPREAD = 8;

struct DSet {
  const uint32_t* ppos;   // frontier positions at the previous level (null: root set)
  const uint32_t* poffs;  // child offsets of the previous level (null: root set)
  const uint32_t* keys;   // keys of this level
  const uint32_t* samp;   // one key sample per line of keys
  uint32_t root_n;
  const uint64_t* bs_word;
  const uint32_t* bs_base;
  const uint64_t* pool;
  const uint32_t* bs_rank;   // rank directory of the bitset sets, or null
  const uint32_t* bs_delta;
  const uint64_t* root_bits; // root sets: level-0 bitmap with a rank per word, or null
  const uint32_t* root_rank;
  uint64_t root_span;
};

__device__ __forceinline__ void dset_range(const DSet& st, uint64_t row, uint32_t& b, uint32_t& e, uint64_t& sidx) {
  if (st.ppos) {
    uint32_t p = st.ppos[row];
    b = st.poffs[p];
    e = st.poffs[p + 1];
    sidx = p;
  } else {
    b = 0;
    e = st.root_n;
    sidx = 0;
  }
}

// Position of x in the sorted keys [b, e) (b < e) through the level's line
// samples: bisect the samples of the lines that start inside the range
// (a 32x smaller, cache-resident array), then the one line that can hold x.
__device__ __forceinline__ bool sampled_find(const uint32_t* keys, const uint32_t* samp, uint32_t b, uint32_t e,
                                             uint32_t x, uint32_t& pos) {
  const uint32_t jf = (b + (1u << LINE_SHIFT) - 1) >> LINE_SHIFT;
  const uint32_t jl = (e - 1) >> LINE_SHIFT;
  uint32_t k = 0;
  if (jl >= jf) {
    const uint32_t* sp = samp + jf;
    uint32_t n = jl - jf + 1;
    while (n > 1) {
      const uint32_t half = n >> 1;
      k = (sp[k + half - 1] <= x) ? k + half : k;
      n -= half;
    }
    k += (sp[k] <= x) ? 1u : 0u;
  }
  uint32_t lo = k ? (jf + k - 1) << LINE_SHIFT : b;
  const uint32_t hi = (uint32_t)min<uint64_t>(e, (uint64_t)(jf + k) << LINE_SHIFT);
  if (hi <= lo) return false;
  uint32_t len = hi - lo;
  while (len > 1) {
    const uint32_t half = len >> 1;
    lo = (keys[lo + half] <= x) ? lo + half : lo;
    len -= half;
  }
  pos = lo;
  return keys[lo] == x;
}

// First position in the sorted keys [b, e) holding a key >= x (e if none),
// through the line samples.
__device__ __forceinline__ uint32_t sampled_lower_bound(const uint32_t* keys, const uint32_t* samp, uint32_t b,
                                                        uint32_t e, uint32_t x) {
  if (b >= e) return b;
  uint32_t pos = b;
  if (sampled_find(keys, samp, b, e, x, pos)) return pos;
  return keys[pos] < x ? pos + 1 : pos;
}

// Membership of x in set [b, e) (descriptor sidx); its position if asked.
__device__ __forceinline__ bool dset_find(const DSet& st, uint32_t b, uint32_t e, uint64_t sidx, uint32_t x,
                                          bool need_pos, uint32_t& pos) {
  if (b >= e) return false;
  if (st.root_bits) {
    if (x >= st.root_span) return false;
    const uint64_t word = st.root_bits[x >> 6];
    if (!((word >> (x & 63u)) & 1ull)) return false;
    if (need_pos) pos = st.root_rank[x >> 6] + (uint32_t)__popcll(word & ((1ull << (x & 63u)) - 1ull));
    return true;
  }
  uint64_t w = st.bs_word[sidx];
  if (w != UINT64_MAX) {
    uint32_t base = st.bs_base[sidx];
    if (x < base || x > st.keys[e - 1]) return false;
    uint32_t d = x - base;
    uint64_t word = st.pool[w + (d >> 6)];
    if (!((word >> (d & 63u)) & 1ull)) return false;
    if (need_pos) {
      if (st.bs_rank)
        pos = st.bs_rank[w + (d >> 6)] + (uint32_t)__popcll(word & ((1ull << (d & 63u)) - 1ull)) + st.bs_delta[sidx];
      else
        (void)sampled_find(st.keys, st.samp, b, e, x, pos);
    }
    return true;
  }
  return sampled_find(st.keys, st.samp, b, e, x, pos);
}

struct LeafAtom {
  const uint32_t* pos;    // frontier position at its last level (non-participant)
  int32_t part;           // participant index at the leaf attribute, or -1
  const uint32_t* run;    // bag: run offsets of the last level; null: one row per node
  const double* anno;     // SUM factor column (trie order), or null
  const uint32_t* gmeta;  // a GROUP BY meta column of this atom (trie order), or null
  uint32_t expand;        // iterate the node's rows (anno or gmeta present)
};

struct LeafArgs {
  uint32_t n_atoms;
  LeafAtom at[MAXA];
  uint32_t sum;
  int32_t lsb;
  uint32_t D;
  // streamed groups (outputs are a prefix of the order)
  const uint32_t* gid;    // group of each frontier row (null: one group)
  uint64_t* gcount;
  int64_t* gacc;          // n_groups x EXACT_MAXD slots
  // materialized tuples
  uint32_t n_cols;
  uint32_t* col_out[MAXV + MAXA];
  int32_t col_src[MAXV + MAXA];  // >= 0: frontier out column; -1: leaf value; -2: group meta
  const uint32_t* gm_col[MAXV + MAXA];  // group meta column of output column c (trie order)
  int32_t gm_atom[MAXV + MAXA];         // its atom
  uint64_t* mult_out;
  double* hi_out;
  double* lo_out;
  uint32_t* err;
  // tuples aggregated in place (GROUP BY outside the order's prefix):
  // gmode 1 = dense array indexed by the mixed-radix key, 2 = hash table
  // (col_out = its key columns, gtag = slot states); counts in gcount and
  // exact digits in gacc at stride D
  uint32_t gmode;
  uint32_t* gtag;
  uint64_t gmask;
  uint64_t radix[MAXV + MAXA];
  // keys of at most 63 bits are packed into one word (column 0 highest),
  // claimed with one compare-and-swap; gkey64 is then the table
  uint64_t* gkey64;
  uint32_t gshift[MAXV + MAXA];
  // dense key spaces of at most GLDS_MAX entries are accumulated per block
  // in LDS and flushed once (few groups would serialize global atomics)
  uint32_t glds;
  uint32_t gspace;
};

constexpr uint64_t KEY64_EMPTY = ~0ull;
constexpr uint32_t GLDS_MAX = 256;

struct ElemArgs {
  uint32_t np;
  DSet set[MAXP];
  const uint64_t* W;      // exclusive scan of per-row work, nrows + 1 entries
  const uint8_t* drv;     // driving participant of each row
  uint64_t nrows;
  uint64_t total;
  const uint64_t* U;      // exclusive scan of per-row work units, nrows + 1 entries
  const uint32_t* urow;   // row of each unit
  uint64_t total_units;
  uint64_t nvblk;         // virtual blocks of J_NW units
  uint32_t need_pos_mask; // participants whose position is needed
  // fill
  uint32_t n_atoms;
  const uint32_t* pos_in[MAXA];
  uint32_t* pos_out[MAXA];
  int32_t part_of_atom[MAXA];
  uint32_t n_outv;
  const uint32_t* outv_in[MAXV];
  uint32_t* outv_out[MAXV];
  int32_t new_outv;       // out column taking the new value, or -1
  const uint32_t* gid_in;
  uint32_t* gid_out;
  uint32_t gid_mode;      // 0 none, 1 copy parent's, 2 own row index
  uint32_t* blk_cnt;
  const uint64_t* blk_off;
  LeafArgs leaf;
};

enum { M_COUNT = 0, M_FILL = 1, M_LEAF_A = 2, M_LEAF_B_COUNT = 3, M_LEAF_B_FILL = 4, M_LEAF_COUNT = 5,
       M_LEAF_B_AGG = 6 };

// Hash-table slot states (GROUP BY upserts)
constexpr uint32_t SLOT_EMPTY = 0, SLOT_BUSY = 1, SLOT_READY = 2;
// A slot being written is re-read at most this many times before the
// upsert gives up and flags an error (the writer publishes right after
// its claim, so the bound is never reached in a correct run)
constexpr uint32_t SLOT_SPIN_MAX = 1u << 22;
constexpr uint32_t ERR_TABLE_FULL = 2u, ERR_SLOT_SPIN = 4u;
// a tuple count (or a row multiplicity) does not fit 64 bits
constexpr uint32_t ERR_COUNT_OVERFLOW = 8u;

__device__ __forceinline__ uint64_t key_mix(uint64_t h, uint32_t v) {
  h ^= v;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  return h;
}

struct WorkArgs {
  uint32_t np;
  DSet set[MAXP];
};

// Driver value DRV_AND: the row's two sets are both bitsets and are
// intersected word by word (AND + popcount over the overlap of their
// windows); its work is counted in words instead of driver elements.
constexpr uint8_t DRV_AND = 0xff;
// Driver value DRV_MERGE: the row's two sorted sets are merged tile by tile
// (MERGE_TILE merged elements per unit).
constexpr uint8_t DRV_MERGE = 0xfe;

// leaf2: the row's two sets feed the two-set leaf (word-AND and merge
// allowed; top-bucket rows get units of TOP_EL elements, counted into
// n_units[0]; merged rows units of MERGE_TILE, counted into n_units[1]).
__global__ void k_work(WorkArgs a, uint64_t nrows, uint32_t* work, uint8_t* drv, uint32_t* units, uint32_t leaf2,
                       unsigned long long* n_units) {
  __shared__ uint64_t s_red[256 / WAVE];
  uint64_t top_units = 0, merge_units = 0;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (uint64_t)gridDim.x * blockDim.x) {
    // Driver: the set whose elements are cheapest to stream and probe into
    // the others; probing a bitset costs one word load, probing a sorted
    // uint array a binary search of ~log2(card) loads.
    uint32_t card[MAXP];
    float probe[MAXP];
    uint32_t bi = 0;
#pragma unroll
    for (int p = 0; p < MAXP; p++) {
      card[p] = 0;
      probe[p] = 1.0f;
      if (p >= (int)a.np) continue;
      uint32_t b, e;
      uint64_t sidx;
      dset_range(a.set[p], r, b, e, sidx);
      card[p] = e - b;
      const bool bs = card[p] && a.set[p].bs_word[sidx] != UINT64_MAX;
      probe[p] = bs ? 1.0f : 2.0f + log2f((float)card[p] + 1.0f);
    }
    float best_cost = 3.0e38f;
#pragma unroll
    for (int p = 0; p < MAXP; p++) {
      if (p >= (int)a.np) continue;
      float c = 0.0f;
#pragma unroll
      for (int q = 0; q < MAXP; q++)
        if (q < (int)a.np && q != p) c += probe[q];
      c = (float)card[p] * (c + 1.0f);
      if (c < best_cost) {
        best_cost = c;
        bi = (uint32_t)p;
      }
    }
    uint32_t best = 0;
    bool empty = false;
#pragma unroll
    for (int p = 0; p < MAXP; p++) {
      if (p == (int)bi) best = card[p];
      if (p < (int)a.np && card[p] == 0) empty = true;
    }
    if (empty) best = 0;
    uint8_t dv = (uint8_t)bi;
    uint32_t chunk = U_EL;
    if (leaf2 && a.np == 2 && !empty && probe[0] > 1.0f && probe[1] > 1.0f) {
      // two sorted sets of similar, large size whose values are dense
      // enough for the merge tiles' LDS bitmaps: merged
      const uint32_t lo = min(card[0], card[1]), hi = max(card[0], card[1]);
      if (lo >= MERGE_MIN && (uint64_t)hi <= (uint64_t)MERGE_RATIO * lo) {
        uint32_t b0, e0, b1, e1;
        uint64_t s0, s1;
        dset_range(a.set[0], r, b0, e0, s0);
        dset_range(a.set[1], r, b1, e1, s1);
        const uint32_t vmin = min(a.set[0].keys[b0], a.set[1].keys[b1]);
        const uint32_t vmax = max(a.set[0].keys[e0 - 1], a.set[1].keys[e1 - 1]);
        if ((uint64_t)(vmax - vmin) + 1 <= MERGE_BM_SPREAD * ((uint64_t)card[0] + card[1])) {
          dv = DRV_MERGE;
          best = card[0] + card[1];
          chunk = MERGE_TILE;
        }
      }
    }
    if (leaf2 && a.np == 2 && !empty) {
      // both bitsets: AND the overlapping words when that moves fewer words
      // than the probe path moves elements and probes
      uint32_t b0, e0, b1, e1;
      uint64_t s0, s1;
      dset_range(a.set[0], r, b0, e0, s0);
      dset_range(a.set[1], r, b1, e1, s1);
      const uint64_t w0 = a.set[0].bs_word[s0], w1 = a.set[1].bs_word[s1];
      if (w0 != UINT64_MAX && w1 != UINT64_MAX) {
        const uint32_t v0 = max(a.set[0].bs_base[s0], a.set[1].bs_base[s1]);
        const uint32_t v1 = min(a.set[0].keys[e0 - 1], a.set[1].keys[e1 - 1]);
        const uint32_t words = v1 >= v0 ? ((v1 - v0) >> 6) + 1 : 0;
        if (2.0f * (float)words < best_cost) {
          dv = DRV_AND;
          best = words;
        }
      }
    }
    work[r] = best;
    drv[r] = dv;
    const bool top = leaf2 && a.np == 2 && dv != DRV_MERGE && (uint64_t)card[0] + card[1] >= TOP_MIN;
    if (top) {
      const float probed = dv == 0 ? probe[1] : probe[0];   // the probed set's cost: 1 for a bitset
      chunk = leaf2_chunk(card[0], card[1], dv == DRV_AND || (dv < 2 && probed == 1.0f));
    }
    units[r] = (best + chunk - 1) / chunk;
    if (top) top_units += units[r];
    if (dv == DRV_MERGE) merge_units += units[r];
  }
  if (n_units) {
    const uint64_t t = block_sum<uint64_t, 256>(top_units, s_red);
    if (threadIdx.x == 0 && t) atomicAdd(&n_units[0], (unsigned long long)t);
    const uint64_t m = block_sum<uint64_t, 256>(merge_units, s_red);
    if (threadIdx.x == 0 && m) atomicAdd(&n_units[1], (unsigned long long)m);
  }
}

// Rows of a leaf hit: for each atom, the range of rows of its leaf node.
struct HitRows {
  uint32_t rb[MAXA], re[MAXA];
  uint64_t mult;  // product of run lengths of the non-expanding atoms
};

template <int NP>
__device__ __forceinline__ void leaf_rows(const LeafArgs& L, uint64_t r, const uint32_t* ppos, HitRows& h) {
  h.mult = 1;
#pragma unroll
  for (int e = 0; e < MAXA; e++) {
    if (e >= (int)L.n_atoms) break;
    const LeafAtom& A = L.at[e];
    uint32_t lp = 0;
    if (A.part >= 0) {
#pragma unroll
      for (int q = 0; q < NP; q++)
        if (q == A.part) lp = ppos[q];
    } else if (A.pos) {
      lp = A.pos[r];
    }
    uint32_t b = lp, en = lp + 1;
    if (A.run) {
      b = A.run[lp];
      en = A.run[lp + 1];
    }
    h.rb[e] = b;
    h.re[e] = en;
    if (!A.expand) h.mult = sat_mul_u64(h.mult, (uint64_t)(en - b));
  }
}

// Product term of one row combination: (hi, lo) with hi + lo exact.  The
// factors are taken in atom order; all but the last are multiplied with
// rounding, the last multiplication is exact (a two-product).
__device__ __forceinline__ void term_of(const LeafArgs& L, const uint32_t* cur, double& hi, double& lo) {
  double p = 1.0, last = 1.0;
  int nf = 0;
#pragma unroll
  for (int e = 0; e < MAXA; e++) {
    if (e >= (int)L.n_atoms) break;
    if (!L.at[e].anno) continue;
    double v = L.at[e].anno[cur[e]];
    if (nf == 0) p = v;
    else if (nf == 1) last = v;
    else {
      p = __dmul_rn(p, last);
      last = v;
    }
    nf++;
  }
  if (nf <= 1) {
    hi = p;
    lo = 0.0;
  } else {
    two_prod(p, last, hi, lo);
  }
}

// Number of row combinations of the expanding atoms (UINT64_MAX when it
// does not fit 64 bits).
__device__ __forceinline__ uint64_t combos(const LeafArgs& L, const HitRows& h) {
  uint64_t c = 1;
#pragma unroll
  for (int e = 0; e < MAXA; e++) {
    if (e >= (int)L.n_atoms) break;
    if (L.at[e].expand) c = sat_mul_u64(c, (uint64_t)(h.re[e] - h.rb[e]));
  }
  return c;
}

// Add v to a tuple count; a count that leaves 64 bits flags an error.
__device__ __forceinline__ void atomic_add_count(uint64_t* c, uint64_t v, uint32_t* err) {
  const uint64_t old = atomicAdd((unsigned long long*)c, (unsigned long long)v);
  if (v == UINT64_MAX || old + v < old) atomicOr(err, ERR_COUNT_OVERFLOW);
}

// Advance the odometer over expanding atoms; false when exhausted.
__device__ __forceinline__ bool next_combo(const LeafArgs& L, const HitRows& h, uint32_t* cur) {
  bool carry = true;
#pragma unroll
  for (int e = MAXA - 1; e >= 0; e--) {
    if (!carry) break;
    if (e >= (int)L.n_atoms || !L.at[e].expand) continue;
    if (++cur[e] < h.re[e]) {
      carry = false;
    } else {
      cur[e] = h.rb[e];
    }
  }
  return !carry;
}

// NP bounds the participants at the attribute (a.np <= NP): the per-set
// arrays stay in registers at the size the plan needs.
template <int MODE, int NP>
__global__ __launch_bounds__(J_NT) void k_elem(ElemArgs a) {
  __shared__ uint64_t s_wcnt[J_NW];
  __shared__ uint64_t s_red[J_NW];
  __shared__ unsigned long long s_cnt;
  __shared__ long long s_acc[EXACT_MAXD];

  constexpr bool GAGG = MODE == M_LEAF_B_AGG;
  __shared__ unsigned long long s_gcnt[GAGG ? GLDS_MAX : 1];
  __shared__ long long s_gdig[GAGG ? GLDS_MAX * EXACT_MAXD : 1];

  const int tid = threadIdx.x;
  const int w = tid / WAVE;
  const int lane = lane_id();
  const LeafArgs& L = a.leaf;
  constexpr bool NEED_POS = !(MODE == M_COUNT || MODE == M_LEAF_COUNT);
  constexpr bool LEAF_AGG = (MODE == M_LEAF_A || MODE == M_LEAF_COUNT);
  const bool one_group = LEAF_AGG && L.gid == nullptr;
  if constexpr (GAGG) {
    if (L.glds) {
      for (uint32_t i = tid; i < GLDS_MAX; i += J_NT) s_gcnt[i] = 0;
      for (uint32_t i = tid; i < GLDS_MAX * EXACT_MAXD; i += J_NT) s_gdig[i] = 0;
      __syncthreads();
    }
  }

  if (LEAF_AGG && tid == 0) {
    s_cnt = 0;
    for (int i = 0; i < EXACT_MAXD; i++) s_acc[i] = 0;
  }
  // one-group aggregation is carried across the block's virtual blocks
  uint64_t run_cnt = 0;
  RegAcc run_acc;
  run_acc.clear();
  uint32_t bad = 0;

  // The grid is capped (a dispatch holds < 2^32 work-items); each block
  // walks virtual blocks of J_NW units.
  for (uint64_t vb = blockIdx.x; vb < a.nvblk; vb += gridDim.x) {
    const uint64_t u = vb * J_NW + w;
    const bool wave_valid = u < a.total_units;

    // the wave's row and chunk (uniform across the wave)
    uint64_t r = 0;
    uint32_t chunk = 0, work = 0, d = 0;
    if (wave_valid) {
      r = a.urow[u];
      chunk = (uint32_t)(u - a.U[r]);
      work = (uint32_t)(a.W[r + 1] - a.W[r]);
      d = a.drv[r];
    }
    uint32_t b[NP], e[NP];
    uint64_t sidx[NP];
    uint32_t bd = 0;
    const uint32_t* dkeys = nullptr;
#pragma unroll
    for (int p = 0; p < NP; p++) {
      b[p] = e[p] = 0;
      sidx[p] = 0;
      if (p < (int)a.np && wave_valid) dset_range(a.set[p], r, b[p], e[p], sidx[p]);
      if (p == (int)d) {
        bd = b[p];
        dkeys = a.set[p].keys;
      }
    }

    bool hit[U_IT];
    uint32_t x[U_IT];
    uint32_t ppos[U_IT][NEED_POS ? NP : 1];
#pragma unroll
    for (int it = 0; it < U_IT; it++) {
      const uint32_t i = chunk * U_EL + it * WAVE + lane;
      const bool valid = wave_valid && i < work;
      hit[it] = valid;
      x[it] = valid ? dkeys[bd + i] : 0u;
      if constexpr (NEED_POS) {
#pragma unroll
        for (int p = 0; p < NP; p++) ppos[it][p] = (p == (int)d) ? bd + i : 0u;
      }
    }
    // probe the other sets; iterations are independent, so their loads overlap
#pragma unroll
    for (int p = 0; p < NP; p++) {
      if (p >= (int)a.np) break;
      if (p == (int)d) continue;
      const bool np_ = NEED_POS && ((a.need_pos_mask >> p) & 1u);
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        uint32_t dummy;
        if (hit[it])
          hit[it] = dset_find(a.set[p], b[p], e[p], sidx[p], x[it], np_, NEED_POS ? ppos[it][NEED_POS ? p : 0] : dummy);
      }
    }

    if (MODE == M_LEAF_COUNT) {
      // every hit is one tuple (set relations, COUNT)
      uint64_t c = 0;
#pragma unroll
      for (int it = 0; it < U_IT; it++) c += hit[it] ? 1 : 0;
      if (one_group) {
        run_cnt += c;
      } else {
        c = wave_sum(c);
        if (wave_valid && lane == 0 && c) atomicAdd((unsigned long long*)&L.gcount[L.gid[r]], (unsigned long long)c);
      }
    } else if (MODE == M_COUNT) {
      uint64_t c = 0;
#pragma unroll
      for (int it = 0; it < U_IT; it++) c += hit[it] ? 1 : 0;
      uint64_t t = block_sum<uint64_t, J_NT>(c, s_red);
      if (tid == 0) a.blk_cnt[vb] = (uint32_t)t;
    } else if (MODE == M_FILL) {
      // order: units in block order, elements in order inside a unit
      uint32_t wc = 0;
#pragma unroll
      for (int it = 0; it < U_IT; it++) wc += (uint32_t)__popcll(ballot(hit[it]));
      if (lane == 0) s_wcnt[w] = wc;
      __syncthreads();
      uint64_t off = a.blk_off[vb];
      for (int j = 0; j < w; j++) off += s_wcnt[j];
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        const uint64_t bal = ballot(hit[it]);
        if (hit[it]) {
          const uint64_t o = off + lanes_below(bal);
#pragma unroll
          for (int at = 0; at < MAXA; at++) {
            if (at >= (int)a.n_atoms) break;
            uint32_t* po = a.pos_out[at];
            if (!po) continue;
            const int32_t pa = a.part_of_atom[at];
            uint32_t v = 0;
            if (pa >= 0) {
#pragma unroll
              for (int q = 0; q < NP; q++)
                if (q == pa) v = ppos[it][q];
            } else {
              v = a.pos_in[at][r];
            }
            po[o] = v;
          }
          for (uint32_t j = 0; j < a.n_outv; j++) {
            uint32_t* ov = a.outv_out[j];
            if (!ov) continue;
            ov[o] = ((int32_t)j == a.new_outv) ? x[it] : a.outv_in[j][r];
          }
          if (a.gid_mode == 1) a.gid_out[o] = a.gid_in[r];
          else if (a.gid_mode == 2) a.gid_out[o] = (uint32_t)o;
        }
        off += (uint64_t)__popcll(bal);
      }
      __syncthreads();
    } else if (MODE == M_LEAF_A) {
      uint64_t cnt = 0;
      RegAcc acc;
      acc.clear();
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        if (!hit[it]) continue;
        HitRows h;
        leaf_rows<NP>(L, r, ppos[it], h);
        const uint64_t nc = combos(L, h);
        cnt = sat_add_u64(cnt, sat_mul_u64(h.mult, nc));
        if (L.sum && nc) {
          uint32_t cur[MAXA];
#pragma unroll
          for (int at = 0; at < MAXA; at++) cur[at] = h.rb[at];
          do {
            double hi, lo;
            term_of(L, cur, hi, lo);
            bool ok = acc.add(hi, L.lsb, L.D, h.mult);
            ok = acc.add(lo, L.lsb, L.D, h.mult) && ok;
            if (!ok) bad |= 1u;
          } while (next_combo(L, h, cur));
        }
      }
      if (cnt == UINT64_MAX) bad |= ERR_COUNT_OVERFLOW;
      if (L.sum) acc.normalize(L.D);
      if (one_group) {
        run_cnt = sat_add_u64(run_cnt, cnt);
#pragma unroll
        for (int i = 0; i < EXACT_MAXD; i++) run_acc.s[i] += acc.s[i];
        if (L.sum) run_acc.normalize(L.D);
      } else {
        // the wave's unit belongs to one row, hence to one group; lane
        // counts below 2^58 cannot wrap the wave's sum
        if (__any(cnt >= (1ull << 58))) bad |= ERR_COUNT_OVERFLOW;
        cnt = wave_sum(cnt);
        if (wave_valid) {
          const uint64_t g = L.gid[r];
          if (lane == 0 && cnt) atomic_add_count(&L.gcount[g], cnt, L.err);
          if (L.sum)
            for (uint32_t i = 0; i < L.D; i++) {
              // normalized lane digits: the wave's sum stays below 2^38
              const int64_t v = wave_sum(acc.s[i]);
              if (lane == 0 && v) atomic_add_digit(L.gacc + g * EXACT_MAXD, i, L.D, v);
            }
        }
      }
    } else if (MODE == M_LEAF_B_COUNT) {
      // rows to materialize; a block's count saturates at UINT32_MAX, which
      // the host's limit of 2^32 - 1 emitted rows then rejects
      uint64_t c = 0;
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        if (!hit[it]) continue;
        HitRows h;
        leaf_rows<NP>(L, r, ppos[it], h);
        c = sat_add_u64(c, combos(L, h));
      }
      c = min(c, (uint64_t)UINT32_MAX);
      uint64_t t = block_sum<uint64_t, J_NT>(c, s_red);
      if (tid == 0) a.blk_cnt[vb] = (uint32_t)min(t, (uint64_t)UINT32_MAX);
    } else if (MODE == M_LEAF_B_FILL) {
      uint64_t m[U_IT];
      uint64_t wtot = 0;
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        m[it] = 0;
        if (hit[it]) {
          HitRows h;
          leaf_rows<NP>(L, r, ppos[it], h);
          m[it] = combos(L, h);
        }
        wtot += wave_sum(m[it]);
      }
      if (lane == 0) s_wcnt[w] = wtot;
      __syncthreads();
      uint64_t off = a.blk_off[vb];
      for (int j = 0; j < w; j++) off += s_wcnt[j];
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        const uint64_t incl = wave_incl_scan(m[it]);
        const uint64_t tot = __shfl(incl, WAVE - 1, WAVE);
        if (m[it]) {
          HitRows h;
          leaf_rows<NP>(L, r, ppos[it], h);
          uint32_t cur[MAXA];
#pragma unroll
          for (int at = 0; at < MAXA; at++) cur[at] = h.rb[at];
          uint64_t o = off + incl - m[it];
          do {
            for (uint32_t c = 0; c < L.n_cols; c++) {
              const int32_t src = L.col_src[c];
              uint32_t v;
              if (src >= 0) v = a.outv_in[src][r];
              else if (src == -1) v = x[it];
              else {
                v = 0;
                const int32_t ga = L.gm_atom[c];
#pragma unroll
                for (int at = 0; at < MAXA; at++)
                  if (at == ga) v = L.gm_col[c][cur[at]];
              }
              L.col_out[c][o] = v;
            }
            L.mult_out[o] = h.mult;
            if (L.sum) {
              double hi, lo;
              term_of(L, cur, hi, lo);
              L.hi_out[o] = hi;
              L.lo_out[o] = lo;
            }
            o++;
          } while (next_combo(L, h, cur));
        }
        off += tot;
      }
      __syncthreads();
    } else if (MODE == M_LEAF_B_AGG) {
      // once the hash table is known to be too small the pass is wasted:
      // skip the remaining units (the host sizes the table and reruns)
      const bool table_full = L.gmode == 2 &&
          (__hip_atomic_load(L.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TABLE_FULL);
#pragma unroll
      for (int it = 0; it < U_IT; it++) {
        if (!hit[it] || table_full) continue;
        HitRows h;
        leaf_rows<NP>(L, r, ppos[it], h);
        if (!combos(L, h)) continue;
        uint32_t cur[MAXA];
#pragma unroll
        for (int at = 0; at < MAXA; at++) cur[at] = h.rb[at];
        do {
          auto val = [&](uint32_t c) -> uint32_t {
            const int32_t src = L.col_src[c];
            if (src >= 0) return a.outv_in[src][r];
            if (src == -1) return x[it];
            uint32_t v = 0;
            const int32_t ga = L.gm_atom[c];
#pragma unroll
            for (int at = 0; at < MAXA; at++)
              if (at == ga) v = L.gm_col[c][cur[at]];
            return v;
          };
          uint64_t slot = 0;
          bool ok = true;
          if (L.gmode == 1) {
            for (uint32_t c = 0; c < L.n_cols; c++) slot = slot * L.radix[c] + val(c);
          } else if (L.gkey64) {
            uint64_t k = 0;
            for (uint32_t c = 0; c < L.n_cols; c++) k |= (uint64_t)val(c) << L.gshift[c];
            uint64_t hs = k * 0x9e3779b97f4a7c15ull;
            hs ^= hs >> 31;
            slot = hs & L.gmask;
            ok = false;
            const uint64_t max_probes = L.gmask < 256 ? L.gmask + 1 : 256;
            for (uint64_t probes = 0; probes < max_probes; probes++) {
              uint64_t cur = L.gkey64[slot];
              if (cur == KEY64_EMPTY) {
                // the swap returns the word's true value, whatever a cached
                // read said
                cur = atomicCAS((unsigned long long*)&L.gkey64[slot], (unsigned long long)KEY64_EMPTY,
                                (unsigned long long)k);
                if (cur == KEY64_EMPTY) cur = k;
              }
              if (cur == k) {
                ok = true;
                break;
              }
              slot = (slot + 1) & L.gmask;
            }
            if (!ok) {
              atomicOr(L.err, ERR_TABLE_FULL);
              break;
            }
          } else {
            uint64_t hs = 0x9e3779b97f4a7c15ull;
            for (uint32_t c = 0; c < L.n_cols; c++) hs = key_mix(hs, val(c));
            slot = hs & L.gmask;
            ok = false;
            // a probe run longer than this means the table is too full: the
            // host grows it and runs the pass again
            const uint64_t max_probes = L.gmask < 256 ? L.gmask + 1 : 256;
            uint64_t probes = 0;
            uint32_t spins = 0;
            while (probes < max_probes) {
              const uint32_t t = __hip_atomic_load(&L.gtag[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
              if (t == SLOT_READY) {
                bool same = true;
                for (uint32_t c = 0; c < L.n_cols && same; c++) same = L.col_out[c][slot] == val(c);
                if (same) {
                  ok = true;
                  break;
                }
                slot = (slot + 1) & L.gmask;
                probes++;
                continue;
              }
              if (t == SLOT_EMPTY && atomicCAS(&L.gtag[slot], SLOT_EMPTY, SLOT_BUSY) == SLOT_EMPTY) {
                for (uint32_t c = 0; c < L.n_cols; c++) L.col_out[c][slot] = val(c);
                __hip_atomic_store(&L.gtag[slot], SLOT_READY, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                ok = true;
                break;
              }
              // claimed by another upsert that is writing its key: read again
              if (++spins > SLOT_SPIN_MAX) break;
            }
            if (!ok) {
              atomicOr(L.err, spins > SLOT_SPIN_MAX ? ERR_SLOT_SPIN : ERR_TABLE_FULL);
              break;  // this lane's remaining tuples wait for the rerun
            }
          }
          if (ok) {
            if (GAGG && L.glds) atomic_add_count((uint64_t*)&s_gcnt[slot], h.mult, L.err);
            else atomic_add_count(&L.gcount[slot], h.mult, L.err);
            if (L.sum) {
              double hi, lo;
              term_of(L, cur, hi, lo);
              int64_t* dig = (GAGG && L.glds) ? (int64_t*)&s_gdig[slot * EXACT_MAXD] : L.gacc + slot * L.D;
              bool fits = atomic_add_term(dig, hi, L.lsb, L.D, h.mult);
              fits = atomic_add_term(dig, lo, L.lsb, L.D, h.mult) && fits;
              if (!fits) bad |= 1u;
            }
          }
        } while (next_combo(L, h, cur));
      }
    }
  }

  if (MODE == M_LEAF_B_AGG && bad) atomicOr(L.err, bad);
  if constexpr (GAGG) {
    if (L.glds) {
      // flush the block's groups, each carried into normalized digits
      __syncthreads();
      for (uint32_t i = tid; i < L.gspace; i += J_NT) {
        const unsigned long long c = s_gcnt[i];
        if (!c) continue;
        atomic_add_count(&L.gcount[i], c, L.err);
        if (L.sum) {
          RegAcc t;
          t.load_shared((const int64_t*)&s_gdig[i * EXACT_MAXD], L.D);
          atomic_add_acc(L.gacc + i * L.D, t, L.D);
        }
      }
    }
  }
  if (LEAF_AGG) {
    if (bad) atomicOr(L.err, bad);
    if (one_group) {
      // reduce the block into LDS, one flush per block
      __syncthreads();
      if (__any(run_cnt >= (1ull << 58))) atomicOr(L.err, ERR_COUNT_OVERFLOW);
      const uint64_t c = wave_sum(run_cnt);
      if (lane == 0 && c) atomic_add_count((uint64_t*)&s_cnt, c, L.err);
      if (MODE == M_LEAF_A && L.sum)
        for (uint32_t i = 0; i < L.D; i++) {
          const int64_t v = wave_sum(run_acc.s[i]);
          if (lane == 0 && v) atomic_add_digit((int64_t*)s_acc, i, L.D, v);
        }
      __syncthreads();
      if (tid == 0) {
        if (s_cnt) atomic_add_count(&L.gcount[0], s_cnt, L.err);
        if (MODE == M_LEAF_A && L.sum) {
          RegAcc t;
          t.load_shared((const int64_t*)s_acc, L.D);
          atomic_add_acc(L.gacc, t, L.D);
        }
      }
    }
  }
}

template <int MODE>
void launch_elem(const ElemArgs& a, unsigned grid, hipStream_t s) {
  if (a.np <= 2) k_elem<MODE, 2><<<grid, J_NT, 0, s>>>(a);
  else if (a.np <= 4) k_elem<MODE, 4><<<grid, J_NT, 0, s>>>(a);
  else k_elem<MODE, MAXP><<<grid, J_NT, 0, s>>>(a);
}

// Row of every work unit.  A thread writes up to UROW_SMALL units of its
// row; rows with more are listed and finished by whole blocks.
constexpr uint64_t UROW_SMALL = 16;

__global__ void k_unit_rows(const uint64_t* U, uint64_t nrows, uint32_t* urow, uint32_t* big, uint32_t* nbig) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t u0 = U[r];
    uint64_t u1 = U[r + 1];
    if (u1 - u0 > UROW_SMALL) {
      big[atomicAdd(nbig, 1u)] = (uint32_t)r;
      u1 = u0 + UROW_SMALL;
    }
    for (uint64_t u = u0; u < u1; u++) urow[u] = (uint32_t)r;
  }
}

__global__ void k_unit_rows_big(const uint64_t* U, const uint32_t* big, const uint32_t* nbig, uint32_t* urow) {
  const uint32_t nb = *nbig;
  for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
    const uint32_t r = big[i];
    for (uint64_t u = U[r] + UROW_SMALL + threadIdx.x; u < U[r + 1]; u += blockDim.x) urow[u] = r;
  }
}

// ---- two-set COUNT leaf with per-unit descriptors ----------------------------
// Probed keys a wave stages in LDS (4 waves x 4 KB per block keeps 8 waves
// per SIMD; 2048 keys halved the occupancy and cost 65%).
constexpr int L2_CAP = 1024;
// Stage at most this many probed keys per driver key: beyond it, bisecting
// the range's line samples reads fewer bytes than staging the range.
constexpr uint32_t L2_STAGE_RATIO = 8;

// For the common leaf of two participating sets and set semantics, every
// work unit is described once: its driver key range, and either the probed
// set's bitset window or the part of the probed sorted keys that the unit's
// driver values can meet.  A wave then needs one descriptor load before it
// streams its driver keys and that key range side by side.
struct UnitDesc {
  uint32_t dstart;   // first driver element (index into the driver's level keys)
  uint32_t dcount;   // driver elements in this unit (1..U_EL; top bucket 1..TOP_EL)
  uint32_t plo;      // uint: first probed key index; bitset: window base value
  uint32_t phi;      // uint: end of probed keys (UINT32_MAX: next unit's plo); bitset: largest value
  uint64_t pword;    // probed set's first bitset word, or UINT64_MAX (sorted keys)
  uint32_t drv;      // driving participant (0 or 1), or DRV_AND: words [plo | phi << 32, +dcount) of
                     // participant 0's pool AND words [pword, +dcount) of participant 1's; or
                     // DRV_MERGE: keys [dstart, +dcount) of participant 0 and [plo, +phi) of
                     // participant 1 form one merge tile, pword = 1 when keys[0][dstart - 1]
                     // belongs to the row (the tile's look-back element)
  uint32_t top;      // 1: the unit's row is in the top bucket; 2: a merge tile (each class
                     // runs as a launch of its own)
};



// First index in [lo, hi) whose value is > x (hi if none).
__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Merge path: the number of elements of the sorted a[0, na) among the
// first d elements of the merge of a and b[0, nb), where an element of a
// goes before an equal element of b.  0 <= d <= na + nb.
__device__ __forceinline__ uint32_t merge_split(const uint32_t* a, uint32_t na, const uint32_t* b, uint32_t nb,
                                                uint64_t d) {
  uint32_t lo = d > nb ? (uint32_t)(d - nb) : 0u;
  uint32_t hi = (uint32_t)min<uint64_t>(d, na);
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (a[mid] <= b[d - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One thread per unit.  Consecutive units of a row split the driver into
// chunks of U_EL sorted keys; a chunk can only meet probed keys from the
// lower bound of its first key up to the lower bound of the next chunk's
// first key (the last chunk: the upper bound of its last key).  Units of a
// merged row are its merge path's tiles.  When top_flag / merge_flag are
// given, units of top-bucket rows / merge tiles are flagged.
__global__ void k_unit_desc(WorkArgs wa, const uint64_t* U, const uint32_t* urow, const uint8_t* drv, uint64_t units,
                            UnitDesc* desc, uint32_t* top_flag, uint32_t* merge_flag) {
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = urow[u];
    const uint64_t u0 = U[r], u1 = U[r + 1];
    uint32_t b[2], e[2];
    uint64_t sidx[2];
    dset_range(wa.set[0], r, b[0], e[0], sidx[0]);
    dset_range(wa.set[1], r, b[1], e[1], sidx[1]);
    const uint32_t d = drv[r];
    UnitDesc t;
    if (merge_flag) merge_flag[u] = d == DRV_MERGE ? 1u : 0u;
    if (d == DRV_MERGE) {
      const uint32_t na = e[0] - b[0], nb = e[1] - b[1];
      const uint64_t d0 = (u - u0) * (uint64_t)MERGE_TILE;
      const uint64_t d1 = min<uint64_t>(d0 + MERGE_TILE, (uint64_t)na + nb);
      const uint32_t* ka = wa.set[0].keys + b[0];
      const uint32_t* kb = wa.set[1].keys + b[1];
      const uint32_t i0 = merge_split(ka, na, kb, nb, d0), i1 = merge_split(ka, na, kb, nb, d1);
      t.drv = DRV_MERGE;
      t.dstart = b[0] + i0;
      t.dcount = i1 - i0;
      t.plo = b[1] + (uint32_t)(d0 - i0);
      t.phi = (uint32_t)(d1 - i1) - (uint32_t)(d0 - i0);
      t.pword = i0 > 0 ? 1u : 0u;
      t.top = 2;
      if (top_flag) top_flag[u] = 0;
      desc[u] = t;
      continue;
    }
    // the row's bucket and unit size, as k_work decided them
    const bool is_top = (uint64_t)(e[0] - b[0]) + (e[1] - b[1]) >= TOP_MIN;
    const bool probes_bitset = d < 2 && (d ? e[0] > b[0] && wa.set[0].bs_word[sidx[0]] != UINT64_MAX
                                               : e[1] > b[1] && wa.set[1].bs_word[sidx[1]] != UINT64_MAX);
    const uint32_t chunk = is_top ? leaf2_chunk(e[0] - b[0], e[1] - b[1], d == DRV_AND || probes_bitset) : U_EL;
    t.top = is_top ? 1u : 0u;
    if (top_flag) top_flag[u] = t.top;
    if (d == DRV_AND) {
      // word k of each window covers base + 64 k; both bases are multiples of 64
      const uint32_t base0 = wa.set[0].bs_base[sidx[0]], base1 = wa.set[1].bs_base[sidx[1]];
      const uint32_t v0 = max(base0, base1);
      const uint32_t v1 = min(wa.set[0].keys[e[0] - 1], wa.set[1].keys[e[1] - 1]);
      const uint32_t words = ((v1 - v0) >> 6) + 1;
      const uint32_t k0 = (uint32_t)(u - u0) * chunk;
      const uint64_t w0 = wa.set[0].bs_word[sidx[0]] + ((v0 - base0) >> 6) + k0;
      t.drv = DRV_AND;
      t.dstart = 0;
      t.dcount = min(chunk, words - k0);
      t.plo = (uint32_t)w0;
      t.phi = (uint32_t)(w0 >> 32);
      t.pword = wa.set[1].bs_word[sidx[1]] + ((v0 - base1) >> 6) + k0;
      desc[u] = t;
      continue;
    }
    const uint32_t db = d ? b[1] : b[0], de = d ? e[1] : e[0];
    const uint32_t pb = d ? b[0] : b[1], pe = d ? e[0] : e[1];
    const uint64_t sq = d ? sidx[0] : sidx[1];
    const uint32_t* dk = d ? wa.set[1].keys : wa.set[0].keys;
    const uint32_t* pk = d ? wa.set[0].keys : wa.set[1].keys;
    const uint32_t* ps = d ? wa.set[0].samp : wa.set[1].samp;
    const uint64_t* bsw = d ? wa.set[0].bs_word : wa.set[1].bs_word;
    const uint32_t* bsb = d ? wa.set[0].bs_base : wa.set[1].bs_base;
    t.drv = d;
    t.dstart = db + (uint32_t)(u - u0) * chunk;
    t.dcount = min(chunk, de - t.dstart);
    t.pword = (pe > pb) ? bsw[sq] : UINT64_MAX;
    if (t.pword != UINT64_MAX) {
      t.plo = bsb[sq];
      t.phi = pk[pe - 1];
    } else if (u0 + 1 == u1 && pe - pb <= (uint32_t)L2_CAP && pe - pb <= 2 * t.dcount + WAVE) {
      // the row's only unit, against a probed set no larger than about
      // twice its driver: the whole set is staged, no search needed
      t.plo = pb;
      t.phi = pe;
    } else {
      // the unit's first (and, for a row's last unit, last) key, loaded
      // together; quinary searches keep the dependent chain short
      const uint32_t first = dk[t.dstart];
      const uint32_t last = u + 1 == u1 ? dk[t.dstart + t.dcount - 1] : 0u;
      t.plo = lower_bound_sampled_quinary(pk, ps, pb, pe, first);
      if (u + 1 == u1) {
        t.phi = last == UINT32_MAX ? pe : lower_bound_sampled_quinary(pk, ps, t.plo, pe, last + 1);
      } else {
        t.phi = UINT32_MAX;
      }
    }
    desc[u] = t;
  }
}

struct Leaf2Args {
  const uint32_t* keys[2];
  const uint32_t* samp[2];
  const uint64_t* pool[2];
  const UnitDesc* desc;
  const uint32_t* list;   // top-bucket launch: the units to run (units = their number)
  uint64_t n_desc;        // descriptors (all units of the leaf)
  uint64_t* ucnt;         // grouped: count of every unit; null: one group, summed into gcount[0]
  uint64_t* gcount;
  uint64_t units;
  uint64_t nvblk;
};

// Groups own contiguous runs of units (frontier rows are in group order):
// a group's count is the difference of the scanned unit counts at the ends
// of its run.
__global__ void k_group_bounds(const uint32_t* urow, const uint32_t* gid, uint64_t units, const uint64_t* uex,
                               uint64_t* gstart, uint64_t* gend) {
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = gid[urow[u]];
    if (u == 0 || gid[urow[u - 1]] != g) gstart[g] = uex[u];
    if (u + 1 == units || gid[urow[u + 1]] != g) gend[g] = uex[u + 1];
  }
}

__global__ void k_group_add(const uint64_t* gstart, const uint64_t* gend, uint64_t n, uint64_t* gcount) {
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (uint64_t)gridDim.x * blockDim.x)
    gcount[g] += gend[g] - gstart[g];
}


// Membership of x[it] (it < nit) in the strictly increasing keys a[0, m),
// m >= 1: a branchless bisection whose trip count depends on m only, so the
// probes of a lane's values are issued together.  nit is wave-uniform.
template <int NIT, class Arr>
__device__ __forceinline__ uint32_t count_members(Arr a, uint32_t m, const uint32_t* x, const bool* v, uint32_t nit) {
  uint32_t lo[NIT];
#pragma unroll
  for (int it = 0; it < NIT; it++) lo[it] = 0;
  uint32_t n = m;
  while (n > 1) {
    const uint32_t half = n >> 1;
#pragma unroll
    for (int it = 0; it < NIT; it++)
      if (it < (int)nit) lo[it] = (a[lo[it] + half] <= x[it]) ? lo[it] + half : lo[it];
    n -= half;
  }
  uint32_t c = 0;
#pragma unroll
  for (int it = 0; it < NIT; it++)
    if (it < (int)nit) c += (v[it] && a[lo[it]] == x[it]) ? 1u : 0u;
  return c;
}

// Number of entries <= x[it] in the sorted a[0, n), n >= 1, for it < nit:
// branchless, trip count set by n alone.
template <int NIT, class Arr>
__device__ __forceinline__ void count_le(Arr a, uint32_t n0, const uint32_t* x, uint32_t nit, uint32_t* k) {
#pragma unroll
  for (int it = 0; it < NIT; it++) k[it] = 0;
  uint32_t n = n0;
  while (n > 1) {
    const uint32_t half = n >> 1;
#pragma unroll
    for (int it = 0; it < NIT; it++)
      if (it < (int)nit) k[it] = (a[k[it] + half - 1] <= x[it]) ? k[it] + half : k[it];
    n -= half;
  }
#pragma unroll
  for (int it = 0; it < NIT; it++)
    if (it < (int)nit) k[it] += (a[k[it]] <= x[it]) ? 1u : 0u;
}

// The wave copies src[0, m) to LDS, U_IT loads in flight per lane.
__device__ __forceinline__ void wave_stage(uint32_t* dst, const uint32_t* src, uint32_t m, int lane) {
  for (uint32_t k0 = 0; k0 < m; k0 += U_IT * WAVE) {
    uint32_t t[U_IT];
#pragma unroll
    for (int j = 0; j < U_IT; j++) {
      const uint32_t i = k0 + j * WAVE + lane;
      t[j] = i < m ? src[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < U_IT; j++) {
      const uint32_t i = k0 + j * WAVE + lane;
      if (i < m) dst[i] = t[j];
    }
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  // LDS operations of one wave complete in order; this keeps the compiler
  // from moving them across the point where lanes read what others wrote
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Probe path of a unit: the unit's driver keys against the probed set's
// bitset, its LDS-staged keys, or its line samples.
template <int NIT>
__device__ __forceinline__ uint32_t probe_unit(const Leaf2Args& a, const UnitDesc& t, uint32_t next_lo, uint32_t* stage,
                                               int lane) {
  uint32_t c = 0;
  const uint32_t* dk = t.drv ? a.keys[1] : a.keys[0];
  const uint32_t* pk = t.drv ? a.keys[0] : a.keys[1];
  const uint64_t* pool = t.drv ? a.pool[0] : a.pool[1];
  const uint32_t nit = (t.dcount + WAVE - 1) / WAVE;
  uint32_t x[NIT];
  bool v[NIT];
#pragma unroll
  for (int it = 0; it < NIT; it++) {
    const uint32_t i = it * WAVE + lane;
    v[it] = i < t.dcount;
    x[it] = v[it] ? dk[t.dstart + i] : 0u;
  }
  if (t.pword != UINT64_MAX) {
#pragma unroll
    for (int it = 0; it < NIT; it++) {
      if (!v[it] || x[it] < t.plo || x[it] > t.phi) continue;
      const uint32_t dd = x[it] - t.plo;
      c += (uint32_t)((pool[t.pword + (dd >> 6)] >> (dd & 63u)) & 1ull);
    }
  } else {
    const uint32_t lo = t.plo;
    const uint32_t hi = t.phi == UINT32_MAX ? next_lo : t.phi;
    const uint32_t m = hi - lo;
    if (m > 0 && m <= (uint32_t)L2_CAP && m <= L2_STAGE_RATIO * t.dcount) {
      wave_stage(stage, pk + lo, m, lane);
      wave_lds_sync();
      c = count_members<NIT>(stage, m, x, v, nit);
      wave_lds_sync();
    } else if (m > 0) {
      // A large range: bisect the line samples inside it (staged in LDS
      // when they fit), then search the one line that can hold x.
      // Samples j in [jf, jl] start lines inside [lo, hi); keys before
      // the first of them belong to the range's first, partial line.
      const uint32_t* sp = t.drv ? a.samp[0] : a.samp[1];
      const uint32_t jf = (lo + (1u << LINE_SHIFT) - 1) >> LINE_SHIFT;
      const uint32_t jl = (hi - 1) >> LINE_SHIFT;
      uint32_t k[NIT];
#pragma unroll
      for (int it = 0; it < NIT; it++) k[it] = 0;
      if (jl >= jf) {
        const uint32_t ns = jl - jf + 1;
        if (ns <= (uint32_t)L2_CAP) {
          wave_stage(stage, sp + jf, ns, lane);
          wave_lds_sync();
          count_le<NIT>(stage, ns, x, nit, k);
          wave_lds_sync();
        } else {
          count_le<NIT>(sp + jf, ns, x, nit, k);
        }
      }
      uint32_t pos[NIT], len[NIT];
#pragma unroll
      for (int it = 0; it < NIT; it++) {
        const uint32_t sb = k[it] ? (jf + k[it] - 1) << LINE_SHIFT : lo;
        const uint32_t se = (uint32_t)min<uint64_t>(hi, (uint64_t)(jf + k[it]) << LINE_SHIFT);
        pos[it] = sb;
        len[it] = se > sb ? se - sb : 0;
      }
#pragma unroll
      for (int step = 0; step < (int)LINE_SHIFT; step++)
#pragma unroll
        for (int it = 0; it < NIT; it++)
          if (it < (int)nit && len[it] > 1) {
            const uint32_t half = len[it] >> 1;
            pos[it] = (pk[pos[it] + half] <= x[it]) ? pos[it] + half : pos[it];
            len[it] -= half;
          }
#pragma unroll
      for (int it = 0; it < NIT; it++)
        if (it < (int)nit) c += (v[it] && len[it] > 0 && pk[pos[it]] == x[it]) ? 1u : 0u;
    }
  }
  return c;
}

typedef const UnitDesc __attribute__((address_space(4)))* CDesc;

__device__ __forceinline__ UnitDesc load_desc(CDesc d, uint64_t u) {
  UnitDesc t;
  t.dstart = d[u].dstart;
  t.dcount = d[u].dcount;
  t.plo = d[u].plo;
  t.phi = d[u].phi;
  t.pword = d[u].pword;
  t.drv = d[u].drv;
  t.top = d[u].top;
  return t;
}

// LIST = false runs every unit but those of the top bucket (NIT = NIT);
// LIST = true runs the top bucket's units, listed in a.list (NIT = TOP_IT).
template <bool LIST, int NIT>
__global__ __launch_bounds__(J_NT) void k_leaf2_count(Leaf2Args a) {
  __shared__ uint32_t s_stage[J_NW][L2_CAP];
  __shared__ unsigned long long s_cnt;
  // w is uniform across the wave: unit indices and descriptors then live in
  // scalar registers and descriptors come through the scalar cache, whose
  // loads are counted apart from the vector loads of the keys
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid / WAVE), lane = lane_id();
  if (tid == 0) s_cnt = 0;
  uint32_t* stage = s_stage[w];
  uint64_t run = 0;  // ungrouped: this lane's part of the block's count
  // The next unit's descriptor is loaded while the current unit is worked
  // on, so its latency overlaps the current unit's key loads.
  // descriptors are read-only here: read through the constant address space
  const CDesc desc = (CDesc)a.desc;
  auto unit_of = [&](uint64_t i) -> uint64_t { return LIST ? (uint64_t)a.list[i] : i; };
  UnitDesc nt{};
  uint64_t nu = 0;
  uint32_t nlo = 0;
  const uint64_t vb0 = xcd_block(blockIdx.x, gridDim.x);
  if (vb0 < a.nvblk && vb0 * J_NW + w < a.units) {
    nu = unit_of(vb0 * J_NW + w);
    nt = load_desc(desc, nu);
    nlo = (nu + 1 < a.n_desc) ? desc[nu + 1].plo : 0u;
  }
  for (uint64_t vb = vb0; vb < a.nvblk; vb += gridDim.x) {
    const uint64_t i = vb * J_NW + w;
    const uint64_t u = nu;
    const UnitDesc t = nt;
    const uint32_t next_lo = nlo;
    const uint64_t in = (vb + gridDim.x) * J_NW + w;
    if (vb + gridDim.x < a.nvblk && in < a.units) {
      nu = unit_of(in);
      nt = load_desc(desc, nu);
      nlo = (nu + 1 < a.n_desc) ? desc[nu + 1].plo : 0u;
    }
    if (i >= a.units) continue;      // wave-uniform; no barrier inside the loop
    if (!LIST && t.top) continue;    // the top bucket's own launch runs it
    uint32_t c = 0;
    if (t.drv == DRV_AND) {
      const uint64_t w0 = (uint64_t)t.plo | ((uint64_t)t.phi << 32);
#pragma unroll
      for (int it = 0; it < NIT; it++) {
        const uint32_t k = it * WAVE + lane;
        if (k < t.dcount) c += (uint32_t)__popcll(a.pool[0][w0 + k] & a.pool[1][t.pword + k]);
      }
    } else {
      c = probe_unit<NIT>(a, t, next_lo, stage, lane);
    }
    if (a.ucnt) {
      // grouped: one count per unit; groups are summed by a scan afterwards
      const uint64_t sc = wave_sum((uint64_t)c);
      if (lane == 0) a.ucnt[u] = sc;
    } else {
      run += c;
    }
  }
  if (!a.ucnt) {
    __syncthreads();
    const uint64_t sc = wave_sum(run);
    if (lane == 0 && sc) atomicAdd(&s_cnt, (unsigned long long)sc);
    __syncthreads();
    if (tid == 0 && s_cnt) atomicAdd((unsigned long long*)&a.gcount[0], s_cnt);
  }
}

// A merge tile, listed in launch order: keys [a0, a0 + na) of participant
// 0 and [b0, b0 + nb) of participant 1; back = 1 when keys[0][a0 - 1] is
// in the row (the tile's look-back element, lb); unit = the unit it belongs
// to; [lo, hi] = the smallest and largest of the tile's keys and lb
// (lo > hi: the tile holds no key).
struct MergeTile {
  uint32_t a0, na, b0, nb, back, unit, lo, hi, lb, pad[7];
};
constexpr int MT_WORDS = sizeof(MergeTile) / 4;
static_assert(MT_WORDS == 16, "a merge tile is read as 16 words, one per lane");

__global__ void k_merge_tiles(const UnitDesc* desc, const uint32_t* list, const uint32_t* k0, const uint32_t* k1,
                              uint64_t n, MergeTile* out) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = list[j];
    const UnitDesc t = desc[u];
    MergeTile m{};
    m.a0 = t.dstart;
    m.na = t.dcount;
    m.b0 = t.plo;
    m.nb = t.phi;
    m.back = (uint32_t)t.pword;
    m.unit = u;
    uint32_t lo = UINT32_MAX, hi = 0;
    if (m.back) {
      m.lb = k0[m.a0 - 1];
      lo = min(lo, m.lb);
      hi = max(hi, m.lb);
    }
    if (m.na) {
      lo = min(lo, k0[m.a0]);
      hi = max(hi, k0[m.a0 + m.na - 1]);
    }
    if (m.nb) {
      lo = min(lo, k1[m.b0]);
      hi = max(hi, k1[m.b0 + m.nb - 1]);
    }
    if (lo > hi) {
      lo = 1;
      hi = 0;
    }
    m.lo = lo;
    m.hi = hi;
    out[j] = m;
  }
}

// 16-byte chunks of keys per thread per tile: the two runs' chunks on the
// 16-byte grid, partial chunks at the ends included (at most
// MERGE_TILE / 4 + 4 of them).
constexpr int M_CH = (int)((MERGE_TILE / 4 + 4 + M_NT - 1) / M_NT);

// Bitmap word of the value offset d: words are XOR-swizzled within groups
// of 32 so that lanes whose values lie 32 words apart (sparse sets) hit
// different banks.
__device__ __forceinline__ uint32_t bm_word(uint32_t d) {
  const uint32_t w = d >> 5;
  return w ^ ((w >> 5) & 31u);
}

// Merge tiles: each block runs one contiguous range of the tile list (the
// ranges of an XCD's blocks are contiguous too, so tiles of one row share
// an L2).  A tile's two runs are loaded as 16-byte chunks, coalesced, and
// the next tile's chunks are loaded while the current one is counted.
// Participant 0's keys of the tile (and its look-back element: a common
// value split across two tiles has its set-0 copy at the end of one and its
// set-1 copy at the start of the next) set bits of an LDS bitmap over the
// tile's value span, one atomic OR per bitmap word a chunk touches; every
// participant-1 key then tests its bit.  The loads, bit sets and tests are
// independent of each other.  A sparser tile is merged instead: its keys
// are staged in LDS, thread k finds merged position k * M_PER (a merge-path
// search) and walks M_PER positions, counting set-1 keys equal to their
// merged set-0 predecessor.
__global__ __launch_bounds__(M_NT) void k_leaf2_merge(Leaf2Args a, const MergeTile* tiles, uint64_t n_tiles) {
  __shared__ __align__(16) uint32_t s_t[MERGE_TILE + 4];
  __shared__ uint64_t s_red[M_NT / WAVE];
  const int tid = threadIdx.x, lane = lane_id();
  const uint64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t per = (n_tiles + gridDim.x - 1) / gridDim.x;
  const uint64_t k0 = lb * per, k1 = min<uint64_t>(n_tiles, k0 + per);
  if (k0 >= k1) return;  // block-uniform, before any barrier
  uint64_t run = 0;
  uint4 r[M_CH], rn[M_CH];
  auto tile_word = [&](uint64_t k) -> uint32_t {
    return (k < k1 && lane < MT_WORDS) ? reinterpret_cast<const uint32_t*>(tiles + k)[lane] : 0u;
  };
  auto unpack = [&](uint32_t w) -> MergeTile {
    MergeTile m{};
    m.a0 = __builtin_amdgcn_readlane(w, 0);
    m.na = __builtin_amdgcn_readlane(w, 1);
    m.b0 = __builtin_amdgcn_readlane(w, 2);
    m.nb = __builtin_amdgcn_readlane(w, 3);
    m.back = __builtin_amdgcn_readlane(w, 4);
    m.unit = __builtin_amdgcn_readlane(w, 5);
    m.lo = __builtin_amdgcn_readlane(w, 6);
    m.hi = __builtin_amdgcn_readlane(w, 7);
    m.lb = __builtin_amdgcn_readlane(w, 8);
    return m;
  };
  // chunk j * M_NT + tid of the tile: set 0's run first, then set 1's
  auto fetch = [&](const MergeTile& m, uint4* x) {
    const KeyRun A = key_run(a.keys[0] + m.a0, m.na), B = key_run(a.keys[1] + m.b0, m.nb);
#pragma unroll
    for (int j = 0; j < M_CH; j++) {
      const uint32_t c = (uint32_t)j * M_NT + (uint32_t)tid;
      x[j] = c < A.nch ? load_chunk(A, c) : c < A.nch + B.nch ? load_chunk(B, c - A.nch) : make_uint4(0, 0, 0, 0);
    }
  };
  MergeTile t = unpack(tile_word(k0));
  fetch(t, r);
  uint32_t wnext = tile_word(k0 + 1);
  for (uint64_t k = k0; k < k1; k++) {
    const MergeTile cur = t;
    // the next tile's keys are in flight while this one is counted
    if (k + 1 < k1) {
      t = unpack(wnext);
      fetch(t, rn);
      wnext = tile_word(k + 2);
    }
    const KeyRun A = key_run(a.keys[0] + cur.a0, cur.na), B = key_run(a.keys[1] + cur.b0, cur.nb);
    const uint32_t na = cur.na, nb = cur.nb, n1 = na + 1, n = na + nb;
    const uint64_t span = cur.lo <= cur.hi ? (uint64_t)(cur.hi - cur.lo) + 1 : 0;
    const bool bitmap = span <= MERGE_BM_SPAN && span <= MERGE_BM_SPREAD * (n + 1);  // block-uniform
    uint32_t c = 0;
    __syncthreads();  // the previous tile's readers are done
    if (bitmap) {
      const uint32_t nw = (uint32_t)((span + 31) >> 5);
      // the swizzle permutes words within groups of 32: clear whole groups
      const uint32_t nz = (nw + 31) & ~31u;
      for (uint32_t i = 4 * (uint32_t)tid; i < nz; i += 4 * M_NT)
        *reinterpret_cast<uint4*>(&s_t[i]) = make_uint4(0u, 0u, 0u, 0u);
      __syncthreads();
      if (tid == 0 && cur.back) {
        const uint32_t d = cur.lb - cur.lo;
        atomicOr(&s_t[bm_word(d)], 1u << (d & 31u));
      }
#pragma unroll
      for (int j = 0; j < M_CH; j++) {
        const uint32_t ch = (uint32_t)j * M_NT + (uint32_t)tid;
        if (ch >= A.nch) continue;
        // the chunk's bits, one atomic per word they fall in
        uint32_t cw = UINT32_MAX, bits = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int64_t i = 4 * (int64_t)ch - A.head + e;
          if (i < 0 || i >= (int64_t)na) continue;
          const uint32_t d = chunk_elem(r[j], e) - cur.lo;
          const uint32_t w = bm_word(d);
          if (w != cw) {
            if (bits) atomicOr(&s_t[cw], bits);
            cw = w;
            bits = 0;
          }
          bits |= 1u << (d & 31u);
        }
        if (bits) atomicOr(&s_t[cw], bits);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < M_CH; j++) {
        const uint32_t ch = (uint32_t)j * M_NT + (uint32_t)tid;
        if (ch < A.nch || ch >= A.nch + B.nch) continue;
        const uint32_t cb = ch - A.nch;
        uint32_t cw = UINT32_MAX, word = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int64_t i = 4 * (int64_t)cb - B.head + e;
          if (i < 0 || i >= (int64_t)nb) continue;
          const uint32_t d = chunk_elem(r[j], e) - cur.lo;
          const uint32_t w = bm_word(d);
          if (w != cw) {
            cw = w;
            word = s_t[w];
          }
          c += (word >> (d & 31u)) & 1u;
        }
      }
    } else {
      // stage: slot 0 the look-back element, set 0's run at 1.., set 1's at n1..
      if (tid == 0) s_t[0] = cur.back ? cur.lb : 0u;
#pragma unroll
      for (int j = 0; j < M_CH; j++) {
        const uint32_t ch = (uint32_t)j * M_NT + (uint32_t)tid;
        const bool in_a = ch < A.nch;
        if (!in_a && ch >= A.nch + B.nch) continue;
        const uint32_t head = in_a ? A.head : B.head, len = in_a ? na : nb;
        const uint32_t cc = in_a ? ch : ch - A.nch;
        const uint32_t base = in_a ? 1u : n1;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int64_t i = 4 * (int64_t)cc - head + e;
          if (i >= 0 && i < (int64_t)len) s_t[base + (uint32_t)i] = chunk_elem(r[j], e);
        }
      }
      __syncthreads();
      const uint32_t d = (uint32_t)tid * M_PER;
      if (d < n) {
        uint32_t lo = d > nb ? d - nb : 0u, hi = min(d, na);
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_t[1 + mid] <= s_t[n1 + d - mid - 1]) lo = mid + 1; else hi = mid;
        }
        uint32_t ia = lo, jb = d - lo;
        bool have = ia > 0 || cur.back != 0;
        uint32_t prev = s_t[ia];  // set 0's element before position ia (slot 0: the look-back)
        uint32_t av = ia < na ? s_t[1 + ia] : 0u;
        uint32_t bv = jb < nb ? s_t[n1 + jb] : 0u;
        const uint32_t end = min(d + (uint32_t)M_PER, n);
        for (uint32_t q = d; q < end; q++) {
          if (ia < na && (jb >= nb || av <= bv)) {
            prev = av;
            have = true;
            ia++;
            av = ia < na ? s_t[1 + ia] : 0u;
          } else {
            c += (have && prev == bv) ? 1u : 0u;
            jb++;
            bv = jb < nb ? s_t[n1 + jb] : 0u;
          }
        }
      }
    }
    const uint64_t sc = block_sum<uint64_t, M_NT>((uint64_t)c, s_red);
    if (a.ucnt) {
      if (tid == 0) a.ucnt[cur.unit] = sc;
    } else {
      run += sc;
    }
#pragma unroll
    for (int j = 0; j < M_CH; j++) r[j] = rn[j];
  }
  if (!a.ucnt && tid == 0 && run) atomicAdd((unsigned long long*)&a.gcount[0], (unsigned long long)run);
}

// ---- finalization ------------------------------------------------------------

__global__ void k_nonzero_flags(const uint64_t* cnt, uint64_t n, uint32_t* flags) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    flags[i] = cnt[i] != 0 ? 1u : 0u;
}

__global__ void k_tag_flags(const uint32_t* tag, uint64_t n, uint32_t* flags) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    flags[i] = tag[i] == SLOT_READY ? 1u : 0u;
}

__global__ void k_key64_flags(const uint64_t* key, uint64_t n, uint32_t* flags) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    flags[i] = key[i] != KEY64_EMPTY ? 1u : 0u;
}

struct UnpackArgs {
  const uint64_t* key;
  const uint32_t* sid;
  uint32_t n_cols;
  uint32_t shift[MAXV + MAXA];
  uint32_t bits[MAXV + MAXA];
  uint32_t* out[MAXV + MAXA];
};

__global__ void k_unpack_keys(UnpackArgs a, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = a.key[a.sid[i]];
    for (uint32_t c = 0; c < a.n_cols; c++)
      a.out[c][i] = a.bits[c] ? (uint32_t)((k >> a.shift[c]) & ((1ull << a.bits[c]) - 1)) : 0u;
  }
}

struct GroupFin {
  const uint64_t* cnt;
  const int64_t* acc;       // stride D
  const uint64_t* off;      // dense: exclusive scan of the non-empty flags
  const uint32_t* sid;      // hash: table slot of each group
  const uint32_t* perm;     // hash: groups in key order
  uint32_t n_cols;
  const uint32_t* key_in[MAXV + MAXA];  // hash: keys of each group (sid order)
  uint64_t radix[MAXV + MAXA];          // dense: mixed radix of the index
  uint32_t* key_out[MAXV + MAXA];
  uint64_t* count_out;
  double* sum_out;
  double* parts;            // exact parts of each sum (EXACT_PARTS per row), or null
  uint32_t sum;
  int32_t lsb;
  uint32_t D;
  uint32_t* err;
};

// Dense GROUP BY: a non-empty index becomes the next output row; its keys
// are the digits of the index, so rows come out in key order.
__global__ void k_dense_finalize(GroupFin f, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    if (f.off[i + 1] == f.off[i]) continue;
    const uint64_t o = f.off[i];
    uint64_t idx = i;
    for (int c = (int)f.n_cols - 1; c >= 0; c--) {
      f.key_out[c][o] = (uint32_t)(idx % f.radix[c]);
      idx /= f.radix[c];
    }
    f.count_out[o] = f.cnt[i];
    if (f.sum) f.sum_out[o] = exact_round(f.acc + i * f.D, f.D, f.lsb, f.err);
    if (f.parts) exact_parts(f.acc + i * f.D, f.D, f.lsb, f.parts + o * EXACT_PARTS, f.err);
  }
}

// Hash GROUP BY: output row i is the i-th group in key order.
__global__ void k_hash_finalize(GroupFin f, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = f.perm[i];
    const uint64_t slot = f.sid[j];
    for (uint32_t c = 0; c < f.n_cols; c++) f.key_out[c][i] = f.key_in[c][j];
    f.count_out[i] = f.cnt[slot];
    if (f.sum) f.sum_out[i] = exact_round(f.acc + slot * f.D, f.D, f.lsb, f.err);
    if (f.parts) exact_parts(f.acc + slot * f.D, f.D, f.lsb, f.parts + i * EXACT_PARTS, f.err);
  }
}

struct FinA {
  const uint64_t* gcount;
  const int64_t* gacc;
  const uint64_t* off;      // exclusive scan of nonzero flags (null: keep all)
  uint32_t n_cols;
  const uint32_t* key_in[MAXV];
  uint32_t* key_out[MAXV];
  uint64_t* count_out;
  double* sum_out;
  double* parts;            // exact parts of each sum (EXACT_PARTS per row), or null
  uint32_t sum;
  int32_t lsb;
  uint32_t D;
  uint32_t* err;
};

__global__ void k_finalize_groups(FinA f, uint64_t n) {
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t o = g;
    if (f.off) {
      if (f.off[g + 1] == f.off[g]) continue;
      o = f.off[g];
    }
    for (uint32_t c = 0; c < f.n_cols; c++) f.key_out[c][o] = f.key_in[c][g];
    f.count_out[o] = f.gcount[g];
    if (f.sum) f.sum_out[o] = exact_round(f.gacc + g * EXACT_MAXD, f.D, f.lsb, f.err);
    if (f.parts) exact_parts(f.gacc + g * EXACT_MAXD, f.D, f.lsb, f.parts + o * EXACT_PARTS, f.err);
  }
}

struct ColsArg {
  const uint32_t* c[MAXV + MAXA];
  uint32_t n;
};

__global__ void k_seg_heads(ColsArg cols, const uint32_t* perm, uint64_t n, uint32_t* head) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t h = (i == 0);
    if (!h) {
      uint32_t p = perm[i], q = perm[i - 1];
      for (uint32_t c = 0; c < cols.n && !h; c++) h = cols.c[c][p] != cols.c[c][q];
    }
    head[i] = h;
  }
}

struct SegAccArgs {
  ColsArg cols;
  const uint32_t* perm;
  const uint64_t* segoff;   // exclusive scan of heads: segment of i = segoff[i+1]-1
  const uint64_t* mult;
  const double* hi;
  const double* lo;
  uint32_t sum;
  int32_t lsb;
  uint32_t D;
  uint64_t* gcount;
  int64_t* gacc;
  uint32_t* key_out[MAXV + MAXA];
  uint32_t* err;
};

__global__ void k_seg_accumulate(SegAccArgs a, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t g = a.segoff[i + 1] - 1;
    const uint32_t p = a.perm[i];
    if (a.segoff[i + 1] != a.segoff[i])
      for (uint32_t c = 0; c < a.cols.n; c++) a.key_out[c][g] = a.cols.c[c][p];
    atomic_add_count(&a.gcount[g], a.mult[p], a.err);
    if (a.sum) {
      int64_t* dig = a.gacc + g * EXACT_MAXD;
      bool ok = atomic_add_term(dig, a.hi[p], a.lsb, a.D, a.mult[p]);
      ok = atomic_add_term(dig, a.lo[p], a.lsb, a.D, a.mult[p]) && ok;
      if (!ok) atomicOr(a.err, 1u);
    }
  }
}

// A dispatch counts work-items in 32 bits: cap the grid and let blocks
// stride over virtual blocks.
unsigned elem_grid(uint64_t nvblk) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nvblk, 32768)); }
// The merge launch: as many blocks as fit on the device at once; each loops
// over a contiguous range of tiles, loading the next while counting one.
unsigned merge_grid() {
  int dev = 0, cus = 256, per = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_leaf2_merge, M_NT, 0) != hipSuccess) per = 1;
  return (unsigned)std::max(1, cus * std::max(1, per));
}
// The two-set leaf walks its virtual blocks with more workgroups in flight
// than the frontier kernels: 131072 (512 per CU) measured 6% faster than
// 32768 on R-MAT-22 triangles, while larger grids lose again.
unsigned leaf_grid(uint64_t nvblk) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nvblk, 131072)); }

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 256 * 64));
}

uint32_t bitlen(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

// ---- host-side frontier --------------------------------------------------------

struct Frontier {
  uint64_t n = 1;                           // starts as the single empty binding
  std::vector<DBuf<uint32_t>> pos;          // per atom (empty: no bound attribute)
  std::vector<DBuf<uint32_t>> outv;         // per output column (empty: not bound yet)
  DBuf<uint32_t> gid;
};

DSet make_dset(const lh_plan_t* p, const Participant& pt, const Frontier& F) {
  const lh_trie* t = p->atoms[pt.atom].trie;
  const Level& L = t->lv[pt.level];
  DSet d{};
  d.keys = L.keys.p;
  d.samp = L.samp.p;
  d.bs_word = L.bs_word.p;
  d.bs_base = L.bs_base.p;
  d.pool = L.pool.p;
  d.bs_rank = L.bs_rank.p;
  d.bs_delta = L.bs_delta.p;
  if (pt.level == 0) {
    d.root_n = (uint32_t)t->lv[0].n;
    d.root_bits = t->root_bits.p;
    d.root_rank = t->root_rank.p;
    d.root_span = t->root_span;
  } else {
    d.ppos = F.pos[pt.atom].p;
    d.poffs = t->lv[pt.level - 1].offs.p;
  }
  return d;
}

// Per-row work (smallest participating set), its exclusive scan, and the
// cut of every row into work units of U_EL elements.
struct DepthWork {
  DBuf<uint64_t> W, U;
  DBuf<uint64_t> n_top;     // two-set leaves: units of the top bucket, then of merged rows (device)
  DBuf<uint8_t> drv;
  DBuf<uint32_t> urow;
  uint64_t total = 0, units = 0, nblk = 0;
};

void depth_work(const lh_plan_t* p, uint32_t d, const Frontier& F, ElemArgs& a, DepthWork& dw, hipStream_t s,
                bool leaf2 = false) {
  const auto& parts = p->parts[d];
  WorkArgs wa{};
  wa.np = (uint32_t)parts.size();
  a.np = wa.np;
  for (uint32_t i = 0; i < wa.np; i++) {
    wa.set[i] = make_dset(p, parts[i], F);
    a.set[i] = wa.set[i];
  }
  DBuf<uint32_t> work(F.n, s), units(F.n, s);
  dw.drv.alloc(F.n, s);
  dw.W.alloc(F.n + 1, s);
  dw.U.alloc(F.n + 1, s);
  {
    ProfScope ps("join_work", s, F.n, 0);
    if (leaf2) {
      dw.n_top.alloc(2, s);
      fill_u64(dw.n_top.p, 0, 2, s);
    }
    k_work<<<grid_for(F.n), 256, 0, s>>>(wa, F.n, work.p, dw.drv.p, units.p, leaf2 ? 1u : 0u,
                                         leaf2 ? (unsigned long long*)dw.n_top.p : nullptr);
  }
  LH_HIP(hipGetLastError());
  dw.total = scan_u32_to_u64(work.p, dw.W.p, F.n, s);
  dw.units = scan_u32_to_u64(units.p, dw.U.p, F.n, s);
  if (dw.units >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "join: more than 2^32 work units at one attribute");
  dw.urow.alloc(dw.units, s);
  if (dw.units) {
    // rows with more than UROW_SMALL units number at most units / UROW_SMALL
    DBuf<uint32_t> big(std::max<uint64_t>(1, std::min<uint64_t>(F.n, dw.units / UROW_SMALL)), s), nbig(1, s);
    fill_u32(nbig.p, 0u, 1, s);
    k_unit_rows<<<grid_for(F.n), 256, 0, s>>>(dw.U.p, F.n, dw.urow.p, big.p, nbig.p);
    LH_HIP(hipGetLastError());
    k_unit_rows_big<<<1024, 256, 0, s>>>(dw.U.p, big.p, nbig.p, dw.urow.p);
    LH_HIP(hipGetLastError());
  }
  dw.nblk = (dw.units + J_NW - 1) / J_NW;
  a.nvblk = dw.nblk;
  a.W = dw.W.p;
  a.drv = dw.drv.p;
  a.nrows = F.n;
  a.total = dw.total;
  a.U = dw.U.p;
  a.urow = dw.urow.p;
  a.total_units = dw.units;
}

bool binds_by(const lh_plan_t* p, uint32_t atom, uint32_t d) {
  const PlanAtom& A = p->atoms[atom];
  for (uint32_t l = 0; l < A.n_levels; l++)
    if (p->depth_of[A.attr_of_level[l]] <= d) return true;
  return false;
}

void step(const lh_plan_t* p, uint32_t d, Frontier& F, hipStream_t s) {
  ElemArgs a{};
  DepthWork dw;
  depth_work(p, d, F, a, dw, s);
  const uint64_t total = dw.total;
  if (total == 0) {
    F.n = 0;
    return;
  }
  const uint64_t nblk = dw.nblk;
  if (nblk >= (1ull << 31)) fail(LH_ERR_OVERFLOW, "join: too much work at one attribute");
  DBuf<uint32_t> bcnt(nblk, s);
  a.blk_cnt = bcnt.p;
  a.need_pos_mask = 0;
  {
    static const char* names[MAXV] = {"join_count_d0", "join_count_d1", "join_count_d2", "join_count_d3",
                                      "join_count_d4", "join_count_d5", "join_count_d6", "join_count_d7",
                                      "join_count_d8", "join_count_d9", "join_count_d10", "join_count_d11",
                                      "join_count_d12", "join_count_d13", "join_count_d14", "join_count_d15"};
    ProfScope ps(names[d], s, F.n, total);
    launch_elem<M_COUNT>(a, elem_grid(nblk), s);
  }
  LH_HIP(hipGetLastError());
  DBuf<uint64_t> boff(nblk + 1, s);
  const uint64_t n_new = scan_u32_to_u64(bcnt.p, boff.p, nblk, s);
  if (n_new >= (1ull << 32)) fail(LH_ERR_OVERFLOW, "join: frontier exceeds 2^32 rows");
  Frontier G;
  G.n = n_new;
  const uint32_t na = (uint32_t)p->atoms.size();
  G.pos.resize(na);
  a.n_atoms = na;
  for (uint32_t e = 0; e < na; e++) {
    a.part_of_atom[e] = -1;
    a.pos_in[e] = F.pos[e].p;
    if (binds_by(p, e, d)) {
      G.pos[e].alloc(n_new, s);
      a.pos_out[e] = G.pos[e].p;
    }
  }
  for (uint32_t i = 0; i < p->parts[d].size(); i++) a.part_of_atom[p->parts[d][i].atom] = (int32_t)i;
  const uint32_t no = (uint32_t)p->out_attrs.size();
  G.outv.resize(no);
  a.n_outv = no;
  a.new_outv = -1;
  for (uint32_t j = 0; j < no; j++) {
    a.outv_in[j] = F.outv[j].p;
    const uint32_t dj = p->depth_of[p->out_attrs[j]];
    if (dj <= d) {
      G.outv[j].alloc(n_new, s);
      a.outv_out[j] = G.outv[j].p;
      if (dj == d) a.new_outv = (int32_t)j;
    }
  }
  a.gid_mode = 0;
  if (p->case_prefix && no > 0) {
    if (d == no - 1) a.gid_mode = 2;
    else if (d > no - 1) a.gid_mode = 1;
  }
  if (a.gid_mode) {
    G.gid.alloc(n_new, s);
    a.gid_out = G.gid.p;
    a.gid_in = F.gid.p;
  }
  a.blk_off = boff.p;
  a.need_pos_mask = 0xffu;
  {
    static const char* names[MAXV] = {"join_fill_d0", "join_fill_d1", "join_fill_d2", "join_fill_d3",
                                      "join_fill_d4", "join_fill_d5", "join_fill_d6", "join_fill_d7",
                                      "join_fill_d8", "join_fill_d9", "join_fill_d10", "join_fill_d11",
                                      "join_fill_d12", "join_fill_d13", "join_fill_d14", "join_fill_d15"};
    ProfScope ps(names[d], s, F.n, total);
    launch_elem<M_FILL>(a, elem_grid(nblk), s);
  }
  LH_HIP(hipGetLastError());
  F = std::move(G);
}

}  // namespace

// GROUP BY outside the order's prefix, aggregated where the leaf finds the
// tuples (section 5): a dense array over the key space when the expected
// output is dense, else a device-wide hash table (open addressing, linear
// probing); either way no tuple is materialized.  Returns false when the
// sort-based path should run instead (asked for, or the table would not
// fit).
bool group_in_place(const lh_plan_t* p, const Frontier& F, ElemArgs& a, uint64_t nblk, uint64_t total,
                    uint32_t no, uint32_t n_cols, bool is_sum, uint32_t D, DBuf<uint32_t>& err,
                    lh_result_impl* res, hipStream_t s) {
  uint32_t impl = p->group_impl;
  if (impl == LH_GROUP_SORT >> 4) return false;
  const uint32_t leaf = p->n_attrs - 1;
  LeafArgs& L = a.leaf;
  // key space: the largest value of every output column
  std::vector<uint32_t> bits(n_cols);
  uint64_t space = 1;
  for (uint32_t c = 0; c < n_cols; c++) {
    uint32_t mx = 0;
    if (c < no) {
      const uint32_t attr = p->out_attrs[c];
      if (p->depth_of[attr] == leaf) {
        L.col_src[c] = -1;
        const Participant& P = p->parts[leaf][0];
        const Level& lv = p->atoms[P.atom].trie->lv[P.level];
        mx = lv.n ? reduce_max_u32(lv.keys.p, lv.n, s) : 0;
      } else {
        L.col_src[c] = (int32_t)c;
        mx = F.n ? reduce_max_u32(F.outv[c].p, F.n, s) : 0;
      }
    } else {
      L.col_src[c] = -2;
      const lh_group_col& G = p->groups[c - no];
      const lh_trie* T = p->atoms[G.atom].trie;
      mx = T->n_rows ? reduce_max_u32(T->meta[G.meta_col].p, T->n_rows, s) : 0;
    }
    L.radix[c] = (uint64_t)mx + 1;
    bits[c] = bitlen(mx);
    space = (space > (1ull << 62) / L.radix[c]) ? (1ull << 62) : space * L.radix[c];
  }
  const uint64_t dense_bytes = 8 + (is_sum ? 8ull * D : 0);
  const bool dense_fits = space <= (1ull << 27) && space * dense_bytes <= (2ull << 30);
  if (impl == 0) impl = (dense_fits && space <= std::max<uint64_t>(4 * total, 1u << 16)) ? 3 : 2;
  if (impl == 3 && !dense_fits) fail(LH_ERR_UNSUPPORTED, "join: the GROUP BY key space is too large for a dense array");
  const uint64_t hash_bytes = 4 + 4ull * n_cols + 8 + (is_sum ? 8ull * D : 0);  // an upper bound
  uint64_t cap = 1024;
  if (impl == 2) {
    const uint64_t want = 2 * std::min<uint64_t>(space, std::max<uint64_t>(total, 512));
    while (cap < want) cap <<= 1;
    if (cap > (1ull << 31) || cap * hash_bytes > (16ull << 30)) return false;
  }
  const uint64_t slots = impl == 3 ? space : cap;
  L.n_cols = n_cols;
  L.gmode = impl == 3 ? 1u : 2u;
  L.glds = (impl == 3 && space <= GLDS_MAX) ? 1u : 0u;
  L.gspace = (uint32_t)std::min<uint64_t>(space, GLDS_MAX);
  DBuf<uint64_t> cnt;
  DBuf<int64_t> acc;
  DBuf<uint32_t> tag;
  std::vector<DBuf<uint32_t>> tkeys;
  DBuf<uint64_t> key64;
  bool counted = false;
  // keys of at most 63 bits: one word per slot, column 0 most significant
  uint32_t key_bits = 0;
  for (uint32_t c = 0; c < n_cols; c++) key_bits += bits[c];
  const bool packed = key_bits <= 63;
  L.gkey64 = nullptr;
  if (packed) {
    uint32_t sh = key_bits;
    for (uint32_t c = 0; c < n_cols; c++) {
      sh -= bits[c];
      L.gshift[c] = sh;
    }
  }
  for (;;) {
    const uint64_t n = impl == 3 ? space : cap;
    cnt.alloc(n, s);
    acc.alloc(is_sum ? n * D : 0, s);
    LH_HIP(hipMemsetAsync(cnt.p, 0, n * sizeof(uint64_t), s));
    if (is_sum) LH_HIP(hipMemsetAsync(acc.p, 0, n * D * sizeof(int64_t), s));
    L.gcount = cnt.p;
    L.gacc = acc.p;
    if (impl == 2 && packed) {
      key64.alloc(n, s);
      LH_HIP(hipMemsetAsync(key64.p, 0xff, n * sizeof(uint64_t), s));
      L.gkey64 = key64.p;
      L.gmask = n - 1;
    } else if (impl == 2) {
      tag.alloc(n, s);
      LH_HIP(hipMemsetAsync(tag.p, 0, n * sizeof(uint32_t), s));
      tkeys.clear();
      for (uint32_t c = 0; c < n_cols; c++) {
        tkeys.emplace_back(n, s);
        L.col_out[c] = tkeys.back().p;
      }
      L.gtag = tag.p;
      L.gmask = n - 1;
    }
    if (total) {
      ProfScope ps(impl == 3 ? "leaf_group_dense" : "leaf_group_hash", s, F.n, total);
      launch_elem<M_LEAF_B_AGG>(a, elem_grid(nblk), s);
      LH_HIP(hipGetLastError());
    }
    const uint32_t e = read_scalar(err.p, s);
    if (e & ERR_SLOT_SPIN) fail(LH_ERR_DEVICE, "join: a GROUP BY hash slot was never published");
    if (impl == 2 && (e & ERR_TABLE_FULL)) {
      // more groups than the estimate: count the tuples exactly once and
      // size the table for them (later overflows double it), from scratch
      fill_u32(err.p, 0, 1, s);
      uint64_t want = 2 * cap;
      if (!counted) {
        counted = true;
        DBuf<uint32_t> bcnt(nblk, s);
        DBuf<uint64_t> boff(nblk + 1, s);
        a.blk_cnt = bcnt.p;
        {
          ProfScope ps("leaf_emit_count", s, F.n, total);
          launch_elem<M_LEAF_B_COUNT>(a, elem_grid(nblk), s);
        }
        LH_HIP(hipGetLastError());
        const uint64_t n_emit = scan_u32_to_u64(bcnt.p, boff.p, nblk, s);
        want = std::max(want, 2 * std::min<uint64_t>(space, n_emit));
      }
      while (cap < want) cap <<= 1;
      if (cap > (1ull << 31) || cap * hash_bytes > (16ull << 30)) return false;
      continue;
    }
    break;
  }
  (void)slots;
  GroupFin f{};
  f.cnt = cnt.p;
  f.acc = acc.p;
  f.n_cols = n_cols;
  f.sum = is_sum ? 1u : 0u;
  f.lsb = L.lsb;
  f.D = D;
  f.err = err.p;
  uint64_t n_groups = 0;
  lh_result& R = res->pub;
  if (impl == 3) {
    DBuf<uint32_t> flags(space, s);
    DBuf<uint64_t> off(space + 1, s);
    k_nonzero_flags<<<grid_for(space), 256, 0, s>>>(cnt.p, space, flags.p);
    LH_HIP(hipGetLastError());
    n_groups = scan_u32_to_u64(flags.p, off.p, space, s);
    res->cols.resize(n_cols);
    for (uint32_t c = 0; c < n_cols; c++) {
      res->cols[c].alloc(n_groups, s);
      f.key_out[c] = res->cols[c].p;
      f.radix[c] = L.radix[c];
    }
    res->counts.alloc(n_groups, s);
    if (is_sum) res->sums.alloc(n_groups, s);
    if (is_sum && p->want_parts) res->parts.alloc(n_groups * EXACT_PARTS, s);
    f.count_out = res->counts.p;
    f.sum_out = res->sums.p;
    f.parts = res->parts.p;
    f.off = off.p;
    if (n_groups) {
      k_dense_finalize<<<grid_for(space), 256, 0, s>>>(f, space);
      LH_HIP(hipGetLastError());
    }
    R.group_impl = 3;
  } else {
    DBuf<uint32_t> flags(cap, s), sid(cap, s);
    if (packed) k_key64_flags<<<grid_for(cap), 256, 0, s>>>(key64.p, cap, flags.p);
    else k_tag_flags<<<grid_for(cap), 256, 0, s>>>(tag.p, cap, flags.p);
    LH_HIP(hipGetLastError());
    n_groups = select_flagged(flags.p, cap, sid.p, s);
    std::vector<DBuf<uint32_t>> gk(n_cols);
    std::vector<const uint32_t*> gp(n_cols);
    UnpackArgs ua{};
    ua.key = key64.p;
    ua.sid = sid.p;
    ua.n_cols = n_cols;
    for (uint32_t c = 0; c < n_cols; c++) {
      gk[c].alloc(n_groups, s);
      if (n_groups && !packed) gather_u32(tkeys[c].p, sid.p, gk[c].p, n_groups, s);
      gp[c] = gk[c].p;
      f.key_in[c] = gk[c].p;
      ua.shift[c] = L.gshift[c];
      ua.bits[c] = bits[c];
      ua.out[c] = gk[c].p;
    }
    if (n_groups && packed) {
      k_unpack_keys<<<grid_for(n_groups), 256, 0, s>>>(ua, n_groups);
      LH_HIP(hipGetLastError());
    }
    DBuf<uint32_t> perm(n_groups, s);
    if (n_groups) lex_sort_perm(gp.data(), bits.data(), n_cols, n_groups, perm.p, s);
    res->cols.resize(n_cols);
    for (uint32_t c = 0; c < n_cols; c++) {
      res->cols[c].alloc(n_groups, s);
      f.key_out[c] = res->cols[c].p;
    }
    res->counts.alloc(n_groups, s);
    if (is_sum) res->sums.alloc(n_groups, s);
    if (is_sum && p->want_parts) res->parts.alloc(n_groups * EXACT_PARTS, s);
    f.count_out = res->counts.p;
    f.sum_out = res->sums.p;
    f.parts = res->parts.p;
    f.sid = sid.p;
    f.perm = perm.p;
    if (n_groups) {
      k_hash_finalize<<<grid_for(n_groups), 256, 0, s>>>(f, n_groups);
      LH_HIP(hipGetLastError());
    }
    R.group_impl = 2;
  }
  R.n_rows = n_groups;
  return true;
}

// ---- materialized joins -----------------------------------------------------------

struct FullArgs {
  const uint32_t* pos[MAXA];  // each atom's position in its last level
  const uint32_t* run[MAXA];  // bag atoms: run offsets of the last level; else null
  uint32_t na;
  uint64_t* counts;
};

__global__ void k_gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}

// Rows a tuple stands for: the product over bag atoms of its run length.
__global__ void k_full_counts(FullArgs a, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t c = 1;
#pragma unroll
    for (int e = 0; e < MAXA; e++)
      if (e < (int)a.na && a.run[e]) {
        const uint32_t q = a.pos[e][i];
        c *= (uint64_t)(a.run[e][q + 1] - a.run[e][q]);
      }
    a.counts[i] = c;
  }
}

// COUNT with every attribute an output (a materialized join) and no GROUP
// BY meta column: Algorithm 1 runs to the last attribute, whose frontier
// holds each distinct output tuple once, in the lexicographic order of the
// attribute order; a tuple's count is the product of its bag runs.  The
// rows are re-sorted only when the declared output order is another one.
lh_result_impl* run_full(const lh_plan_t* p, hipStream_t s) {
  std::unique_ptr<lh_result_impl> res(new lh_result_impl());
  memset(&res->pub, 0, sizeof(res->pub));
  const uint32_t na = (uint32_t)p->atoms.size();
  const uint32_t no = (uint32_t)p->out_attrs.size();
  Frontier F;
  F.pos.resize(na);
  F.outv.resize(no);
  for (uint32_t d = 0; d < p->n_attrs && F.n; d++) step(p, d, F, s);
  const uint64_t n = F.n;
  DBuf<uint64_t> cnt(n, s);
  if (n) {
    FullArgs fa{};
    fa.na = na;
    fa.counts = cnt.p;
    for (uint32_t e = 0; e < na; e++) {
      const PlanAtom& A = p->atoms[e];
      fa.pos[e] = F.pos[e].p;
      fa.run[e] = A.bag ? A.trie->lv[A.n_levels - 1].offs.p : nullptr;
    }
    k_full_counts<<<grid_for(n), 256, 0, s>>>(fa, n);
    LH_HIP(hipGetLastError());
  }
  bool in_order = true;
  for (uint32_t j = 0; j < no; j++) in_order = in_order && p->out_attrs[j] == p->order[j];
  res->cols.resize(no);
  if (in_order || n <= 1) {
    for (uint32_t j = 0; j < no; j++) res->cols[j] = std::move(F.outv[j]);
    res->counts = std::move(cnt);
  } else {
    std::vector<const uint32_t*> cptr(no);
    std::vector<uint32_t> bits(no);
    for (uint32_t j = 0; j < no; j++) {
      cptr[j] = F.outv[j].p;
      bits[j] = bitlen(reduce_max_u32(F.outv[j].p, n, s));
    }
    DBuf<uint32_t> perm(n, s);
    lex_sort_perm(cptr.data(), bits.data(), no, n, perm.p, s);
    for (uint32_t j = 0; j < no; j++) {
      res->cols[j].alloc(n, s);
      gather_u32(F.outv[j].p, perm.p, res->cols[j].p, n, s);
    }
    res->counts.alloc(n, s);
    k_gather_u64<<<grid_for(n), 256, 0, s>>>(cnt.p, perm.p, res->counts.p, n);
    LH_HIP(hipGetLastError());
  }
  lh_result& R = res->pub;
  R.n_rows = n;
  R.n_cols = no;
  R.exact = 0;
  R.group_impl = 0;
  res->colptr.resize(no);
  for (uint32_t j = 0; j < no; j++) res->colptr[j] = res->cols[j].p;
  R.out_keys = no ? res->colptr.data() : nullptr;
  R.counts = res->counts.p;
  R.sums = nullptr;
  uint64_t nj = 0;
  if (n) {
    DBuf<uint64_t> tmp(n + 1, s);
    nj = scan_u64(res->counts.p, tmp.p, n, s);
  }
  R.n_join_tuples = nj;
  LH_HIP(hipStreamSynchronize(s));
  return res.release();
}

lh_result_impl* run_plan(const lh_plan_t* p, hipStream_t s) {
  if (p->blas) return run_dense(p, s);
  if (p->case_full) return run_full(p, s);
  std::unique_ptr<lh_result_impl> res(new lh_result_impl());
  memset(&res->pub, 0, sizeof(res->pub));
  const uint32_t na = (uint32_t)p->atoms.size();
  const uint32_t no = (uint32_t)p->out_attrs.size();
  const uint32_t ngc = (uint32_t)p->groups.size();
  const uint32_t n_cols = no + ngc;
  const uint32_t leaf = p->n_attrs - 1;
  const bool is_sum = p->agg == LH_AGG_SUM;
  const uint32_t D = p->exact_digits;

  Frontier F;
  F.pos.resize(na);
  F.outv.resize(no);
  // keep the group-defining frontier's output columns (streamed groups)
  std::vector<DBuf<uint32_t>> group_keys;
  uint64_t n_groups = 1;
  for (uint32_t d = 0; d < leaf && F.n; d++) {
    step(p, d, F, s);
    if (p->case_prefix && no > 0 && d == no - 1) {
      n_groups = F.n;
      group_keys.clear();
      for (uint32_t j = 0; j < no; j++) {
        group_keys.emplace_back(F.n, s);
        if (F.n)
          LH_HIP(hipMemcpyAsync(group_keys.back().p, F.outv[j].p, F.n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      }
    }
  }
  if (p->case_prefix && no > 0 && F.n == 0 && group_keys.empty()) n_groups = 0;

  DBuf<uint32_t> err(1, s);
  LH_HIP(hipMemsetAsync(err.p, 0, sizeof(uint32_t), s));

  // leaf attribute: intersect and aggregate
  ElemArgs a{};
  DepthWork dw;
  // two sets with set semantics and COUNT: the descriptor-driven leaf, which
  // also intersects two bitsets word by word
  bool all_set = !is_sum;
  for (const auto& A : p->atoms) all_set = all_set && !A.bag;
  const bool leaf2 = p->case_prefix && all_set && p->parts[leaf].size() == 2;
  if (F.n) depth_work(p, leaf, F, a, dw, s, leaf2);
  const uint64_t total = dw.total;
  const uint64_t nblk = dw.nblk;
  if (nblk >= (1ull << 31)) fail(LH_ERR_OVERFLOW, "join: too much work at the last attribute");
  LeafArgs& L = a.leaf;
  L.n_atoms = na;
  L.sum = is_sum ? 1u : 0u;
  L.lsb = p->exact_lsb;
  L.D = D;
  L.err = err.p;
  a.n_atoms = na;
  a.n_outv = no;
  for (uint32_t j = 0; j < no; j++) a.outv_in[j] = F.outv[j].p;
  uint32_t need = 0;
  for (uint32_t e = 0; e < na; e++) {
    const PlanAtom& A = p->atoms[e];
    LeafAtom& LA = L.at[e];
    LA.part = -1;
    for (uint32_t i = 0; i < p->parts[leaf].size(); i++)
      if (p->parts[leaf][i].atom == e) LA.part = (int32_t)i;
    LA.pos = F.pos[e].p;
    LA.run = A.bag ? A.trie->lv[A.n_levels - 1].offs.p : nullptr;
    LA.anno = (is_sum && A.anno >= 0) ? A.trie->annos[A.anno].p : nullptr;
    LA.gmeta = nullptr;
    for (uint32_t g = 0; g < ngc; g++)
      if (p->groups[g].atom == e) {
        // every meta column of the atom that is grouped on has its own
        // output column
        LA.gmeta = A.trie->meta[p->groups[g].meta_col].p;
        L.gm_col[no + g] = LA.gmeta;
        L.gm_atom[no + g] = (int32_t)e;
      }
    LA.expand = (LA.anno || LA.gmeta) ? 1u : 0u;
    if (LA.part >= 0 && (A.bag || LA.expand)) need |= 1u << LA.part;
  }
  a.need_pos_mask = need;

  lh_result& R = res->pub;
  R.n_cols = n_cols;
  R.exact = is_sum ? 1u : 0u;

  if (p->case_prefix) {
    // streamed groups: one accumulator per group of the output prefix
    DBuf<uint64_t> gcount(n_groups ? n_groups : 1, s);
    DBuf<int64_t> gacc(is_sum ? (n_groups ? n_groups : 1) * EXACT_MAXD : 0, s);
    LH_HIP(hipMemsetAsync(gcount.p, 0, gcount.n * sizeof(uint64_t), s));
    if (is_sum) LH_HIP(hipMemsetAsync(gacc.p, 0, gacc.n * sizeof(int64_t), s));
    L.gid = no > 0 ? F.gid.p : nullptr;
    L.gcount = gcount.p;
    L.gacc = gacc.p;
    if (total) {
      if (leaf2) {
        // two sets, set semantics: per-unit descriptors, one load per wave
        DBuf<UnitDesc> desc(dw.units, s);
        WorkArgs wa{};
        wa.np = 2;
        wa.set[0] = a.set[0];
        wa.set[1] = a.set[1];
        // the top bucket (rows whose two sets hold TOP_MIN elements or
        // more, in units of TOP_EL) and the merged rows each run as a launch
        // of their own
        struct UnitCounts {
          uint64_t top, merge;
        };
        const UnitCounts nu = read_scalar(reinterpret_cast<const UnitCounts*>(dw.n_top.p), s);
        const bool split = nu.top != 0, merged = nu.merge != 0;
        DBuf<uint32_t> top_flag(split ? dw.units : 0, s), merge_flag(merged ? dw.units : 0, s);
        {
          ProfScope ps("leaf_units", s, dw.units, 0);
          k_unit_desc<<<grid_for(dw.units), 256, 0, s>>>(wa, dw.U.p, dw.urow.p, dw.drv.p, dw.units, desc.p,
                                                          split ? top_flag.p : nullptr,
                                                          merged ? merge_flag.p : nullptr);
        }
        LH_HIP(hipGetLastError());
        // each class's units in unit order, so that units of one row run
        // close together (and share the L2) as they do in the main launch
        DBuf<uint32_t> top_list(split ? dw.units : 0, s), merge_list(merged ? dw.units : 0, s);
        const uint64_t top_units = split ? select_flagged(top_flag.p, dw.units, top_list.p, s) : 0u;
        const uint64_t merge_units = merged ? select_flagged(merge_flag.p, dw.units, merge_list.p, s) : 0u;
        top_flag.reset();
        merge_flag.reset();
        Leaf2Args l2{};
        l2.keys[0] = a.set[0].keys;
        l2.keys[1] = a.set[1].keys;
        l2.samp[0] = a.set[0].samp;
        l2.samp[1] = a.set[1].samp;
        l2.pool[0] = a.set[0].pool;
        l2.pool[1] = a.set[1].pool;
        l2.desc = desc.p;
        l2.gcount = L.gcount;
        l2.units = dw.units;
        l2.n_desc = dw.units;
        l2.nvblk = nblk;
        DBuf<uint64_t> ucnt(L.gid ? dw.units : 0, s);
        l2.ucnt = ucnt.p;
        {
          ProfScope ps("leaf_aggregate", s, F.n, total);
          k_leaf2_count<false, U_IT><<<leaf_grid(nblk), J_NT, 0, s>>>(l2);
        }
        LH_HIP(hipGetLastError());
        if (top_units) {
          Leaf2Args lt = l2;
          lt.list = top_list.p;
          lt.units = top_units;
          lt.nvblk = (top_units + J_NW - 1) / J_NW;
          ProfScope ps("leaf_top", s, top_units, 0);
          k_leaf2_count<true, TOP_IT><<<leaf_grid(lt.nvblk), J_NT, 0, s>>>(lt);
        }
        LH_HIP(hipGetLastError());
        if (merge_units) {
          DBuf<MergeTile> tiles(merge_units, s);
          k_merge_tiles<<<grid_for(merge_units), 256, 0, s>>>(desc.p, merge_list.p, l2.keys[0], l2.keys[1],
                                                              merge_units, tiles.p);
          LH_HIP(hipGetLastError());
          ProfScope ps("leaf_merge", s, merge_units, 0);
          k_leaf2_merge<<<(unsigned)std::min<uint64_t>(merge_units, merge_grid()), M_NT, 0, s>>>(l2, tiles.p,
                                                                                          merge_units);
        }
        LH_HIP(hipGetLastError());
        if (L.gid) {
          ProfScope ps("leaf_groups", s, dw.units, 0);
          DBuf<uint64_t> uex(dw.units + 1, s), gstart(n_groups, s), gend(n_groups, s);
          scan_u64(ucnt.p, uex.p, dw.units, s);
          fill_u64(gstart.p, 0, n_groups, s);
          fill_u64(gend.p, 0, n_groups, s);
          k_group_bounds<<<grid_for(dw.units), 256, 0, s>>>(dw.urow.p, L.gid, dw.units, uex.p, gstart.p, gend.p);
          LH_HIP(hipGetLastError());
          k_group_add<<<grid_for(n_groups), 256, 0, s>>>(gstart.p, gend.p, n_groups, L.gcount);
        }
      } else {
        ProfScope ps("leaf_aggregate", s, F.n, total);
        if (all_set) launch_elem<M_LEAF_COUNT>(a, elem_grid(nblk), s);
        else launch_elem<M_LEAF_A>(a, elem_grid(nblk), s);
      }
      LH_HIP(hipGetLastError());
    }
    FinA f{};
    f.gcount = gcount.p;
    f.gacc = gacc.p;
    f.sum = L.sum;
    f.lsb = L.lsb;
    f.D = D;
    f.err = err.p;
    uint64_t n_out_rows;
    DBuf<uint64_t> off;
    if (no == 0) {
      n_out_rows = 1;
    } else {
      DBuf<uint32_t> flags(n_groups, s);
      off.alloc(n_groups + 1, s);
      if (n_groups) {
        k_nonzero_flags<<<grid_for(n_groups), 256, 0, s>>>(gcount.p, n_groups, flags.p);
        LH_HIP(hipGetLastError());
      }
      n_out_rows = scan_u32_to_u64(flags.p, off.p, n_groups, s);
      f.off = off.p;
    }
    f.n_cols = no;
    res->cols.resize(no);
    for (uint32_t c = 0; c < no; c++) {
      res->cols[c].alloc(n_out_rows, s);
      f.key_in[c] = c < group_keys.size() ? group_keys[c].p : nullptr;
      f.key_out[c] = res->cols[c].p;
    }
    res->counts.alloc(n_out_rows, s);
    if (is_sum) res->sums.alloc(n_out_rows, s);
    if (is_sum && p->want_parts) res->parts.alloc(n_out_rows * EXACT_PARTS, s);
    f.count_out = res->counts.p;
    f.sum_out = res->sums.p;
    f.parts = res->parts.p;
    const uint64_t nfin = no == 0 ? 1 : (group_keys.empty() ? 0 : n_groups);
    if (nfin) {
      k_finalize_groups<<<grid_for(nfin), 256, 0, s>>>(f, nfin);
      LH_HIP(hipGetLastError());
    }
    R.n_rows = n_out_rows;
  } else if (!group_in_place(p, F, a, nblk, total, no, n_cols, is_sum, D, err, res.get(), s)) {
    // materialize leaf tuples keyed by the output columns, sort, reduce
    R.group_impl = 1;
    uint64_t n_emit = 0;
    DBuf<uint64_t> boff;
    if (total) {
      DBuf<uint32_t> bcnt(nblk, s);
      a.blk_cnt = bcnt.p;
      {
        ProfScope ps("leaf_emit_count", s, F.n, total);
        launch_elem<M_LEAF_B_COUNT>(a, elem_grid(nblk), s);
      }
      LH_HIP(hipGetLastError());
      boff.alloc(nblk + 1, s);
      n_emit = scan_u32_to_u64(bcnt.p, boff.p, nblk, s);
    }
    if (n_emit >= (1ull << 32) - 1) fail(LH_ERR_OVERFLOW, "join: more than 2^32 output tuples to group");
    std::vector<DBuf<uint32_t>> cols(n_cols);
    DBuf<uint64_t> mult(n_emit, s);
    DBuf<double> hi(is_sum ? n_emit : 0, s), lo(is_sum ? n_emit : 0, s);
    L.n_cols = n_cols;
    for (uint32_t c = 0; c < n_cols; c++) {
      cols[c].alloc(n_emit, s);
      L.col_out[c] = cols[c].p;
      if (c < no) {
        const uint32_t attr = p->out_attrs[c];
        L.col_src[c] = (p->depth_of[attr] == leaf) ? -1 : (int32_t)c;
      } else {
        L.col_src[c] = -2;
      }
    }
    L.mult_out = mult.p;
    L.hi_out = hi.p;
    L.lo_out = lo.p;
    if (n_emit) {
      a.blk_off = boff.p;
      ProfScope ps("leaf_emit_fill", s, F.n, total);
      launch_elem<M_LEAF_B_FILL>(a, elem_grid(nblk), s);
      LH_HIP(hipGetLastError());
    }
    // sort tuples by the output columns
    std::vector<const uint32_t*> cptr(n_cols);
    std::vector<uint32_t> bits(n_cols);
    for (uint32_t c = 0; c < n_cols; c++) {
      cptr[c] = cols[c].p;
      bits[c] = bitlen(n_emit ? reduce_max_u32(cols[c].p, n_emit, s) : 0);
    }
    DBuf<uint32_t> perm(n_emit, s);
    lex_sort_perm(cptr.data(), bits.data(), n_cols, n_emit, perm.p, s);
    ColsArg ca{};
    ca.n = n_cols;
    for (uint32_t c = 0; c < n_cols; c++) ca.c[c] = cols[c].p;
    DBuf<uint32_t> head(n_emit, s);
    DBuf<uint64_t> segoff(n_emit + 1, s);
    uint64_t n_seg = 0;
    if (n_emit) {
      k_seg_heads<<<grid_for(n_emit), 256, 0, s>>>(ca, perm.p, n_emit, head.p);
      LH_HIP(hipGetLastError());
      n_seg = scan_u32_to_u64(head.p, segoff.p, n_emit, s);
    }
    // segoff is exclusive; segment of i = (inclusive count) - 1 = segoff[i+1]-1
    DBuf<uint64_t> gcount(n_seg ? n_seg : 1, s);
    DBuf<int64_t> gacc(is_sum ? (n_seg ? n_seg : 1) * EXACT_MAXD : 0, s);
    LH_HIP(hipMemsetAsync(gcount.p, 0, gcount.n * sizeof(uint64_t), s));
    if (is_sum) LH_HIP(hipMemsetAsync(gacc.p, 0, gacc.n * sizeof(int64_t), s));
    std::vector<DBuf<uint32_t>> segkeys(n_cols);
    SegAccArgs sa{};
    sa.cols = ca;
    sa.perm = perm.p;
    sa.segoff = segoff.p;
    sa.mult = mult.p;
    sa.hi = hi.p;
    sa.lo = lo.p;
    sa.sum = L.sum;
    sa.lsb = L.lsb;
    sa.D = D;
    sa.gcount = gcount.p;
    sa.gacc = gacc.p;
    sa.err = err.p;
    for (uint32_t c = 0; c < n_cols; c++) {
      segkeys[c].alloc(n_seg, s);
      sa.key_out[c] = segkeys[c].p;
    }
    if (n_emit) {
      k_seg_accumulate<<<grid_for(n_emit), 256, 0, s>>>(sa, n_emit);
      LH_HIP(hipGetLastError());
    }
    FinA f{};
    f.gcount = gcount.p;
    f.gacc = gacc.p;
    f.sum = L.sum;
    f.lsb = L.lsb;
    f.D = D;
    f.err = err.p;
    f.n_cols = n_cols;
    res->cols.resize(n_cols);
    for (uint32_t c = 0; c < n_cols; c++) {
      res->cols[c].alloc(n_seg, s);
      f.key_in[c] = segkeys[c].p;
      f.key_out[c] = res->cols[c].p;
    }
    res->counts.alloc(n_seg, s);
    if (is_sum) res->sums.alloc(n_seg, s);
    if (is_sum && p->want_parts) res->parts.alloc(n_seg * EXACT_PARTS, s);
    f.count_out = res->counts.p;
    f.sum_out = res->sums.p;
    f.parts = res->parts.p;
    if (n_seg) {
      k_finalize_groups<<<grid_for(n_seg), 256, 0, s>>>(f, n_seg);
      LH_HIP(hipGetLastError());
    }
    R.n_rows = n_seg;
  }
  const uint32_t leaf_err = read_scalar(err.p, s);
  if (leaf_err & ERR_COUNT_OVERFLOW) fail(LH_ERR_OVERFLOW, "join: a tuple count exceeds 2^64 - 1");
  if (leaf_err) fail(LH_ERR_UNSUPPORTED, "an annotation product did not fit the exact accumulator");

  // total contributing tuples
  res->colptr.resize(n_cols);
  for (uint32_t c = 0; c < n_cols; c++) res->colptr[c] = res->cols[c].p;
  R.out_keys = n_cols ? res->colptr.data() : nullptr;
  R.counts = res->counts.p;
  R.sums = is_sum ? res->sums.p : nullptr;
  uint64_t nj = 0;
  if (R.n_rows) {
    DBuf<uint64_t> tmp(R.n_rows + 1, s);
    nj = scan_u64(res->counts.p, tmp.p, R.n_rows, s);
  }
  R.n_join_tuples = nj;
  LH_HIP(hipStreamSynchronize(s));
  return res.release();
}

}  // namespace lh
