// Trie construction (section 2.2): lexicographic sort of the key tuples in
// level order, head flags per level, per-level keys and child offsets,
// set-mode deduplication or bag-mode runs, annotation/meta gathering and the
// per-set uint/bitset layout.
#include <algorithm>
#include <cstring>
#include <memory>

#include "device_common.h"
#include "lh_internal.h"

namespace lh {

namespace {

constexpr int TB_NT = 256;  // rows per tile in the level builder
constexpr int TB_NW = TB_NT / WAVE;

struct LevelCols {
  const uint32_t* k[LH_MAX_KEYS];  // sorted key column per level
  uint32_t n_levels;
};

__device__ __forceinline__ uint32_t head_mask(const LevelCols& c, uint64_t r) {
  // bit l set when row r starts a new node at level l
  // (levels unrolled: constant indices keep the column pointers in registers)
  uint32_t m = 0;
  bool h = (r == 0);
#pragma unroll
  for (uint32_t l = 0; l < LH_MAX_KEYS; l++) {
    if (l < c.n_levels) {
      if (!h) h = c.k[l][r] != c.k[l][r - 1];
      if (h) m |= 1u << l;
    }
  }
  return m;
}

// Heads per level per tile: counts[l * ntiles + tile].
__global__ __launch_bounds__(TB_NT) void k_head_counts(LevelCols c, uint64_t n, uint32_t* counts, uint32_t ntiles) {
  __shared__ uint32_t w_cnt[TB_NW][LH_MAX_KEYS];
  uint64_t r = (uint64_t)blockIdx.x * TB_NT + threadIdx.x;
  uint32_t m = r < n ? head_mask(c, r) : 0;
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (uint32_t l = 0; l < LH_MAX_KEYS; l++) {
    if (l < c.n_levels) {
      uint64_t b = ballot((m >> l) & 1u);
      if (lane_id() == 0) w_cnt[w][l] = (uint32_t)__popcll(b);
    }
  }
  __syncthreads();
  if (threadIdx.x < c.n_levels) {
    uint32_t t = 0;
    for (int j = 0; j < TB_NW; j++) t += w_cnt[j][threadIdx.x];
    counts[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = t;
  }
}

struct EmitArgs {
  LevelCols c;
  uint32_t* keys_out[LH_MAX_KEYS];   // level keys
  uint32_t* offs_out[LH_MAX_KEYS];   // level child offsets (levels 0..L-2)
  uint32_t* run_out;                 // bag: leaf run starts (sorted-row index); may be null
  uint32_t* kept_out;                // set: sorted-row index of each kept row; may be null
  uint32_t* rowkeys_out[LH_MAX_KEYS]; // set: each kept row's keys of the levels above the last; null when not wanted
  uint32_t* parent_out[LH_MAX_KEYS]; // level l >= 1: the level l-1 node above each node; may be null
  const uint32_t* tile_off;          // [l * ntiles + tile]
  uint32_t ntiles;
};

__global__ __launch_bounds__(TB_NT) void k_emit_levels(EmitArgs a, uint64_t n) {
  __shared__ uint32_t w_cnt[TB_NW][LH_MAX_KEYS];
  uint64_t r = (uint64_t)blockIdx.x * TB_NT + threadIdx.x;
  uint32_t m = r < n ? head_mask(a.c, r) : 0;
  const int w = threadIdx.x / WAVE;
  uint32_t rank[LH_MAX_KEYS];
#pragma unroll
  for (uint32_t l = 0; l < LH_MAX_KEYS; l++) {
    rank[l] = 0;
    if (l < a.c.n_levels) {
      uint64_t b = ballot((m >> l) & 1u);
      rank[l] = lanes_below(b);
      if (lane_id() == 0) w_cnt[w][l] = (uint32_t)__popcll(b);
    }
  }
  __syncthreads();
  if (r >= n) return;
  const uint32_t L = a.c.n_levels;
  uint32_t pos_prev = 0;
#pragma unroll
  for (uint32_t l = 0; l < LH_MAX_KEYS; l++) {
    if (l >= L || !((m >> l) & 1u)) continue;
    uint32_t pre = 0;
    for (int j = 0; j < w; j++) pre += w_cnt[j][l];
    uint32_t pos = a.tile_off[(uint64_t)l * a.ntiles + blockIdx.x] + pre + rank[l];
    a.keys_out[l][pos] = a.c.k[l][r];
    if (l > 0 && a.parent_out[l]) {
      // the parent is the last level l-1 node starting at or before row r
      uint32_t pp = 0;
      for (int j = 0; j < w; j++) pp += w_cnt[j][l - 1];
      a.parent_out[l][pos] = a.tile_off[(uint64_t)(l - 1) * a.ntiles + blockIdx.x] + pp + rank[l - 1] +
                             ((m >> (l - 1)) & 1u) - 1u;
    }
    // a head at level l-1 is also a head at l: its first child is pos
    if (l > 0 && ((m >> (l - 1)) & 1u)) a.offs_out[l - 1][pos_prev] = pos;
    if (l + 1 == L) {
      if (a.run_out) a.run_out[pos] = (uint32_t)r;
      if (a.kept_out) a.kept_out[pos] = (uint32_t)r;
#pragma unroll
      for (uint32_t j = 0; j < LH_MAX_KEYS; j++)
        if (j + 1 < L && a.rowkeys_out[j]) a.rowkeys_out[j][pos] = a.c.k[j][r];
    }
    pos_prev = pos;
  }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// Bit t-1 of a block's mask stays set while rows i-1, i are in
// lexicographic order of the last t levels (equal tuples are in order),
// for every i the block visits.  Bits only clear, and a wave stops once
// none is left, so unsorted input costs a fraction of a pass.  Each block
// writes its mask (atomics of every block on one address would serialize);
// k_and_total combines them.
__global__ __launch_bounds__(256) void k_sorted_tails(LevelCols c, uint64_t n, uint32_t all, uint32_t* part) {
  __shared__ uint32_t s_m[256 / WAVE];
  const int K = (int)c.n_levels;
  uint32_t known = all;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = 1 + (uint64_t)blockIdx.x * blockDim.x; i0 < n && known; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    uint32_t m = known;
    bool ord = true;  // order of the suffix from level l on
    // constant level indices: the column pointers stay in registers; each
    // lane loads its row once and takes row i - 1 from the lane below
#pragma unroll
    for (int l = LH_MAX_KEYS - 1; l >= 0; l--) {
      if (l < K) {
        const uint32_t b = i < n ? c.k[l][i] : 0u;
        uint32_t a = (uint32_t)__shfl_up((int)b, 1, 64);
        if (lane == 0 && i < n) a = c.k[l][i - 1];
        ord = a < b || (a == b && ord);
        if (i < n && !ord) m &= ~(1u << (K - 1 - l));
      }
    }
    for (int o = 32; o > 0; o >>= 1) m &= (uint32_t)__shfl_xor((int)m, o, 64);
    known = m;  // uniform over the wave
  }
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x / WAVE] = known;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = all;
    for (int w = 0; w < 256 / WAVE; w++) m &= s_m[w];
    part[blockIdx.x] = m;
  }
}

// AND of the blocks' masks, by one block.
__global__ __launch_bounds__(256) void k_and_total(const uint32_t* part, uint32_t nb, uint32_t all, uint32_t* out) {
  __shared__ uint32_t s_m[256 / WAVE];
  uint32_t m = all;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) m &= part[b];
  for (int o = 32; o > 0; o >>= 1) m &= (uint32_t)__shfl_xor((int)m, o, 64);
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = all;
    for (int w = 0; w < 256 / WAVE; w++) r &= s_m[w];
    *out = r;
  }
}

__global__ void k_line_samples(const uint32_t* keys, uint64_t n_samp, uint32_t* samp) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_samp; j += (uint64_t)gridDim.x * blockDim.x)
    samp[j] = keys[j << LINE_SHIFT];
}

// ---- layouts ---------------------------------------------------------------

struct SetRange {
  const uint32_t* offs;  // parent offsets (null for level 0)
  uint64_t root_n;       // level-0 size
};

__device__ __forceinline__ void set_range(const SetRange& sr, uint64_t s, uint32_t& b, uint32_t& e) {
  if (!sr.offs) { b = 0; e = (uint32_t)sr.root_n; }
  else { b = sr.offs[s]; e = sr.offs[s + 1]; }
}

__global__ void k_layout_words(SetRange sr, const uint32_t* keys, uint64_t n_sets, uint32_t mode,
                               const uint8_t* choice, uint64_t* words) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sets; s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    set_range(sr, s, b, e);
    uint64_t nw = 0;
    if (e > b) {
      uint32_t lo = keys[b], hi = keys[e - 1];
      uint64_t card = e - b;
      uint64_t span = (uint64_t)hi - lo + 1;
      bool bs = false;
      // plain rule: a bitset when the set fills at least 1/32 of its window
      if (mode == LH_LAYOUT_PLAIN || mode == LH_LAYOUT_LEARNED) bs = span <= 32ull * card;
      else if (mode == LH_LAYOUT_BITSET) bs = span <= 4096ull * card;
      if (choice && choice[s]) bs = choice[s] == 2;
      if (bs) nw = (((uint64_t)hi - (lo & ~63u)) >> 6) + 1;
    }
    words[s] = nw;
  }
}

__global__ void k_layout_desc(SetRange sr, const uint32_t* keys, uint64_t n_sets, const uint64_t* words,
                              const uint64_t* woff, uint64_t* bs_word, uint32_t* bs_base) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sets; s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    set_range(sr, s, b, e);
    bool bs = words[s] != 0;
    bs_word[s] = bs ? woff[s] : UINT64_MAX;
    bs_base[s] = (e > b) ? (keys[b] & ~63u) : 0u;
  }
}

// Bitset words from the keys.  A wave takes 64 consecutive keys; the keys
// of one (set, word) pair are consecutive (keys are sorted within a set, and
// sets follow each other), so the pairs are runs of lanes, marked by a
// ballot.  When some run holds more than one key, an OR over each lane's
// rest of its run (doubling steps, bounded by the run's end) gathers each
// word's bits in the run's first lane, which writes the word.  A run that
// goes on in the neighbouring wave (its first or last key's neighbour there
// is in the same word) ORs its part atomically into the word (the pool
// starts zeroed); words without keys stay zero.  Waves without a bitset key do no
// lane exchange at all.  Null bs_word: the keys form one set whose window
// starts at 0 at word 0 (the root index).
__global__ __launch_bounds__(256) void k_layout_fill(const uint32_t* keys, const uint32_t* parent, uint64_t n,
                                                     const uint64_t* bs_word, const uint32_t* bs_base, uint64_t* pool) {
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); j0 < n; j0 += stride) {
    const uint64_t j = j0 + lane;
    uint64_t tag = ~0ull, bits = 0, w = 0;  // tag: set << 32 | word (words < 2^26), ~0 for no key
    if (j < n) {
      const uint32_t st = parent ? parent[j] : 0u;
      const uint64_t w0 = bs_word ? bs_word[st] : 0u;
      if (w0 != UINT64_MAX) {
        const uint32_t d = keys[j] - (bs_word ? bs_base[st] : 0u);
        tag = ((uint64_t)st << 32) | (d >> 6);
        bits = 1ull << (d & 63u);
        w = w0 + (d >> 6);
      }
    }
    const bool live = tag != ~0ull;
    const uint64_t L = ballot(live);
    if (!L) continue;  // uniform: no bitset key in the wave
    const uint64_t prev = __shfl_up(tag, 1, WAVE);
    const bool head = live && (lane == 0 || prev != tag);
    // runs start at heads; lanes without a key are runs of their own
    const uint64_t S = ballot(head) | ~L;
    const uint64_t above = lane < WAVE - 1 ? S >> (lane + 1) : 0ull;
    const uint32_t end = above ? (uint32_t)lane + 1u + (uint32_t)__builtin_ctzll(above) : (uint32_t)WAVE;
    if (L & ~S) {  // uniform: some run holds two keys or more
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) {
        const uint64_t ob = __shfl_down(bits, o, WAVE);
        if ((uint32_t)lane + (uint32_t)o < end) bits |= ob;
      }
    }
    if (head) {
      // does the run go on in the wave before (lane 0) or after (a run
      // reaching the last lane)?  The neighbouring key shares the word when
      // it has the same set and the same offset >> 6.
      const uint32_t st = (uint32_t)(tag >> 32), word = (uint32_t)tag;
      const uint32_t base = bs_word ? bs_base[st] : 0u;
      bool shared = false;
      if (lane == 0 && j > 0)
        shared = (parent ? parent[j - 1] : 0u) == st && ((keys[j - 1] - base) >> 6) == word;
      if (end == (uint32_t)WAVE && j0 + WAVE < n)
        shared = shared || ((parent ? parent[j0 + WAVE] : 0u) == st && ((keys[j0 + WAVE] - base) >> 6) == word);
      if (shared) atomicOr((unsigned long long*)&pool[w], (unsigned long long)bits);
      else pool[w] = bits;
    }
  }
}

__global__ void k_word_popc(const uint64_t* pool, uint64_t n, uint32_t* cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    cnt[i] = (uint32_t)__popcll(pool[i]);
}

__global__ void k_rank_delta(SetRange sr, uint64_t n_sets, const uint64_t* bs_word, const uint32_t* rank,
                             uint32_t* delta) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sets; s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b, e;
    set_range(sr, s, b, e);
    const uint64_t w = bs_word[s];
    delta[s] = w != UINT64_MAX ? b - rank[w] : 0u;
  }
}

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 256 * 64));
}

uint32_t bitlen(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

}  // namespace

__global__ void k_count_bitsets(const uint64_t* bs_word, uint64_t n, unsigned long long* out) {
  uint32_t c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    c += bs_word[i] != UINT64_MAX;
  for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, (unsigned long long)c);
}

uint64_t count_bitsets(const lh_trie* t, uint32_t l, hipStream_t s) {
  const Level& L = t->lv[l];
  if (!L.n_sets || !L.pool_words) return 0;
  DBuf<unsigned long long> c(1, s);
  LH_HIP(hipMemsetAsync(c.p, 0, sizeof(unsigned long long), s));
  k_count_bitsets<<<std::min<unsigned>(grid_for(L.n_sets), 1024), 256, 0, s>>>(L.bs_word.p, L.n_sets, c.p);
  LH_HIP(hipGetLastError());
  return read_scalar(c.p, s);
}

void build_layouts(lh_trie* t, uint32_t l, uint32_t mode, const uint32_t* parent, hipStream_t s) {
  Level& L = t->lv[l];
  L.n_sets = (l == 0) ? 1 : t->lv[l - 1].n;
  SetRange sr{l == 0 ? nullptr : t->lv[l - 1].offs.p, t->lv[0].n};
  L.bs_word.alloc(L.n_sets, s);
  L.bs_base.alloc(L.n_sets, s);
  if (L.n_sets == 0) return;
  DBuf<uint64_t> words(L.n_sets, s), woff(L.n_sets + 1, s);
  DBuf<uint8_t> choice;
  const bool learned = mode == LH_LAYOUT_LEARNED && learned_layout_choices(t, l, s, choice);
  k_layout_words<<<grid_for(L.n_sets), 256, 0, s>>>(sr, L.keys.p, L.n_sets, mode, learned ? choice.p : nullptr,
                                                    words.p);
  LH_HIP(hipGetLastError());
  L.pool_words = scan_u64(words.p, woff.p, L.n_sets, s);
  k_layout_desc<<<grid_for(L.n_sets), 256, 0, s>>>(sr, L.keys.p, L.n_sets, words.p, woff.p, L.bs_word.p, L.bs_base.p);
  LH_HIP(hipGetLastError());
  L.n_bitsets = 0;
  if (L.pool_words) {
    L.pool.alloc(L.pool_words, s);
    ProfScope ps("layout_fill", s, L.n_sets, L.pool_words);
    LH_HIP(hipMemsetAsync(L.pool.p, 0, L.pool_words * sizeof(uint64_t), s));
    k_layout_fill<<<grid_for(L.n), 256, 0, s>>>(L.keys.p, parent, L.n, L.bs_word.p, L.bs_base.p, L.pool.p);
    LH_HIP(hipGetLastError());
  }
  // positions inside bitset sets are needed when a deeper level hangs below
  // or the rows of a bag are reached through them: a rank directory turns
  // them into one load and a popcount
  if (L.pool_words && (l + 1 < t->n_levels || (t->flags & LH_BAG))) {
    DBuf<uint32_t> pc(L.pool_words, s);
    k_word_popc<<<grid_for(L.pool_words), 256, 0, s>>>(L.pool.p, L.pool_words, pc.p);
    LH_HIP(hipGetLastError());
    L.bs_rank.alloc(L.pool_words + 1, s);
    scan_u32_dev(pc.p, L.bs_rank.p, L.pool_words, s);
    L.bs_delta.alloc(L.n_sets, s);
    k_rank_delta<<<grid_for(L.n_sets), 256, 0, s>>>(sr, L.n_sets, L.bs_word.p, L.bs_rank.p, L.bs_delta.p);
    LH_HIP(hipGetLastError());
  }
}

namespace {

struct LevelOffs {
  const uint32_t* offs[LH_MAX_KEYS];  // child offsets of levels 0 .. n_levels-2
  const uint32_t* run;                // bag: run offsets of the last level
  uint32_t n_levels;
};

// Rows under each level-0 node: its child range composed down to the last
// level (and through the runs of a bag trie).
__global__ void k_level0_rows(LevelOffs lo, uint64_t n0, uint32_t* rows) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n0; p += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t b = (uint32_t)p, e = (uint32_t)p + 1;
    for (uint32_t l = 0; l + 1 < lo.n_levels; l++) {
      b = lo.offs[l][b];
      e = lo.offs[l][e];
    }
    if (lo.run) {
      b = lo.run[b];
      e = lo.run[e];
    }
    rows[p] = e - b;
  }
}

}  // namespace

void ensure_column_stats(lh_trie* t, hipStream_t s) {
  if (t->col_stats) return;
  // the first column: its values are the level-0 keys, each shared by the
  // rows under its node
  if (t->n_levels && t->lv[0].n) {
    LevelOffs lo{};
    lo.n_levels = t->n_levels;
    for (uint32_t l = 0; l + 1 < t->n_levels; l++) lo.offs[l] = t->lv[l].offs.p;
    lo.run = (t->flags & LH_BAG) ? t->lv[t->n_levels - 1].offs.p : nullptr;
    DBuf<uint32_t> rows(t->lv[0].n, s);
    k_level0_rows<<<grid_for(t->lv[0].n), 256, 0, s>>>(lo, t->lv[0].n, rows.p);
    LH_HIP(hipGetLastError());
    t->col_distinct[0] = t->lv[0].n;
    t->col_freq_max[0] = reduce_max_u32(rows.p, t->lv[0].n, s);
  } else if (t->n_levels) {
    t->col_distinct[0] = 0;
    t->col_freq_max[0] = 0;
  }
  // A two-level trie without row columns: sort its rows by (level 1,
  // level 0) (level 0 is in order already, so only level 1's bits are
  // sorted) and keep them; the statistics come from the sorted runs and a
  // copy of the trie in the swapped level order takes the rows unsorted.
  if (t->n_levels == 2 && t->annos.empty() && t->meta.empty() && t->key_bits[0] + t->key_bits[1] <= 64 &&
      t->n_rows) {
    const uint32_t* cols[2] = {row_keys(t, 1), row_keys(t, 0)};
    const uint32_t bits[2] = {t->key_bits[1], t->key_bits[0]};
    t->tsorted[0].alloc(t->n_rows, s);
    t->tsorted[1].alloc(t->n_rows, s);
    uint32_t* out[2] = {t->tsorted[0].p, t->tsorted[1].p};
    sort_packed(cols, bits, 2, t->n_rows, nullptr, out, s, 1);
    sorted_run_stats(t->tsorted[0].p, t->n_rows, t->col_distinct[1], t->col_freq_max[1], s);
    t->col_stats = true;
    return;
  }
  for (uint32_t l = 1; l < t->n_levels; l++) {
    if (t->key_max[l] < (1u << 28)) {
      column_freq(row_keys(t, l), t->n_rows, t->key_max[l], t->col_distinct[l], t->col_freq_max[l], s);
    } else {
      t->col_distinct[l] = t->n_rows;
      t->col_freq_max[l] = 1;
    }
  }
  t->col_stats = true;
}

// The presorted-tail mask of the rows into *mask (device): bit t-1 set when
// the rows are in lexicographic order of their last t levels.
static void presorted_mask(const uint32_t* const* col, uint32_t n_keys, uint64_t n, uint32_t* mask, hipStream_t s) {
  LevelCols c{};
  c.n_levels = n_keys;
  for (uint32_t l = 0; l < n_keys; l++) c.k[l] = col[l];
  const uint32_t all = (1u << n_keys) - 1;
  const unsigned nb = grid_for(n);
  DBuf<uint32_t> part(nb, s);
  ProfScope ps("trie_presorted", s, n, 0);
  k_sorted_tails<<<nb, 256, 0, s>>>(c, n, all, part.p);
  LH_HIP(hipGetLastError());
  k_and_total<<<1, 256, 0, s>>>(part.p, nb, all, mask);
  LH_HIP(hipGetLastError());
}

// The most trailing levels whose order a presorted-tail mask shows (0: not
// even the last level's).
static uint32_t tail_of_mask(uint32_t mask, uint32_t n_keys) {
  for (uint32_t t = n_keys; t >= 1; t--)
    if (mask >> (t - 1) & 1u) return t;
  return 0;
}

lh_trie* build_trie(uint64_t n_rows, uint32_t n_keys, const uint32_t* const* keys, uint32_t n_annos,
                    const double* const* annos, uint32_t n_meta, const uint32_t* const* meta,
                    const uint32_t* level_order, uint32_t flags, const uint32_t* sel, uint64_t n_sel,
                    hipStream_t s, uint32_t sorted_tail, bool detect_sorted) {
  const uint64_t n = sel ? n_sel : n_rows;
  sorted_tail = std::min(sorted_tail, n_keys);
  if (n >= (1ull << 32) - 1) fail(LH_ERR_OVERFLOW, "trie build: 2^32 - 1 rows or more");
  const bool bag = (flags & LH_BAG) != 0;
  std::unique_ptr<lh_trie> t(new lh_trie());
  t->magic = TRIE_MAGIC;
  t->n_levels = n_keys;
  t->flags = flags;
  t->n_input = n;
  for (uint32_t l = 0; l < n_keys; l++) t->level_order[l] = level_order ? level_order[l] : l;

  // Input columns in level order (compacted through `sel` if given).
  std::vector<DBuf<uint32_t>> selcols;
  const uint32_t* col[LH_MAX_KEYS];
  for (uint32_t l = 0; l < n_keys; l++) {
    const uint32_t* src = keys[t->level_order[l]];
    if (sel) {
      selcols.emplace_back(n, s);
      gather_u32(src, sel, selcols.back().p, n, s);
      src = selcols.back().p;
    }
    col[l] = src;
  }
  // every level's largest key and, when asked, the presorted tail: one
  // read back for all of them
  struct InputStats {
    uint32_t key_max[LH_MAX_KEYS];
    uint32_t tail_mask;
  };
  {
    DBuf<InputStats> st(1, s);
    LH_HIP(hipMemsetAsync(st.p, 0, sizeof(InputStats), s));
    for (uint32_t l = 0; l < n_keys; l++) max_u32_into(col[l], n, &st.p->key_max[l], s);
    const bool detect = detect_sorted && sorted_tail == 0 && n > 1;
    if (detect) presorted_mask(col, n_keys, n, &st.p->tail_mask, s);
    const InputStats h = read_scalar(st.p, s);
    for (uint32_t l = 0; l < n_keys; l++) {
      t->key_max[l] = h.key_max[l];
      t->key_bits[l] = bitlen(t->key_max[l]);
    }
    if (detect) sorted_tail = tail_of_mask(h.tail_mask, n_keys);
  }

  // The permutation is needed only to carry annotation and meta columns.
  // Keys that pack into one word are sorted as such and unpacked into the
  // sorted columns (no gathers); wider keys take the multi-pass sort.
  const bool need_perm = n_annos || n_meta;
  DBuf<uint32_t> perm(need_perm ? n : 0, s);
  LevelCols lc{};
  lc.n_levels = n_keys;
  std::vector<DBuf<uint32_t>> sorted;
  uint32_t* sorted_p[LH_MAX_KEYS];
  // rows already in order: a set trie reads the input columns as they are;
  // other tries copy them (a bag keeps its sorted columns) with the
  // identity permutation
  const bool in_order = sorted_tail >= n_keys && !need_perm && !bag && !sel;
  const bool copy_order = sorted_tail >= n_keys && !in_order;
  for (uint32_t l = 0; l < n_keys; l++) {
    if (in_order) {
      sorted.emplace_back();
      sorted_p[l] = nullptr;
      lc.k[l] = col[l];
    } else {
      sorted.emplace_back(n, s);
      sorted_p[l] = sorted.back().p;
      lc.k[l] = sorted.back().p;
    }
  }
  if (in_order) {
    // nothing to sort
  } else if (copy_order) {
    for (uint32_t l = 0; l < n_keys && n; l++)
      LH_HIP(hipMemcpyAsync(sorted_p[l], col[l], n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (need_perm && (sel || !bag)) iota_u32(perm.p, n, s);  // else the rows are copied as they are (below)
  } else if (!sort_packed(col, t->key_bits, n_keys, n, need_perm ? perm.p : nullptr, sorted_p, s, sorted_tail)) {
    if (!need_perm) perm.alloc(n, s);
    // a stable sort by the leading levels keeps the presorted tail's order
    lex_sort_perm(col, t->key_bits, n_keys - sorted_tail, n, perm.p, s);
    for (uint32_t l = 0; l < n_keys; l++) gather_u32(col[l], perm.p, sorted_p[l], n, s);
  }

  uint32_t ntiles = (uint32_t)((n + TB_NT - 1) / TB_NT);
  uint64_t cn = (uint64_t)ntiles * n_keys;
  DBuf<uint32_t> counts(cn ? cn : 1, s), toff(cn + 1, s);
  if (n) {
    ProfScope ps("trie_head_counts", s, n, 0);
    k_head_counts<<<ntiles, TB_NT, 0, s>>>(lc, n, counts.p, ntiles);
    LH_HIP(hipGetLastError());
  }
  // scan per level: offsets of level l start at toff[l*ntiles]
  std::vector<uint64_t> level_n(n_keys, 0);
  DBuf<uint32_t> tmp(ntiles + 1, s);
  for (uint32_t l = 0; l < n_keys; l++) {
    uint64_t tot = n ? scan_u32(counts.p + (uint64_t)l * ntiles, tmp.p, ntiles, s) : 0;
    if (n) LH_HIP(hipMemcpyAsync(toff.p + (uint64_t)l * ntiles, tmp.p, ntiles * sizeof(uint32_t),
                                 hipMemcpyDeviceToDevice, s));
    level_n[l] = tot;
  }
  EmitArgs ea{};
  ea.c = lc;
  ea.tile_off = toff.p;
  ea.ntiles = ntiles;
  for (uint32_t l = 0; l < n_keys; l++) {
    Level& L = t->lv[l];
    L.n = level_n[l];
    L.keys.alloc(L.n, s);
    ea.keys_out[l] = L.keys.p;
    if (l + 1 < n_keys) {
      L.offs.alloc(L.n + 1, s);
      ea.offs_out[l] = L.offs.p;
    }
  }
  const uint64_t n_leaf = n_keys ? level_n[n_keys - 1] : 0;
  DBuf<uint32_t> kept;
  if (bag) {
    t->lv[n_keys - 1].offs.alloc(n_leaf + 1, s);
    ea.run_out = t->lv[n_keys - 1].offs.p;
  } else {
    // a set keeps the leaf heads' rows: their keys are written as the
    // heads are found (the row positions only when columns follow them);
    // their last keys are the last level's keys
    for (uint32_t l = 0; l + 1 < n_keys; l++) {
      t->skeys[l].alloc(n_leaf, s);
      ea.rowkeys_out[l] = t->skeys[l].p;
    }
    if (need_perm) {
      kept.alloc(n_leaf, s);
      ea.kept_out = kept.p;
    }
  }
  // parents of each level's nodes, for the bitset fill of levels below 0
  std::vector<DBuf<uint32_t>> parent(n_keys);
  for (uint32_t l = 1; l < n_keys; l++) {
    parent[l].alloc(level_n[l], s);
    ea.parent_out[l] = parent[l].p;
  }
  if (n) {
    ProfScope ps("trie_emit_levels", s, n, 0);
    k_emit_levels<<<ntiles, TB_NT, 0, s>>>(ea, n);
    LH_HIP(hipGetLastError());
  }
  // closing offsets: offs_l[n_l] = n_{l+1}; run[n_leaf] = n
  for (uint32_t l = 0; l + 1 < n_keys; l++) {
    k_set_u32<<<1, 1, 0, s>>>(t->lv[l].offs.p + t->lv[l].n, (uint32_t)level_n[l + 1]);
    LH_HIP(hipGetLastError());
  }
  if (bag) {
    k_set_u32<<<1, 1, 0, s>>>(t->lv[n_keys - 1].offs.p + n_leaf, (uint32_t)n);
    LH_HIP(hipGetLastError());
  }

  for (uint32_t l = 0; l < n_keys; l++) {
    Level& L = t->lv[l];
    const uint64_t ns = (L.n + (1u << LINE_SHIFT) - 1) >> LINE_SHIFT;
    L.samp.alloc(ns, s);
    if (ns) {
      k_line_samples<<<grid_for(ns), 256, 0, s>>>(L.keys.p, ns, L.samp.p);
      LH_HIP(hipGetLastError());
    }
  }

  // Rows in trie order: bag keeps every sorted row, set keeps leaf heads.
  // Their keys are the sorted columns themselves (bag), or the sorted
  // columns at the leaf heads, written by the level emission (set).
  t->n_rows = bag ? n : n_leaf;
  const uint32_t* rowsel = perm.p;  // sorted position -> input row
  DBuf<uint32_t> keptrows;
  if (!bag && need_perm) {  // (a set relation carries neither; kept for safety)
    keptrows.alloc(n_leaf, s);
    gather_u32(perm.p, kept.p, keptrows.p, n_leaf, s);
    rowsel = keptrows.p;
  }
  if (bag)
    for (uint32_t l = 0; l < n_keys; l++) t->skeys[l] = std::move(sorted[l]);
  // annotation / meta columns (bag relations only); `sel` maps rows first
  DBuf<uint32_t> srcrow;
  const uint32_t* rowmap = rowsel;
  if (sel && (n_annos || n_meta)) {
    srcrow.alloc(t->n_rows, s);
    gather_u32(sel, rowsel, srcrow.p, t->n_rows, s);
    rowmap = srcrow.p;
  }
  // a presorted bag keeps its input rows in order: plain copies
  const bool same_rows = copy_order && bag && !sel;
  for (uint32_t a = 0; a < n_annos; a++) {
    t->annos.emplace_back(t->n_rows, s);
    if (same_rows) {
      if (t->n_rows)
        LH_HIP(hipMemcpyAsync(t->annos.back().p, annos[a], t->n_rows * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      gather_f64(annos[a], rowmap, t->annos.back().p, t->n_rows, s);
    }
    t->astats.push_back(anno_stats(t->annos.back().p, t->n_rows, s));
  }
  for (uint32_t m = 0; m < n_meta; m++) {
    t->meta.emplace_back(t->n_rows, s);
    if (same_rows) {
      if (t->n_rows)
        LH_HIP(hipMemcpyAsync(t->meta.back().p, meta[m], t->n_rows * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    } else {
      gather_u32(meta[m], rowmap, t->meta.back().p, t->n_rows, s);
    }
  }

  uint32_t mode = flags & LH_LAYOUT_MASK;
  for (uint32_t l = 0; l < n_keys; l++) build_layouts(t.get(), l, mode, l ? parent[l].p : nullptr, s);
  // root index, when level 0 holds at least one key per 64 of its span
  const uint64_t n0 = t->lv[0].n;
  if (n0) {
    const uint64_t span = (uint64_t)t->key_max[0] + 1;
    if (span <= 64 * n0 && span <= (1ull << 32)) {
      const uint64_t words = (span + 63) / 64;
      t->root_span = span;
      t->root_bits.alloc(words, s);
      t->root_rank.alloc(words + 1, s);
      LH_HIP(hipMemsetAsync(t->root_bits.p, 0, words * sizeof(uint64_t), s));
      k_layout_fill<<<grid_for(n0), 256, 0, s>>>(t->lv[0].keys.p, nullptr, n0, nullptr, nullptr, t->root_bits.p);
      LH_HIP(hipGetLastError());
      DBuf<uint32_t> pc(words, s);
      k_word_popc<<<grid_for(words), 256, 0, s>>>(t->root_bits.p, words, pc.p);
      LH_HIP(hipGetLastError());
      scan_u32_dev(pc.p, t->root_rank.p, words, s);
    }
  }
  LH_HIP(hipStreamSynchronize(s));
  return t.release();
}

}  // namespace lh
