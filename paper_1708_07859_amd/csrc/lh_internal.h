// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lh.h"

namespace lh {

// ---------------------------------------------------------------------------
// Errors: internal code throws lh::Error; the C ABI turns it into lh_status.
// ---------------------------------------------------------------------------
struct Error {
  lh_status status;
  std::string msg;
};

[[noreturn]] void fail(lh_status st, const std::string& msg);

#define LH_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) ::lh::hip_fail(e_, #expr, __FILE__, __LINE__);          \
  } while (0)

[[noreturn]] void hip_fail(hipError_t e, const char* what, const char* file, int line);

// ---------------------------------------------------------------------------
// Device memory: stream-ordered allocations from the device's default pool.
// ---------------------------------------------------------------------------
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
long live_allocations();

// A caller-provided device region that stands in for allocation: while an
// ArenaScope is alive on a host thread, dalloc on that thread bump-allocates
// from [base, base + cap) (256-byte aligned) and fails with LH_ERR_OVERFLOW
// when the region is full; dfree of memory inside a registered region does
// nothing.
struct Arena {
  void* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  size_t peak = 0;
};
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena& a);
  ~ArenaScope();
};
void register_arena_range(void* base, size_t cap);
bool arena_active();

template <class T>
struct DBuf {  // owning device buffer, freed on the stream it was made on
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  DBuf() = default;
  DBuf(size_t count, hipStream_t st) { alloc(count, st); }
  void alloc(size_t count, hipStream_t st) {
    reset();
    s = st;
    n = count;
    p = count ? static_cast<T*>(dalloc(count * sizeof(T), st)) : nullptr;
  }
  void reset() {
    if (p) dfree(p, s);
    p = nullptr;
    n = 0;
  }
  T* release() {
    T* q = p;
    p = nullptr;
    n = 0;
    return q;
  }
  ~DBuf() { reset(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
    return *this;
  }
};

// A 64-byte pinned host buffer per host thread, kept until the process
// ends: a scalar read back into pinned memory skips the staging of a
// pageable copy (about 40 us per read on the sync-heavy paths).
inline void* pinned_scratch() {
  thread_local void* p = nullptr;
  if (!p) LH_HIP(hipHostMalloc(&p, 64, hipHostMallocPortable));
  return p;
}

template <class T>
T read_scalar(const T* dptr, hipStream_t s) {
  static_assert(sizeof(T) <= 64, "read_scalar: at most 64 bytes");
  if (arena_active()) {
    // no host allocation either: read into this frame
    T v;
    LH_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
    return v;
  }
  T* h = static_cast<T*>(pinned_scratch());
  LH_HIP(hipMemcpyAsync(h, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  LH_HIP(hipStreamSynchronize(s));
  return *h;
}

// ---------------------------------------------------------------------------
// Primitives (prims.hip)
// ---------------------------------------------------------------------------
// Exclusive scan of n uint32 values into n+1 uint64 offsets (out[n] = total).
uint64_t scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, hipStream_t s);
// Exclusive scan of n uint64 values into n+1 uint64 offsets; returns total.
uint64_t scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s);
// Exclusive scan, uint32 -> uint32 (caller guarantees the total fits); out has n+1.
uint32_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s);
// The same without reading the total back (it stays in out[n]).
void scan_u32_dev(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s);
uint32_t reduce_max_u32(const uint32_t* in, uint64_t n, hipStream_t s);
// Raise *out (device, set beforehand) to the largest of in[0, n); nothing is read back.
void max_u32_into(const uint32_t* in, uint64_t n, uint32_t* out, hipStream_t s);
// Distinct values and the largest value frequency of a column whose values
// are below `range` (a histogram pass).
void column_freq(const uint32_t* col, uint64_t n, uint32_t range, uint64_t& distinct, uint64_t& freq_max,
                 hipStream_t s);
// Distinct values and the longest run of a sorted column.
void sorted_run_stats(const uint32_t* sorted, uint64_t n, uint64_t& distinct, uint64_t& freq_max, hipStream_t s);
// Indices i < n with flags[i] != 0, in order, into out (n entries); returns count.
uint64_t select_flagged(const uint32_t* flags, uint64_t n, uint32_t* out, hipStream_t s);
void iota_u32(uint32_t* out, uint64_t n, hipStream_t s);
void fill_u32(uint32_t* out, uint32_t v, uint64_t n, hipStream_t s);
void fill_u64(uint64_t* out, uint64_t v, uint64_t n, hipStream_t s);
void gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, uint64_t n, hipStream_t s);
void gather_f64(const double* src, const uint32_t* idx, double* dst, uint64_t n, hipStream_t s);

// Stable LSD radix sort of (key, val) pairs on bits [lo_bit, bits) of key
// (pairs already ordered by the bits below lo_bit keep that order).
// Sorted pairs end in (keys, vals); tmp buffers must hold n entries each.
// vals (and tvals) may be null: keys only.
void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tkeys, uint32_t* tvals,
                      uint64_t n, uint32_t bits, hipStream_t s, uint32_t lo_bit = 0);

// Sort rows lexicographically by cols[0], cols[1], ... when their bits add
// up to at most 64: one packed key per row, radix-sorted, then unpacked into
// the sorted columns (ncols buffers of n).  perm (n entries, may be null)
// receives the input row of each sorted position.  Rows already sorted by
// the last sorted_tail columns are sorted by the others only (stably).  Returns false, doing
// nothing, when the keys do not fit one word.
bool sort_packed(const uint32_t* const* cols, const uint32_t* bits, uint32_t ncols, uint64_t n, uint32_t* perm,
                 uint32_t* const* sorted, hipStream_t s, uint32_t sorted_tail = 0);

// Permutation that sorts rows lexicographically by cols[0], cols[1], ...
// (stable); bits[c] = significant bits of column c.  perm receives n ids.
void lex_sort_perm(const uint32_t* const* cols, const uint32_t* bits, uint32_t ncols,
                   uint64_t n, uint32_t* perm, hipStream_t s);

// Exponent of the lowest set bit over the non-zero finite values (INT32_MAX
// if none), the largest |v| and whether any value is non-finite.
struct AnnoStats {
  int32_t qmin;
  double maxabs;
  uint32_t nonfinite;
};
AnnoStats anno_stats(const double* v, uint64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Tries (trie.hip)
// ---------------------------------------------------------------------------
// A level's keys carry one sample per 2^LINE_SHIFT keys (one 128-byte
// line): samp[j] = keys[j << LINE_SHIFT].
constexpr uint32_t LINE_SHIFT = 5;

struct Level {
  uint64_t n = 0;            // nodes
  DBuf<uint32_t> keys;       // n
  DBuf<uint32_t> samp;       // ceil(n / 32): first key of every 32
  DBuf<uint32_t> offs;       // n+1: children in the next level; last level: run offsets
  uint64_t n_sets = 0;       // sets at this level (1 at level 0, else nodes of level-1)
  DBuf<uint64_t> bs_word;    // n_sets: first word in pool, UINT64_MAX = uint layout
  DBuf<uint32_t> bs_base;    // n_sets: value of bit 0 (multiple of 64)
  DBuf<uint64_t> pool;       // bitset words
  uint64_t pool_words = 0;
  // rank directory of the bitset sets (levels whose positions are used):
  // bs_rank[w] = set bits in the pool before word w, bs_delta[s] = first
  // position of set s minus bs_rank of its first word (mod 2^32)
  DBuf<uint32_t> bs_rank;    // pool_words + 1, or empty
  DBuf<uint32_t> bs_delta;   // n_sets, or empty
  uint64_t n_bitsets = 0;
};

}  // namespace lh

struct lh_trie {
  uint32_t magic;
  uint32_t n_levels = 0;
  uint32_t flags = 0;
  uint64_t n_input = 0;      // input rows
  uint64_t n_rows = 0;       // rows kept (bag: all; set: distinct)
  uint32_t level_order[LH_MAX_KEYS];   // input key column of each level
  uint32_t key_bits[LH_MAX_KEYS];      // significant bits per level
  uint32_t key_max[LH_MAX_KEYS];       // largest key per level
  // column statistics (learned order features), computed on first use
  bool col_stats = false;
  uint64_t col_distinct[LH_MAX_KEYS];  // distinct values of each level's column (kept rows)
  uint64_t col_freq_max[LH_MAX_KEYS];  // largest number of kept rows sharing one value
  lh::Level lv[LH_MAX_KEYS];
  // root index: level 0's keys as a bitmap over [0, root_span) with a rank
  // per 64-bit word, when the span is small next to the keys (membership
  // and position in one load each, whatever level 0's layout)
  uint64_t root_span = 0;
  lh::DBuf<uint64_t> root_bits;
  lh::DBuf<uint32_t> root_rank;
  // two-level tries whose column statistics were taken: the rows sorted by
  // (level 1, level 0), as level-1 and level-0 keys
  lh::DBuf<uint32_t> tsorted[2];
  // rows in trie order (bag: every row; set: one per distinct tuple), per
  // level; a set's last level is not kept here (its rows' last keys are
  // that level's keys): read columns through lh::row_keys
  lh::DBuf<uint32_t> skeys[LH_MAX_KEYS];
  std::vector<lh::DBuf<double>> annos;      // per annotation column
  std::vector<lh::DBuf<uint32_t>> meta;     // per meta column
  std::vector<lh::AnnoStats> astats;
};

namespace lh {

// Level l's column of the trie's rows, in trie order.
inline const uint32_t* row_keys(const lh_trie* t, uint32_t l) {
  return (!(t->flags & LH_BAG) && l + 1 == t->n_levels) ? t->lv[l].keys.p : t->skeys[l].p;
}

constexpr uint32_t TRIE_MAGIC = 0x54524945u;
constexpr uint32_t PLAN_MAGIC = 0x504c414eu;
constexpr uint32_t RESULT_MAGIC = 0x52534c54u;

// Build from device columns, optionally restricted to the rows listed in
// `sel` (n_sel entries).  Columns are in the relation's own column order;
// level_order maps levels to key columns.
// sorted_tail: the input rows (after `sel`) are already in lexicographic
// order of the last sorted_tail levels, which then need no sort passes.
// detect_sorted (with sorted_tail 0): find that tail with one pass over the
// key columns first.
lh_trie* build_trie(uint64_t n_rows, uint32_t n_keys, const uint32_t* const* keys,
                    uint32_t n_annos, const double* const* annos, uint32_t n_meta,
                    const uint32_t* const* meta, const uint32_t* level_order, uint32_t flags,
                    const uint32_t* sel, uint64_t n_sel, hipStream_t s, uint32_t sorted_tail = 0,
                    bool detect_sorted = false);

// Column statistics (col_distinct, col_freq_max), computed once per trie.
void ensure_column_stats(lh_trie* t, hipStream_t s);

// Sets of level l stored as bitsets (a device count).
uint64_t count_bitsets(const lh_trie* t, uint32_t l, hipStream_t s);

// Per-set layout and bitset materialization for one level.
void build_layouts(lh_trie* t, uint32_t level, uint32_t layout_flags, const uint32_t* parent, hipStream_t s);

// Per-set layout choices from the registered learned layout model (0 plain
// rule, 1 uint, 2 bitset); false when no model is registered.
bool learned_layout_choices(const lh_trie* t, uint32_t level, hipStream_t s, DBuf<uint8_t>& choice);

}  // namespace lh

namespace lh {

// ---------------------------------------------------------------------------
// Opt-in kernel timing (hipEvent pairs on the launching stream).
// ---------------------------------------------------------------------------
bool prof_enabled();
struct ProfScope {
  const char* name;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uint64_t rows, elems;
  ProfScope(const char* n, hipStream_t st, uint64_t r = 0, uint64_t el = 0);
  ~ProfScope();
};

}  // namespace lh
