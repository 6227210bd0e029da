// Plans and results: host-side objects shared by the planner, the join
// executor and the C ABI.
#pragma once

#include <memory>
#include <vector>

#include "lh_internal.h"

namespace lh {

constexpr int MAXA = 8;    // atoms per query
constexpr int MAXP = 8;    // participants per attribute
constexpr int MAXV = 16;   // attributes per query

// Intersection algorithm of an attribute position.  The plan records
// ALG_PROBE; the two-set leaf refines it per row (k_work): two bitsets may
// be ANDed word by word, two sorted sets of similar size merged.
enum LevelAlg : uint32_t {
  ALG_PROBE = 0,   // iterate the smallest set, probe the others (bit test or binary search)
  ALG_MERGE = 1,   // merge-path co-iteration of two uint sets (two-set leaf, per row)
  ALG_BSAND = 2,   // word-wise AND of two bitsets (two-set leaf, per row)
};

struct PlanAtom {
  const lh_trie* trie = nullptr;      // trie used by the plan
  lh_trie* owned = nullptr;           // plan-owned copy (filtered or re-ordered)
  uint32_t n_levels = 0;
  uint32_t attr_of_level[LH_MAX_KEYS];
  int32_t anno = -1;                  // annotation column in the trie (SUM); -1 identity
  bool bag = false;
  uint64_t card = 0;                  // base cardinality (rows before filters)
  bool has_eq_filter = false;
};

// A product handed to BLAS (completely dense relations, LH_DENSE_BLAS):
// output (rows x cols) = a (rows x inner) . b (inner x cols), both row-major
// in trie order unless marked as stored transposed.
struct DensePlan {
  const double* a = nullptr;
  const double* b = nullptr;
  uint32_t rows = 0, cols = 0, inner = 0;
  bool a_trans = false, b_trans = false;
};

struct Participant {
  uint32_t atom;
  uint32_t level;  // trie level holding this attribute
};

}  // namespace lh

struct lh_plan_s {
  uint32_t magic = lh::PLAN_MAGIC;
  uint32_t n_attrs = 0;
  std::vector<lh::PlanAtom> atoms;
  uint32_t order[lh::MAXV];                 // attribute at each depth
  uint32_t depth_of[lh::MAXV];              // depth of each attribute
  std::vector<std::vector<lh::Participant>> parts;  // per depth
  std::vector<uint32_t> out_attrs;
  std::vector<lh_group_col> groups;         // atom index refers to plan atoms
  uint32_t agg = LH_AGG_COUNT;
  uint32_t policy = LH_POLICY_PLAIN;
  bool case_prefix = false;                 // outputs = first n_out attributes of the order
  bool case_full = false;                   // COUNT, every attribute an output, no GROUP BY meta column
  uint32_t group_impl = 0;                  // GROUP BY outside the prefix: 0 auto, 1 sort, 2 hash, 3 dense
  bool want_parts = false;                  // SUM: also hand out each sum's exact parts (multi-node plans)
  uint32_t blas = 0;                        // 1: BLAS matrix-vector, 2: matrix-matrix (dense relations)
  lh::DensePlan dense;
  int32_t exact_lsb = 0;
  uint32_t exact_digits = 0;
  double cost = 0.0;
  uint32_t level_alg[lh::MAXV];
  std::vector<lh_trie*> reordered;          // re-sorted tries, shared by atoms over the same relation
  ~lh_plan_s() {
    for (auto& a : atoms)
      if (a.owned) delete a.owned;
    for (lh_trie* t : reordered) delete t;
  }
};

struct lh_result_impl {
  lh_result pub;                            // must stay first
  uint32_t magic = lh::RESULT_MAGIC;
  std::vector<lh::DBuf<uint32_t>> cols;
  std::vector<const uint32_t*> colptr;
  lh::DBuf<uint64_t> counts;
  lh::DBuf<double> sums;
  lh::DBuf<double> parts;                   // want_parts: EXACT_PARTS doubles per row summing exactly to the sum
  std::shared_ptr<void> shared;             // batched results share one output block
};

namespace lh {

lh_plan_t* make_plan(const lh_query* q, hipStream_t s);
lh_result_impl* run_plan(const lh_plan_t* p, hipStream_t s);
// run_plan with every temporary in the static scratch (noalloc.hip); the
// result's rows go to the caller's buffers.  Returns the row count.
uint64_t run_plan_noalloc(const lh_plan_t* p, hipStream_t s, uint64_t max_rows, uint32_t* const* out_keys,
                          uint64_t* counts, double* sums, uint64_t* peak_bytes);
// Dense relations under LH_DENSE_BLAS: mark the plan for a BLAS product.
void plan_dense(const lh_query* q, lh_plan_t* p, hipStream_t s);
lh_result_impl* run_dense(const lh_plan_t* p, hipStream_t s);

// Feature encoding of a join result and logistic regression on tries
// (ml.hip); the C ABI's lh_encode and lh_logreg_fit after validation.
uint32_t encode_features(uint64_t n, uint32_t n_id_cols, const uint32_t* const* ids, uint32_t row_col,
                         uint32_t n_cols, const lh_feature_col* cols, uint32_t bias, uint32_t* out_row,
                         uint32_t* out_feat, double* out_val, hipStream_t s);
void logreg_fit(const lh_trie* x_rows, const lh_trie* x_cols, uint32_t anno, const double* y, uint64_t n_y,
                uint32_t n_feat, uint32_t iters, double step, double* w, double* loss, hipStream_t s);
// Batched execution of many plans; returns false (and does nothing) when
// the plans are not all of a shape the batched executor handles.
bool run_batch(lh_plan_t* const* plans, uint32_t n, hipStream_t s, std::vector<lh_result_impl*>& out);
// Row-union shape: A(i,j) with E(j) (SpMV) or E(j,k) (SpGEMM), order i,j[,k].
int row_union_kind(const lh_plan_t* p);
// Drop the cached batch (and its graph) if it refers to this plan.
void batch_forget_plan(const lh_plan_t* p);
void free_trie(lh_trie* t);

}  // namespace lh
