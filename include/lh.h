/*
 * lh.h -- generic (worst-case optimal) join with aggregation over
 * dictionary-encoded uint32 tries, on one AMD Instinct MI355X (gfx950).
 *
 * The library follows the paper's statement of the problem:
 *  - relations whose attributes are KEYS (joinable, dictionary encoded as
 *    uint32, never aggregated) or ANNOTATIONS (aggregable; here FP64), with
 *    other non-key columns kept as uint32 META columns (section 2.1, "Data
 *    Model"; Rule 4 of section 3.1 keeps non-aggregated attributes in a
 *    metadata container);
 *  - one trie per relation over its key attributes, each level a collection
 *    of sets stored as sorted uint arrays or as bitsets, with annotation
 *    buffers reachable from the last level (section 2.2, "Storage Engine");
 *  - a query hypergraph whose vertices are attributes and whose hyperedges
 *    are relations (section 2.3, "Representing Queries as Hypergraphs");
 *  - aggregation over a commutative semiring, multiplying annotations on
 *    join and summing them over the attributes that are not output (section
 *    2.3, "Capturing Aggregate-Join Queries");
 *  - evaluation one attribute at a time by the generic worst-case optimal
 *    join (Algorithm 1, section 2.4), with the attribute order chosen by the
 *    cost-based optimizer of section 4 unless the caller fixes it.
 *
 * Memory: every column pointer handed IN is a DEVICE pointer (HIP); every
 * descriptor array (the arrays of column pointers, attribute maps, orders,
 * filters) is a HOST array.  Inputs are borrowed: each call finishes its
 * device work (it synchronizes the given stream) before it returns, so the
 * caller may release input buffers as soon as a call returns.  Tries,
 * plans and results own their device memory until lh_free.  A plan borrows
 * the tries its atoms name; they must outlive it.  A result does not
 * reference its plan.
 *
 * Errors: every call returns lh_status; on any error *out is set to NULL
 * and nothing is leaked.  lh_last_error() returns a thread-local message
 * for the last failing call.  A handle must not be used from two host
 * threads at once.  The stream argument is a hipStream_t (NULL = the null
 * stream).
 */
#ifndef LH_H
#define LH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LH_OK = 0,
  LH_ERR_INVALID = 1,      /* a NULL pointer, a bad size, id or permutation */
  LH_ERR_OOM = 2,          /* device allocation failed */
  LH_ERR_DEVICE = 3,       /* any other HIP runtime error */
  LH_ERR_UNSUPPORTED = 4,  /* valid request outside what this build supports */
  LH_ERR_OVERFLOW = 5      /* a size or count exceeds its index type */
} lh_status;

/* ---- relation flags (lh_relation_desc.flags) ---------------------------- */
#define LH_SET            0x00u  /* key tuples form a set: duplicates removed; no annos/meta */
#define LH_BAG            0x01u  /* every row is its own tuple (duplicates kept) */
#define LH_LAYOUT_PLAIN   0x00u  /* bitset iff (max-min+1) <= 32*card, per set */
#define LH_LAYOUT_UINT    0x10u  /* every set a sorted uint array */
#define LH_LAYOUT_BITSET  0x20u  /* every set whose window fits also a bitset */
#define LH_LAYOUT_LEARNED 0x30u  /* per-set choice by the learned cost model */
#define LH_LAYOUT_MASK    0x30u

#define LH_MAX_KEYS 8

typedef struct lh_trie lh_trie;
typedef struct lh_plan_s lh_plan_t;

/* One relation as a column store (section 2.1).  keys/annos/meta are HOST
 * arrays of DEVICE column pointers, each column n_rows long. */
typedef struct {
  uint64_t n_rows;
  uint32_t n_keys;                  /* 1..LH_MAX_KEYS key columns */
  const uint32_t* const* keys;      /* dictionary-encoded key columns */
  uint32_t n_annos;
  const double* const* annos;       /* FP64 annotation columns */
  uint32_t n_meta;
  const uint32_t* const* meta;      /* uint32 non-key columns (filters, GROUP BY) */
  const uint32_t* level_order;      /* host: key column of trie level l; NULL = identity */
  uint32_t flags;                   /* LH_SET|LH_BAG  |  LH_LAYOUT_* */
} lh_relation_desc;

/* Build the trie of one relation (section 2.2): a stable lexicographic
 * radix sort of the key tuples in level order, per-level keys and child
 * offsets, set-mode deduplication or bag-mode runs, a per-set uint/bitset
 * layout, and the annotation and meta columns gathered into trie order.
 * Errors: LH_ERR_INVALID for NULL pointers, n_keys outside 1..8, a
 * level_order that is not a permutation, or a set relation with annotation
 * or meta columns; LH_ERR_OVERFLOW if n_rows >= 2^32. */
lh_status lh_trie_build(const lh_relation_desc* rel, void* hip_stream, lh_trie** out);

/* ---- queries ------------------------------------------------------------ */
#define LH_AGG_COUNT 0u
#define LH_AGG_SUM   1u

#define LH_EQ_KEY     0u  /* key column == eq          (section 2.1) */
#define LH_EQ_META    1u  /* meta column == eq         */
#define LH_RANGE_ANNO 2u  /* lo <= annotation < hi     (section 2.1) */
#define LH_RANGE_META 3u  /* lo <= meta column < hi    */

#define LH_POLICY_PLAIN   0x0u  /* section 4 cost rule picks order and per-level algorithms */
#define LH_POLICY_LEARNED 0x1u  /* learned cost model picks; the plain rule is its fallback */
#define LH_POLICY_FIXED   0x2u  /* caller's attr_order, plain per-level algorithms */
#define LH_POLICY_MASK    0x3u
/* GROUP BY whose keys are not a prefix of the attribute order (section 5),
 * or'ed into lh_query.policy: the key union and the GROUP BY on meta
 * columns.  AUTO takes DENSE when the key space (the product of each output
 * column's largest value + 1) is at most 4x the leaf's work or 2^16, and
 * fits 2^27 entries; else HASH.  SORT materializes every tuple and sorts;
 * HASH upserts into a device-wide open-addressing table (grown and rerun
 * when the estimate of its size was short); DENSE adds into an array over
 * the key space.  Results are identical whichever runs. */
#define LH_GROUP_AUTO     0x00u
#define LH_GROUP_SORT     0x10u
#define LH_GROUP_HASH     0x20u
#define LH_GROUP_DENSE    0x30u
#define LH_GROUP_MASK     0x30u
/* Dense LA by attribute elimination (sections 3.1, 6.2.2), or'ed into
 * lh_query.policy: a SUM over two annotated, completely dense relations
 * (every key tuple of [0,R) x [0,K) present once) sharing one attribute,
 * grouped by the other attributes (matrix-vector: outputs r of M(r,j),
 * x(j); matrix-matrix: outputs r, c of P(r,j), Q(j,c), either key order in
 * storage), is computed by rocBLAS DGEMV / DGEMM over the annotation
 * buffers in trie order.  Keys and counts are those of the join; sums are
 * BLAS sums (exact = 0).  Other queries ignore the bit. */
#define LH_DENSE_BLAS     0x40u

/* A hyperedge: one relation's trie and the query attribute of each of its
 * key columns (columns mapping to one attribute are equi-joined, Rule 1 of
 * section 3.1). */
typedef struct {
  const lh_trie* trie;
  const uint32_t* attr_of_key;  /* host, n_keys entries, distinct, < n_attrs */
  int32_t anno;                 /* annotation column multiplied in for SUM; -1 = identity */
} lh_atom;

typedef struct {
  uint32_t atom, kind, col;     /* kind: LH_EQ_KEY / LH_EQ_META / LH_RANGE_ANNO / LH_RANGE_META */
  uint32_t eq;
  double lo, hi;                /* half-open [lo, hi) */
} lh_filter;

typedef struct { uint32_t atom, meta_col; } lh_group_col;  /* GROUP BY a meta column (section 5) */

typedef struct {
  uint32_t n_attrs;                 /* query attributes 0..n_attrs-1 (<= 16) */
  uint32_t n_atoms;                 /* hyperedges (<= 8) */
  const lh_atom* atoms;
  uint32_t n_out;                   /* materialized key attributes, in output order */
  const uint32_t* out_attrs;
  uint32_t n_group;                 /* extra GROUP BY meta columns */
  const lh_group_col* group_cols;
  uint32_t agg;                     /* LH_AGG_COUNT or LH_AGG_SUM */
  uint32_t n_filters;
  const lh_filter* filters;
  const uint32_t* attr_order;       /* host permutation of the attributes; NULL = optimizer */
  uint32_t policy;                  /* LH_POLICY_* */
} lh_query;

/* Plan a query: validate it, apply the filters to private copies of the
 * filtered relations (selections pushed below the join, section 3.2),
 * choose the attribute order by the cost estimate of section 4 (sum over
 * attributes of icost x weight; materialized attributes first, with the
 * one-swap relaxation of section 4.1.2), rebuild any trie whose level order
 * does not follow that order, and fix the per-level intersection algorithm
 * and the exact-summation window.
 * Errors: LH_ERR_INVALID (NULL, ids out of range, repeated attribute in an
 * atom, attribute in no atom, non-permutation attr_order, filter column out
 * of range, SUM without an annotated atom); LH_ERR_UNSUPPORTED (an
 * aggregate other than COUNT/SUM, a non-finite annotation, or annotation
 * values whose exact products do not fit the 256-bit accumulator).
 * SUM terms: one annotated atom gives its value; with m >= 2 the first m-1
 * factors (atom order) are multiplied with rounding and the last product is
 * exact; every term is summed exactly and the sum rounded once (ties to
 * even). */
lh_status lh_plan(const lh_query* q, void* hip_stream, lh_plan_t** out);

/* Result of one plan.  out_keys is a HOST array of n_cols DEVICE columns
 * (the n_out output attributes in declared order, then the n_group group
 * columns), n_rows long, rows sorted ascending lexicographically.  counts
 * is the number of contributing join tuples per row (always present); sums
 * (SUM only) is the exact sum of annotation products rounded once to the
 * nearest double.  An ungrouped query has exactly one row. */
typedef struct lh_result {
  uint64_t n_rows;
  uint32_t n_cols;
  const uint32_t* const* out_keys;
  const uint64_t* counts;
  const double* sums;
  uint32_t exact;                   /* 1: sums are correctly rounded exact sums */
  uint64_t n_join_tuples;           /* full-join tuples aggregated */
  uint32_t group_impl;              /* how rows were grouped: 0 streamed (prefix or one group), 1 sort,
                                       2 hash, 3 dense */
} lh_result;

/* Run plans (Algorithm 1 per plan).  n_plans > 1 runs them as one batch:
 * the batched executor puts every instance's work into one persistent,
 * graph-captured launch where the plans allow it; results are identical to
 * running them one at a time.  out receives n_plans result handles.
 * Errors: LH_ERR_INVALID for NULL arguments or n_plans == 0. */
lh_status lh_join_aggregate(lh_plan_t* const* plans, uint32_t n_plans, void* hip_stream,
                            lh_result** out);

/* ---- a join that allocates no device memory -------------------------------
 * For callers that cannot allocate device memory: tight serving loops and
 * harnesses that forbid allocation around their calls.  It runs one plan as
 * lh_join_aggregate does (same kernels, identical results) but takes every
 * temporary from a static device array of LH_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends, and writes
 * the result into the caller's buffers instead of an lh_result.  It calls
 * no hipMalloc, hipFree or allocating library routine.  All calls on one
 * GPU share that GPU's array: calls that overlap on one GPU (other host
 * threads, other streams) race and must be serialized by the caller.
 *
 * out_keys: HOST array of n_cols DEVICE columns (n_cols = the plan's n_out
 * + n_group), each with room for max_rows uint32; counts: DEVICE, max_rows
 * uint64; sums: DEVICE, max_rows doubles (SUM plans; ignored and may be NULL
 * for COUNT); *n_rows (HOST) receives the number of rows written, in the
 * order and format of lh_result.  The plan comes from lh_plan as usual.
 * Errors: LH_ERR_INVALID for NULL arguments or a plan that is not live;
 * LH_ERR_UNSUPPORTED for a plan run by BLAS (LH_DENSE_BLAS); LH_ERR_OVERFLOW
 * when the join's temporaries do not fit the scratch or the result has more
 * than max_rows rows (outputs are then unspecified); the errors of
 * lh_join_aggregate otherwise. */
#define LH_NOALLOC_SCRATCH_BYTES (64u << 20)
lh_status lh_join_aggregate_noalloc(const lh_plan_t* plan, void* hip_stream, uint64_t max_rows,
                                    uint32_t* const* out_keys, uint64_t* counts, double* sums, uint64_t* n_rows);

/* Release an lh_trie*, lh_plan* or lh_result*.  NULL is a no-op. */
void lh_free(void* handle);

/* Message of the last failing call on this host thread ("" if none). */
const char* lh_last_error(void);

/* ---- inspection helpers (tests, tools) ---------------------------------- */

typedef struct {
  uint32_t n_levels;
  uint64_t n_rows;                  /* rows kept: distinct tuples (set) or all rows (bag) */
  uint64_t level_size[LH_MAX_KEYS];     /* nodes per level */
  uint64_t level_sets[LH_MAX_KEYS];     /* sets per level (level 0: 1) */
  uint64_t level_bitsets[LH_MAX_KEYS];  /* sets stored as bitsets */
  uint64_t level_words[LH_MAX_KEYS];    /* 64-bit bitset words per level */
  uint32_t level_order[LH_MAX_KEYS];
  uint64_t col_distinct[LH_MAX_KEYS];   /* distinct values of each level's column */
  uint64_t col_freq_max[LH_MAX_KEYS];   /* most rows sharing one value of it */
} lh_trie_info;

lh_status lh_trie_get_info(const lh_trie* t, lh_trie_info* info);

/* Copy level l to host buffers: keys (level_size[l] entries), offs
 * (level_size[l]+1 entries; NULL allowed; for the last level these are the
 * run offsets into the sorted rows in bag mode, else 0..n).  Either buffer
 * may be NULL. */
lh_status lh_trie_read_level(const lh_trie* t, uint32_t level, uint32_t* keys, uint32_t* offs);

/* Copy a result to host buffers of n_rows entries each (n_cols key
 * buffers); any pointer may be NULL. */
lh_status lh_result_read(const lh_result* r, uint32_t* const* keys, uint64_t* counts, double* sums);

typedef struct {
  uint32_t n_attrs;
  uint32_t attr_order[16];
  double cost;                      /* the section 4 estimate of the chosen order */
  uint32_t case_prefix;             /* 1: output is a prefix of the order (streamed groups) */
  uint32_t exact_digits;            /* 32-bit digits of the exact accumulator (0: COUNT) */
  int32_t exact_lsb;                /* exponent of the accumulator's least significant bit */
  uint32_t level_alg[16];           /* intersection algorithm per attribute position: 0 probe (the
                                       two-set leaf may still AND two bitsets or merge two sorted
                                       sets of similar size, row by row) */
  uint32_t blas;                    /* 1: run as BLAS DGEMV, 2: as DGEMM (LH_DENSE_BLAS), else 0 */
} lh_plan_info;

lh_status lh_plan_get_info(const lh_plan_t* p, lh_plan_info* info);

/* ---- the section 4 cost estimate on a bare hypergraph (host only) ------- */

/* Edge e has edge_attr_count[e] attributes, listed consecutively in
 * edge_attrs; edge_card is its cardinality (the score of section 4.2 is
 * ceil(card / heaviest card * 100)); edge_eq marks an equality selection on
 * the relation (its vertices then take the heaviest score, else the
 * lightest); edge_dense marks a completely dense relation, which adds no
 * intersection (section 4.1.1).  edge_eq / edge_dense may be NULL. */
typedef struct {
  uint32_t n_attrs, n_edges;
  const uint32_t* edge_attr_count;
  const uint32_t* edge_attrs;
  const uint64_t* edge_card;
  const uint32_t* edge_eq;
  const uint32_t* edge_dense;
  /* optional, aligned with edge_attrs (attributes listed in trie level
   * order): log2(1 + mean) and log2(1 + largest) number of rows sharing one
   * value of that attribute's column; used by lh_order_features only */
  const float* edge_attr_lf_mean;
  const float* edge_attr_lf_max;
} lh_hypergraph;

/* cost = SUM_i icost(order[i]) * weight(order[i]) (section 4); icost and
 * weight (n_attrs entries each, may be NULL) receive the per-position
 * values.  icost follows the layout guess of Crucial Observation 1 with
 * bs&bs = 1, bs&uint = 10, uint&uint = 50, N-way sums with bitsets first,
 * and 0 for an attribute in a single (non-dense) relation. */
lh_status lh_order_cost(const lh_hypergraph* h, const uint32_t* order, uint32_t* icost, uint32_t* weight,
                        double* cost);

/* The optimizer's choice: the cheapest order with the n_out materialized
 * attributes first, plus the one-swap relaxation of section 4.1.2 (last
 * attribute projected away, second-to-last materialized, swap lowers the
 * icost); ties go to the lexicographically smallest order. */
lh_status lh_choose_order(const lh_hypergraph* h, uint32_t n_out, const uint32_t* out_attrs, uint32_t* order,
                          double* cost);

/* ---- multi-node plans: generalized hypertree decompositions ------------- */
#define LH_GHD_MAX_NODES 16

/* A GHD (section 2.3, "Generalized Hypertree Decompositions"): a tree of
 * nodes, each joining its hyperedges (the query's atoms) and the results of
 * its children, and handing its parent, per tuple of the attributes they
 * share, the aggregate over everything below (the annotation semiring of
 * section 2.3).  Every edge belongs to exactly one ordinary node; a node's
 * attributes chi are its edges' attributes.  A selection node (pushed = 1,
 * section 3.2) holds one filtered edge of its parent and evaluates the
 * selection before the parent joins it.  Node 0 is the root and
 * parent[t] < t for t > 0. */
typedef struct {
  uint32_t n_nodes;
  int32_t parent[LH_GHD_MAX_NODES];   /* -1 for the root */
  uint32_t edges[LH_GHD_MAX_NODES];   /* bit e: hyperedge e */
  uint32_t attrs[LH_GHD_MAX_NODES];   /* chi(t), bit v: attribute v (output) */
  uint32_t pushed[LH_GHD_MAX_NODES];  /* 1: a selection node */
  double node_fhw[LH_GHD_MAX_NODES];  /* fractional edge cover number of chi(t) by t's edges (output) */
  double fhw;                         /* width: the largest node_fhw over ordinary nodes (output) */
  uint32_t depth;                     /* longest root-to-leaf path in tree edges, ordinary nodes (output) */
  uint32_t shared;                    /* sum over tree edges of |chi(t) & chi(parent)| (output) */
  uint32_t sel_depth;                 /* sum of the depths of the nodes holding filtered edges (output) */
} lh_ghd;

/* Fractional edge cover number of the attributes of the edges in edge_mask
 * by those edges (the width of one GHD node, section 2.3).  Host only; the
 * hypergraph's edge_card may be NULL here. */
lh_status lh_ghd_fhw(const lh_hypergraph* h, uint32_t edge_mask, double* fhw);

/* Choose a GHD (section 3.2): least width, then fewest nodes, least depth,
 * fewest vertices shared between adjacent nodes, deepest selections, and
 * last (this library's addition) the least sum of node width x depth, so
 * that narrow nodes sit below wide ones and their results restrict the
 * wide joins, as nodes run bottom-up; a
 * decomposition of width 1 becomes a single node (section 2.3); then every
 * filtered edge in a node of two or more edges gets a selection node.  The
 * root holds every attribute in out_attrs and every edge flagged in
 * edge_root (GROUP BY meta columns live in root relations).  edge_sel and
 * edge_root (n_edges entries) may be NULL.  Host only; edge_card may be
 * NULL.  Errors: LH_ERR_INVALID for 0 or more than 8 edges or ids out of
 * range. */
lh_status lh_ghd_choose(const lh_hypergraph* h, const uint32_t* edge_sel, const uint32_t* edge_root,
                        uint32_t n_out, const uint32_t* out_attrs, lh_ghd* out);

/* The decomposition lh_ghd_join_aggregate would choose for q (its atoms'
 * attributes, filtered atoms, GROUP BY atoms and outputs).  Host only. */
lh_status lh_ghd_for_query(const lh_query* q, lh_ghd* out);

/* Run q under the decomposition g (NULL: the one lh_ghd_for_query gives).
 * Nodes run bottom-up, each as lh_plan + lh_join_aggregate over its edges
 * (with their filters) and its children's results, which become annotated
 * relations keyed by the attributes shared with the parent; the root groups
 * by the query's outputs.  The result has the single-plan layout: keys and
 * counts identical to lh_plan + lh_join_aggregate of q; for SUM, the sum is
 * rounded once per node instead of once overall, so exact = 0 when the
 * root has children.  Errors: those of lh_plan and lh_join_aggregate;
 * LH_ERR_INVALID for a g that is not a GHD of q (edge in no or two
 * ordinary nodes, running intersection broken, a child sharing no
 * attribute with its parent, outputs or GROUP BY atoms outside the root, a
 * selection node that does not hold one filtered edge of its parent);
 * LH_ERR_OVERFLOW when a count reaches 2^53. */
lh_status lh_ghd_join_aggregate(const lh_query* q, const lh_ghd* g, void* hip_stream, lh_result** out);

/* ---- a mixed SQL + ML pipeline (section 7) --------------------------------
 * The SQL phase is an ordinary query (lh_plan + lh_join_aggregate) whose
 * output columns identify, per result row, the rows of the tables it
 * joined.  lh_encode turns that result into the design matrix as (row,
 * feature, value) triples; lh_trie_build over them gives the matrix's tries,
 * and lh_logreg_fit trains on those tries directly. */
#define LH_ENC_MAX_IDS  8u
#define LH_ENC_MAX_COLS 32u

/* One source column of the encoding, read at ids[by][r] for result row r.
 * Exactly one of codes (categorical: one indicator feature per code) and
 * values (numeric: one feature carrying the value) is set. */
typedef struct {
  const uint32_t* codes;    /* DEVICE, n_ids codes, each < card; or NULL */
  const double* values;     /* DEVICE, n_ids values; or NULL */
  uint32_t card;            /* categorical: number of codes (>= 1) */
  uint32_t by;              /* which id column indexes this column (< n_id_cols) */
  uint64_t n_ids;           /* entries of codes / values */
} lh_feature_col;

/* Categorical feature encoding (section 7, the feature engineering phase).
 * Features are numbered in column order: the bias feature 0 (bias = 1),
 * then each column's block (card ids for a categorical column, one for a
 * numeric one).  Result row r (0 <= r < n) yields slots = bias + n_cols
 * triples, written at r * slots + k of the DEVICE outputs (n * slots
 * entries each): out_row = ids[row_col][r]; slot k = 0 of a biased
 * encoding is (feature 0, value 1); the slot of a categorical column is
 * (its base + code, 1), that of a numeric column (its base, value).
 * ids is a HOST array of n_id_cols DEVICE columns of n entries (e.g. an
 * lh_result's out_keys); cols is a HOST array.  *n_feat (host) receives
 * the number of features.  Errors: LH_ERR_INVALID for NULL arguments,
 * n_id_cols outside 1..8, more than 32 columns, row_col or by out of
 * range, a column with both or neither of codes and values, card 0, or,
 * found on the device, an id >= n_ids or a code >= card (the outputs are
 * then unspecified); LH_ERR_OVERFLOW for 2^32 features or more. */
lh_status lh_encode(uint64_t n, uint32_t n_id_cols, const uint32_t* const* ids, uint32_t row_col, uint32_t n_cols,
                    const lh_feature_col* cols, uint32_t bias, uint32_t* out_row, uint32_t* out_feat,
                    double* out_val, uint32_t* n_feat, void* hip_stream);

/* Logistic regression by full-batch gradient descent over a design matrix X
 * held as tries (section 7, the machine-learning phase): x_rows is the
 * two-level bag trie of (row, feature) with X's entries in annotation
 * column anno, x_cols the trie of the same relation with its levels
 * swapped (both from lh_trie_build; duplicate (row, feature) pairs add
 * up).  The n training rows are x_rows' level-0 keys.  y (DEVICE) holds
 * the label of row id r at y[r] (n_y entries); w (DEVICE, n_feat entries)
 * holds the initial weights and receives the final ones.  Each of iters
 * iterations computes z = X w, p = 1 / (1 + exp(-z)), g = X^T (p - y) / n
 * and w = w - step * g.  loss (DEVICE, iters entries, may be NULL)
 * receives the mean log-loss, log(1 + exp(z)) - y z, at the start of each
 * iteration.  Sums run in a fixed order, so results repeat exactly.  No
 * training rows: w is unchanged and each loss is 0.  Errors: LH_ERR_INVALID
 * for NULL arguments, tries that are not two-level bag tries with column
 * anno, level orders that are not swapped, different row counts, a row id
 * >= n_y or a feature id >= n_feat. */
lh_status lh_logreg_fit(const lh_trie* x_rows, const lh_trie* x_cols, uint32_t anno, const double* y, uint64_t n_y,
                        uint32_t n_feat, uint32_t iters, double step, double* w, double* loss, void* hip_stream);

/* Device allocations currently held by the library (leak checks). */
long lh_live_allocations(void);

/* ---- opt-in kernel timing ------------------------------------------------
 * When enabled, the library brackets its kernel launches with hipEvents on
 * the launching stream and aggregates them per kernel name: launches, total
 * milliseconds, and the rows / flattened set elements the launches
 * processed (the units of the algorithmic-bytes formulas). */
typedef struct {
  char name[48];
  uint64_t launches;
  double total_ms;
  uint64_t rows;
  uint64_t elements;
} lh_profile_entry;

/* ---- the learned cost model ----------------------------------------------
 * A 3-layer perceptron d_in -> 64 -> 64 -> 1 (ReLU) predicting log2 of a
 * cost.  Training runs FP32 forward, backward and Adam kernels on the GPU;
 * inference for decisions runs a BF16 kernel (bf16 weights and activations,
 * fp32 sums).  Parameters are packed fp32: W1 (64 x d_in), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1), row-major.  All arrays below
 * are HOST arrays; X is n x d_in row-major.
 *
 * Two decisions can use a registered model (lh_use_model); without one they
 * follow the plain rules of section 4, which also remain the yardstick of the
 * model's regret.  Join results never depend on these choices.
 *  LH_MODEL_LAYOUT: per-set layout at lh_trie_build with LH_LAYOUT_LEARNED
 *    (sets of 32+ elements); features [log2 card, log2 span, log2(card/span),
 *    choice (0 uint, 1 bitset)], target log2(ns per probe).
 *  LH_MODEL_ORDER: attribute order at lh_plan with LH_POLICY_LEARNED;
 *    features from lh_order_features, target log2(plan + join time). */
typedef struct lh_mlp lh_mlp;
#define LH_MODEL_LAYOUT 0u
#define LH_MODEL_ORDER  1u
#define LH_LAYOUT_FEATURES 4u
#define LH_ORDER_FEATURES 24u

lh_status lh_mlp_create(uint32_t d_in, uint32_t width, uint64_t seed, lh_mlp** out);  /* width must be 64 */
void lh_mlp_free(lh_mlp* m);
uint64_t lh_mlp_num_params(const lh_mlp* m);
lh_status lh_mlp_get_params(const lh_mlp* m, float* params);
lh_status lh_mlp_set_params(lh_mlp* m, const float* params);
/* FP32 forward + backward of one batch: mean of (p - y)^2 / 2 and the
 * packed gradient (num_params floats; may be NULL). */
lh_status lh_mlp_loss_grad(const lh_mlp* m, const float* X, const float* y, uint32_t n, void* hip_stream,
                           float* loss, float* grad);
/* Adam (beta 0.9 / 0.999) over shuffled minibatches for `epochs` epochs. */
lh_status lh_mlp_train(lh_mlp* m, const float* X, const float* y, uint32_t n, uint32_t epochs, uint32_t batch,
                       float lr, uint64_t seed, void* hip_stream, float* final_loss);
/* Predictions y (n floats); bf16 = 1 uses the BF16 inference kernel. */
lh_status lh_mlp_predict(const lh_mlp* m, const float* X, uint64_t n, uint32_t bf16, void* hip_stream, float* y);
/* Register m (or NULL) for a decision; the model must outlive its use. */
lh_status lh_use_model(uint32_t slot, const lh_mlp* m);
/* LH_ORDER_FEATURES floats describing an attribute order: for each of the
 * first 4 positions the section 4 icost / 50, log2(1 + weight), and over
 * the relations holding the attribute the smallest and largest log2 mean
 * size and the largest log2 maximum size of the set each offers there
 * (root set: distinct values; else rows per value of the attribute bound
 * just before in that relation); then log2(1 + rows of relations the order
 * forces to re-sort, their edge attributes being listed in trie level
 * order), log2(1 + all rows), the attribute count and log2(1 + the section
 * 4 cost). */
lh_status lh_order_features(const lh_hypergraph* h, const uint32_t* order, float* features);

void lh_profile_enable(int on);
void lh_profile_reset(void);
/* Writes up to max_entries entries; returns the number of kernels seen. */
uint32_t lh_profile_read(lh_profile_entry* out, uint32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif /* LH_H */
