/*
 * Join-aggregate oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU evaluation of an aggregate-join query
 * over annotated relations.  It is used by the test-suite, by the smoke check
 * and by the CPU-baseline leg of the benchmark, and by nothing else: the
 * GPU library never links, loads or calls it, and it shares no code,
 * header or constant with the GPU library.
 *
 * What it computes (paper, section 2.3 "Capturing Aggregate-Join Queries"):
 * the query is a hypergraph whose vertices are key attributes and whose
 * hyperedges are relations; every tuple carries an annotation from a
 * commutative semiring; joining multiplies annotations and the aggregation
 * ordering sums them over every attribute that is not in the output.
 *
 *     Q(o) = SUM over t in sigma(R_1) |x| ... |x| sigma(R_m) with pi_O(t) = o
 *              of PROD_e ann_e(t|e)
 *
 * with (+,x) over the reals for SUM and over the naturals with every
 * annotation equal to 1 for COUNT.  Filters follow section 2.1 (equality on
 * keys, ranges on annotations) widened to equality/ranges on non-key
 * ("meta") columns as the TPC-H Q5 example of section 3.1 filters a metadata
 * attribute.  GROUP BY on non-key columns follows section 5.
 *
 * How: a pairwise hash join, left-deep in atom declaration order (a hash
 * table is built on each next atom keyed by its attributes shared with the
 * running intermediate and probed by the intermediate), followed by hash
 * aggregation keyed by the output attributes and group columns.  This is
 * deliberately NOT the paper's Generic-Join (Algorithm 1), so agreement
 * between the two is evidence.  The probe side of each join is split over
 * OpenMP threads; each keeps its own intermediate tuples and its own
 * aggregation table, and the tables are merged at the end.  Counts and
 * exact accumulators are integers, so the merge does not depend on the
 * order and the result is the same for any thread count.
 *
 * SUM semantics: every term (the product of the tuple's non-identity
 * annotations) is added EXACTLY into a 512-bit fixed-point accumulator with
 * least significant bit 2^-256, and the sum is rounded once to the nearest
 * double (ties to even).  A term with one factor is that factor; with two it
 * is the exact product; with m >= 3 factors the first m-1 are multiplied
 * left to right in atom order with rounding and the last multiplication is
 * exact.  A term that does not fit the accumulator's window sets
 * ORC_E_RANGE.
 *
 * Bag semantics: a relation flagged bag keeps every input row as its own
 * tuple.  A set relation is deduplicated on its key tuple first and may
 * carry no annotation or meta column.
 */
#ifndef LH_ORACLE_H
#define LH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_NOMEM = 2, ORC_E_RANGE = 3 };
enum { ORC_COUNT = 0, ORC_SUM = 1 };
enum { ORC_EQ_KEY = 0, ORC_EQ_META = 1, ORC_RANGE_ANNO = 2, ORC_RANGE_META = 3 };

typedef struct {
  uint64_t n_rows;
  uint32_t n_keys;
  const uint32_t* const* keys;   /* n_keys host columns of n_rows */
  const uint32_t* attr_of_key;   /* query attribute of each key column */
  uint32_t n_annos;
  const double* const* annos;    /* annotation columns */
  uint32_t n_meta;
  const uint32_t* const* meta;   /* non-key, non-aggregated columns */
  int32_t anno;                  /* annotation multiplied in (SUM); -1 = identity */
  uint32_t bag;                  /* 1 = bag (keep duplicates), 0 = set */
} orc_atom;

typedef struct {
  uint32_t atom, kind, col, eq;  /* kind: ORC_EQ_KEY/EQ_META/RANGE_ANNO/RANGE_META */
  double lo, hi;                 /* half-open [lo, hi) for the range kinds */
} orc_filter;

typedef struct { uint32_t atom, meta_col; } orc_group;

typedef struct {
  uint32_t n_attrs;              /* 1..64 */
  uint32_t n_atoms;
  const orc_atom* atoms;
  uint32_t n_out;                /* n_out + n_group <= 128 */
  const uint32_t* out_attrs;
  uint32_t n_group;
  const orc_group* groups;
  uint32_t agg;                  /* ORC_COUNT or ORC_SUM */
  uint32_t n_filters;
  const orc_filter* filters;
} orc_query;

typedef struct {
  uint64_t n_rows;               /* output rows, sorted ascending by key */
  uint32_t n_cols;               /* n_out + n_group */
  uint32_t* keys;                /* n_rows x n_cols, row-major */
  uint64_t* counts;              /* contributing full-join tuples per row */
  double* sums;                  /* SUM only, else NULL */
  uint64_t n_join_tuples;        /* full-join tuples aggregated */
  uint64_t n_intermediate;       /* largest materialized intermediate */
} orc_result;

int orc_join_aggregate(const orc_query* q, orc_result* out);
/* Threads of the probe side: n > 0 fixes the count, 0 restores the OpenMP
 * default; orc_threads() returns the count the next call will use. */
void orc_set_threads(int n);
int orc_threads(void);
void orc_result_free(orc_result* r);

/* Exact sum of products: SUM_i a[i]*b[i] (b == NULL: SUM_i a[i]) rounded
 * once to the nearest double.  *status gets ORC_OK or ORC_E_RANGE. */
double orc_exact_dot(const double* a, const double* b, uint64_t n, int* status);

#ifdef __cplusplus
}
#endif
#endif
