/*
 * Join-aggregate oracle: TEST INFRASTRUCTURE ONLY (see oracle.h for what it
 * computes and why it is shaped as it is).  Plain C with OpenMP over the
 * probe side of each join (thread-local intermediates and aggregation
 * tables, merged exactly), built with -ffp-contract=off so no multiply is
 * fused behind the reader's back.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------
 * Exact fixed-point accumulator: 512-bit two's complement, LSB = 2^-256.
 * ---------------------------------------------------------------------- */
#define ACC_W 8
#define ACC_LSB (-256)

typedef struct { uint64_t w[ACC_W]; } acc_t;

static int bitlen128(u128 m) {
  uint64_t hi = (uint64_t)(m >> 64), lo = (uint64_t)m;
  if (hi) return 128 - __builtin_clzll(hi);
  if (lo) return 64 - __builtin_clzll(lo);
  return 0;
}

/* Add (neg ? -m : m) * 2^e into the accumulator. */
static int acc_add(acc_t* a, u128 m, int e, int neg) {
  if (m == 0) return ORC_OK;
  while (e < ACC_LSB && (m & 1) == 0) { m >>= 1; e++; }
  if (e < ACC_LSB) return ORC_E_RANGE;           /* below the LSB */
  int s = e - ACC_LSB;
  if (s + bitlen128(m) > ACC_W * 64 - 8) return ORC_E_RANGE;  /* keep headroom */
  uint64_t lo = (uint64_t)m, hi = (uint64_t)(m >> 64);
  int limb = s / 64, off = s % 64;
  uint64_t t[ACC_W + 3];
  memset(t, 0, sizeof t);
  if (off == 0) {
    t[limb] = lo;
    t[limb + 1] = hi;
  } else {
    t[limb] = lo << off;
    t[limb + 1] = (lo >> (64 - off)) | (hi << off);
    t[limb + 2] = hi >> (64 - off);
  }
  if (neg) {
    uint64_t borrow = 0;
    for (int i = 0; i < ACC_W; i++) {
      u128 d = (u128)a->w[i] - t[i] - borrow;
      a->w[i] = (uint64_t)d;
      borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
  } else {
    uint64_t carry = 0;
    for (int i = 0; i < ACC_W; i++) {
      u128 s2 = (u128)a->w[i] + t[i] + carry;
      a->w[i] = (uint64_t)s2;
      carry = (uint64_t)(s2 >> 64);
    }
  }
  return ORC_OK;
}

/* Split a finite non-zero double into an integer mantissa and exponent. */
static void split_double(double x, uint64_t* m, int* e, int* neg) {
  int ex;
  double f = frexp(fabs(x), &ex);    /* f in [0.5, 1) */
  *m = (uint64_t)ldexp(f, 53);       /* exact: f has at most 53 bits */
  *e = ex - 53;
  *neg = signbit(x) ? 1 : 0;
}

static uint64_t get_bits(const uint64_t* w, int pos, int len) {
  /* bits [pos, pos+len) of the multi-word integer, len <= 64, pos >= 0 */
  uint64_t r = 0;
  for (int i = 0; i < len; i++) {
    int p = pos + i;
    if ((w[p / 64] >> (p % 64)) & 1) r |= (uint64_t)1 << i;
  }
  return r;
}

static int any_bits_below(const uint64_t* w, int pos) {
  for (int p = 0; p < pos; p++)
    if ((w[p / 64] >> (p % 64)) & 1) return 1;
  return 0;
}

/* Round the exact value once to the nearest double, ties to even. */
static double acc_round(const acc_t* a) {
  uint64_t w[ACC_W];
  memcpy(w, a->w, sizeof w);
  int neg = (int)(w[ACC_W - 1] >> 63);
  if (neg) {
    uint64_t carry = 1;
    for (int i = 0; i < ACC_W; i++) {
      u128 s = (u128)(~w[i]) + carry;
      w[i] = (uint64_t)s;
      carry = (uint64_t)(s >> 64);
    }
  }
  int top = -1;
  for (int i = ACC_W - 1; i >= 0; i--)
    if (w[i]) { top = i * 64 + 63 - __builtin_clzll(w[i]); break; }
  if (top < 0) return 0.0;
  double v;
  if (top < 53) {
    v = ldexp((double)get_bits(w, 0, top + 1), ACC_LSB);
  } else {
    uint64_t m = get_bits(w, top - 52, 53);
    int rbit = (int)get_bits(w, top - 53, 1);
    int sticky = any_bits_below(w, top - 53);
    if (rbit && (sticky || (m & 1))) m++;
    int t = top;
    if (m == ((uint64_t)1 << 53)) { m >>= 1; t++; }
    v = ldexp((double)m, t - 52 + ACC_LSB);
  }
  return neg ? -v : v;
}

/* Add one term, the product of k factors (see oracle.h for the rule). */
static int acc_add_product(acc_t* a, const double* f, int k) {
  for (int i = 0; i < k; i++)
    if (!isfinite(f[i])) return ORC_E_RANGE;
  if (k == 0) return ORC_E_INVALID;
  volatile double p = f[0];
  for (int i = 1; i + 1 < k; i++) p = p * f[i];
  double x = p, y = (k >= 2) ? f[k - 1] : 1.0;
  if (x == 0.0 || y == 0.0) return ORC_OK;
  uint64_t mx, my;
  int ex, ey, nx, ny;
  split_double(x, &mx, &ex, &nx);
  if (k == 1) return acc_add(a, (u128)mx, ex, nx);
  split_double(y, &my, &ey, &ny);
  return acc_add(a, (u128)mx * my, ex + ey, nx ^ ny);
}

double orc_exact_dot(const double* a, const double* b, uint64_t n, int* status) {
  acc_t acc;
  memset(&acc, 0, sizeof acc);
  int st = ORC_OK;
  for (uint64_t i = 0; i < n && st == ORC_OK; i++) {
    double f[2] = {a[i], b ? b[i] : 1.0};
    st = acc_add_product(&acc, f, b ? 2 : 1);
  }
  if (status) *status = st;
  return acc_round(&acc);
}

/* ------------------------------------------------------------------------
 * Hash table from fixed-width uint32 tuples to item indices.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t width;
  uint64_t cap, n;
  uint64_t* slot;      /* item index + 1, 0 = empty */
  const uint32_t** keysrc;  /* where item keys live: (*keysrc)[item*width] */
} htab;

static uint64_t hash_tuple(const uint32_t* k, uint32_t w) {
  uint64_t h = 0x9e3779b97f4a7c15ull ^ w;
  for (uint32_t i = 0; i < w; i++) {
    h ^= k[i];
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
  }
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 29;
  return h;
}

static int ht_init(htab* t, uint32_t width, uint64_t expect, const uint32_t** keysrc) {
  t->width = width;
  t->cap = 16;
  while (t->cap < 2 * expect + 16) t->cap <<= 1;
  t->n = 0;
  t->keysrc = keysrc;
  t->slot = (uint64_t*)calloc(t->cap, sizeof(uint64_t));
  return t->slot ? ORC_OK : ORC_E_NOMEM;
}

static void ht_free(htab* t) { free(t->slot); t->slot = NULL; }

/* Returns the slot of key k: either holding an equal key or empty. */
static uint64_t ht_find(const htab* t, const uint32_t* k) {
  uint64_t mask = t->cap - 1, i = hash_tuple(k, t->width) & mask;
  for (;;) {
    uint64_t s = t->slot[i];
    if (s == 0) return i;
    const uint32_t* kk = *t->keysrc + (s - 1) * t->width;
    if (memcmp(kk, k, t->width * sizeof(uint32_t)) == 0) return i;
    i = (i + 1) & mask;
  }
}

static int ht_grow(htab* t) {
  uint64_t oldcap = t->cap;
  uint64_t* old = t->slot;
  t->cap <<= 1;
  t->slot = (uint64_t*)calloc(t->cap, sizeof(uint64_t));
  if (!t->slot) { t->slot = old; t->cap = oldcap; return ORC_E_NOMEM; }
  for (uint64_t i = 0; i < oldcap; i++) {
    if (!old[i]) continue;
    const uint32_t* k = *t->keysrc + (old[i] - 1) * t->width;
    t->slot[ht_find(t, k)] = old[i];
  }
  free(old);
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Growable arrays.
 * ---------------------------------------------------------------------- */
typedef struct { void* p; uint64_t n, cap; size_t elt; } vec;

static int vec_reserve(vec* v, uint64_t need) {
  if (need <= v->cap) return ORC_OK;
  uint64_t c = v->cap ? v->cap : 64;
  while (c < need) c *= 2;
  void* q = realloc(v->p, c * v->elt);
  if (!q) return ORC_E_NOMEM;
  v->p = q;
  v->cap = c;
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Query evaluation.
 * ---------------------------------------------------------------------- */

/* One aggregation table: group keys, counts and exact sums.  Every thread
 * aggregates into its own table; the tables are merged at the end, which
 * does not depend on the order because counts and accumulators are exact
 * integers. */
typedef struct {
  uint32_t wk;
  vec gkeys;            /* uint32 x wk per group */
  vec gcount;           /* uint64 per group */
  vec gacc;             /* acc_t per group (SUM) */
  htab agg;
  const uint32_t* gkeys_ptr;
  uint64_t n_join;
  int status;
} agg_state;

typedef struct {
  const orc_query* q;
  uint32_t wu;          /* uint32 slots per intermediate tuple: attrs then groups */
  uint32_t wf;          /* factor slots: one per annotated atom */
  int32_t* fslot;       /* factor slot of each atom, -1 if none */
  uint64_t** rows;      /* surviving row ids per atom */
  uint64_t* nrows;
} eval_ctx;

static int row_passes(const orc_query* q, uint32_t ai, uint64_t r) {
  const orc_atom* a = &q->atoms[ai];
  for (uint32_t i = 0; i < q->n_filters; i++) {
    const orc_filter* f = &q->filters[i];
    if (f->atom != ai) continue;
    switch (f->kind) {
      case ORC_EQ_KEY:
        if (a->keys[f->col][r] != f->eq) return 0;
        break;
      case ORC_EQ_META:
        if (a->meta[f->col][r] != f->eq) return 0;
        break;
      case ORC_RANGE_ANNO: {
        double v = a->annos[f->col][r];
        if (!(v >= f->lo && v < f->hi)) return 0;
        break;
      }
      case ORC_RANGE_META: {
        double v = (double)a->meta[f->col][r];
        if (!(v >= f->lo && v < f->hi)) return 0;
        break;
      }
      default:
        return 0;
    }
  }
  return 1;
}

/* Widest aggregation key: output attributes plus group columns. */
#define MAX_KEY_COLS 128

static int validate(const orc_query* q) {
  if (!q || q->n_atoms == 0 || !q->atoms || q->n_attrs == 0 || q->n_attrs > 64) return ORC_E_INVALID;
  if (q->agg != ORC_COUNT && q->agg != ORC_SUM) return ORC_E_INVALID;
  uint64_t seen = 0;
  int annotated = 0;
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    const orc_atom* a = &q->atoms[e];
    if (a->n_keys == 0 || !a->keys || !a->attr_of_key) return ORC_E_INVALID;
    uint64_t mine = 0;
    for (uint32_t c = 0; c < a->n_keys; c++) {
      uint32_t v = a->attr_of_key[c];
      if (v >= q->n_attrs || (mine >> v & 1)) return ORC_E_INVALID;
      mine |= 1ull << v;
    }
    seen |= mine;
    if (a->anno >= 0 && (uint32_t)a->anno >= a->n_annos) return ORC_E_INVALID;
    if (a->anno >= 0) annotated = 1;
    if (!a->bag && (a->n_annos || a->n_meta)) return ORC_E_INVALID;
  }
  if (seen != (q->n_attrs == 64 ? ~0ull : ((1ull << q->n_attrs) - 1))) return ORC_E_INVALID;
  if (q->agg == ORC_SUM && !annotated) return ORC_E_INVALID;
  if (q->n_out > q->n_attrs || (uint64_t)q->n_out + q->n_group > MAX_KEY_COLS) return ORC_E_INVALID;
  uint64_t outs = 0;
  for (uint32_t i = 0; i < q->n_out; i++) {
    uint32_t v = q->out_attrs[i];
    if (v >= q->n_attrs || (outs >> v & 1)) return ORC_E_INVALID;
    outs |= 1ull << v;
  }
  for (uint32_t i = 0; i < q->n_group; i++) {
    if (q->groups[i].atom >= q->n_atoms) return ORC_E_INVALID;
    if (q->groups[i].meta_col >= q->atoms[q->groups[i].atom].n_meta) return ORC_E_INVALID;
  }
  for (uint32_t i = 0; i < q->n_filters; i++) {
    const orc_filter* f = &q->filters[i];
    if (f->atom >= q->n_atoms) return ORC_E_INVALID;
    const orc_atom* a = &q->atoms[f->atom];
    uint32_t lim = f->kind == ORC_EQ_KEY ? a->n_keys
                 : f->kind == ORC_RANGE_ANNO ? a->n_annos
                 : (f->kind == ORC_EQ_META || f->kind == ORC_RANGE_META) ? a->n_meta : 0;
    if (f->col >= lim) return ORC_E_INVALID;
  }
  return ORC_OK;
}

/* Rows of atom e that pass its filters; a set atom keeps the first row of
 * each distinct key tuple. */
static int select_rows(const orc_query* q, uint32_t e, uint64_t** out, uint64_t* nout) {
  const orc_atom* a = &q->atoms[e];
  uint64_t* r = (uint64_t*)malloc((a->n_rows ? a->n_rows : 1) * sizeof(uint64_t));
  if (!r) return ORC_E_NOMEM;
  uint64_t n = 0;
  for (uint64_t i = 0; i < a->n_rows; i++)
    if (row_passes(q, e, i)) r[n++] = i;
  if (!a->bag && n) {
    uint32_t w = a->n_keys;
    uint32_t* keys = (uint32_t*)malloc(n * w * sizeof(uint32_t));
    if (!keys) { free(r); return ORC_E_NOMEM; }
    const uint32_t* kp = keys;
    htab t;
    if (ht_init(&t, w, n, &kp)) { free(keys); free(r); return ORC_E_NOMEM; }
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++) {
      uint32_t* k = keys + m * w;
      for (uint32_t c = 0; c < w; c++) k[c] = a->keys[c][r[i]];
      uint64_t s = ht_find(&t, k);
      if (t.slot[s]) continue;           /* duplicate key tuple */
      t.slot[s] = m + 1;
      r[m++] = r[i];
      if (++t.n * 2 > t.cap && ht_grow(&t)) { ht_free(&t); free(keys); free(r); return ORC_E_NOMEM; }
    }
    n = m;
    ht_free(&t);
    free(keys);
  }
  *out = r;
  *nout = n;
  return ORC_OK;
}

static int agg_init(agg_state* a, uint32_t wk, int is_sum) {
  memset(a, 0, sizeof *a);
  a->wk = wk;
  a->gkeys.elt = sizeof(uint32_t);
  a->gcount.elt = sizeof(uint64_t);
  a->gacc.elt = sizeof(acc_t);
  if (wk) return ht_init(&a->agg, wk, 1024, &a->gkeys_ptr);
  /* no output columns: one group, present even when nothing joins */
  if (vec_reserve(&a->gcount, 1) || (is_sum && vec_reserve(&a->gacc, 1))) return ORC_E_NOMEM;
  ((uint64_t*)a->gcount.p)[0] = 0;
  a->gcount.n = 1;
  if (is_sum) { memset(a->gacc.p, 0, sizeof(acc_t)); a->gacc.n = 1; }
  return ORC_OK;
}

static void agg_free(agg_state* a) {
  free(a->gkeys.p);
  free(a->gcount.p);
  free(a->gacc.p);
  if (a->wk) ht_free(&a->agg);
}

/* Group index of key in table a (created empty when new), or UINT64_MAX
 * when memory runs out. */
static uint64_t agg_group(agg_state* a, const uint32_t* key, int is_sum) {
  if (a->wk == 0) return 0;
  /* the probe key is compared against stored keys only */
  uint64_t s = ht_find(&a->agg, key);
  if (a->agg.slot[s]) return a->agg.slot[s] - 1;
  uint64_t g = a->gcount.n;
  if (vec_reserve(&a->gkeys, (g + 1) * a->wk) || vec_reserve(&a->gcount, g + 1) ||
      (is_sum && vec_reserve(&a->gacc, g + 1)))
    return UINT64_MAX;
  memcpy((uint32_t*)a->gkeys.p + g * a->wk, key, a->wk * sizeof(uint32_t));
  a->gkeys_ptr = (const uint32_t*)a->gkeys.p;
  ((uint64_t*)a->gcount.p)[g] = 0;
  a->gcount.n = g + 1;
  a->gkeys.n = (g + 1) * a->wk;
  if (is_sum) {
    memset((acc_t*)a->gacc.p + g, 0, sizeof(acc_t));
    a->gacc.n = g + 1;
  }
  a->agg.slot[s] = g + 1;
  if (++a->agg.n * 2 > a->agg.cap && ht_grow(&a->agg)) return UINT64_MAX;
  return g;
}

/* x += y, both 512-bit two's complement (merging exact accumulators). */
static void acc_merge(acc_t* x, const acc_t* y) {
  uint64_t carry = 0;
  for (int i = 0; i < ACC_W; i++) {
    u128 s2 = (u128)x->w[i] + y->w[i] + carry;
    x->w[i] = (uint64_t)s2;
    carry = (uint64_t)(s2 >> 64);
  }
}

/* Aggregate one full-join tuple into table a (u: attr values then group
 * values, f: the factors of the annotated atoms, in atom order). */
static void aggregate(const eval_ctx* c, agg_state* a, const uint32_t* u, const double* f) {
  const orc_query* q = c->q;
  uint32_t key[MAX_KEY_COLS];
  for (uint32_t i = 0; i < q->n_out; i++) key[i] = u[q->out_attrs[i]];
  for (uint32_t i = 0; i < q->n_group; i++) key[q->n_out + i] = u[q->n_attrs + i];
  const int is_sum = q->agg == ORC_SUM;
  uint64_t g = agg_group(a, key, is_sum);
  if (g == UINT64_MAX) { a->status = ORC_E_NOMEM; return; }
  ((uint64_t*)a->gcount.p)[g] += 1;
  a->n_join++;
  if (is_sum) {
    int st = acc_add_product((acc_t*)a->gacc.p + g, f, (int)c->wf);
    if (st) a->status = st;
  }
}

/* Fill the slots of tuple (u, f) that atom e's row r binds. */
static void bind_atom(const eval_ctx* c, uint32_t e, uint64_t r, uint32_t* u, double* f) {
  const orc_query* q = c->q;
  const orc_atom* a = &q->atoms[e];
  for (uint32_t k = 0; k < a->n_keys; k++) u[a->attr_of_key[k]] = a->keys[k][r];
  for (uint32_t i = 0; i < q->n_group; i++)
    if (q->groups[i].atom == e) u[q->n_attrs + i] = a->meta[q->groups[i].meta_col][r];
  if (c->fslot[e] >= 0) f[c->fslot[e]] = a->annos[a->anno][r];
}

typedef struct { const uint32_t* K; uint32_t w; } key_cmp_ctx;

static int key_cmp(const void* x, const void* y, void* ctx) {
  const key_cmp_ctx* c = (const key_cmp_ctx*)ctx;
  const uint32_t* a = c->K + *(const uint64_t*)x * c->w;
  const uint32_t* b = c->K + *(const uint64_t*)y * c->w;
  for (uint32_t i = 0; i < c->w; i++)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

static int n_threads_set = 0;

void orc_set_threads(int n) { n_threads_set = n > 0 ? n : 0; }

int orc_threads(void) {
#ifdef _OPENMP
  return n_threads_set > 0 ? n_threads_set : omp_get_max_threads();
#else
  return 1;
#endif
}

/* The running intermediate: one segment of tuples per thread that made
 * them (their order does not matter: the join is a set of tuples and the
 * aggregation is exact). */
typedef struct {
  vec u, f;
  uint64_t n;
} segment;

int orc_join_aggregate(const orc_query* q, orc_result* out) {
  if (!out) return ORC_E_INVALID;
  memset(out, 0, sizeof *out);
  int st = validate(q);
  if (st) return st;
  const int nthr = orc_threads();
  const int is_sum = q->agg == ORC_SUM;

  eval_ctx c;
  memset(&c, 0, sizeof c);
  c.q = q;
  c.wu = q->n_attrs + q->n_group;
  const uint32_t wk = q->n_out + q->n_group;
  c.fslot = (int32_t*)malloc(q->n_atoms * sizeof(int32_t));
  c.rows = (uint64_t**)calloc(q->n_atoms, sizeof(uint64_t*));
  c.nrows = (uint64_t*)calloc(q->n_atoms, sizeof(uint64_t));
  agg_state* tabs = (agg_state*)calloc((size_t)nthr, sizeof(agg_state));
  segment* cur = (segment*)calloc((size_t)nthr, sizeof(segment));
  segment* nxt = (segment*)calloc((size_t)nthr, sizeof(segment));
  int ncur = 1;
  uint32_t* bkeys = NULL;
  uint64_t* chain = NULL;
  if (!c.fslot || !c.rows || !c.nrows || !tabs || !cur || !nxt) { st = ORC_E_NOMEM; goto done; }
  for (int t = 0; t < nthr; t++) {
    cur[t].u.elt = nxt[t].u.elt = sizeof(uint32_t);
    cur[t].f.elt = nxt[t].f.elt = sizeof(double);
    if ((st = agg_init(&tabs[t], wk, is_sum))) goto done;
  }
  for (uint32_t e = 0; e < q->n_atoms; e++) {
    c.fslot[e] = (is_sum && q->atoms[e].anno >= 0) ? (int32_t)c.wf++ : -1;
    if ((st = select_rows(q, e, &c.rows[e], &c.nrows[e]))) goto done;
  }
  const uint32_t wf1 = c.wf ? c.wf : 1;

  /* scan of atom 0 */
  {
    segment* s0 = &cur[0];
    if (vec_reserve(&s0->u, (c.nrows[0] + 1) * c.wu) || vec_reserve(&s0->f, (c.nrows[0] + 1) * wf1)) { st = ORC_E_NOMEM; goto done; }
    for (uint64_t i = 0; i < c.nrows[0]; i++) {
      uint32_t* u = (uint32_t*)s0->u.p + i * c.wu;
      double* f = (double*)s0->f.p + i * wf1;
      memset(u, 0, c.wu * sizeof(uint32_t));
      bind_atom(&c, 0, c.rows[0][i], u, f);
    }
    s0->n = c.nrows[0];
    out->n_intermediate = s0->n;
  }
  if (q->n_atoms == 1) {
    for (uint64_t i = 0; i < cur[0].n && !tabs[0].status; i++)
      aggregate(&c, &tabs[0], (uint32_t*)cur[0].u.p + i * c.wu, (double*)cur[0].f.p + i * wf1);
  }

  uint64_t bound = 0;
  for (uint32_t k = 0; k < q->atoms[0].n_keys; k++) bound |= 1ull << q->atoms[0].attr_of_key[k];

  for (uint32_t e = 1; e < q->n_atoms; e++) {
    const orc_atom* a = &q->atoms[e];
    uint32_t shared_col[64], shared_attr[64], ns = 0;
    for (uint32_t v = 0; v < q->n_attrs; v++) {
      if (!(bound >> v & 1)) continue;
      for (uint32_t k = 0; k < a->n_keys; k++)
        if (a->attr_of_key[k] == v) { shared_col[ns] = k; shared_attr[ns] = v; ns++; }
    }
    /* build side: hash table on the shared attributes of atom e */
    uint64_t nb = c.nrows[e];
    uint32_t wsh = ns ? ns : 1;
    free(bkeys);
    free(chain);
    bkeys = (uint32_t*)malloc((nb + 1) * wsh * sizeof(uint32_t));
    chain = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
    if (!bkeys || !chain) { st = ORC_E_NOMEM; goto done; }
    const uint32_t* bk = bkeys;
    htab ht;
    if ((st = ht_init(&ht, wsh, nb, &bk))) goto done;
    /* head of each key's chain lives in the slot; chain[i] links rows */
    uint64_t* head = NULL;
    {
      vec hv = {0, 0, 0, sizeof(uint64_t)};
      for (uint64_t i = 0; i < nb; i++) {
        uint32_t* k = bkeys + i * wsh;
        if (ns == 0) k[0] = 0;
        for (uint32_t j = 0; j < ns; j++) k[j] = a->keys[shared_col[j]][c.rows[e][i]];
        uint64_t s = ht_find(&ht, k);
        if (ht.slot[s]) {
          uint64_t key_item = ht.slot[s] - 1;          /* first row with this key */
          chain[i] = ((uint64_t*)hv.p)[key_item];      /* previous head */
          ((uint64_t*)hv.p)[key_item] = i;
        } else {
          if (vec_reserve(&hv, i + 1)) { ht_free(&ht); free(hv.p); st = ORC_E_NOMEM; goto done; }
          ((uint64_t*)hv.p)[i] = i;                    /* indexed by the key's first row */
          chain[i] = UINT64_MAX;
          ht.slot[s] = i + 1;
          if (++ht.n * 2 > ht.cap && ht_grow(&ht)) { ht_free(&ht); free(hv.p); st = ORC_E_NOMEM; goto done; }
        }
      }
      head = (uint64_t*)hv.p;
    }
    /* probe side: the running intermediate, split over the threads; each
     * thread appends to its own segment or aggregates into its own table */
    const int last = (e + 1 == q->n_atoms);
    int fail = 0;
    for (int t = 0; t < nthr; t++) nxt[t].n = 0;
#pragma omp parallel num_threads(nthr)
    {
#ifdef _OPENMP
      const int t = omp_get_thread_num();
#else
      const int t = 0;
#endif
      uint32_t probe[64];
      uint32_t* tu = (uint32_t*)malloc(c.wu * sizeof(uint32_t) + 4);
      double* tf = (double*)malloc(wf1 * sizeof(double));
      segment* my = &nxt[t];
      agg_state* tab = &tabs[t];
      if (!tu || !tf) {
#pragma omp atomic write
        fail = 1;
      }
      for (int sg = 0; sg < ncur; sg++) {
        const segment* in = &cur[sg];
#pragma omp for schedule(dynamic, 4096) nowait
        for (uint64_t i = 0; i < in->n; i++) {
          int stop;
#pragma omp atomic read
          stop = fail;
          if (stop || tab->status || !tu || !tf) continue;
          const uint32_t* u = (const uint32_t*)in->u.p + i * c.wu;
          const double* f = (const double*)in->f.p + i * wf1;
          if (ns == 0) probe[0] = 0;
          for (uint32_t j = 0; j < ns; j++) probe[j] = u[shared_attr[j]];
          uint64_t s = ht_find(&ht, probe);
          if (!ht.slot[s]) continue;
          for (uint64_t b = head[ht.slot[s] - 1]; b != UINT64_MAX; b = chain[b]) {
            memcpy(tu, u, c.wu * sizeof(uint32_t));
            memcpy(tf, f, wf1 * sizeof(double));
            bind_atom(&c, e, c.rows[e][b], tu, tf);
            if (last) {
              aggregate(&c, tab, tu, tf);
            } else {
              if (vec_reserve(&my->u, (my->n + 1) * c.wu) || vec_reserve(&my->f, (my->n + 1) * wf1)) {
#pragma omp atomic write
                fail = 1;
                break;
              }
              memcpy((uint32_t*)my->u.p + my->n * c.wu, tu, c.wu * sizeof(uint32_t));
              memcpy((double*)my->f.p + my->n * wf1, tf, wf1 * sizeof(double));
              my->n++;
            }
          }
        }
      }
      free(tu);
      free(tf);
    }
    free(head);
    ht_free(&ht);
    if (fail) { st = ORC_E_NOMEM; goto done; }
    for (int t = 0; t < nthr; t++)
      if (tabs[t].status) { st = tabs[t].status; goto done; }
    if (!last) {
      uint64_t tot = 0;
      for (int t = 0; t < nthr; t++) {
        segment tmp = cur[t];
        cur[t] = nxt[t];
        nxt[t] = tmp;
        tot += cur[t].n;
      }
      ncur = nthr;
      if (tot > out->n_intermediate) out->n_intermediate = tot;
    }
    for (uint32_t k = 0; k < a->n_keys; k++) bound |= 1ull << a->attr_of_key[k];
  }
  for (int t = 0; t < nthr; t++)
    if (tabs[t].status) { st = tabs[t].status; goto done; }

  /* merge the thread tables into the first one */
  for (int t = 1; t < nthr; t++) {
    agg_state* src = &tabs[t];
    for (uint64_t g = 0; g < src->gcount.n; g++) {
      const uint64_t d = agg_group(&tabs[0], (const uint32_t*)src->gkeys.p + g * src->wk, is_sum);
      if (d == UINT64_MAX) { st = ORC_E_NOMEM; goto done; }
      ((uint64_t*)tabs[0].gcount.p)[d] += ((const uint64_t*)src->gcount.p)[g];
      if (is_sum) acc_merge((acc_t*)tabs[0].gacc.p + d, (const acc_t*)src->gacc.p + g);
    }
    tabs[0].n_join += src->n_join;
  }

  /* emit, sorted ascending by key */
  {
    const agg_state* A = &tabs[0];
    uint64_t ng = A->gcount.n;
    if (wk == 0) ng = 1;
    uint64_t* order = (uint64_t*)malloc((ng + 1) * sizeof(uint64_t));
    if (!order) { st = ORC_E_NOMEM; goto done; }
    for (uint64_t i = 0; i < ng; i++) order[i] = i;
    if (wk) {
      key_cmp_ctx cx = {(const uint32_t*)A->gkeys.p, wk};
      qsort_r(order, ng, sizeof(uint64_t), key_cmp, &cx);
    }
    out->n_rows = ng;
    out->n_cols = wk;
    out->keys = (uint32_t*)malloc((ng * wk + 1) * sizeof(uint32_t));
    out->counts = (uint64_t*)malloc((ng + 1) * sizeof(uint64_t));
    out->sums = is_sum ? (double*)malloc((ng + 1) * sizeof(double)) : NULL;
    if (!out->keys || !out->counts || (is_sum && !out->sums)) {
      free(order);
      orc_result_free(out);
      st = ORC_E_NOMEM;
      goto done;
    }
    for (uint64_t i = 0; i < ng; i++) {
      uint64_t g = order[i];
      if (wk) memcpy(out->keys + i * wk, (uint32_t*)A->gkeys.p + g * wk, wk * sizeof(uint32_t));
      out->counts[i] = ((uint64_t*)A->gcount.p)[g];
      if (out->sums) out->sums[i] = acc_round((acc_t*)A->gacc.p + g);
    }
    out->n_join_tuples = A->n_join;
    free(order);
  }

done:
  if (c.rows)
    for (uint32_t e = 0; e < q->n_atoms; e++) free(c.rows[e]);
  free(c.rows);
  free(c.nrows);
  free(c.fslot);
  if (tabs)
    for (int t = 0; t < nthr; t++) agg_free(&tabs[t]);
  free(tabs);
  if (cur)
    for (int t = 0; t < nthr; t++) { free(cur[t].u.p); free(cur[t].f.p); }
  if (nxt)
    for (int t = 0; t < nthr; t++) { free(nxt[t].u.p); free(nxt[t].f.p); }
  free(cur);
  free(nxt);
  free(bkeys);
  free(chain);
  return st;
}

void orc_result_free(orc_result* r) {
  if (!r) return;
  free(r->keys);
  free(r->counts);
  free(r->sums);
  r->keys = NULL;
  r->counts = NULL;
  r->sums = NULL;
}
