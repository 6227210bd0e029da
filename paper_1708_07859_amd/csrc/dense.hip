// Dense linear algebra through attribute elimination (sections 3.1, 6.2.2).
//
// When both relations of a SUM-of-products over one shared attribute are
// completely dense (every key pair of [0,R) x [0,K) present exactly once),
// their annotations, stored in trie order, are already row-major matrices:
// the key attributes carry no information and can be dropped, and the query
// is a matrix-vector or matrix-matrix product over flat FP64 buffers, which
// rocBLAS computes.  The library then only writes the key columns of the
// output.  BLAS sums are not exact, so this route is taken only when the
// query asks for it (LH_DENSE_BLAS).
#include <rocblas/rocblas.h>

#include <cstring>
#include <memory>
#include <mutex>

#include "engine.h"

namespace lh {

namespace {

std::mutex g_blas_mu;
rocblas_handle g_blas[64] = {};

// The handle of the current device, bound to stream s.  The caller holds
// g_blas_mu for as long as it uses the handle (one handle per device is
// shared by every thread).
rocblas_handle blas_handle(hipStream_t s) {
  int dev = 0;
  LH_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(LH_ERR_DEVICE, "dense: device id out of range");
  if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success)
    fail(LH_ERR_DEVICE, "dense: rocblas_create_handle failed");
  if (rocblas_set_stream(g_blas[dev], s) != rocblas_status_success) fail(LH_ERR_DEVICE, "dense: rocblas_set_stream failed");
  return g_blas[dev];
}

// Sizes of a completely dense trie: level l holds every key of [0, size[l])
// under every parent.  Returns false otherwise.
bool dense_sizes(const lh_trie* t, uint32_t* size, hipStream_t s) {
  if (t->n_levels < 1 || t->n_levels > 2) return false;
  uint64_t expect = 1;
  for (uint32_t l = 0; l < t->n_levels; l++) {
    const Level& lv = t->lv[l];
    if (lv.n == 0) return false;
    const uint32_t mx = reduce_max_u32(lv.keys.p, lv.n, s);
    const uint64_t sz = (uint64_t)mx + 1;
    if (sz > (1u << 31) - 1) return false;
    // distinct keys within a set and |level| = (parents) x (max + 1) leave
    // no key of [0, max] out of any set
    expect *= sz;
    if (lv.n != expect) return false;
    size[l] = (uint32_t)sz;
  }
  // one row per key tuple: the annotations are the matrix entries
  return t->n_rows == expect;
}

__global__ void k_dense_keys(uint32_t* k0, uint32_t* k1, uint64_t* cnt, uint64_t rows, uint32_t cols, uint64_t per) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows * cols;
       i += (uint64_t)gridDim.x * blockDim.x) {
    k0[i] = (uint32_t)(i / cols);
    if (k1) k1[i] = (uint32_t)(i % cols);
    cnt[i] = per;
  }
}

}  // namespace

void plan_dense(const lh_query* q, lh_plan_t* p, hipStream_t s) {
  p->blas = 0;
  if (!(q->policy & LH_DENSE_BLAS)) return;
  if (q->agg != LH_AGG_SUM || q->n_atoms != 2 || q->n_filters || q->n_group) return;
  if (q->atoms[0].anno < 0 || q->atoms[1].anno < 0) return;
  uint32_t sz[2][2];
  uint32_t attr[2][2];
  for (uint32_t e = 0; e < 2; e++) {
    const lh_trie* t = q->atoms[e].trie;
    if (!dense_sizes(t, sz[e], s)) return;
    for (uint32_t l = 0; l < t->n_levels; l++) attr[e][l] = q->atoms[e].attr_of_key[t->level_order[l]];
  }
  const lh_trie* t0 = q->atoms[0].trie;
  const lh_trie* t1 = q->atoms[1].trie;
  DensePlan& d = p->dense;
  if (q->n_attrs == 2 && q->n_out == 1 && t0->n_levels + t1->n_levels == 3) {
    // y(r) = SUM_j M(r,j) x(j)
    const uint32_t me = t0->n_levels == 2 ? 0 : 1, xe = 1 - me;
    const uint32_t r = q->out_attrs[0];
    const int rl = attr[me][0] == r ? 0 : (attr[me][1] == r ? 1 : -1);
    if (rl < 0 || attr[xe][0] != attr[me][1 - rl]) return;
    const uint32_t R = sz[me][rl], K = sz[me][1 - rl];
    if (sz[xe][0] != K) return;
    d.a = q->atoms[me].trie->annos[q->atoms[me].anno].p;
    d.b = q->atoms[xe].trie->annos[q->atoms[xe].anno].p;
    d.rows = R;
    d.cols = 1;
    d.inner = K;
    d.a_trans = rl == 1;  // stored (j, r)
    p->blas = 1;
    return;
  }
  if (q->n_attrs == 3 && q->n_out == 2 && t0->n_levels == 2 && t1->n_levels == 2) {
    // O(r,c) = SUM_j P(r,j) Q(j,c), r = out[0], c = out[1]
    const uint32_t r = q->out_attrs[0], c = q->out_attrs[1];
    auto has = [&](uint32_t e, uint32_t v) { return attr[e][0] == v || attr[e][1] == v; };
    int pe = has(0, r) ? 0 : 1;
    const int qe = 1 - pe;
    if (!has(pe, r) || !has(qe, c) || has(pe, c) || has(qe, r)) return;
    const bool pt = attr[pe][1] == r;  // P stored (j, r)
    const bool qt = attr[qe][0] == c;  // Q stored (c, j)
    const uint32_t R = sz[pe][pt ? 1 : 0], Kp = sz[pe][pt ? 0 : 1];
    const uint32_t C = sz[qe][qt ? 0 : 1], Kq = sz[qe][qt ? 1 : 0];
    if (Kp != Kq) return;
    d.a = q->atoms[pe].trie->annos[q->atoms[pe].anno].p;
    d.b = q->atoms[qe].trie->annos[q->atoms[qe].anno].p;
    d.rows = R;
    d.cols = C;
    d.inner = Kp;
    d.a_trans = pt;
    d.b_trans = qt;
    p->blas = 2;
  }
}

lh_result_impl* run_dense(const lh_plan_t* p, hipStream_t s) {
  const DensePlan& d = p->dense;
  std::unique_ptr<lh_result_impl> res(new lh_result_impl());
  memset(&res->pub, 0, sizeof(res->pub));
  const uint64_t n = (uint64_t)d.rows * d.cols;
  const uint32_t n_cols = p->blas == 1 ? 1 : 2;
  res->cols.resize(n_cols);
  for (uint32_t c = 0; c < n_cols; c++) res->cols[c].alloc(n, s);
  res->counts.alloc(n, s);
  res->sums.alloc(n, s);
  std::unique_lock<std::mutex> lk(g_blas_mu);
  rocblas_handle h = blas_handle(s);
  const double one = 1.0, zero = 0.0;
  rocblas_status st;
  {
    ProfScope ps(p->blas == 1 ? "dense_gemv" : "dense_gemm", s, n, (uint64_t)n * d.inner);
    if (p->blas == 1) {
      // row-major M (R x K) is column-major M^T with ld K; stored (j, r) it
      // is column-major M with ld R
      if (!d.a_trans)
        st = rocblas_dgemv(h, rocblas_operation_transpose, (rocblas_int)d.inner, (rocblas_int)d.rows, &one, d.a,
                           (rocblas_int)d.inner, d.b, 1, &zero, res->sums.p, 1);
      else
        st = rocblas_dgemv(h, rocblas_operation_none, (rocblas_int)d.rows, (rocblas_int)d.inner, &one, d.a,
                           (rocblas_int)d.rows, d.b, 1, &zero, res->sums.p, 1);
    } else {
      // row-major O = P Q is column-major O^T = Q^T P^T (ld C)
      const rocblas_operation opq = d.b_trans ? rocblas_operation_transpose : rocblas_operation_none;
      const rocblas_operation opp = d.a_trans ? rocblas_operation_transpose : rocblas_operation_none;
      const rocblas_int ldq = d.b_trans ? (rocblas_int)d.inner : (rocblas_int)d.cols;
      const rocblas_int ldp = d.a_trans ? (rocblas_int)d.rows : (rocblas_int)d.inner;
      st = rocblas_dgemm(h, opq, opp, (rocblas_int)d.cols, (rocblas_int)d.rows, (rocblas_int)d.inner, &one, d.b, ldq,
                         d.a, ldp, &zero, res->sums.p, (rocblas_int)d.cols);
    }
  }
  lk.unlock();
  if (st != rocblas_status_success) fail(LH_ERR_DEVICE, "dense: rocBLAS call failed");
  if (n) {
    const uint64_t b = std::min<uint64_t>((n + 255) / 256, 16384);
    k_dense_keys<<<(unsigned)b, 256, 0, s>>>(res->cols[0].p, n_cols == 2 ? res->cols[1].p : nullptr,
                                             res->counts.p, d.rows, d.cols, d.inner);
    LH_HIP(hipGetLastError());
  }
  res->colptr.resize(n_cols);
  for (uint32_t c = 0; c < n_cols; c++) res->colptr[c] = res->cols[c].p;
  lh_result& R = res->pub;
  R.n_rows = n;
  R.n_cols = n_cols;
  R.out_keys = res->colptr.data();
  R.counts = res->counts.p;
  R.sums = res->sums.p;
  R.exact = 0;
  R.n_join_tuples = n * d.inner;
  LH_HIP(hipStreamSynchronize(s));
  return res.release();
}

}  // namespace lh
