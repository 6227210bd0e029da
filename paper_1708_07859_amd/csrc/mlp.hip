// The learned cost model's network: a 3-layer perceptron d_in -> H -> H -> 1
// with ReLU, trained in FP32 (forward, backward, Adam) and evaluated in
// BF16 on the matrix cores for inference.  It predicts log2 of a cost
// (time) from features.
//
// Parameters are packed as [W1 (H x d_in), b1 (H), W2 (H x H), b2 (H),
// W3 (1 x H), b3 (1)], row-major, fp32.
//
// Training kernels compute one output per thread with a sequential sum, so
// a training run is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <random>

#include "device_common.h"
#include "lh_internal.h"
#include "mlp.h"

namespace lh {

namespace {

// Z[n x o] = X[n x i] W^T + b ; A = relu(Z) when relu
__global__ void k_dense_fwd(const float* X, const float* W, const float* b, float* Z, float* A, uint32_t n,
                            uint32_t din, uint32_t dout, uint32_t relu) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * dout) return;
  const uint32_t s = (uint32_t)(t / dout), o = (uint32_t)(t % dout);
  float z = b[o];
  for (uint32_t i = 0; i < din; i++) z = fmaf(X[(uint64_t)s * din + i], W[(uint64_t)o * din + i], z);
  Z[t] = z;
  if (A) A[t] = relu ? fmaxf(z, 0.0f) : z;
}

// dZ for the output layer of the mean squared error L = mean((p - y)^2) / 2
__global__ void k_mse_grad(const float* P, const float* y, float* dZ, float* loss_terms, uint32_t n) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float d = P[s] - y[s];
  dZ[s] = d / (float)n;
  loss_terms[s] = 0.5f * d * d;
}

// dW[o x i] = sum_s dZ[s, o] X[s, i] ; db[o] = sum_s dZ[s, o]
__global__ void k_dense_grad_w(const float* dZ, const float* X, float* dW, float* db, uint32_t n, uint32_t din,
                               uint32_t dout) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)dout * (din + 1)) return;
  const uint32_t o = (uint32_t)(t / (din + 1)), i = (uint32_t)(t % (din + 1));
  float acc = 0.0f;
  if (i < din) {
    for (uint32_t s = 0; s < n; s++) acc = fmaf(dZ[(uint64_t)s * dout + o], X[(uint64_t)s * din + i], acc);
    dW[(uint64_t)o * din + i] = acc;
  } else {
    for (uint32_t s = 0; s < n; s++) acc += dZ[(uint64_t)s * dout + o];
    db[o] = acc;
  }
}

// dX[s, i] = sum_o dZ[s, o] W[o, i], masked by the ReLU of the layer below
__global__ void k_dense_grad_x(const float* dZ, const float* W, const float* Zbelow, float* dX, uint32_t n,
                               uint32_t din, uint32_t dout) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * din) return;
  const uint32_t s = (uint32_t)(t / din), i = (uint32_t)(t % din);
  float acc = 0.0f;
  for (uint32_t o = 0; o < dout; o++) acc = fmaf(dZ[(uint64_t)s * dout + o], W[(uint64_t)o * din + i], acc);
  dX[t] = (Zbelow && Zbelow[t] <= 0.0f) ? 0.0f : acc;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows(const float* X, const float* y, const uint32_t* idx, float* Xo, float* yo, uint32_t n,
                              uint32_t d) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * (d + 1)) return;
  const uint32_t s = (uint32_t)(t / (d + 1)), j = (uint32_t)(t % (d + 1));
  if (j < d) Xo[(uint64_t)s * d + j] = X[(uint64_t)idx[s] * d + j];
  else yo[s] = y[idx[s]];
}

// ---- BF16 inference -------------------------------------------------------------
// bf16 as the upper 16 bits of an fp32, rounded to nearest even.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- BF16 inference on the matrix cores -------------------------------------------
// One wave evaluates 16 samples at a time with v_mfma_f32_16x16x32_bf16
// (D[16x16] += A[16x32] B[32x16], bf16 operands, fp32 sums).  Operand
// layouts (lane l, 64 lanes): A holds row l%16 at k = 8(l/16)..+7; B holds
// column l%16 at k = 8(l/16)..+7; D holds column l%16 at rows 4(l/16)..+3.
// Layer 1 is X (16 x d_in <= 32) times W1^T in four 16-column blocks; its
// outputs (bias, ReLU, rounded to bf16) go through LDS into layer 2's A
// layout; layer 2 takes two 32-wide k steps per block; the output layer is a
// dot product per sample, reduced over the 16 lanes of a column group.  The
// arithmetic is the one-thread kernel's (bf16 operands and layer outputs,
// exact products, fp32 sums) in another summation order.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 bf16_of(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

constexpr int MF_NT = 256;                // 4 waves per block
constexpr int MF_TILE = 16;               // samples per wave tile

__global__ __launch_bounds__(MF_NT) void k_mlp_bf16_mfma(const uint16_t* wts, uint32_t din, const float* X, float* y,
                                                         uint64_t n) {
  constexpr int H = MLP_H;
  __shared__ uint16_t s_h1[MF_NT / WAVE][MF_TILE * H];
  const int lane = lane_id();
  const int wv = threadIdx.x / WAVE;
  const int col = lane % 16, grp = lane / 16;
  const uint16_t* W1 = wts;
  const uint16_t* B1 = W1 + (uint64_t)H * din;
  const uint16_t* W2 = B1 + H;
  const uint16_t* B2 = W2 + (uint64_t)H * H;
  const uint16_t* W3 = B2 + H;
  const uint16_t* B3 = W3 + H;
  // B operands and biases, held for the whole kernel
  bf16x8 w1[4], w2[4][2];
  float b1[4], b2[4], w3[4];
#pragma unroll
  for (int nb = 0; nb < 4; nb++) {
    const int o = 16 * nb + col;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const uint32_t k = 8 * grp + j;
      w1[nb][j] = bf16_of(k < din ? W1[(uint64_t)o * din + k] : (uint16_t)0);
      w2[nb][0][j] = bf16_of(W2[(uint64_t)o * H + k]);
      w2[nb][1][j] = bf16_of(W2[(uint64_t)o * H + 32 + k]);
    }
    b1[nb] = from_bf16(B1[o]);
    b2[nb] = from_bf16(B2[o]);
    w3[nb] = from_bf16(W3[o]);
  }
  const float b3 = from_bf16(B3[0]);
  uint16_t* h1 = s_h1[wv];
  const uint64_t tiles = (n + MF_TILE - 1) / MF_TILE;
  const uint64_t waves = (uint64_t)gridDim.x * (MF_NT / WAVE);
  for (uint64_t t = (uint64_t)blockIdx.x * (MF_NT / WAVE) + wv; t < tiles; t += waves) {
    const uint64_t s0 = t * MF_TILE;
    // layer 1: A = the tile's inputs, rounded to bf16, zero past d_in and n
    bf16x8 a;
    const uint64_t sa = s0 + col;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const uint32_t k = 8 * grp + j;
      a[j] = bf16_of((sa < n && k < din) ? to_bf16(X[sa * din + k]) : (uint16_t)0);
    }
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w1[nb], c, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; j++) h1[(4 * grp + j) * H + 16 * nb + col] = to_bf16(fmaxf(c[j] + b1[nb], 0.0f));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 2: A = h1 in two 32-wide k steps
    bf16x8 a2[2];
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
      for (int j = 0; j < 8; j++) a2[ks][j] = bf16_of(h1[col * H + 32 * ks + 8 * grp + j]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[0], w2[nb][0], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[1], w2[nb][1], c, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const float h2 = from_bf16(to_bf16(fmaxf(c[j] + b2[nb], 0.0f)));
        part[j] = fmaf(h2, w3[nb], part[j]);
      }
    }
    // output layer: sum the 16 columns of each row group (lanes 16 grp .. +15)
#pragma unroll
    for (int j = 0; j < 4; j++) {
#pragma unroll
      for (int d = 8; d > 0; d >>= 1) part[j] += __shfl_xor(part[j], d, 16);
      const uint64_t sy = s0 + 4 * grp + j;
      if (col == 0 && sy < n) y[sy] = part[j] + b3;
    }
  }
}

__global__ void k_to_bf16(const float* p, uint16_t* q, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = to_bf16(p[i]);
}

unsigned blocks(uint64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

uint64_t Mlp::num_params() const { return (uint64_t)H * din + H + (uint64_t)H * H + H + H + 1; }

Mlp::Mlp(uint32_t d, uint32_t h, uint64_t seed) : din(d), H(h) {
  if (d == 0 || d > 32) fail(LH_ERR_INVALID, "MLP input width must be 1..32");
  if (h != MLP_H) fail(LH_ERR_INVALID, "MLP hidden width must be 64");
  host.assign(num_params(), 0.0f);
  std::mt19937_64 g(seed);
  auto init = [&](float* w, uint32_t fan_in, uint64_t count) {
    std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / (float)fan_in));
    for (uint64_t i = 0; i < count; i++) w[i] = nd(g);
  };
  float* p = host.data();
  init(p, din, (uint64_t)H * din);
  p += (uint64_t)H * din + H;
  init(p, H, (uint64_t)H * H);
  p += (uint64_t)H * H + H;
  init(p, H, H);
}

namespace {

struct Layout3 {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};

Layout3 split(const float* p, uint32_t din, uint32_t H) {
  Layout3 L;
  L.W1 = p;
  L.b1 = L.W1 + (uint64_t)H * din;
  L.W2 = L.b1 + H;
  L.b2 = L.W2 + (uint64_t)H * H;
  L.W3 = L.b2 + H;
  L.b3 = L.W3 + H;
  return L;
}

// Forward + backward of one batch on the device; grad (device) receives
// the packed gradient; returns the mean loss.
float loss_grad_dev(const Mlp& m, const float* dparams, const float* X, const float* y, uint32_t n, float* grad,
                    hipStream_t s) {
  const uint32_t din = m.din, H = m.H;
  Layout3 P = split(dparams, din, H);
  DBuf<float> Z1((uint64_t)n * H, s), A1((uint64_t)n * H, s), Z2((uint64_t)n * H, s), A2((uint64_t)n * H, s),
      Z3(n, s), dZ3(n, s), lt(n, s), dA2((uint64_t)n * H, s), dA1((uint64_t)n * H, s);
  k_dense_fwd<<<blocks((uint64_t)n * H), 256, 0, s>>>(X, P.W1, P.b1, Z1.p, A1.p, n, din, H, 1);
  k_dense_fwd<<<blocks((uint64_t)n * H), 256, 0, s>>>(A1.p, P.W2, P.b2, Z2.p, A2.p, n, H, H, 1);
  k_dense_fwd<<<blocks(n), 256, 0, s>>>(A2.p, P.W3, P.b3, Z3.p, nullptr, n, H, 1, 0);
  k_mse_grad<<<blocks(n), 256, 0, s>>>(Z3.p, y, dZ3.p, lt.p, n);
  float* gW1 = grad;
  float* gb1 = gW1 + (uint64_t)H * din;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (uint64_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H;
  k_dense_grad_w<<<blocks((uint64_t)1 * (H + 1)), 256, 0, s>>>(dZ3.p, A2.p, gW3, gb3, n, H, 1);
  k_dense_grad_x<<<blocks((uint64_t)n * H), 256, 0, s>>>(dZ3.p, P.W3, Z2.p, dA2.p, n, H, 1);
  k_dense_grad_w<<<blocks((uint64_t)H * (H + 1)), 256, 0, s>>>(dA2.p, A1.p, gW2, gb2, n, H, H);
  k_dense_grad_x<<<blocks((uint64_t)n * H), 256, 0, s>>>(dA2.p, P.W2, Z1.p, dA1.p, n, H, H);
  k_dense_grad_w<<<blocks((uint64_t)H * (din + 1)), 256, 0, s>>>(dA1.p, X, gW1, gb1, n, din, H);
  LH_HIP(hipGetLastError());
  std::vector<float> h(n);
  LH_HIP(hipMemcpyAsync(h.data(), lt.p, n * sizeof(float), hipMemcpyDeviceToHost, s));
  LH_HIP(hipStreamSynchronize(s));
  double sum = 0;
  for (float v : h) sum += v;
  return (float)(sum / n);
}

}  // namespace

float Mlp::loss_grad(const float* Xh, const float* yh, uint32_t n, float* grad_h, hipStream_t s) const {
  const uint64_t np = num_params();
  DBuf<float> p(np, s), g(np, s), X((uint64_t)n * din, s), y(n, s);
  LH_HIP(hipMemcpyAsync(p.p, host.data(), np * sizeof(float), hipMemcpyHostToDevice, s));
  LH_HIP(hipMemcpyAsync(X.p, Xh, (uint64_t)n * din * sizeof(float), hipMemcpyHostToDevice, s));
  LH_HIP(hipMemcpyAsync(y.p, yh, n * sizeof(float), hipMemcpyHostToDevice, s));
  float loss = loss_grad_dev(*this, p.p, X.p, y.p, n, g.p, s);
  if (grad_h) {
    LH_HIP(hipMemcpyAsync(grad_h, g.p, np * sizeof(float), hipMemcpyDeviceToHost, s));
    LH_HIP(hipStreamSynchronize(s));
  }
  return loss;
}

float Mlp::train(const float* Xh, const float* yh, uint32_t n, uint32_t epochs, uint32_t batch, float lr,
                 uint64_t seed, hipStream_t s) {
  if (n == 0) fail(LH_ERR_INVALID, "no training samples");
  batch = std::max<uint32_t>(1, std::min(batch, n));
  const uint64_t np = num_params();
  DBuf<float> p(np, s), g(np, s), m1(np, s), m2(np, s), X((uint64_t)n * din, s), y(n, s);
  DBuf<float> Xb((uint64_t)batch * din, s), yb(batch, s);
  DBuf<uint32_t> idx(batch, s);
  LH_HIP(hipMemcpyAsync(p.p, host.data(), np * sizeof(float), hipMemcpyHostToDevice, s));
  LH_HIP(hipMemcpyAsync(X.p, Xh, (uint64_t)n * din * sizeof(float), hipMemcpyHostToDevice, s));
  LH_HIP(hipMemcpyAsync(y.p, yh, n * sizeof(float), hipMemcpyHostToDevice, s));
  LH_HIP(hipMemsetAsync(m1.p, 0, np * sizeof(float), s));
  LH_HIP(hipMemsetAsync(m2.p, 0, np * sizeof(float), s));
  std::mt19937_64 rng(seed);
  std::vector<uint32_t> order(n);
  for (uint32_t i = 0; i < n; i++) order[i] = i;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  uint64_t step = 0;
  float last = 0;
  for (uint32_t ep = 0; ep < epochs; ep++) {
    std::shuffle(order.begin(), order.end(), rng);
    double ep_loss = 0;
    uint32_t nb = 0;
    for (uint32_t b0 = 0; b0 + batch <= n; b0 += batch) {
      LH_HIP(hipMemcpyAsync(idx.p, order.data() + b0, batch * sizeof(uint32_t), hipMemcpyHostToDevice, s));
      k_gather_rows<<<blocks((uint64_t)batch * (din + 1)), 256, 0, s>>>(X.p, y.p, idx.p, Xb.p, yb.p, batch, din);
      ep_loss += loss_grad_dev(*this, p.p, Xb.p, yb.p, batch, g.p, s);
      step++;
      const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
      k_adam<<<blocks(np), 256, 0, s>>>(p.p, g.p, m1.p, m2.p, np, lr, b1, b2, eps, c1, c2);
      LH_HIP(hipGetLastError());
      nb++;
    }
    last = (float)(ep_loss / std::max<uint32_t>(1, nb));
  }
  LH_HIP(hipMemcpyAsync(host.data(), p.p, np * sizeof(float), hipMemcpyDeviceToHost, s));
  LH_HIP(hipStreamSynchronize(s));
  return last;
}

void Mlp::predict_dev(const float* X, float* y, uint64_t n, bool bf16, hipStream_t s) const {
  if (n == 0) return;
  const uint64_t np = num_params();
  if (bf16) {
    DBuf<float> p(np, s);
    DBuf<uint16_t> q(np, s);
    LH_HIP(hipMemcpyAsync(p.p, host.data(), np * sizeof(float), hipMemcpyHostToDevice, s));
    k_to_bf16<<<blocks(np), 256, 0, s>>>(p.p, q.p, np);
    // 16 samples per wave, 4 waves per block; blocks stride over the tiles
    const uint64_t tiles = (n + MF_TILE - 1) / MF_TILE;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((tiles + 3) / 4, 2048));
    k_mlp_bf16_mfma<<<grid, MF_NT, 0, s>>>(q.p, din, X, y, n);
    LH_HIP(hipGetLastError());
  } else {
    DBuf<float> p(np, s), Z1(n * H, s), A1(n * H, s), Z2(n * H, s), A2(n * H, s);
    LH_HIP(hipMemcpyAsync(p.p, host.data(), np * sizeof(float), hipMemcpyHostToDevice, s));
    Layout3 P = split(p.p, din, H);
    k_dense_fwd<<<blocks(n * H), 256, 0, s>>>(X, P.W1, P.b1, Z1.p, A1.p, (uint32_t)n, din, H, 1);
    k_dense_fwd<<<blocks(n * H), 256, 0, s>>>(A1.p, P.W2, P.b2, Z2.p, A2.p, (uint32_t)n, H, H, 1);
    k_dense_fwd<<<blocks(n), 256, 0, s>>>(A2.p, P.W3, P.b3, y, nullptr, (uint32_t)n, H, 1, 0);
    LH_HIP(hipGetLastError());
  }
}

void Mlp::predict(const float* Xh, float* yh, uint64_t n, bool bf16, hipStream_t s) const {
  DBuf<float> X(n * din, s), y(n, s);
  LH_HIP(hipMemcpyAsync(X.p, Xh, n * din * sizeof(float), hipMemcpyHostToDevice, s));
  predict_dev(X.p, y.p, n, bf16, s);
  LH_HIP(hipMemcpyAsync(yh, y.p, n * sizeof(float), hipMemcpyDeviceToHost, s));
  LH_HIP(hipStreamSynchronize(s));
}

}  // namespace lh
