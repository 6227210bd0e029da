// The learned cost model's network (see mlp.hip).
#pragma once

#include <stdint.h>

#include <vector>

#include "lh_internal.h"

namespace lh {

constexpr uint32_t MLP_H = 64;

struct Mlp {
  uint32_t din, H;
  std::vector<float> host;  // packed fp32 parameters
  Mlp(uint32_t d, uint32_t h, uint64_t seed);
  uint64_t num_params() const;
  // FP32 forward + backward of one batch; mean loss; packed gradient to host
  float loss_grad(const float* X, const float* y, uint32_t n, float* grad, hipStream_t s) const;
  // Adam on minibatches (device kernels); returns the last epoch's mean loss
  float train(const float* X, const float* y, uint32_t n, uint32_t epochs, uint32_t batch, float lr, uint64_t seed,
              hipStream_t s);
  // predictions for n samples (host or device arrays); bf16 selects the BF16 kernel
  void predict(const float* X, float* y, uint64_t n, bool bf16, hipStream_t s) const;
  void predict_dev(const float* X, float* y, uint64_t n, bool bf16, hipStream_t s) const;
};

// Models registered for the planner and the trie builder (null: plain rule).
enum ModelSlot : uint32_t { MODEL_LAYOUT = 0, MODEL_ORDER = 1 };
const Mlp* registered_model(uint32_t slot);

// Features (see learned.cpp).
constexpr uint32_t LAYOUT_FEATURES = 4;
constexpr uint32_t ORDER_FEATURES = 24;

}  // namespace lh
