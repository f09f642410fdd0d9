// Fully connected tanh network trained and evaluated on the GPU (the surrogate
// for the reaction derivative tables).  Device buffers, FP32 master weights.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace tefmm {

struct Mlp {
  int n_in = 0, width = 0, n_hidden = 0, n_out = 0;
  int64_t P = 0;                                 // parameter count
  std::vector<int64_t> off_W, off_b;             // offsets of W_l, b_l in theta (l = 0 .. n_hidden)
  std::vector<int> rows, cols;                   // shape of W_l
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  int64_t step = 0;
  int split = 0;  // hidden products with operands as BF16 hi + lo pairs (three MFMAs each)
  // workspace for up to cap rows
  int64_t cap = 0;
  float *acts = nullptr, *y = nullptr, *d0 = nullptr, *d1 = nullptr, *xb = nullptr, *tb = nullptr;
  int* d_idx = nullptr;
  double* d_loss = nullptr;

  ~Mlp();
  hipError_t init(int n_in, int width, int n_hidden, int n_out, uint64_t seed);
  hipError_t reserve(int64_t n);
  hipError_t forward(const float* x, int64_t n, float* out, hipStream_t s);
  hipError_t forward_in(const float* x, int64_t n, float* out, hipStream_t s, float* buf, int64_t stride,
                        int nslab);
  hipError_t loss_grad(const float* x, const float* t, int64_t n, hipStream_t s);
  hipError_t adam(float lr, hipStream_t s);
  hipError_t train(const float* X, const float* T, int64_t n, int epochs, int batch, float lr, uint64_t seed,
                   std::vector<double>& losses, hipStream_t s);

 private:
  void layout();
};

}  // namespace tefmm
