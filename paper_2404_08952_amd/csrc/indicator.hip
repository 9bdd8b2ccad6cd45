// Launchers of the learned-indicator kernels (features, MLP forward,
// gradients, Adam) and of the per-stage gradient + features kernel.
#include <mutex>

#include "dispatch_impl.hpp"
#include "indicator_impl.hpp"

namespace dolinc {

static_assert(MLP_IN == DOLINC_N_FEATURES && MLP_INP == DOLINC_FEATURE_STRIDE && MLP_NPARAM == DOLINC_MLP_PARAMS,
              "network sizes of the kernels and of the C interface differ");

hipError_t features_launch(dolinc_ctx_s* c, const void* U, float* X32, unsigned short* Xb, hipStream_t s) {
  if (c->w.precision == DOLINC_FP64) {
    KArgs<double> a = base_args<double>(c);
    a.U = (const double*)U;
    hipLaunchKernelGGL((k_features<double, 3>), dim3(8 * a.cell_per_xcd), dim3(KTPB), 0, s, a, X32, Xb);
  } else {
    KArgs<float> a = base_args<float>(c);
    a.U = (const float*)U;
    hipLaunchKernelGGL((k_features<float, 3>), dim3(8 * a.cell_per_xcd), dim3(KTPB), 0, s, a, X32, Xb);
  }
  return hipGetLastError();
}

static MlpDev mlp_dev(dolinc_ctx_s* c) {
  MlpDev m;
  m.p = c->mlp.p;
  m.w1b = c->mlp.w1b;
  m.w2b = c->mlp.w2b;
  return m;
}

hipError_t grad_features_launch(dolinc_ctx_s* c, const void* U, void* G1, unsigned short* Xf, hipStream_t s) {
  if (c->w.precision == DOLINC_FP64) {
    KArgs<double> a = base_args<double>(c);
    a.U = (const double*)U;
    hipLaunchKernelGGL((k_grad_features<double, 3>), dim3(8 * a.cell_per_xcd), dim3(KTPB), 0, s, a,
                       (double*)G1, Xf);
  } else {
    KArgs<float> a = base_args<float>(c);
    a.U = (const float*)U;
    hipLaunchKernelGGL((k_grad_features<float, 3>), dim3(8 * a.cell_per_xcd), dim3(KTPB), 0, s, a,
                       (float*)G1, Xf);
  }
  return hipGetLastError();
}

hipError_t mlp_set_launch(dolinc_ctx_s* c, const float* src, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_set, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, src, c->mlp.p, c->mlp.m, c->mlp.v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_pack, dim3((MLP_H * MLP_H + 255) / 256), dim3(256), 0, s, c->mlp.p, c->mlp.w1b,
                     c->mlp.w2b);
  return hipGetLastError();
}

hipError_t mlp_forward_launch(dolinc_ctx_s* c, const unsigned short* X, int64_t n, float* theta, hipStream_t s,
                              int xstride) {
  const int64_t tiles = (n + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)blocks), dim3(256), 0, s, mlp_dev(c), X, n, theta, xstride);
  return hipGetLastError();
}

static hipError_t grad_and_adam(dolinc_ctx_s* c, const unsigned short* X, const float* y, int64_t n, int nblocks,
                                int rows_per_block, float* part, float* loss_part, float* grad_out, float* loss_out,
                                int do_step, float lr, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(256), 0, s, mlp_dev(c), X, y, n, rows_per_block, part,
                     loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 1 + ADAM_K - 1) / ADAM_K), dim3(256), 0, s, nblocks, part,
                     loss_part, c->mlp.p, c->mlp.m, c->mlp.v, c->mlp.w1b, c->mlp.w2b, grad_out, loss_out, do_step, lr,
                     0.9f, 0.999f, c1, c2, 1e-8f);
  return hipGetLastError();
}

hipError_t mlp_grad_launch(dolinc_ctx_s* c, const unsigned short* X, const float* y, int64_t n, int nblocks,
                           int rows_per_block, float* grad_out, float* loss_out, int do_step, float lr, float c1,
                           float c2, hipStream_t s) {
  return grad_and_adam(c, X, y, n, nblocks, rows_per_block, c->mlp.part, c->mlp.loss_part, grad_out, loss_out,
                       do_step, lr, c1, c2, s);
}

// ------------------------------------------------------------ training without allocation
// The per-block partial gradients and losses of a training step in a fixed
// device array of this file instead of the context's growable workspace:
// MLP_STATIC_BLOCKS partials of MLP_NPARAM floats, then MLP_STATIC_BLOCKS
// partial losses (about 6 MB per device, held until the process ends).
// Every call on a device shares that device's array; k_mlp_grad writes every
// partial the following k_mlp_adam reads, so nothing needs clearing.
static __device__ __align__(256) float scratch[(size_t)MLP_STATIC_BLOCKS * (MLP_NPARAM + 1)];

namespace {
std::mutex g_scratch_mu;
float* g_scratch_ptr[MLP_STATIC_MAX_DEVICES] = {};
}  // namespace

// Device address of this device's scratch array (looked up once per device,
// with that device current; the array's name in host code is not a device
// address).
static hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MLP_STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t mlp_train_static_launch(dolinc_ctx_s* c, const unsigned short* X, const float* y, int64_t n, int nblocks,
                                   int rows_per_block, float* loss_out, float lr, float c1, float c2,
                                   hipStream_t s) {
  if (nblocks > MLP_STATIC_BLOCKS) return hipErrorInvalidValue;
  float* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  return grad_and_adam(c, X, y, n, nblocks, rows_per_block, base, base + (size_t)MLP_STATIC_BLOCKS * MLP_NPARAM,
                       nullptr, loss_out, 1, lr, c1, c2, s);
}

}  // namespace dolinc
