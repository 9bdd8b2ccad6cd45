// Learned smoothness indicator: per-cell features and the 24-64-64-1 MLP.
//
// Features (24 per cell): channels q in {rho, p, rho E, |rho u|}, six
// statistics each over the cell's faces in the frame where the cell is
// upwind: Delta = q_N - q_P, g0 = 2 d0 . grad q (DOLINC differential),
// s = g0 - Delta, beta = |s - Delta| / (|s| + |Delta| + eps),
// scale = |q| + mean |Delta|:
//   max|g0|/scale, max|Delta|/scale, max beta, mean beta,
//   min clip(s Delta / (Delta^2 + eps^2), -2, 2), max|s - Delta|/scale,
// each clipped to [-8, 8].  grad p and grad|rho u| by the chain rule.
//
// Network: theta = sigmoid(W3 . tanh(W2 tanh(W1 x + b1) + b2) + b3).
// Matrix-core formulation (wave64): each wave carries 16 cells as the N
// dimension of Z^T = W X^T, so the accumulator tiles of one layer (lane l
// holds units 4(l/16)..4(l/16)+3 of cell l%16) are the B operand of the next
// layer: the forward uses v_mfma_f32_16x16x32_bf16, the backward's products
// v_mfma_f32_16x16x16_bf16.  bf16 operands (round to nearest even), fp32
// accumulation, fp32 biases, last layer on the vector ALU.
#pragma once
#include "residual_impl.hpp"

namespace dolinc {

constexpr int MLP_IN = 24, MLP_INP = 32, MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;
// offsets into the packed parameter vector
constexpr int OFF_W1 = 0, OFF_B1 = MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> bf16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ unsigned short f2bf(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MlpDev {
  const float* p;                // fp32 master parameters (packed)
  const unsigned short* w1b;     // bf16 W1 [64][32] (K padded with zeros)
  const unsigned short* w2b;     // bf16 W2 [64][64]
};

// ---------------------------------------------------------------- features

// tanh x = 2 / (1 + exp(-2x)) - 1 with the hardware base-2 exponential and
// reciprocal (five instructions).  No clamp is needed: for large negative x
// the exponential overflows to +inf and the reciprocal to 0 (tanh = -1), for
// large positive x it underflows to 0 (tanh = 1).
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(x * -2.8853900817779268f);  // -2 log2(e)
  return fmaf(__builtin_amdgcn_rcpf(1.f + e), 2.f, -1.f);
}

// x clamped to [lo, hi] (one v_med3 for fp32)
__device__ __forceinline__ float clampv(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double clampv(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

template <class T, int D>
__device__ __forceinline__ void cell_channels(const T* U, const T* G, T gamma, T* q, T (*gq)[D]) {
  const T rho = U[0];
  T u[D], ke = T(0), mag2 = T(0);
  for (int a = 0; a < D; ++a) {
    u[a] = fdiv(U[1 + a], rho);
    ke += U[1 + a] * u[a];
    mag2 += U[1 + a] * U[1 + a];
  }
  const T E = U[D + 1];
  const T mag = fsqrt(mag2);
  q[0] = rho;
  q[1] = (gamma - T(1)) * (E - T(0.5) * ke);
  q[2] = E;
  q[3] = mag;
  T uu = T(0);
  for (int a = 0; a < D; ++a) uu += u[a] * u[a];
  for (int x = 0; x < D; ++x) {
    const T gr = G[0 * D + x], gE = G[(D + 1) * D + x];
    T ugm = T(0), mgm = T(0);
    for (int a = 0; a < D; ++a) {
      ugm += u[a] * G[(1 + a) * D + x];
      mgm += U[1 + a] * G[(1 + a) * D + x];
    }
    gq[0][x] = gr;
    gq[1][x] = (gamma - T(1)) * (gE - ugm + T(0.5) * uu * gr);
    gq[2][x] = gE;
    gq[3][x] = mag > T(1e-30) ? fdiv(mgm, mag) : T(0);
  }
}

// Running statistics of the features over a cell's faces
template <class T>
struct FeatAcc {
  T mx_g0[4], mx_dl[4], mx_b[4], sm_b[4], mn_r[4], mx_sd[4], sm_dl[4];
  int nface;
  __device__ __forceinline__ void init() {
    for (int k = 0; k < 4; ++k) {
      mx_g0[k] = mx_dl[k] = mx_b[k] = sm_b[k] = mx_sd[k] = sm_dl[k] = T(0);
      mn_r[k] = T(2);
    }
    nface = 0;
  }
};

// One face of the cell: dv = sigma d (the cell's upwind frame), Uo the
// other cell's state, qc / gqc the cell's channels and their gradients.
template <class T, int D>
__device__ __forceinline__ void feat_face(const T* dv, const T* Uo, T gamma, const T* qc, const T (*gqc)[D],
                                          FeatAcc<T>& A) {
  ++A.nface;
  // neighbour channel values
  T qo[4];
  {
    const T rho = Uo[0];
    T ke = T(0), m2 = T(0);
    for (int x = 0; x < D; ++x) {
      ke += fdiv(Uo[1 + x] * Uo[1 + x], rho);
      m2 += Uo[1 + x] * Uo[1 + x];
    }
    qo[0] = rho;
    qo[1] = (gamma - T(1)) * (Uo[D + 1] - T(0.5) * ke);
    qo[2] = Uo[D + 1];
    qo[3] = fsqrt(m2);
  }
  for (int k = 0; k < 4; ++k) {
    T g0 = T(0);
    for (int x = 0; x < D; ++x) g0 += dv[x] * gqc[k][x];
    g0 *= T(2);
    const T delta = qo[k] - qc[k];
    const T sd = g0 - delta;
    const T eps = T(1e-8) * (fabs(qc[k]) + fabs(qo[k])) + T(1e-30);
    const T beta = fdiv(fabs(sd - delta), fabs(sd) + fabs(delta) + eps);
    // eps^2 underflows in FP32 when both channel values are 0; the
    // ratio is then 0 (as in exact arithmetic, where Delta = 0 gives 0)
    const T den = delta * delta + eps * eps;
    T r = den > T(0) ? fdiv(sd * delta, den) : T(0);
    r = clampv(r, T(-2), T(2));
    A.mx_g0[k] = fmax(A.mx_g0[k], fabs(g0));
    A.mx_dl[k] = fmax(A.mx_dl[k], fabs(delta));
    A.mx_b[k] = fmax(A.mx_b[k], beta);
    A.sm_b[k] += beta;
    A.mn_r[k] = fmin(A.mn_r[k], r);
    A.mx_sd[k] = fmax(A.mx_sd[k], fabs(sd - delta));
    A.sm_dl[k] += fabs(delta);
  }
}

template <class T>
__device__ __forceinline__ void feat_finish(const T* qc, const FeatAcc<T>& A, float* feat) {
  const T inv = T(1) / (T)A.nface;
  for (int k = 0; k < 4; ++k) {
    const T rs = fdiv(T(1), fabs(qc[k]) + A.sm_dl[k] * inv + T(1e-8));
    T f[6] = {A.mx_g0[k] * rs, A.mx_dl[k] * rs, A.mx_b[k], A.sm_b[k] * inv, A.mn_r[k], A.mx_sd[k] * rs};
    for (int j = 0; j < 6; ++j) feat[6 * k + j] = (float)clampv(f[j], T(-8), T(8));
  }
}

// Gc: the cell's gradient [NV][D] (from memory or registers)
template <class T, int D>
__device__ void cell_features_from(const KArgs<T>& a, int64_t c, const T* Gc, float* feat,
                                   const T* Ulds = nullptr, int64_t c0 = 0, int n = 0) {
  constexpr int NV = D + 2;
  const int64_t b = c / KTPB;
  const int lane = (int)(c - b * KTPB);
  const int r0 = a.ell_ptr[b], m = (a.ell_ptr[b + 1] - r0) / KTPB;
  const int nfc = a.slot_ptr[c + 1] - a.slot_ptr[c];  // the cell's faces; records beyond are padding
  T qc[4], gqc[4][D];
  T Uc[NV];
  load_row<T, NV>(Uc, Ulds, a.U, c0, n, c);
  cell_channels<T, D>(Uc, Gc, a.gamma, qc, gqc);
  FeatAcc<T> A;
  A.init();
  // face records (sliced ELL) in batches of 4, then the batch's neighbour
  // rows; padding records (sigma = 0) are skipped
  constexpr int GB = 4;
  for (int j = 0; j < m; j += GB) {
    int64_t o[GB];
    T dv[GB][D], sg[GB];
#pragma unroll
    for (int jj = 0; jj < GB; ++jj) {
      const bool ok = j + jj < m;
      const int64_t r = (int64_t)r0 + (int64_t)(ok ? j + jj : j) * KTPB + lane;
      GlbPtr<T> rd = as_glb(a.ell_d + 3 * r);
#pragma unroll
      for (int x = 0; x < D; ++x) dv[jj][x] = rd[x];
      sg[jj] = (ok && j + jj < nfc) ? T(1) : T(0);
      o[jj] = ok ? rec_cell(a.ell_sw[4 * r + 3]) : c;
    }
    T Uo[GB][NV];
#pragma unroll
    for (int jj = 0; jj < GB; ++jj) load_row<T, NV>(Uo[jj], Ulds, a.U, c0, n, o[jj]);
#pragma unroll
    for (int jj = 0; jj < GB; ++jj) {
      if (sg[jj] == T(0)) continue;
      feat_face<T, D>(dv[jj], Uo[jj], a.gamma, qc, gqc, A);
    }
  }
  feat_finish<T>(qc, A, feat);
}

template <class T, int D>
__device__ __forceinline__ void cell_features(const KArgs<T>& a, int64_t c, float* feat) {
  cell_features_from<T, D>(a, c, a.G1 + c * (D + 2) * D, feat);
}

template <class T, int D>
__global__ __launch_bounds__(KTPB) void k_features(KArgs<T> a, float* __restrict__ X32,
                                                    unsigned short* __restrict__ Xb) {
  const int b = xcd_remap(blockIdx.x, a.cell_per_xcd, a.n_cell_blocks);
  if (b < 0) return;
  const int64_t c = (int64_t)b * KTPB + threadIdx.x;
  if (c >= a.nc) return;
  float f[MLP_IN];
  cell_features<T, D>(a, c, f);
  if (X32)
    for (int j = 0; j < MLP_IN; ++j) X32[c * MLP_IN + j] = f[j];
  if (Xb) {
    for (int j = 0; j < MLP_IN; ++j) Xb[c * MLP_INP + j] = f2bf(f[j]);
    for (int j = MLP_IN; j < MLP_INP; ++j) Xb[c * MLP_INP + j] = 0;
  }
}

// ---------------------------------------------------------------- forward
// Biases and output weights of the network (P: pointer type they are read
// through).
template <class P>
struct MlpVec {
  P b1, b2, w3;
  float b3;
};

__device__ __forceinline__ MlpVec<const float*> mlp_vec(const MlpDev& m) {
  return {m.p + OFF_B1, m.p + OFF_B2, m.p + OFF_W3, m.p[OFF_B3]};
}

// Forward of 16 cells with the K = 32 bf16 matrix instruction of gfx950
// (v_mfma_f32_16x16x32_bf16, half as many instructions as K = 16): lane
// group g = l / 16 holds 8 K slots of each operand.  Layer 1: slots 8g..8g+7
// are features 8g..8g+7 (g = 3: W1's zero padding, not read).  Layer 2 takes
// two accumulator tiles t = 2b, 2b + 1 as one K block b: slot 8g + i is
// hidden unit 32b + 4g + i and slot 8g + 4 + i unit 32b + 16 + 4g + i, the
// values lane l already holds; W2 is loaded in the same slot order, so the
// contraction pairs every unit with its own weight whatever order the
// instruction sums its K slots in.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                 0);
}

struct MlpRegs32 {
  v8s w1[4];     // output tile t: W1 rows 16t + l % 16, columns 8g..8g+7
  v8s w2[4][2];  // output tile t, K block b
};

__device__ __forceinline__ v8s load8(const unsigned short* p) {
  return __builtin_bit_cast(v8s, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ void load_weights32(const MlpDev& m, MlpRegs32& R) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, g = l >> 4;
  for (int t = 0; t < 4; ++t) {
    R.w1[t] = load8(m.w1b + (16 * t + r) * MLP_INP + 8 * g);
    for (int b = 0; b < 2; ++b) {
      const unsigned short* w = m.w2b + (16 * t + r) * MLP_H + 32 * b + 4 * g;
      v8s v;
      for (int i = 0; i < 4; ++i) {
        v[i] = (short)w[i];
        v[4 + i] = (short)w[16 + i];
      }
      R.w2[t][b] = v;
    }
  }
}

// theta of the 16 cells whose bf16 features are at X (row stride xstride,
// a multiple of 8, X 16-byte aligned; rows beyond nrow read as zero), for
// lane l's cell l % 16; optionally the hidden activations in accumulator
// layout (H1, H2: lane l holds units 16t + 4g + i of cell l % 16) and the
// logit z3, which the training kernel's backward uses.
// This lane's 8 input slots of the tile at X (zero beyond nrow rows and in
// the padding slots 24..31).
__device__ __forceinline__ v8s mlp_tile_input(const unsigned short* X, int nrow, int xstride) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, g = l >> 4;
  return (r < nrow && 8 * g < MLP_IN) ? load8(X + r * xstride + 8 * g) : v8s{0, 0, 0, 0, 0, 0, 0, 0};
}

template <class P>
__device__ __forceinline__ float mlp_tile_fwd32(const MlpVec<P>& m, const MlpRegs32& R, const unsigned short* X,
                                                int nrow, int xstride, v4f* H1 = nullptr, v4f* H2 = nullptr,
                                                float* z3out = nullptr);

// The same from inputs already loaded (xb: mlp_tile_input of the tile).
template <class P>
__device__ __forceinline__ float mlp_tile_fwd32_x(const MlpVec<P>& m, const MlpRegs32& R, v8s xb, v4f* H1 = nullptr,
                                                  v4f* H2 = nullptr, float* z3out = nullptr) {
  const int l = threadIdx.x & 63;
  const int g = l >> 4;
  v8s h1[2];
  for (int t = 0; t < 4; ++t) {
    v4f acc;
    for (int i = 0; i < 4; ++i) acc[i] = m.b1[16 * t + 4 * g + i];
    acc = mfma32(R.w1[t], xb, acc);
    v4f h;
    for (int i = 0; i < 4; ++i) {
      h[i] = fast_tanh(acc[i]);
      h1[t >> 1][4 * (t & 1) + i] = (short)f2bf(h[i]);
    }
    if (H1) H1[t] = h;
  }
  float part = 0.f;
  for (int t = 0; t < 4; ++t) {
    v4f acc;
    for (int i = 0; i < 4; ++i) acc[i] = m.b2[16 * t + 4 * g + i];
    for (int b = 0; b < 2; ++b) acc = mfma32(R.w2[t][b], h1[b], acc);
    v4f h;
    for (int i = 0; i < 4; ++i) {
      h[i] = fast_tanh(acc[i]);
      part += m.w3[16 * t + 4 * g + i] * h[i];
    }
    if (H2) H2[t] = h;
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  const float z3 = part + m.b3;
  if (z3out) *z3out = z3;
  return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(z3 * -1.4426950408889634f));
}

template <class P>
__device__ __forceinline__ float mlp_tile_fwd32(const MlpVec<P>& m, const MlpRegs32& R, const unsigned short* X,
                                                int nrow, int xstride, v4f* H1, v4f* H2, float* z3out) {
  return mlp_tile_fwd32_x(m, R, mlp_tile_input(X, nrow, xstride), H1, H2, z3out);
}

__global__ __launch_bounds__(256) void k_mlp_fwd(MlpDev m, const unsigned short* __restrict__ X, int64_t n,
                                                 float* __restrict__ theta, int xstride) {
  // biases and output weights in LDS, re-read at every tile (compiler
  // barrier below), the weight matrices in registers: fewer VGPRs, so the
  // kernel leaves room on each SIMD for the kernel it runs beside
  __shared__ float vb[3 * MLP_H + 4];
  for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) {
    vb[i] = m.p[OFF_B1 + i];
    vb[MLP_H + i] = m.p[OFF_B2 + i];
    vb[2 * MLP_H + i] = m.p[OFF_W3 + i];
  }
  if (threadIdx.x == 0) vb[3 * MLP_H] = m.p[OFF_B3];
  __syncthreads();
  MlpRegs32 R;
  load_weights32(m, R);
  const MlpVec<LdsPtr<float>> mv = {as_lds(vb), as_lds(vb + MLP_H), as_lds(vb + 2 * MLP_H), vb[3 * MLP_H]};
  const int l = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t ntile = (n + 15) / 16;
  // the next tile's inputs are loaded before this tile is computed, so the
  // load's latency overlaps the matrix and vector work of the tile
  auto rows = [&](int64_t t) { return (int)((n - t * 16) < 16 ? (n - t * 16) : 16); };
  v8s xb = wave < ntile ? mlp_tile_input(X + wave * 16 * xstride, rows(wave), xstride) : v8s{0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t t = wave; t < ntile; t += nwaves) {
    const int64_t row0 = t * 16;
    const int nrow = rows(t);
    const int64_t tn = t + nwaves;
    const v8s xn = tn < ntile ? mlp_tile_input(X + tn * 16 * xstride, rows(tn), xstride) : v8s{0, 0, 0, 0, 0, 0, 0, 0};
    __asm__ volatile("" ::: "memory");
    const float th = mlp_tile_fwd32_x(mv, R, xb, nullptr, nullptr, nullptr);
    if (l < nrow) theta[row0 + l] = th;
    xb = xn;
  }
}

// ---------------------------------------------------------------- backward
// Per-block partial gradients (packed parameter order) and partial loss.
// Rows [blk * rows_per_block, ...) of the batch; 4 waves per block.
__global__ __launch_bounds__(256) void k_mlp_grad(MlpDev m, const unsigned short* __restrict__ X,
                                                  const float* __restrict__ y, int64_t n, int rows_per_block,
                                                  float* __restrict__ part, float* __restrict__ loss_part) {
  // per wave, unit-major (unit * 16 + row) so that an operand's four rows
  // 4g..4g+3 of one unit are one 8-byte read
  __shared__ __align__(16) unsigned short sd2[4][16 * MLP_H];   // delta2 [u2][row], bf16
  __shared__ __align__(16) unsigned short sh1[4][16 * MLP_H];   // H1 [u1][row], bf16
  __shared__ __align__(16) unsigned short sd1[4][16 * MLP_H];   // delta1 [u1][row], bf16
  __shared__ float red[MLP_NPARAM + 1];
  MlpRegs32 R;
  load_weights32(m, R);
  const auto mv = mlp_vec(m);
  const int l = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r = l & 15, g = l >> 4;
  // W2^T in A layout for delta1 = W2^T delta2: A[m=u1][k=u2] = W2[u2][u1]
  // (K = 32 instruction: slot 8g + i of K block b is u2 = 32b + 4g + i and
  // slot 8g + 4 + i is u2 = 32b + 16 + 4g + i, the order in which each lane
  // holds delta2 in its two accumulator tiles 2b, 2b + 1)
  v8s w2t[4][2];
  for (int t = 0; t < 4; ++t)
    for (int b = 0; b < 2; ++b) {
      v8s v;
      for (int i = 0; i < 4; ++i) {
        v[i] = (short)m.w2b[(32 * b + 4 * g + i) * MLP_H + 16 * t + r];
        v[4 + i] = (short)m.w2b[(32 * b + 16 + 4 * g + i) * MLP_H + 16 * t + r];
      }
      w2t[t][b] = v;
    }
  v4f dW2[4][4], dW1[4][2];
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 4; ++b) dW2[a][b] = v4f{0, 0, 0, 0};
    for (int b = 0; b < 2; ++b) dW1[a][b] = v4f{0, 0, 0, 0};
  }
  float dW3[16], db2[16], db1[16], db3 = 0.f, lsum = 0.f;
  for (int k = 0; k < 16; ++k) dW3[k] = db2[k] = db1[k] = 0.f;
  const float invn = 1.f / (float)n;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  for (int64_t row0 = r0 + 16 * w; row0 < r1; row0 += 64) {
    const int nrow = (int)((r1 - row0) < 16 ? (r1 - row0) : 16);
    v4f H1[4], H2[4];
    float z3;
    const float th = mlp_tile_fwd32(mv, R, X + row0 * MLP_INP, nrow, MLP_INP, H1, H2, &z3);
    const bool valid = r < nrow;
    const float yy = valid ? y[row0 + r] : 0.f;
    const float g3 = valid ? (th - yy) * invn : 0.f;
    if (valid && g == 0) {  // BCE through the logit: softplus(z) - y z
      const float sp = fmaxf(z3, 0.f) + log1pf(expf(-fabsf(z3)));
      lsum += (sp - yy * z3) * invn;
    }
    if (g == 0) db3 += g3;
    // delta2 = g3 W3 (1 - H2^2) in D layout; write bf16 copies to LDS
    v4s d2b[4];
    for (int t = 0; t < 4; ++t) {
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * t + 4 * g + i;
        const float h2 = H2[t][i];
        dW3[4 * t + i] += g3 * h2;
        const float d2 = g3 * m.p[OFF_W3 + u] * (1.f - h2 * h2);
        db2[4 * t + i] += d2;
        const unsigned short bb = f2bf(d2);
        d2b[t][i] = (short)bb;
        sd2[w][u * 16 + r] = bb;
        sh1[w][u * 16 + r] = f2bf(H1[t][i]);
      }
    }
    // delta1 = (W2^T delta2) (1 - H1^2), two K = 32 blocks
    v8s d2k[2];
    for (int b = 0; b < 2; ++b)
      for (int i = 0; i < 4; ++i) {
        d2k[b][i] = d2b[2 * b][i];
        d2k[b][4 + i] = d2b[2 * b + 1][i];
      }
    for (int t = 0; t < 4; ++t) {
      v4f acc = v4f{0, 0, 0, 0};
      for (int b = 0; b < 2; ++b) acc = mfma32(w2t[t][b], d2k[b], acc);
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * t + 4 * g + i;
        const float h1 = H1[t][i];
        const float d1 = acc[i] * (1.f - h1 * h1);
        db1[4 * t + i] += d1;
        sd1[w][u * 16 + r] = f2bf(d1);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // B operands of the two weight-gradient products, which depend on the
    // column tile only: loaded once per row tile
    v4s Bh[4], Bx[2];
    for (int t2 = 0; t2 < 4; ++t2)
      Bh[t2] = *reinterpret_cast<const v4s*>(&sh1[w][(16 * t2 + r) * 16 + 4 * g]);
    for (int t2 = 0; t2 < 2; ++t2)
      for (int i = 0; i < 4; ++i) {
        const int rr = 4 * g + i;
        Bx[t2][i] = rr < nrow ? (short)X[(row0 + rr) * MLP_INP + 16 * t2 + r] : (short)0;
      }
    for (int t = 0; t < 4; ++t) {
      // dW2[u2][u1] += sum_rows delta2[row][u2] H1[row][u1]
      v4s A;
      A = *reinterpret_cast<const v4s*>(&sd2[w][(16 * t + r) * 16 + 4 * g]);
      for (int t2 = 0; t2 < 4; ++t2) dW2[t][t2] = mfma16(A, Bh[t2], dW2[t][t2]);
      // dW1[u1][k] += sum_rows delta1[row][u1] X[row][k]
      v4s A1;
      A1 = *reinterpret_cast<const v4s*>(&sd1[w][(16 * t + r) * 16 + 4 * g]);
      for (int t2 = 0; t2 < 2; ++t2) dW1[t][t2] = mfma16(A1, Bx[t2], dW1[t][t2]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  // block reduction of the four waves' partials in LDS (fixed order)
  for (int k = threadIdx.x; k < MLP_NPARAM + 1; k += blockDim.x) red[k] = 0.f;
  __syncthreads();
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
      for (int t = 0; t < 4; ++t) {
        for (int t2 = 0; t2 < 4; ++t2)
          for (int i = 0; i < 4; ++i) red[OFF_W2 + (16 * t + 4 * g + i) * MLP_H + 16 * t2 + r] += dW2[t][t2][i];
        for (int t2 = 0; t2 < 2; ++t2)
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * t2 + r;
            if (k < MLP_IN) red[OFF_W1 + (16 * t + 4 * g + i) * MLP_IN + k] += dW1[t][t2][i];
          }
      }
      // lane-local sums over the wave's cells: reduce lanes with equal g
      for (int k = 0; k < 16; ++k) {
        float a3 = dW3[k], a2 = db2[k], a1 = db1[k];
        for (int off = 1; off < 16; off <<= 1) {
          a3 += __shfl_xor(a3, off, 64);
          a2 += __shfl_xor(a2, off, 64);
          a1 += __shfl_xor(a1, off, 64);
        }
        if (r == 0) {
          const int u = 16 * (k >> 2) + 4 * g + (k & 3);
          red[OFF_W3 + u] += a3;
          red[OFF_B2 + u] += a2;
          red[OFF_B1 + u] += a1;
        }
      }
      float b3 = db3, ls = lsum;
      for (int off = 1; off < 64; off <<= 1) {
        b3 += __shfl_xor(b3, off, 64);
        ls += __shfl_xor(ls, off, 64);
      }
      if (l == 0) {
        red[OFF_B3] += b3;
        red[MLP_NPARAM] += ls;
      }
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < MLP_NPARAM; k += blockDim.x) part[(int64_t)blockIdx.x * MLP_NPARAM + k] = red[k];
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[MLP_NPARAM];
}

// Sum the per-block partial gradients (and, as index MLP_NPARAM, the
// partial losses): a block takes 32 parameters, its 8 slices of 32 threads
// sum every 8th partial (consecutive threads, consecutive parameters), then
// the slices are added in order, so the result is independent of timing.
// Optional Adam step on the fp32 master parameters with bf16 refresh of W1, W2.
constexpr int ADAM_K = 32, ADAM_SLICES = 8;
__global__ __launch_bounds__(256) void k_mlp_adam(int nparts, const float* __restrict__ part,
                                                  const float* __restrict__ loss_part, float* __restrict__ p,
                                                  float* __restrict__ mom, float* __restrict__ vel,
                                                  unsigned short* __restrict__ w1b, unsigned short* __restrict__ w2b,
                                                  float* __restrict__ grad_out, float* __restrict__ loss_out,
                                                  int do_step, float lr, float b1, float b2, float c1, float c2,
                                                  float eps) {
  __shared__ float sl_sum[ADAM_SLICES][ADAM_K];
  const int kk = threadIdx.x % ADAM_K, sl = threadIdx.x / ADAM_K;
  const int k = blockIdx.x * ADAM_K + kk;
  float acc = 0.f;
  if (k < MLP_NPARAM) {
    for (int b = sl; b < nparts; b += ADAM_SLICES) acc += part[(int64_t)b * MLP_NPARAM + k];
  } else if (k == MLP_NPARAM) {
    for (int b = sl; b < nparts; b += ADAM_SLICES) acc += loss_part[b];
  }
  sl_sum[sl][kk] = acc;
  __syncthreads();
  if (sl != 0 || k > MLP_NPARAM) return;
  float gsum = 0.f;
  for (int j = 0; j < ADAM_SLICES; ++j) gsum += sl_sum[j][kk];
  if (k == MLP_NPARAM) {
    if (loss_out) *loss_out = gsum;
    return;
  }
  if (grad_out) grad_out[k] = gsum;
  if (!do_step) return;
  const float mk = b1 * mom[k] + (1.f - b1) * gsum;
  const float vk = b2 * vel[k] + (1.f - b2) * gsum * gsum;
  mom[k] = mk;
  vel[k] = vk;
  const float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  p[k] = pk;
  if (k < OFF_B1) {
    const int u = k / MLP_IN, j = k % MLP_IN;
    w1b[u * MLP_INP + j] = f2bf(pk);
  } else if (k >= OFF_W2 && k < OFF_B2) {
    w2b[k - OFF_W2] = f2bf(pk);
  }
}

// New parameters: copied from the caller's device array, Adam moments cleared.
__global__ void k_mlp_set(const float* __restrict__ src, float* __restrict__ p, float* __restrict__ mom,
                          float* __restrict__ vel) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= MLP_NPARAM) return;
  p[k] = src[k];
  mom[k] = 0.f;
  vel[k] = 0.f;
}

__global__ void k_mlp_pack(const float* __restrict__ p, unsigned short* __restrict__ w1b,
                           unsigned short* __restrict__ w2b) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < MLP_H * MLP_INP) {
    const int u = k / MLP_INP, j = k % MLP_INP;
    w1b[k] = j < MLP_IN ? f2bf(p[OFF_W1 + u * MLP_IN + j]) : (unsigned short)0;
  }
  if (k < MLP_H * MLP_H) w2b[k] = f2bf(p[OFF_W2 + k]);
}

// First gradient and the indicator's features of a stage: the cell's
// Gauss-linear gradient is stored and, still in registers, feeds the 24
// features, written as bf16 rows 24 wide (48 bytes, coalesced) for the
// network's forward kernel.  The formulas of k_grad + k_features; compiled
// apart from them, so in FP32 a few features may round differently (FP64:
// the same bf16 rows).
template <class T, int D>
__global__ __launch_bounds__(KTPB) void k_grad_features(KArgs<T> a, T* __restrict__ G1out,
                                                         unsigned short* __restrict__ Xf) {
  constexpr int NV = D + 2;
  static_assert(MLP_IN % 8 == 0, "feature rows are stored in 16-byte pieces");
  __shared__ T ul[KTPB * NV];
  __shared__ T g1buf[KTPB * NV * D];
  const int b = xcd_remap(blockIdx.x, a.cell_per_xcd, a.n_cell_blocks);
  if (b < 0) return;
  const int64_t c0 = (int64_t)b * KTPB;
  const int ncl = (int)(a.nc - c0 < KTPB ? a.nc - c0 : KTPB);
  stage_rows(ul, a.U, c0, ncl, NV);
  __syncthreads();
  const int64_t c = c0 + threadIdx.x;
  T g[NV * D];
  if (c < a.nc) {
    const int r0 = a.ell_ptr[b], m = (a.ell_ptr[b + 1] - r0) / KTPB;  // faces per cell in this block
    const int nfc = a.slot_ptr[c + 1] - a.slot_ptr[c];                 // this cell's faces
    const T rv = a.rV[c];
    float f[MLP_IN];
    constexpr int FB = 6;
    if (m <= FB) {
      // one pass: the records (both kinds) and neighbour rows of all the
      // cell's faces are loaded once and serve the gradient, then the
      // features; the same operations in the same order as grad_sums and
      // cell_features_from
      const int lane = threadIdx.x;
      T q[NV];
      load_row<T, NV>(q, ul, a.U, c0, ncl, c);
      int64_t o[FB];
      T Sw[FB][D], dv[FB][D], sg[FB];
#pragma unroll
      for (int jj = 0; jj < FB; ++jj) {
        const bool ok = jj < m;
        const int64_t r = (int64_t)r0 + (int64_t)(ok ? jj : 0) * KTPB + lane;
        GlbPtr<T> rec = as_glb(a.ell_sw + 4 * r);
        GlbPtr<T> rd = as_glb(a.ell_d + 3 * r);
        T v[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) v[x] = rec[x];
        o[jj] = ok ? rec_cell(v[3]) : c;
#pragma unroll
        for (int x = 0; x < D; ++x) {
          Sw[jj][x] = ok ? v[x] : T(0);
          dv[jj][x] = rd[x];
        }
        sg[jj] = (ok && jj < nfc) ? T(1) : T(0);
      }
      T Uo[FB][NV];
#pragma unroll
      for (int jj = 0; jj < FB; ++jj) load_row<T, NV>(Uo[jj], ul, a.U, c0, ncl, o[jj]);
      T acc[NV][D];
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int x = 0; x < D; ++x) acc[k][x] = T(0);
#pragma unroll
      for (int jj = 0; jj < FB; ++jj)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          const T dq = Uo[jj][k] - q[k];
#pragma unroll
          for (int x = 0; x < D; ++x) acc[k][x] += dq * Sw[jj][x];
        }
      for (int k = 0; k < NV; ++k)
        for (int x = 0; x < D; ++x) g[k * D + x] = acc[k][x] * rv;
      T qc[4], gqc[4][D];
      cell_channels<T, D>(q, g, a.gamma, qc, gqc);
      FeatAcc<T> A;
      A.init();
#pragma unroll
      for (int jj = 0; jj < FB; ++jj)
        if (sg[jj] != T(0)) feat_face<T, D>(dv[jj], Uo[jj], a.gamma, qc, gqc, A);
      feat_finish<T>(qc, A, f);
    } else {
      T acc[NV][D];
      grad_sums<T, D, NV, 6>(a, a.U, c, acc, ul, c0, ncl);
      for (int k = 0; k < NV; ++k)
        for (int x = 0; x < D; ++x) g[k * D + x] = acc[k][x] * rv;
      cell_features_from<T, D>(a, c, g, f, ul, c0, ncl);
    }
    unsigned int w[MLP_IN / 2];
    for (int j = 0; j < MLP_IN / 2; ++j) w[j] = (unsigned)f2bf(f[2 * j]) | ((unsigned)f2bf(f[2 * j + 1]) << 16);
    uint4* dst = reinterpret_cast<uint4*>(Xf + c * MLP_IN);
    for (int q = 0; q < MLP_IN / 8; ++q) dst[q] = uint4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
  }
  store_rows_coalesced<T, NV * D>(G1out, c0, ncl, g, g1buf);
}

}  // namespace dolinc
