// Residual kernels, templated on the working type T (double or float).
//
// One residual evaluation (one Runge-Kutta stage) runs:
//   k_grad1  Gauss-linear gradient of U (Sec. 2.3), difference form
//            G1_P = V_P^-1 sum_f sigma S_f (phi_f - phi_P),
//            phi_f - phi_P = (1 - omega)(phi_N - phi_P) on the owner side and
//            omega (phi_P - phi_N) on the neighbour side.
//   k_grad2  the same operator on G1, symmetrised (USR5 only: its
//            differential phi^(2) = 4 d.G2.d sees only the symmetric part).
//   k_flux   per partition: every face entry evaluates the DOLINC
//            differentials (phi^(1) = 2 d.G1, phi^(2) = 4 d.G2.d), the
//            reconstructed left/right states in the DOLINC representation
//            (eq:USR3 / eq:CSR4 form: weight + explicit correction), the
//            optional blend with a Van Leer limited state, and the Riemann
//            flux; fluxes land in LDS.  After a barrier every cell of the
//            partition sums its faces' fluxes in a fixed order (no atomics)
//            and applies the update epilogue.
// Faces on a partition seam are evaluated by both partitions with identical
// operands and code, so both sides see bitwise identical fluxes and the
// scheme stays conservative to round-off.
#pragma once
#include <hip/hip_runtime.h>

#include "coefficients.hpp"
#include "internal.hpp"

namespace dolinc {

constexpr int KTPB = 256;

template <class T>
struct KArgs {
  int64_t nc, max_entries;
  int np, B, per_xcd, n_cell_blocks, cell_per_xcd;
  const int32_t* part_ptr;
  const int2* ent_pn;
  const int32_t* slot_ptr;
  const uint16_t* slots;
  const int32_t* ell_ptr;
  const T* sw;
  const T* ell_sw;
  const T* ell_d;
  const T* dc;
  const T* rV;
  const T* U;
  const T* G1;
  const T* Hf;          // [records][NV] second differentials contracted with the record's d
  const int2* ent_rec;  // [entries] record of the face in its owner / neighbour
  const uchar2* ent_j;  // [entries] the same as positions in the two cells' record lists, or null
  const float* theta;
  const T* Un;
  T* out;
  T alpha, beta, dt;
  int mode;
  T gamma;
  T adv[3];
  T bdir[3];
  T uref[5];
  const int32_t* face_ent;
  int64_t nf;
  T* eUL;
  T* eUR;
  T* eF;
  // positivity rule of the cell averages: per entry the face-side increments
  // [2][NV] (owner side, neighbour side), per cell the scaling theta
  T* estate;
  T* thpos;
};

// Partitions are handed out so that each XCD (workgroups go round-robin
// over the 8 XCDs) walks a contiguous range of partitions: neighbouring
// partitions share seam faces and gathered cells through that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int per_xcd, int n) {
  const int p = (b & 7) * per_xcd + (b >> 3);
  return p < n ? p : -1;
}

template <int PK, int D>
struct NVars {
  static constexpr int value = PK >= 2 ? D + 2 : 1;
};

template <int SCH>
struct SchemeInfo {
  static constexpr int ORD = SCH <= 2 ? 0 : (SCH <= 4 ? 1 : 2);
  static constexpr bool NONLIN = SCH == 6 || SCH == 7;  // ENO3, WENO5
};

// A partition's cells are a contiguous index range, so their rows of a
// per-cell array are staged into LDS with coalesced loads; a gathered row is
// then read from LDS when the cell is local and from global memory when it
// belongs to another partition (generic pointers pick the address space).
template <class T>
__device__ __forceinline__ void stage_rows(T* __restrict__ lds, const T* __restrict__ g, int64_t c0, int n, int w) {
  const int64_t base = c0 * w;
  for (int i = threadIdx.x; i < n * w; i += blockDim.x) lds[i] = g[base + i];
}

// Pointers with an explicit address space: the compiler may otherwise merge
// an LDS branch and an HBM branch into one generic (flat) load.
template <class T>
using LdsPtr = const T __attribute__((address_space(3)))*;
template <class T>
using GlbPtr = const T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ LdsPtr<T> as_lds(const T* p) {
  return (LdsPtr<T>)p;
}
template <class T>
__device__ __forceinline__ GlbPtr<T> as_glb(const T* p) {
  return (GlbPtr<T>)p;
}

// Copy row `row` (W values) into registers, from LDS when the row is one of
// the n staged rows starting at c0, else from HBM.
template <class T, int W>
__device__ __forceinline__ void load_row(T* dst, const T* lds, const T* __restrict__ g, int64_t c0, int n,
                                         int64_t row) {
  const int64_t r = row - c0;
  if (r >= 0 && r < n) {
    LdsPtr<T> src = as_lds(lds + r * W);
#pragma unroll
    for (int k = 0; k < W; ++k) dst[k] = src[k];
  } else {
    GlbPtr<T> src = as_glb(g + row * W);
#pragma unroll
    for (int k = 0; k < W; ++k) dst[k] = src[k];
  }
}

// out[v] = sum_x d_x row[v*D + x] for a row of NV*D values
template <class T, int NV, int D, class P>
__device__ __forceinline__ void contract1(P src, const T* d, T* out) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    T acc = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) acc += d[x] * src[v * D + x];
    out[v] = acc;
  }
}

// out[v] = d . sym(G2_v) . d for a row of NV * D(D+1)/2 values
template <class T, int NV, int D, class P>
__device__ __forceinline__ void contract2(P src, const T* d, T* out) {
  constexpr int NS2 = D * (D + 1) / 2;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    P h = src + v * NS2;
    T acc = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) acc += h[x] * d[x] * d[x];
    if constexpr (D == 3) {
      acc += h[3] * (T(2) * d[0] * d[1]) + h[4] * (T(2) * d[0] * d[2]) + h[5] * (T(2) * d[1] * d[2]);
    } else {
      acc += h[2] * (T(2) * d[0] * d[1]);
    }
    out[v] = acc;
  }
}

// FP32 quotient and square root on the hardware reciprocal / square-root
// units (about 1 ulp, no correction sequence); FP64 stays correctly rounded.
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double fsqrt(double a) { return sqrt(a); }

template <class T>
__device__ __forceinline__ T vanleer_inc(T s, T delta) {
  const T prod = s * delta;
  return prod > T(0) ? fdiv(T(2) * prod, s + delta) : T(0);
}

// Limited increment w_down * psi Delta (w_down = 1 - omega_0, the downwind
// cell's interpolation weight) with its magnitude capped at |Delta|: the
// limited face state stays between the two cell values also where the
// downwind cell is the nearer one (w_down > 1/2), where Van Leer's psi up to
// 2 would otherwise carry it past the downwind value.
template <class T>
__device__ __forceinline__ T limited_inc(T s, T delta, T w_down) {
  const T inc = w_down * vanleer_inc(s, delta);
  return fabs(inc) > fabs(delta) ? delta : inc;
}

// ---------------------------------------------------------------- Euler fluxes
template <class T, int D>
__device__ __forceinline__ void euler_prim(const T* U, T gamma, T& r, T* v, T& E, T& p) {
  r = U[0];
  T ke = T(0);
  for (int a = 0; a < D; ++a) {
    v[a] = fdiv(U[1 + a], r);
    ke += v[a] * U[1 + a];
  }
  E = U[D + 1];
  p = (gamma - T(1)) * (E - T(0.5) * ke);
}

template <class T, int D>
__device__ __forceinline__ void euler_phys(const T* U, T r, const T* v, T E, T p, const T* n, T* F) {
  T un = T(0);
  for (int a = 0; a < D; ++a) un += v[a] * n[a];
  F[0] = r * un;
  for (int a = 0; a < D; ++a) F[1 + a] = U[1 + a] * un + p * n[a];
  F[D + 1] = (E + p) * un;
}

template <class T, int D>
__device__ __forceinline__ void flux_rusanov(const T* UL, const T* UR, const T* S, T gamma, T* F) {
  T area2 = T(0);
  for (int a = 0; a < D; ++a) area2 += S[a] * S[a];
  const T area = fsqrt(area2);
  T rL, vL[D], EL, pL, rR, vR[D], ER, pR;
  euler_prim<T, D>(UL, gamma, rL, vL, EL, pL);
  euler_prim<T, D>(UR, gamma, rR, vR, ER, pR);
  T qL = T(0), qR = T(0);
  for (int a = 0; a < D; ++a) {
    qL += vL[a] * S[a];
    qR += vR[a] * S[a];
  }
  qL = fdiv(qL, area);
  qR = fdiv(qR, area);
  const T cL = fsqrt(fdiv(gamma * pL, rL)), cR = fsqrt(fdiv(gamma * pR, rR));
  const T lam = fmax(fabs(qL) + cL, fabs(qR) + cR);
  T FL[D + 2], FR[D + 2];
  euler_phys<T, D>(UL, rL, vL, EL, pL, S, FL);
  euler_phys<T, D>(UR, rR, vR, ER, pR, S, FR);
  const T diss = T(0.5) * lam * area;
  for (int k = 0; k < D + 2; ++k) F[k] = T(0.5) * (FL[k] + FR[k]) - diss * (UR[k] - UL[k]);
}

template <class T, int D>
__device__ __forceinline__ void flux_hllc(const T* UL, const T* UR, const T* S, T gamma, T* F) {
  T area2 = T(0);
  for (int a = 0; a < D; ++a) area2 += S[a] * S[a];
  const T area = fsqrt(area2);
  T n[D];
  for (int a = 0; a < D; ++a) n[a] = fdiv(S[a], area);
  T rL, vL[D], EL, pL, rR, vR[D], ER, pR;
  euler_prim<T, D>(UL, gamma, rL, vL, EL, pL);
  euler_prim<T, D>(UR, gamma, rR, vR, ER, pR);
  T qL = T(0), qR = T(0);
  for (int a = 0; a < D; ++a) {
    qL += vL[a] * n[a];
    qR += vR[a] * n[a];
  }
  const T cL = fsqrt(fdiv(gamma * pL, rL)), cR = fsqrt(fdiv(gamma * pR, rR));
  const T SL = fmin(qL - cL, qR - cR);
  const T SR = fmax(qL + cL, qR + cR);
  const T Ss = fdiv(pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR), rL * (SL - qL) - rR * (SR - qR));
  // choose the side: the flux is F_K (+ S_K (U*_K - U_K) inside the fan)
  const bool left = SL >= T(0) || Ss >= T(0);
  const T* UK = left ? UL : UR;
  const T rK = left ? rL : rR, EK = left ? EL : ER, pK = left ? pL : pR, qK = left ? qL : qR;
  const T SK = left ? SL : SR;
  T vK[D];
  for (int a = 0; a < D; ++a) vK[a] = left ? vL[a] : vR[a];
  T FK[D + 2];
  euler_phys<T, D>(UK, rK, vK, EK, pK, n, FK);
  const bool star = left ? (SL < T(0)) : (SR > T(0));
  if (star) {
    const T fac = fdiv(rK * (SK - qK), SK - Ss);
    T Us[D + 2];
    Us[0] = fac;
    for (int a = 0; a < D; ++a) Us[1 + a] = fac * (vK[a] + (Ss - qK) * n[a]);
    Us[D + 1] = fac * (fdiv(EK, rK) + (Ss - qK) * (Ss + fdiv(pK, rK * (SK - qK))));
    for (int k = 0; k < D + 2; ++k) FK[k] += SK * (Us[k] - UK[k]);
  }
  for (int k = 0; k < D + 2; ++k) F[k] = FK[k] * area;
}

// ---------------------------------------------------------------- reference-state (perturbation) fluxes
// With a constant reference state U_r, the states are carried as
// perturbations dU = U - U_r and the flux difference F(U) - F(U_r) is
// formed algebraically, so the O(1) part of the flux never appears in
// rounded arithmetic:
//   u - u_r = (dm - u_r drho) / rho,   dk = (dm.u + m_r.du) / 2,
//   dp = (gamma - 1)(dE - dk),
//   d(mass)   = dm.S
//   d(mom)    = dm (u.S) + m_r (du.S) + dp S
//   d(energy) = (dE + dp)(u.S) + (E_r + p_r)(du.S).
// Summed over a closed cell the dropped F(U_r).S terms cancel (sum of S = 0
// in the FP64 geometry), so the residual is unchanged.
template <class T, int D>
struct RefState {
  T r, m[D], u[D], E, p;
};

template <class T, int D>
__device__ __forceinline__ void ref_state(const T* uref, T gamma, RefState<T, D>& R) {
  R.r = uref[0];
  T k = T(0);
  for (int a = 0; a < D; ++a) {
    R.m[a] = uref[1 + a];
    R.u[a] = fdiv(uref[1 + a], uref[0]);
    k += R.m[a] * R.u[a];
  }
  R.E = uref[D + 1];
  R.p = (gamma - T(1)) * (R.E - T(0.5) * k);
}

template <class T, int D>
struct PertState {
  T r, u[D], du[D], dp, p;
};

template <class T, int D>
__device__ __forceinline__ void pert_state(const T* dU, const RefState<T, D>& R, T gamma, PertState<T, D>& P) {
  P.r = R.r + dU[0];
  T dk = T(0);
  for (int a = 0; a < D; ++a) {
    P.du[a] = fdiv(dU[1 + a] - R.u[a] * dU[0], P.r);
    P.u[a] = R.u[a] + P.du[a];
    dk += dU[1 + a] * P.u[a] + R.m[a] * P.du[a];
  }
  P.dp = (gamma - T(1)) * (dU[D + 1] - T(0.5) * dk);
  P.p = R.p + P.dp;
}

// F(U).n - F(U_r).n for the (not necessarily unit) vector n
template <class T, int D>
__device__ __forceinline__ void pert_flux(const T* dU, const PertState<T, D>& P, const RefState<T, D>& R, const T* n,
                                          T* dF) {
  T un = T(0), dun = T(0), dmn = T(0);
  for (int a = 0; a < D; ++a) {
    un += P.u[a] * n[a];
    dun += P.du[a] * n[a];
    dmn += dU[1 + a] * n[a];
  }
  dF[0] = dmn;
  for (int a = 0; a < D; ++a) dF[1 + a] = dU[1 + a] * un + R.m[a] * dun + P.dp * n[a];
  dF[D + 1] = (dU[D + 1] + P.dp) * un + (R.E + R.p) * dun;
}

template <class T, int D>
__device__ __forceinline__ void flux_rusanov_pert(const T* dL, const T* dR, const T* S, const T* uref, T gamma,
                                                  T* F) {
  RefState<T, D> R;
  ref_state<T, D>(uref, gamma, R);
  PertState<T, D> PL, PR;
  pert_state<T, D>(dL, R, gamma, PL);
  pert_state<T, D>(dR, R, gamma, PR);
  T area2 = T(0), qL = T(0), qR = T(0);
  for (int a = 0; a < D; ++a) {
    area2 += S[a] * S[a];
    qL += PL.u[a] * S[a];
    qR += PR.u[a] * S[a];
  }
  const T area = fsqrt(area2);
  qL = fdiv(qL, area);
  qR = fdiv(qR, area);
  const T cL = fsqrt(fdiv(gamma * PL.p, PL.r)), cR = fsqrt(fdiv(gamma * PR.p, PR.r));
  const T lam = fmax(fabs(qL) + cL, fabs(qR) + cR);
  T FL[D + 2], FR[D + 2];
  pert_flux<T, D>(dL, PL, R, S, FL);
  pert_flux<T, D>(dR, PR, R, S, FR);
  const T diss = T(0.5) * lam * area;
  for (int k = 0; k < D + 2; ++k) F[k] = T(0.5) * (FL[k] + FR[k]) - diss * (dR[k] - dL[k]);
}

// HLLC with every jump in difference form: S* - q_K from
//   S* - q_L = (dp_R - dp_L - a_R (q_R - q_L)) / (a_L - a_R),
//   S* - q_R = (dp_R - dp_L - a_L (q_R - q_L)) / (a_L - a_R),
// a_K = rho_K (S_K - q_K), and U*_K - U_K written as multiples of S* - q_K.
template <class T, int D>
__device__ __forceinline__ void flux_hllc_pert(const T* dL, const T* dR, const T* S, const T* uref, T gamma, T* F) {
  RefState<T, D> R;
  ref_state<T, D>(uref, gamma, R);
  PertState<T, D> PL, PR;
  pert_state<T, D>(dL, R, gamma, PL);
  pert_state<T, D>(dR, R, gamma, PR);
  T area2 = T(0);
  for (int a = 0; a < D; ++a) area2 += S[a] * S[a];
  const T area = fsqrt(area2);
  T n[D];
  for (int a = 0; a < D; ++a) n[a] = fdiv(S[a], area);
  T qL = T(0), qR = T(0), dqLR = T(0);
  for (int a = 0; a < D; ++a) {
    qL += PL.u[a] * n[a];
    qR += PR.u[a] * n[a];
    dqLR += (PR.du[a] - PL.du[a]) * n[a];
  }
  const T cL = fsqrt(fdiv(gamma * PL.p, PL.r)), cR = fsqrt(fdiv(gamma * PR.p, PR.r));
  const T SL = fmin(qL - cL, qR - cR);
  const T SR = fmax(qL + cL, qR + cR);
  const T aL = PL.r * (SL - qL), aR = PR.r * (SR - qR);
  const T dpLR = PR.dp - PL.dp;
  const T sL = fdiv(dpLR - aR * dqLR, aL - aR);  // S* - q_L
  const T sR = fdiv(dpLR - aL * dqLR, aL - aR);  // S* - q_R
  const T Ss = qL + sL;
  const bool left = SL >= T(0) || Ss >= T(0);
  const T* dK = left ? dL : dR;
  const PertState<T, D>& PK = left ? PL : PR;
  T FK[D + 2];
  pert_flux<T, D>(dK, PK, R, n, FK);
  const bool star = left ? (SL < T(0)) : (SR > T(0));
  if (star) {
    const T SK = left ? SL : SR;
    const T sK = left ? sL : sR;
    const T qK = left ? qL : qR;
    const T EK = R.E + dK[D + 1];
    const T fr = fdiv(PK.r * sK, SK - Ss);  // fac - rho_K
    const T fac = PK.r + fr;
    FK[0] += SK * fr;
    for (int a = 0; a < D; ++a) FK[1 + a] += SK * (fr * PK.u[a] + fac * sK * n[a]);
    FK[D + 1] += SK * (fdiv(fr * EK, PK.r) + fac * sK * (Ss + fdiv(PK.p, PK.r * (SK - qK))));
  }
  for (int k = 0; k < D + 2; ++k) F[k] = FK[k] * area;
}

// ---------------------------------------------------------------- ENO3 / WENO5 (end of Sec. 2.4)
// Template cells -2..2 of one side (cell 0 upwind, width 1, cell j of width
// gamma^j).  The coefficients of the three quadratics (stencils {0,1,2},
// {-1,0,1}, {-2,-1,0}) are closed forms of eq:coeff and of the derivatives
// of the fitted quadratic, as rational functions of gamma:
//   q_r : value at the face, s_r : slope at the centre of cell 0,
//   k_r : second derivative, w_r : linear weights that reproduce the 5-cell
//   coefficients.
template <class T>
struct NonlinCoef {
  T q[3][3], s[3][3], k[3][3], w[3], g, ig;
};

template <class T>
__device__ __forceinline__ void nonlin_coef(T g, NonlinCoef<T>& c) {
  const T g2 = g * g, g3 = g2 * g, g4 = g2 * g2;
  const T A = g + T(1), B = g2 + g + T(1);
  const T ig = fdiv(T(1), g), iB = fdiv(T(1), B), iAB = fdiv(T(1), A * B);
  const T iCQ = fdiv(T(1), (g2 + T(1)) * (g4 + g3 + g2 + g + T(1)));
  c.g = g;
  c.ig = ig;
  // r = 0: cells 0, 1, 2
  c.q[0][0] = g2 * iB;
  c.q[0][1] = (g2 + T(2) * g + T(2)) * iAB;
  c.q[0][2] = -iAB;
  c.s[0][0] = -(T(2) * g2 + T(4) * g + T(3)) * iAB;
  c.s[0][1] = (T(2) * g3 + T(4) * g2 + T(5) * g + T(1)) * ig * iAB;
  c.s[0][2] = -(T(2) * g + T(1)) * ig * iAB;
  c.k[0][0] = T(6) * iAB;
  c.k[0][1] = T(-6) * ig * iB;
  c.k[0][2] = T(6) * ig * iAB;
  // r = 1: cells -1, 0, 1
  c.q[1][0] = -g3 * iAB;
  c.q[1][1] = g * (T(2) * g2 + T(2) * g + T(1)) * iAB;
  c.q[1][2] = iB;
  c.s[1][0] = -g2 * (T(2) * g + T(1)) * iAB;
  c.s[1][1] = (g - T(1)) * (T(2) * g2 + T(3) * g + T(2)) * iAB;
  c.s[1][2] = (g + T(2)) * iAB;
  c.k[1][0] = T(6) * g2 * iAB;
  c.k[1][1] = T(-6) * g * iB;
  c.k[1][2] = T(6) * g * iAB;
  // r = 2: cells -2, -1, 0
  c.q[2][0] = g3 * iB;
  c.q[2][1] = -g * (g3 + T(3) * g2 + T(2) * g + T(1)) * iAB;
  c.q[2][2] = (T(3) * g3 + T(4) * g2 + T(3) * g + T(1)) * iAB;
  c.s[2][0] = g3 * (g + T(2)) * iAB;
  c.s[2][1] = -g * (g3 + T(5) * g2 + T(4) * g + T(2)) * iAB;
  c.s[2][2] = g * (T(3) * g2 + T(4) * g + T(2)) * iAB;
  c.k[2][0] = T(6) * g4 * iAB;
  c.k[2][1] = T(-6) * g3 * iB;
  c.k[2][2] = T(6) * g3 * iAB;
  c.w[0] = B * iCQ;
  c.w[1] = g2 * A * B * iCQ;
  c.w[2] = g3 * g3 * iCQ;
}

// Face value at the right edge of cell 0 from the upwind cell values
// a0 = phi_0, a1 = phi_1 and the DOLINC differentials D0 = phi_0^(1),
// D1 = phi_1^(1), E0 = phi_0^(2) of this side's frame.  Far cells by the
// recursions of Sec. 2.3 (eq:diffDLC and its one-sided forms).
template <class T, int SCH>
__device__ __forceinline__ T nonlin_side(const NonlinCoef<T>& c, T a0, T a1, T D0, T D1, T E0) {
  const T g = c.g, ig = c.ig;
  const T pm1 = (a1 - D0) * ig + (T(1) - ig) * a0;
  const T pm1_1 = (D1 - E0) * ig + (T(1) - ig) * D0;
  const T pm2 = (a0 - pm1_1 * ig) * ig + (T(1) - ig) * pm1;
  const T p2 = g * (a0 + D1) + (T(1) - g) * a1;
  const T f[3][3] = {{a0, a1, p2}, {pm1, a0, a1}, {pm2, pm1, a0}};  // stencil r: cells -r .. 2-r
  if constexpr (SCH == 6) {
    // Harten's choice with the undivided differences printed for ENO3
    const T left2 = g * (a0 - pm1), right2 = a1 - a0;
    const T d3m2 = g * g * (a0 - (T(1) + g) * pm1 + g * pm2);
    const T d3m1 = a1 - (T(1) + g) * a0 + g * pm1;
    const T d3p0 = ig * ig * (p2 - (T(1) + g) * a1 + g * a0);
    // the upwind candidate must be smaller by a relative margin above the
    // working precision's rounding (1e-10 FP64, 1e-5 FP32): exact ties (a
    // boundary's mirror symmetry makes them) go downwind whatever the rounding
    const T keep = T(1) - (sizeof(T) == 4 ? T(1e-5) : T(1e-10));
    int r;
    if (fabs(left2) < keep * fabs(right2))
      r = fabs(d3m2) < keep * fabs(d3m1) ? 2 : 1;
    else
      r = fabs(d3m1) < keep * fabs(d3p0) ? 1 : 0;
    T out = T(0);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
      if (rr == r) out = c.q[rr][0] * f[rr][0] + c.q[rr][1] * f[rr][1] + c.q[rr][2] * f[rr][2];
    return out;
  } else {
    T num = T(0), den = T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const T q = c.q[r][0] * f[r][0] + c.q[r][1] * f[r][1] + c.q[r][2] * f[r][2];
      const T sl = c.s[r][0] * f[r][0] + c.s[r][1] * f[r][1] + c.s[r][2] * f[r][2];
      const T kk = c.k[r][0] * f[r][0] + c.k[r][1] * f[r][1] + c.k[r][2] * f[r][2];
      const T beta = sl * sl + T(13.0 / 12.0) * kk * kk;
      const T e = T(1e-6) + beta;
      const T alpha = fdiv(c.w[r], e * e);
      num += alpha * q;
      den += alpha;
    }
    return fdiv(num, den);
  }
}

// ---------------------------------------------------------------- face evaluation
// Loads one face entry, reconstructs (U_L, U_R) and returns the
// face-integrated flux F.S (owner -> neighbour).  Cell rows are gathered
// straight from HBM/L2: staging the partition's own rows in LDS cost more in
// occupancy and barriers than it saved.
// REF picks the state the face arithmetic is carried about:
//   0  none: full states;
//   1  (Euler) a constant reference state a.uref: perturbations U - U_ref, flux
//      F(U).S - F(U_ref).S (the dropped terms cancel over closed cells);
//   2  each face side's own cell: the states are carried as increments over
//      the owner's value U_P, the flux as G_P = F.S - F(U_P).S, and the
//      neighbour's share as G_N = F.S - F(U_N).S = G_P - (F(U_N) - F(U_P)).S
//      (difference form).  Cell c sums sigma G_c over its faces; the dropped
//      F(U_c).sum(sigma S) vanishes with the FP64 geometry.  The rounded
//      quantities are then O(h) increments instead of O(1) fluxes: in FP32
//      the rounding of S and of the flux arithmetic enters only through
//      F - F(U_c).  Every law: Euler through the perturbation fluxes,
//      advection and Burgers in closed increment forms below.
// The reconstruction, blend and nonlinear schemes are affine in the cell
// values (coefficients summing to one, differences elsewhere), so they run
// unchanged on the shifted values.  F receives the owner's share (REF 2:
// G_P) and, for REF 2 only, F2 the neighbour's (G_N); with REF 0 / 1 one
// flux serves both cells.
// MODE (Euler with the positivity rule of the cell averages): 0 the whole
// face; 1 the face-side states only, returned as increments over their own
// cells (UL - U_P, UR - U_N) for the per-cell scaling; 2 the flux from the
// scaled increments a.estate, a.thpos (the first pass's output).
template <class T, int D, int PK, int SCH, bool BLEND, int REF = 0, int MODE = 0>
__device__ __forceinline__ void eval_face(const KArgs<T>& a, int64_t e, T* UL, T* UR, T* F, T* F2 = nullptr) {
  constexpr int NV = NVars<PK, D>::value;
  static_assert(REF != 1 || PK >= 2, "the constant reference state is built for the Euler equations");
  static_assert(MODE == 0 || PK >= 2, "the positivity rule is built for the Euler equations");
  constexpr int ORD = SchemeInfo<SCH>::ORD;
  constexpr int DCS = DC_VALUES;  // d per face entry
  const int2 pn = a.ent_pn[e];
  const int64_t P = pn.x, N = pn.y;
  const T* swp = a.sw + 4 * e;
  T S[3] = {swp[0], swp[1], swp[2]};
  const T om = swp[3];
  const T* dcp = a.dc + (int64_t)DCS * e;
  T dc[DCS];
#pragma unroll
  for (int k = 0; k < DCS; ++k) dc[k] = dcp[k];
  T uP[NV], uN[NV], base[NV];
  {
    GlbPtr<T> up = as_glb(a.U + P * NV);
    GlbPtr<T> un = as_glb(a.U + N * NV);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uP[v] = up[v];
      uN[v] = un[v];
    }
  }
  // shift by the reference: the constant state (REF 1) or the owner's value
  // (REF 2: the owner's shifted value is exactly zero)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (REF == 1) {
      base[v] = a.uref[v];
      uP[v] -= base[v];
      uN[v] -= base[v];
    } else if constexpr (REF == 2) {
      base[v] = uP[v];
      uN[v] -= base[v];
      uP[v] = T(0);
    } else {
      base[v] = T(0);
    }
  }
  if constexpr (MODE == 2) {
    // the scaled face-side states: own value + theta_pos x increment
    const T* es = a.estate + (int64_t)2 * NV * e;
    const T tp = a.thpos[P], tn = a.thpos[N];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      UL[v] = uP[v] + tp * es[v];
      UR[v] = uN[v] + tn * es[NV + v];
    }
  } else {
  T gP[NV], gN[NV], hP[NV], hN[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) gP[v] = gN[v] = hP[v] = hN[v] = T(0);
  if constexpr (ORD >= 1 || BLEND) {
    contract1<T, NV, D>(as_glb(a.G1 + P * NV * D), dc, gP);
    contract1<T, NV, D>(as_glb(a.G1 + N * NV * D), dc, gN);
  }
  if constexpr (ORD >= 2) {  // d.H.d of both cells, written per face record by the second-derivative kernel
    // the records from their positions in the cells' lists (2 bytes per
    // entry instead of 8; the block offsets are a small cached array)
    static_assert(ELL_BLOCK == KTPB, "cell blocks of the record lists are workgroups of the cell kernels");
    int64_t rP, rN;
    if (a.ent_j) {
      const uchar2 j = a.ent_j[e];
      rP = (int64_t)a.ell_ptr[P / KTPB] + (int64_t)j.x * KTPB + P % KTPB;
      rN = (int64_t)a.ell_ptr[N / KTPB] + (int64_t)j.y * KTPB + N % KTPB;
    } else {
      const int2 rc = a.ent_rec[e];
      rP = rc.x;
      rN = rc.y;
    }
    GlbPtr<T> hp = as_glb(a.Hf + rP * NV);
    GlbPtr<T> hn = as_glb(a.Hf + rN * NV);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      hP[v] = hp[v];
      hN[v] = hn[v];
    }
  }
  // reconstruction in the DOLINC representation (coefficients from precompute)
  if constexpr (SchemeInfo<SCH>::NONLIN) {
    // left state: frame P -> N, growth g; right state: frame N -> P,
    // growth 1/g, d -> -d (odd differentials change sign)
    NonlinCoef<T> cf;
    // growth rate of the P -> N frame from the owner's weight, in FP64
    const double gd = (double)om / (1.0 - (double)om);
    nonlin_coef<T>((T)gd, cf);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      UL[v] = nonlin_side<T, SCH>(cf, uP[v], uN[v], T(2) * gP[v], T(2) * gN[v], T(4) * hP[v]);
    nonlin_coef<T>((T)((1.0 - (double)om) / (double)om), cf);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      UR[v] = nonlin_side<T, SCH>(cf, uN[v], uP[v], T(-2) * gN[v], T(-2) * gP[v], T(4) * hN[v]);
  } else {
    // coefficients of both sides from the growth rate g = omega / (1 - omega)
    // of the P -> N frame, in FP64 (one reciprocal per side), rounded once
    // to the working type
    double cd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    face_coefficients(SCH, (double)om, cd);
    T c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = (T)cd[k];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (SCH <= 2) {
        UL[v] = uN[v] + c[0] * (uP[v] - uN[v]);
        UR[v] = uP[v] + c[1] * (uN[v] - uP[v]);
      } else if constexpr (SCH == 3) {
        UL[v] = uN[v] + c[0] * (uP[v] - uN[v]) + c[1] * gP[v];
        UR[v] = uP[v] + c[2] * (uN[v] - uP[v]) + c[3] * gN[v];
      } else if constexpr (SCH == 4) {
        UL[v] = uN[v] + c[0] * (uP[v] - uN[v]) + c[1] * gP[v] + c[2] * gN[v];
        UR[v] = UL[v];
      } else if constexpr (SCH == 8) {  // CSR6: symmetric template, both second differentials
        UL[v] = uN[v] + c[0] * (uP[v] - uN[v]) + c[1] * gP[v] + c[2] * gN[v] + c[3] * hP[v] + c[4] * hN[v];
        UR[v] = UL[v];
      } else {
        UL[v] = uN[v] + c[0] * (uP[v] - uN[v]) + c[1] * gP[v] + c[2] * gN[v] + c[3] * hP[v];
        UR[v] = uP[v] + c[4] * (uN[v] - uP[v]) + c[5] * gN[v] + c[6] * gP[v] + c[7] * hN[v];
      }
    }
  }
  if constexpr (BLEND) {
    const float thP = as_glb(a.theta)[P], thN = as_glb(a.theta)[N];
    const T tf = (T)fminf(thP, thN);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T dL = uN[v] - uP[v];
      const T VL = uP[v] + limited_inc(T(2) * gP[v] - dL, dL, T(1) - om);
      const T dR = uP[v] - uN[v];
      const T VR = uN[v] + limited_inc(T(-2) * gN[v] - dR, dR, om);
      UL[v] = tf * UL[v] + (T(1) - tf) * VL;
      UR[v] = tf * UR[v] + (T(1) - tf) * VR;
    }
  }
  }  // MODE != 2
  if constexpr (PK == 0) {
    T an = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) an += a.adv[x] * S[x];
    // REF 2: the states are increments over U_P, so this is the owner's
    // share an (U_up - U_P); the neighbour's subtracts an (U_N - U_P)
    F[0] = an >= T(0) ? an * UL[0] : an * UR[0];
    if constexpr (REF == 2) {
      F2[0] = F[0] - an * uN[0];
      UL[0] += base[0];
      UR[0] += base[0];
    }
  } else if constexpr (PK == 1) {
    T s = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) s += a.bdir[x] * S[x];
    if constexpr (REF == 2) {
      // Godunov's choice among f(u_L), f(u_R) and f(0) (when u = 0 lies
      // between them), f(u) = u^2/2 s, taken among the same values less
      // f(U_P), each formed from its increment: f(U_P + i) - f(U_P) =
      // i (i + 2 U_P) s / 2.  The neighbour's share subtracts
      // f(U_N) - f(U_P) in the same form.
      const T b = base[0];
      const T iL = UL[0], iR = UR[0];
      const T uL = iL + b, uR = iR + b;
      const T dL = T(0.5) * iL * (iL + T(2) * b) * s, dR = T(0.5) * iR * (iR + T(2) * b) * s;
      const T lo = fmin(uL, uR), hi = fmax(uL, uR);
      const bool has0 = lo <= T(0) && hi >= T(0);
      T dmn = fmin(dL, dR), dmx = fmax(dL, dR);
      if (has0) {
        const T d0 = T(-0.5) * b * b * s;
        dmn = fmin(dmn, d0);
        dmx = fmax(dmx, d0);
      }
      F[0] = iL <= iR ? dmn : dmx;
      const T iN = uN[0];
      F2[0] = F[0] - T(0.5) * iN * (iN + T(2) * b) * s;
      UL[0] = uL;
      UR[0] = uR;
    } else {
      const T uL = UL[0], uR = UR[0];
      const T fL = T(0.5) * uL * uL * s, fR = T(0.5) * uR * uR * s;
      const T lo = fmin(uL, uR), hi = fmax(uL, uR);
      const bool has0 = lo <= T(0) && hi >= T(0);
      T fmn = fmin(fL, fR), fmx = fmax(fL, fR);
      if (has0) {
        fmn = fmin(fmn, T(0));
        fmx = fmax(fmx, T(0));
      }
      F[0] = uL <= uR ? fmn : fmx;
    }
  } else if constexpr (REF == 0) {
    // positivity: a side with rho <= 0 or p <= 0 falls back to its cell value
    if constexpr (MODE != 2) {
      T r, vv[D], E, p;
      euler_prim<T, D>(UL, a.gamma, r, vv, E, p);
      if (!(r > T(0) && p > T(0)))
        for (int v = 0; v < NV; ++v) UL[v] = uP[v];
      euler_prim<T, D>(UR, a.gamma, r, vv, E, p);
      if (!(r > T(0) && p > T(0)))
        for (int v = 0; v < NV; ++v) UR[v] = uN[v];
    }
    if constexpr (MODE == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UL[v] -= uP[v];
        UR[v] -= uN[v];
      }
      return;
    }
    if constexpr (PK == 2)
      flux_rusanov<T, D>(UL, UR, S, a.gamma, F);
    else
      flux_hllc<T, D>(UL, UR, S, a.gamma, F);
  } else {
    RefState<T, D> Rf;
    ref_state<T, D>(base, a.gamma, Rf);
    if constexpr (MODE != 2) {
      PertState<T, D> Ps;
      pert_state<T, D>(UL, Rf, a.gamma, Ps);
      if (!(Ps.r > T(0) && Ps.p > T(0)))
        for (int v = 0; v < NV; ++v) UL[v] = uP[v];
      pert_state<T, D>(UR, Rf, a.gamma, Ps);
      if (!(Ps.r > T(0) && Ps.p > T(0)))
        for (int v = 0; v < NV; ++v) UR[v] = uN[v];
    }
    if constexpr (MODE == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UL[v] -= uP[v];
        UR[v] -= uN[v];
      }
      return;
    }
    if constexpr (PK == 2)
      flux_rusanov_pert<T, D>(UL, UR, S, base, a.gamma, F);
    else
      flux_hllc_pert<T, D>(UL, UR, S, base, a.gamma, F);
    if constexpr (REF == 2) {
      // the neighbour's share: G_N = G_P - (F(U_N) - F(U_P)).S
      PertState<T, D> PN;
      pert_state<T, D>(uN, Rf, a.gamma, PN);
      T dF[D + 2];
      pert_flux<T, D>(uN, PN, Rf, S, dF);
#pragma unroll
      for (int v = 0; v < NV; ++v) F2[v] = F[v] - dF[v];
    }
    // exported states are full states
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      UL[v] += base[v];
      UR[v] += base[v];
    }
  }
}

// ---------------------------------------------------------------- kernels
template <class T, int D, int PK, int SCH, bool BLEND, int REF, int MODE, int TPB = KTPB>
__global__ __launch_bounds__(TPB) void k_flux(KArgs<T> a) {
  constexpr int NV = NVars<PK, D>::value;
  constexpr int FW = REF == 2 ? 2 * NV : NV;  // values per entry in LDS (REF 2: owner's, neighbour's share)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int p = xcd_remap(blockIdx.x, a.per_xcd, a.np);
  if (p < 0) return;
  const int64_t c0 = (int64_t)p * a.B;
  const int ncl = (int)(a.nc - c0 < a.B ? a.nc - c0 : a.B);
  // LDS: the partition's face fluxes
  T* Fs = reinterpret_cast<T*>(smem_raw);
  const int e0 = a.part_ptr[p], e1 = a.part_ptr[p + 1];
  for (int e = e0 + (int)threadIdx.x; e < e1; e += TPB) {
    T UL[NV], UR[NV], F[FW];
    eval_face<T, D, PK, SCH, BLEND, REF, MODE>(a, e, UL, UR, F, F + (REF == 2 ? NV : 0));
#pragma unroll
    for (int v = 0; v < FW; ++v) Fs[(e - e0) * FW + v] = F[v];
  }
  __syncthreads();
  const int64_t c1 = c0 + ncl;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += TPB) {
    const int s0 = a.slot_ptr[c], s1 = a.slot_ptr[c + 1];
    T sum[NV], comp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sum[v] = comp[v] = T(0);
    for (int s = s0; s < s1; ++s) {
      const uint16_t sl = a.slots[s];
      const bool nb = (sl >> 15) != 0;
      const T* Fp = Fs + (sl & 0x7fff) * FW + (REF == 2 && nb ? NV : 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T x = nb ? -Fp[v] : Fp[v];
        if constexpr (sizeof(T) == 4) {  // Neumaier compensated sum
          const T t = sum[v] + x;
          comp[v] += fabs(sum[v]) >= fabs(x) ? (sum[v] - t) + x : (x - t) + sum[v];
          sum[v] = t;
        } else {
          sum[v] += x;
        }
      }
    }
    const T rv = a.rV[c];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T R = -(sum[v] + comp[v]) * rv;
      const int64_t i = c * NV + v;
      if (a.mode == 0) {
        a.out[i] = R;
      } else {
        const T un = a.Un ? a.Un[i] : T(0);
        a.out[i] = a.alpha * un + a.beta * (a.U[i] + a.dt * R);
      }
    }
  }
}

// Positivity rule of the cell averages, first pass (Euler): per partition,
// every entry's face-side states as increments over their own cells
// (written to a.estate and kept in LDS with the face area), then for every
// cell of the partition theta_pos, the largest theta in [0, 1] for which
// U* = U_c - theta sum_f a_f e_{c,f} keeps rho >= 1e-6 rho_c and
// p >= 1e-6 p_c (a_f = |S_f| / sum |S|; e_{c,f} the cell's face-side
// increments): 1 when theta = 1 qualifies, else the smaller of the density's
// linear root and the pressure's first positive root of
//   f(theta) = rho* (E* - k) - |m*|^2 / 2,  k = 1e-6 p_c / (gamma - 1).
// With the scaled states U_c + theta_pos e_{c,f} the forward Euler update is
// a convex combination of admissible Lax-Friedrichs updates when
// dt lambda sum |S| / V <= 1/2.  Seam entries are evaluated identically by
// both partitions, so each cell sees all of its face-side states here.
template <class T, int D, int PK, int SCH, bool BLEND, int REF>
__global__ __launch_bounds__(KTPB) void k_pos_states(KArgs<T> a) {
  constexpr int NV = NVars<PK, D>::value;
  constexpr int EW = 2 * NV + 1;  // LDS per entry: both sides' increments, the area
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int p = xcd_remap(blockIdx.x, a.per_xcd, a.np);
  if (p < 0) return;
  const int64_t c0 = (int64_t)p * a.B;
  const int ncl = (int)(a.nc - c0 < a.B ? a.nc - c0 : a.B);
  T* Es = reinterpret_cast<T*>(smem_raw);
  const int e0 = a.part_ptr[p], e1 = a.part_ptr[p + 1];
  for (int e = e0 + (int)threadIdx.x; e < e1; e += KTPB) {
    T eL[NV], eR[NV], F[NV];
    eval_face<T, D, PK, SCH, BLEND, REF, 1>(a, e, eL, eR, F);
    const T* sw = a.sw + 4 * (int64_t)e;
    const T area = fsqrt(sw[0] * sw[0] + sw[1] * sw[1] + sw[2] * sw[2]);
    T* es = a.estate + (int64_t)2 * NV * e;
    T* ls = Es + (e - e0) * EW;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      es[v] = eL[v];
      es[NV + v] = eR[v];
      ls[v] = eL[v];
      ls[NV + v] = eR[v];
    }
    ls[2 * NV] = area;
  }
  __syncthreads();
  const int64_t c1 = c0 + ncl;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += KTPB) {
    const int s0 = a.slot_ptr[c], s1 = a.slot_ptr[c + 1];
    T db[NV], tot = T(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) db[v] = T(0);
    for (int s = s0; s < s1; ++s) {
      const uint16_t sl = a.slots[s];
      const bool nb = (sl >> 15) != 0;
      const T* ls = Es + (sl & 0x7fff) * EW;
      const T ar = ls[2 * NV];
      tot += ar;
#pragma unroll
      for (int v = 0; v < NV; ++v) db[v] += ar * ls[(nb ? NV : 0) + v];
    }
    const T it = fdiv(T(1), tot);
#pragma unroll
    for (int v = 0; v < NV; ++v) db[v] *= it;
    // theta_pos of the cell
    const T* U = a.U + c * NV;
    T r, vv[D], E, pc;
    euler_prim<T, D>(U, a.gamma, r, vv, E, pc);
    constexpr double DEL = 1e-6;
    const T k = T(DEL) * pc / (a.gamma - T(1));
    T mm = T(0), md = T(0), dd = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) {
      mm += U[1 + x] * U[1 + x];
      md += U[1 + x] * db[1 + x];
      dd += db[1 + x] * db[1 + x];
    }
    const T dr = db[0], dE = db[D + 1];
    const T r1 = r - dr, E1 = E - dE;
    T m1 = T(0);
#pragma unroll
    for (int x = 0; x < D; ++x) m1 += (U[1 + x] - db[1 + x]) * (U[1 + x] - db[1 + x]);
    T th = T(1);
    if (!(r1 >= T(DEL) * r && r1 * (E1 - k) - T(0.5) * m1 >= T(0))) {
      T th_r = T(1);
      if (dr > T(0)) th_r = fmin(T(1), fdiv((T(1) - T(DEL)) * r, dr));
      const T A = dr * dE - T(0.5) * dd;
      const T B = -r * dE - dr * (E - k) + md;
      const T C = r * (E - k) - T(0.5) * mm;
      const T disc = fmax(B * B - T(4) * A * C, T(0));
      const T q = T(-0.5) * (B + (B >= T(0) ? T(1) : T(-1)) * fsqrt(disc));
      T th_p = T(1);
      if (A != T(0)) {
        const T ra = fdiv(q, A);
        if (ra > T(0)) th_p = fmin(th_p, ra);
      }
      if (q != T(0)) {
        const T rb = fdiv(C, q);
        if (rb > T(0)) th_p = fmin(th_p, rb);
      }
      th = fmin(th_r, th_p);
    }
    a.thpos[c] = th;
  }
}

template <class T, int D, int PK, int SCH, bool BLEND, int REF>
__global__ __launch_bounds__(KTPB) void k_face_export(KArgs<T> a) {
  constexpr int NV = NVars<PK, D>::value;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.nf) return;
  T UL[NV], UR[NV], F[NV], F2[NV];
  if constexpr (PK >= 2) {
    if (a.estate)  // the positivity rule's first pass has run: its scaled states
      eval_face<T, D, PK, SCH, BLEND, REF, 2>(a, a.face_ent[f], UL, UR, F, F2);
    else
      eval_face<T, D, PK, SCH, BLEND, REF, 0>(a, a.face_ent[f], UL, UR, F, F2);
  } else {
    eval_face<T, D, PK, SCH, BLEND, REF, 0>(a, a.face_ent[f], UL, UR, F, F2);
  }
  if constexpr (REF == 1 || REF == 2) {
    // the full face flux F.S: add back the reference state's physical flux
    // (rounded in the working precision; export only)
    const T* st = REF == 1 ? a.uref : a.U + (int64_t)a.ent_pn[a.face_ent[f]].x * NV;
    const T* sw = a.sw + 4 * (int64_t)a.face_ent[f];
    if constexpr (PK >= 2) {
      T r, vv[D], E, p, Fr[NV];
      euler_prim<T, D>(st, a.gamma, r, vv, E, p);
      euler_phys<T, D>(st, r, vv, E, p, sw, Fr);
      for (int v = 0; v < NV; ++v) F[v] += Fr[v];
    } else {
      T vs = T(0);
      for (int x = 0; x < D; ++x) vs += (PK == 0 ? a.adv[x] : a.bdir[x]) * sw[x];
      F[0] += PK == 0 ? vs * st[0] : T(0.5) * st[0] * st[0] * vs;
    }
  }
  for (int v = 0; v < NV; ++v) {
    a.eUL[f * NV + v] = UL[v];
    a.eUR[f * NV + v] = UR[v];
    if (a.eF) a.eF[f * NV + v] = F[v];
  }
}

// Other cell named by a face record (index bits stored in the 4th slot).
__device__ __forceinline__ int64_t rec_cell(float v) { return (int64_t)__float_as_int(v); }
__device__ __forceinline__ int64_t rec_cell(double v) { return (int64_t)__double_as_longlong(v); }

// Cell-centric Gauss-linear gradient of phi [nc][NQ] -> out [nc][NQ][D].
// SYM: NQ = NV*D input components (a gradient) and the output is the
// symmetrised second derivative [nc][NV][D(D+1)/2].
// Gauss-linear sums of cell c: acc[k][x] = sum_f sigma S_f,x w (phi_o - phi_c)_k
// The cell's face records (sliced ELL: the lanes of a wave read consecutive
// records) are taken GB at a time, then the batch's neighbour rows, so a
// cell waits on two memory latencies per batch.  Padding records name the
// cell itself with zero weight (phi_c - phi_c = 0), leaving the sums as
// they are.  c must be cell lane of the ELL block c / KTPB.
// GB0: records per batch (0: 3 for rows of at most 5 values, else 2; the
// measured optimum of the gradient kernel; the fused indicator kernel
// prefers 6).
template <class T, int D, int NQ, int GB0 = 0>
__device__ __forceinline__ void grad_sums(const KArgs<T>& a, const T* __restrict__ phi, int64_t c, T (*acc)[D],
                                          const T* lds = nullptr, int64_t c0 = 0, int n = 0) {
  constexpr int GB = GB0 > 0 ? GB0 : (NQ <= 5 ? 3 : 2);
  const int64_t b = c / KTPB;
  const int lane = (int)(c - b * KTPB);
  const int r0 = a.ell_ptr[b], m = (a.ell_ptr[b + 1] - r0) / KTPB;
  T q[NQ];
  load_row<T, NQ>(q, lds, phi, c0, n, c);
#pragma unroll
  for (int k = 0; k < NQ; ++k)
#pragma unroll
    for (int x = 0; x < D; ++x) acc[k][x] = T(0);
  for (int j = 0; j < m; j += GB) {
    int64_t o[GB];
    T Sw[GB][D];
#pragma unroll
    for (int jj = 0; jj < GB; ++jj) {
      const bool ok = j + jj < m;
      const int64_t r = (int64_t)r0 + (int64_t)(ok ? j + jj : j) * KTPB + lane;
      GlbPtr<T> rec = as_glb(a.ell_sw + 4 * r);
      T v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) v[x] = rec[x];
      o[jj] = ok ? rec_cell(v[3]) : c;
#pragma unroll
      for (int x = 0; x < D; ++x) Sw[jj][x] = ok ? v[x] : T(0);
    }
    T qo[GB][NQ];
#pragma unroll
    for (int jj = 0; jj < GB; ++jj) load_row<T, NQ>(qo[jj], lds, phi, c0, n, o[jj]);
#pragma unroll
    for (int jj = 0; jj < GB; ++jj)
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const T dq = qo[jj][k] - q[k];
#pragma unroll
        for (int x = 0; x < D; ++x) acc[k][x] += dq * Sw[jj][x];
      }
  }
}

// Second derivatives from the gradient rows phi = G1 [nc][NV][D]: the
// Gauss-linear sums are accumulated directly in symmetrised form,
// acc2[v][(i,j)] = sum_f (dG_{v,i} Sw_j + dG_{v,j} Sw_i) (i < j) and
// sum_f dG_{v,i} Sw_i (i = j), 6 (3-D) accumulators per variable instead of 9.
template <class T, int D, int NV>
__device__ __forceinline__ void grad2_sums(const KArgs<T>& a, const T* __restrict__ phi, int64_t c,
                                           T (*acc2)[D * (D + 1) / 2], const T* lds, int64_t c0, int n) {
  constexpr int NQ = NV * D;
  constexpr int NS2 = D * (D + 1) / 2;
  const int64_t b = c / KTPB;
  const int lane = (int)(c - b * KTPB);
  const int r0 = a.ell_ptr[b], m = (a.ell_ptr[b + 1] - r0) / KTPB;
  T q[NQ];
  load_row<T, NQ>(q, lds, phi, c0, n, c);
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int k = 0; k < NS2; ++k) acc2[v][k] = T(0);
  // one record, then its row (batches of 2 or 3 need more registers and
  // measured slower); the next record is requested before the row, so the
  // two loads of an iteration wait on one memory latency
  T nx[4];
  {
    GlbPtr<T> rec = as_glb(a.ell_sw + 4 * ((int64_t)r0 + lane));
#pragma unroll
    for (int x = 0; x < 4; ++x) nx[x] = m > 0 ? rec[x] : T(0);
  }
  for (int j = 0; j < m; ++j) {
    T v[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) v[x] = nx[x];
    if (j + 1 < m) {
      GlbPtr<T> rec = as_glb(a.ell_sw + 4 * ((int64_t)r0 + (int64_t)(j + 1) * KTPB + lane));
#pragma unroll
      for (int x = 0; x < 4; ++x) nx[x] = rec[x];
    }
    const int64_t o = rec_cell(v[3]);
    T qo[NQ];
    load_row<T, NQ>(qo, lds, phi, c0, n, o);
#pragma unroll
    for (int v2 = 0; v2 < NV; ++v2) {
      T dq[D];
#pragma unroll
      for (int i = 0; i < D; ++i) dq[i] = qo[v2 * D + i] - q[v2 * D + i];
#pragma unroll
      for (int i = 0; i < D; ++i) acc2[v2][i] += dq[i] * v[i];
      if constexpr (D == 3) {
        acc2[v2][3] += dq[0] * v[1] + dq[1] * v[0];
        acc2[v2][4] += dq[0] * v[2] + dq[2] * v[0];
        acc2[v2][5] += dq[1] * v[2] + dq[2] * v[1];
      } else {
        acc2[v2][2] += dq[0] * v[1] + dq[1] * v[0];
      }
    }
  }
}

// Rows of W values for the block's cells c0 .. c0+n-1, written by their
// threads into LDS (row-major), then copied to HBM with consecutive lanes
// on consecutive addresses.  Every thread of the block must call it.
template <class T, int W>
__device__ __forceinline__ void store_rows_coalesced(T* __restrict__ out, int64_t c0, int n, const T* row,
                                                     T* buf) {
  __syncthreads();  // buf may still be read by the caller's earlier phase
  if ((int)threadIdx.x < n) {
#pragma unroll
    for (int k = 0; k < W; ++k) buf[threadIdx.x * W + k] = row[k];
  }
  __syncthreads();
  T* dst = out + c0 * W;
  for (int i = threadIdx.x; i < n * W; i += blockDim.x) dst[i] = buf[i];
}

template <class T, int D, int NQ, bool SYM>
struct GradOut {
  static constexpr int NV = SYM ? NQ / D : NQ;
  static constexpr int W = SYM ? NV * D * (D + 1) / 2 : NQ * D;
  // transposed (coalesced) output when its LDS buffer is at most 32 KiB
  static constexpr bool LDS = (size_t)KTPB * W * sizeof(T) <= 32768;
  static constexpr int LDSN = KTPB * (LDS ? (W > NQ ? W : NQ) : NQ);
};

template <class T, int D, int NQ, bool SYM>
__device__ __forceinline__ void grad_block(const KArgs<T>& a, const T* __restrict__ phi, T* __restrict__ out) {
  using GO = GradOut<T, D, NQ, SYM>;
  __shared__ T lds[GO::LDSN];
  const int b = xcd_remap(blockIdx.x, a.cell_per_xcd, a.n_cell_blocks);
  if (b < 0) return;
  const int64_t c0 = (int64_t)b * KTPB;
  const int n = (int)(a.nc - c0 < KTPB ? a.nc - c0 : KTPB);
  stage_rows(lds, phi, c0, n, NQ);
  __syncthreads();
  const int64_t c = c0 + threadIdx.x;
  T res[GO::W];
  if (c < a.nc) {
    const T rv = a.rV[c];
    if constexpr (!SYM) {
      T acc[NQ][D];
      grad_sums<T, D, NQ>(a, phi, c, acc, lds, c0, n);
#pragma unroll
      for (int k = 0; k < NQ; ++k)
#pragma unroll
        for (int x = 0; x < D; ++x) res[k * D + x] = acc[k][x] * rv;
    } else {
      constexpr int NV = NQ / D;
      constexpr int NS2 = D * (D + 1) / 2;
      T acc2[NV][NS2];
      grad2_sums<T, D, NV>(a, phi, c, acc2, lds, c0, n);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < D; ++i) res[v * NS2 + i] = acc2[v][i] * rv;
#pragma unroll
        for (int k = D; k < NS2; ++k) res[v * NS2 + k] = T(0.5) * acc2[v][k] * rv;
      }
    }
  }
  if constexpr (GO::LDS) {
    store_rows_coalesced<T, GO::W>(out, c0, n, res, lds);
  } else if (c < a.nc) {
#pragma unroll
    for (int k = 0; k < GO::W; ++k) out[c * GO::W + k] = res[k];
  }
}

template <class T, int D, int NQ, bool SYM>
__global__ __launch_bounds__(KTPB) void k_grad(KArgs<T> a, const T* __restrict__ phi, T* __restrict__ out) {
  grad_block<T, D, NQ, SYM>(a, phi, out);
}

// The same with the register budget of 5 waves per SIMD (FP32 second
// derivatives: 98 registers would otherwise allow only 4).
template <class T, int D, int NQ, bool SYM>
__global__ __launch_bounds__(KTPB) __attribute__((amdgpu_waves_per_eu(5))) void k_grad_w5(KArgs<T> a,
                                                                                     const T* __restrict__ phi,
                                                                                     T* __restrict__ out) {
  grad_block<T, D, NQ, SYM>(a, phi, out);
}

// Second differentials of a stage in the form the faces use them: for every
// face record of cell c, h_v = d . H_v . d (H_v the symmetrised Gauss-linear
// derivative of the gradient rows phi = G1, d the face's centre-to-centre
// vector; the quadratic form does not see the record's sign), written to
// Hf[r] of the face record r (ELL order: consecutive lanes, consecutive
// records), so that the flux kernel reads 5 values per side instead of
// gathering both cells' second-derivative rows.  The arithmetic (sums,
// symmetrised values rounded to T, contraction) is that of the row kernel
// followed by the contraction the flux kernel did before.
template <class T, int D, int NV>
__device__ __forceinline__ void hface_block(const KArgs<T>& a, const T* __restrict__ phi, T* __restrict__ out) {
  constexpr int NQ = NV * D;
  constexpr int NS2 = D * (D + 1) / 2;
  __shared__ T lds[KTPB * NQ];
  const int b = xcd_remap(blockIdx.x, a.cell_per_xcd, a.n_cell_blocks);
  if (b < 0) return;
  const int64_t c0 = (int64_t)b * KTPB;
  const int n = (int)(a.nc - c0 < KTPB ? a.nc - c0 : KTPB);
  stage_rows(lds, phi, c0, n, NQ);
  __syncthreads();
  const int64_t c = c0 + threadIdx.x;
  if (c >= a.nc) return;
  T acc2[NV][NS2];
  grad2_sums<T, D, NV>(a, phi, c, acc2, lds, c0, n);
  const T rv = a.rV[c];
  T H[NV * NS2];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int i = 0; i < D; ++i) H[v * NS2 + i] = acc2[v][i] * rv;
#pragma unroll
    for (int k = D; k < NS2; ++k) H[v * NS2 + k] = T(0.5) * acc2[v][k] * rv;
  }
  const int r0 = a.ell_ptr[b];
  const int nfc = a.slot_ptr[c + 1] - a.slot_ptr[c];
  for (int j = 0; j < nfc; ++j) {
    const int64_t r = (int64_t)r0 + (int64_t)j * KTPB + threadIdx.x;
    GlbPtr<T> rd = as_glb(a.ell_d + 3 * r);
    T d[3];
#pragma unroll
    for (int x = 0; x < D; ++x) d[x] = rd[x];
    T h[NV];
    contract2<T, NV, D>(static_cast<const T*>(H), d, h);
    T* o = out + r * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) o[v] = h[v];
  }
}

template <class T, int D, int NV>
__global__ __launch_bounds__(KTPB) void k_hface(KArgs<T> a, const T* __restrict__ phi, T* __restrict__ out) {
  hface_block<T, D, NV>(a, phi, out);
}

template <class T, int D, int NV>
__global__ __launch_bounds__(KTPB) __attribute__((amdgpu_waves_per_eu(5))) void k_hface_w5(KArgs<T> a,
                                                                                     const T* __restrict__ phi,
                                                                                     T* __restrict__ out) {
  hface_block<T, D, NV>(a, phi, out);
}

// Classical sensor: beta = |s - Delta| / (|s| + |Delta| + eps) on every face
// in the frame where the cell is upwind; s = phi_0^(1) - Delta.
template <class T, int D, int NV>
__global__ __launch_bounds__(KTPB) void k_theta(KArgs<T> a, float* __restrict__ theta) {
  const int b = xcd_remap(blockIdx.x, a.cell_per_xcd, a.n_cell_blocks);
  if (b < 0) return;
  const int64_t c = (int64_t)b * KTPB + threadIdx.x;
  if (c >= a.nc) return;
  const int r0 = a.ell_ptr[b];
  const int nfc = a.slot_ptr[c + 1] - a.slot_ptr[c];  // records beyond the cell's faces are padding
  T beta = T(0);
  for (int j = 0; j < nfc; ++j) {
    const int64_t r = (int64_t)r0 + (int64_t)j * KTPB + threadIdx.x;
    GlbPtr<T> rd = as_glb(a.ell_d + 3 * r);
    const int64_t o = rec_cell(a.ell_sw[4 * r + 3]);
#pragma unroll
    for (int q = 0; q < (NV == 1 ? 1 : 2); ++q) {
      const int v = q == 0 ? 0 : NV - 1;
      T dot = T(0);
#pragma unroll
      for (int x = 0; x < D; ++x) dot += rd[x] * a.G1[(c * NV + v) * D + x];
      const T phi0 = a.U[c * NV + v], phi1 = a.U[o * NV + v];
      const T delta = phi1 - phi0;
      const T sdiff = T(2) * dot - delta;
      const T eps = T(1e-8) * (fabs(phi0) + fabs(phi1)) + T(1e-30);
      const T bf = fdiv(fabs(sdiff - delta), fabs(sdiff) + fabs(delta) + eps);
      beta = fmax(beta, bf);
    }
  }
  T th = (T(0.9) - beta) / T(0.3);
  th = th < T(0) ? T(0) : (th > T(1) ? T(1) : th);
  theta[c] = (float)th;
}

}  // namespace dolinc
