// Coefficients of the DOLINC representation (Sec. 2.3-2.4).
//
// Reconstruction weights c_rj of eq:coeff in closed form in the growth rate
// g (USR3, CSR4 as printed; USR5 and CSR6 from the same formula), G_n always
// summed as 1 + g + ... + g^(n-1); far cells folded in with the inversion
// coefficients eq:lCoeffDLC1, eq:rCoeffDLC1, eq:lCoeffDLC2 (and
// eq:rCoeffDLC2 for CSR6) into
//   U_side = phi_other + w (phi_self - phi_other)
//            + k0 phi_self^(1) + k1 phi_other^(1) + k2 phi_self^(2)
//            (+ k3 phi_other^(2), CSR6).
// The flux kernels evaluate them per face from g = omega / (1 - omega)
// (omega and d are all a face entry stores), which trades 8 stored values
// per entry for a few dozen operations in the working precision (in FP32
// the relative error stays below 1e-6 for omega in [0.15, 0.85], where the
// FP32 kernels use it; an FP64 evaluation there cost 24 % of the FP32 flux
// kernel's vector instructions).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/dolinc.h"

namespace dolinc {

// Reciprocal in the working precision: the hardware reciprocal in FP32
// (about 1 ulp), the correctly rounded quotient in FP64.
__device__ __forceinline__ float coef_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double coef_rcp(double x) { return 1.0 / x; }

// DOLINC representation of one side (self = upwind cell of this frame,
// growth rate g from self to other; ig = 1/g): w, k0, k1, k2 (, k3) as in
// the file comment, in the working precision R, each side's divisions
// gathered into one reciprocal of the common denominator.
template <class R>
__device__ __forceinline__ void side_coefficients_r(int scheme, R g, R ig, R* w, R* k0, R* k1, R* k2, R* k3) {
  const R one = R(1), two = R(2), three = R(3);
  *k0 = R(0); *k1 = R(0); *k2 = R(0); *k3 = R(0);
  const R g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g;
  const R G2 = one + g, G3 = G2 + g2, G4 = G3 + g3, G5 = G4 + g4;
  switch (scheme) {
    case DOLINC_FOU:
      *w = one;
      return;
    case DOLINC_CD2:
      *w = g * coef_rcp(G2);
      return;
    case DOLINC_USR3: {
      const R r = coef_rcp(G2 * G3);
      const R c10 = -g3 * r, c11 = g * (one + two * g + two * g2) * r;
      // eq:lCoeffDLC1: a0 = 1 - 1/g, A = -phi_self^(1) / g
      *w = c10 * (one - ig) + c11;
      *k0 = -c10 * ig;
      return;
    }
    case DOLINC_CSR4: {
      const R r = coef_rcp(G3 * G4);
      const R c10 = -g5 * r;
      const R c11 = g2 * (one + two * g + two * g2 + two * g3) * r;
      const R c13 = -r;
      // eq:lCoeffDLC1 for the left far cell, eq:rCoeffDLC1 (a0 = g,
      // A = g phi_other^(1)) for the right one
      *w = c10 * (one - ig) + c11 + c13 * g;
      *k0 = -c10 * ig;
      *k1 = c13 * g;
      return;
    }
    case DOLINC_USR5: {
      const R q = one + g2;
      const R r = coef_rcp(G2 * q * G3 * G5);
      const R c0 = g4 * g5 * G2 * r;
      const R c1 = -g5 * (g5 + three * g4 + three * g3 + three * g2 + two * g + one) * r;
      const R c2 = g2 * (three * g5 * g2 + R(6) * g3 * g3 + R(9) * g5 + R(10) * g4 + R(9) * g3 + R(6) * g2 +
                         three * g + one) * r;
      const R c4 = -G3 * r;
      const R ig2 = ig * ig, ig3 = ig2 * ig;
      // eq:lCoeffDLC2 (phi_-2), eq:lCoeffDLC1 (phi_-1), eq:rCoeffDLC1 (phi_2)
      *w = c0 * (one - ig + ig2) + c1 * (one - ig) + c2 + c4 * g;
      *k0 = -c0 * ig * (one - ig2) - c1 * ig;
      *k1 = -c0 * ig3 + c4 * g;
      *k2 = c0 * ig3;
      return;
    }
    case DOLINC_CSR6: {
      // eq:coeff on the six cells -2..3 with the far cells from eq:lCoeffDLC2
      // (phi_-2), eq:lCoeffDLC1 (phi_-1), eq:rCoeffDLC1 (phi_2) and
      // eq:rCoeffDLC2 (phi_3), collected on phi_0, phi_1 and the differentials
      // (1/2, 3/20, -3/20, 1/60, 1/60 at g = 1)
      const R gm = g2 - g + one;
      const R den = G2 * (one + g2) * G5;
      const R r = coef_rcp(den * gm * G3);
      *w = g * (g5 * g + R(5) * g5 + R(4) * g4 + two * g3 + two * g2 - g - three) * (gm * G3) * r;
      *k0 = g2 * (two * g5 * g + g3 - g + one) * G3 * r;
      *k1 = -g * (g5 * g - g5 + g3 + two) * G3 * r;
      *k2 = g4 * g5 * r;
      *k3 = g2 * r;
      return;
    }
    default:
      *w = one;
  }
}

// Both sides of a face from its weight omega, in the order the flux kernel
// combines them: left state (frame P -> N, growth g): w, 2 k0, 2 k1, 4 k2
// (as many as the scheme uses; the factors 2 and 4 of the DOLINC
// differentials folded in, which multiply d.G1 and d.G2.d), then the right
// state (mirrored frame N -> P, growth 1/g, d -> -d): w, -2 k0, -2 k1, 4 k2.
// CSR4 and CSR6 have one state per face (symmetric template): w, 2 k0,
// 2 k1 (, 4 k2, 4 k3).
template <class R>
__device__ __forceinline__ void face_coefficients_r(int scheme, R om, R* c) {
  const R one = R(1);
  const R g = om * coef_rcp(one - om), ig = (one - om) * coef_rcp(om);
  R w, k0, k1, k2, k3;
  side_coefficients_r<R>(scheme, g, ig, &w, &k0, &k1, &k2, &k3);
  int k = 0;
  c[k++] = w;
  if (scheme == DOLINC_USR3) c[k++] = R(2) * k0;
  if (scheme == DOLINC_CSR4 || scheme == DOLINC_USR5 || scheme == DOLINC_CSR6) {
    c[k++] = R(2) * k0;
    c[k++] = R(2) * k1;
  }
  if (scheme == DOLINC_USR5 || scheme == DOLINC_CSR6) c[k++] = R(4) * k2;
  if (scheme == DOLINC_CSR6) c[k++] = R(4) * k3;
  if (scheme == DOLINC_CSR4 || scheme == DOLINC_CSR6) return;
  side_coefficients_r<R>(scheme, ig, g, &w, &k0, &k1, &k2, &k3);
  c[k++] = w;
  if (scheme == DOLINC_USR3 || scheme == DOLINC_USR5) c[k++] = R(-2) * k0;
  if (scheme == DOLINC_USR5) {
    c[k++] = R(-2) * k1;
    c[k++] = R(4) * k2;
  }
}

}  // namespace dolinc
