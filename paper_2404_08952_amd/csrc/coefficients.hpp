// Coefficients of the DOLINC representation (Sec. 2.3-2.4), FP64.
//
// Reconstruction weights c_rj of eq:coeff in closed form in the growth rate
// g (USR3, CSR4 as printed; USR5 and CSR6 from the same formula), G_n always
// summed as 1 + g + ... + g^(n-1); far cells folded in with the inversion
// coefficients eq:lCoeffDLC1, eq:rCoeffDLC1, eq:lCoeffDLC2 (and
// eq:rCoeffDLC2 for CSR6) into
//   U_side = phi_other + w (phi_self - phi_other)
//            + k0 phi_self^(1) + k1 phi_other^(1) + k2 phi_self^(2)
//            (+ k3 phi_other^(2), CSR6).
// The flux kernels of both precisions evaluate them per face from
// g = omega / (1 - omega) (omega and d are all a face entry stores), which
// trades 8 stored values per entry for a few dozen FP64 operations: each
// side's divisions are gathered into one reciprocal of the common
// denominator, taken as the hardware reciprocal refined by two Newton
// steps.  (In FP32 the same forms cost 32 fewer instructions per entry but
// lose digits on graded faces, 1e-5 relative for USR5 at omega = 0.01, and
// overflow below omega ~ 1e-4.)
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/dolinc.h"

namespace dolinc {

// 1 / x to FP64 accuracy: the hardware reciprocal (an approximation) refined
// by two Newton steps, each of which squares the relative error.
__device__ __forceinline__ double coef_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// DOLINC representation of one side (self = upwind cell of this frame,
// growth rate g from self to other; ig = 1/g): w, k0, k1, k2 (, k3) as in
// the file comment.
__device__ __forceinline__ void side_coefficients(int scheme, double g, double ig, double* w, double* k0, double* k1,
                                                  double* k2, double* k3) {
  const double one = 1.0, two = 2.0, three = 3.0;
  *k0 = 0.0; *k1 = 0.0; *k2 = 0.0; *k3 = 0.0;
  const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g;
  const double G2 = one + g, G3 = G2 + g2, G4 = G3 + g3, G5 = G4 + g4;
  switch (scheme) {
    case DOLINC_FOU:
      *w = one;
      return;
    case DOLINC_CD2:
      *w = g * coef_rcp(G2);
      return;
    case DOLINC_USR3: {
      const double r = coef_rcp(G2 * G3);
      const double c10 = -g3 * r, c11 = g * (one + two * g + two * g2) * r;
      // eq:lCoeffDLC1: a0 = 1 - 1/g, A = -phi_self^(1) / g
      *w = c10 * (one - ig) + c11;
      *k0 = -c10 * ig;
      return;
    }
    case DOLINC_CSR4: {
      const double r = coef_rcp(G3 * G4);
      const double c10 = -g5 * r;
      const double c11 = g2 * (one + two * g + two * g2 + two * g3) * r;
      const double c13 = -r;
      // eq:lCoeffDLC1 for the left far cell, eq:rCoeffDLC1 (a0 = g,
      // A = g phi_other^(1)) for the right one
      *w = c10 * (one - ig) + c11 + c13 * g;
      *k0 = -c10 * ig;
      *k1 = c13 * g;
      return;
    }
    case DOLINC_USR5: {
      const double q = one + g2;
      const double r = coef_rcp(G2 * q * G3 * G5);
      const double c0 = g4 * g5 * G2 * r;
      const double c1 = -g5 * (g5 + three * g4 + three * g3 + three * g2 + two * g + one) * r;
      const double c2 = g2 * (three * g5 * g2 + 6.0 * g3 * g3 + 9.0 * g5 + 10.0 * g4 + 9.0 * g3 + 6.0 * g2 +
                         three * g + one) * r;
      const double c4 = -G3 * r;
      const double ig2 = ig * ig, ig3 = ig2 * ig;
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
      const double gm = g2 - g + one;
      const double den = G2 * (one + g2) * G5;
      const double r = coef_rcp(den * gm * G3);
      *w = g * (g5 * g + 5.0 * g5 + 4.0 * g4 + two * g3 + two * g2 - g - three) * (gm * G3) * r;
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
__device__ __forceinline__ void face_coefficients(int scheme, double om, double* c) {
  const double one = 1.0;
  const double g = om * coef_rcp(one - om), ig = (one - om) * coef_rcp(om);
  double w, k0, k1, k2, k3;
  side_coefficients(scheme, g, ig, &w, &k0, &k1, &k2, &k3);
  int k = 0;
  c[k++] = w;
  if (scheme == DOLINC_USR3) c[k++] = 2.0 * k0;
  if (scheme == DOLINC_CSR4 || scheme == DOLINC_USR5 || scheme == DOLINC_CSR6) {
    c[k++] = 2.0 * k0;
    c[k++] = 2.0 * k1;
  }
  if (scheme == DOLINC_USR5 || scheme == DOLINC_CSR6) c[k++] = 4.0 * k2;
  if (scheme == DOLINC_CSR6) c[k++] = 4.0 * k3;
  if (scheme == DOLINC_CSR4 || scheme == DOLINC_CSR6) return;
  side_coefficients(scheme, ig, g, &w, &k0, &k1, &k2, &k3);
  c[k++] = w;
  if (scheme == DOLINC_USR3 || scheme == DOLINC_USR5) c[k++] = -2.0 * k0;
  if (scheme == DOLINC_USR5) {
    c[k++] = -2.0 * k1;
    c[k++] = 4.0 * k2;
  }
}

}  // namespace dolinc
