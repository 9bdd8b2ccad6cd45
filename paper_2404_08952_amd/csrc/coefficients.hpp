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
// The flux kernels evaluate them per face from g (d and g are all a face
// entry stores), which trades 8 stored values per entry for about a hundred
// FP64 operations.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/dolinc.h"

namespace dolinc {

// DOLINC representation of one side (self = upwind cell of this frame,
// growth rate g from self to other).  w, k0, k1, k2 as in the file comment.
__host__ __device__ inline void side_coefficients(int scheme, double g, double* w, double* k0, double* k1,
                                                  double* k2, double* k3 = nullptr) {
  *k0 = 0.0; *k1 = 0.0; *k2 = 0.0;
  const double ig = 1.0 / g;
  const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g;
  const double G2 = 1.0 + g, G3 = 1.0 + g + g2, G4 = G3 + g3, G5 = G4 + g4;
  switch (scheme) {
    case DOLINC_FOU:
      *w = 1.0;
      return;
    case DOLINC_CD2:
      *w = g / G2;  // linear interpolation with the distance weight
      return;
    case DOLINC_USR3: {
      const double den = G2 * G3;
      const double c10 = -g3 / den, c11 = g * (1.0 + 2.0 * g + 2.0 * g2) / den;
      // eq:lCoeffDLC1: a0 = 1 - 1/g, A = -phi_self^(1) / g
      *w = c10 * (1.0 - ig) + c11;
      *k0 = -c10 * ig;
      return;
    }
    case DOLINC_CSR4: {
      const double den = G3 * G4;
      const double c10 = -g5 / den;
      const double c11 = g2 * (1.0 + 2.0 * g + 2.0 * g2 + 2.0 * g3) / den;
      const double c13 = -1.0 / den;
      // eq:lCoeffDLC1 for the left far cell, eq:rCoeffDLC1 (a0 = g,
      // A = g phi_other^(1)) for the right one
      *w = c10 * (1.0 - ig) + c11 + c13 * g;
      *k0 = -c10 * ig;
      *k1 = c13 * g;
      return;
    }
    case DOLINC_USR5: {
      const double q = 1.0 + g2;
      const double den = G2 * q * G3 * G5;
      const double c0 = g4 * g5 / (q * G3 * G5);
      const double c1 = -g5 * (g5 + 3.0 * g4 + 3.0 * g3 + 3.0 * g2 + 2.0 * g + 1.0) / den;
      const double c2 = g2 * (3.0 * g5 * g2 + 6.0 * g3 * g3 + 9.0 * g5 + 10.0 * g4 + 9.0 * g3 + 6.0 * g2 +
                              3.0 * g + 1.0) / den;
      const double c4 = -1.0 / (G2 * q * G5);
      const double ig2 = ig * ig, ig3 = ig2 * ig;
      // eq:lCoeffDLC2 (phi_-2), eq:lCoeffDLC1 (phi_-1), eq:rCoeffDLC1 (phi_2)
      *w = c0 * (1.0 - ig + ig2) + c1 * (1.0 - ig) + c2 + c4 * g;
      *k0 = -c0 * ig * (1.0 - ig2) - c1 * ig;
      *k1 = -c0 * ig3 + c4 * g;
      *k2 = c0 * ig3;
      return;
    }
    case DOLINC_CSR6: {
      // eq:coeff on the six cells -2..3 with the far cells from eq:lCoeffDLC2
      // (phi_-2), eq:lCoeffDLC1 (phi_-1), eq:rCoeffDLC1 (phi_2) and
      // eq:rCoeffDLC2 (phi_3), collected on phi_0, phi_1 and the differentials
      // (closed forms in g; 1/2, 3/20, -3/20, 1/60, 1/60 at g = 1)
      const double gm = g2 - g + 1.0;
      const double den = G2 * (1.0 + g2) * G5;
      *w = g * (g5 * g + 5.0 * g5 + 4.0 * g4 + 2.0 * g3 + 2.0 * g2 - g - 3.0) / den;
      *k0 = g2 * (2.0 * g5 * g + g3 - g + 1.0) / (den * gm);
      *k1 = -g * (g5 * g - g5 + g3 + 2.0) / (den * gm);
      *k2 = g4 * g5 / (den * gm * G3);
      if (k3) *k3 = g2 / (den * gm * G3);
      return;
    }
    default:
      *w = 1.0;
  }
}

// Both sides of a face in the order the flux kernel combines them: left
// state (frame P -> N, growth g): w, 2 k0, 2 k1, 4 k2 (as many as the scheme
// uses; the factors 2 and 4 of the DOLINC differentials folded in, which
// multiply d.G1 and d.G2.d), then the right state (mirrored frame N -> P,
// growth 1/g, d -> -d): w, -2 k0, -2 k1, 4 k2.  CSR4 and CSR6 have one
// state per face (symmetric template): w, 2 k0, 2 k1 (, 4 k2, 4 k3).
__host__ __device__ inline void face_coefficients(int scheme, double g, double* c) {
  double w, k0, k1, k2, k3 = 0.0;
  side_coefficients(scheme, g, &w, &k0, &k1, &k2, &k3);
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
  side_coefficients(scheme, 1.0 / g, &w, &k0, &k1, &k2);
  c[k++] = w;
  if (scheme == DOLINC_USR3 || scheme == DOLINC_USR5) c[k++] = -2.0 * k0;
  if (scheme == DOLINC_USR5) {
    c[k++] = -2.0 * k1;
    c[k++] = 4.0 * k2;
  }
}

}  // namespace dolinc
