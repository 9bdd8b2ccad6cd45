// FP64 precompute on the device: geometry, face scalars and the per-face
// coefficients of the DOLINC representation.
//
// Geometry (textbook finite volumes; the paper leaves it to the host code):
//   face  : 2-D edge a->b: S = (t_y, -t_x); 3-D: triangle fan about the vertex
//           average c, S = sum of fan triangle area vectors, centre weighted
//           by triangle area.
//   cell  : simplices (x_e, c, p_k, p_k+1), x_e = mean of the face centres;
//           gives exact volume and centroid of the fan-bounded polyhedron.
// Face scalars (Sec. 2.2): d = x_N - x_P, omega = |x_N - x_f| /
// (|x_P - x_f| + |x_N - x_f|), growth rate g = omega / (1 - omega).
// Per face entry: S and omega, and d; the flux kernels evaluate the
// coefficients of the DOLINC representation from omega in the working
// precision (coefficients.hpp).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace dolinc {
namespace {

constexpr int TPB = 256;

__device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ void k_face_geom(int64_t nf, int dim, const int64_t* __restrict__ fptr,
                            const int32_t* __restrict__ fnodes, const double* __restrict__ nodes,
                            double* __restrict__ S, double* __restrict__ xf, double* __restrict__ fanc) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t a = fptr[f], b = fptr[f + 1];
  if (dim == 2) {
    const double* p0 = nodes + 2 * (int64_t)fnodes[a];
    const double* p1 = nodes + 2 * (int64_t)fnodes[a + 1];
    double tx = p1[0] - p0[0], ty = p1[1] - p0[1];
    S[3 * f + 0] = ty;
    S[3 * f + 1] = -tx;
    S[3 * f + 2] = 0.0;
    xf[3 * f + 0] = fanc[3 * f + 0] = 0.5 * (p0[0] + p1[0]);
    xf[3 * f + 1] = fanc[3 * f + 1] = 0.5 * (p0[1] + p1[1]);
    xf[3 * f + 2] = fanc[3 * f + 2] = 0.0;
    return;
  }
  const int m = (int)(b - a);
  double c[3] = {0, 0, 0};
  for (int k = 0; k < m; ++k) {
    const double* p = nodes + 3 * (int64_t)fnodes[a + k];
    c[0] += p[0]; c[1] += p[1]; c[2] += p[2];
  }
  c[0] /= m; c[1] /= m; c[2] /= m;
  double s[3] = {0, 0, 0}, cen[3] = {0, 0, 0}, area = 0.0;
  for (int k = 0; k < m; ++k) {
    const double* q1 = nodes + 3 * (int64_t)fnodes[a + k];
    const double* q2 = nodes + 3 * (int64_t)fnodes[a + (k + 1) % m];
    double u[3] = {q1[0] - c[0], q1[1] - c[1], q1[2] - c[2]};
    double v[3] = {q2[0] - c[0], q2[1] - c[1], q2[2] - c[2]};
    double t[3];
    cross3(u, v, t);
    t[0] *= 0.5; t[1] *= 0.5; t[2] *= 0.5;
    s[0] += t[0]; s[1] += t[1]; s[2] += t[2];
    double at = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    area += at;
    for (int x = 0; x < 3; ++x) cen[x] += at * (c[x] + q1[x] + q2[x]) / 3.0;
  }
  for (int x = 0; x < 3; ++x) {
    S[3 * f + x] = s[x];
    xf[3 * f + x] = cen[x] / area;
    fanc[3 * f + x] = c[x];
  }
}

// One thread per (internal) cell; faces reached through the partition slots.
__global__ void k_cell_geom(int64_t nc, int dim, int B, const int32_t* __restrict__ part_ptr,
                            const int32_t* __restrict__ ent_face, const int32_t* __restrict__ slot_ptr,
                            const uint16_t* __restrict__ slots, const int64_t* __restrict__ fptr,
                            const int32_t* __restrict__ fnodes, const double* __restrict__ nodes,
                            const double* __restrict__ shift, const double* __restrict__ S,
                            const double* __restrict__ xf, const double* __restrict__ fanc,
                            double* __restrict__ V, double* __restrict__ xc, int* __restrict__ flag) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int e0 = part_ptr[c / B];
  const int s0 = slot_ptr[c], s1 = slot_ptr[c + 1];
  double xe[3] = {0, 0, 0}, clo[3] = {0, 0, 0}, sabs = 0.0;
  for (int s = s0; s < s1; ++s) {
    const uint16_t sl = slots[s];
    const int f = ent_face[e0 + (sl & 0x7fff)];
    const double sg = (sl >> 15) ? -1.0 : 1.0;
    for (int x = 0; x < dim; ++x) {
      xe[x] += xf[3 * f + x] - ((sl >> 15) ? shift[(int64_t)dim * f + x] : 0.0);
      clo[x] += sg * S[3 * f + x];
    }
    sabs += sqrt(S[3 * f] * S[3 * f] + S[3 * f + 1] * S[3 * f + 1] + S[3 * f + 2] * S[3 * f + 2]);
  }
  const double inv = 1.0 / (double)(s1 - s0);
  for (int x = 0; x < 3; ++x) xe[x] *= inv;
  double vol = 0.0, mom[3] = {0, 0, 0};
  for (int s = s0; s < s1; ++s) {
    const uint16_t sl = slots[s];
    const int f = ent_face[e0 + (sl & 0x7fff)];
    const bool nb = (sl >> 15) != 0;
    double t[3] = {0, 0, 0};
    if (nb)
      for (int x = 0; x < dim; ++x) t[x] = -shift[(int64_t)dim * f + x];
    const int64_t a = fptr[f];
    const int m = (int)(fptr[f + 1] - a);
    if (dim == 2) {
      const double* pa = nodes + 2 * (int64_t)fnodes[a + (nb ? 1 : 0)];
      const double* pb = nodes + 2 * (int64_t)fnodes[a + (nb ? 0 : 1)];
      double ax = pa[0] + t[0] - xe[0], ay = pa[1] + t[1] - xe[1];
      double bx = pb[0] + t[0] - xe[0], by = pb[1] + t[1] - xe[1];
      double v = 0.5 * (ax * by - ay * bx);
      vol += v;
      mom[0] += v * (xe[0] + (pa[0] + t[0]) + (pb[0] + t[0])) / 3.0;
      mom[1] += v * (xe[1] + (pa[1] + t[1]) + (pb[1] + t[1])) / 3.0;
      continue;
    }
    double fc[3] = {fanc[3 * f] + t[0], fanc[3 * f + 1] + t[1], fanc[3 * f + 2] + t[2]};
    double w[3] = {fc[0] - xe[0], fc[1] - xe[1], fc[2] - xe[2]};
    for (int k = 0; k < m; ++k) {
      int k1 = nb ? (k + 1) % m : k;
      int k2 = nb ? k : (k + 1) % m;
      const double* q1 = nodes + 3 * (int64_t)fnodes[a + k1];
      const double* q2 = nodes + 3 * (int64_t)fnodes[a + k2];
      double u[3] = {q1[0] + t[0] - xe[0], q1[1] + t[1] - xe[1], q1[2] + t[2] - xe[2]};
      double v[3] = {q2[0] + t[0] - xe[0], q2[1] + t[1] - xe[1], q2[2] + t[2] - xe[2]};
      double cr[3];
      cross3(u, v, cr);
      double tv = (w[0] * cr[0] + w[1] * cr[1] + w[2] * cr[2]) / 6.0;
      vol += tv;
      for (int x = 0; x < 3; ++x)
        mom[x] += tv * (xe[x] + fc[x] + (q1[x] + t[x]) + (q2[x] + t[x])) / 4.0;
    }
  }
  V[c] = vol;
  for (int x = 0; x < 3; ++x) xc[3 * c + x] = (x < dim) ? mom[x] / vol : 0.0;
  const double cl = sqrt(clo[0] * clo[0] + clo[1] * clo[1] + clo[2] * clo[2]);
  if (!(vol > 0.0)) atomicOr(flag, 1);
  if (!(cl <= 1e-9 * sabs)) atomicOr(flag, 2);
}

__global__ void k_face_scalars(int64_t nf, int dim, const int32_t* __restrict__ own,
                               const int32_t* __restrict__ nei, const double* __restrict__ xc,
                               const double* __restrict__ shift, const double* __restrict__ xf,
                               double* __restrict__ dvec, double* __restrict__ omega, double* __restrict__ g,
                               int* __restrict__ flag) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int P = own[f], N = nei[f];
  double dP2 = 0.0, dN2 = 0.0;
  for (int x = 0; x < 3; ++x) {
    double sh = x < dim ? shift[(int64_t)dim * f + x] : 0.0;
    double xP = xc[3 * P + x], xN = xc[3 * N + x] + sh;
    dvec[3 * f + x] = xN - xP;
    double a = xP - xf[3 * f + x], b = xN - xf[3 * f + x];
    dP2 += a * a;
    dN2 += b * b;
  }
  const double dP = sqrt(dP2), dN = sqrt(dN2);
  const double om = dN / (dP + dN);
  omega[f] = om;
  g[f] = om / (1.0 - om);
  if (!(om > 0.0 && om < 1.0)) atomicOr(flag, 4);
}

template <class T>
__global__ void k_entry_fill(int64_t ne, const int32_t* __restrict__ ent_face,
                             const double* __restrict__ S, const double* __restrict__ omega,
                             const double* __restrict__ dvec, T* __restrict__ sw, T* __restrict__ dc) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int f = ent_face[e];
  sw[4 * e + 0] = (T)S[3 * f + 0];
  sw[4 * e + 1] = (T)S[3 * f + 1];
  sw[4 * e + 2] = (T)S[3 * f + 2];
  sw[4 * e + 3] = (T)omega[f];
  T* o = dc + (int64_t)DC_VALUES * e;
  o[0] = (T)dvec[3 * f + 0];
  o[1] = (T)dvec[3 * f + 1];
  o[2] = (T)dvec[3 * f + 2];
  // the flux kernels evaluate the coefficients from the growth rate
  // omega / (1 - omega) of the entry's omega (coefficients.hpp)
}

// Auxiliary cells of boundary faces: the mirror image of the boundary cell
// in the face plane, x_O = x_C + 2 ((x_f - x_C).n) n, the same volume;
// outward unit normal and normal centre-to-face distance for the conditions.
__global__ void k_ghost_geom(int64_t ng, int64_t n_int, const int32_t* __restrict__ gh_cell,
                             const int32_t* __restrict__ gh_face, const double* __restrict__ S,
                             const double* __restrict__ xf, double* __restrict__ V, double* __restrict__ xc,
                             double* __restrict__ gh_n, double* __restrict__ gh_dist) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ng) return;
  const int64_t C = gh_cell[k], O = n_int + k, f = gh_face[k];
  V[O] = V[C];
  double a2 = 0.0;
  for (int x = 0; x < 3; ++x) a2 += S[3 * f + x] * S[3 * f + x];
  const double ia = 1.0 / sqrt(a2);
  double dn = 0.0;
  for (int x = 0; x < 3; ++x) {
    gh_n[3 * k + x] = S[3 * f + x] * ia;
    dn += (xf[3 * f + x] - xc[3 * C + x]) * gh_n[3 * k + x];
  }
  for (int x = 0; x < 3; ++x) xc[3 * O + x] = xc[3 * C + x] + 2.0 * dn * gh_n[3 * k + x];
  gh_dist[k] = dn;
}

// Sliced-ELL face records of every cell (layout: see internal.hpp), from
// the per-entry records sw and dc already in the working type.
template <class T>
__global__ void k_ell_fill(int64_t nc, int B, const int32_t* __restrict__ part_ptr,
                           const int32_t* __restrict__ slot_ptr, const uint16_t* __restrict__ slots,
                           const int2* __restrict__ ent_pn, const int32_t* __restrict__ ell_ptr,
                           const T* __restrict__ sw, const T* __restrict__ dc, T* __restrict__ ell_sw,
                           T* __restrict__ ell_d) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int64_t b = c / ELL_BLOCK;
  const int lane = (int)(c - b * ELL_BLOCK);
  const int r0 = ell_ptr[b], m = (ell_ptr[b + 1] - r0) / ELL_BLOCK;
  const int e0 = part_ptr[c / B];
  const int s0 = slot_ptr[c], nf = slot_ptr[c + 1] - s0;
  for (int j = 0; j < m; ++j) {
    const int64_t r = (int64_t)r0 + (int64_t)j * ELL_BLOCK + lane;
    T* q = ell_sw + 4 * r;
    T* dd = ell_d + 3 * r;
    int64_t o = c;
    if (j < nf) {
      const uint16_t sl = slots[s0 + j];
      const bool nb = (sl >> 15) != 0;
      const int64_t e = e0 + (sl & 0x7fff);
      const int2 pn = ent_pn[e];
      o = nb ? pn.x : pn.y;
      const T om = sw[4 * e + 3];
      const T wgt = nb ? -om : T(1) - om;
      const T sg = nb ? T(-1) : T(1);
      for (int x = 0; x < 3; ++x) {
        q[x] = wgt * sw[4 * e + x];
        dd[x] = sg * dc[(int64_t)DC_VALUES * e + x];
      }
    } else {
      for (int x = 0; x < 4; ++x) q[x] = T(0);
      for (int x = 0; x < 3; ++x) dd[x] = T(0);
    }
    if constexpr (sizeof(T) == 4) {
      q[3] = __int_as_float((int)o);
    } else {
      q[3] = __longlong_as_double((long long)o);
    }
  }
}

template <class T>
__global__ void k_recip(int64_t n, const double* __restrict__ V, T* __restrict__ rV) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) rV[c] = (T)(1.0 / V[c]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

hipError_t launch_geometry(dolinc_ctx_s* c, hipStream_t s) {
  DevMesh& m = c->m;
  hipLaunchKernelGGL(k_face_geom, dim3(nblk(c->n_faces)), dim3(TPB), 0, s, c->n_faces, c->dim, m.fptr, m.fnodes,
                     m.nodes, m.S, m.xf, m.fanc);
  hipLaunchKernelGGL(k_cell_geom, dim3(nblk(c->n_interior)), dim3(TPB), 0, s, c->n_interior, c->dim, c->part_cells,
                     m.part_ptr, m.ent_face, m.slot_ptr, m.slots, m.fptr, m.fnodes, m.nodes, m.shift, m.S, m.xf,
                     m.fanc, m.V, m.xc, c->w.flag);
  if (c->n_ghost)
    hipLaunchKernelGGL(k_ghost_geom, dim3(nblk(c->n_ghost)), dim3(TPB), 0, s, c->n_ghost, c->n_interior, m.gh_cell,
                       m.gh_face, m.S, m.xf, m.V, m.xc, m.gh_n, m.gh_dist);
  hipLaunchKernelGGL(k_face_scalars, dim3(nblk(c->n_faces)), dim3(TPB), 0, s, c->n_faces, c->dim, m.face_own,
                     m.face_nei, m.xc, m.shift, m.xf, m.dvec, m.omega, m.g, c->w.flag);
  return hipGetLastError();
}

hipError_t launch_entry_fill(dolinc_ctx_s* c, hipStream_t s) {
  DevMesh& m = c->m;
  if (c->w.precision == DOLINC_FP64) {
    hipLaunchKernelGGL(k_entry_fill<double>, dim3(nblk(c->n_entries)), dim3(TPB), 0, s, c->n_entries,
                       m.ent_face, m.S, m.omega, m.dvec, (double*)c->w.sw, (double*)c->w.dc);
    hipLaunchKernelGGL(k_ell_fill<double>, dim3(nblk(c->n_cells)), dim3(TPB), 0, s, c->n_cells, c->part_cells,
                       m.part_ptr, m.slot_ptr, m.slots, m.ent_pn, m.ell_ptr, (const double*)c->w.sw,
                       (const double*)c->w.dc, (double*)c->w.ell_sw, (double*)c->w.ell_d);
    hipLaunchKernelGGL(k_recip<double>, dim3(nblk(c->n_cells)), dim3(TPB), 0, s, c->n_cells, m.V,
                       (double*)c->w.rV);
  } else {
    hipLaunchKernelGGL(k_entry_fill<float>, dim3(nblk(c->n_entries)), dim3(TPB), 0, s, c->n_entries,
                       m.ent_face, m.S, m.omega, m.dvec, (float*)c->w.sw, (float*)c->w.dc);
    hipLaunchKernelGGL(k_ell_fill<float>, dim3(nblk(c->n_cells)), dim3(TPB), 0, s, c->n_cells, c->part_cells,
                       m.part_ptr, m.slot_ptr, m.slots, m.ent_pn, m.ell_ptr, (const float*)c->w.sw,
                       (const float*)c->w.dc, (float*)c->w.ell_sw, (float*)c->w.ell_d);
    hipLaunchKernelGGL(k_recip<float>, dim3(nblk(c->n_cells)), dim3(TPB), 0, s, c->n_cells, m.V,
                       (float*)c->w.rV);
  }
  return hipGetLastError();
}

}  // namespace dolinc
