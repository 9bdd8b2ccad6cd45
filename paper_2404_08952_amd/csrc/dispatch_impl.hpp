// Launch-side dispatch from runtime parameters to kernel instantiations.
// Included once per working type (kernels_f64.hip, kernels_f32.hip).
#pragma once
#include "residual_impl.hpp"

namespace dolinc {

template <class T>
KArgs<T> base_args(dolinc_ctx_s* c) {
  KArgs<T> a{};
  a.nc = c->n_cells;
  a.np = (int)c->n_parts;
  a.B = c->part_cells;
  a.per_xcd = (int)((c->n_parts + 7) / 8);
  a.n_cell_blocks = (int)((c->n_cells + KTPB - 1) / KTPB);
  a.cell_per_xcd = (a.n_cell_blocks + 7) / 8;
  a.part_ptr = c->m.part_ptr;
  a.ent_pn = c->m.ent_pn;
  a.slot_ptr = c->m.slot_ptr;
  a.slots = c->m.slots;
  a.ell_ptr = c->m.ell_ptr;
  a.sw = (const T*)c->w.sw;
  a.ell_sw = (const T*)c->w.ell_sw;
  a.ell_d = (const T*)c->w.ell_d;
  a.dc = (const T*)c->w.dc;
  a.rV = (const T*)c->w.rV;
  a.G1 = (const T*)c->w.G1;
  a.Hf = (const T*)c->w.Hf;
  a.ent_rec = c->m.ent_rec;
  a.ent_j = c->m.ent_j;
  a.theta = c->w.theta;
  a.gamma = (T)c->params.gamma;
  for (int k = 0; k < 3; ++k) {
    a.adv[k] = (T)c->params.adv_vel[k];
    a.bdir[k] = (T)c->params.burgers_dir[k];
  }
  for (int k = 0; k < 5; ++k) a.uref[k] = (T)c->params.u_ref[k];
  a.face_ent = c->m.face_ent;
  a.nf = c->n_faces;
  a.max_entries = c->max_entries;
  // the positivity rule's workspace (only with params.positivity)
  a.estate = (T*)c->w.estate;
  a.thpos = (T*)c->w.thpos;
  return a;
}

// LDS one workgroup may use on the current device (queried once per process).
inline size_t flux_lds_limit() {
  static size_t lim = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    return (size_t)v;
  }();
  return lim;
}

// pk: 0 advection, 1 Burgers, 2 Euler-Rusanov, 3 Euler-HLLC
inline int pde_kind(const dolinc_params& p) {
  if (p.pde == DOLINC_ADVECTION) return 0;
  if (p.pde == DOLINC_BURGERS) return 1;
  return p.flux == DOLINC_FLUX_HLLC ? 3 : 2;
}

template <class T, int D, int PK, int SCH, bool BL, int REF>
hipError_t go_flux(const KArgs<T>& a0, size_t lds, hipStream_t s, bool exporting) {
  KArgs<T> a = a0;
  if constexpr (PK >= 2 && REF != 1) {
    if (a.thpos) {
      // positivity rule of the cell averages: the face-side increments and
      // theta_pos per cell first (LDS: both increments and the area per entry)
      const size_t lds1 = (size_t)a.max_entries * (2 * NVars<PK, D>::value + 1) * sizeof(T);
      if (lds1 > flux_lds_limit()) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_pos_states<T, D, PK, SCH, BL, REF>), dim3(8 * a.per_xcd), dim3(KTPB), lds1, s, a);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (!exporting) {
        if (lds > flux_lds_limit()) return hipErrorInvalidConfiguration;
        if (a.B >= 2 * KTPB)
          hipLaunchKernelGGL((k_flux<T, D, PK, SCH, BL, REF, 2, 2 * KTPB>), dim3(8 * a.per_xcd), dim3(2 * KTPB), lds,
                             s, a);
        else
          hipLaunchKernelGGL((k_flux<T, D, PK, SCH, BL, REF, 2>), dim3(8 * a.per_xcd), dim3(KTPB), lds, s, a);
        return hipGetLastError();
      }
    }
  }
  if (!a.thpos) a.estate = nullptr;  // export reads the scaled states only after the first pass
  if (exporting) {
    const unsigned nb = (unsigned)((a.nf + KTPB - 1) / KTPB);
    hipLaunchKernelGGL((k_face_export<T, D, PK, SCH, BL, REF>), dim3(nb), dim3(KTPB), 0, s, a);
    return hipGetLastError();
  }
  // LDS holds the partition's face fluxes only (rows are gathered from HBM/L2)
  if (lds > flux_lds_limit()) return hipErrorInvalidConfiguration;
  // partitions of 512 cells or more: 512 threads, so the workgroup still
  // has one thread per cell in the accumulation
  if (a.B >= 2 * KTPB)
    hipLaunchKernelGGL((k_flux<T, D, PK, SCH, BL, REF, 0, 2 * KTPB>), dim3(8 * a.per_xcd), dim3(2 * KTPB), lds, s, a);
  else
    hipLaunchKernelGGL((k_flux<T, D, PK, SCH, BL, REF, 0>), dim3(8 * a.per_xcd), dim3(KTPB), lds, s, a);
  return hipGetLastError();
}

template <class T, int D, int PK, bool BL, int REF>
hipError_t flux_by_scheme(int sch, const KArgs<T>& a, size_t lds, hipStream_t s, bool ex) {
  switch (sch) {
    case 1: return go_flux<T, D, PK, 1, BL, REF>(a, lds, s, ex);
    case 2: return go_flux<T, D, PK, 2, BL, REF>(a, lds, s, ex);
    case 3: return go_flux<T, D, PK, 3, BL, REF>(a, lds, s, ex);
    case 4: return go_flux<T, D, PK, 4, BL, REF>(a, lds, s, ex);
    case 5: return go_flux<T, D, PK, 5, BL, REF>(a, lds, s, ex);
    case 6: return go_flux<T, D, PK, 6, BL, REF>(a, lds, s, ex);
    case 7: return go_flux<T, D, PK, 7, BL, REF>(a, lds, s, ex);
    case 8: return go_flux<T, D, PK, 8, BL, REF>(a, lds, s, ex);
  }
  return hipErrorInvalidValue;
}

template <class T, int PK, bool BL>
hipError_t euler_by_ref(int ref, const KArgs<T>& a, int sch, size_t lds, hipStream_t s, bool ex) {
  if (ref == 1) return flux_by_scheme<T, 3, PK, BL, 1>(sch, a, lds, s, ex);
  if (ref == 2) return flux_by_scheme<T, 3, PK, BL, 2>(sch, a, lds, s, ex);
  return flux_by_scheme<T, 3, PK, BL, 0>(sch, a, lds, s, ex);
}

// LDS of the flux kernel: one flux per face entry, two (the owner's and the
// neighbour's share) in the cell-reference form
inline size_t flux_lds_bytes(const dolinc_ctx_s* c, int nv, size_t el) {
  const int per = c->params.use_u_ref == 2 ? 2 : 1;
  return (size_t)c->max_entries * nv * el * per;
}

template <class T>
hipError_t run_flux(dolinc_ctx_s* c, const KArgs<T>& a, hipStream_t s, bool ex) {
  const int pk = pde_kind(c->params);
  const int nv = c->w.nv;
  const size_t lds = flux_lds_bytes(c, nv, sizeof(T));
  const bool bl = c->params.blend != DOLINC_BLEND_NONE;
  const int sch = c->params.scheme;
  const int ref = c->params.use_u_ref;
  // scalar laws: full states or each face side about its own cell
  const bool cell = ref == 2;
  if (c->dim == 2) {
    if (pk == 0) return cell ? flux_by_scheme<T, 2, 0, false, 2>(sch, a, lds, s, ex)
                             : flux_by_scheme<T, 2, 0, false, 0>(sch, a, lds, s, ex);
    if (pk == 1) return cell ? flux_by_scheme<T, 2, 1, false, 2>(sch, a, lds, s, ex)
                             : flux_by_scheme<T, 2, 1, false, 0>(sch, a, lds, s, ex);
    return hipErrorInvalidValue;
  }
  if (pk == 0) return cell ? flux_by_scheme<T, 3, 0, false, 2>(sch, a, lds, s, ex)
                           : flux_by_scheme<T, 3, 0, false, 0>(sch, a, lds, s, ex);
  if (pk == 1) return cell ? flux_by_scheme<T, 3, 1, false, 2>(sch, a, lds, s, ex)
                           : flux_by_scheme<T, 3, 1, false, 0>(sch, a, lds, s, ex);
  if (pk == 2) return bl ? euler_by_ref<T, 2, true>(ref, a, sch, lds, s, ex) : euler_by_ref<T, 2, false>(ref, a, sch, lds, s, ex);
  return bl ? euler_by_ref<T, 3, true>(ref, a, sch, lds, s, ex) : euler_by_ref<T, 3, false>(ref, a, sch, lds, s, ex);
}

// 3-D Euler second derivatives: the FP32 kernel is built for 5 waves per SIMD
template <class T>
void launch_grad2_euler(dim3 grid, dim3 blk, hipStream_t s, const KArgs<T>& a, const T* g1, T* g2) {
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((k_grad_w5<T, 3, 15, true>), grid, blk, 0, s, a, g1, g2);
  else
    hipLaunchKernelGGL((k_grad<T, 3, 15, true>), grid, blk, 0, s, a, g1, g2);
}

template <class T>
hipError_t run_gradients(dolinc_ctx_s* c, const void* U, void* G1, void* G2, hipStream_t s) {
  KArgs<T> a = base_args<T>(c);
  const dim3 grid(8 * a.cell_per_xcd), blk(KTPB);
  const int nv = c->w.nv;
  const T* u = (const T*)U;
  T* g1 = (T*)G1;
  T* g2 = (T*)G2;
  if (c->dim == 2) {
    if (nv != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_grad<T, 2, 1, false>), grid, blk, 0, s, a, u, g1);
    if (g2) hipLaunchKernelGGL((k_grad<T, 2, 2, true>), grid, blk, 0, s, a, (const T*)g1, g2);
  } else if (nv == 1) {
    hipLaunchKernelGGL((k_grad<T, 3, 1, false>), grid, blk, 0, s, a, u, g1);
    if (g2) hipLaunchKernelGGL((k_grad<T, 3, 3, true>), grid, blk, 0, s, a, (const T*)g1, g2);
  } else {
    hipLaunchKernelGGL((k_grad<T, 3, 5, false>), grid, blk, 0, s, a, u, g1);
    if (g2) launch_grad2_euler<T>(grid, blk, s, a, (const T*)g1, g2);
  }
  return hipGetLastError();
}

template <class T>
hipError_t run_grad2(dolinc_ctx_s* c, const void* G1, void* G2, hipStream_t s) {
  KArgs<T> a = base_args<T>(c);
  const dim3 grid(8 * a.cell_per_xcd), blk(KTPB);
  const int nv = c->w.nv;
  if (c->dim == 2)
    hipLaunchKernelGGL((k_grad<T, 2, 2, true>), grid, blk, 0, s, a, (const T*)G1, (T*)G2);
  else if (nv == 1)
    hipLaunchKernelGGL((k_grad<T, 3, 3, true>), grid, blk, 0, s, a, (const T*)G1, (T*)G2);
  else
    launch_grad2_euler<T>(grid, blk, s, a, (const T*)G1, (T*)G2);
  return hipGetLastError();
}

// Second differentials contracted per face entry (stage path).  3-D Euler
// in FP32 is built for 5 waves per SIMD like the row kernel.
template <class T>
hipError_t run_hface(dolinc_ctx_s* c, const void* G1, void* Hf, hipStream_t s) {
  KArgs<T> a = base_args<T>(c);
  const dim3 grid(8 * a.cell_per_xcd), blk(KTPB);
  const int nv = c->w.nv;
  const T* g1 = (const T*)G1;
  T* hf = (T*)Hf;
  if (c->dim == 2) {
    if (nv != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_hface<T, 2, 1>), grid, blk, 0, s, a, g1, hf);
  } else if (nv == 1) {
    hipLaunchKernelGGL((k_hface<T, 3, 1>), grid, blk, 0, s, a, g1, hf);
  } else if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL((k_hface_w5<T, 3, 5>), grid, blk, 0, s, a, g1, hf);
  } else {
    hipLaunchKernelGGL((k_hface<T, 3, 5>), grid, blk, 0, s, a, g1, hf);
  }
  return hipGetLastError();
}

template <class T>
hipError_t run_theta(dolinc_ctx_s* c, const void* U, const void* G1, float* theta, hipStream_t s) {
  KArgs<T> a = base_args<T>(c);
  a.U = (const T*)U;
  a.G1 = (const T*)G1;
  const dim3 grid(8 * a.cell_per_xcd), blk(KTPB);
  if (c->dim == 2) {
    hipLaunchKernelGGL((k_theta<T, 2, 1>), grid, blk, 0, s, a, theta);
  } else if (c->w.nv == 1) {
    hipLaunchKernelGGL((k_theta<T, 3, 1>), grid, blk, 0, s, a, theta);
  } else {
    hipLaunchKernelGGL((k_theta<T, 3, 5>), grid, blk, 0, s, a, theta);
  }
  return hipGetLastError();
}

// Per-block partial diagnostics: [sum V*U_v (v < nv), min q0, min p | max q0, nonfinite]
template <class T>
__global__ __launch_bounds__(KTPB) void k_diag(int64_t nc, int nv, int euler, T gamma, const T* __restrict__ U,
                                               const double* __restrict__ V, double* __restrict__ part) {
  __shared__ double red[KTPB];
  double acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  double mn0 = 1e300, m2 = euler ? 1e300 : -1e300, bad = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * KTPB + threadIdx.x; c < nc; c += (int64_t)gridDim.x * KTPB) {
    const double vol = V[c];
    double ke = 0.0;
    for (int v = 0; v < nv; ++v) {
      const double x = (double)U[c * nv + v];
      if (!isfinite(x)) bad += 1.0;
      acc[v] += vol * x;
    }
    const double q0 = (double)U[c * nv];
    mn0 = fmin(mn0, q0);
    if (euler) {
      for (int v = 1; v < nv - 1; ++v) ke += (double)U[c * nv + v] * (double)U[c * nv + v];
      const double p = ((double)gamma - 1.0) * ((double)U[c * nv + nv - 1] - 0.5 * ke / q0);
      m2 = fmin(m2, p);
    } else {
      m2 = fmax(m2, q0);
    }
  }
  const int nout = nv + 3;
  for (int k = 0; k < nout; ++k) {
    double x = k < nv ? acc[k] : (k == nv ? mn0 : (k == nv + 1 ? m2 : bad));
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = KTPB / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        double y = red[threadIdx.x + w];
        double z = red[threadIdx.x];
        if (k < nv || k == nv + 2)
          red[threadIdx.x] = z + y;
        else if (k == nv || euler)
          red[threadIdx.x] = fmin(z, y);
        else
          red[threadIdx.x] = fmax(z, y);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nout + k] = red[0];
    __syncthreads();
  }
}

// The partials of k_diag combined in block order into out[nout] (one thread
// per output; the same order every call, so repeated calls agree bit for bit)
template <class T>
__global__ void k_diag_reduce(int nb, int nv, int euler, const double* __restrict__ part, double* __restrict__ out) {
  const int k = threadIdx.x;
  const int nout = nv + 3;
  if (k >= nout) return;
  const bool add = k < nv || k == nv + 2;
  const bool take_min = k == nv || euler;
  double acc = add ? 0.0 : (take_min ? 1e300 : -1e300);
  for (int b = 0; b < nb; ++b) {
    const double x = part[(int64_t)b * nout + k];
    acc = add ? acc + x : (take_min ? fmin(acc, x) : fmax(acc, x));
  }
  out[k] = acc;
}

template <class T>
hipError_t run_diag(dolinc_ctx_s* c, const void* U, double* part, int nblocks, double* out, hipStream_t s) {
  const int euler = c->params.pde == DOLINC_EULER;
  // interior cells only (auxiliary rows follow them)
  hipLaunchKernelGGL(k_diag<T>, dim3(nblocks), dim3(KTPB), 0, s, c->n_interior, c->w.nv, euler, (T)c->params.gamma,
                     (const T*)U, c->m.V, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_reduce<T>, dim3(1), dim3(64), 0, s, nblocks, c->w.nv, euler, (const double*)part, out);
  return hipGetLastError();
}

}  // namespace dolinc
