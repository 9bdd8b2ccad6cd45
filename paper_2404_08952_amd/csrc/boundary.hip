// Non-coupled boundaries through auxiliary cells (Sec. 2.6).
//
// Every boundary face f of a cell C has an auxiliary cell O (internal row
// n_interior + k for the k-th boundary face) on the far side: its centre is
// the mirror image of x_C in the face plane (so omega = 1/2, g = 1 and d is
// normal to the face) and its value is the one whose linear interpolation
// with C gives the boundary-face value T_f:   T_O = T_C + 2 (T_f - T_C),
//   Dirichlet:     T_f given;
//   Neumann:       T_f = T_C + q d_fC (q the outward normal gradient, d_fC
//                  the normal distance from the cell centre to the face);
//   zero gradient: T_f = T_C;
//   slip wall:     (Euler) density and energy copied, momentum reflected in
//                  the face plane.
// The DOLINC differentials of O are those of the field continued across the
// face by the same rule, with R = I - 2 n n^T (n the outward unit normal):
// symmetric conditions grad_O = R grad_C, hess_O = R hess_C R (the momentum
// of a slip wall, a reflected vector field: R grad_C R and
// sum_j R_ij R hess_C,j R); Dirichlet grad_O = -R grad_C, hess_O = -R hess_C R.
// These kernels rewrite the auxiliary rows of U, G1, G2 and theta after each
// of them has been produced for the interior cells.  The stage path keeps
// second differentials only as d.H.d per face record; on the face of
// an auxiliary cell d is normal to the face (R d = -d), so
// d.(R H R).d = d.H.d: the auxiliary side takes the cell side's value, negated
// for Dirichlet, and for the momentum of a slip wall sum_j R_ij h_j.
#include "internal.hpp"

namespace dolinc {
namespace {

constexpr int BTPB = 256;
// (zero gradient is the default branch: T_f = T_C)
constexpr int BC_DIR = DOLINC_BC_DIRICHLET, BC_NEU = DOLINC_BC_NEUMANN, BC_WALL = DOLINC_BC_SLIP_WALL;

struct GhostArgs {
  int64_t ng, n_int;
  int dim, nv, euler;
  const int32_t* cell;
  const int32_t* ent;  // [ng] entry of the boundary face (cell side 0)
  const int2* ent_rec; // [entries] face records of the entry's two cells
  const int32_t* patch;
  const double* n;     // [ng][3]
  const double* dist;  // [ng] (x_f - x_C).n
  const int32_t* bc_type;
  const double* bc_val;  // [n_patches][5]
};

__device__ __forceinline__ void reflection(const GhostArgs& a, int64_t k, double R[3][3]) {
  const double* n = a.n + 3 * k;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * n[i] * n[j];
}

template <class T>
__global__ void k_ghost_values(GhostArgs a, T* __restrict__ U) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ng) return;
  const int64_t C = a.cell[k], O = a.n_int + k;
  const int p = a.patch[k];
  const int typ = a.bc_type[p];
  const double* val = a.bc_val + 5 * p;
  const T* uc = U + C * a.nv;
  T* uo = U + O * a.nv;
  for (int v = 0; v < a.nv; ++v) {
    T tf = uc[v];
    if (typ == BC_DIR) tf = (T)val[v];
    else if (typ == BC_NEU) tf = uc[v] + (T)(val[v] * a.dist[k]);
    uo[v] = uc[v] + T(2) * (tf - uc[v]);
  }
  if (a.euler && typ == BC_WALL) {
    double R[3][3];
    reflection(a, k, R);
    for (int i = 0; i < a.dim; ++i) {
      T m = T(0);
      for (int j = 0; j < a.dim; ++j) m += (T)R[i][j] * uc[1 + j];
      uo[1 + i] = m;
    }
  }
}

// G1 rows [n_rows][nv][dim]
template <class T>
__global__ void k_ghost_grad(GhostArgs a, T* __restrict__ G) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ng) return;
  const int D = a.dim;
  const int64_t C = a.cell[k], O = a.n_int + k;
  const int typ = a.bc_type[a.patch[k]];
  double R[3][3];
  reflection(a, k, R);
  const T* gc = G + C * a.nv * D;
  T* go = G + O * a.nv * D;
  const T sgn = typ == BC_DIR ? T(-1) : T(1);
  for (int v = 0; v < a.nv; ++v)
    for (int x = 0; x < D; ++x) {
      T s = T(0);
      for (int y = 0; y < D; ++y) s += (T)R[x][y] * gc[v * D + y];
      go[v * D + x] = sgn * s;
    }
  if (a.euler && typ == BC_WALL) {
    // momentum Jacobian J[i][x] = d m_i / d x_x -> R J R
    for (int i = 0; i < D; ++i)
      for (int x = 0; x < D; ++x) {
        T s = T(0);
        for (int j = 0; j < D; ++j)
          for (int y = 0; y < D; ++y) s += (T)(R[i][j] * R[y][x]) * gc[(1 + j) * D + y];
        go[(1 + i) * D + x] = s;
      }
  }
}

// symmetric storage xx, yy, (zz), xy, (xz, yz)
__device__ __forceinline__ int sym_index(int D, int i, int j) {
  if (i == j) return i;
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  if (D == 2) return 2;
  return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

// G2 rows [n_rows][nv][dim (dim + 1) / 2]
template <class T>
__global__ void k_ghost_hess(GhostArgs a, T* __restrict__ H) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ng) return;
  const int D = a.dim, NS = D * (D + 1) / 2;
  const int64_t C = a.cell[k], O = a.n_int + k;
  const int typ = a.bc_type[a.patch[k]];
  double R[3][3];
  reflection(a, k, R);
  const T* hc = H + C * a.nv * NS;
  T* ho = H + O * a.nv * NS;
  const T sgn = typ == BC_DIR ? T(-1) : T(1);
  const bool wall = a.euler && typ == BC_WALL;
  for (int v = 0; v < a.nv; ++v) {
    const bool mom = wall && v >= 1 && v <= D;
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j) {
        // (R H R)_ij, and for a reflected vector component sum_w R_{v,w} (R H_w R)_ij
        T s = T(0);
        for (int c = 0; c < D; ++c)
          for (int d = 0; d < D; ++d) {
            const double r2 = R[i][c] * R[d][j];
            if (mom) {
              for (int w = 0; w < D; ++w) s += (T)(R[v - 1][w] * r2) * hc[(1 + w) * NS + sym_index(D, c, d)];
            } else {
              s += (T)r2 * hc[v * NS + sym_index(D, c, d)];
            }
          }
        ho[v * NS + sym_index(D, i, j)] = mom ? s : sgn * s;
      }
  }
}

// Hf [records][nv]: the auxiliary cell's record of every boundary face
template <class T>
__global__ void k_ghost_hface(GhostArgs a, T* __restrict__ Hf) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ng) return;
  const int typ = a.bc_type[a.patch[k]];
  const int2 rc = a.ent_rec[a.ent[k]];
  const T* hc = Hf + (int64_t)rc.x * a.nv;
  T* ho = Hf + (int64_t)rc.y * a.nv;
  const T sgn = typ == BC_DIR ? T(-1) : T(1);
  for (int v = 0; v < a.nv; ++v) ho[v] = sgn * hc[v];
  if (a.euler && typ == BC_WALL) {
    double R[3][3];
    reflection(a, k, R);
    for (int i = 0; i < a.dim; ++i) {
      T m = T(0);
      for (int j = 0; j < a.dim; ++j) m += (T)R[i][j] * hc[1 + j];
      ho[1 + i] = m;
    }
  }
}

__global__ void k_ghost_theta(GhostArgs a, float* __restrict__ th) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ng) return;
  th[a.n_int + k] = th[a.cell[k]];
}

GhostArgs ghost_args(dolinc_ctx_s* c) {
  GhostArgs a{};
  a.ng = c->n_ghost;
  a.n_int = c->n_interior;
  a.dim = c->dim;
  a.nv = c->w.nv;
  a.euler = c->params.pde == DOLINC_EULER;
  a.cell = c->m.gh_cell;
  a.ent = c->m.gh_ent;
  a.ent_rec = c->m.ent_rec;
  a.patch = c->m.gh_patch;
  a.n = c->m.gh_n;
  a.dist = c->m.gh_dist;
  a.bc_type = c->m.bc_type;
  a.bc_val = c->m.bc_val;
  return a;
}

}  // namespace

hipError_t launch_ghost(dolinc_ctx_s* c, int what, void* arr, hipStream_t s) {
  if (c->n_ghost == 0 || !arr) return hipSuccess;
  const GhostArgs a = ghost_args(c);
  const dim3 grid((unsigned)((a.ng + BTPB - 1) / BTPB)), blk(BTPB);
  const bool f64 = c->w.precision == DOLINC_FP64;
  switch (what) {
    case GHOST_U:
      if (f64) hipLaunchKernelGGL(k_ghost_values<double>, grid, blk, 0, s, a, (double*)arr);
      else hipLaunchKernelGGL(k_ghost_values<float>, grid, blk, 0, s, a, (float*)arr);
      break;
    case GHOST_G1:
      if (f64) hipLaunchKernelGGL(k_ghost_grad<double>, grid, blk, 0, s, a, (double*)arr);
      else hipLaunchKernelGGL(k_ghost_grad<float>, grid, blk, 0, s, a, (float*)arr);
      break;
    case GHOST_G2:
      if (f64) hipLaunchKernelGGL(k_ghost_hess<double>, grid, blk, 0, s, a, (double*)arr);
      else hipLaunchKernelGGL(k_ghost_hess<float>, grid, blk, 0, s, a, (float*)arr);
      break;
    case GHOST_HF:
      if (f64) hipLaunchKernelGGL(k_ghost_hface<double>, grid, blk, 0, s, a, (double*)arr);
      else hipLaunchKernelGGL(k_ghost_hface<float>, grid, blk, 0, s, a, (float*)arr);
      break;
    case GHOST_THETA:
      hipLaunchKernelGGL(k_ghost_theta, grid, blk, 0, s, a, (float*)arr);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dolinc
