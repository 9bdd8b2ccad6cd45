// Library-internal declarations shared by the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dolinc.h"
#include "mesh_prep.hpp"

namespace dolinc {

// Per-face record layout (one record per partition entry).
//   sw[e][4]  : S_x, S_y, S_z (0 in 2-D), omega (owner weight)
//   dc[e][3]  : d_x, d_y, d_z.  The flux kernel evaluates the coefficients
//               of the DOLINC representation in FP64 from the growth rate
//               g = omega / (1 - omega) of the entry's omega
//               (face_coefficients, coefficients.hpp): arithmetic is cheaper
//               than 8 more values per entry in a memory-bound kernel.
// Per-cell face records in sliced ELL order: cells are taken in blocks of
// ELL_BLOCK; block b holds m_b = (max faces of a cell in b) records per
// cell, record j of cell lane l at ell_ptr[b] + j * ELL_BLOCK + l, so that
// the lanes of a wave read consecutive records.  A cell with fewer faces is
// padded with records of zero weight that name the cell itself.
//   ell_sw[r][4] : w_o S_x, w_o S_y, w_o S_z, other cell (index bits); S is
//                  the face area vector oriented owner -> neighbour and
//                  w_o = sigma * (weight of the other cell in the face
//                  interpolation), sigma = +1 on the owner side, -1 on the
//                  neighbour side, so the Gauss-linear sum of a cell is
//                  sum_r (phi_o - phi_c) ell_sw[r][0..D).
//   ell_d[r][3]  : sigma d_x, sigma d_y, sigma d_z (0 for padding).  A cell's
//                  records j >= its face count (slot_ptr) are padding.
constexpr int ELL_BLOCK = 256;
// values per face entry in dc: d
constexpr int DC_VALUES = 3;
inline int scheme_order(int scheme) { return scheme <= 2 ? 0 : scheme <= 4 ? 1 : 2; }

struct DevMesh {
  // partitions / entries / slots
  int32_t* part_ptr = nullptr;
  int32_t* ent_face = nullptr;
  int2* ent_pn = nullptr;
  int32_t* slot_ptr = nullptr;
  uint16_t* slots = nullptr;
  int2* ent_rec = nullptr;       // [entries] ELL record of the face in its owner / neighbour cell
  // [entries] the same records as positions in the cells' record lists:
  // record = ell_ptr[cell / ELL_BLOCK] + j * ELL_BLOCK + cell % ELL_BLOCK
  // (null when a cell has more than 255 records)
  uchar2* ent_j = nullptr;
  int32_t* ell_ptr = nullptr;    // [n_cells / ELL_BLOCK + 1] record offsets
  // auxiliary cells of non-coupled boundary faces (row n_interior + k)
  int32_t* gh_cell = nullptr;    // [n_ghost] internal boundary cell
  int32_t* gh_face = nullptr;    // [n_ghost] caller face
  int32_t* gh_patch = nullptr;   // [n_ghost]
  int32_t* gh_ent = nullptr;     // [n_ghost] entry of the boundary face (cell side 0, auxiliary side 1)
  double* gh_n = nullptr;        // [n_ghost][3] outward unit normal
  double* gh_dist = nullptr;     // [n_ghost] (x_f - x_C).n
  int32_t* bc_type = nullptr;    // [n_patches]
  double* bc_val = nullptr;      // [n_patches][5]
  int32_t* face_ent = nullptr;   // one entry per caller face
  int32_t* face_own = nullptr;   // internal owner per caller face
  int32_t* face_nei = nullptr;
  // raw mesh (precompute only)
  double* nodes = nullptr;
  int64_t* fptr = nullptr;
  int32_t* fnodes = nullptr;
  double* shift = nullptr;
  // FP64 geometry
  double* V = nullptr;
  double* xc = nullptr;
  double* S = nullptr;
  double* xf = nullptr;
  double* fanc = nullptr;
  double* omega = nullptr;
  double* g = nullptr;
  double* dvec = nullptr;
};

struct Mlp {
  float* p = nullptr;              // fp32 master parameters
  float* m = nullptr;              // Adam first moment
  float* v = nullptr;              // Adam second moment
  unsigned short* w1b = nullptr;   // bf16 W1 [64][32]
  unsigned short* w2b = nullptr;   // bf16 W2 [64][64]
  float* part = nullptr;           // per-block partial gradients
  float* loss_part = nullptr;
  int part_blocks = 0;             // capacity of part in blocks
  int64_t step = 0;
};

struct Work {
  void* sw = nullptr;
  void* ell_sw = nullptr;
  void* ell_d = nullptr;
  void* dc = nullptr;
  void* rV = nullptr;
  void* G1 = nullptr;
  // second differentials contracted with each face's d, per face record:
  // Hf[r][nv] = d.H.d of record r's cell (ELL order)
  void* Hf = nullptr;
  void* W1 = nullptr;
  void* W2 = nullptr;
  float* theta = nullptr;
  unsigned short* Xf = nullptr;  // learned blend: the stage's bf16 features [n_cells][24]
  void* estate = nullptr;        // positivity rule: face-side increments [entries][2][nv]
  void* thpos = nullptr;         // positivity rule: scaling per cell [n_cells]
  double* diag = nullptr;  // partial sums for diagnostics
  int* flag = nullptr;     // device error flag
  size_t elem = 0;         // sizeof working type
  int scheme = -1, precision = -1, nv = 0, blend = 0;
};

}  // namespace dolinc

struct dolinc_ctx_s {
  int dim = 0;
  int64_t n_cells = 0, n_faces = 0, n_nodes = 0, n_entries = 0, n_parts = 0;
  int part_cells = 256;
  int64_t max_entries = 0, max_cell_faces = 0, n_ell = 0;
  int64_t n_interior = 0, n_ghost = 0;  // n_cells = n_interior + n_ghost rows
  int32_t n_patches = 0;
  std::vector<int32_t> new_of_old;
  dolinc::DevMesh m;
  dolinc::Work w;
  dolinc::Mlp mlp;
  dolinc_params params{};
  bool geometry_done = false;
  bool precomputed = false;
  // learned blend: the network runs on a second stream of the context
  // (default priority) while the second derivatives run on the caller's
  hipStream_t s_net = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // kernel timing (dolinc_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;   // kind per recorded (start, stop) pair
  size_t ev_used = 0;
};

namespace dolinc {

// Auxiliary-cell rows rewritten from the boundary conditions (boundary.hip)
enum { GHOST_U = 0, GHOST_G1 = 1, GHOST_G2 = 2, GHOST_THETA = 3, GHOST_HF = 4 };
hipError_t launch_ghost(dolinc_ctx_s* c, int what, void* arr, hipStream_t s);

// Launchers (kernels.hip / precompute.hip).  Return hipSuccess or an error.
hipError_t launch_geometry(dolinc_ctx_s* c, hipStream_t s);
hipError_t launch_entry_fill(dolinc_ctx_s* c, hipStream_t s);
// stage kernels
hipError_t launch_gradients(dolinc_ctx_s* c, const void* U, void* G1, void* G2, hipStream_t s);
hipError_t launch_grad2(dolinc_ctx_s* c, const void* G1, void* G2, hipStream_t s);
hipError_t launch_theta(dolinc_ctx_s* c, const void* U, const void* G1, float* theta, hipStream_t s);
// mode 0: out = R(Us); mode 1: out = alpha*Un + beta*(Us + dt*R(Us))
hipError_t launch_flux(dolinc_ctx_s* c, const void* Us, const void* Un, void* out, int mode, double alpha,
                       double beta, double dt, hipStream_t s);
hipError_t launch_face_export(dolinc_ctx_s* c, const void* U, void* UL, void* UR, void* F, hipStream_t s);
bool flux_supported(const dolinc_params& p, int dim);
hipError_t features_launch(dolinc_ctx_s* c, const void* U, float* X32, unsigned short* Xb, hipStream_t s);
// network parameters from a device array: copy, Adam moments cleared, bf16 copies
hipError_t mlp_set_launch(dolinc_ctx_s* c, const float* src, hipStream_t s);
hipError_t grad_features_launch(dolinc_ctx_s* c, const void* U, void* G1, unsigned short* Xf, hipStream_t s);
// X rows xstride bf16 wide (24: packed stage features, 32: the API's rows)
hipError_t mlp_forward_launch(dolinc_ctx_s* c, const unsigned short* X, int64_t n, float* theta, hipStream_t s,
                              int xstride);
// Training step with the partials in the library's fixed device array
// (dolinc_mlp_train_step_static): at most MLP_STATIC_BLOCKS blocks.
constexpr int MLP_STATIC_BLOCKS = 256;
constexpr int MLP_STATIC_MAX_DEVICES = 64;
hipError_t mlp_train_static_launch(dolinc_ctx_s* c, const unsigned short* X, const float* y, int64_t n, int nblocks,
                                   int rows_per_block, float* loss_out, float lr, float c1, float c2,
                                   hipStream_t s);
hipError_t mlp_grad_launch(dolinc_ctx_s* c, const unsigned short* X, const float* y, int64_t n, int nblocks,
                           int rows_per_block, float* grad_out, float* loss_out, int do_step, float lr, float c1,
                           float c2, hipStream_t s);

}  // namespace dolinc
