// C ABI of the DOLINC residual library (declarations and contracts in
// include/dolinc.h).  Host orchestration only: every compute step is a HIP
// kernel enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.hpp"

namespace dolinc {
hipError_t flux_f64(dolinc_ctx_s*, const void*, const void*, void*, int, double, double, double, hipStream_t);
hipError_t flux_f32(dolinc_ctx_s*, const void*, const void*, void*, int, double, double, double, hipStream_t);
hipError_t export_f64(dolinc_ctx_s*, const void*, void*, void*, void*, hipStream_t);
hipError_t export_f32(dolinc_ctx_s*, const void*, void*, void*, void*, hipStream_t);
hipError_t grad_f64(dolinc_ctx_s*, const void*, void*, void*, hipStream_t);
hipError_t grad_f32(dolinc_ctx_s*, const void*, void*, void*, hipStream_t);
hipError_t grad2_f64(dolinc_ctx_s*, const void*, void*, hipStream_t);
hipError_t grad2_f32(dolinc_ctx_s*, const void*, void*, hipStream_t);
hipError_t hface_f64(dolinc_ctx_s*, const void*, void*, hipStream_t);
hipError_t hface_f32(dolinc_ctx_s*, const void*, void*, hipStream_t);
hipError_t theta_f64(dolinc_ctx_s*, const void*, const void*, float*, hipStream_t);
hipError_t theta_f32(dolinc_ctx_s*, const void*, const void*, float*, hipStream_t);
hipError_t diag_f64(dolinc_ctx_s*, const void*, double*, int, double*, hipStream_t);
hipError_t diag_f32(dolinc_ctx_s*, const void*, double*, int, double*, hipStream_t);
}  // namespace dolinc

using namespace dolinc;

namespace {

thread_local std::string g_err;
constexpr int KTPB_HOST = 256;

// Live contexts, so that a destroyed or foreign handle is reported instead
// of dereferenced.
std::mutex g_live_mu;
std::set<const void*> g_live;

dolinc_status fail(dolinc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(DOLINC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool valid_ctx(dolinc_ctx c) {
  if (!c) return false;
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count((const void*)c) != 0;
}

// Device copy of a host array, enqueued on stream s (the host array must
// outlive the copy: dolinc_create synchronises s before its host vectors go).
template <class X>
hipError_t upload(X** dst, const X* src, size_t n, hipStream_t s) {
  hipError_t e = hipMalloc((void**)dst, n * sizeof(X) + (n == 0 ? sizeof(X) : 0));
  if (e != hipSuccess) return e;
  if (n) e = hipMemcpyAsync(*dst, src, n * sizeof(X), hipMemcpyHostToDevice, s);
  return e;
}

void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}
template <class X>
void dfree_t(X*& p) {
  void* q = (void*)p;
  dfree(q);
  p = nullptr;
}

void free_work(dolinc_ctx c) {
  Work& w = c->w;
  dfree(w.sw); dfree(w.ell_sw); dfree(w.ell_d); dfree(w.dc); dfree(w.rV); dfree(w.G1); dfree(w.Hf); dfree(w.W1); dfree(w.W2);
  dfree_t(w.theta);
  dfree_t(w.Xf);
  dfree(w.estate);
  dfree(w.thpos);
  w.scheme = w.precision = -1;
  w.nv = 0;
}

void free_mlp(dolinc_ctx c);

void free_all(dolinc_ctx c) {
  free_work(c);
  free_mlp(c);
  DevMesh& m = c->m;
  dfree_t(m.part_ptr); dfree_t(m.ent_face); dfree_t(m.ent_pn); dfree_t(m.slot_ptr); dfree_t(m.slots);
  dfree_t(m.ent_rec); dfree_t(m.ent_j); dfree_t(m.ell_ptr);
  dfree_t(m.gh_cell); dfree_t(m.gh_face); dfree_t(m.gh_patch); dfree_t(m.gh_ent); dfree_t(m.gh_n); dfree_t(m.gh_dist);
  dfree_t(m.bc_type); dfree_t(m.bc_val);
  dfree_t(m.face_ent); dfree_t(m.face_own); dfree_t(m.face_nei);
  dfree_t(m.nodes); dfree_t(m.fptr); dfree_t(m.fnodes); dfree_t(m.shift);
  dfree_t(m.V); dfree_t(m.xc); dfree_t(m.S); dfree_t(m.xf); dfree_t(m.fanc); dfree_t(m.omega); dfree_t(m.g);
  dfree_t(m.dvec);
  dfree_t(c->w.diag);
  dfree_t(c->w.flag);
}

dolinc_status check_params(const dolinc_params* p, int dim) {
  if (!p) return fail(DOLINC_EINVAL, "params is NULL");
  if (p->pde < 0 || p->pde > 2) return fail(DOLINC_EINVAL, "unknown pde");
  if (p->scheme < 1 || p->scheme > 8) return fail(DOLINC_EINVAL, "unknown scheme");
  if (p->precision < 0 || p->precision > 1) return fail(DOLINC_EINVAL, "unknown precision");
  if (p->blend < 0 || p->blend > 3) return fail(DOLINC_EINVAL, "unknown blend");
  if (p->flux < 0 || p->flux > 2) return fail(DOLINC_EINVAL, "unknown flux");
  if (p->pde != DOLINC_EULER && p->flux != DOLINC_FLUX_UPWIND)
    return fail(DOLINC_EINVAL, "scalar equations use the upwind (Godunov) flux");
  if (p->pde == DOLINC_EULER && p->flux == DOLINC_FLUX_UPWIND)
    return fail(DOLINC_EINVAL, "Euler needs the Rusanov or HLLC flux");
  if (p->pde == DOLINC_EULER && dim != 3) return fail(DOLINC_EUNSUPPORTED, "Euler is built for dim = 3");
  if (p->blend != DOLINC_BLEND_NONE && p->pde != DOLINC_EULER)
    return fail(DOLINC_EUNSUPPORTED, "blending is built for the Euler equations");
  if (p->pde == DOLINC_EULER && !(p->gamma > 1.0 && std::isfinite(p->gamma)))
    return fail(DOLINC_EINVAL, "gamma must be > 1");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(p->adv_vel[k]) || !std::isfinite(p->burgers_dir[k]))
      return fail(DOLINC_EINVAL, "non-finite velocity");
  if (p->use_u_ref < 0 || p->use_u_ref > 2) return fail(DOLINC_EINVAL, "use_u_ref must be 0, 1 or 2");
  if (p->positivity) {
    if (p->pde != DOLINC_EULER) return fail(DOLINC_EUNSUPPORTED, "the positivity rule is built for the Euler equations");
    if (p->use_u_ref == 1) return fail(DOLINC_EUNSUPPORTED, "the positivity rule takes use_u_ref 0 or 2");
  }
  if (p->use_u_ref == 1) {
    if (p->pde != DOLINC_EULER)
      return fail(DOLINC_EUNSUPPORTED, "the constant reference state is built for the Euler equations");
    for (int k = 0; k < 5; ++k)
      if (!std::isfinite(p->u_ref[k])) return fail(DOLINC_EINVAL, "non-finite u_ref");
  }
  return DOLINC_OK;
}

// HIP events around a launch when timing is on (kind: 0 grad1, 1 grad2,
// 2 sensor, 3 flux + update)
struct TimedLaunch {
  dolinc_ctx c;
  hipStream_t s;
  size_t slot = (size_t)-1;
  TimedLaunch(dolinc_ctx c_, hipStream_t s_, int kind) : c(c_), s(s_) {
    if (!c->timing) return;
    if (c->ev_used + 2 > c->ev_pool.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      c->ev_pool.push_back(a);
      c->ev_pool.push_back(b);
    }
    slot = c->ev_used;
    c->ev_used += 2;
    c->ev_kind.push_back(kind);
    (void)hipEventRecord(c->ev_pool[slot], s);
  }
  ~TimedLaunch() {
    if (slot != (size_t)-1) (void)hipEventRecord(c->ev_pool[slot + 1], s);
  }
};

// Auxiliary rows of a state the caller passed as const: the state is copied
// into W1 first (only when the mesh has boundary faces).
hipError_t ghost_input(dolinc_ctx c, const void*& U, hipStream_t s) {
  if (!c->n_ghost) return hipSuccess;
  hipError_t e = hipMemcpyAsync(c->w.W1, U, (size_t)c->n_cells * c->w.nv * c->w.elem, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  U = c->w.W1;
  return launch_ghost(c, GHOST_U, c->w.W1, s);
}

hipError_t grad2_launch(dolinc_ctx c, const void* G1, void* G2, hipStream_t s) {
  hipError_t e;
  {
    TimedLaunch t(c, s, 1);
    e = c->w.precision == DOLINC_FP64 ? grad2_f64(c, G1, G2, s) : grad2_f32(c, G1, G2, s);
  }
  if (e != hipSuccess) return e;
  return launch_ghost(c, GHOST_G2, G2, s);
}

// second differentials of a stage, contracted per face record into w.Hf
hipError_t hface_launch(dolinc_ctx c, const void* G1, hipStream_t s) {
  hipError_t e;
  {
    TimedLaunch t(c, s, 1);
    e = c->w.precision == DOLINC_FP64 ? hface_f64(c, G1, c->w.Hf, s) : hface_f32(c, G1, c->w.Hf, s);
  }
  if (e != hipSuccess) return e;
  return launch_ghost(c, GHOST_HF, c->w.Hf, s);
}

hipError_t grad_dispatch(dolinc_ctx c, const void* U, void* G1, void* G2, hipStream_t s) {
  hipError_t e;
  {
    TimedLaunch t(c, s, 0);
    e = c->w.precision == DOLINC_FP64 ? grad_f64(c, U, G1, nullptr, s) : grad_f32(c, U, G1, nullptr, s);
  }
  if (e == hipSuccess) e = launch_ghost(c, GHOST_G1, G1, s);
  if (e != hipSuccess || !G2) return e;
  return grad2_launch(c, G1, G2, s);
}

// gradients (and classical theta) that one residual evaluation of U needs
hipError_t prepare_stage(dolinc_ctx c, const void* U, hipStream_t s) {
  const int ord = scheme_order(c->params.scheme);
  const bool bl = c->params.blend != DOLINC_BLEND_NONE;
  if (c->params.blend == DOLINC_BLEND_LEARNED && c->dim == 3) {
    // first gradient fused with the indicator's features (timed as the
    // indicator); the network then runs on the context's second stream
    // while the second derivatives run on the caller's, which waits for it
    // before the blend weights of the auxiliary cells and the flux kernel
    {
      TimedLaunch t(c, s, 2);
      hipError_t e = grad_features_launch(c, U, c->w.G1, c->w.Xf, s);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(c->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->s_net, c->ev_fork, 0);
    if (e == hipSuccess) e = mlp_forward_launch(c, c->w.Xf, c->n_interior, c->w.theta, c->s_net, DOLINC_N_FEATURES);
    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->s_net);
    if (e == hipSuccess) e = launch_ghost(c, GHOST_G1, c->w.G1, s);
    if (e == hipSuccess && ord >= 2) e = hface_launch(c, c->w.G1, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_join, 0);
    if (e == hipSuccess) e = launch_ghost(c, GHOST_THETA, c->w.theta, s);
    return e;
  }
  if (ord >= 1 || bl) {
    hipError_t e = grad_dispatch(c, U, c->w.G1, nullptr, s);
    if (e == hipSuccess && ord >= 2) e = hface_launch(c, c->w.G1, s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipSuccess;
  if (c->params.blend == DOLINC_BLEND_CLASSICAL) {
    TimedLaunch t(c, s, 2);
    e = c->w.precision == DOLINC_FP64 ? theta_f64(c, U, c->w.G1, c->w.theta, s)
                                      : theta_f32(c, U, c->w.G1, c->w.theta, s);
  }
  if (e != hipSuccess || !bl) return e;
  return launch_ghost(c, GHOST_THETA, c->w.theta, s);
}

hipError_t stage(dolinc_ctx c, const void* Us, const void* Un, void* out, int mode, double al, double be, double dt,
                 hipStream_t s) {
  hipError_t e = prepare_stage(c, Us, s);
  if (e != hipSuccess) return e;
  TimedLaunch t(c, s, 3);
  return c->w.precision == DOLINC_FP64 ? flux_f64(c, Us, Un, out, mode, al, be, dt, s)
                                       : flux_f32(c, Us, Un, out, mode, al, be, dt, s);
}

dolinc_status need_ready(dolinc_ctx c, bool need_mlp = true) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->precomputed) return fail(DOLINC_ESTATE, "dolinc_precompute has not been called");
  if (need_mlp && c->params.blend == DOLINC_BLEND_LEARNED && !c->mlp.p)
    return fail(DOLINC_ESTATE, "blend mode LEARNED needs dolinc_mlp_set first");
  return DOLINC_OK;
}

void free_mlp(dolinc_ctx c) {
  Mlp& m = c->mlp;
  dfree_t(m.p); dfree_t(m.m); dfree_t(m.v); dfree_t(m.w1b); dfree_t(m.w2b); dfree_t(m.part);
  dfree_t(m.loss_part);
  m.part_blocks = 0;
  m.step = 0;
}

constexpr int MLP_N = DOLINC_MLP_PARAMS;
// Training batches: blocks of at least 256 rows, at most 2048 blocks (each
// block writes one partial gradient, so the reduction reads at most 2048).
constexpr int64_t MLP_MIN_ROWS = 256, MLP_MAX_BLOCKS = 2048;
void mlp_grid(int64_t n, int* nblocks, int* rows_per_block) {
  int64_t nb = (n + MLP_MIN_ROWS - 1) / MLP_MIN_ROWS;
  if (nb > MLP_MAX_BLOCKS) nb = MLP_MAX_BLOCKS;
  int64_t rows = (n + nb - 1) / nb;
  rows = (rows + 63) / 64 * 64;
  *rows_per_block = (int)rows;
  *nblocks = (int)((n + rows - 1) / rows);
}

dolinc_status mlp_batch_check(dolinc_ctx c, const uint16_t* X, const float* y, int64_t n) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->mlp.p) return fail(DOLINC_ESTATE, "dolinc_mlp_set has not been called");
  if (!X || !y) return fail(DOLINC_EINVAL, "NULL batch");
  if (n <= 0 || n > (int64_t)1 << 30) return fail(DOLINC_EINVAL, "batch size must be in [1, 2^30]");
  int nb = 0, rows = 0;
  mlp_grid(n, &nb, &rows);
  if (nb > c->mlp.part_blocks) {
    dfree_t(c->mlp.part);
    dfree_t(c->mlp.loss_part);
    c->mlp.part_blocks = 0;
    if (hipMalloc((void**)&c->mlp.part, (size_t)nb * MLP_N * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&c->mlp.loss_part, (size_t)nb * sizeof(float)) != hipSuccess)
      return fail(DOLINC_ENOMEM, "gradient workspace allocation failed");
    c->mlp.part_blocks = nb;
  }
  return DOLINC_OK;
}

}  // namespace

extern "C" {

const char* dolinc_last_error(void) { return g_err.c_str(); }
int32_t dolinc_version(void) { return 100; }

dolinc_status dolinc_mesh_prepare(const dolinc_mesh_desc* mesh, int32_t* new_of_old, dolinc_mesh_stats* stats) {
  if (!mesh) return fail(DOLINC_EINVAL, "mesh is NULL");
  try {
    Prepared P;
    ExtendedDesc X;
    std::string msg;
    dolinc_status st = extend_desc(*mesh, X, msg);
    if (st != DOLINC_OK) return fail(st, msg);
    st = prepare_mesh(X.d, P, msg, X.n_interior);
    if (st != DOLINC_OK) return fail(st, msg);
    if (new_of_old) std::memcpy(new_of_old, P.new_of_old.data(), (size_t)X.n_interior * sizeof(int32_t));
    if (stats) {
      stats->n_parts = P.n_parts;
      stats->n_entries = (int64_t)P.ent_face.size();
      stats->max_entries = P.max_entries;
      stats->max_cell_faces = P.max_cell_faces;
      stats->n_slots = (int64_t)P.slots.size();
      stats->n_rows = P.n_cells;
      stats->n_boundary_faces = (int64_t)X.bface.size();
    }
  } catch (const std::bad_alloc&) {
    return fail(DOLINC_ENOMEM, "host allocation failed");
  }
  return DOLINC_OK;
}

dolinc_status dolinc_create(const dolinc_mesh_desc* mesh, dolinc_stream stream, dolinc_ctx* out) {
  if (!mesh || !out) return fail(DOLINC_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  *out = nullptr;
  dolinc_ctx c = nullptr;
  try {
    Prepared P;
    ExtendedDesc X;
    std::string msg;
    dolinc_status st = extend_desc(*mesh, X, msg);
    if (st != DOLINC_OK) return fail(st, msg);
    st = prepare_mesh(X.d, P, msg, X.n_interior);
    if (st != DOLINC_OK) return fail(st, msg);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(DOLINC_EHIP, "no HIP device");
    c = new dolinc_ctx_s();
    c->dim = P.dim;
    c->n_cells = P.n_cells;
    c->n_faces = P.n_faces;
    c->n_nodes = P.n_nodes;
    c->n_entries = (int64_t)P.ent_face.size();
    c->n_parts = P.n_parts;
    c->part_cells = P.part_cells;
    c->max_entries = P.max_entries;
    c->max_cell_faces = P.max_cell_faces;
    c->new_of_old = P.new_of_old;
    c->n_interior = X.n_interior;
    c->n_ghost = (int64_t)X.bface.size();
    c->n_patches = mesh->face_patch ? mesh->n_patches : 0;
    const int dim = P.dim;
    const int64_t nf = P.n_faces;
    std::vector<int2> pn(c->n_entries);
    for (int64_t e = 0; e < c->n_entries; ++e) pn[e] = make_int2(P.ent_p[e], P.ent_n[e]);
    std::vector<int32_t> fo(nf), fn(nf);
    for (int64_t f = 0; f < nf; ++f) {
      fo[f] = P.new_of_old[X.d.owner[f]];
      fn[f] = P.new_of_old[X.d.neighbour[f]];
    }
    // host sources of the asynchronous uploads below: they live until the
    // stream is synchronised at the end of the set-up
    std::vector<int32_t> gc, gp, ge, bt, ep;
    std::vector<double> bv;
    std::vector<int2> er;
    std::vector<uchar2> ej;
    DevMesh& m = c->m;
    hipError_t e = hipSuccess;
#define UP(dst, src, n)                                       \
  if (e == hipSuccess) e = upload(&(dst), (src), (size_t)(n), s);
    UP(m.part_ptr, P.part_ent_ptr.data(), P.part_ent_ptr.size());
    UP(m.ent_face, P.ent_face.data(), P.ent_face.size());
    UP(m.ent_pn, pn.data(), pn.size());
    UP(m.slot_ptr, P.slot_ptr.data(), P.slot_ptr.size());
    UP(m.slots, P.slots.data(), P.slots.size());
    UP(m.face_ent, P.face_first_ent.data(), P.face_first_ent.size());
    UP(m.face_own, fo.data(), fo.size());
    UP(m.face_nei, fn.data(), fn.size());
    UP(m.nodes, mesh->node_xyz, mesh->n_nodes * dim);
    UP(m.fptr, mesh->face_node_ptr, nf + 1);
    UP(m.fnodes, mesh->face_nodes, mesh->face_node_ptr[nf]);
    UP(m.shift, X.d.neigh_shift, nf * dim);
    if (c->n_ghost) {
      gc.resize(c->n_ghost);
      gp.resize(c->n_ghost);
      ge.resize(c->n_ghost);
      for (int64_t k = 0; k < c->n_ghost; ++k) {
        gc[k] = P.new_of_old[mesh->owner[X.bface[k]]];
        gp[k] = mesh->face_patch[X.bface[k]];
        // the face's entry in its cell's partition: owner (side 0) = the cell
        ge[k] = P.face_first_ent[X.bface[k]];
        if (P.ent_p[ge[k]] != gc[k] || P.ent_n[ge[k]] != (int32_t)(X.n_interior + k)) {
          free_all(c);
          delete c;
          return fail(DOLINC_EMESH, "internal: boundary face entry does not join its cell and auxiliary cell");
        }
      }
      UP(m.gh_cell, gc.data(), gc.size());
      UP(m.gh_ent, ge.data(), ge.size());
      UP(m.gh_face, X.bface.data(), X.bface.size());
      UP(m.gh_patch, gp.data(), gp.size());
      bt.assign(c->n_patches, DOLINC_BC_ZERO_GRADIENT);
      bv.assign((size_t)c->n_patches * 5, 0.0);
      UP(m.bc_type, bt.data(), bt.size());
      UP(m.bc_val, bv.data(), bv.size());
      if (e == hipSuccess) e = hipMalloc((void**)&m.gh_n, (size_t)c->n_ghost * 3 * sizeof(double));
      if (e == hipSuccess) e = hipMalloc((void**)&m.gh_dist, (size_t)c->n_ghost * sizeof(double));
    }
    {
      // sliced-ELL offsets: ELL_BLOCK cells per block, as many records per
      // cell as the block's widest cell has faces
      const int64_t nb = (P.n_cells + ELL_BLOCK - 1) / ELL_BLOCK;
      ep.assign(nb + 1, 0);
      int64_t tot = 0;
      for (int64_t b = 0; b < nb; ++b) {
        int mf = 0;
        const int64_t c1 = std::min<int64_t>(P.n_cells, (b + 1) * ELL_BLOCK);
        for (int64_t cc = b * ELL_BLOCK; cc < c1; ++cc) mf = std::max(mf, P.slot_ptr[cc + 1] - P.slot_ptr[cc]);
        tot += (int64_t)mf * ELL_BLOCK;
        ep[b + 1] = (int32_t)std::min<int64_t>(tot, INT32_MAX);
      }
      if (tot > INT32_MAX && e == hipSuccess) e = hipErrorInvalidValue;  // reported below
      c->n_ell = tot;
      UP(m.ell_ptr, ep.data(), ep.size());
      // every entry names the record of its face in the owner's and in the
      // neighbour's list (a seam face's two entries name the same records)
      er.assign(c->n_entries, make_int2(-1, -1));
      for (int64_t cc = 0; cc < P.n_cells; ++cc) {
        const int64_t b = cc / ELL_BLOCK, ln = cc % ELL_BLOCK;
        const int64_t e0 = P.part_ent_ptr[cc / P.part_cells];
        for (int32_t s = P.slot_ptr[cc]; s < P.slot_ptr[cc + 1]; ++s) {
          const int32_t r = (int32_t)(ep[b] + (int64_t)(s - P.slot_ptr[cc]) * ELL_BLOCK + ln);
          const int side = P.slots[s] >> 15;
          const int64_t eo = e0 + (P.slots[s] & 0x7fff);
          (side ? er[eo].y : er[eo].x) = r;
          const int32_t tw = P.slot_twin[s];
          if (tw >= 0) ((tw & 1) ? er[tw >> 1].y : er[tw >> 1].x) = r;
        }
      }
      for (int64_t k = 0; k < c->n_entries; ++k)
        if ((er[k].x < 0 || er[k].y < 0) && e == hipSuccess) e = hipErrorInvalidValue;  // reported below
      UP(m.ent_rec, er.data(), er.size());
      // the flux kernel reads each entry's records as 2 one-byte positions
      // (checked to give back the same records)
      if (e == hipSuccess) {
        ej.resize(c->n_entries);
        bool fits = true;
        auto pos = [&](int64_t cell, int32_t rec, unsigned char* j) {
          const int64_t b = cell / ELL_BLOCK, ln = cell % ELL_BLOCK;
          const int64_t q = (int64_t)rec - ep[b] - ln;
          if (q < 0 || q % ELL_BLOCK != 0 || q / ELL_BLOCK > 255) return false;
          *j = (unsigned char)(q / ELL_BLOCK);
          return ep[b] + (q / ELL_BLOCK) * ELL_BLOCK + ln == rec;
        };
        for (int64_t k = 0; k < c->n_entries && fits; ++k)
          fits = pos(pn[k].x, er[k].x, &ej[k].x) && pos(pn[k].y, er[k].y, &ej[k].y);
        if (fits) UP(m.ent_j, ej.data(), ej.size());
      }
    }
#undef UP
    const size_t nc = (size_t)P.n_cells;
    auto dm = [&](double** p, size_t n) {
      if (e == hipSuccess) e = hipMalloc((void**)p, n * sizeof(double));
    };
    dm(&m.V, nc);
    dm(&m.xc, 3 * nc);
    dm(&m.S, 3 * (size_t)nf);
    dm(&m.xf, 3 * (size_t)nf);
    dm(&m.fanc, 3 * (size_t)nf);
    dm(&m.omega, nf);
    dm(&m.g, nf);
    dm(&m.dvec, 3 * (size_t)nf);
    if (e == hipSuccess) e = hipMalloc((void**)&c->w.flag, sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&c->w.diag, 1024 * 8 * sizeof(double));
    // the host arrays above must outlive their copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      free_all(c);
      delete c;
      return fail(e == hipErrorOutOfMemory ? DOLINC_ENOMEM : DOLINC_EHIP,
                  std::string("device upload failed: ") + hipGetErrorString(e));
    }
  } catch (const std::bad_alloc&) {
    if (c) {
      free_all(c);
      delete c;
    }
    return fail(DOLINC_ENOMEM, "host allocation failed");
  }
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert((const void*)c);
  }
  *out = c;
  return DOLINC_OK;
}

dolinc_status dolinc_permutation(dolinc_ctx c, int32_t* new_of_old) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!new_of_old) return fail(DOLINC_EINVAL, "NULL output");
  std::memcpy(new_of_old, c->new_of_old.data(), (size_t)c->n_interior * sizeof(int32_t));
  return DOLINC_OK;
}

dolinc_status dolinc_stats(dolinc_ctx c, dolinc_mesh_stats* st) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!st) return fail(DOLINC_EINVAL, "NULL output");
  st->n_parts = c->n_parts;
  st->n_entries = c->n_entries;
  st->max_entries = c->max_entries;
  st->max_cell_faces = c->max_cell_faces;
  st->n_slots = 2 * c->n_faces;
  st->n_rows = c->n_cells;
  st->n_boundary_faces = c->n_ghost;
  return DOLINC_OK;
}

dolinc_status dolinc_set_boundary(dolinc_ctx c, int32_t patch, int32_t type, const double* values) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->precomputed) return fail(DOLINC_ESTATE, "dolinc_precompute has not been called");
  if (patch < 0 || patch >= c->n_patches) return fail(DOLINC_EINVAL, "patch out of range");
  if (type < DOLINC_BC_ZERO_GRADIENT || type > DOLINC_BC_SLIP_WALL) return fail(DOLINC_EINVAL, "unknown boundary type");
  if (type == DOLINC_BC_SLIP_WALL && c->params.pde != DOLINC_EULER)
    return fail(DOLINC_EINVAL, "a slip wall needs the Euler equations");
  double v[5] = {0, 0, 0, 0, 0};
  if (type == DOLINC_BC_DIRICHLET || type == DOLINC_BC_NEUMANN) {
    if (!values) return fail(DOLINC_EINVAL, "this boundary type needs values");
    for (int k = 0; k < c->w.nv; ++k) {
      if (!std::isfinite(values[k])) return fail(DOLINC_EINVAL, "non-finite boundary value");
      v[k] = values[k];
    }
  }
  HIPCHK(hipMemcpy(c->m.bc_type + patch, &type, sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->m.bc_val + 5 * (size_t)patch, v, sizeof(v), hipMemcpyHostToDevice));
  return DOLINC_OK;
}

dolinc_status dolinc_precompute(dolinc_ctx c, const dolinc_params* p, dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  dolinc_status st = check_params(p, c->dim);
  if (st != DOLINC_OK) return st;
  if (p->positivity && c->n_ghost)
    return fail(DOLINC_EUNSUPPORTED, "the positivity rule is built for meshes without boundary faces");
  hipStream_t s = (hipStream_t)stream;
  c->precomputed = false;
  if (!c->geometry_done) {
    HIPCHK(hipMemsetAsync(c->w.flag, 0, sizeof(int), s));
    HIPCHK(launch_geometry(c, s));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, c->w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag & 1) return fail(DOLINC_EMESH, "a cell has non-positive volume");
    if (flag & 2) return fail(DOLINC_EMESH, "a cell is not closed (sum of face area vectors != 0)");
    if (flag & 4) return fail(DOLINC_EMESH, "a face has a degenerate distance weight");
    c->geometry_done = true;
    dfree_t(c->m.nodes);
    dfree_t(c->m.fnodes);
    dfree_t(c->m.fptr);
    dfree_t(c->m.fanc);
  }
  const int nv = p->pde == DOLINC_EULER ? c->dim + 2 : 1;
  const size_t el = p->precision == DOLINC_FP64 ? sizeof(double) : sizeof(float);
  const int ord = scheme_order(p->scheme);
  const bool bl = p->blend != DOLINC_BLEND_NONE;
  {
    // the flux kernel accumulates a partition's face fluxes in LDS
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
      lim = 64 * 1024;
    const size_t per = p->use_u_ref == 2 ? 2 : 1;  // shares per entry
    if ((size_t)c->max_entries * nv * el * per > (size_t)lim)
      return fail(DOLINC_EUNSUPPORTED, "partition face fluxes exceed the LDS of one workgroup (" +
                                           std::to_string(lim / 1024) + " KiB); use a smaller part_cells");
  }
  if (c->w.precision != p->precision || c->w.scheme != p->scheme || c->w.nv != nv || c->w.blend != p->blend ||
      (c->w.estate != nullptr) != (p->positivity != 0)) {
    if (c->s_net) HIPCHK(hipStreamSynchronize(c->s_net));  // the network may still read the old buffers
    free_work(c);
    const size_t nc = (size_t)c->n_cells, ne = (size_t)c->n_entries;
    hipError_t e = hipSuccess;
    auto al = [&](void** q, size_t bytes) {
      if (e == hipSuccess) e = hipMalloc(q, bytes ? bytes : 16);
    };
    al(&c->w.sw, ne * 4 * el);
    al(&c->w.ell_sw, (size_t)c->n_ell * 4 * el);
    al(&c->w.ell_d, (size_t)c->n_ell * 3 * el);
    al(&c->w.dc, ne * (size_t)DC_VALUES * el);
    al(&c->w.rV, nc * el);
    if (ord >= 1 || bl) al(&c->w.G1, nc * nv * c->dim * el);
    if (ord >= 2) al(&c->w.Hf, (size_t)c->n_ell * nv * el);
    al(&c->w.W1, nc * nv * el);
    al(&c->w.W2, nc * nv * el);
    if (bl) al((void**)&c->w.theta, nc * sizeof(float));
    if (p->blend == DOLINC_BLEND_LEARNED && c->dim == 3) al((void**)&c->w.Xf, nc * DOLINC_N_FEATURES * sizeof(unsigned short));
    if (p->positivity) {
      al(&c->w.estate, ne * 2 * nv * el);
      al(&c->w.thpos, nc * el);
    }
    if (e != hipSuccess) {
      free_work(c);
      return fail(DOLINC_ENOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
    }
    c->w.precision = p->precision;
    c->w.scheme = p->scheme;
    c->w.nv = nv;
    c->w.blend = p->blend;
    c->w.elem = el;
  }
  if (p->blend == DOLINC_BLEND_LEARNED && c->dim == 3 && !c->s_net) {
    // the network's stream and the two events that fork it from, and join
    // it back to, the caller's stream in every stage
    hipError_t e = hipStreamCreateWithFlags(&c->s_net, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(DOLINC_EHIP, std::string("stream set-up failed: ") + hipGetErrorString(e));
  }
  c->params = *p;
  HIPCHK(launch_entry_fill(c, s));
  if (bl) HIPCHK(hipMemsetAsync(c->w.theta, 0, (size_t)c->n_cells * sizeof(float), s));
  HIPCHK(hipStreamSynchronize(s));
  c->precomputed = true;
  return DOLINC_OK;
}

dolinc_status dolinc_residual(dolinc_ctx c, const void* U, void* R, dolinc_stream stream) {
  dolinc_status st = need_ready(c);
  if (st != DOLINC_OK) return st;
  if (!U || !R) return fail(DOLINC_EINVAL, "NULL state");
  if (U == R) return fail(DOLINC_EINVAL, "U and R must differ");
  HIPCHK(ghost_input(c, U, (hipStream_t)stream));
  HIPCHK(stage(c, U, nullptr, R, 0, 0.0, 0.0, 0.0, (hipStream_t)stream));
  return DOLINC_OK;
}

static dolinc_status rk_step_impl(dolinc_ctx c, void* U, double dt, hipStream_t s) {
  // SSP-RK3 (third-order TVD Runge-Kutta, Sec. 3); stage outputs in W1, W2,
  // the last stage overwrites U cell by cell after reading it
  // (auxiliary rows of each stage input rewritten from the boundary conditions)
  HIPCHK(launch_ghost(c, GHOST_U, U, s));
  HIPCHK(stage(c, U, U, c->w.W1, 1, 0.0, 1.0, dt, s));
  HIPCHK(launch_ghost(c, GHOST_U, c->w.W1, s));
  HIPCHK(stage(c, c->w.W1, U, c->w.W2, 1, 0.75, 0.25, dt, s));
  HIPCHK(launch_ghost(c, GHOST_U, c->w.W2, s));
  HIPCHK(stage(c, c->w.W2, U, U, 1, 1.0 / 3.0, 2.0 / 3.0, dt, s));
  return DOLINC_OK;
}

dolinc_status dolinc_rk_step(dolinc_ctx c, void* U, double dt, dolinc_stream stream) {
  dolinc_status st = need_ready(c);
  if (st != DOLINC_OK) return st;
  if (!U) return fail(DOLINC_EINVAL, "NULL state");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(DOLINC_EINVAL, "dt must be finite and > 0");
  return rk_step_impl(c, U, dt, (hipStream_t)stream);
}

dolinc_status dolinc_advance(dolinc_ctx c, void* U, double dt, int64_t n, dolinc_stream stream) {
  dolinc_status st = need_ready(c);
  if (st != DOLINC_OK) return st;
  if (!U) return fail(DOLINC_EINVAL, "NULL state");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(DOLINC_EINVAL, "dt must be finite and > 0");
  if (n < 0) return fail(DOLINC_EINVAL, "n_steps must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    st = rk_step_impl(c, U, dt, (hipStream_t)stream);
    if (st != DOLINC_OK) return st;
  }
  return DOLINC_OK;
}

dolinc_status dolinc_set_theta(dolinc_ctx c, const float* theta, dolinc_stream stream) {
  dolinc_status st = need_ready(c);
  if (st != DOLINC_OK) return st;
  if (c->params.blend != DOLINC_BLEND_THETA) return fail(DOLINC_ESTATE, "blend mode is not THETA");
  if (!theta) return fail(DOLINC_EINVAL, "NULL theta");
  HIPCHK(hipMemcpyAsync(c->w.theta, theta, (size_t)c->n_cells * sizeof(float), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  HIPCHK(launch_ghost(c, GHOST_THETA, c->w.theta, (hipStream_t)stream));
  return DOLINC_OK;
}

dolinc_status dolinc_classical_theta(dolinc_ctx c, const void* U, float* theta, dolinc_stream stream) {
  dolinc_status st = need_ready(c, false);
  if (st != DOLINC_OK) return st;
  if (!U || !theta) return fail(DOLINC_EINVAL, "NULL argument");
  if (!c->w.G1) return fail(DOLINC_ESTATE, "no gradient workspace (scheme of order 0 without blend)");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ghost_input(c, U, s));
  HIPCHK(grad_dispatch(c, U, c->w.G1, nullptr, s));
  HIPCHK(c->w.precision == DOLINC_FP64 ? theta_f64(c, U, c->w.G1, theta, s) : theta_f32(c, U, c->w.G1, theta, s));
  HIPCHK(launch_ghost(c, GHOST_THETA, theta, s));
  return DOLINC_OK;
}

dolinc_status dolinc_gradients(dolinc_ctx c, const void* U, void* G1, void* G2, dolinc_stream stream) {
  dolinc_status st = need_ready(c, false);
  if (st != DOLINC_OK) return st;
  if (!U || !G1) return fail(DOLINC_EINVAL, "NULL argument");
  HIPCHK(ghost_input(c, U, (hipStream_t)stream));
  HIPCHK(grad_dispatch(c, U, G1, G2, (hipStream_t)stream));
  return DOLINC_OK;
}

dolinc_status dolinc_face_states(dolinc_ctx c, const void* U, void* UL, void* UR, void* F, dolinc_stream stream) {
  dolinc_status st = need_ready(c);
  if (st != DOLINC_OK) return st;
  if (!U || !UL || !UR) return fail(DOLINC_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ghost_input(c, U, s));
  HIPCHK(prepare_stage(c, U, s));
  HIPCHK(c->w.precision == DOLINC_FP64 ? export_f64(c, U, UL, UR, F, s) : export_f32(c, U, UL, UR, F, s));
  return DOLINC_OK;
}

dolinc_status dolinc_geometry(dolinc_ctx c, double* V, double* xc, double* S, double* xf, double* omega, double* g,
                              dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->geometry_done) return fail(DOLINC_ESTATE, "dolinc_precompute has not been called");
  hipStream_t s = (hipStream_t)stream;
  const size_t nc = (size_t)c->n_cells, nf = (size_t)c->n_faces;
  const int d = c->dim;
  if (V) HIPCHK(hipMemcpyAsync(V, c->m.V, nc * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (xc) HIPCHK(hipMemcpy2DAsync(xc, d * sizeof(double), c->m.xc, 3 * sizeof(double), d * sizeof(double), nc,
                                  hipMemcpyDeviceToDevice, s));
  if (S) HIPCHK(hipMemcpy2DAsync(S, d * sizeof(double), c->m.S, 3 * sizeof(double), d * sizeof(double), nf,
                                 hipMemcpyDeviceToDevice, s));
  if (xf) HIPCHK(hipMemcpy2DAsync(xf, d * sizeof(double), c->m.xf, 3 * sizeof(double), d * sizeof(double), nf,
                                  hipMemcpyDeviceToDevice, s));
  if (omega) HIPCHK(hipMemcpyAsync(omega, c->m.omega, nf * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (g) HIPCHK(hipMemcpyAsync(g, c->m.g, nf * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DOLINC_OK;
}

dolinc_status dolinc_diagnostics(dolinc_ctx c, const void* U, double* out, dolinc_stream stream) {
  dolinc_status st = need_ready(c, false);
  if (st != DOLINC_OK) return st;
  if (!U || !out) return fail(DOLINC_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  int nb = (int)((c->n_interior + KTPB_HOST - 1) / KTPB_HOST);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  HIPCHK(c->w.precision == DOLINC_FP64 ? diag_f64(c, U, c->w.diag, nb, out, s)
                                       : diag_f32(c, U, c->w.diag, nb, out, s));
  return DOLINC_OK;
}

dolinc_status dolinc_features(dolinc_ctx c, const void* U, float* X32, uint16_t* Xbf, dolinc_stream stream) {
  dolinc_status st = need_ready(c, false);
  if (st != DOLINC_OK) return st;
  if (!U) return fail(DOLINC_EINVAL, "NULL state");
  if (c->params.pde != DOLINC_EULER) return fail(DOLINC_EUNSUPPORTED, "features are built for the Euler equations");
  if (!c->w.G1) return fail(DOLINC_ESTATE, "no gradient workspace (scheme of order 0 without blend)");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ghost_input(c, U, s));
  HIPCHK(grad_dispatch(c, U, c->w.G1, nullptr, s));
  HIPCHK(features_launch(c, U, X32, (unsigned short*)Xbf, s));
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_set(dolinc_ctx c, const float* params, dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!params) return fail(DOLINC_EINVAL, "NULL parameters");
  Mlp& m = c->mlp;
  if (!m.p) {
    hipError_t e = hipMalloc((void**)&m.p, MLP_N * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&m.m, MLP_N * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&m.v, MLP_N * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&m.w1b, 64 * 32 * sizeof(unsigned short));
    if (e == hipSuccess) e = hipMalloc((void**)&m.w2b, 64 * 64 * sizeof(unsigned short));
    if (e != hipSuccess) {
      free_mlp(c);
      return fail(DOLINC_ENOMEM, "network allocation failed");
    }
  }
  // copy, Adam moments cleared, bf16 copies refreshed: kernels on the
  // caller's stream (a stage's network work is joined back into the stream
  // it was called on, so it is ordered before this)
  HIPCHK(mlp_set_launch(c, params, (hipStream_t)stream));
  m.step = 0;
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_get(dolinc_ctx c, float* params, dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->mlp.p) return fail(DOLINC_ESTATE, "dolinc_mlp_set has not been called");
  if (!params) return fail(DOLINC_EINVAL, "NULL output");
  HIPCHK(hipMemcpyAsync(params, c->mlp.p, MLP_N * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_forward(dolinc_ctx c, const uint16_t* X, int64_t n, float* theta, dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->mlp.p) return fail(DOLINC_ESTATE, "dolinc_mlp_set has not been called");
  if (!X || !theta) return fail(DOLINC_EINVAL, "NULL argument");
  if (n < 0) return fail(DOLINC_EINVAL, "n must be >= 0");
  if (reinterpret_cast<uintptr_t>(X) % 16 != 0) return fail(DOLINC_EINVAL, "X must be 16-byte aligned");
  if (n == 0) return DOLINC_OK;
  HIPCHK(mlp_forward_launch(c, (const unsigned short*)X, n, theta, (hipStream_t)stream, DOLINC_FEATURE_STRIDE));
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_train_step(dolinc_ctx c, const uint16_t* X, const float* y, int64_t n, float lr,
                                    float* loss, dolinc_stream stream) {
  dolinc_status st = mlp_batch_check(c, X, y, n);
  if (st != DOLINC_OK) return st;
  if (!(std::isfinite(lr) && lr > 0.f)) return fail(DOLINC_EINVAL, "lr must be finite and > 0");
  int nb = 0, rows = 0;
  mlp_grid(n, &nb, &rows);
  const int64_t t = c->mlp.step + 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)t));
  HIPCHK(mlp_grad_launch(c, (const unsigned short*)X, y, n, nb, rows, nullptr, loss, 1, lr, c1, c2,
                         (hipStream_t)stream));
  c->mlp.step = t;
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_train_step_static(dolinc_ctx c, const uint16_t* X, const float* y, int64_t n, float lr,
                                           float* loss, dolinc_stream stream) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  if (!c->mlp.p) return fail(DOLINC_ESTATE, "dolinc_mlp_set has not been called");
  if (!X || !y) return fail(DOLINC_EINVAL, "NULL batch");
  if (n <= 0 || n > DOLINC_MLP_STATIC_MAX_ROWS)
    return fail(DOLINC_EINVAL, "batch size must be in [1, " + std::to_string(DOLINC_MLP_STATIC_MAX_ROWS) +
                                   "] for the training step without allocation");
  if (!(std::isfinite(lr) && lr > 0.f)) return fail(DOLINC_EINVAL, "lr must be finite and > 0");
  int nb = 0, rows = 0;
  mlp_grid(n, &nb, &rows);  // the grid of dolinc_mlp_train_step: the same partials, the same step
  if (nb > MLP_STATIC_BLOCKS) return fail(DOLINC_EINVAL, "internal: batch needs more partials than the scratch holds");
  const int64_t t = c->mlp.step + 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)t));
  HIPCHK(mlp_train_static_launch(c, (const unsigned short*)X, y, n, nb, rows, loss, lr, c1, c2, (hipStream_t)stream));
  c->mlp.step = t;
  return DOLINC_OK;
}

dolinc_status dolinc_mlp_gradient(dolinc_ctx c, const uint16_t* X, const float* y, int64_t n, float* grad,
                                  float* loss, dolinc_stream stream) {
  dolinc_status st = mlp_batch_check(c, X, y, n);
  if (st != DOLINC_OK) return st;
  if (!grad) return fail(DOLINC_EINVAL, "NULL gradient output");
  int nb = 0, rows = 0;
  mlp_grid(n, &nb, &rows);
  HIPCHK(mlp_grad_launch(c, (const unsigned short*)X, y, n, nb, rows, grad, loss, 0, 0.f, 1.f, 1.f,
                         (hipStream_t)stream));
  return DOLINC_OK;
}

dolinc_status dolinc_timing(dolinc_ctx c, int32_t enable, double* ms, int64_t* count) {
  if (!valid_ctx(c)) return fail(DOLINC_ESTATE, "invalid or destroyed context");
  double acc[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
  if (ms || count) {
    for (size_t k = 0; k < c->ev_kind.size(); ++k) {
      HIPCHK(hipEventSynchronize(c->ev_pool[2 * k + 1]));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
      acc[c->ev_kind[k]] += t;
      n[c->ev_kind[k]] += 1;
    }
    for (int k = 0; k < 4; ++k) {
      if (ms) ms[k] = acc[k];
      if (count) count[k] = n[k];
    }
  }
  if (enable) {
    c->ev_used = 0;
    c->ev_kind.clear();
  }
  c->timing = enable != 0;
  return DOLINC_OK;
}

void dolinc_destroy(dolinc_ctx c) {
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!c || !g_live.erase((const void*)c)) return;
  }
  if (c->s_net) (void)hipStreamSynchronize(c->s_net);
  free_all(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->s_net) (void)hipStreamDestroy(c->s_net);
  delete c;
}

}  // extern "C"
