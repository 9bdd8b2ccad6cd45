/*
 * dolinc.h -- C ABI of the MI355X (gfx950) DOLINC explicit-residual library.
 *
 * The library evaluates the semi-discrete finite-volume residual of a
 * hyperbolic conservation law on a face-addressed unstructured mesh with the
 * DOLINC high-order reconstruction of arXiv 2404.08952, and advances cell
 * averages with the third-order TVD (SSP) Runge-Kutta method (Sec. 3).
 *
 * Every compute step runs in HIP kernels on the device.  Plain pointers and
 * sizes only; no C++ types cross this boundary and no function throws.
 *
 * Conventions
 *   - "host" pointers are read during the call only; "device" pointers must
 *     stay valid until the work enqueued on the given stream has finished.
 *   - Cell arrays on the device use the library's INTERNAL cell order (the
 *     mesh is renumbered for locality at creation); dolinc_permutation()
 *     returns the map.  Face arrays exported by the library use the caller's
 *     face order.
 *   - Layout of a state U is [n_rows][n_v] (row-major), n_v = 1 for
 *     advection / Burgers and dim + 2 for Euler (rho, rho*u.., rho*E).
 *     n_rows = n_cells + the number of boundary faces: rows n_cells .. hold
 *     the auxiliary cells of the non-coupled boundary faces (Sec. 2.6); the
 *     library rewrites them from the boundary conditions at every stage, so
 *     their content on input does not matter.  Without boundary faces
 *     n_rows = n_cells.  Per-cell arrays (gradients, theta, features)
 *     likewise have n_rows rows.
 *   - The element type of U, R and the exported gradients is double for
 *     DOLINC_FP64 and float for DOLINC_FP32_MIXED.
 *   - Return values: DOLINC_OK or an error code; dolinc_last_error() gives a
 *     thread-local message.  Arguments are validated before anything is
 *     enqueued; on error nothing is enqueued.
 *   - One context may be used by one host thread / one stream at a time.
 *     Calls on one context that overlap on different streams race.
 *   - With DOLINC_BLEND_LEARNED in 3-D, each stage of dolinc_residual /
 *     dolinc_rk_step / dolinc_advance runs the network on a second stream
 *     that the context owns (created by dolinc_precompute, default
 *     priority), forked from the given stream by an event after the
 *     features and joined back before the flux: all of a call's work is
 *     still ordered on the given stream, so synchronising or recording an
 *     event on it covers the network too.
 */
#ifndef DOLINC_H
#define DOLINC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dolinc_ctx_s* dolinc_ctx;
typedef void* dolinc_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
  DOLINC_OK = 0,
  DOLINC_EINVAL = 1,       /* bad argument                                   */
  DOLINC_EMESH = 2,        /* malformed mesh (unpaired face, V <= 0, ...)    */
  DOLINC_ENOMEM = 3,       /* device or host allocation failed               */
  DOLINC_EHIP = 4,         /* a HIP runtime call failed (no device, ...)     */
  DOLINC_ESTATE = 5,       /* call out of order (e.g. residual before precompute) */
  DOLINC_EUNSUPPORTED = 6  /* valid but not built combination                */
} dolinc_status;

typedef enum { DOLINC_ADVECTION = 0, DOLINC_BURGERS = 1, DOLINC_EULER = 2 } dolinc_pde;

/* k-th order reconstructions of Sec. 2.4 (k cells, r of them upwind of the
 * face): FOU k=1, CD2 k=2, USR3 k=3 r=1, CSR4 k=4 r=1 (first-order DOLINC
 * schemes, inversion eq:lCoeffDLC1 / eq:rCoeffDLC1), USR5 k=5 r=2 (second
 * order DOLINC scheme, inversion eq:lCoeffDLC2), CSR6 k=6 r=2 (the central
 * second-order DOLINC scheme named in Sec. 2.4; one state per face, both
 * cells' second differentials, eq:lCoeffDLC2 / eq:rCoeffDLC2).
 * ENO3 and WENO5 (end of Sec. 2.4; second-order DOLINC schemes): cells -2..2
 * of the face's template are retrieved as for USR5; ENO3 takes the 3-cell
 * stencil that Harten's rule picks with the DOLINC undivided differences
 * printed there (the upwind candidate wins when smaller by a relative 1e-10
 * in FP64, 1e-5 in FP32, else the downwind one); WENO5 weights the
 * three 3-cell stencils with Jiang-Shu smoothness indicators (epsilon 1e-6)
 * and the linear weights that reproduce the 5-cell coefficients of eq:coeff
 * on the graded template.  Applied per conserved variable. */
typedef enum {
  DOLINC_FOU = 1, DOLINC_CD2 = 2, DOLINC_USR3 = 3, DOLINC_CSR4 = 4, DOLINC_USR5 = 5,
  DOLINC_ENO3 = 6, DOLINC_WENO5 = 7, DOLINC_CSR6 = 8
} dolinc_scheme;

/* UPWIND: advection upwind flux (Sec. 3.2) and the Godunov flux of Burgers
 * (Sec. 3.3); RUSANOV: local Lax-Friedrichs (Sec. 3.4); HLLC (Toro). */
typedef enum { DOLINC_FLUX_UPWIND = 0, DOLINC_FLUX_RUSANOV = 1, DOLINC_FLUX_HLLC = 2 } dolinc_flux;

/* FP64: all arithmetic in double.  FP32_MIXED: geometry computed in double
 * and stored rounded to float; the inversion / reconstruction coefficients
 * evaluated in double from each face's stored weight omega in the flux
 * kernel and rounded once to float; gradient, reconstruction, flux and
 * update in float with compensated (Neumaier) face-to-cell sums.  ENO3 /
 * WENO5 form their growth rates from omega in double. */
typedef enum { DOLINC_FP64 = 0, DOLINC_FP32_MIXED = 1 } dolinc_precision;

/* Blend of the high-order face state with a Van Leer limited second-order
 * state: U = theta_f U_high + (1 - theta_f) U_limited, theta_f = min of the
 * two cells' theta.  THETA takes theta per cell from dolinc_set_theta();
 * CLASSICAL computes it every stage from the DOLINC divided-difference
 * sensor (Sec. 2.4, ENO3 indicators); LEARNED computes it every stage with
 * the indicator network set by dolinc_mlp_set(). */
typedef enum {
  DOLINC_BLEND_NONE = 0, DOLINC_BLEND_THETA = 1, DOLINC_BLEND_CLASSICAL = 2, DOLINC_BLEND_LEARNED = 3
} dolinc_blend;

/* Learned indicator: 24 features per cell -> 64 -> 64 -> 1 (tanh, tanh,
 * sigmoid).  Parameters packed as W1[64][24], b1[64], W2[64][64], b2[64],
 * W3[64], b3 (fp32 master copy; the matrix cores use bf16 copies). */
#define DOLINC_MLP_PARAMS 5825
#define DOLINC_N_FEATURES 24
#define DOLINC_FEATURE_STRIDE 32 /* bf16 feature rows are padded to 32 */

typedef struct {
  int32_t dim;                   /* 2 or 3                                          */
  int64_t n_nodes, n_cells, n_faces;
  const double* node_xyz;        /* host [n_nodes][dim]                              */
  const int64_t* face_node_ptr;  /* host [n_faces + 1], CSR into face_nodes          */
  const int32_t* face_nodes;     /* host; owner frame; right-hand normal owner->neigh */
  const int32_t* owner;          /* host [n_faces]                                   */
  const int32_t* neighbour;      /* host [n_faces]; every face has two cells         */
  const double* neigh_shift;     /* host [n_faces][dim]: moves the neighbour's       */
                                 /* geometry into the owner's frame (periodic)       */
  int32_t renumber;              /* 0 keep, 1 reverse Cuthill-McKee, 2 Hilbert curve */
  int32_t part_cells;            /* cells per partition (0 = default 256; <= 1024);  */
                                 /* dolinc_precompute returns EUNSUPPORTED when a    */
                                 /* partition's face fluxes exceed the LDS of one    */
                                 /* workgroup on the device (160 KB on gfx950)       */
  /* Non-coupled boundaries (Sec. 2.6).  NULL: every face has two cells.
   * Otherwise host [n_faces]: -1 for a two-cell face; for a boundary face
   * (neighbour[f] == -1, owner[f] the cell, normal pointing out of the
   * domain, neigh_shift ignored) its boundary patch in [0, n_patches). */
  const int32_t* face_patch;
  int32_t n_patches;
} dolinc_mesh_desc;

/* Boundary conditions of a patch (Sec. 2.6): the auxiliary cell behind each
 * boundary face takes T_O = T_C + 2 (T_f - T_C) with T_f the boundary-face
 * value: DIRICHLET values[v] = T_f; NEUMANN values[v] = q, the outward normal
 * gradient, T_f = T_C + q d_fC (d_fC: normal distance from the cell centre to
 * the face; the auxiliary cell is the cell's mirror image in the face plane);
 * ZERO_GRADIENT T_f = T_C (transmissive); SLIP_WALL (Euler) density and
 * energy copied, momentum reflected in the face plane.  The auxiliary cell's
 * DOLINC differentials are those of the field continued by the same rule. */
typedef enum {
  DOLINC_BC_ZERO_GRADIENT = 0, DOLINC_BC_DIRICHLET = 1, DOLINC_BC_NEUMANN = 2, DOLINC_BC_SLIP_WALL = 3
} dolinc_bc;

typedef struct {
  int32_t pde;                   /* dolinc_pde        */
  int32_t scheme;                /* dolinc_scheme     */
  int32_t flux;                  /* dolinc_flux       */
  int32_t precision;             /* dolinc_precision  */
  int32_t blend;                 /* dolinc_blend      */
  int32_t use_u_ref;             /* the state the face arithmetic is carried about.   */
                                 /* 0: full states.  1 (Euler): a constant reference  */
                                 /* u_ref: reconstruct U - u_ref, flux F(U).S -       */
                                 /* F(u_ref).S in difference form.  2 (every law):    */
                                 /* each face side's own cell: increments over the    */
                                 /* cell value, each cell summing F.S - F(U_c).S over */
                                 /* its faces (u_ref ignored; the FP32 form of        */
                                 /* choice: its rounding enters only through          */
                                 /* F - F(U_c)).  In 1 and 2 the dropped F(.).S terms */
                                 /* cancel over closed cells (FP64 geometry); same    */
                                 /* results as 0 to rounding.  2 keeps two flux       */
                                 /* shares per face entry in LDS                      */
  double gamma;                  /* Euler ratio of specific heats                     */
  double adv_vel[3];             /* advection velocity                                */
  double burgers_dir[3];         /* Burgers flux u^2/2 * burgers_dir                   */
  double u_ref[5];               /* reference state for the FP32 perturbation flux     */
  int32_t positivity;            /* Euler, meshes without boundary faces, use_u_ref 0  */
                                 /* or 2: 1 scales every cell's face-side states      */
                                 /* toward the cell value, U_c + theta_c (U_c,f -     */
                                 /* U_c), with the largest theta_c in [0, 1] for      */
                                 /* which U* = U_c - theta_c sum_f a_f (U_c,f - U_c)  */
                                 /* (a_f = |S_f| / sum |S|) keeps rho and p >= 1e-6   */
                                 /* of the cell's: the update of a cell is then a     */
                                 /* convex combination of first-order Lax-Friedrichs  */
                                 /* updates, admissible for dt lambda sum|S|/V <= 1/2 */
                                 /* (Zhang-Shu style; not in the paper, for shock     */
                                 /* workloads).  A first pass per stage writes the    */
                                 /* increments and theta_c; 0 leaves the states as    */
                                 /* they are.                                         */
} dolinc_params;

typedef struct {                 /* host-side partition statistics                    */
  int64_t n_parts, n_entries, max_entries, max_cell_faces, n_slots;
  int64_t n_rows;                /* rows of device cell arrays (cells + boundary faces) */
  int64_t n_boundary_faces;
} dolinc_mesh_stats;

/* Validate the mesh, renumber cells, build partitions and face entries and
 * upload them (hipMalloc, then copies enqueued on stream s; synchronises s
 * before returning, so the host arrays may be released afterwards).  Defines
 * the problem of Sec. 2.1-2.2: cell averages on a face-addressed mesh, every
 * face shared by two cells (periodic faces carrying a translation, Sec. 2.6)
 * or, with face_patch, a boundary face of one cell on a boundary patch
 * (Sec. 2.6; an auxiliary cell is appended for it, see dolinc_set_boundary).
 * EMESH for unpaired / self faces, out-of-range indices, boundary faces
 * without a valid patch or non-closed cells. */
dolinc_status dolinc_create(const dolinc_mesh_desc* mesh, dolinc_stream s, dolinc_ctx* out);

/* The host part of dolinc_create only (validation, renumbering, partitions);
 * touches no device.  new_of_old (host [n_cells]) and stats may be NULL. */
dolinc_status dolinc_mesh_prepare(const dolinc_mesh_desc* mesh, int32_t* new_of_old,
                                  dolinc_mesh_stats* stats);

/* new_of_old: host [n_cells], filled with the internal index of each caller
 * cell (the auxiliary cell of the k-th boundary face, in caller face order,
 * is row n_cells + k).  ESTATE for an invalid context, EINVAL for NULL. */
dolinc_status dolinc_permutation(dolinc_ctx ctx, int32_t* new_of_old);
/* Partition statistics of the context into host *stats.  ESTATE for an
 * invalid context, EINVAL for NULL. */
dolinc_status dolinc_stats(dolinc_ctx ctx, dolinc_mesh_stats* stats);

/* Condition of boundary patch `patch` (dolinc_bc); values: host double
 * [n_v] for DIRICHLET / NEUMANN (ignored, may be NULL, otherwise).  Every
 * patch starts as ZERO_GRADIENT.  Takes effect for the following calls;
 * needs dolinc_precompute first (n_v comes from the params).  EINVAL for a
 * patch out of range, an unknown type, missing or non-finite values, or
 * SLIP_WALL outside the Euler equations. */
dolinc_status dolinc_set_boundary(dolinc_ctx ctx, int32_t patch, int32_t type, const double* values);

/* FP64 precompute on the device (Sec. 2.2 growth rate g and weight omega,
 * centre distance d, face area vectors, volumes; the flux kernel evaluates
 * the Sec. 2.3-2.4 inversion and reconstruction coefficients, folded into
 * the DOLINC representation eq:USR3 / eq:CSR4, from omega in double), then
 * allocates the gradient and Runge-Kutta workspaces.  Synchronises before
 * returning.  May be called again to change params (re-allocates as
 * needed). */
dolinc_status dolinc_precompute(dolinc_ctx ctx, const dolinc_params* params, dolinc_stream s);

/* The semi-discrete residual R = dU/dt = -V^-1 sum_f sigma F_f of the
 * finite-volume form for cell averages (Sec. 2.2), with face states
 * from the DOLINC reconstruction (Sec. 2.3-2.4, eq:USR3 / eq:CSR4 and the
 * second-order templates), the optional blend and the Riemann flux of the
 * params (Sec. 3).  U, R: device [n_rows][n_v], element type of the
 * precision, internal order, owned by the caller; U != R.  The auxiliary
 * rows of U are rewritten from the boundary conditions.  ESTATE before
 * dolinc_precompute (or with the learned blend before dolinc_mlp_set),
 * EINVAL for NULL or U == R, EHIP if a launch fails. */
dolinc_status dolinc_residual(dolinc_ctx ctx, const void* U, void* R, dolinc_stream s);

/* One step of the third-order TVD (SSP) Runge-Kutta method (Sec. 3,
 * opening paragraph) in place on U (device [n_rows][n_v], caller-owned)
 * with time step dt: three residual stages fused with their stage
 * combinations, the intermediate states in the context's workspaces.
 * ESTATE as for dolinc_residual, EINVAL for NULL U or dt not finite and
 * > 0, EHIP if a launch fails. */
dolinc_status dolinc_rk_step(dolinc_ctx ctx, void* U, double dt, dolinc_stream s);

/* n_steps SSP-RK3 steps (same as calling dolinc_rk_step n_steps times);
 * EINVAL also for n_steps < 0. */
dolinc_status dolinc_advance(dolinc_ctx ctx, void* U, double dt, int64_t n_steps, dolinc_stream s);

/* Per-cell blend weights for DOLINC_BLEND_THETA: device float [n_cells]
 * (internal order, caller-owned), copied into the context on stream s.
 * ESTATE unless the params' blend is THETA, EINVAL for NULL. */
dolinc_status dolinc_set_theta(dolinc_ctx ctx, const float* theta, dolinc_stream s);

/* Classical sensor weight theta per cell for state U: the smoothness ratio
 * of the DOLINC upwind differences (Sec. 2.4, the undivided differences of
 * ENO3) on density and energy, mapped to [0, 1].  U device [n_rows][n_v],
 * theta device float [n_rows] (caller-owned).  ESTATE before precompute or
 * when the scheme keeps no gradient (order 0 without blend), EINVAL for
 * NULL. */
dolinc_status dolinc_classical_theta(dolinc_ctx ctx, const void* U, float* theta, dolinc_stream s);

/* Gauss-linear gradient (Sec. 2.3) of U: G1 device [n_rows][n_v][dim];
 * G2 (may be NULL) the symmetrised gradient of G1, [n_rows][n_v][dim*(dim+1)/2]
 * ordered xx,yy,(zz),xy,(xz,yz).  Element type as U; caller-owned.
 * ESTATE before precompute, EINVAL for NULL U or G1. */
dolinc_status dolinc_gradients(dolinc_ctx ctx, const void* U, void* G1, void* G2, dolinc_stream s);

/* Reconstructed face states (Sec. 2.4, both sides of every face, after the
 * blend and the positivity rules) per face in the caller's face order: UL,
 * UR device [n_faces][n_v]; F (may be NULL) the face-integrated numerical
 * flux [n_faces][n_v] (Sec. 3).  Caller-owned.  ESTATE as for
 * dolinc_residual, EINVAL for NULL U, UL or UR. */
dolinc_status dolinc_face_states(dolinc_ctx ctx, const void* U, void* UL, void* UR, void* F,
                                 dolinc_stream s);

/* FP64 geometry after precompute (Sec. 2.2: volumes, centroids, face area
 * vectors and centres, the distance weight omega and growth rate g of
 * every face): V, xc device double [n_cells], [n_cells][dim] (internal
 * order); S, xf [n_faces][dim], omega, g [n_faces] (caller order).  Any
 * pointer may be NULL.  ESTATE before dolinc_precompute. */
dolinc_status dolinc_geometry(dolinc_ctx ctx, double* V, double* xc, double* S, double* xf,
                              double* omega, double* g, dolinc_stream s);

/* Diagnostics of U into device double out[n_v + 3]: conserved totals
 * sum_c V_c U_c (FP64 sums; the conservation statement of the coupled
 * finite-volume update, Sec. 2.2 and 2.6) for every variable, then min rho
 * (or min u), min p (Euler; else max u) and the count of non-finite entries.
 * Two kernels enqueued on s (per-block partials, then one ordered
 * reduction); does not block.  Calls on one context share the partials'
 * workspace, so two diagnostics calls in flight on different streams race. */
dolinc_status dolinc_diagnostics(dolinc_ctx ctx, const void* U, double* out, dolinc_stream s);

/* Features of state U (Euler): X32 device float [n_cells][24] and/or Xbf
 * device bf16 (uint16) [n_cells][32] (columns 24..31 zero); either may be
 * NULL.  Internal cell order. */
dolinc_status dolinc_features(dolinc_ctx ctx, const void* U, float* X32, uint16_t* Xbf, dolinc_stream s);

/* Set or read back the network parameters: params device
 * float[DOLINC_MLP_PARAMS] (the packing above), copied on stream s; neither
 * call blocks.  Setting resets the Adam moments and step count and refreshes
 * the bf16 copies the matrix cores read; the values are taken as given (no
 * finiteness check on the device).  The first set allocates the network's
 * device memory (ENOMEM if that fails). */
dolinc_status dolinc_mlp_set(dolinc_ctx ctx, const float* params, dolinc_stream s);
dolinc_status dolinc_mlp_get(dolinc_ctx ctx, float* params, dolinc_stream s);

/* theta = network(X) for n rows of bf16 features X (device [n][32], 16-byte
 * aligned: each lane reads 8 features at once; the 8 padding columns are not
 * read); theta device float [n].  EINVAL for a NULL or misaligned X. */
dolinc_status dolinc_mlp_forward(dolinc_ctx ctx, const uint16_t* X, int64_t n, float* theta, dolinc_stream s);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean binary
 * cross entropy of the batch (X device bf16 [n][32], y device float [n]
 * soft labels in [0, 1]).  loss (device float, may be NULL) receives the
 * batch loss before the step. */
dolinc_status dolinc_mlp_train_step(dolinc_ctx ctx, const uint16_t* X, const float* y, int64_t n, float lr,
                                    float* loss, dolinc_stream s);

/* The same training step for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the per-block partial gradients go to a fixed device array of
 * the library (about 6 MB per device, held until the process ends, its
 * device address looked up once per device) instead of the context's
 * workspace, which dolinc_mlp_train_step grows with the batch.  Allocates
 * nothing; needs dolinc_mlp_set first (ESTATE).  n in [1,
 * DOLINC_MLP_STATIC_MAX_ROWS], else EINVAL.  For the same inputs its result
 * equals dolinc_mlp_train_step's bit for bit (same partial grid).  Every
 * call on one device shares that array: two calls in flight on one device
 * (any contexts, any streams) race. */
#define DOLINC_MLP_STATIC_MAX_ROWS 65536
dolinc_status dolinc_mlp_train_step_static(dolinc_ctx ctx, const uint16_t* X, const float* y, int64_t n, float lr,
                                           float* loss, dolinc_stream s);

/* Gradient of the same loss without a step: grad device float[DOLINC_MLP_PARAMS]. */
dolinc_status dolinc_mlp_gradient(dolinc_ctx ctx, const uint16_t* X, const float* y, int64_t n, float* grad,
                                  float* loss, dolinc_stream s);

/* Kernel timing with HIP events recorded around every launch on the stream
 * the kernel runs on.  enable = 1 clears the accumulators and starts
 * recording, 0 stops.  ms (host double[4]) and count (host int64_t[4]), each
 * may be NULL, receive the accumulated milliseconds and launch counts of the
 * kernel kinds {first gradient, second gradient, sensor or indicator, flux + update};
 * reading waits for the recorded events. */
dolinc_status dolinc_timing(dolinc_ctx ctx, int32_t enable, double* ms, int64_t* count);

void dolinc_destroy(dolinc_ctx ctx);
const char* dolinc_last_error(void);
int32_t dolinc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DOLINC_H */
