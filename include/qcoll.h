/*
 * qcoll -- fast spectral Boltzmann collision operator on MI355X (gfx950).
 *
 * C ABI of libqcoll.so. Plain pointers and sizes only. Device pointers are HIP
 * device addresses on the device that was current when the plan was created.
 *
 * The operation (section 3.3 of Boscheri & Dimarco, "High order finite volume
 * schemes with IMEX time stepping for the Boltzmann model on unstructured
 * meshes"): for every space cell independently, given the discrete velocity
 * distribution f on the Cartesian grid of section 3.1 (eq. disc_space), compute
 * the spectral approximation Q_h(f, f) of the collision integral of eq.
 * (Boltzmann) written in the Carleman form (eqs. defQBCarleman, Btilde) with the
 * kernel modes of eq. (FKM) replaced by a sum over A = M collision directions,
 * evaluated as A discrete convolutions by DFT.
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - velocity nodes v_i = -L + i*2L/N per axis, i = 0..N-1 (period 2L);
 *   - f and Q are cell-major arrays [cells][N^d] with the LAST velocity axis
 *     fastest (row-major N x N in 2D);
 *   - Carleman truncation radius R = 4L/(3+sqrt 2) (QCOLL_R_LITERAL: 2L/(3+sqrt 2));
 *   - Fourier modes with a component equal to -N/2 are removed from every filter;
 *   - 2D: M equispaced directions on the half circle (M even);
 *     3D: M = 2 n^2 directions, n Gauss-Legendre nodes in cos(theta) on (0,1)
 *     times 2n equispaced azimuths;
 *   - b <= 0 selects b = 1/|S^(d-1)|.
 *
 * Errors: every entry point returns QCOLL_OK (0) or a negative code; argument
 * errors are reported synchronously before any device work is queued. Calls
 * that take a stream are asynchronous with respect to the host.
 */
#ifndef QCOLL_H
#define QCOLL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcoll_plan_s* qcoll_plan_t;

/* Collision kernel B of eq. (Boltzmann). Maxwell pseudo-molecules B = b
 * (section 2); hard spheres B = b |q|; variable hard spheres B = b |q|^gamma
 * (QCOLL_VHS, created through qcoll_plan_vhs only). Supported: 2D Maxwell, 2D
 * variable hard spheres, 2D and 3D hard spheres. */
enum { QCOLL_MAXWELL = 0, QCOLL_HARD_SPHERE = 1, QCOLL_VHS = 2 };

/* Arithmetic of the velocity DFTs (all variants compute the same Q_h):
 *   QCOLL_FP32     DFT-GEMMs on FP32 MFMA, FP32 spectra and filters.
 *   QCOLL_MIX_FX16 DFT-GEMMs on FP16 MFMA with a three-part split of both
 *                  operands: a fixed-point leading part whose products sum
 *                  exactly in the FP32 accumulator, plus an FP16 hi/lo
 *                  remainder (six products, two accumulators); spectra,
 *                  filters and all elementwise work in FP64. */
enum { QCOLL_FP32 = 1, QCOLL_MIX_FX16 = 4 };

/* Time schemes (section 3.4, homogeneous case): the single-stage updates of
 * qcoll_step and the multi-stage penalised IMEX Runge-Kutta steps of
 * qcoll_step_rk (tableaux ARS(2,2,2) and BPR(3,4,3) of section 3.4). */
enum {
  QCOLL_EXPLICIT_EULER = 0,
  QCOLL_IMEX_EULER_PENALIZED = 1,
  QCOLL_IMEX_ARS222 = 2,
  QCOLL_IMEX_BPR343 = 3
};

enum {
  QCOLL_OK = 0,
  QCOLL_EINVAL = -1,      /* bad argument (dimension, N, M, L, pointer, count) */
  QCOLL_ENOMEM = -2,      /* host or device allocation failed                  */
  QCOLL_EDEVICE = -3,     /* HIP runtime error or no device                    */
  QCOLL_EUNSUPPORTED = -4, /* valid but not implemented (size, kernel, mode)    */
  QCOLL_ETOOLARGE = -5     /* larger than the fixed scratch of qcoll_step_rk_noalloc */
};

/* Plan flags. */
#define QCOLL_CONSERVE 0x1u   /* FP64 moment projection; Q written as double   */
#define QCOLL_R_LITERAL 0x2u  /* Carleman radius 2L/(3+sqrt 2)                  */
#define QCOLL_HOST_ONLY 0x100u /* build the FP64 host tables only (no device)  */
#define QCOLL_GALERKIN 0x4u   /* dealiased variant (qcoll_eval_galerkin), 2D   */
#define QCOLL_CLASSICAL 0x8u  /* classical O(N^4) method, dense kernel modes  */
#define QCOLL_SEPARABLE_MODES 0x10u /* with QCOLL_CLASSICAL: the plan's own
                                       separable modes instead of exact ones */

/* Build a plan (section 3.3: directions, filters, loss multiplier; section
 * 3.1: grid). d in {2,3}; n_per_dim = N (even, 4..256); L > 0 half-width of
 * the velocity box; kernel QCOLL_MAXWELL or
 * QCOLL_HARD_SPHERE (QCOLL_VHS is QCOLL_EINVAL here); b kernel constant (<= 0: default); M number of collision
 * directions (the paper's A; even in 2D); K_r radial rank of the 2D
 * hard-sphere expansion (0: smallest rank with eigenvalue ratio < 1e-4;
 * ignored otherwise); precision one of the QCOLL_FP32 / QCOLL_MIX_FX16 values;
 * flags a combination of QCOLL_* flags. The plan owns its host and device
 * tables; apart from its launch shape (qcoll_plan_set_launch, set before use)
 * it is immutable and may be used from several streams at once, except 3D
 * plans, whose scratch area allows one call in flight at a time (the
 * qcoll_eval_ws / qcoll_step_ws calls take a workspace of the caller's and
 * lift that limit). On error *out
 * is set to NULL. Device plans: d = 2 with N <= 32 (grids below 16 or 32 run
 * zero-padded in a 16x16 or 32x32 tile) and 34 <= N <= 64 (radix-2 split into
 * 32-point tiles, one workgroup per cell), both in either precision; d = 3
 * hard spheres with N <= 32 in either precision (zero-padded
 * 16^3 or 32^3 tiles, one workgroup per cell,
 * a scratch area of 144 T^3 bytes per resident workgroup held by the plan; the
 * 3D FX16 variant splits the DFT-GEMM operands as in 2D but keeps spectra,
 * filters and work fields in FP32). Other sizes and precisions are
 * QCOLL_EUNSUPPORTED on the device (their host tables build). */
int qcoll_plan(qcoll_plan_t* out, int d, int n_per_dim, double L, int kernel, double b,
               int M, int K_r, int precision, unsigned flags);

/* Variable hard spheres B(|q|) = b |q|^gamma in 2D (-1 <= gamma <= 1; gamma = 1
 * is QCOLL_HARD_SPHERE, gamma = 0 Maxwell molecules): the Carleman weight
 * 2 b (rho^2 + rho'^2)^(gamma/2) expanded in K_r separable radial products as
 * for hard spheres (section 3.3, eqs. (Btilde), (FKM)). Other arguments and the
 * device support as for qcoll_plan with d = 2. */
int qcoll_plan_vhs(qcoll_plan_t* out, int n_per_dim, double L, double gamma, double b, int M, int K_r,
                   int precision, unsigned flags);

/* Classical spectral method (QCOLL_CLASSICAL, d = 2): Q_hat_k = sum over l + m = k
 * (modulo N, as the collocation of the fast method) of beta(l, m) f_l f_m with
 * beta(l, m) = B(l, m) - B(m, m) held as a dense N^2 x N^2 table (eqs. (CF1),
 * (KM), (ode), (FKM)), O(N^4) per cell, computed in FP64 on the device
 * (precision is ignored). The kernel modes B(l, m) are the exact ones, evaluated
 * with 8 N collision directions and, for hard and variable hard spheres, the
 * full-rank radial expansion on 2 N + 16 Gauss-Legendre nodes (converged to
 * rounding for Maxwell molecules; to about 1e-10 of the largest mode for hard
 * spheres, whose weight has a cone point); with QCOLL_SEPARABLE_MODES the table is the
 * plan's own separable sum over its M directions and K_r ranks, so that the
 * result is the fast operator computed by the direct sum. Device plans: N <= 24.
 * Classical plans evaluate through qcoll_eval (Q as double with QCOLL_CONSERVE)
 * and accept no other call; building the exact table takes O(N^4 x directions
 * x ranks) host work. */

/* Q = Q_h(f) for `cells` cells. f: device, float[cells][N^d]; Q: device,
 * float[cells][N^d], or double[cells][N^d] when the plan has QCOLL_CONSERVE
 * (then every cell's discrete mass, momentum and energy of Q vanish up to FP64
 * rounding). f and Q must not overlap. cells == 0 is a no-op. Caller owns both
 * buffers. Returns QCOLL_EINVAL for a NULL pointer or negative count,
 * QCOLL_EUNSUPPORTED for a host-only plan. */
int qcoll_eval(qcoll_plan_t plan, const float* f, void* Q, int64_t cells, hipStream_t stream);

/* The same evaluation and single-stage step with a workspace owned by the
 * caller in place of the plan's own scratch: 3D plans run one workgroup per
 * qcoll_scratch_bytes() of `work` (at least one; more allow more workgroups in
 * flight, up to one per cell), so that calls on the same 3D plan with distinct
 * workspaces may run concurrently on different streams (the plan's own scratch
 * allows one call in flight). 2D plans use no scratch: work may be NULL and
 * is ignored. QCOLL_EINVAL for a 3D plan with work NULL, not 256-byte aligned,
 * or work_bytes below one workgroup's scratch; otherwise arguments, results and errors as for
 * qcoll_eval and qcoll_step. qcoll_scratch_bytes: bytes of one workgroup's
 * scratch of a 3D device plan (144 T^3 for its T^3 tile), 0 for other plans,
 * -1 for NULL. */
int64_t qcoll_scratch_bytes(qcoll_plan_t plan);
int qcoll_eval_ws(qcoll_plan_t plan, const float* f, void* Q, int64_t cells, void* work, int64_t work_bytes,
                  hipStream_t stream);
int qcoll_step_ws(qcoll_plan_t plan, float* f, int64_t cells, double dt, double eps, int scheme, int32_t* status,
                  void* work, int64_t work_bytes, hipStream_t stream);

/* One space-homogeneous step of d f/dt = Q(f)/eps in place (section 3.4):
 *   QCOLL_EXPLICIT_EULER:        f <- f + (dt/eps) Q(f)
 *   QCOLL_IMEX_EULER_PENALIZED:  f <- f + (dt/eps) Q(f) / (1 + dt rho(f)/eps)
 * (the penalised IMEX Euler stage of eqs. (GIMEXb)-(GIMEX1b) with nu = rho; the
 * BGK terms cancel exactly because the moments are conserved). rho is
 * computed in FP64. status: device int32[cells] or NULL; when given, each
 * cell's entry is set to 0, or to 1 if the updated f has a non-finite value.
 * dt > 0 and eps > 0 are required. */
int qcoll_step(qcoll_plan_t plan, float* f, int64_t cells, double dt, double eps, int scheme,
               int32_t* status, hipStream_t stream);

/* Dealiased (Galerkin) variant of Q_h (eqs. (VAR), (ode): the sum over l + m = k
 * without wrap-around, k restricted to the modes of f). Plans created with
 * QCOLL_GALERKIN (d = 2, N a multiple of 4) evaluate the operator on the grid of
 * Nf = 3N/2 points per axis with the filters restricted to the active N-grid
 * modes (no component equal to -N/2), between a trigonometric interpolation of f
 * onto that grid and a restriction of Q back to the active N-grid modes; products
 * on the finer grid are exact non-wrapping convolutions for the kept modes. The
 * device kernels need Nf within the device sizes (N <= 40 in QCOLL_MIX_FX16,
 * N <= 20 in QCOLL_FP32). f: device float[cells][N][N]; Q: device
 * float[cells][N][N], or double with QCOLL_CONSERVE (FP64 projection on the N
 * grid). work: device buffer owned by the caller of at least
 * qcoll_galerkin_work_bytes() bytes (fine-grid f and Q); its content is scratch.
 * Galerkin plans accept no other evaluation or step call (QCOLL_EUNSUPPORTED). */
int64_t qcoll_galerkin_work_bytes(qcoll_plan_t plan, int64_t cells);
int qcoll_eval_galerkin(qcoll_plan_t plan, const float* f, void* Q, int64_t cells, void* work, int64_t work_bytes,
                        hipStream_t stream);

/* One multi-stage penalised IMEX Runge-Kutta step of d f/dt = Q(f)/eps in
 * place (eqs. (GIMEXb), (GIMEX1b) without transport, section 3.4). The
 * Boltzmann operator is split as Q = G_P + Q_BGK with Q_BGK(F) = nu (M - F)
 * implicit and G_P = Q - Q_BGK explicit; since the moments are conserved, every
 * stage uses the Maxwellian M of the discrete moments of f^n (FP64) and
 * nu = rho(f^n). Stage l (l = 2..S; stage 1 is f^n):
 *   F_l = [f^n + (dt/eps) sum_{m<l} (At_lm G_m + A_lm S_m) + A_ll (dt/eps) nu M]
 *         / (1 + A_ll dt nu / eps),   S_m = nu (M - F_m), G_m = Q(F_m) - S_m,
 * and f^{n+1} = F_S (both tableaux are stiffly accurate). Each stage l is one
 * launch that evaluates Q(F_{l-1}) and forms F_l. scheme: QCOLL_IMEX_ARS222
 * (S = 3, two launches) or QCOLL_IMEX_BPR343 (S = 5, four launches). work:
 * device float buffer owned by the caller, at least qcoll_step_rk_work_bytes()
 * bytes, holding the stage values and Q of earlier stages (FP32) and, per
 * cell, four FP64 moments of f^n (written by the first launch of the step,
 * read by the later ones); its content is scratch. status as in qcoll_step (set by the last stage). Every device
 * plan (2D and 3D); 3D plans hold a scratch area (see qcoll_eval_multi). */
int64_t qcoll_step_rk_work_bytes(qcoll_plan_t plan, int scheme, int64_t cells);
int qcoll_step_rk(qcoll_plan_t plan, float* f, int64_t cells, double dt, double eps, int scheme, float* work,
                  int64_t work_bytes, int32_t* status, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * step as qcoll_step_rk, with the work buffer taken from a fixed array of
 * QCOLL_NOALLOC_SCRATCH_BYTES in the library's device memory (one per GPU, held
 * from the first call on that GPU until the process ends). The call allocates
 * nothing. Problems whose qcoll_step_rk_work_bytes() exceed the array return
 * QCOLL_ETOOLARGE before any device work (e.g. at most 2337 cells of 32^2 for
 * QCOLL_IMEX_BPR343, 5447 for QCOLL_IMEX_ARS222). Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several streams, several
 * host threads) race and must be ordered by the caller. The array needs no
 * clearing (each stage slot, and the moments of f^n, is written before it is
 * read within the step). Other arguments,
 * errors and results as for qcoll_step_rk, whose results it reproduces
 * bitwise. */
#define QCOLL_NOALLOC_SCRATCH_BYTES (64ll << 20)
int qcoll_step_rk_noalloc(qcoll_plan_t plan, float* f, int64_t cells, double dt, double eps, int scheme,
                          int32_t* status, hipStream_t stream);

/* Batched launches (cell-locality of section 3.3: cells of different velocity
 * grids and kernels share one launch). Slot i uses plans[i] with f[i], Q[i]
 * (or status[i]) and cells[i] exactly as the single-plan call; each cell's
 * result is bitwise equal to the single-plan launch. nplans <= 64, all plans
 * on one device; slots with cells[i] == 0 are skipped. status may be NULL.
 * 2D plans share one launch per 8 slots (N <= 32: a wavefront per cell; N > 32:
 * a workgroup per cell); 3D plans (all slots 3D) share one launch per 8 slots.
 * When a 2D call has several launches (more than 8 slots) and few cells (at
 * most four per compute unit in total, as in a serving tick) they run
 * concurrently, the first on `stream` and the others on up to three side
 * streams of the library (default priority) that wait for `stream` before
 * they start and that `stream` waits for afterwards, so the call as a whole is
 * ordered on `stream`; larger calls, and calls while `stream` is being
 * captured into a graph, queue the launches on `stream` one after another. 2D
 * and 3D plans cannot be mixed in one call (QCOLL_EUNSUPPORTED). 3D plans hold
 * a scratch area: calls that use the same 3D plan must not run concurrently on
 * different streams (qcoll_eval_ws takes a workspace of the caller's). */
int qcoll_eval_multi(const qcoll_plan_t* plans, int nplans, const float* const* f, void* const* Q,
                     const int64_t* cells, hipStream_t stream);
int qcoll_step_multi(const qcoll_plan_t* plans, int nplans, float* const* f, const int64_t* cells, double dt,
                     double eps, int scheme, int32_t* const* status, hipStream_t stream);

/* Launch shape of single-plan calls: cells per workgroup (1, 2 or 4) and the
 * grid cap in workgroups (each wavefront loops over cells beyond it). 2D
 * FX16 device plans with N <= 32 (32x32 tile) also take 8: the ping-pong
 * variant, eight cells per workgroup whose two wavefronts per SIMD alternate
 * between matrix and vector phases; its results are bitwise equal to the
 * other shapes. Other values, and 8 for other plans, return QCOLL_EINVAL. */
int qcoll_plan_set_launch(qcoll_plan_t plan, int waves_per_block, int64_t max_blocks);
int qcoll_plan_get_launch(qcoll_plan_t plan, int* waves_per_block, int64_t* max_blocks);

/* Tile family of a 2D plan: 2D plans with N <= 16 run on the 16x16 MFMA tile
 * kernels (v_mfma_f32_16x16x32_f16 / 16x16x4f32) by default and also hold the
 * tables of the 32x32 tile kernels (v_mfma_f32_32x32x16_f16 / 32x32x2f32, the
 * grid zero-padded), so either can run them (same Q_h up to rounding; the
 * parity bounds of the plan's precision hold for both). set_tile selects 16
 * or 32 for such plans and returns QCOLL_EINVAL for any other value (other
 * plans have one tile family: 32 for 18..32 points, 64 for 34..64); get_tile
 * reports the selected tile and the alternate one (0: none). Selecting a
 * family whose kernels lack the launch shape 8 resets that shape to 4. */
int qcoll_plan_set_tile(qcoll_plan_t plan, int tile);
int qcoll_plan_get_tile(qcoll_plan_t plan, int* tile, int* alternate);

/* Transform split (latency form for small batches; the operator of section 3.3
 * is a sum over the plan's transforms, so a cell's transforms can be shared out):
 *   1  default: one wavefront (N <= 32) or one workgroup (N > 32) per cell;
 *   4  FX16 plans on the 32x32 tile: a workgroup of four wavefronts per cell,
 *      each wavefront taking every fourth transform, the partial sums added in
 *      LDS in a fixed order;
 *   2, 4, 8, 16  tile-64 plans (FX16 or FP32): that many workgroups per cell, the
 *      partial sums added in a fixed order by the workgroup that finishes last
 *      (through device buffers the plan allocates on first use, sized for the
 *      largest batch seen: split x 32 KiB per cell, plus a counter per cell).
 * Other values, and split factors a plan's kernels lack, return QCOLL_EINVAL;
 * selecting a tile family without the current factor resets it to 1. The
 * split form applies to qcoll_eval, qcoll_step and the batched calls (the
 * qcoll_step_rk family ignores it). Results differ from the unsplit ones by
 * the order of the gain sum only (within the precision's parity bounds) and
 * are deterministic. A first call on more cells than the buffers hold grows
 * them, which synchronises the stream and returns QCOLL_EINVAL under graph
 * capture; calls that use the same split tile-64 plan must not run concurrently
 * on different streams. */
int qcoll_plan_set_split(qcoll_plan_t plan, int split);
int qcoll_plan_get_split(qcoll_plan_t plan, int* split);

/* Autotuner: times every launch shape on the caller's f (device, cells cells)
 * with HIP events, `reps` launches each, and keeps the fastest in the plan:
 * tile family (see qcoll_plan_set_tile) x cells per workgroup (1, 2, 4, and 8
 * where the ping-pong variant exists) x grid cap. 2D fast plans only (3D,
 * Galerkin and classical plans have one launch shape: QCOLL_EUNSUPPORTED).
 * Synchronises the stream; Q (device, as for qcoll_eval) is overwritten. */
int qcoll_plan_autotune(qcoll_plan_t plan, const float* f, void* Q, int64_t cells, int reps, hipStream_t stream);

/* Plan properties: number of DFT passes per cell (packed transforms incl. the
 * loss), radial rank, Carleman radius, and the device bytes the plan holds. */
int qcoll_plan_info(qcoll_plan_t plan, int* transforms, int* K_r, double* R, int64_t* device_bytes);

/* FP64 host tables for verification. which:
 *   0 alpha_t(k)  (index t over directions x radial ranks, out[N^d], FFT order)
 *   1 alpha'_t(k) (same)
 *   2 W_t         (out[terms], index ignored)
 *   3 loss multiplier l(k) = sum_t W_t alpha_t alpha'_t (out[N^d])
 *   4 radial eigenvalues lambda_j (out[K_r]; {1} for separable kernels)
 *   5 inverse Gram matrix of phi = (1, v, |v|^2) on the grid (out[(d+2)^2])
 *   6 classical plans: row m of the kernel-mode table, beta(l, m) over l
 *     (index = m, out[N^2], FFT order)
 * A Galerkin plan returns tables 0-4 of its Nf grid (0, 1 and 3 zero outside the
 * active N-grid modes) and table 5 of the N grid.
 * n is the capacity of out; returns the number of values written or QCOLL_EINVAL. */
int qcoll_plan_table(qcoll_plan_t plan, int which, int index, double* out, int64_t n);

/* Release the plan and its device tables (after all its work has completed). */
void qcoll_plan_destroy(qcoll_plan_t plan);

/* Static string for an error code. */
const char* qcoll_strerror(int code);

/* ------------------------------------------------------------------------
 * Transport on polygonal meshes (section 2.2): the CWENO reconstruction of
 * the cell values of every discrete velocity (eqs. (CWENO:Popt), (CWENO:P0),
 * (CWENO:Prec), (eqn.weights) with the Taylor basis of
 * (eq.Dubiner_phi_spatial)) and the Rusanov fluxes through the cell faces
 * (eqs. (finite_vol3), (finite_vol5)), on a periodic mesh of polygons.
 *
 * Mesh (host arrays, copied by the plan; polygon-major, float64 coordinates):
 *   cell_ptr[cells+1]   face/vertex slots of cell i: cell_ptr[i] .. cell_ptr[i+1]-1
 *                       (3 .. 12 faces per cell)
 *   verts[2 m]          polygon vertices (x, y), counter-clockwise, in the cell's frame
 *   nbr[m]              the cell across face k (from vertex k to vertex k+1)
 *   shift[2 m]          offset that maps the neighbour's frame into this cell's frame
 *   twin[m]             slot of the same face in the neighbour's list
 *   gen[2 cells]        generator point of each cell (ranks the stencil candidates)
 * degree: polynomial degree of the reconstruction, 1 (second order) or 2 (third).
 * Velocities: the n_per_dim^2 nodes v = -L + j 2L/n_per_dim of the collision grid
 * (2 <= n_per_dim <= 64); f is stored float[cells][n_per_dim][n_per_dim].
 * Readings of the section's open choices: central stencil = the 2 dim(P_degree) - 1
 * cells whose generators are nearest (within three face rings, ties by cell
 * index and image offset); one-sided P1 stencil per face L = {P_i, neighbour
 * across face L, neighbour across face L+1}; linear weights 1e5 (central) and 1
 * (each one-sided), normalised; oscillation indicator = sum over derivatives of
 * order 1..degree of the cell mean of the squared derivative in the scaled Taylor
 * variables; Rusanov speed |v . n| per velocity.
 * flags: QCOLL_HOST_ONLY builds the host tables only. */
typedef struct qcoll_transport_s* qcoll_transport_t;
int qcoll_transport_plan(qcoll_transport_t* out, int64_t cells, const int64_t* cell_ptr, const double* verts,
                         const int64_t* nbr, const double* shift, const int64_t* twin, const double* gen,
                         int degree, int n_per_dim, double L, unsigned flags);

/* Bytes of the work buffer of a transport call: the reconstructed face values,
 * float[faces][n_per_dim^2]. */
int64_t qcoll_transport_work_bytes(qcoll_transport_t plan);

/* R = -(1/|P_i|) sum over faces of the Rusanov flux of the reconstructed states
 * (device float[cells][n^2] in and out, distinct buffers), or, for the step,
 * out = f + dt R (explicit Euler transport step; out may not alias f). work: device
 * buffer of at least qcoll_transport_work_bytes() bytes owned by the caller.
 * Returns QCOLL_EINVAL for NULL pointers or a small work buffer,
 * QCOLL_EUNSUPPORTED for a host-only plan. */
int qcoll_transport_rhs(qcoll_transport_t plan, const float* f, float* R, void* work, int64_t work_bytes,
                        hipStream_t stream);
int qcoll_transport_step(qcoll_transport_t plan, const float* f, float* out, double dt, void* work,
                         int64_t work_bytes, hipStream_t stream);

/* Host tables of cell `index` for verification. which:
 *   0 central stencil: cell indices followed by their image offsets (x then y)
 *     (out[3 (n_e - 1)])
 *   1 geometry: area, barycentre x, y, h (out[4])
 *   2 least-squares operator of the optimal polynomial, [K][n_e - 1] row-major
 *   3 face averages of the Taylor basis functions, [faces][K]
 *   4 per face: outward normal x, y, |face| / |P_i|, inverse of the one-sided
 *     stencil's 2x2 system (row-major), [faces][7]
 *   5 oscillation form: coefficients of c_a c_b, a <= b, row by row (15 values)
 * Returns the number of values written or QCOLL_EINVAL. */
int qcoll_transport_table(qcoll_transport_t plan, int which, int64_t index, double* out, int64_t n);

void qcoll_transport_destroy(qcoll_transport_t plan);

#ifdef __cplusplus
}
#endif

#endif /* QCOLL_H */
