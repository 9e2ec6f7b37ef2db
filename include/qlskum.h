/*
 * qlskum.h -- C ABI of the MI355X (gfx950) q-LSKUM solver library.
 *
 * The library advances the 2D Euler equations on a point cloud with the
 * q-LSKUM meshfree scheme of "On the performance of GPU accelerated q-LSKUM
 * based meshfree solvers in Fortran, C++, Python, and Julia" (Scientific
 * Computing Report 01:2021): per pseudo-time iteration a local time step,
 * then four Runge-Kutta stages of q-variables (sec. 2.1 eq. (26)),
 * least-squares q-derivatives with inner iterations (eq. (29)), the
 * kinetic split-flux residual over the four split stencils (eqs. (12)-(14),
 * (27)-(28)) and the state update, then the residual norm (sec. 3,
 * Algorithm 1).  Every step runs in the library's HIP kernels.
 *
 * Conventions (all entry points):
 *  - Return an int status (QL_OK or a negative QL_E* code); no call aborts
 *    the process.  ql_last_error() gives a message naming the point
 *    (user numbering) or the argument at fault.
 *  - Sizes are int64_t.  Per-point vectors are component-major ("SoA"):
 *    U[c * n + p], c = 0..3 for (rho, rho u1, rho u2, rho e), p in the
 *    caller's point order.  The library reorders points internally for
 *    memory locality; callers always see their own order.
 *  - Host pointers are borrowed for the duration of the call and copied.
 *    Device pointers (mem = 1) must be device memory on the solver's
 *    device (for example a torch tensor's data_ptr()); they are read or
 *    written in stream order on the solver's stream and must stay valid
 *    until the call returns.
 *  - The library owns every solver buffer.  One solver per host thread;
 *    solvers on one device may share a stream.
 *  - After QL_EDEVICE the solver is poisoned: only ql_destroy and
 *    ql_last_error remain valid.  Calls out of order (a step before an
 *    upload, for example) return QL_ESTATE.
 */
#ifndef QLSKUM_H
#define QLSKUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ql_solver ql_solver;

enum {
    QL_OK = 0,
    QL_EINVAL = -1,      /* bad argument or malformed cloud                   */
    QL_ESINGULAR = -2,   /* a least-squares matrix the scheme inverts is singular */
    QL_ENOMEM = -3,      /* device or host allocation failed                  */
    QL_EDEVICE = -4,     /* HIP runtime error; solver poisoned                */
    QL_ENONFINITE = -5,  /* NaN or Inf in a state                             */
    QL_EPOSITIVITY = -6, /* non-positive density/pressure or q4 >= 0          */
    QL_EDIVERGED = -7,   /* residual blow-up (status of a batched case)       */
    QL_ESTATE = -8       /* call out of order                                 */
};

/* point kinds */
enum { QL_KIND_INTERIOR = 0, QL_KIND_WALL = 1, QL_KIND_OUTER = 2 };

/* Split-stencil membership bits of one neighbour entry (sec. 2 eq. (14)),
 * in the point's frame: s along t = (n_y, -n_x), n along the point's unit
 * normal.  S_PLUS: ds < 0, S_MINUS: ds > 0, N_PLUS: dn < 0, N_MINUS: dn > 0;
 * an entry with |ds| <= 1e-12 |d| (resp. dn) is in neither s (n) half. */
enum { QL_SPLIT_S_PLUS = 1, QL_SPLIT_S_MINUS = 2, QL_SPLIT_N_PLUS = 4, QL_SPLIT_N_MINUS = 8 };

typedef struct {
    double gamma;     /* ratio of specific heats (1.4)                          */
    double mach;      /* freestream Mach number (rho_inf = 1, c_inf = 1)        */
    double alpha_deg; /* angle of attack, degrees                               */
    double cfl;       /* local time step dt = cfl * min|P_i - P| / (|u| + c)     */
    int32_t n_inner;  /* inner iterations of the q-derivatives (3), >= 0        */
    int32_t limiter;  /* 0 none, 1 Venkatakrishnan                              */
    double venkat_k;  /* limiter constant K, eps^2 = (K |P_i - P|)^3            */
    int32_t precision;/* 0 FP64 throughout; 1 mixed: reconstruction, limiter
                         and split fluxes in FP32, least-squares weights,
                         residual sums and the state update in FP64; the
                         q-derivatives in FP64 arithmetic (see mixed_grad)   */
    int32_t reorder;  /* read at upload: 0 caller order, 1 Hilbert curve,
                       * 2 reverse Cuthill-McKee on the neighbour graph      */
    int32_t flux_lds; /* tuning: bytes of LDS in which a flux workgroup stages
                         the records of its 64-point tile and halo (tiles that
                         do not fit read from memory; same results either
                         way); 0 = the library's default, at most 163840      */
    int32_t grad_lds; /* tuning: the same for the q-derivative sweeps (records
                         of 48 and 80 bytes; 32 and 48 for the FP32-data
                         sweeps of mixed_grad 0); 0 = default, at most
                         163840                                               */
    int32_t order;    /* 2: second order, the split fluxes of the modified q
                         of eq. (28) (sec. 2.1); 1: first-order LSKUM, the
                         split fluxes of q itself (sec. 2; no q-derivatives
                         are computed in ql_step, the limiter is unused).
                         Switching between ql_step calls is allowed: a
                         first-order start-up followed by second order     */
    int32_t flux_split;/* 0: one fused flux sweep; 1 (FP64, second order): the
                         s-direction split fluxes in one launch and the
                         n-direction ones with the update in a second (fewer
                         registers per launch, the reconstruction done twice);
                         2 (FP64, second order): one launch per split stencil
                         s+, s-, n+, n- (the kernel splitting of the paper's
                         sec. 5), the last with the update.  The residual's
                         summation grouping changes in the last bits       */
    int32_t outer_bc; /* 0: outer points held at the freestream (Dirichlet);
                         1: kinetic outer condition (sec. 2.1 combines the
                         scheme with it; its formula is left to a reference):
                         outer points are updated like interior points, with
                         their n- split stencil, which would lie beyond the
                         far field, replaced by the mirror image of their n+
                         stencil through the point's tangent line, whose
                         points hold the freestream Maxwellian.  Outer
                         normals point to the far field.  Outer points then
                         count in the residual norm.  Needs non-singular
                         s+, s-, n+ stencils at every outer point
                         (QL_ESINGULAR otherwise, at upload or here)      */
    int32_t mixed_grad;/* precision 1: data of the q-derivative sweeps (whose
                         sums and 2x2 solves are FP64 either way).  0: FP32
                         copies of q and of the inner iterates, widened to
                         FP64: the first pass is then the exact least-squares
                         derivative of the FP32 q that the flux body
                         reconstructs from, and each iterate is rounded to
                         FP32 (2^-24 relative) before the next uses it;
                         1: FP64 q and iterates, as in precision 0.
                         ql_batch_run with mixed_switch > 0 uses 1          */
    double mixed_switch; /* precision 1 in ql_batch_run: a case whose density
                         residual norm falls to mixed_switch x its reference
                         continues with FP64 split fluxes (the FP32 flux body
                         resolves the residual only to a few 1e-6 of its
                         first value); 0 = never.  In [0, 1)                */
} ql_params;

/* Fill *p with the defaults: gamma 1.4, M 0.63, alpha 2, CFL 0.2, 3 inner
 * iterations, limiter off (K = 5), FP64, Hilbert reorder, default LDS
 * budgets (0), second order, fused flux sweep, outer points held. */
void ql_default_params(ql_params *p);

/* Create a solver on HIP device `device`.  `hip_stream` is a hipStream_t
 * (for example torch.cuda.current_stream().cuda_stream) on which every
 * kernel and copy of this solver is enqueued; NULL makes the library create
 * its own stream.  *out receives the handle (NULL on failure).
 * Errors: QL_EINVAL (out NULL), QL_EDEVICE. */
int ql_create(ql_solver **out, int32_t device, void *hip_stream);

/* Free every buffer of the solver (NULL is a no-op). */
int ql_destroy(ql_solver *s);

/* Upload a point cloud (sec. 3: the input data structure copied to the
 * device once).  Host arrays, caller order:
 *   x, y, nx, ny : double[n]   positions and unit normals (frame of the
 *                              split stencils; at wall points the normal
 *                              points into the fluid)
 *   kind         : uint8[n]    QL_KIND_*
 *   nbr_ptr      : int32[n+1]  CSR row pointers, nbr_ptr[0] = 0
 *   nbr_idx      : int32[nnz]  neighbours of each point (no self, in range);
 *                              their order is kept for every sum
 *   nbr_flag     : uint8[nnz]  split membership (QL_SPLIT_* bits) or NULL to
 *                              let the library classify the entries.
 * The library validates the CSR, reorders points (params.reorder), and on
 * the device classifies entries, precomputes least-squares factors and
 * checks that every matrix the scheme inverts is non-singular: the full
 * stencil of every point and each split stencil entering the residual
 * (interior: all four; wall: s+, s-, n-; outer, with params.outer_bc = 1
 * only: s+, s-, n+), each needing >= 2 points and
 * det > 1e-12 (sum ds^2 + sum dn^2)^2.
 * Errors: QL_EINVAL (malformed input), QL_ESINGULAR (message names the
 * point), QL_ENOMEM, QL_EDEVICE.  Any previous cloud and state are dropped. */
int ql_upload_cloud(ql_solver *s, int64_t n, const double *x, const double *y,
                    const double *nx, const double *ny, const uint8_t *kind,
                    const int32_t *nbr_ptr, const int32_t *nbr_idx,
                    const uint8_t *nbr_flag);

/* Set flow and solver parameters (copied).  Errors: QL_EINVAL. */
int ql_set_params(ql_solver *s, const ql_params *p);

/* Set every point to the freestream (rho 1, p 1/gamma, u = M (cos a, sin a))
 * and project the wall points' momentum onto the wall tangent.
 * Errors: QL_ESTATE (no cloud), QL_EDEVICE. */
int ql_init_freestream(ql_solver *s);

/* Set the conserved state from U[4][n] (caller order; mem 0 host, 1 device).
 * project_wall != 0 applies the wall projection m <- m - (m.n) n.
 * Errors: QL_ESTATE, QL_ENONFINITE / QL_EPOSITIVITY (message names the
 * first point), QL_EDEVICE. */
int ql_set_state(ql_solver *s, const double *U, int32_t mem, int32_t project_wall);

/* Run n_iter pseudo-time iterations (sec. 3 Algorithm 1): per iteration the
 * local time step, four stages of four-stage third-order SSP Runge-Kutta,
 * and the residual norm of the first stage's residual.  res_hist (host,
 * nullable) receives [n_iter][ncase][4] residual norms (root mean square
 * over the interior and wall points of each component, and the outer points
 * under the kinetic outer condition; ncase = 1 unless
 * the cloud came from ql_batch_upload).  Enqueues on the solver's
 * stream; synchronises once at the end when res_hist is not NULL.  With
 * res_hist NULL it returns once the work is enqueued, and the next call on
 * the solver collects the outcome: a failure during these iterations is
 * then returned by that call (ql_residual_norm, ql_fetch_state, ...).
 * Errors: QL_ESTATE, QL_EPOSITIVITY / QL_ENONFINITE (the smallest failing
 * point and its own code; the state is then undefined), QL_EDEVICE. */
int ql_step(ql_solver *s, int32_t n_iter, double *res_hist);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): ql_step with
 * the residual history staged in a fixed device array of the library
 * instead of a buffer the solver grows, and no timing events.  Same
 * kernels, same results as ql_step bit for bit.  The array holds 65536
 * doubles per GPU (allocated once per process and device, never freed):
 * n_iter x ncase x 4 must not exceed it, else QL_EINVAL.  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (solvers on
 * several host threads or streams) race; the array keeps the last call's
 * rows.  res_hist and the deferred status as ql_step.  Errors as ql_step,
 * and QL_EINVAL (n_iter over the array's rows). */
int ql_step_static(ql_solver *s, int32_t n_iter, double *res_hist);

/* Residual norms of the last iteration ql_step ran (synchronises when that
 * call returned without a history).  Errors: QL_ESTATE, or the failure of
 * those iterations. */
int ql_residual_norm(const ql_solver *s, double out[4]);

/* Copy the conserved state to U[4][n] in caller order (mem 0 host, 1
 * device).  Synchronises.  Errors: QL_ESTATE, QL_EDEVICE. */
int ql_fetch_state(ql_solver *s, double *U, int32_t mem);

/* Lift and drag coefficients of the current state from the wall pressure:
 * F = -sum (p - p_inf) n ds over wall points, where the wall points in the
 * caller's order form the closed surface polygon and
 * ds = (|S_next - S| + |S - S_prev|)/2; the upper (y > 0), lower (y < 0)
 * and on-axis parts are summed separately, then added.
 * Cl = F.(-sin a, cos a)/q_inf, Cd = F.(cos a, sin a)/q_inf.
 * Errors: QL_ESTATE, QL_EINVAL (fewer than 3 wall points), QL_EDEVICE. */
int ql_forces(ql_solver *s, double *cl, double *cd);

/* Message of the last failing call on this solver ("" if none). */
const char *ql_last_error(const ql_solver *s);

/* --- batched form: many independent cases in one set of launches ------- */

/* Upload ncase independent clouds, concatenated in the caller's order: case
 * c owns caller points case_ptr[c] .. case_ptr[c+1]-1 (case_ptr[0] = 0,
 * case_ptr[ncase] = n, every case non-empty); its neighbour lists index the
 * concatenated arrays and stay inside the case; mach[c] and alpha_deg[c]
 * are its freestream.  Every iteration kernel then advances all cases in
 * one launch.  Arrays and validation as ql_upload_cloud (the library
 * classifies the split stencils), which is the one-case form: there the
 * freestream follows ql_set_params.  Per-case results: ql_step's res_hist
 * becomes [n_iter][ncase][4]; ql_residual_norm and ql_forces report case 0.
 * Errors as ql_upload_cloud. */
int ql_batch_upload(ql_solver *s, int32_t ncase, const int64_t *case_ptr, int64_t n,
                    const double *x, const double *y, const double *nx, const double *ny,
                    const uint8_t *kind, const int32_t *nbr_ptr, const int32_t *nbr_idx,
                    const double *mach, const double *alpha_deg);

/* Number of cases of the uploaded cloud.  Errors: QL_ESTATE. */
int ql_batch_info(const ql_solver *s, int32_t *ncase);

/* Iterate all cases until each one's density residual norm falls to
 * drop x its reference norm, or max_iter iterations.  The reference of case
 * c is ref_res[c] when ref_res is not NULL (e.g. the freestream residual
 * that ql_warm_start reports), else the norm of the first iteration of this
 * call.  Retirement happens on the device, after the residual norms of
 * every iteration: a case whose norm of iteration m (the norm of the state
 * the iteration started from) reaches the drop keeps the state that
 * iteration m leaves, which is the state of ql_step(m) from the same start,
 * and iters_out[c] = m.  Its points stop updating and workgroups holding
 * only retired points skip every sweep, while the other cases go on.  The
 * host reads the active flags every check_every iterations to stop once
 * none is left; after a window in which cases retired, the tiled sweeps
 * are launched over the tiles that still hold an active case only (the
 * results are the same bit for bit).  graph != 0 captures one iteration into a hipGraph on
 * the solver's stream (re-captured after parameter or buffer changes) and
 * replays it.  iters_out[c] (nullable) receives the iterations case c ran,
 * res_out[c][4] (nullable) the norms of its last one.
 * A case whose state fails (positivity lost, or a non-finite value) in
 * iteration m is retired at the end of m with that status, as is a case
 * whose norm exceeds 1e8 x its reference (QL_EDIVERGED); the other cases go
 * on, and ql_batch_status reports every retired case's status.  A failed
 * case's state is not usable: set a new state before stepping again.
 * Errors: as ql_step for failures that name no case; QL_EINVAL (drop <= 0,
 * max_iter < 0, check_every < 1, a reference <= 0 or not finite). */
int ql_batch_run(ql_solver *s, double drop, int32_t max_iter, int32_t check_every, int32_t graph,
                 const double *ref_res, int32_t *iters_out, double *res_out);

/* Progress of long batched runs: after every window of check_every
 * iterations, ql_batch_run calls fn(user, iterations done, cases still
 * active) on the calling thread, between windows (the device is idle for the
 * call's duration; the callback must not call the library on this solver).
 * fn = NULL turns it off.  Errors: QL_EINVAL (NULL solver). */
typedef void (*ql_progress_fn)(void *user, int32_t iterations, int32_t active);
int ql_set_progress(ql_solver *s, ql_progress_fn fn, void *user);

/* Per-case outcome of the last ql_batch_run: status[c] = QL_OK (reached the
 * drop or ran max_iter), QL_EPOSITIVITY or QL_ENONFINITE (case c failed and
 * was retired), QL_EDIVERGED (its norm blew up).  status holds ncase entries (ql_batch_info); all QL_OK
 * before any run.  Errors: QL_EINVAL (NULL), QL_ESTATE (no cloud). */
int ql_batch_status(const ql_solver *s, int32_t *status);

/* Iteration of the last ql_batch_run after which case c moved from FP32 to
 * FP64 split fluxes (params.mixed_switch), or -1: iter[ncase].
 * Errors: QL_EINVAL (NULL), QL_ESTATE (no cloud). */
int ql_batch_switched(const ql_solver *s, int32_t *iter);

/* Lift and drag of every case (as ql_forces), cl[ncase], cd[ncase]. */
int ql_batch_forces(ql_solver *s, double *cl, double *cd);

/* --- warm start: a learned initial state ------------------------------- */

/* A multilayer perceptron on the device, widths[0] inputs -> hidden layers
 * of widths[1 .. nwidth-2] with tanh -> widths[nwidth-1] linear outputs,
 * evaluated and trained with bfloat16 operands on the matrix cores (FP32
 * accumulation; bias, tanh, loss and Adam in FP32).  The initial state of
 * an explicit solve is arbitrary; a network that maps point features
 * (position, wall distance, flow condition) to the converged primitive
 * fields gives a start closer to the solution (the paper's method starts
 * from the freestream; this is an addition to it).  The network object is
 * separate from the solver; max_batch
 * bounds the rows of one training step (inference is chunked).  The
 * library owns all device buffers; hip_stream as in ql_create.
 * Weights are one FP32 vector: for each layer l, W_l row-major
 * (widths[l] x widths[l+1]) then b_l (widths[l+1]).
 * Errors: QL_EINVAL (widths outside 1..4096, fewer than 2, max_batch
 * outside 1..2^26), QL_EDEVICE, QL_ENOMEM. */
typedef struct ql_mlp ql_mlp;
int ql_mlp_create(ql_mlp **out, int32_t device, void *hip_stream, const int32_t *widths,
                  int32_t nwidth, int64_t max_batch);
int ql_mlp_destroy(ql_mlp *m);
const char *ql_mlp_last_error(const ql_mlp *m);
int ql_mlp_num_params(const ql_mlp *m, int64_t *np);

/* Host FP32 weights in / out.  Setting them restarts Adam (moments 0).
 * Errors: QL_EINVAL, QL_ENONFINITE (a weight is not finite), QL_ESTATE
 * (get before any set). */
int ql_mlp_set_weights(ql_mlp *m, const float *w);
int ql_mlp_get_weights(ql_mlp *m, float *w);

/* Y[n][w_out] = network(X[n][w_in]); X, Y device FP32, row-major, enqueued
 * on the network's stream.  Errors: QL_EINVAL, QL_ESTATE (no weights). */
int ql_mlp_forward(ql_mlp *m, const float *X, float *Y, int64_t n);

/* Mean squared error over the n x w_out outputs of one batch (device X, T;
 * 1 <= n <= max_batch) and its gradient: *loss (nullable), grad[np] (host,
 * nullable; the weight layout).  ql_mlp_train_step also applies one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) to the FP32
 * master weights.  Both synchronise when they return values. */
int ql_mlp_gradient(ql_mlp *m, const float *X, const float *T, int64_t n, float *grad,
                    double *loss);
int ql_mlp_train_step(ql_mlp *m, const float *X, const float *T, int64_t n, float lr,
                      double *loss);
int ql_mlp_sync(ql_mlp *m);

/* Distance of every point to the nearest wall point of its case, host
 * d[n] in caller order (+inf for a case without wall points).
 * Errors: QL_ESTATE (no cloud), QL_EINVAL. */
int ql_wall_distance(ql_solver *s, double *d);

/* Warm start of every case of the uploaded cloud.  X (device FP32
 * [n][w_in], caller order) are the network's inputs; its outputs are the
 * standardised (rho, u1, u2, p): prim = out_scale[k] + out_scale[4+k] * y_k.
 * Density and pressure are held at or above rel_floor times their
 * freestream values, wall points get the wall projection, outer points keep
 * the freestream.  Then, per case, the stage-1 residual norms of this warm
 * state and of the freestream are compared; a case starts warm only if its
 * warm density-residual norm is finite and not larger than the cold one
 * (and no point of it failed), else from the freestream.  res_cold and
 * res_warm ([ncase][4], nullable) receive both norms, used[ncase]
 * (nullable) the choice.  The state is then set as by ql_set_state.
 * Errors: QL_EINVAL (network without weights or not 4 outputs, NULL
 * arrays, rel_floor outside (0, 1)), QL_ESTATE, device errors; a failure
 * of the freestream evaluation is reported as by ql_step. */
int ql_warm_start(ql_solver *s, ql_mlp *m, const float *X, const float *out_scale,
                  double rel_floor, double *res_cold, double *res_warm, int32_t *used);

/* --- inspection and timing (tests, benchmarks) ------------------------- */

/* One evaluation of the stage operator at the current state, without
 * updating it: q, the q-derivatives after n_inner inner iterations, the
 * limiter bounds, the residual R and the time step.  Fetch them with
 * ql_debug_fetch.  Errors as ql_step. */
int ql_evaluate(ql_solver *s);

/* The flux sweep's tiles (64 consecutive points of the library's order):
 * *ntile receives their number (0 when the cloud has no tiling: every tile
 * reads from memory), and slots[ntile], when not NULL, the records each
 * tile's LDS image holds (its points plus its halo).  A tile is staged in
 * LDS when slots * record bytes <= the flux_lds budget; the record is 176
 * bytes (FP64 with limiter), 112 (FP64), 96 (mixed with limiter) or 64
 * (mixed).  Errors: QL_EINVAL (NULL), QL_ESTATE (no cloud). */
int ql_flux_tiles(const ql_solver *s, int32_t *ntile, int32_t *slots);

/* Autotuning of the tiled sweeps: times the flux sweep (stage evaluation)
 * and the q-derivative sweeps of the current state for a set of LDS
 * budgets and keeps the fastest in flux_lds and grad_lds.  Results do not
 * depend on the budgets (tiles that do not fit read from memory with the
 * same arithmetic), so tuning never changes an answer.  When cache_path is
 * not NULL the choice is looked up there first, keyed by precision,
 * limiter, size class (log2 n) and mean stencil size, and stored there
 * after tuning (a small JSON object, one entry per line).  chosen[2]
 * (nullable) receives (flux_lds, grad_lds).  The state is not changed.
 * Errors: QL_ESTATE (no state), QL_EINVAL (unreadable or unwritable cache
 * file), device errors. */
int ql_autotune(ql_solver *s, const char *cache_path, int32_t *chosen);

/* Copy an inspection array to host memory `out` in caller order:
 *   0 q [4][n]       1 g [8][n] (q_x rows 0..3, q_y rows 4..7)
 *   2 R [4][n]       3 dt [n]
 *   4 qmax [4][n]    5 qmin [4][n]
 * After ql_evaluate all six hold that evaluation; after ql_step, 0 and 3
 * hold the current state's q and time step.  The bounds are kept as offsets
 * from q (what the limiter uses) and returned as q plus that offset, within
 * an ulp of the bound.  In mixed precision (precision 1, no precision
 * switch) q, g and the bounds are the FP32 values the flux sweep reads,
 * widened.  Errors: QL_EINVAL, QL_ESTATE. */
int ql_debug_fetch(ql_solver *s, int32_t what, double *out);

/* Copy the split-membership flags to uint8 out[nnz] in the caller's CSR
 * entry order.  Errors: QL_ESTATE. */
int ql_debug_flags(ql_solver *s, uint8_t *out);

/* Number of points and neighbour entries of the uploaded cloud. */
int ql_cloud_size(const ql_solver *s, int64_t *n, int64_t *nnz);

/* Kernel timing: when enabled, ql_step brackets every launch with HIP
 * events on the solver's stream.  ql_kernel_time returns, for kernel kind
 * `which` (0 gradient first pass, 1 gradient inner iteration, 2 flux
 * residual + update, 3 residual norm), the summed duration in ms and the
 * launch count since timing was last enabled.  Errors: QL_EINVAL. */
int ql_set_timing(ql_solver *s, int32_t enable);
int ql_kernel_time(const ql_solver *s, int32_t which, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* QLSKUM_H */
