// Internal interface between the host runtime and the HIP kernels of the
// q-LSKUM solver.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ql {

constexpr int kBlock = 256;  // threads per workgroup for every point sweep
constexpr int kXcd = 8;      // MI355X accelerator complex dies
// flux sweep: kFluxTile points per workgroup, kFluxLanes lanes per point
constexpr int kFluxTile = 64;
constexpr int kFluxLanes = kBlock / kFluxTile;
static_assert(kFluxTile * kFluxLanes == kBlock, "flux tile must fill a workgroup");

enum Kind : uint8_t { kInterior = 0, kWall = 1, kOuter = 2 };
enum Split : uint8_t { kSPlus = 1, kSMinus = 2, kNPlus = 4, kNMinus = 8 };
enum ErrCode : int { kErrNone = 0, kErrSingular = 1, kErrPositivity = 2, kErrNonFinite = 3 };

// Device error word: (p << 8) | code of the smallest failing point p, set by
// atomicMin; kErrClear when no point failed.
using ErrWord = unsigned long long;
constexpr ErrWord kErrClear = ~0ull;
inline int err_point(ErrWord w) { return w == kErrClear ? -1 : (int)(w >> 8); }
inline int err_code(ErrWord w) { return w == kErrClear ? kErrNone : (int)(w & 0xff); }

// a batched case whose residual norm exceeds this multiple of its reference
// norm has diverged
constexpr double kDiverged = 1e8;

// Point cloud on the device, in the library's (reordered) point order.
struct DevCloud {
    int n;
    const double2 *xy;   // [n] positions
    const double2 *nrm;  // [n] unit normals (frame: s along (n_y, -n_x))
    const uint8_t *kind; // [n]
    const int *ptr;      // [n+1]
    const int *idx;      // [nnz]
    const uint8_t *flag; // [nnz] split membership
    const double *lsw;   // [n][8] split least-squares factors, 2 per stencil
    const double *lsi;   // [n][3] full-stencil LS inverse (Syy, Sxy, Sxx) / Det
    const double *dmin;  // [n] distance to the nearest neighbour
    // LDS tiling of the point sweeps: tile t = points [t*kFluxTile,
    // (t+1)*kFluxTile); its halo (the neighbours outside the tile) is
    // fhalo_idx[fhalo_ptr[t] .. fhalo_ptr[t+1]); flidx[k] is neighbour entry
    // k's slot in the tile's LDS image (own point j -> j, halo point h ->
    // kFluxTile + h); fmax_slots = the largest image.  fhalo_ptr is null when
    // the cloud has no tiling: every tile reads from memory.
    const int *fhalo_ptr;
    const int *fhalo_idx;
    const uint16_t *flidx;
    int fmax_slots;
    // batched cases: case_of[p]; case_active[c] == 0 freezes case c (nullable:
    // all active); tile_active[t] == 0 skips (64-point) tile t in every
    // tiled sweep (nullable)
    const int *case_of;
    const uint8_t *case_active;
    const uint8_t *tile_active;
    // batched runs: error word of each case [ncase] (nullable)
    ErrWord *case_err;
    // split fluxes of tile t in FP32 (1) or FP64 (0) when a mixed-precision
    // run moves cases to FP64 fluxes: the FP64 and the mixed flux kernels
    // each take only their tiles (null: one kernel takes every tile)
    const uint8_t *tile_prec;
    // conserved freestream of each case [ncase][4] (the kinetic outer
    // condition's far-field Maxwellian)
    const double *uinf;
    // batched runs after retirements: the tiled sweeps launch one workgroup
    // per entry of tile_list[ntile_live] (the tiles that still hold an
    // active case, in tile order) instead of one per tile (null: every tile)
    const int *tile_list;
    int ntile_live;
};

struct FlowParams {
    double gamma, gm1inv, cfl, venkat_k;
    int n_inner, limiter;
    int order;  // 2: modified q of eq. (28); 1: first order (q~ = q)
    // 1: kinetic outer condition (outer points updated; their n- stencil is
    // the mirror image of n+ holding the freestream); 0: outer points held
    int kobc;
    // m = 2/(gamma-1) when it is a small integer (5 for gamma = 1.4), so that
    // beta^(-1/(gamma-1)) = (1/sqrt(beta))^m needs no logarithm; 0 otherwise
    int sqrt_pow;
};

// FP32 shadow copies read by the mixed-precision flux kernel (all nullable):
// q32 [n] (q), g32 [n][2] (q_x, q_y), qmm32 [n][2] (qmax, qmin).
struct Shadow {
    float4 *q32;
    float4 *g32;
    float4 *qmm32;
};

// Retirement of batched cases, applied on the device after every
// iteration's residual norms (on = 0: plain iterations).  A case stops
// (active[c] = 0) at the iteration whose norm is <= *drop * ref[c] (ref[c] < 0
// takes the case's first norm), whose norm exceeds kDiverged * ref[c] or is
// not a number, or in which one of its points failed (case_err[c] set);
// iters[c] counts the iterations it ran, last[c][4] holds their last norms.
struct Retire {
    int on;
    const double *drop;
    double *ref;
    int *iters;
    double *last;
    uint8_t *active;
    const ErrWord *case_err;
    // precision switch (nullable): a case with prec[c] = 1 (FP32 fluxes)
    // whose norm is <= *sw * ref[c] gets prec[c] = 0 and sw_iter[c] = the
    // iteration; the tiles holding it then run FP64 fluxes
    const double *sw;
    uint8_t *prec;
    int *sw_iter;
};

int num_blocks(int n);
int num_flux_tiles(int n);
// workgroups of a tiled sweep: one per tile, or per listed tile
int sweep_grid(const DevCloud &c);

// err_outer receives singular split stencils of outer points (used only by
// the kinetic outer condition), err every other singular matrix.
hipError_t launch_setup(hipStream_t st, int n, const double2 *xy, const double2 *nrm,
                        const uint8_t *kind, const int *ptr, const int *idx, uint8_t *flag,
                        int classify, double *lsw, double *lsi, double *dmin, ErrWord *err,
                        ErrWord *err_outer);
hipError_t launch_freestream(hipStream_t st, int n, const double2 *nrm, const uint8_t *kind,
                             const int *case_of, const double *uinf, double *U);
hipError_t launch_permute_state(hipStream_t st, int n, const double *Uuser, const int *perm,
                                const double2 *nrm, const uint8_t *kind, int project, double *U);
hipError_t launch_unpermute_state(hipStream_t st, int n, const double *U, const int *perm,
                                  double *Uuser);
hipError_t launch_prep(hipStream_t st, const DevCloud &c, const FlowParams &fp, const double *U,
                       double *Un, double2 *q, double *dt, float4 *q32, ErrWord *err);
// q-derivatives (tiled like the flux sweep; lds_budget as there, 0 for the
// default): first pass with the limiter bounds (qmm: qmax - q and qmin - q
// per point), and one inner iteration from the first pass g0 and the
// previous iterate gprev.  gnext may be null when only the FP32 shadow
// (g32) is wanted, and qmm when only the bounds' FP32 shadow (sh.qmm32) is.
hipError_t launch_grad0(hipStream_t st, const DevCloud &c, int lds_budget, const double2 *q,
                        double2 *g, double2 *qmm, int want_bounds, Shadow sh);
hipError_t launch_gradk(hipStream_t st, const DevCloud &c, int lds_budget, const double2 *g0,
                        const double2 *gprev, double2 *gnext, float4 *g32);
// mixed precision: the same sweeps gathering FP32 data (q32 for the first
// pass, the previous FP32 iterate for an inner iteration) with FP64
// positions, differences, sums and solves; FP32 results ([n][2] float4:
// q_x[0..3], q_y[0..3]; bound offsets qmax - q, qmin - q)
hipError_t launch_grad0_f(hipStream_t st, const DevCloud &c, int lds_budget, const float4 *q32,
                          float4 *g0f, float4 *qmm32, int want_bounds);
hipError_t launch_gradk_f(hipStream_t st, const DevCloud &c, int lds_budget, const float4 *g0f,
                          const float4 *gprev, float4 *gnext);
// stage 0: evaluate only (writes Rout); stages 1..4: residual + SSP-RK stage.
// q32next (nullable) receives the FP32 shadow of the new q.  lds_budget =
// bytes of LDS a workgroup may stage its tile image in (tiles with larger
// images read from memory).  split: 0 one fused launch; 2 an s-direction
// launch and an n-direction + update launch; 4 one launch per split stencil
// (s+, s-, n+, n- + update).  Rpart: two [4][n] buffers of partial sums
// (split > 0 only).
hipError_t launch_flux(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                       int lds_budget, const double2 *q, const double2 *g, const double2 *qmm,
                       double *U, double *Un, double *dt, double2 *qnext, double *Rout,
                       float4 *q32next, ErrWord *err, int split, double *const Rpart[2]);
// mixed precision: reconstruction, limiter and split fluxes in FP32 from the
// shadows q32, g32, qmm32; weights, residual sums and the update in FP64.
hipError_t launch_flux_mixed(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                             int lds_budget, const double2 *q, const float4 *q32,
                             const float4 *g32, const float4 *qmm32, double *U, double *Un,
                             double *dt, double2 *qnext, float4 *q32next, double *Rout,
                             ErrWord *err);
// warm start: de-standardisation of the network's (rho, u1, u2, p) and the
// lower bound of rho and p relative to the freestream
struct WarmScale {
    float mean[4], std[4];
    double floor;
};
hipError_t launch_warm_state(hipStream_t st, int n, const int *perm, const uint8_t *kind,
                             const double2 *nrm, const int *case_of, const double *uinf,
                             const float *Y, const WarmScale &sc, double gamma, double *U);
hipError_t launch_select_state(hipStream_t st, int n, const int *case_of, const uint8_t *sel,
                               const double *Uw, double *U);
hipError_t launch_wall_distance(hipStream_t st, int n, const double2 *xy, const int *case_of,
                                const int *wall_lo, const int *wall, double *d);
// residual norms per case into history row *ctr (then *ctr += 1); with
// rt.on, the retirement of cases and the tile activity (and, with rt.prec,
// the tile precision) that follows from it
hipError_t launch_resnorm(hipStream_t st, const double *R, int n, int nchunk, const int *chunk_beg,
                          double *part, int ncase, const int *chunk_ptr, const double *inv_nupd,
                          int *ctr, int cap, double *hist, const Retire &rt,
                          const int *case_of, uint8_t *tile_active, uint8_t *tile_prec);
// Fixed device array (kScratchDoubles doubles, per GPU) that holds the
// residual history of ql_step_static; scratch_address returns its address
// on the current device.
constexpr int kScratchDoubles = 1 << 16;
hipError_t scratch_address(double **ptr);

hipError_t launch_forces(hipStream_t st, int nw, const int *wall, const double2 *xy,
                         const double2 *nrm, const double *U, int n, double gamma, double pinf,
                         double *scratch, double *out);

}  // namespace ql
