// Internal interface between the host runtime and the HIP kernels of the
// q-LSKUM solver.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ql {

constexpr int kBlock = 256;  // threads per workgroup for every point sweep
constexpr int kXcd = 8;      // MI355X accelerator complex dies

enum Kind : uint8_t { kInterior = 0, kWall = 1, kOuter = 2 };
enum Split : uint8_t { kSPlus = 1, kSMinus = 2, kNPlus = 4, kNMinus = 8 };
enum ErrCode : int { kErrNone = 0, kErrSingular = 1, kErrPositivity = 2, kErrNonFinite = 3 };

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
    const double *dmin;  // [n] distance to the nearest neighbour
    // LDS tiling: tile t = points [t*kBlock, (t+1)*kBlock); its halo (the
    // neighbours outside the tile) is halo_idx[halo_ptr[t] .. halo_ptr[t+1]);
    // lidx[k] is neighbour entry k's slot in the tile's LDS image (own point
    // j -> j, halo point h -> kBlock + h).  max_slots = largest image.
    const int *halo_ptr;
    const int *halo_idx;
    const uint16_t *lidx;
    int max_slots;
};

struct FlowParams {
    double gamma, gm1inv, cfl, venkat_k;
    int n_inner, limiter;
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

// Error word on the device: err[0] = smallest failing point (INT_MAX when
// none), err[1] = ErrCode of some failing point.
int num_blocks(int n);

hipError_t launch_setup(hipStream_t st, int n, const double2 *xy, const double2 *nrm,
                        const uint8_t *kind, const int *ptr, const int *idx, uint8_t *flag,
                        int classify, double *lsw, double *dmin, int *err);
hipError_t launch_freestream(hipStream_t st, int n, const double2 *nrm, const uint8_t *kind,
                             const double *Uinf, double *U);
hipError_t launch_permute_state(hipStream_t st, int n, const double *Uuser, const int *perm,
                                const double2 *nrm, const uint8_t *kind, int project, double *U);
hipError_t launch_unpermute_state(hipStream_t st, int n, const double *U, const int *perm,
                                  double *Uuser);
hipError_t launch_prep(hipStream_t st, const DevCloud &c, const FlowParams &fp, const double *U,
                       double *Un, double2 *q, double *dt, float4 *q32, int *err);
hipError_t launch_grad0(hipStream_t st, const DevCloud &c, const double2 *q, double2 *g,
                        double2 *qmm, int want_bounds, Shadow sh);
hipError_t launch_gradk(hipStream_t st, const DevCloud &c, const double2 *q, const double2 *gprev,
                        double2 *gnext, float4 *g32);
// LDS-tiled variants (used when the tile images fit); the inner iteration
// takes the first-pass derivatives g0 instead of q.
bool lds_fits_grad0(const DevCloud &c);
bool lds_fits_gradk(const DevCloud &c);
hipError_t launch_grad0_lds(hipStream_t st, const DevCloud &c, const double2 *q, double2 *g,
                            double2 *qmm, int want_bounds, Shadow sh);
hipError_t launch_gradk_lds(hipStream_t st, const DevCloud &c, const double2 *g0,
                            const double2 *gprev, double2 *gnext, float4 *g32);
// stage 0: evaluate only (writes Rout); stages 1..4: residual + SSP-RK stage.
// q32next (nullable) receives the FP32 shadow of the new q.
hipError_t launch_flux(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                       const double2 *q, const double2 *g, const double2 *qmm, double *U,
                       double *Un, double *dt, double2 *qnext, double *Rout, double *partial,
                       float4 *q32next, int *err);
// mixed precision: reconstruction, limiter and split fluxes in FP32 from the
// shadows q32, g32, qmm32; weights, residual sums and the update in FP64.
hipError_t launch_flux_mixed(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                             const double2 *q, const float4 *q32, const float4 *g32,
                             const float4 *qmm32, double *U, double *Un, double *dt,
                             double2 *qnext, float4 *q32next, double *Rout, double *partial,
                             int *err);
hipError_t launch_resnorm(hipStream_t st, int nblk, const double *partial, double inv_nupd,
                          double *out);
hipError_t launch_forces(hipStream_t st, int nw, const int *wall, const double2 *xy,
                         const double2 *nrm, const double *U, int n, double gamma, double pinf,
                         double *scratch, double *out);

}  // namespace ql
