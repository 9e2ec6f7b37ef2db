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
};

struct FlowParams {
    double gamma, gm1inv, cfl, venkat_k;
    int n_inner, limiter;
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
                       double *Un, double2 *q, double *dt, int *err);
hipError_t launch_grad0(hipStream_t st, const DevCloud &c, const double2 *q, double2 *g,
                        double2 *qmm, int want_bounds);
hipError_t launch_gradk(hipStream_t st, const DevCloud &c, const double2 *q, const double2 *gprev,
                        double2 *gnext);
// stage 0: evaluate only (writes Rout); stages 1..4: residual + SSP-RK stage.
hipError_t launch_flux(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                       const double2 *q, const double2 *g, const double2 *qmm, double *U,
                       double *Un, double *dt, double2 *qnext, double *Rout, double *partial,
                       int *err);
hipError_t launch_resnorm(hipStream_t st, int nblk, const double *partial, double inv_nupd,
                          double *out);
hipError_t launch_forces(hipStream_t st, int nw, const int *wall, const double2 *xy,
                         const double2 *nrm, const double *U, int n, double gamma, double pinf,
                         double *scratch, double *out);

}  // namespace ql
