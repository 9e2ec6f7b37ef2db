// HIP kernels of the q-LSKUM pseudo-time iteration for gfx950 (MI355X).
//
// One work-item per point; points are stored in a locality-preserving
// (Hilbert) order so the neighbour gathers of a workgroup touch a compact
// set of cache lines, and workgroups are remapped so that each of the eight
// XCDs (each with its own L2) walks a contiguous range of points.
//
// Layouts (library order): conserved state U, Un and the residual R are
// component-major U[c*n + p] (coalesced streaming); the gathered per-point
// records are interleaved so that one neighbour costs few 16-byte loads:
// q [n][4], g [n][8] (q_x 0..3, q_y 4..7), limiter bounds [n][8]
// (qmax 0..3, qmin 4..7).
//
// Equations (paper: "On the performance of GPU accelerated q-LSKUM based
// meshfree solvers in Fortran, C++, Python, and Julia", 2021):
//   q-variables              sec. 2.1 eq. (26)
//   q-derivatives            eq. (11) first pass, eq. (29) inner iterations
//   modified q               eq. (28), split fluxes of eq. (27)
//   split-flux derivatives   eqs. (12)-(14)
//   iteration                sec. 3 Algorithm 1
#include "qlskum_internal.h"

#include <climits>
#include <cmath>

namespace ql {

namespace {

// Workgroups are dispatched to the XCDs round-robin; remap the hardware
// workgroup id so that XCD x processes one contiguous slice of the grid.
__device__ __forceinline__ int logical_block() {
    const int nblk = gridDim.x;
    const int b = blockIdx.x;
    const int q = nblk / kXcd, r = nblk % kXcd;
    const int x = b % kXcd, k = b / kXcd;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int point_id() { return logical_block() * kBlock + threadIdx.x; }

__device__ __forceinline__ void report(int *err, int p, int code) {
    atomicMin(&err[0], p);
    atomicExch(&err[1], code);
}

__device__ __forceinline__ void load4(const double2 *a, int p, double v[4]) {
    double2 x0 = a[2 * p], x1 = a[2 * p + 1];
    v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
}

__device__ __forceinline__ void load8(const double2 *a, int p, double v[8]) {
    double2 x0 = a[4 * p], x1 = a[4 * p + 1], x2 = a[4 * p + 2], x3 = a[4 * p + 3];
    v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
    v[4] = x2.x; v[5] = x2.y; v[6] = x3.x; v[7] = x3.y;
}

__device__ __forceinline__ void store4(double2 *a, int p, const double v[4]) {
    a[2 * p] = make_double2(v[0], v[1]);
    a[2 * p + 1] = make_double2(v[2], v[3]);
}

__device__ __forceinline__ void store8(double2 *a, int p, const double v[8]) {
    a[4 * p] = make_double2(v[0], v[1]);
    a[4 * p + 1] = make_double2(v[2], v[3]);
    a[4 * p + 2] = make_double2(v[4], v[5]);
    a[4 * p + 3] = make_double2(v[6], v[7]);
}

__device__ __forceinline__ float4 to_f4(const double v[4]) {
    return make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}

// U -> q (eq. (26)); returns an ErrCode.
__device__ __forceinline__ int cons_to_q(const double U[4], const FlowParams &fp, double q[4]) {
    if (!isfinite(U[0]) || !isfinite(U[1]) || !isfinite(U[2]) || !isfinite(U[3]))
        return kErrNonFinite;
    const double rho = U[0];
    const double u1 = U[1] / rho, u2 = U[2] / rho;
    const double uu = u1 * u1 + u2 * u2;
    const double p = (fp.gamma - 1.0) * (U[3] - 0.5 * rho * uu);
    if (!(rho > 0.0) || !(p > 0.0)) return kErrPositivity;
    const double beta = rho / (2.0 * p);
    q[0] = log(rho) + log(beta) * fp.gm1inv - beta * uu;
    q[1] = 2.0 * beta * u1;
    q[2] = 2.0 * beta * u2;
    q[3] = -2.0 * beta;
    return kErrNone;
}

__device__ __forceinline__ double local_dt(const double U[4], double dmin, const FlowParams &fp) {
    const double rho = U[0];
    const double u1 = U[1] / rho, u2 = U[2] / rho;
    const double uu = u1 * u1 + u2 * u2;
    const double p = (fp.gamma - 1.0) * (U[3] - 0.5 * rho * uu);
    return fp.cfl * dmin / (sqrt(uu) + sqrt(fp.gamma * p / rho));
}

}  // namespace

int num_blocks(int n) { return (n + kBlock - 1) / kBlock; }

// ---------------------------------------------------------------------------
// Cloud set-up: split membership of every neighbour entry (eq. (14) in the
// point's (s, n) frame), nearest-neighbour distance, and the least-squares
// factors of the four split stencils.  The split-flux derivative of eq. (13)
// over stencil b is linear in the perturbations dG_i:
//   dG/ds = sum_i (ds_i Snn - dn_i Ssn)/Det * dG_i     (s stencils)
//   dG/dn = sum_i (dn_i Sss - ds_i Ssn)/Det * dG_i     (n stencils)
// so two factors per stencil, (Snn/Det, Ssn/Det) or (Sss/Det, Ssn/Det),
// turn the residual into a single weighted sum over the neighbours.
// Classification is evaluated without FMA contraction so that the flags are
// the exact IEEE results of the defining expressions.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_setup(int n, const double2 *__restrict__ xy,
                                                  const double2 *__restrict__ nrm,
                                                  const uint8_t *__restrict__ kind,
                                                  const int *__restrict__ ptr,
                                                  const int *__restrict__ idx, uint8_t *flag,
                                                  int classify, double *__restrict__ lsw,
                                                  double *__restrict__ dmin, int *err) {
#pragma clang fp contract(off)
    const int p = point_id();
    if (p >= n) return;
    const double2 P = xy[p], N = nrm[p];
    const double tx = N.y, ty = -N.x;
    double a = 0.0, b = 0.0, c = 0.0, dm2 = INFINITY;
    double ss[4] = {0, 0, 0, 0}, sn[4] = {0, 0, 0, 0}, nn[4] = {0, 0, 0, 0};
    int cnt[4] = {0, 0, 0, 0};
    const int k0 = ptr[p], k1 = ptr[p + 1];
    for (int k = k0; k < k1; ++k) {
        const double2 Q = xy[idx[k]];
        const double dx = Q.x - P.x, dy = Q.y - P.y;
        const double ds = dx * tx + dy * ty;
        const double dn = dx * N.x + dy * N.y;
        const double d2 = dx * dx + dy * dy;
        uint8_t f;
        if (classify) {
            const double tie = 1e-24 * d2;
            f = 0;
            if (ds * ds > tie) f |= (ds < 0.0) ? kSPlus : kSMinus;
            if (dn * dn > tie) f |= (dn < 0.0) ? kNPlus : kNMinus;
            flag[k] = f;
        } else {
            f = flag[k];
        }
        a += dx * dx;
        b += dx * dy;
        c += dy * dy;
        dm2 = fmin(dm2, d2);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (f & (1u << s)) {
                ss[s] += ds * ds;
                sn[s] += ds * dn;
                nn[s] += dn * dn;
                cnt[s] += 1;
            }
        }
    }
    dmin[p] = sqrt(dm2);
    const double D = a * c - b * b;
    bool bad = !(D > 1e-12 * (a + c) * (a + c)) || (k1 - k0) < 2;
    const uint8_t kd = kind[p];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double det = ss[s] * nn[s] - sn[s] * sn[s];
        const double sc = ss[s] + nn[s];
        const bool used = (kd == kInterior) || (kd == kWall && s != 2);
        double f0 = 0.0, f1 = 0.0;
        if (used) {
            if (cnt[s] < 2 || !(det > 1e-12 * sc * sc)) bad = true;
            f0 = ((s < 2) ? nn[s] : ss[s]) / det;
            f1 = sn[s] / det;
        }
        lsw[8 * p + 2 * s] = f0;
        lsw[8 * p + 2 * s + 1] = f1;
    }
    if (bad) report(err, p, kErrSingular);
}

hipError_t launch_setup(hipStream_t st, int n, const double2 *xy, const double2 *nrm,
                        const uint8_t *kind, const int *ptr, const int *idx, uint8_t *flag,
                        int classify, double *lsw, double *dmin, int *err) {
    hipLaunchKernelGGL(k_setup, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, xy, nrm, kind, ptr,
                       idx, flag, classify, lsw, dmin, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State set-up: freestream, caller-order <-> library-order copies, and the
// wall condition's momentum projection m <- m - (m.n) n (rho, rho e kept).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wall_project(double U[4], double2 N) {
    const double mn = U[1] * N.x + U[2] * N.y;
    U[1] = U[1] - mn * N.x;
    U[2] = U[2] - mn * N.y;
}

__global__ void __launch_bounds__(kBlock) k_freestream(int n, const double2 *__restrict__ nrm,
                                                       const uint8_t *__restrict__ kind,
                                                       double u0, double u1, double u2, double u3,
                                                       double *__restrict__ U) {
    const int p = point_id();
    if (p >= n) return;
    double v[4] = {u0, u1, u2, u3};
    if (kind[p] == kWall) wall_project(v, nrm[p]);
#pragma unroll
    for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
}

hipError_t launch_freestream(hipStream_t st, int n, const double2 *nrm, const uint8_t *kind,
                             const double *Uinf, double *U) {
    hipLaunchKernelGGL(k_freestream, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, nrm, kind,
                       Uinf[0], Uinf[1], Uinf[2], Uinf[3], U);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) k_permute_state(int n, const double *__restrict__ Uu,
                                                          const int *__restrict__ perm,
                                                          const double2 *__restrict__ nrm,
                                                          const uint8_t *__restrict__ kind,
                                                          int project, double *__restrict__ U) {
    const int p = point_id();
    if (p >= n) return;
    const int u = perm[p];
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = Uu[(size_t)c * n + u];
    if (project && kind[p] == kWall) wall_project(v, nrm[p]);
#pragma unroll
    for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
}

hipError_t launch_permute_state(hipStream_t st, int n, const double *Uuser, const int *perm,
                                const double2 *nrm, const uint8_t *kind, int project, double *U) {
    hipLaunchKernelGGL(k_permute_state, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, Uuser, perm,
                       nrm, kind, project, U);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) k_unpermute_state(int n, const double *__restrict__ U,
                                                            const int *__restrict__ perm,
                                                            double *__restrict__ Uu) {
    const int p = point_id();
    if (p >= n) return;
    const int u = perm[p];
#pragma unroll
    for (int c = 0; c < 4; ++c) Uu[(size_t)c * n + u] = U[(size_t)c * n + p];
}

hipError_t launch_unpermute_state(hipStream_t st, int n, const double *U, const int *perm,
                                  double *Uuser) {
    hipLaunchKernelGGL(k_unpermute_state, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, U, perm,
                       Uuser);
    return hipGetLastError();
}

// Start of an iteration from a freshly set state: q (eq. (26)), the local
// time step, and the copy Un of the state the Runge-Kutta stages start from.
__global__ void __launch_bounds__(kBlock) k_prep(DevCloud cl, FlowParams fp,
                                                 const double *__restrict__ U,
                                                 double *__restrict__ Un, double2 *__restrict__ q,
                                                 double *__restrict__ dt, float4 *__restrict__ q32,
                                                 int *err) {
    const int n = cl.n;
    const int p = point_id();
    if (p >= n) return;
    double v[4], qq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = U[(size_t)c * n + p];
    const int e = cons_to_q(v, fp, qq);
    if (e != kErrNone) {
        report(err, p, e);
        qq[0] = qq[1] = qq[2] = 0.0;
        qq[3] = -1.0;
    }
    store4(q, p, qq);
    if (q32) q32[p] = to_f4(qq);
#pragma unroll
    for (int c = 0; c < 4; ++c) Un[(size_t)c * n + p] = v[c];
    dt[p] = local_dt(v, cl.dmin[p], fp);
}

hipError_t launch_prep(hipStream_t st, const DevCloud &c, const FlowParams &fp, const double *U,
                       double *Un, double2 *q, double *dt, float4 *q32, int *err) {
    hipLaunchKernelGGL(k_prep, dim3(num_blocks(c.n)), dim3(kBlock), 0, st, c, fp, U, Un, q, dt,
                       q32, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// q-derivatives, first pass: full-stencil least squares of dq_i = q_i - q_p
// (eq. (11)); also the componentwise max / min of q over the point and its
// stencil (bounds of the limited reconstruction).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_grad0(DevCloud cl, const double2 *__restrict__ q,
                                                  double2 *__restrict__ g,
                                                  double2 *__restrict__ qmm, int want_bounds,
                                                  Shadow sh) {
    const int p = point_id();
    if (p >= cl.n) return;
    const double2 P = cl.xy[p];
    double qp[4];
    load4(q, p, qp);
    double a = 0.0, b = 0.0, c = 0.0;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    double mx[4] = {qp[0], qp[1], qp[2], qp[3]}, mn[4] = {qp[0], qp[1], qp[2], qp[3]};
    const int k1 = cl.ptr[p + 1];
    for (int k = cl.ptr[p]; k < k1; ++k) {
        const int i = cl.idx[k];
        const double2 Q = cl.xy[i];
        const double dx = Q.x - P.x, dy = Q.y - P.y;
        double qi[4];
        load4(q, i, qi);
        a += dx * dx;
        b += dx * dy;
        c += dy * dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dq = qi[r] - qp[r];
            sx[r] += dx * dq;
            sy[r] += dy * dq;
            mx[r] = fmax(mx[r], qi[r]);
            mn[r] = fmin(mn[r], qi[r]);
        }
    }
    const double D = a * c - b * b;
    double gv[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gv[r] = (c * sx[r] - b * sy[r]) / D;
        gv[4 + r] = (a * sy[r] - b * sx[r]) / D;
    }
    store8(g, p, gv);
    if (sh.g32) {
        sh.g32[2 * p] = to_f4(gv);
        sh.g32[2 * p + 1] = to_f4(gv + 4);
    }
    if (want_bounds) {
        double bv[8] = {mx[0], mx[1], mx[2], mx[3], mn[0], mn[1], mn[2], mn[3]};
        store8(qmm, p, bv);
        if (sh.qmm32) {
            sh.qmm32[2 * p] = to_f4(bv);
            sh.qmm32[2 * p + 1] = to_f4(bv + 4);
        }
    }
}

hipError_t launch_grad0(hipStream_t st, const DevCloud &c, const double2 *q, double2 *g,
                        double2 *qmm, int want_bounds, Shadow sh) {
    hipLaunchKernelGGL(k_grad0, dim3(num_blocks(c.n)), dim3(kBlock), 0, st, c, q, g, qmm,
                       want_bounds, sh);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// q-derivatives, one inner iteration (eq. (29)): least squares of
//   dq~_i = dq_i - 1/2 [dx (q_x,i - q_x,p) + dy (q_y,i - q_y,p)]
// from the previous iterate (Jacobi: read gprev, write gnext).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_gradk(DevCloud cl, const double2 *__restrict__ q,
                                                  const double2 *__restrict__ gprev,
                                                  double2 *__restrict__ gnext,
                                                  float4 *__restrict__ g32) {
    const int p = point_id();
    if (p >= cl.n) return;
    const double2 P = cl.xy[p];
    double qp[4], gp[8];
    load4(q, p, qp);
    load8(gprev, p, gp);
    double a = 0.0, b = 0.0, c = 0.0;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    const int k1 = cl.ptr[p + 1];
    for (int k = cl.ptr[p]; k < k1; ++k) {
        const int i = cl.idx[k];
        const double2 Q = cl.xy[i];
        const double dx = Q.x - P.x, dy = Q.y - P.y;
        double qi[4], gi[8];
        load4(q, i, qi);
        load8(gprev, i, gi);
        a += dx * dx;
        b += dx * dy;
        c += dy * dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dq = (qi[r] - qp[r]) -
                              0.5 * (dx * (gi[r] - gp[r]) + dy * (gi[4 + r] - gp[4 + r]));
            sx[r] += dx * dq;
            sy[r] += dy * dq;
        }
    }
    const double D = a * c - b * b;
    double gv[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gv[r] = (c * sx[r] - b * sy[r]) / D;
        gv[4 + r] = (a * sy[r] - b * sx[r]) / D;
    }
    store8(gnext, p, gv);
    if (g32) {
        g32[2 * p] = to_f4(gv);
        g32[2 * p + 1] = to_f4(gv + 4);
    }
}

hipError_t launch_gradk(hipStream_t st, const DevCloud &c, const double2 *q, const double2 *gprev,
                        double2 *gnext, float4 *g32) {
    hipLaunchKernelGGL(k_gradk, dim3(num_blocks(c.n)), dim3(kBlock), 0, st, c, q, gprev, gnext,
                       g32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LDS-tiled q-derivatives.  A workgroup owns a tile of kBlock consecutive
// points (a compact patch in Hilbert order); it first copies the records of
// its points and of their neighbours outside the tile (the halo) into LDS,
// then every lane walks its neighbour list through 16-bit slot indices.
// Each record is read from memory once per tile instead of once per use.
// ---------------------------------------------------------------------------
// Tiles whose image exceeds the budget read their neighbours straight from
// memory (a branch that is uniform across the workgroup).
constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per workgroup at most
constexpr int kCap0 = kLdsBudget / 48;  // slots of the first-pass image
constexpr int kCapK = kLdsBudget / 80;  // slots of the inner-iteration image

bool lds_fits_grad0(const DevCloud &c) { return c.max_slots < (1 << 30); }
bool lds_fits_gradk(const DevCloud &c) { return c.max_slots < (1 << 30); }

// first pass: slot record = (q0,q1) (q2,q3) (x,y)
__global__ void __launch_bounds__(kBlock) k_grad0_lds(DevCloud cl, const double2 *__restrict__ q,
                                                      double2 *__restrict__ g,
                                                      double2 *__restrict__ qmm,
                                                      int want_bounds, Shadow sh) {
    extern __shared__ double2 lds[];
    const int n = cl.n;
    const int t = logical_block();
    const int base = t * kBlock;
    const int h0 = cl.halo_ptr[t], nh = cl.halo_ptr[t + 1] - h0;
    const int nown = min(kBlock, n - base);
    const bool in_lds = kBlock + nh <= kCap0;
    if (in_lds) {
        for (int s = threadIdx.x; s < kBlock + nh; s += kBlock) {
            int pt;
            if (s < kBlock) {
                if (s >= nown) continue;
                pt = base + s;
            } else {
                pt = cl.halo_idx[h0 + s - kBlock];
            }
            lds[3 * s] = q[2 * pt];
            lds[3 * s + 1] = q[2 * pt + 1];
            lds[3 * s + 2] = cl.xy[pt];
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j >= nown) return;
    const int p = base + j;
    const double2 q01 = q[2 * p], q23 = q[2 * p + 1], P = cl.xy[p];
    const double qp[4] = {q01.x, q01.y, q23.x, q23.y};
    double a = 0.0, b = 0.0, c = 0.0;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    double mx[4] = {qp[0], qp[1], qp[2], qp[3]}, mn[4] = {qp[0], qp[1], qp[2], qp[3]};
    const int k1 = cl.ptr[p + 1];
    for (int k = cl.ptr[p]; k < k1; ++k) {
        double2 a01, a23, Q;
        if (in_lds) {
            const int li = cl.lidx[k];
            a01 = lds[3 * li];
            a23 = lds[3 * li + 1];
            Q = lds[3 * li + 2];
        } else {
            const int i = cl.idx[k];
            a01 = q[2 * i];
            a23 = q[2 * i + 1];
            Q = cl.xy[i];
        }
        const double qi[4] = {a01.x, a01.y, a23.x, a23.y};
        const double dx = Q.x - P.x, dy = Q.y - P.y;
        a += dx * dx;
        b += dx * dy;
        c += dy * dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dq = qi[r] - qp[r];
            sx[r] += dx * dq;
            sy[r] += dy * dq;
            mx[r] = fmax(mx[r], qi[r]);
            mn[r] = fmin(mn[r], qi[r]);
        }
    }
    const double D = a * c - b * b;
    double gv[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gv[r] = (c * sx[r] - b * sy[r]) / D;
        gv[4 + r] = (a * sy[r] - b * sx[r]) / D;
    }
    store8(g, p, gv);
    if (sh.g32) {
        sh.g32[2 * p] = to_f4(gv);
        sh.g32[2 * p + 1] = to_f4(gv + 4);
    }
    if (want_bounds) {
        double bv[8] = {mx[0], mx[1], mx[2], mx[3], mn[0], mn[1], mn[2], mn[3]};
        store8(qmm, p, bv);
        if (sh.qmm32) {
            sh.qmm32[2 * p] = to_f4(bv);
            sh.qmm32[2 * p + 1] = to_f4(bv + 4);
        }
    }
}

hipError_t launch_grad0_lds(hipStream_t st, const DevCloud &c, const double2 *q, double2 *g,
                            double2 *qmm, int want_bounds, Shadow sh) {
    const size_t shmem = (size_t)min(c.max_slots, kCap0) * 48;
    hipLaunchKernelGGL(k_grad0_lds, dim3(num_blocks(c.n)), dim3(kBlock), shmem, st, c, q, g, qmm,
                       want_bounds, sh);
    return hipGetLastError();
}

// inner iteration: the least squares of eq. (29) is linear in its data, so
//   g^k = LS(dq_i) - 1/2 LS(d.(g^{k-1}_i - g^{k-1}_p)) = g0 - 1/2 LS(...)
// and only the previous iterate is gathered.  slot record = g (4 x double2)
// and (x, y).
__global__ void __launch_bounds__(kBlock) k_gradk_lds(DevCloud cl, const double2 *__restrict__ g0,
                                                      const double2 *__restrict__ gprev,
                                                      double2 *__restrict__ gnext,
                                                      float4 *__restrict__ g32) {
    extern __shared__ double2 lds[];
    const int n = cl.n;
    const int t = logical_block();
    const int base = t * kBlock;
    const int h0 = cl.halo_ptr[t], nh = cl.halo_ptr[t + 1] - h0;
    const int nown = min(kBlock, n - base);
    const bool in_lds = kBlock + nh <= kCapK;
    if (in_lds) {
        for (int s = threadIdx.x; s < kBlock + nh; s += kBlock) {
            int pt;
            if (s < kBlock) {
                if (s >= nown) continue;
                pt = base + s;
            } else {
                pt = cl.halo_idx[h0 + s - kBlock];
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) lds[5 * s + m] = gprev[4 * pt + m];
            lds[5 * s + 4] = cl.xy[pt];
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j >= nown) return;
    const int p = base + j;
    double gp[8];
    load8(gprev, p, gp);
    const double2 P = cl.xy[p];
    double a = 0.0, b = 0.0, c = 0.0;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    const int k1 = cl.ptr[p + 1];
    for (int k = cl.ptr[p]; k < k1; ++k) {
        double gi[8];
        double2 Q;
        if (in_lds) {
            const int li = cl.lidx[k];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double2 v = lds[5 * li + m];
                gi[2 * m] = v.x;
                gi[2 * m + 1] = v.y;
            }
            Q = lds[5 * li + 4];
        } else {
            const int i = cl.idx[k];
            load8(gprev, i, gi);
            Q = cl.xy[i];
        }
        const double dx = Q.x - P.x, dy = Q.y - P.y;
        a += dx * dx;
        b += dx * dy;
        c += dy * dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double f = dx * (gi[r] - gp[r]) + dy * (gi[4 + r] - gp[4 + r]);
            sx[r] += dx * f;
            sy[r] += dy * f;
        }
    }
    const double D = a * c - b * b;
    double gz[8], gv[8];
    load8(g0, p, gz);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gv[r] = gz[r] - 0.5 * ((c * sx[r] - b * sy[r]) / D);
        gv[4 + r] = gz[4 + r] - 0.5 * ((a * sy[r] - b * sx[r]) / D);
    }
    store8(gnext, p, gv);
    if (g32) {
        g32[2 * p] = to_f4(gv);
        g32[2 * p + 1] = to_f4(gv + 4);
    }
}

hipError_t launch_gradk_lds(hipStream_t st, const DevCloud &c, const double2 *g0,
                            const double2 *gprev, double2 *gnext, float4 *g32) {
    const size_t shmem = (size_t)min(c.max_slots, kCapK) * 80;
    hipLaunchKernelGGL(k_gradk_lds, dim3(num_blocks(c.n)), dim3(kBlock), shmem, st, c, g0, gprev,
                       gnext, g32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flux residual + Runge-Kutta stage.
// ---------------------------------------------------------------------------
namespace {

struct Prim {
    double rho, u1, u2, p, sqb, isqb, rhoe;
};

// q~ -> primitive state (inverse of eq. (26)); false if q4 >= 0 or the
// result is not finite (the Maxwellian of q~ does not exist).  One division
// (1/(2 beta)), one square root and one exponential: 1/sqrt(beta) =
// 2 sqrt(beta) / (2 beta), and beta^(-1/(gamma-1)) = (1/sqrt(beta))^m.
// The per-state formulas below are written with explicit fma and no implicit
// contraction, so that two reconstructed states that are bitwise equal give
// bitwise equal fluxes (uniform flow keeps R = 0 exactly).
template <int POW>
__device__ __forceinline__ bool q_to_prim(const double qt[4], const FlowParams &fp, Prim &s) {
#pragma clang fp contract(off)
    const double beta = -0.5 * qt[3];
    const double inv2b = -1.0 / qt[3];
    s.u1 = qt[1] * inv2b;
    s.u2 = qt[2] * inv2b;
    const double uu = fma(s.u1, s.u1, s.u2 * s.u2);
    s.sqb = sqrt(beta);
    s.isqb = (2.0 * s.sqb) * inv2b;
    if (POW > 0) {
        double pw = s.isqb;
#pragma unroll
        for (int j = 1; j < POW; ++j) pw *= s.isqb;
        s.rho = exp(fma(beta, uu, qt[0])) * pw;
    } else {
        s.rho = exp(fma(beta, uu, fma(-log(beta), fp.gm1inv, qt[0])));
    }
    s.p = s.rho * inv2b;
    s.rhoe = fma(s.p, fp.gm1inv, (0.5 * s.rho) * uu);
    return (qt[3] < 0.0) && isfinite(s.rho) && isfinite(s.p) && isfinite(s.u1) &&
           isfinite(s.u2);
}

// Kinetic split flux along the unit direction e; sg = +1 for G+, -1 for G-.
// Half-range moments of the Maxwellian: with S = u_e sqrt(beta),
// A = erfc(-sg S)/2 and B = exp(-S^2)/(2 sqrt(pi beta)),
//   G = [rho(u_e A + sg B), rho u (u_e A + sg B) + p A e,
//        (p + rho e) u_e A + sg (p/2 + rho e) B].
__device__ __forceinline__ void split_flux(const Prim &s, double ex, double ey, double sg,
                                           double G[4]) {
#pragma clang fp contract(off)
    constexpr double kHalfRsqrtPi = 0.28209479177387814347;  // 1 / (2 sqrt(pi))
    const double ue = fma(s.u1, ex, s.u2 * ey);
    const double S = ue * s.sqb;
    const double A = 0.5 * erfc(-sg * S);
    const double B = (exp(-(S * S)) * kHalfRsqrtPi) * s.isqb;
    const double sB = sg * B;
    const double mass = s.rho * fma(ue, A, sB);
    const double pA = s.p * A;
    G[0] = mass;
    G[1] = fma(s.u1, mass, pA * ex);
    G[2] = fma(s.u2, mass, pA * ey);
    G[3] = fma((s.p + s.rhoe) * ue, A, (fma(0.5, s.p, s.rhoe)) * sB);
}

// Venkatakrishnan limiter value for the increment delta of one component.
__device__ __forceinline__ double venkat(double delta, double q, double qmx, double qmn,
                                         double eps2) {
    const double D = (delta > 0.0) ? (qmx - q) : (qmn - q);
    const double num = (D * D + eps2) + 2.0 * delta * D;
    const double den = D * D + 2.0 * delta * delta + delta * D + eps2;
    return (den == 0.0) ? 1.0 : num / den;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

// stage 0: evaluate R only.  stage 1..4: SSP-RK(4,3) stage with L = -R:
//   U1 = Un + dt/2 L(Un); U2 = U1 + dt/2 L(U1);
//   U3 = 2/3 Un + 1/3 (U2 + dt/2 L(U2)); U4 = U3 + dt/2 L(U3);
// then the wall projection, q of the new state into qnext, and at stage 4
// the next iteration's Un and time step.  Stage 1 also writes one partial
// sum of R_c^2 per workgroup (residual norm).
template <bool LIMITER, int POW>
__global__ void __launch_bounds__(kBlock) k_flux(DevCloud cl, FlowParams fp, int stage,
                                                 const double2 *__restrict__ q,
                                                 const double2 *__restrict__ g,
                                                 const double2 *__restrict__ qmm,
                                                 double *__restrict__ U, double *__restrict__ Un,
                                                 double *__restrict__ dt,
                                                 double2 *__restrict__ qnext,
                                                 double *__restrict__ Rout,
                                                 double *__restrict__ partial,
                                                 float4 *__restrict__ q32next, int *err) {
    const int n = cl.n;
    const int p = point_id();
    double R[4] = {0.0, 0.0, 0.0, 0.0};
    bool updated = false;
    if (p < n) {
        const uint8_t kd = cl.kind[p];
        double qp[4];
        load4(q, p, qp);
        if (kd == kOuter) {
            if (stage > 0) {  // held at the far-field state
                store4(qnext, p, qp);
                if (q32next) q32next[p] = to_f4(qp);
            }
            if (Rout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = 0.0;
            }
        } else {
            updated = true;
            const double2 P = cl.xy[p], N = cl.nrm[p];
            const double tx = N.y, ty = -N.x;
            double gp[8], bp[8], w[8];
            load8(g, p, gp);
            if (LIMITER) load8(qmm, p, bp);
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = cl.lsw[8 * p + j];
            const uint8_t fmask = (kd == kWall) ? uint8_t(~kNPlus) : uint8_t(0xff);
            const int k1 = cl.ptr[p + 1];
            bool ok = true;
            for (int k = cl.ptr[p]; k < k1; ++k) {
                const uint8_t f = cl.flag[k] & fmask;
                if (f == 0) continue;
                const int i = cl.idx[k];
                const double2 Q = cl.xy[i];
                const double dx = Q.x - P.x, dy = Q.y - P.y;
                const double ds = dx * tx + dy * ty;
                const double dn = dx * N.x + dy * N.y;
                double qi[4], gi[8], qti[4], qt0[4];
                load4(q, i, qi);
                load8(g, i, gi);
                if (LIMITER) {
                    double bi[8];
                    load8(qmm, i, bi);
                    const double e = fp.venkat_k * sqrt(dx * dx + dy * dy);
                    const double eps2 = e * e * e;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double di = -0.5 * (dx * gi[r] + dy * gi[4 + r]);
                        const double d0 = -0.5 * (dx * gp[r] + dy * gp[4 + r]);
                        qti[r] = qi[r] + venkat(di, qi[r], bi[r], bi[4 + r], eps2) * di;
                        qt0[r] = qp[r] + venkat(d0, qp[r], bp[r], bp[4 + r], eps2) * d0;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        qti[r] = qi[r] - 0.5 * (dx * gi[r] + dy * gi[4 + r]);
                        qt0[r] = qp[r] - 0.5 * (dx * gp[r] + dy * gp[4 + r]);
                    }
                }
                Prim si, s0;
                ok &= q_to_prim<POW>(qti, fp, si);
                ok &= q_to_prim<POW>(qt0, fp, s0);
                if (f & (kSPlus | kSMinus)) {
                    const bool plus = (f & kSPlus) != 0;
                    const double sg = plus ? 1.0 : -1.0;
                    const double wa = plus ? w[0] : w[2], wb = plus ? w[1] : w[3];
                    const double wt = ds * wa - dn * wb;
                    double Gi[4], G0[4];
                    split_flux(si, tx, ty, sg, Gi);
                    split_flux(s0, tx, ty, sg, G0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) R[r] += wt * (Gi[r] - G0[r]);
                }
                if (f & (kNPlus | kNMinus)) {
                    const bool plus = (f & kNPlus) != 0;
                    const double sg = plus ? 1.0 : -1.0;
                    const double wa = plus ? w[4] : w[6], wb = plus ? w[5] : w[7];
                    const double wt = dn * wa - ds * wb;
                    double Gi[4], G0[4];
                    split_flux(si, N.x, N.y, sg, Gi);
                    split_flux(s0, N.x, N.y, sg, G0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) R[r] += wt * (Gi[r] - G0[r]);
                }
            }
            if (!ok) report(err, p, kErrPositivity);
            if (Rout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = R[r];
            }
            if (stage > 0) {
                const double h = 0.5 * dt[p];
                double v[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double u = U[(size_t)c * n + p];
                    if (stage == 3)
                        v[c] = (2.0 / 3.0) * Un[(size_t)c * n + p] + (1.0 / 3.0) * (u - h * R[c]);
                    else
                        v[c] = u - h * R[c];
                }
                if (kd == kWall) wall_project(v, N);
#pragma unroll
                for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
                double qq[4];
                const int e = cons_to_q(v, fp, qq);
                if (e != kErrNone) {
                    report(err, p, e);
                    qq[0] = qq[1] = qq[2] = 0.0;
                    qq[3] = -1.0;
                }
                store4(qnext, p, qq);
                if (q32next) q32next[p] = to_f4(qq);
                if (stage == 4) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) Un[(size_t)c * n + p] = v[c];
                    dt[p] = local_dt(v, cl.dmin[p], fp);
                }
            }
        }
    }
    if (partial != nullptr) {
        // deterministic per-workgroup sums of R_c^2 over the updated points
        __shared__ double red[kBlock / 64][4];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double s = wave_sum(updated ? R[c] * R[c] : 0.0);
            if (lane == 0) red[wv][c] = s;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < kBlock / 64; ++j) s += red[j][threadIdx.x];
            partial[4 * logical_block() + threadIdx.x] = s;
        }
    }
}

hipError_t launch_flux(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                       const double2 *q, const double2 *g, const double2 *qmm, double *U,
                       double *Un, double *dt, double2 *qnext, double *Rout, double *partial,
                       float4 *q32next, int *err) {
    const dim3 grid(num_blocks(c.n)), block(kBlock);
#define QL_FLUX_LAUNCH(LIM, POW)                                                               \
    hipLaunchKernelGGL((k_flux<LIM, POW>), grid, block, 0, st, c, fp, stage, q, g, qmm, U, Un, \
                       dt, qnext, Rout, partial, q32next, err)
    if (fp.sqrt_pow == 5) {  // gamma = 1.4
        if (fp.limiter) QL_FLUX_LAUNCH(true, 5);
        else QL_FLUX_LAUNCH(false, 5);
    } else {
        if (fp.limiter) QL_FLUX_LAUNCH(true, 0);
        else QL_FLUX_LAUNCH(false, 0);
    }
#undef QL_FLUX_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mixed precision flux residual + Runge-Kutta stage.  The reconstruction
// (eq. (28)), the limiter and the split fluxes run in FP32 from the FP32
// shadows of q, its derivatives and its bounds, using the hardware FP32
// exp / sqrt / reciprocal; the geometry, the least-squares weights, the
// residual sums and the state update stay FP64.
// ---------------------------------------------------------------------------
namespace {

struct PrimF {
    float rho, u1, u2, p, sqb, isqb, rhoe;
};

template <int POW>
__device__ __forceinline__ bool q_to_prim_f(const float qt[4], float gm1inv, PrimF &s) {
#pragma clang fp contract(off)
    const float beta = -0.5f * qt[3];
    const float inv2b = -1.0f / qt[3];
    s.u1 = qt[1] * inv2b;
    s.u2 = qt[2] * inv2b;
    const float uu = fmaf(s.u1, s.u1, s.u2 * s.u2);
    s.sqb = sqrtf(beta);
    s.isqb = (2.0f * s.sqb) * inv2b;
    if (POW > 0) {
        float pw = s.isqb;
#pragma unroll
        for (int j = 1; j < POW; ++j) pw *= s.isqb;
        s.rho = __expf(fmaf(beta, uu, qt[0])) * pw;
    } else {
        s.rho = __expf(fmaf(beta, uu, fmaf(-__logf(beta), gm1inv, qt[0])));
    }
    s.p = s.rho * inv2b;
    s.rhoe = fmaf(s.p, gm1inv, (0.5f * s.rho) * uu);
    return (qt[3] < 0.0f) && isfinite(s.rho) && isfinite(s.p) && isfinite(s.u1) &&
           isfinite(s.u2);
}

__device__ __forceinline__ void split_flux_f(const PrimF &s, float ex, float ey, float sg,
                                             float G[4]) {
#pragma clang fp contract(off)
    constexpr float kHalfRsqrtPi = 0.28209479177387814347f;
    const float ue = fmaf(s.u1, ex, s.u2 * ey);
    const float S = ue * s.sqb;
    const float A = 0.5f * erfcf(-sg * S);
    const float B = (__expf(-(S * S)) * kHalfRsqrtPi) * s.isqb;
    const float sB = sg * B;
    const float mass = s.rho * fmaf(ue, A, sB);
    const float pA = s.p * A;
    G[0] = mass;
    G[1] = fmaf(s.u1, mass, pA * ex);
    G[2] = fmaf(s.u2, mass, pA * ey);
    G[3] = fmaf((s.p + s.rhoe) * ue, A, (fmaf(0.5f, s.p, s.rhoe)) * sB);
}

__device__ __forceinline__ float venkat_f(float delta, float q, float qmx, float qmn, float eps2) {
    const float D = (delta > 0.0f) ? (qmx - q) : (qmn - q);
    const float num = (D * D + eps2) + 2.0f * delta * D;
    const float den = D * D + 2.0f * delta * delta + delta * D + eps2;
    return (den == 0.0f) ? 1.0f : num / den;
}

__device__ __forceinline__ void unpack(const float4 a, float *v) {
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

}  // namespace

template <bool LIMITER, int POW>
__global__ void __launch_bounds__(kBlock) k_flux_mixed(
    DevCloud cl, FlowParams fp, int stage, const double2 *__restrict__ q,
    const float4 *__restrict__ q32, const float4 *__restrict__ g32,
    const float4 *__restrict__ qmm32, double *__restrict__ U, double *__restrict__ Un,
    double *__restrict__ dt, double2 *__restrict__ qnext, float4 *__restrict__ q32next,
    double *__restrict__ Rout, double *__restrict__ partial, int *err) {
    const int n = cl.n;
    const int p = point_id();
    double R[4] = {0.0, 0.0, 0.0, 0.0};
    bool updated = false;
    if (p < n) {
        const uint8_t kd = cl.kind[p];
        if (kd == kOuter) {
            if (stage > 0) {
                double qp[4];
                load4(q, p, qp);
                store4(qnext, p, qp);
                q32next[p] = q32[p];
            }
            if (Rout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = 0.0;
            }
        } else {
            updated = true;
            const float gm1inv = (float)fp.gm1inv;
            const float vk = (float)fp.venkat_k;
            const double2 P = cl.xy[p], N = cl.nrm[p];
            const double tx = N.y, ty = -N.x;
            const float txf = (float)tx, tyf = (float)ty, nxf = (float)N.x, nyf = (float)N.y;
            float qp[4], gp[8], bp[8];
            unpack(q32[p], qp);
            unpack(g32[2 * p], gp);
            unpack(g32[2 * p + 1], gp + 4);
            if (LIMITER) {
                unpack(qmm32[2 * p], bp);
                unpack(qmm32[2 * p + 1], bp + 4);
            }
            double w[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = cl.lsw[8 * p + j];
            const uint8_t fmask = (kd == kWall) ? uint8_t(~kNPlus) : uint8_t(0xff);
            const int k1 = cl.ptr[p + 1];
            bool ok = true;
            for (int k = cl.ptr[p]; k < k1; ++k) {
                const uint8_t f = cl.flag[k] & fmask;
                if (f == 0) continue;
                const int i = cl.idx[k];
                const double2 Q = cl.xy[i];
                const double dx = Q.x - P.x, dy = Q.y - P.y;
                const double ds = dx * tx + dy * ty;
                const double dn = dx * N.x + dy * N.y;
                const float dxf = (float)dx, dyf = (float)dy;
                float qi[4], gi[8], qti[4], qt0[4];
                unpack(q32[i], qi);
                unpack(g32[2 * i], gi);
                unpack(g32[2 * i + 1], gi + 4);
                if (LIMITER) {
                    float bi[8];
                    unpack(qmm32[2 * i], bi);
                    unpack(qmm32[2 * i + 1], bi + 4);
                    const float e = vk * sqrtf(dxf * dxf + dyf * dyf);
                    const float eps2 = e * e * e;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float di = -0.5f * (dxf * gi[r] + dyf * gi[4 + r]);
                        const float d0 = -0.5f * (dxf * gp[r] + dyf * gp[4 + r]);
                        qti[r] = qi[r] + venkat_f(di, qi[r], bi[r], bi[4 + r], eps2) * di;
                        qt0[r] = qp[r] + venkat_f(d0, qp[r], bp[r], bp[4 + r], eps2) * d0;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        qti[r] = qi[r] - 0.5f * (dxf * gi[r] + dyf * gi[4 + r]);
                        qt0[r] = qp[r] - 0.5f * (dxf * gp[r] + dyf * gp[4 + r]);
                    }
                }
                PrimF si, s0;
                ok &= q_to_prim_f<POW>(qti, gm1inv, si);
                ok &= q_to_prim_f<POW>(qt0, gm1inv, s0);
                if (f & (kSPlus | kSMinus)) {
                    const bool plus = (f & kSPlus) != 0;
                    const float sg = plus ? 1.0f : -1.0f;
                    const double wt = ds * (plus ? w[0] : w[2]) - dn * (plus ? w[1] : w[3]);
                    float Gi[4], G0[4];
                    split_flux_f(si, txf, tyf, sg, Gi);
                    split_flux_f(s0, txf, tyf, sg, G0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) R[r] += wt * (double)(Gi[r] - G0[r]);
                }
                if (f & (kNPlus | kNMinus)) {
                    const bool plus = (f & kNPlus) != 0;
                    const float sg = plus ? 1.0f : -1.0f;
                    const double wt = dn * (plus ? w[4] : w[6]) - ds * (plus ? w[5] : w[7]);
                    float Gi[4], G0[4];
                    split_flux_f(si, nxf, nyf, sg, Gi);
                    split_flux_f(s0, nxf, nyf, sg, G0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) R[r] += wt * (double)(Gi[r] - G0[r]);
                }
            }
            if (!ok) report(err, p, kErrPositivity);
            if (Rout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = R[r];
            }
            if (stage > 0) {
                const double h = 0.5 * dt[p];
                double v[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double u = U[(size_t)c * n + p];
                    if (stage == 3)
                        v[c] = (2.0 / 3.0) * Un[(size_t)c * n + p] + (1.0 / 3.0) * (u - h * R[c]);
                    else
                        v[c] = u - h * R[c];
                }
                if (kd == kWall) wall_project(v, N);
#pragma unroll
                for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
                double qq[4];
                const int e = cons_to_q(v, fp, qq);
                if (e != kErrNone) {
                    report(err, p, e);
                    qq[0] = qq[1] = qq[2] = 0.0;
                    qq[3] = -1.0;
                }
                store4(qnext, p, qq);
                q32next[p] = to_f4(qq);
                if (stage == 4) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) Un[(size_t)c * n + p] = v[c];
                    dt[p] = local_dt(v, cl.dmin[p], fp);
                }
            }
        }
    }
    if (partial != nullptr) {
        __shared__ double red[kBlock / 64][4];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double sres = wave_sum(updated ? R[c] * R[c] : 0.0);
            if (lane == 0) red[wv][c] = sres;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < kBlock / 64; ++j) acc += red[j][threadIdx.x];
            partial[4 * logical_block() + threadIdx.x] = acc;
        }
    }
}

hipError_t launch_flux_mixed(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                             const double2 *q, const float4 *q32, const float4 *g32,
                             const float4 *qmm32, double *U, double *Un, double *dt,
                             double2 *qnext, float4 *q32next, double *Rout, double *partial,
                             int *err) {
    const dim3 grid(num_blocks(c.n)), block(kBlock);
#define QL_FLUXM_LAUNCH(LIM, POW)                                                             \
    hipLaunchKernelGGL((k_flux_mixed<LIM, POW>), grid, block, 0, st, c, fp, stage, q, q32, g32, \
                       qmm32, U, Un, dt, qnext, q32next, Rout, partial, err)
    if (fp.sqrt_pow == 5) {
        if (fp.limiter) QL_FLUXM_LAUNCH(true, 5);
        else QL_FLUXM_LAUNCH(false, 5);
    } else {
        if (fp.limiter) QL_FLUXM_LAUNCH(true, 0);
        else QL_FLUXM_LAUNCH(false, 0);
    }
#undef QL_FLUXM_LAUNCH
    return hipGetLastError();
}

// Residual norm: sqrt(sum of the workgroup partials / number of updated
// points), reduced in a fixed order.
__global__ void __launch_bounds__(kBlock) k_resnorm(int nblk, const double *__restrict__ partial,
                                                    double inv_nupd, double *__restrict__ out) {
    __shared__ double red[kBlock / 64][4];
    double s[4] = {0, 0, 0, 0};
    for (int j = threadIdx.x; j < nblk; j += kBlock) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += partial[4 * j + c];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double t = wave_sum(s[c]);
        if (lane == 0) red[wv][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) t += red[j][threadIdx.x];
        out[threadIdx.x] = sqrt(t * inv_nupd);
    }
}

hipError_t launch_resnorm(hipStream_t st, int nblk, const double *partial, double inv_nupd,
                          double *out) {
    hipLaunchKernelGGL(k_resnorm, dim3(1), dim3(kBlock), 0, st, nblk, partial, inv_nupd, out);
    return hipGetLastError();
}

// Forces from the wall pressure; wall[j] lists the wall points in the
// caller's order (the surface polygon).  Contributions are computed in
// parallel, then summed by one thread in polygon order, separately for the
// upper, lower and on-axis points.
__global__ void __launch_bounds__(kBlock) k_forces(int nw, const int *__restrict__ wall,
                                                   const double2 *__restrict__ xy,
                                                   const double2 *__restrict__ nrm,
                                                   const double *__restrict__ U, int n,
                                                   double gamma, double pinf,
                                                   double *__restrict__ f,
                                                   double *__restrict__ out) {
    for (int j = threadIdx.x; j < nw; j += kBlock) {
        const int p = wall[j], pn = wall[(j + 1) % nw], pp = wall[(j + nw - 1) % nw];
        const double2 P = xy[p], Pn = xy[pn], Pp = xy[pp];
        const double ds = 0.5 * (sqrt((Pn.x - P.x) * (Pn.x - P.x) + (Pn.y - P.y) * (Pn.y - P.y)) +
                                 sqrt((P.x - Pp.x) * (P.x - Pp.x) + (P.y - Pp.y) * (P.y - Pp.y)));
        const double rho = U[p];
        const double u1 = U[(size_t)n + p] / rho, u2 = U[(size_t)2 * n + p] / rho;
        const double pr = (gamma - 1.0) * (U[(size_t)3 * n + p] - 0.5 * rho * (u1 * u1 + u2 * u2));
        const double2 N = nrm[p];
        f[3 * j] = -(pr - pinf) * N.x * ds;
        f[3 * j + 1] = -(pr - pinf) * N.y * ds;
        f[3 * j + 2] = (P.y > 0.0) ? 0.0 : (P.y < 0.0) ? 1.0 : 2.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double F[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int j = 0; j < nw; ++j) {
            const int h = (int)f[3 * j + 2];
            F[h][0] += f[3 * j];
            F[h][1] += f[3 * j + 1];
        }
        out[0] = (F[0][0] + F[1][0]) + F[2][0];
        out[1] = (F[0][1] + F[1][1]) + F[2][1];
    }
}

hipError_t launch_forces(hipStream_t st, int nw, const int *wall, const double2 *xy,
                         const double2 *nrm, const double *U, int n, double gamma, double pinf,
                         double *scratch, double *out) {
    hipLaunchKernelGGL(k_forces, dim3(1), dim3(kBlock), 0, st, nw, wall, xy, nrm, U, n, gamma,
                       pinf, scratch, out);
    return hipGetLastError();
}

}  // namespace ql
