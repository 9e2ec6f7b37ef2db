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
#include "qlskum_erfc.h"

#include <climits>
#include <cmath>
#include <type_traits>

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

// tile served by this workgroup of a tiled sweep (launched with sweep_grid)
__device__ __forceinline__ int sweep_tile(const DevCloud &cl) {
    const int b = logical_block();
    return cl.tile_list ? cl.tile_list[b] : b;
}

// The point and its code travel in one word, (p << 8) | code, so the
// smallest failing point and the code it reported are always read together.
__device__ __forceinline__ void report(ErrWord *err, int p, int code) {
    atomicMin(err, ((ErrWord)(unsigned)p << 8) | (ErrWord)(unsigned)code);
}

// report to the solver's word and, in a batch, to the point's case word
__device__ __forceinline__ void report_pt(const DevCloud &cl, ErrWord *err, int p, int code) {
    report(err, p, code);
    if (cl.case_err) report(cl.case_err + cl.case_of[p], p, code);
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

// Value of lane l ^ 1 (CTRL kQuadXor1) or l ^ 2 (kQuadXor2) of the same group
// of four lanes: a DPP quad permutation of each 32-bit half (a VALU move, no
// LDS round trip).  Every lane of the quad must be active.
static_assert(kFluxLanes == 4, "the lane groups of the tiled sweeps are DPP quads");
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the kFluxLanes lanes that serve one point, in the fixed order
// (l0 + l1) + (l2 + l3); every lane of the group receives the same value
// (floating-point addition is commutative).
__device__ __forceinline__ double lane_group_sum(double v) {
    v += quad_swap<kQuadXor1>(v);
    v += quad_swap<kQuadXor2>(v);
    return v;
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
                                                  double *__restrict__ lsi,
                                                  double *__restrict__ dmin, ErrWord *err,
                                                  ErrWord *err_outer) {
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
    lsi[3 * p] = c / D;
    lsi[3 * p + 1] = b / D;
    lsi[3 * p + 2] = a / D;
    const uint8_t kd = kind[p];
    // An outer point's factors serve the kinetic outer condition only: its
    // s+, s- and n+ stencils are its own; its n- stencil is the mirror image
    // of n+ through the tangent line, (ds, dn) -> (ds, -dn), whose sums are
    // (Sss, -Ssn, Snn) of n+ -- the n- slot holds (Sss/Det, -Ssn/Det) of n+.
    // A singular outer stencil goes to err_outer, so that a cloud stays
    // usable with the outer points held at the freestream.
    bool bad_outer = false;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int m = (kd == kOuter && s == 3) ? 2 : s;  // stencil whose sums serve slot s
        const double det = ss[m] * nn[m] - sn[m] * sn[m];
        const double sc = ss[m] + nn[m];
        const bool used = (kd == kInterior) || (kd == kWall && s != 2) || kd == kOuter;
        double f0 = 0.0, f1 = 0.0;
        if (used) {
            if (cnt[m] < 2 || !(det > 1e-12 * sc * sc)) {
                if (kd == kOuter) bad_outer = true;
                else bad = true;
            }
            f0 = ((s < 2) ? nn[m] : ss[m]) / det;
            f1 = sn[m] / det;
            if (m != s) f1 = -f1;
        }
        lsw[8 * p + 2 * s] = f0;
        lsw[8 * p + 2 * s + 1] = f1;
    }
    if (bad) report(err, p, kErrSingular);
    if (bad_outer) report(err_outer, p, kErrSingular);
}

hipError_t launch_setup(hipStream_t st, int n, const double2 *xy, const double2 *nrm,
                        const uint8_t *kind, const int *ptr, const int *idx, uint8_t *flag,
                        int classify, double *lsw, double *lsi, double *dmin, ErrWord *err,
                        ErrWord *err_outer) {
    hipLaunchKernelGGL(k_setup, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, xy, nrm, kind, ptr,
                       idx, flag, classify, lsw, lsi, dmin, err, err_outer);
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
                                                       const int *__restrict__ case_of,
                                                       const double *__restrict__ uinf,
                                                       double *__restrict__ U) {
    const int p = point_id();
    if (p >= n) return;
    const double *u = uinf + 4 * case_of[p];
    double v[4] = {u[0], u[1], u[2], u[3]};
    if (kind[p] == kWall) wall_project(v, nrm[p]);
#pragma unroll
    for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
}

hipError_t launch_freestream(hipStream_t st, int n, const double2 *nrm, const uint8_t *kind,
                             const int *case_of, const double *uinf, double *U) {
    hipLaunchKernelGGL(k_freestream, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, nrm, kind,
                       case_of, uinf, U);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Warm start: a state from the network's primitive fields, and the choice
// between it and the freestream per case.
// ---------------------------------------------------------------------------
// Y[caller point][4] = standardised (rho, u1, u2, p); prim = mean + std * Y,
// rho and p held at or above `floor` times their freestream values; outer
// points keep the freestream (their Dirichlet condition); wall points are
// projected.
__global__ void __launch_bounds__(kBlock) k_warm_state(int n, const int *__restrict__ perm,
                                                       const uint8_t *__restrict__ kind,
                                                       const double2 *__restrict__ nrm,
                                                       const int *__restrict__ case_of,
                                                       const double *__restrict__ uinf,
                                                       const float *__restrict__ Y, WarmScale sc,
                                                       double gamma, double *__restrict__ U) {
    const int p = point_id();
    if (p >= n) return;
    const double *u = uinf + 4 * case_of[p];
    double v[4] = {u[0], u[1], u[2], u[3]};
    if (kind[p] != kOuter) {
        const float *y = Y + 4 * (size_t)perm[p];
        double pr[4];
        bool ok = true;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            pr[c] = (double)sc.mean[c] + (double)sc.std[c] * (double)y[c];
            ok = ok && isfinite(pr[c]);
        }
        // a point whose primitive or conserved state is not finite keeps the
        // freestream (fmax would hide a NaN density or pressure)
        if (ok) {
            const double pinf = 1.0 / gamma;  // rho_inf = 1, c_inf = 1
            const double rho = fmax(pr[0], sc.floor);
            const double pp = fmax(pr[3], sc.floor * pinf);
            const double w[4] = {rho, rho * pr[1], rho * pr[2],
                                 pp / (gamma - 1.0) + 0.5 * rho * (pr[1] * pr[1] + pr[2] * pr[2])};
            ok = isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]);
            if (ok) {
                v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; v[3] = w[3];
            }
        }
        if (kind[p] == kWall) wall_project(v, nrm[p]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = v[c];
}

hipError_t launch_warm_state(hipStream_t st, int n, const int *perm, const uint8_t *kind,
                             const double2 *nrm, const int *case_of, const double *uinf,
                             const float *Y, const WarmScale &sc, double gamma, double *U) {
    hipLaunchKernelGGL(k_warm_state, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, perm, kind, nrm,
                       case_of, uinf, Y, sc, gamma, U);
    return hipGetLastError();
}

// U <- Uw at the points of the cases with sel[case] != 0
__global__ void __launch_bounds__(kBlock) k_select_state(int n, const int *__restrict__ case_of,
                                                         const uint8_t *__restrict__ sel,
                                                         const double *__restrict__ Uw,
                                                         double *__restrict__ U) {
    const int p = point_id();
    if (p >= n || !sel[case_of[p]]) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) U[(size_t)c * n + p] = Uw[(size_t)c * n + p];
}

hipError_t launch_select_state(hipStream_t st, int n, const int *case_of, const uint8_t *sel,
                               const double *Uw, double *U) {
    hipLaunchKernelGGL(k_select_state, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, case_of, sel,
                       Uw, U);
    return hipGetLastError();
}

// Distance of every point to the nearest wall point of its case (brute
// force over the case's wall list; walls hold a few hundred points).  A case
// without wall points gets +inf.
__global__ void __launch_bounds__(kBlock) k_wall_distance(int n, const double2 *__restrict__ xy,
                                                          const int *__restrict__ case_of,
                                                          const int *__restrict__ wall_lo,
                                                          const int *__restrict__ wall,
                                                          double *__restrict__ d) {
    const int p = point_id();
    if (p >= n) return;
    const int c = case_of[p];
    const double2 P = xy[p];
    double best = INFINITY;
    for (int k = wall_lo[c]; k < wall_lo[c + 1]; ++k) {
        const double2 W = xy[wall[k]];
        const double dx = W.x - P.x, dy = W.y - P.y;
        best = fmin(best, dx * dx + dy * dy);
    }
    d[p] = sqrt(best);
}

hipError_t launch_wall_distance(hipStream_t st, int n, const double2 *xy, const int *case_of,
                                const int *wall_lo, const int *wall, double *d) {
    hipLaunchKernelGGL(k_wall_distance, dim3(num_blocks(n)), dim3(kBlock), 0, st, n, xy, case_of,
                       wall_lo, wall, d);
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
                                                 ErrWord *err) {
    const int n = cl.n;
    const int p = point_id();
    if (p >= n) return;
    if (cl.case_active && !cl.case_active[cl.case_of[p]]) return;  // retired case: frozen
    double v[4], qq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = U[(size_t)c * n + p];
    const int e = cons_to_q(v, fp, qq);
    if (e != kErrNone) {
        report_pt(cl, err, p, e);
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
                       double *Un, double2 *q, double *dt, float4 *q32, ErrWord *err) {
    hipLaunchKernelGGL(k_prep, dim3(num_blocks(c.n)), dim3(kBlock), 0, st, c, fp, U, Un, q, dt,
                       q32, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// q-derivatives, LDS-tiled with the flux sweep's tiles and lane layout: a
// workgroup owns kFluxTile consecutive points, stages the records its
// entries gather (its own points and its halo) in LDS, and serves each point
// with kFluxLanes lanes that walk every kFluxLanes-th entry; the lane sums
// are combined in a fixed order (lane_group_sum), so each point's sums have
// one order whichever path (LDS or memory) a tile takes.  The full-stencil
// least-squares matrix is inverted once at set-up (lsi = (Syy, Sxy, Sxx)/Det).
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ double lane_group_max(double v) {
    v = fmax(v, quad_swap<kQuadXor1>(v));
    return fmax(v, quad_swap<kQuadXor2>(v));
}

__device__ __forceinline__ double lane_group_min(double v) {
    v = fmin(v, quad_swap<kQuadXor1>(v));
    return fmin(v, quad_swap<kQuadXor2>(v));
}

template <int CTRL>
__device__ __forceinline__ float quad_swap_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float lane_group_max(float v) {
    v = fmaxf(v, quad_swap_f<kQuadXor1>(v));
    return fmaxf(v, quad_swap_f<kQuadXor2>(v));
}

__device__ __forceinline__ float lane_group_min(float v) {
    v = fminf(v, quad_swap_f<kQuadXor1>(v));
    return fminf(v, quad_swap_f<kQuadXor2>(v));
}

// tile set-up shared by the tiled sweeps: image size ns and whether it is
// staged (cap = slots that fit the LDS allocation of the launch)
struct TileInfo {
    int base, nown, h0, ns;
    bool in_lds;
};

__device__ __forceinline__ TileInfo tile_info(const DevCloud &cl, int t, int cap) {
    TileInfo ti;
    ti.base = t * kFluxTile;
    ti.nown = min(kFluxTile, cl.n - ti.base);
    ti.h0 = 0;
    ti.ns = 0;
    if (cl.fhalo_ptr) {
        ti.h0 = cl.fhalo_ptr[t];
        ti.ns = kFluxTile + cl.fhalo_ptr[t + 1] - ti.h0;
    }
    ti.in_lds = cl.fhalo_ptr != nullptr && ti.ns <= cap;
    return ti;
}

// point held by image slot s (own slots beyond the cloud's end return -1)
__device__ __forceinline__ int slot_point(const DevCloud &cl, const TileInfo &ti, int s) {
    if (s < kFluxTile) return s < ti.nown ? ti.base + s : -1;
    return cl.fhalo_idx[ti.h0 + s - kFluxTile];
}

}  // namespace

// Entry loops of the q-derivative sweeps, one instantiation per place the
// gathered records live (LDS image or memory): a loop whose loads may come
// from either would be compiled to generic (flat) loads, which go through
// the vector-memory path even for LDS and wait on both counters.

// first pass: sums of dx dq, dy dq and the componentwise max / min over the
// entries k0 + sub, k0 + sub + kFluxLanes, ... < k1 of point p
template <bool LDS>
__device__ __forceinline__ void grad0_entries(const DevCloud &cl, const double2 *lds,
                                              const double2 *q, int k0, int k1, int sub,
                                              const double qp[4], double2 P, double sx[4],
                                              double sy[4], double mx[4], double mn[4]) {
    constexpr int kRec = 3;
    for (int k = k0 + sub; k < k1; k += kFluxLanes) {
        double qi[4];
        double2 Q;
        if constexpr (LDS) {
            const double2 *r = lds + kRec * (int)cl.flidx[k];
            qi[0] = r[0].x; qi[1] = r[0].y; qi[2] = r[1].x; qi[3] = r[1].y;
            Q = r[2];
        } else {
            const int i = cl.idx[k];
            load4(q, i, qi);
            Q = cl.xy[i];
        }
        const double dx = Q.x - P.x, dy = Q.y - P.y;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dq = qi[r] - qp[r];
            sx[r] = fma(dx, dq, sx[r]);
            sy[r] = fma(dy, dq, sy[r]);
            mx[r] = fmax(mx[r], qi[r]);
            mn[r] = fmin(mn[r], qi[r]);
        }
    }
}

// first pass: full-stencil least squares of dq_i = q_i - q_p (eq. (11)), and
// the componentwise max / min of q over the point and its stencil (bounds of
// the limited reconstruction), stored as offsets from q.  Slot record
// (double2): q 0..1, position 2.  B64 false: the bounds go to the FP32
// shadow only (a compile-time choice: a run-time test costs the FP64 form a
// wave of occupancy).
template <bool B64>
__global__ void __launch_bounds__(kBlock) k_grad0(DevCloud cl, int cap,
                                                  const double2 *__restrict__ q,
                                                  double2 *__restrict__ g,
                                                  double2 *__restrict__ qmm, int want_bounds,
                                                  Shadow sh) {
    constexpr int kRec = 3;
    extern __shared__ double2 lds[];
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    const TileInfo ti = tile_info(cl, t, cap);
    if (ti.in_lds) {
        for (int s0 = threadIdx.x; s0 < ti.ns; s0 += kBlock) {
            const int p0 = slot_point(cl, ti, s0);
            if (p0 >= 0) {
                const double2 a0 = q[2 * p0], a1 = q[2 * p0 + 1], a2 = cl.xy[p0];
                lds[kRec * s0] = a0;
                lds[kRec * s0 + 1] = a1;
                lds[kRec * s0 + 2] = a2;
            }
        }
    }
    __syncthreads();
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = ti.base + j;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    double mx[4] = {0, 0, 0, 0}, mn[4] = {0, 0, 0, 0};
    if (j < ti.nown) {
        double qp[4];
        // the own position from memory on both paths (one load per point; a
        // value that may come from LDS or memory would be a generic load)
        const double2 P = cl.xy[p];
        if (ti.in_lds) {
            const double2 *r = lds + kRec * j;
            qp[0] = r[0].x; qp[1] = r[0].y; qp[2] = r[1].x; qp[3] = r[1].y;
        } else {
            load4(q, p, qp);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) mx[r] = mn[r] = qp[r];
        const int k0 = cl.ptr[p], k1 = cl.ptr[p + 1];
        if (ti.in_lds)
            grad0_entries<true>(cl, lds, q, k0, k1, sub, qp, P, sx, sy, mx, mn);
        else
            grad0_entries<false>(cl, lds, q, k0, k1, sub, qp, P, sx, sy, mx, mn);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sx[r] = lane_group_sum(sx[r]);
        sy[r] = lane_group_sum(sy[r]);
        mx[r] = lane_group_max(mx[r]);
        mn[r] = lane_group_min(mn[r]);
    }
    if (j >= ti.nown) return;
    const double L0 = cl.lsi[3 * p], L1 = cl.lsi[3 * p + 1], L2 = cl.lsi[3 * p + 2];
    double gv[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gv[r] = fma(L0, sx[r], -(L1 * sy[r]));
        gv[4 + r] = fma(L2, sy[r], -(L1 * sx[r]));
    }
    // each of the point's lanes stores one 16-byte part
    g[4 * p + sub] = make_double2(gv[2 * sub], gv[2 * sub + 1]);
    if (sh.g32 && sub < 2) sh.g32[2 * p + sub] = to_f4(gv + 4 * sub);
    if (want_bounds) {
        // bounds are stored as offsets from q (the limiter's D = q_max - q or
        // q_min - q, the same FP64 subtraction it would make per entry)
        double qp[4];
        if (ti.in_lds) {
            const double2 *r = lds + kRec * j;
            qp[0] = r[0].x; qp[1] = r[0].y; qp[2] = r[1].x; qp[3] = r[1].y;
        } else {
            load4(q, p, qp);
        }
        double bv[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bv[r] = mx[r] - qp[r];
            bv[4 + r] = mn[r] - qp[r];
        }
        if (B64) qmm[4 * p + sub] = make_double2(bv[2 * sub], bv[2 * sub + 1]);
        if (sh.qmm32 && sub < 2) sh.qmm32[2 * p + sub] = to_f4(bv + 4 * sub);
    }
}

// entry slots an inner-iteration workgroup stages in LDS (tiles with more
// entries read them from memory)
constexpr int kCapE = 2048;
constexpr int kLdsBytes = 160 * 1024;  // LDS one workgroup may allocate on gfx950

// inner iteration: sums of dx f, dy f with f = dx g_x,i + dy g_y,i over the
// entries of point p.  SRC 0: records and entry slots in LDS; 1: records in
// LDS, entry slots from memory; 2: records from memory.
template <int SRC>
__device__ __forceinline__ void gradk_entries(const DevCloud &cl, const double2 *lds,
                                              const uint16_t *eidx, int e0,
                                              const double2 *gprev, int kb, int k1, int sub,
                                              double2 P, double sx[4], double sy[4]) {
    constexpr int kRec = 5;
#pragma unroll 1
    for (int k = kb + sub; k < k1; k += kFluxLanes) {
        double gi[8];
        double2 Q;
        if constexpr (SRC < 2) {
            const int li = (SRC == 0) ? (int)eidx[k - e0] : (int)cl.flidx[k];
            const double2 *r = lds + kRec * li;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                gi[2 * m] = r[m].x;
                gi[2 * m + 1] = r[m].y;
            }
            Q = r[4];
        } else {
            const int i = cl.idx[k];
            load8(gprev, i, gi);
            Q = cl.xy[i];
        }
        const double dx = Q.x - P.x, dy = Q.y - P.y;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double f = fma(dx, gi[r], dy * gi[4 + r]);
            sx[r] = fma(dx, f, sx[r]);
            sy[r] = fma(dy, f, sy[r]);
        }
    }
}

// one inner iteration (eq. (29)).  The least squares is linear in its data:
//   g^k = LS(dq_i) - 1/2 LS(d.(g^{k-1}_i - g^{k-1}_p)) = g0 - 1/2 LS(...)
// so only the previous iterate is gathered (Jacobi: read gprev, write gnext).
// Slot record (double2): g 0..3, position 4.
__global__ void __launch_bounds__(kBlock) k_gradk(DevCloud cl, int cap,
                                                  const double2 *__restrict__ g0,
                                                  const double2 *__restrict__ gprev,
                                                  double2 *__restrict__ gnext,
                                                  float4 *__restrict__ g32) {
    constexpr int kRec = 5;
    extern __shared__ double2 lds[];
    uint16_t *eidx = reinterpret_cast<uint16_t *>(lds + (size_t)kRec * cap);
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    const TileInfo ti = tile_info(cl, t, cap);
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = ti.base + j;
    const bool own = j < ti.nown;
    int kb = 0, k1 = 0;
    double L0 = 0.0, L1 = 0.0, L2 = 0.0;
    double2 z = make_double2(0.0, 0.0), gq = make_double2(0.0, 0.0);
    if (own) {
        kb = cl.ptr[p];
        k1 = cl.ptr[p + 1];
        L0 = cl.lsi[3 * p];
        L1 = cl.lsi[3 * p + 1];
        L2 = cl.lsi[3 * p + 2];
        z = g0[4 * p + sub];
        gq = gprev[4 * p + sub];
    }
    const int e0 = cl.ptr[ti.base], ne = cl.ptr[ti.base + ti.nown] - e0;
    const bool e_lds = ti.in_lds && ne <= kCapE;
    if (ti.in_lds) {
        for (int s0 = threadIdx.x; s0 < ti.ns; s0 += 2 * kBlock) {
            const int s1 = s0 + kBlock;
            const int p0 = slot_point(cl, ti, s0);
            const int p1 = (s1 < ti.ns) ? slot_point(cl, ti, s1) : -1;
            const int c0 = p0 >= 0 ? p0 : 0, c1 = p1 >= 0 ? p1 : 0;  // in-range reads
            const double2 a0 = gprev[4 * c0], a1 = gprev[4 * c0 + 1], a2 = gprev[4 * c0 + 2],
                          a3 = gprev[4 * c0 + 3], a4 = cl.xy[c0];
            const double2 b0 = gprev[4 * c1], b1 = gprev[4 * c1 + 1], b2 = gprev[4 * c1 + 2],
                          b3 = gprev[4 * c1 + 3], b4 = cl.xy[c1];
            if (p0 >= 0) {
                double2 *d = lds + kRec * s0;
                d[0] = a0; d[1] = a1; d[2] = a2; d[3] = a3; d[4] = a4;
            }
            if (p1 >= 0) {
                double2 *d = lds + kRec * s1;
                d[0] = b0; d[1] = b1; d[2] = b2; d[3] = b3; d[4] = b4;
            }
        }
        if (e_lds)
            for (int e = threadIdx.x; e < ne; e += kBlock) eidx[e] = cl.flidx[e0 + e];
    }
    __syncthreads();
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    if (own) {
        const double2 P = cl.xy[p];  // from memory on both paths (see k_grad0)
        if (e_lds)
            gradk_entries<0>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
        else if (ti.in_lds)
            gradk_entries<1>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
        else
            gradk_entries<2>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sx[r] = lane_group_sum(sx[r]);
        sy[r] = lane_group_sum(sy[r]);
    }
    if (!own) return;
    // lane sub produces components 2 sub, 2 sub + 1 of (q_x[0..3], q_y[0..3])
    double v[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int c = 2 * sub + m, r = c & 3;
        const double ls = (c < 4) ? fma(L0, sx[r], -(L1 * sy[r])) : fma(L2, sy[r], -(L1 * sx[r]));
        v[m] = fma(-0.5, ls - (m == 0 ? gq.x : gq.y), m == 0 ? z.x : z.y);
    }
    if (gnext) gnext[4 * p + sub] = make_double2(v[0], v[1]);
    if (g32) {
        // the FP32 shadow packs (q_x[0..3]) and (q_y[0..3]): lanes 0,1 and 2,3
        // hold halves of one float4, combined through a shuffle of partner lanes
        const double o0 = quad_swap<kQuadXor1>(v[0]), o1 = quad_swap<kQuadXor1>(v[1]);
        if ((sub & 1) == 0)
            g32[2 * p + (sub >> 1)] =
                make_float4((float)v[0], (float)v[1], (float)o0, (float)o1);
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision q-derivatives.  The same sweeps, tiles and lane layout
// with the gathered data in FP32 -- q (first pass) or the previous iterate
// (inner iterations), as FP32 copies -- and the positions in FP64: every
// offset, difference, product and sum, and the 2x2 solve, stays FP64, and
// the results are stored in FP32 for the next sweep and the FP32 flux body.
// Records of 32 and 48 bytes instead of 48 and 80.
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void f4_to_d(float4 a, double v[4]) {
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// first pass over the entries of one point; SRC 0: records in LDS (slot
// numbers from memory), 2: from memory.  Record: q (float4), position.
template <int SRC>
__device__ __forceinline__ void grad0f_entries(const DevCloud &cl, const double2 *lds,
                                               const float4 *q32, int k0, int k1, int sub,
                                               const double qp[4], double2 P, double sx[4],
                                               double sy[4], float mx[4], float mn[4]) {
    constexpr int kRec = 2;
    // two entries in flight per lane (each lane's sums keep their order)
#pragma unroll 2
    for (int k = k0 + sub; k < k1; k += kFluxLanes) {
        float4 a;
        double2 Q;
        if constexpr (SRC == 0) {
            const double2 *r = lds + kRec * (int)cl.flidx[k];
            a = *reinterpret_cast<const float4 *>(r);
            Q = r[1];
        } else {
            const int i = cl.idx[k];
            a = q32[i];
            Q = cl.xy[i];
        }
        const float qf[4] = {a.x, a.y, a.z, a.w};
        const double dx = Q.x - P.x, dy = Q.y - P.y;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // the data are FP32, so their bounds are exact in FP32
            const double dq = (double)qf[r] - qp[r];
            sx[r] = fma(dx, dq, sx[r]);
            sy[r] = fma(dy, dq, sy[r]);
            mx[r] = fmaxf(mx[r], qf[r]);
            mn[r] = fminf(mn[r], qf[r]);
        }
    }
}

// inner iteration over the entries of one point; SRC as gradk_entries.
// Record: q_x (float4), q_y (float4), position.
template <int SRC>
__device__ __forceinline__ void gradkf_entries(const DevCloud &cl, const double2 *lds,
                                               const uint16_t *eidx, int e0,
                                               const float4 *gprev, int kb, int k1, int sub,
                                               double2 P, double sx[4], double sy[4]) {
    constexpr int kRec = 3;
#pragma unroll 1
    for (int k = kb + sub; k < k1; k += kFluxLanes) {
        double gi[8];
        double2 Q;
        if constexpr (SRC < 2) {
            const int li = (SRC == 0) ? (int)eidx[k - e0] : (int)cl.flidx[k];
            const double2 *r = lds + kRec * li;
            f4_to_d(*reinterpret_cast<const float4 *>(r), gi);
            f4_to_d(*reinterpret_cast<const float4 *>(r + 1), gi + 4);
            Q = r[2];
        } else {
            const int i = cl.idx[k];
            f4_to_d(gprev[2 * i], gi);
            f4_to_d(gprev[2 * i + 1], gi + 4);
            Q = cl.xy[i];
        }
        const double dx = Q.x - P.x, dy = Q.y - P.y;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double f = fma(dx, gi[r], dy * gi[4 + r]);
            sx[r] = fma(dx, f, sx[r]);
            sy[r] = fma(dy, f, sy[r]);
        }
    }
}

// components 2 sub, 2 sub + 1 of a point's (q_x[0..3], q_y[0..3]) held as
// two float4
__device__ __forceinline__ double2 lane_pair(const float4 *g, int p, int sub) {
    const float4 a = g[2 * p + (sub >> 1)];
    return (sub & 1) ? make_double2(a.z, a.w) : make_double2(a.x, a.y);
}

}  // namespace

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) k_grad0_f(DevCloud cl, int cap,
                                                    const float4 *__restrict__ q32,
                                                    float4 *__restrict__ g0f,
                                                    float4 *__restrict__ qmm32, int want_bounds) {
    constexpr int kRec = 2;
    extern __shared__ double2 lds[];
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    const TileInfo ti = tile_info(cl, t, cap);
    if (ti.in_lds) {
        for (int s0 = threadIdx.x; s0 < ti.ns; s0 += kBlock) {
            const int p0 = slot_point(cl, ti, s0);
            if (p0 >= 0) {
                const float4 a0 = q32[p0];
                const double2 a1 = cl.xy[p0];
                *reinterpret_cast<float4 *>(lds + kRec * s0) = a0;
                lds[kRec * s0 + 1] = a1;
            }
        }
    }
    __syncthreads();
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = ti.base + j;
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    float mx[4] = {0, 0, 0, 0}, mn[4] = {0, 0, 0, 0};
    double qp[4] = {0, 0, 0, 0};
    if (j < ti.nown) {
        const float4 a = q32[p];
        f4_to_d(a, qp);
        const double2 P = cl.xy[p];
        mx[0] = mn[0] = a.x;
        mx[1] = mn[1] = a.y;
        mx[2] = mn[2] = a.z;
        mx[3] = mn[3] = a.w;
        const int k0 = cl.ptr[p], k1 = cl.ptr[p + 1];
        if (ti.in_lds)
            grad0f_entries<0>(cl, lds, q32, k0, k1, sub, qp, P, sx, sy, mx, mn);
        else
            grad0f_entries<2>(cl, lds, q32, k0, k1, sub, qp, P, sx, sy, mx, mn);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sx[r] = lane_group_sum(sx[r]);
        sy[r] = lane_group_sum(sy[r]);
        mx[r] = lane_group_max(mx[r]);
        mn[r] = lane_group_min(mn[r]);
    }
    if (j >= ti.nown || sub >= 2) return;
    const double L0 = cl.lsi[3 * p], L1 = cl.lsi[3 * p + 1], L2 = cl.lsi[3 * p + 2];
    double gv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        gv[r] = (sub == 0) ? fma(L0, sx[r], -(L1 * sy[r])) : fma(L2, sy[r], -(L1 * sx[r]));
    g0f[2 * p + sub] = to_f4(gv);
    if (want_bounds) {
        // bound offsets from q: lane 0 the maxima, lane 1 the minima
        double bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[r] = (double)(sub == 0 ? mx[r] : mn[r]) - qp[r];
        qmm32[2 * p + sub] = to_f4(bv);
    }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) k_gradk_f(DevCloud cl, int cap,
                                                    const float4 *__restrict__ g0f,
                                                    const float4 *__restrict__ gprev,
                                                    float4 *__restrict__ gnext) {
    constexpr int kRec = 3;
    extern __shared__ double2 lds[];
    uint16_t *eidx = reinterpret_cast<uint16_t *>(lds + (size_t)kRec * cap);
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    const TileInfo ti = tile_info(cl, t, cap);
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = ti.base + j;
    const bool own = j < ti.nown;
    int kb = 0, k1 = 0;
    double L0 = 0.0, L1 = 0.0, L2 = 0.0;
    double2 z = make_double2(0.0, 0.0), gq = make_double2(0.0, 0.0);
    if (own) {
        kb = cl.ptr[p];
        k1 = cl.ptr[p + 1];
        L0 = cl.lsi[3 * p];
        L1 = cl.lsi[3 * p + 1];
        L2 = cl.lsi[3 * p + 2];
        z = lane_pair(g0f, p, sub);
        gq = lane_pair(gprev, p, sub);
    }
    const int e0 = cl.ptr[ti.base], ne = cl.ptr[ti.base + ti.nown] - e0;
    const bool e_lds = ti.in_lds && ne <= kCapE;
    if (ti.in_lds) {
        for (int s0 = threadIdx.x; s0 < ti.ns; s0 += kBlock) {
            const int p0 = slot_point(cl, ti, s0);
            if (p0 >= 0) {
                const float4 a0 = gprev[2 * p0], a1 = gprev[2 * p0 + 1];
                const double2 a2 = cl.xy[p0];
                double2 *d = lds + kRec * s0;
                *reinterpret_cast<float4 *>(d) = a0;
                *reinterpret_cast<float4 *>(d + 1) = a1;
                d[2] = a2;
            }
        }
        if (e_lds)
            for (int e = threadIdx.x; e < ne; e += kBlock) eidx[e] = cl.flidx[e0 + e];
    }
    __syncthreads();
    double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    if (own) {
        const double2 P = cl.xy[p];
        if (e_lds)
            gradkf_entries<0>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
        else if (ti.in_lds)
            gradkf_entries<1>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
        else
            gradkf_entries<2>(cl, lds, eidx, e0, gprev, kb, k1, sub, P, sx, sy);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sx[r] = lane_group_sum(sx[r]);
        sy[r] = lane_group_sum(sy[r]);
    }
    if (!own) return;
    double v[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int c = 2 * sub + m, r = c & 3;
        const double ls = (c < 4) ? fma(L0, sx[r], -(L1 * sy[r])) : fma(L2, sy[r], -(L1 * sx[r]));
        v[m] = fma(-0.5, ls - (m == 0 ? gq.x : gq.y), m == 0 ? z.x : z.y);
    }
    // lanes 0,1 and 2,3 hold halves of one float4 (see k_gradk)
    const double o0 = quad_swap<kQuadXor1>(v[0]), o1 = quad_swap<kQuadXor1>(v[1]);
    if ((sub & 1) == 0)
        gnext[2 * p + (sub >> 1)] = make_float4((float)v[0], (float)v[1], (float)o0, (float)o1);
}

static int lds_cap(const DevCloud &c, int budget, int rec) {
    if (!c.fhalo_ptr) return 0;
    return min(c.fmax_slots, max(budget / rec, 0));
}

// LDS bytes a q-derivative workgroup stages its tile image in when the
// caller gives no budget (records of 48 and 80 bytes; the inner iteration
// also stages 4 KB of entry slots).  Sized so that the 6 workgroups per CU
// that the kernels' registers allow stay resident in 160 KB of LDS
// (measured on the 2.5M cloud: 22 KB runs the inner iteration 12% faster
// than 36 KB, although a few more tiles then read from memory).
constexpr int kGrad0Lds = 32 * 1024;
constexpr int kGradkLds = 22 * 1024;
// The FP32-data inner iteration fits 64 VGPRs, i.e. 8 waves per SIMD: 8
// workgroups per CU when each stays within 20 KB of LDS (images of 48-byte
// records plus 4 KB of entry slots).  The first pass keeps two entries in
// flight per lane at 72 VGPRs (7 waves); its images of 32-byte records fit
// 20 KB as well.
constexpr int kGrad0FLds = 20 * 1024;
constexpr int kGradkFLds = 20 * 1024 - 2 * kCapE;

hipError_t launch_grad0(hipStream_t st, const DevCloud &c, int lds_budget, const double2 *q,
                        double2 *g, double2 *qmm, int want_bounds, Shadow sh) {
    const int rec = 3 * (int)sizeof(double2);
    const int cap = lds_cap(c, lds_budget > 0 ? lds_budget : kGrad0Lds, rec);
    const int ntile = sweep_grid(c);
    if (want_bounds && !qmm) {
        if (!sh.qmm32) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_grad0<false>, dim3(ntile), dim3(kBlock), (size_t)cap * rec, st, c, cap,
                           q, g, qmm, want_bounds, sh);
    } else {
        hipLaunchKernelGGL(k_grad0<true>, dim3(ntile), dim3(kBlock), (size_t)cap * rec, st, c, cap,
                           q, g, qmm, want_bounds, sh);
    }
    return hipGetLastError();
}

hipError_t launch_grad0_f(hipStream_t st, const DevCloud &c, int lds_budget, const float4 *q32,
                          float4 *g0f, float4 *qmm32, int want_bounds) {
    const int rec = 2 * (int)sizeof(double2);
    const int cap = lds_cap(c, lds_budget > 0 ? lds_budget : kGrad0FLds, rec);
    hipLaunchKernelGGL(k_grad0_f, dim3(sweep_grid(c)), dim3(kBlock), (size_t)cap * rec, st,
                       c, cap, q32, g0f, qmm32, want_bounds);
    return hipGetLastError();
}

hipError_t launch_gradk_f(hipStream_t st, const DevCloud &c, int lds_budget, const float4 *g0f,
                          const float4 *gprev, float4 *gnext) {
    const int rec = 3 * (int)sizeof(double2);
    const int cap = min(lds_cap(c, lds_budget > 0 ? lds_budget : kGradkFLds, rec),
                        (kLdsBytes - 2 * kCapE) / rec);
    const size_t shmem = cap > 0 ? (size_t)cap * rec + 2 * kCapE : 0;
    hipLaunchKernelGGL(k_gradk_f, dim3(sweep_grid(c)), dim3(kBlock), shmem, st, c, cap, g0f,
                       gprev, gnext);
    return hipGetLastError();
}

hipError_t launch_gradk(hipStream_t st, const DevCloud &c, int lds_budget, const double2 *g0,
                        const double2 *gprev, double2 *gnext, float4 *g32) {
    const int rec = 5 * (int)sizeof(double2);
    // the image and the entry slots share the workgroup's 160 KB of LDS
    const int cap = min(lds_cap(c, lds_budget > 0 ? lds_budget : kGradkLds, rec),
                        (kLdsBytes - 2 * kCapE) / rec);
    const size_t shmem = cap > 0 ? (size_t)cap * rec + 2 * kCapE : 0;
    hipLaunchKernelGGL(k_gradk, dim3(sweep_grid(c)), dim3(kBlock), shmem, st, c, cap, g0,
                       gprev, gnext, g32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flux residual + Runge-Kutta stage.
// ---------------------------------------------------------------------------
namespace {

// x^K by repeated squaring (x^5 = (x^2)^2 x: three multiplications)
template <int K, class T>
__device__ __forceinline__ T ipow(T x) {
    if constexpr (K == 1) {
        return x;
    } else if constexpr (K % 2 == 0) {
        const T h = ipow<K / 2>(x);
        return h * h;
    } else {
        return ipow<K - 1>(x) * x;
    }
}

constexpr double kHalfRsqrtPi = 0.28209479177387814347;  // 1 / (2 sqrt(pi))

// primitive state with the per-state factors of the split fluxes:
// bk = 1/(2 sqrt(pi beta)), h = p + rho e, k = p/2 + rho e
struct Prim {
    double rho, u1, u2, p, sqb, bk, h, k;
};

// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (each squares the relative error; the result is within an ulp or two of
// the rounded quotient) for d normal and finite -- the flux body's divisors
// (2 beta of a state that passes the positivity check, the limiter's
// denominator, which is zero or at least eps^2) are.  A correctly rounded
// division costs several times more issue slots in this VALU-bound kernel.
__device__ __forceinline__ double fast_rcp(double d) {
#pragma clang fp contract(off)
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

// 1/sqrt(d) from the hardware estimate refined by two Newton steps
// r <- r + (r/2)(1 - d r^2), for d positive, normal and finite (beta of a
// state that passes the positivity check).
__device__ __forceinline__ double fast_rsqrt(double d) {
#pragma clang fp contract(off)
    double r = __builtin_amdgcn_rsq(d);
    r = fma(0.5 * r, fma(-(d * r), r, 1.0), r);
    return fma(0.5 * r, fma(-(d * r), r, 1.0), r);
}

// sqrt(d) for d positive, normal and finite: s = d r with r the hardware
// 1/sqrt estimate, then one Newton correction s + (d - s^2) r/2, which
// squares the estimate's relative error.
__device__ __forceinline__ double fast_sqrt(double d) {
#pragma clang fp contract(off)
    const double r = __builtin_amdgcn_rsq(d);
    const double s = d * r;
    return fma(fma(-s, s, d), 0.5 * r, s);
}

// q~ -> primitive state (inverse of eq. (26)); false if q4 >= 0 or the
// result is not finite (the Maxwellian of q~ does not exist).  One reciprocal
// (1/(2 beta)), one reciprocal square root and one exponential:
// sqrt(beta) = beta / sqrt(beta), and beta^(-1/(gamma-1)) = (1/sqrt(beta))^m.
// The per-state formulas below are written with explicit fma and no implicit
// contraction, so that two reconstructed states that are bitwise equal give
// bitwise equal fluxes (uniform flow keeps R = 0 exactly).
template <int POW>
__device__ __forceinline__ bool q_to_prim(const double qt[4], const FlowParams &fp, Prim &s) {
#pragma clang fp contract(off)
    const double beta = -0.5 * qt[3];
    const double inv2b = -fast_rcp(qt[3]);
    s.u1 = qt[1] * inv2b;
    s.u2 = qt[2] * inv2b;
    const double uu = fma(s.u1, s.u1, s.u2 * s.u2);
    const double isqb = fast_rsqrt(beta);
    s.sqb = beta * isqb;
    if (POW > 0) {
        s.rho = exp_poly(fma(beta, uu, qt[0])) * ipow<POW>(isqb);
    } else {
        s.rho = exp_poly(fma(beta, uu, fma(-log(beta), fp.gm1inv, qt[0])));
    }
    s.p = s.rho * inv2b;
    const double rhoe = fma(s.p, fp.gm1inv, (0.5 * s.rho) * uu);
    s.h = s.p + rhoe;
    s.k = fma(0.5, s.p, rhoe);
    s.bk = kHalfRsqrtPi * isqb;
    return (qt[3] < 0.0) && isfinite(s.rho) && isfinite(s.p) && isfinite(s.u1) &&
           isfinite(s.u2);
}

// Kinetic split flux along the unit direction e; sg = +1 for G+, -1 for G-.
// Half-range moments of the Maxwellian: with S = u_e sqrt(beta),
// A = erfc(-sg S)/2 and B = exp(-S^2)/(2 sqrt(pi beta)) (one exponential
// serves both, see qlskum_erfc.h),
//   G = [rho(u_e A + sg B), rho u (u_e A + sg B) + p A e,
//        (p + rho e) u_e A + sg (p/2 + rho e) B].
__device__ __forceinline__ void split_flux(const Prim &s, double ex, double ey, double sg,
                                           double G[4]) {
#pragma clang fp contract(off)
    const double ue = fma(s.u1, ex, s.u2 * ey);
    const double S = ue * s.sqb;
    const double E = gauss(S);
    const double A = half_erfc(-sg * S, E, fast_rcp(kErfcC64 + fabs(S)));
    const double B = E * s.bk;
    const double sB = sg * B;
    const double mass = s.rho * fma(ue, A, sB);
    const double pA = s.p * A;
    G[0] = mass;
    G[1] = fma(s.u1, mass, pA * ex);
    G[2] = fma(s.u2, mass, pA * ey);
    G[3] = fma(s.h * ue, A, s.k * sB);
}

// Venkatakrishnan limiter value for the increment delta of one component:
//   phi = (D^2 + eps^2 + 2 delta D) / (D^2 + 2 delta^2 + delta D + eps^2)
// with D = qmax - q (delta > 0) or qmin - q, the point's stored offsets dmax
// and dmin.  The denominator is (D + delta/2)^2 + 7/4 delta^2 + eps^2 >=
// eps^2 > 0: callers keep eps^2 at least 1e-300, so that coincident points
// (D = delta = eps = 0, the one 0/0 case) give phi = 1 without a test here.
__device__ __forceinline__ double venkat(double delta, double dmax, double dmin, double eps2) {
#pragma clang fp contract(off)
    const double D = (delta > 0.0) ? dmax : dmin;
    const double a = fma(D, D, eps2);
    const double num = fma(2.0 * delta, D, a);
    const double den = fma(delta, D, fma(2.0 * delta, delta, a));
    return num * fast_rcp(den);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Contribution of one neighbour entry (split flags f, offset (dx, dy) from p
// to i) to the residual of p: the modified states q~_i and q~_p of eq. (28)
// (limited when LIMITER), their split fluxes, and w_b (G(q~_i) - G(q~_p))
// added for each split stencil b the entry belongs to (one s half and one n
// half at most).  w holds p's eight least-squares factors (see k_setup).
// Written with explicit fma and no implicit contraction: a point's residual
// depends only on its data and on the order of its entries, never on the code
// path that gathered them.  Returns false when a modified state has no
// Maxwellian.  FIRST: first-order scheme, the split fluxes of q itself.
// M: the split stencils evaluated (Split bits; 15 all four).  The caller
// masks f with M, so a direction is evaluated when M holds either half.
template <bool LIMITER, int POW, bool FIRST, int M = 15>
__device__ __forceinline__ bool flux_entry(uint8_t f, double dx, double dy, double2 N,
                                           const double qi[4], const double gi[8],
                                           const double bi[8], const double qp[4],
                                           const double gp[8], const double bp[8],
                                           const double w[8], const FlowParams &fp,
                                           double R[4]) {
#pragma clang fp contract(off)
    const double tx = N.y, ty = -N.x;
    const double ds = fma(dx, tx, dy * ty);
    const double dn = fma(dx, N.x, dy * N.y);
    double qti[4], qt0[4];
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qti[r] = qi[r];
            qt0[r] = qp[r];
        }
    } else if (LIMITER) {
        const double e = fp.venkat_k * fast_sqrt(fma(dx, dx, dy * dy));
        const double eps2 = fmax((e * e) * e, 1e-300);
        // -1/2 folded into the offsets: scaling by a power of two commutes
        // with rounding, so delta has the same bits as -1/2 (d . g)
        const double hx = -0.5 * dx, hy = -0.5 * dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double di = fma(hx, gi[r], hy * gi[4 + r]);
            const double d0 = fma(hx, gp[r], hy * gp[4 + r]);
            qti[r] = fma(venkat(di, bi[r], bi[4 + r], eps2), di, qi[r]);
            qt0[r] = fma(venkat(d0, bp[r], bp[4 + r], eps2), d0, qp[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qti[r] = fma(-0.5, fma(dx, gi[r], dy * gi[4 + r]), qi[r]);
            qt0[r] = fma(-0.5, fma(dx, gp[r], dy * gp[4 + r]), qp[r]);
        }
    }
    Prim si, s0;
    bool ok = q_to_prim<POW>(qti, fp, si);
    ok &= q_to_prim<POW>(qt0, fp, s0);
    // both directions without branches (an entry outside a direction's
    // stencils gets weight 0), so that the four split-flux evaluations are
    // independent straight-line work the scheduler can interleave
    double Gs[2][4], Gn[2][4];
    double ws = 0.0, wn = 0.0;
    if (M & (kSPlus | kSMinus)) {
        const bool plus = (f & kSPlus) != 0;
        const double sg = plus ? 1.0 : -1.0;
        ws = (f & (kSPlus | kSMinus)) ? fma(ds, plus ? w[0] : w[2], -(dn * (plus ? w[1] : w[3])))
                                      : 0.0;
        split_flux(si, tx, ty, sg, Gs[0]);
        split_flux(s0, tx, ty, sg, Gs[1]);
    }
    if (M & (kNPlus | kNMinus)) {
        const bool plus = (f & kNPlus) != 0;
        const double sg = plus ? 1.0 : -1.0;
        wn = (f & (kNPlus | kNMinus)) ? fma(dn, plus ? w[4] : w[6], -(ds * (plus ? w[5] : w[7])))
                                      : 0.0;
        split_flux(si, N.x, N.y, sg, Gn[0]);
        split_flux(s0, N.x, N.y, sg, Gn[1]);
    }
    if (M & (kSPlus | kSMinus)) {
#pragma unroll
        for (int r = 0; r < 4; ++r) R[r] = fma(ws, Gs[0][r] - Gs[1][r], R[r]);
    }
    if (M & (kNPlus | kNMinus)) {
#pragma unroll
        for (int r = 0; r < 4; ++r) R[r] = fma(wn, Gn[0][r] - Gn[1][r], R[r]);
    }
    return ok;
}

// Kinetic outer condition, one n+ entry (offset (dx, dy) from outer point p)
// of p's mirrored n- stencil: the mirror image of the neighbour through p's
// tangent line, at offset (ds, -dn) in p's frame, holds the freestream, so
// its modified state is q_inf and its split flux G_inf = Gn-(q_inf) (given);
// p's own modified state is shifted by the mirrored offset as in eq. (28).
// Adds w (G_inf - Gn-(q~_p)) with w the mirrored stencil's n-derivative
// weight (k_setup stores the mirrored factors in p's n- slot).
template <bool LIMITER, int POW, bool FIRST>
__device__ __forceinline__ bool mirror_entry(double dx, double dy, double2 N, const double qp[4],
                                             const double gp[8], const double bp[8],
                                             const double w[8], const double Ginf[4],
                                             const FlowParams &fp, double R[4]) {
#pragma clang fp contract(off)
    const double tx = N.y, ty = -N.x;
    const double ds = fma(dx, tx, dy * ty);
    const double dm = -fma(dx, N.x, dy * N.y);
    const double mx = fma(ds, tx, dm * N.x), my = fma(ds, ty, dm * N.y);
    double qt0[4];
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) qt0[r] = qp[r];
    } else if (LIMITER) {
        const double e = fp.venkat_k * fast_sqrt(fma(mx, mx, my * my));
        const double eps2 = fmax((e * e) * e, 1e-300);
        const double hx = -0.5 * mx, hy = -0.5 * my;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double d0 = fma(hx, gp[r], hy * gp[4 + r]);
            qt0[r] = fma(venkat(d0, bp[r], bp[4 + r], eps2), d0, qp[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) qt0[r] = fma(-0.5, fma(mx, gp[r], my * gp[4 + r]), qp[r]);
    }
    Prim s0;
    const bool ok = q_to_prim<POW>(qt0, fp, s0);
    double G0[4];
    split_flux(s0, N.x, N.y, -1.0, G0);
    const double wm = fma(dm, w[6], -(ds * w[7]));
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = fma(wm, Ginf[r] - G0[r], R[r]);
    return ok;
}

// Gn-(q_inf) along the unit normal N for the case's conserved freestream u
// (the same q -> primitive -> split-flux path as every modified state, so a
// freestream state gives bitwise equal fluxes).
template <int POW>
__device__ __forceinline__ bool freestream_flux(const double *u, double2 N, const FlowParams &fp,
                                                double G[4]) {
    const double v[4] = {u[0], u[1], u[2], u[3]};
    double qi[4];
    bool ok = cons_to_q(v, fp, qi) == kErrNone;
    Prim si;
    ok &= q_to_prim<POW>(qi, fp, si);
    split_flux(si, N.x, N.y, -1.0, G);
    return ok;
}

// SSP-RK(4,3) stage of point p with L = -R:
//   U1 = Un + dt/2 L(Un); U2 = U1 + dt/2 L(U1);
//   U3 = 2/3 Un + 1/3 (U2 + dt/2 L(U2)); U4 = U3 + dt/2 L(U3);
// then the wall projection, q of the new state into qnext (and its FP32
// shadow), and at stage 4 the next iteration's Un and time step.
__device__ __forceinline__ void rk_update(const DevCloud &cl, const FlowParams &fp, int stage,
                                          int p, uint8_t kd, double2 N, const double R[4],
                                          double *U, double *Un, double *dt, double2 *qnext,
                                          float4 *q32next, ErrWord *err) {
    const int n = cl.n;
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
        report_pt(cl, err, p, e);
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

}  // namespace

// ---------------------------------------------------------------------------
// Flux residual + Runge-Kutta stage, LDS-tiled.
//
// A workgroup owns a tile of kFluxTile consecutive points (a compact patch in
// Hilbert order) and serves each point with kFluxLanes lanes: lane l walks the
// point's neighbour entries l, l + kFluxLanes, ... and the partial sums are
// combined by lane_group_sum, so every point's residual is summed in one fixed
// order.  The records that the entries gather (q, q-derivatives, limiter
// bounds, position) of the tile's points and of its halo are first copied
// into LDS; each is read from memory once per tile instead of once per use.
// A tile whose image exceeds the capacity `cap` (slots) reads straight from
// memory (a branch uniform across the workgroup), with the same arithmetic.
//
// stage 0: evaluate R only (into Rout).  stage 1..4: residual + rk_update;
// stage 1 also writes R to Rout for the residual norm.  Frozen points, and
// outer points unless KOBC, are held (q copied to qnext) and carry R = 0.
// Kinetic outer condition (fp.kobc): outer points take their s+, s-, n+
// terms like any point and are updated; the launch that holds n- (M) adds
// the mirrored n- term of mirror_entry (template flag KOBC = fp.kobc there).
// M: the split stencils of this launch (15: all; split launches add the
// other stencils' partial sums Rin).
// ---------------------------------------------------------------------------
int num_flux_tiles(int n) { return (n + kFluxTile - 1) / kFluxTile; }

int sweep_grid(const DevCloud &c) { return c.tile_list ? c.ntile_live : num_flux_tiles(c.n); }

namespace {

// Residual sums of live point p (slot j of its tile) over its entries
// sub, sub + kFluxLanes, ...; IN_LDS: the records come from the tile's LDS
// image, else from memory (one instantiation each, so that no load is
// generic).  Reports a failed reconstruction.
template <bool IN_LDS, bool LIMITER, int POW, bool FIRST, int M, bool KOBC>
__device__ __forceinline__ void flux_point(const DevCloud &cl, const FlowParams &fp,
                                           const double2 *lds, int j, int p, int sub, uint8_t kd,
                                           double2 N, const double2 *q, const double2 *g,
                                           const double2 *qmm, double R[4], ErrWord *err) {
    constexpr int kRec = FIRST ? 3 : (LIMITER ? 11 : 7);
    double qp[4], gp[8], bp[8], w[8];
    const double2 P = cl.xy[p];
    if constexpr (IN_LDS) {
        const double2 *r = lds + kRec * j;
        qp[0] = r[0].x; qp[1] = r[0].y; qp[2] = r[1].x; qp[3] = r[1].y;
#pragma unroll
        for (int m = 0; m < 4 && !FIRST; ++m) {
            gp[2 * m] = r[2 + m].x;
            gp[2 * m + 1] = r[2 + m].y;
            if (LIMITER) {
                bp[2 * m] = r[6 + m].x;
                bp[2 * m + 1] = r[6 + m].y;
            }
        }
    } else {
        load4(q, p, qp);
        if (!FIRST) load8(g, p, gp);
        if (LIMITER) load8(qmm, p, bp);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) w[m] = cl.lsw[8 * p + m];
    // walls drop n+ (its stencil lies in the body), outer points n- (it
    // lies beyond the far field; the mirrored term below replaces it)
    uint8_t fmask = ((kd == kWall) ? uint8_t(~kNPlus) : uint8_t(0xff)) & uint8_t(M);
    if constexpr (KOBC) {
        if (kd == kOuter) fmask &= uint8_t(~kNMinus);
    }
    const int k1 = cl.ptr[p + 1];
    bool ok = true;
#pragma unroll 2
    for (int k = cl.ptr[p] + sub; k < k1; k += kFluxLanes) {
        const uint8_t f = cl.flag[k] & fmask;
        if (f == 0) continue;
        double qi[4], gi[8], bi[8];
        double2 Q;
        if constexpr (IN_LDS) {
            const double2 *r = lds + kRec * (int)cl.flidx[k];
            qi[0] = r[0].x; qi[1] = r[0].y; qi[2] = r[1].x; qi[3] = r[1].y;
#pragma unroll
            for (int m = 0; m < 4 && !FIRST; ++m) {
                gi[2 * m] = r[2 + m].x;
                gi[2 * m + 1] = r[2 + m].y;
                if (LIMITER) {
                    bi[2 * m] = r[6 + m].x;
                    bi[2 * m + 1] = r[6 + m].y;
                }
            }
            Q = r[kRec - 1];
        } else {
            const int i = cl.idx[k];
            load4(q, i, qi);
            if (!FIRST) load8(g, i, gi);
            if (LIMITER) load8(qmm, i, bi);
            Q = cl.xy[i];
        }
        ok &= flux_entry<LIMITER, POW, FIRST, M>(f, Q.x - P.x, Q.y - P.y, N, qi, gi, bi, qp, gp,
                                                 bp, w, fp, R);
    }
    if constexpr (KOBC && (M & kNMinus)) {
        if (kd == kOuter) {
            double Ginf[4];
            ok &= freestream_flux<POW>(cl.uinf + 4 * cl.case_of[p], N, fp, Ginf);
            for (int k = cl.ptr[p] + sub; k < k1; k += kFluxLanes) {
                if (!(cl.flag[k] & kNPlus)) continue;
                const double2 Q = IN_LDS ? lds[kRec * (int)cl.flidx[k] + kRec - 1]
                                         : cl.xy[cl.idx[k]];
                ok &= mirror_entry<LIMITER, POW, FIRST>(Q.x - P.x, Q.y - P.y, N, qp, gp, bp, w,
                                                        Ginf, fp, R);
            }
        }
    }
    if (!ok) report_pt(cl, err, p, kErrPositivity);
}

}  // namespace

template <bool LIMITER, int POW, bool FIRST, int M, bool KOBC>
// Held to 3 waves per SIMD (at most 168 VGPRs), which the straight-line
// two-direction body of flux_entry would otherwise exceed.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_flux(DevCloud cl, FlowParams fp, int stage, int cap,
                                                 const double *__restrict__ Rin,
                                                 const double2 *__restrict__ q,
                                                 const double2 *__restrict__ g,
                                                 const double2 *__restrict__ qmm,
                                                 double *__restrict__ U, double *__restrict__ Un,
                                                 double *__restrict__ dt,
                                                 double2 *__restrict__ qnext,
                                                 double *__restrict__ Rout,
                                                 float4 *__restrict__ q32next, ErrWord *err) {
    // slot record (double2): q 0..1, g 2..5, bound offsets 6..9, position last
    // (first order: q and position only)
    constexpr int kRec = FIRST ? 3 : (LIMITER ? 11 : 7);
    extern __shared__ double2 lds[];
    const int n = cl.n;
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    if (cl.tile_prec && cl.tile_prec[t] != 0) return;  // an FP32-flux tile
    const int base = t * kFluxTile;
    const int nown = min(kFluxTile, n - base);
    int h0 = 0, ns = 0;
    if (cl.fhalo_ptr) {
        h0 = cl.fhalo_ptr[t];
        ns = kFluxTile + cl.fhalo_ptr[t + 1] - h0;
    }
    const bool in_lds = cl.fhalo_ptr != nullptr && ns <= cap;
    if (in_lds) {
        auto slot_point = [&](int s) {
            return s < kFluxTile ? base + s : cl.fhalo_idx[h0 + s - kFluxTile];
        };
        for (int e = threadIdx.x; e < 2 * ns; e += kBlock) {
            const int s = e >> 1;
            if (s >= nown && s < kFluxTile) continue;
            lds[kRec * s + (e & 1)] = q[2 * slot_point(s) + (e & 1)];
        }
        for (int e = threadIdx.x; !FIRST && e < 4 * ns; e += kBlock) {
            const int s = e >> 2;
            if (s >= nown && s < kFluxTile) continue;
            const int pt = slot_point(s);
            lds[kRec * s + 2 + (e & 3)] = g[4 * pt + (e & 3)];
            if (LIMITER) lds[kRec * s + 6 + (e & 3)] = qmm[4 * pt + (e & 3)];
        }
        for (int s = threadIdx.x; s < ns; s += kBlock) {
            if (s >= nown && s < kFluxTile) continue;
            lds[kRec * s + kRec - 1] = cl.xy[slot_point(s)];
        }
    }
    __syncthreads();
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = base + j;
    double R[4] = {0.0, 0.0, 0.0, 0.0};
    uint8_t kd = kOuter;
    bool live = false;
    if (j < nown) {
        kd = cl.kind[p];
        const bool frozen = cl.case_active && !cl.case_active[cl.case_of[p]];
        // outer points are live under the kinetic outer condition: KOBC
        // launches, and split launches without the n- stencil (whose
        // template flag stays false) when fp.kobc is set
        bool outer_live = KOBC;
        if constexpr (!KOBC && !(M & kNMinus)) outer_live = fp.kobc != 0;
        live = (outer_live || kd != kOuter) && !frozen;
    }
    double2 N = make_double2(0.0, 0.0);
    if (live) {
        N = cl.nrm[p];
        if (in_lds)
            flux_point<true, LIMITER, POW, FIRST, M, KOBC>(cl, fp, lds, j, p, sub, kd, N, q, g,
                                                           qmm, R, err);
        else
            flux_point<false, LIMITER, POW, FIRST, M, KOBC>(cl, fp, lds, j, p, sub, kd, N, q, g,
                                                            qmm, R, err);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = lane_group_sum(R[r]);
    if (j >= nown || sub != 0) return;
    if (Rin && live) {  // the other directions' part (split launches)
#pragma unroll
        for (int r = 0; r < 4; ++r) R[r] += Rin[(size_t)r * n + p];
    }
    if (!live) {
        if (stage > 0) {
            double qv[4];
            load4(q, p, qv);
            store4(qnext, p, qv);
            if (q32next) q32next[p] = to_f4(qv);
        }
        if (Rout) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = 0.0;
        }
        return;
    }
    if (Rout) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = R[r];
    }
    if (stage > 0) rk_update(cl, fp, stage, p, kd, N, R, U, Un, dt, qnext, q32next, err);
}

namespace {

template <bool B>
using BoolC = std::integral_constant<bool, B>;
template <int V>
using IntC = std::integral_constant<int, V>;

// call f(BoolC<limiter>, IntC<pow>, BoolC<kobc>) for the run-time flags
// (pow: 5 for gamma = 1.4, else the general form 0)
template <class F>
void dispatch_flow(const FlowParams &fp, F &&f) {
    auto with_pow = [&](auto lim, auto kobc) {
        if (fp.sqrt_pow == 5) f(lim, IntC<5>{}, kobc);
        else f(lim, IntC<0>{}, kobc);
    };
    auto with_kobc = [&](auto lim) {
        if (fp.kobc) with_pow(lim, BoolC<true>{});
        else with_pow(lim, BoolC<false>{});
    };
    if (fp.limiter) with_kobc(BoolC<true>{});
    else with_kobc(BoolC<false>{});
}

}  // namespace

hipError_t launch_flux(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                       int lds_budget, const double2 *q, const double2 *g, const double2 *qmm,
                       double *U, double *Un, double *dt, double2 *qnext, double *Rout,
                       float4 *q32next, ErrWord *err, int split, double *const Rpart[2]) {
    const bool first = fp.order == 1;
    const int rec = (first ? 3 : fp.limiter ? 11 : 7) * (int)sizeof(double2);
    const int cap = lds_cap(c, lds_budget, rec);
    const size_t shmem = (size_t)cap * rec;
    const dim3 grid(sweep_grid(c)), block(kBlock);
    auto go = [&](auto kern, int stg, const double *rin, double *rout) {
        hipLaunchKernelGGL(kern, grid, block, shmem, st, c, fp, stg, cap, rin, q, g, qmm, U, Un,
                           dt, qnext, rout, q32next, err);
    };
    if (first) {  // first order: one fused launch
        if (fp.sqrt_pow == 5) {
            if (fp.kobc) go(k_flux<false, 5, true, 15, true>, stage, nullptr, Rout);
            else go(k_flux<false, 5, true, 15, false>, stage, nullptr, Rout);
        } else {
            if (fp.kobc) go(k_flux<false, 0, true, 15, true>, stage, nullptr, Rout);
            else go(k_flux<false, 0, true, 15, false>, stage, nullptr, Rout);
        }
        return hipGetLastError();
    }
    dispatch_flow(fp, [&](auto lim, auto pw, auto kobc) {
        constexpr bool L = decltype(lim)::value, K = decltype(kobc)::value;
        constexpr int P = decltype(pw)::value;
        if (split == 2) {
            // the s directions, then the n directions with the update
            go(k_flux<L, P, false, kSPlus | kSMinus, false>, 0, nullptr, Rpart[0]);
            go(k_flux<L, P, false, kNPlus | kNMinus, K>, stage, Rpart[0], Rout);
        } else if (split == 4) {
            // one launch per split stencil, the last with the update
            go(k_flux<L, P, false, kSPlus, false>, 0, nullptr, Rpart[0]);
            go(k_flux<L, P, false, kSMinus, false>, 0, Rpart[0], Rpart[1]);
            go(k_flux<L, P, false, kNPlus, false>, 0, Rpart[1], Rpart[0]);
            go(k_flux<L, P, false, kNMinus, K>, stage, Rpart[0], Rout);
        } else {
            go(k_flux<L, P, false, 15, K>, stage, nullptr, Rout);
        }
    });
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mixed precision flux residual + Runge-Kutta stage.  The reconstruction
// (eq. (28)), the limiter and the split fluxes run in FP32 from the FP32
// shadows of q, its derivatives and its bound offsets, using the hardware FP32
// exp / sqrt / reciprocal; the geometry, the least-squares weights, the
// residual sums and the state update stay FP64.  Same tiling and lane
// layout as k_flux; the LDS image holds the FP32 records (16-byte q, 32-byte
// derivatives and bounds) and the FP64 positions.
// ---------------------------------------------------------------------------
namespace {

struct PrimF {
    float rho, u1, u2, p, sqb, isqb, rhoe;
};

template <int POW>
__device__ __forceinline__ bool q_to_prim_f(const float qt[4], float gm1inv, PrimF &s) {
#pragma clang fp contract(off)
    const float beta = -0.5f * qt[3];
    const float inv2b = -__builtin_amdgcn_rcpf(qt[3]);
    s.u1 = qt[1] * inv2b;
    s.u2 = qt[2] * inv2b;
    const float uu = fmaf(s.u1, s.u1, s.u2 * s.u2);
    s.isqb = __builtin_amdgcn_rsqf(beta);
    s.sqb = beta * s.isqb;
    if (POW > 0) {
        s.rho = __expf(fmaf(beta, uu, qt[0])) * ipow<POW>(s.isqb);
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
    const float E = __expf(-(S * S));
    const float A = half_erfc_f(-sg * S, E, __builtin_amdgcn_rcpf(kErfcC32 + fabsf(S)));
    const float B = (E * kHalfRsqrtPi) * s.isqb;
    const float sB = sg * B;
    const float mass = s.rho * fmaf(ue, A, sB);
    const float pA = s.p * A;
    G[0] = mass;
    G[1] = fmaf(s.u1, mass, pA * ex);
    G[2] = fmaf(s.u2, mass, pA * ey);
    G[3] = fmaf((s.p + s.rhoe) * ue, A, (fmaf(0.5f, s.p, s.rhoe)) * sB);
}

// FP32 counterpart of venkat (eps^2 kept at least 1e-30 by the caller)
__device__ __forceinline__ float venkat_f(float delta, float dmax, float dmin, float eps2) {
#pragma clang fp contract(off)
    const float D = (delta > 0.0f) ? dmax : dmin;
    const float a = fmaf(D, D, eps2);
    const float num = fmaf(2.0f * delta, D, a);
    const float den = fmaf(delta, D, fmaf(2.0f * delta, delta, a));
    return num * __builtin_amdgcn_rcpf(den);
}

__device__ __forceinline__ void unpack(const float4 a, float *v) {
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// FP32 counterpart of flux_entry; the weights and sums stay FP64.
template <bool LIMITER, int POW, bool FIRST>
__device__ __forceinline__ bool flux_entry_f(uint8_t f, double dx, double dy, double2 N,
                                             const float qi[4], const float gi[8],
                                             const float bi[8], const float qp[4],
                                             const float gp[8], const float bp[8],
                                             const double w[8], float gm1inv, float vk,
                                             double R[4]) {
#pragma clang fp contract(off)
    const double tx = N.y, ty = -N.x;
    const double ds = fma(dx, tx, dy * ty);
    const double dn = fma(dx, N.x, dy * N.y);
    const float dxf = (float)dx, dyf = (float)dy;
    float qti[4], qt0[4];
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qti[r] = qi[r];
            qt0[r] = qp[r];
        }
    } else if (LIMITER) {
        const float e = vk * __builtin_amdgcn_sqrtf(fmaf(dxf, dxf, dyf * dyf));
        const float eps2 = fmaxf((e * e) * e, 1e-30f);
        const float hx = -0.5f * dxf, hy = -0.5f * dyf;  // as in flux_entry
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float di = fmaf(hx, gi[r], hy * gi[4 + r]);
            const float d0 = fmaf(hx, gp[r], hy * gp[4 + r]);
            qti[r] = fmaf(venkat_f(di, bi[r], bi[4 + r], eps2), di, qi[r]);
            qt0[r] = fmaf(venkat_f(d0, bp[r], bp[4 + r], eps2), d0, qp[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qti[r] = fmaf(-0.5f, fmaf(dxf, gi[r], dyf * gi[4 + r]), qi[r]);
            qt0[r] = fmaf(-0.5f, fmaf(dxf, gp[r], dyf * gp[4 + r]), qp[r]);
        }
    }
    PrimF si, s0;
    bool ok = q_to_prim_f<POW>(qti, gm1inv, si);
    ok &= q_to_prim_f<POW>(qt0, gm1inv, s0);
    // both directions as straight-line code, as in flux_entry
    float Gs[2][4], Gn[2][4];
    const bool sp = (f & kSPlus) != 0, np_ = (f & kNPlus) != 0;
    const double ws = (f & (kSPlus | kSMinus))
                          ? fma(ds, sp ? w[0] : w[2], -(dn * (sp ? w[1] : w[3]))) : 0.0;
    const double wn = (f & (kNPlus | kNMinus))
                          ? fma(dn, np_ ? w[4] : w[6], -(ds * (np_ ? w[5] : w[7]))) : 0.0;
    split_flux_f(si, (float)tx, (float)ty, sp ? 1.0f : -1.0f, Gs[0]);
    split_flux_f(s0, (float)tx, (float)ty, sp ? 1.0f : -1.0f, Gs[1]);
    split_flux_f(si, (float)N.x, (float)N.y, np_ ? 1.0f : -1.0f, Gn[0]);
    split_flux_f(s0, (float)N.x, (float)N.y, np_ ? 1.0f : -1.0f, Gn[1]);
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = fma(ws, (double)(Gs[0][r] - Gs[1][r]), R[r]);
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = fma(wn, (double)(Gn[0][r] - Gn[1][r]), R[r]);
    return ok;
}

// FP32 counterpart of mirror_entry; the weight and the sums stay FP64.
template <bool LIMITER, int POW, bool FIRST>
__device__ __forceinline__ bool mirror_entry_f(double dx, double dy, double2 N, const float qp[4],
                                               const float gp[8], const float bp[8],
                                               const double w[8], const float Ginf[4],
                                               float gm1inv, float vk, double R[4]) {
#pragma clang fp contract(off)
    const double tx = N.y, ty = -N.x;
    const double ds = fma(dx, tx, dy * ty);
    const double dm = -fma(dx, N.x, dy * N.y);
    const float mx = (float)fma(ds, tx, dm * N.x), my = (float)fma(ds, ty, dm * N.y);
    float qt0[4];
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) qt0[r] = qp[r];
    } else if (LIMITER) {
        const float e = vk * __builtin_amdgcn_sqrtf(fmaf(mx, mx, my * my));
        const float eps2 = fmaxf((e * e) * e, 1e-30f);
        const float hx = -0.5f * mx, hy = -0.5f * my;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d0 = fmaf(hx, gp[r], hy * gp[4 + r]);
            qt0[r] = fmaf(venkat_f(d0, bp[r], bp[4 + r], eps2), d0, qp[r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) qt0[r] = fmaf(-0.5f, fmaf(mx, gp[r], my * gp[4 + r]), qp[r]);
    }
    PrimF s0;
    const bool ok = q_to_prim_f<POW>(qt0, gm1inv, s0);
    float G0[4];
    split_flux_f(s0, (float)N.x, (float)N.y, -1.0f, G0);
    const double wm = fma(dm, w[6], -(ds * w[7]));
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = fma(wm, (double)(Ginf[r] - G0[r]), R[r]);
    return ok;
}

// FP32 Gn-(q_inf): q of the conserved freestream in FP64 (as the state's own
// q and its FP32 shadow are formed), then the FP32 flux path.
template <int POW>
__device__ __forceinline__ bool freestream_flux_f(const double *u, double2 N,
                                                  const FlowParams &fp, float G[4]) {
    const double v[4] = {u[0], u[1], u[2], u[3]};
    double qi[4];
    bool ok = cons_to_q(v, fp, qi) == kErrNone;
    const float qf[4] = {(float)qi[0], (float)qi[1], (float)qi[2], (float)qi[3]};
    PrimF si;
    ok &= q_to_prim_f<POW>(qf, (float)fp.gm1inv, si);
    split_flux_f(si, (float)N.x, (float)N.y, -1.0f, G);
    return ok;
}

// Mixed-precision residual sums of live point p, as flux_point: IN_LDS
// selects where the FP32 records and positions come from.
template <bool IN_LDS, bool LIMITER, int POW, bool FIRST, bool KOBC>
__device__ __forceinline__ void flux_point_f(const DevCloud &cl, const FlowParams &fp,
                                             const float4 *ldsf, const double2 *lxy, int j, int p,
                                             int sub, uint8_t kd, double2 N,
                                             const float4 *q32, const float4 *g32,
                                             const float4 *qmm32, double R[4], ErrWord *err) {
    constexpr int kRec = FIRST ? 1 : (LIMITER ? 5 : 3);
    const float gm1inv = (float)fp.gm1inv;
    const float vk = (float)fp.venkat_k;
    float qp[4], gp[8], bp[8];
    double w[8];
    const double2 P = cl.xy[p];
    if constexpr (IN_LDS) {
        const float4 *r = ldsf + kRec * j;
        unpack(r[0], qp);
        if (!FIRST) {
            unpack(r[1], gp);
            unpack(r[2], gp + 4);
        }
        if (LIMITER) {
            unpack(r[3], bp);
            unpack(r[4], bp + 4);
        }
    } else {
        unpack(q32[p], qp);
        if (!FIRST) {
            unpack(g32[2 * p], gp);
            unpack(g32[2 * p + 1], gp + 4);
        }
        if (LIMITER) {
            unpack(qmm32[2 * p], bp);
            unpack(qmm32[2 * p + 1], bp + 4);
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) w[m] = cl.lsw[8 * p + m];
    uint8_t fmask = (kd == kWall) ? uint8_t(~kNPlus) : uint8_t(0xff);
    if constexpr (KOBC) {
        if (kd == kOuter) fmask &= uint8_t(~kNMinus);
    }
    const int k1 = cl.ptr[p + 1];
    bool ok = true;
#pragma unroll 2
    for (int k = cl.ptr[p] + sub; k < k1; k += kFluxLanes) {
        const uint8_t f = cl.flag[k] & fmask;
        if (f == 0) continue;
        float qi[4], gi[8], bi[8];
        double2 Q;
        if constexpr (IN_LDS) {
            const int s = cl.flidx[k];
            const float4 *r = ldsf + kRec * s;
            unpack(r[0], qi);
            if (!FIRST) {
                unpack(r[1], gi);
                unpack(r[2], gi + 4);
            }
            if (LIMITER) {
                unpack(r[3], bi);
                unpack(r[4], bi + 4);
            }
            Q = lxy[s];
        } else {
            const int i = cl.idx[k];
            unpack(q32[i], qi);
            if (!FIRST) {
                unpack(g32[2 * i], gi);
                unpack(g32[2 * i + 1], gi + 4);
            }
            if (LIMITER) {
                unpack(qmm32[2 * i], bi);
                unpack(qmm32[2 * i + 1], bi + 4);
            }
            Q = cl.xy[i];
        }
        ok &= flux_entry_f<LIMITER, POW, FIRST>(f, Q.x - P.x, Q.y - P.y, N, qi, gi, bi, qp, gp,
                                                bp, w, gm1inv, vk, R);
    }
    if constexpr (KOBC) {
        if (kd == kOuter) {
            float Ginf[4];
            ok &= freestream_flux_f<POW>(cl.uinf + 4 * cl.case_of[p], N, fp, Ginf);
            for (int k = cl.ptr[p] + sub; k < k1; k += kFluxLanes) {
                if (!(cl.flag[k] & kNPlus)) continue;
                const double2 Q = IN_LDS ? lxy[cl.flidx[k]] : cl.xy[cl.idx[k]];
                ok &= mirror_entry_f<LIMITER, POW, FIRST>(Q.x - P.x, Q.y - P.y, N, qp, gp, bp,
                                                          w, Ginf, gm1inv, vk, R);
            }
        }
    }
    if (!ok) report_pt(cl, err, p, kErrPositivity);
}

}  // namespace

template <bool LIMITER, int POW, bool FIRST, bool KOBC>
// held to 4 waves per SIMD (at most 128 VGPRs), as k_flux is to 3
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_flux_mixed(
    DevCloud cl, FlowParams fp, int stage, int cap, const double2 *__restrict__ q,
    const float4 *__restrict__ q32, const float4 *__restrict__ g32,
    const float4 *__restrict__ qmm32, double *__restrict__ U, double *__restrict__ Un,
    double *__restrict__ dt, double2 *__restrict__ qnext, float4 *__restrict__ q32next,
    double *__restrict__ Rout, ErrWord *err) {
    // slot record (float4): q 0, g 1..2, bounds 3..4 (first order: q only);
    // positions after cap records
    constexpr int kRec = FIRST ? 1 : (LIMITER ? 5 : 3);
    extern __shared__ float4 ldsf[];
    double2 *lxy = reinterpret_cast<double2 *>(ldsf + (size_t)kRec * cap);
    const int n = cl.n;
    const int t = sweep_tile(cl);
    if (cl.tile_active && !cl.tile_active[t]) return;
    if (cl.tile_prec && cl.tile_prec[t] != 1) return;  // an FP64-flux tile
    const int base = t * kFluxTile;
    const int nown = min(kFluxTile, n - base);
    int h0 = 0, ns = 0;
    if (cl.fhalo_ptr) {
        h0 = cl.fhalo_ptr[t];
        ns = kFluxTile + cl.fhalo_ptr[t + 1] - h0;
    }
    const bool in_lds = cl.fhalo_ptr != nullptr && ns <= cap;
    if (in_lds) {
        auto slot_point = [&](int s) {
            return s < kFluxTile ? base + s : cl.fhalo_idx[h0 + s - kFluxTile];
        };
        for (int e = threadIdx.x; !FIRST && e < 2 * ns; e += kBlock) {
            const int s = e >> 1;
            if (s >= nown && s < kFluxTile) continue;
            const int pt = slot_point(s);
            ldsf[kRec * s + 1 + (e & 1)] = g32[2 * pt + (e & 1)];
            if (LIMITER) ldsf[kRec * s + 3 + (e & 1)] = qmm32[2 * pt + (e & 1)];
        }
        for (int s = threadIdx.x; s < ns; s += kBlock) {
            if (s >= nown && s < kFluxTile) continue;
            const int pt = slot_point(s);
            ldsf[kRec * s] = q32[pt];
            lxy[s] = cl.xy[pt];
        }
    }
    __syncthreads();
    const int j = threadIdx.x / kFluxLanes, sub = threadIdx.x % kFluxLanes;
    const int p = base + j;
    double R[4] = {0.0, 0.0, 0.0, 0.0};
    uint8_t kd = kOuter;
    bool live = false;
    if (j < nown) {
        kd = cl.kind[p];
        const bool frozen = cl.case_active && !cl.case_active[cl.case_of[p]];
        live = (KOBC || kd != kOuter) && !frozen;
    }
    double2 N = make_double2(0.0, 0.0);
    if (live) {
        N = cl.nrm[p];
        if (in_lds)
            flux_point_f<true, LIMITER, POW, FIRST, KOBC>(cl, fp, ldsf, lxy, j, p, sub, kd, N,
                                                          q32, g32, qmm32, R, err);
        else
            flux_point_f<false, LIMITER, POW, FIRST, KOBC>(cl, fp, ldsf, lxy, j, p, sub, kd, N,
                                                           q32, g32, qmm32, R, err);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) R[r] = lane_group_sum(R[r]);
    if (j >= nown || sub != 0) return;
    if (!live) {
        if (stage > 0) {
            double qv[4];
            load4(q, p, qv);
            store4(qnext, p, qv);
            q32next[p] = q32[p];
        }
        if (Rout) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = 0.0;
        }
        return;
    }
    if (Rout) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Rout[(size_t)r * n + p] = R[r];
    }
    if (stage > 0) rk_update(cl, fp, stage, p, kd, N, R, U, Un, dt, qnext, q32next, err);
}

hipError_t launch_flux_mixed(hipStream_t st, const DevCloud &c, const FlowParams &fp, int stage,
                             int lds_budget, const double2 *q, const float4 *q32,
                             const float4 *g32, const float4 *qmm32, double *U, double *Un,
                             double *dt, double2 *qnext, float4 *q32next, double *Rout,
                             ErrWord *err) {
    const bool first = fp.order == 1;
    const int rec = ((first ? 1 : fp.limiter ? 5 : 3) + 1) * (int)sizeof(float4);
    const int cap = lds_cap(c, lds_budget, rec);
    const size_t shmem = (size_t)cap * rec;
    const dim3 grid(sweep_grid(c)), block(kBlock);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, shmem, st, c, fp, stage, cap, q, q32, g32, qmm32, U,
                           Un, dt, qnext, q32next, Rout, err);
    };
    dispatch_flow(fp, [&](auto lim, auto pw, auto kobc) {
        constexpr bool L = decltype(lim)::value, K = decltype(kobc)::value;
        constexpr int P = decltype(pw)::value;
        if (first) go(k_flux_mixed<false, P, true, K>);  // the limiter is unused
        else go(k_flux_mixed<L, P, false, K>);
    });
    return hipGetLastError();
}

// Residual norms per case, in a fixed summation order.  Points are split into
// chunks that never straddle a case (chunk ch = [beg[ch], beg[ch+1])); one
// workgroup sums R_c^2 over a chunk, then one workgroup per case adds that
// case's chunk sums and writes sqrt(sum / updated points) into history row
// (*ctr), and *ctr advances (replays of a captured iteration need no host
// bookkeeping).  Held (outer without the kinetic outer condition) points
// carry R = 0.  In a batched run with retirement the chunks and the norms
// of retired cases are skipped (their last norms are kept in rt.last).
__global__ void __launch_bounds__(kBlock) k_res_chunks(const double *__restrict__ R, int n,
                                                       const int *__restrict__ beg,
                                                       double *__restrict__ part,
                                                       const int *__restrict__ case_of,
                                                       const uint8_t *__restrict__ active) {
    __shared__ double red[kBlock / 64][4];
    const int ch = blockIdx.x;
    const int b = beg[ch], e = beg[ch + 1];
    if (active && b < e && !active[case_of[b]]) return;
    double acc[4] = {0, 0, 0, 0};
    for (int p = b + threadIdx.x; p < e; p += kBlock) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double r = R[(size_t)c * n + p];
            acc[c] += r * r;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double t = wave_sum(acc[c]);
        if (lane == 0) red[wv][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) t += red[j][threadIdx.x];
        part[4 * ch + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_res_cases(int ncase, const int *__restrict__ chunk_ptr,
                                                      const double *__restrict__ part,
                                                      const double *__restrict__ inv_nupd,
                                                      int *ctr, int cap,
                                                      double *__restrict__ hist, Retire rt) {
    __shared__ double red[kBlock / 64][4];
    __shared__ double nv[4];
    const int row = *ctr;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double drop = rt.on ? *rt.drop : 0.0;
    // workgroup cs takes case cs (one workgroup: every case in turn, and it
    // advances the row counter itself)
    for (int cs = blockIdx.x; cs < ncase; cs += gridDim.x) {
        if (rt.on && !rt.active[cs]) continue;
        double acc[4] = {0, 0, 0, 0};
        for (int j = chunk_ptr[cs] + threadIdx.x; j < chunk_ptr[cs + 1]; j += kBlock) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += part[4 * j + c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double t = wave_sum(acc[c]);
            if (lane == 0) red[wv][c] = t;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < kBlock / 64; ++j) t += red[j][threadIdx.x];
            const double v = sqrt(t * inv_nupd[cs]);
            if (row < cap) hist[((size_t)row * ncase + cs) * 4 + threadIdx.x] = v;
            nv[threadIdx.x] = v;
        }
        __syncthreads();
        // retirement: this iteration's norms are those of the state it
        // started from, and the state it leaves is the one a case keeps
        if (rt.on && threadIdx.x == 0 && rt.active[cs]) {
            rt.iters[cs] += 1;
#pragma unroll
            for (int c = 0; c < 4; ++c) rt.last[4 * cs + c] = nv[c];
            double ref = rt.ref[cs];
            if (ref < 0.0) ref = rt.ref[cs] = nv[0];
            if (rt.prec && rt.prec[cs] && nv[0] <= *rt.sw * ref) {
                rt.prec[cs] = 0;
                rt.sw_iter[cs] = rt.iters[cs];
            }
            if (rt.case_err[cs] != kErrClear || nv[0] <= drop * ref ||
                nv[0] > kDiverged * ref || !(nv[0] == nv[0]))
                rt.active[cs] = 0;
        }
    }
    if (gridDim.x == 1 && threadIdx.x == 0) *ctr = row + 1;
}

// advances the history row counter after a k_res_cases of several workgroups
__global__ void k_res_advance(int *ctr) { *ctr += 1; }

// tile t is skipped by every tiled sweep when no case it holds is active;
// its split fluxes are FP32 only while every case it holds is (case_prec
// nullable: no precision switch)
__global__ void __launch_bounds__(kBlock) k_tile_active(int n, int ntile,
                                                        const int *__restrict__ case_of,
                                                        const uint8_t *__restrict__ case_active,
                                                        uint8_t *__restrict__ tile_active,
                                                        const uint8_t *__restrict__ case_prec,
                                                        uint8_t *__restrict__ tile_prec) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ntile) return;
    const int b = t * kFluxTile, e = min(n, b + kFluxTile) - 1;
    uint8_t any = 0, all32 = 1;
    for (int c = case_of[b]; c <= case_of[e]; ++c) {
        any |= case_active[c];
        if (case_prec) all32 &= case_prec[c];
    }
    tile_active[t] = any;
    if (case_prec) tile_prec[t] = all32;
}

hipError_t launch_resnorm(hipStream_t st, const double *R, int n, int nchunk, const int *chunk_beg,
                          double *part, int ncase, const int *chunk_ptr, const double *inv_nupd,
                          int *ctr, int cap, double *hist, const Retire &rt,
                          const int *case_of, uint8_t *tile_active, uint8_t *tile_prec) {
    hipLaunchKernelGGL(k_res_chunks, dim3(nchunk), dim3(kBlock), 0, st, R, n, chunk_beg, part,
                       case_of, rt.on ? rt.active : nullptr);
    hipLaunchKernelGGL(k_res_cases, dim3(ncase), dim3(kBlock), 0, st, ncase, chunk_ptr, part,
                       inv_nupd, ctr, cap, hist, rt);
    if (ncase > 1) hipLaunchKernelGGL(k_res_advance, dim3(1), dim3(1), 0, st, ctr);
    if (rt.on) {
        const int ntile = num_flux_tiles(n);
        hipLaunchKernelGGL(k_tile_active, dim3((ntile + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                           n, ntile, case_of, rt.active, tile_active, rt.prec, tile_prec);
    }
    return hipGetLastError();
}

// Forces from the wall pressure; wall[j] lists the wall points in the
// caller's order (the surface polygon).  Each thread sums a contiguous run of
// the polygon in order, then the runs are added in thread order, separately
// for the upper, lower and on-axis points (a fixed summation order).
__global__ void __launch_bounds__(kBlock) k_forces(int nw, const int *__restrict__ wall,
                                                   const double2 *__restrict__ xy,
                                                   const double2 *__restrict__ nrm,
                                                   const double *__restrict__ U, int n,
                                                   double gamma, double pinf,
                                                   double *__restrict__ f,
                                                   double *__restrict__ out) {
    (void)f;
    __shared__ double part[kBlock][6];
    const int per = (nw + kBlock - 1) / kBlock;
    const int j0 = threadIdx.x * per, j1 = min(nw, j0 + per);
    double F[6] = {0, 0, 0, 0, 0, 0};
    for (int j = j0; j < j1; ++j) {
        const int p = wall[j], pn = wall[(j + 1) % nw], pp = wall[(j + nw - 1) % nw];
        const double2 P = xy[p], Pn = xy[pn], Pp = xy[pp];
        const double ds = 0.5 * (sqrt((Pn.x - P.x) * (Pn.x - P.x) + (Pn.y - P.y) * (Pn.y - P.y)) +
                                 sqrt((P.x - Pp.x) * (P.x - Pp.x) + (P.y - Pp.y) * (P.y - Pp.y)));
        const double rho = U[p];
        const double u1 = U[(size_t)n + p] / rho, u2 = U[(size_t)2 * n + p] / rho;
        const double pr = (gamma - 1.0) * (U[(size_t)3 * n + p] - 0.5 * rho * (u1 * u1 + u2 * u2));
        const double2 N = nrm[p];
        const int h = (P.y > 0.0) ? 0 : (P.y < 0.0) ? 1 : 2;
        F[2 * h] += -(pr - pinf) * N.x * ds;
        F[2 * h + 1] += -(pr - pinf) * N.y * ds;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) part[threadIdx.x][k] = F[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double T[6] = {0, 0, 0, 0, 0, 0};
        for (int t = 0; t < kBlock; ++t)
#pragma unroll
            for (int k = 0; k < 6; ++k) T[k] += part[t][k];
        out[0] = (T[0] + T[2]) + T[4];
        out[1] = (T[1] + T[3]) + T[5];
    }
}

hipError_t launch_forces(hipStream_t st, int nw, const int *wall, const double2 *xy,
                         const double2 *nrm, const double *U, int n, double gamma, double pinf,
                         double *scratch, double *out) {
    hipLaunchKernelGGL(k_forces, dim3(1), dim3(kBlock), 0, st, nw, wall, xy, nrm, U, n, gamma,
                       pinf, scratch, out);
    return hipGetLastError();
}

// Residual history of ql_step_static, for callers that cannot allocate:
// file-scope, so every GPU the library runs on holds one copy until the
// process ends.  Host code uses only the address scratch_address returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double **ptr) {
    return hipGetSymbolAddress((void **)ptr, HIP_SYMBOL(scratch));
}

}  // namespace ql
