/*
 * Plain FP64 CPU oracle of the q-LSKUM pseudo-time iteration.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the solver never calls it and shares
 * no code with it.  It is written to be read against the paper: single
 * thread, caller's point order and neighbour order, every sum in the order
 * the formulas state it, libm transcendentals, compiled without FMA
 * contraction.  A second build of this same source with OpenMP (used only
 * to time the CPU baseline on every host core) runs the loops over points
 * in parallel: each point's arithmetic and the order of every sum over
 * points are unchanged, so its results are the serial build's bit for bit;
 * a failing step reports the smallest failing point in both builds.
 *
 * Paper: "On the performance of GPU accelerated q-LSKUM based meshfree
 * solvers in Fortran, C++, Python, and Julia" (Scientific Computing Report
 * 01:2021, arXiv 2108.07031).  Passages followed:
 *   sec. 2, eqs. (1)-(3)          Euler equations, U, Gx, Gy, e
 *   sec. 2, eqs. (4)-(9)          Maxwellian, moments, CIR splitting
 *   sec. 2, eq. (11)              first-order least-squares gradient
 *   sec. 2, eqs. (12)-(14)        split-flux derivatives on split stencils
 *   sec. 2.1, eqs. (26)-(29)      q-variables, modified q, q-derivatives
 *   sec. 3, Algorithm 1           serial solver: timestep, 4 RK stages of
 *                                 q_variables / q_derivatives /
 *                                 flux_residual / state_update, residue
 * Where the paper is silent (split-flux closed form, limiter, time step,
 * RK coefficients, wall and outer conditions, residual norm, forces) the
 * readings below are the ones the design notes list; each function says
 * which reading it implements.
 *
 * Array layouts: per-point vectors are component-major, U[c*n + p] for
 * c = 0..3 (rho, rho u1, rho u2, rho e); q likewise; the q-derivatives g
 * hold q_x in rows 0..3 and q_y in rows 4..7, g[(r)*n + p].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads the loops over points use (1 in the serial build) */
int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* keep (point, status) of the smallest failing point */
static void note_failure(int64_t p, int st, int64_t *bad, int *code)
{
#ifdef _OPENMP
#pragma omp critical(ora_failure)
#endif
    {
        if (p < *bad) {
            *bad = p;
            *code = st;
        }
    }
}

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ESINGULAR (-2)
#define ORA_ENOMEM (-3)
#define ORA_ENONFINITE (-5)
#define ORA_EPOSITIVITY (-6)

/* split-stencil membership bits of one neighbour (same encoding the solver
 * documents in its public header) */
#define SPLIT_S_PLUS 1u  /* delta s < 0 : stencil of the + split flux along s */
#define SPLIT_S_MINUS 2u /* delta s > 0 */
#define SPLIT_N_PLUS 4u  /* delta n < 0 */
#define SPLIT_N_MINUS 8u /* delta n > 0 */

#define KIND_INTERIOR 0
#define KIND_WALL 1
#define KIND_OUTER 2

typedef struct {
    double gamma, mach, alpha_deg, cfl;
    int32_t n_inner, limiter;
    double venkat_k;
    int32_t order; /* 2: modified q of eq. (28); 1: first order, q~ = q */
    int32_t outer_bc; /* 0: outer points held at the freestream; 1: kinetic outer condition */
} ora_params;

typedef struct {
    int64_t n;
    const double *x, *y, *nx, *ny;
    const uint8_t *kind;
    const int32_t *ptr, *idx;
    const uint8_t *flag;
} ora_cloud;

/* ------------------------------------------------------------------ */
/* State algebra: sec. 2 eqs. (2)-(3), sec. 2.1 eq. (26).              */
/* prim = (rho, u1, u2, p); beta = 1/(2RT) = rho/(2p).                  */
/* ------------------------------------------------------------------ */

void ora_u_to_prim(const double U[4], double gamma, double prim[4])
{
    double rho = U[0];
    double u1 = U[1] / rho;
    double u2 = U[2] / rho;
    double p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u1 * u1 + u2 * u2));
    prim[0] = rho;
    prim[1] = u1;
    prim[2] = u2;
    prim[3] = p;
}

void ora_prim_to_u(const double prim[4], double gamma, double U[4])
{
    double rho = prim[0], u1 = prim[1], u2 = prim[2], p = prim[3];
    U[0] = rho;
    U[1] = rho * u1;
    U[2] = rho * u2;
    U[3] = p / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2);
}

/* eq. (26): q = (ln rho + ln(beta)/(gamma-1) - beta |u|^2, 2 beta u1, 2 beta u2, -2 beta) */
void ora_prim_to_q(const double prim[4], double gamma, double q[4])
{
    double rho = prim[0], u1 = prim[1], u2 = prim[2], p = prim[3];
    double beta = rho / (2.0 * p);
    q[0] = log(rho) + log(beta) / (gamma - 1.0) - beta * (u1 * u1 + u2 * u2);
    q[1] = 2.0 * beta * u1;
    q[2] = 2.0 * beta * u2;
    q[3] = -2.0 * beta;
}

/* inverse of eq. (26) */
void ora_q_to_prim(const double q[4], double gamma, double prim[4])
{
    double beta = -0.5 * q[3];
    double u1 = q[1] / (2.0 * beta);
    double u2 = q[2] / (2.0 * beta);
    double rho = exp(q[0] - log(beta) / (gamma - 1.0) + beta * (u1 * u1 + u2 * u2));
    double p = rho / (2.0 * beta);
    prim[0] = rho;
    prim[1] = u1;
    prim[2] = u2;
    prim[3] = p;
}

/* ------------------------------------------------------------------ */
/* Kinetic split fluxes along a unit direction e (sec. 2 eqs. (4)-(9),  */
/* closed form of the half-range moments <Psi, v_e^{+-} F>, F the 2D   */
/* Maxwellian with internal energy).  sign = +1 for G^+, -1 for G^-.    */
/*   S = u_e sqrt(beta),  A = erfc(-sign S)/2,                          */
/*   B = exp(-S^2) / (2 sqrt(pi beta)),  rho e = p/(gamma-1) + rho|u|^2/2 */
/*   G = [ rho (u_e A + sign B),                                        */
/*         rho u (u_e A + sign B) + p A e,          (global x, y parts) */
/*         (p + rho e) u_e A + sign (p/2 + rho e) B ]                   */
/* ------------------------------------------------------------------ */

void ora_split_flux(const double prim[4], double ex, double ey, int sign, double gamma,
                    double G[4])
{
    const double pi = 3.14159265358979323846;
    double rho = prim[0], u1 = prim[1], u2 = prim[2], p = prim[3];
    double beta = rho / (2.0 * p);
    double ue = u1 * ex + u2 * ey;
    double S = ue * sqrt(beta);
    double sg = (sign > 0) ? 1.0 : -1.0;
    double A = 0.5 * erfc(-sg * S);
    double B = exp(-S * S) / (2.0 * sqrt(pi * beta));
    double rhoe = p / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2);
    double mass = rho * (ue * A + sg * B);
    G[0] = mass;
    G[1] = u1 * mass + p * A * ex;
    G[2] = u2 * mass + p * A * ey;
    G[3] = (p + rhoe) * ue * A + sg * (0.5 * p + rhoe) * B;
}

/* ------------------------------------------------------------------ */
/* Split stencils, sec. 2 eq. (14): N_x^{+-} = {P_i : dx_i <> 0}, taken  */
/* in each point's frame (s along t = (n_y, -n_x), n along the point's   */
/* normal).  Ties (|ds| <= 1e-12 |d|) belong to neither half.  Also     */
/* checks that every least-squares matrix the solver will invert is     */
/* non-singular: the full stencil of every point (eq. (11)) and each    */
/* split stencil that enters the residual (interior: all four; wall:    */
/* s+, s-, n-).  A matrix counts as singular when                       */
/* det <= 1e-12 (sum ds^2 + sum dn^2)^2 or fewer than 2 points.          */
/* ------------------------------------------------------------------ */

static uint8_t classify_one(double dx, double dy, double nx, double ny)
{
    double tx = ny, ty = -nx;
    double ds = dx * tx + dy * ty;
    double dn = dx * nx + dy * ny;
    double d2 = dx * dx + dy * dy;
    double tie = 1e-24 * d2;
    uint8_t f = 0;
    if (ds * ds > tie) f |= (ds < 0.0) ? SPLIT_S_PLUS : SPLIT_S_MINUS;
    if (dn * dn > tie) f |= (dn < 0.0) ? SPLIT_N_PLUS : SPLIT_N_MINUS;
    return f;
}

int ora_classify(int64_t n, const double *x, const double *y, const double *nx,
                 const double *ny, const uint8_t *kind, const int32_t *ptr,
                 const int32_t *idx, uint8_t *flag, int64_t *bad_point)
{
    *bad_point = -1;
    for (int64_t p = 0; p < n; ++p) {
        if (kind[p] > KIND_OUTER) { *bad_point = p; return ORA_EINVAL; }
        double a = 0, b = 0, c = 0;
        double ss[4] = {0, 0, 0, 0}, sn[4] = {0, 0, 0, 0}, nn[4] = {0, 0, 0, 0};
        int cnt[4] = {0, 0, 0, 0};
        for (int32_t k = ptr[p]; k < ptr[p + 1]; ++k) {
            int32_t i = idx[k];
            if (i < 0 || i >= n || i == p) { *bad_point = p; return ORA_EINVAL; }
            double dx = x[i] - x[p], dy = y[i] - y[p];
            uint8_t f = classify_one(dx, dy, nx[p], ny[p]);
            flag[k] = f;
            a += dx * dx;
            b += dx * dy;
            c += dy * dy;
            double ds = dx * ny[p] - dy * nx[p];
            double dn = dx * nx[p] + dy * ny[p];
            for (int s = 0; s < 4; ++s) {
                if (f & (1u << s)) {
                    ss[s] += ds * ds;
                    sn[s] += ds * dn;
                    nn[s] += dn * dn;
                    cnt[s] += 1;
                }
            }
        }
        double D = a * c - b * b;
        if (!(D > 1e-12 * (a + c) * (a + c)) || ptr[p + 1] - ptr[p] < 2) {
            *bad_point = p;
            return ORA_ESINGULAR;
        }
        if (kind[p] == KIND_OUTER) continue;
        for (int s = 0; s < 4; ++s) {
            if (kind[p] == KIND_WALL && s == 2) continue; /* n+ unused at walls */
            double det = ss[s] * nn[s] - sn[s] * sn[s];
            double sc = ss[s] + nn[s];
            if (cnt[s] < 2 || !(det > 1e-12 * sc * sc)) {
                *bad_point = p;
                return ORA_ESINGULAR;
            }
        }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Freestream (unit density, unit speed of sound) and the wall          */
/* condition's momentum projection m <- m - (m.n) n, which keeps rho    */
/* and rho e.                                                           */
/* ------------------------------------------------------------------ */

static void wall_project(double *U, int64_t n, int64_t p, double nx, double ny)
{
    double m1 = U[1 * n + p], m2 = U[2 * n + p];
    double mn = m1 * nx + m2 * ny;
    U[1 * n + p] = m1 - mn * nx;
    U[2 * n + p] = m2 - mn * ny;
}

void ora_freestream(int64_t n, const double *nx, const double *ny, const uint8_t *kind,
                    const ora_params *prm, int project_wall, double *U)
{
    const double pi = 3.14159265358979323846;
    double al = prm->alpha_deg * pi / 180.0;
    double prim[4] = {1.0, prm->mach * cos(al), prm->mach * sin(al), 1.0 / prm->gamma};
    double Uf[4];
    ora_prim_to_u(prim, prm->gamma, Uf);
    for (int64_t p = 0; p < n; ++p) {
        for (int c = 0; c < 4; ++c) U[c * n + p] = Uf[c];
        if (project_wall && kind[p] == KIND_WALL) wall_project(U, n, p, nx[p], ny[p]);
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, timestep(): local pseudo-time step from the state at    */
/* the start of the iteration, dt = CFL * min_i |P_i - P| / (|u| + c).  */
/* ------------------------------------------------------------------ */

void ora_timestep(const ora_cloud *cl, const ora_params *prm, const double *U, double *dt)
{
    int64_t n = cl->n;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double dmin = INFINITY;
        for (int32_t k = cl->ptr[p]; k < cl->ptr[p + 1]; ++k) {
            int32_t i = cl->idx[k];
            double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
            double d = sqrt(dx * dx + dy * dy);
            if (d < dmin) dmin = d;
        }
        double Up[4] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]}, prim[4];
        ora_u_to_prim(Up, prm->gamma, prim);
        double speed = sqrt(prim[1] * prim[1] + prim[2] * prim[2]);
        double c = sqrt(prm->gamma * prim[3] / prim[0]);
        dt[p] = prm->cfl * dmin / (speed + c);
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, q_variables(): eq. (26) at every point.                 */
/* ------------------------------------------------------------------ */

static int q_variables_point(int64_t n, const double *U, double gamma, double *q, int64_t p)
{
    double Up[4] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]}, prim[4], qp[4];
    for (int c = 0; c < 4; ++c)
        if (!isfinite(Up[c])) return ORA_ENONFINITE;
    ora_u_to_prim(Up, gamma, prim);
    if (!(prim[0] > 0.0) || !(prim[3] > 0.0)) return ORA_EPOSITIVITY;
    ora_prim_to_q(prim, gamma, qp);
    for (int c = 0; c < 4; ++c) q[c * n + p] = qp[c];
    return ORA_OK;
}

int ora_q_variables(int64_t n, const double *U, double gamma, double *q, int64_t *bad_point)
{
    int64_t bad = INT64_MAX;
    int code = ORA_OK;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int st = q_variables_point(n, U, gamma, q, p);
        if (st) note_failure(p, st, &bad, &code);
    }
    *bad_point = (code != ORA_OK) ? bad : -1;
    return code;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, q_derivatives(): eq. (29).  First pass: the first-order */
/* full-stencil least squares of eq. (11) with dq_i = q_i - q_0.  Then  */
/* n_inner inner iterations of eq. (29) with                            */
/*   dq~_i = dq_i - 1/2 [dx (q_x,i - q_x,0) + dy (q_y,i - q_y,0)],     */
/* every point reading the previous iterate (Jacobi).  Also returns the */
/* componentwise max and min of q over the point and its stencil, which */
/* bound the limited reconstruction.                                    */
/* ------------------------------------------------------------------ */

static void ls_solve(double a, double b, double c, const double sx[4], const double sy[4],
                     double gx[4], double gy[4])
{
    /* [a b; b c]^{-1} [sx; sy], a = sum dx^2, b = sum dx dy, c = sum dy^2 */
    double D = a * c - b * b;
    for (int r = 0; r < 4; ++r) {
        gx[r] = (c * sx[r] - b * sy[r]) / D;
        gy[r] = (a * sy[r] - b * sx[r]) / D;
    }
}

void ora_q_derivatives(const ora_cloud *cl, int32_t n_inner, const double *q, double *g,
                       double *qmax, double *qmin)
{
    int64_t n = cl->n;
    double *gprev = (double *)malloc(sizeof(double) * 8 * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double a = 0, b = 0, c = 0, sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
        double mx[4], mn[4];
        for (int r = 0; r < 4; ++r) mx[r] = mn[r] = q[r * n + p];
        for (int32_t k = cl->ptr[p]; k < cl->ptr[p + 1]; ++k) {
            int32_t i = cl->idx[k];
            double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
            a += dx * dx;
            b += dx * dy;
            c += dy * dy;
            for (int r = 0; r < 4; ++r) {
                double dq = q[r * n + i] - q[r * n + p];
                sx[r] += dx * dq;
                sy[r] += dy * dq;
                if (q[r * n + i] > mx[r]) mx[r] = q[r * n + i];
                if (q[r * n + i] < mn[r]) mn[r] = q[r * n + i];
            }
        }
        double gx[4], gy[4];
        ls_solve(a, b, c, sx, sy, gx, gy);
        for (int r = 0; r < 4; ++r) {
            g[r * n + p] = gx[r];
            g[(4 + r) * n + p] = gy[r];
            qmax[r * n + p] = mx[r];
            qmin[r * n + p] = mn[r];
        }
    }
    for (int32_t it = 0; it < n_inner; ++it) {
        memcpy(gprev, g, sizeof(double) * 8 * (size_t)n);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            double a = 0, b = 0, c = 0, sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
            for (int32_t k = cl->ptr[p]; k < cl->ptr[p + 1]; ++k) {
                int32_t i = cl->idx[k];
                double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
                a += dx * dx;
                b += dx * dy;
                c += dy * dy;
                for (int r = 0; r < 4; ++r) {
                    double dq = q[r * n + i] - q[r * n + p];
                    double corr = 0.5 * (dx * (gprev[r * n + i] - gprev[r * n + p]) +
                                         dy * (gprev[(4 + r) * n + i] - gprev[(4 + r) * n + p]));
                    double dqt = dq - corr;
                    sx[r] += dx * dqt;
                    sy[r] += dy * dqt;
                }
            }
            double gx[4], gy[4];
            ls_solve(a, b, c, sx, sy, gx, gy);
            for (int r = 0; r < 4; ++r) {
                g[r * n + p] = gx[r];
                g[(4 + r) * n + p] = gy[r];
            }
        }
    }
    free(gprev);
}

/* ------------------------------------------------------------------ */
/* Venkatakrishnan limiter (J. Comput. Phys. 118, 1995), applied per    */
/* pair and per q-component to the increment delta of eq. (28):        */
/*   D = qmax - q if delta > 0, else qmin - q  (that point's bounds),   */
/*   eps^2 = (K |P_i - P_0|)^3,                                         */
/*   phi = [(D^2 + eps^2) + 2 delta D] / [D^2 + 2 delta^2 + delta D + eps^2] */
/* (phi = 1 when the denominator vanishes; no clamp to 1).              */
/* ------------------------------------------------------------------ */

double ora_venkat(double delta, double q, double qmx, double qmn, double eps2)
{
    double D = (delta > 0.0) ? (qmx - q) : (qmn - q);
    double num = (D * D + eps2) + 2.0 * delta * D;
    double den = D * D + 2.0 * delta * delta + delta * D + eps2;
    return (den == 0.0) ? 1.0 : num / den;
}

/* eps^2 = (K |P_i - P_0|)^3 for the offset (dx, dy) */
double ora_venkat_eps2(double K, double dx, double dy)
{
    double e = K * sqrt(dx * dx + dy * dy);
    return e * e * e;
}

/* ------------------------------------------------------------------ */
/* Modified q of one neighbour entry k of point p, eq. (28):            */
/*   q~_i = q_i + phi_i delta_i,  q~_0 = q_p + phi_0 delta_0,           */
/*   delta = -1/2 (dx q_x + dy q_y) at that point,                      */
/* with phi from the limiter above (phi = 1 when it is off); in the     */
/* first-order mode q~ = q.                                              */
/* ------------------------------------------------------------------ */

/* q~ of point j shifted by the offset (dx, dy): q_j - 1/2 (dx q_x,j + dy q_y,j),
 * the increment limited with point j's own bounds and eps from |(dx, dy)|. */
static void shifted_q(const ora_params *prm, int64_t n, const double *q, const double *g,
                      const double *qmax, const double *qmin, int64_t j, double dx, double dy,
                      double out[4])
{
    double eps2 = 0.0;
    if (prm->limiter) eps2 = ora_venkat_eps2(prm->venkat_k, dx, dy);
    for (int r = 0; r < 4; ++r) {
        if (prm->order == 1) { /* first-order LSKUM: split fluxes of q itself */
            out[r] = q[r * n + j];
            continue;
        }
        double d = -0.5 * (dx * g[r * n + j] + dy * g[(4 + r) * n + j]);
        double phi = 1.0;
        if (prm->limiter) phi = ora_venkat(d, q[r * n + j], qmax[r * n + j], qmin[r * n + j], eps2);
        out[r] = q[r * n + j] + phi * d;
    }
}

void ora_modified_q(const ora_cloud *cl, const ora_params *prm, const double *q, const double *g,
                    const double *qmax, const double *qmin, int64_t p, int64_t k, double qti[4],
                    double qt0[4])
{
    int32_t i = cl->idx[k];
    double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
    shifted_q(prm, cl->n, q, g, qmax, qmin, i, dx, dy, qti);
    shifted_q(prm, cl->n, q, g, qmax, qmin, p, dx, dy, qt0);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, flux_residual(): eq. (12) with the split-flux           */
/* perturbations of eq. (27), dG_i = G(q~_i) - G(q~_0), q~ from eq.    */
/* (28) (limited), and the split-flux derivatives of eq. (13) by        */
/* Cramer's rule over each split stencil of eq. (14), in the point's    */
/* (s, n) frame:                                                        */
/*   dG/ds = (sum ds dG * sum dn^2 - sum dn dG * sum ds dn) / Det       */
/*   dG/dn = (sum dn dG * sum ds^2 - sum ds dG * sum ds dn) / Det       */
/*   Det   = sum ds^2 sum dn^2 - (sum ds dn)^2   (sums over the stencil) */
/* Interior: R = dGs+/ds + dGs-/ds + dGn+/dn + dGn-/dn (eq. (12)).      */
/* Wall (normal into the fluid): the n+ term, whose stencil lies in the */
/* body, is dropped.  Outer points carry no residual when they are held */
/* at the freestream (outer_bc 0).  Kinetic outer condition (outer_bc   */
/* 1; the normal points away from the body, to the far field): the own  */
/* n- stencil would lie outside the domain, where the molecules that    */
/* enter come from the freestream Maxwellian.  It is replaced by the    */
/* mirror image of the n+ stencil through the point's tangent line,     */
/* (ds, dn) -> (ds, -dn), whose points hold the uniform freestream      */
/* (q~ = q_inf, no gradient); the point's own modified state for each   */
/* mirrored entry is shifted by the mirrored offset.  So               */
/*   R = dGs+/ds + dGs-/ds + dGn+/dn + dGn-/dn|mirror,                  */
/* with dGn-/dn|mirror the Cramer derivative of eq. (13) over the       */
/* mirrored offsets of Gn-(q_inf) - Gn-(q~_0').                          */
/* ------------------------------------------------------------------ */

typedef struct {
    double ss, sn, nn, sG[4], nG[4];
} bucket;

/* the residual of point p (all four components into R); ORA_EPOSITIVITY
 * when a modified state has no Maxwellian */
static int flux_point(const ora_cloud *cl, const ora_params *prm, const double *q,
                      const double *g, const double *qmax, const double *qmin,
                      const double prinf[4], int64_t p, double *R)
{
    int64_t n = cl->n;
    double gamma = prm->gamma;
    int kobc = prm->outer_bc == 1;
    for (int r = 0; r < 4; ++r) R[r * n + p] = 0.0;
    if (cl->kind[p] == KIND_OUTER && !kobc) return ORA_OK;
    double nx = cl->nx[p], ny = cl->ny[p];
    double tx = ny, ty = -nx;
    bucket bk[4];
    memset(bk, 0, sizeof bk);
    for (int32_t k = cl->ptr[p]; k < cl->ptr[p + 1]; ++k) {
        int32_t i = cl->idx[k];
        uint8_t f = cl->flag[k];
        if (cl->kind[p] == KIND_WALL) f &= (uint8_t)~SPLIT_N_PLUS;
        if (cl->kind[p] == KIND_OUTER) f &= (uint8_t)~SPLIT_N_MINUS;
        if (f == 0) continue;
        double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
        double ds = dx * tx + dy * ty;
        double dn = dx * nx + dy * ny;
        double qti[4], qt0[4];
        ora_modified_q(cl, prm, q, g, qmax, qmin, p, k, qti, qt0);
        if (!(qti[3] < 0.0) || !(qt0[3] < 0.0)) return ORA_EPOSITIVITY;
        double pri[4], pr0[4];
        ora_q_to_prim(qti, gamma, pri);
        ora_q_to_prim(qt0, gamma, pr0);
        for (int r = 0; r < 4; ++r)
            if (!isfinite(pri[r]) || !isfinite(pr0[r])) return ORA_EPOSITIVITY;
        for (int dir = 0; dir < 2; ++dir) {
            uint8_t fp = dir ? SPLIT_N_PLUS : SPLIT_S_PLUS;
            uint8_t fm = dir ? SPLIT_N_MINUS : SPLIT_S_MINUS;
            int sign, b;
            if (f & fp) { sign = 1; b = 2 * dir; }
            else if (f & fm) { sign = -1; b = 2 * dir + 1; }
            else continue;
            double ex = dir ? nx : tx, ey = dir ? ny : ty;
            double Gi[4], G0[4];
            ora_split_flux(pri, ex, ey, sign, gamma, Gi);
            ora_split_flux(pr0, ex, ey, sign, gamma, G0);
            bk[b].ss += ds * ds;
            bk[b].sn += ds * dn;
            bk[b].nn += dn * dn;
            for (int r = 0; r < 4; ++r) {
                double dG = Gi[r] - G0[r];
                bk[b].sG[r] += ds * dG;
                bk[b].nG[r] += dn * dG;
            }
        }
    }
    if (cl->kind[p] == KIND_OUTER) {
        /* the mirrored n+ stencil at the freestream replaces n- */
        memset(&bk[3], 0, sizeof bk[3]);
        double Ginf[4];
        ora_split_flux(prinf, nx, ny, -1, gamma, Ginf);
        for (int32_t k = cl->ptr[p]; k < cl->ptr[p + 1]; ++k) {
            if (!(cl->flag[k] & SPLIT_N_PLUS)) continue;
            int32_t i = cl->idx[k];
            double dx = cl->x[i] - cl->x[p], dy = cl->y[i] - cl->y[p];
            double ds = dx * tx + dy * ty;
            double dn = -(dx * nx + dy * ny);      /* mirrored */
            double mx = ds * tx + dn * nx, my = ds * ty + dn * ny;
            double qt0[4], pr0[4], G0[4];
            shifted_q(prm, n, q, g, qmax, qmin, p, mx, my, qt0);
            if (!(qt0[3] < 0.0)) return ORA_EPOSITIVITY;
            ora_q_to_prim(qt0, gamma, pr0);
            for (int r = 0; r < 4; ++r)
                if (!isfinite(pr0[r])) return ORA_EPOSITIVITY;
            ora_split_flux(pr0, nx, ny, -1, gamma, G0);
            bk[3].ss += ds * ds;
            bk[3].sn += ds * dn;
            bk[3].nn += dn * dn;
            for (int r = 0; r < 4; ++r) {
                double dG = Ginf[r] - G0[r];
                bk[3].sG[r] += ds * dG;
                bk[3].nG[r] += dn * dG;
            }
        }
    }
    double Rp[4] = {0, 0, 0, 0};
    for (int b = 0; b < 4; ++b) {
        if (b == 2 && cl->kind[p] == KIND_WALL) continue;
        double det = bk[b].ss * bk[b].nn - bk[b].sn * bk[b].sn;
        for (int r = 0; r < 4; ++r) {
            double d;
            if (b < 2) d = (bk[b].sG[r] * bk[b].nn - bk[b].nG[r] * bk[b].sn) / det;
            else d = (bk[b].nG[r] * bk[b].ss - bk[b].sG[r] * bk[b].sn) / det;
            Rp[r] += d;
        }
    }
    for (int r = 0; r < 4; ++r) R[r * n + p] = Rp[r];
    return ORA_OK;
}

int ora_flux_residual(const ora_cloud *cl, const ora_params *prm, const double *q,
                      const double *g, const double *qmax, const double *qmin, double *R,
                      int64_t *bad_point)
{
    int64_t n = cl->n;
    double gamma = prm->gamma;
    double qinf[4], prinf[4];
    {
        const double pi = 3.14159265358979323846;
        double al = prm->alpha_deg * pi / 180.0;
        double pr[4] = {1.0, prm->mach * cos(al), prm->mach * sin(al), 1.0 / gamma};
        ora_prim_to_q(pr, gamma, qinf);
        ora_q_to_prim(qinf, gamma, prinf);
    }
    int64_t bad = INT64_MAX;
    int code = ORA_OK;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int st = flux_point(cl, prm, q, g, qmax, qmin, prinf, p, R);
        if (st) note_failure(p, st, &bad, &code);
    }
    *bad_point = (code != ORA_OK) ? bad : -1;
    return code;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, state_update(rk): four-stage third-order SSP Runge-     */
/* Kutta (Kraaijevanger 1991; Spiteri & Ruuth 2002) with L(U) = -R(U):  */
/*   rk1: U1 = Un + dt/2 L(Un)                                          */
/*   rk2: U2 = U1 + dt/2 L(U1)                                          */
/*   rk3: U3 = 2/3 Un + 1/3 (U2 + dt/2 L(U2))                           */
/*   rk4: U4 = U3 + dt/2 L(U3)                                          */
/* Applied pointwise to m values; the update of one point.  Outer points  */
/* are held at the freestream unless the kinetic outer condition is on.  */
/* ------------------------------------------------------------------ */

void ora_rk_stage(int32_t rk, int64_t m, const double *un, const double *u, const double *r,
                  const double *dt, double *out)
{
    for (int64_t j = 0; j < m; ++j) {
        double l = -r[j];
        double h = 0.5 * dt[j];
        if (rk == 3) out[j] = (2.0 / 3.0) * un[j] + (1.0 / 3.0) * (u[j] + h * l);
        else out[j] = u[j] + h * l;
    }
}

void ora_state_update(const ora_cloud *cl, const ora_params *prm, int32_t rk, const double *Un,
                      double *U, const double *R, const double *dt)
{
    int64_t n = cl->n;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue; /* held */
        for (int c = 0; c < 4; ++c) {
            double v;
            ora_rk_stage(rk, 1, &Un[c * n + p], &U[c * n + p], &R[c * n + p], &dt[p], &v);
            U[c * n + p] = v;
        }
        if (cl->kind[p] == KIND_WALL) wall_project(U, n, p, cl->nx[p], cl->ny[p]);
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, residue(): root mean square over the updated points     */
/* (interior and wall; outer too under the kinetic outer condition) of   */
/* each component of the first stage's residual.                        */
/* ------------------------------------------------------------------ */

void ora_residue(const ora_cloud *cl, const ora_params *prm, const double *R, double res[4])
{
    int64_t n = cl->n, m = 0;
    double s[4] = {0, 0, 0, 0};
    for (int64_t p = 0; p < n; ++p) {
        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue;
        m++;
        for (int c = 0; c < 4; ++c) s[c] += R[c * n + p] * R[c * n + p];
    }
    for (int c = 0; c < 4; ++c) res[c] = (m > 0) ? sqrt(s[c] / (double)m) : 0.0;
}

/* ------------------------------------------------------------------ */
/* One evaluation of the stage operator at U: q, its derivatives and    */
/* bounds, the residual and the time step.                              */
/* ------------------------------------------------------------------ */

int ora_evaluate(const ora_cloud *cl, const ora_params *prm, const double *U, double *q,
                 double *g, double *qmax, double *qmin, double *R, double *dt,
                 int64_t *bad_point)
{
    int st = ora_q_variables(cl->n, U, prm->gamma, q, bad_point);
    if (st) return st;
    ora_q_derivatives(cl, prm->n_inner, q, g, qmax, qmin);
    st = ora_flux_residual(cl, prm, q, g, qmax, qmin, R, bad_point);
    if (st) return st;
    if (dt) ora_timestep(cl, prm, U, dt);
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: n_iter pseudo-time iterations from U (in place).        */
/* res_hist (nullable) receives residue() of each iteration, 4 values.  */
/* ------------------------------------------------------------------ */

int ora_run(const ora_cloud *cl, const ora_params *prm, double *U, int32_t n_iter,
            double *res_hist, int64_t *bad_point)
{
    int64_t n = cl->n;
    size_t sz = sizeof(double) * (size_t)n;
    double *Un = (double *)malloc(4 * sz), *q = (double *)malloc(4 * sz);
    double *g = (double *)malloc(8 * sz), *qmax = (double *)malloc(4 * sz);
    double *qmin = (double *)malloc(4 * sz), *R = (double *)malloc(4 * sz);
    double *dt = (double *)malloc(sz);
    int st = ORA_OK;
    *bad_point = -1;
    if (!Un || !q || !g || !qmax || !qmin || !R || !dt) { st = ORA_ENOMEM; goto done; }
    for (int32_t it = 0; it < n_iter; ++it) {
        memcpy(Un, U, 4 * sz);
        ora_timestep(cl, prm, U, dt);
        for (int32_t rk = 1; rk <= 4; ++rk) {
            st = ora_q_variables(n, U, prm->gamma, q, bad_point);
            if (st) goto done;
            ora_q_derivatives(cl, prm->n_inner, q, g, qmax, qmin);
            st = ora_flux_residual(cl, prm, q, g, qmax, qmin, R, bad_point);
            if (st) goto done;
            if (rk == 1 && res_hist) ora_residue(cl, prm, R, &res_hist[4 * (int64_t)it]);
            ora_state_update(cl, prm, rk, Un, U, R, dt);
        }
    }
done:
    free(Un); free(q); free(g); free(qmax); free(qmin); free(R); free(dt);
    return st;
}

/* ------------------------------------------------------------------ */
/* postprocessor(): lift and drag coefficients from the wall pressure.  */
/* Wall points, in the caller's order, form the closed surface polygon; */
/* each carries the arc length ds = (|S_next - S| + |S - S_prev|)/2.    */
/* F = -sum (p - p_inf) n ds (n into the fluid), summed separately over */
/* the upper (y > 0), lower (y < 0) and on-axis wall points, then added */
/* in that order;  Cl = F.(-sin a, cos a)/q_inf, Cd = F.(cos a, sin a)/q_inf, */
/* q_inf = rho_inf |u_inf|^2 / 2.                                       */
/* ------------------------------------------------------------------ */

int ora_forces(const ora_cloud *cl, const ora_params *prm, const double *U, double *cl_out,
               double *cd_out)
{
    const double pi = 3.14159265358979323846;
    int64_t n = cl->n, nw = 0;
    for (int64_t p = 0; p < n; ++p) nw += (cl->kind[p] == KIND_WALL);
    if (nw < 3) return ORA_EINVAL;
    int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)nw);
    if (!w) return ORA_ENOMEM;
    for (int64_t p = 0, j = 0; p < n; ++p)
        if (cl->kind[p] == KIND_WALL) w[j++] = p;
    double pinf = 1.0 / prm->gamma;
    double F[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t j = 0; j < nw; ++j) {
        int64_t p = w[j], pn = w[(j + 1) % nw], pp = w[(j + nw - 1) % nw];
        double ln = sqrt((cl->x[pn] - cl->x[p]) * (cl->x[pn] - cl->x[p]) +
                         (cl->y[pn] - cl->y[p]) * (cl->y[pn] - cl->y[p]));
        double lp = sqrt((cl->x[p] - cl->x[pp]) * (cl->x[p] - cl->x[pp]) +
                         (cl->y[p] - cl->y[pp]) * (cl->y[p] - cl->y[pp]));
        double ds = 0.5 * (ln + lp);
        double Up[4] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]}, prim[4];
        ora_u_to_prim(Up, prm->gamma, prim);
        int h = (cl->y[p] > 0.0) ? 0 : (cl->y[p] < 0.0) ? 1 : 2;
        F[h][0] += -(prim[3] - pinf) * cl->nx[p] * ds;
        F[h][1] += -(prim[3] - pinf) * cl->ny[p] * ds;
    }
    free(w);
    double Fx = (F[0][0] + F[1][0]) + F[2][0];
    double Fy = (F[0][1] + F[1][1]) + F[2][1];
    double al = prm->alpha_deg * pi / 180.0;
    double qinf = 0.5 * 1.0 * prm->mach * prm->mach;
    *cl_out = (-Fx * sin(al) + Fy * cos(al)) / qinf;
    *cd_out = (Fx * cos(al) + Fy * sin(al)) / qinf;
    return ORA_OK;
}
