/*
 * pic_oracle.c -- plain, slow FP64 CPU oracle of the electrostatic PIC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * What it follows (the paper is "A Comparison of Massively Parallel Performance
 * Portable Particle-in-Cell schemes for electrostatic kinetic plasma
 * simulations", PASC'26):
 *   - the PIC loop scatter -> solve -> gather -> push        (Sec. 2, Fig. pic-loop)
 *   - Poisson  Lap(phi) = -rho/eps0,  E = -grad(phi)          (Sec. 2, Eq. poisson)
 *   - neutralising background rho_i = -Q_e / |box|            (Sec. 2, text after Eq. poisson)
 *   - same shape function for scatter and gather (CIC)        (Sec. 2; Sec. 4.2 "Weak scaling")
 *   - equations of motion dx/dt = v, dv/dt = (q/m) E          (Sec. 2, Eq. eom; B_ext = E_ext = 0)
 *   - second-order central FD Laplacian, matrix-free CG       (Sec. 3.2 "PCG solver")
 *   - previous step's solution as the CG starting guess       (Sec. 4.1 "Setup")
 * Readings where the paper is silent (grid centring, gauge, residual norm,
 * integrator, tie-breaking) are stated at each function.  Mixed-precision
 * refinement and the flexible CG used by the learned preconditioner are not in
 * the paper; they follow the textbook definitions cited at each function.
 *
 * Conventions shared with the product (restated, not shared code):
 *   grid: vertex-centred, value i sits at x = i*h, h = L/N, periodic, layout
 *         [iz][iy][ix] with ix fastest;   inv_h = (double)N / L.
 *   Bounded boxes (the PCG solver's Dirichlet and Neumann boundaries, Sec. 3.2
 *   and Table solver_comparison_table; the discretisation is this file's
 *   reading, the paper gives none), bc = 1 or 2, same on all six faces:
 *     Dirichlet (bc 1): phi = 0 on the boundary of [0, L]^3; the unknowns are
 *       the N^3 interior vertices x_i = (i+1) h, h = L/(N+1); a neighbour on
 *       the boundary contributes 0;  inv_h = (double)(N + 1) / L.
 *     Neumann (bc 2): zero normal derivative; the unknowns sit at the cell
 *       centres x_i = (i + 1/2) h, h = L/N; the value across a face mirrors the
 *       value inside (zero flux);  inv_h = (double)N / L.
 *   Floating point: IEEE binary64, round to nearest; this file must be compiled
 *   with -ffp-contract=off and without -ffast-math.
 *
 * Every sum in this file is a plain sequential sum in index order.  Loops whose
 * iterations are independent (one output element each) may run under OpenMP;
 * that changes no rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_IDX(N, ix, iy, iz) ((((int64_t)(iz)) * (N) + (iy)) * (int64_t)(N) + (ix))

int or_abi_version(void) { return 4; }

/* ------------------------------------------------------------------------ */
/* Cell index and CIC fraction of one coordinate.
 * s = x * (N/L); i = floor(s) clamped to [0, N-1]; w = s - i.
 * When x rounds to s == N the clamp gives i = N-1, w = 1: all weight on the
 * periodic image of vertex 0, which is the correct CIC limit.              */
static void or_locate(double xd, int N, double inv_h, int *i, double *w)
{
    double s = xd * inv_h;
    double f = floor(s);
    int ii = (int)f;
    if (ii > N - 1) ii = N - 1;
    if (ii < 0) ii = 0;
    *i = ii;
    *w = s - (double)ii;
}

/* Cell key of each particle: (iz*N + iy)*N + ix.  */
void or_cell_keys(int64_t np, int N, double L, const double *x, const double *y,
                  const double *z, uint32_t *key)
{
    double inv_h = (double)N / L;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        int ix, iy, iz;
        double wx, wy, wz;
        or_locate(x[p], N, inv_h, &ix, &wx);
        or_locate(y[p], N, inv_h, &iy, &wy);
        or_locate(z[p], N, inv_h, &iz, &wz);
        key[p] = (uint32_t)OR_IDX(N, ix, iy, iz);
    }
}

/* ------------------------------------------------------------------------ */
/* Stable sort by cell key, as a counting sort (the textbook stable sort for
 * small integer keys): perm[j] is the input index of the j-th sorted
 * particle; equal keys keep their input order.  cell_start has ncell+1
 * entries: cell_start[c] is the first sorted slot of cell c.              */
int or_sort_by_key(int64_t np, int64_t ncell, const uint32_t *key, int64_t *perm,
                   int64_t *cell_start)
{
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    if (!fill) return -1;
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t p = 0; p < np; ++p) {
        if ((int64_t)key[p] >= ncell) { free(fill); return -2; }
        cell_start[key[p] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    for (int64_t c = 0; c < ncell; ++c) fill[c] = cell_start[c];
    for (int64_t p = 0; p < np; ++p) perm[fill[key[p]]++] = p;
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cloud-in-cell charge deposit (scatter, Fig. pic-loop) plus the uniform
 * neutralising background (Sec. 2) and the zero-mean projection the periodic
 * problem needs.
 *   rho_e[v] = (q / h^3) * sum_p W_p(v),   W_p(v) = prod_d W_d,
 *   W_d = 1 - w_d for the lower vertex, w_d for the upper (periodic) one.
 *   rho = rho_e + rho_bg;  b = rho - mean(rho).
 * Writes rho_e (may be NULL) and b; returns ||b||_2.                         */
double or_deposit(int64_t np, int N, double L, double q, double rho_bg,
                  const double *x, const double *y, const double *z,
                  double *rho_e_out, double *b)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = (double)N / L;
    double qh3 = q * (inv_h * inv_h * inv_h);
    double *acc = (double *)calloc((size_t)n3, sizeof(double));
    if (!acc) return -1.0;
    for (int64_t p = 0; p < np; ++p) {
        int i[3];
        double w[3];
        or_locate(x[p], N, inv_h, &i[0], &w[0]);
        or_locate(y[p], N, inv_h, &i[1], &w[1]);
        or_locate(z[p], N, inv_h, &i[2], &w[2]);
        for (int c = 0; c < 2; ++c) {
            double wz = c ? w[2] : 1.0 - w[2];
            int vz = (i[2] + c) % N;
            for (int bb = 0; bb < 2; ++bb) {
                double wy = bb ? w[1] : 1.0 - w[1];
                int vy = (i[1] + bb) % N;
                for (int a = 0; a < 2; ++a) {
                    double wx = a ? w[0] : 1.0 - w[0];
                    int vx = (i[0] + a) % N;
                    acc[OR_IDX(N, vx, vy, vz)] += (wz * wy) * wx;
                }
            }
        }
    }
    double sum = 0.0;
    for (int64_t v = 0; v < n3; ++v) {
        double re = acc[v] * qh3;
        if (rho_e_out) rho_e_out[v] = re;
        b[v] = re + rho_bg;
        sum += b[v];
    }
    double mean = sum / (double)n3;
    double nb = 0.0;
    for (int64_t v = 0; v < n3; ++v) {
        b[v] = b[v] - mean;
        nb += b[v] * b[v];
    }
    free(acc);
    return sqrt(nb);
}

/* ------------------------------------------------------------------------ */
/* 1/h of the grid of boundary kind bc (conventions above). */
static double or_inv_h(int N, double L, int bc)
{
    return bc == 1 ? (double)(N + 1) / L : (double)N / L;
}

/* Value of u at integer point (ix, iy, iz), each coordinate in [-1, N]: the
 * point itself inside the grid; outside it, the periodic image (bc 0), zero
 * (bc 1, Dirichlet) or the mirrored inside value (bc 2, Neumann). */
static double or_ghost(const double *u, int N, int bc, int ix, int iy, int iz)
{
    int c[3] = {ix, iy, iz};
    for (int d = 0; d < 3; ++d) {
        if (c[d] >= 0 && c[d] < N) continue;
        if (bc == 1) return 0.0;
        if (bc == 2) c[d] = c[d] < 0 ? 0 : N - 1;
        else c[d] = c[d] < 0 ? c[d] + N : c[d] - N;
    }
    return u[OR_IDX(N, c[0], c[1], c[2])];
}

/* Index of the neighbour of coordinate i (step d = -1 or +1) under the
 * boundary rule of bc, or -1 where the neighbour is a Dirichlet zero: the
 * same rule as or_ghost, one axis at a time. */
static int or_nbr(int i, int d, int N, int bc)
{
    int j = i + d;
    if (j >= 0 && j < N) return j;
    if (bc == 1) return -1;
    if (bc == 2) return i;
    return j < 0 ? j + N : j - N;
}

/* A = -Lap_h, the 7-point second-order central-difference operator
 * (Sec. 3.2):  (A u)_i = (6 u_i - sum of 6 neighbours) / h^2, the neighbours
 * taken through the boundary rule of bc (periodic for the PIC loop).
 * Neighbour sum taken as ((xm + xp) + (ym + yp)) + (zm + zp).               */
void or_apply_A_bc(int N, double L, int bc, const double *u, double *Au)
{
    double inv_h = or_inv_h(N, L, bc);
    double inv_h2 = inv_h * inv_h;
#pragma omp parallel for schedule(static)
    for (int iz = 0; iz < N; ++iz) {
        int zm = or_nbr(iz, -1, N, bc), zp = or_nbr(iz, 1, N, bc);
        for (int iy = 0; iy < N; ++iy) {
            int ym = or_nbr(iy, -1, N, bc), yp = or_nbr(iy, 1, N, bc);
            for (int ix = 0; ix < N; ++ix) {
                int xm = or_nbr(ix, -1, N, bc), xp = or_nbr(ix, 1, N, bc);
                double vxm = xm < 0 ? 0.0 : u[OR_IDX(N, xm, iy, iz)];
                double vxp = xp < 0 ? 0.0 : u[OR_IDX(N, xp, iy, iz)];
                double vym = ym < 0 ? 0.0 : u[OR_IDX(N, ix, ym, iz)];
                double vyp = yp < 0 ? 0.0 : u[OR_IDX(N, ix, yp, iz)];
                double vzm = zm < 0 ? 0.0 : u[OR_IDX(N, ix, iy, zm)];
                double vzp = zp < 0 ? 0.0 : u[OR_IDX(N, ix, iy, zp)];
                double t = ((vxm + vxp) + (vym + vyp)) + (vzm + vzp);
                Au[OR_IDX(N, ix, iy, iz)] = (6.0 * u[OR_IDX(N, ix, iy, iz)] - t) * inv_h2;
            }
        }
    }
}

/* The periodic operator of the PIC loop. */
void or_apply_A(int N, double L, const double *u, double *Au)
{
    or_apply_A_bc(N, L, 0, u, Au);
}

static double or_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* r = b - A x;  returns ||r||_2.  */
static double or_true_residual(int N, double L, int bc, const double *b, const double *x,
                               double *r)
{
    int64_t n3 = (int64_t)N * N * N;
    or_apply_A_bc(N, L, bc, x, r);
    for (int64_t i = 0; i < n3; ++i) r[i] = b[i] - r[i];
    return sqrt(or_dot(n3, r, r));
}

double or_residual_norm_bc(int N, double L, int bc, const double *b, const double *x)
{
    int64_t n3 = (int64_t)N * N * N;
    double *r = (double *)malloc(sizeof(double) * (size_t)n3);
    if (!r) return -1.0;
    double nr = or_true_residual(N, L, bc, b, x, r);
    free(r);
    return nr;
}

double or_residual_norm(int N, double L, const double *b, const double *x)
{
    return or_residual_norm_bc(N, L, 0, b, x);
}

/* ------------------------------------------------------------------------ */
/* Preconditioned CG (the PCG solver of Sec. 3.2 with the Jacobi
 * preconditioner of the same section, M^{-1} = diag(A)^{-1} = (h^2/6) I),
 * in the textbook form (Saad, Iterative Methods for Sparse Linear Systems,
 * 2nd ed., Alg. 9.1), starting from the caller's x (the previous step's
 * solution, Sec. 4.1).
 * Stop rule (the paper gives only a tolerance, Sec. 4): the recursively
 * updated residual must satisfy ||r|| <= rtol * ||b||; the true residual
 * b - A x is then computed, and if it fails the same test it replaces r,
 * p restarts from M^{-1} r, and iteration continues (residual replacement).
 * ||b|| = 0 gives x = 0.
 * Bounded boxes (bc 1, 2): the same iteration with the operator of bc and
 * M^{-1} = (h^2/6) I with that grid's h, which is diag(A)^{-1} for Dirichlet;
 * for Neumann it is the inverse of the interior rows' diagonal (the boundary
 * rows' diagonal is (6 - m)/h^2 for a point touching m faces) -- a reading,
 * kept so that the preconditioner stays a scalar.
 * info[0]=iterations, [1]=last recursive ||r||/||b||, [2]=true ||b-Ax||/||b||,
 * [3]=converged (1/0), [4]=residual replacements.                         */
void or_pcg_bc(int N, double L, int bc, const double *b, double *x, double rtol,
               int64_t max_iter, double *info)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = or_inv_h(N, L, bc);
    double minv = 1.0 / (6.0 * (inv_h * inv_h));
    double *r = (double *)malloc(sizeof(double) * (size_t)n3);
    double *z = (double *)malloc(sizeof(double) * (size_t)n3);
    double *p = (double *)malloc(sizeof(double) * (size_t)n3);
    double *q = (double *)malloc(sizeof(double) * (size_t)n3);
    int64_t it = 0, repl = 0;
    int converged = 0;
    double rel = 0.0, trel = 0.0;
    double nb = sqrt(or_dot(n3, b, b));
    if (nb == 0.0) {
        for (int64_t i = 0; i < n3; ++i) x[i] = 0.0;
        info[0] = 0; info[1] = 0.0; info[2] = 0.0; info[3] = 1; info[4] = 0;
        free(r); free(z); free(p); free(q);
        return;
    }
    double tol = rtol * nb;
    double nr = or_true_residual(N, L, bc, b, x, r);
    rel = trel = nr / nb;
    if (nr <= tol) converged = 1;
    for (int64_t i = 0; i < n3; ++i) { z[i] = minv * r[i]; p[i] = z[i]; }
    double rz = or_dot(n3, r, z);
    while (!converged && it < max_iter) {
        or_apply_A_bc(N, L, bc, p, q);
        double alpha = rz / or_dot(n3, p, q);
        for (int64_t i = 0; i < n3; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        ++it;
        double rn = sqrt(or_dot(n3, r, r));
        rel = rn / nb;
        if (rn <= tol) {
            double tn = or_true_residual(N, L, bc, b, x, q);
            trel = tn / nb;
            if (tn <= tol) { converged = 1; break; }
            /* residual replacement: r <- b - A x, restart the direction */
            for (int64_t i = 0; i < n3; ++i) { r[i] = q[i]; z[i] = minv * r[i]; p[i] = z[i]; }
            rz = or_dot(n3, r, z);
            rel = tn / nb;
            ++repl;
            continue;
        }
        for (int64_t i = 0; i < n3; ++i) z[i] = minv * r[i];
        double rz_new = or_dot(n3, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n3; ++i) p[i] = z[i] + beta * p[i];
    }
    if (!converged) trel = or_residual_norm_bc(N, L, bc, b, x) / nb;
    info[0] = (double)it; info[1] = rel; info[2] = trel; info[3] = converged; info[4] = (double)repl;
    free(r); free(z); free(p); free(q);
}

void or_pcg(int N, double L, const double *b, double *x, double rtol, int64_t max_iter,
            double *info)
{
    or_pcg_bc(N, L, 0, b, x, rtol, max_iter, info);
}

/* ------------------------------------------------------------------------ */
/* SSOR preconditioner (Sec. 4.1: the PCG runs used SSOR with 4 inner and 2
 * outer iterations and damping pi/2; the paper defines neither count).
 * Reading: A = D + L + U with D = (6/h^2) I, L the
 * backward neighbours (x-1, y-1, z-1, periodic) and U = L^T the forward ones;
 * one SSOR application is
 *     z = w (2 - w) (D + w U)^{-1} D (D + w L)^{-1} r,     w = damping,
 * with each "triangular" solve (cyclic on the periodic grid) approximated by
 * `inner` Jacobi iterations started from D^{-1} times the right-hand side:
 *     y_0 = D^{-1} r,   y_{j+1} = D^{-1} r + (w/6) (y_j[i-ex] + y_j[i-ey] + y_j[i-ez]),
 *     z_0 = y,          z_{j+1} = y + (w/6) (z_j[i+ex] + z_j[i+ey] + z_j[i+ez]),
 * (D^{-1} w/h^2 = w/6), then z <- w (2 - w) z_inner.  The approximate solves
 * are polynomials in the backward (forward) shift, each the transpose of the
 * other, so the preconditioner is symmetric.  `outer` stationary steps:
 *     z <- z + SSOR(r - A z)   after the first z = SSOR(r).
 * Bounded boxes: D = (6/h^2) I with the box's h and L, U the couplings
 * between unknowns only (no neighbour across a face), which makes the
 * triangular solves true (non-cyclic) ones; A is the operator of bc.       */
static void or_ssor_once(int N, int bc, double inv_h2, double omega, int inner, const double *r,
                         double *z, double *y, double *t)
{
    int64_t n3 = (int64_t)N * N * N;
    double dinv = 1.0 / (6.0 * inv_h2);
    double c = omega / 6.0;
    /* the triangular factors hold the off-diagonal couplings between
     * unknowns: cyclic on the periodic grid, none across a bounded face */
    int tb = bc == 0 ? 0 : 1;
    for (int64_t i = 0; i < n3; ++i) y[i] = dinv * r[i];
    for (int j = 0; j < inner; ++j) {
        for (int iz = 0; iz < N; ++iz) {
            for (int iy = 0; iy < N; ++iy) {
                for (int ix = 0; ix < N; ++ix) {
                    double s = (or_ghost(y, N, tb, ix - 1, iy, iz) + or_ghost(y, N, tb, ix, iy - 1, iz)) +
                               or_ghost(y, N, tb, ix, iy, iz - 1);
                    t[OR_IDX(N, ix, iy, iz)] = dinv * r[OR_IDX(N, ix, iy, iz)] + c * s;
                }
            }
        }
        for (int64_t i = 0; i < n3; ++i) y[i] = t[i];
    }
    for (int64_t i = 0; i < n3; ++i) z[i] = y[i];
    for (int j = 0; j < inner; ++j) {
        for (int iz = 0; iz < N; ++iz) {
            for (int iy = 0; iy < N; ++iy) {
                for (int ix = 0; ix < N; ++ix) {
                    double s = (or_ghost(z, N, tb, ix + 1, iy, iz) + or_ghost(z, N, tb, ix, iy + 1, iz)) +
                               or_ghost(z, N, tb, ix, iy, iz + 1);
                    t[OR_IDX(N, ix, iy, iz)] = y[OR_IDX(N, ix, iy, iz)] + c * s;
                }
            }
        }
        for (int64_t i = 0; i < n3; ++i) z[i] = t[i];
    }
    double sc = omega * (2.0 - omega);
    for (int64_t i = 0; i < n3; ++i) z[i] = sc * z[i];
}

int or_ssor_apply_bc(int N, double L, int bc, double omega, int inner, int outer,
                     const double *r, double *z)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = or_inv_h(N, L, bc);
    double inv_h2 = inv_h * inv_h;
    double *y = (double *)malloc(sizeof(double) * (size_t)n3);
    double *t = (double *)malloc(sizeof(double) * (size_t)n3);
    double *res = (double *)malloc(sizeof(double) * (size_t)n3);
    double *dz = (double *)malloc(sizeof(double) * (size_t)n3);
    if (!y || !t || !res || !dz) { free(y); free(t); free(res); free(dz); return -1; }
    or_ssor_once(N, bc, inv_h2, omega, inner, r, z, y, t);
    for (int o = 1; o < outer; ++o) {
        or_apply_A_bc(N, L, bc, z, res);
        for (int64_t i = 0; i < n3; ++i) res[i] = r[i] - res[i];
        or_ssor_once(N, bc, inv_h2, omega, inner, res, dz, y, t);
        for (int64_t i = 0; i < n3; ++i) z[i] = z[i] + dz[i];
    }
    free(y); free(t); free(res); free(dz);
    return 0;
}

int or_ssor_apply(int N, double L, double omega, int inner, int outer, const double *r, double *z)
{
    return or_ssor_apply_bc(N, L, 0, omega, inner, outer, r, z);
}

/* PCG with the SSOR preconditioner: or_pcg's iteration and stopping rule with
 * z = SSOR(r) in place of the Jacobi scaling.  info as in or_pcg.          */
void or_pcg_ssor_bc(int N, double L, int bc, const double *b, double *x, double rtol,
                    int64_t max_iter, double omega, int inner, int outer, double *info)
{
    int64_t n3 = (int64_t)N * N * N;
    double *r = (double *)malloc(sizeof(double) * (size_t)n3);
    double *z = (double *)malloc(sizeof(double) * (size_t)n3);
    double *p = (double *)malloc(sizeof(double) * (size_t)n3);
    double *q = (double *)malloc(sizeof(double) * (size_t)n3);
    int64_t it = 0, repl = 0;
    int converged = 0;
    double rel = 0.0, trel = 0.0;
    double nb = sqrt(or_dot(n3, b, b));
    if (nb == 0.0) {
        for (int64_t i = 0; i < n3; ++i) x[i] = 0.0;
        info[0] = 0; info[1] = 0.0; info[2] = 0.0; info[3] = 1; info[4] = 0;
        free(r); free(z); free(p); free(q);
        return;
    }
    double tol = rtol * nb;
    double nr = or_true_residual(N, L, bc, b, x, r);
    rel = trel = nr / nb;
    if (nr <= tol) converged = 1;
    or_ssor_apply_bc(N, L, bc, omega, inner, outer, r, z);
    for (int64_t i = 0; i < n3; ++i) p[i] = z[i];
    double rz = or_dot(n3, r, z);
    while (!converged && it < max_iter) {
        or_apply_A_bc(N, L, bc, p, q);
        double alpha = rz / or_dot(n3, p, q);
        for (int64_t i = 0; i < n3; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        ++it;
        double rn = sqrt(or_dot(n3, r, r));
        rel = rn / nb;
        if (rn <= tol) {
            double tn = or_true_residual(N, L, bc, b, x, q);
            trel = tn / nb;
            if (tn <= tol) { converged = 1; break; }
            for (int64_t i = 0; i < n3; ++i) r[i] = q[i];
            or_ssor_apply_bc(N, L, bc, omega, inner, outer, r, z);
            for (int64_t i = 0; i < n3; ++i) p[i] = z[i];
            rz = or_dot(n3, r, z);
            rel = tn / nb;
            ++repl;
            continue;
        }
        or_ssor_apply_bc(N, L, bc, omega, inner, outer, r, z);
        double rz_new = or_dot(n3, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n3; ++i) p[i] = z[i] + beta * p[i];
    }
    if (!converged) trel = or_residual_norm_bc(N, L, bc, b, x) / nb;
    info[0] = (double)it; info[1] = rel; info[2] = trel; info[3] = converged; info[4] = (double)repl;
    free(r); free(z); free(p); free(q);
}

void or_pcg_ssor(int N, double L, const double *b, double *x, double rtol, int64_t max_iter,
                 double omega, int inner, int outer, double *info)
{
    or_pcg_ssor_bc(N, L, 0, b, x, rtol, max_iter, omega, inner, outer, info);
}

/* ------------------------------------------------------------------------ */
/* Field from potential (Sec. 2, Eq. poisson: E = -grad phi) with the
 * second-order central difference that matches the Laplacian:
 *   E_d[i] = -(phi[i+e_d] - phi[i-e_d]) / (2h),
 * a neighbour outside the grid taken through the boundary rule of bc.
 * The gauge is fixed first where the operator has constants in its kernel
 * (periodic, Neumann): phi <- phi - mean(phi) (written back); a Dirichlet
 * potential is unique and left as it is.
 * Returns W_x = (1/2) h^3 sum E_x^2, the energy of the x component
 * (the quantity of Fig. correctness_landau, with eps0 = 1).               */
double or_efield_bc(int N, double L, int bc, double *phi, double *ex, double *ey, double *ez)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = or_inv_h(N, L, bc);
    double ehalf = 0.5 * inv_h;
    double h = L / (double)(bc == 1 ? N + 1 : N);
    if (bc != 1) {
        double s = 0.0;
        for (int64_t i = 0; i < n3; ++i) s += phi[i];
        double mean = s / (double)n3;
        for (int64_t i = 0; i < n3; ++i) phi[i] = phi[i] - mean;
    }
#pragma omp parallel for schedule(static)
    for (int iz = 0; iz < N; ++iz) {
        int zm = or_nbr(iz, -1, N, bc), zp = or_nbr(iz, 1, N, bc);
        for (int iy = 0; iy < N; ++iy) {
            int ym = or_nbr(iy, -1, N, bc), yp = or_nbr(iy, 1, N, bc);
            for (int ix = 0; ix < N; ++ix) {
                int xm = or_nbr(ix, -1, N, bc), xp = or_nbr(ix, 1, N, bc);
                int64_t c = OR_IDX(N, ix, iy, iz);
                double vxm = xm < 0 ? 0.0 : phi[OR_IDX(N, xm, iy, iz)];
                double vxp = xp < 0 ? 0.0 : phi[OR_IDX(N, xp, iy, iz)];
                double vym = ym < 0 ? 0.0 : phi[OR_IDX(N, ix, ym, iz)];
                double vyp = yp < 0 ? 0.0 : phi[OR_IDX(N, ix, yp, iz)];
                double vzm = zm < 0 ? 0.0 : phi[OR_IDX(N, ix, iy, zm)];
                double vzp = zp < 0 ? 0.0 : phi[OR_IDX(N, ix, iy, zp)];
                ex[c] = -(vxp - vxm) * ehalf;
                ey[c] = -(vyp - vym) * ehalf;
                ez[c] = -(vzp - vzm) * ehalf;
            }
        }
    }
    double w = 0.0;
    for (int64_t i = 0; i < n3; ++i) w += ex[i] * ex[i];
    return 0.5 * w * (h * h * h);
}

double or_efield(int N, double L, double *phi, double *ex, double *ey, double *ez)
{
    return or_efield_bc(N, L, 0, phi, ex, ey, ez);
}

/* ------------------------------------------------------------------------ */
/* CIC gather of the three field components at one particle (Sec. 2: the same
 * shape as the scatter).  Sum order: z offset outer, then y, then x; each
 * term ((Wz*Wy)*Wx) * E[v].                                                */
static void or_gather_one(int N, double inv_h, double px, double py, double pz,
                          const double *ex, const double *ey, const double *ez,
                          double *Ep)
{
    int i[3];
    double w[3];
    or_locate(px, N, inv_h, &i[0], &w[0]);
    or_locate(py, N, inv_h, &i[1], &w[1]);
    or_locate(pz, N, inv_h, &i[2], &w[2]);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int c = 0; c < 2; ++c) {
        double wz = c ? w[2] : 1.0 - w[2];
        int vz = (i[2] + c) % N;
        for (int bb = 0; bb < 2; ++bb) {
            double wy = bb ? w[1] : 1.0 - w[1];
            int vy = (i[1] + bb) % N;
            for (int a = 0; a < 2; ++a) {
                double wx = a ? w[0] : 1.0 - w[0];
                int vx = (i[0] + a) % N;
                int64_t v = OR_IDX(N, vx, vy, vz);
                double W = (wz * wy) * wx;
                sx = sx + W * ex[v];
                sy = sy + W * ey[v];
                sz = sz + W * ez[v];
            }
        }
    }
    Ep[0] = sx; Ep[1] = sy; Ep[2] = sz;
}

/* Periodic wrap of one coordinate into [0, L); assumes |step| < L.  The last
 * test catches a tiny negative value whose x + L rounds up to L.          */
static double or_wrap(double xn, double L)
{
    if (xn >= L) xn = xn - L;
    if (xn < 0.0) xn = xn + L;
    if (xn >= L) xn = 0.0;
    return xn;
}

/* Gather + leapfrog push (Eq. eom, electrostatic, no external field):
 *   v <- v + (dt*qm) * E(x);   x <- wrap(x + dt * v);   key <- cell key of x.
 * dt*qm is formed once.  key may be NULL.                                  */
void or_gather_push(int64_t np, int N, double L, double dt, double qm,
                    double *x, double *y, double *z, double *vx, double *vy, double *vz,
                    const double *ex, const double *ey, const double *ez, uint32_t *key)
{
    double inv_h = (double)N / L;
    double coef = dt * qm;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        double Ep[3];
        or_gather_one(N, inv_h, x[p], y[p], z[p], ex, ey, ez, Ep);
        vx[p] = vx[p] + coef * Ep[0];
        vy[p] = vy[p] + coef * Ep[1];
        vz[p] = vz[p] + coef * Ep[2];
        x[p] = or_wrap(x[p] + dt * vx[p], L);
        y[p] = or_wrap(y[p] + dt * vy[p], L);
        z[p] = or_wrap(z[p] + dt * vz[p], L);
        if (key) {
            int ix, iy, iz;
            double w;
            or_locate(x[p], N, inv_h, &ix, &w);
            or_locate(y[p], N, inv_h, &iy, &w);
            or_locate(z[p], N, inv_h, &iz, &w);
            key[p] = (uint32_t)OR_IDX(N, ix, iy, iz);
        }
    }
}

/* Leapfrog start: v^{-1/2} = v^0 - (dt/2) qm E(x^0); positions unchanged.
 * The factor is formed once as (-0.5 * dt) * qm.                          */
void or_half_kick(int64_t np, int N, double L, double dt, double qm,
                  const double *x, const double *y, const double *z,
                  double *vx, double *vy, double *vz,
                  const double *ex, const double *ey, const double *ez)
{
    double inv_h = (double)N / L;
    double coef = (-0.5 * dt) * qm;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        double Ep[3];
        or_gather_one(N, inv_h, x[p], y[p], z[p], ex, ey, ez, Ep);
        vx[p] = vx[p] + coef * Ep[0];
        vy[p] = vy[p] + coef * Ep[1];
        vz[p] = vz[p] + coef * Ep[2];
    }
}

/* CIC gather of a scalar grid field at each particle (same weights and order
 * as or_gather_one); used by the deposit/gather adjoint pin.               */
void or_gather_scalar(int64_t np, int N, double L, const double *x, const double *y,
                      const double *z, const double *F, double *out)
{
    double inv_h = (double)N / L;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        double Ep[3];
        or_gather_one(N, inv_h, x[p], y[p], z[p], F, F, F, Ep);
        out[p] = Ep[0];
    }
}

/* ------------------------------------------------------------------------ */
/* Single-precision operator for the mixed-precision solver: the same
 * neighbour-sum order as or_apply_A, every operation in binary32.          */
static void or_apply_A32(int N, float inv_h2f, const float *u, float *Au)
{
#pragma omp parallel for schedule(static)
    for (int iz = 0; iz < N; ++iz) {
        int zm = (iz + N - 1) % N, zp = (iz + 1) % N;
        for (int iy = 0; iy < N; ++iy) {
            int ym = (iy + N - 1) % N, yp = (iy + 1) % N;
            for (int ix = 0; ix < N; ++ix) {
                int xm = (ix + N - 1) % N, xp = (ix + 1) % N;
                float t = ((u[OR_IDX(N, xm, iy, iz)] + u[OR_IDX(N, xp, iy, iz)]) +
                           (u[OR_IDX(N, ix, ym, iz)] + u[OR_IDX(N, ix, yp, iz)])) +
                          (u[OR_IDX(N, ix, iy, zm)] + u[OR_IDX(N, ix, iy, zp)]);
                Au[OR_IDX(N, ix, iy, iz)] = (6.0f * u[OR_IDX(N, ix, iy, iz)] - t) * inv_h2f;
            }
        }
    }
}

/* FP64 accumulation of a binary32 dot product: each product formed in FP64. */
static double or_dot32(int64_t n, const float *a, const float *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (double)a[i] * (double)b[i];
    return s;
}

/* Mixed-precision solve (not in the paper; classical iterative refinement,
 * Wilkinson / Moler, as analysed by Carson & Higham 2018; with `reliable`,
 * the inner Krylov space is kept across refinements -- "reliable updates",
 * Sleijpen & van der Vorst 1996, as used by Clark et al. 2010):
 *   outer, FP64:  r = b - A x;  stop when ||r|| <= rtol ||b||;
 *   inner, FP32 vectors / FP32 operator / FP32 Jacobi, dot products
 *   accumulated in FP64:  Jacobi-PCG on A d = r from d = 0, stopped when
 *   ||r_in|| <= inner_rtol ||r|| or after max_inner iterations;
 *   outer, FP64:  x <- x + d.
 * The inner right-hand side is r scaled by 1/||r|| before rounding to FP32
 * (and d scaled back), so FP32 range never limits the refinement.
 * Reliable form: an inner solve that ended at its tolerance or its step cap
 * hands its last direction p_j to the next one instead of restarting from
 * p = M r.  In true (unscaled) units the next direction is CG's,
 *   p' = M r' + beta p_j,  beta = (r'.M r') / (r_j.M r_j),
 * with r' = b - A x the recomputed residual standing in for the recursive
 * r_{j+1} (residual replacement) and r_j the residual p_j was built from.  In
 * the scaled variables of each inner solve (r / ||r||) this is
 *   p~' = M r~' + beta~ p~_j,  beta~ = (nr' / nr) (r~'.M r~') / (r~_j.M r~_j),
 * nr, nr' the outer residual norms before and after the refinement.
 * Residual replacement keeps CG's recurrences only while the replaced
 * residual stays close to the recursive one; FP32 inner solves drift from
 * their true residual by about eps32 kappa(A), which at large N exceeds a
 * tight inner tolerance.  So the direction is carried only if the
 * refinement's true reduction nr'/nr is within a factor 4 of the inner
 * solve's recursive one ||r~_in|| / ||r~_0||; otherwise the inner solve
 * restarts from p = M r.  (This is a residual-gap test in the sense of van
 * der Vorst and Ye, SIAM J. Sci. Comput. 22 (2000): the gap between the
 * true residual nr' and the recursively updated one, rec * nr, is at least
 * nr' - rec * nr, so the test refuses the carry once that lower bound of the
 * gap exceeds three times the recursive residual.  The factor is this
 * library's choice.)
 * Progress stop: a refinement makes progress when its true residual falls
 * below 0.9 times the smallest one so far; after 3 refinements in a row
 * without progress the refinement loop ends and FP64 Jacobi-PCG (or_pcg)
 * finishes the solve from the current x with at most max_iter iterations.
 * info: [0]=outer steps, [1]=total inner iterations, [2]=true rel. residual,
 *       [3]=converged, [4]=refinements whose carried direction the gap test
 *       refused (reliable form), [5]=1 if the progress stop switched to FP64
 *       PCG, [6]=FP64 PCG iterations after that switch.                   */
#define OR_MIXED_STALL 3
#define OR_MIXED_PROGRESS 0.9
void or_mixed_pcg_ex(int N, double L, const double *b, double *x, double rtol,
                     int64_t max_outer, double inner_rtol, int64_t max_inner, int reliable,
                     int64_t max_iter, double *info)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = (double)N / L;
    float inv_h2f = (float)(inv_h * inv_h);
    float minvf = (float)(1.0 / (6.0 * (inv_h * inv_h)));
    double *r = (double *)malloc(sizeof(double) * (size_t)n3);
    float *ri = (float *)malloc(sizeof(float) * (size_t)n3);
    float *d = (float *)malloc(sizeof(float) * (size_t)n3);
    float *p = (float *)malloc(sizeof(float) * (size_t)n3);
    float *q = (float *)malloc(sizeof(float) * (size_t)n3);
    float *zz = (float *)malloc(sizeof(float) * (size_t)n3);
    int64_t outer = 0, inner_total = 0;
    int converged = 0;
    double nb = sqrt(or_dot(n3, b, b));
    double trel = 0.0;
    for (int k = 0; k < 7; ++k) info[k] = 0.0;
    if (nb == 0.0) {
        for (int64_t i = 0; i < n3; ++i) x[i] = 0.0;
        info[3] = 1;
        free(r); free(ri); free(d); free(p); free(q); free(zz);
        return;
    }
    int have_dir = 0;        /* reliable form: p holds the last direction */
    double rz_last = 0.0, nr_prev = 0.0, rec_last = 0.0;
    double best = 0.0;       /* smallest true residual so far */
    int stall = 0, switched = 0;
    int64_t refused = 0;
    for (;;) {
        double nr = or_true_residual(N, L, 0, b, x, r);
        trel = nr / nb;
        if (nr <= rtol * nb) { converged = 1; break; }
        if (!isfinite(nr)) break;
        if (outer == 0 || nr < OR_MIXED_PROGRESS * best) { best = nr; stall = 0; }
        else if (++stall >= OR_MIXED_STALL) { switched = 1; break; }
        if (outer >= max_outer) break;
        ++outer;
        double sc = 1.0 / nr;
        for (int64_t i = 0; i < n3; ++i) { ri[i] = (float)(r[i] * sc); d[i] = 0.0f; }
        double n0 = sqrt(or_dot32(n3, ri, ri));
        for (int64_t i = 0; i < n3; ++i) zz[i] = minvf * ri[i];
        double rz = or_dot32(n3, ri, zz);
        /* carry the direction only while the replacement is consistent */
        if (have_dir && !(nr <= 4.0 * rec_last * nr_prev)) {
            have_dir = 0;
            if (reliable) ++refused;
        }
        double bc = reliable && have_dir ? (nr / nr_prev) * (rz / rz_last) : 0.0;
        if (reliable && have_dir && isfinite(bc)) {
            float bf = (float)bc;
            for (int64_t i = 0; i < n3; ++i) p[i] = zz[i] + bf * p[i];
        } else {
            for (int64_t i = 0; i < n3; ++i) p[i] = zz[i];
        }
        have_dir = 0;
        for (int64_t k = 0; k < max_inner; ++k) {
            or_apply_A32(N, inv_h2f, p, q);
            double pq = or_dot32(n3, p, q);
            double alpha = rz / pq;
            if (!isfinite(alpha) || !(pq > 0.0)) break; /* FP32 breakdown */
            float af = (float)alpha;
            for (int64_t i = 0; i < n3; ++i) {
                d[i] = d[i] + af * p[i];
                ri[i] = ri[i] - af * q[i];
            }
            ++inner_total;
            double rn = sqrt(or_dot32(n3, ri, ri));
            for (int64_t i = 0; i < n3; ++i) zz[i] = minvf * ri[i];
            double rz_new = or_dot32(n3, ri, zz);
            if (rn <= inner_rtol * n0 || k + 1 == max_inner) {
                rz_last = rz; /* r_j.M r_j of the residual p_j was built from */
                have_dir = isfinite(rn);
                rec_last = rn / n0; /* the inner solve's recursive reduction */
                break;
            }
            float bf = (float)(rz_new / rz);
            rz = rz_new;
            for (int64_t i = 0; i < n3; ++i) p[i] = zz[i] + bf * p[i];
        }
        for (int64_t i = 0; i < n3; ++i) x[i] = x[i] + nr * (double)d[i];
        nr_prev = nr;
    }
    free(r); free(ri); free(d); free(p); free(q); free(zz);
    if (switched) {
        double pinfo[5];
        or_pcg(N, L, b, x, rtol, max_iter, pinfo);
        converged = (int)pinfo[3];
        trel = pinfo[2];
        info[6] = pinfo[0];
    }
    info[0] = (double)outer; info[1] = (double)inner_total; info[2] = trel; info[3] = converged;
    info[4] = (double)refused; info[5] = switched;
}

void or_mixed_pcg(int N, double L, const double *b, double *x, double rtol,
                  int64_t max_outer, double inner_rtol, int64_t max_inner, double *info)
{
    double full[7];
    or_mixed_pcg_ex(N, L, b, x, rtol, max_outer, inner_rtol, max_inner, 0, 20000, full);
    for (int k = 0; k < 4; ++k) info[k] = full[k];
}

/* ------------------------------------------------------------------------ */
/* Flexible preconditioned CG (not in the paper; Notay, SIAM J. Sci. Comput.
 * 22 (2000); Golub & Ye, SIAM J. Sci. Comput. 21 (1999)) with a possibly
 * nonlinear preconditioner z = M(r) supplied as a callback:
 *   r = b - A x;  z = M(r);  p = z
 *   loop:  q = A p;  alpha = (z.r)/(p.q);  x += alpha p;  r -= alpha q;
 *          stop test as in or_pcg;  z' = M(r);
 *          beta = -(z'.q)/(p.q);  p = z' + beta p.
 * Fallback to Jacobi-PCG from the current x (r = b - A x, p = M_J^{-1} r),
 * permanently for the solve, when (z.r) <= 0, anything is non-finite, or the
 * best ||r|| has not improved by at least 1% over `window` consecutive
 * iterations.  After the switch the iteration is exactly or_pcg's loop.
 * info: [0]=total iterations, [1]=flexible iterations, [2]=true rel.
 * residual, [3]=converged, [4]=fell back (1/0).                           */
typedef void (*or_precond_fn)(const double *r, double *z, void *user);

void or_fcg(int N, double L, const double *b, double *x, double rtol, int64_t max_iter,
            int window, or_precond_fn M, void *user, double *info)
{
    int64_t n3 = (int64_t)N * N * N;
    double inv_h = (double)N / L;
    double minv = 1.0 / (6.0 * (inv_h * inv_h));
    double *r = (double *)malloc(sizeof(double) * (size_t)n3);
    double *z = (double *)malloc(sizeof(double) * (size_t)n3);
    double *p = (double *)malloc(sizeof(double) * (size_t)n3);
    double *q = (double *)malloc(sizeof(double) * (size_t)n3);
    int64_t it = 0, flex_it = 0;
    int converged = 0, fell_back = 0;
    double nb = sqrt(or_dot(n3, b, b));
    if (nb == 0.0) {
        for (int64_t i = 0; i < n3; ++i) x[i] = 0.0;
        info[0] = 0; info[1] = 0; info[2] = 0.0; info[3] = 1; info[4] = 0;
        free(r); free(z); free(p); free(q);
        return;
    }
    double tol = rtol * nb;
    double nr = or_true_residual(N, L, 0, b, x, r);
    double best = nr;
    int since_best = 0;
    if (nr <= tol) converged = 1;
    int flexible = 1;
    double rz = 0.0;
    if (!converged) {
        M(r, z, user);
        rz = or_dot(n3, z, r);
        if (!(rz > 0.0) || !isfinite(rz)) flexible = 0;
        if (flexible) for (int64_t i = 0; i < n3; ++i) p[i] = z[i];
    }
    while (!converged && it < max_iter) {
        if (!flexible) {
            if (!fell_back) {
                fell_back = 1;
                nr = or_true_residual(N, L, 0, b, x, r);
                if (nr <= tol) { converged = 1; break; }
                for (int64_t i = 0; i < n3; ++i) { z[i] = minv * r[i]; p[i] = z[i]; }
                rz = or_dot(n3, r, z);
            }
            or_apply_A(N, L, p, q);
            double alpha = rz / or_dot(n3, p, q);
            for (int64_t i = 0; i < n3; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
            ++it;
            double rn = sqrt(or_dot(n3, r, r));
            if (rn <= tol) {
                double tn = or_true_residual(N, L, 0, b, x, q);
                if (tn <= tol) { converged = 1; break; }
                for (int64_t i = 0; i < n3; ++i) { r[i] = q[i]; z[i] = minv * r[i]; p[i] = z[i]; }
                rz = or_dot(n3, r, z);
                continue;
            }
            for (int64_t i = 0; i < n3; ++i) z[i] = minv * r[i];
            double rz_new = or_dot(n3, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < n3; ++i) p[i] = z[i] + beta * p[i];
            continue;
        }
        or_apply_A(N, L, p, q);
        double pq = or_dot(n3, p, q);
        double alpha = rz / pq;
        if (!isfinite(alpha) || !(pq > 0.0)) { flexible = 0; continue; }
        for (int64_t i = 0; i < n3; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
        ++it; ++flex_it;
        double rn = sqrt(or_dot(n3, r, r));
        if (!isfinite(rn)) { flexible = 0; continue; }
        if (rn <= tol) {
            double tn = or_true_residual(N, L, 0, b, x, z);
            if (tn <= tol) { converged = 1; break; }
            for (int64_t i = 0; i < n3; ++i) r[i] = z[i];
            rn = tn;
        }
        if (rn < 0.99 * best) { best = rn; since_best = 0; }
        else if (++since_best >= window) { flexible = 0; continue; }
        M(r, z, user);
        double zr = or_dot(n3, z, r);
        if (!(zr > 0.0) || !isfinite(zr)) { flexible = 0; continue; }
        double beta = -or_dot(n3, z, q) / pq;
        if (!isfinite(beta)) { flexible = 0; continue; }
        rz = zr;
        for (int64_t i = 0; i < n3; ++i) p[i] = z[i] + beta * p[i];
    }
    double trel = or_residual_norm(N, L, b, x) / nb;
    info[0] = (double)it; info[1] = (double)flex_it; info[2] = trel; info[3] = converged;
    info[4] = fell_back;
    free(r); free(z); free(p); free(q);
}

/* The Jacobi preconditioner as an or_precond_fn (user points at h^2/6). */
void or_precond_jacobi(const double *r, double *z, void *user)
{
    const double *par = (const double *)user; /* par[0] = h^2/6, par[1] = n3 */
    int64_t n3 = (int64_t)par[1];
    for (int64_t i = 0; i < n3; ++i) z[i] = par[0] * r[i];
}

/* ------------------------------------------------------------------------ */
/* The deposit definition evaluated at single vertices (for sampled checks at
 * sizes where the whole grid is out of reach): out[k] = sum over the given
 * particles, in order, of the CIC weight of particle p at vertex vid[k],
 * times q/h^3.  Particles whose cell is not adjacent contribute nothing.   */
void or_deposit_vertices(int64_t np, int N, double L, double q, const double *x,
                         const double *y, const double *z, int64_t nv, const int64_t *vid,
                         double *out)
{
    double inv_h = (double)N / L;
    double qh3 = q * (inv_h * inv_h * inv_h);
    for (int64_t k = 0; k < nv; ++k) {
        int vx = (int)(vid[k] % N), vy = (int)((vid[k] / N) % N), vz = (int)(vid[k] / ((int64_t)N * N));
        double acc = 0.0;
        for (int64_t p = 0; p < np; ++p) {
            int i[3];
            double w[3];
            or_locate(x[p], N, inv_h, &i[0], &w[0]);
            or_locate(y[p], N, inv_h, &i[1], &w[1]);
            or_locate(z[p], N, inv_h, &i[2], &w[2]);
            int c = (vz - i[2] + N) % N, bb = (vy - i[1] + N) % N, a = (vx - i[0] + N) % N;
            if (c > 1 || bb > 1 || a > 1) continue;
            double wz = c ? w[2] : 1.0 - w[2];
            double wy = bb ? w[1] : 1.0 - w[1];
            double wx = a ? w[0] : 1.0 - w[0];
            acc += (wz * wy) * wx;
        }
        out[k] = acc * qh3;
    }
}

/* Threads the OpenMP loops above use (for reporting the CPU baseline). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
#else
int or_num_threads(void) { return 1; }
#endif
