/*
 * Plain FP64 CPU oracle for the Ewald k-space problem (TEST INFRASTRUCTURE).
 *
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library.  The GPU library never links or calls it, and it
 * shares no code, header or table with the GPU path.
 *
 * Everything is double precision, written for clarity, not speed: direct
 * exponentials (no fast-Gaussian-gridding recurrence), one particle at a
 * time, triple loops over the stencil.  The FFT step lives in the Python
 * driver (oracle/se_oracle.py), which uses numpy.fft as a library primitive.
 *
 * Conventions (Coulomb constant 1, box [0,L)^3, grid spacing h = L/M):
 *   grid point j = (jx,jy,jz) sits at x_j = j*h; grids are stored
 *   G[(jz*M + jy)*M + jx] (x fastest).
 *
 * Paper: Saffar Shamshirgar, Hess & Tornberg, "A comparison of the Spectral
 * Ewald and Smooth Particle Mesh Ewald methods in GROMACS" (arXiv:1712.04718).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static long wrap_index(long i, long M)
{
    long r = i % M;
    return r < 0 ? r + M : r;
}

/* First stencil index of the truncated Gaussian along one axis.
 * Section 4 truncates each Gaussian to P grid points per direction; the
 * paper does not say where the P points start.  Reading used here: even P
 * takes the P points nearest to the particle with one more point on the
 * right, i.e. floor(x/h) - P/2 + 1 ... floor(x/h) + P/2; odd P centres on
 * the nearest grid point, round(x/h) -/+ (P-1)/2. */
static long se_first_index(double x, double h, int P)
{
    double u = x / h;
    if (P % 2 == 0)
        return (long)floor(u) - P / 2 + 1;
    return (long)floor(u + 0.5) - (P - 1) / 2;
}

/*
 * SE spreading, eq. (4.5) with the truncation of section 4:
 *   G_j = h^3 * sum_n q_n (2 xi^2 / (pi eta))^{3/2} exp(-2 xi^2 |x_j - x_n|^2 / eta)
 * i.e. H(x_j) of eq. (4.5) times the cell volume h^3 ("charge per cell"),
 * restricted to the P^3 stencil of each particle.  The Gaussian factorises
 * over the three axes (eq. 4.10), so each axis contributes
 *   h * sqrt(a/pi) * exp(-a t^2),  a = 2 xi^2 / eta,  t = j h - x_n .
 * G must hold M^3 doubles; it is overwritten.
 */
void or_se_spread(int N, const double *x, const double *q, double L, int M,
                  int P, double xi, double eta, double *G)
{
    const double h = L / M;
    const double a = 2.0 * xi * xi / eta;
    const double beta = h * sqrt(a / M_PI);
    double *g = (double *)malloc(sizeof(double) * 3 * P);
    long *idx = (long *)malloc(sizeof(long) * 3 * P);
    memset(G, 0, sizeof(double) * (size_t)M * M * M);
    for (int n = 0; n < N; ++n) {
        for (int d = 0; d < 3; ++d) {
            double xd = x[3 * n + d];
            long i0 = se_first_index(xd, h, P);
            for (int j = 0; j < P; ++j) {
                long i = i0 + j;
                double t = (double)i * h - xd;
                g[d * P + j] = beta * exp(-a * t * t);
                idx[d * P + j] = wrap_index(i, M);
            }
        }
        for (int jz = 0; jz < P; ++jz)
            for (int jy = 0; jy < P; ++jy)
                for (int jx = 0; jx < P; ++jx) {
                    long cell = (idx[2 * P + jz] * M + idx[P + jy]) * M + idx[jx];
                    G[cell] += q[n] * g[jx] * g[P + jy] * g[2 * P + jz];
                }
    }
    free(g);
    free(idx);
}

/*
 * SE gathering, eq. (4.9) (the trapezoidal rule applied to eq. 4.8): the
 * potential at x_m is the same window summed against the scaled grid Phi,
 *   phi_m = sum_{j in stencil(m)} Phi_j W(x_j - x_m),
 * where Phi is already multiplied by 4 pi / L^3 and W is the h^3-weighted
 * window used in or_se_spread.  Force, eq. (4.12) read as F = -dE/dx_m:
 *   F_m = -q_m sum_j Phi_j * (2a (x_j - x_m)) * W(x_j - x_m),
 * which is minus twice the expression printed in eq. (4.12); the factor and
 * sign follow from differentiating E = 1/2 sum q phi (eq. 1.2, 1.3) and are
 * pinned by finite differences in the tests.
 * phi (N) and F (3N) are overwritten; either may be NULL.
 */
void or_se_gather(int N, const double *x, const double *q, double L, int M,
                  int P, double xi, double eta, const double *Phi,
                  double *phi, double *F)
{
    const double h = L / M;
    const double a = 2.0 * xi * xi / eta;
    const double beta = h * sqrt(a / M_PI);
#pragma omp parallel for schedule(static)
    for (int m = 0; m < N; ++m) {
        double g[3][64], t[3][64];
        long idx[3][64];
        for (int d = 0; d < 3; ++d) {
            double xd = x[3 * m + d];
            long i0 = se_first_index(xd, h, P);
            for (int j = 0; j < P; ++j) {
                long i = i0 + j;
                t[d][j] = (double)i * h - xd;
                g[d][j] = beta * exp(-a * t[d][j] * t[d][j]);
                idx[d][j] = wrap_index(i, M);
            }
        }
        double s = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        for (int jz = 0; jz < P; ++jz)
            for (int jy = 0; jy < P; ++jy)
                for (int jx = 0; jx < P; ++jx) {
                    long cell = (idx[2][jz] * M + idx[1][jy]) * M + idx[0][jx];
                    double w = Phi[cell] * g[0][jx] * g[1][jy] * g[2][jz];
                    s += w;
                    fx += w * 2.0 * a * t[0][jx];
                    fy += w * 2.0 * a * t[1][jy];
                    fz += w * 2.0 * a * t[2][jz];
                }
        if (phi)
            phi[m] = s;
        if (F) {
            F[3 * m + 0] = -q[m] * fx;
            F[3 * m + 1] = -q[m] * fy;
            F[3 * m + 2] = -q[m] * fz;
        }
    }
}

/*
 * Cardinal B-spline of order p (section 6.1): M_2(u) = 1 - |u - 1| on
 * [0,2], zero elsewhere; M_p(u) = u/(p-1) M_{p-1}(u) + (p-u)/(p-1) M_{p-1}(u-1).
 * Plain recursion, exponential in p, fine for p <= 10.
 */
double or_bspline(int p, double u)
{
    if (p == 1)
        return (u >= 0.0 && u < 1.0) ? 1.0 : 0.0;
    if (p == 2)
        return (u >= 0.0 && u <= 2.0) ? 1.0 - fabs(u - 1.0) : 0.0;
    return u / (p - 1) * or_bspline(p - 1, u) +
           (p - u) / (p - 1) * or_bspline(p - 1, u - 1.0);
}

/* Derivative of M_p: M_p'(u) = M_{p-1}(u) - M_{p-1}(u-1) (differentiating
 * the convolution M_p = M_{p-1} * M_1). */
double or_bspline_deriv(int p, double u)
{
    return or_bspline(p - 1, u) - or_bspline(p - 1, u - 1.0);
}

/*
 * SPME spreading, eq. (6.1), in grid units u = x/h: the p grid points with
 * 0 < u - k < p, i.e. k = floor(u) - p + 1 ... floor(u), receive
 *   Q_k += q_n prod_d M_p(u_d - k_d).
 * Q holds M^3 doubles and is overwritten.  Q is a charge per cell: the
 * B-splines form a partition of unity, so sum(Q) = sum(q).
 */
void or_spme_spread(int N, const double *x, const double *q, double L, int M,
                    int p, double *Q)
{
    const double h = L / M;
    double *wgt = (double *)malloc(sizeof(double) * 3 * p);
    long *idx = (long *)malloc(sizeof(long) * 3 * p);
    memset(Q, 0, sizeof(double) * (size_t)M * M * M);
    for (int n = 0; n < N; ++n) {
        for (int d = 0; d < 3; ++d) {
            double u = x[3 * n + d] / h;
            long k0 = (long)floor(u) - p + 1;
            for (int j = 0; j < p; ++j) {
                long k = k0 + j;
                wgt[d * p + j] = or_bspline(p, u - (double)k);
                idx[d * p + j] = wrap_index(k, M);
            }
        }
        for (int jz = 0; jz < p; ++jz)
            for (int jy = 0; jy < p; ++jy)
                for (int jx = 0; jx < p; ++jx) {
                    long cell = (idx[2 * p + jz] * M + idx[p + jy]) * M + idx[jx];
                    Q[cell] += q[n] * wgt[jx] * wgt[p + jy] * wgt[2 * p + jz];
                }
    }
    free(wgt);
    free(idx);
}

/*
 * SPME gathering, eq. (6.3): phi_m = sum_k Phi_k prod_d M_p(u_d - k_d) with
 * Phi already holding 4 pi / L^3 times the inverse transform.  Force by
 * analytic differentiation of the window (section 3.1):
 *   F_m,d = -q_m sum_k Phi_k (1/h) M_p'(u_d - k_d) prod_{e != d} M_p(u_e - k_e).
 */
void or_spme_gather(int N, const double *x, const double *q, double L, int M,
                    int p, const double *Phi, double *phi, double *F)
{
    const double h = L / M;
#pragma omp parallel for schedule(static)
    for (int m = 0; m < N; ++m) {
        double w[3][16], dw[3][16];
        long idx[3][16];
        for (int d = 0; d < 3; ++d) {
            double u = x[3 * m + d] / h;
            long k0 = (long)floor(u) - p + 1;
            for (int j = 0; j < p; ++j) {
                long k = k0 + j;
                w[d][j] = or_bspline(p, u - (double)k);
                dw[d][j] = or_bspline_deriv(p, u - (double)k) / h;
                idx[d][j] = wrap_index(k, M);
            }
        }
        double s = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        for (int jz = 0; jz < p; ++jz)
            for (int jy = 0; jy < p; ++jy)
                for (int jx = 0; jx < p; ++jx) {
                    long cell = (idx[2][jz] * M + idx[1][jy]) * M + idx[0][jx];
                    double v = Phi[cell];
                    s += v * w[0][jx] * w[1][jy] * w[2][jz];
                    fx += v * dw[0][jx] * w[1][jy] * w[2][jz];
                    fy += v * w[0][jx] * dw[1][jy] * w[2][jz];
                    fz += v * w[0][jx] * w[1][jy] * dw[2][jz];
                }
        if (phi)
            phi[m] = s;
        if (F) {
            F[3 * m + 0] = -q[m] * fx;
            F[3 * m + 1] = -q[m] * fy;
            F[3 * m + 2] = -q[m] * fz;
        }
    }
}

/*
 * Direct (exact) Ewald Fourier-space sum, eqs. (1.5)-(1.7), long-range
 * parts, over all k = 2 pi n / L with n != 0 and |k| <= kcut:
 *   phi_m = (4 pi / V) sum_k c_k Re(e^{i k.x_m} S(k)),
 *   E     = (2 pi / V) sum_k c_k |S(k)|^2,
 *   F_m   = (4 pi q_m / V) sum_k c_k k Im(e^{i k.x_m} S(k)),
 * with c_k = exp(-k^2 / 4 xi^2) / k^2 and S(k) = sum_n q_n e^{-i k.x_n}.
 * The force is -dE/dx_m of the energy line (eq. 1.7 carries a stray 1/2).
 * Any of E, phi, F may be NULL.
 */
void or_ewald_kspace(int N, const double *x, const double *q, double L,
                     double xi, double kcut, double *E, double *phi, double *F)
{
    const double V = L * L * L;
    const double twopiL = 2.0 * M_PI / L;
    const int nmax = (int)ceil(kcut / twopiL);
    double *cs = (double *)malloc(sizeof(double) * N);
    double *sn = (double *)malloc(sizeof(double) * N);
    double e = 0.0;
    if (phi)
        memset(phi, 0, sizeof(double) * N);
    if (F)
        memset(F, 0, sizeof(double) * 3 * N);
    for (int nz = -nmax; nz <= nmax; ++nz)
        for (int ny = -nmax; ny <= nmax; ++ny)
            for (int nx = -nmax; nx <= nmax; ++nx) {
                if (nx == 0 && ny == 0 && nz == 0)
                    continue;
                double kx = twopiL * nx, ky = twopiL * ny, kz = twopiL * nz;
                double k2 = kx * kx + ky * ky + kz * kz;
                if (k2 > kcut * kcut)
                    continue;
                double ck = exp(-k2 / (4.0 * xi * xi)) / k2;
                double C = 0.0, S = 0.0; /* S(k) = C - i S */
                for (int n = 0; n < N; ++n) {
                    double th = kx * x[3 * n] + ky * x[3 * n + 1] + kz * x[3 * n + 2];
                    cs[n] = cos(th);
                    sn[n] = sin(th);
                    C += q[n] * cs[n];
                    S += q[n] * sn[n];
                }
                e += ck * (C * C + S * S);
                for (int m = 0; m < N; ++m) {
                    if (phi)
                        phi[m] += ck * (cs[m] * C + sn[m] * S);
                    if (F) {
                        double im = sn[m] * C - cs[m] * S;
                        F[3 * m + 0] += ck * kx * q[m] * im;
                        F[3 * m + 1] += ck * ky * q[m] * im;
                        F[3 * m + 2] += ck * kz * q[m] * im;
                    }
                }
            }
    if (E)
        *E = 2.0 * M_PI / V * e;
    if (phi)
        for (int m = 0; m < N; ++m)
            phi[m] *= 4.0 * M_PI / V;
    if (F)
        for (int i = 0; i < 3 * N; ++i)
            F[i] *= 4.0 * M_PI / V;
    free(cs);
    free(sn);
}

/*
 * Direct real-space Ewald sum, eqs. (1.5)-(1.7), short-range parts:
 *   phi_m = sum_n sum'_p q_n erfc(xi r)/r,  r = |x_m - x_n + p L| <= rc,
 * the prime dropping the p = 0 term when n = m; E = 1/2 sum_m q_m phi_m;
 *   F_m = q_m sum_n q_n sum'_p (2 xi/sqrt(pi) e^{-xi^2 r^2} + erfc(xi r)/r) r_vec / r^2.
 * Every periodic image within rc is visited explicitly (no cell list), so
 * rc may exceed L/2.  Any of E, phi, F may be NULL.
 */
void or_ewald_real(int N, const double *x, const double *q, double L, double xi,
                   double rc, double *E, double *phi, double *F)
{
    const int np = (int)ceil(rc / L) + 1;
    double e = 0.0;
#pragma omp parallel for schedule(dynamic) reduction(+ : e)
    for (int m = 0; m < N; ++m) {
        double pm = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        for (int n = 0; n < N; ++n)
            for (int pz = -np; pz <= np; ++pz)
                for (int py = -np; py <= np; ++py)
                    for (int px = -np; px <= np; ++px) {
                        if (n == m && px == 0 && py == 0 && pz == 0)
                            continue;
                        double rx = x[3 * m] - x[3 * n] + px * L;
                        double ry = x[3 * m + 1] - x[3 * n + 1] + py * L;
                        double rz = x[3 * m + 2] - x[3 * n + 2] + pz * L;
                        double r2 = rx * rx + ry * ry + rz * rz;
                        if (r2 > rc * rc)
                            continue;
                        double r = sqrt(r2);
                        double ec = erfc(xi * r) / r;
                        pm += q[n] * ec;
                        double fr = q[n] *
                                    (2.0 * xi / sqrt(M_PI) * exp(-xi * xi * r2) + ec) / r2;
                        fx += fr * rx;
                        fy += fr * ry;
                        fz += fr * rz;
                    }
        if (phi)
            phi[m] = pm;
        if (F) {
            F[3 * m] = q[m] * fx;
            F[3 * m + 1] = q[m] * fy;
            F[3 * m + 2] = q[m] * fz;
        }
        e += 0.5 * q[m] * pm;
    }
    if (E)
        *E = e;
}

/* Real-space sums of or_ewald_real for the nt target particles idx[0..nt)
 * only (the sources are all N particles): phi[t], F[3t..3t+2] for
 * particle idx[t]. */
void or_ewald_real_targets(int N, const double *x, const double *q, double L, double xi,
                           double rc, int nt, const int *idx, double *phi, double *F)
{
    const int np = (int)ceil(rc / L) + 1;
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < nt; ++t) {
        const int m = idx[t];
        double pm = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        for (int n = 0; n < N; ++n)
            for (int pz = -np; pz <= np; ++pz)
                for (int py = -np; py <= np; ++py)
                    for (int px = -np; px <= np; ++px) {
                        if (n == m && px == 0 && py == 0 && pz == 0)
                            continue;
                        double rx = x[3 * m] - x[3 * n] + px * L;
                        double ry = x[3 * m + 1] - x[3 * n + 1] + py * L;
                        double rz = x[3 * m + 2] - x[3 * n + 2] + pz * L;
                        double r2 = rx * rx + ry * ry + rz * rz;
                        if (r2 > rc * rc)
                            continue;
                        double r = sqrt(r2);
                        double ec = erfc(xi * r) / r;
                        pm += q[n] * ec;
                        double fr = q[n] *
                                    (2.0 * xi / sqrt(M_PI) * exp(-xi * xi * r2) + ec) / r2;
                        fx += fr * rx;
                        fy += fr * ry;
                        fz += fr * rz;
                    }
        phi[t] = pm;
        F[3 * t] = q[m] * fx;
        F[3 * t + 1] = q[m] * fy;
        F[3 * t + 2] = q[m] * fz;
    }
}
