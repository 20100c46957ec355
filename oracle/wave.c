/*
 * CPU ORACLE (test infrastructure only) -- FP64 acoustic wave solver.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this code.  It shares nothing with the HIP path.
 *
 * What it computes (paper Sec. 2, Eqs. 1-4; discretisation of Sec. 3
 * "Reference Problem": second order in time, high order in space, absorbing
 * layer):
 *
 *   Laplacian  (Lap u)(i) = sum_axes sum_{k=-M..M} a_|k| u(i + k e_axis) / h^2,
 *              u = 0 outside the computational grid, a_k the central
 *              order-2M second-derivative weights (closed form below).
 *   Row k of the leapfrog system (k = 1..N, u^0 = u^-1 = 0):
 *              D u^k = (2 M + Lap) u^{k-1} - B u^{k-2} + s^{k-1}
 *              with M = m/dt^2, D = M + eta/(2dt), B = M - eta/(2dt).
 *   Damping    eta = sigma / vmax^2,
 *              sigma = sigma_max * sum_axes (d_axis/nbl)^2,
 *              sigma_max = 3 vmax ln(1000) / (2 nbl h),
 *              d_axis = distance (in points) into the layer.
 *   Imaging    g -= u^k (lam^k - 2 lam^{k+1} + lam^{k+2}) / dt^2   (Eq. 4 as
 *              the exact derivative of the discrete objective).
 *
 * Everything is plain loops with bounds checks.  OpenMP only splits the
 * outermost loop over independent points; no reduction depends on it.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

#define MAXM 8

/* a[0..M] for space order so = 2M:
 * a_k = 2 (-1)^{k+1} (M!)^2 / (k^2 (M-k)! (M+k)!),  a_0 = -2 sum_{k>=1} a_k. */
int or_fd_coeffs(int so, double *a)
{
    if (so != 4 && so != 8 && so != 16) return -1;
    int M = so / 2;
    double fM = 1.0;
    for (int i = 2; i <= M; ++i) fM *= i;
    double s = 0.0;
    for (int k = 1; k <= M; ++k) {
        double fmk = 1.0, fpk = 1.0;
        for (int i = 2; i <= M - k; ++i) fmk *= i;
        for (int i = 2; i <= M + k; ++i) fpk *= i;
        double v = 2.0 * fM * fM / ((double)k * k * fmk * fpk);
        a[k] = (k % 2 == 1) ? v : -v;
        s += a[k];
    }
    a[0] = -2.0 * s;
    return 0;
}

static void strides(int ndim, const long *N, long *st)
{
    st[ndim - 1] = 1;
    for (int d = ndim - 2; d >= 0; --d) st[d] = st[d + 1] * N[d + 1];
}

static long npoints(int ndim, const long *N)
{
    long n = 1;
    for (int d = 0; d < ndim; ++d) n *= N[d];
    return n;
}

/* out = Lap_h u */
void or_laplacian(int ndim, const long *N, double h, int so,
                  const double *u, double *out)
{
    double a[MAXM + 1];
    or_fd_coeffs(so, a);
    int M = so / 2;
    long st[3];
    strides(ndim, N, st);
    long np = npoints(ndim, N);
    double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        long idx[3], rem = p;
        for (int d = 0; d < ndim; ++d) { idx[d] = rem / st[d]; rem %= st[d]; }
        double acc = 0.0;
        for (int d = 0; d < ndim; ++d) {
            acc += a[0] * u[p];
            for (int k = 1; k <= M; ++k) {
                double l = (idx[d] - k >= 0) ? u[p - k * st[d]] : 0.0;
                double r = (idx[d] + k < N[d]) ? u[p + k * st[d]] : 0.0;
                acc += a[k] * (l + r);
            }
        }
        out[p] = acc * ih2;
    }
}

/* eta(i): damping coefficient of the absorbing layer */
void or_damping(int ndim, const long *N, int nbl, double h, double vmax,
                double *eta)
{
    long st[3];
    strides(ndim, N, st);
    long np = npoints(ndim, N);
    if (nbl <= 0) { memset(eta, 0, sizeof(double) * np); return; }
    double smax = 3.0 * vmax * log(1000.0) / (2.0 * nbl * h);
    for (long p = 0; p < np; ++p) {
        long rem = p;
        double s = 0.0;
        for (int d = 0; d < ndim; ++d) {
            long i = rem / st[d];
            rem %= st[d];
            long dist = 0;
            if (i < nbl) dist = nbl - i;
            else if (i > N[d] - 1 - nbl) dist = i - (N[d] - 1 - nbl);
            double r = (double)dist / nbl;
            s += r * r;
        }
        eta[p] = smax * s / (vmax * vmax);
    }
}

/*
 * One row of the leapfrog system, solved for the new level:
 *   out = [ (2M + Lap) u1 - B u2 + rhs ] / D
 * rhs = rhs_dense (may be NULL) + sparse point terms sp_val[j] at sp_idx[j]
 * (repeated indices add).  out must not alias u1 or u2.
 */
void or_step(int ndim, const long *N, double h, int so, double dt,
             const double *m, const double *eta,
             const double *u1, const double *u2, double *out,
             const double *rhs_dense, int nsp, const long *sp_idx,
             const double *sp_val)
{
    long np = npoints(ndim, N);
    or_laplacian(ndim, N, h, so, u1, out);   /* out <- Lap u1 */
    double idt2 = 1.0 / (dt * dt);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double M = m[p] * idt2;
        double B = M - eta[p] / (2.0 * dt);
        double r = 2.0 * M * u1[p] + out[p] - B * u2[p];
        if (rhs_dense) r += rhs_dense[p];
        out[p] = r;
    }
    for (int j = 0; j < nsp; ++j) out[sp_idx[j]] += sp_val[j];
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double M = m[p] * idt2;
        double D = M + eta[p] / (2.0 * dt);
        out[p] /= D;
    }
}

/* g -= u (l0 - 2 l1 + l2) / dt^2 */
void or_image(long np, double dt, const double *u, const double *l0,
              const double *l1, const double *l2, double *g)
{
    double idt2 = 1.0 / (dt * dt);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p)
        g[p] -= u[p] * (l0[p] - 2.0 * l1[p] + l2[p]) * idt2;
}

/* Born source of row k: out = -(dm/dt^2) (u^k - 2u^{k-1} + u^{k-2}) */
void or_born_rhs(long np, double dt, const double *dm, const double *uk,
                 const double *uk1, const double *uk2, double *out)
{
    double idt2 = 1.0 / (dt * dt);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p)
        out[p] = -dm[p] * idt2 * (uk[p] - 2.0 * uk1[p] + uk2[p]);
}
