/*
 * FP64 CPU oracle for the 25-point, 8th-order acoustic leapfrog propagator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * statement of what the GPU path computes.  It is used by the test-suite, by
 * the smoke check and by the CPU-baseline leg of the benchmark, and by
 * nothing else.  It shares no code, header, table or constant with the HIP
 * library: the two are written independently from the paper.
 *
 * What is computed (paper, Section III):
 *   - Eq. 1, the constant-density acoustic wave equation
 *     (1/V^2) u_tt - lap(u) = f;
 *   - Eq. 2, its second-order leapfrog discretisation
 *     u^{n+1} - Q u^n + u^{n-1} = dt^2 V^2 f^n,  Q = 2 + dt^2 V^2 lap;
 *   - the 25-point Laplacian: four neighbours each way along every axis plus
 *     the centre, with per-axis coefficients c_m / h_a^2.  The centre is
 *     counted once with the sum of the three axis centre coefficients, as the
 *     paper does for the own-cell contribution in its Section IV-C (X/Y
 *     stencil computation);
 *   - Algorithm 1, the time loop, starting from a quiescent field, with one
 *     point source added each step (Section IV-D, time integration);
 *   - a ghost layer of 4 cells on every face (Section IV-B: the local column
 *     is extended by 4 cells on each side), held at zero (Dirichlet) or,
 *     for tests only, filled periodically.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):
 *   - coefficients: the paper never prints them; they are the standard
 *     8th-order central second-derivative weights, computed here from their
 *     closed form c_m = 2 (-1)^{m+1} (p!)^2 / (m^2 (p-m)! (p+m)!), p = 4,
 *     c_0 = -2 sum_{m>=1} c_m;
 *   - a per-cell k = V^2 dt^2 multiplies the Laplacian (Eq. 2 read literally);
 *   - the source value for step n is added to u^{n+1} after the update
 *     (Eq. 2's time index), verbatim as supplied by the caller;
 *   - absorbing sponge (Cerjan et al., Geophysics 1985), applied to both time
 *     levels in single-pass form
 *       u^{n+1} = G (2 u^n - G u^{n-1} + k lap(u^n)),  G = gx(x) gy(y) gz(z),
 *       g(i) = exp(-(alpha (W - d))^2) if d = min(i, n-1-i) < W, else 1;
 *     W = 0 gives G = 1 everywhere, i.e. plain Eq. 2;
 *   - receivers sample u^{n+1} after the source is added; trace row n is the
 *     field at time (n+1) dt.
 *
 * Memory: every field handed across this interface is a dense interior
 * array [nz][ny][nx], x fastest.  Internally each time level is held in a
 * padded array [nz+8][ny+8][nx+8] whose ghost layer is zero (or periodic).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GHOST 4
#define ORACLE_BC_ZERO 0
#define ORACLE_BC_PERIODIC 1

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= (double)i;
    return f;
}

/* The five weights c_0..c_4 of the 8th-order central second derivative
 * (p = 4 neighbours each way), from the closed form stated in the header. */
void oracle_coefficients(double c[5])
{
    const int p = 4;
    const double pf = factorial(p);
    double sum = 0.0;
    for (int m = 1; m <= p; ++m) {
        double sign = (m % 2 == 1) ? 1.0 : -1.0;
        c[m] = 2.0 * sign * pf * pf /
               ((double)(m * m) * factorial(p - m) * factorial(p + m));
        sum += c[m];
    }
    c[0] = -2.0 * sum;
}

/* One axis of the sponge: g(i), i = 0..n-1, for width W and strength alpha. */
void oracle_sponge_profile(int n, int width, double alpha, double *g)
{
    for (int i = 0; i < n; ++i) {
        int d = i < n - 1 - i ? i : n - 1 - i;
        if (d < width) {
            double t = alpha * (double)(width - d);
            g[i] = exp(-t * t);
        } else {
            g[i] = 1.0;
        }
    }
}

/* Index into a padded array [nz+8][ny+8][nx+8]; z, y, x are interior
 * coordinates and may reach -4 .. n+3. */
static inline size_t pidx(int z, int y, int x, int nyp, int nxp)
{
    return ((size_t)(z + GHOST) * (size_t)nyp + (size_t)(y + GHOST)) * (size_t)nxp +
           (size_t)(x + GHOST);
}

/* Interior-index wrap used by the periodic ghost fill. */
static inline int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Fill the ghost layer of a padded array by periodic continuation of the
 * interior (tests only: plane waves on a torus). */
static void fill_periodic(double *a, int nx, int ny, int nz)
{
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST;
    for (int z = -GHOST; z < nz + GHOST; ++z)
        for (int y = -GHOST; y < ny + GHOST; ++y)
            for (int x = -GHOST; x < nx + GHOST; ++x) {
                int inside = z >= 0 && z < nz && y >= 0 && y < ny && x >= 0 && x < nx;
                if (!inside)
                    a[pidx(z, y, x, nyp, nxp)] =
                        a[pidx(wrap(z, nz), wrap(y, ny), wrap(x, nx), nyp, nxp)];
            }
}

/* The 25-point Laplacian at interior point (z, y, x) of a padded array. */
static inline double lap_at(const double *a, int z, int y, int x, int nyp, int nxp,
                            const double c[5], double idx2, double idy2, double idz2)
{
    double centre = a[pidx(z, y, x, nyp, nxp)];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int m = 1; m <= 4; ++m) {
        sx += c[m] * (a[pidx(z, y, x + m, nyp, nxp)] + a[pidx(z, y, x - m, nyp, nxp)]);
        sy += c[m] * (a[pidx(z, y + m, x, nyp, nxp)] + a[pidx(z, y - m, x, nyp, nxp)]);
        sz += c[m] * (a[pidx(z + m, y, x, nyp, nxp)] + a[pidx(z - m, y, x, nyp, nxp)]);
    }
    return c[0] * (idx2 + idy2 + idz2) * centre + idx2 * sx + idy2 * sy + idz2 * sz;
}

/* Laplacian of a caller-filled padded array a_pad [nz+8][ny+8][nx+8]
 * (ghost values as given: zero, periodic or an analytic continuation);
 * result on the interior, dense [nz][ny][nx]. */
int oracle_laplacian(int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *a_pad, double *lap, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || !a_pad || !lap || !(dx > 0) || !(dy > 0) || !(dz > 0))
        return -1;
    double c[5];
    oracle_coefficients(c);
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST;
    const double idx2 = 1.0 / (dx * dx), idy2 = 1.0 / (dy * dy), idz2 = 1.0 / (dz * dz);
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                lap[((size_t)z * ny + y) * nx + x] =
                    lap_at(a_pad, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
    return 0;
}

static void to_padded(const double *dense, double *pad, int nx, int ny, int nz)
{
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            memcpy(&pad[pidx(z, y, 0, nyp, nxp)], &dense[((size_t)z * ny + y) * nx],
                   sizeof(double) * (size_t)nx);
}

static void from_padded(const double *pad, double *dense, int nx, int ny, int nz)
{
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            memcpy(&dense[((size_t)z * ny + y) * nx], &pad[pidx(z, y, 0, nyp, nxp)],
                   sizeof(double) * (size_t)nx);
}

/*
 * Run nt leapfrog steps (Algorithm 1 with Eq. 2).
 *   k        [nz][ny][nx]  V^2 dt^2 per cell;
 *   s        [nt]          source value added at (src) in step j (may be NULL);
 *   rec_zyx  [nrec][3]     receiver interior coordinates (z, y, x);
 *   a_cur    [nz][ny][nx]  in: u^{n0};    out: u^{n0+nt};
 *   a_prev   [nz][ny][nx]  in: u^{n0-1};  out: u^{n0+nt-1};
 *   traces   [nt][nrec]    row j = u^{n0+j+1} at the receivers (may be NULL).
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_run(int nx, int ny, int nz, double dx, double dy, double dz, int bc,
               int sponge_width, double sponge_alpha, const double *k, int nt,
               const double *s, int src_z, int src_y, int src_x, int nrec,
               const int32_t *rec_zyx, double *a_cur, double *a_prev, double *traces,
               int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || nt < 0 || !k || !a_cur || !a_prev)
        return -1;
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || sponge_width < 0)
        return -1;
    if (bc != ORACLE_BC_ZERO && bc != ORACLE_BC_PERIODIC)
        return -1;
    if (s && (src_z < 0 || src_z >= nz || src_y < 0 || src_y >= ny || src_x < 0 || src_x >= nx))
        return -1;
    if (nrec < 0 || (nrec > 0 && (!rec_zyx || !traces)))
        return -1;
    for (int r = 0; r < nrec; ++r) {
        const int32_t *q = &rec_zyx[3 * r];
        if (q[0] < 0 || q[0] >= nz || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nx)
            return -1;
    }
    if (nthreads < 1)
        nthreads = 1;

    double c[5];
    oracle_coefficients(c);
    const double idx2 = 1.0 / (dx * dx), idy2 = 1.0 / (dy * dy), idz2 = 1.0 / (dz * dz);
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST, nzp = nz + 2 * GHOST;
    const size_t npad = (size_t)nxp * nyp * nzp;

    double *gx = malloc(sizeof(double) * (size_t)nx);
    double *gy = malloc(sizeof(double) * (size_t)ny);
    double *gz = malloc(sizeof(double) * (size_t)nz);
    double *prev = calloc(npad, sizeof(double));
    double *cur = calloc(npad, sizeof(double));
    double *next = calloc(npad, sizeof(double));
    if (!gx || !gy || !gz || !prev || !cur || !next) {
        free(gx); free(gy); free(gz); free(prev); free(cur); free(next);
        return -2;
    }
    oracle_sponge_profile(nx, sponge_width, sponge_alpha, gx);
    oracle_sponge_profile(ny, sponge_width, sponge_alpha, gy);
    oracle_sponge_profile(nz, sponge_width, sponge_alpha, gz);
    to_padded(a_cur, cur, nx, ny, nz);
    to_padded(a_prev, prev, nx, ny, nz);

    for (int j = 0; j < nt; ++j) {
        if (bc == ORACLE_BC_PERIODIC)
            fill_periodic(cur, nx, ny, nz);
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    double kk = k[((size_t)z * ny + y) * nx + x];
                    double L = lap_at(cur, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
                    double G = gx[x] * gy[y] * gz[z];
                    next[p] = G * (2.0 * cur[p] - G * prev[p] + kk * L);
                }
        if (s)
            next[pidx(src_z, src_y, src_x, nyp, nxp)] += s[j];
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = &rec_zyx[3 * r];
            traces[(size_t)j * nrec + r] = next[pidx(q[0], q[1], q[2], nyp, nxp)];
        }
        /* rotate: the ghost layer of every buffer stays zero in the
         * Dirichlet case because only interior points are ever written */
        double *t = prev;
        prev = cur;
        cur = next;
        next = t;
    }

    from_padded(cur, a_cur, nx, ny, nz);
    from_padded(prev, a_prev, nx, ny, nz);
    free(gx); free(gy); free(gz); free(prev); free(cur); free(next);
    return 0;
}

/*
 * One step of the same update evaluated only at a list of points, from
 * single-precision copies of u^n, u^{n-1} and k (as a GPU run leaves them),
 * in FP64.  Used to check outputs of full-size runs point by point.
 *   k, u_cur, u_prev  dense [nz][ny][nx] FP32; points outside the interior
 *                     read as zero (Dirichlet ghost layer);
 *   src_value         added when a point is the source (if has_src);
 *   pts_zyx [npts][3], out [npts].
 */
int oracle_step_points(int nx, int ny, int nz, double dx, double dy, double dz,
                       int sponge_width, double sponge_alpha, const float *k,
                       const float *u_cur, const float *u_prev, int has_src, int src_z,
                       int src_y, int src_x, double src_value, int npts,
                       const int32_t *pts_zyx, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !k || !u_cur || !u_prev || npts < 0 ||
        (npts > 0 && (!pts_zyx || !out)))
        return -1;
    double c[5];
    oracle_coefficients(c);
    const double h2[3] = {1.0 / (dz * dz), 1.0 / (dy * dy), 1.0 / (dx * dx)};
    const int dims[3] = {nz, ny, nx};
    for (int i = 0; i < npts; ++i) {
        const int32_t *q = &pts_zyx[3 * i];
        if (q[0] < 0 || q[0] >= nz || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nx)
            return -1;
        size_t p = ((size_t)q[0] * ny + q[1]) * nx + q[2];
        double centre = (double)u_cur[p];
        double L = c[0] * (h2[0] + h2[1] + h2[2]) * centre;
        for (int a = 0; a < 3; ++a) {
            double sa = 0.0;
            for (int m = 1; m <= 4; ++m) {
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int zyx[3] = {q[0], q[1], q[2]};
                    zyx[a] += sgn * m;
                    double v = 0.0;
                    if (zyx[a] >= 0 && zyx[a] < dims[a])
                        v = (double)u_cur[((size_t)zyx[0] * ny + zyx[1]) * nx + zyx[2]];
                    sa += c[m] * v;
                }
            }
            L += h2[a] * sa;
        }
        double g[3];
        for (int a = 0; a < 3; ++a) {
            int d = q[a] < dims[a] - 1 - q[a] ? q[a] : dims[a] - 1 - q[a];
            double t = sponge_alpha * (double)(sponge_width - d);
            g[a] = d < sponge_width ? exp(-t * t) : 1.0;
        }
        double G = g[0] * g[1] * g[2];
        double v = G * (2.0 * centre - G * (double)u_prev[p] + (double)k[p] * L);
        if (has_src && q[0] == src_z && q[1] == src_y && q[2] == src_x)
            v += src_value;
        out[i] = v;
    }
    return 0;
}

/*
 * Discrete adjoint of oracle_run: the gradient with respect to k of a
 * scalar loss whose derivative with respect to the traces is trace_grad
 * (for the misfit 0.5 sum (trace - d_obs)^2 it is the residual).  The
 * source values are fixed inputs (not differentiated).
 *
 * Derivation (Lagrangian of the time loop; not in the paper, whose method
 * is the forward recurrence only): with constraints
 *   C_n = a^{n+1} - G (2 a^n - G a^{n-1} + K L a^n) - s_n e_src,  n = 0..N-1,
 * and multipliers lambda^{n+1}, stationarity in a^m (m = 1..N) gives
 *   lambda^m = R^T g_{m-1} + 2 G lambda^{m+1} + L (K G lambda^{m+1}) - G^2 lambda^{m+2},
 *   lambda^{N+1} = lambda^{N+2} = 0,
 * (L symmetric, G and K diagonal), and the gradient is
 *   dJ/dk = sum_{m=1..N} lambda^m * G * (L a^{m-1}).
 * Every forward level is kept (small grids only).
 *   trace_grad [nt][nrec], grad_k [nz][ny][nx] (overwritten).
 */
int oracle_adjoint(int nx, int ny, int nz, double dx, double dy, double dz, int sponge_width,
                   double sponge_alpha, const double *k, int nt, const double *s, int src_z,
                   int src_y, int src_x, int nrec, const int32_t *rec_zyx,
                   const double *trace_grad, double *grad_k, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || nt < 0 || !k || !grad_k || sponge_width < 0)
        return -1;
    if (!(dx > 0) || !(dy > 0) || !(dz > 0))
        return -1;
    if (s && (src_z < 0 || src_z >= nz || src_y < 0 || src_y >= ny || src_x < 0 || src_x >= nx))
        return -1;
    if (nrec < 0 || (nrec > 0 && (!rec_zyx || !trace_grad)))
        return -1;
    for (int r = 0; r < nrec; ++r) {
        const int32_t *q = &rec_zyx[3 * r];
        if (q[0] < 0 || q[0] >= nz || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nx)
            return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
    double c[5];
    oracle_coefficients(c);
    const double idx2 = 1.0 / (dx * dx), idy2 = 1.0 / (dy * dy), idz2 = 1.0 / (dz * dz);
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST, nzp = nz + 2 * GHOST;
    const size_t npad = (size_t)nxp * nyp * nzp;
    const size_t nint = (size_t)nx * ny * nz;

    double *gx = malloc(sizeof(double) * (size_t)nx);
    double *gy = malloc(sizeof(double) * (size_t)ny);
    double *gz = malloc(sizeof(double) * (size_t)nz);
    double *levels = calloc(npad * (size_t)(nt + 2), sizeof(double)); /* a^{-1} .. a^{N} */
    double *lam = calloc(npad * 3, sizeof(double));                  /* lambda^{m}, ^{m+1}, ^{m+2} */
    double *w = calloc(npad, sizeof(double));
    if (!gx || !gy || !gz || !levels || !lam || !w) {
        free(gx); free(gy); free(gz); free(levels); free(lam); free(w);
        return -2;
    }
    oracle_sponge_profile(nx, sponge_width, sponge_alpha, gx);
    oracle_sponge_profile(ny, sponge_width, sponge_alpha, gy);
    oracle_sponge_profile(nz, sponge_width, sponge_alpha, gz);
#define LEVEL(n) (levels + npad * (size_t)((n) + 1))
#define GPT(z, y, x) (gx[x] * gy[y] * gz[z])

    /* forward, keeping a^0 .. a^N (a^{-1} = a^0 = 0) */
    for (int n = 0; n < nt; ++n) {
        const double *cur = LEVEL(n), *prev = LEVEL(n - 1);
        double *next = LEVEL(n + 1);
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    double kk = k[((size_t)z * ny + y) * nx + x];
                    double L = lap_at(cur, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
                    double G = GPT(z, y, x);
                    next[p] = G * (2.0 * cur[p] - G * prev[p] + kk * L);
                }
        if (s)
            next[pidx(src_z, src_y, src_x, nyp, nxp)] += s[n];
    }

    /* adjoint, from m = N down to 1 */
    for (size_t i = 0; i < nint; ++i)
        grad_k[i] = 0.0;
    double *l0 = lam, *l1 = lam + npad, *l2 = lam + 2 * npad; /* lambda^m, ^{m+1}, ^{m+2} */
    for (int m = nt; m >= 1; --m) {
        /* w = K G lambda^{m+1} */
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    w[p] = k[((size_t)z * ny + y) * nx + x] * GPT(z, y, x) * l1[p];
                }
        const double *am1 = LEVEL(m - 1);
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    double G = GPT(z, y, x);
                    l0[p] = 2.0 * G * l1[p] + lap_at(w, z, y, x, nyp, nxp, c, idx2, idy2, idz2) -
                            G * G * l2[p];
                }
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = &rec_zyx[3 * r];
            l0[pidx(q[0], q[1], q[2], nyp, nxp)] += trace_grad[(size_t)(m - 1) * nrec + r];
        }
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    grad_k[((size_t)z * ny + y) * nx + x] +=
                        l0[p] * GPT(z, y, x) * lap_at(am1, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
                }
        /* rotate: (m, m+1, m+2) -> (m-1, m, m+1) */
        double *t = l2;
        l2 = l1;
        l1 = l0;
        l0 = t;
    }
#undef LEVEL
#undef GPT
    free(gx); free(gy); free(gz); free(levels); free(lam); free(w);
    return 0;
}

/*
 * Tangent-linear model of oracle_run (zero initial levels, zero ghost
 * layer): the derivative of the traces with respect to k along dk.
 * Differentiating the sponge-damped update of Eq. 2,
 *   a^{n+1} = G (2 a^n - G a^{n-1} + K L a^n) + s_n e_src,
 * with the source values fixed gives
 *   da^{n+1} = G (2 da^n - G da^{n-1} + K L da^n + dK L a^n),  da^0 = da^{-1} = 0,
 * and row n of the result is R da^{n+1} (R samples the receivers).  It is
 * the linear map whose transpose oracle_adjoint applies.
 *   dk [nz][ny][nx]; dtraces [nt][nrec] (overwritten).
 * Returns 0, -1 on invalid arguments, -2 when memory runs out.
 */
int oracle_tangent(int nx, int ny, int nz, double dx, double dy, double dz, int sponge_width,
                   double sponge_alpha, const double *k, const double *dk, int nt, const double *s,
                   int src_z, int src_y, int src_x, int nrec, const int32_t *rec_zyx,
                   double *dtraces, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || nt < 0 || !k || !dk || sponge_width < 0)
        return -1;
    if (!(dx > 0) || !(dy > 0) || !(dz > 0))
        return -1;
    if (s && (src_z < 0 || src_z >= nz || src_y < 0 || src_y >= ny || src_x < 0 || src_x >= nx))
        return -1;
    if (nrec < 0 || (nrec > 0 && (!rec_zyx || !dtraces)))
        return -1;
    for (int r = 0; r < nrec; ++r) {
        const int32_t *q = &rec_zyx[3 * r];
        if (q[0] < 0 || q[0] >= nz || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nx)
            return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
    double c[5];
    oracle_coefficients(c);
    const double idx2 = 1.0 / (dx * dx), idy2 = 1.0 / (dy * dy), idz2 = 1.0 / (dz * dz);
    const int nxp = nx + 2 * GHOST, nyp = ny + 2 * GHOST, nzp = nz + 2 * GHOST;
    const size_t npad = (size_t)nxp * nyp * nzp;

    double *gx = malloc(sizeof(double) * (size_t)nx);
    double *gy = malloc(sizeof(double) * (size_t)ny);
    double *gz = malloc(sizeof(double) * (size_t)nz);
    double *buf = calloc(npad * 6, sizeof(double));
    if (!gx || !gy || !gz || !buf) {
        free(gx); free(gy); free(gz); free(buf);
        return -2;
    }
    oracle_sponge_profile(nx, sponge_width, sponge_alpha, gx);
    oracle_sponge_profile(ny, sponge_width, sponge_alpha, gy);
    oracle_sponge_profile(nz, sponge_width, sponge_alpha, gz);
    double *prev = buf, *cur = buf + npad, *next = buf + 2 * npad;          /* a */
    double *dprev = buf + 3 * npad, *dcur = buf + 4 * npad, *dnext = buf + 5 * npad; /* da */

    for (int n = 0; n < nt; ++n) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t p = pidx(z, y, x, nyp, nxp);
                    size_t i = ((size_t)z * ny + y) * nx + x;
                    double G = gx[x] * gy[y] * gz[z];
                    double La = lap_at(cur, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
                    double Lda = lap_at(dcur, z, y, x, nyp, nxp, c, idx2, idy2, idz2);
                    next[p] = G * (2.0 * cur[p] - G * prev[p] + k[i] * La);
                    dnext[p] = G * (2.0 * dcur[p] - G * dprev[p] + k[i] * Lda + dk[i] * La);
                }
        if (s)
            next[pidx(src_z, src_y, src_x, nyp, nxp)] += s[n];
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = &rec_zyx[3 * r];
            dtraces[(size_t)n * nrec + r] = dnext[pidx(q[0], q[1], q[2], nyp, nxp)];
        }
        double *t = prev;
        prev = cur;
        cur = next;
        next = t;
        t = dprev;
        dprev = dcur;
        dcur = dnext;
        dnext = t;
    }
    free(gx); free(gy); free(gz); free(buf);
    return 0;
}
