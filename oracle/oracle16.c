/*
 * Emulation of the reduced-precision storage forms (16-bit fields, FP32
 * arithmetic) on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c, and sharing no code with the HIP
 * library.  The paper runs FP32 throughout; storing the wave fields in 16
 * bits is this project's extension of its Eq. 2 update (reading R16 of the
 * design notes).  The FP64 oracle gives the accuracy of those forms; this
 * file pins the forms themselves: it carries out the same scheme, written
 * from its specification below, in plain C with IEEE FP32 arithmetic
 * (explicit fmaf, no contraction), so that a GPU run can be compared with
 * it bit for bit.
 *
 * The scheme, for one step n -> n+1 (Eq. 2 with the sponge, as oracle.c):
 *   - storage: a 16-bit field holds x * 2^-e, one exponent e per time level,
 *     as IEEE binary16 (FP16) or bfloat16 (BF16), rounded to nearest even;
 *     k is stored once with the exponent ek = ex(max k) - 14, where
 *     max k = f * 2^ex, f in [0.5, 1);
 *   - two-level forms keep u^n and u^{n-1}; u-and-change forms keep u^n and
 *     d^n = u^n - u^{n-1}, d with exponent e_n + 1;
 *   - the exponent of u^{n+1}: with M_n the largest |u^n| written (in FP32,
 *     before rounding to 16 bits) and s_n the source value of the step,
 *     bound = 8 max(M_n, M_{n-1}) + |s_n|, e = ex(bound) - 14, clamped to
 *     [-110, 110] (0 when bound is 0);
 *   - arithmetic in FP32 on the stored (unscaled) values, every power of
 *     two folded into the coefficients, in this order: A = 2^(e_n - e),
 *     B = 2^(e_{n-1} - e) (two levels) or 2^(e_n + 1 - e) (u and change),
 *     C = 2^ek A, weights w = (c / h^2) C;
 *       lap = w_0 U;  for m = 1..4: lap = fma(wx_m, X+m + X-m, lap),
 *                                   lap = fma(wy_m, Y+m + Y-m, lap),
 *                                   lap = fma(wz_m, Z+m + Z-m, lap);
 *       t = fma(K, lap, 2A U);  p = B P (two levels) or fma(-B, D, A U);
 *       t = fma(-g, p, t);  out = g t  (+ s_n 2^-e at the source cell),
 *     g = (gx gy) gz the sponge factor in FP32; stored u^{n+1} = Q(out);
 *     the change d^{n+1} = 0.5 (out - A U) is stored with exponent e + 1;
 *   - receivers read the stored u^{n+1} decoded: Q(out) 2^e.
 * Ghost cells are zero.  Coefficients c_m = 2 (-1)^(m+1) (4!)^2 /
 * (m^2 (4-m)! (4+m)!), c_0 = -2 sum c_m, as exact fractions; the sponge
 * profile is the one of oracle.c, rounded to FP32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE16_F16 1
#define ORACLE16_BF16 2
#define ORACLE16_F16_UV 3
#define ORACLE16_BF16_UV 4

/* IEEE binary16 -> float (exact). */
float oracle16_f16_decode(uint16_t h)
{
    const int sign = h >> 15, ex = (h >> 10) & 0x1f, man = h & 0x3ff;
    float v;
    if (ex == 0)
        v = ldexpf((float)man, -24);
    else if (ex == 31)
        v = man ? NAN : INFINITY;
    else
        v = ldexpf((float)(1024 + man), ex - 25);
    return sign ? -v : v;
}

/* float -> IEEE binary16, round to nearest, ties to even. */
uint16_t oracle16_f16_encode(float x)
{
    if (isnan(x))
        return 0x7e00;
    const uint16_t sign = signbit(x) ? 0x8000 : 0;
    const float a = fabsf(x);
    if (a >= 65520.0f) /* half-way between 65504 and 2^16 rounds up */
        return sign | 0x7c00;
    if (a < 0x1p-14f) { /* subnormal range: a multiple of 2^-24 */
        const float q = rintf(a * 0x1p24f);
        return sign | (uint16_t)q; /* q = 1024 is the smallest normal, encoded alike */
    }
    int ex;
    (void)frexpf(a, &ex); /* a = f 2^ex, f in [0.5, 1) */
    int E = ex - 1;        /* a in [2^E, 2^(E+1)) */
    float q = rintf(ldexpf(a, 10 - E));
    if (q == 2048.0f) {
        q = 1024.0f;
        ++E;
    }
    if (E > 15)
        return sign | 0x7c00;
    return sign | (uint16_t)((E + 15) << 10) | (uint16_t)((int)q - 1024);
}

/* bfloat16 (the upper half of a float) -> float (exact). */
float oracle16_bf16_decode(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float v;
    memcpy(&v, &u, sizeof v);
    return v;
}

/* float -> bfloat16, round to nearest, ties to even: the 16 bits dropped
 * are compared with half of the last kept bit's weight. */
uint16_t oracle16_bf16_encode(float x)
{
    if (isnan(x))
        return 0x7fc0;
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    const uint32_t kept = u >> 16, dropped = u & 0xffffu;
    uint32_t r = kept;
    if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u)))
        r = kept + 1u; /* carries into the exponent when the mantissa overflows */
    return (uint16_t)r;
}

static float dec16(int bf, uint16_t v) { return bf ? oracle16_bf16_decode(v) : oracle16_f16_decode(v); }
static uint16_t enc16(int bf, float x) { return bf ? oracle16_bf16_encode(x) : oracle16_f16_encode(x); }

/* exponent e with bound < 2^(e + 14), as the scheme chooses it */
static int level_exponent(float bound)
{
    if (!(bound > 0.0f) || isinf(bound))
        return 0;
    int ex;
    (void)frexpf(bound, &ex);
    int e = ex - 14;
    if (e < -110)
        e = -110;
    if (e > 110)
        e = 110;
    return e;
}

/* c_0..c_4 of the 8th-order second derivative as doubles rounded once from
 * exact fractions (c_m = num_m / den_m; c_0 = -2 sum c_m over a common
 * denominator). */
static void exact_weights(double c[5])
{
    long long num[5], den[5];
    long long f[9];
    f[0] = 1;
    for (int i = 1; i <= 8; ++i)
        f[i] = f[i - 1] * i;
    for (int m = 1; m <= 4; ++m) {
        num[m] = 2 * f[4] * f[4] * ((m % 2 == 1) ? 1 : -1);
        den[m] = (long long)m * m * f[4 - m] * f[4 + m];
    }
    long long L = 1; /* common denominator */
    for (int m = 1; m <= 4; ++m) {
        long long a = L, b = den[m];
        while (b) {
            long long t = a % b;
            a = b;
            b = t;
        }
        L = L / a * den[m];
    }
    long long s = 0;
    for (int m = 1; m <= 4; ++m)
        s += num[m] * (L / den[m]);
    num[0] = -2 * s;
    den[0] = L;
    for (int m = 0; m <= 4; ++m)
        c[m] = (double)num[m] / (double)den[m];
}

static void sponge_f32(int n, int width, double alpha, float *g)
{
    for (int i = 0; i < n; ++i) {
        int d = i < n - 1 - i ? i : n - 1 - i;
        if (d < width) {
            double t = alpha * (double)(width - d);
            g[i] = (float)exp(-t * t);
        } else {
            g[i] = 1.0f;
        }
    }
}

/*
 * Run nt steps of a 16-bit form from zero fields.
 *   k32        dense [nz][ny][nx] FP32 k = V^2 dt^2 as handed to the GPU;
 *   s          nt FP32 source values (or NULL), src_z < 0 for no source;
 *   rec        [nrec][3] receivers (z, y, x);
 * Outputs: u_bits, d_bits (u-and-change forms; may be NULL otherwise)
 * dense [nz][ny][nx] stored 16-bit values after the last step, exps[nt]
 * the exponent of u^{n+1} of every step, traces [nt][nrec] FP32.
 * Returns 0, or -1 for bad arguments, -2 when out of memory.
 */
int oracle16_run(int nx, int ny, int nz, double dx, double dy, double dz, int sponge_width,
                 double sponge_alpha, int form, const float *k32, int nt, const float *s, int src_z,
                 int src_y, int src_x, int nrec, const int32_t *rec, uint16_t *u_bits, uint16_t *d_bits,
                 int32_t *exps, float *traces)
{
    if (nx < 1 || ny < 1 || nz < 1 || nt < 0 || nrec < 0 || !k32 || form < ORACLE16_F16 ||
        form > ORACLE16_BF16_UV || !u_bits || (nrec > 0 && (!rec || !traces)) || (nt > 0 && !exps))
        return -1;
    const int bf = form == ORACLE16_BF16 || form == ORACLE16_BF16_UV;
    const int uv = form == ORACLE16_F16_UV || form == ORACLE16_BF16_UV;
    if (uv && !d_bits)
        return -1;
    const int G = 4, nxp = nx + 2 * G, nyp = ny + 2 * G, nzp = nz + 2 * G;
    const size_t np = (size_t)nxp * nyp * nzp;
    uint16_t *cur = calloc(np, 2), *sec = calloc(np, 2), *nxt = calloc(np, 2), *nd = calloc(np, 2),
             *kq = calloc(np, 2);
    float *gx = malloc(sizeof(float) * nx), *gy = malloc(sizeof(float) * ny), *gz = malloc(sizeof(float) * nz);
    /* u^n decoded (decoding is exact, so reading it equals decoding each read) */
    float *curf = malloc(sizeof(float) * np);
    if (!cur || !sec || !nxt || !nd || !kq || !gx || !gy || !gz || !curf) {
        free(cur); free(sec); free(nxt); free(nd); free(kq); free(gx); free(gy); free(gz); free(curf);
        return -2;
    }
#define PI(z, y, x) (((size_t)((z) + G) * nyp + (size_t)((y) + G)) * nxp + (size_t)((x) + G))
    /* k: one exponent for the whole field */
    float kmax = 0.0f;
    for (size_t i = 0; i < (size_t)nx * ny * nz; ++i)
        if (k32[i] > kmax)
            kmax = k32[i];
    int ek = 0;
    if (kmax > 0.0f) {
        int ex;
        (void)frexpf(kmax, &ex);
        ek = ex - 14;
    }
    const float k_down = ldexpf(1.0f, -ek), k_scale = ldexpf(1.0f, ek);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                kq[PI(z, y, x)] = enc16(bf, k32[((size_t)z * ny + y) * nx + x] * k_down);

    double c[5];
    exact_weights(c);
    const double ih2[3] = {1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz)};
    const float w0 = (float)(c[0] * (ih2[0] + ih2[1] + ih2[2]));
    float wx[5], wy[5], wz[5];
    for (int m = 1; m <= 4; ++m) {
        wx[m] = (float)(c[m] * ih2[0]);
        wy[m] = (float)(c[m] * ih2[1]);
        wz[m] = (float)(c[m] * ih2[2]);
    }
    sponge_f32(nx, sponge_width, sponge_alpha, gx);
    sponge_f32(ny, sponge_width, sponge_alpha, gy);
    sponge_f32(nz, sponge_width, sponge_alpha, gz);

    /* level exponents and maxima: e_n, e_{n-1}, M_n, M_{n-1} */
    int e_cur = 0, e_prev = 0;
    float m_cur = 0.0f, m_prev = 0.0f;
    for (int n = 0; n < nt; ++n) {
        const float sv = (s && src_z >= 0) ? s[n] : 0.0f;
        const float bound = 8.0f * fmaxf(m_cur, m_prev) + fabsf(sv);
        const int e = level_exponent(bound);
        const float out_inv = ldexpf(1.0f, -e), out_sc = ldexpf(1.0f, e);
        const float A = ldexpf(1.0f, e_cur) * out_inv;
        const float B = (uv ? ldexpf(1.0f, e_cur + 1) : ldexpf(1.0f, e_prev)) * out_inv;
        const float C = k_scale * A;
        const float v0 = w0 * C;
        float vx[5], vy[5], vz[5];
        for (int m = 1; m <= 4; ++m) {
            vx[m] = wx[m] * C;
            vy[m] = wy[m] * C;
            vz[m] = wz[m] * C;
        }
        const float two_a = 2.0f * A;
        const float sval = sv * out_inv;
        for (size_t i = 0; i < np; ++i)
            curf[i] = dec16(bf, cur[i]);
        float m_new = 0.0f;
        /* cells are independent within a step; a maximum does not depend on
         * the order it is taken in */
#pragma omp parallel for reduction(max : m_new) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t p = PI(z, y, x);
                    const float U = curf[p];
                    float lap = v0 * U;
                    for (int m = 1; m <= 4; ++m) {
                        const size_t sy = (size_t)m * nxp, sz = (size_t)m * nxp * nyp;
                        lap = fmaf(vx[m], curf[p + m] + curf[p - m], lap);
                        lap = fmaf(vy[m], curf[p + sy] + curf[p - sy], lap);
                        lap = fmaf(vz[m], curf[p + sz] + curf[p - sz], lap);
                    }
                    const float K = dec16(bf, kq[p]);
                    const float P = dec16(bf, sec[p]);
                    const float g = (gx[x] * gy[y]) * gz[z];
                    float t = fmaf(K, lap, two_a * U);
                    const float pe = uv ? fmaf(-B, P, A * U) : B * P;
                    t = fmaf(-g, pe, t);
                    float out = g * t;
                    if (z == src_z && y == src_y && x == src_x)
                        out = out + sval;
                    nxt[p] = enc16(bf, out);
                    if (uv)
                        nd[p] = enc16(bf, 0.5f * (out - A * U));
                    m_new = fmaxf(m_new, fabsf(out));
                }
        /* roles: the new level becomes u^{n+1}; the second field becomes
         * u^n (two levels) or d^{n+1} (u and change) */
        uint16_t *t16 = sec;
        if (uv) {
            sec = nd;
            nd = t16;
        } else {
            sec = cur;
            cur = t16;
        }
        t16 = cur;
        cur = nxt;
        nxt = t16;
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = &rec[3 * r];
            traces[(size_t)n * nrec + r] = dec16(bf, cur[PI(q[0], q[1], q[2])]) * out_sc;
        }
        exps[n] = e;
        e_prev = e_cur;
        e_cur = e;
        m_prev = m_cur;
        m_cur = m_new * out_sc;
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                u_bits[((size_t)z * ny + y) * nx + x] = cur[PI(z, y, x)];
                if (uv)
                    d_bits[((size_t)z * ny + y) * nx + x] = sec[PI(z, y, x)];
            }
#undef PI
    free(cur); free(sec); free(nxt); free(nd); free(kq); free(gx); free(gy); free(gz); free(curf);
    return 0;
}
