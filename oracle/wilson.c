/*
 * wilson.c -- FP64 CPU reference of the Wilson-action SU(3) configuration
 * generator: Cabibbo-Marinari heatbath with Kennedy-Pendleton SU(2) sampling,
 * SU(2)-subgroup overrelaxation, checkerboard sweeps, Philox4x64-10 random
 * numbers.
 *
 * TEST INFRASTRUCTURE ONLY (see wilson.h).  The paper gauge-fixes ensembles
 * importance-sampled with the standard Wilson action (Sections 1 and 4) and
 * does not describe the generator; the algorithm below is the textbook one
 * (Cabibbo and Marinari 1982; Kennedy and Pendleton 1985; Creutz 1987 for
 * overrelaxation), written out here in plain loops.
 *
 * Definitions (the GPU generator implements the same ones, independently):
 *   action   S = beta sum_{x, mu<nu} (1 - Re Tr U_munu(x) / 3),
 *            U_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
 *   staple   A_mu(x) = sum over nu != mu, ascending, of
 *              [U_nu(x+mu) U_mu(x+nu)^dag] U_nu(x)^dag        (upper)
 *            + [U_nu(x+mu-nu)^dag U_mu(x-nu)^dag] U_nu(x-nu)  (lower),
 *            so the part of S that holds U_mu(x) is -(beta/3) Re Tr(U_mu(x) A_mu(x)).
 *   sweep    for mu = 0..3, for parity p = 0, 1 (parity of x+y+z+t): every
 *            link U_mu(x) with parity(x) = p.  Links of one (mu, p) class
 *            never appear in each other's staples, so their order is free.
 *   link     W = U A; for the subgroups (i, j) = (0,1), (1,2), (0,2) in turn:
 *            a = (Re w_ii + Re w_jj, Im w_ij + Im w_ji, Re w_ij - Re w_ji,
 *                 Im w_ii - Im w_jj), k = |a|; the SU(2) part of the 2x2
 *            block (i, j) of W is (k/2) Q(a/k), Q(q) = q0 + i q.sigma, and
 *            Re Tr(r w) = k Re Tr(r Q(a/k)) / 2 for r in SU(2).
 *              heatbath:       X = Q(x0, xv), x0 drawn from the density
 *                              sqrt(1 - x0^2) exp(c x0) with c = beta k / 3,
 *                              xv = sqrt(1 - x0^2) times a uniform direction;
 *                              r = X Q(a/k)^dag.
 *              overrelaxation: r = (Q(a/k)^dag)^2 (keeps Re Tr(r w), and is
 *                              its own inverse).
 *            then rows i, j of U and of W are multiplied by r (k = 0: the
 *            subgroup is left alone).  After the three subgroups U is
 *            projected to SU(3) by row Gram-Schmidt, row 3 = (row 1 x row 2)^*.
 *   random   Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), key
 *            (seed, 0).  Heatbath of link l = 4 s + mu in heatbath sweep n,
 *            subgroup k: counter (l, n, k, t) gives u1..u4 of attempt t,
 *            counter (l, n, k + 4, 0) gives u5, u6 of the direction.
 *            u = ((x >> 11) + 1) 2^-53 in (0, 1].
 *   x0       c >= 1, Kennedy-Pendleton: lambda^2 = -(ln u1 + cos^2(2 pi u2)
 *            ln u3) / (2 c); accept if u4^2 <= 1 - lambda^2; x0 = 1 - 2 lambda^2.
 *            c < 1 (where Kennedy-Pendleton accepts rarely), plain rejection:
 *            x0 = 2 u1 - 1, accept if u2 <= sqrt(1 - x0^2) exp(c (x0 - 1)).
 *            After WILSON_MAX_ATTEMPTS rejected attempts the subgroup step is
 *            skipped and counted.
 *   direction cos(theta) = 2 u5 - 1, phi = 2 pi u6.
 */
#include "wilson.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx e[3][3]; } m3;

/* ------------------------------------------------------------------ */
/* Philox4x64-10                                                       */
/* ------------------------------------------------------------------ */

void wilsono_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0, p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double unit(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }

static void uniforms(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, double u[4])
{
    const uint64_t ctr[4] = {c0, c1, c2, c3}, key[2] = {seed, 0};
    uint64_t x[4];
    wilsono_philox4x64(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = unit(x[i]);
}

/* x0 from sqrt(1 - x0^2) exp(c x0) on [-1, 1] (c >= 0); counter words (c0,
 * c1, c2, attempt).  Returns 0 and sets *x0, or -1 after WILSON_MAX_ATTEMPTS. */
static int sample_x0(double c, uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, double *x0)
{
    for (uint64_t t = 0; t < WILSON_MAX_ATTEMPTS; ++t) {
        double u[4];
        uniforms(seed, c0, c1, c2, t, u);
        if (c >= 1.0) {
            const double cs = cos(2.0 * M_PI * u[1]);
            const double l2 = -(log(u[0]) + cs * cs * log(u[2])) / (2.0 * c);
            if (u[3] * u[3] <= 1.0 - l2) {
                *x0 = 1.0 - 2.0 * l2;
                return 0;
            }
        } else {
            const double x = 2.0 * u[0] - 1.0;
            if (u[1] <= sqrt(1.0 - x * x) * exp(c * (x - 1.0))) {
                *x0 = x;
                return 0;
            }
        }
    }
    return -1;
}

int wilsono_x0_sample(double c, uint64_t seed, long n, double *out, long *failed)
{
    if (!(c >= 0.0) || n < 0 || !out) return -1;
    long f = 0;
    for (long i = 0; i < n; ++i) {
        double x = NAN;
        if (sample_x0(c, seed, (uint64_t)i, 0, 0, &x)) ++f;
        out[i] = x;
    }
    if (failed) *failed = f;
    return 0;
}

/* ------------------------------------------------------------------ */
/* lattice and matrices                                                */
/* ------------------------------------------------------------------ */

static int dims_ok(const int *d)
{
    if (!d) return 0;
    for (int m = 0; m < 4; ++m)
        if (d[m] < 2 || d[m] > 1024 || (d[m] & 1)) return 0;
    return 1;
}

static long volume(const int *d) { return (long)d[0] * d[1] * d[2] * d[3]; }

static long shift(const int *d, long s, int mu, int step)
{
    int c[4];
    long r = s;
    for (int m = 0; m < 4; ++m) { c[m] = (int)(r % d[m]); r /= d[m]; }
    c[mu] = (c[mu] + step + d[mu]) % d[mu];
    return (((long)c[3] * d[2] + c[2]) * d[1] + c[1]) * d[0] + c[0];
}

static int parity(const int *d, long s)
{
    int p = 0;
    for (int m = 0; m < 4; ++m) { p += (int)(s % d[m]); s /= d[m]; }
    return p & 1;
}

static m3 ld(const double *U, long s, int mu)
{
    const double *p = U + (s * 4 + mu) * 18;
    m3 m;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.e[i][j] = p[(3 * i + j) * 2] + I * p[(3 * i + j) * 2 + 1];
    return m;
}

static void st(double *U, long s, int mu, const m3 *m)
{
    double *p = U + (s * 4 + mu) * 18;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[(3 * i + j) * 2] = creal(m->e[i][j]);
            p[(3 * i + j) * 2 + 1] = cimag(m->e[i][j]);
        }
}

static m3 mm(const m3 *a, const m3 *b)
{
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a->e[i][k] * b->e[k][j];
            r.e[i][j] = s;
        }
    return r;
}

static m3 hc(const m3 *a)
{
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a->e[j][i]);
    return r;
}

static void project_su3(m3 *m)
{
    cplx *a = m->e[0], *b = m->e[1];
    double na = sqrt(creal(a[0] * conj(a[0]) + a[1] * conj(a[1]) + a[2] * conj(a[2])));
    for (int j = 0; j < 3; ++j) a[j] /= na;
    cplx ab = conj(a[0]) * b[0] + conj(a[1]) * b[1] + conj(a[2]) * b[2];
    for (int j = 0; j < 3; ++j) b[j] -= ab * a[j];
    double nb = sqrt(creal(b[0] * conj(b[0]) + b[1] * conj(b[1]) + b[2] * conj(b[2])));
    for (int j = 0; j < 3; ++j) b[j] /= nb;
    m->e[2][0] = conj(a[1] * b[2] - a[2] * b[1]);
    m->e[2][1] = conj(a[2] * b[0] - a[0] * b[2]);
    m->e[2][2] = conj(a[0] * b[1] - a[1] * b[0]);
}

/* the staple A_mu(x) of the definition above */
static m3 staple(const int *d, const double *U, long s, int mu)
{
    m3 A;
    memset(&A, 0, sizeof A);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const long xm = shift(d, s, mu, +1), xn = shift(d, s, nu, +1), xmn = shift(d, xm, nu, -1),
                   xdn = shift(d, s, nu, -1);
        m3 a = ld(U, xm, nu), b = ld(U, xn, mu), c = ld(U, s, nu);
        m3 bd = hc(&b), cd = hc(&c), ab = mm(&a, &bd), up = mm(&ab, &cd);
        m3 e = ld(U, xmn, nu), f = ld(U, xdn, mu), g = ld(U, xdn, nu);
        m3 ed = hc(&e), fd = hc(&f), ef = mm(&ed, &fd), dn = mm(&ef, &g);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A.e[i][j] += up.e[i][j] + dn.e[i][j];
    }
    return A;
}

int wilsono_staple(const int *dims, const double *U, long site, int mu, double *out)
{
    if (!dims_ok(dims) || !U || !out || mu < 0 || mu > 3 || site < 0 || site >= volume(dims)) return -1;
    m3 A = staple(dims, U, site, mu);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            out[(3 * i + j) * 2] = creal(A.e[i][j]);
            out[(3 * i + j) * 2 + 1] = cimag(A.e[i][j]);
        }
    return 0;
}

double wilsono_link_action_sum(const int *dims, const double *U)
{
    if (!dims_ok(dims) || !U) return NAN;
    const long V = volume(dims);
    double *part = malloc(sizeof(double) * V);
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            m3 u = ld(U, s, mu), A = staple(dims, U, s, mu), w = mm(&u, &A);
            acc += creal(w.e[0][0] + w.e[1][1] + w.e[2][2]);
        }
        part[s] = acc;
    }
    double sum = 0.0;
    for (long s = 0; s < V; ++s) sum += part[s];
    free(part);
    return sum;
}

/* ------------------------------------------------------------------ */
/* one link                                                            */
/* ------------------------------------------------------------------ */

/* quaternion product p q, for Q(p) Q(q) = Q(p q) */
static void qmul(const double p[4], const double q[4], double r[4])
{
    r[0] = p[0] * q[0] - (p[1] * q[1] + p[2] * q[2] + p[3] * q[3]);
    r[1] = p[0] * q[1] + q[0] * p[1] - (p[2] * q[3] - p[3] * q[2]);
    r[2] = p[0] * q[2] + q[0] * p[2] - (p[3] * q[1] - p[1] * q[3]);
    r[3] = p[0] * q[3] + q[0] * p[3] - (p[1] * q[2] - p[2] * q[1]);
}

/* rows i, j of m <- Q(r) (rows i, j of m) */
static void rotate_rows(m3 *m, int i, int j, const double r[4])
{
    const cplx r00 = r[0] + I * r[3], r01 = r[2] + I * r[1], r10 = -r[2] + I * r[1], r11 = r[0] - I * r[3];
    for (int c = 0; c < 3; ++c) {
        const cplx a = m->e[i][c], b = m->e[j][c];
        m->e[i][c] = r00 * a + r01 * b;
        m->e[j][c] = r10 * a + r11 * b;
    }
}

static const int SUB[3][2] = {{0, 1}, {1, 2}, {0, 2}};

/* heatbath (kind 0) or overrelaxation (kind 1) of link (s, mu); returns the
 * subgroup steps skipped after WILSON_MAX_ATTEMPTS */
static int update_link(const int *d, double *U, long s, int mu, double beta, uint64_t seed, uint64_t sweep,
                       int kind)
{
    m3 u = ld(U, s, mu), A = staple(d, U, s, mu), w = mm(&u, &A);
    int skipped = 0;
    const uint64_t l = (uint64_t)(s * 4 + mu);
    for (int k = 0; k < 3; ++k) {
        const int i = SUB[k][0], j = SUB[k][1];
        double a[4] = {creal(w.e[i][i]) + creal(w.e[j][j]), cimag(w.e[i][j]) + cimag(w.e[j][i]),
                       creal(w.e[i][j]) - creal(w.e[j][i]), cimag(w.e[i][i]) - cimag(w.e[j][j])};
        const double kn = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
        if (!(kn > 0.0)) continue;
        const double vd[4] = {a[0] / kn, -a[1] / kn, -a[2] / kn, -a[3] / kn};   /* Q(a/k)^dag */
        double r[4];
        if (kind == 0) {
            double x0;
            if (sample_x0(beta * kn / 3.0, seed, l, sweep, (uint64_t)k, &x0)) {
                ++skipped;
                continue;
            }
            double u6[4];
            uniforms(seed, l, sweep, (uint64_t)k + 4, 0, u6);
            const double ct = 2.0 * u6[0] - 1.0, st_ = sqrt(1.0 - ct * ct), ph = 2.0 * M_PI * u6[1];
            const double rad = sqrt(1.0 - x0 * x0);
            const double X[4] = {x0, rad * st_ * cos(ph), rad * st_ * sin(ph), rad * ct};
            qmul(X, vd, r);
        } else {
            qmul(vd, vd, r);
        }
        rotate_rows(&u, i, j, r);
        rotate_rows(&w, i, j, r);
    }
    project_su3(&u);
    st(U, s, mu, &u);
    return skipped;
}

int wilsono_link_update(const int *dims, double *U, long site, int mu, double beta, uint64_t seed, uint64_t sweep,
                        int kind, long *skipped)
{
    if (!dims_ok(dims) || !U || mu < 0 || mu > 3 || site < 0 || site >= volume(dims) || (kind != 0 && kind != 1))
        return -1;
    const int sk = update_link(dims, U, site, mu, beta, seed, sweep, kind);
    if (skipped) *skipped = sk;
    return 0;
}

/* ------------------------------------------------------------------ */
/* sweeps                                                              */
/* ------------------------------------------------------------------ */

int wilsono_sweep(const int *dims, double *U, double beta, uint64_t seed, uint64_t sweep, int kind, long *skipped)
{
    if (!dims_ok(dims) || !U || !(beta >= 0.0) || (kind != 0 && kind != 1)) return -1;
    const long V = volume(dims);
    long sk = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
#pragma omp parallel for schedule(static) reduction(+ : sk)
            for (long s = 0; s < V; ++s)
                if (parity(dims, s) == p) sk += update_link(dims, U, s, mu, beta, seed, sweep, kind);
        }
    if (skipped) *skipped = sk;
    return 0;
}

int wilsono_cold(const int *dims, double *U)
{
    if (!dims_ok(dims) || !U) return -1;
    const long n = volume(dims) * 4;
    memset(U, 0, sizeof(double) * 18 * (size_t)n);
    for (long l = 0; l < n; ++l)
        for (int i = 0; i < 3; ++i) U[l * 18 + (3 * i + i) * 2] = 1.0;
    return 0;
}

int wilsono_generate(const int *dims, double *U, double beta, uint64_t seed, uint64_t first_sweep, long n_update,
                     int n_or, long *skipped)
{
    if (!dims_ok(dims) || !U || !(beta >= 0.0) || n_update < 0 || n_or < 0) return -1;
    long total = 0;
    for (long n = 0; n < n_update; ++n) {
        long sk = 0;
        if (wilsono_sweep(dims, U, beta, seed, first_sweep + (uint64_t)n, 0, &sk)) return -1;
        total += sk;
        for (int o = 0; o < n_or; ++o)
            if (wilsono_sweep(dims, U, beta, seed, 0, 1, NULL)) return -1;
    }
    if (skipped) *skipped = total;
    return 0;
}
