/*
 * lgfo.c -- FP64 CPU oracle for Fourier-accelerated steepest-descent Landau
 * gauge fixing (arXiv:1206.0675, Section 2 and Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY: the independent checker of the GPU library.  It
 * shares no source with it.  Plain loops over sites, C99 complex arithmetic,
 * a textbook radix-2 FFT; OpenMP only splits site loops, and every sum over
 * sites runs serially in site order afterwards.
 *
 * Readings of points the paper leaves open (the same on the GPU side):
 *   - p^2 is the lattice Laplacian eigenvalue sum_mu 4 sin^2(pi n_mu / L_mu)
 *     (lattice spacing 1), so p2max = 16 for even extents; K(p=0) = 0.
 *   - "normalize" divides by the volume V once, after the backward FFT.
 *   - "trace" in Delta and in the exponent of eq. gx: subtract (1/3) Tr(.) 1
 *     after forming X - X^dagger.
 *   - the first-order update is 1 + alpha/2 * dtilde, reunitarised by row
 *     Gram-Schmidt with the third row (a x b)^*, the formula of the 12-real
 *     reconstruction.
 *   - theta = (1/(3V)) sum_x sum_ij |Delta_ij(x)|^2 and
 *     F = (1/(12V)) sum_x sum_mu Re Tr U_mu(x)  (N_c = 3, 4 directions).
 */
#include "lgfo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* lattice geometry                                                    */
/* ------------------------------------------------------------------ */

static int is_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

static int dims_ok(const int *d)
{
    if (!d) return 0;
    for (int m = 0; m < 4; ++m)
        if (!is_pow2(d[m]) || d[m] > 1024) return 0;
    return 1;
}

static long vol(const int *d) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords(const int *d, long s, int c[4])
{
    for (int m = 0; m < 4; ++m) { c[m] = (int)(s % d[m]); s /= d[m]; }
}

static long site_of(const int *d, const int c[4])
{
    return (((long)c[3] * d[2] + c[2]) * d[1] + c[1]) * d[0] + c[0];
}

/* site x + step * mu-hat, periodic */
static long neighbour(const int *d, long s, int mu, int step)
{
    int c[4];
    coords(d, s, c);
    c[mu] = (c[mu] + step + d[mu]) % d[mu];
    return site_of(d, c);
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices                                                */
/* ------------------------------------------------------------------ */

typedef struct { cplx e[3][3]; } mat;

static mat load(const double *p)
{
    mat m;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            m.e[i][j] = p[(3 * i + j) * 2] + I * p[(3 * i + j) * 2 + 1];
    return m;
}

static void store(double *p, const mat *m)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[(3 * i + j) * 2] = creal(m->e[i][j]);
            p[(3 * i + j) * 2 + 1] = cimag(m->e[i][j]);
        }
}

static mat mul(const mat *a, const mat *b)
{
    mat r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a->e[i][k] * b->e[k][j];
            r.e[i][j] = s;
        }
    return r;
}

static mat dag(const mat *a)
{
    mat r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a->e[j][i]);
    return r;
}

static void add_to(mat *a, const mat *b, double f)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a->e[i][j] += f * b->e[i][j];
}

static cplx trace(const mat *a) { return a->e[0][0] + a->e[1][1] + a->e[2][2]; }

/* third row = (first row x second row)^*  (12-real reconstruction) */
static void row3_from_rows12(mat *m)
{
    cplx *a = m->e[0], *b = m->e[1];
    m->e[2][0] = conj(a[1] * b[2] - a[2] * b[1]);
    m->e[2][1] = conj(a[2] * b[0] - a[0] * b[2]);
    m->e[2][2] = conj(a[0] * b[1] - a[1] * b[0]);
}

/* projection to SU(3): normalise row 1; make row 2 orthogonal to row 1 and
 * normalise it; row 3 = (row 1 x row 2)^*. */
static void reunitarise(mat *m)
{
    cplx *a = m->e[0], *b = m->e[1];
    double na = sqrt(creal(a[0] * conj(a[0]) + a[1] * conj(a[1]) + a[2] * conj(a[2])));
    for (int j = 0; j < 3; ++j) a[j] /= na;
    cplx ab = conj(a[0]) * b[0] + conj(a[1]) * b[1] + conj(a[2]) * b[2];
    for (int j = 0; j < 3; ++j) b[j] -= ab * a[j];
    double nb = sqrt(creal(b[0] * conj(b[0]) + b[1] * conj(b[1]) + b[2] * conj(b[2])));
    for (int j = 0; j < 3; ++j) b[j] /= nb;
    row3_from_rows12(m);
}

/* X - X^dagger - (1/3) Tr(X - X^dagger) 1: the anti-Hermitian traceless part
 * (times two) used in Delta and in the exponent of eq. gx. */
static mat antiherm_traceless(const mat *x)
{
    mat xd = dag(x), r = *x;
    add_to(&r, &xd, -1.0);
    cplx tr = trace(&r) / 3.0;
    for (int i = 0; i < 3; ++i) r.e[i][i] -= tr;
    return r;
}

static const double *link_at(const double *U, long s, int mu) { return U + (s * 4 + mu) * 18; }

/* ------------------------------------------------------------------ */
/* Delta, F, theta  (Section 2)                                       */
/* ------------------------------------------------------------------ */

int lgfo_measure(const int *dims, const double *U, double *delta, double *F, double *theta)
{
    if (!dims_ok(dims) || !U) return -1;
    long V = vol(dims);
    double *fs = malloc(sizeof(double) * V), *ts = malloc(sizeof(double) * V);
    if (!fs || !ts) { free(fs); free(ts); return -1; }

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        /* A(x) = sum_nu [U_nu(x - nu) - U_nu(x)]  (the backward difference) */
        mat A = {{{0}}};
        double fsum = 0.0;
        for (int nu = 0; nu < 4; ++nu) {
            mat u = load(link_at(U, s, nu));
            mat ub = load(link_at(U, neighbour(dims, s, nu, -1), nu));
            add_to(&A, &ub, 1.0);
            add_to(&A, &u, -1.0);
            fsum += creal(trace(&u));
        }
        mat D = antiherm_traceless(&A);
        double t = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) t += creal(D.e[i][j] * conj(D.e[i][j]));
        fs[s] = fsum;
        ts[s] = t;
        if (delta) store(delta + s * 18, &D);
    }
    double fsum = 0.0, tsum = 0.0;
    for (long s = 0; s < V; ++s) { fsum += fs[s]; tsum += ts[s]; }
    free(fs);
    free(ts);
    if (F) *F = fsum / (12.0 * (double)V);
    if (theta) *theta = tsum / (3.0 * (double)V);
    return 0;
}

/* ------------------------------------------------------------------ */
/* FFT: radix-2 Cooley-Tukey on each line, one axis after another      */
/* ------------------------------------------------------------------ */

/* In-place DFT of n (power of two) points: x_k <- sum_j x_j exp(sign*2 pi i jk/n). */
static void fft1d(cplx *x, int n, int sign)
{
    for (int i = 1, j = 0; i < n; ++i) {          /* bit-reversal permutation */
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {      /* butterflies */
        int half = len / 2;
        for (int k = 0; k < half; ++k) {
            double ang = sign * 2.0 * M_PI * k / len;
            cplx w = cos(ang) + I * sin(ang);
            for (int b = 0; b < n; b += len) {
                cplx u = x[b + k], v = x[b + k + half] * w;
                x[b + k] = u + v;
                x[b + k + half] = u - v;
            }
        }
    }
}

int lgfo_fft4d(const int *dims, double *data, int sign)
{
    if (!dims_ok(dims) || !data || (sign != 1 && sign != -1)) return -1;
    long V = vol(dims);
    cplx *f = (cplx *)data;
    long stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int n = dims[mu];
        long nlines = V / n;
#pragma omp parallel
        {
            cplx *line = malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
            for (long l = 0; l < nlines; ++l) {
                long lo = l % stride, hi = l / stride;
                long base = hi * stride * n + lo;
                for (int k = 0; k < n; ++k) line[k] = f[base + k * stride];
                fft1d(line, n, sign);
                for (int k = 0; k < n; ++k) f[base + k * stride] = line[k];
            }
            free(line);
        }
        stride *= n;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Fourier acceleration (eq. gx, Algorithm 1 inner loop)               */
/* ------------------------------------------------------------------ */

static double phat2(const int *dims, long s)
{
    int c[4];
    coords(dims, s, c);
    double p2 = 0.0;
    for (int m = 0; m < 4; ++m) {
        double sn = sin(M_PI * c[m] / dims[m]);
        p2 += 4.0 * sn * sn;
    }
    return p2;
}

static double phat2_max(const int *dims)
{
    double p2 = 0.0;
    for (int m = 0; m < 4; ++m) {
        double best = 0.0;
        for (int n = 0; n < dims[m]; ++n) {
            double sn = sin(M_PI * n / dims[m]);
            if (4.0 * sn * sn > best) best = 4.0 * sn * sn;
        }
        p2 += best;
    }
    return p2;
}

static double phat2_min_nonzero(const int *dims)
{
    double best = 1e300;
    for (int m = 0; m < 4; ++m) {
        double sn = sin(M_PI / dims[m]);
        if (4.0 * sn * sn < best) best = 4.0 * sn * sn;
    }
    return best;
}

int lgfo_band_index(const int *dims, int *band)
{
    if (!dims_ok(dims) || !band) return -1;
    long V = vol(dims);
    double pmin = phat2_min_nonzero(dims), pmax = phat2_max(dims);
    for (long s = 0; s < V; ++s) {
        double p2 = phat2(dims, s);
        if (s == 0) { band[s] = -1; continue; }
        int b = (int)floor(16.0 * log(p2 / pmin) / log(pmax / pmin));
        band[s] = b < 0 ? 0 : (b > 15 ? 15 : b);
    }
    return 0;
}

void lgfo_default_opts(lgfo_opts *o)
{
    o->alpha = 0.08;
    o->theta_stop = 1e-15;
    o->max_iter = 100000;
    o->accel = 1;
    o->store12 = 0;
    o->band_scale = NULL;
    o->expo = 0;
}

int lgfo_filter(const lgfo_opts *o, const int *dims, const double *delta, double *out)
{
    if (!o || !dims_ok(dims) || !delta || !out) return -1;
    long V = vol(dims);
    double p2max = phat2_max(dims);
    double *K = malloc(sizeof(double) * V);
    int *band = o->band_scale ? malloc(sizeof(int) * V) : NULL;
    cplx *f = malloc(sizeof(cplx) * V);
    if (!K || !f || (o->band_scale && !band)) { free(K); free(f); free(band); return -1; }
    if (band) lgfo_band_index(dims, band);
    for (long s = 0; s < V; ++s) {
        double p2 = phat2(dims, s);
        K[s] = o->accel ? (s == 0 ? 0.0 : p2max / p2) : 1.0;
        if (band && s != 0) K[s] *= o->band_scale[band[s]];
    }
    for (int e = 0; e < 9; ++e) {                 /* each element of the Delta matrix */
        for (long s = 0; s < V; ++s) f[s] = delta[s * 18 + 2 * e] + I * delta[s * 18 + 2 * e + 1];
        lgfo_fft4d(dims, (double *)f, -1);         /* FFT forward      */
        for (long s = 0; s < V; ++s) f[s] *= K[s]; /* apply p2max/p2   */
        lgfo_fft4d(dims, (double *)f, +1);         /* FFT backward     */
        for (long s = 0; s < V; ++s) {             /* normalise        */
            out[s * 18 + 2 * e] = creal(f[s]) / (double)V;
            out[s * 18 + 2 * e + 1] = cimag(f[s]) / (double)V;
        }
    }
    free(K);
    free(f);
    free(band);
    return 0;
}

int lgfo_band_powers(const int *dims, const double *delta, double *power16, long *count16)
{
    if (!dims_ok(dims) || !delta || !power16) return -1;
    long V = vol(dims);
    int *band = malloc(sizeof(int) * V);
    cplx *f = malloc(sizeof(cplx) * V);
    double *pw = calloc(V, sizeof(double));
    if (!band || !f || !pw) { free(band); free(f); free(pw); return -1; }
    lgfo_band_index(dims, band);
    /* the 8 real components of the anti-Hermitian traceless Delta as four
     * complex fields: Delta_01, Delta_02, Delta_12, Im Delta_00 + i Im Delta_11 */
    for (int c = 0; c < 4; ++c) {
        for (long s = 0; s < V; ++s) {
            const double *d = delta + s * 18;
            if (c == 0) f[s] = d[2] + I * d[3];
            else if (c == 1) f[s] = d[4] + I * d[5];
            else if (c == 2) f[s] = d[10] + I * d[11];
            else f[s] = d[1] + I * d[9];
        }
        lgfo_fft4d(dims, (double *)f, -1);
        for (long s = 0; s < V; ++s) pw[s] += creal(f[s] * conj(f[s]));
    }
    long cnt[16] = {0};
    double sum[16] = {0};
    for (long s = 0; s < V; ++s)
        if (band[s] >= 0) { sum[band[s]] += pw[s]; cnt[band[s]]++; }
    for (int b = 0; b < 16; ++b) {
        power16[b] = cnt[b] ? sum[b] / (double)cnt[b] : 0.0;
        if (count16) count16[b] = cnt[b];
    }
    free(band);
    free(f);
    free(pw);
    return 0;
}

/* ------------------------------------------------------------------ */
/* g(x) and the gauge transformation                                   */
/* ------------------------------------------------------------------ */

int lgfo_gauge(const int *dims, const double *dtilde, double alpha, double *g)
{
    if (!dims_ok(dims) || !dtilde || !g) return -1;
    long V = vol(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        mat d = load(dtilde + s * 18), m;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) m.e[i][j] = (i == j ? 1.0 : 0.0) + 0.5 * alpha * d.e[i][j];
        reunitarise(&m);
        store(g + s * 18, &m);
    }
    return 0;
}

/* exp(X) of a 3x3 complex matrix: halve X until its Frobenius norm is at
 * most 1/2, sum the Taylor series until a term is below 1e-18 of the sum (at
 * most 40 terms), then square the result once per halving. */
static mat expm3(const mat *x)
{
    double nrm = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nrm += creal(x->e[i][j] * conj(x->e[i][j]));
    nrm = sqrt(nrm);
    int halvings = 0;
    double scale = 1.0;
    while (nrm * scale > 0.5) {
        scale *= 0.5;
        ++halvings;
    }
    mat a = *x, sum, term;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a.e[i][j] *= scale;
            sum.e[i][j] = term.e[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int n = 1; n <= 40; ++n) {
        term = mul(&term, &a);
        double tn = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                term.e[i][j] /= (double)n;
                tn += creal(term.e[i][j] * conj(term.e[i][j]));
            }
        add_to(&sum, &term, 1.0);
        if (sqrt(tn) < 1e-18) break;
    }
    for (int k = 0; k < halvings; ++k) sum = mul(&sum, &sum);
    return sum;
}

int lgfo_expm(const double *m, long n, double *out)
{
    if (!m || !out || n < 0) return -1;
    for (long k = 0; k < n; ++k) {
        mat a = load(m + k * 18), e = expm3(&a);
        store(out + k * 18, &e);
    }
    return 0;
}

int lgfo_gauge_exp(const int *dims, const double *dtilde, double alpha, double *g)
{
    if (!dims_ok(dims) || !dtilde || !g) return -1;
    long V = vol(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        mat d = load(dtilde + s * 18);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) d.e[i][j] *= 0.5 * alpha;
        mat e = expm3(&d);
        store(g + s * 18, &e);
    }
    return 0;
}

int lgfo_transform(const int *dims, const double *U, const double *g, double *out)
{
    if (!dims_ok(dims) || !U || !g || !out || U == out) return -1;
    long V = vol(dims);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        mat gx = load(g + s * 18);
        for (int mu = 0; mu < 4; ++mu) {
            mat u = load(link_at(U, s, mu));
            mat gn = load(g + neighbour(dims, s, mu, +1) * 18);
            mat gnd = dag(&gn);
            mat t = mul(&gx, &u);
            mat r = mul(&t, &gnd);
            store(out + (s * 4 + mu) * 18, &r);
        }
    }
    return 0;
}

void lgfo_rebuild_row3(double *m, long n)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        mat a = load(m + k * 18);
        row3_from_rows12(&a);
        store(m + k * 18, &a);
    }
}

void lgfo_unitarity(const double *m, long n, double *max_unit, double *max_det)
{
    double mu = 0.0, md = 0.0;
    for (long k = 0; k < n; ++k) {
        mat a = load(m + k * 18), ad = dag(&a), p = mul(&a, &ad);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double e = cabs(p.e[i][j] - (i == j ? 1.0 : 0.0));
                if (e > mu || isnan(e)) mu = e;
            }
        cplx det = a.e[0][0] * (a.e[1][1] * a.e[2][2] - a.e[1][2] * a.e[2][1])
                 - a.e[0][1] * (a.e[1][0] * a.e[2][2] - a.e[1][2] * a.e[2][0])
                 + a.e[0][2] * (a.e[1][0] * a.e[2][1] - a.e[1][1] * a.e[2][0]);
        double e = cabs(det - 1.0);
        if (e > md || isnan(e)) md = e;
    }
    if (max_unit) *max_unit = mu;
    if (max_det) *max_det = md;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
    double *delta, *dtilde, *g, *Unew, *Gnew;
} work;

static int work_alloc(work *w, long V, int need_G)
{
    w->delta = malloc(sizeof(double) * 18 * V);
    w->dtilde = malloc(sizeof(double) * 18 * V);
    w->g = malloc(sizeof(double) * 18 * V);
    w->Unew = malloc(sizeof(double) * 72 * V);
    w->Gnew = need_G ? malloc(sizeof(double) * 18 * V) : NULL;
    return w->delta && w->dtilde && w->g && w->Unew && (!need_G || w->Gnew);
}

static void work_free(work *w)
{
    free(w->delta); free(w->dtilde); free(w->g); free(w->Unew); free(w->Gnew);
}

/* One gauge transformation of Algorithm 1 given the current Delta:
 * filter, g, U -> g U g^dag(x+mu); G -> g G (reunitarised). */
static void update(const lgfo_opts *o, const int *dims, double *U, double *G, work *w)
{
    long V = vol(dims);
    lgfo_filter(o, dims, w->delta, w->dtilde);
    if (o->expo) lgfo_gauge_exp(dims, w->dtilde, o->alpha, w->g);
    else lgfo_gauge(dims, w->dtilde, o->alpha, w->g);
    lgfo_transform(dims, U, w->g, w->Unew);
    memcpy(U, w->Unew, sizeof(double) * 72 * V);
    if (o->store12) lgfo_rebuild_row3(U, 4 * V);
    if (G) {
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; ++s) {
            mat a = load(w->g + s * 18), b = load(G + s * 18), c = mul(&a, &b);
            reunitarise(&c);
            store(w->Gnew + s * 18, &c);
        }
        memcpy(G, w->Gnew, sizeof(double) * 18 * V);
    }
}

int lgfo_step(const lgfo_opts *o, const int *dims, double *U, long n,
              double *trace_F, double *trace_theta, double *G)
{
    if (!o || !dims_ok(dims) || !U || n < 0) return -1;
    long V = vol(dims);
    work w;
    if (!work_alloc(&w, V, G != NULL)) { work_free(&w); return -1; }
    if (o->store12) lgfo_rebuild_row3(U, 4 * V);
    double F, th;
    lgfo_measure(dims, U, w.delta, &F, &th);
    if (trace_F) trace_F[0] = F;
    if (trace_theta) trace_theta[0] = th;
    for (long k = 1; k <= n; ++k) {
        update(o, dims, U, G, &w);
        lgfo_measure(dims, U, w.delta, &F, &th);
        if (trace_F) trace_F[k] = F;
        if (trace_theta) trace_theta[k] = th;
    }
    work_free(&w);
    return 0;
}

int lgfo_fix(const lgfo_opts *o, const int *dims, double *U, long *iters,
             double *F, double *theta, double *G)
{
    if (!o || !dims_ok(dims) || !U) return -1;
    long V = vol(dims);
    work w;
    if (!work_alloc(&w, V, G != NULL)) { work_free(&w); return -1; }
    if (o->store12) lgfo_rebuild_row3(U, 4 * V);
    double f, th;
    long it = 0;
    lgfo_measure(dims, U, w.delta, &f, &th);
    while (!(th < o->theta_stop) && it < o->max_iter) {   /* while theta >= eps */
        update(o, dims, U, G, &w);
        ++it;
        lgfo_measure(dims, U, w.delta, &f, &th);
    }
    work_free(&w);
    if (iters) *iters = it;
    if (F) *F = f;
    if (theta) *theta = th;
    return th < o->theta_stop ? 0 : 1;
}

/* ------------------------------------------------------------------ */
/* plaquette                                                           */
/* ------------------------------------------------------------------ */

double lgfo_plaquette(const int *dims, const double *U)
{
    if (!dims_ok(dims) || !U) return NAN;
    long V = vol(dims);
    double *ps = malloc(sizeof(double) * V);
    if (!ps) return NAN;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        double acc = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                mat a = load(link_at(U, s, mu));
                mat b = load(link_at(U, neighbour(dims, s, mu, +1), nu));
                mat c = load(link_at(U, neighbour(dims, s, nu, +1), mu));
                mat d = load(link_at(U, s, nu));
                mat cd = dag(&c), dd = dag(&d);
                mat ab = mul(&a, &b), abc = mul(&ab, &cd), p = mul(&abc, &dd);
                acc += creal(trace(&p));
            }
        ps[s] = acc;
    }
    double sum = 0.0;
    for (long s = 0; s < V; ++s) sum += ps[s];
    free(ps);
    return sum / (18.0 * (double)V);
}

int lgfo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
