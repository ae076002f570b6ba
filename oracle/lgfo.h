/*
 * lgfo -- FP64 CPU oracle for Fourier-accelerated steepest-descent Landau
 * gauge fixing (Cardoso, Silva, Bicudo, Oliveira, "Landau Gauge Fixing on
 * GPUs", arXiv:1206.0675).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent checker for the
 * GPU library: only the test suite, the package smoke test and the CPU
 * baseline leg of the benchmark may load it.  It shares no source with the
 * GPU path.  It is plain, slow and written to be read against the paper:
 * each function names the equation or algorithm step it follows.
 *
 * Conventions
 *   dims        int[4] = {Lx, Ly, Lz, Lt}; every extent a power of two >= 2.
 *   site index  s = ((t*Lz + z)*Ly + y)*Lx + x  (x fastest, Section 3.1-3.2).
 *   links       canonical FP64: 72 doubles per site,
 *               [s][mu][i][j][re,im], mu = 0..3 for x, y, z, t.
 *   matrix      18 doubles, row-major 3x3 complex [i][j][re,im].
 *   fields      "per-site matrix fields" (Delta, g, G) are 18 doubles/site.
 *   Periodic boundary conditions in all four directions.
 *   Reductions are summed serially in site order, so results do not depend
 *   on the OpenMP thread count.
 *
 * Every function returns 0 on success and -1 on an invalid argument.
 */
#ifndef LGFO_H
#define LGFO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double alpha;        /* step size of the update (Section 2: 0.08)            */
    double theta_stop;   /* stop when theta < theta_stop (Section 2: 1e-15)      */
    long   max_iter;     /* give up after this many gauge transformations       */
    int    accel;        /* 1: Fourier acceleration p2max/p2 (eq. gx);
                            0: plain steepest descent (the same update, K = 1)  */
    int    store12;      /* 1: links kept as their first two rows, the third
                            rebuilt as (a x b)^* whenever read (Section 3.2)    */
    const double *band_scale; /* NULL, or 16 per-band factors s_b multiplying
                                 the acceleration kernel (learned step)         */
    int    expo;         /* 0: g = reunit(1 + alpha/2 dtilde), first order in
                            alpha then projected to SU(3) (Section 2);
                            1: g = exp(alpha/2 dtilde) exactly (eq. gx as
                            written, without the first-order expansion)        */
} lgfo_opts;

/* Fill opts with the paper's settings: alpha 0.08, theta_stop 1e-15, accel 1. */
void lgfo_default_opts(lgfo_opts *o);

/* Delta(x), F and theta of the current links (Section 2, eqs. for F_U[g],
 * theta and Delta).  delta: 18 doubles per site or NULL. */
int lgfo_measure(const int *dims, const double *U, double *delta, double *F, double *theta);

/* In-place 4D discrete Fourier transform of a complex field (2 doubles per
 * site, canonical site order), unnormalised, kernel exp(sign*i*p.x). */
int lgfo_fft4d(const int *dims, double *data, int sign);

/* The bracket of eq. gx applied to each matrix element of Delta separately
 * (Algorithm 1, inner loop): FFT forward, multiply by K(p), FFT backward,
 * divide by V.  K = p2max/p2 (K(0) = 0) if accel, else 1; times s_b(p) if
 * band_scale is given. */
int lgfo_filter(const lgfo_opts *o, const int *dims, const double *delta, double *out);

/* g(x) = reunit(1 + alpha/2 * dtilde(x)): eq. gx to first order in alpha,
 * then projected to SU(3) by row Gram-Schmidt with row 3 = (row1 x row2)^*. */
int lgfo_gauge(const int *dims, const double *dtilde, double alpha, double *g);

/* g(x) = exp(alpha/2 * dtilde(x)): eq. gx with the exponential evaluated
 * exactly (Taylor series of the 3x3 matrix after scaling by a power of two,
 * then repeated squaring). */
int lgfo_gauge_exp(const int *dims, const double *dtilde, double alpha, double *g);

/* exp(M) of n 3x3 complex matrices (18 doubles each), by the method of
 * lgfo_gauge_exp. */
int lgfo_expm(const double *m, long n, double *out);

/* U_mu(x) -> g(x) U_mu(x) g^dagger(x + mu) for all x, mu (Section 2). */
int lgfo_transform(const int *dims, const double *U, const double *g, double *out);

/* n iterations of Algorithm 1 without a stop test.  trace_F / trace_theta
 * (n+1 entries each, or NULL) receive F and theta before the first update
 * and after each one.  G (18 doubles per site, or NULL) is multiplied from
 * the left by each g, so U_n = G U_0 G^dagger(x+mu). */
int lgfo_step(const lgfo_opts *o, const int *dims, double *U, long n,
              double *trace_F, double *trace_theta, double *G);

/* Algorithm 1: iterate until theta < theta_stop or max_iter updates.
 * Returns 0 when converged, 1 when max_iter was reached. */
int lgfo_fix(const lgfo_opts *o, const int *dims, double *U, long *iters,
             double *F, double *theta, double *G);

/* Mean plaquette (1/(18V)) sum_x sum_{mu<nu} Re Tr U_mu(x) U_nu(x+mu)
 * U_mu^dag(x+nu) U_nu^dag(x): gauge invariant. */
double lgfo_plaquette(const int *dims, const double *U);

/* Replace the third row of each of n matrices by (row1 x row2)^* (eq. for
 * the 12-real parameterisation, Section 3.2). */
void lgfo_rebuild_row3(double *m, long n);

/* Largest |M M^dag - 1| element and |det M - 1| over n matrices. */
void lgfo_unitarity(const double *m, long n, double *max_unit, double *max_det);

/* Learned step: band index (0..15, or -1 for p = 0) of every momentum, and
 * band powers P_b = mean over the band of sum_c |Dhat_c(p)|^2 of the Fourier
 * transform of the 8 independent real components of Delta. */
int lgfo_band_index(const int *dims, int *band);
int lgfo_band_powers(const int *dims, const double *delta, double *power16, long *count16);

/* Number of OpenMP threads the oracle runs with. */
int lgfo_threads(void);

#ifdef __cplusplus
}
#endif
#endif
