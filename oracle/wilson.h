/*
 * wilson -- FP64 CPU reference of the Wilson-action SU(3) configuration
 * generator (heatbath + overrelaxation) that produces the importance-sampled
 * ensembles the paper gauge-fixes (Sections 1 and 4; the paper does not
 * describe the generator, the algorithm is the standard one; definitions in
 * wilson.c).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke test
 * and the CPU-baseline leg of the benchmark; it shares no source with the
 * GPU library.  Conventions as lgfo.h (dims {Lx, Ly, Lz, Lt}, links
 * [s][mu][i][j][re,im]); every extent even.  Functions return 0, or -1 on an
 * invalid argument.
 */
#ifndef WILSONO_H
#define WILSONO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* attempts of the x0 sampler before a subgroup step is skipped */
#define WILSON_MAX_ATTEMPTS 1024

/* Philox4x64-10: out = the four 64-bit words for counter ctr and key. */
void wilsono_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* n draws of the x0 sampler for the density sqrt(1 - x0^2) exp(c x0), c >= 0
 * (Kennedy-Pendleton for c >= 1, plain rejection below), draw i with counter
 * words (i, 0, 0, attempt); draws that ran out of attempts are NaN and
 * counted in *failed. */
int wilsono_x0_sample(double c, uint64_t seed, long n, double *out, long *failed);

/* The staple A_mu(x) of link (site, mu) into out (18 doubles). */
int wilsono_staple(const int *dims, const double *U, long site, int mu, double *out);

/* sum over all links of Re Tr(U_mu(x) A_mu(x)) (= 4 times the sum of Re Tr
 * over all plaquettes); NaN on an invalid argument. */
double wilsono_link_action_sum(const int *dims, const double *U);

/* One link update in place: kind 0 heatbath with heatbath-sweep index
 * `sweep`, kind 1 overrelaxation; *skipped = subgroup steps skipped. */
int wilsono_link_update(const int *dims, double *U, long site, int mu, double beta, uint64_t seed, uint64_t sweep,
                        int kind, long *skipped);

/* One sweep in place (kind 0 heatbath numbered `sweep`, kind 1 overrelaxation). */
int wilsono_sweep(const int *dims, double *U, double beta, uint64_t seed, uint64_t sweep, int kind, long *skipped);

/* All links 1 (cold start). */
int wilsono_cold(const int *dims, double *U);

/* n_update times: one heatbath sweep (numbered first_sweep, first_sweep + 1,
 * ...) then n_or overrelaxation sweeps. */
int wilsono_generate(const int *dims, double *U, double beta, uint64_t seed, uint64_t first_sweep, long n_update,
                     int n_or, long *skipped);

#ifdef __cplusplus
}
#endif

#endif
