/*
 * lgf_wilson.h -- C ABI of the MI355X (gfx950) generator of Wilson-action
 * SU(3) gauge configurations: the importance-sampled ensembles that Landau
 * gauge fixing is applied to (arXiv:1206.0675, Sections 1 and 4: pure-gauge
 * configurations of the standard Wilson action at beta = 5.8, 6.0, 6.2).
 * The paper does not describe its generator; this one is the standard
 * Cabibbo-Marinari heatbath with Kennedy-Pendleton SU(2) sampling plus
 * SU(2)-subgroup overrelaxation.
 *
 * Definitions
 *   action   S = beta sum_{x, mu<nu} (1 - Re Tr U_munu(x) / 3).
 *   staple   A_mu(x) = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 *                      + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu),
 *            the link's share of S being -(beta/3) Re Tr(U_mu(x) A_mu(x)).
 *   sweep    for mu = 0..3, for parity p = 0, 1 of x+y+z+t, every link
 *            U_mu(x) with parity(x) = p (one launch per class: no link of a
 *            class appears in the staple of another).
 *   link     W = U A; for the SU(2) subgroups (0,1), (1,2), (0,2) in turn:
 *            a = (Re w_ii + Re w_jj, Im w_ij + Im w_ji, Re w_ij - Re w_ji,
 *            Im w_ii - Im w_jj), k = |a|, V = Q(a/k) with Q(q) = q0 + i q.sigma;
 *              heatbath        r = X V^dag, X = Q(x0, sqrt(1-x0^2) n), n a
 *                              uniform direction, x0 from the density
 *                              sqrt(1 - x0^2) exp(c x0), c = beta k / 3
 *                              (Kennedy-Pendleton for c >= 1, plain rejection
 *                              below);
 *              overrelaxation  r = (V^dag)^2, which keeps the action exactly;
 *            rows i, j of U and W are multiplied by r; afterwards U is
 *            projected to SU(3) (row Gram-Schmidt, row 3 = (row1 x row2)^*).
 *   random   Philox4x64-10, key (seed, 0); the heatbath of link
 *            l = 4 site + mu in heatbath sweep n, subgroup k, attempt t reads
 *            counter (l, n, k, t) (four uniforms), its direction counter
 *            (l, n, k + 4, 0); u = ((x >> 11) + 1) 2^-53.  At most
 *            LGF_WILSON_MAX_ATTEMPTS attempts; a subgroup step that runs out
 *            is skipped and counted (lgf_wilson_skipped).
 *   A generator's results depend only on (dims, beta, seed, start links and
 *   the sequence of calls), not on the launch shape.
 *
 * Conventions as lgf.h: return LGF_OK or a negative LGF_E_* code; the
 * canonical FP64 link layout; `where` is LGF_HOST or LGF_DEVICE.  Extents
 * must be even, in [2, 1024], with at most 2^31 sites (else
 * LGF_E_UNSUPPORTED_SHAPE).  The generator owns its device memory (the
 * links twice: 576 bytes per site in the canonical layout, 384 in the sweeps'
 * two-row layout) and its stream; every call below
 * returns with its device work finished.
 */
#ifndef LGF_WILSON_H
#define LGF_WILSON_H

#include "lgf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LGF_WILSON_MAX_ATTEMPTS 1024
#define LGF_WILSON_HEATBATH 0
#define LGF_WILSON_OVERRELAX 1

typedef struct lgf_wilson_gen *lgf_wilson_t;

/* A generator for links of shape dims at coupling beta >= 0 with Philox key
 * seed; links start cold (all 1), the heatbath sweep counter at 0. */
int32_t lgf_wilson_create(const int32_t dims[4], double beta, uint64_t seed, lgf_wilson_t *out);
int32_t lgf_wilson_destroy(lgf_wilson_t g);

/* All links 1 and the heatbath sweep counter 0. */
int32_t lgf_wilson_cold(lgf_wilson_t g);

/* Replace the links (canonical layout, copied; not checked for unitarity).
 * The sweeps and the plaquette keep rows 0 and 1 of each link and rebuild
 * row 2 as the complex conjugate of their cross product, which for SU(3)
 * links is the same matrix up to rounding; until the next sweep or cold
 * start, lgf_wilson_store and lgf_wilson_device_links return the loaded
 * links as they were given. */
int32_t lgf_wilson_load(lgf_wilson_t g, const void *links, int32_t where);

/* One sweep: LGF_WILSON_HEATBATH (numbered by the sweep counter, which then
 * grows by one) or LGF_WILSON_OVERRELAX (draws no random numbers). */
int32_t lgf_wilson_sweep(lgf_wilson_t g, int32_t kind);

/* n_update times: one heatbath sweep, then n_or overrelaxation sweeps. */
int32_t lgf_wilson_update(lgf_wilson_t g, int64_t n_update, int32_t n_or);

/* The heatbath sweep counter (the number the next heatbath sweep reads). */
int32_t lgf_wilson_get_sweep(lgf_wilson_t g, uint64_t *n);
int32_t lgf_wilson_set_sweep(lgf_wilson_t g, uint64_t n);

/* <P> = sum_{x, mu<nu} Re Tr U_munu(x) / (18 V), summed in a fixed order. */
int32_t lgf_wilson_plaquette(lgf_wilson_t g, double *plaq);

/* Copy the links out (canonical layout). */
int32_t lgf_wilson_store(lgf_wilson_t g, void *links, int32_t where);

/* Device address of the links in the canonical layout, valid until the
 * generator is destroyed; e.g. for lgf_load_links(ctx, p, LGF_DEVICE).
 * The sweeps work on a second, even-odd copy of the links; this call first
 * rewrites the canonical copy from it when a sweep or cold start has changed
 * the links since (one device pass, then a stream synchronisation), so the
 * buffer holds the current links when the call returns and until the next
 * sweep, update or cold start.  Returns NULL on a device error (message in
 * lgf_wilson_last_error). */
const void *lgf_wilson_device_links(lgf_wilson_t g);

/* Subgroup steps skipped since creation (sampler out of attempts). */
int32_t lgf_wilson_skipped(lgf_wilson_t g, int64_t *n);

const char *lgf_wilson_last_error(lgf_wilson_t g);

#ifdef __cplusplus
}
#endif

#endif
