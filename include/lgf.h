/*
 * lgf.h -- C ABI of the MI355X (gfx950) library for Landau gauge fixing of
 * SU(3) lattice gauge fields by Fourier-accelerated steepest descent
 * (N. Cardoso, P. J. Silva, P. Bicudo, O. Oliveira, "Landau Gauge Fixing on
 * GPUs", Comput. Phys. Commun., arXiv:1206.0675).
 *
 * The method (Section 2 of the paper): maximise over the gauge orbit
 *     F_U[g] = 1/(4 N_c V) sum_x sum_mu Re Tr g(x) U_mu(x) g^dag(x + mu)
 * by iterating (Algorithm 1)
 *     Delta(x) = sum_nu [U_nu(x - nu) - U_nu(x) - h.c. - trace]
 *     g(x)     = exp[ FFT^-1 (alpha/2) (p2max/p2) FFT Delta ](x)     (eq. gx)
 *                (to first order in alpha, then projected to SU(3))
 *     U_mu(x) -> g(x) U_mu(x) g^dag(x + mu)
 * until theta = 1/(N_c V) sum_x Tr Delta(x) Delta^dag(x) < 1e-15.
 *
 * Conventions for every call
 *   - Return value: LGF_OK (0) or a negative LGF_E_* code.  No C++ exception
 *     crosses this boundary.  lgf_last_error() describes the last failure of
 *     a context; lgf_strerror() names a code.
 *   - The library never keeps a caller's pointer after a call returns: data
 *     is copied in and out.  A context owns all the device memory it uses.
 *   - Pointers tagged `where` are host memory (LGF_HOST) or device memory of
 *     the current HIP device (LGF_DEVICE, e.g. torch.Tensor.data_ptr()).
 *     Device pointers are used in stream order on the context's stream.
 *   - Canonical link layout (host or device): FP64, 72 doubles per site,
 *     double index ((((t*Lz + z)*Ly + y)*Lx + x)*4 + mu)*18 + (3*i + j)*2 + c,
 *     mu = 0..3 for x, y, z, t, c = 0 (real) / 1 (imaginary): x fastest, as
 *     the lexicographic (x, y, z, t) order of Section 3.  Per-site matrix
 *     fields (the gauge transformation G) use 18 doubles per site, same order.
 *   - Periodic boundary conditions in all four directions.
 *   - Shapes: each extent a power of two in [4, 128]; in addition the (x, y)
 *     plane and the (z, t) plane must fit the LDS of one workgroup
 *     (FP64: Lx*Ly <= 2048 and Lz*Lt <= 8192).  Otherwise
 *     LGF_E_UNSUPPORTED_SHAPE, returned before any device call.
 *   - A context is used by one host thread at a time; distinct contexts are
 *     independent.
 */
#ifndef LGF_H
#define LGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LGF_OK 0
#define LGF_E_INVALID_ARG (-1)       /* NULL pointer, bad enum, alpha <= 0, ...            */
#define LGF_E_UNSUPPORTED_SHAPE (-2) /* extent not a power of two in [4,128], plane too big */
#define LGF_E_OUT_OF_MEMORY (-3)     /* device allocation failed                            */
#define LGF_E_DEVICE (-4)            /* a HIP runtime call failed                           */
#define LGF_E_NOT_UNITARY (-5)       /* input link with |UU^dag-1| or |det U-1| > tolerance */
#define LGF_E_NONFINITE (-6)         /* NaN/Inf in the input, or theta became non-finite    */
#define LGF_E_NOT_CONVERGED (-7)     /* max_iter reached with theta >= theta_stop           */
#define LGF_E_STATE (-8)             /* call not valid now (e.g. step before load)          */
#define LGF_E_MODEL (-9)             /* learned-step model blob malformed (size or header)  */

/* where a caller's buffer lives */
#define LGF_HOST 0
#define LGF_DEVICE 1

/* arithmetic precision of the iteration */
#define LGF_FP64 0   /* every iteration in FP64                                          */
#define LGF_FP32 1   /* every iteration in FP32 (F, theta sums and g projection in FP64) */
#define LGF_MIXED 2  /* FP32 until theta < theta_switch, then the links are rebuilt in
                        FP64 as G U0 G^dag(x+mu) and FP64 iterations finish the run       */

/* link storage (Section 3.2): full matrix, or the first two rows with the
 * third rebuilt as (a x b)^* when read */
#define LGF_STORE18 18
#define LGF_STORE12 12

/* step kind */
#define LGF_STEP_PLAIN 0    /* eq. gx: (alpha/2) p2max/p2                                  */
#define LGF_STEP_LEARNED 1  /* s_b (alpha/2) p2max/p2 with per-band factors s_b from the
                               network set by lgf_set_model, applied to the band powers of
                               the previous update's spectrum (s = 1 for the first update
                               after a load); an update that neither increases F nor
                               lowers theta is replaced by the plain one (FP64 only)       */

/* how g(x) is formed from the filtered Delta (eq. gx) */
#define LGF_UPDATE_FIRST_ORDER 0  /* g = reunit(1 + (alpha/2) dtilde): first order in alpha, then
                                     projected to SU(3) (Section 2; the paper's choice)          */
#define LGF_UPDATE_EXP 1          /* g = exp((alpha/2) dtilde), the exponential of eq. gx taken
                                     exactly (Cayley-Hamilton form, FP64)                        */

/* acceleration kernel */
#define LGF_ACCEL_FOURIER 1  /* K(p) = p2max/p2, K(0) = 0 (eq. gx)                       */
#define LGF_ACCEL_NONE 0     /* K(p) = 1: plain steepest descent (the same update without
                                Fourier acceleration, Section 2)                          */

typedef struct lgf_params {
    int32_t dims[4];        /* Lx, Ly, Lz, Lt                                           */
    int32_t precision;      /* LGF_FP64 | LGF_FP32 | LGF_MIXED                           */
    int32_t storage;        /* LGF_STORE18 | LGF_STORE12                                 */
    int32_t step;           /* LGF_STEP_PLAIN                                            */
    int32_t accel;          /* LGF_ACCEL_FOURIER | LGF_ACCEL_NONE                        */
    int32_t update;         /* LGF_UPDATE_FIRST_ORDER | LGF_UPDATE_EXP                   */
    int32_t profile;        /* 1: time every kernel launch with HIP events               */
    double alpha;           /* step size, paper: 0.08                                    */
    double theta_stop;      /* stop when theta < theta_stop, paper: 1e-15                */
    double theta_switch;    /* LGF_MIXED: leave FP32 when theta < theta_switch (1e-6)    */
    double unit_tol;        /* lgf_load_links rejects links beyond this (1e-12); <= 0
                               skips the check                                           */
    int64_t max_iter;       /* lgf_fix gives up after this many gauge transformations    */
    int32_t poll_every;     /* lgf_fix reads theta back after this many iterations       */
    int32_t no_graph;       /* 1: lgf_fix launches kernel by kernel instead of replaying
                               a captured graph of poll_every iterations                 */
    void *stream;           /* hipStream_t to run on; NULL: the context creates its own */
    int32_t autotune;       /* 1: time the candidate launch shapes on this lattice at
                               create and keep the fastest (cached per shape in the file
                               named by $LGF_TUNE_CACHE, if set)                         */
    int32_t reserved;
} lgf_params;

typedef struct lgf_stats {
    int64_t iter;           /* gauge transformations applied since the last load         */
    int64_t iter_fp32;      /* ... of which in FP32                                      */
    int64_t iter_fp64;      /* ... of which in FP64                                      */
    int64_t fallbacks;      /* learned steps replaced by the plain step (neither F rose nor
                               theta fell) */
    double F;               /* functional of the current links                           */
    double theta;           /* convergence measure of the current links                  */
    double seconds;         /* wall time of the call                                     */
    int32_t phase;          /* 0: FP32 arithmetic, 1: FP64 arithmetic                    */
    int32_t status;         /* the call's return code                                    */
} lgf_stats;

typedef struct lgf_context *lgf_ctx;

/* Defaults: dims 0, LGF_FP64, LGF_STORE18, LGF_STEP_PLAIN, LGF_ACCEL_FOURIER,
 * alpha 0.08, theta_stop 1e-15 (Section 2), theta_switch 1e-6, unit_tol 1e-12,
 * max_iter 100000, poll_every 16, stream NULL.  Host only. */
int32_t lgf_default_params(lgf_params *p);

/* Check canonical FP64 links on the host, without a context or a GPU: every
 * entry finite, |U U^dag - 1|_max <= tol and |det U - 1| <= tol.  first_bad
 * (may be NULL) receives the index of the first failing link (site*4 + mu) or
 * -1.  Returns LGF_OK, LGF_E_NONFINITE or LGF_E_NOT_UNITARY. */
int32_t lgf_validate_links(const int32_t dims[4], const double *links, double tol, int64_t *first_bad);

/* Validate params (host only: LGF_E_INVALID_ARG / LGF_E_UNSUPPORTED_SHAPE),
 * then allocate the context's device buffers on the current device. */
int32_t lgf_create(const lgf_params *p, lgf_ctx *out);

/* Free everything; NULL is accepted. */
int32_t lgf_destroy(lgf_ctx ctx);

/* Copy in canonical FP64 links (where = LGF_HOST or LGF_DEVICE), check them
 * against unit_tol, lay them out on the device, reset G = 1 and the
 * iteration count.  On error the previous state is invalid (LGF_E_STATE
 * until the next successful load). */
int32_t lgf_load_links(lgf_ctx ctx, const void *links, int32_t where);

/* Copy the current links G(x) U0(x) G^dag(x+mu) out in canonical FP64
 * (formed on the device from the loaded links and the accumulated gauge). */
int32_t lgf_store_links(lgf_ctx ctx, void *links, int32_t where);

/* Accumulated gauge transformation G (18 doubles per site), such that the
 * current links are G(x) U0(x) G^dag(x+mu) for the loaded links U0.
 * lgf_load_gauge replaces G, so the links become G U0 G^dag(x+mu) for the
 * links last loaded: loading the same U0 and a stored G resumes a run bit
 * for bit (checkpoint = U0 + G).  G must be SU(3) to the precision in use. */
int32_t lgf_store_gauge(lgf_ctx ctx, void *G, int32_t where);
int32_t lgf_load_gauge(lgf_ctx ctx, const void *G, int32_t where);

/* F and theta of the current links (Section 2); no update. */
int32_t lgf_measure(lgf_ctx ctx, lgf_stats *out);

/* Exactly n iterations of Algorithm 1 with no stop test, in the current
 * precision phase.  trace (n + 1 entries, or NULL) receives F and theta of
 * the links before the first update and after each update. */
int32_t lgf_step(lgf_ctx ctx, int64_t n, lgf_stats *trace);

/* Algorithm 1: iterate until theta < theta_stop (LGF_OK) or max_iter
 * (LGF_E_NOT_CONVERGED).  theta is read back every poll_every iterations;
 * iterations queued after convergence do nothing.  In LGF_MIXED the FP32
 * phase ends at theta < theta_switch, or once theta has not halved for 512
 * iterations (read at the polls: FP32 rounding of the links stops theta,
 * near 1e-14 at 32^4, so a theta_switch below that still ends the phase),
 * and the run finishes in FP64.  lgf_fix_batch and lgf_batch_fix switch at
 * theta_switch only. */
int32_t lgf_fix(lgf_ctx ctx, lgf_stats *out);

/* ---------------------------------------------------------------------------
 * Batches: many configurations of different shapes gauge-fixed together
 * (each kernel launch of an iteration covers every configuration; iterations
 * are replayed from a captured graph; converged configurations are skipped;
 * LGF_MIXED switches each configuration to FP64 on its own).  The common
 * params apply to all members except dims; the accumulated gauge is always
 * tracked.
 * ------------------------------------------------------------------------- */
typedef struct lgf_batch *lgf_batch_t;

/* dims[i] = {Lx, Ly, Lz, Lt} of member i (each as for lgf_create). */
int32_t lgf_batch_create(const lgf_params *common, int32_t n, const int32_t (*dims)[4], lgf_batch_t *out);
int32_t lgf_batch_destroy(lgf_batch_t b);
/* Copy in member i's canonical FP64 links (validated as by lgf_load_links). */
int32_t lgf_batch_load(lgf_batch_t b, int32_t i, const void *links, int32_t where);
/* Iterate every loaded member to theta < theta_stop or max_iter.  out (n
 * entries, or NULL) receives each member's stats; seconds is the batch wall
 * time.  Returns LGF_OK if every member converged, else the worst status. */
int32_t lgf_batch_fix(lgf_batch_t b, lgf_stats *out);
int32_t lgf_batch_store(lgf_batch_t b, int32_t i, void *links, int32_t where);
int32_t lgf_batch_store_gauge(lgf_batch_t b, int32_t i, void *G, int32_t where);
/* The launch shape the batch runs with, after autotuning if requested:
 * threads per plane block, and the bytes of one row of a (z, t) tile of the
 * Delta layout (tile_bytes / sizeof(complex) plane positions per tile). */
int32_t lgf_batch_config(lgf_batch_t b, int32_t *plane_threads, int32_t *tile_bytes);
const char *lgf_batch_last_error(lgf_batch_t b);

/* One call: create, load host links_in[i], fix, store into links_out[i]
 * (which may alias links_in[i]), destroy.  Returns the worst member status. */
int32_t lgf_fix_batch(const lgf_params *common, int32_t n, const int32_t (*dims)[4], const double *const *links_in,
                      double *const *links_out, lgf_stats *out);

/* ---------------------------------------------------------------------------
 * Allocation-free one call, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It is lgf_create + lgf_load_links + lgf_fix + lgf_store_links
 * + lgf_destroy for one lattice whose links are in device memory, with the
 * same kernels and launch shape as a default context (so the same result
 * bits), but it calls no hipMalloc, hipFree or other allocating routine:
 * every buffer beyond links_in and links_out lives in one static device
 * array of lgf_noalloc_capacity() bytes (64 MiB: up to a 16^4 lattice with
 * 18-real links), which each device the library runs on holds until the
 * process ends.  Lattices that need more return LGF_E_UNSUPPORTED_SHAPE
 * before any device work.
 *   p          params as for lgf_create; precision must be LGF_FP64 and step
 *              LGF_STEP_PLAIN (else LGF_E_INVALID_ARG); p->stream is the
 *              stream used (NULL: the null stream); autotune, no_graph and
 *              profile are ignored (kernel-by-kernel launches, default
 *              launch shape).
 *   links_in   canonical FP64 links on the current device (read only).
 *   links_out  canonical FP64 links on the current device, written with the
 *              gauge-fixed links; may equal links_in.
 *   out        stats (or NULL), filled also for LGF_E_NOT_CONVERGED.
 * The call returns when the result is in links_out.  Every call on a device
 * shares that device's array: calls that overlap on one device race and are
 * not supported.  Errors: as lgf_create, lgf_load_links and lgf_fix; the
 * message is read with lgf_last_error(NULL). */
int32_t lgf_fix_noalloc(const lgf_params *p, const double *links_in, double *links_out, lgf_stats *out);
size_t lgf_noalloc_capacity(void);

/* ---------------------------------------------------------------------------
 * Learned spectral step.  The modes p != 0 fall in 16 bands log-spaced in p^2
 * between the smallest nonzero p^2 of the lattice and p2max.  Features:
 * x_b = log10(P_b / V) / 8 with P_b the mean over band b of sum_c |Dhat_c|^2
 * (the four complex fields of Delta's 8 real components; 0 for an empty
 * band).  Network 16 -> 64 -> 64 -> 16 (ReLU), bfloat16 weights, float32
 * biases and accumulation; factors s_b = exp(clip(y_b, -2.3, 2.3)).
 * Model blob: int32 {0x4C47464D, 1, 16, 64, 64, 16, 0, 0}, bf16 W1[16][64],
 * W2[64][64], W3[64][16], float32 b1[64], b2[64], b3[16]
 * (lgf_model_bytes() bytes).
 * ------------------------------------------------------------------------- */
size_t lgf_model_bytes(void);

/* Set the network a LGF_STEP_LEARNED context uses (copied). LGF_E_MODEL for
 * a blob of the wrong size or header. */
int32_t lgf_set_model(lgf_ctx ctx, const void *blob, size_t bytes);

/* Features x of the band powers of the current links' spectrum, and the
 * network's factors s for them (all 1 without a model): the factors a learned
 * update from these links leaves for the update after it.  The links and the
 * factors the next update uses are not changed. */
int32_t lgf_learned_factors(lgf_ctx ctx, double features[16], double s[16]);

/* Training data at the current links of an FP64 context: the band features
 * x and the log factor ln s* of the one factor, common to all bands, that
 * minimises theta after one update (golden-section search, 20 shrink steps,
 * on ln s in [-2.3, 2.3]; s* = 1 unless it beats the plain step).  log_s
 * holds ln s* for every band that holds modes and 0 for empty bands.  The
 * links are not changed. */
int32_t lgf_linesearch_bands(lgf_ctx ctx, double features[16], double log_s[16]);

typedef struct lgf_train_params {
    int64_t steps;   /* Adam steps                         */
    int32_t batch;   /* minibatch size (<= 1024)            */
    int32_t seed;    /* initial weights and sample order    */
    float lr;        /* Adam learning rate                  */
    float reserved;
} lgf_train_params;

/* Train the network on the GPU on n samples (host float32 arrays X, Y = ln s*,
 * M = band mask, each n x 16): masked mean squared error, Adam on float32
 * master weights, forward with bf16-rounded weights.  blob_out receives the
 * model (*bytes in: capacity, out: size); loss_trace (steps floats, or NULL)
 * the minibatch loss of every step. */
int32_t lgf_mlp_train(const float *X, const float *Y, const float *M, int64_t n, const lgf_train_params *tp,
                      void *blob_out, size_t *bytes, float *loss_trace);

/* Loss and gradient (6288 floats, parameter order W1, b1, W2, b2, W3, b3) of a
 * model on n <= 1024 samples, by the training kernels.  LGF_E_MODEL for a
 * malformed blob. */
int32_t lgf_mlp_grad(const void *blob, size_t bytes, const float *X, const float *Y, const float *M, int64_t n,
                     float *grad, double *loss);

/* Network outputs y (n x 16) for inputs X (n x 16).  LGF_E_MODEL for a
 * malformed blob. */
int32_t lgf_mlp_eval(const void *blob, size_t bytes, const float *X, int64_t n, float *Y);

/* Per-kernel timing collected when params.profile = 1: for kernel k < n
 * (names from lgf_kernel_name), the number of launches and their summed
 * duration in milliseconds measured with HIP events on the context's stream.
 * count receives the number of kernels known.  lgf_profile_reset clears. */
int32_t lgf_profile_read(lgf_ctx ctx, int64_t *launches, double *total_ms, int32_t n, int32_t *count);
int32_t lgf_profile_reset(lgf_ctx ctx);
const char *lgf_kernel_name(int32_t k);

/* The launch shape the context runs with (lgf_params.autotune picks it at
 * lgf_create; the default is 256 threads, or the plane size if smaller, and
 * 128-byte tiles): threads per plane block, and the bytes of one row of a
 * (z, t) tile of the Delta layout.  Either pointer may be NULL. */
int32_t lgf_config(lgf_ctx ctx, int32_t *plane_threads, int32_t *tile_bytes);

/* Bytes of device memory the context holds. */
int32_t lgf_device_bytes(lgf_ctx ctx, int64_t *bytes);

const char *lgf_strerror(int32_t code);
const char *lgf_last_error(lgf_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif
