/*
 * lgf_study.h -- timing study of the 4D-FFT decomposition of the spectral
 * filter (arXiv:1206.0675, Section 3 on splitting the 4D FFT into batches
 * of 1D, 3D plus 1D or 2D plus 2D transforms, and Section 4, which measures
 * the three and finds 2D plus 2D fastest).
 *
 * lgf_fft_study applies F^-1 (p2max / p^2) F / V (eq. gx without the factor
 * alpha / 2; p^2 as the iteration's lattice momentum, K(0) = 0) to four
 * complex FP64 fields in the plain layout in[c][t][z][y][x] (c = 0..3;
 * 4 V complex numbers, 64 V bytes), and writes the result to out.  variant
 * selects how the 4D transform is split into passes over device memory:
 *   LGF_FFT_1DX4    x, y, z forward; t forward, scale, inverse; z, y, x
 *                   inverse (seven launches);
 *   LGF_FFT_2D1D1D  (x, y) forward; z forward; t; z inverse; (x, y) inverse
 *                   (five launches; what 3D plus 1D becomes when a 3D block
 *                   does not fit the LDS of one workgroup);
 *   LGF_FFT_2D2D    (x, y) forward; the iteration's (z, t) kernel (forward,
 *                   scale, inverse); (x, y) inverse (three launches);
 *   LGF_FFT_2D1D1D_MFMA  as LGF_FFT_2D1D1D, with the length-Lt DFTs of the t
 *                   pass computed as real matrix products on the FP64 matrix
 *                   cores instead of FFTs (Lt = 16, 32 or 64, else
 *                   LGF_E_UNSUPPORTED_SHAPE).
 * Every pass stages its lines in LDS and uses the iteration's FFT passes.
 * After one untimed application (whose result is written to out), the
 * filter is applied reps more times to a copy of the input and
 * *ms_per_filter receives the mean duration of one application (HIP events
 * around its launches; 0 when reps = 0).
 *
 * in and out are host (LGF_HOST) or device (LGF_DEVICE) memory and may not
 * overlap; nothing is kept after the call, which allocates and frees its own
 * device buffers.  Extents are powers of two in [4, 64] and an (x, y) or
 * (z, t) plane of one field must fit 64 KB, else LGF_E_UNSUPPORTED_SHAPE;
 * other bad arguments give LGF_E_INVALID_ARG (lgf_last_error(NULL) says which).
 */
#ifndef LGF_STUDY_H
#define LGF_STUDY_H

#include "lgf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LGF_FFT_1DX4 0
#define LGF_FFT_2D1D1D 1
#define LGF_FFT_2D2D 2
#define LGF_FFT_2D1D1D_MFMA 3

int32_t lgf_fft_study(const int32_t dims[4], int32_t variant, const void *in, void *out, int32_t where, int32_t reps,
                      double *ms_per_filter);

#ifdef __cplusplus
}
#endif

#endif
