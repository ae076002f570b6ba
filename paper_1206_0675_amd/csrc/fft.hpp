// Power-of-two complex FFTs over lines held in LDS, for the 2D+2D split of
// the 4D transform (Section 3.2: a batch of 2D (x, y) transforms and a batch
// of 2D (z, t) transforms; here with no separate data-reordering pass).
//
// A line of length L = R1 * R2 is transformed in at most two register-blocked
// passes (the "four-step" factorisation of the DFT):
//   pass A: for each k2 < R2, the R1-point DFT of x[k2 + R2 m] over m, times
//           the twiddle W_L^(k2 j1), written back to position k2 + R2 j1;
//   pass B: for each j1 < R1, the R2-point DFT of the R2 contiguous values at
//           R2 j1 + k2, written back in place.
// Mode n = j1 + R1 j2 then sits at position p = j2 + R2 j1 (a digit
// transposition; mode_of_position() below).  The spectral multiply works in
// that order and the inverse undoes the passes in reverse (B^-1 then A^-1),
// so no permutation pass is ever made.  The R-point DFTs (R <= 16) run in
// registers with compile-time twiddles.  W_L^k = exp(-2 pi i k / L); inverse
// transforms are unnormalised.
//
// A set of lines: line l = l_hi * 2^lo_log + l_lo holds element j at
// buf[l_lo * s_lo + l_hi * s_hi + j * es].  All threads of the block call the
// pass routines; each ends with a barrier.
#pragma once
#include "su3.hpp"

namespace lgf {

struct Lines {
    int lo_log;   // log2 of the number of low line indices
    int hi_log;   // log2 of the number of high line indices
    int s_lo, s_hi, es;
};

// (R1, R2) used for a line of length L; the host builds its mode tables from
// the same function.
__host__ __device__ constexpr int fft_r2(int L) { return L <= 8 ? 1 : (L <= 32 ? 4 : 8); }
__host__ __device__ constexpr int fft_r1(int L) { return L / fft_r2(L); }
__host__ __device__ constexpr int mode_of_position(int L, int p)
{
    return p / fft_r2(L) + fft_r1(L) * (p % fft_r2(L));
}

// cos(i pi / 8), i = 0..8
__device__ __forceinline__ constexpr double cos_pi8(int i)
{
    constexpr double c1 = 0.92387953251128675612818318939678828682;   // cos(pi/8)
    constexpr double c2 = 0.70710678118654752440084436210484903928;   // cos(pi/4)
    constexpr double c3 = 0.38268343236508977172845998403039886676;   // cos(3pi/8)
    return i == 0 ? 1.0 : i == 1 ? c1 : i == 2 ? c2 : i == 3 ? c3 : i == 4 ? 0.0
         : i == 5 ? -c3 : i == 6 ? -c2 : i == 7 ? -c1 : -1.0;
}

// v *= exp(-+ 2 pi i k / span), forward sign unless INV; k < span / 2, span <= 16
template <typename T, int SPAN, int K, bool INV>
__device__ __forceinline__ C2<T> twiddle_const(C2<T> v)
{
    constexpr int i = K * (16 / SPAN);            // angle = i * pi / 8, 0 <= i < 8
    if constexpr (i == 0) return v;
    else if constexpr (i == 4) return INV ? mul_i(v) : mul_mi(v);
    else {
        const T c = (T)cos_pi8(i);
        const T s = (T)cos_pi8(i <= 4 ? 4 - i : i - 4);   // sin(i pi / 8)
        const T sn = INV ? s : -s;
        // explicit fused multiply-adds: the same bits in every kernel that
        // inlines this (the compiler may not contract them differently)
        return mk<T>(fma(-v.y, sn, v.x * c), fma(v.y, c, v.x * sn));
    }
}

template <int N, int B>
__host__ __device__ constexpr int bitrev_c(int v)
{
    int r = 0;
    for (int i = 0; i < B; ++i) r |= ((v >> i) & 1) << (B - 1 - i);
    return r;
}

template <int R>
constexpr int log2_c() { return R <= 1 ? 0 : 1 + log2_c<R / 2>(); }

template <typename T, int R, int SPAN, int BLK, int K, bool INV>
__device__ __forceinline__ void dft_bfly(C2<T>* v)
{
    constexpr int h = SPAN / 2;
    const C2<T> a = v[BLK * SPAN + K], b = v[BLK * SPAN + K + h];
    v[BLK * SPAN + K] = a + b;
    v[BLK * SPAN + K + h] = twiddle_const<T, SPAN, K, INV>(a - b);
    if constexpr (K + 1 < h) dft_bfly<T, R, SPAN, BLK, K + 1, INV>(v);
    else if constexpr (BLK + 1 < R / SPAN) dft_bfly<T, R, SPAN, BLK + 1, 0, INV>(v);
}

template <typename T, int R, int SPAN, bool INV>
__device__ __forceinline__ void dft_stages(C2<T>* v)
{
    dft_bfly<T, R, SPAN, 0, 0, INV>(v);
    if constexpr (SPAN > 2) dft_stages<T, R, SPAN / 2, INV>(v);
}

// In-register R-point DFT, natural order in and out (radix-2 decimation in
// frequency; the final bit reversal is a renaming of registers).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(C2<T>* v)
{
    if constexpr (R > 1) {
        dft_stages<T, R, R, INV>(v);
        C2<T> w[R];
#pragma unroll
        for (int j = 0; j < R; ++j) w[j] = v[bitrev_c<R, log2_c<R>()>(j)];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = w[j];
    }
}

__device__ __forceinline__ void task_split(int t, int R, const Lines& a, int& kk, int& line)
{
    // unit-stride element axis: k fastest; otherwise the unit-stride line
    // index fastest, so neighbouring lanes touch neighbouring LDS words
    if (a.es == 1) {
        kk = t & (R - 1);
        line = t / R;
    } else {
        const int lo = t & ((1 << a.lo_log) - 1), rest = t >> a.lo_log;
        kk = rest & (R - 1);
        line = ((rest / R) << a.lo_log) | lo;
    }
}

__device__ __forceinline__ int line_offset(const Lines& a, int line)
{
    const int l_lo = line & ((1 << a.lo_log) - 1);
    const int l_hi = line >> a.lo_log;
    return l_lo * a.s_lo + l_hi * a.s_hi;
}

template <typename T>
__device__ __forceinline__ C2<T>* line_base(C2<T>* buf, const Lines& a, int line)
{
    return buf + line_offset(a, line);
}

template <typename T>
__device__ __forceinline__ const C2<T>* line_base(const C2<T>* buf, const Lines& a, int line)
{
    return buf + line_offset(a, line);
}

// pass A (forward) or A^-1 (inverse); tw = W_L^k, k < L.  Reads the lines
// from `in` (laid out as ai) and writes them to `out` (laid out as ao; both
// layouts hold the same set of lines): in place when both are the LDS buffer,
// or from / to a global array, which saves an LDS copy of the whole block.
template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void fft_pass_a(const C2<T>* in, const Lines ai, C2<T>* out, const Lines ao,
                                           const C2<T>* __restrict__ tw, int tid, int nth)
{
    const int ntask = R2 << (ao.lo_log + ao.hi_log);
    const int sti = R2 * ai.es, sto = R2 * ao.es;
    for (int t = tid; t < ntask; t += nth) {
        int k2, line;
        task_split(t, R2, ao, k2, line);
        const C2<T>* pi = line_base(in, ai, line) + k2 * ai.es;
        C2<T>* p = line_base(out, ao, line) + k2 * ao.es;
        C2<T> v[R1];
#pragma unroll
        for (int m = 0; m < R1; ++m) v[m] = pi[m * sti];
        if (!INV) {
            dft<T, R1, false>(v);
            if (R2 > 1 && k2 != 0) {
#pragma unroll
                for (int j = 1; j < R1; ++j) v[j] = cmul(v[j], tw[k2 * j]);
            }
        } else {
            if (R2 > 1 && k2 != 0) {
#pragma unroll
                for (int j = 1; j < R1; ++j) v[j] = cmulc(v[j], tw[k2 * j]);
            }
            dft<T, R1, true>(v);
        }
#pragma unroll
        for (int m = 0; m < R1; ++m) p[m * sto] = v[m];
    }
    __syncthreads();
}

template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void fft_pass_a(const C2<T>* in, C2<T>* out, const Lines a, const C2<T>* __restrict__ tw,
                                           int tid, int nth)
{
    fft_pass_a<T, R1, R2, INV>(in, a, out, a, tw, tid, nth);
}

template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void fft_pass_a(C2<T>* buf, const Lines a, const C2<T>* __restrict__ tw, int tid, int nth)
{
    fft_pass_a<T, R1, R2, INV>(buf, buf, a, tw, tid, nth);
}

// pass B (forward) or B^-1 (inverse): R2-point DFTs of contiguous groups
template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void fft_pass_b(C2<T>* buf, const Lines a, int tid, int nth)
{
    if constexpr (R2 > 1) {
        const int ntask = R1 << (a.lo_log + a.hi_log);
        const int es = a.es;
        for (int t = tid; t < ntask; t += nth) {
            int j1, line;
            task_split(t, R1, a, j1, line);
            C2<T>* p = line_base(buf, a, line) + j1 * R2 * es;
            C2<T> u[R2];
#pragma unroll
            for (int k = 0; k < R2; ++k) u[k] = p[k * es];
            dft<T, R2, INV>(u);
#pragma unroll
            for (int k = 0; k < R2; ++k) p[k * es] = u[k];
        }
        __syncthreads();
    }
}

template <typename T, int L>
__device__ __forceinline__ void fft_fwd_L(const C2<T>* in, const Lines& ai, C2<T>* buf, const Lines& a,
                                          const C2<T>* tw, int tid, int nth)
{
    fft_pass_a<T, fft_r1(L), fft_r2(L), false>(in, ai, buf, a, tw, tid, nth);
    fft_pass_b<T, fft_r1(L), fft_r2(L), false>(buf, a, tid, nth);
}

template <typename T, int L>
__device__ __forceinline__ void fft_inv_L(C2<T>* buf, const Lines& a, C2<T>* out, const Lines& ao, const C2<T>* tw,
                                          int tid, int nth)
{
    fft_pass_b<T, fft_r1(L), fft_r2(L), true>(buf, a, tid, nth);
    fft_pass_a<T, fft_r1(L), fft_r2(L), true>(buf, a, out, ao, tw, tid, nth);
}

// Forward transform of every line (output in mode_of_position order), read
// from `in` laid out as ai into buf laid out as a.  L is a power of two in
// [4, LMAX]; kernels built for LMAX = 64 carry no code (and no register
// demand) for longer lines.
template <typename T, int LMAX>
__device__ __forceinline__ void fft_fwd(const C2<T>* in, const Lines ai, C2<T>* buf, int L, const Lines a,
                                        const C2<T>* __restrict__ tw, int tid, int nth)
{
    switch (L) {
    case 4: fft_fwd_L<T, 4>(in, ai, buf, a, tw, tid, nth); break;
    case 8: fft_fwd_L<T, 8>(in, ai, buf, a, tw, tid, nth); break;
    case 16: fft_fwd_L<T, 16>(in, ai, buf, a, tw, tid, nth); break;
    case 32: fft_fwd_L<T, 32>(in, ai, buf, a, tw, tid, nth); break;
    case 64: fft_fwd_L<T, 64>(in, ai, buf, a, tw, tid, nth); break;
    default: if constexpr (LMAX >= 128) fft_fwd_L<T, 128>(in, ai, buf, a, tw, tid, nth); break;
    }
}

template <typename T, int LMAX>
__device__ __forceinline__ void fft_fwd(const C2<T>* in, C2<T>* buf, int L, const Lines a,
                                        const C2<T>* __restrict__ tw, int tid, int nth)
{
    fft_fwd<T, LMAX>(in, a, buf, L, a, tw, tid, nth);
}

// The same transform, in place in buf.
template <typename T, int LMAX>
__device__ __forceinline__ void fft_fwd(C2<T>* buf, int L, const Lines a, const C2<T>* __restrict__ tw, int tid,
                                        int nth)
{
    fft_fwd<T, LMAX>(buf, a, buf, L, a, tw, tid, nth);
}

// Inverse (unnormalised) transform of every line; undoes fft_fwd up to L.
// The result goes to `out` laid out as ao.
template <typename T, int LMAX>
__device__ __forceinline__ void fft_inv(C2<T>* buf, const Lines a, C2<T>* out, const Lines ao, int L,
                                        const C2<T>* __restrict__ tw, int tid, int nth)
{
    switch (L) {
    case 4: fft_inv_L<T, 4>(buf, a, out, ao, tw, tid, nth); break;
    case 8: fft_inv_L<T, 8>(buf, a, out, ao, tw, tid, nth); break;
    case 16: fft_inv_L<T, 16>(buf, a, out, ao, tw, tid, nth); break;
    case 32: fft_inv_L<T, 32>(buf, a, out, ao, tw, tid, nth); break;
    case 64: fft_inv_L<T, 64>(buf, a, out, ao, tw, tid, nth); break;
    default: if constexpr (LMAX >= 128) fft_inv_L<T, 128>(buf, a, out, ao, tw, tid, nth); break;
    }
}

template <typename T, int LMAX>
__device__ __forceinline__ void fft_inv(C2<T>* buf, C2<T>* out, int L, const Lines a, const C2<T>* __restrict__ tw,
                                        int tid, int nth)
{
    fft_inv<T, LMAX>(buf, a, out, a, L, tw, tid, nth);
}

// The same transform, in place in buf.
template <typename T, int LMAX>
__device__ __forceinline__ void fft_inv(C2<T>* buf, int L, const Lines a, const C2<T>* __restrict__ tw, int tid,
                                        int nth)
{
    fft_inv<T, LMAX>(buf, a, buf, a, L, tw, tid, nth);
}

}  // namespace lgf
