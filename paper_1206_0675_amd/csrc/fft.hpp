// Power-of-two complex FFTs over lines held in LDS, for the 2D+2D split of
// the 4D transform (Section 3.2: a batch of 2D (x, y) transforms, then a
// batch of 2D (z, t) transforms; here without any data reordering pass).
//
// Forward transforms are decimation-in-frequency (natural order in,
// bit-reversed order out); inverse transforms are decimation-in-time
// (bit-reversed in, natural out).  The spectral multiply sits between them
// and indexes modes through the bit reversal, so no permutation is ever
// performed.  Radix-4 butterflies (each equal to two radix-2 stages) with one
// radix-2 stage when log2(L) is odd.  Twiddles W_L^k = exp(-2 pi i k / L)
// come from a host-computed table of L entries.
//
// A set of lines is described by Lines: line l = l_hi * 2^lo_log + l_lo holds
// element j at buf[l_lo * s_lo + l_hi * s_hi + j * es].  All threads of the
// block call these routines; they end with a barrier.
#pragma once
#include "su3.hpp"

namespace lgf {

struct Lines {
    int logL;     // log2 of the line length
    int lo_log;   // log2 of the number of low line indices
    int hi_log;   // log2 of the number of high line indices
    int s_lo, s_hi, es;
};

template <typename T>
__device__ __forceinline__ C2<T>* line_ptr(C2<T>* buf, const Lines& a, int line)
{
    const int l_lo = line & ((1 << a.lo_log) - 1);
    const int l_hi = line >> a.lo_log;
    return buf + l_lo * a.s_lo + l_hi * a.s_hi;
}

// Forward (sign -1) transform of every line; output in bit-reversed order.
template <typename T>
__device__ void fft_dif(C2<T>* buf, const Lines a, const C2<T>* __restrict__ tw, int tid, int nth)
{
    const int L = 1 << a.logL;
    const int es = a.es;
    int logspan = a.logL;
    while (logspan >= 2) {
        const int logq = logspan - 2, q = 1 << logq;
        const int twstep = 1 << (a.logL - logspan);
        const int nbf = 1 << (a.lo_log + a.hi_log + a.logL - 2);
        for (int b = tid; b < nbf; b += nth) {
            const int j = b & ((L >> 2) - 1);
            C2<T>* p = line_ptr(buf, a, b >> (a.logL - 2));
            const int k = j & (q - 1);
            const int p0 = ((j >> logq) << logspan) + k;
            C2<T> x0 = p[p0 * es], x1 = p[(p0 + q) * es], x2 = p[(p0 + 2 * q) * es], x3 = p[(p0 + 3 * q) * es];
            C2<T> s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3;
            C2<T> y0 = s02 + s13;
            C2<T> y2 = s02 - s13;
            C2<T> y1 = d02 + mul_mi(d13);   // x0 - i x1 - x2 + i x3
            C2<T> y3 = d02 + mul_i(d13);    // x0 + i x1 - x2 - i x3
            if (k != 0) {
                y1 = cmul(y1, tw[k * twstep]);
                y2 = cmul(y2, tw[2 * k * twstep]);
                y3 = cmul(y3, tw[3 * k * twstep]);
            }
            p[p0 * es] = y0;
            p[(p0 + q) * es] = y2;
            p[(p0 + 2 * q) * es] = y1;
            p[(p0 + 3 * q) * es] = y3;
        }
        __syncthreads();
        logspan -= 2;
    }
    if (logspan == 1) {
        const int nbf = 1 << (a.lo_log + a.hi_log + a.logL - 1);
        for (int b = tid; b < nbf; b += nth) {
            const int j = b & ((L >> 1) - 1);
            C2<T>* p = line_ptr(buf, a, b >> (a.logL - 1));
            C2<T> x0 = p[(2 * j) * es], x1 = p[(2 * j + 1) * es];
            p[(2 * j) * es] = x0 + x1;
            p[(2 * j + 1) * es] = x0 - x1;
        }
        __syncthreads();
    }
}

// Inverse (sign +1, unnormalised) transform of every line; input in
// bit-reversed order, output natural.  Undoes fft_dif up to a factor L.
template <typename T>
__device__ void fft_dit(C2<T>* buf, const Lines a, const C2<T>* __restrict__ tw, int tid, int nth)
{
    const int L = 1 << a.logL;
    const int es = a.es;
    int logspan = (a.logL & 1) ? 1 : 2;
    if (logspan == 1) {
        const int nbf = 1 << (a.lo_log + a.hi_log + a.logL - 1);
        for (int b = tid; b < nbf; b += nth) {
            const int j = b & ((L >> 1) - 1);
            C2<T>* p = line_ptr(buf, a, b >> (a.logL - 1));
            C2<T> x0 = p[(2 * j) * es], x1 = p[(2 * j + 1) * es];
            p[(2 * j) * es] = x0 + x1;
            p[(2 * j + 1) * es] = x0 - x1;
        }
        __syncthreads();
        logspan = 3;
    }
    for (; logspan <= a.logL; logspan += 2) {
        const int logq = logspan - 2, q = 1 << logq;
        const int twstep = 1 << (a.logL - logspan);
        const int nbf = 1 << (a.lo_log + a.hi_log + a.logL - 2);
        for (int b = tid; b < nbf; b += nth) {
            const int j = b & ((L >> 2) - 1);
            C2<T>* p = line_ptr(buf, a, b >> (a.logL - 2));
            const int k = j & (q - 1);
            const int p0 = ((j >> logq) << logspan) + k;
            C2<T> z0 = p[p0 * es], z1 = p[(p0 + q) * es], z2 = p[(p0 + 2 * q) * es], z3 = p[(p0 + 3 * q) * es];
            if (k != 0) {
                const C2<T> w2 = tw[2 * k * twstep];
                z1 = cmulc(z1, w2);
                z3 = cmulc(z3, w2);
            }
            C2<T> a0 = z0 + z1, a1 = z0 - z1, b0 = z2 + z3, b1 = z2 - z3;
            if (k != 0) {
                const C2<T> w1 = tw[k * twstep];
                b0 = cmulc(b0, w1);
                b1 = cmulc(b1, w1);
            }
            b1 = mul_i(b1);
            p[p0 * es] = a0 + b0;
            p[(p0 + 2 * q) * es] = a0 - b0;
            p[(p0 + q) * es] = a1 + b1;
            p[(p0 + 3 * q) * es] = a1 - b1;
        }
        __syncthreads();
    }
}

}  // namespace lgf
