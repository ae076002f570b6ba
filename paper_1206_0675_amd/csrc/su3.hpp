// Device-side complex and SU(3) arithmetic for the gauge-fixing kernels.
//
// Storage conventions (one complex per element, structure of arrays):
//   link field  U[(mu * NE + e) * V + s]   mu = 0..3, e = 0..NE-1
//   gauge field g[e * V + s]
// NE = 9 stores the full 3x3 matrix; NE = 6 stores its first two rows and
// rebuilds the third as (a x b)^*, exact for SU(3) (the 12-real
// parameterisation of Section 3.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgf {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ C2<T> mk(T a, T b) { C2<T> r; r.x = a; r.y = b; return r; }
// Sums, differences and real scalings are never fused with a neighbouring
// product (no contraction inside them), so a value rounds the same way whether
// it is kept in registers or stored and read back between two kernels.
template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b)
{
#pragma clang fp contract(off)
    return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b)
{
#pragma clang fp contract(off)
    return mk<T>(a.x - b.x, a.y - b.y);
}
// Complex products with explicit fused multiply-adds in a fixed order, so
// the same product gives the same bits wherever it is evaluated (the
// compiler may not re-contract them).
template <typename T>
__device__ __forceinline__ C2<T> cfma(C2<T> a, C2<T> b, C2<T> acc)      // acc + a b
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
template <typename T>
__device__ __forceinline__ C2<T> cfmac(C2<T> a, C2<T> b, C2<T> acc)     // acc + a conj(b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.y, b.x, acc.y);
    acc.y = fma(-a.x, b.y, acc.y);
    return acc;
}
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) { return cfma(a, b, mk<T>(T(0), T(0))); }
// a * conj(b)
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) { return cfmac(a, b, mk<T>(T(0), T(0))); }
template <typename T>
__device__ __forceinline__ C2<T> conjg(C2<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ C2<T> scale(C2<T> a, T f)
{
#pragma clang fp contract(off)
    return mk<T>(a.x * f, a.y * f);
}
// i * a and -i * a
template <typename T>
__device__ __forceinline__ C2<T> mul_i(C2<T> a) { return mk<T>(-a.y, a.x); }
template <typename T>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) { return mk<T>(a.y, -a.x); }

template <typename T>
struct M3 {
    C2<T> e[9];
};

// third row = (first row x second row)^*
template <typename T>
__device__ __forceinline__ C2<T> neg(C2<T> a) { return mk<T>(-a.x, -a.y); }

template <typename T>
__device__ __forceinline__ void rebuild_row3(M3<T>& m)
{
    m.e[6] = conjg(cfma(neg(m.e[2]), m.e[4], cmul(m.e[1], m.e[5])));
    m.e[7] = conjg(cfma(neg(m.e[0]), m.e[5], cmul(m.e[2], m.e[3])));
    m.e[8] = conjg(cfma(neg(m.e[1]), m.e[3], cmul(m.e[0], m.e[4])));
}

template <typename T, int NE>
__device__ __forceinline__ void load_mat(M3<T>& m, const C2<T>* __restrict__ base, int64_t stride, int64_t s)
{
#pragma unroll
    for (int e = 0; e < NE; ++e) m.e[e] = base[e * stride + s];
    if (NE == 6) rebuild_row3(m);
}

template <typename T, int NE>
__device__ __forceinline__ void store_mat(const M3<T>& m, C2<T>* __restrict__ base, int64_t stride, int64_t s)
{
#pragma unroll
    for (int e = 0; e < NE; ++e) base[e * stride + s] = m.e[e];
}

// r = a * u * b^dagger.  With ROWS = 2 only the first two rows are formed
// and the third is rebuilt as (row 1 x row 2)^*, as for a link stored in
// the 12-real form.
template <typename T, int ROWS = 3>
__device__ __forceinline__ void a_u_bdag(const M3<T>& a, const M3<T>& u, const M3<T>& b, M3<T>& r)
{
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        C2<T> au[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            au[k] = cfma(a.e[3 * i + 2], u.e[6 + k], cfma(a.e[3 * i + 1], u.e[3 + k], cmul(a.e[3 * i], u.e[k])));
#pragma unroll
        for (int l = 0; l < 3; ++l)
            r.e[3 * i + l] = cfmac(au[2], b.e[3 * l + 2], cfmac(au[1], b.e[3 * l + 1], cmulc(au[0], b.e[3 * l])));
    }
    if (ROWS == 2) rebuild_row3(r);
}

// The eight real degrees of freedom of u - u^dagger - (1/3) Tr(u - u^dagger):
// p[0] = (.)_01, p[1] = (.)_02, p[2] = (.)_12 (complex), and
// p[3] = Im(.)_00 + i Im(.)_11.  The rest follow from anti-Hermiticity and
// tracelessness.
template <typename T>
struct Alg8 {
    C2<T> c[4];
};

// Written without contraction, so the result from a link held in registers
// equals the result from the same link stored and read back.
template <typename T>
__device__ __forceinline__ void alg_accumulate(Alg8<T>& acc, const M3<T>& u, T sign)
{
#pragma clang fp contract(off)
    const T third = T(2) / T(3);
    C2<T> p0 = u.e[1] - conjg(u.e[3]);
    C2<T> p1 = u.e[2] - conjg(u.e[6]);
    C2<T> p2 = u.e[5] - conjg(u.e[7]);
    T tr = third * (u.e[0].y + u.e[4].y + u.e[8].y);
    C2<T> p3 = mk<T>(T(2) * u.e[0].y - tr, T(2) * u.e[4].y - tr);
    acc.c[0] = acc.c[0] + scale(p0, sign);
    acc.c[1] = acc.c[1] + scale(p1, sign);
    acc.c[2] = acc.c[2] + scale(p2, sign);
    acc.c[3] = acc.c[3] + scale(p3, sign);
}

// Re Tr u in FP64, without contraction (see alg_accumulate).
template <typename T>
__device__ __forceinline__ double re_trace(const M3<T>& u)
{
#pragma clang fp contract(off)
    return (double)u.e[0].x + (double)u.e[4].x + (double)u.e[8].x;
}

// |Delta|^2 = sum_ij |Delta_ij|^2 from the packed form (Delta_22 = -i(a + b)).
template <typename T>
__device__ __forceinline__ double alg_norm2(const Alg8<T>& d)
{
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += 2.0 * ((double)d.c[c].x * d.c[c].x + (double)d.c[c].y * d.c[c].y);
    double a = d.c[3].x, b = d.c[3].y;
    return s + a * a + b * b + (a + b) * (a + b);
}

// 1 + D for a packed anti-Hermitian traceless D, projected to SU(3) by row
// Gram-Schmidt (row 3 = (row 1 x row 2)^*), in double precision.
// No contraction anywhere in it, so every kernel that inlines it rounds the
// same way (the launch shape picks among kernels, and must not change bits).
__device__ __forceinline__ void one_plus_alg_reunit(const C2<double> c[4], M3<double>& m)
{
#pragma clang fp contract(off)
    const double a = c[3].x, b = c[3].y;
    C2<double> r0[3] = {mk<double>(1.0, a), c[0], c[1]};
    C2<double> r1[3] = {mk<double>(-c[0].x, c[0].y), mk<double>(1.0, b), c[2]};
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += r0[j].x * r0[j].x + r0[j].y * r0[j].y;
    n0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) r0[j] = scale(r0[j], n0);
    // <r0, r1> = sum_j conj(r0_j) r1_j
    C2<double> ip = mk<double>(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j) ip = ip + cmul(conjg(r0[j]), r1[j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) r1[j] = r1[j] - cmul(ip, r0[j]);
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n1 += r1[j].x * r1[j].x + r1[j].y * r1[j].y;
    n1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) r1[j] = scale(r1[j], n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) { m.e[j] = r0[j]; m.e[3 + j] = r1[j]; }
    rebuild_row3(m);
}

// exp(X) for a packed anti-Hermitian traceless X (c[0] = X01, c[1] = X02,
// c[2] = X12, c[3] = Im X00 + i Im X11), in double: the update of eq. gx
// with the exponential taken exactly instead of to first order.
// Q = -i X is Hermitian and traceless, so by the Cayley-Hamilton theorem
// Q^3 = k1 Q + k0 1 with k1 = Tr(Q^2)/2 and k0 = det Q, and every power
// Q^n = b0 1 + b1 Q + b2 Q^2 with Q^(n+1) = k0 b2 1 + (b0 + k1 b2) Q + b1 Q^2.
// exp(iQ) = f0 1 + f1 Q + f2 Q^2 with f_k = sum_n (i^n / n!) b_k(n), summed
// over 24 terms after Q is scaled by 2^-m so that its eigenvalues (at most
// sqrt(2 k1) in size) are at most 1 (remainder below 1e-24); the result is
// then squared m times.
__device__ __forceinline__ void alg_exp(const C2<double> c[4], M3<double>& m)
{
#pragma clang fp contract(off)
    const double a = c[3].x, b = c[3].y;
    // Q = -i X
    M3<double> q;
    q.e[0] = mk<double>(a, 0.0);
    q.e[4] = mk<double>(b, 0.0);
    q.e[8] = mk<double>(-(a + b), 0.0);
    q.e[1] = mk<double>(c[0].y, -c[0].x);        // -i X01
    q.e[2] = mk<double>(c[1].y, -c[1].x);
    q.e[5] = mk<double>(c[2].y, -c[2].x);
    q.e[3] = conjg(q.e[1]);
    q.e[6] = conjg(q.e[2]);
    q.e[7] = conjg(q.e[5]);
    double k1 = 0.5 * (a * a + b * b + (a + b) * (a + b)) +
                (c[0].x * c[0].x + c[0].y * c[0].y + c[1].x * c[1].x + c[1].y * c[1].y + c[2].x * c[2].x +
                 c[2].y * c[2].y);
    int halvings = 0;
    double sc = 1.0;
    while (2.0 * k1 * sc * sc > 1.0) {
        sc *= 0.5;
        ++halvings;
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) q.e[e] = scale(q.e[e], sc);
    k1 *= sc * sc;
    // det Q (real for Hermitian Q)
    const C2<double> d = cmul(q.e[0], cmul(q.e[4], q.e[8]) - cmul(q.e[5], q.e[7])) -
                         cmul(q.e[1], cmul(q.e[3], q.e[8]) - cmul(q.e[5], q.e[6])) +
                         cmul(q.e[2], cmul(q.e[3], q.e[7]) - cmul(q.e[4], q.e[6]));
    const double k0 = d.x;
    double b0 = 1.0, b1 = 0.0, b2 = 0.0, t = 1.0;           // Q^0, and |i^n / n!|
    double f0r = 0.0, f0i = 0.0, f1r = 0.0, f1i = 0.0, f2r = 0.0, f2i = 0.0;
#pragma unroll
    for (int n = 0; n < 24; ++n) {
        // i^n: n mod 4 = 0, 1, 2, 3 -> 1, i, -1, -i
        const int r = n & 3;
        const double tr = r == 0 ? t : (r == 2 ? -t : 0.0);
        const double ti = r == 1 ? t : (r == 3 ? -t : 0.0);
        f0r += tr * b0; f0i += ti * b0;
        f1r += tr * b1; f1i += ti * b1;
        f2r += tr * b2; f2i += ti * b2;
        const double nb0 = k0 * b2, nb1 = b0 + k1 * b2, nb2 = b1;
        b0 = nb0; b1 = nb1; b2 = nb2;
        t /= (double)(n + 1);
    }
    M3<double> q2;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            q2.e[3 * i + k] = cfma(q.e[3 * i + 2], q.e[6 + k], cfma(q.e[3 * i + 1], q.e[3 + k], cmul(q.e[3 * i], q.e[k])));
    const C2<double> f0 = mk<double>(f0r, f0i), f1 = mk<double>(f1r, f1i), f2 = mk<double>(f2r, f2i);
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = cfma(f2, q2.e[e], cmul(f1, q.e[e]));
    m.e[0] = m.e[0] + f0;
    m.e[4] = m.e[4] + f0;
    m.e[8] = m.e[8] + f0;
    for (int h = 0; h < halvings; ++h) {
        M3<double> s2;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                s2.e[3 * i + k] =
                    cfma(m.e[3 * i + 2], m.e[6 + k], cfma(m.e[3 * i + 1], m.e[3 + k], cmul(m.e[3 * i], m.e[k])));
        m = s2;
    }
}

// Row Gram-Schmidt projection of a general 3x3 matrix to SU(3), in double
// (no contraction, as one_plus_alg_reunit).
__device__ __forceinline__ void reunit(M3<double>& m)
{
#pragma clang fp contract(off)
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += m.e[j].x * m.e[j].x + m.e[j].y * m.e[j].y;
    n0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[j] = scale(m.e[j], n0);
    C2<double> ip = mk<double>(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j) ip = ip + cmul(conjg(m.e[j]), m.e[3 + j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[3 + j] = m.e[3 + j] - cmul(ip, m.e[j]);
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n1 += m.e[3 + j].x * m.e[3 + j].x + m.e[3 + j].y * m.e[3 + j].y;
    n1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[3 + j] = scale(m.e[3 + j], n1);
    rebuild_row3(m);
}

template <typename TO, typename TI>
__device__ __forceinline__ M3<TO> cast_mat(const M3<TI>& a)
{
    M3<TO> r;
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = mk<TO>((TO)a.e[e].x, (TO)a.e[e].y);
    return r;
}

}  // namespace lgf
