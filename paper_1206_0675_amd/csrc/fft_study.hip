// Decompositions of the 4D FFT of the spectral filter, for the comparison the
// paper makes in Sections 3 and 4 (1D FFTs, 3D plus 1D, 2D plus 2D; the
// paper finds 2D plus 2D fastest on its GPU).  Each variant applies the same
// operation, F^-1 (p2max / p^2) F / V with K(0) = 0 (eq. gx without the
// alpha / 2), to four complex fields held in the plain layout
// D[c][t][z][y][x], and differs only in how the 4D transform is split into
// passes over HBM:
//   1D x 4:       x, y, z forward passes; one t pass (forward, scale,
//                 inverse); z, y, x inverse passes.  Seven launches.
//   2D + 1D + 1D: (x, y) plane forward pass; z forward; t (forward, scale,
//                 inverse); z inverse; (x, y) inverse.  Five launches.  This
//                 is what 3D plus 1D becomes here: a 32^3 block of FP64
//                 complex numbers (512 KB) does not fit the 160 KB of LDS.
//   2D + 2D:      (x, y) forward; the (z, t) pass of the iteration (k_zt:
//                 forward, scale, inverse); (x, y) inverse.  Three launches.
//   2D + 1D + 1D with the t DFT on the matrix cores: as 2D + 1D + 1D, the
//                 t pass computing its DFTs as matrix products (MFMA).
// Every pass stages its lines in LDS and uses the iteration's own FFT passes
// (fft.hpp), so only the decomposition changes.  The iteration itself fuses
// the (x, y) passes into the transform and gauge kernels as well.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "lgf_study.h"
#include "runtime.hpp"

namespace lgf {
namespace study {

using rt::fail;

constexpr int kThreads = 256;
constexpr size_t kPassLds = 64 * 1024;

// One 1D pass over lines of length L = 2^logL along an axis whose element
// stride is S: a block takes 2^k lines.  S = 1 (x axis): consecutive rows.
// S > 1: 2^k consecutive positions below the axis, of one outer index.
struct Pass {
    int L, logL, k;
    int S;
};

__device__ __forceinline__ void pass_lines(const Pass& a, int64_t& base, Lines& ag)
{
    const int nl = 1 << a.k;
    if (a.S == 1) {
        base = (int64_t)blockIdx.x * nl * a.L;
        ag = Lines{a.k, 0, a.L, 0, 1};
    } else {
        const int64_t per = a.S >> a.k;
        const int64_t o = blockIdx.x / per, i0 = (blockIdx.x % per) << a.k;
        base = o * (int64_t)a.S * a.L + i0;
        ag = Lines{a.k, 0, 1, 0, a.S};
    }
}

// Forward (INV false) or inverse transform of every line of the pass.
template <int LMAX, bool INV>
__global__ void __launch_bounds__(kThreads) k_study_axis(C2<double>* __restrict__ D, Pass a,
                                                         const C2<double>* __restrict__ tw)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    C2<double>* buf = reinterpret_cast<C2<double>*>(lds_raw);
    const int tid = threadIdx.x, nth = blockDim.x, nl = 1 << a.k, n = nl << a.logL;
    int64_t base;
    Lines ag;
    pass_lines(a, base, ag);
    const Lines al{a.k, 0, 1, 0, nl};   // element e of line l at e * nl + l
    if (!INV) {
        fft_fwd<double, LMAX>(D + base, ag, buf, a.L, al, tw, tid, nth);
        __syncthreads();
        for (int i = tid; i < n; i += nth) {
            const int l = i & (nl - 1), e = i >> a.k;
            D[base + line_offset(ag, l) + (int64_t)e * ag.es] = buf[i];
        }
    } else {
        for (int i = tid; i < n; i += nth) {
            const int l = i & (nl - 1), e = i >> a.k;
            buf[i] = D[base + line_offset(ag, l) + (int64_t)e * ag.es];
        }
        __syncthreads();
        fft_inv<double, LMAX>(buf, al, D + base, ag, a.L, tw, tid, nth);
    }
}

// The t pass of the 1D decompositions: forward t transform, the spectral
// factor c0 / p^2 of every mode (x, y, z already transformed, so positions
// map to modes through the per-axis tables), inverse t transform.
template <int LMAX>
__global__ void __launch_bounds__(kThreads) k_study_t_scale(C2<double>* __restrict__ D, Pass a,
                                                            const C2<double>* __restrict__ tw,
                                                            const double* __restrict__ ptab, double c0, int Lx,
                                                            int Ly, int Lz, int logLx, int logLy)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    C2<double>* buf = reinterpret_cast<C2<double>*>(lds_raw);
    const int tid = threadIdx.x, nth = blockDim.x, nl = 1 << a.k, n = nl << a.logL;
    int64_t base;
    Lines ag;
    pass_lines(a, base, ag);
    const Lines al{a.k, 0, 1, 0, nl};
    const double *tx = ptab, *ty = tx + Lx, *tz = ty + Ly, *tt = tz + Lz;
    const int64_t i0 = base % a.S;   // first position (x, y, z) of the block
    fft_fwd<double, LMAX>(D + base, ag, buf, a.L, al, tw, tid, nth);
    __syncthreads();
    for (int i = tid; i < n; i += nth) {
        const int l = i & (nl - 1), e = i >> a.k;
        const int64_t s3 = i0 + l;
        const int x = (int)(s3 & (Lx - 1)), y = (int)((s3 >> logLx) & (Ly - 1)), z = (int)(s3 >> (logLx + logLy));
        const double p2 = tx[x] + ty[y] + tz[z] + tt[e];
        const double f = p2 > 0.0 ? c0 / p2 : 0.0;
        buf[i] = C2<double>{buf[i].x * f, buf[i].y * f};
    }
    __syncthreads();
    fft_inv<double, LMAX>(buf, al, D + base, ag, a.L, tw, tid, nth);
}

// The same t pass with the length-N DFT done as a real matrix product on the
// FP64 matrix cores (N = 16, 32 or 64): with W = exp(-2 pi i k e / N) =
// C - i S, the forward DFT of a line is [Yr; Yi] = [[C, S], [-S, C]] [Xr; Xi]
// and the inverse uses [[C, -S], [S, C]].  A wave takes 16 lines at a time
// and computes the 2N x 16 product in 16 x 16 tiles with
// v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16],
// and holds D[l / 16 + 4 j][l % 16] in register j).  Modes come out in natural
// order, so the t factor is 4 sin^2(pi k / N) here.
typedef double v4d __attribute__((vector_size(4 * sizeof(double))));

template <int N, bool INV>
__device__ __forceinline__ double dft_matrix(const C2<double>* tw, int r, int q)
{
    const int k = r & (N - 1), e = q & (N - 1);
    const C2<double> w = tw[(k * e) & (N - 1)];      // (cos, -sin) of 2 pi k e / N
    const double C = w.x, S = -w.y;
    const bool lo_r = r < N, lo_q = q < N;
    if (lo_r == lo_q) return C;
    return (lo_r != INV) ? S : -S;                    // forward: S above, -S below
}

template <int N, bool INV>
__device__ __forceinline__ void dft_mfma_group(C2<double>* buf, int nl, int l0, const C2<double>* tw, int lane)
{
    constexpr int MT = N / 8, KS = N / 2;
    v4d acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = v4d{0.0, 0.0, 0.0, 0.0};
    const int col = lane & 15, sub = lane >> 4;
#pragma unroll 4
    for (int ks = 0; ks < KS; ++ks) {
        const int R = 4 * ks + sub;                   // row of [Xr; Xi]
        const C2<double> x = buf[(R & (N - 1)) * nl + l0 + col];
        const double b = R < N ? x.x : x.y;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const double a = dft_matrix<N, INV>(tw, 16 * m + col, R);
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int R = 16 * m + sub + 4 * j;
            C2<double>& y = buf[(R & (N - 1)) * nl + l0 + col];
            if (R < N) y.x = acc[m][j];
            else y.y = acc[m][j];
        }
}

template <int N>
__global__ void __launch_bounds__(kThreads) k_study_t_mfma(C2<double>* __restrict__ D, Pass a,
                                                           const C2<double>* __restrict__ tw,
                                                           const double* __restrict__ ptab, double c0, int Lx,
                                                           int Ly, int Lz, int logLx, int logLy)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    C2<double>* buf = reinterpret_cast<C2<double>*>(lds_raw);
    __shared__ C2<double> tws[N];
    const int tid = threadIdx.x, nth = blockDim.x, nl = 1 << a.k, n = nl * N;
    const int lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
    int64_t base;
    Lines ag;
    pass_lines(a, base, ag);
    const double *tx = ptab, *ty = tx + Lx, *tz = ty + Ly;
    const int64_t i0 = base % a.S;
    if (tid < N) tws[tid] = tw[tid];
    for (int i = tid; i < n; i += nth) {
        const int l = i & (nl - 1), e = i >> a.k;
        buf[i] = D[base + line_offset(ag, l) + (int64_t)e * ag.es];
    }
    __syncthreads();
    // each wave owns the 16-line groups g = wave, wave + nw, ...: no other
    // wave touches their LDS words until the barrier
    for (int g = wave; g < (nl >> 4); g += nw) dft_mfma_group<N, false>(buf, nl, 16 * g, tws, lane);
    __syncthreads();
    for (int i = tid; i < n; i += nth) {
        const int l = i & (nl - 1), kk = i >> a.k;
        const int64_t s3 = i0 + l;
        const int x = (int)(s3 & (Lx - 1)), y = (int)((s3 >> logLx) & (Ly - 1)), z = (int)(s3 >> (logLx + logLy));
        const double st = sin(M_PI * (double)kk / (double)N);
        const double p2 = tx[x] + ty[y] + tz[z] + 4.0 * st * st;
        const double f = p2 > 0.0 ? c0 / p2 : 0.0;
        buf[i] = C2<double>{buf[i].x * f, buf[i].y * f};
    }
    __syncthreads();
    for (int g = wave; g < (nl >> 4); g += nw) dft_mfma_group<N, true>(buf, nl, 16 * g, tws, lane);
    __syncthreads();
    for (int i = tid; i < n; i += nth) {
        const int l = i & (nl - 1), e = i >> a.k;
        D[base + line_offset(ag, l) + (int64_t)e * ag.es] = buf[i];
    }
}

// The (x, y) plane pass: one block per plane, rows at a pitch of Lx + 1 in
// LDS (as the iteration's plane kernels).
template <int LMAX, bool INV>
__global__ void __launch_bounds__(kThreads) k_study_xy(C2<double>* __restrict__ D, int Lx, int Ly, int logLx,
                                                       int logLy, const C2<double>* __restrict__ twx,
                                                       const C2<double>* __restrict__ twy)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    C2<double>* buf = reinterpret_cast<C2<double>*>(lds_raw);
    const int tid = threadIdx.x, nth = blockDim.x, RP = Lx + 1, np = Lx * Ly;
    C2<double>* P = D + (int64_t)blockIdx.x * np;
    const Lines gx{logLy, 0, Lx, 0, 1}, lx{logLy, 0, RP, 0, 1}, ly{logLx, 0, 1, 0, RP};
    if (!INV) {
        fft_fwd<double, LMAX>(P, gx, buf, Lx, lx, twx, tid, nth);
        __syncthreads();
        fft_fwd<double, LMAX>(buf, Ly, ly, twy, tid, nth);
        __syncthreads();
        for (int i = tid; i < np; i += nth) P[i] = buf[(i >> logLx) * RP + (i & (Lx - 1))];
    } else {
        for (int i = tid; i < np; i += nth) buf[(i >> logLx) * RP + (i & (Lx - 1))] = P[i];
        __syncthreads();
        fft_inv<double, LMAX>(buf, Ly, ly, twy, tid, nth);
        __syncthreads();
        fft_inv<double, LMAX>(buf, lx, P, gx, Lx, twx, tid, nth);
    }
}

struct Study : rt::Runner {
    Geo g{};
    int variant = 0;
    C2<double>* D = nullptr;
    C2<double>* D0 = nullptr;
    C2<double>* tw = nullptr;
    double* ptab = nullptr;
    DevState* st = nullptr;
    int tw_off[4] = {};
    double c0 = 0.0;
};

// log2 of the lines per block of a pass: the most that fit kPassLds, at most
// the positions below the axis (S > 1) and at most all the lines
inline int pass_k(int L, int S, int64_t lines)
{
    int k = 0;
    while (((size_t)L << (k + 1)) * sizeof(C2<double>) <= kPassLds && (S == 1 || (1 << (k + 1)) <= S) &&
           ((int64_t)1 << (k + 1)) <= lines)
        ++k;
    return k;
}

inline int32_t axis_pass(Study* s, int ax, bool inv)
{
    const Geo& g = s->g;
    int S = 1;
    for (int m = 0; m < ax; ++m) S *= g.L[m];
    const int64_t lines = 4 * g.V / g.L[ax];
    Pass a{g.L[ax], g.logL[ax], pass_k(g.L[ax], S, lines), S};
    const dim3 grid((unsigned)(lines >> a.k));
    const size_t lds = ((size_t)g.L[ax] << a.k) * sizeof(C2<double>);
    const C2<double>* tw = s->tw + s->tw_off[ax];
    if (inv) return rt::launch(s, rt::K_FIELD, k_study_axis<64, true>, grid, dim3(kThreads), lds, s->D, a, tw);
    return rt::launch(s, rt::K_FIELD, k_study_axis<64, false>, grid, dim3(kThreads), lds, s->D, a, tw);
}

inline int32_t t_scale_pass(Study* s)
{
    const Geo& g = s->g;
    const int S = g.L[0] * g.L[1] * g.L[2];
    const int64_t lines = 4 * g.V / g.L[3];
    Pass a{g.L[3], g.logL[3], pass_k(g.L[3], S, lines), S};
    const dim3 grid((unsigned)(lines >> a.k));
    const size_t lds = ((size_t)g.L[3] << a.k) * sizeof(C2<double>);
    return rt::launch(s, rt::K_ZT, k_study_t_scale<64>, grid, dim3(kThreads), lds, s->D, a,
                      (const C2<double>*)(s->tw + s->tw_off[3]), (const double*)s->ptab, s->c0, g.L[0], g.L[1],
                      g.L[2], g.logL[0], g.logL[1]);
}

inline int32_t t_mfma_pass(Study* s)
{
    const Geo& g = s->g;
    const int S = g.L[0] * g.L[1] * g.L[2];
    const int64_t lines = 4 * g.V / g.L[3];
    Pass a{g.L[3], g.logL[3], pass_k(g.L[3], S, lines), S};
    if (a.k < 4) return fail(s, LGF_E_UNSUPPORTED_SHAPE, "lgf_fft_study: the MFMA t pass needs 16 lines per block");
    const dim3 grid((unsigned)(lines >> a.k));
    const size_t lds = ((size_t)g.L[3] << a.k) * sizeof(C2<double>);
    const C2<double>* tw = s->tw + s->tw_off[3];
    switch (g.L[3]) {
    case 16:
        return rt::launch(s, rt::K_ZT, k_study_t_mfma<16>, grid, dim3(kThreads), lds, s->D, a, tw,
                          (const double*)s->ptab, s->c0, g.L[0], g.L[1], g.L[2], g.logL[0], g.logL[1]);
    case 32:
        return rt::launch(s, rt::K_ZT, k_study_t_mfma<32>, grid, dim3(kThreads), lds, s->D, a, tw,
                          (const double*)s->ptab, s->c0, g.L[0], g.L[1], g.L[2], g.logL[0], g.logL[1]);
    case 64:
        return rt::launch(s, rt::K_ZT, k_study_t_mfma<64>, grid, dim3(kThreads), lds, s->D, a, tw,
                          (const double*)s->ptab, s->c0, g.L[0], g.L[1], g.L[2], g.logL[0], g.logL[1]);
    default:
        return fail(s, LGF_E_UNSUPPORTED_SHAPE, "lgf_fft_study: the MFMA t pass needs Lt = 16, 32 or 64");
    }
}

inline int32_t xy_pass(Study* s, bool inv)
{
    const Geo& g = s->g;
    const dim3 grid((unsigned)(4 * g.NQ));
    const size_t lds = (size_t)(g.L[0] + 1) * g.L[1] * sizeof(C2<double>);
    const C2<double>*twx = s->tw + s->tw_off[0], *twy = s->tw + s->tw_off[1];
    if (inv)
        return rt::launch(s, rt::K_FIELD, k_study_xy<64, true>, grid, dim3(kThreads), lds, s->D, g.L[0], g.L[1],
                          g.logL[0], g.logL[1], twx, twy);
    return rt::launch(s, rt::K_FIELD, k_study_xy<64, false>, grid, dim3(kThreads), lds, s->D, g.L[0], g.L[1],
                      g.logL[0], g.logL[1], twx, twy);
}

// The (z, t) pass of the iteration on the plain layout: one tile spanning the
// whole (x, y) plane (W = Lx Ly) and one chunk per field (DS = V).
inline int32_t zt_pass(Study* s)
{
    Geo z = s->g;
    z.W = z.NP;
    z.logW = z.logNP;
    z.DS = z.V;
    const int l = rt::zt_part_log<double>(z);
    return rt::launch(s, rt::K_ZT, k_zt<double, 64>, dim3(rt::zt_blocks(z, l)), dim3(512), rt::zt_lds<double>(z, l),
                      z, s->D, (const C2<double>*)(s->tw + s->tw_off[2]), (const C2<double>*)(s->tw + s->tw_off[3]),
                      (const double*)s->ptab, s->c0, 1, l, (const DevState*)s->st);
}

inline int32_t filter(Study* s)
{
    switch (s->variant) {
    case LGF_FFT_1DX4:
        for (int ax = 0; ax < 3; ++ax) TRY(axis_pass(s, ax, false));
        TRY(t_scale_pass(s));
        for (int ax = 2; ax >= 0; --ax) TRY(axis_pass(s, ax, true));
        return LGF_OK;
    case LGF_FFT_2D1D1D:
    case LGF_FFT_2D1D1D_MFMA:
        TRY(xy_pass(s, false));
        TRY(axis_pass(s, 2, false));
        TRY(s->variant == LGF_FFT_2D1D1D ? t_scale_pass(s) : t_mfma_pass(s));
        TRY(axis_pass(s, 2, true));
        return xy_pass(s, true);
    default:
        TRY(xy_pass(s, false));
        TRY(zt_pass(s));
        return xy_pass(s, true);
    }
}

inline int32_t run(Study* s, const int32_t* dims, const void* in, void* out, int32_t where, int32_t reps,
                   double* ms)
{
    s->g = rt::make_geo<double>(dims, 128);
    const Geo& g = s->g;
    const size_t bytes = sizeof(C2<double>) * 4 * (size_t)g.V;
    const hipMemcpyKind kin = where == LGF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind kout = where == LGF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIPCHK(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    HIPCHK(s, hipMalloc(&s->D, bytes));
    HIPCHK(s, hipMalloc(&s->D0, bytes));
    const std::vector<C2<double>> tw = rt::twiddles<double>(dims, s->tw_off);
    double p2max = 0.0;
    const std::vector<double> pt = rt::momentum_tables(dims, &p2max);
    HIPCHK(s, hipMalloc(&s->tw, sizeof(C2<double>) * tw.size()));
    HIPCHK(s, hipMalloc(&s->ptab, sizeof(double) * pt.size()));
    HIPCHK(s, hipMalloc(&s->st, sizeof(DevState)));
    HIPCHK(s, hipMemcpy(s->tw, tw.data(), sizeof(C2<double>) * tw.size(), hipMemcpyHostToDevice));
    HIPCHK(s, hipMemcpy(s->ptab, pt.data(), sizeof(double) * pt.size(), hipMemcpyHostToDevice));
    HIPCHK(s, hipMemset(s->st, 0, sizeof(DevState)));
    s->c0 = p2max / (double)g.V;
    for (const void* f : {reinterpret_cast<const void*>(&k_zt<double, 64>),
                          reinterpret_cast<const void*>(&k_study_axis<64, false>),
                          reinterpret_cast<const void*>(&k_study_axis<64, true>),
                          reinterpret_cast<const void*>(&k_study_t_scale<64>),
                          reinterpret_cast<const void*>(&k_study_xy<64, false>),
                          reinterpret_cast<const void*>(&k_study_xy<64, true>),
                          reinterpret_cast<const void*>(&k_study_t_mfma<16>),
                          reinterpret_cast<const void*>(&k_study_t_mfma<32>),
                          reinterpret_cast<const void*>(&k_study_t_mfma<64>)})
        HIPCHK(s, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rt::kMaxLdsZt));
    HIPCHK(s, hipMemcpyAsync(s->D0, in, bytes, kin, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->D, s->D0, bytes, hipMemcpyDeviceToDevice, s->stream));
    TRY(filter(s));
    HIPCHK(s, hipMemcpyAsync(out, s->D, bytes, kout, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    double total = 0.0;
    for (int r = 0; r < reps; ++r) {
        HIPCHK(s, hipMemcpyAsync(s->D, s->D0, bytes, hipMemcpyDeviceToDevice, s->stream));
        hipEvent_t a = nullptr, b = nullptr;
        HIPCHK(s, hipEventCreate(&a));
        HIPCHK(s, hipEventCreate(&b));
        HIPCHK(s, hipEventRecord(a, s->stream));
        const int32_t rc = filter(s);
        HIPCHK(s, hipEventRecord(b, s->stream));
        HIPCHK(s, hipEventSynchronize(b));
        float t = 0.f;
        HIPCHK(s, hipEventElapsedTime(&t, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        TRY(rc);
        total += t;
    }
    if (ms) *ms = reps > 0 ? total / reps : 0.0;
    return LGF_OK;
}

}  // namespace study
}  // namespace lgf

constexpr size_t kMaxStudyPlane = 64 * 1024;

extern "C" int32_t lgf_fft_study(const int32_t dims[4], int32_t variant, const void* in, void* out, int32_t where,
                                 int32_t reps, double* ms_per_filter)
{
    using namespace lgf;
    if (!dims || !in || !out || (where != LGF_HOST && where != LGF_DEVICE) || reps < 0 || variant < LGF_FFT_1DX4 ||
        variant > LGF_FFT_2D1D1D_MFMA)
        return rt::fail(nullptr, LGF_E_INVALID_ARG, "lgf_fft_study: bad argument");
    for (int m = 0; m < 4; ++m)
        if (!rt::pow2_in(dims[m], 4, 64))
            return rt::fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "lgf_fft_study: extents are powers of two in [4, 64]");
    if ((size_t)(dims[0] + 1) * dims[1] * sizeof(C2<double>) > kMaxStudyPlane ||
        (size_t)dims[2] * dims[3] * sizeof(C2<double>) > kMaxStudyPlane)
        return rt::fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "lgf_fft_study: a plane does not fit LDS");
    study::Study s;
    s.variant = variant;
    const int32_t rc = study::run(&s, dims, in, out, where, reps, ms_per_filter);
    if (rc != LGF_OK) rt::g_noctx_err = s.err;
    for (void* p : {(void*)s.D, (void*)s.D0, (void*)s.tw, (void*)s.ptab, (void*)s.st})
        if (p) (void)hipFree(p);
    rt::release_events(&s);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    return rc;
}
