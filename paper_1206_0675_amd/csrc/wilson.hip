// Wilson-action SU(3) configuration generator on gfx950: Cabibbo-Marinari
// heatbath (Kennedy-Pendleton SU(2) sampling) and SU(2)-subgroup
// overrelaxation in checkerboard sweeps, Philox4x64-10 counters.  The
// definitions (action, staple, subgroup order, counters, samplers) are those
// stated in include/lgf_wilson.h; the ensembles stand for the Wilson-action
// configurations the paper gauge-fixes (Sections 1 and 4).
//
// One thread updates one link of a (direction, parity) class; a sweep is
// eight launches.  The links stay in the canonical layout (a link is 144
// contiguous bytes, read as nine 16-byte loads), so a generated field is
// handed to the gauge-fixing context as it is.  Arithmetic is FP64 with
// contraction off, so a link's update does not depend on the launch shape.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "lgf_wilson.h"
#include "runtime.hpp"

using lgf::rt::fail;

namespace lgfw {

#pragma clang fp contract(off)

struct WGeo {
    int L[4];
    int64_t V;
};

struct Cx {
    double re, im;
};

__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return Cx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return Cx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx cconj(Cx a) { return Cx{a.re, -a.im}; }

struct M {
    Cx e[3][3];
};

__device__ __forceinline__ M load_link(const double* __restrict__ U, int64_t l)
{
    const double2* p = reinterpret_cast<const double2*>(U + l * 18);
    M m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = p[k];
        m.e[k / 3][k % 3] = Cx{v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ void store_link(double* __restrict__ U, int64_t l, const M& m)
{
    double2* p = reinterpret_cast<double2*>(U + l * 18);
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im);
}

// Row 2 of an SU(3) matrix from rows 0 and 1: the complex conjugate of
// their cross product (the last step of project_su3).
__device__ __forceinline__ void third_row(M& m)
{
    const Cx* a = m.e[0];
    const Cx* b = m.e[1];
    m.e[2][0] = cconj(csub(cmul(a[1], b[2]), cmul(a[2], b[1])));
    m.e[2][1] = cconj(csub(cmul(a[2], b[0]), cmul(a[0], b[2])));
    m.e[2][2] = cconj(csub(cmul(a[0], b[1]), cmul(a[1], b[0])));
}

// The sweeps keep the links in an even-odd layout of separate matrix
// elements, rows 0 and 1 only: element k < 6 (row k / 3, column k % 3) of
// link (site s, direction mu) at E[((mu * 6 + k) * 2 + parity(s)) * Vh + s / 2]
// (Vh = V / 2; s / 2 numbers the sites of one parity, x fastest, since Lx is
// even), and row 2 is rebuilt on load.  Every link a sweep writes has just
// been projected to SU(3), whose row 2 is that same function of rows 0 and 1.
// The threads of a class launch take consecutive s / 2, so every load and
// store of a link element is one contiguous run across the wavefront.
constexpr int kEoElems = 6;

__device__ __forceinline__ M load_eo(const double2* __restrict__ E, int64_t Vh, int64_t s, int mu, int par)
{
    const double2* p = E + ((int64_t)(mu * kEoElems) * 2 + par) * Vh + (s >> 1);
    M m;
#pragma unroll
    for (int k = 0; k < kEoElems; ++k) {
        const double2 v = p[(int64_t)k * 2 * Vh];
        m.e[k / 3][k % 3] = Cx{v.x, v.y};
    }
    third_row(m);
    return m;
}

__device__ __forceinline__ void store_eo(double2* __restrict__ E, int64_t Vh, int64_t s, int mu, int par, const M& m)
{
    double2* p = E + ((int64_t)(mu * kEoElems) * 2 + par) * Vh + (s >> 1);
#pragma unroll
    for (int k = 0; k < kEoElems; ++k)
        p[(int64_t)k * 2 * Vh] = make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im);
}

// a b with the dagger taken of a (da) and/or b (db); each element summed over
// k = 0, 1, 2 in order
template <bool DA, bool DB>
__device__ __forceinline__ M mul(const M& a, const M& b)
{
    M r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx s{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const Cx x = DA ? cconj(a.e[k][i]) : a.e[i][k];
                const Cx y = DB ? cconj(b.e[j][k]) : b.e[k][j];
                s = cadd(s, cmul(x, y));
            }
            r.e[i][j] = s;
        }
    return r;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 and the samplers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double unit01(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }

__device__ __forceinline__ void uniforms4(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                          double u[4])
{
    uint64_t c[4] = {c0, c1, c2, c3};
    philox(c, seed, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = unit01(c[i]);
}

// x0 with density sqrt(1 - x0^2) exp(c x0); false after the attempt limit
__device__ bool sample_x0(double c, uint64_t seed, uint64_t l, uint64_t n, uint64_t k, double& x0)
{
    for (uint64_t t = 0; t < LGF_WILSON_MAX_ATTEMPTS; ++t) {
        double u[4];
        uniforms4(seed, l, n, k, t, u);
        if (c >= 1.0) {
            const double cs = cos(2.0 * M_PI * u[1]);
            const double l2 = -(log(u[0]) + cs * cs * log(u[2])) / (2.0 * c);
            if (u[3] * u[3] <= 1.0 - l2) {
                x0 = 1.0 - 2.0 * l2;
                return true;
            }
        } else {
            const double x = 2.0 * u[0] - 1.0;
            if (u[1] <= sqrt(1.0 - x * x) * exp(c * (x - 1.0))) {
                x0 = x;
                return true;
            }
        }
    }
    return false;
}

// quaternion product: Q(p) Q(q) = Q(r)
__device__ __forceinline__ void qmul(const double p[4], const double q[4], double r[4])
{
    r[0] = p[0] * q[0] - (p[1] * q[1] + p[2] * q[2] + p[3] * q[3]);
    r[1] = p[0] * q[1] + q[0] * p[1] - (p[2] * q[3] - p[3] * q[2]);
    r[2] = p[0] * q[2] + q[0] * p[2] - (p[3] * q[1] - p[1] * q[3]);
    r[3] = p[0] * q[3] + q[0] * p[3] - (p[1] * q[2] - p[2] * q[1]);
}

// rows i, j of m <- Q(r) (rows i, j)
__device__ __forceinline__ void rotate_rows(M& m, int i, int j, const double r[4])
{
    const Cx r00{r[0], r[3]}, r01{r[2], r[1]}, r10{-r[2], r[1]}, r11{r[0], -r[3]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Cx a = m.e[i][c], b = m.e[j][c];
        m.e[i][c] = cadd(cmul(r00, a), cmul(r01, b));
        m.e[j][c] = cadd(cmul(r10, a), cmul(r11, b));
    }
}

__device__ __forceinline__ void project_su3(M& m)
{
    Cx* a = m.e[0];
    Cx* b = m.e[1];
    double na = 0.0;
    {
        Cx s = cadd(cadd(cmul(a[0], cconj(a[0])), cmul(a[1], cconj(a[1]))), cmul(a[2], cconj(a[2])));
        na = sqrt(s.re);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) a[j] = Cx{a[j].re / na, a[j].im / na};
    const Cx ab = cadd(cadd(cmul(cconj(a[0]), b[0]), cmul(cconj(a[1]), b[1])), cmul(cconj(a[2]), b[2]));
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = csub(b[j], cmul(ab, a[j]));
    double nb = 0.0;
    {
        Cx s = cadd(cadd(cmul(b[0], cconj(b[0])), cmul(b[1], cconj(b[1]))), cmul(b[2], cconj(b[2])));
        nb = sqrt(s.re);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) b[j] = Cx{b[j].re / nb, b[j].im / nb};
    third_row(m);
}

__device__ __forceinline__ int64_t site_of(const WGeo& g, int x, int y, int z, int t)
{
    return (((int64_t)t * g.L[2] + z) * g.L[1] + y) * g.L[0] + x;
}

// ---------------------------------------------------------------------------
// one (direction, parity) class of links
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(256) k_wilson_links(WGeo g, double2* __restrict__ E, double beta, uint64_t seed,
                                                      uint64_t sweep, int mu, int par,
                                                      unsigned long long* __restrict__ skipped)
{
    const int64_t Vh = g.V / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.V / 2) return;
    // the idx-th site of parity par, x fastest
    const int hx = g.L[0] / 2;
    int64_t row = idx / hx;
    const int y = (int)(row % g.L[1]);
    row /= g.L[1];
    const int z = (int)(row % g.L[2]);
    const int t = (int)(row / g.L[2]);
    const int x = 2 * (int)(idx % hx) + ((par + y + z + t) & 1);
    int c[4] = {x, y, z, t};
    const int64_t s = site_of(g, x, y, z, t);
    auto nb = [&](int m1, int d1, int m2, int d2) {
        int q[4] = {c[0], c[1], c[2], c[3]};
        q[m1] = (q[m1] + d1 + g.L[m1]) % g.L[m1];
        if (m2 >= 0) q[m2] = (q[m2] + d2 + g.L[m2]) % g.L[m2];
        return site_of(g, q[0], q[1], q[2], q[3]);
    };
    // staple: per nu != mu (ascending) the upper then the lower term
    M A;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A.e[i][j] = Cx{0.0, 0.0};
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t xm = nb(mu, 1, -1, 0), xn = nb(nu, 1, -1, 0), xmn = nb(mu, 1, nu, -1), xdn = nb(nu, -1, -1, 0);
        M up, dn;
        {   // x + mu and x + nu have the other parity, x - nu too, x + mu - nu this one
            const M a = load_eo(E, Vh, xm, nu, par ^ 1), b = load_eo(E, Vh, xn, mu, par ^ 1);
            const M ab = mul<false, true>(a, b);
            const M cc = load_eo(E, Vh, s, nu, par);
            up = mul<false, true>(ab, cc);
        }
        {
            const M e = load_eo(E, Vh, xmn, nu, par), f = load_eo(E, Vh, xdn, mu, par ^ 1);
            const M ef = mul<true, true>(e, f);
            const M gg = load_eo(E, Vh, xdn, nu, par ^ 1);
            dn = mul<false, false>(ef, gg);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A.e[i][j] = cadd(A.e[i][j], cadd(up.e[i][j], dn.e[i][j]));
    }
    const int64_t l = s * 4 + mu;
    M u = load_eo(E, Vh, s, mu, par);
    M w = mul<false, false>(u, A);
    unsigned nskip = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 1 ? 1 : 0, j = k == 0 ? 1 : 2;     // (0,1), (1,2), (0,2)
        const double a0 = w.e[i][i].re + w.e[j][j].re, a1 = w.e[i][j].im + w.e[j][i].im;
        const double a2 = w.e[i][j].re - w.e[j][i].re, a3 = w.e[i][i].im - w.e[j][j].im;
        const double kn = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
        if (!(kn > 0.0)) continue;
        const double vd[4] = {a0 / kn, -a1 / kn, -a2 / kn, -a3 / kn};   // Q(a/k)^dag
        double r[4];
        if (KIND == LGF_WILSON_HEATBATH) {
            double x0;
            if (!sample_x0(beta * kn / 3.0, seed, (uint64_t)l, sweep, (uint64_t)k, x0)) {
                ++nskip;
                continue;
            }
            double u6[4];
            uniforms4(seed, (uint64_t)l, sweep, (uint64_t)k + 4, 0, u6);
            const double ct = 2.0 * u6[0] - 1.0, st = sqrt(1.0 - ct * ct), ph = 2.0 * M_PI * u6[1];
            const double rad = sqrt(1.0 - x0 * x0);
            const double X[4] = {x0, rad * st * cos(ph), rad * st * sin(ph), rad * ct};
            qmul(X, vd, r);
        } else {
            qmul(vd, vd, r);
        }
        rotate_rows(u, i, j, r);
        rotate_rows(w, i, j, r);
    }
    project_su3(u);
    store_eo(E, Vh, s, mu, par, u);
    if (nskip) atomicAdd(skipped, (unsigned long long)nskip);
}

__device__ __forceinline__ int parity_of(const WGeo& g, int64_t s)
{
    int p = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        p += (int)(s % g.L[m]);
        s /= g.L[m];
    }
    return p & 1;
}

// All links 1 (even-odd layout).
__global__ void k_wilson_cold(WGeo g, double2* __restrict__ E)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= g.V * 4) return;
    const int64_t s = l >> 2;
    const int mu = (int)(l & 3);
    M m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.e[i][j] = Cx{i == j ? 1.0 : 0.0, 0.0};
    store_eo(E, g.V / 2, s, mu, parity_of(g, s), m);
}

// Canonical links U <-> even-odd links E, one thread per link.
template <bool TO_EO>
__global__ void k_wilson_layout(WGeo g, double* __restrict__ U, double2* __restrict__ E)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= g.V * 4) return;
    const int64_t s = l >> 2;
    const int mu = (int)(l & 3), par = parity_of(g, s);
    if (TO_EO) store_eo(E, g.V / 2, s, mu, par, load_link(U, l));
    else store_link(U, l, load_eo(E, g.V / 2, s, mu, par));
}

// Per block: the sum over its sites (one per thread) of the six plaquettes'
// Re Tr, in a fixed order; partial[block].
__global__ void __launch_bounds__(256) k_wilson_plaquette(WGeo g, const double2* __restrict__ E,
                                                          double* __restrict__ partial)
{
    const int64_t Vh = g.V / 2;
    __shared__ double red[256];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (s < g.V) {
        int64_t r = s;
        int c[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            c[m] = (int)(r % g.L[m]);
            r /= g.L[m];
        }
        const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu) {
                int q[4] = {c[0], c[1], c[2], c[3]};
                q[mu] = (q[mu] + 1) % g.L[mu];
                const int64_t xm = site_of(g, q[0], q[1], q[2], q[3]);
                q[mu] = c[mu];
                q[nu] = (q[nu] + 1) % g.L[nu];
                const int64_t xn = site_of(g, q[0], q[1], q[2], q[3]);
                const M a = load_eo(E, Vh, s, mu, par), b = load_eo(E, Vh, xm, nu, par ^ 1);
                const M ab = mul<false, false>(a, b);
                const M cc = load_eo(E, Vh, xn, mu, par ^ 1);
                const M abc = mul<false, true>(ab, cc);
                const M d = load_eo(E, Vh, s, nu, par);
                // Re Tr(abc d^dag) = sum_ij Re(abc_ij conj(d_ij))
                double tr = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) tr += abc.e[i][j].re * d.e[i][j].re + abc.e[i][j].im * d.e[i][j].im;
                acc += tr;
            }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block: the partials in a fixed order, then / (18 V).
__global__ void __launch_bounds__(256) k_wilson_plaquette_final(const double* __restrict__ partial, int64_t n,
                                                                int64_t V, double* __restrict__ out)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a += partial[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / (18.0 * (double)V);
}

}  // namespace lgfw

using namespace lgfw;

struct lgf_wilson_gen : lgf::rt::Runner {
    WGeo g{};
    double beta = 0.0;
    uint64_t seed = 0;
    uint64_t next_sweep = 0;
    double* U = nullptr;      // canonical links, for load, store and hand-off
    double2* E = nullptr;     // even-odd links, what the sweeps work on
    bool canon = true;        // U holds the links of E
    double* partial = nullptr;
    double* out = nullptr;
    unsigned long long* skipped = nullptr;
    int64_t nblk_plaq = 0;
};

namespace {

int32_t sync(lgf_wilson_gen* w)
{
    HIPCHK(w, hipStreamSynchronize(w->stream));
    lgf::rt::prof_collect(w);
    return LGF_OK;
}

int32_t sweep_once(lgf_wilson_gen* w, int kind)
{
    const int64_t n = w->g.V / 2;
    const dim3 grid((unsigned)lgf::rt::blocks_for(n, 256)), block(256);
    const uint64_t num = kind == LGF_WILSON_HEATBATH ? w->next_sweep : 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
            if (kind == LGF_WILSON_HEATBATH)
                TRY(lgf::rt::launch(w, lgf::rt::K_HEATBATH, k_wilson_links<LGF_WILSON_HEATBATH>, grid, block, 0, w->g,
                                    w->E, w->beta, w->seed, num, mu, p, w->skipped));
            else
                TRY(lgf::rt::launch(w, lgf::rt::K_OVERRELAX, k_wilson_links<LGF_WILSON_OVERRELAX>, grid, block, 0,
                                    w->g, w->E, w->beta, w->seed, num, mu, p, w->skipped));
        }
    w->canon = false;
    if (kind == LGF_WILSON_HEATBATH) ++w->next_sweep;
    return LGF_OK;
}

int32_t cold(lgf_wilson_gen* w)
{
    const int64_t nl = w->g.V * 4;
    TRY(lgf::rt::launch(w, lgf::rt::K_LOAD, k_wilson_cold, dim3((unsigned)lgf::rt::blocks_for(nl, 256)), dim3(256), 0,
                        w->g, w->E));
    w->canon = false;
    w->next_sweep = 0;
    return sync(w);
}

// Rewrites U from E when a sweep or cold start has changed the links.
int32_t to_canonical(lgf_wilson_gen* w)
{
    if (w->canon) return LGF_OK;
    const int64_t nl = w->g.V * 4;
    TRY(lgf::rt::launch(w, lgf::rt::K_STORE, k_wilson_layout<false>, dim3((unsigned)lgf::rt::blocks_for(nl, 256)),
                        dim3(256), 0, w->g, w->U, w->E));
    TRY(sync(w));
    w->canon = true;
    return LGF_OK;
}

void release(lgf_wilson_gen* w)
{
    for (void* p : {(void*)w->U, (void*)w->E, (void*)w->partial, (void*)w->out, (void*)w->skipped})
        if (p) (void)hipFree(p);
    lgf::rt::release_events(w);
    if (w->stream) (void)hipStreamDestroy(w->stream);
}

}  // namespace

extern "C" {

int32_t lgf_wilson_create(const int32_t dims[4], double beta, uint64_t seed, lgf_wilson_t* out)
{
    if (!dims || !out) return fail(nullptr, LGF_E_INVALID_ARG, "dims and out must not be NULL");
    *out = nullptr;
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(nullptr, LGF_E_INVALID_ARG, "beta must be finite and >= 0");
    int64_t V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || dims[m] > 1024 || (dims[m] & 1))
            return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "every extent must be even and in [2, 1024]");
        V *= dims[m];
    }
    if (V > (int64_t(1) << 31)) return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "at most 2^31 sites");
    lgf_wilson_gen* w = new (std::nothrow) lgf_wilson_gen();
    if (!w) return fail(nullptr, LGF_E_OUT_OF_MEMORY, "host allocation failed");
    for (int m = 0; m < 4; ++m) w->g.L[m] = dims[m];
    w->g.V = V;
    w->beta = beta;
    w->seed = seed;
    w->nblk_plaq = lgf::rt::blocks_for(V, 256);
    int32_t rc = LGF_OK;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == LGF_OK)
            rc = fail(nullptr, e == hipErrorOutOfMemory ? LGF_E_OUT_OF_MEMORY : LGF_E_DEVICE,
                      std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    chk(hipMalloc(&w->U, sizeof(double) * 72 * (size_t)V), "hipMalloc(links)");
    chk(hipMalloc(&w->E, sizeof(double2) * 4 * kEoElems * (size_t)V), "hipMalloc(even-odd links)");
    chk(hipMalloc(&w->partial, sizeof(double) * (size_t)w->nblk_plaq), "hipMalloc(partial)");
    chk(hipMalloc(&w->out, sizeof(double)), "hipMalloc(out)");
    chk(hipMalloc(&w->skipped, sizeof(unsigned long long)), "hipMalloc(counter)");
    if (rc == LGF_OK) chk(hipMemsetAsync(w->skipped, 0, sizeof(unsigned long long), w->stream), "hipMemsetAsync");
    if (rc == LGF_OK) {
        rc = cold(w);
        if (rc != LGF_OK) lgf::rt::g_noctx_err = w->err;
    }
    if (rc != LGF_OK) {
        release(w);
        delete w;
        return rc;
    }
    *out = w;
    return LGF_OK;
}

int32_t lgf_wilson_destroy(lgf_wilson_t w)
{
    if (!w) return LGF_E_INVALID_ARG;
    (void)hipStreamSynchronize(w->stream);
    release(w);
    delete w;
    return LGF_OK;
}

int32_t lgf_wilson_cold(lgf_wilson_t w)
{
    if (!w) return LGF_E_INVALID_ARG;
    return cold(w);
}

int32_t lgf_wilson_load(lgf_wilson_t w, const void* links, int32_t where)
{
    if (!w) return LGF_E_INVALID_ARG;
    if (!links || (where != LGF_HOST && where != LGF_DEVICE))
        return fail(w, LGF_E_INVALID_ARG, "links must not be NULL; where is LGF_HOST or LGF_DEVICE");
    const int64_t nl = w->g.V * 4;
    HIPCHK(w, hipMemcpyAsync(w->U, links, sizeof(double) * 72 * (size_t)w->g.V,
                             where == LGF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, w->stream));
    TRY(lgf::rt::launch(w, lgf::rt::K_LOAD, k_wilson_layout<true>, dim3((unsigned)lgf::rt::blocks_for(nl, 256)),
                        dim3(256), 0, w->g, w->U, w->E));
    w->canon = true;
    return sync(w);
}

int32_t lgf_wilson_sweep(lgf_wilson_t w, int32_t kind)
{
    if (!w) return LGF_E_INVALID_ARG;
    if (kind != LGF_WILSON_HEATBATH && kind != LGF_WILSON_OVERRELAX)
        return fail(w, LGF_E_INVALID_ARG, "kind is LGF_WILSON_HEATBATH or LGF_WILSON_OVERRELAX");
    TRY(sweep_once(w, kind));
    return sync(w);
}

int32_t lgf_wilson_update(lgf_wilson_t w, int64_t n_update, int32_t n_or)
{
    if (!w) return LGF_E_INVALID_ARG;
    if (n_update < 0 || n_or < 0) return fail(w, LGF_E_INVALID_ARG, "n_update and n_or must be >= 0");
    for (int64_t n = 0; n < n_update; ++n) {
        TRY(sweep_once(w, LGF_WILSON_HEATBATH));
        for (int o = 0; o < n_or; ++o) TRY(sweep_once(w, LGF_WILSON_OVERRELAX));
        if ((n & 15) == 15) TRY(sync(w));   // bounds the queue and the pending profile events
    }
    return sync(w);
}

int32_t lgf_wilson_get_sweep(lgf_wilson_t w, uint64_t* n)
{
    if (!w || !n) return LGF_E_INVALID_ARG;
    *n = w->next_sweep;
    return LGF_OK;
}

int32_t lgf_wilson_set_sweep(lgf_wilson_t w, uint64_t n)
{
    if (!w) return LGF_E_INVALID_ARG;
    w->next_sweep = n;
    return LGF_OK;
}

int32_t lgf_wilson_plaquette(lgf_wilson_t w, double* plaq)
{
    if (!w || !plaq) return LGF_E_INVALID_ARG;
    TRY(lgf::rt::launch(w, lgf::rt::K_PLAQUETTE, k_wilson_plaquette, dim3((unsigned)w->nblk_plaq), dim3(256), 0, w->g,
                        (const double2*)w->E, w->partial));
    TRY(lgf::rt::launch(w, lgf::rt::K_PLAQUETTE, k_wilson_plaquette_final, dim3(1), dim3(256), 0,
                        (const double*)w->partial, w->nblk_plaq, w->g.V, w->out));
    HIPCHK(w, hipMemcpyAsync(plaq, w->out, sizeof(double), hipMemcpyDeviceToHost, w->stream));
    return sync(w);
}

int32_t lgf_wilson_store(lgf_wilson_t w, void* links, int32_t where)
{
    if (!w) return LGF_E_INVALID_ARG;
    if (!links || (where != LGF_HOST && where != LGF_DEVICE))
        return fail(w, LGF_E_INVALID_ARG, "links must not be NULL; where is LGF_HOST or LGF_DEVICE");
    TRY(to_canonical(w));
    HIPCHK(w, hipMemcpyAsync(links, w->U, sizeof(double) * 72 * (size_t)w->g.V,
                             where == LGF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, w->stream));
    return sync(w);
}

const void* lgf_wilson_device_links(lgf_wilson_t w)
{
    if (!w) return nullptr;
    return to_canonical(w) == LGF_OK ? w->U : nullptr;
}

int32_t lgf_wilson_skipped(lgf_wilson_t w, int64_t* n)
{
    if (!w || !n) return LGF_E_INVALID_ARG;
    unsigned long long v = 0;
    HIPCHK(w, hipMemcpyAsync(&v, w->skipped, sizeof v, hipMemcpyDeviceToHost, w->stream));
    TRY(sync(w));
    *n = (int64_t)v;
    return LGF_OK;
}

const char* lgf_wilson_last_error(lgf_wilson_t w) { return w ? w->err.c_str() : lgf::rt::g_noctx_err.c_str(); }

}  // extern "C"
