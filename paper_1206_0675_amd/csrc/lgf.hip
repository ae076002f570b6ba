// Host runtime and C ABI (include/lgf.h) of the gauge-fixing library.
//
// A context owns, per arithmetic precision T in use:
//   U[2]  links, structure of arrays, NE complex per link (ping-pong: the
//         transform reads U[cur] and writes U[1-cur]; the neighbour reads of
//         the fused kernel need the old links intact)
//   g     the gauge transformation of the iteration in flight
//   D     the packed Delta field (4 complex per site) in the tiled layout
//   G     the accumulated gauge (when tracked)
//   tw    FFT twiddles W_L^k for the four extents
// plus FP64 tables of the lattice momenta, the per-plane partial sums, and a
// small device state (iteration, F, theta, stop flag, current buffer) that
// the host reads back only at poll points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lgf.h"

using namespace lgf;

namespace {

enum KernelId {
    K_LOAD, K_STORE, K_MEASURE, K_TRANSFORM_MEASURE, K_ZT, K_GAUGE, K_REDUCE, K_FIELD, K_SWITCH, K_STATE, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {"load",   "store",  "measure", "transform_measure", "zt_fft_scale",
                                           "gauge",  "reduce", "field",   "precision_switch",  "state"};

constexpr size_t kMaxLds = 160 * 1024;
constexpr size_t kMaxLdsZt = 128 * 1024;

template <typename T>
struct Bufs {
    C2<T>* U[2] = {nullptr, nullptr};
    C2<T>* g = nullptr;
    C2<T>* D = nullptr;
    C2<T>* G = nullptr;
    C2<T>* tw = nullptr;     // Lx + Ly + Lz + Lt entries
    Geo geo{};
    int tw_off[4] = {0, 0, 0, 0};
};

struct Pending {
    int k;
    hipEvent_t a, b;
};

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

}  // namespace

// small kernels on the device state (no memset: safe inside graphs)
__global__ void k_state_init(DevState* st)
{
    st->iter = 0;
    st->F = 0.0;
    st->theta = 0.0;
    st->theta_stop = -1.0;
    st->done = 0;
    st->nonfinite = 0;
}

__global__ void k_state_stop(DevState* st, double theta_stop, int valid)
{
    st->theta_stop = theta_stop;
    st->nonfinite = 0;
    st->done = (valid && st->theta < theta_stop) ? 1 : 0;
}

struct lgf_context {
    lgf_params p{};
    int NE = 9;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int phase = 1;            // 1: FP64 arithmetic, 0: FP32
    bool use64 = false, use32 = false;
    bool track = false;
    bool loaded = false;
    bool delta_valid = false; // D and the state hold Delta, F, theta of the current links
    int cur = 0;              // links are in U[cur] (mirrors the device-side update parity)
    Bufs<double> d;
    Bufs<float> f;
    C2<double>* U0 = nullptr; // LGF_MIXED: the links as loaded, FP64
    double* ptab = nullptr;
    double* partial = nullptr;
    DevState* st = nullptr;
    DevState* st_host = nullptr;
    unsigned long long* check = nullptr;
    double* trace_dev = nullptr;
    int64_t trace_cap = 0;
    int64_t iter_fp32 = 0;    // updates done in FP32 before the switch
    int64_t bytes = 0;
    double c0 = 0.0;          // (alpha/2) p2max / V
    int nth_plane = 256;
    int lmax = 64;            // longest axis rounded up to 64 or 128 (kernel variant)
    std::string err;
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;
    int64_t prof_n[K_COUNT] = {};
    double prof_ms[K_COUNT] = {};
};

namespace {

thread_local std::string g_noctx_err;

int32_t fail(lgf_context* c, int32_t code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_noctx_err = msg;
    return code;
}

#define HIPCHK(c, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((c), e_ == hipErrorOutOfMemory ? LGF_E_OUT_OF_MEMORY : LGF_E_DEVICE,      \
                        std::string(#call) + ": " + hipGetErrorString(e_));                      \
    } while (0)

template <typename T>
Bufs<T>& bufs(lgf_context* c);
template <>
Bufs<double>& bufs<double>(lgf_context* c) { return c->d; }
template <>
Bufs<float>& bufs<float>(lgf_context* c) { return c->f; }

hipEvent_t take_event(lgf_context* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_collect(lgf_context* c)
{
    for (auto& pe : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            c->prof_n[pe.k] += 1;
            c->prof_ms[pe.k] += ms;
        }
        c->ev_pool.push_back(pe.a);
        c->ev_pool.push_back(pe.b);
    }
    c->pending.clear();
}

template <typename K, typename... Args>
int32_t launch(lgf_context* c, int kid, K kernel, dim3 grid, dim3 block, size_t lds, Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->p.profile) {
        a = take_event(c);
        b = take_event(c);
        if (a) (void)hipEventRecord(a, c->stream);
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, c->stream, args...);
    hipError_t e = hipGetLastError();
    if (c->p.profile && a && b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back(Pending{kid, a, b});
    }
    if (e != hipSuccess) return fail(c, LGF_E_DEVICE, std::string("launch of ") + kKernelNames[kid] + ": " + hipGetErrorString(e));
    return LGF_OK;
}

#define TRY(expr)                          \
    do {                                   \
        int32_t r_ = (expr);               \
        if (r_ != LGF_OK) return r_;       \
    } while (0)

int32_t sync_state(lgf_context* c)
{
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->p.profile) prof_collect(c);
    return LGF_OK;
}

int32_t set_stop(lgf_context* c, double theta_stop)
{
    return launch(c, K_STATE, k_state_stop, dim3(1), dim3(1), 0, c->st, theta_stop, c->delta_valid ? 1 : 0);
}

// ----------------------------------------------------------------------------
// geometry and tables
// ----------------------------------------------------------------------------
template <typename T>
Geo make_geo(const int32_t* dims)
{
    Geo g{};
    for (int m = 0; m < 4; ++m) {
        g.L[m] = dims[m];
        g.logL[m] = ilog2(dims[m]);
    }
    g.NP = dims[0] * dims[1];
    g.logNP = ilog2(g.NP);
    g.NQ = dims[2] * dims[3];
    g.logNQ = ilog2(g.NQ);
    g.V = (int64_t)g.NP * g.NQ;
    // runs of 64 bytes where the (z, t) block still fits its LDS budget
    int W = (int)(64 / sizeof(C2<T>));
    if (W > g.NP) W = g.NP;
    while (W > 1 && (size_t)W * g.NQ * sizeof(C2<T>) > kMaxLdsZt) W >>= 1;
    g.W = W;
    g.logW = ilog2(W);
    return g;
}

template <typename T>
bool shape_fits(const int32_t* dims, int nth)
{
    const size_t np = (size_t)dims[0] * dims[1], nq = (size_t)dims[2] * dims[3];
    if (4 * np * sizeof(C2<T>) + 2 * nth * sizeof(double) > kMaxLds) return false;
    if (nq * sizeof(C2<T>) > kMaxLdsZt) return false;
    return true;
}

template <typename T>
int32_t alloc_bufs(lgf_context* c, Bufs<T>& b)
{
    const int32_t* dims = c->p.dims;
    b.geo = make_geo<T>(dims);
    const int64_t V = b.geo.V;
    const size_t link = sizeof(C2<T>) * (size_t)4 * c->NE * V;
    const size_t field = sizeof(C2<T>) * (size_t)c->NE * V;
    HIPCHK(c, hipMalloc(&b.U[0], link));
    HIPCHK(c, hipMalloc(&b.U[1], link));
    HIPCHK(c, hipMalloc(&b.g, field));
    HIPCHK(c, hipMalloc(&b.D, sizeof(C2<T>) * (size_t)4 * V));
    c->bytes += 2 * link + field + sizeof(C2<T>) * 4 * V;
    if (c->track) {
        HIPCHK(c, hipMalloc(&b.G, field));
        c->bytes += field;
    }
    std::vector<C2<T>> tw;
    for (int m = 0; m < 4; ++m) {
        b.tw_off[m] = (int)tw.size();
        for (int k = 0; k < dims[m]; ++k) {
            const double a = -2.0 * M_PI * (double)k / (double)dims[m];
            tw.push_back(mk<T>((T)std::cos(a), (T)std::sin(a)));
        }
    }
    HIPCHK(c, hipMalloc(&b.tw, sizeof(C2<T>) * tw.size()));
    HIPCHK(c, hipMemcpy(b.tw, tw.data(), sizeof(C2<T>) * tw.size(), hipMemcpyHostToDevice));
    return LGF_OK;
}

template <typename T>
void free_bufs(Bufs<T>& b)
{
    (void)hipFree(b.U[0]);
    (void)hipFree(b.U[1]);
    (void)hipFree(b.g);
    (void)hipFree(b.D);
    (void)hipFree(b.G);
    (void)hipFree(b.tw);
    b = Bufs<T>();
}

template <typename T, int NE, int LMAX>
int32_t set_lds_attrs(lgf_context* c)
{
    const Geo& g = bufs<T>(c).geo;
    const int mlds = (int)(4 * g.NP * sizeof(C2<T>) + 2 * c->nth_plane * sizeof(double));
    const int glds = (int)(4 * g.NP * sizeof(C2<T>));
    const int zlds = (int)((size_t)g.NQ * g.W * sizeof(C2<T>));
    HIPCHK(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_measure<T, NE, false, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, mlds));
    HIPCHK(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_measure<T, NE, true, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, mlds));
    HIPCHK(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gauge<T, NE, false, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, glds));
    HIPCHK(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gauge<T, NE, true, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, glds));
    HIPCHK(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zt<T, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, zlds));
    return LGF_OK;
}

// ----------------------------------------------------------------------------
// one iteration, enqueued
// ----------------------------------------------------------------------------
// Delta, F, theta of U[cur] with no update (the first line of Algorithm 1).
template <typename T, int NE, int LMAX>
int32_t enqueue_measure(lgf_context* c, double* trace_slot)
{
    Bufs<T>& b = bufs<T>(c);
    const Geo& g = b.geo;
    const size_t lds = 4 * g.NP * sizeof(C2<T>) + 2 * c->nth_plane * sizeof(double);
    TRY(launch(c, K_MEASURE, k_measure<T, NE, false, LMAX>, dim3(g.NQ), dim3(c->nth_plane), lds, g,
               (const C2<T>*)b.U[c->cur], (C2<T>*)nullptr, (const C2<T>*)nullptr, b.D, c->partial,
               (const C2<T>*)(b.tw + b.tw_off[0]), (const C2<T>*)(b.tw + b.tw_off[1]), (const DevState*)c->st));
    TRY(launch(c, K_REDUCE, k_reduce, dim3(1), dim3(256), 0, (const double*)c->partial, g.NQ, g.V, c->st,
               trace_slot, 0));
    c->delta_valid = true;
    return LGF_OK;
}

// filter, g, transform, Delta/F/theta of the new links (the loop body of
// Algorithm 1).  The update flips cur; when the device stop flag is set the
// kernels do nothing and the host learns the real parity at the next poll.
template <typename T, int NE, int LMAX>
int32_t enqueue_update(lgf_context* c, double* trace_slot)
{
    Bufs<T>& b = bufs<T>(c);
    const Geo& g = b.geo;
    const size_t zlds = (size_t)g.NQ * g.W * sizeof(C2<T>);
    const size_t glds = 4 * g.NP * sizeof(C2<T>);
    const size_t mlds = glds + 2 * c->nth_plane * sizeof(double);
    const C2<T>* twx = b.tw + b.tw_off[0];
    const C2<T>* twy = b.tw + b.tw_off[1];
    TRY(launch(c, K_ZT, k_zt<T, LMAX>, dim3((g.NP / g.W) * 4), dim3(512), zlds, g, b.D,
               (const C2<T>*)(b.tw + b.tw_off[2]), (const C2<T>*)(b.tw + b.tw_off[3]), (const double*)c->ptab,
               c->c0, (int)(c->p.accel == LGF_ACCEL_FOURIER), (const DevState*)c->st));
    if (c->track)
        TRY(launch(c, K_GAUGE, k_gauge<T, NE, true, LMAX>, dim3(g.NQ), dim3(c->nth_plane), glds, g, (const C2<T>*)b.D, b.g,
                   b.G, twx, twy, (const DevState*)c->st));
    else
        TRY(launch(c, K_GAUGE, k_gauge<T, NE, false, LMAX>, dim3(g.NQ), dim3(c->nth_plane), glds, g, (const C2<T>*)b.D, b.g,
                   b.G, twx, twy, (const DevState*)c->st));
    TRY(launch(c, K_TRANSFORM_MEASURE, k_measure<T, NE, true, LMAX>, dim3(g.NQ), dim3(c->nth_plane), mlds, g,
               (const C2<T>*)b.U[c->cur], b.U[1 - c->cur], (const C2<T>*)b.g, b.D, c->partial, twx, twy,
               (const DevState*)c->st));
    TRY(launch(c, K_REDUCE, k_reduce, dim3(1), dim3(256), 0, (const double*)c->partial, g.NQ, g.V, c->st,
               trace_slot, 1));
    c->cur ^= 1;
    return LGF_OK;
}

// Kernel variant for the current phase, storage and longest lattice axis.
template <template <typename, int, int> class OP, typename... A>
int32_t dispatch(lgf_context* c, A... args)
{
    const bool big = c->lmax > 64;
    if (c->phase == 1) {
        if (c->NE == 9) return big ? OP<double, 9, 128>::run(c, args...) : OP<double, 9, 64>::run(c, args...);
        return big ? OP<double, 6, 128>::run(c, args...) : OP<double, 6, 64>::run(c, args...);
    }
    if (c->NE == 9) return big ? OP<float, 9, 128>::run(c, args...) : OP<float, 9, 64>::run(c, args...);
    return big ? OP<float, 6, 128>::run(c, args...) : OP<float, 6, 64>::run(c, args...);
}

template <typename T, int NE, int LMAX>
struct OpMeasure {
    static int32_t run(lgf_context* c, double* tr) { return enqueue_measure<T, NE, LMAX>(c, tr); }
};
template <typename T, int NE, int LMAX>
struct OpUpdate {
    static int32_t run(lgf_context* c, double* tr) { return enqueue_update<T, NE, LMAX>(c, tr); }
};

int32_t measure_any(lgf_context* c, double* trace_slot) { return dispatch<OpMeasure>(c, trace_slot); }
int32_t update_any(lgf_context* c, double* trace_slot) { return dispatch<OpUpdate>(c, trace_slot); }

// After a poll: the number of updates that really ran fixes the parity.
void resync_cur(lgf_context* c, int64_t iter_before, int cur_before)
{
    const int64_t ran = c->st_host->iter - iter_before;
    c->cur = (int)((cur_before + ran) & 1);
}

int64_t blocks_for(int64_t n, int per) { return (n + per - 1) / per; }

template <typename T, int NE>
int32_t enqueue_store(lgf_context* c, double* dst)
{
    Bufs<T>& b = bufs<T>(c);
    return launch(c, K_STORE, k_store<T, NE>, dim3((unsigned)blocks_for(4 * b.geo.V, 256)), dim3(256), 0,
                  b.geo.V, (const C2<T>*)b.U[c->cur], dst);
}

int32_t store_any(lgf_context* c, double* dst)
{
    if (c->phase == 1) return c->NE == 9 ? enqueue_store<double, 9>(c, dst) : enqueue_store<double, 6>(c, dst);
    return c->NE == 9 ? enqueue_store<float, 9>(c, dst) : enqueue_store<float, 6>(c, dst);
}

template <typename T, int NE>
int32_t enqueue_load(lgf_context* c, const double* src, C2<T>* U)
{
    const int64_t V = bufs<T>(c).geo.V;
    return launch(c, K_LOAD, k_load<T, NE>, dim3((unsigned)blocks_for(4 * V, 256)), dim3(256), 0, V, src, U,
                  c->check);
}

template <typename T>
int32_t enqueue_identity_G(lgf_context* c)
{
    Bufs<T>& b = bufs<T>(c);
    if (!b.G) return LGF_OK;
    const int64_t V = b.geo.V;
    if (c->NE == 9)
        return launch(c, K_FIELD, k_field_identity<T, 9>, dim3((unsigned)blocks_for(V, 256)), dim3(256), 0, V, b.G);
    return launch(c, K_FIELD, k_field_identity<T, 6>, dim3((unsigned)blocks_for(V, 256)), dim3(256), 0, V, b.G);
}

// LGF_MIXED: leave FP32.  G64 = reunit(G32); U64 = G64 U0 G64^dag(x+mu).
template <int NE>
int32_t enqueue_switch(lgf_context* c)
{
    const Geo& g = c->d.geo;
    TRY(launch(c, K_SWITCH, k_promote_gauge<NE>, dim3((unsigned)blocks_for(g.V, 256)), dim3(256), 0, g.V,
               (const C2<float>*)c->f.G, c->d.G));
    TRY(launch(c, K_SWITCH, k_switch<NE>, dim3((unsigned)blocks_for(4 * g.V, 256)), dim3(256), 0, g,
               (const C2<double>*)c->U0, (const C2<double>*)c->d.G, c->d.U[0]));
    return LGF_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void fill_stats(lgf_context* c, lgf_stats* out, int32_t status, double t0)
{
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->iter = c->st_host->iter;
    if (c->p.precision == LGF_MIXED) {
        out->iter_fp32 = c->phase == 0 ? out->iter : c->iter_fp32;
        out->iter_fp64 = out->iter - out->iter_fp32;
    } else if (c->p.precision == LGF_FP32) {
        out->iter_fp32 = out->iter;
    } else {
        out->iter_fp64 = out->iter;
    }
    out->F = c->st_host->F;
    out->theta = c->st_host->theta;
    out->seconds = t0 > 0 ? now_s() - t0 : 0.0;
    out->phase = c->phase;
    out->status = status;
}

int32_t check_ctx(lgf_context* c, bool need_loaded)
{
    if (!c) return LGF_E_INVALID_ARG;
    if (need_loaded && !c->loaded) return fail(c, LGF_E_STATE, "no links loaded");
    return LGF_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

int32_t lgf_default_params(lgf_params* p)
{
    if (!p) return LGF_E_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    p->precision = LGF_FP64;
    p->storage = LGF_STORE18;
    p->step = LGF_STEP_PLAIN;
    p->accel = LGF_ACCEL_FOURIER;
    p->alpha = 0.08;
    p->theta_stop = 1e-15;
    p->theta_switch = 1e-6;
    p->unit_tol = 1e-12;
    p->max_iter = 100000;
    p->poll_every = 16;
    return LGF_OK;
}

const char* lgf_strerror(int32_t code)
{
    switch (code) {
    case LGF_OK: return "ok";
    case LGF_E_INVALID_ARG: return "invalid argument";
    case LGF_E_UNSUPPORTED_SHAPE: return "unsupported lattice shape";
    case LGF_E_OUT_OF_MEMORY: return "out of device memory";
    case LGF_E_DEVICE: return "HIP runtime error";
    case LGF_E_NOT_UNITARY: return "link not in SU(3) within tolerance";
    case LGF_E_NONFINITE: return "non-finite value";
    case LGF_E_NOT_CONVERGED: return "max_iter reached before theta < theta_stop";
    case LGF_E_STATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

const char* lgf_last_error(lgf_ctx ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

const char* lgf_kernel_name(int32_t k) { return (k >= 0 && k < K_COUNT) ? kKernelNames[k] : nullptr; }

int32_t lgf_validate_links(const int32_t dims[4], const double* links, double tol, int64_t* first_bad)
{
    if (first_bad) *first_bad = -1;
    if (!dims || !links) return LGF_E_INVALID_ARG;
    int64_t V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 1) return LGF_E_INVALID_ARG;
        V *= dims[m];
    }
    for (int64_t li = 0; li < 4 * V; ++li) {
        const double* a = links + li * 18;
        for (int k = 0; k < 18; ++k)
            if (!std::isfinite(a[k])) {
                if (first_bad) *first_bad = li;
                return LGF_E_NONFINITE;
            }
        double worst = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double re = (i == j) ? -1.0 : 0.0, im = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double ar = a[(3 * i + k) * 2], ai = a[(3 * i + k) * 2 + 1];
                    const double br = a[(3 * j + k) * 2], bi = a[(3 * j + k) * 2 + 1];
                    re += ar * br + ai * bi;   // a_ik conj(a_jk)
                    im += ai * br - ar * bi;
                }
                worst = std::fmax(worst, std::sqrt(re * re + im * im));
            }
        auto el = [&](int i, int j, int c) { return a[(3 * i + j) * 2 + c]; };
        auto cm = [](double ar, double ai, double br, double bi, double& r, double& i) {
            r = ar * br - ai * bi;
            i = ar * bi + ai * br;
        };
        double m1r, m1i, m2r, m2i, t1r, t1i, t2r, t2i, t3r, t3i;
        cm(el(1, 1, 0), el(1, 1, 1), el(2, 2, 0), el(2, 2, 1), m1r, m1i);
        cm(el(1, 2, 0), el(1, 2, 1), el(2, 1, 0), el(2, 1, 1), m2r, m2i);
        cm(el(0, 0, 0), el(0, 0, 1), m1r - m2r, m1i - m2i, t1r, t1i);
        cm(el(1, 0, 0), el(1, 0, 1), el(2, 2, 0), el(2, 2, 1), m1r, m1i);
        cm(el(1, 2, 0), el(1, 2, 1), el(2, 0, 0), el(2, 0, 1), m2r, m2i);
        cm(el(0, 1, 0), el(0, 1, 1), m1r - m2r, m1i - m2i, t2r, t2i);
        cm(el(1, 0, 0), el(1, 0, 1), el(2, 1, 0), el(2, 1, 1), m1r, m1i);
        cm(el(1, 1, 0), el(1, 1, 1), el(2, 0, 0), el(2, 0, 1), m2r, m2i);
        cm(el(0, 2, 0), el(0, 2, 1), m1r - m2r, m1i - m2i, t3r, t3i);
        const double dr = t1r - t2r + t3r - 1.0, di = t1i - t2i + t3i;
        worst = std::fmax(worst, std::sqrt(dr * dr + di * di));
        if (worst > tol) {
            if (first_bad) *first_bad = li;
            return LGF_E_NOT_UNITARY;
        }
    }
    return LGF_OK;
}

int32_t lgf_create(const lgf_params* p, lgf_ctx* out)
{
    if (!p || !out) return fail(nullptr, LGF_E_INVALID_ARG, "NULL params or output");
    *out = nullptr;
    if (p->precision != LGF_FP64 && p->precision != LGF_FP32 && p->precision != LGF_MIXED)
        return fail(nullptr, LGF_E_INVALID_ARG, "precision must be LGF_FP64, LGF_FP32 or LGF_MIXED");
    if (p->storage != LGF_STORE18 && p->storage != LGF_STORE12)
        return fail(nullptr, LGF_E_INVALID_ARG, "storage must be LGF_STORE18 or LGF_STORE12");
    if (p->step != LGF_STEP_PLAIN) return fail(nullptr, LGF_E_INVALID_ARG, "unknown step kind");
    if (p->accel != LGF_ACCEL_FOURIER && p->accel != LGF_ACCEL_NONE)
        return fail(nullptr, LGF_E_INVALID_ARG, "accel must be LGF_ACCEL_FOURIER or LGF_ACCEL_NONE");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(nullptr, LGF_E_INVALID_ARG, "alpha must be > 0");
    if (!(p->theta_stop >= 0.0) || !(p->theta_switch >= 0.0))
        return fail(nullptr, LGF_E_INVALID_ARG, "theta_stop and theta_switch must be >= 0");
    if (p->max_iter < 0 || p->poll_every < 1) return fail(nullptr, LGF_E_INVALID_ARG, "max_iter >= 0, poll_every >= 1");
    for (int m = 0; m < 4; ++m)
        if (!pow2_in(p->dims[m], 4, 128))
            return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "each extent must be a power of two in [4, 128]");
    const int np = p->dims[0] * p->dims[1];
    const int nth = np < 64 ? 64 : (np > 256 ? 256 : np);
    const bool use64 = p->precision != LGF_FP32, use32 = p->precision != LGF_FP64;
    if ((use64 && !shape_fits<double>(p->dims, nth)) || (use32 && !shape_fits<float>(p->dims, nth)))
        return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "(x, y) or (z, t) plane too large for one workgroup's LDS");

    lgf_context* c = new (std::nothrow) lgf_context();
    if (!c) return fail(nullptr, LGF_E_OUT_OF_MEMORY, "host allocation failed");
    c->p = *p;
    c->NE = p->storage == LGF_STORE12 ? 6 : 9;
    c->use64 = use64;
    c->use32 = use32;
    c->track = p->track_gauge != 0 || p->precision == LGF_MIXED;
    c->phase = use64 && !use32 ? 1 : 0;
    c->nth_plane = nth;
    for (int m = 0; m < 4; ++m)
        if (p->dims[m] > 64) c->lmax = 128;
    int32_t rc = LGF_OK;
    auto bail = [&](int32_t code) {
        std::string msg = c->err;
        lgf_destroy(c);
        g_noctx_err = msg;
        return code;
    };
    if (p->stream) {
        c->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            c->stream = nullptr;
            c->err = "hipStreamCreateWithFlags failed";
            return bail(LGF_E_DEVICE);
        }
        c->own_stream = true;
    }
    if (use64 && (rc = alloc_bufs<double>(c, c->d)) != LGF_OK) return bail(rc);
    if (use32 && (rc = alloc_bufs<float>(c, c->f)) != LGF_OK) return bail(rc);
    const Geo& g = use64 ? c->d.geo : c->f.geo;
    if (p->precision == LGF_MIXED) {
        const size_t link = sizeof(C2<double>) * (size_t)4 * c->NE * g.V;
        if (hipMalloc(&c->U0, link) != hipSuccess) { c->err = "hipMalloc U0"; return bail(LGF_E_OUT_OF_MEMORY); }
        c->bytes += link;
    }
    // momentum tables, indexed by position after the forward transforms:
    // 4 sin^2(pi n / L) for n = mode_of_position(L, pos)
    std::vector<double> pt;
    double p2max = 0.0;
    for (int m = 0; m < 4; ++m) {
        const int L = p->dims[m];
        double best = 0.0;
        for (int pos = 0; pos < L; ++pos) {
            const double s = std::sin(M_PI * (double)mode_of_position(L, pos) / (double)L);
            pt.push_back(4.0 * s * s);
            best = std::fmax(best, 4.0 * s * s);
        }
        p2max += best;
    }
    c->c0 = 0.5 * p->alpha * (p->accel == LGF_ACCEL_FOURIER ? p2max : 1.0) / (double)g.V;
    if (hipMalloc(&c->ptab, sizeof(double) * pt.size()) != hipSuccess) { c->err = "hipMalloc ptab"; return bail(LGF_E_OUT_OF_MEMORY); }
    if (hipMemcpy(c->ptab, pt.data(), sizeof(double) * pt.size(), hipMemcpyHostToDevice) != hipSuccess) {
        c->err = "hipMemcpy ptab";
        return bail(LGF_E_DEVICE);
    }
    if (hipMalloc(&c->partial, sizeof(double) * 2 * g.NQ) != hipSuccess) { c->err = "hipMalloc partial"; return bail(LGF_E_OUT_OF_MEMORY); }
    if (hipMalloc(&c->st, sizeof(DevState)) != hipSuccess) { c->err = "hipMalloc state"; return bail(LGF_E_OUT_OF_MEMORY); }
    if (hipHostMalloc(&c->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        c->st_host = nullptr;
        c->err = "hipHostMalloc state";
        return bail(LGF_E_OUT_OF_MEMORY);
    }
    std::memset(c->st_host, 0, sizeof(DevState));
    if (hipMalloc(&c->check, sizeof(unsigned long long) * 3) != hipSuccess) { c->err = "hipMalloc check"; return bail(LGF_E_OUT_OF_MEMORY); }
    for (int lm : {64, 128}) {
        if (use64) {
            rc = c->NE == 9 ? (lm == 64 ? set_lds_attrs<double, 9, 64>(c) : set_lds_attrs<double, 9, 128>(c))
                            : (lm == 64 ? set_lds_attrs<double, 6, 64>(c) : set_lds_attrs<double, 6, 128>(c));
            if (rc != LGF_OK) return bail(rc);
        }
        if (use32) {
            rc = c->NE == 9 ? (lm == 64 ? set_lds_attrs<float, 9, 64>(c) : set_lds_attrs<float, 9, 128>(c))
                            : (lm == 64 ? set_lds_attrs<float, 6, 64>(c) : set_lds_attrs<float, 6, 128>(c));
            if (rc != LGF_OK) return bail(rc);
        }
    }
    if ((rc = launch(c, K_STATE, k_state_init, dim3(1), dim3(1), 0, c->st)) != LGF_OK) return bail(rc);
    if ((rc = sync_state(c)) != LGF_OK) return bail(rc);
    *out = c;
    return LGF_OK;
}

int32_t lgf_destroy(lgf_ctx c)
{
    if (!c) return LGF_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_bufs(c->d);
    free_bufs(c->f);
    (void)hipFree(c->U0);
    (void)hipFree(c->ptab);
    (void)hipFree(c->partial);
    (void)hipFree(c->st);
    (void)hipFree(c->check);
    (void)hipFree(c->trace_dev);
    if (c->st_host) (void)hipHostFree(c->st_host);
    for (auto& pe : c->pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LGF_OK;
}

int32_t lgf_load_links(lgf_ctx c, const void* links, int32_t where)
{
    TRY(check_ctx(c, false));
    if (!links || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad links/where");
    c->loaded = false;
    c->delta_valid = false;
    const int64_t V = (c->use64 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 72 * (size_t)V;
    double* src = nullptr;
    if (where == LGF_HOST) {
        HIPCHK(c, hipMalloc(&src, nbytes));
        hipError_t e = hipMemcpyAsync(src, links, nbytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(src);
            return fail(c, LGF_E_DEVICE, std::string("hipMemcpyAsync links: ") + hipGetErrorString(e));
        }
    }
    const double* s = where == LGF_HOST ? src : static_cast<const double*>(links);
    int32_t rc = LGF_OK;
    do {
        if (hipMemsetAsync(c->check, 0, sizeof(unsigned long long) * 3, c->stream) != hipSuccess) {
            rc = fail(c, LGF_E_DEVICE, "hipMemsetAsync check");
            break;
        }
        if (c->p.precision == LGF_MIXED) {
            rc = c->NE == 9 ? enqueue_load<double, 9>(c, s, c->U0) : enqueue_load<double, 6>(c, s, c->U0);
            if (rc == LGF_OK) rc = c->NE == 9 ? enqueue_load<float, 9>(c, s, c->f.U[0]) : enqueue_load<float, 6>(c, s, c->f.U[0]);
        } else if (c->p.precision == LGF_FP64) {
            rc = c->NE == 9 ? enqueue_load<double, 9>(c, s, c->d.U[0]) : enqueue_load<double, 6>(c, s, c->d.U[0]);
        } else {
            rc = c->NE == 9 ? enqueue_load<float, 9>(c, s, c->f.U[0]) : enqueue_load<float, 6>(c, s, c->f.U[0]);
        }
        if (rc != LGF_OK) break;
        if (c->use64 && (rc = enqueue_identity_G<double>(c)) != LGF_OK) break;
        if (c->use32 && (rc = enqueue_identity_G<float>(c)) != LGF_OK) break;
        if ((rc = launch(c, K_STATE, k_state_init, dim3(1), dim3(1), 0, c->st)) != LGF_OK) break;
        unsigned long long chk[3] = {0, 0, 0};
        if (hipMemcpyAsync(chk, c->check, sizeof(chk), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            (rc = sync_state(c)) != LGF_OK) {
            if (rc == LGF_OK) rc = fail(c, LGF_E_DEVICE, "reading the validation result");
            break;
        }
        double du, dd;
        std::memcpy(&du, &chk[0], sizeof(double));
        std::memcpy(&dd, &chk[1], sizeof(double));
        if (chk[2] != 0) {
            rc = fail(c, LGF_E_NONFINITE, "non-finite entries in " + std::to_string(chk[2]) + " links");
            break;
        }
        if (c->p.unit_tol > 0.0 && (du > c->p.unit_tol || dd > c->p.unit_tol)) {
            rc = fail(c, LGF_E_NOT_UNITARY, "max |UU^dag-1| = " + std::to_string(du) + ", max |det U-1| = " +
                                                std::to_string(dd));
            break;
        }
    } while (false);
    if (src) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(src);
    }
    if (rc != LGF_OK) return rc;
    c->cur = 0;
    c->phase = c->use64 && !c->use32 ? 1 : 0;
    c->iter_fp32 = 0;
    c->loaded = true;
    return LGF_OK;
}

int32_t lgf_store_links(lgf_ctx c, void* links, int32_t where)
{
    TRY(check_ctx(c, true));
    if (!links || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad links/where");
    const int64_t V = (c->phase == 1 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 72 * (size_t)V;
    if (where == LGF_DEVICE) {
        TRY(store_any(c, static_cast<double*>(links)));
        return sync_state(c);
    }
    double* dst = nullptr;
    HIPCHK(c, hipMalloc(&dst, nbytes));
    int32_t rc = store_any(c, dst);
    if (rc == LGF_OK && hipMemcpyAsync(links, dst, nbytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        rc = fail(c, LGF_E_DEVICE, "hipMemcpyAsync links out");
    if (rc == LGF_OK) rc = sync_state(c);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(dst);
    return rc;
}

int32_t lgf_store_gauge(lgf_ctx c, void* G, int32_t where)
{
    TRY(check_ctx(c, true));
    if (!c->track) return fail(c, LGF_E_STATE, "gauge not tracked (set track_gauge)");
    if (!G || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad G/where");
    const int64_t V = (c->use64 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 18 * (size_t)V;
    double* dst = where == LGF_DEVICE ? static_cast<double*>(G) : nullptr;
    if (!dst) HIPCHK(c, hipMalloc(&dst, nbytes));
    int32_t rc;
    const dim3 grid((unsigned)blocks_for(V, 256));
    if (c->phase == 1)
        rc = c->NE == 9 ? launch(c, K_FIELD, k_field_store<double, 9>, grid, dim3(256), 0, V, (const C2<double>*)c->d.G, dst)
                        : launch(c, K_FIELD, k_field_store<double, 6>, grid, dim3(256), 0, V, (const C2<double>*)c->d.G, dst);
    else
        rc = c->NE == 9 ? launch(c, K_FIELD, k_field_store<float, 9>, grid, dim3(256), 0, V, (const C2<float>*)c->f.G, dst)
                        : launch(c, K_FIELD, k_field_store<float, 6>, grid, dim3(256), 0, V, (const C2<float>*)c->f.G, dst);
    if (rc == LGF_OK && where == LGF_HOST &&
        hipMemcpyAsync(G, dst, nbytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        rc = fail(c, LGF_E_DEVICE, "hipMemcpyAsync G out");
    if (rc == LGF_OK) rc = sync_state(c);
    if (where == LGF_HOST) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(dst);
    }
    return rc;
}

int32_t lgf_load_gauge(lgf_ctx c, const void* G, int32_t where)
{
    TRY(check_ctx(c, true));
    if (!c->track) return fail(c, LGF_E_STATE, "gauge not tracked (set track_gauge)");
    if (!G || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad G/where");
    const int64_t V = (c->use64 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 18 * (size_t)V;
    double* src = where == LGF_DEVICE ? (double*)G : nullptr;
    if (!src) {
        HIPCHK(c, hipMalloc(&src, nbytes));
        if (hipMemcpyAsync(src, G, nbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            (void)hipFree(src);
            return fail(c, LGF_E_DEVICE, "hipMemcpyAsync G in");
        }
    }
    int32_t rc;
    const dim3 grid((unsigned)blocks_for(V, 256));
    if (c->phase == 1)
        rc = c->NE == 9 ? launch(c, K_FIELD, k_field_load<double, 9>, grid, dim3(256), 0, V, (const double*)src, c->d.G)
                        : launch(c, K_FIELD, k_field_load<double, 6>, grid, dim3(256), 0, V, (const double*)src, c->d.G);
    else
        rc = c->NE == 9 ? launch(c, K_FIELD, k_field_load<float, 9>, grid, dim3(256), 0, V, (const double*)src, c->f.G)
                        : launch(c, K_FIELD, k_field_load<float, 6>, grid, dim3(256), 0, V, (const double*)src, c->f.G);
    if (rc == LGF_OK) rc = sync_state(c);
    if (where == LGF_HOST) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(src);
    }
    return rc;
}

int32_t lgf_measure(lgf_ctx c, lgf_stats* out)
{
    const double t0 = now_s();
    TRY(check_ctx(c, true));
    if (!c->delta_valid) {
        TRY(set_stop(c, -1.0));
        TRY(measure_any(c, nullptr));
    }
    TRY(sync_state(c));
    fill_stats(c, out, LGF_OK, t0);
    return LGF_OK;
}

int32_t lgf_step(lgf_ctx c, int64_t n, lgf_stats* trace)
{
    const double t0 = now_s();
    TRY(check_ctx(c, true));
    if (n < 0) return fail(c, LGF_E_INVALID_ARG, "n must be >= 0");
    double* tr = nullptr;
    if (trace) {
        if (c->trace_cap < n + 1) {
            (void)hipFree(c->trace_dev);
            c->trace_dev = nullptr;
            c->trace_cap = 0;
            HIPCHK(c, hipMalloc(&c->trace_dev, sizeof(double) * 2 * (size_t)(n + 1)));
            c->trace_cap = n + 1;
        }
        tr = c->trace_dev;
    }
    TRY(set_stop(c, -1.0));
    if (!c->delta_valid || trace) TRY(measure_any(c, tr));
    for (int64_t k = 1; k <= n; ++k) TRY(update_any(c, tr ? tr + 2 * k : nullptr));
    TRY(sync_state(c));
    if (c->st_host->nonfinite) return fail(c, LGF_E_NONFINITE, "theta became non-finite");
    if (trace) {
        std::vector<double> h(2 * (size_t)(n + 1));
        HIPCHK(c, hipMemcpy(h.data(), c->trace_dev, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        const int64_t it_end = c->st_host->iter;
        for (int64_t k = 0; k <= n; ++k) {
            fill_stats(c, &trace[k], LGF_OK, 0.0);
            trace[k].iter = it_end - n + k;
            trace[k].F = h[2 * k];
            trace[k].theta = h[2 * k + 1];
        }
    }
    (void)t0;
    return LGF_OK;
}

int32_t lgf_fix(lgf_ctx c, lgf_stats* out)
{
    const double t0 = now_s();
    TRY(check_ctx(c, true));
    for (;;) {
        const bool fp32_mixed = c->p.precision == LGF_MIXED && c->phase == 0;
        const double stop = fp32_mixed ? c->p.theta_switch : c->p.theta_stop;
        TRY(set_stop(c, stop));
        if (!c->delta_valid) TRY(measure_any(c, nullptr));
        TRY(sync_state(c));
        while (!c->st_host->done && c->st_host->iter < c->p.max_iter) {
            const int64_t chunk = std::min<int64_t>(c->p.poll_every, c->p.max_iter - c->st_host->iter);
            const int64_t it0 = c->st_host->iter;
            const int cur0 = c->cur;
            for (int64_t k = 0; k < chunk; ++k) TRY(update_any(c, nullptr));
            TRY(sync_state(c));
            resync_cur(c, it0, cur0);
        }
        if (c->st_host->nonfinite) {
            fill_stats(c, out, LGF_E_NONFINITE, t0);
            return fail(c, LGF_E_NONFINITE, "theta became non-finite");
        }
        if (!c->st_host->done) {
            fill_stats(c, out, LGF_E_NOT_CONVERGED, t0);
            return fail(c, LGF_E_NOT_CONVERGED, "max_iter reached");
        }
        if (!fp32_mixed) break;
        // FP32 phase done: rebuild the links in FP64 on the orbit of the input
        c->iter_fp32 = c->st_host->iter;
        TRY(c->NE == 9 ? enqueue_switch<9>(c) : enqueue_switch<6>(c));
        c->phase = 1;
        c->cur = 0;
        c->delta_valid = false;
    }
    fill_stats(c, out, LGF_OK, t0);
    return LGF_OK;
}

int32_t lgf_profile_read(lgf_ctx c, int64_t* launches, double* total_ms, int32_t n, int32_t* count)
{
    if (!c) return LGF_E_INVALID_ARG;
    if (count) *count = K_COUNT;
    for (int k = 0; k < n && k < K_COUNT; ++k) {
        if (launches) launches[k] = c->prof_n[k];
        if (total_ms) total_ms[k] = c->prof_ms[k];
    }
    return LGF_OK;
}

int32_t lgf_profile_reset(lgf_ctx c)
{
    if (!c) return LGF_E_INVALID_ARG;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    prof_collect(c);
    for (int k = 0; k < K_COUNT; ++k) {
        c->prof_n[k] = 0;
        c->prof_ms[k] = 0.0;
    }
    return LGF_OK;
}

int32_t lgf_device_bytes(lgf_ctx c, int64_t* bytes)
{
    if (!c || !bytes) return LGF_E_INVALID_ARG;
    *bytes = c->bytes;
    return LGF_OK;
}

}  // extern "C"
