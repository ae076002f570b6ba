// Host-side plumbing shared by the single-lattice context and the batch:
// error reporting, checked kernel launches with optional HIP-event timing,
// device buffers of one lattice, geometry and the tables of the FFT and of
// the lattice momenta.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lgf.h"

namespace lgf {
namespace rt {

enum KernelId {
    K_LOAD, K_STORE, K_MEASURE, K_TRANSFORM_MEASURE, K_ZT, K_GAUGE, K_REDUCE, K_FIELD, K_SWITCH, K_STATE,
    K_ZT_FWD, K_BANDS_MLP, K_MLP, K_HEATBATH, K_OVERRELAX, K_PLAQUETTE, K_COUNT
};
inline const char* const kKernelNames[K_COUNT] = {
    "load",  "store", "measure", "transform_measure", "zt_fft_scale", "gauge",    "reduce",   "field",
    "precision_switch", "state", "zt_learned", "bands_mlp", "mlp", "heatbath", "overrelax", "plaquette"};

// Learned-step model blob: int32 header {magic, 1, 16, 64, 64, 16, 0, 0},
// bf16 W1[16][64], W2[64][64], W3[64][16], float32 b1[64], b2[64], b3[16].
constexpr int32_t kModelMagic = 0x4C47464D;
constexpr int kModelWeights = 16 * 64 + 64 * 64 + 64 * 16;
constexpr int kModelBiases = 64 + 64 + 16;
constexpr size_t kModelBytes = 32 + 2 * kModelWeights + 4 * kModelBiases;

inline bool parse_model(const void* blob, size_t bytes, const uint16_t** w, const float** b)
{
    if (!blob || bytes != kModelBytes) return false;
    const int32_t* h = static_cast<const int32_t*>(blob);
    if (h[0] != kModelMagic || h[1] != 1 || h[2] != 16 || h[3] != 64 || h[4] != 64 || h[5] != 16) return false;
    *w = reinterpret_cast<const uint16_t*>(static_cast<const char*>(blob) + 32);
    *b = reinterpret_cast<const float*>(static_cast<const char*>(blob) + 32 + 2 * kModelWeights);
    return true;
}

constexpr size_t kMaxLds = 160 * 1024;
constexpr size_t kMaxLdsZt = 128 * 1024;

inline thread_local std::string g_noctx_err;

struct Pending {
    int k;
    hipEvent_t a, b;
};

// What every object that launches kernels carries.
struct Runner {
    hipStream_t stream = nullptr;
    int profile = 0;
    std::string err;
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;
    int64_t prof_n[K_COUNT] = {};
    double prof_ms[K_COUNT] = {};
};

inline int32_t fail(Runner* c, int32_t code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_noctx_err = msg;
    return code;
}

#define HIPCHK(c, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return ::lgf::rt::fail((c), e_ == hipErrorOutOfMemory ? LGF_E_OUT_OF_MEMORY : LGF_E_DEVICE, \
                                   std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define TRY(expr)                          \
    do {                                   \
        int32_t r_ = (expr);               \
        if (r_ != LGF_OK) return r_;       \
    } while (0)

inline hipEvent_t take_event(Runner* c)
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

inline void prof_collect(Runner* c)
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

inline void release_events(Runner* c)
{
    for (auto& pe : c->pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    c->pending.clear();
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    c->ev_pool.clear();
}

// Launch on the runner's stream; with profiling, bracket the kernel with
// events (read back at the next synchronisation).
template <typename K, typename... Args>
int32_t launch(Runner* c, int kid, K kernel, dim3 grid, dim3 block, size_t lds, Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->profile) {
        a = take_event(c);
        b = take_event(c);
        if (a) (void)hipEventRecord(a, c->stream);
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, c->stream, args...);
    hipError_t e = hipGetLastError();
    if (c->profile && a && b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back(Pending{kid, a, b});
    }
    if (e != hipSuccess)
        return fail(c, LGF_E_DEVICE, std::string("launch of ") + kKernelNames[kid] + ": " + hipGetErrorString(e));
    return LGF_OK;
}

inline int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

inline bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

inline int64_t blocks_for(int64_t n, int per) { return (n + per - 1) / per; }

inline double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device buffers of one lattice in precision T.
template <typename T>
struct Bufs {
    C2<T>* U = nullptr;      // reference (loaded) links; the links are G U G^dag(x+mu)
    C2<T>* D = nullptr;
    C2<T>* G = nullptr;      // accumulated gauge, a pair of buffers: G[cur] is G if cur = 0,
    C2<T>* Gb = nullptr;     // else Gb
    C2<T>* tw = nullptr;     // Lx + Ly + Lz + Lt entries
    int64_t d_cap = 0;       // complex elements allocated for D
    Geo geo{};
    int tw_off[4] = {0, 0, 0, 0};
};

// Optional gaps between the component arrays of a field and between the
// (tile, field) chunks of the Delta layout, so that arrays read at the same
// offsets do not sit a power of two apart.  Both are 0 (no gap): the padded
// layout is switched off until a GPU memory fault seen with it is explained.
constexpr size_t kComponentPadBytes = 0;
constexpr size_t kChunkPadBytes = 0;

// Geometry; the (z, t) tiles hold W plane positions, W * sizeof(complex)
// = tile_bytes where the (z, t) block still fits its LDS budget.
template <typename T>
Geo make_geo(const int32_t* dims, int tile_bytes = 64)
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
    int W = (int)(tile_bytes / (int)sizeof(C2<T>));
    if (W < 1) W = 1;
    if (W > g.NP) W = g.NP;
    while (W > 1 && (size_t)W * g.NQ * sizeof(C2<T>) > kMaxLdsZt) W >>= 1;
    g.W = W;
    g.logW = ilog2(W);
    g.RP = g.L[0] + 1;
    g.NPP = g.L[1] * g.RP;
    g.VS = g.V + (int64_t)(kComponentPadBytes / sizeof(C2<T>));
    g.DS = (int64_t)g.NQ * W + (int64_t)(kChunkPadBytes / sizeof(C2<T>));
    return g;
}

// log2 of the plane positions one (z, t) block transforms: the tile width W,
// halved while the block's LDS exceeds 64 KB (so two blocks share a CU) and,
// on small lattices, while there are fewer than 512 blocks (down to 2
// positions per block).
template <typename T>
int zt_part_log(const Geo& g)
{
    int l = g.logW;
    while (l > 0 && ((size_t)g.NQ << l) * sizeof(C2<T>) > 64 * 1024) --l;
    while (l > 1 && (g.NP >> l) * 4 < 512) --l;
    return l;
}

// Blocks and LDS bytes of the (z, t) launch with parts of 2^l positions.
inline int zt_blocks(const Geo& g, int l) { return (g.NP >> l) * 4; }
template <typename T>
size_t zt_lds(const Geo& g, int l) { return ((size_t)g.NQ << l) * sizeof(C2<T>); }

// The gauge kernel runs its inverse (x, y) FFT two fields at a time when every
// thread holds exactly kGauge2fSites sites of the plane.
inline bool gauge_two_field(const Geo& g, int nth) { return g.NP == kGauge2fSites * nth; }

// Complex elements of the Delta buffer.
inline int64_t delta_elems(const Geo& g) { return (int64_t)(g.NP / g.W) * 4 * g.DS; }

// Tile widths (bytes) a geometry may be rebuilt with after allocation.
constexpr int kTileChoices[3] = {32, 64, 128};

// Default tile width of a single-lattice context: 128 bytes is one cache line
// of every (z, t) tile row, so the plane kernels write and read whole lines
// of Delta (fastest of the three choices at 32^4 in FP64 and 12 reals).
constexpr int kDefaultTileBytes = 128;

// Delta capacity that holds the layout of every tile choice (smaller tiles
// mean more chunks and so more padding).
template <typename T>
int64_t delta_capacity(const int32_t* dims, int tile_bytes)
{
    int64_t cap = delta_elems(make_geo<T>(dims, tile_bytes));
    for (int tb : kTileChoices) cap = std::max(cap, delta_elems(make_geo<T>(dims, tb)));
    return cap;
}

template <typename T>
bool shape_fits(const int32_t* dims, int nth)
{
    const size_t npp = (size_t)(dims[0] + 1) * dims[1], nq = (size_t)dims[2] * dims[3];   // padded plane in LDS
    if (4 * npp * sizeof(C2<T>) + 2 * nth * sizeof(double) > kMaxLds) return false;
    if (nq * sizeof(C2<T>) > kMaxLdsZt) return false;
    return true;
}

// ---------------------------------------------------------------------------
// One plain iteration of Algorithm 1 on one lattice, enqueued.  Shared by the
// context (lgf.hip) and the allocation-free entry point (noalloc.hip), so
// both launch the same kernels with the same shapes.
// ---------------------------------------------------------------------------
template <typename T>
struct IterArgs {
    const C2<T>* U = nullptr;    // loaded links U0
    C2<T>* G0 = nullptr;         // gauge pair; G[cur] current
    C2<T>* G1 = nullptr;
    C2<T>* D = nullptr;          // packed Delta (tiled)
    C2<T>* D1 = nullptr;         // learned step: second Delta buffer (state's dsel picks the current one)
    const C2<T>* tw[4] = {};     // twiddles per axis
    const double* ptab = nullptr;
    double* partial = nullptr;   // per-plane F, theta partials
    DevState* st = nullptr;
    double c0 = 0.0;             // (alpha/2) p2max / V (or (alpha/2) / V without acceleration)
    int accel = 1;
    int expo = 0;
    int nth = 256;               // threads per plane block
};

template <typename T>
size_t measure_lds(const Geo& g, int nth) { return plane_lds_elems(g) * sizeof(C2<T>) + 2 * nth * sizeof(double); }
template <typename T>
size_t gauge_lds(const Geo& g, int nth)
{
    return plane_lds_elems(g) * sizeof(C2<T>) / (gauge_two_field(g, nth) ? 2 : 1);
}

template <typename T, int NE, int LMAX>
int32_t set_plane_lds(Runner* r, const Geo& g, int nth)
{
    for (const void* f : {reinterpret_cast<const void*>(&k_measure<T, NE, LMAX, false>),
                          reinterpret_cast<const void*>(&k_measure<T, NE, LMAX, true>)})
        HIPCHK(r, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)measure_lds<T>(g, nth)));
    for (const void* f : {reinterpret_cast<const void*>(&k_gauge<T, NE, LMAX, false>),
                          reinterpret_cast<const void*>(&k_gauge<T, NE, LMAX, true>)})
        HIPCHK(r, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(plane_lds_elems(g) * sizeof(C2<T>))));
    for (const void* f : {reinterpret_cast<const void*>(&k_gauge2f<T, NE, LMAX, false>),
                          reinterpret_cast<const void*>(&k_gauge2f<T, NE, LMAX, true>)})
        HIPCHK(r, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(plane_lds_elems(g) * sizeof(C2<T>) / 2)));
    HIPCHK(r, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zt_reduce<T, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsZt));
    HIPCHK(r, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zt<T, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)zt_lds<T>(g, g.logW)));
    return LGF_OK;
}

// The plane kernels form each in-plane link once when an x row fits in one
// wavefront.
inline bool measure_once(const Geo& g) { return g.L[0] <= 64; }

// Transform + Delta + F/theta partials + forward (x, y) FFT, then the
// one-block reduction of F and theta (a7).  next = 0: the links of the
// current gauge G[cur]; next = 1: those of G[1 - cur] just formed.
// counts_update as for reduce_state.
template <typename T, int NE, int LMAX>
int32_t enqueue_measure_k(Runner* r, const Geo& g, const IterArgs<T>& a, int next, double* trace, int counts_update,
                          bool reduce = true)
{
    const int kid = next ? K_TRANSFORM_MEASURE : K_MEASURE;
    const size_t lds = measure_lds<T>(g, a.nth);
    if (measure_once(g))
        TRY(launch(r, kid, k_measure<T, NE, LMAX, true>, dim3(g.NQ), dim3(a.nth), lds, g, a.U, (const C2<T>*)a.G0,
                   (const C2<T>*)a.G1, next, a.D, a.D1, a.partial, a.tw[0], a.tw[1], (const DevState*)a.st,
                   BandJob{}));
    else
        TRY(launch(r, kid, k_measure<T, NE, LMAX, false>, dim3(g.NQ), dim3(a.nth), lds, g, a.U, (const C2<T>*)a.G0,
                   (const C2<T>*)a.G1, next, a.D, a.D1, a.partial, a.tw[0], a.tw[1], (const DevState*)a.st,
                   BandJob{}));
    if (!reduce) return LGF_OK;
    return launch(r, K_REDUCE, k_reduce<>, dim3(1), dim3(256), 0, (const double*)a.partial, g.NQ, g.V, a.st, trace,
                  counts_update);
}

// G[1 - cur] = reunit(g G[cur]) with g from the filtered Delta in a.D.
template <typename T, int NE, int LMAX, bool EXPO>
int32_t enqueue_gauge_kx(Runner* r, const Geo& g, const IterArgs<T>& a)
{
    if (gauge_two_field(g, a.nth))
        return launch(r, K_GAUGE, k_gauge2f<T, NE, LMAX, EXPO>, dim3(g.NQ), dim3(a.nth), gauge_lds<T>(g, a.nth), g,
                      (const C2<T>*)a.D, a.G0, a.G1, a.tw[0], a.tw[1], (const DevState*)a.st);
    return launch(r, K_GAUGE, k_gauge<T, NE, LMAX, EXPO>, dim3(g.NQ), dim3(a.nth), gauge_lds<T>(g, a.nth), g,
                  (const C2<T>*)a.D, a.G0, a.G1, a.tw[0], a.tw[1], (const DevState*)a.st);
}

template <typename T, int NE, int LMAX>
int32_t enqueue_gauge_k(Runner* r, const Geo& g, const IterArgs<T>& a)
{
    return a.expo ? enqueue_gauge_kx<T, NE, LMAX, true>(r, g, a) : enqueue_gauge_kx<T, NE, LMAX, false>(r, g, a);
}

template <typename T, int NE, int LMAX>
int32_t enqueue_plain_measure(Runner* r, const Geo& g, const IterArgs<T>& a, double* trace)
{
    return enqueue_measure_k<T, NE, LMAX>(r, g, a, 0, trace, 0);
}

// Filter ((z, t) FFT, spectral scale, inverse), g and G, then the Delta of
// the new links; the reduction flips cur.  Within a captured chunk
// (chunk_pos > 0) the new links' reduction is left to the next update's
// (z, t) launch (k_zt_reduce, chunk_pos 2) or to the reduction that ends the
// chunk; chunk_pos 1 is the chunk's first update, whose (z, t) launch has no
// reduction to run.
enum ChunkPos { kUpdateAlone = 0, kChunkFirst = 1, kChunkNext = 2 };

template <typename T, int NE, int LMAX>
int32_t enqueue_plain_update(Runner* r, const Geo& g, const IterArgs<T>& a, double* trace, int chunk_pos = kUpdateAlone)
{
    const int l = zt_part_log<T>(g);
    if (chunk_pos == kChunkNext)
        TRY(launch(r, K_ZT, k_zt_reduce<T, LMAX>, dim3(zt_blocks(g, l)), dim3(512),
                   std::max(zt_lds<T>(g, l), (size_t)(2 * 512 * sizeof(double))), g, a.D, a.tw[2], a.tw[3], a.ptab,
                   a.c0, a.accel, l, a.st, (const double*)a.partial));
    else
        TRY(launch(r, K_ZT, k_zt<T, LMAX>, dim3(zt_blocks(g, l)), dim3(512), zt_lds<T>(g, l), g, a.D, a.tw[2],
                   a.tw[3], a.ptab, a.c0, a.accel, l, (const DevState*)a.st));
    TRY((enqueue_gauge_k<T, NE, LMAX>(r, g, a)));
    return enqueue_measure_k<T, NE, LMAX>(r, g, a, 1, trace, 1, chunk_pos == kUpdateAlone);
}

template <typename T>
std::vector<C2<T>> twiddles(const int32_t* dims, int* off)
{
    std::vector<C2<T>> tw;
    for (int m = 0; m < 4; ++m) {
        off[m] = (int)tw.size();
        for (int k = 0; k < dims[m]; ++k) {
            const double a = -2.0 * M_PI * (double)k / (double)dims[m];
            tw.push_back(mk<T>((T)std::cos(a), (T)std::sin(a)));
        }
    }
    return tw;
}

// Momentum tables indexed by position after the forward transforms:
// 4 sin^2(pi n / L) for n = mode_of_position(L, pos), four axes in a row;
// p2max receives the largest p^2 on the lattice.
inline std::vector<double> momentum_tables(const int32_t* dims, double* p2max)
{
    std::vector<double> pt;
    double pm = 0.0;
    for (int m = 0; m < 4; ++m) {
        const int L = dims[m];
        double best = 0.0;
        for (int pos = 0; pos < L; ++pos) {
            const double s = std::sin(M_PI * (double)mode_of_position(L, pos) / (double)L);
            pt.push_back(4.0 * s * s);
            best = std::fmax(best, 4.0 * s * s);
        }
        pm += best;
    }
    if (p2max) *p2max = pm;
    return pt;
}

// Buffers of one lattice: the reference links, the gauge pair, Delta (sized
// for every tile choice) and the twiddles.
template <typename T>
int32_t alloc_bufs(Runner* c, const int32_t* dims, int NE, int tile_bytes, Bufs<T>& b, int64_t& bytes)
{
    b.geo = make_geo<T>(dims, tile_bytes);
    const int64_t VS = b.geo.VS;
    const size_t link = sizeof(C2<T>) * (size_t)4 * NE * VS;
    const size_t field = sizeof(C2<T>) * (size_t)kGE * VS;      // G: two rows
    b.d_cap = delta_capacity<T>(dims, tile_bytes);
    const size_t dbytes = sizeof(C2<T>) * (size_t)b.d_cap;
    HIPCHK(c, hipMalloc(&b.U, link));
    HIPCHK(c, hipMalloc(&b.G, field));
    HIPCHK(c, hipMalloc(&b.Gb, field));
    HIPCHK(c, hipMalloc(&b.D, dbytes));
    bytes += link + 2 * field + dbytes;
    std::vector<C2<T>> tw = twiddles<T>(dims, b.tw_off);
    HIPCHK(c, hipMalloc(&b.tw, sizeof(C2<T>) * tw.size()));
    HIPCHK(c, hipMemcpy(b.tw, tw.data(), sizeof(C2<T>) * tw.size(), hipMemcpyHostToDevice));
    return LGF_OK;
}

template <typename T>
void free_bufs(Bufs<T>& b)
{
    (void)hipFree(b.U);
    (void)hipFree(b.D);
    (void)hipFree(b.G);
    (void)hipFree(b.Gb);
    (void)hipFree(b.tw);
    b = Bufs<T>();
}

}  // namespace rt
}  // namespace lgf
