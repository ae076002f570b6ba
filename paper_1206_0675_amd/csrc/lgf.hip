// Host runtime and C ABI (include/lgf.h) of the gauge-fixing library.
//
// A context owns, per arithmetic precision T in use:
//   U[0]  the loaded (reference) links U0, structure of arrays, NE complex
//         per link; never overwritten by the iteration
//   G, Gb the accumulated gauge G = reunit(g_n ... reunit(g_2 g_1)), a pair
//         of buffers with G[cur] current: the links are G U0 G^dag(x+mu),
//         formed where they are needed and never stored
//   D     the packed Delta field (4 complex per site) in the tiled layout
//   tw    FFT twiddles W_L^k for the four extents
// plus FP64 tables of the lattice momenta, the per-plane partial sums, and a
// small device state (iteration, F, theta, stop flag, current buffer) that
// the host reads back only at poll points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "runtime.hpp"

using namespace lgf;

using namespace lgf::rt;

// small kernels on the device state (no memset: safe inside graphs)
__global__ void k_state_init(DevState* st, int phase)
{
    st->iter = 0;
    st->iter_fp32 = 0;
    st->max_iter = 0x7fffffffffffffffLL;   // the host counts iterations for single lattices
    st->F = 0.0;
    st->theta = 0.0;
    st->theta_stop = -1.0;
    st->theta_switch = 0.0;
    st->done = 0;
    st->nonfinite = 0;
    st->cur = 0;
    st->phase = phase;
    st->needs_measure = 1;
    st->switch_pending = 0;
    st->mixed = 0;
    st->fallback = 0;
    st->trial_F = 0.0;
    st->trial_theta = 0.0;
    st->fallbacks = 0;
    st->dsel = 0;
    st->pad0 = 0;
}

__global__ void k_state_phase(DevState* st, int phase)
{
    st->phase = phase;
    st->cur = 0;
    st->needs_measure = 1;
}

__global__ void k_state_stop(DevState* st, double theta_stop, int valid)
{
    st->theta_stop = theta_stop;
    st->nonfinite = 0;
    st->done = (valid && st->theta < theta_stop) ? 1 : 0;
}

struct lgf_context : Runner {
    lgf_params p{};
    int NE = 9;
    bool own_stream = false;
    int phase = 1;            // 1: FP64 arithmetic, 0: FP32
    bool use64 = false, use32 = false;
    bool loaded = false;
    bool delta_valid = false; // D and the state hold Delta, F, theta of the current links
    Bufs<double> d;
    Bufs<float> f;
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
    int tile_bytes = kDefaultTileBytes;   // bytes of one (z, t) tile row: W = tile_bytes / sizeof(complex)
    int lmax = 64;            // longest axis rounded up to 64 or 128 (kernel variant)
    hipStream_t cap_stream = nullptr;          // private stream that graph capture runs on
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // per phase: poll_every updates
    hipGraphExec_t gexec_learned = nullptr;                  // poll_every learned updates
    // learned spectral step (FP64): model, band sums, factors, spare Delta buffers
    bool learned = false;
    int chunk_pos = kUpdateAlone;   // where the next plain update sits in a captured chunk
    bool has_model = false;
    uint16_t* mw = nullptr;       // bf16 W1 | W2 | W3
    float* mb = nullptr;          // b1 | b2 | b3
    double* band_partial = nullptr;   // band powers per (z, t) block of the last learned pass
    double* counts16 = nullptr;
    double* s_cur = nullptr;      // factors the next learned update applies
    double* s_next = nullptr;     // the network's factors from the last update's band powers
    double* s_dev = nullptr;      // factors of lgf_learned_factors and of line-search trials
    double* x_dev = nullptr;
    double* ones_dev = nullptr;
    C2<double>* D2 = nullptr;     // second Delta buffer (st->dsel picks the current one)
    C2<double>* D3 = nullptr;     // filtered Delta of a step (input of k_gauge)
    int8_t* btab = nullptr;       // band of every spectrum position (Delta chunk layout)
    int zt_l = 0;                 // log2 positions per (z, t) block of the learned pass
    double counts_host[16] = {};
};

namespace {

// lgf_fix in LGF_MIXED: updates without theta halving after which the FP32
// phase ends even above theta_switch (FP32 rounding of the links stops theta
// near 1e-14 at 32^4; a switch set below that would otherwise run the FP32
// phase to max_iter).
constexpr int64_t kFp32StallIters = 512;

template <typename T>
Bufs<T>& bufs(lgf_context* c);
template <>
Bufs<double>& bufs<double>(lgf_context* c) { return c->d; }
template <>
Bufs<float>& bufs<float>(lgf_context* c) { return c->f; }

int32_t sync_state(lgf_context* c)
{
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->profile) prof_collect(c);
    return LGF_OK;
}

int32_t set_stop(lgf_context* c, double theta_stop)
{
    return launch(c, K_STATE, k_state_stop, dim3(1), dim3(1), 0, c->st, theta_stop, c->delta_valid ? 1 : 0);
}

// ----------------------------------------------------------------------------
// geometry and tables
// ----------------------------------------------------------------------------
template <typename T, int NE, int LMAX>
int32_t set_lds_attrs(lgf_context* c)
{
    return set_plane_lds<T, NE, LMAX>(c, bufs<T>(c).geo, c->nth_plane);
}

// ----------------------------------------------------------------------------
// one iteration, enqueued
// ----------------------------------------------------------------------------
// Delta, F, theta of the current links G[cur] U0 G[cur]^dag(x+mu) with no
// update (the first line of Algorithm 1).
template <typename T, int NE, int LMAX>
IterArgs<T> iter_args(lgf_context* c)
{
    Bufs<T>& b = bufs<T>(c);
    IterArgs<T> a;
    a.U = b.U;
    a.G0 = b.G;
    a.G1 = b.Gb;
    a.D = b.D;
    for (int m = 0; m < 4; ++m) a.tw[m] = b.tw + b.tw_off[m];
    a.ptab = c->ptab;
    a.partial = c->partial;
    a.st = c->st;
    a.c0 = c->c0;
    a.accel = c->p.accel == LGF_ACCEL_FOURIER ? 1 : 0;
    a.expo = c->p.update == LGF_UPDATE_EXP ? 1 : 0;
    a.nth = c->nth_plane;
    if constexpr (std::is_same<T, double>::value)
        if (c->learned) a.D1 = c->D2;     // the measure writes the current one of the two Delta buffers
    return a;
}

// Delta, F, theta of the current links G[cur] U0 G[cur]^dag(x+mu) with no
// update (the first line of Algorithm 1).
template <typename T, int NE, int LMAX>
int32_t enqueue_measure(lgf_context* c, double* trace_slot)
{
    TRY((enqueue_plain_measure<T, NE, LMAX>(c, bufs<T>(c).geo, iter_args<T, NE, LMAX>(c), trace_slot)));
    c->delta_valid = true;
    return LGF_OK;
}

// filter, g, transform, Delta/F/theta of the new links (the loop body of
// Algorithm 1); see enqueue_plain_update.  When the stop flag is set every
// kernel returns at once.  The launch arguments do not change from one
// iteration to the next, so a chunk of iterations can be captured once in a
// graph and replayed.
template <typename T, int NE, int LMAX>
int32_t enqueue_update(lgf_context* c, double* trace_slot)
{
    return enqueue_plain_update<T, NE, LMAX>(c, bufs<T>(c).geo, iter_args<T, NE, LMAX>(c), trace_slot,
                                             c->chunk_pos);
}

// The reduction that ends a captured chunk of plain updates (k_reduce,
// counts_update 1, on the last update's partials).
template <typename T, int NE, int LMAX>
int32_t enqueue_chunk_end(lgf_context* c)
{
    const Geo& g = bufs<T>(c).geo;
    return launch(c, K_REDUCE, k_reduce<>, dim3(1), dim3(256), 0, (const double*)c->partial, g.NQ, g.V, c->st,
                  (double*)nullptr, 1);
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

template <typename T, int NE, int LMAX>
struct OpChunkEnd {
    static int32_t run(lgf_context* c) { return enqueue_chunk_end<T, NE, LMAX>(c); }
};

int32_t measure_any(lgf_context* c, double* trace_slot) { return dispatch<OpMeasure>(c, trace_slot); }
int32_t update_any(lgf_context* c, double* trace_slot) { return dispatch<OpUpdate>(c, trace_slot); }
int32_t chunk_end_any(lgf_context* c) { return dispatch<OpChunkEnd>(c); }

int32_t learned_update(lgf_context* c, double* trace_slot);

int32_t one_update(lgf_context* c) { return c->learned ? learned_update(c, nullptr) : update_any(c, nullptr); }

// n updates for lgf_fix.  A full chunk of poll_every updates is captured once
// per precision phase into a graph (the launch arguments never change) and
// replayed; shorter chunks, profiling runs and no_graph contexts launch
// kernel by kernel.
int32_t enqueue_chunk(lgf_context* c, int64_t n)
{
    if (c->profile || c->p.no_graph || n != c->p.poll_every) {
        for (int64_t k = 0; k < n; ++k) TRY(one_update(c));
        return LGF_OK;
    }
    hipGraphExec_t& ex = c->learned ? c->gexec_learned : c->gexec[c->phase];
    if (!ex) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t run = c->stream;
        c->stream = c->cap_stream;
        hipGraph_t graph = nullptr;
        int32_t rc = LGF_OK;
        if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(c, LGF_E_DEVICE, "hipStreamBeginCapture failed");
        } else {
            // plain updates: each update's reduction runs in the next update's
            // (z, t) launch, and one reduction ends the chunk
            for (int64_t k = 0; k < n && rc == LGF_OK; ++k) {
                if (!c->learned) c->chunk_pos = k == 0 ? kChunkFirst : kChunkNext;
                rc = one_update(c);
            }
            c->chunk_pos = kUpdateAlone;
            if (rc == LGF_OK && !c->learned) rc = chunk_end_any(c);
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
            if (rc == LGF_OK && e != hipSuccess) rc = fail(c, LGF_E_DEVICE, "hipStreamEndCapture failed");
        }
        c->stream = run;
        if (rc == LGF_OK && hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) {
            ex = nullptr;
            rc = fail(c, LGF_E_DEVICE, "hipGraphInstantiate failed");
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != LGF_OK) return rc;
    }
    HIPCHK(c, hipGraphLaunch(ex, c->stream));
    return LGF_OK;
}


// The current gauge G[cur] (the host copy of the state is current after
// every call).
template <typename T>
C2<T>* g_cur(lgf_context* c)
{
    Bufs<T>& b = bufs<T>(c);
    return c->st_host->cur ? b.Gb : b.G;
}

template <typename T, int NE>
int32_t enqueue_store(lgf_context* c, double* dst)
{
    Bufs<T>& b = bufs<T>(c);
    return launch(c, K_STORE, k_store_gauged<T, NE>, dim3((unsigned)blocks_for(4 * b.geo.V, 256)), dim3(256), 0,
                  b.geo, (const C2<T>*)b.U, (const C2<T>*)g_cur<T>(c), dst);
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
    return launch(c, K_LOAD, k_load<T, NE>, dim3((unsigned)blocks_for(4 * V, 256)), dim3(256), 0, V,
                  bufs<T>(c).geo.VS, src, U,
                  c->check);
}

template <typename T>
int32_t enqueue_identity_G(lgf_context* c)
{
    Bufs<T>& b = bufs<T>(c);
    const int64_t V = b.geo.V;
    return launch(c, K_FIELD, k_field_identity<T, kGE>, dim3((unsigned)blocks_for(V, 256)), dim3(256), 0, V,
                  b.geo.VS, b.G);
}

// LGF_MIXED: leave FP32.  G64[0] = reunit(G32[cur]); the FP64 phase then
// forms G64 U0 G64^dag(x+mu) from the loaded FP64 links (the state's cur is
// reset to 0 with the phase).
int32_t enqueue_switch(lgf_context* c)
{
    const Geo& g = c->d.geo;
    return launch(c, K_SWITCH, k_promote_gauge<>, dim3((unsigned)blocks_for(g.V, 256)), dim3(256), 0, g.V,
                  c->f.geo.VS, g.VS, (const C2<float>*)g_cur<float>(c), c->d.G);
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
    out->fallbacks = c->st_host->fallbacks;
    out->F = c->st_host->F;
    out->theta = c->st_host->theta;
    out->seconds = t0 > 0 ? now_s() - t0 : 0.0;
    out->phase = c->phase;
    out->status = status;
}

// ---------------------------------------------------------------------------
// launch shape: threads per plane block and (z, t) tile width
// ---------------------------------------------------------------------------
int32_t set_all_lds(lgf_context* c)
{
    for (int lm : {64, 128}) {
        if (c->use64)
            TRY(c->NE == 9 ? (lm == 64 ? set_lds_attrs<double, 9, 64>(c) : set_lds_attrs<double, 9, 128>(c))
                           : (lm == 64 ? set_lds_attrs<double, 6, 64>(c) : set_lds_attrs<double, 6, 128>(c)));
        if (c->use32)
            TRY(c->NE == 9 ? (lm == 64 ? set_lds_attrs<float, 9, 64>(c) : set_lds_attrs<float, 9, 128>(c))
                           : (lm == 64 ? set_lds_attrs<float, 6, 64>(c) : set_lds_attrs<float, 6, 128>(c)));
    }
    return LGF_OK;
}

// Rebuild the geometry for nth threads per plane block and tile_bytes-wide
// (z, t) tiles.  D was sized for every tile choice.  Only called from
// lgf_create, before the learned-step tables (laid out by tile) exist.
int32_t configure(lgf_context* c, int nth, int tile_bytes)
{
    if ((c->use64 && !shape_fits<double>(c->p.dims, nth)) || (c->use32 && !shape_fits<float>(c->p.dims, nth)))
        return fail(c, LGF_E_INVALID_ARG, "launch shape does not fit this lattice");
    c->nth_plane = nth;
    c->tile_bytes = tile_bytes;
    if (c->use64) {
        c->d.geo = make_geo<double>(c->p.dims, tile_bytes);
        if (delta_elems(c->d.geo) > c->d.d_cap) return fail(c, LGF_E_STATE, "Delta buffer too small for the tile");
    }
    if (c->use32) {
        c->f.geo = make_geo<float>(c->p.dims, tile_bytes);
        if (delta_elems(c->f.geo) > c->f.d_cap) return fail(c, LGF_E_STATE, "Delta buffer too small for the tile");
    }
    TRY(set_all_lds(c));
    for (auto& ex : c->gexec)
        if (ex) {
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
    c->delta_valid = false;
    return LGF_OK;
}

template <typename T, int NE>
int32_t identity_links(lgf_context* c)
{
    Bufs<T>& b = bufs<T>(c);
    const dim3 gr((unsigned)blocks_for(b.geo.V, 256));
    for (int mu = 0; mu < 4; ++mu)
        TRY(launch(c, K_FIELD, k_field_identity<T, NE>, gr, dim3(256), 0, b.geo.V, b.geo.VS,
                   b.U + (int64_t)mu * NE * b.geo.VS));
    return enqueue_identity_G<T>(c);
}

std::string tune_key(const lgf_context* c)
{
    const int* d = c->p.dims;
    const std::string k = "single/p" + std::to_string(c->p.precision) + "/s" + std::to_string(c->p.storage) + "/" +
                          std::to_string(d[0]) + "x" + std::to_string(d[1]) + "x" + std::to_string(d[2]) + "x" +
                          std::to_string(d[3]);
    return std::to_string(std::hash<std::string>{}(k));
}

// Time each candidate launch shape on identity links (the kernels do the
// same work whatever the values; the state's stop test is off) in the
// context's first precision phase, and keep the fastest.  The choice is
// cached per shape in the file named by $LGF_TUNE_CACHE, if set.
int32_t autotune(lgf_context* c)
{
    const char* cache = std::getenv("LGF_TUNE_CACHE");
    const std::string key = tune_key(c);
    if (cache) {
        std::ifstream in(cache);
        std::string k;
        int nth, tb;
        while (in >> k >> nth >> tb)
            if (k == key) return configure(c, nth, tb);
    }
    if (c->phase == 1) TRY(c->NE == 9 ? (identity_links<double, 9>(c)) : (identity_links<double, 6>(c)));
    else TRY(c->NE == 9 ? (identity_links<float, 9>(c)) : (identity_links<float, 6>(c)));
    const int np = c->p.dims[0] * c->p.dims[1];
    std::vector<std::pair<int, int>> cand;
    for (int nth : {64, 128, 256})
        if (nth <= std::max(64, np) && (!c->use64 || shape_fits<double>(c->p.dims, nth)) &&
            (!c->use32 || shape_fits<float>(c->p.dims, nth)))
            for (int tb : kTileChoices) cand.push_back({nth, tb});
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, LGF_E_DEVICE, "hipEventCreate failed");
    }
    float best = 1e30f;
    std::pair<int, int> pick{c->nth_plane, c->tile_bytes};
    const int saved_profile = c->profile;
    c->profile = 0;
    int32_t rc = LGF_OK;
    for (auto& cd : cand) {
        if ((rc = configure(c, cd.first, cd.second)) != LGF_OK) break;
        if ((rc = launch(c, K_STATE, k_state_init, dim3(1), dim3(1), 0, c->st, c->phase)) != LGF_OK) break;
        if ((rc = measure_any(c, nullptr)) != LGF_OK) break;
        for (int k = 0; k < 2 && rc == LGF_OK; ++k) rc = update_any(c, nullptr);
        if (rc != LGF_OK) break;
        (void)hipEventRecord(e0, c->stream);
        for (int k = 0; k < 6 && rc == LGF_OK; ++k) rc = update_any(c, nullptr);
        if (rc != LGF_OK) break;
        (void)hipEventRecord(e1, c->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(c, LGF_E_DEVICE, "tuning run failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            pick = cd;
        }
    }
    c->profile = saved_profile;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(rc);
    if (cache) {
        std::ofstream out(cache, std::ios::app);
        out << key << " " << pick.first << " " << pick.second << "\n";
    }
    return configure(c, pick.first, pick.second);
}

int32_t check_ctx(lgf_context* c, bool need_loaded)
{
    if (!c) return LGF_E_INVALID_ARG;
    if (need_loaded && !c->loaded) return fail(c, LGF_E_STATE, "no links loaded");
    return LGF_OK;
}

// ---------------------------------------------------------------------------
// learned spectral step
// ---------------------------------------------------------------------------
int32_t ensure_learned_buffers(lgf_context* c)
{
    if (c->D2) return LGF_OK;
    if (!c->use64) return fail(c, LGF_E_STATE, "the learned step and the band line search run in FP64");
    const Geo& g = c->d.geo;
    c->zt_l = zt_part_log<double>(g);
    HIPCHK(c, hipMalloc(&c->D2, sizeof(C2<double>) * (size_t)delta_elems(g)));
    HIPCHK(c, hipMalloc(&c->D3, sizeof(C2<double>) * (size_t)delta_elems(g)));
    const int nblk = zt_blocks(g, c->zt_l);
    HIPCHK(c, hipMalloc(&c->band_partial, sizeof(double) * 16 * nblk));
    for (double** q : {&c->counts16, &c->s_cur, &c->s_next, &c->s_dev, &c->x_dev, &c->ones_dev})
        HIPCHK(c, hipMalloc(q, sizeof(double) * 16));
    HIPCHK(c, hipMalloc(&c->btab, (size_t)g.V));
    c->bytes += 2 * sizeof(C2<double>) * (size_t)delta_elems(g) + (size_t)g.V;
    // Bands: 16 intervals of log p^2 from the smallest nonzero p^2 of the
    // lattice to p2max, b = floor(16 ln(p^2 / pmin) / ln(p2max / pmin)) clipped
    // to [0, 15], none for p = 0.  The band of every spectrum position is
    // tabulated once per tile j of W plane positions, the bands of the G
    // t positions one task of the (z, t) pass's t axis holds side by side:
    // byte ((g Lz + z) W + w) G + k of tile j is the band of t position
    // g G + k, z position z, plane position j W + w.  The mode counts come
    // from the same table.
    double p2max = 0.0;
    const std::vector<double> pt = momentum_tables(c->p.dims, &p2max);
    double pmin = 1e300;
    for (int m = 0; m < 4; ++m) {
        const double sn = std::sin(M_PI / (double)c->p.dims[m]);
        pmin = std::fmin(pmin, 4.0 * sn * sn);
    }
    const double log_range = std::log(p2max / pmin);
    const int* L = c->p.dims;
    const double* tx = pt.data();
    const double* ty = tx + L[0];
    const double* tz = ty + L[1];
    const double* tt = tz + L[2];
    const int W = g.W, NQ = g.NQ, n = NQ * W, G = zt_group(L[3]);
    std::vector<int8_t> tab((size_t)g.V);
    double cnt[16] = {};
    for (int j = 0; j < g.NP / W; ++j)
        for (int t = 0; t < L[3]; ++t)
            for (int z = 0; z < L[2]; ++z)
                for (int w = 0; w < W; ++w) {
                    const int pxy = j * W + w;
                    const double p2 = tx[pxy % L[0]] + ty[pxy / L[0]] + tz[z] + tt[t];
                    int b = -1;
                    if (p2 > 0.0) {
                        b = (int)std::floor(16.0 * std::log(p2 / pmin) / log_range);
                        b = b < 0 ? 0 : (b > 15 ? 15 : b);
                        cnt[b] += 1.0;
                    }
                    tab[(size_t)j * n + ((size_t)((t / G) * L[2] + z) * W + w) * G + t % G] = (int8_t)b;
                }
    std::memcpy(c->counts_host, cnt, sizeof cnt);
    std::vector<double> ones(16, 1.0);
    HIPCHK(c, hipMemcpy(c->btab, tab.data(), tab.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->counts16, cnt, sizeof cnt, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ones_dev, ones.data(), sizeof(double) * 16, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->s_cur, ones.data(), sizeof(double) * 16, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->s_next, ones.data(), sizeof(double) * 16, hipMemcpyHostToDevice));
    for (auto f : {reinterpret_cast<const void*>(&k_zt_learned<double, 64>),
                   reinterpret_cast<const void*>(&k_zt_learned<double, 128>)})
        HIPCHK(c, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)zt_lds<double>(g, c->zt_l)));
    return LGF_OK;
}

MlpDev model_ptrs(lgf_context* c, bool use_model)
{
    if (!use_model || !c->has_model) return MlpDev{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    return MlpDev{c->mw, c->mw + 16 * 64, c->mw + 16 * 64 + 64 * 64, c->mb, c->mb + 64, c->mb + 128};
}

// One update with per-band factors s (device array) from the current Delta
// (left in place): the (z, t) pass with band powers into D3, the candidate
// gauge G[1 - cur] = reunit(g G[cur]), the Delta of its links into the other
// Delta buffer, and the learned reduction in `mode` (k_reduce_learned).
template <int NE, int LMAX>
int32_t enqueue_scaled_update(lgf_context* c, const double* s, int mode, double* trace_slot)
{
    Bufs<double>& b = c->d;
    const Geo& g = b.geo;
    TRY(launch(c, K_ZT_FWD, k_zt_learned<double, LMAX>, dim3(zt_blocks(g, c->zt_l)), dim3(512),
               zt_lds<double>(g, c->zt_l), g, (const C2<double>*)b.D, (const C2<double>*)c->D2, c->D3,
               (const C2<double>*)(b.tw + b.tw_off[2]), (const C2<double>*)(b.tw + b.tw_off[3]),
               (const double*)c->ptab, c->c0, (int)(c->p.accel == LGF_ACCEL_FOURIER), c->zt_l, (const int8_t*)c->btab,
               s, (int)(mode == 1), c->band_partial, (const DevState*)c->st));
    IterArgs<double> a = iter_args<double, NE, LMAX>(c);
    a.D = c->D3;
    TRY((enqueue_gauge_k<double, NE, LMAX>(c, g, a)));
    // the candidate's measure launch also computes the next update's factors
    // from this update's band powers (one block in front of the planes)
    const BandJob job{(const double*)c->band_partial, zt_blocks(g, c->zt_l), 0, (const double*)c->counts16, g.V,
                      model_ptrs(c, true), c->s_next};
    const int kid = K_TRANSFORM_MEASURE;
    const size_t lds = std::max(measure_lds<double>(g, a.nth), (size_t)kBandLdsBytes);
    const dim3 grid(g.NQ + kBandSideBlocks);
    if (measure_once(g))
        TRY(launch(c, kid, k_measure<double, NE, LMAX, true>, grid, dim3(a.nth), lds, g, a.U,
                   (const C2<double>*)b.G, (const C2<double>*)b.Gb, 1, b.D, c->D2, c->partial, a.tw[0], a.tw[1],
                   (const DevState*)c->st, job));
    else
        TRY(launch(c, kid, k_measure<double, NE, LMAX, false>, grid, dim3(a.nth), lds, g, a.U,
                   (const C2<double>*)b.G, (const C2<double>*)b.Gb, 1, b.D, c->D2, c->partial, a.tw[0], a.tw[1],
                   (const DevState*)c->st, job));
    return launch(c, K_REDUCE, k_reduce_learned<>, dim3(1), dim3(256), 0, (const double*)c->partial, g.NQ, g.V,
                  c->st, trace_slot, mode, c->s_cur, (const double*)c->s_next);
}

int32_t scaled_update_any(lgf_context* c, const double* s, int mode, double* tr = nullptr)
{
    const bool big = c->lmax > 64;
    if (c->NE == 9)
        return big ? enqueue_scaled_update<9, 128>(c, s, mode, tr) : enqueue_scaled_update<9, 64>(c, s, mode, tr);
    return big ? enqueue_scaled_update<6, 128>(c, s, mode, tr) : enqueue_scaled_update<6, 64>(c, s, mode, tr);
}

// Band powers of the current spectrum, features and (with a model) the
// network's factors for them into x_dev and s_dev; the state is unchanged.
template <int LMAX>
int32_t enqueue_bands(lgf_context* c, bool use_model)
{
    Bufs<double>& b = c->d;
    const Geo& g = b.geo;
    TRY(launch(c, K_ZT_FWD, k_zt_learned<double, LMAX>, dim3(zt_blocks(g, c->zt_l)), dim3(512),
               zt_lds<double>(g, c->zt_l), g, (const C2<double>*)b.D, (const C2<double>*)c->D2, c->D3,
               (const C2<double>*)(b.tw + b.tw_off[2]), (const C2<double>*)(b.tw + b.tw_off[3]),
               (const double*)c->ptab, c->c0, (int)(c->p.accel == LGF_ACCEL_FOURIER), c->zt_l, (const int8_t*)c->btab,
               (const double*)c->ones_dev, 0, c->band_partial, (const DevState*)c->st));
    return launch(c, K_BANDS_MLP, k_bands_mlp<>, dim3(1), dim3(256), 0, (const double*)c->band_partial,
                  zt_blocks(g, c->zt_l), (const double*)c->counts16, g.V, model_ptrs(c, use_model), c->s_dev,
                  c->x_dev);
}

int32_t bands_any(lgf_context* c, bool use_model)
{
    return c->lmax > 64 ? enqueue_bands<128>(c, use_model) : enqueue_bands<64>(c, use_model);
}

// One learned update (Delta of the current links current, state current):
// the factors s_cur (from the network on the previous update's band powers,
// 1 after a load) give candidate links, kept if F grows; the network's
// factors for the next update come from this update's band powers.  A
// rejected candidate leaves the state as it was and raises st->fallback, and
// the next learned update is the plain one from the same Delta.  Every choice
// is made on the device, so updates can be queued (and captured) back to
// back.
int32_t learned_update(lgf_context* c, double* trace_slot) { return scaled_update_any(c, c->s_cur, 1, trace_slot); }

// theta after one update with factors s, the links kept as they are.
int32_t trial_theta(lgf_context* c, const std::vector<double>& s, double* theta)
{
    HIPCHK(c, hipMemcpyAsync(c->s_dev, s.data(), sizeof(double) * 16, hipMemcpyHostToDevice, c->stream));
    TRY(scaled_update_any(c, c->s_dev, 3));
    TRY(sync_state(c));
    *theta = c->st_host->trial_theta;
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
    case LGF_E_MODEL: return "malformed model blob";
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
    if (p->step != LGF_STEP_PLAIN && p->step != LGF_STEP_LEARNED)
        return fail(nullptr, LGF_E_INVALID_ARG, "unknown step kind");
    if (p->step == LGF_STEP_LEARNED && p->precision != LGF_FP64)
        return fail(nullptr, LGF_E_INVALID_ARG, "the learned step runs in FP64");
    if (p->accel != LGF_ACCEL_FOURIER && p->accel != LGF_ACCEL_NONE)
        return fail(nullptr, LGF_E_INVALID_ARG, "accel must be LGF_ACCEL_FOURIER or LGF_ACCEL_NONE");
    if (p->update != LGF_UPDATE_FIRST_ORDER && p->update != LGF_UPDATE_EXP)
        return fail(nullptr, LGF_E_INVALID_ARG, "update must be LGF_UPDATE_FIRST_ORDER or LGF_UPDATE_EXP");
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
    c->profile = p->profile;
    c->learned = p->step == LGF_STEP_LEARNED;
    c->NE = p->storage == LGF_STORE12 ? 6 : 9;
    c->use64 = use64;
    c->use32 = use32;
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
    if (use64 && (rc = alloc_bufs<double>(c, p->dims, c->NE, kDefaultTileBytes, c->d, c->bytes)) != LGF_OK)
        return bail(rc);
    if (use32 && (rc = alloc_bufs<float>(c, p->dims, c->NE, kDefaultTileBytes, c->f, c->bytes)) != LGF_OK)
        return bail(rc);
    const Geo& g = use64 ? c->d.geo : c->f.geo;
    double p2max = 0.0;
    const std::vector<double> pt = momentum_tables(p->dims, &p2max);
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
    if ((rc = set_all_lds(c)) != LGF_OK) return bail(rc);
    if (p->autotune && (rc = autotune(c)) != LGF_OK) return bail(rc);
    if ((rc = launch(c, K_STATE, k_state_init, dim3(1), dim3(1), 0, c->st, c->phase)) != LGF_OK) return bail(rc);
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
    (void)hipFree(c->ptab);
    (void)hipFree(c->partial);
    (void)hipFree(c->st);
    (void)hipFree(c->check);
    (void)hipFree(c->trace_dev);
    for (void* q : {(void*)c->mw, (void*)c->mb, (void*)c->band_partial, (void*)c->counts16, (void*)c->s_dev,
                    (void*)c->x_dev, (void*)c->ones_dev, (void*)c->D2, (void*)c->D3, (void*)c->btab})
        (void)hipFree(q);
    if (c->st_host) (void)hipHostFree(c->st_host);
    release_events(c);
    if (c->gexec_learned) (void)hipGraphExecDestroy(c->gexec_learned);
    for (auto& ex : c->gexec)
        if (ex) (void)hipGraphExecDestroy(ex);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
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
            rc = c->NE == 9 ? enqueue_load<double, 9>(c, s, c->d.U) : enqueue_load<double, 6>(c, s, c->d.U);
            if (rc == LGF_OK) rc = c->NE == 9 ? enqueue_load<float, 9>(c, s, c->f.U) : enqueue_load<float, 6>(c, s, c->f.U);
        } else if (c->p.precision == LGF_FP64) {
            rc = c->NE == 9 ? enqueue_load<double, 9>(c, s, c->d.U) : enqueue_load<double, 6>(c, s, c->d.U);
        } else {
            rc = c->NE == 9 ? enqueue_load<float, 9>(c, s, c->f.U) : enqueue_load<float, 6>(c, s, c->f.U);
        }
        if (rc != LGF_OK) break;
        if (c->use64 && (rc = enqueue_identity_G<double>(c)) != LGF_OK) break;
        if (c->use32 && (rc = enqueue_identity_G<float>(c)) != LGF_OK) break;
        if ((rc = launch(c, K_STATE, k_state_init, dim3(1), dim3(1), 0, c->st, c->use64 && !c->use32 ? 1 : 0)) != LGF_OK)
            break;
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
    c->phase = c->use64 && !c->use32 ? 1 : 0;
    c->iter_fp32 = 0;
    // the learned step's first update after a load uses the plain factors
    if (c->s_cur) TRY(launch(c, K_STATE, k_fill16<>, dim3(1), dim3(64), 0, c->s_cur, 1.0));
    c->loaded = true;
    return LGF_OK;
}

int32_t lgf_store_links(lgf_ctx c, void* links, int32_t where)
{
    TRY(check_ctx(c, true));
    if (!links || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad links/where");
    const int64_t V = (c->phase == 1 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 72 * (size_t)V;
    TRY(sync_state(c));   // the current gauge buffer is known from the device state
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
    if (!G || (where != LGF_HOST && where != LGF_DEVICE)) return fail(c, LGF_E_INVALID_ARG, "bad G/where");
    const int64_t V = (c->use64 ? c->d.geo : c->f.geo).V;
    const size_t nbytes = sizeof(double) * 18 * (size_t)V;
    double* dst = where == LGF_DEVICE ? static_cast<double*>(G) : nullptr;
    if (!dst) HIPCHK(c, hipMalloc(&dst, nbytes));
    int32_t rc;
    const dim3 grid((unsigned)blocks_for(V, 256));
    if (c->phase == 1)
        rc = launch(c, K_FIELD, k_field_store<double, kGE>, grid, dim3(256), 0, V, c->d.geo.VS, (const C2<double>*)g_cur<double>(c), dst);
    else
        rc = launch(c, K_FIELD, k_field_store<float, kGE>, grid, dim3(256), 0, V, c->f.geo.VS, (const C2<float>*)g_cur<float>(c), dst);
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
    c->delta_valid = false;                 // the links G U0 G^dag(x+mu) change with G
    if (c->s_cur) TRY(launch(c, K_STATE, k_fill16<>, dim3(1), dim3(64), 0, c->s_cur, 1.0));
    if (c->phase == 1)
        rc = launch(c, K_FIELD, k_field_load<double, kGE>, grid, dim3(256), 0, V, c->d.geo.VS, (const double*)src, g_cur<double>(c));
    else
        rc = launch(c, K_FIELD, k_field_load<float, kGE>, grid, dim3(256), 0, V, c->f.geo.VS, (const double*)src, g_cur<float>(c));
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
    if (c->learned) {
        if (!c->has_model) return fail(c, LGF_E_STATE, "the learned step needs lgf_set_model first");
        TRY(ensure_learned_buffers(c));
    }
    TRY(set_stop(c, -1.0));
    if (!c->delta_valid || trace) TRY(measure_any(c, tr));
    if (c->learned) {
        for (int64_t k = 1; k <= n; ++k) {
            TRY(learned_update(c, tr ? tr + 2 * k : nullptr));
            TRY(sync_state(c));
            if (c->st_host->fallback) TRY(learned_update(c, tr ? tr + 2 * k : nullptr));   // the plain update
        }
    } else if (!trace) {
        // captured chunks of poll_every updates (as lgf_fix), then single updates
        int64_t k = 0;
        if (c->p.poll_every > 0)
            for (; n - k >= c->p.poll_every; k += c->p.poll_every) TRY(enqueue_chunk(c, c->p.poll_every));
        for (; k < n; ++k) TRY(update_any(c, nullptr));
    } else {
        for (int64_t k = 1; k <= n; ++k) TRY(update_any(c, tr ? tr + 2 * k : nullptr));
    }
    TRY(sync_state(c));
    if (c->st_host->done) c->delta_valid = false;   // a chunk may have passed its last reduction
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
        if (c->learned) {
            if (!c->has_model) return fail(c, LGF_E_STATE, "the learned step needs lgf_set_model first");
            TRY(ensure_learned_buffers(c));
        }
        TRY(set_stop(c, stop));
        if (!c->delta_valid) TRY(measure_any(c, nullptr));
        TRY(sync_state(c));
        // FP32 phase: theta_switch may lie below where FP32 rounding of the
        // links stops theta; the phase also ends once theta has not halved
        // for kFp32StallIters updates, and the run goes on in FP64
        double best = c->st_host->theta;
        int64_t best_iter = c->st_host->iter;
        bool stalled = false;
        while (!c->st_host->done && c->st_host->iter < c->p.max_iter) {
            const int64_t chunk = std::min<int64_t>(c->p.poll_every, c->p.max_iter - c->st_host->iter);
            TRY(enqueue_chunk(c, chunk));
            TRY(sync_state(c));
            if (fp32_mixed && !c->st_host->done) {
                if (c->st_host->theta < 0.5 * best) {
                    best = c->st_host->theta;
                    best_iter = c->st_host->iter;
                } else if (c->st_host->iter - best_iter >= kFp32StallIters) {
                    stalled = true;
                    break;
                }
            }
        }
        // a captured chunk that ended done has transformed D after the last
        // reduction (k_zt_reduce), so D no longer holds the current Delta
        if (c->st_host->done) c->delta_valid = false;
        if (c->st_host->nonfinite) {
            fill_stats(c, out, LGF_E_NONFINITE, t0);
            return fail(c, LGF_E_NONFINITE, "theta became non-finite");
        }
        if (!c->st_host->done && !stalled) {
            fill_stats(c, out, LGF_E_NOT_CONVERGED, t0);
            return fail(c, LGF_E_NOT_CONVERGED, "max_iter reached");
        }
        if (!fp32_mixed) break;
        // FP32 phase done: rebuild the links in FP64 on the orbit of the input
        c->iter_fp32 = c->st_host->iter;
        TRY(enqueue_switch(c));
        TRY(launch(c, K_STATE, k_state_phase, dim3(1), dim3(1), 0, c->st, 1));
        c->phase = 1;
        c->delta_valid = false;
    }
    fill_stats(c, out, LGF_OK, t0);
    return LGF_OK;
}

int32_t lgf_set_model(lgf_ctx c, const void* blob, size_t bytes)
{
    TRY(check_ctx(c, false));
    const uint16_t* w = nullptr;
    const float* b = nullptr;
    if (!parse_model(blob, bytes, &w, &b)) return fail(c, LGF_E_MODEL, "malformed model blob");
    if (!c->mw) HIPCHK(c, hipMalloc(&c->mw, sizeof(uint16_t) * kModelWeights));
    if (!c->mb) HIPCHK(c, hipMalloc(&c->mb, sizeof(float) * kModelBiases));
    HIPCHK(c, hipMemcpy(c->mw, w, sizeof(uint16_t) * kModelWeights, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mb, b, sizeof(float) * kModelBiases, hipMemcpyHostToDevice));
    c->has_model = true;
    return LGF_OK;
}

int32_t lgf_learned_factors(lgf_ctx c, double features[16], double s[16])
{
    TRY(check_ctx(c, true));
    if (!features || !s) return fail(c, LGF_E_INVALID_ARG, "NULL output");
    if (c->phase != 1) return fail(c, LGF_E_STATE, "the learned step runs in FP64");
    TRY(ensure_learned_buffers(c));
    TRY(set_stop(c, -1.0));
    if (!c->delta_valid) TRY(measure_any(c, nullptr));
    TRY(bands_any(c, true));
    HIPCHK(c, hipMemcpyAsync(features, c->x_dev, sizeof(double) * 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(s, c->s_dev, sizeof(double) * 16, hipMemcpyDeviceToHost, c->stream));
    return sync_state(c);            // D still holds Delta of the current links
}

int32_t lgf_linesearch_bands(lgf_ctx c, double features[16], double log_s[16])
{
    TRY(check_ctx(c, true));
    if (!features || !log_s) return fail(c, LGF_E_INVALID_ARG, "NULL output");
    if (c->phase != 1) return fail(c, LGF_E_STATE, "the band line search runs in FP64");
    TRY(ensure_learned_buffers(c));
    TRY(set_stop(c, -1.0));
    if (!c->delta_valid) TRY(measure_any(c, nullptr));
    TRY(bands_any(c, false));
    HIPCHK(c, hipMemcpyAsync(features, c->x_dev, sizeof(double) * 16, hipMemcpyDeviceToHost, c->stream));
    TRY(sync_state(c));
    c->delta_valid = false;          // the trials below write their own Delta into D
    // one factor for all bands: golden-section search on ln s in [-2.3, 2.3]
    double best = 0.0;
    TRY(trial_theta(c, std::vector<double>(16, 1.0), &best));
    auto eval = [&](double u, double* th) { return trial_theta(c, std::vector<double>(16, std::exp(u)), th); };
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = -2.3, b = 2.3, x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1, f2;
    TRY(eval(x1, &f1));
    TRY(eval(x2, &f2));
    for (int it = 0; it < 20; ++it) {
        if (f1 < f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - gr * (b - a);
            TRY(eval(x1, &f1));
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + gr * (b - a);
            TRY(eval(x2, &f2));
        }
    }
    const double u = f1 < f2 ? x1 : x2, fu = f1 < f2 ? f1 : f2;
    for (int k = 0; k < 16; ++k) log_s[k] = (fu < best && c->counts_host[k] > 0.0) ? u : 0.0;
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

int32_t lgf_config(lgf_ctx c, int32_t* plane_threads, int32_t* tile_bytes)
{
    if (!c) return LGF_E_INVALID_ARG;
    if (plane_threads) *plane_threads = c->nth_plane;
    if (tile_bytes) *tile_bytes = c->tile_bytes;
    return LGF_OK;
}

int32_t lgf_device_bytes(lgf_ctx c, int64_t* bytes)
{
    if (!c || !bytes) return LGF_E_INVALID_ARG;
    *bytes = c->bytes;
    return LGF_OK;
}

}  // extern "C"
