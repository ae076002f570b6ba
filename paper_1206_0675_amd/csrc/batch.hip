// Batched gauge fixing (lgf_batch_* in include/lgf.h): many lattices of
// different shapes iterated together.
//
// Each member owns the buffers of a single-lattice context (its loaded
// links U0, the accumulated gauge G as a pair of buffers, packed Delta, in
// FP32 and/or FP64) plus a device state.  As for a single lattice, the links
// are G U0 G^dag(x+mu), formed where needed and never stored.  One batch iteration is a fixed sequence of launches, each covering
// every member through a work list of (member, plane) or (member, tile,
// field) items walked by a persistent grid:
//   [mixed]  promote G to FP64 and enter FP64 (members whose FP32 phase
//            just ended); the FP64 links are G U0 G^dag from the loaded links
//   per precision phase P in use:
//            measure + reduce (members that need Delta of fresh links),
//            (z,t) pass, (x,y)-inverse + G update, transform + measure, reduce
// Kernels skip members that are done, in the other phase, or mid-switch, so
// one iteration applies at most one gauge transformation to each member and
// members converge and change precision independently.  poll_every
// iterations are captured once in a graph and replayed; the host reads the
// states back between replays.  An optional autotuner times the candidate
// plane block sizes and (z,t) tile widths on identity fields at create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <new>
#include <sstream>

#include "runtime.hpp"

using namespace lgf;
using namespace lgf::rt;

struct lgf_batch : Runner {
    lgf_params p{};
    int n = 0, NE = 9, lmax = 64;
    bool use64 = false, use32 = false, mixed = false, own_stream = false;
    std::vector<std::array<int32_t, 4>> dims;
    struct Member {
        Bufs<double> d;
        Bufs<float> f;
        double* ptab = nullptr;
        double* partial = nullptr;
        double c0 = 0.0;
        bool loaded = false;
    };
    std::vector<Member> m;
    DevState* st = nullptr;
    DevState* st_host = nullptr;
    BatchCfg<double>* c64 = nullptr;
    BatchCfg<float>* c32 = nullptr;
    uint32_t* items_plane = nullptr;
    uint32_t* items_zt64 = nullptr;
    uint32_t* items_zt32 = nullptr;
    int n_plane = 0, n_zt64 = 0, n_zt32 = 0;
    unsigned long long* check = nullptr;
    int nth_plane = 256, tile_bytes = 64, ncu = 256;
    size_t lds_m[2] = {0, 0}, lds_g[2] = {0, 0}, lds_z[2] = {0, 0};   // [0] FP32, [1] FP64
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t bytes = 0;
};

namespace {

constexpr int kZtThreads = 512;

template <typename T>
Bufs<T>& mbufs(lgf_batch::Member& mm);
template <>
Bufs<double>& mbufs<double>(lgf_batch::Member& mm) { return mm.d; }
template <>
Bufs<float>& mbufs<float>(lgf_batch::Member& mm) { return mm.f; }

template <typename T>
BatchCfg<T>*& dcfg(lgf_batch* b);
template <>
BatchCfg<double>*& dcfg<double>(lgf_batch* b) { return b->c64; }
template <>
BatchCfg<float>*& dcfg<float>(lgf_batch* b) { return b->c32; }

template <typename T>
constexpr int prec_index() { return sizeof(T) == 8 ? 1 : 0; }

// (Re)build the geometries for tile_bytes, the descriptors, the work lists
// and the LDS sizes of every kernel.
template <typename T>
int32_t build_tables(lgf_batch* b)
{
    const int P = prec_index<T>();
    std::vector<BatchCfg<T>> host(b->n);
    std::vector<uint32_t> zt;
    size_t lm = 0, lg = 0, lz = 0;
    for (int i = 0; i < b->n; ++i) {
        Bufs<T>& bf = mbufs<T>(b->m[i]);
        bf.geo = make_geo<T>(b->dims[i].data(), b->tile_bytes);
        const Geo& g = bf.geo;
        if (delta_elems(g) > bf.d_cap) return fail(b, LGF_E_STATE, "Delta buffer too small for this tile width");
        BatchCfg<T>& c = host[i];
        c.geo = g;
        c.U = bf.U;
        c.G[0] = bf.G;
        c.G[1] = bf.Gb;
        c.D = bf.D;
        for (int k = 0; k < 4; ++k) c.tw[k] = bf.tw + bf.tw_off[k];
        c.ptab = b->m[i].ptab;
        c.partial = b->m[i].partial;
        c.st = b->st + i;
        c.c0 = b->m[i].c0;
        c.accel = b->p.accel == LGF_ACCEL_FOURIER;
        for (int j = 0; j < (g.NP / g.W) * 4; ++j) zt.push_back(((uint32_t)i << kItemShift) | (uint32_t)j);
        lm = std::max(lm, (size_t)plane_lds_elems(g) * sizeof(C2<T>) + 2 * (size_t)b->nth_plane * sizeof(double));
        lg = std::max(lg, (size_t)plane_lds_elems(g) * sizeof(C2<T>));
        lz = std::max(lz, (size_t)g.NQ * g.W * sizeof(C2<T>));
    }
    BatchCfg<T>*& dc = dcfg<T>(b);
    if (!dc) HIPCHK(b, hipMalloc(&dc, sizeof(BatchCfg<T>) * b->n));
    HIPCHK(b, hipMemcpy(dc, host.data(), sizeof(BatchCfg<T>) * b->n, hipMemcpyHostToDevice));
    uint32_t*& it = P ? b->items_zt64 : b->items_zt32;
    (void)hipFree(it);
    it = nullptr;
    HIPCHK(b, hipMalloc(&it, sizeof(uint32_t) * zt.size()));
    HIPCHK(b, hipMemcpy(it, zt.data(), sizeof(uint32_t) * zt.size(), hipMemcpyHostToDevice));
    (P ? b->n_zt64 : b->n_zt32) = (int)zt.size();
    b->lds_m[P] = lm;
    b->lds_g[P] = lg;
    b->lds_z[P] = lz;
    return LGF_OK;
}

template <typename T, int NE, int LMAX>
int32_t set_batch_lds(lgf_batch* b)
{
    const int P = prec_index<T>();
    HIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_measure<T, NE, false, LMAX, LMAX == 64>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_m[P]));
    HIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_measure<T, NE, true, LMAX, LMAX == 64>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_m[P]));
    for (const void* f : {reinterpret_cast<const void*>(&kb_gauge<T, NE, LMAX, false>),
                          reinterpret_cast<const void*>(&kb_gauge<T, NE, LMAX, true>)})
        HIPCHK(b, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_g[P]));
    HIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&kb_zt<T, LMAX>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_z[P]));
    return LGF_OK;
}

template <typename T>
int32_t lds_for(lgf_batch* b)
{
    const bool big = b->lmax > 64;
    if (b->NE == 9) return big ? set_batch_lds<T, 9, 128>(b) : set_batch_lds<T, 9, 64>(b);
    return big ? set_batch_lds<T, 6, 128>(b) : set_batch_lds<T, 6, 64>(b);
}

int32_t configure(lgf_batch* b, int nth, int tile_bytes)
{
    b->nth_plane = nth;
    b->tile_bytes = tile_bytes;
    if (b->use64) {
        TRY(build_tables<double>(b));
        TRY(lds_for<double>(b));
    }
    if (b->use32) {
        TRY(build_tables<float>(b));
        TRY(lds_for<float>(b));
    }
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return LGF_OK;
}

int grid_for(lgf_batch* b, int items, int per_cu) { return std::max(1, std::min(items, b->ncu * per_cu)); }

// Every extent of the batch is at most 64 when LMAX = 64, so every member's
// x rows fit a wavefront and the plane kernels form each in-plane link once.
template <typename T, int NE, int LMAX>
int32_t phase_sequence(lgf_batch* b)
{
    const int P = prec_index<T>();
    const BatchCfg<T>* cf = dcfg<T>(b);
    const uint32_t* zt = P ? b->items_zt64 : b->items_zt32;
    const int nzt = P ? b->n_zt64 : b->n_zt32;
    const dim3 gp(grid_for(b, b->n_plane, 4)), bp(b->nth_plane), gz(grid_for(b, nzt, 2)), gr(b->n);
    TRY(launch(b, K_MEASURE, kb_measure<T, NE, false, LMAX, LMAX == 64>, gp, bp, b->lds_m[P], cf, (const uint32_t*)b->items_plane,
               b->n_plane, P));
    TRY(launch(b, K_REDUCE, kb_reduce<T>, gr, dim3(256), 0, cf, P, 0));
    TRY(launch(b, K_ZT, kb_zt<T, LMAX>, gz, dim3(kZtThreads), b->lds_z[P], cf, zt, nzt, P));
    if (b->p.update == LGF_UPDATE_EXP)
        TRY(launch(b, K_GAUGE, kb_gauge<T, NE, LMAX, true>, gp, bp, b->lds_g[P], cf, (const uint32_t*)b->items_plane,
                   b->n_plane, P));
    else
        TRY(launch(b, K_GAUGE, kb_gauge<T, NE, LMAX, false>, gp, bp, b->lds_g[P], cf, (const uint32_t*)b->items_plane,
                   b->n_plane, P));
    TRY(launch(b, K_TRANSFORM_MEASURE, kb_measure<T, NE, true, LMAX, LMAX == 64>, gp, bp, b->lds_m[P], cf,
               (const uint32_t*)b->items_plane, b->n_plane, P));
    TRY(launch(b, K_REDUCE, kb_reduce<T>, gr, dim3(256), 0, cf, P, 1));
    return LGF_OK;
}

template <int NE, int LMAX>
int32_t iteration_t(lgf_batch* b)
{
    if (b->mixed) {
        const dim3 gp(grid_for(b, b->n_plane, 4));
        TRY(launch(b, K_SWITCH, kb_promote<>, gp, dim3(256), 0, (const BatchCfg<float>*)b->c32,
                   (const BatchCfg<double>*)b->c64, (const uint32_t*)b->items_plane, b->n_plane));
        TRY(launch(b, K_STATE, kb_switch_done<>, dim3((unsigned)blocks_for(b->n, 64)), dim3(64), 0,
                   (const BatchCfg<double>*)b->c64, b->n));
    }
    if (b->use32) TRY((phase_sequence<float, NE, LMAX>(b)));
    if (b->use64) TRY((phase_sequence<double, NE, LMAX>(b)));
    return LGF_OK;
}

int32_t iteration(lgf_batch* b)
{
    const bool big = b->lmax > 64;
    if (b->NE == 9) return big ? iteration_t<9, 128>(b) : iteration_t<9, 64>(b);
    return big ? iteration_t<6, 128>(b) : iteration_t<6, 64>(b);
}

// poll_every iterations, captured once into a graph (profiling and no_graph
// batches launch kernel by kernel).
int32_t enqueue_chunk(lgf_batch* b)
{
    const int n = b->p.poll_every;
    if (b->profile || b->p.no_graph) {
        for (int k = 0; k < n; ++k) TRY(iteration(b));
        return LGF_OK;
    }
    if (!b->gexec) {
        if (!b->cap_stream) HIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipStream_t run = b->stream;
        b->stream = b->cap_stream;
        hipGraph_t graph = nullptr;
        int32_t rc = LGF_OK;
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(b, LGF_E_DEVICE, "hipStreamBeginCapture failed");
        } else {
            for (int k = 0; k < n && rc == LGF_OK; ++k) rc = iteration(b);
            const hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
            if (rc == LGF_OK && e != hipSuccess) rc = fail(b, LGF_E_DEVICE, "hipStreamEndCapture failed");
        }
        b->stream = run;
        if (rc == LGF_OK && hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
            b->gexec = nullptr;
            rc = fail(b, LGF_E_DEVICE, "hipGraphInstantiate failed");
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != LGF_OK) return rc;
    }
    HIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
    return LGF_OK;
}

DevState initial_state(const lgf_batch* b, bool tuning)
{
    DevState s{};
    s.max_iter = tuning ? 0x7fffffffffffffffLL : b->p.max_iter;
    s.theta_stop = tuning ? -1.0 : b->p.theta_stop;
    s.theta_switch = b->p.theta_switch;
    s.phase = b->use32 ? 0 : 1;
    s.needs_measure = 1;
    s.mixed = (b->mixed && !tuning) ? 1 : 0;
    return s;
}

template <typename T, int NE>
int32_t identity_member(lgf_batch* b, int i)
{
    Bufs<T>& bf = mbufs<T>(b->m[i]);
    const int64_t V = bf.geo.V;
    const dim3 gr((unsigned)blocks_for(V, 256));
    for (int mu = 0; mu < 4; ++mu)
        TRY(launch(b, K_FIELD, k_field_identity<T, NE>, gr, dim3(256), 0, V, bf.geo.VS,
                   bf.U + (int64_t)mu * NE * bf.geo.VS));
    return launch(b, K_FIELD, k_field_identity<T, kGE>, gr, dim3(256), 0, V, bf.geo.VS, bf.G);
}

int32_t identity_all(lgf_batch* b)
{
    for (int i = 0; i < b->n; ++i) {
        if (b->use64) TRY(b->NE == 9 ? (identity_member<double, 9>(b, i)) : (identity_member<double, 6>(b, i)));
        if (b->use32) TRY(b->NE == 9 ? (identity_member<float, 9>(b, i)) : (identity_member<float, 6>(b, i)));
    }
    return LGF_OK;
}

std::string tune_key(const lgf_batch* b)
{
    std::ostringstream k;
    k << "batch/p" << b->p.precision << "/s" << b->p.storage << "/";
    for (int i = 0; i < b->n; ++i)
        k << b->dims[i][0] << "x" << b->dims[i][1] << "x" << b->dims[i][2] << "x" << b->dims[i][3] << ",";
    return std::to_string(std::hash<std::string>{}(k.str()));
}

// Time each candidate launch shape on identity fields (the kernels do the
// same work whatever the values) and keep the fastest.
int32_t autotune(lgf_batch* b)
{
    const char* cache = std::getenv("LGF_TUNE_CACHE");
    const std::string key = tune_key(b);
    if (cache) {
        std::ifstream in(cache);
        std::string k;
        int nth, tb;
        while (in >> k >> nth >> tb)
            if (k == key) return configure(b, nth, tb);
    }
    int max_np = 0;
    for (auto& d : b->dims) max_np = std::max(max_np, d[0] * d[1]);
    std::vector<std::pair<int, int>> cand;
    for (int nth : {64, 128, 256})
        if (nth <= std::max(64, max_np))
            for (int tb : kTileChoices) cand.push_back({nth, tb});
    hipEvent_t e0, e1;
    HIPCHK(b, hipEventCreate(&e0));
    HIPCHK(b, hipEventCreate(&e1));
    float best = 1e30f;
    std::pair<int, int> pick{b->nth_plane, b->tile_bytes};
    const int saved_profile = b->profile;
    b->profile = 0;
    int32_t rc = LGF_OK;
    for (auto& c : cand) {
        if ((rc = configure(b, c.first, c.second)) != LGF_OK) break;
        if ((rc = identity_all(b)) != LGF_OK) break;
        std::vector<DevState> s(b->n, initial_state(b, true));
        if (hipMemcpy(b->st, s.data(), sizeof(DevState) * b->n, hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(b, LGF_E_DEVICE, "tuning state upload");
            break;
        }
        for (int k = 0; k < 2 && rc == LGF_OK; ++k) rc = iteration(b);
        (void)hipEventRecord(e0, b->stream);
        for (int k = 0; k < 6 && rc == LGF_OK; ++k) rc = iteration(b);
        (void)hipEventRecord(e1, b->stream);
        if (rc != LGF_OK || hipEventSynchronize(e1) != hipSuccess) {
            if (rc == LGF_OK) rc = fail(b, LGF_E_DEVICE, "tuning run failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    b->profile = saved_profile;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(rc);
    if (cache) {
        std::ofstream out(cache, std::ios::app);
        out << key << " " << pick.first << " " << pick.second << "\n";
    }
    return configure(b, pick.first, pick.second);
}

int32_t sync_states(lgf_batch* b)
{
    HIPCHK(b, hipMemcpyAsync(b->st_host, b->st, sizeof(DevState) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (b->profile) prof_collect(b);
    return LGF_OK;
}

template <typename T, int NE>
int32_t load_member(lgf_batch* b, int i, const double* src, C2<T>* U)
{
    const int64_t V = mbufs<T>(b->m[i]).geo.V;
    return launch(b, K_LOAD, k_load<T, NE>, dim3((unsigned)blocks_for(4 * V, 256)), dim3(256), 0, V,
                  mbufs<T>(b->m[i]).geo.VS, src, U, b->check);
}

template <typename T, int NE>
int32_t store_member(lgf_batch* b, int i, double* dst)
{
    Bufs<T>& bf = mbufs<T>(b->m[i]);
    const int64_t V = bf.geo.V;
    return launch(b, K_STORE, k_store_gauged<T, NE>, dim3((unsigned)blocks_for(4 * V, 256)), dim3(256), 0, bf.geo,
                  (const C2<T>*)bf.U, (const C2<T>*)(b->st_host[i].cur ? bf.Gb : bf.G), dst);
}

template <typename T, int NE>
int32_t store_member_gauge(lgf_batch* b, int i, double* dst)
{
    Bufs<T>& bf = mbufs<T>(b->m[i]);
    const int64_t V = bf.geo.V;
    return launch(b, K_FIELD, k_field_store<T, kGE>, dim3((unsigned)blocks_for(V, 256)), dim3(256), 0, V, bf.geo.VS,
                  (const C2<T>*)(b->st_host[i].cur ? bf.Gb : bf.G), dst);
}

int32_t check_member(lgf_batch* b, int i)
{
    if (!b) return LGF_E_INVALID_ARG;
    if (i < 0 || i >= b->n) return fail(b, LGF_E_INVALID_ARG, "member index out of range");
    return LGF_OK;
}

}  // namespace

extern "C" {

int32_t lgf_batch_destroy(lgf_batch_t b)
{
    if (!b) return LGF_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& mm : b->m) {
        free_bufs(mm.d);
        free_bufs(mm.f);
        (void)hipFree(mm.ptab);
        (void)hipFree(mm.partial);
    }
    (void)hipFree(b->st);
    if (b->st_host) (void)hipHostFree(b->st_host);
    (void)hipFree(b->c64);
    (void)hipFree(b->c32);
    (void)hipFree(b->items_plane);
    (void)hipFree(b->items_zt64);
    (void)hipFree(b->items_zt32);
    (void)hipFree(b->check);
    release_events(b);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LGF_OK;
}

int32_t lgf_batch_create(const lgf_params* p, int32_t n, const int32_t (*dims)[4], lgf_batch_t* out)
{
    if (!p || !out || !dims || n < 1 || n > (1 << 11)) return fail(nullptr, LGF_E_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    if (p->precision != LGF_FP64 && p->precision != LGF_FP32 && p->precision != LGF_MIXED)
        return fail(nullptr, LGF_E_INVALID_ARG, "precision must be LGF_FP64, LGF_FP32 or LGF_MIXED");
    if (p->storage != LGF_STORE18 && p->storage != LGF_STORE12)
        return fail(nullptr, LGF_E_INVALID_ARG, "storage must be LGF_STORE18 or LGF_STORE12");
    if (p->step != LGF_STEP_PLAIN) return fail(nullptr, LGF_E_INVALID_ARG, "unknown step kind");
    if (p->accel != LGF_ACCEL_FOURIER && p->accel != LGF_ACCEL_NONE)
        return fail(nullptr, LGF_E_INVALID_ARG, "accel must be LGF_ACCEL_FOURIER or LGF_ACCEL_NONE");
    if (p->update != LGF_UPDATE_FIRST_ORDER && p->update != LGF_UPDATE_EXP)
        return fail(nullptr, LGF_E_INVALID_ARG, "update must be LGF_UPDATE_FIRST_ORDER or LGF_UPDATE_EXP");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(nullptr, LGF_E_INVALID_ARG, "alpha must be > 0");
    if (!(p->theta_stop >= 0.0) || !(p->theta_switch >= 0.0) || p->max_iter < 0 || p->poll_every < 1)
        return fail(nullptr, LGF_E_INVALID_ARG, "bad theta_stop/theta_switch/max_iter/poll_every");
    const bool use64 = p->precision != LGF_FP32, use32 = p->precision != LGF_FP64;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 4; ++k)
            if (!pow2_in(dims[i][k], 4, 128))
                return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "each extent must be a power of two in [4, 128]");
        if ((use64 && !shape_fits<double>(dims[i], 256)) || (use32 && !shape_fits<float>(dims[i], 256)))
            return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "(x, y) or (z, t) plane too large for one workgroup's LDS");
        if ((int64_t)dims[i][2] * dims[i][3] >= (1 << kItemShift))
            return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "too many planes in one member");
    }
    lgf_batch* b = new (std::nothrow) lgf_batch();
    if (!b) return fail(nullptr, LGF_E_OUT_OF_MEMORY, "host allocation failed");
    b->p = *p;
    b->profile = p->profile;
    b->n = n;
    b->NE = p->storage == LGF_STORE12 ? 6 : 9;
    b->use64 = use64;
    b->use32 = use32;
    b->mixed = p->precision == LGF_MIXED;
    b->dims.resize(n);
    b->m.resize(n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) {
            b->dims[i][k] = dims[i][k];
            if (dims[i][k] > 64) b->lmax = 128;
        }
    auto bail = [&](int32_t code) {
        const std::string msg = b->err;
        lgf_batch_destroy(b);
        g_noctx_err = msg;
        return code;
    };
#define BTRY(expr)                              \
    do {                                        \
        int32_t r_ = (expr);                    \
        if (r_ != LGF_OK) return bail(r_);      \
    } while (0)
    if (p->stream) {
        b->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            b->stream = nullptr;
            b->err = "hipStreamCreateWithFlags failed";
            return bail(LGF_E_DEVICE);
        }
        b->own_stream = true;
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (b->ncu < 1) b->ncu = 1;
    if (hipMalloc(&b->st, sizeof(DevState) * n) != hipSuccess) { b->err = "hipMalloc states"; return bail(LGF_E_OUT_OF_MEMORY); }
    if (hipHostMalloc(&b->st_host, sizeof(DevState) * n, hipHostMallocDefault) != hipSuccess) {
        b->st_host = nullptr;
        b->err = "hipHostMalloc states";
        return bail(LGF_E_OUT_OF_MEMORY);
    }
    std::memset(b->st_host, 0, sizeof(DevState) * n);
    if (hipMalloc(&b->check, sizeof(unsigned long long) * 3) != hipSuccess) { b->err = "hipMalloc check"; return bail(LGF_E_OUT_OF_MEMORY); }
    std::vector<uint32_t> plane_items;
    for (int i = 0; i < n; ++i) {
        auto& mm = b->m[i];
        const int32_t* d = b->dims[i].data();
        if (use64) BTRY(alloc_bufs<double>(b, d, b->NE, b->tile_bytes, mm.d, b->bytes));
        if (use32) BTRY(alloc_bufs<float>(b, d, b->NE, b->tile_bytes, mm.f, b->bytes));
        const int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
        const int NQ = d[2] * d[3];
        double p2max = 0.0;
        const std::vector<double> pt = momentum_tables(d, &p2max);
        mm.c0 = 0.5 * p->alpha * (p->accel == LGF_ACCEL_FOURIER ? p2max : 1.0) / (double)V;
        if (hipMalloc(&mm.ptab, sizeof(double) * pt.size()) != hipSuccess ||
            hipMemcpy(mm.ptab, pt.data(), sizeof(double) * pt.size(), hipMemcpyHostToDevice) != hipSuccess) {
            b->err = "momentum tables";
            return bail(LGF_E_DEVICE);
        }
        if (hipMalloc(&mm.partial, sizeof(double) * 2 * NQ) != hipSuccess) { b->err = "hipMalloc partial"; return bail(LGF_E_OUT_OF_MEMORY); }
        for (int q = 0; q < NQ; ++q) plane_items.push_back(((uint32_t)i << kItemShift) | (uint32_t)q);
    }
    b->n_plane = (int)plane_items.size();
    if (hipMalloc(&b->items_plane, sizeof(uint32_t) * plane_items.size()) != hipSuccess ||
        hipMemcpy(b->items_plane, plane_items.data(), sizeof(uint32_t) * plane_items.size(), hipMemcpyHostToDevice) != hipSuccess) {
        b->err = "work list";
        return bail(LGF_E_DEVICE);
    }
    BTRY(configure(b, 256, 64));
    if (p->autotune) BTRY(autotune(b));
#undef BTRY
    *out = b;
    return LGF_OK;
}

int32_t lgf_batch_config(lgf_batch_t b, int32_t* plane_threads, int32_t* tile_bytes)
{
    if (!b) return LGF_E_INVALID_ARG;
    if (plane_threads) *plane_threads = b->nth_plane;
    if (tile_bytes) *tile_bytes = b->tile_bytes;
    return LGF_OK;
}

const char* lgf_batch_last_error(lgf_batch_t b) { return b ? b->err.c_str() : g_noctx_err.c_str(); }

int32_t lgf_batch_load(lgf_batch_t b, int32_t i, const void* links, int32_t where)
{
    TRY(check_member(b, i));
    if (!links || (where != LGF_HOST && where != LGF_DEVICE)) return fail(b, LGF_E_INVALID_ARG, "bad links/where");
    auto& mm = b->m[i];
    mm.loaded = false;
    const int64_t V = (int64_t)b->dims[i][0] * b->dims[i][1] * b->dims[i][2] * b->dims[i][3];
    const size_t nbytes = sizeof(double) * 72 * (size_t)V;
    double* src = nullptr;
    if (where == LGF_HOST) {
        HIPCHK(b, hipMalloc(&src, nbytes));
        if (hipMemcpyAsync(src, links, nbytes, hipMemcpyHostToDevice, b->stream) != hipSuccess) {
            (void)hipFree(src);
            return fail(b, LGF_E_DEVICE, "hipMemcpyAsync links");
        }
    }
    const double* s = where == LGF_HOST ? src : static_cast<const double*>(links);
    int32_t rc = LGF_OK;
    unsigned long long chk[3] = {0, 0, 0};
    do {
        if (hipMemsetAsync(b->check, 0, sizeof(chk), b->stream) != hipSuccess) { rc = fail(b, LGF_E_DEVICE, "memset"); break; }
        if (b->mixed) {
            rc = b->NE == 9 ? load_member<double, 9>(b, i, s, mm.d.U) : load_member<double, 6>(b, i, s, mm.d.U);
            if (rc == LGF_OK) rc = b->NE == 9 ? load_member<float, 9>(b, i, s, mm.f.U) : load_member<float, 6>(b, i, s, mm.f.U);
        } else if (b->use64) {
            rc = b->NE == 9 ? load_member<double, 9>(b, i, s, mm.d.U) : load_member<double, 6>(b, i, s, mm.d.U);
        } else {
            rc = b->NE == 9 ? load_member<float, 9>(b, i, s, mm.f.U) : load_member<float, 6>(b, i, s, mm.f.U);
        }
        if (rc != LGF_OK) break;
        const dim3 gr((unsigned)blocks_for(V, 256));
        if (b->use64)
            rc = launch(b, K_FIELD, k_field_identity<double, kGE>, gr, dim3(256), 0, V, mm.d.geo.VS, mm.d.G);
        if (rc == LGF_OK && b->use32)
            rc = launch(b, K_FIELD, k_field_identity<float, kGE>, gr, dim3(256), 0, V, mm.f.geo.VS, mm.f.G);
        if (rc != LGF_OK) break;
        const DevState s0 = initial_state(b, false);
        if (hipMemcpyAsync(b->st + i, &s0, sizeof(DevState), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipMemcpyAsync(chk, b->check, sizeof(chk), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess) {
            rc = fail(b, LGF_E_DEVICE, "loading member");
            break;
        }
        double du, dd;
        std::memcpy(&du, &chk[0], sizeof(double));
        std::memcpy(&dd, &chk[1], sizeof(double));
        if (chk[2] != 0) rc = fail(b, LGF_E_NONFINITE, "non-finite link entries in member " + std::to_string(i));
        else if (b->p.unit_tol > 0.0 && (du > b->p.unit_tol || dd > b->p.unit_tol))
            rc = fail(b, LGF_E_NOT_UNITARY, "member " + std::to_string(i) + ": max |UU^dag-1| = " + std::to_string(du) +
                                                ", max |det U-1| = " + std::to_string(dd));
    } while (false);
    if (src) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipFree(src);
    }
    if (rc == LGF_OK) mm.loaded = true;
    return rc;
}

int32_t lgf_batch_fix(lgf_batch_t b, lgf_stats* out)
{
    if (!b) return LGF_E_INVALID_ARG;
    for (int i = 0; i < b->n; ++i)
        if (!b->m[i].loaded) return fail(b, LGF_E_STATE, "member " + std::to_string(i) + " has no links loaded");
    const double t0 = now_s();
    TRY(sync_states(b));
    const int64_t max_chunks = (b->p.max_iter + 2) / b->p.poll_every + 3;
    for (int64_t ch = 0; ch < max_chunks; ++ch) {
        bool all = true;
        for (int i = 0; i < b->n; ++i) all = all && b->st_host[i].done;
        if (all) break;
        TRY(enqueue_chunk(b));
        TRY(sync_states(b));
    }
    const double secs = now_s() - t0;
    int32_t worst = LGF_OK;
    for (int i = 0; i < b->n; ++i) {
        const DevState& s = b->st_host[i];
        int32_t st = LGF_OK;
        if (s.nonfinite) st = LGF_E_NONFINITE;
        else if (!s.done || !(s.theta < b->p.theta_stop) || s.phase != (b->use64 ? 1 : 0)) st = LGF_E_NOT_CONVERGED;
        if (st != LGF_OK && (worst == LGF_OK || st == LGF_E_NONFINITE)) worst = st;
        if (out) {
            std::memset(&out[i], 0, sizeof(lgf_stats));
            out[i].iter = s.iter;
            out[i].iter_fp32 = s.iter_fp32;
            out[i].iter_fp64 = s.iter - s.iter_fp32;
            out[i].F = s.F;
            out[i].theta = s.theta;
            out[i].seconds = secs;
            out[i].phase = s.phase;
            out[i].status = st;
        }
    }
    if (worst != LGF_OK) fail(b, worst, "not every member converged");
    return worst;
}

int32_t lgf_batch_store(lgf_batch_t b, int32_t i, void* links, int32_t where)
{
    TRY(check_member(b, i));
    if (!links || (where != LGF_HOST && where != LGF_DEVICE)) return fail(b, LGF_E_INVALID_ARG, "bad links/where");
    if (!b->m[i].loaded) return fail(b, LGF_E_STATE, "member has no links loaded");
    TRY(sync_states(b));
    const int64_t V = (int64_t)b->dims[i][0] * b->dims[i][1] * b->dims[i][2] * b->dims[i][3];
    const size_t nbytes = sizeof(double) * 72 * (size_t)V;
    double* dst = where == LGF_DEVICE ? static_cast<double*>(links) : nullptr;
    if (!dst) HIPCHK(b, hipMalloc(&dst, nbytes));
    const bool fp64 = b->st_host[i].phase == 1;
    int32_t rc = fp64 ? (b->NE == 9 ? store_member<double, 9>(b, i, dst) : store_member<double, 6>(b, i, dst))
                      : (b->NE == 9 ? store_member<float, 9>(b, i, dst) : store_member<float, 6>(b, i, dst));
    if (rc == LGF_OK && where == LGF_HOST && hipMemcpyAsync(links, dst, nbytes, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
        rc = fail(b, LGF_E_DEVICE, "hipMemcpyAsync links out");
    if (rc == LGF_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(b, LGF_E_DEVICE, "synchronize");
    if (where == LGF_HOST) (void)hipFree(dst);
    return rc;
}

int32_t lgf_batch_store_gauge(lgf_batch_t b, int32_t i, void* G, int32_t where)
{
    TRY(check_member(b, i));
    if (!G || (where != LGF_HOST && where != LGF_DEVICE)) return fail(b, LGF_E_INVALID_ARG, "bad G/where");
    if (!b->m[i].loaded) return fail(b, LGF_E_STATE, "member has no links loaded");
    TRY(sync_states(b));
    const int64_t V = (int64_t)b->dims[i][0] * b->dims[i][1] * b->dims[i][2] * b->dims[i][3];
    const size_t nbytes = sizeof(double) * 18 * (size_t)V;
    double* dst = where == LGF_DEVICE ? static_cast<double*>(G) : nullptr;
    if (!dst) HIPCHK(b, hipMalloc(&dst, nbytes));
    const bool fp64 = b->st_host[i].phase == 1;
    int32_t rc = fp64 ? (b->NE == 9 ? store_member_gauge<double, 9>(b, i, dst) : store_member_gauge<double, 6>(b, i, dst))
                      : (b->NE == 9 ? store_member_gauge<float, 9>(b, i, dst) : store_member_gauge<float, 6>(b, i, dst));
    if (rc == LGF_OK && where == LGF_HOST && hipMemcpyAsync(G, dst, nbytes, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
        rc = fail(b, LGF_E_DEVICE, "hipMemcpyAsync G out");
    if (rc == LGF_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(b, LGF_E_DEVICE, "synchronize");
    if (where == LGF_HOST) (void)hipFree(dst);
    return rc;
}

int32_t lgf_fix_batch(const lgf_params* common, int32_t n, const int32_t (*dims)[4], const double* const* links_in,
                      double* const* links_out, lgf_stats* out)
{
    if (!links_in || !links_out) return fail(nullptr, LGF_E_INVALID_ARG, "NULL link arrays");
    lgf_batch_t b = nullptr;
    TRY(lgf_batch_create(common, n, dims, &b));
    int32_t rc = LGF_OK;
    for (int i = 0; i < n && rc == LGF_OK; ++i) rc = lgf_batch_load(b, i, links_in[i], LGF_HOST);
    int32_t fixrc = rc == LGF_OK ? lgf_batch_fix(b, out) : rc;
    if (rc == LGF_OK)
        for (int i = 0; i < n && rc == LGF_OK; ++i) rc = lgf_batch_store(b, i, links_out[i], LGF_HOST);
    if (rc != LGF_OK || fixrc != LGF_OK) g_noctx_err = b->err;
    lgf_batch_destroy(b);
    return rc != LGF_OK ? rc : fixrc;
}

}  // extern "C"
