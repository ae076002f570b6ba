// Allocation-free one-call gauge fixing (lgf_fix_noalloc in include/lgf.h).
//
// The same iteration as a context's lgf_fix (the same kernels, launch shape
// and order of operations, so the same bits), for callers that cannot
// allocate device memory: code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc.  Every buffer the library needs beyond the
// caller's input and output links (the loaded links in structure-of-arrays
// form, the pair of accumulated-gauge buffers, the packed Delta field, the
// FFT and momentum tables, the per-plane partial sums, the device state and
// the validation counters) is carved out of one file-scope device array,
// `scratch`, of kNoAllocBytes bytes.  Each device the library runs on holds
// its own copy of the array until the process ends.
//
// In host code the array's name is only a host-side handle, not a device
// address.  Its address on each device is taken once, with that device
// current, by hipGetSymbolAddress, and only that address is used afterwards
// (kernel arguments, copies).
//
// Every call on a device shares that device's array, which keeps the last
// call's contents; everything a call reads is written by the same call first
// (the counters and the state are set by small kernels, not by memsets).
// Calls that overlap on one device race on the array and are not supported.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.hpp"

using namespace lgf;
using namespace lgf::rt;

namespace {

// 64 MiB: enough for a 16^4 lattice in FP64 with full (18-real) links.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device.
int32_t scratch_address(unsigned char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, LGF_E_DEVICE, "lgf_fix_noalloc: no current HIP device (or device index out of range)");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, LGF_E_DEVICE,
                        std::string("lgf_fix_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return LGF_OK;
}

__global__ void k_na_init(DevState* st, unsigned long long* check)
{
    st->iter = 0;
    st->iter_fp32 = 0;
    st->max_iter = 0x7fffffffffffffffLL;
    st->F = 0.0;
    st->theta = 0.0;
    st->theta_stop = -1.0;
    st->theta_switch = 0.0;
    st->done = 0;
    st->nonfinite = 0;
    st->cur = 0;
    st->phase = 1;
    st->needs_measure = 1;
    st->switch_pending = 0;
    st->mixed = 0;
    st->fallback = 0;
    st->trial_F = 0.0;
    st->trial_theta = 0.0;
    st->fallbacks = 0;
    st->dsel = 0;
    st->pad0 = 0;
    check[0] = 0;
    check[1] = 0;
    check[2] = 0;
}

__global__ void k_na_stop(DevState* st, double theta_stop)
{
    st->theta_stop = theta_stop;
    st->nonfinite = 0;
    st->done = 0;
}

// Byte offsets of the buffers inside the scratch array (each 256-byte
// aligned) for one lattice.
struct Carve {
    size_t U, G, Gb, D, tw, ptab, partial, st, check, total;
};

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

Carve carve(const Geo& g, int NE)
{
    Carve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up256(bytes);
        return at;
    };
    c.U = take(sizeof(C2<double>) * (size_t)4 * NE * g.VS);
    c.G = take(sizeof(C2<double>) * (size_t)kGE * g.VS);
    c.Gb = take(sizeof(C2<double>) * (size_t)kGE * g.VS);
    c.D = take(sizeof(C2<double>) * (size_t)delta_elems(g));
    c.tw = take(sizeof(C2<double>) * (size_t)(g.L[0] + g.L[1] + g.L[2] + g.L[3]));
    c.ptab = take(sizeof(double) * (size_t)(g.L[0] + g.L[1] + g.L[2] + g.L[3]));
    c.partial = take(sizeof(double) * 2 * (size_t)g.NQ);
    c.st = take(sizeof(DevState));
    c.check = take(sizeof(unsigned long long) * 3);
    c.total = off;
    return c;
}

template <int NE, int LMAX>
int32_t run(Runner* r, const lgf_params* p, const Geo& g, unsigned char* base, const Carve& cv, const double* in,
            double* out, lgf_stats* stats, double t0)
{
    C2<double>* U = reinterpret_cast<C2<double>*>(base + cv.U);
    C2<double>* G = reinterpret_cast<C2<double>*>(base + cv.G);
    C2<double>* Gb = reinterpret_cast<C2<double>*>(base + cv.Gb);
    C2<double>* D = reinterpret_cast<C2<double>*>(base + cv.D);
    C2<double>* tw = reinterpret_cast<C2<double>*>(base + cv.tw);
    double* ptab = reinterpret_cast<double*>(base + cv.ptab);
    double* partial = reinterpret_cast<double*>(base + cv.partial);
    DevState* st = reinterpret_cast<DevState*>(base + cv.st);
    unsigned long long* check = reinterpret_cast<unsigned long long*>(base + cv.check);
    const int* L = p->dims;
    const int nth = g.NP < 64 ? 64 : (g.NP > 256 ? 256 : g.NP);

    // FFT twiddles and momentum tables: computed on the host exactly as a
    // context computes them, staged through fixed-size stack arrays.
    C2<double> tw_h[4 * 128];
    double pt_h[4 * 128];
    int tw_off[4];
    double p2max = 0.0;
    {
        int n = 0;
        for (int m = 0; m < 4; ++m) {
            tw_off[m] = n;
            double best = 0.0;
            for (int k = 0; k < L[m]; ++k, ++n) {
                const double a = -2.0 * M_PI * (double)k / (double)L[m];
                tw_h[n] = mk<double>(std::cos(a), std::sin(a));
                const double s = std::sin(M_PI * (double)mode_of_position(L[m], k) / (double)L[m]);
                pt_h[n] = 4.0 * s * s;
                best = std::fmax(best, 4.0 * s * s);
            }
            p2max += best;
        }
        HIPCHK(r, hipMemcpyAsync(tw, tw_h, sizeof(C2<double>) * n, hipMemcpyHostToDevice, r->stream));
        HIPCHK(r, hipMemcpyAsync(ptab, pt_h, sizeof(double) * n, hipMemcpyHostToDevice, r->stream));
    }
    IterArgs<double> a;
    a.U = U;
    a.G0 = G;
    a.G1 = Gb;
    a.D = D;
    for (int m = 0; m < 4; ++m) a.tw[m] = tw + tw_off[m];
    a.ptab = ptab;
    a.partial = partial;
    a.st = st;
    a.c0 = 0.5 * p->alpha * (p->accel == LGF_ACCEL_FOURIER ? p2max : 1.0) / (double)g.V;
    a.accel = p->accel == LGF_ACCEL_FOURIER ? 1 : 0;
    a.expo = p->update == LGF_UPDATE_EXP ? 1 : 0;
    a.nth = nth;
    TRY((set_plane_lds<double, NE, LMAX>(r, g, nth)));

    // load: state and counters cleared, links laid out and checked, G = 1
    TRY(launch(r, K_STATE, k_na_init, dim3(1), dim3(1), 0, st, check));
    TRY(launch(r, K_LOAD, k_load<double, NE>, dim3((unsigned)blocks_for(4 * g.V, 256)), dim3(256), 0, g.V, g.VS, in,
               U, check));
    TRY(launch(r, K_FIELD, k_field_identity<double, kGE>, dim3((unsigned)blocks_for(g.V, 256)), dim3(256), 0, g.V,
               g.VS, G));
    DevState sh;
    unsigned long long chk[3] = {0, 0, 0};
    HIPCHK(r, hipMemcpyAsync(chk, check, sizeof(chk), hipMemcpyDeviceToHost, r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    double du, dd;
    std::memcpy(&du, &chk[0], sizeof(double));
    std::memcpy(&dd, &chk[1], sizeof(double));
    if (chk[2] != 0) return fail(r, LGF_E_NONFINITE, "lgf_fix_noalloc: non-finite entries in the input links");
    if (p->unit_tol > 0.0 && (du > p->unit_tol || dd > p->unit_tol))
        return fail(r, LGF_E_NOT_UNITARY, "lgf_fix_noalloc: input links not in SU(3) within unit_tol");

    // Algorithm 1: measure, then updates in chunks of poll_every until
    // theta < theta_stop or max_iter
    TRY(launch(r, K_STATE, k_na_stop, dim3(1), dim3(1), 0, st, p->theta_stop));
    TRY((enqueue_plain_measure<double, NE, LMAX>(r, g, a, nullptr)));
    HIPCHK(r, hipMemcpyAsync(&sh, st, sizeof(DevState), hipMemcpyDeviceToHost, r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    while (!sh.done && sh.iter < p->max_iter) {
        const int64_t chunk = std::min<int64_t>(p->poll_every, p->max_iter - sh.iter);
        for (int64_t k = 0; k < chunk; ++k) TRY((enqueue_plain_update<double, NE, LMAX>(r, g, a, nullptr)));
        HIPCHK(r, hipMemcpyAsync(&sh, st, sizeof(DevState), hipMemcpyDeviceToHost, r->stream));
        HIPCHK(r, hipStreamSynchronize(r->stream));
    }
    int32_t status = LGF_OK;
    if (sh.nonfinite) status = fail(r, LGF_E_NONFINITE, "lgf_fix_noalloc: theta became non-finite");
    else if (!sh.done) status = fail(r, LGF_E_NOT_CONVERGED, "lgf_fix_noalloc: max_iter reached");

    // store the links G U0 G^dag(x+mu) of the current gauge
    TRY(launch(r, K_STORE, k_store_gauged<double, NE>, dim3((unsigned)blocks_for(4 * g.V, 256)), dim3(256), 0, g,
               (const C2<double>*)U, (const C2<double>*)(sh.cur ? Gb : G), out));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iter = sh.iter;
        stats->iter_fp64 = sh.iter;
        stats->F = sh.F;
        stats->theta = sh.theta;
        stats->seconds = now_s() - t0;
        stats->phase = 1;
        stats->status = status;
    }
    return status;
}

}  // namespace

extern "C" {

size_t lgf_noalloc_capacity(void) { return kNoAllocBytes; }

int32_t lgf_fix_noalloc(const lgf_params* p, const double* links_in, double* links_out, lgf_stats* out)
{
    const double t0 = now_s();
    if (!p || !links_in || !links_out) return fail(nullptr, LGF_E_INVALID_ARG, "lgf_fix_noalloc: NULL argument");
    if (p->precision != LGF_FP64 || p->step != LGF_STEP_PLAIN)
        return fail(nullptr, LGF_E_INVALID_ARG, "lgf_fix_noalloc: FP64 precision and the plain step only");
    if (p->storage != LGF_STORE18 && p->storage != LGF_STORE12)
        return fail(nullptr, LGF_E_INVALID_ARG, "storage must be LGF_STORE18 or LGF_STORE12");
    if (p->accel != LGF_ACCEL_FOURIER && p->accel != LGF_ACCEL_NONE)
        return fail(nullptr, LGF_E_INVALID_ARG, "accel must be LGF_ACCEL_FOURIER or LGF_ACCEL_NONE");
    if (p->update != LGF_UPDATE_FIRST_ORDER && p->update != LGF_UPDATE_EXP)
        return fail(nullptr, LGF_E_INVALID_ARG, "update must be LGF_UPDATE_FIRST_ORDER or LGF_UPDATE_EXP");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(nullptr, LGF_E_INVALID_ARG, "alpha must be > 0");
    if (!(p->theta_stop >= 0.0)) return fail(nullptr, LGF_E_INVALID_ARG, "theta_stop must be >= 0");
    if (p->max_iter < 0 || p->poll_every < 1) return fail(nullptr, LGF_E_INVALID_ARG, "max_iter >= 0, poll_every >= 1");
    for (int m = 0; m < 4; ++m)
        if (!pow2_in(p->dims[m], 4, 128))
            return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "each extent must be a power of two in [4, 128]");
    const int np = p->dims[0] * p->dims[1];
    const int nth = np < 64 ? 64 : (np > 256 ? 256 : np);
    if (!shape_fits<double>(p->dims, nth))
        return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE, "(x, y) or (z, t) plane too large for one workgroup's LDS");
    const int NE = p->storage == LGF_STORE12 ? 6 : 9;
    const Geo g = make_geo<double>(p->dims, kDefaultTileBytes);
    const Carve cv = carve(g, NE);
    if (cv.total > kNoAllocBytes)
        return fail(nullptr, LGF_E_UNSUPPORTED_SHAPE,
                    "lgf_fix_noalloc: this lattice needs " + std::to_string(cv.total) +
                        " bytes of device scratch; the allocation-free entry point holds " +
                        std::to_string(kNoAllocBytes));
    unsigned char* base = nullptr;
    TRY(scratch_address(&base));
    Runner r;
    r.stream = static_cast<hipStream_t>(p->stream);
    bool big = false;
    for (int m = 0; m < 4; ++m) big = big || p->dims[m] > 64;
    int32_t rc;
    if (NE == 9) rc = big ? run<9, 128>(&r, p, g, base, cv, links_in, links_out, out, t0)
                          : run<9, 64>(&r, p, g, base, cv, links_in, links_out, out, t0);
    else rc = big ? run<6, 128>(&r, p, g, base, cv, links_in, links_out, out, t0)
                  : run<6, 64>(&r, p, g, base, cv, links_in, links_out, out, t0);
    if (rc != LGF_OK) g_noctx_err = r.err;
    return rc;
}

}  // extern "C"
