// HIP kernels of one Fourier-accelerated steepest-descent iteration
// (Algorithm 1 of Cardoso, Silva, Bicudo, Oliveira, arXiv:1206.0675) on a
// 4D periodic lattice, for gfx950.
//
// The gauge transformations of the iteration compose (Section 2): after n
// steps the links are G U0 G^dag(x+mu) with G = g_n ... g_1 for the loaded
// links U0.  The state kept in memory is U0 and G (reunitarised each step);
// the links themselves are formed where they are needed and never stored.
// One iteration is three launches plus a one-block reduction:
//   k_zt        forward 2D FFT over (z, t) of Delta, multiply by
//               (alpha/2) p2max / (p^2 V) (eq. gx), inverse (z, t).
//   k_gauge     inverse 2D FFT over (x, y), g = reunit(1 + dtilde) and
//               G[1 - cur] = reunit(g G[cur]).
//   k_measure   U' = G U0 G^dag(x+mu) for the new G, Delta(x) of U' packed
//               to 8 reals, per-site F and theta terms, and the forward 2D
//               FFT over each (x, y) plane in LDS.
//   k_reduce    F and theta from per-plane partial sums, in a fixed order;
//               sets the convergence flag and makes G[1 - cur] current.
// Every kernel returns at once when the device flag `done` is set, so
// iterations queued past convergence cost only their launches.
//
// Site index s = q * NP + p with p = y * Lx + x (plane offset) and
// q = t * Lz + z (plane index).  Delta after the (x, y) transform is kept in
// a tiled layout: element (field c, plane position p, plane q) at
//   D[((p / W) * 4 + c) * DS + q * W + p % W]      (DS >= NQ * W)
// so the (x, y) kernels read and write runs of W consecutive complex values
// and the (z, t) kernel reads one contiguous block of NQ * W values.
#pragma once
#include "fft.hpp"
#include "su3.hpp"

namespace lgf {

struct Geo {
    int L[4];       // Lx, Ly, Lz, Lt
    int logL[4];
    int NP, logNP;  // Lx * Ly
    int NQ, logNQ;  // Lz * Lt
    int W, logW;    // tile width of the Delta layout
    int64_t V;
    int64_t VS;     // stride between the component arrays of a link or gauge field:
                    // V plus a pad, so the arrays do not sit a power of two apart
                    // (which would map them onto the same cache sets and channels)
    int64_t DS;     // stride between the (tile, field) chunks of the Delta layout:
                    // NQ * W plus a pad, for the same reason
    int RP, NPP;    // LDS copy of an (x, y) plane: row pitch Lx + 1 and field
                    // pitch Ly * RP (complex); the extra element per row moves
                    // consecutive rows to other banks for the x-axis FFT passes
};

// The accumulated gauge G is reunitarised at every step, so its third row is
// (row 1 x row 2)^* (the same rebuild the projection ends with): G is kept as
// its first two rows, kGE complex per site, whatever the link storage.
constexpr int kGE = 6;

// Complex elements of LDS for the four fields of one (x, y) plane.
__host__ __device__ __forceinline__ int plane_lds_elems(const Geo& g) { return 4 * g.NPP; }
__host__ __device__ __forceinline__ int plane_lds_index(const Geo& g, int c, int p)
{
    return c * g.NPP + (p >> g.logL[0]) * g.RP + (p & (g.L[0] - 1));
}

// buf[di(i)] = src[si(i)] for i < n, spread over the block.  Each thread
// issues U loads before its first LDS write, so U memory round trips overlap
// (a loop of single copies waits out one round trip per element).
template <int U, typename T, typename SrcIdx, typename DstIdx>
__device__ __forceinline__ void gather_to_lds(C2<T>* buf, const C2<T>* __restrict__ src, int n, int tid, int nth,
                                              SrcIdx si, DstIdx di)
{
    int i = tid;
    for (; i + (U - 1) * nth < n; i += U * nth) {
        C2<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[si(i + u * nth)];
#pragma unroll
        for (int u = 0; u < U; ++u) buf[di(i + u * nth)] = v[u];
    }
    for (; i < n; i += nth) buf[di(i)] = src[si(i)];
}

__device__ __forceinline__ int ident_index(int i) { return i; }

// Per-configuration state on the device.  The host reads it back only at
// poll points; kernels of an iteration skip a configuration whose `done` is
// set, so iterations queued past convergence do nothing.
struct DevState {
    int64_t iter;          // gauge transformations applied so far
    int64_t iter_fp32;     // ... of which in FP32 arithmetic
    int64_t max_iter;      // batched runs: stop (unconverged) at this count
    double F, theta;       // of the current links
    double theta_stop;     // done once theta < theta_stop
    double theta_switch;   // batched mixed runs: leave FP32 once theta < theta_switch
    int32_t done;
    int32_t nonfinite;
    int32_t cur;           // the current gauge is G[cur]; the update writes G[1 - cur]
    int32_t phase;         // 0: FP32 arithmetic, 1: FP64
    int32_t needs_measure; // Delta, F, theta of the current links are not computed yet
    int32_t switch_pending;// batched mixed runs: FP32 phase finished, rebuild in FP64
    int32_t mixed;         // batched runs: FP32 phase followed by FP64
    int32_t fallback;      // learned step: the last candidate was rejected, so the next
                           // update is the plain one from the same Delta
    double trial_F, trial_theta;   // learned step: F, theta of the candidate links
    int64_t fallbacks;     // learned step: updates that fell back to the plain factors
    int32_t dsel;          // learned step: Delta of the current links is in the Delta buffer dsel
    int32_t pad0;
};

// Plane handled by block b.  Blocks are dealt to the 8 XCDs round robin
// (XCD b & 7, in order b >> 3 on it), and each XCD has its own L2.  The
// transform reads g and the backward links of the z +- 1 and t +- 1 planes,
// so each XCD gets a (z, t) slab (Lz/nz z by Lt/nt t, nz * nt = 8) walked z
// fastest, so that neighbour planes are read on the same XCD close together
// in time.  Of the slab shapes timed at 32^4 (8 XCDs as 1, 2, 4 or 8 slabs
// along z), nz = 8 (4 z by all t) was fastest.  Other shapes keep the
// identity order.
__host__ __device__ __forceinline__ int plane_of_block(int b, const Geo& geo)
{
    const int Lz = geo.L[2], Lt = geo.L[3];
    const int nz = Lz >= 8 ? 8 : Lz;
    const int nt = 8 / nz;
    if (geo.NQ < 64 || Lt % nt != 0) return b;
    const int zw = Lz / nz, tw = Lt / nt;
    const int x = b & 7, l = b >> 3;
    const int z = (x % nz) * zw + l % zw;
    const int t = (x / nz) * tw + l / zw;
    return t * Lz + z;
}

// ---------------------------------------------------------------------------
// block-wide sum of two doubles through LDS, fixed order
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum2(double a, double b, double* red, int tid, int nth,
                                           double* out_a, double* out_b)
{
    red[2 * tid] = a;
    red[2 * tid + 1] = b;
    __syncthreads();
    for (int h = nth >> 1; h > 0; h >>= 1) {
        if (tid < h) {
            red[2 * tid] += red[2 * (tid + h)];
            red[2 * tid + 1] += red[2 * (tid + h) + 1];
        }
        __syncthreads();
    }
    *out_a = red[0];
    *out_b = red[1];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// a0: canonical FP64 [s][mu][3][3] -> SoA links of type T; validation
// ---------------------------------------------------------------------------
// dev[0], dev[1]: max |U U^dag - 1| and |det U - 1| as double bit patterns
// (non-negative doubles order like their bit patterns); dev[2]: number of
// links with a non-finite entry.
template <typename T, int NE>
__global__ void __launch_bounds__(256) k_load(int64_t V, int64_t VS, const double* __restrict__ src,
                                              C2<T>* __restrict__ U, unsigned long long* __restrict__ dev)
{
    __shared__ double red[2 * 256];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + tid;
    double du = 0.0, dd = 0.0;
    if (li < 4 * V) {
        const int64_t s = li >> 2;
        const int mu = (int)(li & 3);
        M3<double> m;
        const C2<double>* p = reinterpret_cast<const C2<double>*>(src) + li * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) m.e[e] = p[e];
        bool finite = true;
#pragma unroll
        for (int e = 0; e < 9; ++e) finite = finite && isfinite(m.e[e].x) && isfinite(m.e[e].y);
        if (!finite) {
            atomicAdd(&bad, 1);
        } else {
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    C2<double> acc = mk<double>(i == j ? -1.0 : 0.0, 0.0);
                    for (int k = 0; k < 3; ++k) acc = acc + cmulc(m.e[3 * i + k], m.e[3 * j + k]);
                    du = fmax(du, sqrt(acc.x * acc.x + acc.y * acc.y));
                }
            C2<double> det = cmul(m.e[0], cmul(m.e[4], m.e[8]) - cmul(m.e[5], m.e[7]));
            det = det - cmul(m.e[1], cmul(m.e[3], m.e[8]) - cmul(m.e[5], m.e[6]));
            det = det + cmul(m.e[2], cmul(m.e[3], m.e[7]) - cmul(m.e[4], m.e[6]));
            dd = sqrt((det.x - 1.0) * (det.x - 1.0) + det.y * det.y);
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) U[(mu * NE + e) * VS + s] = mk<T>((T)m.e[e].x, (T)m.e[e].y);
    }
    // block max
    red[2 * tid] = du;
    red[2 * tid + 1] = dd;
    __syncthreads();
    for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
        if (tid < h) {
            red[2 * tid] = fmax(red[2 * tid], red[2 * (tid + h)]);
            red[2 * tid + 1] = fmax(red[2 * tid + 1], red[2 * (tid + h) + 1]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicMax(&dev[0], (unsigned long long)__double_as_longlong(red[0]));
        atomicMax(&dev[1], (unsigned long long)__double_as_longlong(red[1]));
        if (bad) atomicAdd(&dev[2], (unsigned long long)bad);
    }
}

// Canonical FP64 links G(x) Uref_mu(x) G^dag(x+mu) from reference links and
// the accumulated gauge: the same arithmetic as the links k_measure forms, so
// the stored links are bit for bit the ones measured.
template <typename T, int NE>
__global__ void __launch_bounds__(256) k_store_gauged(Geo geo, const C2<T>* __restrict__ Uref,
                                                      const C2<T>* __restrict__ G, double* __restrict__ dst)
{
    const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;    // site * 4 + mu
    if (li >= 4 * geo.V) return;
    const int64_t s = li >> 2;
    const int mu = (int)(li & 3);
    int64_t rem = s;
    int c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = (int)(rem & (geo.L[k] - 1));
        rem >>= geo.logL[k];
    }
    c[mu] = (c[mu] + 1) & (geo.L[mu] - 1);
    const int64_t sn = (((int64_t)c[3] * geo.L[2] + c[2]) * geo.L[1] + c[1]) * geo.L[0] + c[0];
    M3<T> a, u, b, r;
    load_mat<T, kGE>(a, G, geo.VS, s);
    load_mat<T, NE>(u, Uref + (int64_t)mu * NE * geo.VS, geo.VS, s);
    load_mat<T, kGE>(b, G, geo.VS, sn);
    a_u_bdag<T, (NE == 6 ? 2 : 3)>(a, u, b, r);
    C2<double>* p = reinterpret_cast<C2<double>*>(dst) + li * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) p[e] = mk<double>((double)r.e[e].x, (double)r.e[e].y);
}

// per-site matrix field (g or G): canonical FP64 [s][3][3] <-> SoA
template <typename T, int NE>
__global__ void __launch_bounds__(256) k_field_store(int64_t V, int64_t VS, const C2<T>* __restrict__ f,
                                                     double* __restrict__ dst)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    M3<T> m;
    load_mat<T, NE>(m, f, VS, s);
    C2<double>* p = reinterpret_cast<C2<double>*>(dst) + s * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) p[e] = mk<double>((double)m.e[e].x, (double)m.e[e].y);
}

template <typename T, int NE>
__global__ void __launch_bounds__(256) k_field_load(int64_t V, int64_t VS, const double* __restrict__ src,
                                                    C2<T>* __restrict__ f)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const C2<double>* p = reinterpret_cast<const C2<double>*>(src) + s * 9;
#pragma unroll
    for (int e = 0; e < NE; ++e) f[e * VS + s] = mk<T>((T)p[e].x, (T)p[e].y);
}

template <typename T, int NE>
__global__ void __launch_bounds__(256) k_field_identity(int64_t V, int64_t VS, C2<T>* __restrict__ f)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int e = 0; e < NE; ++e) f[e * VS + s] = mk<T>((e == 0 || e == 4 || e == 8) ? T(1) : T(0), T(0));
}


// ---------------------------------------------------------------------------
// a1 + a2 + a3(x, y) for one (z, t) plane q: gauge transform, Delta, F and
// theta terms, forward (x, y) FFT of the packed Delta into D.  The links
// are U'_mu(x) = G(x) Uref_mu(x) G^dag(x+mu) for the reference (loaded) links
// Uref and the accumulated gauge G; they are formed here, for the plane's
// own links and the backward neighbours, and never stored.
//   red: 2 * blockDim doubles of LDS; buf: plane_lds_elems(geo) complex of LDS.
// ---------------------------------------------------------------------------
template <typename T, int NE, int LMAX>
__device__ __forceinline__ void measure_plane(const Geo& geo, int q, const C2<T>* __restrict__ Uref,
                                              const C2<T>* __restrict__ G, C2<T>* __restrict__ D,
                                              double* __restrict__ partial, const C2<T>* __restrict__ twx,
                                              const C2<T>* __restrict__ twy, double* red, C2<T>* buf)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int Lx = geo.L[0], Ly = geo.L[1], Lz = geo.L[2], Lt = geo.L[3];
    const int NP = geo.NP;
    const int64_t VS = geo.VS;
    const int z = q & (Lz - 1), t = q >> geo.logL[2];
    const int64_t qzp = (int64_t)(t * Lz + ((z + 1) & (Lz - 1))) * NP;
    const int64_t qzm = (int64_t)(t * Lz + ((z - 1) & (Lz - 1))) * NP;
    const int64_t qtp = (int64_t)(((t + 1) & (Lt - 1)) * Lz + z) * NP;
    const int64_t qtm = (int64_t)(((t - 1) & (Lt - 1)) * Lz + z) * NP;
    const int64_t q0 = (int64_t)q * NP;

    double fsum = 0.0, tsum = 0.0;
    for (int p = tid; p < NP; p += nth) {
        const int x = p & (Lx - 1), y = p >> geo.logL[0];
        const int64_t s = q0 + p;
        const int64_t xp = q0 + y * Lx + ((x + 1) & (Lx - 1)), xm = q0 + y * Lx + ((x - 1) & (Lx - 1));
        const int64_t yp = q0 + (((y + 1) & (Ly - 1)) * Lx + x), ym = q0 + (((y - 1) & (Ly - 1)) * Lx + x);
        Alg8<T> acc;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc.c[c] = mk<T>(T(0), T(0));
        M3<T> gx;
        load_mat<T, kGE>(gx, G, VS, s);
        double f = 0.0;
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            M3<T> u, gn, r;
            load_mat<T, NE>(u, Uref + (int64_t)mu * NE * VS, VS, s);
            load_mat<T, kGE>(gn, G, VS, mu == 0 ? xp : mu == 1 ? yp : mu == 2 ? qzp + p : qtp + p);
            a_u_bdag<T, (NE == 6 ? 2 : 3)>(gx, u, gn, r);
            f += re_trace(r);
            alg_accumulate(acc, r, T(-1));
        }
#pragma unroll 1
        for (int nu = 0; nu < 4; ++nu) {
            M3<T> u, gb, r;
            const int64_t sb = nu == 0 ? xm : nu == 1 ? ym : nu == 2 ? qzm + p : qtm + p;
            load_mat<T, NE>(u, Uref + (int64_t)nu * NE * VS, VS, sb);
            load_mat<T, kGE>(gb, G, VS, sb);
            a_u_bdag<T, (NE == 6 ? 2 : 3)>(gb, u, gx, r);
            alg_accumulate(acc, r, T(1));
        }
        fsum += f;
        tsum += alg_norm2(acc);
#pragma unroll
        for (int c = 0; c < 4; ++c) buf[plane_lds_index(geo, c, p)] = acc.c[c];
    }
    double fb, tb;
    block_sum2(fsum, tsum, red, tid, nth, &fb, &tb);
    if (tid == 0) {
        partial[2 * q] = fb;
        partial[2 * q + 1] = tb;
    }
    // forward FFT along x, then y, of the four fields
    fft_fwd<T, LMAX>(buf, Lx, Lines{geo.logL[1], 2, geo.RP, geo.NPP, 1}, twx, tid, nth);
    fft_fwd<T, LMAX>(buf, Ly, Lines{geo.logL[0], 2, 1, geo.NPP, geo.RP}, twy, tid, nth);
    const int W = geo.W;
    for (int i = tid; i < 4 * NP; i += nth) {
        const int c = i >> geo.logNP, p = i & (NP - 1);
        D[(int64_t)((p >> geo.logW) * 4 + c) * geo.DS + (int64_t)q * W + (p & (W - 1))] =
            buf[plane_lds_index(geo, c, p)];
    }
}

// ---------------------------------------------------------------------------
// Delta of one (z, t) plane with every in-plane link formed once.
//
// A link U'_mu(x) enters Delta at two sites: with a minus sign at x and with
// a plus sign at x + mu.  Threads are laid out so that the x neighbours of a
// site sit in neighbouring lanes of one wavefront (thread = column x of a
// strip of J consecutive rows), so:
//   - the x link a thread forms is handed to the lane of x + 1 by a
//     cross-lane permute (no second formation, no LDS);
//   - the y link of row j is carried in registers to row j + 1 of the same
//     thread; only the first row of each strip forms its backward y link;
//   - the z and t links of the neighbouring planes belong to other blocks and
//     are formed again here.
// That is 4 + 2 + 1/J formations per site instead of 8.  Requires Lx <= 64
// (a row within one wavefront) and blockDim a multiple of Lx.
// For each site of the plane, emit(p, Delta(x)) is called by the thread that
// owns it; fsum and tsum receive the thread's F and theta terms.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void alg_of(const M3<T>& u, Alg8<T>& a)
{
#pragma clang fp contract(off)
    const T third = T(2) / T(3);
    a.c[0] = u.e[1] - conjg(u.e[3]);
    a.c[1] = u.e[2] - conjg(u.e[6]);
    a.c[2] = u.e[5] - conjg(u.e[7]);
    const T tr = third * (u.e[0].y + u.e[4].y + u.e[8].y);
    a.c[3] = mk<T>(T(2) * u.e[0].y - tr, T(2) * u.e[4].y - tr);
}

template <typename T>
__device__ __forceinline__ void alg_add(Alg8<T>& acc, const Alg8<T>& a)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.c[k] = acc.c[k] + a.c[k];
}

template <typename T>
__device__ __forceinline__ void alg_sub(Alg8<T>& acc, const Alg8<T>& a)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.c[k] = acc.c[k] - a.c[k];
}

// a of the lane `src` of this wavefront (every lane of the wavefront calls it)
template <typename T>
__device__ __forceinline__ Alg8<T> alg_from_lane(const Alg8<T>& a, int src)
{
    Alg8<T> b;
#pragma unroll
    for (int k = 0; k < 4; ++k) b.c[k] = mk<T>(__shfl(a.c[k].x, src), __shfl(a.c[k].y, src));
    return b;
}

// r = a U b^dag for the link U of direction base `Umu` at site su
template <typename T, int NE>
__device__ __forceinline__ void link_abdag(const M3<T>& a, const C2<T>* __restrict__ Umu, int64_t VS, int64_t su,
                                           const M3<T>& b, M3<T>& r)
{
    M3<T> u;
    load_mat<T, NE>(u, Umu, VS, su);
    a_u_bdag<T, (NE == 6 ? 2 : 3)>(a, u, b, r);
}

template <typename T, int NE, typename Emit>
__device__ __forceinline__ void plane_delta_once(const Geo& geo, int q, const C2<T>* __restrict__ Uref,
                                                 const C2<T>* __restrict__ G, double& fsum, double& tsum, Emit emit)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int Lx = geo.L[0], Ly = geo.L[1], Lz = geo.L[2], Lt = geo.L[3], lx = geo.logL[0];
    const int64_t VS = geo.VS;
    int nc = nth >> lx;                     // strips of rows
    if (nc > Ly) nc = Ly;
    const int J = Ly / nc;                  // rows per strip
    const int x = tid & (Lx - 1), cr = tid >> lx;
    const bool own = cr < nc;               // spare threads (plane smaller than the block) shadow a strip
    const int cs = own ? cr : (cr & (nc - 1));
    const int src = ((tid & ~(Lx - 1)) | ((x - 1) & (Lx - 1))) & 63;   // lane holding x - 1
    const int z = q & (Lz - 1), t = q >> geo.logL[2];
    const int NP = geo.NP;
    const int64_t q0 = (int64_t)q * NP;
    const int64_t dzp = (int64_t)(t * Lz + ((z + 1) & (Lz - 1))) * NP - q0;
    const int64_t dzm = (int64_t)(t * Lz + ((z - 1) & (Lz - 1))) * NP - q0;
    const int64_t dtp = (int64_t)(((t + 1) & (Lt - 1)) * Lz + z) * NP - q0;
    const int64_t dtm = (int64_t)(((t - 1) & (Lt - 1)) * Lz + z) * NP - q0;
    Alg8<T> ycarry;                         // U'_y of the row below, from the previous row
#pragma unroll
    for (int k = 0; k < 4; ++k) ycarry.c[k] = mk<T>(T(0), T(0));
#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const int y = cs * J + j;
        const int p = (y << lx) + x;
        const int64_t s = q0 + p;
        const int64_t dxp = (int64_t)((x + 1) & (Lx - 1)) - x;
        const int64_t dyp = (int64_t)((((y + 1) & (Ly - 1)) - y) << lx);
        const int64_t dym = (int64_t)((((y - 1) & (Ly - 1)) - y) << lx);
        M3<T> gx;
        load_mat<T, kGE>(gx, G, VS, s);
        // U'_y(x - y): carried from the row below, or formed in the strip's
        // first row.  It enters the sum first either way, so the result does
        // not depend on where the strips start (on the block size).
        Alg8<T> acc;
        if (j == 0) {
            const int64_t sb = s + dym;
            M3<T> gb, r;
            load_mat<T, kGE>(gb, G, VS, sb);
            link_abdag<T, NE>(gb, Uref + (int64_t)NE * VS, VS, sb, gx, r);
            alg_of(r, acc);
        } else {
            acc = ycarry;
        }
        double f = 0.0;
        // forward links U'_mu(x) = G(x) U0_mu(x) G^dag(x + mu)
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            M3<T> gn, r;
            load_mat<T, kGE>(gn, G, VS, s + (mu == 0 ? dxp : mu == 1 ? dyp : mu == 2 ? dzp : dtp));
            link_abdag<T, NE>(gx, Uref + (int64_t)mu * NE * VS, VS, s, gn, r);
            f += re_trace(r);
            Alg8<T> a;
            alg_of(r, a);
            alg_sub(acc, a);
            if (mu == 0) alg_add(acc, alg_from_lane(a, src));    // U'_x(x - x) from the lane of x - 1
            else if (mu == 1) ycarry = a;                         // U'_y(x) for the row above
        }
        // backward links U'_nu(x - nu) = G(x - nu) U0_nu(x - nu) G^dag(x) of the z and t neighbours
#pragma unroll 1
        for (int nu = 2; nu < 4; ++nu) {
            const int64_t sb = s + (nu == 2 ? dzm : dtm);
            M3<T> gb, r;
            load_mat<T, kGE>(gb, G, VS, sb);
            link_abdag<T, NE>(gb, Uref + (int64_t)nu * NE * VS, VS, sb, gx, r);
            Alg8<T> b;
            alg_of(r, b);
            alg_add(acc, b);
        }
        if (own) {
            fsum += f;
            tsum += alg_norm2(acc);
            emit(p, acc);
        }
    }
}

// F and theta partials of plane q, then the forward (x, y) FFT of the four
// fields in buf (LDS, plane_lds_index layout) and the write of D.
template <typename T, int LMAX>
__device__ __forceinline__ void plane_finish(const Geo& geo, int q, double fsum, double tsum, C2<T>* __restrict__ D,
                                             double* __restrict__ partial, const C2<T>* __restrict__ twx,
                                             const C2<T>* __restrict__ twy, double* red, C2<T>* buf)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    double fb, tb;
    block_sum2(fsum, tsum, red, tid, nth, &fb, &tb);
    if (tid == 0) {
        partial[2 * q] = fb;
        partial[2 * q + 1] = tb;
    }
    fft_fwd<T, LMAX>(buf, geo.L[0], Lines{geo.logL[1], 2, geo.RP, geo.NPP, 1}, twx, tid, nth);
    fft_fwd<T, LMAX>(buf, geo.L[1], Lines{geo.logL[0], 2, 1, geo.NPP, geo.RP}, twy, tid, nth);
    const int W = geo.W, NP = geo.NP;
    for (int i = tid; i < 4 * NP; i += nth) {
        const int c = i >> geo.logNP, p = i & (NP - 1);
        D[(int64_t)((p >> geo.logW) * 4 + c) * geo.DS + (int64_t)q * W + (p & (W - 1))] =
            buf[plane_lds_index(geo, c, p)];
    }
}

// The whole of a1 + a2 + a3(x, y) for plane q with links formed once where
// the shape allows it.
template <typename T, int NE, int LMAX>
__device__ __forceinline__ void measure_plane_once(const Geo& geo, int q, const C2<T>* __restrict__ Uref,
                                                   const C2<T>* __restrict__ G, C2<T>* __restrict__ D,
                                                   double* __restrict__ partial, const C2<T>* __restrict__ twx,
                                                   const C2<T>* __restrict__ twy, double* red, C2<T>* buf)
{
    double fsum = 0.0, tsum = 0.0;
    plane_delta_once<T, NE>(geo, q, Uref, G, fsum, tsum, [&](int p, const Alg8<T>& acc) {
#pragma unroll
        for (int c = 0; c < 4; ++c) buf[plane_lds_index(geo, c, p)] = acc.c[c];
    });
    plane_finish<T, LMAX>(geo, q, fsum, tsum, D, partial, twx, twy, red, buf);
}

// ---------------------------------------------------------------------------
// a3(z, t) + a4 + a5(z, t) for one (tile j of W plane positions, field c)
// ---------------------------------------------------------------------------
// ptab: four tables 4 sin^2(pi n / L_mu), indexed by position along the axis
// after the forward transforms (x table first), i.e. for the mode
// n = mode_of_position(L_mu, pos).
// accel = 1: factor c0 / p^2 with c0 = (alpha/2) p2max / V, zero at p = 0;
// accel = 0 (plain steepest descent): the constant c0 = (alpha/2) / V.
// Learned step (a10): band of every spectrum position of the tile being
// transformed (btab: one int8 per position of a tile, in the layout of one
// field of a Delta chunk, -1 for p = 0), and the per-band factors s_b that
// multiply the factor.
struct SpectralScale {
    const double* tx;
    const double* ty;
    const double* tz;
    const double* tt;
    double c0;
    int accel;
    const int8_t* btab = nullptr;   // this tile's band table, or NULL (plain step)
    const double* sb = nullptr;     // 16 factors
    __device__ __forceinline__ double factor(double p2) const
    {
        return accel ? (p2 > 0.0 ? c0 / p2 : 0.0) : c0;
    }
};

__device__ __forceinline__ SpectralScale make_scale(const Geo& geo, const double* ptab, double c0, int accel)
{
    return SpectralScale{ptab, ptab + geo.L[0], ptab + geo.L[0] + geo.L[1], ptab + geo.L[0] + geo.L[1] + geo.L[2],
                         c0, accel, nullptr, nullptr};
}

// Bands of the modes one t-axis task holds: G bytes, aligned to G.
template <int G>
struct alignas(G) BandBytes {
    int8_t b[G];
};

// Values per register group of the t-axis DFT of a line of L points.
__host__ __device__ constexpr int zt_group(int L) { return fft_r2(L) > 1 ? fft_r2(L) : fft_r1(L); }

// The t axis of the (z, t) block: forward DFT, spectral factor and inverse
// DFT of each contiguous group in registers, between the two A passes.
// LEARNED: the factor is multiplied by s_b of the mode's band, and the
// thread adds |Dhat(p)|^2 (before scaling) to bands[b] (the band powers the
// next update's factors come from).  The band table of a tile holds the
// bands of one task's G modes together: byte ((g Lz + z) W + w) G + k is
// the band of t position g G + k, z position z, plane position w of the
// tile (-1 for the zero mode); sc.sb points to the 16 factors in LDS.
template <typename T, int LT, bool LEARNED = false>
__device__ void zt_t_axis(C2<T>* buf, const Lines a, const C2<T>* __restrict__ tw, int tid, int nth,
                          const SpectralScale& sc, const Geo& geo, int logWb, int pxy0, double* bands = nullptr)
{
    constexpr int R1 = fft_r1(LT), R2 = fft_r2(LT);
    constexpr int G = R2 > 1 ? R2 : R1;            // values per register group
    if (R2 > 1) fft_pass_a<T, R1, R2, false>(buf, a, tw, tid, nth);
    const int ntask = (R2 > 1 ? R1 : 1) << a.lo_log;
    const int es = a.es;
    for (int t = tid; t < ntask; t += nth) {
        const int lo = t & ((1 << a.lo_log) - 1);          // (z, w) line
        const int j1 = R2 > 1 ? (t >> a.lo_log) : 0;
        const int w = lo & ((1 << logWb) - 1), zp = lo >> logWb;
        const int pxy = pxy0 + w;
        const double base = sc.tx[pxy & (geo.L[0] - 1)] + sc.ty[pxy >> geo.logL[0]] + sc.tz[zp];
        C2<T>* p = buf + lo + j1 * R2 * es;
        BandBytes<G> bb;
        if constexpr (LEARNED) {
            static_assert(G == zt_group(LT), "band table groups follow the t-axis register groups");
            bb = *reinterpret_cast<const BandBytes<G>*>(
                sc.btab + ((int64_t)(((j1 << geo.logL[2]) + zp) * geo.W + (pxy & (geo.W - 1))) * G));
        }
        C2<T> u[G];
#pragma unroll
        for (int k = 0; k < G; ++k) u[k] = p[k * es];
        dft<T, G, false>(u);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            double f = sc.factor(base + sc.tt[j1 * R2 + k]);
            if constexpr (LEARNED) {
                const int b = bb.b[k];
                if (b >= 0) {
                    const double pw = (double)u[k].x * u[k].x + (double)u[k].y * u[k].y;
#pragma unroll
                    for (int q = 0; q < 16; ++q) bands[q] += (q == b) ? pw : 0.0;
                    f *= sc.sb[b];
                }
            }
            u[k] = scale(u[k], (T)f);
        }
        dft<T, G, true>(u);
#pragma unroll
        for (int k = 0; k < G; ++k) p[k * es] = u[k];
    }
    __syncthreads();
    if (R2 > 1) fft_pass_a<T, R1, R2, true>(buf, a, tw, tid, nth);
}

// One block's share of a (z, t) tile: the W plane positions of tile j are
// split into parts of Wb = 2^logWb positions, and part h of field c is
// transformed here (Wb = W: the whole tile).  The tile in global memory has
// rows of W positions per (z, t) point; the LDS block has rows of Wb.  The
// first z pass reads its lines straight from Din and the last one writes
// them to Dout (the same buffer for the plain step).
template <typename T, int LMAX, bool LEARNED = false>
__device__ void zt_block(const Geo& geo, int j, int c, int h, int logWb, const C2<T>* __restrict__ Din,
                         C2<T>* __restrict__ Dout, const C2<T>* __restrict__ twz, const C2<T>* __restrict__ twt,
                         const SpectralScale& sc, C2<T>* buf, double* bands = nullptr)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int W = geo.W, Wb = 1 << logWb;
    const int64_t off = (int64_t)(j * 4 + c) * geo.DS + h * Wb;
    const int Lz = geo.L[2];
    const Lines zg{logWb, geo.logL[3], 1, Lz * W, W};
    const Lines zl{logWb, geo.logL[3], 1, Lz * Wb, Wb};
    const Lines tl{geo.logL[2] + logWb, 0, 1, 0, Lz * Wb};
    const int pxy0 = j * W + h * Wb;
    fft_fwd<T, LMAX>(Din + off, zg, buf, Lz, zl, twz, tid, nth);
    switch (geo.L[3]) {
    case 4: zt_t_axis<T, 4, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands); break;
    case 8: zt_t_axis<T, 8, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands); break;
    case 16: zt_t_axis<T, 16, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands); break;
    case 32: zt_t_axis<T, 32, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands); break;
    case 64: zt_t_axis<T, 64, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands); break;
    default:
        if constexpr (LMAX >= 128) zt_t_axis<T, 128, LEARNED>(buf, tl, twt, tid, nth, sc, geo, logWb, pxy0, bands);
        break;
    }
    fft_inv<T, LMAX>(buf, zl, Dout + off, zg, Lz, twz, tid, nth);
}

template <typename T, int LMAX>
__device__ void zt_block(const Geo& geo, int j, int c, C2<T>* __restrict__ D, const C2<T>* __restrict__ twz,
                         const C2<T>* __restrict__ twt, const SpectralScale& sc, C2<T>* buf)
{
    zt_block<T, LMAX>(geo, j, c, 0, geo.logW, D, D, twz, twt, sc, buf);
}

// ---------------------------------------------------------------------------
// a5(x, y) + a6 + a8 for one plane q: inverse (x, y) FFT,
// g = reunit(1 + dtilde) and Gout = reunit(g Gin), both in FP64.
// ---------------------------------------------------------------------------
// g from the packed filtered Delta (alpha/2 folded in): reunit(1 + dtilde),
// or exp(dtilde) when expo; then Gout(site) = reunit(g Gt), all in FP64.
template <typename T, bool EXPO>
__device__ __forceinline__ void gauge_site(const C2<double> c[4], const M3<T>& Gt, C2<T>* __restrict__ Gout,
                                           int64_t VS, int64_t site)
{
    M3<double> m;
    if constexpr (EXPO) alg_exp(c, m);
    else one_plus_alg_reunit(c, m);
    M3<double> Gd = cast_mat<double>(Gt), r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.e[3 * i + k] = cfma(m.e[3 * i + 2], Gd.e[6 + k], cfma(m.e[3 * i + 1], Gd.e[3 + k], cmul(m.e[3 * i], Gd.e[k])));
    reunit(r);
    store_mat<T, kGE>(cast_mat<T>(r), Gout, VS, site);
}

template <typename T, int NE, int LMAX, bool EXPO = false>
__device__ void gauge_plane(const Geo& geo, int q, const C2<T>* __restrict__ D, const C2<T>* __restrict__ Gin,
                            C2<T>* __restrict__ Gout, const C2<T>* __restrict__ twx, const C2<T>* __restrict__ twy,
                            C2<T>* buf)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int NP = geo.NP, W = geo.W;
    const int64_t VS = geo.VS;
    gather_to_lds<8>(
        buf, D, 4 * NP, tid, nth,
        [&](int i) {
            const int c = i >> geo.logNP, p = i & (NP - 1);
            return (int64_t)((p >> geo.logW) * 4 + c) * geo.DS + (int64_t)q * W + (p & (W - 1));
        },
        [&](int i) { return plane_lds_index(geo, i >> geo.logNP, i & (NP - 1)); });
    // G of each thread's first PF sites, loaded into registers here so that
    // the loads complete while the FFT runs in LDS
    const int64_t q0 = (int64_t)q * NP;
    constexpr int PF = 4;
    C2<T> gpre[PF][kGE];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int p = tid + k * nth;
        if (p < NP) {
#pragma unroll
            for (int e = 0; e < kGE; ++e) gpre[k][e] = Gin[e * VS + q0 + p];
        }
    }
    __syncthreads();
    fft_inv<T, LMAX>(buf, geo.L[1], Lines{geo.logL[0], 2, 1, geo.NPP, geo.RP}, twy, tid, nth);
    fft_inv<T, LMAX>(buf, geo.L[0], Lines{geo.logL[1], 2, geo.RP, geo.NPP, 1}, twx, tid, nth);
    auto update = [&](int p, const M3<T>& Gt) {
        C2<double> c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const C2<T> v = buf[plane_lds_index(geo, k, p)];
            c[k] = mk<double>((double)v.x, (double)v.y);
        }
        gauge_site<T, EXPO>(c, Gt, Gout, VS, q0 + p);
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int p = tid + k * nth;
        if (p < NP) {
            M3<T> Gt;
#pragma unroll
            for (int e = 0; e < kGE; ++e) Gt.e[e] = gpre[k][e];
            rebuild_row3(Gt);
            update(p, Gt);
        }
    }
    for (int p = tid + PF * nth; p < NP; p += nth) {
        M3<T> Gt;
        load_mat<T, kGE>(Gt, Gin, VS, q0 + p);
        update(p, Gt);
    }
}

// The same update with the inverse (x, y) FFT done two fields at a time in a
// plane buffer of 2 fields (half the LDS of gauge_plane, so more blocks fit
// on a CU).  Each thread keeps the transformed fields 0 and 1 of its sites
// (at most MAXS sites: NP <= MAXS * blockDim) in registers while fields 2
// and 3 go through the buffer; G of its first PF sites is loaded into
// registers before the second transform.
template <typename T, int NE, int LMAX, int MAXS, int PF, bool EXPO = false>
__device__ void gauge_plane_2f(const Geo& geo, int q, const C2<T>* __restrict__ D, const C2<T>* __restrict__ Gin,
                               C2<T>* __restrict__ Gout, const C2<T>* __restrict__ twx, const C2<T>* __restrict__ twy,
                               C2<T>* buf)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int NP = geo.NP, W = geo.W;
    const int64_t VS = geo.VS;
    const int64_t q0 = (int64_t)q * NP;
    const Lines ly{geo.logL[0], 1, 1, geo.NPP, geo.RP};
    const Lines lx{geo.logL[1], 1, geo.RP, geo.NPP, 1};
    C2<T> keep[MAXS][2];
    C2<T> gpre[PF > 0 ? PF : 1][kGE];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        gather_to_lds<8>(
            buf, D, 2 * NP, tid, nth,
            [&](int i) {
                const int c = 2 * half + (i >> geo.logNP), p = i & (NP - 1);
                return (int64_t)((p >> geo.logW) * 4 + c) * geo.DS + (int64_t)q * W + (p & (W - 1));
            },
            [&](int i) { return plane_lds_index(geo, i >> geo.logNP, i & (NP - 1)); });
        if (half == 1) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int p = tid + k * nth;
                if (p < NP) {
#pragma unroll
                    for (int e = 0; e < kGE; ++e) gpre[k][e] = Gin[e * VS + q0 + p];
                }
            }
        }
        __syncthreads();
        fft_inv<T, LMAX>(buf, geo.L[1], ly, twy, tid, nth);
        fft_inv<T, LMAX>(buf, geo.L[0], lx, twx, tid, nth);
        if (half == 0) {
#pragma unroll
            for (int k = 0; k < MAXS; ++k) {
                const int p = tid + k * nth;
                if (p < NP) {
                    keep[k][0] = buf[plane_lds_index(geo, 0, p)];
                    keep[k][1] = buf[plane_lds_index(geo, 1, p)];
                }
            }
            __syncthreads();
        }
    }
    auto update = [&](int p, const C2<T>* v01, const M3<T>& Gt) {
        C2<double> c[4];
        c[0] = mk<double>((double)v01[0].x, (double)v01[0].y);
        c[1] = mk<double>((double)v01[1].x, (double)v01[1].y);
#pragma unroll
        for (int k = 2; k < 4; ++k) {
            const C2<T> v = buf[plane_lds_index(geo, k - 2, p)];
            c[k] = mk<double>((double)v.x, (double)v.y);
        }
        gauge_site<T, EXPO>(c, Gt, Gout, VS, q0 + p);
    };
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
        const int p = tid + k * nth;
        if (p < NP) {
            M3<T> Gt;
            if (k < PF) {
#pragma unroll
                for (int e = 0; e < kGE; ++e) Gt.e[e] = gpre[k < PF ? k : 0][e];
                rebuild_row3(Gt);
            } else {
                load_mat<T, kGE>(Gt, Gin, VS, q0 + p);
            }
            update(p, keep[k], Gt);
        }
    }
}

// ---------------------------------------------------------------------------
// a7: F = sum/(12V), theta = sum/(3V) over the per-plane partials in plane
// order (one block).  counts_update: the partials are of the links of the
// gauge just formed, so the update is counted and that gauge becomes current
// (cur flips).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_state(const double* __restrict__ partial, int nq, int64_t V, DevState* st,
                             double* __restrict__ trace, int counts_update, double* red, int nsum = 0)
{
    // the sums run over the first nsum threads (all of them when 0), so a
    // larger block adds in the same order as a 256-thread k_reduce
    const int tid = threadIdx.x, nth = nsum > 0 ? nsum : (int)blockDim.x;
    double a = 0.0, b = 0.0;
    if (tid < nth)
        for (int i = tid; i < nq; i += nth) {
            a += partial[2 * i];
            b += partial[2 * i + 1];
        }
    double fs, ts;
    block_sum2(a, b, red, tid, nth, &fs, &ts);
    if (tid == 0 && counts_update == 2) {          // candidate links of a learned step: no commit
        st->trial_F = fs / (12.0 * (double)V);
        st->trial_theta = ts / (3.0 * (double)V);
    } else if (tid == 0) {
        const double F = fs / (12.0 * (double)V), th = ts / (3.0 * (double)V);
        if (counts_update) {
            st->iter += 1;
            if (st->phase == 0) st->iter_fp32 += 1;
            st->cur ^= 1;
        }
        st->needs_measure = 0;
        st->F = F;
        st->theta = th;
        if (trace) {
            trace[0] = F;
            trace[1] = th;
        }
        if (!(th == th) || th > 1e300) {
            st->nonfinite = 1;
            st->done = 1;
        } else if (st->mixed && st->phase == 0) {
            if (th < st->theta_switch) st->switch_pending = 1;
            else if (st->iter >= st->max_iter) st->done = 1;
        } else if (th < st->theta_stop || st->iter >= st->max_iter) {
            st->done = 1;
        }
    }
    __syncthreads();
}

// ===========================================================================
// learned step: network on the band powers
// ===========================================================================
__device__ __forceinline__ float bf16_to_float(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Network 16 -> 64 -> 64 -> 16 (ReLU), bf16 weights [in][out] row-major,
// float32 biases, float32 accumulation.
struct MlpDev {
    const uint16_t* W1;
    const uint16_t* W2;
    const uint16_t* W3;
    const float* b1;
    const float* b2;
    const float* b3;
};

// LDS bytes band_factors works in.
constexpr int kBandLdsBytes = 256 * 8 + (16 + 64 + 64 + 256) * 4;

// Band powers -> features -> factors s_b = exp(clip(y_b, -2.3, 2.3)), by one
// block of any size (a multiple of 64): the work is laid out for 256 virtual
// threads, which the block's threads take in turn, so the result does not
// depend on the block size.  The per-block band sums (nblk rows of 16) are
// added in a fixed order: virtual thread v adds elements v, v + 256, ... of
// the flat array (all of band v mod 16, four running sums), then a tree over
// the virtual threads of each band.  Empty bands (count 0) get feature 0.
// Each layer's dot products are split over the virtual threads and their
// parts added in a fixed order.  Without a network (net.W1 NULL) s = 1.
// lds: kBandLdsBytes.  Ends with a barrier.
__device__ __forceinline__ void band_factors(const double* __restrict__ band_partial, int nblk,
                                             const double* __restrict__ count16, int64_t V, const MlpDev& net,
                                             double* __restrict__ s_out, double* __restrict__ x_out, double* lds)
{
    double* red = lds;
    float* x = reinterpret_cast<float*>(lds + 256);
    float* h1 = x + 16;
    float* h2 = h1 + 64;
    float* part = h2 + 64;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int64_t n = (int64_t)nblk * 16;
    for (int v = tid; v < 256; v += nth) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t e = v;
        for (; e + 768 < n; e += 1024) {
            a0 += band_partial[e];
            a1 += band_partial[e + 256];
            a2 += band_partial[e + 512];
            a3 += band_partial[e + 768];
        }
        for (; e < n; e += 256) a0 += band_partial[e];
        red[v] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    for (int h = 128; h >= 16; h >>= 1) {
        for (int v = tid; v < h; v += nth) red[v] += red[v + h];
        __syncthreads();
    }
    if (tid < 16) {
        const double p = red[tid];
        double f = 0.0;
        if (count16[tid] > 0.0) {
            const double pv = p / count16[tid] / (double)V;
            f = log10(pv > 1e-300 ? pv : 1e-300) / 8.0;
        }
        x[tid] = (float)f;
        if (x_out) x_out[tid] = f;
    }
    __syncthreads();
    if (!net.W1) {
        if (tid < 16) s_out[tid] = 1.0;
        __syncthreads();
        return;
    }
    if (tid < 64) {
        float a = net.b1[tid];
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(x[i], bf16_to_float(net.W1[i * 64 + tid]), a);
        h1[tid] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int v = tid; v < 256; v += nth) {   // layer 2: output v mod 64, inputs [16 k, 16 k + 16), k = v / 64
        const int o = v & 63, k = v >> 6;
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(h1[16 * k + i], bf16_to_float(net.W2[(16 * k + i) * 64 + o]), a);
        part[v] = a;
    }
    __syncthreads();
    if (tid < 64) {
        const float a = ((net.b2[tid] + part[tid]) + part[64 + tid]) + (part[128 + tid] + part[192 + tid]);
        h2[tid] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int v = tid; v < 256; v += nth) {   // layer 3: output v mod 16, inputs [4 k, 4 k + 4), k = v / 16
        const int o = v & 15, k = v >> 4;
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) a = fmaf(h2[4 * k + i], bf16_to_float(net.W3[(4 * k + i) * 16 + o]), a);
        part[v] = a;
    }
    __syncthreads();
    if (tid < 16) {
        float a = net.b3[tid];
        for (int k = 0; k < 16; ++k) a += part[16 * k + tid];
        const double y = fmin(fmax((double)a, -2.3), 2.3);
        s_out[tid] = exp(y);
    }
    __syncthreads();
}

// Work of the block that computes the next update's factors inside the
// candidate's measure launch of a learned update (s_out NULL: none), and the
// blocks that launch gets in front of its planes.
constexpr int kBandSideBlocks = 8;
struct BandJob {
    const double* band_partial;
    int nblk;
    int pad;
    const double* count16;
    int64_t V;
    MlpDev net;
    double* s_out;
};

// ===========================================================================
// single-configuration kernels (one lattice per launch)
// ===========================================================================
// The links are never stored: they are G(x) Uref(x) G^dag(x+mu) for the
// reference links Uref (those loaded) and the accumulated gauge G, kept in a
// pair of buffers.  next = 0 measures the current G (G[cur]); next = 1 the
// one k_gauge has just formed (G[1 - cur]).
// ONCE: the link-once plane function (x extent <= 64), else the one that
// forms every link at both of its sites.
// D1 (learned step only, else NULL): a second Delta buffer; Delta of the
// current links is in D if st->dsel = 0, else in D1, and the links of the
// gauge just formed (next = 1) write the other one, so a rejected candidate
// leaves the current Delta in place.
// job.s_out (learned step's candidate only, else NULL): the launch has
// kBandSideBlocks more blocks in front of the planes (the plane to XCD map is
// kept); the first of them runs band_factors for the next update's factors,
// the others return.
template <typename T, int NE, int LMAX, bool ONCE>
__global__ void __launch_bounds__(256) k_measure(Geo geo, const C2<T>* __restrict__ Uref, const C2<T>* G0,
                                                 const C2<T>* G1, int next, C2<T>* D0, C2<T>* D1,
                                                 double* __restrict__ partial, const C2<T>* __restrict__ twx,
                                                 const C2<T>* __restrict__ twy, const DevState* __restrict__ st,
                                                 BandJob job)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    int b = blockIdx.x;
    if (job.s_out) {
        if (b == 0)
            band_factors(job.band_partial, job.nblk, job.count16, job.V, job.net, job.s_out, nullptr, lds_raw);
        if (b < kBandSideBlocks) return;
        b -= kBandSideBlocks;
    }
    const C2<T>* G = (st->cur ^ next) ? G1 : G0;
    C2<T>* D = (D1 && ((st->dsel ^ next) & 1)) ? D1 : D0;
    const int q = plane_of_block(b, geo);
    C2<T>* buf = reinterpret_cast<C2<T>*>(lds_raw + 2 * blockDim.x);
    if constexpr (ONCE) measure_plane_once<T, NE, LMAX>(geo, q, Uref, G, D, partial, twx, twy, lds_raw, buf);
    else measure_plane<T, NE, LMAX>(geo, q, Uref, G, D, partial, twx, twy, lds_raw, buf);
}

// Part h and (tile, field) chunk of block b of a (z, t) launch with
// 2^lnh parts per chunk (blocks = chunks << lnh).  When the chunks are a
// multiple of 8, the parts of one chunk go to blocks of one XCD (blocks are
// dealt to the 8 XCDs round robin), so each cache line of the chunk is read
// into one L2; otherwise the parts of a chunk are consecutive blocks.
__host__ __device__ __forceinline__ void zt_part_of_block(int b, int nchunk, int lnh, int& h, int& chunk)
{
    if (lnh == 0) {
        h = 0;
        chunk = b;
    } else if ((nchunk & 7) == 0) {
        const int xcd = b & 7, l = b >> 3;
        h = l & ((1 << lnh) - 1);
        chunk = ((l >> lnh) << 3) | xcd;
    } else {
        h = b & ((1 << lnh) - 1);
        chunk = b >> lnh;
    }
}

// One block per (tile, field, part of 2^logWb plane positions).
template <typename T, int LMAX>
__global__ void __launch_bounds__(512) k_zt(Geo geo, C2<T>* __restrict__ D, const C2<T>* __restrict__ twz,
                                            const C2<T>* __restrict__ twt, const double* __restrict__ ptab,
                                            double c0, int accel, int logWb, const DevState* __restrict__ st)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    int h, chunk;
    zt_part_of_block(blockIdx.x, (geo.NP >> geo.logW) * 4, geo.logW - logWb, h, chunk);
    zt_block<T, LMAX>(geo, chunk >> 2, chunk & 3, h, logWb, D, D, twz, twt, make_scale(geo, ptab, c0, accel),
                      reinterpret_cast<C2<T>*>(lds_raw));
}

// k_zt preceded, in block 0, by the reduction of the F and theta partials of
// the measure launched before it, committed as k_reduce with counts_update = 1
// commits them.  Inside a captured chunk of updates, update n's reduction
// thus runs in update n + 1's (z, t) launch instead of a launch of its own.
// The blocks that start after block 0 has raised `done` return; those that
// started before transform D all the same, so after a chunk that ends done D
// no longer holds the Delta of the current links.  The sums run over 256
// threads, as in k_reduce, so F and theta come out bit for bit the same.
// LDS: at least 2 * 512 doubles for the reduction.
template <typename T, int LMAX>
__global__ void __launch_bounds__(512) k_zt_reduce(Geo geo, C2<T>* __restrict__ D, const C2<T>* __restrict__ twz,
                                                   const C2<T>* __restrict__ twt, const double* __restrict__ ptab,
                                                   double c0, int accel, int logWb, DevState* st,
                                                   const double* __restrict__ partial)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    if (blockIdx.x == 0) reduce_state(partial, geo.NQ, geo.V, st, nullptr, 1, lds_raw, 256);
    int h, chunk;
    zt_part_of_block(blockIdx.x, (geo.NP >> geo.logW) * 4, geo.logW - logWb, h, chunk);
    zt_block<T, LMAX>(geo, chunk >> 2, chunk & 3, h, logWb, D, D, twz, twt, make_scale(geo, ptab, c0, accel),
                      reinterpret_cast<C2<T>*>(lds_raw));
}

// G[1 - cur] <- reunit(g G[cur]) with g = reunit(1 + dtilde) from D.
// EXPO: g = exp(dtilde) (LGF_UPDATE_EXP) instead of reunit(1 + dtilde).
template <typename T, int NE, int LMAX, bool EXPO>
__global__ void __launch_bounds__(256) k_gauge(Geo geo, const C2<T>* __restrict__ D, C2<T>* G0, C2<T>* G1,
                                               const C2<T>* __restrict__ twx, const C2<T>* __restrict__ twy,
                                               const DevState* __restrict__ st)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    const int cur = st->cur;
    gauge_plane<T, NE, LMAX, EXPO>(geo, plane_of_block(blockIdx.x, geo), D, cur ? G1 : G0, cur ? G0 : G1, twx, twy,
                                   reinterpret_cast<C2<T>*>(lds_raw));
}

// The same with the inverse (x, y) FFT two fields at a time in half the LDS;
// for planes of exactly 4 sites per thread (kGauge2fSites).
constexpr int kGauge2fSites = 4;

template <typename T, int NE, int LMAX, bool EXPO>
__global__ void __launch_bounds__(256) k_gauge2f(Geo geo, const C2<T>* __restrict__ D, C2<T>* G0, C2<T>* G1,
                                                 const C2<T>* __restrict__ twx, const C2<T>* __restrict__ twy,
                                                 const DevState* __restrict__ st)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    const int cur = st->cur;
    gauge_plane_2f<T, NE, LMAX, kGauge2fSites, 0, EXPO>(geo, plane_of_block(blockIdx.x, geo), D, cur ? G1 : G0,
                                                       cur ? G0 : G1, twx, twy, reinterpret_cast<C2<T>*>(lds_raw));
}

template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partial, int nq, int64_t V,
                                                DevState* __restrict__ st, double* __restrict__ trace,
                                                int counts_update)
{
    if (st->done) return;
    __shared__ double red[2 * 256];
    reduce_state(partial, nq, V, st, trace, counts_update, red);
}

// ---------------------------------------------------------------------------
// a9: precision switch.  U_mu(x) = G(x) U0_mu(x) G^dag(x + mu) in FP64 from
// the FP64 links as loaded and the FP32-accumulated gauge, reunitarised in
// FP64 (so the result lies exactly on the gauge orbit of the input); the
// promoted gauge is stored as G64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void promote_site(int64_t VS32, int64_t VS64, int64_t s, const C2<float>* __restrict__ G32,
                                             C2<double>* __restrict__ G64)
{
    M3<float> a;
    load_mat<float, kGE>(a, G32, VS32, s);
    M3<double> m = cast_mat<double>(a);
    reunit(m);
    store_mat<double, kGE>(m, G64, VS64, s);
}

template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_promote_gauge(int64_t V, int64_t VS32, int64_t VS64,
                                                       const C2<float>* __restrict__ G32, C2<double>* __restrict__ G64)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < V) promote_site(VS32, VS64, s, G32, G64);
}

// ===========================================================================
// batched kernels: many lattices of different shapes per launch (a11)
// ===========================================================================
// One descriptor per configuration and precision.  Work items are
// (configuration, plane) for the plane kernels and (configuration, tile,
// field) for the (z, t) kernel, packed as cfg << 20 | index.  Every kernel
// walks its item list with a grid-stride loop (a persistent grid sized to
// the device), and skips the items of configurations that are not in the
// kernel's phase (FP32 / FP64, measure / update) or are done.
template <typename T>
struct BatchCfg {
    Geo geo;
    const C2<T>* U;         // reference (loaded) links; the links are G U G^dag(x+mu)
    C2<T>* G[2];            // accumulated gauge, G[cur] current
    C2<T>* D;
    const C2<T>* tw[4];
    const double* ptab;
    double* partial;
    DevState* st;
    double c0;
    int accel;
    int pad;
};

constexpr int kItemShift = 20;

// gate: 0 = fresh measure of configurations that need one, 1 = update
__device__ __forceinline__ bool batch_active(const DevState* st, int phase, int gate)
{
    if (st->done || st->switch_pending || st->phase != phase) return false;
    return gate == 0 ? st->needs_measure != 0 : st->needs_measure == 0;
}

// NEXT = false: measure the links of the current gauge G[cur] (members that
// need a measure); NEXT = true: those of the gauge k_gauge just formed.
template <typename T, int NE, bool NEXT, int LMAX, bool ONCE>
__global__ void __launch_bounds__(256) kb_measure(const BatchCfg<T>* __restrict__ cfgs, const uint32_t* __restrict__ items,
                                                  int nitems, int phase)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t w = items[it];
        const BatchCfg<T>& bc = cfgs[w >> kItemShift];
        if (!batch_active(bc.st, phase, NEXT ? 1 : 0)) continue;
        const int sel = bc.st->cur ^ (NEXT ? 1 : 0);
        __syncthreads();
        const int q = (int)(w & ((1u << kItemShift) - 1));
        C2<T>* buf = reinterpret_cast<C2<T>*>(lds_raw + 2 * blockDim.x);
        if constexpr (ONCE)
            measure_plane_once<T, NE, LMAX>(bc.geo, q, bc.U, bc.G[sel], bc.D, bc.partial, bc.tw[0], bc.tw[1], lds_raw,
                                            buf);
        else
            measure_plane<T, NE, LMAX>(bc.geo, q, bc.U, bc.G[sel], bc.D, bc.partial, bc.tw[0], bc.tw[1], lds_raw, buf);
    }
}

template <typename T, int LMAX>
__global__ void __launch_bounds__(512) kb_zt(const BatchCfg<T>* __restrict__ cfgs, const uint32_t* __restrict__ items,
                                             int nitems, int phase)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t w = items[it];
        const BatchCfg<T>& bc = cfgs[w >> kItemShift];
        if (!batch_active(bc.st, phase, 1)) continue;
        const int jc = (int)(w & ((1u << kItemShift) - 1));
        __syncthreads();
        zt_block<T, LMAX>(bc.geo, jc >> 2, jc & 3, bc.D, bc.tw[2], bc.tw[3], make_scale(bc.geo, bc.ptab, bc.c0, bc.accel),
                          reinterpret_cast<C2<T>*>(lds_raw));
    }
}

template <typename T, int NE, int LMAX, bool EXPO>
__global__ void __launch_bounds__(256) kb_gauge(const BatchCfg<T>* __restrict__ cfgs, const uint32_t* __restrict__ items,
                                                int nitems, int phase)
{
    HIP_DYNAMIC_SHARED(double, lds_raw)
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t w = items[it];
        const BatchCfg<T>& bc = cfgs[w >> kItemShift];
        if (!batch_active(bc.st, phase, 1)) continue;
        __syncthreads();
        const int cur = bc.st->cur;
        gauge_plane<T, NE, LMAX, EXPO>(bc.geo, (int)(w & ((1u << kItemShift) - 1)), bc.D, bc.G[cur],
                                       bc.G[cur ^ 1], bc.tw[0], bc.tw[1], reinterpret_cast<C2<T>*>(lds_raw));
    }
}

// one block per configuration
template <typename T>
__global__ void __launch_bounds__(256) kb_reduce(const BatchCfg<T>* __restrict__ cfgs, int phase, int gate)
{
    __shared__ double red[2 * 256];
    const BatchCfg<T>& bc = cfgs[blockIdx.x];
    if (!batch_active(bc.st, phase, gate)) return;
    reduce_state(bc.partial, bc.geo.NQ, bc.geo.V, bc.st, nullptr, gate, red);
}

// Mixed runs: the FP32 phase of a configuration ended (switch_pending).
// Step 1: G64[0] = reunit(G32[cur]); step 2: FP64 phase with cur = 0, whose
// links are G64 U0 G64^dag(x+mu) for the loaded FP64 links, to be measured.
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) kb_promote(const BatchCfg<float>* __restrict__ c32,
                                                  const BatchCfg<double>* __restrict__ c64,
                                                  const uint32_t* __restrict__ items, int nitems)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t w = items[it];
        const int cfg = (int)(w >> kItemShift);
        if (!c64[cfg].st->switch_pending || c64[cfg].st->done) continue;
        const Geo& geo = c64[cfg].geo;
        const int64_t q0 = (int64_t)(w & ((1u << kItemShift) - 1)) * geo.NP;
        for (int p = threadIdx.x; p < geo.NP; p += blockDim.x)
            promote_site(c32[cfg].geo.VS, geo.VS, q0 + p, c32[cfg].G[c64[cfg].st->cur], c64[cfg].G[0]);
    }
}

template <int UNUSED = 0>
__global__ void kb_switch_done(const BatchCfg<double>* __restrict__ c64, int ncfg)
{
    const int cfg = blockIdx.x * blockDim.x + threadIdx.x;
    if (cfg >= ncfg) return;
    DevState* st = c64[cfg].st;
    if (!st->switch_pending || st->done) return;
    st->switch_pending = 0;
    st->phase = 1;
    st->cur = 0;
    st->needs_measure = 1;
}

// ===========================================================================
// a10: learned spectral step
// ===========================================================================
// The factor (alpha/2) p2max / (p^2 V) of mode p is multiplied by s_b of the
// mode's band b: 16 bands log-spaced between the smallest nonzero p^2 of the
// lattice and p2max (the zero mode has none).  The factors used by an update
// come from the network applied to the band powers of the previous update's
// spectrum (s = 1 for the first update after a load), so each update makes a
// single (z, t) pass that applies the factors and adds up the band powers of
// the spectrum it transforms, and the network runs in the one-block
// reduction that follows the update.

// Block sum of 16 per-thread values in a fixed order; the 16 sums go to out.
// Within a wavefront the values are halved over lanes four times (lane bit
// 5, 4, 3, 2 selects which half of the remaining values a lane keeps and
// adds its partner's share to), which leaves band
// q = 8 b5 + 4 b4 + 2 b3 + b2 on lanes with those bits; two more exchanges
// add the four lanes of each band.  wred: 16 * (blockDim / 64) doubles of
// LDS.
// One halving step of block_sum16: H values kept of 2 H, partner lane ^ 4 H.
// (A template per step: every index into v is a constant, so v stays in
// registers.)
template <int H>
__device__ __forceinline__ void halve_over_lanes(double* v, int lane)
{
    constexpr int m = 4 * H;
    const bool upper = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double give = upper ? v[i] : v[i + H];
        const double keep = upper ? v[i + H] : v[i];
        v[i] = keep + __shfl(give, lane ^ m);
    }
}

__device__ __forceinline__ void block_sum16(double* v, double* wred, double* __restrict__ out)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (blockDim.x + 63) >> 6;
    halve_over_lanes<8>(v, lane);
    halve_over_lanes<4>(v, lane);
    halve_over_lanes<2>(v, lane);
    halve_over_lanes<1>(v, lane);
    double a = v[0];
    a += __shfl(a, lane ^ 2);
    a += __shfl(a, lane ^ 1);
    const int q = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
    if ((lane & 3) == 0) wred[q * nw + wave] = a;
    __syncthreads();
    if (tid < 16) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += wred[tid * nw + w];
        out[tid] = t;
    }
}

// One block per (tile, field, part) as k_zt: forward (z, t) FFT of the
// current Delta (buffer st->dsel of D0, D1), band powers of the spectrum into
// band_partial[block][16], factors s_b (alpha/2) p2max/(p^2 V), inverse
// (z, t) FFT into Dout.  The current Delta is left as it is.  With
// plain_after_reject, s = 1 while st->fallback is raised (the plain update
// that replaces a rejected candidate).
template <typename T, int LMAX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(LMAX == 64 ? 4 : 1))) k_zt_learned(Geo geo, const C2<T>* D0, const C2<T>* D1, C2<T>* __restrict__ Dout,
                                                    const C2<T>* __restrict__ twz, const C2<T>* __restrict__ twt,
                                                    const double* __restrict__ ptab, double c0, int accel, int logWb,
                                                    const int8_t* __restrict__ btab, const double* __restrict__ sb,
                                                    int plain_after_reject, double* __restrict__ band_partial,
                                                    const DevState* __restrict__ st)
{
    if (st->done) return;
    HIP_DYNAMIC_SHARED(double, lds_raw)
    __shared__ double wred[16 * 8];
    __shared__ double s_lds[16];
    // read after the forward z pass's barrier
    if (threadIdx.x < 16) s_lds[threadIdx.x] = (plain_after_reject && st->fallback) ? 1.0 : sb[threadIdx.x];
    int h, chunk;
    zt_part_of_block(blockIdx.x, (geo.NP >> geo.logW) * 4, geo.logW - logWb, h, chunk);
    const int j = chunk >> 2;
    SpectralScale sc = make_scale(geo, ptab, c0, accel);
    sc.btab = btab + (int64_t)j * geo.NQ * geo.W;
    sc.sb = s_lds;
    double bands[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) bands[q] = 0.0;
    zt_block<T, LMAX, true>(geo, j, chunk & 3, h, logWb, (st->dsel & 1) ? D1 : D0, Dout, twz, twt, sc,
                            reinterpret_cast<C2<T>*>(lds_raw), bands);
    block_sum16(bands, wred, band_partial + (int64_t)blockIdx.x * 16);
}

// Features and factors of the band powers in band_partial (lgf_learned_factors).
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_bands_mlp(const double* __restrict__ band_partial, int nblk,
                                                   const double* __restrict__ count16, int64_t V, MlpDev net,
                                                   double* __restrict__ s_out, double* __restrict__ x_out)
{
    __shared__ double lds[kBandLdsBytes / 8];
    band_factors(band_partial, nblk, count16, V, net, s_out, x_out, lds);
}

// The reduction that ends a learned update, one block.
//   mode 1 (update): F and theta of the new links.  A candidate (st->fallback
//     clear) is committed iff it raised F or lowered theta (near convergence
//     the gain in F is below its rounding; theta still resolves it); a
//     rejected one raises
//     st->fallback, and the next update (its (z, t) pass then takes s = 1)
//     is the plain update from the same Delta, committed as it is.  On
//     commit the gauge and Delta buffers flip and s_cur = s_next (the
//     factors the update's measure launch computed from its band powers).
//   mode 3 (trial of the line search): F and theta recorded as trial values.
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_reduce_learned(const double* __restrict__ partial, int nq, int64_t V,
                                                        DevState* st, double* __restrict__ trace, int mode,
                                                        double* __restrict__ s_cur, const double* __restrict__ s_next)
{
    if (st->done) return;
    __shared__ double red[2 * 256];
    __shared__ int commit;
    const int tid = threadIdx.x, nth = blockDim.x;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < nq; i += nth) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    double fs, ts;
    block_sum2(a, b, red, tid, nth, &fs, &ts);
    const double F = fs / (12.0 * (double)V), th = ts / (3.0 * (double)V);
    if (tid == 0) {
        commit = 0;
        if (mode == 3) {
            st->trial_F = F;
            st->trial_theta = th;
        } else if (st->fallback || F > st->F || th < st->theta) {
            commit = 1;
            st->fallback = 0;
            st->iter += 1;
            st->cur ^= 1;
            st->dsel ^= 1;
            st->F = F;
            st->theta = th;
            if (trace) {
                trace[0] = F;
                trace[1] = th;
            }
            if (!(th == th) || th > 1e300) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (th < st->theta_stop || st->iter >= st->max_iter) {
                st->done = 1;
            }
        } else {
            st->trial_F = F;
            st->trial_theta = th;
            st->fallback = 1;
            st->fallbacks += 1;
        }
    }
    __syncthreads();
    if (commit && tid < 16) s_cur[tid] = s_next[tid];
}

// s = 1 (the first update after a load uses the plain factors).
template <int UNUSED = 0>
__global__ void k_fill16(double* __restrict__ s, double v)
{
    if (threadIdx.x < 16) s[threadIdx.x] = v;
}

}  // namespace lgf
