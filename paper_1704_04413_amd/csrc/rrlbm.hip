// librrlbm: fused stream-and-collide recursive-regularized lattice Boltzmann
// kernels for MI355X (gfx950) and the C-ABI declared in include/rrlbm.h.
//
// Data layout in HBM: row-tiled structure of arrays.  The grid is cut into
// tiles of TY = 4 full rows; a tile stores its Q velocity planes one after the
// other (plane i of the tile = TY*nx values, row-major), so element
// (i, y, x) lives at (y / TY) * Q*TY*nx + i * TY*nx + (y % TY) * nx + x.
// A wavefront's 64 lanes touch 64 consecutive values of one plane, and the
// 2*Q streams a block reads and writes sit inside about three tiles (a few
// MiB) instead of 2*Q planes spread over the whole buffer, which keeps the
// address-translation working set small.  One step is one launch of a pull
// kernel: the thread of node x gathers f_i(x - c_i) from the source buffer (one
// fixed offset per plane, so every stored value is read exactly once),
// collides in registers and writes its Q post-collision values to the
// destination buffer, with the load and store kinds of the cache policy that
// the buffer size selects (Policy).  The two buffers alternate; the state
// kept between steps is post-collision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "collide.hpp"
#include "rrlbm.h"

namespace rr {

// ---------------------------------------------------------------- storage

struct StoreF64 {
    using elem = double;
    using math = double;
    static constexpr bool shifted = false;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = false;
    static __device__ __forceinline__ double load(const double* p) { return *p; }
    static __device__ __forceinline__ double load_nt(const double* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
    static __device__ __forceinline__ void store_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
};

struct StoreF32 {
    using elem = float;
    using math = float;
    static constexpr bool shifted = true;
    static constexpr bool conserve_in_double = true;
    static constexpr bool dithered = false;
    static __device__ __forceinline__ float load(const float* p) { return *p; }
    static __device__ __forceinline__ float load_nt(const float* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
    static __device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
};

// bfloat16 = the upper half of an IEEE float.  The initial state is rounded
// to nearest even; every step rounds stochastically (store_nt_sr): with
// deterministic rounding a near-uniform region sits at a fixed point of the
// rounded update and its 2^-9 rounding bias acts coherently over thousands of
// steps, while a rounding that is unbiased in expectation turns it into noise.
struct StoreBF16 {
    using elem = uint16_t;
    using math = float;
    static constexpr bool shifted = true;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = true;
    static __device__ __forceinline__ float load(const uint16_t* p)
    {
        return __uint_as_float(uint32_t(*p) << 16);
    }
    static __device__ __forceinline__ float load_nt(const uint16_t* p)
    {
        return __uint_as_float(uint32_t(__builtin_nontemporal_load(p)) << 16);
    }
    static __device__ __forceinline__ uint16_t round(float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u); // quiet NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    static __device__ __forceinline__ void store(uint16_t* p, float v) { *p = round(v); }
    static __device__ __forceinline__ void store_nt(uint16_t* p, float v) { __builtin_nontemporal_store(round(v), p); }
    // r: 16 uniform random bits; |v| rounds up with probability (dropped bits) / 2^16
    static __device__ __forceinline__ uint16_t round_sr(float v, uint32_t r)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u); // quiet NaN
        return uint16_t((u + r) >> 16);
    }
    static __device__ __forceinline__ void store_nt_sr(uint16_t* p, float v, uint32_t r)
    {
        __builtin_nontemporal_store(round_sr(v, r), p);
    }
    static __device__ __forceinline__ void store_sr(uint16_t* p, float v, uint32_t r) { *p = round_sr(v, r); }
};

// Counter-based random bits for stochastic rounding: a function of the node
// (y nx + x of its own grid) and of the index of the state being written (0 for
// the initial state, n after n steps) only, so results do not depend on launch
// shape or batching.  The key is Wellons' "lowbias32" integer hash; the stream
// per node is the 32-bit LCG of PCG (O'Neill), of which the top 16 bits are used.
struct Dither {
    uint32_t s;
    static __device__ __forceinline__ uint32_t mix(uint32_t x)
    {
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        return x;
    }
    __device__ __forceinline__ Dither(uint32_t node, uint32_t seq) : s(mix(node ^ mix(seq * 0x9e3779b9u + 0x6a09e667u))) {}
    __device__ __forceinline__ uint32_t next16()
    {
        s = s * 747796405u + 2891336453u;
        return s >> 16;
    }
};

// Writes the Q post-collision values of one node (stochastic rounding where
// the storage asks for it).
template <class L, class S, class T, bool NT = true>
__device__ __forceinline__ void store_node(typename S::elem* __restrict__ fout, int here, int te, const T (&v)[L::Q],
                                           uint32_t node, uint32_t seq)
{
    // NT: non-temporal stores, for state buffers larger than the memory-side
    // cache; ordinary stores leave the written state there for the next step
    if constexpr (S::dithered) {
        Dither dz(node, seq);
        if constexpr (NT)
            static_for<L::Q>([&](auto I) { S::store_nt_sr(fout + here + int(I) * te, v[I], dz.next16()); });
        else
            static_for<L::Q>([&](auto I) { S::store_sr(fout + here + int(I) * te, v[I], dz.next16()); });
    } else {
        if constexpr (NT)
            static_for<L::Q>([&](auto I) { S::store_nt(fout + here + int(I) * te, v[I]); });
        else
            static_for<L::Q>([&](auto I) { S::store(fout + here + int(I) * te, v[I]); });
    }
}

// ----------------------------------------------------------------- layout

constexpr int TY = 4; // rows per tile

struct Layout {
    int nx, ny;
    int te; // elements of one plane of one tile, TY * nx
    int ts; // elements of one tile, Q * te
    __host__ __device__ int row(int y) const { return (y / TY) * ts + (y % TY) * nx; }
    __host__ __device__ int off(int q, int y, int x) const { return row(y) + q * te + x; }
};

inline Layout make_layout(int q, int nx, int ny) { return Layout{ nx, ny, TY * nx, q * TY * nx }; }

inline int64_t layout_elems(int q, int nx, int ny)
{
    return int64_t((ny + TY - 1) / TY) * q * TY * nx;
}

// ------------------------------------------------------------ step kernel

constexpr int BX = 64, BY = TY;

// Minimum waves per SIMD the compiler must leave room for in the step
// kernel (register budget); more resident waves keep more loads in flight
// while other waves run the collision arithmetic.
#ifndef RRLBM_WAVES_PER_EU
#define RRLBM_WAVES_PER_EU 4
#endif

struct StepArgs {
    const void* fin;
    void* fout;
    Layout lay;
    int bx_blocks;  // blocks along x
    int nblocks;    // total blocks of the 1D grid
    int xcd_remap;  // 1: give each XCD a contiguous band of blocks
    Relax rx;       // relaxation factors of ranks 2..4 and 1/tau
    uint32_t seq;   // index of the state written (0: initial state), keys the BF16 dither
    int reverse;    // 1: walk the tiles last to first (every other step with ordinary stores)
};

// The hardware hands consecutive workgroup ids to the 8 XCDs in turn; with
// the remap, XCD k works on the k-th contiguous eighth of the tiles, so
// neighbouring tiles share that XCD's L2.
// With `reverse` the tiles are walked last to first: a step then starts on
// the tiles the previous step wrote last, which are the ones still in the
// memory-side cache.
__device__ __forceinline__ int block_index(const StepArgs& a)
{
    int id = int(blockIdx.x);
    if (a.xcd_remap) {
        const int q = a.nblocks / 8, r = a.nblocks % 8;
        const int xcd = id % 8, local = id / 8;
        id = xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
    }
    return a.reverse ? a.nblocks - 1 - id : id;
}

// One node: gather (pull, periodic, or local when !PULL), collide, store.
// Cache policy of the 2D step, from the size of one state buffer against the
// 256 MiB memory-side cache: POL_STREAM ordinary loads, non-temporal stores
// (large buffers); POL_CACHE ordinary loads and stores, tile order reversed
// every other step (small buffers: the state stays in the cache);
// POL_KEEP non-temporal loads and ordinary stores (buffers about the cache's
// size: the reads no longer evict what the step writes, which the next step
// reads).
enum Policy { POL_STREAM = 0, POL_CACHE = 1, POL_KEEP = 2 };

template <class L, class S, int COLL, bool THERMAL, bool A13P, bool PULL, bool NT = true, bool NTLOAD = false>
__device__ __forceinline__ void node_update(const typename S::elem* __restrict__ fin,
                                            typename S::elem* __restrict__ fout, const Layout& lay, int x,
                                            int y, const Relax& rx, uint32_t seq)
{
    using T = typename S::math;
    constexpr int R = L::R;
    const int nx = lay.nx, ny = lay.ny;

    // periodic source columns / tile rows for every shift in [-R, R]
    int xs[2 * R + 1], ys[2 * R + 1];
    static_for<2 * R + 1>([&](auto D) {
        constexpr int d = int(D) - R;
        int xx = x - d, yy = y - d;
        if constexpr (d > 0) {
            xx += (xx < 0) ? nx : 0;
            yy += (yy < 0) ? ny : 0;
        } else if constexpr (d < 0) {
            xx -= (xx >= nx) ? nx : 0;
            yy -= (yy >= ny) ? ny : 0;
        }
        xs[D] = xx;
        ys[D] = lay.row(yy);
    });

    T v[L::Q];
    const int here = lay.row(y) + x;
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        const int idx = (PULL ? ys[cy + R] + xs[cx + R] : here) + int(I) * lay.te;
        if constexpr (NTLOAD)
            v[I] = S::load_nt(fin + idx);
        else
            v[I] = S::load(fin + idx);
    });

    collide_node<L, T, COLL, THERMAL, S::shifted, A13P, S::conserve_in_double>(v, rx);

    store_node<L, S, T, NT>(fout, here, lay.te, v, uint32_t(y) * uint32_t(nx) + uint32_t(x), seq);
}

template <class L, class S, int COLL, bool THERMAL, bool A13P, bool PULL, int POL>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(RRLBM_WAVES_PER_EU)))
void k_stream_collide(StepArgs a)
{
    const int bid = block_index(a);
    const int x = (bid % a.bx_blocks) * BX + int(threadIdx.x);
    const int y = (bid / a.bx_blocks) * BY + int(threadIdx.y);
    if (x >= a.lay.nx || y >= a.lay.ny) return;
    node_update<L, S, COLL, THERMAL, A13P, PULL, POL == POL_STREAM, POL == POL_KEEP>(
        static_cast<const typename S::elem*>(a.fin), static_cast<typename S::elem*>(a.fout), a.lay, x, y, a.rx,
        a.seq);
}

// ---------------------------------------------------------- batch kernel

// One member of a batch as the persistent kernel sees it.
struct InstDesc {
    void* buf[2];
    Layout lay;
    int lattice;
    int bx_blocks; // work items along x
    int flip;      // index of the buffer holding the member's current state
    Relax rx;
    uint32_t seq;  // index of the state the parity-0 launch writes (BF16 dither key)
};

// Persistent kernel: blocks stride over the work list (member, tile); item w
// belongs to the member i with begin[i] <= w < begin[i+1].  Each item is a
// tile_x by 4 patch of one member, walked 64 columns at a time.  `parity`
// selects the buffer direction of this step for every member.
template <class S>
__global__ __launch_bounds__(BX* BY) void k_batch(const InstDesc* __restrict__ desc, const int* __restrict__ begin,
                                                  int n, int total, int parity, int tile_x)
{
    using E = typename S::elem;
    for (int w = int(blockIdx.x); w < total; w += int(gridDim.x)) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (begin[mid] <= w)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int i = __builtin_amdgcn_readfirstlane(lo);
        const InstDesc& d = desc[i];
        const int local = w - begin[i];
        const int x0 = (local % d.bx_blocks) * tile_x;
        const int y = (local / d.bx_blocks) * BY + int(threadIdx.y);
        const int src = d.flip ^ parity;
        const E* fin = static_cast<const E*>(d.buf[src]);
        E* fout = static_cast<E*>(d.buf[src ^ 1]);
        for (int sub = 0; sub < tile_x; sub += BX) {
            const int x = x0 + sub + int(threadIdx.x);
            if (x < d.lay.nx && y < d.lay.ny) {
                switch (d.lattice) {
                case 0: node_update<D2Q9, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, d.seq + uint32_t(parity)); break;
                case 1: node_update<D2V17, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, d.seq + uint32_t(parity)); break;
                default: node_update<D2V37, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, d.seq + uint32_t(parity)); break;
                }
            }
        }
    }
}

} // namespace rr

#include "closure.hpp"

namespace rr {

// ------------------------------------------------------------ init kernel

struct InitArgs {
    void* f;
    Layout lay;
    const double *rho, *ux, *uy, *theta, *grad, *noise;
    double noise_amp;
    int eq_order;
    double tau;
};

template <class L, class S>
__global__ __launch_bounds__(256) void k_init(InitArgs a)
{
    const int64_t n = int64_t(a.lay.nx) * a.lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int here = a.lay.row(int(k / a.lay.nx)) + int(k % a.lay.nx);
    double f[L::Q];
    const double th = a.theta ? a.theta[k] : 1.0;
    equilibrium_node<L, double, S::shifted>(a.rho[k], a.ux[k], a.uy[k], th, a.eq_order, f);
    if (a.grad) {
        const double du[2][2] = { { a.grad[k], a.grad[2 * n + k] }, { a.grad[n + k], a.grad[3 * n + k] } };
        double f1[L::Q];
        noneq_init_node<L, double>(a.rho[k], a.ux[k], a.uy[k], du, a.tau, a.eq_order, f1);
        static_for<L::Q>([&](auto I) { f[I] += f1[I]; });
    }
    typename S::elem* out = static_cast<typename S::elem*>(a.f);
    static_for<L::Q>([&](auto I) {
        double v = f[I];
        if (a.noise) v += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k];
        S::store(out + here + int(I) * a.lay.te, typename S::math(v));
    });
}

} // namespace rr

#include "moments.hpp"

namespace rr {

// --------------------------------------------------- populations / moments

template <class L, class S>
__global__ __launch_bounds__(256) void k_populations(const void* fsrc, Layout lay, double* out)
{
    const int64_t n = int64_t(lay.nx) * lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int here = lay.row(int(k / lay.nx)) + int(k % lay.nx);
    const typename S::elem* f = static_cast<const typename S::elem*>(fsrc);
    static_for<L::Q>([&](auto I) {
        double v = double(S::load(f + here + int(I) * lay.te));
        if (S::shifted) v += L::v.w[I];
        out[int64_t(I) * n + k] = v;
    });
}

constexpr int MOM_NS = 8; // per-block partial sums of the moments kernel
constexpr int VORT_NS = 2;

template <int NS>
__device__ __forceinline__ void block_sums(double (&val)[NS], double* partial)
{
    __shared__ double red[NS][256];
    const int t = threadIdx.x;
    for (int s = 0; s < NS; ++s) red[s][t] = val[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int s = 0; s < NS; ++s) red[s][t] += red[s][t + w];
        __syncthreads();
    }
    if (t < NS) partial[int64_t(blockIdx.x) * NS + t] = red[t][0];
}

template <class L, int ORDER>
__global__ __launch_bounds__(256) void k_mom_populations(const double* m, int64_t n, Relax rx, double* out)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double v[L::Q];
    mom_node_populations<L, ORDER>(m, n, k, rx, v);
    static_for<L::Q>([&](auto I) { out[int64_t(I) * n + k] = v[I]; });
}

// Diagnostics of one node from its post-collision populations v.
template <class L>
__device__ __forceinline__ void node_diag(const double (&v)[L::Q], int thermal, int64_t k, double* rho_o,
                                          double* ux_o, double* uy_o, double* th_o, double (&val)[MOM_NS])
{
    double r = 0, jx = 0, jy = 0, e2 = 0;
    static_for<L::Q>([&](auto I) {
        constexpr double cx = L::v.cx[I], cy = L::v.cy[I];
        r += v[I];
        jx += cx * v[I];
        jy += cy * v[I];
        e2 += (cx * cx + cy * cy) * v[I];
    });
    const double ux = jx / r, uy = jy / r;
    const double u2 = ux * ux + uy * uy;
    const double th = thermal ? (e2 - r * u2) / (2.0 * r * L::cs2) : 1.0;
    rho_o[k] = r;
    ux_o[k] = ux;
    uy_o[k] = uy;
    th_o[k] = th;
    const bool finite = std::isfinite(r) && std::isfinite(ux) && std::isfinite(uy) && std::isfinite(th);
    if (finite) {
        val[0] = r;
        val[1] = jx;
        val[2] = jy;
        val[3] = 0.5 * e2;
        val[4] = u2;
        val[5] = u2 * u2;
        val[7] = th;
    } else {
        val[6] = 1.0;
    }
}

// rho, u, theta per node (FP64 arithmetic whatever the storage) and block sums
// of [rho, rho ux, rho uy, sum f|c|^2/2, |u|^2, |u|^4, non-finite, theta].
template <class L, class S>
__global__ __launch_bounds__(256) void k_moments(const void* fsrc, Layout lay, int thermal, double* rho_o,
                                                 double* ux_o, double* uy_o, double* th_o, double* partial)
{
    const int64_t n = int64_t(lay.nx) * lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        const int here = lay.row(int(k / lay.nx)) + int(k % lay.nx);
        const typename S::elem* f = static_cast<const typename S::elem*>(fsrc);
        double v[L::Q];
        static_for<L::Q>([&](auto I) {
            v[I] = double(S::load(f + here + int(I) * lay.te));
            if (S::shifted) v[I] += L::v.w[I];
        });
        node_diag<L>(v, thermal, k, rho_o, ux_o, uy_o, th_o, val);
    }
    block_sums<MOM_NS>(val, partial);
}

// The same from the moment representation.
template <class L, int ORDER>
__global__ __launch_bounds__(256) void k_mom_moments(const double* m, int64_t n, Relax rx, double* rho_o,
                                                     double* ux_o, double* uy_o, double* th_o, double* partial)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        double v[L::Q];
        mom_node_populations<L, ORDER>(m, n, k, rx, v);
        node_diag<L>(v, 0, k, rho_o, ux_o, uy_o, th_o, val);
    }
    block_sums<MOM_NS>(val, partial);
}

// Vorticity from the periodic fourth-order centred difference and block sums
// of [omega^2, omega^4].
__global__ __launch_bounds__(256) void k_vorticity(const double* ux, const double* uy, int nx, int ny,
                                                   double* vort, double* partial)
{
    const int64_t n = int64_t(nx) * ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[VORT_NS] = { 0, 0 };
    if (k < n) {
        const int x = int(k % nx), y = int(k / nx);
        auto X = [&](int d) { int t = x + d; t += (t < 0) ? nx : 0; t -= (t >= nx) ? nx : 0; return t; };
        auto Y = [&](int d) { int t = y + d; t += (t < 0) ? ny : 0; t -= (t >= ny) ? ny : 0; return t; };
        const int64_t row = int64_t(y) * nx;
        const double dvy = (-uy[row + X(2)] + 8.0 * uy[row + X(1)] - 8.0 * uy[row + X(-1)] + uy[row + X(-2)]) / 12.0;
        const double dux = (-ux[int64_t(Y(2)) * nx + x] + 8.0 * ux[int64_t(Y(1)) * nx + x]
                            - 8.0 * ux[int64_t(Y(-1)) * nx + x] + ux[int64_t(Y(-2)) * nx + x]) / 12.0;
        const double w = dvy - dux;
        if (vort) vort[k] = w;
        if (std::isfinite(w)) {
            val[0] = w * w;
            val[1] = w * w * w * w;
        }
    }
    block_sums<VORT_NS>(val, partial);
}

} // namespace rr

#include "collide3d.hpp"

// ================================================================== C-ABI

using namespace rr;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum StoreKind { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_MOM = 3 };

struct LatInfo {
    int q, reach, n_eq;
    double cs2;
};

template <class L>
LatInfo info_of()
{
    return { L::Q, L::R, L::NEQ, L::cs2 };
}

bool is_3d(int lattice)
{
    return lattice == LBM_D3Q19 || lattice == LBM_D3Q27 || lattice == LBM_D3V39 || lattice == LBM_D3Q103;
}

bool lattice_info(int lattice, LatInfo* out)
{
    switch (lattice) {
    case LBM_D2Q9: *out = info_of<D2Q9>(); return true;
    case LBM_D2V17: *out = info_of<D2V17>(); return true;
    case LBM_D2V37: *out = info_of<D2V37>(); return true;
    case LBM_D3Q19: *out = info_of<D3Q19>(); return true;
    case LBM_D3Q27: *out = info_of<D3Q27>(); return true;
    case LBM_D3V39: *out = info_of<D3V39>(); return true;
    case LBM_D3Q103: *out = info_of<D3Q103>(); return true;
    }
    return false;
}


} // namespace

struct lbm_ctx {
    int lattice = 0, nx = 0, ny = 0, order = 2;
    int nz = 1, dim = 2; // 3D lattices: rows r = z * ny + y of the layout
    double tau = 1.0, tau3 = 1.0, tau4 = 1.0; // tau_2 = tau; ranks 3, 4 (lbm_set_relaxation)
    uint32_t flags = 0;
    int store = ST_F64, coll = COLL_RR;
    bool thermal = false, a13p = false;
    int q = 0;
    Layout lay{};
    int xcd_remap = 1;
    int pol = POL_STREAM; // cache policy of the step (from the buffer size at init; 3D: RR and BGK)
    void* buf[2] = { nullptr, nullptr };
    int cur = 0;
    int64_t steps = 0;
    hipStream_t stream = nullptr;
    // moments scratch
    double* fields = nullptr; // 5 fields of nx*ny
    double* partial = nullptr;
    double* partial_host = nullptr;
    int64_t nblk = 0;
    // learned closure (isothermal D2V37 only)
    bool closure = false;
    MlpInfer* cl_frags = nullptr;
    float* cl_norm = nullptr;
    unsigned long long* cl_fallbacks = nullptr;
};

namespace {

// Cache policy from the bytes of one state buffer (see Policy), measured on
// the step at 768^2, 1024^2 and 1536^2 for every lattice and storage:
// POL_CACHE wins up to 128 MiB (by up to 20 points of HBM peak), POL_KEEP from
// 256 to 320 MiB (D2V37 FP64 1024^2, 310 MB: 75.7% against 71.5%), POL_STREAM
// elsewhere.  RRLBM_CACHE_POLICY=0/1/2 forces one.
int choose_policy(int64_t buffer_bytes)
{
    if (const char* e = std::getenv("RRLBM_CACHE_POLICY")) {
        const int p = std::atoi(e);
        if (p >= POL_STREAM && p <= POL_KEEP) return p;
    }
    const int64_t MiB = int64_t(1) << 20;
    if (buffer_bytes <= 128 * MiB) return POL_CACHE;
    if (buffer_bytes > 256 * MiB && buffer_bytes <= 320 * MiB) return POL_KEEP;
    return POL_STREAM;
}

Relax relax_of(const lbm_ctx* c)
{
    return Relax{ 1.0 - 1.0 / c->tau, c->order >= 3 ? 1.0 - 1.0 / c->tau3 : 0.0,
                  c->order >= 4 ? 1.0 - 1.0 / c->tau4 : 0.0, 1.0 / c->tau };
}

// ---- moment representation: per-lattice launches (order as a template argument)
template <class L, int ORDER>
hipError_t mom_launch(const lbm_ctx* c, int what, const void* fin, void* fout, InitArgs* ia, double* out, double* r,
                      double* ux, double* uy, double* th)
{
    const int64_t n = int64_t(c->nx) * c->ny;
    const Relax rx = relax_of(c);
    const double* m = static_cast<const double*>(c->buf[c->cur]);
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    switch (what) {
    case 0: k_mom_init<L><<<grid, block, 0, c->stream>>>(*ia); break;
    case 1: k_mom_populations<L, ORDER><<<grid, block, 0, c->stream>>>(m, n, rx, out); break;
    case 2:
        k_mom_moments<L, ORDER><<<dim3(unsigned(c->nblk)), block, 0, c->stream>>>(m, n, rx, r, ux, uy, th,
                                                                                 c->partial);
        break;
    default: {
        const int bxn = (c->nx + BX - 1) / BX, byn = (c->ny + BY - 1) / BY;
        const dim3 g(unsigned(bxn * byn)), blk(BX, BY);
        const double* a = static_cast<const double*>(fin);
        double* o = static_cast<double*>(fout);
        if (c->tau3 == c->tau && c->tau4 == c->tau)
            k_mom_step<L, ORDER, false><<<g, blk, 0, c->stream>>>(a, o, c->nx, c->ny, bxn, rx);
        else
            k_mom_step<L, ORDER, true><<<g, blk, 0, c->stream>>>(a, o, c->nx, c->ny, bxn, rx);
    }
    }
    return hipGetLastError();
}

template <class L>
hipError_t mom_launch_l(const lbm_ctx* c, int what, const void* fin, void* fout, InitArgs* ia, double* out,
                        double* r, double* ux, double* uy, double* th)
{
    switch (c->order) {
    case 2: return mom_launch<L, 2>(c, what, fin, fout, ia, out, r, ux, uy, th);
    case 3: return mom_launch<L, 3>(c, what, fin, fout, ia, out, r, ux, uy, th);
    default: return mom_launch<L, 4>(c, what, fin, fout, ia, out, r, ux, uy, th);
    }
}

// what: 0 initial state (ia), 1 populations (out), 2 diagnostics (r, ux, uy, th), 3 step (fin -> fout)
hipError_t mom_launch_any(const lbm_ctx* c, int what, const void* fin = nullptr, void* fout = nullptr,
                          InitArgs* ia = nullptr, double* out = nullptr, double* r = nullptr, double* ux = nullptr,
                          double* uy = nullptr, double* th = nullptr)
{
    switch (c->lattice) {
    case LBM_D2Q9: return mom_launch_l<D2Q9>(c, what, fin, fout, ia, out, r, ux, uy, th);
    case LBM_D2V17: return mom_launch_l<D2V17>(c, what, fin, fout, ia, out, r, ux, uy, th);
    default: return mom_launch_l<D2V37>(c, what, fin, fout, ia, out, r, ux, uy, th);
    }
}

template <class L, class S, int COLL, bool TH, bool A13P>
hipError_t launch_step_t(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    const int bxn = (c->nx + BX - 1) / BX, byn = (c->ny + BY - 1) / BY;
    StepArgs a{ fin, fout, c->lay, bxn, bxn * byn, c->xcd_remap, relax_of(c), pull ? uint32_t(c->steps + 1) : 0u,
                (c->pol == POL_CACHE && pull && (c->steps & 1)) ? 1 : 0 };
    dim3 grid(unsigned(bxn * byn)), block(BX, BY);
    if constexpr (L::id == LBM_D2V37 && COLL == COLL_RR && !TH) {
        if (pull && c->closure) {
            ClosureArgs ca{ c->cl_frags, c->cl_norm, 1.0 - 0.5 / c->tau, c->cl_fallbacks };
            k_stream_collide_closure<S><<<grid, block, 0, c->stream>>>(a, ca);
            return hipGetLastError();
        }
    }
    if (!pull)
        k_stream_collide<L, S, COLL, TH, A13P, false, POL_STREAM><<<grid, block, 0, c->stream>>>(a);
    else if (c->pol == POL_CACHE)
        k_stream_collide<L, S, COLL, TH, A13P, true, POL_CACHE><<<grid, block, 0, c->stream>>>(a);
    else if (c->pol == POL_KEEP)
        k_stream_collide<L, S, COLL, TH, A13P, true, POL_KEEP><<<grid, block, 0, c->stream>>>(a);
    else
        k_stream_collide<L, S, COLL, TH, A13P, true, POL_STREAM><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_step_s(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    if constexpr (L::id == LBM_D2V37) {
        if (c->thermal) {
            switch (c->coll) {
            case COLL_PR: return launch_step_t<L, S, COLL_PR, true, false>(c, fin, fout, pull);
            case COLL_BGK: return launch_step_t<L, S, COLL_BGK, true, false>(c, fin, fout, pull);
            default:
                return c->a13p ? launch_step_t<L, S, COLL_RR, true, true>(c, fin, fout, pull)
                               : launch_step_t<L, S, COLL_RR, true, false>(c, fin, fout, pull);
            }
        }
    }
    switch (c->coll) {
    case COLL_PR: return launch_step_t<L, S, COLL_PR, false, false>(c, fin, fout, pull);
    case COLL_BGK: return launch_step_t<L, S, COLL_BGK, false, false>(c, fin, fout, pull);
    default: return launch_step_t<L, S, COLL_RR, false, false>(c, fin, fout, pull);
    }
}

template <class L>
hipError_t launch_step_l(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    switch (c->store) {
    case ST_F32: return launch_step_s<L, StoreF32>(c, fin, fout, pull);
    case ST_BF16: return launch_step_s<L, StoreBF16>(c, fin, fout, pull);
    default: return launch_step_s<L, StoreF64>(c, fin, fout, pull);
    }
}

// ---- 3D lattices (FP64 populations; the step always pulls)
template <class L, int MODE>
hipError_t launch_step3_t(const lbm_ctx* c, const void* fin, void* fout)
{
    const int rows = c->ny * c->nz;
    const int bxn = (c->nx + BX - 1) / BX, byn = (rows + BY - 1) / BY;
    // the cache policies are instantiated for the RR and BGK steps; PR streams
    const int pol = MODE != C3_PR ? c->pol : POL_STREAM;
    Step3Args a{ fin, fout, c->lay, c->ny, c->nz, bxn, bxn * byn, c->xcd_remap, relax_of(c), c->order,
                 (pol == POL_CACHE && (c->steps & 1)) ? 1 : 0 };
    const dim3 grid(unsigned(bxn * byn)), block(BX, BY);
    if constexpr (MODE != C3_PR) {
        if (pol == POL_CACHE) {
            k_stream_collide3<L, MODE, POL_CACHE><<<grid, block, 0, c->stream>>>(a);
            return hipGetLastError();
        }
        if (pol == POL_KEEP) {
            k_stream_collide3<L, MODE, POL_KEEP><<<grid, block, 0, c->stream>>>(a);
            return hipGetLastError();
        }
    }
    k_stream_collide3<L, MODE, POL_STREAM><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

template <class L>
hipError_t launch_step3_l(const lbm_ctx* c, const void* fin, void* fout)
{
    switch (c->coll) {
    case COLL_PR: return launch_step3_t<L, C3_PR>(c, fin, fout);
    case COLL_BGK: return launch_step3_t<L, C3_BGK>(c, fin, fout);
    default: return launch_step3_t<L, C3_RR>(c, fin, fout);
    }
}

template <class F>
hipError_t on_lattice3(int lattice, F&& f)
{
    switch (lattice) {
    case LBM_D3Q19: return f(D3Q19{});
    case LBM_D3Q27: return f(D3Q27{});
    case LBM_D3V39: return f(D3V39{});
    default: return f(D3Q103{});
    }
}

hipError_t launch_step(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    if (c->dim == 3) {
        if (!pull) return hipErrorInvalidValue; // 3D contexts are only ever stepped with a pull
        return on_lattice3(c->lattice, [&](auto l) { return launch_step3_l<decltype(l)>(c, fin, fout); });
    }
    if (c->store == ST_MOM) return mom_launch_any(c, 3, fin, fout);
    switch (c->lattice) {
    case LBM_D2Q9: return launch_step_l<D2Q9>(c, fin, fout, pull);
    case LBM_D2V17: return launch_step_l<D2V17>(c, fin, fout, pull);
    default: return launch_step_l<D2V37>(c, fin, fout, pull);
    }
}

// generic dispatch over (lattice, storage) for the auxiliary kernels
template <template <class, class> class F, class... Args>
hipError_t dispatch_ls(const lbm_ctx* c, Args... args)
{
    switch (c->lattice) {
    case LBM_D2Q9:
        switch (c->store) {
        case ST_F32: return F<D2Q9, StoreF32>::run(c, args...);
        case ST_BF16: return F<D2Q9, StoreBF16>::run(c, args...);
        default: return F<D2Q9, StoreF64>::run(c, args...);
        }
    case LBM_D2V17:
        switch (c->store) {
        case ST_F32: return F<D2V17, StoreF32>::run(c, args...);
        case ST_BF16: return F<D2V17, StoreBF16>::run(c, args...);
        default: return F<D2V17, StoreF64>::run(c, args...);
        }
    default:
        switch (c->store) {
        case ST_F32: return F<D2V37, StoreF32>::run(c, args...);
        case ST_BF16: return F<D2V37, StoreBF16>::run(c, args...);
        default: return F<D2V37, StoreF64>::run(c, args...);
        }
    }
}

template <class L, class S>
struct InitOp {
    static hipError_t run(const lbm_ctx* c, InitArgs a)
    {
        const int64_t n = int64_t(c->nx) * c->ny;
        k_init<L, S><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
        return hipGetLastError();
    }
};

template <class L, class S>
struct PopOp {
    static hipError_t run(const lbm_ctx* c, double* out)
    {
        const int64_t n = int64_t(c->nx) * c->ny;
        k_populations<L, S><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream>>>(
            c->buf[c->cur], c->lay, out);
        return hipGetLastError();
    }
};

template <class L, class S>
struct MomOp {
    static hipError_t run(const lbm_ctx* c, double* r, double* ux, double* uy, double* th)
    {
        k_moments<L, S><<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(
            c->buf[c->cur], c->lay, c->thermal ? 1 : 0, r, ux, uy, th, c->partial);
        return hipGetLastError();
    }
};

int validate(int lattice, int nx, int ny, double tau, int reg_order, uint32_t flags, LatInfo* li)
{
    if (!lattice_info(lattice, li)) return fail(LBM_EINVAL, "unknown lattice " + std::to_string(lattice));
    if (is_3d(lattice)) return fail(LBM_EINVAL, "3D lattice: use lbm_init_3d");
    if (nx < li->reach || ny < li->reach || nx < 1 || ny < 1)
        return fail(LBM_EINVAL, "grid " + std::to_string(nx) + "x" + std::to_string(ny) +
                                    " smaller than the lattice reach " + std::to_string(li->reach));
    if (layout_elems(li->q, nx, ny) >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "grid too large");
    if (!std::isfinite(tau) || !(tau > 0.5)) return fail(LBM_ETAU, "tau must be finite and > 1/2");
    const uint32_t known = LBM_THERMAL | LBM_STORE_FP32 | LBM_STORE_BF16 | LBM_STORE_MOMENTS | LBM_COLL_PR |
                           LBM_COLL_BGK | LBM_EQ_INIT_ORDER2 | LBM_A13_PROJECTED;
    if (flags & ~known) return fail(LBM_EINVAL, "unknown flag bits");
    const uint32_t stores = flags & (LBM_STORE_FP32 | LBM_STORE_BF16 | LBM_STORE_MOMENTS);
    if (stores & (stores - 1)) return fail(LBM_EINVAL, "two storage flags");
    if ((flags & LBM_STORE_MOMENTS) && (flags & (LBM_THERMAL | LBM_COLL_PR | LBM_COLL_BGK | LBM_A13_PROJECTED)))
        return fail(LBM_EINVAL, "the moment representation is isothermal recursive regularization only");
    if ((flags & LBM_COLL_PR) && (flags & LBM_COLL_BGK)) return fail(LBM_EINVAL, "two collision flags");
    if ((flags & LBM_THERMAL) && lattice != LBM_D2V37)
        return fail(LBM_EINVAL, "the thermal form needs the D2V37 lattice");
    if (!(flags & LBM_COLL_BGK) && (reg_order < 2 || reg_order > li->n_eq))
        return fail(LBM_EINVAL, "regularization order must be in [2, " + std::to_string(li->n_eq) + "]");
    return LBM_OK;
}

double neumaier(const double* x, int64_t n, int stride)
{
    double s = 0, c = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double v = x[i * stride];
        const double t = s + v;
        c += (std::fabs(s) >= std::fabs(v)) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    return s + c;
}

} // namespace

extern "C" {

int lbm_lattice_info(int lattice, int* q, int* reach, int* n_eq, double* cs2)
{
    LatInfo li;
    if (!lattice_info(lattice, &li)) return fail(LBM_EINVAL, "unknown lattice");
    if (q) *q = li.q;
    if (reach) *reach = li.reach;
    if (n_eq) *n_eq = li.n_eq;
    if (cs2) *cs2 = li.cs2;
    return LBM_OK;
}

int lbm_lattice_velocities(int lattice, int* cx, int* cy, double* w)
{
    const VelTable* t = nullptr;
    switch (lattice) {
    case LBM_D2Q9: t = &D2Q9::v; break;
    case LBM_D2V17: t = &D2V17::v; break;
    case LBM_D2V37: t = &D2V37::v; break;
    default: return fail(LBM_EINVAL, is_3d(lattice) ? "3D lattice: use lbm_lattice_velocities_3d" : "unknown lattice");
    }
    for (int i = 0; i < t->q; ++i) {
        if (cx) cx[i] = t->cx[i];
        if (cy) cy[i] = t->cy[i];
        if (w) w[i] = t->w[i];
    }
    return LBM_OK;
}

int64_t lbm_buffer_elems(int lattice, int nx, int ny, uint32_t flags)
{
    LatInfo li;
    if (!lattice_info(lattice, &li)) return fail(LBM_EINVAL, "unknown lattice");
    if (is_3d(lattice)) return fail(LBM_EINVAL, "3D lattice: use lbm_buffer_elems_3d");
    if (nx < 1 || ny < 1) return fail(LBM_EINVAL, "empty grid");
    if (flags & LBM_STORE_MOMENTS) return int64_t(MOM_K) * nx * ny;
    return layout_elems(li.q, nx, ny);
}

int lbm_init(lbm_ctx** out, int lattice, int nx, int ny, double tau, int reg_order, uint32_t flags,
             void* f_a, void* f_b, const double* rho, const double* ux, const double* uy,
             const double* theta, const double* grad, const double* noise, double noise_amp, void* stream)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    LatInfo li;
    int e = validate(lattice, nx, ny, tau, reg_order, flags, &li);
    if (e) return e;
    if (!f_a || !f_b || f_a == f_b) return fail(LBM_EINVAL, "two distinct population buffers are needed");
    if (!rho || !ux || !uy) return fail(LBM_EINVAL, "rho, ux and uy are required");
    if ((flags & LBM_THERMAL) == 0 && theta)
        return fail(LBM_EINVAL, "theta given for an isothermal run");
    if ((flags & LBM_THERMAL) && grad)
        return fail(LBM_EINVAL, "the f^(1) initial state from velocity gradients is isothermal");
    if (!std::isfinite(noise_amp)) return fail(LBM_EINVAL, "noise_amp not finite");

    lbm_ctx* c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ENOMEM, "context allocation failed");
    c->lattice = lattice;
    c->nx = nx;
    c->ny = ny;
    c->tau = tau;
    c->tau3 = tau;
    c->tau4 = tau;
    c->order = (flags & LBM_COLL_BGK) ? 2 : reg_order;
    c->flags = flags;
    c->store = (flags & LBM_STORE_FP32)      ? ST_F32
               : (flags & LBM_STORE_BF16)    ? ST_BF16
               : (flags & LBM_STORE_MOMENTS) ? ST_MOM
                                             : ST_F64;
    c->coll = (flags & LBM_COLL_PR) ? COLL_PR : (flags & LBM_COLL_BGK) ? COLL_BGK : COLL_RR;
    c->thermal = (flags & LBM_THERMAL) != 0;
    c->a13p = (flags & LBM_A13_PROJECTED) != 0;
    c->q = li.q;
    c->lay = make_layout(li.q, nx, ny);
    {
        const int64_t esz = c->store == ST_F32 ? 4 : c->store == ST_BF16 ? 2 : 8;
        c->pol = choose_policy(esz * (c->store == ST_MOM ? int64_t(MOM_K) * nx * ny : layout_elems(li.q, nx, ny)));
    }
    // tuning knob: RRLBM_XCD_REMAP=0 keeps the hardware's round-robin block order
    if (const char* e = std::getenv("RRLBM_XCD_REMAP")) c->xcd_remap = std::atoi(e) != 0;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->stream = static_cast<hipStream_t>(stream);
    const int64_t n = int64_t(nx) * ny;
    c->nblk = (n + 255) / 256;

    InitArgs ia{ f_a, c->lay, rho, ux, uy, theta, grad, noise, noise_amp,
                 (flags & LBM_EQ_INIT_ORDER2) ? 2 : li.n_eq, tau };
    hipError_t he = hipSuccess;
    if (c->store == ST_MOM) {
        he = mom_launch_any(c, 0, nullptr, nullptr, &ia); // the moments are the state: no collision here
    } else {
        he = dispatch_ls<InitOp>(c, ia);
        if (he == hipSuccess) he = launch_step(c, f_a, f_a, false); // collide in place: post-collision state
    }
    if (he != hipSuccess) {
        delete c;
        return fail(LBM_EDEVICE, std::string("init launch: ") + hipGetErrorString(he));
    }
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int nsteps)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    for (int s = 0; s < nsteps; ++s) {
        hipError_t he = launch_step(c, c->buf[c->cur], c->buf[1 - c->cur], true);
        if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(he));
        c->cur = 1 - c->cur;
        ++c->steps;
    }
    return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->steps : -1; }

int lbm_set_relaxation(lbm_ctx* c, double tau3, double tau4)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->coll == COLL_BGK) return fail(LBM_EINVAL, "BGK has a single relaxation time");
    if (!std::isfinite(tau3) || !(tau3 > 0.5) || !std::isfinite(tau4) || !(tau4 > 0.5))
        return fail(LBM_ETAU, "tau3 and tau4 must be finite and > 1/2");
    c->tau3 = tau3;
    c->tau4 = tau4;
    return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* theta, double* vort, double* sums)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->dim == 3) return fail(LBM_EINVAL, "3D context: use lbm_moments_3d");
    const int64_t n = int64_t(c->nx) * c->ny;
    if (!c->fields) {
        HIP_TRY(hipMalloc(&c->fields, sizeof(double) * 5 * n));
        HIP_TRY(hipMalloc(&c->partial, sizeof(double) * (MOM_NS + VORT_NS) * c->nblk));
        HIP_TRY(hipHostMalloc(&c->partial_host, sizeof(double) * (MOM_NS + VORT_NS) * c->nblk));
    }
    double* r = rho ? rho : c->fields;
    double* vx = ux ? ux : c->fields + n;
    double* vy = uy ? uy : c->fields + 2 * n;
    double* th = theta ? theta : c->fields + 3 * n;
    if (c->store == ST_MOM)
        HIP_TRY(mom_launch_any(c, 2, nullptr, nullptr, nullptr, nullptr, r, vx, vy, th));
    else
        HIP_TRY(dispatch_ls<MomOp>(c, r, vx, vy, th));
    if (vort || sums) {
        k_vorticity<<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(vx, vy, c->nx, c->ny, vort,
                                                                          c->partial + MOM_NS * c->nblk);
        HIP_TRY(hipGetLastError());
    }
    if (sums) {
        HIP_TRY(hipMemcpyAsync(c->partial_host, c->partial, sizeof(double) * (MOM_NS + VORT_NS) * c->nblk,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        const double* pm = c->partial_host;
        const double* pv = c->partial_host + MOM_NS * c->nblk;
        for (int s = 0; s < MOM_NS; ++s) {
            const double v = neumaier(pm + s, c->nblk, MOM_NS);
            static const int slot[MOM_NS] = { 0, 1, 2, 3, 4, 5, 8, 9 };
            sums[slot[s]] = v;
        }
        sums[6] = neumaier(pv, c->nblk, VORT_NS);
        sums[7] = neumaier(pv + 1, c->nblk, VORT_NS);
    }
    return LBM_OK;
}

int lbm_populations(lbm_ctx* c, double* f_out)
{
    if (!c || !f_out) return fail(LBM_EINVAL, "ctx or f_out is NULL");
    if (c->dim == 3) {
        const int64_t n = int64_t(c->nx) * c->ny * c->nz;
        HIP_TRY(on_lattice3(c->lattice, [&](auto l) {
            k_populations<decltype(l), StoreF64><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream>>>(
                c->buf[c->cur], c->lay, f_out);
            return hipGetLastError();
        }));
    } else if (c->store == ST_MOM) {
        HIP_TRY(mom_launch_any(c, 1, nullptr, nullptr, nullptr, f_out));
    } else {
        HIP_TRY(dispatch_ls<PopOp>(c, f_out));
    }
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    if (c->fields) (void)hipFree(c->fields);
    if (c->partial) (void)hipFree(c->partial);
    if (c->partial_host) (void)hipHostFree(c->partial_host);
    if (c->cl_frags) (void)hipFree(c->cl_frags);
    if (c->cl_norm) (void)hipFree(c->cl_norm);
    if (c->cl_fallbacks) (void)hipFree(c->cl_fallbacks);
    delete c;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- 3D

int lbm_lattice_velocities_3d(int lattice, int* cx, int* cy, int* cz, double* w)
{
    const VelTable3* t = nullptr;
    switch (lattice) {
    case LBM_D3Q19: t = &D3Q19::v; break;
    case LBM_D3Q27: t = &D3Q27::v; break;
    case LBM_D3V39: t = &D3V39::v; break;
    case LBM_D3Q103: t = &D3Q103::v; break;
    default: return fail(LBM_EINVAL, "not a 3D lattice");
    }
    for (int i = 0; i < t->q; ++i) {
        if (cx) cx[i] = t->cx[i];
        if (cy) cy[i] = t->cy[i];
        if (cz) cz[i] = t->cz[i];
        if (w) w[i] = t->w[i];
    }
    return LBM_OK;
}

int64_t lbm_buffer_elems_3d(int lattice, int nx, int ny, int nz, uint32_t flags)
{
    LatInfo li;
    if (!is_3d(lattice) || !lattice_info(lattice, &li)) return fail(LBM_EINVAL, "not a 3D lattice");
    if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_EINVAL, "empty grid");
    if (flags & (LBM_STORE_FP32 | LBM_STORE_BF16 | LBM_STORE_MOMENTS))
        return fail(LBM_EINVAL, "3D lattices store FP64 populations");
    if (int64_t(ny) * nz >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "grid too large");
    return layout_elems(li.q, nx, ny * nz);
}

int lbm_init_3d(lbm_ctx** out, int lattice, int nx, int ny, int nz, double tau, int reg_order, uint32_t flags,
                void* f_a, void* f_b, const double* rho, const double* ux, const double* uy, const double* uz,
                const double* noise, double noise_amp, void* stream)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    LatInfo li;
    if (!is_3d(lattice) || !lattice_info(lattice, &li)) return fail(LBM_EINVAL, "not a 3D lattice");
    if (nx < li.reach || ny < li.reach || nz < li.reach || nx < 1 || ny < 1 || nz < 1)
        return fail(LBM_EINVAL, "grid smaller than the lattice reach " + std::to_string(li.reach));
    if (int64_t(ny) * nz >= (int64_t(1) << 31) || layout_elems(li.q, nx, ny * nz) >= (int64_t(1) << 31))
        return fail(LBM_EINVAL, "grid too large");
    if (!std::isfinite(tau) || !(tau > 0.5)) return fail(LBM_ETAU, "tau must be finite and > 1/2");
    const uint32_t known = LBM_COLL_PR | LBM_COLL_BGK | LBM_EQ_INIT_ORDER2;
    if (flags & ~known) return fail(LBM_EINVAL, "3D lattices take LBM_COLL_PR, LBM_COLL_BGK and LBM_EQ_INIT_ORDER2 only");
    if ((flags & LBM_COLL_PR) && (flags & LBM_COLL_BGK)) return fail(LBM_EINVAL, "two collision flags");
    if (!(flags & LBM_COLL_BGK) && (reg_order < 2 || reg_order > li.n_eq))
        return fail(LBM_EINVAL, "regularization order must be in [2, " + std::to_string(li.n_eq) + "]");
    if (!f_a || !f_b || f_a == f_b) return fail(LBM_EINVAL, "two distinct population buffers are needed");
    if (!rho || !ux || !uy || !uz) return fail(LBM_EINVAL, "rho, ux, uy and uz are required");
    if (!std::isfinite(noise_amp)) return fail(LBM_EINVAL, "noise_amp not finite");

    lbm_ctx* c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ENOMEM, "context allocation failed");
    c->lattice = lattice;
    c->dim = 3;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->tau = tau;
    c->tau3 = tau;
    c->tau4 = tau;
    c->order = (flags & LBM_COLL_BGK) ? 2 : reg_order;
    c->flags = flags;
    c->store = ST_F64;
    c->coll = (flags & LBM_COLL_PR) ? COLL_PR : (flags & LBM_COLL_BGK) ? COLL_BGK : COLL_RR;
    c->q = li.q;
    c->lay = make_layout(li.q, nx, ny * nz);
    c->pol = choose_policy(int64_t(sizeof(double)) * layout_elems(li.q, nx, ny * nz));
    if (const char* e = std::getenv("RRLBM_XCD_REMAP")) c->xcd_remap = std::atoi(e) != 0;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->stream = static_cast<hipStream_t>(stream);
    const int64_t n = int64_t(nx) * ny * nz;
    c->nblk = (n + 255) / 256;
    // f^(0) goes to f_b shifted by -c_i; one pull launch then collides it into f_a
    Init3Args ia{ f_b, c->lay, ny, nz, rho, ux, uy, uz, noise, noise_amp,
                  (flags & LBM_EQ_INIT_ORDER2) ? 2 : li.n_eq };
    hipError_t he = on_lattice3(lattice, [&](auto l) {
        k_init3<decltype(l)><<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(ia);
        return hipGetLastError();
    });
    if (he == hipSuccess) he = launch_step(c, f_b, f_a, true); // post-collision state in f_a, cur = 0
    if (he != hipSuccess) {
        delete c;
        return fail(LBM_EDEVICE, std::string("init launch: ") + hipGetErrorString(he));
    }
    *out = c;
    return LBM_OK;
}

int lbm_moments_3d(lbm_ctx* c, double* rho, double* ux, double* uy, double* uz, double* sums)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->dim != 3) return fail(LBM_EINVAL, "2D context: use lbm_moments");
    const int64_t n = int64_t(c->nx) * c->ny * c->nz;
    if (!c->fields) {
        HIP_TRY(hipMalloc(&c->fields, sizeof(double) * 4 * n));
        HIP_TRY(hipMalloc(&c->partial, sizeof(double) * MOM3_NS * c->nblk));
        HIP_TRY(hipHostMalloc(&c->partial_host, sizeof(double) * MOM3_NS * c->nblk));
    }
    double* r = rho ? rho : c->fields;
    double* vx = ux ? ux : c->fields + n;
    double* vy = uy ? uy : c->fields + 2 * n;
    double* vz = uz ? uz : c->fields + 3 * n;
    HIP_TRY(on_lattice3(c->lattice, [&](auto l) {
        k_moments3<decltype(l)><<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(
            static_cast<const double*>(c->buf[c->cur]), c->lay, c->ny, c->nz, r, vx, vy, vz, c->partial);
        return hipGetLastError();
    }));
    if (sums) {
        HIP_TRY(hipMemcpyAsync(c->partial_host, c->partial, sizeof(double) * MOM3_NS * c->nblk,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int s = 0; s < MOM3_NS; ++s) sums[s] = neumaier(c->partial_host + s, c->nblk, MOM3_NS);
    }
    return LBM_OK;
}

} // extern "C"

// ================================================================ batches

// Moves every member's dither key on by the two steps of one graph replay
// (BF16 batches: the replayed launches read it from the descriptors).
__global__ void k_batch_advance(InstDesc* desc, int n)
{
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) desc[i].seq += 2u;
}

struct lbm_batch {
    std::vector<lbm_ctx*> members;
    std::vector<InstDesc> desc;
    std::vector<int> begin;
    int store = ST_F64;
    hipStream_t stream = nullptr;  // members' stream: every replay goes there
    hipStream_t capture = nullptr; // private stream used only to record the graph
    InstDesc* d_desc = nullptr;
    int* d_begin = nullptr;
    int total = 0;
    int tile_x = 64, bpc = 4, num_cu = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <class S>
hipError_t launch_batch(const lbm_batch* b, hipStream_t st, int parity)
{
    const int grid = std::min(b->total, b->num_cu * b->bpc);
    k_batch<S><<<dim3(unsigned(grid)), dim3(BX, BY), 0, st>>>(b->d_desc, b->d_begin, int(b->members.size()),
                                                               b->total, parity, b->tile_x);
    return hipGetLastError();
}

hipError_t launch_batch_any(const lbm_batch* b, hipStream_t st, int parity)
{
    switch (b->store) {
    case ST_F32: return launch_batch<StoreF32>(b, st, parity);
    case ST_BF16: return launch_batch<StoreBF16>(b, st, parity);
    default: return launch_batch<StoreF64>(b, st, parity);
    }
}

void batch_release_graph(lbm_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Rebuilds the work list for the current tile width, uploads it with every
// member's buffer parity, and records the two-step graph.
int batch_prepare(lbm_batch* b)
{
    const int n = int(b->members.size());
    b->desc.resize(n);
    b->begin.assign(n + 1, 0);
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const lbm_ctx* c = b->members[i];
        InstDesc& d = b->desc[i];
        d.buf[0] = c->buf[0];
        d.buf[1] = c->buf[1];
        d.lay = c->lay;
        d.lattice = c->lattice;
        d.bx_blocks = (c->nx + b->tile_x - 1) / b->tile_x;
        d.flip = c->cur;
        d.rx = relax_of(c);
        d.seq = uint32_t(c->steps + 1);
        b->begin[i] = int(total);
        total += int64_t(d.bx_blocks) * ((c->ny + BY - 1) / BY);
    }
    if (total >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "batch work list too long");
    b->begin[n] = int(total);
    b->total = int(total);
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_begin, b->begin.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    batch_release_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e0 = launch_batch_any(b, b->capture, 0);
    hipError_t e1 = (e0 == hipSuccess) ? launch_batch_any(b, b->capture, 1) : e0;
    if (e1 == hipSuccess && b->store == ST_BF16) {
        k_batch_advance<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, b->capture>>>(b->d_desc, n);
        e1 = hipGetLastError();
    }
    hipError_t ec = hipStreamEndCapture(b->capture, &b->graph);
    if (e0 != hipSuccess || e1 != hipSuccess || ec != hipSuccess) {
        batch_release_graph(b);
        return fail(LBM_EDEVICE, std::string("batch graph capture: ") +
                                     hipGetErrorString(e0 != hipSuccess ? e0 : e1 != hipSuccess ? e1 : ec));
    }
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return LBM_OK;
}

// If a member was stepped on its own (or an odd step count left the device's
// dither keys behind, or its relaxation times changed), refresh the
// parities, keys and relaxation factors on the device.
int batch_sync_parity(lbm_batch* b)
{
    const bool dither = b->store == ST_BF16;
    bool stale = false;
    for (size_t i = 0; i < b->members.size(); ++i) {
        InstDesc& d = b->desc[i];
        const lbm_ctx* c = b->members[i];
        if (d.flip != c->cur) {
            d.flip = c->cur;
            stale = true;
        }
        if (dither && d.seq != uint32_t(c->steps + 1)) {
            d.seq = uint32_t(c->steps + 1);
            stale = true;
        }
        const Relax rx = relax_of(c);
        if (d.rx.k2 != rx.k2 || d.rx.k3 != rx.k3 || d.rx.k4 != rx.k4 || d.rx.inv_tau != rx.inv_tau) {
            d.rx = rx;
            stale = true;
        }
    }
    if (stale) {
        HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(InstDesc) * b->desc.size(),
                               hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return LBM_OK;
}

} // namespace

extern "C" {

int lbm_batch_create(lbm_batch** out, lbm_ctx* const* ctxs, int n, int tile_x, int blocks_per_cu)
{
    if (!out || !ctxs) return fail(LBM_EINVAL, "out or ctxs is NULL");
    if (n < 1 || n > 4096) return fail(LBM_EINVAL, "batch size must be in [1, 4096]");
    if (tile_x != 64 && tile_x != 128 && tile_x != 256) return fail(LBM_EINVAL, "tile_x must be 64, 128 or 256");
    if (blocks_per_cu < 1 || blocks_per_cu > 16) return fail(LBM_EINVAL, "blocks_per_cu must be in [1, 16]");
    for (int i = 0; i < n; ++i) {
        const lbm_ctx* c = ctxs[i];
        if (!c) return fail(LBM_EINVAL, "NULL member");
        if (c->dim == 3) return fail(LBM_EINVAL, "batch members must be 2D");
        if (c->coll != COLL_RR || c->thermal)
            return fail(LBM_EINVAL, "batch members must use the isothermal recursive regularization");
        if (c->store == ST_MOM) return fail(LBM_EINVAL, "batch members must store populations");
        if (c->store != ctxs[0]->store) return fail(LBM_EINVAL, "batch members must share the storage type");
        if (c->stream != ctxs[0]->stream) return fail(LBM_EINVAL, "batch members must share the stream");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(LBM_EINVAL, "a context appears twice in the batch");
    }
    lbm_batch* b = new (std::nothrow) lbm_batch;
    if (!b) return fail(LBM_ENOMEM, "batch allocation failed");
    b->members.assign(ctxs, ctxs + n);
    b->store = ctxs[0]->store;
    b->stream = ctxs[0]->stream;
    b->tile_x = tile_x;
    b->bpc = blocks_per_cu;
    int dev = 0, ncu = 0;
    int e = LBM_OK;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        e = fail(LBM_EDEVICE, "cannot query the compute-unit count");
    b->num_cu = ncu;
    if (!e && (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess ||
               hipMalloc(&b->d_desc, sizeof(InstDesc) * n) != hipSuccess ||
               hipMalloc(&b->d_begin, sizeof(int) * (n + 1)) != hipSuccess))
        e = fail(LBM_EDEVICE, "batch device allocation failed");
    if (!e) e = batch_prepare(b);
    if (e) {
        lbm_batch_destroy(b);
        return e;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int nsteps)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    int e = batch_sync_parity(b);
    if (e) return e;
    for (int s = 0; s + 1 < nsteps; s += 2) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    if (b->store == ST_BF16) // the graph advanced the device copies of the keys
        for (InstDesc& d : b->desc) d.seq += uint32_t(nsteps & ~1);
    if (nsteps % 2) {
        HIP_TRY(launch_batch_any(b, b->stream, 0));
        for (lbm_ctx* c : b->members) c->cur ^= 1;
    }
    for (lbm_ctx* c : b->members) c->steps += nsteps;
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, int steps_per_trial, char* report, int report_len)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (steps_per_trial < 2) return fail(LBM_EINVAL, "steps_per_trial must be >= 2");
    const int steps = steps_per_trial & ~1;
    static const int tiles[3] = { 64, 128, 256 };
    static const int bpcs[4] = { 2, 4, 8, 16 };
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::string rep;
    float best = 1e30f;
    int best_t = b->tile_x, best_b = b->bpc, err = LBM_OK;
    for (int t : tiles) {
        for (int bp : bpcs) {
            b->tile_x = t;
            b->bpc = bp;
            if ((err = batch_prepare(b)) != LBM_OK) break;
            if ((err = lbm_batch_step(b, 2)) != LBM_OK) break; // warm-up
            float ms = 0;
            if (hipEventRecord(e0, b->stream) != hipSuccess || lbm_batch_step(b, steps) != LBM_OK ||
                hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                err = fail(LBM_EDEVICE, "autotune timing failed");
                break;
            }
            const float per = ms / steps;
            char line[64];
            std::snprintf(line, sizeof(line), "%d %d %.5f\n", t, bp, per);
            rep += line;
            if (per < best) {
                best = per;
                best_t = t;
                best_b = bp;
            }
        }
        if (err) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tile_x = best_t;
    b->bpc = best_b;
    const int e2 = batch_prepare(b);
    if (report && report_len > 0) {
        std::snprintf(report, size_t(report_len), "%s", rep.c_str());
    }
    return err ? err : e2;
}

int lbm_batch_config(const lbm_batch* b, int* tile_x, int* blocks_per_cu)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (tile_x) *tile_x = b->tile_x;
    if (blocks_per_cu) *blocks_per_cu = b->bpc;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return;
    if (b->stream || b->capture) (void)hipStreamSynchronize(b->stream);
    batch_release_graph(b);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_begin) (void)hipFree(b->d_begin);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

} // extern "C"

// ================================================================ closure

struct lbm_mlp {
    float* theta = nullptr; // caller-owned
    hipStream_t stream = nullptr;
    int64_t max_batch = 0;
    int nblocks = 0;
    int t = 0; // Adam steps taken
    float *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr, *loss = nullptr;
    MlpInfer* fi = nullptr;
    MlpBack* fb = nullptr;
    std::vector<float> loss_host;
};

namespace {

template <class L, class S>
struct SampleOp {
    static hipError_t run(const lbm_ctx* c, int factor, double sf, float* x, float* r)
    {
        const int64_t nc = int64_t(c->nx / factor) * (c->ny / factor);
        k_closure_samples<S><<<dim3(unsigned((nc + 255) / 256)), dim3(256), 0, c->stream>>>(
            c->buf[c->cur], c->lay, factor, sf, x, r);
        return hipGetLastError();
    }
};

hipError_t launch_frags(const float* theta, MlpInfer* fi, MlpBack* fb, hipStream_t st)
{
    k_mlp_frags<<<dim3(12), dim3(256), 0, st>>>(theta, fi, fb); // 44 * 64 + 144 threads
    return hipGetLastError();
}

} // namespace

extern "C" {

int lbm_closure_samples(lbm_ctx* c, int factor, float* x, float* r)
{
    if (!c || !x || !r) return fail(LBM_EINVAL, "ctx, x or r is NULL");
    if (c->lattice != LBM_D2V37 || c->coll != COLL_RR || c->thermal || c->store == ST_MOM)
        return fail(LBM_EINVAL, "closure samples need an isothermal RR D2V37 context storing populations");
    if (factor < 1 || factor > 8 || c->nx % factor || c->ny % factor)
        return fail(LBM_EINVAL, "factor must be in [1, 8] and divide nx and ny");
    const double sf = (1.0 - 0.5 / c->tau) / (1.0 - 1.0 / c->tau);
    if (!std::isfinite(sf)) return fail(LBM_ETAU, "fine tau must differ from 1");
    // fine D2V37 is the only lattice: dispatch on the storage type alone
    hipError_t he = hipSuccess;
    switch (c->store) {
    case ST_F32: he = SampleOp<D2V37, StoreF32>::run(c, factor, sf, x, r); break;
    case ST_BF16: he = SampleOp<D2V37, StoreBF16>::run(c, factor, sf, x, r); break;
    default: he = SampleOp<D2V37, StoreF64>::run(c, factor, sf, x, r); break;
    }
    if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("samples launch: ") + hipGetErrorString(he));
    return LBM_OK;
}

int lbm_mlp_stats(const float* x, const float* r, int64_t n, float* norm, void* stream)
{
    if (!x || !r || !norm || n < 1) return fail(LBM_EINVAL, "x, r, norm or n invalid");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = int(std::min<int64_t>(256, (n + 255) / 256));
    double* part = nullptr;
    HIP_TRY(hipMalloc(&part, sizeof(double) * 4 * STAT_COLS * nb));
    k_col_stats<<<dim3(nb), dim3(256), 0, st>>>(x, r, n, part);
    hipError_t he = hipGetLastError();
    std::vector<double> hp(size_t(4 * STAT_COLS * nb));
    if (he == hipSuccess) he = hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("stats: ") + hipGetErrorString(he));
    std::vector<float> nv(NORM_N, 0.0f);
    for (int i = 0; i < 8; ++i) {
        nv[NORM_IN_STD + i] = 1.0f;
        nv[NORM_IN_LO + i] = -1e30f;
        nv[NORM_IN_HI + i] = 1e30f;
    }
    for (int i = 0; i < 16; ++i) {
        nv[NORM_OUT_STD + i] = 1.0f;
        nv[NORM_OUT_LO + i] = -1e30f;
        nv[NORM_OUT_HI + i] = 1e30f;
    }
    for (int col = 0; col < STAT_COLS; ++col) {
        double s1 = 0, s2 = 0, lo = 1e300, hi = -1e300;
        for (int b = 0; b < nb; ++b) {
            const double* p = hp.data() + size_t(b) * 4 * STAT_COLS;
            s1 += p[col];
            s2 += p[STAT_COLS + col];
            lo = std::min(lo, p[2 * STAT_COLS + col]);
            hi = std::max(hi, p[3 * STAT_COLS + col]);
        }
        const double mean = s1 / double(n);
        const double var = std::max(0.0, s2 / double(n) - mean * mean);
        const double sd = var > 0 ? std::sqrt(var) : 1.0;
        const bool in = col < 7;
        const int j = in ? col : col - 7;
        nv[(in ? NORM_IN_MEAN : NORM_OUT_MEAN) + j] = float(mean);
        nv[(in ? NORM_IN_STD : NORM_OUT_STD) + j] = float(sd);
        nv[(in ? NORM_IN_LO : NORM_OUT_LO) + j] = float((lo - mean) / sd);
        nv[(in ? NORM_IN_HI : NORM_OUT_HI) + j] = float((hi - mean) / sd);
    }
    HIP_TRY(hipMemcpyAsync(norm, nv.data(), sizeof(float) * NORM_N, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return LBM_OK;
}

int lbm_mlp_normalize(float* x, float* r, int64_t n, const float* norm, void* stream)
{
    if (!x || !r || !norm || n < 0) return fail(LBM_EINVAL, "x, r, norm or n invalid");
    if (n == 0) return LBM_OK;
    k_normalize<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream)>>>(x, r, n, norm);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m);

int lbm_mlp_create(lbm_mlp** out, float* theta, int64_t max_batch, void* stream)
{
    if (!out || !theta || max_batch < 1) return fail(LBM_EINVAL, "out, theta or max_batch invalid");
    lbm_mlp* m = new (std::nothrow) lbm_mlp;
    if (!m) return fail(LBM_ENOMEM, "mlp allocation failed");
    m->theta = theta;
    m->stream = static_cast<hipStream_t>(stream);
    m->max_batch = max_batch;
    m->nblocks = int(std::min<int64_t>(128, (max_batch + 63) / 64));
    const int nw = 4 * m->nblocks;
    bool ok = hipMalloc(&m->m, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->v, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->grad, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->partial, sizeof(float) * MLP_NPARAM * nw) == hipSuccess &&
              hipMalloc(&m->loss, sizeof(float) * nw) == hipSuccess &&
              hipMalloc(&m->fi, sizeof(MlpInfer)) == hipSuccess && hipMalloc(&m->fb, sizeof(MlpBack)) == hipSuccess;
    ok = ok && hipMemsetAsync(m->m, 0, sizeof(float) * MLP_NPARAM, m->stream) == hipSuccess &&
         hipMemsetAsync(m->v, 0, sizeof(float) * MLP_NPARAM, m->stream) == hipSuccess;
    if (!ok) {
        lbm_mlp_destroy(m);
        return fail(LBM_EDEVICE, "mlp device allocation failed");
    }
    m->loss_host.resize(size_t(nw));
    *out = m;
    return LBM_OK;
}

int lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t n, float* y)
{
    if (!m || !x || !y || n < 0) return fail(LBM_EINVAL, "mlp, x, y or n invalid");
    if (n == 0) return LBM_OK;
    HIP_TRY(launch_frags(m->theta, m->fi, m->fb, m->stream));
    const int64_t blocks = (n + 63) / 64; // 16 samples per wave, 4 waves per block
    k_mlp_forward<<<dim3(unsigned(blocks)), dim3(256), 0, m->stream>>>(m->fi, x, n, y);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int lbm_mlp_step(lbm_mlp* m, const float* x, const float* t, const int* idx, int64_t batch, float lr, float* grad,
                 double* loss)
{
    if (!m || !x || !t) return fail(LBM_EINVAL, "mlp, x or t is NULL");
    if (batch < 1 || batch > m->max_batch) return fail(LBM_EINVAL, "batch must be in [1, max_batch]");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(LBM_EINVAL, "lr must be finite and >= 0");
    HIP_TRY(launch_frags(m->theta, m->fi, m->fb, m->stream));
    const int nb = int(std::min<int64_t>(m->nblocks, (batch + 63) / 64));
    GradArgs ga{ m->fi, m->fb, x, t, idx, batch, float(2.0 / (double(batch) * MLP_OUT)), m->partial, m->loss };
    k_mlp_grad<<<dim3(unsigned(nb)), dim3(256), 0, m->stream>>>(ga);
    HIP_TRY(hipGetLastError());
    float bc1 = 1.0f, bc2 = 1.0f;
    if (lr > 0.0f) {
        ++m->t;
        bc1 = float(1.0 - std::pow(0.9, m->t));
        bc2 = float(1.0 - std::pow(0.999, m->t));
    }
    k_mlp_reduce_adam<<<dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, m->stream>>>(
        m->partial, 4 * nb, grad ? grad : m->grad, m->theta, m->m, m->v, lr, bc1, bc2);
    HIP_TRY(hipGetLastError());
    if (loss) {
        HIP_TRY(hipMemcpyAsync(m->loss_host.data(), m->loss, sizeof(float) * 4 * nb, hipMemcpyDeviceToHost, m->stream));
        HIP_TRY(hipStreamSynchronize(m->stream));
        double sum = 0;
        for (int w = 0; w < 4 * nb; ++w) sum += m->loss_host[size_t(w)];
        *loss = sum / (double(batch) * MLP_OUT);
    }
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (void* p : { (void*)m->m, (void*)m->v, (void*)m->grad, (void*)m->partial, (void*)m->loss, (void*)m->fi,
                     (void*)m->fb })
        if (p) (void)hipFree(p);
    delete m;
}

int lbm_closure_set(lbm_ctx* c, const float* theta, const float* norm)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!theta) {
        c->closure = false;
        return LBM_OK;
    }
    if (!norm) return fail(LBM_EINVAL, "norm is NULL");
    if (c->lattice != LBM_D2V37 || c->coll != COLL_RR || c->thermal || c->store == ST_MOM)
        return fail(LBM_EINVAL, "the closure needs an isothermal RR D2V37 context storing populations");
    if (!c->cl_frags) {
        HIP_TRY(hipMalloc(&c->cl_frags, sizeof(MlpInfer)));
        HIP_TRY(hipMalloc(&c->cl_norm, sizeof(float) * NORM_N));
        HIP_TRY(hipMalloc(&c->cl_fallbacks, sizeof(unsigned long long)));
    }
    HIP_TRY(launch_frags(theta, c->cl_frags, nullptr, c->stream));
    HIP_TRY(hipMemcpyAsync(c->cl_norm, norm, sizeof(float) * NORM_N, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->cl_fallbacks, 0, sizeof(unsigned long long), c->stream));
    c->closure = true;
    return LBM_OK;
}

int lbm_closure_fallbacks(lbm_ctx* c, int64_t* count)
{
    if (!c || !count) return fail(LBM_EINVAL, "ctx or count is NULL");
    if (!c->cl_fallbacks) {
        *count = 0;
        return LBM_OK;
    }
    unsigned long long v = 0;
    HIP_TRY(hipMemcpyAsync(&v, c->cl_fallbacks, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *count = int64_t(v);
    return LBM_OK;
}

} // extern "C"
