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
// destination buffer with non-temporal stores.  The two buffers alternate; the
// state kept between steps is post-collision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
    static __device__ __forceinline__ double load(const double* p) { return *p; }
    static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
    static __device__ __forceinline__ void store_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
};

struct StoreF32 {
    using elem = float;
    using math = float;
    static constexpr bool shifted = true;
    static __device__ __forceinline__ float load(const float* p) { return *p; }
    static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
    static __device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
};

// bfloat16 = the upper half of an IEEE float; stores round to nearest even.
struct StoreBF16 {
    using elem = uint16_t;
    using math = float;
    static constexpr bool shifted = true;
    static __device__ __forceinline__ float load(const uint16_t* p)
    {
        return __uint_as_float(uint32_t(*p) << 16);
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
};

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
    double keep;    // 1 - 1/tau
    double inv_tau;
    int order;
};

// The hardware hands consecutive workgroup ids to the 8 XCDs in turn; with
// the remap, XCD k works on the k-th contiguous eighth of the tiles, so
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int block_index(const StepArgs& a)
{
    const int id = int(blockIdx.x);
    if (!a.xcd_remap) return id;
    const int q = a.nblocks / 8, r = a.nblocks % 8;
    const int xcd = id % 8, local = id / 8;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <class L, class S, int COLL, bool THERMAL, bool A13P, bool PULL>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(RRLBM_WAVES_PER_EU)))
void k_stream_collide(StepArgs a)
{
    using T = typename S::math;
    using E = typename S::elem;
    constexpr int R = L::R;
    const int bid = block_index(a);
    const int x = (bid % a.bx_blocks) * BX + int(threadIdx.x);
    const int y = (bid / a.bx_blocks) * BY + int(threadIdx.y);
    const Layout& lay = a.lay;
    if (x >= lay.nx || y >= lay.ny) return;
    const E* __restrict__ fin = static_cast<const E*>(a.fin);
    E* __restrict__ fout = static_cast<E*>(a.fout);
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
        v[I] = S::load(fin + idx);
    });

    collide_node<L, T, COLL, THERMAL, S::shifted, A13P>(v, T(a.keep), T(a.inv_tau), a.order);

    static_for<L::Q>([&](auto I) { S::store_nt(fout + here + int(I) * lay.te, v[I]); });
}

// ------------------------------------------------------------ init kernel

struct InitArgs {
    void* f;
    Layout lay;
    const double *rho, *ux, *uy, *theta, *noise;
    double noise_amp;
    int eq_order;
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
    typename S::elem* out = static_cast<typename S::elem*>(a.f);
    static_for<L::Q>([&](auto I) {
        double v = f[I];
        if (a.noise) v += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k];
        S::store(out + here + int(I) * a.lay.te, typename S::math(v));
    });
}

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
        double r = 0, jx = 0, jy = 0, e2 = 0;
        static_for<L::Q>([&](auto I) {
            double v = double(S::load(f + here + int(I) * lay.te));
            if (S::shifted) v += L::v.w[I];
            constexpr double cx = L::v.cx[I], cy = L::v.cy[I];
            r += v;
            jx += cx * v;
            jy += cy * v;
            e2 += (cx * cx + cy * cy) * v;
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

enum StoreKind { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };

struct LatInfo {
    int q, reach, n_eq;
    double cs2;
};

template <class L>
LatInfo info_of()
{
    return { L::Q, L::R, L::NEQ, L::cs2 };
}

bool lattice_info(int lattice, LatInfo* out)
{
    switch (lattice) {
    case LBM_D2Q9: *out = info_of<D2Q9>(); return true;
    case LBM_D2V17: *out = info_of<D2V17>(); return true;
    case LBM_D2V37: *out = info_of<D2V37>(); return true;
    }
    return false;
}


} // namespace

struct lbm_ctx {
    int lattice = 0, nx = 0, ny = 0, order = 2;
    double tau = 1.0;
    uint32_t flags = 0;
    int store = ST_F64, coll = COLL_RR;
    bool thermal = false, a13p = false;
    int q = 0;
    Layout lay{};
    int xcd_remap = 1;
    void* buf[2] = { nullptr, nullptr };
    int cur = 0;
    int64_t steps = 0;
    hipStream_t stream = nullptr;
    // moments scratch
    double* fields = nullptr; // 5 fields of nx*ny
    double* partial = nullptr;
    double* partial_host = nullptr;
    int64_t nblk = 0;
};

namespace {

template <class L, class S, int COLL, bool TH, bool A13P>
hipError_t launch_step_t(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    const int bxn = (c->nx + BX - 1) / BX, byn = (c->ny + BY - 1) / BY;
    StepArgs a{ fin, fout, c->lay, bxn, bxn * byn, c->xcd_remap, 1.0 - 1.0 / c->tau, 1.0 / c->tau, c->order };
    dim3 grid(unsigned(bxn * byn)), block(BX, BY);
    if (pull)
        k_stream_collide<L, S, COLL, TH, A13P, true><<<grid, block, 0, c->stream>>>(a);
    else
        k_stream_collide<L, S, COLL, TH, A13P, false><<<grid, block, 0, c->stream>>>(a);
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

hipError_t launch_step(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
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
    if (nx < li->reach || ny < li->reach || nx < 1 || ny < 1)
        return fail(LBM_EINVAL, "grid " + std::to_string(nx) + "x" + std::to_string(ny) +
                                    " smaller than the lattice reach " + std::to_string(li->reach));
    if (layout_elems(li->q, nx, ny) >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "grid too large");
    if (!std::isfinite(tau) || !(tau > 0.5)) return fail(LBM_ETAU, "tau must be finite and > 1/2");
    const uint32_t known = LBM_THERMAL | LBM_STORE_FP32 | LBM_STORE_BF16 | LBM_COLL_PR | LBM_COLL_BGK |
                           LBM_EQ_INIT_ORDER2 | LBM_A13_PROJECTED;
    if (flags & ~known) return fail(LBM_EINVAL, "unknown flag bits");
    if ((flags & LBM_STORE_FP32) && (flags & LBM_STORE_BF16)) return fail(LBM_EINVAL, "two storage flags");
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
    default: return fail(LBM_EINVAL, "unknown lattice");
    }
    for (int i = 0; i < t->q; ++i) {
        if (cx) cx[i] = t->cx[i];
        if (cy) cy[i] = t->cy[i];
        if (w) w[i] = t->w[i];
    }
    return LBM_OK;
}

int64_t lbm_buffer_elems(int lattice, int nx, int ny)
{
    LatInfo li;
    if (!lattice_info(lattice, &li)) return fail(LBM_EINVAL, "unknown lattice");
    if (nx < 1 || ny < 1) return fail(LBM_EINVAL, "empty grid");
    return layout_elems(li.q, nx, ny);
}

int lbm_init(lbm_ctx** out, int lattice, int nx, int ny, double tau, int reg_order, uint32_t flags,
             void* f_a, void* f_b, const double* rho, const double* ux, const double* uy,
             const double* theta, const double* noise, double noise_amp, void* stream)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    LatInfo li;
    int e = validate(lattice, nx, ny, tau, reg_order, flags, &li);
    if (e) return e;
    if (!f_a || !f_b || f_a == f_b) return fail(LBM_EINVAL, "two distinct population buffers are needed");
    if (!rho || !ux || !uy) return fail(LBM_EINVAL, "rho, ux and uy are required");
    if ((flags & LBM_THERMAL) == 0 && theta)
        return fail(LBM_EINVAL, "theta given for an isothermal run");
    if (!std::isfinite(noise_amp)) return fail(LBM_EINVAL, "noise_amp not finite");

    lbm_ctx* c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ENOMEM, "context allocation failed");
    c->lattice = lattice;
    c->nx = nx;
    c->ny = ny;
    c->tau = tau;
    c->order = (flags & LBM_COLL_BGK) ? 2 : reg_order;
    c->flags = flags;
    c->store = (flags & LBM_STORE_FP32) ? ST_F32 : (flags & LBM_STORE_BF16) ? ST_BF16 : ST_F64;
    c->coll = (flags & LBM_COLL_PR) ? COLL_PR : (flags & LBM_COLL_BGK) ? COLL_BGK : COLL_RR;
    c->thermal = (flags & LBM_THERMAL) != 0;
    c->a13p = (flags & LBM_A13_PROJECTED) != 0;
    c->q = li.q;
    c->lay = make_layout(li.q, nx, ny);
    // tuning knob: RRLBM_XCD_REMAP=0 keeps the hardware's round-robin block order
    if (const char* e = std::getenv("RRLBM_XCD_REMAP")) c->xcd_remap = std::atoi(e) != 0;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->stream = static_cast<hipStream_t>(stream);
    const int64_t n = int64_t(nx) * ny;
    c->nblk = (n + 255) / 256;

    InitArgs ia{ f_a, c->lay, rho, ux, uy, theta, noise, noise_amp,
                 (flags & LBM_EQ_INIT_ORDER2) ? 2 : li.n_eq };
    hipError_t he = dispatch_ls<InitOp>(c, ia);
    if (he == hipSuccess) he = launch_step(c, f_a, f_a, false); // collide in place: post-collision state
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

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* theta, double* vort, double* sums)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
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
    HIP_TRY(dispatch_ls<PopOp>(c, f_out));
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    if (c->fields) (void)hipFree(c->fields);
    if (c->partial) (void)hipFree(c->partial);
    if (c->partial_host) (void)hipHostFree(c->partial_host);
    delete c;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

} // extern "C"
