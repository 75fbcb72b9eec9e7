// Kernels of the 2D population step: storage types (FP64, weight-shifted FP32
// and BF16 with stochastic rounding), the fused pull stream-and-collide kernel,
// the batched persistent kernel, the initial state, and the per-node
// diagnostics.  Templates only; each translation unit instantiates the
// (lattice, storage) pairs it serves.  The layout is the row-tiled one of
// common.hpp.  One step is one launch of a pull kernel: the thread of node x
// gathers f_i(x - c_i) from the source buffer (one fixed offset per plane, so
// every stored value is read exactly once), collides in registers and writes
// its Q post-collision values to the destination buffer, with the load and
// store kinds of the cache policy that the buffer size selects (Policy).  The
// two buffers alternate; the state kept between steps is post-collision.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "collide.hpp"
#include "common.hpp"
#include "storage.hpp"

namespace rr {

// ------------------------------------------------------------ step kernel

// Minimum waves per SIMD the compiler must leave room for in the step
// kernel (register budget); more resident waves keep more loads in flight
// while other waves run the collision arithmetic.
#ifndef RRLBM_WAVES_PER_EU
#define RRLBM_WAVES_PER_EU 4
#endif
// The same for the in-place (AA) step kernel.
#ifndef RRLBM_AA_WAVES_PER_EU
#define RRLBM_AA_WAVES_PER_EU 4
#endif

// Block of the 2D step kernels (pull and in-place): four waves side by side
// along x on one row, 256 consecutive nodes, or one wave per row of a 4-row
// tile (64 x 4).  The wide block measured faster on every lattice and storage
// but the D2Q9 FP64 pull step (% of the HBM peak, 64 x 4 -> 256 x 1: D2V37
// FP64 1024^2 pull 75.9 -> 79.2, in place 80.6 -> 84.3; D2V37 FP32 2048^2
// pull 68.3 -> 72.8; D2Q9 FP64 4096^2 pull 74.3 -> 71.7).  The closure and
// batch kernels keep 64 x 4.
template <class L, class S, bool INPLACE>
struct StepBlock {
    static constexpr bool tall = !INPLACE && L::Q == 9 && sizeof(typename S::elem) == 8;
    static constexpr int x = tall ? BX : 4 * BX, y = tall ? BY : 1;
};

// The launch shape of a 2D step over the whole grid in blocks of B.
template <class B>
inline StepArgs step_blocks(StepArgs a)
{
    a.bx_blocks = (a.lay.nx + B::x - 1) / B::x;
    a.nblocks = a.bx_blocks * ((a.lay.ny + B::y - 1) / B::y);
    return a;
}

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
    using B = StepBlock<L, S, false>;
    const int bid = block_index(a);
    const int x = (bid % a.bx_blocks) * B::x + int(threadIdx.x);
    const int y = (bid / a.bx_blocks) * B::y + int(threadIdx.y);
    if (x >= a.lay.nx || y >= a.lay.ny) return;
    node_update<L, S, COLL, THERMAL, A13P, PULL, POL == POL_STREAM, POL == POL_KEEP>(
        static_cast<const typename S::elem*>(a.fin), static_cast<typename S::elem*>(a.fout), a.lay, x, y, a.rx,
        a.seq);
}

// ------------------------------------------------ single-buffer (AA) step

// Hides v's value from the optimizer (no instruction is emitted).
__device__ __forceinline__ void opaque(int& v) { asm volatile("" : "+v"(v)); }

// One node of the in-place step on one buffer f (the AA pattern).  The state
// alternates between two placements of the post-collision values (see
// state_index).  !SHIFTED (the state after an odd number of steps, or the
// initial populations): the node finds its incoming f_i(x - c_i) in its own
// slot i and leaves its outgoing value i in its own slot opp(i).  SHIFTED
// (after an even number): value i comes from slot opp(i) of the node x - c_i
// and goes to slot i of the node x + c_i.  Either way a thread writes exactly
// the slots it has read, after reading all of them, so threads never touch
// each other's slots within one launch.  The collision, the node key and the
// dither stream are those of the pull step, so both schemes give the same
// states bit for bit.
template <class L, class S, int COLL, bool THERMAL, bool A13P, bool SHIFTED, bool NT>
__device__ __forceinline__ void node_update_aa(typename S::elem* f, const Layout& lay, int x, int y,
                                               const Relax& rx, uint32_t seq)
{
    using T = typename S::math;
    constexpr int R = L::R;
    const int nx = lay.nx, ny = lay.ny;
    const uint32_t node = uint32_t(y) * uint32_t(nx) + uint32_t(x);

    // periodic x + d and row(y + d) for d in [-R, R]
    int xs[2 * R + 1], ys[2 * R + 1];
    auto neighbours = [&](int x0, int y0) {
        static_for<2 * R + 1>([&](auto D) {
            constexpr int d = int(D) - R;
            int xx = x0 + d, yy = y0 + d;
            if constexpr (d < 0) {
                xx += (xx < 0) ? nx : 0;
                yy += (yy < 0) ? ny : 0;
            } else if constexpr (d > 0) {
                xx -= (xx >= nx) ? nx : 0;
                yy -= (yy >= ny) ? ny : 0;
            }
            xs[D] = xx;
            ys[D] = lay.row(yy);
        });
    };
    if constexpr (SHIFTED) neighbours(x, y);

    T v[L::Q];
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        constexpr int o = opp_index<L>(int(I));
        const int idx = SHIFTED ? ys[R - cy] + xs[R - cx] + o * lay.te : lay.row(y) + x + int(I) * lay.te;
        v[I] = S::load(f + idx);
    });

    collide_node<L, T, COLL, THERMAL, S::shifted, A13P, S::conserve_in_double>(v, rx);

    // The stores go to the addresses the loads used; hiding x and y makes the
    // compiler rebuild them here rather than hold all Q across the collision
    // (which spills).
    opaque(x);
    opaque(y);
    if constexpr (SHIFTED) neighbours(x, y);
    const int here = lay.row(y) + x;

    store_node_at<L, S, T, NT>(
        [&](auto I) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
            constexpr int o = opp_index<L>(int(I));
            return f + (SHIFTED ? ys[R + cy] + xs[R + cx] + int(I) * lay.te : here + o * lay.te);
        },
        v, node, seq);
}

// a.fin == a.fout: the one state buffer.
template <class L, class S, int COLL, bool THERMAL, bool A13P, bool SHIFTED, bool NT>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(RRLBM_AA_WAVES_PER_EU)))
void k_stream_collide_aa(StepArgs a)
{
    using B = StepBlock<L, S, true>;
    const int bid = block_index(a);
    const int x = (bid % a.bx_blocks) * B::x + int(threadIdx.x);
    const int y = (bid / a.bx_blocks) * B::y + int(threadIdx.y);
    if (x >= a.lay.nx || y >= a.lay.ny) return;
    node_update_aa<L, S, COLL, THERMAL, A13P, SHIFTED, NT>(static_cast<typename S::elem*>(a.fout), a.lay, x, y,
                                                            a.rx, a.seq);
}

// ---------------------------------------------------------- batch kernel

// Persistent kernel: blocks stride over the work list (member, tile); item w
// belongs to the member i with begin[i] <= w < begin[i+1].  Each item is a
// tile_x by 4 patch of one member walked 64 columns at a time by a 64 x 4
// block, or (WIDE, tile_x >= 256) a tile_x by 1 strip walked 256 columns at a
// time by four waves along the row, the shape of the single steps' blocks.
// `parity` selects the buffer direction of this step for every member.
// LAT: the one lattice of every member of this work list (its own register
// budget), or -1 for a list that mixes lattices (one switch per work item).
template <class S, int LAT, bool WIDE = false>
__global__ __launch_bounds__(BX* BY) void k_batch(const InstDesc* __restrict__ desc, const int* __restrict__ begin,
                                                  int n, int total, int parity, int tile_x)
{
    constexpr int ROWS = WIDE ? 1 : BY, W = BX * BY / ROWS;
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
        const int y = (local / d.bx_blocks) * ROWS + int(threadIdx.y);
        const int src = d.flip ^ parity;
        const E* fin = static_cast<const E*>(d.buf[src]);
        E* fout = static_cast<E*>(d.buf[src ^ 1]);
        for (int sub = 0; sub < tile_x; sub += W) {
            const int x = x0 + sub + int(threadIdx.x);
            if (x < d.lay.nx && y < d.lay.ny) {
                const uint32_t seq = d.seq + uint32_t(parity);
                if constexpr (LAT == 0) {
                    node_update<D2Q9, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq);
                } else if constexpr (LAT == 1) {
                    node_update<D2V17, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq);
                } else if constexpr (LAT == 2) {
                    node_update<D2V37, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq);
                } else {
                    switch (d.lattice) {
                    case 0: node_update<D2Q9, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq); break;
                    case 1: node_update<D2V17, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq); break;
                    default: node_update<D2V37, S, COLL_RR, false, false, true>(fin, fout, d.lay, x, y, d.rx, seq); break;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------ init kernel

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

// --------------------------------------------------- populations / moments

// Diagnostics of one node from its post-collision populations v (a NULL field
// pointer is skipped).
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
    if (rho_o) rho_o[k] = r;
    if (ux_o) ux_o[k] = ux;
    if (uy_o) uy_o[k] = uy;
    if (th_o) th_o[k] = th;
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
// RD: where the state sits (state_index).
template <class L, class S, int RD = 0>
__global__ __launch_bounds__(256) void k_moments(const void* fsrc, Layout lay, int thermal, double* rho_o,
                                                 double* ux_o, double* uy_o, double* th_o, double* partial)
{
    const int64_t n = int64_t(lay.nx) * lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        const int x = int(k % lay.nx), y = int(k / lay.nx);
        const typename S::elem* f = static_cast<const typename S::elem*>(fsrc);
        double v[L::Q];
        static_for<L::Q>([&](auto I) {
            v[I] = double(S::load(f + state_index<L, RD, int(I)>(lay, x, y)));
            if (S::shifted) v[I] += L::v.w[I];
        });
        node_diag<L>(v, thermal, k, rho_o, ux_o, uy_o, th_o, val);
    }
    block_sums<MOM_NS>(val, partial);
}

} // namespace rr
