// Types shared by the host side of the library and its kernels: the row-tiled
// population layout, launch arguments, relaxation factors and the sizes of the
// diagnostic reductions.  No kernel is defined here.
//
// Data layout in HBM: row-tiled structure of arrays.  The grid is cut into
// tiles of TY = 4 full rows; a tile stores its Q velocity planes one after the
// other (plane i of the tile = TY*nx values, row-major), so element
// (i, y, x) lives at (y / TY) * Q*TY*nx + i * TY*nx + (y % TY) * nx + x.
// A wavefront's 64 lanes touch 64 consecutive values of one plane, and the
// 2*Q streams a block reads and writes sit inside about three tiles (a few
// MiB) instead of 2*Q planes spread over the whole buffer, which keeps the
// address-translation working set small.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rr {

enum Coll { COLL_RR = 0, COLL_PR = 1, COLL_BGK = 2 };

// Relaxation of one step: k_n = 1 - 1/tau_n for the non-equilibrium part of
// rank n (Eq. GenRegCollision with one time per order, the Hermite MRT form;
// tau_2 = tau, and 0 above the regularization order), inv_tau = 1/tau (BGK).
struct Relax {
    double k2, k3, k4, inv_tau;
};

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

constexpr int BX = 64, BY = TY; // step blocks: one 64-wide row segment per wave, one tile high

// Cache policy of the step, from the size of one state buffer against the
// 256 MiB memory-side cache: POL_STREAM ordinary loads, non-temporal stores
// (large buffers); POL_CACHE ordinary loads and stores, tile order reversed
// every other step (small buffers: the state stays in the cache);
// POL_KEEP non-temporal loads and ordinary stores (buffers about the cache's
// size: the reads no longer evict what the step writes, which the next step
// reads).
enum Policy { POL_STREAM = 0, POL_CACHE = 1, POL_KEEP = 2 };

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

struct InitArgs {
    void* f;
    Layout lay;
    const double *rho, *ux, *uy, *theta, *grad, *noise;
    double noise_amp;
    int eq_order;
    double tau;
};

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

constexpr int MOM_K = 6;    // values per node of the moment representation
constexpr int MOM_KT = 11;  // values per node of the thermal moment representation
constexpr int MOM_NS = 8;   // per-block partial sums of the 2D moments kernel
constexpr int VORT_NS = 2;  // per-block partial sums of the vorticity kernel
constexpr int MOM3_NS = 8;  // per-block partial sums of the 3D moments kernel

} // namespace rr
