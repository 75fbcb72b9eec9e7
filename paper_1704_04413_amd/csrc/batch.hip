// The persistent batch kernels for one storage kind, chosen at compile time
// (RR_STORE = ST_F64, ST_F32, ST_BF16 or ST_F32D): one per 2D lattice, each walking
// the work list of that lattice's members, and one that walks a list mixing
// every lattice.
#include "context.hpp"
#include "step2d.hpp"

#if !defined(RR_STORE)
#error "compile with -DRR_STORE=<storage kind>"
#endif

namespace rr {

#if RR_STORE == 0
using BatchSto = StoreF64;
#elif RR_STORE == 1
using BatchSto = StoreF32;
#elif RR_STORE == 2
using BatchSto = StoreBF16;
#elif RR_STORE == 3
using BatchSto = StoreF32D;
#else
#error "RR_STORE must be a population storage"
#endif

// lattice: LBM_D2Q9..LBM_D2V37 when every member of the list has it, -1 for a mixed list.
#define RR_BATCH_NAME_(s) batch_launch_##s
#define RR_BATCH_NAME(s) RR_BATCH_NAME_(s)
hipError_t RR_BATCH_NAME(RR_STORE)(int lattice, const InstDesc* desc, const int* begin, int n, int total, int parity,
                                   int tile_x, int grid, hipStream_t st)
{
    const dim3 g = dim3(unsigned(grid));
    if (tile_x >= batch_wide_tile) {
        const dim3 blk = dim3(BX * BY, 1);
        switch (lattice) {
        case LBM_D2Q9: k_batch<BatchSto, 0, true><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
        case LBM_D2V17: k_batch<BatchSto, 1, true><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
        case LBM_D2V37: k_batch<BatchSto, 2, true><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
        default: k_batch<BatchSto, -1, true><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
        }
        return hipGetLastError();
    }
    const dim3 blk = dim3(BX, BY);
    switch (lattice) {
    case LBM_D2Q9: k_batch<BatchSto, 0><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
    case LBM_D2V17: k_batch<BatchSto, 1><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
    case LBM_D2V37: k_batch<BatchSto, 2><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
    default: k_batch<BatchSto, -1><<<g, blk, 0, st>>>(desc, begin, n, total, parity, tile_x); break;
    }
    return hipGetLastError();
}

} // namespace rr
