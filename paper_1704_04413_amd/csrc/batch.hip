// The persistent batch kernel for one storage kind, chosen at compile time
// (RR_STORE = ST_F64, ST_F32 or ST_BF16); it walks a work list of tiles that
// spans members of every 2D lattice.
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
#else
#error "RR_STORE must be a population storage"
#endif

#define RR_BATCH_NAME_(s) batch_launch_##s
#define RR_BATCH_NAME(s) RR_BATCH_NAME_(s)
hipError_t RR_BATCH_NAME(RR_STORE)(const InstDesc* desc, const int* begin, int n, int total, int parity, int tile_x,
                                   int grid, hipStream_t st)
{
    k_batch<BatchSto><<<dim3(unsigned(grid)), dim3(BX, BY), 0, st>>>(desc, begin, n, total, parity, tile_x);
    return hipGetLastError();
}

} // namespace rr
