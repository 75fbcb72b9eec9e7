// The 2D population step for one (lattice, storage) pair, chosen at compile
// time: this file is compiled once per pair (RR_LAT = LBM_D2Q9, LBM_D2V17 or
// LBM_D2V37; RR_STORE = ST_F64, ST_F32, ST_BF16 or ST_F32D), so the pairs
// build in parallel.  It provides the step launch (every collision, thermal
// variant and cache policy) of both schemes, the initial state, the
// population dump and the diagnostics.
#include "context.hpp"
#include "step2d.hpp"

#if !defined(RR_LAT) || !defined(RR_STORE)
#error "compile with -DRR_LAT=<2D lattice id> -DRR_STORE=<storage kind>"
#endif

namespace rr {
namespace {

#if RR_LAT == 0
using Lat = D2Q9;
#elif RR_LAT == 1
using Lat = D2V17;
#elif RR_LAT == 2
using Lat = D2V37;
#else
#error "RR_LAT must be a 2D lattice"
#endif

#if RR_STORE == 0
using Sto = StoreF64;
#elif RR_STORE == 1
using Sto = StoreF32;
#elif RR_STORE == 2
using Sto = StoreBF16;
#elif RR_STORE == 3
using Sto = StoreF32D;
#else
#error "RR_STORE must be a population storage"
#endif

template <int COLL, bool TH, bool A13P>
hipError_t step_t(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    if constexpr (Lat::id == LBM_D2V37 && COLL == COLL_RR && !TH) {
        if (pull && c->closure) return closure_step(c, fin, fout);
    }
    using B = StepBlock<Lat, Sto, false>;
    const StepArgs a = step_blocks<B>(step_args(c, fin, fout, pull));
    const dim3 grid(unsigned(a.nblocks)), block(B::x, B::y);
    if (!pull)
        k_stream_collide<Lat, Sto, COLL, TH, A13P, false, POL_STREAM><<<grid, block, 0, c->stream>>>(a);
    else if (c->pol == POL_CACHE)
        k_stream_collide<Lat, Sto, COLL, TH, A13P, true, POL_CACHE><<<grid, block, 0, c->stream>>>(a);
    else if (c->pol == POL_KEEP)
        k_stream_collide<Lat, Sto, COLL, TH, A13P, true, POL_KEEP><<<grid, block, 0, c->stream>>>(a);
    else
        k_stream_collide<Lat, Sto, COLL, TH, A13P, true, POL_STREAM><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t step(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    if constexpr (Lat::id == LBM_D2V37) {
        if (c->thermal) {
            switch (c->coll) {
            case COLL_PR: return step_t<COLL_PR, true, false>(c, fin, fout, pull);
            case COLL_BGK: return step_t<COLL_BGK, true, false>(c, fin, fout, pull);
            default:
                return c->a13p ? step_t<COLL_RR, true, true>(c, fin, fout, pull)
                               : step_t<COLL_RR, true, false>(c, fin, fout, pull);
            }
        }
    }
    switch (c->coll) {
    case COLL_PR: return step_t<COLL_PR, false, false>(c, fin, fout, pull);
    case COLL_BGK: return step_t<COLL_BGK, false, false>(c, fin, fout, pull);
    default: return step_t<COLL_RR, false, false>(c, fin, fout, pull);
    }
}

template <int COLL, bool TH, bool A13P>
hipError_t step_aa_t(const lbm_ctx* c, bool shifted, uint32_t seq)
{
    using B = StepBlock<Lat, Sto, true>;
    StepArgs a = step_blocks<B>(step_args(c, c->buf[0], c->buf[0], true));
    a.seq = seq;
    // POL_STREAM: non-temporal stores, tiles in order.  POL_CACHE: ordinary
    // stores; POL_KEEP: non-temporal stores where they fill whole lines (the
    // node's own slots) and ordinary ones where they are shifted; with both,
    // the tile order is reversed every other step.
    a.reverse = (c->pol != POL_STREAM && (c->steps & 1)) ? 1 : 0;
    const dim3 grid(unsigned(a.nblocks)), block(B::x, B::y);
    const bool nt = c->pol == POL_STREAM || (c->pol == POL_KEEP && !shifted);
    if (shifted && nt)
        k_stream_collide_aa<Lat, Sto, COLL, TH, A13P, true, true><<<grid, block, 0, c->stream>>>(a);
    else if (shifted)
        k_stream_collide_aa<Lat, Sto, COLL, TH, A13P, true, false><<<grid, block, 0, c->stream>>>(a);
    else if (nt)
        k_stream_collide_aa<Lat, Sto, COLL, TH, A13P, false, true><<<grid, block, 0, c->stream>>>(a);
    else
        k_stream_collide_aa<Lat, Sto, COLL, TH, A13P, false, false><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t step_aa(const lbm_ctx* c, bool shifted, uint32_t seq)
{
    if constexpr (Lat::id == LBM_D2V37) {
        if (c->thermal) {
            switch (c->coll) {
            case COLL_PR: return step_aa_t<COLL_PR, true, false>(c, shifted, seq);
            case COLL_BGK: return step_aa_t<COLL_BGK, true, false>(c, shifted, seq);
            default:
                return c->a13p ? step_aa_t<COLL_RR, true, true>(c, shifted, seq)
                               : step_aa_t<COLL_RR, true, false>(c, shifted, seq);
            }
        }
    }
    switch (c->coll) {
    case COLL_PR: return step_aa_t<COLL_PR, false, false>(c, shifted, seq);
    case COLL_BGK: return step_aa_t<COLL_BGK, false, false>(c, shifted, seq);
    default: return step_aa_t<COLL_RR, false, false>(c, shifted, seq);
    }
}

hipError_t init(const lbm_ctx* c, const InitArgs& a)
{
    const int64_t n = int64_t(c->nx) * c->ny;
    k_init<Lat, Sto><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t populations(const lbm_ctx* c, const void* src, double* out)
{
    const int64_t n = int64_t(c->nx) * c->ny;
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    switch (state_placement(c)) {
    case 1: k_populations<Lat, Sto, 1><<<grid, block, 0, c->stream>>>(src, c->lay, out); break;
    case 2: k_populations<Lat, Sto, 2><<<grid, block, 0, c->stream>>>(src, c->lay, out); break;
    default: k_populations<Lat, Sto, 0><<<grid, block, 0, c->stream>>>(src, c->lay, out);
    }
    return hipGetLastError();
}

hipError_t moments(const lbm_ctx* c, double* r, double* ux, double* uy, double* th, double* partial)
{
    const dim3 grid(unsigned(c->nblk)), block(256);
    const void* f = c->buf[c->cur];
    const int t = c->thermal ? 1 : 0;
    switch (state_placement(c)) {
    case 1: k_moments<Lat, Sto, 1><<<grid, block, 0, c->stream>>>(f, c->lay, t, r, ux, uy, th, partial); break;
    case 2: k_moments<Lat, Sto, 2><<<grid, block, 0, c->stream>>>(f, c->lay, t, r, ux, uy, th, partial); break;
    default: k_moments<Lat, Sto, 0><<<grid, block, 0, c->stream>>>(f, c->lay, t, r, ux, uy, th, partial);
    }
    return hipGetLastError();
}

} // namespace

#define RR_OPS2D_NAME_(l, s) ops2d_##l##_##s
#define RR_OPS2D_NAME(l, s) RR_OPS2D_NAME_(l, s)
const Ops2D& RR_OPS2D_NAME(RR_LAT, RR_STORE)()
{
    static const Ops2D ops{ step, step_aa, init, populations, moments };
    return ops;
}

} // namespace rr
