// The 3D step for one lattice of Table II and one storage, chosen at compile
// time: this file is compiled four times per lattice (RR_LAT3 = LBM_D3Q19,
// LBM_D3Q27, LBM_D3V39 or LBM_D3Q103; RR_STORE3 = ST_F64 or ST_F32D, the
// latter float g = f - w with double arithmetic), so that the parts build in
// parallel.  With RR_AA3 = 0 it provides the pull step for every collision
// and cache policy, the initial state, the population dump and the
// diagnostics; with RR_AA3 = 1 the in-place single-buffer step for every
// collision, and with RR_AA3 = 2 the same kernels with non-temporal stores
// (the single-buffer step calls them for the policies that ask for them).
#include "context.hpp"
#include "storage.hpp"
#include "collide3d.hpp"

#if !defined(RR_LAT3)
#error "compile with -DRR_LAT3=<3D lattice id>"
#endif
#if !defined(RR_AA3)
#define RR_AA3 0
#endif
#if !defined(RR_STORE3)
#define RR_STORE3 0
#endif

#define RR_STEP3_AA_NAME_(l, s) step3d_aa_##l##_##s
#define RR_STEP3_AA_NAME(l, s) RR_STEP3_AA_NAME_(l, s)
#define RR_STEP3_AANT_NAME_(l, s) step3d_aant_##l##_##s
#define RR_STEP3_AANT_NAME(l, s) RR_STEP3_AANT_NAME_(l, s)

namespace rr {

// one in-place step of the single-buffer scheme (the RR_AA3 = 1 unit)
hipError_t RR_STEP3_AA_NAME(RR_LAT3, RR_STORE3)(const lbm_ctx* c, bool shifted);
// its kernels with non-temporal stores (the RR_AA3 = 2 unit); reverse: walk
// the tiles in reverse order
hipError_t RR_STEP3_AANT_NAME(RR_LAT3, RR_STORE3)(const lbm_ctx* c, bool shifted, bool reverse);

namespace {

#if RR_STORE3 == 0
using Sto3 = StoreF64;
#elif RR_STORE3 == 3
using Sto3 = StoreF32D;
#else
#error "RR_STORE3 must be ST_F64 or ST_F32D"
#endif

#if RR_LAT3 == 3
using Lat = D3Q19;
#elif RR_LAT3 == 4
using Lat = D3Q27;
#elif RR_LAT3 == 5
using Lat = D3V39;
#elif RR_LAT3 == 6
using Lat = D3Q103;
#else
#error "RR_LAT3 must be a 3D lattice"
#endif

#if RR_AA3 == 0

template <int MODE>
hipError_t step_t(const lbm_ctx* c, const void* fin, void* fout)
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
            k_stream_collide3<Lat, MODE, POL_CACHE, Sto3><<<grid, block, 0, c->stream>>>(a);
            return hipGetLastError();
        }
        if (pol == POL_KEEP) {
            k_stream_collide3<Lat, MODE, POL_KEEP, Sto3><<<grid, block, 0, c->stream>>>(a);
            return hipGetLastError();
        }
    }
    k_stream_collide3<Lat, MODE, POL_STREAM, Sto3><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t step(const lbm_ctx* c, const void* fin, void* fout)
{
    switch (c->coll) {
    case COLL_PR: return step_t<C3_PR>(c, fin, fout);
    case COLL_BGK: return step_t<C3_BGK>(c, fin, fout);
    default: return step_t<C3_RR>(c, fin, fout);
    }
}

hipError_t init(const lbm_ctx* c, void* dst, const double* rho, const double* ux, const double* uy,
                const double* uz, const double* noise, double noise_amp, int eq_order)
{
    const Init3Args ia{ dst, c->lay, c->ny, c->nz, rho, ux, uy, uz, noise, noise_amp, eq_order };
    // the single-buffer scheme collides the initial populations in place
    if (c->aa)
        k_init3<Lat, false, Sto3><<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(ia);
    else
        k_init3<Lat, true, Sto3><<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(ia);
    return hipGetLastError();
}

hipError_t populations(const lbm_ctx* c, const void* src, double* out)
{
    const int64_t n = int64_t(c->nx) * c->ny * c->nz;
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    const auto* f = static_cast<const typename Sto3::elem*>(src);
    switch (state_placement(c)) {
    case 1: k_populations3<Lat, 1, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, out); break;
    case 2: k_populations3<Lat, 2, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, out); break;
    default: k_populations3<Lat, 0, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, out);
    }
    return hipGetLastError();
}

hipError_t moments(const lbm_ctx* c, double* r, double* ux, double* uy, double* uz, double* partial)
{
    const dim3 grid(unsigned(c->nblk)), block(256);
    const auto* f = static_cast<const typename Sto3::elem*>(c->buf[c->cur]);
    switch (state_placement(c)) {
    case 1: k_moments3<Lat, 1, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, r, ux, uy, uz, partial); break;
    case 2: k_moments3<Lat, 2, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, r, ux, uy, uz, partial); break;
    default: k_moments3<Lat, 0, Sto3><<<grid, block, 0, c->stream>>>(f, c->lay, c->ny, c->nz, r, ux, uy, uz, partial);
    }
    return hipGetLastError();
}

#else // RR_AA3 == 1 or 2

constexpr bool kNT = RR_AA3 == 2;

template <int MODE>
hipError_t step_aa_t(const lbm_ctx* c, bool shifted, bool reverse)
{
    const int rows = c->ny * c->nz;
    const int bxn = (c->nx + BX - 1) / BX, byn = (rows + BY - 1) / BY;
    Step3Args a{ c->buf[0], c->buf[0], c->lay, c->ny, c->nz, bxn, bxn * byn, c->xcd_remap, relax_of(c), c->order,
                 reverse ? 1 : 0 };
    const dim3 grid(unsigned(bxn * byn)), block(BX, BY);
    if (shifted)
        k_stream_collide3_aa<Lat, MODE, true, kNT, Sto3><<<grid, block, 0, c->stream>>>(a);
    else
        k_stream_collide3_aa<Lat, MODE, false, kNT, Sto3><<<grid, block, 0, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t step_aa_any(const lbm_ctx* c, bool shifted, bool reverse)
{
    switch (c->coll) {
    case COLL_PR: return step_aa_t<C3_PR>(c, shifted, reverse);
    case COLL_BGK: return step_aa_t<C3_BGK>(c, shifted, reverse);
    default: return step_aa_t<C3_RR>(c, shifted, reverse);
    }
}

#endif

} // namespace

#if RR_AA3 == 0

#define RR_OPS3D_NAME_(l, s) ops3d_##l##_##s
#define RR_OPS3D_NAME(l, s) RR_OPS3D_NAME_(l, s)
const Ops3D& RR_OPS3D_NAME(RR_LAT3, RR_STORE3)()
{
    static const Ops3D ops{ step, RR_STEP3_AA_NAME(RR_LAT3, RR_STORE3), init, populations, moments };
    return ops;
}

#elif RR_AA3 == 1

// The store kinds of the policies as in 2D: POL_CACHE ordinary stores,
// POL_STREAM non-temporal ones, POL_KEEP non-temporal stores in the step that
// writes a node's own slots only.  The tile order is reversed every other
// step under every policy: with non-temporal stores too, the next step's
// first reads then meet the lines written last (D3V39 FP64 128^3: 70.3% of
// peak with the reversal, 58.7% without).
hipError_t RR_STEP3_AA_NAME(RR_LAT3, RR_STORE3)(const lbm_ctx* c, bool shifted)
{
    const bool nt = c->pol == POL_STREAM || (c->pol == POL_KEEP && !shifted);
    const bool reverse = (c->steps & 1) != 0;
    return nt ? RR_STEP3_AANT_NAME(RR_LAT3, RR_STORE3)(c, shifted, reverse) : step_aa_any(c, shifted, reverse);
}

#else

hipError_t RR_STEP3_AANT_NAME(RR_LAT3, RR_STORE3)(const lbm_ctx* c, bool shifted, bool reverse)
{
    return step_aa_any(c, shifted, reverse);
}

#endif

} // namespace rr
