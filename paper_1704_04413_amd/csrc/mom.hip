// The moment representation (LBM_STORE_MOMENTS) for one 2D lattice, chosen
// at compile time (RR_LAT = LBM_D2Q9, LBM_D2V17 or LBM_D2V37): the step at
// every regularization order, the initial state, the rebuilt populations and
// the diagnostics; for D2V37 also the thermal form.
#include "context.hpp"
#include "step2d.hpp"
#include "moments.hpp"

#if !defined(RR_LAT)
#error "compile with -DRR_LAT=<2D lattice id>"
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

template <class L, int ORDER, bool TH, bool A13P>
__global__ __launch_bounds__(256) void k_mom_populations(const double* m, int64_t n, Relax rx, double* out)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double v[L::Q];
    mom_node_populations<L, ORDER, TH, A13P>(m, n, k, rx, v);
    static_for<L::Q>([&](auto I) { out[int64_t(I) * n + k] = v[I]; });
}

// rho, u (theta) and the block sums of the population form's diagnostics,
// from the populations the moments stand for.
template <class L, int ORDER, bool TH, bool A13P>
__global__ __launch_bounds__(256) void k_mom_moments(const double* m, int64_t n, Relax rx, double* rho_o,
                                                     double* ux_o, double* uy_o, double* th_o, double* partial)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        double v[L::Q];
        mom_node_populations<L, ORDER, TH, A13P>(m, n, k, rx, v);
        node_diag<L>(v, TH ? 1 : 0, k, rho_o, ux_o, uy_o, th_o, val);
    }
    block_sums<MOM_NS>(val, partial);
}

// ORDER: the regularization order of the isothermal form (the thermal form
// takes it from the relaxation factors, zero above the order).
template <int ORDER, bool TH, bool A13P>
hipError_t launch(const lbm_ctx* c, int what, const void* fin, void* fout, const InitArgs* ia, double* out,
                  double* r, double* ux, double* uy, double* th, double* partial)
{
    using L = Lat;
    const int64_t n = int64_t(c->nx) * c->ny;
    const Relax rx = relax_of(c);
    const double* m = static_cast<const double*>(c->buf[c->cur]);
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    switch (what) {
    case 0: k_mom_init<L, TH, A13P><<<grid, block, 0, c->stream>>>(*ia); break;
    case 1: k_mom_populations<L, ORDER, TH, A13P><<<grid, block, 0, c->stream>>>(m, n, rx, out); break;
    case 2:
        k_mom_moments<L, ORDER, TH, A13P>
            <<<dim3(unsigned(c->nblk)), block, 0, c->stream>>>(m, n, rx, r, ux, uy, th, partial);
        break;
    default: {
        constexpr int OX = BX - 2 * L::R;
        const int bxn = (c->nx + OX - 1) / OX, byn = (c->ny + MOM_ROWS - 1) / MOM_ROWS;
        const dim3 g(unsigned(bxn * byn)), blk(BX, MOM_ROWS);
        const double* a = static_cast<const double*>(fin);
        double* o = static_cast<double*>(fout);
        if constexpr (TH)
            k_mom_step<L, ORDER, false, true, A13P><<<g, blk, 0, c->stream>>>(a, o, c->nx, c->ny, bxn, rx);
        else if (c->tau3 == c->tau && c->tau4 == c->tau)
            k_mom_step<L, ORDER, false><<<g, blk, 0, c->stream>>>(a, o, c->nx, c->ny, bxn, rx);
        else
            k_mom_step<L, ORDER, true><<<g, blk, 0, c->stream>>>(a, o, c->nx, c->ny, bxn, rx);
    }
    }
    return hipGetLastError();
}

} // namespace

#define RR_MOM_NAME_(l) mom_launch_##l
#define RR_MOM_NAME(l) RR_MOM_NAME_(l)
hipError_t RR_MOM_NAME(RR_LAT)(const lbm_ctx* c, int what, const void* fin, void* fout, const InitArgs* ia,
                               double* out, double* r, double* ux, double* uy, double* th, double* partial)
{
    if (c->thermal) {
        // the thermal form exists for D2V37 only (lbm_init rejects the others)
        if constexpr (Lat::id == LBM_D2V37) {
            if (c->a13p) return launch<4, true, true>(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
            return launch<4, true, false>(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
        }
        return hipErrorInvalidValue;
    }
    switch (c->order) {
    case 2: return launch<2, false, false>(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    case 3: return launch<3, false, false>(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    default: return launch<4, false, false>(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    }
}

} // namespace rr
