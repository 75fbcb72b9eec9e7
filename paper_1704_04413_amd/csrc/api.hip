// librrlbm: C-ABI of the MI355X (gfx950) recursive-regularized lattice
// Boltzmann library (include/rrlbm.h): contexts, stepping, diagnostics,
// checkpoints, the 3D entry points and batches.  The kernels live in the
// units that instantiate them (step2d.hip per lattice and storage,
// step3d.hip per 3D lattice, mom.hip, batch.hip, closure.hip); this unit
// holds the host logic and the small diagnostic kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "context.hpp"
#include "lattices.hpp"
#include "lattices3d.hpp"

namespace rr {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

const Ops2D& ops2d_0_0();
const Ops2D& ops2d_0_1();
const Ops2D& ops2d_0_2();
const Ops2D& ops2d_1_0();
const Ops2D& ops2d_1_1();
const Ops2D& ops2d_1_2();
const Ops2D& ops2d_2_0();
const Ops2D& ops2d_2_1();
const Ops2D& ops2d_2_2();
const Ops2D& ops2d_0_3();
const Ops2D& ops2d_1_3();
const Ops2D& ops2d_2_3();
const Ops3D& ops3d_3_0();
const Ops3D& ops3d_4_0();
const Ops3D& ops3d_5_0();
const Ops3D& ops3d_6_0();
const Ops3D& ops3d_3_3();
const Ops3D& ops3d_4_3();
const Ops3D& ops3d_5_3();
const Ops3D& ops3d_6_3();
hipError_t mom_launch_0(const lbm_ctx*, int, const void*, void*, const InitArgs*, double*, double*, double*, double*,
                        double*, double*);
hipError_t mom_launch_1(const lbm_ctx*, int, const void*, void*, const InitArgs*, double*, double*, double*, double*,
                        double*, double*);
hipError_t mom_launch_2(const lbm_ctx*, int, const void*, void*, const InitArgs*, double*, double*, double*, double*,
                        double*, double*);
hipError_t batch_launch_0(int, const InstDesc*, const int*, int, int, int, int, int, hipStream_t);
hipError_t batch_launch_1(int, const InstDesc*, const int*, int, int, int, int, int, hipStream_t);
hipError_t batch_launch_2(int, const InstDesc*, const int*, int, int, int, int, int, hipStream_t);
hipError_t batch_launch_3(int, const InstDesc*, const int*, int, int, int, int, int, hipStream_t);

const Ops2D& ops2d(int lattice, int store)
{
    using Get = const Ops2D& (*)();
    static const Get table[3][4] = { { ops2d_0_0, ops2d_0_1, ops2d_0_2, ops2d_0_3 },
                                     { ops2d_1_0, ops2d_1_1, ops2d_1_2, ops2d_1_3 },
                                     { ops2d_2_0, ops2d_2_1, ops2d_2_2, ops2d_2_3 } };
    return table[lattice][store]();
}

const Ops3D& ops3d(int lattice, int store)
{
    const bool f32 = store == ST_F32D;
    switch (lattice) {
    case LBM_D3Q19: return f32 ? ops3d_3_3() : ops3d_3_0();
    case LBM_D3Q27: return f32 ? ops3d_4_3() : ops3d_4_0();
    case LBM_D3V39: return f32 ? ops3d_5_3() : ops3d_5_0();
    default: return f32 ? ops3d_6_3() : ops3d_6_0();
    }
}

hipError_t mom_launch_any(const lbm_ctx* c, int what, const void* fin, void* fout, const InitArgs* ia, double* out,
                          double* r, double* ux, double* uy, double* th, double* partial)
{
    switch (c->lattice) {
    case LBM_D2Q9: return mom_launch_0(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    case LBM_D2V17: return mom_launch_1(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    default: return mom_launch_2(c, what, fin, fout, ia, out, r, ux, uy, th, partial);
    }
}

hipError_t batch_launch(int store, int lattice, const InstDesc* desc, const int* begin, int n, int total, int parity,
                        int tile_x, int grid, hipStream_t st)
{
    switch (store) {
    case ST_F32: return batch_launch_1(lattice, desc, begin, n, total, parity, tile_x, grid, st);
    case ST_BF16: return batch_launch_2(lattice, desc, begin, n, total, parity, tile_x, grid, st);
    case ST_F32D: return batch_launch_3(lattice, desc, begin, n, total, parity, tile_x, grid, st);
    default: return batch_launch_0(lattice, desc, begin, n, total, parity, tile_x, grid, st);
    }
}

// Vorticity from the periodic fourth-order centred difference and block sums
// of [omega^2, omega^4].  Offsets reach +-2, so an axis shorter than 2 nodes
// wraps more than once: indices are reduced modulo the axis length.
__global__ __launch_bounds__(256) void k_vorticity(const double* ux, const double* uy, int nx, int ny,
                                                   double* vort, double* partial)
{
    const int64_t n = int64_t(nx) * ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[VORT_NS] = { 0, 0 };
    if (k < n) {
        const int x = int(k % nx), y = int(k / nx);
        auto X = [&](int d) { return ((x + d) % nx + nx) % nx; };
        auto Y = [&](int d) { return ((y + d) % ny + ny) % ny; };
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
    // block sums (256 threads)
    __shared__ double red[VORT_NS][256];
    const int t = threadIdx.x;
    for (int s = 0; s < VORT_NS; ++s) red[s][t] = val[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int s = 0; s < VORT_NS; ++s) red[s][t] += red[s][t + w];
        __syncthreads();
    }
    if (t < VORT_NS) partial[int64_t(blockIdx.x) * VORT_NS + t] = red[t][0];
}

// ---- allocation-free diagnostics (lbm_moments_noalloc)

constexpr int64_t NOALLOC_MAX_BLOCKS = LBM_NOALLOC_MAX_NODES / 256;
constexpr int64_t NOALLOC_SCRATCH = NOALLOC_MAX_BLOCKS * (MOM_NS + VORT_NS) + LBM_NSUMS;

// Per-block partial sums and the final sums of lbm_moments_noalloc.  Each GPU
// holds its own copy for the life of the process.  On the host this name is
// only a stand-in for the device array: kernels and copies get the address
// from noalloc_scratch_ptr().
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[256] = {}; // per device id
} // namespace

// Device address of `scratch` on the current device, looked up once per device.
hipError_t noalloc_scratch_ptr(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// The LBM_NSUMS totals from the per-block partial sums, on the device: one
// thread per sum, the blocks added in order with the same compensated
// (Neumaier) summation as the host path, so both give the same bits.
__global__ __launch_bounds__(64) void k_reduce_sums(const double* part, int64_t nblk, double* sums)
{
    const int s = int(threadIdx.x);
    if (s >= MOM_NS + VORT_NS) return;
    const double* base = s < MOM_NS ? part + s : part + MOM_NS * nblk + (s - MOM_NS);
    const int stride = s < MOM_NS ? MOM_NS : VORT_NS;
    const int slot = s < MOM_NS ? (s < 6 ? s : s + 2) : 6 + (s - MOM_NS); // [0..5, 8, 9] then [6, 7]
    double acc = 0.0, comp = 0.0;
    for (int64_t i = 0; i < nblk; ++i) {
        const double v = base[i * stride];
        const double t = acc + v;
        comp += (fabs(acc) >= fabs(v)) ? (acc - t) + v : (v - t) + acc;
        acc = t;
    }
    sums[slot] = acc + comp;
}

} // namespace rr

using namespace rr;

namespace {

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

// Cache policy from the bytes of one state buffer (see Policy), measured on
// the step at 768^2, 1024^2 and 1536^2 for every lattice and storage:
// POL_CACHE wins up to 128 MiB (by up to 20 points of HBM peak), POL_KEEP from
// 256 to 320 MiB (D2V37 FP64 1024^2, 310 MB: 75.7% against 71.5%), POL_STREAM
// elsewhere.  The in-place (AA) step takes POL_CACHE at every size: its
// ordinary stores beat non-temporal ones on every lattice and storage
// measured from 166 MiB to 1.2 GB (D2V37 FP64 2048^2: 68.2% against 57.4%;
// D2V17 FP64 2048^2: 78.2 against 58.5%) but one (D2V37 FP64 1024^2: 80.7
// against 81.8%).  The in-place 3D step takes POL_STREAM for buffers above
// 512 MiB up to 2 GiB and POL_CACHE otherwise, the band where its
// non-temporal stores measured faster: at 128^3 they won on D3V39 FP64
// (624 MiB: 70.3% against 68.0%) and D3Q103 (FP64, 1648 MiB: 61.4 against
// 58.5%; FP32, 824 MiB: 57.7-59.4 against 57.5%) and lost on D3Q27 FP64
// (432 MiB: 75.6 against 76.6%) and D3V39 FP32 (312 MiB: 70.1 against
// 78.5%); at 256^3 they lost on every buffer measured (D3Q19 FP64, 2.4 GiB:
// 64.3 against 64.8%; D3Q27, 3.4 GiB: 60.7 against 63.1%; D3V39, 4.9 GiB:
// 58.5 against 59.3%).  RRLBM_CACHE_POLICY=0/1/2 forces one.
int choose_policy(int64_t buffer_bytes, bool aa = false, bool three_d = false)
{
    if (const char* e = std::getenv("RRLBM_CACHE_POLICY")) {
        const int p = std::atoi(e);
        if (p >= POL_STREAM && p <= POL_KEEP) return p;
    }
    const int64_t MiB = int64_t(1) << 20;
    if (aa) return (three_d && buffer_bytes > 512 * MiB && buffer_bytes <= 2048 * MiB) ? POL_STREAM : POL_CACHE;
    if (buffer_bytes <= 128 * MiB) return POL_CACHE;
    if (buffer_bytes > 256 * MiB && buffer_bytes <= 320 * MiB) return POL_KEEP;
    return POL_STREAM;
}

hipError_t launch_step(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    if (c->dim == 3) {
        if (!pull) return hipErrorInvalidValue; // 3D contexts are only ever stepped with a pull
        return ops3d(c->lattice, c->store).step(c, fin, fout);
    }
    if (c->store == ST_MOM) return mom_launch_any(c, 3, fin, fout);
    return ops2d(c->lattice, c->store).step(c, fin, fout, pull);
}

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
                           LBM_COLL_BGK | LBM_EQ_INIT_ORDER2 | LBM_A13_PROJECTED | LBM_MATH_FP64 |
                           LBM_SCHEME_AA;
    if (flags & ~known) return fail(LBM_EINVAL, "unknown flag bits");
    if ((flags & LBM_MATH_FP64) && !(flags & LBM_STORE_FP32))
        return fail(LBM_EINVAL, "LBM_MATH_FP64 goes with LBM_STORE_FP32");
    const uint32_t stores = flags & (LBM_STORE_FP32 | LBM_STORE_BF16 | LBM_STORE_MOMENTS);
    if (stores & (stores - 1)) return fail(LBM_EINVAL, "two storage flags");
    if ((flags & LBM_STORE_MOMENTS) && (flags & (LBM_COLL_PR | LBM_COLL_BGK)))
        return fail(LBM_EINVAL, "the moment representation is recursive regularization only");
    if ((flags & LBM_COLL_PR) && (flags & LBM_COLL_BGK)) return fail(LBM_EINVAL, "two collision flags");
    if ((flags & LBM_SCHEME_AA) && (flags & LBM_STORE_MOMENTS))
        return fail(LBM_EINVAL, "LBM_SCHEME_AA goes with population storage");
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

// Bytes of one state buffer.
int64_t store_bytes(const lbm_ctx* c)
{
    if (c->store == ST_MOM) return int64_t(sizeof(double)) * (c->thermal ? MOM_KT : MOM_K) * c->nx * c->ny;
    const int64_t esz = (c->store == ST_F32 || c->store == ST_F32D) ? 4 : c->store == ST_BF16 ? 2 : 8;
    return esz * layout_elems(c->q, c->nx, c->ny * c->nz);
}

// Fields, vorticity (when `vort_too`) and the per-block sums of a 2D context:
// MOM_NS sums of nblk blocks, then VORT_NS sums of nblk blocks, in `partial`.
hipError_t moments_launch(const lbm_ctx* c, double* r, double* vx, double* vy, double* th, bool vort_too,
                          double* vort, double* partial)
{
    hipError_t he = c->store == ST_MOM ? mom_launch_any(c, 2, nullptr, nullptr, nullptr, nullptr, r, vx, vy, th, partial)
                                       : ops2d(c->lattice, c->store).moments(c, r, vx, vy, th, partial);
    if (he != hipSuccess || !vort_too) return he;
    k_vorticity<<<dim3(unsigned(c->nblk)), dim3(256), 0, c->stream>>>(vx, vy, c->nx, c->ny, vort,
                                                                      partial + MOM_NS * c->nblk);
    return hipGetLastError();
}

// The LBM_NSUMS totals from the per-block partial sums (host, compensated).
void reduce_sums(const double* part, int64_t nblk, double* sums)
{
    const double* pv = part + MOM_NS * nblk;
    static const int slot[MOM_NS] = { 0, 1, 2, 3, 4, 5, 8, 9 };
    for (int s = 0; s < MOM_NS; ++s) sums[slot[s]] = neumaier(part + s, nblk, MOM_NS);
    sums[6] = neumaier(pv, nblk, VORT_NS);
    sums[7] = neumaier(pv + 1, nblk, VORT_NS);
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
    if (flags & LBM_STORE_MOMENTS) return int64_t((flags & LBM_THERMAL) ? MOM_KT : MOM_K) * nx * ny;
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
    if (flags & LBM_SCHEME_AA) {
        if (!f_a || f_b) return fail(LBM_EINVAL, "LBM_SCHEME_AA takes f_a and a NULL f_b");
    } else if (!f_a || !f_b || f_a == f_b) {
        return fail(LBM_EINVAL, "two distinct population buffers are needed");
    }
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
    c->store = (flags & LBM_STORE_FP32)      ? ((flags & LBM_MATH_FP64) ? ST_F32D : ST_F32)
               : (flags & LBM_STORE_BF16)    ? ST_BF16
               : (flags & LBM_STORE_MOMENTS) ? ST_MOM
                                             : ST_F64;
    c->coll = (flags & LBM_COLL_PR) ? COLL_PR : (flags & LBM_COLL_BGK) ? COLL_BGK : COLL_RR;
    c->thermal = (flags & LBM_THERMAL) != 0;
    c->a13p = (flags & LBM_A13_PROJECTED) != 0;
    c->aa = (flags & LBM_SCHEME_AA) != 0;
    c->q = li.q;
    c->lay = make_layout(li.q, nx, ny);
    c->pol = choose_policy(store_bytes(c), c->aa);
    // tuning knob: RRLBM_XCD_REMAP=0 keeps the hardware's round-robin block order
    if (const char* e = std::getenv("RRLBM_XCD_REMAP")) c->xcd_remap = std::atoi(e) != 0;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->stream = static_cast<hipStream_t>(stream);
    const int64_t n = int64_t(nx) * ny;
    c->nblk = (n + 255) / 256;

    hipError_t he = noalloc_scratch_ptr(&c->noalloc_scratch);
    if (he != hipSuccess) {
        delete c;
        return fail(LBM_EDEVICE, std::string("allocation-free scratch lookup: ") + hipGetErrorString(he));
    }
    const int eq_order = (flags & LBM_EQ_INIT_ORDER2) ? 2 : li.n_eq;
    if (c->store == ST_MOM) {
        const InitArgs ia{ f_a, c->lay, rho, ux, uy, theta, grad, noise, noise_amp, eq_order, tau };
        he = mom_launch_any(c, 0, nullptr, nullptr, &ia); // the moments are the state: no collision here
    } else if (c->aa) {
        // f^(0) [+ f^(1)] + noise into f_a, collided in place into the
        // placement of an even step count
        const InitArgs ia{ f_a, c->lay, rho, ux, uy, theta, grad, noise, noise_amp, eq_order, tau };
        he = ops2d(c->lattice, c->store).init(c, ia);
        if (he == hipSuccess) he = ops2d(c->lattice, c->store).step_aa(c, false, 0u);
    } else {
        // f^(0) [+ f^(1)] + noise into f_b, collided node by node into f_a: post-collision state, cur = 0
        const InitArgs ia{ f_b, c->lay, rho, ux, uy, theta, grad, noise, noise_amp, eq_order, tau };
        he = ops2d(c->lattice, c->store).init(c, ia);
        if (he == hipSuccess) he = launch_step(c, f_b, f_a, false);
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
        hipError_t he;
        if (c->aa && c->dim == 3) {
            he = ops3d(c->lattice, c->store).step_aa(c, (c->steps & 1) == 0);
        } else if (c->aa) {
            he = ops2d(c->lattice, c->store).step_aa(c, (c->steps & 1) == 0, uint32_t(c->steps + 1));
        } else {
            he = launch_step(c, c->buf[c->cur], c->buf[1 - c->cur], true);
            c->cur = 1 - c->cur;
        }
        if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(he));
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
    HIP_TRY(moments_launch(c, r, vx, vy, th, vort || sums, vort, c->partial));
    if (sums) {
        HIP_TRY(hipMemcpyAsync(c->partial_host, c->partial, sizeof(double) * (MOM_NS + VORT_NS) * c->nblk,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        reduce_sums(c->partial_host, c->nblk, sums);
    }
    return LBM_OK;
}

int lbm_moments_noalloc(lbm_ctx* c, double* rho, double* ux, double* uy, double* theta, double* vort, double* sums)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->dim == 3) return fail(LBM_EINVAL, "3D context: use lbm_moments_3d");
    if ((vort || sums) && (!ux || !uy))
        return fail(LBM_EINVAL, "ux and uy are required when vort or sums is requested");
    if (c->nblk > NOALLOC_MAX_BLOCKS)
        return fail(LBM_EINVAL, "grid of " + std::to_string(int64_t(c->nx) * c->ny) +
                                    " nodes exceeds the allocation-free limit of " +
                                    std::to_string(int64_t(LBM_NOALLOC_MAX_NODES)) + " nodes");
    if (!c->noalloc_scratch) return fail(LBM_EDEVICE, "no allocation-free scratch for this context");
    double* part = c->noalloc_scratch;
    HIP_TRY(moments_launch(c, rho, ux, uy, theta, vort || sums, vort, part));
    if (sums) {
        double* dsums = part + NOALLOC_MAX_BLOCKS * (MOM_NS + VORT_NS);
        k_reduce_sums<<<dim3(1), dim3(64), 0, c->stream>>>(part, c->nblk, dsums);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(sums, dsums, sizeof(double) * LBM_NSUMS, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

int lbm_populations(lbm_ctx* c, double* f_out)
{
    if (!c || !f_out) return fail(LBM_EINVAL, "ctx or f_out is NULL");
    if (c->dim == 3)
        HIP_TRY(ops3d(c->lattice, c->store).populations(c, c->buf[c->cur], f_out));
    else if (c->store == ST_MOM)
        HIP_TRY(mom_launch_any(c, 1, nullptr, nullptr, nullptr, f_out));
    else
        HIP_TRY(ops2d(c->lattice, c->store).populations(c, c->buf[c->cur], f_out));
    return LBM_OK;
}

// Checkpoint layout: a 64-byte header, then the current state buffer as it
// sits in device memory (storage type, library layout).
struct CkptHeader {
    char magic[8];          // "RRLBMCK1"
    int32_t lattice, nx, ny, nz;
    uint32_t flags;
    int32_t reserved;
    int64_t steps;
    double tau, tau3, tau4;
};
static_assert(sizeof(CkptHeader) == LBM_CHECKPOINT_HEADER_BYTES, "checkpoint header size");

int64_t lbm_checkpoint_bytes(const lbm_ctx* c)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    return int64_t(sizeof(CkptHeader)) + store_bytes(c);
}

int lbm_save(lbm_ctx* c, void* dst, int64_t dst_bytes)
{
    if (!c || !dst) return fail(LBM_EINVAL, "ctx or dst is NULL");
    const int64_t need = int64_t(sizeof(CkptHeader)) + store_bytes(c);
    if (dst_bytes < need) return fail(LBM_EINVAL, "dst holds " + std::to_string(dst_bytes) + " bytes, the checkpoint needs " + std::to_string(need));
    CkptHeader h{};
    std::memcpy(h.magic, "RRLBMCK1", 8);
    h.lattice = c->lattice;
    h.nx = c->nx;
    h.ny = c->ny;
    h.nz = c->nz;
    h.flags = c->flags;
    h.steps = c->steps;
    h.tau = c->tau;
    h.tau3 = c->tau3;
    h.tau4 = c->tau4;
    char* d = static_cast<char*>(dst);
    HIP_TRY(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyDefault, c->stream));
    HIP_TRY(hipMemcpyAsync(d + sizeof(h), c->buf[c->cur], size_t(store_bytes(c)), hipMemcpyDefault, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_load(lbm_ctx* c, const void* src, int64_t src_bytes)
{
    if (!c || !src) return fail(LBM_EINVAL, "ctx or src is NULL");
    const int64_t need = int64_t(sizeof(CkptHeader)) + store_bytes(c);
    if (src_bytes < need) return fail(LBM_EINVAL, "src holds " + std::to_string(src_bytes) + " bytes, the checkpoint needs " + std::to_string(need));
    CkptHeader h{};
    const char* s = static_cast<const char*>(src);
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(&h, s, sizeof(h), hipMemcpyDefault));
    if (std::memcmp(h.magic, "RRLBMCK1", 8) != 0) return fail(LBM_EINVAL, "not a checkpoint of this library");
    if (h.lattice != c->lattice || h.nx != c->nx || h.ny != c->ny || h.nz != c->nz || h.flags != c->flags ||
        h.tau != c->tau)
        return fail(LBM_EINVAL, "the checkpoint was written by a context with other lbm_init arguments");
    if (h.steps < 0 || !(h.tau3 > 0.5) || !(h.tau4 > 0.5)) return fail(LBM_EINVAL, "corrupt checkpoint header");
    HIP_TRY(hipMemcpyAsync(c->buf[0], s + sizeof(h), size_t(store_bytes(c)), hipMemcpyDefault, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->steps = h.steps;
    c->tau3 = h.tau3;
    c->tau4 = h.tau4;
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
    if (flags & (LBM_STORE_BF16 | LBM_STORE_MOMENTS))
        return fail(LBM_EINVAL, "3D lattices store FP64 populations, or FP32 with LBM_MATH_FP64");
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
    const uint32_t known =
        LBM_COLL_PR | LBM_COLL_BGK | LBM_EQ_INIT_ORDER2 | LBM_SCHEME_AA | LBM_STORE_FP32 | LBM_MATH_FP64;
    if (flags & ~known)
        return fail(LBM_EINVAL, "3D lattices take LBM_COLL_PR, LBM_COLL_BGK, LBM_EQ_INIT_ORDER2, LBM_SCHEME_AA and "
                                "LBM_STORE_FP32 | LBM_MATH_FP64 only");
    if (bool(flags & LBM_STORE_FP32) != bool(flags & LBM_MATH_FP64))
        return fail(LBM_EINVAL, "3D FP32 storage computes in double: LBM_STORE_FP32 goes with LBM_MATH_FP64");
    if ((flags & LBM_COLL_PR) && (flags & LBM_COLL_BGK)) return fail(LBM_EINVAL, "two collision flags");
    if (!(flags & LBM_COLL_BGK) && (reg_order < 2 || reg_order > li.n_eq))
        return fail(LBM_EINVAL, "regularization order must be in [2, " + std::to_string(li.n_eq) + "]");
    if (flags & LBM_SCHEME_AA) {
        if (!f_a || f_b) return fail(LBM_EINVAL, "LBM_SCHEME_AA takes f_a and a NULL f_b");
    } else if (!f_a || !f_b || f_a == f_b) {
        return fail(LBM_EINVAL, "two distinct population buffers are needed");
    }
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
    c->store = (flags & LBM_STORE_FP32) ? ST_F32D : ST_F64;
    c->coll = (flags & LBM_COLL_PR) ? COLL_PR : (flags & LBM_COLL_BGK) ? COLL_BGK : COLL_RR;
    c->aa = (flags & LBM_SCHEME_AA) != 0;
    c->q = li.q;
    c->lay = make_layout(li.q, nx, ny * nz);
    c->pol = choose_policy(store_bytes(c), c->aa, true);
    if (const char* e = std::getenv("RRLBM_XCD_REMAP")) c->xcd_remap = std::atoi(e) != 0;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->stream = static_cast<hipStream_t>(stream);
    const int64_t n = int64_t(nx) * ny * nz;
    c->nblk = (n + 255) / 256;
    const int eq_order = (flags & LBM_EQ_INIT_ORDER2) ? 2 : li.n_eq;
    hipError_t he;
    if (c->aa) {
        // f^(0) into f_a, collided in place into the placement of an even step count
        he = ops3d(lattice, c->store).init(c, f_a, rho, ux, uy, uz, noise, noise_amp, eq_order);
        if (he == hipSuccess) he = ops3d(lattice, c->store).step_aa(c, false);
    } else {
        // f^(0) goes to f_b shifted by -c_i; one pull launch then collides it into f_a
        he = ops3d(lattice, c->store).init(c, f_b, rho, ux, uy, uz, noise, noise_amp, eq_order);
        if (he == hipSuccess) he = launch_step(c, f_b, f_a, true); // post-collision state in f_a, cur = 0
    }
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
    HIP_TRY(ops3d(c->lattice, c->store).moments(c, r, vx, vy, vz, c->partial));
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

// By default one persistent kernel walks a single mixed work list and
// switches on each tile's lattice.  RRLBM_BATCH_SPLIT=1 groups the members by
// lattice instead: desc[] lists them lattice by lattice, each lattice has its
// own work list (begin offsets) and its own kernel compiled for that lattice
// alone (so D2Q9 tiles do not run with the register budget D2V37 needs), and
// the lattices' launches are independent branches of the graph;
// RRLBM_BATCH_SPLIT=2 keeps the grouping but records the launches one after
// another.  The three forms gave the same throughput within 3%.
struct lbm_batch {
    std::vector<lbm_ctx*> members;
    std::vector<int> order;       // desc[k] describes members[order[k]]
    std::vector<InstDesc> desc;
    std::vector<int> begin;       // per group: count + 1 offsets
    struct Group {
        int lattice;              // -1: mixed list
        int first, n;             // desc[first .. first + n)
        int begin_off, total;     // begin[begin_off ..], work items
    };
    std::vector<Group> groups;
    bool split = false;    // one work list and kernel per lattice
    bool branches = false; // the groups' launches as independent graph branches
    int store = ST_F64;
    hipStream_t stream = nullptr;        // members' stream: every replay goes there
    hipStream_t capture[3] = {};         // private streams used only to record the graph
    hipEvent_t fork = nullptr, join[2] = {};
    InstDesc* d_desc = nullptr;
    int* d_begin = nullptr;
    int tile_x = 64, bpc = 4, num_cu = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

hipError_t launch_group(const lbm_batch* b, const lbm_batch::Group& g, hipStream_t st, int parity)
{
    const int grid = std::min(g.total, b->num_cu * b->bpc);
    return batch_launch(b->store, g.lattice, b->d_desc + g.first, b->d_begin + g.begin_off, g.n, g.total, parity,
                        b->tile_x, grid, st);
}

hipError_t launch_batch_any(const lbm_batch* b, hipStream_t st, int parity)
{
    for (const auto& g : b->groups) {
        const hipError_t e = launch_group(b, g, st, parity);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void batch_release_graph(lbm_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Records the two-step graph: each group's parity-0 and parity-1 launches in
// a branch of its own (a capture stream per group, forked from and joined to
// the first), then the BF16 key advance.
hipError_t batch_capture(lbm_batch* b)
{
    const int ng = b->branches ? int(b->groups.size()) : 1;
    hipStream_t c0 = b->capture[0];
    hipError_t e = hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipEventRecord(b->fork, c0);
    for (int g = 1; g < ng && le == hipSuccess; ++g) le = hipStreamWaitEvent(b->capture[g], b->fork, 0);
    for (int g = 0; g < int(b->groups.size()) && le == hipSuccess; ++g) {
        hipStream_t st = b->capture[b->branches ? g : 0];
        le = launch_group(b, b->groups[g], st, 0);
        if (le == hipSuccess) le = launch_group(b, b->groups[g], st, 1);
    }
    for (int g = 1; g < ng && le == hipSuccess; ++g) {
        le = hipEventRecord(b->join[g - 1], b->capture[g]);
        if (le == hipSuccess) le = hipStreamWaitEvent(c0, b->join[g - 1], 0);
    }
    if (le == hipSuccess && b->store == ST_BF16) {
        const int n = int(b->desc.size());
        k_batch_advance<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, c0>>>(b->d_desc, n);
        le = hipGetLastError();
    }
    const hipError_t ec = hipStreamEndCapture(c0, &b->graph);
    return le != hipSuccess ? le : ec;
}

// Rebuilds the work lists for the current tile width, uploads them with every
// member's buffer parity, and records the two-step graph.
int batch_prepare(lbm_batch* b)
{
    const int n = int(b->members.size());
    b->order.clear();
    b->groups.clear();
    const int lats[3] = { LBM_D2Q9, LBM_D2V17, LBM_D2V37 };
    for (int li = 0; li < (b->split ? 3 : 1); ++li) {
        lbm_batch::Group g{ b->split ? lats[li] : -1, int(b->order.size()), 0, 0, 0 };
        for (int i = 0; i < n; ++i)
            if (!b->split || b->members[i]->lattice == lats[li]) b->order.push_back(i);
        g.n = int(b->order.size()) - g.first;
        if (g.n > 0) b->groups.push_back(g);
    }
    b->desc.resize(n);
    b->begin.clear();
    for (auto& g : b->groups) {
        g.begin_off = int(b->begin.size());
        int64_t total = 0;
        for (int k = g.first; k < g.first + g.n; ++k) {
            const lbm_ctx* c = b->members[b->order[k]];
            InstDesc& d = b->desc[k];
            d.buf[0] = c->buf[0];
            d.buf[1] = c->buf[1];
            d.lay = c->lay;
            d.lattice = c->lattice;
            d.bx_blocks = (c->nx + b->tile_x - 1) / b->tile_x;
            d.flip = c->cur;
            d.rx = relax_of(c);
            d.seq = uint32_t(c->steps + 1);
            b->begin.push_back(int(total));
            const int rows = b->tile_x >= batch_wide_tile ? 1 : BY; // item height
            total += int64_t(d.bx_blocks) * ((c->ny + rows - 1) / rows);
        }
        if (total >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "batch work list too long");
        b->begin.push_back(int(total));
        g.total = int(total);
    }
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_begin, b->begin.data(), sizeof(int) * b->begin.size(), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    batch_release_graph(b);
    const hipError_t e = batch_capture(b);
    if (e != hipSuccess) {
        batch_release_graph(b);
        return fail(LBM_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
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
    for (size_t k = 0; k < b->desc.size(); ++k) {
        InstDesc& d = b->desc[k];
        const lbm_ctx* c = b->members[b->order[k]];
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
    if (tile_x != 64 && tile_x != 128 && tile_x != 256 && tile_x != 512 && tile_x != 1024)
        return fail(LBM_EINVAL, "tile_x must be 64, 128, 256, 512 or 1024");
    if (blocks_per_cu < 1 || blocks_per_cu > 16) return fail(LBM_EINVAL, "blocks_per_cu must be in [1, 16]");
    for (int i = 0; i < n; ++i) {
        const lbm_ctx* c = ctxs[i];
        if (!c) return fail(LBM_EINVAL, "NULL member");
        if (c->dim == 3) return fail(LBM_EINVAL, "batch members must be 2D");
        if (c->coll != COLL_RR || c->thermal)
            return fail(LBM_EINVAL, "batch members must use the isothermal recursive regularization");
        if (c->store == ST_MOM) return fail(LBM_EINVAL, "batch members must store populations");
        if (c->aa) return fail(LBM_EINVAL, "batch members must use the two-buffer scheme");
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
    if (const char* sp = std::getenv("RRLBM_BATCH_SPLIT")) {
        b->split = std::atoi(sp) != 0;
        b->branches = std::atoi(sp) == 1;
    }
    if (!e) {
        bool ok = true;
        for (auto& cs : b->capture) ok = ok && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
        for (auto& ev : b->join) ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        // at most 3 groups: n + 3 begin offsets
        ok = ok && hipMalloc(&b->d_desc, sizeof(InstDesc) * n) == hipSuccess &&
             hipMalloc(&b->d_begin, sizeof(int) * (n + 3)) == hipSuccess;
        if (!ok) e = fail(LBM_EDEVICE, "batch device allocation failed");
    }
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
    static const int tiles[5] = { 64, 128, 256, 512, 1024 };
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
    (void)hipStreamSynchronize(b->stream);
    batch_release_graph(b);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_begin) (void)hipFree(b->d_begin);
    for (auto cs : b->capture)
        if (cs) (void)hipStreamDestroy(cs);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (auto ev : b->join)
        if (ev) (void)hipEventDestroy(ev);
    delete b;
}

} // extern "C"
