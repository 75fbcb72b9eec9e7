// Host-side state of the library: the context behind lbm_ctx, error
// reporting, and the launch entry points each translation unit provides
// (2D steps per lattice and storage, 3D steps per lattice, the moment
// representation, batches, the learned closure).  The kernels are
// instantiated in those units; this header defines none.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "common.hpp"
#include "rrlbm.h"

namespace rr {

// Population storage kinds (ST_F32D: FP32 storage with FP64 arithmetic) and
// the moment representation.
enum StoreKind { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F32D = 3, ST_MOM = 4 };

struct MlpInfer; // matrix-core weight fragments of the closure network

} // namespace rr

struct lbm_ctx {
    int lattice = 0, nx = 0, ny = 0, order = 2;
    int nz = 1, dim = 2; // 3D lattices: rows r = z * ny + y of the layout
    double tau = 1.0, tau3 = 1.0, tau4 = 1.0; // tau_2 = tau; ranks 3, 4 (lbm_set_relaxation)
    uint32_t flags = 0;
    int store = rr::ST_F64, coll = rr::COLL_RR;
    bool thermal = false, a13p = false;
    bool aa = false; // LBM_SCHEME_AA: the state lives in buf[0] alone, cur stays 0
    int q = 0;
    rr::Layout lay{};
    int xcd_remap = 1;
    int pol = rr::POL_STREAM; // cache policy of the step (from the buffer size at init; 3D: RR and BGK)
    void* buf[2] = { nullptr, nullptr };
    int cur = 0;
    int64_t steps = 0;
    hipStream_t stream = nullptr;
    // moments scratch
    double* fields = nullptr; // 5 fields of nx*ny
    double* partial = nullptr;
    double* partial_host = nullptr;
    int64_t nblk = 0;
    double* noalloc_scratch = nullptr; // this GPU's allocation-free scratch (lbm_moments_noalloc)
    // learned closure (isothermal D2V37 only)
    bool closure = false;
    rr::MlpInfer* cl_frags = nullptr;
    float* cl_norm = nullptr;
    unsigned long long* cl_fallbacks = nullptr;
};

namespace rr {

// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return rr::fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline Relax relax_of(const lbm_ctx* c)
{
    return Relax{ 1.0 - 1.0 / c->tau, c->order >= 3 ? 1.0 - 1.0 / c->tau3 : 0.0,
                  c->order >= 4 ? 1.0 - 1.0 / c->tau4 : 0.0, 1.0 / c->tau };
}

// Launch arguments of one 2D step (pull) or of the local collision of the
// initial state (!pull: no gather, sequence number 0).
inline StepArgs step_args(const lbm_ctx* c, const void* fin, void* fout, bool pull)
{
    const int bxn = (c->nx + BX - 1) / BX, byn = (c->ny + BY - 1) / BY;
    return StepArgs{ fin, fout, c->lay, bxn, bxn * byn, c->xcd_remap, relax_of(c),
                     pull ? uint32_t(c->steps + 1) : 0u,
                     (c->pol == POL_CACHE && pull && (c->steps & 1)) ? 1 : 0 };
}

// Where the current state sits (RD of state_index): 0 two-buffer; with the
// single buffer 1 after an even number of steps, 2 after an odd number.
inline int state_placement(const lbm_ctx* c) { return !c->aa ? 0 : (c->steps & 1) ? 2 : 1; }

// Batch work items at least this wide are one row high (walked by 256-wide
// blocks); narrower ones are four rows high (64 x 4 blocks).
constexpr int batch_wide_tile = 256;

// One 2D (lattice, storage) pair: the kernels of step2d.hip compiled for it.
struct Ops2D {
    // one step fin -> fout (pull), or the local collision of the initial state
    hipError_t (*step)(const lbm_ctx* c, const void* fin, void* fout, bool pull);
    // one in-place step of the single-buffer scheme on buf[0] (shifted: the
    // placement after an even number of steps), the state written keyed `seq`
    hipError_t (*step_aa)(const lbm_ctx* c, bool shifted, uint32_t seq);
    hipError_t (*init)(const lbm_ctx* c, const InitArgs& a);
    hipError_t (*populations)(const lbm_ctx* c, const void* src, double* out);
    // fields (any may be NULL) and per-block sums into `partial` (nblk blocks of MOM_NS)
    hipError_t (*moments)(const lbm_ctx* c, double* r, double* ux, double* uy, double* th, double* partial);
};
// lattice LBM_D2Q9..LBM_D2V37, store ST_F64..ST_F32D
const Ops2D& ops2d(int lattice, int store);

// One 3D (lattice, storage) pair: the kernels of step3d.hip compiled for it
// (storage ST_F64 or ST_F32D).
struct Ops3D {
    hipError_t (*step)(const lbm_ctx* c, const void* fin, void* fout);
    // one in-place step of the single-buffer scheme on buf[0] (shifted: the
    // placement after an even number of steps, or the initial collision when not)
    hipError_t (*step_aa)(const lbm_ctx* c, bool shifted);
    // the initial populations into dst: shifted for the first pull, or in
    // place for the single-buffer scheme
    hipError_t (*init)(const lbm_ctx* c, void* dst, const double* rho, const double* ux, const double* uy,
                       const double* uz, const double* noise, double noise_amp, int eq_order);
    hipError_t (*populations)(const lbm_ctx* c, const void* src, double* out);
    hipError_t (*moments)(const lbm_ctx* c, double* r, double* ux, double* uy, double* uz, double* partial);
};
const Ops3D& ops3d(int lattice, int store);

// Moment representation (mom.hip).  what: 0 initial state (ia), 1 populations
// (out), 2 diagnostics (r, ux, uy, th; sums into partial), 3 step (fin -> fout).
hipError_t mom_launch_any(const lbm_ctx* c, int what, const void* fin = nullptr, void* fout = nullptr,
                          const InitArgs* ia = nullptr, double* out = nullptr, double* r = nullptr,
                          double* ux = nullptr, double* uy = nullptr, double* th = nullptr,
                          double* partial = nullptr);

// Persistent batch launch for one storage kind (batch.hip) over a work list
// whose members all have `lattice` (or mix lattices: -1).
hipError_t batch_launch(int store, int lattice, const InstDesc* desc, const int* begin, int n, int total, int parity,
                        int tile_x, int grid, hipStream_t st);

// Fused closure step of an isothermal RR D2V37 context (closure.hip).
hipError_t closure_step(const lbm_ctx* c, const void* fin, void* fout);

} // namespace rr
