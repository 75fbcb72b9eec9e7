// The learned closure (not part of the paper's method): the fused closure
// step for every storage kind, the network's training kernels and their
// C-ABI entry points (lbm_closure_*, lbm_mlp_*).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "context.hpp"
#include "step2d.hpp"
#include "closure.hpp"

using namespace rr;

namespace rr {

namespace {

template <class S>
void closure_launch(const lbm_ctx* c, const StepArgs& a, const ClosureArgs& ca)
{
    const dim3 grid(unsigned(a.nblocks)), block(BX, BY);
    switch (c->pol) {
    case POL_CACHE: k_stream_collide_closure<S, POL_CACHE><<<grid, block, 0, c->stream>>>(a, ca); break;
    case POL_KEEP: k_stream_collide_closure<S, POL_KEEP><<<grid, block, 0, c->stream>>>(a, ca); break;
    default: k_stream_collide_closure<S, POL_STREAM><<<grid, block, 0, c->stream>>>(a, ca); break;
    }
}

} // namespace

hipError_t closure_step(const lbm_ctx* c, const void* fin, void* fout)
{
    const StepArgs a = step_args(c, fin, fout, true);
    const ClosureArgs ca{ c->cl_frags, c->cl_norm, 1.0 - 0.5 / c->tau, c->cl_fallbacks };
    switch (c->store) {
    case ST_F32: closure_launch<StoreF32>(c, a, ca); break;
    case ST_BF16: closure_launch<StoreBF16>(c, a, ca); break;
    default: closure_launch<StoreF64>(c, a, ca); break;
    }
    return hipGetLastError();
}

} // namespace rr

struct lbm_mlp {
    float* theta = nullptr; // caller-owned
    hipStream_t stream = nullptr;
    int64_t max_batch = 0;
    int nblocks = 0;
    int t = 0; // Adam steps taken
    float *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr, *loss = nullptr;
    MlpInfer* fi = nullptr;
    MlpBack* fb = nullptr;
    std::vector<float> loss_host;
};

namespace {

template <class L, class S>
struct SampleOp {
    static hipError_t run(const lbm_ctx* c, int factor, double sf, float* x, float* r)
    {
        const int64_t nc = int64_t(c->nx / factor) * (c->ny / factor);
        k_closure_samples<S><<<dim3(unsigned((nc + 255) / 256)), dim3(256), 0, c->stream>>>(
            c->buf[c->cur], c->lay, factor, sf, x, r);
        return hipGetLastError();
    }
};

hipError_t launch_frags(const float* theta, MlpInfer* fi, MlpBack* fb, hipStream_t st)
{
    k_mlp_frags<<<dim3(12), dim3(256), 0, st>>>(theta, fi, fb); // 44 * 64 + 144 threads
    return hipGetLastError();
}

} // namespace

extern "C" {

int lbm_closure_samples(lbm_ctx* c, int factor, float* x, float* r)
{
    if (!c || !x || !r) return fail(LBM_EINVAL, "ctx, x or r is NULL");
    if (c->lattice != LBM_D2V37 || c->coll != COLL_RR || c->thermal || c->store == ST_MOM || c->store == ST_F32D ||
        c->aa)
        return fail(LBM_EINVAL, "closure samples need an isothermal RR D2V37 context storing FP64, FP32 or BF16 populations in two buffers");
    if (factor < 1 || factor > 8 || c->nx % factor || c->ny % factor)
        return fail(LBM_EINVAL, "factor must be in [1, 8] and divide nx and ny");
    const double sf = (1.0 - 0.5 / c->tau) / (1.0 - 1.0 / c->tau);
    if (!std::isfinite(sf)) return fail(LBM_ETAU, "fine tau must differ from 1");
    // fine D2V37 is the only lattice: dispatch on the storage type alone
    hipError_t he = hipSuccess;
    switch (c->store) {
    case ST_F32: he = SampleOp<D2V37, StoreF32>::run(c, factor, sf, x, r); break;
    case ST_BF16: he = SampleOp<D2V37, StoreBF16>::run(c, factor, sf, x, r); break;
    default: he = SampleOp<D2V37, StoreF64>::run(c, factor, sf, x, r); break;
    }
    if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("samples launch: ") + hipGetErrorString(he));
    return LBM_OK;
}

int lbm_mlp_stats(const float* x, const float* r, int64_t n, float* norm, void* stream)
{
    if (!x || !r || !norm || n < 1) return fail(LBM_EINVAL, "x, r, norm or n invalid");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = int(std::min<int64_t>(256, (n + 255) / 256));
    double* part = nullptr;
    HIP_TRY(hipMalloc(&part, sizeof(double) * 4 * STAT_COLS * nb));
    k_col_stats<<<dim3(nb), dim3(256), 0, st>>>(x, r, n, part);
    hipError_t he = hipGetLastError();
    std::vector<double> hp(size_t(4 * STAT_COLS * nb));
    if (he == hipSuccess) he = hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (he != hipSuccess) return fail(LBM_EDEVICE, std::string("stats: ") + hipGetErrorString(he));
    std::vector<float> nv(NORM_N, 0.0f);
    for (int i = 0; i < 8; ++i) {
        nv[NORM_IN_STD + i] = 1.0f;
        nv[NORM_IN_LO + i] = -1e30f;
        nv[NORM_IN_HI + i] = 1e30f;
    }
    for (int i = 0; i < 16; ++i) {
        nv[NORM_OUT_STD + i] = 1.0f;
        nv[NORM_OUT_LO + i] = -1e30f;
        nv[NORM_OUT_HI + i] = 1e30f;
    }
    for (int col = 0; col < STAT_COLS; ++col) {
        double s1 = 0, s2 = 0, lo = 1e300, hi = -1e300;
        for (int b = 0; b < nb; ++b) {
            const double* p = hp.data() + size_t(b) * 4 * STAT_COLS;
            s1 += p[col];
            s2 += p[STAT_COLS + col];
            lo = std::min(lo, p[2 * STAT_COLS + col]);
            hi = std::max(hi, p[3 * STAT_COLS + col]);
        }
        const double mean = s1 / double(n);
        const double var = std::max(0.0, s2 / double(n) - mean * mean);
        const double sd = var > 0 ? std::sqrt(var) : 1.0;
        const bool in = col < 7;
        const int j = in ? col : col - 7;
        nv[(in ? NORM_IN_MEAN : NORM_OUT_MEAN) + j] = float(mean);
        nv[(in ? NORM_IN_STD : NORM_OUT_STD) + j] = float(sd);
        nv[(in ? NORM_IN_LO : NORM_OUT_LO) + j] = float((lo - mean) / sd);
        nv[(in ? NORM_IN_HI : NORM_OUT_HI) + j] = float((hi - mean) / sd);
    }
    HIP_TRY(hipMemcpyAsync(norm, nv.data(), sizeof(float) * NORM_N, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return LBM_OK;
}

int lbm_mlp_normalize(float* x, float* r, int64_t n, const float* norm, void* stream)
{
    if (!x || !r || !norm || n < 0) return fail(LBM_EINVAL, "x, r, norm or n invalid");
    if (n == 0) return LBM_OK;
    k_normalize<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream)>>>(x, r, n, norm);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m);

int lbm_mlp_create(lbm_mlp** out, float* theta, int64_t max_batch, void* stream)
{
    if (!out || !theta || max_batch < 1) return fail(LBM_EINVAL, "out, theta or max_batch invalid");
    lbm_mlp* m = new (std::nothrow) lbm_mlp;
    if (!m) return fail(LBM_ENOMEM, "mlp allocation failed");
    m->theta = theta;
    m->stream = static_cast<hipStream_t>(stream);
    m->max_batch = max_batch;
    m->nblocks = int(std::min<int64_t>(128, (max_batch + 63) / 64));
    const int nw = 4 * m->nblocks;
    bool ok = hipMalloc(&m->m, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->v, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->grad, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&m->partial, sizeof(float) * MLP_NPARAM * nw) == hipSuccess &&
              hipMalloc(&m->loss, sizeof(float) * nw) == hipSuccess &&
              hipMalloc(&m->fi, sizeof(MlpInfer)) == hipSuccess && hipMalloc(&m->fb, sizeof(MlpBack)) == hipSuccess;
    ok = ok && hipMemsetAsync(m->m, 0, sizeof(float) * MLP_NPARAM, m->stream) == hipSuccess &&
         hipMemsetAsync(m->v, 0, sizeof(float) * MLP_NPARAM, m->stream) == hipSuccess;
    if (!ok) {
        lbm_mlp_destroy(m);
        return fail(LBM_EDEVICE, "mlp device allocation failed");
    }
    m->loss_host.resize(size_t(nw));
    *out = m;
    return LBM_OK;
}

int lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t n, float* y)
{
    if (!m || !x || !y || n < 0) return fail(LBM_EINVAL, "mlp, x, y or n invalid");
    if (n == 0) return LBM_OK;
    HIP_TRY(launch_frags(m->theta, m->fi, m->fb, m->stream));
    const int64_t blocks = (n + 63) / 64; // 16 samples per wave, 4 waves per block
    k_mlp_forward<<<dim3(unsigned(blocks)), dim3(256), 0, m->stream>>>(m->fi, x, n, y);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int lbm_mlp_step(lbm_mlp* m, const float* x, const float* t, const int* idx, int64_t batch, float lr, float* grad,
                 double* loss)
{
    if (!m || !x || !t) return fail(LBM_EINVAL, "mlp, x or t is NULL");
    if (batch < 1 || batch > m->max_batch) return fail(LBM_EINVAL, "batch must be in [1, max_batch]");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(LBM_EINVAL, "lr must be finite and >= 0");
    HIP_TRY(launch_frags(m->theta, m->fi, m->fb, m->stream));
    const int nb = int(std::min<int64_t>(m->nblocks, (batch + 63) / 64));
    GradArgs ga{ m->fi, m->fb, x, t, idx, batch, float(2.0 / (double(batch) * MLP_OUT)), m->partial, m->loss };
    k_mlp_grad<<<dim3(unsigned(nb)), dim3(256), 0, m->stream>>>(ga);
    HIP_TRY(hipGetLastError());
    float bc1 = 1.0f, bc2 = 1.0f;
    if (lr > 0.0f) {
        ++m->t;
        bc1 = float(1.0 - std::pow(0.9, m->t));
        bc2 = float(1.0 - std::pow(0.999, m->t));
    }
    k_mlp_reduce_adam<<<dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, m->stream>>>(
        m->partial, 4 * nb, grad ? grad : m->grad, m->theta, m->m, m->v, lr, bc1, bc2);
    HIP_TRY(hipGetLastError());
    if (loss) {
        HIP_TRY(hipMemcpyAsync(m->loss_host.data(), m->loss, sizeof(float) * 4 * nb, hipMemcpyDeviceToHost, m->stream));
        HIP_TRY(hipStreamSynchronize(m->stream));
        double sum = 0;
        for (int w = 0; w < 4 * nb; ++w) sum += m->loss_host[size_t(w)];
        *loss = sum / (double(batch) * MLP_OUT);
    }
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (void* p : { (void*)m->m, (void*)m->v, (void*)m->grad, (void*)m->partial, (void*)m->loss, (void*)m->fi,
                     (void*)m->fb })
        if (p) (void)hipFree(p);
    delete m;
}

int lbm_closure_set(lbm_ctx* c, const float* theta, const float* norm)
{
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!theta) {
        c->closure = false;
        return LBM_OK;
    }
    if (!norm) return fail(LBM_EINVAL, "norm is NULL");
    if (c->lattice != LBM_D2V37 || c->coll != COLL_RR || c->thermal || c->store == ST_MOM || c->store == ST_F32D ||
        c->aa)
        return fail(LBM_EINVAL, "the closure needs an isothermal RR D2V37 context storing FP64, FP32 or BF16 populations in two buffers");
    if (!c->cl_frags) {
        HIP_TRY(hipMalloc(&c->cl_frags, sizeof(MlpInfer)));
        HIP_TRY(hipMalloc(&c->cl_norm, sizeof(float) * NORM_N));
        HIP_TRY(hipMalloc(&c->cl_fallbacks, sizeof(unsigned long long) * FALLBACK_SLOTS));
    }
    HIP_TRY(launch_frags(theta, c->cl_frags, nullptr, c->stream));
    HIP_TRY(hipMemcpyAsync(c->cl_norm, norm, sizeof(float) * NORM_N, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->cl_fallbacks, 0, sizeof(unsigned long long) * FALLBACK_SLOTS, c->stream));
    c->closure = true;
    return LBM_OK;
}

int lbm_closure_fallbacks(lbm_ctx* c, int64_t* count)
{
    if (!c || !count) return fail(LBM_EINVAL, "ctx or count is NULL");
    if (!c->cl_fallbacks) {
        *count = 0;
        return LBM_OK;
    }
    unsigned long long v[FALLBACK_SLOTS] = {};
    HIP_TRY(hipMemcpyAsync(v, c->cl_fallbacks, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    unsigned long long total = 0;
    for (unsigned long long x : v) total += x;
    *count = int64_t(total);
    return LBM_OK;
}

} // extern "C"
