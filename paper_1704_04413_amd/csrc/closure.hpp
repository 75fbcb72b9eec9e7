// Learned closure for the higher-order non-equilibrium coefficients (not part
// of the paper's method): a per-node perceptron 8 -> 64 -> 64 -> 9 (tanh-form
// GELU) predicts a residual added to the recursive a1^(3), a1^(4) of the
// isothermal D2V37 collision.  Mass and momentum are untouched whatever the
// network outputs (the residual only enters ranks 3 and 4, which are
// orthogonal to ranks 0 and 1).
//
// Matrix products run on the bfloat16 matrix cores,
// v_mfma_f32_16x16x16_bf16, with FP32 accumulation.  Lane l of a wave holds
//   A (16x16, rows x k):   A[l % 16][(l / 16) * 4 + j]
//   B (16x16, k x cols):   B[(l / 16) * 4 + j][l % 16]
//   D (16x16):             D[(l / 16) * 4 + j][l % 16],     j = 0..3.
// Activations are kept as the B operand with the sample (node) index as the
// column, so a layer's D output is already the next layer's B operand and the
// forward pass needs no transposes; weights are the A operand, prepared once
// as per-lane fragments.  Weight gradients contract over samples and read
// LDS-transposed tiles.
//
// Parameter vector (float32), row-major [in][out]:
//   W1 8x64 | b1 64 | W2 64x64 | b2 64 | W3 64x16 | b3 16   (outputs 9..15 pad)
// Normalisation block (float32, 96 values):
//   in_mean[8] in_std[8] in_lo[8] in_hi[8] out_mean[16] out_std[16] out_lo[16] out_hi[16]
// (inputs 0..6 used, input 7 is the constant 1; outputs 0..8 used; lo/hi are
// the training range in normalised units).  Inputs: rho - 1, ux, uy,
// |u|^2 / c_s^2, ahat_xx, ahat_xy, ahat_yy with ahat = (1 - 1/(2 tau)) a1
// (tau-independent: the viscous stress is -ahat^(2)); outputs: the residual
// of ahat^(3..4) in the order 30, 21, 12, 03, 40, 31, 22, 13, 04.
#pragma once

#include <cstdint>

#include "collide.hpp"
#include "step2d.hpp"

namespace rr {

constexpr int MLP_IN = 8, MLP_H = 64, MLP_OUT = 9, MLP_OUTP = 16;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 5760;
constexpr int MLP_NPARAM = 5776;
constexpr int NORM_IN_MEAN = 0, NORM_IN_STD = 8, NORM_IN_LO = 16, NORM_IN_HI = 24;
constexpr int NORM_OUT_MEAN = 32, NORM_OUT_STD = 48, NORM_OUT_LO = 64, NORM_OUT_HI = 80, NORM_N = 96;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ short f2bf(float v) { return __builtin_bit_cast(short, static_cast<__bf16>(v)); }

__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(uint32_t(uint16_t(b)) << 16); }

// tanh-form GELU and its derivative (Hendrycks & Gimpel), written with
// 0.5 (1 + tanh(u)) = 1 / (1 + e^(-2u)) and the hardware exp2 and reciprocal
// (the results are rounded to bfloat16 or feed bfloat16 products).
__device__ __forceinline__ float sigmoid2u(float z)
{
    // e^(-2u) = 2^(-2 log2(e) c (z + a z^3)), c = sqrt(2/pi), a = 0.044715
    const float k = -2.0f * 1.4426950408889634f * 0.7978845608028654f;
    const float e = __builtin_amdgcn_exp2f(k * z * (1.0f + 0.044715f * z * z));
    return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float gelu_f(float z) { return z * sigmoid2u(z); }

__device__ __forceinline__ float gelu_prime_f(float z)
{
    const float s = sigmoid2u(z);
    // d/dz [z s(v)] = s + z s (1 - s) v',  v = 2c (z + a z^3)
    return s + z * s * (1.0f - s) * (2.0f * 0.7978845608028654f) * (1.0f + 0.134145f * z * z);
}

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weight fragments for inference (what the fused collide kernel stages in LDS).
struct MlpInfer {
    v4s w1[4][64];    // layer 1, output tile t: A[u][k] = W1[k][16t + u]   (k < 8)
    v4s w2[4][4][64]; // layer 2, [t2][t]:       A[u][k] = W2[16t + k][16t2 + u]
    v4s w3[4][64];    // layer 3, input tile t:  A[o][k] = W3[16t + k][o]
    float b1[64], b2[64], b3[16];
};

// Extra fragments the backward pass needs.
struct MlpBack {
    v4s w3b[4][64];    // dH2 tile t:  A[u][k] = W3[16t + u][k]
    v4s w2b[4][4][64]; // dH1 [t][t2]: A[u][k] = W2[16t + u][16t2 + k]
};

// One thread per fragment: builds both fragment sets from the FP32 parameters.
__global__ __launch_bounds__(256) void k_mlp_frags(const float* __restrict__ th, MlpInfer* __restrict__ fi,
                                                   MlpBack* __restrict__ fb)
{
    const int id = int(blockIdx.x) * 256 + int(threadIdx.x);
    const int lane = id & 63, frag = id >> 6; // 44 fragments of 64 lanes
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4s a;
    if (frag < 4) {
        const int t = frag;
        for (int j = 0; j < 4; ++j) a[j] = (kq + j < 8) ? f2bf(th[OFF_W1 + (kq + j) * 64 + 16 * t + r]) : short(0);
        fi->w1[t][lane] = a;
    } else if (frag < 20) {
        const int t2 = (frag - 4) / 4, t = (frag - 4) % 4;
        for (int j = 0; j < 4; ++j) a[j] = f2bf(th[OFF_W2 + (16 * t + kq + j) * 64 + 16 * t2 + r]);
        fi->w2[t2][t][lane] = a;
    } else if (frag < 24) {
        const int t = frag - 20;
        for (int j = 0; j < 4; ++j) a[j] = f2bf(th[OFF_W3 + (16 * t + kq + j) * 16 + r]);
        fi->w3[t][lane] = a;
    } else if (frag < 28) {
        const int t = frag - 24;
        for (int j = 0; j < 4; ++j) a[j] = f2bf(th[OFF_W3 + (16 * t + r) * 16 + kq + j]);
        if (fb) fb->w3b[t][lane] = a;
    } else if (frag < 44) {
        const int t = (frag - 28) / 4, t2 = (frag - 28) % 4;
        for (int j = 0; j < 4; ++j) a[j] = f2bf(th[OFF_W2 + (16 * t + r) * 64 + 16 * t2 + kq + j]);
        if (fb) fb->w2b[t][t2][lane] = a;
    } else if (id < 44 * 64 + 144) {
        const int b = id - 44 * 64;
        if (b < 64)
            fi->b1[b] = th[OFF_B1 + b];
        else if (b < 128)
            fi->b2[b - 64] = th[OFF_B2 + b - 64];
        else
            fi->b3[b - 128] = th[OFF_B3 + b - 128];
    }
}

// Copies a trivially copyable struct from global to LDS with all threads of
// the block, 16 bytes at a time.
template <class S>
__device__ __forceinline__ void stage(S* dst, const S* __restrict__ src)
{
    static_assert(sizeof(S) % 16 == 0, "16-byte staging");
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    const int nthreads = int(blockDim.x * blockDim.y);
    const int tid = int(threadIdx.y * blockDim.x + threadIdx.x);
    for (int i = tid; i < int(sizeof(S) / 16); i += nthreads) d[i] = s[i];
}

// Forward pass of 16 samples held as the B operand xb (k = input feature).
// Returns Y (D layout: out (l/16)*4 + j, sample l % 16); the pre-activations
// and bf16 activations are returned for the backward pass.
struct FwdState {
    v4f z1[4], z2[4];
    v4s h1[4], h2[4];
};

__device__ __forceinline__ v4f mlp_fwd16(const MlpInfer& F, v4s xb, int lane, FwdState& st)
{
    const int kq = (lane >> 4) * 4;
    const v4f zero = { 0.f, 0.f, 0.f, 0.f };
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const v4f d = mfma16(F.w1[t][lane], xb, zero);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float z = d[j] + F.b1[16 * t + kq + j];
            st.z1[t][j] = z;
            st.h1[t][j] = f2bf(gelu_f(z));
        }
    }
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) {
        v4f acc = zero;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = mfma16(F.w2[t2][t][lane], st.h1[t], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float z = acc[j] + F.b2[16 * t2 + kq + j];
            st.z2[t2][j] = z;
            st.h2[t2][j] = f2bf(gelu_f(z));
        }
    }
    v4f y = zero;
#pragma unroll
    for (int t = 0; t < 4; ++t) y = mfma16(F.w3[t][lane], st.h2[t], y);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] += F.b3[kq + j];
    return y;
}

// ------------------------------------------------- fused closure collision

// Closure inputs of one node from its coefficients (isothermal, a1 before
// truncation): rho - 1, ux, uy, |u|^2 / c_s^2, s a1_xx, s a1_xy, s a1_yy.
template <class L, class T>
__device__ __forceinline__ void closure_features(const NodeCoeffs<T>& k, T s, float (&f)[7])
{
    constexpr T cs2 = T(L::cs2);
    f[0] = float(k.drho);
    f[1] = float(k.ux);
    f[2] = float(k.uy);
    f[3] = float((k.ux * k.ux + k.uy * k.uy) / cs2);
    f[4] = float(s * k.a1[2][0]);
    f[5] = float(s * k.a1[1][1]);
    f[6] = float(s * k.a1[0][2]);
}

// Fallback counters are spread over this many slots (by block) so that waves
// of different blocks rarely add to the same address.
constexpr int FALLBACK_SLOTS = 64;

struct ClosureArgs {
    const MlpInfer* frags;
    const float* norm;
    double s;             // 1 - 1/(2 tau)
    unsigned long long* fallbacks; // FALLBACK_SLOTS running counts of nodes that kept the plain recursion
};

// Register budget of the fused closure step, as the minimum number of waves
// per SIMD the compiler must leave room for.
// Four waves per SIMD (at most 128 VGPRs) let loads of some waves overlap the
// network of others: 6% faster at 1024^2 than the unconstrained 140 VGPRs.
#ifndef RRLBM_CLOSURE_WAVES_PER_EU
#define RRLBM_CLOSURE_WAVES_PER_EU 4
#endif

// POL: the cache policy of the plain step (load and store kinds).
template <class S, int POL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RRLBM_CLOSURE_WAVES_PER_EU)))
void k_stream_collide_closure(StepArgs a, ClosureArgs c)
{
    using L = D2V37;
    using T = typename S::math;
    using E = typename S::elem;
    constexpr int R = L::R;
    __shared__ MlpInfer sF;
    __shared__ float snorm[NORM_N];
    __shared__ short xin[4][64 * 8];
    __shared__ float yout[4][64 * 16];
    stage(&sF, c.frags);
    const int tid = int(threadIdx.y) * BX + int(threadIdx.x);
    if (tid < NORM_N) snorm[tid] = c.norm[tid];

    const int bid = block_index(a);
    const Layout& lay = a.lay;
    const int x = (bid % a.bx_blocks) * BX + int(threadIdx.x);
    const int y = (bid / a.bx_blocks) * BY + int(threadIdx.y);
    const bool valid = x < lay.nx && y < lay.ny;
    const int xc = valid ? x : 0, yc = valid ? y : 0; // idle lanes still join the matrix ops
    const E* __restrict__ fin = static_cast<const E*>(a.fin);
    E* __restrict__ fout = static_cast<E*>(a.fout);
    const int nx = lay.nx, ny = lay.ny;

    int xs[2 * R + 1], ys[2 * R + 1];
    static_for<2 * R + 1>([&](auto D) {
        constexpr int d = int(D) - R;
        int xx = xc - d, yy = yc - d;
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
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        const int idx = ys[cy + R] + xs[cx + R] + int(I) * lay.te;
        if constexpr (POL == POL_KEEP)
            v[I] = S::load_nt(fin + idx);
        else
            v[I] = S::load(fin + idx);
    });
    Invariants<L, T, false, S::conserve_in_double> inv;
    inv.take(v);
    NodeCoeffs<T> k;
    node_coeffs<L, T, COLL_RR, false, S::shifted, false>(v, k);

    const T s = T(c.s);
    float feat[7];
    closure_features<L, T>(k, s, feat);
    __syncthreads(); // sF, snorm staged
    const int wave = tid >> 6, lane = tid & 63;
    bool ok = true;
    short* xw = xin[wave];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const float z = (feat[j] - snorm[NORM_IN_MEAN + j]) / snorm[NORM_IN_STD + j];
        ok = ok && z >= snorm[NORM_IN_LO + j] && z <= snorm[NORM_IN_HI + j];
        xw[lane * 8 + j] = f2bf(z);
    }
    xw[lane * 8 + 7] = f2bf(1.0f);
    __syncthreads();
    const int kq = (lane >> 4) * 4;
    float* yw = yout[wave];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int node = 16 * g + (lane & 15);
        v4s xb;
#pragma unroll
        for (int j = 0; j < 4; ++j) xb[j] = (kq + j < 8) ? xw[node * 8 + kq + j] : short(0);
        FwdState st;
        const v4f yv = mlp_fwd16(sF, xb, lane, st);
#pragma unroll
        for (int j = 0; j < 4; ++j) yw[node * 16 + kq + j] = yv[j];
    }
    __syncthreads();
    float r[MLP_OUT];
#pragma unroll
    for (int o = 0; o < MLP_OUT; ++o) {
        const float yo = yw[lane * 16 + o];
        ok = ok && yo >= snorm[NORM_OUT_LO + o] && yo <= snorm[NORM_OUT_HI + o];
        r[o] = yo * snorm[NORM_OUT_STD + o] + snorm[NORM_OUT_MEAN + o];
    }
    const unsigned long long missed = __ballot(valid && !ok);
    if (lane == 0 && missed)
        atomicAdd(c.fallbacks + (blockIdx.x & (FALLBACK_SLOTS - 1)), (unsigned long long)__popcll(missed));
    if (ok) {
        const T inv_s = T(1) / s;
        k.a1[3][0] += T(r[0]) * inv_s;
        k.a1[2][1] += T(r[1]) * inv_s;
        k.a1[1][2] += T(r[2]) * inv_s;
        k.a1[0][3] += T(r[3]) * inv_s;
        k.a1[4][0] += T(r[4]) * inv_s;
        k.a1[3][1] += T(r[5]) * inv_s;
        k.a1[2][2] += T(r[6]) * inv_s;
        k.a1[1][3] += T(r[7]) * inv_s;
        k.a1[0][4] += T(r[8]) * inv_s;
    }
    relax_reconstruct<L, T>(k, T(a.rx.k2), T(a.rx.k3), T(a.rx.k4), v);
    inv.restore(v);
    if (valid) {
        const int here = lay.row(y) + x;
        store_node<L, S, T, POL == POL_STREAM>(fout, here, lay.te, v, uint32_t(y) * uint32_t(nx) + uint32_t(x), a.seq);
    }
}

// ----------------------------------------------------------- training

// Forward pass over n samples x[n][8] (already normalised, x[.][7] = 1):
// y[n][16] (outputs 9..15 are the padding, zero bias).  One wave per 16 samples.
__global__ __launch_bounds__(256) void k_mlp_forward(const MlpInfer* __restrict__ F, const float* __restrict__ x,
                                                     int64_t n, float* __restrict__ y)
{
    __shared__ MlpInfer sF;
    stage(&sF, F);
    __syncthreads();
    const int lane = int(threadIdx.x) & 63;
    const int64_t group = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int kq = (lane >> 4) * 4;
    const int64_t smp = group * 16 + (lane & 15);
    v4s xb;
#pragma unroll
    for (int j = 0; j < 4; ++j) xb[j] = (kq + j < 8 && smp < n) ? f2bf(x[smp * 8 + kq + j]) : short(0);
    FwdState st;
    const v4f yv = mlp_fwd16(sF, xb, lane, st);
    if (smp < n)
#pragma unroll
        for (int j = 0; j < 4; ++j) y[smp * 16 + kq + j] = yv[j];
}

// Gradient of the mean squared error over a batch: forward, backward and
// weight gradients for groups of 16 samples, 4 waves per block; each wave
// accumulates its gradient in matrix-core accumulators and writes it to its
// own row of `partial` (MLP_NPARAM floats), plus its squared-error sum.
// Every wave of a block runs the same number of groups (samples past the
// batch contribute zero), so the block barriers are uniform.
struct GradArgs {
    const MlpInfer* fi;
    const MlpBack* fb;
    const float* x;   // [*][8]
    const float* t;   // [*][16]
    const int* idx;   // batch -> sample row, or NULL for identity
    int64_t batch;
    float inv_bn;     // 2 / (batch * 9)
    float* partial;   // [waves][MLP_NPARAM]
    float* loss;      // [waves]
};

__global__ __launch_bounds__(256) void k_mlp_grad(GradArgs g)
{
    __shared__ MlpInfer sF;
    __shared__ MlpBack sB;
    __shared__ short tX[4][16 * 16], tDY[4][16 * 16];
    __shared__ short tH1[4][4][16 * 16], tH2[4][4][16 * 16], tDZ1[4][4][16 * 16], tDZ2[4][4][16 * 16];
    stage(&sF, g.fi);
    stage(&sB, g.fb);
    __syncthreads();
    const int tid = int(threadIdx.x);
    const int wave = tid >> 6, lane = tid & 63, ln = lane & 15, kq = (lane >> 4) * 4;
    const v4f zero = { 0.f, 0.f, 0.f, 0.f };
    v4f aW1[4], aW2[4][4], aW3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        aW1[a] = zero;
        aW3[a] = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) aW2[a][b] = zero;
    }
    float ab1[4][4] = {}, ab2[4][4] = {}, ab3[4] = {}, lsum = 0.f;
    const int64_t groups = (g.batch + 15) / 16;
    const int64_t per_iter = int64_t(gridDim.x) * 4;
    for (int64_t base = int64_t(blockIdx.x) * 4; base < groups; base += per_iter) {
        const int64_t grp = base + wave;
        const int64_t bi = grp * 16 + ln; // batch position of this lane's sample
        const bool live = grp < groups && bi < g.batch;
        const int64_t row = live ? (g.idx ? int64_t(g.idx[bi]) : bi) : 0;
        v4s xb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            xb[j] = (live && kq + j < 8) ? f2bf(g.x[row * 8 + kq + j]) : short(0);
            tX[wave][(kq + j) * 16 + ln] = xb[j];
        }
        FwdState st;
        const v4f yv = mlp_fwd16(sF, xb, lane, st);
        v4s dyb;
        float dy[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = kq + j;
            const float diff = (live && o < MLP_OUT) ? yv[j] - g.t[row * 16 + o] : 0.f;
            lsum += diff * diff;
            dy[j] = diff * g.inv_bn;
            dyb[j] = f2bf(dy[j]);
            ab3[j] += dy[j];
            tDY[wave][o * 16 + ln] = dyb[j];
        }
        v4s dz2b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4f dh = mfma16(sB.w3b[t][lane], dyb, zero);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float dz = live ? dh[j] * gelu_prime_f(st.z2[t][j]) : 0.f;
                ab2[t][j] += dz;
                dz2b[t][j] = f2bf(dz);
                tDZ2[wave][t][(kq + j) * 16 + ln] = dz2b[t][j];
                tH2[wave][t][(kq + j) * 16 + ln] = live ? st.h2[t][j] : short(0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4f dh = zero;
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) dh = mfma16(sB.w2b[t][t2][lane], dz2b[t2], dh);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float dz = live ? dh[j] * gelu_prime_f(st.z1[t][j]) : 0.f;
                ab1[t][j] += dz;
                tDZ1[wave][t][(kq + j) * 16 + ln] = f2bf(dz);
                tH1[wave][t][(kq + j) * 16 + ln] = live ? st.h1[t][j] : short(0);
            }
        }
        __syncthreads();
        // weight gradients: contract over the 16 samples (k = sample)
        auto rd = [&](const short* tile) {
            v4s v;
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = tile[ln * 16 + kq + j];
            return v;
        };
        const v4s ax = rd(tX[wave]);
        const v4s bdy = rd(tDY[wave]);
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) aW1[tn] = mfma16(ax, rd(tDZ1[wave][tn]), aW1[tn]);
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
            const v4s ah1 = rd(tH1[wave][tm]);
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) aW2[tm][tn] = mfma16(ah1, rd(tDZ2[wave][tn]), aW2[tm][tn]);
            aW3[tm] = mfma16(rd(tH2[wave][tm]), bdy, aW3[tm]);
        }
        __syncthreads();
    }
    // bias sums over the 16 samples of each lane group
    auto red16 = [](float v) {
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        return v;
    };
    float* out = g.partial + int64_t(blockIdx.x * 4 + wave) * MLP_NPARAM;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = kq + j;
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
            if (r < 8) out[OFF_W1 + r * 64 + 16 * tn + ln] = aW1[tn][j];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) out[OFF_W2 + (16 * tm + r) * 64 + 16 * tn + ln] = aW2[tm][tn][j];
            out[OFF_W3 + (16 * tm + r) * 16 + ln] = aW3[tm][j];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float s1 = red16(ab1[t][j]), s2 = red16(ab2[t][j]);
            if (ln == 0) {
                out[OFF_B1 + 16 * t + kq + j] = s1;
                out[OFF_B2 + 16 * t + kq + j] = s2;
            }
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float s3 = red16(ab3[j]);
        if (ln == 0) out[OFF_B3 + kq + j] = s3;
    }
    float l = lsum;
    for (int m = 32; m > 0; m >>= 1) l += __shfl_xor(l, m);
    if (lane == 0) g.loss[blockIdx.x * 4 + wave] = l;
}

// Sums the per-wave gradients (fixed order) into grad[], and when lr > 0
// applies one Adam step (t counts from 1) to the FP32 parameters.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float* __restrict__ partial, int nwaves,
                                                         float* __restrict__ grad, float* __restrict__ th,
                                                         float* __restrict__ m, float* __restrict__ v, float lr,
                                                         float bc1, float bc2)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= MLP_NPARAM) return;
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += partial[int64_t(w) * MLP_NPARAM + i];
    grad[i] = s;
    if (lr > 0.f) {
        const float mi = 0.9f * m[i] + 0.1f * s;
        const float vi = 0.999f * v[i] + 0.001f * s * s;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
    }
}

// ------------------------------------------------------ training samples

// One thread per coarse node: block-averages the factor x factor fine nodes'
// rho, rho u and ahat^(2..4) (from the fine post-collision populations,
// ahat = (1 - 1/(2 tau_f)) / (1 - 1/tau_f) (h - a0) for ranks 2..4), then
// writes the raw closure inputs x[c][0..6] (x[c][7] = 1) and the residual
// r[c][0..8] = ahat^(3..4) - recursion(rho, u, ahat^(2)) (r[c][9..15] = 0).
template <class S>
__global__ __launch_bounds__(256) void k_closure_samples(const void* fsrc, Layout lay, int factor, double sf,
                                                         float* __restrict__ xo, float* __restrict__ ro)
{
    using L = D2V37;
    using T = double;
    const int cnx = lay.nx / factor, cny = lay.ny / factor;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= int64_t(cnx) * cny) return;
    const int cx0 = int(c % cnx) * factor, cy0 = int(c / cnx) * factor;
    const typename S::elem* f = static_cast<const typename S::elem*>(fsrc);
    double rho = 0, jx = 0, jy = 0, ah[5][5] = {};
    for (int dy = 0; dy < factor; ++dy)
        for (int dx = 0; dx < factor; ++dx) {
            const int here = lay.row(cy0 + dy) + cx0 + dx;
            T v[L::Q];
            static_for<L::Q>([&](auto I) { v[I] = T(S::load(f + here + int(I) * lay.te)); });
            NodeCoeffs<T> k;
            node_coeffs<L, T, COLL_PR, false, S::shifted, false>(v, k); // projections of every rank
            rho += k.rho;
            jx += k.rho * k.ux;
            jy += k.rho * k.uy;
            for (int a = 0; a < 5; ++a)
                for (int b = 0; a + b <= 4; ++b) ah[a][b] += sf * k.a1[a][b];
        }
    const double inv = 1.0 / double(factor * factor);
    rho *= inv;
    const double ux = jx * inv / rho, uy = jy * inv / rho;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; a + b <= 4; ++b) ah[a][b] *= inv;
    const double xx = ah[2][0], xy = ah[1][1], yy = ah[0][2];
    const double uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    const double rr[9] = { 3 * ux * xx, 2 * ux * xy + uy * xx, 2 * uy * xy + ux * yy, 3 * uy * yy,
                           6 * uxx * xx, 3 * (uxx * xy + uxy * xx), uyy * xx + uxx * yy + 4 * uxy * xy,
                           3 * (uyy * xy + uxy * yy), 6 * uyy * yy };
    const double hi[9] = { ah[3][0], ah[2][1], ah[1][2], ah[0][3], ah[4][0], ah[3][1], ah[2][2], ah[1][3], ah[0][4] };
    float* x = xo + c * 8;
    x[0] = float(rho - 1.0);
    x[1] = float(ux);
    x[2] = float(uy);
    x[3] = float((ux * ux + uy * uy) / L::cs2);
    x[4] = float(xx);
    x[5] = float(xy);
    x[6] = float(yy);
    x[7] = 1.0f;
    float* r = ro + c * 16;
    for (int o = 0; o < 16; ++o) r[o] = o < 9 ? float(hi[o] - rr[o]) : 0.0f;
}

// Column statistics of x[n][8] (columns 0..6) and r[n][16] (columns 0..8):
// per-block partial sums, squared sums, minima and maxima.
constexpr int STAT_COLS = 16; // 7 input + 9 output columns
__global__ __launch_bounds__(256) void k_col_stats(const float* __restrict__ x, const float* __restrict__ r, int64_t n,
                                                   double* __restrict__ part)
{
    __shared__ double red[4][4 * STAT_COLS];
    const int t = int(threadIdx.x), lane = t & 63, wave = t >> 6;
    double st[4][STAT_COLS]; // sum, sum of squares, min, max
    for (int c = 0; c < STAT_COLS; ++c) {
        st[0][c] = 0;
        st[1][c] = 0;
        st[2][c] = 1e300;
        st[3][c] = -1e300;
    }
    for (int64_t i = int64_t(blockIdx.x) * 256 + t; i < n; i += int64_t(gridDim.x) * 256) {
        for (int c = 0; c < STAT_COLS; ++c) {
            const double v = c < 7 ? double(x[i * 8 + c]) : double(r[i * 16 + c - 7]);
            st[0][c] += v;
            st[1][c] += v * v;
            st[2][c] = v < st[2][c] ? v : st[2][c];
            st[3][c] = v > st[3][c] ? v : st[3][c];
        }
    }
    for (int c = 0; c < STAT_COLS; ++c)
        for (int m = 32; m > 0; m >>= 1) {
            st[0][c] += __shfl_xor(st[0][c], m);
            st[1][c] += __shfl_xor(st[1][c], m);
            const double lo = __shfl_xor(st[2][c], m), hi = __shfl_xor(st[3][c], m);
            st[2][c] = lo < st[2][c] ? lo : st[2][c];
            st[3][c] = hi > st[3][c] ? hi : st[3][c];
        }
    if (lane == 0)
        for (int q = 0; q < 4; ++q)
            for (int c = 0; c < STAT_COLS; ++c) red[wave][q * STAT_COLS + c] = st[q][c];
    __syncthreads();
    if (t < 4 * STAT_COLS) {
        const int q = t / STAT_COLS;
        double v = red[0][t];
        for (int w = 1; w < 4; ++w) {
            const double o = red[w][t];
            v = q < 2 ? v + o : (q == 2 ? (o < v ? o : v) : (o > v ? o : v));
        }
        part[int64_t(blockIdx.x) * 4 * STAT_COLS + t] = v;
    }
}

// x[.][0..6] -> (x - mean) / std, r[.][0..8] -> (r - mean) / std.
__global__ __launch_bounds__(256) void k_normalize(float* __restrict__ x, float* __restrict__ r, int64_t n,
                                                   const float* __restrict__ norm)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 7; ++c)
        x[i * 8 + c] = (x[i * 8 + c] - norm[NORM_IN_MEAN + c]) / norm[NORM_IN_STD + c];
    x[i * 8 + 7] = 1.0f;
    for (int c = 0; c < 9; ++c)
        r[i * 16 + c] = (r[i * 16 + c] - norm[NORM_OUT_MEAN + c]) / norm[NORM_OUT_STD + c];
}

} // namespace rr
