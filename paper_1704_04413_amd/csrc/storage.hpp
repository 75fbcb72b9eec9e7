// Population storage kinds shared by the 2D and 3D kernels: FP64, and the
// weight-shifted FP32 and BF16 forms (g = f - w) with the counter-based
// stochastic rounding of BF16; the store of one node's Q values; the dump of
// the populations as FP64 f; and the block reduction of the diagnostics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "lattices.hpp"

namespace rr {

// ---------------------------------------------------------------- storage

struct StoreF64 {
    using elem = double;
    using math = double;
    static constexpr bool shifted = false;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = false;
    static __device__ __forceinline__ double load(const double* p) { return *p; }
    static __device__ __forceinline__ double load_nt(const double* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
    static __device__ __forceinline__ void store_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
};

struct StoreF32 {
    using elem = float;
    using math = float;
    static constexpr bool shifted = true;
    static constexpr bool conserve_in_double = true;
    static constexpr bool dithered = false;
    static __device__ __forceinline__ float load(const float* p) { return *p; }
    static __device__ __forceinline__ float load_nt(const float* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
    static __device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
};

// FP32 storage with double arithmetic: the same weight-shifted floats in HBM,
// every moment, coefficient and reconstruction in double (the float rounding
// happens once per value, at the store).
struct StoreF32D {
    using elem = float;
    using math = double;
    static constexpr bool shifted = true;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = false;
    static __device__ __forceinline__ double load(const float* p) { return double(*p); }
    static __device__ __forceinline__ double load_nt(const float* p) { return double(__builtin_nontemporal_load(p)); }
    static __device__ __forceinline__ void store(float* p, double v) { *p = float(v); }
    static __device__ __forceinline__ void store_nt(float* p, double v) { __builtin_nontemporal_store(float(v), p); }
};

// bfloat16 = the upper half of an IEEE float.  The initial state is rounded
// to nearest even; every step rounds stochastically (store_nt_sr): with
// deterministic rounding a near-uniform region sits at a fixed point of the
// rounded update and its 2^-9 rounding bias acts coherently over thousands of
// steps, while a rounding that is unbiased in expectation turns it into noise.
struct StoreBF16 {
    using elem = uint16_t;
    using math = float;
    static constexpr bool shifted = true;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = true;
    static __device__ __forceinline__ float load(const uint16_t* p)
    {
        return __uint_as_float(uint32_t(*p) << 16);
    }
    static __device__ __forceinline__ float load_nt(const uint16_t* p)
    {
        return __uint_as_float(uint32_t(__builtin_nontemporal_load(p)) << 16);
    }
    static __device__ __forceinline__ uint16_t round(float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u); // quiet NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    static __device__ __forceinline__ void store(uint16_t* p, float v) { *p = round(v); }
    static __device__ __forceinline__ void store_nt(uint16_t* p, float v) { __builtin_nontemporal_store(round(v), p); }
    // r: 16 uniform random bits; |v| rounds up with probability (dropped bits) / 2^16
    static __device__ __forceinline__ uint16_t round_sr(float v, uint32_t r)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u); // quiet NaN
        return uint16_t((u + r) >> 16);
    }
    static __device__ __forceinline__ void store_nt_sr(uint16_t* p, float v, uint32_t r)
    {
        __builtin_nontemporal_store(round_sr(v, r), p);
    }
    static __device__ __forceinline__ void store_sr(uint16_t* p, float v, uint32_t r) { *p = round_sr(v, r); }
};

// Counter-based random bits for stochastic rounding: a function of the node
// (y nx + x of its own grid) and of the index of the state being written (0 for
// the initial state, n after n steps) only, so results do not depend on launch
// shape or batching.  The key is Wellons' "lowbias32" integer hash; the stream
// per node is the 32-bit LCG of PCG (O'Neill), of which the top 16 bits are used.
struct Dither {
    uint32_t s;
    static __device__ __forceinline__ uint32_t mix(uint32_t x)
    {
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        return x;
    }
    __device__ __forceinline__ Dither(uint32_t node, uint32_t seq) : s(mix(node ^ mix(seq * 0x9e3779b9u + 0x6a09e667u))) {}
    __device__ __forceinline__ uint32_t next16()
    {
        s = s * 747796405u + 2891336453u;
        return s >> 16;
    }
};

// Writes the Q post-collision values of one node, value i to the element
// at(i) points to (stochastic rounding where the storage asks for it, the
// random bits drawn in the order of i whatever the addresses).
template <class L, class S, class T, bool NT, class At>
__device__ __forceinline__ void store_node_at(At&& at, const T (&v)[L::Q], uint32_t node, uint32_t seq)
{
    // NT: non-temporal stores, for state buffers larger than the memory-side
    // cache; ordinary stores leave the written state there for the next step
    if constexpr (S::dithered) {
        Dither dz(node, seq);
        if constexpr (NT)
            static_for<L::Q>([&](auto I) { S::store_nt_sr(at(I), v[I], dz.next16()); });
        else
            static_for<L::Q>([&](auto I) { S::store_sr(at(I), v[I], dz.next16()); });
    } else {
        if constexpr (NT)
            static_for<L::Q>([&](auto I) { S::store_nt(at(I), v[I]); });
        else
            static_for<L::Q>([&](auto I) { S::store(at(I), v[I]); });
    }
}

// The same into the node's own slots (plane i at `here`).
template <class L, class S, class T, bool NT = true>
__device__ __forceinline__ void store_node(typename S::elem* __restrict__ fout, int here, int te, const T (&v)[L::Q],
                                           uint32_t node, uint32_t seq)
{
    // the node's base pointer once, then one uniform plane offset per value
    typename S::elem* const base = fout + here;
    store_node_at<L, S, T, NT>([&](auto I) { return base + int(I) * te; }, v, node, seq);
}

// Where value i of the post-collision state of node (x, y) is held.  RD 0:
// the two-buffer state, plane i at the node.  The single-buffer AA state
// after an even number of steps (RD 1): plane opp(i) at the node; after an
// odd number (RD 2): plane i at the node x + c_i (periodic).
template <class L>
constexpr int opp_index(int i)
{
    return vel_index<L>(-L::v.cx[i], -L::v.cy[i]);
}

template <class L, int RD, int I>
__device__ __forceinline__ int state_index(const Layout& lay, int x, int y)
{
    if constexpr (RD == 0) {
        return lay.row(y) + x + I * lay.te;
    } else if constexpr (RD == 1) {
        constexpr int o = opp_index<L>(I); // folded at compile time
        return lay.row(y) + x + o * lay.te;
    } else {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        int xx = x + cx, yy = y + cy;
        xx += xx < 0 ? lay.nx : 0;
        xx -= xx >= lay.nx ? lay.nx : 0;
        yy += yy < 0 ? lay.ny : 0;
        yy -= yy >= lay.ny ? lay.ny : 0;
        return lay.row(yy) + xx + I * lay.te;
    }
}

// ------------------------------------------------------ dump / reductions

// The state as FP64 populations [i][y][x]; RD: where it sits (state_index).
template <class L, class S, int RD = 0>
__global__ __launch_bounds__(256) void k_populations(const void* fsrc, Layout lay, double* out)
{
    const int64_t n = int64_t(lay.nx) * lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = int(k % lay.nx), y = int(k / lay.nx);
    const typename S::elem* f = static_cast<const typename S::elem*>(fsrc);
    static_for<L::Q>([&](auto I) {
        double v = double(S::load(f + state_index<L, RD, int(I)>(lay, x, y)));
        if (S::shifted) v += L::v.w[I];
        out[int64_t(I) * n + k] = v;
    });
}

template <int NS>
__device__ __forceinline__ void block_sums(double (&val)[NS], double* partial)
{
    __shared__ double red[NS][256];
    const int t = threadIdx.x;
    for (int s = 0; s < NS; ++s) red[s][t] = val[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int s = 0; s < NS; ++s) red[s][t] += red[s][t + w];
        __syncthreads();
    }
    if (t < NS) partial[int64_t(blockIdx.x) * NS + t] = red[t][0];
}

} // namespace rr
