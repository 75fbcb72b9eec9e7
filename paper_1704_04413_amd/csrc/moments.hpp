// Moment representation of the isothermal recursive-regularized step.
//
// With the isothermal recursive regularization at order N, the post-collision
// populations of a node are a function of its (rho, u, a1^(2)) alone: Eq.
// (GenRegCollision) takes a0 from (rho, u) (Eq. HermiteCoeffEq at theta = 1)
// and a1^(3..N) from u and a1^(2) (Eq. MalaspinasRecursiveRelation).  Those six
// values are therefore the whole state between steps.  A step rebuilds every
// pulled population f_i(x - c_i) from the moments of the node x - c_i, and the
// moments of what arrives at x are the new state of x:
//   rho = sum f_i, rho u = sum f_i c_i, a1^(2) = sum f_i H^(2)_i - rho u u.
// This is the same sequence of states as the population form (up to
// rounding), with 2 x 6 values of HBM traffic per node instead of 2 Q.
//
// State layout: six FP64 planes [m][y][x], m = rho, ux, uy, a1_xx, a1_xy,
// a1_yy of the pre-collision populations.
#pragma once

#include "collide.hpp"

namespace rr {

struct StoreMom {
    using elem = double;
    using math = double;
    static constexpr bool shifted = false;
    static constexpr bool conserve_in_double = false;
    static constexpr bool dithered = false;
};

// Coefficient of the basis term (a, b) in population (cx, cy):
// He_a(cx) He_b(cy) / (a! b! c_s^2(a+b)), 0 off the lattice basis.
template <class L>
constexpr double hc(int cx, int cy, int a, int b)
{
    return L::basis(a, b) ? he(a, double(cx), L::cs2) * he(b, double(cy), L::cs2) * inv_norm<L>(a, b) : 0.0;
}

// Post-collision population I of a node with moments (r, ux, uy, a1^(2)) at
// regularization order ORDER with the relaxation rx:
//   f_I = w_I [ r E_I(u) + a1_xx A^xx_I(u) + a1_xy A^xy_I(u) + a1_yy A^yy_I(u) ]
// with E_I = sum_k h_Ik u_x^kx u_y^ky (the equilibrium, a0_k = r u_x^kx u_y^ky at
// theta = 1) and A_I the rank-2..ORDER terms of the expansion after the
// isothermal recursion, each weighted by its relaxation factor k_n: linear in
// a1^(2) with coefficients polynomial in u (degree 0, 1, 2 for ranks 2, 3,
// 4).  Every h is a compile-time constant; zero terms are left out.  PO:
// per-order factors; otherwise k3 = k4 = k2 on the kept ranks and the common
// factor is applied once.
template <class L, int I, int ORDER, bool PO>
__device__ __forceinline__ double mom_pop(double r, double ux, double uy, double axx, double axy, double ayy,
                                          const Relax& rx)
{
    constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
    constexpr double h10 = hc<L>(cx, cy, 1, 0), h01 = hc<L>(cx, cy, 0, 1);
    constexpr double h20 = hc<L>(cx, cy, 2, 0), h11 = hc<L>(cx, cy, 1, 1), h02 = hc<L>(cx, cy, 0, 2);
    constexpr double h30 = hc<L>(cx, cy, 3, 0), h21 = hc<L>(cx, cy, 2, 1), h12 = hc<L>(cx, cy, 1, 2),
                     h03 = hc<L>(cx, cy, 0, 3);
    constexpr double h40 = hc<L>(cx, cy, 4, 0), h31 = hc<L>(cx, cy, 3, 1), h22 = hc<L>(cx, cy, 2, 2),
                     h13 = hc<L>(cx, cy, 1, 3), h04 = hc<L>(cx, cy, 0, 4);
    const double x2 = ux * ux, xy = ux * uy, y2 = uy * uy;
    // equilibrium polynomial
    double e = 1.0;
    if constexpr (h10 != 0.0) e += h10 * ux;
    if constexpr (h01 != 0.0) e += h01 * uy;
    if constexpr (h20 != 0.0) e += h20 * x2;
    if constexpr (h11 != 0.0) e += h11 * xy;
    if constexpr (h02 != 0.0) e += h02 * y2;
    if constexpr (h30 != 0.0) e += h30 * (x2 * ux);
    if constexpr (h21 != 0.0) e += h21 * (x2 * uy);
    if constexpr (h12 != 0.0) e += h12 * (xy * uy);
    if constexpr (h03 != 0.0) e += h03 * (y2 * uy);
    if constexpr (h40 != 0.0) e += h40 * (x2 * x2);
    if constexpr (h31 != 0.0) e += h31 * (x2 * xy);
    if constexpr (h22 != 0.0) e += h22 * (x2 * y2);
    if constexpr (h13 != 0.0) e += h13 * (xy * y2);
    if constexpr (h04 != 0.0) e += h04 * (y2 * y2);
    // non-equilibrium: coefficients of a1_xx, a1_xy, a1_yy, rank by rank
    // rank 3: a1_30 = 3 ux xx, a1_21 = 2 ux xy + uy xx, a1_12 = 2 uy xy + ux yy, a1_03 = 3 uy yy
    // rank 4: a1_40 = 6 ux^2 xx, a1_31 = 3 (ux^2 xy + ux uy xx),
    //         a1_22 = uy^2 xx + ux^2 yy + 4 ux uy xy, a1_13 = 3 (uy^2 xy + ux uy yy), a1_04 = 6 uy^2 yy
    constexpr bool r3 = ORDER >= 3, r4 = ORDER >= 4;
    constexpr double cxx_x = r3 ? 3.0 * h30 : 0.0, cxx_y = r3 ? h21 : 0.0;
    constexpr double cxy_x = r3 ? 2.0 * h21 : 0.0, cxy_y = r3 ? 2.0 * h12 : 0.0;
    constexpr double cyy_x = r3 ? h12 : 0.0, cyy_y = r3 ? 3.0 * h03 : 0.0;
    constexpr double cxx_x2 = r4 ? 6.0 * h40 : 0.0, cxx_xy = r4 ? 3.0 * h31 : 0.0, cxx_y2 = r4 ? h22 : 0.0;
    constexpr double cxy_x2 = r4 ? 3.0 * h31 : 0.0, cxy_xy = r4 ? 4.0 * h22 : 0.0, cxy_y2 = r4 ? 3.0 * h13 : 0.0;
    constexpr double cyy_x2 = r4 ? h22 : 0.0, cyy_xy = r4 ? 3.0 * h13 : 0.0, cyy_y2 = r4 ? 6.0 * h04 : 0.0;
    // per a1 component: k2 c2 + k3 (c_x ux + c_y uy) + k4 (c_x2 x2 + c_xy xy + c_y2 y2)
    double n = 0.0;
    {
        double c = 0.0, p3 = 0.0, p4 = 0.0;
        if constexpr (h20 != 0.0) c += (PO ? rx.k2 : 1.0) * h20;
        if constexpr (cxx_x != 0.0) p3 += cxx_x * ux;
        if constexpr (cxx_y != 0.0) p3 += cxx_y * uy;
        if constexpr (cxx_x2 != 0.0) p4 += cxx_x2 * x2;
        if constexpr (cxx_xy != 0.0) p4 += cxx_xy * xy;
        if constexpr (cxx_y2 != 0.0) p4 += cxx_y2 * y2;
        if constexpr (cxx_x != 0.0 || cxx_y != 0.0) c += PO ? rx.k3 * p3 : p3;
        if constexpr (cxx_x2 != 0.0 || cxx_xy != 0.0 || cxx_y2 != 0.0) c += PO ? rx.k4 * p4 : p4;
        n += c * axx;
    }
    {
        double c = 0.0, p3 = 0.0, p4 = 0.0;
        if constexpr (h11 != 0.0) c += (PO ? rx.k2 : 1.0) * h11;
        if constexpr (cxy_x != 0.0) p3 += cxy_x * ux;
        if constexpr (cxy_y != 0.0) p3 += cxy_y * uy;
        if constexpr (cxy_x2 != 0.0) p4 += cxy_x2 * x2;
        if constexpr (cxy_xy != 0.0) p4 += cxy_xy * xy;
        if constexpr (cxy_y2 != 0.0) p4 += cxy_y2 * y2;
        if constexpr (cxy_x != 0.0 || cxy_y != 0.0) c += PO ? rx.k3 * p3 : p3;
        if constexpr (cxy_x2 != 0.0 || cxy_xy != 0.0 || cxy_y2 != 0.0) c += PO ? rx.k4 * p4 : p4;
        n += c * axy;
    }
    {
        double c = 0.0, p3 = 0.0, p4 = 0.0;
        if constexpr (h02 != 0.0) c += (PO ? rx.k2 : 1.0) * h02;
        if constexpr (cyy_x != 0.0) p3 += cyy_x * ux;
        if constexpr (cyy_y != 0.0) p3 += cyy_y * uy;
        if constexpr (cyy_x2 != 0.0) p4 += cyy_x2 * x2;
        if constexpr (cyy_xy != 0.0) p4 += cyy_xy * xy;
        if constexpr (cyy_y2 != 0.0) p4 += cyy_y2 * y2;
        if constexpr (cyy_x != 0.0 || cyy_y != 0.0) c += PO ? rx.k3 * p3 : p3;
        if constexpr (cyy_x2 != 0.0 || cyy_xy != 0.0 || cyy_y2 != 0.0) c += PO ? rx.k4 * p4 : p4;
        n += c * ayy;
    }
    constexpr double w = L::v.w[I];
    return PO ? w * (r * e + n) : w * (r * e + rx.k2 * n);
}

// Moments (rho, ux, uy, a1^(2)) of the populations v of one node.
template <class L>
__device__ __forceinline__ void node_state(const double (&v)[L::Q], double (&m)[MOM_K])
{
    double r = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
    static_for<L::Q>([&](auto I) {
        constexpr double cx = L::v.cx[I], cy = L::v.cy[I];
        r += v[I];
        jx += cx * v[I];
        jy += cy * v[I];
        pxx += cx * cx * v[I];
        pxy += cx * cy * v[I];
        pyy += cy * cy * v[I];
    });
    const double ux = jx / r, uy = jy / r;
    m[0] = r;
    m[1] = ux;
    m[2] = uy;
    m[3] = pxx - r * L::cs2 - r * ux * ux;
    m[4] = pxy - r * ux * uy;
    m[5] = pyy - r * L::cs2 - r * uy * uy;
}

// One step on a BX x BY tile: the tile's moments and a halo of the lattice
// reach are staged in LDS (periodic wrap), each thread pulls its Q
// populations from there and writes its node's new moments.
template <class L, int ORDER, bool PO>
__global__ __launch_bounds__(BX* BY) void k_mom_step(const double* __restrict__ min, double* __restrict__ mout, int nx,
                                                     int ny, int bx_blocks, Relax rx)
{
    constexpr int R = L::R, TW = BX + 2 * R, TH = BY + 2 * R;
    __shared__ double sm[MOM_K][TH][TW];
    const int x0 = int(blockIdx.x % unsigned(bx_blocks)) * BX;
    const int y0 = int(blockIdx.x / unsigned(bx_blocks)) * BY;
    const int64_t n = int64_t(nx) * ny;
    const int tid = int(threadIdx.y) * BX + int(threadIdx.x);
    // the staged window covers columns x0 - R .. x0 + BX + R - 1: one wrap at
    // most when the grid is at least that wide, a modulo otherwise
    const bool wide = nx >= TW && ny >= TH;
    for (int e = tid; e < TH * TW; e += BX * BY) {
        const int ly = e / TW, lx = e - ly * TW;
        int gx = x0 + lx - R, gy = y0 + ly - R;
        if (wide) {
            gx += gx < 0 ? nx : 0;
            gx -= gx >= nx ? nx : 0;
            gy += gy < 0 ? ny : 0;
            gy -= gy >= ny ? ny : 0;
        } else {
            gx = ((gx % nx) + nx) % nx;
            gy = ((gy % ny) + ny) % ny;
        }
        const int64_t g = int64_t(gy) * nx + gx;
        static_for<MOM_K>([&](auto M) { sm[M][ly][lx] = min[int64_t(M) * n + g]; });
    }
    __syncthreads();
    const int x = x0 + int(threadIdx.x), y = y0 + int(threadIdx.y);
    if (x >= nx || y >= ny) return;
    // accumulate the moments of the arriving populations one at a time
    double r = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        const int ly = int(threadIdx.y) + R - cy, lx = int(threadIdx.x) + R - cx;
        const double f = mom_pop<L, int(I), ORDER, PO>(sm[0][ly][lx], sm[1][ly][lx], sm[2][ly][lx], sm[3][ly][lx],
                                                   sm[4][ly][lx], sm[5][ly][lx], rx);
        r += f;
        if constexpr (cx != 0) jx += double(cx) * f;
        if constexpr (cy != 0) jy += double(cy) * f;
        if constexpr (cx != 0) pxx += double(cx * cx) * f;
        if constexpr (cx != 0 && cy != 0) pxy += double(cx * cy) * f;
        if constexpr (cy != 0) pyy += double(cy * cy) * f;
    });
    const double ux = jx / r, uy = jy / r;
    const double m[MOM_K] = { r, ux, uy, pxx - r * L::cs2 - r * ux * ux, pxy - r * ux * uy,
                              pyy - r * L::cs2 - r * uy * uy };
    const int64_t here = int64_t(y) * nx + x;
    static_for<MOM_K>([&](auto M) { __builtin_nontemporal_store(m[M], mout + int64_t(M) * n + here); });
}

// Initial state: the moments of f^(0) [+ f^(1)] + noise (the populations the
// population form starts from, before its first collision).
template <class L>
__global__ __launch_bounds__(256) void k_mom_init(InitArgs a)
{
    const int64_t n = int64_t(a.lay.nx) * a.lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f[L::Q];
    equilibrium_node<L, double, false>(a.rho[k], a.ux[k], a.uy[k], 1.0, a.eq_order, f);
    if (a.grad) {
        const double du[2][2] = { { a.grad[k], a.grad[2 * n + k] }, { a.grad[n + k], a.grad[3 * n + k] } };
        double f1[L::Q];
        noneq_init_node<L, double>(a.rho[k], a.ux[k], a.uy[k], du, a.tau, a.eq_order, f1);
        static_for<L::Q>([&](auto I) { f[I] += f1[I]; });
    }
    if (a.noise) static_for<L::Q>([&](auto I) { f[I] += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k]; });
    double m[MOM_K];
    node_state<L>(f, m);
    double* out = static_cast<double*>(a.f);
    static_for<MOM_K>([&](auto M) { out[int64_t(M) * n + k] = m[M]; });
}

// Post-collision populations of node k (what the population form stores).
template <class L, int ORDER>
__device__ __forceinline__ void mom_node_populations(const double* __restrict__ m, int64_t n, int64_t k,
                                                     const Relax& rx, double (&v)[L::Q])
{
    const double r = m[k], ux = m[n + k], uy = m[2 * n + k];
    const double axx = m[3 * n + k], axy = m[4 * n + k], ayy = m[5 * n + k];
    static_for<L::Q>([&](auto I) { v[I] = mom_pop<L, int(I), ORDER, true>(r, ux, uy, axx, axy, ayy, rx); });
}

} // namespace rr
