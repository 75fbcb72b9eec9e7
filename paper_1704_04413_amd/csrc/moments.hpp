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
//
// Thermal form (D2V37, App. C): the collision reads the pre-collision
// populations only through their raw moments of order up to three (rho, u,
// theta from orders 0-2, a1^(2) by projection, a1^(3) from the projected
// third moments and the gradient estimates, a1^(4) by the recursion).  The
// state is what that gives before rank 4: planes m = rho, ux, uy,
// sig = (theta - 1) c_s^2, a1_xx, a1_xy, a1_yy, a1_xxx, a1_xxy, a1_xyy,
// a1_yyy, computed once per node from its gathered raw moments; every pull
// then rebuilds only the equilibrium and rank 4.
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

// ------------------------------------------------------------- the step
//
// The step works by velocity rows.  Every velocity with c_y = K pulls from
// the row y - K, so the populations of that class that a row of outputs needs
// were all produced on one source row, each at the source column x - c_x.  One
// pass per class: each thread rebuilds, at its source node, the node's
// coefficients
//   C[a][b] = r u_x^a u_y^b + k_n a1^(a,b)    (n = a + b),
// with a1^(3), a1^(4) from u and a1^(2) (Eq. MalaspinasRecursiveRelation at
// theta = 1), contracts them with the class's c_y factor once,
//   t[a] = sum_b He_b(K) C[a][b] / (a! b! c_s^2(a+b)),
// and gets every population (c_x, K) of the class as w sum_a He_a(c_x) t[a]
// (c_x and -c_x from one even and one odd part: Eq. GenRegCollision).  The
// population (c_x, K) computed at source lane l is the one the output lane
// l + c_x pulls, so a wave moves it c_x lanes with cross-lane moves and adds
// it to that output's moment sums.  Per node that is 2R+1 coefficient builds
// instead of Q (one per pulled population), and the c_y part of the Hermite
// products is shared by a whole class.
//
// A block is one 64-wide segment of source columns by MOM_ROWS rows, one wave
// per row; its outputs are the 64 - 2R inner columns (the outer R on each side
// are the x halo of the pulls).  The moments of the rows the block reads
// (its own and R above and below) are staged in LDS once.

constexpr int MOM_ROWS = 16;

// Coefficients C of a node with moments (r, u, a1^(2)) (see above); entries
// outside the lattice basis are never read.
template <class L, int ORDER, bool PO>
__device__ __forceinline__ void mom_coeffs(double r, double ux, double uy, double axx, double axy, double ayy,
                                           const Relax& rx, double (&C)[5][5])
{
    const double k2 = rx.k2, k3 = PO ? rx.k3 : rx.k2, k4 = PO ? rx.k4 : rx.k2;
    const double rux = r * ux, ruy = r * uy;
    const double rxx = rux * ux, rxy = rux * uy, ryy = ruy * uy;
    C[0][0] = r;
    C[1][0] = rux;
    C[0][1] = ruy;
    C[2][0] = rxx + k2 * axx;
    C[1][1] = rxy + k2 * axy;
    C[0][2] = ryy + k2 * ayy;
    // rank 3: a1_30 = 3 ux xx, a1_21 = 2 ux xy + uy xx, a1_12 = 2 uy xy + ux yy, a1_03 = 3 uy yy
    if constexpr (ORDER >= 3) {
        const double bxx = k3 * axx, bxy = k3 * axy, byy = k3 * ayy;
        C[3][0] = ux * (rxx + 3.0 * bxx);
        C[2][1] = uy * (rxx + bxx) + 2.0 * ux * bxy;
        C[1][2] = ux * (ryy + byy) + 2.0 * uy * bxy;
        C[0][3] = uy * (ryy + 3.0 * byy);
    } else {
        C[3][0] = ux * rxx;
        C[2][1] = uy * rxx;
        C[1][2] = ux * ryy;
        C[0][3] = uy * ryy;
    }
    // rank 4: a1_40 = 6 ux^2 xx, a1_31 = 3 (ux^2 xy + ux uy xx),
    //         a1_22 = uy^2 xx + ux^2 yy + 4 ux uy xy, a1_13 = 3 (uy^2 xy + ux uy yy), a1_04 = 6 uy^2 yy
    const double x2 = ux * ux, xy = ux * uy, y2 = uy * uy;
    if constexpr (ORDER >= 4) {
        const double cxx = k4 * axx, cxy = k4 * axy, cyy = k4 * ayy;
        C[4][0] = x2 * (rxx + 6.0 * cxx);
        C[3][1] = ux * (uy * (rxx + 3.0 * cxx) + 3.0 * ux * cxy);
        C[2][2] = y2 * (rxx + cxx) + x2 * cyy + 4.0 * xy * cxy;
        C[1][3] = uy * (ux * (ryy + 3.0 * cyy) + 3.0 * uy * cxy);
        C[0][4] = y2 * (ryy + 6.0 * cyy);
    } else {
        C[4][0] = x2 * rxx;
        C[3][1] = xy * rxx;
        C[2][2] = y2 * rxx;
        C[1][3] = xy * ryy;
        C[0][4] = y2 * ryy;
    }
}

// Whether t[a] of class K has any term.
template <class L>
constexpr bool class_col(int a, int k)
{
    for (int b = 0; b < 5; ++b)
        if (L::basis(a, b) && he(b, double(k), L::cs2) != 0.0) return true;
    return false;
}

// Post-collision populations of the velocities (c_x, K) of a node with
// coefficients C: emit(c_x, f) for each (c_x as a compile-time constant).
template <class L, int K, class Emit>
__device__ __forceinline__ void class_pops(const double (&C)[5][5], Emit&& emit)
{
    constexpr double cs2 = L::cs2;
    double t[5];
    static_for<5>([&](auto A) {
        double s = 0.0;
        static_for<5>([&](auto B) {
            if constexpr (L::basis(int(A), int(B))) {
                constexpr double h = he(int(B), double(K), cs2) * inv_norm<L>(int(A), int(B));
                if constexpr (h != 0.0) s += h * C[A][B];
            }
        });
        t[A] = s;
    });
    static_for<L::R + 1>([&](auto XI) {
        constexpr int cx = int(XI);
        constexpr int ip = vel_index<L>(cx, K);
        if constexpr (ip >= 0) {
            constexpr double w = L::v.w[ip];
            double e = 0.0, o = 0.0;
            static_for<5>([&](auto A) {
                constexpr double h = w * he(int(A), double(cx), cs2);
                if constexpr (class_col<L>(int(A), K) && h != 0.0) {
                    if constexpr (int(A) % 2 == 0)
                        e += h * t[A];
                    else
                        o += h * t[A];
                }
            });
            if constexpr (cx == 0) {
                emit(std::integral_constant<int, 0>{}, e);
            } else {
                emit(std::integral_constant<int, cx>{}, e + o);
                emit(std::integral_constant<int, -cx>{}, e - o);
            }
        }
    });
}

// Number of velocities with c_y = k.
template <class L>
constexpr int class_size(int k)
{
    int c = 0;
    for (int i = 0; i < L::Q; ++i) c += L::v.cy[i] == k ? 1 : 0;
    return c;
}

// Populations of class K at a node with moments m: through the coefficients
// when the class has three velocities or more, otherwise one at a time
// (mom_pop), which is cheaper for one or two.
template <class L, int K, int ORDER, bool PO, class Emit>
__device__ __forceinline__ void class_from_moments(const double (&m)[MOM_K], const Relax& rx, Emit&& emit)
{
    if constexpr (class_size<L>(K) >= 3) {
        double C[5][5];
        mom_coeffs<L, ORDER, PO>(m[0], m[1], m[2], m[3], m[4], m[5], rx, C);
        class_pops<L, K>(C, emit);
    } else {
        static_for<2 * L::R + 1>([&](auto XI) {
            constexpr int cx = int(XI) - L::R;
            constexpr int ip = vel_index<L>(cx, K);
            if constexpr (ip >= 0)
                emit(std::integral_constant<int, cx>{},
                     mom_pop<L, ip, ORDER, PO>(m[0], m[1], m[2], m[3], m[4], m[5], rx));
        });
    }
}

// Exponents (p, q) of the raw moments a thermal step gathers (p + q <= 3);
// the first six are the isothermal step's.
constexpr int TH_NS = 10;
constexpr int TH_P[TH_NS] = { 0, 1, 0, 2, 1, 0, 3, 2, 1, 0 };
constexpr int TH_Q[TH_NS] = { 0, 0, 1, 0, 1, 2, 0, 1, 2, 3 };

// Thermal state of a node from its raw moments: the population form's steps
// 2-4 (coeffs_from_moments), kept up to rank 3.
template <class L, bool A13P>
__device__ __forceinline__ void thermal_state(const double (&sums)[TH_NS], double (&m)[MOM_KT])
{
    double s[5][5];
    static_for<5>([&](auto a) { static_for<5>([&](auto b) { s[a][b] = 0.0; }); });
    static_for<TH_NS>([&](auto M) { s[TH_P[M]][TH_Q[M]] = sums[M]; });
    NodeCoeffs<double> k;
    coeffs_from_moments<L, double, COLL_RR, true, false, A13P>(s, k);
    const double out[MOM_KT] = { k.rho,      k.ux,       k.uy,       k.sig,      k.a1[2][0], k.a1[1][1],
                                 k.a1[0][2], k.a1[3][0], k.a1[2][1], k.a1[1][2], k.a1[0][3] };
    static_for<MOM_KT>([&](auto M) { m[M] = out[M]; });
}

// Coefficients C[a][b] = a0 + k_n a1 of rank n of a node in the thermal
// state m: the equilibrium with theta, a1^(4) by the thermal recursion, the
// factors k_n zero above the regularization order.
template <class L>
__device__ __forceinline__ void thermal_coeffs(const double (&m)[MOM_KT], const Relax& rx, double (&C)[5][5])
{
    const double ux = m[1], uy = m[2], sig = m[3];
    eq_coeffs<L, double>(m[0], ux, uy, sig, C);
    double a1[5][5];
    a1[2][0] = m[4];
    a1[1][1] = m[5];
    a1[0][2] = m[6];
    a1[3][0] = m[7];
    a1[2][1] = m[8];
    a1[1][2] = m[9];
    a1[0][3] = m[10];
    thermal_rank4<double>(ux, uy, sig, a1);
    static_for<5>([&](auto A) {
        static_for<5>([&](auto B) {
            constexpr int r = int(A) + int(B);
            if constexpr (L::basis(int(A), int(B)) && r >= 2) {
                const double kr = r == 2 ? rx.k2 : r == 3 ? rx.k3 : rx.k4;
                C[A][B] += kr * a1[A][B];
            }
        });
    });
}

// Makes the values materialise here (an empty asm that reads and writes
// them): code that computes them cannot be moved past this point.
template <int N>
__device__ __forceinline__ void pin(double (&a)[N])
{
    static_assert(N == 6 || N == 10, "six or ten sums");
    if constexpr (N == 6)
        asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]));
    else
        asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),
                     "+v"(a[7]), "+v"(a[8]), "+v"(a[9]));
}

// Value of v held by lane (lane - D) of the wave (D in [-3, 3]), by |D|
// one-lane wave shifts of both halves (DPP wave_shr:1 / wave_shl:1); lanes
// whose source is outside the wave get zero.
template <int D>
__device__ __forceinline__ double lane_from(double v)
{
    if constexpr (D == 0) {
        return v;
    } else {
        const long long b = __double_as_longlong(v);
        int lo = int(b), hi = int(b >> 32);
        constexpr int ctrl = D > 0 ? 0x138 : 0x130;
        static_for<(D > 0 ? D : -D)>([&](auto) {
            lo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xF, 0xF, true);
            hi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xF, 0xF, true);
        });
        return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
    }
}

// Isothermal form: eight waves per SIMD (64 VGPRs), and the 67.6 KB of staged
// moments of a 16-row block let two blocks share a CU.  Thermal form (TH):
// eleven staged planes, 123.9 KB, one block and four waves per SIMD.  The
// moments gathered at a node are its raw sums s_pq (p + q <= 2, or 3 for the
// thermal state), in the order of TH_P / TH_Q.
template <class L, int ORDER, bool PO, bool TH = false, bool A13P = false>
__global__ __launch_bounds__(BX* MOM_ROWS) __attribute__((amdgpu_waves_per_eu(TH ? 4 : 8))) void k_mom_step(
    const double* __restrict__ min, double* __restrict__ mout, int nx, int ny, int bx_blocks, Relax rx)
{
    constexpr int R = L::R, OX = BX - 2 * R, SH = MOM_ROWS + 2 * R, NC = 2 * R + 1;
    constexpr int NV = TH ? MOM_KT : MOM_K, NA = TH ? TH_NS : MOM_K, PMAX = TH ? 3 : 2;
    __shared__ double sm[NV][SH][BX];
    const int x0 = int(blockIdx.x % unsigned(bx_blocks)) * OX;
    const int y0 = int(blockIdx.x / unsigned(bx_blocks)) * MOM_ROWS;
    const int64_t n = int64_t(nx) * ny;
    const int lane = int(threadIdx.x), ty = int(threadIdx.y);
    // stage source columns x0 - R .. x0 - R + 63, rows y0 - R .. y0 + MOM_ROWS
    // + R - 1 (periodic: one wrap at most when the grid is at least that
    // large, a modulo otherwise)
    const bool wide = nx >= BX && ny >= SH;
    for (int e = ty * BX + lane; e < SH * BX; e += BX * MOM_ROWS) {
        const int ly = e / BX, lx = e - ly * BX;
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
        static_for<NV>([&](auto M) { sm[M][ly][lx] = min[int64_t(M) * n + g]; });
    }
    __syncthreads();
    const int x = x0 + lane - R, y = y0 + ty;
    double acc[NA];
    static_for<NA>([&](auto M) { acc[M] = 0.0; });
    static_for<NC>([&](auto KI) {
        constexpr int K = int(KI) - R;
        double mv[NV];
        static_for<NV>([&](auto M) { mv[M] = sm[M][ty - K + R][lane]; });
        // row sums of the class at this lane, rs[p] = sum c_x^p f over the
        // populations (c_x, K) arriving here
        double rs[PMAX + 1];
        static_for<PMAX + 1>([&](auto P) { rs[P] = 0.0; });
        auto add = [&](auto CX, double f) {
            constexpr int cx = decltype(CX)::value;
            const double g = lane_from<cx>(f);
            rs[0] += g;
            if constexpr (cx != 0)
                static_for<PMAX>([&](auto P) {
                    constexpr double cp = ipow(double(cx), int(P) + 1);
                    rs[int(P) + 1] += cp * g;
                });
        };
        if constexpr (TH) {
            double C[5][5];
            thermal_coeffs<L>(mv, rx, C);
            class_pops<L, K>(C, add);
        } else {
            class_from_moments<L, K, ORDER, PO>(mv, rx, add);
        }
        static_for<NA>([&](auto S) {
            constexpr int p = TH_P[S], q = TH_Q[S];
            constexpr double kq = ipow(double(K), q);
            if constexpr (q == 0)
                acc[S] += rs[p];
            else if constexpr (K != 0)
                acc[S] += kq * rs[p];
        });
        // one class at a time: the sums are taken here (not sunk to the end
        // with every class's row sums kept alive), and the scheduler does not
        // interleave classes
        pin(acc);
        __builtin_amdgcn_sched_barrier(0);
    });
    if (lane < R || lane >= BX - R || x >= nx || y >= ny) return;
    const int64_t here = int64_t(y) * nx + x;
    if constexpr (TH) {
        double m[MOM_KT];
        thermal_state<L, A13P>(acc, m);
        static_for<MOM_KT>([&](auto M) { __builtin_nontemporal_store(m[M], mout + int64_t(M) * n + here); });
    } else {
        const double r = acc[0], jx = acc[1], jy = acc[2], pxx = acc[3], pxy = acc[4], pyy = acc[5];
        const double ux = jx / r, uy = jy / r;
        const double m[MOM_K] = { r, ux, uy, pxx - r * L::cs2 - r * ux * ux, pxy - r * ux * uy,
                                  pyy - r * L::cs2 - r * uy * uy };
        static_for<MOM_K>([&](auto M) { __builtin_nontemporal_store(m[M], mout + int64_t(M) * n + here); });
    }
}

// Initial state: the moments of f^(0) [+ f^(1)] + noise (the populations the
// population form starts from, before its first collision).
template <class L, bool TH = false, bool A13P = false>
__global__ __launch_bounds__(256) void k_mom_init(InitArgs a)
{
    const int64_t n = int64_t(a.lay.nx) * a.lay.ny;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f[L::Q];
    equilibrium_node<L, double, false>(a.rho[k], a.ux[k], a.uy[k], TH ? a.theta[k] : 1.0, a.eq_order, f);
    if (a.grad) {
        const double du[2][2] = { { a.grad[k], a.grad[2 * n + k] }, { a.grad[n + k], a.grad[3 * n + k] } };
        double f1[L::Q];
        noneq_init_node<L, double>(a.rho[k], a.ux[k], a.uy[k], du, a.tau, a.eq_order, f1);
        static_for<L::Q>([&](auto I) { f[I] += f1[I]; });
    }
    if (a.noise) static_for<L::Q>([&](auto I) { f[I] += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k]; });
    double* out = static_cast<double*>(a.f);
    if constexpr (TH) {
        double sums[TH_NS], m[MOM_KT];
        static_for<TH_NS>([&](auto M) {
            double sum = 0.0;
            static_for<L::Q>([&](auto I) {
                constexpr double c = ipow(double(L::v.cx[I]), TH_P[M]) * ipow(double(L::v.cy[I]), TH_Q[M]);
                sum += c * f[I];
            });
            sums[M] = sum;
        });
        thermal_state<L, A13P>(sums, m);
        static_for<MOM_KT>([&](auto M) { out[int64_t(M) * n + k] = m[M]; });
    } else {
        double m[MOM_K];
        node_state<L>(f, m);
        static_for<MOM_K>([&](auto M) { out[int64_t(M) * n + k] = m[M]; });
    }
}

// Post-collision populations of node k (what the population form stores).
template <class L, int ORDER, bool TH = false, bool A13P = false>
__device__ __forceinline__ void mom_node_populations(const double* __restrict__ m, int64_t n, int64_t k,
                                                     const Relax& rx, double (&v)[L::Q])
{
    if constexpr (TH) {
        double mv[MOM_KT], C[5][5];
        static_for<MOM_KT>([&](auto M) { mv[M] = m[int64_t(M) * n + k]; });
        thermal_coeffs<L>(mv, rx, C);
        static_for<5>([&](auto A) {
            static_for<5>([&](auto B) {
                if constexpr (L::basis(int(A), int(B))) {
                    constexpr double nrm = inv_norm<L>(int(A), int(B));
                    C[A][B] *= nrm;
                }
            });
        });
        reconstruct<L, double>(C, v);
    } else {
        const double r = m[k], ux = m[n + k], uy = m[2 * n + k];
        const double axx = m[3 * n + k], axy = m[4 * n + k], ayy = m[5 * n + k];
        static_for<L::Q>([&](auto I) { v[I] = mom_pop<L, int(I), ORDER, true>(r, ux, uy, axx, axy, ayy, rx); });
    }
}

} // namespace rr
