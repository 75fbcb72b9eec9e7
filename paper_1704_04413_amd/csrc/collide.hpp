// Per-node regularized collision for the HIP kernels.
//
// The node state is held in registers as v[Q], either the plain populations f
// (FP64 storage) or the weight-shifted g = f - w (FP32/BF16 storage).  The
// collision follows the paper's regularized operator (Eq. RegularizedCollision
// with a single tau):
//   1. moments rho, j and the Hermite moments h_k = sum_i H^k_i v_i
//      (sum_i w_i H^k_i = 0 for every basis tensor k != 0, so h_k is the same
//      for f and g);
//   2. theta from the energy moment (thermal) and the equilibrium
//      coefficients a0^(kx,ky) = rho m_kx(ux) m_ky(uy), m_n the raw moments of
//      N(u, (theta-1) c_s^2) -- the closed form of Eq. HermiteCoeffEq, equal to
//      the recursion of App. B;
//   3. a1^(2) = h^(2) - a0^(2) (Eq. a12Proj; exact because the quadrature
//      reproduces sum_i H^(2)_i f^(0)_i = a0^(2) on all three lattices);
//   4. a1^(3), a1^(4): isothermal closed forms of Eq. MalaspinasRecursiveRelation
//      (App. C at theta = 1), or the thermal path of App. C (project a1^(3),
//      average the two estimates of mu c_s^2 grad theta, Eq. TempGradLBM,
//      rebuild with Eq. a1Rec, then the rank-4 forms of the thermal recursion);
//      PR projects every rank instead (h_k - a0_k);
//   5. f_coll_i = w_i sum_k H^k_i [a0^k + (1 - 1/tau) a1^k] / (k_x! k_y! c_s^2|k|)
//      over the lattice basis (Eq. GenRegCollision), a1 kept for ranks 2..N.
// Moments and reconstruction are organised by velocity rows (one row per c_y)
// and by +/- pairs, using H^k_i = He_kx(c_x) He_ky(c_y) (App. C, 2D).
#pragma once

#include "common.hpp"
#include "lattices.hpp"

namespace rr {

// Row moments: r[cy + R][p] = sum over velocities of row c_y of v_i c_x^p, and
// then s[p][q] = sum_i v_i c_x^p c_y^q for p + q <= 4.
template <class L, class T>
__device__ __forceinline__ void raw_moments(const T (&v)[L::Q], T (&s)[5][5])
{
    constexpr int R = L::R;
    T r[2 * R + 1][5];
    static_for<2 * R + 1>([&](auto YI) {
        constexpr int cy = int(YI) - R;
        constexpr int i0 = vel_index<L>(0, cy);
        static_for<5>([&](auto P) { r[YI][P] = T(0); });
        if constexpr (i0 >= 0) r[YI][0] = v[i0];
        static_for<R>([&](auto XI) {
            constexpr int cx = int(XI) + 1;
            constexpr int ip = vel_index<L>(cx, cy), im = vel_index<L>(-cx, cy);
            if constexpr (ip >= 0) {
                static_assert(im >= 0, "lattice rows are symmetric");
                const T e = v[ip] + v[im];
                const T o = v[ip] - v[im];
                r[YI][0] += e;
                r[YI][1] += T(cx) * o;
                r[YI][2] += T(cx * cx) * e;
                r[YI][3] += T(cx * cx * cx) * o;
                r[YI][4] += T(cx * cx * cx * cx) * e;
            }
        });
    });
    static_for<5>([&](auto P) {
        T re[R + 1], ro[R + 1];
        static_for<R>([&](auto YI) {
            constexpr int cy = int(YI) + 1;
            re[cy] = r[R + cy][P] + r[R - cy][P];
            ro[cy] = r[R + cy][P] - r[R - cy][P];
        });
        static_for<5 - int(P)>([&](auto Qd) {
            T acc = (int(Qd) == 0) ? r[R][P] : T(0);
            static_for<R>([&](auto YI) {
                constexpr int cy = int(YI) + 1;
                constexpr double m = ipow(double(cy), int(Qd));
                acc += T(m) * ((int(Qd) % 2 == 0) ? re[cy] : ro[cy]);
            });
            s[P][Qd] = acc;
        });
    });
}

// emit(i, w_i sum_{kx,ky in basis} He_kx(c_x) He_ky(c_y) C[kx][ky]) for every
// velocity i (i as a compile-time constant), row by row.
template <class L, class T, class Emit>
__device__ __forceinline__ void reconstruct_emit(const T (&C)[5][5], Emit&& emit)
{
    constexpr int R = L::R;
    constexpr double cs2 = L::cs2;
    static_for<R + 1>([&](auto YI) {
        constexpr int cy = int(YI);
        // T_kx(+-cy) = te_kx +- to_kx with te (to) the even (odd) ky part
        T te[5], to[5];
        static_for<5>([&](auto KX) {
            T e = T(0), o = T(0);
            static_for<5>([&](auto KY) {
                if constexpr (L::basis(int(KX), int(KY))) {
                    constexpr double h = he(int(KY), double(cy), cs2);
                    if constexpr (int(KY) % 2 == 0)
                        e += T(h) * C[KX][KY];
                    else
                        o += T(h) * C[KX][KY];
                }
            });
            te[KX] = e;
            to[KX] = o;
        });
        static_for<(cy == 0) ? 1 : 2>([&](auto SY) {
            constexpr int yy = (int(SY) == 0) ? cy : -cy;
            T t[5];
            static_for<5>([&](auto KX) { t[KX] = (int(SY) == 0) ? te[KX] + to[KX] : te[KX] - to[KX]; });
            static_for<R + 1>([&](auto XI) {
                constexpr int cx = int(XI);
                constexpr int ip = vel_index<L>(cx, yy), im = vel_index<L>(-cx, yy);
                if constexpr (ip >= 0) {
                    T e = T(0), o = T(0);
                    static_for<5>([&](auto KX) {
                        constexpr double h = he(int(KX), double(cx), cs2);
                        if constexpr (h != 0.0) {
                            if constexpr (int(KX) % 2 == 0)
                                e += T(h) * t[KX];
                            else
                                o += T(h) * t[KX];
                        }
                    });
                    constexpr double w = L::v.w[ip];
                    emit(std::integral_constant<int, ip>{}, T(w) * (e + o));
                    if constexpr (cx != 0) emit(std::integral_constant<int, im>{}, T(w) * (e - o));
                }
            });
        });
    });
}

// out_i = w_i sum_{kx,ky in basis} He_kx(c_x) He_ky(c_y) C[kx][ky].
template <class L, class T>
__device__ __forceinline__ void reconstruct(const T (&C)[5][5], T (&out)[L::Q])
{
    reconstruct_emit<L, T>(C, [&](auto I, T val) { out[I] = val; });
}

// Coefficient C[kx][ky] = value / (kx! ky! c_s^2(kx+ky)) restricted to the basis.
template <class L, class T>
__device__ __forceinline__ void zero_coeffs(T (&C)[5][5])
{
    static_for<5>([&](auto a) { static_for<5>([&](auto b) { C[a][b] = T(0); }); });
}

// Equilibrium coefficients a0[kx][ky] = rho m_kx(ux) m_ky(uy).
template <class T>
__device__ __forceinline__ void eq_factors(T u, T sig, T (&m)[5])
{
    const T u2 = u * u;
    m[0] = T(1);
    m[1] = u;
    m[2] = u2 + sig;
    m[3] = u * (u2 + T(3) * sig);
    m[4] = u2 * u2 + T(6) * sig * u2 + T(3) * sig * sig;
}

// Moments, equilibrium and non-equilibrium Hermite coefficients of one node
// (steps 1-4 above).  C holds a0 (not yet normalised), a1 the
// non-equilibrium coefficients before truncation.
template <class T>
struct NodeCoeffs {
    T rho, drho, ux, uy, sig;
    T C[5][5];
    T a1[5][5];
};

// Isothermal recursion (Eq. MalaspinasRecursiveRelation at theta = 1, in the
// 2D closed forms of App. C): a1^(3), a1^(4) from u and a1^(2).
template <class T>
__device__ __forceinline__ void iso_recursion(T ux, T uy, T (&a1)[5][5])
{
    const T xx = a1[2][0], xy = a1[1][1], yy = a1[0][2];
    const T uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    a1[3][0] = T(3) * ux * xx;
    a1[2][1] = T(2) * ux * xy + uy * xx;
    a1[1][2] = T(2) * uy * xy + ux * yy;
    a1[0][3] = T(3) * uy * yy;
    a1[4][0] = T(6) * uxx * xx;
    a1[3][1] = T(3) * (uxx * xy + uxy * xx);
    a1[2][2] = uyy * xx + uxx * yy + T(4) * uxy * xy;
    a1[1][3] = T(3) * (uyy * xy + uxy * yy);
    a1[0][4] = T(6) * uyy * yy;
}

// Equilibrium coefficients C[kx][ky] = rho m_kx(ux) m_ky(uy) over the basis
// (not yet normalised; C[0][0] = rho, entries off the basis zero).
template <class L, class T>
__device__ __forceinline__ void eq_coeffs(T rho, T ux, T uy, T sig, T (&C)[5][5])
{
    T mx[5], my[5];
    eq_factors<T>(ux, sig, mx);
    eq_factors<T>(uy, sig, my);
    zero_coeffs<L, T>(C);
    static_for<5>([&](auto KX) {
        static_for<5>([&](auto KY) {
            if constexpr (L::basis(int(KX), int(KY)) && int(KX) + int(KY) >= 1) C[KX][KY] = rho * mx[KX] * my[KY];
        });
    });
    C[0][0] = rho;
}

// Rank 4 of the thermal recursion (App. C) from a1^(2), a1^(3), u and
// sig = (theta - 1) c_s^2.
template <class T>
__device__ __forceinline__ void thermal_rank4(T ux, T uy, T sig, T (&a1)[5][5])
{
    const T xx = a1[2][0], xy = a1[1][1], yy = a1[0][2];
    const T bx = sig - ux * ux, by = sig - uy * uy, uxy = ux * uy;
    a1[4][0] = T(4) * ux * a1[3][0] + T(6) * bx * xx;
    a1[3][1] = T(3) * ux * a1[2][1] + uy * a1[3][0] + T(3) * bx * xy - T(3) * uxy * xx;
    a1[2][2] = T(2) * (ux * a1[1][2] + uy * a1[2][1]) + bx * yy + by * xx - T(4) * uxy * xy;
    a1[1][3] = T(3) * uy * a1[1][2] + ux * a1[0][3] + T(3) * by * xy - T(3) * uxy * yy;
    a1[0][4] = T(4) * uy * a1[0][3] + T(6) * by * yy;
}

// Steps 2-4 from the raw moments s[p][q] = sum_i v_i c_x^p c_y^q (orders up
// to 2 for BGK, 3 for the thermal path, 4 for PR of rank 4).
template <class L, class T, int COLL, bool THERMAL, bool SHIFTED, bool A13P>
__device__ __forceinline__ void coeffs_from_moments(const T (&s)[5][5], NodeCoeffs<T>& k)
{
    constexpr T cs2 = T(L::cs2);
    const T s00 = s[0][0];
    const T rho = SHIFTED ? T(1) + s00 : s00;
    const T drho = SHIFTED ? s00 : s00 - T(1);
    const T inv_rho = T(1) / rho;
    const T ux = s[1][0] * inv_rho;
    const T uy = s[0][1] * inv_rho;
    k.rho = rho;
    k.drho = drho;
    k.ux = ux;
    k.uy = uy;

    // Hermite moments h_k = sum_i H^k_i v_i (k != 0)
    const T h20 = s[2][0] - cs2 * s00;
    const T h02 = s[0][2] - cs2 * s00;
    const T h11 = s[1][1];

    T sig = T(0);
    if constexpr (THERMAL) {
        // 2 rho c_s^2 (theta - 1) = sum f |c|^2 - 2 c_s^2 rho - rho |u|^2
        const T thm1 = (h20 + h02 - rho * (ux * ux + uy * uy)) * inv_rho * (T(0.5) / cs2);
        sig = cs2 * thm1;
    }
    k.sig = sig;
    eq_coeffs<L, T>(rho, ux, uy, sig, k.C);
    k.C[0][0] = SHIFTED ? drho : rho;

    auto& C = k.C;
    auto& a1 = k.a1;
    static_for<5>([&](auto a) { static_for<5>([&](auto b) { a1[a][b] = T(0); }); });
    if constexpr (COLL == COLL_BGK) return;
    a1[2][0] = h20 - C[2][0];
    a1[1][1] = h11 - C[1][1];
    a1[0][2] = h02 - C[0][2];

    if constexpr (COLL == COLL_PR) {
        if constexpr (L::NEQ >= 3) {
            const T h30 = s[3][0] - T(3) * cs2 * s[1][0];
            const T h21 = s[2][1] - cs2 * s[0][1];
            const T h12 = s[1][2] - cs2 * s[1][0];
            const T h03 = s[0][3] - T(3) * cs2 * s[0][1];
            if constexpr (L::basis(3, 0)) {
                a1[3][0] = h30 - C[3][0];
                a1[0][3] = h03 - C[0][3];
            }
            if constexpr (L::basis(2, 1)) {
                a1[2][1] = h21 - C[2][1];
                a1[1][2] = h12 - C[1][2];
            }
        }
        if constexpr (L::NEQ >= 4) {
            constexpr T cs4 = cs2 * cs2;
            const T h40 = s[4][0] - T(6) * cs2 * s[2][0] + T(3) * cs4 * s00;
            const T h31 = s[3][1] - T(3) * cs2 * s[1][1];
            const T h22 = s[2][2] - cs2 * (s[2][0] + s[0][2]) + cs4 * s00;
            const T h13 = s[1][3] - T(3) * cs2 * s[1][1];
            const T h04 = s[0][4] - T(6) * cs2 * s[0][2] + T(3) * cs4 * s00;
            if constexpr (L::basis(4, 0)) {
                a1[4][0] = h40 - C[4][0];
                a1[0][4] = h04 - C[0][4];
            }
            if constexpr (L::basis(3, 1)) {
                a1[3][1] = h31 - C[3][1];
                a1[1][3] = h13 - C[1][3];
            }
            if constexpr (L::basis(2, 2)) a1[2][2] = h22 - C[2][2];
        }
    } else if constexpr (!THERMAL) {
        iso_recursion<T>(ux, uy, a1);
    } else {
        // thermal path of App. C
        const T xx = a1[2][0], xy = a1[1][1], yy = a1[0][2];
        const T p30 = s[3][0] - T(3) * cs2 * s[1][0] - C[3][0];
        const T p21 = s[2][1] - cs2 * s[0][1] - C[2][1];
        const T p12 = s[1][2] - cs2 * s[1][0] - C[1][2];
        const T p03 = s[0][3] - T(3) * cs2 * s[0][1] - C[0][3];
        if constexpr (A13P) {
            a1[3][0] = p30;
            a1[2][1] = p21;
            a1[1][2] = p12;
            a1[0][3] = p03;
        } else {
            const T gx = T(0.5) * ((ux * xx - p30 * T(1.0 / 3.0)) + (T(2) * uy * xy + ux * yy - p12));
            const T gy = T(0.5) * ((uy * yy - p03 * T(1.0 / 3.0)) + (T(2) * ux * xy + uy * xx - p21));
            a1[3][0] = T(3) * (ux * xx - gx);
            a1[2][1] = T(2) * ux * xy + uy * xx - gy;
            a1[1][2] = T(2) * uy * xy + ux * yy - gx;
            a1[0][3] = T(3) * (uy * yy - gy);
        }
        thermal_rank4<T>(ux, uy, sig, a1);
    }
}

// Steps 1-4 of one node from its populations v.
template <class L, class T, int COLL, bool THERMAL, bool SHIFTED, bool A13P>
__device__ __forceinline__ void node_coeffs(const T (&v)[L::Q], NodeCoeffs<T>& k)
{
    T s[5][5];
    raw_moments<L, T>(v, s);
    coeffs_from_moments<L, T, COLL, THERMAL, SHIFTED, A13P>(s, k);
}

// Step 5: relax and rebuild the populations,
// C = (a0 + k_n a1) / norm over the basis, k_n of rank n (0 above N).
template <class L, class T>
__device__ __forceinline__ void relax_reconstruct(NodeCoeffs<T>& k, T keep, T k3, T k4, T (&out)[L::Q])
{
    static_for<5>([&](auto KX) {
        static_for<5>([&](auto KY) {
            constexpr int n = int(KX) + int(KY);
            if constexpr (L::basis(int(KX), int(KY)) && n >= 1) {
                T c = k.C[KX][KY];
                if constexpr (n == 2) c += keep * k.a1[KX][KY];
                if constexpr (n == 3) c += k3 * k.a1[KX][KY];
                if constexpr (n == 4) c += k4 * k.a1[KX][KY];
                constexpr double nrm = inv_norm<L>(int(KX), int(KY));
                k.C[KX][KY] = c * T(nrm);
            }
        });
    });
    reconstruct<L, T>(k.C, out);
}

// Conservation in float arithmetic.  Two float effects move the conserved
// moments at every step: the lattice identities behind conservation (for
// instance sum_i w_i c_ix^2 = c_s^2) hold only to the rounding of the folded
// constants, so the rebuild returns rho u (1 + eps) with a fixed eps of a few
// 1e-8; and float sums of 37 populations carry a few ulps of error, which a
// correction towards float-summed input moments would write back into the
// state.  Both act coherently over thousands of steps wherever the flow is
// nearly uniform.  So the mass and momentum (and energy when thermal) of the
// input and of the rebuilt populations are summed in double, where every term
// c_i v_i of a float v_i is exact, and the difference is put back along
// w_i, w_i c_i and w_i (|c_i|^2 - 2 c_s^2), which carry mass, momentum and
// energy only (orthogonality on every lattice).  All Hermite moments, the
// equilibrium and the recursion stay in float.
template <class L, bool THERMAL>
__device__ __forceinline__ void conserved_sums(const float (&v)[L::Q], double (&m)[4])
{
    double m0 = 0.0, mx = 0.0, my = 0.0, me = 0.0;
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
        const double x = double(v[I]);
        m0 += x;
        if constexpr (cx != 0) mx += double(cx) * x;
        if constexpr (cy != 0) my += double(cy) * x;
        if constexpr (THERMAL) me += double(cx * cx + cy * cy) * x;
    });
    m[0] = m0;
    m[1] = mx;
    m[2] = my;
    m[3] = me;
}

// Off (FP64 populations, which conserve to ~1e-16, and BF16 storage, whose
// rounding at the store outweighs all of the above): nothing to do.
template <class L, class T, bool THERMAL, bool ON>
struct Invariants {
    __device__ __forceinline__ void take(const T (&)[L::Q]) {}
    __device__ __forceinline__ void restore(T (&)[L::Q]) const {}
};

template <class L, bool THERMAL>
struct Invariants<L, float, THERMAL, true> {
    double m[4];
    __device__ __forceinline__ void take(const float (&v)[L::Q]) { conserved_sums<L, THERMAL>(v, m); }
    __device__ __forceinline__ void restore(float (&out)[L::Q]) const
    {
        constexpr double cs2 = L::cs2;
        double o[4];
        conserved_sums<L, THERMAL>(out, o);
        const double d0 = m[0] - o[0];
        const float dx = float((m[1] - o[1]) * (1.0 / cs2)), dy = float((m[2] - o[2]) * (1.0 / cs2));
        // energy: the mode w (|c|^2 - 2 c_s^2) has sum w (|c|^2 - 2c_s^2)|c|^2 = 4 c_s^4;
        // the mass correction d0 itself adds 2 c_s^2 d0 to sum |c|^2 v
        const float de = THERMAL ? float((m[3] - o[3] - 2.0 * cs2 * d0) * (1.0 / (4.0 * cs2 * cs2))) : 0.0f;
        const float t0 = float(d0);
        static_for<L::Q>([&](auto I) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I];
            constexpr float w = float(L::v.w[I]);
            float c = t0;
            if constexpr (cx != 0) c += float(cx) * dx;
            if constexpr (cy != 0) c += float(cy) * dy;
            if constexpr (THERMAL) c += float(double(cx * cx + cy * cy) - 2.0 * cs2) * de;
            out[I] += w * c;
        });
    }
};

// The regularized (or BGK) collision of one node, in place, with the
// relaxation rx; CONS: restore the conserved moments summed in double (float
// storage).
template <class L, class T, int COLL, bool THERMAL, bool SHIFTED, bool A13P, bool CONS>
__device__ __forceinline__ void collide_node(T (&v)[L::Q], const Relax& rx)
{
    const T keep = T(rx.k2), inv_tau = T(rx.inv_tau);
    Invariants<L, T, THERMAL, CONS> inv;
    inv.take(v);
    NodeCoeffs<T> k;
    node_coeffs<L, T, COLL, THERMAL, SHIFTED, A13P>(v, k);
    if constexpr (COLL == COLL_BGK) {
        static_for<5>([&](auto KX) {
            static_for<5>([&](auto KY) {
                if constexpr (L::basis(int(KX), int(KY)) && int(KX) + int(KY) >= 1) {
                    constexpr double nrm = inv_norm<L>(int(KX), int(KY));
                    k.C[KX][KY] *= T(nrm);
                }
            });
        });
        // each equilibrium population is folded into its own population as
        // soon as it is built, so the Q equilibrium values are never all live
        reconstruct_emit<L, T>(k.C, [&](auto I, T eq) { v[I] = keep * v[I] + inv_tau * eq; });
        inv.restore(v);
        return;
    }
    relax_reconstruct<L, T>(k, keep, T(rx.k3), T(rx.k4), v);
    inv.restore(v);
}

// First-order (Chapman-Enskog) part of an isothermal initial state (Sec.
// III.B): f^(1)_i = w_i sum_{2 <= |k| <= order} H^k_i a1^k / norm_k with
// a1^(2) = -rho c_s^2 tau (grad u + grad u^T) (the relation of Sec. II.E for
// the isothermal equilibrium; du[a][b] = d u_b / d x_a in lattice units) and
// a1^(3), a1^(4) from the isothermal recursion, over the terms of f^(0).
template <class L, class T>
__device__ __forceinline__ void noneq_init_node(T rho, T ux, T uy, const T (&du)[2][2], T tau, int order,
                                                T (&out)[L::Q])
{
    constexpr T cs2 = T(L::cs2);
    const T m = -rho * cs2 * tau;
    T a1[5][5];
    static_for<5>([&](auto a) { static_for<5>([&](auto b) { a1[a][b] = T(0); }); });
    a1[2][0] = m * T(2) * du[0][0];
    a1[1][1] = m * (du[0][1] + du[1][0]);
    a1[0][2] = m * T(2) * du[1][1];
    iso_recursion<T>(ux, uy, a1);
    T C[5][5];
    zero_coeffs<L, T>(C);
    static_for<5>([&](auto KX) {
        static_for<5>([&](auto KY) {
            constexpr int n = int(KX) + int(KY);
            if constexpr (L::basis(int(KX), int(KY)) && n >= 2) {
                constexpr double nrm = inv_norm<L>(int(KX), int(KY));
                C[KX][KY] = (n <= order) ? a1[KX][KY] * T(nrm) : T(0);
            }
        });
    });
    reconstruct<L, T>(C, out);
}

// Equilibrium populations truncated at Hermite rank `order` (initial state).
template <class L, class T, bool SHIFTED>
__device__ __forceinline__ void equilibrium_node(T rho, T ux, T uy, T theta, int order, T (&out)[L::Q])
{
    const T sig = T(L::cs2) * (theta - T(1));
    T mx[5], my[5];
    eq_factors<T>(ux, sig, mx);
    eq_factors<T>(uy, sig, my);
    T C[5][5];
    zero_coeffs<L, T>(C);
    static_for<5>([&](auto KX) {
        static_for<5>([&](auto KY) {
            constexpr int n = int(KX) + int(KY);
            if constexpr (L::basis(int(KX), int(KY)) && n >= 1) {
                constexpr double nrm = inv_norm<L>(int(KX), int(KY));
                C[KX][KY] = (n <= order) ? rho * mx[KX] * my[KY] * T(nrm) : T(0);
            }
        });
    });
    C[0][0] = SHIFTED ? rho - T(1) : rho;
    reconstruct<L, T>(C, out);
}

} // namespace rr
