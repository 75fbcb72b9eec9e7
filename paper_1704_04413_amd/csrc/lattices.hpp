// Compile-time lattice descriptions for the HIP kernels (Table I of the paper:
// E^9_{2,5} "D2Q9", E^17_{2,7} "D2V17", E^37_{2,9} "D2V37").
//
// Velocities are integers (on-grid condition of Sec. III.A) listed in canonical
// order: ascending c_y, then ascending c_x.  The population planes in device
// memory follow the same order.  Everything here is constexpr so the kernels
// see every velocity, weight and Hermite value as an immediate.
#pragma once

#include <utility>

namespace rr {

struct Group {
    int a, b;   // representative |c_x| >= |c_y| >= 0 of a symmetry group
    double w;   // weight shared by the group
};

struct VelTable {
    int q = 0;
    int cx[37] = {};
    int cy[37] = {};
    double w[37] = {};
};

template <int NG>
constexpr VelTable expand(const Group (&g)[NG])
{
    VelTable t{};
    for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x) {
            const int ax = x < 0 ? -x : x, ay = y < 0 ? -y : y;
            const int hi = ax > ay ? ax : ay, lo = ax > ay ? ay : ax;
            for (int k = 0; k < NG; ++k)
                if (g[k].a == hi && g[k].b == lo) {
                    t.cx[t.q] = x;
                    t.cy[t.q] = y;
                    t.w[t.q] = g[k].w;
                    ++t.q;
                }
        }
    return t;
}

// D2Q9: standard weights 4/9, 1/9, 1/36 on (0,0), (1,0), (1,1); c_s^2 = 1/3.
// Basis: 1, x, y, xx, xy, yy, xxy, xyy, xxyy (the "complete" D2Q9 basis).
struct D2Q9 {
    static constexpr int id = 0, Q = 9, R = 1, NEQ = 4;
    static constexpr double cs2 = 1.0 / 3.0;
    static constexpr Group groups[3] = { { 0, 0, 4.0 / 9.0 }, { 1, 0, 1.0 / 9.0 }, { 1, 1, 1.0 / 36.0 } };
    static constexpr VelTable v = expand(groups);
    static constexpr bool basis(int nx, int ny) { return nx <= 2 && ny <= 2; }
};

// D2V17: weights are the closed forms of Table I, (575+193 sqrt193)/8100 ...,
// evaluated to 25 digits; 1/c_s = sqrt(5 (25 + sqrt193) / 72).
// Basis: every Hermite tensor of rank <= 3.
struct D2V17 {
    static constexpr int id = 1, Q = 17, R = 3, NEQ = 3;
    static constexpr double cs2 = 3.7025186701833984971891510e-1;
    static constexpr Group groups[5] = {
        { 0, 0, 4.0200514690911262594166439e-1 }, { 1, 0, 1.1615486649778154387403546e-1 },
        { 1, 1, 3.3006353622986913949753826e-2 }, { 2, 2, 7.9078602165918131237133241e-5 },
        { 3, 0, 2.5841454978746755955748610e-4 },
    };
    static constexpr VelTable v = expand(groups);
    static constexpr bool basis(int nx, int ny) { return nx + ny <= 3; }
};

// D2V37: weights and 1/c_s = 1.19697977039307435897239 as printed in Table I.
// Basis: every Hermite tensor of rank <= 4.
struct D2V37 {
    static constexpr int id = 2, Q = 37, R = 3, NEQ = 4;
    static constexpr double cs2 = 6.9795332201968308823840726e-1;
    static constexpr Group groups[8] = {
        { 0, 0, 0.23315066913235250228650 }, { 1, 0, 0.10730609154221900241246 },
        { 1, 1, 0.05766785988879488203006 }, { 2, 0, 0.01420821615845075026469 },
        { 2, 1, 0.00535304900051377523273 }, { 2, 2, 0.00101193759267357547541 },
        { 3, 0, 0.00024530102775771734547 }, { 3, 1, 0.00028341425299419821740 },
    };
    static constexpr VelTable v = expand(groups);
    static constexpr bool basis(int nx, int ny) { return nx + ny <= 4; }
};

static_assert(D2Q9::v.q == 9 && D2V17::v.q == 17 && D2V37::v.q == 37, "velocity count");

// Scaled 1D Hermite polynomials in lattice units, He_n(v) with variance c_s^2
// (the 2D tensors of App. C are products He_nx(c_x) He_ny(c_y)).
constexpr double he(int n, double v, double cs2)
{
    switch (n) {
    case 0: return 1.0;
    case 1: return v;
    case 2: return v * v - cs2;
    case 3: return v * v * v - 3.0 * cs2 * v;
    case 4: return v * v * v * v - 6.0 * cs2 * v * v + 3.0 * cs2 * cs2;
    }
    return 0.0;
}

constexpr double factorial(int n) { return n <= 1 ? 1.0 : n * factorial(n - 1); }
constexpr double ipow(double b, int e) { return e == 0 ? 1.0 : b * ipow(b, e - 1); }

// 1 / (n_x! n_y! c_s^(2(n_x+n_y))): the normalisation of each basis term.
template <class L>
constexpr double inv_norm(int nx, int ny)
{
    return 1.0 / (factorial(nx) * factorial(ny) * ipow(L::cs2, nx + ny));
}

// Index of the velocity (x, y) in canonical order, -1 if absent.
template <class L>
constexpr int vel_index(int x, int y)
{
    for (int i = 0; i < L::Q; ++i)
        if (L::v.cx[i] == x && L::v.cy[i] == y) return i;
    return -1;
}

template <class F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

} // namespace rr
