// Compile-time 3D lattices of Table II: E^19_{3,5} "D3Q19", E^27_{3,5}
// "D3Q27", E^39_{3,7} "D3V39", E^103_{3,9} "D3Q103".  Velocities in canonical order: ascending
// c_z, then c_y, then c_x; the population planes follow it.
#pragma once

#include "lattices.hpp"

namespace rr {

struct Group3 {
    int a, b, c; // representative a >= b >= c >= 0 of a symmetry group
    double w;
};

struct VelTable3 {
    int q = 0;
    int cx[103] = {};
    int cy[103] = {};
    int cz[103] = {};
    double w[103] = {};
};

template <int NG>
constexpr VelTable3 expand3(const Group3 (&g)[NG])
{
    VelTable3 t{};
    for (int z = -3; z <= 3; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                int s0 = x < 0 ? -x : x, s1 = y < 0 ? -y : y, s2 = z < 0 ? -z : z;
                // sort descending
                if (s0 < s1) { const int t0 = s0; s0 = s1; s1 = t0; }
                if (s1 < s2) { const int t1 = s1; s1 = s2; s2 = t1; }
                if (s0 < s1) { const int t2 = s0; s0 = s1; s1 = t2; }
                for (int k = 0; k < NG; ++k)
                    if (g[k].a == s0 && g[k].b == s1 && g[k].c == s2) {
                        t.cx[t.q] = x;
                        t.cy[t.q] = y;
                        t.cz[t.q] = z;
                        t.w[t.q] = g[k].w;
                        ++t.q;
                    }
            }
    return t;
}

// D3Q19: 1/3, 1/18, 1/36 on (0,0,0), (1,0,0), (1,1,0); c_s^2 = 1/3.  Basis
// (Table II): ranks 0-2 and the six rank-3 tensors of the xxy kind.
struct D3Q19 {
    static constexpr int id = 3, Q = 19, R = 1, NEQ = 3;
    static constexpr double cs2 = 1.0 / 3.0;
    static constexpr Group3 groups[3] = { { 0, 0, 0, 1.0 / 3.0 }, { 1, 0, 0, 1.0 / 18.0 }, { 1, 1, 0, 1.0 / 36.0 } };
    static constexpr VelTable3 v = expand3(groups);
    static constexpr bool basis(int a, int b, int c)
    {
        const int n = a + b + c;
        if (n <= 2) return true;
        if (n != 3) return false;
        return (a == 2 || b == 2 || c == 2) && (a == 1 || b == 1 || c == 1);
    }
};

// D3Q27: 8/27, 2/27, 1/54, 1/216; c_s^2 = 1/3.  Basis: the 27 tensor products
// with every exponent at most 2 (up to rank 6, xxyyzz).
struct D3Q27 {
    static constexpr int id = 4, Q = 27, R = 1, NEQ = 6;
    static constexpr double cs2 = 1.0 / 3.0;
    static constexpr Group3 groups[4] = { { 0, 0, 0, 8.0 / 27.0 }, { 1, 0, 0, 2.0 / 27.0 }, { 1, 1, 0, 1.0 / 54.0 },
                                          { 1, 1, 1, 1.0 / 216.0 } };
    static constexpr VelTable3 v = expand3(groups);
    static constexpr bool basis(int a, int b, int c) { return a <= 2 && b <= 2 && c <= 2; }
};

// D3V39: 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620 on (0,0,0), (1,0,0),
// (1,1,1), (2,0,0), (2,2,0), (3,0,0); c_s^2 = 2/3.  Basis: every tensor of
// rank <= 3.
struct D3V39 {
    static constexpr int id = 5, Q = 39, R = 3, NEQ = 3;
    static constexpr double cs2 = 2.0 / 3.0;
    static constexpr Group3 groups[6] = { { 0, 0, 0, 1.0 / 12.0 }, { 1, 0, 0, 1.0 / 12.0 },
                                          { 1, 1, 1, 1.0 / 27.0 }, { 2, 0, 0, 2.0 / 135.0 },
                                          { 2, 2, 0, 1.0 / 432.0 }, { 3, 0, 0, 1.0 / 1620.0 } };
    static constexpr VelTable3 v = expand3(groups);
    static constexpr bool basis(int a, int b, int c) { return a + b + c <= 3; }
};

// D3Q103: the 21-digit weights of Table II on (0,0,0), (1,0,0), (1,1,1),
// (2,0,0), (2,1,0), (2,2,0), (2,2,2), (3,0,0), (3,1,1), (3,3,3); c_s =
// 1 / 1.19697977039307435897239.  Basis: every tensor of rank <= 4.
struct D3Q103 {
    static constexpr int id = 6, Q = 103, R = 3, NEQ = 4;
    static constexpr double inv_cs = 1.19697977039307435897239;
    static constexpr double cs2 = 1.0 / (inv_cs * inv_cs);
    static constexpr Group3 groups[10] = {
        { 0, 0, 0, 0.032633351764471159466 }, { 1, 0, 0, 0.097656833590334574221 },
        { 1, 1, 1, 0.028097750290257335627 }, { 2, 0, 0, 0.001045259560430061466 },
        { 2, 1, 0, 0.005705329016894815990 }, { 2, 2, 0, 0.000611939269829747839 },
        { 2, 2, 2, 0.000155964159374283722 }, { 3, 0, 0, 0.000284443251800055207 },
        { 3, 1, 1, 0.000130698375985191585 }, { 3, 3, 3, 0.000001223194501323058 }
    };
    static constexpr VelTable3 v = expand3(groups);
    static constexpr bool basis(int a, int b, int c) { return a + b + c <= 4; }
};

static_assert(D3Q19::v.q == 19 && D3Q27::v.q == 27 && D3V39::v.q == 39 && D3Q103::v.q == 103, "velocity count");

// Sign orbits: the distinct (|c_x|, |c_y|, |c_z|) of a lattice.  Since
// He_n(-x) = (-1)^n He_n(x), every velocity of one orbit sees the same basis
// products up to the sign (-1)^(a sx + b sy + c sz) of its negative axes.
struct Orbits3 {
    int n = 0;
    int ax[103] = {};
    int ay[103] = {};
    int az[103] = {};
};

constexpr Orbits3 orbits3(const VelTable3& v)
{
    Orbits3 o{};
    for (int i = 0; i < v.q; ++i) {
        const int a = v.cx[i] < 0 ? -v.cx[i] : v.cx[i];
        const int b = v.cy[i] < 0 ? -v.cy[i] : v.cy[i];
        const int c = v.cz[i] < 0 ? -v.cz[i] : v.cz[i];
        bool seen = false;
        for (int k = 0; k < o.n; ++k) seen = seen || (o.ax[k] == a && o.ay[k] == b && o.az[k] == c);
        if (!seen) {
            o.ax[o.n] = a;
            o.ay[o.n] = b;
            o.az[o.n] = c;
            ++o.n;
        }
    }
    return o;
}

template <class L>
struct OrbitsOf {
    static constexpr Orbits3 o = orbits3(L::v);
};

// 1 / (a! b! c! c_s^(2(a+b+c))): the normalisation of each 3D basis term.
template <class L>
constexpr double inv_norm3(int a, int b, int c)
{
    return 1.0 / (factorial(a) * factorial(b) * factorial(c) * ipow(L::cs2, a + b + c));
}

} // namespace rr
