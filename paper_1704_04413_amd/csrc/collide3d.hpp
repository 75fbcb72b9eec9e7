// Isothermal regularized collision and step kernels on the 3D lattices of
// Table II (FP64 populations).  Basis exponents reach 4 (D3Q103), so the
// coefficient tables are 5 x 5 x 5 with compile-time holes.
//
// Per node: rho, j and Pi from the populations; a0 of every basis term is
// rho u_x^a u_y^b u_z^c (Eq. HermiteCoeffEq at theta = 1); a1^(2) = Pi -
// c_s^2 rho delta - rho u u (Eq. a12Proj); every higher rank follows the
// isothermal recursion (Eq. MalaspinasRecursiveRelation), whose solution at
// theta = 1 is the sum over index pairs of a1^(2)_pair times the u's of the
// other indices:
//   a1_(a,b,c) = C(a,2) a1_xx u^(a-2,b,c) + C(b,2) a1_yy u^(a,b-2,c)
//              + C(c,2) a1_zz u^(a,b,c-2) + a b a1_xy u^(a-1,b-1,c)
//              + a c a1_xz u^(a-1,b,c-1) + b c a1_yz u^(a,b-1,c-1)
// (App. C gives the 3D forms up to rank 4, a1_xyz and a1_xxyz).  The
// populations are rebuilt with Eq. (GenRegCollision) over the basis,
// f_i = w_i sum_k He_a(c_x) He_b(c_y) He_c(c_z) C_k / (a! b! c! c_s^2n).
// The state between steps is post-collision, pulled like the 2D step.
#pragma once

#include "common.hpp"
#include "lattices3d.hpp"
#include "storage.hpp"

namespace rr {

struct Step3Args {
    const void* fin;
    void* fout;
    Layout lay; // row-tiled over the ny * nz rows, row r = z ny + y
    int ny, nz;
    int bx_blocks;
    int nblocks;   // blocks in the grid
    int xcd_remap; // 1: XCD k takes the k-th contiguous eighth of the tiles
    Relax rx;
    int order;
    int reverse;   // 1: walk the tiles last to first (POL_CACHE, and the single-buffer step, every other step)
};

// Register budget of the 3D step kernel, as the minimum number of waves per
// SIMD the compiler must leave room for.
#ifndef RRLBM_WAVES_PER_EU_3D
#define RRLBM_WAVES_PER_EU_3D 1
#endif

// Modes of collide3: C3_RR regularized with the recursion at order `order`,
// C3_PR regularized by projection (Eq. a1Proj on every kept rank up to
// `order`), C3_BGK single relaxation to the full-basis equilibrium, C3_EQ the
// equilibrium of (eq_rho, eq_u) truncated to ranks <= `order`.
enum { C3_RR = 0, C3_PR = 1, C3_BGK = 2, C3_EQ = 3 };

// Bit 4p + 2q + r set when parity class (p, q, r) of orbit (ax, ay, az)
// holds a basis term with a non-zero product.
template <class L>
constexpr int classes_used(int ax, int ay, int az)
{
    int m = 0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b)
            for (int c = 0; c < 5; ++c)
                if (L::basis(a, b, c) &&
                    he(a, double(ax), L::cs2) * he(b, double(ay), L::cs2) * he(c, double(az), L::cs2) != 0.0)
                    m |= 1 << (4 * (a & 1) + 2 * (b & 1) + (c & 1));
    return m;
}

// emit(I, s) with s = sum over the basis of He_a(c_x) He_b(c_y) He_c(c_z)
// C[a][b][c] for every velocity I, orbit by orbit: the eight parity sums
// P_pqr = sum over (a, b, c) = (p, q, r) mod 2 of the products at
// (|c_x|, |c_y|, |c_z|) are formed once per orbit, and each member adds them
// with the signs of its negative components.
template <class L, class Emit>
__device__ __forceinline__ void reconstruct3(const double (&C)[5][5][5], Emit&& emit)
{
    constexpr double cs2 = L::cs2;
    static_for<OrbitsOf<L>::o.n>([&](auto K) {
        constexpr int ax = OrbitsOf<L>::o.ax[K], ay = OrbitsOf<L>::o.ay[K], az = OrbitsOf<L>::o.az[K];
        constexpr int used = classes_used<L>(ax, ay, az);
        double P[2][2][2];
        static_for<8>([&](auto PC) { P[PC >> 2][(PC >> 1) & 1][PC & 1] = 0.0; });
        static_for<5>([&](auto A) {
            static_for<5>([&](auto B) {
                static_for<5>([&](auto Cc) {
                    constexpr int a = int(A), b = int(B), c = int(Cc);
                    if constexpr (L::basis(a, b, c)) {
                        constexpr double h = he(a, double(ax), cs2) * he(b, double(ay), cs2) * he(c, double(az), cs2);
                        if constexpr (h != 0.0) P[a & 1][b & 1][c & 1] += h * C[a][b][c];
                    }
                });
            });
        });
        static_for<L::Q>([&](auto I) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            if constexpr ((cx < 0 ? -cx : cx) == ax && (cy < 0 ? -cy : cy) == ay && (cz < 0 ? -cz : cz) == az) {
                double s = 0.0;
                static_for<8>([&](auto PC) {
                    constexpr int p = int(PC) >> 2, q = (int(PC) >> 1) & 1, r = int(PC) & 1;
                    if constexpr ((used >> int(PC)) & 1) {
                        constexpr bool neg = ((p && cx < 0) + (q && cy < 0) + (r && cz < 0)) & 1;
                        if constexpr (neg)
                            s -= P[p][q][r];
                        else
                            s += P[p][q][r];
                    }
                });
                emit(I, s);
            }
        });
    });
}

// A[a][b][c] = sum_i He_a(c_x) He_b(c_y) He_c(c_z) g_i on every basis term
// of rank >= 2 (the projection of Eq. a1Proj), orbit by orbit: the signed
// sums G_pqr = sum over the orbit of s_x^p s_y^q s_z^r g_i are formed once
// and each term takes the one of its parity class.
template <class L>
__device__ __forceinline__ void project3(const double (&g)[L::Q], double (&A)[5][5][5])
{
    constexpr double cs2 = L::cs2;
    static_for<5>([&](auto Aa) {
        static_for<5>([&](auto B) {
            static_for<5>([&](auto Cc) {
                if constexpr (L::basis(int(Aa), int(B), int(Cc))) A[Aa][B][Cc] = 0.0;
            });
        });
    });
    static_for<OrbitsOf<L>::o.n>([&](auto K) {
        constexpr int ax = OrbitsOf<L>::o.ax[K], ay = OrbitsOf<L>::o.ay[K], az = OrbitsOf<L>::o.az[K];
        constexpr int used = classes_used<L>(ax, ay, az);
        double G[2][2][2];
        static_for<8>([&](auto PC) { G[PC >> 2][(PC >> 1) & 1][PC & 1] = 0.0; });
        static_for<L::Q>([&](auto I) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            if constexpr ((cx < 0 ? -cx : cx) == ax && (cy < 0 ? -cy : cy) == ay && (cz < 0 ? -cz : cz) == az) {
                static_for<8>([&](auto PC) {
                    constexpr int p = int(PC) >> 2, q = (int(PC) >> 1) & 1, r = int(PC) & 1;
                    if constexpr ((used >> int(PC)) & 1) {
                        constexpr bool neg = ((p && cx < 0) + (q && cy < 0) + (r && cz < 0)) & 1;
                        if constexpr (neg)
                            G[p][q][r] -= g[I];
                        else
                            G[p][q][r] += g[I];
                    }
                });
            }
        });
        static_for<5>([&](auto Aa) {
            static_for<5>([&](auto B) {
                static_for<5>([&](auto Cc) {
                    constexpr int a = int(Aa), b = int(B), c = int(Cc);
                    if constexpr (L::basis(a, b, c) && a + b + c >= 2) {
                        constexpr double h = he(a, double(ax), cs2) * he(b, double(ay), cs2) * he(c, double(az), cs2);
                        if constexpr (h != 0.0) A[a][b][c] += h * G[a & 1][b & 1][c & 1];
                    }
                });
            });
        });
    });
}

// The post-collision value of velocity I goes to out(I, value) as soon as
// it is formed (v is read, never written, except by the PR pass).
template <class L, int MODE, class Out>
__device__ __forceinline__ void collide3(double (&v)[L::Q], const Relax& rx, int order, Out&& out,
                                         double eq_rho = 0.0, double eq_ux = 0.0, double eq_uy = 0.0,
                                         double eq_uz = 0.0)
{
    constexpr double cs2 = L::cs2;
    double r, ux, uy, uz, axx = 0, ayy = 0, azz = 0, axy = 0, axz = 0, ayz = 0;
    if constexpr (MODE == C3_EQ) {
        r = eq_rho;
        ux = eq_ux;
        uy = eq_uy;
        uz = eq_uz;
    } else {
        double s0 = 0, jx = 0, jy = 0, jz = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
        static_for<L::Q>([&](auto I) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            const double f = v[I];
            s0 += f;
            if constexpr (cx != 0) jx += double(cx) * f;
            if constexpr (cy != 0) jy += double(cy) * f;
            if constexpr (cz != 0) jz += double(cz) * f;
            if constexpr (MODE == C3_RR) {
                if constexpr (cx != 0) pxx += double(cx * cx) * f;
                if constexpr (cy != 0) pyy += double(cy * cy) * f;
                if constexpr (cz != 0) pzz += double(cz * cz) * f;
                if constexpr (cx * cy != 0) pxy += double(cx * cy) * f;
                if constexpr (cx * cz != 0) pxz += double(cx * cz) * f;
                if constexpr (cy * cz != 0) pyz += double(cy * cz) * f;
            }
        });
        r = s0;
        const double inv = 1.0 / r;
        ux = jx * inv;
        uy = jy * inv;
        uz = jz * inv;
        if constexpr (MODE == C3_RR) {
            axx = pxx - cs2 * r - r * ux * ux;
            ayy = pyy - cs2 * r - r * uy * uy;
            azz = pzz - cs2 * r - r * uz * uz;
            axy = pxy - r * ux * uy;
            axz = pxz - r * ux * uz;
            ayz = pyz - r * uy * uz;
        }
    }
    const double px[5] = { 1.0, ux, ux * ux, ux * ux * ux, (ux * ux) * (ux * ux) };
    const double py[5] = { 1.0, uy, uy * uy, uy * uy * uy, (uy * uy) * (uy * uy) };
    const double pz[5] = { 1.0, uz, uz * uz, uz * uz * uz, (uz * uz) * (uz * uz) };
    // C[a][b][c] = (a0 + k_n a1) / (a! b! c! c_s^2n) on the basis
    double C[5][5][5];
    static_for<5>([&](auto A) {
        static_for<5>([&](auto B) {
            static_for<5>([&](auto Cc) {
                constexpr int a = int(A), b = int(B), c = int(Cc), n = a + b + c;
                if constexpr (L::basis(a, b, c)) {
                    double val = r * px[a] * py[b] * pz[c];
                    if constexpr (MODE == C3_EQ) {
                        if (n > order) val = 0.0;
                    }
                    if constexpr (MODE == C3_RR && n >= 2) {
                        double t = 0.0;
                        if constexpr (a >= 2) t += double(a * (a - 1) / 2) * axx * px[a - 2] * py[b] * pz[c];
                        if constexpr (b >= 2) t += double(b * (b - 1) / 2) * ayy * px[a] * py[b - 2] * pz[c];
                        if constexpr (c >= 2) t += double(c * (c - 1) / 2) * azz * px[a] * py[b] * pz[c - 2];
                        if constexpr (a >= 1 && b >= 1) t += double(a * b) * axy * px[a - 1] * py[b - 1] * pz[c];
                        if constexpr (a >= 1 && c >= 1) t += double(a * c) * axz * px[a - 1] * py[b] * pz[c - 1];
                        if constexpr (b >= 1 && c >= 1) t += double(b * c) * ayz * px[a] * py[b - 1] * pz[c - 1];
                        const double k = n == 2 ? rx.k2 : n == 3 ? rx.k3 : (n <= order ? rx.k4 : 0.0);
                        val += k * t;
                    }
                    constexpr double nrm = inv_norm3<L>(a, b, c);
                    C[a][b][c] = val * nrm;
                }
            });
        });
    });
    if constexpr (MODE == C3_PR) {
        // f^neq = f - f^eq, then a1 of every kept tensor of rank 2..order by
        // projection onto it
        reconstruct3<L>(C, [&](auto I, double s) { v[I] -= L::v.w[I] * s; });
        double A1[5][5][5];
        project3<L>(v, A1);
        static_for<5>([&](auto A) {
            static_for<5>([&](auto B) {
                static_for<5>([&](auto Cc) {
                    constexpr int a = int(A), b = int(B), c = int(Cc), n = a + b + c;
                    if constexpr (L::basis(a, b, c) && n >= 2) {
                        const double k = n == 2 ? rx.k2 : n == 3 ? rx.k3 : (n <= order ? rx.k4 : 0.0);
                        constexpr double nrm = inv_norm3<L>(a, b, c);
                        C[a][b][c] += k * A1[a][b][c] * nrm;
                    }
                });
            });
        });
    }
    reconstruct3<L>(C, [&](auto I, double s) {
        constexpr double w = L::v.w[I];
        if constexpr (MODE == C3_BGK)
            out(I, rx.k2 * v[I] + rx.inv_tau * (w * s));
        else
            out(I, w * s);
    });
}

// One thread per node.  A block is 64 x 4 nodes and a wave is one 64-wide
// row segment (BX equals the wave size), so the row, its y and z, and every
// source row of the pull are wave-uniform: the base address of each
// (population, source row) pair is scalar and a lane adds only the byte
// offset of its wrapped x, a 32-bit value.
// POL: cache policy as in the 2D step (POL_STREAM ordinary loads and
// non-temporal stores, POL_CACHE ordinary loads and stores, POL_KEEP
// non-temporal loads and ordinary stores).
__device__ __forceinline__ int block_index3(const Step3Args& a)
{
    int bid = int(blockIdx.x);
    if (a.xcd_remap) {
        // the hardware deals blocks to the 8 XCDs round-robin
        const int q = a.nblocks / 8, r = a.nblocks % 8, xcd = bid % 8, local = bid / 8;
        bid = xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
    }
    return a.reverse ? a.nblocks - 1 - bid : bid;
}

// S: StoreF64, or StoreF32D (float g = f - w in memory, double arithmetic;
// f = g + w on the load, g = f - w rounded once at the store).
template <class L, int MODE, int POL, class S = StoreF64>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(RRLBM_WAVES_PER_EU_3D)))
void k_stream_collide3(Step3Args a)
{
    static_assert(BX == 64, "one wave per row segment");
    using E = typename S::elem;
    constexpr int R = L::R;
    const int nx = a.lay.nx, ny = a.ny, nz = a.nz;
    const int bid = block_index3(a);
    const int ty = __builtin_amdgcn_readfirstlane(int(threadIdx.y)); // uniform within a wave
    const int row = (bid / a.bx_blocks) * BY + ty;
    const int x = (bid % a.bx_blocks) * BX + int(threadIdx.x);
    if (row >= ny * nz || x >= nx) return;
    const int y = row % ny, z = row / ny;
    uint32_t xb[2 * R + 1]; // byte offset of the source column, per shift
    int ys[2 * R + 1], zs[2 * R + 1];
    static_for<2 * R + 1>([&](auto D) {
        constexpr int d = int(D) - R;
        int xx = x - d, yy = y - d, zz = z - d;
        if constexpr (d > 0) {
            xx += (xx < 0) ? nx : 0;
            yy += (yy < 0) ? ny : 0;
            zz += (zz < 0) ? nz : 0;
        } else if constexpr (d < 0) {
            xx -= (xx >= nx) ? nx : 0;
            yy -= (yy >= ny) ? ny : 0;
            zz -= (zz >= nz) ? nz : 0;
        }
        xb[D] = uint32_t(xx) * uint32_t(sizeof(E));
        ys[D] = yy;
        zs[D] = zz;
    });
    const char* __restrict__ fin = static_cast<const char*>(a.fin);
    char* __restrict__ fout = static_cast<char*>(a.fout);
    const int64_t plane = int64_t(a.lay.te) * int64_t(sizeof(E));
    const int64_t here_row = int64_t(a.lay.row(row)) * int64_t(sizeof(E));
    const uint32_t xh = uint32_t(x) * uint32_t(sizeof(E));
    double v[L::Q];
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
        const int64_t src_row = int64_t(a.lay.row(zs[cz + R] * ny + ys[cy + R])) * int64_t(sizeof(E));
        const char* base = fin + src_row + int64_t(I) * plane;
        const E* p = reinterpret_cast<const E*>(base + xb[cx + R]);
        double g;
        if constexpr (POL == POL_KEEP)
            g = S::load_nt(p);
        else
            g = S::load(p);
        if constexpr (S::shifted) g += L::v.w[I];
        v[I] = g;
    });
    collide3<L, MODE>(v, a.rx, a.order, [&](auto I, double val) {
        E* p = reinterpret_cast<E*>(fout + here_row + int64_t(I) * plane + xh);
        if constexpr (S::shifted) val -= L::v.w[I];
        if constexpr (POL == POL_STREAM)
            S::store_nt(p, val);
        else
            S::store(p, val);
    });
}

// The index of -c_i.
template <class L>
constexpr int opp_index3(int i)
{
    for (int j = 0; j < L::Q; ++j)
        if (L::v.cx[j] == -L::v.cx[i] && L::v.cy[j] == -L::v.cy[i] && L::v.cz[j] == -L::v.cz[i]) return j;
    return -1;
}

// Hides a wave-uniform value from the optimizer (no instruction is emitted).
__device__ __forceinline__ void opaque_s(int& v) { asm volatile("" : "+s"(v)); }
__device__ __forceinline__ void opaque_v(int& v) { asm volatile("" : "+v"(v)); }

// The in-place step on one buffer (the AA pattern), as in 2D: !SHIFTED (the
// state after an odd number of steps, or the initial populations) reads
// value i from the node's own plane i and writes it to its own plane opp(i);
// SHIFTED (after an even number) reads plane opp(i) of the node x - c_i and
// writes plane i of the node x + c_i.  Each thread writes exactly the slots
// it has read, after reading all of them.  Addressing as in the pull kernel
// (wave-uniform row bases, per-lane byte offsets of x).
template <class L, int MODE, bool SHIFTED, bool NT, class S = StoreF64>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(RRLBM_WAVES_PER_EU_3D)))
void k_stream_collide3_aa(Step3Args a)
{
    static_assert(BX == 64, "one wave per row segment");
    using E = typename S::elem;
    constexpr int R = L::R;
    const int nx = a.lay.nx, ny = a.ny, nz = a.nz;
    const int bid = block_index3(a);
    const int ty = __builtin_amdgcn_readfirstlane(int(threadIdx.y)); // uniform within a wave
    int row = (bid / a.bx_blocks) * BY + ty;
    int x = (bid % a.bx_blocks) * BX + int(threadIdx.x);
    if (row >= ny * nz || x >= nx) return;

    // byte offset of x + d and rows y + d, z + d (periodic), d in [-R, R]
    uint32_t xb[2 * R + 1];
    int ys[2 * R + 1], zs[2 * R + 1];
    auto neighbours = [&](int x0, int row0) {
        const int y0 = row0 % ny, z0 = row0 / ny;
        static_for<2 * R + 1>([&](auto D) {
            constexpr int d = int(D) - R;
            int xx = x0 + d, yy = y0 + d, zz = z0 + d;
            if constexpr (d < 0) {
                xx += (xx < 0) ? nx : 0;
                yy += (yy < 0) ? ny : 0;
                zz += (zz < 0) ? nz : 0;
            } else if constexpr (d > 0) {
                xx -= (xx >= nx) ? nx : 0;
                yy -= (yy >= ny) ? ny : 0;
                zz -= (zz >= nz) ? nz : 0;
            }
            xb[D] = uint32_t(xx) * uint32_t(sizeof(E));
            ys[D] = yy;
            zs[D] = zz;
        });
    };
    char* f = static_cast<char*>(a.fout);
    const int64_t plane = int64_t(a.lay.te) * int64_t(sizeof(E));
    auto slot = [&](int dz, int dy, uint32_t xoff, int i) {
        const int64_t r = int64_t(a.lay.row(zs[dz + R] * ny + ys[dy + R])) * int64_t(sizeof(E));
        return reinterpret_cast<E*>(f + r + int64_t(i) * plane + xoff);
    };
    neighbours(x, row);
    double v[L::Q];
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
        constexpr int o = opp_index3<L>(int(I)); // a compile-time constant, not a run-time search
        double g;
        if constexpr (SHIFTED)
            g = S::load(slot(-cz, -cy, xb[R - cx], o));
        else
            g = S::load(slot(0, 0, xb[R], int(I)));
        if constexpr (S::shifted) g += L::v.w[I];
        v[I] = g;
    });
    // The stores go to the addresses the loads used; hiding the node makes
    // the compiler rebuild them rather than hold all Q across the collision.
    opaque_s(row);
    opaque_v(x);
    neighbours(x, row);
    collide3<L, MODE>(v, a.rx, a.order, [&](auto I, double val) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
        constexpr int o = opp_index3<L>(int(I));
        E* p = SHIFTED ? slot(cz, cy, xb[R + cx], int(I)) : slot(0, 0, xb[R], o);
        if constexpr (S::shifted) val -= L::v.w[I];
        if constexpr (NT)
            S::store_nt(p, val);
        else
            S::store(p, val);
    });
}

struct Init3Args {
    void* f;
    Layout lay;
    int ny, nz;
    const double *rho, *ux, *uy, *uz, *noise;
    double noise_amp;
    int eq_order;
};

// f^(0) over the basis up to rank eq_order plus noise_amp w_i noise_i.
// SHIFT: written for the first pull, value i of node x to node x - c_i, so
// that one step kernel launch gathers f^(0) back at every node and collides
// it (the kept state is post-collision); !SHIFT: value i in the node's own
// plane i, for the in-place local kernel.
template <class L, bool SHIFT = true, class S = StoreF64>
__global__ __launch_bounds__(256) void k_init3(Init3Args a)
{
    const int nx = a.lay.nx, ny = a.ny, nz = a.nz;
    const int64_t n = int64_t(nx) * ny * nz;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = int(k % nx), row = int(k / nx), y = row % ny, z = row / ny;
    double f[L::Q];
    const Relax none{ 0.0, 0.0, 0.0, 0.0 };
    typename S::elem* out = static_cast<typename S::elem*>(a.f);
    collide3<L, C3_EQ>(
        f, none, a.eq_order,
        [&](auto I, double val) {
            constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            if (a.noise) val += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k];
            int xd = SHIFT ? x - cx : x, yd = SHIFT ? y - cy : y, zd = SHIFT ? z - cz : z; // |c| <= reach
            xd += xd < 0 ? nx : (xd >= nx ? -nx : 0);
            yd += yd < 0 ? ny : (yd >= ny ? -ny : 0);
            zd += zd < 0 ? nz : (zd >= nz ? -nz : 0);
            if constexpr (S::shifted) val -= L::v.w[I];
            S::store(out + a.lay.row(zd * ny + yd) + xd + int(I) * a.lay.te, val);
        },
        a.rho[k], a.ux[k], a.uy[k], a.uz[k]);
}

// rho, u per node and block sums of [rho, rho ux, rho uy, rho uz,
// sum f |c|^2 / 2, |u|^2, |u|^4, non-finite].
// Where value I of node (x, y, z) is held: RD 0 the two-buffer state
// (plane I at the node); the single-buffer state after an even number of
// steps (RD 1): plane opp(I) at the node; after an odd number (RD 2): plane
// I at the node x + c_I (periodic).
template <class L, int RD, int I>
__device__ __forceinline__ int state_index3(const Layout& lay, int ny, int nz, int x, int y, int z)
{
    if constexpr (RD == 0) {
        return lay.row(z * ny + y) + x + I * lay.te;
    } else if constexpr (RD == 1) {
        constexpr int o = opp_index3<L>(I); // folded at compile time
        return lay.row(z * ny + y) + x + o * lay.te;
    } else {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
        int xx = x + cx, yy = y + cy, zz = z + cz;
        xx += xx < 0 ? lay.nx : (xx >= lay.nx ? -lay.nx : 0);
        yy += yy < 0 ? ny : (yy >= ny ? -ny : 0);
        zz += zz < 0 ? nz : (zz >= nz ? -nz : 0);
        return lay.row(zz * ny + yy) + xx + I * lay.te;
    }
}

// The state as populations [i][z][y][x].
template <class L, int RD, class S = StoreF64>
__global__ __launch_bounds__(256) void k_populations3(const typename S::elem* f, Layout lay, int ny, int nz,
                                                      double* out)
{
    const int64_t n = int64_t(lay.nx) * ny * nz;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = int(k % lay.nx), row = int(k / lay.nx), y = row % ny, z = row / ny;
    static_for<L::Q>([&](auto I) {
        double v = S::load(f + state_index3<L, RD, int(I)>(lay, ny, nz, x, y, z));
        if constexpr (S::shifted) v += L::v.w[I];
        out[int64_t(I) * n + k] = v;
    });
}

template <class L, int RD = 0, class S = StoreF64>
__global__ __launch_bounds__(256) void k_moments3(const typename S::elem* f, Layout lay, int ny, int nz, double* rho_o,
                                                  double* ux_o, double* uy_o, double* uz_o, double* partial)
{
    const int64_t n = int64_t(lay.nx) * ny * nz;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM3_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        const int x = int(k % lay.nx), row = int(k / lay.nx), y = row % ny, z = row / ny;
        double r = 0, jx = 0, jy = 0, jz = 0, e2 = 0;
        static_for<L::Q>([&](auto I) {
            constexpr double cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            double v = S::load(f + state_index3<L, RD, int(I)>(lay, ny, nz, x, y, z));
            if constexpr (S::shifted) v += L::v.w[I];
            r += v;
            jx += cx * v;
            jy += cy * v;
            jz += cz * v;
            e2 += (cx * cx + cy * cy + cz * cz) * v;
        });
        const double ux = jx / r, uy = jy / r, uz = jz / r;
        const double u2 = ux * ux + uy * uy + uz * uz;
        rho_o[k] = r;
        ux_o[k] = ux;
        uy_o[k] = uy;
        uz_o[k] = uz;
        if (std::isfinite(r) && std::isfinite(u2)) {
            val[0] = r;
            val[1] = jx;
            val[2] = jy;
            val[3] = jz;
            val[4] = 0.5 * e2;
            val[5] = u2;
            val[6] = u2 * u2;
        } else {
            val[7] = 1.0;
        }
    }
    block_sums<MOM3_NS>(val, partial);
}

} // namespace rr
