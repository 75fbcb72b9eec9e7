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

#include "collide.hpp"
#include "lattices3d.hpp"

namespace rr {

struct Step3Args {
    const void* fin;
    void* fout;
    Layout lay; // row-tiled over the ny * nz rows, row r = z ny + y
    int ny, nz;
    int bx_blocks;
    Relax rx;
    int order;
};

// Modes of collide3: C3_RR regularized with the recursion at order `order`,
// C3_PR regularized by projection (Eq. a1Proj on every kept rank up to
// `order`), C3_BGK single relaxation to the full-basis equilibrium, C3_EQ the
// equilibrium of (eq_rho, eq_u) truncated to ranks <= `order`.
enum { C3_RR = 0, C3_PR = 1, C3_BGK = 2, C3_EQ = 3 };

// sum over the basis of He_a(c_x) He_b(c_y) He_c(c_z) C[a][b][c] for
// velocity I (the products are compile-time constants; zeros are skipped)
template <class L, int I>
__device__ __forceinline__ double hsum3(const double (&C)[5][5][5])
{
    constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
    constexpr double cs2 = L::cs2;
    double s = 0.0;
    static_for<5>([&](auto A) {
        static_for<5>([&](auto B) {
            static_for<5>([&](auto Cc) {
                constexpr int a = int(A), b = int(B), c = int(Cc);
                if constexpr (L::basis(a, b, c)) {
                    constexpr double h = he(a, double(cx), cs2) * he(b, double(cy), cs2) * he(c, double(cz), cs2);
                    if constexpr (h != 0.0) s += h * C[a][b][c];
                }
            });
        });
    });
    return s;
}

template <class L, int MODE>
__device__ __forceinline__ void collide3(double (&v)[L::Q], const Relax& rx, int order, double eq_rho = 0.0,
                                         double eq_ux = 0.0, double eq_uy = 0.0, double eq_uz = 0.0)
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
                    C[a][b][c] = val * inv_norm3<L>(a, b, c);
                }
            });
        });
    });
    if constexpr (MODE == C3_PR) {
        // f^neq = f - f^eq, then a1 of every kept tensor of rank 2..order by
        // projection onto it
        static_for<L::Q>([&](auto I) { v[I] -= L::v.w[I] * hsum3<L, int(I)>(C); });
        static_for<5>([&](auto A) {
            static_for<5>([&](auto B) {
                static_for<5>([&](auto Cc) {
                    constexpr int a = int(A), b = int(B), c = int(Cc), n = a + b + c;
                    if constexpr (L::basis(a, b, c) && n >= 2) {
                        double p = 0.0;
                        static_for<L::Q>([&](auto I) {
                            constexpr double h = he(a, double(L::v.cx[I]), cs2) * he(b, double(L::v.cy[I]), cs2) *
                                                 he(c, double(L::v.cz[I]), cs2);
                            if constexpr (h != 0.0) p += h * v[I];
                        });
                        const double k = n == 2 ? rx.k2 : n == 3 ? rx.k3 : (n <= order ? rx.k4 : 0.0);
                        C[a][b][c] += k * p * inv_norm3<L>(a, b, c);
                    }
                });
            });
        });
    }
    static_for<L::Q>([&](auto I) {
        const double s = hsum3<L, int(I)>(C);
        constexpr double w = L::v.w[I];
        if constexpr (MODE == C3_BGK)
            v[I] = rx.k2 * v[I] + rx.inv_tau * (w * s);
        else
            v[I] = w * s;
    });
}

template <class L, int MODE, bool PULL>
__global__ __launch_bounds__(BX* BY) void k_stream_collide3(Step3Args a)
{
    constexpr int R = L::R;
    const int nx = a.lay.nx, ny = a.ny, nz = a.nz;
    const int x = int(blockIdx.x % unsigned(a.bx_blocks)) * BX + int(threadIdx.x);
    const int row = int(blockIdx.x / unsigned(a.bx_blocks)) * BY + int(threadIdx.y);
    if (x >= nx || row >= ny * nz) return;
    const int y = row % ny, z = row / ny;
    int xs[2 * R + 1], ys[2 * R + 1], zs[2 * R + 1];
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
        xs[D] = xx;
        ys[D] = yy;
        zs[D] = zz;
    });
    const double* fin = static_cast<const double*>(a.fin);
    double* fout = static_cast<double*>(a.fout);
    const int here = a.lay.row(row) + x;
    double v[L::Q];
    static_for<L::Q>([&](auto I) {
        constexpr int cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
        const int idx = PULL ? a.lay.row(zs[cz + R] * ny + ys[cy + R]) + xs[cx + R] : here;
        v[I] = fin[idx + int(I) * a.lay.te];
    });
    collide3<L, MODE>(v, a.rx, a.order);
    static_for<L::Q>([&](auto I) { __builtin_nontemporal_store(v[I], fout + here + int(I) * a.lay.te); });
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
template <class L>
__global__ __launch_bounds__(256) void k_init3(Init3Args a)
{
    const int64_t n = int64_t(a.lay.nx) * a.ny * a.nz;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int here = a.lay.row(int(k / a.lay.nx)) + int(k % a.lay.nx);
    double f[L::Q];
    const Relax none{ 0.0, 0.0, 0.0, 0.0 };
    collide3<L, C3_EQ>(f, none, a.eq_order, a.rho[k], a.ux[k], a.uy[k], a.uz[k]);
    double* out = static_cast<double*>(a.f);
    static_for<L::Q>([&](auto I) {
        double val = f[I];
        if (a.noise) val += a.noise_amp * L::v.w[I] * a.noise[int64_t(I) * n + k];
        out[here + int(I) * a.lay.te] = val;
    });
}

// rho, u per node and block sums of [rho, rho ux, rho uy, rho uz,
// sum f |c|^2 / 2, |u|^2, |u|^4, non-finite].
constexpr int MOM3_NS = 8;

template <class L>
__global__ __launch_bounds__(256) void k_moments3(const double* f, Layout lay, int ny, int nz, double* rho_o,
                                                  double* ux_o, double* uy_o, double* uz_o, double* partial)
{
    const int64_t n = int64_t(lay.nx) * ny * nz;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double val[MOM3_NS] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (k < n) {
        const int here = lay.row(int(k / lay.nx)) + int(k % lay.nx);
        double r = 0, jx = 0, jy = 0, jz = 0, e2 = 0;
        static_for<L::Q>([&](auto I) {
            constexpr double cx = L::v.cx[I], cy = L::v.cy[I], cz = L::v.cz[I];
            const double v = f[here + int(I) * lay.te];
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
