/*
 * Plain FP64 reference of the recursive-regularized LBM step on the 3D
 * lattices of Table II (E^19_{3,5} "D3Q19", E^27_{3,5} "D3Q27",
 * E^39_{3,7} "D3V39", E^103_{3,9} "D3Q103"), isothermal.
 *
 * TEST INFRASTRUCTURE ONLY: the tests may load it; the product library never
 * does.  It shares no code, header, table or constant with the HIP library.
 *
 * Written from the paper, on full index tuples:
 *   - Lattices from the symmetry groups and weights of Table II.
 *   - Hermite tensors by the recursion H^(n)_{a1..an} = c_an H^(n-1)_{a1..a(n-1)}
 *     - c_s^2 sum_{k<n} delta_{ak an} H^(n-2)_{without k, n} (Sec. II.A).
 *   - Equilibrium coefficients by the recursion of App. B,
 *     a0^(n) = u_an a0^(n-1) + (theta - 1) c_s^2 sum_k delta_{ak an} a0^(n-2).
 *   - a1^(2) by projection of f - f^(0) (Eq. a12Proj); RR builds every higher
 *     rank with the isothermal recursion Eq. (MalaspinasRecursiveRelation),
 *     a1^(n)_{a1..an} = u_an a1^(n-1)_{a1..a(n-1)}
 *                       + (1/rho) sum_{l<n} a0^(n-2)_{without l, n} a1^(2)_{al an};
 *     PR projects every rank; BGK relaxes f towards f^(0).
 *   - The collision of Eq. (GenRegCollision) as a full contraction over the
 *     tuples whose exponents (n_x, n_y, n_z) belong to the basis of Table II
 *     (multiplicities are implicit), and push streaming on a periodic box.
 * Tuples of rank n are numbered in base 3 (digit k = index a_(k+1), 0 x, 1 y,
 * 2 z) and stored from offset (3^n - 1) / 2.  Populations f[i][z][y][x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O3_MAXQ 103
#define O3_MAXN 6
#define O3_NT 1093 /* sum_{n <= 6} 3^n */

enum { O3_RR = 0, O3_PR = 1, O3_BGK = 2 };

typedef struct {
    int id, Q, nmax;
    int cx[O3_MAXQ], cy[O3_MAXQ], cz[O3_MAXQ];
    double w[O3_MAXQ];
    double cs2;
    double H[O3_MAXQ][O3_NT];
    unsigned char keep[O3_NT]; /* tuple in the basis of Table II */
} o3_lattice_t;

typedef struct {
    int a, b, c; /* representative a >= b >= c >= 0 of a symmetry group */
    double w;
} o3_group_t;

static int pow3(int n)
{
    int r = 1;
    for (int k = 0; k < n; ++k) r *= 3;
    return r;
}
static int t3off(int n) { return (pow3(n) - 1) / 2; }
static int digit(int b, int k) { return (b / pow3(k)) % 3; }
/* tuple b of rank n without its entries k and m (k < m), as rank n-2 */
static int drop2(int b, int n, int k, int m)
{
    int r = 0, p = 1;
    for (int j = 0; j < n; ++j) {
        if (j == k || j == m) continue;
        r += digit(b, j) * p;
        p *= 3;
    }
    return r;
}
/* tuple b of rank n without its last entry */
static int drop_last(int b, int n) { return b % pow3(n - 1); }
static void exponents(int b, int n, int e[3])
{
    e[0] = e[1] = e[2] = 0;
    for (int k = 0; k < n; ++k) e[digit(b, k)]++;
}
static double fact(int n)
{
    double r = 1;
    for (int k = 2; k <= n; ++k) r *= k;
    return r;
}

/* Table II, lower part: which tensors each lattice keeps. */
static int in_basis3(int id, const int e[3])
{
    const int n = e[0] + e[1] + e[2];
    switch (id) {
    case 0: { /* D3Q19: ranks 0-2, and rank 3 of the xxy kind only */
        if (n <= 2) return 1;
        if (n != 3) return 0;
        int two = 0, one = 0;
        for (int a = 0; a < 3; ++a) {
            two += e[a] == 2;
            one += e[a] == 1;
        }
        return two == 1 && one == 1;
    }
    case 1: /* D3Q27: every exponent at most 2 (the complete basis) */
        return e[0] <= 2 && e[1] <= 2 && e[2] <= 2;
    case 2: /* D3V39: every tensor of rank <= 3 */
        return n <= 3;
    case 3: /* D3Q103: every tensor of rank <= 4 */
        return n <= 4;
    }
    return 0;
}

static int cmp3(const void* pa, const void* pb)
{
    const int* a = (const int*)pa;
    const int* b = (const int*)pb;
    if (a[2] != b[2]) return a[2] - b[2];
    if (a[1] != b[1]) return a[1] - b[1];
    return a[0] - b[0];
}

static int build3(int id, o3_lattice_t* L)
{
    static const o3_group_t g19[] = { { 0, 0, 0, 1.0 / 3.0 }, { 1, 0, 0, 1.0 / 18.0 }, { 1, 1, 0, 1.0 / 36.0 } };
    static const o3_group_t g27[] = { { 0, 0, 0, 8.0 / 27.0 }, { 1, 0, 0, 2.0 / 27.0 }, { 1, 1, 0, 1.0 / 54.0 },
                                      { 1, 1, 1, 1.0 / 216.0 } };
    static const o3_group_t g39[] = { { 0, 0, 0, 1.0 / 12.0 }, { 1, 0, 0, 1.0 / 12.0 }, { 1, 1, 1, 1.0 / 27.0 },
                                      { 2, 0, 0, 2.0 / 135.0 }, { 2, 2, 0, 1.0 / 432.0 }, { 3, 0, 0, 1.0 / 1620.0 } };
    /* D3Q103: weights as printed in Table II (21 digits), c_s = 1 / 1.19697977039307435897239 */
    static const o3_group_t g103[] = {
        { 0, 0, 0, 0.032633351764471159466 }, { 1, 0, 0, 0.097656833590334574221 },
        { 1, 1, 1, 0.028097750290257335627 }, { 2, 0, 0, 0.001045259560430061466 },
        { 2, 1, 0, 0.005705329016894815990 }, { 2, 2, 0, 0.000611939269829747839 },
        { 2, 2, 2, 0.000155964159374283722 }, { 3, 0, 0, 0.000284443251800055207 },
        { 3, 1, 1, 0.000130698375985191585 }, { 3, 3, 3, 0.000001223194501323058 }
    };
    const double inv_cs103 = 1.19697977039307435897239;
    const o3_group_t* g;
    int ng;
    switch (id) {
    case 0: g = g19; ng = 3; L->cs2 = 1.0 / 3.0; L->nmax = 3; break;
    case 1: g = g27; ng = 4; L->cs2 = 1.0 / 3.0; L->nmax = 6; break;
    case 2: g = g39; ng = 6; L->cs2 = 2.0 / 3.0; L->nmax = 3; break;
    case 3: g = g103; ng = 10; L->cs2 = 1.0 / (inv_cs103 * inv_cs103); L->nmax = 4; break;
    default: return -1;
    }
    L->id = id;
    int list[O3_MAXQ][4];
    int q = 0;
    for (int z = -3; z <= 3; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                int s[3] = { abs(x), abs(y), abs(z) };
                /* sort descending */
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2 - i; ++j)
                        if (s[j] < s[j + 1]) {
                            int t = s[j];
                            s[j] = s[j + 1];
                            s[j + 1] = t;
                        }
                for (int k = 0; k < ng; ++k)
                    if (g[k].a == s[0] && g[k].b == s[1] && g[k].c == s[2]) {
                        if (q >= O3_MAXQ) return -1;
                        list[q][0] = x;
                        list[q][1] = y;
                        list[q][2] = z;
                        list[q][3] = k;
                        ++q;
                    }
            }
    qsort(list, (size_t)q, sizeof(list[0]), cmp3);
    L->Q = q;
    for (int i = 0; i < q; ++i) {
        L->cx[i] = list[i][0];
        L->cy[i] = list[i][1];
        L->cz[i] = list[i][2];
        L->w[i] = g[list[i][3]].w;
    }
    for (int n = 0; n <= O3_MAXN; ++n)
        for (int b = 0; b < pow3(n); ++b) {
            int e[3];
            exponents(b, n, e);
            L->keep[t3off(n) + b] = (unsigned char)in_basis3(id, e);
        }
    /* Hermite tensors of every rank up to O3_MAXN at every velocity */
    for (int i = 0; i < q; ++i) {
        const double c[3] = { L->cx[i], L->cy[i], L->cz[i] };
        double* H = L->H[i];
        H[0] = 1.0;
        for (int n = 1; n <= O3_MAXN; ++n)
            for (int b = 0; b < pow3(n); ++b) {
                const int an = digit(b, n - 1);
                double v = c[an] * H[t3off(n - 1) + drop_last(b, n)];
                for (int k = 0; k < n - 1; ++k)
                    if (digit(b, k) == an) v -= L->cs2 * H[t3off(n - 2) + drop2(b, n, k, n - 1)];
                H[t3off(n) + b] = v;
            }
    }
    return 0;
}

/* a0 of every rank up to O3_MAXN (App. B). */
static void eq3(const o3_lattice_t* L, double rho, const double u[3], double theta, double* a0)
{
    a0[0] = rho;
    for (int n = 1; n <= O3_MAXN; ++n)
        for (int b = 0; b < pow3(n); ++b) {
            const int an = digit(b, n - 1);
            double v = u[an] * a0[t3off(n - 1) + drop_last(b, n)];
            if (n >= 2)
                for (int k = 0; k < n - 1; ++k)
                    if (digit(b, k) == an) v += (theta - 1.0) * L->cs2 * a0[t3off(n - 2) + drop2(b, n, k, n - 1)];
            a0[t3off(n) + b] = v;
        }
}

/* f_i = w_i sum_{n <= nmax} 1/(n! c_s^2n) sum_{b in basis} H_b(c_i) a_b */
static void hsum3(const o3_lattice_t* L, const double* a, int nmax, double* f)
{
    for (int i = 0; i < L->Q; ++i) {
        double s = 0;
        for (int n = 0; n <= nmax; ++n) {
            const int o = t3off(n), m = pow3(n);
            double sn = 0;
            for (int b = 0; b < m; ++b)
                if (L->keep[o + b]) sn += L->H[i][o + b] * a[o + b];
            s += sn / (fact(n) * pow(L->cs2, n));
        }
        f[i] = L->w[i] * s;
    }
}

static void moments3(const o3_lattice_t* L, const double* f, double* rho, double u[3])
{
    double r = 0, j[3] = { 0, 0, 0 };
    for (int i = 0; i < L->Q; ++i) {
        r += f[i];
        j[0] += L->cx[i] * f[i];
        j[1] += L->cy[i] * f[i];
        j[2] += L->cz[i] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

/* Non-equilibrium coefficients of every rank up to the lattice's maximum. */
static void noneq3(const o3_lattice_t* L, int coll, const double* f, double rho, const double u[3],
                   const double* a0, const double* feq, double* a1)
{
    double g[O3_MAXQ];
    for (int i = 0; i < L->Q; ++i) g[i] = f[i] - feq[i];
    for (int t = 0; t < O3_NT; ++t) a1[t] = 0.0;
    for (int n = 2; n <= L->nmax; ++n) {
        if (coll == O3_RR && n >= 3) {
            for (int b = 0; b < pow3(n); ++b) {
                const int an = digit(b, n - 1);
                const int prev = drop_last(b, n);
                double v = u[an] * a1[t3off(n - 1) + prev];
                for (int l = 0; l < n - 1; ++l) {
                    const int al = digit(b, l);
                    const int pair = al + 3 * an;
                    v += a0[t3off(n - 2) + drop2(b, n, l, n - 1)] * a1[t3off(2) + pair] / rho;
                }
                a1[t3off(n) + b] = v;
            }
        } else {
            for (int b = 0; b < pow3(n); ++b) {
                double s = 0;
                for (int i = 0; i < L->Q; ++i) s += L->H[i][t3off(n) + b] * g[i];
                a1[t3off(n) + b] = s;
            }
        }
    }
}

/* Relaxation times: tau for rank 2 (and BGK), tau3 for rank 3, tau4 for every
 * rank >= 4 (the Hermite MRT form of Eq. GenRegCollision with one time per
 * order; tau3 = tau4 = tau is the single-time operator). */
typedef struct {
    double tau, tau3, tau4;
} o3_times_t;

static void collide3(const o3_lattice_t* L, int coll, int order, o3_times_t tt, const double* f, double* out)
{
    double rho, u[3];
    moments3(L, f, &rho, u);
    double a0[O3_NT], feq[O3_MAXQ];
    eq3(L, rho, u, 1.0, a0);
    hsum3(L, a0, L->nmax, feq);
    if (coll == O3_BGK) {
        for (int i = 0; i < L->Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / tt.tau;
        return;
    }
    double a1[O3_NT], a[O3_NT];
    noneq3(L, coll, f, rho, u, a0, feq, a1);
    const double k2 = 1.0 - 1.0 / tt.tau, k3 = 1.0 - 1.0 / tt.tau3, k4 = 1.0 - 1.0 / tt.tau4;
    for (int n = 0; n <= O3_MAXN; ++n)
        for (int b = 0; b < pow3(n); ++b) {
            double v = a0[t3off(n) + b];
            if (n >= 2 && n <= order) v += (n == 2 ? k2 : n == 3 ? k3 : k4) * a1[t3off(n) + b];
            a[t3off(n) + b] = v;
        }
    hsum3(L, a, L->nmax, out);
}

static int check3(const o3_lattice_t* L, int coll, int order, double tau)
{
    if (coll < O3_RR || coll > O3_BGK) return -2;
    if (coll != O3_BGK && (order < 2 || order > L->nmax)) return -3;
    if (!(tau > 0.5) || !isfinite(tau)) return -4;
    return 0;
}

/* ---- Exported API ------------------------------------------------------ */

int o3_lattice(int id, int* Q, int* nmax, double* cs2, int* cx, int* cy, int* cz, double* w)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
    if (Q) *Q = L.Q;
    if (nmax) *nmax = L.nmax;
    if (cs2) *cs2 = L.cs2;
    for (int i = 0; i < L.Q; ++i) {
        if (cx) cx[i] = L.cx[i];
        if (cy) cy[i] = L.cy[i];
        if (cz) cz[i] = L.cz[i];
        if (w) w[i] = L.w[i];
    }
    return 0;
}

/* basis mask over the tuples of rank n: mask[b] = 1 if kept */
int o3_basis(int id, int n, int* mask)
{
    if (n < 0 || n > O3_MAXN) return -1;
    for (int b = 0; b < pow3(n); ++b) {
        int e[3];
        exponents(b, n, e);
        mask[b] = in_basis3(id, e);
    }
    return 0;
}

/* Hermite tensors of rank n at every velocity: H[i * 3^n + b] */
int o3_hermite(int id, int n, double* H)
{
    static o3_lattice_t L;
    if (build3(id, &L) || n < 0 || n > O3_MAXN) return -1;
    for (int i = 0; i < L.Q; ++i)
        for (int b = 0; b < pow3(n); ++b) H[(int64_t)i * pow3(n) + b] = L.H[i][t3off(n) + b];
    return 0;
}

int o3_equilibrium(int id, int64_t n, const double* rho, const double* ux, const double* uy, const double* uz,
                   double* feq)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double a0[O3_NT], fl[O3_MAXQ];
        const double u[3] = { ux[k], uy[k], uz[k] };
        eq3(&L, rho[k], u, 1.0, a0);
        hsum3(&L, a0, L.nmax, fl);
        for (int i = 0; i < L.Q; ++i) feq[(int64_t)i * n + k] = fl[i];
    }
    return 0;
}

/* Non-equilibrium coefficients of one node (all ranks, full tuples). */
int o3_noneq(int id, int coll, const double* f, double* a1)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
    double rho, u[3], a0[O3_NT], feq[O3_MAXQ];
    moments3(&L, f, &rho, u);
    eq3(&L, rho, u, 1.0, a0);
    hsum3(&L, a0, L.nmax, feq);
    noneq3(&L, coll, f, rho, u, a0, feq, a1);
    return 0;
}

int o3_collide_mrt(int id, int coll, int order, double tau, double tau3, double tau4, int64_t n, const double* f,
                    double* out)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
    int e = check3(&L, coll, order, tau);
    if (e) return e;
    if (!(tau3 > 0.5) || !isfinite(tau3) || !(tau4 > 0.5) || !isfinite(tau4)) return -4;
    const o3_times_t tt = { tau, tau3, tau4 };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[O3_MAXQ], fo[O3_MAXQ];
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        collide3(&L, coll, order, tt, fl, fo);
        for (int i = 0; i < L.Q; ++i) out[(int64_t)i * n + k] = fo[i];
    }
    return 0;
}

/* nsteps of collide-then-stream (push) on a periodic nx x ny x nz box. */
int o3_step_mrt(int id, int coll, int order, double tau, double tau3, double tau4, int nx, int ny, int nz, int nsteps,
                 double* f, double* tmp)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
    int e = check3(&L, coll, order, tau);
    if (e) return e;
    if (!(tau3 > 0.5) || !isfinite(tau3) || !(tau4 > 0.5) || !isfinite(tau4)) return -4;
    const o3_times_t tt = { tau, tau3, tau4 };
    if (nx < 1 || ny < 1 || nz < 1) return -5;
    const int64_t n = (int64_t)nx * ny * nz;
    for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double fl[O3_MAXQ], fo[O3_MAXQ];
                    const int64_t k = ((int64_t)z * ny + y) * nx + x;
                    for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
                    collide3(&L, coll, order, tt, fl, fo);
                    for (int i = 0; i < L.Q; ++i) {
                        const int xd = ((x + L.cx[i]) % nx + nx) % nx;
                        const int yd = ((y + L.cy[i]) % ny + ny) % ny;
                        const int zd = ((z + L.cz[i]) % nz + nz) % nz;
                        tmp[(int64_t)i * n + ((int64_t)zd * ny + yd) * nx + xd] = fo[i];
                    }
                }
        memcpy(f, tmp, sizeof(double) * (size_t)(n * L.Q));
    }
    return 0;
}

int o3_collide(int id, int coll, int order, double tau, int64_t n, const double* f, double* out)
{
    return o3_collide_mrt(id, coll, order, tau, tau, tau, n, f, out);
}

int o3_step(int id, int coll, int order, double tau, int nx, int ny, int nz, int nsteps, double* f, double* tmp)
{
    return o3_step_mrt(id, coll, order, tau, tau, tau, nx, ny, nz, nsteps, f, tmp);
}

int o3_moments(int id, int64_t n, const double* f, double* rho, double* ux, double* uy, double* uz)
{
    static o3_lattice_t L;
    if (build3(id, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[O3_MAXQ], r, u[3];
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        moments3(&L, fl, &r, u);
        rho[k] = r;
        ux[k] = u[0];
        uy[k] = u[1];
        uz[k] = u[2];
    }
    return 0;
}
