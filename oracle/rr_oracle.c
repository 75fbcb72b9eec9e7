/*
 * rr_oracle.c -- plain FP64 CPU reference of the recursive-regularized lattice
 * Boltzmann step (Coreixas, Wissocq, Puigt, Boussuge, Sagaut, "Recursive
 * regularization step for high-order lattice Boltzmann methods").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code,
 * header, table or constant with the HIP library: every lattice constant below
 * is retyped from Table I of the paper and every step is written from the
 * paper's equations in their own order and notation.
 *
 * Conventions
 *   - Lattice units: integer velocities c_i (on-grid condition, Sec. III.A),
 *     c_s^2 = r T_0 from the last row of Table I.
 *   - A rank-n Hermite tensor component is addressed by an n-bit pattern:
 *     bit j set means index alpha_{j+1} = y, clear means x.  The component of
 *     rank n with pattern b is stored at offset (2^n - 1) + b, so ranks 0..4
 *     occupy 31 slots.  Every contraction below runs over all 2^n index tuples,
 *     which is the paper's full contraction ":"; the multiplicities A^(n)
 *     of Eq. (GenRegCollision) are therefore implicit.
 *   - Populations are laid out f[i][y][x] (x fastest) with the velocities in
 *     canonical order: ascending c_y, then ascending c_x.
 *   - Floating point: IEEE double, built with -O2 -ffp-contract=off, no
 *     fast-math.
 *
 * Parity status: every function here is pinned by a CPU test (quadrature and
 * Hermite orthogonality, the closed-form equilibrium, Gauss-Hermite
 * integration of the Maxwellian, the 2D closed forms of App. C, conservation,
 * the fixed point, RR2 == PR2, PR4 == BGK on D2Q9, shear-wave decay).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 37
#define ORC_NT 31 /* tensor slots for ranks 0..4 */

enum { ORC_D2Q9 = 0, ORC_D2V17 = 1, ORC_D2V37 = 2 };
enum { ORC_RR = 0, ORC_PR = 1, ORC_BGK = 2 };

typedef struct {
    int Q;
    int n_eq;                /* highest Hermite order of the lattice basis   */
    double cs2;              /* c_s^2 in lattice units                        */
    int cx[ORC_MAXQ], cy[ORC_MAXQ];
    double w[ORC_MAXQ];
    int basis[5][5];         /* basis[nx][ny] = 1 if H^(nx x's, ny y's) kept  */
    double H[ORC_MAXQ][ORC_NT]; /* Hermite tensors evaluated at every c_i     */
} orc_lattice_t;

typedef struct {
    int coll;       /* ORC_RR, ORC_PR or ORC_BGK                             */
    int order;      /* regularization order N, 2 <= N <= n_eq                */
    int thermal;    /* 0: isothermal (theta = 1), 1: thermal/compressible    */
    int a13_raw;    /* thermal RR: 1 keeps the projected a1^(3) (Sec. II.F), */
                    /* 0 rebuilds it from the averaged gradient (App. C)     */
    double tau;     /* discrete relaxation time (tau-bar of Sec. III.A)      */
    double tau3;    /* relaxation time of the rank-3 coefficients (= tau     */
    double tau4;    /* unless per order, Eq. GenRegCollision), and rank 4   */
} orc_cfg_t;

static int toff(int n, int b) { return (1 << n) - 1 + b; }
static int axis_of(int b, int j) { return (b >> j) & 1; }
static int remove_idx(int b, int i)
{
    int lower = b & ((1 << i) - 1);
    int upper = b >> (i + 1);
    return lower | (upper << i);
}
static int popcount5(int b)
{
    int c = 0;
    while (b) { c += b & 1; b >>= 1; }
    return c;
}
static double fact(int n) { double r = 1; for (int k = 2; k <= n; ++k) r *= k; return r; }
static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* ---- Table I: velocity groups and weights ------------------------------ */

typedef struct { int a, b; double w; } orc_group_t;

static int cmp_vel(const void* pa, const void* pb)
{
    const int* a = (const int*)pa;
    const int* b = (const int*)pb;
    if (a[1] != b[1]) return a[1] - b[1];
    return a[0] - b[0];
}

/* Expand groups by reflections and the x<->y permutation, then sort. */
static void expand_groups(const orc_group_t* g, int ng, orc_lattice_t* L)
{
    int vel[ORC_MAXQ][3];
    double wt[ORC_MAXQ];
    int q = 0;
    for (int k = 0; k < ng; ++k) {
        int cand[8][2] = {
            { g[k].a, g[k].b }, { -g[k].a, g[k].b }, { g[k].a, -g[k].b }, { -g[k].a, -g[k].b },
            { g[k].b, g[k].a }, { -g[k].b, g[k].a }, { g[k].b, -g[k].a }, { -g[k].b, -g[k].a },
        };
        for (int m = 0; m < 8; ++m) {
            int dup = 0;
            for (int p = 0; p < q; ++p)
                if (vel[p][0] == cand[m][0] && vel[p][1] == cand[m][1]) dup = 1;
            if (!dup) {
                vel[q][0] = cand[m][0];
                vel[q][1] = cand[m][1];
                vel[q][2] = q;
                wt[q] = g[k].w;
                ++q;
            }
        }
    }
    qsort(vel, (size_t)q, sizeof(vel[0]), cmp_vel);
    L->Q = q;
    for (int i = 0; i < q; ++i) {
        L->cx[i] = vel[i][0];
        L->cy[i] = vel[i][1];
        L->w[i] = wt[vel[i][2]];
    }
}

/* Hermite tensors up to rank 4, App. C (explicit definitions with deltas). */
static double herm(int n, int b, double cx, double cy, double cs2)
{
    double xi[2] = { cx, cy };
    int a[4];
    for (int j = 0; j < n; ++j) a[j] = axis_of(b, j);
    switch (n) {
    case 0:
        return 1.0;
    case 1:
        return xi[a[0]];
    case 2:
        return xi[a[0]] * xi[a[1]] - cs2 * kd(a[0], a[1]);
    case 3:
        return xi[a[0]] * xi[a[1]] * xi[a[2]]
             - cs2 * (xi[a[0]] * kd(a[1], a[2]) + xi[a[1]] * kd(a[0], a[2]) + xi[a[2]] * kd(a[0], a[1]));
    case 4:
        return xi[a[0]] * xi[a[1]] * xi[a[2]] * xi[a[3]]
             - cs2 * (xi[a[0]] * xi[a[1]] * kd(a[2], a[3]) + xi[a[0]] * xi[a[2]] * kd(a[1], a[3])
                      + xi[a[0]] * xi[a[3]] * kd(a[1], a[2]) + xi[a[1]] * xi[a[2]] * kd(a[0], a[3])
                      + xi[a[1]] * xi[a[3]] * kd(a[0], a[2]) + xi[a[2]] * xi[a[3]] * kd(a[0], a[1]))
             + cs2 * cs2 * (kd(a[0], a[1]) * kd(a[2], a[3]) + kd(a[0], a[2]) * kd(a[1], a[3])
                            + kd(a[0], a[3]) * kd(a[1], a[2]));
    }
    return 0.0;
}

static int build_lattice(int id, orc_lattice_t* L)
{
    memset(L, 0, sizeof(*L));
    if (id == ORC_D2Q9) {
        /* E^9_{2,5}; the weights of groups (1,1) and (2,0) printed in Table I
         * do not sum to one; the standard D2Q9 set (4/9, 1/9, 1/36 on
         * (0,0), (1,0), (1,1)) is the one consistent with c_s^2 = 1/3 and with
         * the basis marks of the same table. */
        orc_group_t g[3] = { { 0, 0, 4.0 / 9.0 }, { 1, 0, 1.0 / 9.0 }, { 1, 1, 1.0 / 36.0 } };
        expand_groups(g, 3, L);
        L->cs2 = 1.0 / 3.0;
        int keep[5][5] = { { 1, 1, 1, 0, 0 }, { 1, 1, 1, 0, 0 }, { 1, 1, 1, 0, 0 }, { 0 }, { 0 } };
        /* basis: 1, x, y, xx, xy, yy, xxy, xyy, xxyy */
        memcpy(L->basis, keep, sizeof(keep));
        L->n_eq = 4;
    } else if (id == ORC_D2V17) {
        const double s = sqrt(193.0);
        orc_group_t g[5] = {
            { 0, 0, (575.0 + 193.0 * s) / 8100.0 },
            { 1, 0, (3355.0 - 91.0 * s) / 18000.0 },
            { 1, 1, (655.0 + 17.0 * s) / 27000.0 },
            { 2, 2, (685.0 - 49.0 * s) / 54000.0 },
            { 3, 0, (1445.0 - 101.0 * s) / 162000.0 },
        };
        expand_groups(g, 5, L);
        L->cs2 = 72.0 / (5.0 * (25.0 + s)); /* (1/c_s)^2 = 5(25+sqrt193)/72 */
        /* basis: all Hermite tensors of rank <= 3 */
        for (int nx = 0; nx <= 4; ++nx)
            for (int ny = 0; ny <= 4; ++ny) L->basis[nx][ny] = (nx + ny <= 3);
        L->n_eq = 3;
    } else if (id == ORC_D2V37) {
        orc_group_t g[8] = {
            { 0, 0, 0.23315066913235250228650 }, { 1, 0, 0.10730609154221900241246 },
            { 1, 1, 0.05766785988879488203006 }, { 2, 0, 0.01420821615845075026469 },
            { 2, 1, 0.00535304900051377523273 }, { 2, 2, 0.00101193759267357547541 },
            { 3, 0, 0.00024530102775771734547 }, { 3, 1, 0.00028341425299419821740 },
        };
        expand_groups(g, 8, L);
        const double inv_cs = 1.19697977039307435897239;
        L->cs2 = 1.0 / (inv_cs * inv_cs);
        /* basis: all Hermite tensors of rank <= 4 */
        for (int nx = 0; nx <= 4; ++nx)
            for (int ny = 0; ny <= 4; ++ny) L->basis[nx][ny] = (nx + ny <= 4);
        L->n_eq = 4;
    } else {
        return -1;
    }
    for (int i = 0; i < L->Q; ++i)
        for (int n = 0; n <= 4; ++n)
            for (int b = 0; b < (1 << n); ++b)
                L->H[i][toff(n, b)] = herm(n, b, (double)L->cx[i], (double)L->cy[i], L->cs2);
    return 0;
}

static int in_basis(const orc_lattice_t* L, int n, int b)
{
    int ny = popcount5(b);
    return L->basis[n - ny][ny];
}

/* ---- Per-node building blocks ------------------------------------------ */

/* Macroscopic moments (Sec. II.A): rho, u and theta from
 * sum f |c|^2 - rho |u|^2 = D rho c_s^2 theta (D = 2, c_s^2 = r T_0). */
static void node_moments(const orc_lattice_t* L, const double* f, int thermal,
                         double* rho, double* ux, double* uy, double* theta)
{
    double r = 0, jx = 0, jy = 0, e2 = 0;
    for (int i = 0; i < L->Q; ++i) {
        r += f[i];
        jx += f[i] * L->cx[i];
        jy += f[i] * L->cy[i];
        e2 += f[i] * (double)(L->cx[i] * L->cx[i] + L->cy[i] * L->cy[i]);
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
    if (thermal)
        *theta = (e2 - r * (*ux * *ux + *uy * *uy)) / (2.0 * r * L->cs2);
    else
        *theta = 1.0;
}

/* Equilibrium Hermite coefficients by the recursion of App. B:
 * a0^(n)_{a1..an} = u_{an} a0^(n-1)_{a1..a(n-1)}
 *                   + (theta-1) c_s^2 sum_{i<n} delta_{ai an} a0^(n-2)_{beta_i}. */
static void eq_coeffs(const orc_lattice_t* L, double rho, double ux, double uy, double theta,
                      double* a0)
{
    const double u[2] = { ux, uy };
    const double sig = (theta - 1.0) * L->cs2;
    memset(a0, 0, sizeof(double) * ORC_NT);
    a0[0] = rho;
    for (int n = 1; n <= 4; ++n) {
        for (int b = 0; b < (1 << n); ++b) {
            int an = axis_of(b, n - 1);
            int prev = b & ((1 << (n - 1)) - 1);
            double v = u[an] * a0[toff(n - 1, prev)];
            for (int i = 0; i < n - 1; ++i)
                if (axis_of(prev, i) == an) v += sig * a0[toff(n - 2, remove_idx(prev, i))];
            a0[toff(n, b)] = v;
        }
    }
}

/* f_i = w_i sum_{n <= nmax} 1/(n! c_s^2n) sum_alpha H^(n)_{i,alpha} a^(n)_alpha,
 * restricted to the lattice basis (App. D, Eq. GenRegCollision with A^(n)
 * implicit in the full contraction). */
static void hermite_sum(const orc_lattice_t* L, const double* a, int nmax, double* f)
{
    for (int i = 0; i < L->Q; ++i) {
        double s = 0;
        for (int n = 0; n <= nmax; ++n) {
            double scale = 1.0 / (fact(n) * pow(L->cs2, (double)n));
            double sn = 0;
            for (int b = 0; b < (1 << n); ++b)
                if (in_basis(L, n, b)) sn += L->H[i][toff(n, b)] * a[toff(n, b)];
            s += scale * sn;
        }
        f[i] = L->w[i] * s;
    }
}

/* Projection of g onto the rank-n Hermite tensors: sum_i H^(n)_{i,alpha} g_i. */
static void project(const orc_lattice_t* L, const double* g, int n, double* a)
{
    for (int b = 0; b < (1 << n); ++b) {
        double s = 0;
        for (int i = 0; i < L->Q; ++i) s += L->H[i][toff(n, b)] * g[i];
        a[toff(n, b)] = s;
    }
}

static int pair_bits(int a, int b) { return a | (b << 1); }
static int triple_bits(int a, int b, int c) { return a | (b << 1) | (c << 2); }

/* Isothermal recursion (Malaspinas; Eq. MalaspinasRecursiveRelation), n >= 3:
 * a1^(n)_{a1..an} = u_{an} a1^(n-1)_{a1..a(n-1)}
 *                   + (1/rho) sum_{l<n} a0^(n-2)_{beta_l} a1^(2)_{al an}. */
static void rr_isothermal(const double* u, double rho, const double* a0, double* a1)
{
    for (int n = 3; n <= 4; ++n) {
        for (int b = 0; b < (1 << n); ++b) {
            int an = axis_of(b, n - 1);
            int prev = b & ((1 << (n - 1)) - 1);
            double v = u[an] * a1[toff(n - 1, prev)];
            for (int l = 0; l < n - 1; ++l)
                v += a0[toff(n - 2, remove_idx(prev, l))] * a1[toff(2, pair_bits(axis_of(prev, l), an))] / rho;
            a1[toff(n, b)] = v;
        }
    }
}

/* Thermal recursion (Eq. RecursiveRelation_ThermalCase), n >= 4. */
static void rr_thermal_high(const double* u, double rho, double theta, double cs2,
                            const double* a0, double* a1)
{
    const double sig = cs2 * (theta - 1.0);
    const int n = 4;
    for (int b = 0; b < (1 << n); ++b) {
        int an = axis_of(b, n - 1);
        int prev = b & ((1 << (n - 1)) - 1);
        double v = u[an] * a1[toff(n - 1, prev)];
        for (int l = 0; l < n - 1; ++l) {
            int al = axis_of(prev, l);
            int rest = remove_idx(prev, l);
            if (al == an) v += sig * a1[toff(n - 2, rest)];
            v += a0[toff(n - 2, rest)] * a1[toff(2, pair_bits(al, an))] / rho;
        }
        for (int l = 0; l < n - 1; ++l) {
            for (int m = l + 1; m < n - 1; ++m) {
                int al = axis_of(prev, l), am = axis_of(prev, m);
                int rest = remove_idx(remove_idx(prev, m), l);
                double t = a1[toff(3, triple_bits(al, am, an))]
                         - u[al] * a1[toff(2, pair_bits(am, an))]
                         - u[am] * a1[toff(2, pair_bits(al, an))]
                         - u[an] * a1[toff(2, pair_bits(al, am))];
                v += a0[toff(n - 3, rest)] * t / rho;
            }
        }
        a1[toff(n, b)] = v;
    }
}

/* Thermal a1^(3), App. C: project, average the two estimates of
 * mu c_s^2 grad(theta) (Eq. TempGradLBM), rebuild with Eq. a1Rec. */
static void rr_thermal_a13(const double* u, const double* p3, double* a1)
{
    double a2[2][2];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) a2[p][q] = a1[toff(2, pair_bits(p, q))];
    double P3[2][2][2];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
            for (int r = 0; r < 2; ++r) P3[p][q][r] = p3[toff(3, triple_bits(p, q, r))];
    double G[2];
    for (int d = 0; d < 2; ++d) {
        int o = 1 - d;
        double est1 = u[d] * a2[d][d] - P3[d][d][d] / 3.0;
        double est2 = 2.0 * u[o] * a2[d][o] + u[d] * a2[o][o] - P3[d][o][o];
        G[d] = 0.5 * (est1 + est2);
    }
    for (int b = 0; b < 8; ++b) {
        int A = axis_of(b, 0), B = axis_of(b, 1), C = axis_of(b, 2);
        a1[toff(3, b)] = u[A] * a2[B][C] + u[B] * a2[A][C] + u[C] * a2[A][B]
                       - (kd(A, B) * G[C] + kd(A, C) * G[B] + kd(B, C) * G[A]);
    }
}

/* Non-equilibrium coefficients a1 for one node (before truncation). */
static void noneq_coeffs(const orc_lattice_t* L, const orc_cfg_t* c, const double* f,
                         const double* feq, double rho, const double* u, double theta,
                         const double* a0, double* a1)
{
    double g[ORC_MAXQ];
    for (int i = 0; i < L->Q; ++i) g[i] = f[i] - feq[i];
    memset(a1, 0, sizeof(double) * ORC_NT);
    project(L, g, 2, a1); /* a1^(2), Eq. a12Proj */
    if (c->coll == ORC_PR) {
        for (int n = 3; n <= 4; ++n) project(L, g, n, a1);
        return;
    }
    if (!c->thermal) {
        rr_isothermal(u, rho, a0, a1);
        return;
    }
    double p3[ORC_NT];
    project(L, g, 3, p3);
    if (c->a13_raw) {
        for (int b = 0; b < 8; ++b) a1[toff(3, b)] = p3[toff(3, b)];
    } else {
        rr_thermal_a13(u, p3, a1);
    }
    rr_thermal_high(u, rho, theta, L->cs2, a0, a1);
}

/* One collision at one node: Eq. RegularizedCollision / GenRegCollision with a
 * single tau; BGK per the explicit scheme of Sec. III.A. */
static void node_collide(const orc_lattice_t* L, const orc_cfg_t* c, const double* f, double* out)
{
    double rho, u[2], theta;
    node_moments(L, f, c->thermal, &rho, &u[0], &u[1], &theta);
    double a0[ORC_NT], feq[ORC_MAXQ];
    eq_coeffs(L, rho, u[0], u[1], theta, a0);
    hermite_sum(L, a0, L->n_eq, feq);
    if (c->coll == ORC_BGK) {
        for (int i = 0; i < L->Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / c->tau;
        return;
    }
    double a1[ORC_NT];
    noneq_coeffs(L, c, f, feq, rho, u, theta, a0, a1);
    /* truncation: only ranks 2..N of the basis carry a non-equilibrium part;
     * rank n relaxes with its own tau_n (Eq. GenRegCollision with one time per
     * order, the Hermite MRT form), tau_2 = tau */
    double a[ORC_NT];
    const double kn[5] = { 0.0, 0.0, 1.0 - 1.0 / c->tau, 1.0 - 1.0 / c->tau3, 1.0 - 1.0 / c->tau4 };
    for (int n = 0; n <= 4; ++n)
        for (int b = 0; b < (1 << n); ++b) {
            double v = a0[toff(n, b)];
            if (n >= 2 && n <= c->order) v += kn[n] * a1[toff(n, b)];
            a[toff(n, b)] = v;
        }
    hermite_sum(L, a, L->n_eq, out);
}

/* ---- Exported API ------------------------------------------------------ */

/* Threads the parallel loops use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Fills Q, n_eq, c_s^2, velocities (canonical order) and weights.
 * cx, cy, w may be NULL.  Returns 0, or -1 for an unknown lattice. */
int orc_lattice(int id, int* Q, int* n_eq, double* cs2, int* cx, int* cy, double* w)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    if (Q) *Q = L.Q;
    if (n_eq) *n_eq = L.n_eq;
    if (cs2) *cs2 = L.cs2;
    for (int i = 0; i < L.Q; ++i) {
        if (cx) cx[i] = L.cx[i];
        if (cy) cy[i] = L.cy[i];
        if (w) w[i] = L.w[i];
    }
    return 0;
}

/* Basis membership: out[nx*5+ny] = 1 if the tensor with nx x's and ny y's
 * belongs to the lattice basis (Table I, bottom). */
int orc_basis(int id, int* out)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    for (int nx = 0; nx < 5; ++nx)
        for (int ny = 0; ny < 5; ++ny) out[nx * 5 + ny] = L.basis[nx][ny];
    return 0;
}

/* Hermite tensor table H[i*31 + slot]. */
int orc_hermite_table(int id, double* H)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    for (int i = 0; i < L.Q; ++i)
        for (int s = 0; s < ORC_NT; ++s) H[i * ORC_NT + s] = L.H[i][s];
    return 0;
}

/* Equilibrium Hermite coefficients (31 slots) of (rho, u, theta). */
int orc_eq_coeffs(int id, double rho, double ux, double uy, double theta, double* a0)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    eq_coeffs(&L, rho, ux, uy, theta, a0);
    return 0;
}

/* Non-equilibrium coefficients a1 (31 slots, before truncation) of one node's
 * populations f[Q]. */
int orc_noneq_coeffs(int id, int coll, int thermal, int a13_raw, const double* f, double* a1)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    orc_cfg_t c = { coll, 4, thermal, a13_raw, 1.0, 1.0, 1.0 };
    double rho, u[2], theta, a0[ORC_NT], feq[ORC_MAXQ];
    node_moments(&L, f, thermal, &rho, &u[0], &u[1], &theta);
    eq_coeffs(&L, rho, u[0], u[1], theta, a0);
    hermite_sum(&L, a0, L.n_eq, feq);
    noneq_coeffs(&L, &c, f, feq, rho, u, theta, a0, a1);
    return 0;
}

/* Recursion entry points on given inputs (for checking the algebra):
 * a1 holds a1^(2) (and a1^(3) for the thermal form) on entry; ranks 3..4
 * (isothermal) or rank 4 (thermal) are written. */
int orc_recursion(int thermal, double rho, double ux, double uy, double theta, double cs2,
                  const double* a0, double* a1)
{
    const double u[2] = { ux, uy };
    if (thermal)
        rr_thermal_high(u, rho, theta, cs2, a0, a1);
    else
        rr_isothermal(u, rho, a0, a1);
    return 0;
}

/* First-order part of the isothermal initial state (Sec. III.B:
 * f ~ f^(0) + f^(1), f^(1) from analytic velocity gradients, expanded over the
 * same Hermite terms as f^(0)).  grad[4][n] = (du_x/dx, du_x/dy, du_y/dx,
 * du_y/dy) per node in lattice units; tau is the discrete relaxation time.
 * a1^(2) = -tau [d_t a0^(2) + div a0^(3)] (Sec. II.E), which with the
 * isothermal equilibrium and the Euler equations is -rho c_s^2 tau S,
 * S = grad u + grad u^T (the traceless form of App. C is the thermal one;
 * both agree for a divergence-free field); a1^(3), a1^(4) follow the
 * isothermal recursion; f1[i*n + k] = w_i sum_{2 <= |k| <= order} ... */
int orc_noneq_init(int id, int order, int64_t n, const double* rho, const double* ux, const double* uy,
                   const double* grad, double tau, double* f1)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    if (order < 2 || order > L.n_eq) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double a0[ORC_NT], a1[ORC_NT], fl[ORC_MAXQ];
        const double u[2] = { ux[k], uy[k] };
        /* du[a][b] = d u_b / d x_a */
        const double du[2][2] = { { grad[0 * n + k], grad[2 * n + k] }, { grad[1 * n + k], grad[3 * n + k] } };
        eq_coeffs(&L, rho[k], u[0], u[1], 1.0, a0);
        for (int t = 0; t < ORC_NT; ++t) a1[t] = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                a1[toff(2, pair_bits(a, b))] = -rho[k] * L.cs2 * tau * (du[a][b] + du[b][a]);
        rr_isothermal(u, rho[k], a0, a1);
        for (int t = 0; t < ORC_NT; ++t)
            if (t >= toff(order + 1, 0)) a1[t] = 0.0;
        hermite_sum(&L, a1, order, fl);
        for (int i = 0; i < L.Q; ++i) f1[(int64_t)i * n + k] = fl[i];
    }
    return 0;
}

/* Equilibrium populations truncated at Hermite order `order` for n_nodes
 * nodes: feq[i*n + k].  theta may be NULL (isothermal). */
int orc_equilibrium(int id, int order, int64_t n, const double* rho, const double* ux,
                    const double* uy, const double* theta, double* feq)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    if (order < 0 || order > L.n_eq) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double a0[ORC_NT], fl[ORC_MAXQ];
        eq_coeffs(&L, rho[k], ux[k], uy[k], theta ? theta[k] : 1.0, a0);
        hermite_sum(&L, a0, order, fl);
        for (int i = 0; i < L.Q; ++i) feq[(int64_t)i * n + k] = fl[i];
    }
    return 0;
}

static int check_cfg(const orc_lattice_t* L, int coll, int order, double tau)
{
    if (coll < ORC_RR || coll > ORC_BGK) return -2;
    if (coll != ORC_BGK && (order < 2 || order > L->n_eq)) return -3;
    if (!(tau > 0.5) || !isfinite(tau)) return -4;
    return 0;
}

static void collide_all(const orc_lattice_t* L, const orc_cfg_t* c, int64_t n, const double* f, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[ORC_MAXQ], fo[ORC_MAXQ];
        for (int i = 0; i < L->Q; ++i) fl[i] = f[(int64_t)i * n + k];
        node_collide(L, c, fl, fo);
        for (int i = 0; i < L->Q; ++i) out[(int64_t)i * n + k] = fo[i];
    }
}

static void step_all(const orc_lattice_t* L, const orc_cfg_t* c, int nx, int ny, int nsteps, double* f,
                     double* tmp)
{
    const int64_t n = (int64_t)nx * ny;
    for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                double fl[ORC_MAXQ], fo[ORC_MAXQ];
                const int64_t k = (int64_t)y * nx + x;
                for (int i = 0; i < L->Q; ++i) fl[i] = f[(int64_t)i * n + k];
                node_collide(L, c, fl, fo);
                for (int i = 0; i < L->Q; ++i) {
                    int xd = ((x + L->cx[i]) % nx + nx) % nx;
                    int yd = ((y + L->cy[i]) % ny + ny) % ny;
                    tmp[(int64_t)i * n + (int64_t)yd * nx + xd] = fo[i];
                }
            }
        }
        memcpy(f, tmp, sizeof(double) * (size_t)(n * L->Q));
    }
}

/* Post-collision populations of every node (no streaming): out = C(f).
 * tau3, tau4: relaxation times of ranks 3 and 4 (pass tau for one time). */
int orc_collide_mrt(int id, int coll, int order, int thermal, int a13_raw, double tau, double tau3, double tau4,
                    int64_t n, const double* f, double* out)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    int e = check_cfg(&L, coll, order, tau);
    if (!e) e = check_cfg(&L, coll, order, tau3);
    if (!e) e = check_cfg(&L, coll, order, tau4);
    if (e) return e;
    orc_cfg_t c = { coll, order, thermal, a13_raw, tau, tau3, tau4 };
    collide_all(&L, &c, n, f, out);
    return 0;
}

int orc_collide(int id, int coll, int order, int thermal, int a13_raw, double tau, int64_t n,
                const double* f, double* out)
{
    return orc_collide_mrt(id, coll, order, thermal, a13_raw, tau, tau, tau, n, f, out);
}

/* nsteps of collide-then-stream on a periodic nx x ny grid (Sec. III.A):
 * f_i(x + c_i, t + 1) = f_i^coll(x, t).  f holds the pre-collision state and
 * is updated in place; tmp is scratch of the same size. */
int orc_step_mrt(int id, int coll, int order, int thermal, int a13_raw, double tau, double tau3, double tau4,
                 int nx, int ny, int nsteps, double* f, double* tmp)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    int e = check_cfg(&L, coll, order, tau);
    if (!e) e = check_cfg(&L, coll, order, tau3);
    if (!e) e = check_cfg(&L, coll, order, tau4);
    if (e) return e;
    if (nx < 1 || ny < 1) return -5;
    orc_cfg_t c = { coll, order, thermal, a13_raw, tau, tau3, tau4 };
    step_all(&L, &c, nx, ny, nsteps, f, tmp);
    return 0;
}

int orc_step(int id, int coll, int order, int thermal, int a13_raw, double tau, int nx, int ny,
             int nsteps, double* f, double* tmp)
{
    return orc_step_mrt(id, coll, order, thermal, a13_raw, tau, tau, tau, nx, ny, nsteps, f, tmp);
}

/* ---- Learned-closure support (not part of the paper's method) ----------
 * The closure replaces nothing of the step above: it adds a learned residual
 * to the isothermal recursive a1^(3), a1^(4).  Coefficients are exchanged in
 * the tau-independent scaling a_hat = (1 - 1/(2 tau)) a1 (the viscous stress
 * is -a_hat^(2)), in the component order 30, 21, 12, 03, 40, 31, 22, 13, 04
 * (n_x, n_y). */

static const int orc_hi_nx[9] = { 3, 2, 1, 0, 4, 3, 2, 1, 0 };

static int pattern_of(int nx, int ny) { return ((1 << ny) - 1) << nx; }

/* Per node of pre-collision f[Q][n] (isothermal): feat[7][n] =
 * (rho - 1, ux, uy, |u|^2 / c_s^2, ahat_xx, ahat_xy, ahat_yy), and
 * rr[9][n] = a_hat of the plain recursive a1^(3..4). */
int orc_closure_inputs(int id, double tau, int64_t n, const double* f, double* feat, double* rr)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    const double s = 1.0 - 0.5 / tau;
    orc_cfg_t c = { ORC_RR, L.n_eq, 0, 0, tau, tau, tau };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[ORC_MAXQ], a0[ORC_NT], feq[ORC_MAXQ], a1[ORC_NT], rho, u[2], th;
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        node_moments(&L, fl, 1, &rho, &u[0], &u[1], &th);
        eq_coeffs(&L, rho, u[0], u[1], 1.0, a0);
        hermite_sum(&L, a0, L.n_eq, feq);
        noneq_coeffs(&L, &c, fl, feq, rho, u, 1.0, a0, a1);
        feat[0 * n + k] = rho - 1.0;
        feat[1 * n + k] = u[0];
        feat[2 * n + k] = u[1];
        feat[3 * n + k] = (u[0] * u[0] + u[1] * u[1]) / L.cs2;
        feat[4 * n + k] = s * a1[toff(2, pattern_of(2, 0))];
        feat[5 * n + k] = s * a1[toff(2, pattern_of(1, 1))];
        feat[6 * n + k] = s * a1[toff(2, pattern_of(0, 2))];
        for (int j = 0; j < 9; ++j) {
            const int nx = orc_hi_nx[j], ny = (j < 4 ? 3 : 4) - nx;
            rr[(int64_t)j * n + k] = s * a1[toff(nx + ny, pattern_of(nx, ny))];
        }
    }
    return 0;
}

/* Projected non-equilibrium coefficients of every node (isothermal
 * equilibrium at the lattice's full order): out[12][n] = a1 for
 * xx, xy, yy, 30, 21, 12, 03, 40, 31, 22, 13, 04, each sum_i H^k_i (f_i - f^(0)_i). */
int orc_noneq_projected(int id, int64_t n, const double* f, double* out)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    static const int nxs[12] = { 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0 };
    static const int nys[12] = { 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4 };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[ORC_MAXQ], a0[ORC_NT], feq[ORC_MAXQ], g[ORC_MAXQ], rho, ux, uy, th;
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        node_moments(&L, fl, 0, &rho, &ux, &uy, &th);
        eq_coeffs(&L, rho, ux, uy, 1.0, a0);
        hermite_sum(&L, a0, L.n_eq, feq);
        for (int i = 0; i < L.Q; ++i) g[i] = fl[i] - feq[i];
        for (int j = 0; j < 12; ++j) {
            const int m = nxs[j] + nys[j];
            const int b = pattern_of(nxs[j], nys[j]);
            double s = 0;
            for (int i = 0; i < L.Q; ++i) s += L.H[i][toff(m, b)] * g[i];
            out[(int64_t)j * n + k] = s;
        }
    }
    return 0;
}

/* Isothermal RR collision of every node with a1^(3..4) += resid / (1 - 1/(2 tau))
 * (resid[9][n] in the a_hat scaling; ranks beyond the order are dropped as
 * in the plain collision).  resid = 0 reproduces orc_collide. */
int orc_collide_closure(int id, int order, double tau, int64_t n, const double* f, const double* resid,
                        double* out)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
    int e = check_cfg(&L, ORC_RR, order, tau);
    if (e) return e;
    orc_cfg_t c = { ORC_RR, order, 0, 0, tau, tau, tau };
    const double inv_s = 1.0 / (1.0 - 0.5 / tau);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[ORC_MAXQ], a0[ORC_NT], feq[ORC_MAXQ], a1[ORC_NT], rho, u[2], th, a[ORC_NT];
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        node_moments(&L, fl, 0, &rho, &u[0], &u[1], &th);
        eq_coeffs(&L, rho, u[0], u[1], 1.0, a0);
        hermite_sum(&L, a0, L.n_eq, feq);
        noneq_coeffs(&L, &c, fl, feq, rho, u, 1.0, a0, a1);
        for (int j = 0; j < 9; ++j) {
            const int nx = orc_hi_nx[j], ny = (j < 4 ? 3 : 4) - nx;
            const double add = resid[(int64_t)j * n + k] * inv_s;
            /* every index order of the (nx, ny) component */
            for (int b = 0; b < (1 << (nx + ny)); ++b)
                if (popcount5(b) == ny) a1[toff(nx + ny, b)] += add;
        }
        const double kk = 1.0 - 1.0 / tau;
        for (int m = 0; m <= 4; ++m)
            for (int b = 0; b < (1 << m); ++b) {
                double v = a0[toff(m, b)];
                if (m >= 2 && m <= order) v += kk * a1[toff(m, b)];
                a[toff(m, b)] = v;
            }
        double fo[ORC_MAXQ];
        hermite_sum(&L, a, L.n_eq, fo);
        for (int i = 0; i < L.Q; ++i) out[(int64_t)i * n + k] = fo[i];
    }
    return 0;
}

/* rho, u (and theta if thermal) of every node of f[Q][n]. */
int orc_moments(int id, int thermal, int64_t n, const double* f, double* rho, double* ux,
                double* uy, double* theta)
{
    orc_lattice_t L;
    if (build_lattice(id, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double fl[ORC_MAXQ], r, vx, vy, th;
        for (int i = 0; i < L.Q; ++i) fl[i] = f[(int64_t)i * n + k];
        node_moments(&L, fl, thermal, &r, &vx, &vy, &th);
        rho[k] = r;
        ux[k] = vx;
        uy[k] = vy;
        if (theta) theta[k] = th;
    }
    return 0;
}
