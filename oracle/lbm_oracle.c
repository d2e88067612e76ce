/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the D3Q27 lattice Boltzmann
 * scheme with a central-Hermite-moment multiple-relaxation-time (CHM-MRT)
 * collision, as described in "Simulation of the FDA Nozzle Benchmark: A
 * Lattice Boltzmann Study" (Huang, Noel, Berg, Hosseini), Sec. 2.1 and
 * Appendix A, together with the boundary treatment of Sec. 2.2
 * ("Simulation details").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker of the GPU library,
 * not part of it.  It is slow on purpose: it evaluates the equilibrium as
 * the Hermite sum of Eq. (4), builds the 27x27 central-moment transform T
 * of Eqs. (7)-(8) entry by entry from the Hermite polynomials of Eq. (A.3),
 * and applies T^-1 S T of Eq. (6) with a Gaussian-elimination solve, in
 * separate streaming and collision passes.  It shares no code, header,
 * table or constant with the GPU path; the few conventions both sides must
 * agree on (population order, flag values, field layout) are re-typed here.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * Conventions (the interface both sides must agree on):
 *   population i <-> velocity c_i = (i%3 - 1, (i/3)%3 - 1, i/9 - 1),
 *                   so the opposite direction of i is 26 - i;
 *   fields are structure-of-arrays, f[i*ncells + cell],
 *   cell = (z*ny + y)*nx + x, x fastest;
 *   flags: 0 fluid, 1 solid, 2 inlet, 3 outlet;
 *   rates[6] = { omega (shear), omega_bulk, omega_3, omega_4, omega_5,
 *                omega_6 } where omega_n relaxes every central moment of
 *                total order n >= 3.
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *   - Eq. (4) prints the prefactor as w_i/(i! theta0^i); the index is the
 *     expansion order n, i.e. w_i/(n! theta0^n).
 *   - Eq. (A.3) prints the Hermite polynomials without theta0; they are
 *     used in the dimensional form H_ab = c_a c_b - theta0 delta_ab etc.
 *   - The expansion to the full order the stencil supports (after
 *     Eq. (A.6)): the sum
 *     of Eq. (4) runs over every tensor component of order n <= 6 in which
 *     no axis appears more than twice; the central moments of Eq. (8) are
 *     the 27 components with each axis appearing at most twice.
 *   - The conserved moments (orders 0 and 1) have T(f^eq - f) = 0, so
 *     their rate is immaterial; zero is used.
 *   - Bulk and shear split of the second-order rates: the trace of the
 *     diagonal second-order central moments relaxes with omega_bulk, the
 *     deviator and the off-diagonal ones with omega.  omega_bulk = omega
 *     is the paper's setting.
 *   - Walls: halfway bounce-back by default (the curved treatment of
 *     Sec. 2.2 at wall distance one half); the linear interpolated rule
 *     with per-link fractions after oracle_set_wall_distances (see there).
 *     Inlet: bounce-back from a wall moving with the prescribed inlet
 *     velocity of Eq. (12) at the inlet cell, wall density 1.  Outlet:
 *     zero gradient by default, sources beyond the last x plane are taken
 *     from the last x plane; constant pressure by non-equilibrium
 *     extrapolation after oracle_set_outlet (see there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 27
#define THETA0 (1.0 / 3.0) /* stencil reference temperature, App. A */

enum { F_FLUID = 0, F_SOLID = 1, F_INLET = 2, F_OUTLET = 3 };
enum { O_OK = 0, O_ERR_ARG = -1, O_ERR_OOM = -2, O_ERR_UNSTABLE = -4 };

/* ------------------------------------------------------------------ */
/* Velocity set: third-order Gauss-Hermite quadrature, App. A,        */
/* Eqs. (A.1)-(A.2): 1-D weights 2/3 (c = 0) and 1/6 (c = +-1), the   */
/* 3-D weight is the product over the three axes.                     */
/* ------------------------------------------------------------------ */
static int g_c[NQ][3];
static double g_w[NQ];

/* Hermite tensor components used by Eq. (4): every index tuple of
 * length n <= 6 over {x,y,z} with no axis appearing more than twice. */
#define MAX_TUPLES 512
static int g_ntuples;
static int g_tuple_n[MAX_TUPLES];
static int g_tuple_idx[MAX_TUPLES][6];
static double g_Hc[NQ][MAX_TUPLES]; /* H_tuple(c_i), tabulated once */

/* central moments (Eq. (8)): index k = p + 3 q + 9 r <-> x^p y^q z^r */
static int g_mom_n[NQ];
static int g_mom_idx[NQ][6];

static int g_ready = 0;

static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

/* App. A, Eq. (A.3): the multivariate Hermite polynomial for the index
 * tuple idx[0..n-1], evaluated at xi.  The cyclic sums of Eq. (A.3) are
 * the sums over every way of pairing some of the indices: each pair
 * contributes -theta0 * delta, each unpaired index contributes xi.  The
 * recursion takes the first index either unpaired or paired with a
 * later index. */
double oracle_hermite(int n, const int *idx, const double *xi)
{
    if (n == 0)
        return 1.0;
    int rest[6];
    for (int k = 1; k < n; ++k)
        rest[k - 1] = idx[k];
    double h = xi[idx[0]] * oracle_hermite(n - 1, rest, xi);
    for (int j = 1; j < n; ++j) {
        if (idx[j] != idx[0])
            continue;
        int rest2[6], m = 0;
        for (int k = 1; k < n; ++k)
            if (k != j)
                rest2[m++] = idx[k];
        h -= THETA0 * oracle_hermite(n - 2, rest2, xi);
    }
    return h;
}

static void enumerate_tuples(int n, int pos, int *cur, int *count)
{
    if (pos == n) {
        int cnt[3] = {0, 0, 0};
        for (int k = 0; k < n; ++k)
            cnt[cur[k]]++;
        if (cnt[0] > 2 || cnt[1] > 2 || cnt[2] > 2)
            return;
        g_tuple_n[g_ntuples] = n;
        for (int k = 0; k < n; ++k)
            g_tuple_idx[g_ntuples][k] = cur[k];
        g_ntuples++;
        return;
    }
    for (int a = 0; a < 3; ++a) {
        cur[pos] = a;
        enumerate_tuples(n, pos + 1, cur, count);
    }
}

static void oracle_init_tables(void)
{
    if (g_ready)
        return;
    for (int i = 0; i < NQ; ++i) {
        g_c[i][0] = i % 3 - 1;
        g_c[i][1] = (i / 3) % 3 - 1;
        g_c[i][2] = i / 9 - 1;
        g_w[i] = w1(g_c[i][0]) * w1(g_c[i][1]) * w1(g_c[i][2]);
    }
    g_ntuples = 0;
    int cur[6];
    for (int n = 0; n <= 6; ++n)
        enumerate_tuples(n, 0, cur, NULL);
    for (int i = 0; i < NQ; ++i) {
        double ci[3] = {g_c[i][0], g_c[i][1], g_c[i][2]};
        for (int t = 0; t < g_ntuples; ++t)
            g_Hc[i][t] = oracle_hermite(g_tuple_n[t], g_tuple_idx[t], ci);
    }
    for (int k = 0; k < NQ; ++k) {
        int p = k % 3, q = (k / 3) % 3, r = k / 9, m = 0;
        for (int a = 0; a < p; ++a)
            g_mom_idx[k][m++] = 0;
        for (int a = 0; a < q; ++a)
            g_mom_idx[k][m++] = 1;
        for (int a = 0; a < r; ++a)
            g_mom_idx[k][m++] = 2;
        g_mom_n[k] = m;
    }
    g_ready = 1;
}

void oracle_velocity_set(int *c, double *w)
{
    oracle_init_tables();
    for (int i = 0; i < NQ; ++i) {
        c[3 * i + 0] = g_c[i][0];
        c[3 * i + 1] = g_c[i][1];
        c[3 * i + 2] = g_c[i][2];
        w[i] = g_w[i];
    }
}

int oracle_num_tuples(void)
{
    oracle_init_tables();
    return g_ntuples;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k)
        f *= k;
    return f;
}

/* Sec. 2.1, Eq. (4) with the coefficients of App. A, Eq. (A.4):
 * f_i^eq = w_i sum_{n<=order} a_n^eq : H_n(c_i) / (n! theta0^n),
 * a_n^eq = rho u^{(x)n}.  order = 6 is the paper's full expansion. */
void oracle_feq(double rho, const double *u, int order, double *feq)
{
    oracle_init_tables();
    double a[MAX_TUPLES], scale[7];
    for (int n = 0; n <= 6; ++n)
        scale[n] = 1.0 / (factorial(n) * pow(THETA0, n));
    for (int t = 0; t < g_ntuples; ++t) {
        double v = rho;
        for (int k = 0; k < g_tuple_n[t]; ++k)
            v *= u[g_tuple_idx[t][k]];
        a[t] = v;
    }
    for (int i = 0; i < NQ; ++i) {
        double s = 0.0;
        for (int t = 0; t < g_ntuples; ++t)
            if (g_tuple_n[t] <= order)
                s += a[t] * g_Hc[i][t] * scale[g_tuple_n[t]];
        feq[i] = g_w[i] * s;
    }
}

/* Sec. 2.1, Eqs. (7)-(8): the central-Hermite-moment transform,
 * T[k][i] = H_k(c_i - u) for the 27 moments k = x^p y^q z^r. */
void oracle_transform(const double *u, double *T)
{
    oracle_init_tables();
    for (int k = 0; k < NQ; ++k)
        for (int i = 0; i < NQ; ++i) {
            double xi[3] = {g_c[i][0] - u[0], g_c[i][1] - u[1], g_c[i][2] - u[2]};
            T[k * NQ + i] = oracle_hermite(g_mom_n[k], g_mom_idx[k], xi);
        }
}

/* Sec. 2.1 (text after Eq. (8)) and App. A: the relaxation matrix S.
 * Diagonal except for the bulk/shear split of the three diagonal
 * second-order moments: S v = omega (v - tr v/3) + omega_bulk tr v/3. */
void oracle_relaxation(const double *rates, double *S)
{
    oracle_init_tables();
    memset(S, 0, sizeof(double) * NQ * NQ);
    for (int k = 0; k < NQ; ++k) {
        int p = k % 3, q = (k / 3) % 3, r = k / 9, n = p + q + r;
        if (n <= 1)
            continue;
        if (n >= 3) {
            S[k * NQ + k] = rates[n - 1]; /* rates[2..5] = omega_3..omega_6 */
            continue;
        }
        int diag = (p == 2 || q == 2 || r == 2);
        if (!diag) {
            S[k * NQ + k] = rates[0];
            continue;
        }
        for (int l = 0; l < NQ; ++l) {
            int pl = l % 3, ql = (l / 3) % 3, rl = l / 9;
            if (pl + ql + rl == 2 && (pl == 2 || ql == 2 || rl == 2))
                S[k * NQ + l] = (k == l ? rates[0] : 0.0) + (rates[1] - rates[0]) / 3.0;
        }
    }
}

/* Gaussian elimination with partial pivoting: solves A x = b, A is n x n
 * row-major and is overwritten.  Returns 0, or -1 for a singular A. */
static int solve_dense(int n, double *A, double *b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col]))
                piv = r;
        if (A[piv * n + col] == 0.0)
            return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                double t = A[col * n + c];
                A[col * n + c] = A[piv * n + c];
                A[piv * n + c] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double m = A[r * n + col] / A[col * n + col];
            if (m == 0.0)
                continue;
            for (int c = col; c < n; ++c)
                A[r * n + c] -= m * A[col * n + c];
            b[r] -= m * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c)
            s -= A[r * n + c] * b[c];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* Sec. 2.1, Eqs. (3), (8): density and velocity of a population set. */
void oracle_cell_moments(const double *f, double *rho, double *u)
{
    oracle_init_tables();
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < NQ; ++i) {
        r += f[i];
        for (int a = 0; a < 3; ++a)
            j[a] += g_c[i][a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a)
        u[a] = j[a] / r;
}

/* Order N of the equilibrium the collision relaxes to (Sec. 2.1,
 * Eq. (4): the Hermite expansion truncated at N).  6, the full expansion
 * the stencil supports, is the paper's choice (App. A after Eq. (A.6));
 * with N < 6 the central moments of f^eq are no longer (rho, 0, ..., 0),
 * and the collision relaxes every moment towards those of the truncated
 * f^eq (N = 2: the classical second-order equilibrium; N = 3 adds the
 * third-order terms the paper mentions for Galilean invariance of the
 * shear stress).  The initial state and the pressure outlet's ghost value
 * keep the full expansion. */
static int g_feq_order = 6;

int oracle_set_equilibrium_order(int order)
{
    if (order < 2 || order > 6)
        return O_ERR_ARG;
    g_feq_order = order;
    return O_OK;
}

/* Sec. 2.1, Eq. (6): the post-collision populations of one cell,
 * f* = f + T^-1 S T (f^eq - f), with f^eq the expansion of order
 * g_feq_order (the full sixth-order one by default) and T evaluated at
 * the cell's own velocity.  Returns 0, or O_ERR_UNSTABLE when rho <= 0 or
 * a value is not finite. */
int oracle_collide(const double *f, const double *rates, double *fout)
{
    oracle_init_tables();
    double rho, u[3], feq[NQ], T[NQ * NQ], S[NQ * NQ], d[NQ], m[NQ], y[NQ];
    oracle_cell_moments(f, &rho, u);
    if (!(rho > 0.0) || !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2])) {
        for (int i = 0; i < NQ; ++i)
            fout[i] = f[i];
        return O_ERR_UNSTABLE;
    }
    oracle_feq(rho, u, g_feq_order, feq);
    oracle_transform(u, T);
    oracle_relaxation(rates, S);
    for (int i = 0; i < NQ; ++i)
        d[i] = feq[i] - f[i];
    for (int k = 0; k < NQ; ++k) {
        double s = 0.0;
        for (int i = 0; i < NQ; ++i)
            s += T[k * NQ + i] * d[i];
        m[k] = s;
    }
    for (int k = 0; k < NQ; ++k) {
        double s = 0.0;
        for (int l = 0; l < NQ; ++l)
            s += S[k * NQ + l] * m[l];
        y[k] = s;
    }
    if (solve_dense(NQ, T, y) != 0)
        return O_ERR_ARG;
    for (int i = 0; i < NQ; ++i)
        fout[i] = f[i] + y[i];
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Streaming (pull form of the left-hand side of Eqs. (3)/(6)) with    */
/* the boundary treatment of Sec. 2.2.                                */
/* ------------------------------------------------------------------ */
typedef struct {
    const uint8_t *flags;
    int nx, ny, nz;
    unsigned periodic; /* bit0 x, bit1 y, bit2 z */
    const double *uin; /* 3*ncells ([c][cell]) or NULL */
    long ncells;
} odom;

static int updatable(uint8_t fl) { return fl == F_FLUID || fl == F_OUTLET; }

/* Outlet condition: 0 zero gradient, 1 constant pressure by
 * non-equilibrium extrapolation (Sec. 2.2, "Simulation details").
 * Reading for the constant-pressure outlet: the ghost cell beyond the last
 * x plane has the velocity and the non-equilibrium part of the last-plane
 * cell it faces and the outlet density rho_out, so a population pulled
 * from it is f*_i(s) - f^eq_i(rho_s, u_s) + f^eq_i(rho_out, u_s) with s the
 * clamped last-plane source and rho_s, u_s its moments. */
static int g_outlet_kind = 0;
static double g_rho_out = 1.0;

void oracle_set_outlet(int kind, double rho_out)
{
    g_outlet_kind = kind;
    g_rho_out = rho_out;
}

static int wrap(int s, int n) { return ((s % n) + n) % n; }

/* Resolve the source of population i at cell (x,y,z).  Returns the kind
 * of link: 0 plain pull from *src, 1 wall (halfway bounce-back), 2 inlet
 * (moving-wall bounce-back; *src is the inlet cell). */
static int resolve(const odom *d, int x, int y, int z, int i, long *src, int *clamped)
{
    *clamped = 0;
    int sx = x - g_c[i][0], sy = y - g_c[i][1], sz = z - g_c[i][2];
    if (d->periodic & 1u)
        sx = wrap(sx, d->nx);
    if (d->periodic & 2u)
        sy = wrap(sy, d->ny);
    if (d->periodic & 4u)
        sz = wrap(sz, d->nz);
    long self = ((long)z * d->ny + y) * d->nx + x;
    /* zero-gradient outlet: sources past the last x plane come from it */
    if (sx >= d->nx && !(d->periodic & 1u) && d->flags[self] == F_OUTLET) {
        sx = d->nx - 1;
        *clamped = 1;
    }
    if (sx < 0 || sx >= d->nx || sy < 0 || sy >= d->ny || sz < 0 || sz >= d->nz)
        return 1;
    long s = ((long)sz * d->ny + sy) * d->nx + sx;
    *src = s;
    if (d->flags[s] == F_SOLID)
        return 1;
    if (d->flags[s] == F_INLET)
        return 2;
    return 0;
}

/* Curved walls (Sec. 2.2, interpolated bounce-back after Bouzidi et al.):
 * q[i*ncells + cell] is the fraction of the link from cell x towards
 * x - c_i at which the wall lies, read for wall links only; NULL keeps the
 * halfway rule (q = 1/2 everywhere).  With f* the post-collision field of
 * the previous step the linear interpolation gives
 *   q <  1/2: f_i(x) = 2q f*_ibar(x) + (1 - 2q) f*_ibar(x + c_i),
 *   q >= 1/2: f_i(x) = f*_ibar(x) / (2q) + (1 - 1/(2q)) f*_i(x),
 * ibar the opposite direction.  f*_ibar(x + c_i) is the value x pulls for
 * direction ibar.  Reading for a cell whose opposite link ibar is not a
 * plain link (a gap one cell wide, or an inlet behind it): with q < 1/2
 * the halfway rule is kept. */
static const double *g_q = NULL;

void oracle_set_wall_distances(const double *q) { g_q = q; }

/* Post-collision population i of cell `cell` of the previous step. */
typedef double (*pop_fn)(const void *ctx, long cell, int i);

/* Pre-collision populations g of one updatable cell. */
static void pull_cell(const odom *d, long cell, pop_fn pop, const void *ctx, double *g)
{
    int x = (int)(cell % d->nx), y = (int)((cell / d->nx) % d->ny), z = (int)(cell / ((long)d->nx * d->ny));
    int kind[NQ];
    long src[NQ];
    /* plain links first: the curved-wall rule reads them */
    for (int i = 0; i < NQ; ++i) {
        int clamped = 0;
        src[i] = cell;
        kind[i] = resolve(d, x, y, z, i, &src[i], &clamped);
        if (kind[i] != 0)
            continue;
        g[i] = pop(ctx, src[i], i);
        if (clamped && g_outlet_kind == 1) {
            double fs[NQ], rs = 0.0, us[3] = {0.0, 0.0, 0.0}, fe[NQ];
            for (int k = 0; k < NQ; ++k)
                fs[k] = pop(ctx, src[i], k);
            oracle_cell_moments(fs, &rs, us);
            oracle_feq(1.0, us, 6, fe); /* f^eq is linear in rho */
            g[i] += (g_rho_out - rs) * fe[i];
        }
    }
    for (int i = 0; i < NQ; ++i) {
        if (kind[i] == 0)
            continue;
        double v = pop(ctx, cell, NQ - 1 - i);
        if (kind[i] == 2) {
            double cu = 0.0;
            if (d->uin)
                for (int a = 0; a < 3; ++a)
                    cu += g_c[i][a] * d->uin[(long)a * d->ncells + src[i]];
            /* wall density 1: + 2 w_i (c_i . u_w) / theta0 */
            v += 2.0 * g_w[i] * cu / THETA0;
        } else if (g_q) {
            double q = g_q[(long)i * d->ncells + cell];
            if (q < 0.5) {
                if (kind[NQ - 1 - i] == 0)
                    v = 2.0 * q * v + (1.0 - 2.0 * q) * g[NQ - 1 - i];
            } else {
                v = v / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * pop(ctx, cell, i);
            }
        }
        g[i] = v;
    }
}

typedef struct {
    const double *f;
    long ncells;
} field_ctx;

static double field_pop(const void *ctx, long cell, int i)
{
    const field_ctx *c = (const field_ctx *)ctx;
    return c->f[(long)i * c->ncells + cell];
}

/* Pre-collision populations g of one updatable cell from the
 * post-collision field f of the previous step. */
static void gather_cell(const odom *d, const double *f, long cell, double *g)
{
    field_ctx c = {f, d->ncells};
    pull_cell(d, cell, field_pop, &c, g);
}

/* Pull streaming pass over the whole field: g = stream(f).  Cells that
 * are not updated (solid, inlet) keep their values. */
void oracle_stream(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, const double *uin,
                   const double *f, double *g)
{
    oracle_init_tables();
    odom d = {flags, nx, ny, nz, periodic, uin, (long)nx * ny * nz};
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < d.ncells; ++cell) {
        double gc[NQ];
        if (updatable(flags[cell])) {
            gather_cell(&d, f, cell, gc);
        } else {
            for (int i = 0; i < NQ; ++i)
                gc[i] = f[(long)i * d.ncells + cell];
        }
        for (int i = 0; i < NQ; ++i)
            g[(long)i * d.ncells + cell] = gc[i];
    }
}

/* Collision pass over the whole field, in place. */
int oracle_collide_field(const uint8_t *flags, long ncells, const double *rates, double *f)
{
    oracle_init_tables();
    int status = O_OK;
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncells; ++cell) {
        if (!updatable(flags[cell]))
            continue;
        double a[NQ], b[NQ];
        for (int i = 0; i < NQ; ++i)
            a[i] = f[(long)i * ncells + cell];
        int st = oracle_collide(a, rates, b);
        if (st != O_OK) {
#pragma omp critical
            status = st;
        }
        for (int i = 0; i < NQ; ++i)
            f[(long)i * ncells + cell] = b[i];
    }
    return status;
}

/* Initial state: f = f^eq(rho, u) at every updatable cell (Eq. (4));
 * other cells are set to zero.  rho == NULL means 1, u == NULL means 0. */
void oracle_init_fields(const uint8_t *flags, long ncells, const double *rho, const double *u, double *f)
{
    oracle_init_tables();
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncells; ++cell) {
        double feq[NQ];
        if (updatable(flags[cell])) {
            double r = rho ? rho[cell] : 1.0;
            double uu[3] = {0.0, 0.0, 0.0};
            if (u)
                for (int a = 0; a < 3; ++a)
                    uu[a] = u[(long)a * ncells + cell];
            oracle_feq(r, uu, 6, feq);
        } else {
            for (int i = 0; i < NQ; ++i)
                feq[i] = 0.0;
        }
        for (int i = 0; i < NQ; ++i)
            f[(long)i * ncells + cell] = feq[i];
    }
}

/* n time steps, each a streaming pass followed by a collision pass.
 * f holds the post-collision state and is updated in place; work is a
 * caller-provided buffer of the same size.  Returns O_ERR_UNSTABLE as soon
 * as a step produced rho <= 0 or a non-finite velocity. */
int oracle_step(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, const double *uin,
                const double *rates, int nsteps, double *f, double *work)
{
    oracle_init_tables();
    long ncells = (long)nx * ny * nz;
    for (int s = 0; s < nsteps; ++s) {
        oracle_stream(flags, nx, ny, nz, periodic, uin, f, work);
        int st = oracle_collide_field(flags, ncells, rates, work);
        memcpy(f, work, sizeof(double) * NQ * ncells);
        if (st != O_OK)
            return st;
    }
    return O_OK;
}

/* Density and velocity of every cell; zero at cells that are not
 * updated. */
void oracle_moments(const uint8_t *flags, long ncells, const double *f, double *rho, double *u)
{
    oracle_init_tables();
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncells; ++cell) {
        double fc[NQ], r = 0.0, uu[3] = {0.0, 0.0, 0.0};
        if (updatable(flags[cell])) {
            for (int i = 0; i < NQ; ++i)
                fc[i] = f[(long)i * ncells + cell];
            oracle_cell_moments(fc, &r, uu);
        }
        rho[cell] = r;
        for (int a = 0; a < 3; ++a)
            u[(long)a * ncells + cell] = uu[a];
    }
}

/* Viscous stress of a pre-collision state (Sec. 2.2, Eq. (19), with the
 * strain rate from the second-order Hermite coefficients, App. A,
 * Eqs. (A.7)-(A.8)).  Reading of the garbled sign and factor: the
 * non-equilibrium second-order central Hermite moment
 *     M_ab = sum_i f_i [(c_ia - u_a)(c_ib - u_b) - theta0 delta_ab]
 * (f^eq contributes nothing to it) equals -2 rho theta0 tau S_ab to
 * leading order, so sigma_ab = 2 rho nu S_ab = -(1 - omega/2) M_ab with
 * nu = theta0 (tau - 1/2), omega = 1/tau.  Out: sigma[6][ncells] in the
 * order xx, yy, zz, xy, xz, yz; zero at cells that are not updated. */
void oracle_stress(const uint8_t *flags, long ncells, const double *f, double omega, double *sigma)
{
    static const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    oracle_init_tables();
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < ncells; ++cell) {
        double out[6] = {0, 0, 0, 0, 0, 0};
        if (updatable(flags[cell])) {
            double fc[NQ], r = 0.0, u[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < NQ; ++i)
                fc[i] = f[(long)i * ncells + cell];
            oracle_cell_moments(fc, &r, u);
            for (int k = 0; k < 6; ++k) {
                const int a = pa[k], b = pb[k];
                double m = 0.0;
                for (int i = 0; i < NQ; ++i) {
                    const double xa = g_c[i][a] - u[a], xb = g_c[i][b] - u[b];
                    m += fc[i] * (xa * xb - (a == b ? THETA0 : 0.0));
                }
                out[k] = -(1.0 - 0.5 * omega) * m;
            }
        }
        for (int k = 0; k < 6; ++k)
            sigma[(long)k * ncells + cell] = out[k];
    }
}

/* ------------------------------------------------------------------ */
/* Sampled run: the post-collision populations after nsteps at a few  */
/* listed cells of a large domain, starting from f^eq(rho0, u0).  Only */
/* the cells inside the dependency cone of the listed cells are       */
/* computed; the arithmetic per cell is the same as oracle_step.      */
/* ------------------------------------------------------------------ */
static int cmp_long(const void *a, const void *b)
{
    long x = *(const long *)a, y = *(const long *)b;
    return (x > y) - (x < y);
}

static long find_slot(const long *sorted, long n, long key)
{
    long lo = 0, hi = n - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        if (sorted[mid] == key)
            return mid;
        if (sorted[mid] < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

static long unique_sorted(long *a, long n)
{
    if (n == 0)
        return 0;
    qsort(a, (size_t)n, sizeof(long), cmp_long);
    long m = 1;
    for (long k = 1; k < n; ++k)
        if (a[k] != a[m - 1])
            a[m++] = a[k];
    return m;
}

/* States of the previous step of the listed cells (sorted), 27 each. */
typedef struct {
    const double *state;
    const long *cells;
    long n;
} cone_ctx;

static double cone_pop(const void *ctx, long cell, int i)
{
    const cone_ctx *c = (const cone_ctx *)ctx;
    return c->state[(long)NQ * find_slot(c->cells, c->n, cell) + i];
}

int oracle_run_cells(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, const double *uin,
                     const double *rho0, const double *u0, const double *rates, int nsteps, long nlist,
                     const long *list, double *out /* 27*nlist, [i][k] */)
{
    oracle_init_tables();
    odom d = {flags, nx, ny, nz, periodic, uin, (long)nx * ny * nz};
    if (nsteps < 0 || nlist <= 0)
        return O_ERR_ARG;
    for (long k = 0; k < nlist; ++k)
        if (list[k] < 0 || list[k] >= d.ncells || !updatable(flags[list[k]]))
            return O_ERR_ARG;
    /* need[t]: sorted cells whose state after step t is required */
    int status = O_OK;
    double *state = NULL;
    long **need = calloc((size_t)nsteps + 1, sizeof(long *));
    long *nneed = calloc((size_t)nsteps + 1, sizeof(long));
    if (!need || !nneed) {
        status = O_ERR_OOM;
        goto done;
    }
    need[nsteps] = malloc(sizeof(long) * (size_t)nlist);
    if (!need[nsteps]) {
        status = O_ERR_OOM;
        goto done;
    }
    memcpy(need[nsteps], list, sizeof(long) * (size_t)nlist);
    nneed[nsteps] = unique_sorted(need[nsteps], nlist);
    for (int t = nsteps; t > 0; --t) {
        long cap = nneed[t] * NQ;
        long *prev = malloc(sizeof(long) * (size_t)cap);
        if (!prev) {
            status = O_ERR_OOM;
            goto done;
        }
        long m = 0;
        for (long k = 0; k < nneed[t]; ++k) {
            long cell = need[t][k];
            int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((long)nx * ny));
            for (int i = 0; i < NQ; ++i) {
                long src = cell;
                int clamped = 0;
                int kind = resolve(&d, x, y, z, i, &src, &clamped);
                prev[m++] = kind == 0 ? src : cell;
            }
        }
        nneed[t - 1] = unique_sorted(prev, m);
        need[t - 1] = prev;
    }
    /* state after step 0: the equilibrium of the initial fields */
    state = malloc(sizeof(double) * NQ * (size_t)nneed[0]);
    if (!state) {
        status = O_ERR_OOM;
        goto done;
    }
    for (long k = 0; k < nneed[0]; ++k) {
        long cell = need[0][k];
        double uu[3] = {0.0, 0.0, 0.0};
        if (u0)
            for (int a = 0; a < 3; ++a)
                uu[a] = u0[(long)a * d.ncells + cell];
        oracle_feq(rho0 ? rho0[cell] : 1.0, uu, 6, state + (long)NQ * k);
    }
    for (int t = 1; t <= nsteps; ++t) {
        double *next = malloc(sizeof(double) * NQ * (size_t)nneed[t]);
        if (!next) {
            status = O_ERR_OOM;
            goto done;
        }
        const long *pc = need[t - 1];
        long npc = nneed[t - 1];
#pragma omp parallel for schedule(dynamic, 64)
        for (long k = 0; k < nneed[t]; ++k) {
            long cell = need[t][k];
            double g[NQ];
            cone_ctx c = {state, pc, npc};
            pull_cell(&d, cell, cone_pop, &c, g);
            int st = oracle_collide(g, rates, next + (long)NQ * k);
            if (st != O_OK) {
#pragma omp critical
                status = st;
            }
        }
        free(state);
        state = next;
    }
    for (long k = 0; k < nlist; ++k) {
        long slot = find_slot(need[nsteps], nneed[nsteps], list[k]);
        for (int i = 0; i < NQ; ++i)
            out[(long)i * nlist + k] = state[(long)NQ * slot + i];
    }
done:
    free(state);
    if (need)
        for (int t = 0; t <= nsteps; ++t)
            free(need[t]);
    free(need);
    free(nneed);
    return status;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (n <= 0: one per processor). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}
