/*
 * fdlb_oracle.c -- plain, slow CPU reference of the finite-difference lattice Boltzmann
 * scheme of Gan, Xu, Zhang, Yu and Li, "Two-dimensional lattice Boltzmann model for
 * compressible flows with high Mach number" (arXiv:0801.4169).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle for the GPU path.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant generator with the HIP library, and the
 * library never calls it.
 *
 * What it computes (paper sections and equations):
 *   - velocity set: Sec. 2, Eq. (dvm_eq_1): v0 = 0 and v_ki = v_k (cos(i pi/4), sin(i pi/4)),
 *     i = 1..8, k = 1..4;
 *   - moments: Sec. 2, Eqs. (n_eq), (nu_eq), (p_eq): n = sum f, n u = sum v f,
 *     P = n T = sum (v - u)^2 f / 2, taken from f (equal to the f^eq sums by construction);
 *   - equilibrium: Sec. 2, Eqs. (feq_eq), (fk_eq1), (f0_eq), (kl_eq);
 *   - update: Sec. 3, Eq. (dis_eq1) with Eqs. (add3), (add4): lines I-IV per spatial
 *     direction alpha, summed over alpha = x, y, plus the BGK term once; any of the four
 *     lines may be left out (orc_params.lines), as Sec. 4 and Fig. 3 do.
 *
 * Readings where the paper is silent or garbled (each is listed in the design notes):
 *   R1  the bracket of Eq. (feq_eq) encloses all five groups (the printed one is unmatched);
 *   R3  P = n T with T = E/n - u^2/2 and E = sum |v|^2 f / 2 (identical to the peculiar
 *       form of Eq. (p_eq)), so the gas has two translational degrees of freedom;
 *   R5  two-dimensional update: every line of Eq. (dis_eq1) is applied per direction and
 *       the x and y contributions are summed in one explicit stage; no cross terms;
 *   R7  every right-hand-side term is taken at the old time level;
 *   R11 a reflecting wall is a specular mirror about the cell face;
 *   R12 Dirichlet ghosts hold f^eq of the prescribed state; outflow copies the edge cell.
 *
 * Canonical evaluation order.  The GPU FP64 path is meant to reproduce this file bit for
 * bit, so every expression below is written with explicit parentheses or temporaries and
 * the file is compiled with -ffp-contract=off (no fused multiply-add).  Sums over the
 * velocities run in ascending index q.  The velocity index is q = 0 for the rest particle
 * and q = 1 + 8 (k - 1) + (i - 1) for speed k and direction i.
 *
 * Precision: REAL is double by default.  Built with -DORC_QUAD, REAL is __float128 and the
 * same algorithm measures the oracle's own FP64 rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_QUAD
typedef __float128 REAL;
#define RABS(a) __builtin_fabsf128(a)
#define RFINITE(a) ((a) == (a) && (a) - (a) == 0)
#else
typedef double REAL;
#define RABS(a) fabs(a)
#define RFINITE(a) isfinite(a)
#endif

#define NQ 33

/* Boundary kinds, one per side (x-, x+, y-, y+). */
enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1, ORC_DIRICHLET = 2, ORC_WALL = 3 };

typedef struct {
    int32_t nx, ny;
    double dx, dy, dt, tau, lambda;
    double v[4];             /* v1..v4 of Eq. (dvm_eq_1) */
    int32_t bc[4];           /* x-, x+, y-, y+ */
    double bc_state[4][4];   /* (rho, ux, uy, T) per side, Dirichlet only */
    int32_t lines;           /* bit 0..3 = lines I..IV of Eq. (dis_eq1); 15 = full scheme */
    int32_t theta_fixed;     /* 0: switching function Eq. (add4); 1: theta := theta_value */
    double theta_value;
    /* Lower segment of a side (the double Mach reflection of Sec. 5.2.2: a wall that begins
     * at x = 0.08, a top state that changes at a moving point).  Ghost cells whose centre
     * coordinate along the side (x on the y sides, y on the x sides) lies below
     * split[s] + split_rate[s] * t, t = (step0 + step) * dt, take bc_lo[s] and its state;
     * bc_lo[s] = 0 (periodic) means the side has no lower segment. */
    int32_t bc_lo[4];
    double bc_lo_state[4][4];
    double split[4], split_rate[4];
    int64_t step0;
} orc_params;

/* Direction table of Eq. (dvm_eq_1) for i = 1..8: cos(i pi/4), sin(i pi/4) with the exact
 * values 0 and +-1 where they are exact, and s = sqrt(2)/2 rounded once otherwise. */
static const double ORC_S = 0.70710678118654757; /* nearest double to sqrt(2)/2 */

static void dir_cs(int i, double *c, double *s)
{
    switch (i) {
    case 1: *c = ORC_S;  *s = ORC_S;  break;
    case 2: *c = 0.0;    *s = 1.0;    break;
    case 3: *c = -ORC_S; *s = ORC_S;  break;
    case 4: *c = -1.0;   *s = 0.0;    break;
    case 5: *c = -ORC_S; *s = -ORC_S; break;
    case 6: *c = 0.0;    *s = -1.0;   break;
    case 7: *c = ORC_S;  *s = -ORC_S; break;
    default: *c = 1.0;   *s = 0.0;    break; /* i = 8 */
    }
}

/* Velocity components, Eq. (dvm_eq_1). */
void orc_velocities(const double v[4], double vx[NQ], double vy[NQ])
{
    vx[0] = 0.0;
    vy[0] = 0.0;
    for (int k = 1; k <= 4; ++k)
        for (int i = 1; i <= 8; ++i) {
            double c, s;
            dir_cs(i, &c, &s);
            int q = 1 + 8 * (k - 1) + (i - 1);
            vx[q] = v[k - 1] * c;
            vy[q] = v[k - 1] * s;
        }
}

/* Mirror maps used by the reflecting wall: the velocity with vx (or vy) reversed. */
static int mirror_x(int q)
{
    if (q == 0) return 0;
    int k = (q - 1) / 8, i = (q - 1) % 8 + 1;
    int im = ((4 - i) % 8 + 8) % 8;
    if (im == 0) im = 8;
    return 1 + 8 * k + (im - 1);
}

static int mirror_y(int q)
{
    if (q == 0) return 0;
    int k = (q - 1) / 8, i = (q - 1) % 8 + 1;
    int im = (i == 8) ? 8 : 8 - i;
    return 1 + 8 * k + (im - 1);
}

int orc_mirror(int axis, int q) { return axis == 0 ? mirror_x(q) : mirror_y(q); }

/* ------------------------------------------------------------------------------------ */
/* Model: constants, weights F_k, equilibrium, moments.                                   */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    REAL vx[NQ], vy[NQ], e[NQ]; /* e_q = |v_q|^2 / 2 */
    REAL v[4];
} model_t;

static void model_init(model_t *m, const double v[4])
{
    double vx[NQ], vy[NQ];
    orc_velocities(v, vx, vy);
    for (int q = 0; q < NQ; ++q) {
        m->vx[q] = (REAL)vx[q];
        m->vy[q] = (REAL)vy[q];
        m->e[q] = (REAL)0.5 * (m->vx[q] * m->vx[q] + m->vy[q] * m->vy[q]);
    }
    for (int k = 0; k < 4; ++k) m->v[k] = (REAL)v[k];
}

/* Weights of Eqs. (fk_eq1), (f0_eq); the index {k+l} of Eq. (kl_eq) is cyclic in 1..4.
 * F[0] is F_0 and F[k] is F_k for k = 1..4. */
static void weights(const model_t *m, REAL th, REAL F[5])
{
    REAL th2 = th * th;
    REAL th3 = th2 * th;
    REAL th4 = th3 * th;
    for (int k = 0; k < 4; ++k) {
        REAL vk2 = m->v[k] * m->v[k];
        REAL a = m->v[(k + 1) % 4] * m->v[(k + 1) % 4];
        REAL b = m->v[(k + 2) % 4] * m->v[(k + 2) % 4];
        REAL d = m->v[(k + 3) % 4] * m->v[(k + 3) % 4];
        REAL num = (REAL)48 * th4 - (REAL)6 * (a + b + d) * th3 + (a * b + b * d + d * a) * th2
                   - a * b * d / (REAL)4 * th;
        REAL den = vk2 * (vk2 - a) * (vk2 - b) * (vk2 - d);
        F[k + 1] = num / den;
    }
    F[0] = (REAL)1 - (REAL)8 * (F[1] + F[2] + F[3] + F[4]);
}

/* Equilibrium of Eq. (feq_eq), read as n F_k times the full bracket (reading R1):
 *   f^eq = n F_k [ (1 - u^2/2T + u^4/8T^2) + (s/T)(1 - u^2/2T) + (s^2/2T^2)(1 - u^2/2T)
 *                  + s^3/6T^3 + s^4/24T^4 ],   s = v_q . u,  theta = T/m with m = 1.
 * It is evaluated as a polynomial in s whose coefficients c0..c4 are those of the bracket. */
static void feq(const model_t *m, REAL n, REAL ux, REAL uy, REAL T, REAL out[NQ])
{
    REAL F[5];
    weights(m, T, F);
    REAL u2 = ux * ux + uy * uy;
    REAL th2 = T * T;
    REAL th3 = th2 * T;
    REAL th4 = th3 * T;
    REAL h = (REAL)1 - u2 / ((REAL)2 * T);
    REAL c0 = h + (u2 * u2) / ((REAL)8 * th2);
    REAL c1 = h / T;
    REAL c2 = h / ((REAL)2 * th2);
    REAL c3 = (REAL)1 / ((REAL)6 * th3);
    REAL c4 = (REAL)1 / ((REAL)24 * th4);
    for (int q = 0; q < NQ; ++q) {
        int k = (q == 0) ? 0 : 1 + (q - 1) / 8;
        REAL nF = n * F[k];
        REAL s = m->vx[q] * ux + m->vy[q] * uy;
        REAL s2 = s * s;
        REAL s3 = s2 * s;
        REAL s4 = s3 * s;
        REAL poly = c0 + c1 * s + c2 * s2 + c3 * s3 + c4 * s4;
        out[q] = nF * poly;
    }
}

/* Moments of Eqs. (n_eq), (nu_eq), (p_eq) taken from f (reading R4), with the pressure
 * from the total energy (reading R3).  out = (n, ux, uy, T, P). */
static void moments(const model_t *m, const REAL f[NQ], REAL out[5])
{
    REAL n = 0, jx = 0, jy = 0, E = 0;
    for (int q = 0; q < NQ; ++q) {
        n = n + f[q];
        jx = jx + m->vx[q] * f[q];
        jy = jy + m->vy[q] * f[q];
        E = E + m->e[q] * f[q];
    }
    REAL ux = jx / n;
    REAL uy = jy / n;
    REAL u2 = ux * ux + uy * uy;
    REAL T = E / n - u2 / (REAL)2;
    out[0] = n;
    out[1] = ux;
    out[2] = uy;
    out[3] = T;
    out[4] = n * T;
}

/* Double-precision views of the model for the Python side and the tests. */
void orc_weights(const double v[4], double T, double F[5])
{
    model_t m;
    model_init(&m, v);
    REAL Fr[5];
    weights(&m, (REAL)T, Fr);
    for (int k = 0; k < 5; ++k) F[k] = (double)Fr[k];
}

void orc_feq(const double v[4], double n, double ux, double uy, double T, double out[NQ])
{
    model_t m;
    model_init(&m, v);
    REAL o[NQ];
    feq(&m, (REAL)n, (REAL)ux, (REAL)uy, (REAL)T, o);
    for (int q = 0; q < NQ; ++q) out[q] = (double)o[q];
}

void orc_moments(const double v[4], const double f[NQ], double out[5])
{
    model_t m;
    model_init(&m, v);
    REAL fr[NQ], o[5];
    for (int q = 0; q < NQ; ++q) fr[q] = (REAL)f[q];
    moments(&m, fr, o);
    for (int k = 0; k < 5; ++k) out[k] = (double)o[k];
}

/* ------------------------------------------------------------------------------------ */
/* Grid: ghost frame, switching function, Eq. (dis_eq1).                                  */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    orc_params p;
    model_t m;
    int nx, ny, gx, gy;        /* gx = nx + 4, gy = ny + 4: two ghost layers per side */
    REAL *g;                   /* f with ghost frame, [NQ][gy][gx] */
    REAL *P;                   /* pressure on the interior plus a one-cell ring, [ny+2][nx+2] */
    REAL *mom;                 /* (n, ux, uy, T) per interior cell, [4][ny][nx] */
    REAL bcf[8][NQ];           /* Dirichlet ghost vectors per side, then per lower segment */
    REAL k1[2][NQ], k2[2][NQ], k3[2][NQ]; /* line coefficients per direction alpha */
    REAL dtau, dtdx, dtdy;
} grid_t;

#define GI(G, q, x, y) ((G)->g[((size_t)(q) * (G)->gy + (size_t)((y) + 2)) * (G)->gx + (size_t)((x) + 2)])
#define PI_(G, x, y) ((G)->P[(size_t)((y) + 1) * (size_t)((G)->nx + 2) + (size_t)((x) + 1)])

static int grid_init(grid_t *G, const orc_params *p)
{
    memset(G, 0, sizeof(*G));
    G->p = *p;
    G->nx = p->nx;
    G->ny = p->ny;
    G->gx = p->nx + 4;
    G->gy = p->ny + 4;
    model_init(&G->m, p->v);
    G->g = (REAL *)calloc((size_t)NQ * G->gx * G->gy, sizeof(REAL));
    G->P = (REAL *)calloc((size_t)(G->nx + 2) * (G->ny + 2), sizeof(REAL));
    G->mom = (REAL *)calloc((size_t)4 * G->nx * G->ny, sizeof(REAL));
    if (!G->g || !G->P || !G->mom) return -1;
    /* Courant numbers of Eq. (add3) and the coefficients of lines I-III. */
    for (int a = 0; a < 2; ++a) {
        REAL dr = (REAL)(a == 0 ? p->dx : p->dy);
        for (int q = 0; q < NQ; ++q) {
            REAL vq = (a == 0) ? G->m.vx[q] : G->m.vy[q];
            REAL c = vq * (REAL)p->dt / dr;
            G->k1[a][q] = c / (REAL)2;
            G->k2[a][q] = c * c / (REAL)2;
            G->k3[a][q] = c * ((REAL)1 - c * c) / (REAL)12;
        }
    }
    G->dtau = (REAL)p->dt / (REAL)p->tau;
    for (int side = 0; side < 4; ++side) {
        if (p->bc[side] == ORC_DIRICHLET)
            feq(&G->m, (REAL)p->bc_state[side][0], (REAL)p->bc_state[side][1],
                (REAL)p->bc_state[side][2], (REAL)p->bc_state[side][3], G->bcf[side]);
        if (p->bc_lo[side] == ORC_DIRICHLET)
            feq(&G->m, (REAL)p->bc_lo_state[side][0], (REAL)p->bc_lo_state[side][1],
                (REAL)p->bc_lo_state[side][2], (REAL)p->bc_lo_state[side][3], G->bcf[4 + side]);
    }
    return 0;
}

static void grid_free(grid_t *G)
{
    free(G->g);
    free(G->P);
    free(G->mom);
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Condition of the ghost cells of `side` at position i along it (row y on the x sides,
 * column x on the y sides) at time t: the side's own, or its lower segment's.  Returns the
 * kind and sets *slot to the index of the Dirichlet vector. */
static int side_kind(const orc_params *p, int side, int i, double t, int *slot)
{
    *slot = side;
    if (p->bc_lo[side] != ORC_PERIODIC) {
        const double d = side < 2 ? p->dy : p->dx;
        const double c = ((double)i + 0.5) * d;
        const double s = p->split[side] + p->split_rate[side] * t;
        if (c < s) {
            *slot = 4 + side;
            return p->bc_lo[side];
        }
    }
    return p->bc[side];
}

/* Ghost layers (two per side, corners unused) from the interior, per boundary kind. */
static void fill_ghosts(grid_t *G, double t)
{
    const int nx = G->nx, ny = G->ny;
    for (int q = 0; q < NQ; ++q) {
        for (int y = 0; y < ny; ++y)
            for (int gl = 1; gl <= 2; ++gl) {
                int xl = -gl, xr = nx - 1 + gl, sl;
                switch (side_kind(&G->p, 0, y, t, &sl)) {
                case ORC_PERIODIC: GI(G, q, xl, y) = GI(G, q, wrap(xl, nx), y); break;
                case ORC_OUTFLOW: GI(G, q, xl, y) = GI(G, q, 0, y); break;
                case ORC_DIRICHLET: GI(G, q, xl, y) = G->bcf[sl][q]; break;
                default: GI(G, q, xl, y) = GI(G, mirror_x(q), -1 - xl, y); break;
                }
                switch (side_kind(&G->p, 1, y, t, &sl)) {
                case ORC_PERIODIC: GI(G, q, xr, y) = GI(G, q, wrap(xr, nx), y); break;
                case ORC_OUTFLOW: GI(G, q, xr, y) = GI(G, q, nx - 1, y); break;
                case ORC_DIRICHLET: GI(G, q, xr, y) = G->bcf[sl][q]; break;
                default: GI(G, q, xr, y) = GI(G, mirror_x(q), 2 * nx - 1 - xr, y); break;
                }
            }
        for (int x = 0; x < nx; ++x)
            for (int gl = 1; gl <= 2; ++gl) {
                int yb = -gl, yt = ny - 1 + gl, sl;
                switch (side_kind(&G->p, 2, x, t, &sl)) {
                case ORC_PERIODIC: GI(G, q, x, yb) = GI(G, q, x, wrap(yb, ny)); break;
                case ORC_OUTFLOW: GI(G, q, x, yb) = GI(G, q, x, 0); break;
                case ORC_DIRICHLET: GI(G, q, x, yb) = G->bcf[sl][q]; break;
                default: GI(G, q, x, yb) = GI(G, mirror_y(q), x, -1 - yb); break;
                }
                switch (side_kind(&G->p, 3, x, t, &sl)) {
                case ORC_PERIODIC: GI(G, q, x, yt) = GI(G, q, x, wrap(yt, ny)); break;
                case ORC_OUTFLOW: GI(G, q, x, yt) = GI(G, q, x, ny - 1); break;
                case ORC_DIRICHLET: GI(G, q, x, yt) = G->bcf[sl][q]; break;
                default: GI(G, q, x, yt) = GI(G, mirror_y(q), x, 2 * ny - 1 - yt); break;
                }
            }
    }
}

static void cell_moments(const grid_t *G, int x, int y, REAL out[5])
{
    REAL f[NQ];
    for (int q = 0; q < NQ; ++q) f[q] = GI(G, q, x, y);
    moments(&G->m, f, out);
}

/* Pressure on the interior and the one-cell ring, moments on the interior. */
static void all_moments(grid_t *G, int nthreads)
{
    const int nx = G->nx, ny = G->ny;
    (void)nthreads;
    /* interior cells plus the x ring (x = -1, nx) of every row */
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = -1; x <= nx; ++x) {
            REAL mo[5];
            cell_moments(G, x, y, mo);
            PI_(G, x, y) = mo[4];
            if (x >= 0 && x < nx)
                for (int c = 0; c < 4; ++c)
                    G->mom[((size_t)c * ny + y) * nx + x] = mo[c];
        }
    /* the y ring (y = -1, ny) */
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int r = 0; r < 2; ++r)
        for (int x = 0; x < nx; ++x) {
            REAL mo[5];
            const int y = r == 0 ? -1 : ny;
            cell_moments(G, x, y, mo);
            PI_(G, x, y) = mo[4];
        }
}

/* Switching function of Eq. (add4) and the line-IV coefficient theta |kappa| (1-|kappa|)/2
 * with kappa of Eq. (add3). */
static REAL av_coeff(const grid_t *G, REAL Pm, REAL P0, REAL Pp, REAL u, REAL dr)
{
    REAL theta;
    if (G->p.theta_fixed)
        theta = (REAL)G->p.theta_value;
    else
        theta = (REAL)G->p.lambda * RABS((Pp - (REAL)2 * P0 + Pm) / (Pp + (REAL)2 * P0 + Pm));
    REAL kap = RABS(u * (REAL)G->p.dt / dr);
    return theta * kap * ((REAL)1 - kap) / (REAL)2;
}

/* One step of Eq. (dis_eq1) on every interior cell; out is [NQ][ny][nx]. */
static void update(const grid_t *G, REAL *out, int nthreads)
{
    const int nx = G->nx, ny = G->ny;
    const int L = G->p.lines;
    (void)nthreads;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            REAL n = G->mom[((size_t)0 * ny + y) * nx + x];
            REAL ux = G->mom[((size_t)1 * ny + y) * nx + x];
            REAL uy = G->mom[((size_t)2 * ny + y) * nx + x];
            REAL T = G->mom[((size_t)3 * ny + y) * nx + x];
            REAL P0 = PI_(G, x, y);
            REAL a[2];
            a[0] = av_coeff(G, PI_(G, x - 1, y), P0, PI_(G, x + 1, y), ux, (REAL)G->p.dx);
            a[1] = av_coeff(G, PI_(G, x, y - 1), P0, PI_(G, x, y + 1), uy, (REAL)G->p.dy);
            REAL fe[NQ];
            feq(&G->m, n, ux, uy, T, fe);
            for (int q = 0; q < NQ; ++q) {
                REAL f0 = GI(G, q, x, y);
                REAL fn = f0;
                for (int al = 0; al < 2; ++al) {
                    int ex = (al == 0), ey = (al == 1);
                    REAL fp1 = GI(G, q, x + ex, y + ey);
                    REAL fm1 = GI(G, q, x - ex, y - ey);
                    REAL fp2 = GI(G, q, x + 2 * ex, y + 2 * ey);
                    REAL fm2 = GI(G, q, x - 2 * ex, y - 2 * ey);
                    REAL d1 = fp1 - fm1;
                    REAL d2 = fp1 - (REAL)2 * f0 + fm1;
                    REAL d3 = fp2 - (REAL)2 * fp1 + (REAL)2 * fm1 - fm2;
                    if (L & 1) fn = fn - G->k1[al][q] * d1; /* line I   */
                    if (L & 2) fn = fn + G->k2[al][q] * d2; /* line II  */
                    if (L & 4) fn = fn + G->k3[al][q] * d3; /* line III */
                    if (L & 8) fn = fn + a[al] * d2;        /* line IV  */
                }
                fn = fn - G->dtau * (f0 - fe[q]);           /* BGK term of line I */
                out[((size_t)q * ny + y) * nx + x] = fn;
            }
        }
    }
}

/* Non-physical state: n <= 0, T <= 0, a non-finite moment, or |kappa| >= 1 somewhere. */
static int nonphysical(const grid_t *G)
{
    const int nx = G->nx, ny = G->ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            REAL n = G->mom[((size_t)0 * ny + y) * nx + x];
            REAL ux = G->mom[((size_t)1 * ny + y) * nx + x];
            REAL uy = G->mom[((size_t)2 * ny + y) * nx + x];
            REAL T = G->mom[((size_t)3 * ny + y) * nx + x];
            if (!(RFINITE(n) && RFINITE(ux) && RFINITE(uy) && RFINITE(T))) return 1;
            if (!(n > 0) || !(T > 0)) return 1;
            if (RABS(ux * (REAL)G->p.dt / (REAL)G->p.dx) >= 1) return 1;
            if (RABS(uy * (REAL)G->p.dt / (REAL)G->p.dy) >= 1) return 1;
        }
    return 0;
}

static void load_interior(grid_t *G, const REAL *f)
{
    const int nx = G->nx, ny = G->ny;
    for (int q = 0; q < NQ; ++q)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                GI(G, q, x, y) = f[((size_t)q * ny + y) * nx + x];
}

/* Runs nsteps from f (in place, [NQ][ny][nx]).  Returns the number of the first step whose
 * input state was non-physical (counting from 0), nsteps + 1 if only the final state is,
 * or -1 if none.  The run continues through non-physical states. */
static long run(const orc_params *p, REAL *f, long nsteps, int nthreads, int *err)
{
    grid_t G;
    *err = 0;
    if (grid_init(&G, p) != 0) {
        grid_free(&G);
        *err = 1;
        return -1;
    }
    long first_bad = -1;
    for (long s = 0; s < nsteps; ++s) {
        load_interior(&G, f);
        fill_ghosts(&G, (double)(p->step0 + s) * p->dt);
        all_moments(&G, nthreads);
        if (first_bad < 0 && nonphysical(&G)) first_bad = s;
        update(&G, f, nthreads);
    }
    load_interior(&G, f);
    fill_ghosts(&G, (double)(p->step0 + nsteps) * p->dt);
    all_moments(&G, nthreads);
    if (first_bad < 0 && nonphysical(&G)) first_bad = nsteps + 1;
    grid_free(&G);
    return first_bad;
}

/* ------------------------------------------------------------------------------------ */
/* Exported driver API (double in, double out).                                           */
/* ------------------------------------------------------------------------------------ */

static int check_params(const orc_params *p)
{
    if (p->nx < 1 || p->ny < 1) return 1;
    if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0) || !(p->tau > 0)) return 1;
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] < 0 || p->bc[s] > 3) return 1;
        if (p->bc[s] == ORC_WALL && ((s < 2 && p->nx < 2) || (s >= 2 && p->ny < 2))) return 1;
        if (p->bc_lo[s] < 0 || p->bc_lo[s] > 3) return 1;
        if (p->bc_lo[s] != ORC_PERIODIC && p->bc[s] == ORC_PERIODIC) return 1;
        if (p->bc_lo[s] == ORC_WALL && ((s < 2 && p->nx < 2) || (s >= 2 && p->ny < 2))) return 1;
    }
    if ((p->bc[0] == ORC_PERIODIC) != (p->bc[1] == ORC_PERIODIC)) return 1;
    if ((p->bc[2] == ORC_PERIODIC) != (p->bc[3] == ORC_PERIODIC)) return 1;
    return 0;
}

/* f := f^eq(rho, ux, uy, T) per cell; fields are [ny][nx], f is [NQ][ny][nx]. */
int orc_init_state(const orc_params *p, const double *rho, const double *ux, const double *uy,
                   const double *T, double *f_out)
{
    if (check_params(p)) return 1;
    model_t m;
    model_init(&m, p->v);
    const size_t nc = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < nc; ++c) {
        REAL fe[NQ];
        feq(&m, (REAL)rho[c], (REAL)ux[c], (REAL)uy[c], (REAL)T[c], fe);
        for (int q = 0; q < NQ; ++q) f_out[(size_t)q * nc + c] = (double)fe[q];
    }
    return 0;
}

/* Runs nsteps from f (double, in place).  first_bad receives the first non-physical step
 * (see run()). */
int orc_run_f(const orc_params *p, double *f, long nsteps, int nthreads, long *first_bad)
{
    if (check_params(p)) return 1;
    const size_t n = (size_t)NQ * p->nx * p->ny;
    REAL *fr = (REAL *)malloc(n * sizeof(REAL));
    if (!fr) return 2;
    for (size_t i = 0; i < n; ++i) fr[i] = (REAL)f[i];
    int err = 0;
    long fb = run(p, fr, nsteps, nthreads, &err);
    for (size_t i = 0; i < n; ++i) f[i] = (double)fr[i];
    free(fr);
    if (first_bad) *first_bad = fb;
    return err ? 2 : 0;
}

/* Initial equilibrium from the fields, nsteps, then the fields (n, ux, uy, T) of the final
 * state.  Everything in between stays in REAL, so the quad build never rounds to double. */
int orc_run_state(const orc_params *p, const double *rho, const double *ux, const double *uy,
                  const double *T, long nsteps, int nthreads, double *rho_o, double *ux_o,
                  double *uy_o, double *T_o, long *first_bad)
{
    if (check_params(p)) return 1;
    model_t m;
    model_init(&m, p->v);
    const size_t nc = (size_t)p->nx * p->ny;
    REAL *fr = (REAL *)malloc((size_t)NQ * nc * sizeof(REAL));
    if (!fr) return 2;
    for (size_t c = 0; c < nc; ++c) {
        REAL fe[NQ];
        feq(&m, (REAL)rho[c], (REAL)ux[c], (REAL)uy[c], (REAL)T[c], fe);
        for (int q = 0; q < NQ; ++q) fr[(size_t)q * nc + c] = fe[q];
    }
    int err = 0;
    long fb = run(p, fr, nsteps, nthreads, &err);
    for (size_t c = 0; c < nc; ++c) {
        REAL f[NQ], mo[5];
        for (int q = 0; q < NQ; ++q) f[q] = fr[(size_t)q * nc + c];
        moments(&m, f, mo);
        rho_o[c] = (double)mo[0];
        ux_o[c] = (double)mo[1];
        uy_o[c] = (double)mo[2];
        T_o[c] = (double)mo[3];
    }
    free(fr);
    if (first_bad) *first_bad = fb;
    return err ? 2 : 0;
}

/* Fields (n, ux, uy, T) of a double-precision f. */
int orc_fields(const orc_params *p, const double *f, double *rho_o, double *ux_o, double *uy_o,
               double *T_o)
{
    model_t m;
    model_init(&m, p->v);
    const size_t nc = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < nc; ++c) {
        REAL fr[NQ], mo[5];
        for (int q = 0; q < NQ; ++q) fr[q] = (REAL)f[(size_t)q * nc + c];
        moments(&m, fr, mo);
        rho_o[c] = (double)mo[0];
        ux_o[c] = (double)mo[1];
        uy_o[c] = (double)mo[2];
        T_o[c] = (double)mo[3];
    }
    return 0;
}

int orc_real_bytes(void) { return (int)sizeof(REAL); }
