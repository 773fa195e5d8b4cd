// fdlb_kernels.hip -- HIP kernels of the FDLB hot path for gfx950 (MI355X).
//
// One time step of the scheme of Gan, Xu, Zhang, Yu and Li (arXiv:0801.4169), Sec. 3,
// Eq. (dis_eq1) with the switching function of Eq. (add4), is ONE fused kernel launch:
//   A1  load the cell's 33 distributions and the halo of its tile (two cells in x and y,
//       boundary conditions applied on the fly)          -> registers / LDS
//   A2  moments n, u, T, P of the cell (Eqs. n_eq, nu_eq, p_eq)
//   A3  switching function theta and kappa per direction (Eqs. add3, add4) from the
//       neighbours' pressure, written by the previous step
//   A4  weights F_k(T) and the polynomial coefficients of f^eq (Eqs. feq_eq, fk_eq1, f0_eq)
//   A5  per velocity: f^eq, lines I-IV in x and y, BGK relaxation
//   A6  store f_new (the other ping-pong half), then the moments of f_new give the
//       pressure the next step's switching function reads, and the non-physical flag.
//
// Work decomposition: one workgroup per TX x TY tile, one thread per cell.  A thread keeps
// its cell's 33 values in registers; neighbours come from an LDS copy of one or two
// velocity planes of the tile plus a two-cell halo (double buffered, one barrier per
// stage).  The halo of the next stage is fetched while the current one computes.
// Workgroups are assigned to tiles so that each XCD (each L2) sweeps a contiguous band.
//
// Float64 mode evaluates every expression in one fixed order without contraction
// (compiled with -ffp-contract=off): sums over velocities run in ascending index, the
// equilibrium is a polynomial in s = v.u with coefficients c0..c4 summed in ascending
// power, and the update adds lines I, II, III, IV for x, then for y, then the BGK term.
// Float32 mode stores f in float32, evaluates f^eq and the stencil in float32 with fused
// multiply-adds, and accumulates the moments in float64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fdlb_internal.h"

namespace fdlb {

// ------------------------------------------------------------------------------------
// Velocity set, Eq. (dvm_eq_1).  q = 0 rest; q = 1 + 8k + (i-1), speed k = 0..3,
// direction i = 1..8 at angle i pi/4.  Components are sign * magnitude, the magnitude being
// v_k on an axis and v_k sqrt(2)/2 on a diagonal.
// ------------------------------------------------------------------------------------
__host__ __device__ constexpr int qk(int q) { return q == 0 ? 0 : (q - 1) / 8; }
__host__ __device__ constexpr int qi(int q) { return q == 0 ? 0 : (q - 1) % 8 + 1; }
__host__ __device__ constexpr int qsx(int q) {
    return q == 0 ? 0 : (qi(q) == 1 || qi(q) == 7 || qi(q) == 8) ? 1 : (qi(q) == 3 || qi(q) == 4 || qi(q) == 5) ? -1 : 0;
}
__host__ __device__ constexpr int qsy(int q) {
    return q == 0 ? 0 : (qi(q) == 1 || qi(q) == 2 || qi(q) == 3) ? 1 : (qi(q) == 5 || qi(q) == 6 || qi(q) == 7) ? -1 : 0;
}
__host__ __device__ constexpr bool qdiag(int q) { return q != 0 && (qi(q) % 2) == 1; }
// velocity with the x (resp. y) component reversed
__host__ __device__ constexpr int qmx(int q) {
    return q == 0 ? 0 : 1 + 8 * qk(q) + ((((4 - qi(q)) % 8 + 8) % 8 == 0 ? 8 : ((4 - qi(q)) % 8 + 8) % 8) - 1);
}
__host__ __device__ constexpr int qmy(int q) { return q == 0 ? 0 : 1 + 8 * qk(q) + ((qi(q) == 8 ? 8 : 8 - qi(q)) - 1); }

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class S>
__device__ __forceinline__ double to_d(S x) { return static_cast<double>(x); }

// ------------------------------------------------------------------------------------
// Moments of a 33-vector, ascending q, float64 (Eqs. n_eq, nu_eq; energy sum |v|^2 f / 2).
// MIR = 0: the vector itself; 1: its mirror in x; 2: its mirror in y (the ghost cell of a
// reflecting side, whose value at q is the cell's value at the mirrored velocity).
// ------------------------------------------------------------------------------------
template <int MIR, class S>
__device__ __forceinline__ void moments33(const Inst &I, const S (&f)[NQ], double &n, double &jx, double &jy,
                                          double &E) {
    n = 0.0;
    jx = 0.0;
    jy = 0.0;
    E = 0.0;
    static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int src = MIR == 0 ? q : MIR == 1 ? qmx(q) : qmy(q);
        const double fq = to_d(f[src]);
        n = n + fq;
        if constexpr (q > 0) {
            constexpr int k = qk(q);
            const double mag = qdiag(q) ? I.vs[k] : I.v[k];
            if constexpr (qsx(q) > 0) jx = jx + mag * fq;
            if constexpr (qsx(q) < 0) jx = jx - mag * fq;
            if constexpr (qsy(q) > 0) jy = jy + mag * fq;
            if constexpr (qsy(q) < 0) jy = jy - mag * fq;
            const double e = qdiag(q) ? I.edg[k] : I.eax[k];
            E = E + e * fq;
        }
    });
}

// (n, jx, jy, E) -> u, T, P = n T (reading: T = E/n - u^2/2, two degrees of freedom)
__device__ __forceinline__ void primitive(double n, double jx, double jy, double E, double &ux, double &uy,
                                          double &T, double &P) {
    ux = jx / n;
    uy = jy / n;
    const double u2 = ux * ux + uy * uy;
    T = E / n - u2 / 2.0;
    P = n * T;
}

__device__ __forceinline__ bool nonphysical(const Inst &I, double n, double ux, double uy, double T) {
    const double s = n + ux + uy + T;
    if (!(s - s == 0.0)) return true;  // a NaN or an infinity
    if (!(n > 0.0) || !(T > 0.0)) return true;
    if (fabs(ux * I.dt / I.dx) >= 1.0) return true;
    if (fabs(uy * I.dt / I.dy) >= 1.0) return true;
    return false;
}

// Line-IV coefficient theta |kappa| (1 - |kappa|) / 2, Eqs. (add3), (add4).
__device__ __forceinline__ double av_coeff(double lam, double Pm, double P0, double Pp, double u, double dt,
                                           double dr) {
    const double th = lam * fabs((Pp - 2.0 * P0 + Pm) / (Pp + 2.0 * P0 + Pm));
    const double kap = fabs(u * dt / dr);
    return th * kap * (1.0 - kap) / 2.0;
}

// Polynomial form of Eq. (feq_eq): f^eq_q = (n F_k) (c0 + c1 s + c2 s^2 + c3 s^3 + c4 s^4).
struct Coef {
    double c0, c1, c2, c3, c4;
    double nF[5];
};

__device__ __forceinline__ void equilibrium_coefs(const Inst &I, double n, double ux, double uy, double T,
                                                  Coef &C) {
    const double th2 = T * T;
    const double th3 = th2 * T;
    const double th4 = th3 * T;
    double F[5];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double num = 48.0 * th4 - I.FA[k] * th3 + I.FB[k] * th2 - I.FC[k] * T;
        F[k + 1] = num / I.Fden[k];
    }
    F[0] = 1.0 - 8.0 * (F[1] + F[2] + F[3] + F[4]);
    const double u2 = ux * ux + uy * uy;
    const double h = 1.0 - u2 / (2.0 * T);
    C.c0 = h + (u2 * u2) / (8.0 * th2);
    C.c1 = h / T;
    C.c2 = h / (2.0 * th2);
    C.c3 = 1.0 / (6.0 * th3);
    C.c4 = 1.0 / (24.0 * th4);
#pragma unroll
    for (int k = 0; k < 5; ++k) C.nF[k] = n * F[k];
}

// x (resp. y) part of s = v . u for velocity q, as a signed product.
template <int Q, class A>
__device__ __forceinline__ A s_of(A mag, A ux, A uy) {
    constexpr int sx = qsx(Q), sy = qsy(Q);
    if constexpr (sx != 0 && sy != 0) {
        const A a = mag * ux;
        const A b = mag * uy;
        return (sx > 0 ? a : -a) + (sy > 0 ? b : -b);
    } else if constexpr (sx != 0) {
        const A a = mag * ux;
        return sx > 0 ? a : -a;
    } else if constexpr (sy != 0) {
        const A b = mag * uy;
        return sy > 0 ? b : -b;
    } else {
        return A(0);
    }
}

// Arithmetic policy.  Exact: separate multiply and add (matches a plain evaluation with
// no contraction).  Fused: fma.
template <bool FUSE, class A>
__device__ __forceinline__ A madd(A x, A k, A d) {
    if constexpr (FUSE) {
        return __builtin_fma(k, d, x);
    } else {
        const A t = k * d;
        return x + t;
    }
}
template <bool FUSE, class A>
__device__ __forceinline__ A msub(A x, A k, A d) {
    if constexpr (FUSE) {
        return __builtin_fma(-k, d, x);
    } else {
        const A t = k * d;
        return x - t;
    }
}
template <bool FUSE>
__device__ __forceinline__ float madd(float x, float k, float d) {
    if constexpr (FUSE) return __builtin_fmaf(k, d, x); else { const float t = k * d; return x + t; }
}
template <bool FUSE>
__device__ __forceinline__ float msub(float x, float k, float d) {
    if constexpr (FUSE) return __builtin_fmaf(-k, d, x); else { const float t = k * d; return x - t; }
}

// Per-cell coefficients in the arithmetic type of the per-velocity work.
template <class A>
struct CellA {
    A c0, c1, c2, c3, c4;
    A nF[5];
    A ux, uy, ax, ay, dtau;
};

// One direction alpha of Eq. (dis_eq1): lines I, II, III, IV.  SGN is the sign of the
// velocity component (0: only line IV, since c = 0 there).
template <int SGN, bool FUSE, class A>
__device__ __forceinline__ A lines_alpha(A fn, A f0, A fm2, A fm1, A fp1, A fp2, A k1, A k2, A k3, A av) {
    const A d2 = fp1 - A(2) * f0 + fm1;
    if constexpr (SGN != 0) {
        const A d1 = fp1 - fm1;
        const A d3 = fp2 - A(2) * fp1 + A(2) * fm1 - fm2;
        fn = SGN > 0 ? msub<FUSE>(fn, k1, d1) : madd<FUSE>(fn, k1, d1);  // line I
        fn = madd<FUSE>(fn, k2, d2);                                     // line II
        fn = SGN > 0 ? madd<FUSE>(fn, k3, d3) : msub<FUSE>(fn, k3, d3);  // line III
    }
    fn = madd<FUSE>(fn, av, d2);  // line IV
    return fn;
}

template <class S, int TX, int TY>
struct StepSmem {
    S buf[2][2][TY + 4][TX + 4];
};

// Source of a value of plane q at cell (x, y) that may lie outside the grid (boundary
// conditions of Sec. 5, readings R10-R12).  dside >= 0: the Dirichlet vector of that side;
// otherwise element offset `off` of plane q mirrored per `flip` (bit 0: x, bit 1: y).
struct Src {
    int off;
    int flip;
    int dside;
};

__device__ __forceinline__ Src map_cell(const Inst &I, int x, int y) {
    Src s{0, 0, -1};
    const int nx = I.nx, ny = I.ny;
    if ((unsigned)x >= (unsigned)nx) {
        const int side = x < 0 ? 0 : 1;
        const int kind = I.bc[side];
        if (kind == BC_DIRICHLET) {
            s.dside = side;
        } else if (kind == BC_PERIODIC) {
            x = ((x % nx) + nx) % nx;
        } else if (kind == BC_OUTFLOW) {
            x = x < 0 ? 0 : nx - 1;
        } else {
            x = x < 0 ? -1 - x : 2 * nx - 1 - x;
            s.flip |= 1;
        }
    }
    if ((unsigned)y >= (unsigned)ny) {
        const int side = y < 0 ? 2 : 3;
        const int kind = I.bc[side];
        if (kind == BC_DIRICHLET) {
            if (s.dside < 0) s.dside = side;
        } else if (kind == BC_PERIODIC) {
            y = ((y % ny) + ny) % ny;
        } else if (kind == BC_OUTFLOW) {
            y = y < 0 ? 0 : ny - 1;
        } else {
            y = y < 0 ? -1 - y : 2 * ny - 1 - y;
            s.flip |= 2;
        }
    }
    // cells further out than the stencil reaches only occur for idle threads of partial
    // tiles: clamp so every address stays inside the grid
    x = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    s.off = y * I.fpitch + x;
    return s;
}

template <int Q, class S>
__device__ __forceinline__ S load_src(const Inst &I, const S *__restrict__ fin, const Src &s, bool simple) {
    if (simple) return fin[(size_t)Q * I.fplane + s.off];
    if (s.dside >= 0) return static_cast<S>(I.bcf[s.dside][Q]);
    const int qq = s.flip == 0 ? Q : s.flip == 1 ? qmx(Q) : s.flip == 2 ? qmy(Q) : qmx(qmy(Q));
    return fin[(size_t)qq * I.fplane + s.off];
}

// Pressure of the neighbour (x, y) (at most one cell outside the grid).
__device__ __forceinline__ double load_P(const Inst &I, const double *__restrict__ P,
                                         const double *__restrict__ PW, int x, int y) {
    const int nx = I.nx, ny = I.ny;
    if ((unsigned)x >= (unsigned)nx) {
        const int side = x < 0 ? 0 : 1;
        const int kind = I.bc[side];
        const int yc = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        if (kind == BC_DIRICHLET) return I.bcP[side];
        if (kind == BC_WALL) return PW[side * I.wlen + yc];
        x = kind == BC_PERIODIC ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
    }
    if ((unsigned)y >= (unsigned)ny) {
        const int side = y < 0 ? 2 : 3;
        const int kind = I.bc[side];
        const int xc = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
        if (kind == BC_DIRICHLET) return I.bcP[side];
        if (kind == BC_WALL) return PW[side * I.wlen + xc];
        y = kind == BC_PERIODIC ? ((y % ny) + ny) % ny : (y < 0 ? 0 : ny - 1);
    }
    x = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    return P[y * I.ppitch + x];
}

// XCD-aware order: consecutive workgroup ids go round-robin over the 8 XCDs; give each XCD
// a contiguous run of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, local = b / 8;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Pressure of the cell and of the mirror images next to reflecting sides, after the
// cell's 33 values are final.
template <class S>
__device__ __forceinline__ void write_pressures(const Inst &I, const S (&f)[NQ], int x, int y, double *__restrict__ Pout,
                                                double *__restrict__ PWout) {
    double n, jx, jy, E, ux, uy, T, P;
    moments33<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P);
    Pout[y * I.ppitch + x] = P;
    if (nonphysical(I, n, ux, uy, T)) *I.flag = 1;
    if ((x == 0 && I.bc[0] == BC_WALL) || (x == I.nx - 1 && I.bc[1] == BC_WALL)) {
        moments33<1>(I, f, n, jx, jy, E);
        primitive(n, jx, jy, E, ux, uy, T, P);
        if (x == 0 && I.bc[0] == BC_WALL) PWout[0 * I.wlen + y] = P;
        if (x == I.nx - 1 && I.bc[1] == BC_WALL) PWout[1 * I.wlen + y] = P;
    }
    if ((y == 0 && I.bc[2] == BC_WALL) || (y == I.ny - 1 && I.bc[3] == BC_WALL)) {
        moments33<2>(I, f, n, jx, jy, E);
        primitive(n, jx, jy, E, ux, uy, T, P);
        if (y == 0 && I.bc[2] == BC_WALL) PWout[2 * I.wlen + x] = P;
        if (y == I.ny - 1 && I.bc[3] == BC_WALL) PWout[3 * I.wlen + x] = P;
    }
}

// ------------------------------------------------------------------------------------
// The fused step kernel.
// ------------------------------------------------------------------------------------
template <class S, class A, bool FUSE, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void step_kernel(const Inst *__restrict__ insts, const Tile *__restrict__ tiles,
                                                      int ntiles, int half) {
    constexpr int NT = TX * TY;
    constexpr int NH = 4 * (TX + TY);
    constexpr int NSLOT = (NH + NT - 1) / NT;
    __shared__ StepSmem<S, TX, TY> sm;

    const Tile tile = tiles[xcd_remap(blockIdx.x, ntiles)];
    const Inst &I = insts[tile.inst];
    const S *__restrict__ fin = static_cast<const S *>(I.f[half]);
    S *__restrict__ fout = static_cast<S *>(I.f[1 - half]);
    const double *__restrict__ Pin = I.P[half];
    const double *__restrict__ PWin = I.PW[half];
    double *__restrict__ Pout = I.P[1 - half];
    double *__restrict__ PWout = I.PW[1 - half];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = tile.x0 + tx, y = tile.y0 + ty;
    const int nx = I.nx, ny = I.ny;
    const bool valid = x < nx && y < ny;
    // a tile whose halo lies inside the grid needs no boundary mapping at all
    const bool simple = tile.x0 >= 2 && tile.y0 >= 2 && tile.x0 + TX + 2 <= nx && tile.y0 + TY + 2 <= ny;

    Src own;
    if (simple) own = Src{y * I.fpitch + x, 0, -1};
    else own = map_cell(I, x, y);
    Src hs[NSLOT];
    int hl[NSLOT];  // LDS position (ly * (TX + 4) + lx), -1 if the slot is unused
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const int hid = tid + j * NT;
        hl[j] = -1;
        hs[j] = Src{0, 0, -1};
        if (hid < NH) {
            int lx, ly;
            if (hid < 4 * TX) {
                const int r = hid / TX;
                lx = hid % TX + 2;
                ly = r < 2 ? r : TY + r;
            } else {
                const int h2 = hid - 4 * TX;
                const int c = h2 / TY;
                ly = h2 % TY + 2;
                lx = c < 2 ? c : TX + c;
            }
            hl[j] = ly * (TX + 4) + lx;
            const int X = tile.x0 + lx - 2, Y = tile.y0 + ly - 2;
            if (simple) hs[j] = Src{Y * I.fpitch + X, 0, -1};
            else hs[j] = map_cell(I, X, Y);
        }
    }

    // A1: own distributions
    S f[NQ];
    static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        f[q] = load_src<q>(I, fin, own, simple);
    });
    // halo of the first stage (rest particle) in flight during the moments
    S h0[NSLOT], h1[NSLOT];
#pragma unroll
    for (int j = 0; j < NSLOT; ++j)
        if (hl[j] >= 0) h0[j] = load_src<0>(I, fin, hs[j], simple);

    // A2: moments
    double n, jx, jy, E, ux, uy, T, P0;
    moments33<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P0);

    // A3: switching function and line-IV coefficients
    double Pxm, Pxp, Pym, Pyp;
    if (simple) {
        Pxm = Pin[y * I.ppitch + x - 1];
        Pxp = Pin[y * I.ppitch + x + 1];
        Pym = Pin[(y - 1) * I.ppitch + x];
        Pyp = Pin[(y + 1) * I.ppitch + x];
    } else {
        Pxm = load_P(I, Pin, PWin, x - 1, y);
        Pxp = load_P(I, Pin, PWin, x + 1, y);
        Pym = load_P(I, Pin, PWin, x, y - 1);
        Pyp = load_P(I, Pin, PWin, x, y + 1);
    }
    const double ax = av_coeff(I.lam, Pxm, P0, Pxp, ux, I.dt, I.dx);
    const double ay = av_coeff(I.lam, Pym, P0, Pyp, uy, I.dt, I.dy);

    // A4: equilibrium coefficients
    Coef C;
    equilibrium_coefs(I, n, ux, uy, T, C);
    CellA<A> ca;
    ca.c0 = static_cast<A>(C.c0);
    ca.c1 = static_cast<A>(C.c1);
    ca.c2 = static_cast<A>(C.c2);
    ca.c3 = static_cast<A>(C.c3);
    ca.c4 = static_cast<A>(C.c4);
#pragma unroll
    for (int k = 0; k < 5; ++k) ca.nF[k] = static_cast<A>(C.nF[k]);
    ca.ux = static_cast<A>(ux);
    ca.uy = static_cast<A>(uy);
    ca.ax = static_cast<A>(ax);
    ca.ay = static_cast<A>(ay);
    ca.dtau = static_cast<A>(I.dtau);

    const int own_l = (ty + 2) * (TX + 4) + (tx + 2);
    const size_t own_out = (size_t)y * I.fpitch + x;
    int b = 0;

    // A5: per velocity.  Stage 0 is the rest particle; stage 1 + 4k + j holds the pair of
    // opposite velocities q = 1 + 8k + j and q + 4 (s and -s share their powers).
    auto compute_q = [&](auto qc, const S *pl, A feq) {
        constexpr int q = decltype(qc)::value;
        constexpr int k = qk(q);
        constexpr int dg = qdiag(q) ? 1 : 0;
        const A f0 = static_cast<A>(f[q]);
        const A xm2 = static_cast<A>(pl[own_l - 2]), xm1 = static_cast<A>(pl[own_l - 1]);
        const A xp1 = static_cast<A>(pl[own_l + 1]), xp2 = static_cast<A>(pl[own_l + 2]);
        const A ym2 = static_cast<A>(pl[own_l - 2 * (TX + 4)]), ym1 = static_cast<A>(pl[own_l - (TX + 4)]);
        const A yp1 = static_cast<A>(pl[own_l + (TX + 4)]), yp2 = static_cast<A>(pl[own_l + 2 * (TX + 4)]);
        A fn = f0;
        if constexpr (qsx(q) != 0)
            fn = lines_alpha<qsx(q), FUSE, A>(fn, f0, xm2, xm1, xp1, xp2, static_cast<A>(I.k1[0][dg][k]),
                                              static_cast<A>(I.k2[0][dg][k]), static_cast<A>(I.k3[0][dg][k]), ca.ax);
        else
            fn = lines_alpha<0, FUSE, A>(fn, f0, xm2, xm1, xp1, xp2, A(0), A(0), A(0), ca.ax);
        if constexpr (qsy(q) != 0)
            fn = lines_alpha<qsy(q), FUSE, A>(fn, f0, ym2, ym1, yp1, yp2, static_cast<A>(I.k1[1][dg][k]),
                                              static_cast<A>(I.k2[1][dg][k]), static_cast<A>(I.k3[1][dg][k]), ca.ay);
        else
            fn = lines_alpha<0, FUSE, A>(fn, f0, ym2, ym1, yp1, yp2, A(0), A(0), A(0), ca.ay);
        fn = msub<FUSE>(fn, ca.dtau, f0 - feq);  // BGK
        const S out = static_cast<S>(fn);
        if (valid) fout[(size_t)q * I.fplane + own_out] = out;
        f[q] = out;
    };

    // stage 0: rest particle
    {
        S *pl = &sm.buf[b][0][0][0];
        pl[own_l] = f[0];
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) pl[hl[j]] = h0[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) {
                h0[j] = load_src<1>(I, fin, hs[j], simple);
                h1[j] = load_src<5>(I, fin, hs[j], simple);
            }
        const A feq0 = ca.nF[0] * ca.c0;
        compute_q(std::integral_constant<int, 0>{}, pl, feq0);
        b ^= 1;
    }
    static_for<0, 16>([&](auto sc) {
        constexpr int st = decltype(sc)::value;
        constexpr int k = st / 4;
        constexpr int qa = 1 + 8 * k + (st % 4);
        constexpr int qb = qa + 4;
        S *pa = &sm.buf[b][0][0][0];
        S *pb = &sm.buf[b][1][0][0];
        pa[own_l] = f[qa];
        pb[own_l] = f[qb];
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) {
                pa[hl[j]] = h0[j];
                pb[hl[j]] = h1[j];
            }
        __syncthreads();
        if constexpr (st + 1 < 16) {
            constexpr int na = 1 + 8 * ((st + 1) / 4) + ((st + 1) % 4);
#pragma unroll
            for (int j = 0; j < NSLOT; ++j)
                if (hl[j] >= 0) {
                    h0[j] = load_src<na>(I, fin, hs[j], simple);
                    h1[j] = load_src<na + 4>(I, fin, hs[j], simple);
                }
        }
        // equilibrium of the pair: the powers of s are shared, odd terms change sign
        const A mag = static_cast<A>(qdiag(qa) ? I.vs[k] : I.v[k]);
        const A s = s_of<qa, A>(mag, ca.ux, ca.uy);
        const A s2 = s * s;
        const A s3 = s2 * s;
        const A s4 = s3 * s;
        const A t1 = ca.c1 * s, t2 = ca.c2 * s2, t3 = ca.c3 * s3, t4 = ca.c4 * s4;
        const A pp = ca.c0 + t1 + t2 + t3 + t4;
        const A pm = ca.c0 - t1 + t2 - t3 + t4;
        const A feqa = ca.nF[k + 1] * pp;
        const A feqb = ca.nF[k + 1] * pm;
        compute_q(std::integral_constant<int, qa>{}, pa, feqa);
        compute_q(std::integral_constant<int, qb>{}, pb, feqb);
        b ^= 1;
    });

    // A6: pressure for the next step's switching function, wall images, flag
    if (valid) write_pressures(I, f, x, y, Pout, PWout);
}

// ------------------------------------------------------------------------------------
// Auxiliary kernels (not on the per-step path).
// ------------------------------------------------------------------------------------

// f := f^eq(fields) of half `half` (fields: rho, ux, uy, T planes of nx * ny float64).
template <class S>
__global__ __launch_bounds__(256) void fill_kernel(const Inst *__restrict__ insts, int inst, const double *__restrict__ fields, int half) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const size_t c = (size_t)y * I.nx + x, plane = (size_t)I.nx * I.ny;
    const double n = fields[c], ux = fields[plane + c], uy = fields[2 * plane + c], T = fields[3 * plane + c];
    Coef C;
    equilibrium_coefs(I, n, ux, uy, T, C);
    S *f = static_cast<S *>(I.f[half]);
    const size_t off = (size_t)y * I.fpitch + x;
    f[off] = static_cast<S>(C.nF[0] * C.c0);
    static_for<1, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double mag = qdiag(q) ? I.vs[qk(q)] : I.v[qk(q)];
        const double s = s_of<q, double>(mag, ux, uy);
        const double s2 = s * s;
        const double s3 = s2 * s;
        const double s4 = s3 * s;
        const double poly = C.c0 + C.c1 * s + C.c2 * s2 + C.c3 * s3 + C.c4 * s4;
        f[(size_t)q * I.fplane + off] = static_cast<S>(C.nF[qk(q) + 1] * poly);
    });
}

// Pressure plane, wall images and flag of half `half` from its distributions.
template <class S>
__global__ __launch_bounds__(256) void derive_kernel(const Inst *__restrict__ insts, int inst, int half) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const S *fin = static_cast<const S *>(I.f[half]);
    S f[NQ];
    const size_t off = (size_t)y * I.fpitch + x;
    static_for<0, NQ>([&](auto qc) { f[decltype(qc)::value] = fin[(size_t)decltype(qc)::value * I.fplane + off]; });
    write_pressures(I, f, x, y, I.P[half], I.PW[half]);
}

// Dirichlet ghost vectors f^eq(state) rounded to storage, and their pressures.
template <class S>
__global__ void bc_setup_kernel(Inst *insts, int inst) {
    Inst &I = insts[inst];
    const int side = threadIdx.x;
    if (side >= 4) return;
    if (I.bc[side] != BC_DIRICHLET) {
        I.bcP[side] = 0.0;
        return;
    }
    const double n = I.bcstate[side][0], ux = I.bcstate[side][1], uy = I.bcstate[side][2], T = I.bcstate[side][3];
    Coef C;
    equilibrium_coefs(I, n, ux, uy, T, C);
    S g[NQ];
    g[0] = static_cast<S>(C.nF[0] * C.c0);
    static_for<1, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double mag = qdiag(q) ? I.vs[qk(q)] : I.v[qk(q)];
        const double s = s_of<q, double>(mag, ux, uy);
        const double s2 = s * s;
        const double s3 = s2 * s;
        const double s4 = s3 * s;
        const double poly = C.c0 + C.c1 * s + C.c2 * s2 + C.c3 * s3 + C.c4 * s4;
        g[q] = static_cast<S>(C.nF[qk(q) + 1] * poly);
    });
    static_for<0, NQ>([&](auto qc) { I.bcf[side][decltype(qc)::value] = to_d(g[decltype(qc)::value]); });
    double m, jx, jy, E, vx, vy, T2, P;
    moments33<0>(I, g, m, jx, jy, E);
    primitive(m, jx, jy, E, vx, vy, T2, P);
    I.bcP[side] = P;
}

// (rho, ux, uy, T) of every cell of half `half`.
template <class S>
__global__ __launch_bounds__(256) void moments_kernel(const Inst *__restrict__ insts, int inst, int half, double *__restrict__ out) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const S *fin = static_cast<const S *>(I.f[half]);
    S f[NQ];
    const size_t off = (size_t)y * I.fpitch + x;
    static_for<0, NQ>([&](auto qc) { f[decltype(qc)::value] = fin[(size_t)decltype(qc)::value * I.fplane + off]; });
    double n, jx, jy, E, ux, uy, T, P;
    moments33<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P);
    const size_t c = (size_t)y * I.nx + x, plane = (size_t)I.nx * I.ny;
    out[c] = n;
    out[plane + c] = ux;
    out[2 * plane + c] = uy;
    out[3 * plane + c] = T;
}

// Totals of (n, jx, jy, E) per 256-cell block in a fixed tree order; the flag is OR-ed.
constexpr int kDiagBlock = 256;
template <class S>
__global__ __launch_bounds__(256) void diag_kernel(const Inst *__restrict__ insts, int inst, int half, double *__restrict__ partials) {
    const Inst &I = insts[inst];
    __shared__ double red[4][kDiagBlock];
    const long cell = (long)blockIdx.x * kDiagBlock + threadIdx.x;
    const long ncell = (long)I.nx * I.ny;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (cell < ncell) {
        const int x = (int)(cell % I.nx), y = (int)(cell / I.nx);
        const S *fin = static_cast<const S *>(I.f[half]);
        S f[NQ];
        const size_t off = (size_t)y * I.fpitch + x;
        static_for<0, NQ>([&](auto qc) { f[decltype(qc)::value] = fin[(size_t)decltype(qc)::value * I.fplane + off]; });
        moments33<0>(I, f, v[0], v[1], v[2], v[3]);
        double ux, uy, T, P;
        primitive(v[0], v[1], v[2], v[3], ux, uy, T, P);
        if (nonphysical(I, v[0], ux, uy, T)) *I.flag = 1;
    }
    for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = kDiagBlock / 2; w > 0; w /= 2) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = red[c][threadIdx.x] + red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[4 * (long)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void diag_final_kernel(const double *__restrict__ partials, int nparts, double *__restrict__ sums) {
    const int c = threadIdx.x;
    if (c >= 4) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s = s + partials[4 * (long)i + c];
    sums[c] = s;
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
template <class S, class A, bool FUSE, int SHAPE>
static hipError_t launch_step_t(const Inst *insts, const Tile *tiles, int ntiles, int half, hipStream_t s) {
    constexpr int TX = kTileShapes[SHAPE].tx, TY = kTileShapes[SHAPE].ty;
    hipLaunchKernelGGL((step_kernel<S, A, FUSE, TX, TY>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles, ntiles,
                       half);
    return hipGetLastError();
}

template <class S, class A, bool FUSE>
static hipError_t launch_step_p(int shape, const Inst *insts, const Tile *tiles, int ntiles, int half,
                                hipStream_t s) {
    switch (shape) {
    case 0: return launch_step_t<S, A, FUSE, 0>(insts, tiles, ntiles, half, s);
    case 1: return launch_step_t<S, A, FUSE, 1>(insts, tiles, ntiles, half, s);
    case 2: return launch_step_t<S, A, FUSE, 2>(insts, tiles, ntiles, half, s);
    case 3: return launch_step_t<S, A, FUSE, 3>(insts, tiles, ntiles, half, s);
    case 4: return launch_step_t<S, A, FUSE, 4>(insts, tiles, ntiles, half, s);
    case 5: return launch_step_t<S, A, FUSE, 5>(insts, tiles, ntiles, half, s);
    case 6: return launch_step_t<S, A, FUSE, 6>(insts, tiles, ntiles, half, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(int prec, int shape, const Inst *insts, const Tile *tiles, int ntiles, int half,
                       hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (prec == PREC_F64) return launch_step_p<double, double, false>(shape, insts, tiles, ntiles, half, s);
    return launch_step_p<float, float, true>(shape, insts, tiles, ntiles, half, s);
}

static dim3 grid16(int nx, int ny) { return dim3((nx + 15) / 16, (ny + 15) / 16); }

hipError_t launch_fill(int prec, const Inst *insts, int inst, int nx, int ny, const double *fields, int half,
                       hipStream_t s) {
    if (prec == PREC_F64)
        hipLaunchKernelGGL(fill_kernel<double>, grid16(nx, ny), dim3(256), 0, s, insts, inst, fields, half);
    else
        hipLaunchKernelGGL(fill_kernel<float>, grid16(nx, ny), dim3(256), 0, s, insts, inst, fields, half);
    return hipGetLastError();
}

hipError_t launch_derive(int prec, const Inst *insts, int inst, int nx, int ny, int half, hipStream_t s) {
    if (prec == PREC_F64)
        hipLaunchKernelGGL(derive_kernel<double>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half);
    else
        hipLaunchKernelGGL(derive_kernel<float>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half);
    return hipGetLastError();
}

hipError_t launch_bc_setup(int prec, Inst *insts, int inst, hipStream_t s) {
    if (prec == PREC_F64)
        hipLaunchKernelGGL(bc_setup_kernel<double>, dim3(1), dim3(64), 0, s, insts, inst);
    else
        hipLaunchKernelGGL(bc_setup_kernel<float>, dim3(1), dim3(64), 0, s, insts, inst);
    return hipGetLastError();
}

hipError_t launch_moments(int prec, const Inst *insts, int inst, int nx, int ny, int half, double *out,
                          hipStream_t s) {
    if (prec == PREC_F64)
        hipLaunchKernelGGL(moments_kernel<double>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half, out);
    else
        hipLaunchKernelGGL(moments_kernel<float>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half, out);
    return hipGetLastError();
}

int diag_blocks(int nx, int ny) { return (int)(((long)nx * ny + kDiagBlock - 1) / kDiagBlock); }

hipError_t launch_diag(int prec, const Inst *insts, int inst, int nx, int ny, int half, double *partials,
                       int npart_offset, hipStream_t s) {
    const int nb = diag_blocks(nx, ny);
    double *p = partials + 4 * (long)npart_offset;
    if (prec == PREC_F64)
        hipLaunchKernelGGL(diag_kernel<double>, dim3(nb), dim3(kDiagBlock), 0, s, insts, inst, half, p);
    else
        hipLaunchKernelGGL(diag_kernel<float>, dim3(nb), dim3(kDiagBlock), 0, s, insts, inst, half, p);
    return hipGetLastError();
}

hipError_t launch_diag_final(const double *partials, int nparts, double *sums, hipStream_t s) {
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, partials, nparts, sums);
    return hipGetLastError();
}

}  // namespace fdlb
