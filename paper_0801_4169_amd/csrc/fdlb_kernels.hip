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
// Work decomposition: one workgroup per TX x TY tile, one thread per cell.  Neighbours
// come from an LDS copy of a pair of velocity planes of the tile plus a two-cell halo
// (double buffered, one barrier per stage), and the planes of the next stages are in
// flight while the current one computes.  Three bodies:
//   step_body        (float32; float64 with FDLB_STREAM_EDGE=0 on edge tiles): the cell's
//                    33 values in registers, moments recomputed from them;
//   step_body_stream (float64): the moments stored by the previous step start the
//                    equilibrium at once, the planes stream through the stages, and the
//                    new moments are summed as the new values appear;
//   step_body_dev    (deviation storage): f rebuilt in float64 from float32 deviations.
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

// Line-IV coefficient theta |kappa| (1 - |kappa|) / 2, Eqs. (add3), (add4).  theta =
// lam |dP / sum P| + th0: th0 = 0 with the switching function (the fused multiply-add rounds
// the product once, so the value is that of the plain product), lam = 0 and th0 = the frozen
// value when theta is frozen (Sec. 4).
__device__ __forceinline__ double av_coeff(double lam, double th0, double Pm, double P0, double Pp, double u,
                                           double dt, double dr) {
    const double th = __builtin_fma(lam, fabs((Pp - 2.0 * P0 + Pm) / (Pp + 2.0 * P0 + Pm)), th0);
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

// ------------------------------------------------------------------------------------
// Moments with float64 accumulation and fused multiply-adds (any order is fine for the
// float32 and deviation paths; the float64 path uses moments33 above).
// ------------------------------------------------------------------------------------
template <int MIR, class S>
__device__ __forceinline__ void moments33_fast(const Inst &I, const S (&f)[NQ], double &n, double &jx,
                                               double &jy, double &E) {
    n = 0.0;
    jx = 0.0;
    jy = 0.0;
    E = 0.0;
    static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int src = MIR == 0 ? q : MIR == 1 ? qmx(q) : qmy(q);
        const double fq = static_cast<double>(f[src]);
        n += fq;
        if constexpr (q > 0) {
            constexpr int k = qk(q);
            const double mag = qdiag(q) ? I.vs[k] : I.v[k];
            if constexpr (qsx(q) > 0) jx = __builtin_fma(mag, fq, jx);
            if constexpr (qsx(q) < 0) jx = __builtin_fma(-mag, fq, jx);
            if constexpr (qsy(q) > 0) jy = __builtin_fma(mag, fq, jy);
            if constexpr (qsy(q) < 0) jy = __builtin_fma(-mag, fq, jy);
            E = __builtin_fma(qdiag(q) ? I.edg[k] : I.eax[k], fq, E);
        }
    });
}

template <int MIR, class S>
__device__ __forceinline__ void moments_of(const Inst &I, const S (&f)[NQ], double &n, double &jx, double &jy,
                                           double &E) {
    if constexpr (std::is_same<S, double>::value)
        moments33<MIR>(I, f, n, jx, jy, E);
    else
        moments33_fast<MIR>(I, f, n, jx, jy, E);
}

// ------------------------------------------------------------------------------------
// Float64 per-velocity update: Eq. (dis_eq1) in the fixed order (no contraction).
// ------------------------------------------------------------------------------------
struct CellD {
    double c0, c1, c2, c3, c4;
    double nF[5];
    double ux, uy, ax, ay;
};

// One direction alpha: lines I, II, III, IV added one by one.  SGN is the sign of the
// velocity component; for a zero component the coefficients of lines I-III are zero and
// only line IV remains.
template <int SGN>
__device__ __forceinline__ double lines_alpha(double fn, double f0, double fm2, double fm1, double fp1, double fp2,
                                              double k1, double k2, double k3, double av) {
    const double d2 = fp1 - 2.0 * f0 + fm1;
    if constexpr (SGN != 0) {
        const double d1 = fp1 - fm1;
        const double d3 = fp2 - 2.0 * fp1 + 2.0 * fm1 - fm2;
        const double t1 = k1 * d1;
        fn = SGN > 0 ? fn - t1 : fn + t1;  // line I
        const double t2 = k2 * d2;
        fn = fn + t2;  // line II
        const double t3 = k3 * d3;
        fn = SGN > 0 ? fn + t3 : fn - t3;  // line III
    }
    const double t4 = av * d2;
    return fn + t4;  // line IV
}

template <int Q>
__device__ __forceinline__ double update_f64(const Inst &I, const CellD &c, double f0, double feq, double xm2,
                                             double xm1, double xp1, double xp2, double ym2, double ym1, double yp1,
                                             double yp2) {
    constexpr int k = qk(Q), dg = qdiag(Q) ? 1 : 0;
    double fn = f0;
    if constexpr (qsx(Q) != 0)
        fn = lines_alpha<qsx(Q)>(fn, f0, xm2, xm1, xp1, xp2, I.k1[0][dg][k], I.k2[0][dg][k], I.k3[0][dg][k], c.ax);
    else
        fn = lines_alpha<0>(fn, f0, xm2, xm1, xp1, xp2, 0.0, 0.0, 0.0, c.ax);
    if constexpr (qsy(Q) != 0)
        fn = lines_alpha<qsy(Q)>(fn, f0, ym2, ym1, yp1, yp2, I.k1[1][dg][k], I.k2[1][dg][k], I.k3[1][dg][k], c.ay);
    else
        fn = lines_alpha<0>(fn, f0, ym2, ym1, yp1, yp2, 0.0, 0.0, 0.0, c.ay);
    const double t = I.dtau * (f0 - feq);  // BGK
    return fn - t;
}

// Equilibrium of the opposite pair (q, q + 4): the powers of s = v . u are shared, the odd
// ones change sign.  Same order as the plain evaluation c0 + c1 s + c2 s^2 + c3 s^3 + c4 s^4.
template <int QA>
__device__ __forceinline__ void feq_pair_f64(const Inst &I, const CellD &c, double &fa, double &fb) {
    constexpr int k = qk(QA);
    const double mag = qdiag(QA) ? I.vs[k] : I.v[k];
    const double s = s_of<QA, double>(mag, c.ux, c.uy);
    const double s2 = s * s;
    const double s3 = s2 * s;
    const double s4 = s3 * s;
    const double t1 = c.c1 * s, t2 = c.c2 * s2, t3 = c.c3 * s3, t4 = c.c4 * s4;
    fa = c.nF[k + 1] * (c.c0 + t1 + t2 + t3 + t4);
    fb = c.nF[k + 1] * (c.c0 - t1 + t2 - t3 + t4);
}

// ------------------------------------------------------------------------------------
// Float32 per-velocity update.  The same scheme, restated as weights on the five points of
// each direction (line IV folded into line II), with fused multiply-adds:
//   coefficient of f(+1) = K - (k1 + 2 k3), of f(-1) = K + (k1 + 2 k3), of f(+-2) = +-k3,
//   of f(0) = 1 - dt/tau - 2 K_x - 2 K_y, with K = c^2/2 + theta |kappa| (1 - |kappa|)/2,
// for a positive velocity component (the signs of k1, k3 flip with it).
// ------------------------------------------------------------------------------------
struct CellF {
    float c0, c1, c2, c3, c4;
    float nF[5];
    float ux, uy, pA, pB;  // pA = ux + uy, pB = uy - ux
    float ax, ay, omd, dtau;
};

template <int Q>
__device__ __forceinline__ float update_f32(const Inst &I, const CellF &c, float f0, float feq, float xm2,
                                            float xm1, float xp1, float xp2, float ym2, float ym1, float yp1,
                                            float yp2) {
    constexpr int k = qk(Q), dg = qdiag(Q) ? 1 : 0, sx = qsx(Q), sy = qsy(Q);
    float Kx = c.ax, Ky = c.ay;
    if constexpr (sx != 0) Kx = I.kf[1][0][dg][k] + c.ax;
    if constexpr (sy != 0) Ky = I.kf[1][1][dg][k] + c.ay;
    float fn = (c.omd - 2.0f * (Kx + Ky)) * f0;
    fn = __builtin_fmaf(c.dtau, feq, fn);
    if constexpr (sx != 0) {
        const float kk = I.kkf[0][dg][k], k3 = I.kf[2][0][dg][k];
        fn = __builtin_fmaf(sx > 0 ? Kx - kk : Kx + kk, xp1, fn);
        fn = __builtin_fmaf(sx > 0 ? Kx + kk : Kx - kk, xm1, fn);
        fn = __builtin_fmaf(sx > 0 ? k3 : -k3, xp2 - xm2, fn);
    } else {
        fn = __builtin_fmaf(Kx, xp1 + xm1, fn);
    }
    if constexpr (sy != 0) {
        const float kk = I.kkf[1][dg][k], k3 = I.kf[2][1][dg][k];
        fn = __builtin_fmaf(sy > 0 ? Ky - kk : Ky + kk, yp1, fn);
        fn = __builtin_fmaf(sy > 0 ? Ky + kk : Ky - kk, ym1, fn);
        fn = __builtin_fmaf(sy > 0 ? k3 : -k3, yp2 - ym2, fn);
    } else {
        fn = __builtin_fmaf(Ky, yp1 + ym1, fn);
    }
    return fn;
}

template <int QA>
__device__ __forceinline__ void feq_pair_f32(const Inst &I, const CellF &c, float &fa, float &fb) {
    constexpr int i = qi(QA), k = qk(QA);
    float s;
    if constexpr (i == 1) s = I.vsf[k] * c.pA;
    else if constexpr (i == 2) s = I.vf[k] * c.uy;
    else if constexpr (i == 3) s = I.vsf[k] * c.pB;
    else s = -(I.vf[k] * c.ux);
    const float s2 = s * s;
    const float ev = __builtin_fmaf(__builtin_fmaf(c.c4, s2, c.c2), s2, c.c0);
    const float od = s * __builtin_fmaf(c.c3, s2, c.c1);
    fa = c.nF[k + 1] * (ev + od);
    fb = c.nF[k + 1] * (ev - od);
}

template <class S>
struct CellOf;
template <>
struct CellOf<double> { using type = CellD; };
template <>
struct CellOf<float> { using type = CellF; };

template <int Q, class S, class C>
__device__ __forceinline__ S update_q(const Inst &I, const C &c, S f0, S feq, S xm2, S xm1, S xp1, S xp2, S ym2,
                                      S ym1, S yp1, S yp2) {
    if constexpr (std::is_same<S, double>::value)
        return update_f64<Q>(I, c, f0, feq, xm2, xm1, xp1, xp2, ym2, ym1, yp1, yp2);
    else
        return update_f32<Q>(I, c, f0, feq, xm2, xm1, xp1, xp2, ym2, ym1, yp1, yp2);
}

template <int QA, class S, class C>
__device__ __forceinline__ void feq_pair(const Inst &I, const C &c, S &fa, S &fb) {
    if constexpr (std::is_same<S, double>::value)
        feq_pair_f64<QA>(I, c, fa, fb);
    else
        feq_pair_f32<QA>(I, c, fa, fb);
}

__device__ __forceinline__ void make_cell(const Coef &C, double ux, double uy, double ax, double ay, double dtau,
                                          CellD &c) {
    c.c0 = C.c0;
    c.c1 = C.c1;
    c.c2 = C.c2;
    c.c3 = C.c3;
    c.c4 = C.c4;
#pragma unroll
    for (int k = 0; k < 5; ++k) c.nF[k] = C.nF[k];
    c.ux = ux;
    c.uy = uy;
    c.ax = ax;
    c.ay = ay;
    (void)dtau;
}

__device__ __forceinline__ void make_cell(const Coef &C, double ux, double uy, double ax, double ay, double dtau,
                                          CellF &c) {
    c.c0 = (float)C.c0;
    c.c1 = (float)C.c1;
    c.c2 = (float)C.c2;
    c.c3 = (float)C.c3;
    c.c4 = (float)C.c4;
#pragma unroll
    for (int k = 0; k < 5; ++k) c.nF[k] = (float)C.nF[k];
    c.ux = (float)ux;
    c.uy = (float)uy;
    c.pA = (float)(ux + uy);
    c.pB = (float)(uy - ux);
    c.ax = (float)ax;
    c.ay = (float)ay;
    c.omd = (float)(1.0 - dtau);
    c.dtau = (float)dtau;
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

// Condition of side `side` at position i along it (row on the x sides, column on the y
// sides) at time t: the side's own or its lower segment's; `slot` receives the Dirichlet
// slot (4..7 for a lower segment).  Same expressions as the oracle, so the choice is the
// same bit for bit.
__device__ __forceinline__ int side_kind(const Inst &I, int side, int i, double t, int &slot) {
    slot = side;
    if (I.bclo[side] != BC_PERIODIC) {
        const double d = side < 2 ? I.dy : I.dx;
        const double c = ((double)i + 0.5) * d;
        const double sp = I.split0[side] + I.split1[side] * t;
        if (c < sp) {
            slot = 4 + side;
            return I.bclo[side];
        }
    }
    return I.bc[side];
}

// Time of the current step for the moving side segments.
__device__ __forceinline__ double step_time(const Inst &I) { return (double)(*I.clock) * I.dt; }

__device__ __forceinline__ Src map_cell(const Inst &I, int x, int y, double t) {
    Src s{0, 0, -1};
    const int nx = I.nx, ny = I.ny;
    if ((unsigned)x >= (unsigned)nx) {
        const int side = x < 0 ? 0 : 1;
        int slot;
        const int kind = side_kind(I, side, y, t, slot);
        if (kind == BC_DIRICHLET) {
            s.dside = slot;
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
        int slot;
        const int kind = side_kind(I, side, x, t, slot);
        if (kind == BC_DIRICHLET) {
            if (s.dside < 0) s.dside = slot;
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

// Pressure of the neighbour (x, y) (at most one cell outside the grid) at time t.
__device__ __forceinline__ double load_P(const Inst &I, const double *__restrict__ P,
                                         const double *__restrict__ PW, int x, int y, double t) {
    const int nx = I.nx, ny = I.ny;
    if ((unsigned)x >= (unsigned)nx) {
        const int side = x < 0 ? 0 : 1;
        const int yc = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        int slot;
        const int kind = side_kind(I, side, yc, t, slot);
        if (kind == BC_DIRICHLET) return I.bcP[slot];
        if (kind == BC_WALL) return PW[side * I.wlen + yc];
        x = kind == BC_PERIODIC ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
    }
    if ((unsigned)y >= (unsigned)ny) {
        const int side = y < 0 ? 2 : 3;
        const int xc = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
        int slot;
        const int kind = side_kind(I, side, xc, t, slot);
        if (kind == BC_DIRICHLET) return I.bcP[slot];
        if (kind == BC_WALL) return PW[side * I.wlen + xc];
        y = kind == BC_PERIODIC ? ((y % ny) + ny) % ny : (y < 0 ? 0 : ny - 1);
    }
    x = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    return P[y * I.ppitch + x];
}

// As load_P, with the pressure of a cell inside the grid taken as n T of its stored
// moments (the same product the step that stored them formed).
__device__ __forceinline__ double load_P_m(const Inst &I, const double *__restrict__ M,
                                           const double *__restrict__ PW, int x, int y, double t) {
    const int nx = I.nx, ny = I.ny;
    if ((unsigned)x >= (unsigned)nx) {
        const int side = x < 0 ? 0 : 1;
        const int yc = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        int slot;
        const int kind = side_kind(I, side, yc, t, slot);
        if (kind == BC_DIRICHLET) return I.bcP[slot];
        if (kind == BC_WALL) return PW[side * I.wlen + yc];
        x = kind == BC_PERIODIC ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
    }
    if ((unsigned)y >= (unsigned)ny) {
        const int side = y < 0 ? 2 : 3;
        const int xc = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
        int slot;
        const int kind = side_kind(I, side, xc, t, slot);
        if (kind == BC_DIRICHLET) return I.bcP[slot];
        if (kind == BC_WALL) return PW[side * I.wlen + xc];
        y = kind == BC_PERIODIC ? ((y % ny) + ny) % ny : (y < 0 ? 0 : ny - 1);
    }
    x = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
    y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
    const size_t c = (size_t)y * I.ppitch + x;
    return M[c] * M[3 * (size_t)I.mplane + c];
}

// XCD-aware order: consecutive workgroup ids go round-robin over the 8 XCDs; give each XCD
// a contiguous run of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, local = b / 8;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <class S>
constexpr bool stream_moments();
template <class S>
constexpr bool stream_edge();

// Moments and pressure of the cell (from its final 33 values) and the pressure of the
// mirror images next to reflecting sides.  Returns 1 if the cell's state is non-physical.
template <class S>
__device__ __forceinline__ int write_pressures(const Inst &I, const S (&f)[NQ], int x, int y,
                                               double *__restrict__ Pout, double *__restrict__ Mout,
                                               double *__restrict__ PWout) {
    double n, jx, jy, E, ux, uy, T, P;
    moments_of<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P);
    Pout[y * I.ppitch + x] = P;
    if (stream_moments<S>()) {
        Mout[y * I.ppitch + x] = n;
        Mout[I.mplane + y * I.ppitch + x] = ux;
        Mout[2 * I.mplane + y * I.ppitch + x] = uy;
        Mout[3 * I.mplane + y * I.ppitch + x] = T;
    }
    const int bad = nonphysical(I, n, ux, uy, T) ? 1 : 0;
    // a wall on the side or on its lower segment: the mirror image's pressure
    auto wall = [&](int side) { return I.bc[side] == BC_WALL || I.bclo[side] == BC_WALL; };
    if ((x == 0 && wall(0)) || (x == I.nx - 1 && wall(1))) {
        moments_of<1>(I, f, n, jx, jy, E);
        primitive(n, jx, jy, E, ux, uy, T, P);
        if (x == 0 && wall(0)) PWout[0 * I.wlen + y] = P;
        if (x == I.nx - 1 && wall(1)) PWout[1 * I.wlen + y] = P;
    }
    if ((y == 0 && wall(2)) || (y == I.ny - 1 && wall(3))) {
        moments_of<2>(I, f, n, jx, jy, E);
        primitive(n, jx, jy, E, ux, uy, T, P);
        if (y == 0 && wall(2)) PWout[2 * I.wlen + x] = P;
        if (y == I.ny - 1 && wall(3)) PWout[3 * I.wlen + x] = P;
    }
    return bad;
}

// ------------------------------------------------------------------------------------
// The fused step kernel.
//
// Tiles come in three kinds, each compiled as its own specialised body:
//   INTERIOR: the tile and its two-cell halo lie inside the grid -- no boundary logic,
//             every address is a per-plane base (scalar) plus a 32-bit offset;
//   TUBE:     as INTERIOR along x, and the tile spans the whole periodic height of the grid
//             (ny == TY): the y halo is the tile's own rows, written into LDS twice;
//   EDGE:     everything else; halo cells are mapped through the side conditions.
// ------------------------------------------------------------------------------------
constexpr int MODE_INTERIOR = 0, MODE_TUBE = 1, MODE_EDGE = 2;

// Optimisation barrier for a uniform integer: after it the compiler cannot reuse values it
// derived from `v` earlier, so per-stage plane offsets and constant loads happen inside each
// stage instead of all being hoisted to the kernel entry (where they would not fit in the
// scalar register file).  Emits no instruction.  Used on integers only: pointers keep the
// global address space the compiler inferred for them.
template <class T>
__device__ __forceinline__ T opaque(T v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Distribution memory is addressed through explicit global (address space 1) pointers so
// every access is a global_load / global_store with a scalar base and 32-bit offset.
#define GLOBAL_AS __attribute__((address_space(1)))

#ifndef FDLB_NT_STORE
#define FDLB_NT_STORE 1  // new distributions are written with non-temporal stores (they are
                         // not read again in the step; keeping them out of L2 leaves room for
                         // the halo rows neighbouring tiles re-read)
#endif

// Store of a new distribution value (never read again within the step).
template <class T>
__device__ __forceinline__ void store_out(GLOBAL_AS T *p, T v) {
#if FDLB_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

template <int Q, int MODE, class S>
__device__ __forceinline__ S fetch(const Inst &I, const GLOBAL_AS char *fin, size_t pb, const Src &s) {
    if constexpr (MODE != MODE_EDGE) {
        return *reinterpret_cast<const GLOBAL_AS S *>(fin + (size_t)Q * pb + (uint32_t)s.off);
    } else {
        if (s.dside >= 0) return static_cast<S>(I.bcf[s.dside][Q]);
        const int qq = s.flip == 0 ? Q : s.flip == 1 ? qmx(Q) : s.flip == 2 ? qmy(Q) : qmx(qmy(Q));
        return reinterpret_cast<const GLOBAL_AS S *>(fin)[(size_t)qq * I.fplane + s.off];
    }
}

#ifndef FDLB_HALO_DMA
#define FDLB_HALO_DMA 1  // float32 interior body: halo of all planes loaded at once, into LDS
#endif
#define LDS_AS __attribute__((address_space(3)))

// The float32 interior body with one halo cell per thread loads the halo cells of all 33
// planes when it loads its own cells, straight into LDS (global_load_lds: no registers), so
// a plane's halo lines are read while the neighbouring tiles read the same lines as their
// own and are still in L2.  Loaded one stage ahead instead, a halo line is read a whole
// workgroup lifetime after its owner read it, and mostly comes from HBM a second time.
template <class S, int TX, int TY, int MODE>
constexpr bool halo_dma() {
    return FDLB_HALO_DMA != 0 && std::is_same<S, float>::value && MODE == MODE_INTERIOR &&
           4 * (TX + TY) <= TX * TY;
}
#ifndef FDLB_HALO_DMA_PACKED
#define FDLB_HALO_DMA_PACKED 1  // one slot per halo cell (else whole wavefronts per plane)
#endif
// A load into LDS writes the slots of the active lanes only, so the planes' halo rows can
// follow each other at the halo's own length (160 cells for a 32 x 8 tile, where the third
// wavefront has 32 active lanes).  That keeps a 32 x 8 workgroup at 28 416 bytes of LDS, and
// five of them share a CU (measured: 4.7 resident waves per SIMD); at whole wavefronts (32 512
// bytes, allocated as 32 768) only four did (3.8 waves per SIMD), and the kernel was 1.5% slower.
// 64 spare slots at the end keep every slot a wavefront could address inside the array.
template <int TX, int TY>
constexpr int halo_dma_width() {
    return FDLB_HALO_DMA_PACKED ? 4 * (TX + TY) : (4 * (TX + TY) + 63) / 64 * 64;
}
template <int TX, int TY>
constexpr int halo_dma_size() {
    return NQ * halo_dma_width<TX, TY>() + (FDLB_HALO_DMA_PACKED ? 64 : 0);
}

template <class S, int TX, int TY, int MODE>
__device__ __forceinline__ void step_body(const Inst *__restrict__ insts, const Tile &tile, int io,
                                          StepSmem<S, TX, TY> &sm, S *hdma) {
    const int bin = io_in(io), bout = io_out(io);
    const Inst &I = insts[tile.inst];
    constexpr int NT = TX * TY;
    constexpr int H0 = MODE == MODE_TUBE ? 4 * TX : 0;  // the tube body loads only the x halo
    constexpr int NHALL = 4 * (TX + TY);
    constexpr int NSLOT = (NHALL - H0 + NT - 1) / NT;
    constexpr int LW = TX + 4;
    using Cell = typename CellOf<S>::type;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = tile.x0 + tx, y = tile.y0 + ty;
    const int nx = I.nx, ny = I.ny;
    const bool valid = MODE != MODE_EDGE || (x < nx && y < ny);
    const GLOBAL_AS char *fin = (const GLOBAL_AS char *)(I.f[bin]);
    GLOBAL_AS char *fout = (GLOBAL_AS char *)(I.f[bout]);
    const size_t pb = (size_t)I.fplane * sizeof(S);
    const double *__restrict__ Pin = I.P[bin];
    double *__restrict__ Pout = I.P[bout];

    // offsets: bytes for INTERIOR / TUBE, elements (with mapping) for EDGE
    Src own;
    double tnow = 0.0;
    if constexpr (MODE != MODE_EDGE) own = Src{(int)((y * I.fpitch + x) * (int)sizeof(S)), 0, -1};
    else {
        tnow = step_time(I);
        own = map_cell(I, x, y, tnow);
    }
    Src hs[NSLOT];
    int hl[NSLOT];
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const int hid = tid + j * NT + H0;
        hl[j] = -1;
        hs[j] = Src{0, 0, -1};
        if (hid < NHALL) {
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
            hl[j] = ly * LW + lx;
            const int X = tile.x0 + lx - 2, Y = tile.y0 + ly - 2;
            if constexpr (MODE != MODE_EDGE) hs[j] = Src{(int)((Y * I.fpitch + X) * (int)sizeof(S)), 0, -1};
            else hs[j] = map_cell(I, X, Y, tnow);
        }
    }

    // A1: own distributions.  With halo_dma the halo cells of plane q go to LDS beside the
    // own load of plane q (thread tid's halo cell lands in hdma[q * HW + tid]); otherwise the
    // first halo stage is in flight during the moments and each stage prefetches the next.
    constexpr bool HALL = halo_dma<S, TX, TY, MODE>();
    constexpr int HW = halo_dma_width<TX, TY>();
    static_assert(!HALL || (NSLOT == 1 && H0 == 0), "one halo cell per thread, indexed by tid");
    S f[NQ];
    const int wbase = __builtin_amdgcn_readfirstlane(tid >> 6) << 6;
    static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        f[q] = fetch<q, MODE, S>(I, fin, pb, own);
        if constexpr (HALL)
            if (hl[0] >= 0)
                __builtin_amdgcn_global_load_lds(
                    (const GLOBAL_AS void *)(fin + (size_t)q * pb + (uint32_t)hs[0].off),
                    (LDS_AS void *)(hdma + q * HW + wbase), 4, 0, 0);  // float only
    });
    S h0[NSLOT], h1[NSLOT];
    if constexpr (!HALL) {
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) h0[j] = fetch<0, MODE, S>(I, fin, pb, hs[j]);
    }

    // A2: moments
    double n, jx, jy, E, ux, uy, T, P0;
    moments_of<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P0);

    // A3: switching function and line-IV coefficients from the neighbours' pressure
    double Pxm, Pxp, Pym, Pyp;
    if constexpr (MODE == MODE_INTERIOR) {
        const GLOBAL_AS double *pc = (const GLOBAL_AS double *)Pin + (y * I.ppitch + x);
        Pxm = pc[-1];
        Pxp = pc[1];
        Pym = pc[-I.ppitch];
        Pyp = pc[I.ppitch];
    } else if constexpr (MODE == MODE_TUBE) {
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        Pxm = Pin[y * I.ppitch + x - 1];
        Pxp = Pin[y * I.ppitch + x + 1];
        Pym = Pin[ym * I.ppitch + x];
        Pyp = Pin[yp * I.ppitch + x];
    } else {
        const double *PWin = I.PW[bin];
        Pxm = load_P(I, Pin, PWin, x - 1, y, tnow);
        Pxp = load_P(I, Pin, PWin, x + 1, y, tnow);
        Pym = load_P(I, Pin, PWin, x, y - 1, tnow);
        Pyp = load_P(I, Pin, PWin, x, y + 1, tnow);
    }
    const double ax = av_coeff(I.lam, I.th0, Pxm, P0, Pxp, ux, I.dt, I.dx);
    const double ay = av_coeff(I.lam, I.th0, Pym, P0, Pyp, uy, I.dt, I.dy);

    // A4: equilibrium coefficients
    Coef C;
    equilibrium_coefs(I, n, ux, uy, T, C);
    Cell cell;
    make_cell(C, ux, uy, ax, ay, I.dtau, cell);

    const int own_l = (ty + 2) * LW + (tx + 2);
    const uint32_t own_b = MODE != MODE_EDGE ? (uint32_t)own.off : (uint32_t)((y * I.fpitch + x) * (int)sizeof(S));
    int b = 0;

    auto put = [&](S *pl, S v) {
        pl[own_l] = v;
        if constexpr (MODE == MODE_TUBE) {
            if (ty >= TY - 2) pl[own_l - TY * LW] = v;  // y = -2, -1 are rows ny - 2, ny - 1
            if (ty < 2) pl[own_l + TY * LW] = v;        // y = ny, ny + 1 are rows 0, 1
        }
    };
    // A5: one velocity from the LDS plane `pl`; A6: store it
    auto compute = [&](auto qc, const Inst &Is, GLOBAL_AS char *fo, size_t pbs, const S *pl, S feq) {
        constexpr int q = decltype(qc)::value;
        const S out = update_q<q, S>(Is, cell, f[q], feq, pl[own_l - 2], pl[own_l - 1], pl[own_l + 1],
                                     pl[own_l + 2], pl[own_l - 2 * LW], pl[own_l - LW], pl[own_l + LW],
                                     pl[own_l + 2 * LW]);
        if (valid) store_out(reinterpret_cast<GLOBAL_AS S *>(fo + (size_t)q * pbs + own_b), out);
        f[q] = out;
    };

    // stage 0: rest particle
    {
        const Inst &Is = insts[opaque(tile.inst)];
        const GLOBAL_AS char *fi = fin;
        GLOBAL_AS char *fo = fout;
        const size_t pbs = opaque(pb);
        S *pl = &sm.buf[b][0][0][0];
        put(pl, f[0]);
        if constexpr (HALL) {
            // the compiler does not order LDS reads after loads into LDS: wait for this
            // wave's loads (each wave reads back only the slots its own lanes loaded)
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (hl[0] >= 0) pl[hl[0]] = hdma[tid];
        } else {
#pragma unroll
            for (int j = 0; j < NSLOT; ++j)
                if (hl[j] >= 0) pl[hl[j]] = h0[j];
        }
        __syncthreads();
        if constexpr (!HALL) {
#pragma unroll
            for (int j = 0; j < NSLOT; ++j)
                if (hl[j] >= 0) {
                    h0[j] = fetch<1, MODE, S>(Is, fi, pbs, hs[j]);
                    h1[j] = fetch<5, MODE, S>(Is, fi, pbs, hs[j]);
                }
        }
        compute(std::integral_constant<int, 0>{}, Is, fo, pbs, pl, static_cast<S>(cell.nF[0] * cell.c0));
        b ^= 1;
    }
    // stages 1..16: opposite pairs q = 1 + 8k + j and q + 4
    static_for<0, 16>([&](auto sc) {
        constexpr int st = decltype(sc)::value;
        constexpr int qa = 1 + 8 * (st / 4) + (st % 4);
        constexpr int qb = qa + 4;
        const Inst &Is = insts[opaque(tile.inst)];
        const GLOBAL_AS char *fi = fin;
        GLOBAL_AS char *fo = fout;
        const size_t pbs = opaque(pb);
        S *pa = &sm.buf[b][0][0][0];
        S *pbuf = &sm.buf[b][1][0][0];
        put(pa, f[qa]);
        put(pbuf, f[qb]);
        if constexpr (HALL) {
            if (hl[0] >= 0) {
                pa[hl[0]] = hdma[qa * HW + tid];
                pbuf[hl[0]] = hdma[qb * HW + tid];
            }
        } else {
#pragma unroll
            for (int j = 0; j < NSLOT; ++j)
                if (hl[j] >= 0) {
                    pa[hl[j]] = h0[j];
                    pbuf[hl[j]] = h1[j];
                }
        }
        __syncthreads();
        if constexpr (!HALL && st + 1 < 16) {
            constexpr int na = 1 + 8 * ((st + 1) / 4) + ((st + 1) % 4);
#pragma unroll
            for (int j = 0; j < NSLOT; ++j)
                if (hl[j] >= 0) {
                    h0[j] = fetch<na, MODE, S>(Is, fi, pbs, hs[j]);
                    h1[j] = fetch<na + 4, MODE, S>(Is, fi, pbs, hs[j]);
                }
        }
        S fa, fb;
        feq_pair<qa, S>(Is, cell, fa, fb);
        compute(std::integral_constant<int, qa>{}, Is, fo, pbs, pa, fa);
        compute(std::integral_constant<int, qb>{}, Is, fo, pbs, pbuf, fb);
        b ^= 1;
    });

    // A6: pressure for the next step's switching function, wall images, flag (one store
    // per workgroup)
    int bad = 0;
    if constexpr (MODE == MODE_EDGE) {
        if (valid) bad = write_pressures(I, f, x, y, Pout, I.M[bout], I.PW[bout]);
    } else {
        double n2, jx2, jy2, E2, ux2, uy2, T2, P2;
        moments_of<0>(I, f, n2, jx2, jy2, E2);
        primitive(n2, jx2, jy2, E2, ux2, uy2, T2, P2);
        ((GLOBAL_AS double *)Pout)[y * I.ppitch + x] = P2;
        bad = nonphysical(I, n2, ux2, uy2, T2) ? 1 : 0;
    }
    if (__syncthreads_or(bad) && tid == 0) *I.flag = 1;
}

// ------------------------------------------------------------------------------------
// Stages: stage 0 is the rest particle; stage 1 + 4k + j holds the opposite pair
// q = 1 + 8k + j and q + 4 (they share the powers of s in f^eq).
// ------------------------------------------------------------------------------------
constexpr int NSTAGE = 17;
__host__ __device__ constexpr int stage_qa(int st) { return st == 0 ? 0 : 1 + 8 * ((st - 1) / 4) + ((st - 1) % 4); }
__host__ __device__ constexpr int stage_qb(int st) { return st == 0 ? -1 : stage_qa(st) + 4; }

// One term of the moments of Eqs. (n_eq), (nu_eq) and the energy, added to the running sums.
// Float64: the same operation as one iteration of moments33 (so feeding the terms in
// ascending q reproduces it exactly); float32 path: fused, any order.
template <int Q, class S>
__device__ __forceinline__ void acc_term(const Inst &I, S v, double &n, double &jx, double &jy, double &E) {
    const double fq = static_cast<double>(v);
    constexpr int k = qk(Q);
    if constexpr (std::is_same<S, double>::value) {
        n = n + fq;
        if constexpr (Q > 0) {
            const double mag = qdiag(Q) ? I.vs[k] : I.v[k];
            if constexpr (qsx(Q) > 0) jx = jx + mag * fq;
            if constexpr (qsx(Q) < 0) jx = jx - mag * fq;
            if constexpr (qsy(Q) > 0) jy = jy + mag * fq;
            if constexpr (qsy(Q) < 0) jy = jy - mag * fq;
            const double e = qdiag(Q) ? I.edg[k] : I.eax[k];
            E = E + e * fq;
        }
    } else {
        n += fq;
        if constexpr (Q > 0) {
            const double mag = qdiag(Q) ? I.vs[k] : I.v[k];
            if constexpr (qsx(Q) > 0) jx = __builtin_fma(mag, fq, jx);
            if constexpr (qsx(Q) < 0) jx = __builtin_fma(-mag, fq, jx);
            if constexpr (qsy(Q) > 0) jy = __builtin_fma(mag, fq, jy);
            if constexpr (qsy(Q) < 0) jy = __builtin_fma(-mag, fq, jy);
            E = __builtin_fma(qdiag(Q) ? I.edg[k] : I.eax[k], fq, E);
        }
    }
}

// ------------------------------------------------------------------------------------
// Streaming body for INTERIOR and TUBE tiles.  The cell's moments come from the moment
// planes the previous step wrote (bit-identical to recomputing them), so the coefficients
// are ready while the first planes are still in flight; the planes then stream through
// the stages with a PD-deep prefetch, and the new moments are accumulated as the new
// values appear, in ascending q (pair partners q + 4 are held until their turn).
// ------------------------------------------------------------------------------------
template <class S, int TX, int TY, int MODE, int PD>
__device__ __forceinline__ void step_body_stream(const Inst *__restrict__ insts, const Tile &tile, int io,
                                                 StepSmem<S, TX, TY> &sm) {
    const int bin = io_in(io), bout = io_out(io);
    // EDGE: every cell and halo cell goes through the side mapping; the pressures of the
    // mirror images beside walls are left to wall_pressure_kernel (they need the cell's 33
    // new values summed in mirrored order).
    constexpr int NT = TX * TY;
    constexpr int H0 = MODE == MODE_TUBE ? 4 * TX : 0;  // the tube body loads only the x halo
    constexpr int NHALL = 4 * (TX + TY);
    constexpr int NSLOT = (NHALL - H0 + NT - 1) / NT;
    constexpr int LW = TX + 4;
    using Cell = typename CellOf<S>::type;
    const Inst &I = insts[tile.inst];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = tile.x0 + tx, y = tile.y0 + ty;
    const int ny = I.ny;
    const bool valid = MODE != MODE_EDGE || (x < I.nx && y < ny);
    const GLOBAL_AS char *fin = (const GLOBAL_AS char *)(I.f[bin]);
    GLOBAL_AS char *fout = (GLOBAL_AS char *)(I.f[bout]);
    const size_t pb = (size_t)I.fplane * sizeof(S);

    // offsets: bytes for INTERIOR / TUBE, elements (with mapping) for EDGE
    Src own;
    double tnow = 0.0;
    if constexpr (MODE != MODE_EDGE) own = Src{(int)((y * I.fpitch + x) * (int)sizeof(S)), 0, -1};
    else {
        tnow = step_time(I);
        own = map_cell(I, x, y, tnow);
    }
    Src hs[NSLOT];
    int hl[NSLOT];
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const int hid = tid + j * NT + H0;
        hl[j] = -1;
        hs[j] = Src{0, 0, -1};
        if (hid < NHALL) {
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
            hl[j] = ly * LW + lx;
            const int X = tile.x0 + lx - 2, Y = tile.y0 + ly - 2;
            if constexpr (MODE != MODE_EDGE) hs[j] = Src{(int)((Y * I.fpitch + X) * (int)sizeof(S)), 0, -1};
            else hs[j] = map_cell(I, X, Y, tnow);
        }
    }

    // prefetch ring: own and halo values of the next PD stages
    S po[PD][2];
    S ph[PD][2][NSLOT];
    auto load_stage = [&](auto stc, const Inst &Is, size_t pbs) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD, qa = stage_qa(st), qb = stage_qb(st);
        po[slot][0] = fetch<qa, MODE, S>(Is, fin, pbs, own);
        if constexpr (qb >= 0) po[slot][1] = fetch<qb, MODE, S>(Is, fin, pbs, own);
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) {
                ph[slot][0][j] = fetch<qa, MODE, S>(Is, fin, pbs, hs[j]);
                if constexpr (qb >= 0) ph[slot][1][j] = fetch<qb, MODE, S>(Is, fin, pbs, hs[j]);
            }
    };
    static_for<0, PD>([&](auto stc) { load_stage(stc, I, pb); });

    // A2: moments of the cell from the previous step; A3: switching function
    // (an edge tile's idle threads read their clamped cell; M and f planes share the pitch)
    const GLOBAL_AS double *Mc =
        (const GLOBAL_AS double *)I.M[bin] + (MODE == MODE_EDGE ? own.off : y * I.ppitch + x);
    const double n = Mc[0], ux = Mc[I.mplane], uy = Mc[2 * I.mplane], T = Mc[3 * I.mplane];
    const double P0 = n * T;
    double Pxm, Pxp, Pym, Pyp;
    // the neighbours' pressure: n T of their stored moments (no pressure plane)
    if constexpr (MODE == MODE_EDGE) {
        const double *Min = I.M[bin], *PWin = I.PW[bin];
        Pxm = load_P_m(I, Min, PWin, x - 1, y, tnow);
        Pxp = load_P_m(I, Min, PWin, x + 1, y, tnow);
        Pym = load_P_m(I, Min, PWin, x, y - 1, tnow);
        Pyp = load_P_m(I, Min, PWin, x, y + 1, tnow);
    } else {
        const GLOBAL_AS double *Mn = (const GLOBAL_AS double *)I.M[bin];
        const GLOBAL_AS double *MT = Mn + 3 * (size_t)I.mplane;
        const int c = y * I.ppitch + x;
        Pxm = Mn[c - 1] * MT[c - 1];
        Pxp = Mn[c + 1] * MT[c + 1];
        if constexpr (MODE == MODE_INTERIOR) {
            Pym = Mn[c - I.ppitch] * MT[c - I.ppitch];
            Pyp = Mn[c + I.ppitch] * MT[c + I.ppitch];
        } else {
            const int cm = (y == 0 ? ny - 1 : y - 1) * I.ppitch + x, cp = (y == ny - 1 ? 0 : y + 1) * I.ppitch + x;
            Pym = Mn[cm] * MT[cm];
            Pyp = Mn[cp] * MT[cp];
        }
    }
    const double ax = av_coeff(I.lam, I.th0, Pxm, P0, Pxp, ux, I.dt, I.dx);
    const double ay = av_coeff(I.lam, I.th0, Pym, P0, Pyp, uy, I.dt, I.dy);

    // A4: equilibrium coefficients
    Coef C;
    equilibrium_coefs(I, n, ux, uy, T, C);
    Cell cell;
    make_cell(C, ux, uy, ax, ay, I.dtau, cell);

    const int own_l = (ty + 2) * LW + (tx + 2);
    const uint32_t own_b = MODE != MODE_EDGE ? (uint32_t)own.off : (uint32_t)((y * I.fpitch + x) * (int)sizeof(S));
    auto put = [&](S *pl, S v) {
        pl[own_l] = v;
        if constexpr (MODE == MODE_TUBE) {
            if (ty >= TY - 2) pl[own_l - TY * LW] = v;  // y = -2, -1 are rows ny - 2, ny - 1
            if (ty < 2) pl[own_l + TY * LW] = v;        // y = ny, ny + 1 are rows 0, 1
        }
    };
    auto update = [&](auto qc, const Inst &Is, const S *pl, S f0, S feq) {
        constexpr int q = decltype(qc)::value;
        return update_q<q, S>(Is, cell, f0, feq, pl[own_l - 2], pl[own_l - 1], pl[own_l + 1], pl[own_l + 2],
                              pl[own_l - 2 * LW], pl[own_l - LW], pl[own_l + LW], pl[own_l + 2 * LW]);
    };

    double n2 = 0.0, jx2 = 0.0, jy2 = 0.0, E2 = 0.0;
    S hold[3];
    int b = 0;
    static_for<0, NSTAGE>([&](auto stc) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD, qa = stage_qa(st), qb = stage_qb(st);
        const Inst &Is = insts[opaque(tile.inst)];
        const size_t pbs = opaque(pb);
        S *pa = &sm.buf[b][0][0][0];
        S *pbuf = &sm.buf[b][1][0][0];
        const S fa0 = po[slot][0];
        S fb0 = fa0;
        put(pa, fa0);
        if constexpr (qb >= 0) {
            fb0 = po[slot][1];
            put(pbuf, fb0);
        }
#pragma unroll
        for (int j = 0; j < NSLOT; ++j)
            if (hl[j] >= 0) {
                pa[hl[j]] = ph[slot][0][j];
                if constexpr (qb >= 0) pbuf[hl[j]] = ph[slot][1][j];
            }
        __syncthreads();
        if constexpr (st + PD < NSTAGE) load_stage(std::integral_constant<int, st + PD>{}, Is, pbs);
        if constexpr (qb < 0) {
            const S fn = update(std::integral_constant<int, 0>{}, Is, pa, fa0, static_cast<S>(cell.nF[0] * cell.c0));
            if (valid) store_out(reinterpret_cast<GLOBAL_AS S *>(fout + own_b), fn);
            acc_term<0>(Is, fn, n2, jx2, jy2, E2);
        } else {
            S fea, feb;
            feq_pair<qa, S>(Is, cell, fea, feb);
            const S fna = update(std::integral_constant<int, qa>{}, Is, pa, fa0, fea);
            const S fnb = update(std::integral_constant<int, qb>{}, Is, pbuf, fb0, feb);
            if (valid) {
                store_out(reinterpret_cast<GLOBAL_AS S *>(fout + (size_t)qa * pbs + own_b), fna);
                store_out(reinterpret_cast<GLOBAL_AS S *>(fout + (size_t)qb * pbs + own_b), fnb);
            }
            // ascending q within the speed group: 1..4 as they come, 5..7 held, then 8
            constexpr int j = (st - 1) % 4;
            acc_term<qa>(Is, fna, n2, jx2, jy2, E2);
            if constexpr (j < 3) {
                hold[j] = fnb;
            } else {
                acc_term<qa + 1>(Is, hold[0], n2, jx2, jy2, E2);
                acc_term<qa + 2>(Is, hold[1], n2, jx2, jy2, E2);
                acc_term<qa + 3>(Is, hold[2], n2, jx2, jy2, E2);
                acc_term<qb>(Is, fnb, n2, jx2, jy2, E2);
            }
        }
        b ^= 1;
    });

    // A6: moments and pressure for the next step, flag (one store per workgroup)
    double ux2, uy2, T2, P2;
    primitive(n2, jx2, jy2, E2, ux2, uy2, T2, P2);
    if (valid) {
        GLOBAL_AS double *Mo = (GLOBAL_AS double *)I.M[bout] + (y * I.ppitch + x);
        Mo[0] = n2;
        Mo[I.mplane] = ux2;
        Mo[2 * I.mplane] = uy2;
        Mo[3 * I.mplane] = T2;
        // the pressure plane only for a register-resident edge body, which reads it
        if constexpr (!stream_edge<S>()) ((GLOBAL_AS double *)I.P[bout])[y * I.ppitch + x] = P2;
    }
    const int bad = valid && nonphysical(I, n2, ux2, uy2, T2) ? 1 : 0;
    if (__syncthreads_or(bad) && tid == 0) *I.flag = 1;
}

#ifndef FDLB_PREFETCH
#define FDLB_PREFETCH 2  // stages of look-ahead of the streaming body
#endif
// Interior body per precision (measured): float64 streams the planes and reads the
// moments the previous step stored; float32 keeps the cell's 33 values in registers and
// recomputes its moments (its extra moment traffic would cost more than the recompute).
// FDLB_STREAM = 0 / 1 forces one body for both precisions.
#ifndef FDLB_STREAM
#define FDLB_STREAM -1
#endif
template <class S>
constexpr bool use_stream() {
    return FDLB_STREAM < 0 ? std::is_same<S, double>::value : FDLB_STREAM != 0;
}
template <class S>
constexpr bool stream_moments() {
    return use_stream<S>();
}
// Edge tiles through the streaming body too (float64): the wall-image pressures then come
// from wall_pressure_kernel after the step.
template <class S>
constexpr bool stream_edge() {
    return use_stream<S>() && FDLB_STREAM_EDGE != 0;
}

// Minimum waves per SIMD asked of the step kernels' register allocation (0: the compiler's
// own choice).  FDLB_STEP_WAVES applies to the float64 and float32 kernels, FDLB_DEV_WAVES
// to the deviation kernels.
#ifndef FDLB_STEP_WAVES
#define FDLB_STEP_WAVES 0
#endif
#ifndef FDLB_DEV_WAVES
#define FDLB_DEV_WAVES 0
#endif
#if FDLB_STEP_WAVES > 0
#define FDLB_STEP_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(FDLB_STEP_WAVES)))
#else
#define FDLB_STEP_WAVES_ATTR
#endif
#if FDLB_DEV_WAVES > 0
#define FDLB_DEV_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(FDLB_DEV_WAVES)))
#else
#define FDLB_DEV_WAVES_ATTR
#endif

// One kernel per tile kind, so the common interior kernel gets its own (small) register
// allocation; the host splits the tile table by kind (same rule as tile_kind below).
template <class S, int TX, int TY, int MODE>
__global__ __launch_bounds__(TX *TY) FDLB_STEP_WAVES_ATTR void step_kernel(const Inst *__restrict__ insts, const Tile *__restrict__ tiles,
                                                      int ntiles, int io) {
    __shared__ StepSmem<S, TX, TY> sm;
    constexpr bool HD = halo_dma<S, TX, TY, MODE>() && !use_stream<S>();
    __shared__ S hdma[HD ? halo_dma_size<TX, TY>() : 1];
    const Tile tile = tiles[xcd_remap(blockIdx.x, ntiles)];
    if constexpr (!use_stream<S>() || (MODE == MODE_EDGE && !stream_edge<S>()))
        step_body<S, TX, TY, MODE>(insts, tile, io, sm, hdma);
    else
        step_body_stream<S, TX, TY, MODE, FDLB_PREFETCH>(insts, tile, io, sm);
}

// ------------------------------------------------------------------------------------
// Two steps per pass (float64, tiles whose tile and four cells around it lie inside the
// grid).  The stencil of Eq. (dis_eq1) reaches two cells, so two steps of a TX x TY tile
// need step n on the tile and four cells around it (R0) and step n + 1 on the tile and the
// two-cell cross around it (R1).  Phase 1 streams the planes of step n through LDS and takes
// step n + 1 on R1 into LDS (all 33 planes), phase 2 takes step n + 2 on the tile from
// there.  Each cell-update runs the same functions in the same order as the single-step
// streaming body (moments of step n from the stored moment planes, the neighbours'
// pressure as n T of their moments, the new moments summed in ascending q), so the result
// is that of two single steps bit for bit, for half the memory traffic.
// ------------------------------------------------------------------------------------
// The staged planes use an odd row pitch (TX + 9 doubles): lanes that walk down a halo
// column then fall on distinct LDS banks.
template <int TX, int TY>
struct Step2Smem {
    double stage[2][2][TY + 8][TX + 9];  // planes of step n on R0 (a pair per stage, double buffered)
    double f1[NQ][TY + 4][TX + 4];       // step n + 1 on R1
    double P1[TY + 2][TX + 2];           // its pressure on the tile and the one-cell ring
};

template <int TX, int TY>
constexpr int step2_threads() {
    return (TX * TY + 4 * (TX + TY) + 63) / 64 * 64;  // one thread per cell of R1
}

template <int TX, int TY, int PD>
__device__ __forceinline__ void step2_body(const Inst *__restrict__ insts, const Tile &tile, int io,
                                           Step2Smem<TX, TY> &sm) {
    constexpr int NT = step2_threads<TX, TY>();
    constexpr int NTILE = TX * TY;
    constexpr int NR1 = NTILE + 4 * (TX + TY);
    constexpr int R0W = TX + 8, R0H = TY + 8, NR0 = R0W * R0H, R0P = TX + 9;  // R0P: LDS row pitch
    constexpr int NSL = (NR0 + NT - 1) / NT;  // R0 cells each thread stages per plane
    const Inst &I = insts[tile.inst];
    const int bin = io_in(io), bout = io_out(io);
    const bool ring = (tile.flags & kTileRing) != 0;
    const int tid = threadIdx.x;

    // this thread's cell of R1 (tile-local; -2..TX+1, -2..TY+1, cross-shaped)
    int lx, ly;
    if (tid < NTILE) {
        lx = tid % TX;
        ly = tid / TX;
    } else {
        const int hid = tid - NTILE;
        if (hid < 4 * TX) {
            const int r = hid / TX;
            lx = hid % TX;
            ly = r < 2 ? r - 2 : TY + r - 2;
        } else {
            const int h2 = min(hid - 4 * TX, 4 * TY - 1);  // threads past R1 take its last cell
            const int c = h2 / TY;
            ly = h2 % TY;
            lx = c < 2 ? c - 2 : TX + c - 2;
        }
    }
    const bool active = tid < NR1;
    const GLOBAL_AS char *fin = (const GLOBAL_AS char *)(I.f[bin]);
    GLOBAL_AS char *fout = (GLOBAL_AS char *)(I.f[bout]);
    GLOBAL_AS char *fmid = (GLOBAL_AS char *)(I.f[2]);
    const size_t pb = (size_t)I.fplane * sizeof(double);

    // R0 staging: slot j of this thread is cell r0 = tid + j NT of the (TX+8) x (TY+8)
    // rectangle; its corners beyond the stencils' reach are loaded from a clamped cell and
    // never read (the loads stay unconditional)
    int r0off[NSL], r0l[NSL];
#pragma unroll
    for (int j = 0; j < NSL; ++j) {
        const int r0 = min(tid + j * NT, NR0 - 1);
        r0l[j] = tid + j * NT < NR0 ? (r0 / R0W) * R0P + r0 % R0W : -1;
        const int X = tile.x0 + r0 % R0W - 4, Y = tile.y0 + r0 / R0W - 4;
        r0off[j] = (Y * I.fpitch + X) * (int)sizeof(double);
    }
    double pr[PD][2][NSL];
    auto load_stage = [&](auto stc, const Inst &Is, size_t pbs) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD, qa = stage_qa(st), qb = stage_qb(st);
#pragma unroll
        for (int j = 0; j < NSL; ++j) {
            pr[slot][0][j] = *reinterpret_cast<const GLOBAL_AS double *>(fin + (size_t)qa * pbs + (uint32_t)r0off[j]);
            if constexpr (qb >= 0)
                pr[slot][1][j] = *reinterpret_cast<const GLOBAL_AS double *>(fin + (size_t)qb * pbs + (uint32_t)r0off[j]);
        }
    };
    static_for<0, PD>([&](auto stc) { load_stage(stc, I, pb); });

    // phase 1 set-up: moments of step n from the moment planes, switching function from the
    // neighbours' n T (all of R1's neighbours lie inside the grid)
    const int x = tile.x0 + lx, y = tile.y0 + ly;
    const int c = y * I.ppitch + x;
    const GLOBAL_AS double *Mn = (const GLOBAL_AS double *)I.M[bin];
    const GLOBAL_AS double *MT = Mn + 3 * (size_t)I.mplane;
    const double n = Mn[c], ux = Mn[c + I.mplane], uy = Mn[c + 2 * I.mplane], T = MT[c];
    const double P0 = n * T;
    const double Pxm = Mn[c - 1] * MT[c - 1];
    const double Pxp = Mn[c + 1] * MT[c + 1];
    const double Pym = Mn[c - I.ppitch] * MT[c - I.ppitch];
    const double Pyp = Mn[c + I.ppitch] * MT[c + I.ppitch];
    CellD cell;
    {
        const double ax = av_coeff(I.lam, I.th0, Pxm, P0, Pxp, ux, I.dt, I.dx);
        const double ay = av_coeff(I.lam, I.th0, Pym, P0, Pyp, uy, I.dt, I.dy);
        Coef C;
        equilibrium_coefs(I, n, ux, uy, T, C);
        make_cell(C, ux, uy, ax, ay, I.dtau, cell);
    }
    const int o0 = (ly + 4) * R0P + (lx + 4);  // own cell in the R0 frame
    const int o1x = lx + 2, o1y = ly + 2;         // own cell in the R1 frame
    const uint32_t own_b = (uint32_t)(c * (int)sizeof(double));
    const bool mid_store = ring && tid < NTILE;

    auto update0 = [&](auto qc, const Inst &Is, const double *pl, double feq) {
        constexpr int q = decltype(qc)::value;
        return update_f64<q>(Is, cell, pl[o0], feq, pl[o0 - 2], pl[o0 - 1], pl[o0 + 1], pl[o0 + 2], pl[o0 - 2 * R0P],
                             pl[o0 - R0P], pl[o0 + R0P], pl[o0 + 2 * R0P]);
    };
    double n1 = 0.0, jx1 = 0.0, jy1 = 0.0, E1 = 0.0;
    double hold[3];
    int b = 0;
    static_for<0, NSTAGE>([&](auto stc) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD, qa = stage_qa(st), qb = stage_qb(st);
        const Inst &Is = insts[opaque(tile.inst)];
        const size_t pbs = opaque(pb);
        double *pa = &sm.stage[b][0][0][0];
        double *pbuf = &sm.stage[b][1][0][0];
#pragma unroll
        for (int j = 0; j < NSL; ++j)
            if (r0l[j] >= 0) {
                pa[r0l[j]] = pr[slot][0][j];
                if constexpr (qb >= 0) pbuf[r0l[j]] = pr[slot][1][j];
            }
        __syncthreads();
        if constexpr (st + PD < NSTAGE) load_stage(std::integral_constant<int, st + PD>{}, Is, pbs);
        if constexpr (qb < 0) {
            const double fn = update0(std::integral_constant<int, 0>{}, Is, pa, cell.nF[0] * cell.c0);
            if (active) sm.f1[0][o1y][o1x] = fn;
            if (mid_store) store_out(reinterpret_cast<GLOBAL_AS double *>(fmid + own_b), fn);
            acc_term<0>(Is, fn, n1, jx1, jy1, E1);
        } else {
            double fea, feb;
            feq_pair_f64<qa>(Is, cell, fea, feb);
            const double fna = update0(std::integral_constant<int, qa>{}, Is, pa, fea);
            const double fnb = update0(std::integral_constant<int, qb>{}, Is, pbuf, feb);
            if (active) {
                sm.f1[qa][o1y][o1x] = fna;
                sm.f1[qb][o1y][o1x] = fnb;
            }
            if (mid_store) {
                store_out(reinterpret_cast<GLOBAL_AS double *>(fmid + (size_t)qa * pbs + own_b), fna);
                store_out(reinterpret_cast<GLOBAL_AS double *>(fmid + (size_t)qb * pbs + own_b), fnb);
            }
            constexpr int j = (st - 1) % 4;
            acc_term<qa>(Is, fna, n1, jx1, jy1, E1);
            if constexpr (j < 3) {
                hold[j] = fnb;
            } else {
                acc_term<qa + 1>(Is, hold[0], n1, jx1, jy1, E1);
                acc_term<qa + 2>(Is, hold[1], n1, jx1, jy1, E1);
                acc_term<qa + 3>(Is, hold[2], n1, jx1, jy1, E1);
                acc_term<qb>(Is, fnb, n1, jx1, jy1, E1);
            }
        }
        b ^= 1;
    });

    // moments of step n + 1; pressure ring for the second switching function
    double ux1, uy1, T1, P1;
    primitive(n1, jx1, jy1, E1, ux1, uy1, T1, P1);
    const double P1m = n1 * T1;  // n T of the moments, as the next step reads them
    if (active && lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) sm.P1[ly + 1][lx + 1] = P1m;
    int bad = tid < NTILE && nonphysical(I, n1, ux1, uy1, T1) ? 1 : 0;
    if (mid_store) {
        GLOBAL_AS double *Mo = (GLOBAL_AS double *)I.M[2] + c;
        Mo[0] = n1;
        Mo[I.mplane] = ux1;
        Mo[2 * I.mplane] = uy1;
        Mo[3 * I.mplane] = T1;
    }
    __syncthreads();

    // phase 2: step n + 2 on the tile from LDS
    if (tid < NTILE) {
        CellD cell2;
        {
            const double ax = av_coeff(I.lam, I.th0, sm.P1[ly + 1][lx], P1m, sm.P1[ly + 1][lx + 2], ux1, I.dt, I.dx);
            const double ay = av_coeff(I.lam, I.th0, sm.P1[ly][lx + 1], P1m, sm.P1[ly + 2][lx + 1], uy1, I.dt, I.dy);
            Coef C;
            equilibrium_coefs(I, n1, ux1, uy1, T1, C);
            make_cell(C, ux1, uy1, ax, ay, I.dtau, cell2);
        }
        auto update1 = [&](auto qc, const Inst &Is, double feq) {
            constexpr int q = decltype(qc)::value;
            const double(&pl)[TY + 4][TX + 4] = sm.f1[q];
            return update_f64<q>(Is, cell2, pl[o1y][o1x], feq, pl[o1y][o1x - 2], pl[o1y][o1x - 1], pl[o1y][o1x + 1],
                                 pl[o1y][o1x + 2], pl[o1y - 2][o1x], pl[o1y - 1][o1x], pl[o1y + 1][o1x],
                                 pl[o1y + 2][o1x]);
        };
        double n2 = 0.0, jx2 = 0.0, jy2 = 0.0, E2 = 0.0;
        double hold2[3];
        static_for<0, NSTAGE>([&](auto stc) {
            constexpr int st = decltype(stc)::value;
            constexpr int qa = stage_qa(st), qb = stage_qb(st);
            const Inst &Is = insts[opaque(tile.inst)];
            const size_t pbs = opaque(pb);
            if constexpr (qb < 0) {
                const double fn = update1(std::integral_constant<int, 0>{}, Is, cell2.nF[0] * cell2.c0);
                store_out(reinterpret_cast<GLOBAL_AS double *>(fout + own_b), fn);
                acc_term<0>(Is, fn, n2, jx2, jy2, E2);
            } else {
                double fea, feb;
                feq_pair_f64<qa>(Is, cell2, fea, feb);
                const double fna = update1(std::integral_constant<int, qa>{}, Is, fea);
                const double fnb = update1(std::integral_constant<int, qb>{}, Is, feb);
                store_out(reinterpret_cast<GLOBAL_AS double *>(fout + (size_t)qa * pbs + own_b), fna);
                store_out(reinterpret_cast<GLOBAL_AS double *>(fout + (size_t)qb * pbs + own_b), fnb);
                constexpr int j = (st - 1) % 4;
                acc_term<qa>(Is, fna, n2, jx2, jy2, E2);
                if constexpr (j < 3) {
                    hold2[j] = fnb;
                } else {
                    acc_term<qa + 1>(Is, hold2[0], n2, jx2, jy2, E2);
                    acc_term<qa + 2>(Is, hold2[1], n2, jx2, jy2, E2);
                    acc_term<qa + 3>(Is, hold2[2], n2, jx2, jy2, E2);
                    acc_term<qb>(Is, fnb, n2, jx2, jy2, E2);
                }
            }
        });
        double ux2, uy2, T2, P2;
        primitive(n2, jx2, jy2, E2, ux2, uy2, T2, P2);
        GLOBAL_AS double *Mo = (GLOBAL_AS double *)I.M[bout] + c;
        Mo[0] = n2;
        Mo[I.mplane] = ux2;
        Mo[2 * I.mplane] = uy2;
        Mo[3 * I.mplane] = T2;
        bad |= nonphysical(I, n2, ux2, uy2, T2) ? 1 : 0;
    }
    if (__syncthreads_or(bad) && tid == 0) *I.flag = 1;
}

#ifndef FDLB_STEP2_PREFETCH
#define FDLB_STEP2_PREFETCH 2  // stages of look-ahead of the two-step body's first phase
#endif
template <int TX, int TY>
__global__ __launch_bounds__((step2_threads<TX, TY>())) void step2_kernel(const Inst *__restrict__ insts,
                                                                       const Tile *__restrict__ tiles, int ntiles,
                                                                       int io) {
    __shared__ Step2Smem<TX, TY> sm;
    const Tile tile = tiles[xcd_remap(blockIdx.x, ntiles)];
    step2_body<TX, TY, FDLB_STEP2_PREFETCH>(insts, tile, io, sm);
}

// ------------------------------------------------------------------------------------
// Deviation storage (precision FDLB_F32_DEV).
//
// A cell stores its moments M = (n, ux, uy, T) in float64 and its distributions as
// g_q = f_q - f^eq_q(M) in float32.  At high Mach number the f_q themselves are large and
// of both signs (their sum n is a small difference of them), so rounding f_q to float32
// loses the temperature; g is small wherever the flow is near equilibrium and carries no
// such cancellation.  The step:
//   rebuild f = f^eq(M) + g in float64 for the tile and its halo (LDS, one plane pair per
//   stage, as in the other bodies); switching function from P = n T of the stored M;
//   Eq. (dis_eq1) in float64 with the collision toward f^eq(M) (the same values that
//   rebuilt the cell); then the new moments M' of f_new in float64 and
//   g' = f_new - f^eq(M'), stored in float32.
// f^eq here is evaluated with fused multiply-adds, the same function on both sides of the
// round trip, so rebuilding reproduces f_new up to the float32 rounding of g' alone.
// ------------------------------------------------------------------------------------
struct DevCell {
    double c0, c1, c2, c3, c4;
    double nF[5];
    double ux, uy;
};

// The coefficients of equilibrium_coefs with one division (1/T) and fused multiply-adds.
__device__ __forceinline__ void dev_cell(const Inst &I, double n, double ux, double uy, double T, DevCell &d) {
    const double iT = 1.0 / T;
    const double iT2 = iT * iT;
    double sF = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double num = __builtin_fma(__builtin_fma(__builtin_fma(48.0, T, -I.FA[k]), T, I.FB[k]), T, -I.FC[k]) * T;
        const double F = num * I.Fdinv[k];
        d.nF[k + 1] = n * F;
        sF += F;
    }
    d.nF[0] = n * __builtin_fma(-8.0, sF, 1.0);
    const double u2 = __builtin_fma(ux, ux, uy * uy);
    const double h = __builtin_fma(-0.5 * u2, iT, 1.0);
    d.c0 = __builtin_fma(0.125 * (u2 * u2), iT2, h);
    d.c1 = h * iT;
    d.c2 = 0.5 * h * iT2;
    d.c3 = iT2 * iT * (1.0 / 6.0);
    d.c4 = iT2 * iT2 * (1.0 / 24.0);
    d.ux = ux;
    d.uy = uy;
}

// Line-IV coefficient (Eqs. add3, add4) with one division; theta as in av_coeff.
__device__ __forceinline__ double av_dev(double lam, double th0, double Pm, double P0, double Pp, double u,
                                         double cdr) {
    const double th = __builtin_fma(lam, fabs((Pp - 2.0 * P0 + Pm) / (Pp + 2.0 * P0 + Pm)), th0);
    const double kap = fabs(u * cdr);
    return th * kap * (1.0 - kap) * 0.5;
}

// s = v_q . u of the deviation body (a diagonal with one fused multiply-add).
template <int Q>
__device__ __forceinline__ double dev_s(const Inst &I, double ux, double uy) {
    constexpr int k = qk(Q), sx = qsx(Q), sy = qsy(Q);
    if constexpr (sx != 0 && sy != 0) {
        const double m = I.vs[k];
        return __builtin_fma(sx > 0 ? m : -m, ux, (sy > 0 ? m : -m) * uy);
    } else {
        return s_of<Q, double>(I.v[k], ux, uy);
    }
}

// f^eq of the pair (qa, qa + 4): even and odd powers of s = v . u (qa = 0: the rest value).
template <int QA>
__device__ __forceinline__ void dev_feq_pair(const Inst &I, const DevCell &d, double &fa, double &fb) {
    if constexpr (QA == 0) {
        fa = d.nF[0] * d.c0;
        fb = fa;
    } else {
        constexpr int k = qk(QA);
        const double s = dev_s<QA>(I, d.ux, d.uy);
        const double s2 = s * s;
        const double ev = __builtin_fma(__builtin_fma(d.c4, s2, d.c2), s2, d.c0);
        const double od = s * __builtin_fma(d.c3, s2, d.c1);
        fa = d.nF[k + 1] * (ev + od);
        fb = d.nF[k + 1] * (ev - od);
    }
}

// Eq. (dis_eq1) for one velocity in float64 as weights on the five points of each
// direction (the float32 update's form), with fused multiply-adds.
template <int Q>
__device__ __forceinline__ double update_dev(const Inst &I, double ax, double ay, double omd, double f0,
                                             double feq, double xm2, double xm1, double xp1, double xp2, double ym2,
                                             double ym1, double yp1, double yp2) {
    constexpr int k = qk(Q), dg = qdiag(Q) ? 1 : 0, sx = qsx(Q), sy = qsy(Q);
    double Kx = ax, Ky = ay;
    if constexpr (sx != 0) Kx = I.k2[0][dg][k] + ax;
    if constexpr (sy != 0) Ky = I.k2[1][dg][k] + ay;
    double fn = (omd - 2.0 * (Kx + Ky)) * f0;
    fn = __builtin_fma(I.dtau, feq, fn);
    if constexpr (sx != 0) {
        const double k3 = I.k3[0][dg][k];
        const double kk = I.kk[0][dg][k];
        fn = __builtin_fma(sx > 0 ? Kx - kk : Kx + kk, xp1, fn);
        fn = __builtin_fma(sx > 0 ? Kx + kk : Kx - kk, xm1, fn);
        fn = __builtin_fma(sx > 0 ? k3 : -k3, xp2 - xm2, fn);
    } else {
        fn = __builtin_fma(Kx, xp1 + xm1, fn);
    }
    if constexpr (sy != 0) {
        const double k3 = I.k3[1][dg][k];
        const double kk = I.kk[1][dg][k];
        fn = __builtin_fma(sy > 0 ? Ky - kk : Ky + kk, yp1, fn);
        fn = __builtin_fma(sy > 0 ? Ky + kk : Ky - kk, ym1, fn);
        fn = __builtin_fma(sy > 0 ? k3 : -k3, yp2 - ym2, fn);
    } else {
        fn = __builtin_fma(Ky, yp1 + ym1, fn);
    }
    return fn;
}

// g of plane Q at a (mapped) cell; a Dirichlet ghost is its state's equilibrium, g = 0.
// Offsets are elements (M and f planes share the row pitch).
template <int Q, int MODE>
__device__ __forceinline__ float fetch_g(const Inst &I, const GLOBAL_AS char *gin, size_t pb, const Src &s) {
    if constexpr (MODE != MODE_EDGE) {
        return *reinterpret_cast<const GLOBAL_AS float *>(gin + (size_t)Q * pb + (uint32_t)s.off * 4u);
    } else {
        if (s.dside >= 0) return 0.0f;
        const int qq = s.flip == 0 ? Q : s.flip == 1 ? qmx(Q) : s.flip == 2 ? qmy(Q) : qmx(qmy(Q));
        return reinterpret_cast<const GLOBAL_AS float *>(gin)[(size_t)qq * I.fplane + s.off];
    }
}

// Stored moments of a (mapped) cell; the mirror image across a wall has the normal
// velocity component reversed; a Dirichlet ghost has its side's state.
template <int MODE>
__device__ __forceinline__ void load_m(const Inst &I, const GLOBAL_AS double *Min, const Src &s, double &n,
                                       double &ux, double &uy, double &T) {
    if constexpr (MODE == MODE_EDGE) {
        if (s.dside >= 0) {
            n = I.bcstate[s.dside][0];
            ux = I.bcstate[s.dside][1];
            uy = I.bcstate[s.dside][2];
            T = I.bcstate[s.dside][3];
            return;
        }
    }
    const GLOBAL_AS double *m = Min + (uint32_t)s.off;
    n = m[0];
    ux = m[I.mplane];
    uy = m[2 * I.mplane];
    T = m[3 * I.mplane];
    if constexpr (MODE == MODE_EDGE) {
        if (s.flip & 1) ux = -ux;
        if (s.flip & 2) uy = -uy;
    }
}

// Materialises a value in vector registers at this point of the program.  The new values
// of a stage are only used after the last stage; without this the compiler sinks each
// stage's arithmetic to that use and keeps all the LDS operands of all stages alive.
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

// Equilibrium coefficients of the halo cells, one row per field (c0..c4, ux, uy, nF0..4),
// indexed by halo id: the halo threads keep them here rather than in registers.
constexpr int kHaloFields = 12;

// P holds the pressure of the tile and its one-cell ring only (the switching function reads
// the neighbours at +-1), which keeps a 32 x 8 tile's block within 32 KiB: five blocks fit
// the 160 KiB of a CU.
template <int TX, int TY, int UPS, int NHC>
struct DevSmem {
    double buf[2][2 * UPS][TY + 4][TX + 4];
    double P[(TY + 2) * (TX + 2)];
    double hc[kHaloFields][NHC];
};

// Halo cells a tile kind loads (the tube kind only its x halo).
template <int TX, int TY, int MODE>
constexpr int dev_halo_cells() {
    return 4 * (TX + TY) - (MODE == MODE_TUBE ? 4 * TX : 0);
}

// f^eq of the pair (qa, qa + 4) of halo cell `h` from the LDS coefficient rows.
template <int QA, int NH>
__device__ __forceinline__ void dev_feq_pair_lds(const Inst &I, const double (&hc)[kHaloFields][NH], int h, double &fa,
                                                 double &fb) {
    if constexpr (QA == 0) {
        fa = hc[7][h] * hc[0][h];
        fb = fa;
    } else {
        constexpr int k = qk(QA);
        const double s = dev_s<QA>(I, hc[5][h], hc[6][h]);
        const double s2 = s * s;
        const double ev = __builtin_fma(__builtin_fma(hc[4][h], s2, hc[2][h]), s2, hc[0][h]);
        const double od = s * __builtin_fma(hc[3][h], s2, hc[1][h]);
        fa = hc[8 + k][h] * (ev + od);
        fb = hc[8 + k][h] * (ev - od);
    }
}

// One body for the three tile kinds (side mapping only in EDGE tiles).
template <int TX, int TY, int MODE, int PD, int UPS>
__device__ __forceinline__ void step_body_dev(const Inst *__restrict__ insts, const Tile &tile, int io,
                                              DevSmem<TX, TY, UPS, dev_halo_cells<TX, TY, MODE>()> &sm) {
    const int bin = io_in(io), bout = io_out(io);
    const Inst &I = insts[tile.inst];
    constexpr int NT = TX * TY;
    constexpr int H0 = MODE == MODE_TUBE ? 4 * TX : 0;  // the tube body loads only the x halo
    constexpr int NHALL = 4 * (TX + TY);
    constexpr int NSLOT = (NHALL - H0 + NT - 1) / NT;
    constexpr int LW = TX + 4;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = tile.x0 + tx, y = tile.y0 + ty;
    const bool valid = MODE != MODE_EDGE || (x < I.nx && y < I.ny);
    const GLOBAL_AS char *gin = (const GLOBAL_AS char *)(I.f[bin]);
    GLOBAL_AS char *gout = (GLOBAL_AS char *)(I.f[bout]);
    const size_t pb = (size_t)I.fplane * sizeof(float);
    const GLOBAL_AS double *Min = (const GLOBAL_AS double *)I.M[bin];

    Src own;
    double tnow = 0.0;
    if constexpr (MODE != MODE_EDGE) own = Src{y * I.fpitch + x, 0, -1};
    else {
        tnow = step_time(I);
        own = map_cell(I, x, y, tnow);
    }
    Src hs[NSLOT];
    int hl[NSLOT];
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const int hid = tid + j * NT + H0;
        hl[j] = -1;
        hs[j] = Src{0, 0, -1};
        if (hid < NHALL) {
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
            hl[j] = ly * LW + lx;
            const int X = tile.x0 + lx - 2, Y = tile.y0 + ly - 2;
            if constexpr (MODE != MODE_EDGE) hs[j] = Src{Y * I.fpitch + X, 0, -1};
            else hs[j] = map_cell(I, X, Y, tnow);
        } else if constexpr (MODE != MODE_EDGE) {
            hs[j] = own;  // no halo cell: loads stay unconditional (a load under a branch makes
                          // the compiler wait for every load in flight where the branch joins)
        }
    }

    // Units: unit 0 is the rest plane, unit u >= 1 the plane pair of stage u of the other
    // bodies (stage_qa / stage_qb); a stage here processes UPS units between two barriers.
    constexpr int NSTG = (NSTAGE + UPS - 1) / UPS;

    // prefetch ring: g of the next PD stages (own cell and halo slots) in flight while the
    // equilibrium coefficients are formed and while earlier stages compute
    float go[PD][UPS][2], gh[PD][UPS][2][NSLOT];
    auto load_stage = [&](auto stc, const Inst &Is, size_t pbs) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD;
        static_for<0, UPS>([&](auto ic) {
            constexpr int i = decltype(ic)::value, u = st * UPS + i;
            if constexpr (u < NSTAGE) {
                constexpr int qa = stage_qa(u), qb = stage_qb(u);
                go[slot][i][0] = fetch_g<qa, MODE>(Is, gin, pbs, own);
                go[slot][i][1] = 0.0f;
                if constexpr (qb >= 0) go[slot][i][1] = fetch_g<qb, MODE>(Is, gin, pbs, own);
#pragma unroll
                for (int j = 0; j < NSLOT; ++j) {
                    gh[slot][i][0][j] = 0.0f;
                    gh[slot][i][1][j] = 0.0f;
                    if (MODE != MODE_EDGE || hl[j] >= 0) {
                        gh[slot][i][0][j] = fetch_g<qa, MODE>(Is, gin, pbs, hs[j]);
                        if constexpr (qb >= 0) gh[slot][i][1][j] = fetch_g<qb, MODE>(Is, gin, pbs, hs[j]);
                    }
                }
            }
        });
    };
    static_for<0, (PD < NSTG ? PD : NSTG)>([&](auto stc) { load_stage(stc, I, pb); });

    const int own_l = (ty + 2) * LW + (tx + 2);
    // an own value goes to LDS; in a tube tile also to the halo rows it wraps onto
    // (y = -2, -1 are rows ny - 2, ny - 1; y = ny, ny + 1 are rows 0, 1)
    auto put = [&](double *pl, double v) {
        pl[own_l] = v;
        if constexpr (MODE == MODE_TUBE) {
            if (ty >= TY - 2) pl[own_l - TY * LW] = v;
            if (ty < 2) pl[own_l + TY * LW] = v;
        }
    };
    // pressure ring: index of local cell (lx, ly), -1 <= lx <= TX, -1 <= ly <= TY
    constexpr int PWD = TX + 2;
    const int own_p = (ty + 1) * PWD + (tx + 1);
    DevCell dc;
    {
        double n, ux, uy, T;
        load_m<MODE>(I, Min, own, n, ux, uy, T);
        dev_cell(I, n, ux, uy, T, dc);
        const double P0 = n * T;
        sm.P[own_p] = P0;
        if constexpr (MODE == MODE_TUBE) {
            if (ty == TY - 1) sm.P[own_p - TY * PWD] = P0;  // y = -1 is row ny - 1
            if (ty == 0) sm.P[own_p + TY * PWD] = P0;       // y = ny is row 0
        }
    }
    constexpr int NH = dev_halo_cells<TX, TY, MODE>();
#pragma unroll
    for (int j = 0; j < NSLOT; ++j)
        if (MODE != MODE_EDGE || hl[j] >= 0) {
            double n, ux, uy, T;
            load_m<MODE>(I, Min, hs[j], n, ux, uy, T);
            if (hl[j] >= 0) {
                DevCell d;
                dev_cell(I, n, ux, uy, T, d);
                const int h = tid + j * NT;  // halo id relative to H0
                sm.hc[0][h] = d.c0;
                sm.hc[1][h] = d.c1;
                sm.hc[2][h] = d.c2;
                sm.hc[3][h] = d.c3;
                sm.hc[4][h] = d.c4;
                sm.hc[5][h] = d.ux;
                sm.hc[6][h] = d.uy;
#pragma unroll
                for (int k = 0; k < 5; ++k) sm.hc[7 + k][h] = d.nF[k];
                // only the ring one cell out is read by the switching function
                const int lx = hl[j] % LW - 2, ly = hl[j] / LW - 2;
                if (lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) sm.P[(ly + 1) * PWD + (lx + 1)] = n * T;
            }
        }

    const double omd = 1.0 - I.dtau;
    double ax = 0.0, ay = 0.0;
    // the new values are needed again after the last stage: g' is taken against their own
    // moments
    double fnew[NQ];
    int b = 0;
    static_for<0, NSTG>([&](auto stc) {
        constexpr int st = decltype(stc)::value;
        constexpr int slot = st % PD;
        const Inst &Is = insts[opaque(tile.inst)];
        const size_t pbs = opaque(pb);
        // rebuild f for the stage's planes: own cell (its f^eq is also the collision
        // target) and halo
        double e[UPS][2], f0[UPS][2];
        static_for<0, UPS>([&](auto ic) {
            constexpr int i = decltype(ic)::value, u = st * UPS + i;
            if constexpr (u < NSTAGE) {
                constexpr int qa = stage_qa(u), qb = stage_qb(u);
                double *pa = &sm.buf[b][2 * i][0][0];
                double *pbuf = &sm.buf[b][2 * i + 1][0][0];
                dev_feq_pair<qa>(Is, dc, e[i][0], e[i][1]);
                f0[i][0] = e[i][0] + static_cast<double>(go[slot][i][0]);
                f0[i][1] = e[i][1] + static_cast<double>(go[slot][i][1]);
                put(pa, f0[i][0]);
                if constexpr (qb >= 0) put(pbuf, f0[i][1]);
#pragma unroll
                for (int j = 0; j < NSLOT; ++j)
                    if (hl[j] >= 0) {
                        double ha, hb;
                        dev_feq_pair_lds<qa, NH>(Is, sm.hc, tid + j * NT, ha, hb);
                        pa[hl[j]] = ha + static_cast<double>(gh[slot][i][0][j]);
                        if constexpr (qb >= 0) pbuf[hl[j]] = hb + static_cast<double>(gh[slot][i][1][j]);
                    }
            }
        });
        __syncthreads();
        if constexpr (st == 0) {
            // switching function from the neighbours' P (written before the first barrier)
            const double P0 = sm.P[own_p];
            ax = av_dev(Is.lam, Is.th0, sm.P[own_p - 1], P0, sm.P[own_p + 1], dc.ux, Is.cdx);
            ay = av_dev(Is.lam, Is.th0, sm.P[own_p - PWD], P0, sm.P[own_p + PWD], dc.uy, Is.cdy);
        }
        if constexpr (st + PD < NSTG) load_stage(std::integral_constant<int, st + PD>{}, Is, pbs);
        static_for<0, UPS>([&](auto ic) {
            constexpr int i = decltype(ic)::value, u = st * UPS + i;
            if constexpr (u < NSTAGE) {
                constexpr int qa = stage_qa(u), qb = stage_qb(u);
                const double *pa = &sm.buf[b][2 * i][0][0];
                const double *pbuf = &sm.buf[b][2 * i + 1][0][0];
                fnew[qa] = update_dev<qa>(Is, ax, ay, omd, f0[i][0], e[i][0], pa[own_l - 2], pa[own_l - 1],
                                          pa[own_l + 1], pa[own_l + 2], pa[own_l - 2 * LW], pa[own_l - LW],
                                          pa[own_l + LW], pa[own_l + 2 * LW]);
                pin(fnew[qa]);
                if constexpr (qb >= 0) {
                    fnew[qb] = update_dev<qb>(Is, ax, ay, omd, f0[i][1], e[i][1], pbuf[own_l - 2], pbuf[own_l - 1],
                                              pbuf[own_l + 1], pbuf[own_l + 2], pbuf[own_l - 2 * LW],
                                              pbuf[own_l - LW], pbuf[own_l + LW], pbuf[own_l + 2 * LW]);
                    pin(fnew[qb]);
                }
            }
        });
        b ^= 1;
    });

    // new moments (float64), g' relative to them, flag
    double n2, jx2, jy2, E2;
    moments33_fast<0>(I, fnew, n2, jx2, jy2, E2);
    const double in2 = 1.0 / n2;
    const double ux2 = jx2 * in2, uy2 = jy2 * in2;
    const double T2 = __builtin_fma(-0.5, __builtin_fma(ux2, ux2, uy2 * uy2), E2 * in2);
    const int bad = valid && nonphysical(I, n2, ux2, uy2, T2) ? 1 : 0;
    DevCell dn;
    dev_cell(I, n2, ux2, uy2, T2, dn);
    const uint32_t own_b = (uint32_t)(y * I.fpitch + x) * 4u;
    if (valid) {
        static_for<0, NSTAGE>([&](auto stc) {
            constexpr int st = decltype(stc)::value;
            constexpr int qa = stage_qa(st), qb = stage_qb(st);
            const size_t pbs = opaque(pb);
            double ea, eb;
            dev_feq_pair<qa>(I, dn, ea, eb);
            const float ga = static_cast<float>(fnew[qa] - ea);
            const float gb = qb >= 0 ? static_cast<float>(fnew[qb] - eb) : 0.0f;
            store_out(reinterpret_cast<GLOBAL_AS float *>(gout + (size_t)qa * pbs + own_b), ga);
            if constexpr (qb >= 0)
                store_out(reinterpret_cast<GLOBAL_AS float *>(gout + (size_t)qb * pbs + own_b), gb);
        });
        GLOBAL_AS double *Mo = (GLOBAL_AS double *)I.M[bout] + (y * I.ppitch + x);
        Mo[0] = n2;
        Mo[I.mplane] = ux2;
        Mo[2 * I.mplane] = uy2;
        Mo[3 * I.mplane] = T2;
    }
    if (__syncthreads_or(bad) && tid == 0) *I.flag = 1;
}

#ifndef FDLB_DEV_PREFETCH
#define FDLB_DEV_PREFETCH 3  // stages of look-ahead of the deviation body
#endif
#ifndef FDLB_DEV_UPS
#define FDLB_DEV_UPS 1       // plane units (rest plane or plane pair) per stage
#endif
template <int TX, int TY, int MODE>
__global__ __launch_bounds__(TX *TY) FDLB_DEV_WAVES_ATTR void step_kernel_dev(const Inst *__restrict__ insts,
                                                          const Tile *__restrict__ tiles, int ntiles, int io) {
    __shared__ DevSmem<TX, TY, FDLB_DEV_UPS, dev_halo_cells<TX, TY, MODE>()> sm;
    const Tile tile = tiles[xcd_remap(blockIdx.x, ntiles)];
    step_body_dev<TX, TY, MODE, FDLB_DEV_PREFETCH, FDLB_DEV_UPS>(insts, tile, io, sm);
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
    if (write_pressures(I, f, x, y, I.P[half], I.M[half], I.PW[half])) *I.flag = 1;
}

// Dirichlet ghost vectors f^eq(state) rounded to storage, and their pressures.
template <class S>
__global__ void bc_setup_kernel(Inst *insts, int inst) {
    Inst &I = insts[inst];
    const int side = threadIdx.x;  // Dirichlet slot: sides 0..3, their lower segments 4..7
    if (side >= 8) return;
    if ((side < 4 ? I.bc[side] : I.bclo[side - 4]) != BC_DIRICHLET) {
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
    moments_of<0>(I, g, m, jx, jy, E);
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
    moments_of<0>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P);
    const size_t c = (size_t)y * I.nx + x, plane = (size_t)I.nx * I.ny;
    out[c] = n;
    out[plane + c] = ux;
    out[2 * plane + c] = uy;
    out[3 * plane + c] = T;
}

// Totals of (n, jx, jy, E) per 256-cell block; the flag is OR-ed.
constexpr int kDiagBlock = 256;

// Sum of v[0..3] over a 256-thread block, in a fixed order: an xor butterfly inside each
// 64-lane wavefront (every lane ends with the same bits, addition being commutative), then
// the four wavefront sums in order.  The result is valid in thread 0.
__device__ __forceinline__ void block_sum4(double (&v)[4], double (&red)[4][kDiagBlock / 64]) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v[c] = v[c] + __shfl_xor(v[c], m, 64);
    const int wave = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0)
        for (int c = 0; c < 4; ++c) red[c][wave] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) {
            double t = red[c][0];
            for (int w = 1; w < kDiagBlock / 64; ++w) t = t + red[c][w];
            v[c] = t;
        }
}
template <class S>
__global__ __launch_bounds__(256) void diag_kernel(const Inst *__restrict__ insts, int inst, int half, double *__restrict__ partials) {
    const Inst &I = insts[inst];
    __shared__ double red[4][kDiagBlock / 64];
    const long cell = (long)blockIdx.x * kDiagBlock + threadIdx.x;
    const long ncell = (long)I.nx * I.ny;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (cell < ncell) {
        const int x = (int)(cell % I.nx), y = (int)(cell / I.nx);
        const S *fin = static_cast<const S *>(I.f[half]);
        S f[NQ];
        const size_t off = (size_t)y * I.fpitch + x;
        static_for<0, NQ>([&](auto qc) { f[decltype(qc)::value] = fin[(size_t)decltype(qc)::value * I.fplane + off]; });
        moments_of<0>(I, f, v[0], v[1], v[2], v[3]);
        double ux, uy, T, P;
        primitive(v[0], v[1], v[2], v[3], ux, uy, T, P);
        if (nonphysical(I, v[0], ux, uy, T)) *I.flag = 1;
    }
    block_sum4(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partials[4 * (long)blockIdx.x + c] = v[c];
}

// ---- deviation layout (g planes float32, moment planes float64) ----------------------

// g := 0, M := fields: the state f = f^eq(fields) exactly.
__global__ __launch_bounds__(256) void fill_dev_kernel(const Inst *__restrict__ insts, int inst,
                                                       const double *__restrict__ fields, int half) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const size_t c = (size_t)y * I.nx + x, plane = (size_t)I.nx * I.ny;
    float *g = static_cast<float *>(I.f[half]);
    const size_t off = (size_t)y * I.fpitch + x;
    for (int q = 0; q < NQ; ++q) g[(size_t)q * I.fplane + off] = 0.0f;
    double *M = I.M[half];
    const size_t mo = (size_t)y * I.ppitch + x;
    for (int a = 0; a < 4; ++a) M[(size_t)a * I.mplane + mo] = fields[a * plane + c];
}

// Non-physical flag of the stored moments.
__global__ __launch_bounds__(256) void check_dev_kernel(const Inst *__restrict__ insts, int inst, int half) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const double *M = I.M[half];
    const size_t mo = (size_t)y * I.ppitch + x;
    if (nonphysical(I, M[mo], M[I.mplane + mo], M[2 * I.mplane + mo], M[3 * I.mplane + mo])) *I.flag = 1;
}

// (rho, ux, uy, T): the stored moments.
__global__ __launch_bounds__(256) void moments_dev_kernel(const Inst *__restrict__ insts, int inst, int half,
                                                          double *__restrict__ out) {
    const Inst &I = insts[inst];
    const int x = blockIdx.x * 16 + threadIdx.x % 16, y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= I.nx || y >= I.ny) return;
    const double *M = I.M[half];
    const size_t mo = (size_t)y * I.ppitch + x;
    const size_t c = (size_t)y * I.nx + x, plane = (size_t)I.nx * I.ny;
    for (int a = 0; a < 4; ++a) out[a * plane + c] = M[(size_t)a * I.mplane + mo];
}

// Totals of (n, jx, jy, E) of f = f^eq(M) + g: the moments of f^eq(M) in closed form plus
// those of g; fixed tree order as diag_kernel.
__global__ __launch_bounds__(256) void diag_dev_kernel(const Inst *__restrict__ insts, int inst, int half,
                                                       double *__restrict__ partials) {
    const Inst &I = insts[inst];
    __shared__ double red[4][kDiagBlock / 64];
    const long cell = (long)blockIdx.x * kDiagBlock + threadIdx.x;
    const long ncell = (long)I.nx * I.ny;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (cell < ncell) {
        const int x = (int)(cell % I.nx), y = (int)(cell / I.nx);
        const float *gin = static_cast<const float *>(I.f[half]);
        float g[NQ];
        const size_t off = (size_t)y * I.fpitch + x;
        static_for<0, NQ>([&](auto qc) { g[decltype(qc)::value] = gin[(size_t)decltype(qc)::value * I.fplane + off]; });
        double gn, gx, gy, gE;
        moments33_fast<0>(I, g, gn, gx, gy, gE);
        const double *M = I.M[half];
        const size_t mo = (size_t)y * I.ppitch + x;
        const double n = M[mo], ux = M[I.mplane + mo], uy = M[2 * I.mplane + mo], T = M[3 * I.mplane + mo];
        v[0] = n + gn;
        v[1] = n * ux + gx;
        v[2] = n * uy + gy;
        v[3] = n * (T + (ux * ux + uy * uy) / 2.0) + gE;
        if (nonphysical(I, n, ux, uy, T)) *I.flag = 1;
    }
    block_sum4(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partials[4 * (long)blockIdx.x + c] = v[c];
}

__global__ __launch_bounds__(kDiagBlock) void diag_final_kernel(const double *__restrict__ partials, int nparts,
                                                                double *__restrict__ sums) {
    // each thread sums a fixed strided subset in order, then block_sum4: deterministic
    __shared__ double red[4][kDiagBlock / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kDiagBlock)
        for (int c = 0; c < 4; ++c) v[c] = v[c] + partials[4 * (long)i + c];
    block_sum4(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) sums[c] = v[c];
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
template <class S, int SHAPE, int MODE>
static hipError_t launch_step_m(const Inst *insts, const Tile *tiles, int ntiles, int io, hipStream_t s) {
    constexpr int TX = kTileShapes[SHAPE].tx, TY = kTileShapes[SHAPE].ty;
    hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles, ntiles,
                       io);
    return hipGetLastError();
}

template <class S, int SHAPE>
static hipError_t launch_step_t(int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                                hipStream_t s) {
    if (kind == MODE_INTERIOR) return launch_step_m<S, SHAPE, MODE_INTERIOR>(insts, tiles, ntiles, io, s);
    if (kind == MODE_TUBE) return launch_step_m<S, SHAPE, MODE_TUBE>(insts, tiles, ntiles, io, s);
    return launch_step_m<S, SHAPE, MODE_EDGE>(insts, tiles, ntiles, io, s);
}

// Deviation layout: one kernel per tile kind, as for the other storages.
template <class S, int SHAPE>
static hipError_t launch_step_dev(int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                                  hipStream_t s) {
    constexpr int TX = kTileShapes[SHAPE].tx, TY = kTileShapes[SHAPE].ty;
    if (kind == MODE_INTERIOR)
        hipLaunchKernelGGL((step_kernel_dev<TX, TY, MODE_INTERIOR>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles,
                           ntiles, io);
    else if (kind == MODE_TUBE)
        hipLaunchKernelGGL((step_kernel_dev<TX, TY, MODE_TUBE>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles,
                           ntiles, io);
    else
        hipLaunchKernelGGL((step_kernel_dev<TX, TY, MODE_EDGE>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles,
                           ntiles, io);
    return hipGetLastError();
}

struct DevTag {};

template <class S, int SHAPE>
static hipError_t launch_step_any(int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                                  hipStream_t s) {
    if constexpr (std::is_same<S, DevTag>::value)
        return launch_step_dev<S, SHAPE>(kind, insts, tiles, ntiles, io, s);
    else
        return launch_step_t<S, SHAPE>(kind, insts, tiles, ntiles, io, s);
}

template <class S>
static hipError_t launch_step_p(int shape, int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                                hipStream_t s) {
    switch (shape) {
    case 0: return launch_step_any<S, 0>(kind, insts, tiles, ntiles, io, s);
    case 1: return launch_step_any<S, 1>(kind, insts, tiles, ntiles, io, s);
    case 2: return launch_step_any<S, 2>(kind, insts, tiles, ntiles, io, s);
    case 3: return launch_step_any<S, 3>(kind, insts, tiles, ntiles, io, s);
    case 4: return launch_step_any<S, 4>(kind, insts, tiles, ntiles, io, s);
    case 5: return launch_step_any<S, 5>(kind, insts, tiles, ntiles, io, s);
    case 6: return launch_step_any<S, 6>(kind, insts, tiles, ntiles, io, s);
    case 7: return launch_step_any<S, 7>(kind, insts, tiles, ntiles, io, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------------------------
// Bandwidth reference: every stored plane of the interior tiles copied from half `half`
// to the other half, one thread per cell as in the step, in the same tile order and
// XCD-aware remap, batches of planes in flight, non-temporal stores.  No halo, no moment
// planes, no arithmetic: the practical ceiling of the step's compulsory f traffic.
// ------------------------------------------------------------------------------------
template <class S, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void plane_copy_kernel(const Inst *__restrict__ insts,
                                                            const Tile *__restrict__ tiles, int ntiles, int half) {
    const Tile tile = tiles[xcd_remap(blockIdx.x, ntiles)];
    const Inst &I = insts[tile.inst];
    const int x = tile.x0 + (int)threadIdx.x % TX, y = tile.y0 + (int)threadIdx.x / TX;
    const GLOBAL_AS S *in = (const GLOBAL_AS S *)(I.f[half]) + ((size_t)y * I.fpitch + x);
    GLOBAL_AS S *out = (GLOBAL_AS S *)(I.f[1 - half]) + ((size_t)y * I.fpitch + x);
    constexpr int B = 11;  // planes in flight per thread (33 = 3 x 11)
    for (int q0 = 0; q0 < NQ; q0 += B) {
        S v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = in[(size_t)(q0 + k) * I.fplane];
#pragma unroll
        for (int k = 0; k < B; ++k) store_out(out + (size_t)(q0 + k) * I.fplane, v[k]);
    }
}

template <class S, int SHAPE>
static hipError_t launch_copy_s(const Inst *insts, const Tile *tiles, int ntiles, int half, hipStream_t s) {
    constexpr int TX = kTileShapes[SHAPE].tx, TY = kTileShapes[SHAPE].ty;
    hipLaunchKernelGGL((plane_copy_kernel<S, TX, TY>), dim3(ntiles), dim3(TX * TY), 0, s, insts, tiles, ntiles, half);
    return hipGetLastError();
}

template <class S>
static hipError_t launch_copy_p(int shape, const Inst *insts, const Tile *tiles, int ntiles, int half,
                                hipStream_t s) {
    switch (shape) {
    case 0: return launch_copy_s<S, 0>(insts, tiles, ntiles, half, s);
    case 1: return launch_copy_s<S, 1>(insts, tiles, ntiles, half, s);
    case 2: return launch_copy_s<S, 2>(insts, tiles, ntiles, half, s);
    case 3: return launch_copy_s<S, 3>(insts, tiles, ntiles, half, s);
    case 4: return launch_copy_s<S, 4>(insts, tiles, ntiles, half, s);
    case 5: return launch_copy_s<S, 5>(insts, tiles, ntiles, half, s);
    case 6: return launch_copy_s<S, 6>(insts, tiles, ntiles, half, s);
    case 7: return launch_copy_s<S, 7>(insts, tiles, ntiles, half, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_plane_copy(int prec, int shape, const Inst *insts, const Tile *tiles, int ntiles, int half,
                             hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    // the deviation layout's g planes are float32 like the float32 layout's f planes
    if (prec == PREC_F64) return launch_copy_p<double>(shape, insts, tiles, ntiles, half, s);
    return launch_copy_p<float>(shape, insts, tiles, ntiles, half, s);
}

hipError_t launch_step2(const Inst *insts, const Tile *tiles, int ntiles, int io, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    constexpr int TX = kTileShapes[kTwoStepShape].tx, TY = kTileShapes[kTwoStepShape].ty;
    hipLaunchKernelGGL((step2_kernel<TX, TY>), dim3(ntiles), dim3(step2_threads<TX, TY>()), 0, s, insts, tiles,
                       ntiles, io);
    return hipGetLastError();
}

hipError_t launch_step(int prec, int shape, int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                       hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (prec == PREC_F64) return launch_step_p<double>(shape, kind, insts, tiles, ntiles, io, s);
    if (prec == PREC_DEV) return launch_step_p<DevTag>(shape, kind, insts, tiles, ntiles, io, s);
    return launch_step_p<float>(shape, kind, insts, tiles, ntiles, io, s);
}

int tile_kind(int x0, int y0, int tx, int ty, int nx, int ny, int bc_y) {
    const bool xin = x0 >= 2 && x0 + tx + 2 <= nx;
    const bool yin = y0 >= 2 && y0 + ty + 2 <= ny;
    if (xin && yin) return MODE_INTERIOR;
    if (xin && ny == ty && y0 == 0 && bc_y == BC_PERIODIC) return MODE_TUBE;
    return MODE_EDGE;
}

static dim3 grid16(int nx, int ny) { return dim3((nx + 15) / 16, (ny + 15) / 16); }

hipError_t launch_fill(int prec, const Inst *insts, int inst, int nx, int ny, const double *fields, int half,
                       hipStream_t s) {
    if (prec == PREC_DEV)
        hipLaunchKernelGGL(fill_dev_kernel, grid16(nx, ny), dim3(256), 0, s, insts, inst, fields, half);
    else if (prec == PREC_F64)
        hipLaunchKernelGGL(fill_kernel<double>, grid16(nx, ny), dim3(256), 0, s, insts, inst, fields, half);
    else
        hipLaunchKernelGGL(fill_kernel<float>, grid16(nx, ny), dim3(256), 0, s, insts, inst, fields, half);
    return hipGetLastError();
}

hipError_t launch_derive(int prec, const Inst *insts, int inst, int nx, int ny, int half, hipStream_t s) {
    if (prec == PREC_DEV)
        hipLaunchKernelGGL(check_dev_kernel, grid16(nx, ny), dim3(256), 0, s, insts, inst, half);
    else if (prec == PREC_F64)
        hipLaunchKernelGGL(derive_kernel<double>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half);
    else
        hipLaunchKernelGGL(derive_kernel<float>, grid16(nx, ny), dim3(256), 0, s, insts, inst, half);
    return hipGetLastError();
}

hipError_t launch_bc_setup(int prec, Inst *insts, int inst, hipStream_t s) {
    if (prec == PREC_F64 || prec == PREC_DEV)
        hipLaunchKernelGGL(bc_setup_kernel<double>, dim3(1), dim3(64), 0, s, insts, inst);
    else
        hipLaunchKernelGGL(bc_setup_kernel<float>, dim3(1), dim3(64), 0, s, insts, inst);
    return hipGetLastError();
}

hipError_t launch_moments(int prec, const Inst *insts, int inst, int nx, int ny, int half, double *out,
                          hipStream_t s) {
    if (prec == PREC_DEV)
        hipLaunchKernelGGL(moments_dev_kernel, grid16(nx, ny), dim3(256), 0, s, insts, inst, half, out);
    else if (prec == PREC_F64)
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
    if (prec == PREC_DEV)
        hipLaunchKernelGGL(diag_dev_kernel, dim3(nb), dim3(kDiagBlock), 0, s, insts, inst, half, p);
    else if (prec == PREC_F64)
        hipLaunchKernelGGL(diag_kernel<double>, dim3(nb), dim3(kDiagBlock), 0, s, insts, inst, half, p);
    else
        hipLaunchKernelGGL(diag_kernel<float>, dim3(nb), dim3(kDiagBlock), 0, s, insts, inst, half, p);
    return hipGetLastError();
}

// Advances the step clock of the moving side segments (one per step, after the step).
// The pressure of the mirror image of each cell beside a reflecting side (a wall on the
// side or on its lower segment), from the cell's 33 values of half `half` summed in the
// mirrored order: the same values write_pressures gives.  Block (i, side, instance).
__global__ __launch_bounds__(256) void wall_pressure_kernel(const Inst *__restrict__ insts, int half) {
    const Inst &I = insts[blockIdx.z];
    const int side = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (!(I.bc[side] == BC_WALL || I.bclo[side] == BC_WALL)) return;
    if (i >= (side < 2 ? I.ny : I.nx)) return;
    const int x = side == 0 ? 0 : side == 1 ? I.nx - 1 : i;
    const int y = side == 2 ? 0 : side == 3 ? I.ny - 1 : i;
    const double *fin = static_cast<const double *>(I.f[half]);
    const size_t off = (size_t)y * I.fpitch + x;
    double f[NQ];
    static_for<0, NQ>([&](auto qc) { f[decltype(qc)::value] = fin[(size_t)decltype(qc)::value * I.fplane + off]; });
    double n, jx, jy, E, ux, uy, T, P;
    if (side < 2) moments_of<1>(I, f, n, jx, jy, E);
    else moments_of<2>(I, f, n, jx, jy, E);
    primitive(n, jx, jy, E, ux, uy, T, P);
    I.PW[half][side * I.wlen + i] = P;
}

hipError_t launch_wall_pressure(const Inst *insts, int k, int maxlen, int half, hipStream_t s) {
    hipLaunchKernelGGL(wall_pressure_kernel, dim3((maxlen + 255) / 256, 4, k), dim3(256), 0, s, insts, half);
    return hipGetLastError();
}

__global__ void tick_kernel(int64_t *clock) {
    if (threadIdx.x == 0) clock[0] = clock[0] + 1;
}

hipError_t launch_tick(int64_t *clock, hipStream_t s) {
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, s, clock);
    return hipGetLastError();
}

// Fixed scratch of the allocation-free diagnostics (fdlb_diag_noalloc): the per-block
// partial totals of launch_diag, then the four final sums.  Every block writes its own
// four partials and the final kernel writes the sums, so nothing needs clearing between
// calls.  Each GPU holds its own copy for the life of the process; host code must use
// the address diag_scratch_address returns, never the symbol itself.
static __device__ __align__(256) double scratch[4 * kDiagScratchParts + 4];

hipError_t diag_scratch_address(double **ptr) {
    return hipGetSymbolAddress(reinterpret_cast<void **>(ptr), HIP_SYMBOL(scratch));
}

hipError_t launch_diag_final(const double *partials, int nparts, double *sums, hipStream_t s) {
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kDiagBlock), 0, s, partials, nparts, sums);
    return hipGetLastError();
}

}  // namespace fdlb
