// fdlb_vn.hip -- von Neumann stability sweep of the scheme on the GPU (Sec. 4 of the paper,
// Eqs. gi_j_eq and pian_fki_eq).
//
// For a uniform equilibrium (n, ux, uy, T) and a Fourier mode exp(i k x) along x (phase
// phi = k dx), one step of Eq. (dis_eq1) multiplies the perturbation's 33 amplitudes by
//   G(phi) = (1 - dt/tau + L(phi)) I + (dt/tau) J,   J_ij = d f^eq_i / d f_j,
// where L(phi) collects lines I-IV of Eq. (dis_eq1) for velocity i (c = v_ix dt / dx):
//   line I    -(c/2)(e^{i phi} - e^{-i phi})                 = -i c sin(phi)
//   line II   (c^2/2)(e^{i phi} - 2 + e^{-i phi})             = c^2 (cos(phi) - 1)
//   line III  c(1 - c^2)/12 (e^{2i phi} - 2e^{i phi} + 2e^{-i phi} - e^{-2i phi})
//                                                             = i c(1 - c^2)/6 (sin(2 phi) - 2 sin(phi))
//   line IV   theta |kappa|(1 - |kappa|)/2 (e^{i phi} - 2 + e^{-i phi}), kappa = ux dt / dx,
// with the switching function frozen at theta (the analysis linearises about a uniform
// state, where Eq. (add4) would give zero).  J is the chain rule of Eq. (pian_fki_eq) through
// n = sum f, u = sum v f / n and T = sum |v - u|^2 f / (2 n), with the derivatives of the
// equilibrium of Eq. (feq_eq) and its weights F_k(T) of Eqs. (fk_eq1), (f0_eq) in closed form.
//
// G is strongly non-normal at high Mach number (entries of J ~ 1e5), so its eigenvalues are
// computed in double-double arithmetic (about 32 significant digits): a Householder
// reduction to Hessenberg form, then the single-shift QR algorithm with Wilkinson shifts and
// Givens rotations.  One 64-lane wavefront per matrix, the matrix in LDS.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/fdlb.h"

namespace fdlb_vn {

constexpr int N = 33;

// ---- double-double arithmetic (error-free transformations) ---------------------------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd mkdd(double a) { return {a, 0.0}; }
__device__ __forceinline__ dd operator+(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd operator-(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd operator-(dd a, dd b) { return a + (-b); }
__device__ __forceinline__ dd operator*(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd operator*(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd operator/(dd a, dd b) {
    // long division: three quotient digits
    const double q1 = a.hi / b.hi;
    dd r = a - b * q1;
    const double q2 = r.hi / b.hi;
    r = r - b * q2;
    const double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return q + mkdd(q3);
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
    if (!(a.hi > 0.0)) return mkdd(0.0);
    // one Newton step from the float64 root doubles its digits
    const double x = sqrt(a.hi);
    const dd xx = two_prod(x, x);
    const dd r = a - xx;
    return quick_two_sum(x, r.hi / (2.0 * x)) + mkdd(0.0);
}
__device__ __forceinline__ double to_d(dd a) { return a.hi + a.lo; }
__device__ __forceinline__ dd dd_abs(dd a) { return a.hi < 0.0 ? -a : a; }
__device__ __forceinline__ bool lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// sin and cos of x in double-double: Taylor series of x / 2^8, then eight angle doublings
__device__ void dd_sincos(double x, dd &s, dd &c) {
    const dd y = mkdd(ldexp(x, -8));
    const dd y2 = y * y;
    dd ts = y, tc = mkdd(1.0), term_s = y, term_c = mkdd(1.0);
    for (int k = 1; k <= 14; ++k) {
        term_s = -(term_s * y2) / mkdd((double)((2 * k) * (2 * k + 1)));
        term_c = -(term_c * y2) / mkdd((double)((2 * k - 1) * (2 * k)));
        ts = ts + term_s;
        tc = tc + term_c;
    }
    for (int k = 0; k < 8; ++k) {
        const dd s2 = (ts * tc) * 2.0;
        const dd c2 = mkdd(1.0) - (ts * ts) * 2.0;
        ts = s2;
        tc = c2;
    }
    s = ts;
    c = tc;
}

struct cdd {
    dd re, im;
};
__device__ __forceinline__ cdd operator+(cdd a, cdd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cdd operator-(cdd a, cdd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cdd operator*(cdd a, cdd b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cdd operator*(cdd a, dd b) { return {a.re * b, a.im * b}; }
__device__ __forceinline__ cdd conj(cdd a) { return {a.re, -a.im}; }
__device__ __forceinline__ dd norm2(cdd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ dd cabs(cdd a) { return dd_sqrt(norm2(a)); }
__device__ __forceinline__ dd cabs1(cdd a) { return dd_abs(a.re) + dd_abs(a.im); }
__device__ __forceinline__ cdd cdiv(cdd a, cdd b) {
    const dd d = norm2(b);
    const cdd t = a * conj(b);
    return {t.re / d, t.im / d};
}
__device__ __forceinline__ cdd csqrt(cdd z) {
    // principal root: sqrt((|z| + re) / 2) + i sign(im) sqrt((|z| - re) / 2)
    const dd r = cabs(z);
    dd a = dd_sqrt((r + z.re) * 0.5);
    dd b = dd_sqrt((r - z.re) * 0.5);
    if (z.im.hi < 0.0) b = -b;
    return {a, b};
}

// ---- the amplification matrix ----------------------------------------------------------
// Velocity q: 0 rest; 1 + 8k + (i - 1) speed k, direction i pi/4 (Eq. dvm_eq_1), with the
// exact components 0 and +-1 on the axes and sqrt(2)/2 on the diagonals.
__device__ void velocity(const fdlb_vn_case &cs, int q, dd r2, dd &vx, dd &vy) {
    if (q == 0) {
        vx = vy = mkdd(0.0);
        return;
    }
    const int k = (q - 1) / 8, i = (q - 1) % 8 + 1;
    const double v = cs.v[k];
    const dd d = r2 * v;  // v sqrt(2)/2
    const dd z = mkdd(0.0), a = mkdd(v);
    switch (i) {
    case 1: vx = d; vy = d; break;
    case 2: vx = z; vy = a; break;
    case 3: vx = -d; vy = d; break;
    case 4: vx = -a; vy = z; break;
    case 5: vx = -d; vy = -d; break;
    case 6: vx = z; vy = -a; break;
    case 7: vx = d; vy = -d; break;
    default: vx = a; vy = z; break;
    }
}

// F_k(T) and dF_k/dT for k = 0..4 (Eqs. fk_eq1, f0_eq, kl_eq: the index k + l is cyclic)
__device__ void weights(const fdlb_vn_case &cs, dd T, dd F[5], dd dF[5]) {
    dd sF = mkdd(0.0), sdF = mkdd(0.0);
    const dd T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    for (int k = 0; k < 4; ++k) {
        const dd vk2 = mkdd(cs.v[k]) * cs.v[k];
        const dd a = mkdd(cs.v[(k + 1) % 4]) * cs.v[(k + 1) % 4];
        const dd b = mkdd(cs.v[(k + 2) % 4]) * cs.v[(k + 2) % 4];
        const dd d = mkdd(cs.v[(k + 3) % 4]) * cs.v[(k + 3) % 4];
        const dd A = (a + b + d) * 6.0, B = a * b + b * d + d * a, C = (a * b * d) * 0.25;
        const dd den = vk2 * (vk2 - a) * (vk2 - b) * (vk2 - d);
        F[k + 1] = (T4 * 48.0 - A * T3 + B * T2 - C * T) / den;
        dF[k + 1] = (T3 * 192.0 - A * T2 * 3.0 + B * T * 2.0 - C) / den;
        sF = sF + F[k + 1];
        sdF = sdF + dF[k + 1];
    }
    F[0] = mkdd(1.0) - sF * 8.0;
    dF[0] = -(sdF * 8.0);
}

// Row i of J = d f^eq / d f and the diagonal of G(phi) into H (LDS, row-major).
__device__ void build_row(const fdlb_vn_case &cs, double phi, int i, cdd *H) {
    const dd r2 = dd_sqrt(mkdd(2.0)) * 0.5;
    const dd n = mkdd(cs.rho), ux = mkdd(cs.ux), uy = mkdd(cs.uy), T = mkdd(cs.T);
    dd F[5], dF[5];
    weights(cs, T, F, dF);
    const int k = i == 0 ? 0 : 1 + (i - 1) / 8;
    dd vxi, vyi;
    velocity(cs, i, r2, vxi, vyi);
    const dd u2 = ux * ux + uy * uy;
    const dd iT = mkdd(1.0) / T;
    const dd h = mkdd(1.0) - u2 * iT * 0.5;
    const dd c0 = h + (u2 * u2) * (iT * iT) * 0.125;
    const dd c1 = h * iT;
    const dd c2 = h * (iT * iT) * 0.5;
    const dd c3 = (iT * iT * iT) / mkdd(6.0);
    const dd c4 = (iT * iT * iT * iT) / mkdd(24.0);
    const dd s = vxi * ux + vyi * uy;
    const dd P = c0 + c1 * s + c2 * (s * s) + c3 * (s * s * s) + c4 * (s * s * s * s);
    // dP/ds and dP/d(u^2) at fixed T; dP/dT at fixed u
    const dd Ps = c1 + c2 * s * 2.0 + c3 * (s * s) * 3.0 + c4 * (s * s * s) * 4.0;
    const dd c0u = -(iT * 0.5) + u2 * (iT * iT) * 0.25;
    const dd c1u = -((iT * iT) * 0.5);
    const dd c2u = -((iT * iT * iT) * 0.25);
    const dd Pu2 = c0u + c1u * s + c2u * (s * s);
    const dd hT = u2 * (iT * iT) * 0.5;
    const dd c0T = hT - (u2 * u2) * (iT * iT * iT) * 0.25;
    const dd c1T = hT * iT - h * (iT * iT);
    const dd c2T = hT * (iT * iT) * 0.5 - h * (iT * iT * iT);
    const dd c3T = -((iT * iT * iT * iT) * 0.5);
    const dd c4T = -((iT * iT * iT * iT * iT) / mkdd(6.0));
    const dd PT = c0T + c1T * s + c2T * (s * s) + c3T * (s * s * s) + c4T * (s * s * s * s);
    const dd dn = F[k] * P;
    const dd dux = n * F[k] * (Ps * vxi + Pu2 * ux * 2.0);
    const dd duy = n * F[k] * (Ps * vyi + Pu2 * uy * 2.0);
    const dd dT = n * (dF[k] * P + F[k] * PT);
    const dd dtau = mkdd(cs.dt) / mkdd(cs.tau);
    const dd in = mkdd(1.0) / n;
    for (int j = 0; j < N; ++j) {
        dd vxj, vyj;
        velocity(cs, j, r2, vxj, vyj);
        const dd ex = vxj - ux, ey = vyj - uy;
        const dd Jij = dn + dux * ex * in + duy * ey * in + dT * ((ex * ex + ey * ey) * 0.5 - T) * in;
        H[i * N + j] = {dtau * Jij, mkdd(0.0)};
    }
    // the diagonal: lines I-IV for an x wave, and 1 - dt/tau
    dd sn, cn, s2n, c2n;
    dd_sincos(phi, sn, cn);
    s2n = (sn * cn) * 2.0;
    c2n = mkdd(1.0) - (sn * sn) * 2.0;
    (void)c2n;
    const dd c = vxi * cs.dt / mkdd(cs.dx);
    const dd kap = dd_abs(ux * cs.dt / mkdd(cs.dx));
    const dd av = mkdd(cs.theta) * kap * (mkdd(1.0) - kap) * 0.5;
    dd re = mkdd(1.0) - dtau, im = mkdd(0.0);
    if (cs.lines & 1) im = im - c * sn;
    if (cs.lines & 2) re = re + (c * c) * (cn - mkdd(1.0));
    if (cs.lines & 4) im = im + c * (mkdd(1.0) - c * c) / mkdd(6.0) * (s2n - sn * 2.0);
    if (cs.lines & 8) re = re + av * (cn - mkdd(1.0)) * 2.0;
    H[i * N + i] = H[i * N + i] + cdd{re, im};
}

// ---- eigenvalues ---------------------------------------------------------------------------
struct VnSmem {
    cdd H[N * N];
    cdd v[N];         // Householder vector
    cdd w[N];         // its products with H
    cdd rot[2];       // Givens rotation (c in rot[0].re, s in rot[1])
    cdd mu;
    int state[4];     // lo, hi, done flag, failure flag
};

// Householder reduction of H to upper Hessenberg form (similarity: same eigenvalues).
__device__ void hessenberg(VnSmem &sm) {
    const int t = threadIdx.x;
    for (int k = 0; k < N - 2; ++k) {
        if (t == 0) {
            // x = H[k+1.., k]; v = x + e^{i arg x0} |x| e1, normalised
            dd nx2 = mkdd(0.0);
            for (int i = k + 1; i < N; ++i) nx2 = nx2 + norm2(sm.H[i * N + k]);
            const dd nx = dd_sqrt(nx2);
            const cdd x0 = sm.H[(k + 1) * N + k];
            const dd a0 = cabs(x0);
            cdd ph = {mkdd(1.0), mkdd(0.0)};
            if (a0.hi > 0.0) ph = {x0.re / a0, x0.im / a0};
            for (int i = 0; i < N; ++i) sm.v[i] = {mkdd(0.0), mkdd(0.0)};
            for (int i = k + 1; i < N; ++i) sm.v[i] = sm.H[i * N + k];
            sm.v[k + 1] = sm.v[k + 1] + ph * nx;
            dd nv2 = mkdd(0.0);
            for (int i = k + 1; i < N; ++i) nv2 = nv2 + norm2(sm.v[i]);
            const dd inv = nv2.hi > 0.0 ? mkdd(1.0) / dd_sqrt(nv2) : mkdd(0.0);
            for (int i = k + 1; i < N; ++i) sm.v[i] = sm.v[i] * inv;
        }
        __syncthreads();
        // left: H = H - 2 v (v^H H), one column per lane
        if (t < N) {
            cdd s = {mkdd(0.0), mkdd(0.0)};
            for (int i = k + 1; i < N; ++i) s = s + conj(sm.v[i]) * sm.H[i * N + t];
            for (int i = k + 1; i < N; ++i) sm.H[i * N + t] = sm.H[i * N + t] - sm.v[i] * s * mkdd(2.0);
        }
        __syncthreads();
        // right: H = H - 2 (H v) v^H, one row per lane
        if (t < N) {
            cdd s = {mkdd(0.0), mkdd(0.0)};
            for (int j = k + 1; j < N; ++j) s = s + sm.H[t * N + j] * sm.v[j];
            for (int j = k + 1; j < N; ++j) sm.H[t * N + j] = sm.H[t * N + j] - s * conj(sm.v[j]) * mkdd(2.0);
        }
        __syncthreads();
    }
}

// Single-shift QR on the Hessenberg matrix; returns the largest |eigenvalue| (NaN if the
// iteration does not converge).
__device__ double spectral_radius(VnSmem &sm) {
    const int t = threadIdx.x;
    const dd eps = mkdd(ldexp(1.0, -104));
    dd best = mkdd(0.0);
    if (t == 0) {
        sm.state[1] = N - 1;
        sm.state[3] = 0;
    }
    __syncthreads();
    int iter = 0, total = 0;
    while (true) {
        // thread 0: deflation and shift
        if (t == 0) {
            int hi = sm.state[1];
            int l = hi;
            sm.state[2] = 0;
            if (hi < 0) {
                sm.state[2] = 2;  // all eigenvalues found
            } else {
                while (l > 0) {
                    const dd sub = cabs1(sm.H[l * N + l - 1]);
                    const dd diag = cabs1(sm.H[l * N + l]) + cabs1(sm.H[(l - 1) * N + l - 1]);
                    if (!lt(diag * eps, sub)) break;
                    --l;
                }
                if (l > 0) sm.H[l * N + l - 1] = {mkdd(0.0), mkdd(0.0)};
                if (l == hi) {
                    const dd a = cabs(sm.H[hi * N + hi]);
                    if (lt(best, a)) best = a;
                    sm.state[1] = hi - 1;
                    sm.state[2] = 1;  // one eigenvalue deflated
                } else {
                    sm.state[0] = l;
                    const cdd a = sm.H[(hi - 1) * N + hi - 1], b = sm.H[(hi - 1) * N + hi];
                    const cdd c = sm.H[hi * N + hi - 1], d = sm.H[hi * N + hi];
                    cdd mu;
                    if (iter > 0 && iter % 12 == 0) {
                        // exceptional shift
                        mu = d + cdd{cabs1(c) * 0.75, mkdd(0.0)};
                    } else {
                        // Wilkinson: the eigenvalue of the trailing 2 x 2 block closer to d
                        const cdd half = (a - d) * mkdd(0.5);
                        const cdd disc = csqrt(half * half + b * c);
                        const cdd m = (a + d) * mkdd(0.5);
                        const cdd e1 = m + disc, e2 = m - disc;
                        mu = lt(cabs1(e1 - d), cabs1(e2 - d)) ? e1 : e2;
                    }
                    sm.mu = mu;
                }
            }
        }
        __syncthreads();
        const int flag = sm.state[2];
        if (flag == 2) break;
        if (flag == 1) {
            iter = 0;
            __syncthreads();
            continue;
        }
        if (++total > 60 * N) {
            if (t == 0) sm.state[3] = 1;
            __syncthreads();
            break;
        }
        ++iter;
        const int l = sm.state[0], hi = sm.state[1];
        // one QR sweep over rows / columns l..hi (bulge chase)
        for (int k = l; k < hi; ++k) {
            if (t == 0) {
                cdd x, y;
                if (k == l) {
                    x = sm.H[l * N + l] - sm.mu;
                    y = sm.H[(l + 1) * N + l];
                } else {
                    x = sm.H[k * N + k - 1];
                    y = sm.H[(k + 1) * N + k - 1];
                }
                const dd ax = cabs(x), r = dd_sqrt(norm2(x) + norm2(y));
                dd cr;
                cdd s;
                if (r.hi == 0.0) {
                    cr = mkdd(1.0);
                    s = {mkdd(0.0), mkdd(0.0)};
                } else if (ax.hi == 0.0) {
                    cr = mkdd(0.0);
                    s = conj(y) * (mkdd(1.0) / cabs(y));
                } else {
                    cr = ax / r;
                    const cdd ph = {x.re / ax, x.im / ax};
                    s = ph * conj(y) * (mkdd(1.0) / r);
                }
                sm.rot[0] = {cr, mkdd(0.0)};
                sm.rot[1] = s;
            }
            __syncthreads();
            const dd cr = sm.rot[0].re;
            const cdd s = sm.rot[1];
            // rows k, k+1 over columns max(l, k-1)..hi
            const int j = t + (k > l ? k - 1 : l);
            if (j <= hi) {
                const cdd hk = sm.H[k * N + j], hk1 = sm.H[(k + 1) * N + j];
                sm.H[k * N + j] = hk * cr + s * hk1;
                sm.H[(k + 1) * N + j] = hk1 * cr - conj(s) * hk;
            }
            __syncthreads();
            // columns k, k+1 over rows l..min(k+2, hi)
            const int i = t + l;
            if (i <= (k + 2 < hi ? k + 2 : hi)) {
                const cdd hk = sm.H[i * N + k], hk1 = sm.H[i * N + k + 1];
                sm.H[i * N + k] = hk * cr + hk1 * conj(s);
                sm.H[i * N + k + 1] = hk1 * cr - hk * s;
            }
            __syncthreads();
        }
    }
    if (sm.state[3]) return __builtin_nan("");
    return to_d(best);
}

__global__ __launch_bounds__(64) void vn_kernel(const fdlb_vn_case *__restrict__ cases, int ncases,
                                                const double *__restrict__ phis, int nphi, double *__restrict__ out,
                                                double *__restrict__ gout) {
    __shared__ VnSmem sm;
    const int m = blockIdx.x, c = m / nphi, p = m % nphi;
    if (c >= ncases) return;
    const fdlb_vn_case cs = cases[c];
    if (threadIdx.x < N) build_row(cs, phis[p], threadIdx.x, sm.H);
    __syncthreads();
    if (gout) {
        // the matrix itself (re hi, re lo, im hi, im lo per entry)
        for (int e = threadIdx.x; e < N * N; e += 64) {
            double *o = gout + ((size_t)m * N * N + e) * 4;
            o[0] = sm.H[e].re.hi;
            o[1] = sm.H[e].re.lo;
            o[2] = sm.H[e].im.hi;
            o[3] = sm.H[e].im.lo;
        }
        return;
    }
    hessenberg(sm);
    const double r = spectral_radius(sm);
    if (threadIdx.x == 0) out[m] = r;
}

}  // namespace fdlb_vn

namespace {
fdlb_status vn_run(const fdlb_vn_case *cases, int32_t ncases, const double *phis, int32_t nphi, double *radius,
                   double *matrix, void *stream) {
    if (!cases || !phis || ncases < 1 || nphi < 1 || (!radius && !matrix)) return FDLB_EINVAL;
    if ((int64_t)ncases * nphi > (int64_t)1 << 24) return FDLB_EINVAL;
    for (int i = 0; i < ncases; ++i) {
        const fdlb_vn_case &c = cases[i];
        if (!(c.rho > 0) || !(c.T > 0) || !(c.dx > 0) || !(c.dt > 0) || !(c.tau > 0)) return FDLB_EINVAL;
        if (c.lines < 0 || c.lines > 15) return FDLB_EINVAL;
        for (int k = 0; k < 4; ++k) {
            if (!(c.v[k] > 0)) return FDLB_EINVAL;
            for (int l = 0; l < k; ++l)
                if (c.v[k] == c.v[l]) return FDLB_EINVAL;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nm = (size_t)ncases * nphi;
    const size_t nmat = matrix ? nm * fdlb_vn::N * fdlb_vn::N * 4 : 0;
    fdlb_vn_case *dc = nullptr;
    double *dp = nullptr, *dr = nullptr, *dg = nullptr;
    fdlb_status st = FDLB_OK;
    hipError_t e;
    if ((e = hipMalloc(&dc, sizeof(fdlb_vn_case) * ncases)) != hipSuccess ||
        (e = hipMalloc(&dp, sizeof(double) * nphi)) != hipSuccess ||
        (e = hipMalloc(&dr, sizeof(double) * nm)) != hipSuccess ||
        (nmat && (e = hipMalloc(&dg, sizeof(double) * nmat)) != hipSuccess))
        st = e == hipErrorOutOfMemory ? FDLB_ENOMEM : FDLB_EDEVICE;
    if (st == FDLB_OK &&
        ((e = hipMemcpyAsync(dc, cases, sizeof(fdlb_vn_case) * ncases, hipMemcpyHostToDevice, s)) != hipSuccess ||
         (e = hipMemcpyAsync(dp, phis, sizeof(double) * nphi, hipMemcpyHostToDevice, s)) != hipSuccess))
        st = FDLB_EDEVICE;
    if (st == FDLB_OK) {
        hipLaunchKernelGGL(fdlb_vn::vn_kernel, dim3((unsigned)nm), dim3(64), 0, s, dc, ncases, dp, nphi, dr, dg);
        if (hipGetLastError() != hipSuccess) st = FDLB_EDEVICE;
    }
    if (st == FDLB_OK && radius &&
        hipMemcpyAsync(radius, dr, sizeof(double) * nm, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = FDLB_EDEVICE;
    if (st == FDLB_OK && matrix &&
        hipMemcpyAsync(matrix, dg, sizeof(double) * nmat, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = FDLB_EDEVICE;
    if (st == FDLB_OK && hipStreamSynchronize(s) != hipSuccess) st = FDLB_EDEVICE;
    if (dc) (void)hipFree(dc);
    if (dp) (void)hipFree(dp);
    if (dr) (void)hipFree(dr);
    if (dg) (void)hipFree(dg);
    return st;
}
}  // namespace

extern "C" {

fdlb_status fdlb_vn_sweep(const fdlb_vn_case *cases, int32_t ncases, const double *phis, int32_t nphi,
                          double *radius, void *stream) {
    if (!radius) return FDLB_EINVAL;
    return vn_run(cases, ncases, phis, nphi, radius, nullptr, stream);
}

fdlb_status fdlb_vn_matrix(const fdlb_vn_case *cs, double phi, double *matrix, void *stream) {
    if (!matrix) return FDLB_EINVAL;
    return vn_run(cs, 1, &phi, 1, nullptr, matrix, stream);
}

}  // extern "C"
