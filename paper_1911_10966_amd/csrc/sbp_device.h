// Device helpers shared by the residual kernels and their vector-Jacobian products: reciprocal,
// log-mean series, node primitives, the two-point fluxes contracted with a metric vector, the
// viscous flux in entropy variables, and block/index mappings.
#pragma once

#include "sbp_internal.h"

#include <math.h>

namespace sbp {
namespace {

constexpr int NT_OF(int nodes) { return ((nodes + 63) / 64) * 64; }

// Reciprocal: hardware estimate refined by two Newton steps (a few ulp; no IEEE fixup needed
// for the strictly positive, finite operands used here).
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Square root of a strictly positive, normal operand (a metric norm, a sound speed squared): the
// hardware reciprocal square root refined by Goldschmidt's iteration and two Newton corrections
// (about 1 ulp), without the scaling and special-case handling of the general square root.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// A polynomial coefficient held in scalar registers: the empty asm statement makes the value opaque
// to constant folding, so each Horner step below is one v_fma_f64 with a scalar addend (as an
// immediate the compiler copies every coefficient into vector registers, two extra vector moves
// per step).
__device__ __forceinline__ double sreg(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// With z = (a-b)/(a+b) and u = z^2:  log(a/b) = 2 artanh z = 2 z F(u),  F(u) = sum_k u^k/(2k+1),
// so the logarithmic mean is (a+b)/(2 F(u)) and its inverse 2 F(u)/(a+b).  For u < 1e-2 the
// series below (F through u^7, G = 1/F through u^7) are accurate to < 1e-17 relative.
__device__ __forceinline__ double series_F(double u) {
    double r = sreg(1.0 / 15.0);
    r = fma(r, u, sreg(1.0 / 13.0));
    r = fma(r, u, sreg(1.0 / 11.0));
    r = fma(r, u, sreg(1.0 / 9.0));
    r = fma(r, u, sreg(1.0 / 7.0));
    r = fma(r, u, sreg(1.0 / 5.0));
    r = fma(r, u, sreg(1.0 / 3.0));
    return fma(r, u, 1.0);
}
__device__ __forceinline__ double series_G(double u) {
    // coefficients of 1/F(u): g_k = -sum_{i=1..k} g_{k-i}/(2i+1), g_0 = 1
    double r = sreg(-25865068.0 / 1915538625.0);
    r = fma(r, u, sreg(-10719068.0 / 638512875.0));
    r = fma(r, u, sreg(-10196.0 / 467775.0));
    r = fma(r, u, sreg(-428.0 / 14175.0));
    r = fma(r, u, sreg(-44.0 / 945.0));
    r = fma(r, u, sreg(-4.0 / 45.0));
    r = fma(r, u, sreg(-1.0 / 3.0));
    return fma(r, u, 1.0);
}

constexpr double LOGMEAN_U = 1e-2;

struct Node {
    double rho, u1, u2, u3, beta, lrho, lbeta, k;  // beta = rho / (2P) = 1/(2RT), k = |U|^2
};

__device__ __forceinline__ void primitives(const double q[5], double gm1, Node &n, double &P,
                                           bool &ok) {
    n.rho = q[0];
    const double ir = rcp(q[0]);
    n.u1 = q[1] * ir;
    n.u2 = q[2] * ir;
    n.u3 = q[3] * ir;
    n.k = n.u1 * n.u1 + n.u2 * n.u2 + n.u3 * n.u3;
    P = gm1 * (q[4] - 0.5 * q[0] * n.k);
    ok = (q[0] > 0.0) && (P > 0.0) && isfinite(q[4]) && isfinite(n.k);
    n.beta = ok ? 0.5 * q[0] * rcp(P) : 1.0;
    n.lrho = ok ? log(q[0]) : 0.0;
    n.lbeta = ok ? log(n.beta) : 0.0;
}

// Primitives of a neighbour node without the logarithms (see flux_n<FLUX, true>); ir = 1/rho.
__device__ __forceinline__ void primitives_nolog(const double q[5], double gm1, Node &n, double &P,
                                                 double &ir) {
    n.rho = q[0];
    ir = rcp(q[0]);
    n.u1 = q[1] * ir;
    n.u2 = q[2] * ir;
    n.u3 = q[3] * ir;
    n.k = n.u1 * n.u1 + n.u2 * n.u2 + n.u3 * n.u3;
    P = gm1 * (q[4] - 0.5 * q[0] * n.k);
    n.beta = 0.5 * q[0] * rcp(P);
    n.lrho = 0.0;
    n.lbeta = 0.0;
}
__device__ __forceinline__ void primitives_nolog(const double q[5], double gm1, Node &n, double &P) {
    double ir;
    primitives_nolog(q, gm1, n, P, ir);
}

// Nodal inviscid flux (eq. ns_iflux) contracted with (n0, n1, n2): [rho U_n, rho U_n U + P n,
// U_n (rho E + P)].
__device__ __forceinline__ void euler_flux_n(const Node &a, double P, double rhoE, double n0,
                                             double n1, double n2, double f[5]) {
    const double un = a.u1 * n0 + a.u2 * n1 + a.u3 * n2;
    const double m = a.rho * un;
    f[0] = m;
    f[1] = fma(m, a.u1, P * n0);
    f[2] = fma(m, a.u2, P * n1);
    f[3] = fma(m, a.u3, P * n2);
    f[4] = un * (rhoE + P);
}

// Two-point flux F#(a, b) contracted with the vector (n0, n1, n2).
// FLUX 0: Chandrashekar (entropy conservative), 1: central, 2: Kennedy-Gruber; 3 (standard DC)
// uses the central flux at interfaces.
// LAZY: b.lrho and b.lbeta are not set; they are computed only in the (rare) direct branch.
template <int FLUX, bool LAZY = false>
__device__ __forceinline__ void flux_n(const Node &a, const Node &b, double n0, double n1, double n2,
                                       double gm1, double f[5]) {
    const double ub1 = 0.5 * (a.u1 + b.u1), ub2 = 0.5 * (a.u2 + b.u2), ub3 = 0.5 * (a.u3 + b.u3);
    const double un = ub1 * n0 + ub2 * n1 + ub3 * n2;
    if constexpr (FLUX == 0) {
        const double sr = a.rho + b.rho, dr = a.rho - b.rho;
        const double sb = a.beta + b.beta, db = a.beta - b.beta;
        const double irb = rcp(sr * sb);  // one reciprocal for 1/(rho_i + rho_j), 1/(beta_i + beta_j)
        const double isr = sb * irb;
        const double isb = sr * irb;
        const double zr = dr * isr, ur = zr * zr;
        double rho_hat;
        if (ur < LOGMEAN_U) rho_hat = 0.5 * sr * series_G(ur);
        else rho_hat = dr * rcp(a.lrho - (LAZY ? log(b.rho) : b.lrho));
        const double zb = db * isb, ub = zb * zb;
        double ibeta_hat;
        if (ub < LOGMEAN_U) ibeta_hat = 2.0 * isb * series_F(ub);
        else ibeta_hat = (a.lbeta - (LAZY ? log(b.beta) : b.lbeta)) * rcp(db);
        const double pt = 0.5 * sr * isb;  // rho_bar / (2 beta_bar)
        const double fr = rho_hat * un;
        f[0] = fr;
        f[1] = fma(fr, ub1, pt * n0);
        f[2] = fma(fr, ub2, pt * n1);
        f[3] = fma(fr, ub3, pt * n2);
        const double kb = 0.5 * (a.k + b.k);
        const double ubsq = ub1 * ub1 + ub2 * ub2 + ub3 * ub3;
        f[4] = fma(fr, (0.5 / gm1) * ibeta_hat - 0.5 * kb + ubsq, pt * un);
    } else {
        // pressures and specific total energies from the staged node data
        const double Pa = 0.5 * a.rho / a.beta, Pb = 0.5 * b.rho / b.beta;
        if constexpr (FLUX == 1 || FLUX == 3) {
            const double una = a.u1 * n0 + a.u2 * n1 + a.u3 * n2;
            const double unb = b.u1 * n0 + b.u2 * n1 + b.u3 * n2;
            const double ma = a.rho * una, mb = b.rho * unb;
            const double Ha = (Pa / gm1 + 0.5 * a.rho * a.k + Pa) / a.rho;
            const double Hb = (Pb / gm1 + 0.5 * b.rho * b.k + Pb) / b.rho;
            f[0] = 0.5 * (ma + mb);
            f[1] = 0.5 * (ma * a.u1 + mb * b.u1 + (Pa + Pb) * n0);
            f[2] = 0.5 * (ma * a.u2 + mb * b.u2 + (Pa + Pb) * n1);
            f[3] = 0.5 * (ma * a.u3 + mb * b.u3 + (Pa + Pb) * n2);
            f[4] = 0.5 * (ma * Ha + mb * Hb);
        } else {
            const double rb = 0.5 * (a.rho + b.rho), Pbar = 0.5 * (Pa + Pb);
            const double Ea = Pa / (gm1 * a.rho) + 0.5 * a.k, Eb = Pb / (gm1 * b.rho) + 0.5 * b.k;
            const double fr = rb * un;
            f[0] = fr;
            f[1] = fr * ub1 + Pbar * n0;
            f[2] = fr * ub2 + Pbar * n1;
            f[3] = fr * ub3 + Pbar * n2;
            f[4] = fr * 0.5 * (Ea + Eb) + Pbar * un;
        }
    }
}

// Chandrashekar flux contracted with (n0, n1, n2) for the volume pair loop, from node data held as
// halves: rho/2, U/2 and |U|^2/4 (beta and the logarithms in full).  A sum of two halves is the
// arithmetic mean, exactly (scaling by 2 commutes with rounding), and every other quantity below is
// the one of flux_n<0> up to an exact power-of-2 factor, so the result equals flux_n<0> for the full
// values bit for bit, with six multiplications by 1/2 and one doubling fewer.  igm1 = 1/(gamma-1).
__device__ __forceinline__ void flux_pair_half(const Node &a, const Node &b, double n0, double n1,
                                               double n2, double igm1, double f[5]) {
    const double ub1 = a.u1 + b.u1, ub2 = a.u2 + b.u2, ub3 = a.u3 + b.u3;
    const double un = ub1 * n0 + ub2 * n1 + ub3 * n2;
    const double rb = a.rho + b.rho, dr = a.rho - b.rho;  // mean density, half the difference
    const double sb = a.beta + b.beta, db = a.beta - b.beta;
    const double irb = rcp(rb * sb);
    const double isr = sb * irb;  // 1 / mean density
    const double isb = rb * irb;  // 1 / (beta_i + beta_j)
    const double zr = dr * isr, ur = zr * zr;
    double rho_hat;
    if (ur < LOGMEAN_U) rho_hat = rb * series_G(ur);
    else rho_hat = (dr + dr) * rcp(a.lrho - b.lrho);
    const double zb = db * isb, ub = zb * zb;
    double ib;  // half the inverse logarithmic mean of beta
    if (ub < LOGMEAN_U) ib = isb * series_F(ub);
    else ib = (0.5 * (a.lbeta - b.lbeta)) * rcp(db);
    const double pt = rb * isb;  // rho_bar / (2 beta_bar)
    const double fr = rho_hat * un;
    f[0] = fr;
    f[1] = fma(fr, ub1, pt * n0);
    f[2] = fma(fr, ub2, pt * n1);
    f[3] = fma(fr, ub3, pt * n2);
    const double kh = a.k + b.k;  // half the mean of |U|^2
    const double ubsq = ub1 * ub1 + ub2 * ub2 + ub3 * ub3;
    f[4] = fma(fr, igm1 * ib - kh + ubsq, pt * un);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Map dispatch
// slot b to a virtual block so that every XCD walks one contiguous range of elements: face
// neighbours of an element are then mostly resident in the same L2.
__device__ __forceinline__ long long xcd_block(long long b, long long B) {
    constexpr long long X = 8;
    const long long per = B / X, rem = B % X;
    const long long x = b % X, slot = b / X;
    return x * per + (x < rem ? x : rem) + slot;
}

// Uncontracted viscous flux F^V_m[c] (m = 0..2; c = 0..2 momentum, 3 energy) from the
// entropy-variable gradients g[j][c] = dW_{c+1}/dx_j: stresses of eq. tau with
// dU_k = T (dW_{k+1} + U_k dW_5), heat flux +kappa dT/dx_m with dT = T^2 dW_5.
__device__ __forceinline__ void visc_flux_full(const double g[3][4], double u1, double u2, double u3,
                                               double T, double mu, double kap, double F[3][4]) {
    const double u[3] = {u1, u2, u3};
    double du[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) du[k][j] = T * fma(u[k], g[j][3], g[j][k]);
    const double div23 = (2.0 / 3.0) * (du[0][0] + du[1][1] + du[2][2]);
    const double T2k = kap * T * T;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
        for (int i = 0; i < 3; ++i) F[m][i] = mu * (du[i][m] + du[m][i] - (i == m ? div23 : 0.0));
        F[m][3] = fma(F[m][0], u[0], fma(F[m][1], u[1], fma(F[m][2], u[2], T2k * g[m][3])));
    }
}

// sum_m n_m F^V_m for the rank-one gradient g_j = n_j dw / J (the interior-penalty term):
// dU = v n^T / J with v_k = T (dw_k + U_k dw_5), which gives momentum (mu/J)(|n|^2 v + (v.n) n / 3)
// and energy U . momentum + kappa T^2 |n|^2 dw_5 / J.
__device__ __forceinline__ void visc_flux_rank1(double n0, double n1, double n2, double iJ,
                                                const double dw[4], double u1, double u2, double u3,
                                                double T, double mu, double kap, double out[4]) {
    const double v0 = T * fma(u1, dw[3], dw[0]);
    const double v1 = T * fma(u2, dw[3], dw[1]);
    const double v2 = T * fma(u3, dw[3], dw[2]);
    const double nn = n0 * n0 + n1 * n1 + n2 * n2;
    const double vn = v0 * n0 + v1 * n1 + v2 * n2;
    const double c1 = mu * iJ * nn, c2 = mu * iJ * vn * (1.0 / 3.0);
    out[0] = fma(c1, v0, c2 * n0);
    out[1] = fma(c1, v1, c2 * n1);
    out[2] = fma(c1, v2, c2 * n2);
    out[3] = fma(u1, out[0], fma(u2, out[1], fma(u3, out[2], kap * T * T * nn * iJ * dw[3])));
}

template <int N>
__device__ __forceinline__ int tangential_index(int l, int i1, int i2, int i3) {
    return l == 0 ? i2 + N * i3 : (l == 1 ? i1 + N * i3 : i1 + N * i2);
}


__device__ __forceinline__ int find_problem(const long long *start, int n, long long v) {
    int lo = 0, hi = n;  // start[lo] <= v < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ ResArgs problem_view(const GroupArgs &g, const ProbDev &P, double *out) {
    ResArgs a;
    a.q = (const SBP_GLOBAL double *)(g.q + P.off);
    a.out = (SBP_GLOBAL double *)(out + P.off);
    a.metric = (const SBP_GLOBAL double *)P.metric;
    a.jac = (const SBP_GLOBAL double *)P.jac;
    a.nbr = (const SBP_GLOBAL int32_t *)P.nbr;
    a.trace = (SBP_GLOBAL double *)P.trace;
    a.aux = (SBP_GLOBAL double *)P.thb;
    a.bc = (const SBP_GLOBAL double *)P.bc;
    a.src = (const SBP_GLOBAL double *)P.src;
    a.orient = (const SBP_GLOBAL int32_t *)P.orient;
    a.status = g.status;
    a.D = g.D;
    a.K = P.K;
    a.nodes = P.nodes;
    a.gamma = P.gamma;
    a.R = P.R;
    a.mu = P.mu;
    a.Pr = P.Pr;
    a.eta = P.eta;
    a.w_end = P.w_end;
    a.isw = P.isw;
    a.kap = P.kap;
    a.iface_diss = P.iface_diss;
    a.two_point = P.two_point;
    return a;
}

// Entropy-stable matrix interface dissipation |n| R |Lambda| T R^T (w_i - w_nu) for face states a
// (own) and b (partner), n = (n0, n1, n2) the averaged metric row: the Roe-type dissipation in
// entropy variables, eigenvectors of the flux Jacobian in n/|n| at the Chandrashekar-flux averages,
// scaled so that R T R^T = dq/dw.  Both nodes carry their logarithms.
__device__ __forceinline__ void matrix_dissipation(const Node &a, const Node &b, double n0, double n1,
                                                   double n2, double gamma, double R, double out[5]) {
    const double gm1 = gamma - 1.0;
    // logarithmic means of rho and beta (series near equal states, as in the flux)
    const double sr = a.rho + b.rho, dr = a.rho - b.rho;
    const double sb = a.beta + b.beta, db = a.beta - b.beta;
    const double irb = rcp(sr * sb);
    const double isr = sb * irb, isb = sr * irb;
    const double zr = dr * isr, ur = zr * zr;
    const double rho_hat = ur < LOGMEAN_U ? 0.5 * sr * series_G(ur) : dr * rcp(a.lrho - b.lrho);
    const double zb = db * isb, ub_ = zb * zb;
    const double ibeta_hat = ub_ < LOGMEAN_U ? 2.0 * isb * series_F(ub_) : (a.lbeta - b.lbeta) * rcp(db);
    const double p_hat = 0.5 * sr * isb;  // rho_bar / (2 beta_bar)
    const double a_hat = sqrt_pos(gamma * p_hat * rcp(rho_hat));
    const double u1 = 0.5 * (a.u1 + b.u1), u2 = 0.5 * (a.u2 + b.u2), u3 = 0.5 * (a.u3 + b.u3);
    const double ubsq = u1 * u1 + u2 * u2 + u3 * u3;
    const double h_hat = 0.5 * gamma / gm1 * ibeta_hat + ubsq - 0.25 * (a.k + b.k);
    const double nn = sqrt_pos(n0 * n0 + n1 * n1 + n2 * n2);
    const double inn = rcp(nn);
    const double e0 = n0 * inn, e1 = n1 * inn, e2 = n2 * inn;
    const double vn = u1 * e0 + u2 * e1 + u3 * e2;
    // entropy-variable jump (w_1 up to a constant that cancels)
    const double R2 = 2.0 * R;
    double dw[5];
    dw[0] = R * ((a.lbeta - b.lbeta) / gm1 + (a.lrho - b.lrho) - (a.beta * a.k - b.beta * b.k));
    dw[1] = R2 * (a.beta * a.u1 - b.beta * b.u1);
    dw[2] = R2 * (a.beta * a.u2 - b.beta * b.u2);
    dw[3] = R2 * (a.beta * a.u3 - b.beta * b.u3);
    dw[4] = -R2 * (a.beta - b.beta);
    const double iR = rcp(R);
    // acoustic waves
    const double ca = rho_hat * iR / (2.0 * gamma);
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = 0.0;
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
        const double s = (double)sg;
        const double r[5] = {1.0, fma(s * a_hat, e0, u1), fma(s * a_hat, e1, u2), fma(s * a_hat, e2, u3),
                             fma(s * a_hat, vn, h_hat)};
        const double proj = r[0] * dw[0] + r[1] * dw[1] + r[2] * dw[2] + r[3] * dw[3] + r[4] * dw[4];
        const double k = fabs(fma(s, a_hat, vn)) * ca * proj;
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c] = fma(k, r[c], out[c]);
    }
    // entropy wave
    {
        const double r[5] = {1.0, u1, u2, u3, 0.5 * ubsq};
        const double proj = r[0] * dw[0] + r[1] * dw[1] + r[2] * dw[2] + r[3] * dw[3] + r[4] * dw[4];
        const double k = fabs(vn) * rho_hat * gm1 / gamma * iR * proj;
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c] = fma(k, r[c], out[c]);
    }
    // shear waves: (I - e e^T) acting on v = dw_U + U_bar dw_5
    {
        const double v0 = fma(u1, dw[4], dw[1]), v1 = fma(u2, dw[4], dw[2]), v2 = fma(u3, dw[4], dw[3]);
        const double ve = v0 * e0 + v1 * e1 + v2 * e2;
        const double t0 = v0 - ve * e0, t1 = v1 - ve * e1, t2 = v2 - ve * e2;
        const double k = fabs(vn) * p_hat * iR;
        out[1] = fma(k, t0, out[1]);
        out[2] = fma(k, t1, out[2]);
        out[3] = fma(k, t2, out[3]);
        out[4] = fma(k, u1 * t0 + u2 * t1 + u3 * t2, out[4]);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] *= nn;
}

// Data of the partner node of a face node: state, metric row of the face direction and, when the
// interior penalty needs it, J.
struct FaceNbr {
    double q[5];
    double A[3];
    double J;
};

// Kind of the face across which an element sees neighbour index nb.
enum FaceKind : int {
    FACE_INVALID = 0,    // a mesh error
    FACE_INTERIOR = 1,   // a valid neighbour
    FACE_DIRICHLET = 2,  // nb == -1 with boundary data present
    FACE_SLIP = 3,       // nb == -2 on an inviscid problem
    FACE_WALL = 4,       // nb == -3: adiabatic no-slip wall
};

template <class Args>  // ResArgs or VjpArgs
__device__ __forceinline__ int face_kind(const Args &a, long long nb) {
    if (nb >= 0 && nb < a.K) return FACE_INTERIOR;
    if (nb == -1) return a.bc != nullptr ? FACE_DIRICHLET : FACE_INVALID;
    if (nb == -2) return a.mu == 0.0 ? FACE_SLIP : FACE_INVALID;
    return nb == -3 ? FACE_WALL : FACE_INVALID;
}

// Where the partner of a face node lies on the neighbour across face f = 2 l + side of element e:
// the neighbour's face fp, the partner's local node index lno and tangential index tp on face fp,
// and the sign sg (-s s') that turns the neighbour's direction l' = fp / 2 into the own direction
// l.  (ta, tb) are the own face node's tangential indices.  Without an orientation table faces are
// aligned: fp = f ^ 1, the same tangential indices (local index aligned_lno), sg = 1.  An invalid table entry gives ok =
// false and the aligned partner (so that every index stays inside the neighbour element).
// ORIENT = false compiles the aligned case only (kernels launched for problems without a table).
struct FaceLink {
    int fp, lno, tp;
    double sg;
    bool ok;
};

template <int N, bool ORIENT = true, class Args>  // Args: ResArgs or VjpArgs
__device__ __forceinline__ FaceLink face_link(const Args &a, long long e, int f, int ta, int tb,
                                              int aligned_lno) {
    FaceLink r;
    r.ok = true;
    if (!ORIENT || a.orient == nullptr) {
        // aligned faces: the caller's mirrored node index
        r.fp = f ^ 1;
        r.lno = aligned_lno;
        r.tp = ta + N * tb;
        r.sg = 1.0;
        return r;
    }
    int code = 0;
    r.fp = f ^ 1;
    const int o = a.orient[e * 6 + f];
    if (o >= 0 && o < 64 && (o & 7) < 6) {
        r.fp = o & 7;
        code = o >> 3;
    } else {
        r.ok = false;
    }
    const int x = (code & 1) ? tb : ta, y = (code & 1) ? ta : tb;
    const int ap = (code & 2) ? N - 1 - x : x, bp = (code & 4) ? N - 1 - y : y;
    const int lp = r.fp >> 1, ilp = (r.fp & 1) ? N - 1 : 0;
    r.lno = lp == 0 ? ilp + N * ap + N * N * bp
                    : (lp == 1 ? ap + N * ilp + N * N * bp : ap + N * bp + N * N * ilp);
    r.tp = ap + N * bp;
    r.sg = ((r.fp & 1) == (f & 1)) ? -1.0 : 1.0;
    return r;
}

// Partner of a face node: node pg of the neighbour (metric row of its direction l, times sg) or,
// on a boundary face, a ghost at the own node pg with the own metrics (l the own direction, sg = 1)
// and J carrying the prescribed state (Dirichlet), the own state with the momentum reflected
// about the face (slip wall), or the own state with the momentum reversed (no-slip wall: zero
// velocity and the own temperature on average).
template <bool VISC>
__device__ __forceinline__ void load_face_nbr(const ResArgs &a, long long pg, int kind, int l,
                                              double sg, FaceNbr &n) {
    const long long nodes = a.nodes;
    const SBP_GLOBAL double *qs = kind == FACE_DIRICHLET ? a.bc : a.q;
#pragma unroll
    for (int c = 0; c < 5; ++c) n.q[c] = qs[c * nodes + pg];
#pragma unroll
    for (int m = 0; m < 3; ++m) n.A[m] = sg * a.metric[(3 * l + m) * nodes + pg];
    n.J = (VISC && a.eta != 0.0) ? a.jac[pg] : 1.0;
    if (kind == FACE_SLIP) {
        const double mn = (n.q[1] * n.A[0] + n.q[2] * n.A[1] + n.q[3] * n.A[2]) *
                          rcp(n.A[0] * n.A[0] + n.A[1] * n.A[1] + n.A[2] * n.A[2]);
#pragma unroll
        for (int m = 0; m < 3; ++m) n.q[1 + m] = fma(-2.0 * mn, n.A[m], n.q[1 + m]);
    } else if (kind == FACE_WALL) {
#pragma unroll
        for (int m = 0; m < 3; ++m) n.q[1 + m] = -n.q[1 + m];
    }
}

// Interface terms at one face node i of face (l, s) with partner data nb: the EC shared flux
// replacing the own flux, the Lax-Friedrichs dissipation and, for viscous problems, the interior
// penalty (v[0..4]) and the SAT^theta increment of theta_l (v[5..8]).
// Own-side quantities of a face node that do not depend on the face: primitives, pressure, sound
// speed, temperature, conservative state and 1/J.
struct FaceOwn {
    Node m;
    double P, c, T, iJ;
    const double *q;
};

__device__ __forceinline__ FaceOwn face_own(const ResArgs &a, const Node &m, double P,
                                            const double q[5], double iJ) {
    FaceOwn o;
    o.m = m;
    o.P = P;
    o.c = sqrt_pos(a.gamma * P * rcp(m.rho));
    o.T = rcp(2.0 * a.R * m.beta);
    o.iJ = iJ;
    o.q = q;
    return o;
}

// MD selects the matrix interface dissipation at compile time: its registers would otherwise be
// reserved by every launch (iface_diss is uniform per problem group).
template <int FLUX, bool VISC, bool MD = false>
__device__ __forceinline__ void face_terms(const ResArgs &a, const FaceOwn &ow, const double Ai[3],
                                           const FaceNbr &nb, double s, double v[9]) {
    const Node &mi = ow.m;
    const double Pi = ow.P, *qi = ow.q, iJi = ow.iJ;
    const double gm1 = a.gamma - 1.0, isw = a.isw;
    const double *qn = nb.q;
    const double An0 = nb.A[0], An1 = nb.A[1], An2 = nb.A[2];
    Node o;
    double Pn, irn;
    primitives_nolog(qn, gm1, o, Pn, irn);
    const double n0 = 0.5 * (Ai[0] + An0), n1 = 0.5 * (Ai[1] + An1), n2 = 0.5 * (Ai[2] + An2);
    double f[5];
    flux_n<FLUX, true>(mi, o, n0, n1, n2, gm1, f);
    if constexpr (FLUX == 3) {
        // no j = i volume term to cancel against: keep the own-flux part of the SAT
        double fo[5];
        euler_flux_n(mi, Pi, qi[4], Ai[0], Ai[1], Ai[2], fo);
#pragma unroll
        for (int c = 0; c < 5; ++c) f[c] -= fo[c];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = -s * isw * f[c];
    if constexpr (MD) {
        Node ob = o;  // the partner's logarithms were not needed by the flux's series branch
        ob.lrho = log(o.rho);
        ob.lbeta = log(o.beta);
        double md[5];
        matrix_dissipation(mi, ob, n0, n1, n2, a.gamma, a.R, md);
        const double cf = -0.5 * isw;
#pragma unroll
        for (int c = 0; c < 5; ++c) v[c] = fma(cf, md[c], v[c]);
    } else if (a.iface_diss) {
        const double nn = sqrt_pos(n0 * n0 + n1 * n1 + n2 * n2);
        const double li = fabs(mi.u1 * n0 + mi.u2 * n1 + mi.u3 * n2) + ow.c * nn;
        const double lo = fabs(o.u1 * n0 + o.u2 * n1 + o.u3 * n2) + sqrt_pos(a.gamma * Pn * irn) * nn;
        const double cf = -0.5 * fmax(li, lo) * isw;
#pragma unroll
        for (int c = 0; c < 5; ++c) v[c] = fma(cf, qi[c] - qn[c], v[c]);
    }
    if constexpr (VISC) {
        const double iTi = 2.0 * a.R * mi.beta, iTn = 2.0 * a.R * o.beta;
        const double wi[4] = {mi.u1 * iTi, mi.u2 * iTi, mi.u3 * iTi, -iTi};
        const double wn[4] = {o.u1 * iTn, o.u2 * iTn, o.u3 * iTn, -iTn};
        const double mct = -0.5 * s * isw;
        double dw[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            dw[c] = wi[c] - wn[c];
            v[5 + c] = mct * dw[c];  // (s / (2 w_end)) (w_nu - w_i)
        }
        if (a.eta != 0.0) {
            const double iJn = rcp(nb.J);
            double pi_[4], pn_[4];
            visc_flux_rank1(Ai[0], Ai[1], Ai[2], iJi, dw, mi.u1, mi.u2, mi.u3, ow.T, a.mu, a.kap, pi_);
            visc_flux_rank1(An0, An1, An2, iJn, dw, o.u1, o.u2, o.u3, rcp(iTn), a.mu, a.kap, pn_);
            const double cf = -0.5 * a.eta * isw;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c + 1] = fma(cf, pi_[c] + pn_[c], v[c + 1]);
        }
    }
}

template <int FLUX, bool VISC, bool MD = false>
__device__ __forceinline__ void face_terms(const ResArgs &a, const FaceOwn &ow, const double Ai[3],
                                           long long pg, int kind, int l, double sg, double s,
                                           double v[9]) {
    FaceNbr nb;
    load_face_nbr<VISC>(a, pg, kind, l, sg, nb);
    face_terms<FLUX, VISC, MD>(a, ow, Ai, nb, s, v);
}

}  // namespace
}  // namespace sbp
