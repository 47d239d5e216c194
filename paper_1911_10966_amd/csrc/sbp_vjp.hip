// Vector-Jacobian product qbar = (d(dq/dt)/dq)^T gbar of the ES-C residual, written by hand.
//
// Every element recomputes its forward intermediates; nothing of the forward pass is stored.
// Contributions that the forward scatters to a neighbour (interface SAT, dissipation, SAT^theta,
// SAT^V, interior penalty) are gathered instead: an element evaluates, for its own face node,
// the derivative of both its own and its neighbour's interface term, so no atomics are needed.
// The BR1 operator reaches neighbours of neighbours, which takes two kernels:
//   k_vjp_visc   cotangents of the gradients theta_a at every node (written to a buffer) and the
//                part of qbar that comes through the state dependence of the viscous fluxes;
//   k_vjp_main   the inviscid volume and interface terms, the interior penalty, the transposed
//                gradient operator with its SAT (reading neighbour theta cotangents), and the map
//                from primitive cotangents to qbar.
// Two passes add to qbar afterwards: k_vjp_bnd the boundary faces, and k_vjp_md the matrix
// interface dissipation (iface_diss = 2).
// Pair terms of the flux-differencing sum use the same cyclic pairing and LDS mailbox as the
// forward kernel; cotangents are accumulated on the node quantities (rho, U, beta) and mapped to
// conservative variables once per node.
#include "sbp_device.h"

namespace sbp {
namespace {

__device__ __forceinline__ double series_Fp(double u) {  // dF/du
    double r = sreg(7.0 / 15.0);
    r = fma(r, u, sreg(6.0 / 13.0));
    r = fma(r, u, sreg(5.0 / 11.0));
    r = fma(r, u, sreg(4.0 / 9.0));
    r = fma(r, u, sreg(3.0 / 7.0));
    r = fma(r, u, sreg(2.0 / 5.0));
    return fma(r, u, sreg(1.0 / 3.0));
}
__device__ __forceinline__ double series_Gp(double u) {  // dG/du
    double r = sreg(7.0 * (-25865068.0 / 1915538625.0));
    r = fma(r, u, sreg(6.0 * (-10719068.0 / 638512875.0)));
    r = fma(r, u, sreg(5.0 * (-10196.0 / 467775.0)));
    r = fma(r, u, sreg(4.0 * (-428.0 / 14175.0)));
    r = fma(r, u, sreg(3.0 * (-44.0 / 945.0)));
    r = fma(r, u, sreg(2.0 * (-4.0 / 45.0)));
    return fma(r, u, sreg(-1.0 / 3.0));
}

// Cotangents of one node's quantities (rho, U, beta, log rho, log beta, |U|^2).
struct NodeBar {
    double rho, u1, u2, u3, beta, lrho, lbeta, k;
};

// Reverse of flux_n<0> (Chandrashekar flux contracted with a constant vector n).
template <bool LAZY = false>
__device__ __forceinline__ void flux_n_vjp(const Node &a, const Node &b, double n0, double n1,
                                           double n2, double gm1, const double fb[5], NodeBar &ab,
                                           NodeBar &bb) {
    const double ub1 = 0.5 * (a.u1 + b.u1), ub2 = 0.5 * (a.u2 + b.u2), ub3 = 0.5 * (a.u3 + b.u3);
    const double un = ub1 * n0 + ub2 * n1 + ub3 * n2;
    const double sr = a.rho + b.rho, dr = a.rho - b.rho;
    const double isr = rcp(sr);
    const double zr = dr * isr, ur = zr * zr;
    const bool ser_r = ur < LOGMEAN_U;
    double rho_hat, Gr = 0.0, iLr = 0.0;
    if (ser_r) {
        Gr = series_G(ur);
        rho_hat = 0.5 * sr * Gr;
    } else {
        iLr = rcp(a.lrho - (LAZY ? log(b.rho) : b.lrho));
        rho_hat = dr * iLr;
    }
    const double sb = a.beta + b.beta, db = a.beta - b.beta;
    const double isb = rcp(sb);
    const double zb = db * isb, ubb = zb * zb;
    const bool ser_b = ubb < LOGMEAN_U;
    double ibh, Fb = 0.0, idb = 0.0;
    if (ser_b) {
        Fb = series_F(ubb);
        ibh = 2.0 * isb * Fb;
    } else {
        idb = rcp(db);
        ibh = (a.lbeta - (LAZY ? log(b.beta) : b.lbeta)) * idb;
    }
    const double pt = 0.5 * sr * isb;
    const double fr = rho_hat * un;
    const double c = 0.5 / gm1;
    const double kbar = 0.5 * (a.k + b.k);
    const double ubsq = ub1 * ub1 + ub2 * ub2 + ub3 * ub3;
    const double E = c * ibh - 0.5 * kbar + ubsq;
    // reverse sweep
    const double frb = fb[0] + fb[1] * ub1 + fb[2] * ub2 + fb[3] * ub3 + fb[4] * E;
    double u1b = fb[1] * fr + 2.0 * fb[4] * fr * ub1;
    double u2b = fb[2] * fr + 2.0 * fb[4] * fr * ub2;
    double u3b = fb[3] * fr + 2.0 * fb[4] * fr * ub3;
    const double ptb = fb[1] * n0 + fb[2] * n1 + fb[3] * n2 + fb[4] * un;
    const double Eb = fb[4] * fr;
    const double unb = fb[4] * pt + frb * rho_hat;
    const double rhb = frb * un;
    const double ibhb = Eb * c;
    const double kbb = -0.5 * Eb;
    u1b = fma(unb, n0, u1b);
    u2b = fma(unb, n1, u2b);
    u3b = fma(unb, n2, u3b);
    double srb = ptb * 0.5 * isb;
    double isbb = ptb * 0.5 * sr;
    double drb = 0.0, lrb = 0.0;
    if (ser_r) {
        srb += rhb * 0.5 * Gr;
        const double urb = rhb * 0.5 * sr * series_Gp(ur);
        const double zrb = 2.0 * zr * urb;
        drb += zrb * isr;
        const double isrb = zrb * dr;
        srb -= isr * isr * isrb;
    } else {
        drb += rhb * iLr;
        lrb = -rhb * dr * iLr * iLr;
    }
    double dbb = 0.0, lbb = 0.0;
    if (ser_b) {
        isbb += ibhb * 2.0 * Fb;
        const double ubbb = ibhb * 2.0 * isb * series_Fp(ubb);
        const double zbb = 2.0 * zb * ubbb;
        dbb += zbb * isb;
        isbb += zbb * db;
    } else {
        const double Lb = a.lbeta - (LAZY ? log(b.beta) : b.lbeta);
        lbb = ibhb * idb;
        dbb -= ibhb * Lb * idb * idb;
    }
    const double sbb = -isb * isb * isbb;
    ab.rho = srb + drb;
    bb.rho = srb - drb;
    ab.beta = sbb + dbb;
    bb.beta = sbb - dbb;
    ab.lrho = lrb;
    bb.lrho = -lrb;
    ab.lbeta = lbb;
    bb.lbeta = -lbb;
    ab.u1 = bb.u1 = 0.5 * u1b;
    ab.u2 = bb.u2 = 0.5 * u2b;
    ab.u3 = bb.u3 = 0.5 * u3b;
    ab.k = bb.k = 0.5 * kbb;
}

// Reverse of flux_n<2> (Kennedy-Gruber split form contracted with a constant vector n): with
// P = rho/(2 beta) and E = P/((gamma-1) rho) + |U|^2/2 = 1/(2 (gamma-1) beta) + |U|^2/2 per node,
// f = rho_bar U_bar.n [1, U_bar, E_bar] + P_bar [0, n, U_bar.n] (bars: arithmetic means).
__device__ __forceinline__ void kg_flux_n_vjp(const Node &a, const Node &b, double n0, double n1,
                                              double n2, double gm1, const double fb[5], NodeBar &ab,
                                              NodeBar &bb) {
    const double ub1 = 0.5 * (a.u1 + b.u1), ub2 = 0.5 * (a.u2 + b.u2), ub3 = 0.5 * (a.u3 + b.u3);
    const double un = ub1 * n0 + ub2 * n1 + ub3 * n2;
    const double rbar = 0.5 * (a.rho + b.rho);
    const double iba = 1.0 / a.beta, ibb = 1.0 / b.beta;
    const double Pbar = 0.25 * (a.rho * iba + b.rho * ibb);
    const double c = 0.5 / gm1;
    const double Ebar = 0.5 * (c * iba + 0.5 * a.k + c * ibb + 0.5 * b.k);
    const double fr = rbar * un;
    // reverse sweep
    const double frb = fb[0] + fb[1] * ub1 + fb[2] * ub2 + fb[3] * ub3 + fb[4] * Ebar;
    const double Ebarb = fb[4] * fr;
    const double Pbarb = fb[1] * n0 + fb[2] * n1 + fb[3] * n2 + fb[4] * un;
    const double unb = frb * rbar + fb[4] * Pbar;
    const double rbarb = frb * un;
    const double u1b = fb[1] * fr + unb * n0, u2b = fb[2] * fr + unb * n1, u3b = fb[3] * fr + unb * n2;
    // Pbar = (rho_a/beta_a + rho_b/beta_b)/4, Ebar = (c/beta_a + k_a/2 + c/beta_b + k_b/2)/2
    ab.rho = 0.5 * rbarb + 0.25 * Pbarb * iba;
    bb.rho = 0.5 * rbarb + 0.25 * Pbarb * ibb;
    ab.beta = -(0.25 * Pbarb * a.rho + 0.5 * Ebarb * c) * iba * iba;
    bb.beta = -(0.25 * Pbarb * b.rho + 0.5 * Ebarb * c) * ibb * ibb;
    ab.lrho = bb.lrho = 0.0;
    ab.lbeta = bb.lbeta = 0.0;
    ab.u1 = bb.u1 = 0.5 * u1b;
    ab.u2 = bb.u2 = 0.5 * u2b;
    ab.u3 = bb.u3 = 0.5 * u3b;
    ab.k = bb.k = 0.25 * Ebarb;
}

// Reverse of the nodal inviscid flux contracted with n, F(a).n = [rho U_n, rho U_n U + P n,
// rho U_n H] with P = rho/(2 beta) and H = gamma/(2 (gamma-1) beta) + |U|^2/2; adds the
// cotangents of a's quantities for the output cotangent fb to ab.
__device__ __forceinline__ void euler_flux_n_vjp(const Node &a, double n0, double n1, double n2,
                                                 double gm1, const double fb[5], NodeBar &ab) {
    const double un = a.u1 * n0 + a.u2 * n1 + a.u3 * n2;
    const double m = a.rho * un;
    const double ib = 1.0 / a.beta;
    const double g2 = 0.5 * (gm1 + 1.0) / gm1;
    const double H = fma(g2, ib, 0.5 * a.k);
    const double mb = fb[0] + fb[1] * a.u1 + fb[2] * a.u2 + fb[3] * a.u3 + fb[4] * H;
    const double Pb = fb[1] * n0 + fb[2] * n1 + fb[3] * n2;
    const double Hb = fb[4] * m;
    ab.u1 += fb[1] * m + mb * a.rho * n0;
    ab.u2 += fb[2] * m + mb * a.rho * n1;
    ab.u3 += fb[3] * m + mb * a.rho * n2;
    ab.rho += mb * un + 0.5 * Pb * ib;
    ab.beta -= (0.5 * Pb * a.rho + Hb * g2) * ib * ib;
    ab.k += 0.5 * Hb;
}

__device__ __forceinline__ void zero_bar(NodeBar &z) {
    z.rho = z.u1 = z.u2 = z.u3 = z.beta = z.lrho = z.lbeta = z.k = 0.0;
}

// Reverse of flux_n<1> (central flux (F(a) + F(b))/2 contracted with n).
__device__ __forceinline__ void central_flux_n_vjp(const Node &a, const Node &b, double n0, double n1,
                                                   double n2, double gm1, const double fb[5],
                                                   NodeBar &ab, NodeBar &bb) {
    double h[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) h[c] = 0.5 * fb[c];
    zero_bar(ab);
    zero_bar(bb);
    euler_flux_n_vjp(a, n0, n1, n2, gm1, h, ab);
    euler_flux_n_vjp(b, n0, n1, n2, gm1, h, bb);
}

// Reverse of the two-point flux of the volume form FLUX (0 Chandrashekar, 1 central,
// 2 Kennedy-Gruber; the standard DC form 3 uses the central flux at interfaces).
template <int FLUX, bool LAZY = false>
__device__ __forceinline__ void two_point_vjp(const Node &a, const Node &b, double n0, double n1,
                                              double n2, double gm1, const double fb[5], NodeBar &ab,
                                              NodeBar &bb) {
    if constexpr (FLUX == 2) kg_flux_n_vjp(a, b, n0, n1, n2, gm1, fb, ab, bb);
    else if constexpr (FLUX == 1 || FLUX == 3) central_flux_n_vjp(a, b, n0, n1, n2, gm1, fb, ab, bb);
    else flux_n_vjp<LAZY>(a, b, n0, n1, n2, gm1, fb, ab, bb);
}

// Folds the cotangents of log rho, log beta and |U|^2 into (rho, U, beta) of the same node.
__device__ __forceinline__ void reduce_bar(const Node &n, const NodeBar &z, double out[5]) {
    out[0] = z.rho + z.lrho / n.rho;
    out[1] = fma(2.0 * n.u1, z.k, z.u1);
    out[2] = fma(2.0 * n.u2, z.k, z.u2);
    out[3] = fma(2.0 * n.u3, z.k, z.u3);
    out[4] = z.beta + z.lbeta / n.beta;
}

// Reverse of the uncontracted viscous flux F^V_m[c] (m = 0..2, c = 0..3 momentum/energy) as a
// function of the entropy-variable gradients g, the velocity and the temperature.
__device__ __forceinline__ void visc_flux_vjp(const double g[3][4], const double u[3], double T,
                                              double mu, double kap, const double Fb[3][4],
                                              double gb[3][4], double ub[3], double &Tb) {
    double du[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) du[k][j] = T * fma(u[k], g[j][3], g[j][k]);
    const double div = du[0][0] + du[1][1] + du[2][2];
    double dub[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) dub[k][j] = 0.0;
    double divb = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        gb[m][3] = Fb[m][3] * kap * T * T;
        Tb += Fb[m][3] * g[m][3] * 2.0 * kap * T;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double tau = mu * (du[i][m] + du[m][i] - (i == m ? (2.0 / 3.0) * div : 0.0));
            ub[i] += Fb[m][3] * tau;
            const double taub = mu * (Fb[m][i] + Fb[m][3] * u[i]);
            dub[i][m] += taub;
            dub[m][i] += taub;
            if (i == m) divb -= (2.0 / 3.0) * taub;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) dub[k][k] += divb;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        gb[j][0] = gb[j][1] = gb[j][2] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gb[j][k] += T * dub[k][j];
            gb[j][3] += T * u[k] * dub[k][j];
            ub[k] += T * g[j][3] * dub[k][j];
            Tb += fma(u[k], g[j][3], g[j][k]) * dub[k][j];
        }
}

// Reverse of visc_flux_rank1 (the interior-penalty flux): accumulates the cotangents of dw, U, T
// for the output cotangent ob.
__device__ __forceinline__ void visc_flux_rank1_vjp(double n0, double n1, double n2, double iJ,
                                                    const double dw[4], const double u[3], double T,
                                                    double mu, double kap, const double ob[4],
                                                    double dwb[4], double ub[3], double &Tb) {
    const double n[3] = {n0, n1, n2};
    double v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = T * fma(u[k], dw[3], dw[k]);
    const double nn = n0 * n0 + n1 * n1 + n2 * n2;
    const double vn = v[0] * n0 + v[1] * n1 + v[2] * n2;
    const double c1 = mu * iJ * nn, c2 = mu * iJ * vn * (1.0 / 3.0);
    double oe[3], c2b = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double out = fma(c1, v[k], c2 * n[k]);
        ub[k] = fma(ob[3], out, ub[k]);
        oe[k] = fma(ob[3], u[k], ob[k]);
        c2b = fma(oe[k], n[k], c2b);
    }
    const double vnb = c2b * mu * iJ * (1.0 / 3.0);
    const double t3 = kap * T * T * nn * iJ;
    dwb[3] = fma(ob[3], t3, dwb[3]);
    Tb += ob[3] * 2.0 * kap * T * nn * iJ * dw[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vb = fma(c1, oe[k], vnb * n[k]);
        dwb[k] = fma(T, vb, dwb[k]);
        dwb[3] = fma(T * u[k], vb, dwb[3]);
        ub[k] = fma(T * dw[3], vb, ub[k]);
        Tb += fma(u[k], dw[3], dw[k]) * vb;
    }
}

// Cotangents of (rho, U, beta, P, T) of a node mapped to its conservative variables, with
// beta = rho/(2P), T = P/(rho R), P = (gamma-1)(q_5 - rho |U|^2 / 2), U = m/rho.
__device__ __forceinline__ void prim_vjp(const double q[5], double gm1, double R, double rb,
                                         double ub[3], double bb, double Pb, double Tb,
                                         double qb[5]) {
    const double rho = q[0];
    const double ir = 1.0 / rho;
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double k = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double P = gm1 * (q[4] - 0.5 * rho * k);
    const double T = P / (rho * R);
    const double beta = 0.5 * rho / P;
    Pb += Tb / (rho * R);
    rb -= Tb * T * ir;
    rb += bb * 0.5 / P;
    Pb -= bb * beta / P;
    qb[4] = gm1 * Pb;
    rb -= gm1 * Pb * 0.5 * k;
#pragma unroll
    for (int d = 0; d < 3; ++d) ub[d] -= gm1 * Pb * rho * u[d];
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        qb[1 + d] = ub[d] * ir;
        s += ub[d] * u[d];
    }
    qb[0] = rb - s * ir;
}

struct NodeFull {
    double q[5];
    double u[3];
    double P, T, rho;
};

__device__ __forceinline__ void load_node(const double *q, long long nodes, long long g, double gm1,
                                          double R, NodeFull &n) {
#pragma unroll
    for (int c = 0; c < 5; ++c) n.q[c] = q[c * nodes + g];
    n.rho = n.q[0];
    const double ir = 1.0 / n.rho;
    n.u[0] = n.q[1] * ir;
    n.u[1] = n.q[2] * ir;
    n.u[2] = n.q[3] * ir;
    n.P = gm1 * (n.q[4] - 0.5 * n.rho * (n.u[0] * n.u[0] + n.u[1] * n.u[1] + n.u[2] * n.u[2]));
    n.T = n.P / (n.rho * R);
}

// ------------------------------------------------------------------------------------------
// Pass 1: cotangents of the BR1 gradients, and the state-dependence part of the viscous flux.
// ------------------------------------------------------------------------------------------
template <int N, int EPW>
__global__ void __launch_bounds__(NT_OF(EPW * N * N * N))
k_vjp_visc(const VjpArgs a) {
    constexpr int N2 = N * N, N3 = N * N * N, NODES = EPW * N3;
    __shared__ double s_buf[8 * NODES];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    if (tid < N2) s_D[tid] = a.D[tid];
    const int slot = tid / N3;
    const int ln = tid - slot * N3;
    const long long e = xcd_block(blockIdx.x, gridDim.x) * EPW + slot;
    const bool active = (tid < NODES) && (e < a.K);
    const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
    const int idx[3] = {i1, i2, i3};
    const int stride[3] = {1, N, N2};
    const long long nodes = a.nodes;
    const long long g = e * N3 + ln;
    const double gm1 = a.gamma - 1.0;
    const double isw = 1.0 / a.w_end;
    const double mu = a.mu;
    const double kap = a.mu * a.gamma * a.R / ((a.gamma - 1.0) * a.Pr);

    NodeFull me;
    double A[3][3];
    double J = 1.0, rb[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        load_node(a.q, nodes, g, gm1, a.R, me);
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[l][m] = a.metric[(3 * l + m) * nodes + g];
        J = a.jac[g];
        const double iJ = 1.0 / J;
#pragma unroll
        for (int c = 0; c < 4; ++c) rb[c] = a.gbar[(c + 1) * nodes + g] * iJ;
    } else {
        me.q[0] = 1.0; me.q[1] = me.q[2] = me.q[3] = 0.0; me.q[4] = 1.0;
        me.rho = 1.0; me.u[0] = me.u[1] = me.u[2] = 0.0; me.P = 1.0; me.T = 1.0;
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[l][m] = 0.0;
    }
    const double iJ = 1.0 / J;
    const double iT = 1.0 / me.T;
    const double w[4] = {me.u[0] * iT, me.u[1] * iT, me.u[2] * iT, -iT};
    if (tid < NODES) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            s_buf[c * NODES + tid] = w[c];
            s_buf[(4 + c) * NODES + tid] = rb[c];
        }
    }
    __syncthreads();
    double th[3][4], fhb[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int c = 0; c < 4; ++c) th[d][c] = fhb[d][c] = 0.0;
        if (tid < NODES) {
            const int il = idx[d];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const int pn = tid + (b - il) * stride[d];
                const double dd = s_D[il * N + b];   // theta_d = D_d w
                const double dt = s_D[b * N + il];   // fhat_d cotangent = D_d^T rbar
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    th[d][c] = fma(dd, s_buf[c * NODES + pn], th[d][c]);
                    fhb[d][c] = fma(dt, s_buf[(4 + c) * NODES + pn], fhb[d][c]);
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int il = idx[d];
            if (il != 0 && il != N - 1) continue;
            const int side = (il == N - 1) ? 1 : 0;
            const double s = side ? 1.0 : -1.0;
            const long long nb = a.nbr[e * 6 + 2 * d + side];
            const int kind = face_kind(a, nb);
            if (kind == FACE_INVALID) {
                atomicOr(a.status, FLAG_MESH);
                continue;
            }
            if (kind != FACE_INTERIOR) {
                // boundary ghost: the prescribed state, or (adiabatic wall) the own state with the
                // velocity reversed; SAT^V vanishes (Dirichlet) or keeps no energy flux (wall)
                double wn[4];
                if (kind == FACE_DIRICHLET) {
                    NodeFull o;
                    load_node(a.bc, nodes, g, gm1, a.R, o);
                    const double iTn = 1.0 / o.T;
                    wn[0] = o.u[0] * iTn; wn[1] = o.u[1] * iTn; wn[2] = o.u[2] * iTn; wn[3] = -iTn;
                } else {
                    wn[0] = -w[0]; wn[1] = -w[1]; wn[2] = -w[2]; wn[3] = w[3];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) th[d][c] = fma(0.5 * s * isw, wn[c] - w[c], th[d][c]);
                if (kind == FACE_WALL) fhb[d][3] = fma(-s * isw, rb[3], fhb[d][3]);
                continue;
            }
            const int ta = d == 0 ? i2 : i1, tb = d == 2 ? i2 : i3;
            const FaceLink k = face_link<N>(a, e, 2 * d + side, ta, tb, ln + (N - 1 - 2 * il) * stride[d]);
            if (!k.ok) atomicOr(a.status, FLAG_MESH);
            const long long pg = nb * N3 + k.lno;
            NodeFull o;
            load_node(a.q, nodes, pg, gm1, a.R, o);
            const double iTn = 1.0 / o.T;
            const double wn[4] = {o.u[0] * iTn, o.u[1] * iTn, o.u[2] * iTn, -iTn};
            const double iJn = 1.0 / a.jac[pg];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                th[d][c] = fma(0.5 * s * isw, wn[c] - w[c], th[d][c]);
                // own SAT^V half and the neighbour's SAT^V at the partner node (the orientation
                // sign of the neighbour's flux meets its side sign: -s either way)
                const double rbn = a.gbar[(c + 1) * nodes + pg] * iJn;
                fhb[d][c] = fma(-0.5 * s * isw, rb[c] + rbn, fhb[d][c]);
            }
        }
    }
    double gr[3][4];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            gr[j][c] = (A[0][j] * th[0][c] + A[1][j] * th[1][c] + A[2][j] * th[2][c]) * iJ;
    double Fb[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            Fb[m][c] = A[0][m] * fhb[0][c] + A[1][m] * fhb[1][c] + A[2][m] * fhb[2][c];
    double gb[3][4], ub[3] = {0.0, 0.0, 0.0}, Tb = 0.0;
    visc_flux_vjp(gr, me.u, me.T, mu, kap, Fb, gb, ub, Tb);
    if (active) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                a.thb[(d * 4 + c) * nodes + g] =
                    (A[d][0] * gb[0][c] + A[d][1] * gb[1][c] + A[d][2] * gb[2][c]) * iJ;
        double qb[5];
        prim_vjp(me.q, gm1, a.R, 0.0, ub, 0.0, 0.0, Tb, qb);
#pragma unroll
        for (int c = 0; c < 5; ++c) a.qbar[c * nodes + g] = qb[c];
    }
}

// Reverse of the interface terms (shared two-point flux, with the own-flux part for the DC form;
// Lax-Friedrichs dissipation; interior penalty) at one face node with outward sign s, partner
// state qn with metric row An and 1/J iJn, and partner cotangent rbn (the partner's own view of
// the same pair; zero for a boundary ghost).  BND: the partner is a boundary ghost of kind `kind`
// (Dirichlet data is a constant; a wall ghost is the own state with the momentum reversed or
// reflected, differentiated through the own state).  Accumulates the cotangents of the own node's
// (rho, U, beta) in acc, of P and T, of q directly (qdir), and of the entropy variables (wb).
template <bool VISC, bool BND, int FLUX>
__device__ __forceinline__ void face_term_vjp(const VjpArgs &a, const Node &me, const double q[5],
                                              const double rb[5], const double Al[3], double iJ,
                                              double Pme, double Tme, const double wme[4], double s,
                                              int kind, const double qn[5], const double rbn[5],
                                              const double An[3], double iJn, double acc[5],
                                              double &Pb, double &Tb, double qdir[5], double wb[4]) {
    const double gm1 = a.gamma - 1.0;
    const double isw = 1.0 / a.w_end;
    const double mu = a.mu;
    const double kap = a.mu * a.gamma * a.R / ((a.gamma - 1.0) * a.Pr);
    Node o;
    double Pn;
    primitives_nolog(qn, gm1, o, Pn);
    const double n0 = 0.5 * (Al[0] + An[0]), n1 = 0.5 * (Al[1] + An[1]),
                 n2 = 0.5 * (Al[2] + An[2]);
    double fb[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) fb[c] = -s * isw * (rb[c] - rbn[c]);
    NodeBar ab, bb;
    two_point_vjp<FLUX, true>(me, o, n0, n1, n2, gm1, fb, ab, bb);
    if constexpr (FLUX == 3) {
        // the DC form keeps the own-flux part of the SAT: +(s/w_end) F(q_i).A_i
        double fo[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) fo[c] = s * isw * rb[c];
        euler_flux_n_vjp(me, Al[0], Al[1], Al[2], gm1, fo, ab);
    }
    double ra[5];
    reduce_bar(me, ab, ra);
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += ra[c];
    if (BND && (kind == FACE_SLIP || kind == FACE_WALL)) {
        // a wall ghost's primitives: rho and beta are the own ones, U reversed (no-slip) or
        // reflected about the face (slip; the reflection is symmetric)
        double rg[5];
        reduce_bar(o, bb, rg);
        acc[0] += rg[0];
        acc[4] += rg[4];
        if (kind == FACE_WALL) {
            acc[1] -= rg[1]; acc[2] -= rg[2]; acc[3] -= rg[3];
        } else {
            const double ia2 = rcp(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]);
            const double un = (rg[1] * An[0] + rg[2] * An[1] + rg[3] * An[2]) * ia2;
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[1 + m] += rg[1 + m] - 2.0 * un * An[m];
        }
    }
    if (a.iface_diss == 1) {  // Lax-Friedrichs; the matrix dissipation has a pass of its own
        const double nn = sqrt_pos(n0 * n0 + n1 * n1 + n2 * n2);
        const double unm = me.u1 * n0 + me.u2 * n1 + me.u3 * n2;
        const double cme = sqrt_pos(a.gamma * Pme * rcp(me.rho));
        const double li = fabs(unm) + cme * nn;
        const double lo = fabs(o.u1 * n0 + o.u2 * n1 + o.u3 * n2) + sqrt_pos(a.gamma * Pn * rcp(o.rho)) * nn;
        const double lam = fmax(li, lo);
        double t_own = 0.0, t_nb = 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            t_own += (q[c] - qn[c]) * rb[c];
            t_nb += (qn[c] - q[c]) * rbn[c];
        }
        // d(q_i - q_ghost)/dq_i: identity (interior, Dirichlet), twice the momentum
        // (no-slip wall), twice its normal part (slip wall)
        if (!BND || kind == FACE_DIRICHLET) {
#pragma unroll
            for (int c = 0; c < 5; ++c) qdir[c] -= 0.5 * lam * isw * (rb[c] - rbn[c]);
        } else if (kind == FACE_WALL) {
#pragma unroll
            for (int c = 1; c < 4; ++c) qdir[c] -= lam * isw * rb[c];
        } else {
            // twice the projection on the face normal An
            const double rn = (rb[1] * An[0] + rb[2] * An[1] + rb[3] * An[2]) *
                              rcp(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]);
#pragma unroll
            for (int m = 0; m < 3; ++m) qdir[1 + m] -= lam * isw * rn * An[m];
        }
        // lambda depends on this node in the own view when li >= lo (ties go to the own
        // side) and in the neighbour's view only when li > lo (a wall ghost's speed equals
        // the own one: the own view carries it)
        double lb = 0.0;
        if (li >= lo || (BND && kind != FACE_DIRICHLET)) lb -= 0.5 * isw * t_own;
        if (li > lo) lb -= 0.5 * isw * t_nb;
        if (lb != 0.0) {
            const double sgn = unm >= 0.0 ? lb : -lb;
            acc[1] = fma(sgn, n0, acc[1]);
            acc[2] = fma(sgn, n1, acc[2]);
            acc[3] = fma(sgn, n2, acc[3]);
            const double cb = lb * nn;
            Pb += cb * a.gamma / (2.0 * cme * me.rho);
            acc[0] -= cb * cme / (2.0 * me.rho);
        }
    }
    if constexpr (VISC) {
        if (a.eta != 0.0) {
            // interior penalty X = -(eta/(2 w_end)) [Phi_i(A_i dw/J_i) + Phi_nu(A_nu dw/J_nu)],
            // with cotangent rbar_i - rbar_nu (the neighbour's term is -X; a ghost has none)
            const double iTn = 2.0 * a.R * o.beta;
            const double wn[4] = {o.u1 * iTn, o.u2 * iTn, o.u3 * iTn, -iTn};
            double dw[4], ob[4], dwb[4] = {0.0, 0.0, 0.0, 0.0};
            const double cf = -0.5 * a.eta * isw;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                dw[c] = wme[c] - wn[c];
                ob[c] = cf * (rb[c + 1] - rbn[c + 1]);
            }
            const double umv[3] = {me.u1, me.u2, me.u3};
            const double unv[3] = {o.u1, o.u2, o.u3};
            double ubi[3] = {0.0, 0.0, 0.0}, ubn[3] = {0.0, 0.0, 0.0}, Tbn = 0.0;
            visc_flux_rank1_vjp(Al[0], Al[1], Al[2], iJ, dw, umv, Tme, mu, kap, ob, dwb,
                                ubi, Tb);
            visc_flux_rank1_vjp(An[0], An[1], An[2], iJn, dw, unv, rcp(iTn), mu, kap, ob, dwb,
                                ubn, Tbn);
            acc[1] += ubi[0];
            acc[2] += ubi[1];
            acc[3] += ubi[2];
            if (BND && kind == FACE_WALL) {
                // dw = (2 U/T, 0); the ghost's velocity is -U, its temperature the own one
#pragma unroll
                for (int c = 0; c < 3; ++c) wb[c] += 2.0 * dwb[c];
                acc[1] -= ubn[0];
                acc[2] -= ubn[1];
                acc[3] -= ubn[2];
                Tb += Tbn;
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) wb[c] += dwb[c];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Pass 2: everything else; adds to the partial qbar of pass 1 when VISC.
// ------------------------------------------------------------------------------------------
template <int N, int EPW, bool VISC, bool OR, int FLUX>
__global__ void __launch_bounds__(NT_OF(EPW * N * N * N))
__attribute__((amdgpu_waves_per_eu(OR ? 2 : 1, 8)))  // the orientation lookup would cost a wave
k_vjp_main(const VjpArgs a) {
    constexpr int N2 = N * N, N3 = N * N * N, NODES = EPW * N3;
    constexpr int F_RHO = 0, F_U1 = 1, F_U2 = 2, F_U3 = 3, F_B = 4, F_LR = 5, F_LB = 6, F_K = 7;
    constexpr int F_A = 8, F_RB = 11, F_MSG = 16;
    __shared__ double s_buf[21 * NODES];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    if (tid < N2) s_D[tid] = a.D[tid];
    const int slot = tid / N3;
    const int ln = tid - slot * N3;
    const long long e = xcd_block(blockIdx.x, gridDim.x) * EPW + slot;
    const bool active = (tid < NODES) && (e < a.K);
    const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
    const int idx[3] = {i1, i2, i3};
    const int stride[3] = {1, N, N2};
    const long long nodes = a.nodes;
    const long long g = e * N3 + ln;
    const double gm1 = a.gamma - 1.0;
    const double w_end = a.w_end;
    const double isw = 1.0 / w_end;

    double q[5], A[3][3], J = 1.0, rb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (active) {
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = a.q[c * nodes + g];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[l][m] = a.metric[(3 * l + m) * nodes + g];
        J = a.jac[g];
        const double iJ0 = 1.0 / J;
#pragma unroll
        for (int c = 0; c < 5; ++c) rb[c] = a.gbar[c * nodes + g] * iJ0;
    } else {
        q[0] = 1.0; q[1] = q[2] = q[3] = 0.0; q[4] = 1.0;
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[l][m] = 0.0;
    }
    Node me;
    double Pme;
    bool ok;
    primitives(q, gm1, me, Pme, ok);
    if (active && !ok) atomicOr(a.status, FLAG_NONPHYSICAL);
    if (tid < NODES) {
        s_buf[F_RHO * NODES + tid] = me.rho;
        s_buf[F_U1 * NODES + tid] = me.u1;
        s_buf[F_U2 * NODES + tid] = me.u2;
        s_buf[F_U3 * NODES + tid] = me.u3;
        s_buf[F_B * NODES + tid] = me.beta;
        s_buf[F_LR * NODES + tid] = me.lrho;
        s_buf[F_LB * NODES + tid] = me.lbeta;
        s_buf[F_K * NODES + tid] = me.k;
#pragma unroll
        for (int c = 0; c < 5; ++c) s_buf[(F_RB + c) * NODES + tid] = rb[c];
    }
    // own accumulators: cotangents of rho, U, beta (and P, T below), plus direct qbar terms
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double Pb = 0.0, Tb = 0.0;
    double qdir[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    // ---- inviscid volume pairs ------------------------------------------------------------
    if constexpr (FLUX == 3) {
        // standard DC form, -sum_l D_l (A_l . F(q)): the transposed line operator applied to
        // rbar, then the reverse of the node's own contracted flux
        __syncthreads();
        if (tid < NODES) {
            NodeBar vb;
            zero_bar(vb);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int il = idx[l];
                double cl[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const double dd = s_D[b * N + il];
                    const int pn = tid + (b - il) * stride[l];
#pragma unroll
                    for (int c = 0; c < 5; ++c) cl[c] = fma(-dd, s_buf[(F_RB + c) * NODES + pn], cl[c]);
                }
                euler_flux_n_vjp(me, A[l][0], A[l][1], A[l][2], gm1, cl, vb);
            }
            double ra[5];
            reduce_bar(me, vb, ra);
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[c] += ra[c];
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (tid < NODES) {
                s_buf[(F_A + 0) * NODES + tid] = A[l][0];
                s_buf[(F_A + 1) * NODES + tid] = A[l][1];
                s_buf[(F_A + 2) * NODES + tid] = A[l][2];
            }
            __syncthreads();
            const int il = idx[l];
            const int st = stride[l];
            auto pair = [&](int b, bool send) {
                const int pn = tid + (b - il) * st;
                Node o;
                o.rho = s_buf[F_RHO * NODES + pn];
                o.u1 = s_buf[F_U1 * NODES + pn];
                o.u2 = s_buf[F_U2 * NODES + pn];
                o.u3 = s_buf[F_U3 * NODES + pn];
                o.beta = s_buf[F_B * NODES + pn];
                o.lrho = s_buf[F_LR * NODES + pn];
                o.lbeta = s_buf[F_LB * NODES + pn];
                o.k = s_buf[F_K * NODES + pn];
                const double n0 = A[l][0] + s_buf[(F_A + 0) * NODES + pn];
                const double n1 = A[l][1] + s_buf[(F_A + 1) * NODES + pn];
                const double n2 = A[l][2] + s_buf[(F_A + 2) * NODES + pn];
                const double dab = s_D[il * N + b], dba = s_D[b * N + il];
                double fb[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) fb[c] = -dab * rb[c] - dba * s_buf[(F_RB + c) * NODES + pn];
                NodeBar ab, bb;
                two_point_vjp<FLUX>(me, o, n0, n1, n2, gm1, fb, ab, bb);
                double ra[5];
                reduce_bar(me, ab, ra);
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] += ra[c];
                if (send) {
                    double rbb[5];
                    reduce_bar(o, bb, rbb);
#pragma unroll
                    for (int c = 0; c < 5; ++c) s_buf[(F_MSG + c) * NODES + pn] = rbb[c];
                }
            };
#pragma unroll
            for (int r = 1; 2 * r < N; ++r) {
                int b = il + r;
                if (b >= N) b -= N;
                if (tid < NODES) pair(b, true);
                __syncthreads();
                if (tid < NODES) {
#pragma unroll
                    for (int c = 0; c < 5; ++c) acc[c] += s_buf[(F_MSG + c) * NODES + tid];
                }
                __syncthreads();
            }
            if constexpr (N % 2 == 0) {
                // both nodes of the pair evaluate it; each keeps its own cotangent
                if (tid < NODES) {
                    int b = il + N / 2;
                    if (b >= N) b -= N;
                    pair(b, false);
                }
            }
            __syncthreads();
        }
    }

    // ---- interface SAT and dissipation (own and neighbour view) ----------------------------
    double wme[4] = {0.0, 0.0, 0.0, 0.0}, wb[4] = {0.0, 0.0, 0.0, 0.0};
    const double Tme = 0.5 / (a.R * me.beta);
    if (VISC) {
        const double iT = 1.0 / Tme;
        wme[0] = me.u1 * iT; wme[1] = me.u2 * iT; wme[2] = me.u3 * iT; wme[3] = -iT;
    }
    const double mu = a.mu;
    const double kap = a.mu * a.gamma * a.R / ((a.gamma - 1.0) * a.Pr);
    const double iJ = rcp(J);
    if (active) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int il = idx[l];
            if (il != 0 && il != N - 1) continue;
            const int side = (il == N - 1) ? 1 : 0;
            const double s = side ? 1.0 : -1.0;
            const long long nb = a.nbr[e * 6 + 2 * l + side];
            const int kind = face_kind(a, nb);
            if (kind == FACE_INVALID) {
                atomicOr(a.status, FLAG_MESH);
                continue;
            }
            if (kind != FACE_INTERIOR) {
                atomicExch(a.bnd_seen, a.gen);  // boundary faces: k_vjp_bnd
                continue;
            }
            // partner: the neighbour's node, with its metric row of direction l' (signed)
            const int ta = l == 0 ? i2 : i1, tb = l == 2 ? i2 : i3;
            const FaceLink k = face_link<N, OR>(a, e, 2 * l + side, ta, tb, ln + (N - 1 - 2 * il) * stride[l]);
            if (!k.ok) atomicOr(a.status, FLAG_MESH);
            const long long pg = nb * N3 + k.lno;
            const int lp = k.fp >> 1;
            double An[3], qn[5], rbn[5];
#pragma unroll
            for (int m = 0; m < 3; ++m) An[m] = k.sg * a.metric[(3 * lp + m) * nodes + pg];
            const double iJn = rcp(a.jac[pg]);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                qn[c] = a.q[c * nodes + pg];
                rbn[c] = a.gbar[c * nodes + pg] * iJn;
            }
            face_term_vjp<VISC, false, FLUX>(a, me, q, rb, A[l], iJ, Pme, Tme, wme, s, kind, qn, rbn, An, iJn,
                                       acc, Pb, Tb, qdir, wb);
        }
    }

    if constexpr (VISC) {
        // ---- transposed gradient operator D_a^T thetabar_a and its SAT -----------------------
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double thb_me[4] = {0.0, 0.0, 0.0, 0.0};
            if (active) {
#pragma unroll
                for (int c = 0; c < 4; ++c) thb_me[c] = a.thb[(d * 4 + c) * nodes + g];
            }
            __syncthreads();
            if (tid < NODES) {
#pragma unroll
                for (int c = 0; c < 4; ++c) s_buf[c * NODES + tid] = thb_me[c];
            }
            __syncthreads();
            if (tid < NODES) {
                const int il = idx[d];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const double dt = s_D[b * N + il];
                    const int pn = tid + (b - il) * stride[d];
#pragma unroll
                    for (int c = 0; c < 4; ++c) wb[c] = fma(dt, s_buf[c * NODES + pn], wb[c]);
                }
            }
            if (active) {
                const int il = idx[d];
                if (il == 0 || il == N - 1) {
                    const int side = (il == N - 1) ? 1 : 0;
                    const double s = side ? 1.0 : -1.0;
                    const long long nb = a.nbr[e * 6 + 2 * d + side];
                    if (face_kind(a, nb) == FACE_INTERIOR) {
                        // own SAT^theta and the neighbour's (its direction l', signed) at the partner
                        const int ta = d == 0 ? i2 : i1, tb = d == 2 ? i2 : i3;
                        const FaceLink k = face_link<N, OR>(a, e, 2 * d + side, ta, tb,
                                                            ln + (N - 1 - 2 * il) * stride[d]);
                        const long long pg = nb * N3 + k.lno;
                        const int dp = k.fp >> 1;
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            wb[c] = fma(-0.5 * s * isw, thb_me[c] + k.sg * a.thb[(dp * 4 + c) * nodes + pg],
                                        wb[c]);
                    }
                }
            }
        }
        // w = (U/T, -1/T)
        const double iT = 1.0 / Tme;
        acc[1] = fma(wb[0], iT, acc[1]);
        acc[2] = fma(wb[1], iT, acc[2]);
        acc[3] = fma(wb[2], iT, acc[3]);
        Tb += (-(wb[0] * me.u1 + wb[1] * me.u2 + wb[2] * me.u3) + wb[3]) * iT * iT;
    }

    if (active) {
        double ub[3] = {acc[1], acc[2], acc[3]};
        double qb[5];
        prim_vjp(q, gm1, a.R, acc[0], ub, acc[4], Pb, Tb, qb);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            double v = qb[c] + qdir[c];
            if (VISC) v += a.qbar[c * nodes + g];
            a.qbar[c * nodes + g] = v;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Pass 3: boundary faces (Dirichlet, slip and no-slip walls), one thread per node; adds to qbar.
// Kept out of pass 2 so that its registers do not lower that kernel's occupancy.
// ------------------------------------------------------------------------------------------
template <int N, bool VISC, int FLUX>
__device__ __forceinline__ void bnd_node(const VjpArgs &a, long long g) {
    constexpr int N2 = N * N, N3 = N * N * N;
    const long long e = g / N3;
    const int ln = (int)(g - e * N3);
    const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
    const int idx[3] = {i1, i2, i3};
    int kinds[3] = {FACE_INTERIOR, FACE_INTERIOR, FACE_INTERIOR};
    bool any = false;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int il = idx[l];
        if (il != 0 && il != N - 1) continue;
        const int k = face_kind(a, a.nbr[e * 6 + 2 * l + (il == N - 1 ? 1 : 0)]);
        if (k >= FACE_DIRICHLET) {
            kinds[l] = k;
            any = true;
        }
    }
    if (!any) return;
    const long long nodes = a.nodes;
    const double gm1 = a.gamma - 1.0;
    const double isw = 1.0 / a.w_end;
    double q[5], rb[5];
    const double iJ = rcp(a.jac[g]);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        q[c] = a.q[c * nodes + g];
        rb[c] = a.gbar[c * nodes + g] * iJ;
    }
    Node me;
    double Pme;
    bool ok;
    primitives(q, gm1, me, Pme, ok);
    const double Tme = 0.5 / (a.R * me.beta);
    double wme[4] = {0.0, 0.0, 0.0, 0.0};
    if (VISC) {
        const double iT = 1.0 / Tme;
        wme[0] = me.u1 * iT; wme[1] = me.u2 * iT; wme[2] = me.u3 * iT; wme[3] = -iT;
    }
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, qdir[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double wb[4] = {0.0, 0.0, 0.0, 0.0};
    double Pb = 0.0, Tb = 0.0;
    const double zero[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int kind = kinds[l];
        if (kind == FACE_INTERIOR) continue;
        const double s = idx[l] == N - 1 ? 1.0 : -1.0;
        double Al[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) Al[m] = a.metric[(3 * l + m) * nodes + g];
        // the ghost state (own metrics and J)
        double qn[5];
        if (kind == FACE_DIRICHLET) {
#pragma unroll
            for (int c = 0; c < 5; ++c) qn[c] = a.bc[c * nodes + g];
        } else {
            qn[0] = q[0];
            qn[4] = q[4];
            if (kind == FACE_WALL) {
                qn[1] = -q[1]; qn[2] = -q[2]; qn[3] = -q[3];
            } else {
                const double mn = (q[1] * Al[0] + q[2] * Al[1] + q[3] * Al[2]) *
                                  rcp(Al[0] * Al[0] + Al[1] * Al[1] + Al[2] * Al[2]);
#pragma unroll
                for (int m = 0; m < 3; ++m) qn[1 + m] = fma(-2.0 * mn, Al[m], q[1 + m]);
            }
        }
        face_term_vjp<VISC, true, FLUX>(a, me, q, rb, Al, iJ, Pme, Tme, wme, s, kind, qn, zero, Al, iJ, acc, Pb,
                                  Tb, qdir, wb);
        if constexpr (VISC) {
            // transposed SAT^theta of the boundary face: (s/(2 w_end)) (w_ghost - w_i)
            double thb_me[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) thb_me[c] = a.thb[(l * 4 + c) * nodes + g];
            if (kind == FACE_DIRICHLET) {
#pragma unroll
                for (int c = 0; c < 4; ++c) wb[c] = fma(-0.5 * s * isw, thb_me[c], wb[c]);
            } else if (kind == FACE_WALL) {
                // w_ghost - w_i = (-2 U/T, 0)
#pragma unroll
                for (int c = 0; c < 3; ++c) wb[c] = fma(-s * isw, thb_me[c], wb[c]);
            }
        }
    }
    if constexpr (VISC) {
        const double iT = 1.0 / Tme;
        acc[1] = fma(wb[0], iT, acc[1]);
        acc[2] = fma(wb[1], iT, acc[2]);
        acc[3] = fma(wb[2], iT, acc[3]);
        Tb += (-(wb[0] * me.u1 + wb[1] * me.u2 + wb[2] * me.u3) + wb[3]) * iT * iT;
    }
    double ub[3] = {acc[1], acc[2], acc[3]};
    double qb[5];
    prim_vjp(q, gm1, a.R, acc[0], ub, acc[4], Pb, Tb, qb);
#pragma unroll
    for (int c = 0; c < 5; ++c) a.qbar[c * nodes + g] += qb[c] + qdir[c];
}

// A grid of a few blocks per CU walks the nodes: when no boundary face was met, the pass is one
// load per thread.
constexpr long long kBndBlocks = 1024;

template <int N, bool VISC, int FLUX>
__global__ void __launch_bounds__(256) k_vjp_bnd(const VjpArgs a) {
    // nothing to do unless the main pass met a boundary face in this launch
    if (__hip_atomic_load(a.bnd_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != a.gen) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < a.nodes; g += stride)
        bnd_node<N, VISC, FLUX>(a, g);
}

// Reverse of matrix_dissipation (sbp_device.h): cotangents of both nodes' quantities from the
// cotangent ob of its output.  The forward values are recomputed first; the reverse then walks
// the shear, entropy and acoustic waves, the entropy-variable jump and the averages.
__device__ __forceinline__ void matrix_dissipation_vjp(const Node &a, const Node &b, double n0,
                                                       double n1, double n2, double gamma, double R,
                                                       const double ob[5], NodeBar &ab, NodeBar &bb) {
    const double gm1 = gamma - 1.0;
    // ---- forward values
    const double sr = a.rho + b.rho, dr = a.rho - b.rho;
    const double sb = a.beta + b.beta, db = a.beta - b.beta;
    const double irb = rcp(sr * sb);
    const double isr = sb * irb, isb = sr * irb;
    const double zr = dr * isr, ur = zr * zr;
    const bool ser_r = ur < LOGMEAN_U;
    const double Gr = ser_r ? series_G(ur) : 0.0;
    const double iLr = ser_r ? 0.0 : rcp(a.lrho - b.lrho);
    const double rho_hat = ser_r ? 0.5 * sr * Gr : dr * iLr;
    const double zb = db * isb, ub_ = zb * zb;
    const bool ser_b = ub_ < LOGMEAN_U;
    const double Fb = ser_b ? series_F(ub_) : 0.0;
    const double idb = ser_b ? 0.0 : rcp(db);
    const double ibeta_hat = ser_b ? 2.0 * isb * Fb : (a.lbeta - b.lbeta) * idb;
    const double p_hat = 0.5 * sr * isb;
    const double irh = rcp(rho_hat);
    const double a_hat = sqrt_pos(gamma * p_hat * irh);
    const double u[3] = {0.5 * (a.u1 + b.u1), 0.5 * (a.u2 + b.u2), 0.5 * (a.u3 + b.u3)};
    const double ubsq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double h_hat = 0.5 * gamma / gm1 * ibeta_hat + ubsq - 0.25 * (a.k + b.k);
    const double nn = sqrt_pos(n0 * n0 + n1 * n1 + n2 * n2);
    const double inn = rcp(nn);
    const double en[3] = {n0 * inn, n1 * inn, n2 * inn};
    const double vn = u[0] * en[0] + u[1] * en[1] + u[2] * en[2];
    const double R2 = 2.0 * R;
    const double ua[3] = {a.u1, a.u2, a.u3}, uo[3] = {b.u1, b.u2, b.u3};
    double dw[5];
    dw[0] = R * ((a.lbeta - b.lbeta) / gm1 + (a.lrho - b.lrho) - (a.beta * a.k - b.beta * b.k));
#pragma unroll
    for (int m = 0; m < 3; ++m) dw[1 + m] = R2 * (a.beta * ua[m] - b.beta * uo[m]);
    dw[4] = -R2 * (a.beta - b.beta);
    const double iR = rcp(R);
    const double ca = rho_hat * iR / (2.0 * gamma);
    const double svn = vn >= 0.0 ? 1.0 : -1.0, avn = fabs(vn);

    // ---- reverse
    double S[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) S[c] = nn * ob[c];
    double rhb = 0.0, ibhb = 0.0, phb = 0.0, ahb = 0.0, hb = 0.0, vnb = 0.0, usqb = 0.0, cab = 0.0;
    double uba[3] = {0.0, 0.0, 0.0};  // cotangent of the averaged velocity
    double dwb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // shear waves: out_U += ks t, out_E += ks (u.t), t = (I - e e^T) v, v = dw_U + u dw_4
    {
        double v[3], t[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m] = fma(u[m], dw[4], dw[1 + m]);
        const double ve = v[0] * en[0] + v[1] * en[1] + v[2] * en[2];
#pragma unroll
        for (int m = 0; m < 3; ++m) t[m] = v[m] - ve * en[m];
        const double ks = avn * p_hat * iR;
        const double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
        const double ksb = S[1] * t[0] + S[2] * t[1] + S[3] * t[2] + S[4] * ut;
        double tb[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            tb[m] = ks * fma(S[4], u[m], S[1 + m]);
            uba[m] += ks * S[4] * t[m];
        }
        const double te = tb[0] * en[0] + tb[1] * en[1] + tb[2] * en[2];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double vb = tb[m] - te * en[m];
            uba[m] += vb * dw[4];
            dwb[4] += vb * u[m];
            dwb[1 + m] += vb;
        }
        vnb += svn * p_hat * iR * ksb;
        phb += avn * iR * ksb;
    }
    // entropy wave: out += ke re, re = [1, u, |u|^2/2], ke = |vn| rho_hat (gm1/gamma)/R (re.dw)
    {
        const double ce = gm1 / gamma * iR;
        const double re[5] = {1.0, u[0], u[1], u[2], 0.5 * ubsq};
        const double pe = re[0] * dw[0] + re[1] * dw[1] + re[2] * dw[2] + re[3] * dw[3] + re[4] * dw[4];
        const double ke = avn * rho_hat * ce * pe;
        const double keb = S[0] * re[0] + S[1] * re[1] + S[2] * re[2] + S[3] * re[3] + S[4] * re[4];
        const double peb = avn * rho_hat * ce * keb;
        vnb += svn * rho_hat * ce * pe * keb;
        rhb += avn * ce * pe * keb;
        // re's cotangent: ke S + peb dw
#pragma unroll
        for (int m = 0; m < 3; ++m) uba[m] += fma(ke, S[1 + m], peb * dw[1 + m]);
        usqb += 0.5 * fma(ke, S[4], peb * dw[4]);
#pragma unroll
        for (int c = 0; c < 5; ++c) dwb[c] += peb * re[c];
    }
    // acoustic waves: out += k r, r = [1, u + s a e, h + s a vn], k = |vn + s a| ca (r.dw)
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
        const double sv = (double)sg;
        const double r[5] = {1.0, fma(sv * a_hat, en[0], u[0]), fma(sv * a_hat, en[1], u[1]),
                             fma(sv * a_hat, en[2], u[2]), fma(sv * a_hat, vn, h_hat)};
        const double pr = r[0] * dw[0] + r[1] * dw[1] + r[2] * dw[2] + r[3] * dw[3] + r[4] * dw[4];
        const double lam = fma(sv, a_hat, vn);
        const double alam = fabs(lam), slam = lam >= 0.0 ? 1.0 : -1.0;
        const double k = alam * ca * pr;
        const double kb = S[0] * r[0] + S[1] * r[1] + S[2] * r[2] + S[3] * r[3] + S[4] * r[4];
        const double lamb = slam * ca * pr * kb;
        cab += alam * pr * kb;
        const double prb = alam * ca * kb;
        double rbv[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            rbv[c] = fma(k, S[c], prb * dw[c]);
            dwb[c] += prb * r[c];
        }
        vnb += lamb;
        ahb += sv * lamb;
#pragma unroll
        for (int m = 0; m < 3; ++m) uba[m] += rbv[1 + m];
        ahb += sv * (rbv[1] * en[0] + rbv[2] * en[1] + rbv[3] * en[2] + rbv[4] * vn);
        hb += rbv[4];
        vnb += sv * a_hat * rbv[4];
    }
    rhb += cab * iR / (2.0 * gamma);
    // entropy-variable jump
    ab.lbeta = R * dwb[0] / gm1;
    bb.lbeta = -ab.lbeta;
    ab.lrho = R * dwb[0];
    bb.lrho = -ab.lrho;
    ab.beta = -R * dwb[0] * a.k - R2 * dwb[4];
    bb.beta = R * dwb[0] * b.k + R2 * dwb[4];
    ab.k = -R * dwb[0] * a.beta;
    bb.k = R * dwb[0] * b.beta;
    double uab[3], uob[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        ab.beta += R2 * dwb[1 + m] * ua[m];
        bb.beta -= R2 * dwb[1 + m] * uo[m];
        uab[m] = R2 * dwb[1 + m] * a.beta;
        uob[m] = -R2 * dwb[1 + m] * b.beta;
    }
    // averages: vn = u.e, h_hat, |u|^2, u = (u_a + u_b)/2
#pragma unroll
    for (int m = 0; m < 3; ++m) uba[m] += vnb * en[m];
    ibhb += 0.5 * gamma / gm1 * hb;
    usqb += hb;
    ab.k -= 0.25 * hb;
    bb.k -= 0.25 * hb;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        uba[m] += 2.0 * u[m] * usqb;
        uab[m] += 0.5 * uba[m];
        uob[m] += 0.5 * uba[m];
    }
    ab.u1 = uab[0]; ab.u2 = uab[1]; ab.u3 = uab[2];
    bb.u1 = uob[0]; bb.u2 = uob[1]; bb.u3 = uob[2];
    // a_hat = sqrt(gamma p_hat / rho_hat), p_hat = sr / (2 sb)
    phb += ahb * a_hat / (2.0 * p_hat);
    rhb -= ahb * a_hat * irh * 0.5;
    double srb = 0.5 * phb * isb, sbb = -p_hat * phb * isb, drb = 0.0, dbb = 0.0;
    // logarithmic means
    if (ser_r) {
        srb += 0.5 * Gr * rhb;
        const double urb = rhb * 0.5 * sr * series_Gp(ur);
        drb += urb * 2.0 * zr * isr;
        srb -= urb * 2.0 * ur * isr;
    } else {
        drb += rhb * iLr;
        const double Lb = -rhb * rho_hat * iLr;
        ab.lrho += Lb;
        bb.lrho -= Lb;
    }
    if (ser_b) {
        sbb -= ibeta_hat * isb * ibhb;
        const double ubb = ibhb * 2.0 * isb * series_Fp(ub_);
        dbb += ubb * 2.0 * zb * isb;
        sbb -= ubb * 2.0 * ub_ * isb;
    } else {
        ab.lbeta += ibhb * idb;
        bb.lbeta -= ibhb * idb;
        dbb -= ibhb * ibeta_hat * idb;
    }
    ab.rho = srb + drb;
    bb.rho = srb - drb;
    ab.beta += sbb + dbb;
    bb.beta += sbb - dbb;
}

// ------------------------------------------------------------------------------------------
// Pass 4 (iface_diss = 2): the matrix interface dissipation; adds to qbar.  One workgroup per
// element, one thread per (face, face node) item: most nodes of small elements lie on a face, and
// a per-node loop over directions would run three passes of the whole reverse sweep per wave.
// Across an interior face the two sides' terms are -M(q_i, q_nu)/(2 w_end) and its negative (M is
// odd in the exchange of the states and even in the sign of the normal), so the own node's
// cotangent is (dM/dq_i)^T applied to -(rbar_i - rbar_nu)/(2 w_end).  A boundary ghost has no
// cotangent of its own; a wall ghost is an image of the own state and is differentiated with it.
// Each item leaves the cotangents of its node's (rho, U, beta) in an LDS slot; each node then adds
// its (at most three) slots in direction order and maps them to conservative variables.
// ------------------------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(NT_OF(6 * N * N)) k_vjp_md(const VjpArgs a) {
    constexpr int N2 = N * N, N3 = N * N * N, ITEMS = 6 * N2;
    constexpr int NT = NT_OF(ITEMS);
    __shared__ double slot[5 * ITEMS];
    const long long e = blockIdx.x;
    const long long nodes = a.nodes;
    const double gm1 = a.gamma - 1.0;
    const double isw = 1.0 / a.w_end;
    const int it = threadIdx.x;
    if (it < ITEMS) {
        const int f = it / N2, t = it - f * N2;
        const int l = f >> 1, side = f & 1;
        const int ta = t % N, tb = t / N;
        const int il = side ? N - 1 : 0;
        const int st = l == 0 ? 1 : (l == 1 ? N : N2);
        const int ln = l == 0 ? il + N * ta + N2 * tb : (l == 1 ? ta + N * il + N2 * tb : ta + N * tb + N2 * il);
        const long long g = e * N3 + ln;
        const long long nb = a.nbr[e * 6 + f];
        const int kind = face_kind(a, nb);
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // cotangents of the node's rho, U, beta
        if (kind != FACE_INVALID) {  // (an invalid face is flagged by the main pass)
            double q[5], cb[5], Al[3], An[3], qn[5];
            const double iJ = rcp(a.jac[g]);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                q[c] = a.q[c * nodes + g];
                cb[c] = -0.5 * isw * a.gbar[c * nodes + g] * iJ;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) Al[m] = An[m] = a.metric[(3 * l + m) * nodes + g];
            if (kind == FACE_INTERIOR) {
                const FaceLink k = face_link<N>(a, e, f, ta, tb, ln + (N - 1 - 2 * il) * st);
                const long long pg = nb * N3 + k.lno;
                const int lp = k.fp >> 1;
#pragma unroll
                for (int m = 0; m < 3; ++m) An[m] = k.sg * a.metric[(3 * lp + m) * nodes + pg];
                const double iJn = rcp(a.jac[pg]);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    qn[c] = a.q[c * nodes + pg];
                    cb[c] += 0.5 * isw * a.gbar[c * nodes + pg] * iJn;
                }
            } else if (kind == FACE_DIRICHLET) {
#pragma unroll
                for (int c = 0; c < 5; ++c) qn[c] = a.bc[c * nodes + g];
            } else {
                // wall ghosts: the own state with the momentum reversed (no-slip) or reflected
                // about the face (slip)
                qn[0] = q[0];
                qn[4] = q[4];
                if (kind == FACE_WALL) {
                    qn[1] = -q[1]; qn[2] = -q[2]; qn[3] = -q[3];
                } else {
                    const double mn = (q[1] * Al[0] + q[2] * Al[1] + q[3] * Al[2]) *
                                      rcp(Al[0] * Al[0] + Al[1] * Al[1] + Al[2] * Al[2]);
#pragma unroll
                    for (int m = 0; m < 3; ++m) qn[1 + m] = fma(-2.0 * mn, Al[m], q[1 + m]);
                }
            }
            Node me, o;
            double Pme, Pn;
            bool ok;
            primitives(q, gm1, me, Pme, ok);
            primitives_nolog(qn, gm1, o, Pn);
            o.lrho = log(o.rho);
            o.lbeta = log(o.beta);
            NodeBar ab, bb;
            matrix_dissipation_vjp(me, o, 0.5 * (Al[0] + An[0]), 0.5 * (Al[1] + An[1]),
                                   0.5 * (Al[2] + An[2]), a.gamma, a.R, cb, ab, bb);
            reduce_bar(me, ab, acc);
            if (kind == FACE_WALL || kind == FACE_SLIP) {
                // the ghost's rho and beta are the own ones; its velocity the reversed or
                // reflected one
                double rg[5];
                reduce_bar(o, bb, rg);
                acc[0] += rg[0];
                acc[4] += rg[4];
                if (kind == FACE_WALL) {
                    acc[1] -= rg[1]; acc[2] -= rg[2]; acc[3] -= rg[3];
                } else {
                    const double un = (rg[1] * Al[0] + rg[2] * Al[1] + rg[3] * Al[2]) *
                                      rcp(Al[0] * Al[0] + Al[1] * Al[1] + Al[2] * Al[2]);
#pragma unroll
                    for (int m = 0; m < 3; ++m) acc[1 + m] += rg[1 + m] - 2.0 * un * Al[m];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) slot[c * ITEMS + it] = acc[c];
    }
    __syncthreads();
    for (int ln = threadIdx.x; ln < N3; ln += NT) {
        const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        bool any = false;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int il = l == 0 ? i1 : (l == 1 ? i2 : i3);
            if (il != 0 && il != N - 1) continue;
            any = true;
            const int at = (2 * l + (il == N - 1 ? 1 : 0)) * N2 + tangential_index<N>(l, i1, i2, i3);
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[c] += slot[c * ITEMS + at];
        }
        if (!any) continue;
        const long long g = e * N3 + ln;
        double q[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = a.q[c * nodes + g];
        double ub[3] = {acc[1], acc[2], acc[3]};
        double qb[5];
        prim_vjp(q, gm1, a.R, acc[0], ub, acc[4], 0.0, 0.0, qb);
#pragma unroll
        for (int c = 0; c < 5; ++c) a.qbar[c * nodes + g] += qb[c];
    }
}

template <int N, int EPW, bool OR, int FLUX>
int launch_vjp_f(const VjpArgs &a, hipStream_t s) {
    constexpr int NT = NT_OF(EPW * N * N * N);
    const long long blocks = (a.K + EPW - 1) / EPW;
    long long nb = (a.nodes + 255) / 256;
    if (nb > kBndBlocks) nb = kBndBlocks;
    if (a.mu != 0.0) {
        hipLaunchKernelGGL((k_vjp_visc<N, EPW>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL((k_vjp_main<N, EPW, true, OR, FLUX>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL((k_vjp_bnd<N, true, FLUX>), dim3((unsigned)nb), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_vjp_main<N, EPW, false, OR, FLUX>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL((k_vjp_bnd<N, false, FLUX>), dim3((unsigned)nb), dim3(256), 0, s, a);
    }
    if (hipGetLastError() != hipSuccess) return -1;
    if (a.iface_diss == 2) {
        hipLaunchKernelGGL((k_vjp_md<N>), dim3((unsigned)a.K), dim3(NT_OF(6 * N * N)), 0, s, a);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

template <int N, int EPW, bool OR>
int launch_vjp_or(const VjpArgs &a, hipStream_t s) {
    switch (a.two_point) {
        case 0: return launch_vjp_f<N, EPW, OR, 0>(a, s);
        case 1: return launch_vjp_f<N, EPW, OR, 1>(a, s);
        case 2: return launch_vjp_f<N, EPW, OR, 2>(a, s);
        case 3: return launch_vjp_f<N, EPW, OR, 3>(a, s);
        default: return -1;
    }
}

template <int N, int EPW>
int launch_vjp_n(const VjpArgs &a, hipStream_t s) {
    return a.orient != nullptr ? launch_vjp_or<N, EPW, true>(a, s) : launch_vjp_or<N, EPW, false>(a, s);
}

}  // namespace

int launch_vjp(int p, const VjpArgs &a, hipStream_t s) {
    switch (p) {
        case 1: return launch_vjp_n<2, 8>(a, s);
        case 2: return launch_vjp_n<3, 2>(a, s);
        case 3: return launch_vjp_n<4, 1>(a, s);
        case 4: return launch_vjp_n<5, 1>(a, s);
        case 5: return launch_vjp_n<6, 1>(a, s);
        case 6: return launch_vjp_n<7, 1>(a, s);
        case 7: return launch_vjp_n<8, 1>(a, s);
        case 8: return launch_vjp_n<9, 1>(a, s);
        default: return -1;
    }
}

}  // namespace sbp
