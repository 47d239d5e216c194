// gfx950 kernels of the ES-C residual for high degrees, N = p + 1 from 10 to 16 (arXiv 1911.10966,
// section "Discretization of the compressible Navier-Stokes equations"; the cost study of the
// Taylor-Green section goes up to p = 15).  FP64 throughout.
//
// An element of N^3 nodes no longer fits one workgroup's LDS (N = 16: 4096 nodes x 24 doubles),
// so the residual is split into passes over node planes.  Each pass holds a plane of N^2 nodes
// (one thread per node) in LDS, and a plane contains complete lines of two directions:
//   pass A, planes of constant xi3:  volume pairs and interface terms of xi1 and xi2, BR1 gradient
//           theta_1, theta_2 (kept in a per-node scratch);
//   pass B, planes of constant xi2:  volume pairs and interface terms of xi3, theta_3; with all
//           three gradients at hand, the viscous flux, the contravariant fluxes fhat_l, the xi3
//           divergence and the own half of SAT^V on xi3 faces (fhat_1, fhat_2 to scratch, xi3 face
//           traces of fhat_3);
//   pass C, planes of constant xi3:  xi1 and xi2 divergence of fhat, SAT^V (the neighbour's fhat
//           read from the scratch or the traces) and the division by J.
// Inviscid problems run passes A and B only (B divides by J).  The arithmetic of each term is
// that of the element kernel; only the grouping into passes differs.
#include "sbp_device.h"

namespace sbp {
namespace {

constexpr int F_RHO = 0, F_U1 = 1, F_U2 = 2, F_U3 = 3, F_B = 4, F_LR = 5, F_LB = 6, F_K = 7;
constexpr int F_A0 = 8, F_A1 = 11, F_MSG0 = 14, F_MSG1 = 19;
constexpr int PLANE_FIELDS = 24;  // doubles of LDS per node: node data 8, metric rows 6, mailboxes 10

// Scratch layout (aux, viscous only): [0..3] theta_1, [4..7] theta_2 at every node (pass A to B),
// [8..11] fhat_1, [12..15] fhat_2 (pass B to C).
constexpr int AUX_TH = 0, AUX_FH = 8;

__device__ __forceinline__ void stage_node(double *s_buf, int NODES, int tid, const Node &me) {
    s_buf[F_RHO * NODES + tid] = me.rho;
    s_buf[F_U1 * NODES + tid] = me.u1;
    s_buf[F_U2 * NODES + tid] = me.u2;
    s_buf[F_U3 * NODES + tid] = me.u3;
    s_buf[F_B * NODES + tid] = me.beta;
    s_buf[F_LR * NODES + tid] = me.lrho;
    s_buf[F_LB * NODES + tid] = me.lbeta;
    s_buf[F_K * NODES + tid] = me.k;
}

__device__ __forceinline__ Node staged_node(const double *s_buf, int NODES, int i) {
    Node o;
    o.rho = s_buf[F_RHO * NODES + i];
    o.u1 = s_buf[F_U1 * NODES + i];
    o.u2 = s_buf[F_U2 * NODES + i];
    o.u3 = s_buf[F_U3 * NODES + i];
    o.beta = s_buf[F_B * NODES + i];
    o.lrho = s_buf[F_LR * NODES + i];
    o.lbeta = s_buf[F_LB * NODES + i];
    o.k = s_buf[F_K * NODES + i];
    return o;
}

// Volume term of one direction along the plane's lines:
//   acc -= sum_j D(i, j) (A_i + A_j) . F#(q_i, q_j)          (two-point fluxes), or
//   acc -= sum_j D(i, j) A_j . F(q_j)                         (standard DC form).
// For two-point fluxes every pair is evaluated once: in round r a node takes the pair with the
// node r places further along its line (cyclically), keeps D(i, j) f and leaves D(j, i) f in the
// partner's mailbox.  The metric rows of consecutive calls alternate between two LDS areas
// (slot = 0, 1) and the mailboxes between two areas by `round`, so one barrier per round suffices.
// All threads of the block call it; `on` marks threads that own a node; ls is the LDS stride of the
// direction and il the node's index along it.
template <int N, int FLUX>
__device__ __forceinline__ void line_volume(double *s_buf, int NODES, const double *s_D, int tid,
                                            bool on, int il, int ls, const double Al[3], int slot,
                                            int &round, const Node &me, double Pme, double rhoE,
                                            double gm1, double acc[5]) {
    if constexpr (FLUX == 3) {
        if (on) {
            double f[5];
            euler_flux_n(me, Pme, rhoE, Al[0], Al[1], Al[2], f);
#pragma unroll
            for (int c = 0; c < 5; ++c) s_buf[(F_MSG0 + c) * NODES + tid] = f[c];
        }
        __syncthreads();
        if (on) {
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const double dd = s_D[il * N + b];
                const int pn = tid + (b - il) * ls;
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] = fma(-dd, s_buf[(F_MSG0 + c) * NODES + pn], acc[c]);
            }
        }
        __syncthreads();
    } else {
        const int fa = slot ? F_A1 : F_A0;
        if (on) {
            s_buf[(fa + 0) * NODES + tid] = Al[0];
            s_buf[(fa + 1) * NODES + tid] = Al[1];
            s_buf[(fa + 2) * NODES + tid] = Al[2];
        }
        __syncthreads();
        auto pair = [&](int b, double f[5]) {
            const int pn = tid + (b - il) * ls;
            const Node o = staged_node(s_buf, NODES, pn);
            const double n0 = Al[0] + s_buf[(fa + 0) * NODES + pn];
            const double n1 = Al[1] + s_buf[(fa + 1) * NODES + pn];
            const double n2 = Al[2] + s_buf[(fa + 2) * NODES + pn];
            flux_n<FLUX>(me, o, n0, n1, n2, gm1, f);
            return pn;
        };
#pragma unroll
        for (int r = 1; 2 * r < N; ++r) {
            const int fm = (round & 1) ? F_MSG1 : F_MSG0;
            ++round;
            int b = il + r;
            if (b >= N) b -= N;
            if (on) {
                double f[5];
                const int pn = pair(b, f);
                const double dab = s_D[il * N + b], dba = s_D[b * N + il];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    acc[c] = fma(-dab, f[c], acc[c]);
                    s_buf[(fm + c) * NODES + pn] = dba * f[c];
                }
            }
            __syncthreads();
            if (on) {
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] -= s_buf[(fm + c) * NODES + tid];
            }
        }
        if constexpr (N % 2 == 0) {
            if (on) {
                int b = il + N / 2;
                if (b >= N) b -= N;
                double f[5];
                pair(b, f);
                const double dab = s_D[il * N + b];
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] = fma(-dab, f[c], acc[c]);
            }
        }
    }
}

// D along a line of a staged plane field block: sum_b D(il, b) s[pn(b)] for 4 components.
template <int N>
__device__ __forceinline__ void line_grad4(const double *s_buf, int NODES, int field, const double *s_D,
                                           int tid, int il, int ls, double out[4]) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
        const double dd = s_D[il * N + b];
        const int pn = tid + (b - il) * ls;
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c] = fma(dd, s_buf[(field + c) * NODES + pn], out[c]);
    }
}

// Locates the block's problem and its first plane.
__device__ __forceinline__ int plane_problem(const GroupArgs &g, long long &vb) {
    vb = xcd_block(blockIdx.x, gridDim.x);
    return find_problem(g.block_start, g.n, vb);
}

// ---- pass A: planes of constant xi3 (directions xi1, xi2) -------------------------------------
template <int N, int PPB, bool VISC, int FLUX, bool MD, bool OR>
__global__ void __launch_bounds__(NT_OF(PPB * N * N)) k_plane_a(const GroupArgs g) {
    constexpr int N2 = N * N, N3 = N2 * N, NODES = PPB * N2;
    constexpr int ITEMS = PPB * 4 * N;  // face nodes of the plane: 2 directions x 2 sides x N
    constexpr int NV = VISC ? 9 : 5;
    static_assert(NV * ITEMS <= (PLANE_FIELDS - 8) * NODES, "face slots exceed the LDS tile");
    __shared__ double s_buf[PLANE_FIELDS * NODES];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    if (tid < N2) s_D[tid] = g.D[tid];
    long long vb;
    const int pb = plane_problem(g, vb);
    const ResArgs a = problem_view(g, g.probs[pb], g.out);
    const long long nodes = a.nodes, nplanes = a.K * N;
    const long long P0 = (vb - g.block_start[pb]) * PPB;
    const int pp = tid / N2, ln = tid - pp * N2;
    const long long pl = P0 + pp;
    const bool on = tid < NODES && pl < nplanes;
    const int i1 = ln % N, i2 = ln / N;
    const long long gn = pl * N2 + ln;  // = e N^3 + i1 + N i2 + N^2 i3
    const double gm1 = a.gamma - 1.0;

    double q[5], A0[3], A1[3];
    if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = a.q[c * nodes + gn];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            A0[m] = a.metric[m * nodes + gn];
            A1[m] = a.metric[(3 + m) * nodes + gn];
        }
    } else {
        q[0] = 1.0; q[1] = q[2] = q[3] = 0.0; q[4] = 1.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) A0[m] = A1[m] = 0.0;
    }
    Node me;
    double Pme;
    bool ok;
    primitives(q, gm1, me, Pme, ok);
    if (on && !ok) atomicOr(a.status, FLAG_NONPHYSICAL);
    if (tid < NODES) stage_node(s_buf, NODES, tid, me);

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int round = 0;
    line_volume<N, FLUX>(s_buf, NODES, s_D, tid, tid < NODES, i1, 1, A0, 0, round, me, Pme, q[4], gm1, acc);
    line_volume<N, FLUX>(s_buf, NODES, s_D, tid, tid < NODES, i2, N, A1, 1, round, me, Pme, q[4], gm1, acc);
    __syncthreads();

    // interface terms of the xi1 and xi2 faces as (face, face node) items
    double *fsl = s_buf + 8 * NODES;  // [NV][ITEMS]
    for (int it = tid; it < ITEMS; it += blockDim.x) {
        const int ip = it / (4 * N), rem = it - ip * 4 * N;
        const int f = rem / N, t = rem - f * N;  // f = 2 l + side, l in {0, 1}
        const int l = f >> 1, side = f & 1;
        const long long ipl = P0 + ip;
        double v[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] = 0.0;
        if (ipl < nplanes) {
            const long long e = ipl / N;
            const int j3 = (int)(ipl - e * N);
            const long long nb = a.nbr[e * 6 + f];
            const int kind = face_kind(a, nb);
            if (kind == FACE_INVALID) {
                atomicOr(a.status, FLAG_MESH);
            } else {
                const int il = side ? N - 1 : 0;
                const int j1 = l == 0 ? il : t, j2 = l == 0 ? t : il;
                const int lno = j1 + N * j2 + N2 * j3;
                const long long go = e * N3 + lno;
                long long pg = go;
                int lp = l;
                double sg = 1.0;
                if (kind == FACE_INTERIOR) {
                    const FaceLink k = face_link<N, OR>(a, e, f, t, j3, lno + (N - 1 - 2 * il) * (l == 0 ? 1 : N));
                    if (!k.ok) atomicOr(a.status, FLAG_MESH);
                    pg = nb * N3 + k.lno;
                    lp = k.fp >> 1;
                    sg = k.sg;
                }
                double qi[5], Ai[3];
#pragma unroll
                for (int c = 0; c < 5; ++c) qi[c] = a.q[c * nodes + go];
#pragma unroll
                for (int m = 0; m < 3; ++m) Ai[m] = a.metric[(3 * l + m) * nodes + go];
                const Node mi = staged_node(s_buf, NODES, ip * N2 + j1 + N * j2);
                const double Pi = gm1 * (qi[4] - 0.5 * qi[0] * mi.k);
                const double iJi = (VISC && a.eta != 0.0) ? rcp(a.jac[go]) : 1.0;
                face_terms<FLUX, VISC, MD>(a, face_own(a, mi, Pi, qi, iJi), Ai, pg, kind, lp, sg,
                                           side ? 1.0 : -1.0, v);
            }
        }
#pragma unroll
        for (int c = 0; c < NV; ++c) fsl[c * ITEMS + it] = v[c];
    }
    __syncthreads();
    double dth[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    if (on) {
        const int idx[2] = {i1, i2};
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            if (idx[l] != 0 && idx[l] != N - 1) continue;
            const int side = idx[l] == N - 1 ? 1 : 0;
            const int it = pp * 4 * N + (2 * l + side) * N + (l == 0 ? i2 : i1);
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[c] += fsl[c * ITEMS + it];
            if constexpr (VISC) {
#pragma unroll
                for (int c = 0; c < 4; ++c) dth[l][c] = fsl[(5 + c) * ITEMS + it];
            }
        }
    }

    if constexpr (VISC) {
        // BR1 gradients theta_1, theta_2 (w = (U/T, -1/T); W_1 is not needed)
        const double iT = 2.0 * a.R * me.beta;
        if (tid < NODES) {
            s_buf[0 * NODES + tid] = me.u1 * iT;
            s_buf[1 * NODES + tid] = me.u2 * iT;
            s_buf[2 * NODES + tid] = me.u3 * iT;
            s_buf[3 * NODES + tid] = -iT;
        }
        __syncthreads();
        if (on) {
            line_grad4<N>(s_buf, NODES, 0, s_D, tid, i1, 1, dth[0]);
            line_grad4<N>(s_buf, NODES, 0, s_D, tid, i2, N, dth[1]);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a.aux[(AUX_TH + c) * nodes + gn] = dth[0][c];
                a.aux[(AUX_TH + 4 + c) * nodes + gn] = dth[1][c];
            }
        }
    }
    if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) a.out[c * nodes + gn] = acc[c];
    }
}

// ---- pass B: planes of constant xi2 (direction xi3) --------------------------------------------
template <int N, int PPB, bool VISC, int FLUX, bool MD, bool OR>
__global__ void __launch_bounds__(NT_OF(PPB * N * N)) k_plane_b(const GroupArgs g) {
    constexpr int N2 = N * N, N3 = N2 * N, NODES = PPB * N2;
    constexpr int ITEMS = PPB * 2 * N;  // face nodes of the plane: 2 sides x N
    constexpr int NV = VISC ? 9 : 5;
    static_assert(NV * ITEMS <= (PLANE_FIELDS - 8) * NODES, "face slots exceed the LDS tile");
    __shared__ double s_buf[PLANE_FIELDS * NODES];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    if (tid < N2) s_D[tid] = g.D[tid];
    long long vb;
    const int pb = plane_problem(g, vb);
    const ResArgs a = problem_view(g, g.probs[pb], g.out);
    const long long nodes = a.nodes, nplanes = a.K * N;
    const long long P0 = (vb - g.block_start[pb]) * PPB;
    const int pp = tid / N2, ln = tid - pp * N2;  // ln = i1 + N i3
    const long long pl = P0 + pp;
    const bool on = tid < NODES && pl < nplanes;
    const int i1 = ln % N, i3 = ln / N;
    const long long e = pl / N;
    const int i2 = (int)(pl - e * N);
    const long long gn = e * N3 + i1 + N * i2 + N2 * i3;
    const double gm1 = a.gamma - 1.0;

    double q[5], A[3][3], J = 1.0;
    if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = a.q[c * nodes + gn];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                A[l][m] = (VISC || l == 2) ? a.metric[(3 * l + m) * nodes + gn] : 0.0;
        J = a.jac[gn];
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
    if (on && !ok) atomicOr(a.status, FLAG_NONPHYSICAL);
    if (tid < NODES) stage_node(s_buf, NODES, tid, me);

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int round = 0;
    line_volume<N, FLUX>(s_buf, NODES, s_D, tid, tid < NODES, i3, N, A[2], 0, round, me, Pme, q[4], gm1, acc);
    __syncthreads();

    double *fsl = s_buf + 8 * NODES;  // [NV][ITEMS]
    for (int it = tid; it < ITEMS; it += blockDim.x) {
        const int ip = it / (2 * N), rem = it - ip * 2 * N;
        const int side = rem / N, t = rem - side * N;  // t = i1 of the face node
        const long long ipl = P0 + ip;
        double v[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] = 0.0;
        if (ipl < nplanes) {
            const long long ee = ipl / N;
            const int j2 = (int)(ipl - ee * N);
            const long long nb = a.nbr[ee * 6 + 4 + side];
            const int kind = face_kind(a, nb);
            if (kind == FACE_INVALID) {
                atomicOr(a.status, FLAG_MESH);
            } else {
                const int il = side ? N - 1 : 0;
                const int lno = t + N * j2 + N2 * il;
                const long long go = ee * N3 + lno;
                long long pg = go;
                int lp = 2;
                double sg = 1.0;
                if (kind == FACE_INTERIOR) {
                    const FaceLink k = face_link<N, OR>(a, ee, 4 + side, t, j2, lno + (N - 1 - 2 * il) * N2);
                    if (!k.ok) atomicOr(a.status, FLAG_MESH);
                    pg = nb * N3 + k.lno;
                    lp = k.fp >> 1;
                    sg = k.sg;
                }
                double qi[5], Ai[3];
#pragma unroll
                for (int c = 0; c < 5; ++c) qi[c] = a.q[c * nodes + go];
#pragma unroll
                for (int m = 0; m < 3; ++m) Ai[m] = a.metric[(6 + m) * nodes + go];
                const Node mi = staged_node(s_buf, NODES, ip * N2 + t + N * il);
                const double Pi = gm1 * (qi[4] - 0.5 * qi[0] * mi.k);
                const double iJi = (VISC && a.eta != 0.0) ? rcp(a.jac[go]) : 1.0;
                face_terms<FLUX, VISC, MD>(a, face_own(a, mi, Pi, qi, iJi), Ai, pg, kind, lp, sg,
                                           side ? 1.0 : -1.0, v);
            }
        }
#pragma unroll
        for (int c = 0; c < NV; ++c) fsl[c * ITEMS + it] = v[c];
    }
    __syncthreads();
    double th2[4] = {0.0, 0.0, 0.0, 0.0};
    bool face3 = false, wall3 = false;
    const int side3 = i3 == N - 1 ? 1 : 0;
    if (on && (i3 == 0 || i3 == N - 1)) {
        const int it = pp * 2 * N + side3 * N + i1;
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[c] += fsl[c * ITEMS + it];
        if constexpr (VISC) {
#pragma unroll
            for (int c = 0; c < 4; ++c) th2[c] = fsl[(5 + c) * ITEMS + it];
        }
        const long long nb = a.nbr[e * 6 + 4 + side3];
        face3 = nb >= 0 && nb < a.K;
        wall3 = face_kind(a, nb) == FACE_WALL;
    }
    if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[c] += a.out[c * nodes + gn];  // pass A's terms
    }
    const double iJ = rcp(J);

    if constexpr (VISC) {
        const double iT = 2.0 * a.R * me.beta;
        const double T = rcp(iT);
        if (tid < NODES) {
            s_buf[0 * NODES + tid] = me.u1 * iT;
            s_buf[1 * NODES + tid] = me.u2 * iT;
            s_buf[2 * NODES + tid] = me.u3 * iT;
            s_buf[3 * NODES + tid] = -iT;
        }
        __syncthreads();
        double th[3][4];
#pragma unroll
        for (int c = 0; c < 4; ++c) th[2][c] = th2[c];
        if (on) {
            line_grad4<N>(s_buf, NODES, 0, s_D, tid, i3, N, th[2]);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                th[0][c] = a.aux[(AUX_TH + c) * nodes + gn];
                th[1][c] = a.aux[(AUX_TH + 4 + c) * nodes + gn];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) th[0][c] = th[1][c] = 0.0;
        }
        double gr[3][4];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                gr[j][c] = (A[0][j] * th[0][c] + A[1][j] * th[1][c] + A[2][j] * th[2][c]) * iJ;
        double FV[3][4];
        visc_flux_full(gr, me.u1, me.u2, me.u3, T, a.mu, a.kap, FV);
        double fh[3][4];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                fh[l][c] = fma(A[l][0], FV[0][c], fma(A[l][1], FV[1][c], A[l][2] * FV[2][c]));
        if (on) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a.aux[(AUX_FH + c) * nodes + gn] = fh[0][c];
                a.aux[(AUX_FH + 4 + c) * nodes + gn] = fh[1][c];
            }
            if (i3 == 0 || i3 == N - 1) {
                SBP_GLOBAL double *tr = a.trace + ((e * 6 + 4 + side3) * 4) * N2 + i1 + N * i2;
#pragma unroll
                for (int c = 0; c < 4; ++c) tr[c * N2] = fh[2][c];
                if (face3) {
                    const double cs = -0.5 * (side3 ? 1.0 : -1.0) * a.isw;
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c + 1] = fma(cs, fh[2][c], acc[c + 1]);
                } else if (wall3) {
                    // adiabatic wall: no energy part in the boundary viscous flux
                    acc[4] = fma(-(side3 ? 1.0 : -1.0) * a.isw, fh[2][3], acc[4]);
                }
            }
        }
        __syncthreads();
        if (tid < NODES) {
#pragma unroll
            for (int c = 0; c < 4; ++c) s_buf[(4 + c) * NODES + tid] = fh[2][c];
        }
        __syncthreads();
        if (on) {
            double dv[4] = {0.0, 0.0, 0.0, 0.0};
            line_grad4<N>(s_buf, NODES, 4, s_D, tid, i3, N, dv);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c + 1] += dv[c];
#pragma unroll
            for (int c = 0; c < 5; ++c) a.out[c * nodes + gn] = acc[c];
        }
    } else {
        if (on) {
#pragma unroll
            for (int c = 0; c < 5; ++c)
                a.out[c * nodes + gn] = a.src ? fma(acc[c], iJ, a.src[c * nodes + gn]) : acc[c] * iJ;
        }
    }
}

// ---- pass C (viscous): planes of constant xi3, divergence of fhat_1, fhat_2, SAT^V, 1/J ---------
template <int N, int PPB>
__global__ void __launch_bounds__(NT_OF(PPB * N * N)) k_plane_c(const GroupArgs g) {
    constexpr int N2 = N * N, N3 = N2 * N, NODES = PPB * N2;
    __shared__ double s_buf[8 * NODES];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    if (tid < N2) s_D[tid] = g.D[tid];
    long long vb;
    const int pb = plane_problem(g, vb);
    const ResArgs a = problem_view(g, g.probs[pb], g.out);
    const long long nodes = a.nodes, nplanes = a.K * N;
    const long long P0 = (vb - g.block_start[pb]) * PPB;
    const int pp = tid / N2, ln = tid - pp * N2;
    const long long pl = P0 + pp;
    const bool on = tid < NODES && pl < nplanes;
    const int i1 = ln % N, i2 = ln / N;
    const long long e = pl / N;
    const int i3 = (int)(pl - e * N);
    const long long gn = pl * N2 + ln;
    double fh[2][4];
    if (on) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            fh[0][c] = a.aux[(AUX_FH + c) * nodes + gn];
            fh[1][c] = a.aux[(AUX_FH + 4 + c) * nodes + gn];
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) fh[0][c] = fh[1][c] = 0.0;
    }
    if (tid < NODES) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            s_buf[c * NODES + tid] = fh[0][c];
            s_buf[(4 + c) * NODES + tid] = fh[1][c];
        }
    }
    __syncthreads();
    if (!on) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    line_grad4<N>(s_buf, NODES, 0, s_D, tid, i1, 1, acc);
    line_grad4<N>(s_buf, NODES, 4, s_D, tid, i2, N, acc);
    // SAT^V = (s / (2 w_end)) (fhat_l,nu - fhat_l,i) on every face of the node
    const int idx[3] = {i1, i2, i3};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int il = idx[l];
        if (il != 0 && il != N - 1) continue;
        const int side = il == N - 1 ? 1 : 0;
        const long long nb = a.nbr[e * 6 + 2 * l + side];
        if (nb < 0 || nb >= a.K) {
            // adiabatic wall across a xi1 or xi2 face (xi3 walls are done in pass B)
            if (l < 2 && face_kind(a, nb) == FACE_WALL)
                acc[3] = fma(-(side ? 1.0 : -1.0) * a.isw, fh[l][3], acc[3]);
            continue;
        }
        const double cs = 0.5 * (side ? 1.0 : -1.0) * a.isw;
        // the neighbour's fhat of its direction l' at the partner node: the per-node scratch
        // for l' = 0, 1, the xi3 face trace for l' = 2
        const int ta = l == 0 ? i2 : i1, tb = l == 2 ? i2 : i3;
        const int lne = (int)(gn - e * N3);  // element-local node index
        const FaceLink k = face_link<N>(a, e, 2 * l + side, ta, tb,
                                        lne + (N - 1 - 2 * il) * (l == 0 ? 1 : (l == 1 ? N : N2)));
        const int lp = k.fp >> 1;
        double fn[4];
        if (lp < 2) {
            const long long pg = nb * N3 + k.lno;
#pragma unroll
            for (int c = 0; c < 4; ++c) fn[c] = k.sg * a.aux[(AUX_FH + 4 * lp + c) * nodes + pg];
        } else {
            const SBP_GLOBAL double *tr = a.trace + ((nb * 6 + k.fp) * 4) * N2 + k.tp;
#pragma unroll
            for (int c = 0; c < 4; ++c) fn[c] = k.sg * tr[c * N2];
        }
        if (l < 2) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = fma(cs, fn[c] - fh[l][c], acc[c]);
        } else {
            // the own half was added with the xi3 divergence
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = fma(cs, fn[c], acc[c]);
        }
    }
    const double iJ = rcp(a.jac[gn]);
    double r[5];
    r[0] = a.out[gn] * iJ;
#pragma unroll
    for (int c = 0; c < 4; ++c) r[c + 1] = (a.out[(c + 1) * nodes + gn] + acc[c]) * iJ;
#pragma unroll
    for (int c = 0; c < 5; ++c) a.out[c * nodes + gn] = a.src ? r[c] + a.src[c * nodes + gn] : r[c];
}

// Curl-form metrics for elements too large for one thread per node: a workgroup holds the
// element's coordinates in LDS and walks its nodes.
template <int N>
__global__ void __launch_bounds__(256)
k_metrics_big(const double *x, double *metric, double *jac, const double *D, long long K) {
    constexpr int N2 = N * N, N3 = N2 * N, PER = (N3 + 255) / 256;
    __shared__ double s_x[3 * N3];
    __shared__ double s_V[N3];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    const long long e = blockIdx.x;
    const long long nodes = K * N3;
    for (int i = tid; i < N2; i += 256) s_D[i] = D[i];
    for (int i = tid; i < 3 * N3; i += 256) {
        const int m = i / N3, n = i - m * N3;
        s_x[i] = x[m * nodes + e * N3 + n];
    }
    __syncthreads();
    auto dl = [&](const double *arr, int node, int dir) {
        const int st = dir == 0 ? 1 : (dir == 1 ? N : N2);
        const int il = (node / st) % N;
        double r = 0.0;
        for (int b = 0; b < N; ++b) r = fma(s_D[il * N + b], arr[node + (b - il) * st], r);
        return r;
    };
    for (int k = 0; k < PER; ++k) {
        const int node = tid + 256 * k;
        if (node >= N3) break;
        double dx[3][3];
        for (int m = 0; m < 3; ++m)
            for (int i = 0; i < 3; ++i) dx[m][i] = dl(s_x + m * N3, node, i);
        jac[e * N3 + node] = dx[0][0] * (dx[1][1] * dx[2][2] - dx[1][2] * dx[2][1]) -
                             dx[0][1] * (dx[1][0] * dx[2][2] - dx[1][2] * dx[2][0]) +
                             dx[0][2] * (dx[1][0] * dx[2][1] - dx[1][1] * dx[2][0]);
    }
    for (int n = 0; n < 3; ++n) {
        const int m = (n + 1) % 3, l = (n + 2) % 3;
        double cc[PER][3];
        for (int k = 0; k < PER; ++k) cc[k][0] = cc[k][1] = cc[k][2] = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            __syncthreads();
            for (int node = tid; node < N3; node += 256)
                s_V[node] = s_x[l * N3 + node] * dl(s_x + m * N3, node, i);
            __syncthreads();
            // V_i enters c_(i+1) through D_(i+2) with + and c_(i+2) through D_(i+1) with -
            for (int k = 0; k < PER; ++k) {
                const int node = tid + 256 * k;
                if (node >= N3) break;
                cc[k][(i + 1) % 3] += dl(s_V, node, (i + 2) % 3);
                cc[k][(i + 2) % 3] -= dl(s_V, node, (i + 1) % 3);
            }
        }
        for (int k = 0; k < PER; ++k) {
            const int node = tid + 256 * k;
            if (node >= N3) break;
            for (int ii = 0; ii < 3; ++ii) metric[(3 * ii + n) * nodes + e * N3 + node] = -cc[k][ii];
        }
    }
}

template <int N, int PPB, bool VISC, int FLUX, bool MD, bool OR = false>
int launch_planes_k(const GroupArgs &g, hipStream_t s) {
    constexpr int NT = NT_OF(PPB * N * N);
    const dim3 grid((unsigned)g.total_blocks);
    KernelTimer &tm = residual_timer();
    if (tm.enabled && hipEventRecord(tm.begin, s) != hipSuccess) return -1;
    hipLaunchKernelGGL((k_plane_a<N, PPB, VISC, FLUX, MD, OR>), grid, dim3(NT), 0, s, g);
    hipLaunchKernelGGL((k_plane_b<N, PPB, VISC, FLUX, MD, OR>), grid, dim3(NT), 0, s, g);
    if constexpr (VISC) hipLaunchKernelGGL((k_plane_c<N, PPB>), grid, dim3(NT), 0, s, g);
    if (hipGetLastError() != hipSuccess) return -1;
    if (tm.enabled && hipEventRecord(tm.end, s) != hipSuccess) return -1;
    return 0;
}

template <int N, int PPB>
int launch_planes_f(bool visc, int flux, const GroupArgs &g, hipStream_t s) {
    switch (flux) {
        case 0: return visc ? launch_planes_k<N, PPB, true, 0, false>(g, s) : launch_planes_k<N, PPB, false, 0, false>(g, s);
        case 1: return visc ? launch_planes_k<N, PPB, true, 1, false>(g, s) : launch_planes_k<N, PPB, false, 1, false>(g, s);
        case 2: return visc ? launch_planes_k<N, PPB, true, 2, false>(g, s) : launch_planes_k<N, PPB, false, 2, false>(g, s);
        case 3: return visc ? launch_planes_k<N, PPB, true, 3, false>(g, s) : launch_planes_k<N, PPB, false, 3, false>(g, s);
        default: return -1;
    }
}

// Matrix interface dissipation: one plane per workgroup, Chandrashekar and Kennedy-Gruber fluxes.
template <int N>
int launch_planes_md(bool visc, int flux, const GroupArgs &g, hipStream_t s) {
    switch (flux) {
        case 0: return visc ? launch_planes_k<N, 1, true, 0, true>(g, s) : launch_planes_k<N, 1, false, 0, true>(g, s);
        case 2: return visc ? launch_planes_k<N, 1, true, 2, true>(g, s) : launch_planes_k<N, 1, false, 2, true>(g, s);
        default: return -1;
    }
}

// Problems with a face-orientation table: one plane per workgroup, every flux and dissipation.
template <int N>
int launch_planes_or(bool visc, int flux, bool md, const GroupArgs &g, hipStream_t s) {
    if (md) {
        switch (flux) {
            case 0: return visc ? launch_planes_k<N, 1, true, 0, true, true>(g, s) : launch_planes_k<N, 1, false, 0, true, true>(g, s);
            case 2: return visc ? launch_planes_k<N, 1, true, 2, true, true>(g, s) : launch_planes_k<N, 1, false, 2, true, true>(g, s);
            default: return -1;
        }
    }
    switch (flux) {
        case 0: return visc ? launch_planes_k<N, 1, true, 0, false, true>(g, s) : launch_planes_k<N, 1, false, 0, false, true>(g, s);
        case 1: return visc ? launch_planes_k<N, 1, true, 1, false, true>(g, s) : launch_planes_k<N, 1, false, 1, false, true>(g, s);
        case 2: return visc ? launch_planes_k<N, 1, true, 2, false, true>(g, s) : launch_planes_k<N, 1, false, 2, false, true>(g, s);
        case 3: return visc ? launch_planes_k<N, 1, true, 3, false, true>(g, s) : launch_planes_k<N, 1, false, 3, false, true>(g, s);
        default: return -1;
    }
}

template <int N>
int launch_planes_n(int ppb, bool visc, int flux, bool md, bool orient, const GroupArgs &g,
                    hipStream_t s) {
    if (orient) return ppb == 1 ? launch_planes_or<N>(visc, flux, md, g, s) : -1;
    if (md) return ppb == 1 ? launch_planes_md<N>(visc, flux, g, s) : -1;
    return ppb == 2 ? launch_planes_f<N, 2>(visc, flux, g, s) : launch_planes_f<N, 1>(visc, flux, g, s);
}

}  // namespace

int launch_group_residual_planes(int p, int ppb, bool visc, int flux, bool md, bool orient,
                                 const GroupArgs &g, hipStream_t s) {
    switch (p) {
        case 9: return launch_planes_n<10>(ppb, visc, flux, md, orient, g, s);
        case 10: return launch_planes_n<11>(ppb, visc, flux, md, orient, g, s);
        case 11: return launch_planes_n<12>(ppb, visc, flux, md, orient, g, s);
        case 12: return launch_planes_n<13>(ppb, visc, flux, md, orient, g, s);
        case 13: return launch_planes_n<14>(ppb, visc, flux, md, orient, g, s);
        case 14: return launch_planes_n<15>(ppb, visc, flux, md, orient, g, s);
        case 15: return launch_planes_n<16>(ppb, visc, flux, md, orient, g, s);
        default: return -1;
    }
}

int launch_metrics_big(int p, long long K, const double *x, double *metric, double *jac,
                       const double *D, hipStream_t s) {
#define SBP_MET(NN)                                                                              \
    hipLaunchKernelGGL((k_metrics_big<NN>), dim3((unsigned)K), dim3(256), 0, s, x, metric, jac, D, K); \
    break;
    switch (p) {
        case 10: SBP_MET(11)
        case 11: SBP_MET(12)
        case 12: SBP_MET(13)
        case 13: SBP_MET(14)
        case 14: SBP_MET(15)
        case 15: SBP_MET(16)
        default: return -1;
    }
#undef SBP_MET
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sbp
