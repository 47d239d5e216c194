// gfx950 kernels of the ES-C SBP-SAT residual (arXiv 1911.10966, section "Discretization of the
// compressible Navier-Stokes equations").  FP64 throughout.
//
// Residual kernel layout: one workgroup holds EPW elements, one thread per node (wave64 tiles of
// the element's N^3 nodes).  Node data needed by line partners (rho, U, beta = rho/(2P), log rho,
// log beta, |U|^2, the metric row of the current direction) is staged in LDS.  The flux-differencing
// sum over each line uses the symmetry of the two-point flux: in round r a node evaluates the pair
// with the node r places further along the line (cyclically), keeps D(a,b) f and hands D(b,a) f to
// its partner through an LDS mailbox, so every pair is evaluated once.
#include "sbp_device.h"

namespace sbp {
namespace {

// Doubles of LDS per node in the residual kernel.  Viscous tiles: node data (8), two metric-row
// areas (6), two mailboxes (10).  Inviscid tiles use fewer registers, so LDS is what limits their
// occupancy: they keep one metric-row area and recompute |U|^2 of a partner instead of staging it,
// 20 fields, which lets a CU hold 4 waves per SIMD of N = 5 elements.  For N >= 6 the face slots of
// the interface work items (6 N^2 x 9 or x 5 per element) reuse the fields from 8 on.
constexpr int tile_fields(bool visc) { return visc ? 24 : 20; }

// Doubles between consecutive LDS fields: the node count rounded up to a multiple of 64 when that
// costs at most 5% more LDS.  Fields then lie a multiple of 512 bytes apart, so the reads of all
// fields of one node pair up in ds_read2st64 instructions from a single address.
constexpr int field_stride(int nodes) {
    const int r = (nodes + 63) / 64 * 64;
    return (r - nodes) * 20 <= nodes ? r : nodes;
}

// Element size from which the interface terms run as (face, face node) work items.
constexpr int kFaceItemsFrom = 6;

// D along the cyclic pairing of the pair loop, row-major in (round, node index i): rows
// r - 1 = 0 .. N/2 - 1 hold D(i, i + r), rows N/2 + r - 1 hold D(i, i - r) (indices mod N), so
// that a round reads its weights at a constant offset from the node's own index.
template <int N>
constexpr int kRotRows = N / 2 + (N - 1) / 2;
template <int N>
__device__ __forceinline__ double rotated_D(const double *D, int t) {
    const int row = t / N, i = t - row * N;
    const int j = row < N / 2 ? (i + row + 1) % N : (i - (row - N / 2 + 1) + N) % N;
    return D[i * N + j];
}

// One tile of EPW elements (first element ebase) of one problem; all threads of the block call it.
// MD: matrix interface dissipation (iface_diss = 2) instead of Lax-Friedrichs.  OR: the problem has
// a face-orientation table (unstructured faces); without it the aligned partners are compiled in.
template <int N, int EPW, bool VISC, int FLUX, bool MD, bool OR>
__device__ __forceinline__ void residual_tile(const ResArgs &a, long long ebase, double *s_buf,
                                              const double *s_D, const double *s_Dr, int *s_face) {
    constexpr int N2 = N * N, N3 = N * N * N, NODES = EPW * N3;
    constexpr int FS = field_stride(NODES);
    constexpr bool COMPACT = !VISC;  // see tile_fields
    constexpr int LDS_FIELDS = tile_fields(VISC);
    constexpr int F_RHO = 0, F_U1 = 1, F_U2 = 2, F_U3 = 3, F_B = 4, F_LR = 5, F_LB = 6;
    constexpr int F_K = COMPACT ? -1 : 7;
    constexpr int F_A0 = COMPACT ? 7 : 8, F_A1 = COMPACT ? 7 : 11;
    constexpr int F_MSG0 = COMPACT ? 10 : 14, F_MSG1 = COMPACT ? 15 : 19;

    const int tid = threadIdx.x;
    const int slot = tid / N3;
    const int ln = tid - slot * N3;
    const long long e = ebase + slot;
    const bool active = (tid < NODES) && (e < a.K);
    const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
    const int idx[3] = {i1, i2, i3};
    const int stride[3] = {1, N, N2};
    const long long nodes = a.nodes;
    const long long g = e * N3 + ln;
    const double gm1 = a.gamma - 1.0;
    const double isw = a.isw;

    // ---- node-local primitives --------------------------------------------------------------
    double q[5];
    double A[3][3];
    double J = 1.0;
    if (active) {
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = a.q[c * nodes + g];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[l][m] = a.metric[(3 * l + m) * nodes + g];
        J = a.jac[g];
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
    // The entropy-conservative pair loop works on halves (flux_pair_half): rho, U and |U|^2 of the
    // node are scaled by 1/2, 1/2 and 1/4 here, staged so, and scaled back exactly after the loop.
    constexpr bool HALF = (FLUX == 0);
    if constexpr (HALF) {
        me.rho *= 0.5;
        me.u1 *= 0.5;
        me.u2 *= 0.5;
        me.u3 *= 0.5;
        me.k *= 0.25;
    }
    if (tid < NODES) {
        s_buf[F_RHO * FS + tid] = me.rho;
        s_buf[F_U1 * FS + tid] = me.u1;
        s_buf[F_U2 * FS + tid] = me.u2;
        s_buf[F_U3 * FS + tid] = me.u3;
        s_buf[F_B * FS + tid] = me.beta;
        s_buf[F_LR * FS + tid] = me.lrho;
        s_buf[F_LB * FS + tid] = me.lbeta;
        if constexpr (!COMPACT) s_buf[F_K * FS + tid] = me.k;
    }
    // neighbour index and kind of the tile's faces, decoded once per face (visible to all threads
    // after the first barrier below); a mesh error is flagged here
    if (tid < EPW * 6) {
        const long long ee = ebase + tid / 6;
        int nbv = 0, kind = FACE_INVALID;
        if (ee < a.K) {
            const long long nb = a.nbr[ee * 6 + tid % 6];
            kind = face_kind(a, nb);
            if (kind == FACE_INVALID) atomicOr(a.status, FLAG_MESH);
            nbv = (int)nb;
        }
        s_face[2 * tid] = nbv;
        s_face[2 * tid + 1] = kind;
    }

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    // ---- inviscid volume term: -sum_l sum_j D(i_l, j_l) (A_l,i + A_l,j) . F#(q_i, q_j) ----------
    // (the j = i terms cancel exactly against the own-flux part of the interface SAT).  The metric
    // rows of consecutive directions and the mailboxes of consecutive rounds alternate between two
    // LDS areas, so one barrier per round suffices.
    if constexpr (FLUX == 3) {
        // standard DC: -sum_l D_l (A_l . F) with the nodal fluxes, one direction at a time
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (tid < NODES) {
                double f[5];
                euler_flux_n(me, Pme, q[4], A[l][0], A[l][1], A[l][2], f);
#pragma unroll
                for (int c = 0; c < 5; ++c) s_buf[(F_MSG0 + c) * FS + tid] = f[c];
            }
            __syncthreads();
            if (tid < NODES) {
                const int il = idx[l];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const double dd = s_D[il * N + b];
                    const int pn = tid + (b - il) * stride[l];
#pragma unroll
                    for (int c = 0; c < 5; ++c) acc[c] = fma(-dd, s_buf[(F_MSG0 + c) * FS + pn], acc[c]);
                }
            }
            __syncthreads();
        }
    } else {
        int round = 0;
        const double igm1 = 1.0 / gm1;
        // With two metric areas, the next direction's row goes into the other area during the last
        // full round of the current direction and is published by that round's barrier.  The other
        // area was last read by the previous direction, whose reads all precede a barrier of the
        // current direction unless a half-round (even N) follows its last barrier and the current
        // direction has only one full round; those cases stage after the rounds, with a barrier.
        constexpr bool EARLY = !COMPACT && (N % 2 == 1 ? N >= 3 : N >= 6);
    #pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int fa = (l & 1) ? F_A1 : F_A0;
            if constexpr (COMPACT && N % 2 == 0) {
                // one metric area: the last half-round of the previous direction still reads it
                if (l > 0) __syncthreads();
            }
            if (!EARLY || l == 0) {
                if (tid < NODES) {
                    s_buf[(fa + 0) * FS + tid] = A[l][0];
                    s_buf[(fa + 1) * FS + tid] = A[l][1];
                    s_buf[(fa + 2) * FS + tid] = A[l][2];
                }
                __syncthreads();
            }
            const int il = idx[l];
            const int st = stride[l];
            auto pair = [&](int b, double f[5]) {
                const int pn = tid + (b - il) * st;
                Node o;
                o.rho = s_buf[F_RHO * FS + pn];
                o.u1 = s_buf[F_U1 * FS + pn];
                o.u2 = s_buf[F_U2 * FS + pn];
                o.u3 = s_buf[F_U3 * FS + pn];
                o.beta = s_buf[F_B * FS + pn];
                o.lrho = s_buf[F_LR * FS + pn];
                o.lbeta = s_buf[F_LB * FS + pn];
                if constexpr (COMPACT) o.k = fma(o.u1, o.u1, fma(o.u2, o.u2, o.u3 * o.u3));
                else o.k = s_buf[F_K * FS + pn];
                const double n0 = A[l][0] + s_buf[(fa + 0) * FS + pn];
                const double n1 = A[l][1] + s_buf[(fa + 1) * FS + pn];
                const double n2 = A[l][2] + s_buf[(fa + 2) * FS + pn];
                if constexpr (HALF) flux_pair_half(me, o, n0, n1, n2, igm1, f);
                else flux_n<FLUX>(me, o, n0, n1, n2, gm1, f);
                return pn;
            };
    #pragma unroll
            for (int r = 1; 2 * r < N; ++r) {
                const int fm = (round & 1) ? F_MSG1 : F_MSG0;
                ++round;
                int b = il + r;
                if (b >= N) b -= N;
                if (tid < NODES) {
                    double f[5];
                    const int pn = pair(b, f);
                    const double dab = s_Dr[(r - 1) * N + il];  // D(i, i + r)
    #pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        acc[c] = fma(-dab, f[c], acc[c]);
                        s_buf[(fm + c) * FS + pn] = f[c];
                    }
                    if constexpr (EARLY) {
                        if (l < 2 && 2 * (r + 1) >= N) {  // last full round: stage the next row
                            const int fn = ((l + 1) & 1) ? F_A1 : F_A0;
                            s_buf[(fn + 0) * FS + tid] = A[l + 1][0];
                            s_buf[(fn + 1) * FS + tid] = A[l + 1][1];
                            s_buf[(fn + 2) * FS + tid] = A[l + 1][2];
                        }
                    }
                }
                __syncthreads();
                if (tid < NODES) {
                    // the pair flux posted by the node r places back: weight D(i, i - r)
                    const double dba = s_Dr[(N / 2 + r - 1) * N + il];
    #pragma unroll
                    for (int c = 0; c < 5; ++c) acc[c] = fma(-dba, s_buf[(fm + c) * FS + tid], acc[c]);
                }
            }
            if constexpr (N % 2 == 0) {
                if (tid < NODES) {
                    int b = il + N / 2;
                    if (b >= N) b -= N;
                    double f[5];
                    pair(b, f);
                    const double dab = s_Dr[(N / 2 - 1) * N + il];
    #pragma unroll
                    for (int c = 0; c < 5; ++c) acc[c] = fma(-dab, f[c], acc[c]);
                }
            }
        }
        __syncthreads();
        if constexpr (HALF) {
            me.rho *= 2.0;
            me.u1 *= 2.0;
            me.u2 *= 2.0;
            me.u3 *= 2.0;
            me.k *= 4.0;
        }
    }

    const double iJ = rcp(J);

    // ---- interface terms: EC interface flux, Lax-Friedrichs dissipation, SAT^theta, IP --------
    // The SAT^theta increments stay in LDS until the gradient phase (fields 8.. are free after the
    // pair loop): in the face slots for N >= 6, in per-node fields 8 + 4 l + c otherwise.
    // `faces` marks the node's interior faces (SAT^V), `sfaces` interior and boundary faces.
    int faces = 0, sfaces = 0, wfaces = 0;  // interior, all valid, no-slip wall faces
    if constexpr (N >= kFaceItemsFrom) {
        // (face, face node) work items spread over all lanes: only 6/N of the nodes lie on a face
        // of a given direction, so a per-node loop over directions would leave most lanes idle.
        // Each item leaves its terms in an LDS face slot (over the metric/mailbox areas); each
        // node then adds its (at most three) slots in direction order.  Node data staged for the
        // pair loop are still in LDS; own q, metrics and J are re-read (cache-resident).
        constexpr int NT = NT_OF(NODES);
        constexpr int FACE_ITEMS = EPW * 6 * N2;
        constexpr int NV = VISC ? 9 : 5;
        static_assert(NV * 6 <= (LDS_FIELDS - 8) * N, "face slots exceed the LDS tile");
        double *fsl = s_buf + 8 * FS;  // [NV][FACE_ITEMS]
        // at most two items per thread, as straight-line code (a loop here keeps both items' values
        // live and costs a third of the register file)
        static_assert(FACE_ITEMS <= 2 * NT, "at most two face items per thread");
        auto face_item = [&](const int it) {
            const int es = it / (6 * N2);
            const int rem = it - es * 6 * N2;
            const int f = rem / N2, t = rem - f * N2;
            const int l = f >> 1, side = f & 1;
            const long long ee = ebase + es;
            double v[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) v[c] = 0.0;
            const long long nb = s_face[2 * (es * 6 + f)];
            const int kind = s_face[2 * (es * 6 + f) + 1];
            if (kind != FACE_INVALID) {
                const int il = side ? N - 1 : 0;
                const int ta = t % N, tb = t / N;
                const int lno = l == 0 ? il + N * ta + N2 * tb
                                       : (l == 1 ? ta + N * il + N2 * tb : ta + N * tb + N2 * il);
                const int pl = es * N3 + lno;
                const long long go = ee * N3 + lno;
                long long pg = go;
                int lp = l;
                double sg = 1.0;
                if (kind == FACE_INTERIOR) {
                    const FaceLink k = face_link<N, OR>(a, ee, f, ta, tb,
                                                    lno + (N - 1 - 2 * il) * (l == 0 ? 1 : (l == 1 ? N : N2)));
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
                Node mi;  // the staged node data (halves of rho, U, |U|^2 for the ES-C pair loop)
                constexpr double H = HALF ? 2.0 : 1.0;
                mi.rho = H * s_buf[F_RHO * FS + pl];
                mi.u1 = H * s_buf[F_U1 * FS + pl];
                mi.u2 = H * s_buf[F_U2 * FS + pl];
                mi.u3 = H * s_buf[F_U3 * FS + pl];
                mi.beta = s_buf[F_B * FS + pl];
                mi.lrho = s_buf[F_LR * FS + pl];
                mi.lbeta = s_buf[F_LB * FS + pl];
                if constexpr (COMPACT) mi.k = fma(mi.u1, mi.u1, fma(mi.u2, mi.u2, mi.u3 * mi.u3));
                else mi.k = (H * H) * s_buf[F_K * FS + pl];
                const double Pi = gm1 * (qi[4] - 0.5 * qi[0] * mi.k);
                const double iJi = (VISC && a.eta != 0.0) ? rcp(a.jac[go]) : 1.0;
                face_terms<FLUX, VISC, MD>(a, face_own(a, mi, Pi, qi, iJi), Ai, pg, kind, lp, sg,
                                           side ? 1.0 : -1.0, v);
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) fsl[c * FACE_ITEMS + it] = v[c];
        };
        if (tid < FACE_ITEMS) face_item(tid);
        if constexpr (FACE_ITEMS > NT) {
            if (tid + NT < FACE_ITEMS) face_item(tid + NT);
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int il = idx[l];
                if (il != 0 && il != N - 1) continue;
                const int side = (il == N - 1) ? 1 : 0;
                const int kind = s_face[2 * (slot * 6 + 2 * l + side) + 1];
                if (kind == FACE_INVALID) continue;
                if (kind == FACE_INTERIOR) faces |= 1 << l;
                if (kind == FACE_WALL) wfaces |= 1 << l;
                sfaces |= 1 << l;
                const int it = (slot * 6 + 2 * l + side) * N2 + tangential_index<N>(l, i1, i2, i3);
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] += fsl[c * FACE_ITEMS + it];
            }
        }
    } else {
        // small elements: most nodes lie on faces, so each node walks its own faces
        const FaceOwn own = face_own(a, me, Pme, q, iJ);
        if (active) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int il = idx[l];
                if (il != 0 && il != N - 1) continue;
                const int side = (il == N - 1) ? 1 : 0;
                const long long nb = s_face[2 * (slot * 6 + 2 * l + side)];
                const int kind = s_face[2 * (slot * 6 + 2 * l + side) + 1];
                if (kind == FACE_INVALID) continue;
                if (kind == FACE_INTERIOR) faces |= 1 << l;
                if (kind == FACE_WALL) wfaces |= 1 << l;
                sfaces |= 1 << l;
                long long pg = g;
                int lp = l;
                double sg = 1.0;
                if (kind == FACE_INTERIOR) {
                    const int ta = l == 0 ? i2 : i1, tb = l == 2 ? i2 : i3;
                    const FaceLink k = face_link<N, OR>(a, e, 2 * l + side, ta, tb,
                                                    ln + (N - 1 - 2 * il) * stride[l]);
                    if (!k.ok) atomicOr(a.status, FLAG_MESH);
                    pg = nb * N3 + k.lno;
                    lp = k.fp >> 1;
                    sg = k.sg;
                }
                double v[9];
                face_terms<FLUX, VISC, MD>(a, own, A[l], pg, kind, lp, sg, side ? 1.0 : -1.0, v);
#pragma unroll
                for (int c = 0; c < 5; ++c) acc[c] += v[c];
                if constexpr (VISC) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) s_buf[(8 + 4 * l + c) * FS + tid] = v[5 + c];
                }
            }
        }
    }

    double T = 1.0, th[3][4];
    if constexpr (VISC) {
        // ---- BR1 gradient theta_a = D_a w from the lines (w = (U/T, -1/T); W_1 is not needed) --
        const double iT = 2.0 * a.R * me.beta;
        T = rcp(iT);
        const double w[4] = {me.u1 * iT, me.u2 * iT, me.u3 * iT, -iT};
        if (tid < NODES) {
#pragma unroll
            for (int c = 0; c < 4; ++c) s_buf[c * FS + tid] = w[c];
        }
        __syncthreads();
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int c = 0; c < 4; ++c) th[d][c] = 0.0;
            if (sfaces & (1 << d)) {
                if constexpr (N >= kFaceItemsFrom) {
                    constexpr int FACE_ITEMS = EPW * 6 * N2;
                    const int side = idx[d] == N - 1 ? 1 : 0;
                    const int it = (slot * 6 + 2 * d + side) * N2 + tangential_index<N>(d, i1, i2, i3);
#pragma unroll
                    for (int c = 0; c < 4; ++c) th[d][c] = s_buf[8 * FS + (5 + c) * FACE_ITEMS + it];
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) th[d][c] = s_buf[(8 + 4 * d + c) * FS + tid];
                }
            }
            if (tid < NODES) {
                const int il = idx[d];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const double dd = s_D[il * N + b];
                    const int pn = tid + (b - il) * stride[d];
#pragma unroll
                    for (int c = 0; c < 4; ++c) th[d][c] = fma(dd, s_buf[c * FS + pn], th[d][c]);
                }
            }
        }
    }

    if constexpr (VISC) {
        // ---- viscous flux, contravariant fluxes fhat_l, traces, divergence, own SAT^V ----------
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
        if (active) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int il = idx[l];
                if (il != 0 && il != N - 1) continue;
                const int side = (il == N - 1) ? 1 : 0;
                const int t = tangential_index<N>(l, i1, i2, i3);
                SBP_GLOBAL double *tr = a.trace + ((e * 6 + 2 * l + side) * 4) * N2 + t;
#pragma unroll
                for (int c = 0; c < 4; ++c) tr[c * N2] = fh[l][c];
                if (faces & (1 << l)) {
                    const double cs = -0.5 * (side ? 1.0 : -1.0) * isw;
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c + 1] = fma(cs, fh[l][c], acc[c + 1]);
                } else if (wfaces & (1 << l)) {
                    // adiabatic wall: the boundary viscous flux keeps the own momentum part and
                    // has no energy part
                    acc[4] = fma(-(side ? 1.0 : -1.0) * isw, fh[l][3], acc[4]);
                }
            }
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            __syncthreads();
            if (tid < NODES) {
#pragma unroll
                for (int c = 0; c < 4; ++c) s_buf[(4 + c) * FS + tid] = fh[l][c];
            }
            __syncthreads();
            if (tid < NODES) {
                const int il = idx[l];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const double dd = s_D[il * N + b];
                    const int pn = tid + (b - il) * stride[l];
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c + 1] = fma(dd, s_buf[(4 + c) * FS + pn], acc[c + 1]);
                }
            }
        }
    }

    if (active) {
        if (a.src) {
#pragma unroll
            for (int c = 0; c < 5; ++c) a.out[c * nodes + g] = fma(acc[c], iJ, a.src[c * nodes + g]);
        } else {
#pragma unroll
            for (int c = 0; c < 5; ++c) a.out[c * nodes + g] = acc[c] * iJ;
        }
    }
}

// Residual over a group of problems.  Non-persistent: one block per element tile.  Persistent:
// a grid sized to the resident capacity walks the tiles (the grid is a multiple of the XCD count,
// so the XCD-contiguous remap of tile indices still holds).
template <int N, int EPW, bool VISC, int FLUX, bool PERSIST, int WPE, bool MD, bool OR>
__global__ void __launch_bounds__(NT_OF(EPW * N * N * N))
__attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1, 8)))
k_residual(const GroupArgs g) {
    constexpr int N2 = N * N, NODES = EPW * N * N * N;
    __shared__ double s_buf[tile_fields(VISC) * field_stride(NODES)];
    __shared__ double s_D[N2];
    __shared__ double s_Dr[kRotRows<N> * N];
    __shared__ int s_face[2 * 6 * EPW];
    if (threadIdx.x < N2) s_D[threadIdx.x] = g.D[threadIdx.x];
    if (threadIdx.x < kRotRows<N> * N) s_Dr[threadIdx.x] = rotated_D<N>(g.D, threadIdx.x);
    if constexpr (!PERSIST) {
        const long long vb = xcd_block(blockIdx.x, gridDim.x);
        const int b = find_problem(g.block_start, g.n, vb);
        const ResArgs a = problem_view(g, g.probs[b], g.out);
        residual_tile<N, EPW, VISC, FLUX, MD, OR>(a, (vb - g.block_start[b]) * EPW, s_buf, s_D, s_Dr,
                                                  s_face);
    } else {
        for (long long it = blockIdx.x; it < g.total_blocks; it += gridDim.x) {
            const long long vb = xcd_block(it, g.total_blocks);
            const int b = find_problem(g.block_start, g.n, vb);
            const ResArgs a = problem_view(g, g.probs[b], g.out);
            residual_tile<N, EPW, VISC, FLUX, MD, OR>(a, (vb - g.block_start[b]) * EPW, s_buf, s_D, s_Dr,
                                                  s_face);
            __syncthreads();
        }
    }
}

// Neighbour half of SAT^V, (s/(2 w_end)) fhat_l,nu, for node gl of a problem.
template <int N>
__device__ __forceinline__ bool visc_fixup_add(const ResArgs &a, long long gl, double add[4]) {
    constexpr int N2 = N * N, N3 = N * N * N;
    const long long e = gl / N3;
    const int ln = (int)(gl - e * N3);
    const int i1 = ln % N, i2 = (ln / N) % N, i3 = ln / N2;
    const int idx[3] = {i1, i2, i3};
    bool any = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) add[c] = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int il = idx[l];
        if (il != 0 && il != N - 1) continue;
        const int side = (il == N - 1) ? 1 : 0;
        const double s = side ? 1.0 : -1.0;
        const long long nb = a.nbr[e * 6 + 2 * l + side];
        if (nb < 0 || nb >= a.K) continue;
        const int ta = l == 0 ? i2 : i1, tb = l == 2 ? i2 : i3;
        const int strd = l == 0 ? 1 : (l == 1 ? N : N2);
        const FaceLink k = face_link<N>(a, e, 2 * l + side, ta, tb, ln + (N - 1 - 2 * il) * strd);
        const SBP_GLOBAL double *tr = a.trace + ((nb * 6 + k.fp) * 4) * N2 + k.tp;
        const double cf = 0.5 * s * k.sg / a.w_end;
#pragma unroll
        for (int c = 0; c < 4; ++c) add[c] = fma(cf, tr[c * N2], add[c]);
        any = true;
    }
    return any;
}

template <int N>
__global__ void __launch_bounds__(256) k_group_fixup(const GroupArgs g) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.total_nodes) return;
    const int b = find_problem(g.node_start, g.n, v);
    const ResArgs a = problem_view(g, g.probs[b], g.out);
    const long long gl = v - g.node_start[b];
    double add[4];
    if (!visc_fixup_add<N>(a, gl, add)) return;
    const double iJ = 1.0 / a.jac[gl];
#pragma unroll
    for (int c = 0; c < 4; ++c) a.out[(c + 1) * a.nodes + gl] += add[c] * iJ;
}

// RK4 stage update (and, for viscous problems, the neighbour half of SAT^V) over a group.
template <int N, bool VISC>
__global__ void __launch_bounds__(256) k_group_rk_stage(const GroupArgs g, const RkGroupArgs r) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.total_nodes) return;
    const int b = find_problem(g.node_start, g.n, v);
    const ProbDev &P = g.probs[b];
    const ResArgs a = problem_view(g, P, const_cast<double *>(r.k));
    const long long gl = v - g.node_start[b];
    double kk[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) kk[c] = a.out[c * a.nodes + gl];
    if constexpr (VISC) {
        double add[4];
        if (visc_fixup_add<N>(a, gl, add)) {
            const double iJ = 1.0 / a.jac[gl];
#pragma unroll
            for (int c = 0; c < 4; ++c) kk[c + 1] = fma(add[c], iJ, kk[c + 1]);
        }
    }
    const double dt = r.dt[P.dt_index];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const long long i = P.off + c * a.nodes + gl;
        const double q = r.q[i];
        switch (r.stage) {
            case 0:
                r.acc[i] = fma(dt / 6.0, kk[c], q);
                r.qs[i] = fma(0.5 * dt, kk[c], q);
                break;
            case 1:
                r.acc[i] = fma(dt / 3.0, kk[c], r.acc[i]);
                r.qs[i] = fma(0.5 * dt, kk[c], q);
                break;
            case 2:
                r.acc[i] = fma(dt / 3.0, kk[c], r.acc[i]);
                r.qs[i] = fma(dt, kk[c], q);
                break;
            default:
                r.q[i] = fma(dt / 6.0, kk[c], r.acc[i]);
                break;
        }
    }
}


// Curl-form metrics J dxi_i/dx_n = -[curl_xi(X_l grad_xi X_m)]_i, (n, m, l) cyclic, and
// J = det(dx/dxi), with every derivative the collocation derivative D along a line of the element.
template <int N>
__global__ void __launch_bounds__(NT_OF(N * N * N))
k_metrics(const double *x, double *metric, double *jac, const double *D, long long K) {
    constexpr int N2 = N * N, N3 = N * N * N;
    __shared__ double s_x[3 * N3];
    __shared__ double s_V[3 * N3];
    __shared__ double s_D[N2];
    const int tid = threadIdx.x;
    const long long e = blockIdx.x;
    const long long nodes = K * N3;
    if (tid < N2) s_D[tid] = D[tid];
    const bool act = tid < N3;
    const int i1 = tid % N, i2 = (tid / N) % N, i3 = tid / N2;
    const int idx[3] = {i1, i2, i3};
    const int stride[3] = {1, N, N2};
    const long long g = e * N3 + tid;
    if (act) {
#pragma unroll
        for (int m = 0; m < 3; ++m) s_x[m * N3 + tid] = x[m * nodes + g];
    }
    __syncthreads();
    auto dline = [&](const double *arr, int dir) {
        double r = 0.0;
        const int il = idx[dir];
#pragma unroll
        for (int b = 0; b < N; ++b) r = fma(s_D[il * N + b], arr[tid + (b - il) * stride[dir]], r);
        return r;
    };
    double dx[3][3];  // dx[m][i] = dx_m/dxi_i
    if (act) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int i = 0; i < 3; ++i) dx[m][i] = dline(s_x + m * N3, i);
        const double Jv = dx[0][0] * (dx[1][1] * dx[2][2] - dx[1][2] * dx[2][1]) -
                          dx[0][1] * (dx[1][0] * dx[2][2] - dx[1][2] * dx[2][0]) +
                          dx[0][2] * (dx[1][0] * dx[2][1] - dx[1][1] * dx[2][0]);
        jac[g] = Jv;
    }
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int m = (n + 1) % 3, l = (n + 2) % 3;
        __syncthreads();
        if (act) {
            const double xl = s_x[l * N3 + tid];
#pragma unroll
            for (int i = 0; i < 3; ++i) s_V[i * N3 + tid] = xl * dx[m][i];
        }
        __syncthreads();
        if (act) {
            const double c0 = dline(s_V + 2 * N3, 1) - dline(s_V + 1 * N3, 2);
            const double c1 = dline(s_V + 0 * N3, 2) - dline(s_V + 2 * N3, 0);
            const double c2 = dline(s_V + 1 * N3, 0) - dline(s_V + 0 * N3, 1);
            metric[(3 * 0 + n) * nodes + g] = -c0;
            metric[(3 * 1 + n) * nodes + g] = -c1;
            metric[(3 * 2 + n) * nodes + g] = -c2;
        }
    }
}

// ---- launchers ---------------------------------------------------------------------------
// Schedules per degree: {elements per workgroup, persistent grid}.  Entry 0 is the default.
constexpr Schedule kSched2[] = {{8, 0, 0}, {16, 0, 0}, {8, 1, 0}, {16, 1, 0}, {8, 0, 4}};
constexpr Schedule kSched3[] = {{2, 0, 0}, {7, 0, 0}, {2, 1, 0}, {7, 1, 0}, {7, 0, 4}};
constexpr Schedule kSched4[] = {{1, 0, 0}, {2, 0, 0}, {4, 0, 0}, {1, 1, 0}, {2, 1, 0}, {1, 0, 4}, {2, 0, 4}};
constexpr Schedule kSched5[] = {{1, 0, 0}, {2, 0, 0}, {1, 1, 0}, {2, 1, 0}, {1, 0, 4}, {2, 0, 4}, {1, 0, 3}};
constexpr Schedule kSchedBig[] = {{1, 0, 0}, {1, 1, 0}, {1, 0, 4}, {1, 0, 3}};
constexpr Schedule kSchedPlanes[] = {{1, 0, 0}, {2, 0, 0}};  // planes per workgroup

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cus = n;
        else
            cus = 256;
    }
    return cus;
}

template <int N, int EPW, bool VISC, int FLUX, bool PERSIST, int WPE = 0, bool MD = false,
          bool OR = false>
int launch_res_k(const GroupArgs &g, hipStream_t s) {
    constexpr int NT = NT_OF(EPW * N * N * N);
    auto kern = k_residual<N, EPW, VISC, FLUX, PERSIST, WPE, MD, OR>;
    long long grid = g.total_blocks;
    if (PERSIST) {
        static int per_cu = 0;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0) != hipSuccess ||
                per_cu <= 0)
                per_cu = 1;
        }
        long long cap = (long long)per_cu * device_cus();
        cap = (cap / 8) * 8;
        if (cap < 8) cap = 8;
        if (grid > cap) grid = cap;
    }
    KernelTimer &tm = residual_timer();
    if (tm.enabled && hipEventRecord(tm.begin, s) != hipSuccess) return -1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), 0, s, g);
    if (hipGetLastError() != hipSuccess) return -1;
    if (tm.enabled && hipEventRecord(tm.end, s) != hipSuccess) return -1;
    return 0;
}

// Chandrashekar flux: every schedule; other fluxes: the default schedule only.
template <int N, int EPW, bool PERSIST>
int launch_res_e(bool visc, int flux, const GroupArgs &g, hipStream_t s) {
    if (flux == 0)
        return visc ? launch_res_k<N, EPW, true, 0, PERSIST>(g, s)
                    : launch_res_k<N, EPW, false, 0, PERSIST>(g, s);
    if (PERSIST) return -1;
    switch (flux) {
        case 1: return visc ? launch_res_k<N, EPW, true, 1, false>(g, s) : launch_res_k<N, EPW, false, 1, false>(g, s);
        case 2: return visc ? launch_res_k<N, EPW, true, 2, false>(g, s) : launch_res_k<N, EPW, false, 2, false>(g, s);
        case 3: return visc ? launch_res_k<N, EPW, true, 3, false>(g, s) : launch_res_k<N, EPW, false, 3, false>(g, s);
        default: return -1;
    }
}

// Matrix interface dissipation: default schedule, Chandrashekar and Kennedy-Gruber fluxes.
template <int N, int EPW>
int launch_res_md(bool visc, int flux, const GroupArgs &g, hipStream_t s) {
    switch (flux) {
        case 0: return visc ? launch_res_k<N, EPW, true, 0, false, 0, true>(g, s)
                            : launch_res_k<N, EPW, false, 0, false, 0, true>(g, s);
        case 2: return visc ? launch_res_k<N, EPW, true, 2, false, 0, true>(g, s)
                            : launch_res_k<N, EPW, false, 2, false, 0, true>(g, s);
        default: return -1;
    }
}

// Problems with a face-orientation table: default schedule, every flux and dissipation.
template <int N, int EPW>
int launch_res_or(bool visc, int flux, bool md, const GroupArgs &g, hipStream_t s) {
    if (md) {
        switch (flux) {
            case 0: return visc ? launch_res_k<N, EPW, true, 0, false, 0, true, true>(g, s)
                                : launch_res_k<N, EPW, false, 0, false, 0, true, true>(g, s);
            case 2: return visc ? launch_res_k<N, EPW, true, 2, false, 0, true, true>(g, s)
                                : launch_res_k<N, EPW, false, 2, false, 0, true, true>(g, s);
            default: return -1;
        }
    }
    switch (flux) {
        case 0: return visc ? launch_res_k<N, EPW, true, 0, false, 0, false, true>(g, s)
                            : launch_res_k<N, EPW, false, 0, false, 0, false, true>(g, s);
        case 1: return visc ? launch_res_k<N, EPW, true, 1, false, 0, false, true>(g, s)
                            : launch_res_k<N, EPW, false, 1, false, 0, false, true>(g, s);
        case 2: return visc ? launch_res_k<N, EPW, true, 2, false, 0, false, true>(g, s)
                            : launch_res_k<N, EPW, false, 2, false, 0, false, true>(g, s);
        case 3: return visc ? launch_res_k<N, EPW, true, 3, false, 0, false, true>(g, s)
                            : launch_res_k<N, EPW, false, 3, false, 0, false, true>(g, s);
        default: return -1;
    }
}

template <int N, int EPW, bool PERSIST, int WPE = 0>
int launch_res_e0(bool visc, const GroupArgs &g, hipStream_t s) {
    return visc ? launch_res_k<N, EPW, true, 0, PERSIST, WPE>(g, s)
                : launch_res_k<N, EPW, false, 0, PERSIST, WPE>(g, s);
}

template <int N>
int launch_fixup(const GroupArgs &g, hipStream_t s) {
    const long long nb = (g.total_nodes + 255) / 256;
    hipLaunchKernelGGL((k_group_fixup<N>), dim3((unsigned)nb), dim3(256), 0, s, g);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int launch_rkg(bool visc, const GroupArgs &g, const RkGroupArgs &r, hipStream_t s) {
    const long long nb = (g.total_nodes + 255) / 256;
    if (visc) hipLaunchKernelGGL((k_group_rk_stage<N, true>), dim3((unsigned)nb), dim3(256), 0, s, g, r);
    else hipLaunchKernelGGL((k_group_rk_stage<N, false>), dim3((unsigned)nb), dim3(256), 0, s, g, r);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int schedule_count(int p) {
    switch (p) {
        case 1: return (int)(sizeof(kSched2) / sizeof(Schedule));
        case 2: return (int)(sizeof(kSched3) / sizeof(Schedule));
        case 3: return (int)(sizeof(kSched4) / sizeof(Schedule));
        case 4: return (int)(sizeof(kSched5) / sizeof(Schedule));
        case 5: case 6: case 7: case 8: return (int)(sizeof(kSchedBig) / sizeof(Schedule));
        case 9: case 10: case 11: case 12: case 13: case 14: case 15:
            return (int)(sizeof(kSchedPlanes) / sizeof(Schedule));
        default: return 0;
    }
}

Schedule schedule_of(int p, int v) {
    switch (p) {
        case 1: return kSched2[v];
        case 2: return kSched3[v];
        case 3: return kSched4[v];
        case 4: return kSched5[v];
        default: return p >= kFirstPlaneP ? kSchedPlanes[v] : kSchedBig[v];
    }
}

int launch_group_residual(int p, bool visc, int flux, bool md, bool orient, int variant,
                          const GroupArgs &g, hipStream_t s, bool fixup) {
    if (variant < 0 || variant >= schedule_count(p)) return -1;
    if ((flux != 0 || md || orient) && variant != 0) return -1;
    const Schedule sc = schedule_of(p, variant);
    // high degrees: plane passes, which finish SAT^V themselves (no fixup)
    if (p >= kFirstPlaneP) return launch_group_residual_planes(p, sc.epw, visc, flux, md, orient, g, s);
    int rc = -1;
    const bool P1 = sc.persistent != 0;
    if (orient) {
        switch (p) {
            case 1: rc = launch_res_or<2, 8>(visc, flux, md, g, s); break;
            case 2: rc = launch_res_or<3, 2>(visc, flux, md, g, s); break;
            case 3: rc = launch_res_or<4, 1>(visc, flux, md, g, s); break;
            case 4: rc = launch_res_or<5, 1>(visc, flux, md, g, s); break;
            case 5: rc = launch_res_or<6, 1>(visc, flux, md, g, s); break;
            case 6: rc = launch_res_or<7, 1>(visc, flux, md, g, s); break;
            case 7: rc = launch_res_or<8, 1>(visc, flux, md, g, s); break;
            case 8: rc = launch_res_or<9, 1>(visc, flux, md, g, s); break;
            default: return -1;
        }
    } else if (md) {
        switch (p) {
            case 1: rc = launch_res_md<2, 8>(visc, flux, g, s); break;
            case 2: rc = launch_res_md<3, 2>(visc, flux, g, s); break;
            case 3: rc = launch_res_md<4, 1>(visc, flux, g, s); break;
            case 4: rc = launch_res_md<5, 1>(visc, flux, g, s); break;
            case 5: rc = launch_res_md<6, 1>(visc, flux, g, s); break;
            case 6: rc = launch_res_md<7, 1>(visc, flux, g, s); break;
            case 7: rc = launch_res_md<8, 1>(visc, flux, g, s); break;
            case 8: rc = launch_res_md<9, 1>(visc, flux, g, s); break;
            default: return -1;
        }
    } else if (flux == 0) {
#define SBP_CASE(NN, EE)                                                                \
    if (sc.epw == EE && sc.wpe == 0) rc = P1 ? launch_res_e0<NN, EE, true>(visc, g, s)  \
                                             : launch_res_e0<NN, EE, false>(visc, g, s);
#define SBP_CASEW(NN, EE, WW)                                                           \
    if (sc.epw == EE && sc.wpe == WW && !P1) rc = launch_res_e0<NN, EE, false, WW>(visc, g, s);
        switch (p) {
            case 1: SBP_CASE(2, 8) SBP_CASE(2, 16) SBP_CASEW(2, 8, 4) break;
            case 2: SBP_CASE(3, 2) SBP_CASE(3, 7) SBP_CASEW(3, 7, 4) break;
            case 3: SBP_CASE(4, 1) SBP_CASE(4, 2) SBP_CASE(4, 4) SBP_CASEW(4, 1, 4) SBP_CASEW(4, 2, 4) break;
            case 4: SBP_CASE(5, 1) SBP_CASE(5, 2) SBP_CASEW(5, 1, 4) SBP_CASEW(5, 2, 4) SBP_CASEW(5, 1, 3) break;
            case 5: SBP_CASE(6, 1) SBP_CASEW(6, 1, 4) SBP_CASEW(6, 1, 3) break;
            case 6: SBP_CASE(7, 1) SBP_CASEW(7, 1, 4) SBP_CASEW(7, 1, 3) break;
            case 7: SBP_CASE(8, 1) SBP_CASEW(8, 1, 4) SBP_CASEW(8, 1, 3) break;
            case 8: SBP_CASE(9, 1) SBP_CASEW(9, 1, 4) SBP_CASEW(9, 1, 3) break;
            default: return -1;
        }
#undef SBP_CASE
#undef SBP_CASEW
    } else {
        switch (p) {
            case 1: rc = launch_res_e<2, 8, false>(visc, flux, g, s); break;
            case 2: rc = launch_res_e<3, 2, false>(visc, flux, g, s); break;
            case 3: rc = launch_res_e<4, 1, false>(visc, flux, g, s); break;
            case 4: rc = launch_res_e<5, 1, false>(visc, flux, g, s); break;
            case 5: rc = launch_res_e<6, 1, false>(visc, flux, g, s); break;
            case 6: rc = launch_res_e<7, 1, false>(visc, flux, g, s); break;
            case 7: rc = launch_res_e<8, 1, false>(visc, flux, g, s); break;
            case 8: rc = launch_res_e<9, 1, false>(visc, flux, g, s); break;
            default: return -1;
        }
    }
    if (rc != 0) return rc;
    if (visc && fixup) {
        switch (p) {
            case 1: return launch_fixup<2>(g, s);
            case 2: return launch_fixup<3>(g, s);
            case 3: return launch_fixup<4>(g, s);
            case 4: return launch_fixup<5>(g, s);
            case 5: return launch_fixup<6>(g, s);
            case 6: return launch_fixup<7>(g, s);
            case 7: return launch_fixup<8>(g, s);
            case 8: return launch_fixup<9>(g, s);
            default: return -1;
        }
    }
    return 0;
}

int launch_group_rk_stage(int p, bool visc, const GroupArgs &g, const RkGroupArgs &r, hipStream_t s) {
    switch (p) {
        case 1: return launch_rkg<2>(visc, g, r, s);
        case 2: return launch_rkg<3>(visc, g, r, s);
        case 3: return launch_rkg<4>(visc, g, r, s);
        case 4: return launch_rkg<5>(visc, g, r, s);
        case 5: return launch_rkg<6>(visc, g, r, s);
        case 6: return launch_rkg<7>(visc, g, r, s);
        case 7: return launch_rkg<8>(visc, g, r, s);
        case 8: return launch_rkg<9>(visc, g, r, s);
        // plane passes leave a finished dq/dt: the stage kernel adds no SAT^V half
        case 9: case 10: case 11: case 12: case 13: case 14: case 15:
            return launch_rkg<2>(false, g, r, s);
        default: return -1;
    }
}

KernelTimer &residual_timer() {
    static KernelTimer t;
    return t;
}


int launch_metrics(int p, long long K, const double *x, double *metric, double *jac,
                   const double *D, hipStream_t s) {
#define SBP_MET(NN)                                                                              \
    hipLaunchKernelGGL((k_metrics<NN>), dim3((unsigned)K), dim3(NT_OF(NN * NN * NN)), 0, s, x,   \
                       metric, jac, D, K);                                                        \
    break;
    switch (p) {
        case 1: SBP_MET(2)
        case 2: SBP_MET(3)
        case 3: SBP_MET(4)
        case 4: SBP_MET(5)
        case 5: SBP_MET(6)
        case 6: SBP_MET(7)
        case 7: SBP_MET(8)
        case 8: SBP_MET(9)
        case 9: SBP_MET(10)
        case 10: case 11: case 12: case 13: case 14: case 15:
            return launch_metrics_big(p, K, x, metric, jac, D, s);
        default: return -1;
    }
#undef SBP_MET
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sbp
