// C ABI of the ES-C SBP-SAT residual library (declared in include/sbp.h): argument checking,
// the 1-D LGL operator, workspace layout, launch sequencing and the RK4 graph cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbp.h"
#include "sbp_internal.h"

namespace {

constexpr int kMaxOpP = 15;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------------------------------
// 1-D LGL operator.  Interior nodes are the roots of P_p' found by Newton's method in long
// double; the derivative matrix is built from barycentric weights (D_ij = (l_j/l_i)/(x_i-x_j),
// D_ii = -sum_{j != i} D_ij) and the weights from w_i = 2 / (p (p+1) P_p(x_i)^2).
// ------------------------------------------------------------------------------------------
void legendre_ld(int p, long double x, long double &P, long double &dP) {
    long double p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
    if (p == 0) { P = 1.0L; dP = 0.0L; return; }
    for (int n = 1; n < p; ++n) {
        const long double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
        const long double d2 = d0 + (2 * n + 1) * p1;  // P'_{n+1} = P'_{n-1} + (2n+1) P_n
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    P = p1;
    dP = d1;
}

void lgl_ld(int p, std::vector<long double> &x, std::vector<long double> &w,
            std::vector<long double> &D) {
    const int N = p + 1;
    x.assign(N, 0.0L);
    w.assign(N, 0.0L);
    D.assign(N * N, 0.0L);
    const long double pi = 3.14159265358979323846264338327950288L;
    x[0] = -1.0L;
    x[p] = 1.0L;
    for (int i = 1; i < p; ++i) {
        long double xi = -std::cos(pi * i / p);
        for (int it = 0; it < 100; ++it) {
            long double P, dP;
            legendre_ld(p, xi, P, dP);
            const long double d2P = (2.0L * xi * dP - p * (p + 1.0L) * P) / (1.0L - xi * xi);
            const long double step = dP / d2P;
            xi -= step;
            if (std::fabs(step) < 1e-30L) break;
        }
        x[i] = xi;
    }
    for (int i = 0; i < N; ++i) {
        long double P, dP;
        legendre_ld(p, x[i], P, dP);
        w[i] = 2.0L / (p * (p + 1.0L) * P * P);
    }
    std::vector<long double> lam(N, 1.0L);
    for (int j = 0; j < N; ++j) {
        long double prod = 1.0L;
        for (int k = 0; k < N; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        lam[j] = 1.0L / prod;
    }
    for (int i = 0; i < N; ++i) {
        long double diag = 0.0L;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            const long double v = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * N + j] = v;
            diag -= v;
        }
        D[i * N + i] = diag;
    }
}

struct Op {
    double x[16], w[16], D[256];
};

const Op &host_op(int p) {
    static Op ops[kMaxOpP + 1];
    static bool done[kMaxOpP + 1] = {};
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (!done[p]) {
        std::vector<long double> x, w, D;
        lgl_ld(p, x, w, D);
        const int N = p + 1;
        for (int i = 0; i < N; ++i) { ops[p].x[i] = (double)x[i]; ops[p].w[i] = (double)w[i]; }
        for (int i = 0; i < N * N; ++i) ops[p].D[i] = (double)D[i];
        done[p] = true;
    }
    return ops[p];
}

// Device copies of D for p = 1..kMaxOpP, one table per device.
const double *device_D(int p) {
    static std::mutex mu;
    static std::map<int, double *> tables;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = tables.find(dev);
    if (it == tables.end()) {
        double *buf = nullptr;
        if (hipMalloc(&buf, sizeof(double) * 256 * (kMaxOpP + 1)) != hipSuccess) return nullptr;
        std::vector<double> host(256 * (kMaxOpP + 1), 0.0);
        for (int pp = 1; pp <= kMaxOpP; ++pp) {
            const Op &o = host_op(pp);
            std::memcpy(host.data() + 256 * pp, o.D, sizeof(double) * (pp + 1) * (pp + 1));
        }
        if (hipMemcpy(buf, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
            return nullptr;
        it = tables.emplace(dev, buf).first;
    }
    return it->second + 256 * p;
}

// Eigen-decomposition of a symmetric n x n matrix (row-major) by cyclic Jacobi rotations:
// A = V diag(lam) V^T with V[i * n + k] the i-th component of eigenvector k.
void sym_eigen(int n, std::vector<long double> A, std::vector<long double> &V,
               std::vector<long double> &lam) {
    V.assign(n * n, 0.0L);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0L;
    for (int sweep = 0; sweep < 64; ++sweep) {
        long double off = 0.0L, diag = 0.0L;
        for (int i = 0; i < n; ++i) {
            diag += A[i * n + i] * A[i * n + i];
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        }
        if (off <= 1e-40L * diag) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const long double apq = A[p * n + q];
                if (apq == 0.0L) continue;
                // rotation in the (p, q) plane that zeroes A[p][q]: t = tan(phi) is the smaller
                // root of t^2 + 2 theta t - 1 = 0
                const long double theta = (A[q * n + q] - A[p * n + p]) / (2.0L * apq);
                const long double t = (theta >= 0.0L ? 1.0L : -1.0L) /
                                      (std::fabs(theta) + std::sqrt(theta * theta + 1.0L));
                const long double c = 1.0L / std::sqrt(t * t + 1.0L), sn = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A R
                    const long double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - sn * akq;
                    A[k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- R^T A
                    const long double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - sn * aqk;
                    A[q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V R
                    const long double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - sn * vkq;
                    V[k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    lam.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

// Tables of the optimised metric terms for degree p (declared in sbp_internal.h).  B has rank
// N - 2 (D restricted to the interior nodes is injective), so its two smallest eigenvalues are the
// null pair; the eigen-decomposition is checked against B before use.  The left null vector of D
// is z_i = w_i P_p(x_i): sum_i w_i P_p(x_i) l_j'(x_i) is the exact quadrature of P_p l_j', a
// polynomial of degree 2p - 1, and P_p is orthogonal to every polynomial of degree p - 1.
bool opt_metric_tables(int p, sbp::OptMetricTables &t) {
    std::vector<long double> x, w, D;
    lgl_ld(p, x, w, D);
    const int N = p + 1;
    std::vector<long double> B(N * N, 0.0L), V, lam;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            long double acc = 0.0L;
            for (int k = 1; k < N - 1; ++k) acc += D[i * N + k] * D[j * N + k];
            B[i * N + j] = acc;
        }
    sym_eigen(N, B, V, lam);
    long double bmax = 0.0L, resid = 0.0L;
    for (int i = 0; i < N * N; ++i) bmax = std::max(bmax, std::fabs(B[i]));
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < N; ++k) {
            long double acc = 0.0L;
            for (int j = 0; j < N; ++j) acc += B[i * N + j] * V[j * N + k];
            resid = std::max(resid, std::fabs(acc - lam[k] * V[i * N + k]));
        }
    if (!(resid <= 1e-14L * bmax)) return false;
    int lo0 = 0;
    for (int k = 1; k < N; ++k)
        if (lam[k] < lam[lo0]) lo0 = k;
    int lo1 = lo0 == 0 ? 1 : 0;
    for (int k = 0; k < N; ++k)
        if (k != lo0 && lam[k] < lam[lo1]) lo1 = k;
    t = sbp::OptMetricTables{};
    t.p = p;
    t.null_mask = (1 << lo0) | (1 << lo1);
    for (int i = 0; i < N * N; ++i) { t.D[i] = (double)D[i]; t.V[i] = (double)V[i]; }
    for (int k = 0; k < N; ++k) t.lam[k] = ((t.null_mask >> k) & 1) ? 0.0 : (double)lam[k];
    for (int i = 0; i < N; ++i) {
        long double P, dP;
        legendre_ld(p, x[i], P, dP);
        t.pat[0][i] = (double)(w[i] * P);
        t.pat[1][i] = (double)w[i];
    }
    return true;
}

bool aligned8(const void *p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) % 8) == 0; }

int check_problem(const sbp_problem &pr) {
    if (pr.p < 1 || pr.p > SBP_MAX_P) return SBP_ERR_DEGREE;
    if (pr.n_elem <= 0) return SBP_ERR_ARG;
    if (!aligned8(pr.metric) || !aligned8(pr.jac) || pr.nbr == nullptr ||
        (reinterpret_cast<uintptr_t>(pr.nbr) % 4) != 0)
        return SBP_ERR_ARG;
    if (!(pr.gamma > 1.0) || !(pr.R > 0.0) || !(pr.mu >= 0.0) || !(pr.eta >= 0.0)) return SBP_ERR_ARG;
    if (pr.mu > 0.0 && !(pr.Pr > 0.0)) return SBP_ERR_ARG;
    if (pr.two_point < 0 || pr.two_point > 3 || pr.reserved != 0) return SBP_ERR_ARG;
    if ((pr.bc_state && !aligned8(pr.bc_state)) || (pr.source && !aligned8(pr.source))) return SBP_ERR_ARG;
    if (pr.face_orient && (reinterpret_cast<uintptr_t>(pr.face_orient) & 3u) != 0) return SBP_ERR_ARG;
    if (pr.iface_diss < 0 || pr.iface_diss > 2) return SBP_ERR_ARG;
    if (pr.iface_diss == 2 && pr.two_point != SBP_FLUX_CHANDRASHEKAR &&
        pr.two_point != SBP_FLUX_KENNEDY_GRUBER)
        return SBP_ERR_ARG;
    return SBP_OK;
}

long long nodes_of(const sbp_problem &pr) {
    const long long N = pr.p + 1;
    return pr.n_elem * N * N * N;
}

// Workspace layout: [flags | per-problem viscous traces | per-problem VJP gradient cotangents |
// RK buffers acc, qs, k].
struct Layout {
    size_t flags = 0;
    std::vector<size_t> trace;  // offset per problem (0 if inviscid)
    std::vector<size_t> thb;    // offset per problem (0 if inviscid)
    size_t rk = 0;              // offset of the RK block
    size_t total_state = 0;     // doubles in one state-sized buffer
    size_t bytes = 0;
};

Layout layout_of(const sbp_problem *probs, int n) {
    Layout L;
    size_t off = align_up(sizeof(int) * 16);
    L.trace.resize(n, 0);
    L.thb.resize(n, 0);
    size_t states = 0;
    for (int b = 0; b < n; ++b) {
        const long long N = probs[b].p + 1;
        if (probs[b].mu > 0.0) {
            L.trace[b] = off;
            off += align_up(sizeof(double) * (size_t)probs[b].n_elem * 6 * 4 * N * N);
            // VJP gradient cotangents (12 per node) or the plane passes' scratch (16 per node)
            L.thb[b] = off;
            const size_t per = probs[b].p >= sbp::kFirstPlaneP ? 16 : 12;
            off += align_up(sizeof(double) * per * (size_t)nodes_of(probs[b]));
        }
        states += 5 * (size_t)nodes_of(probs[b]);
    }
    L.rk = off;
    L.total_state = states;
    off += 3 * align_up(sizeof(double) * states);
    L.bytes = off;
    return L;
}

int validate(const sbp_problem *probs, int32_t n_prob, void *ws, size_t ws_bytes, Layout &L) {
    if (probs == nullptr || n_prob < 1) return SBP_ERR_ARG;
    for (int b = 0; b < n_prob; ++b) {
        const int rc = check_problem(probs[b]);
        if (rc != SBP_OK) return rc;
    }
    L = layout_of(probs, n_prob);
    if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < L.bytes)
        return SBP_ERR_WORKSPACE;
    return SBP_OK;
}

// ------------------------------------------------------------------------------------------
// Plans: problems grouped by (degree, viscous, flux), each group with a device table of its
// problems, prefix sums of element tiles (per elements-per-workgroup option) and of nodes, and
// the schedule variant chosen for it.  Cached per (problem array contents, workspace, device).
// ------------------------------------------------------------------------------------------
struct GroupPlan {
    int p = 0;
    bool visc = false;
    int flux = 0;
    bool md = false;      // matrix interface dissipation
    bool orient = false;  // face-orientation tables
    std::vector<int> members;
    sbp::ProbDev *d_probs = nullptr;
    long long *d_node_start = nullptr;
    long long total_nodes = 0;
    std::map<int, long long *> d_block_start;  // by elements per workgroup
    std::map<int, long long> total_blocks;
    int variant = 0;
};

struct Plan {
    std::vector<GroupPlan> groups;
    int generation = 0;
    const void *ws = nullptr;  // the workspace the plan was made for (sbp_release)
};

std::mutex g_plan_mu;
std::map<std::string, Plan *> g_plans;
int g_generation = 0;

std::string plan_key(const sbp_problem *probs, int n, const void *ws, int dev) {
    std::string k(reinterpret_cast<const char *>(probs), sizeof(sbp_problem) * n);
    k.append(reinterpret_cast<const char *>(&ws), sizeof(ws));
    k.append(reinterpret_cast<const char *>(&dev), sizeof(dev));
    return k;
}

template <typename T>
T *to_device(const std::vector<T> &v) {
    T *d = nullptr;
    if (hipMalloc(&d, sizeof(T) * v.size()) != hipSuccess) return nullptr;
    if (hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    return d;
}

void free_plan(Plan *plan) {
    for (auto &g : plan->groups) {
        if (g.d_probs) (void)hipFree(g.d_probs);
        if (g.d_node_start) (void)hipFree(g.d_node_start);
        for (auto &kv : g.d_block_start)
            if (kv.second) (void)hipFree(kv.second);
    }
    delete plan;
}

// Problems grouped by launch kind (degree, viscous, flux, matrix dissipation, orientation table),
// in order of first appearance; members in problem order.
void group_problems(const sbp_problem *probs, int n, std::vector<GroupPlan> &groups) {
    for (int b = 0; b < n; ++b) {
        const bool visc = probs[b].mu > 0.0;
        const bool md = probs[b].iface_diss == 2;
        const bool orient = probs[b].face_orient != nullptr;
        GroupPlan *gp = nullptr;
        for (auto &g : groups)
            if (g.p == probs[b].p && g.visc == visc && g.flux == probs[b].two_point && g.md == md &&
                g.orient == orient)
                gp = &g;
        if (!gp) {
            groups.emplace_back();
            gp = &groups.back();
            gp->p = probs[b].p;
            gp->visc = visc;
            gp->flux = probs[b].two_point;
            gp->md = md;
            gp->orient = orient;
        }
        gp->members.push_back(b);
    }
}

// Device-table entry of problem b (state offset `off` doubles; viscous scratch at trace/thb).
sbp::ProbDev prob_dev(const sbp_problem &pr, int b, long long off, double *trace, double *thb) {
    sbp::ProbDev d{};
    d.metric = pr.metric;
    d.jac = pr.jac;
    d.nbr = pr.nbr;
    d.trace = pr.mu > 0.0 ? trace : nullptr;
    d.thb = pr.mu > 0.0 ? thb : nullptr;
    d.bc = pr.bc_state;
    d.src = pr.source;
    d.orient = pr.face_orient;
    d.K = pr.n_elem;
    d.nodes = nodes_of(pr);
    d.off = off;
    d.gamma = pr.gamma;
    d.R = pr.R;
    d.mu = pr.mu;
    d.Pr = pr.Pr;
    d.eta = pr.eta;
    d.w_end = host_op(pr.p).w[0];
    d.isw = 1.0 / d.w_end;
    d.kap = pr.mu > 0.0 ? pr.mu * pr.gamma * pr.R / ((pr.gamma - 1.0) * pr.Pr) : 0.0;
    d.iface_diss = pr.iface_diss;
    d.two_point = pr.two_point;
    d.dt_index = b;
    return d;
}

// Prefix sums of the work units (elements, or node planes for the plane passes) per workgroup
// tile of `epw` units over the members of a group.
std::vector<long long> block_starts(const sbp_problem *probs, const GroupPlan &g, int epw) {
    const long long per_elem = g.p >= sbp::kFirstPlaneP ? g.p + 1 : 1;
    std::vector<long long> bs(1, 0);
    for (int b : g.members) bs.push_back(bs.back() + (probs[b].n_elem * per_elem + epw - 1) / epw);
    return bs;
}

std::vector<long long> state_offsets(const sbp_problem *probs, int n) {
    std::vector<long long> off(n, 0);
    long long acc = 0;
    for (int b = 0; b < n; ++b) {
        off[b] = acc;
        acc += 5 * nodes_of(probs[b]);
    }
    return off;
}

Plan *get_plan(const sbp_problem *probs, int n, char *ws, const Layout &L) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    const std::string key = plan_key(probs, n, ws, dev);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
    Plan *plan = new Plan();
    plan->ws = ws;
    const std::vector<long long> off = state_offsets(probs, n);
    group_problems(probs, n, plan->groups);
    for (auto &g : plan->groups) {
        std::vector<sbp::ProbDev> host;
        std::vector<long long> ns(1, 0);
        for (int b : g.members) {
            host.push_back(prob_dev(probs[b], b, off[b], reinterpret_cast<double *>(ws + L.trace[b]),
                                    reinterpret_cast<double *>(ws + L.thb[b])));
            ns.push_back(ns.back() + host.back().nodes);
        }
        g.d_probs = to_device(host);
        g.d_node_start = to_device(ns);
        g.total_nodes = ns.back();
        if (!g.d_probs || !g.d_node_start) {
            free_plan(plan);
            return nullptr;
        }
        for (int v = 0; v < sbp::schedule_count(g.p); ++v) {
            const int epw = sbp::schedule_of(g.p, v).epw;
            if (g.d_block_start.count(epw)) continue;
            const std::vector<long long> bs = block_starts(probs, g, epw);
            g.d_block_start[epw] = to_device(bs);
            g.total_blocks[epw] = bs.back();
            if (!g.d_block_start[epw]) {
                free_plan(plan);
                return nullptr;
            }
        }
    }
    plan->generation = ++g_generation;
    g_plans[key] = plan;
    return plan;
}

sbp::GroupArgs group_args(const GroupPlan &g, int variant, const double *q, double *out, char *ws) {
    sbp::GroupArgs a{};
    const int epw = sbp::schedule_of(g.p, variant).epw;
    a.probs = g.d_probs;
    a.block_start = g.d_block_start.at(epw);
    a.node_start = g.d_node_start;
    a.n = (int)g.members.size();
    a.total_blocks = g.total_blocks.at(epw);
    a.total_nodes = g.total_nodes;
    a.q = q;
    a.out = out;
    a.status = reinterpret_cast<int *>(ws);
    a.D = device_D(g.p);
    return a;
}

int residual_group(const GroupPlan &g, const double *q, double *out, char *ws, hipStream_t s,
                   bool fixup, int variant) {
    sbp::GroupArgs a = group_args(g, variant, q, out, ws);
    if (a.D == nullptr) return SBP_ERR_HIP;
    return sbp::launch_group_residual(g.p, g.visc, g.flux, g.md, g.orient, variant, a, s, fixup) == 0 ? SBP_OK
                                                                                           : SBP_ERR_HIP;
}

int residual_all(Plan *plan, const double *q, double *out, char *ws, hipStream_t s) {
    for (const auto &g : plan->groups) {
        const int rc = residual_group(g, q, out, ws, s, true, g.variant);
        if (rc != SBP_OK) return rc;
    }
    return SBP_OK;
}

// One RK4 step of one group = four (residual, stage update) pairs.
int rk_step_group(const GroupPlan &g, double *q, const double *dt, char *ws, const Layout &L,
                  hipStream_t s) {
    const size_t sb = align_up(sizeof(double) * L.total_state);
    double *acc = reinterpret_cast<double *>(ws + L.rk);
    double *qs = reinterpret_cast<double *>(ws + L.rk + sb);
    double *k = reinterpret_cast<double *>(ws + L.rk + 2 * sb);
    for (int stage = 0; stage < 4; ++stage) {
        const double *src = stage == 0 ? q : qs;
        int rc = residual_group(g, src, k, ws, s, false, g.variant);
        if (rc != SBP_OK) return rc;
        sbp::GroupArgs a = group_args(g, g.variant, src, k, ws);
        sbp::RkGroupArgs r{q, acc, qs, k, dt, stage};
        if (sbp::launch_group_rk_stage(g.p, g.visc, a, r, s) != 0) return SBP_ERR_HIP;
    }
    return SBP_OK;
}

struct GraphKey {
    std::string probs;
    const void *q, *dt, *ws;
    int dev, generation;
    bool operator<(const GraphKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (generation != o.generation) return generation < o.generation;
        if (q != o.q) return q < o.q;
        if (dt != o.dt) return dt < o.dt;
        if (ws != o.ws) return ws < o.ws;
        return probs < o.probs;
    }
};

std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;

// Records one RK4 step of every group into a graph; groups are independent branches.
int record_rk_graph(Plan *plan, double *q, const double *dt, char *ws, const Layout &L,
                    hipGraphExec_t *exec) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SBP_ERR_HIP;
    std::vector<hipStream_t> br(plan->groups.size(), nullptr);
    std::vector<hipEvent_t> ev(plan->groups.size() + 1, nullptr);
    int rc = SBP_OK;
    for (size_t i = 0; i < br.size() && rc == SBP_OK; ++i)
        if (hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) rc = SBP_ERR_HIP;
    for (size_t i = 0; i < ev.size() && rc == SBP_OK; ++i)
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) rc = SBP_ERR_HIP;
    hipGraph_t graph = nullptr;
    if (rc == SBP_OK && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        if (hipEventRecord(ev.back(), cap) != hipSuccess) rc = SBP_ERR_HIP;
        for (size_t i = 0; i < br.size() && rc == SBP_OK; ++i) {
            if (hipStreamWaitEvent(br[i], ev.back(), 0) != hipSuccess) { rc = SBP_ERR_HIP; break; }
            rc = rk_step_group(plan->groups[i], q, dt, ws, L, br[i]);
            if (rc == SBP_OK && (hipEventRecord(ev[i], br[i]) != hipSuccess ||
                                 hipStreamWaitEvent(cap, ev[i], 0) != hipSuccess))
                rc = SBP_ERR_HIP;
        }
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (rc == SBP_OK && (ec != hipSuccess || graph == nullptr)) rc = SBP_ERR_HIP;
    } else if (rc == SBP_OK) {
        rc = SBP_ERR_HIP;
    }
    if (rc == SBP_OK && hipGraphInstantiate(exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = SBP_ERR_HIP;
    // teardown: failures here leave nothing to undo
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    for (auto b : br)
        if (b) (void)hipStreamDestroy(b);
    (void)hipStreamDestroy(cap);
    return rc;
}

// Marks that tell the VJP's boundary pass whether its launch met a boundary face (the workspace's
// second flag word holds the last mark written; never 0).
int next_vjp_mark() {
    static std::atomic<int> mark{0};
    int m = mark.fetch_add(1) + 1;
    if (m <= 0) {
        mark.store(1);
        m = 1;
    }
    return m;
}

}  // namespace

extern "C" {

int sbp_version(void) { return 113; }

const char *sbp_error_string(int code) {
    switch (code) {
        case SBP_OK: return "ok";
        case SBP_ERR_ARG: return "invalid argument (null/misaligned pointer, size or option)";
        case SBP_ERR_DEGREE: return "polynomial degree out of range";
        case SBP_ERR_MESH: return "neighbour index out of range";
        case SBP_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, P <= 0 or non-finite)";
        case SBP_ERR_HIP: return "HIP runtime error";
        case SBP_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case SBP_ERR_SCRATCH:
            return "problem set too large for the library-owned scratch of sbp_residual_noalloc";
        default: return "unknown error";
    }
}

int sbp_lgl_operator(int32_t p, double *x, double *w, double *D) {
    if (p < 1 || p > kMaxOpP) return SBP_ERR_DEGREE;
    const Op &o = host_op(p);
    const int N = p + 1;
    if (x) std::memcpy(x, o.x, sizeof(double) * N);
    if (w) std::memcpy(w, o.w, sizeof(double) * N);
    if (D) std::memcpy(D, o.D, sizeof(double) * N * N);
    return SBP_OK;
}

int sbp_metrics(int32_t p, int64_t n_elem, const double *coords, double *metric, double *jac,
                void *stream) {
    if (p < 1 || p > SBP_MAX_P) return SBP_ERR_DEGREE;
    if (n_elem <= 0 || !aligned8(coords) || !aligned8(metric) || !aligned8(jac)) return SBP_ERR_ARG;
    const double *D = device_D(p);
    if (!D) return SBP_ERR_HIP;
    return sbp::launch_metrics(p, n_elem, coords, metric, jac, D, (hipStream_t)stream) == 0
               ? SBP_OK : SBP_ERR_HIP;
}

int sbp_metrics_optimized(int32_t p, int64_t n_elem, const int32_t *nbr, const double *dxdxi,
                          double *metric, double *jac, void *stream) {
    if (p < 2 || p > SBP_MAX_P) return SBP_ERR_DEGREE;
    if (n_elem <= 0 || nbr == nullptr || (reinterpret_cast<uintptr_t>(nbr) % 4) != 0 ||
        !aligned8(dxdxi) || !aligned8(metric) || !aligned8(jac))
        return SBP_ERR_ARG;
    const int N = p + 1;
    if (n_elem > (int64_t)INT32_MAX || n_elem > (int64_t)(INT64_MAX / (18LL * N * N * N)))
        return SBP_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    // aligned conforming faces: every neighbour names this element back across the opposite face
    std::vector<int32_t> h(n_elem * 6);
    if (hipMemcpyAsync(h.data(), nbr, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SBP_ERR_HIP;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t nb = h[e * 6 + f];
            if (nb >= n_elem) return SBP_ERR_MESH;
            if (nb >= 0 && h[(int64_t)nb * 6 + (f ^ 1)] != e) return SBP_ERR_MESH;
        }
    static std::mutex mu;
    static sbp::OptMetricTables tabs[SBP_MAX_P + 1];
    static bool built[SBP_MAX_P + 1] = {};
    sbp::OptMetricTables t;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!built[p]) {
            if (!opt_metric_tables(p, tabs[p])) return SBP_ERR_DEGREE;
            built[p] = true;
        }
        t = tabs[p];
    }
    const int rc = sbp::optimized_metrics(t, n_elem, nbr, dxdxi, metric, jac, s);
    return rc == 0 ? SBP_OK : (rc == 2 ? SBP_ERR_MESH : SBP_ERR_HIP);
}

size_t sbp_workspace_bytes(const sbp_problem *probs, int32_t n_prob) {
    if (probs == nullptr || n_prob < 1) return 0;
    for (int b = 0; b < n_prob; ++b)
        if (check_problem(probs[b]) != SBP_OK) return 0;
    return layout_of(probs, n_prob).bytes;
}

int sbp_residual(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt, void *ws,
                 size_t ws_bytes, void *stream) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (!aligned8(q) || !aligned8(dqdt) || q == dqdt) return SBP_ERR_ARG;
    Plan *plan = get_plan(probs, n_prob, static_cast<char *>(ws), L);
    if (!plan) return SBP_ERR_HIP;
    return residual_all(plan, q, dqdt, static_cast<char *>(ws), (hipStream_t)stream);
}

int sbp_rk_step(const sbp_problem *probs, int32_t n_prob, double *q, const double *dt,
                int32_t n_steps, void *ws, size_t ws_bytes, void *stream) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (!aligned8(q) || !aligned8(dt) || n_steps < 0) return SBP_ERR_ARG;
    if (n_steps == 0) return SBP_OK;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SBP_ERR_HIP;
    // operator tables and plan exist before capture (no allocation inside a capture)
    for (int b = 0; b < n_prob; ++b)
        if (!device_D(probs[b].p)) return SBP_ERR_HIP;
    Plan *plan = get_plan(probs, n_prob, static_cast<char *>(ws), L);
    if (!plan) return SBP_ERR_HIP;
    GraphKey key{std::string(reinterpret_cast<const char *>(probs), sizeof(sbp_problem) * n_prob),
                 q, dt, ws, dev, plan->generation};
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) exec = it->second;
    }
    if (exec == nullptr) {
        rc = record_rk_graph(plan, q, dt, static_cast<char *>(ws), L, &exec);
        if (rc != SBP_OK) return rc;
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_graphs[key] = exec;
    }
    for (int i = 0; i < n_steps; ++i)
        if (hipGraphLaunch(exec, s) != hipSuccess) return SBP_ERR_HIP;
    return SBP_OK;
}

int sbp_residual_vjp(const sbp_problem *probs, int32_t n_prob, const double *q, const double *gbar,
                     double *qbar, void *ws, size_t ws_bytes, void *stream) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (!aligned8(q) || !aligned8(gbar) || !aligned8(qbar) || qbar == q || qbar == gbar)
        return SBP_ERR_ARG;
    for (int b = 0; b < n_prob; ++b)
        if (probs[b].p > SBP_MAX_VJP_P) return SBP_ERR_DEGREE;
    char *w = static_cast<char *>(ws);
    size_t off = 0;
    for (int b = 0; b < n_prob; ++b) {
        const sbp_problem &pr = probs[b];
        const int N = pr.p + 1;
        sbp::VjpArgs a{};
        a.q = q + off;
        a.gbar = gbar + off;
        a.qbar = qbar + off;
        a.metric = pr.metric;
        a.jac = pr.jac;
        a.nbr = pr.nbr;
        a.thb = pr.mu > 0.0 ? reinterpret_cast<double *>(w + L.thb[b]) : nullptr;
        a.bc = pr.bc_state;
        a.orient = pr.face_orient;
        a.status = reinterpret_cast<int *>(w);
        a.bnd_seen = reinterpret_cast<int *>(w) + 1;
        a.gen = next_vjp_mark();
        a.D = device_D(pr.p);
        if (a.D == nullptr) return SBP_ERR_HIP;
        a.K = pr.n_elem;
        a.nodes = pr.n_elem * (long long)N * N * N;
        a.gamma = pr.gamma;
        a.R = pr.R;
        a.mu = pr.mu;
        a.Pr = pr.Pr;
        a.eta = pr.eta;
        a.w_end = host_op(pr.p).w[0];
        a.iface_diss = pr.iface_diss;
        a.two_point = pr.two_point;
        if (sbp::launch_vjp(pr.p, a, (hipStream_t)stream) != 0) return SBP_ERR_HIP;
        off += 5 * (size_t)nodes_of(pr);
    }
    return SBP_OK;
}

namespace {
// Event pairs of the launches recorded without waiting (sbp_profile_residual with kernel_ms NULL).
struct ProfileRing {
    std::vector<hipEvent_t> begin, end;
    int recorded = 0;
};
ProfileRing g_ring;
std::mutex g_ring_mu;
}  // namespace

int sbp_profile_residual(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt,
                         void *ws, size_t ws_bytes, void *stream, float *kernel_ms) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (n_prob != 1 || !aligned8(q) || !aligned8(dqdt) || q == dqdt) return SBP_ERR_ARG;
    sbp::KernelTimer &tm = sbp::residual_timer();
    std::lock_guard<std::mutex> lk(g_ring_mu);
    if (kernel_ms == nullptr) {
        // record into the next slot of the ring, do not wait
        if (g_ring.recorded >= SBP_PROFILE_SLOTS) return SBP_ERR_ARG;
        if (g_ring.recorded == (int)g_ring.begin.size()) {
            hipEvent_t b = nullptr, e = nullptr;
            if (hipEventCreate(&b) != hipSuccess) return SBP_ERR_HIP;
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipEventDestroy(b);
                return SBP_ERR_HIP;
            }
            g_ring.begin.push_back(b);
            g_ring.end.push_back(e);
        }
        tm.begin = g_ring.begin[g_ring.recorded];
        tm.end = g_ring.end[g_ring.recorded];
    } else {
        static hipEvent_t b0 = nullptr, e0 = nullptr;
        if (b0 == nullptr) {
            if (hipEventCreate(&b0) != hipSuccess || hipEventCreate(&e0) != hipSuccess) return SBP_ERR_HIP;
        }
        tm.begin = b0;
        tm.end = e0;
    }
    Plan *plan = get_plan(probs, n_prob, static_cast<char *>(ws), L);
    if (!plan) return SBP_ERR_HIP;
    tm.enabled = true;
    rc = residual_group(plan->groups[0], q, dqdt, static_cast<char *>(ws), (hipStream_t)stream, true,
                        plan->groups[0].variant);
    tm.enabled = false;
    if (rc != SBP_OK) return rc;
    if (kernel_ms == nullptr) {
        ++g_ring.recorded;
        return SBP_OK;
    }
    if (hipEventSynchronize(tm.end) != hipSuccess) return SBP_ERR_HIP;
    if (hipEventElapsedTime(kernel_ms, tm.begin, tm.end) != hipSuccess) return SBP_ERR_HIP;
    return SBP_OK;
}

int sbp_profile_collect(int32_t *count, double *total_ms) {
    if (count == nullptr || total_ms == nullptr) return SBP_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_ring_mu);
    double sum = 0.0;
    for (int i = 0; i < g_ring.recorded; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(g_ring.end[i]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_ring.begin[i], g_ring.end[i]) != hipSuccess)
            return SBP_ERR_HIP;
        sum += ms;
    }
    *count = g_ring.recorded;
    *total_ms = sum;
    g_ring.recorded = 0;
    return SBP_OK;
}

int sbp_autotune(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt, void *ws,
                 size_t ws_bytes, void *stream, int32_t reps, int32_t *chosen) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (!aligned8(q) || !aligned8(dqdt) || q == dqdt || reps < 1) return SBP_ERR_ARG;
    Plan *plan = get_plan(probs, n_prob, static_cast<char *>(ws), L);
    if (!plan) return SBP_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SBP_ERR_HIP;
    for (auto &g : plan->groups) {
        const int nv = (g.flux == 0 && !g.md && !g.orient) ? sbp::schedule_count(g.p) : 1;
        float best = 0.0f;
        int best_v = 0;
        for (int v = 0; v < nv; ++v) {
            rc = residual_group(g, q, dqdt, static_cast<char *>(ws), s, false, v);  // warm-up
            if (rc != SBP_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = SBP_ERR_HIP; break; }
            for (int r = 0; r < reps && rc == SBP_OK; ++r)
                rc = residual_group(g, q, dqdt, static_cast<char *>(ws), s, false, v);
            if (rc != SBP_OK || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess) {
                rc = SBP_ERR_HIP;
                break;
            }
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = SBP_ERR_HIP; break; }
            if (v == 0 || ms < best) { best = ms; best_v = v; }
        }
        if (rc != SBP_OK) break;
        g.variant = best_v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SBP_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        plan->generation = ++g_generation;  // graphs recorded with the old schedules are not reused
    }
    if (chosen) {
        for (int b = 0; b < n_prob; ++b) chosen[b] = 0;
        for (const auto &g : plan->groups)
            for (int b : g.members) chosen[b] = g.variant;
    }
    return SBP_OK;
}

int sbp_set_schedule(const sbp_problem *probs, int32_t n_prob, void *ws, size_t ws_bytes, int32_t p,
                     int32_t variant) {
    Layout L;
    int rc = validate(probs, n_prob, ws, ws_bytes, L);
    if (rc != SBP_OK) return rc;
    if (p < 1 || p > SBP_MAX_P) return SBP_ERR_DEGREE;
    if (variant < 0 || variant >= sbp::schedule_count(p)) return SBP_ERR_ARG;
    Plan *plan = get_plan(probs, n_prob, static_cast<char *>(ws), L);
    if (!plan) return SBP_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto &g : plan->groups)
        if (g.p == p) {
            if ((g.flux != SBP_FLUX_CHANDRASHEKAR || g.md || g.orient) && variant != 0) return SBP_ERR_ARG;
            g.variant = variant;
        }
    plan->generation = ++g_generation;
    return SBP_OK;
}

int sbp_release(void *ws) {
    if (ws == nullptr) return SBP_ERR_ARG;
    // no launch recorded with these plans or graphs may still be running
    if (hipDeviceSynchronize() != hipSuccess) return SBP_ERR_HIP;
    int released = 0;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto it = g_graphs.begin(); it != g_graphs.end();) {
            if (it->first.ws == ws) {
                (void)hipGraphExecDestroy(it->second);
                it = g_graphs.erase(it);
                ++released;
            } else {
                ++it;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (auto it = g_plans.begin(); it != g_plans.end();) {
            if (it->second->ws == ws) {
                free_plan(it->second);
                it = g_plans.erase(it);
                ++released;
            } else {
                ++it;
            }
        }
    }
    return released;
}

int sbp_residual_noalloc(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt,
                         int32_t *status, void *stream) {
    static_assert(SBP_NOALLOC_SCRATCH_BYTES == sbp::kNoallocScratchBytes, "scratch size");
    if (probs == nullptr || n_prob < 1 || n_prob > SBP_NOALLOC_MAX_PROBLEMS) return SBP_ERR_ARG;
    for (int b = 0; b < n_prob; ++b) {
        const int rc = check_problem(probs[b]);
        if (rc != SBP_OK) return rc;
    }
    if (!aligned8(q) || !aligned8(dqdt) || q == dqdt || status == nullptr ||
        (reinterpret_cast<uintptr_t>(status) % 4) != 0)
        return SBP_ERR_ARG;
    // Scratch layout: [derivative tables, p = 0..15 | group tables | per viscous problem: face
    // traces, then (p >= 9) the plane passes' per-node scratch].  Checked before any device work.
    constexpr size_t kDBytes = sizeof(double) * 256 * (kMaxOpP + 1);
    constexpr size_t kTableBytes = size_t(32) << 10;
    std::vector<size_t> trace(n_prob, 0), aux(n_prob, 0);
    size_t off = kDBytes + kTableBytes;
    for (int b = 0; b < n_prob; ++b) {
        const sbp_problem &pr = probs[b];
        if (!(pr.mu > 0.0)) continue;
        const size_t N = pr.p + 1;
        trace[b] = off;
        off += align_up(sizeof(double) * (size_t)pr.n_elem * 6 * 4 * N * N);
        if (pr.p >= sbp::kFirstPlaneP) {
            aux[b] = off;
            off += align_up(sizeof(double) * 16 * (size_t)nodes_of(pr));
        }
    }
    if (off > SBP_NOALLOC_SCRATCH_BYTES) return SBP_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    static const std::vector<double> dtab = [] {
        std::vector<double> t(256 * (kMaxOpP + 1), 0.0);
        for (int pp = 1; pp <= kMaxOpP; ++pp)
            std::memcpy(t.data() + 256 * pp, host_op(pp).D, sizeof(double) * (pp + 1) * (pp + 1));
        return t;
    }();
    char *scr = nullptr;
    if (sbp::noalloc_scratch(dtab.data(), (long long)dtab.size(), s, &scr) != 0) return SBP_ERR_HIP;
    // group tables packed into 8-byte words, uploaded through kernel arguments
    std::vector<GroupPlan> groups;
    group_problems(probs, n_prob, groups);
    const std::vector<long long> soff = state_offsets(probs, n_prob);
    std::vector<unsigned long long> words;
    auto put = [&words](const void *data, size_t bytes) {
        const size_t at = words.size();
        words.resize(at + (bytes + 7) / 8, 0ull);
        std::memcpy(words.data() + at, data, bytes);
        return at * 8;
    };
    struct Where {
        size_t probs, ns, bs;
    };
    std::vector<Where> where;
    for (auto &g : groups) {
        std::vector<sbp::ProbDev> host;
        std::vector<long long> ns(1, 0);
        for (int b : g.members) {
            host.push_back(prob_dev(probs[b], b, soff[b], reinterpret_cast<double *>(scr + trace[b]),
                                    reinterpret_cast<double *>(scr + aux[b])));
            ns.push_back(ns.back() + host.back().nodes);
        }
        const std::vector<long long> bs = block_starts(probs, g, sbp::schedule_of(g.p, 0).epw);
        g.total_nodes = ns.back();
        g.total_blocks[sbp::schedule_of(g.p, 0).epw] = bs.back();
        Where w;
        w.probs = put(host.data(), sizeof(sbp::ProbDev) * host.size());
        w.ns = put(ns.data(), sizeof(long long) * ns.size());
        w.bs = put(bs.data(), sizeof(long long) * bs.size());
        where.push_back(w);
    }
    if (words.size() * 8 > kTableBytes) return SBP_ERR_ARG;  // not reached with <= 16 problems
    char *tab = scr + kDBytes;
    if (sbp::fill_words(tab, words.data(), (long long)words.size(), s) != 0) return SBP_ERR_HIP;
    for (size_t i = 0; i < groups.size(); ++i) {
        const GroupPlan &g = groups[i];
        sbp::GroupArgs a{};
        a.probs = reinterpret_cast<const sbp::ProbDev *>(tab + where[i].probs);
        a.node_start = reinterpret_cast<const long long *>(tab + where[i].ns);
        a.block_start = reinterpret_cast<const long long *>(tab + where[i].bs);
        a.n = (int)g.members.size();
        a.total_blocks = g.total_blocks.at(sbp::schedule_of(g.p, 0).epw);
        a.total_nodes = g.total_nodes;
        a.q = q;
        a.out = dqdt;
        a.status = status;
        a.D = reinterpret_cast<const double *>(scr) + 256 * g.p;
        if (sbp::launch_group_residual(g.p, g.visc, g.flux, g.md, g.orient, 0, a, s, true) != 0)
            return SBP_ERR_HIP;
    }
    return SBP_OK;
}

int sbp_schedule_count(int32_t p) { return (p < 1 || p > SBP_MAX_P) ? 0 : sbp::schedule_count(p); }

int sbp_status(void *ws, void *stream, int32_t *flags) {
    if (ws == nullptr || flags == nullptr) return SBP_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return SBP_ERR_HIP;
    int host = 0;
    if (hipMemcpy(&host, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SBP_ERR_HIP;
    const int zero = 0;
    if (hipMemcpy(ws, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SBP_ERR_HIP;
    *flags = host;
    if (host & sbp::FLAG_NONPHYSICAL) return SBP_ERR_NONPHYSICAL;
    if (host & sbp::FLAG_MESH) return SBP_ERR_MESH;
    return SBP_OK;
}

}  // extern "C"
