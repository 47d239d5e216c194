// Internal declarations shared by the C-ABI layer (sbp_capi.cpp) and the gfx950 kernels
// (sbp_kernels.hip, sbp_planes.hip, sbp_vjp.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbp {

enum : int { FLAG_NONPHYSICAL = 1, FLAG_MESH = 2 };

// Device code reaches the problem arrays through pointers read from memory (the group's problem
// table), whose address space the compiler cannot infer; without this qualifier every access
// becomes a flat instruction, which also counts against the LDS wait counter.
#if defined(__HIP_DEVICE_COMPILE__)
#define SBP_GLOBAL __attribute__((address_space(1)))
#else
#define SBP_GLOBAL
#endif

// Everything a residual launch for one problem needs.  Arrays are device pointers.
struct ResArgs {
    const SBP_GLOBAL double *q;       // SoA [5][nodes]
    SBP_GLOBAL double *out;           // SoA [5][nodes]
    const SBP_GLOBAL double *metric;  // SoA [9][nodes]
    const SBP_GLOBAL double *jac;     // [nodes]
    const SBP_GLOBAL int32_t *nbr;    // [K][6]
    SBP_GLOBAL double *trace;         // viscous face traces [K][6][4][N^2] (mu > 0 only)
    SBP_GLOBAL double *aux;           // viscous per-node scratch of the plane kernels, [16][nodes]
    const SBP_GLOBAL double *bc;      // Dirichlet state of boundary faces, SoA [5][nodes], or null
    const SBP_GLOBAL double *src;     // source added to dq/dt, SoA [5][nodes], or null
    const SBP_GLOBAL int32_t *orient; // face orientation [K][6] (f' + 8 code), or null (aligned)
    int *status;                      // sticky flags
    const double *D;       // [N*N] collocation derivative
    long long K;
    long long nodes;
    double gamma, R, mu, Pr, eta;
    double w_end;          // end weight of the 1-D norm
    double isw;            // 1 / w_end
    double kap;            // thermal conductivity mu c_p / Pr
    int iface_diss;
    int two_point;
};

// Static per-problem data of a group launch (device table entry).  `off` is the offset, in
// doubles, of the problem's component-0 block in the concatenated state arrays.
struct ProbDev {
    const double *metric;
    const double *jac;
    const int32_t *nbr;
    double *trace;
    double *thb;
    const double *bc;
    const double *src;
    const int32_t *orient;
    long long K;
    long long nodes;
    long long off;
    double gamma, R, mu, Pr, eta;
    double w_end;
    double isw;
    double kap;
    int iface_diss;
    int two_point;
    int dt_index;
    int pad;
};

// One launch over all problems of a group (same degree, viscosity on/off and flux).
struct GroupArgs {
    const ProbDev *probs;          // device [n]
    const long long *block_start;  // device [n+1]: prefix sums of element tiles per problem
    const long long *node_start;   // device [n+1]: prefix sums of nodes per problem
    int n;
    long long total_blocks;
    long long total_nodes;
    const double *q;               // base of the concatenated input state
    double *out;                   // base of the concatenated output
    int *status;
    const double *D;
};

// RK4 stage update over a group: base pointers of the concatenated buffers.
struct RkGroupArgs {
    double *q;
    double *acc;
    double *qs;
    const double *k;
    const double *dt;              // device [n_prob of the whole set], indexed by ProbDev::dt_index
    int stage;
};

// Schedules of the residual kernel: elements per workgroup and whether the grid is persistent.
struct Schedule {
    int epw;
    int persistent;
    int wpe;        // minimum waves per SIMD requested from the register allocator (0: none)
};
int schedule_count(int p);
Schedule schedule_of(int p, int variant);
// md: matrix interface dissipation (iface_diss = 2; default schedule, fluxes 0 and 2 only).
// orient: the group's problems carry face-orientation tables (default schedule).
int launch_group_residual(int p, bool visc, int flux, bool md, bool orient, int variant,
                          const GroupArgs &g, hipStream_t s, bool fixup);
int launch_group_rk_stage(int p, bool visc, const GroupArgs &g, const RkGroupArgs &r, hipStream_t s);
// Degrees whose elements exceed one workgroup (p >= 9) run as passes over node planes; a
// schedule's `epw` is then the number of planes per workgroup.
constexpr int kFirstPlaneP = 9;
int launch_group_residual_planes(int p, int ppb, bool visc, int flux, bool md, bool orient,
                                 const GroupArgs &g, hipStream_t s);
int launch_metrics_big(int p, long long K, const double *x, double *metric, double *jac,
                       const double *D, hipStream_t s);



// Library-owned scratch of the allocation-free residual (sbp_noalloc.hip): bytes of the device
// array, words per table-upload launch (carried in kernel arguments), the upload itself, and the
// per-device address of the array (set up on the first call on a device, which also writes the
// collocation-derivative tables d_tables[n_words] at its start and waits for stream s).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kFillWords = 256;
int fill_words(void *dst, const unsigned long long *src, long long n, hipStream_t s);
int noalloc_scratch(const double *d_tables, long long n_words, hipStream_t s, char **ptr);

// Optional event timing of the main residual kernel (see sbp_profile in the C ABI).
struct KernelTimer {
    bool enabled = false;
    hipEvent_t begin = nullptr, end = nullptr;
};
KernelTimer &residual_timer();

// Vector-Jacobian product of the residual (Chandrashekar flux) for one problem.
struct VjpArgs {
    const double *q;       // SoA [5][nodes]
    const double *gbar;    // cotangent of dq/dt, SoA [5][nodes]
    double *qbar;          // result, SoA [5][nodes]
    const double *metric;
    const double *jac;
    const int32_t *nbr;
    double *thb;           // cotangents of the BR1 gradients, [3][4][nodes] (mu > 0 only)
    const double *bc;      // Dirichlet state of boundary faces, SoA [5][nodes], or null
    const int32_t *orient; // face orientation [K][6] (f' + 8 code), or null (aligned faces)
    int *status;
    int *bnd_seen;         // set to `gen` by the pass that meets a boundary face
    int gen;               // this launch's mark (distinct per launch)
    const double *D;
    long long K;
    long long nodes;
    double gamma, R, mu, Pr, eta;
    double w_end;
    int iface_diss;
    int two_point;         // volume form: 0 Chandrashekar, 1 central, 2 Kennedy-Gruber, 3 standard DC
};
int launch_vjp(int p, const VjpArgs &a, hipStream_t s);
int launch_metrics(int p, long long K, const double *x, double *metric, double *jac,
                   const double *D, hipStream_t s);

// Optimised metric terms (reading of the metric-terms paragraph after eq. discGCLconvection):
// analytic metrics from the mapping derivative, face-normal values corrected by the least-norm
// amount that meets every element's compatibility conditions, then the other entries moved by the
// least-norm amount that satisfies the discrete GCL.  The host supplies the degree's tables.
struct OptMetricTables {
    int p;
    double D[256];      // collocation derivative, row-major
    double V[256];      // V[i * N + k]: component i of the k-th eigenvector of B = D diag(0,1..1,0) D^T
    double lam[16];     // eigenvalues of B; exactly 0 on its two-dimensional null space
    int null_mask;      // bit k set: eigenvector k belongs to that null space
    double pat[2][16];  // face patterns: [0] the left null vector of D, [1] the LGL weights
};
// 0 on success, 1 on a HIP error, 2 when the compatibility system did not converge.
int optimized_metrics(const OptMetricTables &t, long long K, const int32_t *nbr,
                      const double *dxdxi, double *metric, double *jac, hipStream_t s);

}  // namespace sbp
