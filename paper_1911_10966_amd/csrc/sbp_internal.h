// Internal declarations shared by the C-ABI layer (sbp_capi.cpp) and the gfx950 kernels
// (sbp_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbp {

enum : int { FLAG_NONPHYSICAL = 1, FLAG_MESH = 2 };

// Everything a residual launch for one problem needs.  Arrays are device pointers.
struct ResArgs {
    const double *q;       // SoA [5][nodes]
    double *out;           // SoA [5][nodes]
    const double *metric;  // SoA [9][nodes]
    const double *jac;     // [nodes]
    const int32_t *nbr;    // [K][6]
    double *trace;         // viscous face traces [K][6][4][N^2] (mu > 0 only)
    int *status;           // sticky flags
    const double *D;       // [N*N] collocation derivative
    long long K;
    long long nodes;
    double gamma, R, mu, Pr, eta;
    double w_end;          // end weight of the 1-D norm
    int iface_diss;
    int two_point;
};

// RK4 stage update, see launch_rk_stage.
struct RkArgs {
    double *q;
    double *acc;
    double *qs;
    const double *k;
    const double *dt;      // device scalar
    long long n;           // number of doubles (5 * nodes)
    int stage;
};

// Main residual kernel; with fixup the neighbour half of SAT^V is added by a second kernel,
// without it the caller must apply it (launch_rk_fixup_stage does, for RK stages).
int launch_residual(int p, const ResArgs &a, hipStream_t s, bool fixup = true);
int launch_rk_fixup_stage(int p, const ResArgs &a, const RkArgs &r, hipStream_t s);

// Optional event timing of the main residual kernel (see sbp_profile in the C ABI).
struct KernelTimer {
    bool enabled = false;
    hipEvent_t begin = nullptr, end = nullptr;
};
KernelTimer &residual_timer();
int launch_rk_stage(const RkArgs &a, hipStream_t s);

// Vector-Jacobian product of the residual (Chandrashekar flux) for one problem.
struct VjpArgs {
    const double *q;       // SoA [5][nodes]
    const double *gbar;    // cotangent of dq/dt, SoA [5][nodes]
    double *qbar;          // result, SoA [5][nodes]
    const double *metric;
    const double *jac;
    const int32_t *nbr;
    double *thb;           // cotangents of the BR1 gradients, [3][4][nodes] (mu > 0 only)
    int *status;
    const double *D;
    long long K;
    long long nodes;
    double gamma, R, mu, Pr, eta;
    double w_end;
    int iface_diss;
};
int launch_vjp(int p, const VjpArgs &a, hipStream_t s);
int launch_metrics(int p, long long K, const double *x, double *metric, double *jac,
                   const double *D, hipStream_t s);

}  // namespace sbp
