/*
 * sbp.h -- C ABI of the MI355X (gfx950) library that evaluates the semi-discrete residual of the
 * entropy-stable SBP-SAT discontinuous collocation discretization (ES-C) of the compressible
 * Navier-Stokes equations on conforming curvilinear hexahedra, as defined in Rojas, Boukharfane,
 * Dalcin, Del Rey Fernandez, Ranocha, Keyes and Parsani, "On the robustness and performance of
 * entropy stable discontinuous collocation methods for the compressible Navier-Stokes equations"
 * (arXiv 1911.10966), section "Discretization of the compressible Navier-Stokes equations".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - N = p + 1 Legendre-Gauss-Lobatto nodes per direction (Notation section, Definition "SBP").
 * - Element e has N^3 nodes numbered i1 + N*i2 + N*N*i3 (xi_1 fastest).  Node-wise arrays are
 *   structure-of-arrays: component c of node n of a problem with K elements sits at [c*K*N^3 + e*N^3 + n].
 * - State q = [rho, rho U_1, rho U_2, rho U_3, rho E] (eq. compressible_ns), 5 components.
 * - metric: 9 components, entry 3*l + m is J dxi_l/dx_m (0-based l, m) at the node; jac: J > 0.
 *   These are the diagonal matrices [A_lm] and J_kappa of the linear convection-diffusion section.
 *   The residual is entropy conservative only when the metrics satisfy the discrete geometric
 *   conservation law (eq. discGCLconvection); sbp_metrics() produces such metrics (curl form).
 * - nbr: [K][6] int32, face f = 2*l + s (s = 0 for the xi_l = -1 face, 1 for xi_l = +1) of element e
 *   touches element nbr[e*6 + f]; faces are conforming, and aligned (the neighbour's opposite face,
 *   same tangential node indices) unless the problem carries a face_orient table (unstructured
 *   meshes, below).  Periodic grids list wrap-around neighbours.  A negative entry
 *   makes the face a boundary face of the kind it names (SBP_BC_*, below); any other entry outside
 *   [0, K) is a mesh error (sticky flag, SBP_ERR_MESH from sbp_status()).
 * - Pointers marked "device" are HIP device allocations owned by the caller; the library never
 *   frees them and keeps no reference after the call returns (stream-ordered work may still read
 *   them until the stream reaches that point).  All device arrays must be 8-byte aligned.
 * - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued asynchronously; argument
 *   and launch errors are returned immediately.  Non-physical states (rho <= 0, P <= 0 or a
 *   non-finite value) raise a sticky device flag that sbp_status() reports.
 * - Return codes: SBP_OK or a negative SBP_ERR_* code; sbp_error_string() describes it.
 */
#ifndef SBP_H
#define SBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBP_OK 0
#define SBP_ERR_ARG (-1)         /* null/misaligned pointer, bad size, bad option value       */
#define SBP_ERR_DEGREE (-2)      /* p outside [1, SBP_MAX_P]                                   */
#define SBP_ERR_MESH (-3)        /* neighbour index outside [0, K)                             */
#define SBP_ERR_NONPHYSICAL (-4) /* reported by sbp_status: rho <= 0, P <= 0 or non-finite    */
#define SBP_ERR_HIP (-5)         /* a HIP runtime call failed                                  */
#define SBP_ERR_WORKSPACE (-6)   /* workspace missing or smaller than sbp_workspace_bytes()    */
#define SBP_ERR_SCRATCH (-7)     /* problem set exceeds SBP_NOALLOC_SCRATCH_BYTES              */

#define SBP_MAX_P 15      /* degrees 1..8 run one workgroup per element tile; 9..15 (the cost */
                         /* study of the Taylor-Green section goes up to p = 15) run as      */
                         /* passes over node planes                                          */
#define SBP_MAX_VJP_P 8  /* sbp_residual_vjp covers degrees 1..8                             */

#define SBP_FLUX_CHANDRASHEKAR 0 /* entropy-conservative two-point flux (ES-C)                 */
#define SBP_FLUX_CENTRAL 1       /* arithmetic mean of the nodal fluxes                        */
#define SBP_FLUX_KENNEDY_GRUBER 2 /* split form SF-KG                                          */
#define SBP_FLUX_DC 3            /* standard DC: SBP derivative of the nodal fluxes, central   */
                                 /* interface flux                                             */

/* One problem: a mesh of K elements of degree p.  Constants follow the constituent relations of
 * the compressible Navier-Stokes section: P = rho R T, c_p = gamma R / (gamma - 1), constant
 * viscosity mu and conductivity kappa = mu c_p / Pr; mu == 0 evaluates the Euler residual only. */
typedef struct sbp_problem {
    int32_t p;              /* polynomial degree, 1..SBP_MAX_P                                 */
    int32_t iface_diss;     /* interface dissipation: 0 none (entropy conservative), 1 local   */
                            /* Lax-Friedrichs, 2 entropy-stable matrix dissipation             */
                            /* |n| R|Lambda|T R^T (w_i - w_nu) (Roe-type, in entropy variables; */
                            /* with the Chandrashekar or Kennedy-Gruber flux, default schedule) */
    int64_t n_elem;         /* K > 0                                                           */
    const int32_t *nbr;     /* device [K][6]                                                   */
    const double *metric;   /* device SoA [9][K*N^3]                                           */
    const double *jac;      /* device [K*N^3]                                                  */
    double gamma, R, mu, Pr;
    double eta;             /* interior-penalty coefficient >= 0                               */
    int32_t two_point;      /* SBP_FLUX_*: inviscid volume form and interface flux            */
    int32_t reserved;       /* must be 0                                                       */
    /* Optional device SoA [5][K*N^3] arrays (NULL = absent):
     * bc_state: prescribed state of SBP_BC_DIRICHLET faces; only the entries at their face nodes
     *   are read.  Without bc_state, nbr == SBP_BC_DIRICHLET is a mesh error.
     * source: forcing added to dq/dt (e.g. of a manufactured solution). */
    const double *bc_state;
    const double *source;
    /* Optional device [K][6] int32 (NULL = aligned faces): face orientation of unstructured
     * meshes.  For an interior face f of element e, face_orient[e*6 + f] = f' + 8*code: the
     * neighbour's face f' = 2*l' + s' (any of its six) and the orientation code (0..7) of its
     * face-node grid on the own one.  With the own face node's tangential indices (a, b) (the two
     * indices other than i_l, in increasing direction order), the partner node has tangential
     * indices (a', b') = (F_a(x), F_b(y)), (x, y) = (b, a) if bit 0 of code is set, else (a, b),
     * F_a(x) = N-1-x if bit 1 is set (else x), F_b(y) = N-1-y if bit 2 is set (else y).  The
     * partner's metric row and contravariant viscous flux are those of its direction l', times
     * -1 when s' == s.  Entries of boundary faces are not read; an entry outside that range on an
     * interior face is a mesh error (sticky flag).  NULL means f' = f ^ 1 and code 0. */
    const int32_t *face_orient;
} sbp_problem;

/* Boundary kinds, written into nbr in place of a neighbour index.  A boundary face node's partner
 * is a ghost node with the own node's metrics and J; the inviscid SAT, interface dissipation,
 * SAT^theta and interior penalty keep their interface form with that partner (the boundary SATs
 * of the references the paper names for walls and far fields are not given in it; these forms are
 * entropy stable, see each kind).
 * SBP_BC_DIRICHLET: the ghost carries bc_state; SAT^V vanishes (the boundary viscous flux is the
 *   own one).  A far field is this kind with free-stream data.
 * SBP_BC_SLIP_WALL (inviscid problems only; with mu > 0 a mesh error): the ghost is the own state
 *   with the momentum reflected about the face, m - 2 (m.n) n, n = A_l/|A_l|.  The shared flux
 *   then carries the pressure alone, the wall produces no entropy with iface_diss 0, and the
 *   dissipation acts on the normal momentum.
 * SBP_BC_ADIABATIC_WALL: no-slip wall with no heat flux.  The ghost is the own state with the
 *   momentum reversed (zero velocity and the own temperature on average); SAT^V is
 *   -(s / w_end) fhat_l,i on the energy equation only (the wall does no work and passes no heat).
 *   Mass and energy are conserved exactly, and the wall's entropy terms are the dissipation and
 *   the interior penalty alone. */
#define SBP_BC_DIRICHLET (-1)
#define SBP_BC_SLIP_WALL (-2)
#define SBP_BC_ADIABATIC_WALL (-3)

/* Library version, for diagnostics. */
int sbp_version(void);

/* Human-readable text for a return code (static storage). */
const char *sbp_error_string(int code);

/* The 1-D degree-p LGL SBP operator (Notation section, Definition "SBP"): nodes x[N] in [-1, 1],
 * quadrature weights w[N] (the diagonal norm P) and the collocation derivative D[N*N] (row-major,
 * D = P^{-1} Q, exact for polynomials of degree <= p).  Host pointers owned by the caller.
 * Any of x, w, D may be NULL.  Returns SBP_ERR_DEGREE for p outside [1, 15]. */
int sbp_lgl_operator(int32_t p, double *x, double *w, double *D);

/* Curl-form metric terms J dxi_l/dx_m and Jacobian J from nodal coordinates (linear
 * convection-diffusion section: metric terms [A_lm] satisfying eq. discGCLconvection).
 * coords: device SoA [3][K*N^3] physical coordinates; metric: device [9][K*N^3] out; jac: device
 * [K*N^3] out.  The derivatives are the degree-p collocation derivative along each direction. */
int sbp_metrics(int32_t p, int64_t n_elem, const double *coords, double *metric, double *jac,
                void *stream);

/* Optimised metric terms (the paragraph after eq. discGCLconvection: analytic metrics on the faces,
 * and volume metrics that satisfy the discrete GCL while staying as close as possible to the
 * analytic ones), for meshes whose faces are aligned and conforming.  Steps:
 * 1. analytic metrics J dxi_l/dx_m = (a_{l+1} x a_{l+2})_m and J = a_1 . (a_2 x a_3) from the
 *    covariant vectors a_i = dx/dxi_i at the nodes;
 * 2. the face-normal components (J dxi_l/dx_m on the faces normal to xi_l) take one value per face
 *    node, the mean of the two elements' analytic values, corrected by the least-norm amount (2-norm
 *    over all face nodes of the mesh) for which every element can satisfy the GCL: with those values
 *    held, the GCL of an element has a solution only if 7 linear combinations of its face values
 *    vanish (tensor products of the LGL weights and of the left null vector of D; the all-weights
 *    one is the closure of the element's surface);
 * 3. per element and m, the other entries move by the least-norm amount (2-norm) that makes
 *    sum_l D_l [J dxi_l/dx_m] vanish at every node.
 * The result satisfies eq. discGCLconvection to rounding, both elements of a face store identical
 * face-normal values, and on affine elements it equals the analytic metrics.
 * p: 2..SBP_MAX_P; nbr: device int32 [K][6] as in sbp_problem (negative entries are boundary
 * faces; every non-negative entry must name an element whose opposite face names this element
 * back, i.e. no face_orient rotations); dxdxi: device SoA [9][K*N^3], entry 3*m + i is dx_m/dxi_i
 * (0-based) at the node, e.g. the closed-form derivative of the mapping; metric: device [9][K*N^3]
 * out, as for sbp_metrics; jac: device [K*N^3] out (the analytic J).  All arrays are owned by the
 * caller; metric and jac must not overlap the inputs.
 * The call is synchronous: it reads the neighbour table on the host, allocates temporary device
 * memory (about (18 N^2 + 90) doubles per element) and waits for the stream before returning.
 * Returns SBP_ERR_DEGREE for p outside [2, SBP_MAX_P], SBP_ERR_ARG for bad sizes or pointers,
 * SBP_ERR_MESH for a neighbour entry >= K or a face that is not paired back (and if the face
 * compatibility system does not converge, which does not happen on valid meshes), SBP_ERR_HIP for
 * runtime errors. */
int sbp_metrics_optimized(int32_t p, int64_t n_elem, const int32_t *nbr, const double *dxdxi,
                          double *metric, double *jac, void *stream);

/* Device workspace (bytes) needed by sbp_residual, sbp_rk_step and sbp_residual_vjp for this
 * problem set.  0 on invalid arguments. */
size_t sbp_workspace_bytes(const sbp_problem *probs, int32_t n_prob);

/* Semi-discrete residual dq/dt (eqs. discEL and NSL, divided by J): Hadamard flux differencing with
 * the two-point flux and averaged metrics, interface SATs (entropy-conservative flux plus optional
 * Lax-Friedrichs dissipation) and, for mu > 0, the BR1/interior-penalty viscous operator in entropy
 * variables.  probs: host array of n_prob >= 1 problems; q, dqdt: device arrays holding the problems'
 * SoA blocks back to back (problem b at offset 5 * sum_{b'<b} K_b' N_b'^3).  ws: device workspace of
 * ws_bytes >= sbp_workspace_bytes(probs, n_prob), owned by the caller; calls sharing a workspace
 * must be serialized on one stream.  dqdt must not alias q. */
int sbp_residual(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt,
                 void *ws, size_t ws_bytes, void *stream);

/* Classical fourth-order Runge-Kutta steps with fixed time steps: q <- RK4(q, dt[b]) n_steps times,
 * k1 = f(q), k2 = f(q + dt/2 k1), k3 = f(q + dt/2 k2), k4 = f(q + dt k3),
 * q <- q + dt/6 (k1 + 2 k2 + 2 k3 + k4), f the residual of sbp_residual.  The paper advances its
 * semi-discretization with an adaptive fifth-order Dormand-Prince pair (numerical results section,
 * time integration); this entry point instead takes the fixed steps dt the caller supplies, which
 * is what a step of the paper's method costs without the error control.
 * q: device in/out, same layout as sbp_residual; dt: device [n_prob].  The four stages of a step are
 * recorded once into a HIP graph per (problem set, q, dt, workspace) and replayed; the graph and
 * the launch plan stay cached until sbp_release(ws). */
int sbp_rk_step(const sbp_problem *probs, int32_t n_prob, double *q, const double *dt,
                int32_t n_steps, void *ws, size_t ws_bytes, void *stream);

/* Vector-Jacobian product qbar = (d(dq/dt)/dq)^T gbar of the residual of sbp_residual, with each
 * element recomputing its forward intermediates (no two-point fluxes are stored) and interface
 * terms gathered from both sides (no atomics).  q, gbar, qbar: device, same layout as q; qbar must
 * not alias q or gbar.  Available for every volume form (two_point 0..3) and interface dissipation
 * that sbp_residual accepts, on periodic or bounded problems (Dirichlet data is held fixed; wall
 * ghosts are differentiated through the own state) and with or without a face_orient table;
 * degrees above SBP_MAX_VJP_P give SBP_ERR_DEGREE, and invalid neighbour or orientation entries
 * raise the mesh flag as in sbp_residual.  A source term does not enter the product.  Non-smooth
 * points follow fixed conventions: d|x|/dx = +1 at x = 0, and the maximum in the Lax-Friedrichs
 * dissipation takes the own side on ties (a wall ghost's speed equals the own one, so the own
 * side carries it). */
int sbp_residual_vjp(const sbp_problem *probs, int32_t n_prob, const double *q, const double *gbar,
                     double *qbar, void *ws, size_t ws_bytes, void *stream);

/* Profiling variant of sbp_residual for one problem (n_prob == 1): the same launches, with HIP
 * events recorded on `stream` around the main residual kernel (around all plane passes for
 * p > 8).  With kernel_ms (host pointer) the call waits for the end event and stores that kernel's
 * duration in *kernel_ms.  With kernel_ms NULL it only records the events, into the next of at
 * most SBP_PROFILE_SLOTS slots (SBP_ERR_ARG when all are taken), and returns without waiting;
 * sbp_profile_collect() reads them.  Not thread-safe; not for use under graph capture. */
#define SBP_PROFILE_SLOTS 4096
int sbp_profile_residual(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt,
                         void *ws, size_t ws_bytes, void *stream, float *kernel_ms);

/* Waits for every launch recorded by sbp_profile_residual with kernel_ms NULL since the last call,
 * stores their number in *count and the sum of their main-kernel durations (ms) in *total_ms (host
 * pointers), and empties the slots. */
int sbp_profile_collect(int32_t *count, double *total_ms);

/* Autotuner: for each group of problems sharing degree, viscosity on/off and flux, times every
 * schedule of the residual kernel (elements per workgroup, one block per element tile or a
 * persistent grid; node planes per workgroup for p > 8) on these inputs, `reps` launches each after a warm-up, and keeps the fastest for
 * later calls with the same problem array and workspace.  Waits for `stream`.  dqdt is scratch
 * output.  chosen: optional host [n_prob] receiving the schedule index of each problem's group. */
int sbp_autotune(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt, void *ws,
                 size_t ws_bytes, void *stream, int32_t reps, int32_t *chosen);

/* Allocation-free residual, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result of sbp_residual with the
 * default schedule, computed by the same kernels, with no caller workspace and no allocation.  The
 * viscous face traces, the plane passes' scratch and the small device tables live in one
 * library-owned device array of SBP_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends;
 * its address is looked up, and the collocation-derivative tables written into it, on the first
 * call on each device (that call waits for `stream` once).
 * probs, n_prob (1..SBP_NOALLOC_MAX_PROBLEMS), q, dqdt, stream: as in sbp_residual.
 * status: device int32 owned by the caller; the launches OR the flag bits of sbp_status() into it
 * (bit 0 non-physical state, bit 1 mesh error) and never clear it: the caller zeroes it.
 * Needs, per viscous problem, 192 N^2 K bytes of face traces plus, for p >= 9, 128 N^3 K bytes of
 * per-node scratch (each rounded up to 256 B), all within SBP_NOALLOC_SCRATCH_BYTES less 64 KiB;
 * a larger set returns SBP_ERR_SCRATCH before any device work.  Every call on a GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other streams, other threads) race and give
 * wrong results; serialize them. */
#define SBP_NOALLOC_SCRATCH_BYTES (64u << 20)
#define SBP_NOALLOC_MAX_PROBLEMS 16
int sbp_residual_noalloc(const sbp_problem *probs, int32_t n_prob, const double *q, double *dqdt,
                         int32_t *status, void *stream);

/* Number of residual schedules available for degree p (0 if p is out of range). */
int sbp_schedule_count(int32_t p);

/* Pins schedule `variant` (0 <= variant < sbp_schedule_count(p); 0 is the default) for the groups of
 * degree p of this problem array and workspace, as sbp_autotune would.  Host call; no device work. */
int sbp_set_schedule(const sbp_problem *probs, int32_t n_prob, void *ws, size_t ws_bytes, int32_t p,
                     int32_t variant);

/* Waits for `stream`, then reports and clears the workspace's sticky device flags, which every
 * residual, RK4 and VJP launch with this workspace may raise (the calls themselves do not read them
 * back, so that they stay asynchronous):
 *   *flags (host) receives the flag word: bit 0 (value 1) a non-physical state (rho <= 0, P <= 0 or
 *   a non-finite value), bit 1 (value 2) a mesh error (a neighbour index outside [0, K) that names
 *   no boundary kind, boundary data missing for a Dirichlet face, a slip wall on a viscous problem,
 *   or an invalid face_orient entry); 0 when neither was seen since the last sbp_status call.
 * Returns SBP_ERR_NONPHYSICAL if bit 0 is set, else SBP_ERR_MESH if bit 1 is set, else SBP_OK;
 * SBP_ERR_ARG for a null ws or flags, SBP_ERR_HIP if the wait or the copy fails. */
int sbp_status(void *ws, void *stream, int32_t *flags);

/* Releases what the library caches for calls made with workspace `ws`: the launch plans (small
 * device tables of the problem groups, made on the first call of a problem set) and the recorded
 * RK4 graphs.  Call it before the workspace is freed or reused for another problem set; later calls
 * with `ws` make new plans.  Waits for the whole device first (no cached plan or graph may be in
 * use).  Returns the number of plans and graphs released (>= 0), SBP_ERR_ARG for a null ws or
 * SBP_ERR_HIP if the wait fails. */
int sbp_release(void *ws);

#ifdef __cplusplus
}
#endif

#endif /* SBP_H */
