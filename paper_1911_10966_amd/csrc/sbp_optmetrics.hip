// Optimised metric terms on gfx950 (metric-terms paragraph after eq. discGCLconvection: analytic
// surface metrics, volume metrics as close as possible to the analytic ones under the discrete
// GCL), for aligned conforming meshes.
//
// Notation: element arrays hold node i1 + N i2 + N^2 i3; for a fixed physical direction m the
// unknowns of an element are a_l = A_lm (l = 1..3), the GCL is M a = sum_l D_l a_l = 0, and the
// entries of a_l on the two faces normal to xi_l (the face-normal values) are "held".
//
// 1. Analytic metrics A_l = a_{l+1} x a_{l+2} from the covariant vectors a_i = dx/dxi_i, and
//    J = a_1 . (a_2 x a_3).
// 2. Surface step.  With the held values fixed, M a = 0 is solvable for the other entries only if
//    y^T M a = 0 for every y in the left null space of M on the other entries.  That space is
//    spanned by the tensor products of the 1-D vectors w (the LGL weights, D^T w = e_p - e_0) and z
//    (the left null vector of D), so with f_l,+ and f_l,- the values on the faces normal to xi_l the
//    conditions read, for k = (k_1, k_2, k_3) in {z, w}^3,
//        sum over l with k_l = w of <t_{k,l}, f_l,+ - f_l,->  = 0,
//    t_{k,l} the tensor product of the two other factors on the face (k = zzz is void).  Each face
//    node carries one value, the mean of the analytic values of its two elements, plus the
//    least-norm correction x = -G^T y over all face nodes of the mesh, where G stacks every
//    element's 7 conditions and (G G^T) y = G f.  G G^T couples an element to its face neighbours
//    through the 4x4 Gram matrices of the face patterns; it is solved by conjugate gradients with
//    deterministic reductions.  G f is summed per element without rounding error beyond the
//    result's own (compensated summation), so that it stays in the range of G: each face moment
//    enters two elements with opposite signs and the same value.
// 3. Volume step, per element and m: the other entries move by -M_f^T (M_f M_f^T)^+ M a, the
//    least-norm change that satisfies the GCL.  M_f M_f^T = B (+) B (+) B (a Kronecker sum) with
//    B = D diag(0, 1, ..., 1, 0) D^T, so its pseudo-inverse is applied in the tensor eigenbasis of
//    B: three 1-D transforms, a division by lambda_i + lambda_j + lambda_k (zero on the 8 null
//    combinations), three inverse transforms.
#include <hip/hip_runtime.h>

#include <vector>

#include "sbp_internal.h"

namespace sbp {
namespace {

constexpr int kThreads = 256;
constexpr int kConds = 7;      // conditions k = 1..7; bit l of k set: factor w along xi_l, else z
constexpr int kMaxIter = 20000;
constexpr int kCheckEvery = 16;
constexpr double kTol2 = 1e-24;  // squared relative residual of the compatibility system

// Scalars of the conjugate-gradient iteration, per component m (offsets into the scalar block).
enum { S_RR = 0, S_PAP = 3, S_ALPHA = 6, S_BETA = 9, S_TOL2 = 12, S_DONE = 15, S_COUNT = 18 };

struct Pats {
    double pat[2][16];
    double gram[2][2];
    int N;
};

// Node index of face (l, side) at tangential position (ta, tb): ta runs along the lower of the two
// other directions, tb along the higher one.
__device__ __forceinline__ int face_node(int N, int l, int side, int ta, int tb) {
    const int il = side ? N - 1 : 0;
    if (l == 0) return il + N * (ta + N * tb);
    if (l == 1) return ta + N * (il + N * tb);
    return ta + N * (tb + N * il);
}

__device__ __forceinline__ int lower_other(int l) { return l == 0 ? 1 : 0; }
__device__ __forceinline__ int upper_other(int l) { return l == 2 ? 1 : 2; }

__device__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kThreads)
k_om_analytic(const double *F, double *metric, double *jac, long long nodes) {
    const long long n = blockIdx.x * (long long)kThreads + threadIdx.x;
    if (n >= nodes) return;
    double a[3][3];  // a[i][m] = dx_m/dxi_i, input entry 3 m + i
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int i = 0; i < 3; ++i) a[i][m] = F[(3 * m + i) * nodes + n];
    double J = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const double *u = a[(l + 1) % 3], *v = a[(l + 2) % 3];
        const double c0 = u[1] * v[2] - u[2] * v[1];
        const double c1 = u[2] * v[0] - u[0] * v[2];
        const double c2 = u[0] * v[1] - u[1] * v[0];
        metric[(3 * l + 0) * nodes + n] = c0;
        metric[(3 * l + 1) * nodes + n] = c1;
        metric[(3 * l + 2) * nodes + n] = c2;
        if (l == 0) J = a[0][0] * c0 + a[0][1] * c1 + a[0][2] * c2;
    }
    jac[n] = J;
}

// Face-normal values, one per face node: the mean of the two elements' values (own value on a
// boundary face).  fb[((e * 6 + f) * 3 + m) * N^2 + ta + N tb].
__global__ void __launch_bounds__(kThreads)
k_om_faces(const double *metric, const int32_t *nbr, double *fb, long long K, int N) {
    const int N2 = N * N, N3 = N2 * N;
    const long long idx = blockIdx.x * (long long)kThreads + threadIdx.x;
    if (idx >= K * 18 * N2) return;
    const int t = (int)(idx % N2);
    long long r = idx / N2;
    const int m = (int)(r % 3);
    r /= 3;
    const int f = (int)(r % 6);
    const long long e = r / 6;
    const int l = f >> 1, side = f & 1, ta = t % N, tb = t / N;
    const double *A = metric + (3 * l + m) * (K * N3);
    double v = A[e * N3 + face_node(N, l, side, ta, tb)];
    const int nb = nbr[e * 6 + f];
    if (nb >= 0) v = (v + A[(long long)nb * N3 + face_node(N, l, side ^ 1, ta, tb)]) * 0.5;
    fb[idx] = v;
}

// <t_{k,l}, face>: the face values weighted by the patterns of k along the two other directions.
__device__ double face_moment(const double *face, const Pats &P, int k, int l) {
    const int N = P.N;
    const double *s = P.pat[(k >> lower_other(l)) & 1];
    const double *t = P.pat[(k >> upper_other(l)) & 1];
    double acc = 0.0;
    for (int tb = 0; tb < N; ++tb) {
        double row = 0.0;
        for (int ta = 0; ta < N; ++ta) row += s[ta] * face[ta + N * tb];
        acc += t[tb] * row;
    }
    return acc;
}

// b = G f per element, condition and m (compensated sum of the face moments), which starts the
// iteration: r = p = b, y = 0; block partial sums of b.b.
__global__ void __launch_bounds__(kThreads)
k_om_rhs(const double *fb, Pats P, double *y, double *r, double *pd, double *part, long long K) {
    __shared__ double red[kThreads];
    const int N2 = P.N * P.N;
    const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
    const int c = blockIdx.y, m = c / kConds, k = c % kConds + 1;
    double val = 0.0;
    if (e < K) {
        double s = 0.0, comp = 0.0;  // Neumaier summation
        for (int l = 0; l < 3; ++l) {
            if (!((k >> l) & 1)) continue;
            for (int side = 1; side >= 0; --side) {
                const double mom = face_moment(fb + ((e * 6 + 2 * l + side) * 3 + m) * N2, P, k, l);
                const double term = side ? mom : -mom;
                const double tsum = s + term;
                comp += (fabs(s) >= fabs(term)) ? (s - tsum) + term : (term - tsum) + s;
                s = tsum;
            }
        }
        val = s + comp;
        const long long i = (long long)c * K + e;
        y[i] = 0.0;
        r[i] = val;
        pd[i] = val;
    }
    const double sum = block_sum(val * val, red);
    if (threadIdx.x == 0) part[(long long)c * gridDim.x + blockIdx.x] = sum;
}

// Ap = (G G^T) p: per element, condition k and m,
//   sum over l with k_l = w, over both faces normal to xi_l, over k' with k'_l = w of
//   gram(k, k' on the face) (p_e,k' - p_neighbour,k')   (no neighbour term on a boundary face).
__global__ void __launch_bounds__(kThreads)
k_om_apply(const double *pd, const int32_t *nbr, Pats P, double *Ap, double *part, long long K) {
    __shared__ double red[kThreads];
    const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
    const int c = blockIdx.y, m = c / kConds, k = c % kConds + 1;
    double acc = 0.0, own = 0.0;
    if (e < K) {
        for (int l = 0; l < 3; ++l) {
            if (!((k >> l) & 1)) continue;
            const int l1 = lower_other(l), l2 = upper_other(l);
            for (int side = 0; side < 2; ++side) {
                const int nb = nbr[e * 6 + 2 * l + side];
                for (int k2 = 1; k2 <= kConds; ++k2) {
                    if (!((k2 >> l) & 1)) continue;
                    const double g = P.gram[(k >> l1) & 1][(k2 >> l1) & 1] *
                                     P.gram[(k >> l2) & 1][(k2 >> l2) & 1];
                    const long long base = (long long)(m * kConds + k2 - 1) * K;
                    const double d = pd[base + e] - (nb >= 0 ? pd[base + nb] : 0.0);
                    acc += g * d;
                }
            }
        }
        Ap[(long long)c * K + e] = acc;
        own = pd[(long long)c * K + e];
    }
    const double sum = block_sum(own * acc, red);
    if (threadIdx.x == 0) part[(long long)c * gridDim.x + blockIdx.x] = sum;
}

// Per m, the sum of the block partials of its 7 conditions, in a fixed order.
__device__ double reduce_m(const double *part, int nbx, int m, double *red) {
    double v = 0.0;
    const int n = kConds * nbx;
    for (int i = threadIdx.x; i < n; i += kThreads) v += part[(long long)m * n + i];
    return block_sum(v, red);
}

// First reduction: rr = b.b, the stopping threshold, and a component with b = 0 is done at once.
__global__ void __launch_bounds__(kThreads) k_om_start(const double *part, int nbx, double *sc) {
    __shared__ double red[kThreads];
    for (int m = 0; m < 3; ++m) {
        const double rr = reduce_m(part, nbx, m, red);
        if (threadIdx.x == 0) {
            sc[S_RR + m] = rr;
            sc[S_TOL2 + m] = kTol2 * rr;
            sc[S_DONE + m] = (rr > 0.0) ? 0.0 : 1.0;
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_om_alpha(const double *part, int nbx, double *sc) {
    __shared__ double red[kThreads];
    for (int m = 0; m < 3; ++m) {
        const double pap = reduce_m(part, nbx, m, red);
        if (threadIdx.x == 0) {
            sc[S_PAP + m] = pap;
            sc[S_ALPHA + m] = (sc[S_DONE + m] != 0.0 || !(pap > 0.0)) ? 0.0 : sc[S_RR + m] / pap;
        }
    }
}

// y += alpha p, r -= alpha Ap; block partials of r.r.
__global__ void __launch_bounds__(kThreads)
k_om_update(double *y, double *r, const double *pd, const double *Ap, const double *sc, double *part,
            long long K) {
    __shared__ double red[kThreads];
    const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
    const int c = blockIdx.y, m = c / kConds;
    const double alpha = sc[S_ALPHA + m];
    double rv = 0.0;
    if (e < K) {
        const long long i = (long long)c * K + e;
        y[i] += alpha * pd[i];
        rv = r[i] - alpha * Ap[i];
        r[i] = rv;
    }
    const double sum = block_sum(rv * rv, red);
    if (threadIdx.x == 0) part[(long long)c * gridDim.x + blockIdx.x] = sum;
}

// rr_new, beta = rr_new / rr; a component whose residual has reached its threshold is frozen
// (alpha = 0 from then on), so that later rounding cannot move its solution.
__global__ void __launch_bounds__(kThreads) k_om_beta(const double *part, int nbx, double *sc) {
    __shared__ double red[kThreads];
    for (int m = 0; m < 3; ++m) {
        const double rrn = reduce_m(part, nbx, m, red);
        if (threadIdx.x == 0) {
            if (sc[S_DONE + m] != 0.0) {
                sc[S_BETA + m] = 0.0;
            } else {
                const double rr = sc[S_RR + m];
                sc[S_BETA + m] = rr > 0.0 ? rrn / rr : 0.0;
                sc[S_RR + m] = rrn;
                if (rrn <= sc[S_TOL2 + m]) sc[S_DONE + m] = 1.0;
            }
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_om_direction(double *pd, const double *r, const double *sc, long long K) {
    const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
    const int c = blockIdx.y, m = c / kConds;
    if (e >= K) return;
    const long long i = (long long)c * K + e;
    pd[i] = r[i] + sc[S_BETA + m] * pd[i];
}

// Held entries = face mean + correction, x = -(G^T y) at the face node:
//   -sum over k with k_l = w of t_{k,l}(ta, tb) (y_minus - y_plus),
// y_minus the multiplier of the element whose + face this is and y_plus that of the element
// whose - face it is (zero where there is none).  Both elements of a face compute the same
// operands in the same order, so they store the same value.
__global__ void __launch_bounds__(kThreads)
k_om_held(const double *fb, const double *y, const int32_t *nbr, Pats P, double *metric,
          long long K) {
    const int N = P.N, N2 = N * N, N3 = N2 * N;
    const long long idx = blockIdx.x * (long long)kThreads + threadIdx.x;
    if (idx >= K * 18 * N2) return;
    const int t = (int)(idx % N2);
    long long rr = idx / N2;
    const int m = (int)(rr % 3);
    rr /= 3;
    const int f = (int)(rr % 6);
    const long long e = rr / 6;
    const int l = f >> 1, side = f & 1, ta = t % N, tb = t / N;
    const int l1 = lower_other(l), l2 = upper_other(l);
    const int nb = nbr[e * 6 + f];
    double x = 0.0;
    for (int k = 1; k <= kConds; ++k) {
        if (!((k >> l) & 1)) continue;
        const long long base = (long long)(m * kConds + k - 1) * K;
        const long long emin = side ? e : (long long)nb, eplus = side ? (long long)nb : e;
        const double ym = (emin >= 0) ? y[base + emin] : 0.0;
        const double yp = (eplus >= 0) ? y[base + eplus] : 0.0;
        const double w = P.pat[(k >> l1) & 1][ta] * P.pat[(k >> l2) & 1][tb];
        x -= w * (ym - yp);
    }
    metric[(3 * l + m) * (K * N3) + e * N3 + face_node(N, l, side, ta, tb)] = fb[idx] + x;
}

// One 1-D transform along direction ax of an element array in LDS: dst = (I (x) M (x) I) src with
// M(i, j) = mat[i * ri + j * rj].
__device__ void line_transform(const double *src, double *dst, const double *mat, int ri, int rj,
                               int ax, int N) {
    const int N3 = N * N * N;
    const int stride = ax == 0 ? 1 : (ax == 1 ? N : N * N);
    for (int n = threadIdx.x; n < N3; n += kThreads) {
        const int i = (n / stride) % N;
        const int b = n - i * stride;
        double acc = 0.0;
        for (int j = 0; j < N; ++j) acc += mat[i * ri + j * rj] * src[b + j * stride];
        dst[n] = acc;
    }
}

// Volume step for element blockIdx.x and component m = blockIdx.y.  tab: D[256], V[256], lam[16],
// then the null mask as a double.
__global__ void __launch_bounds__(kThreads)
k_om_volume(double *metric, const double *tab, long long K, int N) {
    extern __shared__ double sm[];
    const int N2 = N * N, N3 = N2 * N;
    double *b0 = sm, *b1 = sm + N3;
    const double *D = tab, *V = tab + 256, *lam = tab + 512;
    const int null_mask = (int)tab[528];
    const long long e = blockIdx.x, nodes = K * N3;
    const int m = blockIdx.y;
    double *a[3];
    for (int l = 0; l < 3; ++l) a[l] = metric + (3 * l + m) * nodes + e * N3;
    // r = -M a
    for (int n = threadIdx.x; n < N3; n += kThreads) {
        const int i1 = n % N, i2 = (n / N) % N, i3 = n / N2;
        double acc = 0.0;
        for (int j = 0; j < N; ++j) acc += D[i1 * N + j] * a[0][j + N * i2 + N2 * i3];
        for (int j = 0; j < N; ++j) acc += D[i2 * N + j] * a[1][i1 + N * j + N2 * i3];
        for (int j = 0; j < N; ++j) acc += D[i3 * N + j] * a[2][i1 + N * i2 + N2 * j];
        b0[n] = -acc;
    }
    __syncthreads();
    // into the eigenbasis: (V^T (x) V^T (x) V^T) r
    line_transform(b0, b1, V, 1, N, 0, N);
    __syncthreads();
    line_transform(b1, b0, V, 1, N, 1, N);
    __syncthreads();
    line_transform(b0, b1, V, 1, N, 2, N);
    __syncthreads();
    for (int n = threadIdx.x; n < N3; n += kThreads) {
        const int i1 = n % N, i2 = (n / N) % N, i3 = n / N2;
        const bool all_null = ((null_mask >> i1) & 1) && ((null_mask >> i2) & 1) && ((null_mask >> i3) & 1);
        b1[n] = all_null ? 0.0 : b1[n] / (lam[i1] + lam[i2] + lam[i3]);
    }
    __syncthreads();
    // back: (V (x) V (x) V)
    line_transform(b1, b0, V, N, 1, 0, N);
    __syncthreads();
    line_transform(b0, b1, V, N, 1, 1, N);
    __syncthreads();
    line_transform(b1, b0, V, N, 1, 2, N);
    __syncthreads();
    // a_l += D_l^T y on the entries off the faces normal to xi_l
    for (int n = threadIdx.x; n < N3; n += kThreads) {
        const int i1 = n % N, i2 = (n / N) % N, i3 = n / N2;
        if (i1 > 0 && i1 < N - 1) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += D[j * N + i1] * b0[j + N * i2 + N2 * i3];
            a[0][n] += acc;
        }
        if (i2 > 0 && i2 < N - 1) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += D[j * N + i2] * b0[i1 + N * j + N2 * i3];
            a[1][n] += acc;
        }
        if (i3 > 0 && i3 < N - 1) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += D[j * N + i3] * b0[i1 + N * i2 + N2 * j];
            a[2][n] += acc;
        }
    }
}

unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

int optimized_metrics(const OptMetricTables &t, long long K, const int32_t *nbr,
                      const double *dxdxi, double *metric, double *jac, hipStream_t s) {
    const int N = t.p + 1, N2 = N * N, N3 = N2 * N;
    const long long nodes = K * N3;
    const unsigned nbx = blocks_for(K);
    const long long n_fb = K * 18 * N2, n_vec = (long long)3 * kConds * K;
    const long long n_part = (long long)3 * kConds * nbx;
    const long long n_tab = 544;
    const long long total = n_fb + 4 * n_vec + n_part + 32 + n_tab;
    double *buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * total) != hipSuccess) return 1;
    double *fb = buf, *y = fb + n_fb, *r = y + n_vec, *pd = r + n_vec, *Ap = pd + n_vec;
    double *part = Ap + n_vec, *sc = part + n_part, *tab = sc + 32;

    std::vector<double> htab(n_tab, 0.0);
    for (int i = 0; i < N * N; ++i) { htab[i] = t.D[i]; htab[256 + i] = t.V[i]; }
    for (int i = 0; i < N; ++i) htab[512 + i] = t.lam[i];
    htab[528] = (double)t.null_mask;
    Pats P{};
    P.N = N;
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < N; ++i) P.pat[a][i] = t.pat[a][i];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double g = 0.0;
            for (int i = 0; i < N; ++i) g += t.pat[a][i] * t.pat[b][i];
            P.gram[a][b] = g;
        }

    int rc = 0;
    bool converged = false;
    double done[3] = {0.0, 0.0, 0.0};
    const dim3 gv(nbx, 3 * kConds);
    if (hipMemcpyAsync(tab, htab.data(), sizeof(double) * n_tab, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        rc = 1;
        goto out;
    }
    hipLaunchKernelGGL(k_om_analytic, dim3(blocks_for(nodes)), dim3(kThreads), 0, s, dxdxi, metric,
                       jac, nodes);
    hipLaunchKernelGGL(k_om_faces, dim3(blocks_for(n_fb)), dim3(kThreads), 0, s, metric, nbr, fb, K, N);
    hipLaunchKernelGGL(k_om_rhs, gv, dim3(kThreads), 0, s, fb, P, y, r, pd, part, K);
    hipLaunchKernelGGL(k_om_start, dim3(1), dim3(kThreads), 0, s, part, (int)nbx, sc);
    if (hipGetLastError() != hipSuccess) { rc = 1; goto out; }
    for (int it = 0; it < kMaxIter; ++it) {
        if (it % kCheckEvery == 0) {
            if (hipMemcpyAsync(done, sc + S_DONE, sizeof(done), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = 1;
                goto out;
            }
            if (done[0] != 0.0 && done[1] != 0.0 && done[2] != 0.0) { converged = true; break; }
        }
        hipLaunchKernelGGL(k_om_apply, gv, dim3(kThreads), 0, s, pd, nbr, P, Ap, part, K);
        hipLaunchKernelGGL(k_om_alpha, dim3(1), dim3(kThreads), 0, s, part, (int)nbx, sc);
        hipLaunchKernelGGL(k_om_update, gv, dim3(kThreads), 0, s, y, r, pd, Ap, sc, part, K);
        hipLaunchKernelGGL(k_om_beta, dim3(1), dim3(kThreads), 0, s, part, (int)nbx, sc);
        hipLaunchKernelGGL(k_om_direction, gv, dim3(kThreads), 0, s, pd, r, sc, K);
        if (hipGetLastError() != hipSuccess) { rc = 1; goto out; }
    }
    if (!converged) {
        if (hipMemcpyAsync(done, sc + S_DONE, sizeof(done), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = 1;
            goto out;
        }
        converged = done[0] != 0.0 && done[1] != 0.0 && done[2] != 0.0;
    }
    if (!converged) { rc = 2; goto out; }
    hipLaunchKernelGGL(k_om_held, dim3(blocks_for(n_fb)), dim3(kThreads), 0, s, fb, y, nbr, P, metric, K);
    hipLaunchKernelGGL(k_om_volume, dim3((unsigned)K, 3), dim3(kThreads), 2 * N3 * sizeof(double), s,
                       metric, tab, K, N);
    if (hipGetLastError() != hipSuccess) rc = 1;
out:
    if (hipStreamSynchronize(s) != hipSuccess) rc = 1;
    (void)hipFree(buf);  // nothing left to report after a failure
    return rc;
}

}  // namespace sbp
