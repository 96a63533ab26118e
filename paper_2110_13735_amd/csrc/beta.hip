// Kernel-mode tables (Lemma of section 'Fast spectral approximation of the BNE operator', polar forms of section 'Expansion of the kernel modes').
//
// beta(k,l) = int_{B(0,R)^2} Btilde(z,y) delta(z.y) e^{i(z.k + y.l)} dz dy is
// evaluated through the expansion of both plane waves in angular harmonics
// (Jacobi–Anger in 2-D, Funk–Hecke / Rayleigh in 3-D).  The great-circle
// constraint delta(e.e') keeps even orders only and couples equal orders:
//
//   d = 3, Btilde = 4 C:  beta = 32 pi^2 C sum_{n even} (2n+1) P_n(0)
//                                 P_n(cos g) J_n(|k|) J_n(|l|),
//                         J_n(s) = int_0^R r j_n(r s) dr   (spherical j_n)
//   d = 2, Btilde = 2 C:  beta = 8 pi C sum_{n even} eps_n (-1)^{n/2}
//                                 cos(n g) A_n(|k|) A_n(|l|),
//                         A_n(s) = int_0^R J_n(r s) dr     (cylindrical J_n)
//
// with g the angle between k and l (eps_0 = 1, eps_n = 2).  This is a
// different route from the paper's rectangle rules (eqs. beta2D, beta3D):
// the angular integrals are done exactly, the radial ones by Gauss–Legendre
// quadrature of Bessel values from Miller's backward recurrence.  Only |k|^2,
// |l|^2 and |k.l| enter, so the table is exactly invariant under signed axis
// permutations and even in each argument.
#include "bnq_internal.h"

namespace bnq {

// Bessel values at x for even orders 0, 2, ..., 2(M-1), times `w`, written to
// out[m * stride].  sph = 1: spherical j_n, normalised by sum (2n+1) j_n^2 = 1;
// sph = 0: cylindrical J_n, normalised by J_0 + 2 sum J_{2k} = 1.
__device__ static void even_bessel(int sph, double x, int M, double w, double *out, int stride) {
    for (int m = 0; m < M; ++m) out[m * stride] = 0.0;
    if (x == 0.0) {
        out[0] = w;
        return;
    }
    if (x < 1e-3) {
        // leading two terms of the power series
        double t = 1.0;  // x^n / (2n+1)!!  or  (x/2)^n / n!
        for (int n = 0; n < 2 * M; ++n) {
            if (n > 0) t *= sph ? x / (2.0 * n + 1.0) : 0.5 * x / n;
            if (t < 1e-300) break;
            if ((n & 1) == 0) {
                double corr = sph ? 1.0 - x * x / (2.0 * (2.0 * n + 3.0)) : 1.0 - 0.25 * x * x / (n + 1.0);
                out[(n / 2) * stride] = w * t * corr;
            }
        }
        return;
    }
    // start index well above the turning point; with seed 1e-60 the values
    // stay inside the double range for every x >= 1e-3 used here
    int nstart = (int)ceil(x + 15.0 * cbrt(x) + 30.0);
    double yp1 = 0.0, y = 1e-60, S = 0.0, y1 = 0.0;
    for (int n = nstart; n >= 0; --n) {
        if (sph) {
            S += (2.0 * n + 1.0) * y * y;
        } else if ((n & 1) == 0) {
            S += (n == 0 ? 1.0 : 2.0) * y;
        }
        if ((n & 1) == 0 && n / 2 < M) out[(n / 2) * stride] = y;
        if (n == 1) y1 = y;
        double ym1 = (sph ? (2.0 * n + 1.0) : (2.0 * n)) / x * y - yp1;
        yp1 = y;
        y = ym1;
    }
    double scale;
    if (sph) {
        // y now holds y_{-1}; out[0] is y_0
        double j0 = sin(x) / x, j1 = sin(x) / (x * x) - cos(x) / x;
        double sg = fabs(j0) >= fabs(j1) ? copysign(1.0, j0) * copysign(1.0, out[0])
                                         : copysign(1.0, j1) * copysign(1.0, y1);
        scale = sg / sqrt(S);
    } else {
        scale = 1.0 / S;
    }
    for (int m = 0; m < M; ++m) out[m * stride] *= scale * w;
}

// Stage 1: one block per q = |a|^2, one thread per Gauss–Legendre node on
// [0, R]; weighted Bessel values go to scratch S[q][m][node].
__global__ void radial_nodes_kernel(int d, double R, int M, int nq, const double *glx, const double *glw,
                                    double *S) {
    const int q = blockIdx.x;
    const int t = threadIdx.x;
    if (t >= nq) return;
    const double s = sqrt((double)q);
    const double rho = 0.5 * R * (glx[t] + 1.0);
    const double w = 0.5 * R * glw[t] * (d == 3 ? rho : 1.0);
    even_bessel(d == 3, rho * s, M, w, S + (int64_t)q * M * nq + t, nq);
}

// Stage 2: J[q][m] = sum over nodes in a fixed order.
__global__ void radial_sum_kernel(int qmax, int M, int nq, const double *S, double *J) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(qmax + 1) * M) return;
    const double *row = S + i * nq;
    double acc = 0.0;
    for (int k = 0; k < nq; ++k) acc += row[k];
    J[i] = acc;
}

void launch_radial(int d, double R, int qmax, int M, int nq, const double *glx, const double *glw,
                   double *S, double *J, hipStream_t s) {
    hipLaunchKernelGGL(radial_nodes_kernel, dim3(qmax + 1), dim3(nq), 0, s, d, R, M, nq, glx, glw, S);
    const int64_t n = (int64_t)(qmax + 1) * M;
    hipLaunchKernelGGL(radial_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, qmax, M, nq, S, J);
}

// K[kc][a] = beta(a, b_c[kc]) for a in A, stored as [a0][a2 (padded)][a1]
// (FP64: idx_K, read by the vector-unit kernel) or [a0][a1][a2 (padded)]
// (FP32: idx_Kx, read by the matrix-core kernel); the x padding holds zeros.
// Every value is formed in FP64; an FP32 table holds it rounded to nearest.
template <typename T>
__global__ void beta_rows_kernel(Geo g, Radial rad, const int *canon, T *K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int kc = blockIdx.y;
    if (i >= g.nak) return;
    const int A = 2 * g.N - 1;
    int a0, a1, a2;
    if constexpr (sizeof(T) == 8) {
        a1 = (int)(i % A) - (g.N - 1);
        a2 = (int)((i / A) % g.kax) - (g.N - 1) - KPADLO;
        a0 = g.d == 3 ? (int)(i / ((int64_t)A * g.kax)) - (g.N - 1) : 0;
    } else {
        a2 = (int)(i % g.kax) - (g.N - 1) - KPADLO;
        a1 = (int)((i / g.kax) % A) - (g.N - 1);
        a0 = g.d == 3 ? (int)(i / ((int64_t)A * g.kax)) - (g.N - 1) : 0;
    }
    double v = 0.0;
    if (a2 >= -(g.N - 1) && a2 <= g.N - 1) {
        const int b0 = canon[3 * kc], b1 = canon[3 * kc + 1], b2 = canon[3 * kc + 2];
        const int qa = a0 * a0 + a1 * a1 + a2 * a2;
        const int qb = b0 * b0 + b1 * b1 + b2 * b2;
        const int dab = abs(a0 * b0 + a1 * b1 + a2 * b2);
        v = beta_series(rad, qa, qb, (double)dab);
    }
    K[(int64_t)kc * g.nak + i] = (T)v;
}

void launch_beta_rows(const Geo &g, const Radial &rad, const int *canon, int ncanon, double *K, hipStream_t s) {
    dim3 grid((unsigned)((g.nak + 255) / 256), (unsigned)ncanon);
    hipLaunchKernelGGL(beta_rows_kernel<double>, grid, dim3(256), 0, s, g, rad, canon, K);
}

void launch_beta_rows(const Geo &g, const Radial &rad, const int *canon, int ncanon, float *K, hipStream_t s) {
    dim3 grid((unsigned)((g.nak + 255) / 256), (unsigned)ncanon);
    hipLaunchKernelGGL(beta_rows_kernel<float>, grid, dim3(256), 0, s, g, rad, canon, K);
}

// beta(a, a) for |a|^2 = q, q = 0 .. qmax
__global__ void beta_diag_kernel(Radial rad, int qmax, double *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q <= qmax) out[q] = beta_series(rad, q, q, (double)q);
}

void launch_beta_diag(const Radial &rad, int qmax, double *out, hipStream_t s) {
    hipLaunchKernelGGL(beta_diag_kernel, dim3((unsigned)((qmax + 256) / 256)), dim3(256), 0, s, rad, qmax, out);
}

__device__ static inline void mode_of(const Geo &g, int64_t i, int &k0, int &k1, int &k2) {
    k2 = (int)(i % g.N) - g.h;
    k1 = (int)((i / g.N) % g.N) - g.h;
    k0 = g.d == 3 ? (int)(i / ((int64_t)g.N * g.N)) - g.h : 0;
}

// Pair weights on I_N x I_N, [l][m] order:
//   wc = beta(l,m) - beta(m,m)                      (only where l+m in I_N; 0 elsewhere)
//   wq = beta(l,m) - beta(l+m,l) - beta(l,l+m)
template <typename T>
__global__ void weights_kernel(Geo g, Radial rad, T *wc, T *wq) {
    const int64_t im = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t il = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
    if (im >= g.nm || il >= g.nm) return;
    int l0, l1, l2, m0, m1, m2;
    mode_of(g, il, l0, l1, l2);
    mode_of(g, im, m0, m1, m2);
    double c, q;
    pair_weights(rad, g, l0, l1, l2, m0, m1, m2, c, q);
    const int64_t o = il * g.nm + im;
    wc[o] = (T)c;
    wq[o] = (T)q;
}

template <typename T>
static void launch_weights_t(const Geo &g, const Radial &rad, T *wc, T *wq, hipStream_t s) {
    unsigned gy = (unsigned)(g.nm < 65535 ? g.nm : 32768);
    unsigned gz = (unsigned)((g.nm + gy - 1) / gy);
    dim3 grid((unsigned)((g.nm + 255) / 256), gy, gz);
    hipLaunchKernelGGL(weights_kernel<T>, grid, dim3(256), 0, s, g, rad, wc, wq);
}

void launch_weights(const Geo &g, const Radial &rad, double *wc, double *wq, hipStream_t s) {
    launch_weights_t(g, rad, wc, wq, s);
}

void launch_weights(const Geo &g, const Radial &rad, float *wc, float *wq, hipStream_t s) {
    launch_weights_t(g, rad, wc, wq, s);
}

// Pair weights at n index pairs (l, m) (flattened I_N indices): which = 1
// gives wc, 2 gives wq; for table sets that hold no weight tables.
__global__ void pair_weights_at_kernel(Geo g, Radial rad, const int64_t *idx, int64_t n, int which, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int l0, l1, l2, m0, m1, m2;
    mode_of(g, idx[i] / g.nm, l0, l1, l2);
    mode_of(g, idx[i] % g.nm, m0, m1, m2);
    double c, q;
    pair_weights(rad, g, l0, l1, l2, m0, m1, m2, c, q);
    out[i] = which == 1 ? c : q;
}

void launch_pair_weights_at(const Geo &g, const Radial &rad, const int64_t *idx, int64_t n, int which, double *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(pair_weights_at_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rad, idx, n,
                       which, out);
}

template <typename T>
__global__ void gather_kernel(const T *base, const int64_t *idx, int64_t n, double *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)base[idx[i]];
}

void launch_gather(const double *base, const int64_t *idx, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, base, idx, n, out);
}

void launch_gather(const float *base, const int64_t *idx, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, base, idx, n, out);
}

}  // namespace bnq
