// Trilinear term by the separated-kernel transform route, d = 2 (section
// 'Fast computation of the collision modes', eqs. betadD and alphap; appendix
// 'Fast evaluation of the collision kernel').
//
// With the kernel modes written as the rank-P sum
//   beta(a, b) = C sum_p alpha_p(a) alpha'_p(b),   C = pi / P,  theta_p = p pi / P,
//   alpha_p(a) = 2 C_phi phi(a . e_p),  alpha'_p(b) = phi(b . e_p^perp),  phi(s) = 2 sin(R s) / s,
// the trilinear sum T1_n = sum_{a,b} beta(a,b) G_{n-a} G_{n-b} G_{a+b-n} is
//   T1_n = C M^-6 sum_p sum_{j in [0,M)^2} Gt_j e^{2 pi i n.j/M} A_pj(n) B_pj(n),
//   A_pj(n) = sum_x gc_p(x - j) Gt_x e^{-2 pi i n.x/M},  B_pj likewise with gc'_p,
// on the doubled grid M = 2N:
//   Gt_x   = sum_{k in I_N} G_k e^{2 pi i k.x/M}            (spectrum extended by zeros),
//   gc_p(y) = sum_{a in (-N,N)^2} alpha_p(a) cos(2 pi a.y/M)  (real: alpha_p is even).
// On the doubled grid every index sum that occurs (a + k with a in (-N,N),
// k in I_N; a + b - n) stays clear of the period, so this is the linear
// Galerkin sum, equal to the direct one for the same kernel modes.
//
// Work: every (p, j) needs two M x M -> N x N transforms, done as DFTs by
// matrix along each axis: 6 N^3 complex multiply-adds, P (2N)^2 times.  At
// N = 32 that is about 1.3e12 flops per evaluation against 4.8e9 for the
// direct trilinear sum: the route is kept for what it computes, not for speed.
#include "bnq_internal.h"

namespace bnq {

namespace {

__device__ double sep_phi(double R, double s) {
    const double x = R * s;
    if (fabs(x) < 1e-3) {
        const double x2 = x * x;
        return 2.0 * R * (1.0 - x2 / 6.0 * (1.0 - x2 / 20.0));
    }
    return 2.0 * sin(x) / s;
}

// nonnegative residue of v modulo m
__device__ __forceinline__ int pmod(int v, int m) {
    const int r = v % m;
    return r < 0 ? r + m : r;
}

// al[p][a], alp[p][a] for a in (-N, N)^2 in row-major order
__global__ void sep_alpha_kernel(int N, int P, double R, double Cphi, double *al, double *alp) {
    const int w = 2 * N - 1, na = w * w;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (i >= na) return;
    const double a0 = (double)(i / w - (N - 1)), a1 = (double)(i % w - (N - 1));
    double sn, cs;
    sincospi((double)p / P, &sn, &cs);
    al[(int64_t)p * na + i] = 2.0 * Cphi * sep_phi(R, a0 * cs + a1 * sn);
    alp[(int64_t)p * na + i] = sep_phi(R, -a0 * sn + a1 * cs);
}

// gc[p][y] = (gc_p(y), gc'_p(y)), y in [0, M)^2 row-major; the angle's alpha
// rows and the cosine table in LDS
__global__ void sep_gc_kernel(int N, int M, const double *al, const double *alp, double2 *gc) {
    extern __shared__ double sh[];
    const int w = 2 * N - 1, na = w * w;
    double *sa = sh, *sb = sh + na, *cs = sh + 2 * na;
    const int p = blockIdx.y;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        sa[i] = al[(int64_t)p * na + i];
        sb[i] = alp[(int64_t)p * na + i];
    }
    for (int t = threadIdx.x; t < M; t += blockDim.x) cs[t] = cospi(2.0 * t / M);
    __syncthreads();
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= M * M) return;
    const int y0 = y / M, y1 = y % M;
    double ga = 0.0, gb = 0.0;
    for (int i0 = 0; i0 < w; ++i0) {
        // t = (a0 y0 + a1 y1) mod M along the row a0 = i0 - (N - 1)
        int t = pmod((i0 - (N - 1)) * y0 - (N - 1) * y1, M);
        const double *ra = sa + i0 * w, *rb = sb + i0 * w;
        for (int i1 = 0; i1 < w; ++i1) {
            const double c = cs[t];
            ga += ra[i1] * c;
            gb += rb[i1] * c;
            t += y1;
            if (t >= M) t -= M;
        }
    }
    gc[(int64_t)p * M * M + y] = make_double2(ga, gb);
}

// Gt[x] = sum_{k in I_N} G_k e^{2 pi i k.x/M}, x in [0, M)^2 row-major
__global__ void sep_gt_kernel(int N, int M, const double2 *__restrict__ G, double2 *gt) {
    extern __shared__ double2 tw[];  // e^{2 pi i t/M}
    for (int t = threadIdx.x; t < M; t += blockDim.x) {
        double sn, c;
        sincospi(2.0 * t / M, &sn, &c);
        tw[t] = make_double2(c, sn);
    }
    __syncthreads();
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= M * M) return;
    const int x0 = x / M, x1 = x % M, h = N / 2;
    double re = 0.0, im = 0.0;
    for (int k0 = 0; k0 < N; ++k0) {
        int t = pmod((k0 - h) * x0 - h * x1, M);
        for (int k1 = 0; k1 < N; ++k1) {
            const double2 g = G[k0 * N + k1], e = tw[t];
            re += g.x * e.x - g.y * e.y;
            im += g.x * e.y + g.y * e.x;
            t += x1;
            if (t >= M) t -= M;
        }
    }
    gt[x] = make_double2(re, im);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One block per (chunk of shifts j, angle p).  LDS holds Gt and (gc_p, gc'_p)
// over the doubled grid, the first-axis transforms of one round of output
// rows and the twiddles w^t = e^{-2 pi i t/M}.  Outputs n0 go in rounds of
// nc <= 256 / N rows so that each thread owns at most one (n0, n1) per
// round (SEP_ROUNDS rounds at most); its sums over the block's shifts stay
// in registers and are written once to the block's partial array.
constexpr int SEP_THREADS = 256;
constexpr int SEP_ROUNDS = 4;
constexpr int SEP_TMAX = 512;  // M * nc

__global__ void __launch_bounds__(SEP_THREADS)
sep_t1_kernel(int N, int M, int nc, int jc, const double2 *__restrict__ gc, const double2 *__restrict__ gt,
              double2 *part) {
    extern __shared__ double2 sm[];
    const int MM = M * M;
    double2 *sG = sm, *sC = sm + MM, *sTA = sm + 2 * MM, *sTB = sTA + SEP_TMAX, *sW = sTB + SEP_TMAX;
    const int p = blockIdx.y, tid = threadIdx.x, h = N / 2;
    for (int i = tid; i < MM; i += SEP_THREADS) {
        sG[i] = gt[i];
        sC[i] = gc[(int64_t)p * MM + i];
    }
    for (int t = tid; t < M; t += SEP_THREADS) {
        double sn, c;
        sincospi(2.0 * t / M, &sn, &c);
        sW[t] = make_double2(c, -sn);
    }
    __syncthreads();
    const int rounds = (N + nc - 1) / nc;
    double2 acc[SEP_ROUNDS];
#pragma unroll
    for (int r = 0; r < SEP_ROUNDS; ++r) acc[r] = make_double2(0.0, 0.0);
    const int jlo = blockIdx.x * jc, jhi = min(MM, jlo + jc);
    for (int j = jlo; j < jhi; ++j) {
        const int j0 = j / M, j1 = j % M;
        const double2 gj = sG[j];
#pragma unroll
        for (int r = 0; r < SEP_ROUNDS; ++r) {
            if (r < rounds) {
                const int n0b = r * nc, ncr = min(nc, N - n0b);
                // first axis: T[x1][n0l] = sum_x0 gc(x0 - j0, x1 - j1) Gt(x0, x1) w^{n0 x0}
                for (int o = tid; o < M * ncr; o += SEP_THREADS) {
                    const int x1 = o % M, n0l = o / M;
                    const int nm = pmod(n0b + n0l - h, M);
                    const int v = pmod(x1 - j1, M);
                    int u = pmod(-j0, M), t = 0;
                    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                    for (int x0 = 0; x0 < M; ++x0) {
                        const double2 c = sC[u * M + v], g = sG[x0 * M + x1], e = sW[t];
                        const double2 ge = cmul(g, e);
                        ar += c.x * ge.x;
                        ai += c.x * ge.y;
                        br += c.y * ge.x;
                        bi += c.y * ge.y;
                        if (++u == M) u = 0;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    sTA[x1 * nc + n0l] = make_double2(ar, ai);
                    sTB[x1 * nc + n0l] = make_double2(br, bi);
                }
                __syncthreads();
                // second axis and the product: one (n0, n1) per thread
                if (tid < ncr * N) {
                    const int n1s = tid % N, n0l = tid / N;
                    const int n1 = n1s - h, n0 = n0b + n0l - h;
                    const int nm = pmod(n1, M);
                    double2 A = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
                    int t = 0;
                    for (int x1 = 0; x1 < M; ++x1) {
                        const double2 e = sW[t];
                        const double2 a = cmul(sTA[x1 * nc + n0l], e), b = cmul(sTB[x1 * nc + n0l], e);
                        A.x += a.x;
                        A.y += a.y;
                        B.x += b.x;
                        B.y += b.y;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    // Gt_j e^{+2 pi i n.j/M} = Gt_j conj(w^{n.j})
                    const double2 wj = sW[pmod(n0 * j0 + n1 * j1, M)];
                    const double2 ej = cmul(gj, make_double2(wj.x, -wj.y));
                    const double2 q = cmul(ej, cmul(A, B));
                    acc[r].x += q.x;
                    acc[r].y += q.y;
                }
                __syncthreads();
            }
        }
    }
    const int64_t base = ((int64_t)p * gridDim.x + blockIdx.x) * N * N;
#pragma unroll
    for (int r = 0; r < SEP_ROUNDS; ++r) {
        if (r < rounds) {
            const int n0b = r * nc, ncr = min(nc, N - n0b);
            if (tid < ncr * N) part[base + (int64_t)(n0b + tid / N) * N + tid % N] = acc[r];
        }
    }
}

// T1[i] = scale * sum over the partial arrays, in array order
__global__ void sep_reduce_kernel(int nparts, int nm, double scale, const double2 *__restrict__ part, double2 *T1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nm) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nparts; ++b) {
        const double2 v = part[(int64_t)b * nm + i];
        re += v.x;
        im += v.y;
    }
    T1[i] = make_double2(scale * re, scale * im);
}

}  // namespace

size_t sep_t1_lds_bytes(int M) { return sizeof(double2) * (2 * (size_t)M * M + 2 * SEP_TMAX + M); }

void sep_shape(int N, int P, int *nc, int *jc, int *nbj) {
    const int M = 2 * N, MM = M * M;
    *nc = std::min(N, SEP_THREADS / N);
    const int want = std::max(1, (2048 + P - 1) / P);  // blocks per angle
    *jc = (MM + want - 1) / want;
    *nbj = (MM + *jc - 1) / *jc;
}

// Angles at which the half-period rectangle rule reproduces beta(a, b) to
// rounding for every a, b in (-N, N)^2: the angular integrand has the
// spectrum of e^{i x cos(.)} with x <= R (|a| + |b|) < 2 sqrt(2) R N, whose
// Bessel coefficients are negligible past order x + 12 x^(1/3) + 24, and the
// rule integrates every order below 2P exactly.
int sep_auto_angles(int N, double R) {
    const double x = 2.0 * std::sqrt(2.0) * R * N;
    return (int)std::ceil(0.5 * x + 6.0 * std::cbrt(x)) + 12;
}

bool sep_supported(int N) {
    if (N < 2 || N > 32 || (N & 1)) return false;
    int nc = std::min(N, SEP_THREADS / N);
    return 2 * N * nc <= SEP_TMAX && (N + nc - 1) / nc <= SEP_ROUNDS && sep_t1_lds_bytes(2 * N) <= 160 * 1024;
}

void launch_sep_tables(int N, int P, double R, double Cphi, double *al, double *alp, double2 *gc, hipStream_t s) {
    const int w = 2 * N - 1, na = w * w, M = 2 * N;
    hipLaunchKernelGGL(sep_alpha_kernel, dim3((na + 255) / 256, P), dim3(256), 0, s, N, P, R, Cphi, al, alp);
    const size_t lds = sizeof(double) * (2 * (size_t)na + M);
    hipLaunchKernelGGL(sep_gc_kernel, dim3((M * M + 255) / 256, P), dim3(256), lds, s, N, M, al, alp, gc);
}

void launch_sep_t1(int N, int P, const double2 *Ghat, const double2 *gc, double2 *gt, double2 *part, double2 *T1,
                   hipStream_t s) {
    const int M = 2 * N;
    int nc, jc, nbj;
    sep_shape(N, P, &nc, &jc, &nbj);
    hipLaunchKernelGGL(sep_gt_kernel, dim3((M * M + 255) / 256), dim3(256), sizeof(double2) * M, s, N, M, Ghat, gt);
    hipLaunchKernelGGL(sep_t1_kernel, dim3(nbj, P), dim3(SEP_THREADS), sep_t1_lds_bytes(M), s, N, M, nc, jc, gc, gt,
                       part);
    const double M2 = (double)M * M;
    const double scale = M_PI / P / (M2 * M2 * M2);
    hipLaunchKernelGGL(sep_reduce_kernel, dim3((N * N + 255) / 256), dim3(256), 0, s, nbj * P, N * N, scale, part, T1);
}

hipError_t sep_prepare() {
    return hipFuncSetAttribute((const void *)sep_t1_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sep_t1_lds_bytes(64));
}

}  // namespace bnq
