// Trilinear term by the separated-kernel transform route (section 'Fast
// computation of the collision modes', eqs. betadD, alphap and alphapprime;
// appendix 'Fast evaluation of the collision kernel').  Written out below for
// d = 2; the d = 3 kernels further down follow the same steps over (2N)^3
// with the directions of eq. alphapprime.
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
// N = 32 that is about 1.2e12 flops per evaluation against 1.9e9 for the
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
// nc <= 256 / N rows so that each thread (2-D: each lane pair) owns at most
// one (n0, n1) per round (SEP_ROUNDS rounds at most); its sums over the
// block's shifts stay in registers and are written once to the block's
// partial array.
constexpr int SEP_THREADS = 512;  // 3-D: two waves per SIMD over the one workgroup an LDS-full CU holds
constexpr int SEP_OUT = 256;      // bound on the outputs of one round (nc N in 2-D)
constexpr int SEP_ROUNDS = 4;
constexpr int SEP_TMAX = 512;  // M * nc

// 2-D: 16 waves; the sums of one output are split over the lanes l and
// l ^ 32 of a wave (one half of the transform axis each) and combined by a
// cross-lane exchange, so that the one workgroup an LDS-full CU holds still
// keeps four waves per SIMD.
constexpr int SEP2_THREADS = 1024;

__global__ void __launch_bounds__(SEP2_THREADS)
sep_t1_kernel(int N, int M, int nc, int jc, const double2 *__restrict__ gc, const double2 *__restrict__ gt,
              double2 *part) {
    extern __shared__ double2 sm[];
    const int MM = M * M;
    double2 *sG = sm, *sC = sm + MM, *sTA = sm + 2 * MM, *sTB = sTA + SEP_TMAX, *sW = sTB + SEP_TMAX;
    const int p = blockIdx.y, tid = threadIdx.x, h = N / 2;
    const int lane = tid & 63, half = lane >> 5;
    const int slot = (tid >> 6) * 32 + (lane & 31);  // output slot, shared by lanes l and l ^ 32
    const int xlo = half * N;                         // this lane's half of the axis: [xlo, xlo + N)
    for (int i = tid; i < MM; i += SEP2_THREADS) {
        sG[i] = gt[i];
        sC[i] = gc[(int64_t)p * MM + i];
    }
    for (int t = tid; t < M; t += SEP2_THREADS) {
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
                for (int o = slot; o < M * ncr; o += SEP2_THREADS / 2) {
                    const int x1 = o % M, n0l = o / M;
                    const int nm = pmod(n0b + n0l - h, M);
                    const int v = pmod(x1 - j1, M);
                    int u = pmod(xlo - j0, M), t = (nm * xlo) % M;
                    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                    for (int x0 = xlo; x0 < xlo + N; ++x0) {
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
                    ar += __shfl_xor(ar, 32);
                    ai += __shfl_xor(ai, 32);
                    br += __shfl_xor(br, 32);
                    bi += __shfl_xor(bi, 32);
                    if (half == 0) {
                        sTA[x1 * nc + n0l] = make_double2(ar, ai);
                        sTB[x1 * nc + n0l] = make_double2(br, bi);
                    }
                }
                __syncthreads();
                // second axis and the product: one (n0, n1) per lane pair
                if (slot < ncr * N) {
                    const int n1s = slot % N, n0l = slot / N;
                    const int n1 = n1s - h, n0 = n0b + n0l - h;
                    const int nm = pmod(n1, M);
                    double2 A = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
                    int t = (nm * xlo) % M;
                    for (int x1 = xlo; x1 < xlo + N; ++x1) {
                        const double2 e = sW[t];
                        const double2 a = cmul(sTA[x1 * nc + n0l], e), b = cmul(sTB[x1 * nc + n0l], e);
                        A.x += a.x;
                        A.y += a.y;
                        B.x += b.x;
                        B.y += b.y;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    A.x += __shfl_xor(A.x, 32);
                    A.y += __shfl_xor(A.y, 32);
                    B.x += __shfl_xor(B.x, 32);
                    B.y += __shfl_xor(B.y, 32);
                    if (half == 0) {
                        // Gt_j e^{+2 pi i n.j/M} = Gt_j conj(w^{n.j})
                        const double2 wj = sW[pmod(n0 * j0 + n1 * j1, M)];
                        const double2 ej = cmul(gj, make_double2(wj.x, -wj.y));
                        const double2 q = cmul(ej, cmul(A, B));
                        acc[r].x += q.x;
                        acc[r].y += q.y;
                    }
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
            if (half == 0 && slot < ncr * N) part[base + (int64_t)(n0b + slot / N) * N + slot % N] = acc[r];
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

// ---------------------------------------------------------------- d = 3
// Directions e_r = (sin t_p cos f_q, sin t_p sin f_q, cos t_p), t_p = p pi / M1,
// f_q = q pi / M2, r = q + M2 p (eq. alphapprime), C = pi^2 / (M1 M2):
//   alpha_r(a)  = 4 C_phi sin t_p phi3(a . e_r),   phi3(s) = int_{-R}^{R} |r| e^{i r s} dr,
//   alpha'_r(b) = psi(|b - (b . e_r) e_r|),        psi(s)  = int_0^pi phi3(s cos t) dt
//                                                          = 2 pi R J_1(R s) / s.
__device__ double sep_phi3(double R, double s) {
    const double x = R * s;
    if (fabs(x) < 0.05) {
        // 2 R^2 sum_k (-1)^k x^{2k} / ((2k)! (2k + 2))
        const double x2 = x * x;
        return 2.0 * R * R * (0.5 - x2 / 8.0 + x2 * x2 / 144.0 - x2 * x2 * x2 / 5760.0);
    }
    const double h = sin(0.5 * x);
    return 2.0 * R * R * (sin(x) / x - 2.0 * h * h / (x * x));
}

__device__ double sep_psi3(double R, double s) {
    const double x = R * s;
    if (fabs(x) < 1e-3) {
        const double x2 = x * x;
        return M_PI * R * R * (1.0 - x2 / 8.0 + x2 * x2 / 192.0);
    }
    return 2.0 * M_PI * R * R * j1(x) / x;
}

__global__ void sep_alpha3_kernel(int N, int M1, int M2, double R, double Cphi, double *al, double *alp) {
    const int w = 2 * N - 1, na = w * w * w;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y, p = r / M2, q = r % M2;
    if (i >= na) return;
    const double a0 = (double)(i / (w * w) - (N - 1)), a1 = (double)((i / w) % w - (N - 1)),
                 a2 = (double)(i % w - (N - 1));
    double st, ct, sf, cf;
    sincospi((double)p / M1, &st, &ct);
    sincospi((double)q / M2, &sf, &cf);
    const double e0 = st * cf, e1 = st * sf, e2 = ct;
    const double pr = a0 * e0 + a1 * e1 + a2 * e2;
    const double perp = sqrt(fmax(a0 * a0 + a1 * a1 + a2 * a2 - pr * pr, 0.0));
    al[(int64_t)r * na + i] = 4.0 * Cphi * st * sep_phi3(R, pr);
    alp[(int64_t)r * na + i] = sep_psi3(R, perp);
}

// gc[r][y] over y in [0, M)^3 row-major
__global__ void sep_gc3_kernel(int N, int M, const double *al, const double *alp, double2 *gc) {
    extern __shared__ double sh[];
    const int w = 2 * N - 1, na = w * w * w;
    double *sa = sh, *sb = sh + na, *cs = sh + 2 * na;
    const int r = blockIdx.y;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        sa[i] = al[(int64_t)r * na + i];
        sb[i] = alp[(int64_t)r * na + i];
    }
    for (int t = threadIdx.x; t < M; t += blockDim.x) cs[t] = cospi(2.0 * t / M);
    __syncthreads();
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= M * M * M) return;
    const int y0 = y / (M * M), y1 = (y / M) % M, y2 = y % M;
    double ga = 0.0, gb = 0.0;
    for (int i0 = 0; i0 < w; ++i0)
        for (int i1 = 0; i1 < w; ++i1) {
            int t = pmod((i0 - (N - 1)) * y0 + (i1 - (N - 1)) * y1 - (N - 1) * y2, M);
            const double *ra = sa + (i0 * w + i1) * w, *rb = sb + (i0 * w + i1) * w;
            for (int i2 = 0; i2 < w; ++i2) {
                const double c = cs[t];
                ga += ra[i2] * c;
                gb += rb[i2] * c;
                t += y2;
                if (t >= M) t -= M;
            }
        }
    gc[(int64_t)r * M * M * M + y] = make_double2(ga, gb);
}

// Gt[x] = sum_{k in I_N} G_k e^{2 pi i k.x/M}, x in [0, M)^3 row-major
__global__ void sep_gt3_kernel(int N, int M, const double2 *__restrict__ G, double2 *gt) {
    extern __shared__ double2 tw[];
    for (int t = threadIdx.x; t < M; t += blockDim.x) {
        double sn, c;
        sincospi(2.0 * t / M, &sn, &c);
        tw[t] = make_double2(c, sn);
    }
    __syncthreads();
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= M * M * M) return;
    const int x0 = x / (M * M), x1 = (x / M) % M, x2 = x % M, h = N / 2;
    double re = 0.0, im = 0.0;
    for (int k0 = 0; k0 < N; ++k0)
        for (int k1 = 0; k1 < N; ++k1) {
            int t = pmod((k0 - h) * x0 + (k1 - h) * x1 - h * x2, M);
            for (int k2 = 0; k2 < N; ++k2) {
                const double2 g = G[(k0 * N + k1) * N + k2], e = tw[t];
                re += g.x * e.x - g.y * e.y;
                im += g.x * e.y + g.y * e.x;
                t += x2;
                if (t >= M) t -= M;
            }
        }
    gt[x] = make_double2(re, im);
}

// As sep_t1_kernel, with three passes: x0 -> n0 (in rounds of nc rows n0),
// x1 -> n1, then x2 -> n2 and the product.
constexpr int SEP3_T1MAX = 512;  // nc M^2
constexpr int SEP3_T2MAX = 256;  // nc N M

__global__ void __launch_bounds__(SEP_THREADS)
sep_t1_3_kernel(int N, int M, int nc, int jc, const double2 *__restrict__ gc, const double2 *__restrict__ gt,
                double2 *part) {
    extern __shared__ double2 sm[];
    const int MM = M * M, M3 = MM * M;
    double2 *sG = sm, *sC = sm + M3, *sAA = sm + 2 * M3, *sAB = sAA + SEP3_T1MAX, *sBA = sAB + SEP3_T1MAX,
            *sBB = sBA + SEP3_T2MAX, *sW = sBB + SEP3_T2MAX;
    const int r = blockIdx.y, tid = threadIdx.x, h = N / 2;
    for (int i = tid; i < M3; i += SEP_THREADS) {
        sG[i] = gt[i];
        sC[i] = gc[(int64_t)r * M3 + i];
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
    for (int k = 0; k < SEP_ROUNDS; ++k) acc[k] = make_double2(0.0, 0.0);
    const int jlo = blockIdx.x * jc, jhi = min(M3, jlo + jc);
    for (int j = jlo; j < jhi; ++j) {
        const int j0 = j / MM, j1 = (j / M) % M, j2 = j % M;
        const double2 gj = sG[j];
#pragma unroll
        for (int k = 0; k < SEP_ROUNDS; ++k) {
            if (k < rounds) {
                const int n0b = k * nc, ncr = min(nc, N - n0b);
                // x0 -> n0: T1[n0l][x1][x2]
                for (int o = tid; o < ncr * MM; o += SEP_THREADS) {
                    const int x2 = o % M, x1 = (o / M) % M, n0l = o / MM;
                    const int nm = pmod(n0b + n0l - h, M);
                    const int v = pmod(x1 - j1, M) * M + pmod(x2 - j2, M);
                    int u = pmod(-j0, M), t = 0;
                    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                    for (int x0 = 0; x0 < M; ++x0) {
                        const double2 c = sC[u * MM + v], g = sG[x0 * MM + x1 * M + x2], e = sW[t];
                        const double2 ge = cmul(g, e);
                        ar += c.x * ge.x;
                        ai += c.x * ge.y;
                        br += c.y * ge.x;
                        bi += c.y * ge.y;
                        if (++u == M) u = 0;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    sAA[o] = make_double2(ar, ai);
                    sAB[o] = make_double2(br, bi);
                }
                __syncthreads();
                // x1 -> n1: T2[n0l][n1][x2]
                if (tid < ncr * N * M) {
                    const int x2 = tid % M, n1s = (tid / M) % N, n0l = tid / (M * N);
                    const int nm = pmod(n1s - h, M);
                    double2 A = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
                    int t = 0;
                    for (int x1 = 0; x1 < M; ++x1) {
                        const double2 e = sW[t];
                        const double2 a = cmul(sAA[(n0l * M + x1) * M + x2], e),
                                      b = cmul(sAB[(n0l * M + x1) * M + x2], e);
                        A.x += a.x;
                        A.y += a.y;
                        B.x += b.x;
                        B.y += b.y;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    sBA[tid] = A;
                    sBB[tid] = B;
                }
                __syncthreads();
                // x2 -> n2 and the product: one (n0, n1, n2) per thread
                if (tid < ncr * N * N) {
                    const int n2s = tid % N, n1s = (tid / N) % N, n0l = tid / (N * N);
                    const int n2 = n2s - h, n1 = n1s - h, n0 = n0b + n0l - h;
                    const int nm = pmod(n2, M);
                    double2 A = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
                    int t = 0;
                    for (int x2 = 0; x2 < M; ++x2) {
                        const double2 e = sW[t];
                        const double2 a = cmul(sBA[(n0l * N + n1s) * M + x2], e),
                                      b = cmul(sBB[(n0l * N + n1s) * M + x2], e);
                        A.x += a.x;
                        A.y += a.y;
                        B.x += b.x;
                        B.y += b.y;
                        t += nm;
                        if (t >= M) t -= M;
                    }
                    const double2 wj = sW[pmod(n0 * j0 + n1 * j1 + n2 * j2, M)];
                    const double2 q = cmul(cmul(gj, make_double2(wj.x, -wj.y)), cmul(A, B));
                    acc[k].x += q.x;
                    acc[k].y += q.y;
                }
                __syncthreads();
            }
        }
    }
    const int NN = N * N;
    const int64_t base = ((int64_t)r * gridDim.x + blockIdx.x) * NN * N;
#pragma unroll
    for (int k = 0; k < SEP_ROUNDS; ++k) {
        if (k < rounds) {
            const int n0b = k * nc, ncr = min(nc, N - n0b);
            if (tid < ncr * NN) part[base + (int64_t)n0b * NN + tid] = acc[k];
        }
    }
}

}  // namespace

size_t sep_t1_lds_bytes(int d, int M) {
    return d == 2 ? sizeof(double2) * (2 * (size_t)M * M + 2 * SEP_TMAX + M)
                  : sizeof(double2) * (2 * (size_t)M * M * M + 2 * SEP3_T1MAX + 2 * SEP3_T2MAX + M);
}

int sep_directions(int d, int angles) { return d == 2 ? angles : 2 * angles * angles; }

void sep_shape(int d, int N, int P, int *nc, int *jc, int *nbj) {
    const int M = 2 * N, Md = d == 2 ? M * M : M * M * M;
    *nc = d == 2 ? std::min(N, SEP_OUT / N) : std::min(N, SEP3_T1MAX / (M * M));
    const int want = std::max(1, (2048 + P - 1) / P);  // blocks per direction
    *jc = (Md + want - 1) / want;
    *nbj = (Md + *jc - 1) / *jc;
}

// Angles at which the half-period rectangle rule reproduces beta(a, b) to
// rounding for every a, b in (-N, N)^2: the angular integrand has the
// spectrum of e^{i x cos(.)} with x <= R (|a| + |b|) < 2 sqrt(2) R N, whose
// Bessel coefficients are negligible past order x + 12 x^(1/3) + 24, and the
// rule integrates every order below 2P exactly.  (The 3-D polar rule
// converges at second order only: there the caller chooses the count.)
int sep_auto_angles(int N, double R) {
    const double x = 2.0 * std::sqrt(2.0) * R * N;
    return (int)std::ceil(0.5 * x + 6.0 * std::cbrt(x)) + 12;
}

bool sep_supported(int d, int N) {
    if (N < 2 || (N & 1)) return false;
    const int M = 2 * N;
    int nc, jc, nbj;
    sep_shape(d, N, 1, &nc, &jc, &nbj);
    if (nc < 1 || (N + nc - 1) / nc > SEP_ROUNDS || sep_t1_lds_bytes(d, M) > 160 * 1024) return false;
    if (d == 2) return N <= 32 && M * nc <= SEP_TMAX && nc * N <= SEP_OUT;
    return d == 3 && N <= 8 && nc * M * M <= SEP3_T1MAX && nc * N * M <= SEP3_T2MAX && nc * N * M <= SEP_THREADS &&
           nc * N * N <= SEP_THREADS;
}

void launch_sep_tables(int d, int N, int angles, double R, double Cphi, double *al, double *alp, double2 *gc,
                       hipStream_t s) {
    const int w = 2 * N - 1, M = 2 * N;
    if (d == 2) {
        const int na = w * w, P = angles;
        hipLaunchKernelGGL(sep_alpha_kernel, dim3((na + 255) / 256, P), dim3(256), 0, s, N, P, R, Cphi, al, alp);
        const size_t lds = sizeof(double) * (2 * (size_t)na + M);
        hipLaunchKernelGGL(sep_gc_kernel, dim3((M * M + 255) / 256, P), dim3(256), lds, s, N, M, al, alp, gc);
        return;
    }
    const int na = w * w * w, M1 = angles, M2 = 2 * angles, P = M1 * M2;
    hipLaunchKernelGGL(sep_alpha3_kernel, dim3((na + 255) / 256, P), dim3(256), 0, s, N, M1, M2, R, Cphi, al, alp);
    const size_t lds = sizeof(double) * (2 * (size_t)na + M);
    hipLaunchKernelGGL(sep_gc3_kernel, dim3((M * M * M + 255) / 256, P), dim3(256), lds, s, N, M, al, alp, gc);
}

void launch_sep_t1(int d, int N, int P, const double2 *Ghat, const double2 *gc, double2 *gt, double2 *part,
                   double2 *T1, hipStream_t s) {
    const int M = 2 * N;
    int nc, jc, nbj;
    sep_shape(d, N, P, &nc, &jc, &nbj);
    const double M2 = (double)M * M;
    if (d == 2) {
        hipLaunchKernelGGL(sep_gt_kernel, dim3((M * M + 255) / 256), dim3(256), sizeof(double2) * M, s, N, M, Ghat,
                           gt);
        hipLaunchKernelGGL(sep_t1_kernel, dim3(nbj, P), dim3(SEP2_THREADS), sep_t1_lds_bytes(2, M), s, N, M, nc, jc,
                           gc, gt, part);
        const double scale = M_PI / P / (M2 * M2 * M2);  // C M^-3d, C = pi / P
        hipLaunchKernelGGL(sep_reduce_kernel, dim3((N * N + 255) / 256), dim3(256), 0, s, nbj * P, N * N, scale, part,
                           T1);
        return;
    }
    const int M3 = M * M * M, N3 = N * N * N;
    hipLaunchKernelGGL(sep_gt3_kernel, dim3((M3 + 255) / 256), dim3(256), sizeof(double2) * M, s, N, M, Ghat, gt);
    hipLaunchKernelGGL(sep_t1_3_kernel, dim3(nbj, P), dim3(SEP_THREADS), sep_t1_lds_bytes(3, M), s, N, M, nc, jc, gc,
                       gt, part);
    double scale = M_PI * M_PI / P;  // C M^-3d, C = pi^2 / (M1 M2) = pi^2 / P
    for (int k = 0; k < 9; ++k) scale /= M;
    hipLaunchKernelGGL(sep_reduce_kernel, dim3((N3 + 255) / 256), dim3(256), 0, s, nbj * P, N3, scale, part, T1);
}

hipError_t sep_prepare() {
    hipError_t e = hipFuncSetAttribute((const void *)sep_t1_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sep_t1_lds_bytes(2, 64));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)sep_t1_3_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sep_t1_lds_bytes(3, 16));
}

}  // namespace bnq
