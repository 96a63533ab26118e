// Evaluation of the Galerkin modes Qhat_n (Lemma of Section 3.3) and of the
// grid values Q_j on gfx950, FP64.
//
//   forward DFT      G_k = N^-d sum_j f_j e^{-2 pi i k.j/N}        (Section 4.3, step 2a)
//   pair sums        Qc_s = sum_{l+m=s} wc(l,m) G_l G_m   (s in I_N)
//                    W_s  = sum_{l+m=s} wq(l,m) G_l G_m   (s in Eg)
//   outer sum        X_n  = sum_k G_k W_{n-k}
//   trilinear sum    T1_n = sum_{k+l+m=n} beta(k+m,l+m) G_k G_l G_m
//                         = sum_b G_{n-b} sum_p beta(n-p, b) G_p G_{b-p}
//   combination      Qhat = Qc - alpha (T1 + X)           (Section 3.1 decomposition)
//   inverse DFT      Q_j = c (L/pi)^(d+gamma) Re sum_n Qhat_n e^{2 pi i n.j/N}
//
// The pair sums stream the two pair-weight tables once per evaluation
// (HBM-bound).  The trilinear sum, which dominates, is evaluated for each b
// in the frame where b is canonical (b = R b_c, R a signed axis permutation):
// beta(n-p, b) = beta(R^-1(n-p), b_c) because the kernel modes depend only on
// |.|^2 and |a.b|, so one table row per canonical b_c serves the whole orbit,
// read contiguously, and the spectrum is rotated instead (G_R(q) = G(R q)).
// Inside a b, the sum over p is a Toeplitz product along every axis; each lane
// owns 8 consecutive outputs along x and slides a 16-value register window of
// the table row across the inner index, so every loaded value feeds 16 FMAs.
#include "bnq_internal.h"

namespace bnq {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// ---------------------------------------------------------------------------
// DFT along one axis.  in/out are [e0][N][N] (axis 0 extent e0); the axis
// `ax` has extent N.  tw[t] = exp(-2 pi i t / N); sign = -1 forward, +1 inverse.
template <typename Tin>
__device__ __forceinline__ double2 load_c(const Tin *p, int64_t i);
template <>
__device__ __forceinline__ double2 load_c<double>(const double *p, int64_t i) {
    return make_double2(p[i], 0.0);
}
template <>
__device__ __forceinline__ double2 load_c<double2>(const double2 *p, int64_t i) {
    return p[i];
}

template <typename Tin, int MODE>  // MODE 0: complex out, 1: real part * scale
__global__ void dft_axis_kernel(Geo g, const Tin *in, double2 *out, double *rout, int ax, int sign,
                                double scale, const double2 *tw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const int N = g.N, h = g.h;
    const int64_t stride = ax == 2 ? 1 : (ax == 1 ? N : (int64_t)N * N);
    const int kpos = (int)((i / stride) % N);
    const int k = kpos - h;
    const int64_t base = i - (int64_t)kpos * stride;
    double re = 0.0, im = 0.0;
    for (int jp = 0; jp < N; ++jp) {
        const int j = jp - h;
        int t = (k * j) % N;
        if (t < 0) t += N;
        double2 w = tw[t];
        if (sign > 0) w.y = -w.y;
        const double2 v = load_c<Tin>(in, base + (int64_t)jp * stride);
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
    }
    if (MODE == 0)
        out[i] = make_double2(re * scale, im * scale);
    else
        rout[i] = re * scale;
}

void launch_dft_forward_real(const Geo &g, const double *f, double2 *tmp, double2 *out,
                             const double2 *tw, hipStream_t s) {
    const unsigned nb = (unsigned)((g.nm + 255) / 256);
    const double sc = 1.0 / g.N;
    if (g.d == 2) {
        hipLaunchKernelGGL((dft_axis_kernel<double, 0>), dim3(nb), dim3(256), 0, s, g, f, tmp, (double *)nullptr, 2, -1, sc, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, (const double2 *)tmp, out, (double *)nullptr, 1, -1, sc, tw);
    } else {
        hipLaunchKernelGGL((dft_axis_kernel<double, 0>), dim3(nb), dim3(256), 0, s, g, f, out, (double *)nullptr, 2, -1, sc, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, (const double2 *)out, tmp, (double *)nullptr, 1, -1, sc, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, (const double2 *)tmp, out, (double *)nullptr, 0, -1, sc, tw);
    }
}

void launch_inverse_real(const Geo &g, const double2 *Qh, double2 *tmp, double2 *tmp2, double *Q,
                         const double2 *tw, double scale, hipStream_t s) {
    const unsigned nb = (unsigned)((g.nm + 255) / 256);
    if (g.d == 2) {
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, Qh, tmp, (double *)nullptr, 1, +1, 1.0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 1>), dim3(nb), dim3(256), 0, s, g, (const double2 *)tmp, (double2 *)nullptr, Q, 2, +1, scale, tw);
    } else {
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, Qh, tmp, (double *)nullptr, 0, +1, 1.0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), dim3(nb), dim3(256), 0, s, g, (const double2 *)tmp, tmp2, (double *)nullptr, 1, +1, 1.0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 1>), dim3(nb), dim3(256), 0, s, g, (const double2 *)tmp2, (double2 *)nullptr, Q, 2, +1, scale, tw);
    }
}

// ---------------------------------------------------------------------------
// Rotated spectra: Gr[r][q] = G(R_r q) if R_r q in I_N, else 0, q in Ext.
__global__ void rotate_kernel(Geo g, const double2 *G, const Rot *rots, double2 *Gr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= g.next) return;
    const int X = g.N + 1;
    int q[3];
    q[2] = (int)(i % X) - g.h;
    q[1] = (int)((i / X) % X) - g.h;
    q[0] = g.d == 3 ? (int)(i / ((int64_t)X * X)) - g.h : 0;
    const Rot R = rots[r];
    int y[3];
    for (int a = 0; a < 3; ++a) y[a] = R.sgn[a] * q[R.perm[a]];
    const bool in = y[1] >= -g.h && y[1] < g.h && y[2] >= -g.h && y[2] < g.h &&
                    (g.d == 2 ? y[0] == 0 : (y[0] >= -g.h && y[0] < g.h));
    Gr[(int64_t)r * g.next + i] = in ? G[idx_I(g, y[0], y[1], y[2])] : make_double2(0.0, 0.0);
}

void launch_rotate(const Geo &g, const double2 *G, const Rot *rots, int nrot, double2 *Gr, hipStream_t s) {
    dim3 grid((unsigned)((g.next + 255) / 256), (unsigned)nrot);
    hipLaunchKernelGGL(rotate_kernel, grid, dim3(256), 0, s, g, G, rots, Gr);
}

// ---------------------------------------------------------------------------
// Pair sums.  One block = a 4 x 4 x 16 tile of outputs s (16 x 16 in 2-D);
// all lanes walk the same l over the tile's reachable box, so G_l is a
// broadcast load and the weight rows are read in 128-byte runs.
constexpr int PT0 = 4, PT1 = 4, PT2 = 16;

__global__ __launch_bounds__(256) void pairs_kernel(Geo g, const double2 *G, const double *wc,
                                                    const double *wq, double2 *Qc, double2 *W, int want_c,
                                                    int want_w) {
    const int N = g.N, h = g.h;
    const int t0 = g.d == 3 ? PT0 : 1, t1 = g.d == 3 ? PT1 : 16, t2 = PT2;
    const int nt2 = (2 * N + t2 - 1) / t2, nt1 = (2 * N + t1 - 1) / t1;
    int bid = blockIdx.x;
    const int b2 = bid % nt2;
    bid /= nt2;
    const int b1 = bid % nt1;
    const int b0 = bid / nt1;
    const int tid = threadIdx.x;
    const int s2 = b2 * t2 + tid % t2 - N;
    const int s1 = b1 * t1 + (tid / t2) % t1 - N;
    const int s0 = g.d == 3 ? b0 * t0 + tid / (t2 * t1) - N : 0;
    const bool valid = s2 < N && s1 < N && (g.d == 2 || s0 < N);
    const bool inI = s2 >= -h && s2 < h && s1 >= -h && s1 < h && (g.d == 2 || (s0 >= -h && s0 < h));
    // reachable l box of the tile: l and s - l in I_N
    int lo[3], hi[3];
    const int smin[3] = {g.d == 3 ? b0 * t0 - N : 0, b1 * t1 - N, b2 * t2 - N};
    const int smax[3] = {g.d == 3 ? min(b0 * t0 + t0 - 1 - N, N - 1) : 0, min(b1 * t1 + t1 - 1 - N, N - 1),
                         min(b2 * t2 + t2 - 1 - N, N - 1)};
    for (int a = 0; a < 3; ++a) {
        const int ilo = (a == 0 && g.d == 2) ? 0 : -h, ihi = (a == 0 && g.d == 2) ? 0 : h - 1;
        lo[a] = max(ilo, smin[a] - ihi);
        hi[a] = min(ihi, smax[a] - ilo);
    }
    double2 accw = make_double2(0.0, 0.0), accc = make_double2(0.0, 0.0);
    const bool do_c = want_c && inI;
    for (int l0 = lo[0]; l0 <= hi[0]; ++l0) {
        const int m0 = s0 - l0;
        const bool ok0 = g.d == 2 || (m0 >= -h && m0 < h);
        for (int l1 = lo[1]; l1 <= hi[1]; ++l1) {
            const int m1 = s1 - l1;
            const bool ok1 = ok0 && m1 >= -h && m1 < h;
            for (int l2 = lo[2]; l2 <= hi[2]; ++l2) {
                const int m2 = s2 - l2;
                if (valid && ok1 && m2 >= -h && m2 < h) {
                    const int64_t il = idx_I(g, l0, l1, l2), im = idx_I(g, m0, m1, m2);
                    const double2 p = cmul(G[il], G[im]);
                    const int64_t o = il * g.nm + im;
                    if (want_w) {
                        const double w = wq[o];
                        accw.x = fma(w, p.x, accw.x);
                        accw.y = fma(w, p.y, accw.y);
                    }
                    if (do_c) {
                        const double w = wc[o];
                        accc.x = fma(w, p.x, accc.x);
                        accc.y = fma(w, p.y, accc.y);
                    }
                }
            }
        }
    }
    if (!valid) return;
    if (want_w) W[idx_E(g, s0, s1, s2)] = accw;
    if (do_c) Qc[idx_I(g, s0, s1, s2)] = accc;
}

void launch_pairs(const Geo &g, const double2 *G, const double *wc, const double *wq, double2 *Qc,
                  double2 *W, int want_c, int want_w, hipStream_t s) {
    const int N = g.N;
    const int t0 = g.d == 3 ? PT0 : 1, t1 = g.d == 3 ? PT1 : 16, t2 = PT2;
    const int nb = ((2 * N + t2 - 1) / t2) * ((2 * N + t1 - 1) / t1) * (g.d == 3 ? (2 * N + t0 - 1) / t0 : 1);
    hipLaunchKernelGGL(pairs_kernel, dim3(nb), dim3(256), 0, s, g, G, wc, wq, Qc, W, want_c, want_w);
}

// ---------------------------------------------------------------------------
// Outer sum X_n = sum_k G_k W_{n-k}; n - k always lies in Eg.
__global__ __launch_bounds__(256) void outer_kernel(Geo g, const double2 *G, const double2 *W, double2 *X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const int N = g.N, h = g.h;
    const int n2 = (int)(i % N) - h, n1 = (int)((i / N) % N) - h;
    const int n0 = g.d == 3 ? (int)(i / ((int64_t)N * N)) - h : 0;
    double2 acc = make_double2(0.0, 0.0);
    const int k0lo = g.d == 3 ? -h : 0, k0hi = g.d == 3 ? h - 1 : 0;
    for (int k0 = k0lo; k0 <= k0hi; ++k0)
        for (int k1 = -h; k1 < h; ++k1) {
            const double2 *Grow = G + idx_I(g, k0, k1, -h);
            const double2 *Wrow = W + idx_E(g, n0 - k0, n1 - k1, n2 + h);
            for (int k2 = 0; k2 < N; ++k2) {
                const double2 a = Grow[k2], b = Wrow[-k2];
                acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
                acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
            }
        }
    X[i] = acc;
}

void launch_outer(const Geo &g, const double2 *G, const double2 *W, double2 *X, hipStream_t s) {
    hipLaunchKernelGGL(outer_kernel, dim3((unsigned)((g.nm + 255) / 256)), dim3(256), 0, s, g, G, W, X);
}

// ---------------------------------------------------------------------------
// Trilinear sum.  One 64-lane workgroup per slot; each slot walks its static
// list of items (b, range of <= 64 tasks) and accumulates into its own
// partial array (no atomics; the slots are summed in a fixed order later).
constexpr int T1_NPAD = 64;  // padded inner row length (N <= 64)

__global__ __launch_bounds__(64) void trilinear_kernel(Geo g, const int *slot_off, const T1Item *items,
                                                       const T1B *bdesc, const double *K, const double2 *Gr,
                                                       const Rot *rots, double2 *part) {
    __shared__ double2 P[T1_ROWS][T1_NPAD];
    const int slot = blockIdx.x;
    const int lane = threadIdx.x;
    double2 *mypart = part + (int64_t)slot * g.nm;
    const int N = g.N;
    const int A = 2 * N - 1;
    const int it_end = slot_off[slot + 1];
    for (int it = slot_off[slot]; it < it_end; ++it) {
        const T1Item item = items[it];
        const T1B B = bdesc[item.b];
        const Rot R = rots[B.rot];
        const double2 *G = Gr + (int64_t)B.rot * g.next;
        const double *Krow = K + (int64_t)B.kc * g.na;
        const bool active = lane < item.nt;
        const int t = item.t0 + lane;
        const int wny = B.wnhi[1] - B.wnlo[1] + 1;
        const int xb = t % B.nxb;
        const int rest = t / B.nxb;
        const int ny = B.wnlo[1] + rest % wny;
        const int nz = B.wnlo[0] + rest / wny;
        const int x0 = B.wnlo[2] + xb * T1_RB;
        const int wpx = B.wphi[2] - B.wplo[2] + 1;
        const int wpxp = (wpx + 7) & ~7;
        const int wpy = B.wphi[1] - B.wplo[1] + 1;
        const int nrows = wpy * (B.wphi[0] - B.wplo[0] + 1);
        const int base = x0 - B.wplo[2];  // a_x = base + i - u
        double zr[T1_RB], zi[T1_RB];
#pragma unroll
        for (int i = 0; i < T1_RB; ++i) zr[i] = zi[i] = 0.0;
        for (int r0 = 0; r0 < nrows; r0 += T1_ROWS) {
            const int nr = min(T1_ROWS, nrows - r0);
            __syncthreads();
            for (int e = lane; e < nr * wpxp; e += 64) {
                const int rr = e / wpxp, u = e - rr * wpxp;
                const int row = r0 + rr;
                const int py = B.wplo[1] + row % wpy, pz = B.wplo[0] + row / wpy;
                double2 v = make_double2(0.0, 0.0);
                if (u < wpx) {
                    const int px = B.wplo[2] + u;
                    v = cmul(G[idx_X(g, pz, py, px)], G[idx_X(g, B.bc[0] - pz, B.bc[1] - py, B.bc[2] - px)]);
                }
                P[rr][u] = v;
            }
            __syncthreads();
            if (!active) continue;
            for (int rr = 0; rr < nr; ++rr) {
                const int row = r0 + rr;
                const int py = B.wplo[1] + row % wpy, pz = B.wplo[0] + row / wpy;
                const double *Kr = Krow + ((int64_t)(g.d == 3 ? nz - pz + N - 1 : 0) * A + (ny - py + N - 1)) * A + (N - 1);
                // kw[s] = K(a_x = base - ub + s - 8), clamped into the row
                double kw[16];
#pragma unroll
                for (int s = 0; s < 16; ++s) kw[s] = Kr[min(max(base + s - 8, 1 - N), N - 1)];
                for (int ub = 0; ub < wpxp; ub += 8) {
                    if (ub > 0) {
#pragma unroll
                        for (int s = 0; s < 8; ++s) kw[8 + s] = kw[s];
#pragma unroll
                        for (int s = 0; s < 8; ++s) kw[s] = Kr[min(max(base - ub + s - 8, 1 - N), N - 1)];
                    }
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const double2 p = P[rr][ub + jj];
#pragma unroll
                        for (int i = 0; i < T1_RB; ++i) {
                            const double k = kw[i - jj + 8];
                            zr[i] = fma(k, p.x, zr[i]);
                            zi[i] = fma(k, p.y, zi[i]);
                        }
                    }
                }
            }
        }
        if (active) {
            const int np[3] = {nz, ny, 0};
#pragma unroll
            for (int i = 0; i < T1_RB; ++i) {
                const int nx = x0 + i;
                if (nx <= B.wnhi[2]) {
                    const double2 gk = G[idx_X(g, nz - B.bc[0], ny - B.bc[1], nx - B.bc[2])];
                    const double2 c = cmul(gk, make_double2(zr[i], zi[i]));
                    const int v[3] = {np[0], np[1], nx};
                    const int o0 = R.sgn[0] * v[R.perm[0]];
                    const int o1 = R.sgn[1] * v[R.perm[1]];
                    const int o2 = R.sgn[2] * v[R.perm[2]];
                    double2 *dst = mypart + idx_I(g, o0, o1, o2);
                    double2 cur = *dst;
                    cur.x += c.x;
                    cur.y += c.y;
                    *dst = cur;
                }
            }
        }
    }
}

void launch_trilinear(const Geo &g, int nslots, const int *slot_off, const T1Item *items, const T1B *bdesc,
                      const double *K, const double2 *Gr, const Rot *rots, double2 *part, hipStream_t s) {
    hipLaunchKernelGGL(trilinear_kernel, dim3(nslots), dim3(64), 0, s, g, slot_off, items, bdesc, K, Gr, rots, part);
}

__global__ void zero_kernel(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void launch_zero(void *p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 8;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, s, (double *)p, n);
}

__global__ void reduce_partials_kernel(Geo g, int nslots, const double2 *part, double2 *T1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < nslots; ++s) {
        const double2 v = part[(int64_t)s * g.nm + i];
        re += v.x;
        im += v.y;
    }
    T1[i] = make_double2(re, im);
}

void launch_reduce_partials(const Geo &g, int nslots, const double2 *part, double2 *T1, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((g.nm + 255) / 256)), dim3(256), 0, s, g, nslots, part, T1);
}

// Qhat = [Qc] - alpha ([T1] + [X]) with the selected terms; optionally the
// real part of the n = 0 mode is removed (exact discrete mass conservation).
__global__ void combine_kernel(Geo g, const double2 *Qc, const double2 *T1, const double2 *X, int terms,
                               double alpha, int mass_fix, double2 *Qh, double2 *Qh_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    double re = 0.0, im = 0.0;
    if (terms & 1) {
        re = Qc[i].x;
        im = Qc[i].y;
    }
    double qr = 0.0, qi = 0.0;
    if (terms & 4) {
        qr += T1[i].x;
        qi += T1[i].y;
    }
    if (terms & 2) {
        qr += X[i].x;
        qi += X[i].y;
    }
    re -= alpha * qr;
    im -= alpha * qi;
    if (mass_fix && i == idx_I(g, 0, 0, 0)) re = 0.0;
    Qh[i] = make_double2(re, im);
    if (Qh_out) Qh_out[i] = make_double2(re, im);
}

void launch_combine(const Geo &g, const double2 *Qc, const double2 *T1, const double2 *X, int terms, double alpha,
                    int mass_fix, double2 *Qh, double2 *Qh_out, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((g.nm + 255) / 256)), dim3(256), 0, s, g, Qc, T1, X, terms,
                       alpha, mass_fix, Qh, Qh_out);
}

}  // namespace bnq
