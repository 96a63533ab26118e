// Evaluation of the Galerkin modes Qhat_n (Lemma of section 'Fast spectral approximation of the BNE operator') and of the
// grid values Q_j on gfx950, FP64.
//
//   forward DFT      G_k = N^-d sum_j f_j e^{-2 pi i k.j/N}        (section 'Numerical scheme for the velocity rescaled BNE', step 2a)
//   pair sums        Qc_s = sum_{l+m=s} wc(l,m) G_l G_m   (s in I_N)
//                    W_s  = sum_{l+m=s} wq(l,m) G_l G_m   (s in Eg)
//   outer sum        X_n  = sum_k G_k W_{n-k}
//   trilinear sum    T1_n = sum_{k+l+m=n} beta(k+m,l+m) G_k G_l G_m
//                         = sum_b G_{n-b} sum_p beta(n-p, b) G_p G_{b-p}
//   combination      Qhat = Qc - alpha (T1 + X)           (section 'The Carleman representation' decomposition)
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


__device__ __forceinline__ const void *sel_ptr(const Inst &I, const IOs &io, int z, int sel) {
    switch (sel) {
        case BUF_IN: return io.in[z];
        case BUF_OUT: return io.out[z];
        case BUF_TMP: return I.tmp;
        case BUF_TMP2: return I.tmp2;
        case BUF_GHAT: return I.Ghat;
        case BUF_QH: return I.Qh;
        case BUF_Y: return I.ybuf;
        default: return I.k[sel - BUF_K0];
    }
}

// ---------------------------------------------------------------------------
// DFT along one axis.  in/out are [e0][N][N] (axis 0 extent e0); the axis
// `ax` has extent N.  tw[t] = exp(-2 pi i t / N); sign = -1 forward, +1 inverse.
__device__ __forceinline__ double2 load_c(const double *p, int64_t i) { return make_double2(glob(p)[i], 0.0); }
__device__ __forceinline__ double2 load_c(const double2 *p, int64_t i) { return ld2(p, i); }

// MODE 0: complex out; 1: real part.  smode: scale 1, 1/N or Inst::pref.
template <typename Tin, int MODE>
__global__ void dft_axis_kernel(Geo g, const Inst *D, IOs io, int sin, int sout, int ax, int sign, int smode,
                                const double2 *tw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    const Tin *in = (const Tin *)sel_ptr(I, io, z, sin);
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
        const double2 v = load_c(in, base + (int64_t)jp * stride);
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
    }
    const double scale = smode == 0 ? 1.0 : (smode == 1 ? 1.0 / N : I.pref);
    if (MODE == 0)
        st2((double2 *)sel_ptr(I, io, z, sout), i, make_double2(re * scale, im * scale));
    else
        glob((double *)sel_ptr(I, io, z, sout))[i] = re * scale;
}

static dim3 grid_nm(const Geo &g, const IOs &io) { return dim3((unsigned)((g.nm + 255) / 256), 1, (unsigned)io.n); }

void launch_dft_forward_real(const Geo &g, const Inst *D, const IOs &io, const double2 *tw, hipStream_t s) {
    const dim3 gr = grid_nm(g, io);
    if (g.d == 2) {
        hipLaunchKernelGGL((dft_axis_kernel<double, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_IN, (int)BUF_TMP, 2, -1, 1, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_TMP, (int)BUF_GHAT, 1, -1, 1, tw);
    } else {
        hipLaunchKernelGGL((dft_axis_kernel<double, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_IN, (int)BUF_GHAT, 2, -1, 1, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_GHAT, (int)BUF_TMP, 1, -1, 1, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_TMP, (int)BUF_GHAT, 0, -1, 1, tw);
    }
}

void launch_inverse_real(const Geo &g, const Inst *D, const IOs &io, const double2 *tw, hipStream_t s) {
    const dim3 gr = grid_nm(g, io);
    if (g.d == 2) {
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_QH, (int)BUF_TMP, 1, +1, 0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 1>), gr, dim3(256), 0, s, g, D, io, (int)BUF_TMP, (int)BUF_OUT, 2, +1, 2, tw);
    } else {
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_QH, (int)BUF_TMP, 0, +1, 0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 0>), gr, dim3(256), 0, s, g, D, io, (int)BUF_TMP, (int)BUF_TMP2, 1, +1, 0, tw);
        hipLaunchKernelGGL((dft_axis_kernel<double2, 1>), gr, dim3(256), 0, s, g, D, io, (int)BUF_TMP2, (int)BUF_OUT, 2, +1, 2, tw);
    }
}

// ---------------------------------------------------------------------------
// Rotated spectra: Gr[r][q] = G(R_r q) if R_r q in I_N, else 0, q in Ext.
// Only instances that evaluate the trilinear term.
__global__ void rotate_kernel(Geo g, const Inst *D, IOs io, const Rot *rots, int prec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const Inst &I = D[io.inst[blockIdx.z]];
    if (i >= g.next || !(I.terms & 4)) return;
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
    const int64_t o = (int64_t)r * g.next + i;
    if (prec == 0) {
        st2(I.Gr, o, in ? ld2(I.Ghat, idx_I(g, y[0], y[1], y[2])) : make_double2(0.0, 0.0));
    } else {
        const float2 v = in ? ld2f(I.G32, idx_I(g, y[0], y[1], y[2])) : make_float2(0.0f, 0.0f);
        st2f(I.Gr32, o, v);
    }
}

void launch_rotate(const Geo &g, int prec, const Inst *D, const IOs &io, const Rot *rots, int nrot, hipStream_t s) {
    dim3 grid((unsigned)((g.next + 255) / 256), (unsigned)nrot, (unsigned)io.n);
    hipLaunchKernelGGL(rotate_kernel, grid, dim3(256), 0, s, g, D, io, rots, prec);
}

// FP32c: the spectrum rounded to FP32 (round to nearest).
__global__ void spectrum_f32_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const Inst &I = D[io.inst[blockIdx.z]];
    const double2 v = ld2(I.Ghat, i);
    st2f(I.G32, i, make_float2((float)v.x, (float)v.y));
}

void launch_spectrum_f32(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(spectrum_f32_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io);
}

// ---------------------------------------------------------------------------
// Pair sums.  A workgroup of 256 lanes owns 256/ext whole x-rows of outputs
// s at one s0 (s over E_g when the launch has W sums, ext = 2N; over I_N
// otherwise, ext = N).  All lanes walk the same l over the rows' reachable
// box, so G_l is a uniform (scalar) load and, for fixed l, the weights
// w[l][s - l] of the lanes are contiguous runs of the table row of l.  The
// plane m_0 = s_0 - l_0 of the spectrum is staged in LDS for the l_0 it
// serves.  Weights come through a buffer resource over the N table rows of
// one (l_0, l_1): a lane whose m = s - l falls outside I_N gets an offset past
// the end, so that its load returns zero without touching memory.
template <typename T, bool WW, bool CC, bool OTF>
__device__ __forceinline__ void pairs_body(const Geo &g, const typename V2<T>::type *G, const T *wc, const T *wq,
                                           const Radial &rad, typename V2<T>::type *gp, int s0, int s1, int s2,
                                           bool valid, bool do_c, int l0lo, int l0hi, int l1lo, int l1hi,
                                           double2 &accw, double2 &accc) {
    using T2 = typename V2<T>::type;
    const int N = g.N, h = g.h;
    const int64_t nm = g.nm;
    const uint32_t OOB = 0x80000000u;
    for (int l0 = l0lo; l0 <= l0hi; ++l0) {
        const int m0 = s0 - l0;  // in I_N by the choice of the l0 range
        __syncthreads();         // the previous plane is no longer read
        {
            const T2 *Gm = G + idx_I(g, m0, -h, -h);
            for (int i = threadIdx.x; i < N * N; i += blockDim.x) gp[i] = ldT2(Gm, i);
        }
        __syncthreads();
        for (int l1 = l1lo; l1 <= l1hi; ++l1) {
            const int m1 = s1 - l1;
            const bool ok1 = valid && m1 >= -h && m1 < h;
            const int64_t il0 = idx_I(g, l0, l1, -h);  // first of the N table rows of this (l0, l1)
            const int mrow = (int)idx_I(g, m0, ok1 ? m1 : -h, -h);
            const int grow = ((ok1 ? m1 : -h) + h) * N;
            const T2 *Gl = G + il0;
            __amdgpu_buffer_rsrc_t rq, rc;
            if constexpr (WW && !OTF)
                rq = __builtin_amdgcn_make_buffer_rsrc((void *)(wq + il0 * nm), (short)0,
                                                       (int)((int64_t)N * nm * sizeof(T)), 0x00020000);
            if constexpr (CC && !OTF)
                rc = __builtin_amdgcn_make_buffer_rsrc((void *)(wc + il0 * nm), (short)0,
                                                       (int)((int64_t)N * nm * sizeof(T)), 0x00020000);
            // FP64: every term goes straight into the FP64 sums.  FP32c: the
            // N terms of one l-row are summed in FP32, the row sums in FP64.
            T wr = 0, wi = 0, cr = 0, ci = 0;
#pragma unroll 8
            for (int j = 0; j < N; ++j) {
                const int m2 = s2 - (j - h);
                const bool ok = ok1 && m2 >= -h && m2 < h;
                const T2 gl = ld_uniform(Gl, j);  // uniform over the wave
                const T2 gm = gp[grow + (ok ? m2 + h : 0)];
                const uint32_t vo = ok ? (uint32_t)((mrow + m2 + h) * (int)sizeof(T)) : OOB;
                const int so = (int)((int64_t)j * nm * sizeof(T));
                const T2 p = cmulT(gl, gm);
                // weights formed here instead of read (FP64 only)
                double owc = 0.0, owq = 0.0;
                if constexpr (OTF)
                    if (ok) pair_weights(rad, g, l0, l1, j - h, m0, m1, m2, owc, owq);
                if constexpr (WW) {
                    T a1;
                    if constexpr (OTF)
                        a1 = owq;
                    else if constexpr (sizeof(T) == 8)
                        a1 = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rq, vo, so, 0));
                    else
                        a1 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rq, vo, so, 0));
                    if constexpr (sizeof(T) == 8) {
                        accw.x = fma(a1, p.x, accw.x);
                        accw.y = fma(a1, p.y, accw.y);
                    } else {
                        wr = fmaf(a1, p.x, wr);
                        wi = fmaf(a1, p.y, wi);
                    }
                }
                if constexpr (CC) {
                    const uint32_t vc = do_c ? vo : OOB;
                    T a2;
                    if constexpr (OTF)
                        a2 = do_c ? owc : 0.0;
                    else if constexpr (sizeof(T) == 8)
                        a2 = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, vc, so, 0));
                    else
                        a2 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, vc, so, 0));
                    if constexpr (sizeof(T) == 8) {
                        accc.x = fma(a2, p.x, accc.x);
                        accc.y = fma(a2, p.y, accc.y);
                    } else {
                        cr = fmaf(a2, p.x, cr);
                        ci = fmaf(a2, p.y, ci);
                    }
                }
            }
            if constexpr (sizeof(T) == 4) {
                accw.x += wr;
                accw.y += wi;
                accc.x += cr;
                accc.y += ci;
            }
        }
    }
}

template <typename T, bool OTF>
__global__ __launch_bounds__(256) void pairs_kernel(Geo g, const Inst *D, IOs io, const T *wc, const T *wq,
                                                    Radial rad, int ext) {
    extern __shared__ unsigned char pairs_lds[];
    const Inst &I = D[io.inst[blockIdx.z]];
    const int want_c = (I.terms & 1) != 0, want_w = (I.terms & 2) != 0;
    if (!want_c && !want_w) return;
    using T2 = typename V2<T>::type;
    const T2 *G;
    if constexpr (sizeof(T) == 8)
        G = I.Ghat;
    else
        G = I.G32;
    const int N = g.N, h = g.h;
    const int lo = ext == N ? -h : -N;
    const int rows = 256 / ext;  // s1 rows per workgroup
    const int tid = threadIdx.x;
    const int s2 = tid % ext + lo;
    const int r = tid / ext;
    const int s1 = blockIdx.x * rows + r + lo;
    const int K = pair_split(g);
    const int c = (int)blockIdx.y % K;  // slice of the split l axis
    const int s0 = g.d == 3 ? (int)blockIdx.y / K + lo : 0;
    const bool valid = r < rows && s1 < lo + ext;
    const bool inI = valid && s2 >= -h && s2 < h && s1 >= -h && s1 < h && (g.d == 2 || (s0 >= -h && s0 < h));
    // reachable box of l: l and s - l in I_N for some s of the workgroup
    const int s1min = blockIdx.x * rows + lo, s1max = min(s1min + rows - 1, lo + ext - 1);
    // an instance without W sums has nothing to do outside I_N
    if (!want_w && (s1max < -h || s1min >= h || (g.d == 3 && (s0 < -h || s0 >= h)))) return;
    int l0lo = g.d == 3 ? max(-h, s0 - (h - 1)) : 0, l0hi = g.d == 3 ? min(h - 1, s0 + h) : 0;
    int l1lo = max(-h, s1min - (h - 1)), l1hi = min(h - 1, s1max + h);
    {
        // this workgroup's slice [-h + c w, -h + (c + 1) w) of the split axis
        const int wsl = (N + K - 1) / K, clo = -h + c * wsl, chi = clo + wsl - 1;  // the last slices may be empty
        if (g.d == 3) {
            l0lo = max(l0lo, clo);
            l0hi = min(l0hi, chi);
        } else {
            l1lo = max(l1lo, clo);
            l1hi = min(l1hi, chi);
        }
    }
    double2 accw = make_double2(0.0, 0.0), accc = make_double2(0.0, 0.0);
    const bool do_c = want_c && inI;
    T2 *gp = (T2 *)pairs_lds;
    // a wave whose lanes all lie outside I_N issues no classical-weight loads
    const bool wave_c = __builtin_amdgcn_ballot_w64(do_c) != 0;
    if (want_w && wave_c)
        pairs_body<T, true, true, OTF>(g, G, wc, wq, rad, gp, s0, s1, s2, valid, do_c, l0lo, l0hi, l1lo, l1hi, accw, accc);
    else if (want_w)
        pairs_body<T, true, false, OTF>(g, G, wc, wq, rad, gp, s0, s1, s2, valid, do_c, l0lo, l0hi, l1lo, l1hi, accw, accc);
    else
        pairs_body<T, false, true, OTF>(g, G, wc, wq, rad, gp, s0, s1, s2, valid, do_c, l0lo, l0hi, l1lo, l1hi, accw, accc);
    if (!valid) return;
    if (want_w) st2(I.ppart + (int64_t)c * g.neg, idx_E(g, s0, s1, s2), accw);
    if (do_c) st2(I.ppart + (int64_t)K * g.neg + (int64_t)c * g.nm, idx_I(g, s0, s1, s2), accc);
}

// Pair sums for launches with W sums (outputs over E_g), folded along x: lane
// k (0 <= k < N) of an output row owns s_2 = k - N (A) and s_2 = k (B).  At
// step t of the l_2 walk (l_2 = t - N/2) exactly one of them has m_2 = s_2 -
// l_2 in I_N: A while t <= k, B after; in both cases m_2 + N/2 = (k - t) mod
// N.  So every lane of every weight load carries a useful term, where the
// unfolded walk over 2N outputs wastes half of them.  The l_1 range is the
// wave's own (its output rows), the l_0 range the workgroup's.
template <typename T, bool WW, bool CC, bool OTF>
__device__ __forceinline__ void pairs_w_body(const Geo &g, const typename V2<T>::type *G, const T *wc, const T *wq,
                                             const Radial &rad, typename V2<T>::type *gp, int s0, int s1, int k,
                                             bool valid, bool dcA, bool dcB, int l0lo, int l0hi, int l1lo, int l1hi,
                                             double2 (&aw)[2], double2 (&ac)[2]) {
    using T2 = typename V2<T>::type;
    const int N = g.N, h = g.h;
    const int64_t nm = g.nm;
    const uint32_t OOB = 0x80000000u;
    for (int l0 = l0lo; l0 <= l0hi; ++l0) {
        const int m0 = s0 - l0;
        __syncthreads();  // the previous plane is no longer read
        {
            const T2 *Gm = G + idx_I(g, m0, -h, -h);
            for (int i = threadIdx.x; i < N * N; i += blockDim.x) gp[i] = ldT2(Gm, i);
        }
        __syncthreads();
        for (int l1 = l1lo; l1 <= l1hi; ++l1) {
            const int m1 = s1 - l1;
            const bool ok1 = valid && m1 >= -h && m1 < h;
            const int64_t il0 = idx_I(g, l0, l1, -h);
            const int mrow = (int)idx_I(g, m0, ok1 ? m1 : -h, -h);
            const int grow = ((ok1 ? m1 : -h) + h) * N;
            const T2 *Gl = G + il0;
            __amdgpu_buffer_rsrc_t rq, rc;
            if constexpr (WW && !OTF)
                rq = __builtin_amdgcn_make_buffer_rsrc((void *)(wq + il0 * nm), (short)0,
                                                       (int)((int64_t)N * nm * sizeof(T)), 0x00020000);
            if constexpr (CC && !OTF)
                rc = __builtin_amdgcn_make_buffer_rsrc((void *)(wc + il0 * nm), (short)0,
                                                       (int)((int64_t)N * nm * sizeof(T)), 0x00020000);
            // FP32c: the N terms of one l-row in FP32, row sums in FP64
            T wr[2] = {0, 0}, wi[2] = {0, 0}, cr[2] = {0, 0}, ci[2] = {0, 0};
#pragma unroll 8
            for (int t = 0; t < N; ++t) {
                const bool isA = t <= k;
                const int mi = isA ? k - t : k - t + N;
                const T2 gl = ld_uniform(Gl, t);  // uniform over the wave
                const T2 gm = gp[grow + mi];
                const uint32_t vo = ok1 ? (uint32_t)((mrow + mi) * (int)sizeof(T)) : OOB;
                const int so = (int)((int64_t)t * nm * sizeof(T));
                const T2 p = cmulT(gl, gm);
                // weights formed here instead of read (FP64 only)
                double owc = 0.0, owq = 0.0;
                if constexpr (OTF)
                    if (ok1) pair_weights(rad, g, l0, l1, t - h, m0, m1, mi - h, owc, owq);
                if constexpr (WW) {
                    T a;
                    if constexpr (OTF)
                        a = owq;
                    else if constexpr (sizeof(T) == 8)
                        a = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rq, vo, so, 0));
                    else
                        a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rq, vo, so, 0));
                    const T aA = isA ? a : (T)0, aB = isA ? (T)0 : a;
                    if constexpr (sizeof(T) == 8) {
                        aw[0].x = fma(aA, p.x, aw[0].x);
                        aw[0].y = fma(aA, p.y, aw[0].y);
                        aw[1].x = fma(aB, p.x, aw[1].x);
                        aw[1].y = fma(aB, p.y, aw[1].y);
                    } else {
                        wr[0] = fmaf(aA, p.x, wr[0]);
                        wi[0] = fmaf(aA, p.y, wi[0]);
                        wr[1] = fmaf(aB, p.x, wr[1]);
                        wi[1] = fmaf(aB, p.y, wi[1]);
                    }
                }
                if constexpr (CC) {
                    const uint32_t vc = (isA ? dcA : dcB) ? vo : OOB;
                    T a;
                    if constexpr (OTF)
                        a = (isA ? dcA : dcB) ? owc : 0.0;
                    else if constexpr (sizeof(T) == 8)
                        a = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, vc, so, 0));
                    else
                        a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, vc, so, 0));
                    const T aA = isA ? a : (T)0, aB = isA ? (T)0 : a;
                    if constexpr (sizeof(T) == 8) {
                        ac[0].x = fma(aA, p.x, ac[0].x);
                        ac[0].y = fma(aA, p.y, ac[0].y);
                        ac[1].x = fma(aB, p.x, ac[1].x);
                        ac[1].y = fma(aB, p.y, ac[1].y);
                    } else {
                        cr[0] = fmaf(aA, p.x, cr[0]);
                        ci[0] = fmaf(aA, p.y, ci[0]);
                        cr[1] = fmaf(aB, p.x, cr[1]);
                        ci[1] = fmaf(aB, p.y, ci[1]);
                    }
                }
            }
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    aw[e].x += wr[e];
                    aw[e].y += wi[e];
                    ac[e].x += cr[e];
                    ac[e].y += ci[e];
                }
            }
        }
    }
}

template <typename T, bool OTF>
__global__ __launch_bounds__(256) void pairs_w_kernel(Geo g, const Inst *D, IOs io, const T *wc, const T *wq,
                                                      Radial rad) {
    extern __shared__ unsigned char pairs_lds[];
    const Inst &I = D[io.inst[blockIdx.z]];
    const int want_c = (I.terms & 1) != 0, want_w = (I.terms & 2) != 0;
    if (!want_c && !want_w) return;
    using T2 = typename V2<T>::type;
    const T2 *G;
    if constexpr (sizeof(T) == 8)
        G = I.Ghat;
    else
        G = I.G32;
    const int N = g.N, h = g.h;
    const int rows = 256 / N;  // output rows per workgroup, N lanes each
    const int tid = threadIdx.x;
    const int k = tid % N, r = tid / N;
    const int s1 = blockIdx.x * rows + r - N;
    const int K = pair_split(g);
    const int c = (int)blockIdx.y % K;
    const int s0 = g.d == 3 ? (int)blockIdx.y / K - N : 0;
    const bool valid = r < rows && s1 < N;
    const bool rowI = valid && s1 >= -h && s1 < h && (g.d == 2 || (s0 >= -h && s0 < h));
    const bool dcA = want_c && rowI && k >= h, dcB = want_c && rowI && k < h;  // output in I_N
    const int s1min = blockIdx.x * rows - N, s1max = min(s1min + rows - 1, N - 1);
    if (!want_w && (s1max < -h || s1min >= h || (g.d == 3 && (s0 < -h || s0 >= h)))) return;
    int l0lo = g.d == 3 ? max(-h, s0 - (h - 1)) : 0, l0hi = g.d == 3 ? min(h - 1, s0 + h) : 0;
    // the wave's own output rows
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
    const int ws1min = s1min + wv * 64 / N, ws1max = min(s1min + (wv * 64 + 63) / N, s1max);
    int l1lo = max(-h, ws1min - (h - 1)), l1hi = min(h - 1, ws1max + h);
    {
        const int wsl = (N + K - 1) / K, clo = -h + c * wsl, chi = clo + wsl - 1;
        if (g.d == 3) {
            l0lo = max(l0lo, clo);
            l0hi = min(l0hi, chi);
        } else {
            l1lo = max(l1lo, clo);
            l1hi = min(l1hi, chi);
        }
    }
    double2 aw[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    double2 ac[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    T2 *gp = (T2 *)pairs_lds;
    const bool wave_c = __builtin_amdgcn_ballot_w64(dcA || dcB) != 0;
    if (want_w && wave_c)
        pairs_w_body<T, true, true, OTF>(g, G, wc, wq, rad, gp, s0, s1, k, valid, dcA, dcB, l0lo, l0hi, l1lo, l1hi, aw, ac);
    else if (want_w)
        pairs_w_body<T, true, false, OTF>(g, G, wc, wq, rad, gp, s0, s1, k, valid, dcA, dcB, l0lo, l0hi, l1lo, l1hi, aw, ac);
    else
        pairs_w_body<T, false, true, OTF>(g, G, wc, wq, rad, gp, s0, s1, k, valid, dcA, dcB, l0lo, l0hi, l1lo, l1hi, aw, ac);
    if (!valid) return;
    const int s2[2] = {k - N, k};
    if (want_w)
        for (int e = 0; e < 2; ++e) st2(I.ppart + (int64_t)c * g.neg, idx_E(g, s0, s1, s2[e]), aw[e]);
    double2 *qp = I.ppart + (int64_t)K * g.neg + (int64_t)c * g.nm;
    if (dcA) st2(qp, idx_I(g, s0, s1, s2[0]), ac[0]);
    if (dcB) st2(qp, idx_I(g, s0, s1, s2[1]), ac[1]);
}

// W and Qc as the sums of the slices, in slice order.
__global__ void pairs_reduce_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = D[io.inst[blockIdx.z]];
    const int K = pair_split(g);
    if ((I.terms & 2) && i < g.neg) {
        double2 a = make_double2(0.0, 0.0);
        for (int c = 0; c < K; ++c) {
            const double2 v = ld2(I.ppart + (int64_t)c * g.neg, i);
            a.x += v.x;
            a.y += v.y;
        }
        st2(I.W, i, a);
    }
    if ((I.terms & 1) && i < g.nm) {
        double2 a = make_double2(0.0, 0.0);
        for (int c = 0; c < K; ++c) {
            const double2 v = ld2(I.ppart + (int64_t)K * g.neg + (int64_t)c * g.nm, i);
            a.x += v.x;
            a.y += v.y;
        }
        st2(I.Qc, i, a);
    }
}

void launch_pairs_reduce(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(pairs_reduce_kernel, dim3((unsigned)((g.neg + 255) / 256), 1, (unsigned)io.n), dim3(256), 0,
                       s, g, D, io);
}

void launch_pairs(const Geo &g, int prec, const Inst *D, const IOs &io, const void *wc, const void *wq, int w_any,
                  const Radial *otf, hipStream_t s) {
    const int N = g.N;
    const size_t lds = (size_t)N * N * (prec == 0 ? sizeof(double2) : sizeof(float2));  // one m_0 plane of G
    const Radial rad = otf ? *otf : Radial{};
    if (w_any) {
        // outputs over E_g, x folded: N lanes per output row
        const int rows = 256 / N;
        dim3 grid((unsigned)((2 * N + rows - 1) / rows), (unsigned)((g.d == 3 ? 2 * N : 1) * pair_split(g)),
                  (unsigned)io.n);
        if (prec == 0 && otf)
            hipLaunchKernelGGL((pairs_w_kernel<double, true>), grid, dim3(256), lds, s, g, D, io, (const double *)wc,
                               (const double *)wq, rad);
        else if (prec == 0)
            hipLaunchKernelGGL((pairs_w_kernel<double, false>), grid, dim3(256), lds, s, g, D, io, (const double *)wc,
                               (const double *)wq, rad);
        else
            hipLaunchKernelGGL((pairs_w_kernel<float, false>), grid, dim3(256), lds, s, g, D, io, (const float *)wc,
                               (const float *)wq, rad);
        return;
    }
    const int ext = N;
    const int rows = 256 / ext;
    dim3 grid((unsigned)((ext + rows - 1) / rows), (unsigned)((g.d == 3 ? ext : 1) * pair_split(g)), (unsigned)io.n);
    if (prec == 0 && otf)
        hipLaunchKernelGGL((pairs_kernel<double, true>), grid, dim3(256), lds, s, g, D, io, (const double *)wc,
                           (const double *)wq, rad, ext);
    else if (prec == 0)
        hipLaunchKernelGGL((pairs_kernel<double, false>), grid, dim3(256), lds, s, g, D, io, (const double *)wc,
                           (const double *)wq, rad, ext);
    else
        hipLaunchKernelGGL((pairs_kernel<float, false>), grid, dim3(256), lds, s, g, D, io, (const float *)wc,
                           (const float *)wq, rad, ext);
}

// ---------------------------------------------------------------------------
// Outer sum X_n = sum_k G_k W_{n-k}; n - k always lies in Eg.  A lane owns 4
// consecutive outputs along x and walks k_2 in blocks of 4: block b needs
// W at x-offsets c_b - 4 .. c_b + 3 (c_b = n_2 + N/2 - 4b), of which the upper
// half is the previous block's lower half, so each loaded W value serves 4
// outputs.  G_k is uniform across the wave (scalar loads).  The k box is split
// into slices along k_0 (3-D) or k_1 (2-D), one workgroup per slice and
// partial array, added in slice order by outer_reduce_kernel.
__device__ __forceinline__ void outer_macs(double2 (&acc)[4], double2 gk, const double2 (&lo)[4],
                                           const double2 (&hi)[4], int jj) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 w = i - jj >= 0 ? hi[i - jj] : lo[i - jj + 4];
        acc[i].x = fma(gk.x, w.x, fma(-gk.y, w.y, acc[i].x));
        acc[i].y = fma(gk.x, w.y, fma(gk.y, w.x, acc[i].y));
    }
}

__global__ __launch_bounds__(256) void outer_kernel(Geo g, const Inst *D, IOs io) {
    const Inst &I = D[io.inst[blockIdx.z]];
    if (!(I.terms & 2)) return;
    const int N = g.N, h = g.h, nq = (N + 3) / 4;  // x-quads per row
    const int64_t rowsq = (int64_t)(g.d == 3 ? N : 1) * N * nq;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = outer_split(g), c = blockIdx.y;
    const int wsl = (N + K - 1) / K;
    const bool valid = q < rowsq;
    const int64_t qq = valid ? q : 0;
    const int n2a = (int)(qq % nq) * 4 - h, n1 = (int)((qq / nq) % N) - h;
    const int n0 = g.d == 3 ? (int)(qq / ((int64_t)nq * N)) - h : 0;
    const double2 *G = I.Ghat, *W = I.W;
    double2 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = make_double2(0.0, 0.0);
    // slice of the split axis
    int k0lo = g.d == 3 ? -h : 0, k0hi = g.d == 3 ? h - 1 : 0, k1lo = -h, k1hi = h - 1;
    if (g.d == 3) {
        k0lo = -h + c * wsl;
        k0hi = min(h - 1, k0lo + wsl - 1);
    } else {
        k1lo = -h + c * wsl;
        k1hi = min(h - 1, k1lo + wsl - 1);
    }
    const int E = 2 * N;
    const int nb = N / 4;  // full blocks of 4 k_2
    for (int k0 = k0lo; k0 <= k0hi; ++k0)
        for (int k1 = k1lo; k1 <= k1hi; ++k1) {
            const double2 *Grow = G + idx_I(g, k0, k1, -h);
            const double2 *Wrow = W + idx_E(g, n0 - k0, n1 - k1, -N);  // x-offset x at Wrow[x + N]
            // W at x-offset c_b + e, clamped into the row (clamped values only
            // reach outputs past the window, which are not stored)
            auto wat = [&](int x) { return ld2(Wrow, min(max(x, -N), N - 1) + N); };
            const int c0 = n2a + h;
            double2 A[4], B[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) A[e] = wat(c0 + e);
            int b = 0;
            for (; b + 1 < nb; b += 2) {
                const int cb = c0 - 4 * b;
#pragma unroll
                for (int e = 0; e < 4; ++e) B[e] = wat(cb - 4 + e);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) outer_macs(acc, ld2(Grow, 4 * b + jj), B, A, jj);
#pragma unroll
                for (int e = 0; e < 4; ++e) A[e] = wat(cb - 8 + e);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) outer_macs(acc, ld2(Grow, 4 * b + 4 + jj), A, B, jj);
            }
            // an odd last block and the last N mod 4 values of k_2
            for (int t = 4 * b; t < N; ++t) {
                const double2 gk = ld2(Grow, t);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double2 w = wat(c0 + i - t);
                    acc[i].x = fma(gk.x, w.x, fma(-gk.y, w.y, acc[i].x));
                    acc[i].y = fma(gk.x, w.y, fma(gk.y, w.x, acc[i].y));
                }
            }
            (void)E;
        }
    if (!valid) return;
    double2 *part = I.xpart + (int64_t)c * g.nm;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (n2a + i < h) st2(part, idx_I(g, n0, n1, n2a + i), acc[i]);
}

__global__ void outer_reduce_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = D[io.inst[blockIdx.z]];
    if (i >= g.nm || !(I.terms & 2)) return;
    double2 a = make_double2(0.0, 0.0);
    for (int c = 0; c < outer_split(g); ++c) {
        const double2 v = ld2(I.xpart + (int64_t)c * g.nm, i);
        a.x += v.x;
        a.y += v.y;
    }
    st2(I.X, i, a);
}

void launch_outer(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    const int64_t rowsq = (int64_t)(g.d == 3 ? g.N : 1) * g.N * ((g.N + 3) / 4);
    hipLaunchKernelGGL(outer_kernel, dim3((unsigned)((rowsq + 255) / 256), (unsigned)outer_split(g), (unsigned)io.n),
                       dim3(256), 0, s, g, D, io);
    hipLaunchKernelGGL(outer_reduce_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io);
}

// ---------------------------------------------------------------------------
// Trilinear sum: FP64 in t1_pairs.hip (vector units), FP32c in t1_mfma.hip
// (matrix cores, 4 partial arrays per workgroup).
void launch_trilinear(int prec, int Nmax, int nslots, const int *lo, const int *hi, const T1Item *items,
                      const Inst *D, int nq, int *qctr, hipStream_t s) {
    if (prec == 0)
        launch_t1_pairs(nslots, lo, hi, items, D, nq, qctr, s);
    else
        launch_t1_mfma(Nmax, nslots / T1M_WAVES, lo, hi, items, D, nq, qctr, s);
}

int trilinear_blocks_per_cu(int prec, int N) { return prec == 0 ? t1_pairs_blocks_per_cu() : t1_mfma_blocks_per_cu(N); }

__global__ void zero_kernel(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void launch_zero(void *p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 8;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, s, (double *)p, n);
}

// Partial arrays of the instances that evaluate the trilinear term.
__global__ void zero_part_kernel(Geo g, const Inst *D, IOs io) {
    const Inst &I = D[io.inst[blockIdx.z]];
    if (!(I.terms & 4)) return;
    const int64_t n = (int64_t)I.nslots * g.nm * 2;
    const gptr<double> p = glob((double *)I.part);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void launch_zero_part(const Geo &g, const Inst *D, const IOs &io, int max_slots, hipStream_t s) {
    const int64_t n = (int64_t)max_slots * g.nm * 2;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_part_kernel, dim3(nb, 1, (unsigned)io.n), dim3(256), 0, s, g, D, io);
}

// Trilinear partial arrays -> T1, in two passes with a fixed order.  Pass 1:
// a workgroup sums one chunk of consecutive slots for 64 outputs (4 slot
// phases per output, combined in LDS in phase order) and leaves the sum in
// the chunk's first slot; pass 2 adds the chunk sums in chunk order.  The
// chunks spread the slots over enough workgroups to fill the device also
// when N^d is small.
constexpr int RP_OUT = 64, RP_PH = 4;

__global__ void __launch_bounds__(RP_OUT * RP_PH) reduce_chunks_kernel(Geo g, const Inst *D, IOs io, int chunk) {
    const Inst &I = D[io.inst[blockIdx.z]];
    const int s0 = blockIdx.y * chunk;
    if (!(I.terms & 4) || s0 >= I.nslots) return;  // uniform over the workgroup
    const int lane = threadIdx.x % RP_OUT, ph = threadIdx.x / RP_OUT;
    const int64_t i = (int64_t)blockIdx.x * RP_OUT + lane;
    const int s1 = min(I.nslots, s0 + chunk);
    double re = 0.0, im = 0.0;
    if (i < g.nm)
        for (int s = s0 + ph; s < s1; s += RP_PH) {
            const double2 v = ld2(I.part, (int64_t)s * g.nm + i);
            re += v.x;
            im += v.y;
        }
    __shared__ double2 red[RP_PH][RP_OUT];
    red[ph][lane] = make_double2(re, im);
    __syncthreads();
    if (ph == 0 && i < g.nm) {
        for (int q = 1; q < RP_PH; ++q) {
            re += red[q][lane].x;
            im += red[q][lane].y;
        }
        st2(I.part, (int64_t)s0 * g.nm + i, make_double2(re, im));
    }
}

__global__ void reduce_final_kernel(Geo g, const Inst *D, IOs io, int chunk) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = D[io.inst[blockIdx.z]];
    if (i >= g.nm || !(I.terms & 4)) return;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < I.nslots; s += chunk) {
        const double2 v = ld2(I.part, (int64_t)s * g.nm + i);
        re += v.x;
        im += v.y;
    }
    st2(I.T1, i, make_double2(re, im));
}

void launch_reduce_partials(const Geo &g, const Inst *D, const IOs &io, int max_slots, hipStream_t s) {
    if (max_slots < 1) return;
    const int64_t bx = (g.nm + RP_OUT - 1) / RP_OUT;
    const int64_t want = std::max<int64_t>(1, (1024 + bx - 1) / bx);  // chunks for >= 1024 workgroups
    const int nch = (int)std::min<int64_t>(want, std::max(1, max_slots / (2 * RP_PH)));
    const int chunk = (max_slots + nch - 1) / nch;
    const int ny = (max_slots + chunk - 1) / chunk;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)bx, (unsigned)ny, (unsigned)io.n), dim3(RP_OUT * RP_PH), 0,
                       s, g, D, io, chunk);
    hipLaunchKernelGGL(reduce_final_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io, chunk);
}

// Qhat = [Qc] - alpha ([T1] + [X]) with the selected terms; optionally the
// real part of the n = 0 mode is removed (exact discrete mass conservation).
__global__ void combine_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    const int terms = I.terms;
    double re = 0.0, im = 0.0;
    if (terms & 1) {
        const double2 v = ld2(I.Qc, i);
        re = v.x;
        im = v.y;
    }
    double qr = 0.0, qi = 0.0;
    if (terms & 4) {
        const double2 v = ld2(I.T1, i);
        qr += v.x;
        qi += v.y;
    }
    if (terms & 2) {
        const double2 v = ld2(I.X, i);
        qr += v.x;
        qi += v.y;
    }
    re -= I.alpha * qr;
    im -= I.alpha * qi;
    if (I.mass_fix && i == idx_I(g, 0, 0, 0)) re = 0.0;
    st2(I.Qh, i, make_double2(re, im));
    if (io.qhat[z]) st2(io.qhat[z], i, make_double2(re, im));
}

void launch_combine(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io);
}

}  // namespace bnq
