// Internal declarations shared by the host runtime and the HIP kernels of
// libbnq.  Not part of the public ABI (see include/bnq.h).
//
// Geometry.  A d-dimensional mode grid is stored as 3-D with axis 0 trivial
// (extent 1, mode 0) when d = 2.  Axis 2 is the fastest (C order).
//   I_N   : modes {-N/2 .. N/2-1} per axis, storage index k + N/2
//   Eg    : pair sums l + m live in {-N .. N-1} per axis (2N values; the top
//           value N-1 is never reached, which lets the outer sum read W at
//           n - k without bounds checks), storage index s + N
//   A     : trilinear kernel-mode rows, arguments {-(N-1) .. N-1} per axis.
//           A row is stored [a0][a2][a1] (axis 1 fastest, so that lanes that
//           own consecutive y read consecutive addresses); axis 2 (x) is
//           padded with zeros by KPADLO below and KPADHI above, which lets
//           the trilinear kernel's sliding window run past the window edges
//           without clamping.
//   Ext   : rotated spectra, modes {-N/2 .. N/2} per axis (N+1 values),
//           storage index q + N/2
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bnq.h"

namespace bnq {

struct Geo {
    int d, N, h;
    int e0;       // extent of axis 0 in I_N (1 or N)
    int lo0;      // lowest mode of axis 0 (0 or -N/2)
    int64_t nm;   // |I_N| = N^d
    int eg0;      // extent of axis 0 in Eg (1 or 2N)
    int64_t neg;  // |Eg|
    int ea0;      // extent of axis 0 in A (1 or 2N-1)
    int64_t na;   // |A|
    int kax;      // padded x extent of a stored row (2N-1 + KPADLO + KPADHI)
    int64_t nak;  // stored row length ea0 * kax * (2N-1)
    int ex0;      // extent of axis 0 in Ext (1 or N+1)
    int64_t next; // |Ext|
    int psplit;   // slices of the l box of the pair sums (1 .. pair_split_max), chosen per plan
};

__host__ __device__ inline int64_t idx_I(const Geo &g, int k0, int k1, int k2) {
    return ((int64_t)(k0 - g.lo0) * g.N + (k1 + g.h)) * g.N + (k2 + g.h);
}
__host__ __device__ inline int64_t idx_E(const Geo &g, int s0, int s1, int s2) {
    const int E = 2 * g.N;
    return ((int64_t)(g.d == 3 ? s0 + g.N : 0) * E + (s1 + g.N)) * E + (s2 + g.N);
}
__host__ __device__ inline int64_t idx_A(const Geo &g, int a0, int a1, int a2) {
    const int A = 2 * g.N - 1;
    return ((int64_t)(g.d == 3 ? a0 + g.N - 1 : 0) * A + (a1 + g.N - 1)) * A + (a2 + g.N - 1);
}
constexpr int KPADLO = 16, KPADHI = 8;
// offset of a = (a0, a1, a2) inside a stored trilinear row
__host__ __device__ inline int64_t idx_K(const Geo &g, int a0, int a1, int a2) {
    const int A = 2 * g.N - 1;
    return ((int64_t)(g.d == 3 ? a0 + g.N - 1 : 0) * g.kax + (a2 + g.N - 1 + KPADLO)) * A + (a1 + g.N - 1);
}
// offset of a inside a stored trilinear row of the x-fastest layout (the FP32
// rows, read by the matrix-core trilinear kernel): [a0][a1][a2 + pad], x
// padded as in idx_K
__host__ __device__ inline int64_t idx_Kx(const Geo &g, int a0, int a1, int a2) {
    const int A = 2 * g.N - 1;
    return ((int64_t)(g.d == 3 ? a0 + g.N - 1 : 0) * A + (a1 + g.N - 1)) * g.kax + (a2 + g.N - 1 + KPADLO);
}
__host__ __device__ inline int64_t idx_X(const Geo &g, int q0, int q1, int q2) {
    const int X = g.N + 1;
    return ((int64_t)(g.d == 3 ? q0 + g.h : 0) * X + (q1 + g.h)) * X + (q2 + g.h);
}

// Signed axis permutation: (R x)_i = sgn[i] * x[perm[i]].
struct Rot {
    int perm[3];
    int sgn[3];
};

// Per-b description for the trilinear sum in the rotated frame of b = R b_c.
struct T1B {
    int kc;          // row of the trilinear kernel-mode table (canonical b_c)
    int rot;         // index of R
    int bc[3];       // canonical b_c (components >= 0)
    int wnlo[3], wnhi[3];  // output window in the rotated frame
    int wplo[3], wphi[3];  // inner window in the rotated frame
    int nxb;         // x-blocks of the output window
    int pad;         // outputs per x-block (6, 7 or 8; always 8 for FP32c)
};

// A group of the matrix-core trilinear sum: the b = R b_c (canonical row kc)
// whose rotated frames share the lower edge of the x window (3-D), or all of
// them (2-D); outputs n' and inner modes p' run over the union of the
// members' windows (first value and length per rotated axis).
struct T1G {
    int kc;
    int bc[3];
    int wn0[3], wnl[3];
    int wp0[3], wpl[3];
    int nrot;
    int rot[24];
};

struct T1Item {
    int b;     // index into the T1B array
    int t0;    // first task
    int nt;    // number of tasks (<= 64)
    int inst;  // instance (index into the launch's Inst array)
    int slot;  // static schedule: the item's list in its instance's own plan,
               // which names the partial arrays it adds into (the list may
               // run on another workgroup in a batch); unused when dynamic
};

constexpr int T1_RB = 8;      // outputs per lane along x

// Radial tables for the kernel-mode series.
struct Radial {
    const double *J;     // [qmax+1][M] radial integrals of even order 2m
    const int *mcut;     // [qmax+1] last order index needed for |a|^2 = q
    const double *coef;  // [M] series coefficients (include C_phi)
    const double *lrA;   // [2M] Legendre recurrence constants (2n+1)/(n+1)
    const double *lrB;   // [2M] n/(n+1)
    const double *bdiag; // [qmax+1] beta(a, a) for |a|^2 = q (the series at x = 1)
    int M;
    int d;
};

// Kernel-mode series value for |a|^2 = qa, |b|^2 = qb, |a.b| = dab.  Not
// inlined, so that every kernel that forms kernel modes (the tables, and the
// pair sums that form their weights on the fly) runs the same code.
[[maybe_unused]] static __device__ __noinline__ double beta_series(const Radial &rad, int qa, int qb, double dab) {
    const int mc = min(rad.mcut[qa], rad.mcut[qb]);
    double x = 1.0;
    if (qa > 0 && qb > 0) x = fmin(1.0, dab / sqrt((double)qa * (double)qb));
    const double *Ja = rad.J + (int64_t)qa * rad.M;
    const double *Jb = rad.J + (int64_t)qb * rad.M;
    double sum = rad.coef[0] * (Ja[0] * Jb[0]);
    // (pm, p) = (P_{2m-2}, P_{2m-1}); Legendre (3-D) or Chebyshev (2-D)
    double pm = 1.0, p = x;
    for (int m = 1; m <= mc; ++m) {
        const int n = 2 * m - 1;
        const double p2 = rad.d == 3 ? rad.lrA[n] * x * p - rad.lrB[n] * pm : 2.0 * x * p - pm;
        sum += rad.coef[m] * (Ja[m] * Jb[m]) * p2;
        const double p3 = rad.d == 3 ? rad.lrA[n + 1] * x * p2 - rad.lrB[n + 1] * p : 2.0 * x * p2 - p;
        pm = p2;
        p = p3;
    }
    return sum;
}

// Pair weights of modes l, m in I_N:
//   wc = beta(l,m) - beta(m,m)  where l + m is in I_N, else 0
//   wq = beta(l,m) - beta(l+m,l) - beta(l,l+m)
[[maybe_unused]] static __device__ __noinline__ void pair_weights(const Radial &rad, const Geo &g, int l0, int l1, int l2, int m0,
                                                 int m1, int m2, double &wc, double &wq) {
    const int s0 = l0 + m0, s1 = l1 + m1, s2 = l2 + m2;
    const int ql = l0 * l0 + l1 * l1 + l2 * l2;
    const int qm = m0 * m0 + m1 * m1 + m2 * m2;
    const int qs = s0 * s0 + s1 * s1 + s2 * s2;
    const double blm = beta_series(rad, ql, qm, (double)abs(l0 * m0 + l1 * m1 + l2 * m2));
    const double bmm = rad.bdiag[qm];
    // beta(l+m, l) = beta(l, l+m): the series is symmetric in its arguments,
    // bit for bit (products of the two radial factors commute)
    const double bsl = beta_series(rad, qs, ql, (double)abs(s0 * l0 + s1 * l1 + s2 * l2));
    const double bls = bsl;
    const int hi = g.h - 1, lo = -g.h;
    const bool inI = s1 >= lo && s1 <= hi && s2 >= lo && s2 <= hi && (g.d == 2 || (s0 >= lo && s0 <= hi));
    wc = inI ? blm - bmm : 0.0;
    wq = blm - bsl - bls;
}

// Pointers read from memory (the Inst and IOs tables) are generic; kernels
// convert them to the global address space so that their accesses compile to
// global (not flat) memory instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__host__ __device__ __forceinline__ gptr<T> glob(T *p) {
    return (gptr<T>)p;
}
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld2(const double2 *p, int64_t i) {
    const dvec2 v = ((gptr<const dvec2>)p)[i];
    return make_double2(v.x, v.y);
}
typedef float fvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld2f(const float2 *p, int64_t i) {
    const fvec2 v = ((gptr<const fvec2>)p)[i];
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2f(float2 *p, int64_t i, float2 a) {
    fvec2 v;
    v.x = a.x;
    v.y = a.y;
    ((gptr<fvec2>)p)[i] = v;
}
__device__ __forceinline__ void st2(double2 *p, int64_t i, double2 a) {
    dvec2 v;
    v.x = a.x;
    v.y = a.y;
    ((gptr<dvec2>)p)[i] = v;
}

// complex products; FP64 / FP32 element types of the trilinear kernels
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

template <typename T>
struct V2;
template <>
struct V2<double> {
    using type = double2;
};
template <>
struct V2<float> {
    using type = float2;
};

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cmulT(double2 a, double2 b) { return cmul(a, b); }
__device__ __forceinline__ float2 cmulT(float2 a, float2 b) { return cmulf(a, b); }
__device__ __forceinline__ double2 ldT2(const double2 *p, int64_t i) { return ld2(p, i); }
__device__ __forceinline__ float2 ldT2(const float2 *p, int64_t i) { return ld2f(p, i); }
// A load through the constant address space: with a wave-uniform address it
// becomes a scalar load (the value lands in scalar registers and costs no
// vector memory instruction).  Only for data no kernel writes while the
// reading kernel runs.
__device__ __forceinline__ double2 ld_uniform(const double2 *p, int64_t i) {
    const __attribute__((address_space(4))) double *q = (const __attribute__((address_space(4))) double *)p;
    return make_double2(q[2 * i], q[2 * i + 1]);
}
__device__ __forceinline__ float2 ld_uniform(const float2 *p, int64_t i) {
    const __attribute__((address_space(4))) float *q = (const __attribute__((address_space(4))) float *)p;
    return make_float2(q[2 * i], q[2 * i + 1]);
}
// A geometry or a pointer held in device memory, read the same way.
__device__ __forceinline__ Geo ld_uniform_geo(const Geo *p) {
    typedef const __attribute__((address_space(4))) Geo CGeo;
    const CGeo *q = (const CGeo *)p;
    Geo g;
    g.d = q->d;
    g.N = q->N;
    g.h = q->h;
    g.e0 = q->e0;
    g.lo0 = q->lo0;
    g.nm = q->nm;
    g.eg0 = q->eg0;
    g.neg = q->neg;
    g.ea0 = q->ea0;
    g.na = q->na;
    g.kax = q->kax;
    g.nak = q->nak;
    g.ex0 = q->ex0;
    g.next = q->next;
    g.psplit = q->psplit;
    return g;
}
template <typename T>
__device__ __forceinline__ T *ld_uniform_ptr(T *const *p) {
    typedef T *const __attribute__((address_space(4))) CP;
    return *(CP *)p;
}


// ---- instances --------------------------------------------------------------
// Every evaluation kernel runs over a set of instances that share the geometry
// and the tables (one plan alone, or a batch group); blockIdx.z (or the work
// item) selects the instance.
constexpr int BNQ_MAXB = 64;  // instances per launch

// Workspace of one instance (device memory, fixed for the plan's lifetime).
// The pair sums split the l box of every output into psplit slices along l_0
// (3-D) or l_1 (2-D), one workgroup and partial array each, added in slice
// order: the l-chunking of these sums.  The workspace holds pair_split_max
// slices, so a plan can take any count up to it.
__host__ __device__ inline int pair_split(const Geo &g) { return g.psplit; }
__host__ __device__ inline int pair_split_max(int N) { return N < 32 ? N : 32; }
// default: 32 slices for the classical sums alone (eps = 0), 16 with W sums
// (measured at 3-D N = 32: 0.94 / 0.97 / 1.03 ms at 32 / 16 / 8 slices for
// eps = 0; 3.45 / 3.44 / 3.60 ms with W sums)
__host__ __device__ inline int pair_split_default(int d, int N, int eps) {
    const int k = (d == 3 && eps == 0) ? 32 : 16;
    return N < k ? N : k;
}

// The outer sum likewise splits its k box into this many slices (k_0 in 3-D,
// k_1 in 2-D).
__host__ __device__ inline int outer_split(const Geo &g) { return g.N < 16 ? g.N : 16; }

struct Inst {
    double2 *Ghat, *tmp, *tmp2, *Gr, *W, *Qc, *T1, *X, *Qh, *part;
    double2 *xpart;  // outer-sum partials: outer_split(g) arrays over I_N
    double2 *ppart;  // pair-sum partials: pair_split(g) arrays over E_g (W), then as many over I_N (Qc)
    float2 *G32, *Gr32;  // FP32c: rounded spectrum and rotated spectra
    double *ybuf, *k[4];
    double alpha;  // -eps hbar^d
    double pref;   // c (L/pi)^(d+gamma)
    int terms;     // BNQ_T_* mask actually evaluated
    int mass_fix;  // 1: Re Qhat_0 := 0
    int nslots;    // trilinear partial arrays in part
    int corr_mom;  // 1: project Q onto zero mass, momentum and energy
    double hstep;  // velocity step 2 L / N
    const double *ginv;  // inverse Gram matrix of {1, v, |v|^2} over the grid, (d+2)^2
    // health of the state written by the last stage of a step: two flag
    // words in host-visible memory ([0] a non-finite value, [1] a value at or
    // above fbound), set by the device, read and cleared by the host
    int *health;
    double fbound;  // 1/alpha for Fermi-Dirac statistics (alpha > 0), else +inf
    // The instance's geometry, tables and trilinear work descriptors, read by
    // the trilinear kernels per work item, so that one launch can serve
    // instances of different (d, N).
    Geo geo;
    const void *K;      // kernel-mode rows: double (FP64) or float (FP32c)
    const void *t1d;    // work descriptors: T1B (FP64) or T1G (FP32c)
    const Rot *rots;    // the rotations the descriptors index
};

// Buffers a kernel can be pointed at.
enum BufSel { BUF_IN = 0, BUF_OUT, BUF_TMP, BUF_TMP2, BUF_GHAT, BUF_QH, BUF_Y, BUF_K0 };

// Per-call pointers, passed by value: instance z of a launch is Inst[inst[z]],
// reads grid values from in[z] and writes them to out[z].
struct IOs {
    const double *in[BNQ_MAXB];
    double *out[BNQ_MAXB];
    double2 *qhat[BNQ_MAXB];  // optional copy of Qhat (may be NULL)
    double dt[BNQ_MAXB];
    int inst[BNQ_MAXB];
    int n;
};

// ---- launchers (defined in the .hip files) --------------------------------
void launch_radial(int d, double R, int qmax, int M, int nq, const double *glx, const double *glw,
                   double *S, double *J, hipStream_t s);
// tables in FP64 or FP32 (values formed in FP64, rounded to nearest)
void launch_beta_rows(const Geo &g, const Radial &rad, const int *canon, int ncanon, double *K,
                      hipStream_t s);
void launch_beta_rows(const Geo &g, const Radial &rad, const int *canon, int ncanon, float *K, hipStream_t s);
void launch_weights(const Geo &g, const Radial &rad, double *wc, double *wq, hipStream_t s);
void launch_weights(const Geo &g, const Radial &rad, float *wc, float *wq, hipStream_t s);
void launch_gather(const double *base, const int64_t *idx, int64_t n, double *out, hipStream_t s);
void launch_gather(const float *base, const int64_t *idx, int64_t n, double *out, hipStream_t s);
// trilinear term by the separated-kernel transform route, d = 2 (t1_separated.hip)
bool sep_supported(int d, int N);
int sep_auto_angles(int N, double R);
int sep_directions(int d, int angles);  // P: the angle count in 2-D, M1 M2 = 2 angles^2 in 3-D
void sep_shape(int d, int N, int P, int *nc, int *jc, int *nbj);
hipError_t sep_prepare();
void launch_sep_tables(int d, int N, int angles, double R, double Cphi, double *al, double *alp, double2 *gc,
                       hipStream_t s);
void launch_sep_t1(int d, int N, int P, const double2 *Ghat, const double2 *gc, double2 *gt, double2 *part,
                   double2 *T1, hipStream_t s);
void launch_beta_diag(const Radial &rad, int qmax, double *out, hipStream_t s);
void launch_pair_weights_at(const Geo &g, const Radial &rad, const int64_t *idx, int64_t n, int which, double *out,
                            hipStream_t s);

// DFT of grid values io.in -> Ghat (forward, scale N^-d) and Qh -> io.out
// (inverse, real part, scale Inst::pref).
void launch_dft_forward_real(const Geo &g, const Inst *D, const IOs &io, const double2 *tw, hipStream_t s);
void launch_inverse_real(const Geo &g, const Inst *D, const IOs &io, const double2 *tw, hipStream_t s);
// prec 0: FP64; 1: FP32c (spectra and tables rounded to FP32, sums combined in FP64)
void launch_spectrum_f32(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
void launch_rotate(const Geo &g, int prec, const Inst *D, const IOs &io, const Rot *rots, int nrot, hipStream_t s);
void launch_pairs_reduce(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
// w_any: some instance of the launch needs the W pair sums; otf (FP64 only):
// form the pair weights from these radial tables instead of reading wc, wq
void launch_pairs(const Geo &g, int prec, const Inst *D, const IOs &io, const void *wc, const void *wq, int w_any,
                  const Radial *otf, hipStream_t s);
void launch_outer(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
void launch_zero_part(const Geo &g, const Inst *D, const IOs &io, int max_slots, hipStream_t s);
// Trilinear sum over the item ranges [lo[i], hi[i]) of the nslots slots
// (static, nq = 0) or of the nq queues (dynamic tickets, nq > 0).  An item
// names its instance in D, whose geometry, kernel-mode rows and descriptors
// (Inst::geo, K, t1d, rots) it uses: the instances of one launch may differ
// in (d, N).  prec 0: FP64 (double rows); 1: FP32c (float rows, spectra
// Inst::Gr32, the matrix-core kernel for rows of at most N + 1 inner values:
// every instance of the launch has N <= Nmax, and Nmax selects the kernel,
// see t1_mfma_class).
void launch_trilinear(int prec, int Nmax, int nslots, const int *lo, const int *hi, const T1Item *items,
                      const Inst *D, int nq, int *qctr, hipStream_t s);
void launch_t1_pairs(int nslots, const int *lo, const int *hi, const T1Item *items, const Inst *D, int nq,
                     int *qctr, hipStream_t s);
// FP32c: matrix-core kernel, nwg workgroups of T1M_WAVES waves, partial array
// T1M_WAVES wg + wave
void launch_t1_mfma(int Nmax, int nwg, const int *lo, const int *hi, const T1Item *items, const Inst *D, int nq,
                    int *qctr, hipStream_t s);
// the matrix-core kernel variant that serves N (instances of one launch must
// share it: the variants differ in LDS, hence in resident workgroups)
int t1_mfma_class(int N);
int t1_pairs_blocks_per_cu();
int t1_mfma_blocks_per_cu(int N);
constexpr int T1M_WAVES = 8;     // waves (partial arrays) per matrix-core workgroup
constexpr int T1M_BLOCK = 128;   // outputs of a matrix-core item
constexpr int T1M_KLINE = 1536;  // kernel-mode values a matrix-core item stages per inner row (LDS floats)
int trilinear_blocks_per_cu(int prec, int N);  // resident trilinear workgroups per CU (0 on error)
void launch_zero(void *p, int64_t bytes, hipStream_t s);
void launch_reduce_partials(const Geo &g, const Inst *D, const IOs &io, int max_slots, hipStream_t s);
void launch_combine(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
void launch_moments_fix(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);

// Stage updates: y = in + a dt k[ks] into Inst::ybuf (to_out = 0) or into
// io.out (to_out = 1); the final RK4 / SSP-RK2 combinations update io.out.
void launch_stage(const Geo &g, const Inst *D, const IOs &io, double a, int ks, int to_out, hipStream_t s);
void launch_rk4_final(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
void launch_ssprk2_final(const Geo &g, const Inst *D, const IOs &io, hipStream_t s);
// Moments of grid values f on [-L, L)^d: two passes over nblk workgroups with
// fixed reduction trees; res receives MOM_OUT values: rho, u[3], E_c, e, H,
// max f, min f, excluded + non-finite nodes, non-finite nodes (the order of
// bnq_moments, plus the non-finite count).  scratch holds
// moments_scratch_doubles(nblk) doubles; the raw first-pass totals (sum f,
// sum v f per storage axis, sum |v|^2 f, ...) end at moments_sums_offset.
constexpr int MOM_BLOCKS = 256;
constexpr int MOM_FIELDS = 12;
constexpr int MOM_OUT = 11;
constexpr size_t moments_sums_offset(int nblk) { return (size_t)nblk * (MOM_FIELDS + 1); }
constexpr size_t moments_scratch_doubles(int nblk) { return moments_sums_offset(nblk) + MOM_FIELDS; }
void launch_moments(const Geo &g, const double *f, double L, double alpha, double *scratch, int nblk, double *res,
                    hipStream_t s);
// Allocation-free entry point: a static device array of this many doubles
// per device (step.hip), and its address on the current device.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = 4096;
static_assert(moments_scratch_doubles(MOM_BLOCKS) <= NOALLOC_SCRATCH_DOUBLES, "moment partials fit the static scratch");
hipError_t noalloc_scratch(double **out);

// A limit state on the grid (kinds as BNQ_EQ_*): M(v) with r2 = |v - u|^2
//   kind 0: c0 exp(-r2 / 2T)                       (c0 = rho (2 pi T)^(-d/2))
//   kind 1, 2: c0 / (exp(r2 / 2T - log_z) + sgn)   (c0 = 1/|alpha|; sgn = -1
//              uses expm1, and a zero denominator marks the node excluded)
//   kind 3: c0 for r2 <= A2, else 0                (c0 = rho / |D(u, A)|)
struct EqDev {
    int kind, d, bose;
    double c0, u[3], log_z, T, A2;
};
// out_fill (if non-NULL) <- M on the grid (0 at excluded nodes); if f is
// non-NULL, part/out receive sum |f - M|, max |f - M|, sum M, excluded
// nodes, sum f over them (unscaled sums)
void launch_equilibrium(const Geo &g, double L, const EqDev &q, const double *f, double *out_fill, double *part,
                        int nblk, double *out, hipStream_t s);
constexpr int EQ_FIELDS = 5;

// out = G + dt (K - div_xi((A xi - B) G)) on the xi grid (B per storage axis),
// the divergence through the N x N real spectral differentiation matrix D
void launch_drift_update(const Geo &g, const double *G, const double *K, const double *D, double A,
                         const double *B3, double dt, double *out, hipStream_t s);
void launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);

// host: ln K_nu (FD p = ln z, BE p = -ln z) and the limit-state solve
double complete_fd_be_log(double nu, int fermi, double p);
int solve_equilibrium(int d, double alpha, double rho, const double *u, double e, bnq_equilibrium *out, char *err,
                      size_t errlen);

}  // namespace bnq
