// Trilinear sum T1 of the Galerkin operator (section 'Fast spectral
// approximation of the BNE operator', the Q_{1,q} term) on the matrix cores,
// FP32c precision pattern: FP32 kernel modes and pair products, FP32 products
// summed by the matrix core over eight inner rows, FP64 totals.
//
// For a canonical b_c and the rotations R of a group (the b = R b_c whose
// rotated frames share the lower edge of the x window), the sum over the
// inner modes is a real Toeplitz matrix times a complex one:
//     Y_R(n') = sum_{p'} K(n' - p') P_R(p'),   K(a) = beta(a, b_c),
//     P_R(p') = G(R p') G(R (b_c - p')),
// with one K shared by every rotation and one P_R shared by every output:
//     Y[n', (R, re/im)] = sum_{p'} A[n', p'] B[p', (R, re/im)],
//     A[n', p'] = K(n' - p').
// The outputs n' and inner modes p' run over the union of the group's
// windows (a mode outside one rotation's own window meets a zero P_R, or an
// output that is not written).  Then T1(R n') += G(R (n' - b_c)) Y_R(n').
//
// A workgroup of 8 waves takes an item (group, block of 128 outputs n' in the
// flattened window, x fastest); each wave owns one tile of 16 outputs and up
// to 3 tiles of 16 columns (8 rotations x re/im), and adds its results into
// its own partial array.  The item names its instance, whose geometry, rows
// and descriptors it uses, so one launch can serve instances of different
// (d, N) (of one kernel variant).  Inner rows (p'_y, p'_z) are walked in order.  For
// every row the workgroup stages in LDS, while the previous row runs on the
// matrix cores,
//   - the pair products of the row (one p'_x and rotation per thread, from
//     the rotated spectra), in the matrix core's B fragment layout;
//   - the kernel-mode values the block's outputs meet in that row: for each
//     x-line of outputs in the block, K(a) along a_x over every n'_x - p'_x,
//     from the x-fastest kernel-mode row.
// Each lane then reads its A values from LDS at fixed offsets.
// v_mfma_f32_16x16x4_f32 lane layout: A[i][k] and B[k][j] in lane i + 16 k
// (resp. j + 16 k), the result D[4 (l / 16) + r][l % 16] in register r of
// lane l.
#include "bnq_internal.h"

namespace bnq {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int MW = 8;                 // waves per workgroup
constexpr int MTL = 1;                // output tiles of 16 per wave
constexpr int NTH = 64 * MW;          // threads per workgroup
constexpr int MBLK = MW * MTL * 16;   // outputs per item
static_assert(MBLK == T1M_BLOCK && MW == T1M_WAVES, "item shape known to the host");
constexpr int NTM = 3;                // column tiles of 16 (8 rotations) per item
constexpr int EPS = MTL * 16 + 2;     // epilogue row stride (doubles; the wave's outputs + 2 against bank conflicts)
constexpr int EPW = 16 * EPS;         // epilogue doubles per wave (16 columns)

// A pointer that is the same in every lane, read from memory that the kernel
// also writes: the compiler cannot see that it is uniform, and a buffer
// resource built from it would make every buffer load a loop over lanes.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void decode(const T1G &G, int m, int &n0, int &n1, int &n2) {
    n2 = G.wn0[2] + m % G.wnl[2];
    const int q = m / G.wnl[2];
    n1 = G.wn0[1] + q % G.wnl[1];
    n0 = G.wn0[0] + q / G.wnl[1];
}

// Pair-product staging.  The B fragment (s, t) of a row (k-step s, column
// tile t) is 64 floats: column 16 t + j at inner offset 4 s + k in float
// k * 16 + j; rotation r fills columns 2 r (re) and 2 r + 1 (im), so a
// fragment is 32 complex values, (k, r mod 8) at float2 k * 8 + r mod 8.
// Thread tid stages, in slot q, the pair e = tid + NTH q: fragment f = e / 16
// (fragments numbered s * NT + t), entries (2 k2, r8) and (2 k2 + 1, r8) with
// k2 = (e / 8) mod 2 and r8 = e mod 8, i.e. inner offsets u and u + 1
// (u = 4 s + 2 k2) of rotation r = 8 t + r8.  Each spectrum factor of the
// pair comes with one 16-byte load of two consecutive values.  Entries past
// the row or past the group's rotations are zeros, so every entry of the
// row's fragments is written.
template <int NP>
struct PStage {
    int rbase[NP];  // float2 offset of the slot's rotated spectrum, -1: zero
    int u[NP];      // inner offset p'_x - wp0_x of the pair's first entry
    int sidx[NP];   // float2 index of the first entry in the fragment buffer, -1: not staged
    int lim[NP];    // entries of the pair inside the row: 0, 1 or 2
};
template <int NP>
struct PVals {
    f4v x[NP], y[NP];  // the spectrum values, multiplied when stored
};

// byte offset past every buffer: a load there returns zero
constexpr int OOB = 0x7ffffff0;

template <int NP>
__device__ __forceinline__ void pstage_setup(const Geo &g, const T1G &G, int KS, int NT, int tid, PStage<NP> &S) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int e = tid + NTH * q;
        const int f = e >> 4, k2 = (e >> 3) & 1, r8 = e & 7;
        const int s = NT == 1 ? f : (NT == 2 ? f >> 1 : (f * 21846) >> 16);  // f / NT for f < 3 * 64
        const int t = f - s * NT;
        const int r = 8 * t + r8, u = 4 * s + 2 * k2;
        S.sidx[q] = s < KS ? f * 32 + 16 * k2 + r8 : -1;
        S.u[q] = u;
        const int lim = (s < KS && r < G.nrot) ? min(max(G.wpl[2] - u, 0), 2) : 0;
        S.lim[q] = lim;
        S.rbase[q] = lim > 0 ? (int)(G.rot[r] * g.next) : -1;
    }
}

// hp, hq: float2 offsets of p' = (pz, py, wp0_x) and of b_c - p' in a
// rotated spectrum; the pair (u, u + 1) of slot q reads G_r(p' + u e_x),
// G_r(p' + (u + 1) e_x) (in range: p' + u lies in I_N, so p' + (u + 1) e_x
// lies in the stored {-N/2..N/2}) and G_r(b_c - p' - u e_x) with its
// neighbour: G_r(b_c - p' - (u + 1) e_x) when both entries are in the row
// (that mode is then in I_N), else G_r(b_c - p' - (u - 1) e_x), which is in
// the stored range as well.  Nothing waits for the loads here.
template <int NP>
__device__ __forceinline__ void pstage_load(__amdgpu_buffer_rsrc_t gr, int hp, int hq, const PStage<NP> &S,
                                            PVals<NP> &V) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int b = S.rbase[q];
        const int ox = b >= 0 ? 8 * (b + hp + S.u[q]) : OOB;
        const int oy = b >= 0 ? 8 * (b + hq - S.u[q] - (S.lim[q] == 2 ? 1 : 0)) : OOB;
        V.x[q] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(gr, ox, 0, 0));
        V.y[q] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(gr, oy, 0, 0));
    }
}

template <int NP>
__device__ __forceinline__ void pstage_store(const PStage<NP> &S, const PVals<NP> &V, float *bs) {
#pragma unroll
    for (int q = 0; q < NP; ++q)
        if (S.sidx[q] >= 0) {
            const f4v x = V.x[q], y = V.y[q];
            const bool two = S.lim[q] == 2;
            // y holds (y_{u+1}, y_u) when both entries are in the row, else (y_u, y_{u-1})
            const float2 yu = two ? make_float2(y[2], y[3]) : make_float2(y[0], y[1]);
            const float2 p0 = S.lim[q] > 0 ? cmulf(make_float2(x[0], x[1]), yu) : make_float2(0.0f, 0.0f);
            const float2 p1 = two ? cmulf(make_float2(x[2], x[3]), make_float2(y[0], y[1])) : make_float2(0.0f, 0.0f);
            float2 *b2 = reinterpret_cast<float2 *>(bs);
            b2[S.sidx[q]] = p0;
            b2[S.sidx[q] + 8] = p1;
        }
}

// Kernel-mode staging.  The block's outputs cover nl x-lines; line l holds
// K(a) for a = (nz - pz, ny - py, ax0 + x), x < lw, at float l * lw4 + x
// (lw4: lw rounded up to a multiple of 4), with lw = (window x length) +
// 4 KS - 1 and ax0 = wn0_x - wp0_x - 4 KS + 1: every n'_x - p'_x of the line
// and of the row (a_y, a_z clamped into the row: a clamped value only meets a
// zero pair product or an output that is not written).  A thread stages 4
// consecutive values of a line with one 16-byte load and one 16-byte LDS
// store (the padding values past lw are never read); T1M_KLINE <= 4 NTH, so
// one slot per thread, and the waves past the block's lines issue nothing.
constexpr int KSL = (T1M_KLINE / 4 + NTH - 1) / NTH;
static_assert(T1M_KLINE % 4 == 0 && KSL == 1, "one 16-byte kernel-mode slot per thread");
struct KStage {
    int ny[KSL], nz[KSL];  // the slot's output line
    int ax[KSL];           // a_x of its first value, -1000: not staged
};
struct KVals {
    f4v v[KSL];
};

__device__ __forceinline__ void kstage_setup(const T1G &G, int l0, int nl, int lw4, int ax0, int tid, KStage &S) {
#pragma unroll
    for (int q = 0; q < KSL; ++q) {
        const int e = 4 * (tid + NTH * q);
        const int l = e / lw4, x = e - l * lw4;
        const int L = l0 + l;
        S.ny[q] = G.wn0[1] + L % G.wnl[1];
        S.nz[q] = G.wn0[0] + L / G.wnl[1];
        S.ax[q] = e < nl * lw4 ? ax0 + x : -1000;
    }
}

__device__ __forceinline__ void kstage_load(const Geo &g, __amdgpu_buffer_rsrc_t kr, int pz, int py, const KStage &S,
                                            KVals &V) {
    const int N1 = g.N - 1;
#pragma unroll
    for (int q = 0; q < KSL; ++q) {
        const int a0 = g.d == 3 ? min(max(S.nz[q] - pz, -N1), N1) : 0;
        const int a1 = min(max(S.ny[q] - py, -N1), N1);
        const int off = S.ax[q] > -1000 ? 4 * (int)idx_Kx(g, a0, a1, S.ax[q]) : OOB;
        V.v[q] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(kr, off, 0, 0));
    }
}

__device__ __forceinline__ void kstage_store(const KStage &S, const KVals &V, int tid, float *kl) {
#pragma unroll
    for (int q = 0; q < KSL; ++q)
        if (S.ax[q] > -1000) reinterpret_cast<f4v *>(kl)[tid + NTH * q] = V.v[q];
}

// The rows and the epilogue of one item with NT column tiles.  KSM: k-steps
// of 4 inner values per row the instantiation holds (a row has at most N + 1
// inner values); buf: 2 row buffers of RB floats.
template <int KSM, int NT>
__device__ __forceinline__ void t1m_item(const Geo &g, const T1G &G, const Inst &I, const float *K, const Rot *rots,
                                         int t0, int wg, float *buf) {
    constexpr int BF = KSM * NTM * 64;       // B fragment floats of a row
    constexpr int RB = BF + T1M_KLINE;       // row buffer floats
    constexpr int NP = (KSM * NT * 16 + NTH - 1) / NTH;  // entry pairs per thread (16 per fragment)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    // the descriptor fields the rows use, uniform and in scalar registers
    // (re-read from memory they would cost a wait per row)
    auto rfl = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    const int wpl0 = rfl(G.wpl[0]), wpl1 = rfl(G.wpl[1]), wpl2 = rfl(G.wpl[2]);
    const int wp00 = rfl(G.wp0[0]), wp01 = rfl(G.wp0[1]), px0 = rfl(G.wp0[2]);
    const int c0 = rfl(G.bc[0]), c1 = rfl(G.bc[1]), c2 = rfl(G.bc[2]);
    const int nrot = rfl(G.nrot);
    const int W = rfl(G.wnl[0] * G.wnl[1] * G.wnl[2]);
    const int KS = (wpl2 + 3) >> 2;
    const int nrows = wpl0 * wpl1;
    const int lnx = rfl(G.wnl[2]);
    const int m0 = t0 * MBLK;
    const int l0 = m0 / lnx;
    const int nlines = (min(m0 + MBLK, W) - 1) / lnx - l0 + 1;
    const int lw4 = (lnx + 4 * KS - 1 + 3) & ~3;
    const int ax0 = rfl(G.wn0[2]) - px0 - 4 * KS + 1;
    const int mbase = m0 + wave * (MTL * 16);
    // this lane's A values: K line of its output, at x - u + 4 KS - 1
    int abase[MTL];
#pragma unroll
    for (int tm = 0; tm < MTL; ++tm) {
        const int m = min(mbase + tm * 16 + li, W - 1);
        abase[tm] = (m / lnx - l0) * lw4 + m % lnx + 4 * KS - 1 - lk;
    }
    const int kc = __builtin_amdgcn_readfirstlane(G.kc);
    const __amdgpu_buffer_rsrc_t kr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(K + (int64_t)kc * g.nak), (short)0, (int)(g.nak * (int64_t)sizeof(float)), 0x00020000);
    const __amdgpu_buffer_rsrc_t gr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(I.Gr32), (short)0, (int)((g.d == 3 ? 48 : 8) * g.next * (int64_t)sizeof(float2)),
        0x00020000);
    const int X = g.N + 1, h = g.h, d3 = g.d == 3;
    auto hp_of = [&](int pz, int py) { return ((d3 ? pz + h : 0) * X + (py + h)) * X + h + px0; };
    auto hq_of = [&](int pz, int py) { return ((d3 ? c0 - pz + h : 0) * X + (c1 - py + h)) * X + (c2 - px0 + h); };
    f4v acc[MTL][NT];
    double z[MTL][NT][4];
#pragma unroll
    for (int tm = 0; tm < MTL; ++tm)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[tm][t] = (f4v){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < 4; ++r) z[tm][t][r] = 0.0;
        }
    PStage<NP> ps;
    KStage ks;
    PVals<NP> pv;
    KVals kv;
    pstage_setup(g, G, KS, NT, tid, ps);
    kstage_setup(G, l0, nlines, lw4, ax0, tid, ks);
    __syncthreads();  // the previous item's epilogue is done with the buffers
    pstage_load(gr, hp_of(wp00, wp01), hq_of(wp00, wp01), ps, pv);
    kstage_load(g, kr, wp00, wp01, ks, kv);
    pstage_store(ps, pv, buf);
    kstage_store(ks, kv, tid, buf + BF);
    __syncthreads();
    int cur = 0;
    int pyi = 0, pzi = 0;
    for (int row = 0; row < nrows; ++row) {
        const bool more = row + 1 < nrows;
        const int npyi = pyi + 1 < wpl1 ? pyi + 1 : 0;
        const int npzi = pyi + 1 < wpl1 ? pzi : pzi + 1;
        // the next row's pair products and kernel-mode values are fetched
        // while this row runs on the matrix cores
        if (more) {
            const int pz = wp00 + npzi, py = wp01 + npyi;
            pstage_load(gr, hp_of(pz, py), hq_of(pz, py), ps, pv);
            kstage_load(g, kr, pz, py, ks, kv);
        }
        const float *bf = buf + cur * RB;
        const float *kl = bf + BF;
        // operands in chunks of three k-steps (entries past the row are
        // finite values of the buffer that no matrix product uses); the
        // waves issue them at raised priority, so that a wave with matrix
        // products to issue goes before the other waves' staging
        // instructions (529.7 against 537.0 ms per evaluation at 3-D N=32)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s0 = 0; s0 < KSM; s0 += 3) {
            if (s0 < KS) {
                float av[MTL][3], bv[NT][3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
#pragma unroll
                    for (int tm = 0; tm < MTL; ++tm) av[tm][j] = kl[abase[tm] - 4 * (s0 + j)];
#pragma unroll
                    for (int t = 0; t < NT; ++t) bv[t][j] = bf[((s0 + j) * NT + t) * 64 + lane];
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (s0 + j < KS) {
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int tm = 0; tm < MTL; ++tm) acc[tm][t] = mfma4(av[tm][j], bv[t][j], acc[tm][t]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // FP64 totals of the FP32 sums of every eight rows (at most 32 KS
        // terms each)
        if ((row & 7) == 7 || !more) {
#pragma unroll
            for (int tm = 0; tm < MTL; ++tm)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) z[tm][t][r] += (double)acc[tm][t][r];
                    acc[tm][t] = (f4v){0.0f, 0.0f, 0.0f, 0.0f};
                }
        }
        if (more) {
            float *nb = buf + (cur ^ 1) * RB;
            pstage_store(ps, pv, nb);
            kstage_store(ks, kv, tid, nb + BF);
        }
        __syncthreads();
        cur ^= 1;
        pyi = npyi;
        pzi = npzi;
    }
    // Epilogue, one column tile at a time: the wave's results go through LDS
    // ([column][output]) so that in each round all lanes hold one rotation:
    // distinct outputs n' map to distinct modes R n' and the
    // read-modify-writes of a round never meet.
    double *ep = reinterpret_cast<double *>(buf) + wave * EPW;
    double2 *mypart = I.part + (int64_t)(wg * MW + wave) * g.nm;
    const int m = mbase + lane;
    int n0 = 0, n1 = 0, n2 = 0;
    if (lane < MTL * 16 && m < W) decode(G, m, n0, n1, n2);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        __syncthreads();
#pragma unroll
        for (int tm = 0; tm < MTL; ++tm)
#pragma unroll
            for (int r = 0; r < 4; ++r) ep[li * EPS + tm * 16 + 4 * lk + r] = z[tm][t][r];
        __syncthreads();
        for (int qq = 0; qq < 8; ++qq) {
            const int rr = 8 * t + qq;
            if (rr >= nrot) break;
            if (lane < MTL * 16 && m < W) {
                const Rot R = rots[G.rot[rr]];
                const int v[3] = {n0, n1, n2};
                const int o0 = R.sgn[0] * v[R.perm[0]];
                const int o1 = R.sgn[1] * v[R.perm[1]];
                const int o2 = R.sgn[2] * v[R.perm[2]];
                const bool in = o1 >= -h && o1 < h && o2 >= -h && o2 < h && (g.d == 2 || (o0 >= -h && o0 < h));
                if (in) {
                    const float2 gq =
                        ld2f(I.Gr32 + (int64_t)G.rot[rr] * g.next, idx_X(g, n0 - c0, n1 - c1, n2 - c2));
                    const double yr = ep[(2 * qq) * EPS + lane], yi = ep[(2 * qq + 1) * EPS + lane];
                    const double2 cc = cmul(make_double2(gq.x, gq.y), make_double2(yr, yi));
                    const int64_t o = idx_I(g, o0, o1, o2);
                    double2 cv = ld2(mypart, o);
                    cv.x += cc.x;
                    cv.y += cc.y;
                    st2(mypart, o, cv);
                }
            }
            // the next round may read back modes written in this one
            __threadfence_block();
        }
    }
}

template <int KSM>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4, 4))) void t1_mfma_kernel(const int *lo, const int *hi, const T1Item *items,
                                                      const Inst *D, int nq, int *qctr) {
    constexpr int RB = KSM * NTM * 64 + T1M_KLINE;
    static_assert(2 * RB >= 2 * MW * EPW, "epilogue fits the row buffers");
    __shared__ __align__(16) float buf[2 * RB];
    __shared__ int tick;
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    int it = nq ? -1 : lo[wg] - 1;
    const int it_end = nq ? 0 : hi[wg];
    int q = nq ? (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % (unsigned)nq) : 0;
    int qseen = 0;
    for (;;) {
        if (nq == 0) {
            if (++it >= it_end) break;
        } else {
            int got = -1;
            while (qseen < nq) {
                __syncthreads();
                if (tid == 0) tick = atomicAdd(qctr + q, 1);
                __syncthreads();
                const int tk = __builtin_amdgcn_readfirstlane(tick);
                if (tk < hi[q] - lo[q]) {
                    got = lo[q] + tk;
                    break;
                }
                ++qseen;
                q = q + 1 == nq ? 0 : q + 1;
            }
            if (got < 0) break;
            it = got;
        }
        // the item is the same for the whole workgroup; saying so keeps its
        // descriptors and buffer resources in scalar registers (otherwise
        // every buffer load becomes a loop over lanes)
        it = __builtin_amdgcn_readfirstlane(it);
        const T1Item item = items[it];
        const Inst &I = D[item.inst];
        // the instance's geometry, rows and descriptors: scalar loads (no
        // kernel writes the instance table during the launch)
        const Geo g = ld_uniform_geo(&I.geo);
        const float *K = (const float *)ld_uniform_ptr(&I.K);
        const Rot *rots = ld_uniform_ptr(&I.rots);
        const T1G &G = ((const T1G *)ld_uniform_ptr(&I.t1d))[item.b];
        const int NT = (2 * G.nrot + 15) >> 4;
        // the workgroup whose partial arrays the item adds into: static, the
        // item's own list; dynamic, this one
        const int pw = nq ? wg : __builtin_amdgcn_readfirstlane(item.slot);
        if (NT == 3)
            t1m_item<KSM, 3>(g, G, I, K, rots, item.t0, pw, buf);
        else if (NT == 2)
            t1m_item<KSM, 2>(g, G, I, K, rots, item.t0, pw, buf);
        else
            t1m_item<KSM, 1>(g, G, I, K, rots, item.t0, pw, buf);
    }
}

template <int KSM>
int blocks_per_cu() {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, t1_mfma_kernel<KSM>, NTH, 0) == hipSuccess ? nb : 0;
}

}  // namespace

// rows hold at most N + 1 inner values: k-steps of 4 per row
int t1_mfma_class(int N) { return N <= 34 ? 9 : (N <= 50 ? 13 : 17); }

void launch_t1_mfma(int Nmax, int nwg, const int *lo, const int *hi, const T1Item *items, const Inst *D, int nq,
                    int *qctr, hipStream_t s) {
    switch (t1_mfma_class(Nmax)) {
        case 9: hipLaunchKernelGGL(t1_mfma_kernel<9>, dim3(nwg), dim3(NTH), 0, s, lo, hi, items, D, nq, qctr); break;
        case 13: hipLaunchKernelGGL(t1_mfma_kernel<13>, dim3(nwg), dim3(NTH), 0, s, lo, hi, items, D, nq, qctr); break;
        default: hipLaunchKernelGGL(t1_mfma_kernel<17>, dim3(nwg), dim3(NTH), 0, s, lo, hi, items, D, nq, qctr); break;
    }
}

int t1_mfma_blocks_per_cu(int N) {
    const int c = t1_mfma_class(N);
    return c == 9 ? blocks_per_cu<9>() : (c == 13 ? blocks_per_cu<13>() : blocks_per_cu<17>());
}

}  // namespace bnq
