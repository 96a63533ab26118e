// Trilinear sum T1 of the Galerkin operator, FP32c precision pattern (section
// 'Fast spectral approximation of the BNE operator'): one inner row at a time.
#include "bnq_internal.h"

namespace bnq {
namespace {

// ---------------------------------------------------------------------------
// Trilinear sum.  One 64-lane workgroup per slot; each slot walks its static
// list of items (b, range of <= 64 tasks) and accumulates into its own
// partial array (no atomics; the slots are summed in a fixed order later).
//
// A task is 8 consecutive outputs along x at one (y, z); tasks are numbered
// y fastest so that the lanes of a wave read consecutive addresses of the
// y-fastest kernel-mode rows.  For every inner row (py, pz) a lane slides a
// 16-value window K(a_x), a_x = base + i - u, over the inner index u in blocks
// of 8: block k uses lo_k[s] = K(base - 8k - 8 + s) and hi_k[s] =
// K(base - 8k + s) = lo_{k-1}[s].  Four 8-value arrays rotate (at compile
// time: the number of full blocks is a template parameter) so that the values
// of block k + 2 are loaded while block k computes, and the next row's first
// three arrays are loaded at the start of the current row.
//
// Kernel-mode values come through a buffer resource over the canonical row:
// one 32-bit lane offset per window, the 8 values of a window at scalar
// offsets s * 8A.  The pair products of a row are uniform across the wave:
// the next row's are formed (one p_x per lane, from the rotated spectrum)
// while the current row computes, then written to a two-row LDS ring and read
// as broadcasts.
template <typename T>
struct T1Ctx {
    __amdgpu_buffer_rsrc_t kr;         // canonical kernel-mode row
    int voff;                          // byte offset of K(a_x = base) at this row's (a_z, a_y)
    int sA;                            // bytes between consecutive a_x
    const typename V2<T>::type *ps;    // LDS: pair products of the current row
};

template <typename T>
__device__ __forceinline__ T t1_kload(const T1Ctx<T> &c, int voff, int s) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(c.kr, voff, s * c.sA, 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(c.kr, voff, s * c.sA, 0));
}

// Block K of a row: lo_K = K(base - 8K - 8 + s), hi_K = lo_{K-1}; issues the
// loads of lo_{K+2} into nx (two blocks ahead) when PF.
template <typename T, int K, bool PF>
__device__ __forceinline__ void t1_full(const T1Ctx<T> &c, const T (&lo)[8], const T (&hi)[8], T (&nx)[8],
                                        T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    if constexpr (PF) {
        const int vq = c.voff - (8 * (K + 2) + 8) * c.sA;
#pragma unroll
        for (int s = 0; s < 8; ++s) nx[s] = t1_kload(c, vq, s);
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        const auto p = c.ps[8 * K + jj];
#pragma unroll
        for (int i = 0; i < T1_RB; ++i) {
            const T k = (i - jj < 0) ? lo[i - jj + 8] : hi[i - jj];
            zr[i] = fma(k, p.x, zr[i]);
            zi[i] = fma(k, p.y, zi[i]);
        }
    }
}

template <typename T, int R>
__device__ __forceinline__ void t1_tail_n(const T1Ctx<T> &c, int u0, const T (&lo)[8], const T (&hi)[8],
                                          T (&zr)[T1_RB], T (&zi)[T1_RB]) {
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
        const auto p = c.ps[u0 + jj];
#pragma unroll
        for (int i = 0; i < T1_RB; ++i) {
            const T k = (i - jj < 0) ? lo[i - jj + 8] : hi[i - jj];
            zr[i] = fma(k, p.x, zr[i]);
            zi[i] = fma(k, p.y, zi[i]);
        }
    }
}

// The last rem (< 8) inner values of a row, straight-line code per rem.
template <typename T>
__device__ __forceinline__ void t1_tail(const T1Ctx<T> &c, int u0, int rem, const T (&lo)[8], const T (&hi)[8],
                                        T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    switch (rem) {
        case 1: t1_tail_n<T, 1>(c, u0, lo, hi, zr, zi); break;
        case 2: t1_tail_n<T, 2>(c, u0, lo, hi, zr, zi); break;
        case 3: t1_tail_n<T, 3>(c, u0, lo, hi, zr, zi); break;
        case 4: t1_tail_n<T, 4>(c, u0, lo, hi, zr, zi); break;
        case 5: t1_tail_n<T, 5>(c, u0, lo, hi, zr, zi); break;
        case 6: t1_tail_n<T, 6>(c, u0, lo, hi, zr, zi); break;
        case 7: t1_tail_n<T, 7>(c, u0, lo, hi, zr, zi); break;
        default: break;
    }
}

// Blocks K .. NF-1 of a row, then the tail, over a four-slot ring: lo_j
// lives in R[(j + 1) % 4] (R[0] = hi_0 = lo_{-1}, R[1] = lo_0, R[2] = lo_1 on
// entry); block K reads R[(K + 1) % 4] and R[K % 4] and refills R[(K + 3) % 4]
// with lo_{K+2}, needed two blocks later.
template <typename T, int NF, int K>
__device__ __forceinline__ void t1_blocks(const T1Ctx<T> &c, int rem, T (&R)[4][8], T (&zr)[T1_RB],
                                          T (&zi)[T1_RB]) {
    if constexpr (K < NF) {
        t1_full<T, K, (K + 2 <= NF)>(c, R[(K + 1) % 4], R[K % 4], R[(K + 3) % 4], zr, zi);
        t1_blocks<T, NF, K + 1>(c, rem, R, zr, zi);
    } else {
        t1_tail<T>(c, 8 * K, rem, R[(K + 1) % 4], R[K % 4], zr, zi);
    }
}

// the first three ring slots of a row whose window offset is v
template <typename T>
__device__ __forceinline__ void t1_ring_start(const T1Ctx<T> &c, int v, T (&R)[4][8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        R[0][s] = t1_kload(c, v, s);
        R[1][s] = t1_kload(c, v - 8 * c.sA, s);
        R[2][s] = t1_kload(c, v - 16 * c.sA, s);
    }
}

// Walks the inner rows in (pz, py) order; the window offset of a row drops
// by one value per py step (a_y = ny - py) and by one a_z plane per pz step.
struct T1Rows {
    int voff, py, pz, wpy, dz, dy;  // current offset, (py, pz) indices in the window; byte steps
    __device__ __forceinline__ int next() const { return py + 1 < wpy ? voff - dy : voff - dz + (wpy - 1) * dy; }
    __device__ __forceinline__ void advance(bool more) {
        const int vn = next();
        const bool wrap = py + 1 >= wpy;
        voff = more ? vn : voff;
        pz = more && wrap ? pz + 1 : pz;
        py = more ? (wrap ? 0 : py + 1) : py;
    }
};

// Pair products P_b(p) = G_R(p) G_R(b_c - p) of the inner window, formed on
// the fly from the rotated spectrum (one lane per p_x of a row).
template <typename T>
struct T1Pairs {
    using T2 = typename V2<T>::type;
    const T2 *G;     // rotated spectrum G_R on {-N/2 .. N/2}^d
    int X, h, d3;    // N + 1, N / 2, d == 3
    int px, qx;      // storage x-indices of p_x and b_c,x - p_x for this lane
    int bz, by;      // b_c,z and b_c,y
    int pzlo, pylo;  // inner window start
    __device__ __forceinline__ T2 at(int pzi, int pyi) const {
        const int pz = pzlo + pzi, py = pylo + pyi;
        const int64_t ip = ((int64_t)(d3 ? pz + h : 0) * X + (py + h)) * X + px;
        const int64_t iq = ((int64_t)(d3 ? bz - pz + h : 0) * X + (by - py + h)) * X + qx;
        return cmulT(ldT2(G, ip), ldT2(G, iq));
    }
};

// One inner row: compute it from the ring R and the staged pair products
// ps[cur], while the next row's first ring slots (into Rn) and pair products
// are fetched.  Past the last row the fetches repeat the last row's
// addresses and the staged pair products are zero, so that rows can run in
// pairs without branches (an odd row count ends with one row that adds
// nothing).
template <typename T, int NF>
__device__ __forceinline__ void t1_row(T1Ctx<T> &c, T1Rows &rw, int row, int nrows, int wpx, int lane,
                                       const T1Pairs<T> &pr, typename V2<T>::type (*ps)[64], int cur, T (&R)[4][8],
                                       T (&Rn)[4][8], T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    const bool more = row + 1 < nrows;
    const int vn = more ? rw.next() : rw.voff;
    const bool wrap = rw.py + 1 >= rw.wpy;
    const int npy = more ? (wrap ? 0 : rw.py + 1) : rw.py;
    const int npz = more && wrap ? rw.pz + 1 : rw.pz;
    const auto pn = pr.at(npz, npy);
    t1_ring_start(c, vn, Rn);
    c.voff = rw.voff;
    c.ps = ps[cur];
    t1_blocks<T, NF, 0>(c, wpx - 8 * NF, R, zr, zi);
    __syncthreads();
    const bool keep = more && lane < wpx;
    ps[cur ^ 1][lane].x = keep ? pn.x : (T)0;
    ps[cur ^ 1][lane].y = keep ? pn.y : (T)0;
    __syncthreads();
    rw.advance(more);
}

// All inner rows of an item.  FP64 accumulates every row in zr/zi; FP32
// accumulates a pair of rows (at most 128 terms per output) in FP32 and adds
// it to the FP64 totals Zr/Zi.
template <typename T, int NF>
__device__ __forceinline__ void t1_rows(T1Ctx<T> &c, T1Rows rw, int nrows, int wpx, int lane, const T1Pairs<T> &pr,
                                        typename V2<T>::type (*ps)[64], double (&Zr)[T1_RB], double (&Zi)[T1_RB]) {
    T RA[4][8], RB[4][8];
    T zr[T1_RB], zi[T1_RB];
#pragma unroll
    for (int i = 0; i < T1_RB; ++i) zr[i] = zi[i] = (T)0;
    t1_ring_start(c, rw.voff, RA);
    {
        const auto p0 = pr.at(0, 0);
        const bool keep = lane < wpx;
        ps[0][lane].x = keep ? p0.x : (T)0;
        ps[0][lane].y = keep ? p0.y : (T)0;
    }
    __syncthreads();
    for (int row = 0; row < nrows; row += 2) {
        t1_row<T, NF>(c, rw, row, nrows, wpx, lane, pr, ps, 0, RA, RB, zr, zi);
        t1_row<T, NF>(c, rw, row + 1, nrows, wpx, lane, pr, ps, 1, RB, RA, zr, zi);
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int i = 0; i < T1_RB; ++i) {
                Zr[i] += (double)zr[i];
                Zi[i] += (double)zi[i];
                zr[i] = zi[i] = 0.0f;
            }
        }
    }
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int i = 0; i < T1_RB; ++i) {
            Zr[i] = zr[i];
            Zi[i] = zi[i];
        }
    }
}

template <typename T>
__device__ __forceinline__ const typename V2<T>::type *rotated_of(const Inst &I) {
    if constexpr (sizeof(T) == 8)
        return I.Gr;
    else
        return I.Gr32;
}

// Static schedule (nq = 0): slot blockIdx.x walks items[lo[slot] ..
// hi[slot]).  Dynamic schedule (nq > 0): the items are nq queues, queue q
// being items[lo[q] .. hi[q]), one per XCD; a wave takes the next item of its
// XCD's queue by ticket (qctr, zeroed before the launch), then of the other
// queues.  Either way a wave adds into partial array blockIdx.x of the item's
// instance.  A long evaluation is cut into several launches, each over its
// own ranges, which continue the same partial sums.
template <typename T>
__global__ __launch_bounds__(64) void trilinear_kernel(Geo g, const int *lo, const int *hi, const T1Item *items,
                                                       const T1B *bdesc, const T *K, const Inst *D,
                                                       const Rot *rots, int nq, int *qctr) {
    using T2 = typename V2<T>::type;
    __shared__ T2 ps[2][64];
    const int slot = blockIdx.x;
    const int lane = threadIdx.x;
    const int A = 2 * g.N - 1;
    int it = nq ? -1 : lo[slot] - 1;
    const int it_end = nq ? 0 : hi[slot];
    int q = nq ? (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % (unsigned)nq) : 0;
    int qseen = 0;
    for (;;) {
        if (nq == 0) {
            if (++it >= it_end) break;
        } else {
            int got = -1;
            while (qseen < nq) {
                int tk = 0;
                if (lane == 0) tk = atomicAdd(qctr + q, 1);
                tk = __builtin_amdgcn_readfirstlane(tk);
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
        const T1Item item = items[it];
        const T1B B = bdesc[item.b];
        const Inst &I = D[item.inst];
        double2 *mypart = I.part + (int64_t)slot * g.nm;
        const bool active = lane < item.nt;
        const int t = item.t0 + (active ? lane : 0);
        const int wny = B.wnhi[1] - B.wnlo[1] + 1;
        const int ny = B.wnlo[1] + t % wny;
        const int rest = t / wny;
        const int xb = rest % B.nxb;
        const int nz = B.wnlo[0] + rest / B.nxb;
        const int x0 = B.wnlo[2] + xb * T1_RB;
        const int base = x0 - B.wplo[2];  // a_x = base + i - u
        const int wpx = B.wphi[2] - B.wplo[2] + 1;
        T1Ctx<T> c;
        c.kr = __builtin_amdgcn_make_buffer_rsrc((void *)(K + (int64_t)B.kc * g.nak), (short)0,
                                                 (int)(g.nak * (int64_t)sizeof(T)), 0x00020000);
        c.sA = A * (int)sizeof(T);
        T1Rows rw;
        rw.voff = (int)(idx_K(g, nz - B.wplo[0], ny - B.wplo[1], base) * (int64_t)sizeof(T));
        rw.py = 0;
        rw.pz = 0;
        rw.wpy = B.wphi[1] - B.wplo[1] + 1;
        rw.dy = (int)sizeof(T);
        rw.dz = (g.d == 3 ? g.kax * A : 0) * (int)sizeof(T);
        const int nrows = rw.wpy * (B.wphi[0] - B.wplo[0] + 1);
        const T2 *G = rotated_of<T>(I) + (int64_t)B.rot * g.next;
        T1Pairs<T> pr;
        pr.G = G;
        pr.X = g.N + 1;
        pr.h = g.h;
        pr.d3 = g.d == 3;
        pr.px = B.wplo[2] + min(lane, wpx - 1) + g.h;
        pr.qx = B.bc[2] - (B.wplo[2] + min(lane, wpx - 1)) + g.h;
        pr.bz = B.bc[0];
        pr.by = B.bc[1];
        pr.pzlo = B.wplo[0];
        pr.pylo = B.wplo[1];
        double zr[T1_RB], zi[T1_RB];
#pragma unroll
        for (int i = 0; i < T1_RB; ++i) zr[i] = zi[i] = 0.0;
        switch (wpx >> 3) {
            case 0: t1_rows<T, 0>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 1: t1_rows<T, 1>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 2: t1_rows<T, 2>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 3: t1_rows<T, 3>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 4: t1_rows<T, 4>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 5: t1_rows<T, 5>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 6: t1_rows<T, 6>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            case 7: t1_rows<T, 7>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
            default: t1_rows<T, 8>(c, rw, nrows, wpx, lane, pr, ps, zr, zi); break;
        }
        if (active) {
            const Rot R = rots[B.rot];
#pragma unroll
            for (int i = 0; i < T1_RB; ++i) {
                const int nx = x0 + i;
                if (nx <= B.wnhi[2]) {
                    const T2 gq = ldT2(G, idx_X(g, nz - B.bc[0], ny - B.bc[1], nx - B.bc[2]));
                    const double2 cc = cmul(make_double2(gq.x, gq.y), make_double2(zr[i], zi[i]));
                    const int v[3] = {nz, ny, nx};
                    const int o0 = R.sgn[0] * v[R.perm[0]];
                    const int o1 = R.sgn[1] * v[R.perm[1]];
                    const int o2 = R.sgn[2] * v[R.perm[2]];
                    const int64_t o = idx_I(g, o0, o1, o2);
                    double2 cur = ld2(mypart, o);
                    cur.x += cc.x;
                    cur.y += cc.y;
                    st2(mypart, o, cur);
                }
            }
        }
        // the next item may read back outputs written here by other lanes
        __threadfence_block();
    }
}


}  // namespace

void launch_t1_rows(const Geo &g, int nslots, const int *lo, const int *hi, const T1Item *items,
                     const T1B *bdesc, const float *K, const Inst *D, const Rot *rots, int nq, int *qctr,
                     hipStream_t s) {
    hipLaunchKernelGGL(trilinear_kernel<float>, dim3(nslots), dim3(64), 0, s, g, lo, hi, items, bdesc, K, D,
                       rots, nq, qctr);
}

int t1_rows_blocks_per_cu() {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, trilinear_kernel<float>, 64, 0) == hipSuccess ? nb : 0;
}

}  // namespace bnq
