// Trilinear sum T1 of the Galerkin operator, FP64 (section 'Fast spectral
// approximation of the BNE operator'): inner rows in pairs.
#include "bnq_internal.h"

namespace bnq {
namespace {

// ---------------------------------------------------------------------------
// Trilinear sum.  One 64-lane workgroup per slot; each slot walks its static
// list of items (b, range of <= 64 tasks) and accumulates into its own
// partial array (no atomics; the slots are summed in a fixed order later).
//
// A task is RB consecutive outputs along x at one (y, z), RB = 6, 7 or 8
// chosen per b so that the blocks cover the output row with the least
// overhang (the width is T1B::pad; FP32c items always have 8); tasks are numbered
// y fastest so that the lanes of a wave read consecutive addresses of the
// y-fastest kernel-mode rows.  The inner rows (pz, py) are taken in pairs of
// one plane, A = (pz, py) and B = (pz, py + 1): B needs a_y = ny - py - 1,
// the value just below A's in the table, so one 16-byte load per lane brings
// both (a pair at the end of a plane with an odd row count has an empty B).
// For its two rows a lane slides a 16-value window K(a_x), a_x = base + i -
// u, over the inner index u in blocks of 8: block k uses lo_k[s] = K(base -
// 8k - 8 + s) and hi_k[s] = K(base - 8k + s) = lo_{k-1}[s].  Three 8-value
// arrays rotate (at compile time: the number of full blocks is a template
// parameter) so that the values of block k + 1 are loaded while block k
// computes, and the next pair's first two arrays are loaded at the start of
// the current pair.
//
// Kernel-mode values come through a buffer resource over the canonical row:
// one 32-bit lane offset per window, the 8 values of a window at scalar
// offsets s * 8A.  The pair products of a row are uniform across the wave:
// the next pair's are formed (one p_x per lane, from the rotated spectrum)
// while the current pair computes, then written to a two-stage LDS ring and
// read as broadcasts.
template <typename T>
struct T1Ctx {
    __amdgpu_buffer_rsrc_t kr;            // canonical kernel-mode row
    int voff;                             // byte offset of K(a_x = base) at row A's (a_z, a_y)
    int sA;                               // bytes between consecutive a_x
    const typename V2<T>::type (*PA)[4], (*PB)[4];  // pair-product columns of rows A and B
};

// (K at row B, K at row A) of slot s of the window at voff: neighbours in the
// y-fastest table, one load
template <typename T>
__device__ __forceinline__ typename V2<T>::type t1_kload(const T1Ctx<T> &c, int voff, int s) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(c.kr, voff - 8, s * c.sA, 0));
    else
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(c.kr, voff - 4, s * c.sA, 0));
}

// column registers of pair products a row of NF full blocks can need
// (positions below 8 NF + 8, never more than 64)
template <int NF>
constexpr int t1_ncol() { return (8 * NF + 7) / 16 + 1 < 4 ? (8 * NF + 7) / 16 + 1 : 4; }

// The FMAs at inner position u: zr[i] += k[i] P(u).x,
// zi[i] += k[i] P(u).y, P(u) taken from lane u % 16 of each 16-lane row of
// (px, py) by a DPP row broadcast.  A DPP source needs two wait states after
// a VALU write of it (five after a VALU write of EXEC).  The sources here are
// the pair-product columns, which only LDS loads write, so no wait is
// written; the test suite checks the compiled kernel for both conditions (no
// VALU write of a DPP source within two wait states of its read, no v_cmpx).
// The statement is volatile so that the loads placed between steps keep
// their places.
#define T1_BC32(OP)                                                      \
    OP " %0, %16, %20 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %17, %20 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %16, %21 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %17, %21 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %16, %22 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %17, %22 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %3, %16, %23 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %17, %23 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %4, %16, %24 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %12, %17, %24 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %16, %25 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %13, %17, %25 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %6, %16, %26 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %14, %17, %26 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %7, %16, %27 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %15, %17, %27 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %0, %18, %28 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %19, %28 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %18, %29 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %19, %29 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %18, %30 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %19, %30 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %3, %18, %31 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %19, %31 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %4, %18, %32 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %12, %19, %32 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %18, %33 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %13, %19, %33 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %6, %18, %34 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %14, %19, %34 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %7, %18, %35 row_newbcast:%36 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %15, %19, %35 row_newbcast:%36 row_mask:0xf bank_mask:0xf"

#define T1_BC28(OP)                                                      \
    OP " %0, %14, %18 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %7, %15, %18 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %14, %19 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %15, %19 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %14, %20 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %15, %20 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %3, %14, %21 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %15, %21 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %4, %14, %22 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %15, %22 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %14, %23 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %12, %15, %23 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %6, %14, %24 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %13, %15, %24 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %0, %16, %25 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %7, %17, %25 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %16, %26 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %17, %26 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %16, %27 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %17, %27 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %3, %16, %28 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %17, %28 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %4, %16, %29 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %17, %29 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %16, %30 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %12, %17, %30 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %6, %16, %31 row_newbcast:%32 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %13, %17, %31 row_newbcast:%32 row_mask:0xf bank_mask:0xf"

#define T1_BC24(OP)                                                      \
    OP " %0, %12, %16 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %6, %13, %16 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %12, %17 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %7, %13, %17 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %12, %18 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %13, %18 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %3, %12, %19 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %13, %19 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %4, %12, %20 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %13, %20 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %12, %21 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %13, %21 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %0, %14, %22 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %6, %15, %22 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %1, %14, %23 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %7, %15, %23 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %2, %14, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %8, %15, %24 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %3, %14, %25 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %9, %15, %25 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %4, %14, %26 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %10, %15, %26 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"  \
    OP " %5, %14, %27 row_newbcast:%28 row_mask:0xf bank_mask:0xf\n\t"   \
    OP " %11, %15, %27 row_newbcast:%28 row_mask:0xf bank_mask:0xf"

// The 4 RB FMAs of both rows of a pair at inner position u for the first RB
// outputs (the block width of the item, 6, 7 or 8): row A with its pair
// product pa and window values ka, then row B with pb and kb.
template <typename T, int U, int RB>
__device__ __forceinline__ void t1_fma(T (&zr)[T1_RB], T (&zi)[T1_RB], const typename V2<T>::type &pa,
                                       const typename V2<T>::type &pb, const T (&ka)[8], const T (&kb)[8]) {
    if constexpr (sizeof(T) == 8) {
        if constexpr (RB == 8)
            asm volatile(T1_BC32("v_fmac_f64_dpp") : "+v"(zr[0]), "+v"(zr[1]), "+v"(zr[2]), "+v"(zr[3]), "+v"(zr[4]), "+v"(zr[5]), "+v"(zr[6]), "+v"(zr[7]), "+v"(zi[0]), "+v"(zi[1]), "+v"(zi[2]), "+v"(zi[3]), "+v"(zi[4]), "+v"(zi[5]), "+v"(zi[6]), "+v"(zi[7]) : "v"(pa.x), "v"(pa.y), "v"(pb.x), "v"(pb.y), "v"(ka[0]), "v"(ka[1]), "v"(ka[2]), "v"(ka[3]), "v"(ka[4]), "v"(ka[5]), "v"(ka[6]), "v"(ka[7]), "v"(kb[0]), "v"(kb[1]), "v"(kb[2]), "v"(kb[3]), "v"(kb[4]), "v"(kb[5]), "v"(kb[6]), "v"(kb[7]), "i"(U % 16));
        else if constexpr (RB == 7)
            asm volatile(T1_BC28("v_fmac_f64_dpp") : "+v"(zr[0]), "+v"(zr[1]), "+v"(zr[2]), "+v"(zr[3]), "+v"(zr[4]), "+v"(zr[5]), "+v"(zr[6]), "+v"(zi[0]), "+v"(zi[1]), "+v"(zi[2]), "+v"(zi[3]), "+v"(zi[4]), "+v"(zi[5]), "+v"(zi[6]) : "v"(pa.x), "v"(pa.y), "v"(pb.x), "v"(pb.y), "v"(ka[0]), "v"(ka[1]), "v"(ka[2]), "v"(ka[3]), "v"(ka[4]), "v"(ka[5]), "v"(ka[6]), "v"(kb[0]), "v"(kb[1]), "v"(kb[2]), "v"(kb[3]), "v"(kb[4]), "v"(kb[5]), "v"(kb[6]), "i"(U % 16));
        else
            asm volatile(T1_BC24("v_fmac_f64_dpp") : "+v"(zr[0]), "+v"(zr[1]), "+v"(zr[2]), "+v"(zr[3]), "+v"(zr[4]), "+v"(zr[5]), "+v"(zi[0]), "+v"(zi[1]), "+v"(zi[2]), "+v"(zi[3]), "+v"(zi[4]), "+v"(zi[5]) : "v"(pa.x), "v"(pa.y), "v"(pb.x), "v"(pb.y), "v"(ka[0]), "v"(ka[1]), "v"(ka[2]), "v"(ka[3]), "v"(ka[4]), "v"(ka[5]), "v"(kb[0]), "v"(kb[1]), "v"(kb[2]), "v"(kb[3]), "v"(kb[4]), "v"(kb[5]), "i"(U % 16));
    } else {
        static_assert(RB == 8, "FP32 items have 8-wide blocks");
        asm volatile(T1_BC32("v_fmac_f32_dpp") : "+v"(zr[0]), "+v"(zr[1]), "+v"(zr[2]), "+v"(zr[3]), "+v"(zr[4]), "+v"(zr[5]), "+v"(zr[6]), "+v"(zr[7]), "+v"(zi[0]), "+v"(zi[1]), "+v"(zi[2]), "+v"(zi[3]), "+v"(zi[4]), "+v"(zi[5]), "+v"(zi[6]), "+v"(zi[7]) : "v"(pa.x), "v"(pa.y), "v"(pb.x), "v"(pb.y), "v"(ka[0]), "v"(ka[1]), "v"(ka[2]), "v"(ka[3]), "v"(ka[4]), "v"(ka[5]), "v"(ka[6]), "v"(ka[7]), "v"(kb[0]), "v"(kb[1]), "v"(kb[2]), "v"(kb[3]), "v"(kb[4]), "v"(kb[5]), "v"(kb[6]), "v"(kb[7]), "i"(U % 16));
    }
}

// Inner position u = 8 K + jj of both rows of a pair: row A (the .y halves of
// the window, pair products PA) then row B (.x halves, PB).
template <typename T, int U, int JJ, int RB>
__device__ __forceinline__ void t1_pos(const typename V2<T>::type (&lo)[8], const typename V2<T>::type (&hi)[8],
                                       const typename V2<T>::type (&PA)[4], const typename V2<T>::type (&PB)[4],
                                       T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    // positions stay below 64 (a row has at most N <= 64 inner values); the
    // clamp only keeps the never-taken tail of an 8-block row in bounds
    constexpr int C = U / 16 < 4 ? U / 16 : 3;
    T ka[8], kb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        ka[i] = i - JJ < 0 ? lo[i - JJ + 8].y : hi[i - JJ].y;
        kb[i] = i - JJ < 0 ? lo[i - JJ + 8].x : hi[i - JJ].x;
    }
    t1_fma<T, U, RB>(zr, zi, PA[C], PB[C], ka, kb);
}

// Block K of a pair: lo_K = K(base - 8K - 8 + s), hi_K = lo_{K-1}; issues the
// loads of lo_{K+1} into nx first.
template <typename T, int K, int RB>
__device__ __forceinline__ void t1_full(const T1Ctx<T> &c, const typename V2<T>::type (&lo)[8],
                                        const typename V2<T>::type (&hi)[8], typename V2<T>::type (&nx)[8],
                                        T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    const int vq = c.voff - (8 * (K + 1) + 8) * c.sA;
#pragma unroll
    for (int s = 0; s < 8; ++s) nx[s] = t1_kload(c, vq, s);
    t1_pos<T, 8 * K + 0, 0, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 1, 1, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 2, 2, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 3, 3, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 4, 4, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 5, 5, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 6, 6, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    t1_pos<T, 8 * K + 7, 7, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
}

// the last rem (< 8) positions 8 NF + jj of a pair: uniform branches that
// update the accumulators in place
template <typename T, int NF, int RB>
__device__ __forceinline__ void t1_tail(const T1Ctx<T> &c, int rem, const typename V2<T>::type (&lo)[8],
                                        const typename V2<T>::type (&hi)[8], T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    if (rem > 0) t1_pos<T, 8 * NF + 0, 0, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 1) t1_pos<T, 8 * NF + 1, 1, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 2) t1_pos<T, 8 * NF + 2, 2, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 3) t1_pos<T, 8 * NF + 3, 3, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 4) t1_pos<T, 8 * NF + 4, 4, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 5) t1_pos<T, 8 * NF + 5, 5, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
    if (rem > 6) t1_pos<T, 8 * NF + 6, 6, RB>(lo, hi, *c.PA, *c.PB, zr, zi);
}

// Steps K .. NF of a pair (K < NF: full block K, K = NF: the tail).  Slot
// block j (lo_j, j = -1 .. NF) of the pair is S[j + 1]; S[0] and S[1] arrive
// from the previous pair.  Step K computes block K from S[K + 1] (lo) and
// S[K] (hi) while loading lo_{K+1} into S[K + 2]; the last steps load the
// next pair's first two slot blocks (N0 at step max(NF - 1, 0), N1 at step
// NF), so that at most four slot blocks are live at once.
template <typename T, int NF, int K, int RB>
__device__ __forceinline__ void t1_steps(const T1Ctx<T> &c, int rem, int vn, typename V2<T>::type (&S)[NF + 2][8],
                                         typename V2<T>::type (&N0)[8], typename V2<T>::type (&N1)[8],
                                         T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    if constexpr (K == (NF > 0 ? NF - 1 : 0)) {
#pragma unroll
        for (int s = 0; s < 8; ++s) N0[s] = t1_kload(c, vn, s);
    }
    if constexpr (K == NF) {
#pragma unroll
        for (int s = 0; s < 8; ++s) N1[s] = t1_kload(c, vn - 8 * c.sA, s);
    }
    if constexpr (K < NF) {
        t1_full<T, K, RB>(c, S[K + 1], S[K], S[K + 2], zr, zi);
        t1_steps<T, NF, K + 1, RB>(c, rem, vn, S, N0, N1, zr, zi);
    } else {
        t1_tail<T, NF, RB>(c, rem, S[K + 1], S[K], zr, zi);
    }
}

// the first two slot blocks of a pair whose window offset is v
template <typename T>
__device__ __forceinline__ void t1_ring_start(const T1Ctx<T> &c, int v, typename V2<T>::type (&N0)[8],
                                              typename V2<T>::type (&N1)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        N0[s] = t1_kload(c, v, s);
        N1[s] = t1_kload(c, v - 8 * c.sA, s);
    }
}

// Walks the row pairs in (pz, py) order, py = 0, 2, 4, ... within a plane;
// the window offset of row (pz, py) is voff0 - pz dz - py dy.
struct T1Rows {
    int voff0, voff, py, pz, wpy, dz, dy;
    __device__ __forceinline__ void next(int &z, int &y) const {
        y = py + 2 < wpy ? py + 2 : 0;
        z = py + 2 < wpy ? pz : pz + 1;
    }
    __device__ __forceinline__ int offset(int z, int y) const { return voff0 - z * dz - y * dy; }
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

// Pair products of the next pair: lane l stores P(l) of rows A and B (zero
// past the window, for an empty B, or past the last pair), then reads back
// P(16 c + l % 16) of both rows for every column c.  The rows belong to the
// single wavefront of the workgroup, whose LDS accesses complete in program
// order.
template <typename T, int NC>
__device__ __forceinline__ void t1_exchange(typename V2<T>::type (*pl)[64], int lane, bool keepa, bool keepb,
                                            const typename V2<T>::type &pa, const typename V2<T>::type &pb,
                                            typename V2<T>::type (&PA)[4], typename V2<T>::type (&PB)[4]) {
    typename V2<T>::type va, vb;
    va.x = keepa ? pa.x : (T)0;
    va.y = keepa ? pa.y : (T)0;
    vb.x = keepb ? pb.x : (T)0;
    vb.y = keepb ? pb.y : (T)0;
    pl[0][lane] = va;
    pl[1][lane] = vb;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
        PA[cc] = pl[0][16 * cc + (lane & 15)];
        PB[cc] = pl[1][16 * cc + (lane & 15)];
    }
}

// One pair of inner rows: compute it from its first two slot blocks (N0,
// N1 on entry; they are replaced by the next pair's) and its pair-product
// columns (PA, PB; replaced by the next pair's).  Past the last pair the
// fetches repeat the last pair's addresses and the pair products are zero.
template <typename T, int NF, int RB>
__device__ __forceinline__ void t1_pair(T1Ctx<T> &c, T1Rows &rw, int k, int npairs, int wpx, int lane,
                                        const T1Pairs<T> &pr, typename V2<T>::type (*pl)[64],
                                        typename V2<T>::type (&N0)[8], typename V2<T>::type (&N1)[8],
                                        typename V2<T>::type (&PA)[4], typename V2<T>::type (&PB)[4],
                                        T (&zr)[T1_RB], T (&zi)[T1_RB]) {
    using T2 = typename V2<T>::type;
    const bool more = k + 1 < npairs;
    int npz, npy;
    rw.next(npz, npy);
    npz = more ? npz : rw.pz;
    npy = more ? npy : rw.py;
    const bool hasb = npy + 1 < rw.wpy;
    const auto pna = pr.at(npz, npy);
    const auto pnb = pr.at(npz, hasb ? npy + 1 : npy);
    const int vn = rw.offset(npz, npy);
    T2 S[NF + 2][8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        S[0][s] = N0[s];
        S[1][s] = N1[s];
    }
    c.voff = rw.voff;
    c.PA = &PA;
    c.PB = &PB;
    t1_steps<T, NF, 0, RB>(c, wpx - 8 * NF, vn, S, N0, N1, zr, zi);
    const bool keepa = more && lane < wpx;
    t1_exchange<T, t1_ncol<NF>()>(pl, lane, keepa, keepa && hasb, pna, pnb, PA, PB);
    rw.pz = npz;
    rw.py = npy;
    rw.voff = vn;
}

// All row pairs of an item.  FP64 accumulates every pair in zr/zi; FP32
// accumulates one pair (at most 128 terms per output) in FP32 and adds it to
// the FP64 totals Zr/Zi.
template <typename T, int NF, int RB>
__device__ __forceinline__ void t1_rows(T1Ctx<T> &c, T1Rows rw, int npairs, int wpx, int lane, const T1Pairs<T> &pr,
                                        typename V2<T>::type (*pl)[64], double (&Zr)[T1_RB], double (&Zi)[T1_RB]) {
    typename V2<T>::type N0[8], N1[8], PA[4], PB[4];
    T zr[T1_RB], zi[T1_RB];
#pragma unroll
    for (int i = 0; i < T1_RB; ++i) zr[i] = zi[i] = (T)0;
    t1_ring_start(c, rw.voff, N0, N1);
    {
        const bool hasb = 1 < rw.wpy;
        const bool keepa = lane < wpx;
        t1_exchange<T, t1_ncol<NF>()>(pl, lane, keepa, keepa && hasb, pr.at(0, 0), pr.at(0, hasb ? 1 : 0), PA, PB);
    }
    for (int k = 0; k < npairs; ++k) {
        t1_pair<T, NF, RB>(c, rw, k, npairs, wpx, lane, pr, pl, N0, N1, PA, PB, zr, zi);
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

// rows of an item with NF = wpx / 8 full blocks (a compile-time constant)
template <typename T, int RB>
__device__ __forceinline__ void t1_rows_nf(T1Ctx<T> &c, T1Rows rw, int npairs, int wpx, int lane,
                                           const T1Pairs<T> &pr, typename V2<T>::type (*pl)[64], double (&Zr)[T1_RB],
                                           double (&Zi)[T1_RB]) {
    switch (wpx >> 3) {
        case 0: t1_rows<T, 0, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 1: t1_rows<T, 1, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 2: t1_rows<T, 2, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 3: t1_rows<T, 3, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 4: t1_rows<T, 4, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 5: t1_rows<T, 5, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 6: t1_rows<T, 6, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        case 7: t1_rows<T, 7, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
        default: t1_rows<T, 8, RB>(c, rw, npairs, wpx, lane, pr, pl, Zr, Zi); break;
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
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void trilinear_kernel(const int *lo, const int *hi, const T1Item *items,
                                                       const Inst *D, int nq, int *qctr) {
    using T2 = typename V2<T>::type;
    __shared__ T2 pl[2][64];  // pair products of rows A and B, one p_x per lane
    const int slot = blockIdx.x;
    const int lane = threadIdx.x;
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
        const Inst &I = D[item.inst];
        // the instance's geometry, rows and descriptors: scalar loads (no
        // kernel writes the instance table during the launch)
        const Geo g = ld_uniform_geo(&I.geo);
        const T *K = (const T *)ld_uniform_ptr(&I.K);
        const Rot *rots = ld_uniform_ptr(&I.rots);
        const T1B B = ((const T1B *)ld_uniform_ptr(&I.t1d))[item.b];
        const int A = 2 * g.N - 1;
        // static: the item's own list names its partial array; dynamic: the
        // wave's slot
        double2 *mypart = I.part + (int64_t)(nq ? slot : item.slot) * g.nm;
        const bool active = lane < item.nt;
        const int t = item.t0 + (active ? lane : 0);
        const int wny = B.wnhi[1] - B.wnlo[1] + 1;
        const int ny = B.wnlo[1] + t % wny;
        const int rest = t / wny;
        const int xb = rest % B.nxb;
        const int nz = B.wnlo[0] + rest / B.nxb;
        // outputs per task along x: the item's block width (6, 7 or 8)
        const int rb = __builtin_amdgcn_readfirstlane(B.pad);
        const int x0 = B.wnlo[2] + xb * rb;
        const int base = x0 - B.wplo[2];  // a_x = base + i - u
        const int wpx = B.wphi[2] - B.wplo[2] + 1;
        T1Ctx<T> c;
        // the row is uniform; saying so keeps the buffer resource in scalar
        // registers (otherwise every load becomes a loop over lanes)
        const int kc = __builtin_amdgcn_readfirstlane(B.kc);
        c.kr = __builtin_amdgcn_make_buffer_rsrc((void *)(K + (int64_t)kc * g.nak), (short)0,
                                                 (int)(g.nak * (int64_t)sizeof(T)), 0x00020000);
        c.sA = A * (int)sizeof(T);
        T1Rows rw;
        rw.voff0 = (int)(idx_K(g, nz - B.wplo[0], ny - B.wplo[1], base) * (int64_t)sizeof(T));
        rw.voff = rw.voff0;
        rw.py = 0;
        rw.pz = 0;
        rw.wpy = B.wphi[1] - B.wplo[1] + 1;
        rw.dy = (int)sizeof(T);
        rw.dz = (g.d == 3 ? g.kax * A : 0) * (int)sizeof(T);
        const int npairs = (rw.wpy + 1) / 2 * (B.wphi[0] - B.wplo[0] + 1);
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
        if constexpr (sizeof(T) == 8) {
            if (rb == 6)
                t1_rows_nf<T, 6>(c, rw, npairs, wpx, lane, pr, pl, zr, zi);
            else if (rb == 7)
                t1_rows_nf<T, 7>(c, rw, npairs, wpx, lane, pr, pl, zr, zi);
            else
                t1_rows_nf<T, 8>(c, rw, npairs, wpx, lane, pr, pl, zr, zi);
        } else {
            t1_rows_nf<T, 8>(c, rw, npairs, wpx, lane, pr, pl, zr, zi);
        }
        if (active) {
            const Rot R = rots[B.rot];
#pragma unroll
            for (int i = 0; i < T1_RB; ++i) {
                const int nx = x0 + i;
                if (i < rb && nx <= B.wnhi[2]) {
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

void launch_t1_pairs(int nslots, const int *lo, const int *hi, const T1Item *items, const Inst *D, int nq,
                     int *qctr, hipStream_t s) {
    hipLaunchKernelGGL(trilinear_kernel<double>, dim3(nslots), dim3(64), 0, s, lo, hi, items, D, nq, qctr);
}

int t1_pairs_blocks_per_cu() {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, trilinear_kernel<double>, 64, 0) == hipSuccess ? nb : 0;
}

}  // namespace bnq
