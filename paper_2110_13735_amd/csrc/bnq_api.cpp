// Host runtime of libbnq: the C ABI of include/bnq.h, plans, the shared
// kernel-mode table cache and the orchestration of the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bnq.h"
#include "bnq_internal.h"

using namespace bnq;

namespace {

thread_local std::string g_err;

bnq_status fail(bnq_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(BNQ_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                            \
    } while (0)

#define LAUNCHCHK()                                                                    \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return fail(BNQ_EHIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                           \
    } while (0)

const double kR = 2.0 * M_PI / (3.0 + std::sqrt(2.0));  // R = S, pi = (3 + sqrt 2) S / 2
const int kNq = 128;                                    // radial Gauss–Legendre nodes
const int kMaxSlots = 4096;                             // trilinear partial arrays (upper bound)
const int kCusPerXcd = 32;                              // compute units per XCD on gfx950

// ---------------------------------------------------------------------------
Geo make_geo(int d, int N) {
    Geo g;
    g.d = d;
    g.N = N;
    g.h = N / 2;
    g.e0 = d == 3 ? N : 1;
    g.lo0 = d == 3 ? -N / 2 : 0;
    g.nm = (int64_t)g.e0 * N * N;
    g.eg0 = d == 3 ? 2 * N : 1;
    g.neg = (int64_t)g.eg0 * 2 * N * 2 * N;
    g.ea0 = d == 3 ? 2 * N - 1 : 1;
    g.na = (int64_t)g.ea0 * (2 * N - 1) * (2 * N - 1);
    g.kax = 2 * N - 1 + KPADLO + KPADHI;
    g.nak = (int64_t)g.ea0 * g.kax * (2 * N - 1);
    g.ex0 = d == 3 ? N + 1 : 1;
    g.next = (int64_t)g.ex0 * (N + 1) * (N + 1);
    g.psplit = pair_split_default(d, N, 1);
    return g;
}

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2.0L * j - 1) * z * p2 - (j - 1.0L) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1);
            long double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs((double)(z - z1)) < 1e-19) break;
        }
        x[i] = (double)-z;
        x[n - 1 - i] = (double)z;
        w[i] = w[n - 1 - i] = (double)(2.0L / ((1 - z * z) * pp * pp));
    }
}

int mcut_of(double q) {
    const double x = kR * std::sqrt(q);
    return (int)std::ceil((x + 10.0 * std::cbrt(x) + 30.0) / 2.0);
}

// Signed axis permutations: 48 in 3-D; in 2-D the 8 that fix axis 0.
std::vector<Rot> make_group(int d) {
    std::vector<Rot> out;
    int p[3] = {0, 1, 2};
    do {
        if (d == 2 && p[0] != 0) continue;
        for (int sm = 0; sm < 8; ++sm) {
            if (d == 2 && (sm & 1)) continue;
            Rot r;
            for (int i = 0; i < 3; ++i) {
                r.perm[i] = p[i];
                r.sgn[i] = (sm >> i) & 1 ? -1 : 1;
            }
            out.push_back(r);
        }
    } while (std::next_permutation(p, p + 3));
    return out;
}

int rot_index(const std::vector<Rot> &grp, const int *perm, const int *sgn) {
    for (size_t r = 0; r < grp.size(); ++r)
        if (std::equal(perm, perm + 3, grp[r].perm) && std::equal(sgn, sgn + 3, grp[r].sgn)) return (int)r;
    return -1;
}

// b = R b_c with b_c components sorted |b| descending (ties by axis index);
// in 2-D axis 0 stays fixed.
void canonicalize(int d, const int *b, int *bc, int *perm, int *sgn) {
    int ax[3] = {0, 1, 2};
    const int first = d == 3 ? 0 : 1;
    std::stable_sort(ax + first, ax + 3, [&](int i, int j) { return std::abs(b[i]) > std::abs(b[j]); });
    for (int j = 0; j < 3; ++j) bc[j] = std::abs(b[ax[j]]);
    for (int j = 0; j < 3; ++j) perm[ax[j]] = j;
    for (int i = 0; i < 3; ++i) sgn[i] = b[i] < 0 ? -1 : 1;
}

// ---------------------------------------------------------------------------
// Shared kernel-mode tables for one (d, N, C_phi).
struct TableSet {
    int refs = 0;
    int d = 0, N = 0;
    double Cphi = 0;
    int device = 0;
    Geo g;
    int qmax = 0, M = 0;
    double *J = nullptr, *coef = nullptr, *lrA = nullptr, *lrB = nullptr, *bdiag = nullptr;
    int *mcut = nullptr;
    std::vector<int> canon;      // 3 per row
    std::vector<int> canon_row;  // [N][N][N] -> row or -1
    int ncanon = 0;
    int *canon_d = nullptr;
    // kernel-mode tables, each precision built when a plan first needs it
    double *K = nullptr, *wc = nullptr, *wq = nullptr;
    float *K32 = nullptr, *wc32 = nullptr, *wq32 = nullptr;
    size_t bytes = 0;
    Radial radial() const {
        Radial r;
        r.J = J;
        r.mcut = mcut;
        r.coef = coef;
        r.lrA = lrA;
        r.lrB = lrB;
        r.bdiag = bdiag;
        r.M = M;
        r.d = d;
        return r;
    }
};

std::mutex g_cache_mu;
std::vector<TableSet *> g_cache;

void canon_list(int d, int N, std::vector<int> &canon, std::vector<int> &row) {
    canon.clear();
    row.assign((size_t)N * N * N, -1);
    int n = 0;
    if (d == 3) {
        for (int c0 = 0; c0 < N; ++c0)
            for (int c1 = 0; c1 <= c0; ++c1)
                for (int c2 = 0; c2 <= c1; ++c2) {
                    canon.insert(canon.end(), {c0, c1, c2});
                    row[((size_t)c0 * N + c1) * N + c2] = n++;
                }
    } else {
        for (int c1 = 0; c1 < N; ++c1)
            for (int c2 = 0; c2 <= c1; ++c2) {
                canon.insert(canon.end(), {0, c1, c2});
                row[((size_t)0 * N + c1) * N + c2] = n++;
            }
    }
}

// Bytes of the radial tables of a table set, and of its kernel-mode tables
// (trilinear rows plus the two pair-weight tables) in FP64 and in FP32.
size_t table_bytes_radial(int d, int N) {
    const int qmax = d * N * N;
    const int M = mcut_of(qmax) + 1;
    return sizeof(double) * ((size_t)(qmax + 1) * (M + 1)) + sizeof(int) * (qmax + 1);
}

size_t table_values(int d, int N) {
    Geo g = make_geo(d, N);
    std::vector<int> canon, row;
    canon_list(d, N, canon, row);
    return (canon.size() / 3) * (size_t)g.nak + 2 * (size_t)g.nm * g.nm;
}

size_t table_bytes_f64(int d, int N) { return sizeof(double) * table_values(d, N); }
size_t table_bytes_f32(int d, int N) { return sizeof(float) * table_values(d, N); }

void free_tables(TableSet *t) {
    hipFree(t->J);
    hipFree(t->coef);
    hipFree(t->lrA);
    hipFree(t->lrB);
    hipFree(t->bdiag);
    hipFree(t->mcut);
    hipFree(t->canon_d);
    hipFree(t->K);
    hipFree(t->wc);
    hipFree(t->wq);
    hipFree(t->K32);
    hipFree(t->wc32);
    hipFree(t->wq32);
    delete t;
}

template <typename T>
bnq_status dalloc(T **p, size_t count, const char *what) {
    *p = nullptr;
    if (count == 0) return BNQ_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        hipGetLastError();
        return fail(BNQ_ENOMEM, "hipMalloc of %zu bytes for %s failed: %s", count * sizeof(T), what,
                    hipGetErrorString(e));
    }
    return BNQ_OK;
}

template <typename T>
bnq_status upload(T **p, const std::vector<T> &v, const char *what) {
    bnq_status st = dalloc(p, v.size(), what);
    if (st) return st;
    HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return BNQ_OK;
}

bnq_status build_tables(TableSet *t, hipStream_t s) {
    const int d = t->d, N = t->N;
    t->g = make_geo(d, N);
    t->qmax = d * N * N;
    t->M = mcut_of(t->qmax) + 1;
    bnq_status st;
    // host constants
    std::vector<double> glx, glw;
    gauss_legendre(kNq, glx, glw);
    std::vector<int> mcut(t->qmax + 1);
    for (int q = 0; q <= t->qmax; ++q) mcut[q] = std::min(mcut_of(q), t->M - 1);
    std::vector<double> coef(t->M), lrA(2 * t->M + 4), lrB(2 * t->M + 4);
    double p0 = 1.0;  // P_{2m}(0)
    for (int m = 0; m < t->M; ++m) {
        if (m > 0) p0 *= -(2.0 * m - 1.0) / (2.0 * m);
        if (d == 3)
            coef[m] = 32.0 * M_PI * M_PI * t->Cphi * (4.0 * m + 1.0) * p0;
        else
            coef[m] = 8.0 * M_PI * t->Cphi * (m == 0 ? 1.0 : 2.0) * ((m & 1) ? -1.0 : 1.0);
    }
    for (size_t n = 0; n < lrA.size(); ++n) {
        lrA[n] = (2.0 * n + 1.0) / (n + 1.0);
        lrB[n] = (double)n / (n + 1.0);
    }
    double *glx_d = nullptr, *glw_d = nullptr;
    if ((st = upload(&glx_d, glx, "nodes")) || (st = upload(&glw_d, glw, "weights"))) {
        hipFree(glx_d);
        return st;
    }
    if ((st = upload(&t->mcut, mcut, "mcut")) || (st = upload(&t->coef, coef, "coef")) ||
        (st = upload(&t->lrA, lrA, "lrA")) || (st = upload(&t->lrB, lrB, "lrB")) ||
        (st = dalloc(&t->J, (size_t)(t->qmax + 1) * t->M, "radial table"))) {
        hipFree(glx_d);
        hipFree(glw_d);
        return st;
    }
    double *scratch = nullptr;
    if ((st = dalloc(&scratch, (size_t)(t->qmax + 1) * t->M * kNq, "radial scratch"))) {
        hipFree(glx_d);
        hipFree(glw_d);
        return st;
    }
    launch_radial(d, kR, t->qmax, t->M, kNq, glx_d, glw_d, scratch, t->J, s);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
    if ((st = dalloc(&t->bdiag, (size_t)t->qmax + 1, "kernel-mode diagonal"))) {
        hipFree(scratch);
        hipFree(glx_d);
        hipFree(glw_d);
        return st;
    }
    launch_beta_diag(t->radial(), t->qmax, t->bdiag, s);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
    hipFree(scratch);
    hipFree(glx_d);
    hipFree(glw_d);
    canon_list(d, N, t->canon, t->canon_row);
    t->ncanon = (int)(t->canon.size() / 3);
    if ((st = upload(&t->canon_d, t->canon, "canonical list"))) return st;
    t->bytes = table_bytes_radial(d, N);
    return BNQ_OK;
}

// Kernel-mode tables of one precision (T = double: FP64 plans; T = float:
// FP32c plans), built on first need.  Each value is formed in FP64 from the
// radial table; the FP32 tables hold it rounded to nearest, so they never
// need the FP64 ones.  The trilinear rows and the two pair-weight tables are
// built separately: an FP64 set whose weights do not fit (3-D N = 48: rows
// 168 GB, weights 196 GB) keeps the rows only, and its plans form the pair
// weights on the fly.
template <typename T>
bnq_status build_table(TableSet *t, T **out, size_t n, const char *what, bool rows, hipStream_t s) {
    if (*out) return BNQ_OK;
    const Geo &g = t->g;
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const size_t need = sizeof(T) * n * (rows ? 1 : 2);
    if (need > freeb) return fail(BNQ_ENOMEM, "%s %s need %zu bytes, %zu free", sizeof(T) == 8 ? "FP64" : "FP32",
                                  what, need, freeb);
    T *a = nullptr, *b = nullptr;
    bnq_status st;
    if ((st = dalloc(&a, n, what)) || (!rows && (st = dalloc(&b, n, what)))) {
        hipFree(a);
        return st;
    }
    const Radial rad = t->radial();
    if (rows)
        launch_beta_rows(g, rad, t->canon_d, t->ncanon, a, s);
    else
        launch_weights(g, rad, a, b, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(a);
        hipFree(b);
        return fail(BNQ_EHIP, "%s build failed: %s", what, hipGetErrorString(e));
    }
    out[0] = a;
    if (!rows) out[1] = b;
    t->bytes += need;
    return BNQ_OK;
}

// The table set of (d, N, C_phi) on the current device, with the kernel-mode
// tables of precision prec, shared by every plan that uses it (refcounted).
// FP64 sets get their weight tables unless weights = false or they do not
// fit; *weights_out says whether the set holds them.
bnq_status acquire_tables(int d, int N, double Cphi, int prec, bool weights, hipStream_t s, TableSet **out,
                          bool *weights_out) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    TableSet *t = nullptr;
    for (TableSet *c : g_cache)
        if (c->d == d && c->N == N && c->Cphi == Cphi && c->device == dev) t = c;
    bnq_status st;
    const bool fresh = t == nullptr;
    if (fresh) {
        t = new TableSet;
        t->d = d;
        t->N = N;
        t->Cphi = Cphi;
        t->device = dev;
        if ((st = build_tables(t, s))) {
            free_tables(t);
            return st;
        }
    }
    const size_t nk = (size_t)t->ncanon * t->g.nak, nw = (size_t)t->g.nm * t->g.nm;
    if (prec == BNQ_FP32C) {
        // both weight tables come in one call (wc32, wq32 are adjacent members)
        float *w2[2] = {t->wc32, t->wq32};
        st = build_table(t, &t->K32, nk, "trilinear kernel-mode table", true, s);
        if (!st) st = build_table(t, w2, nw, "pair weight tables", false, s);
        t->wc32 = w2[0];
        t->wq32 = w2[1];
    } else {
        st = build_table(t, &t->K, nk, "trilinear kernel-mode table", true, s);
        if (!st && weights && !t->wc) {
            size_t freeb = 0, totalb = 0;
            HIPCHK(hipMemGetInfo(&freeb, &totalb));
            // keep 8 GB for plan workspaces; without room the weights are formed on the fly
            if (2 * sizeof(double) * nw + ((size_t)8 << 30) <= freeb) {
                double *w2[2] = {nullptr, nullptr};
                st = build_table(t, w2, nw, "pair weight tables", false, s);
                t->wc = w2[0];
                t->wq = w2[1];
            }
        }
    }
    if (st) {
        if (fresh) free_tables(t);
        return st;
    }
    if (fresh) g_cache.push_back(t);
    t->refs++;
    *out = t;
    if (weights_out) *weights_out = prec == BNQ_FP32C ? true : t->wc != nullptr;
    return BNQ_OK;
}

void release_tables(TableSet *t) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (--t->refs > 0) return;
    g_cache.erase(std::remove(g_cache.begin(), g_cache.end(), t), g_cache.end());
    free_tables(t);
}

// ---------------------------------------------------------------------------
// 1-D counts of the Galerkin sums (per axis; a d-D count is the d-th power).
void counts_1d(int N, double &c1, double &w1, double &o1, double &t1) {
    const int h = N / 2;
    auto in = [&](int k) { return k >= -h && k < h; };
    c1 = w1 = o1 = t1 = 0;
    for (int l = -h; l < h; ++l)
        for (int m = -h; m < h; ++m) {
            w1 += 1;
            if (in(l + m)) c1 += 1;
        }
    for (int n = -h; n < h; ++n)
        for (int k = -h; k < h; ++k)
            if (n - k >= -N && n - k <= N - 2) o1 += 1;
    for (int k = -h; k < h; ++k)
        for (int l = -h; l < h; ++l)
            for (int m = -h; m < h; ++m)
                if (in(k + l + m)) t1 += 1;
}

}  // namespace

// ---------------------------------------------------------------------------
namespace {
// Trilinear work distribution: slots = resident waves / slot_div; the items
// are split into one run per XCD (xcd = 1) or dealt over all slots as one run.
struct T1Tune {
    int slot_div = 1;
    int xcd = 1;
};
const T1Tune kTuneCandidates[] = {{1, 1}, {2, 1}, {1, 0}, {2, 0}};
constexpr int kNumTune = 4;
std::mutex g_tune_mu;
// (device, d, N, precision) -> index in kTuneCandidates chosen by
// bnq_plan_autotune or set by bnq_tune_set
std::map<std::tuple<int, int, int, int>, int> g_tune;
// (device, d, N, precision, eps == 0) -> pair-sum slices chosen by
// bnq_plan_autotune_pairs or set by bnq_tune_pairs_set
std::map<std::tuple<int, int, int, int, int>, int> g_tune_pairs;
const int kPairSplitCandidates[] = {8, 16, 32};
constexpr int kNumPairSplit = 3;
}  // namespace

struct bnq_plan_s {
    bnq_params p;
    Geo g;
    TableSet *tabs = nullptr;
    double alpha = 0, pref = 0;
    std::vector<Rot> grp;
    Rot *rots_d = nullptr;
    double2 *tw = nullptr;
    double2 *Ghat = nullptr, *tmp = nullptr, *tmp2 = nullptr, *Gr = nullptr, *W = nullptr, *Qc = nullptr,
            *T1 = nullptr, *X = nullptr, *Qh = nullptr, *part = nullptr, *ppart = nullptr,
            *xpart = nullptr;
    float2 *G32 = nullptr, *Gr32 = nullptr;  // FP32c spectra
    int nbdesc = 0;
    double *kbuf[4] = {nullptr, nullptr, nullptr, nullptr}, *ybuf = nullptr;
    double *mom_part = nullptr, *mom_out = nullptr;
    int *health = nullptr;  // two flag words in pinned, device-coherent host memory
    double *ginv = nullptr;  // inverse Gram matrix for BNQ_CORR_MOMENTS
    double *dmat = nullptr;  // N x N spectral differentiation matrix (rescaled scheme)
    bool otf = false;        // FP64 pair weights formed on the fly (no weight tables)
    // BNQ_FLAG_T1_SEPARATED: angle count, alpha rows, their cosine transforms
    // over the doubled grid, the spectrum there and the per-block partials
    int sepP = 0;
    double *sep_al = nullptr, *sep_alp = nullptr;
    double2 *sep_gc = nullptr, *sep_gt = nullptr, *sep_part = nullptr;
    int nslots = 0;
    T1Item *items = nullptr;
    T1B *bdesc = nullptr;         // FP64: one descriptor per b
    T1G *gdesc = nullptr;         // FP32c: one descriptor per group of b (matrix-core kernel)
    std::vector<T1Item> items_h;  // per-list item lists (host copy), list offsets
    std::vector<float> icost_h;   // model cost of each item of items_h
    std::vector<int> off_h;       // (dynamic schedule: queue offsets)
    int nq = 0;                   // dynamic schedule: queues (0 = static)
    int *qctr = nullptr;
    int nchunk = 1;               // trilinear launches per evaluation
    int *t1cut = nullptr;         // their item ranges (t1_cuts)
    T1Tune tune;                  // trilinear work distribution
    Inst ih{};                    // workspace pointers and scalars (host copy)
    Inst *inst_d = nullptr;       // device copy, one entry
    std::atomic<int> nbatch{0};   // batches holding this plan (they copy its workspace pointers)
    double counts[4] = {0, 0, 0, 0};
    // timing
    bool timing = false;
    struct Ev {
        int fam;
        hipEvent_t a, b;
    };
    std::vector<Ev> evs;
    std::vector<hipEvent_t> pool;
    hipStream_t last = nullptr;
};

struct bnq_batch_s;


namespace {

hipEvent_t ev_get(bnq_plan_s *P) {
    if (!P->pool.empty()) {
        hipEvent_t e = P->pool.back();
        P->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Span {
    bnq_plan_s *P;
    int fam;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Span(bnq_plan_s *P_, int fam_, hipStream_t s_) : P(P_), fam(fam_), s(s_) {
        if (P && P->timing) {
            a = ev_get(P);
            if (a) hipEventRecord(a, s);
        }
    }
    ~Span() {
        if (P && P->timing && a) {
            hipEvent_t b = ev_get(P);
            if (b) {
                hipEventRecord(b, s);
                P->evs.push_back({fam, a, b});
            } else {
                P->pool.push_back(a);
            }
        }
    }
};

bnq_status validate(const bnq_params *p) {
    if (!p) return fail(BNQ_EINVAL, "params is NULL");
    if (p->d != 2 && p->d != 3) return fail(BNQ_EINVAL, "d must be 2 or 3 (got %d)", p->d);
    if (p->N < 2 || p->N > 64 || (p->N & 1)) return fail(BNQ_EINVAL, "N must be even in [2, 64] (got %d)", p->N);
    if (p->eps < -1 || p->eps > 1) return fail(BNQ_EINVAL, "eps must be -1, 0 or 1 (got %d)", p->eps);
    if (!(p->L > 0) || !std::isfinite(p->L)) return fail(BNQ_EINVAL, "L must be positive");
    if (!(p->hbar > 0) || !(p->C_phi > 0) || !(p->c >= 0)) return fail(BNQ_EINVAL, "hbar, C_phi must be > 0, c >= 0");
    if (p->precision != BNQ_FP64 && p->precision != BNQ_FP32C)
        return fail(BNQ_EINVAL, "precision must be BNQ_FP64 or BNQ_FP32C (got %d)", p->precision);
    if (p->terms < 0 || p->terms > BNQ_T_ALL) return fail(BNQ_EINVAL, "bad terms mask %d", p->terms);
    if (p->correction != BNQ_CORR_NONE && p->correction != BNQ_CORR_MASS && p->correction != BNQ_CORR_MOMENTS)
        return fail(BNQ_EINVAL, "bad correction %d", p->correction);
    if (p->schedule != BNQ_SCHED_STATIC && p->schedule != BNQ_SCHED_DYNAMIC)
        return fail(BNQ_EINVAL, "bad schedule %d", p->schedule);
    if (p->flags & ~(BNQ_FLAG_WEIGHTS_OTF | BNQ_FLAG_T1_SEPARATED | BNQ_FLAG_NO_FERMI_BOUND))
        return fail(BNQ_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->angles < 0) return fail(BNQ_EINVAL, "angles must be >= 0 (got %d)", p->angles);
    if (p->angles > 0 && !(p->flags & BNQ_FLAG_T1_SEPARATED))
        return fail(BNQ_EINVAL, "angles is read only with BNQ_FLAG_T1_SEPARATED");
    if ((p->flags & BNQ_FLAG_T1_SEPARATED) && (p->precision != BNQ_FP64 || !sep_supported(p->d, p->N)))
        return fail(BNQ_ENOTSUP, "the separated-kernel trilinear route is FP64, d = 2 with N <= 32 or d = 3 with N <= 8");
    if (p->angles > (p->d == 2 ? 4096 : 64))
        return fail(BNQ_EINVAL, "angles must be <= %d in %d-D (got %d)", p->d == 2 ? 4096 : 64, p->d, p->angles);
    if ((p->flags & BNQ_FLAG_T1_SEPARATED) && p->d == 3 && p->angles == 0)
        return fail(BNQ_EINVAL, "the 3-D separated route needs an explicit angle count");
    if ((p->flags & BNQ_FLAG_WEIGHTS_OTF) && p->precision != BNQ_FP64)
        return fail(BNQ_ENOTSUP, "weights on the fly are an FP64 mode");
    return BNQ_OK;
}

// workspace of the separated-kernel trilinear route (0 without the flag)
size_t sep_bytes(const bnq_params *p) {
    if (!(p->flags & BNQ_FLAG_T1_SEPARATED)) return 0;
    const size_t N = p->N, M = 2 * N, w = 2 * N - 1;
    const size_t na = p->d == 2 ? w * w : w * w * w, Md = p->d == 2 ? M * M : M * M * M,
                 Nd = p->d == 2 ? N * N : N * N * N;
    const int Pn = sep_directions(p->d, p->angles > 0 ? p->angles : sep_auto_angles(p->N, kR));
    int nc, jc, nbj;
    sep_shape(p->d, p->N, Pn, &nc, &jc, &nbj);
    return sizeof(double) * 2 * Pn * na + sizeof(double2) * (Pn * Md + Md + (size_t)Pn * nbj * Nd);
}

size_t plan_workspace_bytes(const bnq_params *p, int nslots_est) {
    Geo g = make_geo(p->d, p->N);
    const size_t c = sizeof(double2), r = sizeof(double);
    const size_t nrot = p->d == 3 ? 48 : 8;
    const size_t f32 = p->precision == BNQ_FP32C ? sizeof(float2) * ((size_t)g.nm + nrot * g.next) : 0;
    if (p->eps == 0 || !(p->terms & BNQ_T_QTRI)) nslots_est = 0;  // no trilinear partial arrays
    return c * (6 * (size_t)g.nm + g.neg + nrot * g.next + (size_t)nslots_est * g.nm +
                (size_t)pair_split_max(g.N) * ((size_t)g.neg + g.nm) + (size_t)outer_split(g) * g.nm) +
           r * 5 * (size_t)g.nm + f32 + sep_bytes(p);
}

// Inverse of the Gram matrix of c = (1, v_1..v_d, |v|^2) over the velocity
// nodes (long double sums, Gauss–Jordan with partial pivoting).
bnq_status gram_inverse(int d, int N, double hstep, std::vector<double> &out) {
    const int m = d + 2, h = N / 2;
    long double G[5][10] = {};
    const int n0 = d == 3 ? N : 1;
    for (int a = 0; a < n0; ++a)
        for (int b = 0; b < N; ++b)
            for (int e = 0; e < N; ++e) {
                long double v[3] = {d == 3 ? (long double)(a - h) * hstep : 0.0L, (long double)(b - h) * hstep,
                                    (long double)(e - h) * hstep};
                long double c[5];
                c[0] = 1.0L;
                int k = 1;
                for (int x = (d == 3 ? 0 : 1); x < 3; ++x) c[k++] = v[x];
                c[m - 1] = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                for (int r = 0; r < m; ++r)
                    for (int q = 0; q < m; ++q) G[r][q] += c[r] * c[q];
            }
    for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) G[r][m + q] = r == q ? 1.0L : 0.0L;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs((double)G[r][col]) > std::fabs((double)G[piv][col])) piv = r;
        if (G[piv][col] == 0.0L) return fail(BNQ_EINVAL, "singular moment Gram matrix (N too small)");
        for (int q = 0; q < 2 * m; ++q) std::swap(G[col][q], G[piv][q]);
        const long double pv = G[col][col];
        for (int q = 0; q < 2 * m; ++q) G[col][q] /= pv;
        for (int r = 0; r < m; ++r)
            if (r != col) {
                const long double f = G[r][col];
                for (int q = 0; q < 2 * m; ++q) G[r][q] -= f * G[col][q];
            }
    }
    out.assign((size_t)m * m, 0.0);
    for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) out[(size_t)r * m + q] = (double)G[r][m + q];
    return BNQ_OK;
}

// Trilinear terms of one evaluation, and the number of launches it is cut
// into: at most about 2e13 terms (one to two seconds) per launch, so that no
// single kernel runs for tens of seconds at 3-D N = 48.
double t1_terms(int d, int N) {
    double c1, w1, o1, t1;
    counts_1d(N, c1, w1, o1, t1);
    return std::pow(t1, d);
}

int t1_chunks(double terms) { return std::max(1, (int)std::ceil(terms / 2e13)); }

// Static item lists of a trilinear launch over nslots partial arrays: one
// per 64-lane workgroup (FP64), one per 4-wave matrix-core workgroup (FP32c).
int t1_lists(int prec, int nslots) { return prec ? nslots / T1M_WAVES : nslots; }

// Item ranges of the launches: off holds the nl + 1 boundaries of the nl
// slot lists (or queues); launch r covers [cut[r nl + i], cut[(r + 1) nl + i])
// of list i, so the launches together walk every list once, in order.  The
// cuts split each list by model cost (cost[k] of item k), so that every
// launch gives each list the same share of its work also when a list holds
// items of very different sizes (a batch's instances of different N).
std::vector<int> t1_cuts(const std::vector<int> &off, const std::vector<float> &cost, int nchunk) {
    const size_t nl = off.size() - 1;
    std::vector<int> cut((nchunk + 1) * nl);
    for (size_t i = 0; i < nl; ++i) {
        double total = 0;
        for (int k = off[i]; k < off[i + 1]; ++k) total += cost[k];
        int k = off[i];
        double acc = 0;
        cut[i] = off[i];
        for (int r = 1; r < nchunk; ++r) {
            const double target = total * r / nchunk;
            while (k < off[i + 1] && acc + 0.5 * cost[k] <= target) acc += cost[k++];
            cut[r * nl + i] = k;
        }
        cut[nchunk * nl + i] = off[i + 1];
    }
    return cut;
}

bnq_status build_t1_work_mfma(bnq_plan_s *P);

bnq_status build_t1_work(bnq_plan_s *P) {
    if (P->p.precision == BNQ_FP32C) return build_t1_work_mfma(P);
    const Geo &g = P->g;
    const TableSet *t = P->tabs;
    const int d = g.d, N = g.N, h = g.h;
    std::vector<T1B> bd;
    struct It {
        T1Item it;
        double cost;
    };
    std::vector<It> items;
    const int b0lo = d == 3 ? -N + 1 : 0, b0hi = d == 3 ? N - 2 : 0;
    for (int b0 = b0lo; b0 <= b0hi; ++b0)
        for (int b1 = -N + 1; b1 <= N - 2; ++b1)
            for (int b2 = -N + 1; b2 <= N - 2; ++b2) {
                const int b[3] = {b0, b1, b2};
                int bc[3], perm[3], sgn[3];
                canonicalize(d, b, bc, perm, sgn);
                T1B B;
                B.rot = rot_index(P->grp, perm, sgn);
                B.kc = t->canon_row[((size_t)bc[0] * N + bc[1]) * N + bc[2]];
                if (B.rot < 0 || B.kc < 0) return fail(BNQ_EINVAL, "internal: canonical form of b not found");
                int lo[3], ext[3];
                for (int i = 0; i < 3; ++i) {
                    const int j = perm[i];
                    const bool triv = d == 2 && i == 0;
                    lo[j] = triv ? 0 : -h + (sgn[i] < 0 ? 1 : 0);
                    ext[j] = triv ? 1 : N;
                }
                bool empty = false;
                for (int j = 0; j < 3; ++j) {
                    const int L0 = lo[j], H0 = lo[j] + ext[j] - 1, c = bc[j];
                    B.bc[j] = c;
                    B.wnlo[j] = L0 + c;
                    B.wnhi[j] = H0;
                    B.wplo[j] = std::max(L0, c - H0);
                    B.wphi[j] = std::min(H0, c - L0);
                    if (B.wnlo[j] > B.wnhi[j] || B.wplo[j] > B.wphi[j]) empty = true;
                }
                if (empty) continue;
                const int wnx = B.wnhi[2] - B.wnlo[2] + 1;
                // FP64: the block width among 8, 7, 6 whose blocks overhang the
                // output row least (the kernel's time per block grows with its
                // width).  FP32c keeps 8: measured, narrower blocks made its
                // kernel slower
                int rb = T1_RB;
                if (P->p.precision != BNQ_FP32C)
                    for (int w = T1_RB - 1; w >= 6; --w)
                        if ((wnx + w - 1) / w * w < (wnx + rb - 1) / rb * rb) rb = w;
                B.nxb = (wnx + rb - 1) / rb;
                B.pad = rb;
                const int ntasks = B.nxb * (B.wnhi[1] - B.wnlo[1] + 1) * (B.wnhi[0] - B.wnlo[0] + 1);
                const int wpx = B.wphi[2] - B.wplo[2] + 1;
                const double rows = (double)(B.wphi[1] - B.wplo[1] + 1) * (B.wphi[0] - B.wplo[0] + 1);
                const double cost = rows * ((wpx + 7) / 8 + 2) * rb / T1_RB + 8;
                const int bi = (int)bd.size();
                bd.push_back(B);
                for (int t0 = 0; t0 < ntasks; t0 += 64) {
                    It x;
                    x.it.b = bi;
                    x.it.t0 = t0;
                    x.it.nt = std::min(64, ntasks - t0);
                    x.it.inst = 0;
                    x.it.slot = 0;
                    x.cost = cost;
                    items.push_back(x);
                }
            }
    // Static, deterministic assignment.  One slot per resident wave (compute
    // units x waves per CU).  Workgroups are dispatched to the XCDs round
    // robin, so slot s runs on XCD s % nx and each XCD has its own L2.  The
    // items, ordered by canonical row, rotation, b and task, are cut into nx
    // contiguous runs of equal cost, one per XCD, so that a canonical row and
    // a b's pair products are fetched into one L2 only.  Within an XCD the
    // run is dealt to its slots in snake order: the slots walk through the run
    // nearly in lockstep (sharing the rows in flight) and receive similar
    // total cost.
    std::stable_sort(items.begin(), items.end(), [&](const It &a, const It &b) {
        const T1B &A = bd[a.it.b], &Bb = bd[b.it.b];
        if (A.kc != Bb.kc) return A.kc < Bb.kc;
        if (A.rot != Bb.rot) return A.rot < Bb.rot;
        if (a.it.b != b.it.b) return a.it.b < b.it.b;
        return a.it.t0 < b.it.t0;
    });
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = trilinear_blocks_per_cu(P->p.precision == BNQ_FP32C ? 1 : 0, N);
    if (cus <= 0 || per_cu <= 0) return fail(BNQ_EHIP, "trilinear occupancy query failed");
    const int nx = P->tune.xcd ? std::max(1, cus / kCusPerXcd) : 1;
    int ns_want = std::min(kMaxSlots, std::max(1, cus * per_cu / std::max(1, P->tune.slot_div)));
    ns_want = std::max(nx, ns_want - ns_want % nx);
    if (P->p.schedule == BNQ_SCHED_DYNAMIC) {
        // one queue per XCD run of the sorted items; every resident wave runs
        std::vector<int> qoff(1, 0);
        double total = 0, acc = 0;
        for (const It &x : items) total += x.cost;
        std::vector<T1Item> flat;
        std::vector<float> fcost;
        flat.reserve(items.size());
        size_t i = 0;
        for (int x = 0; x < nx; ++x) {
            const double cut = total * (x + 1) / nx;
            for (; i < items.size() && (x == nx - 1 || acc + 0.5 * items[i].cost <= cut); ++i) {
                acc += items[i].cost;
                flat.push_back(items[i].it);
                fcost.push_back((float)items[i].cost);
            }
            qoff.push_back((int)flat.size());
        }
        P->nslots = ns_want;
        P->nbdesc = (int)bd.size();
        P->nq = nx;
        P->items_h = flat;
        P->icost_h = fcost;
        P->off_h = qoff;
        bnq_status st;
        P->nchunk = t1_chunks(t1_terms(d, N));
        if ((st = upload(&P->bdesc, bd, "trilinear b descriptors")) ||
            (!flat.empty() && (st = upload(&P->items, flat, "trilinear items"))) ||
            (st = upload(&P->t1cut, t1_cuts(qoff, fcost, P->nchunk), "trilinear queues")) ||
            (st = dalloc(&P->qctr, (size_t)((nx + 1) & ~1), "trilinear queue tickets")))
            return st;
        return dalloc(&P->part, (size_t)ns_want * g.nm, "trilinear partial sums");
    }
    const int ns = (int)std::max<size_t>(1, std::min<size_t>(ns_want, items.size()));
    std::vector<std::vector<It>> per(ns);
    if (ns < ns_want) {
        for (size_t i = 0; i < items.size(); ++i) per[i].push_back(items[i]);
    } else {
        double total = 0;
        for (const It &x : items) total += x.cost;
        const int spx = ns / nx;  // slots per XCD
        size_t i = 0;
        double acc = 0;
        for (int x = 0; x < nx; ++x) {
            const double cut = total * (x + 1) / nx;
            size_t k = 0;
            for (; i < items.size() && (x == nx - 1 || acc + 0.5 * items[i].cost <= cut); ++i, ++k) {
                acc += items[i].cost;
                const size_t round = k / spx, j = k % spx;
                const size_t sj = (round & 1) ? spx - 1 - j : j;
                per[x + nx * sj].push_back(items[i]);
            }
        }
    }
    std::vector<int> off(ns + 1, 0);
    std::vector<T1Item> flat;
    std::vector<float> fcost;
    flat.reserve(items.size());
    for (int s = 0; s < ns; ++s) {
        off[s] = (int)flat.size();
        for (const It &x : per[s]) {
            flat.push_back(x.it);
            flat.back().slot = s;
            fcost.push_back((float)x.cost);
        }
    }
    off[ns] = (int)flat.size();
    P->nslots = ns;
    P->nbdesc = (int)bd.size();
    P->items_h = flat;
    P->icost_h = fcost;
    P->off_h = off;
    P->nchunk = t1_chunks(t1_terms(d, N));
    bnq_status st;
    if ((st = upload(&P->bdesc, bd, "trilinear b descriptors")) || (st = upload(&P->items, flat, "trilinear items")) ||
        (st = upload(&P->t1cut, t1_cuts(off, fcost, P->nchunk), "trilinear slot ranges")))
        return st;
    return dalloc(&P->part, (size_t)ns * g.nm, "trilinear partial sums");
}

// FP32c: groups of b for the matrix-core kernel and their items (a group and
// a block of T1M_BLOCK outputs of its window).  The groups, ordered by
// canonical row, are cut into one contiguous run of equal cost per XCD and
// dealt to that XCD's workgroups in snake order (static schedule), or made
// the XCD's queue (dynamic schedule), as for the FP64 kernel.
bnq_status build_t1_work_mfma(bnq_plan_s *P) {
    const Geo &g = P->g;
    const TableSet *t = P->tabs;
    const int d = g.d, N = g.N, h = g.h;
    std::vector<T1G> gd;
    std::vector<std::array<int, 3>> glo, ghi;  // member window edges (lower edge lo_j of the rotated I_N)
    std::map<std::pair<int, int>, int> gidx;   // (row, lo_x) -> group
    const int b0lo = d == 3 ? -N + 1 : 0, b0hi = d == 3 ? N - 2 : 0;
    for (int b0 = b0lo; b0 <= b0hi; ++b0)
        for (int b1 = -N + 1; b1 <= N - 2; ++b1)
            for (int b2 = -N + 1; b2 <= N - 2; ++b2) {
                const int b[3] = {b0, b1, b2};
                int bc[3], perm[3], sgn[3];
                canonicalize(d, b, bc, perm, sgn);
                const int rot = rot_index(P->grp, perm, sgn);
                const int kc = t->canon_row[((size_t)bc[0] * N + bc[1]) * N + bc[2]];
                if (rot < 0 || kc < 0) return fail(BNQ_EINVAL, "internal: canonical form of b not found");
                int lo[3];
                for (int i = 0; i < 3; ++i) lo[perm[i]] = (d == 2 && i == 0) ? 0 : -h + (sgn[i] < 0 ? 1 : 0);
                bool empty = false;
                for (int j = 0; j < 3; ++j) {
                    if (d == 2 && j == 0) continue;
                    const int L0 = lo[j], H0 = lo[j] + N - 1, c = bc[j];
                    if (L0 + c > H0 || std::max(L0, c - H0) > std::min(H0, c - L0)) empty = true;
                }
                if (empty) continue;
                const auto key = std::make_pair(kc, d == 3 ? lo[2] : 0);
                auto it = gidx.find(key);
                int gi;
                if (it == gidx.end()) {
                    gi = (int)gd.size();
                    gidx[key] = gi;
                    T1G G{};
                    G.kc = kc;
                    for (int j = 0; j < 3; ++j) G.bc[j] = bc[j];
                    gd.push_back(G);
                    glo.push_back({INT32_MAX, INT32_MAX, INT32_MAX});
                    ghi.push_back({INT32_MIN, INT32_MIN, INT32_MIN});
                } else {
                    gi = it->second;
                }
                T1G &G = gd[gi];
                if (G.nrot >= 24) return fail(BNQ_EINVAL, "internal: more than 24 rotations in a trilinear group");
                G.rot[G.nrot++] = rot;
                for (int j = 0; j < 3; ++j) {
                    glo[gi][j] = std::min(glo[gi][j], lo[j]);
                    ghi[gi][j] = std::max(ghi[gi][j], lo[j]);
                }
            }
    struct It {
        T1Item it;
        double cost;
    };
    std::vector<It> items;
    for (size_t gi = 0; gi < gd.size(); ++gi) {
        T1G &G = gd[gi];
        for (int j = 0; j < 3; ++j) {
            if (d == 2 && j == 0) {
                G.wn0[j] = G.wp0[j] = 0;
                G.wnl[j] = G.wpl[j] = 1;
                continue;
            }
            const int c = G.bc[j], la = glo[gi][j], lb = ghi[gi][j];
            // outputs: lo + c .. lo + N - 1; inner: max(lo, c - lo - N + 1) .. min(lo + N - 1, c - lo)
            G.wn0[j] = la + c;
            G.wnl[j] = lb + N - 1 - (la + c) + 1;
            const int p0 = std::min(std::max(la, c - la - N + 1), std::max(lb, c - lb - N + 1));
            const int p1 = std::max(std::min(la + N - 1, c - la), std::min(lb + N - 1, c - lb));
            G.wp0[j] = p0;
            G.wpl[j] = p1 - p0 + 1;
        }
        const int W = G.wnl[0] * G.wnl[1] * G.wnl[2];
        const double rows = (double)G.wpl[0] * G.wpl[1];
        const int KS = (G.wpl[2] + 3) / 4, NT = (2 * G.nrot + 15) / 16;
        // the kernel stages rows of more than 64 inner values for at most 8 rotations
        if (4 * KS > 64 && G.nrot > 8) return fail(BNQ_ENOTSUP, "trilinear rows of %d values in 3-D", G.wpl[2]);
        const double cost = rows * (KS * NT * 2 * 32 + 150) + NT * 8 * 1000;
        for (int mb = 0; mb * T1M_BLOCK < W; ++mb) {
            // kernel-mode values the item stages per row: its output x-lines
            // times every n'_x - p'_x
            const int lnx = G.wnl[2], m0 = mb * T1M_BLOCK;
            const int nlines = (std::min(m0 + T1M_BLOCK, W) - 1) / lnx - m0 / lnx + 1;
            const int lw4 = (lnx + 4 * KS - 1 + 3) & ~3;  // line stride in LDS
            if (nlines * lw4 > T1M_KLINE)
                return fail(BNQ_ENOTSUP, "trilinear item stages %d kernel-mode values per row (at most %d)",
                            nlines * lw4, T1M_KLINE);
            It x;
            x.it.b = (int)gi;
            x.it.t0 = mb;
            x.it.nt = 0;
            x.it.inst = 0;
            x.it.slot = 0;
            x.cost = cost;
            items.push_back(x);
        }
    }
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = trilinear_blocks_per_cu(1, N);
    if (cus <= 0 || per_cu <= 0) return fail(BNQ_EHIP, "trilinear occupancy query failed");
    const int nx = P->tune.xcd ? std::max(1, cus / kCusPerXcd) : 1;
    int nwg = std::min(kMaxSlots / T1M_WAVES, std::max(1, cus * per_cu / std::max(1, P->tune.slot_div)));
    nwg = std::max(nx, nwg - nwg % nx);
    double total = 0;
    for (const It &x : items) total += x.cost;
    std::vector<int> off(1, 0);
    std::vector<T1Item> flat;
    std::vector<float> fcost;
    flat.reserve(items.size());
    if (P->p.schedule == BNQ_SCHED_DYNAMIC) {
        size_t i = 0;
        double acc = 0;
        for (int x = 0; x < nx; ++x) {
            const double cut = total * (x + 1) / nx;
            for (; i < items.size() && (x == nx - 1 || acc + 0.5 * items[i].cost <= cut); ++i) {
                acc += items[i].cost;
                flat.push_back(items[i].it);
                fcost.push_back((float)items[i].cost);
            }
            off.push_back((int)flat.size());
        }
        P->nq = nx;
    } else {
        std::vector<std::vector<It>> per(nwg);
        const int wpx = nwg / nx;  // workgroups per XCD
        size_t i = 0;
        double acc = 0;
        for (int x = 0; x < nx; ++x) {
            const double cut = total * (x + 1) / nx;
            size_t k = 0;
            for (; i < items.size() && (x == nx - 1 || acc + 0.5 * items[i].cost <= cut); ++i, ++k) {
                acc += items[i].cost;
                const size_t round = k / wpx, j = k % wpx;
                const size_t sj = (round & 1) ? wpx - 1 - j : j;
                per[x + nx * sj].push_back(items[i]);
            }
        }
        off.assign(nwg + 1, 0);
        for (int w = 0; w < nwg; ++w) {
            off[w] = (int)flat.size();
            for (const It &x : per[w]) {
                flat.push_back(x.it);
                flat.back().slot = w;
                fcost.push_back((float)x.cost);
            }
        }
        off[nwg] = (int)flat.size();
    }
    P->nslots = nwg * T1M_WAVES;
    P->nbdesc = (int)gd.size();
    P->items_h = flat;
    P->icost_h = fcost;
    P->off_h = off;
    P->nchunk = t1_chunks(t1_terms(d, N));
    bnq_status st;
    if ((st = upload(&P->gdesc, gd, "trilinear groups")) ||
        (!flat.empty() && (st = upload(&P->items, flat, "trilinear items"))) ||
        (st = upload(&P->t1cut, t1_cuts(off, fcost, P->nchunk), P->nq ? "trilinear queues" : "trilinear lists")) ||
        (P->nq && (st = dalloc(&P->qctr, (size_t)((P->nq + 1) & ~1), "trilinear queue tickets"))))
        return st;
    return dalloc(&P->part, (size_t)P->nslots * g.nm, "trilinear partial sums");
}

// Rebuilds the trilinear work lists and partial arrays for P->tune.
bnq_status rebuild_t1(bnq_plan_s *P, hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    hipFree(P->bdesc);
    hipFree(P->gdesc);
    hipFree(P->items);
    hipFree(P->t1cut);
    hipFree(P->part);
    hipFree(P->qctr);
    P->qctr = nullptr;
    P->nq = 0;
    P->bdesc = nullptr;
    P->gdesc = nullptr;
    P->items = nullptr;
    P->t1cut = nullptr;
    P->part = nullptr;
    bnq_status st = build_t1_work(P);
    if (st) return st;
    P->ih.part = P->part;
    P->ih.nslots = P->nslots;
    P->ih.t1d = P->p.precision == BNQ_FP32C ? (const void *)P->gdesc : (const void *)P->bdesc;
    HIPCHK(hipMemcpy(P->inst_d, &P->ih, sizeof(Inst), hipMemcpyHostToDevice));
    return BNQ_OK;
}

void destroy_plan(bnq_plan_s *P) {
    if (!P) return;
    hipFree(P->rots_d);
    hipFree(P->tw);
    hipFree(P->Ghat);
    hipFree(P->tmp);
    hipFree(P->tmp2);
    hipFree(P->Gr);
    hipFree(P->W);
    hipFree(P->ppart);
    hipFree(P->xpart);
    hipFree(P->Qc);
    hipFree(P->T1);
    hipFree(P->X);
    hipFree(P->Qh);
    hipFree(P->part);
    hipFree(P->G32);
    hipFree(P->Gr32);
    for (double *k : P->kbuf) hipFree(k);
    hipFree(P->ybuf);
    hipFree(P->mom_part);
    hipFree(P->mom_out);
    if (P->health) hipHostFree(P->health);
    hipFree(P->ginv);
    hipFree(P->dmat);
    hipFree(P->t1cut);
    hipFree(P->items);
    hipFree(P->bdesc);
    hipFree(P->gdesc);
    hipFree(P->inst_d);
    hipFree(P->qctr);
    hipFree(P->sep_al);
    hipFree(P->sep_alp);
    hipFree(P->sep_gc);
    hipFree(P->sep_gt);
    hipFree(P->sep_part);
    for (auto &e : P->evs) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    for (auto e : P->pool) hipEventDestroy(e);
    if (P->tabs) release_tables(P->tabs);
    delete P;
}

// One trilinear sum over the work of a set of instances: a plan alone, a
// batch group, or every instance of a batch whose sums share one launch.  The
// set's lists (static) or queues (dynamic) hold, per slot or queue, the
// instances' own items one instance after the other, so that every
// instance's partial sums are formed in exactly the order of its solo
// evaluation (static schedule).  nchunk launches walk the ranges t1cut.
struct TriSet {
    int prec = 0;               // 0 FP64, 1 FP32c
    int Nmax = 0;               // largest N of the set (selects the matrix-core variant)
    int nslots = 0;             // partial arrays the launch writes per instance (at most)
    int nq = 0;                 // dynamic schedule: queues (0 = static)
    int nchunk = 1;
    const int *t1cut = nullptr; // (nchunk + 1) x (nq or lists) item ranges
    const T1Item *items = nullptr;
    const Inst *D = nullptr;    // the instances the items index
    int *qctr = nullptr;        // queue tickets (dynamic)
};

// A set of instances evaluated together: one plan alone, or the instances of
// a batch that share geometry and tables.  Kernels index the device array D.
// The trilinear sum runs over tri, or, in a batch (tri_shared), in a launch
// shared with the instances of other groups.
struct Exec {
    Geo g;
    const TableSet *t = nullptr;
    const double2 *tw = nullptr;
    const Rot *rots = nullptr;
    int nrot = 0;
    TriSet tri;
    bool tri_shared = false;
    const Inst *D = nullptr;
    int prec = 0;               // 0 FP64, 1 FP32c
    bool otf = false;           // FP64: pair weights formed on the fly
    int sepP = 0;               // > 0: trilinear term by the separated-kernel route
    const double2 *sep_gc = nullptr;
    double2 *sep_gt = nullptr, *sep_part = nullptr;
    std::vector<Inst> Dh;       // host copies of D
    bnq_plan_s *timer = nullptr;  // plan whose timing spans record this run
};

Exec exec_of(bnq_plan_s *P) {
    Exec E;
    E.g = P->g;
    E.t = P->tabs;
    E.tw = P->tw;
    E.rots = P->rots_d;
    E.nrot = (int)P->grp.size();
    E.D = P->inst_d;
    E.prec = P->p.precision == BNQ_FP32C ? 1 : 0;
    E.tri.prec = E.prec;
    E.tri.Nmax = P->g.N;
    E.tri.nslots = P->nslots;
    E.tri.nq = P->nq;
    E.tri.nchunk = P->nchunk;
    E.tri.t1cut = P->t1cut;
    E.tri.items = P->items;
    E.tri.D = P->inst_d;
    E.tri.qctr = P->qctr;
    E.otf = P->otf;
    E.sepP = P->sepP;
    E.sep_gc = P->sep_gc;
    E.sep_gt = P->sep_gt;
    E.sep_part = P->sep_part;
    E.Dh.assign(1, P->ih);
    E.timer = P;
    return E;
}

// Chunks of at most BNQ_MAXB instances, IOs filled by fill(io, z, instance).
template <typename F>
std::vector<IOs> make_ios(int n, const double *dt, F fill) {
    std::vector<IOs> v;
    for (int z0 = 0; z0 < n; z0 += BNQ_MAXB) {
        IOs io;
        std::memset(&io, 0, sizeof io);
        io.n = std::min(BNQ_MAXB, n - z0);
        for (int z = 0; z < io.n; ++z) {
            io.inst[z] = z0 + z;
            io.dt[z] = dt ? dt[z0 + z] : 0.0;
            fill(io, z, z0 + z);
        }
        v.push_back(io);
    }
    return v;
}

int terms_of(const Exec &E) {
    int any = 0;
    for (const Inst &I : E.Dh) any |= I.terms;
    return any;
}

int max_slots_of(const Exec &E) {
    int m = 0;
    for (const Inst &I : E.Dh)
        if (I.terms & BNQ_T_QTRI) m = std::max(m, I.nslots);
    return m;
}

// The phases of an evaluation before its trilinear sum: spectra, pair sums,
// outer sum, and the rotated spectra and cleared partial arrays the
// trilinear sum reads and writes (or the whole separated-kernel route).
bnq_status collide_pre(const Exec &E, const std::vector<IOs> &ios, hipStream_t s) {
    const Geo &g = E.g;
    const int any = terms_of(E), max_slots = max_slots_of(E);
    {
        Span sp(E.timer, 0, s);
        for (const IOs &io : ios) {
            launch_dft_forward_real(g, E.D, io, E.tw, s);
            LAUNCHCHK();
            if (E.prec) {
                launch_spectrum_f32(g, E.D, io, s);
                LAUNCHCHK();
            }
        }
    }
    if (any & (BNQ_T_CLASSICAL | BNQ_T_QMULT)) {
        Span sp(E.timer, 1, s);
        for (const IOs &io : ios) {
            const Radial rad = E.t->radial();
            launch_pairs(g, E.prec, E.D, io, E.prec ? (const void *)E.t->wc32 : (const void *)E.t->wc,
                         E.prec ? (const void *)E.t->wq32 : (const void *)E.t->wq, (any & BNQ_T_QMULT) != 0, E.otf ? &rad : nullptr, s);
            LAUNCHCHK();
            launch_pairs_reduce(g, E.D, io, s);
            LAUNCHCHK();
        }
    }
    if (any & BNQ_T_QMULT) {
        Span sp(E.timer, 2, s);
        for (const IOs &io : ios) {
            launch_outer(g, E.D, io, s);
            LAUNCHCHK();
        }
    }
    if ((any & BNQ_T_QTRI) && E.sepP) {
        Span sp(E.timer, 3, s);
        for (const IOs &io : ios)
            for (int z = 0; z < io.n; ++z) {
                const Inst &I = E.Dh[io.inst[z]];
                if (!(I.terms & BNQ_T_QTRI)) continue;
                launch_sep_t1(g.d, g.N, E.sepP, I.Ghat, E.sep_gc, E.sep_gt, E.sep_part, I.T1, s);
                LAUNCHCHK();
            }
    } else if (any & BNQ_T_QTRI) {
        Span sp(E.timer, 4, s);
        for (const IOs &io : ios) {
            launch_rotate(g, E.prec, E.D, io, E.rots, E.nrot, s);
            LAUNCHCHK();
            launch_zero_part(g, E.D, io, max_slots, s);
            LAUNCHCHK();
        }
    }
    return BNQ_OK;
}

bool has_tri_launch(const Exec &E) { return (terms_of(E) & BNQ_T_QTRI) && !E.sepP; }

bnq_status run_tri(const TriSet &T, bnq_plan_s *timer, hipStream_t s) {
    const int nl = T.nq ? T.nq : t1_lists(T.prec, T.nslots);
    for (int r = 0; r < T.nchunk; ++r) {
        if (T.nq) {
            launch_zero(T.qctr, (int64_t)((T.nq + 1) & ~1) * (int64_t)sizeof(int), s);  // whole 8-byte words
            LAUNCHCHK();
        }
        Span sp(timer, 3, s);
        launch_trilinear(T.prec, T.Nmax, T.nslots, T.t1cut + (size_t)r * nl, T.t1cut + (size_t)(r + 1) * nl, T.items,
                         T.D, T.nq, T.qctr, s);
        LAUNCHCHK();
    }
    return BNQ_OK;
}

// The phases after the trilinear sum: partial arrays reduced, combined, the
// inverse transform, the moment projection.
bnq_status collide_post(const Exec &E, const std::vector<IOs> &ios, hipStream_t s) {
    const Geo &g = E.g;
    if (has_tri_launch(E)) {
        const int max_slots = max_slots_of(E);
        Span sp(E.timer, 4, s);
        for (const IOs &io : ios) {
            launch_reduce_partials(g, E.D, io, max_slots, s);
            LAUNCHCHK();
        }
    }
    {
        Span sp(E.timer, 5, s);
        for (const IOs &io : ios) {
            launch_combine(g, E.D, io, s);
            LAUNCHCHK();
            launch_inverse_real(g, E.D, io, E.tw, s);
            LAUNCHCHK();
        }
        int any_mom = 0;
        for (const Inst &I : E.Dh) any_mom |= I.corr_mom;
        if (any_mom)
            for (const IOs &io : ios) {
                launch_moments_fix(g, E.D, io, s);
                LAUNCHCHK();
            }
    }
    return BNQ_OK;
}

// One evaluation of every instance of the groups Es (instances and buffers
// per group in ios[i]): all groups' phases before the trilinear sums, the
// sums (each group's own launch, or the shared launches of sets), then all
// groups' phases after them.
bnq_status collide_groups(const std::vector<const Exec *> &Es, const std::vector<std::vector<IOs>> &ios,
                          const std::vector<TriSet> &sets, hipStream_t s) {
    bnq_status st;
    for (size_t i = 0; i < Es.size(); ++i)
        if ((st = collide_pre(*Es[i], ios[i], s))) return st;
    for (const Exec *E : Es)
        if (has_tri_launch(*E) && !E->tri_shared && (st = run_tri(E->tri, E->timer, s))) return st;
    for (const TriSet &T : sets)
        if ((st = run_tri(T, nullptr, s))) return st;
    for (size_t i = 0; i < Es.size(); ++i)
        if ((st = collide_post(*Es[i], ios[i], s))) return st;
    return BNQ_OK;
}

bnq_status run_collide(const Exec &E, const std::vector<IOs> &ios, hipStream_t s) {
    return collide_groups({&E}, {ios}, {}, s);
}

// One time step of every instance of the groups Es: f[i][j] (instance j of
// group i) advanced in place by dt[i][j].  Every stage evaluates all groups
// together (collide_groups), so a batch's trilinear sums share launches.
bnq_status step_groups(const std::vector<const Exec *> &Es, const std::vector<double *const *> &f,
                       const std::vector<const double *> &dt, const std::vector<TriSet> &sets, int scheme,
                       hipStream_t s) {
    if (scheme != BNQ_EULER && scheme != BNQ_SSPRK2 && scheme != BNQ_RK4)
        return fail(BNQ_EINVAL, "unknown scheme %d", scheme);
    const size_t ng = Es.size();
    auto coll = [&](int stage) {
        std::vector<std::vector<IOs>> io(ng);
        for (size_t i = 0; i < ng; ++i)
            io[i] = make_ios((int)Es[i]->Dh.size(), dt[i], [&](IOs &x, int z, int j) {
                x.in[z] = stage == 0 ? f[i][j] : Es[i]->Dh[j].ybuf;
                x.out[z] = Es[i]->Dh[j].k[stage];
            });
        return collide_groups(Es, io, sets, s);
    };
    std::vector<std::vector<IOs>> upd(ng);
    for (size_t i = 0; i < ng; ++i)
        upd[i] = make_ios((int)Es[i]->Dh.size(), dt[i], [&](IOs &x, int z, int j) {
            x.in[z] = f[i][j];
            x.out[z] = f[i][j];
        });
    // kind 0: stage value (a, ks, to_out), 1: SSP-RK2 final, 2: RK4 final
    auto update = [&](int kind, double a, int ks, int to_out) -> bnq_status {
        for (size_t i = 0; i < ng; ++i) {
            Span sp(Es[i]->timer, 6, s);
            for (const IOs &io : upd[i]) {
                if (kind == 0)
                    launch_stage(Es[i]->g, Es[i]->D, io, a, ks, to_out, s);
                else if (kind == 1)
                    launch_ssprk2_final(Es[i]->g, Es[i]->D, io, s);
                else
                    launch_rk4_final(Es[i]->g, Es[i]->D, io, s);
                LAUNCHCHK();
            }
        }
        return BNQ_OK;
    };
    bnq_status st;
    if ((st = coll(0))) return st;
    if (scheme == BNQ_EULER) return update(0, 1.0, 0, 1);
    if (scheme == BNQ_SSPRK2) {
        if ((st = update(0, 1.0, 0, 0)) || (st = coll(1))) return st;
        return update(1, 0.0, 0, 0);
    }
    const double a[3] = {0.5, 0.5, 1.0};
    for (int stg = 1; stg < 4; ++stg)
        if ((st = update(0, a[stg - 1], stg - 1, 0)) || (st = coll(stg))) return st;
    return update(2, 0.0, 0, 0);
}

// One time step of every instance of E: f[i] advanced in place by dt[i].
bnq_status run_step(const Exec &E, double *const *f, const double *dt, int scheme, hipStream_t s) {
    return step_groups({&E}, {f}, {dt}, {}, scheme, s);
}

// Status recorded in the plan's health flags by steps that have completed on
// the device (read without synchronisation): ENONFINITE before EBOUND.
bnq_status health_status(const bnq_plan_s *P, int member) {
    const volatile int *h = P->health;
    if (h[0])
        return member >= 0 ? fail(BNQ_ENONFINITE, "a step of instance %d wrote a non-finite value", member)
                           : fail(BNQ_ENONFINITE, "a step wrote a non-finite value");
    if (h[1])
        return member >= 0
                   ? fail(BNQ_EBOUND, "a step of instance %d wrote a value at or above 1/alpha (fermion bound)", member)
                   : fail(BNQ_EBOUND, "a step wrote a value at or above 1/alpha (fermion bound)");
    return BNQ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

void bnq_params_default(bnq_params *p) {
    if (!p) return;
    p->d = 3;
    p->N = 16;
    p->eps = 0;
    p->precision = BNQ_FP64;
    p->terms = BNQ_T_ALL;
    p->correction = BNQ_CORR_NONE;
    p->hbar = 1.0;
    p->C_phi = 1.0;
    p->c = 1.0;
    p->L = 8.0;
    p->schedule = BNQ_SCHED_STATIC;
    p->flags = 0;
    p->angles = 0;
}

bnq_status bnq_plan_footprint(const bnq_params *p, size_t *plan_bytes, size_t *table_bytes_out) {
    bnq_status st = validate(p);
    if (st) return st;
    if (plan_bytes) *plan_bytes = plan_workspace_bytes(p, kMaxSlots);
    if (table_bytes_out) {
        // the radial tables of a new table set, plus the kernel-mode tables
        // of the plan's precision unless the cached set already has them
        // (FP64 with weights on the fly: the trilinear rows only)
        const bool f32 = p->precision == BNQ_FP32C, otf = (p->flags & BNQ_FLAG_WEIGHTS_OTF) != 0;
        Geo g = make_geo(p->d, p->N);
        const size_t wbytes = sizeof(double) * 2 * (size_t)g.nm * g.nm;
        const size_t km = f32 ? table_bytes_f32(p->d, p->N) : table_bytes_f64(p->d, p->N) - (otf ? wbytes : 0);
        size_t tb = table_bytes_radial(p->d, p->N) + km;
        std::lock_guard<std::mutex> lk(g_cache_mu);
        int dev = 0;
        hipGetDevice(&dev);
        for (TableSet *t : g_cache)
            if (t->d == p->d && t->N == p->N && t->Cphi == p->C_phi && t->device == dev)
                tb = f32 ? (t->K32 ? 0 : km) : (t->K ? (otf || t->wc ? 0 : wbytes) : km);
        *table_bytes_out = tb;
    }
    return BNQ_OK;
}

bnq_status bnq_plan(const bnq_params *p, bnq_stream_t stream, bnq_plan_t *out) {
    if (!out) return fail(BNQ_EINVAL, "out is NULL");
    *out = nullptr;
    bnq_status st = validate(p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    bnq_plan_s *P = new bnq_plan_s;
    P->p = *p;
    P->g = make_geo(p->d, p->N);
    P->g.psplit = pair_split_default(p->d, p->N, p->eps);
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_pairs.find(std::make_tuple(dev, p->d, p->N, (int)p->precision, p->eps == 0 ? 1 : 0));
        if (it != g_tune_pairs.end()) P->g.psplit = it->second;
    }
    const Geo &g = P->g;
    P->alpha = -(double)p->eps * std::pow(p->hbar, p->d);
    P->pref = p->c * std::pow(p->L / M_PI, p->d + (p->d == 3 ? 1 : 0));
    P->grp = make_group(p->d);
    P->last = s;
    bool have_w = true;
    if ((st = acquire_tables(p->d, p->N, p->C_phi, p->precision, !(p->flags & BNQ_FLAG_WEIGHTS_OTF), s, &P->tabs,
                             &have_w))) {
        destroy_plan(P);
        return st;
    }
    P->otf = p->precision == BNQ_FP64 && (!have_w || (p->flags & BNQ_FLAG_WEIGHTS_OTF));
    std::vector<double2> tw(p->N);
    for (int t = 0; t < p->N; ++t) {
        const long double a = 2.0L * (long double)M_PI * t / p->N;
        tw[t] = make_double2((double)std::cos(a), (double)-std::sin(a));
    }
    // D[j][m] = Re of (inverse DFT . i k . DFT) along one axis, k in I_N:
    // -(1/N) sum_k k sin(2 pi k (j - m) / N)
    std::vector<double> dm((size_t)p->N * p->N);
    for (int j = 0; j < p->N; ++j)
        for (int m = 0; m < p->N; ++m) {
            long double acc = 0;
            for (int k = -p->N / 2; k < p->N / 2; ++k)
                acc -= k * std::sin(2.0L * (long double)M_PI * k * (j - m) / p->N);
            dm[(size_t)j * p->N + m] = (double)(acc / p->N);
        }
    const size_t nm = g.nm;
    if ((st = upload(&P->rots_d, P->grp, "rotations")) || (st = upload(&P->tw, tw, "twiddles")) ||
        (st = upload(&P->dmat, dm, "differentiation matrix")) ||
        (st = dalloc(&P->Ghat, nm, "spectrum")) || (st = dalloc(&P->tmp, nm, "dft scratch")) ||
        (st = dalloc(&P->tmp2, nm, "dft scratch")) || (st = dalloc(&P->Gr, P->grp.size() * (size_t)g.next, "rotated spectra")) ||
        (st = dalloc(&P->W, (size_t)g.neg, "pair sum W")) || (st = dalloc(&P->Qc, nm, "classical modes")) ||
        (st = dalloc(&P->ppart, (size_t)pair_split_max(g.N) * ((size_t)g.neg + nm), "pair sum slices")) ||
        (st = dalloc(&P->xpart, (size_t)outer_split(g) * nm, "outer sum slices")) ||
        (st = dalloc(&P->T1, nm, "trilinear modes")) || (st = dalloc(&P->X, nm, "outer modes")) ||
        (st = dalloc(&P->Qh, nm, "modes")) || (st = dalloc(&P->ybuf, nm, "stage")) ||
        (st = dalloc(&P->mom_part, moments_scratch_doubles(MOM_BLOCKS), "moment partials")) ||
        (st = dalloc(&P->mom_out, (size_t)MOM_OUT, "moments"))) {
        destroy_plan(P);
        return st;
    }
    for (int k = 0; k < 4; ++k)
        if ((st = dalloc(&P->kbuf[k], nm, "stage"))) {
            destroy_plan(P);
            return st;
        }
    {
        const hipError_t e = hipHostMalloc((void **)&P->health, 2 * sizeof(int), hipHostMallocCoherent);
        if (e != hipSuccess) {
            P->health = nullptr;
            destroy_plan(P);
            return fail(BNQ_ENOMEM, "health flags: %s", hipGetErrorString(e));
        }
        P->health[0] = P->health[1] = 0;
    }
    if (p->precision == BNQ_FP32C &&
        ((st = dalloc(&P->G32, nm, "FP32 spectrum")) ||
         (st = dalloc(&P->Gr32, P->grp.size() * (size_t)g.next, "FP32 rotated spectra")))) {
        destroy_plan(P);
        return st;
    }
    if (p->flags & BNQ_FLAG_T1_SEPARATED) {
        const int N = p->N, M = 2 * N, w = 2 * N - 1, d = p->d;
        const size_t na = d == 2 ? (size_t)w * w : (size_t)w * w * w, Md = d == 2 ? (size_t)M * M : (size_t)M * M * M,
                     Nd = d == 2 ? (size_t)N * N : (size_t)N * N * N;
        const int angles = p->angles > 0 ? p->angles : sep_auto_angles(N, kR);
        const int Pn = sep_directions(d, angles);
        int nc, jc, nbj;
        sep_shape(d, N, Pn, &nc, &jc, &nbj);
        P->sepP = Pn;
        hipError_t e = sep_prepare();
        if (e != hipSuccess) {
            destroy_plan(P);
            return fail(BNQ_EHIP, "separated route: %s", hipGetErrorString(e));
        }
        if ((st = dalloc(&P->sep_al, (size_t)Pn * na, "alpha rows")) ||
            (st = dalloc(&P->sep_alp, (size_t)Pn * na, "alpha' rows")) ||
            (st = dalloc(&P->sep_gc, (size_t)Pn * Md, "alpha transforms")) ||
            (st = dalloc(&P->sep_gt, Md, "spectrum on the doubled grid")) ||
            (st = dalloc(&P->sep_part, (size_t)Pn * nbj * Nd, "separated-route partials"))) {
            destroy_plan(P);
            return st;
        }
        launch_sep_tables(d, N, angles, kR, p->C_phi, P->sep_al, P->sep_alp, P->sep_gc, s);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
            destroy_plan(P);
            return fail(BNQ_EHIP, "separated route tables: %s", hipGetErrorString(e));
        }
    }
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(std::make_tuple(dev, p->d, p->N, (int)p->precision));
        if (it != g_tune.end()) P->tune = kTuneCandidates[it->second];
    }
    // work lists and per-slot partial arrays only for plans with the trilinear term
    if (p->eps != 0 && (p->terms & BNQ_T_QTRI) && (st = build_t1_work(P))) {
        destroy_plan(P);
        return st;
    }
    {
        Inst &I = P->ih;
        I.Ghat = P->Ghat;
        I.tmp = P->tmp;
        I.tmp2 = P->tmp2;
        I.Gr = P->Gr;
        I.W = P->W;
        I.ppart = P->ppart;
        I.xpart = P->xpart;
        I.Qc = P->Qc;
        I.T1 = P->T1;
        I.X = P->X;
        I.Qh = P->Qh;
        I.part = P->part;
        I.G32 = P->G32;
        I.Gr32 = P->Gr32;
        I.ybuf = P->ybuf;
        for (int k = 0; k < 4; ++k) I.k[k] = P->kbuf[k];
        I.alpha = P->alpha;
        I.pref = P->pref;
        I.terms = p->eps == 0 ? (p->terms & BNQ_T_CLASSICAL) : p->terms;
        I.mass_fix = p->correction == BNQ_CORR_MASS;
        I.nslots = P->nslots;
        I.corr_mom = p->correction == BNQ_CORR_MOMENTS;
        I.hstep = 2.0 * p->L / p->N;
        I.ginv = nullptr;
        I.health = P->health;
        I.fbound = (P->alpha > 0 && !(p->flags & BNQ_FLAG_NO_FERMI_BOUND)) ? 1.0 / P->alpha : INFINITY;
        I.geo = P->g;
        I.K = p->precision == BNQ_FP32C ? (const void *)P->tabs->K32 : (const void *)P->tabs->K;
        I.t1d = p->precision == BNQ_FP32C ? (const void *)P->gdesc : (const void *)P->bdesc;
        I.rots = P->rots_d;
        if (I.corr_mom) {
            std::vector<double> gi;
            if ((st = gram_inverse(p->d, p->N, I.hstep, gi)) || (st = upload(&P->ginv, gi, "moment Gram matrix"))) {
                destroy_plan(P);
                return st;
            }
            I.ginv = P->ginv;
        }
        if ((st = upload(&P->inst_d, std::vector<Inst>(1, I), "instance descriptor"))) {
            destroy_plan(P);
            return st;
        }
    }
    double c1, w1, o1, t1;
    counts_1d(p->N, c1, w1, o1, t1);
    const int d = p->d;
    P->counts[0] = std::pow(c1, d);
    P->counts[1] = std::pow(w1, d);
    P->counts[2] = std::pow(o1, d);
    P->counts[3] = std::pow(t1, d);
    *out = P;
    return BNQ_OK;
}

bnq_status bnq_plan_destroy(bnq_plan_t plan) {
    if (!plan) return BNQ_OK;
    if (plan->nbatch > 0) return fail(BNQ_EINVAL, "plan is held by %d batch(es): destroy them first", (int)plan->nbatch);
    hipStreamSynchronize(plan->last);
    destroy_plan(plan);
    return BNQ_OK;
}

bnq_status bnq_collide(bnq_plan_t P, const double *f, double *Q, void *Qhat, bnq_stream_t stream) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    if (!f || !Q) return fail(BNQ_EINVAL, "f and Q must be device pointers");
    if ((const void *)f == (const void *)Q) return fail(BNQ_EINVAL, "f and Q must not alias");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    const Exec E = exec_of(P);
    return run_collide(E, make_ios(1, nullptr, [&](IOs &io, int z, int) {
                           io.in[z] = f;
                           io.out[z] = Q;
                           io.qhat[z] = (double2 *)Qhat;
                       }), s);
}

bnq_status bnq_step(bnq_plan_t P, double *f, double dt, int32_t scheme, bnq_stream_t stream) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    if (!f) return fail(BNQ_EINVAL, "f is NULL");
    if (!std::isfinite(dt)) return fail(BNQ_EINVAL, "dt must be finite");
    bnq_status st;
    if ((st = health_status(P, -1))) return st;
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    const Exec E = exec_of(P);
    return run_step(E, &f, &dt, scheme, s);
}

bnq_status bnq_moments(bnq_plan_t P, const double *f, double *out_host, bnq_stream_t stream) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    if (!f || !out_host) return fail(BNQ_EINVAL, "f and out_host must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    {
        Span sp(P, 7, s);
        launch_moments(P->g, f, P->p.L, P->alpha, P->mom_part, MOM_BLOCKS, P->mom_out, s);
        LAUNCHCHK();
    }
    double r[MOM_OUT];
    HIPCHK(hipMemcpyAsync(r, P->mom_out, sizeof r, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < BNQ_MOMENTS_LEN; ++k) out_host[k] = r[k];
    if (r[10] > 0) return fail(BNQ_ENONFINITE, "f holds %.0f non-finite values", r[10]);
    if (P->p.eps == -1 && r[7] * std::fabs(P->alpha) >= 1.0)
        return fail(BNQ_EBOUND, "fermion bound violated: max f = %.17g >= 1/|alpha|", r[7]);
    return BNQ_OK;
}

bnq_status bnq_health(bnq_plan_t P, int32_t wait, int32_t clear, int32_t *flags_host, bnq_stream_t stream) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    if (wait) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    const int fl = (P->health[0] ? BNQ_HEALTH_NONFINITE : 0) | (P->health[1] ? BNQ_HEALTH_BOUND : 0);
    if (flags_host) *flags_host = fl;
    const bnq_status st = health_status(P, -1);
    if (clear) P->health[0] = P->health[1] = 0;
    return st;
}

bnq_status bnq_moments_noalloc(const bnq_params *p, const double *f, double *out, bnq_stream_t stream) {
    bnq_status st = validate(p);
    if (st) return st;
    if (!f || !out) return fail(BNQ_EINVAL, "f and out must be device pointers");
    const Geo g = make_geo(p->d, p->N);
    const int nblk = MOM_BLOCKS;  // as bnq_moments: the same reduction order, the same bits
    if (moments_scratch_doubles(nblk) > NOALLOC_SCRATCH_DOUBLES)
        return fail(BNQ_EINVAL, "N^d = %lld needs %zu doubles of scratch, more than the %zu available", (long long)g.nm,
                    moments_scratch_doubles(nblk), NOALLOC_SCRATCH_DOUBLES);
    double *scr = nullptr;
    const hipError_t e = noalloc_scratch(&scr);
    if (e != hipSuccess) return fail(BNQ_EHIP, "static scratch address: %s", hipGetErrorString(e));
    const double alpha = -(double)p->eps * std::pow(p->hbar, p->d);
    launch_moments(g, f, p->L, alpha, scr, nblk, out, (hipStream_t)stream);
    LAUNCHCHK();
    return BNQ_OK;
}

bnq_status bnq_equilibrium_solve(int32_t d, int32_t eps, double hbar, double rho, const double *u, double e,
                                 bnq_equilibrium *out) {
    if (!out) return fail(BNQ_EINVAL, "out is NULL");
    if (eps < -1 || eps > 1) return fail(BNQ_EINVAL, "eps must be -1, 0 or 1 (got %d)", eps);
    if (!(hbar > 0) || !std::isfinite(hbar)) return fail(BNQ_EINVAL, "hbar must be positive and finite");
    const double alpha = -(double)eps * std::pow(hbar, d == 3 ? 3 : 2);
    char err[256] = "";
    const int st = solve_equilibrium(d, alpha, rho, u, e, out, err, sizeof err);
    if (st) return fail((bnq_status)st, "%s", err);
    return BNQ_OK;
}

bnq_status bnq_fd_be_log(double nu, int32_t fermi, double p, double *out) {
    if (!out) return fail(BNQ_EINVAL, "out is NULL");
    if (!(nu >= 1.0) || !std::isfinite(nu) || !std::isfinite(p) || (!fermi && !(p >= 0.0)) ||
        (!fermi && nu <= 1.0 && p == 0.0))
        return fail(BNQ_EINVAL, "need nu >= 1, finite p, and p >= 0 (p > 0 for nu = 1) for Bose-Einstein");
    *out = complete_fd_be_log(nu, fermi ? 1 : 0, p);
    return BNQ_OK;
}

}  // extern "C"

namespace {

// device form of a limit state for the plan's grid
bnq_status eq_dev(const bnq_plan_s *P, const bnq_equilibrium *q, EqDev &E) {
    if (!q) return fail(BNQ_EINVAL, "equilibrium is NULL");
    if (q->d != P->g.d) return fail(BNQ_EINVAL, "equilibrium of d = %d for a plan of d = %d", q->d, P->g.d);
    const int d = q->d;
    E.kind = q->kind;
    E.d = d;
    E.bose = q->alpha < 0;
    for (int i = 0; i < 3; ++i) E.u[i] = q->u[i];
    E.log_z = q->log_z;
    E.T = q->T;
    E.A2 = 0;
    switch (q->kind) {
        case BNQ_EQ_MAXWELL: E.c0 = q->rho * std::pow(2.0 * M_PI * q->T, -0.5 * d); break;
        case BNQ_EQ_QUANTUM: E.c0 = 1.0 / std::fabs(q->alpha); break;
        case BNQ_EQ_CONDENSATE:
            E.c0 = 1.0 / std::fabs(q->alpha);
            E.bose = 1;
            E.log_z = 0.0;
            break;
        case BNQ_EQ_SATURATED:
            E.A2 = q->A * q->A;
            E.c0 = q->rho / (std::pow(M_PI, 0.5 * d) * std::pow(q->A, d) / std::tgamma(0.5 * d + 1.0));
            break;
        default: return fail(BNQ_EINVAL, "no limit state identified (kind %d)", q->kind);
    }
    if (q->kind != BNQ_EQ_SATURATED && !(E.T > 0)) return fail(BNQ_EINVAL, "temperature must be positive");
    return BNQ_OK;
}

}  // namespace

extern "C" {

bnq_status bnq_equilibrium_fill(bnq_plan_t P, const bnq_equilibrium *q, double *out, bnq_stream_t stream) {
    if (!P || !out) return fail(BNQ_EINVAL, "plan and out must be non-NULL");
    EqDev E;
    bnq_status st = eq_dev(P, q, E);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    launch_equilibrium(P->g, P->p.L, E, nullptr, out, nullptr, MOM_BLOCKS, nullptr, s);
    LAUNCHCHK();
    return BNQ_OK;
}

bnq_status bnq_equilibrium_distance(bnq_plan_t P, const double *f, const bnq_equilibrium *q, double *out_host,
                                    bnq_stream_t stream) {
    if (!P || !f || !out_host) return fail(BNQ_EINVAL, "plan, f and out_host must be non-NULL");
    EqDev E;
    bnq_status st = eq_dev(P, q, E);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    static_assert(EQ_FIELDS <= MOM_FIELDS, "moment buffers hold the distance partials");
    launch_equilibrium(P->g, P->p.L, E, f, nullptr, P->mom_part, MOM_BLOCKS, P->mom_out, s);
    LAUNCHCHK();
    double r[EQ_FIELDS];
    HIPCHK(hipMemcpyAsync(r, P->mom_out, sizeof r, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double dv = std::pow(2.0 * P->p.L / P->p.N, P->p.d);
    out_host[0] = dv * r[0];
    out_host[1] = r[1];
    out_host[2] = dv * r[2];
    out_host[3] = r[3];
    out_host[4] = dv * r[4];
    return BNQ_OK;
}

}  // extern "C"

namespace {

// Sums of x over the xi grid (xi_j = 2 pi j / N): r[0] = sum x, r[1..3] =
// sum xi x per storage axis, r[4] = sum |xi|^2 x (the moment kernel on a box
// of half-width pi).
bnq_status xi_sums(bnq_plan_s *P, const double *x, hipStream_t s, double r[5]) {
    launch_moments(P->g, x, M_PI, 0.0, P->mom_part, MOM_BLOCKS, P->mom_out, s);
    LAUNCHCHK();
    double buf[MOM_FIELDS];
    HIPCHK(hipMemcpyAsync(buf, P->mom_part + moments_sums_offset(MOM_BLOCKS), sizeof buf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (buf[9] > 0) return fail(BNQ_ENONFINITE, "%.0f non-finite values", buf[9]);
    for (int k = 0; k < 5; ++k) r[k] = buf[k];
    return BNQ_OK;
}

// limit state of (rho, u, e) into st (T, log_z, kind); EINVAL when it has no
// finite temperature
bnq_status rescaled_limit(const bnq_plan_s *P, bnq_rescaled_state *st) {
    bnq_equilibrium q;
    char err[256] = "";
    const int rc = solve_equilibrium(P->g.d, P->alpha, st->rho, st->u, st->e, &q, err, sizeof err);
    if (rc) return fail((bnq_status)rc, "%s", err);
    if (q.kind == BNQ_EQ_SATURATED || q.kind == BNQ_EQ_UNKNOWN)
        return fail(BNQ_EINVAL, "degenerate Fermi-Dirac moments (ratio %.17g): no finite temperature", q.ratio);
    st->T = q.T;
    st->log_z = q.log_z;
    st->kind = q.kind;
    return BNQ_OK;
}

}  // namespace

extern "C" {

bnq_status bnq_rescaled_init(bnq_plan_t P, const double *G, double omega, const double *u_ref,
                             bnq_rescaled_state *st, bnq_stream_t stream) {
    if (!P || !G || !u_ref || !st) return fail(BNQ_EINVAL, "plan, G, u_ref and st must be non-NULL");
    if (!(omega > 0) || !std::isfinite(omega)) return fail(BNQ_EINVAL, "omega must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    const int d = P->g.d, off = d == 3 ? 0 : 1;  // storage axis of u[0]
    double r[5];
    bnq_status rc = xi_sums(P, G, s, r);
    if (rc) return rc;
    const double dxi = std::pow(2.0 * M_PI / P->g.N, d), a = P->p.L / (M_PI * omega);
    bnq_rescaled_state n{};
    n.omega = omega;
    n.rho = dxi * r[0];
    if (!(n.rho > 0)) return fail(BNQ_EINVAL, "G has no positive mass");
    double cr = 0, c2 = 0;  // (u_ref - u) . sum xi G and |u_ref - u|^2
    for (int i = 0; i < d; ++i) {
        n.u[i] = a * dxi * r[1 + off + i] / n.rho + u_ref[i];
        cr += (u_ref[i] - n.u[i]) * r[1 + off + i];
        c2 += (u_ref[i] - n.u[i]) * (u_ref[i] - n.u[i]);
    }
    n.e = 0.5 * dxi * (a * a * r[4] + 2.0 * a * cr + c2 * r[0]) / n.rho;
    if ((rc = rescaled_limit(P, &n))) return rc;
    *st = n;
    return BNQ_OK;
}

bnq_status bnq_step_rescaled(bnq_plan_t P, double *G, bnq_rescaled_state *st, double dt, bnq_stream_t stream) {
    if (!P || !G || !st) return fail(BNQ_EINVAL, "plan, G and st must be non-NULL");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(BNQ_EINVAL, "dt must be positive and finite");
    if (!(st->omega > 0) || !(st->rho > 0) || !(st->e > 0))
        return fail(BNQ_EINVAL, "state needs omega, rho and e positive");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    const Geo &g = P->g;
    const int d = g.d, off = d == 3 ? 0 : 1;
    const double L = P->p.L, om = st->omega, sc = M_PI * om / L;
    // the plan's operator with the quantum parameter alpha s^d and the
    // prefactor c s^-gamma, for this evaluation only
    Inst I = P->ih;
    I.alpha = P->alpha * std::pow(sc, d);
    I.pref = P->p.c * std::pow(sc, -(double)(d == 3 ? 1 : 0));
    HIPCHK(hipMemcpyAsync(P->inst_d, &I, sizeof I, hipMemcpyHostToDevice, s));
    Exec E = exec_of(P);
    E.Dh[0] = I;
    double *K = P->kbuf[0];
    const std::vector<IOs> io = make_ios(1, nullptr, [&](IOs &x, int z, int) {
        x.in[z] = G;
        x.out[z] = K;
    });
    bnq_status rc = run_collide(E, io, s);
    HIPCHK(hipMemcpyAsync(P->inst_d, &P->ih, sizeof(Inst), hipMemcpyHostToDevice, s));
    if (rc) {
        hipStreamSynchronize(s);  // I is read by the copy above
        return rc;
    }
    double r[5];
    if ((rc = xi_sums(P, K, s, r))) return rc;
    const double dxi = std::pow(2.0 * M_PI / g.N, d), a = L / (M_PI * om);
    bnq_rescaled_state n = *st;
    n.rho = st->rho + dt * dxi * r[0];
    double u2 = 0;
    for (int i = 0; i < d; ++i) {
        n.u[i] = (st->rho * st->u[i] + dt * dxi * (a * r[1 + off + i] + st->u[i] * r[0])) / n.rho;
        u2 += n.u[i] * n.u[i];
    }
    n.e = (st->rho * st->e + dt * 0.5 * dxi * a * a * r[4]) / n.rho;
    if ((rc = rescaled_limit(P, &n))) return rc;
    n.omega = P->alpha != 0.0 ? std::sqrt(n.T) : std::sqrt(n.T + u2 / d);
    const double A = (n.omega - om) / (dt * om);
    double B3[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) B3[off + i] = sc * (n.u[i] - st->u[i]) / dt;
    launch_drift_update(g, G, K, P->dmat, A, B3, dt, P->ybuf, s);
    LAUNCHCHK();
    launch_copy(G, P->ybuf, g.nm, s);
    LAUNCHCHK();
    *st = n;
    return BNQ_OK;
}

bnq_status bnq_table_lookup(bnq_plan_t P, int32_t table, int64_t n, const int32_t *a, const int32_t *b,
                            double *out) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    if (n < 0 || (n > 0 && (!a || !b || !out))) return fail(BNQ_EINVAL, "bad arrays");
    if (n == 0) return BNQ_OK;
    const Geo &g = P->g;
    const TableSet *t = P->tabs;
    const int N = g.N, h = g.h, d = g.d;
    std::vector<int64_t> idx(n);
    for (int64_t i = 0; i < n; ++i) {
        const int *x = a + 3 * i, *y = b + 3 * i;
        if (d == 2 && (x[0] != 0 || y[0] != 0)) return fail(BNQ_EINVAL, "d = 2 vectors need component 0 = 0");
        if (table == 0) {
            for (int c = 0; c < 3; ++c)
                if (std::abs(x[c]) > N - 1 || std::abs(y[c]) > N - 1)
                    return fail(BNQ_EINVAL, "pair %lld outside the trilinear table range", (long long)i);
            int bc[3], perm[3], sgn[3];
            canonicalize(d, y, bc, perm, sgn);
            int ap[3];
            for (int c = 0; c < 3; ++c) ap[perm[c]] = sgn[c] * x[c];
            const int kc = t->canon_row[((size_t)bc[0] * N + bc[1]) * N + bc[2]];
            // the FP64 rows are y-fastest, the FP32 ones x-fastest
            idx[i] = (int64_t)kc * g.nak + (t->K ? idx_K(g, ap[0], ap[1], ap[2]) : idx_Kx(g, ap[0], ap[1], ap[2]));
        } else if (table == 1 || table == 2) {
            for (int c = (d == 3 ? 0 : 1); c < 3; ++c)
                if (x[c] < -h || x[c] >= h || y[c] < -h || y[c] >= h)
                    return fail(BNQ_EINVAL, "pair %lld outside I_N", (long long)i);
            idx[i] = idx_I(g, x[0], x[1], x[2]) * g.nm + idx_I(g, y[0], y[1], y[2]);
        } else {
            return fail(BNQ_EINVAL, "table must be 0, 1 or 2");
        }
    }
    int64_t *idx_d = nullptr;
    double *out_d = nullptr;
    bnq_status st;
    if ((st = upload(&idx_d, idx, "lookup indices")) || (st = dalloc(&out_d, (size_t)n, "lookup output"))) {
        hipFree(idx_d);
        return st;
    }
    // the FP64 tables if the set has them, else the FP32 ones; weights of a
    // set that holds none are formed here by the code of the pair sums
    const Radial rad = t->radial();
    if (table == 0)
        t->K ? launch_gather(t->K, idx_d, n, out_d, nullptr) : launch_gather(t->K32, idx_d, n, out_d, nullptr);
    else if (t->wc)
        launch_gather(table == 1 ? t->wc : t->wq, idx_d, n, out_d, nullptr);
    else if (t->wc32 && !t->K)
        launch_gather(table == 1 ? t->wc32 : t->wq32, idx_d, n, out_d, nullptr);
    else
        launch_pair_weights_at(g, rad, idx_d, n, table, out_d, nullptr);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpy(out, out_d, sizeof(double) * n, hipMemcpyDeviceToHost);
    hipFree(idx_d);
    hipFree(out_d);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(BNQ_EHIP, "lookup failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return BNQ_OK;
}

bnq_status bnq_plan_counts(bnq_plan_t P, double *counts) {
    if (!P || !counts) return fail(BNQ_EINVAL, "NULL argument");
    for (int i = 0; i < 4; ++i) counts[i] = P->counts[i];
    return BNQ_OK;
}

bnq_status bnq_plan_autotune(bnq_plan_t P, const double *f, int32_t reps, double *ms_host, int32_t *choice_host,
                             bnq_stream_t stream) {
    if (!P || !f) return fail(BNQ_EINVAL, "plan and f must be non-NULL");
    if (reps < 1) return fail(BNQ_EINVAL, "reps must be >= 1");
    if (P->nbatch > 0) return fail(BNQ_EINVAL, "plan is held by a batch, whose copy of its work would go stale");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    double ms[kNumTune];
    for (int c = 0; c < kNumTune; ++c) ms[c] = 0.0;
    int best = 0;
    if (P->ih.terms & BNQ_T_QTRI) {
        double *Q = nullptr;
        bnq_status st;
        if ((st = dalloc(&Q, (size_t)P->g.nm, "autotune output"))) return st;
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            hipFree(Q);
            if (a) hipEventDestroy(a);
            return fail(BNQ_EHIP, "event creation failed");
        }
        const bool timing = P->timing;
        P->timing = false;
        for (int c = 0; c < kNumTune && !st; ++c) {
            P->tune = kTuneCandidates[c];
            if ((st = rebuild_t1(P, s))) break;
            if ((st = bnq_collide(P, f, Q, nullptr, stream))) break;  // warm-up
            hipEventRecord(a, s);
            for (int r = 0; r < reps && !st; ++r) st = bnq_collide(P, f, Q, nullptr, stream);
            hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess) st = fail(BNQ_EHIP, "autotune timing failed");
            float t = 0;
            hipEventElapsedTime(&t, a, b);
            ms[c] = t / reps;
            if (ms[c] < ms[best]) best = c;
        }
        P->timing = timing;
        hipEventDestroy(a);
        hipEventDestroy(b);
        hipFree(Q);
        if (st) return st;
        P->tune = kTuneCandidates[best];
        if ((st = rebuild_t1(P, s))) return st;
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[std::make_tuple(dev, P->p.d, P->p.N, (int)P->p.precision)] = best;
    }
    if (ms_host)
        for (int c = 0; c < kNumTune; ++c) ms_host[c] = ms[c];
    if (choice_host) *choice_host = best;
    return BNQ_OK;
}

bnq_status bnq_plan_autotune_pairs(bnq_plan_t P, const double *f, int32_t reps, double *ms_host,
                                   int32_t *split_host, bnq_stream_t stream) {
    if (!P || !f) return fail(BNQ_EINVAL, "plan and f must be non-NULL");
    if (reps < 1) return fail(BNQ_EINVAL, "reps must be >= 1");
    if (P->nbatch > 0) return fail(BNQ_EINVAL, "plan is held by a batch, whose copy of its work would go stale");
    hipStream_t s = (hipStream_t)stream;
    P->last = s;
    const int any = P->ih.terms;
    double ms[kNumPairSplit];
    for (int c = 0; c < kNumPairSplit; ++c) ms[c] = 0.0;
    if (!(any & (BNQ_T_CLASSICAL | BNQ_T_QMULT))) {  // no pair sums to time
        if (ms_host)
            for (int c = 0; c < kNumPairSplit; ++c) ms_host[c] = 0.0;
        if (split_host) *split_host = P->g.psplit;
        return BNQ_OK;
    }
    // candidates capped at the largest split the workspace holds; a cap that
    // repeats the previous candidate is not run again
    const int smax = pair_split_max(P->g.N);
    int best = -1, best_k = P->g.psplit;
    double *Q = nullptr;
    bnq_status st;
    if ((st = dalloc(&Q, (size_t)P->g.nm, "autotune output"))) return st;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        hipFree(Q);
        if (a) hipEventDestroy(a);
        return fail(BNQ_EHIP, "event creation failed");
    }
    const bool timing = P->timing;
    P->timing = false;
    // one evaluation forms the spectrum the pair sums read
    st = bnq_collide(P, f, Q, nullptr, stream);
    for (int c = 0, prev = 0; c < kNumPairSplit && !st; ++c) {
        const int k = std::min(kPairSplitCandidates[c], smax);
        if (k == prev) continue;
        prev = k;
        Exec E = exec_of(P);
        E.timer = nullptr;
        E.g.psplit = k;
        const Radial rad = E.t->radial();
        const std::vector<IOs> ios = make_ios(1, nullptr, [](IOs &, int, int) {});
        auto run = [&]() {
            for (const IOs &io : ios) {
                launch_pairs(E.g, E.prec, E.D, io, E.prec ? (const void *)E.t->wc32 : (const void *)E.t->wc,
                             E.prec ? (const void *)E.t->wq32 : (const void *)E.t->wq, (any & BNQ_T_QMULT) != 0,
                             E.otf ? &rad : nullptr, s);
                launch_pairs_reduce(E.g, E.D, io, s);
            }
        };
        run();  // warm-up
        hipEventRecord(a, s);
        for (int r = 0; r < reps; ++r) run();
        hipEventRecord(b, s);
        const hipError_t e1 = hipGetLastError(), e2 = hipEventSynchronize(b);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            st = fail(BNQ_EHIP, "pair-sum autotune failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
            break;
        }
        float t = 0;
        hipEventElapsedTime(&t, a, b);
        ms[c] = t / reps;
        if (best < 0 || ms[c] < ms[best]) {
            best = c;
            best_k = k;
        }
    }
    P->timing = timing;
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(Q);
    if (st) return st;
    // the pair sums rewrite W and Qc from the spectrum; the split kept is the
    // one every later evaluation of this plan uses
    P->g.psplit = best_k;
    P->ih.geo = P->g;
    HIPCHK(hipMemcpy(P->inst_d, &P->ih, sizeof(Inst), hipMemcpyHostToDevice));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_pairs[std::make_tuple(dev, P->p.d, P->p.N, (int)P->p.precision, P->p.eps == 0 ? 1 : 0)] = best_k;
    }
    if (ms_host)
        for (int c = 0; c < kNumPairSplit; ++c) ms_host[c] = ms[c];
    if (split_host) *split_host = best_k;
    return BNQ_OK;
}

bnq_status bnq_tune_pairs_get(int32_t d, int32_t N, int32_t precision, int32_t eps, int32_t *split) {
    if (!split) return fail(BNQ_EINVAL, "split is NULL");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_pairs.find(std::make_tuple(dev, (int)d, (int)N, (int)precision, eps == 0 ? 1 : 0));
    *split = it == g_tune_pairs.end() ? 0 : it->second;
    return BNQ_OK;
}

bnq_status bnq_tune_pairs_set(int32_t d, int32_t N, int32_t precision, int32_t eps, int32_t split) {
    if (d != 2 && d != 3) return fail(BNQ_EINVAL, "d must be 2 or 3");
    if (N < 2 || N > 64 || (N & 1)) return fail(BNQ_EINVAL, "N must be even in [2, 64]");
    if (precision != BNQ_FP64 && precision != BNQ_FP32C) return fail(BNQ_EINVAL, "unknown precision %d", precision);
    if (split < 0 || split > pair_split_max(N))
        return fail(BNQ_EINVAL, "split %d outside 0 .. %d", split, pair_split_max(N));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto key = std::make_tuple(dev, (int)d, (int)N, (int)precision, eps == 0 ? 1 : 0);
    if (split == 0)
        g_tune_pairs.erase(key);
    else
        g_tune_pairs[key] = split;
    return BNQ_OK;
}

bnq_status bnq_tune_get(int32_t d, int32_t N, int32_t precision, int32_t *choice) {
    if (!choice) return fail(BNQ_EINVAL, "choice is NULL");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(dev, (int)d, (int)N, (int)precision));
    *choice = it == g_tune.end() ? -1 : it->second;
    return BNQ_OK;
}

bnq_status bnq_tune_set(int32_t d, int32_t N, int32_t precision, int32_t choice) {
    if (choice < -1 || choice >= kNumTune) return fail(BNQ_EINVAL, "choice %d outside -1 .. %d", choice, kNumTune - 1);
    if (d != 2 && d != 3) return fail(BNQ_EINVAL, "d must be 2 or 3");
    if (precision != BNQ_FP64 && precision != BNQ_FP32C) return fail(BNQ_EINVAL, "unknown precision %d", precision);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto key = std::make_tuple(dev, (int)d, (int)N, (int)precision);
    if (choice < 0)
        g_tune.erase(key);
    else
        g_tune[key] = choice;
    return BNQ_OK;
}

bnq_status bnq_plan_set_timing(bnq_plan_t P, int32_t enable) {
    if (!P) return fail(BNQ_EINVAL, "plan is NULL");
    HIPCHK(hipStreamSynchronize(P->last));
    for (auto &e : P->evs) {
        P->pool.push_back(e.a);
        P->pool.push_back(e.b);
    }
    P->evs.clear();
    P->timing = enable != 0;
    return BNQ_OK;
}

bnq_status bnq_plan_timing(bnq_plan_t P, double *ms, int64_t *launches) {
    if (!P || !ms || !launches) return fail(BNQ_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(P->last));
    for (int k = 0; k < BNQ_NKERNELS; ++k) {
        ms[k] = 0;
        launches[k] = 0;
    }
    for (auto &e : P->evs) {
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
        ms[e.fam] += t;
        launches[e.fam] += 1;
    }
    return BNQ_OK;
}

const char *bnq_status_string(bnq_status s) {
    switch (s) {
        case BNQ_OK: return "ok";
        case BNQ_EINVAL: return "invalid argument";
        case BNQ_ENOMEM: return "out of device memory";
        case BNQ_EHIP: return "HIP runtime error";
        case BNQ_ENOTSUP: return "not supported";
        case BNQ_ENONFINITE: return "non-finite value";
        case BNQ_EBOUND: return "fermion bound violated";
    }
    return "unknown status";
}

const char *bnq_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches (a fixed set of plans and state arrays evaluated together).
struct bnq_batch_s {
    // instances that share geometry and tables: one launch per kernel
    struct Group {
        Exec E;
        std::vector<int> members;  // positions in the batch
        Inst *D = nullptr;
    };
    // one trilinear sum per stage over the instances of several groups
    struct Shared {
        TriSet T;
        Inst *D = nullptr;
        int *t1cut = nullptr;
        T1Item *items = nullptr;
        int *qctr = nullptr;
    };
    std::vector<bnq_plan_s *> plans;
    std::vector<double *> f;
    std::vector<Group> groups;
    std::vector<Shared> shared;
    hipGraphExec_t gexec = nullptr;  // captured step, replayed while (scheme, dt, stream) match
    int g_scheme = -1;
    std::vector<double> g_dt;
    hipStream_t g_stream = nullptr;
};

namespace {

void destroy_batch(bnq_batch_s *B) {
    if (!B) return;
    if (B->gexec) hipGraphExecDestroy(B->gexec);
    for (auto &G : B->groups) hipFree(G.D);
    for (auto &S : B->shared) {
        hipFree(S.D);
        hipFree(S.t1cut);
        hipFree(S.items);
        hipFree(S.qctr);
    }
    delete B;
}

std::vector<TriSet> shared_sets(const bnq_batch_s *B) {
    std::vector<TriSet> v;
    for (const auto &S : B->shared) v.push_back(S.T);
    return v;
}

bnq_status batch_step_enqueue(bnq_batch_s *B, const double *dt, int scheme, hipStream_t s) {
    std::vector<const Exec *> Es;
    std::vector<std::vector<double *>> fs(B->groups.size());
    std::vector<std::vector<double>> dts(B->groups.size());
    std::vector<double *const *> fp;
    std::vector<const double *> dp;
    for (size_t i = 0; i < B->groups.size(); ++i) {
        const auto &G = B->groups[i];
        Es.push_back(&G.E);
        for (int m : G.members) {
            fs[i].push_back(B->f[m]);
            dts[i].push_back(dt[m]);
        }
        fp.push_back(fs[i].data());
        dp.push_back(dts[i].data());
    }
    return step_groups(Es, fp, dp, shared_sets(B), scheme, s);
}

}  // namespace

extern "C" {

bnq_status bnq_batch_create(int32_t n, const bnq_plan_t *plans, double *const *f, bnq_batch_t *out) {
    if (!out) return fail(BNQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !plans || !f) return fail(BNQ_EINVAL, "need n >= 1 plans and state arrays");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !f[i]) return fail(BNQ_EINVAL, "plan or state %d is NULL", i);
        if (plans[i]->sepP) return fail(BNQ_ENOTSUP, "plan %d uses the separated-kernel trilinear route", i);
        if (plans[i]->tabs->device != dev) return fail(BNQ_EINVAL, "plan %d lives on another device", i);
        for (int j = 0; j < i; ++j) {
            if (plans[j] == plans[i]) return fail(BNQ_EINVAL, "plan %d appears twice", i);
            if (f[j] == f[i]) return fail(BNQ_EINVAL, "state array %d appears twice", i);
        }
    }
    bnq_batch_s *B = new bnq_batch_s;
    B->plans.assign(plans, plans + n);
    B->f.assign(f, f + n);
    // Groups: instances that share geometry, tables, precision and the
    // pair-sum split run each kernel as one launch.
    std::map<std::tuple<const TableSet *, int, int>, int> gidx;
    for (int i = 0; i < n; ++i) {
        const bnq_plan_s *Pi = plans[i];
        const auto key = std::make_tuple((const TableSet *)Pi->tabs, (int)Pi->p.precision + 2 * (int)Pi->otf,
                                         Pi->g.psplit);
        auto it = gidx.find(key);
        if (it == gidx.end()) {
            gidx[key] = (int)B->groups.size();
            B->groups.emplace_back();
            B->groups.back().members.push_back(i);
        } else {
            B->groups[it->second].members.push_back(i);
        }
    }
    for (auto &G : B->groups) {
        // rotations and transforms come from a member with the trilinear term
        // if there is one (plans without it build no work lists)
        bnq_plan_s *P0 = plans[G.members[0]];
        for (int m : G.members)
            if (plans[m]->ih.terms & BNQ_T_QTRI) {
                P0 = plans[m];
                break;
            }
        G.E = exec_of(P0);
        G.E.timer = nullptr;
        G.E.tri_shared = true;
        G.E.Dh.clear();
        for (int m : G.members) G.E.Dh.push_back(plans[m]->ih);
        bnq_status st;
        if ((st = upload(&G.D, G.E.Dh, "batch instance descriptors"))) {
            destroy_batch(B);
            return st;
        }
        G.E.D = G.D;
    }
    // Shared trilinear sums: every instance with the term whose kernel
    // variant and schedule agree (dynamic queues also need equal slot
    // counts: any wave may take any instance's item) joins one launch per
    // stage.  Members are ordered by decreasing trilinear work, so that in a
    // queue the large instances' items come first and the small ones fill
    // the tail.
    std::map<std::tuple<int, int, int, int>, std::vector<int>> sidx;
    for (int i = 0; i < n; ++i) {
        const bnq_plan_s *Pi = plans[i];
        if (!(Pi->ih.terms & BNQ_T_QTRI)) continue;
        const int prec = Pi->p.precision == BNQ_FP32C ? 1 : 0;
        const auto key = std::make_tuple(prec, prec ? t1_mfma_class(Pi->g.N) : 0, Pi->nq, Pi->nq ? Pi->nslots : 0);
        sidx[key].push_back(i);
    }
    for (auto &kv : sidx) {
        std::vector<int> mem = kv.second;
        std::stable_sort(mem.begin(), mem.end(), [&](int a, int b) {
            return t1_terms(plans[a]->g.d, plans[a]->g.N) > t1_terms(plans[b]->g.d, plans[b]->g.N);
        });
        B->shared.emplace_back();
        auto &S = B->shared.back();
        const bnq_plan_s *Q0 = plans[mem[0]];
        S.T.prec = Q0->p.precision == BNQ_FP32C ? 1 : 0;
        S.T.nq = Q0->nq;
        std::vector<Inst> Dh;
        double terms = 0;
        for (int m : mem) {
            Dh.push_back(plans[m]->ih);
            S.T.Nmax = std::max(S.T.Nmax, plans[m]->g.N);
            S.T.nslots = std::max(S.T.nslots, plans[m]->nslots);
            terms += t1_terms(plans[m]->g.d, plans[m]->g.N);
        }
        std::vector<int> off;
        std::vector<T1Item> items;
        std::vector<float> cost;
        if (S.T.nq) {
            // dynamic: queue x holds every member's queue-x items, member by member
            off.assign(1, 0);
            for (int x = 0; x < S.T.nq; ++x) {
                for (size_t j = 0; j < mem.size(); ++j) {
                    const bnq_plan_s *P = plans[mem[j]];
                    for (int k = P->off_h[x]; k < P->off_h[x + 1]; ++k) {
                        T1Item it = P->items_h[k];
                        it.inst = (int)j;
                        items.push_back(it);
                        cost.push_back(P->icost_h[k]);
                    }
                }
                off.push_back((int)items.size());
            }
        } else {
            // static: every member's list sl runs as list (sl + o_j) mod nl of
            // the set (its items keep their own list in T1Item::slot, hence
            // their partial arrays).  Members that fill every list take
            // o_j = 0; the others, whose few items sit in their first lists,
            // are placed one after another around the ring of lists, so that
            // small instances do not all load the same workgroups.  In a set
            // list the members' items are interleaved by their relative
            // position in their own lists: instances of one cell have the same
            // items, so the workgroups walk the kernel-mode rows once for all
            // of them (each row is read for every instance while it is in L2)
            // instead of once per instance; every instance's own items keep
            // their order.
            const int nl = t1_lists(S.T.prec, S.T.nslots);
            struct Ent {
                double r;  // relative position in the member's list
                int j, k;  // member, index into its items_h
            };
            std::vector<std::vector<Ent>> per(nl);
            int ring = 0;
            for (size_t j = 0; j < mem.size(); ++j) {
                const bnq_plan_s *P = plans[mem[j]];
                const int nlj = t1_lists(S.T.prec, P->nslots);
                int used = 0;
                for (int sl = 0; sl < nlj; ++sl)
                    if (P->off_h[sl + 1] > P->off_h[sl]) used = sl + 1;
                const int o = used >= nl ? 0 : ring;
                if (used < nl) ring = (ring + used) % nl;
                for (int sl = 0; sl < nlj; ++sl) {
                    const int L = (sl + o) % nl, k0 = P->off_h[sl], n_sl = P->off_h[sl + 1] - k0;
                    for (int k = k0; k < k0 + n_sl; ++k) per[L].push_back({(k - k0 + 0.5) / n_sl, (int)j, k});
                }
            }
            off.assign(nl + 1, 0);
            for (int L = 0; L < nl; ++L) {
                std::stable_sort(per[L].begin(), per[L].end(), [](const Ent &a, const Ent &b) { return a.r < b.r; });
                off[L] = (int)items.size();
                for (const Ent &e : per[L]) {
                    const bnq_plan_s *P = plans[mem[e.j]];
                    T1Item x = P->items_h[e.k];
                    x.inst = e.j;
                    items.push_back(x);
                    cost.push_back(P->icost_h[e.k]);
                }
            }
            off[nl] = (int)items.size();
        }
        // launches per evaluation: by the trilinear terms of the whole set
        S.T.nchunk = t1_chunks(terms);
        bnq_status st;
        if ((st = upload(&S.D, Dh, "batch trilinear instances")) ||
            (st = upload(&S.t1cut, t1_cuts(off, cost, S.T.nchunk), S.T.nq ? "batch queues" : "batch slot ranges")) ||
            (S.T.nq && (st = dalloc(&S.qctr, (size_t)((S.T.nq + 1) & ~1), "batch queue tickets"))) ||
            (!items.empty() && (st = upload(&S.items, items, "batch trilinear items")))) {
            destroy_batch(B);
            return st;
        }
        S.T.D = S.D;
        S.T.t1cut = S.t1cut;
        S.T.items = S.items;
        S.T.qctr = S.qctr;
    }
    for (auto *P : B->plans) ++P->nbatch;
    *out = B;
    return BNQ_OK;
}

bnq_status bnq_batch_layout(bnq_batch_t B, int32_t *groups, int32_t *trilinear_sets) {
    if (!B) return fail(BNQ_EINVAL, "batch is NULL");
    if (groups) *groups = (int32_t)B->groups.size();
    if (trilinear_sets) *trilinear_sets = (int32_t)B->shared.size();
    return BNQ_OK;
}

bnq_status bnq_batch_destroy(bnq_batch_t B) {
    if (!B) return BNQ_OK;
    if (B->g_stream) hipStreamSynchronize(B->g_stream);
    for (auto *P : B->plans) {
        hipStreamSynchronize(P->last);
        --P->nbatch;
    }
    destroy_batch(B);
    return BNQ_OK;
}

bnq_status bnq_batch_collide(bnq_batch_t B, double *const *Q, void *const *Qhat, bnq_stream_t stream) {
    if (!B || !Q) return fail(BNQ_EINVAL, "batch and Q must be non-NULL");
    const int n = (int)B->f.size();
    for (int i = 0; i < n; ++i) {
        if (!Q[i]) return fail(BNQ_EINVAL, "Q[%d] is NULL", i);
        if ((const void *)Q[i] == (const void *)B->f[i]) return fail(BNQ_EINVAL, "Q[%d] aliases its state", i);
    }
    hipStream_t s = (hipStream_t)stream;
    for (auto *P : B->plans) P->last = s;
    std::vector<const Exec *> Es;
    std::vector<std::vector<IOs>> ios;
    for (auto &G : B->groups) {
        Es.push_back(&G.E);
        ios.push_back(make_ios((int)G.members.size(), nullptr, [&](IOs &io, int z, int j) {
            const int i = G.members[j];
            io.in[z] = B->f[i];
            io.out[z] = Q[i];
            io.qhat[z] = Qhat ? (double2 *)Qhat[i] : nullptr;
        }));
    }
    return collide_groups(Es, ios, shared_sets(B), s);
}

bnq_status bnq_batch_step(bnq_batch_t B, const double *dt, int32_t scheme, int32_t use_graph, bnq_stream_t stream) {
    if (!B || !dt) return fail(BNQ_EINVAL, "batch and dt must be non-NULL");
    const int n = (int)B->f.size();
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(dt[i])) return fail(BNQ_EINVAL, "dt[%d] must be finite", i);
    for (int i = 0; i < n; ++i) {
        bnq_status st = health_status(B->plans[i], i);
        if (st) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    for (auto *P : B->plans) P->last = s;
    if (!use_graph) return batch_step_enqueue(B, dt, scheme, s);
    if (!s) return fail(BNQ_EINVAL, "graph replay needs a non-default stream");
    const std::vector<double> dtv(dt, dt + n);
    if (!B->gexec || B->g_scheme != scheme || B->g_dt != dtv || B->g_stream != s) {
        if (B->gexec) {
            HIPCHK(hipStreamSynchronize(B->g_stream ? B->g_stream : s));
            hipGraphExecDestroy(B->gexec);
            B->gexec = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        bnq_status st = batch_step_enqueue(B, dt, scheme, s);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (st) {
            if (graph) hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(BNQ_EHIP, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&B->gexec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            B->gexec = nullptr;
            return fail(BNQ_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        B->g_scheme = scheme;
        B->g_dt = dtv;
        B->g_stream = s;
    }
    HIPCHK(hipGraphLaunch(B->gexec, s));
    return BNQ_OK;
}

}  // extern "C"
