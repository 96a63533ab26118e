/*
 * CPU oracle for the truncated, periodised Boltzmann–Nordheim collision
 * operator in Fourier–Galerkin form (Mouton & Rey, arXiv 2110.13735).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and used
 * by tests/, by the smoke check and by the CPU-baseline leg of the benchmark.
 * The product library never links, loads or calls it, and it shares no source
 * with the GPU path.
 *
 * Everything is plain FP64 with no blocking or fusion beyond the definitions:
 *
 *  (1) Kernel modes (Lemma on the Fourier modes of the truncated terms,
 *      section 'Fast spectral approximation of the BNE operator'):
 *        beta(k,l) = \int_{B(0,R)^2} Btilde(z,y) delta(z.y) e^{i(z.k+y.l)} dz dy
 *      evaluated by quadrature of its polar form (section 'Expansion of the kernel modes'):
 *        2-D Maxwell molecules, Btilde = 2 C_phi:
 *          beta(k,l) = 2 C_phi \int_0^pi phi(k.e_t) phi(l.e_{t+pi/2}) dt,
 *          phi(s) = \int_{-R}^{R} e^{i r s} dr = 2R sinc(Rs),
 *          rectangle rule theta_p = p pi / M (eq. beta2D; the integrand is
 *          pi-periodic, so the rule converges spectrally);
 *        3-D hard spheres, Btilde = 4 C_phi:
 *          beta(k,l) = 2 C_phi \int_{S^2} phi3(k.e) psi(|Pi_{e-perp} l|) de,
 *          phi3(s) = \int_{-R}^{R} |r| e^{i r s} dr,
 *          psi(s)  = \int_0^pi phi3(s cos t) dt = 2 pi R J_1(R s)/s,
 *          (psi taken without the sin factor, as the surface measure of the
 *          great circle requires), Gauss–Legendre in cos(theta) about l times
 *          the trapezoidal rule in the azimuth.
 *      beta depends only on |k|^2, |l|^2 and |k.l| (invariance of Btilde
 *      under a common rotation, evenness in each argument); tables are filled
 *      through a memo keyed on those three integers.
 *
 *  (2) Galerkin sums (same Lemma, with F = G = H and the Q4 term read as
 *      F(xi) G(xi+z+y) H(xi+y)), for n in I_N and all indices in I_N:
 *        Qc_n = sum_{l+m=n} [beta(l,m) - beta(m,m)] G_l G_m
 *        Qq_n = sum_{k+l+m=n} [beta(k+m,l+m) + beta(l,m) - beta(l+m,l)
 *                              - beta(l,l+m)] G_k G_l G_m
 *      and the factored pieces used to check the trilinear term separately:
 *        W_s  = sum_{l+m=s} [beta(l,m) - beta(l+m,l) - beta(l,l+m)] G_l G_m
 *        X_n  = sum_k G_k W_{n-k},
 *        T1_n = sum_{k+l+m=n} beta(k+m,l+m) G_k G_l G_m    (the Q_{1,q} term).
 *
 * Index conventions: d in {2,3}; a grid of N^d values in C order, storage
 * index = mode + N/2.  A d = 2 problem is stored as 3-D with a first axis of
 * extent 1 holding mode 0 only.  Complex arrays are interleaved (re, im).
 * Kernel-mode tables span X x X, X = {-N, ..., N-1}^d, in [a][b] order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Gauss–Legendre nodes on [-1, 1] by Newton iteration on P_n.               */
static void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* phi(s) = int_{-R}^{R} e^{irs} dr = 2 sin(Rs)/s. */
static double phi2(double R, double s) {
    double x = R * s;
    if (fabs(x) < 1e-4) return 2.0 * R * (1.0 - x * x / 6.0 + x * x * x * x / 120.0);
    return 2.0 * sin(x) / s;
}

/* phi3(s) = int_{-R}^{R} |r| e^{irs} dr = 2R sin(Rs)/s + 2 (cos(Rs) - 1)/s^2. */
static double phi3(double R, double s) {
    double x = R * s;
    if (fabs(x) < 0.5) {
        /* R^2 sum_k (-1)^k 2 x^{2k} / ((2k)! (2k+2)) */
        double x2 = x * x, term = 1.0, sum = 0.0;
        for (int k = 0; k < 12; ++k) {
            sum += term / (2.0 * k + 2.0);
            term *= -x2 / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
        }
        return 2.0 * R * R * sum;
    }
    return 2.0 * R * sin(x) / s + 2.0 * (cos(x) - 1.0) / (s * s);
}

/* psi(s) = int_0^pi phi3(s cos t) dt = 2 pi R J_1(Rs)/s. */
static double psi3(double R, double s) {
    double x = R * s;
    if (fabs(x) < 1e-6) return OR_PI * R * R * (1.0 - x * x / 8.0);
    return 2.0 * OR_PI * R * j1(x) / s;
}

/* Angular node counts.  Both rules integrate functions whose spectrum in the
 * angle is that of e^{i x cos(.)} with x up to R(|k|+|l|); the coefficients
 * J_n(x) are below 1e-17 once n > x + 10 x^(1/3) + 20.  Doubling the counts
 * changes beta by less than 1e-14 (checked in tests). */
static int band(double x) { return (int)ceil(x + 10.0 * cbrt(x) + 20.0); }
static int nodes_2d(double ka, double lb, double R) {
    return band(R * (ka + lb)) / 2 + 8;
}
static void nodes_3d(double ka, double lb, double R, int *nt, int *nph) {
    *nt = band(R * (ka + lb)) / 2 + 24;
    *nph = 2 * (band(R * ka) / 2 + 4);
}

/* 2-D kernel mode from the rectangle rule. */
double or_beta2_vec(double R, double Cphi, double k0, double k1, double l0, double l1, int M) {
    double s = 0.0;
    for (int p = 0; p < M; ++p) {
        double th = OR_PI * p / M;
        double c = cos(th), sn = sin(th);
        /* e_t = (c, sn), e_{t+pi/2} = (-sn, c) */
        s += phi2(R, k0 * c + k1 * sn) * phi2(R, -l0 * sn + l1 * c);
    }
    return 2.0 * Cphi * OR_PI / M * s;
}

/* 3-D kernel mode from |k|, |l| and cos(angle(k,l)); frame with l along z:
 * beta = 2 C_phi int_{-1}^{1} psi(|l| sqrt(1-t^2))
 *                  int_0^{2pi} phi3(|k| (sg sqrt(1-t^2) cos p + cg t)) dp dt. */
double or_beta3_inv(double R, double Cphi, double ka, double lb, double cg, int nt, int nph) {
    double *x = (double *)malloc(sizeof(double) * nt);
    double *w = (double *)malloc(sizeof(double) * nt);
    gauss_legendre(nt, x, w);
    double sg2 = 1.0 - cg * cg;
    double sg = sg2 > 0.0 ? sqrt(sg2) : 0.0;
    double tot = 0.0;
    for (int i = 0; i < nt; ++i) {
        double t = x[i];
        double st = sqrt(fmax(0.0, 1.0 - t * t));
        double ps = psi3(R, lb * st);
        double inner = 0.0;
        for (int p = 0; p < nph; ++p) {
            double ph = 2.0 * OR_PI * p / nph;
            inner += phi3(R, ka * (sg * st * cos(ph) + cg * t));
        }
        tot += w[i] * ps * inner * (2.0 * OR_PI / nph);
    }
    free(x);
    free(w);
    return 2.0 * Cphi * tot;
}

/* beta for integer vectors (d = 2 uses components 1,2 of a 3-vector). */
static double beta_from_invariants(int d, double R, double Cphi, int64_t a2, int64_t b2, int64_t ab) {
    double ka = sqrt((double)a2), lb = sqrt((double)b2);
    if (d == 2) {
        /* place k on the first axis, l at the matching angle */
        double cg = (a2 == 0 || b2 == 0) ? 1.0 : (double)ab / (ka * lb);
        if (cg > 1.0) cg = 1.0;
        if (cg < -1.0) cg = -1.0;
        double sg = sqrt(fmax(0.0, 1.0 - cg * cg));
        return or_beta2_vec(R, Cphi, ka, 0.0, lb * cg, lb * sg, nodes_2d(ka, lb, R));
    }
    double cg = (a2 == 0 || b2 == 0) ? 1.0 : (double)ab / (ka * lb);
    if (cg > 1.0) cg = 1.0;
    if (cg < -1.0) cg = -1.0;
    int nt, nph;
    nodes_3d(ka, lb, R, &nt, &nph);
    return or_beta3_inv(R, Cphi, ka, lb, cg, nt, nph);
}

/* Exported: beta for a list of integer vector pairs (3 ints each; d = 2 uses
 * the last two).  `scale` multiplies the default node counts (tests use it to
 * check convergence). */
void or_beta_pairs(int d, double R, double Cphi, int64_t n, const int32_t *a, const int32_t *b,
                   double *out, double scale) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *x = a + 3 * i, *y = b + 3 * i;
        int64_t a2 = (int64_t)x[0] * x[0] + (int64_t)x[1] * x[1] + (int64_t)x[2] * x[2];
        int64_t b2 = (int64_t)y[0] * y[0] + (int64_t)y[1] * y[1] + (int64_t)y[2] * y[2];
        int64_t ab = (int64_t)x[0] * y[0] + (int64_t)x[1] * y[1] + (int64_t)x[2] * y[2];
        if (scale == 1.0) {
            out[i] = beta_from_invariants(d, R, Cphi, a2, b2, ab < 0 ? -ab : ab);
        } else {
            double ka = sqrt((double)a2), lb = sqrt((double)b2);
            if (d == 2) {
                int M = (int)ceil(scale * nodes_2d(ka, lb, R));
                out[i] = or_beta2_vec(R, Cphi, x[1], x[2], y[1], y[2], M);
            } else {
                int nt, nph;
                nodes_3d(ka, lb, R, &nt, &nph);
                nt = (int)ceil(scale * nt);
                nph = 2 * (int)ceil(scale * nph / 2);
                double cg = (a2 == 0 || b2 == 0) ? 1.0 : (double)ab / (ka * lb);
                if (cg > 1.0) cg = 1.0;
                if (cg < -1.0) cg = -1.0;
                out[i] = or_beta3_inv(R, Cphi, ka, lb, cg, nt, nph);
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Memo keyed on (|a|^2, |b|^2, |a.b|): open addressing on 64-bit keys.       */
typedef struct {
    uint64_t *keys;
    double *vals;
    int64_t cap;
    int64_t count;
} memo_t;

static uint64_t hash64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static void memo_init(memo_t *m, int64_t cap) {
    int64_t c = 1;
    while (c < 2 * cap) c <<= 1;
    m->cap = c;
    m->count = 0;
    m->keys = (uint64_t *)malloc(sizeof(uint64_t) * c);
    m->vals = (double *)malloc(sizeof(double) * c);
    for (int64_t i = 0; i < c; ++i) m->keys[i] = UINT64_MAX;
}

static void memo_grow(memo_t *m);

static int64_t memo_slot(const memo_t *m, uint64_t key) {
    int64_t i = (int64_t)(hash64(key) & (uint64_t)(m->cap - 1));
    while (m->keys[i] != UINT64_MAX && m->keys[i] != key) i = (i + 1) & (m->cap - 1);
    return i;
}

static void memo_insert(memo_t *m, uint64_t key) {
    if (2 * (m->count + 1) > m->cap) memo_grow(m);
    int64_t i = memo_slot(m, key);
    if (m->keys[i] == UINT64_MAX) {
        m->keys[i] = key;
        m->count++;
    }
}

static void memo_grow(memo_t *m) {
    memo_t n;
    memo_init(&n, m->cap);
    for (int64_t i = 0; i < m->cap; ++i)
        if (m->keys[i] != UINT64_MAX) {
            int64_t j = memo_slot(&n, m->keys[i]);
            n.keys[j] = m->keys[i];
            n.vals[j] = m->vals[i];
            n.count++;
        }
    free(m->keys);
    free(m->vals);
    *m = n;
}

static void memo_free(memo_t *m) {
    free(m->keys);
    free(m->vals);
}

static uint64_t inv_key(int64_t a2, int64_t b2, int64_t ab) {
    if (ab < 0) ab = -ab;
    return ((uint64_t)a2 << 42) | ((uint64_t)b2 << 21) | (uint64_t)ab;
}

static void memo_evaluate(memo_t *m, int d, double R, double Cphi) {
    int64_t nk = 0;
    int64_t *slots = (int64_t *)malloc(sizeof(int64_t) * m->count);
    for (int64_t i = 0; i < m->cap; ++i)
        if (m->keys[i] != UINT64_MAX) slots[nk++] = i;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nk; ++q) {
        uint64_t key = m->keys[slots[q]];
        int64_t a2 = (int64_t)(key >> 42), b2 = (int64_t)((key >> 21) & ((1u << 21) - 1)),
                ab = (int64_t)(key & ((1u << 21) - 1));
        m->vals[slots[q]] = beta_from_invariants(d, R, Cphi, a2, b2, ab);
    }
    free(slots);
}

/* ------------------------------------------------------------------------- */
/* Index helpers.  ext[i] = extent of axis i; lo[i] = lowest mode of axis i.  */
typedef struct {
    int d, N;
    int lo[3], hi[3];    /* I_N bounds per axis (axis 0 is {0} when d = 2) */
    int xlo[3], xn[3];   /* X bounds: first value and extent per axis      */
    int64_t xsize;       /* |X| */
    int64_t gsize;       /* |I_N| */
} geom_t;

static void geom_init(geom_t *g, int d, int N) {
    g->d = d;
    g->N = N;
    for (int i = 0; i < 3; ++i) {
        if (d == 2 && i == 0) {
            g->lo[i] = g->hi[i] = 0;
            g->xlo[i] = 0;
            g->xn[i] = 1;
        } else {
            g->lo[i] = -N / 2;
            g->hi[i] = N / 2 - 1;
            g->xlo[i] = -N;
            g->xn[i] = 2 * N;
        }
    }
    g->xsize = (int64_t)g->xn[0] * g->xn[1] * g->xn[2];
    g->gsize = (int64_t)(g->hi[0] - g->lo[0] + 1) * (g->hi[1] - g->lo[1] + 1) * (g->hi[2] - g->lo[2] + 1);
}

static inline int64_t gidx(const geom_t *g, int a, int b, int c) {
    int n1 = g->hi[1] - g->lo[1] + 1, n2 = g->hi[2] - g->lo[2] + 1;
    return ((int64_t)(a - g->lo[0]) * n1 + (b - g->lo[1])) * n2 + (c - g->lo[2]);
}
static inline int64_t xidx(const geom_t *g, int a, int b, int c) {
    return ((int64_t)(a - g->xlo[0]) * g->xn[1] + (b - g->xlo[1])) * g->xn[2] + (c - g->xlo[2]);
}
static inline int in_grid(const geom_t *g, int a, int b, int c) {
    return a >= g->lo[0] && a <= g->hi[0] && b >= g->lo[1] && b <= g->hi[1] && c >= g->lo[2] &&
           c <= g->hi[2];
}

/* Exported: |X| for the table builder. */
int64_t or_xsize(int d, int N) {
    geom_t g;
    geom_init(&g, d, N);
    return g.xsize;
}

/* Exported: dense table beta(a,b), a,b in X, [a][b] order. */
int or_beta_table(int d, int N, double R, double Cphi, double *out) {
    geom_t g;
    geom_init(&g, d, N);
    int64_t X = g.xsize;
    int32_t *vec = (int32_t *)malloc(sizeof(int32_t) * 3 * X);
    int64_t *nrm = (int64_t *)malloc(sizeof(int64_t) * X);
    int64_t q = 0;
    for (int a = 0; a < g.xn[0]; ++a)
        for (int b = 0; b < g.xn[1]; ++b)
            for (int c = 0; c < g.xn[2]; ++c, ++q) {
                vec[3 * q] = a + g.xlo[0];
                vec[3 * q + 1] = b + g.xlo[1];
                vec[3 * q + 2] = c + g.xlo[2];
                nrm[q] = (int64_t)vec[3 * q] * vec[3 * q] + (int64_t)vec[3 * q + 1] * vec[3 * q + 1] +
                         (int64_t)vec[3 * q + 2] * vec[3 * q + 2];
            }
    memo_t m;
    memo_init(&m, 1 << 16);
    for (int64_t i = 0; i < X; ++i)
        for (int64_t j = 0; j < X; ++j) {
            int64_t ab = (int64_t)vec[3 * i] * vec[3 * j] + (int64_t)vec[3 * i + 1] * vec[3 * j + 1] +
                         (int64_t)vec[3 * i + 2] * vec[3 * j + 2];
            memo_insert(&m, inv_key(nrm[i], nrm[j], ab));
        }
    memo_evaluate(&m, d, R, Cphi);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < X; ++i)
        for (int64_t j = 0; j < X; ++j) {
            int64_t ab = (int64_t)vec[3 * i] * vec[3 * j] + (int64_t)vec[3 * i + 1] * vec[3 * j + 1] +
                         (int64_t)vec[3 * i + 2] * vec[3 * j + 2];
            out[i * X + j] = m.vals[memo_slot(&m, inv_key(nrm[i], nrm[j], ab))];
        }
    memo_free(&m);
    free(vec);
    free(nrm);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Complex helpers on interleaved doubles. */
typedef struct {
    double re, im;
} cplx;
static inline cplx cmul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}
static inline cplx cget(const double *G, int64_t i) {
    cplx r = {G[2 * i], G[2 * i + 1]};
    return r;
}

#define BT(a0, a1, a2, b0, b1, b2) (btab[xidx(g, a0, a1, a2) * g->xsize + xidx(g, b0, b1, b2)])

/* Classical sum for one output mode n (gain_only: the Q1c term alone,
 * sum beta(l,m) G_l G_m, the scale against which cancellation is measured). */
static cplx classical_mode(const geom_t *g, const double *G, const double *btab, const int *n, int gain_only) {
    cplx acc = {0.0, 0.0};
    for (int l0 = g->lo[0]; l0 <= g->hi[0]; ++l0)
        for (int l1 = g->lo[1]; l1 <= g->hi[1]; ++l1)
            for (int l2 = g->lo[2]; l2 <= g->hi[2]; ++l2) {
                int m0 = n[0] - l0, m1 = n[1] - l1, m2 = n[2] - l2;
                if (!in_grid(g, m0, m1, m2)) continue;
                double w = BT(l0, l1, l2, m0, m1, m2);
                if (!gain_only) w -= BT(m0, m1, m2, m0, m1, m2);
                cplx p = cmul(cget(G, gidx(g, l0, l1, l2)), cget(G, gidx(g, m0, m1, m2)));
                acc.re += w * p.re;
                acc.im += w * p.im;
            }
    return acc;
}

/* Quantum sum for one output mode n.  which = 0: all four terms, 1: Q_{1,q}
 * only (T1). */
static cplx quantum_mode(const geom_t *g, const double *G, const double *btab, const int *n, int which) {
    cplx acc = {0.0, 0.0};
    for (int k0 = g->lo[0]; k0 <= g->hi[0]; ++k0)
        for (int k1 = g->lo[1]; k1 <= g->hi[1]; ++k1)
            for (int k2 = g->lo[2]; k2 <= g->hi[2]; ++k2) {
                cplx gk = cget(G, gidx(g, k0, k1, k2));
                for (int l0 = g->lo[0]; l0 <= g->hi[0]; ++l0)
                    for (int l1 = g->lo[1]; l1 <= g->hi[1]; ++l1)
                        for (int l2 = g->lo[2]; l2 <= g->hi[2]; ++l2) {
                            int m0 = n[0] - k0 - l0, m1 = n[1] - k1 - l1, m2 = n[2] - k2 - l2;
                            if (!in_grid(g, m0, m1, m2)) continue;
                            double w = BT(k0 + m0, k1 + m1, k2 + m2, l0 + m0, l1 + m1, l2 + m2);
                            if (which == 0)
                                w += BT(l0, l1, l2, m0, m1, m2) - BT(l0 + m0, l1 + m1, l2 + m2, l0, l1, l2) -
                                     BT(l0, l1, l2, l0 + m0, l1 + m1, l2 + m2);
                            cplx p = cmul(cmul(gk, cget(G, gidx(g, l0, l1, l2))), cget(G, gidx(g, m0, m1, m2)));
                            acc.re += w * p.re;
                            acc.im += w * p.im;
                        }
            }
    return acc;
}

static void mode_of(const geom_t *g, int64_t i, int *n) {
    int n1 = g->hi[1] - g->lo[1] + 1, n2 = g->hi[2] - g->lo[2] + 1;
    n[2] = (int)(i % n2) + g->lo[2];
    n[1] = (int)((i / n2) % n1) + g->lo[1];
    n[0] = (int)(i / ((int64_t)n1 * n2)) + g->lo[0];
}

/* Exported: direct sums for every output mode (or a subset when nsel >= 0:
 * `sel` lists linear output indices).  want: bit0 classical, bit1 quantum
 * (all four terms), bit2 T1 alone.  Outputs are complex over I_N (only the
 * selected entries are written); bit3 writes the classical gain term to Qg. */
void or_sums_direct(int d, int N, const double *G, const double *btab, int want, int64_t nsel,
                    const int64_t *sel, double *Qc, double *Qq, double *T1, double *Qg) {
    geom_t g;
    geom_init(&g, d, N);
    int64_t nout = nsel >= 0 ? nsel : g.gsize;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nout; ++q) {
        int64_t i = nsel >= 0 ? sel[q] : q;
        int n[3];
        mode_of(&g, i, n);
        if (want & 8) {
            cplx c = classical_mode(&g, G, btab, n, 1);
            Qg[2 * i] = c.re;
            Qg[2 * i + 1] = c.im;
        }
        if (want & 1) {
            cplx c = classical_mode(&g, G, btab, n, 0);
            Qc[2 * i] = c.re;
            Qc[2 * i + 1] = c.im;
        }
        if (want & 2) {
            cplx c = quantum_mode(&g, G, btab, n, 0);
            Qq[2 * i] = c.re;
            Qq[2 * i + 1] = c.im;
        }
        if (want & 4) {
            cplx c = quantum_mode(&g, G, btab, n, 1);
            T1[2 * i] = c.re;
            T1[2 * i + 1] = c.im;
        }
    }
}

/* Exported: the pair sum W_s over s in X (only s in E = {-N..N-2}^d can be
 * non-zero) and the outer sum X_n = sum_k G_k W_{n-k} over n in I_N. */
void or_factored(int d, int N, const double *G, const double *btab, double *W, double *Xo) {
    geom_t g;
    geom_init(&g, d, N);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < g.xsize; ++s) {
        int s2 = (int)(s % g.xn[2]) + g.xlo[2];
        int s1 = (int)((s / g.xn[2]) % g.xn[1]) + g.xlo[1];
        int s0 = (int)(s / ((int64_t)g.xn[1] * g.xn[2])) + g.xlo[0];
        cplx acc = {0.0, 0.0};
        for (int l0 = g.lo[0]; l0 <= g.hi[0]; ++l0)
            for (int l1 = g.lo[1]; l1 <= g.hi[1]; ++l1)
                for (int l2 = g.lo[2]; l2 <= g.hi[2]; ++l2) {
                    int m0 = s0 - l0, m1 = s1 - l1, m2 = s2 - l2;
                    if (!in_grid(&g, m0, m1, m2)) continue;
#define BTG(a0, a1, a2, b0, b1, b2) (btab[xidx(&g, a0, a1, a2) * g.xsize + xidx(&g, b0, b1, b2)])
                    double w = BTG(l0, l1, l2, m0, m1, m2) - BTG(s0, s1, s2, l0, l1, l2) -
                               BTG(l0, l1, l2, s0, s1, s2);
                    cplx p = cmul(cget(G, gidx(&g, l0, l1, l2)), cget(G, gidx(&g, m0, m1, m2)));
                    acc.re += w * p.re;
                    acc.im += w * p.im;
                }
        W[2 * s] = acc.re;
        W[2 * s + 1] = acc.im;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < g.gsize; ++i) {
        int n[3];
        mode_of(&g, i, n);
        cplx acc = {0.0, 0.0};
        for (int k0 = g.lo[0]; k0 <= g.hi[0]; ++k0)
            for (int k1 = g.lo[1]; k1 <= g.hi[1]; ++k1)
                for (int k2 = g.lo[2]; k2 <= g.hi[2]; ++k2) {
                    int s0 = n[0] - k0, s1 = n[1] - k1, s2 = n[2] - k2;
                    int64_t si = xidx(&g, s0, s1, s2);
                    cplx p = cmul(cget(G, gidx(&g, k0, k1, k2)), cget(W, si));
                    acc.re += p.re;
                    acc.im += p.im;
                }
        Xo[2 * i] = acc.re;
        Xo[2 * i + 1] = acc.im;
    }
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* 3-D kernel modes by their Funk–Hecke series, for full-size checks where a
 * quadrature per value is too slow.  Expanding both plane waves of the
 * Lemma's integral in spherical harmonics, the delta(z.y) constraint gives
 * int_{S^2} delta(e.e') P_n(e'.l) de' = 2 pi P_n(0) P_n(e.l), and with
 * Btilde = 4 C_phi (hard spheres)
 *   beta(k,l) = 32 pi^2 C_phi sum_{n even} (2n+1) P_n(0) P_n(cos g)
 *               J_n(|k|) J_n(|l|),   J_n(s) = int_0^R r j_n(r s) dr,
 * g the angle between k and l (odd n drop out: P_n(0) = 0).  The radial
 * integrals come from the caller (oracle.radial_series: Gauss–Legendre over
 * spherical Bessel values), J[q * nm + m] = J_{2m}(sqrt q), and mcut[q] the
 * number of even orders kept for |k|^2 = q; the series is cut at the smaller
 * of the two counts.  Pinned against the quadrature above. */
static double beta3_series(const double *J, int nm, const int *mcut, double Cphi, int64_t qa, int64_t qb,
                           int64_t ab) {
    const int mc = mcut[qa] < mcut[qb] ? mcut[qa] : mcut[qb];
    double x = 1.0;
    if (qa > 0 && qb > 0) {
        x = (double)(ab < 0 ? -ab : ab) / sqrt((double)qa * (double)qb);
        if (x > 1.0) x = 1.0;
    }
    const double *Ja = J + qa * nm, *Jb = J + qb * nm;
    /* P_{2m}(0) = (-1)^m (2m-1)!! / (2m)!!, and (pe, po) = (P_{2m}(x),
     * P_{2m+1}(x)) by the three-term recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1} */
    double p0 = 1.0, pe = 1.0, po = x, sum = Ja[0] * Jb[0];
    for (int m = 1; m < mc; ++m) {
        p0 *= -(2.0 * m - 1.0) / (2.0 * m);
        const double pe1 = ((4.0 * m - 1.0) * x * po - (2.0 * m - 1.0) * pe) / (2.0 * m);
        const double po1 = ((4.0 * m + 1.0) * x * pe1 - 2.0 * m * po) / (2.0 * m + 1.0);
        pe = pe1;
        po = po1;
        sum += (4.0 * m + 1.0) * p0 * pe * Ja[m] * Jb[m];
    }
    return 32.0 * OR_PI * OR_PI * Cphi * sum;
}

/* Exported: beta for n pairs of integer 3-vectors by the series. */
void or_beta3_series_pairs(int64_t n, const int32_t *a, const int32_t *b, double *out, const double *J, int nm,
                           const int *mcut, double Cphi) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *x = a + 3 * i, *y = b + 3 * i;
        const int64_t qa = (int64_t)x[0] * x[0] + (int64_t)x[1] * x[1] + (int64_t)x[2] * x[2];
        const int64_t qb = (int64_t)y[0] * y[0] + (int64_t)y[1] * y[1] + (int64_t)y[2] * y[2];
        const int64_t ab = (int64_t)x[0] * y[0] + (int64_t)x[1] * y[1] + (int64_t)x[2] * y[2];
        out[i] = beta3_series(J, nm, mcut, Cphi, qa, qb, ab);
    }
}

static inline int64_t dot3(int a0, int a1, int a2, int b0, int b1, int b2) {
    return (int64_t)a0 * b0 + (int64_t)a1 * b1 + (int64_t)a2 * b2;
}
#define BS(a0, a1, a2, b0, b1, b2) \
    beta3_series(J, nm, mcut, Cphi, dot3(a0, a1, a2, a0, a1, a2), dot3(b0, b1, b2, b0, b1, b2), dot3(a0, a1, a2, b0, b1, b2))

/* Exported: 3-D Galerkin sums at selected output modes (linear indices in
 * I_N, `sel`), with kernel modes from the series, written at the same
 * positions of the output arrays (complex, over I_N):
 *   want & 1: Qc_n = sum_{l+m=n} [beta(l,m) - beta(m,m)] G_l G_m and the gain
 *             term Qg_n = sum_{l+m=n} beta(l,m) G_l G_m;
 *   want & 4: T1_n = sum_{k+l+m=n} beta(k+m, l+m) G_k G_l G_m;
 *   want & 2: X_n = sum_k G_k W_{n-k} from the pair sum W over X (or_w_series).
 * Every index in I_N, as in the Lemma; the direct sums, no reordering. */
void or_series_modes(int N, const double *G, const double *J, int nm, const int *mcut, double Cphi, int want,
                     int64_t nsel, const int64_t *sel, const double *W, double *Qc, double *Qg, double *T1,
                     double *Xo) {
    geom_t gg;
    geom_init(&gg, 3, N);
    const geom_t *g = &gg;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nsel; ++q) {
        const int64_t i = sel[q];
        int n[3];
        mode_of(g, i, n);
        if (want & 1) {
            long double cr = 0.0L, ci = 0.0L, c2r = 0.0L, c2i = 0.0L;
            for (int l0 = g->lo[0]; l0 <= g->hi[0]; ++l0)
                for (int l1 = g->lo[1]; l1 <= g->hi[1]; ++l1)
                    for (int l2 = g->lo[2]; l2 <= g->hi[2]; ++l2) {
                        const int m0 = n[0] - l0, m1 = n[1] - l1, m2 = n[2] - l2;
                        if (!in_grid(g, m0, m1, m2)) continue;
                        const double blm = BS(l0, l1, l2, m0, m1, m2), bmm = BS(m0, m1, m2, m0, m1, m2);
                        const cplx p = cmul(cget(G, gidx(g, l0, l1, l2)), cget(G, gidx(g, m0, m1, m2)));
                        cr += (blm - bmm) * p.re;
                        ci += (blm - bmm) * p.im;
                        c2r += blm * p.re;
                        c2i += blm * p.im;
                    }
            Qc[2 * i] = (double)cr;
            Qc[2 * i + 1] = (double)ci;
            Qg[2 * i] = (double)c2r;
            Qg[2 * i + 1] = (double)c2i;
        }
        if (want & 4) {
            long double ar = 0.0L, ai = 0.0L;
            for (int k0 = g->lo[0]; k0 <= g->hi[0]; ++k0)
                for (int k1 = g->lo[1]; k1 <= g->hi[1]; ++k1)
                    for (int k2 = g->lo[2]; k2 <= g->hi[2]; ++k2) {
                        const cplx gk = cget(G, gidx(g, k0, k1, k2));
                        for (int l0 = g->lo[0]; l0 <= g->hi[0]; ++l0)
                            for (int l1 = g->lo[1]; l1 <= g->hi[1]; ++l1)
                                for (int l2 = g->lo[2]; l2 <= g->hi[2]; ++l2) {
                                    const int m0 = n[0] - k0 - l0, m1 = n[1] - k1 - l1, m2 = n[2] - k2 - l2;
                                    if (!in_grid(g, m0, m1, m2)) continue;
                                    const double w = BS(k0 + m0, k1 + m1, k2 + m2, l0 + m0, l1 + m1, l2 + m2);
                                    const cplx p = cmul(cmul(gk, cget(G, gidx(g, l0, l1, l2))),
                                                        cget(G, gidx(g, m0, m1, m2)));
                                    ar += w * p.re;
                                    ai += w * p.im;
                                }
                    }
            T1[2 * i] = (double)ar;
            T1[2 * i + 1] = (double)ai;
        }
        if (want & 2) {
            long double ar = 0.0L, ai = 0.0L;
            for (int k0 = g->lo[0]; k0 <= g->hi[0]; ++k0)
                for (int k1 = g->lo[1]; k1 <= g->hi[1]; ++k1)
                    for (int k2 = g->lo[2]; k2 <= g->hi[2]; ++k2) {
                        const cplx p = cmul(cget(G, gidx(g, k0, k1, k2)),
                                            cget(W, xidx(g, n[0] - k0, n[1] - k1, n[2] - k2)));
                        ar += p.re;
                        ai += p.im;
                    }
            Xo[2 * i] = (double)ar;
            Xo[2 * i + 1] = (double)ai;
        }
    }
}

/* Exported: the pair sum W_s = sum_{l+m=s} [beta(l,m) - beta(l+m,l) -
 * beta(l,l+m)] G_l G_m over s in X = {-N .. N-1}^3 (3-D, series kernel modes),
 * complex, X order. */
void or_w_series(int N, const double *G, const double *J, int nm, const int *mcut, double Cphi, double *W) {
    geom_t gg;
    geom_init(&gg, 3, N);
    const geom_t *g = &gg;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < g->xsize; ++s) {
        const int s2 = (int)(s % g->xn[2]) + g->xlo[2];
        const int s1 = (int)((s / g->xn[2]) % g->xn[1]) + g->xlo[1];
        const int s0 = (int)(s / ((int64_t)g->xn[1] * g->xn[2])) + g->xlo[0];
        long double ar = 0.0L, ai = 0.0L;
        for (int l0 = g->lo[0]; l0 <= g->hi[0]; ++l0)
            for (int l1 = g->lo[1]; l1 <= g->hi[1]; ++l1)
                for (int l2 = g->lo[2]; l2 <= g->hi[2]; ++l2) {
                    const int m0 = s0 - l0, m1 = s1 - l1, m2 = s2 - l2;
                    if (!in_grid(g, m0, m1, m2)) continue;
                    const double w = BS(l0, l1, l2, m0, m1, m2) - BS(s0, s1, s2, l0, l1, l2) -
                                     BS(l0, l1, l2, s0, s1, s2);
                    const cplx p = cmul(cget(G, gidx(g, l0, l1, l2)), cget(G, gidx(g, m0, m1, m2)));
                    ar += w * p.re;
                    ai += w * p.im;
                }
        W[2 * s] = (double)ar;
        W[2 * s + 1] = (double)ai;
    }
}
#undef BS
