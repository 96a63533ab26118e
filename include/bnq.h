/*
 * bnq.h — C ABI of libbnq, an MI355X (gfx950) implementation of the
 * spectral-Galerkin collision operator of the homogeneous Boltzmann–Nordheim
 * equation (Mouton & Rey, "On deterministic numerical methods for the quantum
 * Boltzmann–Nordheim equation I", arXiv 2110.13735).
 *
 * Problem (section 'Convergence towards a steady state', homogeneous equation; section 'Application to the space homogeneous BNE', classical method
 * lambda = 0, omega = 1, mu = (L/pi)^d):
 *     d f_j / dt = c (L/pi)^(d+gamma) Q_j,     j in I_N = {-N/2 .. N/2-1}^d,
 * on the velocity grid v_j = 2 L j / N of [-L, L)^d, where Q_j is the grid
 * value of the truncated, periodised operator Q^R_alpha(G) (section 'Truncation and periodization of the BNE operator',
 * indicator of Filbet–Hu–Jin, R = S = 2 pi / (3 + sqrt 2) as in section 'Validation of spectral accuracy')
 * evaluated through the Fourier–Galerkin sums of the kernel-mode Lemma
 * (section 'Fast spectral approximation of the BNE operator'):
 *     Qhat_n = sum_{l+m=n} [beta(l,m) - beta(m,m)] G_l G_m
 *            - alpha sum_{k+l+m=n} [beta(k+m,l+m) + beta(l,m) - beta(l+m,l)
 *                                   - beta(l,l+m)] G_k G_l G_m,
 *     G_k = N^-d sum_j f_j e^{-2 pi i k.j/N},
 *     Q_j = Re sum_{n in I_N} Qhat_n e^{2 pi i n.j/N},
 * with every index in I_N (linear, non-wrapping sums) and
 *     alpha = -eps hbar^d   (eps = +1 bosons, -1 fermions, 0 classical).
 * Kernels: d = 2 Maxwell molecules (gamma = 0, Btilde = 2 C_phi) and d = 3
 * hard spheres (gamma = 1, Btilde = 4 C_phi), b = 1 (section 'Fast computation of the collision modes').
 *
 * Memory: every pointer named f, Q, Qhat is a DEVICE pointer owned by the
 * caller (e.g. a torch tensor's data_ptr()).  f and Q are FP64 arrays of N^d
 * values in C order with storage index j + N/2 (d = 2: [N][N], d = 3:
 * [N][N][N]).  Qhat is interleaved complex128 in the same order, indexed
 * n + N/2.  Host pointers are named *_host.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  All calls are
 * asynchronous on that stream unless stated otherwise.
 *
 * Errors: every call returns a bnq_status; nothing else crosses the ABI.
 * bnq_last_error() returns a thread-local message for the last failure.
 * Plans are not thread-safe; the shared kernel-mode table cache is.
 */
#ifndef BNQ_H
#define BNQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BNQ_OK = 0,
    BNQ_EINVAL = -1,     /* bad argument (d, N, eps, L, null pointer, ...) */
    BNQ_ENOMEM = -2,     /* device allocation failed or table budget exceeded */
    BNQ_EHIP = -3,       /* a HIP runtime call failed */
    BNQ_ENOTSUP = -4,    /* valid but not implemented (kernel, precision, N) */
    BNQ_ENONFINITE = -5, /* health check: non-finite value in f */
    BNQ_EBOUND = -6      /* health check: fermion f >= 1/|alpha| */
} bnq_status;

typedef void *bnq_stream_t; /* hipStream_t */
typedef struct bnq_plan_s *bnq_plan_t;
typedef struct bnq_batch_s *bnq_batch_t;

/* term selection bits (all set = the full operator) */
#define BNQ_T_CLASSICAL 1 /* Q1c - Q2c                           */
#define BNQ_T_QMULT 2     /* Q2q - Q3q - Q4q  (through W and X)   */
#define BNQ_T_QTRI 4      /* Q1q              (the trilinear T1)  */
#define BNQ_T_ALL 7

#define BNQ_FP64 0
#define BNQ_FP32C 1 /* FP32 spectra, tables and products; sums combined in FP64 (see bnq_params) */

#define BNQ_CORR_NONE 0 /* the paper's scheme */
#define BNQ_CORR_MASS 1 /* subtract the mean of Q so that sum_j Q_j = 0 exactly */
/* replace Q by the L2-closest grid function with zero discrete mass, momentum
 * and kinetic energy (Q minus its projection onto span{1, v, |v|^2} over the
 * velocity nodes); not part of the paper's scheme */
#define BNQ_CORR_MOMENTS 2

#define BNQ_RK4 0
#define BNQ_EULER 1
#define BNQ_SSPRK2 2

typedef struct {
    int32_t d;          /* 2 or 3 */
    int32_t N;          /* even, 2 <= N <= 64 (3-D FP64 tables need N <= 32) */
    int32_t eps;        /* +1 boson, -1 fermion, 0 classical */
    int32_t precision;  /* BNQ_FP64, or BNQ_FP32C: Ghat, the rotated spectra, the
                           weight tables and the trilinear rows rounded to FP32
                           (tables converted from the FP64 ones on first use),
                           products and short partial sums (<= N pair terms, <= 2
                           trilinear rows) in FP32, every longer sum in FP64; DFTs,
                           the outer sum, combination and time stepping stay FP64.
                           Parity bar against the FP64 oracle: 1e-5. */
    int32_t terms;      /* BNQ_T_* mask, default BNQ_T_ALL */
    int32_t correction; /* BNQ_CORR_* */
    double hbar;        /* default 1 */
    double C_phi;       /* default 1 */
    double c;           /* collision scaling, default 1 */
    double L;           /* velocity box half-width, > 0 */
    int32_t schedule;   /* trilinear work distribution: BNQ_SCHED_STATIC (default;
                           fixed per-wave lists, results bitwise reproducible) or
                           BNQ_SCHED_DYNAMIC (waves take items by atomic ticket from
                           their XCD's queue; balances waves that the hardware issues
                           at different rates; the summation order, hence the last
                           bits, may change from run to run) */
    int32_t flags;      /* BNQ_FLAG_* bits, default 0 */
    int32_t angles;     /* BNQ_FLAG_T1_SEPARATED only: d = 2, the angle count P of
                           eq. alphap, 1..4096, 0 (default) = enough angles to
                           reproduce the converged kernel modes to rounding;
                           d = 3, the polar count M1 of eq. alphapprime (M2 =
                           2 M1 azimuthal), 1..64, required */
} bnq_params;

/* FP64 only: the pair sums form their weights w_c, w_q from the kernel-mode
 * series on the fly instead of reading the two N^d x N^d tables (the same
 * code forms both, so the results are bitwise those of the tables).  A plan
 * gets this mode without the flag when its table set's FP64 weight tables do
 * not fit the free device memory (3-D N = 48: the trilinear rows take 168 GB,
 * the weights would take 196 GB more); the pair sums then cost about 1000
 * flops per weight instead of 16 bytes of HBM traffic. */
#define BNQ_FLAG_WEIGHTS_OTF 1

/* FP64, d = 2 with N <= 32 or d = 3 with N <= 8: the trilinear term Q_{1,q}
 * is evaluated by the transform route of the appendix 'Fast evaluation of
 * the collision kernel' with the rank-P kernel modes of section 'Fast
 * computation of the collision modes' (eq. betadD): beta(a,b) = C sum_r
 * alpha_r(a) alpha'_r(b) over P directions.
 *   d = 2 (eq. alphap): P = angles, theta_p = p pi / P, C = pi / P.  With the
 *     default angle count the rule reproduces the converged kernel modes to
 *     rounding and the route equals the direct trilinear sum.
 *   d = 3 (eq. alphapprime): M1 = angles polar and M2 = 2 angles azimuthal
 *     directions, P = M1 M2, C = pi^2 / P; angles is required (1..64).  The
 *     polar rule converges at second order, so this is the rank-P operator of
 *     that rule, not the converged one.
 * The spectrum is extended by zeros to the doubled grid (2N)^d, on which the
 * route gives the linear Galerkin sum.  It costs about P (2N)^d transforms
 * of size (2N)^d -> N^d per evaluation (1.2e12 flops at d = 2, N = 32,
 * against 1.9e9 for the direct sum).  The other terms keep the converged
 * kernel-mode tables.  Plans with this flag are refused by bnq_batch_create
 * (ENOTSUP).  Other precisions or sizes: ENOTSUP. */
#define BNQ_FLAG_T1_SEPARATED 2

/* The step health flags (bnq_step, bnq_batch_step, bnq_health) do not record
 * Fermi-Dirac values at or above 1/|alpha|; non-finite values are still
 * recorded.  For experiments whose data start above that bound, as some of
 * the runs of section 'Relaxation towards equilibrium' do (a Maxwellian
 * datum with hbar close to the saturation threshold), and whose maximum is
 * then followed with bnq_moments. */
#define BNQ_FLAG_NO_FERMI_BOUND 4

#define BNQ_SCHED_STATIC 0
#define BNQ_SCHED_DYNAMIC 1

/* Fill *p with defaults: d = 3, N = 16, eps = 0, FP64, all terms, no
 * correction, hbar = C_phi = c = 1, L = 8. */
void bnq_params_default(bnq_params *p);

/* Build a plan: validates *p, attaches the kernel-mode tables shared by
 * every plan with the same (d, N, C_phi), and allocates the plan's workspace
 * on the current device.  The tables are the kernel modes beta(k,l) of the
 * Lemma of section 'Fast spectral approximation of the BNE operator' (the
 * integral over B(0,R)^2 of Btilde delta(z.y) e^{i(z.k + y.l)}), on the
 * arguments the sums of bnq_collide read: the pair weights
 * beta(l,m) - beta(m,m) and beta(l,m) - beta(l+m,l) - beta(l,l+m) for l, m in
 * I_N, and beta(a,b) for the trilinear term, a, b in {-(N-1) .. N-1}^d.  The tables of the plan's precision are built on
 * first use: every value is computed in FP64 on the device and stored in
 * FP64 (BNQ_FP64) or rounded to FP32 (BNQ_FP32C), so an FP32c plan never
 * needs the FP64 tables (at 3-D N = 48 they take 364 GB, the FP32 ones
 * 182 GB; an FP64 plan there keeps the 168 GB of trilinear rows and forms
 * its pair weights on the fly: BNQ_FLAG_WEIGHTS_OTF).  Tables are built on
 * `stream` and the call synchronises it.
 * Errors: EINVAL, ENOTSUP, ENOMEM (also when the tables do not fit the free
 * device memory), EHIP.  On error *out is NULL. */
bnq_status bnq_plan(const bnq_params *p, bnq_stream_t stream, bnq_plan_t *out);

/* Release the plan (waits for its stream work); drops its reference to the
 * shared tables (freed with the last reference).  NULL is accepted.
 * Errors: EINVAL while a batch holds the plan (destroy the batch first). */
bnq_status bnq_plan_destroy(bnq_plan_t plan);

/* Device bytes the plan would need: *plan_bytes for its own workspace,
 * *table_bytes for the shared tables of its precision (0 if already
 * resident; with BNQ_FLAG_WEIGHTS_OTF the FP64 trilinear rows only).  Host
 * only. */
bnq_status bnq_plan_footprint(const bnq_params *p, size_t *plan_bytes, size_t *table_bytes);

/* Q = c (L/pi)^(d+gamma) Re IDFT(Qhat) for the grid distribution f (the right
 * hand side of the semi-discrete equation).  If Qhat is non-NULL the
 * Galerkin modes Qhat_n (before the prefactor) are also written.  f and Q
 * must not alias.  Defined by: G_k, step 2(a) of section 'Numerical scheme for
 * the velocity rescaled BNE' (normalisation N^-d); Qhat_n, the Fourier modes
 * of the six Carleman terms in the Lemma of section 'Fast spectral
 * approximation of the BNE operator', assembled with the signs of section
 * 'The Carleman representation' (Q = Q+c - Q-c - alpha (Q1q + Q2q - Q3q -
 * Q4q)); the prefactor, the classical method of section 'Application to the
 * space homogeneous BNE' (lambda = 0, omega = 1, mu = (L/pi)^d).
 * Errors: EINVAL (null f or Q), EHIP. */
bnq_status bnq_collide(bnq_plan_t plan, const double *f, double *Q, void *Qhat, bnq_stream_t stream);

/* Advance f (in place) by one step of size dt of d f/dt = c (L/pi)^(d+gamma) Q(f)
 * (the semi-discrete equation of the classical method, section 'Application
 * to the space homogeneous BNE'; the forward Euler scheme of section
 * 'Numerical scheme for the velocity rescaled BNE' with lambda = 0, its
 * second-order Runge-Kutta remark, and the strong-stability-preserving RK2
 * of the relaxation experiments of section 'Trends to equilibrium') with
 * scheme BNQ_RK4 (classical fourth order), BNQ_SSPRK2 (Shu–Osher second
 * order) or BNQ_EULER, state and stage arithmetic in FP64.
 * Health: the kernel that writes the new state records, in the plan's health
 * flags (host-visible memory, no host synchronisation), whether it wrote a
 * non-finite value (BNQ_HEALTH_NONFINITE) or, for fermions (eps = -1), a
 * value f >= 1/|alpha| (BNQ_HEALTH_BOUND).  bnq_step reads the flags before
 * enqueuing: once a step that set them has completed on the device, every
 * later bnq_step returns ENONFINITE (or EBOUND) and enqueues nothing, so f
 * keeps the state that step wrote.  bnq_health() reads (optionally waiting
 * for the stream) and clears them.
 * Errors: EINVAL, EHIP, ENONFINITE, EBOUND. */
bnq_status bnq_step(bnq_plan_t plan, double *f, double dt, int32_t scheme, bnq_stream_t stream);

#define BNQ_HEALTH_NONFINITE 1
#define BNQ_HEALTH_BOUND 2
/* Health flags of the plan's steps (bnq_step, and bnq_batch_step for a plan
 * in a batch): *flags_host (optional) <- BNQ_HEALTH_* bits recorded by the
 * steps that have completed; wait != 0 first synchronises `stream`, so that
 * every step enqueued on it is included; clear != 0 resets the flags
 * afterwards.  Returns ENONFINITE or EBOUND when the flags are set (before
 * clearing), else OK.  Errors: EINVAL, EHIP. */
bnq_status bnq_health(bnq_plan_t plan, int32_t wait, int32_t clear, int32_t *flags_host, bnq_stream_t stream);

/* Discrete moments (section 'Numerical results' diagnostics, classical method), written to the
 * host array out_host[BNQ_MOMENTS_LEN] in this order:
 *   rho, u[0], u[1], u[2] (u[2] = 0 when d = 2), E_c, e, H, fmax, fmin,
 *   n_excluded
 * with rho = dv sum f, u = dv sum v f / rho, E_c = dv sum |v|^2 f,
 * e = dv sum |v-u|^2 f / (2 rho), H = dv sum [f ln f + (1-alpha f)/alpha
 * ln(1-alpha f)] (alpha != 0) or dv sum f ln f (alpha = 0) over the nodes with
 * f > 0 and 1 - alpha f > 0, n_excluded = number of other nodes, dv =
 * (2L/N)^d.  Synchronises `stream`.  Returns ENONFINITE if f holds a NaN or
 * Inf, EBOUND if eps = -1 and max f >= 1/|alpha| (moments still written). */
#define BNQ_MOMENTS_LEN 10
bnq_status bnq_moments(bnq_plan_t plan, const double *f, double *out_host, bnq_stream_t stream);

/* bnq_moments without any allocation and without a plan, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that must not call the allocator).  The grid is given by p's d, N, L and
 * the entropy's alpha by p's eps and hbar (other fields are validated as by
 * bnq_plan and otherwise ignored).  f is a DEVICE array of N^d FP64 values;
 * out is a DEVICE array of BNQ_MOMENTS_LEN + 1 doubles, written
 * asynchronously on `stream` with the values of bnq_moments in the same
 * order, followed by the number of non-finite values of f (no status is
 * returned for them: nothing is synchronised).  The partial sums live in a
 * static device array of 32 KiB per device (enough for every valid N), kept
 * until the process ends and shared by every call on that device: calls
 * that overlap on one device (other streams, other host threads) race.
 * Errors: EINVAL (params, null pointers, a grid whose partials would not fit
 * the array), EHIP. */
bnq_status bnq_moments_noalloc(const bnq_params *p, const double *f, double *out, bnq_stream_t stream);

/* ---- limit states (section 'Convergence towards a steady state') --------
 * The state a solution relaxes to, for given mass rho, mean velocity u and
 * internal energy e = (1/rho) int |v - u|^2 / 2 f dv.  With alpha = -eps
 * hbar^d (the paper's alpha: > 0 Fermi-Dirac, < 0 Bose-Einstein) and
 * ratio = |alpha| rho (d / (4 pi e))^(d/2):
 *  BNQ_EQ_MAXWELL     alpha = 0: rho (2 pi T)^(-d/2) exp(-|v - u|^2 / 2T),
 *                     T = 2e/d;
 *  BNQ_EQ_QUANTUM     ratio inside I_eq: the quantum Maxwellian
 *                     (1/|alpha|) / (z^-1 exp(|v - u|^2 / 2T) + sgn alpha),
 *                     z from eq. eq_fugacity by Brent's method (in ln z for
 *                     Fermi-Dirac), T from eq. mom2_qmaxwell;
 *  BNQ_EQ_CONDENSATE  3-D Bose-Einstein with ratio at or beyond the end of
 *                     I_eq: z = 1, the condensed mass m0 at v = u from eq.
 *                     m0critical_bosons_3d, and T such that the z = 1 part
 *                     carries the internal energy rho e (eq.
 *                     Tcritical_bosons_3d as printed conserves the energy
 *                     only at the critical ratio, where both agree);
 *  BNQ_EQ_SATURATED   Fermi-Dirac at the end of I_eq (the equality
 *                     critical_FD, to a relative 1e-9): rho / |D(u, A)| on
 *                     the ball D(u, A), A = sqrt(2 e (d + 2) / d);
 *  BNQ_EQ_UNKNOWN     Fermi-Dirac beyond it: no limit state is identified.
 * The complete Fermi-Dirac / Bose-Einstein integrals K_nu are evaluated by
 * composite Gauss-Legendre quadrature to about 1e-15 relative. */
#define BNQ_EQ_MAXWELL 0
#define BNQ_EQ_QUANTUM 1
#define BNQ_EQ_CONDENSATE 2
#define BNQ_EQ_SATURATED 3
#define BNQ_EQ_UNKNOWN 4
typedef struct {
    int32_t kind;   /* BNQ_EQ_* */
    int32_t d;
    double alpha;   /* -eps hbar^d */
    double rho;
    double u[3];    /* components in the order of the moments' u (d = 2: u[0], u[1]) */
    double e;
    double z;       /* fugacity (1 for a condensate; may overflow for degenerate FD) */
    double log_z;   /* ln z, always finite */
    double T;
    double m0;      /* condensed mass (BNQ_EQ_CONDENSATE), else 0 */
    double A;       /* radius of the saturated ball (Fermi-Dirac), else 0 */
    double ratio;   /* |alpha| rho (d / (4 pi e))^(d/2); 0 when alpha = 0 */
} bnq_equilibrium;

/* Limit state for (d, eps, hbar, rho, u[d], e).  Host only.  Errors: EINVAL
 * (d not 2 or 3, rho or e not positive and finite, no root bracketed). */
bnq_status bnq_equilibrium_solve(int32_t d, int32_t eps, double hbar, double rho, const double *u_host, double e,
                                 bnq_equilibrium *out_host);

/* ln K_nu of the complete Fermi-Dirac (fermi = 1, p = ln z) or Bose-Einstein
 * (fermi = 0, p = -ln z >= 0) integral K_nu(z) = Gamma(nu)^-1 int_0^inf
 * x^(nu-1) / (z^-1 e^x +- 1) dx, the quadrature the solver uses.  Host only;
 * for tests.  Errors: EINVAL (nu < 1, or p < 0 with fermi = 0). */
bnq_status bnq_fd_be_log(double nu, int32_t fermi, double p, double *out_host);

/* The limit state on the plan's grid (v_j = 2 L j / N), FP64, on `stream`:
 * out[j] = its value at v_j, with 0 written at the nodes where it is not a
 * finite function: for a condensate the node of the grid cell that holds u
 * (|v_j - u|_inf < L / N), where the mass m0 sits, and for BNQ_EQ_QUANTUM
 * Bose-Einstein only a node with v_j = u if z = 1 exactly.  The plan's d must match.  Errors:
 * EINVAL (null pointers, d mismatch, BNQ_EQ_UNKNOWN), EHIP. */
bnq_status bnq_equilibrium_fill(bnq_plan_t plan, const bnq_equilibrium *eq_host, double *out, bnq_stream_t stream);

/* Distance of grid data f to the limit state, over the nodes where the state
 * is finite: out_host[0] = Delta v sum |f - M|, [1] = max |f - M|,
 * [2] = Delta v sum M, [3] = number of excluded nodes (where M is infinite),
 * [4] = Delta v sum f over them (to compare with a condensate's m0).
 * Synchronises `stream`.  Errors as bnq_equilibrium_fill. */
/* ---- velocity-rescaled scheme (sections 'A rescaling velocity model of the
 * BNE' and 'Numerical scheme for the velocity rescaled BNE', lambda = 1,
 * mu = 1) ------------------------------------------------------------------
 * The distribution is held as G on the plan's grid read as xi_j = 2 pi j / N
 * (j in I_N): f(v) = s^d G(xi) with xi = s (v - u) and s = pi omega / L, so
 * f lives on u + [-L/omega, L/omega)^d, a box that follows the mean velocity
 * and the temperature.  The state carries the moments the scheme advances. */
typedef struct {
    double rho, u[3], e;  /* mass, mean velocity (order of the moments' u), internal energy */
    double omega;         /* velocity scale */
    double T, log_z;      /* temperature and ln fugacity of the last limit-state solve */
    int32_t kind;         /* its BNQ_EQ_* kind */
    int32_t reserved;
} bnq_rescaled_state;

/* State for G (device, N^d FP64) at velocity scale omega > 0 around u_ref
 * (host, d components): rho, u, e of f = s^d G on u_ref + [-L/omega,
 * L/omega)^d, and the limit state of those moments.  Synchronises `stream`.
 * Errors: EINVAL, EHIP. */
bnq_status bnq_rescaled_init(bnq_plan_t plan, const double *G, double omega, const double *u_ref_host,
                             bnq_rescaled_state *st_host, bnq_stream_t stream);

/* One forward Euler step of the rescaled scheme (its steps 2-5), G in place:
 *  K = c s^-gamma Q^R_{alpha s^d}(G) (the plan's operator with the quantum
 *      parameter alpha s^d: the same tables);
 *  rho, rho u, rho e advanced by dt Delta xi times the sums of K against 1,
 *      L xi / (pi omega) + u and |L xi / (pi omega)|^2 / 2;
 *  T from the limit state of the new moments (bnq_equilibrium_solve's
 *      rules), omega' = sqrt(T) (alpha != 0) or sqrt(T + |u'|^2 / d);
 *  G' = G + dt (K - div_xi((a xi - b) G)), a = (omega' - omega) / (dt
 *      omega), b = s (u' - u) / dt, the divergence by spectral
 *      differentiation (Re of the inverse DFT of i k times the DFT, k in I_N).
 * Synchronises `stream` (the temperature solve is host code).  Errors: EINVAL
 * (dt or the state not positive, or new moments with no finite temperature:
 * a degenerate Fermi-Dirac state; G is then unchanged), EHIP. */
bnq_status bnq_step_rescaled(bnq_plan_t plan, double *G, bnq_rescaled_state *st_host, double dt,
                             bnq_stream_t stream);

#define BNQ_EQDIST_LEN 5
bnq_status bnq_equilibrium_distance(bnq_plan_t plan, const double *f, const bnq_equilibrium *eq_host,
                                    double *out_host, bnq_stream_t stream);

/* Kernel modes beta(a_i, b_i) read back from the plan's device tables, for
 * n integer vector pairs a_host[3*i..], b_host[3*i..] (d = 2 uses components
 * 1 and 2; component 0 must be 0).  Requires |a|_inf <= N-1 and
 * |b|_inf <= N-1 (the trilinear table) -- or, with table = 1, a and b in
 * I_N (the classical weight table: returns beta(a,b) - beta(b,b)), table = 2
 * (the quantum pair weight: beta(a,b) - beta(a+b,a) - beta(a,a+b)).
 * Values come from the FP64 tables if the table set holds them, else from
 * the FP32 ones (rounded to nearest).  Synchronous; for tests and
 * diagnostics.  Errors: EINVAL (out of range). */
bnq_status bnq_table_lookup(bnq_plan_t plan, int32_t table, int64_t n, const int32_t *a_host,
                            const int32_t *b_host, double *out_host);

/* Work counts per evaluation of Qhat (plain Galerkin counts): classical pairs,
 * W pairs, outer-sum pairs, trilinear terms; written to counts_host[4]. */
bnq_status bnq_plan_counts(bnq_plan_t plan, double *counts_host);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of each kernel family.  enable = 1 starts (and clears) recording,
 * 0 stops.  bnq_plan_timing() synchronises the plan's last stream and writes
 * for each family k < BNQ_NKERNELS: ms_host[k] = total milliseconds,
 * launches_host[k] = number of launches.  Families: 0 dft, 1 pairs (classical
 * + W), 2 outer sum, 3 trilinear, 4 partial reduction, 5 combine/inverse,
 * 6 step update, 7 moments. */
#define BNQ_NKERNELS 8
bnq_status bnq_plan_set_timing(bnq_plan_t plan, int32_t enable);
bnq_status bnq_plan_timing(bnq_plan_t plan, double *ms_host, int64_t *launches_host);

/* Autotuner.  Times the candidate trilinear work distributions of this plan
 * (slots = resident waves or half of them; items dealt per XCD or over all
 * slots) on one evaluation of f (device, the plan's layout), reps timed
 * evaluations each, keeps the fastest for this plan, and records it for the
 * device and (d, N) so that plans created afterwards in the process start
 * with it.  ms_host (optional, 4 doubles) receives the mean time per
 * evaluation of each candidate, choice_host (optional) the chosen index.
 * Synchronises the stream.  Results stay within the parity tolerance of the
 * default distribution but may differ from it in the last bits (a different
 * summation order).  No-op for plans without the trilinear term.
 * Errors: EINVAL (also while a batch holds the plan), ENOMEM, EHIP. */
bnq_status bnq_plan_autotune(bnq_plan_t plan, const double *f, int32_t reps, double *ms_host, int32_t *choice_host,
                             bnq_stream_t stream);

/* The process's record of tuned trilinear work distributions, per device and
 * (d, N, precision): the index (0 .. 3, the candidates of bnq_plan_autotune)
 * that plans created afterwards on the current device start with.
 * bnq_tune_get(): *choice = the recorded index, or -1 if none.
 * bnq_tune_set(): records choice for the current device (-1 removes the
 *   record), e.g. from a table persisted by an earlier process; plans that
 *   exist keep theirs.  Errors: EINVAL (choice outside -1 .. 3, d not 2 or 3,
 *   unknown precision). */
bnq_status bnq_tune_get(int32_t d, int32_t N, int32_t precision, int32_t *choice);
bnq_status bnq_tune_set(int32_t d, int32_t N, int32_t precision, int32_t choice);

/* The l-chunking of the pair sums (section 'Fast spectral approximation of
 * the BNE operator', the classical and W sums over pairs (l, m)): the l box
 * of every output is cut into `split` slices, one workgroup and partial array
 * each, added in slice order.  A plan starts with the split recorded for
 * (device, d, N, precision, eps == 0), else 32 slices for eps = 0 in 3-D and
 * 16 otherwise (at most N).  The split changes the summation order, hence the
 * last bits of a result, within the parity tolerance.
 * bnq_plan_autotune_pairs(): times the pair sums (classical, and W when the
 *   plan has them) with 8, 16 and 32 slices, each capped at min(N, 32) (a
 *   count that repeats the previous one is not run again), on f
 *   (device, the plan's layout; one evaluation first forms the spectrum),
 *   reps timed runs each; keeps the fastest for this plan and records it for
 *   plans created afterwards.  ms_host (optional, 3 doubles): mean time of
 *   each candidate (0 where not run); split_host (optional): the split kept.
 *   Synchronises the stream.  A plan without pair sums keeps its split and
 *   records nothing.  Errors: EINVAL (also while a batch holds the plan),
 *   ENOMEM, EHIP.
 * bnq_tune_pairs_get(): *split = the recorded split for (d, N, precision,
 *   eps == 0) on the current device, or 0 if none.
 * bnq_tune_pairs_set(): records split (1 .. min(N, 32); 0 removes the record).
 *   Errors: EINVAL. */
bnq_status bnq_plan_autotune_pairs(bnq_plan_t plan, const double *f, int32_t reps, double *ms_host,
                                   int32_t *split_host, bnq_stream_t stream);
bnq_status bnq_tune_pairs_get(int32_t d, int32_t N, int32_t precision, int32_t eps, int32_t *split);
bnq_status bnq_tune_pairs_set(int32_t d, int32_t N, int32_t precision, int32_t eps, int32_t split);

/* ---- Batches ------------------------------------------------------------
 * Many independent instances of the same problem (the homogeneous equation
 * of section 'Convergence towards a steady state', each with its own plan and
 * state) evaluated together.  Plans that share (d, N, C_phi), precision and
 * pair-sum split form a group: each group runs one launch per kernel for all
 * of its instances.  The trilinear sums of every instance of every group run
 * as one shared launch per stage over the merged work lists (instances of
 * different (d, N) included); instances of different precision, matrix-core
 * variant or dynamic queue layout get a shared launch each.  Under the static
 * schedule every instance's result is bitwise identical to what its own plan
 * computes alone (an instance's list runs whole on one workgroup, its items in
 * order, into its own partial arrays).
 *
 * bnq_batch_create(): plans[i] (distinct, same device) and its state f[i]
 *   (device, FP64, the plan's layout; distinct).  The batch keeps these
 *   pointers: plans and states must outlive it (bnq_plan_destroy refuses a
 *   plan a batch holds), a plan must not be used on its own while a batch
 *   call that includes it is in flight, and a held plan cannot be autotuned.
 *   Errors: EINVAL (NULL / duplicate / other device), ENOMEM.
 * bnq_batch_collide(): Q[i] <- operator of f[i] (as bnq_collide), Qhat[i]
 *   optional (Qhat may be NULL, or hold NULL entries).
 * bnq_batch_step(): advances every f[i] in place by dt[i] (host array of n)
 *   with scheme (as bnq_step).  Each member's health flags are recorded as
 *   by bnq_step (read them with bnq_health on the member's plan); if a
 *   member's flags are set by a completed step, the call returns ENONFINITE
 *   or EBOUND (the message names the member) and enqueues nothing: the
 *   caller removes that member (a new batch) and steps the others on.  use_graph != 0 captures the whole step into a
 *   HIP graph on the first call and replays it while (scheme, dt, stream)
 *   are unchanged (a change recaptures); it needs a non-default stream.
 * bnq_batch_destroy(): waits for the batch's work and frees its arrays (not
 *   the plans or states).
 * bnq_batch_layout(): *groups = number of groups, *trilinear_sets = number
 *   of shared trilinear launches per stage (either pointer may be NULL). */
bnq_status bnq_batch_create(int32_t n, const bnq_plan_t *plans, double *const *f, bnq_batch_t *out);
bnq_status bnq_batch_destroy(bnq_batch_t batch);
bnq_status bnq_batch_layout(bnq_batch_t batch, int32_t *groups, int32_t *trilinear_sets);
bnq_status bnq_batch_collide(bnq_batch_t batch, double *const *Q, void *const *Qhat, bnq_stream_t stream);
bnq_status bnq_batch_step(bnq_batch_t batch, const double *dt, int32_t scheme, int32_t use_graph,
                          bnq_stream_t stream);

const char *bnq_status_string(bnq_status s);
const char *bnq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BNQ_H */
