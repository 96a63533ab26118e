// Time stepping and moments on the velocity grid, FP64.
//
// Classical method of section 'Application to the space homogeneous BNE': d f/dt = c (L/pi)^(d+gamma) Q(f); the RK
// stage combinations are plain FP64 vector updates.  Moments and entropy
// follow the diagnostics list of section 'Numerical results' (classical method, omega = 1):
//   rho = dv sum f, u = dv sum v f / rho, E_c = dv sum |v|^2 f,
//   e = dv sum |v - u|^2 f / (2 rho)   (a second pass, after u is known),
//   H = dv sum [f ln f + (1 - alpha f)/alpha ln(1 - alpha f)]   (alpha != 0)
//     = dv sum f ln f                                          (alpha  = 0)
// over nodes with f > 0 and 1 - alpha f > 0.  Reductions use a fixed
// assignment of nodes to blocks and a fixed tree, so results are
// bit-reproducible.
#include <algorithm>
#include <mutex>
#include <vector>

#include "bnq_internal.h"

namespace bnq {

static dim3 grid_nm(const Geo &g, const IOs &io) { return dim3((unsigned)((g.nm + 255) / 256), 1, (unsigned)io.n); }

// Health of a state value written by the last stage of a step: a wave that
// wrote a non-finite value, or a Fermi-Dirac value at or above 1/alpha,
// records it in the instance's two host-visible flag words (plain stores of
// 1 by one lane per wave; no host synchronisation).  Every lane of the wave
// must reach this call.
__device__ __forceinline__ void record_health(const Inst &I, bool valid, double v) {
    const bool nf = valid && !isfinite(v);
    const bool bd = valid && v >= I.fbound;  // false for NaN
    const unsigned long long mnf = __ballot(nf), mbd = __ballot(bd);
    if ((threadIdx.x & 63) == 0 && I.health) {
        volatile int *h = I.health;
        if (mnf) h[0] = 1;
        if (mbd) h[1] = 1;
    }
}

// y = in + a dt k[ks], into Inst::ybuf (to_out = 0) or io.out (to_out = 1,
// the last stage of an Euler step: its values are health-checked)
__global__ void stage_kernel(Geo g, const Inst *D, IOs io, double a, int ks, int to_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.nm;
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    double v = 0.0;
    if (valid) {
        const gptr<double> y = glob(to_out ? io.out[z] : I.ybuf);
        v = fma(a * io.dt[z], glob((const double *)I.k[ks])[i], glob(io.in[z])[i]);
        y[i] = v;
    }
    if (to_out) record_health(I, valid, v);
}

void launch_stage(const Geo &g, const Inst *D, const IOs &io, double a, int ks, int to_out, hipStream_t s) {
    hipLaunchKernelGGL(stage_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io, a, ks, to_out);
}

// f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4), f = io.out
__global__ void rk4_final_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.nm;
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    double v = 0.0;
    if (valid) {
        const gptr<double> f = glob(io.out[z]);
        const double k0 = glob((const double *)I.k[0])[i], k1 = glob((const double *)I.k[1])[i];
        const double k2 = glob((const double *)I.k[2])[i], k3 = glob((const double *)I.k[3])[i];
        v = f[i] + (io.dt[z] / 6.0) * (k0 + 2.0 * k1 + 2.0 * k2 + k3);
        f[i] = v;
    }
    record_health(I, valid, v);
}

void launch_rk4_final(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(rk4_final_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io);
}

// Shu–Osher SSP-RK2: y = f + dt k1;  f <- (f + y + dt k(y)) / 2, f = io.out
__global__ void ssprk2_final_kernel(Geo g, const Inst *D, IOs io) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.nm;
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    double v = 0.0;
    if (valid) {
        const gptr<double> f = glob(io.out[z]);
        v = 0.5 * (f[i] + fma(io.dt[z], glob((const double *)I.k[1])[i], glob((const double *)I.ybuf)[i]));
        f[i] = v;
    }
    record_health(I, valid, v);
}

void launch_ssprk2_final(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(ssprk2_final_kernel, grid_nm(g, io), dim3(256), 0, s, g, D, io);
}

// Conservation correction: Q <- Q - sum_k lambda_k c_k with c = (1, v, |v|^2)
// and lambda = Gram^-1 (sum_j c_k(j) Q_j), the L2-closest grid function with
// zero discrete mass, momentum and energy.  One workgroup per instance, fixed
// reduction tree.
__global__ __launch_bounds__(256) void moments_fix_kernel(Geo g, const Inst *D, IOs io) {
    const int z = blockIdx.z;
    const Inst &I = D[io.inst[z]];
    if (!I.corr_mom) return;
    const gptr<double> Q = glob(io.out[z]);
    const int m = g.d + 2;
    __shared__ double red[256][5];
    __shared__ double lam[5];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < g.nm; i += 256) {
        const double q = Q[i];
        const double x2 = (double)((int)(i % g.N) - g.h) * I.hstep;
        const double x1 = (double)((int)((i / g.N) % g.N) - g.h) * I.hstep;
        const double x0 = g.d == 3 ? (double)((int)(i / ((int64_t)g.N * g.N)) - g.h) * I.hstep : 0.0;
        acc[0] += q;
        if (g.d == 3) {
            acc[1] += x0 * q;
            acc[2] += x1 * q;
            acc[3] += x2 * q;
        } else {
            acc[1] += x1 * q;
            acc[2] += x2 * q;
        }
        acc[m - 1] += (x0 * x0 + x1 * x1 + x2 * x2) * q;
    }
    for (int k = 0; k < 5; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 5; ++k) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        __syncthreads();
    }
    if (threadIdx.x < m) {
        double l = 0.0;
        for (int k = 0; k < m; ++k) l += I.ginv[threadIdx.x * m + k] * red[0][k];
        lam[threadIdx.x] = l;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < g.nm; i += 256) {
        const double x2 = (double)((int)(i % g.N) - g.h) * I.hstep;
        const double x1 = (double)((int)((i / g.N) % g.N) - g.h) * I.hstep;
        const double x0 = g.d == 3 ? (double)((int)(i / ((int64_t)g.N * g.N)) - g.h) * I.hstep : 0.0;
        double c = lam[0] + lam[m - 1] * (x0 * x0 + x1 * x1 + x2 * x2);
        if (g.d == 3)
            c += lam[1] * x0 + lam[2] * x1 + lam[3] * x2;
        else
            c += lam[1] * x1 + lam[2] * x2;
        Q[i] = Q[i] - c;
    }
}

void launch_moments_fix(const Geo &g, const Inst *D, const IOs &io, hipStream_t s) {
    hipLaunchKernelGGL(moments_fix_kernel, dim3(1, 1, (unsigned)io.n), dim3(256), 0, s, g, D, io);
}

// fields: 0 sum f, 1-3 sum v f, 4 sum |v|^2 f, 5 sum entropy density,
//         6 max f, 7 min f, 8 excluded nodes, 9 non-finite nodes
__global__ __launch_bounds__(256) void moments_part_kernel(Geo g, const double *f, double L, double alpha,
                                                           double *part) {
    __shared__ double red[256][MOM_FIELDS];
    double acc[MOM_FIELDS];
    for (int k = 0; k < MOM_FIELDS; ++k) acc[k] = 0.0;
    acc[6] = -INFINITY;
    acc[7] = INFINITY;
    const double hstep = 2.0 * L / g.N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nm;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = f[i];
        const double x2 = (double)((int)(i % g.N) - g.h) * hstep;
        const double x1 = (double)((int)((i / g.N) % g.N) - g.h) * hstep;
        const double x0 = g.d == 3 ? (double)((int)(i / ((int64_t)g.N * g.N)) - g.h) * hstep : 0.0;
        if (!isfinite(v)) {
            acc[9] += 1.0;
            continue;
        }
        acc[0] += v;
        acc[1] += x0 * v;
        acc[2] += x1 * v;
        acc[3] += x2 * v;
        acc[4] += (x0 * x0 + x1 * x1 + x2 * x2) * v;
        acc[6] = fmax(acc[6], v);
        acc[7] = fmin(acc[7], v);
        const double om = 1.0 - alpha * v;
        if (v > 0.0 && om > 0.0) {
            double hden = v * log(v);
            if (alpha != 0.0) hden += om / alpha * log(om);
            acc[5] += hden;
        } else {
            acc[8] += 1.0;
        }
    }
    for (int k = 0; k < MOM_FIELDS; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < MOM_FIELDS; ++k) {
                const double a = red[threadIdx.x][k], b = red[threadIdx.x + w][k];
                red[threadIdx.x][k] = k == 6 ? fmax(a, b) : (k == 7 ? fmin(a, b) : a + b);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < MOM_FIELDS) part[(int64_t)blockIdx.x * MOM_FIELDS + threadIdx.x] = red[0][threadIdx.x];
}

// Field k of the per-block partials: sums, except the maximum (k = 6) and
// minimum (k = 7) of f; a fixed tree over 256 threads per field.
__device__ __forceinline__ double mom_op(int k, double a, double b) {
    return k == 6 ? fmax(a, b) : (k == 7 ? fmin(a, b) : a + b);
}

__global__ void __launch_bounds__(256) moments_final_kernel(int nblk, const double *part, double *out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    for (int k = 0; k < MOM_FIELDS; ++k) {
        double a = k == 6 ? -INFINITY : (k == 7 ? INFINITY : 0.0);
        for (int b = t; b < nblk; b += 256) a = mom_op(k, a, part[(int64_t)b * MOM_FIELDS + k]);
        red[t] = a;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) red[t] = mom_op(k, red[t], red[t + w]);
            __syncthreads();
        }
        if (t == 0) out[k] = red[0];
        __syncthreads();
    }
}

// Second pass: sum |v - u|^2 f over the finite nodes, with u = (sum v f) /
// (sum f) from the first pass's totals (the internal energy without the
// cancellation of E_c - rho |u|^2 when the drift is large).
__global__ __launch_bounds__(256) void moments_center_kernel(Geo g, const double *f, double L, const double *sums,
                                                             double *part2) {
    __shared__ double red[256];
    const double s0 = sums[0];
    const double u0 = s0 != 0.0 ? sums[1] / s0 : 0.0, u1 = s0 != 0.0 ? sums[2] / s0 : 0.0,
                 u2 = s0 != 0.0 ? sums[3] / s0 : 0.0;
    const double hstep = 2.0 * L / g.N;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nm;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = f[i];
        if (!isfinite(v)) continue;
        const double w2 = (double)((int)(i % g.N) - g.h) * hstep - u2;
        const double w1 = (double)((int)((i / g.N) % g.N) - g.h) * hstep - u1;
        const double w0 = g.d == 3 ? (double)((int)(i / ((int64_t)g.N * g.N)) - g.h) * hstep - u0 : 0.0;
        acc += (w0 * w0 + w1 * w1 + w2 * w2) * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part2[blockIdx.x] = red[0];
}

// Totals of the second pass (fixed tree) and the reported moments:
//   res = rho, u (axis order of the used axes, zero-padded to 3), E_c, e, H,
//         max f, min f, excluded + non-finite nodes, non-finite nodes.
__global__ void __launch_bounds__(256) moments_finish_kernel(Geo g, double L, int nblk, const double *part2,
                                                             const double *sums, double *res) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int b = t; b < nblk; b += 256) a += part2[b];
    red[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t != 0) return;
    const double h = 2.0 * L / g.N;
    const double dv = g.d == 3 ? h * h * h : h * h;
    const double rho = dv * sums[0];
    const int first = g.d == 3 ? 0 : 1;
    double u[3] = {0.0, 0.0, 0.0};
    for (int i = first; i < 3; ++i) u[i - first] = rho != 0.0 ? dv * sums[1 + i] / rho : 0.0;
    res[0] = rho;
    res[1] = u[0];
    res[2] = u[1];
    res[3] = u[2];
    res[4] = dv * sums[4];
    res[5] = rho != 0.0 ? dv * red[0] / (2.0 * rho) : 0.0;
    res[6] = dv * sums[5];
    res[7] = sums[6];
    res[8] = sums[7];
    res[9] = sums[8] + sums[9];
    res[10] = sums[9];
}

// scratch: nblk x MOM_FIELDS first-pass partials, nblk second-pass partials,
// MOM_FIELDS totals (moments_scratch_doubles(nblk) doubles)
void launch_moments(const Geo &g, const double *f, double L, double alpha, double *scratch, int nblk, double *res,
                    hipStream_t s) {
    double *part = scratch, *part2 = scratch + (size_t)nblk * MOM_FIELDS, *sums = part2 + nblk;
    hipLaunchKernelGGL(moments_part_kernel, dim3(nblk), dim3(256), 0, s, g, f, L, alpha, part);
    hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(256), 0, s, nblk, part, sums);
    hipLaunchKernelGGL(moments_center_kernel, dim3(nblk), dim3(256), 0, s, g, f, L, sums, part2);
    hipLaunchKernelGGL(moments_finish_kernel, dim3(1), dim3(256), 0, s, g, L, nblk, part2, sums, res);
}

// Device memory of the allocation-free moments entry point: a file-scope
// array, one copy per device, shared by every such call on that device.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

// Address of this device's copy of `scratch` (the array's name is a host-side
// stand-in and must never be passed to a kernel).  Looked up once per device
// with that device current, then cached.
hipError_t noalloc_scratch(double **out) {
    static std::mutex mu;
    static std::vector<double *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        double *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Rescaled scheme: G + dt (K - div((A xi - B) G)); each axis's derivative is
// the N-term row of D along that axis's line.
__global__ __launch_bounds__(256) void drift_update_kernel(Geo g, const double *G, const double *K, const double *D,
                                                           double A, double B0, double B1, double B2, double dt,
                                                           double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nm) return;
    const int N = g.N;
    const int j2 = (int)(i % N), j1 = (int)((i / N) % N), j0 = g.d == 3 ? (int)(i / ((int64_t)N * N)) : 0;
    const double h = 2.0 * M_PI / N;
    const int64_t base2 = i - j2, base1 = i - (int64_t)j1 * N, base0 = i - (int64_t)j0 * N * N;
    double div = 0.0;
    for (int m = 0; m < N; ++m) {
        const double xi = (m - g.h) * h;
        div += D[j2 * N + m] * ((A * xi - B2) * G[base2 + m]);
        div += D[j1 * N + m] * ((A * xi - B1) * G[base1 + (int64_t)m * N]);
        if (g.d == 3) div += D[j0 * N + m] * ((A * xi - B0) * G[base0 + (int64_t)m * N * N]);
    }
    out[i] = G[i] + dt * (K[i] - div);
}

void launch_drift_update(const Geo &g, const double *G, const double *K, const double *D, double A,
                         const double *B3, double dt, double *out, hipStream_t s) {
    hipLaunchKernelGGL(drift_update_kernel, dim3((unsigned)((g.nm + 255) / 256)), dim3(256), 0, s, g, G, K, D, A,
                       B3[0], B3[1], B3[2], dt, out);
}

__global__ void copy_kernel(double *dst, const double *src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

void launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(256), 0, s, dst, src, n);
}

// ---------------------------------------------------------------------------
// Limit state on the grid: value at node i, or excluded (not finite there).
__device__ static double eq_value(const Geo &g, const EqDev &q, double hstep, int64_t i, bool &excl) {
    const double x2 = (double)((int)(i % g.N) - g.h) * hstep;
    const double x1 = (double)((int)((i / g.N) % g.N) - g.h) * hstep;
    const double x0 = g.d == 3 ? (double)((int)(i / ((int64_t)g.N * g.N)) - g.h) * hstep : 0.0;
    // u holds the velocity components in the order of the used axes
    const double w0 = g.d == 3 ? x0 - q.u[0] : 0.0;
    const double w1 = x1 - q.u[g.d == 3 ? 1 : 0];
    const double w2 = x2 - q.u[g.d == 3 ? 2 : 1];
    const double r2 = w0 * w0 + w1 * w1 + w2 * w2;
    // a condensate's mass sits at v = u: the node of the grid cell holding u
    excl = q.kind == BNQ_EQ_CONDENSATE && fmax(fabs(w0), fmax(fabs(w1), fabs(w2))) < 0.5 * hstep;
    if (excl) return 0.0;
    switch (q.kind) {
        case BNQ_EQ_MAXWELL: return q.c0 * exp(-r2 / (2.0 * q.T));
        case BNQ_EQ_SATURATED: return r2 <= q.A2 ? q.c0 : 0.0;
        default: {
            const double a = r2 / (2.0 * q.T) - q.log_z;
            const double den = q.bose ? expm1(a) : exp(a) + 1.0;
            if (!(den > 0.0)) {
                excl = true;
                return 0.0;
            }
            return q.c0 / den;
        }
    }
}

__global__ __launch_bounds__(256) void equilibrium_kernel(Geo g, double hstep, EqDev q, const double *f,
                                                          double *out_fill, double *part) {
    __shared__ double red[256][EQ_FIELDS];
    double acc[EQ_FIELDS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nm;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool excl;
        const double m = eq_value(g, q, hstep, i, excl);
        if (out_fill) out_fill[i] = m;
        if (!f) continue;
        if (excl) {
            acc[3] += 1.0;
            acc[4] += f[i];
        } else {
            const double dlt = fabs(f[i] - m);
            acc[0] += dlt;
            acc[1] = fmax(acc[1], dlt);
            acc[2] += m;
        }
    }
    if (!f) return;
    for (int k = 0; k < EQ_FIELDS; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < EQ_FIELDS; ++k) {
                const double a = red[threadIdx.x][k], b = red[threadIdx.x + w][k];
                red[threadIdx.x][k] = k == 1 ? fmax(a, b) : a + b;
            }
        __syncthreads();
    }
    if (threadIdx.x < EQ_FIELDS) part[(int64_t)blockIdx.x * EQ_FIELDS + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void equilibrium_final_kernel(int nblk, const double *part, double *out) {
    const int k = threadIdx.x;
    if (k >= EQ_FIELDS) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double v = part[(int64_t)b * EQ_FIELDS + k];
        a = k == 1 ? fmax(a, v) : a + v;
    }
    out[k] = a;
}

void launch_equilibrium(const Geo &g, double L, const EqDev &q, const double *f, double *out_fill, double *part,
                        int nblk, double *out, hipStream_t s) {
    hipLaunchKernelGGL(equilibrium_kernel, dim3(nblk), dim3(256), 0, s, g, 2.0 * L / g.N, q, f, out_fill, part);
    if (f) hipLaunchKernelGGL(equilibrium_final_kernel, dim3(1), dim3(64), 0, s, nblk, part, out);
}

}  // namespace bnq
