// Kernels of the inference stages around the likelihood (gfx950):
// prior + bijection to the unconstrained space, posterior gradient, Adam
// (multi-start MAP) and HMC leapfrog / Metropolis accept with a Philox
// counter-based generator.  All per-particle or per-element; float64 where
// a value feeds an energy or a sum over parameters.
#include <math.h>
#include <stdint.h>

#include "lens_internal.h"
#include "lens_philox.h"
#include "lens_sampler.h"

namespace lens {

// ---------------------------------------------------------------------------
// Bijection and prior (per parameter)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double softplus_d(double x) {
    return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x));
}

// theta = T(u), dtheta/du, log|dtheta/du|, d log|dtheta/du| / du
__device__ __forceinline__ void bijection(const PriorRow& r, double u, double& th, double& dth,
                                          double& logj, double& dlogj) {
    const int kind = (int)r.kind;
    if (kind == LENS_PRIOR_UNIFORM || kind == LENS_PRIOR_TRUNCNORMAL) {
        const double s = 1.0 / (1.0 + exp(-u));
        const double w = r.hi - r.lo;
        th = r.lo + w * s;
        dth = w * s * (1.0 - s);
        logj = log(w) - softplus_d(-u) - softplus_d(u);
        dlogj = 1.0 - 2.0 * s;
    } else if (kind == LENS_PRIOR_LOGNORMAL) {
        th = exp(u);
        dth = th;
        logj = u;
        dlogj = 1.0;
    } else {
        th = u;
        dth = 1.0;
        logj = 0.0;
        dlogj = 0.0;
    }
}

// log prior density of theta and its derivative
__device__ __forceinline__ void log_prior(const PriorRow& r, double th, double& lp, double& dlp) {
    const int kind = (int)r.kind;
    if (kind == LENS_PRIOR_UNIFORM) {
        lp = r.cst;
        dlp = 0.0;
    } else if (kind == LENS_PRIOR_LOGNORMAL) {
        const double lx = log(th);
        const double z = (lx - r.a) / r.b;
        lp = r.cst - 0.5 * z * z - lx;
        dlp = (-z / r.b - 1.0) / th;
    } else {
        const double z = (th - r.a) / r.b;
        lp = r.cst - 0.5 * z * z;
        dlp = -z / r.b;
    }
}

// u = T^-1(theta); a bounded parameter at (or beyond) an end of its support
// maps to the logit of 2^-24 (or 1 - 2^-24), a log-normal one <= 0 to log 1e-30.
__global__ void k_inverse_bijection(int P, int d, const PriorRow* __restrict__ table,
                                    const float* __restrict__ theta, float* __restrict__ u) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P * d) return;
    const PriorRow& r = table[q % d];
    const int kind = (int)r.kind;
    const double th = (double)theta[q];
    double v;
    if (kind == LENS_PRIOR_UNIFORM || kind == LENS_PRIOR_TRUNCNORMAL) {
        const double lim = 5.9604644775390625e-08;   // 2^-24
        const double p = fmin(fmax((th - r.lo) / (r.hi - r.lo), lim), 1.0 - lim);
        v = log(p) - log1p(-p);
    } else if (kind == LENS_PRIOR_LOGNORMAL) {
        v = log(fmax(th, 1e-30));
    } else {
        v = th;
    }
    u[q] = (float)v;
}

__global__ void k_bijection(int P, int d, const PriorRow* __restrict__ table,
                            const float* __restrict__ u, float* __restrict__ theta) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P * d) return;
    const int j = q % d;
    double th, dth, lj, dlj;
    bijection(table[j], (double)u[q], th, dth, lj, dlj);
    theta[q] = (float)th;
}

// logp = logL(theta) + log prior(theta) [+ log J]; grad_u = (g_theta + dlp) dth [+ dlogJ].
// One wave per particle: lane j (and j + 64) evaluates parameter j; lane 0
// then sums the log-prior and log-Jacobian terms in parameter order.
constexpr int POST_WAVES = 4;   // particles per 256-thread work-group

__global__ __launch_bounds__(256) void k_posterior(int P, int d, const PriorRow* __restrict__ table,
                                                   const float* __restrict__ u, const double* __restrict__ logl,
                                                   const float* __restrict__ gtheta, int with_jac, ParamMask skip,
                                                   double* __restrict__ logp, float* __restrict__ grad_u) {
    __shared__ double terms[POST_WAVES][2][PARAM_MASK_BITS];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = blockIdx.x * POST_WAVES + wv;
    const bool active = p < P;
    const double L = active ? logl[p] : 0.0;
    const bool finite = isfinite(L);
    if (active) {
        const float* up = u + (size_t)p * d;
        const float* gp = gtheta + (size_t)p * d;
        float* go = grad_u + (size_t)p * d;
        const float z = isnan(L) ? __builtin_nanf("") : 0.0f;
        for (int j = lane; j < d; j += 64) {
            double lp = 0.0, lj = 0.0;
            if (!finite) {
                go[j] = z;
            } else if (skip.test(j)) {   // not a parameter (backward-modelled intensity)
                go[j] = 0.0f;
            } else {
                double th, dth, dlj, dlp;
                bijection(table[j], (double)up[j], th, dth, lj, dlj);
                log_prior(table[j], th, lp, dlp);
                go[j] = (float)(((double)gp[j] + dlp) * dth + (with_jac ? dlj : 0.0));
            }
            terms[wv][0][j] = lp;
            terms[wv][1][j] = lj;
        }
    }
    __syncthreads();
    if (active && lane == 0) {
        if (!finite) {
            logp[p] = L;
        } else {
            double lp_sum = 0.0, lj_sum = 0.0;
            for (int j = 0; j < d; ++j) {
                if (skip.test(j)) continue;
                lp_sum += terms[wv][0][j];
                lj_sum += terms[wv][1][j];
            }
            logp[p] = L + lp_sum + (with_jac ? lj_sum : 0.0);
        }
    }
}

// ---------------------------------------------------------------------------
// Adam on loss = -logp (Kingma & Ba 2015), element-wise
// ---------------------------------------------------------------------------
__global__ void k_adam(int P, int d, const float* __restrict__ grad_u, const double* __restrict__ logp,
                       float* __restrict__ u, float* __restrict__ m, float* __restrict__ v,
                       const int* __restrict__ step, AdamHyper hp, float* __restrict__ loss) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P * d) return;
    const int k = *step + 1;
    const float g = -grad_u[q];
    const float mq = fmaf(hp.beta1, m[q], (1.0f - hp.beta1) * g);
    const float vq = fmaf(hp.beta2, v[q], (1.0f - hp.beta2) * g * g);
    m[q] = mq;
    v[q] = vq;
    const double bc1 = 1.0 - pow((double)hp.beta1, (double)k);
    const double bc2 = 1.0 - pow((double)hp.beta2, (double)k);
    const double lr = (double)hp.lr * pow((double)hp.decay, (double)(k - 1));
    const double mh = (double)mq / bc1, vh = (double)vq / bc2;
    u[q] = (float)((double)u[q] - lr * mh / (sqrt(vh) + (double)hp.eps));
    if (q % d == 0 && loss) loss[q / d] = (float)(-logp[q / d]);
}

__global__ void k_add_int(int* c, int inc) { *c += inc; }
__global__ void k_set_int(int* c, int val) { *c = val; }
__global__ void k_set_u64(unsigned long long* c, unsigned long long val) { *c = val; }

// Philox4x32-10 and Box-Muller come from lens_philox.h.
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) { return philox4x32_10(c, k); }
__device__ __forceinline__ double uniform01(uint32_t w) { return philox_uniform01(w); }
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
    philox_box_muller(a, b, z0, z1);
}

// Momenta for one chain: words of counter blocks (chain, t, 0..), 4 normals per block.
__device__ __forceinline__ double momentum(uint2 key, uint32_t chain, uint32_t t, int j) {
    const uint4 w = philox(make_uint4(chain, t, (uint32_t)(j >> 2), 0u), key);
    double z0, z1;
    if ((j & 2) == 0) box_muller(w.x, w.y, z0, z1);
    else box_muller(w.z, w.w, z0, z1);
    return (j & 1) ? z1 : z0;
}

// Start of a transition: save the state, draw momenta, H0, first half kick + drift.
__global__ void k_hmc_begin(int C, int d, HmcArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const uint32_t t = (uint32_t)(*a.transition0 + (uint64_t)*a.tcount);
    const uint2 key = make_uint2((uint32_t)(a.seed & 0xffffffffu), (uint32_t)(a.seed >> 32));
    float* u = a.u + (size_t)c * d;
    float* g = a.grad + (size_t)c * d;
    float* u0 = a.u0 + (size_t)c * d;
    float* g0 = a.g0 + (size_t)c * d;
    float* p = a.p + (size_t)c * d;
    const float eps = a.eps_dev ? *a.eps_dev : a.eps;
    double kin = 0.0;
    for (int j = 0; j < d; ++j) {
        const double im = (double)a.inv_mass[j];
        // a zero inverse mass freezes the coordinate (no momentum, no motion)
        const double pj = im > 0.0 ? momentum(key, (uint32_t)c, t, j) / sqrt(im) : 0.0;
        kin += pj * pj * im;
        u0[j] = u[j];
        g0[j] = g[j];
        const float ph = (float)(pj + 0.5 * (double)eps * (double)g[j]);
        p[j] = ph;
        u[j] = fmaf(eps * a.inv_mass[j], ph, u[j]);
    }
    a.logp0[c] = a.logp[c];
    a.h0[c] = -a.logp[c] + 0.5 * kin;
}

// Interior of the trajectory: full kick with the new gradient, then drift.
__global__ void k_hmc_kick_drift(int C, int d, HmcArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= C * d) return;
    const int j = q % d;
    const float eps = a.eps_dev ? *a.eps_dev : a.eps;
    const float ph = fmaf(eps, a.grad[q], a.p[q]);
    a.p[q] = ph;
    a.u[q] = fmaf(eps * a.inv_mass[j], ph, a.u[q]);
}

// End: last half kick, H1, Metropolis accept (float64 energies), sample.
__global__ void k_hmc_end(int C, int d, HmcArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int tl = *a.tcount;
    const uint32_t t = (uint32_t)(*a.transition0 + (uint64_t)tl);
    const uint2 key = make_uint2((uint32_t)(a.seed & 0xffffffffu), (uint32_t)(a.seed >> 32));
    float* u = a.u + (size_t)c * d;
    float* g = a.grad + (size_t)c * d;
    float* p = a.p + (size_t)c * d;
    const float eps = a.eps_dev ? *a.eps_dev : a.eps;
    double kin = 0.0;
    for (int j = 0; j < d; ++j) {
        const double pj = (double)p[j] + 0.5 * (double)eps * (double)g[j];
        kin += pj * pj * (double)a.inv_mass[j];
    }
    const double h1 = -a.logp[c] + 0.5 * kin;
    if (a.accprob) {
        const double h0 = a.h0[c];
        a.accprob[c] = (isfinite(h0) && isfinite(h1)) ? fmin(1.0, exp(h0 - h1)) : 0.0;
    }
    const uint4 w = philox(make_uint4((uint32_t)c, t, (uint32_t)((d + 3) / 4), 0u), key);
    const double lu = log(uniform01(w.x));
    const bool accept = isfinite(h1) && (lu < a.h0[c] - h1);
    if (!accept) {
        const float* u0 = a.u0 + (size_t)c * d;
        const float* g0 = a.g0 + (size_t)c * d;
        for (int j = 0; j < d; ++j) { u[j] = u0[j]; g[j] = g0[j]; }
        a.logp[c] = a.logp0[c];
    }
    if (a.accepts && accept) a.accepts[c] += 1;
    if (a.samples) {
        float* s = a.samples + ((size_t)tl * C + c) * d;
        for (int j = 0; j < d; ++j) s[j] = u[j];
    }
}

// ---------------------------------------------------------------------------
// Burn-in adaptation.  Step size: dual averaging (Hoffman & Gelman 2014,
// Sec. 3.2.1; gamma 0.05, t0 10, kappa 0.75) on the chain mean of the
// acceptance statistic, one shared step size.  Mass matrix (Sec. 3.3): the
// variance of the positions over a window of transitions, from per-chain
// Welford sums combined across chains.
// ---------------------------------------------------------------------------
__global__ void k_hmc_adapt_init(int n, double* state, float* eps_dev, float eps0, double* wmean, double* wm2,
                                 int* wcount) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) {
        wmean[q] = 0.0;
        wm2[q] = 0.0;
    }
    if (q == 0) {
        state[0] = log(10.0 * (double)eps0);
        state[1] = log((double)eps0);
        state[2] = 0.0;
        state[3] = 0.0;
        state[4] = 0.0;
        *eps_dev = eps0;
        *wcount = 0;
    }
}

__global__ __launch_bounds__(256) void k_hmc_adapt(int C, AdaptArgs a) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int c = tid; c < C; c += 256) s += a.accprob[c];
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid != 0) return;
    const double alpha = red[0] / (double)C;
    if (a.eps_trace) a.eps_trace[*a.tcount] = *a.eps_dev;
    constexpr double GAMMA = 0.05, T0 = 10.0, KAPPA = 0.75;
    double* st = a.state;
    const double m = st[4] + 1.0;
    const double eta = 1.0 / (m + T0);
    const double hb = (1.0 - eta) * st[3] + eta * ((double)a.delta - alpha);
    const double le = st[0] - sqrt(m) / GAMMA * hb;
    const double w = pow(m, -KAPPA);
    const double leb = w * le + (1.0 - w) * st[2];
    st[1] = le;
    st[2] = leb;
    st[3] = hb;
    st[4] = m;
    *a.eps_dev = (float)exp(le);
    if (a.eps_final) *a.eps_final = (float)exp(leb);
}

// After transition t of the run (t = *tcount): positions of transitions
// t >= window_start enter each chain's running mean and sum of squared
// deviations (Welford); k_hmc_wcount then counts the window sample.
__global__ void k_hmc_welford(int C, int d, const float* __restrict__ u, const int* __restrict__ tcount,
                              int window_start, double* __restrict__ wmean, double* __restrict__ wm2,
                              const int* __restrict__ wcount) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= C * d || *tcount < window_start) return;
    const double n = (double)(*wcount + 1);
    const double x = (double)u[q];
    const double dl = x - wmean[q];
    const double mn = wmean[q] + dl / n;
    wmean[q] = mn;
    wm2[q] = fma(dl, x - mn, wm2[q]);
}

__global__ void k_hmc_wcount(const int* tcount, int window_start, int* wcount) {
    if (*tcount >= window_start) *wcount += 1;
}

// Variance over chains and window transitions of coordinate j (work-group j):
// grand mean of the chain means, then sum_c M2_c + n sum_c (mean_c - grand)^2
// over n C - 1; fixed-order sums.
__global__ __launch_bounds__(256) void k_hmc_window_var(int C, int d, const double* __restrict__ wmean,
                                                        const double* __restrict__ wm2,
                                                        const int* __restrict__ wcount, float* __restrict__ var) {
    __shared__ double red[256];
    const int j = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int c = tid; c < C; c += 256) s += wmean[(size_t)c * d + j];
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    const double gm = red[0] / (double)C;
    __syncthreads();
    const double n = (double)(*wcount);
    s = 0.0;
    for (int c = tid; c < C; c += 256) {
        const double dm = wmean[(size_t)c * d + j] - gm;
        s += wm2[(size_t)c * d + j] + n * dm * dm;
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) var[j] = (n * C > 1.0) ? (float)(red[0] / (n * C - 1.0)) : __builtin_nanf("");
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline dim3 blocks_for(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_hmc_adapt_init(int C, int d, double* state, float* eps_dev, float eps0, double* wmean, double* wm2,
                                 int* wcount, hipStream_t st) {
    const long n = (long)C * d;
    hipLaunchKernelGGL(k_hmc_adapt_init, blocks_for(n > 0 ? n : 1, 256), dim3(256), 0, st, (int)n, state, eps_dev,
                       eps0, wmean, wm2, wcount);
    return hipGetLastError();
}

hipError_t launch_hmc_adapt(int C, const AdaptArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_adapt, dim3(1), dim3(256), 0, st, C, a);
    return hipGetLastError();
}

hipError_t launch_hmc_welford(int C, int d, const float* u, const int* tcount, int window_start, double* wmean,
                              double* wm2, int* wcount, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_welford, blocks_for((long)C * d, 256), dim3(256), 0, st, C, d, u, tcount, window_start,
                       wmean, wm2, wcount);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_hmc_wcount, dim3(1), dim3(1), 0, st, tcount, window_start, wcount);
    return hipGetLastError();
}

hipError_t launch_hmc_window_var(int C, int d, const double* wmean, const double* wm2, const int* wcount, float* var,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_window_var, dim3(d), dim3(256), 0, st, C, d, wmean, wm2, wcount, var);
    return hipGetLastError();
}

hipError_t launch_bijection(int P, int d, const PriorRow* table, const float* u, float* theta,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_bijection, blocks_for((long)P * d, 256), dim3(256), 0, st, P, d, table, u,
                       theta);
    return hipGetLastError();
}

hipError_t launch_posterior(int P, int d, const PriorRow* table, const float* u, const double* logl,
                            const float* gtheta, int with_jac, double* logp, float* grad_u,
                            hipStream_t st, const ParamMask& skip) {
    if (d < 1 || d > PARAM_MASK_BITS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_posterior, dim3((P + POST_WAVES - 1) / POST_WAVES), dim3(64 * POST_WAVES), 0, st, P, d,
                       table, u, logl, gtheta, with_jac, skip, logp, grad_u);
    return hipGetLastError();
}

hipError_t launch_adam(int P, int d, const float* grad_u, const double* logp, float* u, float* m,
                       float* v, const int* step, const AdamHyper& hp, float* loss,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_adam, blocks_for((long)P * d, 256), dim3(256), 0, st, P, d, grad_u, logp, u,
                       m, v, step, hp, loss);
    return hipGetLastError();
}

hipError_t launch_add_int(int* c, int inc, hipStream_t st) {
    hipLaunchKernelGGL(k_add_int, dim3(1), dim3(1), 0, st, c, inc);
    return hipGetLastError();
}

hipError_t launch_set_int(int* c, int val, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, c, val);
    return hipGetLastError();
}

hipError_t launch_set_int_host(int* c, int val, hipStream_t st) { return launch_set_int(c, val, st); }

hipError_t launch_set_u64(unsigned long long* c, unsigned long long val, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, c, val);
    return hipGetLastError();
}

hipError_t launch_hmc_begin(int C, int d, const HmcArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_begin, blocks_for(C, 64), dim3(64), 0, st, C, d, a);
    return hipGetLastError();
}

hipError_t launch_hmc_kick_drift(int C, int d, const HmcArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_kick_drift, blocks_for((long)C * d, 256), dim3(256), 0, st, C, d, a);
    return hipGetLastError();
}

hipError_t launch_hmc_end(int C, int d, const HmcArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_end, blocks_for(C, 64), dim3(64), 0, st, C, d, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch helpers: best particle per system, centred fixed-size image views
// ---------------------------------------------------------------------------
// One work-group per system: minimum of val over the system's particles
// [p0[k], p0[k+1]) and the (global) index of its first occurrence; NaN counts
// as +inf.
__global__ __launch_bounds__(256) void k_segment_argmin(const int* __restrict__ p0,
                                                        const float* __restrict__ val,
                                                        float* __restrict__ best, int* __restrict__ arg) {
    const int k = blockIdx.x, t = threadIdx.x;
    const int a = p0[k], b = p0[k + 1];
    float bv = __builtin_inff();
    int bi = b;
    for (int i = a + t; i < b; i += 256) {
        float x = val[i];
        if (x != x) x = __builtin_inff();
        if (x < bv || (x == bv && i < bi)) {
            bv = x;
            bi = i;
        }
    }
    __shared__ float sv[256];
    __shared__ int si[256];
    sv[t] = bv;
    si[t] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            const float ov = sv[t + o];
            const int oi = si[t + o];
            if (ov < sv[t] || (ov == sv[t] && oi < si[t])) {
                sv[t] = ov;
                si[t] = oi;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        best[k] = sv[0];
        arg[k] = si[0] < b ? si[0] : a;
    }
}

// out[k][i][j] = system k's image at the centre-aligned position of pixel
// (i, j) of a side x side grid with the same pixel scale: source row
// i + (ny - side) / 2 (likewise columns); a half-integer offset averages the
// two neighbours, pixels outside the image count as zero.
__global__ void k_center_views(int side, const ViewSrc* __restrict__ src, float* __restrict__ out) {
    const int k = blockIdx.y;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= side * side) return;
    const ViewSrc v = src[k];
    const int i = q / side, j = q - i * side;
    const int r2 = 2 * i + (v.ny - side), c2 = 2 * j + (v.nx - side);
    const int r0 = (r2 - (r2 & 1)) / 2, r1 = (r2 + (r2 & 1)) / 2;
    const int c0 = (c2 - (c2 & 1)) / 2, c1 = (c2 + (c2 & 1)) / 2;
    auto at = [&](int r, int c) -> double {
        return (r >= 0 && r < v.ny && c >= 0 && c < v.nx) ? (double)v.data[(size_t)r * v.nx + c] : 0.0;
    };
    const double val = 0.25 * (at(r0, c0) + at(r0, c1) + at(r1, c0) + at(r1, c1));
    out[(size_t)k * side * side + q] = (float)val;
}

hipError_t launch_inverse_bijection(int P, int d, const PriorRow* table, const float* theta, float* u,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_inverse_bijection, blocks_for((long)P * d, 256), dim3(256), 0, st, P, d, table, theta, u);
    return hipGetLastError();
}

hipError_t launch_segment_argmin(int S, const int* p0, const float* val, float* best, int* arg,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_segment_argmin, dim3(S), dim3(256), 0, st, p0, val, best, arg);
    return hipGetLastError();
}

hipError_t launch_center_views(int S, int side, const ViewSrc* src, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_center_views, dim3((side * side + 255) / 256, S), dim3(256), 0, st, side, src, out);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// SVI (Sec. 3: eq. vi, eq. elbo, eq. elbo-grad; Sec. 3.2: AdaBelief).
// Surrogate N(mu, L L^T) over the unconstrained parameters; phi = mu, then
// the lower triangle of L row by row, diagonal entries stored as rho with
// L_jj = softplus(rho) + SVI_DIAG_SHIFT.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }

// One work-group of 256 threads draws 256 samples: eps by Philox4x32-10 with
// counters (sample, step, block, SVI_RNG_TAG) and Box-Muller, u = mu + L eps,
// log q(u) = -|eps|^2/2 - log det L - (d/2) log 2 pi.  eps is stored [d][n].
__global__ __launch_bounds__(256) void k_svi_draw(SviArgs a) {
    __shared__ double Lp[SVI_MAX_D * (SVI_MAX_D + 1) / 2];
    __shared__ double mu[SVI_MAX_D];
    __shared__ double logdet;
    const int d = a.d, n = a.n;
    const int r = threadIdx.x;
    if (r < d) {
        const int t0 = r * (r + 1) / 2;
        mu[r] = (double)a.phi[r];
        for (int c = 0; c < r; ++c) Lp[t0 + c] = (double)a.phi[d + t0 + c];
        Lp[t0 + r] = softplus_d((double)a.phi[d + t0 + r]) + SVI_DIAG_SHIFT;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sl = 0.0;
        for (int j = 0; j < d; ++j) sl += log(Lp[j * (j + 3) / 2]);
        logdet = sl;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t step = (uint32_t)*a.step;
    const uint2 key = make_uint2((uint32_t)(a.seed & 0xffffffffu), (uint32_t)(a.seed >> 32));
    double* eps = a.eps;
    double ss = 0.0;
    for (int b = 0; 4 * b < d; ++b) {
        const uint4 w = philox(make_uint4((uint32_t)i, step, (uint32_t)b, SVI_RNG_TAG), key);
        double z[4];
        box_muller(w.x, w.y, z[0], z[1]);
        box_muller(w.z, w.w, z[2], z[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * b + q;
            if (j < d) {
                eps[(size_t)j * n + i] = z[q];
                ss += z[q] * z[q];
            }
        }
    }
    a.logq[i] = -0.5 * ss - logdet - 0.5 * (double)d * 1.8378770664093454836;   // log 2 pi
    for (int j = 0; j < d; ++j) {
        const double* Lr = Lp + j * (j + 1) / 2;
        double acc = mu[j];
        for (int c = 0; c <= j; ++c) acc = fma(Lr[c], eps[(size_t)c * n + i], acc);
        a.u[(size_t)i * d + j] = (float)acc;
    }
}

// Work-group 0: the ELBO estimate mean(log q - logp).  Work-group 1 + e: the
// pathwise gradient of entry e of phi,
//   mu_j:      -mean_i g_ij
//   L_rc:      -mean_i g_ir eps_ic                      (c < r)
//   rho_r:     (-mean_i g_ir eps_ir - 1/L_rr) sigmoid(rho_r)
// with g = dlogp/du, each a fixed-order float64 sum; then (if update) one
// Adam or AdaBelief step of that entry.  Every work-group reads and writes
// only its own entry of phi, m and s.
__global__ __launch_bounds__(256) void k_svi_reduce(SviArgs a) {
    __shared__ double red[256];
    const int n = a.n, d = a.d, tid = threadIdx.x;
    const int e = (int)blockIdx.x - 1;
    int r = 0, c = 0;
    double acc = 0.0;
    bool frozen = false;
    if (e >= d) {
        const int t = e - d;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        c = t - r * (r + 1) / 2;
        frozen = ((a.frozen >> r) & 1u) || ((a.frozen >> c) & 1u);
    } else if (e >= 0) {
        frozen = (a.frozen >> e) & 1u;
    }
    if (e < 0) {
        for (int i = tid; i < n; i += 256) acc += a.logq[i] - a.logp[i];
    } else if (frozen) {
        acc = 0.0;
    } else if (e < d) {
        for (int i = tid; i < n; i += 256) acc -= (double)a.grad_u[(size_t)i * d + e];
    } else {
        const double* ec = a.eps + (size_t)c * n;
        for (int i = tid; i < n; i += 256) acc -= (double)a.grad_u[(size_t)i * d + r] * ec[i];
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid != 0) return;
    double v = red[0] / (double)n;
    if (e < 0) {
        if (a.elbo) a.elbo[a.call_step ? *a.call_step : 0] = v;
        return;
    }
    if (e >= d && r == c && !frozen) {
        const double rho = (double)a.phi[e];
        v = (v - 1.0 / (softplus_d(rho) + SVI_DIAG_SHIFT)) * sigmoid_d(rho);
    }
    if (a.grad_phi) a.grad_phi[e] = (float)v;
    if (!a.update || frozen) return;
    const int k = *a.step + 1;
    const double b1 = (double)a.beta1, b2 = (double)a.beta2, ep = (double)a.eps_opt;
    const double m = b1 * (double)a.m[e] + (1.0 - b1) * v;
    double s;
    if (a.optimizer == SVI_OPT_ADABELIEF) {
        const double dv = v - m;
        s = b2 * (double)a.s[e] + (1.0 - b2) * dv * dv + ep;
    } else {
        s = b2 * (double)a.s[e] + (1.0 - b2) * v * v;
    }
    a.m[e] = (float)m;
    a.s[e] = (float)s;
    const double mh = m / (1.0 - pow(b1, (double)k));
    const double sh = s / (1.0 - pow(b2, (double)k));
    a.phi[e] = (float)((double)a.phi[e] - (double)a.lr * mh / (sqrt(sh) + ep));
}

// mean, covariance L L^T [d][d] and its diagonal, each optional.
__global__ void k_svi_moments(int d, const float* __restrict__ phi, float* __restrict__ mean,
                              float* __restrict__ cov, float* __restrict__ var) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d * d) return;
    const int i = q / d, j = q - (q / d) * d;
    auto Lat = [&](int r, int c) -> double {
        const int t = r * (r + 1) / 2 + c;
        const double x = (double)phi[d + t];
        return r == c ? softplus_d(x) + SVI_DIAG_SHIFT : x;
    };
    double acc = 0.0;
    const int kmax = i < j ? i : j;
    for (int k = 0; k <= kmax; ++k) acc = fma(Lat(i, k), Lat(j, k), acc);
    if (cov) cov[q] = (float)acc;
    if (i == j) {
        if (var) var[i] = (float)acc;
        if (mean) mean[i] = phi[i];
    }
}

hipError_t launch_svi_draw(const SviArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_svi_draw, blocks_for(a.n, 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_svi_reduce(const SviArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_svi_reduce, dim3((unsigned)(1 + svi_num_params(a.d))), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_svi_moments(int d, const float* phi, float* mean, float* cov, float* var, hipStream_t st) {
    hipLaunchKernelGGL(k_svi_moments, blocks_for((long)d * d, 256), dim3(256), 0, st, d, phi, mean, cov, var);
    return hipGetLastError();
}

}  // namespace lens
