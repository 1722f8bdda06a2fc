// Backward ("linear inversion") likelihood: the Sersic intensities are solved
// for, not sampled (Sec. 3: forward vs backward modelling of the surface
// brightness).  For fixed nonlinear parameters the model image is
// m = sum_k A_k B_k, with B_k the PSF-convolved, downsampled image of light
// component k at unit intensity; the intensities minimise
// chi^2 = sum w (d - m)^2, i.e. solve M A = b with M_kl = sum w B_k B_l and
// b_k = sum w B_k d.  The component images come from a render pass that
// writes each component's image separately and the ordinary PSF kernel;
// the kernels here set the intensities to 1, reduce and solve the normal
// equations per particle in float64, assemble the model image at the solved
// intensities from the component images, and clear the intensity entries of
// the gradient (which, by the envelope theorem, is the forward gradient at
// the solved intensities).
#include <math.h>
#include <stdint.h>

#include "lens_backward.h"
#include "lens_internal.h"

namespace lens {

__global__ void k_bwd_expand(int P, BwdSlots s, const float* __restrict__ theta, float* __restrict__ th1) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)P * s.d) return;
    const int j = (int)(q % s.d);
    float v = theta[q];
    for (int c = 0; c < s.K; ++c)
        if (s.slot[c] == j) v = 1.0f;
    th1[q] = v;
}

// Solve M x = b (K x K, symmetric positive semi-definite) by Cholesky in
// index order; a component whose pivot is not above BWD_PIVOT_REL x max diag
// is left out (x_k = 0).
template <int K>
__device__ void solve_skip(const double (&M)[K][K], const double (&b)[K], double (&x)[K]) {
    double Lc[K][K];
    bool on[K];
    double dmax = 0.0;
    for (int j = 0; j < K; ++j) dmax = fmax(dmax, M[j][j]);
    const double tol = BWD_PIVOT_REL * dmax;
    for (int j = 0; j < K; ++j) {
        double s = M[j][j];
        for (int i = 0; i < j; ++i)
            if (on[i]) s -= Lc[j][i] * Lc[j][i];
        on[j] = s > tol;
        if (!on[j]) continue;
        Lc[j][j] = sqrt(s);
        for (int r = j + 1; r < K; ++r) {
            double t = M[r][j];
            for (int i = 0; i < j; ++i)
                if (on[i]) t -= Lc[r][i] * Lc[j][i];
            Lc[r][j] = t / Lc[j][j];
        }
    }
    double y[K];
    for (int j = 0; j < K; ++j) {
        if (!on[j]) continue;
        double t = b[j];
        for (int i = 0; i < j; ++i)
            if (on[i]) t -= Lc[j][i] * y[i];
        y[j] = t / Lc[j][j];
    }
    for (int j = K - 1; j >= 0; --j) {
        if (!on[j]) {
            x[j] = 0.0;
            continue;
        }
        double t = y[j];
        for (int r = j + 1; r < K; ++r)
            if (on[r]) t -= Lc[r][j] * x[r];
        x[j] = t / Lc[j][j];
    }
}

// One work-group of 256 threads per particle: fixed-order float64 sums of
// the K(K+1)/2 + K normal-equation entries over the pixels, then one thread
// solves.
template <int K>
__global__ __launch_bounds__(256) void k_bwd_normal(int P, BwdSlots s, int npix, const float* __restrict__ B,
                                                    const float* __restrict__ data,
                                                    const float* __restrict__ invvar,
                                                    const float* __restrict__ consts,
                                                    const float* __restrict__ theta, float* __restrict__ theta_full,
                                                    float* __restrict__ amp) {
    constexpr int NM = K * (K + 1) / 2;
    constexpr int NV = NM + K;
    __shared__ double red[NV][256];
    const int p = blockIdx.x, tid = threadIdx.x;
    const float* Bp = B + (size_t)p * K * npix;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int pix = tid; pix < npix; pix += 256) {
        const double w = (double)invvar[pix], dd = (double)data[pix];
        double bk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) bk[k] = (double)Bp[(size_t)k * npix + pix];
        int v = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double wb = w * bk[k];
#pragma unroll
            for (int l = 0; l <= k; ++l) {
                acc[v] = fma(wb, bk[l], acc[v]);
                ++v;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) acc[NM + k] = fma(w * bk[k], dd, acc[NM + k]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][tid] = acc[v];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
#pragma unroll
            for (int v = 0; v < NV; ++v) red[v][tid] += red[v][tid + h];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const int d = s.d;
    const bool valid = consts[(size_t)p * CSTRIDE + C_VALID] == 1.0f;
    double M[K][K], b[K], x[K];
    int v = 0;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l <= k; ++l) {
            M[k][l] = red[v][0];
            M[l][k] = red[v][0];
            ++v;
        }
    for (int k = 0; k < K; ++k) b[k] = red[NM + k][0];
    if (valid) {
        solve_skip<K>(M, b, x);
    } else {
        for (int k = 0; k < K; ++k) x[k] = __builtin_nan("");
    }
    const float* tp = theta + (size_t)p * d;
    float* tf = theta_full + (size_t)p * d;
    for (int j = 0; j < d; ++j) tf[j] = tp[j];
    for (int k = 0; k < K; ++k) {
        tf[s.slot[k]] = valid ? (float)x[k] : 0.0f;
        if (amp) amp[(size_t)p * K + k] = (float)x[k];
    }
}

// K > BWD_SMALL_K (a shapelet source's coefficients are components too):
// one work-group of 256 threads per particle.  Pixels are staged in tiles of
// BWD_TILE through LDS as float64 w B_k and B_k; thread t owns entries t,
// t + 256, ... of the packed list (the lower triangle of M row by row, then
// b), each summed over the pixels in order.  Wave 0 then factors M in LDS by
// the same pivot-skipping Cholesky as solve_skip (lanes over the rows of a
// column) and lane 0 substitutes.
constexpr int BWD_TILE = 32;
constexpr int BWD_ENT = (BWD_MAX_K * (BWD_MAX_K + 1) / 2 + BWD_MAX_K + 255) / 256;

__global__ __launch_bounds__(256) void k_bwd_normal_big(int P, BwdSlots s, int npix, const float* __restrict__ B,
                                                       const float* __restrict__ data,
                                                       const float* __restrict__ invvar,
                                                       const float* __restrict__ consts,
                                                       const float* __restrict__ theta,
                                                       float* __restrict__ theta_full, float* __restrict__ amp) {
    __shared__ double wb[BWD_MAX_K][BWD_TILE];
    __shared__ double bt[BWD_MAX_K + 1][BWD_TILE];   // row K: the data
    __shared__ double M[BWD_MAX_K][BWD_MAX_K];
    __shared__ double rhs[BWD_MAX_K], xs[BWD_MAX_K];
    __shared__ int on[BWD_MAX_K];
    const int K = s.K, p = blockIdx.x, tid = threadIdx.x;
    const int nm = K * (K + 1) / 2, ne = nm + K;
    const float* Bp = B + (size_t)p * K * npix;
    int ek[BWD_ENT], el[BWD_ENT];
    double acc[BWD_ENT];
#pragma unroll
    for (int q = 0; q < BWD_ENT; ++q) {
        const int e = tid + 256 * q;
        ek[q] = -1;
        el[q] = -1;
        acc[q] = 0.0;
        if (e < nm) {
            int k = 0;
            while ((k + 1) * (k + 2) / 2 <= e) ++k;
            ek[q] = k;
            el[q] = e - k * (k + 1) / 2;
        } else if (e < ne) {
            ek[q] = e - nm;
            el[q] = K;   // the data row
        }
    }
    for (int p0 = 0; p0 < npix; p0 += BWD_TILE) {
        __syncthreads();
        for (int q = tid; q < (K + 1) * BWD_TILE; q += 256) {
            const int k = q / BWD_TILE, t = q - k * BWD_TILE, pix = p0 + t;
            const bool in = pix < npix;
            const double w = in ? (double)invvar[pix] : 0.0;
            const double v = in ? (k < K ? (double)Bp[(size_t)k * npix + pix] : (double)data[pix]) : 0.0;
            bt[k][t] = v;
            if (k < K) wb[k][t] = w * v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < BWD_ENT; ++q) {
            if (ek[q] < 0) continue;
            const int k = ek[q], l = el[q];
            double a = acc[q];
            for (int t = 0; t < BWD_TILE; ++t) a = fma(wb[k][t], bt[l][t], a);
            acc[q] = a;
        }
    }
#pragma unroll
    for (int q = 0; q < BWD_ENT; ++q) {
        if (ek[q] < 0) continue;
        if (el[q] < K) {
            M[ek[q]][el[q]] = acc[q];
        } else {
            rhs[ek[q]] = acc[q];
        }
    }
    __syncthreads();
    // pivot threshold relative to the largest diagonal entry
    double dmax = 0.0;
    for (int j = 0; j < K; ++j) dmax = fmax(dmax, M[j][j]);
    const double tol = BWD_PIVOT_REL * dmax;
    // in-place Cholesky of the lower triangle, column by column: every thread
    // evaluates the pivot (same value), the first wave the column below it;
    // every thread reaches every barrier
    for (int j = 0; j < K; ++j) {
        double sj = M[j][j];
        for (int i = 0; i < j; ++i)
            if (on[i]) sj -= M[j][i] * M[j][i];
        const bool onj = sj > tol;
        const double ljj = onj ? sqrt(sj) : 1.0;
        __syncthreads();
        if (tid == 0) {
            on[j] = onj ? 1 : 0;
            M[j][j] = ljj;
        }
        if (onj && tid < 64) {
            for (int r = j + 1 + tid; r < K; r += 64) {
                double t = M[r][j];
                for (int i = 0; i < j; ++i)
                    if (on[i]) t -= M[r][i] * M[j][i];
                M[r][j] = t / ljj;
            }
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const bool valid = consts[(size_t)p * CSTRIDE + C_VALID] == 1.0f;
    for (int j = 0; j < K; ++j) {   // L y = b
        if (!on[j]) continue;
        double t = rhs[j];
        for (int i = 0; i < j; ++i)
            if (on[i]) t -= M[j][i] * xs[i];
        xs[j] = t / M[j][j];
    }
    for (int j = K - 1; j >= 0; --j) {   // L^T x = y
        if (!on[j]) {
            xs[j] = 0.0;
            continue;
        }
        double t = xs[j];
        for (int r = j + 1; r < K; ++r)
            if (on[r]) t -= M[r][j] * xs[r];
        xs[j] = t / M[j][j];
    }
    const int d = s.d;
    const float* tp = theta + (size_t)p * d;
    float* tf = theta_full + (size_t)p * d;
    for (int j = 0; j < d; ++j) tf[j] = tp[j];
    for (int k = 0; k < K; ++k) {
        const double x = valid ? xs[k] : (double)__builtin_nan("");
        tf[s.slot[k]] = valid ? (float)x : 0.0f;
        if (amp) amp[(size_t)p * K + k] = (float)x;
    }
}

// Pre-PSF model image at the solved intensities, sum_k A_k b_k, from the
// component images b_k of the split render (the PSF is linear, so this is
// the image the render would produce at those intensities; NaN images of an
// invalid particle stay NaN).
__global__ void k_bwd_assemble(int P, BwdSlots s, int npix, const float* __restrict__ comp,
                               const float* __restrict__ theta_full, float* __restrict__ out) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)P * npix) return;
    const long p = q / npix;
    const long pix = q - p * npix;
    double acc = 0.0;
    for (int k = 0; k < s.K; ++k)
        acc = fma((double)theta_full[p * s.d + s.slot[k]], (double)comp[(p * s.K + k) * npix + pix], acc);
    out[q] = (float)acc;
}

__global__ void k_bwd_zero_slots(int P, BwdSlots s, float* __restrict__ grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P * s.K) return;
    const int p = q / s.K, k = q - (q / s.K) * s.K;
    grad[(size_t)p * s.d + s.slot[k]] = 0.0f;
}

hipError_t launch_bwd_expand(int P, const BwdSlots& s, const float* theta, float* th1, hipStream_t st) {
    const long total = (long)P * s.d;
    hipLaunchKernelGGL(k_bwd_expand, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, s, theta, th1);
    return hipGetLastError();
}

hipError_t launch_bwd_normal(int P, const BwdSlots& s, int npix, const float* B, const float* data,
                             const float* invvar, const float* consts, const float* theta, float* theta_full,
                             float* amp, hipStream_t st) {
    switch (s.K) {
#define LENS_BWD_CASE(KK)                                                                                  \
    case KK:                                                                                               \
        hipLaunchKernelGGL(k_bwd_normal<KK>, dim3(P), dim3(256), 0, st, P, s, npix, B, data, invvar, consts,   \
                           theta, theta_full, amp);                                                        \
        break;
        LENS_BWD_CASE(1) LENS_BWD_CASE(2) LENS_BWD_CASE(3) LENS_BWD_CASE(4) LENS_BWD_CASE(5) LENS_BWD_CASE(6)
#undef LENS_BWD_CASE
        default:
            if (s.K < 1 || s.K > BWD_MAX_K) return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_bwd_normal_big, dim3(P), dim3(256), 0, st, P, s, npix, B, data, invvar, consts,
                               theta, theta_full, amp);
    }
    return hipGetLastError();
}

hipError_t launch_bwd_assemble(int P, const BwdSlots& s, int npix, const float* comp, const float* theta_full,
                               float* out, hipStream_t st) {
    const long total = (long)P * npix;
    hipLaunchKernelGGL(k_bwd_assemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, s, npix, comp,
                       theta_full, out);
    return hipGetLastError();
}

hipError_t launch_bwd_zero_slots(int P, const BwdSlots& s, float* grad, hipStream_t st) {
    hipLaunchKernelGGL(k_bwd_zero_slots, dim3((unsigned)((P * s.K + 255) / 256)), dim3(256), 0, st, P, s, grad);
    return hipGetLastError();
}

}  // namespace lens
