// HIP kernels (gfx950) of the batched strong-lens forward model, Gaussian
// log-likelihood and its adjoint gradient.
//
// Model (paper Sec. 3): elliptical power-law (EPL) or SIE mass + external
// shear; elliptical Sersic lens light evaluated on the image plane and
// Sersic sources evaluated at beta = theta - alpha; integer supersampling
// (Sec. 4.2 footnote), mean downsampling, PSF convolution, Gaussian logL.
//
// Kernels, in launch order for one call over P particles:
//   k_prologue  one thread per particle: derived constants (float words) into
//               a per-particle block read later with wave-uniform loads.
//   k_render    grid (P, pixel chunks): each thread owns whole pixels and sums
//               their s*s sub-pixel values (ray shooting + light) -> image.
//   k_psf       one work-group per particle: image tile in LDS with a zero
//               halo, register-blocked direct correlation with the flipped
//               PSF (= true convolution), residual and chi^2 (float64 sum),
//               then the adjoint (correlation with the unflipped PSF) of the
//               residual, written back in place.
//   k_adjoint   grid (P, pixel chunks): recomputes every sub-pixel and
//               accumulates the reverse-mode sums that the gradient needs;
//               fixed-order work-group reduction to float64 partials.
//   k_finalize  one thread per particle: sums the partials in fixed order and
//               applies the per-particle chain rule -> dlogL/dtheta.
//
// Parametrisation used on the device (equivalent to the rotated-frame
// definition, but smooth in the complex ellipticity eps = e1 + i e2, so the
// gradient with respect to e1, e2 stays well conditioned as |eps| -> 0):
//   c = |eps|, q = (1-c)/(1+c), w = (x - x0) + i (y - y0).
//   EPL (Tessore & Metcalf 2015): U = (w - eps conj(w))/(1+c) equals
//   e^{i phi}(q x' + i y') in the image frame, so R = |U|, V0 = U/R and
//       alpha = theta_E sqrt(1-c^2) (b/R)^(t-1) V0 S(z),  z = -conj(eps) V0^2,
//       S(z) = sum_n c_n z^n,  c_n = prod_{k<=n} (2k-2+t)/(2k+2-t),
//   with b = theta_E sqrt(q), t = gamma - 1.  SIE is the t = 1 member.
//   Sersic: R^2 = q x'^2 + y'^2/q = a11 dx^2 + 2 a12 dx dy + a22 dy^2 with
//       a11 = (1+c^2-2e1)/(1-c^2), a22 = (1+c^2+2e1)/(1-c^2), a12 = -2e2/(1-c^2).
#include <math.h>

#include <type_traits>

#include "lens_internal.h"

namespace lens {

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

constexpr float HALF_LN2 = 0.34657359027997264f;

// ---------------------------------------------------------------------------
// Precision split.  Near the cusp of a compact Sersic profile the model value
// is very sensitive to the evaluation point; FP32 rounding of the grid
// coordinates (~1e-7") or of the deflection (~1e-7 relative) would change
// pixel values by ~1e-4 relative.  Near the optimum the residual d - m is a
// small difference of large numbers, so the model value itself must be good
// to ~1e-8 relative for the gradient to keep its accuracy.  Hence:
//   float64: grid coordinates, mass deflection, shear, lens equation, the
//            Sersic values of the model image, the sub-pixel sum, the PSF
//            convolution of the model and the residual (float64 FMA issues
//            at the rate of unpacked float32 FMA on this GPU; exp2/log2 are
//            evaluated by range reduction + polynomials, below);
//   float32: the adjoint sweep (Sersic derivatives, series derivatives,
//            chain rule), whose terms need only ~1e-7 relative accuracy.
// ---------------------------------------------------------------------------
struct SersicK {
    double xc, yc, a11, a12, a22, ie, ku, ku0, bl, a12x2;   // model value (float64)
    float a11f, a12f, a22f, ief, kuf, ku0f, blf, kap2;  // adjoint (float32)
};

template <int NC>
struct PK {
    double x0, y0, e1, e2, ua, ub, ue, c0, k0, k1, g1, g2;
    float e1f, e2f, k1f;
    int kp, kpa;
    bool quad;   // float32 adjoint series by the quadratic-division recurrence (|e| < 0.55)
    SersicK s[NC > 0 ? NC : 1];
};

// Per-particle constants are read through the constant address space: they
// do not change during a kernel, so uniform loads of them are scalar loads
// even through a pointer the compiler cannot otherwise reason about.
typedef const __attribute__((address_space(4))) float cfloat_t;
typedef const __attribute__((address_space(4))) double cdouble_t;

__device__ __forceinline__ double ldd(const float* __restrict__ C, int w) {
    return *(cdouble_t*)(C + w);
}
__device__ __forceinline__ float ldf(const float* __restrict__ C, int w) { return *(cfloat_t*)(C + w); }

__device__ __forceinline__ SersicK load_sersic(const float* __restrict__ S) {
    SersicK q;
    q.xc = ldd(S, S_XC); q.yc = ldd(S, S_YC);
    q.a11 = ldd(S, S_A11); q.a12 = ldd(S, S_A12); q.a22 = ldd(S, S_A22);
    q.ie = ldd(S, S_IE); q.ku = ldd(S, S_KU); q.ku0 = ldd(S, S_KU0); q.bl = ldd(S, S_BL);
    q.a12x2 = ldd(S, S_A12X2);
    q.a11f = (float)q.a11; q.a12f = (float)q.a12; q.a22f = (float)q.a22;
    // the exponent constants are stored times 256 (exp2_256); the float32
    // copies undo the power-of-two factor exactly
    q.ief = (float)q.ie; q.kuf = (float)(q.ku * (1.0 / 256.0)); q.ku0f = (float)(q.ku0 * (1.0 / 256.0));
    q.blf = (float)(q.bl * (1.0 / 256.0));
    q.kap2 = ldf(S, S_KAP2);
    return q;
}

template <int NC>
__device__ __forceinline__ PK<NC> load_pk(const float* __restrict__ C) {
    PK<NC> k;
    k.x0 = ldd(C, D_X0); k.y0 = ldd(C, D_Y0); k.e1 = ldd(C, D_E1); k.e2 = ldd(C, D_E2);
    k.ua = ldd(C, D_UA); k.ub = ldd(C, D_UB); k.ue = ldd(C, D_UE); k.c0 = ldd(C, D_C0);
    k.k0 = ldd(C, D_K0); k.k1 = ldd(C, D_K1); k.g1 = ldd(C, D_G1); k.g2 = ldd(C, D_G2);
    k.e1f = (float)k.e1; k.e2f = (float)k.e2; k.k1f = (float)(k.k1 * (1.0 / 256.0));
    k.kp = (int)ldf(C, C_KP);
    k.kpa = (int)ldf(C, C_KPA);
    k.quad = fma(k.e1, k.e1, k.e2 * k.e2) < 0.3025;
#pragma unroll
    for (int c = 0; c < NC; ++c) k.s[c] = load_sersic(C + C_SERS + c * SERS_STRIDE);
    return k;
}

// The pointer itself, hidden from loop-invariant code motion and from the
// scheduler (an empty volatile asm statement), so that the constants read
// through it are loaded (scalar loads) where they are used instead of being
// kept live, and spilled, across the whole sub-pixel loop.
__device__ __forceinline__ const float* opaque(const float* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// ---------------------------------------------------------------------------
// float64 exp2 / log2 for the model values (no float64 transcendental
// instructions exist).  Table-driven (Tang's method): 256-entry tables in
// LDS reduce the argument to a tiny interval where a degree-2 (exp2) or
// degree-3 (log2) polynomial suffices; truncation errors are 4.2e-10
// relative (exp2) and 6e-12 absolute (log2), against the ~3e-8 relative
// accuracy the model values need.  Every kernel that evaluates them fills
// the tables first (init_math_tab).
// ---------------------------------------------------------------------------
constexpr double LN2_D = 0.69314718055994530942;

struct MathTab {
    double2 lg[256];   // (2/c_j, log2(1/c_j) - 1), c_j = 1 + (j + 1/2)/256
    double ex[256];    // 2^(j/256)
};
__shared__ MathTab g_tab;

// The work-group fills the table; ends with a barrier.
__device__ __forceinline__ void init_math_tab() {
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
        const double ic = 1.0 / (1.0 + (j + 0.5) / 256.0);
        g_tab.lg[j] = make_double2(2.0 * ic, -log2(ic) - 1.0);
        g_tab.ex[j] = exp2(j / 256.0);
    }
    __syncthreads();
}

// log2 x for normal x > 0: x = f 2^q, f in [1/2, 1) (frexp), so with
// m = 2 f in [1, 2) and e = q - 1, log2 x = e + log2 c_j + log2(1 + r),
// c_j the table point of m's leading eight fraction bits (those of x),
// r = m/c_j - 1 = f (2/c_j) - 1, |r| < 2^-9, by the series of log(1 + r)
// to r^3 (truncation below 6e-12).  The table folds the -1 of e in.
__device__ __forceinline__ double log2_d(double x) {
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);
    const int j = (int)((hi >> 12) & 255u);
    const double2 t = g_tab.lg[j];
    const double f = __builtin_amdgcn_frexp_mant(x);
    const int q = __builtin_amdgcn_frexp_exp(x);
    const double r = fma(f, t.x, -1.0);
    constexpr double k = 1.0 / LN2_D;
    double p = fma(r, k / 3.0, -k / 2.0);
    p = fma(r, p, k);
    return fma(r, p, (double)q + t.y);
}

// 2^(t/256) for t in [-281600, 281600] (callers bound the argument; they
// pass t = 256 v for 2^v, with the factor 256 folded into their constants,
// which is exact): t = 256 n + i + f, i in [0, 256), |f| <= 1/2;
// 2^(t/256) = 2^n 2^(i/256) e^y, y = f ln2/256, |y| < 0.00136, by
// e^y = 1 + y + y^2/2 (truncation below 4.2e-10 relative).
__device__ __forceinline__ double exp2_256(double t) {
    const double jd = rint(t);
    const int ji = (int)jd;
    const double f = t - jd;
    constexpr double c = LN2_D / 256.0;
    const double p = fma(f, fma(f, c * c / 2.0, c), 1.0);
    return __builtin_amdgcn_ldexp(g_tab.ex[ji & 255] * p, ji >> 8);
}

// ---------------------------------------------------------------------------
// Sersic value and adjoint, given the offset (dx, dy) from the centre
// ---------------------------------------------------------------------------
// Model value I_e exp(-b_n [(R/R_e)^(1/n) - 1]) in float64.
__device__ __forceinline__ double sersic_val(double dx, double dy, const SersicK& s) {
    double r2 = fma(dx, fma(s.a11, dx, s.a12x2 * dy), dy * (s.a22 * dy));
    r2 = fmax(r2, RMIN2D);
    const double u = exp2_256(fma(s.ku, log2_d(r2), s.ku0));   // (R/R_e)^(1/n)
    return s.ie * exp2_256(fmin(fmax(fma(-s.bl, u, s.bl), -281600.0), 281600.0));
}

// Accumulates, for the adjoint gs of this sub-pixel value, the sums that
// the per-particle chain rule needs (see k_finalize), and for a source the
// adjoint of its evaluation point (gbx, gby).
template <bool SRC>
__device__ __forceinline__ void sersic_adj(float dx, float dy, float gs, const SersicK& s, float* a,
                                           float& gbx, float& gby) {
    float r2 = fmaf(s.a11f * dx, dx, fmaf(2.0f * s.a12f * dx, dy, s.a22f * dy * dy));
    const bool cl = r2 < RMIN2;
    r2 = cl ? RMIN2 : r2;
    const float L = flog2(r2);
    const float u = fexp2(fmaf(s.kuf, L, s.ku0f));
    const float E = fexp2(s.blf * (1.0f - u));
    const float gE = gs * E;
    const float wu = gE * s.ief * u;
    const float qp = cl ? 0.0f : wu * frcp(r2);
    const float tx = qp * dx, ty = qp * dy;
    a[AS_E] += gE;
    a[AS_WU] += wu;
    a[AS_WUL] = fmaf(wu, L, a[AS_WUL]);
    a[AS_QX] += tx;
    a[AS_QY] += ty;
    a[AS_QXX] = fmaf(tx, dx, a[AS_QXX]);
    a[AS_QXY] = fmaf(tx, dy, a[AS_QXY]);
    a[AS_QYY] = fmaf(ty, dy, a[AS_QYY]);
    if (SRC) {
        gbx = fmaf(s.kap2, fmaf(s.a11f, tx, s.a12f * ty), gbx);
        gby = fmaf(s.kap2, fmaf(s.a12f, tx, s.a22f * ty), gby);
    }
}

// ---------------------------------------------------------------------------
// Shapelet source (Cartesian basis of Refregier 2003).  With u = dx/beta,
// v = dy/beta the basis function (n1, n2) is (1/beta) psi_n1(u) psi_n2(v),
// psi_n = pi^(-1/4) h_n e^{-u^2/2} (Hermite functions), where h_0 = 1 and
// h_{n+1} = sqrt(2/(n+1)) u h_n - sqrt(n/(n+1)) h_{n-1} (stable recurrence of
// the normalised functions); psi_n' = sqrt(n/2) psi_{n-1} - sqrt((n+1)/2)
// psi_{n+1}.  Coefficients are in the kernels' layout (sh_row).
// ---------------------------------------------------------------------------
__constant__ constexpr double SH_A[SH_CAP + 1] = {1.4142135623730951, 1.0, 0.816496580927726, 0.7071067811865476,
                                                   0.6324555320336759, 0.5773502691896257, 0.5345224838248488, 0.5,
                                                   0.4714045207910317};
__constant__ constexpr double SH_B[SH_CAP + 1] = {0.0, 0.7071067811865476, 0.816496580927726, 0.8660254037844386,
                                                   0.8944271909999159, 0.9128709291752769, 0.9258200997725514,
                                                   0.9354143466934853, 0.9428090415820634};
__constant__ constexpr float SH_D[SH_CAP + 2] = {0.0f, 0.70710678f, 1.0f, 1.22474487f, 1.41421356f,
                                                 1.58113883f, 1.73205081f, 1.87082869f, 2.0f, 2.12132034f};

template <typename T, int N>
__device__ __forceinline__ void hermite_h(T u, T (&h)[N]) {
    h[0] = (T)1;
    if (N > 1) h[1] = (T)SH_A[0] * u;
#pragma unroll
    for (int n = 1; n + 1 < N; ++n) h[n + 1] = (T)SH_A[n] * u * h[n] - (T)SH_B[n] * h[n - 1];
}

// Value of the shapelet source at the source-plane point (bx, by), float64.
__device__ __forceinline__ double shapelet_val(double bx, double by, const float* __restrict__ C) {
    const float* H = C + C_SHAP;
    const double ib = ldd(H, SH_IB);
    const double u = (bx - ldd(H, SH_XC)) * ib, v = (by - ldd(H, SH_YC)) * ib;
    double hu[SH_CAP + 1], hv[SH_CAP + 1];
    hermite_h(u, hu);
    hermite_h(v, hv);
    double F = 0.0;
#pragma unroll
    for (int n2 = 0; n2 <= SH_CAP; ++n2) {
        double t = 0.0;
#pragma unroll
        for (int n1 = 0; n1 <= SH_CAP - n2; ++n1) t = fma(ldd(H, SH_CD + 2 * (sh_row(n2) + n1)), hu[n1], t);
        F = fma(t, hv[n2], F);
    }
    const double E = ldd(H, SH_E0) * exp2_256(fmax(-(u * u + v * v) * (256.0 * 0.7213475204444817), -281600.0));
    return E * F;
}

// Adjoint of the shapelet value for the adjoint gs of the sub-pixel value at
// the source-plane offset (dx, dy) from its centre: accumulates the sums of
// the AH_* layout into a[] and adds the source-plane gradient to (gbx, gby).
__device__ __forceinline__ void shapelet_adj(float dx, float dy, float gs, const float* __restrict__ C, float* a,
                                             float& gbx, float& gby) {
    const float* H = C + C_SHAP;
    const float ib = (float)ldd(H, SH_IB);
    const float u = dx * ib, v = dy * ib;
    float hu[SH_CAP + 2], hv[SH_CAP + 2];
    hermite_h(u, hu);
    hermite_h(v, hv);
    const float W = gs * (float)ldd(H, SH_E0) * fexp2(-(u * u + v * v) * 0.72134752f);
    float F = 0.f, Fu = 0.f, Fv = 0.f;
#pragma unroll
    for (int n2 = 0; n2 <= SH_CAP; ++n2) {
        float th = 0.f, tg = 0.f;
#pragma unroll
        for (int n1 = 0; n1 <= SH_CAP - n2; ++n1) {
            const float c = ldf(H, SH_CF + sh_row(n2) + n1);
            const float g1 = SH_D[n1] * (n1 > 0 ? hu[n1 > 0 ? n1 - 1 : 0] : 0.f) - SH_D[n1 + 1] * hu[n1 + 1];
            th = fmaf(c, hu[n1], th);
            tg = fmaf(c, g1, tg);
        }
        const float g2 = SH_D[n2] * (n2 > 0 ? hv[n2 > 0 ? n2 - 1 : 0] : 0.f) - SH_D[n2 + 1] * hv[n2 + 1];
        F = fmaf(th, hv[n2], F);
        Fu = fmaf(tg, hv[n2], Fu);
        Fv = fmaf(th, g2, Fv);
        const float wv = W * hv[n2];
#pragma unroll
        for (int n1 = 0; n1 <= SH_CAP - n2; ++n1) a[AH_C + sh_row(n2) + n1] = fmaf(wv, hu[n1], a[AH_C + sh_row(n2) + n1]);
    }
    a[AH_U] = fmaf(W, Fu, a[AH_U]);
    a[AH_V] = fmaf(W, Fv, a[AH_V]);
    a[AH_B] = fmaf(W, fmaf(u, Fu, fmaf(v, Fv, F)), a[AH_B]);
    gbx = fmaf(W * Fu, ib, gbx);
    gby = fmaf(W * Fv, ib, gby);
}

// ---------------------------------------------------------------------------
// EPL series S(z) = sum a_n z^n with real coefficients at complex z.
//
// With r = 2 Re z and s = |z|^2, z is a root of w^2 - r w + s, so dividing
// the polynomial by that real quadratic leaves the remainder A z + B:
//   b_k = a_k + r b_{k+1} - s b_{k+2}  (k = K .. 1),  S = a_0 + z b_1 - s b_2.
// Two real FMAs per term instead of the four of a complex Horner step (the
// second-order recurrence of Goertzel's algorithm; Knuth, TAOCP vol. 2,
// Sec. 4.6.4).  Its rounding error grows like 1/(1 - |z|)^2 near the real
// axis: negligible in float64 for every |z| < 1, but above |z| ~ 0.55 worse
// than Horner in float32, so the float32 adjoint series switch to Horner
// there (|z| = c, uniform over a particle, so the branch does not diverge).
// S in float64 (it sets the deflection); S'(z) and dS/dt in float32 (adjoint
// only), each from its own coefficient array.  Coefficients are read with
// wave-uniform (scalar) loads, four per step; the arrays hold a_0 .. a_kp
// with kp + 1 a multiple of 4.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void series_d(const float* __restrict__ C, int kp, double zx, double zy,
                                         double& sx, double& sy) {
    cdouble_t* cS = (cdouble_t*)(C + C_COEF_S);
    const double r = 2.0 * zx, s = fma(zx, zx, zy * zy);
    double b1 = 0.0, b2 = 0.0;
    int base = kp - 3;
    for (; base >= 4; base -= 4) {
        const double a_[4] = {cS[base + 3], cS[base + 2], cS[base + 1], cS[base]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double b = fma(r, b1, fma(-s, b2, a_[q]));
            b2 = b1;
            b1 = b;
        }
    }
    const double a_[3] = {cS[3], cS[2], cS[1]};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double b = fma(r, b1, fma(-s, b2, a_[q]));
        b2 = b1;
        b1 = b;
    }
    sx = fma(zx, b1, fma(-s, b2, cS[0]));
    sy = zy * b1;
}

// float32 S'(z) -> (dx, dy) and, with WT, dS/dt -> (tx, ty).
template <bool WT>
__device__ __forceinline__ void series_adj_horner(const float* __restrict__ C, int kp, float zx, float zy,
                                                  float& dx, float& dy, float& tx, float& ty) {
    cfloat_t* cZ = (cfloat_t*)(C + C_COEF_Z);
    cfloat_t* cT = (cfloat_t*)(C + C_COEF_T);
    dx = 0.f; dy = 0.f; tx = 0.f; ty = 0.f;
    for (int base = kp - 3; base >= 0; base -= 4) {
        const float cz_[4] = {cZ[base + 3], cZ[base + 2], cZ[base + 1], cZ[base]};
        float ct_[4] = {0.f, 0.f, 0.f, 0.f};
        if (WT) {
            ct_[0] = cT[base + 3]; ct_[1] = cT[base + 2]; ct_[2] = cT[base + 1]; ct_[3] = cT[base];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float ndx = fmaf(dx, zx, fmaf(-dy, zy, cz_[q]));
            const float ndy = fmaf(dx, zy, dy * zx);
            dx = ndx; dy = ndy;
            if (WT) {
                const float ntx = fmaf(tx, zx, fmaf(-ty, zy, ct_[q]));
                const float nty = fmaf(tx, zy, ty * zx);
                tx = ntx; ty = nty;
            }
        }
    }
}

template <bool WT>
__device__ __forceinline__ void series_adj_quad(const float* __restrict__ C, int kp, float zx, float zy,
                                                float& dx, float& dy, float& tx, float& ty) {
    cfloat_t* cZ = (cfloat_t*)(C + C_COEF_Z);
    cfloat_t* cT = (cfloat_t*)(C + C_COEF_T);
    const float r = 2.0f * zx, s = fmaf(zx, zx, zy * zy);
    float d1 = 0.f, d2 = 0.f, t1 = 0.f, t2 = 0.f;
    int base = kp - 3;
    for (; base >= 4; base -= 4) {
        const float cz_[4] = {cZ[base + 3], cZ[base + 2], cZ[base + 1], cZ[base]};
        float ct_[4] = {0.f, 0.f, 0.f, 0.f};
        if (WT) {
            ct_[0] = cT[base + 3]; ct_[1] = cT[base + 2]; ct_[2] = cT[base + 1]; ct_[3] = cT[base];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float b = fmaf(r, d1, fmaf(-s, d2, cz_[q]));
            d2 = d1;
            d1 = b;
            if (WT) {
                const float bt = fmaf(r, t1, fmaf(-s, t2, ct_[q]));
                t2 = t1;
                t1 = bt;
            }
        }
    }
    const float cz_[3] = {cZ[3], cZ[2], cZ[1]};
    float ct_[3] = {0.f, 0.f, 0.f};
    if (WT) {
        ct_[0] = cT[3]; ct_[1] = cT[2]; ct_[2] = cT[1];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float b = fmaf(r, d1, fmaf(-s, d2, cz_[q]));
        d2 = d1;
        d1 = b;
        if (WT) {
            const float bt = fmaf(r, t1, fmaf(-s, t2, ct_[q]));
            t2 = t1;
            t1 = bt;
        }
    }
    dx = fmaf(zx, d1, fmaf(-s, d2, cZ[0]));
    dy = zy * d1;
    tx = 0.f; ty = 0.f;
    if (WT) {
        tx = fmaf(zx, t1, fmaf(-s, t2, cT[0]));
        ty = zy * t1;
    }
}

template <bool WT>
__device__ __forceinline__ void series_adj(const float* __restrict__ C, int kp, bool quad, float zx, float zy,
                                           float& dx, float& dy, float& tx, float& ty) {
    if (quad) series_adj_quad<WT>(C, kp, zx, zy, dx, dy, tx, ty);
    else series_adj_horner<WT>(C, kp, zx, zy, dx, dy, tx, ty);
}

// 1/sqrt(x) in float64: hardware estimate (relative error below 5.3e-8,
// measured over 1e-12..1e8) + one Newton step (error below 4e-15).
__device__ __forceinline__ double rsqrt_d(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// Intermediates of the deflection kept (as float32) for the adjoint.
struct MassState {
    float wx, wy, ux, uy, vx, vy, ir, A, B, zx, zy, sx, sy, f, L2, ax, ay;
    bool inside;
};

// Mass deflection in float64; with KEEP the float32 intermediates are saved.
template <int MASS, bool KEEP, int NC>
__device__ __forceinline__ void deflect(double x, double y, const PK<NC>& k,
                                        const float* __restrict__ C, double& ax, double& ay,
                                        MassState* ms) {
    const double wx = x - k.x0, wy = y - k.y0;
    const double ux = fma(k.ua, wx, -k.ue * wy);
    const double uy = fma(k.ub, wy, -k.ue * wx);
    double r2 = fma(ux, ux, uy * uy);
    const bool inside = r2 < RMIN2D;
    r2 = inside ? RMIN2D : r2;
    const double ir = rsqrt_d(r2);
    const double vx = ux * ir, vy = uy * ir;
    const double A = fma(vx, vx, -vy * vy), B = 2.0 * vx * vy;
    const double zx = -fma(k.e1, A, k.e2 * B);
    const double zy = -fma(k.e1, B, -k.e2 * A);
    double sx, sy;
    series_d(C, k.kp, zx, zy, sx, sy);
    double f = k.c0, L2 = 0.0;
    if (MASS == LENS_MASS_EPL) {
        L2 = log2_d(r2);
        f *= exp2_256(fma(-k.k1, L2, k.k0));
    }
    ax = inside ? 0.0 : f * fma(vx, sx, -vy * sy);
    ay = inside ? 0.0 : f * fma(vx, sy, vy * sx);
    if (KEEP) {
        ms->wx = (float)wx; ms->wy = (float)wy; ms->ux = (float)ux; ms->uy = (float)uy;
        ms->vx = (float)vx; ms->vy = (float)vy; ms->ir = (float)ir;
        ms->A = (float)A; ms->B = (float)B; ms->zx = (float)zx; ms->zy = (float)zy;
        ms->sx = (float)sx; ms->sy = (float)sy; ms->f = (float)f; ms->L2 = (float)L2;
        ms->ax = (float)ax; ms->ay = (float)ay; ms->inside = inside;
    }
}

// series_d at N points of one particle at once: each point's operations
// are those of series_d, in the same order; the coefficients are loaded once.
template <int N>
__device__ __forceinline__ void series_d_n(const float* __restrict__ C, int kp, const double (&zx)[N],
                                           const double (&zy)[N], double (&sx)[N], double (&sy)[N]) {
    cdouble_t* cS = (cdouble_t*)(C + C_COEF_S);
    double r[N], s[N], b1[N], b2[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        r[n] = 2.0 * zx[n];
        s[n] = fma(zx[n], zx[n], zy[n] * zy[n]);
        b1[n] = 0.0;
        b2[n] = 0.0;
    }
    int base = kp - 3;
    for (; base >= 4; base -= 4) {
        const double a_[4] = {cS[base + 3], cS[base + 2], cS[base + 1], cS[base]};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int n = 0; n < N; ++n) {
                const double b = fma(r[n], b1[n], fma(-s[n], b2[n], a_[q]));
                b2[n] = b1[n];
                b1[n] = b;
            }
    }
    const double a_[3] = {cS[3], cS[2], cS[1]};
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const double b = fma(r[n], b1[n], fma(-s[n], b2[n], a_[q]));
            b2[n] = b1[n];
            b1[n] = b;
        }
    const double c0 = cS[0];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        sx[n] = fma(zx[n], b1[n], fma(-s[n], b2[n], c0));
        sy[n] = zy[n] * b1[n];
    }
}

// Mass deflection (float64) at N points of one particle: per point the
// operations of deflect, in the same order.
template <int MASS, int N>
__device__ __forceinline__ void deflect_n(const double (&x)[N], const double (&y)[N], const PK<0>& k,
                                          const float* __restrict__ C, double (&ax)[N], double (&ay)[N]) {
    double r2[N], vx[N], vy[N], zx[N], zy[N];
    bool inside[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        const double wx = x[n] - k.x0, wy = y[n] - k.y0;
        const double ux = fma(k.ua, wx, -k.ue * wy);
        const double uy = fma(k.ub, wy, -k.ue * wx);
        double q = fma(ux, ux, uy * uy);
        inside[n] = q < RMIN2D;
        q = inside[n] ? RMIN2D : q;
        r2[n] = q;
        const double ir = rsqrt_d(q);
        vx[n] = ux * ir;
        vy[n] = uy * ir;
        const double A = fma(vx[n], vx[n], -vy[n] * vy[n]), B = 2.0 * vx[n] * vy[n];
        zx[n] = -fma(k.e1, A, k.e2 * B);
        zy[n] = -fma(k.e1, B, -k.e2 * A);
    }
    double sx[N], sy[N];
    series_d_n<N>(C, k.kp, zx, zy, sx, sy);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double f = k.c0;
        if (MASS == LENS_MASS_EPL) f *= exp2_256(fma(-k.k1, log2_d(r2[n]), k.k0));
        ax[n] = inside[n] ? 0.0 : f * fma(vx[n], sx[n], -vy[n] * sy[n]);
        ay[n] = inside[n] ? 0.0 : f * fma(vx[n], sy[n], vy[n] * sx[n]);
    }
}

// Model values at N sub-pixels of one particle, each component's float64
// constants loaded right before the component is evaluated (the ~40
// float64 constants of a particle do not fit the scalar register file
// together) and shared by the N points.  Per point the sum runs over the
// lens lights, then the sources, then the shapelet source, as always.
template <int MASS, int NL, int NS, int SH, int N>
__device__ __forceinline__ void subpix_value_n(const double (&x)[N], const double (&y)[N],
                                               const float* __restrict__ C, double (&v)[N]) {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = 0.0;
#pragma unroll
    for (int c = 0; c < NL; ++c) {
        const SersicK s = load_sersic(opaque(C + C_SERS + c * SERS_STRIDE));
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += sersic_val(x[n] - s.xc, y[n] - s.yc, s);
    }
    const float* Cm = opaque(C);
    const PK<0> k = load_pk<0>(Cm);
    double ax[N], ay[N], bx[N], by[N];
    deflect_n<MASS, N>(x, y, k, Cm, ax, ay);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        bx[n] = x[n] - ax[n] - fma(k.g1, x[n], k.g2 * y[n]);
        by[n] = y[n] - ay[n] - fma(k.g2, x[n], -k.g1 * y[n]);
    }
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        const SersicK s = load_sersic(opaque(C + C_SERS + (NL + c) * SERS_STRIDE));
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += sersic_val(bx[n] - s.xc, by[n] - s.yc, s);
    }
    if (SH) {
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += shapelet_val(bx[n], by[n], opaque(C));
    }
}

// Reverse sweep of one sub-pixel: accumulates into acc[] (layout A_*).
template <int MASS, int NL, int NS, int SH>
__device__ __forceinline__ void subpix_adjoint(double x, double y, float gs, const PK<NL + NS>& k,
                                               const float* __restrict__ C, float* acc) {
    float dummy0 = 0.f, dummy1 = 0.f;
#pragma unroll
    for (int c = 0; c < NL; ++c)
        sersic_adj<false>((float)(x - k.s[c].xc), (float)(y - k.s[c].yc), gs, k.s[c],
                          acc + A_SERS + A_SERS_STRIDE * c, dummy0, dummy1);

    MassState m;
    double axd, ayd;
    deflect<MASS, true, NL + NS>(x, y, k, C, axd, ayd, &m);
    const double bx = x - axd - fma(k.g1, x, k.g2 * y);
    const double by = y - ayd - fma(k.g2, x, -k.g1 * y);

    // sources at beta, collecting the adjoint of beta
    float gbx = 0.f, gby = 0.f;
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        const SersicK& sc = k.s[NL + c];
        sersic_adj<true>((float)(bx - sc.xc), (float)(by - sc.yc), gs, sc,
                         acc + A_SERS + A_SERS_STRIDE * (NL + c), gbx, gby);
    }
    if (SH)
        shapelet_adj((float)(bx - ldd(C + C_SHAP, SH_XC)), (float)(by - ldd(C + C_SHAP, SH_YC)), gs, C,
                     acc + A_SERS + A_SERS_STRIDE * (NL + NS), gbx, gby);

    // G = dL/dalpha = -dL/dbeta (mass and shear deflections enter beta alike)
    const float xf = (float)x, yf = (float)y;
    float Gx = -gbx, Gy = -gby;
    acc[A_SH] = fmaf(Gx, xf, fmaf(-Gy, yf, acc[A_SH]));        // Re(G theta)
    acc[A_SH + 1] = fmaf(Gx, yf, fmaf(Gy, xf, acc[A_SH + 1]));  // Im(G theta)
    if (m.inside) { Gx = 0.f; Gy = 0.f; }

    float dx, dy, tx, ty;
    series_adj<MASS == LENS_MASS_EPL>(C, k.kpa, k.quad, m.zx, m.zy, dx, dy, tx, ty);
    const float vx = m.vx, vy = m.vy, sx = m.sx, sy = m.sy;
    const float h = fmaf(Gx, m.ax, Gy * m.ay);                // Re(conj(G) alpha)
    acc[A_H] += h;
    const float vbx = Gx * m.f, vby = Gy * m.f;               // adjoint of V = V0 S
    if (MASS == LENS_MASS_EPL) {
        const float vtx = fmaf(vx, tx, -vy * ty), vty = fmaf(vx, ty, vy * tx);   // V0 dS/dt
        acc[A_T] += fmaf(vbx, vtx, fmaf(vby, vty, -h * (HALF_LN2 * m.L2)));
    }
    // Zb = Vb conj(V0 S'(z))
    const float vdx = fmaf(vx, dx, -vy * dy), vdy = fmaf(vx, dy, vy * dx);
    const float zbx = fmaf(vbx, vdx, vby * vdy);
    const float zby = fmaf(vby, vdx, -vbx * vdy);
    acc[A_ZE] = fmaf(zbx, m.A, fmaf(zby, m.B, acc[A_ZE]));            // Zb conj(V0)^2
    acc[A_ZE + 1] = fmaf(zby, m.A, fmaf(-zbx, m.B, acc[A_ZE + 1]));
    // adjoint of V0: Vb conj(S) - 2 Zb eps conj(V0)
    const float px = fmaf(k.e1f, vx, k.e2f * vy), py = fmaf(k.e2f, vx, -k.e1f * vy);
    const float gvx = fmaf(vbx, sx, vby * sy) - 2.0f * fmaf(zbx, px, -zby * py);
    const float gvy = fmaf(vby, sx, -vbx * sy) - 2.0f * fmaf(zbx, py, zby * px);
    // adjoint of U through V0 = U/|U| and ln R (slope factor)
    const float rho = (MASS == LENS_MASS_EPL) ? -2.0f * k.k1f * h : 0.0f;
    const float sv = fmaf(gvx, vx, gvy * vy) - rho;
    const float gux = fmaf(-vx, sv, gvx) * m.ir;
    const float guy = fmaf(-vy, sv, gvy) * m.ir;
    acc[A_UB] += gux;
    acc[A_UB + 1] += guy;
    acc[A_UW] = fmaf(gux, m.wx, fmaf(-guy, m.wy, acc[A_UW]));          // conj(GU) conj(w)
    acc[A_UW + 1] = fmaf(-gux, m.wy, fmaf(-guy, m.wx, acc[A_UW + 1]));
    acc[A_UC] = fmaf(gux, m.ux, fmaf(guy, m.uy, acc[A_UC]));            // Re(conj(GU) U)
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a work-group of NT threads (fixed order).  red: >= NT/64 doubles of LDS.
template <int NT = 256>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_prologue(ModelInfo mi, int P, const float* __restrict__ theta,
                           float* __restrict__ consts) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float* th = theta + (size_t)p * mi.d;
    float* C = consts + (size_t)p * CSTRIDE;
    bool finite = true;
    for (int k = 0; k < mi.d; ++k) finite = finite && isfinite(th[k]);
    const bool epl = mi.mass_model == LENS_MASS_EPL;
    int o = 0;
    const double tE = th[o++];
    const double gam = epl ? (double)th[o++] : 2.0;
    const double e1 = th[o], e2 = th[o + 1];
    const double x0 = th[o + 2], y0 = th[o + 3], g1 = th[o + 4], g2 = th[o + 5];
    o += 6;
    const double c2 = e1 * e1 + e2 * e2, c = sqrt(c2);
    const double t = gam - 1.0;
    bool ok = c < 1.0 && tE > 0.0 && t > 0.0 && t < 2.0;
    const double ip = 1.0 / (1.0 + c);
    double* Dm = reinterpret_cast<double*>(C);
    Dm[D_X0 / 2] = x0; Dm[D_Y0 / 2] = y0; Dm[D_E1 / 2] = e1; Dm[D_E2 / 2] = e2;
    Dm[D_UA / 2] = (1.0 - e1) * ip;
    Dm[D_UB / 2] = (1.0 + e1) * ip;
    Dm[D_UE / 2] = e2 * ip;
    Dm[D_C0 / 2] = tE * sqrt(fmax(1.0 - c2, 0.0));
    const double b = tE * sqrt(fmax((1.0 - c) / (1.0 + c), 0.0));
    Dm[D_K0 / 2] = 256.0 * ((t - 1.0) * log2(b));   // both times 256 (exp2_256)
    Dm[D_K1 / 2] = 256.0 * (0.5 * (t - 1.0));
    Dm[D_G1 / 2] = g1; Dm[D_G2 / 2] = g2;
    const int nc = mi.n_lens_light + mi.n_source;
    for (int k = 0; k < nc; ++k, o += 7) {
        const double Re = th[o], n = th[o + 1], se1 = th[o + 2], se2 = th[o + 3];
        const double cs2 = se1 * se1 + se2 * se2;
        ok = ok && cs2 < 1.0 && Re > 0.0 && n > 0.0;
        const double D = 1.0 - cs2;
        float* S = C + C_SERS + k * SERS_STRIDE;
        double* Sd = reinterpret_cast<double*>(S);
        Sd[S_XC / 2] = th[o + 4]; Sd[S_YC / 2] = th[o + 5];
        Sd[S_A11 / 2] = (1.0 + cs2 - 2.0 * se1) / D;
        Sd[S_A22 / 2] = (1.0 + cs2 + 2.0 * se1) / D;
        Sd[S_A12 / 2] = -2.0 * se2 / D;
        Sd[S_A12X2 / 2] = -4.0 * se2 / D;
        Sd[S_IE / 2] = th[o + 6];
        const double bn = 1.9992 * n - 0.3271;
        Sd[S_KU / 2] = 256.0 * (0.5 / n);              // exponent constants times 256 (exp2_256)
        Sd[S_KU0 / 2] = 256.0 * (-log2(Re) / n);
        Sd[S_BL / 2] = 256.0 * (bn * 1.4426950408889634);
        S[S_KAP2] = (float)(-bn / n);
    }
    if (mi.n_shapelet) {
        // shapelet source: scale, centre, coefficients re-ordered into rows of n2
        const double beta = th[o];
        ok = ok && beta > 0.0;
        float* H = C + C_SHAP;
        double* Hd = reinterpret_cast<double*>(H);
        const double ib = 1.0 / beta;
        Hd[SH_XC / 2] = th[o + 1];
        Hd[SH_YC / 2] = th[o + 2];
        Hd[SH_IB / 2] = ib;
        Hd[SH_E0 / 2] = 0.56418958354775628695 * ib;   // pi^(-1/2) / beta
        for (int q = 0; q < SH_NB; ++q) {
            Hd[SH_CD / 2 + q] = 0.0;
            H[SH_CF + q] = 0.0f;
        }
        int k = 0;
        for (int n = 0; n <= mi.sh_nmax; ++n)
            for (int n2 = 0; n2 <= n; ++n2, ++k) {
                const int q = sh_row(n2) + (n - n2);
                Hd[SH_CD / 2 + q] = th[o + 3 + k];
                H[SH_CF + q] = th[o + 3 + k];
            }
    }
    // Series coefficients c_n(t), (n+1) c_{n+1} for S'(z), and dc_n/dt = c_n D_n,
    // D_n = sum_{k<=n} [1/(2k-2+t) + 1/(2k+2-t)], |z| = c, c_n decreasing.
    // Truncation after z^K leaves at most c_{K+1} c^{K+1}/(1-c) in S (kept
    // below 2^-31: the deflection must be good to ~3e-9 relative), and at
    // most (K+1) c_{K+1} c^K/(1-c)^2 in S' and c_{K+1}(D_{K+1}+1) c^{K+1}/(1-c)^2
    // in dS/dt (below 2^-25: float32 adjoint).
    double* cS = reinterpret_cast<double*>(C + C_COEF_S);
    float* cZ = C + C_COEF_Z;
    float* cT = C + C_COEF_T;
    cS[0] = 1.0; cT[0] = 0.0f;
    int K = -1, KA = -1;
    if (ok) {
        double cn = 1.0, Dn = 0.0, cpow = 1.0;   // c_n, D_n, c^n
        const double om = 1.0 - c;
        for (int n = 0; n < KMAX_TERMS; ++n) {
            const double a = 2.0 * (n + 1) - 2.0 + t, bb = 2.0 * (n + 1) + 2.0 - t;
            const double cn1 = cn * a / bb, Dn1 = Dn + 1.0 / a + 1.0 / bb;
            cS[n + 1] = cn1;
            cZ[n] = (float)((n + 1) * cn1);
            cT[n + 1] = (float)(cn1 * Dn1);
            const double tail_s = cn1 * cpow * c / om;
            const double tail_a = fmax((n + 1) * cn1 * cpow, cn1 * (Dn1 + 1.0) * cpow * c) / (om * om);
            if (KA < 0 && tail_a < 2.9802322387695312e-08) KA = n;
            if (K < 0 && tail_s < 4.656612873077393e-10) K = n;
            if (K >= 0 && KA >= 0) break;
            cn = cn1; Dn = Dn1; cpow *= c;
        }
        if (K < 0) K = KMAX_TERMS - 1;
        if (KA < 0) KA = KMAX_TERMS - 1;
        // S' keeps one term more than the S' bound asks, so that S'(0) = c_1 always
        KA = KA < 1 ? 1 : KA;
    } else {
        K = 0; KA = 1;
    }
    const int KP = ((K + 1 + 3) / 4) * 4 - 1;     // S: c_0..c_K
    const int KPA = ((KA + 1 + 3) / 4) * 4 - 1;   // adjoint: S' terms 0..KA-1, dS/dt terms 0..KA
    for (int n = K + 1; n <= KP; ++n) cS[n] = 0.0;
    for (int n = KA + 1; n <= KPA; ++n) cT[n] = 0.0f;
    for (int n = KA; n <= KPA; ++n) cZ[n] = 0.0f;
    C[C_KP] = (float)KP;
    C[C_KPA] = (float)KPA;
    C[C_VALID] = !finite ? 2.0f : (ok ? 1.0f : 0.0f);
}

// Sub-pixel sum of N pixels of one particle (N = 1 or 2), each at its own
// (i, j); the pixels' sub-pixels are visited in the same order.
template <int MASS, int NL, int NS, int SH, int N>
__device__ __forceinline__ void pixel_values(const float* __restrict__ C, const Geo& g, const int (&pix)[N],
                                             double (&acc)[N]) {
    int i[N], j[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        i[n] = pix[n] / g.nx;
        j[n] = pix[n] - i[n] * g.nx;
        acc[n] = 0.0;
    }
    for (int a = 0; a < g.s; ++a) {
        double y[N];
#pragma unroll
        for (int n = 0; n < N; ++n) y[n] = ((double)(g.s * i[n] + a) - g.cy) * g.h;
        for (int b = 0; b < g.s; ++b) {
            double x[N], v[N];
#pragma unroll
            for (int n = 0; n < N; ++n) x[n] = ((double)(g.s * j[n] + b) - g.cx) * g.h;
            subpix_value_n<MASS, NL, NS, SH, N>(x, y, C, v);
#pragma unroll
            for (int n = 0; n < N; ++n) acc[n] += v[n];
        }
    }
}

// Renders pixels [pix0, pix1) of one particle (whole work-group).  Each
// thread takes its pixels two at a time (pix and pix + blockDim.x), so that
// constants and series coefficients are loaded once for both; a last odd
// pixel is rendered alone, with the same operations.
template <int MASS, int NL, int NS, int SH>
__device__ __forceinline__ void render_chunk(const float* __restrict__ C, const Geo& g, int pix0,
                                             int pix1, float* __restrict__ out) {
    if (C[C_VALID] != 1.0f) {
        for (int pix = pix0 + threadIdx.x; pix < pix1; pix += blockDim.x) out[pix] = __builtin_nanf("");
        return;
    }
    const int step = blockDim.x;
    int pix = pix0 + threadIdx.x;
    for (; pix + step < pix1; pix += 2 * step) {
        const int pp[2] = {pix, pix + step};
        double acc[2];
        pixel_values<MASS, NL, NS, SH, 2>(C, g, pp, acc);
        out[pix] = (float)(acc[0] * (double)g.inv_s2);
        out[pix + step] = (float)(acc[1] * (double)g.inv_s2);
    }
    if (pix < pix1) {
        const int pp[1] = {pix};
        double acc[1];
        pixel_values<MASS, NL, NS, SH, 1>(C, g, pp, acc);
        out[pix] = (float)(acc[0] * (double)g.inv_s2);
    }
}

// Reverse sweep over pixels [pix0, pix1) of one particle; writes the
// work-group's NACC float64 sums to outp.  red: LDS [NACC][4] doubles.
// Ends with a barrier, so red can be reused by the caller.
template <int MASS, int NL, int NS, int SH>
__device__ __forceinline__ void adjoint_chunk(const float* __restrict__ C, const Geo& g, int pix0,
                                              int pix1, const float* __restrict__ gp,
                                              double* __restrict__ outp, double (*red)[4]) {
    constexpr int NACC = A_SERS + A_SERS_STRIDE * (NL + NS) + SH * AH_SIZE;
    if (C[C_VALID] != 1.0f) {
        if (threadIdx.x < NACC) outp[threadIdx.x] = 0.0;
        return;
    }
    const PK<NL + NS> k = load_pk<NL + NS>(C);
    float acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = 0.f;
    for (int pix = pix0 + threadIdx.x; pix < pix1; pix += blockDim.x) {
        const int i = pix / g.nx, j = pix - i * g.nx;
        const float gs = gp[pix] * g.inv_s2;
        for (int a = 0; a < g.s; ++a) {
            const double y = ((double)(g.s * i + a) - g.cy) * g.h;
            for (int b = 0; b < g.s; ++b) {
                const double x = ((double)(g.s * j + b) - g.cx) * g.h;
                subpix_adjoint<MASS, NL, NS, SH>(x, y, gs, k, C, acc);
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
        const double v = wave_sum((double)acc[q]);
        if (lane == 0) red[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        const int q = threadIdx.x;
        outp[q] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
    }
    __syncthreads();
}

template <int MASS, int NL, int NS, int SH>
__global__ __launch_bounds__(256) void k_render(const float* __restrict__ consts, Geo g, int ppb,
                                                float* __restrict__ img) {
    init_math_tab();
    const int p = blockIdx.x;
    const int pix0 = blockIdx.y * ppb;
    render_chunk<MASS, NL, NS, SH>(consts + (size_t)p * CSTRIDE, g, pix0, min(pix0 + ppb, g.npix),
                                   img + (size_t)p * g.npix);
}

// Backward modelling: the image of each light component at the intensity in
// its constants (the unit-intensity images when every intensity is 1), in
// one pass, so the deflection is evaluated once per sub-pixel.
// img [(p K + c)][npix], K = NL + NS + nb: lens-light components first, then
// the Sersic sources, then the nb shapelet basis functions (coefficient order
// of the parameter vector) at their coefficients.
template <int MASS, int NL, int NS, int SH>
__global__ __launch_bounds__(256) void k_render_split(const float* __restrict__ consts, Geo g, int ppb, int sh_nmax,
                                                      float* __restrict__ img) {
    constexpr int NC = NL + NS;
    constexpr int NSH = SH ? SH_NB : 0;
    init_math_tab();
    const int p = blockIdx.x;
    const int pix0 = blockIdx.y * ppb, pix1 = min(pix0 + ppb, g.npix);
    const int nb = SH ? (sh_nmax + 1) * (sh_nmax + 2) / 2 : 0;
    const int K = NC + nb;
    const float* C = consts + (size_t)p * CSTRIDE;
    float* out = img + (size_t)p * K * g.npix;
    if (C[C_VALID] != 1.0f) {
        for (int pix = pix0 + threadIdx.x; pix < pix1; pix += blockDim.x)
            for (int c = 0; c < K; ++c) out[(size_t)c * g.npix + pix] = __builtin_nanf("");
        return;
    }
    for (int pix = pix0 + threadIdx.x; pix < pix1; pix += blockDim.x) {
        const int i = pix / g.nx, j = pix - i * g.nx;
        double acc[NC + NSH];
#pragma unroll
        for (int c = 0; c < NC + NSH; ++c) acc[c] = 0.0;
        for (int a = 0; a < g.s; ++a) {
            const double y = ((double)(g.s * i + a) - g.cy) * g.h;
            for (int b = 0; b < g.s; ++b) {
                const double x = ((double)(g.s * j + b) - g.cx) * g.h;
#pragma unroll
                for (int c = 0; c < NL; ++c) {
                    const SersicK sk = load_sersic(opaque(C + C_SERS + c * SERS_STRIDE));
                    acc[c] += sersic_val(x - sk.xc, y - sk.yc, sk);
                }
                const float* Cm = opaque(C);
                const PK<0> k = load_pk<0>(Cm);
                double ax, ay;
                deflect<MASS, false, 0>(x, y, k, Cm, ax, ay, nullptr);
                const double bx = x - ax - fma(k.g1, x, k.g2 * y);
                const double by = y - ay - fma(k.g2, x, -k.g1 * y);
#pragma unroll
                for (int c = 0; c < NS; ++c) {
                    const SersicK sk = load_sersic(opaque(C + C_SERS + (NL + c) * SERS_STRIDE));
                    acc[NL + c] += sersic_val(bx - sk.xc, by - sk.yc, sk);
                }
                if (SH) {
                    // each basis function at its coefficient (kernels' layout)
                    const float* H = opaque(C) + C_SHAP;
                    const double ib = ldd(H, SH_IB);
                    const double u = (bx - ldd(H, SH_XC)) * ib, v = (by - ldd(H, SH_YC)) * ib;
                    double hu[SH_CAP + 1], hv[SH_CAP + 1];
                    hermite_h(u, hu);
                    hermite_h(v, hv);
                    const double E = ldd(H, SH_E0) * exp2_256(fmax(-(u * u + v * v) * (256.0 * 0.7213475204444817), -281600.0));
#pragma unroll
                    for (int n2 = 0; n2 <= SH_CAP; ++n2) {
                        const double ev = E * hv[n2];
#pragma unroll
                        for (int n1 = 0; n1 <= SH_CAP - n2; ++n1) {
                            const int q = sh_row(n2) + n1;
                            acc[NC + q] = fma(ev * ldd(H, SH_CD + 2 * q), hu[n1], acc[NC + q]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) out[(size_t)c * g.npix + pix] = (float)(acc[c] * (double)g.inv_s2);
        if (SH) {
            // basis (n1, n2) is coefficient n (n + 1)/2 + n2 of the parameter vector, n = n1 + n2
#pragma unroll
            for (int n2 = 0; n2 <= SH_CAP; ++n2)
#pragma unroll
                for (int n1 = 0; n1 <= SH_CAP - n2; ++n1) {
                    const int n = n1 + n2;
                    if (n <= sh_nmax)
                        out[(size_t)(NC + n * (n + 1) / 2 + n2) * g.npix + pix] =
                            (float)(acc[NC + sh_row(n2) + n1] * (double)g.inv_s2);
                }
        }
    }
}

// Four waves per SIMD (at most 128 VGPRs): measured faster than the three the
// register demand would otherwise give, with the few spills left outside the
// sub-pixel loops.
template <int MASS, int NL, int NS, int SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_adjoint(
    const float* __restrict__ consts, Geo g, int ppb, const float* __restrict__ gimg, double* __restrict__ partial) {
    constexpr int NACC = A_SERS + A_SERS_STRIDE * (NL + NS) + SH * AH_SIZE;
    __shared__ double red[NACC][4];
    init_math_tab();
    const int p = blockIdx.x;
    const int pix0 = blockIdx.y * ppb;
    adjoint_chunk<MASS, NL, NS, SH>(consts + (size_t)p * CSTRIDE, g, pix0, min(pix0 + ppb, g.npix),
                                    gimg + (size_t)p * g.npix,
                                    partial + ((size_t)p * gridDim.y + blockIdx.y) * NACC, red);
}

// With a shapelet source (48 more accumulators): the same pass with no cap on
// the registers.
template <int MASS, int NL, int NS, int SH>
__global__ __launch_bounds__(256) void k_adjoint_sh(const float* __restrict__ consts, Geo g, int ppb,
                                                    const float* __restrict__ gimg, double* __restrict__ partial) {
    constexpr int NACC = A_SERS + A_SERS_STRIDE * (NL + NS) + SH * AH_SIZE;
    __shared__ double red[NACC][4];
    init_math_tab();
    const int p = blockIdx.x;
    const int pix0 = blockIdx.y * ppb;
    adjoint_chunk<MASS, NL, NS, SH>(consts + (size_t)p * CSTRIDE, g, pix0, min(pix0 + ppb, g.npix),
                                    gimg + (size_t)p * g.npix,
                                    partial + ((size_t)p * gridDim.y + blockIdx.y) * NACC, red);
}

// Register-blocked correlation of an LDS tile with a K x K kernel:
// m[r] = sum_{u,v} w[u][v] tile[i+u][j0+v+r]; accumulator type T (float64 for
// the model convolution, float32 for the adjoint).
// Global-memory load through a pointer the compiler cannot place (one read
// from a descriptor in memory would otherwise be a flat load).
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

template <int K, int RW, typename T>
__device__ __forceinline__ void correlate(const float* lds, int stride, int i, int j0,
                                          const T* __restrict__ w, T (&m)[RW]) {
    constexpr int NQ = (RW + K - 1 + 3) / 4;
#pragma unroll
    for (int r = 0; r < RW; ++r) m[r] = (T)0;
    // rows stay a loop: unrolled (small K) the compiler would hoist all K^2
    // taps into registers for the whole strip loop
#pragma unroll 1
    for (int u = 0; u < K; ++u) {
        const float4* row = reinterpret_cast<const float4*>(lds + (i + u) * stride + j0);
        T seg[4 * NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float4 t4 = row[q];
            seg[4 * q] = (T)t4.x; seg[4 * q + 1] = (T)t4.y; seg[4 * q + 2] = (T)t4.z;
            seg[4 * q + 3] = (T)t4.w;
        }
        const T* wr = w + u * K;
#pragma unroll
        for (int v = 0; v < K; ++v) {
            // PSF weights: wave-uniform, read-only during the kernel, read as
            // constant memory so that they are scalar loads also where the
            // pointer comes from a descriptor in memory (batch plans)
            const T wv = *(const __attribute__((address_space(4))) T*)(wr + v);
#pragma unroll
            for (int r = 0; r < RW; ++r) m[r] = fma(wv, seg[v + r], m[r]);
        }
    }
}

constexpr int PSF_RW = 4;

inline void psf_tile(const Geo& g, int K, int& stride, int& rows) {
    const int nsx = (g.nx + PSF_RW - 1) / PSF_RW;
    const int nq = (PSF_RW + K - 1 + 3) / 4;
    stride = (nsx - 1) * PSF_RW + 4 * nq;
    rows = g.ny + K - 1;
}

// One particle's PSF stage (whole work-group): the image buf[ny][nx] is
// loaded into an LDS tile with a zero halo; mode 0 writes the convolved
// model to out, modes 1-2 compute chi^2 -> logL, mode 2 also replaces buf by
// the adjoint image (correlation of the residual w (d - m) with the PSF).
template <int K, int MODE, int NT>
__device__ __forceinline__ void psf_body(float valid, const Geo& g, float* buf,
                                         const double* __restrict__ wflip,
                                         const float* __restrict__ wpsf,
                                         const float* __restrict__ data,
                                         const float* __restrict__ invvar, float* out, float* logl,
                                         double* logl64, int stride, int rows, float* lds,
                                         double* red) {
    constexpr int H = (K - 1) / 2;
    constexpr int RW = PSF_RW;
    const int tid = threadIdx.x;
    if (MODE != 0 && valid != 1.0f) {
        if (tid == 0) {
            const float v = valid == 2.0f ? __builtin_nanf("") : -__builtin_inff();
            *logl = v;
            if (logl64) *logl64 = (double)v;
        }
        return;
    }
    const int total = rows * stride;
    for (int q = tid; q < total; q += NT) lds[q] = 0.f;
    __syncthreads();
    for (int pix = tid; pix < g.npix; pix += NT) {
        const int i = pix / g.nx, j = pix - i * g.nx;
        lds[(i + H) * stride + j + H] = buf[pix];
    }
    __syncthreads();
    const int nsx = (g.nx + RW - 1) / RW, nstrips = nsx * g.ny;
    double chi = 0.0;
    for (int st = tid; st < nstrips; st += NT) {
        const int i = st / nsx, j0 = (st - i * nsx) * RW;
        double m[RW];
        correlate<K, RW, double>(lds, stride, i, j0, wflip, m);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int j = j0 + r;
            if (j < g.nx) {
                const int idx = i * g.nx + j;
                if (MODE == 0) {
                    out[idx] = (float)m[r];
                } else {
                    const double dlt = (double)ldg(data + idx) - m[r];
                    const double w = (double)ldg(invvar + idx);
                    chi = fma(w * dlt, dlt, chi);
                    if (MODE == 2) buf[idx] = (float)(w * dlt);
                }
            }
        }
    }
    if (MODE == 0) {
        __syncthreads();
        return;
    }
    chi = block_sum<NT>(chi, red);
    if (tid == 0) {
        *logl = (float)(-0.5 * chi);
        if (logl64) *logl64 = -0.5 * chi;
    }
    if (MODE == 2) {
        __syncthreads();
        for (int pix = tid; pix < g.npix; pix += NT) {
            const int i = pix / g.nx, j = pix - i * g.nx;
            lds[(i + H) * stride + j + H] = buf[pix];
        }
        __syncthreads();
        for (int st = tid; st < nstrips; st += NT) {
            const int i = st / nsx, j0 = (st - i * nsx) * RW;
            float m[RW];
            correlate<K, RW, float>(lds, stride, i, j0, wpsf, m);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int j = j0 + r;
                if (j < g.nx) buf[i * g.nx + j] = m[r];
            }
        }
    }
    __syncthreads();
}

// At most 128 VGPRs (four waves per SIMD): with a small K and 256 threads
// the compiler would otherwise keep all K^2 float64 taps in registers and
// run one wave per SIMD.
template <int K, int MODE, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_psf(const float* __restrict__ consts, Geo g, float* img,
                                             const double* __restrict__ wflip,
                                             const float* __restrict__ wpsf,
                                             const float* __restrict__ data,
                                             const float* __restrict__ invvar, float* out,
                                             float* logl, double* logl64, int stride, int rows) {
    extern __shared__ float4 lds4[];
    __shared__ double red[NT / 64];
    const int p = blockIdx.x;
    psf_body<K, MODE, NT>(consts[(size_t)p * CSTRIDE + C_VALID], g, img + (size_t)p * g.npix, wflip, wpsf,
                      data, invvar, out ? out + (size_t)p * g.npix : nullptr, logl ? logl + p : nullptr,
                      logl64 ? logl64 + p : nullptr, stride, rows, reinterpret_cast<float*>(lds4), red);
}

// Chain rule of one particle: sums its nchunks partial rows (fixed order) and
// maps the accumulated adjoint sums to dlogL/dtheta in the canonical order.
__device__ void finalize_particle(const ModelInfo& mi, int nchunks, const float* __restrict__ th,
                                  float valid, const double* __restrict__ base,
                                  float* __restrict__ g) {
    const int nc = mi.n_lens_light + mi.n_source;
    const int nacc = n_acc(mi);
    if (valid != 1.0f) {
        const float v = valid == 2.0f ? __builtin_nanf("") : 0.0f;
        for (int q = 0; q < mi.d; ++q) g[q] = v;
        return;
    }
    auto acc = [&](int q) {
        double s = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) s += base[(size_t)ch * nacc + q];
        return s;
    };
    const bool epl = mi.mass_model == LENS_MASS_EPL;
    int o = 0;
    const double tE = th[o++];
    const double t = epl ? (double)th[o++] - 1.0 : 1.0;
    const double e1 = th[o], e2 = th[o + 1];
    const double c2 = e1 * e1 + e2 * e2, c = sqrt(c2);
    const double H = acc(A_H);
    // alpha = theta_E sqrt(1-c^2) (b/R)^(t-1) V0 S,  b = theta_E sqrt((1-c)/(1+c))
    g[0] = (float)(H * t / tE);
    if (epl) {
        const double lnb = log(tE) + 0.5 * log((1.0 - c) / (1.0 + c));
        g[1] = (float)(acc(A_T) + lnb * H);
    }
    const double gc = -H * c / (1.0 - c2) - (t - 1.0) * H / (1.0 - c2) - acc(A_UC) / (1.0 + c);
    const double ec1 = c > 0.0 ? e1 / c : 0.0, ec2 = c > 0.0 ? e2 / c : 0.0;
    g[o] = (float)(gc * ec1 - acc(A_ZE) - acc(A_UW) / (1.0 + c));
    g[o + 1] = (float)(gc * ec2 + acc(A_ZE + 1) + acc(A_UW + 1) / (1.0 + c));
    const double ubx = acc(A_UB), uby = acc(A_UB + 1);
    const double wbx = (ubx - (ubx * e1 + uby * e2)) / (1.0 + c);
    const double wby = (uby - (ubx * e2 - uby * e1)) / (1.0 + c);
    g[o + 2] = (float)(-wbx);
    g[o + 3] = (float)(-wby);
    g[o + 4] = (float)acc(A_SH);
    g[o + 5] = (float)acc(A_SH + 1);
    o += 6;
    for (int k = 0; k < nc; ++k, o += 7) {
        const int ab = A_SERS + A_SERS_STRIDE * k;
        const double Re = th[o], n = th[o + 1], se1 = th[o + 2], se2 = th[o + 3], Ie = th[o + 6];
        const double bn = 1.9992 * n - 0.3271;
        const double kap = -bn / (2.0 * n);
        const double aE = acc(ab + AS_E), aWU = acc(ab + AS_WU), aWUL = acc(ab + AS_WUL);
        const double qxx = acc(ab + AS_QXX), qxy = acc(ab + AS_QXY), qyy = acc(ab + AS_QYY);
        const double qx = acc(ab + AS_QX), qy = acc(ab + AS_QY);
        // I = I_e exp(-b_n (u - 1)), u = (R/R_e)^(1/n)
        g[o + 6] = (float)aE;
        g[o] = (float)(bn / (n * Re) * aWU);
        const double wulnr = 0.34657359027997264 * aWUL - log(Re) * aWU;   // sum W u ln(R/R_e)
        g[o + 1] = (float)(-1.9992 * (aWU - Ie * aE) + bn / (n * n) * wulnr);
        const double cs2 = se1 * se1 + se2 * se2, D = 1.0 - cs2, D2 = D * D;
        const double a11 = (1.0 + cs2 - 2.0 * se1) / D, a22 = (1.0 + cs2 + 2.0 * se1) / D,
                     a12 = -2.0 * se2 / D;
        const double gA11 = kap * qxx, gA12 = 2.0 * kap * qxy, gA22 = kap * qyy;
        const double n11 = 1.0 + cs2 - 2.0 * se1, n22 = 1.0 + cs2 + 2.0 * se1;
        const double d11_1 = (2.0 * se1 - 2.0) / D + n11 * 2.0 * se1 / D2;
        const double d11_2 = 2.0 * se2 / D + n11 * 2.0 * se2 / D2;
        const double d22_1 = (2.0 * se1 + 2.0) / D + n22 * 2.0 * se1 / D2;
        const double d22_2 = 2.0 * se2 / D + n22 * 2.0 * se2 / D2;
        const double d12_1 = -4.0 * se2 * se1 / D2;
        const double d12_2 = -2.0 / D - 4.0 * se2 * se2 / D2;
        g[o + 2] = (float)(gA11 * d11_1 + gA12 * d12_1 + gA22 * d22_1);
        g[o + 3] = (float)(gA11 * d11_2 + gA12 * d12_2 + gA22 * d22_2);
        g[o + 4] = (float)(-2.0 * kap * (a11 * qx + a12 * qy));
        g[o + 5] = (float)(-2.0 * kap * (a12 * qx + a22 * qy));
    }
    if (mi.n_shapelet) {
        // V = (1/beta) G((x - x_c)/beta, (y - y_c)/beta): dV/dbeta = -(V + u V_u + v V_v)/beta,
        // dV/dx_c = -V_u/beta; the coefficients' sums are their derivatives
        const int ab = A_SERS + A_SERS_STRIDE * nc;
        const double ib = 1.0 / (double)th[o];
        g[o] = (float)(-ib * acc(ab + AH_B));
        g[o + 1] = (float)(-ib * acc(ab + AH_U));
        g[o + 2] = (float)(-ib * acc(ab + AH_V));
        int k = 0;
        for (int n = 0; n <= mi.sh_nmax; ++n)
            for (int n2 = 0; n2 <= n; ++n2, ++k) g[o + 3 + k] = (float)acc(ab + AH_C + sh_row(n2) + (n - n2));
    }
}

// Particle p's partial rows start at row p * row_stride; the first nchunks are summed.
__global__ void k_finalize(ModelInfo mi, int P, int nchunks, int row_stride, const float* __restrict__ theta,
                           const float* __restrict__ consts, const double* __restrict__ partial,
                           float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int nacc = n_acc(mi);
    finalize_particle(mi, nchunks, theta + (size_t)p * mi.d, consts[(size_t)p * CSTRIDE + C_VALID],
                      partial + (size_t)p * row_stride * nacc, grad + (size_t)p * mi.d);
}

// ---------------------------------------------------------------------------
// Uneven batch: persistent render / adjoint over a cost-sorted work list,
// PSF stage per PSF size, finalize over all particles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int next_item(int* counter, int* slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return it;
}

template <int MASS, int NL, int NS>
__global__ __launch_bounds__(256) void k_batch_render(const BatchSys* __restrict__ sys,
                                                      const WorkItem* __restrict__ items, int n_items,
                                                      int* __restrict__ counter,
                                                      const float* __restrict__ consts,
                                                      float* __restrict__ img) {
    __shared__ int slot;
    init_math_tab();
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const BatchSys& S = sys[w.sys];
        const int pix0 = w.chunk * S.ppb;
        render_chunk<MASS, NL, NS, 0>(consts + (size_t)(S.p0 + w.p) * CSTRIDE, S.g, pix0,
                                   min(pix0 + S.ppb, S.g.npix),
                                   img + S.img_off + (size_t)w.p * S.g.npix);
    }
}

template <int MASS, int NL, int NS>
// Four waves per SIMD (at most 128 VGPRs): measured faster than the three the
// register demand would otherwise give, with the few spills left outside the
// sub-pixel loops.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch_adjoint(const BatchSys* __restrict__ sys,
                                                       const WorkItem* __restrict__ items, int n_items,
                                                       int* __restrict__ counter,
                                                       const float* __restrict__ consts,
                                                       const float* __restrict__ gimg,
                                                       double* __restrict__ partial) {
    constexpr int NACC = A_SERS + A_SERS_STRIDE * (NL + NS);
    __shared__ double red[NACC][4];
    __shared__ int slot;
    init_math_tab();
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const BatchSys& S = sys[w.sys];
        const int pix0 = w.chunk * S.ppb;
        adjoint_chunk<MASS, NL, NS, 0>(consts + (size_t)(S.p0 + w.p) * CSTRIDE, S.g, pix0,
                                    min(pix0 + S.ppb, S.g.npix),
                                    gimg + S.img_off + (size_t)w.p * S.g.npix,
                                    partial + (S.part_off + (size_t)w.p * S.nch + w.chunk) * NACC, red);
    }
}

// One work-group per (system, particle) of one PSF size class.
template <int K, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch_psf(const BatchSys* __restrict__ sys,
                                                   const WorkItem* __restrict__ items,
                                                   const float* __restrict__ consts, float* img,
                                                   float* logl, double* logl64) {
    extern __shared__ float4 lds4[];
    __shared__ double red[NT / 64];
    const WorkItem w = items[blockIdx.x];
    const BatchSys& S = sys[w.sys];
    const int gp = S.p0 + w.p;
    psf_body<K, 2, NT>(consts[(size_t)gp * CSTRIDE + C_VALID], S.g, img + S.img_off + (size_t)w.p * S.g.npix,
                   S.wflip, S.wpsf, S.data, S.invvar, nullptr, logl + gp, logl64 ? logl64 + gp : nullptr,
                   S.stride, S.rows,
                   reinterpret_cast<float*>(lds4), red);
}

__global__ void k_batch_finalize(ModelInfo mi, int N, const BatchSys* __restrict__ sys,
                                 const int* __restrict__ particle_sys, const float* __restrict__ theta,
                                 const float* __restrict__ consts, const double* __restrict__ partial,
                                 float* __restrict__ grad) {
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= N) return;
    const BatchSys& S = sys[particle_sys[gp]];
    const int nacc = n_acc(mi);
    const int p = gp - S.p0;
    finalize_particle(mi, S.nch, theta + (size_t)gp * mi.d, consts[(size_t)gp * CSTRIDE + C_VALID],
                      partial + (S.part_off + (size_t)p * S.nch) * nacc, grad + (size_t)gp * mi.d);
}

// ---------------------------------------------------------------------------
// Tiled PSF stage for images whose whole tile does not fit the LDS (large
// cutouts): grid (particle, pixel tile); each work-group stages a
// PSF_TH x PSF_TW output tile plus its (K-1)/2 halo in LDS.
//   pass 1 (MODE 0|1|2): model m = image (*) PSF in float64;
//     MODE 0 writes m; MODE 1|2 write the tile's float64 chi^2 partial and
//     MODE 2 the residual w (d - m) to res;
//   pass 2: the adjoint image, correlation of res with the PSF (float32),
//     into img (every tile reads only res, so img can be overwritten);
//   k_chi_reduce sums each particle's tile partials in tile order.
// ---------------------------------------------------------------------------
constexpr int PSF_TH = 32, PSF_TW = 128;

template <int K>
struct TileDims {
    static constexpr int NQ = (PSF_RW + K - 1 + 3) / 4;
    static constexpr int STRIDE = PSF_TW - PSF_RW + 4 * NQ;   // floats, multiple of 4
    static constexpr int ROWS = PSF_TH + K - 1;
};

// Loads the tile at (i0, j0) of src [ny][nx] with its halo into lds; zero
// outside the image.
template <int K>
__device__ __forceinline__ void load_tile(const Geo& g, const float* __restrict__ src, int i0, int j0,
                                          float* lds) {
    constexpr int H = (K - 1) / 2, ST = TileDims<K>::STRIDE, R = TileDims<K>::ROWS;
    for (int q = threadIdx.x; q < R * ST; q += 256) {
        const int r = q / ST, c = q - r * ST;
        const int gi = i0 + r - H, gj = j0 + c - H;
        const bool in = c < PSF_TW + K - 1 && gi >= 0 && gi < g.ny && gj >= 0 && gj < g.nx;
        lds[q] = in ? src[(size_t)gi * g.nx + gj] : 0.f;
    }
    __syncthreads();
}

template <int K, int MODE>
__global__ __launch_bounds__(256) void k_psf_tile(const float* __restrict__ consts, Geo g, int tiles_x,
                                                  const float* __restrict__ img, float* __restrict__ res,
                                                  const double* __restrict__ wflip,
                                                  const float* __restrict__ data,
                                                  const float* __restrict__ invvar, float* __restrict__ out,
                                                  double* __restrict__ chi_part) {
    __shared__ float4 lds4[TileDims<K>::ROWS * TileDims<K>::STRIDE / 4];
    __shared__ double red[4];
    float* lds = reinterpret_cast<float*>(lds4);
    const int p = blockIdx.x, tile = blockIdx.y;
    const int i0 = (tile / tiles_x) * PSF_TH, j0 = (tile - (tile / tiles_x) * tiles_x) * PSF_TW;
    const size_t base = (size_t)p * g.npix;
    if (MODE != 0 && consts[(size_t)p * CSTRIDE + C_VALID] != 1.0f) {
        // no valid profile: zero residual and partial (logL set by k_chi_reduce)
        if (MODE == 2)
            for (int q = threadIdx.x; q < PSF_TH * PSF_TW; q += 256) {
                const int i = i0 + q / PSF_TW, j = j0 + q % PSF_TW;
                if (i < g.ny && j < g.nx) res[base + (size_t)i * g.nx + j] = 0.f;
            }
        if (threadIdx.x == 0) chi_part[(size_t)p * gridDim.y + tile] = 0.0;
        return;
    }
    load_tile<K>(g, img + base, i0, j0, lds);
    constexpr int NS = PSF_TW / PSF_RW;   // strips per tile row
    double chi = 0.0;
    for (int st = threadIdx.x; st < PSF_TH * NS; st += 256) {
        const int li = st / NS, lj = (st - li * NS) * PSF_RW;
        const int i = i0 + li;
        double m[PSF_RW];
        correlate<K, PSF_RW, double>(lds, TileDims<K>::STRIDE, li, lj, wflip, m);
#pragma unroll
        for (int r = 0; r < PSF_RW; ++r) {
            const int j = j0 + lj + r;
            if (i < g.ny && j < g.nx) {
                const size_t idx = (size_t)i * g.nx + j;
                if (MODE == 0) {
                    out[base + idx] = (float)m[r];
                } else {
                    const double dlt = (double)ldg(data + idx) - m[r];
                    const double w = (double)ldg(invvar + idx);
                    chi = fma(w * dlt, dlt, chi);
                    if (MODE == 2) res[base + idx] = (float)(w * dlt);
                }
            }
        }
    }
    if (MODE != 0) {
        chi = block_sum<256>(chi, red);
        if (threadIdx.x == 0) chi_part[(size_t)p * gridDim.y + tile] = chi;
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_psf_tile_adj(Geo g, int tiles_x, const float* __restrict__ res,
                                                      const float* __restrict__ wpsf, float* __restrict__ img) {
    __shared__ float4 lds4[TileDims<K>::ROWS * TileDims<K>::STRIDE / 4];
    float* lds = reinterpret_cast<float*>(lds4);
    const int p = blockIdx.x, tile = blockIdx.y;
    const int i0 = (tile / tiles_x) * PSF_TH, j0 = (tile - (tile / tiles_x) * tiles_x) * PSF_TW;
    const size_t base = (size_t)p * g.npix;
    load_tile<K>(g, res + base, i0, j0, lds);
    constexpr int NS = PSF_TW / PSF_RW;
    for (int st = threadIdx.x; st < PSF_TH * NS; st += 256) {
        const int li = st / NS, lj = (st - li * NS) * PSF_RW;
        const int i = i0 + li;
        float m[PSF_RW];
        correlate<K, PSF_RW, float>(lds, TileDims<K>::STRIDE, li, lj, wpsf, m);
#pragma unroll
        for (int r = 0; r < PSF_RW; ++r) {
            const int j = j0 + lj + r;
            if (i < g.ny && j < g.nx) img[base + (size_t)i * g.nx + j] = m[r];
        }
    }
}

// logL of every particle from its tile partials (fixed tile order).
__global__ void k_chi_reduce(int P, int ntiles, const float* __restrict__ consts,
                             const double* __restrict__ chi_part, float* __restrict__ logl,
                             double* __restrict__ logl64) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float valid = consts[(size_t)p * CSTRIDE + C_VALID];
    double v;
    if (valid != 1.0f) {
        v = valid == 2.0f ? (double)__builtin_nanf("") : -(double)__builtin_inff();
    } else {
        double chi = 0.0;
        for (int t = 0; t < ntiles; ++t) chi += chi_part[(size_t)p * ntiles + t];
        v = -0.5 * chi;
    }
    logl[p] = (float)v;
    if (logl64) logl64[p] = v;
}

// Sums the nch partial rows of every particle into its first row, so that
// k_finalize can then run with one row per particle.  One wave per
// (particle, accumulator): lane l sums rows l, l + 64, ... in order, then a
// fixed butterfly over the lanes (deterministic; the rounding order differs
// from k_finalize's serial sum over the rows).
__global__ __launch_bounds__(64) void k_partial_sum(int nch, int nacc, double* __restrict__ partial) {
    const int a = blockIdx.y, lane = threadIdx.x;
    double* base = partial + (size_t)blockIdx.x * nch * nacc;
    double s = 0.0;
    for (int ch = lane; ch < nch; ch += 64) s += base[(size_t)ch * nacc + a];
    s = wave_sum(s);
    if (lane == 0) base[a] = s;
}

// In place, for every (particle, accumulator): the sum over the particle's
// nch partial rows in row order (the order k_finalize sums them) into row 0,
// so k_finalize then reads one row with the same result.  Each thread writes
// only its own column.
__global__ void k_presum_rows(int P, int nch, int nacc, double* __restrict__ partial) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)P * nacc) return;
    const int p = (int)(i / nacc), a = (int)(i % nacc);
    double* base = partial + (size_t)p * nch * nacc;
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += base[(size_t)ch * nacc + a];
    base[a] = s;
}

__global__ void k_flip(int K, const float* __restrict__ psf, double* __restrict__ flipped) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * K) return;
    const int u = q / K, v = q - u * K;
    flipped[(K - 1 - u) * K + (K - 1 - v)] = (double)psf[q];
}

// ---------------------------------------------------------------------------
// Launchers: template dispatch on (mass model, #lens light, #sources) and K
// ---------------------------------------------------------------------------
template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<mass>, IC<n_lens_light>, IC<n_source>) for the compiled
// combinations; returns false for any other.
template <int M, class F>
bool dispatch_ls(int nl, int ns, F&& f) {
    switch (nl * 4 + ns) {
        case 0 * 4 + 1: f(IC<M>{}, IC<0>{}, IC<1>{}); return true;
        case 0 * 4 + 2: f(IC<M>{}, IC<0>{}, IC<2>{}); return true;
        case 0 * 4 + 3: f(IC<M>{}, IC<0>{}, IC<3>{}); return true;
        case 1 * 4 + 1: f(IC<M>{}, IC<1>{}, IC<1>{}); return true;
        case 1 * 4 + 2: f(IC<M>{}, IC<1>{}, IC<2>{}); return true;
        case 1 * 4 + 3: f(IC<M>{}, IC<1>{}, IC<3>{}); return true;
        case 2 * 4 + 1: f(IC<M>{}, IC<2>{}, IC<1>{}); return true;
        case 2 * 4 + 2: f(IC<M>{}, IC<2>{}, IC<2>{}); return true;
        case 2 * 4 + 3: f(IC<M>{}, IC<2>{}, IC<3>{}); return true;
        case 3 * 4 + 1: f(IC<M>{}, IC<3>{}, IC<1>{}); return true;
        case 3 * 4 + 2: f(IC<M>{}, IC<3>{}, IC<2>{}); return true;
        case 3 * 4 + 3: f(IC<M>{}, IC<3>{}, IC<3>{}); return true;
        default: return false;
    }
}

// Models without a shapelet source (the uneven batch's kernels).
template <class F>
bool dispatch_model(const ModelInfo& mi, F&& f) {
    if (mi.n_shapelet) return false;
    if (mi.mass_model == LENS_MASS_EPL)
        return dispatch_ls<LENS_MASS_EPL>(mi.n_lens_light, mi.n_source, f);
    return dispatch_ls<LENS_MASS_SIE>(mi.n_lens_light, mi.n_source, f);
}

// Calls f(IC<mass>, IC<n_lens_light>, IC<n_source>, IC<n_shapelet>); a
// shapelet source is compiled with at most one lens light and one Sersic source.
template <class F>
bool dispatch_model_sh(const ModelInfo& mi, F&& f) {
    if (!mi.n_shapelet) return dispatch_model(mi, [&](auto M, auto NL, auto NS) { f(M, NL, NS, IC<0>{}); });
    if (mi.n_lens_light > 1 || mi.n_source > 1) return false;
    auto g = [&](auto M) {
        switch (mi.n_lens_light * 2 + mi.n_source) {
            case 0: f(M, IC<0>{}, IC<0>{}, IC<1>{}); return true;
            case 1: f(M, IC<0>{}, IC<1>{}, IC<1>{}); return true;
            case 2: f(M, IC<1>{}, IC<0>{}, IC<1>{}); return true;
            case 3: f(M, IC<1>{}, IC<1>{}, IC<1>{}); return true;
            default: return false;
        }
    };
    return mi.mass_model == LENS_MASS_EPL ? g(IC<LENS_MASS_EPL>{}) : g(IC<LENS_MASS_SIE>{});
}

hipError_t launch_prologue(const ModelInfo& mi, int P, const float* theta, float* consts,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_prologue, dim3((P + 63) / 64), dim3(64), 0, st, mi, P, theta, consts);
    return hipGetLastError();
}

hipError_t launch_render(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                         float* img, hipStream_t st) {
    const int nch = chunks_for(g.npix, ppt);
    const dim3 grid(P, nch);
    const int ppb = 256 * ppt;
    const bool done = dispatch_model_sh(mi, [&](auto M, auto NL, auto NS, auto SH) {
        hipLaunchKernelGGL((k_render<decltype(M)::value, decltype(NL)::value, decltype(NS)::value, decltype(SH)::value>),
                           grid, dim3(256), 0, st, consts, g, ppb, img);
    });
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_render_split(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                               float* img, hipStream_t st) {
    const int nch = chunks_for(g.npix, ppt);
    const dim3 grid(P, nch);
    const int ppb = 256 * ppt;
    const bool done = dispatch_model_sh(mi, [&](auto M, auto NL, auto NS, auto SH) {
        hipLaunchKernelGGL(
            (k_render_split<decltype(M)::value, decltype(NL)::value, decltype(NS)::value, decltype(SH)::value>), grid,
            dim3(256), 0, st, consts, g, ppb, mi.sh_nmax, img);
    });
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adjoint(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                          const float* gimg, double* partial, hipStream_t st) {
    const int nch = chunks_for(g.npix, ppt);
    const dim3 grid(P, nch);
    const int ppb = 256 * ppt;
    const bool done = dispatch_model_sh(mi, [&](auto M, auto NL, auto NS, auto SH) {
        constexpr int m = decltype(M)::value, l = decltype(NL)::value, n = decltype(NS)::value,
                      h = decltype(SH)::value;
        if constexpr (h != 0)
            hipLaunchKernelGGL((k_adjoint_sh<m, l, n, h>), grid, dim3(256), 0, st, consts, g, ppb, gimg, partial);
        else
            hipLaunchKernelGGL((k_adjoint<m, l, n, h>), grid, dim3(256), 0, st, consts, g, ppb, gimg, partial);
    });
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

// Work-group size of the PSF pass: the LDS tile limits the work-groups per
// CU, so large images get more threads per work-group to keep the SIMDs fed;
// the score counts resident waves per SIMD (up to 4) times the fraction of
// threads busy over the image's row strips.
int psf_threads(size_t shm, int nstrips) {
    int best = 256;
    double best_score = -1.0;
    for (int nt : {256, 512, 1024}) {
        const int by_lds = shm > 0 ? (int)((160 * 1024) / shm) : 64;
        const int blocks = std::min(by_lds, 2048 / nt);
        if (blocks < 1) continue;
        const int waves = blocks * nt / 256;
        const int rounds = (nstrips + nt - 1) / nt;
        const double eff = rounds > 0 ? (double)nstrips / ((double)nt * rounds) : 1.0;
        const double score = std::min(waves, 4) * eff;
        if (score > best_score + 1e-9) {
            best_score = score;
            best = nt;
        }
    }
    return best;
}

int psf_strips(const Geo& g) { return ((g.nx + PSF_RW - 1) / PSF_RW) * g.ny; }

template <int K, int MODE, int NT>
static void launch_psf_kernel(size_t shm, int P, const float* consts, const Geo& g, float* img, const double* wflip,
                              const float* wpsf, const float* data, const float* invvar, float* out, float* logl,
                              double* logl64, int stride, int rows, hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_psf<K, MODE, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)MAX_LDS_BYTES);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_psf<K, MODE, NT>), dim3(P), dim3(NT), shm, st, consts, g, img, wflip, wpsf, data, invvar,
                       out, logl, logl64, stride, rows);
}

template <int K>
static hipError_t launch_psf_k(const Geo& g, int mode, int P, const float* consts, float* img,
                               const double* wflip, const float* wpsf, const float* data,
                               const float* invvar, float* out, float* logl, double* logl64,
                               hipStream_t st) {
    int stride, rows;
    psf_tile(g, K, stride, rows);
    const size_t shm = (size_t)stride * rows * sizeof(float);
    if (mode == 0) {
        launch_psf_kernel<K, 0, 256>(shm, P, consts, g, img, wflip, wpsf, data, invvar, out, logl, logl64, stride,
                                     rows, st);
    } else if (mode == 1) {
        launch_psf_kernel<K, 1, 256>(shm, P, consts, g, img, wflip, wpsf, data, invvar, out, logl, logl64, stride,
                                     rows, st);
    } else {
        const int nt = psf_threads(shm, psf_strips(g));
        if (nt == 1024)
            launch_psf_kernel<K, 2, 1024>(shm, P, consts, g, img, wflip, wpsf, data, invvar, out, logl, logl64,
                                          stride, rows, st);
        else if (nt == 512)
            launch_psf_kernel<K, 2, 512>(shm, P, consts, g, img, wflip, wpsf, data, invvar, out, logl, logl64,
                                         stride, rows, st);
        else
            launch_psf_kernel<K, 2, 256>(shm, P, consts, g, img, wflip, wpsf, data, invvar, out, logl, logl64,
                                         stride, rows, st);
    }
    return hipGetLastError();
}

hipError_t launch_psf(const ModelInfo& mi, const Geo& g, int K, int mode, int P,
                      const float* consts, float* img, const double* wflip, const float* wpsf,
                      const float* data, const float* invvar, float* out, float* logl,
                      double* logl64, hipStream_t st) {
    (void)mi;
    switch (K) {
#define LENS_PSF_CASE(KK) \
    case KK: return launch_psf_k<KK>(g, mode, P, consts, img, wflip, wpsf, data, invvar, out, logl, logl64, st);
        LENS_PSF_CASE(1) LENS_PSF_CASE(3) LENS_PSF_CASE(5) LENS_PSF_CASE(7) LENS_PSF_CASE(9)
        LENS_PSF_CASE(11) LENS_PSF_CASE(13) LENS_PSF_CASE(15) LENS_PSF_CASE(17) LENS_PSF_CASE(19)
        LENS_PSF_CASE(21) LENS_PSF_CASE(23) LENS_PSF_CASE(25) LENS_PSF_CASE(27) LENS_PSF_CASE(29)
        LENS_PSF_CASE(31)
#undef LENS_PSF_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const ModelInfo& mi, int P, int nchunks, const float* theta,
                           const float* consts, const double* partial, float* grad,
                           hipStream_t st, int row_stride) {
    if (row_stride < nchunks) row_stride = nchunks;
    hipLaunchKernelGGL(k_finalize, dim3((P + 63) / 64), dim3(64), 0, st, mi, P, nchunks, row_stride, theta,
                       consts, partial, grad);
    return hipGetLastError();
}

hipError_t launch_batch_render(const ModelInfo& mi, int grid, const BatchSys* sys,
                               const WorkItem* items, int n_items, int* counter,
                               const float* consts, float* img, hipStream_t st) {
    const bool done = dispatch_model(mi, [&](auto M, auto NL, auto NS) {
        hipLaunchKernelGGL(
            (k_batch_render<decltype(M)::value, decltype(NL)::value, decltype(NS)::value>),
            dim3(grid), dim3(256), 0, st, sys, items, n_items, counter, consts, img);
    });
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_batch_adjoint(const ModelInfo& mi, int grid, const BatchSys* sys,
                                const WorkItem* items, int n_items, int* counter,
                                const float* consts, const float* gimg, double* partial,
                                hipStream_t st) {
    const bool done = dispatch_model(mi, [&](auto M, auto NL, auto NS) {
        hipLaunchKernelGGL(
            (k_batch_adjoint<decltype(M)::value, decltype(NL)::value, decltype(NS)::value>),
            dim3(grid), dim3(256), 0, st, sys, items, n_items, counter, consts, gimg, partial);
    });
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int K, int NT>
static void launch_batch_psf_kernel(int n_items, const BatchSys* sys, const WorkItem* items, const float* consts,
                                    float* img, float* logl, double* logl64, size_t shm, hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_psf<K, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)MAX_LDS_BYTES);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_batch_psf<K, NT>), dim3(n_items), dim3(NT), shm, st, sys, items, consts, img, logl,
                       logl64);
}

template <int K>
static hipError_t launch_batch_psf_k(int n_items, const BatchSys* sys, const WorkItem* items,
                                     const float* consts, float* img, float* logl, double* logl64,
                                     size_t shm, int nt, hipStream_t st) {
    if (nt == 1024)
        launch_batch_psf_kernel<K, 1024>(n_items, sys, items, consts, img, logl, logl64, shm, st);
    else if (nt == 512)
        launch_batch_psf_kernel<K, 512>(n_items, sys, items, consts, img, logl, logl64, shm, st);
    else
        launch_batch_psf_kernel<K, 256>(n_items, sys, items, consts, img, logl, logl64, shm, st);
    return hipGetLastError();
}

hipError_t launch_batch_psf(int K, int n_items, const BatchSys* sys, const WorkItem* items,
                            const float* consts, float* img, float* logl, double* logl64,
                            size_t shm, int nt, hipStream_t st) {
    switch (K) {
#define LENS_BPSF_CASE(KK) \
    case KK: return launch_batch_psf_k<KK>(n_items, sys, items, consts, img, logl, logl64, shm, nt, st);
        LENS_BPSF_CASE(1) LENS_BPSF_CASE(3) LENS_BPSF_CASE(5) LENS_BPSF_CASE(7) LENS_BPSF_CASE(9)
        LENS_BPSF_CASE(11) LENS_BPSF_CASE(13) LENS_BPSF_CASE(15) LENS_BPSF_CASE(17) LENS_BPSF_CASE(19)
        LENS_BPSF_CASE(21) LENS_BPSF_CASE(23) LENS_BPSF_CASE(25) LENS_BPSF_CASE(27) LENS_BPSF_CASE(29)
        LENS_BPSF_CASE(31)
#undef LENS_BPSF_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_finalize(const ModelInfo& mi, int N, const BatchSys* sys,
                                 const int* particle_sys, const float* theta, const float* consts,
                                 const double* partial, float* grad, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_finalize, dim3((N + 63) / 64), dim3(64), 0, st, mi, N, sys, particle_sys,
                       theta, consts, partial, grad);
    return hipGetLastError();
}

int batch_blocks_per_cu(const ModelInfo& mi, bool adjoint) {
    int nb = 0;
    dispatch_model(mi, [&](auto M, auto NL, auto NS) {
        constexpr int m = decltype(M)::value, l = decltype(NL)::value, s = decltype(NS)::value;
        if (adjoint)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_adjoint<m, l, s>, 256, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_render<m, l, s>, 256, 0);
    });
    return nb > 0 ? nb : 1;
}

hipError_t launch_flip(int K, const float* psf, double* flipped, hipStream_t st) {
    hipLaunchKernelGGL(k_flip, dim3((K * K + 255) / 256), dim3(256), 0, st, K, psf, flipped);
    return hipGetLastError();
}

int psf_num_tiles(const Geo& g) {
    return ((g.nx + PSF_TW - 1) / PSF_TW) * ((g.ny + PSF_TH - 1) / PSF_TH);
}

template <int K>
static hipError_t launch_psf_tiled_k(const Geo& g, int mode, int P, const float* consts, float* img, float* res,
                                     const double* wflip, const float* wpsf, const float* data,
                                     const float* invvar, float* out, float* logl, double* logl64,
                                     double* chi_part, hipStream_t st) {
    const int tiles_x = (g.nx + PSF_TW - 1) / PSF_TW;
    const int nt = psf_num_tiles(g);
    const dim3 grid(P, nt);
    if (mode == 0) {
        hipLaunchKernelGGL((k_psf_tile<K, 0>), grid, dim3(256), 0, st, consts, g, tiles_x, img, res, wflip, data,
                           invvar, out, chi_part);
        return hipGetLastError();
    }
    if (mode == 1)
        hipLaunchKernelGGL((k_psf_tile<K, 1>), grid, dim3(256), 0, st, consts, g, tiles_x, img, res, wflip, data,
                           invvar, out, chi_part);
    else
        hipLaunchKernelGGL((k_psf_tile<K, 2>), grid, dim3(256), 0, st, consts, g, tiles_x, img, res, wflip, data,
                           invvar, out, chi_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chi_reduce, dim3((P + 63) / 64), dim3(64), 0, st, P, nt, consts, chi_part, logl, logl64);
    e = hipGetLastError();
    if (e != hipSuccess || mode != 2) return e;
    hipLaunchKernelGGL((k_psf_tile_adj<K>), grid, dim3(256), 0, st, g, tiles_x, res, wpsf, img);
    return hipGetLastError();
}

hipError_t launch_psf_tiled(const Geo& g, int K, int mode, int P, const float* consts, float* img, float* res,
                            const double* wflip, const float* wpsf, const float* data, const float* invvar,
                            float* out, float* logl, double* logl64, double* chi_part, hipStream_t st) {
    switch (K) {
#define LENS_TPSF_CASE(KK)                                                                                  \
    case KK:                                                                                                \
        return launch_psf_tiled_k<KK>(g, mode, P, consts, img, res, wflip, wpsf, data, invvar, out, logl,  \
                                      logl64, chi_part, st);
        LENS_TPSF_CASE(1) LENS_TPSF_CASE(3) LENS_TPSF_CASE(5) LENS_TPSF_CASE(7) LENS_TPSF_CASE(9)
        LENS_TPSF_CASE(11) LENS_TPSF_CASE(13) LENS_TPSF_CASE(15) LENS_TPSF_CASE(17) LENS_TPSF_CASE(19)
        LENS_TPSF_CASE(21) LENS_TPSF_CASE(23) LENS_TPSF_CASE(25) LENS_TPSF_CASE(27) LENS_TPSF_CASE(29)
        LENS_TPSF_CASE(31)
#undef LENS_TPSF_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_presum_rows(int P, int nch, int nacc, double* partial, hipStream_t st) {
    const long long n = (long long)P * nacc;
    hipLaunchKernelGGL(k_presum_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nch, nacc, partial);
    return hipGetLastError();
}

hipError_t launch_partial_sum(int P, int nch, int nacc, double* partial, hipStream_t st) {
    hipLaunchKernelGGL(k_partial_sum, dim3(P, nacc), dim3(64), 0, st, nch, nacc, partial);
    return hipGetLastError();
}

void psf_tile_dims(const Geo& g, int K, int& stride, int& rows) { psf_tile(g, K, stride, rows); }

size_t psf_lds_bytes(const Geo& g, int K) {
    int stride, rows;
    psf_tile(g, K, stride, rows);
    return (size_t)stride * rows * sizeof(float);
}

}  // namespace lens
