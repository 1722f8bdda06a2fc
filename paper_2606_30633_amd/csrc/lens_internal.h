// Internal declarations shared by the HIP kernels and the C-ABI host layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lens_api.h"

namespace lens {

// ---------------------------------------------------------------------------
// Per-particle constant block (float words), written by the prologue kernel
// and read by every per-sub-pixel kernel through wave-uniform (scalar) loads.
// ---------------------------------------------------------------------------
constexpr int C_VALID = 0;    // 1 valid, 0 no valid profile (-inf), 2 non-finite (NaN)
constexpr int C_KP = 1;       // padded length KP of the float64 series S (KP+1 multiple of 4), as float
constexpr int C_KPA = 2;      // padded length of the float32 series S'(z), dS/dt (adjoint), as float
// Mass block in float64 (word offsets, 8-byte aligned):
constexpr int D_X0 = 4;       // mass centre
constexpr int D_Y0 = 6;
constexpr int D_E1 = 8;       // mass ellipticity eps = e1 + i e2
constexpr int D_E2 = 10;
constexpr int D_UA = 12;      // U = (w - eps conj(w)) / (1 + |eps|):
constexpr int D_UB = 14;      //   Ux = UA wx - UE wy,  Uy = UB wy - UE wx
constexpr int D_UE = 16;
constexpr int D_C0 = 18;      // theta_E sqrt(1 - c^2)  (= 2b/(1+q))
constexpr int D_K0 = 20;      // 256 (t-1) log2 b   (exponent constants carry a factor 256:
constexpr int D_K1 = 22;      // 256 (t-1)/2         the float64 exp2 takes 256 v)
constexpr int D_G1 = 24;      // external shear
constexpr int D_G2 = 26;
constexpr int C_SERS = 32;    // Sersic components: SERS_STRIDE words each, float64 fields
constexpr int SERS_STRIDE = 24;
constexpr int S_XC = 0, S_YC = 2, S_A11 = 4, S_A12 = 6, S_A22 = 8, S_IE = 10,
              S_KU = 12, S_KU0 = 14, S_BL = 16;   // float64 (word offsets); KU = 256/(2n),
                                                  // KU0 = -256 log2(R_e)/n, BL = 256 b_n/ln 2
constexpr int S_KAP2 = 18;                         // float32
constexpr int S_A12X2 = 20;                        // float64: 2 a12
constexpr int MAX_COMP = LENS_MAX_LENS_LIGHT + LENS_MAX_SOURCE;
constexpr int KMAX_PAD = 128;            // entries per coefficient array
constexpr int C_COEF_S = 176;            // float64 c_0..c_KP (2 words each)
constexpr int C_COEF_Z = C_COEF_S + 2 * KMAX_PAD;   // float (m+1) c_{m+1}: S'(z)
constexpr int C_COEF_T = C_COEF_Z + KMAX_PAD;       // float dc_n/dt
// Shapelet source block: float64 scalars, then the coefficients in the
// kernels' layout: rows n2 = 0..SH_CAP, each n1 = 0..SH_CAP - n2 (zero where
// n1 + n2 > n_max), as float64 and as float32.
constexpr int SH_CAP = LENS_MAX_SHAPELET_NMAX;
constexpr int SH_NB = (SH_CAP + 1) * (SH_CAP + 2) / 2;    // 45
constexpr int C_SHAP = C_COEF_T + KMAX_PAD;                // 688
constexpr int SH_XC = 0, SH_YC = 2, SH_IB = 4, SH_E0 = 6;   // centre, 1/beta, pi^(-1/2)/beta (float64)
constexpr int SH_CD = 8;                                   // float64 coefficients (2 words each)
constexpr int SH_CF = SH_CD + 2 * SH_NB;                   // float32 coefficients
constexpr int CSTRIDE = C_SHAP + ((SH_CF + SH_NB + 3) / 4) * 4;   // 832 words
constexpr int KMAX_TERMS = KMAX_PAD - 1;

// First index of row n2 in the kernels' coefficient layout.
__host__ __device__ constexpr int sh_row(int n2) { return n2 * (SH_CAP + 1) - n2 * (n2 - 1) / 2; }

static_assert(C_SERS + MAX_COMP * SERS_STRIDE <= C_COEF_S, "constant layout");
static_assert(C_COEF_S % 4 == 0 && C_COEF_Z % 4 == 0 && C_COEF_T % 4 == 0 && CSTRIDE % 4 == 0,
              "16-byte alignment of the coefficient arrays");

// Adjoint accumulator layout (per particle, summed over sub-pixels).
constexpr int A_H = 0;        // sum Re(conj(G) alpha)
constexpr int A_T = 1;        // slope term
constexpr int A_ZE = 2;       // complex, 2 words
constexpr int A_UW = 4;       // complex
constexpr int A_UC = 6;
constexpr int A_UB = 7;       // complex
constexpr int A_SH = 9;       // complex: sum G * theta
constexpr int A_SERS = 11;    // 8 words per Sersic component
constexpr int A_SERS_STRIDE = 8;
constexpr int AS_E = 0, AS_WU = 1, AS_WUL = 2, AS_QXX = 3, AS_QXY = 4, AS_QYY = 5,
              AS_QX = 6, AS_QY = 7;

// Shapelet accumulators after the Sersic ones: sum W (V + u V_u + v V_v),
// sum W V_u, sum W V_v, then one per coefficient (kernels' layout), with W
// the adjoint of the sub-pixel value and V the source's value at beta.
constexpr int AH_B = 0, AH_U = 1, AH_V = 2, AH_C = 3;
constexpr int AH_SIZE = AH_C + SH_NB;

__host__ __device__ inline int n_acc(int ncomp, int n_shapelet = 0) {
    return A_SERS + A_SERS_STRIDE * ncomp + n_shapelet * AH_SIZE;
}

constexpr float RMIN2 = 1e-12f;   // radii are clamped to 1e-6 arcsec
constexpr double RMIN2D = 1e-12;

// Grid geometry of one system, passed by value to kernels.
struct Geo {
    int nx, ny, s, npix;
    double h;         // pix_scale / s
    double cx, cy;    // (s*nx - 1)/2, (s*ny - 1)/2
    float inv_s2;
};

inline Geo make_geo(const lens_model_desc& d) {
    Geo g;
    g.nx = d.nx; g.ny = d.ny; g.s = d.supersample; g.npix = d.nx * d.ny;
    g.h = (double)d.pix_scale / (double)d.supersample;
    g.cx = 0.5 * (double)(d.supersample * d.nx - 1);
    g.cy = 0.5 * (double)(d.supersample * d.ny - 1);
    g.inv_s2 = 1.0f / (float)(d.supersample * d.supersample);
    return g;
}

struct ModelInfo {
    int mass_model, n_lens_light, n_source, n_shapelet, sh_nmax, d;
};

// Model layout of a descriptor (which must be valid: see desc_valid).
inline ModelInfo model_info(const lens_model_desc& d) {
    ModelInfo mi;
    mi.mass_model = d.mass_model;
    mi.n_lens_light = d.n_lens_light;
    mi.n_source = d.n_source;
    mi.n_shapelet = d.n_shapelet;
    mi.sh_nmax = d.n_shapelet ? d.shapelet_nmax : 0;
    const int nb = d.n_shapelet ? (mi.sh_nmax + 1) * (mi.sh_nmax + 2) / 2 : 0;
    mi.d = (d.mass_model == LENS_MASS_EPL ? 8 : 7) + 7 * (d.n_lens_light + d.n_source) +
           (d.n_shapelet ? 3 + nb : 0);
    return mi;
}

__host__ __device__ inline int n_acc(const ModelInfo& mi) { return n_acc(mi.n_lens_light + mi.n_source, mi.n_shapelet); }

// Descriptor checks shared by every entry point (single system).
inline bool desc_valid(const lens_model_desc* d) {
    if (!d) return false;
    if (d->nx < 1 || d->ny < 1 || d->nx > LENS_MAX_SIDE || d->ny > LENS_MAX_SIDE) return false;
    if (!(d->pix_scale > 0.0f) || !(d->pix_scale < 3.0e38f)) return false;
    if (d->supersample < 1 || d->supersample > 16) return false;
    if (d->psf_size < 1 || d->psf_size > LENS_MAX_PSF || (d->psf_size % 2) == 0) return false;
    if (d->mass_model != LENS_MASS_SIE && d->mass_model != LENS_MASS_EPL) return false;
    if (d->n_lens_light < 0 || d->n_lens_light > LENS_MAX_LENS_LIGHT) return false;
    if (d->n_source < 0 || d->n_source > LENS_MAX_SOURCE) return false;
    if (d->n_shapelet != 0 && d->n_shapelet != 1) return false;
    if (d->n_source + d->n_shapelet < 1) return false;
    if (d->n_shapelet) {
        if (d->shapelet_nmax < 0 || d->shapelet_nmax > LENS_MAX_SHAPELET_NMAX) return false;
        if (d->n_lens_light > 1 || d->n_source > 1) return false;
    }
    return true;
}

// Launchers (lens_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_prologue(const ModelInfo& mi, int P, const float* theta, float* consts,
                           hipStream_t st);
hipError_t launch_render(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                         float* img, hipStream_t st);
// mode 0: PSF-convolve img -> out (images); 1: logL; 2: logL + adjoint image (in place)
// wflip: flipped PSF in float64 (model convolution), wpsf: PSF in float32 (adjoint).
hipError_t launch_psf(const ModelInfo& mi, const Geo& g, int K, int mode, int P,
                      const float* consts, float* img, const double* wflip, const float* wpsf,
                      const float* data, const float* invvar, float* out, float* logl,
                      double* logl64, hipStream_t st);
// img [(p K + c)][npix]: each of the K light components' images of particle p.
hipError_t launch_render_split(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                               float* img, hipStream_t st);
hipError_t launch_adjoint(const ModelInfo& mi, const Geo& g, int P, int ppt, const float* consts,
                          const float* gimg, double* partial, hipStream_t st);
// Particle p's partial rows start at row p * max(row_stride, nchunks).
hipError_t launch_finalize(const ModelInfo& mi, int P, int nchunks, const float* theta,
                           const float* consts, const double* partial, float* grad,
                           hipStream_t st, int row_stride = 0);
hipError_t launch_flip(int K, const float* psf, double* flipped, hipStream_t st);
// Tiled PSF stage (images whose whole LDS tile exceeds MAX_LDS_BYTES): modes as
// launch_psf; res [P][npix] float scratch (modes 2), chi_part [P][psf_num_tiles]
// float64 scratch (modes 1, 2).
hipError_t launch_psf_tiled(const Geo& g, int K, int mode, int P, const float* consts, float* img, float* res,
                            const double* wflip, const float* wpsf, const float* data, const float* invvar,
                            float* out, float* logl, double* logl64, double* chi_part, hipStream_t st);
int psf_num_tiles(const Geo& g);
// Sum each particle's nch partial rows into its first row (k_finalize then
// takes nchunks = 1): in row order (the direct finalize's order) ...
hipError_t launch_presum_rows(int P, int nch, int nacc, double* partial, hipStream_t st);
// ... or lane-strided with a fixed butterfly (many rows).
hipError_t launch_partial_sum(int P, int nch, int nacc, double* partial, hipStream_t st);
size_t psf_lds_bytes(const Geo& g, int K);
constexpr size_t MAX_LDS_BYTES = 160 * 1024 - 256;   // dynamic part; statics need < 256 B

// Uneven batch: per-system descriptor (device) and work items.
struct BatchSys {
    Geo g;
    int K, P, p0;            // PSF size, particles, first global particle
    int ppb, nch;            // pixels per work item, items per particle
    long long img_off;       // float offset of particle 0's image
    long long part_off;      // partial-row offset of particle 0
    const double* wflip;     // flipped PSF (float64)
    const float* wpsf;       // PSF (float32)
    const float* data;
    const float* invvar;
    int stride, rows;        // LDS tile of the PSF stage
};

struct WorkItem {
    int sys, p, chunk;       // p: particle within its system
};

hipError_t launch_batch_render(const ModelInfo& mi, int grid, const BatchSys* sys,
                               const WorkItem* items, int n_items, int* counter,
                               const float* consts, float* img, hipStream_t st);
hipError_t launch_batch_adjoint(const ModelInfo& mi, int grid, const BatchSys* sys,
                                const WorkItem* items, int n_items, int* counter,
                                const float* consts, const float* gimg, double* partial,
                                hipStream_t st);
hipError_t launch_batch_psf(int K, int n_items, const BatchSys* sys, const WorkItem* items,
                            const float* consts, float* img, float* logl, double* logl64, size_t shm, int nt,
                            hipStream_t st);
// Work-group size (256, 512 or 1024) of the PSF pass for an LDS tile of shm
// bytes over nstrips row strips; psf_strips counts the strips of an image.
int psf_threads(size_t shm, int nstrips);
int psf_strips(const Geo& g);
hipError_t launch_batch_finalize(const ModelInfo& mi, int N, const BatchSys* sys,
                                 const int* particle_sys, const float* theta, const float* consts,
                                 const double* partial, float* grad, hipStream_t st);
int batch_blocks_per_cu(const ModelInfo& mi, bool adjoint);
hipError_t launch_set_int_host(int* c, int val, hipStream_t st);
void psf_tile_dims(const Geo& g, int K, int& stride, int& rows);

inline int chunks_for(int npix, int ppt) {
    const int per_block = 256 * ppt;
    return (npix + per_block - 1) / per_block;
}

}  // namespace lens
