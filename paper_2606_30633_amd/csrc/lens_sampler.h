// Internal declarations of the inference-stage kernels (lens_sampler.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lens {

// One prior row on the device (float64): kind, (a, b) = (lo, hi) of a uniform
// or (mu, sigma) otherwise, [lo, hi] of the sigmoid map, log-density constant.
struct PriorRow {
    double kind, a, b, lo, hi, cst, pad0, pad1;
};

struct AdamHyper {
    float lr, decay, beta1, beta2, eps;
};

// Pointers and scalars of one HMC run (device pointers).
struct HmcArgs {
    float* u;          // [C][d] position
    float* grad;       // [C][d] dlogp/du at u
    double* logp;      // [C]
    float* u0;         // [C][d] saved start of the transition
    float* g0;         // [C][d]
    double* logp0;     // [C]
    float* p;          // [C][d] momentum
    double* h0;        // [C] initial energy
    const float* inv_mass;   // [d]
    float* samples;    // [T][C][d] or null
    int* accepts;      // [C] or null
    const int* tcount; // transitions done in this run
    uint64_t seed;
    const unsigned long long* transition0;   // index of this run's first transition (device memory)
    float eps;
    const float* eps_dev;   // if set: the step size, read on the device (adaptive runs)
    double* accprob;        // [C] or null: min(1, exp(H0 - H1)) of each chain's transition
};

// Burn-in adaptation: dual-averaged shared step size (Hoffman & Gelman 2014)
// and per-chain Welford sums of the positions over a window of transitions.
struct AdaptArgs {
    double* state;          // [0] mu, [1] log eps, [2] log eps_bar, [3] H_bar, [4] m
    const double* accprob;  // [C]
    float* eps_dev;         // the step size of the next transition
    float* eps_trace;       // [T] or null: the step size each transition used
    float* eps_final;       // or null: exp(log eps_bar) after the last update
    const int* tcount;      // transitions done in this run
    float delta;            // target acceptance
};

// SVI: surrogate draws, ELBO + pathwise gradient, optimizer step.
constexpr int SVI_MAX_D = 50;                 // 8 + 7 * (3 lens-light + 3 source components)
constexpr double SVI_DIAG_SHIFT = 1e-10;
constexpr uint32_t SVI_RNG_TAG = 1u;          // counter word 3 (HMC draws use 0)
constexpr int SVI_OPT_ADAM = 0, SVI_OPT_ADABELIEF = 1;

inline int svi_num_params(int d) { return d + d * (d + 1) / 2; }

struct SviArgs {
    float* phi;            // [np] surrogate parameters (updated in place if update)
    float* m;              // [np] first moment
    float* s;              // [np] second moment
    float* u;              // [n][d] sample points
    double* eps;           // [d][n] standard normals
    double* logq;          // [n]
    const double* logp;    // [n] target at u
    const float* grad_u;   // [n][d] dlogp/du at u
    float* grad_phi;       // [np] or null
    double* elbo;          // ELBO output (indexed by *call_step) or null
    const int* step;       // SVI step: Philox counter word 1; bias correction uses step + 1
    const int* call_step;  // index into elbo, or null for index 0
    uint64_t seed;
    uint64_t frozen;       // bit j: coordinate j is not a parameter; mu_j and L's row and column j stay fixed
    int n, d;
    int update, optimizer;
    float lr, beta1, beta2, eps_opt;
};

// Observed image of one system of a batch (device pointer) for k_center_views.
struct ViewSrc {
    const float* data;
    int nx, ny;
};

// Host: validated prior table [d][5] (kind, a, b, c, d) -> device rows.
// Returns false on an unknown kind or an empty support.
bool build_prior_rows(int d, const float* h_table, PriorRow* rows);

hipError_t launch_bijection(int P, int d, const PriorRow* table, const float* u, float* theta,
                            hipStream_t st);
// A set of parameter indices 0..127 (the largest model, EPL with one lens
// light, one Sersic source and an n_max = 8 shapelet source, has 70).
constexpr int PARAM_MASK_BITS = 128;
struct ParamMask {
    uint64_t w[2] = {0, 0};
    __host__ __device__ bool test(int j) const { return (w[j >> 6] >> (j & 63)) & 1u; }
    __host__ void set(int j) { w[j >> 6] |= (uint64_t)1 << (j & 63); }
};

// skip: j in skip -> entry j is not a parameter (no prior or Jacobian term, gradient 0).
// One wave per particle (parameters over the lanes); the log-prior and
// log-Jacobian sums run in parameter order.  d <= PARAM_MASK_BITS.
hipError_t launch_posterior(int P, int d, const PriorRow* table, const float* u, const double* logl,
                            const float* gtheta, int with_jac, double* logp, float* grad_u,
                            hipStream_t st, const ParamMask& skip = ParamMask{});
hipError_t launch_adam(int P, int d, const float* grad_u, const double* logp, float* u, float* m,
                       float* v, const int* step, const AdamHyper& hp, float* loss,
                       hipStream_t st);
hipError_t launch_add_int(int* c, int inc, hipStream_t st);
hipError_t launch_set_int(int* c, int val, hipStream_t st);
// *c = val (a kernel, so that a captured graph can read values set between replays)
hipError_t launch_set_u64(unsigned long long* c, unsigned long long val, hipStream_t st);
hipError_t launch_hmc_begin(int C, int d, const HmcArgs& a, hipStream_t st);
hipError_t launch_hmc_kick_drift(int C, int d, const HmcArgs& a, hipStream_t st);
hipError_t launch_hmc_end(int C, int d, const HmcArgs& a, hipStream_t st);
hipError_t launch_hmc_adapt_init(int C, int d, double* state, float* eps_dev, float eps0, double* wmean, double* wm2,
                                 int* wcount, hipStream_t st);
hipError_t launch_hmc_adapt(int C, const AdaptArgs& a, hipStream_t st);
hipError_t launch_hmc_welford(int C, int d, const float* u, const int* tcount, int window_start, double* wmean,
                              double* wm2, int* wcount, hipStream_t st);
hipError_t launch_hmc_window_var(int C, int d, const double* wmean, const double* wm2, const int* wcount, float* var,
                                 hipStream_t st);

hipError_t launch_svi_draw(const SviArgs& a, hipStream_t st);
hipError_t launch_svi_reduce(const SviArgs& a, hipStream_t st);
hipError_t launch_svi_moments(int d, const float* phi, float* mean, float* cov, float* var, hipStream_t st);

hipError_t launch_inverse_bijection(int P, int d, const PriorRow* table, const float* theta, float* u,
                                    hipStream_t st);
hipError_t launch_segment_argmin(int S, const int* p0, const float* val, float* best, int* arg,
                                 hipStream_t st);
hipError_t launch_center_views(int S, int side, const ViewSrc* src, float* out, hipStream_t st);

}  // namespace lens
