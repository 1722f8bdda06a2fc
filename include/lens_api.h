/*
 * lens_api.h -- C ABI of the batched strong-lens likelihood library (liblens.so).
 *
 * The library evaluates, for many parameter vectors ("particles" or "chains")
 * of one lens system at once, the forward model of the paper's Sec. 3
 * (elliptical power-law or SIE mass + external shear, elliptical Sersic lens
 * light and sources, a supersampled pixel grid as in the Sec. 4.2 footnote),
 * downsampling, PSF convolution and a Gaussian log-likelihood, together with
 * the gradient of the log-likelihood with respect to every parameter.  On
 * top of that it runs the paper's multi-start MAP stage (Sec. 3: gradient
 * descent with Adam, every particle independent, Sec. 3.1) and HMC
 * transitions (Sec. 3: HMC; Sec. 3.1: independent chains).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers owned by the caller; h_* are host
 *    pointers, read during the call only.  The library never frees caller
 *    memory and never keeps caller pointers beyond a call, except the
 *    system arrays handed to lens_plan_create (PSF, data, inverse variance),
 *    which must stay valid and unchanged while the plan lives.
 *  - Every compute call is asynchronous on the given stream (a hipStream_t
 *    passed as void*; NULL is the default stream).  Launch errors are
 *    returned as LENS_EHIP; faults inside kernels surface at the caller's
 *    next synchronisation.
 *  - Arrays are row-major float32.  Parameters are [P][d] in the canonical
 *    order (see lens_num_params); images are [P][ny][nx], row = y.
 *  - Results are bitwise deterministic for a given plan and launch shape:
 *    no floating-point atomics; reductions run in a fixed order.
 *  - A particle whose parameters are not all finite gets logL = NaN and a
 *    NaN gradient.  A particle with an ellipticity |e| >= 1 on any
 *    component has no valid profile: logL = -inf and gradient 0.
 *  - Functions return a lens_status and never throw.
 *  - Plans, batch plans and networks own scratch buffers that every call on
 *    them uses: calls on one object must be ordered (one stream, or
 *    synchronise between streams); distinct objects may run concurrently.
 *    An object is used from one host thread at a time.
 *
 * Canonical parameter order (d = n_mass + 7 * (n_lens_light + n_source)
 * + n_shapelet * (3 + nb)):
 *   mass   : theta_E ["], [gamma (EPL only)], e1, e2, x ["], y ["]
 *   shear  : g1, g2                                      (n_mass = 7 | 8)
 *   Sersic : R_e ["], n, e1, e2, x ["], y ["], I_e       per component,
 *            lens-light components first, then sources.
 *   shapelet source (optional): beta ["], x ["], y ["], c_0 .. c_{nb-1},
 *            nb = (n_max + 1)(n_max + 2)/2 coefficients of the Cartesian
 *            basis phi_{n1}(x - x_c; beta) phi_{n2}(y - y_c; beta),
 *            phi_n(u; beta) = [2^n sqrt(pi) n! beta]^(-1/2) H_n(u/beta)
 *            exp(-u^2 / (2 beta^2)) (Refregier 2003), ordered by
 *            n = n1 + n2, then n2 (coefficient k <-> (n - n2, n2)).
 */
#ifndef LENS_API_H
#define LENS_API_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lens_status;
#define LENS_OK            0
#define LENS_EINVAL       -1   /* bad argument (NULL pointer, size, descriptor) */
#define LENS_EUNSUPPORTED -2   /* valid request outside what the library builds */
#define LENS_EHIP         -3   /* a HIP runtime call or kernel launch failed */
#define LENS_ENOMEM       -4   /* device or host allocation failed */
#define LENS_ESCRATCH     -5   /* request larger than the fixed scratch of lens_loglike_grad_noalloc */

#define LENS_MASS_SIE 0        /* singular isothermal ellipsoid (gamma = 2) */
#define LENS_MASS_EPL 1        /* elliptical power law, free slope gamma */

#define LENS_MAX_LENS_LIGHT 3
#define LENS_MAX_SOURCE     3
#define LENS_MAX_SHAPELET_NMAX 8   /* shapelet order: up to 45 coefficients */
#define LENS_MAX_PSF       31
#define LENS_MAX_SIDE    2048

/* Geometry and composition of one lens system (Sec. 3 model components).
 * Sub-pixel (a, b) of pixel (i, j) sits at
 *   x = (s*j + b - (s*nx - 1)/2) * pix_scale / s,
 *   y = (s*i + a - (s*ny - 1)/2) * pix_scale / s          (arcsec).      */
typedef struct lens_model_desc {
    int32_t nx, ny;         /* image size in pixels, 1..LENS_MAX_SIDE */
    float   pix_scale;      /* arcsec per pixel, > 0 */
    int32_t supersample;    /* s >= 1: s x s sub-pixels per pixel, averaged */
    int32_t psf_size;       /* odd K, 1..LENS_MAX_PSF; PSF centre at (K-1)/2 */
    int32_t mass_model;     /* LENS_MASS_SIE | LENS_MASS_EPL (+ external shear) */
    int32_t n_lens_light;   /* 0..LENS_MAX_LENS_LIGHT Sersic components at theta */
    int32_t n_source;       /* 0..LENS_MAX_SOURCE Sersic components at beta */
    int32_t n_shapelet;     /* 0 or 1 shapelet source at beta (Sec. 3: Sersic profiles
                               and/or shapelets for the source light); at least one
                               source in all: n_source + n_shapelet >= 1.  With a
                               shapelet source, n_lens_light and n_source are 0 or 1. */
    int32_t shapelet_nmax;  /* its order n_max, 0..LENS_MAX_SHAPELET_NMAX (ignored
                               without a shapelet source) */
} lens_model_desc;

typedef struct lens_plan lens_plan;   /* opaque; owns device scratch */

/* Human-readable text of a status code (static storage). */
const char* lens_status_string(lens_status s);

/* Number of parameters d of a model, or -1 if the descriptor is invalid. */
int32_t lens_num_params(const lens_model_desc* desc);

/* Create a plan for one system and up to max_particles particles per call.
 *   d_psf    [K][K]   PSF, used as given (normally normalised to sum 1);
 *                     convolution is m = sum_{u,v} P[u][v] img[i-u+h][j-v+h],
 *                     zero outside the image, h = (K-1)/2.
 *   d_data   [ny][nx] observed image d.
 *   d_invvar [ny][nx] inverse variance w = 1/sigma^2 per pixel (>= 0).
 * The plan copies desc, allocates its device scratch (proportional to
 * max_particles * nx * ny) and keeps the three device pointers.
 * Cutout size (Sec. 2: O(10^4) pixels for galaxy-scale HST cutouts, O(10^6)
 * for a cluster-scale lens): when one particle's image with its (K-1)/2 halo
 * fits a work-group's LDS (up to about 180 x 180 px) the PSF stage convolves
 * whole images; larger images (up to LENS_MAX_SIDE per side) are convolved
 * by 32 x 128-pixel tiles with halos, with chi^2 reduced per tile and then
 * over the tiles in a fixed order; such plans hold two more buffers, the
 * residual [max_particles][ny][nx] (float) and the tile partials.
 * Errors: LENS_EINVAL for a bad descriptor/pointer, LENS_ENOMEM. */
lens_status lens_plan_create(const lens_model_desc* desc, const float* d_psf,
                             const float* d_data, const float* d_invvar,
                             int32_t max_particles, lens_plan** out);
lens_status lens_plan_destroy(lens_plan* plan);

/* Tuning knob of the sub-pixel kernels: pixels handled per thread of one
 * work-group (1..64).  Changes only the launch shape, never the result
 * beyond float rounding of the reductions. */
lens_status lens_plan_set_pixels_per_thread(lens_plan* plan, int32_t ppt);

/* Forward model (Sec. 3): PSF-convolved, downsampled model images.
 *   d_theta [P][d] in, d_images [P][ny][nx] out.  1 <= P <= max_particles. */
lens_status lens_forward(lens_plan* plan, int32_t P, const float* d_theta,
                         float* d_images, void* stream);

/* Gaussian log-likelihood logL = -1/2 sum_pix w (d - m)^2 per particle
 * (the constant -1/2 sum log(2 pi / w) is not included).
 *   d_theta [P][d] in, d_logl [P] out. */
lens_status lens_loglike(lens_plan* plan, int32_t P, const float* d_theta,
                         float* d_logl, void* stream);

/* logL and its gradient dlogL/dtheta by a hand-written adjoint.
 *   d_theta [P][d] in; d_logl [P] out; d_grad [P][d] out;
 *   d_logl64 [P] out, optional (NULL): logL accumulated in float64. */
lens_status lens_loglike_grad(lens_plan* plan, int32_t P, const float* d_theta,
                              float* d_logl, float* d_grad, double* d_logl64,
                              void* stream);

/* Allocation-free logL + gradient, for callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops, and
 * harnesses that forbid hipMalloc.  It computes what lens_loglike_grad
 * computes on a plan with the default 4 pixels per thread (same kernels,
 * same launch shape, hence bit-identical results), without a plan: the
 * caller passes the system arrays and the descriptor on every call.
 *   desc, d_psf [K][K], d_data [ny][nx], d_invvar [ny][nx]: as for
 *   lens_plan_create (read during the call only);
 *   d_theta [P][d] in; d_logl [P], d_grad [P][d] out; d_logl64 [P] out,
 *   optional (NULL).
 * Scratch: one static device array of LENS_NOALLOC_SCRATCH_BYTES on each
 * GPU the call runs on, reserved from library load until the process ends;
 * its device address is looked up once per device on the first call there.
 * One call needs, each part rounded up to 256 bytes,
 *   8 K^2 + 4 * 832 P + 4 nx ny P + 8 P ceil(nx ny / 1024) (11 + 8 n_comp + 48 n_shapelet)
 * bytes, n_comp = n_lens_light + n_source: about 46.1 KB per particle at
 * 100 x 100 px with three Sersic components, so up to ~1450 particles per
 * call there (split larger batches into several calls).
 * Every call on one GPU uses the same array and leaves the last call's
 * contents in it: calls that overlap on one GPU (two streams, or two host
 * threads, without ordering) race and give wrong results; order them.
 * Every scratch word a kernel reads is written earlier in the same call,
 * so no clearing is needed.  No hipMalloc, hipFree or other allocating
 * call is made.
 * Errors: LENS_EINVAL (bad descriptor, NULL pointer, P < 1),
 * LENS_EUNSUPPORTED (image + PSF tile beyond the LDS), LENS_ESCRATCH
 * (the call needs more than LENS_NOALLOC_SCRATCH_BYTES; nothing is launched),
 * LENS_EHIP. */
#define LENS_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
lens_status lens_loglike_grad_noalloc(const lens_model_desc* desc, const float* d_psf,
                                      const float* d_data, const float* d_invvar, int32_t P,
                                      const float* d_theta, float* d_logl, float* d_grad,
                                      double* d_logl64, void* stream);

/* Backward modelling (Sec. 3: the lens and source intensities solved by
 * linear inversion instead of sampled).  For each particle the K =
 * n_lens_light + n_source + nb linear amplitudes (the Sersic intensities,
 * then the nb shapelet coefficients, at most 51 in all) are set to the
 * weighted least-squares solution A of the normal equations M A = b,
 * M_kl = sum w B_k B_l, b_k = sum w B_k d, with B_k the model image of
 * component k at unit intensity (Cholesky in component order; a component
 * whose pivot is <= 1e-12 x max_k M_kk, i.e. no flux in the cutout or an
 * image that is a combination of the earlier components', gets A_k = 0).
 * logL and its gradient are those at the solved intensities; the gradient is
 * with respect to the nonlinear parameters (envelope theorem), its intensity
 * entries are 0.
 *   d_theta [P][d] in (intensity entries ignored); d_logl [P], d_grad [P][d]
 *   out; d_amp [P][K] out, optional: the solved intensities (NaN for a
 *   particle with an invalid ellipticity, whose logL is -inf).
 * Requires P * K <= max_particles (the K component images of every
 * particle are held together in the plan's image buffers).  Allocates its
 * scratch (two parameter arrays and one model-image array of max_particles
 * rows) on first use.
 * Errors: LENS_EINVAL for P * K above max_particles. */
lens_status lens_loglike_grad_backward(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                                       float* d_grad, float* d_amp, void* stream);

/* Backward modelling in the inference stages (the paper models its real
 * system this way, App. B).  With enable != 0 the plan's posterior path
 * (lens_logpost_grad, lens_map_adam, lens_hmc_run, lens_hmc_adapt and the
 * SVI calls) uses the backward likelihood above; the intensity entries of u
 * are not parameters: they add no prior or Jacobian term and their gradient
 * is 0 (Adam leaves them where they are; for HMC give them a zero inverse
 * mass, which freezes a coordinate; SVI holds mu_j and the whole row and
 * column j of L fixed for them, since nothing would bound the surrogate's
 * width there).  Those calls then require P * K <= max_particles (n draws
 * for SVI).  Allocates the backward scratch when enabled; captured graphs
 * are dropped.  Not callable during capture.
 * Errors: LENS_EINVAL for a model without light components. */
lens_status lens_plan_set_backward(lens_plan* plan, int32_t enable);

/* ---------------------------------------------------------------------------
 * Prior and bijection to the unconstrained space (Sec. 3.1: the tilde
 * quantities are the parameters mapped to an unconstrained space; Sec. 4.2,
 * eq. sim-dist: uniform, normal, log-normal and truncated-normal priors).
 * Per parameter j, theta_j = T_j(u_j):
 *   LENS_PRIOR_UNIFORM     (a, b): theta = a + (b - a) sigmoid(u)
 *   LENS_PRIOR_TRUNCNORMAL (mu, sigma, lo, hi): theta = lo + (hi - lo) sigmoid(u),
 *                          density N(mu, sigma) restricted to [lo, hi]
 *   LENS_PRIOR_NORMAL      (mu, sigma): theta = u
 *   LENS_PRIOR_LOGNORMAL   (mu, sigma): log theta ~ N(mu, sigma), theta = exp(u)
 * The log prior is the sum of the per-parameter log densities of theta.
 * ------------------------------------------------------------------------- */
#define LENS_PRIOR_UNIFORM     0
#define LENS_PRIOR_NORMAL      1
#define LENS_PRIOR_LOGNORMAL   2
#define LENS_PRIOR_TRUNCNORMAL 3

/* Set the plan's prior.  h_table [d][5] host floats, row = (kind, a, b, c, d)
 * with the arguments above (unused entries ignored).  Copied to the device.
 * Errors: LENS_EINVAL for an unknown kind, sigma <= 0, or an empty interval. */
lens_status lens_plan_set_prior(lens_plan* plan, const float* h_table);

/* Log posterior in the unconstrained space and its gradient:
 *   logp(u) = logL(T(u)) + log prior(T(u)) [+ log|dT/du| if with_jacobian]
 *   d_u [P][d] in; d_logp [P] out (float64); d_grad [P][d] out = dlogp/du;
 *   d_theta [P][d] out, optional: T(u) rounded to float32 (the point at
 *   which the likelihood is evaluated).
 * The MAP objective omits the Jacobian (its optimum is the MAP of theta);
 * the HMC target includes it.  Requires lens_plan_set_prior. */
lens_status lens_logpost_grad(lens_plan* plan, int32_t P, const float* d_u,
                              int32_t with_jacobian, float* d_theta, double* d_logp,
                              float* d_grad, void* stream);

/* u = T^-1(theta) for starting points given in the constrained space
 * (d_theta, d_u [P][d]).  Bounded parameters are clamped to the logit of
 * [2^-24, 1 - 2^-24] of their support; log-normal ones to theta >= 1e-30.
 * Requires lens_plan_set_prior. */
lens_status lens_to_unconstrained(lens_plan* plan, int32_t P, const float* d_theta, float* d_u,
                                  void* stream);

/* HIP graphs.  The iterative calls below (lens_map_adam, lens_hmc_run,
 * lens_hmc_adapt, lens_svi_run, lens_batch_map_adam, lens_batch_loglike_grad)
 * take a use_graph flag instead of explicit graph handles: with use_graph != 0
 * the plan captures one step (one transition, one SVI step) on its own stream
 * into a graph it owns, instantiates it, and replays it on the caller's stream
 * once per step.  The graph is kept across calls and re-captured only when its
 * key changes: the particle count, every device pointer the step touches, the
 * hyper-parameters baked into kernel arguments (learning rate, decay, betas,
 * eps, step size, leapfrog count, seed, window start, target acceptance) and
 * the launch tiles.  Values that change from step to step or call to call
 * live in plan-owned device memory that the kernels read, written by small
 * kernels outside the graph before the replays: the Adam / SVI step counters,
 * the HMC transition counter and the index of a run's first transition
 * (transition0), the adapted step size.  A caller that keeps its buffers and
 * hyper-parameters fixed therefore replays one instantiated graph for a whole
 * run.  Captured graphs are dropped by lens_plan_set_backward and destroyed
 * with the plan.  Timing (lens_plan_enable_timing) records no events inside
 * replayed graphs. */

/* Multi-start MAP (Sec. 3, Sec. 3.1: every particle descends independently;
 * Sec. 3.2: Adam for MAP).  Runs n_steps Adam updates (Kingma & Ba 2015,
 * bias-corrected) of loss(u) = -(logL + log prior)(T(u)) on all P particles.
 *   d_u [P][d] in/out; d_m, d_v [P][d] in/out Adam moments (zero to start);
 *   d_loss [P] out: the loss at the last evaluated point (before the last
 *   update).  The step counter (1-based, for the bias correction and the
 *   learning-rate schedule lr_k = lr * decay^(k-1)) lives in the plan:
 *   lens_map_reset restarts it.  use_graph != 0 captures one step into a HIP
 *   graph on first use and replays it (the graph is re-captured when P or
 *   any pointer or hyper-parameter changes). */
lens_status lens_map_reset(lens_plan* plan);
lens_status lens_map_adam(lens_plan* plan, int32_t P, float* d_u, float* d_m, float* d_v,
                          int32_t n_steps, float lr, float decay, float beta1, float beta2,
                          float eps, float* d_loss, int32_t use_graph, void* stream);

/* HMC transitions (Sec. 3: HMC; Sec. 3.1: independent chains per GPU),
 * target logp(u) with the Jacobian, diagonal mass matrix.  One transition:
 * momenta p ~ N(0, M) from Philox4x32-10 (Salmon et al. 2011) with key =
 * seed and counter = (chain, transition, block, 0), Box-Muller in float64;
 * n_leapfrog steps of half kick / drift / half kick with step size eps;
 * energy H = -logp + p^T M^-1 p / 2 in float64; Metropolis accept with the
 * uniform from counter block ceil(d/4).
 *   d_u [C][d], d_grad [C][d] (= dlogp/du), d_logp [C] (float64): the chain
 *   state, in/out; must be consistent on entry (lens_logpost_grad with
 *   with_jacobian = 1).  d_inv_mass [d]: M^-1 diagonal (an entry of 0
 *   freezes that coordinate: no momentum, no motion).
 *   d_samples [n_transitions][C][d] out, optional; d_accepts [C] in/out,
 *   optional: incremented on every accepted transition.
 *   transition0: index of the first transition (counter word 1); successive
 *   transitions use transition0 + 1, ...  use_graph as for lens_map_adam. */
lens_status lens_hmc_run(lens_plan* plan, int32_t C, float* d_u, float* d_grad, double* d_logp,
                         const float* d_inv_mass, float eps, int32_t n_leapfrog,
                         int32_t n_transitions, uint64_t seed, uint64_t transition0,
                         float* d_samples, int32_t* d_accepts, int32_t use_graph, void* stream);

/* HMC burn-in with adaptation: the transitions of lens_hmc_run, with
 *  - one step size shared by all chains, adapted after every transition by
 *    dual averaging (Hoffman & Gelman 2014, Sec. 3.2.1: mu = log(10 eps0),
 *    gamma 0.05, t0 10, kappa 0.75) towards a chain-mean acceptance
 *    statistic min(1, exp(H0 - H1)) of target_accept;
 *  - the mass-matrix fit of Sec. 3.3: the variance of the positions over
 *    the transitions t >= window_start (all chains, ddof 1), from per-chain
 *    Welford sums combined in a fixed order.
 * Transition t (0-based in this call) uses Philox counter word 1 =
 * transition0 + t, like lens_hmc_run.  The step-size state, the window sums
 * and the counters restart at every call.
 *   d_u, d_grad, d_logp: chain state in/out as for lens_hmc_run;
 *   d_inv_mass [d]: the inverse mass matrix used during this burn-in;
 *   d_eps_trace [n_transitions] out, optional: the step size of each transition;
 *   d_eps_final [1] out, optional: the adapted step size exp(log eps_bar);
 *   d_var [d] out, optional: the window variances (the next inverse mass
 *   matrix; NaN if the window holds fewer than 2 samples).
 * use_graph as for lens_map_adam (eps0 is not part of the captured graph).
 * Allocates its state (2 x max_particles x d doubles) on first use.
 * Errors: LENS_EINVAL for target_accept outside (0, 1) or eps0 <= 0. */
lens_status lens_hmc_adapt(lens_plan* plan, int32_t C, float* d_u, float* d_grad, double* d_logp,
                           const float* d_inv_mass, float eps0, float target_accept, int32_t n_leapfrog,
                           int32_t n_transitions, int32_t window_start, uint64_t seed, uint64_t transition0,
                           float* d_eps_trace, float* d_eps_final, float* d_var, int32_t use_graph, void* stream);

/* ---------------------------------------------------------------------------
 * Stochastic variational inference (Sec. 3: eq. vi, eq. elbo, eq. elbo-grad;
 * Sec. 3.2: AdaBelief as the SVI optimizer).  The surrogate is a Gaussian
 * q(u) = N(mu, L L^T) over the unconstrained parameters u, fitted to the
 * HMC target logp(u) (with the bijection's Jacobian) by minimising the
 * Monte-Carlo ELBO = mean_i [log q(u_i) - logp(u_i)] over n draws
 * u_i = mu + L eps_i.
 *
 * Surrogate parameters phi (float32, length lens_svi_num_params(d) =
 * d + d(d+1)/2): mu, then the lower triangle of L row by row; a diagonal
 * entry holds rho with L_jj = softplus(rho) + 1e-10 (a guard against underflow
 * only: conditional posterior widths reach ~4e-6 on a 100x100 system).
 *
 * eps_i: Philox4x32-10 with key = seed and counters (i, step, block, 1),
 * Box-Muller in float64 (the HMC draws use counter word 3 = 0, so the two
 * streams never meet).  The ELBO gradient is the reparameterised (pathwise)
 * estimator: the derivative of the sample mean with the eps_i held fixed,
 * reduced over the draws in float64 in a fixed order (deterministic).
 * A draw whose target is not finite (an ellipticity |e| >= 1) contributes a
 * zero gradient and makes the ELBO +inf.
 *
 * Plan scratch: draws, their normals and log q for up to max_particles draws;
 * the target reuses the plan's posterior buffers.  Requires
 * lens_plan_set_prior and d <= 50.
 * ------------------------------------------------------------------------- */
#define LENS_OPT_ADAM      0   /* Kingma & Ba 2015 */
#define LENS_OPT_ADABELIEF 1   /* Zhuang et al. 2020 */

/* d + d(d+1)/2, or -1 for d outside [1, 50]. */
int32_t lens_svi_num_params(int32_t d);

/* Restart the plan's SVI step counter (draws and bias correction) at 0. */
lens_status lens_svi_reset(lens_plan* plan);

/* ELBO estimate and its gradient at phi, draws of step `step`, no update.
 *   d_phi [np] in; d_elbo [1] out (float64); d_grad_phi [np] out, optional;
 *   d_u [n][d] out, optional: the draws u_i (float32, the points at which
 *   the target is evaluated). */
lens_status lens_svi_elbo_grad(lens_plan* plan, int32_t n, const float* d_phi, uint64_t seed,
                               int32_t step, double* d_elbo, float* d_grad_phi, float* d_u,
                               void* stream);

/* n_steps SVI iterations with n draws each.  Step k (the plan's counter,
 * from lens_svi_reset) draws with counter word 1 = k and applies one Adam
 * or AdaBelief update with bias corrections 1 - beta^(k+1):
 *   Adam:      m = b1 m + (1-b1) g;  s = b2 s + (1-b2) g^2
 *   AdaBelief: m = b1 m + (1-b1) g;  s = b2 s + (1-b2) (g-m)^2 + eps
 *   phi -= lr m^ / (sqrt(s^) + eps)
 *   d_phi, d_m, d_s [np] in/out (moments zero to start); d_elbo [n_steps]
 *   out, optional: the ELBO of each step, at phi before its update.
 *   The paper's SVI setting: AdaBelief, lr 1e-4, beta1 0.95, beta2 0.99;
 *   eps must be > 0 (1e-16 is AdaBelief's usual value).
 *   use_graph as for lens_map_adam.
 * Errors: LENS_EINVAL for an unknown optimizer or hyper-parameters out of
 * range. */
lens_status lens_svi_run(lens_plan* plan, int32_t n, float* d_phi, float* d_m, float* d_s,
                         int32_t n_steps, int32_t optimizer, float lr, float beta1, float beta2,
                         float eps, uint64_t seed, double* d_elbo, int32_t use_graph, void* stream);

/* Surrogate moments: d_mean [d] = mu, d_cov [d][d] = L L^T, d_var [d] its
 * diagonal (e.g. the inverse mass matrix of HMC); each optional. */
lens_status lens_svi_moments(int32_t d, const float* d_phi, float* d_mean, float* d_cov, float* d_var,
                             void* stream);

/* ---------------------------------------------------------------------------
 * Uneven batch: many lens systems of different image size, supersampling and
 * PSF size, each with its own particles, evaluated together (the paper models
 * samples of many systems, Sec. 4.2; this is the one-GPU form of that
 * workload).  All systems share the model composition (mass model and the
 * numbers of Sersic components), hence d.
 *
 * The render and adjoint stages each run as ONE persistent launch: work-groups
 * take (system, particle, pixel-chunk) items from a list sorted by cost
 * (largest first) through an integer atomic counter; the PSF stage runs one
 * launch per distinct PSF size.  The pixel-chunk size per system ("tile",
 * pixels per thread) is chosen by lens_batch_autotune.
 * ------------------------------------------------------------------------- */
typedef struct lens_batch_plan lens_batch_plan;

/* h_descs [S] host; h_psf, h_data, h_invvar [S] host arrays of DEVICE pointers
 * (same meaning and lifetime rules as lens_plan_create); h_particles [S]
 * particles per system (>= 1).  Parameters, logL and gradients of a batch
 * call are packed by system in order: system k's particles occupy rows
 * [sum_{j<k} P_j, sum_{j<=k} P_j).
 * Errors: LENS_EINVAL, LENS_EUNSUPPORTED (different model compositions, or an
 * image + PSF tile that does not fit the 160 KB LDS), LENS_ENOMEM. */
lens_status lens_batch_plan_create(int32_t S, const lens_model_desc* h_descs,
                                   const float* const* h_psf, const float* const* h_data,
                                   const float* const* h_invvar, const int32_t* h_particles,
                                   lens_batch_plan** out);
lens_status lens_batch_plan_destroy(lens_batch_plan* plan);
/* Current total particle count N (the sum of the current per-system counts). */
int64_t lens_batch_total_particles(const lens_batch_plan* plan);

/* Per-call particle counts (Sec. 4.2: each system carries its own number of
 * particles).  h_particles [S] host, 1 <= h_particles[k] <= the count given
 * to lens_batch_plan_create for system k (the buffers' capacity).  Later
 * calls pack parameters, logL and gradients by the new counts, as described
 * at lens_batch_plan_create; the work list and PSF launch classes are rebuilt
 * on the host (synchronous: waits for the device), and every captured graph
 * of the plan is re-captured on its next use.  The Adam step counter of
 * lens_batch_map_adam is kept.  Equal counts return at once.
 * Errors: LENS_EINVAL (NULL, or a count out of range), LENS_ENOMEM, LENS_EHIP. */
lens_status lens_batch_set_particles(lens_batch_plan* plan, const int32_t* h_particles);
lens_status lens_batch_get_particles(const lens_batch_plan* plan, int32_t* h_particles);

/* The same per-call form in one call: lens_batch_set_particles(h_particles)
 * then lens_batch_loglike_grad; d_theta [N][d], N = sum of h_particles.
 * Errors: those of the two calls. */
lens_status lens_batch_loglike_grad_counts(lens_batch_plan* plan, const int32_t* h_particles,
                                           const float* d_theta, float* d_logl, float* d_grad,
                                           int32_t use_graph, void* stream);

/* logL and dlogL/dtheta for every particle of every system.
 *   d_theta [N][d] in, d_logl [N] out, d_grad [N][d] out, N = total particles.
 * use_graph != 0: the whole sequence is captured into a HIP graph on first
 * use and replayed (re-captured when a pointer or the tiles change). */
lens_status lens_batch_loglike_grad(lens_batch_plan* plan, const float* d_theta, float* d_logl,
                                    float* d_grad, int32_t use_graph, void* stream);

/* Tiles: pixels per thread of a work item, per system (1..64). */
lens_status lens_batch_get_tiles(const lens_batch_plan* plan, int32_t* h_ppt);
lens_status lens_batch_set_tiles(lens_batch_plan* plan, const int32_t* h_ppt);

/* Autotuner: groups the systems into size classes (supersampling x image-side
 * bucket), tries tiles {1, 2, 4, 8} per class by coordinate descent, then the
 * work-group size {256, 512, 1024} of each PSF launch (one per PSF size and
 * LDS tile class), timing full batch calls on d_theta with HIP events, and
 * keeps the fastest.  If cache_path is not NULL, a cached choice for the same
 * batch geometry (image sizes, PSF sizes and particle counts) is used without
 * timing, and a new choice is written there (JSON: the tile of each system,
 * then the work-group size of each PSF launch).  Synchronous. */
lens_status lens_batch_autotune(lens_batch_plan* plan, const float* d_theta, const char* cache_path,
                                void* stream);

/* Inference stage over the whole batch (Sec. 3: multi-start MAP; Sec. 4.2:
 * many systems modelled together).  One prior, set as for a single plan
 * (lens_plan_set_prior), serves every system.  Arrays are packed as for
 * lens_batch_loglike_grad: d_u, d_m, d_v, d_grad, d_theta [N][d];
 * d_logp [N] float64; d_loss [N].  Semantics per particle are those of
 * lens_logpost_grad and lens_map_adam; the Adam step counter lives in the
 * batch plan (lens_batch_map_reset restarts it).  use_graph as for
 * lens_batch_loglike_grad.  Errors: LENS_EINVAL (NULL pointer, no prior,
 * invalid hyper-parameter), LENS_EHIP. */
lens_status lens_batch_set_prior(lens_batch_plan* plan, const float* h_table);
lens_status lens_batch_logpost_grad(lens_batch_plan* plan, const float* d_u, int32_t with_jacobian,
                                    float* d_theta, double* d_logp, float* d_grad, void* stream);
lens_status lens_batch_to_unconstrained(lens_batch_plan* plan, const float* d_theta, float* d_u,
                                        void* stream);
lens_status lens_batch_map_reset(lens_batch_plan* plan);
lens_status lens_batch_map_adam(lens_batch_plan* plan, float* d_u, float* d_m, float* d_v,
                                int32_t n_steps, float lr, float decay, float beta1, float beta2,
                                float eps, float* d_loss, int32_t use_graph, void* stream);

/* Best particle of every system (the multi-start MAP estimate is the best
 * particle, Sec. 3): d_best [S] = min over system k's particles of d_val
 * [N] (NaN counts as +inf), d_arg [S] = its global row (first on ties). */
lens_status lens_batch_argmin(lens_batch_plan* plan, const float* d_val, float* d_best,
                              int32_t* d_arg, void* stream);

/* d_out [S][side][side]: each system's observed image on a centred
 * side x side grid of the same pixel scale (pixel (i, j) takes source row
 * i + (ny - side) / 2 and column j + (nx - side) / 2; a half-integer offset
 * averages the two neighbours; outside the image, zero).  This is the
 * learned initializer's view of a system (side = 64).  1 <= side <= 256. */
lens_status lens_batch_center_views(lens_batch_plan* plan, int32_t side, float* d_out, void* stream);

/* ---------------------------------------------------------------------------
 * Learned initializer.  A convolutional network regresses, from a 64x64
 * image of a system, 14 lens parameters and their log-variances; its
 * Gaussian proposals replace part of the prior-sampled starting particles of
 * the multi-start MAP stage (Sec. 3: MAP by multi-start gradient descent).
 * The network is not part of the paper; it is trained here on images that
 * lens_forward simulates.
 *
 * Architecture (fixed): input [B][64][64] bf16 (one channel); six 3x3
 * convolutions, padding 1, ReLU, channels 32-32-64-64-128-128, strides
 * 1-2-1-2-1-2; global average pooling; dense 128 -> 256 (ReLU) -> 28.
 * Outputs [B][28]: mu_k (k < 14) and log sigma_k^2 (14 + k) of the
 * standardised targets.  Flat parameter vector (float32), in this order:
 * for each convolution W[cout][3][3][cin] then bias[cout]; dense W[256][128],
 * bias[256]; dense W[28][256], bias[28].
 * All contractions run on BF16 matrix cores with FP32 accumulation; the
 * activations and gradients passed between layers are bf16 (round to
 * nearest even).  Training loss: mean over the batch of the Gaussian
 * negative log-likelihood sum_k [(z_k - mu_k)^2 e^{-s_k} + s_k] / 2.
 * ------------------------------------------------------------------------- */
typedef struct lens_cnn lens_cnn;
#define LENS_CNN_SIDE    64
#define LENS_CNN_TARGETS 14
#define LENS_CNN_OUTPUTS 28
/* Largest max_batch: activation offsets stay within 32-bit integers. */
#define LENS_CNN_MAX_BATCH 8192

/* Network with room for batches up to max_batch (1 .. LENS_CNN_MAX_BATCH);
 * weights He-initialised from Philox4x32-10 with the given seed.
 * Errors: LENS_EINVAL, LENS_ENOMEM. */
lens_status lens_cnn_create(int32_t max_batch, uint64_t seed, lens_cnn** out);
lens_status lens_cnn_destroy(lens_cnn* net);
int64_t lens_cnn_num_params(void);
/* d_params [lens_cnn_num_params()] float32 device copy in/out. */
lens_status lens_cnn_get_params(lens_cnn* net, float* d_params, void* stream);
lens_status lens_cnn_set_params(lens_cnn* net, const float* d_params, void* stream);

/* Network input from surface-brightness images: optional Gaussian noise
 * N(0, sigma^2) (Philox, key seed, counter counter0 + pixel index), then
 * asinh(x / (3 sigma)), rounded to bf16.  d_images [n][64][64] float,
 * d_out [n][64][64] bf16 (uint16 storage). */
lens_status lens_cnn_prepare_images(int32_t n_images, const float* d_images, float sigma,
                                    int32_t add_noise, uint64_t seed, uint64_t counter0,
                                    uint16_t* d_out, void* stream);

/* Inference: d_img [B][64][64] bf16 -> d_out [B][28] float. */
lens_status lens_cnn_forward(lens_cnn* net, int32_t B, const uint16_t* d_img, float* d_out,
                             void* stream);
/* Mean loss over the batch (d_loss [1]) and, if d_grads != NULL, its gradient
 * with respect to the flat parameter vector.  d_target [B][14] standardised. */
lens_status lens_cnn_loss_grad(lens_cnn* net, int32_t B, const uint16_t* d_img,
                               const float* d_target, float* d_loss, float* d_grads,
                               void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean loss. */
lens_status lens_cnn_train_step(lens_cnn* net, int32_t B, const uint16_t* d_img,
                                const float* d_target, float lr, float* d_loss, void* stream);

/* Proposal map: d parameters with the prior table of lens_plan_set_prior;
 * h_slot[j] = k routes network output k (0..13) to parameter j, -1 draws
 * parameter j from its prior; target k is standardised as
 * (theta - h_mean[k]) / h_std[k]; sigma is the image noise level used by the
 * input transform. */
lens_status lens_cnn_set_target_map(lens_cnn* net, int32_t d, const float* h_prior_table,
                                    const int32_t* h_slot, const float* h_mean,
                                    const float* h_std, float sigma);

/* Starting particles for S systems: d_img64 [S][64][64] float images (crop or
 * zero-pad to 64x64 at the native pixel scale), n_per_system draws each:
 * a mapped parameter is drawn from the network's Gaussian
 * N(mean_k + std_k mu_k, (std_k e^{s_k/2})^2) truncated to the parameter's
 * prior support (inverse CDF), or from its prior when the support holds less
 * than half of that Gaussian; the others from the prior; Philox4x32-10 with
 * the given seed, counter (system, draw, parameter).  d_theta_out [S][n][d];
 * d_flags [S] (optional): 1 if, for some mapped parameter, the support holds
 * less than 99 % of the network's Gaussian, else 0.  Falling back to
 * prior-sampled starts is the caller's decision (see the time-to-MAP
 * driver).  Requires lens_cnn_set_target_map. */
lens_status init_propose(lens_cnn* net, int32_t S, const float* d_img64, int32_t n_per_system,
                         uint64_t seed, float* d_theta_out, int32_t* d_flags, void* stream);

/* Plain multi-start starting points: n_per_system draws from the prior for
 * each of S systems (the prior branch of init_propose: Philox4x32-10 with
 * the given seed, counter (system, draw, parameter), inverse-CDF draws).
 * h_prior_table [d][5] as for lens_plan_set_prior; d_theta_out [S][n][d].
 * Synchronous on stream (a small descriptor is staged through device memory
 * that is freed before returning). */
lens_status lens_prior_sample(int32_t d, const float* h_prior_table, int32_t S, int32_t n_per_system,
                              uint64_t seed, float* d_theta_out, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (diagnostics, not part of the model).
 * With timing enabled, every kernel a plan launches is bracketed by two HIP
 * events recorded on the call's stream; lens_plan_read_timing synchronises
 * on those events, writes per-kernel totals and resets them.  Kernel slots:
 * LENS_K_PROLOGUE .. LENS_K_FINALIZE.  Timing must be off while a stream is
 * being captured into a graph.
 *   h_ms    [LENS_NUM_KERNEL_SLOTS] total milliseconds per slot (out)
 *   h_count [LENS_NUM_KERNEL_SLOTS] launches per slot (out)
 * Up to 65536 launches per slot are recorded between reads; more are
 * counted but not timed (LENS_EUNSUPPORTED from the read).
 * ------------------------------------------------------------------------- */
#define LENS_K_PROLOGUE 0
#define LENS_K_RENDER   1
#define LENS_K_PSF      2
#define LENS_K_ADJOINT  3
#define LENS_K_FINALIZE 4
#define LENS_K_POSTERIOR 5   /* bijection, prior, Adam / HMC kick and accept */
#define LENS_NUM_KERNEL_SLOTS 8

lens_status lens_plan_enable_timing(lens_plan* plan, int32_t enable);
lens_status lens_plan_read_timing(lens_plan* plan, double* h_ms, int64_t* h_count);
/* The same for a batch plan's likelihood sequence (lens_batch_loglike_grad
 * and the batched posterior): slots PROLOGUE, RENDER (the persistent render
 * launch), PSF (all PSF-class launches of one call together), ADJOINT (the
 * persistent adjoint launch), FINALIZE. */
lens_status lens_batch_enable_timing(lens_batch_plan* plan, int32_t enable);
lens_status lens_batch_read_timing(lens_batch_plan* plan, double* h_ms, int64_t* h_count);

#ifdef __cplusplus
}
#endif
#endif /* LENS_API_H */
