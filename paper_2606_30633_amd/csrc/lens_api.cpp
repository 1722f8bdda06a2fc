// C-ABI host layer: argument validation, plan objects, launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "lens_internal.h"
#include "lens_backward.h"
#include "lens_sampler.h"
#include "lens_timer.h"

using namespace lens;

// One captured HIP graph and the arguments it was captured with.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key.clear();
    }
};

struct lens_plan {
    lens_model_desc desc;
    ModelInfo mi;
    Geo geo;
    int max_particles;
    int ppt;
    const float* psf;
    const float* data;
    const float* invvar;
    double* psf_flip;
    float* consts;
    float* imgbuf;
    double* partial;
    bool tiled;               // PSF stage by pixel tiles (the whole-image LDS tile does not fit)
    float* resbuf;            // [maxP][npix] residual w (d - m) of the tiled PSF stage
    double* chi_part;         // [maxP][tiles] chi^2 partials of the tiled PSF stage
    size_t partial_words;
    KernelTimer timer;
    // inference stages
    PriorRow* prior;          // [d] device, null until lens_plan_set_prior
    float* theta;             // [maxP][d] T(u)
    float* gtheta;            // [maxP][d] dlogL/dtheta
    float* logl;              // [maxP]
    double* logl64;           // [maxP]
    double* logp;             // [maxP] (MAP path)
    float* gradu;             // [maxP][d] (MAP path)
    float* hmc_u0;            // [maxP][d]
    float* hmc_g0;            // [maxP][d]
    float* hmc_p;             // [maxP][d]
    double* hmc_logp0;        // [maxP]
    double* hmc_h0;           // [maxP]
    float* svi_u;             // [maxP][d] surrogate samples
    double* svi_eps;          // [d][maxP] their standard normals
    double* svi_logq;         // [maxP]
    int backward;             // posterior path uses the backward likelihood (lens_plan_set_backward)
    double* hmc_accprob;      // [maxP] adaptation statistic (lens_hmc_adapt; on first use)
    double* hmc_state;        // [8] dual-averaging state
    float* hmc_eps;           // [1] device step size
    double* hmc_wmean;        // [maxP][d] window means (Welford)
    double* hmc_wm2;          // [maxP][d] window sums of squared deviations
    float* bwd_thx;           // [maxP][d] parameters with unit intensities (backward likelihood; on first use)
    float* bwd_img;           // [maxP][npix] PSF-convolved component images, K per particle
    float* bwd_theta;         // [maxP][d] parameters with the solved intensities
    int* counters;            // [0] MAP step, [1] HMC transitions in this run, [2..3] HMC first transition (64-bit),
                              // [4] SVI step, [5] SVI steps in this run, [6] step of lens_svi_elbo_grad,
                              // [7] window samples of lens_hmc_adapt
    hipStream_t cap_stream;
    GraphCache map_graph, hmc_graph, svi_graph, adapt_graph;
};

namespace {

bool desc_ok(const lens_model_desc* d) { return desc_valid(d); }

int nparams(const lens_model_desc* d) { return model_info(*d).d; }

lens_status hip_status(hipError_t e) { return e == hipSuccess ? LENS_OK : LENS_EHIP; }


}  // namespace

namespace lens {

bool build_prior_rows(int d, const float* h_table, PriorRow* rows) {
    const double half_log_2pi = 0.91893853320467274178;
    for (int j = 0; j < d; ++j) {
        const float* r = h_table + 5 * j;
        const int kind = (int)r[0];
        PriorRow& q = rows[j];
        q.kind = kind;
        q.a = r[1];
        q.b = r[2];
        q.pad0 = q.pad1 = 0.0;
        if (kind == LENS_PRIOR_UNIFORM) {
            if (!(r[2] > r[1])) return false;
            q.lo = r[1];
            q.hi = r[2];
            q.cst = -std::log((double)r[2] - (double)r[1]);
        } else if (kind == LENS_PRIOR_NORMAL || kind == LENS_PRIOR_LOGNORMAL) {
            if (!(r[2] > 0.0f)) return false;
            q.lo = q.hi = 0.0;
            q.cst = -std::log((double)r[2]) - half_log_2pi;
        } else if (kind == LENS_PRIOR_TRUNCNORMAL) {
            if (!(r[2] > 0.0f) || !(r[4] > r[3])) return false;
            q.lo = r[3];
            q.hi = r[4];
            const double zl = ((double)r[3] - r[1]) / r[2], zh = ((double)r[4] - r[1]) / r[2];
            const double mass = 0.5 * (std::erfc(-zh / std::sqrt(2.0)) - std::erfc(-zl / std::sqrt(2.0)));
            q.cst = -std::log((double)r[2]) - half_log_2pi - std::log(mass);
        } else {
            return false;
        }
    }
    return true;
}

}  // namespace lens

extern "C" {

const char* lens_status_string(lens_status s) {
    switch (s) {
        case LENS_OK: return "ok";
        case LENS_EINVAL: return "invalid argument";
        case LENS_EUNSUPPORTED: return "unsupported configuration";
        case LENS_EHIP: return "HIP runtime error";
        case LENS_ENOMEM: return "out of memory";
        case LENS_ESCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
        default: return "unknown status";
    }
}

int32_t lens_num_params(const lens_model_desc* desc) {
    if (!desc_ok(desc)) return -1;
    return nparams(desc);
}

lens_status lens_plan_destroy(lens_plan* plan) {
    if (!plan) return LENS_EINVAL;
    if (plan->psf_flip) (void)hipFree(plan->psf_flip);
    if (plan->consts) (void)hipFree(plan->consts);
    if (plan->imgbuf) (void)hipFree(plan->imgbuf);
    if (plan->partial) (void)hipFree(plan->partial);
    if (plan->resbuf) (void)hipFree(plan->resbuf);
    if (plan->chi_part) (void)hipFree(plan->chi_part);
    plan->map_graph.reset();
    plan->hmc_graph.reset();
    plan->svi_graph.reset();
    plan->adapt_graph.reset();
    void* bufs[] = {plan->prior, plan->theta, plan->gtheta, plan->logl, plan->logl64, plan->logp,
                    plan->gradu, plan->hmc_u0, plan->hmc_g0, plan->hmc_p, plan->hmc_logp0,
                    plan->hmc_h0, plan->svi_u, plan->svi_eps, plan->svi_logq, plan->hmc_accprob,
                    plan->hmc_state, plan->hmc_eps, plan->hmc_wmean, plan->hmc_wm2, plan->bwd_thx,
                    plan->bwd_img, plan->bwd_theta, plan->counters};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    plan->timer.release();
    delete plan;
    return LENS_OK;
}

lens_status lens_plan_create(const lens_model_desc* desc, const float* d_psf, const float* d_data,
                             const float* d_invvar, int32_t max_particles, lens_plan** out) {
    if (!out) return LENS_EINVAL;
    *out = nullptr;
    if (!desc_ok(desc) || !d_psf || !d_data || !d_invvar || max_particles < 1) return LENS_EINVAL;
    lens_plan* p = new (std::nothrow) lens_plan();
    if (!p) return LENS_ENOMEM;
    p->desc = *desc;
    p->mi = model_info(*desc);
    p->geo = make_geo(*desc);
    p->max_particles = max_particles;
    p->ppt = 4;
    p->psf = d_psf;
    p->data = d_data;
    p->invvar = d_invvar;
    p->tiled = psf_lds_bytes(p->geo, desc->psf_size) > MAX_LDS_BYTES;
    const size_t npix = (size_t)desc->nx * desc->ny;
    const int nacc = n_acc(p->mi);
    p->partial_words = (size_t)max_particles * chunks_for((int)npix, 1) * nacc;
    const int K = desc->psf_size;
    if (hipMalloc(&p->psf_flip, sizeof(double) * K * K) != hipSuccess ||
        hipMalloc(&p->consts, sizeof(float) * CSTRIDE * (size_t)max_particles) != hipSuccess ||
        hipMalloc(&p->imgbuf, sizeof(float) * npix * (size_t)max_particles) != hipSuccess ||
        hipMalloc(&p->partial, sizeof(double) * p->partial_words) != hipSuccess) {
        lens_plan_destroy(p);
        return LENS_ENOMEM;
    }
    if (p->tiled &&
        (hipMalloc(&p->resbuf, sizeof(float) * npix * (size_t)max_particles) != hipSuccess ||
         hipMalloc(&p->chi_part, sizeof(double) * psf_num_tiles(p->geo) * (size_t)max_particles) != hipSuccess)) {
        lens_plan_destroy(p);
        return LENS_ENOMEM;
    }
    const size_t Pd = (size_t)max_particles * p->mi.d;
    const size_t Pn = (size_t)max_particles;
    if (hipMalloc(&p->theta, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->gtheta, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->logl, sizeof(float) * Pn) != hipSuccess ||
        hipMalloc(&p->logl64, sizeof(double) * Pn) != hipSuccess ||
        hipMalloc(&p->logp, sizeof(double) * Pn) != hipSuccess ||
        hipMalloc(&p->gradu, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->hmc_u0, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->hmc_g0, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->hmc_p, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->hmc_logp0, sizeof(double) * Pn) != hipSuccess ||
        hipMalloc(&p->hmc_h0, sizeof(double) * Pn) != hipSuccess ||
        hipMalloc(&p->svi_u, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&p->svi_eps, sizeof(double) * Pd) != hipSuccess ||
        hipMalloc(&p->svi_logq, sizeof(double) * Pn) != hipSuccess ||
        hipMalloc(&p->counters, sizeof(int) * 8) != hipSuccess) {
        lens_plan_destroy(p);
        return LENS_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        lens_plan_destroy(p);
        return LENS_EHIP;
    }
    if (launch_set_int(p->counters, 0, nullptr) != hipSuccess ||
        launch_set_int(p->counters + 1, 0, nullptr) != hipSuccess ||
        launch_set_int(p->counters + 4, 0, nullptr) != hipSuccess ||
        launch_flip(K, d_psf, p->psf_flip, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        lens_plan_destroy(p);
        return LENS_EHIP;
    }
    *out = p;
    return LENS_OK;
}

lens_status lens_plan_set_pixels_per_thread(lens_plan* plan, int32_t ppt) {
    if (!plan || ppt < 1 || ppt > 64) return LENS_EINVAL;
    plan->ppt = ppt;
    return LENS_OK;
}

static lens_status front(lens_plan* plan, int32_t P, const float* d_theta, hipStream_t st) {
    hipError_t e;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PROLOGUE, st);
        e = launch_prologue(plan->mi, P, d_theta, plan->consts, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_RENDER, st);
        e = launch_render(plan->mi, plan->geo, P, plan->ppt, plan->consts, plan->imgbuf, st);
    }
    return hip_status(e);
}

// PSF stage of a plan (modes of launch_psf): the whole image per work-group
// when its tile fits the LDS, else by pixel tiles.
static hipError_t plan_psf(lens_plan* plan, int mode, int P, float* img, float* out, float* logl,
                           double* logl64, hipStream_t st) {
    if (!plan->tiled)
        return launch_psf(plan->mi, plan->geo, plan->desc.psf_size, mode, P, plan->consts, img, plan->psf_flip,
                          plan->psf, plan->data, plan->invvar, out, logl, logl64, st);
    return launch_psf_tiled(plan->geo, plan->desc.psf_size, mode, P, plan->consts, img, plan->resbuf,
                            plan->psf_flip, plan->psf, plan->data, plan->invvar, out, logl, logl64,
                            plan->chi_part, st);
}

// Chain rule from the adjoint partial rows; many rows per particle (large
// images) are first summed in place in the same order.
static hipError_t plan_finalize(lens_plan* plan, int P, const float* d_theta, float* d_grad, hipStream_t st) {
    constexpr int kPreSumRows = 64;
    const int nch = chunks_for(plan->geo.npix, plan->ppt);
    if (nch == 1) return launch_finalize(plan->mi, P, 1, d_theta, plan->consts, plan->partial, d_grad, st);
    // the chunk sums in many threads, then the chain rule per particle: few
    // rows are summed in row order (results equal the direct finalize bit for
    // bit), many by the lane-parallel tree
    const hipError_t e = nch <= kPreSumRows ? launch_presum_rows(P, nch, n_acc(plan->mi), plan->partial, st)
                                            : launch_partial_sum(P, nch, n_acc(plan->mi), plan->partial, st);
    if (e != hipSuccess) return e;
    return launch_finalize(plan->mi, P, 1, d_theta, plan->consts, plan->partial, d_grad, st, nch);
}

lens_status lens_forward(lens_plan* plan, int32_t P, const float* d_theta, float* d_images,
                         void* stream) {
    if (!plan || !d_theta || !d_images || P < 1 || P > plan->max_particles) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
    return hip_status(plan_psf(plan, 0, P, plan->imgbuf, d_images, nullptr, nullptr, st));
}

lens_status lens_loglike(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                         void* stream) {
    if (!plan || !d_theta || !d_logl || P < 1 || P > plan->max_particles) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
    return hip_status(plan_psf(plan, 1, P, plan->imgbuf, nullptr, d_logl, nullptr, st));
}

// Enqueues logL + gradient for theta (no argument checks).
static lens_status loglike_grad_enqueue(lens_plan* plan, int32_t P, const float* d_theta,
                                        float* d_logl, float* d_grad, double* d_logl64,
                                        hipStream_t st) {
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    hipError_t e;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
        e = plan_psf(plan, 2, P, plan->imgbuf, nullptr, d_logl, d_logl64, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_ADJOINT, st);
        e = launch_adjoint(plan->mi, plan->geo, P, plan->ppt, plan->consts, plan->imgbuf,
                           plan->partial, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    TimedLaunch tl(&plan->timer, LENS_K_FINALIZE, st);
    return hip_status(plan_finalize(plan, P, d_theta, d_grad, st));
}

lens_status lens_loglike_grad(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                              float* d_grad, double* d_logl64, void* stream) {
    if (!plan || !d_theta || !d_logl || !d_grad || P < 1 || P > plan->max_particles)
        return LENS_EINVAL;
    return loglike_grad_enqueue(plan, P, d_theta, d_logl, d_grad, d_logl64, (hipStream_t)stream);
}

static BwdSlots bwd_slots(const lens_plan* plan) {
    BwdSlots s{};
    const int ns = plan->desc.n_lens_light + plan->desc.n_source;
    s.d = plan->mi.d;
    const int base = plan->desc.mass_model == LENS_MASS_EPL ? 8 : 7;
    for (int k = 0; k < ns; ++k) s.slot[k] = base + 7 * k + 6;
    // shapelet coefficients: linear amplitudes after the Sersic intensities
    const int nb = plan->mi.n_shapelet ? (plan->mi.sh_nmax + 1) * (plan->mi.sh_nmax + 2) / 2 : 0;
    for (int k = 0; k < nb; ++k) s.slot[ns + k] = base + 7 * ns + 3 + k;
    s.K = ns + nb;
    return s;
}

static lens_status bwd_alloc(lens_plan* plan) {
    if (plan->bwd_thx) return LENS_OK;
    const size_t Pd = (size_t)plan->max_particles * plan->mi.d;
    const size_t npix = (size_t)plan->geo.npix;
    if (hipMalloc(&plan->bwd_thx, sizeof(float) * Pd) != hipSuccess ||
        hipMalloc(&plan->bwd_img, sizeof(float) * npix * plan->max_particles) != hipSuccess ||
        hipMalloc(&plan->bwd_theta, sizeof(float) * Pd) != hipSuccess) {
        for (float** b : {&plan->bwd_thx, &plan->bwd_img, &plan->bwd_theta})
            if (*b) {
                (void)hipFree(*b);
                *b = nullptr;
            }
        return LENS_ENOMEM;
    }
    return LENS_OK;
}

// Enqueues the backward likelihood (scratch allocated; P K <= max_particles checked).
static lens_status backward_enqueue(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                                    float* d_grad, float* d_amp, double* d_logl64, hipStream_t st) {
    const BwdSlots s = bwd_slots(plan);
    const int PK = P * s.K;
    const size_t npix = (size_t)plan->geo.npix;
    // all intensities 1, one render pass writing each component's image
    if (launch_bwd_expand(P, s, d_theta, plan->bwd_thx, st) != hipSuccess) return LENS_EHIP;
    hipError_t e;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PROLOGUE, st);
        e = launch_prologue(plan->mi, P, plan->bwd_thx, plan->consts, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_RENDER, st);
        e = launch_render_split(plan->mi, plan->geo, P, plan->ppt, plan->consts, plan->imgbuf, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
        e = plan_psf(plan, 0, PK, plan->imgbuf, plan->bwd_img, nullptr, nullptr, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_FINALIZE, st);
        e = launch_bwd_normal(P, s, (int)npix, plan->bwd_img, plan->data, plan->invvar, plan->consts, d_theta,
                              plan->bwd_theta, d_amp, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    // logL and gradient at the solved intensities: constants of those
    // parameters, the model image assembled from the component images (no
    // second render), then the PSF / logL / adjoint pass of the forward path
    {
        TimedLaunch tl(&plan->timer, LENS_K_PROLOGUE, st);
        e = launch_prologue(plan->mi, P, plan->bwd_theta, plan->consts, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_FINALIZE, st);
        e = launch_bwd_assemble(P, s, (int)npix, plan->imgbuf, plan->bwd_theta, plan->bwd_img, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
        e = plan_psf(plan, 2, P, plan->bwd_img, nullptr, d_logl, d_logl64, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_ADJOINT, st);
        e = launch_adjoint(plan->mi, plan->geo, P, plan->ppt, plan->consts, plan->bwd_img, plan->partial, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_FINALIZE, st);
        e = plan_finalize(plan, P, plan->bwd_theta, d_grad, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    return hip_status(launch_bwd_zero_slots(P, s, d_grad, st));
}

// The posterior path can take P particles (the backward likelihood holds K images per particle).
static bool posterior_fits(const lens_plan* plan, int32_t P) {
    if (P < 1 || P > plan->max_particles) return false;
    return !plan->backward || (long)P * bwd_slots(plan).K <= plan->max_particles;
}

lens_status lens_loglike_grad_backward(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                                       float* d_grad, float* d_amp, void* stream) {
    if (!plan || !d_theta || !d_logl || !d_grad || P < 1) return LENS_EINVAL;
    const BwdSlots s = bwd_slots(plan);
    if (s.K < 1 || s.K > BWD_MAX_K || (long)P * s.K > plan->max_particles) return LENS_EINVAL;
    lens_status r = bwd_alloc(plan);
    if (r != LENS_OK) return r;
    return backward_enqueue(plan, P, d_theta, d_logl, d_grad, d_amp, nullptr, (hipStream_t)stream);
}

lens_status lens_plan_set_backward(lens_plan* plan, int32_t enable) {
    if (!plan) return LENS_EINVAL;
    if (enable) {
        const int K = bwd_slots(plan).K;
        if (K < 1 || K > BWD_MAX_K) return LENS_EINVAL;
        lens_status r = bwd_alloc(plan);
        if (r != LENS_OK) return r;
    }
    plan->backward = enable ? 1 : 0;
    plan->map_graph.reset();
    plan->hmc_graph.reset();
    plan->svi_graph.reset();
    plan->adapt_graph.reset();
    return LENS_OK;
}

// Enqueues logp(u) and dlogp/du (no argument checks).  theta_out may be null.
static lens_status logpost_enqueue(lens_plan* plan, int32_t P, const float* d_u, int with_jac,
                                   float* theta_out, double* d_logp, float* d_grad,
                                   hipStream_t st) {
    const int d = plan->mi.d;
    float* th = theta_out ? theta_out : plan->theta;
    {
        TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, st);
        if (launch_bijection(P, d, plan->prior, d_u, th, st) != hipSuccess) return LENS_EHIP;
    }
    ParamMask skip;
    lens_status s;
    if (plan->backward) {
        const BwdSlots bs = bwd_slots(plan);
        for (int k = 0; k < bs.K; ++k) skip.set(bs.slot[k]);
        s = backward_enqueue(plan, P, th, plan->logl, plan->gtheta, nullptr, plan->logl64, st);
    } else {
        s = loglike_grad_enqueue(plan, P, th, plan->logl, plan->gtheta, plan->logl64, st);
    }
    if (s != LENS_OK) return s;
    TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, st);
    return hip_status(launch_posterior(P, d, plan->prior, d_u, plan->logl64, plan->gtheta,
                                       with_jac, d_logp, d_grad, st, skip));
}

lens_status lens_plan_set_prior(lens_plan* plan, const float* h_table) {
    if (!plan || !h_table) return LENS_EINVAL;
    const int d = plan->mi.d;
    std::vector<PriorRow> rows(d);
    if (!build_prior_rows(d, h_table, rows.data())) return LENS_EINVAL;
    if (!plan->prior && hipMalloc(&plan->prior, sizeof(PriorRow) * d) != hipSuccess)
        return LENS_ENOMEM;
    if (hipMemcpy(plan->prior, rows.data(), sizeof(PriorRow) * d, hipMemcpyHostToDevice) != hipSuccess)
        return LENS_EHIP;
    plan->map_graph.reset();
    plan->hmc_graph.reset();
    plan->svi_graph.reset();
    plan->adapt_graph.reset();
    return LENS_OK;
}

lens_status lens_to_unconstrained(lens_plan* plan, int32_t P, const float* d_theta, float* d_u,
                                  void* stream) {
    if (!plan || !d_theta || !d_u || P < 1 || !plan->prior) return LENS_EINVAL;
    return hip_status(launch_inverse_bijection(P, plan->mi.d, plan->prior, d_theta, d_u, (hipStream_t)stream));
}

lens_status lens_logpost_grad(lens_plan* plan, int32_t P, const float* d_u, int32_t with_jacobian,
                              float* d_theta, double* d_logp, float* d_grad, void* stream) {
    if (!plan || !d_u || !d_logp || !d_grad || !posterior_fits(plan, P)) return LENS_EINVAL;
    if (!plan->prior) return LENS_EINVAL;
    return logpost_enqueue(plan, P, d_u, with_jacobian != 0, d_theta, d_logp, d_grad,
                           (hipStream_t)stream);
}

}  // extern "C"

// Runs `repeats` copies of the work that `enqueue` puts on a stream, either
// eagerly on st or through a HIP graph captured once per key.
template <class F>
static lens_status run_maybe_graph(lens_plan* plan, GraphCache& gc, const std::vector<uint64_t>& key,
                                   bool use_graph, int repeats, hipStream_t st, F&& enqueue) {
    if (!use_graph) {
        for (int r = 0; r < repeats; ++r) {
            lens_status s = enqueue(st);
            if (s != LENS_OK) return s;
        }
        return LENS_OK;
    }
    if (!gc.exec || gc.key != key) {
        gc.reset();
        hipGraph_t graph = nullptr;
        plan->timer.capturing = true;
        if (hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            plan->timer.capturing = false;
            return LENS_EHIP;
        }
        lens_status s = enqueue(plan->cap_stream);
        hipError_t e = hipStreamEndCapture(plan->cap_stream, &graph);
        plan->timer.capturing = false;
        if (s != LENS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return LENS_EHIP;
        e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            gc.exec = nullptr;
            return LENS_EHIP;
        }
        gc.key = key;
    }
    for (int r = 0; r < repeats; ++r)
        if (hipGraphLaunch(gc.exec, st) != hipSuccess) return LENS_EHIP;
    return LENS_OK;
}

extern "C" {

static uint64_t fbits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

lens_status lens_map_reset(lens_plan* plan) {
    if (!plan) return LENS_EINVAL;
    if (launch_set_int(plan->counters, 0, nullptr) != hipSuccess) return LENS_EHIP;
    return hip_status(hipDeviceSynchronize());
}

lens_status lens_map_adam(lens_plan* plan, int32_t P, float* d_u, float* d_m, float* d_v,
                          int32_t n_steps, float lr, float decay, float beta1, float beta2,
                          float eps, float* d_loss, int32_t use_graph, void* stream) {
    if (!plan || !d_u || !d_m || !d_v || !posterior_fits(plan, P) || n_steps < 0)
        return LENS_EINVAL;
    if (!plan->prior || !(lr > 0.0f) || !(decay > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const AdamHyper hp{lr, decay, beta1, beta2, eps};
    const int d = plan->mi.d;
    auto step = [&](hipStream_t s) -> lens_status {
        lens_status r = logpost_enqueue(plan, P, d_u, 0, nullptr, plan->logp, plan->gradu, s);
        if (r != LENS_OK) return r;
        TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
        if (launch_adam(P, d, plan->gradu, plan->logp, d_u, d_m, d_v, plan->counters, hp, d_loss, s) !=
            hipSuccess)
            return LENS_EHIP;
        return hip_status(launch_add_int(plan->counters, 1, s));
    };
    const std::vector<uint64_t> key = {(uint64_t)P, (uint64_t)(uintptr_t)d_u, (uint64_t)(uintptr_t)d_m,
                                       (uint64_t)(uintptr_t)d_v, (uint64_t)(uintptr_t)d_loss,
                                       fbits(lr), fbits(decay), fbits(beta1), fbits(beta2), fbits(eps),
                                       (uint64_t)plan->ppt};
    return run_maybe_graph(plan, plan->map_graph, key, use_graph != 0, n_steps, st, step);
}

lens_status lens_hmc_run(lens_plan* plan, int32_t C, float* d_u, float* d_grad, double* d_logp,
                         const float* d_inv_mass, float eps, int32_t n_leapfrog,
                         int32_t n_transitions, uint64_t seed, uint64_t transition0,
                         float* d_samples, int32_t* d_accepts, int32_t use_graph, void* stream) {
    if (!plan || !d_u || !d_grad || !d_logp || !d_inv_mass || !posterior_fits(plan, C) ||
        n_leapfrog < 1 || n_transitions < 0 || !(eps > 0.0f))
        return LENS_EINVAL;
    if (!plan->prior) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int d = plan->mi.d;
    HmcArgs a{};
    a.u = d_u; a.grad = d_grad; a.logp = d_logp;
    a.u0 = plan->hmc_u0; a.g0 = plan->hmc_g0; a.logp0 = plan->hmc_logp0;
    a.p = plan->hmc_p; a.h0 = plan->hmc_h0; a.inv_mass = d_inv_mass;
    a.samples = d_samples; a.accepts = d_accepts;
    a.tcount = plan->counters + 1;
    a.seed = seed;
    a.transition0 = reinterpret_cast<const unsigned long long*>(plan->counters + 2);
    a.eps = eps;
    auto transition = [&](hipStream_t s) -> lens_status {
        {
            TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
            if (launch_hmc_begin(C, d, a, s) != hipSuccess) return LENS_EHIP;
        }
        for (int l = 0; l < n_leapfrog; ++l) {
            if (l > 0) {
                TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
                if (launch_hmc_kick_drift(C, d, a, s) != hipSuccess) return LENS_EHIP;
            }
            lens_status r = logpost_enqueue(plan, C, d_u, 1, nullptr, d_logp, d_grad, s);
            if (r != LENS_OK) return r;
        }
        {
            TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
            if (launch_hmc_end(C, d, a, s) != hipSuccess) return LENS_EHIP;
        }
        return hip_status(launch_add_int(plan->counters + 1, 1, s));
    };
    // transition counter of this run starts at zero and its first transition's
    // index is written to device memory (outside any graph: a captured graph
    // reads both, so it is not re-captured for a new transition0)
    if (launch_set_int(plan->counters + 1, 0, st) != hipSuccess ||
        launch_set_u64(reinterpret_cast<unsigned long long*>(plan->counters + 2), transition0, st) != hipSuccess)
        return LENS_EHIP;
    const std::vector<uint64_t> key = {(uint64_t)C, (uint64_t)(uintptr_t)d_u, (uint64_t)(uintptr_t)d_grad,
                                       (uint64_t)(uintptr_t)d_logp, (uint64_t)(uintptr_t)d_inv_mass,
                                       fbits(eps), (uint64_t)n_leapfrog, seed,
                                       (uint64_t)(uintptr_t)d_samples, (uint64_t)(uintptr_t)d_accepts,
                                       (uint64_t)plan->ppt};
    return run_maybe_graph(plan, plan->hmc_graph, key, use_graph != 0, n_transitions, st, transition);
}

int32_t lens_svi_num_params(int32_t d) {
    return (d < 1 || d > SVI_MAX_D) ? -1 : svi_num_params(d);
}

lens_status lens_svi_reset(lens_plan* plan) {
    if (!plan) return LENS_EINVAL;
    if (launch_set_int(plan->counters + 4, 0, nullptr) != hipSuccess) return LENS_EHIP;
    return hip_status(hipDeviceSynchronize());
}

// Shared part of the SVI calls: draws, target at the draws, reduction (+ update).
static lens_status svi_step_enqueue(lens_plan* plan, const SviArgs& a, hipStream_t s) {
    {
        TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
        if (launch_svi_draw(a, s) != hipSuccess) return LENS_EHIP;
    }
    lens_status r = logpost_enqueue(plan, a.n, a.u, 1, nullptr, plan->logp, plan->gradu, s);
    if (r != LENS_OK) return r;
    TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
    return hip_status(launch_svi_reduce(a, s));
}

static SviArgs svi_args(lens_plan* plan, int32_t n, float* d_phi, uint64_t seed) {
    SviArgs a{};
    a.phi = d_phi;
    a.u = plan->svi_u;
    a.eps = plan->svi_eps;
    a.logq = plan->svi_logq;
    a.logp = plan->logp;
    a.grad_u = plan->gradu;
    a.seed = seed;
    a.n = n;
    a.d = plan->mi.d;
    if (plan->backward) {
        const BwdSlots bs = bwd_slots(plan);
        for (int k = 0; k < bs.K; ++k) a.frozen |= (uint64_t)1 << bs.slot[k];
    }
    return a;
}

lens_status lens_svi_elbo_grad(lens_plan* plan, int32_t n, const float* d_phi, uint64_t seed,
                               int32_t step, double* d_elbo, float* d_grad_phi, float* d_u,
                               void* stream) {
    if (!plan || !d_phi || !d_elbo || !posterior_fits(plan, n) || step < 0) return LENS_EINVAL;
    if (!plan->prior || plan->mi.d > SVI_MAX_D) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    SviArgs a = svi_args(plan, n, const_cast<float*>(d_phi), seed);
    if (d_u) a.u = d_u;
    a.grad_phi = d_grad_phi;
    a.elbo = d_elbo;
    a.step = plan->counters + 6;
    a.call_step = nullptr;
    a.update = 0;
    if (launch_set_int(plan->counters + 6, step, st) != hipSuccess) return LENS_EHIP;
    return svi_step_enqueue(plan, a, st);
}

lens_status lens_svi_run(lens_plan* plan, int32_t n, float* d_phi, float* d_m, float* d_s,
                         int32_t n_steps, int32_t optimizer, float lr, float beta1, float beta2,
                         float eps, uint64_t seed, double* d_elbo, int32_t use_graph, void* stream) {
    if (!plan || !d_phi || !d_m || !d_s || !posterior_fits(plan, n) || n_steps < 0)
        return LENS_EINVAL;
    if (!plan->prior || plan->mi.d > SVI_MAX_D) return LENS_EINVAL;
    if ((optimizer != LENS_OPT_ADAM && optimizer != LENS_OPT_ADABELIEF) || !(lr > 0.0f) ||
        !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    SviArgs a = svi_args(plan, n, d_phi, seed);
    a.m = d_m;
    a.s = d_s;
    a.elbo = d_elbo;
    a.step = plan->counters + 4;
    a.call_step = plan->counters + 5;
    a.update = 1;
    a.optimizer = optimizer == LENS_OPT_ADABELIEF ? SVI_OPT_ADABELIEF : SVI_OPT_ADAM;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps_opt = eps;
    auto step = [&](hipStream_t s) -> lens_status {
        lens_status r = svi_step_enqueue(plan, a, s);
        if (r != LENS_OK) return r;
        if (launch_add_int(plan->counters + 4, 1, s) != hipSuccess) return LENS_EHIP;
        return hip_status(launch_add_int(plan->counters + 5, 1, s));
    };
    // steps of this run are counted from zero (outside any graph): the ELBO index
    if (launch_set_int(plan->counters + 5, 0, st) != hipSuccess) return LENS_EHIP;
    const std::vector<uint64_t> key = {(uint64_t)n, (uint64_t)(uintptr_t)d_phi, (uint64_t)(uintptr_t)d_m,
                                       (uint64_t)(uintptr_t)d_s, (uint64_t)(uintptr_t)d_elbo,
                                       (uint64_t)optimizer, fbits(lr), fbits(beta1), fbits(beta2),
                                       fbits(eps), seed, (uint64_t)plan->ppt};
    return run_maybe_graph(plan, plan->svi_graph, key, use_graph != 0, n_steps, st, step);
}

lens_status lens_svi_moments(int32_t d, const float* d_phi, float* d_mean, float* d_cov, float* d_var,
                             void* stream) {
    if (d < 1 || d > SVI_MAX_D || !d_phi) return LENS_EINVAL;
    return hip_status(launch_svi_moments(d, d_phi, d_mean, d_cov, d_var, (hipStream_t)stream));
}

lens_status lens_hmc_adapt(lens_plan* plan, int32_t C, float* d_u, float* d_grad, double* d_logp,
                           const float* d_inv_mass, float eps0, float target_accept, int32_t n_leapfrog,
                           int32_t n_transitions, int32_t window_start, uint64_t seed, uint64_t transition0,
                           float* d_eps_trace, float* d_eps_final, float* d_var, int32_t use_graph, void* stream) {
    if (!plan || !d_u || !d_grad || !d_logp || !d_inv_mass || !posterior_fits(plan, C) ||
        n_leapfrog < 1 || n_transitions < 0 || window_start < 0 || !(eps0 > 0.0f) ||
        !(target_accept > 0.0f && target_accept < 1.0f))
        return LENS_EINVAL;
    if (!plan->prior) return LENS_EINVAL;
    const int d = plan->mi.d;
    const size_t Pd = (size_t)plan->max_particles * d;
    if (!plan->hmc_accprob) {
        if (hipMalloc(&plan->hmc_accprob, sizeof(double) * plan->max_particles) != hipSuccess ||
            hipMalloc(&plan->hmc_state, sizeof(double) * 8) != hipSuccess ||
            hipMalloc(&plan->hmc_eps, sizeof(float) * 2) != hipSuccess ||
            hipMalloc(&plan->hmc_wmean, sizeof(double) * Pd) != hipSuccess ||
            hipMalloc(&plan->hmc_wm2, sizeof(double) * Pd) != hipSuccess) {
            void** bs[] = {(void**)&plan->hmc_accprob, (void**)&plan->hmc_state, (void**)&plan->hmc_eps,
                           (void**)&plan->hmc_wmean, (void**)&plan->hmc_wm2};
            for (void** b : bs)
                if (*b) {
                    (void)hipFree(*b);
                    *b = nullptr;
                }
            return LENS_ENOMEM;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    HmcArgs a{};
    a.u = d_u; a.grad = d_grad; a.logp = d_logp;
    a.u0 = plan->hmc_u0; a.g0 = plan->hmc_g0; a.logp0 = plan->hmc_logp0;
    a.p = plan->hmc_p; a.h0 = plan->hmc_h0; a.inv_mass = d_inv_mass;
    a.tcount = plan->counters + 1;
    a.seed = seed;
    a.transition0 = reinterpret_cast<const unsigned long long*>(plan->counters + 2);
    a.eps = eps0;
    a.eps_dev = plan->hmc_eps;
    a.accprob = plan->hmc_accprob;
    AdaptArgs ad{};
    ad.state = plan->hmc_state;
    ad.accprob = plan->hmc_accprob;
    ad.eps_dev = plan->hmc_eps;
    ad.eps_trace = d_eps_trace;
    ad.eps_final = d_eps_final;
    ad.tcount = plan->counters + 1;
    ad.delta = target_accept;
    int* wcount = plan->counters + 7;
    auto transition = [&](hipStream_t s) -> lens_status {
        {
            TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
            if (launch_hmc_begin(C, d, a, s) != hipSuccess) return LENS_EHIP;
        }
        for (int l = 0; l < n_leapfrog; ++l) {
            if (l > 0) {
                TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
                if (launch_hmc_kick_drift(C, d, a, s) != hipSuccess) return LENS_EHIP;
            }
            lens_status r = logpost_enqueue(plan, C, d_u, 1, nullptr, d_logp, d_grad, s);
            if (r != LENS_OK) return r;
        }
        TimedLaunch tl(&plan->timer, LENS_K_POSTERIOR, s);
        if (launch_hmc_end(C, d, a, s) != hipSuccess || launch_hmc_adapt(C, ad, s) != hipSuccess ||
            launch_hmc_welford(C, d, d_u, plan->counters + 1, window_start, plan->hmc_wmean, plan->hmc_wm2,
                               wcount, s) != hipSuccess)
            return LENS_EHIP;
        return hip_status(launch_add_int(plan->counters + 1, 1, s));
    };
    // state, step size, window sums and counters start afresh (outside any graph)
    if (launch_hmc_adapt_init(C, d, plan->hmc_state, plan->hmc_eps, eps0, plan->hmc_wmean, plan->hmc_wm2, wcount,
                              st) != hipSuccess ||
        launch_set_int(plan->counters + 1, 0, st) != hipSuccess ||
        launch_set_u64(reinterpret_cast<unsigned long long*>(plan->counters + 2), transition0, st) != hipSuccess)
        return LENS_EHIP;
    const std::vector<uint64_t> key = {(uint64_t)C, (uint64_t)(uintptr_t)d_u, (uint64_t)(uintptr_t)d_grad,
                                       (uint64_t)(uintptr_t)d_logp, (uint64_t)(uintptr_t)d_inv_mass,
                                       (uint64_t)n_leapfrog, seed, (uint64_t)window_start,
                                       fbits(target_accept), (uint64_t)(uintptr_t)d_eps_trace,
                                       (uint64_t)(uintptr_t)d_eps_final, (uint64_t)plan->ppt};
    lens_status r = run_maybe_graph(plan, plan->adapt_graph, key, use_graph != 0, n_transitions, st, transition);
    if (r != LENS_OK) return r;
    if (d_var)
        return hip_status(launch_hmc_window_var(C, d, plan->hmc_wmean, plan->hmc_wm2, wcount, d_var, st));
    return LENS_OK;
}

lens_status lens_plan_enable_timing(lens_plan* plan, int32_t enable) {
    if (!plan) return LENS_EINVAL;
    plan->timer.enabled = enable != 0;
    return LENS_OK;
}

lens_status lens_plan_read_timing(lens_plan* plan, double* h_ms, int64_t* h_count) {
    if (!plan || !h_ms || !h_count) return LENS_EINVAL;
    return plan->timer.read(h_ms, h_count);
}

}  // extern "C"
