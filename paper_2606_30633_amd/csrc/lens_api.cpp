// C-ABI host layer: argument validation, plan objects, launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <new>
#include <vector>

#include "lens_internal.h"

using namespace lens;

// Event pairs around kernel launches of one plan (diagnostic timing).
struct KernelTimer {
    static constexpr int kMaxRecords = 65536;
    bool enabled = false;
    std::vector<hipEvent_t> ev[LENS_NUM_KERNEL_SLOTS];
    int used[LENS_NUM_KERNEL_SLOTS] = {0};
    int64_t count[LENS_NUM_KERNEL_SLOTS] = {0};

    hipEvent_t take(int slot) {
        auto& v = ev[slot];
        if (used[slot] >= (int)v.size()) {
            if ((int)v.size() >= 2 * kMaxRecords) return nullptr;
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            v.push_back(e);
        }
        return v[used[slot]++];
    }
    void release() {
        for (auto& v : ev)
            for (auto e : v) (void)hipEventDestroy(e);
        for (auto& v : ev) v.clear();
    }
};

// Records start/stop events around one launch when timing is enabled.
struct TimedLaunch {
    KernelTimer* t;
    int slot;
    hipStream_t st;
    hipEvent_t stop = nullptr;
    TimedLaunch(KernelTimer* t_, int slot_, hipStream_t st_) : t(t_), slot(slot_), st(st_) {
        if (!t->enabled) return;
        t->count[slot]++;
        hipEvent_t start = t->take(slot);
        stop = start ? t->take(slot) : nullptr;
        if (start && stop) (void)hipEventRecord(start, st);
        else stop = nullptr;
    }
    ~TimedLaunch() {
        if (stop) (void)hipEventRecord(stop, st);
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
    size_t partial_words;
    KernelTimer timer;
};

namespace {

bool desc_ok(const lens_model_desc* d) {
    if (!d) return false;
    if (d->nx < 1 || d->ny < 1 || d->nx > LENS_MAX_SIDE || d->ny > LENS_MAX_SIDE) return false;
    if (!(d->pix_scale > 0.0f) || !std::isfinite(d->pix_scale)) return false;
    if (d->supersample < 1 || d->supersample > 16) return false;
    if (d->psf_size < 1 || d->psf_size > LENS_MAX_PSF || (d->psf_size % 2) == 0) return false;
    if (d->mass_model != LENS_MASS_SIE && d->mass_model != LENS_MASS_EPL) return false;
    if (d->n_lens_light < 0 || d->n_lens_light > LENS_MAX_LENS_LIGHT) return false;
    if (d->n_source < 1 || d->n_source > LENS_MAX_SOURCE) return false;
    return true;
}

int nparams(const lens_model_desc* d) {
    return (d->mass_model == LENS_MASS_EPL ? 8 : 7) + 7 * (d->n_lens_light + d->n_source);
}

lens_status hip_status(hipError_t e) { return e == hipSuccess ? LENS_OK : LENS_EHIP; }

}  // namespace

extern "C" {

const char* lens_status_string(lens_status s) {
    switch (s) {
        case LENS_OK: return "ok";
        case LENS_EINVAL: return "invalid argument";
        case LENS_EUNSUPPORTED: return "unsupported configuration";
        case LENS_EHIP: return "HIP runtime error";
        case LENS_ENOMEM: return "out of memory";
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
    p->mi.mass_model = desc->mass_model;
    p->mi.n_lens_light = desc->n_lens_light;
    p->mi.n_source = desc->n_source;
    p->mi.d = nparams(desc);
    p->geo = make_geo(*desc);
    p->max_particles = max_particles;
    p->ppt = 4;
    p->psf = d_psf;
    p->data = d_data;
    p->invvar = d_invvar;
    if (psf_lds_bytes(p->geo, desc->psf_size) > MAX_LDS_BYTES) {
        delete p;
        return LENS_EUNSUPPORTED;
    }
    const size_t npix = (size_t)desc->nx * desc->ny;
    const int nacc = n_acc(desc->n_lens_light + desc->n_source);
    p->partial_words = (size_t)max_particles * chunks_for((int)npix, 1) * nacc;
    const int K = desc->psf_size;
    if (hipMalloc(&p->psf_flip, sizeof(double) * K * K) != hipSuccess ||
        hipMalloc(&p->consts, sizeof(float) * CSTRIDE * (size_t)max_particles) != hipSuccess ||
        hipMalloc(&p->imgbuf, sizeof(float) * npix * (size_t)max_particles) != hipSuccess ||
        hipMalloc(&p->partial, sizeof(double) * p->partial_words) != hipSuccess) {
        lens_plan_destroy(p);
        return LENS_ENOMEM;
    }
    if (launch_flip(K, d_psf, p->psf_flip, nullptr) != hipSuccess ||
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

lens_status lens_forward(lens_plan* plan, int32_t P, const float* d_theta, float* d_images,
                         void* stream) {
    if (!plan || !d_theta || !d_images || P < 1 || P > plan->max_particles) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
    return hip_status(launch_psf(plan->mi, plan->geo, plan->desc.psf_size, 0, P, plan->consts,
                                 plan->imgbuf, plan->psf_flip, plan->psf, plan->data,
                                 plan->invvar, d_images, nullptr, nullptr, st));
}

lens_status lens_loglike(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                         void* stream) {
    if (!plan || !d_theta || !d_logl || P < 1 || P > plan->max_particles) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
    return hip_status(launch_psf(plan->mi, plan->geo, plan->desc.psf_size, 1, P, plan->consts,
                                 plan->imgbuf, plan->psf_flip, plan->psf, plan->data,
                                 plan->invvar, nullptr, d_logl, nullptr, st));
}

lens_status lens_loglike_grad(lens_plan* plan, int32_t P, const float* d_theta, float* d_logl,
                              float* d_grad, double* d_logl64, void* stream) {
    if (!plan || !d_theta || !d_logl || !d_grad || P < 1 || P > plan->max_particles)
        return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    lens_status s = front(plan, P, d_theta, st);
    if (s != LENS_OK) return s;
    hipError_t e;
    {
        TimedLaunch tl(&plan->timer, LENS_K_PSF, st);
        e = launch_psf(plan->mi, plan->geo, plan->desc.psf_size, 2, P, plan->consts, plan->imgbuf,
                       plan->psf_flip, plan->psf, plan->data, plan->invvar, nullptr, d_logl,
                       d_logl64, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(&plan->timer, LENS_K_ADJOINT, st);
        e = launch_adjoint(plan->mi, plan->geo, P, plan->ppt, plan->consts, plan->imgbuf,
                           plan->partial, st);
    }
    if (e != hipSuccess) return LENS_EHIP;
    const int nch = chunks_for(plan->geo.npix, plan->ppt);
    TimedLaunch tl(&plan->timer, LENS_K_FINALIZE, st);
    return hip_status(launch_finalize(plan->mi, P, nch, d_theta, plan->consts, plan->partial,
                                      d_grad, st));
}

lens_status lens_plan_enable_timing(lens_plan* plan, int32_t enable) {
    if (!plan) return LENS_EINVAL;
    plan->timer.enabled = enable != 0;
    return LENS_OK;
}

lens_status lens_plan_read_timing(lens_plan* plan, double* h_ms, int64_t* h_count) {
    if (!plan || !h_ms || !h_count) return LENS_EINVAL;
    KernelTimer& t = plan->timer;
    lens_status st = LENS_OK;
    for (int k = 0; k < LENS_NUM_KERNEL_SLOTS; ++k) {
        double tot = 0.0;
        for (int r = 0; r + 1 < t.used[k]; r += 2) {
            if (hipEventSynchronize(t.ev[k][r + 1]) != hipSuccess) return LENS_EHIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t.ev[k][r], t.ev[k][r + 1]) != hipSuccess) return LENS_EHIP;
            tot += ms;
        }
        if (t.count[k] * 2 > t.used[k]) st = LENS_EUNSUPPORTED;
        h_ms[k] = tot;
        h_count[k] = t.count[k];
        t.used[k] = 0;
        t.count[k] = 0;
    }
    return st;
}

}  // extern "C"
