// C-ABI host layer of the uneven batch: per-system descriptors, cost-sorted
// work lists, PSF size classes, graph capture and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lens_internal.h"
#include "lens_sampler.h"
#include "lens_timer.h"

using namespace lens;

namespace {

bool desc_ok(const lens_model_desc& d) { return desc_valid(&d); }

struct PsfClass {
    std::pair<int, int> key{0, 0};   // (K, images per CU by LDS)
    int K = 0;
    int n = 0;
    size_t shm = 0;
    int nt = 256;   // work-group size
    WorkItem* items = nullptr;
};

}  // namespace

struct lens_batch_plan {
    KernelTimer timer;
    int S = 0;
    int N = 0;
    ModelInfo mi{};
    std::vector<lens_model_desc> desc;
    std::vector<int> P, p0, ppt;
    std::vector<int> Pcap;         // particles per system the buffers were sized for
    std::vector<const float*> psf, data, invvar;
    std::vector<double*> wflip;
    float* consts = nullptr;
    float* img = nullptr;
    double* partial = nullptr;
    BatchSys* d_sys = nullptr;
    WorkItem* d_items = nullptr;
    int n_items = 0;
    int* d_counter = nullptr;
    int* d_particle_sys = nullptr;
    std::vector<PsfClass> classes;
    std::map<std::pair<int, int>, int> psf_nt;   // work-group size chosen by the autotuner, per class
    int grid_render = 0, grid_adjoint = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<uint64_t> graph_key;
    uint64_t tiles_version = 0;
    // inference stage over all packed particles (one prior for every system)
    int* d_p0 = nullptr;          // [S + 1] first particle of each system
    ViewSrc* d_views = nullptr;   // [S]
    PriorRow* prior = nullptr;    // [d], null until lens_batch_set_prior
    float* theta = nullptr;       // [N][d] T(u)
    float* gtheta = nullptr;      // [N][d] dlogL/dtheta
    float* logl = nullptr;        // [N]
    double* logl64 = nullptr;     // [N]
    double* logp = nullptr;       // [N]
    float* gradu = nullptr;       // [N][d]
    int* map_step = nullptr;      // Adam steps taken since lens_batch_map_reset
    hipGraphExec_t map_graph = nullptr;
    std::vector<uint64_t> map_key;
};

static void free_classes(lens_batch_plan* b) {
    for (auto& c : b->classes)
        if (c.items) (void)hipFree(c.items);
    b->classes.clear();
}

// Uploads the particle packing (the system of each particle, the first
// particle of each system) for the current counts P.
static lens_status upload_packing(lens_batch_plan* b) {
    std::vector<int> psys(b->N);
    for (int k = 0; k < b->S; ++k)
        for (int p = 0; p < b->P[k]; ++p) psys[b->p0[k] + p] = k;
    std::vector<int> p0(b->p0);
    p0.push_back(b->N);
    if (hipMemcpy(b->d_particle_sys, psys.data(), sizeof(int) * (size_t)b->N, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(b->d_p0, p0.data(), sizeof(int) * (size_t)(b->S + 1), hipMemcpyHostToDevice) != hipSuccess)
        return LENS_EHIP;
    return LENS_OK;
}

// (Re)builds descriptors and work lists for the current tiles.
static lens_status rebuild(lens_batch_plan* b) {
    const int nacc = n_acc(b->mi);
    std::vector<BatchSys> sys(b->S);
    std::vector<WorkItem> items;
    std::vector<long long> cost;
    long long img_off = 0, part_off = 0;
    for (int k = 0; k < b->S; ++k) {
        BatchSys& q = sys[k];
        q.g = make_geo(b->desc[k]);
        q.K = b->desc[k].psf_size;
        q.P = b->P[k];
        q.p0 = b->p0[k];
        q.ppb = 256 * b->ppt[k];
        q.nch = chunks_for(q.g.npix, b->ppt[k]);
        q.img_off = img_off;
        q.part_off = part_off;
        q.wflip = b->wflip[k];
        q.wpsf = b->psf[k];
        q.data = b->data[k];
        q.invvar = b->invvar[k];
        psf_tile_dims(q.g, q.K, q.stride, q.rows);
        img_off += (long long)q.P * q.g.npix;
        part_off += (long long)q.P * q.nch;
        const int s2 = q.g.s * q.g.s;
        for (int p = 0; p < q.P; ++p)
            for (int c = 0; c < q.nch; ++c) {
                items.push_back({k, p, c});
                cost.push_back((long long)std::min(q.ppb, q.g.npix - c * q.ppb) * s2);
            }
    }
    (void)nacc;
    // longest-processing-time first; ties keep (system, particle, chunk) order
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<WorkItem> sorted(items.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];

    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    b->n_items = (int)sorted.size();
    if (hipMalloc(&b->d_items, sizeof(WorkItem) * sorted.size()) != hipSuccess) return LENS_ENOMEM;
    if (hipMemcpy(b->d_items, sorted.data(), sizeof(WorkItem) * sorted.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(b->d_sys, sys.data(), sizeof(BatchSys) * b->S, hipMemcpyHostToDevice) != hipSuccess)
        return LENS_EHIP;

    // PSF classes: one launch per (K, LDS tile class) over its (system,
    // particle) pairs.  The tile class is the number of an image's LDS tiles
    // that fit one CU (1, 2, 3, 4 or more), so that small images are not
    // given the LDS, hence the CU, that the largest image of their K needs.
    free_classes(b);
    std::map<std::pair<int, int>, std::vector<WorkItem>> byK;
    std::map<std::pair<int, int>, size_t> shm;
    std::map<std::pair<int, int>, int> strips;
    for (int k = 0; k < b->S; ++k) {
        const size_t bytes = (size_t)sys[k].stride * sys[k].rows * sizeof(float);
        const int fit = std::min<int>(4, std::max<int>(1, (int)((160 * 1024) / bytes)));
        const std::pair<int, int> key{sys[k].K, fit};
        for (int p = 0; p < b->P[k]; ++p) byK[key].push_back({k, p, 0});
        shm[key] = std::max(shm[key], bytes);
        strips[key] = std::max(strips[key], psf_strips(sys[k].g));
    }
    for (auto& kv : byK) {
        PsfClass c;
        c.K = kv.first.first;
        c.n = (int)kv.second.size();
        c.shm = shm[kv.first];
        c.key = kv.first;
        const auto ov = b->psf_nt.find(kv.first);
        c.nt = ov != b->psf_nt.end() ? ov->second : psf_threads(c.shm, strips[kv.first]);
        if (hipMalloc(&c.items, sizeof(WorkItem) * c.n) != hipSuccess) return LENS_ENOMEM;
        b->classes.push_back(c);
        if (hipMemcpy(c.items, kv.second.data(), sizeof(WorkItem) * c.n, hipMemcpyHostToDevice) !=
            hipSuccess)
            return LENS_EHIP;
    }
    b->tiles_version++;
    return LENS_OK;
}

static lens_status enqueue(lens_batch_plan* b, const float* theta, float* logl, float* grad,
                           hipStream_t st, double* logl64 = nullptr) {
    KernelTimer* t = &b->timer;
    {
        TimedLaunch tl(t, LENS_K_PROLOGUE, st);
        if (launch_prologue(b->mi, b->N, theta, b->consts, st) != hipSuccess) return LENS_EHIP;
    }
    if (launch_set_int_host(b->d_counter, 0, st) != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(t, LENS_K_RENDER, st);
        if (launch_batch_render(b->mi, b->grid_render, b->d_sys, b->d_items, b->n_items, b->d_counter,
                                b->consts, b->img, st) != hipSuccess)
            return LENS_EHIP;
    }
    {
        TimedLaunch tl(t, LENS_K_PSF, st);
        for (const auto& c : b->classes)
            if (launch_batch_psf(c.K, c.n, b->d_sys, c.items, b->consts, b->img, logl, logl64, c.shm, c.nt, st) !=
                hipSuccess)
                return LENS_EHIP;
    }
    if (launch_set_int_host(b->d_counter + 1, 0, st) != hipSuccess) return LENS_EHIP;
    {
        TimedLaunch tl(t, LENS_K_ADJOINT, st);
        if (launch_batch_adjoint(b->mi, b->grid_adjoint, b->d_sys, b->d_items, b->n_items,
                                 b->d_counter + 1, b->consts, b->img, b->partial, st) != hipSuccess)
            return LENS_EHIP;
    }
    TimedLaunch tl(t, LENS_K_FINALIZE, st);
    if (launch_batch_finalize(b->mi, b->N, b->d_sys, b->d_particle_sys, theta, b->consts, b->partial,
                              grad, st) != hipSuccess)
        return LENS_EHIP;
    return LENS_OK;
}

extern "C" {

lens_status lens_batch_plan_destroy(lens_batch_plan* b) {
    if (!b) return LENS_EINVAL;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->map_graph) (void)hipGraphExecDestroy(b->map_graph);
    free_classes(b);
    for (double* w : b->wflip)
        if (w) (void)hipFree(w);
    void* bufs[] = {b->consts, b->img,    b->partial, b->d_sys,  b->d_items, b->d_counter, b->d_particle_sys,
                    b->d_p0,   b->d_views, b->prior,  b->theta,  b->gtheta,  b->logl,      b->logl64,
                    b->logp,   b->gradu,  b->map_step};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    b->timer.release();
    delete b;
    return LENS_OK;
}

lens_status lens_batch_plan_create(int32_t S, const lens_model_desc* h_descs,
                                   const float* const* h_psf, const float* const* h_data,
                                   const float* const* h_invvar, const int32_t* h_particles,
                                   lens_batch_plan** out) {
    if (!out) return LENS_EINVAL;
    *out = nullptr;
    if (S < 1 || !h_descs || !h_psf || !h_data || !h_invvar || !h_particles) return LENS_EINVAL;
    for (int k = 0; k < S; ++k) {
        if (!desc_ok(h_descs[k]) || !h_psf[k] || !h_data[k] || !h_invvar[k] || h_particles[k] < 1)
            return LENS_EINVAL;
        if (h_descs[k].mass_model != h_descs[0].mass_model ||
            h_descs[k].n_lens_light != h_descs[0].n_lens_light ||
            h_descs[k].n_source != h_descs[0].n_source || h_descs[k].n_shapelet != 0)
            return LENS_EUNSUPPORTED;
        if (psf_lds_bytes(make_geo(h_descs[k]), h_descs[k].psf_size) > MAX_LDS_BYTES)
            return LENS_EUNSUPPORTED;
    }
    lens_batch_plan* b = new (std::nothrow) lens_batch_plan();
    if (!b) return LENS_ENOMEM;
    b->S = S;
    b->mi = model_info(h_descs[0]);
    long long N = 0, npix_tot = 0, rows_max = 0;
    for (int k = 0; k < S; ++k) {
        b->desc.push_back(h_descs[k]);
        b->P.push_back(h_particles[k]);
        b->Pcap.push_back(h_particles[k]);
        b->p0.push_back((int)N);
        b->ppt.push_back(4);
        b->psf.push_back(h_psf[k]);
        b->data.push_back(h_data[k]);
        b->invvar.push_back(h_invvar[k]);
        const long long npix = (long long)h_descs[k].nx * h_descs[k].ny;
        N += h_particles[k];
        npix_tot += npix * h_particles[k];
        rows_max += (long long)h_particles[k] * chunks_for((int)npix, 1);
    }
    if (N > (1LL << 30)) {
        delete b;
        return LENS_EUNSUPPORTED;
    }
    b->N = (int)N;
    const int nacc = n_acc(b->mi);
    b->wflip.assign(S, nullptr);
    bool ok = hipMalloc(&b->consts, sizeof(float) * CSTRIDE * (size_t)N) == hipSuccess &&
              hipMalloc(&b->img, sizeof(float) * (size_t)npix_tot) == hipSuccess &&
              hipMalloc(&b->partial, sizeof(double) * (size_t)rows_max * nacc) == hipSuccess &&
              hipMalloc(&b->d_sys, sizeof(BatchSys) * S) == hipSuccess &&
              hipMalloc(&b->d_counter, sizeof(int) * 4) == hipSuccess &&
              hipMalloc(&b->d_particle_sys, sizeof(int) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->d_p0, sizeof(int) * (size_t)(S + 1)) == hipSuccess &&
              hipMalloc(&b->d_views, sizeof(ViewSrc) * (size_t)S) == hipSuccess &&
              hipMalloc(&b->theta, sizeof(float) * (size_t)N * b->mi.d) == hipSuccess &&
              hipMalloc(&b->gtheta, sizeof(float) * (size_t)N * b->mi.d) == hipSuccess &&
              hipMalloc(&b->gradu, sizeof(float) * (size_t)N * b->mi.d) == hipSuccess &&
              hipMalloc(&b->logl, sizeof(float) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->logl64, sizeof(double) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->logp, sizeof(double) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->map_step, sizeof(int)) == hipSuccess;
    for (int k = 0; ok && k < S; ++k)
        ok = hipMalloc(&b->wflip[k], sizeof(double) * h_descs[k].psf_size * h_descs[k].psf_size) ==
             hipSuccess;
    if (!ok) {
        lens_batch_plan_destroy(b);
        return LENS_ENOMEM;
    }
    for (int k = 0; k < S; ++k)
        if (launch_flip(h_descs[k].psf_size, h_psf[k], b->wflip[k], nullptr) != hipSuccess) {
            lens_batch_plan_destroy(b);
            return LENS_EHIP;
        }
    std::vector<ViewSrc> views(S);
    for (int k = 0; k < S; ++k) views[k] = {h_data[k], h_descs[k].nx, h_descs[k].ny};
    if (upload_packing(b) != LENS_OK ||
        hipMemcpy(b->d_views, views.data(), sizeof(ViewSrc) * (size_t)S, hipMemcpyHostToDevice) !=
            hipSuccess ||
        launch_set_int(b->map_step, 0, nullptr) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        lens_batch_plan_destroy(b);
        return LENS_EHIP;
    }
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu < 1) ncu = 1;
    b->grid_render = ncu * batch_blocks_per_cu(b->mi, false);
    b->grid_adjoint = ncu * batch_blocks_per_cu(b->mi, true);
    lens_status s = rebuild(b);
    if (s != LENS_OK) {
        lens_batch_plan_destroy(b);
        return s;
    }
    *out = b;
    return LENS_OK;
}

int64_t lens_batch_total_particles(const lens_batch_plan* b) { return b ? (int64_t)b->N : -1; }

lens_status lens_batch_get_tiles(const lens_batch_plan* b, int32_t* h_ppt) {
    if (!b || !h_ppt) return LENS_EINVAL;
    for (int k = 0; k < b->S; ++k) h_ppt[k] = b->ppt[k];
    return LENS_OK;
}

lens_status lens_batch_set_tiles(lens_batch_plan* b, const int32_t* h_ppt) {
    if (!b || !h_ppt) return LENS_EINVAL;
    for (int k = 0; k < b->S; ++k)
        if (h_ppt[k] < 1 || h_ppt[k] > 64) return LENS_EINVAL;
    bool same = true;
    for (int k = 0; k < b->S; ++k) same = same && b->ppt[k] == h_ppt[k];
    if (same) return LENS_OK;
    if (hipDeviceSynchronize() != hipSuccess) return LENS_EHIP;
    for (int k = 0; k < b->S; ++k) b->ppt[k] = h_ppt[k];
    return rebuild(b);
}

lens_status lens_batch_set_particles(lens_batch_plan* b, const int32_t* h_particles) {
    if (!b || !h_particles) return LENS_EINVAL;
    for (int k = 0; k < b->S; ++k)
        if (h_particles[k] < 1 || h_particles[k] > b->Pcap[k]) return LENS_EINVAL;
    bool same = true;
    for (int k = 0; k < b->S; ++k) same = same && b->P[k] == h_particles[k];
    if (same) return LENS_OK;
    if (hipDeviceSynchronize() != hipSuccess) return LENS_EHIP;
    int n = 0;
    for (int k = 0; k < b->S; ++k) {
        b->P[k] = h_particles[k];
        b->p0[k] = n;
        n += h_particles[k];
    }
    b->N = n;
    const lens_status s = upload_packing(b);
    return s != LENS_OK ? s : rebuild(b);
}

lens_status lens_batch_loglike_grad_counts(lens_batch_plan* b, const int32_t* h_particles, const float* d_theta,
                                           float* d_logl, float* d_grad, int32_t use_graph, void* stream) {
    if (!b || !h_particles || !d_theta || !d_logl || !d_grad) return LENS_EINVAL;
    const lens_status s = lens_batch_set_particles(b, h_particles);
    if (s != LENS_OK) return s;
    return lens_batch_loglike_grad(b, d_theta, d_logl, d_grad, use_graph, stream);
}

lens_status lens_batch_get_particles(const lens_batch_plan* b, int32_t* h_particles) {
    if (!b || !h_particles) return LENS_EINVAL;
    for (int k = 0; k < b->S; ++k) h_particles[k] = b->P[k];
    return LENS_OK;
}

lens_status lens_batch_loglike_grad(lens_batch_plan* b, const float* d_theta, float* d_logl,
                                    float* d_grad, int32_t use_graph, void* stream) {
    if (!b || !d_theta || !d_logl || !d_grad) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) return enqueue(b, d_theta, d_logl, d_grad, st);
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)d_theta, (uint64_t)(uintptr_t)d_logl,
                                       (uint64_t)(uintptr_t)d_grad, b->tiles_version};
    if (!b->graph || b->graph_key != key) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
            return LENS_EHIP;
        b->timer.capturing = true;
        lens_status s = enqueue(b, d_theta, d_logl, d_grad, b->cap_stream);
        b->timer.capturing = false;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (s != LENS_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return s != LENS_OK ? s : LENS_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->graph = nullptr;
            return LENS_EHIP;
        }
        b->graph_key = key;
    }
    return hipGraphLaunch(b->graph, st) == hipSuccess ? LENS_OK : LENS_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Inference stage over the packed particles of all systems
// ---------------------------------------------------------------------------
static lens_status batch_hip(hipError_t e) { return e == hipSuccess ? LENS_OK : LENS_EHIP; }

// logp(u) = logL(T(u)) + log prior(T(u)) [+ log|dT/du|] and dlogp/du (no argument checks)
static lens_status batch_logpost(lens_batch_plan* b, const float* u, int with_jac, float* theta_out,
                                 double* logp, float* grad_u, hipStream_t st) {
    float* th = theta_out ? theta_out : b->theta;
    if (launch_bijection(b->N, b->mi.d, b->prior, u, th, st) != hipSuccess) return LENS_EHIP;
    lens_status s = enqueue(b, th, b->logl, b->gtheta, st, b->logl64);
    if (s != LENS_OK) return s;
    return batch_hip(launch_posterior(b->N, b->mi.d, b->prior, u, b->logl64, b->gtheta, with_jac, logp,
                                      grad_u, st));
}

static uint64_t batch_fbits(float f) {
    uint32_t v;
    std::memcpy(&v, &f, 4);
    return v;
}

extern "C" {

lens_status lens_batch_set_prior(lens_batch_plan* b, const float* h_table) {
    if (!b || !h_table) return LENS_EINVAL;
    std::vector<PriorRow> rows(b->mi.d);
    if (!build_prior_rows(b->mi.d, h_table, rows.data())) return LENS_EINVAL;
    if (!b->prior && hipMalloc(&b->prior, sizeof(PriorRow) * b->mi.d) != hipSuccess) return LENS_ENOMEM;
    if (hipMemcpy(b->prior, rows.data(), sizeof(PriorRow) * b->mi.d, hipMemcpyHostToDevice) != hipSuccess)
        return LENS_EHIP;
    if (b->map_graph) (void)hipGraphExecDestroy(b->map_graph);
    b->map_graph = nullptr;
    b->map_key.clear();
    return LENS_OK;
}

lens_status lens_batch_logpost_grad(lens_batch_plan* b, const float* d_u, int32_t with_jacobian,
                                    float* d_theta, double* d_logp, float* d_grad, void* stream) {
    if (!b || !d_u || !d_logp || !d_grad || !b->prior) return LENS_EINVAL;
    return batch_logpost(b, d_u, with_jacobian != 0, d_theta, d_logp, d_grad, (hipStream_t)stream);
}

lens_status lens_batch_map_reset(lens_batch_plan* b) {
    if (!b) return LENS_EINVAL;
    if (launch_set_int(b->map_step, 0, nullptr) != hipSuccess) return LENS_EHIP;
    return batch_hip(hipDeviceSynchronize());
}

lens_status lens_batch_map_adam(lens_batch_plan* b, float* d_u, float* d_m, float* d_v, int32_t n_steps,
                                float lr, float decay, float beta1, float beta2, float eps, float* d_loss,
                                int32_t use_graph, void* stream) {
    if (!b || !d_u || !d_m || !d_v || n_steps < 0 || !b->prior) return LENS_EINVAL;
    if (!(lr > 0.0f) || !(decay > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const AdamHyper hp{lr, decay, beta1, beta2, eps};
    auto step = [&](hipStream_t s) -> lens_status {
        lens_status r = batch_logpost(b, d_u, 0, nullptr, b->logp, b->gradu, s);
        if (r != LENS_OK) return r;
        if (launch_adam(b->N, b->mi.d, b->gradu, b->logp, d_u, d_m, d_v, b->map_step, hp, d_loss, s) !=
            hipSuccess)
            return LENS_EHIP;
        return batch_hip(launch_add_int(b->map_step, 1, s));
    };
    if (!use_graph) {
        for (int r = 0; r < n_steps; ++r) {
            lens_status s = step(st);
            if (s != LENS_OK) return s;
        }
        return LENS_OK;
    }
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)d_u, (uint64_t)(uintptr_t)d_m,
                                       (uint64_t)(uintptr_t)d_v, (uint64_t)(uintptr_t)d_loss,
                                       batch_fbits(lr),          batch_fbits(decay),
                                       batch_fbits(beta1),       batch_fbits(beta2),
                                       batch_fbits(eps),         b->tiles_version};
    if (!b->map_graph || b->map_key != key) {
        if (b->map_graph) (void)hipGraphExecDestroy(b->map_graph);
        b->map_graph = nullptr;
        b->map_key.clear();
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return LENS_EHIP;
        b->timer.capturing = true;
        lens_status s = step(b->cap_stream);
        b->timer.capturing = false;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (s != LENS_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return s != LENS_OK ? s : LENS_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&b->map_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->map_graph = nullptr;
            return LENS_EHIP;
        }
        b->map_key = key;
    }
    for (int r = 0; r < n_steps; ++r)
        if (hipGraphLaunch(b->map_graph, st) != hipSuccess) return LENS_EHIP;
    return LENS_OK;
}

lens_status lens_batch_to_unconstrained(lens_batch_plan* b, const float* d_theta, float* d_u, void* stream) {
    if (!b || !d_theta || !d_u || !b->prior) return LENS_EINVAL;
    return batch_hip(launch_inverse_bijection(b->N, b->mi.d, b->prior, d_theta, d_u, (hipStream_t)stream));
}

lens_status lens_batch_argmin(lens_batch_plan* b, const float* d_val, float* d_best, int32_t* d_arg,
                              void* stream) {
    if (!b || !d_val || !d_best || !d_arg) return LENS_EINVAL;
    return batch_hip(launch_segment_argmin(b->S, b->d_p0, d_val, d_best, d_arg, (hipStream_t)stream));
}

lens_status lens_batch_center_views(lens_batch_plan* b, int32_t side, float* d_out, void* stream) {
    if (!b || !d_out || side < 1 || side > LENS_MAX_SIDE) return LENS_EINVAL;
    return batch_hip(launch_center_views(b->S, side, b->d_views, d_out, (hipStream_t)stream));
}

lens_status lens_batch_enable_timing(lens_batch_plan* b, int32_t enable) {
    if (!b) return LENS_EINVAL;
    b->timer.enabled = enable != 0;
    return LENS_OK;
}

lens_status lens_batch_read_timing(lens_batch_plan* b, double* h_ms, int64_t* h_count) {
    if (!b || !h_ms || !h_count) return LENS_EINVAL;
    return b->timer.read(h_ms, h_count);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
namespace {

// Work-group size of each PSF launch class (in the order of b->classes);
// captured graphs are re-captured on their next use.
lens_status set_psf_threads(lens_batch_plan* b, const std::vector<int>& nts) {
    if (nts.size() != b->classes.size()) return LENS_EINVAL;
    for (int nt : nts)
        if (nt != 256 && nt != 512 && nt != 1024) return LENS_EINVAL;
    for (size_t i = 0; i < nts.size(); ++i) {
        b->classes[i].nt = nts[i];
        b->psf_nt[b->classes[i].key] = nts[i];
    }
    b->tiles_version++;
    return LENS_OK;
}

uint64_t geometry_hash(const lens_batch_plan* b) {
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the batch geometry
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)b->S);
    mix((uint64_t)b->mi.mass_model * 64 + b->mi.n_lens_light * 8 + b->mi.n_source);
    for (int k = 0; k < b->S; ++k) {
        const lens_model_desc& d = b->desc[k];
        uint32_t ps;
        std::memcpy(&ps, &d.pix_scale, 4);
        mix(((uint64_t)d.nx << 32) | (uint64_t)d.ny);
        mix(((uint64_t)d.supersample << 32) | (uint64_t)d.psf_size);
        mix(((uint64_t)ps << 32) | (uint64_t)b->P[k]);
    }
    return h;
}

// Cache file: {"<hex hash>": [ppt per system..., PSF work-group size per class...], ...}
std::map<std::string, std::vector<int>> read_cache(const char* path) {
    std::map<std::string, std::vector<int>> out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while (true) {
        const size_t q0 = txt.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = txt.find('"', q0 + 1);
        const size_t lb = txt.find('[', q1);
        const size_t rb = txt.find(']', lb);
        if (q1 == std::string::npos || lb == std::string::npos || rb == std::string::npos) break;
        std::vector<int> v;
        const char* p = txt.c_str() + lb + 1;
        const char* end = txt.c_str() + rb;
        while (p < end) {
            char* nx = nullptr;
            const long x = std::strtol(p, &nx, 10);
            if (nx == p) { ++p; continue; }
            v.push_back((int)x);
            p = nx;
        }
        out[txt.substr(q0 + 1, q1 - q0 - 1)] = v;
        pos = rb + 1;
    }
    return out;
}

bool write_cache(const char* path, const std::map<std::string, std::vector<int>>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        std::fprintf(f, "  \"%s\": [", kv.first.c_str());
        for (size_t j = 0; j < kv.second.size(); ++j)
            std::fprintf(f, "%s%d", j ? ", " : "", kv.second[j]);
        std::fprintf(f, "]%s\n", ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" lens_status lens_batch_autotune(lens_batch_plan* b, const float* d_theta,
                                           const char* cache_path, void* stream) {
    if (!b || !d_theta) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char key[32];
    std::snprintf(key, sizeof key, "%016llx", (unsigned long long)geometry_hash(b));
    std::map<std::string, std::vector<int>> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        const int C = (int)b->classes.size();
        if (it != cache.end() && ((int)it->second.size() == b->S || (int)it->second.size() == b->S + C)) {
            const lens_status r = lens_batch_set_tiles(b, it->second.data());
            if (r != LENS_OK || (int)it->second.size() == b->S) return r;
            std::vector<int> nts(it->second.begin() + b->S, it->second.end());
            return set_psf_threads(b, nts);
        }
    }
    float* logl = nullptr;
    float* grad = nullptr;
    if (hipMalloc(&logl, sizeof(float) * b->N) != hipSuccess ||
        hipMalloc(&grad, sizeof(float) * (size_t)b->N * b->mi.d) != hipSuccess) {
        if (logl) (void)hipFree(logl);
        return LENS_ENOMEM;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto time_once = [&]() -> float {
        if (enqueue(b, d_theta, logl, grad, st) != LENS_OK) return 1e30f;   // warm-up
        float best = 1e30f;
        for (int r = 0; r < 2; ++r) {
            (void)hipEventRecord(e0, st);
            if (enqueue(b, d_theta, logl, grad, st) != LENS_OK) return 1e30f;
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    // size classes: supersampling x image-side bucket of 32 px
    std::map<int, std::vector<int>> cls;
    for (int k = 0; k < b->S; ++k) {
        const int side = std::max(b->desc[k].nx, b->desc[k].ny);
        cls[b->desc[k].supersample * 1000 + side / 32].push_back(k);
    }
    std::vector<int> cur(b->S, 4);
    lens_status s = lens_batch_set_tiles(b, cur.data());
    float best = s == LENS_OK ? time_once() : 1e30f;
    const int cand[4] = {1, 2, 4, 8};
    for (const auto& kv : cls) {
        if (s != LENS_OK) break;
        int keep = cur[kv.second[0]];
        for (int c : cand) {
            if (c == keep) continue;
            std::vector<int> trial = cur;
            for (int k : kv.second) trial[k] = c;
            if ((s = lens_batch_set_tiles(b, trial.data())) != LENS_OK) break;
            const float t = time_once();
            if (t < best) {
                best = t;
                keep = c;
            }
        }
        for (int k : kv.second) cur[k] = keep;
    }
    if (s == LENS_OK) s = lens_batch_set_tiles(b, cur.data());
    // then the work-group size of each PSF launch class, with the tiles fixed
    std::vector<int> nts;
    for (const auto& c : b->classes) nts.push_back(c.nt);
    if (s == LENS_OK) best = time_once();
    for (size_t i = 0; s == LENS_OK && i < nts.size(); ++i) {
        int keep = nts[i];
        for (int nt : {256, 512, 1024}) {
            if (nt == keep) continue;
            std::vector<int> trial = nts;
            trial[i] = nt;
            if ((s = set_psf_threads(b, trial)) != LENS_OK) break;
            const float t = time_once();
            if (t < best) {
                best = t;
                keep = nt;
            }
        }
        nts[i] = keep;
    }
    if (s == LENS_OK) s = set_psf_threads(b, nts);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(logl);
    (void)hipFree(grad);
    if (s == LENS_OK && cache_path) {
        cache[key] = cur;
        cache[key].insert(cache[key].end(), nts.begin(), nts.end());
        if (!write_cache(cache_path, cache)) return LENS_EINVAL;
    }
    return s;
}
