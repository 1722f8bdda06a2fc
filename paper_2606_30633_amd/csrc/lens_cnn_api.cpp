// C-ABI host layer of the learned initializer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "lens_cnn.h"

using namespace lens;

struct lens_cnn {
    CnnNet net;
};

namespace {

const int kChannels[CNN_CONV] = {32, 32, 64, 64, 128, 128};
const int kStrides[CNN_CONV] = {1, 2, 1, 2, 1, 2};

long long layout(CnnNet& n) {
    long long off = 0;
    int cin = 1;
    for (int l = 0; l < CNN_CONV; ++l) {
        CnnLayer& L = n.conv[l];
        L.cin = cin;
        L.cout = kChannels[l];
        L.stride = kStrides[l];
        L.w_off = off;
        off += (long long)L.cout * 9 * L.cin;
        L.b_off = off;
        off += L.cout;
        cin = L.cout;
    }
    n.fc1 = {CNN_C6, CNN_H1, 1, off, off + (long long)CNN_H1 * CNN_C6};
    off += (long long)CNN_H1 * CNN_C6 + CNN_H1;
    n.fc2 = {CNN_H1, CNN_OUT, 1, off, off + (long long)CNN_OUT * CNN_H1};
    off += (long long)CNN_OUT * CNN_H1 + CNN_OUT;
    return off;
}

template <class T>
bool alloc(T** p, size_t n) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * n) == hipSuccess;
}

}  // namespace

extern "C" {

int64_t lens_cnn_num_params(void) {
    CnnNet n{};
    return layout(n);
}

lens_status lens_cnn_destroy(lens_cnn* c) {
    if (!c) return LENS_EINVAL;
    CnnNet& n = c->net;
    if (n.train_graph) (void)hipGraphExecDestroy(n.train_graph);
    if (n.cap_stream) (void)hipStreamDestroy(n.cap_stream);
    void* bufs[] = {n.params, n.grads, n.adam_m, n.adam_v, n.wbf, n.pooled, n.dpooled, n.hidden, n.dhidden, n.out,
                    n.dout, n.wpart, n.colpart, n.losspart, n.c0part, n.tmap, n.prep, n.img_stage, n.tgt_stage,
                    n.hyper, n.loss_dev};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 0; l < CNN_CONV; ++l) {
        if (n.act[l]) (void)hipFree(n.act[l]);
        if (n.dact[l]) (void)hipFree(n.dact[l]);
    }
    delete c;
    return LENS_OK;
}

lens_status lens_cnn_create(int32_t max_batch, uint64_t seed, lens_cnn** out) {
    if (!out) return LENS_EINVAL;
    *out = nullptr;
    if (max_batch < 1 || max_batch > LENS_CNN_MAX_BATCH) return LENS_EINVAL;
    lens_cnn* c = new (std::nothrow) lens_cnn();
    if (!c) return LENS_ENOMEM;
    CnnNet& n = c->net;
    n.max_batch = max_batch;
    n.nparams = layout(n);
    const size_t B = (size_t)max_batch;
    size_t wpart = 0;
    bool ok = alloc(&n.params, n.nparams) && alloc(&n.grads, n.nparams) && alloc(&n.adam_m, n.nparams) &&
              alloc(&n.adam_v, n.nparams) && alloc(&n.wbf, n.nparams);
    int H = CNN_IN;
    for (int l = 0; ok && l < CNN_CONV; ++l) {
        H /= kStrides[l];
        const size_t sz = B * H * H * kChannels[l];
        ok = alloc(&n.act[l], sz) && alloc(&n.dact[l], sz);
        const size_t w = (size_t)wgrad_splits((long long)B * H * H) * n.conv[l].cout * 9 * n.conv[l].cin;
        wpart = w > wpart ? w : wpart;
    }
    ok = ok && alloc(&n.pooled, B * CNN_C6) && alloc(&n.dpooled, B * CNN_C6) && alloc(&n.hidden, B * CNN_H1) &&
         alloc(&n.dhidden, B * CNN_H1) && alloc(&n.out, B * CNN_OUT) && alloc(&n.dout, B * CNN_OUT) &&
         alloc(&n.wpart, wpart) && alloc(&n.colpart, (size_t)colpart_capacity(max_batch)) &&
         alloc(&n.losspart, B / 256 + 1) && alloc(&n.c0part, B * 32 * 10) && alloc(&n.tmap, 1) &&
         alloc(&n.prep, B * CNN_IN * CNN_IN) &&
         alloc(&n.img_stage, B * CNN_IN * CNN_IN) && alloc(&n.tgt_stage, B * CNN_NT) && alloc(&n.hyper, 2) &&
         alloc(&n.loss_dev, 1) && hipStreamCreateWithFlags(&n.cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        lens_cnn_destroy(c);
        return LENS_ENOMEM;
    }
    if (hipMemset(n.adam_m, 0, sizeof(float) * n.nparams) != hipSuccess ||
        hipMemset(n.adam_v, 0, sizeof(float) * n.nparams) != hipSuccess ||
        hipMemset(n.params, 0, sizeof(float) * n.nparams) != hipSuccess || cnn_init(n, seed, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        lens_cnn_destroy(c);
        return LENS_EHIP;
    }
    n.step = 0;
    *out = c;
    return LENS_OK;
}

lens_status lens_cnn_get_params(lens_cnn* c, float* d_params, void* stream) {
    if (!c || !d_params) return LENS_EINVAL;
    return hipMemcpyAsync(d_params, c->net.params, sizeof(float) * c->net.nparams, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream) == hipSuccess
               ? LENS_OK
               : LENS_EHIP;
}

lens_status lens_cnn_set_params(lens_cnn* c, const float* d_params, void* stream) {
    if (!c || !d_params) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(c->net.params, d_params, sizeof(float) * c->net.nparams, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        cnn_params_to_bf16(c->net, st) != hipSuccess)
        return LENS_EHIP;
    return LENS_OK;
}

lens_status lens_cnn_prepare_images(int32_t n_images, const float* d_images, float sigma, int32_t add_noise,
                                    uint64_t seed, uint64_t counter0, uint16_t* d_out, void* stream) {
    if (n_images < 1 || !d_images || !d_out || !(sigma > 0.0f)) return LENS_EINVAL;
    return cnn_prepare((long long)n_images * CNN_IN * CNN_IN, d_images, sigma, add_noise, seed, counter0,
                       reinterpret_cast<__bf16*>(d_out), (hipStream_t)stream) == hipSuccess
               ? LENS_OK
               : LENS_EHIP;
}

lens_status lens_cnn_forward(lens_cnn* c, int32_t B, const uint16_t* d_img, float* d_out, void* stream) {
    if (!c || !d_img || !d_out || B < 1 || B > c->net.max_batch) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (cnn_forward(c->net, B, reinterpret_cast<const __bf16*>(d_img), st) != hipSuccess) return LENS_EHIP;
    return hipMemcpyAsync(d_out, c->net.out, sizeof(float) * B * CNN_OUT, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? LENS_OK
               : LENS_EHIP;
}

lens_status lens_cnn_loss_grad(lens_cnn* c, int32_t B, const uint16_t* d_img, const float* d_target, float* d_loss,
                               float* d_grads, void* stream) {
    if (!c || !d_img || !d_target || !d_loss || B < 1 || B > c->net.max_batch) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const __bf16* img = reinterpret_cast<const __bf16*>(d_img);
    if (cnn_forward(c->net, B, img, st) != hipSuccess || cnn_backward(c->net, B, img, d_target, d_loss, st) != hipSuccess)
        return LENS_EHIP;
    if (d_grads &&
        hipMemcpyAsync(d_grads, c->net.grads, sizeof(float) * c->net.nparams, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return LENS_EHIP;
    return LENS_OK;
}

lens_status lens_cnn_train_step(lens_cnn* c, int32_t B, const uint16_t* d_img, const float* d_target, float lr,
                                float* d_loss, void* stream) {
    if (!c || !d_img || !d_target || !d_loss || !(lr > 0.0f) || B < 1 || B > c->net.max_batch) return LENS_EINVAL;
    CnnNet& n = c->net;
    hipStream_t st = (hipStream_t)stream;
    // the batch, the targets, the learning rate and the step go to net-owned
    // device memory (outside the graph); one captured step per batch size
    n.step += 1;
    if (hipMemcpyAsync(n.img_stage, d_img, sizeof(uint16_t) * B * CNN_IN * CNN_IN, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(n.tgt_stage, d_target, sizeof(float) * B * CNN_NT, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        cnn_set_hyper(n, lr, n.step, st) != hipSuccess)
        return LENS_EHIP;
    if (!n.train_graph || n.graph_batch != B) {
        if (n.train_graph) (void)hipGraphExecDestroy(n.train_graph);
        n.train_graph = nullptr;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(n.cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return LENS_EHIP;
        const hipError_t e1 = cnn_forward(n, B, n.img_stage, n.cap_stream);
        const hipError_t e2 = e1 == hipSuccess ? cnn_backward(n, B, n.img_stage, n.tgt_stage, n.loss_dev, n.cap_stream)
                                               : e1;
        const hipError_t e3 = e2 == hipSuccess ? cnn_adam(n, n.cap_stream) : e2;
        const hipError_t ec = hipStreamEndCapture(n.cap_stream, &g);
        if (e3 != hipSuccess || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return LENS_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&n.train_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            n.train_graph = nullptr;
            return LENS_EHIP;
        }
        n.graph_batch = B;
    }
    if (hipGraphLaunch(n.train_graph, st) != hipSuccess) return LENS_EHIP;
    return hipMemcpyAsync(d_loss, n.loss_dev, sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess ? LENS_OK
                                                                                                        : LENS_EHIP;
}

lens_status lens_cnn_set_target_map(lens_cnn* c, int32_t d, const float* h_prior_table, const int32_t* h_slot,
                                    const float* h_mean, const float* h_std, float sigma) {
    if (!c || d < 1 || d > CNN_MAXD || !h_prior_table || !h_slot || !h_mean || !h_std || !(sigma > 0.0f))
        return LENS_EINVAL;
    CnnTargetMap m{};
    m.d = d;
    for (int j = 0; j < d; ++j) {
        const float* r = h_prior_table + 5 * j;
        const int kind = (int)r[0];
        if (kind < LENS_PRIOR_UNIFORM || kind > LENS_PRIOR_TRUNCNORMAL) return LENS_EINVAL;
        m.prior_kind[j] = kind;
        m.prior[j][0] = r[1];
        m.prior[j][1] = r[2];
        m.prior[j][2] = r[3];
        m.prior[j][3] = r[4];
        if (h_slot[j] < -1 || h_slot[j] >= CNN_NT) return LENS_EINVAL;
        m.cnn_slot[j] = h_slot[j];
    }
    for (int k = 0; k < CNN_NT; ++k) {
        if (!(h_std[k] > 0.0f)) return LENS_EINVAL;
        m.mean[k] = h_mean[k];
        m.stdv[k] = h_std[k];
    }
    if (hipMemcpy(c->net.tmap, &m, sizeof(m), hipMemcpyHostToDevice) != hipSuccess) return LENS_EHIP;
    c->net.sigma = sigma;
    c->net.has_map = true;
    return LENS_OK;
}

lens_status init_propose(lens_cnn* c, int32_t S, const float* d_img64, int32_t n_per_system, uint64_t seed,
                         float* d_theta_out, int32_t* d_flags, void* stream) {
    if (!c || !c->net.has_map || S < 1 || !d_img64 || n_per_system < 1 || !d_theta_out) return LENS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    CnnNet& n = c->net;
    CnnTargetMap hm;
    if (hipMemcpy(&hm, n.tmap, sizeof(hm), hipMemcpyDeviceToHost) != hipSuccess) return LENS_EHIP;
    for (int s0 = 0; s0 < S; s0 += n.max_batch) {
        const int b = (S - s0) < n.max_batch ? (S - s0) : n.max_batch;
        if (cnn_prepare((long long)b * CNN_IN * CNN_IN, d_img64 + (size_t)s0 * CNN_IN * CNN_IN, n.sigma, 0, 0, 0,
                        n.prep, st) != hipSuccess ||
            cnn_forward(n, b, n.prep, st) != hipSuccess ||
            cnn_propose(b, s0, n_per_system, hm.d, n.out, n.tmap, seed,
                        d_theta_out + (size_t)s0 * n_per_system * hm.d, d_flags ? d_flags + s0 : nullptr,
                        st) != hipSuccess)
            return LENS_EHIP;
    }
    return LENS_OK;
}

lens_status lens_prior_sample(int32_t d, const float* h_prior_table, int32_t S, int32_t n_per_system,
                              uint64_t seed, float* d_theta_out, void* stream) {
    if (d < 1 || d > CNN_MAXD || !h_prior_table || S < 1 || n_per_system < 1 || !d_theta_out) return LENS_EINVAL;
    CnnTargetMap m{};
    m.d = d;
    for (int j = 0; j < d; ++j) {
        const float* r = h_prior_table + 5 * j;
        const int kind = (int)r[0];
        if (kind < LENS_PRIOR_UNIFORM || kind > LENS_PRIOR_TRUNCNORMAL) return LENS_EINVAL;
        if (kind == LENS_PRIOR_UNIFORM ? !(r[2] > r[1]) : !(r[2] > 0.0f)) return LENS_EINVAL;
        if (kind == LENS_PRIOR_TRUNCNORMAL && !(r[4] > r[3])) return LENS_EINVAL;
        m.prior_kind[j] = kind;
        for (int i = 0; i < 4; ++i) m.prior[j][i] = r[1 + i];
        m.cnn_slot[j] = -1;
    }
    hipStream_t st = (hipStream_t)stream;
    CnnTargetMap* dm = nullptr;
    if (hipMalloc(&dm, sizeof(m)) != hipSuccess) return LENS_ENOMEM;
    lens_status s = LENS_OK;
    if (hipMemcpyAsync(dm, &m, sizeof(m), hipMemcpyHostToDevice, st) != hipSuccess ||
        cnn_propose(S, 0, n_per_system, d, nullptr, dm, seed, d_theta_out, nullptr, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        s = LENS_EHIP;
    (void)hipFree(dm);
    return s;
}

}  // extern "C"
