// Allocation-free logL + gradient: the kernels and launch sequence of
// lens_loglike_grad, with every scratch buffer carved out of one fixed
// static device array instead of a plan's hipMalloc'd buffers.
//
// The array's name is only a host-side stand-in for a device symbol: host
// code never passes it to a kernel or a copy.  The device address of each
// GPU's copy is looked up once per device with hipGetSymbolAddress (with
// that device current) and every launch takes that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lens_internal.h"

// Per-GPU scratch of the allocation-free entry point (LENS_NOALLOC_SCRATCH_BYTES).
static __device__ __align__(256) unsigned char scratch[LENS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device address of the current device's scratch array, looked up on the
// first call on that device.
lens_status scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LENS_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LENS_EHIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LENS_OK;
}

}  // namespace

using namespace lens;

extern "C" lens_status lens_loglike_grad_noalloc(const lens_model_desc* desc, const float* d_psf,
                                                 const float* d_data, const float* d_invvar, int32_t P,
                                                 const float* d_theta, float* d_logl, float* d_grad,
                                                 double* d_logl64, void* stream) {
    if (!desc_valid(desc) || !d_psf || !d_data || !d_invvar || !d_theta || !d_logl || !d_grad || P < 1)
        return LENS_EINVAL;
    const ModelInfo mi = model_info(*desc);
    const Geo g = make_geo(*desc);
    const int K = desc->psf_size;
    if (psf_lds_bytes(g, K) > MAX_LDS_BYTES) return LENS_EUNSUPPORTED;
    // the launch shape of a plan at its default of 4 pixels per thread
    constexpr int kPpt = 4;
    const int nch = chunks_for(g.npix, kPpt);
    const int nacc = n_acc(mi);
    const size_t b_flip = align256(sizeof(double) * (size_t)K * K);
    const size_t b_consts = align256(sizeof(float) * (size_t)CSTRIDE * (size_t)P);
    const size_t b_img = align256(sizeof(float) * (size_t)g.npix * (size_t)P);
    const size_t b_part = align256(sizeof(double) * (size_t)P * nch * nacc);
    if (b_flip + b_consts + b_img + b_part > (size_t)LENS_NOALLOC_SCRATCH_BYTES) return LENS_ESCRATCH;

    void* base = nullptr;
    const lens_status s = scratch_ptr(&base);
    if (s != LENS_OK) return s;
    unsigned char* b = static_cast<unsigned char*>(base);
    double* flip = reinterpret_cast<double*>(b);
    float* consts = reinterpret_cast<float*>(b + b_flip);
    float* img = reinterpret_cast<float*>(b + b_flip + b_consts);
    double* part = reinterpret_cast<double*>(b + b_flip + b_consts + b_img);

    // Every scratch word a kernel reads is written earlier in this sequence
    // (flip, constants, images, partial rows), so nothing needs clearing.
    hipStream_t st = (hipStream_t)stream;
    if (launch_flip(K, d_psf, flip, st) != hipSuccess) return LENS_EHIP;
    if (launch_prologue(mi, P, d_theta, consts, st) != hipSuccess) return LENS_EHIP;
    if (launch_render(mi, g, P, kPpt, consts, img, st) != hipSuccess) return LENS_EHIP;
    if (launch_psf(mi, g, K, 2, P, consts, img, flip, d_psf, d_data, d_invvar, nullptr, d_logl, d_logl64, st) !=
        hipSuccess)
        return LENS_EHIP;
    if (launch_adjoint(mi, g, P, kPpt, consts, img, part, st) != hipSuccess) return LENS_EHIP;
    if (launch_finalize(mi, P, nch, d_theta, consts, part, d_grad, st) != hipSuccess) return LENS_EHIP;
    return LENS_OK;
}
