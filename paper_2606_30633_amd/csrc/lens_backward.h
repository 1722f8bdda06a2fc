// Internal declarations of the backward ("linear inversion") likelihood (lens_backward.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace lens {

constexpr int BWD_MAX_K = 6;                  // light components (3 lens light + 3 source)
constexpr double BWD_PIVOT_REL = 1e-12;       // pivot threshold, relative to the largest diagonal of M

// Positions of the K intensities in a parameter vector of length d.
struct BwdSlots {
    int K, d;
    int slot[BWD_MAX_K];
};

// thx[(p K + k)][j] = theta[p][j], with the intensities set to 1 for component k and 0 otherwise.
hipError_t launch_bwd_expand(int P, const BwdSlots& s, const float* theta, float* thx, hipStream_t st);
// Per particle: normal equations from the K unit-intensity model images B [(p K + k)][npix], solve,
// theta_full = theta with the intensities replaced by the solution; amp [P][K] (optional).
hipError_t launch_bwd_normal(int P, const BwdSlots& s, int npix, const float* B, const float* data,
                             const float* invvar, const float* consts_expanded, const float* theta,
                             float* theta_full, float* amp, hipStream_t st);
// grad[p][slot] = 0 for every intensity slot.
hipError_t launch_bwd_zero_slots(int P, const BwdSlots& s, float* grad, hipStream_t st);

}  // namespace lens
