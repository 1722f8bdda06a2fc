// Internal declarations of the backward ("linear inversion") likelihood (lens_backward.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace lens {

constexpr int BWD_SMALL_K = 6;                // light components solved in registers (Sersic only)
constexpr int BWD_MAX_K = 51;                 // with a shapelet source: 1 + 1 Sersic + 45 coefficients
constexpr double BWD_PIVOT_REL = 1e-12;       // pivot threshold, relative to the largest diagonal of M

// Positions of the K intensities in a parameter vector of length d.
struct BwdSlots {
    int K, d;
    int slot[BWD_MAX_K];
};

// th1[p][j] = theta[p][j], with every intensity set to 1.
hipError_t launch_bwd_expand(int P, const BwdSlots& s, const float* theta, float* th1, hipStream_t st);
// Per particle: normal equations from the K unit-intensity model images B [(p K + k)][npix], solve,
// theta_full = theta with the intensities replaced by the solution; amp [P][K] (optional);
// consts: the particles' constants (their validity flags).
hipError_t launch_bwd_normal(int P, const BwdSlots& s, int npix, const float* B, const float* data,
                             const float* invvar, const float* consts, const float* theta,
                             float* theta_full, float* amp, hipStream_t st);
// out [P][npix] = sum_k A_k comp[(p K + k)] with A_k read from theta_full's intensity slots.
hipError_t launch_bwd_assemble(int P, const BwdSlots& s, int npix, const float* comp, const float* theta_full,
                               float* out, hipStream_t st);
// grad[p][slot] = 0 for every intensity slot.
hipError_t launch_bwd_zero_slots(int P, const BwdSlots& s, float* grad, hipStream_t st);

}  // namespace lens
