// Mass mapping: messenger filter and sampler for complex shear data and the
// spin-2 operator; persistent form (H = W <= 128) and streamed form.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_kernels.hpp"

namespace mf {

struct ShearArgs {
    const ProbDev* probs;
    const ItemDev* items;     // one per (problem, chain); .pair = chain
    int32_t n_items;
    const float2* gamma;      // concatenated complex shear data
    const float* nbar;        // concatenated Nbar per component (+inf missing)
    const float* nP;          // concatenated n P_E(|k|)
    float b_ratio;            // P_B / P_E
    const float2* tw;         // W_N^r, r < N
    uint32_t key0, key1;
    uint32_t sweep0;          // global index of the first sweep
    int32_t stochastic;       // 1: sampler, 0: Wiener filter
    Levels lv;                // cooling levels (by value)
    int32_t burn_in, n_samples, thin;
    float2* samples;          // [problem][chain][sample][H][W] kappa, or null
    int32_t chains;
    const float2* state_in;   // model shear A kappa per chain, or null (zero)
    float2* state_out;        // or null
    float2* kappa_out;        // kappa after the last sweep (filter), or null
};

hipError_t launch_resident_shear(int N, const ShearArgs& a, hipStream_t s);

// Streamed form (size classes the persistent kernel does not hold): per sweep
// a row kernel (inverse row FFT, shear-space pixel step, forward row FFT) and
// a column kernel over mirror-paired column tiles (forward column FFT, E/B
// Fourier step, multiplication by D, inverse column FFT).  On a sweep that
// emits kappa the column kernel also writes F_col^-1(kappa^) to `kfield` and
// an emission kernel finishes the inverse transform into `out`.
struct ShearStreamArgs {
    const ProbDev* probs;
    const ItemDev* items;     // one per (problem, chain); .pair = chain
    int32_t n_items;
    float2* field;            // chain fields (shear space), items' layout
    float2* kfield;           // kappa staging, same layout
    const float2* gamma;      // concatenated complex shear data
    const float* nbar;        // concatenated Nbar per component (+inf missing)
    const float* nP;          // concatenated n P_E(|k|)
    const float2* nPt;        // column-pair copy: [pix_off/2 + (kx/2) H + ky] = (nP(ky,kx), nP(ky,kx+1))
    float b_ratio;
    const float2* tw_row;     // W_W^r
    const float2* tw_col;     // W_H^r
    uint32_t key0, key1;
    uint32_t sweep;           // global sweep index
    float lambda;             // cooling level: T = lambda * tau
    int32_t stochastic;
    int32_t emit;             // column kernel: stage kappa this sweep
    // emission kernel: kappa to samples [problem][chain][sample][H][W] (slot >= 0) or kappa_out
    float2* samples;
    int32_t chains, n_samples, slot;
    float2* kappa_out;
};

enum ShearRowMode : int32_t { kShearInv = 1, kShearFwd = 2, kShearInvFwd = 3, kShearEmit = 4 };
hipError_t launch_shear_row(int W, int H, int mode, const ShearStreamArgs& a, hipStream_t s);
hipError_t launch_shear_col(int W, int H, const ShearStreamArgs& a, hipStream_t s);
// field <- state_in (or zero) for every item
hipError_t launch_shear_init(int W, int H, const ShearStreamArgs& a, const float2* state_in, hipStream_t s);

}  // namespace mf
