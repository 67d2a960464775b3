// Mass mapping: messenger filter and sampler for complex shear data and the
// spin-2 operator, persistent form (H = W <= 128).
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
    const double* lambda;     // [n_levels] cooling levels
    const int32_t* level_sweeps;
    int32_t n_levels;
    int32_t burn_in, n_samples, thin;
    float2* samples;          // [problem][chain][sample][H][W] kappa, or null
    int32_t chains;
    const float2* state_in;   // model shear A kappa per chain, or null (zero)
    float2* state_out;        // or null
    float2* kappa_out;        // kappa after the last sweep (filter), or null
};

hipError_t launch_resident_shear(int N, const ShearArgs& a, hipStream_t s);

}  // namespace mf
