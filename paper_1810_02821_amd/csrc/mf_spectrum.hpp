// Hierarchical sampler: the persistent sampler's sweep alternated with the
// draw of band amplitudes of the power spectrum given the signal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_kernels.hpp"

namespace mf {

struct SpectrumArgs {
    const ProbDev* probs;
    const ItemDev* items;     // one per (problem, pair)
    int32_t n_items;
    float2* field;            // final pair states
    const float2* state_in;   // start states or null
    float init_scale;
    const float4* pcoef;      // sampler pixel tables (lambda = 1)
    const float2* psrc;
    const float2* tw;         // W_N^r, r < N
    uint32_t key0, key1;
    uint32_t iter0;           // global index of the first iteration
    int32_t sweeps;           // messenger sweeps per iteration
    int32_t burn_in, n_samples, thin;
    float* samples;           // [problem][chain][sample][H][W] or null
    int32_t chains;           // chains per problem
    int32_t chains_pad;       // 2 * pairs: chain slots of theta_in / theta_out
    const int16_t* band;      // per-mode band index (concatenated)
    const int32_t* band_base; // first band of each problem
    const int32_t* band_count;// bands of each problem
    const int32_t* dof;       // degrees of freedom per band (concatenated)
    const double* theta0;     // plan amplitudes per band (start when theta_in is null)
    const double* theta_in;   // [problem][chain_pad][band] or null
    double* theta_out;        // [problem][chain_pad][band] or null
    double* theta_samples;    // [problem][chain][sample][band] or null
    double prior_beta;
};

hipError_t launch_resident_spectrum(int N, const SpectrumArgs& a, hipStream_t s);

}  // namespace mf
