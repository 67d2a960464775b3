// Persistent LDS-resident form of the sampler: one workgroup keeps one chain
// pair's whole image on chip for every sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_kernels.hpp"

namespace mf {

struct ResidentArgs {
    const ProbDev* probs;
    const ItemDev* items;
    int32_t n_items;
    float2* field;            // final pair states [item] (pixel space)
    const float2* state_in;   // start states or null
    float init_scale;         // dispersed starts when state_in is null and > 0
    const float4* pcoef;      // per pixel pair: (1-a, sqrt(T(1-a))) x 2
    const float2* psrc;       // per pixel pair: a d x 2
    const float4* mcoef;      // per mode pair: (f/n, w/n) x 2
    const float2* tw;         // W_N^r, r < N
    uint32_t key0, key1;
    uint32_t sweep0;          // global index of the first sweep
    int32_t burn_in, n_samples, thin;
    float* samples;           // [problem][chain][sample][H][W] or null
    int32_t chains;
};

// Deterministic messenger solve (Wiener filter / adjoint) of one problem per
// workgroup, cooling levels and the residual test on the device.
struct SolveArgs {
    const ProbDev* probs;
    const ItemDev* items;     // one per problem
    int32_t n_items;
    const float* src;         // concatenated d (kSrcData) or g (kSrcGrad)
    int32_t src_kind;
    const float* s_init;      // concatenated start, or null for zero
    float* s_out;             // concatenated result
    const float* nbar;        // concatenated Nbar (+inf missing)
    const float* nP;          // concatenated n P(|k|)
    const float2* tw;         // W_N^r, r < N
    Levels lv;                // cooling levels of this launch
    int32_t total0;           // sweeps run by earlier launches of the same solve
    double tol;               // residual tolerance of the final level (<= 0: none; only in the last launch)
    int32_t max_sweeps;
    int32_t check_every;
    double* info;             // [item][3]: sweeps run, converged (1, 0, or -1 non-finite), last residual
};

bool resident_supported(int H, int W);
hipError_t launch_resident_solve(int N, const SolveArgs& a, hipStream_t s);
hipError_t launch_resident_sample(int N, const ResidentArgs& a, hipStream_t s);
// Build the sampler's per-call coefficient tables (lambda = 1) for every problem.
hipError_t launch_sampler_coefs(const ProbDev* probs, int n_problems, const float* d, const float* nbar,
                                const float* nP, float4* pcoef, float2* psrc, float4* mcoef, hipStream_t s);

}  // namespace mf
