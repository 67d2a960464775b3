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

// Streamed form (any size class): the streamed sampler's row kernel for the
// pixel step, a column kernel over mirror-paired column tiles for the Fourier
// step with per-chain amplitudes, and small kernels for the amplitude draw.
// Per-item state: theta, band powers and chi-square sums [item][2][kNB]
// (FP64), coefficients [item][kNB] (float4 f_A/n, w_A/n, f_B/n, w_B/n).
struct SpectrumStreamArgs {
    const ProbDev* probs;
    const ItemDev* items;
    int32_t n_items;
    float2* field;            // pair fields, items' layout
    const float2* tw_col;     // W_H^r
    const int16_t* band;      // per-mode band index (concatenated)
    const int16_t* bandt;     // the same, column-major per problem: [pix_off + kx H + ky]
    const int32_t* band_base;
    const int32_t* band_count;
    const int32_t* dof;
    const double* theta0;     // plan amplitudes per band
    const double* theta_in;   // [problem][chain_pad][band] or null
    double* theta_out;        // [problem][chain_pad][band] or null
    double* theta_samples;    // [problem][chain][sample][band] or null
    double* theta;            // per-item amplitudes
    double* pw;               // per-item band powers
    double* chi;              // per-item chi-square sums
    float4* coef;             // per-item coefficient tables
    uint32_t key0, key1;
    uint32_t sweep;           // global sweep index (column kernel)
    uint32_t iteration;       // global iteration index (chi-square draw)
    int32_t add_power;        // 1: the column kernel adds the band powers of its result to pw
    int32_t chains, chains_pad, n_samples;
    double prior_beta;
};

// Amplitudes from theta_in / theta0, cleared sums, coefficients, theta_out.
hipError_t launch_spectrum_init(const SpectrumStreamArgs& a, hipStream_t s);
// Column FFT, Fourier step with per-chain amplitudes, band powers when
// a.add_power is set, inverse column FFT (H in 16..2048, W a power of two >= 16).
hipError_t launch_spectrum_col(int W, int H, const SpectrumStreamArgs& a, hipStream_t s);
// Chi-square sums of iteration a.iteration and the new amplitudes; slot >= 0
// writes theta samples to that sample slot.
hipError_t launch_spectrum_draw(const SpectrumStreamArgs& a, int max_total_dof, int64_t slot, hipStream_t s);

}  // namespace mf
