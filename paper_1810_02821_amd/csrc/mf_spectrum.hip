// Hierarchical sampler (Sec. 5): Algorithm 1 for the signal, alternated with a
// draw of the band amplitudes theta_b of the power spectrum given the signal.
// One workgroup owns one chain pair of an N x N band-spectrum problem and runs
// every iteration on chip, like the persistent sampler.
//
// Each chain of the pair has its own amplitudes, so the Fourier-space step can
// no longer apply one real filter to the complex pair field Z = Z_A + i Z_B.
// With f_+- = (f_A +- f_B)/2 and w_+- = (w_A +- w_B)/2 (real and even in k),
//     S(k) = f_+ Z(k) + f_- conj(Z(-k)) + w_+ eta(k) + w_- conj(eta(-k))
// gives chain A (real part of the inverse transform) the update f_A Z_A + w_A
// noise and chain B (imaginary part) f_B Z_B + w_B noise, exactly.  The
// mirrored values Z(-k) and eta(-k) come through LDS.
//
// The amplitudes given the signal are inverse-gamma: theta_b = (2 beta_0 +
// sigma_b / n^2) / x_b, with sigma_b the band power of the chain's signal and
// x_b a chi-square variate of m_b + nu_0 degrees of freedom, the sum of squared
// normals from stage 3 of the stream (flat index over the bands' degrees of
// freedom, counter word 1 = the global iteration).
#include "mf_device.hpp"
#include "mf_resident.hpp"
#include "mf_resident_fft.hpp"
#include "mf_spectrum.hpp"

namespace mf {

namespace {

constexpr uint32_t kStageSpectrum = 3;
constexpr int kNB = kMaxBandsPerProblem;

struct SpecShared {
    float4 coef[kNB];      // (f_A/n, w_A/n, f_B/n, w_B/n) per band
    double theta[2][kNB];  // current amplitudes, chains A and B
    double pw[2][kNB];     // band powers of the last signal, in units of n^2
    double chi[2][kNB];    // chi-square sums
    int32_t dof[kNB];      // degrees of freedom per band
    int32_t pre[kNB + 1];  // their prefix sums (flat index of each band's first variate)
};

template <int N>
__device__ __forceinline__ unsigned mirror(unsigned ky, unsigned kx) {
    return ((N - ky) & (N - 1)) * N + ((N - kx) & (N - 1));
}

// f/n and w/n of both chains for every band, from the current amplitudes.
__device__ __forceinline__ void refresh_coef(SpecShared& sh, int nb, double T, double n) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        float c[4];
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            const double nP = n * sh.theta[ch][b];
            const double f = nP / (nP + T);
            const double w = sqrt(n * nP * T / (nP + T));
            c[2 * ch] = (float)(f / n);
            c[2 * ch + 1] = (float)(w / n);
        }
        sh.coef[b] = make_float4(c[0], c[1], c[2], c[3]);
    }
}

// Fourier-space step on layout D (thread (k1, jx) holds modes (k1 + P k2, 2 jx + q)
// at v[8 q + k2]); on return v holds S(k)/n.  Every thread must call it.
template <int N>
__device__ __forceinline__ void harmonic_pair(float2 (&v)[16], float2* lds, const SpectrumArgs& a,
                                              const ProbDev& pr, const SpecShared& sh, uint32_t sweep,
                                              int pair, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
    const int16_t* band = a.band + pr.pix_off;
    __syncthreads();  // other threads may still read the forward transform's last exchange
    // 1. Z to LDS in natural mode order
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
        *reinterpret_cast<float4*>(lds + ky * N + 2 * jx) = make_float4(v[k2].x, v[k2].y, v[8 + k2].x, v[8 + k2].y);
    }
    __syncthreads();
    // 2. filter part: f_+ Z(k) + f_- conj(Z(-k))
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned kx = 2 * jx + q;
            const float4 c = sh.coef[band[ky * N + kx]];
            const float fp = 0.5f * (c.x + c.z), fm = 0.5f * (c.x - c.z);
            const float2 zm = lds[mirror<N>(ky, kx)];
            float2& z = v[8 * q + k2];
            z = make_float2(fmaf(fp, z.x, fm * zm.x), fmaf(fp, z.y, -fm * zm.y));
        }
    }
    __syncthreads();
    // 3. noise part: w_+ eta(k), and eta to LDS for the mirrored term
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const unsigned ky = k1 + P * k2;
        const uint32_t e2 = (uint32_t)(ky * (N / 2) + jx);
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStageHarmonic, (uint32_t)pair, a.key0, a.key1);
        *reinterpret_cast<float4*>(lds + ky * N + 2 * jx) = make_float4(z.a.x, z.a.y, z.b.x, z.b.y);
        const float4 c0 = sh.coef[band[ky * N + 2 * jx]];
        const float4 c1 = sh.coef[band[ky * N + 2 * jx + 1]];
        const float wp0 = 0.5f * (c0.y + c0.w), wp1 = 0.5f * (c1.y + c1.w);
        v[k2] = make_float2(fmaf(wp0, z.a.x, v[k2].x), fmaf(wp0, z.a.y, v[k2].y));
        v[8 + k2] = make_float2(fmaf(wp1, z.b.x, v[8 + k2].x), fmaf(wp1, z.b.y, v[8 + k2].y));
    }
    __syncthreads();
    // 4. w_- conj(eta(-k))
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned kx = 2 * jx + q;
            const float4 c = sh.coef[band[ky * N + kx]];
            const float wm = 0.5f * (c.y - c.w);
            const float2 em = lds[mirror<N>(ky, kx)];
            float2& z = v[8 * q + k2];
            z = make_float2(fmaf(wm, em.x, z.x), fmaf(-wm, em.y, z.y));
        }
    }
    __syncthreads();
}

// Band powers of both chains of the signal S/n held on layout D:
// X_A = (S(k) + conj S(-k))/2, X_B = (S(k) - conj S(-k))/(2i).
template <int N>
__device__ __forceinline__ void band_powers(const float2 (&v)[16], float2* lds, const SpectrumArgs& a,
                                            const ProbDev& pr, SpecShared& sh, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
    const int16_t* band = a.band + pr.pix_off;
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
        *reinterpret_cast<float4*>(lds + ky * N + 2 * jx) = make_float4(v[k2].x, v[k2].y, v[8 + k2].x, v[8 + k2].y);
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
        int b[2];
        double pa[2], pb[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned kx = 2 * jx + q;
            b[q] = band[ky * N + kx];
            const float2 s = v[8 * q + k2];
            const float2 m = lds[mirror<N>(ky, kx)];
            const double ar = 0.5 * ((double)s.x + m.x), ai = 0.5 * ((double)s.y - m.y);
            const double br = 0.5 * ((double)s.y + m.y), bi = 0.5 * ((double)s.x - m.x);
            pa[q] = ar * ar + ai * ai;
            pb[q] = br * br + bi * bi;
        }
        // the two modes of a thread are neighbours in k_x and mostly share a band
        if (b[0] == b[1]) {
            atomicAdd(&sh.pw[0][b[0]], pa[0] + pa[1]);
            atomicAdd(&sh.pw[1][b[0]], pb[0] + pb[1]);
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                atomicAdd(&sh.pw[0][b[q]], pa[q]);
                atomicAdd(&sh.pw[1][b[q]], pb[q]);
            }
        }
    }
    __syncthreads();
}

// chi-square sums: thread tid owns a contiguous chunk of the flat variate index.
template <int N>
__device__ __forceinline__ void chi_square(const SpectrumArgs& a, const ProbDev& pr, SpecShared& sh, int nb,
                                           uint32_t iteration, int pair, unsigned tid) {
    constexpr int NT = Res<N>::NT;
    const int total = sh.pre[nb];
    const int chunk = 2 * ((total + 2 * NT - 1) / (2 * NT));
    const int e0 = (int)tid * chunk;
    if (e0 >= total) return;
    const int e1 = min(total, e0 + chunk);
    int b = 0;
    while (sh.pre[b + 1] <= e0) ++b;
    double accA = 0.0, accB = 0.0;
    for (int e = e0; e < e1; e += 2) {
        const Normals2 z = pair_normals((uint32_t)(e >> 1), iteration, (uint32_t)pr.pid, kStageSpectrum,
                                        (uint32_t)pair, a.key0, a.key1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ee = e + h;
            if (ee >= e1) break;
            if (ee >= sh.pre[b + 1]) {
                atomicAdd(&sh.chi[0][b], accA);
                atomicAdd(&sh.chi[1][b], accB);
                accA = accB = 0.0;
                while (sh.pre[b + 1] <= ee) ++b;
            }
            const float2 zz = h ? z.b : z.a;
            accA += (double)zz.x * zz.x;
            accB += (double)zz.y * zz.y;
        }
    }
    atomicAdd(&sh.chi[0][b], accA);
    atomicAdd(&sh.chi[1][b], accB);
}

template <int N>
__global__ __launch_bounds__(Res<N>::NT, 4) void resident_spectrum_kernel(SpectrumArgs a) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT;
    __shared__ __align__(16) float2 lds[Res<N>::LDS];
    __shared__ SpecShared sh;
    __shared__ float2 twl[Res<N>::TWS];  // twiddle tables of the four passes
    const unsigned tid = threadIdx.x;
    fill_twiddle_tables<N>(twl, a.tw, tid);
    __syncthreads();
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
    const int nb = a.band_count[it.prob];
    const int bbase = a.band_base[it.prob];
    const double n = (double)N * N;
    const double T = pr.tau;
    const int c0 = 2 * it.pair, c1 = 2 * it.pair + 1;

    // amplitudes, degrees of freedom, coefficient table
    for (int t = tid; t < 2 * nb; t += NT) {
        const int ch = t / nb, b = t % nb;
        const int c = ch ? c1 : c0;
        sh.theta[ch][b] = a.theta_in ? a.theta_in[(int64_t)a.chains_pad * bbase + (int64_t)c * nb + b]
                                     : a.theta0[bbase + b];
        sh.pw[ch][b] = 0.0;
        sh.chi[ch][b] = 0.0;
    }
    if (tid == 0) {
        int acc = 0;
        for (int b = 0; b < nb; ++b) {
            sh.dof[b] = a.dof[bbase + b];
            sh.pre[b] = acc;
            acc += sh.dof[b];
        }
        sh.pre[nb] = acc;
    }
    __syncthreads();
    refresh_coef(sh, nb, T, n);

    float2 v[16];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int x = 2 * j + P * m;
        if (a.state_in) {
            v[m] = a.state_in[it.field_off + (int64_t)y * N + x];
            v[8 + m] = a.state_in[it.field_off + (int64_t)y * N + x + 1];
        } else if (a.init_scale > 0.f) {
            const uint32_t e2 = (uint32_t)((y * N + x) >> 1);
            const Normals2 z = pair_normals(e2, 0u, (uint32_t)pr.pid, kStageInit, (uint32_t)it.pair, a.key0, a.key1);
            v[m] = cscale(z.a, a.init_scale);
            v[8 + m] = cscale(z.b, a.init_scale);
        } else {
            v[m] = v[8 + m] = make_float2(0.f, 0.f);
        }
    }
    __syncthreads();

    const int64_t iters = (int64_t)a.burn_in + (int64_t)a.n_samples * a.thin;
    for (int64_t i = 0; i < iters; ++i) {
        const uint32_t g = a.iter0 + (uint32_t)i;
        for (int k = 0; k < a.sweeps; ++k) {
            const uint32_t sweep = g * (uint32_t)a.sweeps + (uint32_t)k;
            const float4* pcoef = per_sweep(a.pcoef);
            const float2* psrc = per_sweep(a.psrc);
            const float2* tw = twl + per_sweep_zero();
            unsigned t = tid;
            asm volatile("" : "+v"(t));
            {
                // pixel step t = (1-a) s + a d + sqrt(T(1-a)) xi (spectrum-independent tables)
                const unsigned yy = t / (P / 2), jj = t % (P / 2);
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    __builtin_amdgcn_sched_barrier(0);
                    const uint32_t e2 = (uint32_t)(yy * (N / 2) + jj + (P / 2) * m);
                    const int64_t pp = pr.pix_off / 2 + e2;
                    const float4 c = pcoef[pp];
                    const float2 src = psrc[pp];
                    const Normals2 z =
                        pair_normals(e2, sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)it.pair, a.key0, a.key1);
                    float2& s0 = v[m];
                    float2& s1 = v[8 + m];
                    s0.x = fmaf(c.x, s0.x, fmaf(c.y, z.a.x, src.x));
                    s0.y = fmaf(c.x, s0.y, fmaf(c.y, z.a.y, src.x));
                    s1.x = fmaf(c.z, s1.x, fmaf(c.w, z.b.x, src.y));
                    s1.y = fmaf(c.z, s1.y, fmaf(c.w, z.b.y, src.y));
                }
            }
            forward_fft<N>(v, lds, tw, t);
            unsigned t2 = tid;
            asm volatile("" : "+v"(t2));
            harmonic_pair<N>(v, lds, a, pr, sh, sweep, it.pair, t2);
            if (k == a.sweeps - 1) {
                // spectrum draw from this signal: band powers, chi-square sums, new amplitudes
                band_powers<N>(v, lds, a, pr, sh, t2);
                chi_square<N>(a, pr, sh, nb, g, it.pair, t2);
                __syncthreads();
                const bool emit = i >= a.burn_in && ((i - a.burn_in + 1) % a.thin) == 0;
                const int64_t slot = emit ? (i - a.burn_in + 1) / a.thin - 1 : 0;
                for (int u = tid; u < 2 * nb; u += NT) {
                    const int ch = u / nb, b = u % nb;
                    const double x = sh.chi[ch][b];
                    if (sh.dof[b] > 0 && x > 0.0) sh.theta[ch][b] = (2.0 * a.prior_beta + sh.pw[ch][b]) / x;
                    sh.pw[ch][b] = 0.0;
                    sh.chi[ch][b] = 0.0;
                    const int c = ch ? c1 : c0;
                    if (emit && a.theta_samples && c < a.chains)
                        a.theta_samples[(int64_t)a.chains * a.n_samples * bbase +
                                        ((int64_t)c * a.n_samples + slot) * nb + b] = sh.theta[ch][b];
                }
                __syncthreads();
                refresh_coef(sh, nb, T, n);
                __syncthreads();
            }
            inverse_fft<N>(v, lds, tw, t2);
        }
        if (a.samples && i >= a.burn_in && ((i - a.burn_in + 1) % a.thin) == 0) {
            const int64_t slot = (i - a.burn_in + 1) / a.thin - 1;
            const int64_t nn = (int64_t)N * N;
            const int64_t base = (int64_t)a.chains * a.n_samples * pr.pix_off;
            float* o0 = a.samples + base + ((int64_t)c0 * a.n_samples + slot) * nn + (int64_t)y * N;
            float* o1 = a.samples + base + ((int64_t)c1 * a.n_samples + slot) * nn + (int64_t)y * N;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int x = 2 * j + P * m;
                *reinterpret_cast<float2*>(o0 + x) = make_float2(v[m].x, v[8 + m].x);
                if (c1 < a.chains) *reinterpret_cast<float2*>(o1 + x) = make_float2(v[m].y, v[8 + m].y);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int64_t o = it.field_off + (int64_t)y * N + 2 * j + P * m;
        a.field[o] = v[m];
        a.field[o + 1] = v[8 + m];
    }
    if (a.theta_out)
        for (int u = tid; u < 2 * nb; u += NT) {
            const int ch = u / nb, b = u % nb;
            const int c = ch ? c1 : c0;
            a.theta_out[(int64_t)a.chains_pad * bbase + (int64_t)c * nb + b] = sh.theta[ch][b];
        }
}

}  // namespace

hipError_t launch_resident_spectrum(int N, const SpectrumArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.n_items);
    switch (N) {
        case 32: hipLaunchKernelGGL(resident_spectrum_kernel<32>, grid, dim3(Res<32>::NT), 0, s, a); break;
        case 64: hipLaunchKernelGGL(resident_spectrum_kernel<64>, grid, dim3(Res<64>::NT), 0, s, a); break;
        case 128: hipLaunchKernelGGL(resident_spectrum_kernel<128>, grid, dim3(Res<128>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
