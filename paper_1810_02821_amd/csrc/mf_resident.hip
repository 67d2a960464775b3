// Persistent LDS-resident sampler: one workgroup owns one chain pair of an
// N x N image and runs every sweep of Algorithm 1 without leaving the chip;
// only emitted samples and the final state reach HBM.  The field stays in
// registers between the passes of the 2D FFT (mf_resident_fft.hpp).
#include "mf_device.hpp"
#include "mf_resident.hpp"
#include "mf_resident_fft.hpp"

namespace mf {

namespace {

// --------------------------------------------------------------- updates --
// Pixel-space messenger draw on layout A: t = (1-a) s + a d + sqrt(T(1-a)) xi,
// with (1-a, sqrt(T(1-a))) and a d read from per-call tables.
template <int N>
__device__ __forceinline__ void pixel_update(float2 (&v)[16], const ResidentArgs& a, const ProbDev& pr, int pair,
                                             uint32_t sweep, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        // keep the eight Philox chains from being interleaved (register pressure)
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t e2 = (uint32_t)(y * (N / 2) + j + (P / 2) * m);  // pixel pair index in the image
        const int64_t pp = pr.pix_off / 2 + e2;
        const float4 c = a.pcoef[pp];   // (1-a, sigma) of pixels x, x+1
        const float2 src = a.psrc[pp];  // a d of pixels x, x+1
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)pair, a.key0, a.key1);
        float2& s0 = v[m];
        float2& s1 = v[8 + m];
        s0.x = fmaf(c.x, s0.x, fmaf(c.y, z.a.x, src.x));
        s0.y = fmaf(c.x, s0.y, fmaf(c.y, z.a.y, src.x));
        s1.x = fmaf(c.z, s1.x, fmaf(c.w, z.b.x, src.y));
        s1.y = fmaf(c.z, s1.y, fmaf(c.w, z.b.y, src.y));
    }
}

// Fourier-space draw on layout D: S = (f T + w eta) / n, (f/n, w/n) from a table.
template <int N>
__device__ __forceinline__ void harmonic_update(float2 (&v)[16], const ResidentArgs& a, const ProbDev& pr, int pair,
                                                uint32_t sweep, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const unsigned ky = k1 + P * k2;
        const uint32_t e2 = (uint32_t)(ky * (N / 2) + jx);  // mode pair index
        const float4 c = a.mcoef[pr.pix_off / 2 + e2];     // (f, w) of modes kx, kx+1
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStageHarmonic, (uint32_t)pair, a.key0, a.key1);
        float2& s0 = v[k2];
        float2& s1 = v[8 + k2];
        s0.x = fmaf(c.x, s0.x, c.y * z.a.x);
        s0.y = fmaf(c.x, s0.y, c.y * z.a.y);
        s1.x = fmaf(c.z, s1.x, c.w * z.b.x);
        s1.y = fmaf(c.z, s1.y, c.w * z.b.y);
    }
}

template <int N>
__global__ __launch_bounds__(Res<N>::NT, 4) void resident_sample_kernel(ResidentArgs a) {
    constexpr int P = Res<N>::P;
    __shared__ __align__(16) float2 lds[Res<N>::LDS];
    __shared__ float2 twl[Res<N>::TWS];  // twiddle tables of the four passes
    const unsigned tid = threadIdx.x;
    fill_twiddle_tables<N>(twl, a.tw, tid);
    __syncthreads();  // the first forward pass reads twiddles before any exchange barrier
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const unsigned y = tid / (P / 2), j = tid % (P / 2);

    // initial state in layout A
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

    const int64_t n = (int64_t)N * N;
    const int64_t K = (int64_t)a.burn_in + (int64_t)a.n_samples * a.thin;
    const int c0 = 2 * it.pair, c1 = 2 * it.pair + 1;
    for (int64_t k = 0; k < K; ++k) {
        const uint32_t sweep = a.sweep0 + (uint32_t)k;
        ResidentArgs ak = a;
        ak.pcoef = per_sweep(a.pcoef);
        ak.psrc = per_sweep(a.psrc);
        ak.mcoef = per_sweep(a.mcoef);
        const float2* tw = twl + per_sweep_zero();
        // The first half of the sweep (pixel draw, forward FFT) keeps what it
        // indexes by the thread id (LDS bases, counter words) live across
        // sweeps; the second half recomputes its own from an opaque copy of
        // the id each sweep, since keeping both halves' live spills registers
        // (16 complex values per thread, 4 waves per SIMD).
        unsigned t = tid;
        pixel_update<N>(v, ak, pr, it.pair, sweep, t);
        forward_fft<N>(v, lds, tw, t);
        unsigned t2 = tid;
        asm volatile("" : "+v"(t2));
        harmonic_update<N>(v, ak, pr, it.pair, sweep, t2);
        inverse_fft<N>(v, lds, tw, t2);
        if (a.samples && k >= a.burn_in && ((k - a.burn_in + 1) % a.thin) == 0) {
            const int64_t slot = (k - a.burn_in + 1) / a.thin - 1;
            const int64_t base = (int64_t)a.chains * a.n_samples * pr.pix_off;
            float* o0 = a.samples + base + ((int64_t)c0 * a.n_samples + slot) * n + (int64_t)y * N;
            float* o1 = a.samples + base + ((int64_t)c1 * a.n_samples + slot) * n + (int64_t)y * N;
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
}

// Per-call coefficient tables of the sampler at lambda = 1 (pairs of elements):
//   pcoef = (1 - a, sqrt(T (1 - a))) for pixels 2e, 2e+1;  psrc = a d
//   mcoef = (f / n, w / n) for modes 2e, 2e+1 with f = nP/(nP+T), w = sqrt(n nP T/(nP+T))
__global__ void sampler_coef_kernel(const ProbDev* probs, const float* d, const float* nbar, const float* nP,
                                    float4* pcoef, float2* psrc, float4* mcoef) {
    const ProbDev pr = probs[blockIdx.y];
    const int64_t n = (int64_t)pr.H * pr.W;
    const double T = pr.tau;
    const double inv_n = 1.0 / (double)n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n / 2; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = pr.pix_off + 2 * e;
        float oma[2], sig[2], src[2], f[2], w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double nb = nbar[g + q];
            const double aa = isinf(nb) ? 0.0 : T / (T + nb);
            oma[q] = (float)(1.0 - aa);
            sig[q] = (float)sqrt(T * (1.0 - aa));
            src[q] = aa > 0.0 ? (float)(aa * (double)d[g + q]) : 0.f;
            const double P = nP[g + q];
            f[q] = (float)(P / (P + T) * inv_n);
            w[q] = (float)sqrt(P * T / (P + T) * inv_n);
        }
        pcoef[g / 2] = make_float4(oma[0], sig[0], oma[1], sig[1]);
        psrc[g / 2] = make_float2(src[0], src[1]);
        mcoef[g / 2] = make_float4(f[0], w[0], f[1], w[1]);
    }
}

}  // namespace

bool resident_supported(int H, int W) { return H == W && (H == 32 || H == 64 || H == 128); }

hipError_t launch_sampler_coefs(const ProbDev* probs, int n_problems, const float* d, const float* nbar,
                                const float* nP, float4* pcoef, float2* psrc, float4* mcoef, hipStream_t s) {
    hipLaunchKernelGGL(sampler_coef_kernel, dim3(32, n_problems), dim3(256), 0, s, probs, d, nbar, nP, pcoef, psrc,
                       mcoef);
    return hipGetLastError();
}

hipError_t launch_resident_sample(int N, const ResidentArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.n_items);
    switch (N) {
        case 32: hipLaunchKernelGGL(resident_sample_kernel<32>, grid, dim3(Res<32>::NT), 0, s, a); break;
        case 64: hipLaunchKernelGGL(resident_sample_kernel<64>, grid, dim3(Res<64>::NT), 0, s, a); break;
        case 128: hipLaunchKernelGGL(resident_sample_kernel<128>, grid, dim3(Res<128>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
