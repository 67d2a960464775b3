// Persistent deterministic solve (Wiener filter or adjoint): one workgroup
// owns one problem of N x N pixels and runs every cooling level and the
// convergence phase of the messenger iteration with the variates set to zero
// (Sec. 2.2).  The residual test of the convergence phase is reduced in FP64
// through LDS on the device, so no sweep waits for the host.
#include "mf_device.hpp"
#include "mf_resident.hpp"
#include "mf_resident_fft.hpp"

namespace mf {

namespace {

// Deterministic sweeps (variates set to zero, Sec. 2.2) with a general source:
// t = (1 - a) s + src, src = a d (Wiener filter) or T g (adjoint solve).  The
// real problem rides in the real channel of the complex field.
template <int N>
__device__ __forceinline__ void pixel_solve(float2 (&v)[16], float (&tprev)[16], const SolveArgs& a,
                                            const ProbDev& pr, unsigned tid, float T, bool save, bool check,
                                            double& acc) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t pix = pr.pix_off + (int64_t)y * N + 2 * j + q + P * m;
            const float aa = T * __builtin_amdgcn_rcpf(T + a.nbar[pix]);
            const float sv = a.src[pix];
            const float src = a.src_kind == kSrcData ? (aa > 0.f ? aa * sv : 0.f) : T * sv;
            const float t = fmaf(1.0f - aa, v[8 * q + m].x, src);
            if (check) {
                const double dd = (double)t - (double)tprev[8 * q + m];
                acc += dd * dd;
            }
            if (save) tprev[8 * q + m] = t;
            v[8 * q + m] = make_float2(t, 0.f);
        }
    }
}

template <int N>
__device__ __forceinline__ void harmonic_solve(float2 (&v)[16], const SolveArgs& a, const ProbDev& pr, unsigned tid,
                                               float T) {
    constexpr int P = Res<N>::P;
    constexpr float inv_n = 1.0f / (float)(N * N);
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
        const float2 np = *reinterpret_cast<const float2*>(a.nP + pr.pix_off + (int64_t)ky * N + 2 * jx);
        v[k2] = cscale(v[k2], np.x * __builtin_amdgcn_rcpf(np.x + T) * inv_n);
        v[8 + k2] = cscale(v[8 + k2], np.y * __builtin_amdgcn_rcpf(np.y + T) * inv_n);
    }
}

// Sum a double over the workgroup; every thread gets the total.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const unsigned w = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

template <int N>
__global__ __launch_bounds__(Res<N>::NT, 4) void resident_solve_kernel(SolveArgs a) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT;
    __shared__ __align__(16) float2 lds[Res<N>::LDS];
    __shared__ double red[NT / 64];
    __shared__ float2 twl[Res<N>::TWS];  // twiddle tables of the four passes
    const unsigned tid = threadIdx.x;
    fill_twiddle_tables<N>(twl, a.tw, tid);
    __syncthreads();
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const unsigned y = tid / (P / 2), j = tid % (P / 2);

    float2 v[16];
    float tprev[16];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t pix = pr.pix_off + (int64_t)y * N + 2 * j + q + P * m;
            v[8 * q + m] = make_float2(a.s_init ? a.s_init[pix] : 0.f, 0.f);
            tprev[8 * q + m] = 0.f;
        }

    auto sweep = [&](float lam, bool save, bool check) -> double {
        const float T = lam * pr.tau;
        unsigned t = tid;
        asm volatile("" : "+v"(t));
        double acc = 0.0;
        pixel_solve<N>(v, tprev, a, pr, t, T, save, check, acc);
        forward_fft<N>(v, lds, twl + per_sweep_zero(), t);
        unsigned t2 = tid;
        asm volatile("" : "+v"(t2));
        harmonic_solve<N>(v, a, pr, t2, T);
        inverse_fft<N>(v, lds, twl + per_sweep_zero(), t2);
        return check ? block_sum<NT>(acc, red) : 0.0;
    };

    int total = a.total0;
    for (int lv = 0; lv < a.lv.n; ++lv) {
        const float lam = (float)a.lv.lambda[lv];
        for (int k = 0; k < a.lv.sweeps[lv]; ++k) {
            sweep(lam, false, false);
            ++total;
        }
    }
    double residual = __builtin_nan("");
    int converged = a.tol > 0 ? 0 : 1;
    if (a.tol > 0) {
        const double lam = a.lv.lambda[a.lv.n - 1];
        const double T = lam * (double)pr.tau;
        // ||b||^2 with b = N_eff^-1 d (data) or g (gradient) at the final level
        double bb = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int64_t pix = pr.pix_off + (int64_t)y * N + 2 * j + q + P * m;
                const double nb = a.nbar[pix];
                const double b = a.src_kind == kSrcData ? (isinf(nb) ? 0.0 : (double)a.src[pix] / (nb + T))
                                                        : (double)a.src[pix];
                bb += b * b;
            }
        const double bnorm = sqrt(block_sum<NT>(bb, red));
        const int levels_total = total;
        while (total < a.max_sweeps) {
            const int c = total + 1;
            const bool check = (c % a.check_every == 0) && (c - 1 >= levels_total + 1);
            const bool save = ((c + 1) % a.check_every == 0);
            const double acc = sweep((float)lam, save, check);
            ++total;
            if (check) {
                residual = bnorm == 0.0 ? 0.0 : sqrt(acc) / (T * bnorm);  // NaN stays NaN
                if (residual <= a.tol) {
                    converged = 1;
                    break;
                }
                if (!isfinite(residual)) {  // NaN or Inf in the inputs or the iterate: stop
                    converged = -1;
                    break;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) a.s_out[pr.pix_off + (int64_t)y * N + 2 * j + q + P * m] = v[8 * q + m].x;
    if (tid == 0 && a.info) {
        a.info[3 * blockIdx.x + 0] = (double)total;
        a.info[3 * blockIdx.x + 1] = (double)converged;
        a.info[3 * blockIdx.x + 2] = residual;
    }
}

}  // namespace

hipError_t launch_resident_solve(int N, const SolveArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.n_items);
    switch (N) {
        case 32: hipLaunchKernelGGL(resident_solve_kernel<32>, grid, dim3(Res<32>::NT), 0, s, a); break;
        case 64: hipLaunchKernelGGL(resident_solve_kernel<64>, grid, dim3(Res<64>::NT), 0, s, a); break;
        case 128: hipLaunchKernelGGL(resident_solve_kernel<128>, grid, dim3(Res<128>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
