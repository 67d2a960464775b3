// Persistent LDS-resident sampler: one workgroup owns one chain pair of an
// N x N image (N = 8 P, P in {4, 8, 16}) and runs every sweep of Algorithm 1
// without leaving the chip; only emitted samples and the final state reach HBM.
//
// The field lives in registers, 16 complex values per thread (N^2/16 threads).
// A 2D FFT is four passes, radix-8 and radix-P along each dimension:
//   rows    x = x0 + P m,  kx = k1 + 8 k2   (pass A: radix-8 over m,  pass B: radix-P over x0)
//   columns y = y0 + 8 m,  ky = k1 + P k2   (pass C: radix-P over m,  pass D: radix-8 over y0)
// with twiddles W_N^(x0 k1) after A and W_N^(y0 k1) after C.  The forward
// transform runs A, B, C, D (decimation in frequency); the inverse runs the
// transposed passes D', C', B', A' (decimation in time), so the Fourier-space
// update happens in pass D's registers and the pixel-space update in pass A's,
// and LDS is touched only for the three exchanges between passes.
#include "mf_device.hpp"
#include "mf_resident.hpp"

namespace mf {

namespace {

template <int N>
struct Res {
    static constexpr int P = N / 8;
    static constexpr int NT = N * N / 16;      // threads per workgroup
    static constexpr int PITCH = N + 1;        // LDS row pitch (complex)
    static constexpr int TB = 16 / P;          // radix-P tasks per thread
};

template <int R, bool INV>
__device__ __forceinline__ void dft_slice(float2* v) {
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[i];
    dft<R, INV>(t);
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Hide a table pointer from loop-invariant code motion: the tables are re-read
// (from cache) every sweep instead of being held in registers across sweeps.
template <typename T>
__device__ __forceinline__ const T* per_sweep(const T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

template <bool INV>
__device__ __forceinline__ float2 twiddle(float2 v, const float2* __restrict__ tw, int idx) {
    const float2 w = tw[idx];
    return INV ? cmulc(v, w) : cmul(v, w);
}

// ---------------------------------------------------------------- passes --
// Thread coordinates in each layout (tid in [0, NT)):
//   A: y = tid / (P/2), j = tid % (P/2); holds x = 2j + q + P m   at v[8q + m]
//   B: tasks t = tid*TB + i: y = t / 8, k1 = t % 8; holds x0      at v[P i + x0]
//   C: kx = tid % N, y0 = tid / N + i P/2;          holds m       at v[P i + m]
//   D: jx = tid % (N/2), k1 = tid / (N/2);  kx = 2jx + q; holds y0 at v[8q + y0]
// LDS layouts between passes (row, column):
//   E1 (A<->B): (y, k1 P + x0)     E2 (B<->C): (y, kx)     E3 (C<->D): (k1 8 + y0, kx)

template <int N, bool INV>
__device__ __forceinline__ void pass_A(float2 (&v)[16], const float2* __restrict__ tw, int tid) {
    constexpr int P = Res<N>::P;
    const int j = tid % (P / 2);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int x0 = 2 * j + q;
        if (INV) {
            dft_slice<8, true>(v + 8 * q);
        } else {
            dft_slice<8, false>(v + 8 * q);
#pragma unroll
            for (int k1 = 1; k1 < 8; ++k1) v[8 * q + k1] = twiddle<false>(v[8 * q + k1], tw, x0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_A(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH;
    const int y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
#pragma unroll
        for (int q = 0; q < 2; ++q) lds[y * PITCH + k1 * P + 2 * j + q] = v[8 * q + k1];
}

template <int N>
__device__ __forceinline__ void load_A_from_E1(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH;
    const int y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
#pragma unroll
        for (int q = 0; q < 2; ++q) v[8 * q + k1] = lds[y * PITCH + k1 * P + 2 * j + q];
}

template <int N>
__device__ __forceinline__ void load_B_from_E1(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int t = tid * TB + i, y = t / 8, k1 = t % 8;
#pragma unroll
        for (int x0 = 0; x0 < P; ++x0) v[P * i + x0] = lds[y * PITCH + k1 * P + x0];
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_B(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int t = tid * TB + i, y = t / 8, k1 = t % 8;
#pragma unroll
        for (int x0 = 0; x0 < P; ++x0) lds[y * PITCH + k1 * P + x0] = v[P * i + x0];
    }
}

// pass B: forward radix-P over x0 -> k2 (no twiddle after);
// inverse: radix-P over k2 -> x0, then twiddle conj W_N^(x0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_B(float2 (&v)[16], const float2* __restrict__ tw, int tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (INV) {
            const int k1 = (tid * TB + i) % 8;
#pragma unroll
            for (int x0 = 1; x0 < P; ++x0) v[P * i + x0] = twiddle<true>(v[P * i + x0], tw, x0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_B(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int t = tid * TB + i, y = t / 8, k1 = t % 8;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) lds[y * PITCH + k1 + 8 * k2] = v[P * i + k2];
    }
}

template <int N>
__device__ __forceinline__ void load_B_from_E2(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int t = tid * TB + i, y = t / 8, k1 = t % 8;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) v[P * i + k2] = lds[y * PITCH + k1 + 8 * k2];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E2(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
    const int kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) v[P * i + m] = lds[(y0 + 8 * m) * PITCH + kx];
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_C(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
    const int kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) lds[(y0 + 8 * m) * PITCH + kx] = v[P * i + m];
    }
}

// pass C: forward radix-P over m -> k1, then twiddle W_N^(y0 k1);
// inverse: radix-P over k1 -> m (the twiddle was applied in D').
template <int N, bool INV>
__device__ __forceinline__ void pass_C(float2 (&v)[16], const float2* __restrict__ tw, int tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (!INV) {
            const int y0 = tid / N + i * (P / 2);
#pragma unroll
            for (int k1 = 1; k1 < P; ++k1) v[P * i + k1] = twiddle<false>(v[P * i + k1], tw, y0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E3_from_C(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
    const int kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) lds[(k1 * 8 + y0) * PITCH + kx] = v[P * i + k1];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E3(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int P = Res<N>::P, PITCH = Res<N>::PITCH, TB = Res<N>::TB;
    const int kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const int y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) v[P * i + k1] = lds[(k1 * 8 + y0) * PITCH + kx];
    }
}

template <int N>
__device__ __forceinline__ void load_D_from_E3(const float2* lds, float2 (&v)[16], int tid) {
    constexpr int PITCH = Res<N>::PITCH;
    const int jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0)
#pragma unroll
        for (int q = 0; q < 2; ++q) v[8 * q + y0] = lds[(k1 * 8 + y0) * PITCH + 2 * jx + q];
}

template <int N>
__device__ __forceinline__ void store_E3_from_D(float2* lds, const float2 (&v)[16], int tid) {
    constexpr int PITCH = Res<N>::PITCH;
    const int jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0)
#pragma unroll
        for (int q = 0; q < 2; ++q) lds[(k1 * 8 + y0) * PITCH + 2 * jx + q] = v[8 * q + y0];
}

// pass D: forward radix-8 over y0 -> k2 (ky = k1 + P k2);
// inverse: radix-8 over k2 -> y0, then twiddle conj W_N^(y0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_D(float2 (&v)[16], const float2* __restrict__ tw, int tid) {
    const int k1 = tid / (N / 2);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        dft_slice<8, INV>(v + 8 * q);
        if (INV) {
#pragma unroll
            for (int y0 = 1; y0 < 8; ++y0) v[8 * q + y0] = twiddle<true>(v[8 * q + y0], tw, y0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void forward_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, int tid) {
    pass_A<N, false>(v, tw, tid);
    store_E1_from_A<N>(lds, v, tid);
    __syncthreads();
    load_B_from_E1<N>(lds, v, tid);
    __syncthreads();
    pass_B<N, false>(v, tw, tid);
    store_E2_from_B<N>(lds, v, tid);
    __syncthreads();
    load_C_from_E2<N>(lds, v, tid);
    __syncthreads();
    pass_C<N, false>(v, tw, tid);
    store_E3_from_C<N>(lds, v, tid);
    __syncthreads();
    load_D_from_E3<N>(lds, v, tid);
    __syncthreads();
    pass_D<N, false>(v, tw, tid);
}

template <int N>
__device__ __forceinline__ void inverse_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, int tid) {
    pass_D<N, true>(v, tw, tid);
    store_E3_from_D<N>(lds, v, tid);
    __syncthreads();
    load_C_from_E3<N>(lds, v, tid);
    __syncthreads();
    pass_C<N, true>(v, tw, tid);
    store_E2_from_C<N>(lds, v, tid);
    __syncthreads();
    load_B_from_E2<N>(lds, v, tid);
    __syncthreads();
    pass_B<N, true>(v, tw, tid);
    store_E1_from_B<N>(lds, v, tid);
    __syncthreads();
    load_A_from_E1<N>(lds, v, tid);
    __syncthreads();
    pass_A<N, true>(v, tw, tid);
}

// --------------------------------------------------------------- updates --
// Pixel-space messenger draw on layout A: t = (1-a) s + a d + sqrt(T(1-a)) xi.
template <int N>
__device__ __forceinline__ void pixel_update(float2 (&v)[16], const ResidentArgs& a, const ProbDev& pr, int pair,
                                             uint32_t sweep, int tid, float T) {
    constexpr int P = Res<N>::P;
    const int y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        // keep the eight Philox chains from being interleaved (register pressure)
        __builtin_amdgcn_sched_barrier(0);
        const int x = 2 * j + P * m;
        const int64_t pix = pr.pix_off + (int64_t)y * N + x;
        const float2 nb = *reinterpret_cast<const float2*>(a.nbar + pix);
        const float2 dd = *reinterpret_cast<const float2*>(a.d + pix);
        const uint32_t e2 = (uint32_t)(y * (N / 2) + j + (P / 2) * m);
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)pair, a.key0, a.key1);
        const float nbv[2] = {nb.x, nb.y}, dv[2] = {dd.x, dd.y};
        const float2 zz[2] = {z.a, z.b};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // a = T/(T+Nbar) is 1 at the smallest-noise pixel (Nbar = 0) and
            // 0 on missing ones; 1 - a may come out as -1 ulp, so the variance
            // T(1-a) is clamped at 0 below.
            const float aa = T * __builtin_amdgcn_rcpf(T + nbv[q]);
            const float oma = 1.0f - aa;
            const float src = aa > 0.f ? aa * dv[q] : 0.f;
            const float sig = __builtin_amdgcn_sqrtf(fmaxf(T * oma, 0.f));
            float2& s = v[8 * q + m];
            s.x = fmaf(oma, s.x, fmaf(sig, zz[q].x, src));
            s.y = fmaf(oma, s.y, fmaf(sig, zz[q].y, src));
        }
    }
}

// Fourier-space draw on layout D: S = f T / n + w eta / n.
template <int N>
__device__ __forceinline__ void harmonic_update(float2 (&v)[16], const ResidentArgs& a, const ProbDev& pr, int pair,
                                                uint32_t sweep, int tid, float T) {
    constexpr int P = Res<N>::P;
    constexpr float inv_n = 1.0f / (float)(N * N);
    const int jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const int ky = k1 + P * k2;
        const int64_t mode = pr.pix_off + (int64_t)ky * N + 2 * jx;
        const float2 np = *reinterpret_cast<const float2*>(a.nP + mode);
        const uint32_t e2 = (uint32_t)(ky * (N / 2) + jx);
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStageHarmonic, (uint32_t)pair, a.key0, a.key1);
        const float npv[2] = {np.x, np.y};
        const float2 zz[2] = {z.a, z.b};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float rden = __builtin_amdgcn_rcpf(npv[q] + T);
            const float f = npv[q] * rden * inv_n;
            const float w = __builtin_amdgcn_sqrtf(npv[q] * T * rden * inv_n);
            float2& s = v[8 * q + k2];
            s.x = fmaf(f, s.x, w * zz[q].x);
            s.y = fmaf(f, s.y, w * zz[q].y);
        }
    }
}

template <int N>
__global__ __launch_bounds__(Res<N>::NT, 4) void resident_sample_kernel(ResidentArgs a) {
    constexpr int P = Res<N>::P;
    __shared__ float2 lds[N * Res<N>::PITCH];
    const int tid = threadIdx.x;
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const int y = tid / (P / 2), j = tid % (P / 2);

    // initial state in layout A
    float2 v[16];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int x = 2 * j + q + P * m;
            float2 s0 = make_float2(0.f, 0.f);
            if (a.state_in) {
                s0 = a.state_in[it.field_off + (int64_t)y * N + x];
            } else if (a.init_scale > 0.f && q == 0) {
                const uint32_t e2 = (uint32_t)((y * N + x) >> 1);
                const Normals2 z = pair_normals(e2, 0u, (uint32_t)pr.pid, kStageInit, (uint32_t)it.pair, a.key0, a.key1);
                v[8 * 1 + m] = cscale(z.b, a.init_scale);
                s0 = cscale(z.a, a.init_scale);
            } else if (a.init_scale > 0.f) {
                continue;  // set together with q == 0
            }
            v[8 * q + m] = s0;
        }

    const float T = pr.tau;  // lambda = 1
    const int64_t n = (int64_t)N * N;
    const int64_t K = (int64_t)a.burn_in + (int64_t)a.n_samples * a.thin;
    const int c0 = 2 * it.pair, c1 = 2 * it.pair + 1;
    for (int64_t k = 0; k < K; ++k) {
        const uint32_t sweep = a.sweep0 + (uint32_t)k;
        ResidentArgs ak = a;
        ak.nbar = per_sweep(a.nbar);
        ak.d = per_sweep(a.d);
        ak.nP = per_sweep(a.nP);
        const float2* tw = per_sweep(a.tw);
        // Everything indexed by the thread id (LDS addresses, counter words of
        // the normal stream) is recomputed each sweep rather than kept live.
        int t = tid;
        asm volatile("" : "+v"(t));
        pixel_update<N>(v, ak, pr, it.pair, sweep, t, T);
        forward_fft<N>(v, lds, tw, t);
        harmonic_update<N>(v, ak, pr, it.pair, sweep, t, T);
        inverse_fft<N>(v, lds, tw, t);
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
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) a.field[it.field_off + (int64_t)y * N + 2 * j + q + P * m] = v[8 * q + m];
}

}  // namespace

bool resident_supported(int H, int W) { return H == W && (H == 32 || H == 64 || H == 128); }

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
