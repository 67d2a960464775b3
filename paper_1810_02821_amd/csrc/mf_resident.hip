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
//
// LDS exchanges use pitch N with per-exchange XOR swizzles of the column, and
// 16-byte accesses where a thread moves two adjacent elements, so that every
// 16- or 32-lane phase of an LDS instruction touches distinct banks.
#include "mf_device.hpp"
#include "mf_resident.hpp"

namespace mf {

namespace {

template <int N>
struct Res {
    static constexpr int P = N / 8;
    static constexpr int NT = N * N / 16;                  // threads per workgroup
    static constexpr int TB = 16 / P;                      // radix-P tasks per thread
    static constexpr int R1 = 32 / P;                      // pass-A rows per 16-lane phase
    static constexpr int SW2 = (N < 32 ? N : 32) - 1;
};

// E1 (between passes A and B): row y, column k1 P + x0
template <int N>
__device__ __forceinline__ unsigned e1(unsigned r, unsigned c) {
    constexpr unsigned P = Res<N>::P, R1 = Res<N>::R1;
    return r * N + (c ^ (P * (r % R1) + 2 * ((r / R1) % (P / 2))));
}
// E2 (between passes B and C): row y, column kx
template <int N>
__device__ __forceinline__ unsigned e2(unsigned r, unsigned c) {
    return r * N + (c ^ (r & (unsigned)Res<N>::SW2));
}
// E3 (between passes C and D): row 8 k1 + y0, column kx
template <int N>
__device__ __forceinline__ unsigned e3(unsigned r, unsigned c) {
    return r * N + c;
}

__device__ __forceinline__ void st2(float2* lds, unsigned i, float2 a, float2 b) {
    *reinterpret_cast<float4*>(lds + i) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void ld2(const float2* lds, unsigned i, float2& a, float2& b) {
    const float4 q = *reinterpret_cast<const float4*>(lds + i);
    a = make_float2(q.x, q.y);
    b = make_float2(q.z, q.w);
}

template <int R, bool INV>
__device__ __forceinline__ void dft_slice(float2* v) {
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[i];
    dft<R, INV>(t);
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Hide a pointer from loop-invariant code motion: tables are re-read (from
// cache) every sweep instead of being held in registers across sweeps.
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
//   A: y = tid / (P/2), j = tid % (P/2); holds x = 2j + q + P m     at v[8q + m]
//   B: t = tid + i NT (i < TB): y = t % N, k1 = t / N; holds x0    at v[P i + x0]
//   C: kx = tid % N, y0 = tid / N + i P/2 (i < TB);   holds m      at v[P i + m]
//   D: jx = tid % (N/2), k1 = tid / (N/2); kx = 2jx + q; holds y0  at v[8q + y0]

template <int N, bool INV>
__device__ __forceinline__ void pass_A(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned j = tid % (P / 2);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        dft_slice<8, INV>(v + 8 * q);
        if (!INV) {
            const unsigned x0 = 2 * j + q;
#pragma unroll
            for (int k1 = 1; k1 < 8; ++k1) v[8 * q + k1] = twiddle<false>(v[8 * q + k1], tw, x0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_A(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) st2(lds, e1<N>(y, k1 * P + 2 * j), v[k1], v[8 + k1]);
}

template <int N>
__device__ __forceinline__ void load_A_from_E1(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P;
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) ld2(lds, e1<N>(y, k1 * P + 2 * j), v[k1], v[8 + k1]);
}

template <int N>
__device__ __forceinline__ void load_B_from_E1(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int x0 = 0; x0 < P; x0 += 2) ld2(lds, e1<N>(y, k1 * P + x0), v[P * i + x0], v[P * i + x0 + 1]);
    }
}

template <int N>
__device__ __forceinline__ void store_E1_from_B(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int x0 = 0; x0 < P; x0 += 2) st2(lds, e1<N>(y, k1 * P + x0), v[P * i + x0], v[P * i + x0 + 1]);
    }
}

// pass B: forward radix-P over x0 -> k2 (no twiddle after);
// inverse: radix-P over k2 -> x0, then twiddle conj W_N^(x0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_B(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (INV) {
            const unsigned k1 = (tid + i * NT) / N;
#pragma unroll
            for (int x0 = 1; x0 < P; ++x0) v[P * i + x0] = twiddle<true>(v[P * i + x0], tw, x0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_B(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) lds[e2<N>(y, k1 + 8 * k2)] = v[P * i + k2];
    }
}

template <int N>
__device__ __forceinline__ void load_B_from_E2(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, NT = Res<N>::NT, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned t = tid + i * NT, y = t % N, k1 = t / N;
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) v[P * i + k2] = lds[e2<N>(y, k1 + 8 * k2)];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E2(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) v[P * i + m] = lds[e2<N>(y0 + 8 * m, kx)];
    }
}

template <int N>
__device__ __forceinline__ void store_E2_from_C(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int m = 0; m < P; ++m) lds[e2<N>(y0 + 8 * m, kx)] = v[P * i + m];
    }
}

// pass C: forward radix-P over m -> k1, then twiddle W_N^(y0 k1);
// inverse: radix-P over k1 -> m (the twiddle was applied in D').
template <int N, bool INV>
__device__ __forceinline__ void pass_C(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        dft_slice<P, INV>(v + P * i);
        if (!INV) {
            const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
            for (int k1 = 1; k1 < P; ++k1) v[P * i + k1] = twiddle<false>(v[P * i + k1], tw, y0 * k1);
        }
    }
}

template <int N>
__device__ __forceinline__ void store_E3_from_C(float2* lds, const float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) lds[e3<N>(k1 * 8 + y0, kx)] = v[P * i + k1];
    }
}

template <int N>
__device__ __forceinline__ void load_C_from_E3(const float2* lds, float2 (&v)[16], unsigned tid) {
    constexpr int P = Res<N>::P, TB = Res<N>::TB;
    const unsigned kx = tid % N;
#pragma unroll
    for (int i = 0; i < TB; ++i) {
        const unsigned y0 = tid / N + i * (P / 2);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) v[P * i + k1] = lds[e3<N>(k1 * 8 + y0, kx)];
    }
}

template <int N>
__device__ __forceinline__ void load_D_from_E3(const float2* lds, float2 (&v)[16], unsigned tid) {
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0) ld2(lds, e3<N>(k1 * 8 + y0, 2 * jx), v[y0], v[8 + y0]);
}

template <int N>
__device__ __forceinline__ void store_E3_from_D(float2* lds, const float2 (&v)[16], unsigned tid) {
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
#pragma unroll
    for (int y0 = 0; y0 < 8; ++y0) st2(lds, e3<N>(k1 * 8 + y0, 2 * jx), v[y0], v[8 + y0]);
}

// pass D: forward radix-8 over y0 -> k2 (ky = k1 + P k2);
// inverse: radix-8 over k2 -> y0, then twiddle conj W_N^(y0 k1).
template <int N, bool INV>
__device__ __forceinline__ void pass_D(float2 (&v)[16], const float2* __restrict__ tw, unsigned tid) {
    const unsigned k1 = tid / (N / 2);
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
__device__ __forceinline__ void forward_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, unsigned tid) {
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
__device__ __forceinline__ void inverse_fft(float2 (&v)[16], float2* lds, const float2* __restrict__ tw, unsigned tid) {
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
    __shared__ __align__(16) float2 lds[N * N];
    const unsigned tid = threadIdx.x;
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
        const float2* tw = per_sweep(a.tw);
        // Everything indexed by the thread id (LDS addresses, counter words of
        // the normal stream) is recomputed each sweep rather than kept live.
        // Each half of the sweep gets its own copy so that the forward pass's
        // LDS addresses are not kept alive for reuse by the inverse pass.
        unsigned t = tid;
        asm volatile("" : "+v"(t));
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


// ------------------------------------------------------------ solve kernel --
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
    __shared__ __align__(16) float2 lds[N * N];
    __shared__ double red[NT / 64];
    const unsigned tid = threadIdx.x;
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
        forward_fft<N>(v, lds, a.tw, t);
        unsigned t2 = tid;
        asm volatile("" : "+v"(t2));
        harmonic_solve<N>(v, a, pr, t2, T);
        inverse_fft<N>(v, lds, a.tw, t2);
        return check ? block_sum<NT>(acc, red) : 0.0;
    };

    int total = 0;
    for (int lv = 0; lv < a.n_levels; ++lv) {
        const float lam = (float)a.lambda[lv];
        for (int k = 0; k < a.sweeps[lv]; ++k) {
            sweep(lam, false, false);
            ++total;
        }
    }
    double residual = __builtin_nan("");
    int converged = a.tol > 0 ? 0 : 1;
    if (a.tol > 0) {
        const double lam = a.lambda[a.n_levels - 1];
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
                residual = bnorm > 0 ? sqrt(acc) / (T * bnorm) : 0.0;
                if (residual <= a.tol) {
                    converged = 1;
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

namespace {
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
