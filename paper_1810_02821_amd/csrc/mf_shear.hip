// Mass mapping (Sec. 5): the messenger Wiener filter and sampler for complex
// shear data gamma = A kappa + n with the spin-2 operator A = F^-1 D F,
// D_k = (k_1 + i k_2)^2 / |k|^2 (D_0 = 0), and a complex convergence
// kappa = kappa_E + i kappa_B with spectra P_E and P_B = r P_E.  One
// workgroup owns one chain of an N x N problem for every sweep, on chip.
//
// The state between sweeps is the model shear A kappa (pixel space):
//   t      = (1 - a) A kappa + a gamma + sqrt(T (1 - a)) xi        (shear space)
//   u(k)   = conj(D_k) F(t)(k)
//   kappa^ = f_+ u(k) + f_- conj(u(-k)) + w_+ eta(k) + w_- conj(eta(-k))
// with f_+- = (f_E +- f_B)/2, w_+- = (w_E +- w_B)/2: the E and B parts of u are
// the spectra of the real fields Re and Im of F^-1 u, and each gets its own
// Wiener-sampler step.  At k = 0 (no data) f = 0 and w draws the prior.  The
// next state is F^-1(D kappa^); on sweeps that emit a sample (and after the
// last sweep of a filter) kappa itself is F^-1(kappa^), written out before the
// field is transformed back.
#include "mf_device.hpp"
#include "mf_resident.hpp"
#include "mf_resident_fft.hpp"
#include "mf_shear.hpp"

namespace mf {

namespace {

template <int N>
__device__ __forceinline__ int signed_freq(unsigned k) {
    return k < (unsigned)(N / 2) ? (int)k : (int)k - N;  // numpy fftfreq * N
}

// D at mode (ky, kx) in unshifted FFT order (D_0 = 0 falls out of x = y = 0).
template <int N>
__device__ __forceinline__ float2 ks(unsigned ky, unsigned kx) {
    const float x = (float)signed_freq<N>(kx), y = (float)signed_freq<N>(ky);
    const float r = __builtin_amdgcn_rcpf(fmaxf(fmaf(x, x, y * y), 1.f));
    return make_float2((x * x - y * y) * r, 2.f * x * y * r);
}

// D at the mirror -k of (ky, kx): equal to D(k), except that on exactly one
// Nyquist line (where -k aliases to the same frequency in that component) the
// mixed term changes sign.
template <int N>
__device__ __forceinline__ float2 ks_mirror(float2 d, unsigned ky, unsigned kx) {
    const bool flip = (ky == (unsigned)(N / 2)) != (kx == (unsigned)(N / 2));
    return make_float2(d.x, flip ? -d.y : d.y);
}

template <int N>
__device__ __forceinline__ unsigned mirror_index(unsigned ky, unsigned kx) {
    return ((N - ky) & (N - 1)) * N + ((N - kx) & (N - 1));
}

__device__ __forceinline__ float2 mulc(float2 z, float2 d) {  // conj(d) z
    return make_float2(fmaf(d.x, z.x, d.y * z.y), fmaf(d.x, z.y, -d.y * z.x));
}

struct Filt {
    float fp, fm, wp, wm;
};

// f/n and w/n of the E and B fields at one mode (the 1/n of the inverse
// transform folded in), combined as (f_+, f_-, w_+, w_-).  At k = 0 the
// messenger variance is taken to infinity, which leaves f = 0 and the prior w.
__device__ __forceinline__ Filt filt(float nP, float r, float T, float inv_n, float n, bool k0) {
    const float Te = k0 ? 1e20f : T;
    const float nPB = r * nP;
    const float rE = __builtin_amdgcn_rcpf(nP + Te), rB = __builtin_amdgcn_rcpf(nPB + Te);
    const float fE = k0 ? 0.f : nP * rE * inv_n;
    const float fB = k0 ? 0.f : nPB * rB * inv_n;
    const float wE = __builtin_amdgcn_sqrtf(n * nP * (Te * rE)) * inv_n;
    const float wB = __builtin_amdgcn_sqrtf(n * nPB * (Te * rB)) * inv_n;
    return {0.5f * (fE + fB), 0.5f * (fE - fB), 0.5f * (wE + wB), 0.5f * (wE - wB)};
}

template <int N>
__device__ __forceinline__ void harmonic_shear(float2 (&v)[16], float2* lds, const ShearArgs& a, const ProbDev& pr,
                                               float T, uint32_t sweep, int chain, unsigned tid) {
    constexpr int P = Res<N>::P;
    __syncthreads();  // other threads may still read the forward transform's last exchange
    constexpr float n = (float)(N * N);
    constexpr float inv_n = 1.0f / (float)(N * N);
    const unsigned jx = tid % (N / 2), k1 = tid / (N / 2);
    const float* nP = a.nP + pr.pix_off;
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        const unsigned ky = k1 + P * k2;
        *reinterpret_cast<float4*>(lds + ky * N + 2 * jx) = make_float4(v[k2].x, v[k2].y, v[8 + k2].x, v[8 + k2].y);
    }
    __syncthreads();
    // filter part: f_+ u(k) + f_- conj(u(-k)), u = conj(D) Z
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const unsigned ky = k1 + P * k2;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned kx = 2 * jx + q;
            const unsigned mi = mirror_index<N>(ky, kx);
            const Filt c = filt(nP[ky * N + kx], a.b_ratio, T, inv_n, n, ky == 0 && kx == 0);
            const float2 d = ks<N>(ky, kx);
            const float2 u = mulc(v[8 * q + k2], d);
            const float2 um = mulc(lds[mi], ks_mirror<N>(d, ky, kx));
            v[8 * q + k2] = make_float2(fmaf(c.fp, u.x, c.fm * um.x), fmaf(c.fp, u.y, -c.fm * um.y));
        }
    }
    __syncthreads();
    if (!a.stochastic) return;
    // noise: w_+ eta(k) now, eta to LDS for w_- conj(eta(-k))
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const unsigned ky = k1 + P * k2;
        const uint32_t e2 = (uint32_t)(ky * (N / 2) + jx);
        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStageHarmonic, (uint32_t)chain, a.key0, a.key1);
        *reinterpret_cast<float4*>(lds + ky * N + 2 * jx) = make_float4(z.a.x, z.a.y, z.b.x, z.b.y);
        const Filt c0 = filt(nP[ky * N + 2 * jx], a.b_ratio, T, inv_n, n, ky == 0 && jx == 0);
        const Filt c1 = filt(nP[ky * N + 2 * jx + 1], a.b_ratio, T, inv_n, n, false);
        v[k2] = make_float2(fmaf(c0.wp, z.a.x, v[k2].x), fmaf(c0.wp, z.a.y, v[k2].y));
        v[8 + k2] = make_float2(fmaf(c1.wp, z.b.x, v[8 + k2].x), fmaf(c1.wp, z.b.y, v[8 + k2].y));
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
        __builtin_amdgcn_sched_barrier(0);
        const unsigned ky = k1 + P * k2;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const unsigned kx = 2 * jx + q;
            const Filt c = filt(nP[ky * N + kx], a.b_ratio, T, inv_n, n, ky == 0 && kx == 0);
            const float2 em = lds[mirror_index<N>(ky, kx)];
            float2& z = v[8 * q + k2];
            z = make_float2(fmaf(c.wm, em.x, z.x), fmaf(-c.wm, em.y, z.y));
        }
    }
    __syncthreads();
}

template <int N>
__global__ __launch_bounds__(Res<N>::NT, 4) void resident_shear_kernel(ShearArgs a) {
    constexpr int P = Res<N>::P;
    __shared__ __align__(16) float2 lds[Res<N>::LDS];
    __shared__ float2 twl[Res<N>::TWS];  // twiddle tables of the four passes
    const unsigned tid = threadIdx.x;
    fill_twiddle_tables<N>(twl, a.tw, tid);
    __syncthreads();
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const unsigned y = tid / (P / 2), j = tid % (P / 2);
    const int64_t nn = (int64_t)N * N;

    float2 v[16];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int64_t o = it.field_off + (int64_t)y * N + 2 * j + P * m;
        v[m] = a.state_in ? a.state_in[o] : make_float2(0.f, 0.f);
        v[8 + m] = a.state_in ? a.state_in[o + 1] : make_float2(0.f, 0.f);
    }

    int64_t k = 0;
    for (int lv = 0; lv < a.lv.n; ++lv) {
        const float T = (float)(a.lv.lambda[lv] * (double)pr.tau);
        for (int s = 0; s < a.lv.sweeps[lv]; ++s, ++k) {
            const uint32_t sweep = a.sweep0 + (uint32_t)k;
            const float2* tw = twl + per_sweep_zero();
            unsigned t = tid;
            asm volatile("" : "+v"(t));
            {
                // pixel step in shear space
                const unsigned yy = t / (P / 2), jj = t % (P / 2);
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    __builtin_amdgcn_sched_barrier(0);
                    const uint32_t e2 = (uint32_t)(yy * (N / 2) + jj + (P / 2) * m);
                    const int64_t px = pr.pix_off + 2 * (int64_t)e2;
                    const float2 nb = *reinterpret_cast<const float2*>(a.nbar + px);
                    const float4 g = *reinterpret_cast<const float4*>(a.gamma + px);
                    const float a0 = T * __builtin_amdgcn_rcpf(T + nb.x), a1 = T * __builtin_amdgcn_rcpf(T + nb.y);
                    const float2 g0 = a0 > 0.f ? make_float2(a0 * g.x, a0 * g.y) : make_float2(0.f, 0.f);
                    const float2 g1 = a1 > 0.f ? make_float2(a1 * g.z, a1 * g.w) : make_float2(0.f, 0.f);
                    float2& s0 = v[m];
                    float2& s1 = v[8 + m];
                    s0 = make_float2(fmaf(1.f - a0, s0.x, g0.x), fmaf(1.f - a0, s0.y, g0.y));
                    s1 = make_float2(fmaf(1.f - a1, s1.x, g1.x), fmaf(1.f - a1, s1.y, g1.y));
                    if (a.stochastic) {
                        const Normals2 z = pair_normals(e2, sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)it.pair,
                                                        a.key0, a.key1);
                        const float sg0 = __builtin_amdgcn_sqrtf(fmaxf(T * (1.f - a0), 0.f));
                        const float sg1 = __builtin_amdgcn_sqrtf(fmaxf(T * (1.f - a1), 0.f));
                        s0 = make_float2(fmaf(sg0, z.a.x, s0.x), fmaf(sg0, z.a.y, s0.y));
                        s1 = make_float2(fmaf(sg1, z.b.x, s1.x), fmaf(sg1, z.b.y, s1.y));
                    }
                }
            }
            forward_fft<N>(v, lds, tw, t);
            unsigned t2 = tid;
            asm volatile("" : "+v"(t2));
            harmonic_shear<N>(v, lds, a, pr, T, sweep, it.pair, t2);
            const bool last = lv == a.lv.n - 1 && s == a.lv.sweeps[lv] - 1;
            const bool emit = a.samples && k >= a.burn_in && ((k - a.burn_in + 1) % a.thin) == 0;
            if (emit || (last && a.kappa_out)) {
                // kappa = F^-1 kappa^, written out, then transformed back
                unsigned t3 = tid;
                asm volatile("" : "+v"(t3));
                const float2* tw3 = twl + per_sweep_zero();
                inverse_fft<N>(v, lds, tw3, t3);
                float2* o;
                if (emit) {
                    const int64_t slot = (k - a.burn_in + 1) / a.thin - 1;
                    o = a.samples + (int64_t)a.chains * a.n_samples * pr.pix_off +
                        ((int64_t)it.pair * a.n_samples + slot) * nn;
                } else {
                    o = a.kappa_out + pr.pix_off;
                }
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int64_t px = (int64_t)y * N + 2 * j + P * m;
                    o[px] = v[m];
                    o[px + 1] = v[8 + m];
                }
                unsigned t4 = tid;
                asm volatile("" : "+v"(t4));
                forward_fft<N>(v, lds, tw3, t4);
            }
            // next state: F^-1 (D kappa^); after the round trip through pixel space
            // the unnormalised forward transform returned n kappa^
            const float back = (emit || (last && a.kappa_out)) ? 1.0f / (float)(N * N) : 1.0f;
            unsigned t5 = tid;
            asm volatile("" : "+v"(t5));
            const float2* tw5 = twl + per_sweep_zero();
            {
                const unsigned jx = t5 % (N / 2), k1 = t5 / (N / 2);
#pragma unroll
                for (int k2 = 0; k2 < 8; ++k2) {
                    const unsigned ky = k1 + P * k2;
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        v[8 * q + k2] = cmul(v[8 * q + k2], cscale(ks<N>(ky, 2 * jx + q), back));
                }
            }
            inverse_fft<N>(v, lds, tw5, t5);
        }
    }
    if (a.state_out) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int64_t o = it.field_off + (int64_t)y * N + 2 * j + P * m;
            a.state_out[o] = v[m];
            a.state_out[o + 1] = v[8 + m];
        }
    }
}

}  // namespace

hipError_t launch_resident_shear(int N, const ShearArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)a.n_items);
    switch (N) {
        case 32: hipLaunchKernelGGL(resident_shear_kernel<32>, grid, dim3(Res<32>::NT), 0, s, a); break;
        case 64: hipLaunchKernelGGL(resident_shear_kernel<64>, grid, dim3(Res<64>::NT), 0, s, a); break;
        case 128: hipLaunchKernelGGL(resident_shear_kernel<128>, grid, dim3(Res<128>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
