// Streamed form of the hierarchical sampler (Sec. 5) for size classes the
// persistent kernel does not hold: the streamed sampler's row kernel does the
// pixel step; the column kernel below does the Fourier step with each chain's
// own band amplitudes, and two small kernels draw the amplitudes.
//
// The Fourier step of a pair whose chains have different spectra combines
// every mode k with its mirror -k (mf_spectrum.hip derives the update).
// Column tiles are therefore made of mirror pairs of columns: tile j of an
// item holds columns c = j TC/2 + i (i < TC/2) in its first TC/2 slots and
// their mirrors W - c in the others, with the two self-mirror columns 0 and
// W/2 both in tile 0.  After the column transforms a tile holds both modes of
// every pair it updates.
//
// On the last sweep of an iteration the tile also adds the band powers of
// both chains (FP64) to per-item sums; the draw then needs only those sums and
// the chi-square variates, as in the persistent kernel.
#include "mf_device.hpp"
#include "mf_kernels.hpp"
#include "mf_spectrum.hpp"
#include "mf_streamed_fft.hpp"

namespace mf {

namespace {

constexpr int kNB = kMaxBandsPerProblem;
constexpr uint32_t kStageSpectrum = 3;

// Tiles of the mirror-paired column kernel, timed on the hierarchical and
// mass-mapping samplers: 16 columns below 512 rows (512 threads at 256), 8
// columns from 512 rows with 256 threads at 512, 512 at 1024 and 1024 at 2048
// (at 512 and 1024 rows 3.8-11.6% faster than 16 columns of 512 and 1024
// threads).
template <int L>
struct PairShape {
    static constexpr int TC = L >= 512 ? 8 : 16;
    static constexpr int NTH = L >= 2048 ? 1024 : (L == 1024 ? 512 : (L == 256 ? 512 : 256));
    static constexpr int TPC = NTH / TC;
    static constexpr int SEG = L + 32 / TC;
};

// Opaque copies: the compiler cannot keep values derived from them live across
// the transforms (which would raise register pressure).
__device__ __forceinline__ unsigned opaque(unsigned v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ const float2* opaque(const float2* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Column held by slot s of tile j.
__device__ __forceinline__ int pair_column(int j, int s, int half, int W) {
    if (s < half) return j * half + s;
    const int c = j * half + (s - half);
    return c == 0 ? W / 2 : W - c;
}

// Harmonic-stage normal of mode index e (same element mapping as the other
// samplers: the pair call j = e / 2 gives .a to even e and .b to odd e).
__device__ __forceinline__ float2 mode_normal(uint32_t e, uint32_t sweep, uint32_t pid, uint32_t pair, uint32_t k0,
                                              uint32_t k1) {
    const Normals2 z = pair_normals(e >> 1, sweep, pid, kStageHarmonic, pair, k0, k1);
    return (e & 1u) ? z.b : z.a;
}

template <int L>
__global__ __launch_bounds__(PairShape<L>::NTH) void col_pair_kernel(SpectrumStreamArgs a, int W) {
    constexpr int TC = PairShape<L>::TC, NTH = PairShape<L>::NTH, TPC = PairShape<L>::TPC;
    // padded exchange layouts from 256 rows (the HBM-side passes) where they
    // keep the resident workgroups per CU, else the XOR swizzle
    constexpr int kExtra = 8 * L + (int)(sizeof(double) * 2 * kNB + sizeof(float4) * kNB);  // twiddles and tables beside the tile
    constexpr bool kPad = L >= 256 && lds_keeps_blocks(TC * PairShape<L>::SEG * 8 + kExtra,
                                                       TC * PairLayout<L, TC>::SEG * 8 + kExtra);
    constexpr int A1 = kPad ? PairLayout<L, TC>::A1 : -1, AN = kPad ? PairLayout<L, TC>::AN : -1;
    constexpr int AD = kPad ? PairLayout<L, TC>::AD : -1;
    constexpr int SEG = kPad ? PairLayout<L, TC>::SEG : PairShape<L>::SEG;
    constexpr int H = L;
    constexpr int half = TC / 2;
    __shared__ float2 lds[TC * SEG];
    __shared__ double pw[2][kNB];
    __shared__ float4 coef[kNB];
    __shared__ float2 twl[L >= 256 ? L : 1];  // twiddles in LDS (hierarchical 2048^2 sweep +7%)
    const unsigned tid = threadIdx.x;
    // tile fastest: an XCD runs neighbouring tiles of one item together, so
    // the cache lines they share meet in its L2
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int item = (int)(t / (W / TC));
    const int j = (int)(t % (W / TC));
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    float2* fld = a.field + it.field_off;

    auto col_of = [&](int s) { return pair_column(j, s, half, W); };
    if constexpr (L >= 256) {
        // first forward pass straight from HBM (plan of mf_streamed_fft.hpp)
        col_first_forward<L, TC, NTH, SEG, A1>(lds, fld, W, tid, col_of);
    } else {
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            lds[s * SEG + swz(y)] = fld[(int64_t)y * W + pair_column(j, s, half, W)];
        }
    }
    for (unsigned u = tid; u < 2 * kNB; u += NTH) pw[u / kNB][u % kNB] = 0.0;
    for (unsigned u = tid; u < kNB; u += NTH) coef[u] = a.coef[(int64_t)item * kNB + u];
    if constexpr (L >= 256)
        for (unsigned i = tid; i < (unsigned)L; i += NTH) twl[i] = a.tw_col[i];
    __syncthreads();
    const unsigned cid = tid / TPC, lane = tid % TPC;
    if constexpr (L >= 256) col_forward_rest<L, TPC, A1>(lds + cid * SEG, lane, twl);
    else stockham_fft<L, 1, TPC, false>(lds + cid * SEG, lane, a.tw_col);

    const int16_t* band = a.band + pr.pix_off;
    const uint32_t pid = (uint32_t)pr.pid, pair = (uint32_t)it.pair;
    // Fourier step of mode k (slot s, row ky, band b) and its mirror -k (slot
    // p, row my; band(-k) = band(k): same |k|), given the chain pair's
    // harmonic normals at k and -k
    auto update = [&](int s, int p, int ky, int my, bool self, int b, float2 hk, float2 hm) {
        float2& zk = lds[s * SEG + lpos<AN>(ky)];
        float2& zm = lds[p * SEG + lpos<AN>(my)];
        const float2 Zk = zk, Zm = zm;
        const float4 c = coef[b];
        const float fp = 0.5f * (c.x + c.z), fm = 0.5f * (c.x - c.z);
        const float wp = 0.5f * (c.y + c.w), wm = 0.5f * (c.y - c.w);
        // S(k) = f_+ Z(k) + f_- conj Z(-k) + w_+ eta(k) + w_- conj eta(-k), and with k, -k swapped
        const float2 Sk = make_float2(fmaf(fp, Zk.x, fm * Zm.x) + fmaf(wp, hk.x, wm * hm.x),
                                      fmaf(fp, Zk.y, -fm * Zm.y) + fmaf(wp, hk.y, -wm * hm.y));
        const float2 Sm = make_float2(fmaf(fp, Zm.x, fm * Zk.x) + fmaf(wp, hm.x, wm * hk.x),
                                      fmaf(fp, Zm.y, -fm * Zk.y) + fmaf(wp, hm.y, -wm * hk.y));
        zk = Sk;
        if (!self) zm = Sm;
        if (a.add_power) {
            // X_A(k) = (S(k) + conj S(-k))/2, X_B(k) = (S(k) - conj S(-k))/(2i); |X(-k)| = |X(k)|
            const double ar = 0.5 * ((double)Sk.x + Sm.x), ai = 0.5 * ((double)Sk.y - Sm.y);
            const double br = 0.5 * ((double)Sk.y + Sm.y), bi = 0.5 * ((double)Sk.x - Sm.x);
            const double wgt = self ? 1.0 : 2.0;
            atomicAdd(&pw[0][b], wgt * (ar * ar + ai * ai));
            atomicAdd(&pw[1][b], wgt * (br * br + bi * bi));
        }
    };
    if (j == 0) {
        // tile 0: one job per mode pair {k, -k}, a first-half slot with its
        // partner slot; the self-mirror columns 0 (slot 0) and W/2 (slot
        // half) take the rows ky <= H/2, whose partners -ky lie in the same column
        const int jobs = half * H + H / 2 + 1;
#pragma unroll 1
        for (int q = opaque(tid); q < jobs; q += NTH) {
            int s, ky;
            if (q < half * H) {
                s = q % half;
                ky = q / half;
                if (s == 0 && ky > H / 2) continue;
            } else {
                s = half;
                ky = q - half * H;
            }
            const bool self_col = s == 0 || s == half;
            const int p = self_col ? s : s + half;
            const int my = (H - ky) & (H - 1);
            const bool self = self_col && my == ky;
            const uint32_t ek = (uint32_t)(ky * W + pair_column(j, s, half, W));
            const uint32_t em = (uint32_t)(my * W + pair_column(j, p, half, W));
            const float2 hk = mode_normal(ek, a.sweep, pid, pair, a.key0, a.key1);
            const float2 hm = self ? hk : mode_normal(em, a.sweep, pid, pair, a.key0, a.key1);
            update(s, p, ky, my, self, band[ek], hk, hm);
        }
    } else {
        // other tiles: one thread per row ky, all `half` columns c0 + s and
        // their mirrors W - c0 - s.  A Philox call gives the normals of an
        // element pair, so the direct columns take half/2 calls and the
        // mirror columns half/2 + 1 (the pair holding W - c0 - 2pp - 1 also
        // holds the next column pair's first mirror): the same normals as one
        // call per mode, in 9 calls per row instead of 16 at half = 8.  Band
        // indices come from the column-major map, contiguous across the lanes' rows.
        const int c0 = j * half;
        const int16_t* bt = a.bandt + pr.pix_off + (int64_t)c0 * H;
#pragma unroll 1
        for (int ky = opaque(tid); ky < H; ky += NTH) {
            const int my = (H - ky) & (H - 1);
            const uint32_t rk = (uint32_t)(ky * W), rm = (uint32_t)(my * W);
            // mirror normal of slot 2pp (.a of the pair holding W - c0 - 2pp)
            float2 carry = pair_normals((rm + (uint32_t)(W - c0)) >> 1, a.sweep, pid, kStageHarmonic, pair, a.key0,
                                        a.key1).a;
#pragma unroll 1
            for (int pp = 0; pp < half / 2; ++pp) {
                const Normals2 zd = pair_normals((rk + (uint32_t)(c0 + 2 * pp)) >> 1, a.sweep, pid, kStageHarmonic,
                                                 pair, a.key0, a.key1);
                const Normals2 zm = pair_normals((rm + (uint32_t)(W - c0 - 2 * pp - 2)) >> 1, a.sweep, pid,
                                                 kStageHarmonic, pair, a.key0, a.key1);
                const int b0 = bt[(int64_t)(2 * pp) * H + ky], b1 = bt[(int64_t)(2 * pp + 1) * H + ky];
                update(2 * pp, 2 * pp + half, ky, my, false, b0, zd.a, carry);
                update(2 * pp + 1, 2 * pp + 1 + half, ky, my, false, b1, zd.b, zm.b);
                carry = zm.a;
            }
        }
    }
    __syncthreads();
    if (a.add_power)
        for (unsigned u = tid; u < 2 * kNB; u += NTH) {
            const double v = pw[u / kNB][u % kNB];
            if (v != 0.0) atomicAdd(&a.pw[((int64_t)item * 2 + u / kNB) * kNB + u % kNB], v);
        }
    if constexpr (L >= 256) {
        // inverse transform, its last pass straight to HBM
        col_inverse_head<L, TPC, AN>(lds + opaque(cid) * SEG, opaque(lane), twl + opaque(0u));
        col_last_inverse<L, TC, NTH, SEG, AD>(lds, fld, W, opaque(tid), twl + opaque(0u), col_of);
    } else {
        stockham_fft<L, 1, TPC, true>(lds + opaque(cid) * SEG, opaque(lane), opaque(a.tw_col));
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            fld[(int64_t)y * W + pair_column(j, s, half, W)] = lds[s * SEG + swz(y)];
        }
    }
}

// Chi-square sums of one iteration.  Block (item, y): variates [y chunk,
// (y + 1) chunk) of the item's flat index over its bands' degrees of freedom;
// each thread sums an even-length contiguous run in registers and flushes at
// band boundaries.
constexpr int kChiThreads = 256;
constexpr int kChiChunk = 4096;

__global__ __launch_bounds__(kChiThreads) void spectrum_chi_kernel(SpectrumStreamArgs a) {
    __shared__ double acc[2][kNB];
    __shared__ int32_t pre[kNB + 1];
    const int item = blockIdx.x;
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    const int nb = a.band_count[it.prob], bbase = a.band_base[it.prob];
    for (int u = threadIdx.x; u < 2 * kNB; u += blockDim.x) acc[u / kNB][u % kNB] = 0.0;
    if (threadIdx.x == 0) {
        int s = 0;
        for (int b = 0; b < nb; ++b) {
            pre[b] = s;
            s += a.dof[bbase + b];
        }
        pre[nb] = s;
    }
    __syncthreads();
    constexpr int per = kChiChunk / kChiThreads;  // even
    const int e0 = (int)blockIdx.y * kChiChunk + (int)threadIdx.x * per;
    const int e1 = min(pre[nb], e0 + per);
    if (e0 < e1) {
        int b = 0;
        while (pre[b + 1] <= e0) ++b;
        double sa = 0.0, sb = 0.0;
        for (int e = e0; e < e1; e += 2) {
            const Normals2 z = pair_normals((uint32_t)(e >> 1), a.iteration, (uint32_t)pr.pid, kStageSpectrum,
                                            (uint32_t)it.pair, a.key0, a.key1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ee = e + h;
                if (ee >= e1) break;
                if (ee >= pre[b + 1]) {
                    atomicAdd(&acc[0][b], sa);
                    atomicAdd(&acc[1][b], sb);
                    sa = sb = 0.0;
                    while (pre[b + 1] <= ee) ++b;
                }
                const float2 zz = h ? z.b : z.a;
                sa += (double)zz.x * zz.x;
                sb += (double)zz.y * zz.y;
            }
        }
        atomicAdd(&acc[0][b], sa);
        atomicAdd(&acc[1][b], sb);
    }
    __syncthreads();
    for (int u = threadIdx.x; u < 2 * nb; u += blockDim.x) {
        const double v = acc[u / nb][u % nb];
        if (v != 0.0) atomicAdd(&a.chi[((int64_t)item * 2 + u / nb) * kNB + u % nb], v);
    }
}

// draw = 1: new amplitudes theta = (2 beta_0 + sigma/n^2) / x from the sums,
// written to the theta samples (slot >= 0); the sums cleared.  Always: the
// coefficient table for the next sweeps and theta_out.  One block per item.
__global__ void spectrum_theta_kernel(SpectrumStreamArgs a, int draw, int64_t slot) {
    const int item = blockIdx.x;
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    const int nb = a.band_count[it.prob], bbase = a.band_base[it.prob];
    const double n = (double)pr.H * pr.W, T = pr.tau;
    for (int u = threadIdx.x; u < 2 * nb; u += blockDim.x) {
        const int ch = u / nb, b = u % nb;
        const int64_t k = ((int64_t)item * 2 + ch) * kNB + b;
        const int c = 2 * it.pair + ch;
        double th = a.theta[k];
        if (draw) {
            const double x = a.chi[k];
            if (a.dof[bbase + b] > 0 && x > 0.0) th = (2.0 * a.prior_beta + a.pw[k]) / x;
            a.theta[k] = th;
            a.pw[k] = 0.0;
            a.chi[k] = 0.0;
            if (slot >= 0 && a.theta_samples && c < a.chains)
                a.theta_samples[(int64_t)a.chains * a.n_samples * bbase + ((int64_t)c * a.n_samples + slot) * nb + b] =
                    th;
        }
        if (a.theta_out) a.theta_out[(int64_t)a.chains_pad * bbase + (int64_t)c * nb + b] = th;
    }
    __syncthreads();
    float4* coef = a.coef + (int64_t)item * kNB;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        float c[4];
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            const double nP = n * a.theta[((int64_t)item * 2 + ch) * kNB + b];
            c[2 * ch] = (float)(nP / (nP + T) / n);
            c[2 * ch + 1] = (float)(sqrt(n * nP * T / (nP + T)) / n);
        }
        coef[b] = make_float4(c[0], c[1], c[2], c[3]);
    }
}

// Start amplitudes (theta_in or the plan's) and cleared sums.
__global__ void spectrum_init_kernel(SpectrumStreamArgs a) {
    const int item = blockIdx.x;
    const ItemDev it = a.items[item];
    const int nb = a.band_count[it.prob], bbase = a.band_base[it.prob];
    for (int u = threadIdx.x; u < 2 * nb; u += blockDim.x) {
        const int ch = u / nb, b = u % nb;
        const int64_t k = ((int64_t)item * 2 + ch) * kNB + b;
        const int c = 2 * it.pair + ch;
        a.theta[k] = a.theta_in ? a.theta_in[(int64_t)a.chains_pad * bbase + (int64_t)c * nb + b] : a.theta0[bbase + b];
        a.pw[k] = 0.0;
        a.chi[k] = 0.0;
    }
}

}  // namespace

hipError_t launch_spectrum_init(const SpectrumStreamArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(spectrum_init_kernel, dim3((unsigned)a.n_items), dim3(128), 0, s, a);
    hipLaunchKernelGGL(spectrum_theta_kernel, dim3((unsigned)a.n_items), dim3(128), 0, s, a, 0, (int64_t)-1);
    return hipGetLastError();
}

hipError_t launch_spectrum_col(int W, int H, const SpectrumStreamArgs& a, hipStream_t s) {
    switch (H) {
#define MF_CASE(LL)                                                                                    \
    case LL:                                                                                           \
        if (W < PairShape<LL>::TC) return hipErrorInvalidValue;                                        \
        hipLaunchKernelGGL(col_pair_kernel<LL>, dim3((unsigned)((int64_t)a.n_items * (W / PairShape<LL>::TC))), \
                           dim3(PairShape<LL>::NTH), 0, s, a, W);                                      \
        break;
        MF_CASE(16) MF_CASE(32) MF_CASE(64) MF_CASE(128) MF_CASE(256) MF_CASE(512) MF_CASE(1024) MF_CASE(2048)
#undef MF_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spectrum_draw(const SpectrumStreamArgs& a, int max_total_dof, int64_t slot, hipStream_t s) {
    const int blocks = max_total_dof > 0 ? (max_total_dof + kChiChunk - 1) / kChiChunk : 1;
    hipLaunchKernelGGL(spectrum_chi_kernel, dim3((unsigned)a.n_items, (unsigned)blocks), dim3(kChiThreads), 0, s, a);
    hipLaunchKernelGGL(spectrum_theta_kernel, dim3((unsigned)a.n_items), dim3(128), 0, s, a, 1, slot);
    return hipGetLastError();
}

}  // namespace mf
