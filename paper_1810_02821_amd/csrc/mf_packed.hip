// Column step of the streamed sampler for packed items: two single-chain
// problems of one size class share a complex field, chain 0 of problem A in
// the real part and chain 0 of problem B in the imaginary part.  Each keeps
// its own coefficients (noise, data, spectrum, tau) and its own random stream
// (pair 0, the words a lone chain uses), so every chain equals the one the
// unpacked sampler draws; the transforms are shared.
//
// With Z = F(t_A + i t_B), problem A's spectrum is (Z(k) + conj Z(-k)) / 2 and
// B's (Z(k) - conj Z(-k)) / 2i.  Algorithm 1's Fourier step of each chain
// (S_A = f_A A + w_A Re-part draw, S_B likewise; the Re part of w eta is
// (w eta(k) + w conj eta(-k)) / 2) recombines into
//   S(k) = f+ Z(k) + f- conj Z(-k)
//          + w_A (eta_A(k) + conj eta_A(-k)) / 2 + i w_B (eta_B(k) + conj eta_B(-k)) / 2,
// f+- = (f_A +- f_B) / 2, so every mode meets its mirror -k.  Column tiles
// hold mirror pairs of columns (columns c and W - c, with the self-mirror
// columns 0 and W/2 together in tile 0), as in the hierarchical sampler.
#include "mf_device.hpp"
#include "mf_kernels.hpp"
#include "mf_streamed_fft.hpp"

namespace mf {

namespace {

// Tile of the packed column step: 16 columns (8 and their mirrors), 8 from
// 1024 rows; 32 threads per column at 256 and 512 rows (at 256, 512 threads
// ran the uneven batch's 256^2 class 1.8% faster than 256), 64 at 1024 (8 x
// 512: 7% faster on 1024^2 problems than 16 x 1024), 128 at 2048.
template <int L>
struct PackShape {
    static constexpr int TC = L >= 1024 ? 8 : 16;
    static constexpr int NTH = L >= 2048 ? 1024 : (L >= 256 ? 512 : 256);
    static constexpr int TPC = NTH / TC;
    static constexpr int SEG = L + 32 / TC;
};

// Opaque copies: values derived from them are not kept live across the transforms.
__device__ __forceinline__ unsigned opaque_u(unsigned v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Column held by slot s of tile j (slots s < half: columns j half + s; the
// others their mirrors W - c, with column 0's mirror slot holding W/2).
__device__ __forceinline__ int mirror_column(int j, int s, int half, int W) {
    if (s < half) return j * half + s;
    const int c = j * half + (s - half);
    return c == 0 ? W / 2 : W - c;
}

// Harmonic-stage normal of mode e of pair 0 of problem pid.
__device__ __forceinline__ float2 chain0_mode_normal(uint32_t e, uint32_t sweep, uint32_t pid, uint32_t k0,
                                                     uint32_t k1) {
    const Normals2 z = pair_normals(e >> 1, sweep, pid, kStageHarmonic, 0u, k0, k1);
    return (e & 1u) ? z.b : z.a;
}

template <int L>
__global__ __launch_bounds__(PackShape<L>::NTH) void col_pack_kernel(SweepArgs a, int W) {
    constexpr int TC = PackShape<L>::TC, NTH = PackShape<L>::NTH, TPC = PackShape<L>::TPC;
    // padded exchange layouts from 256 rows (the HBM-side passes) where they
    // keep the resident workgroups per CU, else the XOR swizzle
    constexpr int kExtra = 8 * L;  // twiddles and tables beside the tile
    constexpr bool kPad = L >= 256 && lds_keeps_blocks(TC * PackShape<L>::SEG * 8 + kExtra,
                                                       TC * PairLayout<L, TC>::SEG * 8 + kExtra);
    constexpr int A1 = kPad ? PairLayout<L, TC>::A1 : -1, AN = kPad ? PairLayout<L, TC>::AN : -1;
    constexpr int AD = kPad ? PairLayout<L, TC>::AD : -1;
    constexpr int SEG = kPad ? PairLayout<L, TC>::SEG : PackShape<L>::SEG;
    constexpr int H = L;
    constexpr int half = TC / 2;
    __shared__ float2 lds[TC * SEG];
    __shared__ float2 twl[L >= 256 ? L : 1];
    const unsigned tid = threadIdx.x;
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int item = (int)(t / (W / TC));
    const int j = (int)(t % (W / TC));
    const ItemDev it = a.items[item];
    const ProbDev pa = a.probs[it.prob];
    const ProbDev pb = it.pair >= 0 ? a.probs[it.pair] : pa;
    float2* fld = a.field + it.field_off;

    auto col_of = [&](int s) { return mirror_column(j, s, half, W); };
    if constexpr (L >= 256) {
        col_first_forward<L, TC, NTH, SEG, A1>(lds, fld, W, tid, col_of);
        for (unsigned i = tid; i < (unsigned)L; i += NTH) twl[i] = a.tw_col[i];
    } else {
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            lds[s * SEG + swz(y)] = fld[(int64_t)y * W + mirror_column(j, s, half, W)];
        }
    }
    __syncthreads();
    const unsigned cid = tid / TPC, lane = tid % TPC;
    if constexpr (L >= 256) col_forward_rest<L, TPC, A1>(lds + cid * SEG, lane, twl);
    else stockham_fft<L, 1, TPC, false>(lds + cid * SEG, lane, a.tw_col);

    const float TA = a.lambda * pa.tau, TB = a.lambda * pb.tau;
    const float inv_n = 1.0f / ((float)H * (float)W);
    const uint32_t pidA = (uint32_t)pa.pid, pidB = (uint32_t)pb.pid;
    // Fourier step of mode k (slot s, row ky) and its mirror -k (slot p, row
    // my), given both problems' n P(k) (= n P(-k): isotropic spectra) and
    // harmonic normals at k and -k
    auto update = [&](int s, int p, int ky, int my, bool self, float PA, float PB, float2 hkA, float2 hmA,
                      float2 hkB, float2 hmB) {
        float2& zk = lds[s * SEG + lpos<AN>(ky)];
        float2& zm = lds[p * SEG + lpos<AN>(my)];
        const float2 Zk = zk, Zm = zm;
        const float rA = __builtin_amdgcn_rcpf(PA + TA), rB = __builtin_amdgcn_rcpf(PB + TB);
        const float fA = PA * rA * inv_n, fB = PB * rB * inv_n;
        const float wA = __builtin_amdgcn_sqrtf(PA * TA * rA * inv_n), wB = __builtin_amdgcn_sqrtf(PB * TB * rB * inv_n);
        const float fp = 0.5f * (fA + fB), fm = 0.5f * (fA - fB);
        float2 Nk = make_float2(0.f, 0.f), Nm = Nk;
        if (a.stochastic) {
            const float ha = 0.5f * wA, hb = it.pair >= 0 ? 0.5f * wB : 0.f;
            // w_A (eta_A(k) + conj eta_A(-k)) / 2 + i w_B (eta_B(k) + conj eta_B(-k)) / 2, and with k, -k swapped
            Nk = make_float2(fmaf(ha, hkA.x + hmA.x, -hb * (hkB.y - hmB.y)), fmaf(ha, hkA.y - hmA.y, hb * (hkB.x + hmB.x)));
            Nm = make_float2(fmaf(ha, hmA.x + hkA.x, -hb * (hmB.y - hkB.y)), fmaf(ha, hmA.y - hkA.y, hb * (hmB.x + hkB.x)));
        }
        const float2 Sk = make_float2(fmaf(fp, Zk.x, fm * Zm.x) + Nk.x, fmaf(fp, Zk.y, -fm * Zm.y) + Nk.y);
        const float2 Sm = make_float2(fmaf(fp, Zm.x, fm * Zk.x) + Nm.x, fmaf(fp, Zm.y, -fm * Zk.y) + Nm.y);
        zk = Sk;
        if (!self) zm = Sm;
    };
    if (j == 0) {
        // tile 0: one job per mode pair {k, -k}; the self-mirror columns 0
        // (slot 0) and W/2 (slot half) take the rows ky <= H/2
        const int jobs = half * H + H / 2 + 1;
#pragma unroll 1
        for (int q = opaque_u(tid); q < jobs; q += NTH) {
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
            const uint32_t ek = (uint32_t)(ky * W + mirror_column(j, s, half, W));
            const uint32_t em = (uint32_t)(my * W + mirror_column(j, p, half, W));
            float2 hkA{}, hmA{}, hkB{}, hmB{};
            if (a.stochastic) {
                hkA = chain0_mode_normal(ek, a.sweep, pidA, a.key0, a.key1);
                hmA = self ? hkA : chain0_mode_normal(em, a.sweep, pidA, a.key0, a.key1);
                hkB = chain0_mode_normal(ek, a.sweep, pidB, a.key0, a.key1);
                hmB = self ? hkB : chain0_mode_normal(em, a.sweep, pidB, a.key0, a.key1);
            }
            update(s, p, ky, my, self, a.nP[pa.pix_off + ek], a.nP[pb.pix_off + ek], hkA, hmA, hkB, hmB);
        }
    } else {
        // other tiles: one thread per row ky, all `half` columns c0 + s and
        // their mirrors W - c0 - s.  A Philox call gives the normals of an
        // element pair {2e, 2e+1}: the direct columns take half/2 calls per
        // problem, and the mirror columns half/2 + 1, because the pair that
        // holds W - c0 - 2pp - 1 (.b) also holds W - c0 - 2pp - 2 (.a), the
        // next column pair's first mirror.  The same normals as one call per
        // mode, in 9 calls per problem instead of 16 at half = 8.  The
        // coefficients come from the column-pair table nPt, whose rows of one
        // column pair are contiguous (the lanes' rows are).
        const int c0 = j * half;
        const float2* nptA = a.nPt + pa.pix_off / 2 + (int64_t)(c0 / 2) * H;
        const float2* nptB = a.nPt + pb.pix_off / 2 + (int64_t)(c0 / 2) * H;
#pragma unroll 1
        for (int ky = opaque_u(tid); ky < H; ky += NTH) {
            const int my = (H - ky) & (H - 1);
            const uint32_t rk = (uint32_t)(ky * W), rm = (uint32_t)(my * W);
            float2 cA{}, cB{};  // mirror normal of slot 2pp (.a of the pair holding W - c0 - 2pp)
            if (a.stochastic) {
                const uint32_t e = (rm + (uint32_t)(W - c0)) >> 1;
                cA = pair_normals(e, a.sweep, pidA, kStageHarmonic, 0u, a.key0, a.key1).a;
                cB = pair_normals(e, a.sweep, pidB, kStageHarmonic, 0u, a.key0, a.key1).a;
            }
#pragma unroll 1
            for (int pp = 0; pp < half / 2; ++pp) {
                float2 dA0{}, dA1{}, dB0{}, dB1{}, mA1{}, mB1{}, nA{}, nB{};
                if (a.stochastic) {
                    const uint32_t ed = (rk + (uint32_t)(c0 + 2 * pp)) >> 1;
                    const Normals2 zA = pair_normals(ed, a.sweep, pidA, kStageHarmonic, 0u, a.key0, a.key1);
                    const Normals2 zB = pair_normals(ed, a.sweep, pidB, kStageHarmonic, 0u, a.key0, a.key1);
                    dA0 = zA.a;
                    dA1 = zA.b;
                    dB0 = zB.a;
                    dB1 = zB.b;
                    const uint32_t emx = (rm + (uint32_t)(W - c0 - 2 * pp - 2)) >> 1;
                    const Normals2 mA = pair_normals(emx, a.sweep, pidA, kStageHarmonic, 0u, a.key0, a.key1);
                    const Normals2 mB = pair_normals(emx, a.sweep, pidB, kStageHarmonic, 0u, a.key0, a.key1);
                    mA1 = mA.b;  // column W - c0 - 2pp - 1
                    mB1 = mB.b;
                    nA = mA.a;   // column W - c0 - 2pp - 2: the next pair's slot 2pp + 2
                    nB = mB.a;
                }
                const float2 PA = nptA[(int64_t)pp * H + ky], PB = nptB[(int64_t)pp * H + ky];
                update(2 * pp, 2 * pp + half, ky, my, false, PA.x, PB.x, dA0, cA, dB0, cB);
                update(2 * pp + 1, 2 * pp + 1 + half, ky, my, false, PA.y, PB.y, dA1, mA1, dB1, mB1);
                cA = nA;
                cB = nB;
            }
        }
    }
    __syncthreads();
    if constexpr (L >= 256) {
        col_inverse_head<L, TPC, AN>(lds + opaque_u(cid) * SEG, opaque_u(lane), twl + opaque_u(0u));
        col_last_inverse<L, TC, NTH, SEG, AD>(lds, fld, W, opaque_u(tid), twl + opaque_u(0u), col_of);
    } else {
        stockham_fft<L, 1, TPC, true>(lds + opaque_u(cid) * SEG, opaque_u(lane), a.tw_col);
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            fld[(int64_t)y * W + mirror_column(j, s, half, W)] = lds[s * SEG + swz(y)];
        }
    }
}

}  // namespace

hipError_t launch_col_pack(int W, int H, const SweepArgs& a, hipStream_t s) {
    if (!is_pow2(W) || !is_pow2(H) || W < 16 || !a.nPt) return hipErrorInvalidValue;
    switch (H) {
#define MF_PACK_CASE(N)                                                                                  \
    case N:                                                                                              \
        hipLaunchKernelGGL((col_pack_kernel<N>), dim3((unsigned)((int64_t)a.n_items * (W / PackShape<N>::TC))), \
                           dim3(PackShape<N>::NTH), 0, s, a, W);                                         \
        break;
        MF_PACK_CASE(16) MF_PACK_CASE(32) MF_PACK_CASE(64) MF_PACK_CASE(128) MF_PACK_CASE(256) MF_PACK_CASE(512)
        MF_PACK_CASE(1024) MF_PACK_CASE(2048)
#undef MF_PACK_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf
