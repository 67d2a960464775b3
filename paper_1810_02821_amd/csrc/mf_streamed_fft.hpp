// Transform plan shared by the streamed row kernels (sampler and mass
// mapping): one radix sequence per length for the plain and the fused kernels,
// so that both round every butterfly alike.
#pragma once
#include <algorithm>

#include "mf_device.hpp"

namespace mf {

// Transform plan of the fused streamed kernels: a radix-16 pass at one end,
// a radix-RL pass at the other, radix-RM passes between them.  L = 256 uses
// 16 x 4 x 4, so that its RL pass has enough butterflies for every lane and
// holds few values per thread; longer transforms use radix 16 and the
// remainder (2048 = 16 x 16 x 8).
template <int L>
constexpr int last_radix() {
    if (L == 256) return 4;
    int r = L;
    while (r > 16) r /= 16;
    return r;
}
template <int L>
constexpr int middle_radix() { return L == 256 ? 4 : 16; }

// Radix-RM Stockham passes over LDS with NS = NS0, RM NS0, ... while
// NS * RM * TAIL <= L and NS * TAIL < L: all passes before a final pass of
// radix TAIL.  The first pass reads layout AI; with AI >= 0 every pass writes
// the padded layout pad_of picks for it, otherwise the XOR swizzle.
template <int L, int RM, int NS, int TAIL, int TPG, bool INV, int AI = -1>
__device__ __forceinline__ void passes_before(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    if constexpr (NS * RM * TAIL <= L && NS * TAIL < L) {
        constexpr int AO = AI >= 0 ? pad_of(L, RM, NS) : -1;
        stockham_pass<L, RM, NS, TPG, INV, AI, AO>(buf, lane, tw);
        passes_before<L, RM, NS * RM, TAIL, TPG, INV, AO>(buf, lane, tw);
    }
}
// Layout passes_before<L, RM, NS, TAIL, ..., AI> leaves its output in, and the
// largest pad among its input and the layouts it writes.
constexpr int pad_after(int L, int RM, int NS, int TAIL, int AI) {
    int a = AI;
    for (; NS * RM * TAIL <= L && NS * TAIL < L; NS *= RM) a = AI >= 0 ? pad_of(L, RM, NS) : -1;
    return a;
}
constexpr int pad_max(int L, int RM, int NS, int TAIL, int AI) {
    int m = AI;
    for (; NS * RM * TAIL <= L && NS * TAIL < L; NS *= RM) {
        const int a = AI >= 0 ? pad_of(L, RM, NS) : -1;
        m = a > m ? a : m;
    }
    return m;
}

// Column tiles in padded layouts: TC slots of SEG elements.  The phases that
// cross slots are the first forward pass, whose 32 lanes (slot c = l mod TC,
// butterfly j = l / TC) store elements 16 j + r in layout A1, and the last
// inverse pass, whose lanes load elements j + r L/16 in layout AD.  Their
// bank-pair multiplicities (the most of 32 lanes sharing one), summed:
constexpr int tile_conflicts(int TC, int SEG, int A1, int AD) {
    int total = 0;
    for (int phase = 0; phase < 2; ++phase) {
        int worst = 1;
        for (int j0 = 0; j0 < 64; j0 += 32 / TC) {
            int cnt[32] = {};
            for (int l = 0; l < 32; ++l) {
                const int c = l % TC, j = j0 + l / TC;
                const int i = phase == 0 ? 16 * j : j;
                const int A = phase == 0 ? A1 : AD;
                const int b = (c * SEG + i + A * (i >> 5)) & 31;
                cnt[b] += 1;
                worst = cnt[b] > worst ? cnt[b] : worst;
            }
        }
        total += worst;
    }
    return total;
}
// Slot stride of such a tile: the smallest of the 32 strides from `need` up
// with the fewest conflicts.
constexpr int tile_seg(int TC, int A1, int AD, int need) {
    int best = need, bc = 1 << 30;
    for (int sg = need; sg < need + 32; ++sg) {
        const int c = tile_conflicts(TC, sg, A1, AD);
        if (c < bc) {
            bc = c;
            best = sg;
        }
    }
    return best;
}

// One plan per transform length for every row kernel (the fused and the plain
// row kernels, and hence split and resumed runs, then round alike): inverse
// 16, RM..., RL and forward RL, RM..., 16 from 256 points up (powers of two;
// other lengths, which only the plain kernels serve, take stockham_fft).
template <int L, int TPG>
__device__ __forceinline__ void row_inverse(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    if constexpr (L >= 256 && is_pow2(L)) {
        constexpr int RL = last_radix<L>();
        stockham_pass<L, 16, 1, TPG, true>(buf, lane, tw);
        passes_before<L, middle_radix<L>(), 16, RL, TPG, true>(buf, lane, tw);
        stockham_pass<L, RL, L / RL, TPG, true>(buf, lane, tw);
    } else {
        stockham_fft<L, 1, TPG, true>(buf, lane, tw);
    }
}
template <int L, int TPG>
__device__ __forceinline__ void row_forward(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    if constexpr (L >= 256 && is_pow2(L)) {
        constexpr int RL = last_radix<L>();
        stockham_pass<L, RL, 1, TPG, false>(buf, lane, tw);
        passes_before<L, middle_radix<L>(), RL, 16, TPG, false>(buf, lane, tw);
        stockham_pass<L, 16, L / 16, TPG, false>(buf, lane, tw);
    } else {
        stockham_fft<L, 1, TPG, false>(buf, lane, tw);
    }
}

// Value of the neighbouring lane (lane ^ 1) in one DPP move (quad_perm 1,0,3,2).
__device__ __forceinline__ float swap_lanes(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Column tiles of the mirror-paired column kernels (L >= 256): TC slot columns
// of L rows, slot c of column col_of(c), each its own LDS segment of SEG.
// The first forward radix-16 pass reads its inputs straight from HBM (a wave
// covers TC slots of 64/TC rows) and writes its outputs to LDS; the rest of
// the forward transform (radix RM..., RL) runs in LDS and leaves the modes in
// natural order.  The helpers take the exchange layouts of PairLayout (or
// the XOR swizzle, layout -1, for every exchange).
template <int L, int TC>
struct PairLayout {
    static constexpr int RL = last_radix<L>(), RM = middle_radix<L>();
    static constexpr int A1 = pad_of(L, 16, 1);                  // first forward pass writes
    static constexpr int AC = pad_after(L, RM, 16, RL, A1);      // middle forward passes leave
    static constexpr int AN = pad_of(L, RL, L / RL);             // natural-order modes
    static constexpr int AF = pad_of(L, RL, 1);                  // first inverse pass writes
    static constexpr int AD = pad_after(L, RM, RL, 16, AF);      // middle inverse passes leave
    static constexpr int AMAX = std::max({pad_max(L, RM, 16, RL, A1), AN, pad_max(L, RM, RL, 16, AF)});
    static constexpr int SEG = tile_seg(TC, A1, AD, pad_len(L, AMAX));
};

// LDS per CU on gfx950, and whether a kernel whose LDS grows from `before`
// to `after` bytes per workgroup keeps as many resident workgroups per CU,
// or at least four (small tiles, whose launches are rarely LDS-bound).
constexpr int kLdsPerCU = 160 * 1024;
constexpr bool lds_keeps_blocks(int before, int after) {
    const int b = kLdsPerCU / before, a = kLdsPerCU / after;
    return a >= (b < 4 ? b : 4);
}

template <int L, int TC, int NTH, int SEG, int A1 = -1, typename ColOf>
__device__ __forceinline__ void col_first_forward(float2* lds, const float2* fld, int W, unsigned tid, ColOf col_of) {
    constexpr int NT16 = L / 16;
    constexpr int IT16 = (TC * NT16 + NTH - 1) / NTH;
#pragma unroll
    for (int i = 0; i < IT16; ++i) {
        const unsigned b = tid + i * NTH;
        if ((TC * NT16) % NTH == 0 || b < (unsigned)(TC * NT16)) {
            const unsigned c = b % TC, j = b / TC;
            const int64_t col = col_of((int)c);
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = fld[(int64_t)(j + r * NT16) * W + col];
            dft<16, false>(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) lds[c * SEG + lpos_run<A1, 16>(j, r)] = v[r];
        }
    }
}
template <int L, int TPC, int A1 = -1>
__device__ __forceinline__ void col_forward_rest(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    constexpr int RL = last_radix<L>(), RM = middle_radix<L>();
    constexpr int AC = pad_after(L, RM, 16, RL, A1);
    constexpr int AN = A1 >= 0 ? pad_of(L, RL, L / RL) : -1;
    passes_before<L, RM, 16, RL, TPC, false, A1>(buf, lane, tw);
    stockham_pass<L, RL, L / RL, TPC, false, AC, AN>(buf, lane, tw);
}
// Inverse counterpart: radix RL, RM... in LDS, then the last radix-16 pass
// writes natural-order rows straight to HBM.
template <int L, int TPC, int AN = -1>
__device__ __forceinline__ void col_inverse_head(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    constexpr int RL = last_radix<L>();
    constexpr int AF = AN >= 0 ? pad_of(L, RL, 1) : -1;
    stockham_pass<L, RL, 1, TPC, true, AN, AF>(buf, lane, tw);
    passes_before<L, middle_radix<L>(), RL, 16, TPC, true, AF>(buf, lane, tw);
}
template <int L, int TC, int NTH, int SEG, int AD = -1, typename ColOf>
__device__ __forceinline__ void col_last_inverse(const float2* lds, float2* fld, int W, unsigned tid,
                                                 const float2* __restrict__ tw, ColOf col_of) {
    constexpr int NT16 = L / 16;
    constexpr int IT16 = (TC * NT16 + NTH - 1) / NTH;
#pragma unroll
    for (int i = 0; i < IT16; ++i) {
        const unsigned b = tid + i * NTH;
        if ((TC * NT16) % NTH == 0 || b < (unsigned)(TC * NT16)) {
            const unsigned c = b % TC, j = b / TC;
            const int64_t col = col_of((int)c);
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = lds[c * SEG + lpos_step<AD, NT16>(j, r)];
#pragma unroll
            for (int r = 1; r < 16; ++r) v[r] = cmulc(v[r], tw[r * j]);
            dft<16, true>(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) fld[(int64_t)(j + r * NT16) * W + col] = v[r];
        }
    }
}

}  // namespace mf
