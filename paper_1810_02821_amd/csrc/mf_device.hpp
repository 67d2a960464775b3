// Device building blocks of the messenger-field sweep for gfx950:
// complex arithmetic, small in-register DFTs, a Stockham FFT pass over LDS,
// and the counter-based normal generator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV> __device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Twiddle W_N^j = exp(-2 pi i j / N) for the forward transform; the inverse
// transform uses its conjugate.  Values are FP64-evaluated constants rounded
// to FP32.
constexpr float kC8 = 0.70710678118654752f;   // cos(pi/4)
constexpr float kC16 = 0.92387953251128676f;  // cos(pi/8)
constexpr float kS16 = 0.38268343236508977f;  // sin(pi/8)

template <bool INV> __device__ __forceinline__ float2 tw_apply(float2 v, float c, float s) {
    // v * (c - i s) forward, v * (c + i s) inverse
    return INV ? make_float2(fmaf(v.x, c, -v.y * s), fmaf(v.y, c, v.x * s))
               : make_float2(fmaf(v.x, c, v.y * s), fmaf(v.y, c, -v.x * s));
}

// ------------------------------------------------------- in-register DFTs --
// Natural order in and out: v[k] <- sum_n v[n] exp(-+2 pi i n k / R).
template <bool INV> __device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV> __device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV> __device__ __forceinline__ void dft8(float2 (&v)[8]) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    o1 = cscale(tw_apply<INV>(o1, 1.0f, 1.0f), kC8);  // W8^1
    o2 = mul_mi<INV>(o2);                              // W8^2
    o3 = cscale(tw_apply<INV>(o3, -1.0f, 1.0f), kC8); // W8^3 = -c - i c (fwd)
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16 = 4 x 4: inner DFT4 over stride-4 groups, twiddle W16^(n1 k1), outer DFT4.
template <bool INV> __device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4<INV>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
    // element (n1, k1) sits at v[n1 + 4 k1]; multiply by W16^(n1 k1)
    v[1 + 4] = tw_apply<INV>(v[1 + 4], kC16, kS16);      // W^1
    v[2 + 4] = cscale(tw_apply<INV>(v[2 + 4], 1.f, 1.f), kC8); // W^2
    v[3 + 4] = tw_apply<INV>(v[3 + 4], kS16, kC16);      // W^3
    v[1 + 8] = cscale(tw_apply<INV>(v[1 + 8], 1.f, 1.f), kC8); // W^2
    v[2 + 8] = mul_mi<INV>(v[2 + 8]);                    // W^4
    v[3 + 8] = cscale(tw_apply<INV>(v[3 + 8], -1.f, 1.f), kC8); // W^6
    v[1 + 12] = tw_apply<INV>(v[1 + 12], kS16, kC16);    // W^3
    v[2 + 12] = cscale(tw_apply<INV>(v[2 + 12], -1.f, 1.f), kC8); // W^6
    v[3 + 12] = tw_apply<INV>(v[3 + 12], -kC16, -kS16);  // W^9 = -W^1
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // now X[k1 + 4 k2] sits at v[4 k1 + k2]: transpose to natural order
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
}

// 3-point DFT: with u = v1 + v2 and the primitive root exp(-+2 pi i/3) =
// -1/2 -+ i sqrt(3)/2, X0 = v0 + u, X1,2 = (v0 - u/2) -+ i (sqrt(3)/2) (v1 - v2).
constexpr float kS3 = 0.86602540378443865f;  // sin(pi/3)
template <bool INV> __device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
    const float2 u = cadd(a1, a2);
    const float2 m = make_float2(fmaf(-0.5f, u.x, a0.x), fmaf(-0.5f, u.y, a0.y));
    const float2 dd = mul_mi<INV>(cscale(csub(a1, a2), kS3));
    a0 = cadd(a0, u);
    a1 = cadd(m, dd);
    a2 = csub(m, dd);
}

template <int R, bool INV> __device__ __forceinline__ void dft(float2 (&v)[R]) {
    if constexpr (R == 2) dft2<INV>(v[0], v[1]);
    else if constexpr (R == 3) dft3<INV>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 16) dft16<INV>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ------------------------------------------------- Stockham pass over LDS --
// Two families of LDS layouts for the element exchanges between passes.
//
// Layout -1: element i at swz(i).  The low five bits (one row of the 64 x
// 4-byte banks for 8-byte elements) are XORed with a function of the higher
// bits, which keeps every read and write of every pass below free of bank
// conflicts for lengths 16..2048 (within one transform per 32 lanes).  Any
// element's position needs its own address arithmetic.
//
// Layout A >= 0: element i at i + A floor(i / 32), that is A unused elements
// after every block of 32.  The elements a thread reads (j + r NT) or writes
// (o + r NS) then sit at one base plus constant offsets, which the ds
// instructions take as immediates.  A is chosen per exchange by pad_of so
// that the writing pass is free of bank conflicts within 32 lanes; the reads
// (32 consecutive elements per 32 lanes) are free of them for every A.
__host__ __device__ __forceinline__ unsigned swz(unsigned i) {
    const unsigned h = i >> 5;
    return i ^ (((h & 7u) ^ (((h >> 1) & 3u) << 3)) & 31u);
}
template <int A>
__host__ __device__ __forceinline__ unsigned lpos(unsigned i) {
    if constexpr (A < 0) return swz(i);
    else return i + (unsigned)A * (i >> 5);
}

// Element j + r STEP of an exchange in layout A (reads of a pass with STEP =
// L / R): a base and constant offsets when STEP is a multiple of 32.
template <int A, int STEP>
__host__ __device__ __forceinline__ unsigned lpos_step(unsigned j, int r) {
    if constexpr (A >= 0 && STEP % 32 == 0) return lpos<A>(j) + r * (STEP + A * (STEP / 32));
    else return lpos<A>(j + r * STEP);
}
// Element R j + r (r < R) in layout A (writes of a first pass, NS = 1): the
// run stays inside one block of 32 when R divides 32.
template <int A, int R>
__host__ __device__ __forceinline__ unsigned lpos_run(unsigned j, int r) {
    if constexpr (A >= 0 && 32 % R == 0) return lpos<A>(R * j) + r;
    else return lpos<A>(R * j + r);
}

// Element o + r NS in layout A, written by a radix-R pass after NS points
// with o = (j / NS) NS R + j mod NS: a base and constant offsets when NS is a
// multiple of 32, or when NS divides 32 and NS R is a multiple of 32 (then
// o's low five bits are j mod NS < NS, so o + r NS stays in the block of
// o + (r NS mod 32)).
template <int A, int R, int NS>
__host__ __device__ __forceinline__ unsigned lpos_write(unsigned o, int r) {
    if constexpr (A >= 0 && NS % 32 == 0) return lpos<A>(o) + r * (NS + A * (NS / 32));
    else if constexpr (A >= 0 && 32 % NS == 0 && (NS * R) % 32 == 0) return lpos<A>(o) + r * NS + A * ((r * NS) >> 5);
    else return lpos<A>(o + r * NS);
}

// True if the 32 lanes l < min(32, L / R) of a radix-R pass after NS points,
// writing element (l / NS) NS R + l % NS + NS r for one r, hit 32 distinct
// bank pairs under layout A, for every r.
constexpr bool pad_writes_ok(int L, int R, int NS, int A) {
    const int lanes = L / R < 32 ? L / R : 32;
    for (int r = 0; r < R; ++r) {
        unsigned seen = 0;
        for (int l = 0; l < lanes; ++l) {
            const int i = (l / NS) * NS * R + l % NS + NS * r;
            const unsigned bit = 1u << ((i + A * (i >> 5)) & 31);
            if (seen & bit) return false;
            seen |= bit;
        }
    }
    return true;
}
// Smallest pad for the exchange a radix-R pass after NS points writes.
constexpr int pad_of(int L, int R, int NS) {
    for (int A = 1; A <= 32; ++A)
        if (pad_writes_ok(L, R, NS, A)) return A;
    return 1;
}
// Elements an exchange of length L occupies under layout A (up to and
// including the position of element L - 1).
constexpr int pad_len(int L, int A) { return A < 0 ? L : L + A * ((L - 1) / 32); }

// One radix-R pass of a length-L transform held in `buf`, reading the
// exchange in layout AI and writing in layout AO.  `lane` in [0, TPG)
// indexes the TPG threads that own this transform; NS is the product of the
// radices already applied.  Input in the Stockham order of the previous pass,
// output in the order of the next; after the last pass the sequence is in
// natural order.  `tw` holds W_L^r, r < L.  The pass reads every element into
// registers before writing (in place), so it needs the two barriers; every
// thread of the block must call it.
template <int L, int R, int NS, int TPG, bool INV, int AI = -1, int AO = -1>
__device__ __forceinline__ void stockham_pass(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    constexpr int NT = L / R;
    constexpr int TPT = (NT + TPG - 1) / TPG;
    float2 v[TPT][R];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const unsigned j = lane + t * TPG;
        if ((NT % TPG) == 0 || j < (unsigned)NT) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[t][r] = buf[lpos_step<AI, NT>(j, r)];
            if constexpr (NS > 1) {
                const unsigned k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float2 w = tw[(r * k) * (L / (NS * R))];
                    v[t][r] = INV ? cmulc(v[t][r], w) : cmul(v[t][r], w);
                }
            }
            dft<R, INV>(v[t]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const unsigned j = lane + t * TPG;
        if ((NT % TPG) == 0 || j < (unsigned)NT) {
            const unsigned k = j % NS;
            const unsigned o = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[lpos_write<AO, R, NS>(o, r)] = v[t][r];
        }
    }
    __syncthreads();
}

// Transform lengths: 2^a 3^b with a >= 1 (even sides).
constexpr bool is_pow2(int L) { return L > 0 && (L & (L - 1)) == 0; }

// Radix plan: radix-16 passes while 16 divides what is left, then one
// radix-8/4/2 pass for the rest of the power of two, then radix-3 passes.
template <int REM>
constexpr int next_radix() {
    return REM % 16 == 0 ? 16 : REM % 8 == 0 ? 8 : REM % 4 == 0 ? 4 : REM % 2 == 0 ? 2 : 3;
}
// A whole transform in LDS, reading layout AI and leaving its natural-order
// output in layout AOUT; with AI >= 0 the exchanges between its passes take
// the pads pad_of picks, otherwise the XOR swizzle.
template <int L, int NS, int TPG, bool INV, int AI = -1, int AOUT = -1>
__device__ __forceinline__ void stockham_fft(float2* buf, unsigned lane, const float2* __restrict__ tw) {
    if constexpr (NS < L) {
        constexpr int R = next_radix<L / NS>();
        static_assert((L / NS) % R == 0, "transform length must be 2^a 3^b");
        constexpr int AO = NS * R == L ? AOUT : (AI >= 0 ? pad_of(L, R, NS) : -1);
        stockham_pass<L, R, NS, TPG, INV, AI, AO>(buf, lane, tw);
        stockham_fft<L, NS * R, TPG, INV, AO, AOUT>(buf, lane, tw);
    }
}

// Row stride in LDS of a transform of length L: the swizzle permutes within
// 32-element blocks, so a length that is neither a power of two nor a
// multiple of 32 takes whole blocks.
template <int L>
constexpr int lds_stride() { return (is_pow2(L) || L % 32 == 0) ? L : (L + 31) / 32 * 32; }

// Workgroups are handed to the eight XCDs round-robin.  Renumber them so that
// each XCD runs a contiguous range of logical blocks: neighbouring tiles that
// share cache lines or table rows then meet in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned x = b & 7u, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// -------------------------------------------------------- normal variates --
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11): words 0 and
// 2 are multiplied by two odd constants; the high halves are mixed with words
// 1, 3 and the round key, the low halves move to words 1 and 3; the key is
// bumped by two Weyl constants after every round.
struct Philox4 {
    uint32_t x, y, z, w;
};

// a ^ b ^ c in one gfx950 VALU instruction (v_bitop3_b32, truth table 0x96 =
// odd parity); the compiler does not form it on its own here.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
    // round 1 in plain C: with uniform counter words most of it folds to scalar ops
    {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Box-Muller on the top 24 bits of two words: u1 in (0, 1], u2 in [0, 1),
// both exact in FP32.  v_log_f32 is log2 and v_sin/v_cos take revolutions.
__device__ __forceinline__ float2 box_muller(uint32_t xa, uint32_t xb) {
    const float u1 = (float)((xa >> 8) + 1u) * 0x1p-24f;
    const float u2 = (float)(xb >> 8) * 0x1p-24f;
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    return make_float2(r * __builtin_amdgcn_cosf(u2), r * __builtin_amdgcn_sinf(u2));
}

enum : uint32_t { kStagePixel = 0, kStageHarmonic = 1, kStageInit = 2 };

// Four normals for elements (2j, 2j+1) of one chain pair: .a for 2j, .b for 2j+1;
// .x feeds chain 2p (or the real part), .y chain 2p+1 (or the imaginary part).
struct Normals2 {
    float2 a, b;
};
__device__ __forceinline__ Normals2 pair_normals(uint32_t j, uint32_t sweep, uint32_t prob, uint32_t stage,
                                                 uint32_t pair, uint32_t k0, uint32_t k1) {
    const Philox4 r = philox4x32_10(j, sweep, (prob << 8) | stage, pair, k0, k1);
    return {box_muller(r.x, r.y), box_muller(r.z, r.w)};
}

}  // namespace mf
