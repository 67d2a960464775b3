// Mass mapping (Sec. 5) on the streamed kernels, for size classes the
// persistent kernel does not hold (256^2 and more, or H != W).  The sweep is
// the one of mf_shear.hip:
//   t      = (1 - a) A kappa + a gamma + sqrt(T (1 - a)) xi        (row kernel)
//   u(k)   = conj(D_k) F(t)(k)
//   kappa^ = f_+ u(k) + f_- conj(u(-k)) + w_+ eta(k) + w_- conj(eta(-k))
//   state  = F^-1(D kappa^)                                        (column kernel)
// The E/B split needs each mode k together with its mirror -k, so the column
// kernel uses mirror-paired tiles as the streamed hierarchical sampler does:
// tile j of an item holds columns c = j TC/2 + i and their mirrors W - c,
// with the self-mirror columns 0 and W/2 both in tile 0.
// Contraction within a source expression only, as in mf_streamed.hip: the
// fused and the plain row kernels round alike, so split runs repeat
// uninterrupted ones bit for bit.
#pragma clang fp contract(on)
#include "mf_device.hpp"
#include "mf_kernels.hpp"
#include "mf_shear.hpp"
#include "mf_streamed_fft.hpp"

namespace mf {

namespace {

constexpr int kRowThreads = 256;

// Rows per block of the shear row kernels: 2048 / L, and 8 at 512 points (as
// the sampler's fused row kernel; 1.3% faster than 4 on a 512^2 run).
template <int L>
struct ShearRowShape {
    static constexpr int ROWS = L == 512 ? 8 : ((2048 / L) < 1 ? 1 : (2048 / L));
    static constexpr int TPR = kRowThreads / ROWS;
};

// Tiles of the mirror-paired column kernel, timed on the hierarchical and
// mass-mapping samplers: 16 columns below 512 rows (512 threads at 256), 8
// columns from 512 rows with 256 threads at 512, 512 at 1024 and 1024 at 2048
// (at 512 and 1024 rows 3.8-11.6% faster than 16 columns of 512 and 1024
// threads).
template <int L>
struct ShearColShape {
    static constexpr int TC = L >= 512 ? 8 : 16;
    static constexpr int NTH = L >= 2048 ? 1024 : (L == 1024 ? 512 : (L == 256 ? 512 : 256));
    static constexpr int TPC = NTH / TC;
    static constexpr int SEG = L + 32 / TC;
};

__device__ __forceinline__ unsigned opaque(unsigned v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ const float2* opaque(const float2* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Signed frequency of index k of an n-point transform (numpy's fftfreq * n).
__device__ __forceinline__ int sfreq(int k, int n) { return k < n / 2 ? k : k - n; }

// D at mode (ky, kx) of an H x W grid (k_1 along x); D_0 = 0.
__device__ __forceinline__ float2 ks(int ky, int kx, int H, int W) {
    const float x = (float)sfreq(kx, W), y = (float)sfreq(ky, H);
    const float r = __builtin_amdgcn_rcpf(fmaxf(fmaf(x, x, y * y), 1.f));
    return make_float2((x * x - y * y) * r, 2.f * x * y * r);
}

// D at -k from D at k: equal, except that the mixed term changes sign when
// exactly one component of k is a Nyquist index (-k aliases to itself there).
__device__ __forceinline__ float2 ks_mirror(float2 d, int ky, int kx, int H, int W) {
    const bool flip = (ky == H / 2) != (kx == W / 2);
    return make_float2(d.x, flip ? -d.y : d.y);
}

__device__ __forceinline__ float2 mulc(float2 z, float2 d) {  // conj(d) z
    return make_float2(fmaf(d.x, z.x, d.y * z.y), fmaf(d.x, z.y, -d.y * z.x));
}

struct Filt {
    float fp, fm, wp, wm;
};

// f/n and w/n of the E and B fields at one mode, as (f_+, f_-, w_+, w_-); at
// k = 0 the messenger variance goes to infinity: f = 0 and w draws the prior.
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

__device__ __forceinline__ float2 mode_normal(uint32_t e, uint32_t sweep, uint32_t pid, uint32_t chain,
                                              uint32_t k0, uint32_t k1) {
    const Normals2 z = pair_normals(e >> 1, sweep, pid, kStageHarmonic, chain, k0, k1);
    return (e & 1u) ? z.b : z.a;
}

__device__ __forceinline__ int pair_column(int j, int s, int half, int W) {
    if (s < half) return j * half + s;
    const int c = j * half + (s - half);
    return c == 0 ? W / 2 : W - c;
}

// Rows of all items (item fastest).  kShearInv / kShearFwd bits as in the
// sampler's row kernel; kShearEmit: inverse row FFT of the kappa staging field
// into the samples (slot >= 0) or kappa_out.
template <int L, int MODE>
__global__ __launch_bounds__(kRowThreads) void shear_row_kernel(ShearStreamArgs a, int H) {
    constexpr int ROWS = ShearRowShape<L>::ROWS, TPR = ShearRowShape<L>::TPR;
    constexpr int W = L;
    __shared__ float2 lds[ROWS * L];
    __shared__ int32_t row_item[ROWS], row_y[ROWS];  // one division per row
    const unsigned tid = threadIdx.x;
    const int64_t total_rows = (int64_t)a.n_items * H;
    const int64_t grow0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * ROWS;
    for (unsigned r = tid; r < (unsigned)ROWS; r += kRowThreads) {
        const int64_t g = grow0 + r;
        row_item[r] = g < total_rows ? (int32_t)(g % a.n_items) : -1;
        row_y[r] = g < total_rows ? (int32_t)(g / a.n_items) : 0;
    }
    __syncthreads();
    const float2* src = (MODE & kShearEmit) ? a.kfield : a.field;
#pragma unroll
    for (int i = 0; i < ROWS * L / kRowThreads; ++i) {
        const unsigned e = tid + i * kRowThreads;
        const unsigned r = e / L, x = e % L;
        float2 v = make_float2(0.f, 0.f);
        if (row_item[r] >= 0) v = src[a.items[row_item[r]].field_off + (int64_t)row_y[r] * W + x];
        lds[r * L + swz(x)] = v;
    }
    __syncthreads();
    const unsigned rid = tid / TPR, lane = tid % TPR;
    const bool valid = row_item[rid] >= 0;
    const int item = valid ? row_item[rid] : 0;
    const int y = row_y[rid];
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    float2* row = lds + rid * L;

    if constexpr ((MODE & kShearInv) || (MODE & kShearEmit)) row_inverse<L, TPR>(row, lane, a.tw_row);
    if constexpr (MODE & kShearEmit) {
        if (valid) {
            const int64_t n = (int64_t)H * W;
            float2* o = a.slot >= 0 ? a.samples + (int64_t)a.chains * a.n_samples * pr.pix_off +
                                          ((int64_t)it.pair * a.n_samples + a.slot) * n
                                    : a.kappa_out + pr.pix_off;
            for (unsigned x = lane; x < (unsigned)L; x += TPR) o[(int64_t)y * W + x] = row[swz(x)];
        }
        return;
    }
    if constexpr (!(MODE & kShearFwd)) {
        if (valid)
            for (unsigned x = lane; x < (unsigned)L; x += TPR) a.field[it.field_off + (int64_t)y * W + x] = row[swz(x)];
        return;
    }
    // pixel step in shear space: t = (1 - a) s + a gamma (+ sqrt(T (1 - a)) xi)
    const float T = a.lambda * pr.tau;
    for (unsigned pp = lane; pp < (unsigned)L / 2; pp += TPR) {
        const unsigned x = 2 * pp;
        const int64_t px = pr.pix_off + (int64_t)y * W + x;
        const float2 nb = *reinterpret_cast<const float2*>(a.nbar + px);
        const float4 g = *reinterpret_cast<const float4*>(a.gamma + px);
        const float a0 = T * __builtin_amdgcn_rcpf(T + nb.x), a1 = T * __builtin_amdgcn_rcpf(T + nb.y);
        const float2 g0 = a0 > 0.f ? make_float2(a0 * g.x, a0 * g.y) : make_float2(0.f, 0.f);
        const float2 g1 = a1 > 0.f ? make_float2(a1 * g.z, a1 * g.w) : make_float2(0.f, 0.f);
        float2 s0 = row[swz(x)], s1 = row[swz(x + 1)];
        s0 = make_float2(fmaf(1.f - a0, s0.x, g0.x), fmaf(1.f - a0, s0.y, g0.y));
        s1 = make_float2(fmaf(1.f - a1, s1.x, g1.x), fmaf(1.f - a1, s1.y, g1.y));
        if (a.stochastic && valid) {
            const uint32_t j2 = (uint32_t)(((int64_t)y * W + x) >> 1);
            const Normals2 z = pair_normals(j2, a.sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)it.pair, a.key0, a.key1);
            const float sg0 = __builtin_amdgcn_sqrtf(fmaxf(T * (1.f - a0), 0.f));
            const float sg1 = __builtin_amdgcn_sqrtf(fmaxf(T * (1.f - a1), 0.f));
            s0 = make_float2(fmaf(sg0, z.a.x, s0.x), fmaf(sg0, z.a.y, s0.y));
            s1 = make_float2(fmaf(sg1, z.b.x, s1.x), fmaf(sg1, z.b.y, s1.y));
        }
        row[swz(x)] = s0;
        row[swz(x + 1)] = s1;
    }
    __syncthreads();
    row_forward<L, TPR>(row, opaque(lane), opaque(a.tw_row));
    if (valid)
        for (unsigned x = lane; x < (unsigned)L; x += TPR) a.field[it.field_off + (int64_t)y * W + x] = row[swz(x)];
}

// Middle sweeps' row step for rows of 256 and more, arranged as the sampler's
// row_kernel_f: the first inverse pass reads the row from HBM, the last
// inverse pass, the shear-space pixel step and the first forward pass run in
// registers (pixel pairs split across neighbouring lanes, normals swapped with
// DPP), and the last forward pass writes the row to HBM.
template <int L>
__global__ __launch_bounds__(kRowThreads) void shear_row_kernel_f(ShearStreamArgs a, int H) {
    constexpr int ROWS = ShearRowShape<L>::ROWS, TPR = ShearRowShape<L>::TPR;
    constexpr int W = L;
    constexpr int RL = last_radix<L>();
    constexpr int NT16 = L / 16;
    constexpr int IT16 = (NT16 + TPR - 1) / TPR;
    constexpr int NTL = L / RL;
    constexpr int ITL = NTL / TPR;
    static_assert(L >= 256 && NTL % TPR == 0 && RL % 2 == 0, "shear_row_kernel_f shape");
    // padded LDS layouts, as in the sampler's fused row kernel
    constexpr int RM = middle_radix<L>();
    constexpr int A1 = pad_of(L, 16, 1), AC = pad_after(L, RM, 16, RL, A1);
    constexpr int AF = pad_of(L, RL, 1), AD = pad_after(L, RM, RL, 16, AF);
    constexpr int AMAX = pad_max(L, RM, 16, RL, A1) > pad_max(L, RM, RL, 16, AF) ? pad_max(L, RM, 16, RL, A1)
                                                                                 : pad_max(L, RM, RL, 16, AF);
    constexpr int LP = pad_len(L, AMAX);  // row stride in LDS
    __shared__ float2 lds[ROWS * LP];
    __shared__ int32_t row_item[ROWS], row_y[ROWS];
    const unsigned tid = threadIdx.x;
    const int64_t total_rows = (int64_t)a.n_items * H;
    const int64_t grow0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * ROWS;
    for (unsigned r = tid; r < (unsigned)ROWS; r += kRowThreads) {
        const int64_t g = grow0 + r;
        row_item[r] = g < total_rows ? (int32_t)(g % a.n_items) : -1;
        row_y[r] = g < total_rows ? (int32_t)(g / a.n_items) : 0;
    }
    __syncthreads();
    const unsigned rid = tid / TPR, lane = tid % TPR;
    const bool valid = row_item[rid] >= 0;
    const int item = valid ? row_item[rid] : 0;
    const int y = row_y[rid];
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    float2* row = lds + rid * LP;
    float2* frow = a.field + it.field_off + (int64_t)y * W;

    // first inverse pass from HBM (a row past the end reads row 0 of item 0,
    // whose results are never stored)
#pragma unroll
    for (int i = 0; i < IT16; ++i) {
        const unsigned j = lane + i * TPR;
        if (NT16 % TPR == 0 || j < (unsigned)NT16) {
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = frow[j + r * NT16];
            dft<16, true>(v);
#pragma unroll
            for (int r = 0; r < 16; ++r) row[lpos_run<A1, 16>(j, r)] = v[r];
        }
    }
    __syncthreads();
    passes_before<L, RM, 16, RL, TPR, true, A1>(row, lane, a.tw_row);

    // last inverse pass, pixel step t = (1 - a) s + a gamma (+ sqrt(T (1 - a)) xi),
    // first forward pass
    {
        const float T = a.lambda * pr.tau;
        const bool odd = lane & 1u;
        float2 v[ITL][RL];
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPR;
#pragma unroll
            for (int r = 0; r < RL; ++r) v[i][r] = row[lpos_step<AC, NTL>(j, r)];
#pragma unroll
            for (int r = 1; r < RL; ++r) v[i][r] = cmulc(v[i][r], a.tw_row[r * j]);
            dft<RL, true>(v[i]);
            float2 z[RL];
#pragma unroll
            for (int r = 0; r < RL; ++r) z[r] = make_float2(0.f, 0.f);
            if (a.stochastic) {
#pragma unroll
                for (int h = 0; h < RL / 2; ++h) {
                    const int rr = odd ? h + RL / 2 : h;
                    const unsigned xe = (j & ~1u) + rr * NTL;
                    const uint32_t pj = (uint32_t)(((int64_t)y * W + xe) >> 1);
                    const Normals2 nz = pair_normals(pj, a.sweep, (uint32_t)pr.pid, kStagePixel,
                                                     (uint32_t)it.pair, a.key0, a.key1);
                    const float2 send = odd ? nz.a : nz.b;
                    const float2 recv = make_float2(swap_lanes(send.x), swap_lanes(send.y));
                    if (odd) {
                        z[h + RL / 2] = nz.b;
                        z[h] = recv;
                    } else {
                        z[h] = nz.a;
                        z[h + RL / 2] = recv;
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int64_t px = pr.pix_off + (int64_t)y * W + j + r * NTL;
                const float a0 = T * __builtin_amdgcn_rcpf(T + a.nbar[px]);
                const float2 g = a.gamma[px];
                const float2 g0 = a0 > 0.f ? make_float2(a0 * g.x, a0 * g.y) : make_float2(0.f, 0.f);
                float2 s0 = make_float2(fmaf(1.f - a0, v[i][r].x, g0.x), fmaf(1.f - a0, v[i][r].y, g0.y));
                if (a.stochastic && valid) {
                    const float sg0 = __builtin_amdgcn_sqrtf(fmaxf(T * (1.f - a0), 0.f));
                    s0 = make_float2(fmaf(sg0, z[r].x, s0.x), fmaf(sg0, z[r].y, s0.y));
                }
                v[i][r] = s0;
            }
            dft<RL, false>(v[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPR;
#pragma unroll
            for (int r = 0; r < RL; ++r) row[lpos_run<AF, RL>(j, r)] = v[i][r];
        }
        __syncthreads();
    }

    // middle forward passes, then the last one (NS = L/16) to HBM
    passes_before<L, RM, RL, 16, TPR, false, AF>(row, opaque(lane), opaque(a.tw_row));
    if (valid) {
        const unsigned lane2 = opaque(lane);
        const float2* tw = opaque(a.tw_row);
#pragma unroll
        for (int i = 0; i < IT16; ++i) {
            const unsigned j = lane2 + i * TPR;
            if (NT16 % TPR == 0 || j < (unsigned)NT16) {
                float2 v[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = row[lpos_step<AD, NT16>(j, r)];
#pragma unroll
                for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw[r * j]);
                dft<16, false>(v);
#pragma unroll
                for (int r = 0; r < 16; ++r) frow[j + r * NT16] = v[r];
            }
        }
    }
}

template <int L>
__global__ __launch_bounds__(ShearColShape<L>::NTH) void shear_col_kernel(ShearStreamArgs a, int W) {
    constexpr int TC = ShearColShape<L>::TC, NTH = ShearColShape<L>::NTH, TPC = ShearColShape<L>::TPC;
    // padded exchange layouts from 256 rows (the HBM-side passes) where they
    // keep the resident workgroups per CU, else the XOR swizzle; an emission
    // sweep's round trip starts and ends in the natural-order layout AN
    constexpr int kExtra = 8 * L;  // the twiddle table beside the tile
    constexpr bool kPad = L >= 256 && lds_keeps_blocks(TC * ShearColShape<L>::SEG * 8 + kExtra,
                                                       TC * PairLayout<L, TC>::SEG * 8 + kExtra);
    constexpr int A1 = kPad ? PairLayout<L, TC>::A1 : -1, AN = kPad ? PairLayout<L, TC>::AN : -1;
    constexpr int AD = kPad ? PairLayout<L, TC>::AD : -1;
    constexpr int SEG = kPad ? PairLayout<L, TC>::SEG : ShearColShape<L>::SEG;
    constexpr int H = L;
    constexpr int half = TC / 2;
    __shared__ float2 lds[TC * SEG];
    __shared__ float2 twl[L >= 256 ? L : 1];  // twiddles of the HBM-side passes
    const unsigned tid = threadIdx.x;
    // tile fastest: an XCD runs neighbouring tiles of one item together
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int item = (int)(t / (W / TC));
    const int j = (int)(t % (W / TC));
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    const float2* fin = a.field + it.field_off;

    auto col_of = [&](int s) { return pair_column(j, s, half, W); };
    const unsigned cid = tid / TPC, lane = tid % TPC;
    if constexpr (L >= 256) {
        // first forward pass straight from HBM (plan of mf_streamed_fft.hpp)
        for (unsigned i = tid; i < (unsigned)L; i += NTH) twl[i] = a.tw_col[i];
        col_first_forward<L, TC, NTH, SEG, A1>(lds, fin, W, tid, col_of);
        __syncthreads();
        col_forward_rest<L, TPC, A1>(lds + cid * SEG, lane, twl);
    } else {
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            lds[s * SEG + swz(y)] = fin[(int64_t)y * W + pair_column(j, s, half, W)];
        }
        __syncthreads();
        stockham_fft<L, 1, TPC, false>(lds + cid * SEG, lane, a.tw_col);
    }

    // E/B Fourier step of mode k (slot s, row ky) and its mirror -k (slot p,
    // row my), given n P(k) and the chain's harmonic normals at k and -k
    const float T = a.lambda * pr.tau;
    const float n = (float)H * (float)W;
    const float inv_n = 1.0f / n;
    const float* nP = a.nP + pr.pix_off;
    const uint32_t pid = (uint32_t)pr.pid, chain = (uint32_t)it.pair;
    auto update = [&](int s, int p, int ky, int my, bool self, float nPk, float2 hk, float2 hm) {
        const int ck = pair_column(j, s, half, W);
        float2& zk = lds[s * SEG + lpos<AN>(ky)];
        float2& zm = lds[p * SEG + lpos<AN>(my)];
        const float2 dk = ks(ky, ck, H, W), dm = ks_mirror(dk, ky, ck, H, W);
        const float2 uk = mulc(zk, dk), um = mulc(zm, dm);
        const Filt c = filt(nPk, a.b_ratio, T, inv_n, n, ky == 0 && ck == 0);
        float2 Sk = make_float2(fmaf(c.fp, uk.x, c.fm * um.x), fmaf(c.fp, uk.y, -c.fm * um.y));
        float2 Sm = make_float2(fmaf(c.fp, um.x, c.fm * uk.x), fmaf(c.fp, um.y, -c.fm * uk.y));
        if (a.stochastic) {
            Sk = make_float2(Sk.x + fmaf(c.wp, hk.x, c.wm * hm.x), Sk.y + fmaf(c.wp, hk.y, -c.wm * hm.y));
            Sm = make_float2(Sm.x + fmaf(c.wp, hm.x, c.wm * hk.x), Sm.y + fmaf(c.wp, hm.y, -c.wm * hk.y));
        }
        if (!a.emit) {  // next state D kappa^ at once (an emitting sweep stages kappa^ first)
            Sk = cmul(Sk, dk);
            Sm = cmul(Sm, dm);
        }
        zk = Sk;
        if (!self) zm = Sm;
    };
    if (j == 0 || H < NTH / 2) {
        // one job per mode pair {k, -k} (see col_pair_kernel): tile 0, whose
        // columns 0 and W/2 pair with themselves, and columns too short to
        // give every thread a row
        const int jobs = half * H + (j == 0 ? H / 2 + 1 : 0);
#pragma unroll 1
        for (int q = opaque(tid); q < jobs; q += NTH) {
            int s, ky;
            if (q < half * H) {
                s = q % half;
                ky = q / half;
                if (j == 0 && s == 0 && ky > H / 2) continue;
            } else {
                s = half;
                ky = q - half * H;
            }
            const bool self_col = j == 0 && (s == 0 || s == half);
            const int p = self_col ? s : s + half;
            const int my = (H - ky) & (H - 1);
            const bool self = self_col && my == ky;
            const int ck = pair_column(j, s, half, W), cm = pair_column(j, p, half, W);
            float2 hk{}, hm{};
            if (a.stochastic) {
                hk = mode_normal((uint32_t)(ky * W + ck), a.sweep, pid, chain, a.key0, a.key1);
                hm = self ? hk : mode_normal((uint32_t)(my * W + cm), a.sweep, pid, chain, a.key0, a.key1);
            }
            update(s, p, ky, my, self, nP[ky * W + ck], hk, hm);
        }
    } else {
        // one thread per row across the tile's columns and their
        // mirrors, each Philox call serving two modes (see col_pair_kernel);
        // n P from the column-pair table, contiguous across the lanes' rows
        const int c0 = j * half;
        const float2* npt = a.nPt + pr.pix_off / 2 + (int64_t)(c0 / 2) * H;
#pragma unroll 1
        for (int ky = opaque(tid); ky < H; ky += NTH) {
            const int my = (H - ky) & (H - 1);
            const uint32_t rk = (uint32_t)(ky * W), rm = (uint32_t)(my * W);
            float2 carry{};  // mirror normal of slot 2pp (.a of the pair holding W - c0 - 2pp)
            if (a.stochastic)
                carry = pair_normals((rm + (uint32_t)(W - c0)) >> 1, a.sweep, pid, kStageHarmonic, chain, a.key0,
                                     a.key1).a;
#pragma unroll 1
            for (int pp = 0; pp < half / 2; ++pp) {
                float2 d0{}, d1{}, m1{}, nx{};
                if (a.stochastic) {
                    const Normals2 zd = pair_normals((rk + (uint32_t)(c0 + 2 * pp)) >> 1, a.sweep, pid,
                                                     kStageHarmonic, chain, a.key0, a.key1);
                    const Normals2 zm = pair_normals((rm + (uint32_t)(W - c0 - 2 * pp - 2)) >> 1, a.sweep, pid,
                                                     kStageHarmonic, chain, a.key0, a.key1);
                    d0 = zd.a;
                    d1 = zd.b;
                    m1 = zm.b;
                    nx = zm.a;
                }
                const float2 np = npt[(int64_t)pp * H + ky];
                update(2 * pp, 2 * pp + half, ky, my, false, np.x, d0, carry);
                update(2 * pp + 1, 2 * pp + 1 + half, ky, my, false, np.y, d1, m1);
                carry = nx;
            }
        }
    }
    __syncthreads();
    if (a.emit) {
        // stage F_col^-1(kappa^) for the emission kernel, then transform back
        // (the unnormalised round trip returns H kappa^) and take D kappa^
        stockham_fft<L, 1, TPC, true, AN, AN>(lds + opaque(cid) * SEG, opaque(lane), opaque(a.tw_col));
        float2* kout = a.kfield + it.field_off;
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            kout[(int64_t)y * W + pair_column(j, s, half, W)] = lds[s * SEG + lpos<AN>(y)];
        }
        stockham_fft<L, 1, TPC, false, AN, AN>(lds + opaque(cid) * SEG, opaque(lane), opaque(a.tw_col));
        const float back = 1.0f / (float)H;
        for (unsigned e = opaque(tid); e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            float2& v = lds[s * SEG + lpos<AN>(y)];
            v = cmul(v, cscale(ks(y, pair_column(j, s, half, W), H, W), back));
        }
        __syncthreads();
    }
    float2* fout = a.field + it.field_off;
    if constexpr (L >= 256) {
        // inverse transform, its last pass straight to HBM
        col_inverse_head<L, TPC, AN>(lds + opaque(cid) * SEG, opaque(lane), twl + opaque(0u));
        col_last_inverse<L, TC, NTH, SEG, AD>(lds, fout, W, opaque(tid), twl + opaque(0u), col_of);
    } else {
        stockham_fft<L, 1, TPC, true>(lds + opaque(cid) * SEG, opaque(lane), opaque(a.tw_col));
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const int s = (int)(e % TC), y = (int)(e / TC);
            fout[(int64_t)y * W + pair_column(j, s, half, W)] = lds[s * SEG + swz(y)];
        }
    }
}

__global__ void shear_init_kernel(ShearStreamArgs a, int64_t n, const float2* state_in) {
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = a.items[e / n].field_off + e % n;
        a.field[o] = state_in ? state_in[o] : make_float2(0.f, 0.f);
    }
}

}  // namespace

hipError_t launch_shear_row(int W, int H, int mode, const ShearStreamArgs& a, hipStream_t s) {
    const int64_t rows = (int64_t)a.n_items * H;
    switch (W) {
#define MF_CASE(LL)                                                                                          \
    case LL: {                                                                                               \
        const dim3 grid((unsigned)((rows + ShearRowShape<LL>::ROWS - 1) / ShearRowShape<LL>::ROWS));         \
        if (mode == kShearFwd) hipLaunchKernelGGL((shear_row_kernel<LL, kShearFwd>), grid, dim3(kRowThreads), 0, s, a, H); \
        else if (mode == kShearInvFwd && LL >= 256)                                                          \
            hipLaunchKernelGGL((shear_row_kernel_f<(LL >= 256 ? LL : 256)>), grid, dim3(kRowThreads), 0, s, a, H); \
        else if (mode == kShearInvFwd)                                                                       \
            hipLaunchKernelGGL((shear_row_kernel<LL, kShearInvFwd>), grid, dim3(kRowThreads), 0, s, a, H);   \
        else if (mode == kShearInv) hipLaunchKernelGGL((shear_row_kernel<LL, kShearInv>), grid, dim3(kRowThreads), 0, s, a, H); \
        else if (mode == kShearEmit) hipLaunchKernelGGL((shear_row_kernel<LL, kShearEmit>), grid, dim3(kRowThreads), 0, s, a, H); \
        else return hipErrorInvalidValue;                                                                    \
        break;                                                                                               \
    }
        MF_CASE(16) MF_CASE(32) MF_CASE(64) MF_CASE(128) MF_CASE(256) MF_CASE(512) MF_CASE(1024) MF_CASE(2048)
#undef MF_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_shear_col(int W, int H, const ShearStreamArgs& a, hipStream_t s) {
    switch (H) {
#define MF_CASE(LL)                                                                                              \
    case LL:                                                                                                     \
        if (W < ShearColShape<LL>::TC || !a.nPt) return hipErrorInvalidValue;                                    \
        hipLaunchKernelGGL(shear_col_kernel<LL>, dim3((unsigned)((int64_t)a.n_items * (W / ShearColShape<LL>::TC))), \
                           dim3(ShearColShape<LL>::NTH), 0, s, a, W);                                            \
        break;
        MF_CASE(16) MF_CASE(32) MF_CASE(64) MF_CASE(128) MF_CASE(256) MF_CASE(512) MF_CASE(1024) MF_CASE(2048)
#undef MF_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_shear_init(int W, int H, const ShearStreamArgs& a, const float2* state_in, hipStream_t s) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(shear_init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, n, state_in);
    return hipGetLastError();
}

}  // namespace mf
