// Streamed form of the messenger sweep: the complex field of every work item
// stays in HBM between two kernels per sweep.
//
//   row kernel:    [inverse row FFT -> emit sample] -> pixel-space draw of t
//                  (Algorithm 1, first two lines) -> forward row FFT
//   column kernel: forward column FFT -> Fourier-space draw of s (lines 4-5)
//                  -> inverse column FFT
//
// Each 1D transform is a Stockham FFT staged in LDS.  Rows (columns) of all
// work items of one launch are flattened, so small images still fill a block.
// Floating-point contraction only within a source expression: the fused and
// the plain row kernels then round every butterfly alike (with contraction
// across inlined calls, whether a product meets its sum in one basic block,
// and so becomes an FMA, depends on the kernel), and a run split into several
// calls reproduces the uninterrupted run bit for bit.
#pragma clang fp contract(on)
#include <type_traits>

#include "mf_device.hpp"
#include "mf_kernels.hpp"
#include "mf_streamed_fft.hpp"

namespace mf {

namespace {

constexpr int kThreads = 256;

// Fresh copies of a lane index / table pointer: the forward and inverse
// transforms use the same LDS addresses and twiddles, and without this the
// compiler keeps them all live from one transform to the other.
__device__ __forceinline__ unsigned fresh(unsigned v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ const float2* fresh(const float2* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Work-field elements: FP32 pairs, or FP16 / BF16 pairs (4 bytes) when the
// sampler stores the field in reduced precision.  Arithmetic is FP32: loads
// widen, stores round to nearest even (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32).
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 widen(float2 e) { return e; }
__device__ __forceinline__ float2 widen(f16x2 e) { return make_float2((float)e.x, (float)e.y); }
__device__ __forceinline__ float2 widen(bf16x2 e) { return make_float2((float)e.x, (float)e.y); }
__device__ __forceinline__ void narrow_to(float2& e, float2 v) { e = v; }
__device__ __forceinline__ void narrow_to(f16x2& e, float2 v) {
    e.x = (_Float16)v.x;
    e.y = (_Float16)v.y;
}
__device__ __forceinline__ void narrow_to(bf16x2& e, float2 v) {
    e.x = (__bf16)v.x;
    e.y = (__bf16)v.y;
}
template <typename E>
__device__ __forceinline__ E narrow(float2 v) {
    E e;
    narrow_to(e, v);
    return e;
}

// Runs fn with a value of the field's element type (the storage flag is
// uniform, so this is one scalar branch around the whole access loop).
template <typename Fn>
__device__ __forceinline__ void with_storage(int32_t st, Fn&& fn) {
    if (st == kStoreF16) fn(f16x2{});
    else if (st == kStoreBF16) fn(bf16x2{});
    else fn(float2{});
}

__device__ __forceinline__ float pix_a(float T, float nb) {
    // a = T / (T + Nbar); Nbar = +inf on missing pixels gives a = 0
    return T * __builtin_amdgcn_rcpf(T + nb);
}

// Sample emission of one row segment value at pixel x: both chains of a
// pair, or, packed, chain 0 of each of the two problems.
struct RowEmit {
    float* o0;
    float* o1;
    __device__ __forceinline__ void put(unsigned x, float2 s) const {
        if (o0) o0[x] = s.x;
        if (o1) o1[x] = s.y;
    }
};
__device__ __forceinline__ RowEmit row_emit(const SweepArgs& a, const ItemDev& it, int y, int W) {
    RowEmit e{nullptr, nullptr};
    if (a.packed) {
        const ProbDev pa = a.probs[it.prob];
        const int64_t na = (int64_t)pa.H * pa.W;
        e.o0 = a.samples + (int64_t)a.n_samples * pa.pix_off + (int64_t)a.emit_index * na + (int64_t)y * W;
        if (it.pair >= 0) {
            const ProbDev pb = a.probs[it.pair];
            e.o1 = a.samples + (int64_t)a.n_samples * pb.pix_off + (int64_t)a.emit_index * na + (int64_t)y * W;
        }
        return e;
    }
    const ProbDev pr = a.probs[it.prob];
    const int64_t base = (int64_t)a.chains * a.n_samples * pr.pix_off;
    const int64_t n = (int64_t)pr.H * pr.W;
    const int c0 = 2 * it.pair, c1 = 2 * it.pair + 1;
    e.o0 = a.samples + base + ((int64_t)c0 * a.n_samples + a.emit_index) * n + (int64_t)y * W;
    if (c1 < a.chains) e.o1 = a.samples + base + ((int64_t)c1 * a.n_samples + a.emit_index) * n + (int64_t)y * W;
    return e;
}

// The second problem of a packed item (its own one when the item has no partner).
__device__ __forceinline__ ProbDev partner_of(const SweepArgs& a, const ItemDev& it, const ProbDev& pr) {
    return it.pair >= 0 ? a.probs[it.pair] : pr;
}

// Rows per block of the fused row kernel: twice row_kernel's at 512 pixels
// (every lane busy in the radix-16 passes: the uneven batch's 512^2 row launch
// 14% faster), the same elsewhere (twice as many rows ran the uneven batch's
// 256^2 rows 5%, 1024^2 8% and 2048^2 4% slower).
// The autotuner may pick another of the shapes of fused_row_candidates.
template <int L>
struct RowShapeF {
    static constexpr int ROWS = L == 512 ? 8 : 2048 / L;
    static constexpr int TPR = kThreads / ROWS;
};

constexpr int pow2_floor(int v) {
    int q = 1;
    while (2 * q <= v) q *= 2;
    return q;
}
// Rows per block of the plain row kernels: a power of two, about 2048 pixels.
constexpr int rows_per_block(int L) { return L >= 2048 ? 1 : pow2_floor(2048 / L); }

template <int L>
struct RowShape {
    static constexpr int ROWS = rows_per_block(L);  // rows per block
    static constexpr int TPR = kThreads / ROWS;     // threads per row
    static constexpr int LS = lds_stride<L>();      // LDS row stride
    static constexpr int NE = ROWS * L;             // pixels per block
    static constexpr int NL = (NE + kThreads - 1) / kThreads;  // load / store iterations
};

// Rows of all work items are enumerated with the item index fastest,
// g = y * n_items + item, so that the rows one block (and one XCD) handles
// share the rows of the problem tables; with one item per problem
// (rows_by_item) they run y fastest within each item instead, so that a block
// and its neighbours stay inside one problem's rows and pages.
template <int L, int MODE>
__global__ __launch_bounds__(kThreads) void row_kernel(SweepArgs a, int H) {
    constexpr int ROWS = RowShape<L>::ROWS;
    constexpr int TPR = RowShape<L>::TPR;
    constexpr int LS = RowShape<L>::LS;
    constexpr int NE = RowShape<L>::NE;
    constexpr int W = L;
    __shared__ float2 lds[ROWS * LS];
    __shared__ double red[kThreads];

    // (item, row) of each of the block's rows, one division per row
    __shared__ int32_t row_item[ROWS], row_y[ROWS];

    const unsigned tid = threadIdx.x;
    const unsigned rid = tid / TPR;
    const unsigned lane = tid % TPR;
    const int64_t total_rows = (int64_t)a.n_items * H;
    const int64_t grow0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * ROWS;
    for (unsigned r = tid; r < (unsigned)ROWS; r += kThreads) {
        const int64_t g = grow0 + r;
        row_item[r] = g < total_rows ? (int32_t)(a.rows_by_item ? g / H : g % a.n_items) : -1;
        row_y[r] = g < total_rows ? (int32_t)(a.rows_by_item ? g % H : g / a.n_items) : 0;
    }
    __syncthreads();

    // ---- load ROWS rows (coalesced along x)
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        const E* fld = reinterpret_cast<const E*>(a.field);
#pragma unroll
        for (int i = 0; i < RowShape<L>::NL; ++i) {
            const unsigned e = tid + i * kThreads;
            if (NE % kThreads != 0 && e >= (unsigned)NE) break;
            const unsigned r = e / L, x = e % L;
            float2 v = make_float2(0.f, 0.f);
            if (row_item[r] >= 0) v = widen(fld[a.items[row_item[r]].field_off + (int64_t)row_y[r] * W + x]);
            lds[r * LS + swz(x)] = v;
        }
    });
    __syncthreads();

    const bool valid = row_item[rid] >= 0;
    const int item = valid ? row_item[rid] : 0;
    const int y = row_y[rid];
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    float2* row = lds + rid * LS;

    if constexpr (MODE & kRowInv) {
        row_inverse<L, TPR>(row, lane, a.tw_row);
        if (a.s_save && valid)
            for (unsigned x = lane; x < (unsigned)L; x += TPR)
                a.s_save[it.field_off + (int64_t)y * W + x] = row[swz(x)];
        if (a.emit_index >= 0 && valid) {
            const RowEmit em = row_emit(a, it, y, W);
            for (unsigned x = lane; x < (unsigned)L; x += TPR) em.put(x, row[swz(x)]);
        }
        if constexpr (!(MODE & kRowFwd)) {
            if (a.pix_mode == kPixAdjoint) {
                // transpose of the pixel step on the last reverse sweep
                const float T = a.lambda * pr.tau;
                for (unsigned x = lane; x < (unsigned)L; x += TPR) {
                    const int64_t pix = pr.pix_off + (int64_t)y * W + x;
                    const float aa = pix_a(T, a.nbar[pix]);
                    const float2 tb = row[swz(x)];
                    if (valid) a.grad_d[pix] += aa * tb.x;
                    row[swz(x)] = cscale(tb, 1.0f - aa);
                }
            }
            if (valid)
                with_storage(a.storage, [&](auto e0) {
                    using E = decltype(e0);
                    E* fld = reinterpret_cast<E*>(a.field) + it.field_off + (int64_t)y * W;
                    for (unsigned x = lane; x < (unsigned)L; x += TPR) fld[x] = narrow<E>(row[swz(x)]);
                });
            return;
        }
    }

    if constexpr (MODE & kRowFwd) {
        if (a.pix_mode == kPixAdjoint) {
            // transpose of the pixel step: grad_d += a t, t <- (1 - a) t
            const float T = a.lambda * pr.tau;
            for (unsigned x = lane; x < (unsigned)L; x += TPR) {
                const int64_t pix = pr.pix_off + (int64_t)y * W + x;
                const float aa = pix_a(T, a.nbar[pix]);
                const float2 tb = row[swz(x)];
                if (valid) a.grad_d[pix] += aa * tb.x;
                row[swz(x)] = cscale(tb, 1.0f - aa);
            }
            __syncthreads();
        } else if (a.pix_mode == kPixIdentity) {
            __syncthreads();
        } else {
            // ---- pixel-space messenger update t = (1 - a) s + src + sigma_t xi
            const float T = a.lambda * pr.tau;
            double acc = 0.0;
            if (a.packed) {
                // chain 0 of problem A (real part) and of problem B (imaginary
                // part), each with its own tables and stream (pair 0, words .x)
                const ProbDev pb = partner_of(a, it, pr);
                const float TB = a.lambda * pb.tau;
#pragma unroll 2
                for (unsigned pp = lane; pp < (unsigned)L / 2; pp += TPR) {
                    const unsigned x = 2 * pp;
                    const int64_t off = (int64_t)y * W + x;
                    const float2 na = *reinterpret_cast<const float2*>(a.nbar + pr.pix_off + off);
                    const float2 da = *reinterpret_cast<const float2*>(a.src + pr.pix_off + off);
                    const float2 nbb = *reinterpret_cast<const float2*>(a.nbar + pb.pix_off + off);
                    const float2 db = *reinterpret_cast<const float2*>(a.src + pb.pix_off + off);
                    const uint32_t j = (uint32_t)(off >> 1);
                    const Normals2 za = pair_normals(j, a.sweep, (uint32_t)pr.pid, kStagePixel, 0u, a.key0, a.key1);
                    const Normals2 zb = pair_normals(j, a.sweep, (uint32_t)pb.pid, kStagePixel, 0u, a.key0, a.key1);
                    const float aA[2] = {pix_a(T, na.x), pix_a(T, na.y)}, aB[2] = {pix_a(TB, nbb.x), pix_a(TB, nbb.y)};
                    const float dA[2] = {da.x, da.y}, dB[2] = {db.x, db.y};
                    const float zA[2] = {za.a.x, za.b.x}, zB[2] = {zb.a.x, zb.b.x};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        float2& sv = row[swz(x + q)];
                        const float omA = 1.0f - aA[q], omB = 1.0f - aB[q];
                        const float sA = aA[q] > 0.f ? aA[q] * dA[q] : 0.f, sB = aB[q] > 0.f ? aB[q] * dB[q] : 0.f;
                        const float gA = __builtin_amdgcn_sqrtf(fmaxf(T * omA, 0.f));
                        const float gB = __builtin_amdgcn_sqrtf(fmaxf(TB * omB, 0.f));
                        // an item without a partner keeps its imaginary part at zero
                        sv = make_float2(fmaf(omA, sv.x, fmaf(gA, zA[q], sA)),
                                         it.pair >= 0 ? fmaf(omB, sv.y, fmaf(gB, zB[q], sB)) : 0.f);
                    }
                }
            } else
#pragma unroll 2
            for (unsigned pp = lane; pp < (unsigned)L / 2; pp += TPR) {
                const unsigned x = 2 * pp;
                const int64_t pix = pr.pix_off + (int64_t)y * W + x;
                const float2 nb = *reinterpret_cast<const float2*>(a.nbar + pix);
                const float2 sv = *reinterpret_cast<const float2*>(a.src + pix);
                float aa[2] = {pix_a(T, nb.x), pix_a(T, nb.y)};
                float sr[2] = {sv.x, sv.y};
                float2 s[2] = {row[swz(x)], row[swz(x + 1)]};
                float2 z[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                if (a.stochastic && valid) {
                    const uint32_t j = (uint32_t)(((int64_t)y * W + x) >> 1);
                    const Normals2 nz = pair_normals(j, a.sweep, (uint32_t)pr.pid, kStagePixel, (uint32_t)it.pair,
                                                     a.key0, a.key1);
                    z[0] = nz.a;
                    z[1] = nz.b;
                }
                float2 t[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float oma = 1.0f - aa[q];
                    float src;
                    if (a.src_kind == kSrcData) src = aa[q] > 0.f ? aa[q] * sr[q] : 0.f;
                    else src = T * sr[q];
                    const float sig = a.stochastic ? __builtin_amdgcn_sqrtf(fmaxf(T * oma, 0.f)) : 0.f;
                    t[q].x = fmaf(oma, s[q].x, fmaf(sig, z[q].x, src));
                    t[q].y = a.real_only ? 0.f : fmaf(oma, s[q].y, fmaf(sig, z[q].y, src));
                }
                if (valid) {
                    const int64_t f = it.field_off + (int64_t)y * W + x;
                    if (a.check_t) {
                        const float2 p0 = a.t_save[f], p1 = a.t_save[f + 1];
                        const double d0 = (double)t[0].x - p0.x, d1 = (double)t[1].x - p1.x;
                        const double e0 = (double)t[0].y - p0.y, e1 = (double)t[1].y - p1.y;
                        acc += d0 * d0 + d1 * d1 + e0 * e0 + e1 * e1;
                    }
                    if (a.save_t) {
                        a.t_save[f] = t[0];
                        a.t_save[f + 1] = t[1];
                    }
                }
                row[swz(x)] = t[0];
                row[swz(x + 1)] = t[1];
            }
            if (a.check_t) {
                red[tid] = acc;
                __syncthreads();
                if (lane == 0 && valid) {
                    double s = 0.0;
                    for (int i = 0; i < TPR; ++i) s += red[rid * TPR + i];
                    a.partials[(int64_t)y * a.n_items + item] = s;
                }
            }
            __syncthreads();
        }
        row_forward<L, TPR>(row, fresh(lane), fresh(a.tw_row));
        if (valid)
            with_storage(a.storage, [&](auto e0) {
                using E = decltype(e0);
                E* fld = reinterpret_cast<E*>(a.field) + it.field_off + (int64_t)y * W;
                for (unsigned x = lane; x < (unsigned)L; x += TPR) fld[x] = narrow<E>(row[swz(x)]);
            });
    }
}


// Row kernel of a middle sweep (inverse row FFT, emission, pixel-space update,
// forward row FFT) for rows of 256 pixels and more, with half the LDS traffic
// and barriers of row_kernel:
//   A. the first inverse radix-16 pass reads the row from HBM into registers;
//   B. the middle inverse passes run in LDS;
//   C. the last inverse pass (radix RL) leaves pixels x = j + r L/RL in
//      registers, which are emitted, updated and fed to the first forward pass
//      (radix RL, the same pixels) without touching LDS.  A pixel pair
//      (x, x + 1) sits in neighbouring lanes: each lane draws half of the
//      pair's Philox calls and swaps the other half's normals with DPP;
//   D. the middle forward passes run in LDS and the last one writes the
//      natural-order row straight to HBM.
// The same arithmetic, pass for pass and pixel for pixel, as row_kernel with
// the plan of row_inverse / row_forward, so the two round identically.
// Variants of the fused row kernel: pixel tables read in stage C (wide
// launches, whose blocks hide the latency), read beside the field loads
// (launches too small to fill the GPU), or either kind of item, a.packed
// telling at run time whether each carries two single-chain problems (the
// packed launches: built with both paths it takes 100 VGPRs at 512 points,
// where a packed-only build took 130 and lost a wave per SIMD).
enum RowVariant : int { kRowLoadLate = 0, kRowPrefetch = 1, kRowAny = 2 };

// The 2048-point wide build asks for six waves per SIMD (77 VGPRs instead of
// 83, no spills), which keeps six blocks per CU.
template <int L, int ROWS_, int VAR>
__global__ __launch_bounds__(kThreads, (L == 2048 && ROWS_ == 1 && VAR == kRowLoadLate) ? 6 : 1)
void row_kernel_f(SweepArgs a, int H) {
    constexpr bool kPrefetch = VAR == kRowPrefetch;
    constexpr int ROWS = ROWS_;
    constexpr int TPR = kThreads / ROWS;
    constexpr int W = L;
    constexpr int RL = last_radix<L>();
    constexpr int NT16 = L / 16;                    // radix-16 butterflies per row
    constexpr int IT16 = (NT16 + TPR - 1) / TPR;
    constexpr int NTL = L / RL;                     // last-radix butterflies per row
    constexpr int ITL = NTL / TPR;
    static_assert(L >= 256 && NTL % TPR == 0 && RL % 2 == 0, "row_kernel_f shape");
    // padded LDS layouts: stage A writes A1, the middle inverse passes leave
    // AC, stage C writes AF, the middle forward passes leave AD
    constexpr int RM = middle_radix<L>();
    constexpr int A1 = pad_of(L, 16, 1), AC = pad_after(L, RM, 16, RL, A1);
    constexpr int AF = pad_of(L, RL, 1), AD = pad_after(L, RM, RL, 16, AF);
    constexpr int AMAX = pad_max(L, RM, 16, RL, A1) > pad_max(L, RM, RL, 16, AF) ? pad_max(L, RM, 16, RL, A1)
                                                                                 : pad_max(L, RM, RL, 16, AF);
    constexpr int LP = pad_len(L, AMAX);  // row stride in LDS
    __shared__ float2 lds[ROWS * LP];
    // twiddles in LDS up to 1024 points (1024^2 -8%, 512^2 -6%, 256^2 -5% per
    // sweep); at 2048 the extra 16 KiB would cost a resident block (+3%)
    constexpr bool kTwLds = L <= 1024;
    __shared__ float2 twl[kTwLds ? L : 1];
    static_assert(ROWS * LP >= kThreads, "residual partials fit in the rows");
    double* red = reinterpret_cast<double*>(lds);  // residual partials, once stage C has read the rows
    __shared__ int32_t row_item[ROWS], row_y[ROWS];

    const unsigned tid = threadIdx.x;
    const unsigned rid = tid / TPR;
    const unsigned lane = tid % TPR;
    const int64_t total_rows = (int64_t)a.n_items * H;
    const int64_t grow0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * ROWS;
    for (unsigned r = tid; r < (unsigned)ROWS; r += kThreads) {
        const int64_t g = grow0 + r;
        row_item[r] = g < total_rows ? (int32_t)(a.rows_by_item ? g / H : g % a.n_items) : -1;
        row_y[r] = g < total_rows ? (int32_t)(a.rows_by_item ? g % H : g / a.n_items) : 0;
    }
    __syncthreads();
    const bool valid = row_item[rid] >= 0;
    const int item = valid ? row_item[rid] : 0;
    const int y = row_y[rid];
    // One record read before the field: the item carries its problem's
    // offset, tau and index.  The twiddle loads go out beside it (the table
    // is visible after stage A's barrier); with kPrefetch the pixel tables of
    // stage C go out beside the field loads, so that a block waits for memory
    // twice before it computes.
    const ItemDev it = a.items[item];
    const float2* twr;
    if constexpr (kTwLds) {
        for (unsigned i = tid; i < (unsigned)L; i += kThreads) twl[i] = a.tw_row[i];
        twr = twl;
    } else {
        twr = a.tw_row;
    }
    const ProbDev pr{H, W, it.pix_off, it.tau, it.pid};
    float2* row = lds + rid * LP;
    const int64_t frow = it.field_off + (int64_t)y * W;
    float pnb[kPrefetch ? ITL : 1][kPrefetch ? RL : 1], psr[kPrefetch ? ITL : 1][kPrefetch ? RL : 1];
    if constexpr (kPrefetch) {
        const int64_t prow = pr.pix_off + (int64_t)y * W;
#pragma unroll
        for (int i = 0; i < ITL; ++i)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const unsigned x = lane + i * TPR + r * NTL;
                pnb[i][r] = a.nbar[prow + x];
                psr[i][r] = a.src[prow + x];
            }
    }

    // ---- A: first inverse pass (NS = 1), inputs from HBM
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        const E* fld = reinterpret_cast<const E*>(a.field) + frow;
        float2 v[IT16][16];
#pragma unroll
        for (int i = 0; i < IT16; ++i) {
            const unsigned j = lane + i * TPR;
            if (NT16 % TPR == 0 || j < (unsigned)NT16) {
                // unconditional loads (a row past the end reads row 0 of item 0,
                // whose results are never stored), so that all 16 are in flight
                // at once instead of each behind its own branch
#pragma unroll
                for (int r = 0; r < 16; ++r) v[i][r] = widen(fld[j + r * NT16]);
                dft<16, true>(v[i]);
#pragma unroll
                for (int r = 0; r < 16; ++r) row[lpos_run<A1, 16>(j, r)] = v[i][r];
            }
        }
    });
    __syncthreads();

    // ---- B: middle inverse passes
    passes_before<L, RM, 16, RL, TPR, true, A1>(row, lane, twr);

    // ---- C: last inverse pass, emission, pixel update, first forward pass
    {
        const float T = a.lambda * pr.tau;
        const bool odd = lane & 1u;
        double acc = 0.0;
        float2 v[ITL][RL];
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPR;
#pragma unroll
            for (int r = 0; r < RL; ++r) v[i][r] = row[lpos_step<AC, NTL>(j, r)];
#pragma unroll
            for (int r = 1; r < RL; ++r) v[i][r] = cmulc(v[i][r], twr[r * j]);
            dft<RL, true>(v[i]);
            // v[i][r] is now the state at pixel x = j + r NTL
            if (a.emit_index >= 0 && valid) {
                const RowEmit em = row_emit(a, it, y, W);
#pragma unroll
                for (int r = 0; r < RL; ++r) em.put(j + r * NTL, v[i][r]);
            }
            if (VAR == kRowAny && a.packed) {
                // two single-chain problems: for each pixel pair the even lane
                // draws problem A's normals, the odd lane problem B's, and each
                // passes the other the word of the other pixel
                const ProbDev pb = partner_of(a, it, pr);
                const float TB = a.lambda * pb.tau;
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const unsigned x = j + r * NTL;
                    const int64_t off = (int64_t)y * W + x;
                    const uint32_t pj = (uint32_t)(off >> 1);
                    const Normals2 nz = pair_normals(pj, a.sweep, (uint32_t)(odd ? pb.pid : pr.pid), kStagePixel, 0u,
                                                     a.key0, a.key1);
                    // even lane (pixel 2pj): keeps A's .a, sends A's .b; odd lane (pixel 2pj+1): keeps B's .b, sends B's .a
                    const float keep = odd ? nz.b.x : nz.a.x;
                    const float recv = swap_lanes(odd ? nz.a.x : nz.b.x);
                    const float zA = odd ? recv : keep, zB = odd ? keep : recv;
                    const float aA = pix_a(T, a.nbar[pr.pix_off + off]), aB = pix_a(TB, a.nbar[pb.pix_off + off]);
                    const float dA = a.src[pr.pix_off + off], dB = a.src[pb.pix_off + off];
                    const float omA = 1.0f - aA, omB = 1.0f - aB;
                    const float sA = aA > 0.f ? aA * dA : 0.f, sB = aB > 0.f ? aB * dB : 0.f;
                    const float gA = __builtin_amdgcn_sqrtf(fmaxf(T * omA, 0.f));
                    const float gB = __builtin_amdgcn_sqrtf(fmaxf(TB * omB, 0.f));
                    // an item without a partner keeps its imaginary part at zero
                    v[i][r] = make_float2(fmaf(omA, v[i][r].x, fmaf(gA, zA, sA)),
                                          it.pair >= 0 ? fmaf(omB, v[i][r].y, fmaf(gB, zB, sB)) : 0.f);
                }
                dft<RL, false>(v[i]);
                continue;
            }
            // normals: the even lane draws the pairs of r < RL/2, the odd lane
            // those of r >= RL/2; each passes its partner the half it needs
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
                const unsigned x = j + r * NTL;
                float nb, sr;
                if constexpr (kPrefetch) {
                    nb = pnb[i][r];
                    sr = psr[i][r];
                } else {
                    const int64_t pix = pr.pix_off + (int64_t)y * W + x;
                    nb = a.nbar[pix];
                    sr = a.src[pix];
                }
                const float aa = pix_a(T, nb);
                const float oma = 1.0f - aa;
                float src;
                if (a.src_kind == kSrcData) src = aa > 0.f ? aa * sr : 0.f;
                else src = T * sr;
                const float sig = a.stochastic ? __builtin_amdgcn_sqrtf(fmaxf(T * oma, 0.f)) : 0.f;
                float2 t;
                t.x = fmaf(oma, v[i][r].x, fmaf(sig, z[r].x, src));
                t.y = a.real_only ? 0.f : fmaf(oma, v[i][r].y, fmaf(sig, z[r].y, src));
                if (valid) {
                    const int64_t f = frow + x;
                    if (a.check_t) {
                        const float2 p0 = a.t_save[f];
                        const double d0 = (double)t.x - p0.x, e0 = (double)t.y - p0.y;
                        acc += d0 * d0 + e0 * e0;
                    }
                    if (a.save_t) a.t_save[f] = t;
                }
                v[i][r] = t;
            }
            dft<RL, false>(v[i]);
        }
        if (a.check_t) {
            __syncthreads();  // every thread has read its row
            red[tid] = acc;
            __syncthreads();
            if (lane == 0 && valid) {
                double sum = 0.0;
                for (int k = 0; k < TPR; ++k) sum += red[rid * TPR + k];
                a.partials[(int64_t)y * a.n_items + item] = sum;
            }
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

    // ---- D: middle forward passes, then the last one (NS = L/16) to HBM
    passes_before<L, RM, RL, 16, TPR, false, AF>(row, fresh(lane), twr + fresh(0u));
    if (valid)
        with_storage(a.storage, [&](auto e0) {
            using E = decltype(e0);
            E* fld = reinterpret_cast<E*>(a.field) + frow;
            const unsigned lane2 = fresh(lane);
            const float2* tw = twr + fresh(0u);
            float2 v[IT16][16];
#pragma unroll
            for (int i = 0; i < IT16; ++i) {
                const unsigned j = lane2 + i * TPR;
                if (NT16 % TPR == 0 || j < (unsigned)NT16) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) v[i][r] = row[lpos_step<AD, NT16>(j, r)];
#pragma unroll
                    for (int r = 1; r < 16; ++r) v[i][r] = cmul(v[i][r], tw[r * j]);
                    dft<16, false>(v[i]);
#pragma unroll
                    for (int r = 0; r < 16; ++r) fld[j + r * NT16] = narrow<E>(v[i][r]);
                }
            }
        });
}

// Column tiles: TC columns of one item per block of NTH threads; each column
// is its own LDS segment of L + 32/TC elements (the tile load then hits
// distinct banks).  The default shape fills at most ~128 KiB of LDS; the
// autotuner may pick another feasible (TC, NTH).
// Default tile of a column length (16 columns, 8 from 1025 rows so that the
// tile fits in LDS) and its threads.
constexpr int col_tc_of(int L) { return L > 1024 ? 8 : 16; }
constexpr int col_nth_of(int L) { return L >= 1024 ? 1024 : (L >= 512 ? 512 : 256); }

template <int L>
struct ColShape {
    static constexpr int TC = col_tc_of(L);
    static constexpr int NTH = col_nth_of(L);
    static constexpr int TPC = NTH / TC;
    static constexpr int SEG = lds_stride<L>() + 32 / TC;
};

// Column tiles of an item: W / TC, or one more ragged tile when TC does not
// divide W (sides 2^a 3^b); a ragged tile's missing columns are transformed
// as zeros and never stored.
__device__ __forceinline__ int tiles_per_item(int W, int tc) { return (W + tc - 1) / tc; }

template <int L, int TC_, int NTH_>
__global__ __launch_bounds__(NTH_) void col_kernel_t(SweepArgs a, int W) {
    constexpr int TC = TC_;
    constexpr int NTH = NTH_;
    constexpr int TPC = NTH / TC;
    constexpr int SEG = lds_stride<L>() + 32 / TC;
    constexpr int H = L;
    __shared__ float2 lds[TC * SEG];
    // twiddles in LDS, or in L2 for 4-column tiles of 2048 rows (as in col_kernel_f; identical values)
    constexpr bool kTwLds = !col_tw_in_l2(L, TC);
    __shared__ float2 twl[kTwLds ? L : 1];
    const float2* twp = kTwLds ? twl : a.tw_col;
    const unsigned tid = threadIdx.x;
    // tiles enumerated with the tile fastest: t = item * tiles + tile.  An
    // XCD then runs neighbouring tiles of one item together, and the cache
    // lines they share (a 128-byte line spans 16 columns) meet in its L2.
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int tpi = tiles_per_item(W, TC);
    const int item = (int)(t / tpi);
    const int x0 = (int)(t % tpi) * TC;
    const unsigned ncol = (unsigned)min(TC, W - x0);  // columns of this tile
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    const int64_t f0 = it.field_off + x0;

    if constexpr (kTwLds)
        for (unsigned i = tid; i < (unsigned)L; i += NTH) twl[i] = a.tw_col[i];  // visible after the tile barrier
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        const E* fld = reinterpret_cast<const E*>(a.field) + f0;
#pragma unroll 4
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const unsigned c = e % TC, y = e / TC;
            lds[c * SEG + swz(y)] = c < ncol ? widen(fld[(int64_t)y * W + c]) : make_float2(0.f, 0.f);
        }
    });
    __syncthreads();
    const unsigned cid = tid / TPC, lane = tid % TPC;
    stockham_fft<L, 1, TPC, false>(lds + cid * SEG, lane, twp);

    const float T = a.lambda * pr.tau;
    if (a.t_store) {
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const unsigned c = e % TC, y = e / TC;
            if (c < ncol) a.t_store[it.field_off + (int64_t)y * W + x0 + c] = lds[c * SEG + swz(y)];
        }
    }
    if (a.t_load) {
        // band sums of Re(conj(F sbar) F t) T/(nP + T)^2: the derivative of a
        // sweep's Fourier filter f = nP/(nP + T) with respect to a band amplitude
        __shared__ double bacc[kMaxBandsPerProblem];
        for (unsigned b = tid; b < (unsigned)kMaxBandsPerProblem; b += NTH) bacc[b] = 0.0;
        __syncthreads();
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const unsigned c = e % TC, y = e / TC;
            if (c >= ncol) continue;
            const int64_t mode = (int64_t)y * W + x0 + c;
            const int b = a.band[pr.pix_off + mode];
            if (b < 0) continue;
            const float2 v = lds[c * SEG + swz(y)];
            const float2 tt = a.t_load[it.field_off + mode];
            const double P = a.nP[pr.pix_off + mode];
            const double den = P + (double)T;
            atomicAdd(&bacc[b], ((double)v.x * tt.x + (double)v.y * tt.y) * (double)T / (den * den));
        }
        __syncthreads();
        for (unsigned b = tid; b < (unsigned)kMaxBandsPerProblem; b += NTH)
            a.band_slots[t * kMaxBandsPerProblem + b] += bacc[b];
        __syncthreads();
    }

    // ---- Fourier-space update S = f T / n + w eta / n on column pairs
    const float inv_n = 1.0f / ((float)H * (float)W);
#pragma unroll 1
    for (unsigned e = tid; e < (unsigned)((TC / 2) * L); e += NTH) {
        const unsigned j = e % (TC / 2), ky = e / (TC / 2);
        if (2 * j >= ncol) continue;  // W is even, so column pairs are whole
        const int kx = x0 + 2 * j;
        const int64_t mode = (int64_t)ky * W + kx;
        const float2 np = *reinterpret_cast<const float2*>(a.nP + pr.pix_off + mode);
        float2 z[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        if (a.stochastic) {
            const Normals2 nz = pair_normals((uint32_t)(mode >> 1), a.sweep, (uint32_t)pr.pid, kStageHarmonic,
                                             (uint32_t)it.pair, a.key0, a.key1);
            z[0] = nz.a;
            z[1] = nz.b;
        }
        const float npv[2] = {np.x, np.y};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float P = npv[q];
            const float rden = __builtin_amdgcn_rcpf(P + T);
            const float f = P * rden * inv_n;
            float2& v = lds[(2 * j + q) * SEG + swz(ky)];
            float2 o = cscale(v, f);
            if (a.stochastic) {
                const float w = __builtin_amdgcn_sqrtf(P * T * rden * inv_n);
                o.x = fmaf(w, z[q].x, o.x);
                o.y = fmaf(w, z[q].y, o.y);
            }
            v = o;
        }
    }
    __syncthreads();
    stockham_fft<L, 1, TPC, true>(lds + fresh(cid) * SEG, fresh(lane), twp + fresh(0u));

    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        E* fld = reinterpret_cast<E*>(a.field) + f0;
#pragma unroll 4
        for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH) {
            const unsigned c = e % TC, y = e / TC;
            if (c < ncol) fld[(int64_t)y * W + c] = narrow<E>(lds[c * SEG + swz(y)]);
        }
    });
}

// Column kernel of the sampler and the Wiener iteration for H >= 256, with
// half the LDS traffic and barriers of col_kernel_t:
//   A. the first forward radix-16 pass reads its inputs from HBM into
//      registers (a wave covers TC columns of 64/TC rows, as the tile load
//      does) and writes its outputs to LDS;
//   B. the middle forward passes run in LDS;
//   C. the last forward pass, the Fourier-space update and the first inverse
//      pass run in registers, one thread owning the same rows of a column
//      pair (2p, 2p+1), so one Philox call serves both modes of a pair and
//      the column-pair table nPt gives both coefficients in one coalesced load;
//   D. the middle inverse passes run in LDS and the last one writes its
//      outputs, in natural order, straight to HBM.
// The twiddle table sits in LDS beside the tile (16 KiB at 2048 rows): with
// one or two workgroups per CU every wave waits for the same twiddles, and an
// LDS read returns much sooner than an L2 hit (2048^2 sweep -6%, 1024^2 -10%).
// Same arithmetic per mode as col_kernel_t, with the plan of the row kernels
// (forward 16, RM..., RL; inverse RL, RM..., 16).  Every sweep of a run takes
// the same column kernel, so split runs still repeat uninterrupted ones.
template <int L, int TC_, int NTH_>
__global__ __launch_bounds__(NTH_) void col_kernel_f(SweepArgs a, int W) {
    constexpr int TC = TC_;
    constexpr int NTH = NTH_;
    constexpr int TPC = NTH / TC;
    constexpr int H = L;
    constexpr int RL = last_radix<L>();
    // padded layouts (as in the fused row kernel) where they keep the
    // resident workgroups per CU, else the XOR swizzle: phase A writes A1,
    // the middle forward passes leave AC, phase C writes AF, the middle
    // inverse passes leave AD; the slot stride keeps phases A and D free of
    // conflicts
    constexpr int RM = middle_radix<L>();
    constexpr int P1 = pad_of(L, 16, 1), PF = pad_of(L, RL, 1);
    constexpr int PMAX = pad_max(L, RM, 16, RL, P1) > pad_max(L, RM, RL, 16, PF) ? pad_max(L, RM, 16, RL, P1)
                                                                                 : pad_max(L, RM, RL, 16, PF);
    constexpr int PSEG = tile_seg(TC, P1, pad_after(L, RM, RL, 16, PF), pad_len(L, PMAX));
    constexpr int kExtra = col_tw_in_l2(L, TC) ? 0 : 8 * L;
    constexpr bool kPad = lds_keeps_blocks(TC * (L + 32 / TC) * 8 + kExtra, TC * PSEG * 8 + kExtra);
    constexpr int A1 = kPad ? P1 : -1, AC = pad_after(L, RM, 16, RL, A1);
    constexpr int AF = kPad ? PF : -1, AD = pad_after(L, RM, RL, 16, AF);
    constexpr int SEG = kPad ? PSEG : L + 32 / TC;
    constexpr int NT16 = L / 16;                            // radix-16 butterflies per column
    constexpr int IT16 = (TC * NT16 + NTH - 1) / NTH;       // per thread in phases A and D
    constexpr int NTL = L / RL;                             // last-radix butterflies per column
    constexpr int TPP = NTH / (TC / 2);                     // threads per column pair in phase C
    constexpr int ITL = (NTL + TPP - 1) / TPP;
    static_assert(L >= 256 && TC % 2 == 0 && NTH % (TC / 2) == 0, "col_kernel_f shape");
    __shared__ float2 lds[TC * SEG];
    // twiddles W_H^r in LDS: LDS latency instead of L2's for every pass; the
    // 4-column tiles of 2048 rows (the default there) read them from L2
    // instead, so that two workgroups fit in a CU's LDS and one's memory
    // phases overlap the other's (2048^2 sweep -3.5%)
    constexpr bool kTwLds = !col_tw_in_l2(L, TC);
    __shared__ float2 twl[kTwLds ? L : 1];
    const float2* twp = kTwLds ? twl : a.tw_col;
    const unsigned tid = threadIdx.x;
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int item = (int)(t / (W / TC));
    const int x0 = (int)(t % (W / TC)) * TC;
    // one record read before the field (the item carries its problem's
    // offset, tau and index); the twiddles go out beside it and the mode
    // table of phase C beside the field loads
    const ItemDev it = a.items[item];
    if constexpr (kTwLds)
        for (unsigned i = tid; i < (unsigned)L; i += NTH) twl[i] = a.tw_col[i];  // visible after phase A's barrier
    const ProbDev pr{H, W, it.pix_off, it.tau, it.pid};
    const int64_t f0 = it.field_off + x0;
    float2 pnp[ITL][RL];
    {
        const unsigned pp = tid / TPP, lane = tid % TPP;
        const float2* npt = a.nPt + pr.pix_off / 2 + (int64_t)((x0 + 2 * (int)pp) / 2) * H;
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPP;
#pragma unroll
            for (int r = 0; r < RL; ++r)
                pnp[i][r] = NTL % TPP == 0 || j < (unsigned)NTL ? npt[j + r * NTL] : make_float2(0.f, 0.f);
        }
    }

    // ---- A: first forward pass (NS = 1), inputs from HBM
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        const E* fld = reinterpret_cast<const E*>(a.field) + f0;
        float2 v[IT16][16];
#pragma unroll
        for (int i = 0; i < IT16; ++i) {
            const unsigned b = tid + i * NTH;
            if ((TC * NT16) % NTH == 0 || b < (unsigned)(TC * NT16)) {
                const unsigned c = b % TC, j = b / TC;
#pragma unroll
                for (int r = 0; r < 16; ++r) v[i][r] = widen(fld[(int64_t)(j + r * NT16) * W + c]);
            }
        }
#pragma unroll
        for (int i = 0; i < IT16; ++i) {
            const unsigned b = tid + i * NTH;
            if ((TC * NT16) % NTH == 0 || b < (unsigned)(TC * NT16)) {
                const unsigned c = b % TC, j = b / TC;
                dft<16, false>(v[i]);
#pragma unroll
                for (int r = 0; r < 16; ++r) lds[c * SEG + lpos_run<A1, 16>(j, r)] = v[i][r];
            }
        }
    });
    __syncthreads();

    // ---- B: middle forward passes
    {
        const unsigned cid = tid / TPC, lane = tid % TPC;
        passes_before<L, RM, 16, RL, TPC, false, A1>(lds + cid * SEG, lane, twp);
    }

    // ---- C: last forward pass + Fourier-space update + first inverse pass
    {
        const float T = a.lambda * pr.tau;
        const float inv_n = 1.0f / ((float)H * (float)W);
        const unsigned pp = tid / TPP, lane = tid % TPP;
        const int kx0 = x0 + 2 * (int)pp;
        float2 v[ITL][2][RL];
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPP;
            if (NTL % TPP == 0 || j < (unsigned)NTL) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < RL; ++r) v[i][q][r] = lds[(2 * pp + q) * SEG + lpos_step<AC, NTL>(j, r)];
#pragma unroll
                for (int r = 1; r < RL; ++r) {
                    const float2 w = twp[r * j];
                    v[i][0][r] = cmul(v[i][0][r], w);
                    v[i][1][r] = cmul(v[i][1][r], w);
                }
                dft<RL, false>(v[i][0]);
                dft<RL, false>(v[i][1]);
                // v[i][q][r] now holds mode (ky, kx0 + q), ky = j + r NTL
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const unsigned ky = j + r * NTL;
                    const float2 np = pnp[i][r];
                    float2 z[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                    if (a.stochastic) {
                        const int64_t mode = (int64_t)ky * W + kx0;
                        const Normals2 nz = pair_normals((uint32_t)(mode >> 1), a.sweep, (uint32_t)pr.pid,
                                                         kStageHarmonic, (uint32_t)it.pair, a.key0, a.key1);
                        z[0] = nz.a;
                        z[1] = nz.b;
                    }
                    const float npv[2] = {np.x, np.y};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const float P = npv[q];
                        const float rden = __builtin_amdgcn_rcpf(P + T);
                        const float f = P * rden * inv_n;
                        float2 o = cscale(v[i][q][r], f);
                        if (a.stochastic) {
                            const float w = __builtin_amdgcn_sqrtf(P * T * rden * inv_n);
                            o.x = fmaf(w, z[q].x, o.x);
                            o.y = fmaf(w, z[q].y, o.y);
                        }
                        v[i][q][r] = o;
                    }
                }
                dft<RL, true>(v[i][0]);
                dft<RL, true>(v[i][1]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITL; ++i) {
            const unsigned j = lane + i * TPP;
            if (NTL % TPP == 0 || j < (unsigned)NTL) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < RL; ++r) lds[(2 * pp + q) * SEG + lpos_run<AF, RL>(j, r)] = v[i][q][r];
            }
        }
        __syncthreads();
    }

    // ---- D: middle inverse passes, then the last one (NS = L/16) to HBM
    {
        const unsigned cid = fresh(tid) / TPC, lane = fresh(tid) % TPC;
        passes_before<L, RM, RL, 16, TPC, true, AF>(lds + cid * SEG, lane, twp + fresh(0u));
    }
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        E* fld = reinterpret_cast<E*>(a.field) + f0;
        const unsigned tid2 = fresh(tid);
        const float2* tw = twp + fresh(0u);
        float2 v[IT16][16];
#pragma unroll
        for (int i = 0; i < IT16; ++i) {
            const unsigned b = tid2 + i * NTH;
            if ((TC * NT16) % NTH == 0 || b < (unsigned)(TC * NT16)) {
                const unsigned c = b % TC, j = b / TC;
#pragma unroll
                for (int r = 0; r < 16; ++r) v[i][r] = lds[c * SEG + lpos_step<AD, NT16>(j, r)];
#pragma unroll
                for (int r = 1; r < 16; ++r) v[i][r] = cmulc(v[i][r], tw[r * j]);
                dft<16, true>(v[i]);
#pragma unroll
                for (int r = 0; r < 16; ++r) fld[(int64_t)(j + r * NT16) * W + c] = narrow<E>(v[i][r]);
            }
        }
    });
}

__global__ void band_slots_reduce_kernel(SweepArgs a, int tiles_per_item, const int32_t* band_base,
                                         const int32_t* band_count, double* out) {
    const int item = blockIdx.x;
    const ItemDev it = a.items[item];
    const int cnt = band_count[it.prob];
    for (int b = threadIdx.x; b < cnt; b += blockDim.x) {
        double s = 0.0;
        for (int64_t t = (int64_t)item * tiles_per_item; t < (int64_t)(item + 1) * tiles_per_item; ++t)
            s += a.band_slots[t * kMaxBandsPerProblem + b];
        out[band_base[it.prob] + b] = s;
    }
}

// Shapes the launcher can use (tile width, threads), per column length.
struct ColCfg {
    int tc, nth;
};

// ------------------------------------------------------------ elementwise --
__global__ void init_kernel(SweepArgs a, int H, int W, const float2* state_in, float init_scale) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total / 2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = 2 * e;
        const int item = (int)(g / n);
        const int64_t i = g % n;
        const ItemDev it = a.items[item];
        float2 v0 = make_float2(0.f, 0.f), v1 = v0;
        if (state_in) {
            v0 = state_in[it.field_off + i];
            v1 = state_in[it.field_off + i + 1];
        } else if (init_scale > 0.f) {
            const ProbDev pr = a.probs[it.prob];
            const Normals2 nz = pair_normals((uint32_t)(i >> 1), 0u, (uint32_t)pr.pid, kStageInit,
                                             (uint32_t)it.pair, a.key0, a.key1);
            v0 = cscale(nz.a, init_scale);
            v1 = cscale(nz.b, init_scale);
        }
        with_storage(a.storage, [&](auto e0) {
            using E = decltype(e0);
            E* fld = reinterpret_cast<E*>(a.field) + it.field_off + i;
            fld[0] = narrow<E>(v0);
            fld[1] = narrow<E>(v1);
        });
    }
}

__global__ void copy_out_real_kernel(SweepArgs a, int H, int W, float* out) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        out[a.probs[it.prob].pix_off + i] = a.field[it.field_off + i].x;
    }
}

__global__ void copy_out_pairs_kernel(SweepArgs a, int H, int W, float2* out) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        with_storage(a.storage, [&](auto e0) {
            using E = decltype(e0);
            out[it.field_off + i] = widen(reinterpret_cast<const E*>(a.field)[it.field_off + i]);
        });
    }
}

__global__ void grad_d_kernel(SweepArgs a, int H, int W, const float* v, float* grad_d) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        const ProbDev pr = a.probs[it.prob];
        const float nb = a.nbar[pr.pix_off + i];
        // N^-1 v with N = Nbar + tau; 0 on missing pixels (Nbar = +inf)
        grad_d[pr.pix_off + i] = v[pr.pix_off + i] * __builtin_amdgcn_rcpf(nb + pr.tau);
    }
}

__global__ void scale_kernel(const float* x, const float* r, float* y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e] * r[e];
}

// ------------------------------------------------------ sample moments --
// Problem of a concatenated pixel index (problems are in pix_off order).
__device__ __forceinline__ int problem_of(const ProbDev* probs, int n_problems, int64_t g) {
    int lo = 0, hi = n_problems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (probs[mid].pix_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Shifted sums over one slice of the chain-sample axis: with K the pixel's
// first sample, acc = (sum (x - K), sum (x - K)^2) in FP64 (accumulated
// across slices with atomics).
__global__ void moments_kernel(const ProbDev* probs, int n_problems, int64_t total_px, const float* samples,
                               int64_t m, int64_t slice, double2* acc) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_px) return;
    const ProbDev pr = probs[problem_of(probs, n_problems, g)];
    const int64_t n = (int64_t)pr.H * pr.W;
    const float* x = samples + m * pr.pix_off + (g - pr.pix_off);
    const double K = x[0];
    const int64_t k0 = (int64_t)blockIdx.y * slice, k1 = min(m, k0 + slice);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
    for (int64_t k = k0; k < k1; ++k) {
        const double d = (double)x[k * n] - K;
        s1 += d;
        s2 = fma(d, d, s2);
    }
    atomicAdd(&acc[g].x, s1);
    atomicAdd(&acc[g].y, s2);
}

__global__ void moments_finish_kernel(const float* samples, const ProbDev* probs, int n_problems, int64_t total_px,
                                      int64_t m, const double2* acc, double* mean, double* var) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total_px;
         g += (int64_t)gridDim.x * blockDim.x) {
        const ProbDev pr = probs[problem_of(probs, n_problems, g)];
        const double K = samples[m * pr.pix_off + (g - pr.pix_off)];
        const double2 a = acc[g];
        mean[g] = K + a.x / (double)m;
        if (var) var[g] = m > 1 ? (a.y - a.x * a.x / (double)m) / (double)(m - 1) : 0.0;
    }
}

__global__ void zero_kernel(double2* p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = make_double2(0.0, 0.0);
}

// Pack z = x + i y into the field so one complex FFT gives both spectra.
__global__ void pack_pair_kernel(SweepArgs a, int H, int W, const float* x, const float* y) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        const int64_t p = a.probs[it.prob].pix_off + i;
        a.field[it.field_off + i] = make_float2(x[p], y[p]);
    }
}

// Forward row FFTs only (for the band reduction).
template <int L>
__global__ __launch_bounds__(kThreads) void row_fft_kernel(SweepArgs a, int H) {
    constexpr int ROWS = RowShape<L>::ROWS;
    constexpr int TPR = RowShape<L>::TPR;
    constexpr int LS = RowShape<L>::LS;
    constexpr int NE = RowShape<L>::NE;
    __shared__ float2 lds[ROWS * LS];
    const unsigned tid = threadIdx.x;
    const int64_t total_rows = (int64_t)a.n_items * H;
    const int64_t grow0 = (int64_t)blockIdx.x * ROWS;
    for (int i = 0; i < RowShape<L>::NL; ++i) {
        const unsigned e = tid + i * kThreads;
        if (e >= (unsigned)NE) break;
        const int64_t gr = grow0 + e / L;
        lds[(e / L) * LS + swz(e % L)] =
            gr < total_rows ? a.field[a.items[gr / H].field_off + (gr % H) * L + e % L] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    stockham_fft<L, 1, TPR, false>(lds + (tid / TPR) * LS, tid % TPR, a.tw_row);
    for (int i = 0; i < RowShape<L>::NL; ++i) {
        const unsigned e = tid + i * kThreads;
        if (e >= (unsigned)NE) break;
        const int64_t gr = grow0 + e / L;
        if (gr < total_rows) a.field[a.items[gr / H].field_off + (gr % H) * L + e % L] = lds[(e / L) * LS + swz(e % L)];
    }
}

template <int L>
__global__ __launch_bounds__(ColShape<L>::NTH) void col_fft_kernel(SweepArgs a, int W) {
    constexpr int TC = ColShape<L>::TC;
    constexpr int NTH = ColShape<L>::NTH;
    constexpr int TPC = ColShape<L>::TPC;
    constexpr int SEG = ColShape<L>::SEG;
    __shared__ float2 lds[TC * SEG];
    const unsigned tid = threadIdx.x;
    const int tpi = tiles_per_item(W, TC);
    const int x0 = (int)(blockIdx.x % tpi) * TC;
    const unsigned ncol = (unsigned)min(TC, W - x0);
    const ItemDev it = a.items[blockIdx.x / tpi];
    float2* fld = a.field + it.field_off + x0;
    for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH)
        lds[(e % TC) * SEG + swz(e / TC)] = e % TC < ncol ? fld[(int64_t)(e / TC) * W + e % TC] : make_float2(0.f, 0.f);
    __syncthreads();
    stockham_fft<L, 1, TPC, false>(lds + (tid / TPC) * SEG, tid % TPC, a.tw_col);
    for (unsigned e = tid; e < (unsigned)(TC * L); e += NTH)
        if (e % TC < ncol) fld[(int64_t)(e / TC) * W + e % TC] = lds[(e % TC) * SEG + swz(e / TC)];
}

// Per-block, per-band partial sums of Re(conj(X_k) Y_k) with X = (Z_k + conj Z_-k)/2,
// Y = (Z_k - conj Z_-k)/(2i) from the packed spectrum Z; FP64 accumulation.
constexpr int kMaxBands = 64;
__global__ __launch_bounds__(kThreads) void band_partial_kernel(SweepArgs a, int H, int W, const int16_t* band,
                                                                 int32_t nb_max, double* partial) {
    __shared__ double acc[kMaxBands];
    const int tid = threadIdx.x;
    for (int b = tid; b < kMaxBands; b += kThreads) acc[b] = 0.0;
    __syncthreads();
    const int64_t n = (int64_t)H * W;
    const int item = blockIdx.y;
    const ItemDev it = a.items[item];
    const ProbDev pr = a.probs[it.prob];
    const float2* Z = a.field + it.field_off;
    for (int64_t m = (int64_t)blockIdx.x * kThreads + tid; m < n; m += (int64_t)gridDim.x * kThreads) {
        const int b = band[pr.pix_off + m];
        if (b < 0) continue;
        const int ky = (int)(m / W), kx = (int)(m % W);
        const int64_t mm = (int64_t)((H - ky) % H) * W + (W - kx) % W;
        const float2 zk = Z[m], zm = Z[mm];
        // X = (zk + conj zm)/2, Y = (zk - conj zm)/(2i)
        const double xr = 0.5 * ((double)zk.x + zm.x), xi = 0.5 * ((double)zk.y - zm.y);
        const double yr = 0.5 * ((double)zk.y + zm.y), yi = -0.5 * ((double)zk.x - zm.x);
        atomicAdd(&acc[b], xr * yr + xi * yi);  // LDS atomic
    }
    __syncthreads();
    for (int b = tid; b < nb_max; b += kThreads)
        partial[((int64_t)item * gridDim.x + blockIdx.x) * nb_max + b] = acc[b];
}

__global__ void band_sum_kernel(SweepArgs a, const double* partial, int nblocks, int32_t nb_max,
                                const int32_t* band_base, const int32_t* band_count, const double* scale,
                                double* out) {
    const int item = blockIdx.x;
    const ItemDev it = a.items[item];
    const int base = band_base[it.prob];
    const int cnt = band_count[it.prob];
    for (int b = threadIdx.x; b < cnt; b += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nblocks; ++k) s += partial[((int64_t)item * nblocks + k) * nb_max + b];
        out[base + b] = scale ? s * scale[base + b] : s;
    }
}

__global__ void load_real_kernel(SweepArgs a, int H, int W, const float* s_init) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        a.field[it.field_off + i] = make_float2(s_init ? s_init[a.probs[it.prob].pix_off + i] : 0.f, 0.f);
    }
}

// ------------------------------------------------------ plan plumbing --
__global__ void fill_items_kernel(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n, int per, int local,
                                  int64_t hw) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int pid = pids[i / per];
        const int q = i % per;
        const ProbDev pr = probs[pid];
        out[i] = ItemDev{pid, q, local ? (int64_t)i * hw : (int64_t)per * pr.pix_off + (int64_t)q * hw, pr.pix_off,
                         pr.tau, pr.pid};
    }
}

__global__ void fill_packed_items_kernel(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n_pids,
                                         int64_t hw) {
    const int n = (n_pids + 1) / 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const ProbDev pr = probs[pids[2 * i]];
        out[i] = ItemDev{pids[2 * i], 2 * i + 1 < n_pids ? pids[2 * i + 1] : -1, (int64_t)i * hw, pr.pix_off, pr.tau,
                         pr.pid};
    }
}

// Packed work field from single-chain states: the real part of problem A's
// pair-0 state, and of B's, or zero / dispersed (stage-2 words .x of each
// problem's pair 0) starts.
__global__ void pack_init_kernel(SweepArgs a, int H, int W, const float2* state_in, float init_scale) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total / 2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = 2 * e;
        const int item = (int)(g / n);
        const int64_t i = g % n;
        const ItemDev it = a.items[item];
        const ProbDev pa = a.probs[it.prob];
        const ProbDev pb = it.pair >= 0 ? a.probs[it.pair] : pa;
        float2 v0 = make_float2(0.f, 0.f), v1 = v0;
        if (state_in) {
            v0 = make_float2(state_in[pa.pix_off + i].x, state_in[pb.pix_off + i].x);
            v1 = make_float2(state_in[pa.pix_off + i + 1].x, state_in[pb.pix_off + i + 1].x);
        } else if (init_scale > 0.f) {
            const Normals2 za = pair_normals((uint32_t)(i >> 1), 0u, (uint32_t)pa.pid, kStageInit, 0u, a.key0, a.key1);
            const Normals2 zb = pair_normals((uint32_t)(i >> 1), 0u, (uint32_t)pb.pid, kStageInit, 0u, a.key0, a.key1);
            v0 = make_float2(init_scale * za.a.x, init_scale * zb.a.x);
            v1 = make_float2(init_scale * za.b.x, init_scale * zb.b.x);
        }
        if (it.pair < 0) v0.y = v1.y = 0.f;  // no partner: the imaginary part stays zero
        a.field[it.field_off + i] = v0;
        a.field[it.field_off + i + 1] = v1;
    }
}

__global__ void pack_copy_out_kernel(SweepArgs a, int H, int W, float2* out) {
    const int64_t n = (int64_t)H * W;
    const int64_t total = (int64_t)a.n_items * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int item = (int)(e / n);
        const int64_t i = e % n;
        const ItemDev it = a.items[item];
        const float2 v = a.field[it.field_off + i];
        out[a.probs[it.prob].pix_off + i] = make_float2(v.x, 0.f);
        if (it.pair >= 0) out[a.probs[it.pair].pix_off + i] = make_float2(v.y, 0.f);
    }
}

__global__ void zero_words_kernel(uint32_t* p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

__global__ void fill_int_kernel(int32_t* p, int32_t v, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ void band_dof_kernel(const int32_t* modes, int32_t prior_dof, int32_t* dof, int n) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x)
        dof[b] = max(0, modes[b] + prior_dof);
}

__global__ void add_kernel(const float* x, float* y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] += x[e];
}

// One block per item: any NaN or infinity in the item's field lowers the
// flag to the item's problem index (packed items: the real part belongs to
// problem `prob`, the imaginary part to `pair`).
// Each item's field is scanned by `per` consecutive blocks (enough blocks over
// all items to keep every CU streaming).
__global__ void finite_check_kernel(SweepArgs a, int64_t n, int32_t per, int32_t* flag) {
    const ItemDev it = a.items[blockIdx.x / per];
    const int64_t b0 = blockIdx.x % per;
    bool bad_a = false, bad_b = false;
    with_storage(a.storage, [&](auto e0) {
        using E = decltype(e0);
        const E* fld = reinterpret_cast<const E*>(a.field) + it.field_off;
        for (int64_t i = b0 * blockDim.x + threadIdx.x; i < n; i += (int64_t)per * blockDim.x) {
            const float2 v = widen(fld[i]);
            bad_a |= !isfinite(v.x);
            bad_b |= !isfinite(v.y);
        }
    });
    if (!a.packed) bad_a |= bad_b;
    const bool any_a = __syncthreads_or(bad_a), any_b = __syncthreads_or(bad_b);
    if (threadIdx.x == 0) {
        if (any_a) atomicMin(flag, it.prob);
        if (a.packed && any_b && it.pair >= 0) atomicMin(flag, it.pair);
    }
}

// Loss terms per item (one item per problem, real fields).
__global__ __launch_bounds__(kThreads) void loss_terms_kernel(SweepArgs a, int64_t n, const float* d,
                                                              const float* s_wf, const float* s_true, float* grad_s,
                                                              float* grad_d, double* part) {
    __shared__ double red[2][kThreads];
    const ItemDev it = a.items[blockIdx.y];
    const ProbDev pr = a.probs[it.prob];
    double lik = 0.0, l2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const int64_t g = pr.pix_off + i;
        const float nb = a.nbar[g];
        const float sv = s_wf[g];
        const float e = sv - s_true[g];
        // N_eff^-1 (d - s) with N_eff = Nbar + tau; 0 on missing pixels (Nbar = +inf)
        const double r = isinf(nb) ? 0.0 : ((double)d[g] - (double)sv) / ((double)nb + (double)pr.tau);
        lik += r * ((double)d[g] - (double)sv);
        l2 += (double)e * (double)e;
        grad_s[g] = e;
        grad_d[g] = (float)r;
    }
    red[0][threadIdx.x] = lik;
    red[1][threadIdx.x] = l2;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        o[0] = red[0][0];
        o[1] = red[1][0];
    }
}

__global__ void loss_finish_kernel(SweepArgs a, const double* part, int nblocks, const double* power,
                                   const double* amps, const int32_t* band_modes, const int32_t* band_base,
                                   const int32_t* band_count, double* loss, double* grad_bands) {
    __shared__ double red[64];
    const ItemDev it = a.items[blockIdx.x];
    const ProbDev pr = a.probs[it.prob];
    const double n = (double)pr.H * (double)pr.W;
    const int base = band_base[it.prob], cnt = band_count[it.prob];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += blockDim.x) {
        const double* o = part + ((int64_t)blockIdx.x * nblocks + k) * 2;
        acc += 0.5 * (o[0] + o[1]);
    }
    for (int b = threadIdx.x; b < cnt; b += blockDim.x) {
        const double th = amps[base + b], pw = power[base + b], m = (double)band_modes[base + b];
        acc += 0.5 * (pw / (n * n * th) + m * log(n * th));
        if (grad_bands) grad_bands[base + b] += -0.5 * pw / (n * n * th * th) + 0.5 * m / th;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[it.prob] = red[0];
}

// The transform lengths: powers of two (every kernel) and the other even
// 2^a 3^b in [16, 2048] (the plain row and column kernels and the helpers).
template <int... Ls>
struct Lengths {};
using Pow2Lengths = Lengths<16, 32, 64, 128, 256, 512, 1024, 2048>;
using MixedLengths = Lengths<18, 24, 36, 48, 54, 72, 96, 108, 144, 162, 192, 216, 288, 324, 384, 432, 486, 576,
                             648, 768, 864, 972, 1152, 1296, 1458, 1536, 1728, 1944>;

// Call f(std::integral_constant<int, L>) for the length L of the list; false
// if L is not in it.
template <typename F, int... Ls>
bool with_length(int L, Lengths<Ls...>, F&& f) {
    return ((L == Ls ? (f(std::integral_constant<int, Ls>{}), true) : false) || ...);
}
template <typename F>
bool with_any_length(int L, F&& f) {
    return with_length(L, Pow2Lengths{}, f) || with_length(L, MixedLengths{}, f);
}

template <int MODE>
hipError_t launch_row_mode(int W, int H, const SweepArgs& a, hipStream_t s) {
    const int rows = rows_per_block(W);
    const int64_t total = (int64_t)a.n_items * H;
    dim3 grid((unsigned)((total + rows - 1) / rows));
    // middle sweeps of the sampler and the Wiener iteration on rows of 256 and
    // more (powers of two)
    const bool fused = MODE == kRowInvFwd && W >= 256 && is_pow2(W) && a.pix_mode == kPixUpdate && !a.s_save &&
                       !a.plain_kernels;
    if (fused) {
        const int rows_w = a.row_rows > 0 ? a.row_rows : (W == 512 ? 8 : 2048 / W);
        const int rows_n = a.row_rows_narrow > 0 ? a.row_rows_narrow : narrow_row_rows(W);
        const bool narrow = (total + rows_w - 1) / rows_w < kFillBlocks;
        const int rows_f = narrow ? rows_n : rows_w;
        const int var = a.packed ? kRowAny : (narrow ? kRowPrefetch : kRowLoadLate);
        const dim3 grid((unsigned)((total + rows_f - 1) / rows_f));
#define MF_ROWF_CASE(LL, RR)                                                                             \
    if (W == LL && rows_f == RR) {                                                                        \
        if (var == kRowAny)                                                                            \
            hipLaunchKernelGGL((row_kernel_f<LL, RR, kRowAny>), grid, dim3(kThreads), 0, s, a, H);     \
        else if (var == kRowPrefetch)                                                                     \
            hipLaunchKernelGGL((row_kernel_f<LL, RR, kRowPrefetch>), grid, dim3(kThreads), 0, s, a, H);   \
        else                                                                                              \
            hipLaunchKernelGGL((row_kernel_f<LL, RR, kRowLoadLate>), grid, dim3(kThreads), 0, s, a, H);   \
        return hipGetLastError();                                                                         \
    }
        MF_ROWF_CASE(256, 8) MF_ROWF_CASE(256, 4) MF_ROWF_CASE(256, 16)
        MF_ROWF_CASE(512, 8) MF_ROWF_CASE(512, 4) MF_ROWF_CASE(512, 2)
        MF_ROWF_CASE(1024, 2) MF_ROWF_CASE(1024, 1) MF_ROWF_CASE(1024, 4)
        MF_ROWF_CASE(2048, 1) MF_ROWF_CASE(2048, 2)
#undef MF_ROWF_CASE
        return hipErrorInvalidValue;
    }
    const bool ok = with_any_length(W, [&](auto c) {
        constexpr int N = decltype(c)::value;
        hipLaunchKernelGGL((row_kernel<N, MODE>), grid, dim3(kThreads), 0, s, a, H);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}


dim3 elementwise_grid(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

}  // namespace

int fused_row_candidates(int W, int* rows, int max_n) {
    static const int table[][2] = {{256, 8}, {256, 4}, {256, 16}, {512, 8}, {512, 4}, {512, 2},
                                   {1024, 2}, {1024, 1}, {1024, 4}, {2048, 1}, {2048, 2}};
    int n = 0;
    for (const auto& r : table)
        if (r[0] == W && n < max_n) rows[n++] = r[1];
    return n;
}

int narrow_row_rows(int W) {
    int rows[8];
    const int n = fused_row_candidates(W, rows, 8);
    int best = n > 0 ? rows[0] : 0;
    for (int i = 1; i < n; ++i) best = rows[i] < best ? rows[i] : best;
    return best;
}

int row_blocks_per_item(int W, int H) {
    const int rows = rows_per_block(W);
    return (H + rows - 1) / rows;
}

hipError_t launch_row(int W, int H, int row_mode, const SweepArgs& a, hipStream_t s) {
    switch (row_mode) {
        case kRowInv: return launch_row_mode<kRowInv>(W, H, a, s);
        case kRowFwd: return launch_row_mode<kRowFwd>(W, H, a, s);
        case kRowInvFwd: return launch_row_mode<kRowInvFwd>(W, H, a, s);
        default: return hipErrorInvalidValue;
    }
}

#define MF_COL_CASE(LL, TCC, NN)                                                              \
    if (H == LL && tc == TCC && nth == NN) {                                                   \
        hipLaunchKernelGGL((col_kernel_t<LL, TCC, NN>), grid, dim3(NN), 0, s, a, W);           \
        return hipGetLastError();                                                              \
    }
// H >= 256 without the gradient's stored transforms: the fused kernel
#define MF_COL_CASE_F(LL, TCC, NN)                                                            \
    if (H == LL && tc == TCC && nth == NN) {                                                   \
        if (fused)                                                                             \
            hipLaunchKernelGGL((col_kernel_f<LL, TCC, NN>), grid, dim3(NN), 0, s, a, W);       \
        else                                                                                   \
            hipLaunchKernelGGL((col_kernel_t<LL, TCC, NN>), grid, dim3(NN), 0, s, a, W);       \
        return hipGetLastError();                                                              \
    }

hipError_t launch_col_shape(int W, int H, int tc, int nth, const SweepArgs& a, hipStream_t s) {
    if (tc < 2) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((int64_t)a.n_items * ((W + tc - 1) / tc)));
    const bool fused = !a.t_store && !a.t_load && a.nPt && !a.plain_kernels;
    MF_COL_CASE(16, 16, 256) MF_COL_CASE(32, 16, 256) MF_COL_CASE(64, 16, 256) MF_COL_CASE(128, 16, 256)
    MF_COL_CASE_F(256, 16, 256) MF_COL_CASE_F(256, 8, 256) MF_COL_CASE_F(256, 16, 512) MF_COL_CASE_F(256, 8, 512)
    MF_COL_CASE_F(256, 4, 128) MF_COL_CASE_F(256, 4, 256)
    MF_COL_CASE_F(512, 16, 512) MF_COL_CASE_F(512, 8, 512) MF_COL_CASE_F(512, 16, 256) MF_COL_CASE_F(512, 16, 1024)
    MF_COL_CASE_F(512, 8, 256) MF_COL_CASE_F(512, 4, 256)
    MF_COL_CASE_F(1024, 16, 1024) MF_COL_CASE_F(1024, 8, 1024) MF_COL_CASE_F(1024, 8, 512) MF_COL_CASE_F(1024, 16, 512)
    MF_COL_CASE_F(1024, 4, 256)
    MF_COL_CASE_F(2048, 8, 1024) MF_COL_CASE_F(2048, 8, 512) MF_COL_CASE_F(2048, 4, 512) MF_COL_CASE_F(2048, 4, 256)
    // the other 2^a 3^b lengths: the plain kernel in its default tile
    bool launched = false;
    const bool ok = with_length(H, MixedLengths{}, [&](auto c) {
        constexpr int N = decltype(c)::value;
        if (tc == col_tc_of(N) && nth == col_nth_of(N)) {
            hipLaunchKernelGGL((col_kernel_t<N, col_tc_of(N), col_nth_of(N)>), grid, dim3(col_nth_of(N)), 0, s, a, W);
            launched = true;
        }
    });
    return ok && launched ? hipGetLastError() : hipErrorInvalidValue;
}
#undef MF_COL_CASE
#undef MF_COL_CASE_F

// Tile shapes per column length; the first one for a length is its default
// (the autotuner's choice on MI355X for the sampler's column kernel).  The
// lengths with a factor 3 have their one default tile.
int col_shape_candidates(int H, int* tc, int* nth, int max_n) {
    static const int table[][3] = {{16, 16, 256}, {32, 16, 256}, {64, 16, 256}, {128, 16, 256},
                                   {256, 8, 256}, {256, 16, 256}, {256, 16, 512}, {256, 8, 512},
                                   {256, 4, 128}, {256, 4, 256},
                                   {512, 8, 256}, {512, 16, 512}, {512, 8, 512}, {512, 16, 256},
                                   {512, 16, 1024}, {512, 4, 256},
                                   {1024, 4, 256}, {1024, 8, 512}, {1024, 16, 1024}, {1024, 8, 1024},
                                   {1024, 16, 512},
                                   {2048, 4, 256}, {2048, 8, 512}, {2048, 8, 1024}, {2048, 4, 512}};
    int n = 0;
    for (const auto& r : table)
        if (r[0] == H && n < max_n) {
            tc[n] = r[1];
            nth[n] = r[2];
            ++n;
        }
    if (n == 0 && max_n > 0 && !is_pow2(H)) {
        tc[0] = col_tc_of(H);
        nth[0] = col_nth_of(H);
        n = 1;
    }
    return n;
}

void narrow_col_shape(int H, int* tc, int* nth) {
    int t[16], n[16];
    const int k = col_shape_candidates(H, t, n, 16);
    int b = 0;
    for (int i = 1; i < k; ++i)
        if (t[i] < t[b] || (t[i] == t[b] && n[i] < n[b])) b = i;
    *tc = k > 0 ? t[b] : col_tc_of(H);
    *nth = k > 0 ? n[b] : col_nth_of(H);
}

hipError_t launch_band_slots_reduce(int W, int H, int tc, const SweepArgs& a, const int32_t* band_base,
                                    const int32_t* band_count, double* out, hipStream_t s) {
    (void)H;
    hipLaunchKernelGGL(band_slots_reduce_kernel, dim3(a.n_items), dim3(64), 0, s, a, (W + tc - 1) / tc, band_base,
                       band_count,
                       out);
    return hipGetLastError();
}

hipError_t launch_init_items(int W, int H, const SweepArgs& a, const float2* state_in, float init_scale,
                             hipStream_t s) {
    const int64_t total = (int64_t)a.n_items * H * W / 2;
    hipLaunchKernelGGL(init_kernel, elementwise_grid(total), dim3(256), 0, s, a, H, W, state_in, init_scale);
    return hipGetLastError();
}

hipError_t launch_copy_out_real(int W, int H, const SweepArgs& a, float* out, hipStream_t s) {
    hipLaunchKernelGGL(copy_out_real_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a, H,
                       W, out);
    return hipGetLastError();
}

hipError_t launch_copy_out_pairs(int W, int H, const SweepArgs& a, float2* out, hipStream_t s) {
    hipLaunchKernelGGL(copy_out_pairs_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a,
                       H, W, out);
    return hipGetLastError();
}

hipError_t launch_moments(const ProbDev* probs, int n_problems, int64_t total_px, const float* samples, int64_t m,
                          double2* acc, double* mean, double* var, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel, elementwise_grid(total_px), dim3(256), 0, s, acc, total_px);
    // enough slices of the chain-sample axis to keep about 2^18 threads reading
    int64_t slices = ((int64_t)1 << 18) / total_px;
    slices = slices < 1 ? 1 : (slices > m ? m : slices);
    if (slices > 65535) slices = 65535;
    const int64_t slice = (m + slices - 1) / slices;
    slices = (m + slice - 1) / slice;
    const dim3 grid((unsigned)((total_px + 255) / 256), (unsigned)slices);
    hipLaunchKernelGGL(moments_kernel, grid, dim3(256), 0, s, probs, n_problems, total_px, samples, m, slice, acc);
    hipLaunchKernelGGL(moments_finish_kernel, elementwise_grid(total_px), dim3(256), 0, s, samples, probs, n_problems,
                       total_px, m, acc, mean, var);
    return hipGetLastError();
}

hipError_t launch_scale(const float* x, const float* r, float* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, elementwise_grid(n), dim3(256), 0, s, x, r, y, n);
    return hipGetLastError();
}

hipError_t launch_grad_d(int W, int H, const SweepArgs& a, const float* v, float* grad_d, hipStream_t s) {
    hipLaunchKernelGGL(grad_d_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a, H, W, v,
                       grad_d);
    return hipGetLastError();
}

hipError_t launch_load_real(int W, int H, const SweepArgs& a, const float* s_init, hipStream_t s) {
    hipLaunchKernelGGL(load_real_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a, H, W,
                       s_init);
    return hipGetLastError();
}

hipError_t launch_band_power(int W, int H, const SweepArgs& a, const float* x, const float* y,
                             const int16_t* band, const int32_t* band_base, const int32_t* band_count,
                             const double* scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(pack_pair_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a, H, W,
                       x, y);
    const int rows = rows_per_block(W);
    const int64_t total_rows = (int64_t)a.n_items * H;
    const dim3 rgrid((unsigned)((total_rows + rows - 1) / rows));
    if (!with_any_length(W, [&](auto c) {
            hipLaunchKernelGGL(row_fft_kernel<decltype(c)::value>, rgrid, dim3(kThreads), 0, s, a, H);
        }))
        return hipErrorInvalidValue;
    const int tc = col_tc_of(H);
    const dim3 cgrid((unsigned)((int64_t)a.n_items * ((W + tc - 1) / tc)));
    if (!with_any_length(H, [&](auto c) {
            constexpr int N = decltype(c)::value;
            hipLaunchKernelGGL(col_fft_kernel<N>, cgrid, dim3(ColShape<N>::NTH), 0, s, a, W);
        }))
        return hipErrorInvalidValue;
    // partial buffer: the caller provides a.partials sized n_items * nblocks * kMaxBands
    const int nblocks = 64;
    hipLaunchKernelGGL(band_partial_kernel, dim3(nblocks, a.n_items), dim3(kThreads), 0, s, a, H, W, band,
                       (int32_t)kMaxBands, a.partials);
    hipLaunchKernelGGL(band_sum_kernel, dim3(a.n_items), dim3(64), 0, s, a, a.partials, nblocks,
                       (int32_t)kMaxBands, band_base, band_count, scale, out);
    return hipGetLastError();
}

hipError_t launch_fill_items(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n_pids, int per,
                             int local, int64_t hw, hipStream_t s) {
    const int n = n_pids * per;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_items_kernel, elementwise_grid(n), dim3(256), 0, s, out, probs, pids, n, per, local, hw);
    return hipGetLastError();
}

hipError_t launch_fill_packed_items(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n_pids, int64_t hw,
                                    hipStream_t s) {
    if (n_pids <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_packed_items_kernel, elementwise_grid((n_pids + 1) / 2), dim3(256), 0, s, out, probs, pids,
                       n_pids, hw);
    return hipGetLastError();
}

hipError_t launch_pack_init(int W, int H, const SweepArgs& a, const float2* state_in, float init_scale,
                            hipStream_t s) {
    hipLaunchKernelGGL(pack_init_kernel, elementwise_grid((int64_t)a.n_items * H * W / 2), dim3(256), 0, s, a, H, W,
                       state_in, init_scale);
    return hipGetLastError();
}

hipError_t launch_pack_copy_out(int W, int H, const SweepArgs& a, float2* state_out, hipStream_t s) {
    hipLaunchKernelGGL(pack_copy_out_kernel, elementwise_grid((int64_t)a.n_items * H * W), dim3(256), 0, s, a, H, W,
                       state_out);
    return hipGetLastError();
}

hipError_t launch_zero_words(void* p, int64_t n_words, hipStream_t s) {
    if (n_words <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, elementwise_grid(n_words), dim3(256), 0, s, static_cast<uint32_t*>(p),
                       n_words);
    return hipGetLastError();
}

hipError_t launch_fill_int(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_int_kernel, elementwise_grid(n), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_band_dof(const int32_t* modes, int32_t prior_dof, int32_t* dof, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(band_dof_kernel, elementwise_grid(n), dim3(256), 0, s, modes, prior_dof, dof, n);
    return hipGetLastError();
}

hipError_t launch_add(const float* x, float* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(add_kernel, elementwise_grid(n), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_finite_check(int W, int H, const SweepArgs& a, int32_t* flag, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    const int64_t n = (int64_t)H * W;
    int64_t per = (2048 + a.n_items - 1) / a.n_items;  // about 2048 blocks in all
    const int64_t most = (n + 255) / 256;
    per = per < 1 ? 1 : (per > most ? most : per);
    hipLaunchKernelGGL(finite_check_kernel, dim3((unsigned)(a.n_items * per)), dim3(256), 0, s, a, n, (int32_t)per,
                       flag);
    return hipGetLastError();
}

hipError_t launch_loss_terms(int W, int H, const SweepArgs& a, const float* d, const float* s_wf,
                             const float* s_true, float* grad_s, float* grad_d, double* part, hipStream_t s) {
    hipLaunchKernelGGL(loss_terms_kernel, dim3(kLossBlocks, a.n_items), dim3(kThreads), 0, s, a, (int64_t)H * W, d,
                       s_wf, s_true, grad_s, grad_d, part);
    return hipGetLastError();
}

hipError_t launch_loss_finish(const SweepArgs& a, const double* part, const double* power, const double* amps,
                              const int32_t* band_modes, const int32_t* band_base, const int32_t* band_count,
                              double* loss, double* grad_bands, hipStream_t s) {
    hipLaunchKernelGGL(loss_finish_kernel, dim3(a.n_items), dim3(64), 0, s, a, part, kLossBlocks, power, amps,
                       band_modes, band_base, band_count, loss, grad_bands);
    return hipGetLastError();
}

}  // namespace mf
