// Kernel-side descriptors and host launchers shared by the HIP sources and
// the host plan code.  No torch types; plain pointers only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

// One problem as the kernels see it.
struct ProbDev {
    int32_t H, W;
    int64_t pix_off;    // offset in concatenated pixel / mode arrays
    float tau;          // min observed noise variance
    int32_t pid;        // problem index (random-stream counter word)
};

// One unit of work: a chain pair of a problem (or a single real solve).  It
// repeats the problem record's offset, tau and index, so that a streamed block
// reads one record before it can address its field and tables, not two in turn.
struct ItemDev {
    int32_t prob;
    int32_t pair;
    int64_t field_off;  // float2 offset of this item's field in the work buffer
    int64_t pix_off;    // = probs[prob].pix_off
    float tau;          // = probs[prob].tau
    int32_t pid;        // = probs[prob].pid
};

// Cooling levels carried by value in the kernel arguments of the persistent
// kernels (no device table to upload), so that a call that launches them can
// be captured into a caller's graph.  Longer schedules run in several launches.
constexpr int kMaxLevels = 128;
struct Levels {
    double lambda[kMaxLevels];
    int32_t sweeps[kMaxLevels];
    int32_t n;
};

// What the right-hand side pointer holds.
enum SrcKind : int32_t {
    kSrcData = 0,   // b = N_eff^-1 d, pixel source a * d
    kSrcGrad = 1,   // b = g (adjoint solve), pixel source T * g
};

struct SweepArgs {
    const ProbDev* probs;
    const ItemDev* items;
    int32_t n_items;
    float2* field;            // work buffer: items' complex fields
    const float* src;         // concatenated data d or adjoint rhs g
    int32_t src_kind;
    const float* nbar;        // concatenated Nbar (+inf missing)
    const float* nP;          // concatenated n P(|k|) per mode (unshifted order)
    const float2* nPt;        // column-pair table: [pix_off/2 + (kx/2) H + ky] = (nP(ky,kx), nP(ky,kx+1)), or null
    const float2* tw_row;     // twiddles W_W^r
    const float2* tw_col;     // twiddles W_H^r
    float lambda;             // cooling level: T = lambda * tau
    int32_t stochastic;       // 1: draw variates (sampler), 0: Wiener iteration
    uint32_t key0, key1;      // Philox key
    uint32_t sweep;           // global sweep index of the pixel / harmonic draws
    // sample emission (row kernel, inverse pass)
    float* samples;           // [problem][chain][sample][H][W] or null
    int32_t emit_index;       // sample slot to write, < 0: none
    int32_t chains;           // chains per problem
    int32_t n_samples;        // samples per chain
    // residual support (row kernel, forward pass)
    float2* t_save;           // messenger snapshot buffer (same layout as field), or null
    int32_t save_t;           // 1: write t to t_save
    int32_t check_t;          // 1: accumulate |t - t_save|^2 into partials
    double* partials;         // [item][row block] partial sums
    int32_t real_only;        // 1: the imaginary channel is unused (Wiener / adjoint)
    // reverse-mode sweeps (unrolled gradient)
    int32_t pix_mode;         // kPixUpdate, kPixAdjoint or kPixIdentity (row kernel)
    float* grad_d;            // kPixAdjoint: grad_d += a t (concatenated pixels)
    float2* s_save;           // row kernel: state after the inverse row FFT (field layout), or null
    float2* t_store;          // col kernel: forward 2D transform of t (field layout), or null
    const float2* t_load;     // col kernel: stored transform to pair with for band sums, or null
    double* band_slots;       // col kernel: per-tile band sums [tile][kMaxBandsPerProblem], accumulated
    const int16_t* band;      // per-mode band index (concatenated), -1 = none
    int32_t storage;          // kStoreF32 / kStoreF16 / kStoreBF16: element type of `field`
    int32_t plain_kernels;    // 1: row_kernel / col_kernel_t only (no fused variants)
    int32_t rows_by_item;     // row enumeration: 1 g = item H + y (one item per problem), 0 g = y n_items + item
    int32_t row_rows;         // rows per block of the fused row kernel (0: the default shape)
    int32_t row_rows_narrow;  // the same when that shape leaves CUs idle (0: the narrow default)
    int32_t packed;           // 1: each item carries two single-chain problems, chain 0 of problem `prob`
                              // in the real part and chain 0 of problem `pair` (-1: none) in the imaginary
                              // part, each with its own tables and random stream (sampler, streamed form)
};

// Element type of the work field (row, column, init and copy-out kernels of
// the sampler): FP32 pairs, or FP16 / BF16 pairs of 4 bytes.
enum Storage : int32_t { kStoreF32 = 0, kStoreF16 = 1, kStoreBF16 = 2 };

enum PixMode : int32_t {
    kPixUpdate = 0,    // messenger step t = (1 - a) s + src (+ sigma xi)
    kPixAdjoint = 1,   // transpose of the pixel step: grad_d += a t, t <- (1 - a) t
    kPixIdentity = 2,  // leave the row as it is
};

// Host launchers (defined in mf_streamed.hip).  mode bit 1: inverse row FFT +
// emission first; bit 2: pixel update + forward row FFT.
enum RowMode : int32_t { kRowInv = 1, kRowFwd = 2, kRowInvFwd = 3 };
hipError_t launch_row(int W, int H, int row_mode, const SweepArgs& a, hipStream_t s);
// Column kernel with an explicit tile shape (TC columns, nth threads), and the
// shapes available for a column length (returns how many were written).
hipError_t launch_col_shape(int W, int H, int tc, int nth, const SweepArgs& a, hipStream_t s);
int col_shape_candidates(int H, int* tc, int* nth, int max_n);
// Rows per block of the fused row kernel available for a row length (the
// first is the default; none below 256 points or for non-powers of two).
int fused_row_candidates(int W, int* rows, int max_n);
// A launch whose grid in the default (or tuned) shape would have fewer blocks
// than the GPU has CUs (a single solve, a few chains) takes the narrow shape
// instead: tuned on one item, else the candidate with the most blocks.
constexpr int kFillBlocks = 256;
// Column tiles that read their twiddles from L2 instead of LDS: 4 columns of
// 2048 rows, so that two workgroups fit in a CU's LDS and one's memory phases
// overlap the other's.
constexpr bool col_tw_in_l2(int L, int tc) { return L == 2048 && tc <= 4; }
void narrow_col_shape(int H, int* tc, int* nth);
int narrow_row_rows(int W);
// Sum per-tile band slots into out[band_base[prob] + b] for every item.
hipError_t launch_band_slots_reduce(int W, int H, int tc, const SweepArgs& a, const int32_t* band_base,
                                    const int32_t* band_count, double* out, hipStream_t s);
int row_blocks_per_item(int W, int H);

// Elementwise helpers (mf_streamed.hip).
hipError_t launch_init_items(int W, int H, const SweepArgs& a, const float2* state_in, float init_scale,
                             hipStream_t s);
hipError_t launch_copy_out_real(int W, int H, const SweepArgs& a, float* out, hipStream_t s);
hipError_t launch_copy_out_pairs(int W, int H, const SweepArgs& a, float2* out, hipStream_t s);
// Per-pixel mean and unbiased variance over the m = chains * n_samples values
// of every pixel in a sample array [problem][chain][sample][H][W]; acc is a
// 16-byte-per-pixel workspace.
hipError_t launch_moments(const ProbDev* probs, int n_problems, int64_t total_px, const float* samples, int64_t m,
                          double2* acc, double* mean, double* var, hipStream_t s);
// y[i] = x[i] * r[i] for i < n (y may be x).
hipError_t launch_scale(const float* x, const float* r, float* y, int64_t n, hipStream_t s);
hipError_t launch_grad_d(int W, int H, const SweepArgs& a, const float* v, float* grad_d, hipStream_t s);
hipError_t launch_load_real(int W, int H, const SweepArgs& a, const float* s_init, hipStream_t s);
// Band cross-power of two real fields per item (a.partials must hold
// n_items * kBandBlocks * kMaxBands doubles); out[band_base[p] + b] = scale * sum.
constexpr int kBandBlocks = 64;
constexpr int kMaxBandsPerProblem = 64;
hipError_t launch_band_power(int W, int H, const SweepArgs& a, const float* x, const float* y,
                             const int16_t* band, const int32_t* band_base, const int32_t* band_count,
                             const double* scale, double* out, hipStream_t s);

// Work lists built on the device: item i = (pids[i / per], i % per,
// field_off), field_off = per * pix_off + (i % per) * hw, or i * hw with
// `local` (a field of the class's items only).
hipError_t launch_fill_items(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n_pids, int per,
                             int local, int64_t hw, hipStream_t s);
// Packed work list: item i = (pids[2i], pids[2i+1] or -1, i * hw).
hipError_t launch_fill_packed_items(ItemDev* out, const ProbDev* probs, const int32_t* pids, int n_pids, int64_t hw,
                                    hipStream_t s);
// Packed work field from the pair states [problem][1][H][W] (real parts), or
// zero / dispersed starts; and back (imaginary parts of the states set to 0).
hipError_t launch_pack_init(int W, int H, const SweepArgs& a, const float2* state_in, float init_scale,
                            hipStream_t s);
hipError_t launch_pack_copy_out(int W, int H, const SweepArgs& a, float2* state_out, hipStream_t s);
// Mirror-paired column kernel of the packed sampler (powers of two).
hipError_t launch_col_pack(int W, int H, const SweepArgs& a, hipStream_t s);
// Zero n 4-byte words (a kernel, so that captured graphs hold no memset node).
hipError_t launch_zero_words(void* p, int64_t n_words, hipStream_t s);
// flag[0] = min(flag[0], problem) for every item whose field (H x W elements
// of the given storage) holds a NaN or an infinity.
hipError_t launch_finite_check(int W, int H, const SweepArgs& a, int32_t* flag, hipStream_t s);
hipError_t launch_fill_int(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// Loss terms of a band-spectrum problem at s (one item per problem, d and s
// concatenated, d already divided by the response): per item FP64 partial
// sums of N_eff^-1 (d - s)^2 and (s - s_true)^2 into part[item][block][2],
// grad_s = s - s_true and grad_d = N_eff^-1 (d - s) (both concatenated).
constexpr int kLossBlocks = 64;
hipError_t launch_loss_terms(int W, int H, const SweepArgs& a, const float* d, const float* s_wf,
                             const float* s_true, float* grad_s, float* grad_d, double* part, hipStream_t s);
// loss[prob] = sum of the item's partials / 2 + the band terms
// 1/2 sum_b (power_b / (n^2 theta_b) + m_b ln(n theta_b)); grad_bands[b] +=
// -1/2 power_b / (n^2 theta_b^2) + m_b / (2 theta_b).
hipError_t launch_loss_finish(const SweepArgs& a, const double* part, const double* power, const double* amps,
                              const int32_t* band_modes, const int32_t* band_base, const int32_t* band_count,
                              double* loss, double* grad_bands, hipStream_t s);
// dof[b] = max(0, modes[b] + prior_dof) for b < n.
hipError_t launch_band_dof(const int32_t* modes, int32_t prior_dof, int32_t* dof, int n, hipStream_t s);
// y[i] += x[i] (float) for i < n.
hipError_t launch_add(const float* x, float* y, int64_t n, hipStream_t s);

}  // namespace mf
