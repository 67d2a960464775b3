/*
 * mf.h - messenger-field Wiener filter and Wiener-posterior sampler for
 *        AMD Instinct MI355X (gfx950).
 *
 * The method (Jeffrey, Heavens & Fortio, "Fast Sampling from Wiener Posteriors
 * for Image Data with Dataflow Engines"):
 *   data model d = A s + n with A = I or a diagonal response (Sec. 1.1, Eq. 1,
 *   and Algorithm 1's A_i terms; mass mapping uses the spin-2 operator of
 *   Sec. 5, see mf_shear_wiener); diagonal pixel noise
 *   covariance N, missing pixels having infinite variance (Sec. 1.1); a
 *   statistically homogeneous signal whose covariance S is diagonal in Fourier
 *   space with an isotropic power spectrum P(|k|) (Eq. 8-9).  The Wiener filter
 *   s_W = S (S + N)^-1 d (Eq. 2-3) is the mean of the Wiener posterior (Eq. 7);
 *   Algorithm 1 (Sec. 2.2) draws posterior samples with a messenger field t of
 *   covariance T = tau I, tau = min N, alternating a pixel-space draw of t and a
 *   Fourier-space draw of s; with its Gaussian variates set to zero the same
 *   iteration converges to s_W (Sec. 2.2).
 *
 * Conventions used throughout:
 *   - images are H x W, row-major, float32; several problems are concatenated
 *     in one array in problem order (mf_plan_pixel_offset gives the offsets);
 *   - wavenumbers are integer grid indices, |k| = sqrt(kx^2 + ky^2); P is in the
 *     synthesis convention s_x = sum_k s_k exp(+2 pi i k.x/N), <|s_k|^2> = P;
 *   - tau = min N_i over observed pixels (1 if none is observed); a cooling
 *     level lambda >= 1 uses T = lambda tau with Nbar = N - tau fixed, whose fixed
 *     point is the Wiener filter for noise N + (lambda - 1) tau;
 *   - two chains travel as the real and imaginary parts of one complex field
 *     (a "pair"); chain 2p is Re and chain 2p+1 is Im of pair p;
 *   - Gaussian variates come from Philox4x32-10 with Box-Muller (Sec. 3.2 uses
 *     Box-Muller on the CPU): key = (seed lo, seed hi), counter =
 *     (elem >> 1, global sweep, (problem << 8) | stage, pair); words (x0,x1)
 *     feed element 2j and (x2,x3) element 2j+1; u1 = ((x>>8)+1) 2^-24,
 *     u2 = (x>>8) 2^-24, z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = ... sin(...).
 *     stage 0 = pixel draw of t (elem = row-major pixel), stage 1 = Fourier
 *     draw of s (elem = row-major mode index in unshifted FFT order), stage 2 =
 *     dispersed initial state, stage 3 = chi-square variates of the
 *     power-spectrum draw (mf_sample_spectrum).  The stream does not depend on
 *     how the work is tiled or batched, so every execution form yields the
 *     same samples.
 *
 * Memory: every pointer argument documented "device" is memory on the current
 * HIP device owned by the caller; the plan owns its own tables and workspaces
 * and frees them in mf_plan_destroy.  mf_plan_create allocates the tables;
 * mf_plan_reserve allocates the workspaces of the calls it names.  A call
 * whose workspaces were reserved allocates nothing; a call that needs more
 * than was reserved allocates it on first use, except on a stream that is
 * being captured into a graph, where it fails with MF_ERR_INVALID_ARG
 * instead.  "host" pointers are read during the call only.
 *
 * Asynchrony: every entry point enqueues its kernels on `stream` (a
 * hipStream_t; NULL is the null stream).  Work lists and cooling levels are
 * built on the device or passed in kernel arguments, so mf_sample,
 * mf_sample_spectrum, mf_shear_sample (check_finite = 0), mf_wiener and
 * mf_wiener_backward (tol <= 0, info NULL), mf_wiener_backward_unrolled,
 * mf_band_power, mf_band_loss (tol <= 0, info NULL) and mf_sample_moments
 * neither allocate (after mf_plan_reserve) nor synchronise, and can be
 * captured into a caller's HIP graph.  A call synchronises `stream` only to
 * return a result to the host: mf_info, a convergence test (tol > 0), the
 * non-finite check of the samplers (check_finite = 1), and the table upload
 * of mf_plan_create / mf_plan_set_spectrum.  A plan must not be used from two
 * streams or threads at once.
 *
 * Errors: every entry point returns an mf_status; no C++ exception crosses the
 * boundary.  mf_last_error() returns a thread-local message for the last
 * failure on the calling thread.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_plan_s* mf_plan;
typedef void* mf_stream; /* hipStream_t */

typedef enum {
    MF_OK = 0,
    MF_ERR_INVALID_ARG = 1,      /* a pointer, size, variance or count is invalid */
    MF_ERR_UNSUPPORTED_SIZE = 2, /* H or W outside the supported sides (see mf_problem), or a form that the size
                                    does not support */
    MF_ERR_OUT_OF_MEMORY = 3,    /* a plan table or workspace could not be allocated */
    MF_ERR_DEVICE = 4,           /* a HIP runtime call failed */
    MF_ERR_NOT_CONVERGED = 5,    /* tol > 0 not reached within max_sweeps (result still written) */
    MF_ERR_NONFINITE = 6         /* a solve's residual test saw NaN/Inf (that problem stops; outputs written), or
                                    a sampler's non-finite check found a chain state holding NaN/Inf */
} mf_status;

/* Power spectrum P(|k|) of the signal (Eq. 9). */
enum { MF_PK_POWERLAW = 0, MF_PK_BANDS = 1 };
typedef struct {
    int32_t kind;              /* MF_PK_POWERLAW or MF_PK_BANDS */
    double amp, k0, n;         /* powerlaw: P(k) = amp * (k + k0)^(-n), P > 0 everywhere */
    int32_t n_bands;           /* bands: P(k) = band_amps[b] for band_edges[b] <= k < band_edges[b+1] */
    const double* band_edges;  /* host, n_bands + 1 increasing values; the last band is closed */
    const double* band_amps;   /* host, n_bands values > 0 */
} mf_spectrum;

/* One image problem, d = A s + n (Eq. 1) with a diagonal A. */
typedef struct {
    int32_t H, W;              /* image size; each an even 2^a 3^b in [16, 2048] (the transforms of Eq. 8
                                  run as radix-16/8/4/2 and radix-3 passes).  Sides with a factor 3 run on
                                  the streamed kernels (the persistent form needs H = W in {32, 64, 128});
                                  mf_sample_spectrum and mass mapping need powers of two */
    const float* noise_var;    /* host, H*W: N_i > 0, +INFINITY marks a missing pixel */
    mf_spectrum spectrum;
    const float* response;     /* host, H*W: the diagonal of A (finite; 0 = a pixel without
                                  response), or NULL for A = I.  Algorithm 1's definitions
                                  then use tau = min N_i / A_i^2 and Nbar_i = N_i - tau A_i^2;
                                  every entry point takes d and returns dL/dd in the units of
                                  the data, and the plan works with d_i / A_i and N_i / A_i^2 */
} mf_problem;

/* Cooling schedule of the Wiener filter (zero-variate Algorithm 1).
 * Level j runs sweeps[j] sweeps at T = lambda[j] tau.  Then, if tol > 0, the
 * last level continues until the residual r = ||t_k - t_{k-1}|| / (T ||b||)
 * (b = N_eff^-1 d, so r = ||(S^-1 + N_eff^-1) s - b|| / ||b||) is <= tol,
 * tested on sweeps whose global count is a multiple of check_every, or until
 * max_sweeps sweeps have run in total. */
typedef struct {
    int32_t n_levels;          /* >= 1 */
    const double* lambda;      /* host, n_levels values >= 1 (the last is normally 1) */
    const int32_t* sweeps;     /* host, n_levels values >= 0 */
    double tol;                /* <= 0: no convergence phase */
    int32_t max_sweeps;        /* total cap when tol > 0 */
    int32_t check_every;       /* >= 2 when tol > 0 */
} mf_schedule;

/* Per-problem outcome of an iterative solve (host). */
typedef struct {
    int32_t sweeps;            /* sweeps run */
    int32_t converged;         /* 1 if tol was reached (or tol <= 0) */
    double residual;           /* last tested residual, NaN if none was tested */
} mf_info;

/* Execution forms of the sampler. */
enum {
    MF_FORM_AUTO = 0,          /* persistent LDS-resident kernel where the image fits, else streamed */
    MF_FORM_PERSISTENT = 1,    /* one launch runs every sweep of every chain pair (H = W <= 128) */
    MF_FORM_STREAMED = 2,      /* two kernels per sweep over all pairs, field in HBM between them */
    MF_FORM_PLAIN = 3          /* one chain pair at a time, per-sweep kernels, no batching */
};

/* Plan flags. */
enum {
    MF_FLAG_NONE = 0,
    MF_FLAG_AUTOTUNE = 1,      /* time the column-tile shapes and the fused row kernel's rows per workgroup
                                  of each streamed size class (sides >= 256) at plan creation and keep the
                                  fastest of each; with MF_TUNE_CACHE=<file> in the environment the
                                  choices are read from / appended to that file */
    MF_FLAG_GRAPH = 2,         /* capture the streamed sweep loops of each size class (mf_sample,
                                  mf_sample_spectrum, mf_shear_wiener, mf_shear_sample) as HIP graphs,
                                  once per launch configuration (pointers, counts, seeds, sweep range,
                                  schedule), and replay them; the plan keeps up to 8 graphs */
    MF_FLAG_STREAMED_SOLVE = 4, /* run mf_wiener / mf_wiener_backward on the streamed kernels for every size
                                  class; without it, classes with H = W in {32, 64, 128} use the persistent
                                  solve kernel (one workgroup per problem, every level and the residual
                                  test on the device, no host synchronisation per check) */
    MF_FLAG_INF_AS_1E8 = 8     /* give missing pixels (noise +inf, or response 0) the noise variance 1e8,
                                  the finite stand-in for infinite noise of Sec. 3.2, instead of the exact
                                  limit a = 0; the results differ by O(T / 1e8) */
};

/* Storage of the streamed sampler's pair field in HBM between its two kernels
 * per sweep (the reduced-bitwidth trade-off of Sec. 3.2).  Arithmetic
 * stays FP32: each kernel widens what it loads and rounds (to nearest even)
 * what it stores, so a sweep adds two roundings of the field, one after the
 * row transforms and one after the column transforms.  Applies to the streamed
 * and plain forms; the persistent form keeps the field in registers and
 * ignores it.  state_in / state_out and the samples stay FP32.  FP16 holds
 * magnitudes up to 65504: the row-transformed field reaches W times the
 * largest |t| of a row, so data and signal must be scaled well inside that
 * (values of order 1 are fine up to 2048 columns); BF16 has FP32's range and
 * an 8-bit significand. */
enum {
    MF_STORAGE_FP32 = 0,       /* 8 bytes per pixel per chain pair (default) */
    MF_STORAGE_FP16 = 1,       /* 4 bytes: IEEE binary16 pairs, unit roundoff 2^-11 */
    MF_STORAGE_BF16 = 2        /* 4 bytes: bfloat16 pairs, unit roundoff 2^-8 */
};

/* Arguments of mf_sample. */
typedef struct {
    uint64_t seed;             /* Philox key */
    int32_t chains_per_problem;/* >= 1; pairs = ceil(chains / 2), an odd count drops the last Im chain */
    int32_t burn_in;           /* sweeps before the first sample (>= 0) */
    int32_t n_samples;         /* samples per chain (>= 0) */
    int32_t thin;              /* sweeps per sample after burn-in (>= 1) */
    int64_t sweep_offset;      /* global sweep index of the first sweep (for resuming a chain) */
    float init_scale;          /* > 0: start from init_scale * stage-2 normals (ignored if state_in) */
    int32_t form;              /* MF_FORM_* */
    int32_t storage;           /* MF_STORAGE_*: precision of the streamed field between kernels */
    int32_t check_finite;      /* 1: after the run, synchronise and return MF_ERR_NONFINITE if a chain's final
                                  state holds NaN or Inf (a non-finite value anywhere in a chain's history reaches
                                  its final state: every sweep mixes all pixels through the transforms); the
                                  samples and states are still written.  0: no check, no synchronisation */
    const mf_schedule* cooling;/* host, or NULL: levels (lambda_j >= 1, sweeps_j) run before the burn-in,
                                  sampling with T = lambda_j tau (the posterior for noise
                                  N + (lambda_j - 1) tau), global sweep indices sweep_offset, ...; the
                                  burn-in then starts at sweep_offset + sum_j sweeps_j.  tol is ignored.
                                  These sweeps run on the streamed kernels for every form. */
} mf_sample_args;

/* Arguments of mf_sample_spectrum. */
typedef struct {
    uint64_t seed;             /* Philox key */
    int32_t chains_per_problem;/* >= 1; pairs = ceil(chains / 2) */
    int32_t burn_in;           /* iterations before the first sample (>= 0) */
    int32_t n_samples;         /* samples per chain (>= 0) */
    int32_t thin;              /* iterations per sample after burn-in (>= 1) */
    int32_t sweeps_per_draw;   /* messenger sweeps per iteration, before each spectrum draw (>= 1) */
    int32_t prior_dof;         /* nu_0: inverse-gamma prior of shape nu_0/2 on each band amplitude */
    double prior_beta;         /* beta_0 >= 0: its scale (nu_0 = beta_0 = 0: Jeffreys' 1/theta) */
    int64_t iteration_offset;  /* global index of the first iteration (for resuming a chain) */
    float init_scale;          /* > 0: dispersed start as in mf_sample (ignored if state_in) */
    int32_t check_finite;      /* as in mf_sample_args (the chains' final signal states are checked) */
} mf_spectrum_args;

/* Create a plan for n_problems problems (Algorithm 1's definitions: tau, Nbar,
 * n P(|k|) evaluated in FP64 and stored in FP32, FFT twiddles evaluated in FP64).
 * Copies all tables to the current device.  *out receives the plan. */
mf_status mf_plan_create(mf_plan* out, int32_t n_problems, const mf_problem* problems,
                         uint32_t flags, mf_stream stream);

/* Release the plan and every device buffer it owns. NULL is accepted. */
mf_status mf_plan_destroy(mf_plan plan);

/* Workspace reservation: the calls named in `calls`, with at most
 * chains_per_problem chains (samplers, moments), the given storage (mf_sample)
 * and at most unrolled_sweeps sweeps with a checkpoint every checkpoint_every
 * (mf_wiener_backward_unrolled), will allocate nothing.  Workspaces are sized
 * for every problem of the plan at once (the sampler's work field included,
 * for calls without state_out), kept until mf_plan_destroy and never shrunk;
 * a later reservation only grows them.  Allocates synchronously (no stream). */
enum {
    MF_RESERVE_SOLVE = 1,      /* mf_wiener, mf_wiener_backward, mf_band_power, mf_band_loss */
    MF_RESERVE_SAMPLE = 2,     /* mf_sample */
    MF_RESERVE_SPECTRUM = 4,   /* mf_sample_spectrum */
    MF_RESERVE_SHEAR = 8,      /* mf_shear_wiener, mf_shear_sample */
    MF_RESERVE_UNROLLED = 16,  /* mf_wiener_backward_unrolled */
    MF_RESERVE_MOMENTS = 32    /* mf_sample_moments */
};
typedef struct {
    uint32_t calls;            /* MF_RESERVE_* bits */
    int32_t chains_per_problem;/* >= 1 when a sampler or moments bit is set */
    int32_t storage;           /* MF_STORAGE_* of the mf_sample calls */
    int32_t unrolled_sweeps;   /* K >= 1 with MF_RESERVE_UNROLLED */
    int32_t checkpoint_every;  /* C >= 1 with MF_RESERVE_UNROLLED */
} mf_reserve;
mf_status mf_plan_reserve(mf_plan plan, const mf_reserve* reserve);

/* Replace the spectrum of one problem (same kind and band count for bands).
 * Used by gradient-based training loops over band amplitudes.  The new tables
 * (n P(|k|) evaluated in FP64, Eq. 9) are copied on `stream`, after the work
 * already queued there, and the call synchronises `stream` before it returns. */
mf_status mf_plan_set_spectrum(mf_plan plan, int32_t problem, const mf_spectrum* spectrum, mf_stream stream);

/* Element offset of problem p in concatenated image arrays (p == n_problems
 * gives the total pixel count); -1 on a bad argument. */
int64_t mf_plan_pixel_offset(mf_plan plan, int32_t problem);

/* tau of problem p (host copy), or -1 on a bad argument. */
double mf_plan_tau(mf_plan plan, int32_t problem);

/* Wiener filter of every problem (Algorithm 1 with G(0,1) -> 0, Sec. 2.2).
 *   d       device, concatenated float32 data (values on missing pixels are ignored)
 *   s_init  device, concatenated start (NULL: zero); may be s_out
 *   s_out   device, concatenated result
 *   info    host array of n_problems entries, or NULL (then no host sync unless tol > 0)
 * The convergence phase (tol > 0) runs at the last level and tests, every
 * check_every sweeps (never on the first sweep of the phase), the residual
 * ||t_k - t_{k-1}|| / (T ||b||) of Sec. 2.2 in FP64, b = N_eff^-1 d at that level.
 * Returns MF_ERR_NOT_CONVERGED if any problem missed tol (s_out still holds the
 * last iterate), MF_ERR_NONFINITE if a tested residual was NaN or Inf (NaN in
 * the data of an observed pixel, say); that problem's iteration stops there. */
mf_status mf_wiener(mf_plan plan, const float* d, const mf_schedule* schedule,
                    const float* s_init, float* s_out, mf_info* info, mf_stream stream);

/* Draw posterior samples (Algorithm 1).
 *   d            device, concatenated float32 data
 *   state_in     device, complex pair states [problem][pair][H][W] (float2), or NULL
 *   state_out    device, same layout, final states, or NULL
 *   samples_out  device, float32 [problem][chain][sample][H][W] concatenated over
 *                problems (problem p starts at chains * n_samples * pixel_offset(p)), or NULL
 */
mf_status mf_sample(mf_plan plan, const float* d, const mf_sample_args* args,
                    const float* state_in, float* state_out, float* samples_out,
                    mf_stream stream);

/* mf_sample for callers that cannot allocate device memory: code under HIP
 * graph capture without a prior mf_plan_reserve, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments and results as mf_sample
 * (the same kernels, bit for bit), but every workspace (work lists,
 * persistent coefficient tables, d / A with a response, the 16-bit field)
 * lives in a static device array of 16 MiB per GPU, held until the process
 * ends, and the call allocates nothing (no hipMalloc, no graph instantiation:
 * MF_FLAG_GRAPH is ignored).  state_out is required (it holds the chains' work
 * field).  MF_ERR_INVALID_ARG if the plan and call need more than 16 MiB (for
 * example more than about 800,000 pixels of persistent-form problems, or the
 * 16-bit field of a large streamed plan) or if the plan's device is not
 * current.  Every call on one GPU shares that GPU's array and overwrites it:
 * calls that overlap on one GPU (two streams, two threads) race. */
mf_status mf_sample_noalloc(mf_plan plan, const float* d, const mf_sample_args* args,
                            const float* state_in, float* state_out, float* samples_out, mf_stream stream);

/* Hierarchical sampler (Sec. 5): samples of the signal and of the band
 * amplitudes theta_b of the power spectrum.  Every problem needs a band
 * spectrum (MF_ERR_INVALID_ARG otherwise).  Size classes with H = W in {32,
 * 64, 128} run one persistent kernel per call; every other size class runs
 * the streamed kernels (one row and one column launch per sweep, two more per
 * iteration), whose per-item amplitude sums live in a plan workspace that is
 * allocated on first use.  Iteration i (global g = iteration_offset
 * + i) runs sweeps_per_draw sweeps of Algorithm 1 (global sweep indices
 * g * sweeps_per_draw + k) with the current amplitudes, then draws each band
 * amplitude from its conditional given the signal,
 *     theta_b | s ~ InvGamma((m_b + nu_0)/2, beta_0 + sigma_b / (2 n^2)),
 * m_b the modes of band b, sigma_b = sum_{k in b} |s_k|^2 (unnormalised DFT);
 * the draw is (2 beta_0 + sigma_b / n^2) / x with x the sum of m_b + nu_0
 * squared normals from stream stage 3 (a band with no degrees of freedom, or
 * a zero sum, keeps its amplitude).  Each chain has its own amplitudes.  A
 * sample is (s, theta) after iteration i when i >= burn_in and (i - burn_in +
 * 1) is a multiple of thin.
 *   d                  device, concatenated float32 data
 *   state_in/out       device, pair states as in mf_sample, or NULL
 *   theta_in/out       device float64 [problem][2 * pairs][band] (problem p starts at
 *                      2 * pairs * band_base(p), band_base = the problem's first band
 *                      in plan order), or NULL; theta_in NULL starts from the plan's
 *                      amplitudes
 *   samples_out        device float32, as in mf_sample, or NULL
 *   theta_samples_out  device float64 [problem][chain][sample][band] (problem p starts at
 *                      chains * n_samples * band_base(p)), or NULL */
mf_status mf_sample_spectrum(mf_plan plan, const float* d, const mf_spectrum_args* args,
                             const float* state_in, const double* theta_in, float* state_out,
                             double* theta_out, float* samples_out, double* theta_samples_out,
                             mf_stream stream);

/* Arguments of mf_shear_sample. */
typedef struct {
    uint64_t seed;             /* Philox key */
    int32_t chains_per_problem;/* >= 1; one chain per stream index (no pairing) */
    int32_t burn_in;           /* sweeps before the first sample (>= 0) */
    int32_t n_samples;         /* samples per chain (>= 0) */
    int32_t thin;              /* sweeps per sample after burn-in (>= 1) */
    int64_t sweep_offset;      /* global sweep index of the first sweep */
    float b_ratio;             /* P_B / P_E >= 0 (0: no B modes) */
    int32_t check_finite;      /* as in mf_sample_args (the chains' final states A kappa are checked) */
} mf_shear_args;

/* Mass mapping (Sec. 5): complex shear data gamma = A kappa + n with the
 * spin-2 operator A = F^-1 D F, D_k = (k_1 + i k_2)^2 / |k|^2 (k_1 along x,
 * integer frequencies in FFT order; D_0 = 0), convergence kappa = kappa_E + i
 * kappa_B with the problem's spectrum as P_E and P_B = b_ratio P_E, noise
 * variance noise_var per component.  The messenger field lives in shear
 * space (T = tau I, tau = min N); the Fourier step removes D and applies the
 * Wiener step of each real field (E = real part, B = imaginary part of
 * kappa); k = 0 is drawn from the prior.  Problems take no response
 * (MF_ERR_INVALID_ARG).  Size classes with H = W in {32, 64, 128} run one
 * persistent kernel per call; every other class runs the streamed kernels
 * (a row and a mirror-paired column launch per sweep, plus one row launch per
 * emitted kappa), whose staging field is a plan workspace allocated on first
 * use.
 *   gamma       device, concatenated complex shear (float2 per pixel)
 *   kappa_out   device, concatenated complex convergence (float2 per pixel)
 * mf_shear_wiener runs the schedule's sweeps from kappa = 0 (tol must be <= 0)
 * and writes kappa after the last sweep.  mf_shear_sample draws samples of
 * kappa, float2 [problem][chain][sample][H][W] (problem p starts at chains *
 * n_samples * pixel_offset(p)); its state is the model shear A kappa per
 * chain, float2 [problem][chain][H][W]. */
mf_status mf_shear_wiener(mf_plan plan, const float* gamma, const mf_schedule* schedule, float b_ratio,
                          float* kappa_out, mf_stream stream);
mf_status mf_shear_sample(mf_plan plan, const float* gamma, const mf_shear_args* args,
                          const float* state_in, float* state_out, float* samples_out, mf_stream stream);

/* Per-pixel mean and variance of posterior samples (the maps of Sec. 4.1,
 * Fig. 3) over all chains and samples of every problem.
 *   samples    device float32 [problem][chain][sample][H][W], as written by mf_sample
 *              or mf_sample_spectrum with the same chains and n_samples
 *   mean_out   device float64, concatenated images
 *   var_out    device float64, concatenated images (unbiased, over chains * n_samples
 *              values; 0 when there is one value), or NULL
 * Sums are shifted by each pixel's first sample and accumulated in FP64. */
mf_status mf_sample_moments(mf_plan plan, const float* samples, int32_t chains, int32_t n_samples,
                            double* mean_out, double* var_out, mf_stream stream);

/* Vector-Jacobian product of the Wiener-filter map (d, P) -> s_W by implicit
 * differentiation of the normal equations (S^-1 + N^-1) s_W = N^-1 d read off
 * Eq. 7: v solves (S^-1 + N^-1) v = grad_s by the messenger iteration (pixel
 * step t = (1 - a) v + T grad_s), then
 *   grad_d     = A^T N^-1 v (0 on missing pixels; N^-1 v when A = I) device, concatenated
 *   grad_bands = sum_{k in b} Re(conj(v_k) s_k) / (n^2 theta_b^2)  device float64,
 *                bands of every band-spectrum problem concatenated (NULL allowed)
 * with v_k, s_k the unnormalised DFTs of v and s_wf.  grad_bands needs s_wf.
 *   s_wf, grad_s device, concatenated;  v_out device or NULL (the adjoint field).
 */
mf_status mf_wiener_backward(mf_plan plan, const float* s_wf, const float* grad_s,
                             const mf_schedule* schedule, float* grad_d, double* grad_bands,
                             float* v_out, mf_info* info, mf_stream stream);

/* Gradient of a truncated Wiener iteration ("unrolled" mode).  s_K is the
 * result of the schedule's sweeps (tol must be <= 0: a fixed sweep count,
 * cooling levels included) from s_0 = 0.  The call re-runs those sweeps, keeping
 * the state every checkpoint_every sweeps, then runs the transposed sweeps in
 * reverse (sweep k maps t_k = (1 - a_k) s_{k-1} + a_k d, s_k = F^-1 f_k F t_k;
 * its transpose filters by f_k, then scales by 1 - a_k), recomputing each
 * segment from its checkpoint and storing that segment's transforms F t_k:
 *   grad_d     = dL/dd                                   device, concatenated
 *   grad_bands = dL/dtheta for band-spectrum problems    device float64, or NULL
 *                (sum over sweeps and over modes of the band of
 *                 Re(conj(F sbar_k) F t_k) T_k / (n P_k + T_k)^2)
 *   s_out      = s_K                                     device, or NULL
 * for dL/ds_K = grad_s (device, concatenated).  Workspace: (ceil(K/C) + C + 2)
 * complex fields per size class, allocated by the plan on first use. */
mf_status mf_wiener_backward_unrolled(mf_plan plan, const float* d, const mf_schedule* schedule,
                                      int32_t checkpoint_every, const float* grad_s, float* s_out,
                                      float* grad_d, double* grad_bands, mf_stream stream);

/* Loss of the differentiation workload for band-spectrum problems (every
 * problem of the plan must have one), at the Wiener filter s = s_wf (Eq. 2-3):
 *   L_p = 1/2 s^T S^-1 s + 1/2 (d - A s)^T N^-1 (d - A s) + 1/2 sum_k ln(n P_k)
 *         + 1/2 ||s - s_true||^2,
 * the negative log-posterior of Eq. 5-7 up to constants plus an L2 distance to
 * a reference field, with the plan's own N (its response A, and 1e8 on missing
 * pixels under MF_FLAG_INF_AS_1E8; pixels without data or response carry no
 * likelihood term).  With P_k = theta_b on band b, s^T S^-1 s =
 * sum_b sigma_b / (n^2 theta_b) and sum_k ln(n P_k) = sum_b m_b ln(n theta_b)
 * (sigma_b the band power of the unnormalised DFT of s, m_b the band's modes).
 * Gradients (NULL: not computed) with respect to d and the band amplitudes:
 * explicit terms plus, through s_W, the implicit VJP of mf_wiener_backward for
 * dL/ds = s - s_true (the log-posterior part is stationary at s_W), solved with
 * adjoint_schedule.
 *   d, s_wf, s_true  device, concatenated (s_wf from mf_wiener with the same plan)
 *   loss_out         device float64 [n_problems]
 *   grad_d           device, concatenated, or NULL
 *   grad_bands       device float64 [mf_plan_total_bands], or NULL
 *   info             host [n_problems] outcome of the adjoint solve, or NULL
 * Returns MF_ERR_NOT_CONVERGED if the adjoint missed its tol (outputs written). */
mf_status mf_band_loss(mf_plan plan, const float* d, const float* s_wf, const float* s_true,
                       const mf_schedule* adjoint_schedule, double* loss_out, float* grad_d, double* grad_bands,
                       mf_info* info, mf_stream stream);

/* Band cross-power sum_{k in b} Re(conj(x_k) y_k) of two concatenated real
 * fields (unnormalised DFTs) for every band-spectrum problem; device float64 out. */
mf_status mf_band_power(mf_plan plan, const float* x, const float* y, double* out,
                        mf_stream stream);

/* Column-kernel tile of the streamed size class H x W in use by the plan (the
 * autotuner's choice under MF_FLAG_AUTOTUNE, else the default): *cols columns
 * per workgroup of *threads threads.  MF_ERR_INVALID_ARG if the plan has no
 * problem of that size. */
mf_status mf_plan_tile_shape(mf_plan plan, int32_t H, int32_t W, int32_t* cols, int32_t* threads);

/* Rows per workgroup of the fused streamed row kernel (rows of 256 points and
 * more, powers of two) for the size class H x W: the autotuner's choice under
 * MF_FLAG_AUTOTUNE, else the default; 0 where no fused row kernel runs.
 * MF_ERR_INVALID_ARG if the plan has no problem of that size. */
mf_status mf_plan_row_shape(mf_plan plan, int32_t H, int32_t W, int32_t* rows);

/* Shapes of the size class H x W for launches too small to fill the GPU: a
 * launch whose grid in the shapes above would have fewer workgroups than the
 * GPU has compute units (256; a single Wiener solve or adjoint of a 256^2 or
 * 512^2 image, a few chains) uses these instead.  Under MF_FLAG_AUTOTUNE they
 * are timed on one work item; otherwise they are the candidates with the most
 * workgroups.  *cols x *threads: column tile; *rows: rows per workgroup of the
 * fused row kernel (0 where none runs).  Every shape computes the same values
 * bit for bit.  MF_ERR_INVALID_ARG if the plan has no problem of that size. */
mf_status mf_plan_narrow_shape(mf_plan plan, int32_t H, int32_t W, int32_t* cols, int32_t* threads,
                               int32_t* rows);

/* Number of bands over all band-spectrum problems (length of grad_bands). */
int32_t mf_plan_total_bands(mf_plan plan);

const char* mf_status_string(mf_status status);
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
