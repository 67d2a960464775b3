// Host side of the messenger-field library: plan creation (Algorithm 1's
// definitions evaluated in FP64), the sweep-loop drivers of every execution
// form, and the C entry points declared in mf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "mf_kernels.hpp"
#include "mf_resident.hpp"
#include "mf_spectrum.hpp"
#include "mf_shear.hpp"
#include "mf_static.hpp"

namespace {

thread_local std::string g_last_error;

mf_status fail(mf_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

#define MF_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(MF_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
// Image sides: 2^a 3^b with a >= 1 (even, so that pixel and mode pairs stay
// within a row) in [16, 2048]; the DFT of Eq. 8 runs as radix-16/8/4/2 and
// radix-3 passes.
bool size_ok(int v) {
    if (v < 16 || v > 2048 || (v & 1)) return false;
    while (v % 2 == 0) v /= 2;
    while (v % 3 == 0) v /= 3;
    return v == 1;
}
// The hierarchical sampler and mass mapping (the extensions of Sec. 5) run
// on power-of-two sides only.
mf_status pow2_sides(mf_plan p, const char* what);

struct HostProblem {
    int H = 0, W = 0;
    int64_t pix_off = 0;
    double tau = 1.0;
    int kind = MF_PK_POWERLAW;
    int n_bands = 0;
    int band_base = 0;
    std::vector<double> edges, amps;
    std::vector<int32_t> band_modes;  // modes per band (band spectra)
    double amp = 1, k0 = 1, n = 2;
};

// A device buffer that grows on demand and is freed with the plan.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace

struct mf_plan_s {
    int device = 0;
    uint32_t flags = 0;
    std::vector<HostProblem> probs;
    int64_t total_px = 0;
    int total_bands = 0;
    // (H, W) -> problems of that size, in problem order
    std::map<std::pair<int, int>, std::vector<int>> classes;
    // device tables
    mf::ProbDev* d_probs = nullptr;
    float* d_nbar = nullptr;
    float* d_nP = nullptr;
    float2* d_nPt = nullptr;  // column-pair copy of nP for the streamed column kernel
    int16_t* d_band = nullptr;
    int16_t* d_bandt = nullptr;  // the band map column-major per problem: [pix_off + kx H + ky]
    int32_t* d_band_base = nullptr;
    int32_t* d_band_count = nullptr;
    double* d_band_scale = nullptr;  // 1 / (n^2 theta_b^2)
    std::map<int, float2*> d_tw;     // W_L^r for every transform length L
    // workspaces
    DevBuf items, field, t_save, partials, aux, coef;
    DevBuf field_adj, ckpt, tstore, slots;  // unrolled-gradient workspaces
    DevBuf sched;                           // persistent solve: levels, sweeps, per-item outcome
    DevBuf spec;                            // hierarchical sampler: dof and start amplitudes per band
    DevBuf hier;                            // streamed hierarchical sampler: per-item amplitudes and sums
    DevBuf hfield;                          // streamed sampler field in FP16 / BF16 storage
    DevBuf kfield;                          // streamed mass mapping: kappa staging field
    // column-kernel tile shape per size class: (H, W) -> (tc, nth)
    std::map<std::pair<int, int>, std::pair<int, int>> col_shape;
    std::map<std::pair<int, int>, std::pair<int, int>> col_shape_narrow;  // tuned on one item
    std::map<std::pair<int, int>, int> row_rows_narrow;
    // rows per block of the fused row kernel per size class (absent: default)
    std::map<std::pair<int, int>, int> row_rows;
    // captured sweep loops of the streamed sampler, keyed by launch configuration
    struct GraphEntry {
        std::vector<uint64_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    std::vector<float> host_nbar;    // for residual norms
    bool has_response = false;       // some problem has a diagonal A != I
    float* d_rinv = nullptr;         // 1 / A_i per pixel (0 without response), when has_response
    DevBuf dprime;                   // d / A of the current call
    // problem ids per size class (all, then the band-spectrum ones) for work
    // lists built on the device: (H, W) -> (offset in d_class_pids, count)
    int32_t* d_class_pids = nullptr;
    std::map<std::pair<int, int>, std::pair<int, int>> class_all, class_band;
    int32_t* d_band_modes = nullptr;  // modes per band, concatenated
    double* d_band_amps = nullptr;    // the plan's band amplitudes, concatenated
    int32_t* d_flag = nullptr;        // non-finite check: lowest problem index with a non-finite state
    DevBuf lossbuf;                   // mf_band_loss: grad_s, explicit grad_d, partial sums, band powers
    ~mf_plan_s() {
        (void)hipFree(d_probs);
        (void)hipFree(d_nbar);
        (void)hipFree(d_nP);
        (void)hipFree(d_nPt);
        (void)hipFree(d_band);
        (void)hipFree(d_bandt);
        (void)hipFree(d_band_base);
        (void)hipFree(d_band_count);
        (void)hipFree(d_band_scale);
        (void)hipFree(d_rinv);
        (void)hipFree(d_class_pids);
        (void)hipFree(d_band_modes);
        (void)hipFree(d_band_amps);
        (void)hipFree(d_flag);
        dprime.release();
        lossbuf.release();
        for (auto& kv : d_tw) (void)hipFree(kv.second);
        items.release();
        field.release();
        t_save.release();
        partials.release();
        aux.release();
        coef.release();
        field_adj.release();
        ckpt.release();
        tstore.release();
        slots.release();
        sched.release();
        spec.release();
        hier.release();
        hfield.release();
        kfield.release();
        for (auto& g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

mf_status read_finite_flag(mf_plan p, hipStream_t s);

// P(|k|) of one problem, evaluated in FP64 (Eq. 9).
double spectrum_at(const HostProblem& p, double k) {
    if (p.kind == MF_PK_POWERLAW) return p.amp * std::pow(k + p.k0, -p.n);
    const int nb = p.n_bands;
    for (int b = 0; b < nb; ++b) {
        const bool in = k >= p.edges[b] && (k < p.edges[b + 1] || (b == nb - 1 && k <= p.edges[b + 1]));
        if (in) return p.amps[b];
    }
    return 0.0;
}

int band_of(const HostProblem& p, double k) {
    const int nb = p.n_bands;
    for (int b = 0; b < nb; ++b)
        if (k >= p.edges[b] && (k < p.edges[b + 1] || (b == nb - 1 && k <= p.edges[b + 1]))) return b;
    return -1;
}

double kmag(int ky_idx, int kx_idx, int H, int W) {
    const double ky = ky_idx < H - H / 2 ? ky_idx : ky_idx - H;  // numpy fftfreq * N order
    const double kx = kx_idx < W - W / 2 ? kx_idx : kx_idx - W;
    return std::sqrt(ky * ky + kx * kx);
}

mf_status copy_spectrum(HostProblem& hp, const mf_spectrum& s, int pidx) {
    hp.kind = s.kind;
    if (s.kind == MF_PK_POWERLAW) {
        if (!(s.amp > 0) || !std::isfinite(s.amp) || !std::isfinite(s.k0) || !std::isfinite(s.n) || s.k0 <= 0)
            return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(pidx) + ": power law needs amp > 0, k0 > 0");
        hp.amp = s.amp;
        hp.k0 = s.k0;
        hp.n = s.n;
        hp.n_bands = 0;
        return MF_OK;
    }
    if (s.kind != MF_PK_BANDS) return fail(MF_ERR_INVALID_ARG, "unknown spectrum kind");
    if (s.n_bands < 1 || s.n_bands > mf::kMaxBandsPerProblem || !s.band_edges || !s.band_amps)
        return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(pidx) + ": bands need 1..64 bands and arrays");
    hp.n_bands = s.n_bands;
    hp.edges.assign(s.band_edges, s.band_edges + s.n_bands + 1);
    hp.amps.assign(s.band_amps, s.band_amps + s.n_bands);
    for (int b = 0; b < s.n_bands; ++b) {
        if (!(hp.edges[b + 1] > hp.edges[b])) return fail(MF_ERR_INVALID_ARG, "band edges must increase");
        if (!(hp.amps[b] > 0) || !std::isfinite(hp.amps[b])) return fail(MF_ERR_INVALID_ARG, "band amplitudes must be > 0");
    }
    return MF_OK;
}

// Upload n P(|k|) (FP64 -> FP32) for one problem; also its band map, mode
// counts, amplitudes and scales.  The copies are ordered on `stream` after
// the work already queued there, and complete before the call returns.
mf_status upload_spectrum(mf_plan p, int i, hipStream_t stream) {
    HostProblem& hp = p->probs[i];
    hp.band_modes.assign(hp.n_bands, 0);
    const int H = hp.H, W = hp.W;
    const double n = (double)H * W;
    std::vector<float> nP((size_t)H * W);
    std::vector<int16_t> band((size_t)H * W, -1);
    for (int ky = 0; ky < H; ++ky)
        for (int kx = 0; kx < W; ++kx) {
            const double k = kmag(ky, kx, H, W);
            const double P = spectrum_at(hp, k);
            if (!(P > 0) || !std::isfinite(n * P))
                return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": P(k) must be finite and > 0 on every mode");
            nP[(size_t)ky * W + kx] = (float)(n * P);
            if (hp.kind == MF_PK_BANDS) {
                const int b = band_of(hp, k);
                band[(size_t)ky * W + kx] = (int16_t)b;
                if (b >= 0) ++hp.band_modes[b];
            }
        }
    MF_HIP(hipMemcpyAsync(p->d_nP + hp.pix_off, nP.data(), nP.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    // column pairs: entry (kx/2) H + ky holds (nP(ky, kx), nP(ky, kx + 1)) for even kx
    std::vector<float2> nPt((size_t)H * W / 2);
    for (int kx = 0; kx < W; kx += 2)
        for (int ky = 0; ky < H; ++ky)
            nPt[(size_t)(kx / 2) * H + ky] = make_float2(nP[(size_t)ky * W + kx], nP[(size_t)ky * W + kx + 1]);
    MF_HIP(hipMemcpyAsync(p->d_nPt + hp.pix_off / 2, nPt.data(), nPt.size() * sizeof(float2), hipMemcpyHostToDevice,
                          stream));
    MF_HIP(hipMemcpyAsync(p->d_band + hp.pix_off, band.data(), band.size() * sizeof(int16_t), hipMemcpyHostToDevice,
                          stream));
    // column-major copy: a column's modes are contiguous (the row-per-thread
    // Fourier step of the mirror-paired column kernel reads it across rows)
    std::vector<int16_t> bandt((size_t)H * W);
    for (int kx = 0; kx < W; ++kx)
        for (int ky = 0; ky < H; ++ky) bandt[(size_t)kx * H + ky] = band[(size_t)ky * W + kx];
    MF_HIP(hipMemcpyAsync(p->d_bandt + hp.pix_off, bandt.data(), bandt.size() * sizeof(int16_t),
                          hipMemcpyHostToDevice, stream));
    std::vector<double> sc(hp.n_bands);
    if (hp.kind == MF_PK_BANDS) {
        for (int b = 0; b < hp.n_bands; ++b) sc[b] = 1.0 / (n * n * hp.amps[b] * hp.amps[b]);
        MF_HIP(hipMemcpyAsync(p->d_band_scale + hp.band_base, sc.data(), sc.size() * sizeof(double),
                              hipMemcpyHostToDevice, stream));
        MF_HIP(hipMemcpyAsync(p->d_band_amps + hp.band_base, hp.amps.data(), hp.n_bands * sizeof(double),
                              hipMemcpyHostToDevice, stream));
        MF_HIP(hipMemcpyAsync(p->d_band_modes + hp.band_base, hp.band_modes.data(), hp.n_bands * sizeof(int32_t),
                              hipMemcpyHostToDevice, stream));
    }
    MF_HIP(hipStreamSynchronize(stream));  // the host vectors die on return
    return MF_OK;
}

mf_status upload_twiddles(mf_plan p, int L) {
    if (p->d_tw.count(L)) return MF_OK;
    std::vector<float2> tw(L);
    for (int r = 0; r < L; ++r) {
        const double ang = -2.0 * M_PI * (double)r / (double)L;
        tw[r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    float2* d = nullptr;
    MF_HIP(hipMalloc(&d, L * sizeof(float2)));
    p->d_tw[L] = d;
    MF_HIP(hipMemcpy(d, tw.data(), L * sizeof(float2), hipMemcpyHostToDevice));
    return MF_OK;
}

mf_status validate_schedule(const mf_schedule* s) {
    if (!s) return fail(MF_ERR_INVALID_ARG, "schedule is NULL");
    if (s->n_levels < 1 || !s->lambda || !s->sweeps) return fail(MF_ERR_INVALID_ARG, "schedule needs >= 1 level");
    for (int j = 0; j < s->n_levels; ++j) {
        if (!(s->lambda[j] >= 1.0) || !std::isfinite(s->lambda[j]))
            return fail(MF_ERR_INVALID_ARG, "cooling levels need 1 <= lambda < inf");
        if (s->sweeps[j] < 0) return fail(MF_ERR_INVALID_ARG, "negative sweep count");
    }
    if (s->tol > 0 && (s->check_every < 2 || s->max_sweeps < 1))
        return fail(MF_ERR_INVALID_ARG, "tol > 0 needs check_every >= 2 and max_sweeps >= 1");
    return MF_OK;
}

std::pair<int, int> class_shape(mf_plan p, int H, int W) {
    auto it = p->col_shape.find({H, W});
    if (it != p->col_shape.end()) return it->second;
    int tc[8], nth[8];
    mf::col_shape_candidates(H, tc, nth, 8);  // the first candidate is the default shape
    return {tc[0], nth[0]};
}

// The tile of a launch over n_items work items: the class's shape, or its
// narrow shape when the class's shape would leave CUs idle.  A default tile
// that reads its twiddles from L2 relies on a second workgroup per CU to hide
// them; a launch giving each CU at most two such tiles has none to overlap and
// takes the widest candidate with LDS twiddles that still gives every CU a
// workgroup (one 2048^2 field: 8 x 512 instead of 4 x 256).
std::pair<int, int> class_shape(mf_plan p, int H, int W, int64_t n_items) {
    const auto wide = class_shape(p, H, W);
    const int64_t tiles = n_items * ((W + wide.first - 1) / wide.first);
    if (tiles >= mf::kFillBlocks) {
        if (tiles <= 2 * mf::kFillBlocks && mf::col_tw_in_l2(H, wide.first) &&
            p->col_shape.find({H, W}) == p->col_shape.end()) {
            int tc[8], nth[8];
            const int k = mf::col_shape_candidates(H, tc, nth, 8);
            int b = -1;
            for (int i = 0; i < k; ++i)
                if (!mf::col_tw_in_l2(H, tc[i]) && n_items * ((W + tc[i] - 1) / tc[i]) >= mf::kFillBlocks &&
                    (b < 0 || tc[i] > tc[b]))
                    b = i;
            if (b >= 0) return {tc[b], nth[b]};
        }
        return wide;
    }
    auto it = p->col_shape_narrow.find({H, W});
    if (it != p->col_shape_narrow.end()) return it->second;
    int tc = 0, nth = 0;
    mf::narrow_col_shape(H, &tc, &nth);
    return {tc, nth};
}

hipError_t launch_col_class(mf_plan p, int W, int H, const mf::SweepArgs& a, hipStream_t s) {
    const auto sh = class_shape(p, H, W, a.n_items);
    return mf::launch_col_shape(W, H, sh.first, sh.second, a, s);
}

mf::SweepArgs base_args(mf_plan p, int H, int W) {
    mf::SweepArgs a{};
    a.probs = p->d_probs;
    a.nbar = p->d_nbar;
    a.nP = p->d_nP;
    a.nPt = p->d_nPt;
    a.tw_row = p->d_tw.at(W);
    a.tw_col = p->d_tw.at(H);
    a.lambda = 1.0f;
    a.emit_index = -1;
    auto rr = p->row_rows.find({H, W});
    a.row_rows = rr == p->row_rows.end() ? 0 : rr->second;
    auto rn = p->row_rows_narrow.find({H, W});
    a.row_rows_narrow = rn == p->row_rows_narrow.end() ? 0 : rn->second;
    return a;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Launch the graph cached under `key`, or capture `enqueue` (on the plan's
// capture stream) as a new graph, cache it and launch it.  The plan keeps up
// to 8 graphs; keys begin with a tag for the loop they capture.
template <typename Fn>
mf_status run_graph(mf_plan p, const std::vector<uint64_t>& key, hipStream_t s, Fn&& enqueue) {
    if (capturing(s)) return enqueue(s);  // the caller is capturing its own graph: record the launches there
    for (auto& e : p->graphs)
        if (e.key == key) {
            MF_HIP(hipGraphLaunch(e.exec, s));
            return MF_OK;
        }
    if (!p->cap_stream) MF_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    MF_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    mf_status st = enqueue(p->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (st != MF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(MF_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(MF_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (p->graphs.size() >= 8) {  // keep the cache small
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        (void)hipGraphDestroy(p->graphs.front().graph);
        p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back({key, graph, exec});
    MF_HIP(hipGraphLaunch(exec, s));
    return MF_OK;
}

template <typename T>
uint64_t bits_of(T v) {
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    return b;
}

// Grow a plan workspace to `bytes`.  A call on a stream that is being
// captured must not allocate: its workspaces come from mf_plan_reserve.
mf_status ws(DevBuf& b, size_t bytes, hipStream_t s) {
    if (bytes <= b.bytes) return MF_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(MF_ERR_INVALID_ARG, "a workspace this call needs was not reserved (mf_plan_reserve), and the "
                                        "stream is being captured");
    hipError_t e = b.ensure(bytes);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? MF_ERR_OUT_OF_MEMORY : MF_ERR_DEVICE,
                    std::string("workspace allocation: ") + hipGetErrorString(e));
    return MF_OK;
}

// Items workspace for work lists of up to `per` items per problem (two
// regions: the list and, for residual tests, the converged subset).
mf_status ensure_items(mf_plan p, int per, hipStream_t s) {
    size_t max_items = 0;
    for (auto& kv : p->classes) max_items = std::max(max_items, kv.second.size() * (size_t)per);
    return ws(p->items, 2 * (max_items + 1) * sizeof(mf::ItemDev), s);
}

// Build the work list of size class `cls` on the device: `per` items per
// problem (all problems, or only the band-spectrum ones), field offsets in
// the concatenated layout (per * pix_off + q * H * W) or, with `local`, i * H * W.
template <typename ItemPtr, typename Count>
mf_status class_items_at(mf_plan p, mf::ItemDev* base, size_t cap, std::pair<int, int> cls, int per, bool local,
                         bool bands_only, hipStream_t s, ItemPtr* out, Count* n_out) {
    const auto& tab = bands_only ? p->class_band : p->class_all;
    auto it = tab.find(cls);
    const int n_pids = it == tab.end() ? 0 : it->second.second;
    const size_t n = (size_t)n_pids * per;
    *out = base;
    *n_out = (Count)n;
    if (n == 0) return MF_OK;
    if (n > cap) return fail(MF_ERR_INVALID_ARG, "internal: items workspace too small");
    MF_HIP(mf::launch_fill_items(base, p->d_probs, p->d_class_pids + it->second.first, n_pids, per, local ? 1 : 0,
                                 (int64_t)cls.first * cls.second, s));
    return MF_OK;
}

template <typename ItemPtr, typename Count>
mf_status class_items(mf_plan p, std::pair<int, int> cls, int per, bool local, bool bands_only, hipStream_t s,
                      ItemPtr* out, Count* n_out) {
    return class_items_at(p, p->items.as<mf::ItemDev>(), p->items.bytes / sizeof(mf::ItemDev), cls, per, local,
                          bands_only, s, out, n_out);
}

// A work item built on the host (with its copy of the problem record).
mf::ItemDev item_of(mf_plan p, int pid, int pair, int64_t field_off) {
    const HostProblem& hp = p->probs[pid];
    return mf::ItemDev{pid, pair, field_off, hp.pix_off, (float)hp.tau, pid};
}

// Upload a host-built work list at element offset `slot` of the items
// workspace (the residual tests' shrinking lists; those calls synchronise).
mf_status put_items(mf_plan p, const std::vector<mf::ItemDev>& it, size_t slot, hipStream_t s,
                    mf::ItemDev** out) {
    const size_t need = (slot + it.size()) * sizeof(mf::ItemDev);
    if (need > p->items.bytes) return fail(MF_ERR_INVALID_ARG, "internal: items workspace too small");
    mf::ItemDev* d = p->items.as<mf::ItemDev>() + slot;
    MF_HIP(hipMemcpyAsync(d, it.data(), it.size() * sizeof(mf::ItemDev), hipMemcpyHostToDevice, s));
    MF_HIP(hipStreamSynchronize(s));  // the host vector may die right after
    *out = d;
    return MF_OK;
}

// -------------------------------------------------------------------------
// Deterministic solve (Wiener filter or adjoint) on the streamed kernels for
// the problems of one size class.  Field layout: one complex field per problem
// at field_off = pix_off (float2 units).
// -------------------------------------------------------------------------
mf_status solve_class(mf_plan p, const std::vector<int>& pids, int H, int W, const float* src, int src_kind,
                      const mf_schedule* sch, const float* s_init, std::vector<double>& bnorm2,
                      std::vector<mf_info>& info, hipStream_t s) {
    const int n_items = (int)pids.size();
    std::vector<mf::ItemDev> items(n_items);  // host copy for the residual bookkeeping
    for (int i = 0; i < n_items; ++i) items[i] = item_of(p, pids[i], 0, p->probs[pids[i]].pix_off);
    mf::ItemDev* d_items = nullptr;
    int n_dev = 0;
    mf_status st = class_items(p, {H, W}, 1, false, false, s, &d_items, &n_dev);
    if (st != MF_OK) return st;
    mf::SweepArgs a = base_args(p, H, W);
    a.items = d_items;
    a.n_items = n_items;
    a.rows_by_item = 1;  // one item per problem
    a.field = p->field.as<float2>();
    a.src = src;
    a.src_kind = src_kind;
    a.stochastic = 0;
    a.real_only = 1;
    a.t_save = p->t_save.as<float2>();
    a.partials = p->partials.as<double>();
    MF_HIP(mf::launch_load_real(W, H, a, s_init, s));

    bool first = true;
    int total = 0;
    auto sweep = [&](double lam, bool save_t, bool check_t) -> mf_status {
        a.lambda = (float)lam;
        a.save_t = save_t;
        a.check_t = check_t;
        MF_HIP(mf::launch_row(W, H, first ? mf::kRowFwd : mf::kRowInvFwd, a, s));
        a.save_t = a.check_t = 0;
        MF_HIP(launch_col_class(p, W, H, a, s));
        first = false;
        ++total;
        return MF_OK;
    };
    for (int j = 0; j < sch->n_levels; ++j)
        for (int k = 0; k < sch->sweeps[j]; ++k)
            if ((st = sweep(sch->lambda[j], false, false)) != MF_OK) return st;
    const int levels_total = total;
    std::vector<int> done(n_items, 0);
    for (int i = 0; i < n_items; ++i) info[pids[i]] = {total, sch->tol > 0 ? 0 : 1, std::nan("")};
    if (sch->tol > 0) {
        const double lam = sch->lambda[sch->n_levels - 1];
        std::vector<double> part((size_t)n_items * H);
        int remaining = n_items;
        std::vector<mf::ItemDev> live = items;
        while (total < sch->max_sweeps && remaining > 0) {
            const int c = total + 1;  // count after this sweep
            const bool check = (c % sch->check_every == 0) && (c - 1 >= levels_total + 1);
            const bool save = ((c + 1) % sch->check_every == 0);
            if ((st = sweep(lam, save, check)) != MF_OK) return st;
            if (!check) continue;
            MF_HIP(hipMemcpyAsync(part.data(), a.partials, (size_t)a.n_items * H * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            MF_HIP(hipStreamSynchronize(s));
            std::vector<mf::ItemDev> conv, keep;
            for (int i = 0; i < a.n_items; ++i) {
                double acc = 0;  // row partials are indexed y * n_items + item
                for (int y = 0; y < H; ++y) acc += part[(size_t)y * a.n_items + i];
                const int pid = live[i].prob;
                const double T = lam * p->probs[pid].tau;
                const double r = bnorm2[pid] == 0.0 ? 0.0 : std::sqrt(acc) / (T * std::sqrt(bnorm2[pid]));
                info[pid].residual = r;
                info[pid].sweeps = total;
                if (r <= sch->tol) {
                    info[pid].converged = 1;
                    conv.push_back(live[i]);
                } else if (!std::isfinite(r)) {
                    info[pid].converged = -1;  // non-finite: stop iterating this problem
                    conv.push_back(live[i]);
                } else {
                    keep.push_back(live[i]);
                }
            }
            if (!conv.empty()) {
                // finish converged items with the inverse row pass and drop them
                mf::ItemDev* d_conv = nullptr;
                if ((st = put_items(p, conv, (size_t)n_items, s, &d_conv)) != MF_OK) return st;
                mf::SweepArgs b = a;
                b.items = d_conv;
                b.n_items = (int)conv.size();
                MF_HIP(mf::launch_row(W, H, mf::kRowInv, b, s));
                remaining -= (int)conv.size();
                live = keep;
                if (!live.empty()) {
                    if ((st = put_items(p, live, 0, s, &d_items)) != MF_OK) return st;
                }
                a.items = d_items;
                a.n_items = (int)live.size();
                MF_HIP(hipStreamSynchronize(s));
            }
        }
        for (auto& it : live) info[it.prob].sweeps = total;
        if (!live.empty() && !first) {
            MF_HIP(mf::launch_row(W, H, mf::kRowInv, a, s));
        }
        return MF_OK;
    }
    if (!first) MF_HIP(mf::launch_row(W, H, mf::kRowInv, a, s));
    return MF_OK;
}

// Workspaces of the deterministic solves, the adjoint, the band reductions
// and the band loss (with_t: the residual test's messenger snapshot).
mf_status ensure_solve_workspace(mf_plan p, bool with_t, hipStream_t s) {
    size_t max_items = 0, max_rows = 0;
    for (auto& kv : p->classes) {
        max_items = std::max(max_items, kv.second.size());
        max_rows = std::max(max_rows, kv.second.size() * (size_t)kv.first.first);
    }
    mf_status st;
    if ((st = ensure_items(p, 1, s)) != MF_OK) return st;
    if ((st = ws(p->field, (size_t)p->total_px * sizeof(float2), s)) != MF_OK) return st;
    if (with_t && (st = ws(p->t_save, (size_t)p->total_px * sizeof(float2), s)) != MF_OK) return st;
    size_t part = std::max(max_rows, max_items * mf::kBandBlocks * 64);
    if ((st = ws(p->partials, part * sizeof(double), s)) != MF_OK) return st;
    // persistent solve: per-problem outcome
    if ((st = ws(p->sched, (size_t)p->probs.size() * 3 * sizeof(double), s)) != MF_OK) return st;
    // adjoint field v when the caller does not keep it
    if ((st = ws(p->aux, (size_t)p->total_px * sizeof(float), s)) != MF_OK) return st;
    if (p->has_response && (st = ws(p->dprime, (size_t)p->total_px * sizeof(float), s)) != MF_OK) return st;
    return MF_OK;
}

// ||b||^2 per problem with b = N_eff^-1 d at cooling level lam (data) or b = g.
mf_status rhs_norms(mf_plan p, const float* src, int src_kind, double lam, std::vector<double>& out,
                    hipStream_t s) {
    std::vector<float> h((size_t)p->total_px);
    MF_HIP(hipMemcpyAsync(h.data(), src, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    out.assign(p->probs.size(), 0.0);
    for (size_t i = 0; i < p->probs.size(); ++i) {
        const HostProblem& hp = p->probs[i];
        const double T = lam * hp.tau;
        double acc = 0;
        for (int64_t e = 0; e < (int64_t)hp.H * hp.W; ++e) {
            const double nb = p->host_nbar[hp.pix_off + e];
            double b;
            if (src_kind == mf::kSrcData) b = std::isfinite(nb) ? (double)h[hp.pix_off + e] / (nb + T) : 0.0;
            else b = h[hp.pix_off + e];
            acc += b * b;
        }
        out[i] = acc;
    }
    return MF_OK;
}

// The data the kernels see: d itself, or d / A when some problem has a response.
mf_status plan_data(mf_plan p, const float* d, hipStream_t s, const float** out) {
    *out = d;
    if (!p->has_response) return MF_OK;
    mf_status st = ws(p->dprime, (size_t)p->total_px * sizeof(float), s);
    if (st != MF_OK) return st;
    MF_HIP(mf::launch_scale(d, p->d_rinv, p->dprime.as<float>(), p->total_px, s));
    *out = p->dprime.as<float>();
    return MF_OK;
}

// dL/dd from dL/d(d/A): multiply by 1/A in place.
mf_status data_gradient(mf_plan p, float* g, hipStream_t s) {
    if (!p->has_response || !g) return MF_OK;
    MF_HIP(mf::launch_scale(g, p->d_rinv, g, p->total_px, s));
    return MF_OK;
}

mf_status pow2_sides(mf_plan p, const char* what) {
    for (auto& kv : p->classes)
        if (!is_pow2(kv.first.first) || !is_pow2(kv.first.second))
            return fail(MF_ERR_UNSUPPORTED_SIZE, std::string(what) + " needs power-of-two sides (a problem is " +
                                                     std::to_string(kv.first.first) + " x " +
                                                     std::to_string(kv.first.second) + ")");
    return MF_OK;
}

// Shear problems: no response, power-of-two sides.
mf_status shear_check(mf_plan p) {
    if (p->has_response) return fail(MF_ERR_INVALID_ARG, "shear problems take no response");
    return pow2_sides(p, "mass mapping");
}

// Mass mapping on the streamed kernels for one size class: per sweep the row
// kernel and the mirror-paired column kernel; on a sweep that emits kappa
// (or the last sweep of a filter) the emission kernel after them.
mf_status shear_streamed(mf_plan p, const mf::ItemDev* di, int n_items, int H, int W, const float* gamma,
                         float b_ratio, int chains, const std::vector<double>& lam, const std::vector<int32_t>& sweeps,
                         int stochastic, uint64_t seed, int64_t sweep_offset, int burn_in, int n_samples, int thin,
                         const float* state_in, float* state_out, float* samples, float* kappa_out, hipStream_t s) {
    // workspaces sized by ensure_shear_workspace
    float2* field = state_out ? reinterpret_cast<float2*>(state_out) : p->field.as<float2>();
    mf::ShearStreamArgs a{};
    if (samples || kappa_out) a.kfield = p->kfield.as<float2>();
    a.probs = p->d_probs;
    a.items = di;
    a.n_items = n_items;
    a.field = field;
    a.gamma = reinterpret_cast<const float2*>(gamma);
    a.nbar = p->d_nbar;
    a.nP = p->d_nP;
    a.nPt = p->d_nPt;
    a.b_ratio = b_ratio;
    a.tw_row = p->d_tw.at(W);
    a.tw_col = p->d_tw.at(H);
    a.key0 = (uint32_t)(seed & 0xffffffffu);
    a.key1 = (uint32_t)(seed >> 32);
    a.stochastic = stochastic;
    a.samples = reinterpret_cast<float2*>(samples);
    a.chains = chains;
    a.n_samples = n_samples;
    a.kappa_out = reinterpret_cast<float2*>(kappa_out);
    const float2* sin = reinterpret_cast<const float2*>(state_in);
    int64_t total = 0;
    for (int32_t k : sweeps) total += k;
    auto enqueue = [&](hipStream_t cs) -> mf_status {
        mf::ShearStreamArgs aa = a;
        if (sin != field) MF_HIP(mf::launch_shear_init(W, H, aa, sin, cs));
        int64_t k = 0;
        for (size_t lv = 0; lv < lam.size(); ++lv) {
            aa.lambda = (float)lam[lv];
            for (int32_t i = 0; i < sweeps[lv]; ++i, ++k) {
                aa.sweep = (uint32_t)(sweep_offset + k);
                const bool emit = samples && k >= burn_in && ((k - burn_in + 1) % thin) == 0;
                const bool last_kappa = kappa_out && k == total - 1;
                aa.emit = emit || last_kappa;
                aa.slot = emit ? (int)((k - burn_in + 1) / thin - 1) : -1;
                MF_HIP(mf::launch_shear_row(W, H, k == 0 ? mf::kShearFwd : mf::kShearInvFwd, aa, cs));
                MF_HIP(mf::launch_shear_col(W, H, aa, cs));
                if (aa.emit) MF_HIP(mf::launch_shear_row(W, H, mf::kShearEmit, aa, cs));
            }
        }
        if (total > 0) MF_HIP(mf::launch_shear_row(W, H, mf::kShearInv, aa, cs));
        return MF_OK;
    };
    if (!(p->flags & MF_FLAG_GRAPH)) return enqueue(s);
    std::vector<uint64_t> key = {3, (uint64_t)H, (uint64_t)W, (uint64_t)n_items, (uint64_t)(uintptr_t)di,
                                 (uint64_t)(uintptr_t)gamma, (uint64_t)(uintptr_t)field,
                                 (uint64_t)(uintptr_t)a.kfield, (uint64_t)(uintptr_t)sin,
                                 (uint64_t)(uintptr_t)samples, (uint64_t)(uintptr_t)kappa_out, bits_of(b_ratio),
                                 (uint64_t)chains, (uint64_t)stochastic, seed, (uint64_t)sweep_offset,
                                 (uint64_t)burn_in, (uint64_t)n_samples, (uint64_t)thin, lam.size()};
    for (size_t lv = 0; lv < lam.size(); ++lv) {
        key.push_back(bits_of(lam[lv]));
        key.push_back((uint64_t)sweeps[lv]);
    }
    return run_graph(p, key, s, enqueue);
}

// Workspaces of the mass-mapping calls with `chains` chains per problem
// (field: a state field for calls without state_out, needed by the streamed
// classes and by the non-finite check; kappa: the streamed emission staging).
mf_status ensure_shear_workspace(mf_plan p, int chains, bool field, bool check, bool kappa, hipStream_t s) {
    mf_status st = ensure_items(p, chains, s);
    if (st != MF_OK) return st;
    bool any_streamed = false;
    for (auto& kv : p->classes) any_streamed |= !mf::resident_supported(kv.first.first, kv.first.second);
    if (field && (any_streamed || check) &&
        (st = ws(p->field, (size_t)p->total_px * chains * sizeof(float2), s)) != MF_OK)
        return st;
    if (any_streamed && kappa && (st = ws(p->kfield, (size_t)p->total_px * chains * sizeof(float2), s)) != MF_OK)
        return st;
    return MF_OK;
}

hipError_t shear_check_class(mf_plan p, int H, int W, const mf::ItemDev* di, int n_items, float* fin,
                             hipStream_t s) {
    mf::SweepArgs c = base_args(p, H, W);
    c.items = di;
    c.n_items = n_items;
    c.field = reinterpret_cast<float2*>(fin);
    return mf::launch_finite_check(W, H, c, p->d_flag, s);
}

mf_status launch_shear(mf_plan p, const float* gamma, float b_ratio, int chains, const std::vector<double>& lam,
                       const std::vector<int32_t>& sweeps, int stochastic, uint64_t seed, int64_t sweep_offset,
                       int burn_in, int n_samples, int thin, const float* state_in, float* state_out,
                       float* samples, float* kappa_out, bool check, hipStream_t s) {
    const int L = (int)lam.size();
    mf_status st = ensure_shear_workspace(p, chains, !state_out, check, samples || kappa_out, s);
    if (st != MF_OK) return st;
    // the chains' final states: the caller's, or the plan field (streamed classes, non-finite check)
    float* fin = state_out ? state_out : reinterpret_cast<float*>(p->field.as<float2>());
    if (check) MF_HIP(mf::launch_fill_int(p->d_flag, INT32_MAX, 1, s));
    for (auto& kv : p->classes) {
        const int N = kv.first.first, W = kv.first.second;
        mf::ItemDev* di = nullptr;
        int n_items = 0;
        if ((st = class_items(p, kv.first, chains, false, false, s, &di, &n_items)) != MF_OK) return st;
        if (!mf::resident_supported(N, W)) {
            st = shear_streamed(p, di, n_items, N, W, gamma, b_ratio, chains, lam, sweeps, stochastic, seed,
                                sweep_offset, burn_in, n_samples, thin, state_in, state_out, samples, kappa_out, s);
            if (st != MF_OK) return st;
            if (check) MF_HIP(shear_check_class(p, N, W, di, n_items, fin, s));
            continue;
        }
        if (L > mf::kMaxLevels)
            return fail(MF_ERR_INVALID_ARG, "the persistent mass-mapping kernel takes at most 128 cooling levels");
        mf::ShearArgs r{};
        r.probs = p->d_probs;
        r.items = di;
        r.n_items = n_items;
        r.gamma = reinterpret_cast<const float2*>(gamma);
        r.nbar = p->d_nbar;
        r.nP = p->d_nP;
        r.b_ratio = b_ratio;
        r.tw = p->d_tw.at(N);
        r.key0 = (uint32_t)(seed & 0xffffffffu);
        r.key1 = (uint32_t)(seed >> 32);
        r.sweep0 = (uint32_t)sweep_offset;
        r.stochastic = stochastic;
        r.lv.n = L;
        for (int j = 0; j < L; ++j) {
            r.lv.lambda[j] = lam[j];
            r.lv.sweeps[j] = sweeps[j];
        }
        r.burn_in = burn_in;
        r.n_samples = n_samples;
        r.thin = thin;
        r.samples = reinterpret_cast<float2*>(samples);
        r.chains = chains;
        r.state_in = reinterpret_cast<const float2*>(state_in);
        r.state_out = check ? reinterpret_cast<float2*>(fin) : reinterpret_cast<float2*>(state_out);
        r.kappa_out = reinterpret_cast<float2*>(kappa_out);
        MF_HIP(mf::launch_resident_shear(N, r, s));
        if (check) MF_HIP(shear_check_class(p, N, W, di, n_items, fin, s));
    }
    return check ? read_finite_flag(p, s) : MF_OK;
}

// Real part of the field buffer of one streamed size class into `out`.
mf_status copy_class_real(mf_plan p, const std::vector<int>& pids, int H, int W, float* out, hipStream_t s) {
    (void)pids;
    mf::ItemDev* d = nullptr;
    int n_items = 0;
    mf_status st = class_items(p, {H, W}, 1, false, false, s, &d, &n_items);
    if (st != MF_OK) return st;
    mf::SweepArgs a = base_args(p, H, W);
    a.items = d;
    a.n_items = n_items;
    a.field = p->field.as<float2>();
    MF_HIP(mf::launch_copy_out_real(W, H, a, out, s));
    return MF_OK;
}

// Deterministic solve of one size class in the persistent kernel: one
// workgroup per problem runs every level and the residual test on the device.
// The levels travel in the kernel arguments, at most kMaxLevels per launch; a
// longer schedule continues in further launches from the stored result.
mf_status solve_class_resident(mf_plan p, const std::vector<int>& pids, int N, const float* src, int src_kind,
                               const mf_schedule* sch, const float* s_init, float* out, std::vector<mf_info>& info,
                               bool want_info, hipStream_t s) {
    mf::ItemDev* d_items = nullptr;
    int n_items = 0;
    mf_status st = class_items(p, {N, N}, 1, false, false, s, &d_items, &n_items);
    if (st != MF_OK) return st;
    mf::SolveArgs a{};
    a.probs = p->d_probs;
    a.items = d_items;
    a.n_items = n_items;
    a.src = src;
    a.src_kind = src_kind;
    a.s_out = out;
    a.nbar = p->d_nbar;
    a.nP = p->d_nP;
    a.tw = p->d_tw.at(N);
    a.max_sweeps = sch->max_sweeps;
    a.check_every = sch->check_every > 0 ? sch->check_every : 1;
    double* d_info = p->sched.as<double>();
    const int L = sch->n_levels;
    int total = 0;
    for (int j0 = 0; j0 < L; j0 += mf::kMaxLevels) {
        const int j1 = std::min(L, j0 + mf::kMaxLevels);
        const bool last = j1 == L;
        a.lv.n = j1 - j0;
        for (int j = j0; j < j1; ++j) {
            a.lv.lambda[j - j0] = sch->lambda[j];
            a.lv.sweeps[j - j0] = sch->sweeps[j];
        }
        a.total0 = total;
        a.s_init = j0 == 0 ? s_init : out;
        a.tol = last ? sch->tol : 0.0;
        a.info = last && want_info ? d_info : nullptr;
        MF_HIP(mf::launch_resident_solve(N, a, s));
        for (int j = j0; j < j1; ++j) total += sch->sweeps[j];
    }
    if (!want_info) {
        for (int pid : pids) info[pid] = {total, 1, std::nan("")};
        return MF_OK;
    }
    std::vector<double> h((size_t)n_items * 3);
    MF_HIP(hipMemcpyAsync(h.data(), d_info, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n_items; ++i)
        info[pids[i]] = {(int32_t)h[3 * i], (int32_t)h[3 * i + 1], h[3 * i + 2]};
    return MF_OK;
}

bool solve_resident(mf_plan p, int H, int W) {
    return !(p->flags & MF_FLAG_STREAMED_SOLVE) && mf::resident_supported(H, W);
}

// Run the deterministic solve of every problem and write the real result to
// `out` (concatenated).  The streamed classes also leave it in the field buffer.
mf_status run_solve(mf_plan p, const float* src, int src_kind, const mf_schedule* sch, const float* s_init,
                    float* out, mf_info* info_out, hipStream_t s) {
    mf_status st = validate_schedule(sch);
    if (st != MF_OK) return st;
    if ((st = ensure_solve_workspace(p, sch->tol > 0, s)) != MF_OK) return st;
    bool any_streamed = false;
    for (auto& kv : p->classes) any_streamed = any_streamed || !solve_resident(p, kv.first.first, kv.first.second);
    std::vector<double> bn;
    if (sch->tol > 0 && any_streamed) {
        if ((st = rhs_norms(p, src, src_kind, sch->lambda[sch->n_levels - 1], bn, s)) != MF_OK) return st;
    }
    std::vector<mf_info> info(p->probs.size());
    const bool want_info = info_out != nullptr || sch->tol > 0;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        if (solve_resident(p, H, W)) {
            st = solve_class_resident(p, kv.second, H, src, src_kind, sch, s_init, out, info, want_info, s);
            if (st != MF_OK) return st;
            continue;
        }
        if ((st = solve_class(p, kv.second, H, W, src, src_kind, sch, s_init, bn, info, s)) != MF_OK) return st;
        if ((st = copy_class_real(p, kv.second, H, W, out, s)) != MF_OK) return st;
    }
    bool all = true, finite = true;
    for (auto& i : info) {
        if (i.converged < 0) {
            finite = false;
            i.converged = 0;
        }
        all = all && i.converged;
    }
    if (info_out) {
        MF_HIP(hipStreamSynchronize(s));
        std::copy(info.begin(), info.end(), info_out);
    }
    if (!finite) return fail(MF_ERR_NONFINITE, "the residual test saw a non-finite value");
    if (!all) return fail(MF_ERR_NOT_CONVERGED, "tolerance not reached within max_sweeps");
    return MF_OK;
}

// -------------------------------------------------------------------------
// Sampler
// -------------------------------------------------------------------------
// Enqueue the streamed sweep loop of one size class on stream s.
mf_status enqueue_streamed(mf_plan p, const mf::ItemDev* d_items, int n_items, int H, int W, const float* d,
                           const mf_sample_args* g, float2* work, const float2* state_in, float* samples,
                           bool packed, hipStream_t s) {
    mf::SweepArgs a = base_args(p, H, W);
    a.items = d_items;
    a.n_items = n_items;
    a.rows_by_item = g->chains_per_problem <= 2;  // one chain pair per problem
    a.field = work;
    a.src = d;
    a.src_kind = mf::kSrcData;
    a.stochastic = 1;
    a.key0 = (uint32_t)(g->seed & 0xffffffffu);
    a.key1 = (uint32_t)(g->seed >> 32);
    a.samples = samples;
    a.chains = g->chains_per_problem;
    a.n_samples = g->n_samples;
    a.storage = g->storage;
    a.packed = packed ? 1 : 0;
    if (packed)  // two single-chain problems per field: gather their states (or starts)
        MF_HIP(mf::launch_pack_init(W, H, a, state_in, state_in ? 0.f : g->init_scale, s));
    else if (state_in != work)  // copy the given states, or make zero / dispersed starts
        MF_HIP(mf::launch_init_items(W, H, a, state_in, state_in ? 0.f : g->init_scale, s));
    const int64_t K = (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin;
    auto emit_of = [&](int64_t k) -> int {
        if (!samples || k < g->burn_in) return -1;
        const int64_t q = k - g->burn_in + 1;
        return (q % g->thin == 0) ? (int)(q / g->thin - 1) : -1;
    };
    for (int64_t k = 0; k < K; ++k) {
        a.sweep = (uint32_t)(g->sweep_offset + k);
        a.emit_index = k > 0 ? emit_of(k - 1) : -1;
        MF_HIP(mf::launch_row(W, H, k == 0 ? mf::kRowFwd : mf::kRowInvFwd, a, s));
        a.emit_index = -1;
        if (packed) MF_HIP(mf::launch_col_pack(W, H, a, s));
        else MF_HIP(launch_col_class(p, W, H, a, s));
    }
    if (K > 0) {
        a.emit_index = emit_of(K - 1);
        MF_HIP(mf::launch_row(W, H, mf::kRowInv, a, s));
    }
    return MF_OK;
}

// Cooling levels before a sampler's burn-in (streamed kernels, no emission):
// w ends holding the pair states s after the last cooling sweep.
mf_status cool_streamed(mf_plan p, const mf::ItemDev* d_items, int n_items, int H, int W, const float* d,
                        const mf_sample_args* g, int storage, float2* w, const float2* state_in, hipStream_t s) {
    mf::SweepArgs a = base_args(p, H, W);
    a.items = d_items;
    a.n_items = n_items;
    a.rows_by_item = g->chains_per_problem <= 2;  // one chain pair per problem
    a.field = w;
    a.src = d;
    a.src_kind = mf::kSrcData;
    a.stochastic = 1;
    a.key0 = (uint32_t)(g->seed & 0xffffffffu);
    a.key1 = (uint32_t)(g->seed >> 32);
    a.storage = storage;
    if (state_in != w) MF_HIP(mf::launch_init_items(W, H, a, state_in, state_in ? 0.f : g->init_scale, s));
    int64_t k = 0;
    for (int j = 0; j < g->cooling->n_levels; ++j) {
        a.lambda = (float)g->cooling->lambda[j];
        for (int32_t i = 0; i < g->cooling->sweeps[j]; ++i, ++k) {
            a.sweep = (uint32_t)(g->sweep_offset + k);
            MF_HIP(mf::launch_row(W, H, k == 0 ? mf::kRowFwd : mf::kRowInvFwd, a, s));
            MF_HIP(launch_col_class(p, W, H, a, s));
        }
    }
    if (k > 0) MF_HIP(mf::launch_row(W, H, mf::kRowInv, a, s));
    return MF_OK;
}

// The streamed sampler for one size class; with MF_FLAG_GRAPH the whole sweep
// loop is captured once per launch configuration and replayed as one graph.
mf_status sample_streamed(mf_plan p, const mf::ItemDev* d_items, int n_items, int H, int W, const float* d,
                          const mf_sample_args* g, float2* work, const float2* state_in, float* samples,
                          bool graphs, bool packed, hipStream_t s) {
    if (!(p->flags & MF_FLAG_GRAPH) || !graphs)
        return enqueue_streamed(p, d_items, n_items, H, W, d, g, work, state_in, samples, packed, s);
    const auto sh = class_shape(p, H, W, n_items);
    const std::vector<uint64_t> key = {1, (uint64_t)H, (uint64_t)W, (uint64_t)n_items, (uint64_t)(uintptr_t)d_items,
                                       (uint64_t)(uintptr_t)d, (uint64_t)(uintptr_t)work,
                                       (uint64_t)(uintptr_t)state_in, (uint64_t)(uintptr_t)samples, g->seed,
                                       (uint64_t)g->sweep_offset, (uint64_t)g->burn_in, (uint64_t)g->n_samples,
                                       (uint64_t)g->thin, (uint64_t)g->chains_per_problem, bits_of(g->init_scale),
                                       (uint64_t)sh.first, (uint64_t)sh.second, (uint64_t)g->storage,
                                       (uint64_t)packed};
    return run_graph(p, key, s, [&](hipStream_t cs) {
        return enqueue_streamed(p, d_items, n_items, H, W, d, g, work, state_in, samples, packed, cs);
    });
}

// The hierarchical sampler on the streamed kernels for one size class: per
// iteration, sweeps_per_draw sweeps (row kernel, mirror-paired column kernel;
// the last one adds the band powers), then the chi-square sums and the new
// amplitudes.  Samples are emitted by the next row kernel's inverse pass.
mf_status spectrum_streamed(mf_plan p, const mf::ItemDev* di, int n_items, int H, int W, int max_dof, const float* d,
                            const mf_spectrum_args* g, float2* work, const float2* state_in, const double* theta_in,
                            double* theta_out, float* samples, double* theta_samples, const int32_t* d_dof,
                            const double* d_th0, hipStream_t s) {
    constexpr int kNB = mf::kMaxBandsPerProblem;
    const size_t nd = (size_t)n_items * 2 * kNB;  // hier sized by ensure_spectrum_workspace
    double* theta = p->hier.as<double>();
    mf::SweepArgs a = base_args(p, H, W);
    a.items = di;
    a.n_items = n_items;
    a.field = work;
    a.src = d;
    a.src_kind = mf::kSrcData;
    a.stochastic = 1;
    a.key0 = (uint32_t)(g->seed & 0xffffffffu);
    a.key1 = (uint32_t)(g->seed >> 32);
    a.samples = samples;
    a.chains = g->chains_per_problem;
    a.n_samples = g->n_samples;
    mf::SpectrumStreamArgs r{};
    r.probs = p->d_probs;
    r.items = di;
    r.n_items = n_items;
    r.field = work;
    r.tw_col = p->d_tw.at(H);
    r.band = p->d_band;
    r.bandt = p->d_bandt;
    r.band_base = p->d_band_base;
    r.band_count = p->d_band_count;
    r.dof = d_dof;
    r.theta0 = d_th0;
    r.theta_in = theta_in;
    r.theta_out = theta_out;
    r.theta_samples = theta_samples;
    r.theta = theta;
    r.pw = theta + nd;
    r.chi = theta + 2 * nd;
    r.coef = reinterpret_cast<float4*>(theta + 3 * nd);
    r.key0 = a.key0;
    r.key1 = a.key1;
    r.chains = g->chains_per_problem;
    r.chains_pad = 2 * ((g->chains_per_problem + 1) / 2);
    r.n_samples = g->n_samples;
    r.prior_beta = g->prior_beta;
    const int64_t iters = (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin;
    const int K = g->sweeps_per_draw;
    auto slot_of = [&](int64_t i) -> int64_t {
        if (i < g->burn_in) return -1;
        const int64_t q = i - g->burn_in + 1;
        return (q % g->thin == 0) ? q / g->thin - 1 : -1;
    };
    auto enqueue = [&](hipStream_t cs) -> mf_status {
        mf::SweepArgs aa = a;
        mf::SpectrumStreamArgs rr = r;
        if (state_in != work)  // copy the given states, or make zero / dispersed starts
            MF_HIP(mf::launch_init_items(W, H, aa, state_in, state_in ? 0.f : g->init_scale, cs));
        MF_HIP(mf::launch_spectrum_init(rr, cs));
        for (int64_t i = 0; i < iters; ++i) {
            const int64_t gi = g->iteration_offset + i;
            for (int k = 0; k < K; ++k) {
                aa.sweep = (uint32_t)(gi * K + k);
                aa.emit_index = (samples && k == 0 && i > 0) ? (int)slot_of(i - 1) : -1;
                MF_HIP(mf::launch_row(W, H, (i == 0 && k == 0) ? mf::kRowFwd : mf::kRowInvFwd, aa, cs));
                rr.sweep = aa.sweep;
                rr.add_power = k == K - 1;
                MF_HIP(mf::launch_spectrum_col(W, H, rr, cs));
            }
            rr.iteration = (uint32_t)gi;
            MF_HIP(mf::launch_spectrum_draw(rr, max_dof, slot_of(i), cs));
        }
        if (iters > 0) {
            aa.emit_index = samples ? (int)slot_of(iters - 1) : -1;
            MF_HIP(mf::launch_row(W, H, mf::kRowInv, aa, cs));
        }
        return MF_OK;
    };
    if (!(p->flags & MF_FLAG_GRAPH)) return enqueue(s);
    const std::vector<uint64_t> key = {2, (uint64_t)H, (uint64_t)W, (uint64_t)n_items, (uint64_t)(uintptr_t)di,
                                       (uint64_t)(uintptr_t)d, (uint64_t)(uintptr_t)work,
                                       (uint64_t)(uintptr_t)state_in, (uint64_t)(uintptr_t)theta_in,
                                       (uint64_t)(uintptr_t)theta_out, (uint64_t)(uintptr_t)samples,
                                       (uint64_t)(uintptr_t)theta_samples, (uint64_t)(uintptr_t)d_dof,
                                       (uint64_t)(uintptr_t)d_th0, (uint64_t)(uintptr_t)theta, g->seed,
                                       (uint64_t)g->iteration_offset, (uint64_t)g->burn_in, (uint64_t)g->n_samples,
                                       (uint64_t)g->thin, (uint64_t)K, (uint64_t)g->chains_per_problem,
                                       (uint64_t)g->prior_dof, bits_of(g->prior_beta), bits_of(g->init_scale),
                                       (uint64_t)max_dof};
    return run_graph(p, key, s, enqueue);
}

// Time every column-tile shape and every fused-row-kernel shape of each
// streamed size class on a scratch field and keep the fastest of each (all
// shapes do the same arithmetic, element for element).  Choices can be
// persisted in the file named by MF_TUNE_CACHE: lines "gfx950 H W tc nth"
// (column tiles) and "gfx950-rows H W rows" (rows per fused row block).
mf_status autotune(mf_plan p) {
    const char* cache_path = std::getenv("MF_TUNE_CACHE");
    std::map<std::pair<int, int>, std::pair<int, int>> cached;
    std::map<std::pair<int, int>, int> cached_rows;
    std::map<std::pair<int, int>, std::array<int, 3>> cached_narrow;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[256];
            while (std::fgets(line, sizeof line, f)) {
                char arch[64];
                int H, W, x, y, z;
                const int n = std::sscanf(line, "%63s %d %d %d %d %d", arch, &H, &W, &x, &y, &z);
                if (n == 5 && std::string(arch) == "gfx950") cached[{H, W}] = {x, y};
                else if (n >= 4 && std::string(arch) == "gfx950-rows") cached_rows[{H, W}] = x;
                else if (n == 6 && std::string(arch) == "gfx950-narrow") cached_narrow[{H, W}] = {x, y, z};
            }
            std::fclose(f);
        }
    }
    auto time_launches = [&](auto&& launch, float* ms_out) -> mf_status {
        hipEvent_t e0, e1;
        MF_HIP(hipEventCreate(&e0));
        MF_HIP(hipEventCreate(&e1));
        hipError_t e = launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e != hipSuccess) return fail(MF_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
        return MF_OK;
    };
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        if (H < 256 && W < 256) continue;  // small classes run on the persistent kernel or are launch-bound
        int tc[8], nth[8], rows[8];
        const int nc = H >= 256 ? mf::col_shape_candidates(H, tc, nth, 8) : 0;
        const int nr = mf::fused_row_candidates(W, rows, 8);
        auto cc = cached.find({H, W});
        auto cr = cached_rows.find({H, W});
        auto cn = cached_narrow.find({H, W});
        if (cc != cached.end()) p->col_shape[{H, W}] = cc->second;
        if (cr != cached_rows.end()) p->row_rows[{H, W}] = cr->second;
        if (cn != cached_narrow.end()) {
            p->col_shape_narrow[{H, W}] = {cn->second[0], cn->second[1]};
            if (cn->second[2] > 0) p->row_rows_narrow[{H, W}] = cn->second[2];
        }
        const bool tune_col = nc > 1 && cc == cached.end();
        const bool tune_row = nr > 1 && cr == cached_rows.end();
        const bool tune_narrow = (nc > 1 || nr > 1) && cn == cached_narrow.end();
        // whether the class's shapes (as chosen so far) leave CUs idle on one item
        auto narrow_need = [&](bool* col_narrow, bool* row_narrow) {
            const auto wide = class_shape(p, H, W);
            auto rw = p->row_rows.find({H, W});
            const int rows_w = rw != p->row_rows.end() ? rw->second : (nr > 0 ? rows[0] : 0);
            *col_narrow = nc > 1 && (W + wide.first - 1) / wide.first < mf::kFillBlocks;
            *row_narrow = nr > 1 && rows_w > 0 && (H + rows_w - 1) / rows_w < mf::kFillBlocks;
        };
        bool col_narrow = false, row_narrow = false;
        narrow_need(&col_narrow, &row_narrow);
        if (!tune_col && !tune_row && !(tune_narrow && (col_narrow || row_narrow))) continue;
        const int pid = kv.second[0];
        const int n_items = std::max(1, std::min(16, (int)(2 * (4096 * 4096 / ((int64_t)H * W)))));
        std::vector<mf::ItemDev> items(n_items);
        for (int i = 0; i < n_items; ++i) items[i] = item_of(p, pid, i, (int64_t)i * H * W);
        DevBuf fld, it, src;
        MF_HIP(fld.ensure((size_t)n_items * H * W * sizeof(float2)));
        MF_HIP(it.ensure(items.size() * sizeof(mf::ItemDev)));
        MF_HIP(src.ensure((size_t)p->total_px * sizeof(float)));
        MF_HIP(hipMemcpy(it.p, items.data(), items.size() * sizeof(mf::ItemDev), hipMemcpyHostToDevice));
        MF_HIP(hipMemset(fld.p, 0, (size_t)n_items * H * W * sizeof(float2)));
        MF_HIP(hipMemset(src.p, 0, (size_t)p->total_px * sizeof(float)));
        mf::SweepArgs a = base_args(p, H, W);
        a.items = it.as<mf::ItemDev>();
        a.n_items = n_items;
        a.field = fld.as<float2>();
        a.src = src.as<float>();
        a.src_kind = mf::kSrcData;
        a.stochastic = 1;
        mf_status st = MF_OK;
        if (tune_col) {
            float best = 1e30f;
            int bi = 0;
            for (int ci = 0; ci < nc && st == MF_OK; ++ci) {
                float ms = 0.f;
                st = time_launches([&] { return mf::launch_col_shape(W, H, tc[ci], nth[ci], a, nullptr); }, &ms);
                if (ms < best) {
                    best = ms;
                    bi = ci;
                }
            }
            if (st != MF_OK) return st;
            p->col_shape[{H, W}] = {tc[bi], nth[bi]};
            if (cache_path)
                if (FILE* f = std::fopen(cache_path, "a")) {
                    std::fprintf(f, "gfx950 %d %d %d %d\n", H, W, tc[bi], nth[bi]);
                    std::fclose(f);
                }
        }
        if (tune_row) {
            float best = 1e30f;
            int bi = 0;
            for (int ri = 0; ri < nr && st == MF_OK; ++ri) {
                float ms = 0.f;
                mf::SweepArgs b = a;
                b.row_rows = rows[ri];
                st = time_launches([&] { return mf::launch_row(W, H, mf::kRowInvFwd, b, nullptr); }, &ms);
                if (ms < best) {
                    best = ms;
                    bi = ri;
                }
            }
            if (st != MF_OK) return st;
            p->row_rows[{H, W}] = rows[bi];
            if (cache_path)
                if (FILE* f = std::fopen(cache_path, "a")) {
                    std::fprintf(f, "gfx950-rows %d %d %d\n", H, W, rows[bi]);
                    std::fclose(f);
                }
        }
        // the shapes of launches too small to fill the GPU, timed on one item
        // (a single solve); only where the class's shapes would leave CUs idle
        narrow_need(&col_narrow, &row_narrow);
        if (tune_narrow && (col_narrow || row_narrow)) {
            mf::SweepArgs b = a;
            b.n_items = 1;
            int ntc = 0, nnth = 0;
            mf::narrow_col_shape(H, &ntc, &nnth);
            int nrows = mf::narrow_row_rows(W);
            if (col_narrow) {
                float best = 1e30f;
                for (int ci = 0; ci < nc && st == MF_OK; ++ci) {
                    float ms = 0.f;
                    st = time_launches([&] { return mf::launch_col_shape(W, H, tc[ci], nth[ci], b, nullptr); }, &ms);
                    if (ms < best) {
                        best = ms;
                        ntc = tc[ci];
                        nnth = nth[ci];
                    }
                }
            }
            if (row_narrow) {
                float best = 1e30f;
                for (int ri = 0; ri < nr && st == MF_OK; ++ri) {
                    float ms = 0.f;
                    mf::SweepArgs c = b;
                    c.row_rows = c.row_rows_narrow = rows[ri];  // this shape in either regime
                    st = time_launches([&] { return mf::launch_row(W, H, mf::kRowInvFwd, c, nullptr); }, &ms);
                    if (ms < best) {
                        best = ms;
                        nrows = rows[ri];
                    }
                }
            }
            if (st != MF_OK) return st;
            p->col_shape_narrow[{H, W}] = {ntc, nnth};
            if (nrows > 0) p->row_rows_narrow[{H, W}] = nrows;
            if (cache_path)
                if (FILE* f = std::fopen(cache_path, "a")) {
                    std::fprintf(f, "gfx950-narrow %d %d %d %d %d\n", H, W, ntc, nnth, nrows);
                    std::fclose(f);
                }
        }
    }
    return MF_OK;
}

// Buffers of one sampler call: plan workspaces, or any other device memory
// of the same sizes.
struct SampleWs {
    mf::ItemDev* items = nullptr;  // work lists
    size_t items_cap = 0;          // in items
    float4* coef = nullptr;        // persistent tables: 40 bytes per pixel pair
    float* dprime = nullptr;       // d / A (response plans)
    float2* field = nullptr;       // work field when state_out is NULL
    float2* hfield = nullptr;      // 16-bit work field (4 bytes per element)
    bool graphs = true;            // MF_FLAG_GRAPH may capture and instantiate graphs (which allocates)
};

mf_status validate_sample(const mf_sample_args* g, const float* state_out, const float* samples_out) {
    if (g->chains_per_problem < 1 || g->burn_in < 0 || g->n_samples < 0 || g->thin < 1 || g->sweep_offset < 0)
        return fail(MF_ERR_INVALID_ARG, "need chains >= 1, burn_in >= 0, n_samples >= 0, thin >= 1, sweep_offset >= 0");
    if (g->sweep_offset + (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin > 0xffffffffLL)
        return fail(MF_ERR_INVALID_ARG, "sweep index exceeds 2^32");
    if (g->form < MF_FORM_AUTO || g->form > MF_FORM_PLAIN) return fail(MF_ERR_INVALID_ARG, "unknown form");
    if (g->storage < MF_STORAGE_FP32 || g->storage > MF_STORAGE_BF16) return fail(MF_ERR_INVALID_ARG, "unknown storage");
    if (g->cooling) {
        const mf_status sc = validate_schedule(g->cooling);
        if (sc != MF_OK) return sc;
        int64_t n_cool = 0;
        for (int j = 0; j < g->cooling->n_levels; ++j) n_cool += g->cooling->sweeps[j];
        if (g->sweep_offset + n_cool + (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin > 0xffffffffLL)
            return fail(MF_ERR_INVALID_ARG, "sweep index exceeds 2^32");
    }
    if (g->n_samples > 0 && !samples_out && !state_out)
        return fail(MF_ERR_INVALID_ARG, "nothing to write: samples_out and state_out are NULL");
    return MF_OK;
}

bool sample_any_persistent(mf_plan p, int form) {
    bool any = false;
    for (auto& kv : p->classes)
        any |= form == MF_FORM_PERSISTENT || (form == MF_FORM_AUTO && mf::resident_supported(kv.first.first, kv.first.second));
    return any;
}

// Workspaces of mf_sample with `pairs` chain pairs per problem.
mf_status ensure_sample_workspace(mf_plan p, int pairs, int storage, int form, bool need_field, hipStream_t s) {
    mf_status st = ensure_items(p, pairs, s);
    if (st != MF_OK) return st;
    const size_t field_elems = (size_t)p->total_px * pairs;
    // single-chain problems on the streamed kernels run packed two to a field,
    // in a workspace field whatever state_out is
    bool packs = false;
    if (pairs == 1 && storage == MF_STORAGE_FP32)
        for (auto& kv : p->classes)
            packs |= kv.second.size() >= 2 && !mf::resident_supported(kv.first.first, kv.first.second);
    if ((need_field || packs) && (st = ws(p->field, field_elems * sizeof(float2), s)) != MF_OK) return st;
    if (storage != MF_STORAGE_FP32 && (st = ws(p->hfield, field_elems * 4, s)) != MF_OK) return st;
    if (sample_any_persistent(p, form) &&
        (st = ws(p->coef, (size_t)p->total_px / 2 * (sizeof(float4) + sizeof(float2) + sizeof(float4)), s)) != MF_OK)
        return st;
    if (p->has_response && (st = ws(p->dprime, (size_t)p->total_px * sizeof(float), s)) != MF_OK) return st;
    return MF_OK;
}

// Lowest problem whose chain states hold a NaN or an infinity (after a
// synchronisation of the stream), or MF_OK.
mf_status read_finite_flag(mf_plan p, hipStream_t s) {
    int32_t h = 0;
    MF_HIP(hipMemcpyAsync(&h, p->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    if (h != INT32_MAX)
        return fail(MF_ERR_NONFINITE, "problem " + std::to_string(h) + ": a chain state holds NaN or Inf");
    return MF_OK;
}

// Algorithm 1 for every problem (mf_sample), on the buffers of `w`.
mf_status sample_impl(mf_plan p, const float* d, const mf_sample_args* g, const float* state_in, float* state_out,
                      float* samples_out, const SampleWs& w, hipStream_t s) {
    int64_t n_cool = 0;
    if (g->cooling)
        for (int j = 0; j < g->cooling->n_levels; ++j) n_cool += g->cooling->sweeps[j];
    mf_sample_args gm = *g;  // the sampling phase after the cooling levels
    gm.sweep_offset += n_cool;
    gm.cooling = nullptr;
    if (p->has_response) {
        MF_HIP(mf::launch_scale(d, p->d_rinv, w.dprime, p->total_px, s));
        d = w.dprime;
    }
    const int pairs = (g->chains_per_problem + 1) / 2;
    float2* work = state_out ? reinterpret_cast<float2*>(state_out) : w.field;
    const float2* sin = reinterpret_cast<const float2*>(state_in);
    float2* hwork = g->storage != MF_STORAGE_FP32 ? w.hfield : nullptr;
    float4* pcoef = nullptr;
    float2* psrc = nullptr;
    float4* mcoef = nullptr;
    if (sample_any_persistent(p, g->form)) {
        const size_t half = (size_t)p->total_px / 2;
        pcoef = w.coef;
        psrc = reinterpret_cast<float2*>(pcoef + half);
        mcoef = reinterpret_cast<float4*>(psrc + half);
        MF_HIP(mf::launch_sampler_coefs(p->d_probs, (int)p->probs.size(), d, p->d_nbar, p->d_nP, pcoef, psrc, mcoef,
                                        s));
    }
    if (g->check_finite) MF_HIP(mf::launch_fill_int(p->d_flag, INT32_MAX, 1, s));
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        int form = g->form;
        if (form == MF_FORM_AUTO) form = mf::resident_supported(H, W) ? MF_FORM_PERSISTENT : MF_FORM_STREAMED;
        if (form == MF_FORM_PERSISTENT && !mf::resident_supported(H, W))
            return fail(MF_ERR_UNSUPPORTED_SIZE, "the persistent form needs H = W in {32, 64, 128}");
        // one chain per problem on the streamed kernels: two problems share a
        // complex field (no imaginary chain computed only to be dropped)
        const int n_pids = (int)kv.second.size();
        const bool packed = form == MF_FORM_STREAMED && g->chains_per_problem == 1 && g->storage == MF_STORAGE_FP32 &&
                            n_cool == 0 && n_pids >= 2 && w.field && is_pow2(H) && is_pow2(W);
        mf::ItemDev* di = nullptr;
        int n_items = 0;
        mf_status st = MF_OK;
        if (packed) {
            n_items = (n_pids + 1) / 2;
            if ((size_t)n_items > w.items_cap) return fail(MF_ERR_INVALID_ARG, "internal: items workspace too small");
            di = w.items;
            MF_HIP(mf::launch_fill_packed_items(di, p->d_probs, p->d_class_pids + p->class_all.at(kv.first).first, n_pids,
                                                (int64_t)H * W, s));
            st = sample_streamed(p, di, n_items, H, W, d, &gm, w.field, sin, samples_out, w.graphs, true, s);
            if (st != MF_OK) return st;
            mf::SweepArgs a = base_args(p, H, W);
            a.items = di;
            a.n_items = n_items;
            a.field = w.field;
            a.packed = 1;
            if (state_out) MF_HIP(mf::launch_pack_copy_out(W, H, a, work, s));
            if (g->check_finite) MF_HIP(mf::launch_finite_check(W, H, a, p->d_flag, s));
            continue;
        }
        st = class_items_at(p, w.items, w.items_cap, kv.first, pairs, false, false, s, &di, &n_items);
        if (st != MF_OK) return st;
        const float2* cin = sin;  // the state the sampling phase starts from
        if (n_cool > 0) {
            float2* cw = (form != MF_FORM_PERSISTENT && hwork) ? hwork : work;
            st = cool_streamed(p, di, n_items, H, W, d, g, cw == hwork ? g->storage : MF_STORAGE_FP32, cw, sin, s);
            if (st != MF_OK) return st;
            cin = cw;
        }
        mf::SweepArgs chk = base_args(p, H, W);
        chk.items = di;
        chk.n_items = n_items;
        chk.field = work;
        if (form == MF_FORM_PERSISTENT) {
            mf::ResidentArgs r{};
            r.probs = p->d_probs;
            r.items = di;
            r.n_items = n_items;
            r.field = work;
            r.state_in = cin;
            r.init_scale = g->init_scale;
            r.pcoef = pcoef;
            r.psrc = psrc;
            r.mcoef = mcoef;
            r.tw = p->d_tw.at(W);
            r.key0 = (uint32_t)(g->seed & 0xffffffffu);
            r.key1 = (uint32_t)(g->seed >> 32);
            r.sweep0 = (uint32_t)gm.sweep_offset;
            r.burn_in = g->burn_in;
            r.n_samples = g->n_samples;
            r.thin = g->thin;
            r.samples = samples_out;
            r.chains = g->chains_per_problem;
            MF_HIP(mf::launch_resident_sample(H, r, s));
        } else {
            float2* wf = hwork ? hwork : work;
            if (form == MF_FORM_STREAMED) {
                st = sample_streamed(p, di, n_items, H, W, d, &gm, wf, cin, samples_out, w.graphs, false, s);
            } else {  // plain: one chain pair per launch sequence
                for (int i = 0; i < n_items && st == MF_OK; ++i)
                    st = sample_streamed(p, di + i, 1, H, W, d, &gm, wf, cin, samples_out, w.graphs, false, s);
            }
            if (st == MF_OK && hwork && state_out) {  // final states widened to FP32
                mf::SweepArgs a = base_args(p, H, W);
                a.items = di;
                a.n_items = n_items;
                a.field = hwork;
                a.storage = g->storage;
                MF_HIP(mf::launch_copy_out_pairs(W, H, a, work, s));
            }
            if (hwork) {
                chk.field = hwork;
                chk.storage = g->storage;
            }
        }
        if (st != MF_OK) return st;
        // a NaN or an infinity anywhere in a chain's history reaches its final
        // state (every sweep mixes all pixels through the transforms)
        if (g->check_finite) MF_HIP(mf::launch_finite_check(W, H, chk, p->d_flag, s));
    }
    return g->check_finite ? read_finite_flag(p, s) : MF_OK;
}

// Workspaces of mf_sample_spectrum with `pairs` chain pairs per problem.
mf_status ensure_spectrum_workspace(mf_plan p, int pairs, bool need_field, hipStream_t s) {
    mf_status st = ensure_items(p, pairs, s);
    if (st != MF_OK) return st;
    if (need_field && (st = ws(p->field, (size_t)p->total_px * pairs * sizeof(float2), s)) != MF_OK) return st;
    if ((st = ws(p->spec, (size_t)std::max(1, p->total_bands) * sizeof(int32_t), s)) != MF_OK) return st;
    if ((st = ws(p->coef, (size_t)p->total_px / 2 * (sizeof(float4) + sizeof(float2) + sizeof(float4)), s)) != MF_OK)
        return st;
    if (p->has_response && (st = ws(p->dprime, (size_t)p->total_px * sizeof(float), s)) != MF_OK) return st;
    size_t max_items = 0;
    for (auto& kv : p->classes)
        if (!mf::resident_supported(kv.first.first, kv.first.second))
            max_items = std::max(max_items, kv.second.size() * (size_t)pairs);
    if (max_items > 0) {
        constexpr int kNB = mf::kMaxBandsPerProblem;
        const size_t nd = max_items * 2 * kNB;
        if ((st = ws(p->hier, 3 * nd * sizeof(double) + max_items * kNB * sizeof(float4), s)) != MF_OK) return st;
    }
    return MF_OK;
}

// Workspaces of the unrolled gradient for K sweeps with a checkpoint every C:
// sized for the largest size class (classes run one after another).
mf_status ensure_unrolled_workspace(mf_plan p, int K, int C, hipStream_t s) {
    mf_status st = ensure_items(p, 1, s);
    if (st != MF_OK) return st;
    if (p->has_response && (st = ws(p->dprime, (size_t)p->total_px * sizeof(float), s)) != MF_OK) return st;
    size_t n_max = 0, tiles_max = 0;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        n_max = std::max(n_max, kv.second.size() * (size_t)H * W);
        const int tc = class_shape(p, H, W, (int64_t)kv.second.size()).first;  // one item per problem
        tiles_max = std::max(tiles_max, kv.second.size() * (size_t)((W + tc - 1) / tc));
    }
    const size_t ncp = (size_t)(K + C - 1) / C;
    if ((st = ws(p->field, n_max * sizeof(float2), s)) != MF_OK) return st;
    if ((st = ws(p->field_adj, n_max * sizeof(float2), s)) != MF_OK) return st;
    if ((st = ws(p->ckpt, ncp * n_max * sizeof(float2), s)) != MF_OK) return st;
    if ((st = ws(p->tstore, (size_t)std::min(C, K) * n_max * sizeof(float2), s)) != MF_OK) return st;
    return ws(p->slots, tiles_max * mf::kMaxBandsPerProblem * sizeof(double), s);
}

// The implicit VJP of mf_wiener_backward: the adjoint solve, then N^-1 v and
// the band sums per size class.
mf_status backward_impl(mf_plan p, const float* s_wf, const float* grad_s, const mf_schedule* schedule,
                        float* grad_d, double* grad_bands, float* v_out, mf_info* info, hipStream_t s) {
    mf_status st = validate_schedule(schedule);
    if (st != MF_OK) return st;
    if ((st = ensure_solve_workspace(p, schedule->tol > 0, s)) != MF_OK) return st;
    float* v = v_out ? v_out : p->aux.as<float>();
    st = run_solve(p, grad_s, mf::kSrcGrad, schedule, nullptr, v, info, s);
    if (st != MF_OK && st != MF_ERR_NOT_CONVERGED) return st;
    const mf_status conv = st;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        mf::SweepArgs a = base_args(p, H, W);
        a.field = p->field.as<float2>();
        a.partials = p->partials.as<double>();
        if (grad_d) {
            if ((st = class_items(p, kv.first, 1, false, false, s, &a.items, &a.n_items)) != MF_OK) return st;
            MF_HIP(mf::launch_grad_d(W, H, a, v, grad_d, s));
        }
        if (!grad_bands || p->total_bands <= 0) continue;
        if ((st = class_items(p, kv.first, 1, false, true, s, &a.items, &a.n_items)) != MF_OK) return st;
        if (a.n_items == 0) continue;
        MF_HIP(mf::launch_band_power(W, H, a, v, s_wf, p->d_band, p->d_band_base, p->d_band_count,
                                     p->d_band_scale, grad_bands, s));
    }
    if ((st = data_gradient(p, grad_d, s)) != MF_OK) return st;
    return conv;
}

// Workspace of mf_band_loss: grad_s and the explicit grad_d (floats per
// pixel), FP64 partial sums per item and block, band powers.
struct LossWs {
    float* grad_s;
    float* grad_d;
    double* part;
    double* power;
};
size_t align256(size_t b) { return (b + 255) / 256 * 256; }
LossWs loss_ws(mf_plan p) {
    char* b = p->lossbuf.as<char>();
    const size_t px = align256((size_t)p->total_px * sizeof(float));
    const size_t part = align256(p->probs.size() * mf::kLossBlocks * 2 * sizeof(double));
    return {reinterpret_cast<float*>(b), reinterpret_cast<float*>(b + px), reinterpret_cast<double*>(b + 2 * px),
            reinterpret_cast<double*>(b + 2 * px + part)};
}
mf_status ensure_loss_workspace(mf_plan p, hipStream_t s) {
    const size_t px = align256((size_t)p->total_px * sizeof(float));
    const size_t part = align256(p->probs.size() * mf::kLossBlocks * 2 * sizeof(double));
    return ws(p->lossbuf, 2 * px + part + (size_t)std::max(1, p->total_bands) * sizeof(double), s);
}

}  // namespace

// =========================================================================
// C entry points
// =========================================================================
extern "C" {

const char* mf_status_string(mf_status st) {
    switch (st) {
        case MF_OK: return "ok";
        case MF_ERR_INVALID_ARG: return "invalid argument";
        case MF_ERR_UNSUPPORTED_SIZE: return "unsupported size";
        case MF_ERR_OUT_OF_MEMORY: return "out of memory";
        case MF_ERR_DEVICE: return "device error";
        case MF_ERR_NOT_CONVERGED: return "not converged";
        case MF_ERR_NONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char* mf_last_error(void) { return g_last_error.c_str(); }

mf_status mf_plan_create(mf_plan* out, int32_t n_problems, const mf_problem* problems, uint32_t flags,
                         mf_stream stream) {
    if (!out) return fail(MF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_problems < 1 || n_problems >= (1 << 24) || !problems)
        return fail(MF_ERR_INVALID_ARG, "need 1 <= n_problems < 2^24 and a problem array");
    mf_plan p = new (std::nothrow) mf_plan_s();
    if (!p) return fail(MF_ERR_OUT_OF_MEMORY, "host allocation failed");
    if (flags & ~(uint32_t)(MF_FLAG_AUTOTUNE | MF_FLAG_GRAPH | MF_FLAG_STREAMED_SOLVE | MF_FLAG_INF_AS_1E8)) {
        delete p;
        return fail(MF_ERR_INVALID_ARG, "unknown plan flags");
    }
    p->flags = flags;
    (void)hipGetDevice(&p->device);
    int64_t off = 0;
    int bands = 0;
    p->probs.resize(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        const mf_problem& q = problems[i];
        HostProblem& hp = p->probs[i];
        if (!size_ok(q.H) || !size_ok(q.W)) {
            delete p;
            return fail(MF_ERR_UNSUPPORTED_SIZE, "problem " + std::to_string(i) +
                                                     ": H and W must be even 2^a 3^b in [16, 2048]");
        }
        if (!q.noise_var) {
            delete p;
            return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": noise_var is NULL");
        }
        hp.H = q.H;
        hp.W = q.W;
        hp.pix_off = off;
        off += (int64_t)q.H * q.W;
        mf_status st = copy_spectrum(hp, q.spectrum, i);
        if (st != MF_OK) {
            delete p;
            return st;
        }
        hp.band_base = bands;
        bands += hp.n_bands;
        p->classes[{q.H, q.W}].push_back(i);
    }
    p->total_px = off;
    p->total_bands = bands;
    p->host_nbar.resize(off);
    std::vector<mf::ProbDev> pd(n_problems);
    std::vector<float> rinv;
    for (int i = 0; i < n_problems; ++i) p->has_response = p->has_response || problems[i].response;
    if (p->has_response) rinv.assign(off, 1.0f);
    std::vector<double> neff;
    for (int i = 0; i < n_problems; ++i) {
        HostProblem& hp = p->probs[i];
        const float* nv = problems[i].noise_var;
        const float* A = problems[i].response;
        double tau = INFINITY;
        const int64_t n = (int64_t)hp.H * hp.W;
        // with a response, the plan holds the A = I problem for d/A and N/A^2
        neff.assign(n, INFINITY);
        for (int64_t e = 0; e < n; ++e) {
            const float v = nv[e];
            if (std::isnan(v) || v <= 0.f) {
                delete p;
                return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": noise variances must be > 0 (+inf = missing)");
            }
            double a = 1.0;
            if (A) {
                a = A[e];
                if (!std::isfinite(a)) {
                    delete p;
                    return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": response values must be finite");
                }
                rinv[hp.pix_off + e] = a != 0.0 ? (float)(1.0 / a) : 0.0f;
            }
            if (std::isfinite(v) && a != 0.0) neff[e] = (double)v / (a * a);
            else if (flags & MF_FLAG_INF_AS_1E8) neff[e] = 1e8;
            if (std::isfinite(neff[e])) tau = std::min(tau, neff[e]);
        }
        if (!std::isfinite(tau)) tau = 1.0;  // every pixel missing: any T samples the prior
        hp.tau = tau;
        for (int64_t e = 0; e < n; ++e)
            p->host_nbar[hp.pix_off + e] = std::isfinite(neff[e]) ? (float)(neff[e] - tau) : INFINITY;
        pd[i] = {hp.H, hp.W, hp.pix_off, (float)tau, i};
    }
    std::vector<int32_t> bb(n_problems), bc(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        bb[i] = p->probs[i].band_base;
        bc[i] = p->probs[i].n_bands;
    }
#define MF_TRY(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            delete p;                                                             \
            return fail(e_ == hipErrorOutOfMemory ? MF_ERR_OUT_OF_MEMORY : MF_ERR_DEVICE, \
                        std::string(#call) + ": " + hipGetErrorString(e_));       \
        }                                                                         \
    } while (0)
    MF_TRY(hipMalloc(&p->d_probs, n_problems * sizeof(mf::ProbDev)));
    MF_TRY(hipMalloc(&p->d_nbar, off * sizeof(float)));
    MF_TRY(hipMalloc(&p->d_nP, off * sizeof(float)));
    MF_TRY(hipMalloc(&p->d_nPt, off / 2 * sizeof(float2)));
    MF_TRY(hipMalloc(&p->d_band, off * sizeof(int16_t)));
    MF_TRY(hipMalloc(&p->d_bandt, off * sizeof(int16_t)));
    MF_TRY(hipMalloc(&p->d_band_base, n_problems * sizeof(int32_t)));
    MF_TRY(hipMalloc(&p->d_band_count, n_problems * sizeof(int32_t)));
    MF_TRY(hipMalloc(&p->d_band_scale, std::max(bands, 1) * sizeof(double)));
    MF_TRY(hipMalloc(&p->d_band_amps, std::max(bands, 1) * sizeof(double)));
    MF_TRY(hipMalloc(&p->d_band_modes, std::max(bands, 1) * sizeof(int32_t)));
    MF_TRY(hipMalloc(&p->d_flag, sizeof(int32_t)));
    {
        // problem ids per size class: all of them, then the band-spectrum ones
        std::vector<int32_t> ids;
        for (auto& kv : p->classes) {
            p->class_all[kv.first] = {(int)ids.size(), (int)kv.second.size()};
            ids.insert(ids.end(), kv.second.begin(), kv.second.end());
        }
        for (auto& kv : p->classes) {
            const int off = (int)ids.size();
            for (int pid : kv.second)
                if (p->probs[pid].kind == MF_PK_BANDS) ids.push_back(pid);
            p->class_band[kv.first] = {off, (int)ids.size() - off};
        }
        MF_TRY(hipMalloc(&p->d_class_pids, ids.size() * sizeof(int32_t)));
        MF_TRY(hipMemcpy(p->d_class_pids, ids.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    MF_TRY(hipMemcpy(p->d_probs, pd.data(), n_problems * sizeof(mf::ProbDev), hipMemcpyHostToDevice));
    MF_TRY(hipMemcpy(p->d_nbar, p->host_nbar.data(), off * sizeof(float), hipMemcpyHostToDevice));
    MF_TRY(hipMemcpy(p->d_band_base, bb.data(), n_problems * sizeof(int32_t), hipMemcpyHostToDevice));
    MF_TRY(hipMemcpy(p->d_band_count, bc.data(), n_problems * sizeof(int32_t), hipMemcpyHostToDevice));
    if (p->has_response) {
        MF_TRY(hipMalloc(&p->d_rinv, off * sizeof(float)));
        MF_TRY(hipMemcpy(p->d_rinv, rinv.data(), off * sizeof(float), hipMemcpyHostToDevice));
    }
#undef MF_TRY
    for (int i = 0; i < n_problems; ++i) {
        mf_status st = upload_spectrum(p, i, (hipStream_t)stream);
        if (st != MF_OK) {
            delete p;
            return st;
        }
    }
    for (auto& kv : p->classes) {
        mf_status st = upload_twiddles(p, kv.first.first);
        if (st == MF_OK) st = upload_twiddles(p, kv.first.second);
        if (st != MF_OK) {
            delete p;
            return st;
        }
    }
    {
        // the static scratch of mf_sample_noalloc on this device
        const hipError_t e = mf::static_scratch_setup(p->device);
        if (e != hipSuccess) {
            delete p;
            return fail(MF_ERR_DEVICE, std::string("static scratch setup: ") + hipGetErrorString(e));
        }
    }
    if (flags & MF_FLAG_AUTOTUNE) {
        mf_status st = autotune(p);
        if (st != MF_OK) {
            delete p;
            return st;
        }
    }
    *out = p;
    return MF_OK;
}

mf_status mf_plan_destroy(mf_plan plan) {
    delete plan;
    return MF_OK;
}

mf_status mf_plan_set_spectrum(mf_plan p, int32_t problem, const mf_spectrum* spectrum, mf_stream stream) {
    if (!p || !spectrum || problem < 0 || problem >= (int)p->probs.size())
        return fail(MF_ERR_INVALID_ARG, "bad plan, problem index or spectrum");
    HostProblem& hp = p->probs[problem];
    const int old_kind = hp.kind, old_nb = hp.n_bands;
    HostProblem tmp = hp;
    mf_status st = copy_spectrum(tmp, *spectrum, problem);
    if (st != MF_OK) return st;
    if (tmp.kind != old_kind || tmp.n_bands != old_nb)
        return fail(MF_ERR_INVALID_ARG, "set_spectrum must keep the spectrum kind and band count");
    hp = tmp;
    return upload_spectrum(p, problem, (hipStream_t)stream);
}

mf_status mf_plan_reserve(mf_plan p, const mf_reserve* r) {
    if (!p || !r) return fail(MF_ERR_INVALID_ARG, "plan and reserve are required");
    const uint32_t known = MF_RESERVE_SOLVE | MF_RESERVE_SAMPLE | MF_RESERVE_SPECTRUM | MF_RESERVE_SHEAR |
                           MF_RESERVE_UNROLLED | MF_RESERVE_MOMENTS;
    if (r->calls & ~known) return fail(MF_ERR_INVALID_ARG, "unknown reserve bits");
    const bool chains = r->calls & (MF_RESERVE_SAMPLE | MF_RESERVE_SPECTRUM | MF_RESERVE_SHEAR | MF_RESERVE_MOMENTS);
    if (chains && r->chains_per_problem < 1) return fail(MF_ERR_INVALID_ARG, "chains_per_problem must be >= 1");
    if ((r->calls & MF_RESERVE_SAMPLE) && (r->storage < MF_STORAGE_FP32 || r->storage > MF_STORAGE_BF16))
        return fail(MF_ERR_INVALID_ARG, "unknown storage");
    if ((r->calls & MF_RESERVE_UNROLLED) && (r->unrolled_sweeps < 1 || r->checkpoint_every < 1))
        return fail(MF_ERR_INVALID_ARG, "the unrolled reserve needs unrolled_sweeps >= 1 and checkpoint_every >= 1");
    const hipStream_t s = nullptr;  // allocation only
    const int pairs = (r->chains_per_problem + 1) / 2;
    mf_status st = MF_OK;
    if (r->calls & MF_RESERVE_SOLVE) {
        if ((st = ensure_solve_workspace(p, true, s)) != MF_OK) return st;
        if ((st = ensure_loss_workspace(p, s)) != MF_OK) return st;
    }
    if ((r->calls & MF_RESERVE_SAMPLE) &&
        (st = ensure_sample_workspace(p, pairs, r->storage, MF_FORM_AUTO, true, s)) != MF_OK)
        return st;
    if ((r->calls & MF_RESERVE_SPECTRUM) && (st = ensure_spectrum_workspace(p, pairs, true, s)) != MF_OK) return st;
    if ((r->calls & MF_RESERVE_SHEAR) &&
        (st = ensure_shear_workspace(p, r->chains_per_problem, true, true, true, s)) != MF_OK)
        return st;
    if ((r->calls & MF_RESERVE_UNROLLED) &&
        (st = ensure_unrolled_workspace(p, r->unrolled_sweeps, r->checkpoint_every, s)) != MF_OK)
        return st;
    if ((r->calls & MF_RESERVE_MOMENTS) && (st = ws(p->aux, (size_t)p->total_px * 2 * sizeof(double), s)) != MF_OK)
        return st;
    return MF_OK;
}

int64_t mf_plan_pixel_offset(mf_plan p, int32_t problem) {
    if (!p || problem < 0 || problem > (int)p->probs.size()) return -1;
    if (problem == (int)p->probs.size()) return p->total_px;
    return p->probs[problem].pix_off;
}

double mf_plan_tau(mf_plan p, int32_t problem) {
    if (!p || problem < 0 || problem >= (int)p->probs.size()) return -1;
    return p->probs[problem].tau;
}

int32_t mf_plan_total_bands(mf_plan p) { return p ? p->total_bands : -1; }

mf_status mf_plan_row_shape(mf_plan p, int32_t H, int32_t W, int32_t* rows) {
    if (!p || !rows) return fail(MF_ERR_INVALID_ARG, "plan and rows are required");
    if (!p->classes.count({H, W})) return fail(MF_ERR_INVALID_ARG, "the plan has no problem of that size");
    auto it = p->row_rows.find({H, W});
    int r[8];
    const int n = mf::fused_row_candidates(W, r, 8);
    *rows = it != p->row_rows.end() ? it->second : (n > 0 ? r[0] : 0);
    return MF_OK;
}

mf_status mf_plan_narrow_shape(mf_plan p, int32_t H, int32_t W, int32_t* cols, int32_t* threads, int32_t* rows) {
    if (!p || !cols || !threads || !rows) return fail(MF_ERR_INVALID_ARG, "plan, cols, threads and rows are required");
    if (!p->classes.count({H, W})) return fail(MF_ERR_INVALID_ARG, "the plan has no problem of that size");
    auto it = p->col_shape_narrow.find({H, W});
    int tc = 0, nth = 0;
    mf::narrow_col_shape(H, &tc, &nth);
    if (it != p->col_shape_narrow.end()) {
        tc = it->second.first;
        nth = it->second.second;
    }
    auto rn = p->row_rows_narrow.find({H, W});
    *cols = tc;
    *threads = nth;
    *rows = rn != p->row_rows_narrow.end() ? rn->second : mf::narrow_row_rows(W);
    return MF_OK;
}

mf_status mf_plan_tile_shape(mf_plan p, int32_t H, int32_t W, int32_t* cols, int32_t* threads) {
    if (!p || !cols || !threads) return fail(MF_ERR_INVALID_ARG, "plan, cols and threads are required");
    if (!p->classes.count({H, W})) return fail(MF_ERR_INVALID_ARG, "the plan has no problem of that size");
    const auto sh = class_shape(p, H, W);
    *cols = sh.first;
    *threads = sh.second;
    return MF_OK;
}

mf_status mf_wiener(mf_plan p, const float* d, const mf_schedule* schedule, const float* s_init, float* s_out,
                    mf_info* info, mf_stream stream) {
    if (!p || !d || !s_out) return fail(MF_ERR_INVALID_ARG, "plan, d and s_out are required");
    const float* dd = nullptr;
    mf_status st = plan_data(p, d, (hipStream_t)stream, &dd);
    if (st != MF_OK) return st;
    return run_solve(p, dd, mf::kSrcData, schedule, s_init, s_out, info, (hipStream_t)stream);
}

mf_status mf_wiener_backward(mf_plan p, const float* s_wf, const float* grad_s, const mf_schedule* schedule,
                             float* grad_d, double* grad_bands, float* v_out, mf_info* info, mf_stream stream) {
    if (!p || !grad_s) return fail(MF_ERR_INVALID_ARG, "plan and grad_s are required");
    if (grad_bands && !s_wf) return fail(MF_ERR_INVALID_ARG, "grad_bands needs s_wf");
    return backward_impl(p, s_wf, grad_s, schedule, grad_d, grad_bands, v_out, info, (hipStream_t)stream);
}

mf_status mf_band_loss(mf_plan p, const float* d, const float* s_wf, const float* s_true,
                       const mf_schedule* adjoint_schedule, double* loss_out, float* grad_d, double* grad_bands,
                       mf_info* info, mf_stream stream) {
    if (!p || !d || !s_wf || !s_true || !loss_out)
        return fail(MF_ERR_INVALID_ARG, "plan, d, s_wf, s_true and loss_out are required");
    if ((grad_d || grad_bands) && !adjoint_schedule)
        return fail(MF_ERR_INVALID_ARG, "gradients need an adjoint schedule");
    for (size_t i = 0; i < p->probs.size(); ++i)
        if (p->probs[i].kind != MF_PK_BANDS)
            return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + " has no band spectrum");
    hipStream_t s = (hipStream_t)stream;
    mf_status st = ensure_solve_workspace(p, adjoint_schedule && adjoint_schedule->tol > 0, s);
    if (st != MF_OK) return st;
    if ((st = ensure_loss_workspace(p, s)) != MF_OK) return st;
    const LossWs L = loss_ws(p);
    const float* dd = d;
    if ((st = plan_data(p, d, s, &dd)) != MF_OK) return st;
    // band powers sigma_b = sum_{k in b} |s_k|^2 of the filtered image
    if ((st = mf_band_power(p, s_wf, s_wf, L.power, stream)) != MF_OK) return st;
    // pixel terms: N_eff^-1 (d - s) and the L2 term's s - s_true (the adjoint source)
    std::map<std::pair<int, int>, size_t> part_off;
    size_t off = 0;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        mf::SweepArgs a = base_args(p, H, W);
        if ((st = class_items(p, kv.first, 1, false, false, s, &a.items, &a.n_items)) != MF_OK) return st;
        part_off[kv.first] = off;
        MF_HIP(mf::launch_loss_terms(W, H, a, dd, s_wf, s_true, L.grad_s, L.grad_d, L.part + off, s));
        off += (size_t)a.n_items * mf::kLossBlocks * 2;
    }
    mf_status conv = MF_OK;
    if (grad_d || grad_bands) {
        // implicit part: only the L2 term sends a gradient through s_W (the
        // log-posterior part is stationary there)
        conv = backward_impl(p, s_wf, L.grad_s, adjoint_schedule, grad_d, grad_bands, nullptr, info, s);
        if (conv != MF_OK && conv != MF_ERR_NOT_CONVERGED) return conv;
    }
    if (grad_d) {
        if ((st = data_gradient(p, L.grad_d, s)) != MF_OK) return st;
        MF_HIP(mf::launch_add(L.grad_d, grad_d, p->total_px, s));
    }
    for (auto& kv : p->classes) {
        mf::SweepArgs a = base_args(p, kv.first.first, kv.first.second);
        if ((st = class_items(p, kv.first, 1, false, false, s, &a.items, &a.n_items)) != MF_OK) return st;
        MF_HIP(mf::launch_loss_finish(a, L.part + part_off[kv.first], L.power, p->d_band_amps, p->d_band_modes,
                                      p->d_band_base, p->d_band_count, loss_out, grad_bands, s));
    }
    if (conv != MF_OK) return fail(conv, "adjoint tolerance not reached within max_sweeps");
    return MF_OK;
}

mf_status mf_wiener_backward_unrolled(mf_plan p, const float* d, const mf_schedule* sch, int32_t C,
                                      const float* grad_s, float* s_out, float* grad_d, double* grad_bands,
                                      mf_stream stream) {
    if (!p || !d || !grad_s || !grad_d) return fail(MF_ERR_INVALID_ARG, "plan, d, grad_s and grad_d are required");
    mf_status st = validate_schedule(sch);
    if (st != MF_OK) return st;
    if (sch->tol > 0) return fail(MF_ERR_INVALID_ARG, "the unrolled gradient needs a fixed sweep count (tol <= 0)");
    if (C < 1) return fail(MF_ERR_INVALID_ARG, "checkpoint_every must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    if ((st = plan_data(p, d, s, &d)) != MF_OK) return st;
    std::vector<double> lam;
    for (int j = 0; j < sch->n_levels; ++j)
        for (int k = 0; k < sch->sweeps[j]; ++k) lam.push_back(sch->lambda[j]);
    const int K = (int)lam.size();
    const int ncp = (K + C - 1) / C;
    MF_HIP(mf::launch_zero_words(grad_d, p->total_px, s));
    if (grad_bands && p->total_bands > 0) MF_HIP(mf::launch_zero_words(grad_bands, 2 * (int64_t)p->total_bands, s));
    if (s_out) MF_HIP(mf::launch_zero_words(s_out, p->total_px, s));
    if (K == 0) return MF_OK;  // s_K = s_0 = 0 does not depend on d or P
    if ((st = ensure_unrolled_workspace(p, K, C, s)) != MF_OK) return st;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        const size_t n_cls = (size_t)kv.second.size() * H * W;
        mf::ItemDev* di = nullptr;
        int n_items = 0;
        if ((st = class_items(p, kv.first, 1, true, false, s, &di, &n_items)) != MF_OK) return st;
        const auto sh = class_shape(p, H, W, n_items);
        const size_t n_tiles = (size_t)n_items * ((W + sh.first - 1) / sh.first);
        float2* F = p->field.as<float2>();
        float2* FA = p->field_adj.as<float2>();
        float2* ck = p->ckpt.as<float2>();
        float2* ts = p->tstore.as<float2>();
        mf::SweepArgs a = base_args(p, H, W);
        // the recomputed and reverse sweeps store and load transforms, which only
        // the plain kernels do: the first forward pass runs on them too, so that
        // the recomputed states repeat the checkpointed ones bit for bit
        a.plain_kernels = 1;
        a.items = di;
        a.n_items = n_items;
        a.src = d;
        a.src_kind = mf::kSrcData;
        a.stochastic = 0;
        a.real_only = 1;
        a.band = p->d_band;
        a.grad_d = grad_d;
        // ---- forward sweeps, keeping s_{jC}
        a.field = F;
        MF_HIP(mf::launch_load_real(W, H, a, nullptr, s));
        MF_HIP(mf::launch_zero_words(ck, 2 * (int64_t)n_cls, s));
        for (int k = 1; k <= K; ++k) {
            a.lambda = (float)lam[k - 1];
            a.pix_mode = mf::kPixUpdate;
            a.s_save = (k - 1 > 0 && (k - 1) % C == 0) ? ck + (size_t)((k - 1) / C) * n_cls : nullptr;
            MF_HIP(mf::launch_row(W, H, k == 1 ? mf::kRowFwd : mf::kRowInvFwd, a, s));
            a.s_save = nullptr;
            MF_HIP(launch_col_class(p, W, H, a, s));
        }
        MF_HIP(mf::launch_row(W, H, mf::kRowInv, a, s));
        if (s_out) MF_HIP(mf::launch_copy_out_real(W, H, a, s_out, s));
        // ---- reverse sweeps, each segment recomputed from its checkpoint
        MF_HIP(mf::launch_zero_words(p->slots.p, 2 * (int64_t)n_tiles * mf::kMaxBandsPerProblem, s));
        mf::SweepArgs b = a;
        b.field = FA;
        b.band_slots = p->slots.as<double>();
        MF_HIP(mf::launch_load_real(W, H, b, grad_s, s));
        bool first = true;
        for (int j = ncp - 1; j >= 0; --j) {
            const int k0 = j * C, k1 = std::min(K, k0 + C);
            mf::SweepArgs f = a;
            f.field = F;
            MF_HIP(mf::launch_init_items(W, H, f, ck + (size_t)j * n_cls, 0.f, s));
            for (int k = k0 + 1; k <= k1; ++k) {
                f.lambda = (float)lam[k - 1];
                f.pix_mode = mf::kPixUpdate;
                MF_HIP(mf::launch_row(W, H, k == k0 + 1 ? mf::kRowFwd : mf::kRowInvFwd, f, s));
                f.t_store = ts + (size_t)(k - k0 - 1) * n_cls;
                MF_HIP(launch_col_class(p, W, H, f, s));
                f.t_store = nullptr;
            }
            for (int k = k1; k >= k0 + 1; --k) {
                mf::SweepArgs r = b;
                if (first) {
                    r.pix_mode = mf::kPixIdentity;
                    MF_HIP(mf::launch_row(W, H, mf::kRowFwd, r, s));
                } else {
                    r.pix_mode = mf::kPixAdjoint;  // transpose of sweep k+1's pixel step
                    r.lambda = (float)lam[k];
                    MF_HIP(mf::launch_row(W, H, mf::kRowInvFwd, r, s));
                }
                first = false;
                r.lambda = (float)lam[k - 1];
                r.t_load = ts + (size_t)(k - k0 - 1) * n_cls;
                MF_HIP(launch_col_class(p, W, H, r, s));
            }
        }
        mf::SweepArgs r = b;
        r.pix_mode = mf::kPixAdjoint;  // transpose of sweep 1's pixel step
        r.lambda = (float)lam[0];
        MF_HIP(mf::launch_row(W, H, mf::kRowInv, r, s));
        if (grad_bands && p->total_bands > 0)
            MF_HIP(mf::launch_band_slots_reduce(W, H, sh.first, r, p->d_band_base, p->d_band_count, grad_bands, s));
    }
    return data_gradient(p, grad_d, s);
}

mf_status mf_shear_wiener(mf_plan p, const float* gamma, const mf_schedule* sch, float b_ratio, float* kappa_out,
                          mf_stream stream) {
    if (!p || !gamma || !kappa_out) return fail(MF_ERR_INVALID_ARG, "plan, gamma and kappa_out are required");
    mf_status st = validate_schedule(sch);
    if (st != MF_OK) return st;
    if (sch->tol > 0) return fail(MF_ERR_INVALID_ARG, "the shear filter runs a fixed schedule (tol <= 0)");
    if (!(b_ratio >= 0.f) || !std::isfinite(b_ratio)) return fail(MF_ERR_INVALID_ARG, "b_ratio must be >= 0");
    if ((st = shear_check(p)) != MF_OK) return st;
    std::vector<double> lam(sch->lambda, sch->lambda + sch->n_levels);
    std::vector<int32_t> sw(sch->sweeps, sch->sweeps + sch->n_levels);
    int total = 0;
    for (int k : sw) total += k;
    if (total < 1) return fail(MF_ERR_INVALID_ARG, "the schedule runs no sweep");
    return launch_shear(p, gamma, b_ratio, 1, lam, sw, 0, 0, 0, 0, 0, 1, nullptr, nullptr, nullptr, kappa_out, false,
                        (hipStream_t)stream);
}

mf_status mf_shear_sample(mf_plan p, const float* gamma, const mf_shear_args* g, const float* state_in,
                          float* state_out, float* samples_out, mf_stream stream) {
    if (!p || !gamma || !g) return fail(MF_ERR_INVALID_ARG, "plan, gamma and args are required");
    if (g->chains_per_problem < 1 || g->burn_in < 0 || g->n_samples < 0 || g->thin < 1 || g->sweep_offset < 0 ||
        !(g->b_ratio >= 0.f) || !std::isfinite(g->b_ratio))
        return fail(MF_ERR_INVALID_ARG,
                    "need chains >= 1, burn_in >= 0, n_samples >= 0, thin >= 1, sweep_offset >= 0, b_ratio >= 0");
    const int64_t K = (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin;
    if (g->sweep_offset + K > 0xffffffffLL || K > 0x7fffffffLL)
        return fail(MF_ERR_INVALID_ARG, "sweep index exceeds 2^32");
    mf_status st = shear_check(p);
    if (st != MF_OK) return st;
    if (K == 0) return MF_OK;
    return launch_shear(p, gamma, g->b_ratio, g->chains_per_problem, {1.0}, {(int32_t)K}, 1, g->seed,
                        g->sweep_offset, g->burn_in, g->n_samples, g->thin, state_in, state_out, samples_out,
                        nullptr, g->check_finite != 0, (hipStream_t)stream);
}

mf_status mf_sample_moments(mf_plan p, const float* samples, int32_t chains, int32_t n_samples, double* mean_out,
                            double* var_out, mf_stream stream) {
    if (!p || !samples || !mean_out) return fail(MF_ERR_INVALID_ARG, "plan, samples and mean_out are required");
    if (chains < 1 || n_samples < 1) return fail(MF_ERR_INVALID_ARG, "need chains >= 1 and n_samples >= 1");
    hipStream_t s = (hipStream_t)stream;
    mf_status st = ws(p->aux, (size_t)p->total_px * 2 * sizeof(double), s);
    if (st != MF_OK) return st;
    MF_HIP(mf::launch_moments(p->d_probs, (int)p->probs.size(), p->total_px, samples, (int64_t)chains * n_samples,
                              p->aux.as<double2>(), mean_out, var_out, s));
    return MF_OK;
}

mf_status mf_band_power(mf_plan p, const float* x, const float* y, double* out, mf_stream stream) {
    if (!p || !x || !y || !out) return fail(MF_ERR_INVALID_ARG, "plan, x, y and out are required");
    hipStream_t s = (hipStream_t)stream;
    mf_status st = ensure_solve_workspace(p, false, s);
    if (st != MF_OK) return st;
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        mf::SweepArgs a = base_args(p, H, W);
        if ((st = class_items(p, kv.first, 1, false, true, s, &a.items, &a.n_items)) != MF_OK) return st;
        if (a.n_items == 0) continue;
        a.field = p->field.as<float2>();
        a.partials = p->partials.as<double>();
        MF_HIP(mf::launch_band_power(W, H, a, x, y, p->d_band, p->d_band_base, p->d_band_count, nullptr, out, s));
    }
    return MF_OK;
}

mf_status mf_sample(mf_plan p, const float* d, const mf_sample_args* g, const float* state_in, float* state_out,
                    float* samples_out, mf_stream stream) {
    if (!p || !d || !g) return fail(MF_ERR_INVALID_ARG, "plan, d and args are required");
    hipStream_t s = (hipStream_t)stream;
    mf_status st = validate_sample(g, state_out, samples_out);
    if (st != MF_OK) return st;
    const int pairs = (g->chains_per_problem + 1) / 2;
    if ((st = ensure_sample_workspace(p, pairs, g->storage, g->form, !state_out, s)) != MF_OK) return st;
    SampleWs w;
    w.items = p->items.as<mf::ItemDev>();
    w.items_cap = p->items.bytes / sizeof(mf::ItemDev);
    w.coef = p->coef.as<float4>();
    w.dprime = p->dprime.as<float>();
    w.field = p->field.as<float2>();
    w.hfield = p->hfield.as<float2>();
    return sample_impl(p, d, g, state_in, state_out, samples_out, w, s);
}

mf_status mf_sample_noalloc(mf_plan p, const float* d, const mf_sample_args* g, const float* state_in,
                            float* state_out, float* samples_out, mf_stream stream) {
    if (!p || !d || !g) return fail(MF_ERR_INVALID_ARG, "plan, d and args are required");
    if (!state_out) return fail(MF_ERR_INVALID_ARG, "mf_sample_noalloc needs state_out (the chains' work field)");
    mf_status st = validate_sample(g, state_out, samples_out);
    if (st != MF_OK) return st;
    int dev = -1;
    MF_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(MF_ERR_INVALID_ARG, "the plan's device must be current");
    char* base = static_cast<char*>(mf::static_scratch(dev));
    if (!base) return fail(MF_ERR_DEVICE, "the static scratch of this device is not set up");
    // layout: work lists, persistent tables, d / A, 16-bit field (256-byte aligned)
    const int pairs = (g->chains_per_problem + 1) / 2;
    size_t max_items = 0;
    for (auto& kv : p->classes) max_items = std::max(max_items, kv.second.size() * (size_t)pairs);
    const size_t items_b = align256((max_items + 1) * sizeof(mf::ItemDev));
    const size_t coef_b = sample_any_persistent(p, g->form)
                              ? align256((size_t)p->total_px / 2 * (sizeof(float4) + sizeof(float2) + sizeof(float4)))
                              : 0;
    const size_t dp_b = p->has_response ? align256((size_t)p->total_px * sizeof(float)) : 0;
    const size_t hf_b = g->storage != MF_STORAGE_FP32 ? align256((size_t)p->total_px * pairs * 4) : 0;
    const size_t need = items_b + coef_b + dp_b + hf_b;
    if (need > mf::kStaticScratchBytes)
        return fail(MF_ERR_INVALID_ARG, "mf_sample_noalloc needs " + std::to_string(need) +
                                            " bytes of scratch for this plan and call; the static scratch holds " +
                                            std::to_string(mf::kStaticScratchBytes));
    SampleWs w;
    w.items = reinterpret_cast<mf::ItemDev*>(base);
    w.items_cap = max_items + 1;
    w.coef = coef_b ? reinterpret_cast<float4*>(base + items_b) : nullptr;
    w.dprime = dp_b ? reinterpret_cast<float*>(base + items_b + coef_b) : nullptr;
    w.hfield = hf_b ? reinterpret_cast<float2*>(base + items_b + coef_b + dp_b) : nullptr;
    w.graphs = false;
    return sample_impl(p, d, g, state_in, state_out, samples_out, w, (hipStream_t)stream);
}

mf_status mf_sample_spectrum(mf_plan p, const float* d, const mf_spectrum_args* g, const float* state_in,
                             const double* theta_in, float* state_out, double* theta_out, float* samples_out,
                             double* theta_samples_out, mf_stream stream) {
    if (!p || !d || !g) return fail(MF_ERR_INVALID_ARG, "plan, d and args are required");
    if (g->chains_per_problem < 1 || g->burn_in < 0 || g->n_samples < 0 || g->thin < 1 || g->sweeps_per_draw < 1 ||
        g->iteration_offset < 0 || !(g->prior_beta >= 0) || !std::isfinite(g->prior_beta))
        return fail(MF_ERR_INVALID_ARG,
                    "need chains >= 1, burn_in >= 0, n_samples >= 0, thin >= 1, sweeps_per_draw >= 1, "
                    "iteration_offset >= 0, prior_beta >= 0");
    const int64_t iters = (int64_t)g->burn_in + (int64_t)g->n_samples * g->thin;
    if ((g->iteration_offset + iters) * (int64_t)g->sweeps_per_draw > 0xffffffffLL)
        return fail(MF_ERR_INVALID_ARG, "sweep index exceeds 2^32");
    for (size_t i = 0; i < p->probs.size(); ++i) {
        const HostProblem& hp = p->probs[i];
        if (hp.kind != MF_PK_BANDS)
            return fail(MF_ERR_INVALID_ARG, "problem " + std::to_string(i) + " has no band spectrum");
    }
    mf_status st0 = pow2_sides(p, "the hierarchical sampler");
    if (st0 != MF_OK) return st0;
    hipStream_t s = (hipStream_t)stream;
    const int pairs = (g->chains_per_problem + 1) / 2;
    st0 = ensure_spectrum_workspace(p, pairs, !state_out, s);
    if (st0 != MF_OK) return st0;
    if ((st0 = plan_data(p, d, s, &d)) != MF_OK) return st0;
    float2* work = state_out ? reinterpret_cast<float2*>(state_out) : p->field.as<float2>();
    // degrees of freedom per band (modes + prior_dof, at least 0) on the
    // device; the start amplitudes are the plan's
    const int nbt = p->total_bands;
    std::vector<int32_t> dof(nbt);
    for (const HostProblem& hp : p->probs)
        for (int b = 0; b < hp.n_bands; ++b) dof[hp.band_base + b] = std::max(0, hp.band_modes[b] + g->prior_dof);
    int32_t* d_dof = p->spec.as<int32_t>();
    MF_HIP(mf::launch_band_dof(p->d_band_modes, g->prior_dof, d_dof, nbt, s));
    const double* d_th0 = p->d_band_amps;
    // pixel tables of the sampler (the pixel step does not depend on the spectrum)
    const size_t half = (size_t)p->total_px / 2;
    float4* pcoef = p->coef.as<float4>();
    float2* psrc = reinterpret_cast<float2*>(pcoef + half);
    float4* mcoef = reinterpret_cast<float4*>(psrc + half);
    MF_HIP(mf::launch_sampler_coefs(p->d_probs, (int)p->probs.size(), d, p->d_nbar, p->d_nP, pcoef, psrc, mcoef, s));
    if (g->check_finite) MF_HIP(mf::launch_fill_int(p->d_flag, INT32_MAX, 1, s));
    for (auto& kv : p->classes) {
        const int H = kv.first.first, W = kv.first.second;
        mf::ItemDev* di = nullptr;
        int n_items = 0;
        mf_status st = class_items(p, kv.first, pairs, false, false, s, &di, &n_items);
        if (st != MF_OK) return st;
        if (!mf::resident_supported(H, W)) {
            int max_dof = 0;
            for (int pid : kv.second) {
                int tot = 0;
                for (int b = 0; b < p->probs[pid].n_bands; ++b) tot += dof[p->probs[pid].band_base + b];
                max_dof = std::max(max_dof, tot);
            }
            st = spectrum_streamed(p, di, n_items, H, W, max_dof, d, g, work,
                                   reinterpret_cast<const float2*>(state_in), theta_in, theta_out, samples_out,
                                   theta_samples_out, d_dof, d_th0, s);
            if (st != MF_OK) return st;
        } else {
        mf::SpectrumArgs r{};
        r.probs = p->d_probs;
        r.items = di;
        r.n_items = n_items;
        r.field = work;
        r.state_in = reinterpret_cast<const float2*>(state_in);
        r.init_scale = g->init_scale;
        r.pcoef = pcoef;
        r.psrc = psrc;
        r.tw = p->d_tw.at(H);
        r.key0 = (uint32_t)(g->seed & 0xffffffffu);
        r.key1 = (uint32_t)(g->seed >> 32);
        r.iter0 = (uint32_t)g->iteration_offset;
        r.sweeps = g->sweeps_per_draw;
        r.burn_in = g->burn_in;
        r.n_samples = g->n_samples;
        r.thin = g->thin;
        r.samples = samples_out;
        r.chains = g->chains_per_problem;
        r.chains_pad = 2 * pairs;
        r.band = p->d_band;
        r.band_base = p->d_band_base;
        r.band_count = p->d_band_count;
        r.dof = d_dof;
        r.theta0 = d_th0;
        r.theta_in = theta_in;
        r.theta_out = theta_out;
        r.theta_samples = theta_samples_out;
        r.prior_beta = g->prior_beta;
        MF_HIP(mf::launch_resident_spectrum(H, r, s));
        }
        if (g->check_finite) {
            mf::SweepArgs chk = base_args(p, H, W);
            chk.items = di;
            chk.n_items = n_items;
            chk.field = work;
            MF_HIP(mf::launch_finite_check(W, H, chk, p->d_flag, s));
        }
    }
    return g->check_finite ? read_finite_flag(p, s) : MF_OK;
}

}  // extern "C"
