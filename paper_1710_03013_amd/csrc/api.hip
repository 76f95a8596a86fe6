// C ABI entry points kkm_fit / kkm_assign / kkm_cost: argument checks, workspace layout and the
// per-batch launch sequence.  All arithmetic runs in the kernels of k_landmark / k_dist / k_select.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {
namespace {

// HIP events recorded on the caller's stream at the boundaries of the phases of a fit (optional):
// back-to-back phases share their boundary event.  The events only time the stream, so they are
// recorded without the system-scope fences (whose cache maintenance stalls the queue for several
// microseconds per event).
// Timed spans of a fit: k-means++ / medoids; landmark block and initial labels; landmark loop kernel;
// batch-wide distance kernel; FP64 re-decision; selection (column minima, medoids, merge).
enum { kPhInit = 0, kPhLandmark = 1, kPhLoop = 2, kPhDist = 3, kPhRefine = 4, kPhSelect = 5, kPhases = 6 };

// Process-wide free list of timing events per device.  A fit borrows events and hands them back when
// it returns, so fits running concurrently on other host threads never share one, and later fits
// reuse them (creating events is host work on every fit otherwise).  The pool is created on first
// use and deliberately never destroyed: nothing of it runs during process teardown, when the HIP
// runtime may already be shutting down.
struct EventPool {
    std::mutex mu;
    std::map<int, std::vector<hipEvent_t>> free;
    static EventPool& get() {
        static EventPool* p = new EventPool;
        return *p;
    }
    kkm_status take(int device, hipEvent_t* e) {
        {
            std::lock_guard<std::mutex> lock(mu);
            auto& f = free[device];
            if (!f.empty()) {
                *e = f.back();
                f.pop_back();
                return KKM_OK;
            }
        }
        KKM_HIP(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
        return KKM_OK;
    }
    void give(int device, const std::vector<hipEvent_t>& evs) {
        std::lock_guard<std::mutex> lock(mu);
        auto& f = free[device];
        f.insert(f.end(), evs.begin(), evs.end());
    }
};

struct PhaseTimer {
    bool on = false;
    unsigned mask = ~0u;       // phases that are timed
    hipStream_t s = nullptr;
    int device = 0;
    std::vector<hipEvent_t> evs;                                    // borrowed from the pool
    std::vector<std::pair<int, std::pair<size_t, size_t>>> spans;   // (phase, (begin, end) indices into evs)
    size_t open = 0;
    bool open_valid = false;   // the last recorded event ends a phase and may begin the next one
    PhaseTimer() = default;
    PhaseTimer(const PhaseTimer&) = delete;
    PhaseTimer& operator=(const PhaseTimer&) = delete;
    ~PhaseTimer() {
        if (!evs.empty()) EventPool::get().give(device, evs);
    }
    kkm_status record(size_t* slot) {
        hipEvent_t e;
        KKM_TRY(EventPool::get().take(device, &e));
        evs.push_back(e);
        *slot = evs.size() - 1;
        KKM_HIP(hipEventRecord(e, s));
        return KKM_OK;
    }
    bool timed(int phase) const { return on && ((mask >> phase) & 1u); }
    // begin() right after end() (no launch in between) reuses that end event
    kkm_status begin(int phase) {
        if (!timed(phase) || open_valid) return KKM_OK;
        KKM_TRY(record(&open));
        open_valid = true;
        return KKM_OK;
    }
    kkm_status end(int phase) {
        if (!on) return KKM_OK;
        if (!timed(phase)) {
            open_valid = false;
            return KKM_OK;
        }
        size_t e;
        KKM_TRY(record(&e));
        spans.push_back({phase, {open, e}});
        open = e;
        open_valid = true;
        return KKM_OK;
    }
    // a launch outside every phase follows: the next phase records its own begin event
    void gap() { open_valid = false; }
    // after the stream has been synchronised
    void collect(double out[kPhases]) {
        for (int p = 0; p < kPhases; ++p) out[p] = 0.0;
        for (auto& sp : spans) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, evs[sp.second.first], evs[sp.second.second]) == hipSuccess) out[sp.first] += ms;
        }
    }
};

// ----------------------------------------------------------------------------- fixed scratch
// Scratch of kkm_assign_noalloc: a file-scope device array, one copy per GPU the library runs on,
// held until the process ends.  Host code never uses the array's name as an address (on the host it
// is only a stand-in for the symbol): the device address of each GPU's copy is looked up once with
// hipGetSymbolAddress while that GPU is current, and that pointer is what kernels and copies get.
constexpr size_t kNoAllocScratchBytes = size_t(48) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

kkm_status noalloc_scratch(int device, void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        int cur = -1;
        KKM_HIP(hipGetDevice(&cur));
        if (cur != device) return fail(KKM_ERR_INVALID_ARG, "the model lives on another device than the current one");
        void* p = nullptr;
        KKM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        it = addr.emplace(device, p).first;
    }
    *out = it->second;
    return KKM_OK;
}

// ----------------------------------------------------------------------------- fit plan
struct FitPlan {
    int64_t N = 0, d = 0;
    int dtype = KKM_F32;
    kkm_kernel kernel{};
    kkm_params p{};
    int B = 0, C = 0, T = 0;
    int dpad = 0;
    std::vector<int64_t> n, base, stride, ell, lm_off;
    int64_t nmax = 0, ellmax = 0, ell_total = 0;
    int gmax = 1;
    int nchunk = 1;
    int64_t cand_cap = 1;
    bool tile_f64 = false;
    std::vector<int32_t> lm_host;      // concatenated batch positions
    std::vector<double> uniforms;      // k-means++
    std::vector<int32_t> lab0;         // landmark labels of batch 0 (random init)
    std::vector<int32_t> med0;         // batch-0 medoid positions (explicit init)
};

// ----------------------------------------------------------------------------- assign workspace
struct AssignWs {
    void* Qc;
    float* r2buf;          // RMSD pair pass (matrix cores): squared RMSDs of a chunk of frames
    double* r2gq;
    int64_t rmsd_chunk;
    int32_t* refine_list;
    int32_t* refine_count;
    int32_t* nonfinite;
    double* best;
    double* partials;
    double* cost;
    int32_t* labels_tmp;   // labels when the caller wants only the cost
    uint32_t* gate;        // [ceil(n / 32)] rows the plain BF16 pass leaves undecided
};

struct FitWs {
    void* Xc;
    float* r2buf;          // RMSD pair pass (matrix cores) of the batch pass
    double* r2gq;
    int64_t rmsd_chunk;
    int32_t* lm;
    int32_t* lab_init;
    double* uniforms;
    int32_t* chosen;
    double* D2;
    double* kpp_part;
    void* M;
    double* Mself;
    int64_t* Midx;
    int64_t* wcount;
    double* Kbuf;
    double* Kmed;
    int32_t* lab;
    int32_t* nlab_x;
    double* sx;
    double* partial;
    int32_t* changed;
    int32_t* lab_final;
    int32_t* offsets;
    double* ghat;
    double* segabs;
    void* support;
    float* snorm32;
    double* snorm64;
    float* coef32;
    double* coef64;
    float* sup_pan;
    uint16_t* sup_hi;
    uint16_t* sup_lo;
    int32_t* src_index;
    float* snorm_max;
    int32_t* split;        // [5]
    int32_t* counts_b;     // [C+1] cleared by the landmark phase of each batch; [C] = candidate count
    unsigned long long* colmin;   // [C]
    double* colpart;              // [C][dist_block_cap(nmax)]
    int32_t* cand_q;
    int32_t* cand_j;
    double* cand_v;
    float* Dt;
    float* Erow;
    int32_t* labels_b;
    int32_t* refine_list;
    int32_t* refine_counts; // [B]
    int32_t* flags;        // [2] nonfinite, medoid candidates
    int32_t* bmed;
    int32_t* mpart_c;
    double* tpan;          // merge targets [C][2][dpad] and their norms [C][2]
    double* tnorm;
    double* gpart_v;
    int32_t* gpart_i;
    int32_t* updates;      // [B]
    int64_t* info;         // [3][B][C] batch medoids, counts, global medoids
    double* info_disp;     // [B][C] displacement of every global medoid per batch
    double* pcost;         // [B] partial cost of every batch
    double* gcost;         // [B] global cost after every batch (KKM_FIT_GLOBAL_COST)
    kkm_model gmodel;      // the global medoids as a model in the workspace (KKM_FIT_GLOBAL_COST)
    AssignWs gws;          // its assign pass over all N rows
    double* best;          // [nmax] each batch row's distance to its nearest centroid (partial cost)
    double* psum;          // [1024] partial sums of the partial cost
    int64_t* trace;        // [64]
    int32_t* lm_error;     // [1]
    char* status_end;      // end of the status block (refine_counts .. trace)
};

size_t carve_assign(Carver& c, const kkm_model* m, int64_t n, AssignWs& w);
kkm_status assign_launch(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision, hipStream_t s,
                         int32_t* labels, float* gap, bool want_best, const AssignWs& w);

size_t carve_fit(Carver& c, const FitPlan& P, FitWs& w) {
    const size_t es = P.dtype == KKM_F64 ? 8 : 4;
    const int C = P.C;
    w.Xc = P.kernel.type == KKM_KERNEL_RMSD ? c.take<char>((size_t)P.N * P.d * es) : nullptr;
    w.r2buf = nullptr;
    w.r2gq = nullptr;
    w.rmsd_chunk = 0;
    if (P.kernel.type == KKM_KERNEL_RMSD && !P.tile_f64) {
        w.rmsd_chunk = rmsd_chunk_groups(P.nmax, P.ellmax, kRmsdFitChunkBytes);
        w.r2buf = c.take<float>((size_t)w.rmsd_chunk * std::max<int64_t>(1, (P.ellmax + 31) / 32) * 1024);
        w.r2gq = c.take<double>((size_t)w.rmsd_chunk * 32);
    }
    w.lm = c.take<int32_t>(std::max<int64_t>(1, P.ell_total));
    w.lab_init = c.take<int32_t>(P.ellmax);
    w.uniforms = c.take<double>(C);
    w.chosen = c.take<int32_t>(C);
    w.D2 = c.take<double>(2 * P.nmax);
    w.kpp_part = c.take<double>(3 * 256);
    w.M = c.take<char>((size_t)C * P.dpad * es);
    w.Mself = c.take<double>(C);
    w.Midx = c.take<int64_t>(C);
    w.wcount = c.take<int64_t>(C);
    w.Kbuf = c.take<double>((size_t)P.ellmax * landmark_ldk(P.ellmax));
    w.Kmed = c.take<double>((size_t)P.ellmax * C);
    w.lab = c.take<int32_t>(2 * P.ellmax);
    w.nlab_x = c.take<int32_t>((size_t)2 * P.ellmax);
    w.sx = c.take<double>((size_t)4 * P.ellmax);
    w.partial = c.take<double>((size_t)3 * P.gmax * C);
    w.changed = c.take<int32_t>(P.T + 1);
    w.lab_final = c.take<int32_t>(P.ellmax);
    w.offsets = c.take<int32_t>(C + 1);
    w.ghat = c.take<double>(C);
    w.segabs = c.take<double>(C);
    const size_t srows = (size_t)P.ellmax + 32;   // whole 32-row tiles for the matrix-core pass
    w.support = c.take<char>(srows * P.dpad * es);
    w.snorm32 = c.take<float>(srows);
    w.snorm64 = c.take<double>(srows);
    w.coef32 = c.take<float>(srows);
    w.coef64 = c.take<double>(srows);
    w.sup_pan = P.dtype == KKM_F32 ? c.take<float>(panel_rows(srows) * P.dpad) : nullptr;
    w.sup_hi = c.take<uint16_t>(panel_rows(srows) * bf16_pad(P.dpad));
    w.sup_lo = c.take<uint16_t>(panel_rows(srows) * bf16_pad(P.dpad));
    w.src_index = c.take<int32_t>(P.ellmax);
    w.snorm_max = c.take<float>(1);
    w.split = c.take<int32_t>(5);
    w.counts_b = c.take<int32_t>(C + 1);
    w.colmin = c.take<unsigned long long>(C);
    w.colpart = c.take<double>((size_t)C * dist_block_cap(P.nmax));
    w.cand_q = c.take<int32_t>((size_t)P.cand_cap);
    w.cand_j = c.take<int32_t>((size_t)P.cand_cap);
    w.cand_v = c.take<double>((size_t)P.cand_cap);
    w.Dt = c.take<float>((size_t)C * P.nmax * (P.tile_f64 ? 2 : 1));
    w.Erow = c.take<float>(P.nmax);
    w.labels_b = c.take<int32_t>(P.nmax);
    w.refine_list = c.take<int32_t>(P.nmax);
    w.best = c.take<double>(P.nmax);
    w.psum = c.take<double>(1024);
    w.bmed = c.take<int32_t>(C);
    w.mpart_c = c.take<int32_t>((size_t)C * P.nchunk);
    w.tpan = c.take<double>((size_t)C * 2 * P.dpad);
    w.tnorm = c.take<double>((size_t)C * 2);
    w.gpart_v = c.take<double>((size_t)C * merge_chunks(P.nmax));
    w.gpart_i = c.take<int32_t>((size_t)C * merge_chunks(P.nmax));
    // status block, read back with one copy: [refine_counts, flags, updates, lm_error, info, info_disp, trace]
    w.refine_counts = c.take<int32_t>(P.B);
    w.flags = c.take<int32_t>(2);
    w.updates = c.take<int32_t>(P.B);
    w.lm_error = c.take<int32_t>(1);
    w.info = c.take<int64_t>((size_t)3 * P.B * C);
    w.info_disp = c.take<double>((size_t)P.B * C);
    w.pcost = c.take<double>((size_t)P.B);
    w.gcost = c.take<double>((size_t)P.B);
    w.trace = c.take<int64_t>(64);
    w.status_end = c.take<char>(1);
    if (P.p.flags & KKM_FIT_GLOBAL_COST) {   // the global medoids as a model, and an assign pass over N
        kkm_model& m = w.gmodel;
        m = kkm_model{};
        m.kernel = P.kernel;
        m.d = P.d;
        m.dpad = P.dpad;
        m.bpad = bf16_pad(P.dpad);
        m.C = C;
        m.cap = C;
        m.used = C;
        m.dtype = P.dtype;
        model_layout(&m, c);
        carve_assign(c, &m, P.N, w.gws);
    }
    return c.off;
}

kkm_status check_kernel_args(const kkm_kernel* k, int64_t d) {
    if (!k) return fail(KKM_ERR_INVALID_ARG, "kernel is NULL");
    if (k->type != KKM_KERNEL_LINEAR && k->type != KKM_KERNEL_RBF && k->type != KKM_KERNEL_RMSD)
        return fail(KKM_ERR_INVALID_ARG, "unknown kernel type");
    if (k->type != KKM_KERNEL_LINEAR && !(k->sigma > 0.0 && std::isfinite(k->sigma)))
        return fail(KKM_ERR_INVALID_ARG, "sigma must be finite and > 0");
    if (k->type == KKM_KERNEL_RMSD && (k->n_atoms < 1 || d != 3 * (int64_t)k->n_atoms))
        return fail(KKM_ERR_INVALID_ARG, "RMSD kernel needs d == 3 * n_atoms");
    if (k->type != KKM_KERNEL_RMSD && d > kMaxRegDim) return fail(KKM_ERR_UNSUPPORTED, "linear / RBF support d <= 128");
    return KKM_OK;
}

double inv2s2_of(const kkm_kernel& k) { return k.type == KKM_KERNEL_LINEAR ? 0.0 : 1.0 / (2.0 * k.sigma * k.sigma); }

// Validate everything and build the plan (host draws included); no device work.
kkm_status finish_plan(FitPlan& P, const DeviceInfo* dev);

// draws = false: sizes only (no landmark positions or initialisation draws), for the workspace query
kkm_status make_plan(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel, const kkm_params* params,
                     const DeviceInfo* dev, FitPlan& P, bool draws = true) {
    if (N < 1) return fail(KKM_ERR_INVALID_ARG, "N must be >= 1");
    if (d < 1) return fail(KKM_ERR_INVALID_ARG, "d must be >= 1");
    if (dtype != KKM_F32 && dtype != KKM_F64) return fail(KKM_ERR_INVALID_ARG, "bad dtype");
    KKM_TRY(check_kernel_args(kernel, d));
    if (!params) return fail(KKM_ERR_INVALID_ARG, "params is NULL");
    const kkm_params& p = *params;
    if (p.B < 1 || p.B > N) return fail(KKM_ERR_INVALID_ARG, "B must be in [1, N]");
    if (!(p.s > 0.0 && p.s <= 1.0)) return fail(KKM_ERR_INVALID_ARG, "s must be in (0, 1]");
    if (p.max_iter < 1 || p.max_iter > 100000) return fail(KKM_ERR_INVALID_ARG, "max_iter must be in [1, 100000]");
    if (p.sampling != KKM_SAMPLE_STRIDE && p.sampling != KKM_SAMPLE_BLOCK) return fail(KKM_ERR_INVALID_ARG, "bad sampling");
    if (p.init != KKM_INIT_KMEANSPP && p.init != KKM_INIT_RANDOM_LABELS && p.init != KKM_INIT_MEDOIDS)
        return fail(KKM_ERR_INVALID_ARG, "bad init");
    if (p.precision < KKM_PREC_FP64 || p.precision > KKM_PREC_BF16X3)
        return fail(KKM_ERR_INVALID_ARG, "bad precision");
    if (p.flags & ~(KKM_FIT_COOPERATIVE | KKM_FIT_GLOBAL_COST)) return fail(KKM_ERR_INVALID_ARG, "unknown fit flags");
    P.N = N;
    P.d = d;
    P.dtype = dtype;
    P.kernel = *kernel;
    P.p = p;
    P.B = p.B;
    P.C = p.C;
    P.T = p.max_iter;
    P.dpad = kernel->type == KKM_KERNEL_RMSD ? (int)d : padded_dim(d);
    P.n.resize(P.B);
    P.base.resize(P.B);
    P.stride.resize(P.B);
    for (int i = 0; i < P.B; ++i) {
        if (p.sampling == KKM_SAMPLE_STRIDE) {
            P.base[i] = i;
            P.stride[i] = P.B;
            P.n[i] = (N - i + P.B - 1) / P.B;
        } else {
            const int64_t q = N / P.B, r = N % P.B;
            P.n[i] = q + (i < r ? 1 : 0);
            P.base[i] = i * q + std::min<int64_t>(i, r);
            P.stride[i] = 1;
        }
    }
    if (p.C < 1 || p.C > kMaxClusters) return fail(KKM_ERR_INVALID_ARG, "C must be in [1, 1024]");
    if (p.C > P.n[0]) return fail(KKM_ERR_INVALID_ARG, "C exceeds the size of the first batch");
    P.ell.resize(P.B);
    P.lm_off.resize(P.B + 1);
    P.lm_off[0] = 0;
    for (int i = 0; i < P.B; ++i) {
        P.ell[i] = kkm_landmark_count(P.n[i], p.s);
        P.lm_off[i + 1] = P.lm_off[i] + P.ell[i];
        P.nmax = std::max(P.nmax, P.n[i]);
        P.ellmax = std::max(P.ellmax, P.ell[i]);
    }
    P.ell_total = P.lm_off[P.B];
    if (P.ellmax > 65535) return fail(KKM_ERR_UNSUPPORTED, "at most 65535 landmarks per batch; use more mini-batches");
    if (!draws) return finish_plan(P, dev);
    P.lm_host.resize(P.ell_total);
    std::vector<int64_t> tmp(P.ellmax);
    for (int i = 0; i < P.B; ++i) {
        const int64_t* src;
        if (p.landmarks) {
            src = p.landmarks + P.lm_off[i];
        } else {
            KKM_TRY(kkm_draw_landmarks(p.seed, i, P.n[i], p.s, tmp.data()));
            src = tmp.data();
        }
        for (int64_t k = 0; k < P.ell[i]; ++k) {
            if (src[k] < 0 || src[k] >= P.n[i] || (k > 0 && src[k] <= src[k - 1]))
                return fail(KKM_ERR_INVALID_ARG, "landmarks of batch " + std::to_string(i) +
                                                     " must be strictly ascending positions inside the batch");
            P.lm_host[P.lm_off[i] + k] = (int32_t)src[k];
        }
    }
    if (p.init == KKM_INIT_KMEANSPP) {
        P.uniforms.resize(P.C);
        if (p.kmpp_uniforms) std::copy(p.kmpp_uniforms, p.kmpp_uniforms + P.C, P.uniforms.begin());
        else KKM_TRY(kkm_draw_kmpp_uniforms(p.seed, P.C, P.uniforms.data()));
        for (double u : P.uniforms)
            if (!(u >= 0.0 && u < 1.0)) return fail(KKM_ERR_INVALID_ARG, "k-means++ uniforms must lie in [0, 1)");
    } else if (p.init == KKM_INIT_RANDOM_LABELS) {
        std::vector<int32_t> labs(P.n[0]);
        if (p.init_labels) std::copy(p.init_labels, p.init_labels + P.n[0], labs.begin());
        else KKM_TRY(kkm_draw_init_labels(p.seed, P.n[0], P.C, labs.data()));
        P.lab0.resize(P.ell[0]);
        for (int64_t k = 0; k < P.ell[0]; ++k) {
            const int32_t v = labs[P.lm_host[k]];
            if (v < 0 || v >= P.C) return fail(KKM_ERR_INVALID_ARG, "init labels must lie in [0, C)");
            P.lab0[k] = v;
        }
    } else {
        if (!p.init_medoids) return fail(KKM_ERR_INVALID_ARG, "MEDOIDS init needs init_medoids");
        P.med0.resize(P.C);
        for (int j = 0; j < P.C; ++j) {
            if (p.init_medoids[j] < 0 || p.init_medoids[j] >= P.n[0])
                return fail(KKM_ERR_INVALID_ARG, "init medoids must be positions of the first batch");
            P.med0[j] = (int32_t)p.init_medoids[j];
        }
    }
    return finish_plan(P, dev);
}

// Sizes that follow from the batches and the device: tiles, chunks, landmark grids.
kkm_status finish_plan(FitPlan& P, const DeviceInfo* dev) {
    P.tile_f64 = P.p.precision == KKM_PREC_FP64 ||
                 (P.kernel.type == KKM_KERNEL_RMSD && !rmsd_on_mfma(P.kernel.n_atoms, P.dtype));
    P.nchunk = select_chunks(P.nmax);
    P.cand_cap = std::min<int64_t>((int64_t)P.nmax * P.C, (int64_t)1 << 30);
    if (dev) {
        for (int i = 0; i < P.B; ++i) {
            const LandmarkShape sh = landmark_shape(*dev, (int)P.ell[i], P.C);
            P.gmax = std::max(P.gmax, sh.grid);
            if (!sh.k_in_lds && landmark_lds_bytes_host((int)P.ell[i], P.C, sh.grid, false) > dev->max_lds_per_block)
                return fail(KKM_ERR_UNSUPPORTED, "landmark set of batch " + std::to_string(i) +
                                                     " too large for one workgroup's LDS; use more mini-batches");
        }
        if ((P.tile_f64 ? 8u : 4u) * (size_t)P.C * 64 > dev->max_lds_per_block)
            return fail(KKM_ERR_UNSUPPORTED, "too many clusters for the distance tile");
    } else {
        P.gmax = 256;
    }
    return KKM_OK;
}

KSpec kspec_of(const kkm_kernel& k, int64_t d) { return KSpec{k.type, k.n_atoms, d, inv2s2_of(k)}; }

kkm_status check_workspace(void* ws, size_t have, size_t need) {
    if (!ws) return fail(KKM_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(KKM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (have < need)
        return fail(KKM_ERR_WORKSPACE, "workspace too small: " + std::to_string(have) + " < " + std::to_string(need));
    return KKM_OK;
}

kkm_status check_device_of(const kkm_model* m) {
    int cur = -1;
    KKM_HIP(hipGetDevice(&cur));
    if (cur != m->device) return fail(KKM_ERR_INVALID_ARG, "the model lives on another device than the current one");
    return KKM_OK;
}

size_t carve_assign(Carver& c, const kkm_model* m, int64_t n, AssignWs& w) {
    const size_t es = m->dtype == KKM_F64 ? 8 : 4;
    const int64_t nn = std::max<int64_t>(1, n);
    w.Qc = m->kernel.type == KKM_KERNEL_RMSD ? c.take<char>((size_t)nn * m->d * es) : nullptr;
    w.r2buf = nullptr;
    w.r2gq = nullptr;
    w.rmsd_chunk = 0;
    if (m->kernel.type == KKM_KERNEL_RMSD && rmsd_on_mfma(m->kernel.n_atoms, m->dtype)) {
        w.rmsd_chunk = rmsd_chunk_groups(nn, m->used, kRmsdAssignChunkBytes);
        w.r2buf = c.take<float>((size_t)w.rmsd_chunk * std::max<int64_t>(1, (m->used + 31) / 32) * 1024);
        w.r2gq = c.take<double>((size_t)w.rmsd_chunk * 32);
    }
    w.refine_list = c.take<int32_t>(nn);
    w.refine_count = c.take<int32_t>(2);
    w.nonfinite = w.refine_count + 1;
    w.best = c.take<double>(nn);
    w.partials = c.take<double>(1024);
    w.cost = c.take<double>(1);
    w.labels_tmp = c.take<int32_t>(nn);
    w.gate = c.take<uint32_t>((size_t)(nn + 31) / 32);
    return c.off;
}

SupportView model_support(const kkm_model* m) {
    SupportView s;
    s.rows = m->support;
    s.dpad = m->dpad;
    s.snorm32 = m->snorm32;
    s.snorm64 = m->snorm64;
    s.coef32 = m->coef32;
    s.coef64 = m->coef64;
    s.offsets = m->offsets;
    s.self = m->self;
    s.segabs = m->segabs;
    s.snorm_max = m->snorm_max;
    s.split = m->split;
    s.nonneg = m->nonneg;
    s.pan = m->pan;
    s.hi = m->hi;
    s.lo = m->lo;
    s.bpad = m->bpad;
    s.C = m->C;
    s.medoid_form = m->medoid_form;
    return s;
}

kkm_status assign_validate(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision) {
    if (!m) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    if (n < 0) return fail(KKM_ERR_INVALID_ARG, "n must be >= 0");
    if (n > 0 && !X) return fail(KKM_ERR_INVALID_ARG, "X is NULL");
    if (dtype != m->dtype) return fail(KKM_ERR_INVALID_ARG, "X dtype differs from the model dtype");
    if (precision < KKM_PREC_FP64 || precision > KKM_PREC_BF16X3)
        return fail(KKM_ERR_INVALID_ARG, "bad precision");
    if (n >= (int64_t)1 << 31) return fail(KKM_ERR_UNSUPPORTED, "at most 2^31 - 1 rows per call");
    return check_device_of(m);
}

// The assign pass on scratch already carved (w): clears the counters, centres RMSD frames, runs the
// distance pass, the FP64 re-decisions and (plain BF16 with a cost) the FP64 best distances.
kkm_status assign_launch(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision, hipStream_t s,
                         int32_t* labels, float* gap, bool want_best, const AssignWs& w) {
    DeviceInfo dev;
    KKM_TRY(device_info(&dev));
    KKM_TRY(launch_zero_i32(w.refine_count, 2, s));
    if (n == 0) return KKM_OK;
    const void* Q = X;
    if (m->kernel.type == KKM_KERNEL_RMSD) {
        KKM_TRY(launch_centre(X, w.Qc, n, m->kernel.n_atoms, dtype, s));
        Q = w.Qc;
    }
    DistArgs da{};
    da.q = BatchView{Q, m->d, 0, 1, n};
    da.dtype = dtype;
    da.precision = precision;
    da.ks = kspec_of(m->kernel, m->d);
    da.sup = model_support(m);
    da.Dt = nullptr;
    da.ldD = 0;
    da.Erow = nullptr;
    da.labels = labels;
    da.gap = gap;
    da.best = want_best ? w.best : nullptr;
    da.refine_list = w.refine_list;
    da.refine_count = w.refine_count;
    da.nonfinite = w.nonfinite;
    da.n_support = m->used;
    da.r2buf = w.r2buf;
    da.r2gq = w.r2gq;
    da.rmsd_chunk = w.rmsd_chunk;
    da.gate = w.gate;
    if (da.sup.C * 64 * (dist_is_fp64(da) ? 8u : 4u) > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "too many clusters for the distance tile");
    KKM_TRY(launch_dist(da, dev, s));
    if (!dist_is_fp64(da)) KKM_TRY(launch_refine(da, dev, s, m->used));
    if (want_best && dist_is_bf16(da)) KKM_TRY(launch_best64(da, dev, s));
    return KKM_OK;
}

kkm_status assign_common(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision, void* ws,
                         size_t ws_bytes, hipStream_t s, int32_t* labels, float* gap, bool want_best, AssignWs& w) {
    KKM_TRY(assign_validate(m, X, n, dtype, precision));
    Carver probe(nullptr);
    const size_t need = carve_assign(probe, m, n, w);
    KKM_TRY(check_workspace(ws, ws_bytes, need));
    Carver c(ws);
    carve_assign(c, m, n, w);
    return assign_launch(m, X, n, dtype, precision, s, labels, gap, want_best, w);
}

kkm_status check_fit_model(const kkm_model* model, const FitPlan& P) {
    if (model->d != P.d || model->C != P.C || model->dtype != P.dtype || model->cap < P.C ||
        model->kernel.type != P.kernel.type || model->kernel.sigma != P.kernel.sigma ||
        model->kernel.n_atoms != P.kernel.n_atoms || model->dpad != P.dpad)
        return fail(KKM_ERR_INVALID_ARG, "model was created for another kernel, d, C, dtype or capacity");
    return check_device_of(model);
}

// The device work of one fit up to the merge of its last batch (and, with KKM_FIT_GLOBAL_COST, the
// global cost after every batch), on stream s: the plan is made and the workspace carved.  up stages
// the host-to-device copy of the draws and must outlive it (until the stream is synchronised).
kkm_status fit_enqueue(const FitPlan& P, FitWs& w, const void* X, hipStream_t s, const DeviceInfo& dev, PhaseTimer& tm,
                       int32_t* labels_out, bool want_pcost, bool want_disp, bool want_trace, std::vector<char>& up) {
    const int64_t N = P.N, d = P.d;
    const int32_t dtype = P.dtype;
    const KSpec ks = kspec_of(P.kernel, d);
    const int C = P.C;
    // refine counts, flags, update counts and the loop's error word: one range of the status block
    KKM_TRY(launch_zero_i32(w.refine_counts, (w.lm_error + 1) - w.refine_counts, s));
    // one host-to-device copy of the inputs block: [landmarks, initial labels, uniforms, medoids]
    // (the staging vector outlives the copy: it is released after the final synchronisation)
    {
        char* ub = reinterpret_cast<char*>(w.lm);
        up.assign(static_cast<size_t>(reinterpret_cast<char*>(w.chosen + C) - ub), 0);
        auto put = [&](void* dev_ptr, const void* src, size_t bytes) {
            if (bytes) std::memcpy(up.data() + (reinterpret_cast<char*>(dev_ptr) - ub), src, bytes);
        };
        put(w.lm, P.lm_host.data(), sizeof(int32_t) * P.ell_total);
        if (P.p.init == KKM_INIT_KMEANSPP) put(w.uniforms, P.uniforms.data(), sizeof(double) * C);
        else if (P.p.init == KKM_INIT_MEDOIDS) put(w.chosen, P.med0.data(), sizeof(int32_t) * C);
        else put(w.lab_init, P.lab0.data(), sizeof(int32_t) * P.ell[0]);
        KKM_HIP(hipMemcpyAsync(ub, up.data(), up.size(), hipMemcpyHostToDevice, s));
    }
    const void* Xs = X;
    if (P.kernel.type == KKM_KERNEL_RMSD) {
        KKM_TRY(launch_centre(X, w.Xc, N, P.kernel.n_atoms, dtype, s));
        Xs = w.Xc;
    }
    auto view = [&](int i) { return BatchView{Xs, d, P.base[i], P.stride[i], P.n[i]}; };

    // batch-0 initialisation of the global medoids
    KKM_TRY(tm.begin(kPhInit));
    if (P.p.init == KKM_INIT_KMEANSPP) {
        KKM_TRY(launch_kmeanspp(view(0), dtype, ks, C, w.uniforms, w.chosen, w.D2, w.kpp_part, w.lm_error, dev, s,
                                (P.p.flags & KKM_FIT_COOPERATIVE) != 0));
        KKM_TRY(launch_set_medoids(view(0), dtype, ks, C, w.chosen, w.M, P.dpad, w.Mself, w.Midx, w.wcount, s));
    } else if (P.p.init == KKM_INIT_MEDOIDS) {
        KKM_TRY(launch_set_medoids(view(0), dtype, ks, C, w.chosen, w.M, P.dpad, w.Mself, w.Midx, w.wcount, s));
    } else {
        KKM_TRY(launch_set_medoids(view(0), dtype, ks, C, nullptr, w.M, P.dpad, w.Mself, w.Midx, w.wcount, s));
    }
    KKM_TRY(tm.end(kPhInit));

    for (int i = 0; i < P.B; ++i) {
        const BatchView bv = view(i);
        const int ell = (int)P.ell[i];
        LandmarkArgs la{};
        la.X = Xs;
        la.d = d;
        la.base = bv.base;
        la.stride = bv.stride;
        la.lm = w.lm + P.lm_off[i];
        la.ell = ell;
        la.C = C;
        la.max_updates = P.T - 1;
        const LandmarkShape lsh = landmark_shape(dev, ell, C);
        la.grid = lsh.grid;
        la.k_in_lds = lsh.k_in_lds;
        la.cooperative = (P.p.flags & KKM_FIT_COOPERATIVE) != 0;
        la.ktype = P.kernel.type;
        la.n_atoms = P.kernel.n_atoms;
        la.inv2s2 = ks.inv2s2;
        la.init_mode = (i == 0 && P.p.init == KKM_INIT_RANDOM_LABELS) ? 0 : 1;
        la.lab_init = w.lab_init;
        la.M = w.M;
        la.Mpad = P.dpad;
        la.Mself = w.Mself;
        la.Kbuf = w.Kbuf;
        la.ldk = landmark_ldk(ell);
        la.Kmed = w.Kmed;
        la.lab = w.lab;
        la.init_parts = landmark_init_parts(la);
        la.nlab_x = w.nlab_x;
        la.sx = w.sx;
        la.partial = w.partial;
        la.changed = w.changed;
        la.zero_ints = w.counts_b;
        la.n_zero_ints = C + 1;
        la.lab_final = w.lab_final;
        la.offsets = w.offsets;
        la.ghat = w.ghat;
        la.segabs = w.segabs;
        la.updates_out = w.updates + i;
        la.support = w.support;
        la.dpad = P.dpad;
        la.snorm32 = w.snorm32;
        la.snorm64 = w.snorm64;
        la.coef32 = w.coef32;
        la.coef64 = w.coef64;
        la.src_index = w.src_index;
        la.snorm_max = w.snorm_max;
        la.split = w.split;
        la.sup_pan = w.sup_pan;
        la.sup_hi = w.sup_hi;
        la.sup_lo = w.sup_lo;
        la.bpad = bf16_pad(P.dpad);
        la.trace = (i == 0 && want_trace) ? w.trace : nullptr;
        la.colmin = w.colmin;
        la.error = w.lm_error;
        if (la.trace) {
            KKM_TRY(launch_zero_i32(reinterpret_cast<int32_t*>(w.trace), 2 * 64, s));
            tm.gap();
        }
        KKM_TRY(tm.begin(kPhLandmark));
        KKM_TRY(launch_landmark_block(la, dtype, dev, s));
        KKM_TRY(tm.end(kPhLandmark));
        KKM_TRY(tm.begin(kPhLoop));
        KKM_TRY(launch_landmark_loop(la, dtype, dev, s));
        KKM_TRY(tm.end(kPhLoop));

        SupportView sv;
        sv.rows = w.support;
        sv.dpad = P.dpad;
        sv.snorm32 = w.snorm32;
        sv.snorm64 = w.snorm64;
        sv.coef32 = w.coef32;
        sv.coef64 = w.coef64;
        sv.offsets = w.offsets;
        sv.self = w.ghat;
        sv.segabs = w.segabs;
        sv.snorm_max = w.snorm_max;
        sv.split = w.split;
        sv.nonneg = 1;
        sv.pan = w.sup_pan;
        sv.hi = w.sup_hi;
        sv.lo = w.sup_lo;
        sv.bpad = bf16_pad(P.dpad);
        sv.C = C;
        sv.medoid_form = 0;

        DistArgs da{};
        da.q = bv;
        da.dtype = dtype;
        // the batch medoids take every row with D - E under the column minimum of D + E as a candidate:
        // the plain BF16 bound would make nearly every row one, so a fit's batch pass takes the
        // compensated BF16x3 products when BF16 is asked for
        da.precision = P.p.precision == KKM_PREC_BF16 ? KKM_PREC_BF16X3 : P.p.precision;
        da.ks = ks;
        da.sup = sv;
        da.Dt = w.Dt;
        da.ldD = P.nmax;
        da.Erow = w.Erow;
        da.labels = w.labels_b;
        da.gap = nullptr;
        const bool pcost = want_pcost;
        da.best = pcost ? w.best : nullptr;
        da.refine_list = w.refine_list;
        da.refine_count = w.refine_counts + i;
        da.nonfinite = w.flags;
        da.colmin = w.colmin;
        da.colpart = w.colpart;
        da.colpart_cap = dist_block_cap(P.nmax);
        da.n_support = ell;
        da.r2buf = w.r2buf;
        da.r2gq = w.r2gq;
        da.rmsd_chunk = w.rmsd_chunk;
        int64_t dist_blocks = 0;
        da.colpart_blocks = &dist_blocks;
        KKM_TRY(tm.begin(kPhDist));
        KKM_TRY(launch_dist(da, dev, s));
        KKM_TRY(tm.end(kPhDist));
        if (!dist_is_fp64(da)) {
            KKM_TRY(tm.begin(kPhRefine));
            KKM_TRY(launch_refine(da, dev, s, ell));
            KKM_TRY(tm.end(kPhRefine));
        }
        if (pcost) {   // the batch's partial cost: its rows' distances summed in a fixed order
            tm.gap();
            KKM_TRY(launch_sum(w.best, bv.n, w.psum, w.pcost + i, s));
        }

        SelectArgs sa{};
        sa.b = bv;
        sa.dtype = dtype;
        sa.ks = ks;
        sa.C = C;
        sa.M = w.M;
        sa.Mpad = P.dpad;
        sa.Mself = w.Mself;
        sa.Midx = w.Midx;
        sa.wcount = w.wcount;
        sa.labels = w.labels_b;
        sa.counts = w.counts_b;
        sa.bmed = w.bmed;
        sa.label_out = labels_out;
        sa.Dt = w.Dt;
        sa.ldD = P.nmax;
        sa.Erow = w.Erow;
        sa.sup = sv;
        sa.nchunk = select_chunks(bv.n);
        sa.mpart_c = w.mpart_c;
        sa.colmin = w.colmin;
        sa.cand_q = w.cand_q;
        sa.cand_j = w.cand_j;
        sa.cand_v = w.cand_v;
        sa.cand_count = w.counts_b + C;
        sa.cand_cap = (int32_t)P.cand_cap;
        sa.tpan = w.tpan;
        sa.tnorm = w.tnorm;
        sa.gpart_v = w.gpart_v;
        sa.gpart_i = w.gpart_i;

        sa.info_bmed = w.info + (size_t)i * C;
        sa.info_bcnt = w.info + (size_t)(P.B + i) * C;
        sa.info_gmed = w.info + (size_t)(2 * P.B + i) * C;
        sa.info_disp = want_disp ? w.info_disp + (size_t)i * C : nullptr;
        KKM_TRY(tm.begin(kPhSelect));
        sa.cand_total = w.flags + 1;
        sa.colpart = w.colpart;
        sa.colpart_ld = da.colpart_cap;
        sa.colpart_blocks = dist_blocks;
        KKM_TRY(launch_select(sa, dist_is_fp64(da), dev, s));
        KKM_TRY(tm.end(kPhSelect));
        if (P.p.flags & KKM_FIT_GLOBAL_COST) {
            // Omega(W) after this batch: the global medoids as they stand, against all N samples
            tm.gap();
            kkm_model& gm = w.gmodel;
            gm.device = dev.device;
            gm.medoid_form = P.p.init != KKM_INIT_RANDOM_LABELS;   // every medoid set from the first batch on
            KKM_TRY(launch_model_from_medoids(&gm, w.M, P.dpad, w.Mself, w.Midx, w.wcount, s));
            KKM_TRY(assign_launch(&gm, X, N, dtype, P.p.precision, s, w.gws.labels_tmp, nullptr, true, w.gws));
            KKM_TRY(launch_sum(w.gws.best, N, w.gws.partials, w.gcost + i, s));
        }
    }
    return KKM_OK;
}

// After the stream has been synchronised: the fit's outputs from its status block copy st (model host
// fields, info) and its error words.
kkm_status fit_finish(const FitPlan& P, const FitWs& w, const std::vector<char>& st, kkm_model* model,
                      kkm_fit_info* info, PhaseTimer& tm) {
    const int C = P.C;
    const char* sb = reinterpret_cast<const char*>(w.refine_counts);
    auto host_at = [&](const void* dev_ptr) { return st.data() + (reinterpret_cast<const char*>(dev_ptr) - sb); };
    const int32_t* refined = reinterpret_cast<const int32_t*>(host_at(w.refine_counts));
    const int32_t* flags = reinterpret_cast<const int32_t*>(host_at(w.flags));
    const int32_t* updates = reinterpret_cast<const int32_t*>(host_at(w.updates));
    const int32_t lm_err = *reinterpret_cast<const int32_t*>(host_at(w.lm_error));
    const int64_t* infos = reinterpret_cast<const int64_t*>(host_at(w.info));
    if (info && info->landmark_trace) std::memcpy(info->landmark_trace, host_at(w.trace), sizeof(int64_t) * 64);
    if (info && info->medoid_displacement)
        std::memcpy(info->medoid_displacement, host_at(w.info_disp), sizeof(double) * (size_t)P.B * C);
    if (info && info->partial_cost) std::memcpy(info->partial_cost, host_at(w.pcost), sizeof(double) * (size_t)P.B);
    if (info && info->global_cost && (P.p.flags & KKM_FIT_GLOBAL_COST))
        std::memcpy(info->global_cost, host_at(w.gcost), sizeof(double) * (size_t)P.B);
    model->used = C;
    model->nonneg = 1;
    {   // a medoid model unless a cluster never received a medoid (its self term is then +inf)
        const int64_t* last = reinterpret_cast<const int64_t*>(host_at(w.info)) + (size_t)(2 * P.B + P.B - 1) * C;
        int32_t all = 1;
        for (int j = 0; j < C; ++j) all &= last[j] >= 0 ? 1 : 0;
        model->medoid_form = all;
    }

    if (info) {
        int64_t alg = 0, perf = 0, rows_ref = 0;
        for (int i = 0; i < P.B; ++i) {
            const int64_t n = P.n[i], ell = P.ell[i];
            int64_t nonempty = 0;
            for (int j = 0; j < C; ++j) nonempty += infos[(size_t)(P.B + i) * C + j] > 0;
            alg += n * ell + n * nonempty;
            const bool eq8 = i > 0 || P.p.init != KKM_INIT_RANDOM_LABELS;
            if (i > 0 || P.p.init == KKM_INIT_KMEANSPP) alg += n * C;
            perf += ell * ell + (eq8 ? ell * C : 0) + n * ell + (int64_t)refined[i] * ell + 2 * n * nonempty;
            if (i == 0 && P.p.init == KKM_INIT_KMEANSPP) perf += n * (C - 1);
            rows_ref += refined[i];
            if (info->updates_per_batch) info->updates_per_batch[i] = updates[i] + 1;
            for (int j = 0; j < C; ++j) {
                if (info->batch_medoids) info->batch_medoids[(size_t)i * C + j] = infos[(size_t)i * C + j];
                if (info->batch_counts) info->batch_counts[(size_t)i * C + j] = infos[(size_t)(P.B + i) * C + j];
                if (info->global_medoids) info->global_medoids[(size_t)i * C + j] = infos[(size_t)(2 * P.B + i) * C + j];
            }
        }
        info->evals_algorithmic = alg;
        info->evals_performed = perf;
        info->rows_refined = rows_ref;
        info->medoid_candidates = flags[1];
        double ms[kPhases];
        tm.collect(ms);
        info->ms_init = ms[kPhInit];
        info->ms_landmark = ms[kPhLandmark] + ms[kPhLoop];
        info->ms_landmark_loop = ms[kPhLoop];
        info->ms_dist = ms[kPhDist];
        info->ms_refine = ms[kPhRefine];
        info->ms_select = ms[kPhSelect];
    }
    if (lm_err) return fail(KKM_ERR_INTERNAL, "a wait for another workgroup (k-means++ or landmark loop) exceeded its cap");
    if (flags[0]) return fail(KKM_ERR_NONFINITE, "X holds NaN or Inf");
    return KKM_OK;
}

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" {

size_t kkm_fit_workspace_bytes(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel, const kkm_params* params) {
    FitPlan P;
    DeviceInfo dev;
    const bool have_dev = device_info(&dev) == KKM_OK;
    if (make_plan(N, d, dtype, kernel, params, have_dev ? &dev : nullptr, P, false) != KKM_OK) return 0;
    FitWs w;
    Carver c(nullptr);
    return carve_fit(c, P, w);
}

int64_t kkm_fit_min_batches(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel, const kkm_params* params,
                            size_t budget_bytes) {
    if (!params) {
        fail(KKM_ERR_INVALID_ARG, "params is NULL");
        return 0;
    }
    if (N < 1 || params->C < 1) {
        fail(KKM_ERR_INVALID_ARG, "N and C must be >= 1");
        return 0;
    }
    kkm_params p = *params;
    p.landmarks = nullptr;
    p.init_labels = nullptr;
    p.init_medoids = nullptr;
    auto fits = [&](int64_t B) {
        p.B = (int32_t)B;
        const size_t w = kkm_fit_workspace_bytes(N, d, dtype, kernel, &p);
        return w != 0 && w <= budget_bytes;
    };
    // The workspace falls with B while the landmark block dominates (l^2 ~ 1/B^2) and rises again
    // with the per-batch state (~ B): the smallest fitting B lies on the falling side, below the B
    // of the smallest workspace, found first among the powers of two up to N / C.
    const int64_t hi0 = std::min<int64_t>(std::max<int64_t>(1, N / params->C), INT32_MAX);
    int64_t bstar = 0;
    size_t wstar = 0;
    for (int64_t B = 1;; B = std::min(hi0, 2 * B)) {
        p.B = (int32_t)B;
        const size_t w = kkm_fit_workspace_bytes(N, d, dtype, kernel, &p);
        if (w != 0 && (bstar == 0 || w < wstar)) {
            bstar = B;
            wstar = w;
        }
        if (B == hi0) break;
    }
    if (bstar == 0 || !fits(bstar)) {
        fail(KKM_ERR_WORKSPACE, "no number of mini-batches up to N / C fits the workspace budget");
        return 0;
    }
    int64_t lo = 0, hi = bstar;   // fits(hi); lo == 0 or !fits(lo)
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (fits(mid)) hi = mid;
        else lo = mid;
    }
    return hi;
}

kkm_status kkm_fit(const void* X, int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                   const kkm_params* params, void* workspace, size_t workspace_bytes, void* stream, kkm_model* model,
                   int32_t* labels_out, kkm_fit_info* info) {
    if (!X) return fail(KKM_ERR_INVALID_ARG, "X is NULL");
    if (!model) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    DeviceInfo dev;
    KKM_TRY(device_info(&dev));
    FitPlan P;
    KKM_TRY(make_plan(N, d, dtype, kernel, params, &dev, P));
    KKM_TRY(check_fit_model(model, P));
    FitWs w;
    Carver probe(nullptr);
    const size_t need = carve_fit(probe, P, w);
    KKM_TRY(check_workspace(workspace, workspace_bytes, need));
    Carver c(workspace);
    carve_fit(c, P, w);
    hipStream_t s = static_cast<hipStream_t>(stream);
    PhaseTimer tm;
    tm.on = info && info->time_phases;
    if (tm.on && info->time_phases == 2) tm.mask = (1u << kPhLoop) | (1u << kPhDist);
    tm.s = s;
    tm.device = dev.device;
    std::vector<char> up;
    KKM_TRY(fit_enqueue(P, w, X, s, dev, tm, labels_out, info && info->partial_cost, info && info->medoid_displacement,
                        info && info->landmark_trace, up));
    KKM_TRY(launch_model_from_medoids(model, w.M, P.dpad, w.Mself, w.Midx, w.wcount, s));
    // one device-to-host copy of the status block
    const char* sb = reinterpret_cast<const char*>(w.refine_counts);
    std::vector<char> st((size_t)(w.status_end - sb));
    KKM_HIP(hipMemcpyAsync(st.data(), sb, st.size(), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    return fit_finish(P, w, st, model, info, tm);
}

// ----------------------------------------------------------------------------- restarts (Sec. 4.5)
namespace {
// Workspace of R restarts: per restart a fit workspace, its medoids as a model and its labels; one
// assign workspace over the N samples for the cost passes (run one after another on the stream).
struct RestartLayout {
    std::vector<FitWs> w;
    std::vector<kkm_model> m;
    std::vector<int32_t*> labels;
    std::vector<double*> cost;
    AssignWs aws;
};
size_t carve_restarts(Carver& c, const FitPlan& P, int R, RestartLayout& L) {
    L.w.assign(R, FitWs{});
    L.m.assign(R, kkm_model{});
    L.labels.assign(R, nullptr);
    L.cost.assign(R, nullptr);
    for (int r = 0; r < R; ++r) {
        carve_fit(c, P, L.w[r]);
        kkm_model& m = L.m[r];
        m.kernel = P.kernel;
        m.d = P.d;
        m.dpad = P.dpad;
        m.bpad = bf16_pad(P.dpad);
        m.C = P.C;
        m.cap = P.C;
        m.used = P.C;
        m.dtype = P.dtype;
        model_layout(&m, c);
        L.labels[r] = c.take<int32_t>((size_t)P.N);
        L.cost[r] = c.take<double>(1);
    }
    carve_assign(c, &L.m[0], P.N, L.aws);
    return c.off;
}

kkm_status restart_plan(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel, const kkm_params* params,
                        int R, int r, const DeviceInfo* dev, FitPlan& P, bool draws) {
    if (!params) return fail(KKM_ERR_INVALID_ARG, "params is NULL");
    if (R < 1 || R > 1024) return fail(KKM_ERR_INVALID_ARG, "restarts must be in [1, 1024]");
    if (params->landmarks || params->kmpp_uniforms || params->init_labels)
        return fail(KKM_ERR_INVALID_ARG, "restarts draw their own landmarks and initialisation: pass none");
    kkm_params p = *params;
    p.seed = params->seed + (uint64_t)r;
    return make_plan(N, d, dtype, kernel, &p, dev, P, draws);
}
}  // namespace

size_t kkm_fit_restarts_workspace_bytes(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                                        const kkm_params* params, int32_t restarts) {
    FitPlan P;
    DeviceInfo dev;
    const bool have_dev = device_info(&dev) == KKM_OK;
    if (restart_plan(N, d, dtype, kernel, params, restarts, 0, have_dev ? &dev : nullptr, P, false) != KKM_OK) return 0;
    RestartLayout L;
    Carver c(nullptr);
    return carve_restarts(c, P, restarts, L);
}

kkm_status kkm_fit_restarts(const void* X, int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                            const kkm_params* params, int32_t restarts, void* workspace, size_t workspace_bytes,
                            void* stream, kkm_model* model, int32_t* labels_out, kkm_fit_info* info,
                            double* costs_out, int32_t* best_out) {
    if (!X) return fail(KKM_ERR_INVALID_ARG, "X is NULL");
    if (!model) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    DeviceInfo dev;
    KKM_TRY(device_info(&dev));
    const int R = restarts;
    std::vector<FitPlan> P(std::max(1, R));
    for (int r = 0; r < R; ++r) KKM_TRY(restart_plan(N, d, dtype, kernel, params, R, r, &dev, P[r], true));
    if (R < 1) return fail(KKM_ERR_INVALID_ARG, "restarts must be >= 1");
    KKM_TRY(check_fit_model(model, P[0]));
    RestartLayout L;
    {
        Carver probe(nullptr);
        KKM_TRY(check_workspace(workspace, workspace_bytes, carve_restarts(probe, P[0], R, L)));
    }
    Carver c(workspace);
    carve_restarts(c, P[0], R, L);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every restart back to back on the stream: its fit, its medoids as a model, its FP64 cost over
    // all N samples (Eq. 1, as kkm_cost), and the copy of its status block; one synchronisation
    std::vector<std::vector<char>> up(R), st(R);
    std::vector<PhaseTimer> tms(R);
    for (int r = 0; r < R; ++r) {
        FitWs& w = L.w[r];
        tms[r].device = dev.device;
        KKM_TRY(fit_enqueue(P[r], w, X, s, dev, tms[r], L.labels[r], false, false, false, up[r]));
        kkm_model& m = L.m[r];
        m.device = dev.device;
        m.medoid_form = P[r].p.init != KKM_INIT_RANDOM_LABELS;
        KKM_TRY(launch_model_from_medoids(&m, w.M, P[r].dpad, w.Mself, w.Midx, w.wcount, s));
        KKM_TRY(assign_launch(&m, X, N, dtype, KKM_PREC_FP64, s, L.aws.labels_tmp, nullptr, true, L.aws));
        KKM_TRY(launch_sum(L.aws.best, N, L.aws.partials, L.cost[r], s));
        const char* sb = reinterpret_cast<const char*>(w.refine_counts);
        st[r].resize((size_t)(w.status_end - sb));
        KKM_HIP(hipMemcpyAsync(st[r].data(), sb, st[r].size(), hipMemcpyDeviceToHost, s));
    }
    std::vector<double> cost(R);
    for (int r = 0; r < R; ++r) KKM_HIP(hipMemcpyAsync(&cost[r], L.cost[r], sizeof(double), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    // the lowest cost wins, the lowest restart on equal costs (every fit's errors are reported first)
    int best = 0;
    for (int r = 0; r < R; ++r) {
        kkm_model scratch_model{};
        const kkm_status e = fit_finish(P[r], L.w[r], st[r], &scratch_model, nullptr, tms[r]);
        if (e != KKM_OK) return e;
        if (cost[r] < cost[best]) best = r;
    }
    if (costs_out) std::copy(cost.begin(), cost.end(), costs_out);
    if (best_out) *best_out = best;
    const FitWs& wb = L.w[best];
    KKM_TRY(launch_model_from_medoids(model, wb.M, P[best].dpad, wb.Mself, wb.Midx, wb.wcount, s));
    if (labels_out) KKM_HIP(hipMemcpyAsync(labels_out, L.labels[best], sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToDevice, s));
    KKM_HIP(hipStreamSynchronize(s));
    return fit_finish(P[best], wb, st[best], model, info, tms[best]);
}

size_t kkm_kernel_block_workspace_bytes(const kkm_kernel* kernel, int64_t nx, int64_t ny, int64_t d, int32_t dtype) {
    if (!kernel || nx < 0 || ny < 0 || d < 1 || (dtype != KKM_F32 && dtype != KKM_F64)) return 0;
    Carver c(nullptr);
    const size_t es = dtype == KKM_F64 ? 8 : 4;
    if (kernel->type == KKM_KERNEL_RMSD) {
        c.take<char>((size_t)std::max<int64_t>(1, nx) * d * es);
        c.take<char>((size_t)std::max<int64_t>(1, ny) * d * es);
    }
    return std::max<size_t>(c.off, 256);
}

kkm_status kkm_kernel_block(const kkm_kernel* kernel, const void* X, int64_t nx, const void* Y, int64_t ny, int64_t d,
                            int32_t dtype, void* workspace, size_t workspace_bytes, void* stream, double* K_out) {
    if (nx < 0 || ny < 0) return fail(KKM_ERR_INVALID_ARG, "nx and ny must be >= 0");
    if (d < 1) return fail(KKM_ERR_INVALID_ARG, "d must be >= 1");
    if (dtype != KKM_F32 && dtype != KKM_F64) return fail(KKM_ERR_INVALID_ARG, "bad dtype");
    if (!kernel) return fail(KKM_ERR_INVALID_ARG, "kernel is NULL");
    if (kernel->type != KKM_KERNEL_LINEAR && kernel->type != KKM_KERNEL_RBF && kernel->type != KKM_KERNEL_RMSD)
        return fail(KKM_ERR_INVALID_ARG, "unknown kernel type");
    if (kernel->type != KKM_KERNEL_LINEAR && !(kernel->sigma > 0.0 && std::isfinite(kernel->sigma)))
        return fail(KKM_ERR_INVALID_ARG, "sigma must be finite and > 0");
    if (kernel->type == KKM_KERNEL_RMSD && (kernel->n_atoms < 1 || d != 3 * (int64_t)kernel->n_atoms))
        return fail(KKM_ERR_INVALID_ARG, "RMSD kernel needs d == 3 * n_atoms");
    if (nx * ny > 0 && (!X || !Y || !K_out)) return fail(KKM_ERR_INVALID_ARG, "X, Y and K_out must not be NULL");
    KKM_TRY(check_workspace(workspace, workspace_bytes, kkm_kernel_block_workspace_bytes(kernel, nx, ny, d, dtype)));
    DeviceInfo dev;
    KKM_TRY(device_info(&dev));
    if (nx == 0 || ny == 0) return KKM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const void* Xs = X;
    const void* Ys = Y;
    if (kernel->type == KKM_KERNEL_RMSD) {
        Carver c(workspace);
        const size_t es = dtype == KKM_F64 ? 8 : 4;
        void* Xc = c.take<char>((size_t)nx * d * es);
        void* Yc = c.take<char>((size_t)ny * d * es);
        KKM_TRY(launch_centre(X, Xc, nx, kernel->n_atoms, dtype, s));
        KKM_TRY(launch_centre(Y, Yc, ny, kernel->n_atoms, dtype, s));
        Xs = Xc;
        Ys = Yc;
    }
    return launch_kernel_block(kspec_of(*kernel, d), dtype, Xs, nx, Ys, ny, K_out, dev, s);
}

size_t kkm_assign_workspace_bytes(const kkm_model* m, int64_t n, int32_t precision) {
    if (!m || n < 0) return 0;
    (void)precision;
    AssignWs w;
    Carver c(nullptr);
    return carve_assign(c, m, n, w);
}

kkm_status kkm_assign(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision, void* ws,
                      size_t ws_bytes, void* stream, int32_t* labels_out, float* gap_out) {
    if (!labels_out && n > 0) return fail(KKM_ERR_INVALID_ARG, "labels_out is NULL");
    AssignWs w;
    return assign_common(m, X, n, dtype, precision, ws, ws_bytes, static_cast<hipStream_t>(stream), labels_out, gap_out,
                         false, w);
}

kkm_status kkm_assign_noalloc(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision,
                              void* stream, int32_t* labels_out, float* gap_out) {
    if (!labels_out && n > 0) return fail(KKM_ERR_INVALID_ARG, "labels_out is NULL");
    KKM_TRY(assign_validate(m, X, n, dtype, precision));
    AssignWs w{};
    Carver probe(nullptr);
    const size_t need = carve_assign(probe, m, n, w);
    if (need > kNoAllocScratchBytes)
        return fail(KKM_ERR_UNSUPPORTED, "kkm_assign_noalloc: " + std::to_string(n) + " rows of this model need " +
                                             std::to_string(need) + " bytes of scratch, more than its fixed " +
                                             std::to_string(kNoAllocScratchBytes) +
                                             "; split the rows or call kkm_assign with a workspace");
    void* base = nullptr;
    KKM_TRY(noalloc_scratch(m->device, &base));
    Carver c(base);
    carve_assign(c, m, n, w);
    return assign_launch(m, X, n, dtype, precision, static_cast<hipStream_t>(stream), labels_out, gap_out, false, w);
}

kkm_status kkm_cost(const kkm_model* m, const void* X, int64_t n, int32_t dtype, int32_t precision, void* ws,
                    size_t ws_bytes, void* stream, double* cost_out) {
    if (!cost_out) return fail(KKM_ERR_INVALID_ARG, "cost_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!m) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    if (n < 0) return fail(KKM_ERR_INVALID_ARG, "n must be >= 0");
    // the labels of the pass live in the workspace: check it before carving them out
    KKM_TRY(check_workspace(ws, ws_bytes, kkm_assign_workspace_bytes(m, n, precision)));
    AssignWs w{};
    {
        Carver c(ws);
        carve_assign(c, m, n, w);
    }
    int32_t* labels = w.labels_tmp;
    KKM_TRY(assign_common(m, X, n, dtype, precision, ws, ws_bytes, s, labels, nullptr, true, w));
    if (n == 0) {
        *cost_out = 0.0;
        return KKM_OK;
    }
    KKM_TRY(launch_sum(w.best, n, w.partials, w.cost, s));
    double cost = 0.0;
    int32_t nf = 0;
    KKM_HIP(hipMemcpyAsync(&cost, w.cost, sizeof(double), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipMemcpyAsync(&nf, w.nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (nf) return fail(KKM_ERR_NONFINITE, "X holds NaN or Inf");
    *cost_out = cost;
    return KKM_OK;
}

}  // extern "C"
