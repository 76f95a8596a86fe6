// Argument blocks and host launchers of the device kernels (one struct per kernel family).
#pragma once

#include "kkm_internal.hpp"

namespace kkm {

// A view of one mini-batch: row j of the batch is row (base + j * stride) of X.
struct BatchView {
    const void* X;
    int64_t d;
    int64_t base;
    int64_t stride;
    int64_t n;
};

// ---------------------------------------------------------------- landmark phase (k_landmark.hip)
struct LandmarkArgs {
    const void* X;          // samples (dtype of the fit), RMSD: centred frames
    int64_t d, base, stride;
    const int32_t* lm;      // [ell] batch positions of the landmarks, ascending
    int32_t ell, C, max_updates, grid;
    int32_t ktype, n_atoms;
    double inv2s2;
    int32_t init_mode;      // 0: lab_init, 1: nearest valid global medoid (Eq. 8)
    int32_t init_parts;     // > 0: Eq. 8 minima of the medoid column tiles, (value, cluster) pairs as
                            // doubles in Kmed ([ell][init_parts][2]), combined by the loop kernel;
                            // 0: the initial labels are in lab (landmark_init_parts sets it)
    const int32_t* lab_init;// [ell]
    const void* M;          // [C][Mpad] global medoid rows (dtype of the fit)
    int64_t Mpad;
    const double* Mself;    // [C] K(m,m), +inf where the medoid is unset
    double* Kbuf;           // [ell][ldk] scratch: K_LL
    int64_t ldk;            // row stride of Kbuf (ell rounded up to even)
    double* Kmed;           // [ell][C] scratch: the Eq. 8 minima of the medoid tiles (init_parts)
    int32_t* lab;           // [2][ell] scratch: initial labels, then final labels
    int32_t* nlab_x;        // [2][ell] scratch: labels after an update, exchanged between workgroups
                            // (two halves used by alternate updates)
    double* sx;             // [2][ell][2] scratch: S of a changed landmark at its old and new label
    double* partial;        // [3][grid][C] scratch: each workgroup's part of the g^ sums, three
                            // buffers used by successive exchanges in turn
    int32_t* changed;       // [max_updates+1] scratch
    int32_t* zero_ints;     // ints to clear for the later kernels of the batch
    int32_t n_zero_ints;
    // outputs
    int32_t* lab_final;     // [ell]
    int32_t* offsets;       // [C+1]
    double* ghat;           // [C] (+inf for clusters without landmarks)
    double* segabs;         // [C]
    int32_t* updates_out;   // [1] landmark label updates performed
    void* support;          // [ell][dpad]
    int64_t dpad;
    float* snorm32;
    double* snorm64;
    float* coef32;
    double* coef64;
    int32_t* src_index;     // [ell] batch position of each support row
    float* snorm_max;       // [1]
    float* sup_pan;         // FP32 panel copy of the support (float input), or null
    uint16_t* sup_hi;       // bfloat16 panels of the split of the support rows (dpad >= 16)
    uint16_t* sup_lo;
    int64_t bpad;
    int32_t* split;         // [5] cluster runs of the distance pass's four wavefronts
    int32_t k_in_lds;       // own rows of the landmark block kept in LDS (else in Kbuf)
    int32_t cooperative;    // host: launch the loop kernel cooperatively
    int64_t* trace;         // [64] device wall-clock stamps of workgroup 0, or null
    unsigned long long* colmin;   // [C] set to the empty value for the batch's distance pass
    int32_t* error;         // [1] set when a wait for another workgroup exceeded its cap
};
// Workgroups of the landmark phase for a landmark set of size ell (KKM_LANDMARK_ROWS rows each).
struct LandmarkShape {
    int grid;        // workgroups of the loop kernel
    int k_in_lds;    // own rows of K_LL in LDS
};
LandmarkShape landmark_shape(const DeviceInfo& dev, int ell, int C);
size_t landmark_lds_bytes_host(int ell, int C, int G, bool k_in_lds);
inline int64_t landmark_ldk(int64_t ell) { return (ell + 15) & ~int64_t(15); }
// K_LL (+ K(x_l, m_j)) and the initial landmark labels; then the landmark loop and the support.
kkm_status launch_landmark_block(const LandmarkArgs& a, int dtype, const DeviceInfo& dev, hipStream_t s);
// The init_parts value for these arguments (the medoid column tiles of the landmark block kernel).
int landmark_init_parts(const LandmarkArgs& a);
kkm_status launch_landmark_loop(const LandmarkArgs& a, int dtype, const DeviceInfo& dev, hipStream_t s);

// ---------------------------------------------------------------- sparse-centroid distances (k_dist.hip)
// Support of the centroids being assigned to: rows in CSR order, coefficients, self terms.
struct SupportView {
    const void* rows;       // [ns][dpad] (dtype)
    int64_t dpad;
    const float* snorm32;
    const double* snorm64;
    const float* coef32;
    const double* coef64;
    const int32_t* offsets; // [C+1]
    const double* self;     // [C]
    const double* segabs;   // [C]
    const float* snorm_max; // [1]
    const int32_t* split;   // [5] cluster runs of the four wavefronts of a distance tile
    int32_t nonneg;         // every coefficient >= 0 (error bounds may scale with the sums)
    const float* pan;       // FP32 panel copy of the rows (float models), or null
    const uint16_t* hi;     // bfloat16 panel of the high parts of the rows (or null)
    const uint16_t* lo;     // bfloat16 panel of the remainders
    int64_t bpad;
    int32_t C;
    int32_t medoid_form;    // every cluster one support row (row j), coefficient 1, every self term finite
};

struct DistArgs {
    BatchView q;            // query rows (RMSD: centred)
    int32_t dtype;          // dtype of both query rows and support rows
    int32_t precision;      // KKM_PREC_*
    KSpec ks;
    SupportView sup;
    // outputs
    float* Dt;              // [C][ldD] distances (transposed), or null
    int64_t ldD;
    float* Erow;            // [n] per-row error bound of every D entry, or null
    int32_t* labels;        // [n]
    float* gap;             // [n] or null
    double* best;           // [n] best distance, or null
    int32_t* refine_list;   // [n]
    int32_t* refine_count;  // [1]
    int32_t* nonfinite;     // [1]
    unsigned long long* colmin;   // [C] non-null in a fit: the pass then writes colpart (the medoid
                                  // candidate kernel folds it into min over rows of D + Erow)
    double* colpart;        // [C][colpart_cap] per-workgroup minima of D + Erow (with colmin)
    int64_t colpart_cap;
    int64_t* colpart_blocks;// host out (with colmin): workgroups of the pass
    int64_t n_support;      // rows of sup (offsets[C])
    // RMSD on the matrix cores: a pair pass leaves the squared RMSD of every (query, support) pair of
    // a chunk of query groups (32 frames each), which the distance pass then reads back
    float* r2buf;           // [rmsd_chunk][ceil(n_support / 32)][1024]
    double* r2gq;           // [rmsd_chunk * 32] G = sum of squared coordinates of each query frame
    int64_t rmsd_chunk;     // query groups per chunk
    int64_t grp0, grp_n;    // the chunk being reduced (set by the launcher)
    // Plain BF16 assign against a medoid model: the BF16 pass marks the rows it cannot decide in one
    // 32-bit word per group of 32 rows (no list, no atomics), BF16x3 re-decides the marked rows and
    // lists for FP64 those it cannot decide either
    uint32_t* gate;         // [ceil(n / 32)], or null (BF16 rows straight to FP64)
    int32_t gate_mode;      // 0 none, 1 write the marks (BF16 pass), 2 read them (BF16x3 pass)
};
// Query groups per chunk of the RMSD pair pass: its buffer of squared RMSDs stays under cap_bytes.
inline int64_t rmsd_chunk_groups(int64_t n, int64_t n_support, size_t cap_bytes) {
    const int64_t tiles = std::max<int64_t>(1, (n_support + 31) / 32);
    const int64_t groups = std::max<int64_t>(1, (n + 31) / 32);
    return std::min<int64_t>(groups, std::max<int64_t>(1, (int64_t)(cap_bytes / ((size_t)tiles * 4096))));
}
// Pair-pass buffers of a fit's batch pass and of an assign call.
constexpr size_t kRmsdFitChunkBytes = size_t(64) << 20;
constexpr size_t kRmsdAssignChunkBytes = size_t(16) << 20;
kkm_status launch_dist(const DistArgs& a, const DeviceInfo& dev, hipStream_t s);
// Matrix-core distance pass (k_mfma.hip): linear / RBF, float samples, FP32, BF16 or BF16x3.
bool mfma_dist_applies(const DistArgs& a);
// KKM_DIST_VALU=1 in the environment: every distance pass on the VALU kernels.
bool mfma_disabled();
// True when the RMSD distance pass of float frames with n_atoms atoms runs on the matrix cores.
inline bool rmsd_on_mfma(int n_atoms, int dtype) { return !mfma_disabled() && rmsd_mfma_ok(n_atoms, dtype); }
kkm_status launch_dist_mfma(const DistArgs& a, const DeviceInfo& dev, hipStream_t s);
// True when launch_dist evaluates (and stores Dt) in FP64 for these arguments.
bool dist_is_fp64(const DistArgs& a);
// LDS bytes the distance tile needs for C clusters.
size_t dist_lds_bytes(const DistArgs& a);
// Workgroups of any distance pass over n rows (bound for colpart_cap).
inline int64_t dist_block_cap(int64_t n) { return (n + 15) / 16 + 1; }
// colmin[j] <- ord_enc(min over the first nblk entries of colpart row j) (~0: none finite).
// FP64 re-decision of the rows listed by launch_dist (n_support: support rows of a.sup).
kkm_status launch_refine(const DistArgs& a, const DeviceInfo& dev, hipStream_t s, int64_t n_support);
// True when launch_dist runs the plain BF16 matrix-core pass for these arguments.
bool dist_is_bf16(const DistArgs& a);
// a.best[q] <- the FP64 distance of row q to the cluster of a.labels[q] (after launch_refine).
kkm_status launch_best64(const DistArgs& a, const DeviceInfo& dev, hipStream_t s);
// K[i * ny + j] = kappa(x_i, y_j) in FP64 for rows of length ks.d (RMSD: centred frames).
kkm_status launch_kernel_block(const KSpec& ks, int dtype, const void* X, int64_t nx, const void* Y, int64_t ny,
                               double* K, const DeviceInfo& dev, hipStream_t s);
// Deterministic FP64 sum of best[0..n) into out[0] (partials: >= 1024 doubles of scratch).
kkm_status launch_sum(const double* best, int64_t n, double* partials, double* out, hipStream_t s);

// ---------------------------------------------------------------- selection steps (k_select.hip)
struct SelectArgs {
    BatchView b;            // the batch
    int32_t dtype;
    KSpec ks;
    int32_t C;
    // global medoid state
    void* M;                // [C][Mpad]
    int64_t Mpad;
    double* Mself;          // [C]
    int64_t* Midx;          // [C] sample index
    int64_t* wcount;        // [C] running |w_j|
    // batch state
    const int32_t* labels;  // [n] batch labels (after FP64 re-decisions)
    int32_t* counts;        // [C] out: |w_j^i|
    int32_t* bmed;          // [C] out: batch medoid positions (-1: empty)
    int32_t* label_out;     // [N] caller labels (scatter), or null
    const float* Dt;        // [C][ldD] distances of the batch pass (float or double)
    int64_t ldD;
    const float* Erow;      // [n] error bound of each row's distances
    const unsigned long long* colmin;   // [C] ord_enc(min over rows of D + E), used when colpart_blocks == 0
    const double* colpart;  // [C][colpart_ld] per-block column minima of D + E from the distance pass
    int64_t colpart_ld;
    int64_t colpart_blocks; // blocks of the distance pass (0: take colmin)
    SupportView sup;        // support of the batch centroids (FP64 re-evaluation of candidates)
    int32_t nchunk;         // select_chunks(n)
    int32_t* mpart_c;       // [C][nchunk] member-count partials
    int32_t* cand_q;        // [cand_cap] candidate rows
    int32_t* cand_j;        // [cand_cap] their clusters
    double* cand_v;         // [cand_cap] their FP64 distances
    int32_t* cand_count;    // [1] (cleared before the batch)
    int32_t cand_cap;
    int32_t* cand_total;    // [1] accumulates cand_count over batches, or null
    double* tpan;           // [C][2][Mpad] merge targets (m_j^i, m_j) in FP64, written by the settle pass
    double* tnorm;          // [C][2] their squared norms
    double* gpart_v;        // [C][mchunk] merge partials (set by launch_select)
    int32_t* gpart_i;
    int32_t mchunk;
    // per-batch info rows (device, length C) or null
    int64_t* info_bmed;
    int64_t* info_bcnt;
    int64_t* info_gmed;
    double* info_disp;      // displacement of every global medoid (kernel space), or null
};
int select_chunks(int64_t n);
// Merge partials per cluster for a batch of n rows (the workspace holds C * merge_chunks(nmax)).
int merge_chunks(int64_t n);
// Member counts, label scatter, batch medoids (Eq. 10) and the merge (Eq. 11-13).
// tile_f64: the distance tile Dt holds doubles (FP64 precision) rather than floats.
kkm_status launch_select(const SelectArgs& a, bool tile_f64, const DeviceInfo& dev, hipStream_t s);

// k-means++ on a batch: uniforms[C] device, chosen[C] device out, D2 [2n] and part [768] scratch,
// error as for the landmark loop.
kkm_status launch_kmeanspp(const BatchView& b, int dtype, const KSpec& ks, int C, const double* uniforms,
                           int32_t* chosen, double* D2, double* part, int32_t* error, const DeviceInfo& dev,
                           hipStream_t s, bool cooperative = false);
// Global medoids <- batch rows `chosen` (valid, counts 0), or all unset when chosen == null.
kkm_status launch_set_medoids(const BatchView& b, int dtype, const KSpec& ks, int C, const int32_t* chosen,
                              void* M, int64_t Mpad, double* Mself, int64_t* Midx, int64_t* wcount, hipStream_t s);
// Write a fitted model (support = the C medoid rows, coefficient 1) from the global medoid state.
kkm_status launch_model_from_medoids(kkm_model* m, const void* M, int64_t Mpad, const double* Mself,
                                     const int64_t* Midx, const int64_t* wcount, hipStream_t s);
// Self terms a^T K_SS a of a model's segments (FP64) and its norm / coefficient arrays from rows.
kkm_status launch_model_prepare(kkm_model* m, hipStream_t s);
// RMSD: centre each frame of X (n rows, 3A values) into Y.
kkm_status launch_centre(const void* X, void* Y, int64_t n, int A, int dtype, hipStream_t s);
// Set n ints to zero (a kernel, so that the call can sit inside a captured graph).
kkm_status launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
// *dst += *src on the device.
kkm_status launch_add_i32(int32_t* dst, const int32_t* src, hipStream_t s);
// Set n 64-bit words to v (a kernel, for the same reason).
kkm_status launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
kkm_status launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

}  // namespace kkm
