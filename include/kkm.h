/*
 * kkm.h -- C ABI of libkkm: mini-batch kernel k-means with a-priori sparse
 * (landmark) centroids on AMD Instinct MI355X (gfx950).
 *
 * Method: M. J. Ferrarotti, S. Decherchi, W. Rocchia, "Distributed Kernel
 * K-Means for Large Scale Clustering".  Sec. 2 (Eq. 1-7) defines kernel
 * k-means and the medoid approximation; Sec. 3.1 (Eq. 8-13) the mini-batch
 * scheme (batch fetching, initialisation, inner loop, batch medoids, merge);
 * Sec. 3.2 (Eq. 14-18) the landmark-restricted centroids.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Sample matrices are row-major, n rows of d values, float32 or float64
 *   (kkm_dtype).  RMSD frames are rows of 3*n_atoms values ordered
 *   x0 y0 z0 x1 y1 z1 ...
 * - "device" pointers are HIP device memory owned by the caller; "host"
 *   pointers are ordinary host memory owned by the caller.  The library keeps
 *   no pointer to caller memory after a call returns, and never allocates
 *   device memory inside kkm_fit / kkm_assign / kkm_cost: all scratch lives in
 *   the caller's workspace, sized by the matching *_workspace_bytes call.
 *   The workspace must be 256-byte aligned (hipMalloc memory is).
 * - stream is a hipStream_t (NULL = the default stream).  kkm_assign only
 *   enqueues work; kkm_fit and kkm_cost synchronise the stream before they
 *   return because they hand back host data.
 * - Ties: every argmin takes the lowest index (cluster index for labels,
 *   sample position for medoids).
 * - Errors: arguments are checked before any device work; on failure nothing
 *   is enqueued, outputs are unspecified, and kkm_last_error() describes the
 *   cause.  No entry point aborts or throws.
 * - A model may be used by concurrent kkm_assign / kkm_cost calls on
 *   different streams; kkm_fit writing a model must not overlap its use.
 */
#ifndef KKM_H
#define KKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kkm_status {
    KKM_OK = 0,
    KKM_ERR_INVALID_ARG = -1,   /* an argument is out of range or inconsistent */
    KKM_ERR_WORKSPACE = -2,     /* workspace NULL, misaligned or smaller than required */
    KKM_ERR_DEVICE = -3,        /* no usable GPU, or a HIP call failed */
    KKM_ERR_NONFINITE = -4,     /* the input holds NaN or Inf */
    KKM_ERR_INTERNAL = -5,
    KKM_ERR_UNSUPPORTED = -6    /* a size beyond what this build handles (message says which) */
} kkm_status;

/* Kernel functions.  The paper keeps the Mercer kernel generic (Sec. 2). */
enum kkm_kernel_type {
    KKM_KERNEL_LINEAR = 0,      /* K(x,y) = x.y */
    KKM_KERNEL_RBF = 1,         /* K(x,y) = exp(-||x-y||^2 / (2 sigma^2)) */
    KKM_KERNEL_RMSD = 2         /* K(x,y) = exp(-RMSD(x,y)^2 / (2 sigma^2)), RMSD after optimal
                                   superposition (proper rotation + translation), equal atom weights */
};

enum kkm_dtype { KKM_F32 = 0, KKM_F64 = 1 };

/* Arithmetic of the dominant n x |L| kernel block (and of kkm_assign).  FP32, BF16 and BF16X3
 * decide every label whose margin is below a computed error bound again in FP64, so labels
 * equal those of exact arithmetic except where the FP64 margin itself vanishes.  The bfloat16
 * forms run on the matrix cores for float32 samples with d >= 9 (padded to 16); other inputs
 * take the FP32 path. */
enum kkm_precision {
    KKM_PREC_FP64 = 0,
    KKM_PREC_FP32 = 1,
    KKM_PREC_BF16 = 2,          /* x.y from one bfloat16 product hi*hi' (FP32 accumulation) on MFMA: the
                                   cheap gating pass; the rows under its (wider) bound are decided again
                                   with the BF16X3 products, and those still undecided in FP64; kkm_cost
                                   then takes each row's distance to its cluster in FP64.  In kkm_fit the
                                   batch pass feeds the medoid candidates, whose bound needs the
                                   compensated products: a fit asked for BF16 runs BF16X3 there */
    KKM_PREC_BF16X3 = 3         /* x.y from split-bf16 products hi*hi' + hi*lo' + lo*hi' on MFMA */
};

/* kkm_params.flags bits */
enum kkm_fit_flags {
    KKM_FIT_GLOBAL_COST = 2,    /* also take the global cost Omega(W) after every batch (Sec. 4.1, Fig. 4):
                                   Eq. 1 over all N samples with the global medoids of that moment, in
                                   the fit's precision, into kkm_fit_info.global_cost; the workspace then
                                   holds a medoid model and an assign pass over N rows more */
    KKM_FIT_COOPERATIVE = 1     /* launch the kernels whose workgroups wait for each other (k-means++ and
                                   the landmark loop) cooperatively, so that all their workgroups are
                                   resident together even while other streams keep the GPU busy (a
                                   plain launch then only guarantees a bounded wait, reported as
                                   KKM_ERR_DEVICE); costs some microseconds per launch */
};

enum kkm_sampling {
    KKM_SAMPLE_STRIDE = 0,      /* X^i = { x_(i + jB) }           (Sec. 3.1) */
    KKM_SAMPLE_BLOCK = 1        /* X^i = a contiguous run         (Sec. 3.1) */
};

enum kkm_init {
    KKM_INIT_KMEANSPP = 0,      /* kernel k-means++ on batch 0    (Sec. 3.1) */
    KKM_INIT_RANDOM_LABELS = 1, /* uniform random labels on batch 0 */
    KKM_INIT_MEDOIDS = 2        /* caller-given batch-0 medoids */
};

typedef struct kkm_kernel {
    int32_t type;               /* enum kkm_kernel_type */
    int32_t n_atoms;            /* RMSD only: d == 3 * n_atoms */
    double sigma;               /* RBF / RMSD width, > 0 */
} kkm_kernel;

typedef struct kkm_params {
    int32_t C;                  /* clusters, 1 <= C <= size of batch 0 */
    int32_t B;                  /* mini-batches, 1 <= B <= N */
    double s;                   /* landmark fraction s = |L| B / N (Eq. 18), 0 < s <= 1;
                                   batch i has l_i = clamp(floor(s n_i + 1/2), 1, n_i) landmarks */
    int32_t max_iter;           /* T >= 1: at most T label updates per batch (Sec. 3.1 inner loop) */
    int32_t sampling;           /* enum kkm_sampling */
    int32_t init;               /* enum kkm_init */
    int32_t precision;          /* enum kkm_precision */
    int32_t flags;              /* enum kkm_fit_flags bits, 0 by default */
    uint64_t seed;              /* draws not given below come from the SplitMix64 streams of this seed */
    const int64_t* landmarks;   /* host or NULL: concatenation over batches of l_i ascending
                                   batch positions (uniform without replacement, Sec. 3.2) */
    const double* kmpp_uniforms;/* host or NULL: C values in [0,1) for k-means++ */
    const int32_t* init_labels; /* host or NULL: n_0 labels in [0,C) for RANDOM_LABELS */
    const int64_t* init_medoids;/* host: C batch-0 positions for MEDOIDS */
} kkm_params;

/* Optional host outputs of kkm_fit; every pointer may be NULL. */
typedef struct kkm_fit_info {
    int32_t* updates_per_batch; /* [B] label updates made on each batch: landmark-only updates until the
                                   landmark labels repeat (<= T-1), plus the batch-wide pass */
    int64_t* batch_medoids;     /* [B*C] sample index of m_j^i (Eq. 10), -1 if cluster j was empty */
    int64_t* batch_counts;      /* [B*C] |w_j^i| */
    int64_t* global_medoids;    /* [B*C] sample index of m_j after merging batch i (Eq. 12), -1 unset */
    int64_t evals_algorithmic;  /* out: sum_i n_i l_i (Eq. 18) + n_i C (Eq. 8 / k-means++) + n_i C_i (merge) */
    int64_t evals_performed;    /* out: kernel evaluations the device carried out */
    int64_t rows_refined;       /* out: labels re-decided in FP64 */
    int64_t medoid_candidates;  /* out: medoid candidates re-evaluated in FP64 */
    int32_t time_phases;        /* in: 1 records HIP events on the stream around each phase; 2 only around
                                   the landmark loop kernel and the batch-wide distance kernel (three
                                   events per batch; the other ms_* stay 0); 0 none */
    int32_t reserved;
    double ms_init;             /* out (time_phases): k-means++ / initial medoids */
    double ms_landmark;         /* out: landmark block, initial labels, landmark loop, centroid support */
    double ms_dist;             /* out: batch-wide distance kernel (Eq. 15-17 over every batch sample) */
    double ms_refine;           /* out: FP64 re-decision of near-tie rows */
    double ms_select;           /* out: member counts, batch medoids (Eq. 10), merge (Eq. 11-13) */
    double ms_landmark_loop;    /* out: the landmark loop kernel alone (part of ms_landmark) */
    int64_t* landmark_trace;    /* host [64] or NULL: device wall-clock stamps (100 MHz) taken by the first
                                   workgroup at the steps of batch 0's landmark phase: [0] count, then
                                   start, block done, init done, and per update: sort, sums, barrier,
                                   g^, barrier (profiling aid) */
    double* medoid_displacement; /* host [B*C] or NULL: kernel-space displacement of each global medoid
                                   at batch i, ||phi(m_j after batch i) - phi(m_j before)|| =
                                   sqrt(K(n,n) - 2 K(n,o) + K(o,o)) in FP64 (the sampling-quality
                                   observable of Sec. 4.1, Fig. 4); 0 when m_j is kept, NaN when it
                                   was unset before the batch */
    double* partial_cost;       /* host [B] or NULL: the partial cost Omega(W^i) of every batch (Sec. 4.1,
                                   Fig. 4), Eq. 1 over the batch's rows with the batch's centroids of
                                   Eq. 14 after its loop: the sum of each row's distance to its nearest
                                   centroid, summed in FP64 in a fixed order (a row decided in FP32 adds
                                   its distance formed from FP32 sums, within the row's error bound) */
    double* global_cost;        /* host [B] or NULL (needs KKM_FIT_GLOBAL_COST in kkm_params.flags): the
                                   global cost Omega(W) after the merge of every batch (Sec. 4.1, Fig. 4),
                                   Eq. 1 over all N samples against the global medoids of that moment,
                                   summed in FP64 in a fixed order as kkm_cost does */
} kkm_fit_info;

/* A clustering model: C sparse centroids w_j = sum_{l in segment j} a_l phi(s_l), kept resident in
 * device memory with the self terms a^T K a in FP64.  A fitted model holds the C global medoids
 * (one support row each, a = 1, Sec. 3.1). */
typedef struct kkm_model kkm_model;

/* Allocate an empty model on the current HIP device for samples of dimension d, C clusters and at
 * most max_support support rows (>= C for kkm_fit).  The model owns its device memory until
 * kkm_model_free. */
kkm_status kkm_model_create(const kkm_kernel* kernel, int64_t d, int32_t C, int64_t max_support,
                            int32_t dtype, kkm_model** out);

/* Load general sparse centroids from host: support [n_support*d] rows, offsets [C+1] (segment j is
 * rows offsets[j]..offsets[j+1]-1; an empty segment disables cluster j), coef [n_support].  The self
 * terms a^T K_SS a are computed on the device in FP64.  Synchronous. */
kkm_status kkm_model_load(kkm_model* model, const void* support, int64_t n_support,
                          const int64_t* offsets, const double* coef);

/* Copy a model to host.  support: [n_used*d] in the model dtype; offsets [C+1]; coef [n_used];
 * self [C] (a^T K a, +inf for disabled clusters); counts [C] (|w_j| of a fitted model, else 0);
 * medoid_index [C] (sample index of a fitted medoid, else -1).  Any pointer may be NULL. */
kkm_status kkm_model_export(const kkm_model* model, void* support, int64_t* offsets, double* coef,
                            double* self, int64_t* counts, int64_t* medoid_index);

/* Shape of a model: dimension, clusters, support rows in use. */
kkm_status kkm_model_shape(const kkm_model* model, int64_t* d, int32_t* C, int64_t* n_used);

void kkm_model_free(kkm_model* model);

/* ---------------------------------------------------------------- fit (Sec. 3.1-3.2) */

/* Workspace bytes kkm_fit needs for these sizes (0 if the arguments are invalid). */
size_t kkm_fit_workspace_bytes(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                               const kkm_params* params);

/* The memory knob of Sec. 3.3 (Eq. 19 gives the smallest number of mini-batches for the paper's own
 * footprint model): the smallest B, with every other field of *params as given (its B, landmarks,
 * init_labels and init_medoids are not read), for which kkm_fit's workspace for N x d samples is at
 * most budget_bytes (X itself is the caller's and not counted).  The workspace falls with B while the
 * landmark block dominates and rises again with the per-batch state; B is searched on the falling
 * side, below the B (a power of two up to N / C) of the smallest workspace: the B returned fits,
 * and B - 1 does not.  Host only, no device work.  Returns 0 when no B fits or an argument is
 * invalid (kkm_last_error says which). */
int64_t kkm_fit_min_batches(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                            const kkm_params* params, size_t budget_bytes);

/* Cluster X (device, N x d) with the paper's mini-batch landmark kernel k-means:
 *   for each batch i (stride or block sampling): draw l_i landmarks; initialise their labels (batch 0:
 *   k-means++ / random / given medoids; later batches: nearest global medoid, Eq. 8); iterate
 *   Eq. 15-17 on the landmarks until they stop changing or T-1 updates were made; label the whole
 *   batch once from the final centroids; take the batch medoids (Eq. 10); merge them into the global
 *   medoids with alpha = |w_j^i| / (|w_j^i| + |w_j|) (Eq. 11-13; empty clusters keep theirs).
 * Because Eq. 16-17 read only landmark labels, the landmark-only loop followed by one full pass gives
 * exactly the labels of the paper's loop over the whole batch with at most T updates.
 * Outputs: model (created with this kernel, d, C, dtype and max_support >= C) receives the global
 * medoids; labels_out (device [N] int32, or NULL) receives each sample's label from its own batch.
 * Returns KKM_ERR_NONFINITE if X holds NaN/Inf (results are then meaningless). */
kkm_status kkm_fit(const void* X, int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                   const kkm_params* params, void* workspace, size_t workspace_bytes, void* stream,
                   kkm_model* model, int32_t* labels_out, kkm_fit_info* info);

/* ---------------------------------------------------------------- restarts (Sec. 4.5) */

/* Workspace bytes of kkm_fit_restarts (0 if the arguments are invalid). */
size_t kkm_fit_restarts_workspace_bytes(int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                                        const kkm_params* params, int32_t restarts);

/* Best of several restarts (Sec. 4.5 keeps the lowest-cost run of five kernel k-means++ fits): fit number r
 * (r = 0 .. restarts-1) is kkm_fit with seed params->seed + r (its own landmarks and k-means++ draws:
 * params->landmarks, kmpp_uniforms and init_labels must be NULL), followed by its cost, Eq. 1 over all N
 * samples in FP64 with the fit's medoids (as kkm_cost in FP64).  All fits and costs run back to back on
 * stream out of one workspace, with one synchronisation; the lowest cost wins (the lowest r on equal
 * costs) and is written to model, labels_out and info as kkm_fit writes its result.  costs_out: host
 * [restarts] or NULL; best_out: host, the winning r, or NULL.  Synchronous. */
kkm_status kkm_fit_restarts(const void* X, int64_t N, int64_t d, int32_t dtype, const kkm_kernel* kernel,
                            const kkm_params* params, int32_t restarts, void* workspace, size_t workspace_bytes,
                            void* stream, kkm_model* model, int32_t* labels_out, kkm_fit_info* info,
                            double* costs_out, int32_t* best_out);

/* ---------------------------------------------------------------- assign / cost (Eq. 1-2) */

size_t kkm_assign_workspace_bytes(const kkm_model* model, int64_t n, int32_t precision);

/* labels_out[i] = argmin_j K(x_i,x_i) - 2 sum_l a_l K(x_i, s_l) + a^T K a  (Eq. 2), for the n rows of
 * X (device).  gap_out (device [n] float, or NULL) receives (d2 - d1) / max(|d1|, |d2|, |K(x,x)|),
 * best and second-best distance.  Enqueued on stream; returns without waiting. */
kkm_status kkm_assign(const kkm_model* model, const void* X, int64_t n, int32_t dtype, int32_t precision,
                      void* workspace, size_t workspace_bytes, void* stream,
                      int32_t* labels_out, float* gap_out);

/* kkm_assign without a workspace, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same labels and margins as
 * kkm_assign, with the scratch taken from a fixed 48 MiB device array that the library holds on every
 * GPU it runs on until the process ends.  Allocates nothing.  Rows of n * (16.125 bytes + for RMSD one
 * centred frame and its squared RMSDs to the support) plus fixed parts must fit that array (about
 * 3 million rows of d = 64, 55 000 frames of 50 atoms against 50 medoids): a larger n returns
 * KKM_ERR_UNSUPPORTED and enqueues nothing.  All calls on one GPU share
 * its array: calls that overlap on that GPU (other streams or host threads) race and must be
 * serialised by the caller.  Enqueued on stream; returns without waiting. */
kkm_status kkm_assign_noalloc(const kkm_model* model, const void* X, int64_t n, int32_t dtype, int32_t precision,
                              void* stream, int32_t* labels_out, float* gap_out);

/* *cost_out (host) = sum_i min_j ||phi(x_i) - w_j||^2  (Eq. 1 with Eq. 2 labels), summed in FP64 in a
 * fixed order (the same bits on every run).  Uses the workspace of kkm_assign.  Synchronous. */
kkm_status kkm_cost(const kkm_model* model, const void* X, int64_t n, int32_t dtype, int32_t precision,
                    void* workspace, size_t workspace_bytes, void* stream, double* cost_out);

/* ---------------------------------------------------------------- kernel block (Sec. 2, Eq. 16) */

/* Workspace bytes of kkm_kernel_block (0 if the arguments are invalid): RMSD needs a centred copy of
 * both row sets, the other kernels none (256 is returned then). */
size_t kkm_kernel_block_workspace_bytes(const kkm_kernel* kernel, int64_t nx, int64_t ny, int64_t d, int32_t dtype);

/* The kernel matrix between two row sets, K_out[i * ny + j] = K(x_i, y_j) in FP64 (Sec. 2 writes every
 * feature-space inner product as K; the landmark block of Eq. 16 is K(X_L, X_L)).  X: device [nx*d],
 * Y: device [ny*d], rows in dtype; K_out: device [nx*ny] doubles.  Linear: x.y; RBF from explicit
 * coordinate differences; RMSD: both frame sets are centred into the workspace, the 3x3 correlation
 * of each pair is summed in FP64 and the largest eigenvalue of its 4x4 key matrix is found by
 * Newton's method on the characteristic polynomial, solved again by Jacobi rotations where Newton
 * converges slowly (a multiple or nearly multiple largest root: collinear or symmetric frames).  These
 * are the FP64 evaluations the library's re-decisions, medoid and merge steps use.  Enqueued on
 * stream; returns without waiting. */
kkm_status kkm_kernel_block(const kkm_kernel* kernel, const void* X, int64_t nx, const void* Y, int64_t ny, int64_t d,
                            int32_t dtype, void* workspace, size_t workspace_bytes, void* stream, double* K_out);

/* ---------------------------------------------------------------- host-only helpers (no GPU) */

/* l = clamp(floor(s n + 1/2), 1, n). */
int64_t kkm_landmark_count(int64_t n, double s);

/* The draws kkm_fit makes when the caller passes none (SplitMix64 streams keyed by seed, purpose and
 * batch; Lemire bounded integers; partial Fisher-Yates).  out: [kkm_landmark_count(n,s)] ascending
 * positions / [C] uniforms / [n] labels. */
kkm_status kkm_draw_landmarks(uint64_t seed, int32_t batch, int64_t n, double s, int64_t* out);
kkm_status kkm_draw_kmpp_uniforms(uint64_t seed, int32_t C, double* out);
kkm_status kkm_draw_init_labels(uint64_t seed, int64_t n, int32_t C, int32_t* out);

/* Description of the last error on the calling thread (valid until its next call). */
const char* kkm_last_error(void);

/* Library version string. */
const char* kkm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KKM_H */
