// Selection steps of a mini-batch, all in FP64:
//
//   kernel k-means++ seeding of the first batch (D^2 sampling in feature space);
//   batch member counts |w_j^i| and the scatter of batch labels to caller order;
//   batch medoids m_j^i = argmin_x d_last(x, j) over the batch (Eq. 10);
//   the merge m_j <- argmin_x K(x,x) - 2(1-alpha) K(x, m_j) - 2 alpha K(x, m_j^i)
//   with alpha = |w_j^i| / (|w_j^i| + |w_j|) (Eq. 11-13; alpha = 0 leaves m_j alone);
//   building model arrays from medoids or from general sparse centroids;
//   centring of RMSD frames.
//
// Every argmin keeps the lowest index on ties; minima are order-independent, so the chunked
// reductions give the same result as a sequential scan.
#include <cstdlib>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {

namespace {

template <typename TI>
__device__ __forceinline__ const TI* brow(const BatchView& b, int64_t pos) {
    return static_cast<const TI*>(b.X) + (b.base + pos * b.stride) * b.d;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// (value, index) minimum with the lowest index on equal values
__device__ __forceinline__ void vmin(double& v, int64_t& i, double v2, int64_t i2) {
    if (v2 < v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__device__ void block_vmin(double& v, int64_t& i) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    sv[threadIdx.x] = v;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            double a = sv[threadIdx.x];
            int64_t ia = si[threadIdx.x];
            vmin(a, ia, sv[threadIdx.x + w], si[threadIdx.x + w]);
            sv[threadIdx.x] = a;
            si[threadIdx.x] = ia;
        }
        __syncthreads();
    }
    v = sv[0];
    i = si[0];
    __syncthreads();
}

// ----------------------------------------------------------------------------- k-means++
// Kernel k-means++ (Sec. 3.1) as one kernel whose workgroups are all resident: workgroup g owns the
// contiguous rows [g R, (g + 1) R).  Pick k >= 1: every workgroup folds medoid k - 1 into its rows of
// D^2 (D2 buffers alternate between picks), publishes its row sum, and once every sum of the pick is
// there, every workgroup derives the same pick -- the owner chunk from the prefix of the G sums (in
// workgroup order), then the row inside it by an ordered scan of that chunk.  The picked index is the
// first row whose running sum exceeds u_k times the total (rows in index order; a pick with no mass
// falls back to floor(u_k n)).
//
// The sums are their own signal: pick k uses buffer k % 3 of part, filled with -1 (sums are >= 0)
// before the launch, and the readers wait until every slot of it holds a sum.  Workgroup g clears its
// slot of buffer (k + 1) % 3 at the start of pick k, before publishing its pick-k sum: that buffer
// was last read in pick k - 2, which every workgroup has finished once all pick k - 1 sums exist --
// and g saw them all before starting pick k; a reader of pick k + 1 in turn waits for g's pick-k sum
// first, so it cannot find the old value.  Only the owner workgroup searches its own rows for the
// pick (its D^2 values are its own) and publishes it as chosen[k], filled with -1 before the launch;
// the others wait for it.
struct KppArgs {
    BatchView b;
    KSpec ks;
    int32_t C;
    const double* uniforms;   // [C]
    int32_t* chosen;          // [C] out
    double* D2;               // [2][n]
    double* part;             // [3][G], filled with -1 before the launch
    int32_t* error;           // set when a wait exceeded its cap
    int32_t lds_rows;         // own rows staged in LDS (linear / RBF, when they fit)
};

constexpr unsigned kKppSpinCap = 1u << 26;
constexpr int kKppMaxGrid = 256;  // <= 256: one partial per thread in the owner search

// The values exchanged between the workgroups (D^2 rows, per-workgroup sums) are written and read as
// relaxed device-scope atomics, which pass the per-XCD L2 caches; a workgroup's sum is then published
// only after every thread's stores have completed (no L2 write-back or invalidation).
template <typename T>
__device__ __forceinline__ void kput(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ T kget(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes the workgroup's sum of pick k (thread 0, which cleared the workgroup's slot for pick
// k + 1 at the start of the pick: that store is complete first).
__device__ __forceinline__ void kpp_publish(const KppArgs& a, int k, double gsum) {
    if (threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        kput(a.part + (int64_t)(k % 3) * gridDim.x + blockIdx.x, gsum);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
}

// Thread t < G: workgroup t's sum of pick k, once it is there (bounded wait; a wait past the cap
// reports the error and goes on with what it read, never a hang).
__device__ __forceinline__ double kpp_wait_sum(const KppArgs& a, int k) {
    const int G = gridDim.x, t = threadIdx.x;
    if (t >= G) return 0.0;
    const double* p = a.part + (int64_t)(k % 3) * G + t;
    double v = kget(p);
    unsigned polls = 0;
    while (v < 0.0) {
        __builtin_amdgcn_s_sleep(1);
        if (++polls > kKppSpinCap) {
            atomicOr(a.error, 1);
            break;
        }
        v = kget(p);
    }
    return v;
}

// Inclusive scan of one value per thread over the workgroup in a fixed order: within each wavefront
// by shuffles, then the wavefront totals in wavefront order.  *excl is the previous thread's
// inclusive value, bit for bit (the same additions of the same operands).  Returns the total.
__device__ __forceinline__ double block_scan(double v, double* sh, double* excl, double* incl) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    const double xprev = __shfl_up(x, 1, 64);
    if (lane == 63) sh[w] = x;
    __syncthreads();
    double base = 0.0;   // sum of the totals of the earlier wavefronts, in order
    for (int i = 0; i < w; ++i) base = i == 0 ? sh[0] : base + sh[i];
    double total = 0.0;
    for (int i = 0; i < nw; ++i) total = i == 0 ? sh[0] : total + sh[i];
    *incl = w == 0 ? x : base + x;
    *excl = lane > 0 ? (w == 0 ? xprev : base + xprev) : base;
    __syncthreads();
    return total;
}

template <typename TI, int DP>
__global__ __launch_bounds__(256) void kmeanspp_kernel(KppArgs a) {
    extern __shared__ __align__(16) unsigned char kpp_smem[];
    __shared__ double sh[256];
    __shared__ int32_t pick_sh;
    __shared__ int32_t owner_sh;
    __shared__ double base_sh;
    constexpr int XS = DP + 1;                       // padded LDS row stride of the own rows
    const int64_t n = a.b.n;
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    const int64_t R = (n + G - 1) / G;
    auto chunk = [&](int wg, int64_t* lo, int64_t* hi) {
        *lo = min<int64_t>(n, (int64_t)wg * R);
        *hi = min<int64_t>(n, *lo + R);
    };
    auto slice = [&](int64_t lo, int64_t hi, int64_t* qlo, int64_t* qhi) {   // thread t's contiguous part
        const int64_t w = (hi - lo + nt - 1) / nt;
        *qlo = min<int64_t>(hi, lo + (int64_t)t * w);
        *qhi = min<int64_t>(hi, *qlo + w);
    };
    const TI* X = static_cast<const TI*>(a.b.X);
    auto row = [&](int64_t q) { return X + (a.b.base + q * a.b.stride) * a.b.d; };
    int64_t lo, hi, tlo, thi;
    chunk(g, &lo, &hi);
    slice(lo, hi, &tlo, &thi);
    // linear / RBF with the own rows in LDS (the rows are read once; every pick reads LDS)
    const bool lds_rows = DP > 0 && a.lds_rows != 0;
    TI* xs = reinterpret_cast<TI*>(kpp_smem);                                      // [R][XS] + medoid row
    double* d2own = reinterpret_cast<double*>(kpp_smem + ((sizeof(TI) * (R + 1) * XS + 15) & ~size_t(15)));   // [R]
    if (lds_rows) {   // four elements per thread at a time, loads issued unconditionally (clamped, masked)
        const int64_t nel = (hi - lo) * DP;
        for (int64_t p0 = t; p0 < nel; p0 += 4 * (int64_t)nt) {
            TI v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = min(p0 + u * (int64_t)nt, nel - 1);
                const int64_t r = p / DP;
                const int c = (int)(p - r * DP);
                v[u] = row(lo + r)[min(c, (int)a.b.d - 1)] * (c < a.b.d ? TI(1) : TI(0));
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = p0 + u * (int64_t)nt;
                if (p < nel) xs[(p / DP) * XS + (p - (p / DP) * DP)] = v[u];
            }
        }
        __syncthreads();
    }
    int32_t prev = (int32_t)min<int64_t>((int64_t)floor(a.uniforms[0] * (double)n), n - 1);
    if (g == 0 && t == 0) a.chosen[0] = prev;
    for (int k = 1; k < a.C; ++k) {
        const int cur = k & 1, old = cur ^ 1;
        double* D2 = a.D2 + (int64_t)cur * n;
        const double* D2o = a.D2 + (int64_t)old * n;
        // fold medoid k - 1 into the own rows; row sums in order (thread slice, then threads)
        if (t == 0 && k + 1 < a.C) kput(a.part + (int64_t)((k + 1) % 3) * G + g, -1.0);   // (see above)
        const TI* m = row(prev);
        // the medoid row, read once per pick into LDS (after the own rows); the evaluation below
        // names it through the LDS array itself, so that its reads stay LDS reads
        TI* const ms = xs + R * XS;
        if (lds_rows) {
            for (int c = t; c < DP; c += nt) ms[c] = c < a.b.d ? m[c] : TI(0);
            __syncthreads();
        }
        const double kmm = lds_rows ? kself64(a.ks, (const TI*)ms) : kself64(a.ks, m);
        double ts = 0.0;
        for (int64_t q = tlo; q < thi; ++q) {
            double v;
            if (lds_rows) {
                if constexpr (DP > 0) {
                    // both rows are zero past d in LDS, so the sum runs over DP dimensions with no
                    // clamp or mask (the padded terms add fma(0, 0, acc) = acc, as the masked terms of
                    // the general evaluator do), all reads in flight together
                    const TI* x = xs + (q - lo) * XS;
                    double acc = 0.0;
                    if (a.ks.type == KKM_KERNEL_LINEAR) {
#pragma unroll
                        for (int k = 0; k < DP; ++k) acc = fma((double)x[k], (double)ms[k], acc);
                    } else {
#pragma unroll
                        for (int k = 0; k < DP; ++k) {
                            const double df = (double)x[k] - (double)ms[k];
                            acc = fma(df, df, acc);
                        }
                        acc = ::exp(-acc * a.ks.inv2s2);
                    }
                    v = (kself64(a.ks, x) - 2.0 * acc) + kmm;
                }
                v = v > 0.0 ? v : 0.0;
                if (k > 1) v = fmin(d2own[q - lo], v);
                d2own[q - lo] = v;
            } else {
                const TI* x = row(q);
                v = (kself64(a.ks, x) - 2.0 * k64p<DP>(a.ks, x, m)) + kmm;
                v = v > 0.0 ? v : 0.0;
                if (k > 1) v = fmin(D2o[q], v);
                D2[q] = v;
            }
            ts += v;
        }
        if (!lds_rows) __builtin_amdgcn_s_waitcnt(0);   // (the owner search below reads other threads' D^2)
        double e0, i0;
        const double gsum = block_scan(ts, sh, &e0, &i0);
        kpp_publish(a, k, gsum);
        // every workgroup derives the same pick: owner chunk from the partials, then the row
        double pe, pi;
        const double total = block_scan(kpp_wait_sum(a, k), sh, &pe, &pi);   // G <= 256
        const double u = a.uniforms[k];
        if (t == 0) {
            pick_sh = (int32_t)min<int64_t>((int64_t)floor(u * (double)n), n - 1);   // no mass: fallback
            owner_sh = -1;
        }
        __syncthreads();
        const double thr = u * total;
        if (total > 0.0 && t < G && pi > thr && pe <= thr) {   // at most one thread
            owner_sh = t;
            base_sh = pe;
        }
        __syncthreads();
        const int owner = owner_sh;
        if (owner == g) {   // the pick lies in this workgroup's rows: find it (rows in order) and publish it
            auto d2 = [&](int64_t q) { return lds_rows ? d2own[q - lo] : (double)D2[q]; };
            double cs = 0.0;
            for (int64_t q = tlo; q < thi; ++q) cs += d2(q);
            double ce, ci;
            (void)block_scan(cs, sh, &ce, &ci);
            const double base = base_sh;
            if (base + ci > thr && base + ce <= thr) {   // at most one thread
                double loc = base + ce;
                int64_t pk = thi - 1;
                for (int64_t q = tlo; q < thi; ++q) {
                    loc += d2(q);
                    if (loc > thr) {
                        pk = q;
                        break;
                    }
                }
                pick_sh = (int32_t)pk;
            }
            __syncthreads();
            if (t == 0) kput(a.chosen + k, pick_sh);   // (the fallback when rounding left no row)
        } else if (owner >= 0) {   // wait for the owner's pick (bounded; past the cap: error reported)
            if (t == 0) {
                int32_t v = kget(a.chosen + k);
                unsigned polls = 0;
                while (v < 0) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++polls > kKppSpinCap) {
                        atomicOr(a.error, 1);
                        v = pick_sh;
                        break;
                    }
                    v = kget(a.chosen + k);
                }
                pick_sh = v;
            }
            __syncthreads();
        } else if (g == 0 && t == 0) {
            kput(a.chosen + k, pick_sh);   // no mass: the fallback pick
        }
        prev = pick_sh;
        __syncthreads();
    }
}

template <typename TI>
__global__ void set_medoids_kernel(BatchView b, KSpec ks, int C, const int32_t* chosen, TI* M, int64_t Mpad,
                                   double* Mself, int64_t* Midx, int64_t* wcount) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < C; j += gridDim.x * blockDim.x) {
        wcount[j] = 0;
        if (!chosen) {
            Mself[j] = kInf;
            Midx[j] = -1;
            for (int64_t c = 0; c < Mpad; ++c) M[j * Mpad + c] = TI(0);
            continue;
        }
        const TI* x = brow<TI>(b, chosen[j]);
        for (int64_t c = 0; c < Mpad; ++c) M[j * Mpad + c] = c < b.d ? x[c] : TI(0);
        Mself[j] = kself64(ks, x);
        Midx[j] = b.base + (int64_t)chosen[j] * b.stride;
    }
}

// ----------------------------------------------------------------------------- batch medoids (Eq. 10)
// The batch-wide distance pass leaves, for every cluster j, U_j = min over rows of D + E (an upper
// bound on the smallest exact distance).  Candidates are the rows with D - E <= U_j; each is
// re-evaluated in FP64 and the lowest (value, position) is the batch medoid.
constexpr int kRowsPerBlock = 256;

// Grid (row chunks) x (clusters): member counts per chunk, label scatter, and the candidates of the
// block: rows with D - E <= U_j, where U_j is the minimum of the distance pass's per-block column
// minima (every block reduces them itself; the minimum is exact in any order).  The block then
// evaluates its candidates in FP64,
//   d(x, j) = K(x,x) - 2 sum_l a_l K(x, s_l) + self_j,
// a group of lanes per candidate over the segment's support rows, and appends (row, cluster, value)
// to the candidate list.  (Large grids, where the evaluation's registers would cost occupancy, take
// medoid_candidates_multi_kernel and candidate_eval_kernel instead.)
template <typename TD, typename TI, int DP>
__global__ __launch_bounds__(256) void medoid_candidates_kernel(SelectArgs a) {
    const int j = blockIdx.y, chunk = blockIdx.x;
    const int64_t q = (int64_t)chunk * kRowsPerBlock + threadIdx.x;
    const bool active = q < a.b.n;
    __shared__ int cnt, ncand, base;
    __shared__ int32_t cq[kRowsPerBlock];
    __shared__ double umin[kRowsPerBlock / 64];
    if (threadIdx.x == 0) {
        cnt = 0;
        ncand = 0;
    }
    // the row's label, distance and bound are loaded first: their loads overlap the column minimum
    const int64_t qa = active ? q : 0;
    const TD* Dt = static_cast<const TD*>(static_cast<const void*>(a.Dt)) + (int64_t)j * a.ldD;
    const int lab = a.labels[qa];
    const double D = (double)Dt[qa];
    const double Eq = (double)a.Erow[qa];
    double U;
    if (a.colpart_blocks > 0) {
        double v = kInf;
        for (int64_t b = threadIdx.x; b < a.colpart_blocks; b += blockDim.x)
            v = fmin(v, a.colpart[(int64_t)j * a.colpart_ld + b]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
        if ((threadIdx.x & 63) == 0) umin[threadIdx.x >> 6] = v;
        __syncthreads();
        v = umin[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmin(v, umin[w]);
        U = v < kInf ? v : ord_dec(~0ull);
    } else {
        __syncthreads();
        U = ord_dec(a.colmin[j]);
    }
    if (active) {
        if (j == 0 && a.label_out) a.label_out[a.b.base + q * a.b.stride] = lab;
        if (lab == j) atomicAdd(&cnt, 1);
        if (D < kInf && D - Eq <= U) cq[atomicAdd(&ncand, 1)] = (int32_t)q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.mpart_c[(int64_t)j * a.nchunk + chunk] = cnt;
        base = ncand ? atomicAdd(a.cand_count, ncand) : 0;
    }
    __syncthreads();
    // groups of L lanes per candidate, L the power of two (<= 64) covering the segment, so that
    // short segments put several candidates on one wavefront
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const TI* rows = static_cast<const TI*>(a.sup.rows);
    const int lo = a.sup.offsets[j], hi = a.sup.offsets[j + 1];
    int L = 64;
    while (L > 1 && L / 2 >= hi - lo) L >>= 1;
    const int per_wave = 64 / L, sub = lane / L, sl = lane % L;
    for (int c0 = wave * per_wave; c0 < ncand; c0 += nwaves * per_wave) {
        const int c = c0 + sub;
        const bool ok = c < ncand && base + c < a.cand_cap;   // (beyond the capacity: the list is full)
        const int64_t qq = ok ? cq[c] : 0;
        const TI* x = brow<TI>(a.b, qq);
        double f = 0.0;
        if (ok)
            for (int l = lo + sl; l < hi; l += L) f += a.sup.coef64[l] * k64p<DP>(a.ks, x, rows + (int64_t)l * a.sup.dpad);
        for (int o = L / 2; o >= 1; o >>= 1) f += __shfl_xor(f, o, 64);   // within the lane group
        if (ok && sl == 0) {
            a.cand_q[base + c] = (int32_t)qq;
            a.cand_j[base + c] = j;
            a.cand_v[base + c] = kself64(a.ks, x) - 2.0 * f + a.sup.self[j];
        }
    }
}

// d(x_q, j) as above by one wavefront (all 64 lanes take part; every lane returns the value).  Linear
// / RBF: each support row of the segment is split over DP / 4 lanes, four dimensions each (one load of
// the candidate's row and one of the support row per lane), the lane parts added by a butterfly in a
// fixed order, and the rows' terms a_l K(x, s_l) added across the pass's rows by a butterfly and pass
// after pass: FP64 up to the order of the roundings.  RMSD: a support row per lane.
template <typename TI, int DP>
__device__ __forceinline__ double eval_candidate_wave(const SelectArgs& a, int64_t q, int j) {
    const int lane = threadIdx.x & 63;
    const TI* rows = static_cast<const TI*>(a.sup.rows);
    const TI* x = brow<TI>(a.b, q);
    const int lo = a.sup.offsets[j], hi = a.sup.offsets[j + 1];
    const double sj = a.sup.self[j];
    if constexpr (DP == 0) {
        double f = 0.0;
        for (int l = lo + lane; l < hi; l += 64) f += a.sup.coef64[l] * k64p<DP>(a.ks, x, rows + (int64_t)l * a.sup.dpad);
        f = wave_sum(f);
        return kself64(a.ks, x) - 2.0 * f + sj;
    } else {
        constexpr int LPR = DP >= 4 ? DP / 4 : 1;   // lanes per support row
        constexpr int RPP = 64 / LPR;               // support rows per pass
        const int d = (int)a.ks.d;
        const bool lin = a.ks.type == KKM_KERNEL_LINEAR;
        const int sub = lane % LPR, rr = lane / LPR, k0 = 4 * sub;
        // the lane's four dimensions of the candidate (zero past d)
        double xv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) xv[k] = k0 + k < d ? (double)x[min(k0 + k, d - 1)] : 0.0;
        double xx = 0.0;   // linear: K(x, x) from the same lane parts
        if (lin) {
#pragma unroll
            for (int k = 0; k < 4; ++k) xx = fma(xv[k], xv[k], xx);
#pragma unroll
            for (int o = 1; o < LPR; o <<= 1) xx += __shfl_xor(xx, o, 64);
        }
        double f = 0.0;
        for (int l0 = lo; l0 < hi; l0 += RPP) {
            const int l = l0 + rr;
            const bool on = l < hi;
            const TI* sr = rows + (int64_t)(on ? l : lo) * a.sup.dpad;
            double p = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double y = k0 + k < d ? (double)sr[min(k0 + k, DP - 1)] : 0.0;
                if (lin) {
                    p = fma(xv[k], y, p);
                } else {
                    const double t = xv[k] - y;
                    p = fma(t, t, p);
                }
            }
#pragma unroll
            for (int o = 1; o < LPR; o <<= 1) p += __shfl_xor(p, o, 64);
            const double kv = lin ? p : ::exp(-p * a.ks.inv2s2);
            double term = on ? a.sup.coef64[on ? l : lo] * kv : 0.0;
#pragma unroll
            for (int o = LPR; o < 64; o <<= 1) term += __shfl_xor(term, o, 64);
            f += term;
        }
        return (lin ? xx : 1.0) - 2.0 * f + sj;
    }
}

// The large-grid form of the candidate scan: a block takes JPB clusters of its row chunk, so that the
// rows' labels and bounds are read once for all of them and the grid is JPB times smaller; per
// cluster the same member counts, label scatter and candidates as above, appended as (row, cluster)
// and, for linear / RBF, evaluated by the block (a wavefront per candidate, eval_candidate_wave);
// RMSD candidates are evaluated by candidate_eval_kernel.
template <typename TD, typename TI, int DP, int JPB>
__global__ __launch_bounds__(256) void medoid_candidates_multi_kernel(SelectArgs a) {
    static_assert(kRowsPerBlock == 256, "a row per thread");
    const int jb = blockIdx.y * JPB, chunk = blockIdx.x;
    const int64_t q = (int64_t)chunk * kRowsPerBlock + threadIdx.x;
    const bool active = q < a.b.n;
    __shared__ int cnt[JPB], ncand, base;
    __shared__ int32_t cq[JPB * kRowsPerBlock], cj[JPB * kRowsPerBlock];
    __shared__ double umin[JPB][kRowsPerBlock / 64];
    if (threadIdx.x < JPB) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) ncand = 0;
    // the row's label, bound and distances are loaded first: their loads overlap the column minima
    const int64_t qa = active ? q : 0;
    const TD* Dt = static_cast<const TD*>(static_cast<const void*>(a.Dt));
    const int lab = a.labels[qa];
    const double Eq = (double)a.Erow[qa];
    double D[JPB], U[JPB];
#pragma unroll
    for (int jj = 0; jj < JPB; ++jj) D[jj] = (double)Dt[(int64_t)min(jb + jj, a.C - 1) * a.ldD + qa];
    if (a.colpart_blocks > 0) {
        double v[JPB];
#pragma unroll
        for (int jj = 0; jj < JPB; ++jj) v[jj] = kInf;
        // two strides of partials at a time, their loads issued together (index clamped, value
        // masked; the minimum is exact in any order)
        for (int64_t b0 = threadIdx.x; b0 < a.colpart_blocks; b0 += 2 * (int64_t)blockDim.x) {
            double c[2][JPB];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int64_t b = min<int64_t>(b0 + u * (int64_t)blockDim.x, a.colpart_blocks - 1);
#pragma unroll
                for (int jj = 0; jj < JPB; ++jj) c[u][jj] = a.colpart[(int64_t)min(jb + jj, a.C - 1) * a.colpart_ld + b];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (b0 + u * (int64_t)blockDim.x < a.colpart_blocks)
#pragma unroll
                    for (int jj = 0; jj < JPB; ++jj) v[jj] = fmin(v[jj], c[u][jj]);
        }
#pragma unroll
        for (int jj = 0; jj < JPB; ++jj) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v[jj] = fmin(v[jj], __shfl_xor(v[jj], o, 64));
            if ((threadIdx.x & 63) == 0) umin[jj][threadIdx.x >> 6] = v[jj];
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < JPB; ++jj) {
            double w = umin[jj][0];
            for (int i = 1; i < (int)(blockDim.x >> 6); ++i) w = fmin(w, umin[jj][i]);
            U[jj] = w < kInf ? w : ord_dec(~0ull);
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < JPB; ++jj) U[jj] = ord_dec(a.colmin[min(jb + jj, a.C - 1)]);
    }
    if (active) {
        if (jb == 0 && a.label_out) a.label_out[a.b.base + q * a.b.stride] = lab;
#pragma unroll
        for (int jj = 0; jj < JPB; ++jj) {
            const int j = jb + jj;
            if (j < a.C) {
                if (lab == j) atomicAdd(&cnt[jj], 1);
                if (D[jj] < kInf && D[jj] - Eq <= U[jj]) {
                    const int c = atomicAdd(&ncand, 1);
                    cq[c] = (int32_t)q;
                    cj[c] = j;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < JPB && jb + (int)threadIdx.x < a.C) a.mpart_c[(int64_t)(jb + threadIdx.x) * a.nchunk + chunk] = cnt[threadIdx.x];
    if (threadIdx.x == 0) base = ncand ? atomicAdd(a.cand_count, ncand) : 0;
    __syncthreads();
    for (int c = threadIdx.x; c < ncand; c += blockDim.x)
        if (base + c < a.cand_cap) {
            a.cand_q[base + c] = cq[c];
            a.cand_j[base + c] = cj[c];
        }
    if constexpr (DP > 0) {
        const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
        for (int c = wave; c < ncand; c += nwaves) {   // (uniform over the wavefront)
            if (base + c >= a.cand_cap) break;          // (beyond the capacity: the list is full)
            const double v = eval_candidate_wave<TI, DP>(a, cq[c], cj[c]);
            if ((threadIdx.x & 63) == 0) a.cand_v[base + c] = v;
        }
    }
}

// One wavefront per listed candidate (the large-grid path, RMSD).
template <typename TI, int DP>
__global__ __launch_bounds__(256) void candidate_eval_kernel(SelectArgs a) {
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6), nw = gridDim.x * 4;
    const int count = min(*a.cand_count, a.cand_cap);
    for (int i = gw; i < count; i += nw) {
        const double v = eval_candidate_wave<TI, DP>(a, a.cand_q[i], a.cand_j[i]);
        if ((threadIdx.x & 63) == 0) a.cand_v[i] = v;
    }
}

// Batch medoid of cluster j among the evaluated candidates, and its member count, by one block.
__device__ void reduce_cluster(const SelectArgs& a, int j, int32_t* members, int32_t* med) {
    const int count = min(*a.cand_count, a.cand_cap);
    double bv = kInf;
    int64_t bi = INT64_MAX;
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        if (a.cand_j[i] == j) vmin(bv, bi, a.cand_v[i], a.cand_q[i]);
    block_vmin(bv, bi);
    __shared__ int32_t sh_c;
    if (threadIdx.x == 0) sh_c = 0;
    __syncthreads();
    int32_t c = 0;
    for (int k = threadIdx.x; k < a.nchunk; k += blockDim.x) c += a.mpart_c[(int64_t)j * a.nchunk + k];
    if (c) atomicAdd(&sh_c, c);
    __syncthreads();
    *members = sh_c;
    // no candidate only when every distance is +inf or NaN (non-finite input, reported separately)
    *med = sh_c == 0 ? -1 : (bi == INT64_MAX ? 0 : (int32_t)bi);
    __syncthreads();
}

__device__ __forceinline__ double merge_alpha(int32_t members, int64_t w) {
    const double den = (double)members + (double)w;
    return den > 0.0 ? (double)members / den : 0.0;
}

// ----------------------------------------------------------------------------- merge (Eq. 11-13)
// Grid (row chunks) x (clusters): score(x) = K(x,x) - 2 alpha K(x, m_j^i) - 2 (1 - alpha) K(x, m_j)
// for the chunk's rows, block minimum (lowest position on ties).  Chunk 0 records m_j^i and |w_j^i|.
template <typename TI, int DP>
__global__ __launch_bounds__(256) void merge_partial_kernel(SelectArgs a) {
    const int j = blockIdx.y, chunk = blockIdx.x;
    int32_t mem = 0, med = -1;
    reduce_cluster(a, j, &mem, &med);
    if (chunk == 0 && threadIdx.x == 0) {
        a.counts[j] = mem;
        a.bmed[j] = med;
    }
    const double alpha = merge_alpha(mem, a.wcount[j]);
    if (!(alpha > 0.0) || med < 0) return;   // uniform over the block
    const int64_t q = (int64_t)chunk * kRowsPerBlock + threadIdx.x;
    double bv = kInf;
    int64_t bi = INT64_MAX;
    if (q < a.b.n) {
        const TI* x = brow<TI>(a.b, q);
        double sc = kself64(a.ks, x) - 2.0 * alpha * k64p<DP>(a.ks, x, brow<TI>(a.b, med));
        if (alpha < 1.0)
            sc = sc - 2.0 * (1.0 - alpha) * k64p<DP>(a.ks, x, static_cast<const TI*>(a.M) + (int64_t)j * a.Mpad);
        bv = sc;
        bi = q;
    }
    block_vmin(bv, bi);
    if (threadIdx.x == 0) {
        const int64_t at = (int64_t)j * a.mchunk + chunk;
        a.gpart_v[at] = bv;
        a.gpart_i[at] = bi == INT64_MAX ? -1 : (int32_t)bi;
    }
}

// Linear / RBF kernels.  Block = kMergeRows batch rows x kMergeTJ clusters (two targets each).  The
// block first settles its clusters: the batch medoid m_j^i is the lowest (value, position) candidate
// (two exact LDS minimum passes: the ordered value, then the position among the candidates holding
// it), |w_j^i| the sum of the member-count partials, and alpha_j; the blocks of row chunk 0 record
// them.  Wave w then scores the targets (m_j^i and m_j) of clusters 4w..4w+3 against all kMergeRows
// rows, one row per lane, so that every target value read from LDS (a broadcast) feeds a row and
// every row value feeds eight targets.  Rows are staged
// through LDS dimension-major in chunks of 16 dimensions (coalesced global reads).  Scores follow
// the per-row merge formula in FP64 (explicit differences for RBF); the (value, position) minimum
// of each cluster over the block's rows goes to gpart (kMergeRows-row chunks: merge_chunks).
constexpr int kMergeTJ = 16;
constexpr int kMergeRows = 64;
constexpr int kMergeXs = kMergeRows + 4;   // LDS row stride of the staged chunk

// Settles clusters j0 .. j0 + kMergeTJ - 1 into LDS (all threads of the block): batch medoid cmed
// (-1 when empty), alpha calpha (0 when the cluster takes no merge step); record: also writes
// counts[j] and bmed[j].
__device__ void merge_settle(const SelectArgs& a, int j0, bool record, unsigned long long* cmin, int32_t* cpos,
                             int32_t* cmem, int32_t* cmed, double* calpha) {
    if (threadIdx.x < kMergeTJ) {
        cmin[threadIdx.x] = ~0ull;
        cpos[threadIdx.x] = INT32_MAX;
        cmem[threadIdx.x] = 0;
    }
    // member counts: the 16 threads of cluster jj = t / 16 sum its chunk partials k = t % 16, t % 16
    // + 16, ... (integers: exact in any order), then across the 16 threads.  The first eight
    // partials of each thread and the thread's own entry of the candidate list are requested before
    // the candidate count is known (the entry is masked by the count afterwards), so that the reads
    // overlap; the entry stays in registers for the second pass.
    static_assert(kMergeTJ * 16 == 256, "16 threads per cluster");
    constexpr int MU = 8;
    const int mjj = (int)threadIdx.x >> 4, msub = (int)threadIdx.x & 15;
    const bool mon = j0 + mjj < a.C;
    const int32_t* mp = a.mpart_c + (int64_t)min(j0 + mjj, a.C - 1) * a.nchunk;
    int32_t cpart[MU];
#pragma unroll
    for (int u = 0; u < MU; ++u) cpart[u] = mp[min(msub + 16 * u, a.nchunk - 1)];
    const int i0 = threadIdx.x, ic = min(i0, a.cand_cap - 1);
    const int32_t cj0 = a.cand_j[ic], cq0 = a.cand_q[ic];
    const double cv0 = a.cand_v[ic];
    const int64_t wc0 = a.wcount[min(j0 + (int)threadIdx.x, a.C - 1)];   // (|w_j| of thread t < 16's cluster)
    __syncthreads();
    const int count = min(*a.cand_count, a.cand_cap);
    auto note_min = [&](int32_t cj, double v) {
        const int jj = cj - j0;
        if (jj >= 0 && jj < kMergeTJ && !isnan(v)) atomicMin(&cmin[jj], ord_enc(v + 0.0));   // -0 counts as +0
    };
    if (i0 < count) note_min(cj0, cv0);
    for (int i = i0 + (int)blockDim.x; i < count; i += blockDim.x) note_min(a.cand_j[i], a.cand_v[i]);
    int32_t msum = 0;
#pragma unroll
    for (int u = 0; u < MU; ++u) msum += (mon && msub + 16 * u < a.nchunk) ? cpart[u] : 0;
    for (int k0 = msub + 16 * MU; k0 < a.nchunk; k0 += 16 * MU) {
#pragma unroll
        for (int u = 0; u < MU; ++u) cpart[u] = mp[min(k0 + 16 * u, a.nchunk - 1)];
#pragma unroll
        for (int u = 0; u < MU; ++u) msum += (mon && k0 + 16 * u < a.nchunk) ? cpart[u] : 0;
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) msum += __shfl_xor(msum, o, 64);
    if (msub == 0) cmem[mjj] = msum;
    __syncthreads();
    auto note_pos = [&](int32_t cj, double v, int32_t q) {
        const int jj = cj - j0;
        if (jj >= 0 && jj < kMergeTJ && !isnan(v) && ord_enc(v + 0.0) == cmin[jj]) atomicMin(&cpos[jj], q);
    };
    if (i0 < count) note_pos(cj0, cv0, cq0);
    for (int i = i0 + (int)blockDim.x; i < count; i += blockDim.x) note_pos(a.cand_j[i], a.cand_v[i], a.cand_q[i]);
    __syncthreads();
    if (threadIdx.x < kMergeTJ && j0 + (int)threadIdx.x < a.C) {
        const int j = j0 + threadIdx.x;
        const int32_t mem = cmem[threadIdx.x];
        // no candidate only when every distance is +inf or NaN (non-finite input, reported separately)
        const int32_t med = mem == 0 ? -1 : (cpos[threadIdx.x] == INT32_MAX ? 0 : cpos[threadIdx.x]);
        const double alpha = merge_alpha(mem, wc0);
        const bool on = alpha > 0.0 && med >= 0;
        cmed[threadIdx.x] = med;
        calpha[threadIdx.x] = on ? alpha : 0.0;
        if (record) {
            a.counts[j] = mem;
            a.bmed[j] = med;
        }
    } else if (threadIdx.x < kMergeTJ) {   // past the last cluster: no medoid, no merge step
        cmed[threadIdx.x] = -1;
        calpha[threadIdx.x] = 0.0;
    }
    __syncthreads();
}

// Large merge grids: the clusters are settled once, a block per kMergeTJ clusters, instead of by
// every row chunk (whose repeated reads of the candidate list would dominate the merge).  With
// TARGETS (linear / RBF: the matrix-core merge) the block also writes its clusters' targets -- target
// 2 jj the batch medoid m_j^i, 2 jj + 1 the global medoid m_j, zero when the merge does not use it --
// in FP64 to tpan[j][2][Mpad], and their squared norms (summed in order) to tnorm[j][2].

template <typename TI, int DP, bool TARGETS>
__global__ __launch_bounds__(256) void merge_settle_kernel(SelectArgs a) {
    __shared__ unsigned long long cmin[kMergeTJ];
    __shared__ int32_t cpos[kMergeTJ], cmem[kMergeTJ], cmed[kMergeTJ];
    __shared__ double calpha[kMergeTJ];
    const int j0 = blockIdx.x * kMergeTJ;
    merge_settle(a, j0, true, cmin, cpos, cmem, cmed, calpha);
    if constexpr (TARGETS && DP > 0) {
        // value p of the block is dimension k = p % DP of target tt = p / DP; the loads are issued
        // together (clamped, masked afterwards), the panel written from registers, and the norms
        // summed over eight strided parts, then the parts in order
        constexpr int NT = 2 * kMergeTJ, TPER = (DP * NT + 255) / 256;
        __shared__ double part[8][NT];
        // the targets' rows as element offsets from X (m_j^i) or M (m_j), -1 when the target is not
        // used (offsets rather than pointers: a pointer read back from LDS makes flat loads)
        __shared__ int64_t toff[NT];
        const int d = a.b.d, t = threadIdx.x;
        const int last = min(2 * a.C - 2 * j0, NT) - 1;
        if (t < NT) {
            const int tt = min(t, last), jj = tt / 2, j = j0 + jj;
            const bool med = (tt & 1) == 0;
            const double alpha = calpha[jj];
            const bool on = med ? alpha > 0.0 : (alpha > 0.0 && alpha < 1.0);
            toff[t] = !on ? -1 : med ? (a.b.base + (int64_t)max(cmed[jj], 0) * a.b.stride) * a.b.d : (int64_t)j * a.Mpad;
        }
        __syncthreads();
        const TI* Xb = static_cast<const TI*>(a.b.X);
        const TI* Mb = static_cast<const TI*>(a.M);
        double tv[TPER];
#pragma unroll
        for (int u = 0; u < TPER; ++u) {
            const int p = min(t + 256 * u, DP * NT - 1), tt = min(p / DP, last), k = p % DP;
            const int64_t o = toff[tt];
            const TI* src = ((tt & 1) == 0 ? Xb : Mb) + (o < 0 ? 0 : o);
            tv[u] = o >= 0 && k < d ? (double)src[min(k, d - 1)] : 0.0;
        }
        // (value u of thread t is dimension t % DP of target t / DP + u * (256 / DP) when the block
        // covers 256 values at a time: the panel address steps by a uniform amount)
        double* tp = a.tpan + ((int64_t)j0 * 2) * a.Mpad;
#pragma unroll
        for (int u = 0; u < TPER; ++u) {
            const int p = t + 256 * u, tt = p / DP, k = p % DP;
            if constexpr (DP * NT >= 256) {
                if (tt <= last) tp[(t / DP) * a.Mpad + k] = tv[u];
                tp += (256 / DP) * a.Mpad;
            } else {
                if (p < DP * NT && tt <= last) a.tpan[((int64_t)j0 * 2 + tt) * a.Mpad + k] = tv[u];
            }
        }
        __shared__ double tl[NT][DP + 1];
#pragma unroll
        for (int u = 0; u < TPER; ++u) {
            const int p = t + 256 * u;
            if (p < DP * NT) tl[p / DP][p % DP] = tv[u];
        }
        __syncthreads();
        {
            const int tt = t & (NT - 1), pt = t / NT;   // eight parts of 32 targets
            double s2 = 0.0;
            for (int k = pt; k < DP; k += 8) s2 = fma(tl[tt][k], tl[tt][k], s2);
            part[pt][tt] = s2;
        }
        __syncthreads();
        if (t < NT && t <= last) {
            double v = 0.0;
            for (int q = 0; q < 8; ++q) v += part[q][t];
            a.tnorm[(int64_t)j0 * 2 + t] = v;
        }
    }
}

// SETTLED: the clusters were settled by merge_settle_kernel (read back from counts / bmed).
template <typename TI, int DP, bool SETTLED>
__global__ __launch_bounds__(256) void merge_tile_kernel(SelectArgs a) {
    constexpr int NT = 2 * kMergeTJ;
    constexpr int CH = DP < 16 ? DP : 16;
    __shared__ double Ts[DP][NT];
    __shared__ TI Xs[CH][kMergeXs];
    __shared__ unsigned long long cmin[kMergeTJ];
    __shared__ int32_t cpos[kMergeTJ], cmem[kMergeTJ], cmed[kMergeTJ];
    __shared__ double calpha[kMergeTJ];
    const int j0 = blockIdx.y * kMergeTJ, chunk = blockIdx.x;
    const int d = a.b.d;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row0 = (int64_t)chunk * kMergeRows;
    const int nrows = (int)min<int64_t>(kMergeRows, a.b.n - row0);
    // Staging of the block's rows, CH dimensions at a time: element u of a thread is (row p / CH,
    // dimension p % CH) for p = threadIdx.x + 256 u.  Every load is issued unconditionally (row and
    // dimension clamped into range, the value scaled by a 0 / 1 mask, which keeps every bit of the
    // values inside the tile), so a stage's loads are in flight together; the first stage's loads
    // are issued before the clusters are settled.
    constexpr int XPER = kMergeRows * CH / 256;
    static_assert(XPER * 256 == kMergeRows * CH, "staging covers the chunk exactly");
    auto stage_load = [&](int k0, TI (&v)[XPER]) {
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int p = threadIdx.x + 256 * u;
            const int r = p / CH, k = p - r * CH;
            const TI x = brow<TI>(a.b, row0 + min(r, nrows - 1))[min(k0 + k, d - 1)];
            v[u] = x * ((r < nrows && k0 + k < d) ? TI(1) : TI(0));
        }
    };
    TI xst[XPER];
    stage_load(0, xst);
    if constexpr (SETTLED) {
        if (threadIdx.x < kMergeTJ && j0 + (int)threadIdx.x < a.C) {
            const int j = j0 + threadIdx.x;
            const int32_t med = a.bmed[j];
            const double alpha = merge_alpha(a.counts[j], a.wcount[j]);
            cmed[threadIdx.x] = med;
            calpha[threadIdx.x] = alpha > 0.0 && med >= 0 ? alpha : 0.0;
        } else if (threadIdx.x < kMergeTJ) {   // past the last cluster: no medoid, no merge step
            cmed[threadIdx.x] = -1;
            calpha[threadIdx.x] = 0.0;
        }
        __syncthreads();
    } else {
        // settle the block's clusters (the same result as one block reducing each cluster)
        merge_settle(a, j0, chunk == 0, cmin, cpos, cmem, cmed, calpha);
    }
    // targets, dimension-major: t = 2 (j - j0) is m_j^i, t + 1 is m_j (zero when unused); every
    // load issued unconditionally (cluster, row and dimension clamped, the value masked), so the
    // thread's loads are in flight together
    constexpr int TPER = (DP * NT + 255) / 256;
    double tx[TPER];
#pragma unroll
    for (int u = 0; u < TPER; ++u) {
        const int pc = min((int)threadIdx.x + 256 * u, DP * NT - 1);
        const int k = pc / NT, t = pc - k * NT;
        const int jj = t / 2, j = min(j0 + jj, a.C - 1);
        const double alpha = calpha[jj];
        const bool med = (t & 1) == 0;
        // (a cluster past the last one, or without a medoid, reads row 0: a valid address, masked)
        const int mrow = j0 + jj < a.C ? max(cmed[jj], 0) : 0;
        const TI* src = med ? brow<TI>(a.b, mrow) : static_cast<const TI*>(a.M) + (int64_t)j * a.Mpad;
        const bool on = j0 + jj < a.C && k < d && (med ? alpha > 0.0 : (alpha > 0.0 && alpha < 1.0));
        tx[u] = (double)src[min(k, d - 1)] * (on ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < TPER; ++u) {
        const int p = threadIdx.x + 256 * u;
        if (p < DP * NT) Ts[p / NT][p - (p / NT) * NT] = tx[u];
    }
    const bool lin = a.ks.type == KKM_KERNEL_LINEAR;
    double acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = 0.0;
    double xx = 0.0;
#pragma unroll 1
    for (int k0 = 0; k0 < DP; k0 += CH) {
        if (k0 > 0) stage_load(k0, xst);
        __syncthreads();   // previous chunk consumed (and Ts written, on the first pass)
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int p = threadIdx.x + 256 * u;
            Xs[p - (p / CH) * CH][p / CH] = xst[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < CH; ++k) {
            const double xv = (double)Xs[k][lane];
            const double* tk = &Ts[k0 + k][8 * wave];
            double tv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) tv[t] = tk[t];
            if (lin) {
                xx = fma(xv, xv, xx);
#pragma unroll
                for (int t = 0; t < 8; ++t) acc[t] = fma(xv, tv[t], acc[t]);
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const double df = xv - tv[t];
                    acc[t] = fma(df, df, acc[t]);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = j0 + 4 * wave + c;
        if (j >= a.C) break;   // uniform over the wave
        const double alpha = calpha[4 * wave + c];
        double bv = kInf;
        int64_t bi = INT64_MAX;
        if (alpha > 0.0 && lane < nrows) {
            const double k1 = lin ? acc[2 * c] : ::exp(-acc[2 * c] * a.ks.inv2s2);
            double sc = (lin ? xx : 1.0) - 2.0 * alpha * k1;
            if (alpha < 1.0) {
                const double k2 = lin ? acc[2 * c + 1] : ::exp(-acc[2 * c + 1] * a.ks.inv2s2);
                sc = sc - 2.0 * (1.0 - alpha) * k2;
            }
            bv = sc;
            bi = row0 + lane;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double v2 = __shfl_xor(bv, o, 64);
            const int64_t i2 = __shfl_xor(bi, o, 64);
            vmin(bv, bi, v2, i2);
        }
        if (lane == 0) {
            const int64_t at = (int64_t)j * a.mchunk + chunk;
            a.gpart_v[at] = bv;
            a.gpart_i[at] = bi == INT64_MAX ? -1 : (int32_t)bi;
        }
    }
}

// The same merge on the FP64 matrix cores (linear / RBF): the dot products of the block's 64 rows
// with its 32 targets run on v_mfma_f64_16x16x4f64, four dimensions a step (the A operand a target,
// the B operand a row), and each score follows from them in FP64: d(x, t) = ||x||^2 + ||t||^2 - 2 x.t
// (at least 0), K = exp(-d / (2 sigma^2)) for RBF or x.t for the linear kernel.  This is the FP64
// value of the merge formula up to the order of its roundings (a few units of 2^-53 of ||x||^2 +
// ||t||^2 in d), so the argmin is the FP64 one except between candidates equal to that order, and
// no re-evaluation follows.  Wavefront w takes rows 16w .. 16w + 15 of the block and both 16-target
// halves.  The FP64 product leaves output row 4v + l/16 of column l%16 in register v of lane l, so
// A-operand row i carries target 4(i%4) + i/4 of the half: lane l then holds targets 4(l/16) + v
// for row 16w + l%16, i.e. both targets (m_j^i, m_j) of two clusters per half.  Norms are summed in a fixed order (strided parts, then the
// parts in order), so the result does not depend on scheduling.
//
// The grid is one-dimensional, one workgroup per (row chunk, cluster group) tile, numbered chunk-major.
// Consecutive workgroups are dealt to the eight XCDs in turn, so workgroup b takes tile
// (b % 8) * per + b / 8 (per = tiles / 8, rounded up): the cluster groups of one row chunk then run on
// one XCD and read the chunk's rows through one L2.  Targets are staged in LDS at the data's
// precision (they are rows of X), which keeps a workgroup's LDS small enough for five per CU.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename TI, int DP, bool SETTLED>
__global__ __launch_bounds__(256) void merge_mfma_kernel(SelectArgs a) {
    constexpr int NT = 2 * kMergeTJ;                 // 32 targets
    constexpr int XS = kMergeRows + 4;               // LDS row stride of the staged rows
    static_assert(256 % DP == 0, "a thread's staged values share one dimension");
    __shared__ TI Ts[DP][NT + 2];
    __shared__ TI Xs[DP][XS];
    __shared__ double part[4][kMergeRows];
    __shared__ double xn[kMergeRows], tn[NT];
    __shared__ double wv[4][kMergeTJ];
    __shared__ int32_t wi[4][kMergeTJ];
    __shared__ unsigned long long cmin[kMergeTJ];
    __shared__ int32_t cpos[kMergeTJ], cmem[kMergeTJ], cmed[kMergeTJ];
    __shared__ double calpha[kMergeTJ];
    const int ngrp = (a.C + kMergeTJ - 1) / kMergeTJ, ntile = a.mchunk * ngrp;
    const int tile = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;   // (padding of the grid to a multiple of eight)
    const int chunk = tile / ngrp, j0 = (tile - chunk * ngrp) * kMergeTJ;
    const int d = a.b.d;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t row0 = (int64_t)chunk * kMergeRows;
    const int nrows = (int)min<int64_t>(kMergeRows, a.b.n - row0);
    // the block's rows, dimension-major (rows and dimensions past the end: zero).  Every load is issued
    // unconditionally (row and dimension clamped into range, the value masked afterwards), so that
    // all of a thread's loads are in flight together.  Value u of thread t is dimension t % DP of row
    // t / DP + u * (256 / DP): the address steps by a uniform amount (rows past the end read the last
    // row), with no multiplication per load.
    constexpr int XPER = kMergeRows * DP / 256, RPU = 256 / DP;
    static_assert(XPER * 256 == kMergeRows * DP, "row staging covers the block exactly");
    TI xv[XPER];
    {
        const int64_t rs = a.b.stride * a.b.d;   // elements between consecutive batch rows
        const TI* xb = static_cast<const TI*>(a.b.X) + (a.b.base + row0 * a.b.stride) * a.b.d + min(t % DP, d - 1);
        const TI* xlast = xb + (int64_t)(nrows - 1) * rs;
        const TI* xp = xb + (int64_t)(t / DP) * rs;
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            xv[u] = *(t / DP + u * RPU < nrows ? xp : xlast);
            xp += RPU * rs;
        }
    }
    if constexpr (SETTLED) {
        if (t < kMergeTJ && j0 + t < a.C) {
            const int j = j0 + t;
            const int32_t med = a.bmed[j];
            const double alpha = merge_alpha(a.counts[j], a.wcount[j]);
            cmed[t] = med;
            calpha[t] = alpha > 0.0 && med >= 0 ? alpha : 0.0;
        } else if (t < kMergeTJ) {   // past the last cluster: no medoid, no merge step
            cmed[t] = -1;
            calpha[t] = 0.0;
        }
        __syncthreads();
    } else {
        merge_settle(a, j0, chunk == 0, cmin, cpos, cmem, cmed, calpha);
    }
    // targets, dimension-major: target 2 jj is m_j^i, 2 jj + 1 is m_j (zero when unused); with the
    // clusters settled beforehand, read from the settle pass's FP64 panel (coalesced) with their norms
    if constexpr (SETTLED) {
        constexpr int TPER = (DP * NT + 255) / 256;
        const int last = min(2 * a.C - 2 * j0, NT) - 1;   // the block's last target (clusters past C: zero)
        double tv[TPER];
        if constexpr (DP * NT >= 256) {   // value u of thread t: dimension t % DP of target t / DP + u * (256 / DP)
            const double* tb = a.tpan + ((int64_t)j0 * 2) * a.Mpad + t % DP;
            const double* tlast = tb + (int64_t)last * a.Mpad;
            const double* tp = tb + (int64_t)(t / DP) * a.Mpad;
#pragma unroll
            for (int u = 0; u < TPER; ++u) {
                tv[u] = *(t / DP + u * RPU <= last ? tp : tlast);
                tp += RPU * a.Mpad;
            }
        } else {
#pragma unroll
            for (int u = 0; u < TPER; ++u) {
                const int p = min(t + 256 * u, DP * NT - 1), tt = p / DP, k = p - tt * DP;
                tv[u] = a.tpan[((int64_t)j0 * 2 + min(tt, last)) * a.Mpad + k];
            }
        }
#pragma unroll
        for (int u = 0; u < TPER; ++u) {
            const int p = t + 256 * u, tt = p / DP, k = p - tt * DP;
            if (p < DP * NT) Ts[k][tt] = tt <= last ? (TI)tv[u] : TI(0);   // (exact: values of X)
        }
        if (t < NT) tn[t] = t <= last ? a.tnorm[(int64_t)j0 * 2 + t] : 0.0;
    } else {
        for (int p = t; p < DP * NT; p += 256) {
            const int k = p / NT, tt = p - k * NT;
            const int jj = tt / 2, j = min(j0 + jj, a.C - 1);
            const double alpha = calpha[jj];
            const bool med = (tt & 1) == 0;
            const int mrow = j0 + jj < a.C ? max(cmed[jj], 0) : 0;
            const TI* src = med ? brow<TI>(a.b, mrow) : static_cast<const TI*>(a.M) + (int64_t)j * a.Mpad;
            const bool on = j0 + jj < a.C && k < d && (med ? alpha > 0.0 : (alpha > 0.0 && alpha < 1.0));
            Ts[k][tt] = on ? src[k] : TI(0);
        }
    }
#pragma unroll
    for (int u = 0; u < XPER; ++u) {
        const int p = t + 256 * u, r = p / DP, k = p - r * DP;
        Xs[k][r] = (r < nrows && k < d) ? xv[u] : TI(0);
    }
    __syncthreads();
    // squared norms in a fixed order: rows in four parts, (unsettled) targets summed in order
    {
        const int r = t & 63, pr = t >> 6;
        double sx = 0.0;
        for (int k = pr; k < DP; k += 4) {
            const double v = Xs[k][r];
            sx = fma(v, v, sx);
        }
        part[pr][r] = sx;
        if constexpr (!SETTLED) {
            if (t < NT) {
                double st = 0.0;
                for (int k = 0; k < d; ++k) st = fma((double)Ts[k][t], (double)Ts[k][t], st);
                tn[t] = st;
            }
        }
        __syncthreads();
        if (t < kMergeRows) xn[t] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
        __syncthreads();
    }
    // the products: wave w, rows 16w + l%16; target halves h = 0, 1
    doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int q4 = lane >> 4, c16 = lane & 15;
    const int ta = 4 * (c16 & 3) + (c16 >> 2);   // the target of A-operand row c16
    // (fully unrolled: a loop would move the accumulators between register files every iteration)
#pragma unroll
    for (int s = 0; s < DP / 4; ++s) {
        const int k = 4 * s + q4;
        const double xv = (double)Xs[k][16 * wave + c16];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Ts[k][ta], xv, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Ts[k][16 + ta], xv, acc1, 0, 0, 0);
    }
    // scores of the lane's four clusters for its row, then the wavefront's minimum per cluster over
    // its 16 rows (lanes of one quarter): the minimum value by a butterfly, then the lowest row
    // holding it from a ballot of the lanes equal to it
    const bool lin = a.ks.type == KKM_KERNEL_LINEAR;
    const int r = 16 * wave + c16;
    const double xx = xn[r];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const doublex4 acc = h == 0 ? acc0 : acc1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int jj = 8 * h + 2 * q4 + c;              // cluster of targets 2jj, 2jj + 1
            const int t1 = 2 * jj;
            const double alpha = calpha[jj];
            double bv = kInf;
            if (alpha > 0.0 && r < nrows) {
                double k1, k2 = 0.0;
                if (lin) {
                    k1 = acc[2 * c];
                    k2 = acc[2 * c + 1];
                } else {
                    k1 = ::exp(-fmax(xx + tn[t1] - 2.0 * acc[2 * c], 0.0) * a.ks.inv2s2);
                    if (alpha < 1.0) k2 = ::exp(-fmax(xx + tn[t1 + 1] - 2.0 * acc[2 * c + 1], 0.0) * a.ks.inv2s2);
                }
                double sc = (lin ? xx : 1.0) - 2.0 * alpha * k1;
                if (alpha < 1.0) sc = sc - 2.0 * (1.0 - alpha) * k2;
                bv = sc;
            }
            double mv = bv;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) mv = fmin(mv, __shfl_xor(mv, o, 64));
            // (a NaN score never equals the minimum; a quarter without finite scores has no row)
            const uint32_t eq = (uint32_t)(__ballot(bv == mv && mv < kInf) >> (16 * q4)) & 0xffffu;
            const int32_t bi = eq ? 16 * wave + __builtin_ctz(eq) : INT32_MAX;
            bv = mv;
            if (c16 == 0) {
                wv[wave][jj] = bv;
                wi[wave][jj] = bi;
            }
        }
    }
    __syncthreads();
    // the block's minimum per cluster over the four wavefronts (rows ascending)
    if (t < kMergeTJ && j0 + t < a.C) {
        double bv = wv[0][t];
        int32_t bi = wi[0][t];
        for (int w = 1; w < 4; ++w)
            if (wv[w][t] < bv || (wv[w][t] == bv && wi[w][t] < bi)) {
                bv = wv[w][t];
                bi = wi[w][t];
            }
        const int64_t at = (int64_t)(j0 + t) * a.mchunk + chunk;
        a.gpart_v[at] = bv;
        a.gpart_i[at] = bi == INT32_MAX ? -1 : (int32_t)(row0 + bi);
    }
}

// One wavefront per cluster: the merged medoid is the lowest (score, position) over the chunk
// partials; |w_j| += |w_j^i|; per-batch info rows.
template <typename TI>
__global__ __launch_bounds__(64) void merge_final_kernel(SelectArgs a) {
    const int j = blockIdx.x, lane = threadIdx.x;
    if (j == 0 && lane == 0 && a.cand_total) *a.cand_total += *a.cand_count;
    // the chunk partials, eight per lane at a time, every index and value requested before any is
    // used -- the first eight together with the cluster's counts (clamped, masked by selects: an
    // absent partial is (+inf, INT64_MAX), which never wins)
    constexpr int PU = 8;
    int32_t ii[PU];
    double vv[PU];
    auto load8 = [&](int c0) {
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int64_t at = (int64_t)j * a.mchunk + min(c0 + 64 * u, a.mchunk - 1);
            ii[u] = a.gpart_i[at];
            vv[u] = a.gpart_v[at];
        }
    };
    const int32_t mem = a.counts[j], med = a.bmed[j];
    const int64_t wc = a.wcount[j];
    load8(lane);
    // (all of them issued here, before any is waited for, rather than the partials after the test)
#pragma unroll
    for (int u = 0; u < PU; ++u) asm volatile("" :: "v"(ii[u]), "v"(vv[u]), "v"(mem), "v"(med), "v"(wc));
    const double alpha = merge_alpha(mem, wc);
    if (alpha > 0.0 && med >= 0) {
        double bv = kInf;
        int64_t bi = INT64_MAX;
        for (int c0 = lane; c0 < a.mchunk; c0 += 64 * PU) {
            if (c0 != lane) load8(c0);
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const bool ok = c0 + 64 * u < a.mchunk && ii[u] >= 0;
                vmin(bv, bi, ok ? vv[u] : kInf, ok ? (int64_t)ii[u] : INT64_MAX);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double v2 = __shfl_xor(bv, o, 64);
            const int64_t i2 = __shfl_xor(bi, o, 64);
            vmin(bv, bi, v2, i2);
        }
        if (bi == INT64_MAX) bi = med;
        const TI* x = brow<TI>(a.b, bi);
        TI* M = static_cast<TI*>(a.M) + (int64_t)j * a.Mpad;
        if (a.info_disp && lane == 0) {   // (reads the old medoid row before the copy below replaces it)
            const double koo = a.Mself[j];
            double dsp = __builtin_nan("");
            if (koo < kInf) {
                const double v = kself64(a.ks, x) - 2.0 * k64(a.ks, x, M) + koo;
                dsp = sqrt(v > 0.0 ? v : 0.0);
            }
            a.info_disp[j] = dsp;
        }
        for (int64_t c = lane; c < a.Mpad; c += 64) M[c] = c < a.b.d ? x[c] : TI(0);
        if (lane == 0) {
            a.Mself[j] = kself64(a.ks, x);
            a.Midx[j] = a.b.base + bi * a.b.stride;
        }
    } else if (a.info_disp && lane == 0) {   // m_j kept
        a.info_disp[j] = a.Mself[j] < kInf ? 0.0 : __builtin_nan("");
    }
    if (lane == 0) {
        a.wcount[j] += mem;
        if (a.info_bmed) a.info_bmed[j] = med >= 0 ? a.b.base + (int64_t)med * a.b.stride : -1;
        if (a.info_bcnt) a.info_bcnt[j] = mem;
        if (a.info_gmed) a.info_gmed[j] = a.Mself[j] < kInf ? a.Midx[j] : -1;
    }
}

// ----------------------------------------------------------------------------- models
template <typename TI>
__global__ __launch_bounds__(1024) void model_from_medoids_kernel(kkm_model m, const TI* M, int64_t Mpad,
                                                                  const double* Mself, const int64_t* Midx,
                                                                  const int64_t* wcount, KSpec ks) {
    __shared__ float red[1024];
    float mx = 0.0f;
    TI* S = static_cast<TI*>(m.support);
    for (int j = threadIdx.x; j < m.C; j += blockDim.x) {
        const TI* src = M + (int64_t)j * Mpad;
        TI* dst = S + (int64_t)j * m.dpad;
        double n64 = 0.0;
        float n32 = 0.0f;
        const bool panels = m.kernel.type != KKM_KERNEL_RMSD;   // power-of-two padded rows only
        // 16 elements at a time: their loads are issued unconditionally (index clamped into the row,
        // values past it scaled to zero), then copied, summed in order and split into the panels
        const int64_t rlen = min((int64_t)m.dpad, Mpad);
        for (int64_t c0 = 0; c0 < m.dpad; c0 += 16) {
            TI v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t c = c0 + u;
                v[u] = src[min(c, rlen - 1)] * (c < rlen ? TI(1) : TI(0));
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = (int)(c0 + u);
                if (c >= m.dpad) break;
                dst[c] = v[u];
                n64 = fma((double)v[u], (double)v[u], n64);
                n32 = fmaf((float)v[u], (float)v[u], n32);
                if (panels && m.pan) m.pan[panel32_index(j, c, m.dpad)] = c < m.d ? (float)v[u] : 0.0f;
                if (!panels && m.pan && m.kernel.n_atoms % 2 == 0 && c < m.d)
                    m.pan[rmsd_panel_index(j, c / 3, c % 3, m.kernel.n_atoms / 2)] = (float)v[u];
                if (panels && m.dpad >= 16) {
                    uint16_t hi = 0, lo = 0;
                    if (c < m.d) bf16_split((float)v[u], hi, lo);
                    m.hi[panel16_index(j, c, m.dpad)] = hi;
                    m.lo[panel16_index(j, c, m.dpad)] = lo;
                }
            }
        }
        m.snorm64[j] = n64;
        m.snorm32[j] = n32;
        m.coef64[j] = 1.0;
        m.coef32[j] = 1.0f;
        m.offsets[j] = j;
        m.self[j] = Mself[j];
        m.segabs[j] = 1.0;
        m.counts[j] = wcount[j];
        m.medoid_index[j] = Mself[j] < kInf ? Midx[j] : -1;
        mx = fmaxf(mx, n32);
    }
    if (threadIdx.x == 0) m.offsets[m.C] = m.C;
    if (threadIdx.x < 5) m.split[threadIdx.x] = threadIdx.x == 4 ? m.C : (m.C * threadIdx.x + 3) / 4;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *m.snorm_max = red[0];
    (void)ks;
}

// norms of every support row and the maximum (single block)
template <typename TI>
__global__ __launch_bounds__(1024) void model_norms_kernel(kkm_model m) {
    __shared__ float red[1024];
    float mx = 0.0f;
    const TI* S = static_cast<const TI*>(m.support);
    for (int64_t l = threadIdx.x; l < m.used; l += blockDim.x) {
        double n64 = 0.0;
        float n32 = 0.0f;
        for (int64_t c = 0; c < m.d; ++c) {
            const TI v = S[l * m.dpad + c];
            n64 = fma((double)v, (double)v, n64);
            n32 = fmaf((float)v, (float)v, n32);
        }
        m.snorm64[l] = n64;
        m.snorm32[l] = n32;
        m.coef32[l] = (float)m.coef64[l];
        if (m.pan && m.kernel.type != KKM_KERNEL_RMSD)
            for (int c = 0; c < m.dpad; ++c) m.pan[panel32_index(l, c, m.dpad)] = c < m.d ? (float)S[l * m.dpad + c] : 0.0f;
        if (m.pan && m.kernel.type == KKM_KERNEL_RMSD && m.kernel.n_atoms % 2 == 0)
            for (int c = 0; c < m.d; ++c) m.pan[rmsd_panel_index(l, c / 3, c % 3, m.kernel.n_atoms / 2)] = (float)S[l * m.dpad + c];
        if (m.dpad >= 16 && m.kernel.type != KKM_KERNEL_RMSD)
            for (int c = 0; c < m.dpad; ++c) {
                uint16_t hi = 0, lo = 0;
                if (c < m.d) bf16_split((float)S[l * m.dpad + c], hi, lo);
                m.hi[panel16_index(l, c, m.dpad)] = hi;
                m.lo[panel16_index(l, c, m.dpad)] = lo;
            }
        mx = fmaxf(mx, n32);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *m.snorm_max = red[0];
    if (threadIdx.x < 5) {
        const int t = threadIdx.x;
        int j = 0;
        if (t == 4) j = m.C;
        else if (t > 0) {
            const int64_t target = (m.used * t + 3) / 4;
            while (j < m.C && m.offsets[j] < target) ++j;
        }
        m.split[t] = j;
    }
}

// self term a^T K_SS a of segment j (one block per cluster), fixed summation order
template <typename TI>
__global__ __launch_bounds__(256) void model_self_kernel(kkm_model m, KSpec ks) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const int lo = m.offsets[j], hi = m.offsets[j + 1];
    const int64_t len = hi - lo;
    const TI* S = static_cast<const TI*>(m.support);
    double s = 0.0, sa = 0.0;
    for (int64_t p = threadIdx.x; p < len * len; p += blockDim.x) {
        const int64_t r = lo + p / len, c = lo + p % len;
        s += m.coef64[r] * m.coef64[c] * k64(ks, S + r * m.dpad, S + c * m.dpad);
    }
    for (int64_t p = threadIdx.x; p < len; p += blockDim.x) sa += fabs(m.coef64[lo + p]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) m.self[j] = len > 0 ? red[0] : kInf;
    __syncthreads();
    red[threadIdx.x] = sa;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) m.segabs[j] = red[0];
}

// One wavefront per frame (four per workgroup, grid-stride): lane l reads elements l, l + 64, ...
// of the frame's 3A coordinates (coalesced), whose axis is (l + k) mod 3 at step k since 64 = 1
// mod 3; the three sums are reduced by a fixed butterfly, and the centred frame is written from a
// second, cached read.
template <typename TI>
__global__ __launch_bounds__(256) void centre_kernel(const TI* __restrict__ X, TI* __restrict__ Y, int64_t n, int A) {
    const int lane = threadIdx.x & 63;
    const int64_t D = 3 * (int64_t)A;
    for (int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); f < n; f += (int64_t)gridDim.x * 4) {
        const TI* x = X + f * D;
        TI* y = Y + f * D;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        int axis = lane % 3;
        for (int64_t e = lane; e < D; e += 64) {
            const double v = (double)x[e];
            sx += axis == 0 ? v : 0.0;
            sy += axis == 1 ? v : 0.0;
            sz += axis == 2 ? v : 0.0;
            axis = axis == 2 ? 0 : axis + 1;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            sx += __shfl_xor(sx, o, 64);
            sy += __shfl_xor(sy, o, 64);
            sz += __shfl_xor(sz, o, 64);
        }
        const double cx = sx / A, cy = sy / A, cz = sz / A;
        axis = lane % 3;
        for (int64_t e = lane; e < D; e += 64) {
            const double c = axis == 0 ? cx : (axis == 1 ? cy : cz);
            y[e] = (TI)((double)x[e] - c);
            axis = axis == 2 ? 0 : axis + 1;
        }
    }
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}


}  // namespace

kkm_status launch_kmeanspp(const BatchView& b, int dtype, const KSpec& ks, int C, const double* uniforms,
                           int32_t* chosen, double* D2, double* part, int32_t* error, const DeviceInfo& dev,
                           hipStream_t s, bool cooperative) {
    if (b.n <= 0) return fail(KKM_ERR_INVALID_ARG, "k-means++ on an empty batch");
    // workgroups: at least KKM_KPP_WGS (default 128) when the rows allow, more when that lets every
    // workgroup keep its rows in LDS; at most kKppMaxGrid and the CUs
    static const int want = [] {
        const char* e = std::getenv("KKM_KPP_WGS");
        const int v = e ? std::atoi(e) : 0;
        return v > 0 ? std::min(v, kKppMaxGrid) : 128;
    }();
    const int dp = eval_dp(ks.type, ks.d);
    const size_t es = dtype == KKM_F64 ? 8 : 4;
    const int gmax = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kKppMaxGrid, (int64_t)dev.num_cus, b.n}));
    int G = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)want, std::min<int64_t>(gmax, (b.n + 255) / 256)));
    auto lds_for = [&](int g) {
        const int64_t R = (b.n + g - 1) / g;
        return ((es * (size_t)(R + 1) * (dp + 1) + 15) & ~size_t(15)) + 8 * (size_t)R;
    };
    bool lds_rows = false;
    if (dp > 0) {
        for (int g = G; g <= gmax; g = g < gmax ? std::min(gmax, g + std::max(1, g / 8)) : gmax + 1)
            if (lds_for(g) + 4096 <= dev.max_lds_per_block) {
                G = g;
                lds_rows = true;
                break;
            }
    }
    const size_t lds = lds_rows ? lds_for(G) : 0;
    KppArgs a{b, ks, C, uniforms, chosen, D2, part, error, lds_rows ? 1 : 0};
    // (the sums' buffers and the picks start empty: -1)
    KKM_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(part), 3 * (int64_t)G, 0xBFF0000000000000ull, s));
    KKM_TRY(launch_fill_i32(chosen, C, -1, s));
    return dispatch_dp(dp, [&]<int DP>() -> kkm_status {
        const void* fn = dtype == KKM_F64 ? reinterpret_cast<const void*>(&kmeanspp_kernel<double, DP>)
                                          : reinterpret_cast<const void*>(&kmeanspp_kernel<float, DP>);
        KKM_TRY(allow_dynamic_lds(fn, lds));
        int per_cu = 0;
        KKM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds));
        if (per_cu * dev.num_cus < G) return fail(KKM_ERR_DEVICE, "k-means++ grid does not fit co-resident");
        void* params[] = {&a};
        if (cooperative) KKM_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(256), params, lds, s));
        else KKM_HIP(hipLaunchKernel(fn, dim3(G), dim3(256), params, lds, s));
        return KKM_OK;
    });
}

kkm_status launch_set_medoids(const BatchView& b, int dtype, const KSpec& ks, int C, const int32_t* chosen, void* M,
                              int64_t Mpad, double* Mself, int64_t* Midx, int64_t* wcount, hipStream_t s) {
    if (dtype == KKM_F64)
        hipLaunchKernelGGL(set_medoids_kernel<double>, dim3(nblocks(C, 256)), dim3(256), 0, s, b, ks, C, chosen,
                           static_cast<double*>(M), Mpad, Mself, Midx, wcount);
    else
        hipLaunchKernelGGL(set_medoids_kernel<float>, dim3(nblocks(C, 256)), dim3(256), 0, s, b, ks, C, chosen,
                           static_cast<float*>(M), Mpad, Mself, Midx, wcount);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

// KKM_MERGE_VALU=1 in the environment: the merge scores on the VALU (explicit differences) instead of
// the FP64 matrix cores.
bool merge_on_mfma() {
    static const bool valu = [] {
        const char* e = std::getenv("KKM_MERGE_VALU");
        return e && e[0] == '1';
    }();
    return !valu;
}

int select_chunks(int64_t n) { return (int)std::max<int64_t>(1, (n + kRowsPerBlock - 1) / kRowsPerBlock); }
int merge_chunks(int64_t n) { return (int)std::max<int64_t>(1, (n + kMergeRows - 1) / kMergeRows); }

// The matrix-core merge's one-dimensional grid: its (row chunk, cluster group) tiles, padded to a
// multiple of the eight XCDs.
static unsigned merge_mfma_blocks(int64_t n, int C) {
    const int64_t tiles = (int64_t)merge_chunks(n) * ((C + kMergeTJ - 1) / kMergeTJ);
    return (unsigned)(8 * ((tiles + 7) / 8));
}

kkm_status launch_select(const SelectArgs& a0, bool tile_f64, const DeviceInfo& dev, hipStream_t s) {
    const dim3 grid(a0.nchunk, a0.C);
    SelectArgs a = a0;
    const dim3 tgrid(merge_chunks(a.b.n), (a.C + kMergeTJ - 1) / kMergeTJ);
    // (more than 1024 tile blocks: the merge settles the clusters once first)
    const bool settle_first = (int64_t)tgrid.x * tgrid.y > 1024;
    auto run = [&]<typename TI, int DP>() -> kkm_status {
        a.mchunk = DP == 0 ? a.nchunk : merge_chunks(a.b.n);
        // candidates evaluated by the blocks that find them when the grid is small; otherwise listed
        // for a later pass (the evaluation's registers would halve the large grid's occupancy)
        const bool fused = (int64_t)grid.x * grid.y <= 2048;
        if (fused) {
            if (tile_f64) hipLaunchKernelGGL((medoid_candidates_kernel<double, TI, DP>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((medoid_candidates_kernel<float, TI, DP>), grid, dim3(256), 0, s, a);
        } else {
            // (five clusters a workgroup: with the evaluation's registers, seven workgroups per CU still
            // hold the mixture64 grid of 79 x 20 at once)
            constexpr int JPB = 5;
            const dim3 mgrid(a.nchunk, (a.C + JPB - 1) / JPB);
            if (tile_f64) hipLaunchKernelGGL((medoid_candidates_multi_kernel<double, TI, DP, JPB>), mgrid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((medoid_candidates_multi_kernel<float, TI, DP, JPB>), mgrid, dim3(256), 0, s, a);
            if constexpr (DP == 0) {   // (RMSD candidates: a wavefront each, far fewer workgroups than the scan)
                KKM_HIP(hipGetLastError());
                hipLaunchKernelGGL((candidate_eval_kernel<TI, DP>), dim3((unsigned)std::max(1, dev.num_cus / 2)), dim3(256), 0,
                                   s, a);
            }
        }
        KKM_HIP(hipGetLastError());
        if constexpr (DP == 0) {
            hipLaunchKernelGGL((merge_partial_kernel<TI, DP>), grid, dim3(256), 0, s, a);
        } else {
            if (settle_first) {
                if (merge_on_mfma() && a.tpan && a.tnorm)
                    hipLaunchKernelGGL((merge_settle_kernel<TI, DP, true>), dim3(tgrid.y), dim3(256), 0, s, a);
                else hipLaunchKernelGGL((merge_settle_kernel<TI, DP, false>), dim3(tgrid.y), dim3(256), 0, s, a);
                KKM_HIP(hipGetLastError());
            }
            if (merge_on_mfma() && (!settle_first || (a.tpan && a.tnorm))) {
                const dim3 mgrid(merge_mfma_blocks(a.b.n, a.C));
                if (settle_first) hipLaunchKernelGGL((merge_mfma_kernel<TI, DP, true>), mgrid, dim3(256), 0, s, a);
                else hipLaunchKernelGGL((merge_mfma_kernel<TI, DP, false>), mgrid, dim3(256), 0, s, a);
            } else if (settle_first) {
                hipLaunchKernelGGL((merge_tile_kernel<TI, DP, true>), tgrid, dim3(256), 0, s, a);
            } else {
                hipLaunchKernelGGL((merge_tile_kernel<TI, DP, false>), tgrid, dim3(256), 0, s, a);
            }
        }
        KKM_HIP(hipGetLastError());
        hipLaunchKernelGGL(merge_final_kernel<TI>, dim3(a.C), dim3(64), 0, s, a);
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    };
    return dispatch_dp(eval_dp(a.ks.type, a.ks.d), [&]<int DP>() -> kkm_status {
        if (a.dtype == KKM_F64) return run.template operator()<double, DP>();
        return run.template operator()<float, DP>();
    });
}

kkm_status launch_model_from_medoids(kkm_model* m, const void* M, int64_t Mpad, const double* Mself,
                                     const int64_t* Midx, const int64_t* wcount, hipStream_t s) {
    const KSpec ks{m->kernel.type, m->kernel.n_atoms, m->d, 0.0};
    if (m->dtype == KKM_F64)
        hipLaunchKernelGGL(model_from_medoids_kernel<double>, dim3(1), dim3(1024), 0, s, *m,
                           static_cast<const double*>(M), Mpad, Mself, Midx, wcount, ks);
    else
        hipLaunchKernelGGL(model_from_medoids_kernel<float>, dim3(1), dim3(1024), 0, s, *m,
                           static_cast<const float*>(M), Mpad, Mself, Midx, wcount, ks);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status launch_model_prepare(kkm_model* m, hipStream_t s) {
    const double sg = m->kernel.sigma;
    const KSpec ks{m->kernel.type, m->kernel.n_atoms, m->d, m->kernel.type == KKM_KERNEL_LINEAR ? 0.0 : 1.0 / (2.0 * sg * sg)};
    if (m->dtype == KKM_F64) {
        hipLaunchKernelGGL(model_norms_kernel<double>, dim3(1), dim3(1024), 0, s, *m);
        KKM_HIP(hipGetLastError());
        hipLaunchKernelGGL(model_self_kernel<double>, dim3(m->C), dim3(256), 0, s, *m, ks);
    } else {
        hipLaunchKernelGGL(model_norms_kernel<float>, dim3(1), dim3(1024), 0, s, *m);
        KKM_HIP(hipGetLastError());
        hipLaunchKernelGGL(model_self_kernel<float>, dim3(m->C), dim3(256), 0, s, *m, ks);
    }
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status launch_centre(const void* X, void* Y, int64_t n, int A, int dtype, hipStream_t s) {
    if (n <= 0) return KKM_OK;
    // four frames per workgroup; at most 64K workgroups, each looping over frames
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 3) / 4, 65536);
    if (dtype == KKM_F64)
        hipLaunchKernelGGL(centre_kernel<double>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const double*>(X), static_cast<double*>(Y), n, A);
    else
        hipLaunchKernelGGL(centre_kernel<float>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const float*>(X), static_cast<float*>(Y), n, A);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

__global__ void add_i32_kernel(int32_t* dst, const int32_t* src) {
    if (threadIdx.x == 0) *dst += *src;
}

kkm_status launch_add_i32(int32_t* dst, const int32_t* src, hipStream_t s) {
    hipLaunchKernelGGL(add_i32_kernel, dim3(1), dim3(64), 0, s, dst, src);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

kkm_status launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return KKM_OK;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)std::min<int64_t>(1024, nblocks(n, 256))), dim3(256), 0, s, p, n, v);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return KKM_OK;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)std::min<int64_t>(1024, nblocks(n, 256))), dim3(256), 0, s, p, n, v);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status launch_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return KKM_OK;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)std::min<int64_t>(1024, nblocks(n, 256))), dim3(256), 0, s, p, n);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

}  // namespace kkm
