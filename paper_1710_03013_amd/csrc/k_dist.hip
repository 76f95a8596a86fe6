// Distances from a tile of samples to sparse centroids, and the label decision (Eq. 2, 15, 17):
//
//   d(x, j) = K(x,x) - 2 sum_{l in segment j} a_l K(x, s_l) + a^T K_SS a
//
// Used for the batch-wide pass of a fit (support = the landmarks of the final centroids,
// a_l = 1/c_j, self = g^) and for assigning new samples to a model (support = medoids or any
// sparse centroids).  Work split: a workgroup of four wavefronts owns 64 samples, one per lane;
// each wavefront takes a contiguous run of clusters holding about a quarter of the support rows;
// support rows are read with wave-uniform addresses (scalar loads, broadcast to every lane).
//
// FP32 evaluation carries a per-row bound E on the error of every d(x, j).  A row whose best and
// second-best distances are within 2E is listed and decided again in FP64 (launch_refine), so the
// label equals the exact-arithmetic label wherever the FP64 margin is non-zero.
#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {

namespace {

constexpr float kU32 = 5.9604645e-8f;  // unit roundoff of float

// ----------------------------------------------------------------------------- evaluators
// linear / RBF with the sample row held in registers (DP = padded length)
template <typename TI, typename TC, int DP>
struct EvalDot {
    static constexpr bool kPerLaneRows = false;
    static constexpr bool kStaged = false;
    TC x[DP];
    TC qn, kqq;
    const TI* rows;
    int64_t dpad;
    const float* sn32;
    const double* sn64;
    int type;
    TC inv2s2;
    int64_t d;
    float snmax;
    int nonneg;

    __device__ bool load(const DistArgs& a, int64_t q) {
        const TI* r = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        nonneg = a.sup.nonneg;
        bool ok = true;
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            TI v = k < a.q.d ? r[k] : TI(0);
            ok = ok && isfinite((double)v);
            x[k] = (TC)v;
        }
        qn = TC(0);
#pragma unroll
        for (int k = 0; k < DP; ++k) qn = fma(x[k], x[k], qn);
        type = a.ks.type;
        kqq = type == KKM_KERNEL_LINEAR ? qn : TC(1);
        rows = static_cast<const TI*>(a.sup.rows);
        dpad = a.sup.dpad;
        sn32 = a.sup.snorm32;
        sn64 = a.sup.snorm64;
        inv2s2 = (TC)a.ks.inv2s2;
        d = a.q.d;
        snmax = *a.sup.snorm_max;
        return ok;
    }
    __device__ __forceinline__ TC eval(int l) const {
        const TI* s = rows + (int64_t)l * dpad;
        TC dot = TC(0);
#pragma unroll
        for (int k = 0; k < DP; ++k) dot = fma(x[k], (TC)s[k], dot);
        const TC sn = sizeof(TC) == 8 ? (TC)sn64[l] : (TC)sn32[l];
        return kfun_from_dot(type, dot, qn, sn, inv2s2);
    }
    // bound on |computed - exact| of d(x, j) for a segment of `len` rows (FP32 only)
    __device__ __forceinline__ float bound(int len, float acc, float g, float segabs) const {
        if (sizeof(TC) == 8) return 0.0f;
        const float u = kU32;
        const float q = (float)qn;
        float ef;
        float extra = 0.0f;
        if (type == KKM_KERNEL_LINEAR) {
            const float kmax = sqrtf(q * snmax) * 1.0001f;
            ef = ((float)(d + 2) * u * kmax + (float)(len + 2) * u * kmax) * segabs;
            extra = (float)(d + 2) * u * q;
        } else {
            const float rho = (float)(2 * d + 6) * u * (q + snmax) * (float)inv2s2;
            const float mass = nonneg ? fabsf(acc) * 1.0001f + 1e-30f : segabs;
            ef = (rho + (float)(len + 8) * u) * mass;
        }
        const float e = 2.0f * ef + 3.0f * u * (fabsf((float)kqq) + 2.0f * fabsf(acc) + fabsf(g)) + extra;
        return 2.0f * e;
    }
};

// any kernel type in FP64, rows read from memory (RMSD rows centred)
template <typename TI>
struct EvalGeneric64 {
    static constexpr bool kPerLaneRows = true;
    static constexpr bool kStaged = false;
    const TI* xr;
    const TI* rows;
    int64_t dpad;
    KSpec ks;
    double kqq;

    __device__ bool load(const DistArgs& a, int64_t q) {
        xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        bool ok = true;
        for (int64_t k = 0; k < a.q.d; ++k) ok = ok && isfinite((double)xr[k]);
        ks = a.ks;
        rows = static_cast<const TI*>(a.sup.rows);
        dpad = a.sup.dpad;
        kqq = kself64(ks, xr);
        return ok;
    }
    __device__ __forceinline__ double eval(int l) const { return k64(ks, xr, rows + (int64_t)l * dpad); }
    __device__ __forceinline__ float bound(int, float, float, float) const { return 0.0f; }
};

// RMSD in FP64 with the workgroup's sample rows staged in LDS as TS, coordinate-major ([3A][QT]:
// the lanes reading one coordinate of their samples touch consecutive words), so that an
// evaluation reads only its support row from memory.  The sums are those of the FP64 RMSD kernel
// function, term for term in the same order (staging converts nothing that the reads would not).
template <typename TI, typename TS>
struct EvalRmsd64 {
    static constexpr bool kPerLaneRows = true;
    static constexpr bool kStaged = true;
    const TS* xs;     // the lane's sample: coordinate k at xs[k * qt]
    int qt;
    const TI* rows;
    int64_t dpad;
    int A;
    double inv2s2, Ga, kqq;

    // all threads of the workgroup: rows q0 .. q0 + QT - 1 (the last row repeated past the end)
    __device__ static void stage(const DistArgs& a, TS* st, int QT, int64_t q0) {
        const int D3 = (int)a.q.d;
        const TI* X = static_cast<const TI*>(a.q.X);
        for (int e = threadIdx.x; e < QT * D3; e += blockDim.x) {
            const int sm = e / D3, k = e - sm * D3;
            const int64_t qs = min<int64_t>(q0 + sm, a.q.n - 1);
            st[k * QT + sm] = (TS)X[(a.q.base + qs * a.q.stride) * a.q.d + k];
        }
    }
    __device__ bool load(const DistArgs& a, int64_t q) {
        const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        bool ok = true;
        for (int64_t k = 0; k < a.q.d; ++k) ok = ok && isfinite((double)xr[k]);
        A = a.ks.n_atoms;
        double g = 0.0;
        for (int t = 0; t < A; ++t) {
            const double ax = xr[3 * t], ay = xr[3 * t + 1], az = xr[3 * t + 2];
            g = fma(ax, ax, fma(ay, ay, fma(az, az, g)));
        }
        Ga = g;
        kqq = kself64(a.ks, xr);
        rows = static_cast<const TI*>(a.sup.rows);
        dpad = a.sup.dpad;
        inv2s2 = a.ks.inv2s2;
        return ok;
    }
    __device__ __forceinline__ double eval(int l) const {
        const TI* b = rows + (int64_t)l * dpad;
        double R[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        double Gb = 0.0;
#pragma unroll 8
        for (int t = 0; t < A; ++t) {
            const double ax = xs[(3 * t) * qt], ay = xs[(3 * t + 1) * qt], az = xs[(3 * t + 2) * qt];
            const double bx = b[3 * t], by = b[3 * t + 1], bz = b[3 * t + 2];
            R[0] = fma(ax, bx, R[0]); R[1] = fma(ax, by, R[1]); R[2] = fma(ax, bz, R[2]);
            R[3] = fma(ay, bx, R[3]); R[4] = fma(ay, by, R[4]); R[5] = fma(ay, bz, R[5]);
            R[6] = fma(az, bx, R[6]); R[7] = fma(az, by, R[7]); R[8] = fma(az, bz, R[8]);
            Gb = fma(bx, bx, fma(by, by, fma(bz, bz, Gb)));
        }
        return ::exp(-rmsd2_from_corr64(R, Ga, Gb, A) * inv2s2);
    }
    __device__ __forceinline__ float bound(int, float, float, float) const { return 0.0f; }
};

template <typename T> struct TcOf;
template <typename TI, typename TC, int DP> struct TcOf<EvalDot<TI, TC, DP>> { using type = TC; };
template <typename TI> struct TcOf<EvalGeneric64<TI>> { using type = double; };
template <typename TI, typename TS> struct TcOf<EvalRmsd64<TI, TS>> { using type = double; };

// ----------------------------------------------------------------------------- tile kernel
// LPQ lanes per sample: a workgroup owns QT = 64 / LPQ samples; lane (ql, part) takes the support
// rows l = lo + part, lo + part + LPQ, ... of every segment, and the LPQ partial sums are combined
// by a fixed xor-butterfly, so the result does not depend on timing.
template <class Ev, int LPQ>
__global__ __launch_bounds__(256) void dist_kernel(DistArgs a) {
    using TC = typename TcOf<Ev>::type;
    constexpr int QT = 64 / LPQ;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TC* Dl = reinterpret_cast<TC*>(smem_raw);      // [C][QT]
    __shared__ float Ew[4][QT];
    __shared__ int jb[5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ql = lane % QT, part = lane / QT;
    const int64_t q = (int64_t)blockIdx.x * QT + ql;
    const bool active = q < a.q.n;
    const int C = a.sup.C;
    const int32_t* off = a.sup.offsets;

    if (threadIdx.x < 5) jb[threadIdx.x] = a.sup.split[threadIdx.x];
    Ev ev;
    if constexpr (Ev::kStaged) {   // the tile's rows into LDS after Dl (ordered by the barrier below)
        auto* st = reinterpret_cast<std::remove_const_t<std::remove_pointer_t<decltype(ev.xs)>>*>(
            smem_raw + sizeof(TC) * (size_t)C * QT);
        Ev::stage(a, st, QT, (int64_t)blockIdx.x * QT);
        ev.xs = st + ql;
        ev.qt = QT;
    }
    const bool ok = ev.load(a, active ? q : 0);
    if (active && part == 0 && !ok) atomicOr(a.nonfinite, 1);
    __syncthreads();

    float emax = 0.0f;
    const int j0 = jb[wave], j1 = jb[wave + 1];
    for (int j = j0; j < j1; ++j) {
        const int lo = off[j], hi = off[j + 1];
        TC acc = TC(0);
        for (int l = lo + part; l < hi; l += LPQ) {
            const TC coef = sizeof(TC) == 8 ? (TC)a.sup.coef64[l] : (TC)a.sup.coef32[l];
            acc = fma(coef, ev.eval(l), acc);
        }
        if constexpr (LPQ >= 2) acc += __shfl_xor(acc, QT, 64);
        if constexpr (LPQ >= 4) acc += __shfl_xor(acc, 2 * QT, 64);
        const double g = a.sup.self[j];
        TC D;
        if (hi > lo && g < kInf) {
            D = ev.kqq - TC(2) * acc + (TC)g;
            emax = fmaxf(emax, ev.bound(hi - lo, (float)acc, (float)g, (float)a.sup.segabs[j]));
        } else {
            D = (TC)kInf;
        }
        if (part == 0) Dl[j * QT + ql] = D;
    }
    if (part == 0) Ew[wave][ql] = emax;
    __syncthreads();

    const float E = fmaxf(fmaxf(Ew[0][ql], Ew[1][ql]), fmaxf(Ew[2][ql], Ew[3][ql]));
    bool need = false;   // row listed for the FP64 re-decision
    if (wave == 0 && part == 0 && active) {
        TC best = (TC)kInf, second = (TC)kInf;
        int bj = 0;
        for (int j = 0; j < C; ++j) {
            const TC D = Dl[j * QT + ql];
            if (D < best) { second = best; best = D; bj = j; }
            else if (D < second) { second = D; }
        }
        a.labels[q] = bj;
        if (a.best) a.best[q] = (double)best;
        if (a.Erow) a.Erow[q] = E;
        if (a.gap) {
            const double scale = fmax(fmax(fabs((double)best), fabs((double)second)), fabs((double)ev.kqq));
            a.gap[q] = second < (TC)kInf ? (float)(((double)second - (double)best) / (scale > 0 ? scale : 1.0))
                                         : __builtin_huge_valf();
        }
        const double gap = (double)second - (double)best;
        const double scale = fmax(fmax(fabs((double)best), fabs((double)second)), fabs((double)ev.kqq));
        need = E > 0.0f && gap <= 2.0 * (double)E && gap + 2.0 * (double)E >= kTieMargin * scale;
    }
    if (wave == 0) append_rows(need, q, a.refine_count, a.refine_list);
    if (a.Dt) {
        // store the tile and lower each column's running minimum of D + E (order-independent)
        TC* Dt = static_cast<TC*>(static_cast<void*>(a.Dt));
        for (int j = wave; j < C; j += 4) {
            const TC D = Dl[j * QT + ql];
            if (active && part == 0) Dt[(int64_t)j * a.ldD + q] = D;
            if (a.colmin) {
                double v = (active && part == 0) ? (double)D + (double)E : kInf;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
                if (lane == 0) a.colpart[(int64_t)j * a.colpart_cap + blockIdx.x] = v;
            }
        }
    }
}

// ----------------------------------------------------------------------------- FP64 re-decision
// One wavefront per listed row: lanes evaluate a_l K(x, s_l) in FP64 for 256 support rows at a
// time into LDS, each lane then adds the part of its clusters' segments (in row order), and the
// best / second-best cluster is found by a wave reduction (lowest index on ties).

template <typename TI, int DP>
__global__ __launch_bounds__(256) void refine_kernel(DistArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int C = a.sup.C;
    double* Kv = reinterpret_cast<double*>(smem_raw) + (size_t)wave * (256 + C);   // [256]
    double* facc = Kv + 256;                                                       // [C]
    const int32_t* off = a.sup.offsets;
    const int64_t ns = off[C];
    const TI* rows = static_cast<const TI*>(a.sup.rows);
    const int count = *a.refine_count;
    for (int i = blockIdx.x * 4 + wave; i < count; i += gridDim.x * 4) {
        const int64_t q = a.refine_list[i];
        const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        for (int j = lane; j < C; j += 64) facc[j] = 0.0;
        for (int64_t base = 0; base < ns; base += 256) {
            const int lim = (int)min<int64_t>(256, ns - base);
            for (int t = lane; t < lim; t += 64)
                Kv[t] = a.sup.coef64[base + t] * k64p<DP>(a.ks, xr, rows + (base + t) * a.sup.dpad);
            wave_sync_lds();
            for (int j = lane; j < C; j += 64) {
                const int64_t lo = max<int64_t>(off[j], base), hi = min<int64_t>(off[j + 1], base + lim);
                double s = facc[j];
                for (int64_t l = lo; l < hi; ++l) s += Kv[l - base];
                facc[j] = s;
            }
            wave_sync_lds();
        }
        const double kqq = kself64(a.ks, xr);
        double b1 = kInf, b2 = kInf;
        int i1 = C;
        for (int j = lane; j < C; j += 64) {
            const double g = a.sup.self[j];
            const double D = (off[j + 1] > off[j] && g < kInf) ? kqq - 2.0 * facc[j] + g : kInf;
            if (D < b1) { b2 = b1; b1 = D; i1 = j; }
            else if (D < b2) { b2 = D; }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const double c1 = __shfl_xor(b1, o, 64), c2 = __shfl_xor(b2, o, 64);
            const int j1 = __shfl_xor(i1, o, 64);
            if (c1 < b1 || (c1 == b1 && j1 < i1)) {
                b2 = fmin(b1, c2);
                b1 = c1;
                i1 = j1;
            } else {
                b2 = fmin(b2, c1);
            }
        }
        if (lane == 0) {
            a.labels[q] = i1 < C ? i1 : 0;
            if (a.best) a.best[q] = b1;
            if (a.gap) {
                const double scale = fmax(fmax(fabs(b1), fabs(b2)), fabs(kqq));
                a.gap[q] = b2 < kInf ? (float)((b2 - b1) / (scale > 0 ? scale : 1.0)) : __builtin_huge_valf();
            }
        }
        wave_sync_lds();
    }
}

// A whole block per listed row (supports of hundreds of rows and more): 1024 threads (512 when the
// support and the clusters number at most 512), one support row each per pass of up to kRefineChunk
// rows, so that every row's loads and exponential are in
// flight at once; then per-cluster sums in row order and a reduction of best / second best
// (lowest cluster on ties).  For linear / RBF the listed row is staged once in LDS as doubles,
// zero past d; support rows are read over their padded length DP (the stored row stride) with the
// dimensions past d masked, which adds fma(0, 0, acc) = acc: the same sum as the FP64 evaluation
// elsewhere.
constexpr int kRefineChunk = 2048;
constexpr int kRefineThreads = 1024;

// K(x, s) in FP64 with x as DP doubles in LDS (zero past d) and s a stored support row of DP values.
template <int DP, typename TI>
__device__ __forceinline__ double k64_staged(const KSpec& ks, const double* xs, const TI* __restrict__ s) {
    const int d = (int)ks.d;
    constexpr int CH = DP < 16 ? DP : 16;
    double acc = 0.0;
    if (ks.type == KKM_KERNEL_LINEAR) {
#pragma unroll 1
        for (int c0 = 0; c0 < DP; c0 += CH) {
            double y[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) y[k] = (double)s[c0 + k];
#pragma unroll
            for (int k = 0; k < CH; ++k) acc = fma(xs[c0 + k], c0 + k < d ? y[k] : 0.0, acc);
        }
        return acc;
    }
#pragma unroll 1
    for (int c0 = 0; c0 < DP; c0 += CH) {
        double y[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) y[k] = (double)s[c0 + k];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const double t = c0 + k < d ? xs[c0 + k] - y[k] : 0.0;
            acc = fma(t, t, acc);
        }
    }
    return ::exp(-acc * ks.inv2s2);
}

template <typename TI, int DP>
__global__ __launch_bounds__(kRefineThreads) void refine_block_kernel(DistArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int NW = kRefineThreads / 64;
    const int C = a.sup.C;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double* Kv = reinterpret_cast<double*>(smem_raw);   // [kRefineChunk]
    double* facc = Kv + kRefineChunk;                     // [C]
    __shared__ double xs[DP > 0 ? DP : 1];
    __shared__ double rb1[NW], rb2[NW];
    __shared__ int ri1[NW];
    const int32_t* off = a.sup.offsets;
    const int64_t ns = off[C];
    const TI* rows = static_cast<const TI*>(a.sup.rows);
    const int count = *a.refine_count;
    auto merge = [](double& x1, double& x2, int& y1, double c1, double c2, int j1) {
        if (c1 < x1 || (c1 == x1 && j1 < y1)) {
            x2 = fmin(x1, c2);
            x1 = c1;
            y1 = j1;
        } else {
            x2 = fmin(x2, c1);
        }
    };
    if constexpr (DP > 0 && DP * sizeof(TI) <= 256) {
        // One pass holds the whole support (a support row per thread, a cluster per thread): the
        // thread's support row, its coefficient and its cluster's segment bounds and self term are
        // requested together with the listed row's index, before the listed row itself can be read.
        // The sums are those of the general pass below, term for term.
        if (ns <= (int64_t)blockDim.x && C <= (int)blockDim.x) {
            if ((int)blockIdx.x >= count) return;   // (uniform over the block)
            const bool has = t < ns;
            const int64_t ls = min<int64_t>(t, max<int64_t>(ns - 1, 0));
            const TI* srow = rows + ls * a.sup.dpad;
            const int d = (int)a.ks.d;
            const int jc = min(t, C - 1);
            const int nwc = (C + 63) / 64;   // wavefronts holding clusters
            for (int i = blockIdx.x; i < count; i += gridDim.x) {
                // (the listed row's index first: the wait for it then covers no other load)
                const int64_t q = a.refine_list[i];
                // (only the threads that own a support row load one: the block's loads pass
                // through one CU, whose load bandwidth the whole support already takes)
                TI y[DP];
                if (has) {
#pragma unroll
                    for (int k = 0; k < DP; ++k) y[k] = srow[k];
                } else {
#pragma unroll
                    for (int k = 0; k < DP; ++k) y[k] = TI(0);
                }
                const double cf = a.sup.coef64[ls];
                const int32_t olo = off[jc], ohi = off[jc + 1];
                const double gself = a.sup.self[jc];
                const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
                if (t < DP) xs[t] = t < a.q.d ? (double)xr[t] : 0.0;
                // dimensions past d: zero here and in the staged listed row, so that they add
                // fma(0, 0, acc) = acc, as the masked terms of the general pass do
                if (d < DP) {
#pragma unroll
                    for (int k = 0; k < DP; ++k) y[k] = k < d ? y[k] : TI(0);
                }
                __syncthreads();
                if (has) {
                    // (8 dimensions at a time: the compiler is kept from converting or reading ahead
                    // the next part, so that the FP64 values do not crowd out the support row)
                    constexpr int CH = DP < 8 ? DP : 8;
                    double acc = 0.0;
                    if (a.ks.type == KKM_KERNEL_LINEAR) {
#pragma unroll
                        for (int c0 = 0; c0 < DP; c0 += CH) {
#pragma unroll
                            for (int k = c0; k < c0 + CH; ++k) asm volatile("" : "+v"(y[k]) :: "memory");
#pragma unroll
                            for (int k = c0; k < c0 + CH; ++k) acc = fma(xs[k], (double)y[k], acc);
                        }
                    } else {
#pragma unroll
                        for (int c0 = 0; c0 < DP; c0 += CH) {
#pragma unroll
                            for (int k = c0; k < c0 + CH; ++k) asm volatile("" : "+v"(y[k]) :: "memory");
#pragma unroll
                            for (int k = c0; k < c0 + CH; ++k) {
                                const double df = xs[k] - (double)y[k];
                                acc = fma(df, df, acc);
                            }
                        }
                        acc = ::exp(-acc * a.ks.inv2s2);
                    }
                    Kv[t] = cf * acc;
                }
                __syncthreads();
                if (wave < nwc) {
                    const double kqq = kself64(a.ks, xr);
                    double b1 = kInf, b2 = kInf;
                    int i1 = C;
                    if (t < C) {
                        double sj = 0.0;
                        for (int l = olo; l < ohi; ++l) sj += Kv[l];
                        const double D = (ohi > olo && gself < kInf) ? kqq - 2.0 * sj + gself : kInf;
                        if (D < b1) {
                            b1 = D;
                            i1 = t;
                        }
                    }
                    for (int o = 32; o >= 1; o >>= 1)
                        merge(b1, b2, i1, __shfl_xor(b1, o, 64), __shfl_xor(b2, o, 64), __shfl_xor(i1, o, 64));
                    if (lane == 0) {
                        rb1[wave] = b1;
                        rb2[wave] = b2;
                        ri1[wave] = i1;
                    }
                }
                __syncthreads();
                if (t == 0) {
                    const double kqq = kself64(a.ks, xr);
                    double v1 = rb1[0], v2 = rb2[0];
                    int j1 = ri1[0];
                    for (int w = 1; w < nwc; ++w) merge(v1, v2, j1, rb1[w], rb2[w], ri1[w]);
                    a.labels[q] = j1 < C ? j1 : 0;
                    if (a.best) a.best[q] = v1;
                    if (a.gap) {
                        const double scale = fmax(fmax(fabs(v1), fabs(v2)), fabs(kqq));
                        a.gap[q] = v2 < kInf ? (float)((v2 - v1) / (scale > 0 ? scale : 1.0)) : __builtin_huge_valf();
                    }
                }
                __syncthreads();
            }
            return;
        }
    }
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t q = a.refine_list[i];
        const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        if constexpr (DP > 0) {
            if (t < DP) xs[t] = t < a.q.d ? (double)xr[t] : 0.0;
        }
        for (int j = t; j < C; j += blockDim.x) facc[j] = 0.0;
        for (int64_t base = 0; base < ns; base += kRefineChunk) {
            const int lim = (int)min<int64_t>(kRefineChunk, ns - base);
            __syncthreads();
            for (int l = t; l < lim; l += blockDim.x) {
                const TI* s = rows + (base + l) * a.sup.dpad;
                const double cf = a.sup.coef64[base + l];   // loaded with the row
                double v;
                if constexpr (DP > 0) v = k64_staged<DP>(a.ks, xs, s);
                else v = k64(a.ks, xr, s);
                Kv[l] = cf * v;
            }
            __syncthreads();
            for (int j = t; j < C; j += blockDim.x) {
                const int64_t lo = max<int64_t>(off[j], base), hi = min<int64_t>(off[j + 1], base + lim);
                double sj = facc[j];
#pragma unroll 8
                for (int64_t l = lo; l < hi; ++l) sj += Kv[l - base];
                facc[j] = sj;
            }
        }
        __syncthreads();
        const double kqq = kself64(a.ks, xr);
        double b1 = kInf, b2 = kInf;
        int i1 = C;
        for (int j = t; j < C; j += blockDim.x) {
            const double g = a.sup.self[j];
            const double D = (off[j + 1] > off[j] && g < kInf) ? kqq - 2.0 * facc[j] + g : kInf;
            if (D < b1) { b2 = b1; b1 = D; i1 = j; }
            else if (D < b2) { b2 = D; }
        }
        for (int o = 32; o >= 1; o >>= 1)
            merge(b1, b2, i1, __shfl_xor(b1, o, 64), __shfl_xor(b2, o, 64), __shfl_xor(i1, o, 64));
        if (lane == 0) {
            rb1[wave] = b1;
            rb2[wave] = b2;
            ri1[wave] = i1;
        }
        __syncthreads();
        if (t == 0) {
            double v1 = rb1[0], v2 = rb2[0];
            int j1 = ri1[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) merge(v1, v2, j1, rb1[w], rb2[w], ri1[w]);
            a.labels[q] = j1 < C ? j1 : 0;
            if (a.best) a.best[q] = v1;
            if (a.gap) {
                const double scale = fmax(fmax(fabs(v1), fabs(v2)), fabs(kqq));
                a.gap[q] = v2 < kInf ? (float)((v2 - v1) / (scale > 0 ? scale : 1.0)) : __builtin_huge_valf();
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------- FP64 best distance
// best[q] = K(x,x) - 2 sum_{l in segment u_q} a_l K(x, s_l) + self_{u_q} in FP64 for the label u_q the
// pass (and its re-decisions) settled on: the plain BF16 pass decides labels within its bound, but
// its own distances are too coarse for a cost, so the cost takes this exact value of the chosen
// cluster instead (one segment per row).
template <typename TI, int DP>
__global__ __launch_bounds__(256) void best64_kernel(DistArgs a) {
    const int32_t* off = a.sup.offsets;
    const TI* rows = static_cast<const TI*>(a.sup.rows);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.q.n; q += (int64_t)gridDim.x * blockDim.x) {
        const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + q * a.q.stride) * a.q.d;
        const int j = a.labels[q];
        const int lo = off[j], hi = off[j + 1];
        double f = 0.0;
        for (int l = lo; l < hi; ++l) f = fma(a.sup.coef64[l], k64p<DP>(a.ks, xr, rows + (int64_t)l * a.sup.dpad), f);
        const double g = a.sup.self[j];
        a.best[q] = (hi > lo && g < kInf) ? kself64(a.ks, xr) - 2.0 * f + g : kInf;
    }
}

// ----------------------------------------------------------------------------- deterministic sum
__global__ __launch_bounds__(256) void sum_partial_kernel(const double* __restrict__ v, int64_t n, int64_t chunk,
                                                          double* __restrict__ out) {
    __shared__ double red[256];
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min<int64_t>(n, lo + chunk);
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ----------------------------------------------------------------------------- kernel block
// K[i][j] = kappa(x_i, y_j) in FP64, one work-item per entry (grid-stride), consecutive work-items
// on consecutive j so that the K stores are coalesced.  RMSD rows are centred frames.
template <typename TI>
__global__ __launch_bounds__(256) void kernel_block_kernel(KSpec ks, const TI* __restrict__ X, int64_t nx,
                                                           const TI* __restrict__ Y, int64_t ny,
                                                           double* __restrict__ K) {
    const int64_t total = nx * ny;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ny, j = e - i * ny;
        K[e] = k64(ks, X + i * ks.d, Y + j * ks.d);
    }
}

// One wavefront per cluster: minimum of the workgroup partials of D + E.
template <class Ev, int LPQ>
kkm_status launch_dist_lpq(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    using TC = typename TcOf<Ev>::type;
    constexpr int QT = 64 / LPQ;
    size_t lds = sizeof(TC) * (size_t)a.sup.C * QT;
    if constexpr (Ev::kStaged) lds += sizeof(*Ev{}.xs) * (size_t)QT * a.q.d;
    if (lds > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "too many clusters for the distance tile (C=" + std::to_string(a.sup.C) + ")");
    const void* fn = reinterpret_cast<const void*>(&dist_kernel<Ev, LPQ>);
    KKM_TRY(allow_dynamic_lds(fn, lds));
    const unsigned blocks = (unsigned)((a.q.n + QT - 1) / QT);
    if (a.colmin && (int64_t)blocks > a.colpart_cap) return fail(KKM_ERR_INTERNAL, "column partials too small");
    hipLaunchKernelGGL((dist_kernel<Ev, LPQ>), dim3(blocks), dim3(256), lds, s, a);
    KKM_HIP(hipGetLastError());
    if (a.colmin && a.colpart_blocks) *a.colpart_blocks = blocks;
    return KKM_OK;
}

// Lanes per sample: more when there are few 64-sample tiles for the device and the segments are
// long enough to split.
int dist_lpq(const DistArgs& a, const DeviceInfo& dev, bool per_lane_rows) {
    const int64_t tiles = (a.q.n + 63) / 64;
    const double seg = (double)a.n_support / std::max(1, a.sup.C);
    // only the evaluators that read support rows per lane gain: the register-row evaluator streams
    // wave-uniform support rows through the scalar cache, which split lanes would turn into gathers
    if (per_lane_rows && tiles < 2 * (int64_t)dev.num_cus && seg >= 2.0) return seg >= 6.0 ? 4 : 2;
    return 1;
}

template <class Ev>
kkm_status launch_dist_ev(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    const int lpq = dist_lpq(a, dev, Ev::kPerLaneRows);
    if (lpq == 4) return launch_dist_lpq<Ev, 4>(a, dev, s);
    if (lpq == 2) return launch_dist_lpq<Ev, 2>(a, dev, s);
    return launch_dist_lpq<Ev, 1>(a, dev, s);
}

// RMSD: the sample tile staged in LDS as doubles when the workgroup's LDS stays within 64 KB (two
// or more workgroups per CU), else as floats (float input only), else read from memory per lane.
template <typename TI>
kkm_status launch_dist_rmsd(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    const size_t QT = 64 / (size_t)dist_lpq(a, dev, true);
    const size_t base = sizeof(double) * (size_t)a.sup.C * QT, cap = 64 * 1024;
    if (base + sizeof(double) * QT * (size_t)a.q.d <= cap) return launch_dist_ev<EvalRmsd64<TI, double>>(a, dev, s);
    if constexpr (std::is_same_v<TI, float>) {
        if (base + sizeof(float) * QT * (size_t)a.q.d <= cap) return launch_dist_ev<EvalRmsd64<TI, float>>(a, dev, s);
    }
    return launch_dist_ev<EvalGeneric64<TI>>(a, dev, s);
}

template <typename TI, typename TC>
kkm_status launch_dist_dot(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    switch (a.sup.dpad) {
        case 4: return launch_dist_ev<EvalDot<TI, TC, 4>>(a, dev, s);
        case 8: return launch_dist_ev<EvalDot<TI, TC, 8>>(a, dev, s);
        case 16: return launch_dist_ev<EvalDot<TI, TC, 16>>(a, dev, s);
        case 32: return launch_dist_ev<EvalDot<TI, TC, 32>>(a, dev, s);
        case 64: return launch_dist_ev<EvalDot<TI, TC, 64>>(a, dev, s);
        case 128: return launch_dist_ev<EvalDot<TI, TC, 128>>(a, dev, s);
        default: return fail(KKM_ERR_INTERNAL, "unexpected padded dimension");
    }
}

}  // namespace

bool dist_is_fp64(const DistArgs& a) {
    return a.precision == KKM_PREC_FP64 || (a.ks.type == KKM_KERNEL_RMSD && !mfma_dist_applies(a));
}

size_t dist_lds_bytes(const DistArgs& a) { return (dist_is_fp64(a) ? 8 : 4) * (size_t)a.sup.C * 64; }  // LPQ = 1

kkm_status launch_dist(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    if (a.q.n <= 0) return KKM_OK;
    if (mfma_dist_applies(a)) return launch_dist_mfma(a, dev, s);
    const bool f64 = a.dtype == KKM_F64;
    if (a.ks.type == KKM_KERNEL_RMSD) return f64 ? launch_dist_rmsd<double>(a, dev, s) : launch_dist_rmsd<float>(a, dev, s);
    if (dist_is_fp64(a)) {
        return f64 ? launch_dist_ev<EvalGeneric64<double>>(a, dev, s) : launch_dist_ev<EvalGeneric64<float>>(a, dev, s);
    }
    if (a.q.d > kMaxRegDim) return fail(KKM_ERR_UNSUPPORTED, "FP32 path supports d <= 128");
    return f64 ? launch_dist_dot<double, float>(a, dev, s) : launch_dist_dot<float, float>(a, dev, s);
}

kkm_status launch_refine(const DistArgs& a, const DeviceInfo& dev, hipStream_t s, int64_t n_support) {
    if (a.q.n <= 0) return KKM_OK;
    const bool per_block = n_support > 256;   // large supports: a whole block per listed row
    const size_t lds = per_block ? sizeof(double) * (kRefineChunk + (size_t)a.sup.C)
                                 : sizeof(double) * 4 * (256 + (size_t)a.sup.C);
    // (the listed rows are usually few: one workgroup per CU, each taking rows in turn; supports and
    // cluster counts up to 512 take half-size workgroups, two per CU, so that twice the rows run at
    // once; workgroups without a row leave at once)
    const bool half = per_block && n_support <= kRefineThreads / 2 && a.sup.C <= kRefineThreads / 2;
    const unsigned threads = half ? kRefineThreads / 2 : kRefineThreads;
    const unsigned blocks = per_block ? (unsigned)std::min<int64_t>(a.q.n, (half ? 2 : 1) * (int64_t)dev.num_cus)
                                      : (unsigned)std::min<int64_t>((a.q.n + 3) / 4, 2 * (int64_t)dev.num_cus);
    return dispatch_dp(eval_dp(a.ks.type, a.ks.d), [&]<int DP>() -> kkm_status {
        if (per_block) {
            if (a.dtype == KKM_F64)
                hipLaunchKernelGGL((refine_block_kernel<double, DP>), dim3(blocks), dim3(threads), lds, s, a);
            else
                hipLaunchKernelGGL((refine_block_kernel<float, DP>), dim3(blocks), dim3(threads), lds, s, a);
        } else {
            if (a.dtype == KKM_F64)
                hipLaunchKernelGGL((refine_kernel<double, DP>), dim3(blocks), dim3(256), lds, s, a);
            else
                hipLaunchKernelGGL((refine_kernel<float, DP>), dim3(blocks), dim3(256), lds, s, a);
        }
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    });
}

kkm_status launch_kernel_block(const KSpec& ks, int dtype, const void* X, int64_t nx, const void* Y, int64_t ny,
                               double* K, const DeviceInfo& dev, hipStream_t s) {
    const int64_t total = nx * ny;
    if (total <= 0) return KKM_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 64 * (int64_t)dev.num_cus);
    if (dtype == KKM_F64)
        hipLaunchKernelGGL(kernel_block_kernel<double>, dim3(blocks), dim3(256), 0, s, ks,
                           static_cast<const double*>(X), nx, static_cast<const double*>(Y), ny, K);
    else
        hipLaunchKernelGGL(kernel_block_kernel<float>, dim3(blocks), dim3(256), 0, s, ks,
                           static_cast<const float*>(X), nx, static_cast<const float*>(Y), ny, K);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

bool dist_is_bf16(const DistArgs& a) { return a.precision == KKM_PREC_BF16 && mfma_dist_applies(a); }

kkm_status launch_best64(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    if (a.q.n <= 0 || !a.best) return KKM_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>((a.q.n + 255) / 256, 16 * (int64_t)dev.num_cus);
    return dispatch_dp(eval_dp(a.ks.type, a.ks.d), [&]<int DP>() -> kkm_status {
        if (a.dtype == KKM_F64) hipLaunchKernelGGL((best64_kernel<double, DP>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((best64_kernel<float, DP>), dim3(blocks), dim3(256), 0, s, a);
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    });
}

kkm_status launch_sum(const double* best, int64_t n, double* partials, double* out, hipStream_t s) {
    const int64_t P = 1024;
    const int64_t chunk = std::max<int64_t>(1, (n + P - 1) / P);
    const int64_t blocks = std::max<int64_t>(1, (n + chunk - 1) / chunk);
    hipLaunchKernelGGL(sum_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s, best, n, chunk, partials);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_partial_kernel, dim3(1), dim3(256), 0, s, partials, blocks, blocks, out);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

}  // namespace kkm
