// Landmark phase of one mini-batch:
//
//   1. the landmark kernel block K_LL = K(x_l, x_m) in FP64 and, for the Eq. 8 initialisation,
//      K(x_l, m_j) for the global medoids (landmark_k_kernel, 32 x 32 tiles; RMSD frames:
//      landmark_block_kernel, 32 x 32 tiles);
//   2. the initial landmark labels: given, or the nearest global medoid (Eq. 8, with K(m,m)) --
//      taken by landmark_k_kernel itself when the medoid columns fit one tile; else each medoid
//      tile leaves the minimum over its columns per row, and the loop kernel combines them (RMSD:
//      landmark_init_kernel);
//   3. one kernel for the landmark loop, all workgroups resident (Eq. 14-17 restricted to the
//      landmarks):
//        counting sort of the landmarks by label  -> CSR segments L_j, c_j = |L_j|
//        S[m][j]  = sum_{m' in L_j} K(l_m, l_m')                (so f^(l_m, j) = S / c_j, Eq. 17)
//        g^_j     = 1/c_j^2 sum_{m in L_j} S[m][j]              (Eq. 16)
//        u_m      = argmin_j K(l_m,l_m) - 2 S[m][j]/c_j + g^_j  (Eq. 15, +inf when c_j = 0)
//      until no landmark label changes or max_updates updates were made;
//   4. the centroid support of the final labels: landmark rows in CSR order with a_l = 1/c_j,
//      their squared norms, the segment offsets and g^ -- the input of the batch-wide pass.
//
// Eq. 16-17 read only landmark labels, so the labels of the whole batch are not needed inside the
// loop; one pass over the batch from the final centroids reproduces the paper's full loop.
//
// Every sum has a fixed order that depends only on the labels (CSR order within a segment, row
// order, then workgroup order), so results are bitwise repeatable.  Cross-workgroup data is written
// and read with device-scope accesses, so the waits on it need no cache maintenance.
#include <cstdlib>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {

namespace {

// Threads per workgroup of the loop kernel: one workgroup per CU (its LDS holds the own rows of K),
// so a wide workgroup is what gives each SIMD several wavefronts to interleave.
constexpr int kLoopThreads = 1024;
// Updates that change at most this many landmark labels move g^ by the pair formula (no exchange).
constexpr int kPairMax = 64;
constexpr int kPairPerWave = (kPairMax + kLoopThreads / 64 - 1) / (kLoopThreads / 64);   // changes per wavefront
// Published labels carry the update that produced them above their low kLabelBits bits (labels are
// below 1024), so a reader can wait on the label itself.
constexpr int kLabelBits = 11;

struct LdsLayout {
    double* K;         // [R][ell] own rows of the landmark block (when staged in LDS)
    double* red;       // [max(kLoopThreads, C)] partial-sum scratch
    int32_t* lbl;      // [ell]
    int32_t* perm;     // [ell]
    int32_t* off;      // [C+1]
    uint8_t* rank;     // [ell] rank within its 64-landmark chunk among equal labels
    uint16_t* chunk;   // [nchunks][C] count, then base, per chunk and label
    double* S;         // [R][C]
    double* gh;        // [C]
    double* kself;     // [R] K(l, l) of the own landmarks
    int32_t* qoff;     // [C+1] first 64-element chunk of each segment (chunks per row: qoff[C])
    double* part;      // [R][nq_max] chunk partial sums, nq_max = ceil(ell/64) + C
    int32_t* lmv;      // [ell] position of every landmark in the batch
    int32_t* nlab;     // [ell] labels after an update
    int32_t* chg;      // [ell + 1] changed landmarks in index order; chg[ell] = their number
    int32_t* cnt;      // [C] landmarks per cluster
    double* rcnt;      // [C] 1 / c_j
    uint64_t* cmask;   // [nchunks] changed-landmark ballot of every 64-landmark chunk
    int32_t* ccnt;     // [nchunks] its population count
    double* T;         // [C] sum over m, m' in L_j of K(m, m')  (= c_j^2 g^_j)
    double* dT;        // [C] its change over one update (pair path)
    int32_t* pab;      // [kPairMax] old | new << 16 label of change t (pair path)
    double* psa;       // [kPairMax] S[m_t][old]  before the update
    double* psb;       // [kPairMax] S[m_t][new]  before the update
    double* pwa;       // [kPairMax] sum_t' delta_t'(old_t) K(m_t, m_t')
    double* pwb;       // [kPairMax] sum_t' delta_t'(new_t) K(m_t, m_t')
};

// Row stride of K_LL (in HBM and LDS): a multiple of 16 doubles, so every row starts on a 128-byte
// line and the block kernel's row segments are whole lines.
__host__ __device__ inline int k_ld(int ell) { return (ell + 15) & ~15; }

__device__ __forceinline__ size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t landmark_lds_bytes(int ell, int C, int R, bool k_in_lds) {
    const int nchunks = (ell + 63) / 64;
    size_t b = 0;
    if (k_in_lds) b += sizeof(double) * (size_t)R * k_ld(ell);
    b = (b + 15) & ~size_t(15); b += sizeof(double) * (size_t)(C > kLoopThreads ? C : kLoopThreads);
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * (C + 1);
    b = (b + 15) & ~size_t(15); b += ell;
    b = (b + 15) & ~size_t(15); b += sizeof(uint16_t) * (size_t)nchunks * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * (size_t)R * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * R;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * (C + 1);
    b = (b + 15) & ~size_t(15); b += sizeof(double) * (size_t)R * ((ell + 63) / 64 + C);
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * (ell + 1);
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * C;
    b = (b + 15) & ~size_t(15); b += sizeof(uint64_t) * nchunks;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * nchunks;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * 2 * (size_t)C;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * kPairMax;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * 4 * kPairMax;
    return (b + 15) & ~size_t(15);
}

__device__ LdsLayout carve_lds(unsigned char* base, int ell, int C, int R, bool k_in_lds) {
    const int nchunks = (ell + 63) / 64;
    LdsLayout L;
    size_t b = 0;
    L.K = reinterpret_cast<double*>(base);
    if (k_in_lds) b += sizeof(double) * (size_t)R * k_ld(ell);
    b = al16(b); L.red = reinterpret_cast<double*>(base + b); b += sizeof(double) * (size_t)(C > kLoopThreads ? C : kLoopThreads);
    b = al16(b); L.lbl = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.perm = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.off = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * (C + 1);
    b = al16(b); L.rank = reinterpret_cast<uint8_t*>(base + b); b += ell;
    b = al16(b); L.chunk = reinterpret_cast<uint16_t*>(base + b); b += sizeof(uint16_t) * (size_t)nchunks * C;
    b = al16(b); L.S = reinterpret_cast<double*>(base + b); b += sizeof(double) * (size_t)R * C;
    b = al16(b); L.gh = reinterpret_cast<double*>(base + b); b += sizeof(double) * C;
    b = al16(b); L.kself = reinterpret_cast<double*>(base + b); b += sizeof(double) * R;
    b = al16(b); L.qoff = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * (C + 1);
    b = al16(b); L.part = reinterpret_cast<double*>(base + b); b += sizeof(double) * (size_t)R * ((ell + 63) / 64 + C);
    b = al16(b); L.lmv = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.nlab = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.chg = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * (ell + 1);
    b = al16(b); L.cnt = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * C;
    b = al16(b); L.rcnt = reinterpret_cast<double*>(base + b); b += sizeof(double) * C;
    b = al16(b); L.cmask = reinterpret_cast<uint64_t*>(base + b); b += sizeof(uint64_t) * nchunks;
    b = al16(b); L.ccnt = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * nchunks;
    b = al16(b); L.T = reinterpret_cast<double*>(base + b); b += sizeof(double) * C;
    L.dT = L.T + C; b += sizeof(double) * C;
    b = al16(b); L.pab = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * kPairMax;
    b = al16(b); L.psa = reinterpret_cast<double*>(base + b);
    L.psb = L.psa + kPairMax;
    L.pwa = L.psb + kPairMax;
    L.pwb = L.pwa + kPairMax;
    return L;
}

// Stable counting sort of the ell labels in L.lbl into L.perm / L.off (whole workgroup).
__device__ __forceinline__ void csr_sort(const LdsLayout& L, int ell, int C) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int nchunks = (ell + 63) / 64;
    for (int i = tid; i < nchunks * C; i += nt) L.chunk[i] = 0;
    __syncthreads();
    // ranks inside each 64-landmark chunk: the lanes holding the same label are the AND, over the
    // label's bits, of the ballot of that bit (or of its complement); the equal lanes below a lane
    // are its rank, all of them the label's count in the chunk, which the label's first lane stores
    const int nbits = C > 1 ? 32 - __builtin_clz((unsigned)(C - 1)) : 1;
    for (int ch = wave; ch < nchunks; ch += nwaves) {
        const int m = ch * 64 + lane;
        const bool valid = m < ell;
        const int lab = valid ? L.lbl[m] : 0;
        uint64_t eq = __ballot(valid);
        for (int bt = 0; bt < nbits; ++bt) {
            const bool on = (lab >> bt) & 1;
            const uint64_t bb = __ballot(valid && on);
            eq &= on ? bb : ~bb;
        }
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int rk = (int)__popcll(eq & below);
        if (valid) {
            L.rank[m] = (uint8_t)rk;
            if (rk == 0) L.chunk[ch * C + lab] = (uint16_t)__popcll(eq);
        }
    }
    __syncthreads();
    // per label: exclusive prefix over chunks (in place) and the total count
    for (int j = tid; j < C; j += nt) {
        int run = 0;
        for (int ch = 0; ch < nchunks; ++ch) {
            const int t = L.chunk[ch * C + j];
            L.chunk[ch * C + j] = (uint16_t)run;
            run += t;
        }
        L.off[j + 1] = run;
    }
    __syncthreads();
    // segment offsets = exclusive scan of the counts, and qoff = exclusive scan of the number of
    // 64-element chunks ceil(len_j / 64) of every segment (first wave)
    if (wave == 0) {
        int carry = 0, qcarry = 0;
        for (int base = 0; base < C; base += 64) {
            const int j = base + lane;
            const int cnt = (j < C) ? L.off[j + 1] : 0;
            int v = cnt, q = (cnt + 63) / 64;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(v, o, 64);
                const int tq = __shfl_up(q, o, 64);
                if (lane >= o) { v += t; q += tq; }
            }
            if (j < C) {
                L.off[j + 1] = carry + v;
                L.qoff[j + 1] = qcarry + q;
            }
            carry += __shfl(v, 63, 64);
            qcarry += __shfl(q, 63, 64);
        }
        if (lane == 0) {
            L.off[0] = 0;
            L.qoff[0] = 0;
        }
    }
    __syncthreads();
    for (int m = tid; m < ell; m += nt) {
        const int lab = L.lbl[m];
        L.perm[L.off[lab] + L.chunk[(m >> 6) * C + lab] + L.rank[m]] = m;
    }
    __syncthreads();
}

// S[r][j] = sum over segment j (CSR of L.lbl) of own row r, from scratch: every 64-element chunk of a
// segment is summed in order by one thread, then the chunk sums of each (row, segment) in order.
// Also sets L.cnt.  Whole workgroup; expects csr_sort(L) done.
__device__ __forceinline__ void full_sums(const LdsLayout& L, const double* Krows, int ldk, int nr, int C) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nq = L.qoff[C];
    for (int p = tid; p < nr * nq; p += nt) {
        const int r = p / nq, qi = p - r * nq;
        int lo_j = 0, hi_j = C;                 // segment j with qoff[j] <= qi < qoff[j+1]
        while (hi_j - lo_j > 1) {
            const int mid = (lo_j + hi_j) >> 1;
            if (L.qoff[mid] <= qi) lo_j = mid; else hi_j = mid;
        }
        const int j = lo_j;
        const int k0 = L.off[j] + (qi - L.qoff[j]) * 64;
        const int k1 = min(L.off[j + 1], k0 + 64);
        const double* Kr = Krows + (int64_t)r * ldk;
        double s = 0.0;
#pragma unroll 8
        for (int k = k0; k < k1; ++k) s += Kr[L.perm[k]];
        L.part[p] = s;
    }
    __syncthreads();
    for (int p = tid; p < nr * C; p += nt) {
        const int r = p / C, j = p - r * C;
        double s = 0.0;
        for (int qi = L.qoff[j]; qi < L.qoff[j + 1]; ++qi) s += L.part[r * nq + qi];
        L.S[p] = s;
    }
    for (int j = tid; j < C; j += nt) L.cnt[j] = L.off[j + 1] - L.off[j];
    __syncthreads();
}

// Values exchanged between the workgroups of the loop kernel (cluster partial sums, new labels) are
// written and read as relaxed device-scope atomics: those accesses pass the per-XCD L2 caches, so
// a value whose store has completed is what every other workgroup's device-scope load returns.
template <typename T>
__device__ __forceinline__ void xput(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ T xget(T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// The cluster partial sums of an exchange are their own signal: exchange e of a batch uses buffer
// e % 3 of partial ([3][grid][C]), whose slots hold kNoPart until written, and the readers wait on
// the slots themselves (bounded: past kSpinCap polls the workgroup records an error and proceeds,
// so the kernel always terminates).  Buffer 0 is filled before the loop (reset_batch_state); a
// workgroup clears its slots of buffer (e + 1) % 3 during exchange e, before publishing its sums:
// that buffer was last read in exchange e - 2, which every workgroup has finished once all sums of
// exchange e - 1 exist, and the workgroup read them all before exchange e; a reader of exchange
// e + 1 waits for this workgroup's exchange-e sums first, so it cannot find the old values.
// Every workgroup takes the same exchanges (the choice follows from the shared labels).
constexpr unsigned kSpinCap = 1u << 26;
constexpr unsigned long long kNoPart = 0x7ff4dead0badf00dull;   // a NaN pattern no sum produces
__device__ __forceinline__ bool no_part(double v) { return (unsigned long long)__double_as_longlong(v) == kNoPart; }

// Counters the loop and the later kernels of the batch expect cleared (one workgroup).
__device__ __forceinline__ void reset_batch_state(const LandmarkArgs& a) {
    for (int i = threadIdx.x; i <= a.max_updates; i += blockDim.x) a.changed[i] = 0;
    for (int i = threadIdx.x; i < a.n_zero_ints; i += blockDim.x) a.zero_ints[i] = 0;
    for (int i = threadIdx.x; i < a.C; i += blockDim.x) a.colmin[i] = ~0ull;
    for (int i = threadIdx.x; i < 2 * a.ell; i += blockDim.x) a.nlab_x[i] = 0;   // no update published yet
    for (int i = threadIdx.x; i < a.grid * a.C; i += blockDim.x) a.partial[i] = __longlong_as_double((long long)kNoPart);
    // (the error flag accumulates over the fit: cleared once by the host)
    if (threadIdx.x == 0) *reinterpret_cast<unsigned int*>(a.snorm_max) = 0u;
}

// Wall-clock stamp of workgroup 0 (profiling aid): slot 0 holds the count, which thread 0 also
// keeps in ns (no load on the timed path).
__device__ __forceinline__ void stamp(const LandmarkArgs& a, int& ns) {
    if (a.trace && blockIdx.x == 0 && threadIdx.x == 0 && ns < 63) {
        a.trace[1 + ns] = (int64_t)wall_clock64();
        a.trace[0] = ++ns;
    }
}

// 1. K_LL in FP64, one 32 x 32 tile per workgroup (4 entries per thread), the two row sets staged
//    in LDS as doubles.  Linear and RBF kernels are symmetric: only tiles on or above the diagonal
//    are evaluated and mirrored.  Block 0 also clears the loop's counters.
template <typename TI>
__global__ __launch_bounds__(256) void landmark_block_kernel(LandmarkArgs a, int tiles) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int ell = a.ell;
    const bool sym = a.ktype != KKM_KERNEL_RMSD;
    int tr = blockIdx.y, tc = blockIdx.x;
    if (sym) {   // blockIdx.x enumerates the upper-triangular tiles (tr <= tc)
        int t = blockIdx.x;
        tr = 0;
        while (t >= tiles - tr) { t -= tiles - tr; ++tr; }
        tc = tr + t;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0) reset_batch_state(a);
    double* A = reinterpret_cast<double*>(smem);          // [32][d]
    double* Bm = A + 32 * a.d;                             // [32][d]
    __shared__ int64_t rowa[32], rowb[32];                 // element offsets of the tile's rows
    const int r0 = tr * 32, c0 = tc * 32;
    const TI* X = static_cast<const TI*>(a.X);
    if (threadIdx.x < 32) {
        const int ra = min(ell - 1, r0 + (int)threadIdx.x), rb = min(ell - 1, c0 + (int)threadIdx.x);
        rowa[threadIdx.x] = (a.base + (int64_t)a.lm[ra] * a.stride) * a.d;
        rowb[threadIdx.x] = (a.base + (int64_t)a.lm[rb] * a.stride) * a.d;
    }
    __syncthreads();
    // four elements per thread at a time: their loads are issued before the LDS stores
    const int64_t nel = 32 * a.d;
    for (int64_t i0 = threadIdx.x; i0 < nel; i0 += 4 * (int64_t)blockDim.x) {
        double va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = min(i0 + u * (int64_t)blockDim.x, nel - 1);
            const int r = (int)(i / a.d);
            const int64_t c = i - (int64_t)r * a.d;
            va[u] = (double)X[rowa[r] + c];
            vb[u] = (double)X[rowb[r] + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * (int64_t)blockDim.x;
            if (i < nel) {
                A[i] = va[u];
                Bm[i] = vb[u];
            }
        }
    }
    __syncthreads();
    const KSpec ks{a.ktype, a.n_atoms, a.d, a.inv2s2};
    const int tx = threadIdx.x & 31, ty0 = threadIdx.x >> 5;   // rows ty0, ty0 + 8, ty0 + 16, ty0 + 24
    for (int k = 0; k < 4; ++k) {
        const int ty = ty0 + 8 * k;
        const int r = r0 + ty, c = c0 + tx;
        if (r < ell && c < ell && (!sym || tr < tc || ty <= tx)) {
            const double v = k64(ks, A + ty * a.d, Bm + tx * a.d);
            a.Kbuf[(int64_t)r * a.ldk + c] = v;
            if (sym) a.Kbuf[(int64_t)c * a.ldk + r] = v;
        }
    }
}

// 2. Initial label of one landmark: given, or argmin_j K(x,x) - 2 K(x, m_j) + K(m_j, m_j) (Eq. 8)
//    over the clusters with a medoid, lowest j on ties.
template <typename TI, int DP>
__global__ __launch_bounds__(256) void landmark_init_kernel(LandmarkArgs a) {
    const int r = blockIdx.x;
    if (a.init_mode == 0) {
        if (threadIdx.x == 0) a.lab[r] = a.lab_init[r];
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    double* x = reinterpret_cast<double*>(smem);          // [d]
    const TI* X = static_cast<const TI*>(a.X);
    const TI* xr = X + (a.base + (int64_t)a.lm[r] * a.stride) * a.d;
    for (int64_t c = threadIdx.x; c < a.d; c += blockDim.x) x[c] = (double)xr[c];
    __syncthreads();
    const KSpec ks{a.ktype, a.n_atoms, a.d, a.inv2s2};
    const double kxx = kself64(ks, x);
    const TI* M = static_cast<const TI*>(a.M);
    double bv = kInf;
    int bj = a.C;
    for (int j = threadIdx.x; j < a.C; j += blockDim.x) {
        const double ms = a.Mself[j];
        if (!(ms < kInf)) continue;
        const double dj = kxx - 2.0 * k64p<DP>(ks, x, M + (int64_t)j * a.Mpad) + ms;
        if (dj < bv) { bv = dj; bj = j; }
    }
    __shared__ double sv[256];
    __shared__ int si[256];
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bj;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            const double v2 = sv[threadIdx.x + w];
            const int i2 = si[threadIdx.x + w];
            if (v2 < sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.lab[r] = si[0] < a.C ? si[0] : 0;
}

// 1'. Linear / RBF kernels: K_LL and, for the Eq. 8 initialisation, K(x_l, m_j) for the C global
//     medoids, in FP64: one T x T tile of the (landmarks) x (landmarks, medoids) matrix per
//     workgroup (T = 32, or 64 for rows of 4 dimensions), (T/16)^2 entries per thread, both row sets
//     staged in LDS 16 dimensions at a time.
//     Same arithmetic as the FP64 evaluator (dimension order; explicit differences for RBF).
//     Block (0, 0) also clears the loop's counters.
template <typename TI, int DP, bool LIN, int T>
__global__ __launch_bounds__(256) void landmark_k_kernel(LandmarkArgs a) {
    constexpr int CH = DP < 16 ? DP : 16;
    constexpr int NI = T / 16;   // entries per thread along each side
    __shared__ double As[CH][T + 1];
    __shared__ double Bs[CH][T + 1];
    const int ell = a.ell, C = a.C, d = (int)a.d;
    // medoid columns start on a tile boundary; when they fit one tile, its workgroups also take the
    // Eq. 8 labels of their rows (lowest j among equal minima over the clusters with a medoid)
    const int mc0 = (ell + T - 1) / T * T;
    const int ncol = a.init_mode ? mc0 + C : ell;
    const bool init_here = a.init_mode && C <= T;
    const int parts = a.init_parts;   // > 0: this tile's minimum per row, combined by the loop kernel
    const int r0 = blockIdx.y * T, c0 = blockIdx.x * T;
    if (blockIdx.x == 0 && blockIdx.y == 0) reset_batch_state(a);
    if (blockIdx.x == 0 && !a.init_mode)   // given initial labels
        for (int r = r0 + (int)threadIdx.x; r < min(ell, r0 + T); r += blockDim.x) a.lab[r] = a.lab_init[r];
    if (c0 >= ncol || (c0 >= ell && c0 < mc0)) return;   // uniform
    const TI* X = static_cast<const TI*>(a.X) + a.base * a.d;
    const TI* M = static_cast<const TI*>(a.M);
    const int64_t rs = a.stride * a.d;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    constexpr bool lin = LIN;
    double acc[NI][NI];
    double kxx[NI];   // linear kernel: K(x_r, x_r) by the same FMA chain as the diagonal entry
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        kxx[i] = 0.0;
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = 0.0;
    }
    // staging: element p = threadIdx.x + 256 u of a stage is (row rr = p / CH, dimension k = p % CH);
    // the row starts are resolved once, and each stage issues all its loads before the LDS stores
    constexpr int PER = T * CH / 256;
    static_assert(PER * 256 == T * CH, "staging covers the tile exactly");
    // The tile's row starts are resolved once into LDS (one index load per thread, all in flight
    // together); every element load is then issued unconditionally -- rows past the tile are clamped
    // to a real row and dimensions past d to the last one, the values scaled by a 0 / 1 mask -- so
    // the loads of a stage are in flight together instead of one branch and one wait each.  (Scaling
    // by 1 keeps every value bit for bit; masked entries add exact zeros.)
    // (held as element offsets from X or M, not as pointers: a pointer read back from LDS would
    // turn the element loads into flat ones)
    __shared__ int64_t rowo[2][T];
    __shared__ int rowm[2][T];
    __shared__ float rowok[2][T];
    if (threadIdx.x < 2 * T) {
        const int side = threadIdx.x / T, t = threadIdx.x - side * T;
        const int g = (side == 0 ? r0 : c0) + t;
        const bool cm = side == 1 && g >= mc0 && g < ncol;
        rowo[side][t] = cm ? (int64_t)(g - mc0) * a.Mpad : (int64_t)a.lm[min(g, ell - 1)] * rs;
        rowm[side][t] = cm ? 1 : 0;
        rowok[side][t] = (g < ell || cm) ? 1.0f : 0.0f;
    }
    __syncthreads();
    const TI* pa[PER];
    const TI* pb[PER];
    int kk[PER];
    double ma[PER], mb[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = threadIdx.x + 256 * u;
        const int rr = p / CH;
        kk[u] = p - rr * CH;
        pa[u] = X + rowo[0][rr];
        pb[u] = (rowm[1][rr] ? M : X) + rowo[1][rr];
        ma[u] = rowok[0][rr];
        mb[u] = rowok[1][rr];
    }
    // every stage's values are requested before the first is used (kept at the data's precision
    // until their stage), so that the stages wait for one round of loads instead of one each
    constexpr int NS = DP / CH;
    TI ra[NS][PER], rb[NS][PER];
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int dc = min(st * CH + kk[u], d - 1);
            ra[st][u] = pa[u][dc];
            rb[st][u] = pb[u][dc];
        }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int k0 = st * CH;
        double va[PER], vb[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const double in = k0 + kk[u] < d ? 1.0 : 0.0;
            va[u] = (double)ra[st][u] * (ma[u] * in);
            vb[u] = (double)rb[st][u] * (mb[u] * in);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int p = threadIdx.x + 256 * u;
            As[kk[u]][p / CH] = va[u];
            Bs[kk[u]][p / CH] = vb[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < CH; ++k) {
            double av[NI], bw[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) av[i] = As[k][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < NI; ++j) bw[j] = Bs[k][tx + 16 * j];
            if constexpr (lin) {
#pragma unroll
                for (int i = 0; i < NI; ++i) kxx[i] = fma(av[i], av[i], kxx[i]);
            }
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if constexpr (lin) {
                        acc[i][j] = fma(av[i], bw[j], acc[i][j]);
                    } else {
                        const double t = av[i] - bw[j];
                        acc[i][j] = fma(t, t, acc[i][j]);
                    }
                }
        }
    }
    if ((init_here && c0 == mc0) || (parts > 0 && c0 >= mc0)) {
        // Eq. 8 for rows r0 + ty + 16 i over the tile's medoid columns (all of them when they fit
        // one tile): the 16 lanes of a row (tx) hold them; the lowest cluster among equal minima
        const int mb = c0 - mc0;   // the tile's first medoid
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int r = r0 + ty + 16 * i;
            const double kself_r = lin ? kxx[i] : 1.0;   // RBF: exp(0)
            double bv = kInf;
            int bj = C;
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                const int m = mb + tx + 16 * j;
                if (m < C) {
                    const double ms = a.Mself[m];
                    if (ms < kInf) {
                        const double kv = lin ? acc[i][j] : ::exp(-acc[i][j] * a.inv2s2);
                        const double v = kself_r - 2.0 * kv + ms;
                        if (bj == C || v < bv) { bv = v; bj = m; }
                    }
                }
            }
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                const double v2 = __shfl_xor(bv, o, 64);
                const int j2 = __shfl_xor(bj, o, 64);
                if (j2 < C && (bj == C || v2 < bv || (v2 == bv && j2 < bj))) { bv = v2; bj = j2; }
            }
            if (tx == 0 && r < ell) {
                if (parts > 0) {
                    double* pp = a.Kmed + ((int64_t)r * parts + mb / T) * 2;
                    pp[0] = bv;
                    pp[1] = (double)bj;   // (C when the tile has no medoid set)
                } else {
                    a.lab[r] = bj < C ? bj : 0;
                }
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
            if (r < ell && c < ncol) {
                const double v = lin ? acc[i][j] : ::exp(-acc[i][j] * a.inv2s2);
                if (c < ell) a.Kbuf[(int64_t)r * a.ldk + c] = v;   // (medoid columns: taken above)
            }
        }
}

// 3-4. The landmark loop and the centroid support (grid <= device CUs, all workgroups resident).
//
// Workgroup wg owns landmark rows [r0, r1): their rows of K (in LDS when they fit) and of S.  Every
// workgroup keeps all landmark labels, cluster counts and T_j = c_j^2 g^_j.  Before the first update
// the own parts of sum_{m in L_j} S[m][j] are exchanged and summed in the same order everywhere.
// An update is then
//   Eq. 15 for the own rows, publish their labels (and S at the old and new label of a changed row)
//   -> wait for every label of the update -> the changed list, own rows of S follow the changes
//   (incrementally in landmark order, or from scratch), and T follows either by the pair formula
//   (at most kPairMax changes, no exchange) or by a new exchange of the partial sums.
// No workgroup waits on a grid-wide barrier: every published value carries its own signal (labels
// are tagged with their update, partial sums replace a sentinel), and every buffer is rewritten
// only once its readers have provably moved past it (the label / S exchange alternates between two
// halves, the partial sums rotate over three buffers).
// KL: the own rows of K_LL are staged in LDS (else read from HBM); a compile-time choice, so the
// reads compile to LDS or global instructions rather than generic ones.
template <typename TI, bool KL>
__global__ __launch_bounds__(kLoopThreads) void landmark_phase_kernel(LandmarkArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int wg = blockIdx.x, G = gridDim.x;
    const int ell = a.ell, C = a.C;
    const int ldk = (int)a.ldk;
    const int R = (ell + G - 1) / G;
    const int r0 = min(ell, wg * R), r1 = min(ell, r0 + R), nr = r1 - r0;
    LdsLayout L = carve_lds(smem, ell, C, R, KL);
    const TI* X = static_cast<const TI*>(a.X);
    auto row = [&](int pos) { return X + (a.base + (int64_t)pos * a.stride) * a.d; };
    const double* const Kg = a.Kbuf + (int64_t)r0 * ldk;
    const double* const Krows = KL ? L.K : Kg;     // own row r at Krows + r * ldk
    int ns = 0;   // trace stamps taken (thread 0 of workgroup 0)

    stamp(a, ns);
    // The own rows of K are one contiguous, 16-byte aligned block, copied to LDS as double2: the
    // first KU per thread are loaded before the CSR sort of the labels and stored after it.
    typedef double dvec2 __attribute__((ext_vector_type(2)));
    constexpr int KU = 8;
    const int64_t n2 = KL ? (int64_t)nr * ldk / 2 : 0;
    const dvec2* ksrc = reinterpret_cast<const dvec2*>(Kg);
    dvec2* kdst = reinterpret_cast<dvec2*>(L.K);
    dvec2 kv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
        const int64_t i = tid + (int64_t)u * nt;
        if (i < n2) kv[u] = ksrc[i];
    }
    for (int m = tid; m < ell; m += nt) {
        int lb;
        if (a.init_parts > 0) {   // Eq. 8: the medoid tiles' minima in tile (= cluster) order
            const double* pp = a.Kmed + (int64_t)m * a.init_parts * 2;
            double bv = kInf;
            int bj = C;
            for (int p = 0; p < a.init_parts; ++p) {
                const double v2 = pp[2 * p];
                const int j2 = (int)pp[2 * p + 1];
                if (j2 < C && (bj == C || v2 < bv || (v2 == bv && j2 < bj))) {
                    bv = v2;
                    bj = j2;
                }
            }
            lb = bj < C ? bj : 0;
        } else {
            lb = a.lab[m];
        }
        L.lbl[m] = lb;
        L.lmv[m] = a.lm[m];
    }
    for (int r = tid; r < nr; r += nt) L.kself[r] = a.Kbuf[(int64_t)(r0 + r) * ldk + r0 + r];
    __syncthreads();
    stamp(a, ns);

    csr_sort(L, ell, C);
    if constexpr (KL) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t i = tid + (int64_t)u * nt;
            if (i < n2) kdst[i] = kv[u];
        }
        for (int64_t i0 = (int64_t)KU * nt; i0 < n2; i0 += (int64_t)KU * nt) {
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int64_t i = i0 + tid + (int64_t)u * nt;
                if (i < n2) kv[u] = ksrc[i];
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int64_t i = i0 + tid + (int64_t)u * nt;
                if (i < n2) kdst[i] = kv[u];
            }
        }
        __syncthreads();
    }
    stamp(a, ns);
    full_sums(L, Krows, ldk, nr, C);
    stamp(a, ns);

    const int nsub = C < nt ? nt / C : 1;     // threads per cluster in the partial reduction
    // T_j and g^_j from every workgroup's part of sum_{m in L_j} S[m][j] (in row order), exchanged
    // through the partial buffers (see kNoPart), then summed in a fixed order; also 1 / c_j
    int nexch = 0;
    auto exchange_T = [&]() {
        const int e = nexch++;
        double* Pw = a.partial + (int64_t)(e % 3) * G * C;
        double* Pn = a.partial + (int64_t)((e + 1) % 3) * G * C;
        for (int j = tid; j < C; j += nt) xput(Pn + (int64_t)wg * C + j, __longlong_as_double((long long)kNoPart));
        __builtin_amdgcn_s_waitcnt(0);   // (the clears complete before the sums are published)
        for (int j = tid; j < C; j += nt) {
            double acc = 0.0;
            int r = 0;
            for (; r + 8 <= nr; r += 8) {
                int lb[8];
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    lb[u] = L.lbl[r0 + r + u];
                    v[u] = L.S[(r + u) * C + j];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += lb[u] == j ? v[u] : 0.0;
            }
            for (; r < nr; ++r) acc += L.lbl[r0 + r] == j ? L.S[r * C + j] : 0.0;
            xput(Pw + (int64_t)wg * C + j, acc);
            L.rcnt[j] = L.cnt[j] > 0 ? 1.0 / (double)L.cnt[j] : 0.0;
        }
        stamp(a, ns);
        // nsub interleaved sub-sums per cluster, then in order (each sub-sum's loads, up to eight at a
        // time, are issued before they are added in workgroup order)
        for (int p = tid; p < nsub * C; p += nt) {
            const int j = p % C, sub = p / C;
            double acc = 0.0;
            for (int g0 = sub; g0 < G; g0 += 8 * nsub) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int g = g0 + u * nsub;
                    v[u] = g < G ? xget(Pw + (int64_t)g * C + j) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {   // (a slot not yet written: wait for it, bounded)
                    const int g = g0 + u * nsub;
                    if (g < G && no_part(v[u])) {
                        unsigned polls = 0;
                        do {
                            __builtin_amdgcn_s_sleep(1);
                            if (++polls > kSpinCap) {
                                atomicOr(a.error, 1);
                                v[u] = 0.0;
                                break;
                            }
                            v[u] = xget(Pw + (int64_t)g * C + j);
                        } while (no_part(v[u]));
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (g0 + u * nsub < G) acc += v[u];
            }
            L.red[p] = acc;
        }
        __syncthreads();
        for (int j = tid; j < C; j += nt) {
            double acc = 0.0;
            for (int sub = 0; sub < nsub; ++sub) acc += L.red[sub * C + j];
            const double cj = (double)L.cnt[j];
            L.T[j] = acc;
            L.gh[j] = cj > 0.0 ? acc / (cj * cj) : kInf;
        }
        __syncthreads();
        stamp(a, ns);
    };
    exchange_T();
    int it = 0, buf = 0;     // buf: which half of the double-buffered label / S exchange this update uses
    for (;;) {
        if (it >= a.max_updates) break;
        int32_t* nlx = a.nlab_x + (int64_t)buf * ell;
        double* sx = a.sx + (int64_t)buf * 2 * ell;
        const int epoch = it + 1;   // published with the labels of this update

        // Eq. 15 for the own rows (one wavefront per row; lowest j among equal minima); a changed row
        // also publishes S at its old and new label (for the pair update of g^)
        for (int r = wave; r < nr; r += nwaves) {
            double bv = kInf;
            int bj = C;
            for (int j = lane; j < C; j += 64) {
                if (L.cnt[j] == 0) continue;
                const double dj = L.kself[r] - 2.0 * L.S[r * C + j] * L.rcnt[j] + L.gh[j];
                if (bj == C || dj < bv) { bv = dj; bj = j; }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double v2 = __shfl_xor(bv, o, 64);
                const int j2 = __shfl_xor(bj, o, 64);
                if (j2 < C && (bj == C || v2 < bv || (v2 == bv && j2 < bj))) { bv = v2; bj = j2; }
            }
            if (lane == 0) {
                const int m = r0 + r, old = L.lbl[m], nl = bj < C ? bj : old;
                if (nl != old) {
                    xput(sx + 2 * (int64_t)m, L.S[r * C + old]);
                    xput(sx + 2 * (int64_t)m + 1, L.S[r * C + nl]);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_s_waitcnt(0);   // the S values are complete before the label appears
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                }
                xput(nlx + m, nl | (epoch << kLabelBits));
            }
        }
        stamp(a, ns);
        // new labels (each lane waits until its landmark's label of this update has appeared: no grid
        // barrier) and the changed landmarks in index order: every wavefront takes whole 64-landmark
        // chunks (ballot of the changes, mask and count kept in LDS), then writes its chunks' entries
        // after the prefix of the lower chunks' counts
        // With one chunk per wavefront, a lane that sees its landmark change loads the S values
        // published with the label right away (they are complete before the label appears), so
        // their loads overlap the other wavefronts' waits; the pair update then finds them in LDS.
        const bool pre_sx = (ell + 63) / 64 <= nwaves;
        {
            const int nchunks = (ell + 63) / 64;
            uint64_t* cmask = L.cmask;
            int32_t* ccnt = L.ccnt;
            double sa = 0.0, sb = 0.0;
            for (int ch = wave; ch < nchunks; ch += nwaves) {
                const int m = ch * 64 + lane;
                bool chg = false;
                if (m < ell) {
                    int v = xget(nlx + m);
                    unsigned polls = 0;
                    while (((unsigned)v >> kLabelBits) != (unsigned)epoch) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++polls > kSpinCap) {   // bounded: report, keep the old label
                            atomicOr(a.error, 1);
                            v = L.lbl[m];
                            break;
                        }
                        v = xget(nlx + m);
                    }
                    const int nl = v & ((1 << kLabelBits) - 1);
                    L.nlab[m] = nl;
                    chg = nl != L.lbl[m];
                    if (chg && pre_sx) {
                        sa = xget(sx + 2 * (int64_t)m);
                        sb = xget(sx + 2 * (int64_t)m + 1);
                    }
                }
                const uint64_t mask = __ballot(chg);
                if (lane == 0) {
                    cmask[ch] = mask;
                    ccnt[ch] = (int)__popcll(mask);
                }
            }
            __syncthreads();
            for (int ch = wave; ch < nchunks; ch += nwaves) {
                int base_out = 0;
                for (int c = 0; c < ch; ++c) base_out += ccnt[c];
                const uint64_t mask = cmask[ch];
                if ((mask >> lane) & 1ull) {
                    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                    const int pos = base_out + below;
                    L.chg[pos] = ch * 64 + lane;
                    if (pre_sx && pos < kPairMax) {
                        L.psa[pos] = sa;
                        L.psb[pos] = sb;
                    }
                }
                if (ch == nchunks - 1 && lane == 0) L.chg[ell] = base_out + ccnt[ch];
            }
            __syncthreads();
        }
        const int nch = L.chg[ell];
        stamp(a, ns);
        ++it;
        if (nch == 0) break;

        // Few changes: the change of T_j follows from the old S values of the changed landmarks and K
        // between changed landmarks, with delta_t(j) = [j = new_t] - [j = old_t]:
        //   dT_j = sum_t delta_t(j) (2 S[m_t][j] + sum_t' delta_t'(j) K(m_t, m_t'))
        // (every workgroup evaluates it in the same order, so T stays identical everywhere)
        const bool pair = nch <= kPairMax;
        if (pair) {
            // K between the changed landmarks, loaded first so that these loads and the loads of the
            // published S values below (when not loaded already) are in flight together: wavefront w takes the changes
            // t = w + u * nwaves (u < kPairPerWave covers kPairMax with kLoopThreads threads), lane t'
            // the change t'
            double kv[kPairPerWave];
#pragma unroll
            for (int u = 0; u < kPairPerWave; ++u) {
                const int t = wave + u * nwaves;
                kv[u] = (t < nch && lane < nch) ? a.Kbuf[(int64_t)L.chg[t] * ldk + L.chg[lane]] : 0.0;
            }
            for (int t = tid; t < nch; t += nt) {
                const int m = L.chg[t];
                L.pab[t] = L.lbl[m] | (L.nlab[m] << 16);
                if (!pre_sx) {
                    L.psa[t] = xget(sx + 2 * (int64_t)m);
                    L.psb[t] = xget(sx + 2 * (int64_t)m + 1);
                }
            }
            __syncthreads();
            // one wavefront per change t, lanes over the changes t'
#pragma unroll
            for (int u = 0; u < kPairPerWave; ++u) {
                const int t = wave + u * nwaves;
                if (t >= nch) break;   // the same in every lane of the wavefront
                const int abt = L.pab[t];
                const int at = abt & 0xffff, bt = abt >> 16;
                double wa = 0.0, wb = 0.0;
                if (lane < nch) {
                    const int ab2 = L.pab[lane];
                    const int a2 = ab2 & 0xffff, b2 = ab2 >> 16;
                    wa = (double)((b2 == at) - (a2 == at)) * kv[u];
                    wb = (double)((b2 == bt) - (a2 == bt)) * kv[u];
                }
                wa = wave_sum(wa);
                wb = wave_sum(wb);
                if (lane == 0) {
                    L.pwa[t] = wa;
                    L.pwb[t] = wb;
                }
            }
            __syncthreads();
            // (branch-free, eight changes per step with their reads issued first; a change that does
            // not touch cluster j adds and subtracts exact zeros, so the sum is the one in change order)
            for (int j = tid; j < C; j += nt) {
                double dt = 0.0;
                for (int t0 = 0; t0 < nch; t0 += 8) {
                    int ab[8];
                    double vb[8], va[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int t = min(t0 + u, nch - 1);
                        ab[u] = t0 + u < nch ? L.pab[t] : -1;
                        vb[u] = 2.0 * L.psb[t] + L.pwb[t];
                        va[u] = 2.0 * L.psa[t] + L.pwa[t];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        dt += (ab[u] >= 0 && (ab[u] >> 16) == j) ? vb[u] : 0.0;
                        dt -= (ab[u] >= 0 && (ab[u] & 0xffff) == j) ? va[u] : 0.0;
                    }
                }
                L.dT[j] = dt;
            }
            // (the next workgroup barrier orders these before the update below overwrites pab's source labels)
        }

        // own rows of S: from scratch (sort + segment sums, ~ell steps per row) only when the
        // incremental update (every own entry of S walks the changed list) would take longer
        if ((int64_t)nch * ((nr * C + nt - 1) / nt) > (int64_t)ell) {
            __syncthreads();
            for (int m = tid; m < ell; m += nt) L.lbl[m] = L.nlab[m];
            __syncthreads();
            csr_sort(L, ell, C);
            full_sums(L, Krows, ldk, nr, C);
        } else {
            // S[r][j] -= K(r, m) for changes leaving j, += for changes entering j, in index order.
            // The old and new labels of change t are packed (old | new << 16) into the CSR
            // permutation, which is stale until the next sort anyway.
            for (int t = tid; t < nch; t += nt) {
                const int m = L.chg[t];
                L.perm[t] = L.lbl[m] | (L.nlab[m] << 16);
            }
            __syncthreads();
            for (int p = tid; p < nr * C; p += nt) {
                const int r = p / C, j = p - r * C;
                const double* Kr = Krows + (int64_t)r * ldk;
                double sv = L.S[p];
                int t = 0;
                for (; t + 4 <= nch; t += 4) {
                    int ab[4];
                    double kv4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ab[u] = L.perm[t + u];
                        kv4[u] = Kr[L.chg[t + u]];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        sv = (ab[u] & 0xffff) == j ? sv - kv4[u] : sv;
                        sv = (ab[u] >> 16) == j ? sv + kv4[u] : sv;
                    }
                }
                for (; t < nch; ++t) {
                    const int ab = L.perm[t];
                    const double kx = Kr[L.chg[t]];
                    sv = (ab & 0xffff) == j ? sv - kx : sv;
                    sv = (ab >> 16) == j ? sv + kx : sv;
                }
                L.S[p] = sv;
            }
            for (int t = tid; t < nch; t += nt) {
                const int m = L.chg[t];
                atomicSub(L.cnt + L.lbl[m], 1);
                atomicAdd(L.cnt + L.nlab[m], 1);
            }
            __syncthreads();
            for (int t = tid; t < nch; t += nt) L.lbl[L.chg[t]] = L.nlab[L.chg[t]];
            __syncthreads();
        }
        if (pair) {
            for (int j = tid; j < C; j += nt) {
                const double cj = (double)L.cnt[j];
                const double T = L.T[j] + L.dT[j];
                L.T[j] = T;
                L.gh[j] = cj > 0.0 ? T / (cj * cj) : kInf;
                L.rcnt[j] = cj > 0.0 ? 1.0 / cj : 0.0;
            }
            __syncthreads();
        } else {
            exchange_T();
        }
        buf ^= 1;
        stamp(a, ns);
    }
    // Support rows: wavefront gw takes the landmarks m = gw + u GW (u < 2 per round; rows m in
    // [ell, ell + 32) are the zero padding for whole-tile loads, kept at position m).  The first 64
    // dimensions of its first landmark are loaded before the CSR sort of the final labels, which then
    // fixes each landmark's position k in the support.
    TI* sup = static_cast<TI*>(a.support);
    const int PD = (int)a.dpad;
    const int GW = G * nwaves, kend = ell + 32;
    const int mfirst = wg * nwaves + wave;
    const TI pre = (mfirst < ell && lane < a.d) ? row(L.lmv[mfirst])[lane] : TI(0);
    // CSR of the final labels for the support
    csr_sort(L, ell, C);
    stamp(a, ns);

    // 4. outputs: final labels, segments, g^, and the support of the final centroids
    for (int r = tid; r < nr; r += nt) a.lab_final[r0 + r] = L.lbl[r0 + r];
    stamp(a, ns);
    if (wg == 0) {
        for (int j = tid; j <= C; j += nt) a.offsets[j] = L.off[j];
        for (int j = tid; j < C; j += nt) {
            const int cnt = L.off[j + 1] - L.off[j];
            a.ghat[j] = cnt > 0 ? L.gh[j] : kInf;
            a.segabs[j] = cnt > 0 ? 1.0 : 0.0;
        }
        // contiguous cluster runs holding about a quarter of the support each (distance pass): split
        // q (q = 1, 2, 3) is the first cluster j <= C with off[j] >= ceil(ell q / 4), found by the one
        // thread j where the offsets cross it (they ascend)
        if (tid == 0) {
            a.split[0] = 0;
            a.split[4] = C;
        }
        for (int j = tid; j <= C; j += nt) {
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                const int want = (ell * q + 3) / 4;
                if ((j == C || L.off[j] >= want) && (j == 0 || L.off[j - 1] < want)) a.split[q] = j;
            }
        }
        if (tid == 0) *a.updates_out = it;
        for (int m = tid; m < ell; m += nt) a.lab[ell + m] = L.lbl[m];   // final landmark labels
    }
    // support rows (one wavefront per row, lanes over the dimensions; two rows at a time): row copy,
    // FP32 / bfloat16 panels, norms
    const bool panels = a.ktype != KKM_KERNEL_RMSD;   // power-of-two padded rows only
    // RMSD frames: the matrix-core cross-covariance panel (float frames, even atom count)
    const bool rpanel = !panels && a.sup_pan && (a.n_atoms % 2) == 0;
    const int rsteps = a.n_atoms / 2;
    float nmax = 0.0f;
    for (int m0 = mfirst; m0 < kend; m0 += 2 * GW) {
        const bool first = m0 == mfirst;
        const TI* srcq[2];
        int kq[2], cntq[2], posq[2];
        bool realq[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int m = m0 + u * GW;
            realq[u] = m < ell;
            kq[u] = m;   // padding rows keep their index
            cntq[u] = 1;
            posq[u] = 0;
            if (realq[u]) {
                const int j = L.lbl[m];
                kq[u] = L.off[j] + L.chunk[(m >> 6) * C + j] + L.rank[m];   // CSR position
                cntq[u] = L.off[j + 1] - L.off[j];
                posq[u] = L.lmv[m];
            }
            srcq[u] = row(posq[u]);
        }
        double n64[2] = {0.0, 0.0};
        float n32[2] = {0.0f, 0.0f};
        auto emit = [&](int c, const TI (&val)[2]) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = kq[u];
                if (m0 + u * GW >= kend) continue;   // uniform over the wavefront
                sup[(int64_t)k * PD + c] = val[u];
                n64[u] = fma((double)val[u], (double)val[u], n64[u]);
                const float f = (float)val[u];
                n32[u] = fmaf(f, f, n32[u]);
                if (panels && a.sup_pan) a.sup_pan[panel32_index(k, c, PD)] = f;
                if (rpanel && c < a.d) a.sup_pan[rmsd_panel_index(k, c / 3, c % 3, rsteps)] = f;
                if (panels && PD >= 16) {
                    uint16_t hi = 0, lo = 0;
                    if (realq[u] && c < a.d) bf16_split(f, hi, lo);
                    a.sup_hi[panel16_index(k, c, PD)] = hi;
                    a.sup_lo[panel16_index(k, c, PD)] = lo;
                }
            }
        };
        {
            const int c = lane;
            TI val[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                val[u] = (first && u == 0) ? pre : ((realq[u] && c < a.d) ? srcq[u][c] : TI(0));
            if (c < PD) emit(c, val);
        }
        for (int c = lane + 64; c < PD; c += 64) {
            TI val[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) val[u] = (realq[u] && c < a.d) ? srcq[u][c] : TI(0);
            emit(c, val);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (m0 + u * GW >= kend) continue;   // uniform over the wavefront
            const int k = kq[u];
            const double s64 = wave_sum(n64[u]);
            const float s32 = wave_sum(n32[u]);
            if (lane == 0) {
                a.snorm64[k] = s64;
                a.snorm32[k] = s32;
                a.coef64[k] = realq[u] ? 1.0 / (double)cntq[u] : 0.0;
                a.coef32[k] = realq[u] ? (float)(1.0 / (double)cntq[u]) : 0.0f;
                if (realq[u]) a.src_index[k] = posq[u];
            }
            nmax = fmaxf(nmax, s32);
        }
    }
    // one atomic per workgroup for the largest squared norm (non-negative floats order as integers)
    if (lane == 0) L.red[wave] = (double)nmax;
    __syncthreads();
    if (tid == 0) {
        float mx = 0.0f;
        for (int w = 0; w < nwaves; ++w) mx = fmaxf(mx, (float)L.red[w]);
        if (mx > 0.0f) atomicMax(reinterpret_cast<unsigned int*>(a.snorm_max), __float_as_uint(mx));
    }
    stamp(a, ns);
}

}  // namespace

size_t landmark_lds_bytes_host(int ell, int C, int G, bool k_in_lds) {
    const int R = (ell + G - 1) / G;
    return landmark_lds_bytes(ell, C, R, k_in_lds);
}

LandmarkShape landmark_shape(const DeviceInfo& dev, int ell, int C) {
    // at least 4 landmark rows per workgroup and at most KKM_LANDMARK_WGS workgroups (default 64):
    // the loop is bound by its cross-workgroup waits, whose cost grows with the grid; the grid is widened
    // (up to the device) when that lets the own rows of K_LL stay in LDS
    static int cap = [] {
        const char* e = std::getenv("KKM_LANDMARK_WGS");
        const int v = e ? std::atoi(e) : 0;
        return v > 0 ? v : 64;
    }();
    static const bool k_lds_allowed = [] {
        const char* e = std::getenv("KKM_LANDMARK_K_IN_LDS");
        return !(e && e[0] == '0');
    }();
    const int gmax = std::max(1, std::min(dev.num_cus, ell));
    const int G0 = std::max(1, std::min((ell + 3) / 4, std::min(cap, gmax)));
    auto widen = [&](bool k_in_lds) {
        for (int G = G0; G <= gmax; G = G < gmax ? std::min(gmax, G + std::max(1, G / 8)) : gmax + 1)
            if (landmark_lds_bytes_host(ell, C, G, k_in_lds) <= dev.max_lds_per_block) return G;
        return 0;
    };
    if (k_lds_allowed)
        if (const int G = widen(true)) return LandmarkShape{G, 1};
    // K_LL rows from HBM: the per-row parts of the LDS still shrink with a wider grid
    const int G = widen(false);
    return LandmarkShape{G ? G : G0, 0};
}

static kkm_status check_landmark_args(const LandmarkArgs& args, const DeviceInfo& dev, size_t* lds_out) {
    if (args.ldk != k_ld(args.ell)) return fail(KKM_ERR_INTERNAL, "landmark block stride");
    const size_t lds = landmark_lds_bytes_host(args.ell, args.C, args.grid, args.k_in_lds != 0);
    if (lds > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "landmark set too large for one workgroup's LDS (l=" +
                                             std::to_string(args.ell) + ", C=" + std::to_string(args.C) +
                                             "); use more mini-batches");
    if (sizeof(double) * 64 * (size_t)args.d > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "sample dimension too large");
    *lds_out = lds;
    return KKM_OK;
}

int landmark_init_parts(const LandmarkArgs& a) {
    const int dp = eval_dp(a.ktype, a.d);
    if (dp == 0 || !a.init_mode) return 0;   // (RMSD: landmark_init_kernel; given labels)
    const int T = dp >= 8 ? 32 : 64;         // the block kernel's tile (launch_landmark_block)
    return a.C > T ? (a.C + T - 1) / T : 0;
}

kkm_status launch_landmark_block(const LandmarkArgs& args, int dtype, const DeviceInfo& dev, hipStream_t stream) {
    size_t lds = 0;
    KKM_TRY(check_landmark_args(args, dev, &lds));
    const size_t lds_tile = sizeof(double) * 64 * (size_t)args.d;
    const size_t lds_row = sizeof(double) * (size_t)args.d;
    return dispatch_dp(eval_dp(args.ktype, args.d), [&]<int DP>() -> kkm_status {
        if constexpr (DP > 0) {
            // 32 x 32 tiles (four times the workgroups of 64 x 64, so more of them overlap their row
            // gathers); 64 x 64 for rows of 4 dimensions, where a 32-row stage would not fill the block
            constexpr int T = DP >= 8 ? 32 : 64;
            // columns: the landmarks, then (from the next tile boundary) the medoids
            const int ncol = args.init_mode ? (args.ell + T - 1) / T * T + args.C : args.ell;
            const dim3 kgrid((unsigned)((ncol + T - 1) / T), (unsigned)((args.ell + T - 1) / T));
            const bool lin = args.ktype == KKM_KERNEL_LINEAR;
            if (dtype == KKM_F64) {
                if (lin) hipLaunchKernelGGL((landmark_k_kernel<double, DP, true, T>), kgrid, dim3(256), 0, stream, args);
                else hipLaunchKernelGGL((landmark_k_kernel<double, DP, false, T>), kgrid, dim3(256), 0, stream, args);
            } else {
                if (lin) hipLaunchKernelGGL((landmark_k_kernel<float, DP, true, T>), kgrid, dim3(256), 0, stream, args);
                else hipLaunchKernelGGL((landmark_k_kernel<float, DP, false, T>), kgrid, dim3(256), 0, stream, args);
            }
            // (the block kernel takes the initial labels itself, or leaves per-tile minima for the loop)
            if (args.init_mode && args.C > T && args.init_parts != (args.C + T - 1) / T)
                return fail(KKM_ERR_INTERNAL, "Eq. 8 tile minima: init_parts does not match the tiles");
        } else {
            const int tiles = (args.ell + 31) / 32;
            const dim3 bgrid((unsigned)tiles, (unsigned)tiles);
            if (dtype == KKM_F64) {
                hipLaunchKernelGGL(landmark_block_kernel<double>, bgrid, dim3(256), lds_tile, stream, args, tiles);
                KKM_HIP(hipGetLastError());
                hipLaunchKernelGGL((landmark_init_kernel<double, DP>), dim3(args.ell), dim3(256), lds_row, stream, args);
            } else {
                hipLaunchKernelGGL(landmark_block_kernel<float>, bgrid, dim3(256), lds_tile, stream, args, tiles);
                KKM_HIP(hipGetLastError());
                hipLaunchKernelGGL((landmark_init_kernel<float, DP>), dim3(args.ell), dim3(256), lds_row, stream, args);
            }
        }
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    });
}

kkm_status launch_landmark_loop(const LandmarkArgs& args, int dtype, const DeviceInfo& dev, hipStream_t stream) {
    size_t lds = 0;
    KKM_TRY(check_landmark_args(args, dev, &lds));
    const int G = args.grid;
    LandmarkArgs a = args;
    void* params[] = {&a};
    const bool kl = args.k_in_lds != 0;
    const void* fn = dtype == KKM_F64
                         ? (kl ? reinterpret_cast<const void*>(&landmark_phase_kernel<double, true>)
                               : reinterpret_cast<const void*>(&landmark_phase_kernel<double, false>))
                         : (kl ? reinterpret_cast<const void*>(&landmark_phase_kernel<float, true>)
                               : reinterpret_cast<const void*>(&landmark_phase_kernel<float, false>));
    KKM_TRY(allow_dynamic_lds(fn, lds));
    int per_cu = 0;
    KKM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kLoopThreads, lds));
    if (per_cu * dev.num_cus < G)
        return fail(KKM_ERR_DEVICE, "landmark loop grid does not fit co-resident on the device");
    // The grid fits the device at once, so a plain launch makes every workgroup resident as soon as
    // the CUs are free (work of other streams only delays the exchanges; their waits are bounded and
    // report an error).  A cooperative launch gives the same guarantee formally but costs ~20 us of
    // queue synchronisation per launch; KKM_LANDMARK_COOPERATIVE=1 selects it.
    static const bool coop = [] {
        const char* e = std::getenv("KKM_LANDMARK_COOPERATIVE");
        return e && e[0] == '1';
    }();
    if (coop || args.cooperative)
        KKM_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(kLoopThreads), params, (unsigned)lds, stream));
    else KKM_HIP(hipLaunchKernel(fn, dim3(G), dim3(kLoopThreads), params, (unsigned)lds, stream));
    return KKM_OK;
}

}  // namespace kkm
