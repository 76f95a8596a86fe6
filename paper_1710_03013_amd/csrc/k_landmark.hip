// Landmark phase of one mini-batch, as one cooperative kernel:
//
//   1. the landmark kernel block K_LL = K(x_l, x_m), FP64, each workgroup its own rows;
//   2. the initial landmark labels: given, or the nearest global medoid (Eq. 8, with K(m,m));
//   3. the landmark loop (Eq. 14-17 restricted to the landmarks):
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
// order, then workgroup order), so results are bitwise repeatable.  Cross-workgroup data is
// published with a release fence before the grid barrier and read with agent-scope atomic loads.
#include <hip/hip_cooperative_groups.h>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace cg = cooperative_groups;

namespace kkm {

namespace {

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LdsLayout {
    int32_t* lbl;      // [ell]
    int32_t* perm;     // [ell]
    int32_t* off;      // [C+1]
    uint8_t* rank;     // [ell] rank within its 64-landmark chunk among equal labels
    uint16_t* chunk;   // [nchunks][C] count, then base, per chunk and label
    double* S;         // [R][C]
    double* gh;        // [C]
    double* kself;     // [R]
};

__device__ __forceinline__ size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t landmark_lds_bytes(int ell, int C, int R) {
    const int nchunks = (ell + 63) / 64;
    size_t b = 0;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * ell;
    b = (b + 15) & ~size_t(15); b += sizeof(int32_t) * (C + 1);
    b = (b + 15) & ~size_t(15); b += ell;
    b = (b + 15) & ~size_t(15); b += sizeof(uint16_t) * (size_t)nchunks * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * (size_t)R * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * C;
    b = (b + 15) & ~size_t(15); b += sizeof(double) * R;
    return (b + 15) & ~size_t(15);
}

__device__ LdsLayout carve_lds(unsigned char* base, int ell, int C, int R) {
    const int nchunks = (ell + 63) / 64;
    LdsLayout L;
    size_t b = 0;
    b = al16(b); L.lbl = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.perm = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * ell;
    b = al16(b); L.off = reinterpret_cast<int32_t*>(base + b); b += sizeof(int32_t) * (C + 1);
    b = al16(b); L.rank = reinterpret_cast<uint8_t*>(base + b); b += ell;
    b = al16(b); L.chunk = reinterpret_cast<uint16_t*>(base + b); b += sizeof(uint16_t) * (size_t)nchunks * C;
    b = al16(b); L.S = reinterpret_cast<double*>(base + b); b += sizeof(double) * (size_t)R * C;
    b = al16(b); L.gh = reinterpret_cast<double*>(base + b); b += sizeof(double) * C;
    b = al16(b); L.kself = reinterpret_cast<double*>(base + b);
    return L;
}

// Stable counting sort of the ell labels in L.lbl into L.perm / L.off (whole workgroup).
__device__ void csr_sort(const LdsLayout& L, int ell, int C) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int nchunks = (ell + 63) / 64;
    for (int i = tid; i < nchunks * C; i += nt) L.chunk[i] = 0;
    __syncthreads();
    // ranks inside each 64-landmark chunk, one distinct label at a time
    for (int ch = wave; ch < nchunks; ch += nwaves) {
        const int m = ch * 64 + lane;
        const bool valid = m < ell;
        const int lab = valid ? L.lbl[m] : -1;
        uint64_t remaining = __ballot(valid);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        while (remaining) {
            const int leader = __ffsll((unsigned long long)remaining) - 1;
            const int cur = __shfl(lab, leader, 64);
            const uint64_t mask = __ballot(valid && lab == cur);
            if (valid && lab == cur) L.rank[m] = (uint8_t)__popcll(mask & below);
            if (lane == 0) L.chunk[ch * C + cur] = (uint16_t)__popcll(mask);
            remaining &= ~mask;
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
    // exclusive scan of the counts into the segment offsets (first wave)
    if (wave == 0) {
        int carry = 0;
        for (int base = 0; base < C; base += 64) {
            const int j = base + lane;
            int v = (j < C) ? L.off[j + 1] : 0;
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(v, o, 64);
                if (lane >= o) v += t;
            }
            if (j < C) L.off[j + 1] = carry + v;
            carry += __shfl(v, 63, 64);
        }
        if (lane == 0) L.off[0] = 0;
    }
    __syncthreads();
    for (int m = tid; m < ell; m += nt) {
        const int lab = L.lbl[m];
        L.perm[L.off[lab] + L.chunk[(m >> 6) * C + lab] + L.rank[m]] = m;
    }
    __syncthreads();
}

template <typename TI>
__global__ __launch_bounds__(256) void landmark_phase_kernel(LandmarkArgs a) {
    cg::grid_group grid = cg::this_grid();
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int wg = blockIdx.x, G = gridDim.x;
    const int ell = a.ell, C = a.C;
    const int R = (ell + G - 1) / G;
    const int r0 = min(ell, wg * R), r1 = min(ell, r0 + R), nr = r1 - r0;
    LdsLayout L = carve_lds(smem, ell, C, R);
    const TI* X = static_cast<const TI*>(a.X);
    const KSpec ks{a.ktype, a.n_atoms, a.d, a.inv2s2};
    auto row = [&](int pos) { return X + (a.base + (int64_t)pos * a.stride) * a.d; };

    if (wg == 0) {
        for (int i = tid; i <= a.max_updates; i += nt) a.changed[i] = 0;
        for (int i = tid; i < a.n_zero_ints; i += nt) a.zero_ints[i] = 0;
        if (tid == 0) *reinterpret_cast<unsigned int*>(a.snorm_max) = 0u;
    }

    // 1. own rows of the landmark block
    for (int64_t idx = tid; idx < (int64_t)nr * ell; idx += nt) {
        const int r = (int)(idx / ell), c = (int)(idx % ell);
        a.Kbuf[(int64_t)(r0 + r) * ell + c] = k64(ks, row(a.lm[r0 + r]), row(a.lm[c]));
    }
    for (int r = tid; r < nr; r += nt) L.kself[r] = kself64(ks, row(a.lm[r0 + r]));

    // 2. initial labels of own rows
    for (int r = tid; r < nr; r += nt) {
        int lab = 0;
        if (a.init_mode == 0) {
            lab = a.lab_init[r0 + r];
        } else {
            const TI* x = row(a.lm[r0 + r]);
            const TI* M = static_cast<const TI*>(a.M);
            const double kxx = L.kself[r];
            double best = kInf;
            for (int j = 0; j < C; ++j) {
                const double ms = a.Mself[j];
                if (!(ms < kInf)) continue;
                const double dj = kxx - 2.0 * k64(ks, x, M + (int64_t)j * a.Mpad) + ms;
                if (dj < best) { best = dj; lab = j; }
            }
        }
        a.lab[r0 + r] = lab;
    }
    __threadfence();
    grid.sync();

    // 3. the landmark loop
    int cur = 0, it = 0;
    for (;;) {
        const int32_t* labc = a.lab + (int64_t)cur * ell;
        for (int i = tid; i < ell; i += nt) L.lbl[i] = ld_agent(labc + i);
        __syncthreads();
        csr_sort(L, ell, C);

        // S[r][j] for own rows: short segments one lane each, long ones a whole wave
        for (int r = wave; r < nr; r += nwaves) {
            const double* Krow = a.Kbuf + (int64_t)(r0 + r) * ell;
            for (int j = lane; j < C; j += 64) {
                const int lo = L.off[j], hi = L.off[j + 1];
                if (hi - lo < 64) {
                    double s = 0.0;
                    for (int k = lo; k < hi; ++k) s += Krow[L.perm[k]];
                    L.S[r * C + j] = s;
                }
            }
            for (int j = 0; j < C; ++j) {
                const int lo = L.off[j], hi = L.off[j + 1];
                if (hi - lo >= 64) {
                    double s = 0.0;
                    for (int k = lo + lane; k < hi; k += 64) s += Krow[L.perm[k]];
                    s = wave_sum(s);
                    if (lane == 0) L.S[r * C + j] = s;
                }
            }
        }
        __syncthreads();
        // partial g^ of this workgroup, own rows in order
        for (int j = tid; j < C; j += nt) {
            double acc = 0.0;
            for (int r = 0; r < nr; ++r)
                if (L.lbl[r0 + r] == j) acc += L.S[r * C + j];
            a.partial[(int64_t)wg * C + j] = acc;
        }
        __threadfence();
        grid.sync();
        for (int j = tid; j < C; j += nt) {
            double acc = 0.0;
            for (int g = 0; g < G; ++g) acc += ld_agent(a.partial + (int64_t)g * C + j);
            const double cj = (double)(L.off[j + 1] - L.off[j]);
            L.gh[j] = cj > 0.0 ? acc / (cj * cj) : kInf;
        }
        __syncthreads();
        if (it >= a.max_updates) break;

        // Eq. 15 on own rows
        int32_t* labn = a.lab + (int64_t)(1 - cur) * ell;
        for (int r = tid; r < nr; r += nt) {
            double best = kInf;
            int bj = L.lbl[r0 + r];
            bool found = false;
            for (int j = 0; j < C; ++j) {
                const int cnt = L.off[j + 1] - L.off[j];
                if (cnt == 0) continue;
                const double dj = L.kself[r] - 2.0 * L.S[r * C + j] / (double)cnt + L.gh[j];
                if (!found || dj < best) { best = dj; bj = j; found = true; }
            }
            labn[r0 + r] = bj;
            if (bj != L.lbl[r0 + r]) atomicAdd(a.changed + it, 1);
        }
        __threadfence();
        grid.sync();
        ++it;
        if (ld_agent(a.changed + (it - 1)) == 0) break;
        cur = 1 - cur;
    }

    // 4. outputs: final labels, segments, g^, and the support of the final centroids
    for (int r = tid; r < nr; r += nt) a.lab_final[r0 + r] = L.lbl[r0 + r];
    if (wg == 0) {
        for (int j = tid; j <= C; j += nt) a.offsets[j] = L.off[j];
        for (int j = tid; j < C; j += nt) {
            const int cnt = L.off[j + 1] - L.off[j];
            a.ghat[j] = cnt > 0 ? L.gh[j] : kInf;
            a.segabs[j] = cnt > 0 ? 1.0 : 0.0;
        }
        if (tid == 0) *a.updates_out = it;
    }
    TI* sup = static_cast<TI*>(a.support);
    for (int k = wg * nt + tid; k < ell; k += G * nt) {
        const int m = L.perm[k];
        const int j = L.lbl[m];
        const int cnt = L.off[j + 1] - L.off[j];
        const TI* src = row(a.lm[m]);
        TI* dst = sup + (int64_t)k * a.dpad;
        double n64 = 0.0;
        for (int64_t c = 0; c < a.dpad; ++c) {
            const TI v = c < a.d ? src[c] : TI(0);
            dst[c] = v;
            n64 = fma((double)v, (double)v, n64);
        }
        float n32 = 0.0f;
        for (int64_t c = 0; c < a.d; ++c) n32 = fmaf((float)src[c], (float)src[c], n32);
        a.snorm64[k] = n64;
        a.snorm32[k] = n32;
        a.coef64[k] = 1.0 / (double)cnt;
        a.coef32[k] = (float)(1.0 / (double)cnt);
        a.src_index[k] = a.lm[m];
        atomicMax(reinterpret_cast<unsigned int*>(a.snorm_max), __float_as_uint(n32));
    }
}

}  // namespace

size_t landmark_lds_bytes_host(int ell, int C, int G) {
    const int R = (ell + G - 1) / G;
    return landmark_lds_bytes(ell, C, R);
}

int landmark_grid(const DeviceInfo& dev, int ell) {
    int G = (ell + 3) / 4;
    if (G > dev.num_cus) G = dev.num_cus;
    if (G < 1) G = 1;
    return G;
}

kkm_status launch_landmark_phase(const LandmarkArgs& args, int dtype, const DeviceInfo& dev, hipStream_t stream) {
    const int G = args.grid;
    const size_t lds = landmark_lds_bytes_host(args.ell, args.C, G);
    if (lds > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "landmark set too large for one workgroup's LDS (l=" +
                                             std::to_string(args.ell) + ", C=" + std::to_string(args.C) +
                                             "); use more mini-batches");
    LandmarkArgs a = args;
    void* params[] = {&a};
    const void* fn = dtype == KKM_F64 ? reinterpret_cast<const void*>(&landmark_phase_kernel<double>)
                                      : reinterpret_cast<const void*>(&landmark_phase_kernel<float>);
    if (lds > 65536) KKM_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    KKM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds));
    if (per_cu * dev.num_cus < G)
        return fail(KKM_ERR_DEVICE, "landmark loop grid does not fit co-resident on the device");
    KKM_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(256), params, (unsigned)lds, stream));
    return KKM_OK;
}

}  // namespace kkm
