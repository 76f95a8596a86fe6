// Distances to sparse centroids with the dot products on the matrix cores (linear / RBF kernels):
//
//   d(x, j) = K(x,x) - 2 sum_{l in segment j} a_l K(x, s_l) + self_j,
//   K(x, s) = x.s (linear) or exp(-(||x||^2 + ||s||^2 - 2 x.s) / (2 sigma^2)) (RBF).
//
// A workgroup owns 32 samples (the N dimension of a 32x32 MFMA tile); the support is cut into four
// cluster-aligned quarters walked in 32-row tiles (the M dimension) aligned to multiples of 32.  With
// four wavefronts each walks one quarter; with eight, wavefronts w and w + 4 take the first and the
// second half of quarter w's tiles, each summing into its own copy of the per-cluster sums, which
// are added (first half + second half) before the decision: twice the wavefronts, half the chain
// of dependent tiles each.  The two lane halves take contiguous halves of the dimensions as their share of
// the K index (any order of K gives the same dot product); the support is read from its panel
// layout, in which each step's fragment is 64 consecutive vectors.  Result lane l holds rows 8(i/4) + 4(l/32) + i%4 of sample l%32 (i = 0..15): the kernel
// function is applied in registers, and each segment's sum is a masked sum over the lane's 16
// values plus one exchange with the partner lane l^32, accumulated in the order of the tiles.
//
// Precision: FP32 (v_mfma_f32_32x32x2_f32); BF16 -- x.s ~ hi.hi' with hi = bfloat16(x), one
// v_mfma_f32_32x32x16_bf16 per 16 dimensions, FP32 accumulation; or BF16x3 -- x = hi + lo with hi,
// lo in bfloat16 and x.s ~ hi.hi' + hi.lo' + lo.hi' (three products).  Every form carries a per-row
// error bound, and rows whose margin is under it are decided again in FP64 (launch_refine): BF16 is
// the cheap pass that gates that refinement.
//
// Error of the bfloat16 forms (u = 2^-8, the unit roundoff of bfloat16 with round-to-nearest-even;
// hi = RNE(x), lo = RNE(x - hi), r = x - hi - lo):  |x - hi| <= u|x|, |hi| <= (1 + u)|x|,
// |lo| <= u(1 + u)|x|, |r| <= u|x - hi| <= u^2|x|.
//   BF16:   x.y - hi.hi' = (x - hi) y + hi (y - hi'), so per product |.| <= u(2 + u)|x||y|.
//   BF16x3: x.y - (hi.hi' + hi.lo' + lo.hi') = lo.lo' + hi.r' + r.hi' + lo.r' + r.lo' + r.r', each
//           term bounded by the facts above: in all <= u^2 (3 + 6u)|x||y| <= 3 u^2 (1 + 2^-7)|x||y|.
// Summed over the dimensions this is at most the constant times sum_k |x_k||y_k| <= ||x|| ||y||.  The
// bfloat16 products are exact in FP32; their FP32 accumulation adds the (P DP + 2) u32 terms
// (P = products per dimension).  Inputs below 2^-118 in magnitude (bfloat16 subnormal remainders) are
// outside these relative bounds.
#include <cstdlib>

#include <type_traits>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kU32 = 5.9604645e-8f;     // unit roundoff of float
constexpr float kUbf1 = 7.8277588e-3f;    // BF16:   u (2 + u) = 2^-7 (1 + 2^-9), u = 2^-8
constexpr float kUbf3 = 4.6134e-5f;       // BF16x3: 3 u^2 (1 + 2^-7) = 3 * 2^-16 * (1 + 2^-7), rounded up

// precision modes of the pass (kPmRmsd: RMSD frames, FP32 cross-covariance and FP64 eigenvalue)
constexpr int kPmF32 = 0, kPmBf16 = 1, kPmBf16x3 = 3, kPmRmsd = 4;

// (e2s = log2(e) / (2 sigma^2) rounded to float, so the exponent takes one product: its two roundings,
// the constant's and the product's, are those of d2 / (2 sigma^2) times log2(e))
__device__ __forceinline__ float rbf_or_dot(int type, float dot, float qn, float sn, float e2s) {
    if (type == KKM_KERNEL_LINEAR) return dot;
    float d2 = qn + sn - 2.0f * dot;
    d2 = d2 > 0.0f ? d2 : 0.0f;
    return __builtin_amdgcn_exp2f(-d2 * e2s);
}

// x.s for the 32 support rows of panel tile `tile` and the wavefront's 32 samples: lane l ends up with
// rows 8(i/4) + 4(l/32) + i%4 of sample l%32 in acc[i].  xq: the lane half's dimensions of its sample
// (FP32), bh / bl: their bfloat16 split (BF16 forms).
template <int DP, int PM>
__device__ __forceinline__ floatx16 mfma_tile(const SupportView& sup, int64_t tile, int lane, const float* xq,
                                              const bf16x8* bh, const bf16x8* bl) {
    constexpr int H = DP / 2;
    floatx16 acc = {};
    if constexpr (PM == kPmBf16) {
        const bf16x8* ah = reinterpret_cast<const bf16x8*>(sup.hi) + tile * (H / 8) * 64 + lane;
        bf16x8 xh[H / 8];
#pragma unroll
        for (int v = 0; v < H / 8; ++v) xh[v] = ah[v * 64];
#pragma unroll
        for (int v = 0; v < H / 8; ++v) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[v], bh[v], acc, 0, 0, 0);
    } else if constexpr (PM == kPmBf16x3) {
        const bf16x8* ah = reinterpret_cast<const bf16x8*>(sup.hi) + tile * (H / 8) * 64 + lane;
        const bf16x8* al = reinterpret_cast<const bf16x8*>(sup.lo) + tile * (H / 8) * 64 + lane;
        bf16x8 xh[H / 8], xl[H / 8];
#pragma unroll
        for (int v = 0; v < H / 8; ++v) {
            xh[v] = ah[v * 64];
            xl[v] = al[v * 64];
        }
#pragma unroll
        for (int v = 0; v < H / 8; ++v) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[v], bh[v], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[v], bl[v], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[v], bh[v], acc, 0, 0, 0);
        }
    } else {
        constexpr int VW = H < 4 ? H : 4;
        const float* pb = sup.pan + (tile * (H / VW) * 64 + lane) * VW;
        float af[H];
#pragma unroll
        for (int g = 0; g < H / VW; ++g) {
            if constexpr (VW == 4) {
                const float4 t = *reinterpret_cast<const float4*>(pb + g * 64 * VW);
                af[4 * g] = t.x;
                af[4 * g + 1] = t.y;
                af[4 * g + 2] = t.z;
                af[4 * g + 3] = t.w;
            } else {
                const float2 t = *reinterpret_cast<const float2*>(pb + g * 64 * VW);
                af[2 * g] = t.x;
                af[2 * g + 1] = t.y;
            }
        }
#pragma unroll
        for (int s = 0; s < H; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[s], xq[s], acc, 0, 0, 0);
    }
    return acc;
}

// The lane half's dimensions of sample row xr (zero past d).
template <typename TI, int DP>
__device__ __forceinline__ void load_query_rows(const TI* xr, int64_t d, bool vec_ok, int h, float* xq) {
    constexpr int H = DP / 2;
    const bool xvec = H % 4 == 0 && d == DP && vec_ok;
    if (xvec) {
        const float4* x4 = reinterpret_cast<const float4*>(xr + h * H);
#pragma unroll
        for (int v = 0; v < H / 4; ++v) {
            const float4 t = x4[v];
            xq[4 * v] = t.x;
            xq[4 * v + 1] = t.y;
            xq[4 * v + 2] = t.z;
            xq[4 * v + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int dim = h * H + s;
            xq[s] = dim < d ? (float)xr[dim] : 0.0f;
        }
    }
}

// The squared norm of the sample over both lane halves, the finiteness of the lane's part, and the
// bfloat16 split for the BF16 forms.
template <int DP, int PM>
__device__ __forceinline__ float finish_query(const float* xq, bf16x8* bh, bf16x8* bl, bool& ok) {
    constexpr int H = DP / 2;
    float qn = 0.0f;
    ok = true;
#pragma unroll
    for (int s = 0; s < H; ++s) {
        ok = ok && isfinite(xq[s]);
        qn = fmaf(xq[s], xq[s], qn);
    }
    qn += __shfl_xor(qn, 32, 64);
    if constexpr (PM != kPmF32) {
#pragma unroll
        for (int v = 0; v < H / 8; ++v)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float x = xq[8 * v + t];
                const __bf16 hi = (__bf16)x;
                bh[v][t] = hi;
                if constexpr (PM == kPmBf16x3) bl[v][t] = (__bf16)(x - (float)hi);
            }
    }
    return qn;
}

template <typename TI, int DP, int PM>
__device__ __forceinline__ float load_query(const TI* xr, int64_t d, bool vec_ok, int h, float* xq, bf16x8* bh,
                                            bf16x8* bl, bool& ok) {
    load_query_rows<TI, DP>(xr, d, vec_ok, h, xq);
    return finish_query<DP, PM>(xq, bh, bl, ok);
}

// ----------------------------------------------------------------------------- RMSD frames
// The superposition of two centred frames needs their 3x3 correlation R = sum_a x_a s_a^T: nine dot
// products over the atoms, i.e. nine GEMM planes for a tile of query and support frames.  They run on
// v_mfma_f32_16x16x4f32, four atoms per step (the A operand a support coordinate, the B operand a
// query coordinate); per pair the squared RMSD then comes from the largest eigenvalue of the 4x4 key
// matrix of R in FP64 (Laguerre's method, Jacobi rotations where it does not settle), r^2 =
// max(0, (G_x + G_s - 2 lambda) / A).
//
// Error: the FP32 accumulation of the A products of each entry (in any order) gives |dR_pq| <=
// (A + 2) u32 sum_a |x_ap||s_aq| <= (A + 2) u32 sqrt(G_xp G_sq), so ||dR||_F <= (A + 2) u32
// sqrt(G_x G_s); the key matrix is linear in R with ||N(dR)||_F = 2 ||dR||_F, so (Weyl) |d lambda| <=
// 2 (A + 2) u32 sqrt(G_x G_s), and r^2 moves by at most 4 (A + 2) u32 sqrt(G_x G_s) / A, plus the FP64
// solve (accepted within kPairSolveTol (G_x + G_s) / A) and the float rounding of r^2.  The frames
// themselves are the centred float rows that the FP64 re-decision reads too.
constexpr double kPairSolveTol = 1e-10;

// Bound on |r^2 computed - exact| for a query of norm Gq against supports of norm at most Gs (above).
__device__ __forceinline__ float rmsd_r2_bound(float Gq, float Gs, int A) {
    return (4.0f * (A + 2) * kU32 * sqrtf(Gq * Gs) * 1.0001f + (kU32 + (float)kPairSolveTol) * (Gq + Gs)) / (float)A;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// The pair pass: every squared RMSD of a chunk of query groups against the whole support, at full
// occupancy (its registers hold four pairs per lane), written in the lane layout of a 32 x 32
// accumulator tile so that the distance passes read it back lane for lane:
//   r2[((g - g0) * ntiles + t) * 1024 + i * 64 + l]  is the pair (support row 32 t + 8(i/4) + 4(l/32)
//   + i%4, query 32 g + l%32),
// and gq[(g - g0) * 32 + c] holds G of query 32 g + c in FP64 (0 past the last row).  Workgroup
// (g - g0, y) stages the 32 frames of group g in LDS and takes support tiles y T .. y T + T - 1 (T =
// tiles_per_block, so the staging serves T tiles); on each its wavefront w takes the 16 x 16 block of
// support half w/2 and query half w%2, nine accumulators of four values each.
struct RmsdPairsArgs {
    BatchView q;           // centred float frames
    const float* pan;      // support panel (rmsd_panel_index)
    const double* snorm64; // G of each support row
    int32_t A;
    int64_t g0;
    int32_t ntiles;
    int32_t tiles_per_block;
    float* r2;
    double* gq;
    int32_t* nonfinite;
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void rmsd_pairs_kernel(RmsdPairsArgs p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int A = p.A, nst = (A + 3) / 4, nsteps2 = A / 2;
    // value ((t * 3 + c) * 2 + qh) * 64 + l: coordinate c of atom 4t + l/16 of query 16 qh + l%16
    float* xs = reinterpret_cast<float*>(smem_raw);
    __shared__ double gpart[4][64];
    __shared__ double gqs[32];
    const int64_t g = p.g0 + blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float* X = static_cast<const float*>(p.q.X);
    int bad = 0;
    {   // wavefront w fills the rows w, w + 4, ... of 64 values (row (t * 3 + c) * 2 + qh): its query half
        // qh = w % 2 is fixed, so each lane reads one frame, query 16 qh + l%16, throughout
        const int64_t qq = g * 32 + 16 * (wave & 1) + (lane & 15);
        const bool qok = qq < p.q.n;
        const float* row = X + (p.q.base + (qok ? qq : 0) * p.q.stride) * p.q.d;
        const int a4 = lane >> 4;
        int t = 0, c = wave >> 1;   // t * 3 + c advances by 2 per row taken
        for (int r = wave; r < nst * 6; r += 4) {
            const int atom = 4 * t + a4;
            float v = 0.0f;
            if (qok && atom < A) {
                v = row[3 * atom + c];
                bad |= !isfinite(v);
            }
            xs[r * 64 + lane] = v;
            c += 2;
            if (c >= 3) {
                c -= 3;
                ++t;
            }
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0 && blockIdx.y == 0) atomicOr(p.nonfinite, 1);
    {   // G of each query in FP64: the wavefronts split the steps, lane l takes query l%32 and
        // (lane half) atoms 4t + {0,1} or {2,3}
        const int qc = lane & 31, hf = lane >> 5, nw = blockDim.x >> 6;
        double gs = 0.0;
        for (int t = wave; t < nst; t += nw)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const double v = xs[((t * 3 + c) * 2 + (qc >> 4)) * 64 + (2 * hf + k) * 16 + (qc & 15)];
                    gs = fma(v, v, gs);
                }
        gpart[wave][lane] = gs;
        __syncthreads();
        if (threadIdx.x < 32) {
            double G = 0.0;
            for (int w = 0; w < nw; ++w) G += gpart[w][threadIdx.x] + gpart[w][threadIdx.x + 32];
            gqs[threadIdx.x] = G;
            if (blockIdx.y == 0) p.gq[blockIdx.x * 32 + threadIdx.x] = G;
        }
        __syncthreads();
    }
    const int sh = wave >> 1, qh = wave & 1;
    const int la = lane >> 4, lr = lane & 15;
    const double Gq = gqs[16 * qh + lr];
    const int tile0 = blockIdx.y * p.tiles_per_block;
    const int tile_end = min(p.ntiles, tile0 + p.tiles_per_block);
    for (int tile = tile0; tile < tile_end; ++tile) {
    floatx4 c[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) c[k] = floatx4{};
    // the lane's panel values of atom 4t + la (support row 32 tile + 16 sh + lr): consecutive steps
    // lie 384 floats apart
    const float* sb = p.pan + rmsd_panel_index((int64_t)tile * 32 + 16 * sh + lr, la, 0, nsteps2);
    for (int t = 0; t < nst; ++t, sb += 384) {
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        if (4 * t + la < A) {   // (atoms past A, in the last step when A % 4 == 2: zero)
            s0 = sb[0];
            s1 = sb[64];
            s2 = sb[128];
        }
        const float* xb = xs + (6 * t + qh) * 64 + lane;
        const float x0 = xb[0], x1 = xb[128], x2 = xb[256];
        c[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(s0, x0, c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1, x0, c[1], 0, 0, 0);
        c[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2, x0, c[2], 0, 0, 0);
        c[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(s0, x1, c[3], 0, 0, 0);
        c[4] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1, x1, c[4], 0, 0, 0);
        c[5] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2, x1, c[5], 0, 0, 0);
        c[6] = __builtin_amdgcn_mfma_f32_16x16x4f32(s0, x2, c[6], 0, 0, 0);
        c[7] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1, x2, c[7], 0, 0, 0);
        c[8] = __builtin_amdgcn_mfma_f32_16x16x4f32(s2, x2, c[8], 0, 0, 0);
    }
    // lane l holds rows 4(l/16) + v of the block, column l%16
    float* out = p.r2 + ((int64_t)blockIdx.x * p.ntiles + tile) * 1024 + 16 * qh + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int rho = 16 * sh + 4 * la + v;   // support row within the tile
        const double Gs = p.snorm64[(int64_t)tile * 32 + rho];
        double R[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = (double)c[k][v];
        // a frame collapsed onto its centroid has R = 0 and lambda = 0
        const double r2 =
            (Gs > 0.0 && Gq > 0.0) ? rmsd2_from_corr64(R, Gq, Gs, A, kPairSolveTol) : (Gq + Gs) / A;
        out[(4 * (rho >> 3) + (rho & 3)) * 64 + ((rho >> 2) & 1) * 32] = (float)r2;
    }
    }   // tiles
}

// (eight wavefronts per workgroup run on small grids: two such workgroups per CU need four wavefronts
// per SIMD, i.e. at most 128 registers)
template <typename TI, int DP, int PM, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 8 && DP <= 64 ? 4 : 1)))
void mfma_dist_kernel(DistArgs a) {
    constexpr bool RM = PM == kPmRmsd;        // RMSD frames
    constexpr bool BF = PM == kPmBf16 || PM == kPmBf16x3;   // bfloat16 operands
    constexpr bool BF3 = PM == kPmBf16x3;     // with the remainder products
    constexpr int H = DP / 2;                      // dimensions per lane half
    constexpr int NH = NW / 4;                     // wavefronts per quarter of the support
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int C = a.sup.C;
    float* Dl = reinterpret_cast<float*>(smem_raw);   // [NH][C][32]; copy 0 ends up holding D
    // segment metadata of the support, read once per workgroup: offsets, self terms, |a| sums
    double* mself = reinterpret_cast<double*>(smem_raw + sizeof(float) * (size_t)NH * C * 32);   // [C]
    float2* mseg = reinterpret_cast<float2*>(mself + C);   // [C]: the |a| sum and the summation term
    int32_t* off = reinterpret_cast<int32_t*>(mseg + C);                                    // [C+1]
    __shared__ float Ew[4][32];
    __shared__ float Eg[4][32];
    __shared__ double Bw1[4][32], Bw2[4][32];
    __shared__ int Iw[4][32];
    __shared__ float Es[32];
    __shared__ float Pt[NW][36 * 33];
    __shared__ int jb[5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int type = a.ks.type;
    const float inv2s2 = (float)a.ks.inv2s2;
    const float e2s = inv2s2 * 1.4426950408889634f;   // exponent scale of the tile's kernel values

    float snmax = 0.0f;

    // groups of 32 samples, grid-stride (RMSD: the groups of the pair pass's chunk)
    const int64_t g_begin = RM ? a.grp0 : 0;
    const int64_t g_end = RM ? a.grp0 + a.grp_n : (a.q.n + 31) / 32;
    const int64_t r2_tiles = (a.n_support + 31) / 32;
    for (int64_t grp = g_begin + blockIdx.x; grp < g_end; grp += gridDim.x) {
    const int64_t q = grp * 32 + col;
    const bool active = q < a.q.n;
    const bool first = grp == g_begin + (int64_t)blockIdx.x;

    // the sample's half of the dimensions, its squared norm, and its bf16 split (RMSD: G_x of the
    // lane's frame, left by the pair pass, which also flagged non-finite frames)
    const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + (active ? q : 0) * a.q.stride) * a.q.d;
    float xq[H];
    bf16x8 bh[BF ? H / 8 : 1], bl[BF3 ? H / 8 : 1];
    bool ok;
    float qn;
    if constexpr (RM) {
        qn = (float)a.r2gq[(grp - g_begin) * 32 + col];
        ok = true;
    } else {
        load_query_rows<TI, DP>(xr, a.q.d, (reinterpret_cast<uintptr_t>(a.q.X) & 15) == 0, h, xq);
    }
    if (first) {
        // segment metadata of the support, read once per workgroup while the first group's rows
        // are in flight: offsets; per cluster its self term (+inf for an empty segment, which no
        // row decision counts), its |a| sum and the (length + c) u32 term of its sum's error bound
        if (threadIdx.x < 5) jb[threadIdx.x] = a.sup.split[threadIdx.x];
        const float lc = !RM && type == KKM_KERNEL_LINEAR ? 2.0f : 8.0f;
        for (int j = threadIdx.x; j <= C; j += blockDim.x) {
            const int o = a.sup.offsets[j];
            off[j] = o;
            if (j < C) {
                const int o1 = a.sup.offsets[j + 1];
                mself[j] = o1 > o ? a.sup.self[j] : kInf;
                mseg[j] = make_float2((float)a.sup.segabs[j], ((float)(o1 - o) + lc) * kU32);
            }
        }
        snmax = *a.sup.snorm_max;
        __syncthreads();
    }
    if constexpr (!RM) qn = finish_query<DP, PM>(xq, bh, bl, ok);
    if (active && !ok) atomicOr(a.nonfinite, 1);   // either half may hold the bad value
    const float kqq = type == KKM_KERNEL_LINEAR ? qn : 1.0f;
    const int quarter = wave & 3, half = wave >> 2;
    const int j0 = jb[quarter], j1 = jb[quarter + 1];
    const int start = off[j0], end = off[j1];
    float* Dw = Dl + (size_t)half * C * 32;     // this wavefront's per-cluster sums
    float* P = Pt[wave];                         // [36 rows][33]: one tile of a_l K(x, s_l), 4 rows of slack
    for (int p = lane; p < (j1 - j0) * 32; p += 64) Dw[j0 * 32 + p] = 0.0f;
    // the wavefront's tiles: all of the quarter's, or the first (half 0) or second half of them
    const int t0 = start & ~31;
    const int ntiles = end > t0 ? (end - t0 + 31) / 32 : 0;
    const int tsplit = t0 + 32 * ((ntiles + NH - 1) / NH);
    const int rbeg = half == 0 ? t0 : tsplit;
    const int rend = half == NH - 1 ? end : min(end, tsplit);
    int jc = j0;                                 // first segment that may still receive rows
    while (jc < j1 && off[jc + 1] <= rbeg) ++jc;
    wave_sync_lds();
    for (int r0 = rbeg; r0 < rend; r0 += 32) {
        const int tile_end = min(r0 + 32, end);
        // A fragment: support row r0 + col, the lane half's dimensions, read from the panel of the
        // tile (64 consecutive vectors per step group)
        const int64_t tile = r0 >> 5;
        floatx16 acc;
        if constexpr (RM) {   // the squared RMSDs of the tile, from the pair pass
            const float* rb = a.r2buf + ((grp - g_begin) * r2_tiles + tile) * 1024 + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = rb[64 * i];
        } else {
            acc = mfma_tile<DP, PM>(a.sup, tile, lane, xq, bh, bl);
        }
        // segments meeting the tile (the first 64 of them): a prefix of the lanes, offsets ascend
        int sj = jc + lane;
        int o0 = sj < j1 ? off[sj] : end;
        int o1 = sj < j1 ? off[sj + 1] : end;
        int nseg = __popcll(__ballot(sj < j1 && o0 < tile_end));
        // epilogue: a_l K(x, s_l) for the lane's rows l = r0 + 8(i/4) + 4h + i%4
        float v[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int rb = r0 + 8 * b + 4 * h;
            const float4 sn4 = *reinterpret_cast<const float4*>(a.sup.snorm32 + rb);
            const float4 cf4 = *reinterpret_cast<const float4*>(a.sup.coef32 + rb);
            if constexpr (RM) {   // acc holds the squared RMSD
                v[4 * b + 0] = cf4.x * __builtin_amdgcn_exp2f(-acc[4 * b + 0] * e2s);
                v[4 * b + 1] = cf4.y * __builtin_amdgcn_exp2f(-acc[4 * b + 1] * e2s);
                v[4 * b + 2] = cf4.z * __builtin_amdgcn_exp2f(-acc[4 * b + 2] * e2s);
                v[4 * b + 3] = cf4.w * __builtin_amdgcn_exp2f(-acc[4 * b + 3] * e2s);
            } else {
                v[4 * b + 0] = cf4.x * rbf_or_dot(type, acc[4 * b + 0], qn, sn4.x, e2s);
                v[4 * b + 1] = cf4.y * rbf_or_dot(type, acc[4 * b + 1], qn, sn4.y, e2s);
                v[4 * b + 2] = cf4.z * rbf_or_dot(type, acc[4 * b + 2], qn, sn4.z, e2s);
                v[4 * b + 3] = cf4.w * rbf_or_dot(type, acc[4 * b + 3], qn, sn4.w, e2s);
            }
        }
        // (the register path is compiled for short rows only, where it costs no occupancy)
        if (DP <= 32 && nseg <= 2) {
            // one or two (long) segments: masked sums of the lane's 16 values and its partner's
#pragma unroll 1
            for (int k = 0; k < nseg; ++k) {
                // (k is the same in every lane: a lane read instead of a shuffle)
                const int lo = max(__builtin_amdgcn_readlane(o0, k), r0);
                const int hi = min(__builtin_amdgcn_readlane(o1, k), tile_end);
                float part = 0.0f;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int row = r0 + 8 * (i / 4) + 4 * h + (i % 4);
                    part += (row >= lo && row < hi) ? v[i] : 0.0f;
                }
                part += __shfl_xor(part, 32, 64);
                if (h == 0 && hi > lo) Dw[(jc + k) * 32 + col] += part;
            }
            if (nseg > 0) jc += __builtin_amdgcn_readlane(o1, nseg - 1) > tile_end ? nseg - 1 : nseg;
        } else {
            // short segments: the tile through LDS; lane half h takes every other segment, lane col
            // its sample, each adding its rows in row order.  Each step takes two segments per lane
            // (k0 + h and k0 + 2 + h) and reads their first four rows without a branch (rows past a
            // segment's end count as zeros, which leaves the ordered sums unchanged); longer segments
            // continue four rows at a time.  A lane past the last segment adds its zero into Es, which
            // is free until the decision.
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) P[(8 * b + 4 * h + c) * 33 + col] = v[4 * b + c];
            wave_sync_lds();
            // (r <= r0 + 31, so the four rows read lie within the buffer's 36; rows at or past hi,
            // the slack rows among them, are read but replaced by zeros)
            auto rows4 = [&](int r, int hi, float part) {
                const float* pr = P + (r - r0) * 33 + col;
                float x[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) x[e] = pr[e * 33];
#pragma unroll
                for (int e = 0; e < 4; ++e) part += r + e < hi ? x[e] : 0.0f;
                return part;
            };
            for (;;) {
                for (int k0 = 0; k0 < nseg; k0 += 4) {
                    int lo[2], hi[2];
                    float part[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int k = k0 + 2 * u + h, kc = min(k, nseg - 1);
                        const int a0 = off[jc + kc], a1 = off[jc + kc + 1];
                        lo[u] = max(a0, r0);
                        hi[u] = k < nseg ? min(a1, tile_end) : lo[u];
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) part[u] = rows4(lo[u], hi[u], 0.0f);
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        for (int r = lo[u] + 4; r < hi[u]; r += 4) part[u] = rows4(r, hi[u], part[u]);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int k = k0 + 2 * u + h;
                        *(k < nseg ? &Dw[(jc + k) * 32 + col] : &Es[col]) += part[u];
                    }
                }
                // the last counted segment may continue in the next tile
                if (__builtin_amdgcn_readlane(o1, nseg - 1) > tile_end) {
                    jc += nseg - 1;
                    break;
                }
                jc += nseg;
                if (nseg < 64) break;
                sj = jc + lane;
                o0 = sj < j1 ? off[sj] : end;
                o1 = sj < j1 ? off[sj + 1] : end;
                nseg = __popcll(__ballot(sj < j1 && o0 < tile_end));
                if (nseg == 0) break;
            }
        }
        wave_sync_lds();
    }

    // distances, error bounds and the wave's best / second best per sample (lane half h takes
    // every other cluster; lowest cluster index on equal distances).  The row decision compares
    // D = K(x,x) + g_j - 2 f_j formed in FP64 from the FP32 sums f_j, so its error is that of the
    // f_j alone (K(x,x) is common to the row and cancels in every difference): ef bounds |f_j - exact|.
    // The stored FP32 distances carry in addition their rounding and, for the linear kernel, the
    // error of the FP32 norm (row bound Ecol, used by the medoid candidates).
    // (with eight wavefronts the first four decide: the two halves' sums are complete here)
    if constexpr (NH > 1) __syncthreads();
    float egap = 0.0f, ecol = 0.0f;
    double b1 = kInf, b2 = kInf;
    int i1 = C;
    const float dot_rel = BF3 ? kUbf3 + (3.0f * DP + 2.0f) * kU32
                        : BF ? kUbf1 + (DP + 3.0f) * kU32 : (DP + 2.0f) * kU32;
    const float kmax = sqrtf(qn * snmax) * 1.0001f;
    // (branch-free, so that the unrolled iterations' LDS reads are issued together; one copy of the
    // loop per kernel form)
    const bool nonneg = a.sup.nonneg != 0;
    float rho;   // relative error of each kernel value
    if constexpr (RM) {
        // K = exp(-r^2 / (2 sigma^2)): the r^2 bound times 1 / (2 sigma^2), the float rounding of the
        // exponent's argument and a few ulps of the exponential
        rho = rmsd_r2_bound(qn, snmax, a.ks.n_atoms) * inv2s2 +
              (inv2s2 * (qn + snmax) / (float)a.ks.n_atoms + 4.0f) * kU32;
    } else {
        // RBF: exp's relative error is rho (from the squared-distance error) plus a few ulps, so the
        // sum's error scales with the sum of |a_l| K: the sum itself when no a_l is negative
        rho = (2.0f * dot_rel * kmax + (DP + 6.0f) * kU32 * (qn + snmax)) * inv2s2;
    }
    // (the pairs of clusters are walked with a trip count common to the wavefront; a lane whose
    // cluster is past the quarter's end reads a valid one, discards the result and stores it into its
    // wavefront's free tile buffer)
    const int jend = half == 0 ? j1 : j0;
    auto decide = [&](auto lin_c) {
        constexpr bool LIN = decltype(lin_c)::value;
        const float elin = LIN ? (DP + 2.0f) * kU32 * qn : 0.0f;
#pragma unroll 4
        for (int jp = j0; jp < jend; jp += 2) {
            const int jj = jp + h;
            const bool in = jj < j1;
            const int jr = in ? jj : jp;
            const double g = mself[jr];
            const float2 sg = mseg[jr];
            const float segabs = sg.x, lterm = sg.y;
            float accf = Dl[jr * 32 + col];
            if constexpr (NH > 1) accf += Dl[(size_t)C * 32 + jr * 32 + col];
            const bool live = in && g < kInf;
            const double Dc = (double)kqq + g - 2.0 * (double)accf;
            float ef;
            if constexpr (LIN) {
                ef = (dot_rel * kmax + lterm * kmax) * segabs;
            } else {
                const float mass = nonneg ? fabsf(accf) * 1.0001f + 1e-30f : segabs;
                ef = (rho + lterm) * mass;
            }
            // (plus the FP64 rounding of D and of the self term, 4 units of 2^-53 of the magnitudes)
            const float eg =
                2.0f * ef * 1.0001f + (float)(4.5e-16 * (fabs((double)kqq) + fabs(g) + 2.0 * fabs((double)accf)));
            const float Df = (float)Dc;
            const float e = 2.0f * ef + 2.0f * kU32 * fabsf(Df) + elin;
            egap = live ? fmaxf(egap, eg) : egap;
            ecol = live ? fmaxf(ecol, 2.0f * e) : ecol;
            const double D64 = live ? Dc : kInf;
            *(in ? &Dl[jj * 32 + col] : &P[col]) = live ? Df : __builtin_huge_valf();
            const bool lt1 = D64 < b1, lt2 = D64 < b2;
            b2 = lt1 ? b1 : (lt2 ? D64 : b2);
            b1 = lt1 ? D64 : b1;
            i1 = lt1 ? jj : i1;
        }
    };
    if (!RM && type == KKM_KERNEL_LINEAR) decide(std::true_type{});
    else decide(std::false_type{});
    {   // merge the two lane halves
        const double c1 = __shfl_xor(b1, 32, 64), c2 = __shfl_xor(b2, 32, 64);
        const int k1 = __shfl_xor(i1, 32, 64);
        if (c1 < b1 || (c1 == b1 && k1 < i1)) {
            b2 = fmin(b1, c2);
            b1 = c1;
            i1 = k1;
        } else {
            b2 = fmin(b2, c1);
        }
        egap = fmaxf(egap, __shfl_xor(egap, 32, 64));
        ecol = fmaxf(ecol, __shfl_xor(ecol, 32, 64));
    }
    if (h == 0 && half == 0) {
        Ew[wave][col] = ecol;
        Eg[wave][col] = egap;
        Bw1[wave][col] = b1;
        Bw2[wave][col] = b2;
        Iw[wave][col] = i1;
    }
    __syncthreads();

    const float E = fmaxf(fmaxf(Ew[0][col], Ew[1][col]), fmaxf(Ew[2][col], Ew[3][col]));
    const float EG = fmaxf(fmaxf(Eg[0][col], Eg[1][col]), fmaxf(Eg[2][col], Eg[3][col]));
    bool need = false;   // row listed for the FP64 re-decision
    if (wave == 0 && h == 0 && active) {
        // waves hold ascending cluster ranges: a later wave wins only with a smaller distance
        double best = Bw1[0][col], second = Bw2[0][col];
        int bj = Iw[0][col];
        for (int w = 1; w < 4; ++w) {
            const double c1 = Bw1[w][col], c2 = Bw2[w][col];
            if (c1 < best) {
                second = fmin(best, c2);
                best = c1;
                bj = Iw[w][col];
            } else {
                second = fmin(second, c1);
            }
        }
        if (bj >= C) bj = 0;
        a.labels[q] = bj;
        if (a.best) a.best[q] = best;
        if (a.Erow) a.Erow[q] = E;
        const double scale = fmax(fmax(fabs(best), fabs(second)), fabs((double)kqq));
        if (a.gap)
            a.gap[q] = second < kInf ? (float)((second - best) / (scale > 0 ? scale : 1.0)) : __builtin_huge_valf();
        const double gap = second - best;
        need = gap <= 2.0 * (double)EG && gap + 2.0 * (double)EG >= kTieMargin * scale;
    }
    if (wave == 0) append_rows(need, q, a.refine_count, a.refine_list);
    if (a.Dt) {
        // the D tile through LDS: consecutive threads store consecutive samples of one cluster, and
        // thread j takes the column minimum of cluster j over the group's samples (each thread starting
        // at sample j mod 32, so that a wavefront's reads fall in distinct banks)
        // (E of a sample slot past the last row is +inf, which removes it from the minima)
        if (wave == 0 && h == 0) Es[col] = active ? E : __builtin_huge_valf();
        __syncthreads();
        float* Dt = a.Dt;
        const int64_t q0 = grp * 32;
        for (int p = threadIdx.x; p < C * 32; p += NW * 64) {
            const int c = p & 31;
            if (q0 + c < a.q.n) Dt[(int64_t)(p >> 5) * a.ldD + q0 + c] = Dl[p];
        }
        if (a.colmin) {
            for (int jj = threadIdx.x; jj < C; jj += NW * 64) {
                double vv = kInf;
#pragma unroll 8
                for (int k = 0; k < 32; ++k) {
                    const int c = (k + jj) & 31;
                    vv = fmin(vv, (double)Dl[jj * 32 + c] + (double)Es[c]);
                }
                a.colpart[(int64_t)jj * a.colpart_cap + grp] = vv;
            }
        }
    }
    __syncthreads();   // the group's LDS (Dl, Pt, per-wave results) is reused by the next group
    }   // groups
}

// Assign against a medoid model: every cluster has one support row with coefficient 1 and the self
// term of that row (1 for RBF, ||m||^2 for linear).  Then d(x, j) = K(x,x) + self_j - 2 K(x, m_j) is
// an increasing function of e_j = ||m_j||^2 - 2 x.m_j for both kernels (RBF: 2 - 2 exp(-(||x||^2 +
// e_j) / (2 sigma^2)); linear: ||x||^2 + e_j), so the label is the argmin of e_j: the pass needs no
// exponential and no segment sums, and only the best and second-best e become distances.
// One wavefront per 32 samples (grid-stride over groups), walking every 32-row tile of the support;
// lane l keeps the best two of its rows 8(i/4) + 4(l/32) + i%4 of each tile (visited in ascending
// order, so the lowest index wins a tie), then merges with its partner lane l^32.
//
// Error bound of e: |x.m computed - exact| <= dot_rel kmax (kmax >= ||x|| ||m||), the FP32 norm
// ||m||^2 and the subtraction add rounding of at most 3 u32 (snmax + 2 kmax): Ee.  A row whose two
// smallest e are within 2 Ee is listed for the FP64 re-decision, unless the exact relative margin
// in d is provably below kTieMargin (the bound on it follows from 1 - exp(-t) <= t for RBF).
template <typename TI, int DP, int PM>
__global__ __launch_bounds__(256) void mfma_assign1_kernel(DistArgs a) {
    constexpr int H = DP / 2;
    constexpr bool RM = PM == kPmRmsd;
    constexpr bool BF = PM == kPmBf16 || PM == kPmBf16x3, BF3 = PM == kPmBf16x3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int C = a.sup.C;
    const int ntiles = (C + 31) / 32;
    const bool lin = a.ks.type == KKM_KERNEL_LINEAR;
    const float c2 = (float)a.ks.inv2s2;
    const float snmax = *a.sup.snorm_max;
    const float dot_rel = BF3 ? kUbf3 + (3.0f * DP + 2.0f) * kU32 : BF ? kUbf1 + (DP + 3.0f) * kU32 : (DP + 2.0f) * kU32;
    const bool vec_ok = (reinterpret_cast<uintptr_t>(a.q.X) & 15) == 0;
    // (RMSD: the groups of the pair pass's chunk, whose squared RMSDs it reads)
    const int64_t g_begin = RM ? a.grp0 : 0;
    const int64_t g_end = RM ? a.grp0 + a.grp_n : (a.q.n + 31) / 32;
    for (int64_t grp = g_begin + (int64_t)blockIdx.x * 4 + wave; grp < g_end; grp += (int64_t)gridDim.x * 4) {
        // (re-decision pass of the plain BF16 cascade: only the groups with marked rows, and in them
        // only the marked rows are written)
        const uint32_t gmask = a.gate_mode == 2 ? a.gate[grp] : 0xffffffffu;
        if (gmask == 0u) continue;
        const int64_t q = grp * 32 + col;
        const bool active = q < a.q.n && ((gmask >> col) & 1u);
        const TI* xr = static_cast<const TI*>(a.q.X) + (a.q.base + (q < a.q.n ? q : 0) * a.q.stride) * a.q.d;
        float xq[H];
        bf16x8 bh[BF ? H / 8 : 1], bl[BF3 ? H / 8 : 1];
        bool ok;
        float qn;
        if constexpr (RM) {   // (G of the frame from the pair pass, which flagged non-finite frames)
            qn = (float)a.r2gq[(grp - g_begin) * 32 + col];
            ok = true;
        } else {
            qn = load_query<TI, DP, PM>(xr, a.q.d, vec_ok, h, xq, bh, bl, ok);
        }
        if (active && !ok) atomicOr(a.nonfinite, 1);
        float e1 = __builtin_huge_valf(), e2 = __builtin_huge_valf();
        int j1 = C;
        for (int t = 0; t < ntiles; ++t) {
            floatx16 acc;
            if constexpr (RM) {
                const float* rb = a.r2buf + ((grp - g_begin) * ((a.n_support + 31) / 32) + t) * 1024 + lane;
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[i] = rb[64 * i];
            } else {
                acc = mfma_tile<DP, PM>(a.sup, t, lane, xq, bh, bl);
            }
            // best and second best of the lane's rows (branch-free; a NaN changes neither), the rows
            // past the last cluster masked only in the last, partial tile
            auto take = [&](float e, int j) {
                const bool lt = e < e1;
                e2 = lt ? e1 : fminf(e2, e);
                j1 = lt ? j : j1;
                e1 = lt ? e : e1;
            };
            auto epilogue = [&](auto masked) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int rb = 32 * t + 8 * b + 4 * h;
                    const float4 sn4 = *reinterpret_cast<const float4*>(a.sup.snorm32 + rb);
                    const float sn[4] = {sn4.x, sn4.y, sn4.z, sn4.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int j = rb + c;
                        // RBF / linear: e = ||m||^2 - 2 x.m; RMSD: e = r^2 (d = 2 - 2 exp(-r^2 / (2 sigma^2)))
                        const float ev = RM ? acc[4 * b + c] : fmaf(-2.0f, acc[4 * b + c], sn[c]);
                        take(decltype(masked)::value && j >= C ? __builtin_huge_valf() : ev, j);
                    }
                }
            };
            if (32 * t + 32 <= C) epilogue(std::false_type{});
            else epilogue(std::true_type{});
        }
        {   // the partner lane holds the interleaved rows of every tile
            const float o1 = __shfl_xor(e1, 32, 64), o2 = __shfl_xor(e2, 32, 64);
            const int k1 = __shfl_xor(j1, 32, 64);
            if (o1 < e1 || (o1 == e1 && k1 < j1)) {
                e2 = fminf(e1, o2);
                e1 = o1;
                j1 = k1;
            } else {
                e2 = fminf(e2, o1);
            }
        }
        bool need = false;
        if (h == 0 && active) {
            const int bj = j1 < C ? j1 : 0;
            const float kmax = sqrtf(qn * snmax) * 1.0001f;
            const float Ee = RM ? rmsd_r2_bound(qn, snmax, a.ks.n_atoms) + kU32 * (qn + snmax) / (float)a.ks.n_atoms
                                : 2.0f * dot_rel * kmax + 3.0f * kU32 * (snmax + 2.0f * kmax);
            const double g1 = a.sup.self[bj];
            double D1, D2, kqq;
            if (RM) {
                kqq = 1.0;
                const float K1 = exp_neg(fmaxf(e1, 0.0f) * c2);
                const float K2 = e2 < __builtin_huge_valf() ? exp_neg(fmaxf(e2, 0.0f) * c2) : 0.0f;
                D1 = kqq + g1 - 2.0 * (double)K1;
                D2 = e2 < __builtin_huge_valf() ? 2.0 - 2.0 * (double)K2 : kInf;
            } else if (lin) {
                kqq = qn;
                D1 = (double)qn + (double)e1 + (g1 - (double)a.sup.snorm32[bj]);
                D2 = (double)qn + (double)e2;
            } else {
                kqq = 1.0;
                const float K1 = exp_neg(fmaxf(qn + e1, 0.0f) * c2);
                const float K2 = e2 < __builtin_huge_valf() ? exp_neg(fmaxf(qn + e2, 0.0f) * c2) : 0.0f;
                D1 = kqq + g1 - 2.0 * (double)K1;
                D2 = e2 < __builtin_huge_valf() ? 2.0 - 2.0 * (double)K2 : kInf;
            }
            a.labels[q] = bj;
            if (a.best) a.best[q] = D1;
            if (a.gap) {
                const double scale = fmax(fmax(fabs(D1), fabs(D2)), fabs(kqq));
                a.gap[q] = D2 < kInf ? (float)((D2 - D1) / (scale > 0 ? scale : 1.0)) : __builtin_huge_valf();
            }
            const float ge = e2 - e1;
            if (ge <= 2.0f * Ee) {
                // upper bound on the exact relative margin of d
                const float qlo = qn * (1.0f - (DP + 2.0f) * kU32);
                float ub;
                if (lin) ub = (ge + 2.0f * Ee) / fmaxf(qlo, 1e-30f);
                else if (RM) ub = 2.0f * exp_neg(fmaxf(e1 - Ee, 0.0f) * c2) * (ge + 2.0f * Ee) * c2;
                else ub = 2.0f * exp_neg(fmaxf(qlo + e1 - Ee, 0.0f) * c2) * (ge + 2.0f * Ee) * c2;
                need = !(ub < (float)kTieMargin);
            }
        }
        if (a.gate_mode == 1) {   // BF16 pass of the cascade: mark, do not list
            const uint32_t mk = (uint32_t)(__ballot(need) & 0xffffffffull);
            if (lane == 0) a.gate[grp] = mk;
        } else {
            append_rows(need, q, a.refine_count, a.refine_list);
        }
    }
}

size_t mfma_lds_dynamic(size_t C, int nw) {
    return sizeof(float) * (size_t)(nw / 4) * C * 32 + sizeof(double) * 2 * C + sizeof(int32_t) * (C + 1);
}
size_t mfma_lds_static(int nw) {
    return sizeof(float) * ((size_t)nw * 36 * 33 + 4 * 32 * 2 + 32) + sizeof(double) * 4 * 32 * 2 + sizeof(int) * 4 * 32 +
           64;
}

template <typename TI, int PM, int NW>
kkm_status launch_mfma_nw(const DistArgs& a, hipStream_t s, int64_t groups, unsigned blocks) {
    const size_t lds = mfma_lds_dynamic((size_t)a.sup.C, NW);
    auto go = [&](auto fn) -> kkm_status {
        KKM_TRY(allow_dynamic_lds(reinterpret_cast<const void*>(fn), lds));
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(NW * 64), lds, s, a);
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    };
    if constexpr (PM == kPmRmsd) {
        return go(mfma_dist_kernel<TI, 16, PM, NW>);
    } else {
    switch (a.sup.dpad) {
        case 4: if constexpr (PM == kPmF32) return go(mfma_dist_kernel<TI, 4, PM, NW>); break;
        case 8: if constexpr (PM == kPmF32) return go(mfma_dist_kernel<TI, 8, PM, NW>); break;
        case 16: return go(mfma_dist_kernel<TI, 16, PM, NW>);
        case 32: return go(mfma_dist_kernel<TI, 32, PM, NW>);
        case 64: return go(mfma_dist_kernel<TI, 64, PM, NW>);
        case 128: return go(mfma_dist_kernel<TI, 128, PM, NW>);
        default: break;
    }
    return fail(KKM_ERR_UNSUPPORTED, "matrix-core distance pass: unsupported padded dimension");
    }
}

// The RMSD pair pass over query groups [g0, g0 + ng) (chunk buffers of a).
kkm_status launch_rmsd_pairs(const DistArgs& a, int64_t g0, int64_t ng, hipStream_t s) {
    RmsdPairsArgs p{};
    p.q = a.q;
    p.pan = a.sup.pan;
    p.snorm64 = a.sup.snorm64;
    p.A = a.ks.n_atoms;
    p.g0 = g0;
    p.ntiles = (int32_t)std::max<int64_t>(1, (a.n_support + 31) / 32);
    // tiles per workgroup: the staging of a group's frames is shared by several tiles while the grid
    // still holds about 2048 workgroups
    p.tiles_per_block = (int32_t)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, ng * p.ntiles / 2048));
    p.r2 = a.r2buf;
    p.gq = a.r2gq;
    p.nonfinite = a.nonfinite;
    const dim3 grid((unsigned)ng, (unsigned)((p.ntiles + p.tiles_per_block - 1) / p.tiles_per_block));
    const size_t lds = sizeof(float) * 384 * (size_t)((p.A + 3) / 4);
    KKM_TRY(allow_dynamic_lds(reinterpret_cast<const void*>(rmsd_pairs_kernel), lds));
    hipLaunchKernelGGL(rmsd_pairs_kernel, grid, dim3(256), lds, s, p);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

// Every chunk of query groups: the pair pass, then the reduction f(a, g0, ng).
template <typename F>
kkm_status rmsd_chunks(const DistArgs& a, hipStream_t s, F&& f) {
    if (!a.r2buf || !a.r2gq || a.rmsd_chunk < 1 || !a.sup.pan)
        return fail(KKM_ERR_INTERNAL, "RMSD pair pass without its buffers");
    const int64_t groups = (a.q.n + 31) / 32;
    for (int64_t g0 = 0; g0 < groups; g0 += a.rmsd_chunk) {
        const int64_t ng = std::min<int64_t>(a.rmsd_chunk, groups - g0);
        KKM_TRY(launch_rmsd_pairs(a, g0, ng, s));
        DistArgs b = a;
        b.grp0 = g0;
        b.grp_n = ng;
        KKM_TRY(f(b, ng));
    }
    return KKM_OK;
}

// Eight wavefronts per distance workgroup below this many 32-sample groups per CU (KKM_DIST_EIGHT
// overrides it).
static int dist_eight_groups_per_cu() {
    static const int v = [] {
        const char* e = std::getenv("KKM_DIST_EIGHT");
        const int x = e ? std::atoi(e) : 0;
        return x > 0 ? x : 2;
    }();
    return v;
}

template <typename TI, int PM>
kkm_status launch_mfma_t(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    const size_t C = (size_t)a.sup.C;
    if (mfma_lds_dynamic(C, 4) + mfma_lds_static(4) > dev.max_lds_per_block)
        return fail(KKM_ERR_UNSUPPORTED, "too many clusters for the distance tile");
    // 32 samples per group; a bounded grid of workgroups, each looping over groups
    const int64_t groups = (a.q.n + 31) / 32;
    if constexpr (PM == kPmRmsd) {
        // the tiles are read back from the pair pass: four wavefronts per workgroup, a grid per chunk
        if (a.colmin && groups > a.colpart_cap) return fail(KKM_ERR_INTERNAL, "column partials too small");
        KKM_TRY(rmsd_chunks(a, s, [&](const DistArgs& b, int64_t ng) {
            const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ng, 8 * (int64_t)dev.num_cus));
            return launch_mfma_nw<TI, PM, 4>(b, s, ng, blocks);
        }));
        if (a.colmin && a.colpart_blocks) *a.colpart_blocks = groups;
        return KKM_OK;
    }
    // Eight wavefronts per workgroup when four would leave the SIMDs under two wavefronts each
    // (few groups: the pass is bound by each wavefront's chain of tiles), where their LDS fits;
    // otherwise four, which duplicate less per-group work.
    const bool eight = groups < (int64_t)dist_eight_groups_per_cu() * dev.num_cus &&
                       mfma_lds_dynamic(C, 8) + mfma_lds_static(8) <= dev.max_lds_per_block;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(groups, 8 * (int64_t)dev.num_cus));
    if (a.colmin && groups > a.colpart_cap) return fail(KKM_ERR_INTERNAL, "column partials too small");
    const kkm_status st = eight ? launch_mfma_nw<TI, PM, 8>(a, s, groups, blocks)
                                : launch_mfma_nw<TI, PM, 4>(a, s, groups, blocks);
    if (st != KKM_OK) return st;
    if (a.colmin && a.colpart_blocks) *a.colpart_blocks = groups;
    return KKM_OK;
}

}  // namespace

bool mfma_disabled() {
    static const bool off = [] {
        const char* e = std::getenv("KKM_DIST_VALU");
        return e && e[0] == '1';
    }();
    return off;
}

bool mfma_dist_applies(const DistArgs& a) {
    if (mfma_disabled() || a.precision == KKM_PREC_FP64 || a.dtype != KKM_F32) return false;
    if (a.ks.type == KKM_KERNEL_RMSD) return rmsd_mfma_ok(a.ks.n_atoms, a.dtype) && a.sup.pan != nullptr;
    if (a.precision == KKM_PREC_BF16X3) return a.sup.hi && a.sup.lo && a.sup.dpad >= 16;
    if (a.precision == KKM_PREC_BF16) return a.sup.hi && a.sup.dpad >= 16;
    return a.sup.pan != nullptr;
}

template <int PM>
kkm_status launch_assign1(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    const int64_t groups = (a.q.n + 31) / 32;
    auto blocks_for = [&](int64_t g) {
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>((g + 3) / 4, 16 * (int64_t)dev.num_cus));
    };
    if constexpr (PM == kPmRmsd) {
        return rmsd_chunks(a, s, [&](const DistArgs& b, int64_t ng) -> kkm_status {
            hipLaunchKernelGGL((mfma_assign1_kernel<float, 16, PM>), dim3(blocks_for(ng)), dim3(256), 0, s, b);
            KKM_HIP(hipGetLastError());
            return KKM_OK;
        });
    } else {
    const unsigned blocks = blocks_for(groups);
    auto go = [&](auto fn) -> kkm_status {
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, s, a);
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    };
    switch (a.sup.dpad) {
        case 4: if constexpr (PM == kPmF32) return go(mfma_assign1_kernel<float, 4, PM>); break;
        case 8: if constexpr (PM == kPmF32) return go(mfma_assign1_kernel<float, 8, PM>); break;
        case 16: return go(mfma_assign1_kernel<float, 16, PM>);
        case 32: return go(mfma_assign1_kernel<float, 32, PM>);
        case 64: return go(mfma_assign1_kernel<float, 64, PM>);
        case 128: return go(mfma_assign1_kernel<float, 128, PM>);
        default: break;
    }
    return fail(KKM_ERR_UNSUPPORTED, "matrix-core assign: unsupported padded dimension");
    }
}

kkm_status launch_dist_mfma(const DistArgs& a, const DeviceInfo& dev, hipStream_t s) {
    if (a.q.n <= 0) return KKM_OK;
    if (a.ks.type == KKM_KERNEL_RMSD) {
        if (a.sup.medoid_form && !a.Dt && !a.colmin && !a.Erow) return launch_assign1<kPmRmsd>(a, dev, s);
        return launch_mfma_t<float, kPmRmsd>(a, dev, s);
    }
    if (a.sup.medoid_form && !a.Dt && !a.colmin && !a.Erow) {
        if (a.precision == KKM_PREC_BF16X3) return launch_assign1<kPmBf16x3>(a, dev, s);
        if (a.precision == KKM_PREC_BF16) {
            if (!a.gate || !a.sup.lo) return launch_assign1<kPmBf16>(a, dev, s);
            // the cascade: BF16 marks its undecided rows, BF16x3 re-decides them and lists for FP64
            // the rows it cannot decide either
            DistArgs b = a;
            b.gate_mode = 1;
            KKM_TRY(launch_assign1<kPmBf16>(b, dev, s));
            b.gate_mode = 2;
            return launch_assign1<kPmBf16x3>(b, dev, s);
        }
        return launch_assign1<kPmF32>(a, dev, s);
    }
    if (a.precision == KKM_PREC_BF16X3) return launch_mfma_t<float, kPmBf16x3>(a, dev, s);
    if (a.precision == KKM_PREC_BF16) return launch_mfma_t<float, kPmBf16>(a, dev, s);
    return launch_mfma_t<float, kPmF32>(a, dev, s);
}

}  // namespace kkm
