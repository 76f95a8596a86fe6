// Internal declarations of libkkm: status plumbing, the model layout, launch helpers and the device
// building blocks shared by the kernels (kernel functions, wavefront reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/kkm.h"

namespace kkm {

// ----------------------------------------------------------------------------- host status
void set_error(const std::string& msg);
kkm_status fail(kkm_status code, const std::string& msg);

#define KKM_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::kkm::fail(KKM_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define KKM_TRY(expr)                          \
    do {                                       \
        kkm_status s_ = (expr);                \
        if (s_ != KKM_OK) return s_;           \
    } while (0)

// ----------------------------------------------------------------------------- constants
constexpr int kWave = 64;
constexpr int kMaxClusters = 1024;        // C limit of the device kernels
constexpr int kMaxRegDim = 128;           // register-resident query rows (linear / RBF)
constexpr double kInf = __builtin_huge_val();

// Padded dimension of stored support rows: the register-resident row length the distance
// kernels are instantiated for.
inline int padded_dim(int64_t d) {
    if (d <= 4) return 4;
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    return 128;
}

// Row stride of the bfloat16 split arrays (the matrix-core K step is 16).
inline int bf16_pad(int dpad) { return dpad < 16 ? 16 : dpad; }

// Panel layouts of the support for the matrix-core pass.  Rows are grouped in tiles of 32; within a
// tile the operand fragment that one MFMA step (or group of steps) needs from the 64 lanes is stored
// as 64 consecutive vectors in lane order, lane = 32 h + (row % 32) holding dimensions
// h (DP/2) + [vector start, vector start + width).  FP32 panels use vectors of min(4, DP/2) floats,
// bfloat16 panels vectors of 8 (DP >= 16 only).  Both hold exactly 32 DP elements per tile.
// rows to allocate for panels covering rows [0, rows): whole tiles
inline size_t panel_rows(size_t rows) { return (rows + 31) & ~size_t(31); }

__host__ __device__ inline int64_t panel32_index(int64_t r, int c, int DP) {
    const int H = DP / 2, VW = H < 4 ? H : 4;
    const int h = c / H, s = c - h * H;
    const int g = s / VW, e = s - g * VW;
    return (((r >> 5) * (H / VW) + g) * 64 + h * 32 + (int)(r & 31)) * VW + e;
}
__host__ __device__ inline int64_t panel16_index(int64_t r, int c, int DP) {
    const int H = DP / 2;
    const int h = c / H, s = c - h * H;
    return (((r >> 5) * (H / 8) + (s >> 3)) * 64 + h * 32 + (int)(r & 31)) * 8 + (s & 7);
}

// Panel layout of RMSD support frames for the matrix-core cross-covariance: per 32-row tile, for
// every pair of atoms t = a / 2 and coordinate q, the 64 values one MFMA operand needs, lane
// 32 (a % 2) + row % 32 holding coordinate q of atom a of that row.  A tile holds 32 * 3 * A values
// (A even), the same count as 32 rows of the frames themselves.
__host__ __device__ inline int64_t rmsd_panel_index(int64_t r, int atom, int q, int nsteps) {
    return (((r >> 5) * nsteps + (atom >> 1)) * 3 + q) * 64 + (atom & 1) * 32 + (int)(r & 31);
}
// RMSD frames take the matrix-core path for float frames with an even atom count up to this many.
constexpr int kRmsdMfmaMaxAtoms = 64;   // (the pair pass stages 384 A bytes of LDS per workgroup)
inline bool rmsd_mfma_ok(int n_atoms, int dtype) {
    return dtype == KKM_F32 && n_atoms >= 2 && n_atoms % 2 == 0 && n_atoms <= kRmsdMfmaMaxAtoms;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over the caller's workspace (or a size probe when base == nullptr).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        size_t at = off;
        off = align256(off + count * sizeof(T));
        return base ? reinterpret_cast<T*>(base + at) : nullptr;
    }
};

// Per-device facts queried once.
struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    size_t max_lds_per_block = 0;
    bool coop = false;
};
kkm_status device_info(DeviceInfo* out);
// Allow a kernel more than 64 KiB of dynamic LDS (no-op below that; once per device and kernel).
kkm_status allow_dynamic_lds(const void* fn, size_t bytes);

}  // namespace kkm

// ----------------------------------------------------------------------------- the model
// Device-resident sparse centroids.  Support rows are stored padded to `dpad` columns with zeros
// (RMSD: centred frames, also padded), in the model dtype.
struct kkm_model {
    kkm_kernel kernel;
    int64_t d = 0;
    int32_t dpad = 0;
    int32_t C = 0;
    int64_t cap = 0;          // support rows allocated
    int64_t used = 0;         // support rows in use
    int32_t dtype = KKM_F32;
    int device = 0;
    void* block = nullptr;    // one allocation holding everything below
    void* support = nullptr;  // [cap][dpad] (dtype)
    float* snorm32 = nullptr; // [cap] ||s||^2 (RBF / linear) or G (RMSD), FP32
    double* snorm64 = nullptr;// [cap] same in FP64
    float* coef32 = nullptr;  // [cap]
    double* coef64 = nullptr; // [cap]
    int32_t* offsets = nullptr; // [C+1]
    double* self = nullptr;   // [C] a^T K a (FP64); +inf disables the cluster
    double* segabs = nullptr; // [C] sum_l |a_l| over segment j
    float* snorm_max = nullptr; // [1] max ||s||^2 over the support (error bounds)
    int32_t* split = nullptr;   // [5] cluster runs of the four wavefronts of a distance tile
    int32_t nonneg = 1;         // every coefficient >= 0
    float* pan = nullptr;       // FP32 panel copy of the support (float models only)
    uint16_t* hi = nullptr;     // bfloat16 panel of the high parts of the support rows (dpad >= 16)
    uint16_t* lo = nullptr;     // [cap + 32][bpad] bfloat16 remainders
    int32_t bpad = 0;
    int64_t* counts = nullptr;  // [C] |w_j| of a fitted model
    int64_t* medoid_index = nullptr; // [C]
    int32_t medoid_form = 0;    // support row j is cluster j's only row, coefficient 1, no cluster disabled
};

namespace kkm {

// Carve the device arrays of model m (its kernel, d, dpad, bpad, C, cap and dtype set) from c: the
// layout of kkm_model_create's one allocation, also used for models that live in a workspace.
void model_layout(kkm_model* m, Carver& c);

// ----------------------------------------------------------------------------- device helpers
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    // fixed butterfly: the result depends only on the 64 inputs, not on timing
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// bfloat16 split of a float: hi = RNE(x), lo = RNE(x - hi), as raw 16-bit patterns.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const __bf16 b = (__bf16)x;
    return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ void bf16_split(float x, uint16_t& hi, uint16_t& lo) {
    const __bf16 h = (__bf16)x;
    hi = __builtin_bit_cast(uint16_t, h);
    lo = bf16_bits(x - (float)h);
}

// Order-preserving map of doubles to unsigned 64-bit integers (for atomicMin on values).
__device__ __forceinline__ unsigned long long ord_enc(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_dec(unsigned long long e) {
    const unsigned long long b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    return __longlong_as_double((long long)b);
}

// LDS writes of a wavefront become visible to its other lanes.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Appends q to list for the lanes with flag set, with one atomic per wavefront (call from all lanes
// of the wavefront).  List order across wavefronts is unspecified.
__device__ __forceinline__ void append_rows(bool flag, int64_t q, int32_t* count, int32_t* list) {
    const unsigned long long m = __ballot(flag);
    if (m == 0ull) return;
    const int lane = (int)(threadIdx.x & 63);
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader, 64);
    if (flag) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)q;
}

__device__ __forceinline__ float exp_neg(float a) {     // exp(-a), a >= 0
    return __builtin_amdgcn_exp2f(-a * 1.4426950408889634f);
}
__device__ __forceinline__ double exp_neg(double a) { return ::exp(-a); }

// Kernel-function evaluation from a dot product and the two squared norms (linear / RBF).
template <typename T>
__device__ __forceinline__ T kfun_from_dot(int type, T dot, T qn, T sn, T inv2s2) {
    if (type == KKM_KERNEL_LINEAR) return dot;
    T d2 = qn + sn - T(2) * dot;
    d2 = d2 > T(0) ? d2 : T(0);
    return exp_neg(d2 * inv2s2);
}

// FP64 kernel evaluation between two rows of length d (linear / RBF), RBF from explicit
// differences.  Rows may be float or double.
template <typename TA, typename TB>
__device__ inline double kfun64_rows(int type, const TA* __restrict__ a, const TB* __restrict__ b, int64_t d,
                                     double inv2s2) {
    double acc = 0.0;
    if (type == KKM_KERNEL_LINEAR) {
        for (int64_t k = 0; k < d; ++k) acc = fma((double)a[k], (double)b[k], acc);
        return acc;
    }
    for (int64_t k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        acc = fma(t, t, acc);
    }
    return ::exp(-acc * inv2s2);
}

// Kernel specification as the device sees it.
struct KSpec {
    int type;        // enum kkm_kernel_type
    int n_atoms;     // RMSD
    int64_t d;       // row length
    double inv2s2;   // 1 / (2 sigma^2)
};

// Determinant of a 4x4 matrix by the Laplace expansion over 2x2 minors of rows (0,1) and (2,3).
template <typename T>
__device__ __forceinline__ T det4(const T m[4][4]) {
    T s0 = m[0][0] * m[1][1] - m[1][0] * m[0][1];
    T s1 = m[0][0] * m[1][2] - m[1][0] * m[0][2];
    T s2 = m[0][0] * m[1][3] - m[1][0] * m[0][3];
    T s3 = m[0][1] * m[1][2] - m[1][1] * m[0][2];
    T s4 = m[0][1] * m[1][3] - m[1][1] * m[0][3];
    T s5 = m[0][2] * m[1][3] - m[1][2] * m[0][3];
    T c5 = m[2][2] * m[3][3] - m[3][2] * m[2][3];
    T c4 = m[2][1] * m[3][3] - m[3][1] * m[2][3];
    T c3 = m[2][1] * m[3][2] - m[3][1] * m[2][2];
    T c2 = m[2][0] * m[3][3] - m[3][0] * m[2][3];
    T c1 = m[2][0] * m[3][2] - m[3][0] * m[2][2];
    T c0 = m[2][0] * m[3][1] - m[3][0] * m[2][1];
    return s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
}

// Horn's symmetric, traceless 4x4 key matrix of the correlation R[p][q] = sum_a x_ap y_aq
// (row-major R[3p+q]); its largest eigenvalue is the best superposition overlap.
template <typename T>
__device__ __forceinline__ void horn_key(const T R[9], T N[4][4]) {
    const T Sxx = R[0], Sxy = R[1], Sxz = R[2], Syx = R[3], Syy = R[4], Syz = R[5];
    const T Szx = R[6], Szy = R[7], Szz = R[8];
    N[0][0] = Sxx + Syy + Szz; N[0][1] = Syz - Szy;        N[0][2] = Szx - Sxz;         N[0][3] = Sxy - Syx;
    N[1][1] = Sxx - Syy - Szz; N[1][2] = Sxy + Syx;        N[1][3] = Szx + Sxz;
    N[2][2] = -Sxx + Syy - Szz; N[2][3] = Syz + Szy;
    N[3][3] = -Sxx - Syy + Szz;
    N[1][0] = N[0][1]; N[2][0] = N[0][2]; N[3][0] = N[0][3];
    N[2][1] = N[1][2]; N[3][1] = N[1][3]; N[3][2] = N[2][3];
}

// Largest eigenvalue of a symmetric 4x4 matrix by cyclic Jacobi rotations (Golub and Van Loan,
// "Matrix Computations", Sec. 8.5): each rotation zeroes one off-diagonal pair; sweeps repeat until
// the off-diagonal mass is negligible against the diagonal.  Backward stable, so the eigenvalue is
// accurate to a few units of roundoff of ||N|| whatever the multiplicity.  N is overwritten.
__device__ __forceinline__ double sym4_max_eig_jacobi(double (&N)[4][4]) {
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < 4; ++i) {
            diag += N[i][i] * N[i][i];
            for (int j = i + 1; j < 4; ++j) off += N[i][j] * N[i][j];
        }
        if (off <= 1e-36 * diag || off == 0.0) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const double apq = N[p][q];
                if (apq == 0.0) continue;
                // rotation angle: t = tan(theta) as the smaller root of t^2 + 2 tau t - 1 = 0
                const double tau = (N[q][q] - N[p][p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < 4; ++k) {   // columns p, q
                    const double kp = N[k][p], kq = N[k][q];
                    N[k][p] = c * kp - sn * kq;
                    N[k][q] = sn * kp + c * kq;
                }
                for (int k = 0; k < 4; ++k) {   // rows p, q
                    const double pk = N[p][k], qk = N[q][k];
                    N[p][k] = c * pk - sn * qk;
                    N[q][k] = sn * pk + c * qk;
                }
                N[p][q] = N[q][p] = 0.0;
            }
    }
    return fmax(fmax(N[0][0], N[1][1]), fmax(N[2][2], N[3][3]));
}

// The Jacobi solve of the key matrix of R, out of line (it is rare) and with R passed by value, so
// that no array of the caller has its address taken and the caller's solve stays in registers.
static __device__ __attribute__((noinline)) double key_max_eig_jacobi(double r0, double r1, double r2, double r3,
                                                                       double r4, double r5, double r6, double r7,
                                                                       double r8) {
    const double R[9] = {r0, r1, r2, r3, r4, r5, r6, r7, r8};
    double N[4][4];
    horn_key(R, N);
    return sym4_max_eig_jacobi(N);
}

// Iterations after which the root iteration gives up: from the upper bound a simple largest root is
// reached in about five.
constexpr int kRootSteps = 20;

// Largest eigenvalue of the key matrix from its characteristic polynomial
// P(lambda) = lambda^4 + c2 lambda^2 + c1 lambda + c0.  For Horn's matrix tr(N^2) = 4 ||R||_F^2 and
// tr(N^3) = 24 det R, so c2 = -tr(N^2)/2 = -2 ||R||_F^2, c1 = -tr(N^3)/3 = -8 det R and c0 = det N.
// P has only real roots (N is symmetric), so Laguerre's iteration for degree n = 4,
//   lambda <- lambda - n P / (P' + sqrt((n - 1) ((n - 1) P'^2 - n P P''))),
// started from the upper bound (Ga + Gb)/2 decreases monotonically onto the largest root and
// converges cubically at a simple root (Press et al., "Numerical Recipes", Sec. 9.5; the method is
// globally convergent for real-rooted polynomials); it needs about half of Newton's steps from the
// same start.
//
// Near a multiple root the iteration converges only linearly and P's rounding can stop it away from
// the root, so the root is accepted only with an a-posteriori check: eta(lambda) bounds the error of
// P as computed (the coefficients' rounding -- relative 10 u for the sum of squares, 5 u of the
// absolute cofactor terms m1 of det R and 10 u of the absolute minor products M0 of det N -- and the
// evaluation's, 4 u of each term), so the exact root lies within about (|P| + eta) / P'(lambda) of
// the computed one; it is kept when that is at most tol (Ga + Gb) / 2, and otherwise (or when the
// iteration does not settle within kRootSteps steps) the pair is solved by Jacobi rotations of the
// key matrix.  Returns RMSD^2 = max(0, (Ga + Gb - 2 lambda) / A), within tol (Ga + Gb) / A plus
// roundoff.  (FP64 callers keep tol = 1e-13; a caller whose R carries FP32 rounding may pass a larger
// tol, well under that rounding, and so rarely needs the rotations.)
// Coefficients of the key matrix's characteristic polynomial, P(l) = l^4 + c2 l^2 + c1 l + c0, and
// the terms of the bound on its rounding: |P computed - P| <= u (((4 l^2 + e2) l + e1) l + e0).
struct KeyPoly {
    double c2, c1, c0;
    double e2, e1, e0;
};

__device__ __forceinline__ KeyPoly key_poly(const double R[9]) {
    double f2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) f2 = fma(R[k], R[k], f2);
    const double p48 = R[4] * R[8], p57 = R[5] * R[7], p38 = R[3] * R[8], p56 = R[5] * R[6];
    const double p37 = R[3] * R[7], p46 = R[4] * R[6];
    const double detR = R[0] * (p48 - p57) - R[1] * (p38 - p56) + R[2] * (p37 - p46);
    const double m1 = fabs(R[0]) * (fabs(p48) + fabs(p57)) + fabs(R[1]) * (fabs(p38) + fabs(p56)) +
                      fabs(R[2]) * (fabs(p37) + fabs(p46));
    double N[4][4];
    horn_key(R, N);
    // det N over the 2x2 minors of rows (0,1) and (2,3), with the sum of their absolute products
    double c0 = 0.0, M0 = 0.0;
    constexpr int ja[6] = {0, 0, 0, 1, 1, 2}, jb[6] = {1, 2, 3, 2, 3, 3};
    constexpr double sg[6] = {1.0, -1.0, 1.0, 1.0, -1.0, 1.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a0 = ja[k], b0 = jb[k], a1 = ja[5 - k], b1 = jb[5 - k];
        const double s1 = N[0][a0] * N[1][b0], s2 = N[1][a0] * N[0][b0];
        const double t1 = N[2][a1] * N[3][b1], t2 = N[3][a1] * N[2][b1];
        c0 = fma(sg[k] * (s1 - s2), t1 - t2, c0);
        M0 = fma(fabs(s1) + fabs(s2), fabs(t1) + fabs(t2), M0);
    }
    KeyPoly k;
    k.c2 = -2.0 * f2;
    k.c1 = -8.0 * detR;
    k.c0 = c0;
    k.e2 = 14.0 * fabs(k.c2);
    k.e1 = 4.0 * fabs(k.c1) + 48.0 * m1;
    k.e0 = 4.0 * fabs(c0) + 10.0 * M0;
    return k;
}

// One Laguerre step on P from lam (above the largest root).  good: the step is defined (else it is
// not taken); conv: the step was below stop or P(lam) within its rounding bound.
__device__ __forceinline__ void key_root_step(const KeyPoly& k, double& lam, double stop, bool& good, bool& conv) {
    constexpr double u = 0x1p-53;
    const double l2 = lam * lam;
    const double p = (l2 + k.c2) * l2 + k.c1 * lam + k.c0;
    const double dp = (4.0 * l2 + 2.0 * k.c2) * lam + k.c1;
    const double ddp = 12.0 * l2 + 2.0 * k.c2;
    const double eta = u * (((4.0 * l2 + k.e2) * lam + k.e1) * lam + k.e0);
    const double H = 3.0 * (3.0 * dp * dp - 4.0 * p * ddp);   // >= 0 for real roots (rounding: clamped)
    // (the square root and the quotient from the hardware approximations with one Newton-Raphson
    // correction each: the iteration corrects any small error of a step, and both the stopping
    // test on P and the acceptance below evaluate P exactly)
    // (branch-free: H <= 0 gives an infinite or NaN reciprocal root, replaced by a zero root)
    const double y = __builtin_amdgcn_rsq(H);
    double sh = H * y;
    sh = fma(0.5 * sh, fma(-sh, y, 1.0), sh);
    sh = H > 0.0 ? sh : 0.0;
    const double den = dp + sh;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    const double step = 4.0 * p * r;
    good = den > 0.0;
    conv = good & ((fabs(step) <= stop) | (fabs(p) <= eta));
    lam = good ? lam - step : lam;
}

// The a-posteriori check of a settled root: the exact root within tol E0 of lam.
__device__ __forceinline__ bool key_root_ok(const KeyPoly& k, double lam, double E0, double tol) {
    constexpr double u = 0x1p-53;
    const double l2 = lam * lam;
    const double p = (l2 + k.c2) * l2 + k.c1 * lam + k.c0;
    const double dp = (4.0 * l2 + 2.0 * k.c2) * lam + k.c1;
    const double eta = u * (((4.0 * l2 + k.e2) * lam + k.e1) * lam + k.e0);
    return dp > 0.0 && fabs(p) + eta <= tol * E0 * dp;
}

// The stopping step for a tolerance: with cubic convergence, after a step of 1e-3 tol the error is
// far below tol.
__device__ __forceinline__ double key_stop(double E0, double tol) { return fmax(1e-15, 1e-3 * tol) * E0; }

__device__ inline double rmsd2_from_corr64(const double R[9], double Ga, double Gb, int A, double tol = 1e-13) {
    const KeyPoly k = key_poly(R);
    const double E0 = 0.5 * (Ga + Gb), stop = key_stop(E0, tol);
    double lam = E0;
    bool settled = false;
    for (int it = 0; it < kRootSteps; ++it) {
        bool good, conv;
        key_root_step(k, lam, stop, good, conv);
        if (!good | conv) {
            settled = conv;
            break;
        }
    }
    if (!(settled && key_root_ok(k, lam, E0, tol)))
        lam = key_max_eig_jacobi(R[0], R[1], R[2], R[3], R[4], R[5], R[6], R[7], R[8]);
    const double r2 = (Ga + Gb - 2.0 * lam) / A;
    return r2 > 0.0 ? r2 : 0.0;
}

// FP64 RMSD kernel between two centred frames (AoS rows x0 y0 z0 x1 ...).
template <typename TA, typename TB>
__device__ inline double rmsd_kfun64(const TA* __restrict__ a, const TB* __restrict__ b, int A, double inv2s2) {
    double R[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double Ga = 0.0, Gb = 0.0;
    // unrolled so that the loads of several atoms are in flight together (the sums stay in order)
#pragma unroll 8
    for (int t = 0; t < A; ++t) {
        const double ax = a[3 * t], ay = a[3 * t + 1], az = a[3 * t + 2];
        const double bx = b[3 * t], by = b[3 * t + 1], bz = b[3 * t + 2];
        R[0] = fma(ax, bx, R[0]); R[1] = fma(ax, by, R[1]); R[2] = fma(ax, bz, R[2]);
        R[3] = fma(ay, bx, R[3]); R[4] = fma(ay, by, R[4]); R[5] = fma(ay, bz, R[5]);
        R[6] = fma(az, bx, R[6]); R[7] = fma(az, by, R[7]); R[8] = fma(az, bz, R[8]);
        Ga = fma(ax, ax, fma(ay, ay, fma(az, az, Ga)));
        Gb = fma(bx, bx, fma(by, by, fma(bz, bz, Gb)));
    }
    return ::exp(-rmsd2_from_corr64(R, Ga, Gb, A) * inv2s2);
}

// K(a, b) in FP64 for any kernel type (RMSD rows must be centred).
template <typename TA, typename TB>
__device__ inline double k64(const KSpec& ks, const TA* __restrict__ a, const TB* __restrict__ b) {
    if (ks.type == KKM_KERNEL_RMSD) return rmsd_kfun64(a, b, ks.n_atoms, ks.inv2s2);
    return kfun64_rows(ks.type, a, b, ks.d, ks.inv2s2);
}

// K(a, b) in FP64 for rows of length ks.d <= DP (linear / RBF), in chunks of 16 dimensions.  Every
// load of a chunk is issued unconditionally (an index past the row end is clamped to its last
// element and the value masked to zero afterwards), so the chunk's loads are in flight together
// instead of one branch and one wait per element; the live registers stay bounded by the chunk.
// Rows of at most 16 dimensions take one chunk and no loop, so that the loads of several calls in a
// row can be in flight together too.  Masked dimensions add fma(0, 0, acc) = acc exactly, so the
// sum is the plain one in order.  DP == 0 (RMSD) falls back to k64.
template <int DP, typename TA, typename TB>
__device__ __forceinline__ double k64p(const KSpec& ks, const TA* __restrict__ a, const TB* __restrict__ b) {
    if constexpr (DP == 0) {
        return k64(ks, a, b);
    } else {
        constexpr int CH = DP < 16 ? DP : 16;
        const int d = (int)ks.d;   // 1 <= d <= DP
        const bool lin = ks.type == KKM_KERNEL_LINEAR;
        double acc = 0.0;
        auto chunk = [&](int c0) {
            double va[CH], vb[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int i = min(c0 + k, d - 1);
                const double x = (double)a[i], y = (double)b[i];
                const bool in = c0 + k < d;
                va[k] = in ? x : 0.0;
                vb[k] = in ? y : 0.0;
            }
            if (lin) {
#pragma unroll
                for (int k = 0; k < CH; ++k) acc = fma(va[k], vb[k], acc);
            } else {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const double t = va[k] - vb[k];
                    acc = fma(t, t, acc);
                }
            }
        };
        if constexpr (DP <= 16) {
            chunk(0);
        } else {
#pragma unroll 1
            for (int c0 = 0; c0 < d; c0 += CH) chunk(c0);
        }
        return lin ? acc : ::exp(-acc * ks.inv2s2);
    }
}

// Margin below which a label need not be re-decided: the exact relative margin is then provably
// under 5e-7 (labels are only promised to equal the exact ones where it exceeds 1e-6).
constexpr double kTieMargin = 5e-7;

// Compile-time row length for k64p: the padded dimension for linear / RBF, 0 for RMSD.
inline int eval_dp(int ktype, int64_t d) { return ktype == KKM_KERNEL_RMSD ? 0 : padded_dim(d); }

// Calls F.template operator()<DP>() for the DP of eval_dp.
template <typename F>
inline kkm_status dispatch_dp(int dp, F&& f) {
    switch (dp) {
        case 0: return f.template operator()<0>();
        case 4: return f.template operator()<4>();
        case 8: return f.template operator()<8>();
        case 16: return f.template operator()<16>();
        case 32: return f.template operator()<32>();
        case 64: return f.template operator()<64>();
        case 128: return f.template operator()<128>();
        default: return KKM_ERR_INTERNAL;
    }
}

// K(a, a) in FP64.
template <typename TA>
__device__ inline double kself64(const KSpec& ks, const TA* __restrict__ a) {
    if (ks.type != KKM_KERNEL_LINEAR) return 1.0;
    double acc = 0.0;
    for (int64_t k = 0; k < ks.d; ++k) acc = fma((double)a[k], (double)a[k], acc);
    return acc;
}

}  // namespace kkm
