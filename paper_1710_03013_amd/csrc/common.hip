// Host-side plumbing of libkkm: thread-local errors, device facts, the random-draw specification
// and the model lifecycle (create / load / export / free).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "kkm_internal.hpp"
#include "kkm_launch.hpp"

namespace kkm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

kkm_status fail(kkm_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

kkm_status device_info(DeviceInfo* out) {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = -1;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(KKM_ERR_DEVICE, "no HIP device available");
    KKM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    if (cache[dev].device != dev) {
        hipDeviceProp_t p;
        KKM_HIP(hipGetDeviceProperties(&p, dev));
        DeviceInfo di;
        di.device = dev;
        di.num_cus = p.multiProcessorCount;
        di.max_lds_per_block = p.sharedMemPerBlock;
        int coop = 0;
        KKM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        di.coop = coop != 0;
        cache[dev] = di;
    }
    *out = cache[dev];
    return KKM_OK;
}

kkm_status allow_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 65536) return KKM_OK;
    // raise a kernel's dynamic-LDS limit once per device and kernel, to the largest size asked for
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> raised;
    int dev = 0;
    KKM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    size_t& have = raised[{dev, fn}];
    if (bytes <= have) return KKM_OK;
    KKM_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
    return KKM_OK;
}

// ----------------------------------------------------------------------------- draws
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) streams keyed by (seed, purpose, batch); bounded
// integers by Lemire's multiply-shift with rejection; uniforms as (r >> 11) * 2^-53.
namespace rng {
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
struct Stream {
    uint64_t state;
    uint64_t next() { return mix64(state += kGolden); }
    uint64_t bounded(uint64_t n) {
        uint64_t x = next();
        unsigned __int128 m = (unsigned __int128)x * n;
        uint64_t low = (uint64_t)m;
        if (low < n) {
            const uint64_t threshold = (0 - n) % n;
            while (low < threshold) {
                x = next();
                m = (unsigned __int128)x * n;
                low = (uint64_t)m;
            }
        }
        return (uint64_t)(m >> 64);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};
inline Stream stream(uint64_t seed, uint64_t purpose, uint64_t batch) {
    uint64_t key = mix64(seed + kGolden * (1 + purpose));
    key = mix64(key + kGolden * (1 + batch));
    return Stream{key};
}
constexpr uint64_t kLandmarks = 0, kInitLabels = 1, kKmeanspp = 2;
}  // namespace rng

}  // namespace kkm

using namespace kkm;

extern "C" {

int64_t kkm_landmark_count(int64_t n, double s) {
    if (n <= 0 || !(s > 0.0)) return 0;
    double l = std::floor(s * (double)n + 0.5);
    if (l < 1.0) l = 1.0;
    if (l > (double)n) l = (double)n;
    return (int64_t)l;
}

kkm_status kkm_draw_landmarks(uint64_t seed, int32_t batch, int64_t n, double s, int64_t* out) {
    if (!out || n <= 0 || !(s > 0.0 && s <= 1.0) || batch < 0) return fail(KKM_ERR_INVALID_ARG, "kkm_draw_landmarks: bad argument");
    const int64_t ell = kkm_landmark_count(n, s);
    if (ell == n) {
        for (int64_t i = 0; i < n; ++i) out[i] = i;
        return KKM_OK;
    }
    // partial Fisher-Yates shuffle of 0..n-1 (first ell positions), then the picks in ascending
    // order via a bitmap over 0..n-1; the buffers are kept per thread between calls
    rng::Stream g = rng::stream(seed, rng::kLandmarks, (uint64_t)batch);
    static thread_local std::vector<int64_t> idx;
    static thread_local std::vector<uint64_t> bits;
    if ((int64_t)idx.size() < n) idx.resize(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    for (int64_t k = 0; k < ell; ++k) {
        const int64_t r = k + (int64_t)g.bounded((uint64_t)(n - k));
        std::swap(idx[k], idx[r]);
    }
    const int64_t nw = (n + 63) / 64;
    bits.assign(nw, 0ull);
    for (int64_t k = 0; k < ell; ++k) bits[idx[k] >> 6] |= 1ull << (idx[k] & 63);
    int64_t o = 0;
    for (int64_t wi = 0; wi < nw; ++wi)
        for (uint64_t b = bits[wi]; b; b &= b - 1) out[o++] = wi * 64 + __builtin_ctzll(b);
    return KKM_OK;
}

kkm_status kkm_draw_kmpp_uniforms(uint64_t seed, int32_t C, double* out) {
    if (!out || C <= 0) return fail(KKM_ERR_INVALID_ARG, "kkm_draw_kmpp_uniforms: bad argument");
    rng::Stream g = rng::stream(seed, rng::kKmeanspp, 0);
    for (int32_t k = 0; k < C; ++k) out[k] = g.uniform();
    return KKM_OK;
}

kkm_status kkm_draw_init_labels(uint64_t seed, int64_t n, int32_t C, int32_t* out) {
    if (!out || n <= 0 || C <= 0) return fail(KKM_ERR_INVALID_ARG, "kkm_draw_init_labels: bad argument");
    rng::Stream g = rng::stream(seed, rng::kInitLabels, 0);
    for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)g.bounded((uint64_t)C);
    return KKM_OK;
}

const char* kkm_last_error(void) { return g_last_error.c_str(); }

const char* kkm_version(void) { return "libkkm 0.1 (gfx950)"; }

// ----------------------------------------------------------------------------- models
static kkm_status check_kernel(const kkm_kernel* k, int64_t d) {
    if (!k) return fail(KKM_ERR_INVALID_ARG, "kernel is NULL");
    if (k->type != KKM_KERNEL_LINEAR && k->type != KKM_KERNEL_RBF && k->type != KKM_KERNEL_RMSD)
        return fail(KKM_ERR_INVALID_ARG, "unknown kernel type");
    if (k->type != KKM_KERNEL_LINEAR && !(k->sigma > 0.0 && std::isfinite(k->sigma)))
        return fail(KKM_ERR_INVALID_ARG, "sigma must be finite and > 0");
    if (k->type == KKM_KERNEL_RMSD && (k->n_atoms < 1 || d != 3 * (int64_t)k->n_atoms))
        return fail(KKM_ERR_INVALID_ARG, "RMSD kernel needs d == 3 * n_atoms");
    return KKM_OK;
}

}  // extern "C"

namespace kkm {
void model_layout(kkm_model* m, Carver& c) {
    const size_t es = m->dtype == KKM_F64 ? 8 : 4;
    const size_t rows = (size_t)m->cap + 32;   // the matrix-core pass reads whole 32-row tiles
    const int C = m->C;
    m->support = c.take<char>(rows * m->dpad * es);
    m->snorm32 = c.take<float>(rows);
    m->snorm64 = c.take<double>(rows);
    m->coef32 = c.take<float>(rows);
    m->coef64 = c.take<double>(rows);
    m->pan = m->dtype == KKM_F32 ? c.take<float>(panel_rows(rows) * m->dpad) : nullptr;
    m->hi = c.take<uint16_t>(panel_rows(rows) * m->bpad);
    m->lo = c.take<uint16_t>(panel_rows(rows) * m->bpad);
    m->offsets = c.take<int32_t>(C + 1);
    m->self = c.take<double>(C);
    m->segabs = c.take<double>(C);
    m->snorm_max = c.take<float>(1);
    m->split = c.take<int32_t>(5);
    m->counts = c.take<int64_t>(C);
    m->medoid_index = c.take<int64_t>(C);
}
}  // namespace kkm

extern "C" {

kkm_status kkm_model_create(const kkm_kernel* kernel, int64_t d, int32_t C, int64_t max_support, int32_t dtype,
                            kkm_model** out) {
    if (!out) return fail(KKM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    KKM_TRY(check_kernel(kernel, d));
    if (d < 1) return fail(KKM_ERR_INVALID_ARG, "d must be >= 1");
    if (C < 1 || C > kMaxClusters) return fail(KKM_ERR_INVALID_ARG, "C out of range [1, 1024]");
    if (max_support < 1) return fail(KKM_ERR_INVALID_ARG, "max_support must be >= 1");
    if (dtype != KKM_F32 && dtype != KKM_F64) return fail(KKM_ERR_INVALID_ARG, "bad dtype");
    if (kernel->type != KKM_KERNEL_RMSD && d > kMaxRegDim)
        return fail(KKM_ERR_UNSUPPORTED, "linear / RBF models support d <= 128");
    DeviceInfo dev;
    KKM_TRY(device_info(&dev));
    kkm_model* m = new kkm_model();
    m->kernel = *kernel;
    m->d = d;
    m->dpad = kernel->type == KKM_KERNEL_RMSD ? (int32_t)d : padded_dim(d);
    m->bpad = bf16_pad(m->dpad);
    m->C = C;
    m->cap = max_support;
    m->used = 0;
    m->dtype = dtype;
    m->device = dev.device;
    Carver cv(nullptr);
    auto layout = [&](Carver& c) { model_layout(m, c); };
    layout(cv);
    void* block = nullptr;
    hipError_t e = hipMalloc(&block, cv.off);
    if (e != hipSuccess) {
        delete m;
        return fail(KKM_ERR_DEVICE, std::string("hipMalloc for the model failed: ") + hipGetErrorString(e));
    }
    e = hipMemset(block, 0, cv.off);
    if (e != hipSuccess) {
        hipFree(block);
        delete m;
        return fail(KKM_ERR_DEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    m->block = block;
    Carver c2(block);
    layout(c2);
    // an empty model: every cluster disabled
    std::vector<double> inf(C, kInf);
    std::vector<int32_t> zoff(C + 1, 0);
    std::vector<int64_t> minus(C, -1);
    e = hipMemcpy(m->self, inf.data(), sizeof(double) * C, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->offsets, zoff.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->medoid_index, minus.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(block);
        delete m;
        return fail(KKM_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = m;
    return KKM_OK;
}

kkm_status kkm_model_load(kkm_model* m, const void* support, int64_t n_support, const int64_t* offsets,
                          const double* coef) {
    if (!m || !support || !offsets || !coef) return fail(KKM_ERR_INVALID_ARG, "kkm_model_load: NULL argument");
    if (n_support < 0 || n_support > m->cap) return fail(KKM_ERR_INVALID_ARG, "n_support exceeds the model capacity");
    if (offsets[0] != 0 || offsets[m->C] != n_support) return fail(KKM_ERR_INVALID_ARG, "offsets must run from 0 to n_support");
    for (int j = 0; j < m->C; ++j)
        if (offsets[j + 1] < offsets[j]) return fail(KKM_ERR_INVALID_ARG, "offsets must be non-decreasing");
    int32_t nonneg = 1;
    for (int64_t l = 0; l < n_support; ++l) {
        if (!std::isfinite(coef[l])) return fail(KKM_ERR_NONFINITE, "non-finite coefficient");
        if (coef[l] < 0.0) nonneg = 0;
    }
    const size_t es = m->dtype == KKM_F64 ? 8 : 4;
    std::vector<char> rows((size_t)std::max<int64_t>(1, n_support) * m->dpad * es, 0);
    for (int64_t l = 0; l < n_support; ++l) {
        const char* src = static_cast<const char*>(support) + (size_t)l * m->d * es;
        for (int64_t c = 0; c < m->d; ++c) {
            double v = m->dtype == KKM_F64 ? reinterpret_cast<const double*>(src)[c] : reinterpret_cast<const float*>(src)[c];
            if (!std::isfinite(v)) return fail(KKM_ERR_NONFINITE, "non-finite support value");
        }
        std::memcpy(rows.data() + (size_t)l * m->dpad * es, src, (size_t)m->d * es);
    }
    if (m->kernel.type == KKM_KERNEL_RMSD) {   // centre the frames on the host (load is not a hot path)
        const int A = m->kernel.n_atoms;
        for (int64_t l = 0; l < n_support; ++l) {
            char* r = rows.data() + (size_t)l * m->dpad * es;
            for (int ax = 0; ax < 3; ++ax) {
                double c = 0.0;
                for (int a = 0; a < A; ++a)
                    c += m->dtype == KKM_F64 ? reinterpret_cast<double*>(r)[3 * a + ax] : reinterpret_cast<float*>(r)[3 * a + ax];
                c /= A;
                for (int a = 0; a < A; ++a) {
                    if (m->dtype == KKM_F64) reinterpret_cast<double*>(r)[3 * a + ax] -= c;
                    else reinterpret_cast<float*>(r)[3 * a + ax] = (float)((double)reinterpret_cast<float*>(r)[3 * a + ax] - c);
                }
            }
        }
    }
    std::vector<int32_t> off32(m->C + 1);
    for (int j = 0; j <= m->C; ++j) off32[j] = (int32_t)offsets[j];
    int cur = -1;
    KKM_HIP(hipGetDevice(&cur));
    if (cur != m->device) KKM_HIP(hipSetDevice(m->device));
    KKM_HIP(hipMemcpy(m->support, rows.data(), (size_t)n_support * m->dpad * es, hipMemcpyHostToDevice));
    if (n_support > 0) KKM_HIP(hipMemcpy(m->coef64, coef, sizeof(double) * n_support, hipMemcpyHostToDevice));
    KKM_HIP(hipMemcpy(m->offsets, off32.data(), sizeof(int32_t) * (m->C + 1), hipMemcpyHostToDevice));
    std::vector<int64_t> zero(m->C, 0), minus(m->C, -1);
    KKM_HIP(hipMemcpy(m->counts, zero.data(), sizeof(int64_t) * m->C, hipMemcpyHostToDevice));
    KKM_HIP(hipMemcpy(m->medoid_index, minus.data(), sizeof(int64_t) * m->C, hipMemcpyHostToDevice));
    m->used = n_support;
    m->nonneg = nonneg;
    int32_t medoids = n_support == m->C ? 1 : 0;   // one row per cluster, in cluster order, coefficient 1
    for (int j = 0; medoids && j < m->C; ++j) medoids = offsets[j] == j && coef[j] == 1.0;
    m->medoid_form = medoids;
    KKM_TRY(launch_model_prepare(m, nullptr));
    KKM_HIP(hipDeviceSynchronize());
    if (cur != m->device) KKM_HIP(hipSetDevice(cur));
    return KKM_OK;
}

kkm_status kkm_model_export(const kkm_model* m, void* support, int64_t* offsets, double* coef, double* self,
                            int64_t* counts, int64_t* medoid_index) {
    if (!m) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    const size_t es = m->dtype == KKM_F64 ? 8 : 4;
    if (support && m->used > 0) {
        std::vector<char> rows((size_t)m->used * m->dpad * es);
        KKM_HIP(hipMemcpy(rows.data(), m->support, rows.size(), hipMemcpyDeviceToHost));
        for (int64_t l = 0; l < m->used; ++l)
            std::memcpy(static_cast<char*>(support) + (size_t)l * m->d * es, rows.data() + (size_t)l * m->dpad * es,
                        (size_t)m->d * es);
    }
    if (offsets) {
        std::vector<int32_t> o(m->C + 1);
        KKM_HIP(hipMemcpy(o.data(), m->offsets, sizeof(int32_t) * (m->C + 1), hipMemcpyDeviceToHost));
        for (int j = 0; j <= m->C; ++j) offsets[j] = o[j];
    }
    if (coef && m->used > 0) KKM_HIP(hipMemcpy(coef, m->coef64, sizeof(double) * m->used, hipMemcpyDeviceToHost));
    if (self) KKM_HIP(hipMemcpy(self, m->self, sizeof(double) * m->C, hipMemcpyDeviceToHost));
    if (counts) KKM_HIP(hipMemcpy(counts, m->counts, sizeof(int64_t) * m->C, hipMemcpyDeviceToHost));
    if (medoid_index) KKM_HIP(hipMemcpy(medoid_index, m->medoid_index, sizeof(int64_t) * m->C, hipMemcpyDeviceToHost));
    return KKM_OK;
}

kkm_status kkm_model_shape(const kkm_model* m, int64_t* d, int32_t* C, int64_t* n_used) {
    if (!m) return fail(KKM_ERR_INVALID_ARG, "model is NULL");
    if (d) *d = m->d;
    if (C) *C = m->C;
    if (n_used) *n_used = m->used;
    return KKM_OK;
}

void kkm_model_free(kkm_model* m) {
    if (!m) return;
    if (m->block) (void)hipFree(m->block);
    delete m;
}

}  // extern "C"
