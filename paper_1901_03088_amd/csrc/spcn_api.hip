// spcn_api.hip -- host side of the C ABI declared in include/spcn.h: argument validation,
// workspace layout, error reporting and dispatch to the kernel launchers.
#include "spcn_internal.h"

#include <atomic>
#include <math.h>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

namespace spcn {

static thread_local char g_err[512];

// option id -> (value, min, max)
constexpr int N_OPT = 4;
static std::atomic<int> g_opt[N_OPT] = {{6}, {3}, {8}, {15}};   // fastest measured on a 2-gigapixel slide
static const int g_opt_lo[N_OPT] = {0, 0, 1, 12};
static const int g_opt_hi[N_OPT] = {9, 5, 16, 18};

int option(int id) { return (id >= 0 && id < N_OPT) ? g_opt[id].load(std::memory_order_relaxed) : 0; }

spcn_status fail(spcn_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

spcn_status hip_fail(hipError_t e, const char* what) {
    return fail(SPCN_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Compute-unit count of the current device, queried once per device (thread-safe: a relaxed atomic
// per device, 0 until known; concurrent first calls may both query, and store the same value).
spcn_status dev_info(DevInfo* out) {
    static std::atomic<int> cached_cus[64];
    int id = 0;
    hipError_t e = hipGetDevice(&id);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (id < 0 || id >= 64) return fail(SPCN_E_UNSUPPORTED, "device id %d out of range", id);
    int cus = cached_cus[id].load(std::memory_order_relaxed);
    if (cus == 0) {
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, id);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(MultiprocessorCount)");
        cus = cus > 0 ? cus : 1;
        cached_cus[id].store(cus, std::memory_order_relaxed);
    }
    out->id = id;
    out->cus = cus;
    return SPCN_OK;
}

ParamsK make_params(const spcn_params* p) {
    ParamsK k{};
    for (int c = 0; c < 3; ++c) k.i0[c] = p->i0[c];
    k.lambda = p->lambda;
    k.white_sum = p->white_sum;
    k.q = p->percentile / 100.0f;
    k.q64 = (double)p->percentile / 100.0;
    k.hist_hi[0] = p->hist_hi[0];
    k.hist_hi[1] = p->hist_hi[1];
    k.hist_hi_dev = p->hist_hi_dev;
    k.auto_range = p->auto_range;
    return k;
}

static bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

static bool pow2(float x) {
    if (!finite_pos(x)) return false;
    int e;
    float m = frexpf(x, &e);
    return m == 0.5f;
}

static spcn_status check_params(const spcn_params* p, bool u8_input) {
    if (!p) return fail(SPCN_E_ARG, "params is NULL");
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(p->i0[c])) return fail(SPCN_E_ARG, "i0[%d] = %g must be finite and > 0", c, (double)p->i0[c]);
    if (u8_input)
        for (int c = 0; c < 3; ++c)
            if (p->i0[c] > 65536.0f) return fail(SPCN_E_ARG, "i0[%d] = %g too large", c, (double)p->i0[c]);
    if (!(isfinite(p->lambda) && p->lambda >= 0.0f))
        return fail(SPCN_E_ARG, "lambda = %g must be finite and >= 0", (double)p->lambda);
    if (!(isfinite(p->percentile) && p->percentile > 0.0f && p->percentile <= 100.0f))
        return fail(SPCN_E_ARG, "percentile = %g must lie in (0, 100]", (double)p->percentile);
    for (int j = 0; j < 2; ++j) {
        if (!pow2(p->hist_hi[j]) || p->hist_hi[j] < 0.00390625f || p->hist_hi[j] > 256.0f)
            return fail(SPCN_E_ARG, "hist_hi[%d] = %g must be a power of two in [2^-8, 2^8]", j,
                        (double)p->hist_hi[j]);
    }
    if (p->auto_range != 0 && p->auto_range != 1) return fail(SPCN_E_ARG, "auto_range = %d must be 0 or 1",
                                                              (int)p->auto_range);
    if (((uintptr_t)p->hist_hi_dev) & 3) return fail(SPCN_E_ARG, "hist_hi_dev must be 4-byte aligned");
    return SPCN_OK;
}

static spcn_status check_image(const void* ptr, int64_t height, int64_t width, const char* name) {
    if (!ptr) return fail(SPCN_E_ARG, "%s is NULL", name);
    if (height <= 0 || width <= 0) return fail(SPCN_E_ARG, "%s: height and width must be > 0 (got %lld x %lld)",
                                               name, (long long)height, (long long)width);
    if (height > ((int64_t)1 << 36) / width) return fail(SPCN_E_ARG, "%s: more than 2^36 pixels", name);
    if (((uintptr_t)ptr) & 3) return fail(SPCN_E_ARG, "%s must be 4-byte aligned", name);
    return SPCN_OK;
}

static spcn_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return SPCN_OK;
    if (!ws) return fail(SPCN_E_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
    if (ws_bytes < need) return fail(SPCN_E_WORKSPACE, "workspace has %zu bytes, need %zu", ws_bytes, need);
    if (((uintptr_t)ws) & 255) return fail(SPCN_E_WORKSPACE, "workspace must be 256-byte aligned");
    return SPCN_OK;
}

}  // namespace spcn

using namespace spcn;

#define SPCN_CHECK(x)                         \
    do {                                      \
        spcn_status s_ = (x);                 \
        if (s_ != SPCN_OK) return s_;         \
    } while (0)

extern "C" {

void spcn_default_params(spcn_params* p) {
    if (!p) return;
    for (int c = 0; c < 3; ++c) p->i0[c] = 255.0f;
    p->lambda = 0.01f;
    p->white_sum = 660;
    p->percentile = 99.0f;
    p->hist_hi[0] = 4.0f;
    p->hist_hi[1] = 4.0f;
    p->hist_hi_dev = nullptr;
    p->auto_range = 1;
}

size_t spcn_workspace_size(int op, int64_t n_px, int64_t n_items, int64_t n_samples) {
    if (n_px < 0 || n_items < 0 || n_samples < 0) return 0;
    switch (op) {
        case SPCN_OP_DENSITIES:
        case SPCN_OP_NORMALIZE:
            return u8_workspace_bytes();
        case SPCN_OP_ESTIMATE_BASIS:
            return basis_workspace_bytes(n_samples);
        case SPCN_OP_ESTIMATE_BATCHED:
            return basis_batched_workspace_bytes(n_items, n_samples);
        case SPCN_OP_NORMALIZE_BATCHED:
            return batched_workspace_bytes(n_items, n_px);
        case SPCN_OP_FORWARD_F32:
            return f32_forward_workspace_bytes(n_px, n_items);
        case SPCN_OP_BACKWARD_F32:
            return f32_backward_workspace_bytes(n_px, n_items);
        case SPCN_OP_ESTIMATE_I0:
            return n_samples <= kMaxI0Samples ? i0_workspace_bytes(n_samples) : 0;
        case SPCN_OP_SAMPLE_PERCENTILE:
            return n_samples <= kMaxI0Samples ? sample_pctl_workspace_bytes(n_samples) : 0;
        case SPCN_OP_BAND_PERCENTILES:
            return n_items <= kMaxBands ? band_workspace_bytes(n_items) : 0;
        case SPCN_OP_STREAM_NORMALIZE:
            return stream_workspace_bytes(n_px, n_items);
        case SPCN_OP_BANDWIDTH_PROBE:
            return probe_sink_bytes();
        case SPCN_OP_EXACT_PERCENTILE:
            return exact_workspace_bytes();
        default:
            return 0;
    }
}

spcn_status spcn_densities(const uint8_t* img, int64_t height, int64_t width, const float* w,
                           const spcn_params* p, float* h_out, uint64_t* hist_out, float* p99_out,
                           int32_t* flags_out, float* hist_hi_out, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    SPCN_CHECK(check_params(p, true));
    if (!w) return fail(SPCN_E_ARG, "w is NULL");
    if (!hist_out) return fail(SPCN_E_ARG, "hist_out is NULL");
    if (h_out && (((uintptr_t)h_out) & 15)) return fail(SPCN_E_ARG, "h_out must be 16-byte aligned");
    SPCN_CHECK(check_ws(ws, ws_bytes, u8_workspace_bytes()));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_densities(img, height * width, w, make_params(p), h_out, hist_out, p99_out, flags_out,
                                    hist_hi_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_densities launch");
    return SPCN_OK;
}

}  // extern "C"

// spcn_normalize's host-side argument checks (everything but the workspace).
static spcn_status check_normalize(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                                   const float* w_tgt, const float* scale_tgt, const float* i0_out,
                                   const spcn_params* p, uint8_t* out) {
    SPCN_CHECK(check_image(src, height, width, "src"));
    SPCN_CHECK(check_image(out, height, width, "out"));
    SPCN_CHECK(check_params(p, true));
    if (!w_src || !w_tgt || !scale_tgt) return fail(SPCN_E_ARG, "w_src, w_tgt and scale_tgt must be non-NULL");
    const int64_t n = height * width;
    if ((const void*)src < (const void*)(out + 3 * n) && (const void*)out < (const void*)(src + 3 * n))
        return fail(SPCN_E_ARG, "out must not overlap src");
    for (int c = 0; c < 3; ++c) {
        const float io = i0_out ? i0_out[c] : p->i0[c];
        if (!finite_pos(io)) return fail(SPCN_E_ARG, "i0_out[%d] = %g must be finite and > 0", c, (double)io);
    }
    return SPCN_OK;
}

// spcn_normalize's checks and launches, with the workspace the caller or the library provides.
static spcn_status normalize_into(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                                  const float* w_tgt, const float* scale_tgt, const float* i0_out,
                                  const spcn_params* p, uint8_t* out, const spcn_norm_stats* st,
                                  void* ws, size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_normalize(src, height, width, w_src, w_tgt, scale_tgt, i0_out, p, out));
    const int64_t n = height * width;
    float io[3];
    for (int c = 0; c < 3; ++c) io[c] = i0_out ? i0_out[c] : p->i0[c];
    SPCN_CHECK(check_ws(ws, ws_bytes, u8_workspace_bytes()));
    uint64_t* hist = st && st->hist ? st->hist : static_cast<uint64_t*>(ws);
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_normalize(src, n, w_src, w_tgt, scale_tgt, io, make_params(p), out, hist, ws,
                                    st ? st->p99_src : nullptr, st ? st->scale : nullptr,
                                    st ? st->flags : nullptr, st ? st->hist_hi : nullptr, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_normalize launch");
    return SPCN_OK;
}

extern "C" {

spcn_status spcn_normalize(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                           const float* w_tgt, const float* scale_tgt, const float* i0_out,
                           const spcn_params* p, uint8_t* out, const spcn_norm_stats* st,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
    return normalize_into(src, height, width, w_src, w_tgt, scale_tgt, i0_out, p, out, st, ws, ws_bytes, stream);
}

// Scratch of spcn_normalize_noalloc: the histogram and range words of one normalisation (the same
// layout as the caller workspace of spcn_normalize).  Every device holds its own copy for the life
// of the process; its device address is looked up once per device (the array's name is only a
// host-side stand-in) and kept in g_scratch.
constexpr size_t kStaticScratchBytes = 8192;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];
static std::atomic<void*> g_scratch[64];
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (dev is the current device).
static spcn_status scratch_address(int dev, void** out) {
    void* ptr = g_scratch[dev].load(std::memory_order_acquire);
    if (!ptr) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ptr = g_scratch[dev].load(std::memory_order_relaxed);
        if (!ptr) {
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            if (!ptr) return fail(SPCN_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
            g_scratch[dev].store(ptr, std::memory_order_release);
        }
    }
    *out = ptr;
    return SPCN_OK;
}

spcn_status spcn_normalize_noalloc(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                                   const float* w_tgt, const float* scale_tgt, const float* i0_out,
                                   const spcn_params* p, uint8_t* out, const spcn_norm_stats* st,
                                   hipStream_t stream) {
    SPCN_CHECK(check_normalize(src, height, width, w_src, w_tgt, scale_tgt, i0_out, p, out));
    const size_t need = u8_workspace_bytes();
    if (need > kStaticScratchBytes)
        return fail(SPCN_E_WORKSPACE, "spcn_normalize_noalloc needs %zu bytes of scratch, above its static %zu",
                    need, kStaticScratchBytes);
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    void* ws = nullptr;
    SPCN_CHECK(scratch_address(dev.id, &ws));
    return normalize_into(src, height, width, w_src, w_tgt, scale_tgt, i0_out, p, out, st, ws, kStaticScratchBytes,
                          stream);
}

spcn_status spcn_recolor(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                         const float* w_tgt, const float* scale_tgt, const float* i0_out,
                         const spcn_params* p, const uint64_t* hist, uint8_t* out,
                         const spcn_norm_stats* st, hipStream_t stream) {
    SPCN_CHECK(check_image(src, height, width, "src"));
    SPCN_CHECK(check_image(out, height, width, "out"));
    SPCN_CHECK(check_params(p, true));
    if (!w_src || !w_tgt || !scale_tgt || !hist)
        return fail(SPCN_E_ARG, "w_src, w_tgt, scale_tgt and hist must be non-NULL");
    const int64_t n = height * width;
    if ((const void*)src < (const void*)(out + 3 * n) && (const void*)out < (const void*)(src + 3 * n))
        return fail(SPCN_E_ARG, "out must not overlap src");
    float io[3];
    for (int c = 0; c < 3; ++c) io[c] = i0_out ? i0_out[c] : p->i0[c];
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(io[c])) return fail(SPCN_E_ARG, "i0_out[%d] = %g must be finite and > 0", c, (double)io[c]);
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_recolor(src, n, w_src, w_tgt, scale_tgt, io, make_params(p), out, hist,
                                  st ? st->p99_src : nullptr, st ? st->scale : nullptr, st ? st->flags : nullptr,
                                  st ? st->hist_hi : nullptr, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_recolor launch");
    return SPCN_OK;
}

static spcn_status check_fit(float lambda_nmf, int64_t n_samples, int32_t n_iter, int64_t max_samples) {
    if (!(isfinite(lambda_nmf) && lambda_nmf >= 0.0f))
        return fail(SPCN_E_ARG, "lambda_nmf = %g must be finite and >= 0", (double)lambda_nmf);
    if (n_samples < 1 || n_samples > max_samples)
        return fail(SPCN_E_ARG, "n_samples = %lld must lie in [1, %lld]", (long long)n_samples, (long long)max_samples);
    if (n_iter < 0 || n_iter > 100000) return fail(SPCN_E_ARG, "n_iter = %d must lie in [0, 100000]", (int)n_iter);
    return SPCN_OK;
}

spcn_status spcn_estimate_basis(const uint8_t* img, int64_t height, int64_t width, const spcn_params* p,
                                float lambda_nmf, int64_t n_samples, uint64_t seed, int32_t n_iter,
                                const float* w_init, float* w_out, float* sample_p99, float* hist_hi_out,
                                int32_t* flags_out,
                                void* ws, size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    SPCN_CHECK(check_params(p, true));
    SPCN_CHECK(check_fit(lambda_nmf, n_samples, n_iter, kMaxBasisSamples));
    if (!w_out) return fail(SPCN_E_ARG, "w_out is NULL");
    SPCN_CHECK(check_ws(ws, ws_bytes, basis_workspace_bytes(n_samples)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_estimate_basis(img, height * width, make_params(p), lambda_nmf, n_samples, seed, n_iter,
                                         w_init, w_out, sample_p99, hist_hi_out, flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_estimate_basis launch");
    return SPCN_OK;
}

spcn_status spcn_estimate_i0(const uint8_t* img, int64_t height, int64_t width, int64_t n_samples, uint64_t seed,
                             int32_t white_sum, float percentile, float* i0_out, int32_t* flags_out, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    if (n_samples < 1 || n_samples > kMaxI0Samples)
        return fail(SPCN_E_ARG, "n_samples = %lld must lie in [1, %lld]", (long long)n_samples, (long long)kMaxI0Samples);
    if (white_sum < 1 || white_sum > 765) return fail(SPCN_E_ARG, "white_sum = %d must lie in [1, 765]", (int)white_sum);
    if (!(percentile > 0.0f && percentile <= 100.0f))
        return fail(SPCN_E_ARG, "percentile = %g must lie in (0, 100]", (double)percentile);
    if (!i0_out) return fail(SPCN_E_ARG, "i0_out is NULL");
    SPCN_CHECK(check_ws(ws, ws_bytes, i0_workspace_bytes(n_samples)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_estimate_i0(img, height * width, white_sum, n_samples, seed, (double)percentile / 100.0,
                                      i0_out, flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_estimate_i0 launch");
    return SPCN_OK;
}

spcn_status spcn_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                  const spcn_params* p, int64_t band_rows, float* band_p99, float* p99_out,
                                  int32_t* flags_out, void* ws, size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    SPCN_CHECK(check_params(p, true));
    if (!w) return fail(SPCN_E_ARG, "w is NULL");
    if (!p99_out) return fail(SPCN_E_ARG, "p99_out is NULL");
    if (band_rows < 1) return fail(SPCN_E_ARG, "band_rows = %lld must be >= 1", (long long)band_rows);
    const int64_t n_bands = (height + band_rows - 1) / band_rows;
    if (n_bands > kMaxBands)
        return fail(SPCN_E_ARG, "%lld bands exceed the limit of %lld", (long long)n_bands, (long long)kMaxBands);
    SPCN_CHECK(check_ws(ws, ws_bytes, band_workspace_bytes(n_bands)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_band_percentiles(img, height, width, w, make_params(p), band_rows, band_p99, p99_out,
                                           flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_band_percentiles launch");
    return SPCN_OK;
}

spcn_status spcn_sample_percentile(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                   const spcn_params* p, int64_t n_samples, uint64_t seed, float* p99_out,
                                   int32_t* flags_out, void* ws, size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    SPCN_CHECK(check_params(p, true));
    if (!w) return fail(SPCN_E_ARG, "w is NULL");
    if (!p99_out) return fail(SPCN_E_ARG, "p99_out is NULL");
    if (n_samples < 1 || n_samples > kMaxI0Samples)
        return fail(SPCN_E_ARG, "n_samples = %lld must lie in [1, %lld]", (long long)n_samples, (long long)kMaxI0Samples);
    SPCN_CHECK(check_ws(ws, ws_bytes, sample_pctl_workspace_bytes(n_samples)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_sample_percentile(img, height * width, w, make_params(p), n_samples, seed, p99_out,
                                            flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_sample_percentile launch");
    return SPCN_OK;
}

spcn_status spcn_exact_percentile(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                  const spcn_params* p, float* p99_out, int32_t* flags_out, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_image(img, height, width, "img"));
    SPCN_CHECK(check_params(p, true));
    if (!w) return fail(SPCN_E_ARG, "w is NULL");
    if (!p99_out) return fail(SPCN_E_ARG, "p99_out is NULL");
    SPCN_CHECK(check_ws(ws, ws_bytes, exact_workspace_bytes()));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_exact_percentile(img, height * width, w, make_params(p), p99_out, flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_exact_percentile launch");
    return SPCN_OK;
}

spcn_status spcn_recolor_p99(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                             const float* w_tgt, const float* scale_tgt, const float* i0_out,
                             const spcn_params* p, const float* p99_src, uint8_t* out, float* scale_out,
                             int32_t* flags_out, hipStream_t stream) {
    SPCN_CHECK(check_image(src, height, width, "src"));
    SPCN_CHECK(check_image(out, height, width, "out"));
    SPCN_CHECK(check_params(p, true));
    if (!w_src || !w_tgt || !scale_tgt) return fail(SPCN_E_ARG, "w_src, w_tgt and scale_tgt must be non-NULL");
    if (!p99_src) return fail(SPCN_E_ARG, "p99_src is NULL");
    const int64_t n = height * width;
    if ((const void*)src < (const void*)(out + 3 * n) && (const void*)out < (const void*)(src + 3 * n))
        return fail(SPCN_E_ARG, "out must not overlap src");
    float io[3];
    for (int c = 0; c < 3; ++c) io[c] = i0_out ? i0_out[c] : p->i0[c];
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(io[c])) return fail(SPCN_E_ARG, "i0_out[%d] = %g must be finite and > 0", c, (double)io[c]);
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_recolor_p99(src, height * width, w_src, w_tgt, scale_tgt, io, make_params(p), out, p99_src,
                                      scale_out, flags_out, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_recolor_p99 launch");
    return SPCN_OK;
}

spcn_status spcn_normalize_streamed(const uint8_t* host_src, uint8_t* host_out, int64_t height, int64_t width,
                                    const float* w_src, const float* w_tgt, const float* scale_tgt,
                                    const float* i0_out, const spcn_params* p, int64_t chunk_rows,
                                    const spcn_norm_stats* st, void* ws, size_t ws_bytes, hipStream_t compute,
                                    hipStream_t copy_in, hipStream_t copy_out) {
    if (!host_src || !host_out) return fail(SPCN_E_ARG, "host_src and host_out must be non-NULL");
    if (height <= 0 || width <= 0) return fail(SPCN_E_ARG, "height and width must be positive");
    if (height > ((int64_t)1 << 36) / width) return fail(SPCN_E_ARG, "image of %lld x %lld pixels is too large",
                                                         (long long)height, (long long)width);
    SPCN_CHECK(check_params(p, true));
    if (!w_src || !w_tgt || !scale_tgt) return fail(SPCN_E_ARG, "w_src, w_tgt and scale_tgt must be non-NULL");
    if (chunk_rows < 1 || chunk_rows * width > ((int64_t)1 << 30))
        return fail(SPCN_E_ARG, "chunk_rows = %lld must be >= 1 with at most 2^30 pixels per chunk",
                    (long long)chunk_rows);
    SPCN_CHECK(check_ws(ws, ws_bytes, stream_workspace_bytes(width, chunk_rows)));
    if (copy_in == compute || copy_out == compute)
        return fail(SPCN_E_ARG, "copy streams must differ from the compute stream");
    const int64_t n = height * width;
    if ((const void*)host_src < (const void*)(host_out + 3 * n) && (const void*)host_out < (const void*)(host_src + 3 * n))
        return fail(SPCN_E_ARG, "host_out must not overlap host_src");
    float io[3];
    for (int c = 0; c < 3; ++c) io[c] = i0_out ? i0_out[c] : p->i0[c];
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(io[c])) return fail(SPCN_E_ARG, "i0_out[%d] = %g must be finite and > 0", c, (double)io[c]);
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_stream_normalize(host_src, host_out, height, width, w_src, w_tgt, scale_tgt, io,
                                           make_params(p), chunk_rows, ws, ws_bytes, st ? st->p99_src : nullptr,
                                           st ? st->scale : nullptr, st ? st->flags : nullptr, dev, compute, copy_in,
                                           copy_out);
    if (e != hipSuccess) return hip_fail(e, "spcn_normalize_streamed");
    return SPCN_OK;
}

int64_t spcn_stream_resident_chunks(int64_t height, int64_t width, int64_t chunk_rows, size_t ws_bytes) {
    if (height <= 0 || width <= 0 || chunk_rows < 1 || chunk_rows > ((int64_t)1 << 30) / width) return 0;
    return stream_resident_chunks(height, width, chunk_rows, ws_bytes);
}

spcn_status spcn_estimate_basis_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t max_tile_px,
                                        const spcn_params* p, float lambda_nmf, int64_t n_samples,
                                        uint64_t seed, int32_t n_iter, const float* w_init, float* w_out,
                                        float* sample_p99, float* hist_hi_out, int32_t* flags_out, void* ws,
                                        size_t ws_bytes,
                                        hipStream_t stream) {
    (void)max_tile_px;
    if (!tiles) return fail(SPCN_E_ARG, "tiles is NULL");
    if (n_tiles < 1) return fail(SPCN_E_ARG, "n_tiles = %d must be >= 1", (int)n_tiles);
    SPCN_CHECK(check_params(p, true));
    SPCN_CHECK(check_fit(lambda_nmf, n_samples, n_iter, basis_tile_max_samples()));
    if (!w_out) return fail(SPCN_E_ARG, "w_out is NULL");
    SPCN_CHECK(check_ws(ws, ws_bytes, basis_batched_workspace_bytes(n_tiles, n_samples)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_estimate_basis_batched(tiles, n_tiles, make_params(p), lambda_nmf, n_samples, seed, n_iter,
                                                 w_init, w_out, sample_p99, hist_hi_out, flags_out, ws, dev,
                                                 stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_estimate_basis_batched launch");
    return SPCN_OK;
}

spcn_status spcn_normalize_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t total_px, const float* w_src,
                                   const float* w_tgt, const float* scale_tgt, const float* i0_out,
                                   const spcn_params* p, float* p99_out, float* scale_out, int32_t* flags_out,
                                   uint64_t* hist_out, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!tiles) return fail(SPCN_E_ARG, "tiles is NULL");
    if (n_tiles < 1 || n_tiles > batched_max_tiles())
        return fail(SPCN_E_ARG, "n_tiles = %d must lie in [1, %lld]", (int)n_tiles, (long long)batched_max_tiles());
    if (total_px < 1 || total_px > ((int64_t)1 << 40)) return fail(SPCN_E_ARG, "total_px = %lld out of range", (long long)total_px);
    SPCN_CHECK(check_params(p, true));
    if (!w_src || !w_tgt || !scale_tgt) return fail(SPCN_E_ARG, "w_src, w_tgt and scale_tgt must be non-NULL");
    float io[3];
    for (int c = 0; c < 3; ++c) io[c] = i0_out ? i0_out[c] : p->i0[c];
    for (int c = 0; c < 3; ++c)
        if (!finite_pos(io[c])) return fail(SPCN_E_ARG, "i0_out[%d] = %g must be finite and > 0", c, (double)io[c]);
    SPCN_CHECK(check_ws(ws, ws_bytes, batched_workspace_bytes(n_tiles, total_px)));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_normalize_batched(tiles, n_tiles, total_px, w_src, w_tgt, scale_tgt, io, make_params(p),
                                            p99_out, scale_out, flags_out, hist_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_normalize_batched launch");
    return SPCN_OK;
}

static spcn_status check_f32(const float* x, int64_t n, int64_t height, int64_t width, const float* w_src,
                             int64_t w_src_stride, const float* w_tgt, int64_t w_tgt_stride, const float* scale_tgt,
                             int64_t scale_stride, const spcn_params* p) {
    if (!x) return fail(SPCN_E_ARG, "x is NULL");
    if (n < 1 || height < 1 || width < 1) return fail(SPCN_E_ARG, "n, height and width must be >= 1");
    if (height > (((int64_t)1 << 31) - 1) / width) return fail(SPCN_E_ARG, "more than 2^31 - 1 pixels per sample");
    if (n > 65535) return fail(SPCN_E_ARG, "n = %lld exceeds 65535 samples", (long long)n);
    if (((uintptr_t)x) & 3) return fail(SPCN_E_ARG, "x must be 4-byte aligned");
    if (!w_src || !w_tgt || !scale_tgt) return fail(SPCN_E_ARG, "w_src, w_tgt and scale_tgt must be non-NULL");
    if (w_src_stride < 0 || w_tgt_stride < 0 || scale_stride < 0) return fail(SPCN_E_ARG, "strides must be >= 0");
    SPCN_CHECK(check_params(p, false));
    return SPCN_OK;
}

spcn_status spcn_normalize_f32(const float* x, int64_t n, int64_t height, int64_t width, const float* w_src,
                               int64_t w_src_stride, const float* w_tgt, int64_t w_tgt_stride, const float* scale_tgt,
                               int64_t scale_stride, const float* i0_out, const spcn_params* p, float* y,
                               float* p99_out, float* scale_out, int64_t* sel_idx, int32_t* flags_out, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_f32(x, n, height, width, w_src, w_src_stride, w_tgt, w_tgt_stride, scale_tgt, scale_stride, p));
    if (!y) return fail(SPCN_E_ARG, "y is NULL");
    const int64_t n_px = height * width;
    if ((const void*)x < (const void*)(y + 3 * n * n_px) && (const void*)y < (const void*)(x + 3 * n * n_px))
        return fail(SPCN_E_ARG, "y must not overlap x");
    SPCN_CHECK(check_ws(ws, ws_bytes, f32_forward_workspace_bytes(n_px, n)));
    F32Args a{x, n, n_px, w_src, w_src_stride, w_tgt, w_tgt_stride, scale_tgt, scale_stride, {0, 0, 0}};
    for (int c = 0; c < 3; ++c) {
        a.i0_out[c] = i0_out ? i0_out[c] : p->i0[c];
        if (!finite_pos(a.i0_out[c])) return fail(SPCN_E_ARG, "i0_out[%d] must be finite and > 0", c);
    }
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_forward_f32(a, make_params(p), y, p99_out, scale_out, sel_idx, flags_out, ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_normalize_f32 launch");
    return SPCN_OK;
}

spcn_status spcn_normalize_backward(const float* x, int64_t n, int64_t height, int64_t width, const float* w_src,
                                    int64_t w_src_stride, const float* w_tgt, int64_t w_tgt_stride,
                                    const float* scale_tgt, int64_t scale_stride, const float* i0_out,
                                    const spcn_params* p, const float* p99, const int64_t* sel_idx,
                                    const int32_t* flags, const float* grad_y, float* grad_x, float* grad_w_tgt,
                                    float* grad_scale, void* ws, size_t ws_bytes, hipStream_t stream) {
    SPCN_CHECK(check_f32(x, n, height, width, w_src, w_src_stride, w_tgt, w_tgt_stride, scale_tgt, scale_stride, p));
    if (!p99 || !sel_idx || !flags) return fail(SPCN_E_ARG, "p99, sel_idx and flags (saved forward state) are required");
    if (!grad_y || !grad_x || !grad_w_tgt || !grad_scale)
        return fail(SPCN_E_ARG, "grad_y, grad_x, grad_w_tgt and grad_scale must be non-NULL");
    const int64_t n_px = height * width;
    SPCN_CHECK(check_ws(ws, ws_bytes, f32_backward_workspace_bytes(n_px, n)));
    F32Args a{x, n, n_px, w_src, w_src_stride, w_tgt, w_tgt_stride, scale_tgt, scale_stride, {0, 0, 0}};
    for (int c = 0; c < 3; ++c) {
        a.i0_out[c] = i0_out ? i0_out[c] : p->i0[c];
        if (!finite_pos(a.i0_out[c])) return fail(SPCN_E_ARG, "i0_out[%d] must be finite and > 0", c);
    }
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_backward_f32(a, make_params(p), p99, sel_idx, flags, grad_y, grad_x, grad_w_tgt, grad_scale,
                                       ws, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_normalize_backward launch");
    return SPCN_OK;
}

spcn_status spcn_bandwidth_probe(const void* src, void* dst, int64_t bytes, int32_t mode, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
    if (mode < 0 || mode > 3)
        return fail(SPCN_E_ARG, "mode = %d must be 0 or 2 (copy) or 1 or 3 (read)", (int)mode);
    const bool copy = mode == 0 || mode == 2;
    if (!src) return fail(SPCN_E_ARG, "src is NULL");
    if (copy && !dst) return fail(SPCN_E_ARG, "dst is NULL");
    if (bytes < 16 || (bytes & 15) || bytes > ((int64_t)1 << 40))
        return fail(SPCN_E_ARG, "bytes = %lld must be a multiple of 16 in [16, 2^40]", (long long)bytes);
    if ((((uintptr_t)src) | (copy ? (uintptr_t)dst : 0)) & 15) return fail(SPCN_E_ARG, "src and dst must be 16-byte aligned");
    if (copy && (const uint8_t*)src < (const uint8_t*)dst + bytes && (const uint8_t*)dst < (const uint8_t*)src + bytes)
        return fail(SPCN_E_ARG, "dst must not overlap src");
    if (!copy) SPCN_CHECK(check_ws(ws, ws_bytes, probe_sink_bytes()));
    DevInfo dev;
    SPCN_CHECK(dev_info(&dev));
    hipError_t e = launch_probe(static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), static_cast<uint32_t*>(ws),
                                bytes, mode, dev, stream);
    if (e != hipSuccess) return hip_fail(e, "spcn_bandwidth_probe launch");
    return SPCN_OK;
}

spcn_status spcn_set_option(int opt, int value) {
    if (opt < 0 || opt >= N_OPT) return fail(SPCN_E_ARG, "unknown option %d", opt);
    if (value < g_opt_lo[opt] || value > g_opt_hi[opt])
        return fail(SPCN_E_ARG, "option %d: value %d outside [%d, %d]", opt, value, g_opt_lo[opt], g_opt_hi[opt]);
    g_opt[opt].store(value, std::memory_order_relaxed);
    return SPCN_OK;
}

int spcn_get_option(int opt) { return (opt >= 0 && opt < N_OPT) ? g_opt[opt].load(std::memory_order_relaxed) : -1; }

const char* spcn_status_string(spcn_status s) {
    switch (s) {
        case SPCN_OK: return "ok";
        case SPCN_E_ARG: return "invalid argument";
        case SPCN_E_WORKSPACE: return "workspace missing or too small";
        case SPCN_E_HIP: return "HIP runtime error";
        case SPCN_E_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* spcn_last_error(void) { return g_err; }

const char* spcn_version(void) { return "spcn-gfx950 0.1"; }

}  // extern "C"
