// spcn_internal.h -- shared declarations of libspcn's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/spcn.h"

namespace spcn {

constexpr int kBins = SPCN_HIST_BINS;

// Error reporting: host-side, thread-local detail of the last failure.
spcn_status fail(spcn_status s, const char* fmt, ...);
spcn_status hip_fail(hipError_t e, const char* what);
#define SPCN_HIP_TRY(call)                                              \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::spcn::hip_fail(e_, #call);       \
    } while (0)

// Process-wide tuning options (spcn_set_option).
int option(int id);

// Device properties of the current device (cached per device id).
struct DevInfo {
    int id;
    int cus;
};
spcn_status dev_info(DevInfo* out);

// Plain-old-data view of the parameters the kernels need (host -> kernel argument).
struct ParamsK {
    float i0[3];
    float lambda;
    int32_t white_sum;
    float q;            // percentile / 100 as float (q64 below is the exact value used)
    double q64;         // (double)percentile / 100
    float hist_hi[2];
    const float* hist_hi_dev;   // device range replacing hist_hi, or NULL
    int32_t auto_range;         // one automatic retry at a doubled range (single-image paths)
};
ParamsK make_params(const spcn_params* p);

// ---- uint8 single-image path (spcn_u8.hip)
struct U8Work {             // device scratch carved out of the caller's workspace
    uint64_t* hist;         // [2][256] accumulator
};
size_t u8_workspace_bytes();

// ctl_ws: the caller's u8 workspace (u8_workspace_bytes), whose range and retry words follow the
// histogram slot; hist may be that slot or a caller array.
hipError_t launch_densities(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                            float* h_out, uint64_t* hist, float* p99_out, int32_t* flags_out, float* range_out,
                            void* ctl_ws, const DevInfo& dev, hipStream_t s);
hipError_t launch_recolor(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                          const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                          uint8_t* out, const uint64_t* hist, float* p99_out, float* scale_out,
                          int32_t* flags_out, float* range_out, const DevInfo& dev, hipStream_t s);
hipError_t launch_normalize(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                            const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                            uint8_t* out, uint64_t* hist, void* ctl_ws, float* p99_out, float* scale_out,
                            int32_t* flags_out, float* range_out, const DevInfo& dev, hipStream_t s);

// ---- basis estimation (spcn_basis.hip)
size_t basis_workspace_bytes(int64_t n_samples);
hipError_t launch_estimate_basis(const uint8_t* img, int64_t n_px, const ParamsK& pk, float lambda_nmf,
                                 int64_t n_samples, uint64_t seed, int32_t n_iter, const float* w_init,
                                 float* w_out, float* sample_p99, float* range_out, int32_t* flags_out, void* ws,
                                 const DevInfo& dev, hipStream_t s);
size_t basis_batched_workspace_bytes(int64_t n_tiles, int64_t n_samples);
int64_t basis_tile_max_samples();
constexpr int64_t kMaxBasisSamples = 262144;
constexpr int64_t kMaxI0Samples = 1048576;
constexpr int64_t kMaxBands = 65536;
hipError_t launch_zero_hist(uint64_t* hist, hipStream_t s);
// pass 1 adding to hist (not cleared)
hipError_t launch_count(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk, uint64_t* hist,
                        const DevInfo& dev, hipStream_t s);
// exact order statistic over all non-white pixels (colour table + radix selection)
size_t exact_workspace_bytes();
hipError_t launch_exact_percentile(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                                   float* p99_out, int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s);
size_t stream_workspace_bytes(int64_t width, int64_t chunk_rows);
int64_t stream_resident_chunks(int64_t height, int64_t width, int64_t chunk_rows, size_t ws_bytes);
hipError_t launch_stream_normalize(const uint8_t* host_src, uint8_t* host_out, int64_t height, int64_t width,
                                   const float* w_src, const float* w_tgt, const float* scale_tgt,
                                   const float i0_out[3], const ParamsK& pk, int64_t chunk_rows, void* ws,
                                   size_t ws_bytes, float* p99_out, float* scale_out, int32_t* flags_out, const DevInfo& dev,
                                   hipStream_t compute, hipStream_t copy_in, hipStream_t copy_out);
size_t sample_pctl_workspace_bytes(int64_t n_samples);
hipError_t launch_sample_percentile(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk, int64_t n_s,
                                    uint64_t seed, float* p99_out, int32_t* flags_out, void* ws, const DevInfo& dev,
                                    hipStream_t s);
size_t band_workspace_bytes(int64_t n_bands);
hipError_t launch_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                   const ParamsK& pk, int64_t band_rows, float* band_out, float* median_out,
                                   int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s);
hipError_t launch_recolor_p99(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                              const float* scale_tgt, const float i0_out[3], const ParamsK& pk, uint8_t* out,
                              const float* p99_in, float* scale_out, int32_t* flags_out, const DevInfo& dev,
                              hipStream_t s);
size_t i0_workspace_bytes(int64_t n_samples);
hipError_t launch_estimate_i0(const uint8_t* img, int64_t n_px, int32_t white_sum, int64_t n_s, uint64_t seed,
                              double q, float* i0_out, int32_t* flags_out, void* ws, const DevInfo& dev,
                              hipStream_t s);
hipError_t launch_estimate_basis_batched(const spcn_tile* tiles, int32_t n_tiles, const ParamsK& pk,
                                         float lambda_nmf, int64_t n_samples, uint64_t seed,
                                         int32_t n_iter, const float* w_init, float* w_out,
                                         float* sample_p99, float* range_out, int32_t* flags_out, void* ws,
                                         const DevInfo& dev, hipStream_t s);

// ---- batched persistent normalisation (spcn_batched.hip)
size_t batched_workspace_bytes(int64_t n_tiles, int64_t total_px);
int64_t batched_max_tiles();
// ---- bandwidth reference kernels (spcn_probe.hip)
size_t probe_sink_bytes();
hipError_t launch_probe(const uint8_t* src, uint8_t* dst, uint32_t* sink, int64_t n, int mode, const DevInfo& dev,
                        hipStream_t s);

hipError_t launch_normalize_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t total_px,
                                    const float* w_src, const float* w_tgt, const float* scale_tgt,
                                    const float i0_out[3], const ParamsK& pk, float* p99_out,
                                    float* scale_out, int32_t* flags_out, uint64_t* hist_out, void* ws,
                                    const DevInfo& dev, hipStream_t s);

// ---- differentiable float path (spcn_f32.hip)
size_t f32_forward_workspace_bytes(int64_t n_px, int64_t n);
size_t f32_backward_workspace_bytes(int64_t n_px, int64_t n);
struct F32Args {
    const float* x; int64_t n, n_px;
    const float* w_src; int64_t w_src_stride;
    const float* w_tgt; int64_t w_tgt_stride;
    const float* scale_tgt; int64_t scale_stride;
    float i0_out[3];
};
hipError_t launch_forward_f32(const F32Args& a, const ParamsK& pk, float* y, float* p99_out,
                              float* scale_out, int64_t* sel_idx, int32_t* flags_out, void* ws,
                              const DevInfo& dev, hipStream_t s);
hipError_t launch_backward_f32(const F32Args& a, const ParamsK& pk, const float* p99,
                               const int64_t* sel_idx, const int32_t* flags, const float* grad_y,
                               float* grad_x, float* grad_w_tgt, float* grad_scale, void* ws,
                               const DevInfo& dev, hipStream_t s);

}  // namespace spcn
