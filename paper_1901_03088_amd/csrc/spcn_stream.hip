// spcn_stream.hip -- out-of-core normalisation of a slide held in pinned host memory (the paper's
// divide and conquer of Sec. 3.2 item 3, for slides that do not fit in, or arrive outside, HBM).
//
// The slide is cut into chunks of chunk_rows rows.  Pass 1 copies each chunk into one of two
// device staging buffers and adds its non-white pixels to one exact histogram; pass 2 copies each
// chunk again, recolours it into one of two output staging buffers and copies the result back.
// Copies run on their own streams and overlap the kernels of the previous / next chunk; events
// order every reuse of a staging buffer.  Calls that overlap on one device share the ordering
// events and must be serialised by the caller.  The histogram is exact, so the result equals
// spcn_normalize on the whole slide byte for byte.
#include "spcn_internal.h"
#include "spcn_device.hpp"

#include <mutex>

namespace spcn {

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Eight ordering events per device, created once and kept for the life of the process (an event
// may be re-recorded while earlier waits on it are still pending: each wait captured its state).
struct Events {
    hipEvent_t in_ready[2], in_free[2], out_ready[2], out_free[2];
};

hipError_t device_events(Events** out) {
    static std::mutex mu;
    static Events* cache[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!cache[dev]) {
        Events* ev = new Events();
        hipEvent_t* all[] = {&ev->in_ready[0], &ev->in_ready[1], &ev->in_free[0], &ev->in_free[1],
                             &ev->out_ready[0], &ev->out_ready[1], &ev->out_free[0], &ev->out_free[1]};
        for (hipEvent_t* x : all)
            if ((e = hipEventCreateWithFlags(x, hipEventDisableTiming)) != hipSuccess) return e;
        cache[dev] = ev;
    }
    *out = cache[dev];
    return hipSuccess;
}

}  // namespace

size_t stream_workspace_bytes(int64_t width, int64_t chunk_rows) {
    if (width <= 0 || chunk_rows <= 0) return 0;
    const size_t chunk = al256((size_t)(chunk_rows * width * 3));
    return al256(2 * kHistBins * sizeof(uint64_t)) + 4 * chunk;
}

hipError_t launch_stream_normalize(const uint8_t* host_src, uint8_t* host_out, int64_t height, int64_t width,
                                   const float* w_src, const float* w_tgt, const float* scale_tgt,
                                   const float i0_out[3], const ParamsK& pk, int64_t chunk_rows, void* ws,
                                   float* p99_out, float* scale_out, int32_t* flags_out, const DevInfo& dev,
                                   hipStream_t compute, hipStream_t copy_in, hipStream_t copy_out) {
    const size_t chunk = al256((size_t)(chunk_rows * width * 3));
    uint8_t* p = static_cast<uint8_t*>(ws);
    uint64_t* hist = reinterpret_cast<uint64_t*>(p); p += al256(2 * kHistBins * sizeof(uint64_t));
    uint8_t* in[2] = {p, p + chunk};
    uint8_t* out[2] = {p + 2 * chunk, p + 3 * chunk};
    const int64_t n_chunks = (height + chunk_rows - 1) / chunk_rows;
    Events* evp = nullptr;
    hipError_t e = device_events(&evp);
    if (e != hipSuccess) return e;
    Events& ev = *evp;
    auto rows_of = [&](int64_t c) { return (c + 1) * chunk_rows <= height ? chunk_rows : height - c * chunk_rows; };
    bool in_used[2] = {false, false}, out_used[2] = {false, false};

    if ((e = launch_zero_hist(hist, compute)) != hipSuccess) return e;
    // ---- pass 1: stream the chunks in, count
    for (int64_t c = 0; c < n_chunks; ++c) {
        const int s = (int)(c & 1);
        const int64_t px = rows_of(c) * width;
        if (in_used[s] && (e = hipStreamWaitEvent(copy_in, ev.in_free[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(in[s], host_src + 3 * c * chunk_rows * width, (size_t)(3 * px), hipMemcpyHostToDevice,
                                copy_in)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.in_ready[s], copy_in)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(compute, ev.in_ready[s], 0)) != hipSuccess) return e;
        if ((e = launch_count(in[s], px, w_src, pk, hist, dev, compute)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.in_free[s], compute)) != hipSuccess) return e;
        in_used[s] = true;
    }
    // ---- pass 2: stream the chunks in again, recolour, stream the results out
    for (int64_t c = 0; c < n_chunks; ++c) {
        const int s = (int)(c & 1);
        const int64_t px = rows_of(c) * width;
        if (in_used[s] && (e = hipStreamWaitEvent(copy_in, ev.in_free[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(in[s], host_src + 3 * c * chunk_rows * width, (size_t)(3 * px), hipMemcpyHostToDevice,
                                copy_in)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.in_ready[s], copy_in)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(compute, ev.in_ready[s], 0)) != hipSuccess) return e;
        if (out_used[s] && (e = hipStreamWaitEvent(compute, ev.out_free[s], 0)) != hipSuccess) return e;
        const bool first = c == 0;
        if ((e = launch_recolor(in[s], px, w_src, w_tgt, scale_tgt, i0_out, pk, out[s], hist, first ? p99_out : nullptr,
                                first ? scale_out : nullptr, first ? flags_out : nullptr, dev, compute)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.in_free[s], compute)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.out_ready[s], compute)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(copy_out, ev.out_ready[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(host_out + 3 * c * chunk_rows * width, out[s], (size_t)(3 * px), hipMemcpyDeviceToHost,
                                copy_out)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.out_free[s], copy_out)) != hipSuccess) return e;
        in_used[s] = true;
        out_used[s] = true;
    }
    // the caller's compute stream completes after the last copy out
    if ((e = hipEventRecord(ev.out_free[0], copy_out)) != hipSuccess) return e;
    return hipStreamWaitEvent(compute, ev.out_free[0], 0);
}

}  // namespace spcn
