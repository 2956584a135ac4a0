// spcn_stream.hip -- out-of-core normalisation of a slide held in pinned host memory (the paper's
// divide and conquer of Sec. 3.2 item 3, for slides that do not fit in, or arrive outside, HBM).
//
// The slide is cut into chunks of chunk_rows rows.  Pass 1 copies each chunk to the device and adds
// its non-white pixels to one exact histogram; pass 2 recolours each chunk and copies the result
// back.  The first R chunks (as many as the workspace holds beyond its minimum) stay resident
// between the passes and are recoloured in place, so only the other chunks cross the link twice;
// those go through two device input and two output staging buffers.  Copies run on their own
// streams and overlap the kernels of the previous / next chunk; events order every reuse of a
// staging buffer, and both copy streams first wait for the work already queued on the compute
// stream (the workspace and the host buffers may still be in use there).  Calls that overlap on
// one device share the ordering events and must be serialised by the caller.  The histogram is
// exact, so the result equals spcn_normalize on the whole slide byte for byte.
#include "spcn_internal.h"
#include "spcn_device.hpp"

#include <mutex>

namespace spcn {

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Nine ordering events per device, created once and kept for the life of the process (an event
// may be re-recorded while earlier waits on it are still pending: each wait captured its state).
struct Events {
    hipEvent_t in_ready[2], in_free[2], out_ready[2], out_free[2], entry;
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
                             &ev->out_ready[0], &ev->out_ready[1], &ev->out_free[0], &ev->out_free[1],
                             &ev->entry};
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

int64_t stream_resident_chunks(int64_t height, int64_t width, int64_t chunk_rows, size_t ws_bytes) {
    const size_t base = stream_workspace_bytes(width, chunk_rows);
    if (base == 0 || ws_bytes <= base) return 0;
    const size_t chunk = al256((size_t)(chunk_rows * width * 3));
    const int64_t n_chunks = (height + chunk_rows - 1) / chunk_rows;
    const int64_t r = (int64_t)((ws_bytes - base) / chunk);
    return r < n_chunks ? r : n_chunks;
}

hipError_t launch_stream_normalize(const uint8_t* host_src, uint8_t* host_out, int64_t height, int64_t width,
                                   const float* w_src, const float* w_tgt, const float* scale_tgt,
                                   const float i0_out[3], const ParamsK& pk, int64_t chunk_rows, void* ws,
                                   size_t ws_bytes, float* p99_out, float* scale_out, int32_t* flags_out,
                                   const DevInfo& dev, hipStream_t compute, hipStream_t copy_in,
                                   hipStream_t copy_out) {
    const size_t chunk = al256((size_t)(chunk_rows * width * 3));
    uint8_t* p = static_cast<uint8_t*>(ws);
    uint64_t* hist = reinterpret_cast<uint64_t*>(p); p += al256(2 * kHistBins * sizeof(uint64_t));
    uint8_t* in[2] = {p, p + chunk};
    uint8_t* out[2] = {p + 2 * chunk, p + 3 * chunk};
    uint8_t* resident = p + 4 * chunk;                 // slot c holds chunk c < n_res
    const int64_t n_chunks = (height + chunk_rows - 1) / chunk_rows;
    const int64_t n_res = stream_resident_chunks(height, width, chunk_rows, ws_bytes);
    Events* evp = nullptr;
    hipError_t e = device_events(&evp);
    if (e != hipSuccess) return e;
    Events& ev = *evp;
    auto rows_of = [&](int64_t c) { return (c + 1) * chunk_rows <= height ? chunk_rows : height - c * chunk_rows; };
    auto host_in = [&](int64_t c) { return host_src + 3 * c * chunk_rows * width; };
    auto host_res = [&](int64_t c) { return host_out + 3 * c * chunk_rows * width; };
    bool in_used[2] = {false, false}, out_used[2] = {false, false};

    // nothing is copied before the work already queued on the compute stream is done
    if ((e = hipEventRecord(ev.entry, compute)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(copy_in, ev.entry, 0)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(copy_out, ev.entry, 0)) != hipSuccess) return e;
    if ((e = launch_zero_hist(hist, compute)) != hipSuccess) return e;
    // ---- pass 1: stream the chunks in, count; resident chunks keep their own slots
    for (int64_t c = 0; c < n_chunks; ++c) {
        const int s = (int)(c & 1);
        const int64_t px = rows_of(c) * width;
        const bool res = c < n_res;
        uint8_t* dst = res ? resident + c * chunk : in[s];
        if (!res && in_used[s] && (e = hipStreamWaitEvent(copy_in, ev.in_free[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(dst, host_in(c), (size_t)(3 * px), hipMemcpyHostToDevice, copy_in)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.in_ready[s], copy_in)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(compute, ev.in_ready[s], 0)) != hipSuccess) return e;
        if ((e = launch_count(dst, px, w_src, pk, hist, dev, compute)) != hipSuccess) return e;
        if (!res) {
            if ((e = hipEventRecord(ev.in_free[s], compute)) != hipSuccess) return e;
            in_used[s] = true;
        }
    }
    // ---- pass 2a: resident chunks, recoloured in place (every pass-2 kernel reads a unit before the
    // same thread writes it) and copied out; no copy in, so the link carries only their results
    for (int64_t c = 0; c < n_res; ++c) {
        const int64_t px = rows_of(c) * width;
        uint8_t* buf = resident + c * chunk;
        const bool first = c == 0;
        if ((e = launch_recolor(buf, px, w_src, w_tgt, scale_tgt, i0_out, pk, buf, hist, first ? p99_out : nullptr,
                                first ? scale_out : nullptr, first ? flags_out : nullptr, nullptr, dev,
                                compute)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.out_ready[0], compute)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(copy_out, ev.out_ready[0], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(host_res(c), buf, (size_t)(3 * px), hipMemcpyDeviceToHost, copy_out)) != hipSuccess)
            return e;
    }
    // ---- pass 2b: the other chunks are streamed in again, recoloured and streamed out
    for (int64_t c = n_res; c < n_chunks; ++c) {
        const int s = (int)(c & 1);
        const int64_t px = rows_of(c) * width;
        if (in_used[s] && (e = hipStreamWaitEvent(copy_in, ev.in_free[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(in[s], host_in(c), (size_t)(3 * px), hipMemcpyHostToDevice, copy_in)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.in_ready[s], copy_in)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(compute, ev.in_ready[s], 0)) != hipSuccess) return e;
        if (out_used[s] && (e = hipStreamWaitEvent(compute, ev.out_free[s], 0)) != hipSuccess) return e;
        const bool first = c == 0;
        if ((e = launch_recolor(in[s], px, w_src, w_tgt, scale_tgt, i0_out, pk, out[s], hist, first ? p99_out : nullptr,
                                first ? scale_out : nullptr, first ? flags_out : nullptr, nullptr, dev,
                                compute)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.in_free[s], compute)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev.out_ready[s], compute)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(copy_out, ev.out_ready[s], 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(host_res(c), out[s], (size_t)(3 * px), hipMemcpyDeviceToHost, copy_out)) != hipSuccess)
            return e;
        if ((e = hipEventRecord(ev.out_free[s], copy_out)) != hipSuccess) return e;
        in_used[s] = true;
        out_used[s] = true;
    }
    // the caller's compute stream completes after the last copy out
    if ((e = hipEventRecord(ev.out_free[0], copy_out)) != hipSuccess) return e;
    return hipStreamWaitEvent(compute, ev.out_free[0], 0);
}

}  // namespace spcn
