// spcn_probe.hip -- memory-bandwidth reference kernels for the roofline of the passes (measurement
// infrastructure: they compute nothing of the method).  A grid-stride copy of a buffer into another
// (pass 2's traffic: n bytes read, n written) and a grid-stride read with an XOR reduction (pass 1's
// traffic: n bytes read), both with 16-byte accesses through buffer resources, 12 per thread and
// tile, the next tile's loads in flight, in the launch shape of the recolour pass (256 threads,
// 8 workgroups per CU).  Each comes with the passes' streaming cache policy (loads nt, stores sc1 nt)
// and with the default policy.
#include "spcn_internal.h"

namespace spcn {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufDword3 = 0x00020000;
constexpr int PROBE_THREADS = 256;
constexpr int PROBE_UNROLL = 12;   // 192 bytes per thread and tile, as the recolour pass
constexpr int kLoadStream = 2;     // the passes' streaming policy: loads nt
constexpr int kStoreStream = 18;   // stores sc1 nt

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* base, int64_t off, int64_t bytes) {
    const uint64_t addr = reinterpret_cast<uint64_t>(base) + (uint64_t)off;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)bytes);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, n, kBufDword3);
}

// COPY: dst = src; else read src, one XOR word per thread into sink.  The loads of a workgroup's
// next tile are issued before the current tile is stored (as the recolour pass does).  LA, SA: cache
// policy of the loads and stores.
template <bool COPY, int LA, int SA>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe(const uint8_t* src, uint8_t* dst, uint32_t* sink, int64_t n) {
    constexpr int64_t TILE = (int64_t)PROBE_THREADS * PROBE_UNROLL * 16;
    const int64_t tiles = (n + TILE - 1) / TILE;
    const int tid = threadIdx.x;
    auto rsrc = [&](const void* base, int64_t t) {     // empty past the last tile
        const int64_t off = t < tiles ? t * TILE : 0;
        const int64_t len = t < tiles ? (n - off < TILE ? n - off : TILE) : 0;
        return tile_rsrc(base, off, len);
    };
    u32x4 acc = {0u, 0u, 0u, 0u};
    int64_t t = blockIdx.x;
    u32x4 cur[PROBE_UNROLL];
    {
        const __amdgpu_buffer_rsrc_t rs = rsrc(src, t);
#pragma unroll
        for (int j = 0; j < PROBE_UNROLL; ++j)
            cur[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (tid + j * PROBE_THREADS), 0, LA);
    }
    for (; t < tiles; t += gridDim.x) {
        const __amdgpu_buffer_rsrc_t rn = rsrc(src, t + gridDim.x);
        u32x4 nxt[PROBE_UNROLL];
#pragma unroll
        for (int j = 0; j < PROBE_UNROLL; ++j)
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b128(rn, 16 * (tid + j * PROBE_THREADS), 0, LA);
        if (COPY) {
            const __amdgpu_buffer_rsrc_t ws = rsrc(dst, t);
#pragma unroll
            for (int j = 0; j < PROBE_UNROLL; ++j)
                __builtin_amdgcn_raw_buffer_store_b128(cur[j], ws, 16 * (tid + j * PROBE_THREADS), 0, SA);
        } else {
#pragma unroll
            for (int j = 0; j < PROBE_UNROLL; ++j) acc ^= cur[j];
        }
#pragma unroll
        for (int j = 0; j < PROBE_UNROLL; ++j) cur[j] = nxt[j];
    }
    if (!COPY) sink[blockIdx.x * PROBE_THREADS + tid] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

}  // namespace

constexpr int PROBE_MAX_GRID = 4096;

size_t probe_sink_bytes() { return (size_t)PROBE_MAX_GRID * PROBE_THREADS * sizeof(uint32_t); }

hipError_t launch_probe(const uint8_t* src, uint8_t* dst, uint32_t* sink, int64_t n, int mode, const DevInfo& dev,
                        hipStream_t s) {
    const int grid = dev.cus * 8 < PROBE_MAX_GRID ? dev.cus * 8 : PROBE_MAX_GRID;
    switch (mode) {
    case 0: hipLaunchKernelGGL((k_probe<true, kLoadStream, kStoreStream>), dim3(grid), dim3(PROBE_THREADS), 0, s, src, dst, sink, n); break;
    case 1: hipLaunchKernelGGL((k_probe<false, kLoadStream, 0>), dim3(grid), dim3(PROBE_THREADS), 0, s, src, dst, sink, n); break;
    case 2: hipLaunchKernelGGL((k_probe<true, 0, 0>), dim3(grid), dim3(PROBE_THREADS), 0, s, src, dst, sink, n); break;
    default: hipLaunchKernelGGL((k_probe<false, 0, 0>), dim3(grid), dim3(PROBE_THREADS), 0, s, src, dst, sink, n); break;
    }
    return hipGetLastError();
}

}  // namespace spcn
