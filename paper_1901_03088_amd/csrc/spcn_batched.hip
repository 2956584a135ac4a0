// spcn_batched.hip -- a batch of uneven uint8 tiles, each with its own source basis, normalised to
// one target (Eqs. 1-4 per tile; batch-to-one-target as in Sec. 3.2 item 6) in ONE persistent launch.
//
// k_tiles_setup   one workgroup per tile: FP64 basis quantities, fixed-point pass-1 tables and FP32
//                 pass-2 tables of the tile into the workspace; zeroes the tile's histogram/counters.
// k_tiles_plan    one workgroup: item offsets of every tile, item -> tile map, queue reset.
// k_tiles_run     persistent (one workgroup per CU): dequeues items from a global counter.  Items
//                 0 .. P-1 are pass-1 chunks (tile-major), items P .. 2P-1 the pass-2 chunks in the same
//                 order.  The last pass-1 chunk of a tile (per-tile arrival counter) takes the tile's
//                 percentile and publishes its recolouring constants with a release store of ready[t];
//                 a pass-2 chunk of tile t waits for ready[t].  Every pass-1 chunk of t was dequeued
//                 before any pass-2 chunk of t by a workgroup that is running and never waits, so the
//                 wait always ends; it is also bounded (SPIN_LIMIT) and reports an error instead of
//                 hanging.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int RUN_THREADS = 1024;
constexpr int RUN_UNROLL = 2;                 // pass-2 units per thread and iteration
constexpr int RUN_P1_UNROLL = 2;              // pass-1 units per thread and iteration (1: ~1% slower)
constexpr int MIN_CHUNK_LOG2 = 12;           // smallest work item: 4096 units = 16384 pixels
constexpr uint32_t SPIN_LIMIT = 1u << 26;
constexpr int MAX_TILES = 8192;

struct TileInfo {
    int64_t units;          // full 4-pixel units
    int32_t tail;           // remaining pixels (0..3)
    int32_t n_chunks;       // pass-1 items of the tile (>= 1)
    int64_t item0;          // first pass-1 item of the tile
    int32_t shift;          // fixed-point resolution u of the pass-1 tables
    int32_t ok;             // basis usable
    int32_t bad;            // descriptor unusable (null or misaligned pointer, empty tile): skipped
    int32_t pad;
    float hh[2];            // histogram range of the tile's stains
};

struct BatchHead {
    uint32_t queue;         // next item to hand out
    uint32_t p1_items;
    int32_t error;          // a wait hit SPIN_LIMIT
    int32_t pad;
};

struct BatchWs {
    BatchHead* head;
    TileInfo* info;         // [n]
    Basis64* basis;         // [n]
    int4* tab;              // [n][3 * 256]
    float2* ftab;           // [n][3 * 256]
    RecolourConsts* K;      // [n]
    uint64_t* hist;         // [n][512]
    uint32_t* done;         // [n]
    uint32_t* ready;        // [n]
    double* od;             // [3][256] FP64 optical densities (Eq. 1), for the near-edge path
    int32_t* item_tile;     // [max items]
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline int64_t max_items_for(int64_t n_tiles, int64_t total_px) {
    return total_px / (4 * ((int64_t)1 << MIN_CHUNK_LOG2)) + n_tiles;
}

__host__ __device__ inline BatchWs carve(void* ws, int64_t n, int64_t total_px) {
    uint8_t* p = static_cast<uint8_t*>(ws);
    BatchWs w;
    w.head = reinterpret_cast<BatchHead*>(p); p += a256(sizeof(BatchHead));
    w.info = reinterpret_cast<TileInfo*>(p); p += a256(n * sizeof(TileInfo));
    w.basis = reinterpret_cast<Basis64*>(p); p += a256(n * sizeof(Basis64));
    w.tab = reinterpret_cast<int4*>(p); p += a256(n * 3 * kHistBins * sizeof(int4));
    w.ftab = reinterpret_cast<float2*>(p); p += a256(n * 3 * kHistBins * sizeof(float2));
    w.K = reinterpret_cast<RecolourConsts*>(p); p += a256(n * sizeof(RecolourConsts));
    w.hist = reinterpret_cast<uint64_t*>(p); p += a256(n * 2 * kHistBins * sizeof(uint64_t));
    w.done = reinterpret_cast<uint32_t*>(p); p += a256(n * sizeof(uint32_t));
    w.ready = reinterpret_cast<uint32_t*>(p); p += a256(n * sizeof(uint32_t));
    w.od = reinterpret_cast<double*>(p); p += a256(3 * kHistBins * sizeof(double));
    w.item_tile = reinterpret_cast<int32_t*>(p); p += a256(max_items_for(n, total_px) * sizeof(int32_t));
    return w;
}

struct SetupArgs {
    const spcn_tile* tiles;
    const float* w_src;         // [n][6]
    P1Params pp;
    int chunk_log2;             // 4-pixel units per work item = 2^chunk_log2
    BatchWs w;
};

__global__ __launch_bounds__(256) void k_tiles_setup(SetupArgs a) {
    __shared__ Basis64 B;
    __shared__ int s_shift;
    const int t = blockIdx.x;
    __shared__ float s_hh[2];
    if (threadIdx.x == 0) {
        derive_basis(a.w_src + 6 * t, a.pp.lambda, B);
        s_hh[0] = resolve_range(a.pp.range ? a.pp.range + 2 * t : nullptr, a.pp.hist_hi[0]);
        s_hh[1] = resolve_range(a.pp.range ? a.pp.range + 2 * t + 1 : nullptr, a.pp.hist_hi[1]);
        const int u = table_shift(B, a.pp.i0, s_hh);
        s_shift = u < 16 ? u : 16;                 // the byte-permute layout works in <= 2^16 units
        const spcn_tile T = a.tiles[t];
        const int64_t n_px = T.height * T.width;
        TileInfo I;
        I.units = n_px >> 2;
        I.tail = (int32_t)(n_px & 3);
        I.n_chunks = (int32_t)((I.units + ((int64_t)1 << a.chunk_log2) - 1) >> a.chunk_log2);
        if (I.n_chunks < 1) I.n_chunks = 1;
        I.item0 = 0;
        I.shift = s_shift;
        I.ok = B.ok;
        I.bad = !T.src || !T.out || (((uintptr_t)T.src | (uintptr_t)T.out) & 3) || T.height <= 0 || T.width <= 0;
        I.pad = 0;
        I.hh[0] = s_hh[0];
        I.hh[1] = s_hh[1];
        if (I.bad) { I.units = 0; I.tail = 0; I.n_chunks = 1; }
        a.w.info[t] = I;
        a.w.basis[t] = B;
        a.w.done[t] = 0;
        a.w.ready[t] = 0;
    }
    for (int i = threadIdx.x; i < 2 * kHistBins; i += blockDim.x) a.w.hist[(int64_t)t * 2 * kHistBins + i] = 0;
    if (t == 0)
        for (int i = threadIdx.x; i < 3 * kHistBins; i += blockDim.x)
            a.w.od[i] = od_u8((double)a.pp.i0[i / kHistBins], i % kHistBins);
    __syncthreads();
    const int k = threadIdx.x;
    const int u = s_shift;
    const double sig0 = ldexp(256.0 / (double)s_hh[0], u), sig1 = ldexp(256.0 / (double)s_hh[1], u);
    for (int c = 0; c < 3; ++c) {
        const double od = B.ok ? od_u8((double)a.pp.i0[c], k) : 0.0;
        const int g = c == 0 ? kGuardUnits - 2 * kGuardUnits : 0;   // shifted guard of the byte-permute layout
        int4 e;
        e.x = __double2int_rn((B.pc[0][c] * od + (c == 0 ? B.pconst[0] : 0.0)) * sig0) + g;
        e.y = __double2int_rn((B.q[0][c] * od + (c == 0 ? B.fconst[0] : 0.0)) * sig0) + g;
        e.z = __double2int_rn((B.pc[1][c] * od + (c == 0 ? B.pconst[1] : 0.0)) * sig1) + g;
        e.w = __double2int_rn((B.q[1][c] * od + (c == 0 ? B.fconst[1] : 0.0)) * sig1) + g;
        a.w.tab[((int64_t)t * 3 + c) * kHistBins + k] = e;
        float2 f;
        f.x = (float)(B.q[0][c] * od + (c == 0 ? B.fconst[0] : 0.0));
        f.y = (float)(B.q[1][c] * od + (c == 0 ? B.fconst[1] : 0.0));
        a.w.ftab[((int64_t)t * 3 + c) * kHistBins + k] = f;
    }
}


// Exclusive scan of the tiles' chunk counts -> first item of every tile, then the item -> tile map.
// The caller's total_px must bound the tiles' pixel count (it sized the workspace); otherwise the
// whole batch is refused.
__global__ __launch_bounds__(1024) void k_tiles_plan(BatchWs w, int n_tiles, int64_t total_px, int64_t cap_items,
                                                     int32_t* flags_out) {
    __shared__ int32_t s_off[MAX_TILES];
    __shared__ int32_t s_part[1024];
    __shared__ unsigned long long s_px;
    const int t0 = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    if (t0 == 0) s_px = 0;
    __syncthreads();
    int run = 0;
    int64_t px = 0;
    for (int i = 0; i < per; ++i) {
        const int t = t0 * per + i;
        if (t < n_tiles) {
            const TileInfo I = w.info[t];
            s_off[t] = run;
            run += I.n_chunks;
            px += 4 * I.units + I.tail;
        }
    }
    s_part[t0] = run;
    atomicAdd(&s_px, (unsigned long long)px);
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = t0 >= o ? s_part[t0 - o] : 0;
        __syncthreads();
        s_part[t0] += v;
        __syncthreads();
    }
    const int excl = t0 ? s_part[t0 - 1] : 0;
    for (int i = 0; i < per; ++i) {
        const int t = t0 * per + i;
        if (t < n_tiles) { s_off[t] += excl; w.info[t].item0 = s_off[t]; }
    }
    int total = s_part[1023];
    const bool fits = total <= cap_items && (int64_t)s_px <= total_px;
    if (t0 == 0) {
        w.head->queue = 0;
        w.head->p1_items = fits ? (uint32_t)total : 0u;
        w.head->error = fits ? 0 : 2;
    }
    for (int t = t0; t < n_tiles; t += 1024) {
        if (!flags_out) break;
        const int f = (!fits || w.info[t].bad) ? SPCN_FLAG_BATCH : 0;
        flags_out[2 * t] = f;
        flags_out[2 * t + 1] = f;
    }
    if (!fits) return;
    __syncthreads();
    for (int it = t0; it < total; it += 1024) {
        int lo = 0, hi = n_tiles - 1;           // last tile whose first item is <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= it) lo = mid; else hi = mid - 1;
        }
        w.item_tile[it] = lo;
    }
}

struct RunArgs {
    const spcn_tile* tiles;
    const float* w_tgt;
    const float* scale_tgt;
    float i0_out[3];
    P1Params pp;
    double q;
    int chunk_log2;
    BatchWs w;
    float* p99_out;
    float* scale_out;
    int32_t* flags_out;
};

struct RunLds {
    P1FLds<true> p1;
    P2Lds<1> p2;
    FinalShared F;
    RecolourConsts K;
    uint64_t h[2 * kHistBins];
    int item, tile, last, go;
};

__global__ __launch_bounds__(RUN_THREADS) void k_tiles_run(RunArgs a) {
    __shared__ RunLds S;
    const int tid = threadIdx.x;
    const uint32_t p1_items = a.w.head->p1_items;
    const uint32_t n_items = 2 * p1_items;
    for (;;) {
        if (tid == 0) {
            const uint32_t it = atomicAdd(&a.w.head->queue, 1u);
            S.item = (int)it;
            S.tile = it < n_items ? a.w.item_tile[it < p1_items ? it : it - p1_items] : -1;
        }
        __syncthreads();
        const uint32_t item = (uint32_t)S.item;
        if (item >= n_items) break;
        const bool first = item < p1_items;
        const int t = S.tile;
        const TileInfo I = a.w.info[t];
        const spcn_tile T = a.tiles[t];
        const int chunk = (int)((first ? item : item - p1_items) - I.item0);
        const int64_t u0 = (int64_t)chunk << a.chunk_log2;
        const int cnt = (int)min((int64_t)1 << a.chunk_log2, I.units - u0);
        const bool last_chunk = chunk == I.n_chunks - 1;

        if (first) {
            // ---- pass 1 of one chunk: tables of the tile, LDS histogram, merge, maybe finalise
            using Y = P1FLayout<true>;
            const int4* gt = a.w.tab + (int64_t)t * 3 * kHistBins;
            char* pb = reinterpret_cast<char*>(S.p1.mem);
            for (int i = tid; i < 3 * kHistBins * Y::kCopies; i += RUN_THREADS) {
                const int c = i / (kHistBins * Y::kCopies), k = (i / Y::kCopies) % kHistBins, r = i % Y::kCopies;
                const uint32_t off = (c == 0 ? 0u : c == 1 ? Y::kG : (Y::kBRegion | Y::kB)) + ((uint32_t)k << 8);
                *reinterpret_cast<int4*>(pb + off + r * 16) = gt[c * kHistBins + k];
            }
            uint32_t* words = reinterpret_cast<uint32_t*>(S.p1.mem);
            for (int i = tid; i < kHistBins * 2 * Y::kCols; i += RUN_THREADS)
                words[(Y::kHRegion + (uint32_t)(i / (2 * Y::kCols)) * 256u + Y::kH) / 4 + (i % (2 * Y::kCols))] = 0u;
            for (int i = tid; i < 3 * kHistBins; i += RUN_THREADS)
                S.p1.od[i / kHistBins][i % kHistBins] = a.w.od[i];   // computed once by k_tiles_setup
            if (tid == 0) { S.p1.B = a.w.basis[t]; S.p1.shift = I.shift; }
            __syncthreads();
            P1Params pp = a.pp;                        // the tile's range
            pp.hist_hi[0] = I.hh[0];
            pp.hist_hi[1] = I.hh[1];
            pp.range = nullptr;
            if (cnt > 0 && !I.bad) {
                const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(T.src, u0, cnt);
                if (I.shift == 16) p1f_run<true, RUN_P1_UNROLL, true>(S.p1, pp, rs, cnt, tid, RUN_THREADS);
                else p1f_run<true, RUN_P1_UNROLL, false>(S.p1, pp, rs, cnt, tid, RUN_THREADS);
            }
            if (last_chunk && tid == 0 && I.tail && !I.bad) p1f_tail(S.p1, pp, T.src + 12 * I.units, I.tail);
            p1f_merge(S.p1, reinterpret_cast<unsigned long long*>(a.w.hist + (int64_t)t * 2 * kHistBins));
            __syncthreads();
            if (tid == 0) {
                const uint32_t prev = __hip_atomic_fetch_add(&a.w.done[t], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                S.last = prev == (uint32_t)I.n_chunks - 1;
            }
            __syncthreads();
            if (S.last) {
                // every chunk of the tile has merged: percentile, scale, recolouring constants
                // (atomic loads read the counts at the device coherence point, whatever this XCD's L2 holds)
                uint64_t* gh = a.w.hist + (int64_t)t * 2 * kHistBins;
                if (tid < 2 * kHistBins) S.h[tid] = __hip_atomic_load(gh + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                block_percentiles(S.h, a.q, I.hh, S.F);
                if (tid == 0) {
                    double s[2];
                    int fl[2];
                    for (int j = 0; j < 2; ++j) {
                        fl[j] = stain_flags(S.F, j, I.ok) | (I.bad ? SPCN_FLAG_BATCH : 0);
                        s[j] = stain_scale((double)a.scale_tgt[j], S.F.P[j], fl[j]);
                        if (a.p99_out) a.p99_out[2 * t + j] = (float)S.F.P[j];
                        if (a.scale_out) a.scale_out[2 * t + j] = (float)s[j];
                        if (a.flags_out) a.flags_out[2 * t + j] = fl[j];
                    }
                    RecolourConsts K;
                    make_recolour(K, a.w_tgt, s, a.i0_out, a.w.basis[t]);
                    a.w.K[t] = K;
                    __hip_atomic_store(&a.w.ready[t], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        } else {
            // ---- pass 2 of one chunk: wait for the tile's constants, recolour
            if (tid == 0) {
                uint32_t spins = 0;
                int go = 1;
                while (__hip_atomic_load(&a.w.ready[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > SPIN_LIMIT) {
                        go = 0;
                        atomicOr(&a.w.head->error, 1);
                        if (a.flags_out) {
                            atomicOr(a.flags_out + 2 * t, SPCN_FLAG_BATCH | SPCN_FLAG_TIMEOUT);
                            atomicOr(a.flags_out + 2 * t + 1, SPCN_FLAG_BATCH | SPCN_FLAG_TIMEOUT);
                        }
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // pairs with the release of ready[t]
                S.go = go && !I.bad;
                if (go) S.K = a.w.K[t];
            }
            const float2* gf = a.w.ftab + (int64_t)t * 3 * kHistBins;
            for (int i = tid; i < 3 * kHistBins; i += RUN_THREADS) S.p2.ftab[i] = gf[i];
            __syncthreads();
            if (S.go) {
                const RecolourConsts K = S.K;
                if (cnt > 0)
                    p2_chunk<1, RUN_UNROLL>(S.p2, K, chunk_rsrc(T.src, u0, cnt), chunk_rsrc(T.out, u0, cnt), cnt, tid,
                                            RUN_THREADS);
                if (last_chunk && tid == 0 && I.tail)
                    p2_tail(S.p2, K, T.src + 12 * I.units, T.out + 12 * I.units, I.tail);
            }
        }
        __syncthreads();
    }
}

}  // namespace

int64_t batched_max_tiles() { return MAX_TILES; }

size_t batched_workspace_bytes(int64_t n_tiles, int64_t total_px) {
    if (n_tiles <= 0) return 0;
    const int64_t n = n_tiles;
    size_t b = a256(sizeof(BatchHead)) + a256(n * sizeof(TileInfo)) + a256(n * sizeof(Basis64)) +
               a256(n * 3 * kHistBins * sizeof(int4)) + a256(n * 3 * kHistBins * sizeof(float2)) +
               a256(n * sizeof(RecolourConsts)) + a256(n * 2 * kHistBins * sizeof(uint64_t)) +
               2 * a256(n * sizeof(uint32_t)) + a256(3 * kHistBins * sizeof(double)) +
               a256(max_items_for(n, total_px) * sizeof(int32_t));
    return b;
}

hipError_t launch_normalize_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t total_px, const float* w_src,
                                    const float* w_tgt, const float* scale_tgt, const float i0_out[3],
                                    const ParamsK& pk, float* p99_out, float* scale_out, int32_t* flags_out,
                                    void* ws, const DevInfo& dev, hipStream_t s) {
    BatchWs w = carve(ws, n_tiles, total_px);
    SetupArgs sa{};
    const int chunk_log2 = option(SPCN_OPT_BATCH_CHUNK);
    sa.tiles = tiles; sa.w_src = w_src; sa.w = w; sa.chunk_log2 = chunk_log2;
    for (int c = 0; c < 3; ++c) sa.pp.i0[c] = pk.i0[c];
    sa.pp.lambda = pk.lambda; sa.pp.white_sum = pk.white_sum;
    sa.pp.hist_hi[0] = pk.hist_hi[0]; sa.pp.hist_hi[1] = pk.hist_hi[1];
    sa.pp.range = pk.hist_hi_dev;    // [n_tiles][2] when given
    hipLaunchKernelGGL(k_tiles_setup, dim3(n_tiles), dim3(256), 0, s, sa);
    hipLaunchKernelGGL(k_tiles_plan, dim3(1), dim3(1024), 0, s, w, (int)n_tiles, total_px,
                       max_items_for(n_tiles, total_px), flags_out);
    RunArgs ra{};
    ra.tiles = tiles; ra.w_tgt = w_tgt; ra.scale_tgt = scale_tgt;
    for (int c = 0; c < 3; ++c) ra.i0_out[c] = i0_out[c];
    ra.pp = sa.pp; ra.q = pk.q64; ra.w = w; ra.chunk_log2 = chunk_log2;
    ra.p99_out = p99_out; ra.scale_out = scale_out; ra.flags_out = flags_out;
    hipLaunchKernelGGL(k_tiles_run, dim3(dev.cus), dim3(RUN_THREADS), 0, s, ra);
    return hipGetLastError();
}

}  // namespace spcn
