// spcn_batched.hip -- a batch of uneven uint8 tiles, each with its own source basis, normalised to
// one target (Eqs. 1-4 per tile; batch-to-one-target as in Sec. 3.2 item 6), with no host
// synchronisation, so the whole batch can be captured into one graph.
//
// k_tiles_setup   one workgroup per tile: FP64 basis quantities, fixed-point pass-1 tables and FP32
//                 pass-2 tables of the tile into the workspace; zeroes the tile's histogram.
// k_tiles_plan    one workgroup: pass-1 items and pass-2 chunks of every tile (two exclusive scans),
//                 item -> tile and chunk -> tile maps, queue reset.
// k_tiles_p1      persistent pass 1 (one 1024-thread workgroup per CU, the wide byte-permute layout):
//                 dequeues pass-1 items (2^chunk_log2 units of one tile) from a global counter and adds
//                 each item's exact histogram to its tile's.
// k_tiles_check   one workgroup per tile: the tile's Eq. 3 percentile.  A stain whose percentile lies
//                 in the open last bin (with auto_range) gets twice its range: the tile's pass-1 tables
//                 are rebuilt, its histogram cleared and the tile marked for a second pass 1; every
//                 other tile gets its scale and recolouring constants.
// k_tiles_p1 again (retry round): the items of marked tiles only; then k_tiles_check finishes them.
// k_tiles_p2      grid-stride pass 2 over fixed chunks of 4096 units (256 threads x 16 units, as the
//                 single-image recolour): a workgroup loads a tile's tables and constants into LDS
//                 when its next chunk belongs to another tile.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int P1_THREADS = 1024;
constexpr int P1_UNROLL = 4;                  // pass-1 units per thread and iteration (as the slide's pass 1)
constexpr int P2_THREADS = 256;
constexpr int P2_UNROLL = 16;                 // pass-2 units per thread and chunk
constexpr int P2_CHUNK_LOG2 = 12;             // 4096 units = P2_THREADS * P2_UNROLL
constexpr int P2_GROUP = 4;                   // adjacent chunks a workgroup takes per step of its walk
static_assert((1 << P2_CHUNK_LOG2) == P2_THREADS * P2_UNROLL, "one pass-2 chunk per workgroup pass");
constexpr int MIN_CHUNK_LOG2 = 12;            // smallest pass-1 item: 4096 units = 16384 pixels
constexpr int MAX_TILES = 8192;

struct TileInfo {
    int64_t units;          // full 4-pixel units
    int32_t tail;           // remaining pixels (0..3)
    int32_t n_chunks;       // pass-1 items of the tile (>= 1)
    int64_t item0;          // first pass-1 item of the tile
    int64_t chunk0;         // first pass-2 chunk of the tile
    int32_t p2_chunks;      // pass-2 chunks of the tile (>= 1)
    int32_t shift;          // fixed-point resolution u of the pass-1 tables
    int32_t ok;             // basis usable
    int32_t bad;            // descriptor unusable (null or misaligned pointer, empty tile): skipped
    float hh[2];            // histogram range of the tile's stains
};

struct BatchHead {
    uint32_t queue;         // next pass-1 item to hand out (first round)
    uint32_t p1_items;
    uint32_t p2_chunks;
    int32_t error;          // the tiles hold more than the workspace was sized for
};

struct BatchWs {
    BatchHead* head;
    TileInfo* info;         // [n]
    Basis64* basis;         // [n]
    int4* tab;              // [n][3 * 256]
    float2* ftab;           // [n][3 * 256]
    RecolourConsts* K;      // [n]
    uint64_t* hist;         // [n][512]
    uint32_t* retry;        // [n] bit j: stain j's range was doubled, pass 1 of the tile runs again
    double* od;             // [3][256] FP64 optical densities (Eq. 1), for the near-edge path
    int32_t* item_tile;     // [max items]
    int32_t* chunk_tile;    // [max chunks]
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Upper bound of the work units of a batch cut into pieces of 2^log2 units (one partial piece per tile).
__host__ __device__ inline int64_t max_pieces(int64_t n_tiles, int64_t total_px, int log2) {
    return total_px / (4 * ((int64_t)1 << log2)) + n_tiles;
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
    w.retry = reinterpret_cast<uint32_t*>(p); p += a256(n * sizeof(uint32_t));
    w.od = reinterpret_cast<double*>(p); p += a256(3 * kHistBins * sizeof(double));
    w.item_tile = reinterpret_cast<int32_t*>(p); p += a256(max_pieces(n, total_px, MIN_CHUNK_LOG2) * sizeof(int32_t));
    w.chunk_tile = reinterpret_cast<int32_t*>(p); p += a256(max_pieces(n, total_px, P2_CHUNK_LOG2) * sizeof(int32_t));
    return w;
}

// Fixed-point pass-1 table entries of one tile for intensity k (thread k of 256), in the shifted-guard
// form of the byte-permute layout (see spcn_passes.hpp).
__device__ void tile_p1_entries(const Basis64& B, const float i0[3], const float hh[2], int u, int k, int4* tab) {
    const double sig0 = ldexp(256.0 / (double)hh[0], u), sig1 = ldexp(256.0 / (double)hh[1], u);
    for (int c = 0; c < 3; ++c) {
        const double od = B.ok ? od_u8((double)i0[c], k) : 0.0;
        const int g = c == 0 ? kGuardUnits - 2 * kGuardUnits : 0;
        int4 e;
        e.x = __double2int_rn((B.pc[0][c] * od + (c == 0 ? B.pconst[0] : 0.0)) * sig0) + g;
        e.y = __double2int_rn((B.q[0][c] * od + (c == 0 ? B.fconst[0] : 0.0)) * sig0) + g;
        e.z = __double2int_rn((B.pc[1][c] * od + (c == 0 ? B.pconst[1] : 0.0)) * sig1) + g;
        e.w = __double2int_rn((B.q[1][c] * od + (c == 0 ? B.fconst[1] : 0.0)) * sig1) + g;
        tab[c * kHistBins + k] = e;
    }
}

__device__ inline int tile_shift(const Basis64& B, const float i0[3], const float hh[2]) {
    const int u = table_shift(B, i0, hh);
    return u < 16 ? u : 16;                 // the byte-permute layout works in <= 2^16 units
}

struct SetupArgs {
    const spcn_tile* tiles;
    const float* w_src;         // [n][6]
    P1Params pp;
    int chunk_log2;             // 4-pixel units per pass-1 item = 2^chunk_log2
    BatchWs w;
};

__global__ __launch_bounds__(256) void k_tiles_setup(SetupArgs a) {
    __shared__ Basis64 B;
    __shared__ int s_shift;
    __shared__ float s_hh[2];
    const int t = blockIdx.x;
    if (threadIdx.x == 0) {
        derive_basis(a.w_src + 6 * t, a.pp.lambda, B);
        s_hh[0] = resolve_range(a.pp.range ? a.pp.range + 2 * t : nullptr, a.pp.hist_hi[0]);
        s_hh[1] = resolve_range(a.pp.range ? a.pp.range + 2 * t + 1 : nullptr, a.pp.hist_hi[1]);
        s_shift = tile_shift(B, a.pp.i0, s_hh);
        const spcn_tile T = a.tiles[t];
        const int64_t n_px = T.height * T.width;
        TileInfo I;
        I.units = n_px >> 2;
        I.tail = (int32_t)(n_px & 3);
        I.n_chunks = (int32_t)((I.units + ((int64_t)1 << a.chunk_log2) - 1) >> a.chunk_log2);
        I.p2_chunks = (int32_t)((I.units + ((int64_t)1 << P2_CHUNK_LOG2) - 1) >> P2_CHUNK_LOG2);
        I.item0 = 0;
        I.chunk0 = 0;
        I.shift = s_shift;
        I.ok = B.ok;
        I.bad = !T.src || !T.out || (((uintptr_t)T.src | (uintptr_t)T.out) & 3) || T.height <= 0 || T.width <= 0;
        I.hh[0] = s_hh[0];
        I.hh[1] = s_hh[1];
        if (I.bad) { I.units = 0; I.tail = 0; }
        if (I.n_chunks < 1) I.n_chunks = 1;      // a tile of fewer than 4 pixels still has its tail
        if (I.p2_chunks < 1) I.p2_chunks = 1;
        a.w.info[t] = I;
        a.w.basis[t] = B;
        a.w.retry[t] = 0;
    }
    for (int i = threadIdx.x; i < 2 * kHistBins; i += blockDim.x) a.w.hist[(int64_t)t * 2 * kHistBins + i] = 0;
    if (t == 0)
        for (int i = threadIdx.x; i < 3 * kHistBins; i += blockDim.x)
            a.w.od[i] = od_u8((double)a.pp.i0[i / kHistBins], i % kHistBins);
    __syncthreads();
    const int k = threadIdx.x;
    tile_p1_entries(B, a.pp.i0, s_hh, s_shift, k, a.w.tab + (int64_t)t * 3 * kHistBins);
    for (int c = 0; c < 3; ++c) {
        const double od = B.ok ? od_u8((double)a.pp.i0[c], k) : 0.0;
        float2 f;
        f.x = (float)(B.q[0][c] * od + (c == 0 ? B.fconst[0] : 0.0));
        f.y = (float)(B.q[1][c] * od + (c == 0 ? B.fconst[1] : 0.0));
        a.w.ftab[((int64_t)t * 3 + c) * kHistBins + k] = f;
    }
}

// Exclusive scan (1024 threads) of per-tile counts read by get(t); off_out(t, first) receives each
// tile's first index.  Returns the total on every thread.
template <class Get, class Put>
__device__ int scan_tiles(int n_tiles, int32_t* s_off, int32_t* s_part, Get get, Put put) {
    const int t0 = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    int run = 0;
    for (int i = 0; i < per; ++i) {
        const int t = t0 * per + i;
        if (t < n_tiles) { s_off[t] = run; run += get(t); }
    }
    s_part[t0] = run;
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
        if (t < n_tiles) { s_off[t] += excl; put(t, s_off[t]); }
    }
    const int total = s_part[1023];
    __syncthreads();
    return total;
}

// Item and chunk plans (the maps are filled by k_tiles_maps).  The caller's total_px must bound the tiles' pixel count (it sized the
// workspace); otherwise the whole batch is refused (nothing is processed, SPCN_FLAG_BATCH).
__global__ __launch_bounds__(1024) void k_tiles_plan(BatchWs w, int n_tiles, int64_t total_px, int chunk_log2,
                                                     int32_t* flags_out) {
    __shared__ int32_t s_off[MAX_TILES];
    __shared__ int32_t s_part[1024];
    __shared__ unsigned long long s_px;
    const int t0 = threadIdx.x;
    if (t0 == 0) s_px = 0;
    __syncthreads();
    int64_t px = 0;
    for (int t = t0; t < n_tiles; t += 1024) px += 4 * w.info[t].units + w.info[t].tail;
    atomicAdd(&s_px, (unsigned long long)px);
    const int items = scan_tiles(n_tiles, s_off, s_part, [&](int t) { return w.info[t].n_chunks; },
                                 [&](int t, int first) { w.info[t].item0 = first; });
    const bool fits = items <= max_pieces(n_tiles, total_px, chunk_log2) && (int64_t)s_px <= total_px;
    const int chunks = scan_tiles(n_tiles, s_off, s_part, [&](int t) { return w.info[t].p2_chunks; },
                                  [&](int t, int first) { w.info[t].chunk0 = first; });
    const bool fits2 = fits && chunks <= max_pieces(n_tiles, total_px, P2_CHUNK_LOG2);
    if (t0 == 0) {
        w.head->queue = 0;
        w.head->p1_items = fits2 ? (uint32_t)items : 0u;
        w.head->p2_chunks = fits2 ? (uint32_t)chunks : 0u;
        w.head->error = fits2 ? 0 : 2;
    }
    if (flags_out)
        for (int t = t0; t < n_tiles; t += 1024) {
            const int f = (!fits2 || w.info[t].bad) ? SPCN_FLAG_BATCH : 0;
            flags_out[2 * t] = f;
            flags_out[2 * t + 1] = f;
        }
}

// The item -> tile and chunk -> tile maps: workgroup t writes tile t's entries (nothing for a
// refused batch).
__global__ __launch_bounds__(256) void k_tiles_maps(BatchWs w) {
    if (w.head->error) return;
    const int t = blockIdx.x;
    const TileInfo I = w.info[t];
    for (int i = threadIdx.x; i < I.n_chunks; i += blockDim.x) w.item_tile[I.item0 + i] = t;
    for (int i = threadIdx.x; i < I.p2_chunks; i += blockDim.x) w.chunk_tile[I.chunk0 + i] = t;
}

struct P1RunArgs {
    const spcn_tile* tiles;
    P1Params pp;
    int chunk_log2;
    int round;              // 0: every item from the queue; 1: items of tiles marked for a retry
    BatchWs w;
};

// Pass 1 of one item: the tile's tables into LDS, the item's pixels into the LDS histogram, merged
// into the tile's histogram.
__device__ void p1_item(P1FLds<true>& S, const P1RunArgs& a, int t, uint32_t item) {
    using Y = P1FLayout<true>;
    const int tid = threadIdx.x;
    const TileInfo I = a.w.info[t];
    const spcn_tile T = a.tiles[t];
    const int chunk = (int)(item - (uint32_t)I.item0);
    const int64_t u0 = (int64_t)chunk << a.chunk_log2;
    const int cnt = (int)min((int64_t)1 << a.chunk_log2, I.units - u0);
    const int4* gt = a.w.tab + (int64_t)t * 3 * kHistBins;
    char* pb = reinterpret_cast<char*>(S.mem);
    for (int i = tid; i < 3 * kHistBins * Y::kCopies; i += P1_THREADS) {
        const int c = i / (kHistBins * Y::kCopies), k = (i / Y::kCopies) % kHistBins, r = i % Y::kCopies;
        const uint32_t off = (c == 0 ? 0u : c == 1 ? Y::kG : (Y::kBRegion | Y::kB)) + ((uint32_t)k << 8);
        *reinterpret_cast<int4*>(pb + off + r * 16) = gt[c * kHistBins + k];
    }
    uint32_t* words = reinterpret_cast<uint32_t*>(S.mem);
    for (int i = tid; i < kHistBins * 2 * Y::kCols; i += P1_THREADS)
        words[Y::hist_word(i / (2 * Y::kCols), i % (2 * Y::kCols))] = 0u;
    if (tid == 0) { S.B = a.w.basis[t]; S.shift = I.shift; }
    __syncthreads();
    P1Params pp = a.pp;                        // the tile's range
    pp.hist_hi[0] = I.hh[0];
    pp.hist_hi[1] = I.hh[1];
    pp.range = nullptr;
    if (cnt > 0 && !I.bad) {
        const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(T.src, u0, cnt);
        if (I.shift == 16) p1f_run<true, P1_UNROLL, true>(S, pp, rs, cnt, tid, P1_THREADS);
        else p1f_run<true, P1_UNROLL, false>(S, pp, rs, cnt, tid, P1_THREADS);
    }
    if (chunk == I.n_chunks - 1 && tid == 0 && I.tail && !I.bad) p1f_tail(S, pp, T.src + 12 * I.units, I.tail);
    p1f_merge(S, reinterpret_cast<unsigned long long*>(a.w.hist + (int64_t)t * 2 * kHistBins));
    __syncthreads();                           // the LDS is reused by the next item
}

__global__ __launch_bounds__(P1_THREADS) void k_tiles_p1(P1RunArgs a) {
    __shared__ P1FLds<true> S;
    __shared__ uint32_t s_item;
    const uint32_t n_items = a.w.head->p1_items;
    for (int i = threadIdx.x; i < 3 * kHistBins; i += P1_THREADS)
        S.od[i / kHistBins][i % kHistBins] = a.w.od[i];   // computed once by k_tiles_setup
    uint32_t next = blockIdx.x;                // the retry round walks the items statically
    for (;;) {
        // the next item: from the queue, or (retry round) the next one of a marked tile
        if (threadIdx.x == 0) {
            uint32_t item = n_items;
            if (a.round == 0) {
                item = atomicAdd(&a.w.head->queue, 1u);
            } else {
                for (; next < n_items; next += gridDim.x)
                    if (a.w.retry[a.w.item_tile[next]] != 0u) break;
                item = next;
                next += gridDim.x;
            }
            s_item = item;
        }
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= n_items) break;
        p1_item(S, a, a.w.item_tile[item], item);
    }
}

struct CheckArgs {
    const float* w_tgt;
    const float* scale_tgt;
    float i0[3];
    float i0_out[3];
    double q;
    int auto_range;
    int round;              // 0: after the first pass 1; 1: after the retry pass 1
    BatchWs w;
    float* p99_out;
    float* scale_out;
    int32_t* flags_out;
    uint64_t* hist_out;
};

// One workgroup (256 threads) per tile: Eq. 3's percentile, then either the retry set-up or the
// tile's scale and recolouring constants.
__global__ __launch_bounds__(256) void k_tiles_check(CheckArgs a) {
    __shared__ FinalShared F;
    __shared__ uint64_t s_h[2 * kHistBins];
    __shared__ int s_bits;
    __shared__ float s_hh[2];
    __shared__ int s_shift;
    const int t = blockIdx.x, tid = threadIdx.x;
    if (a.w.head->error) return;               // the batch was refused: its tiles keep SPCN_FLAG_BATCH
    const uint32_t prev = a.w.retry[t];
    if (a.round == 1 && prev == 0u) return;    // finished in the first round
    const TileInfo I = a.w.info[t];
    uint64_t* gh = a.w.hist + (int64_t)t * 2 * kHistBins;
    s_h[tid] = gh[tid];
    s_h[kHistBins + tid] = gh[kHistBins + tid];
    __syncthreads();
    block_percentiles(s_h, a.q, I.hh, F);
    const Basis64& B = a.w.basis[t];
    if (tid == 0) {
        int bits = 0;
        if (a.round == 0 && a.auto_range && !I.bad)
            for (int j = 0; j < 2; ++j)
                if (F.kstar[j] == kHistBins - 1 && I.hh[j] < 256.0f) bits |= 1 << j;
        s_bits = bits;
        if (bits) {
            for (int j = 0; j < 2; ++j) s_hh[j] = (bits >> j & 1) ? 2.0f * I.hh[j] : I.hh[j];
            s_shift = tile_shift(B, a.i0, s_hh);
        }
    }
    __syncthreads();
    if (s_bits) {   // rebuild the tile's pass-1 tables at the new range and clear its histogram
        tile_p1_entries(B, a.i0, s_hh, s_shift, tid, a.w.tab + (int64_t)t * 3 * kHistBins);
        gh[tid] = 0;
        gh[kHistBins + tid] = 0;
        if (tid == 0) {
            a.w.info[t].hh[0] = s_hh[0];
            a.w.info[t].hh[1] = s_hh[1];
            a.w.info[t].shift = s_shift;
            a.w.retry[t] = (uint32_t)s_bits;
        }
        return;
    }
    if (a.hist_out) {
        a.hist_out[(int64_t)t * 2 * kHistBins + tid] = s_h[tid];
        a.hist_out[(int64_t)t * 2 * kHistBins + kHistBins + tid] = s_h[kHistBins + tid];
    }
    if (tid == 0) {
        double s[2];
        int fl[2];
        for (int j = 0; j < 2; ++j) {
            fl[j] = stain_flags(F, j, I.ok) | (I.bad ? SPCN_FLAG_BATCH : 0) | ((prev >> j & 1) ? SPCN_FLAG_RANGE_RETRY : 0) |
                    scale_flag(a.scale_tgt[j]);
            s[j] = stain_scale((double)a.scale_tgt[j], F.P[j], fl[j]);
            if (a.p99_out) a.p99_out[2 * t + j] = (float)F.P[j];
            if (a.scale_out) a.scale_out[2 * t + j] = (float)s[j];
            if (a.flags_out) a.flags_out[2 * t + j] = fl[j];
        }
        RecolourConsts K;
        make_recolour(K, a.w_tgt, s, a.i0_out, B);
        a.w.K[t] = K;
    }
}

struct P2RunArgs {
    const spcn_tile* tiles;
    BatchWs w;
};

// Grid-stride pass 2 over the batch's chunks (chunk c of the batch: its tile from the map, then the
// chunk's units within that tile), loads of the next chunk in flight while one is recoloured.  The
// walk takes P2_GROUP adjacent chunks per step of the grid (step k of workgroup b: chunk
// (k / P2_GROUP) * P2_GROUP * grid + b * P2_GROUP + k % P2_GROUP), so a workgroup mostly stays on
// one tile and reloads its tables only when the tile changes.
__global__ __launch_bounds__(P2_THREADS, 3) void k_tiles_p2(P2RunArgs a) {
    __shared__ P2Lds<1> T2;
    __shared__ RecolourConsts s_K;
    const int tid = threadIdx.x;
    const int64_t n = a.w.head->p2_chunks;
    constexpr int64_t CH = (int64_t)1 << P2_CHUNK_LOG2;
    struct Where { int t; int64_t u0; int cnt; bool last; };
    auto where = [&](int64_t c) -> Where {     // wave-uniform
        Where r{-1, 0, 0, false};
        if (c < n) {
            r.t = __builtin_amdgcn_readfirstlane(a.w.chunk_tile[c]);
            const TileInfo& I = a.w.info[r.t];
            r.u0 = (c - I.chunk0) << P2_CHUNK_LOG2;
            r.cnt = I.bad ? 0 : (int)min(CH, I.units - r.u0);
            r.last = c - I.chunk0 == I.p2_chunks - 1;
        }
        return r;
    };
    const int64_t span = (int64_t)P2_GROUP * gridDim.x;
    auto chunk_at = [&](int64_t k) { return (k / P2_GROUP) * span + (int64_t)blockIdx.x * P2_GROUP + k % P2_GROUP; };
    Where cw = where(chunk_at(0));             // t = -1 past the end (chunk_at increases with k)
    u32x3 cur[P2_UNROLL];
    {
        const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(cw.t >= 0 ? a.tiles[cw.t].src : nullptr, cw.u0, cw.cnt);
#pragma unroll
        for (int j = 0; j < P2_UNROLL; ++j)
            cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * P2_THREADS), 0, kLoadStream);
    }
    int staged = -1;
    for (int64_t k = 0; cw.t >= 0; ++k) {     // workgroup-uniform
        const Where nw = where(chunk_at(k + 1));   // past the end: an empty range, the loads return zeros
        u32x3 nxt[P2_UNROLL];
        {
            const __amdgpu_buffer_rsrc_t rn = chunk_rsrc(nw.t >= 0 ? a.tiles[nw.t].src : nullptr, nw.u0, nw.cnt);
#pragma unroll
            for (int j = 0; j < P2_UNROLL; ++j)
                nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * P2_THREADS), 0, kLoadStream);
        }
        if (cw.t != staged) {                  // the tile's tables and constants
            __syncthreads();
            const float2* gf = a.w.ftab + (int64_t)cw.t * 3 * kHistBins;
            for (int i = tid; i < 3 * kHistBins; i += P2_THREADS) T2.ftab[i] = gf[i];
            if (tid == 0) s_K = a.w.K[cw.t];
            staged = cw.t;
            __syncthreads();
        }
        const RecolourConsts K = uniform_consts(s_K);
        const spcn_tile T = a.tiles[cw.t];
        const __amdgpu_buffer_rsrc_t ws = chunk_rsrc(T.out, cw.u0, cw.cnt);
#pragma unroll
        for (int j = 0; j < P2_UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) p2_densities(T2, 0u, K, px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            __builtin_amdgcn_raw_buffer_store_b96(recolour_unit(h0, h1, K), ws, 12 * (tid + j * P2_THREADS), 0, kStoreStream);
        }
        const TileInfo& I = a.w.info[cw.t];
        if (cw.last && tid == 0 && I.tail && !I.bad)
            p2_tail(T2, K, T.src + 12 * I.units, T.out + 12 * I.units, I.tail);
#pragma unroll
        for (int j = 0; j < P2_UNROLL; ++j) cur[j] = nxt[j];
        cw = nw;
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
               a256(n * sizeof(uint32_t)) + a256(3 * kHistBins * sizeof(double)) +
               a256(max_pieces(n, total_px, MIN_CHUNK_LOG2) * sizeof(int32_t)) +
               a256(max_pieces(n, total_px, P2_CHUNK_LOG2) * sizeof(int32_t));
    return b;
}

hipError_t launch_normalize_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t total_px, const float* w_src,
                                    const float* w_tgt, const float* scale_tgt, const float i0_out[3],
                                    const ParamsK& pk, float* p99_out, float* scale_out, int32_t* flags_out,
                                    uint64_t* hist_out, void* ws, const DevInfo& dev, hipStream_t s) {
    BatchWs w = carve(ws, n_tiles, total_px);
    SetupArgs sa{};
    const int chunk_log2 = option(SPCN_OPT_BATCH_CHUNK);
    sa.tiles = tiles; sa.w_src = w_src; sa.w = w; sa.chunk_log2 = chunk_log2;
    for (int c = 0; c < 3; ++c) sa.pp.i0[c] = pk.i0[c];
    sa.pp.lambda = pk.lambda; sa.pp.white_sum = pk.white_sum;
    sa.pp.hist_hi[0] = pk.hist_hi[0]; sa.pp.hist_hi[1] = pk.hist_hi[1];
    sa.pp.range = pk.hist_hi_dev;    // [n_tiles][2] when given
    hipLaunchKernelGGL(k_tiles_setup, dim3(n_tiles), dim3(256), 0, s, sa);
    hipLaunchKernelGGL(k_tiles_plan, dim3(1), dim3(1024), 0, s, w, (int)n_tiles, total_px, chunk_log2, flags_out);
    hipLaunchKernelGGL(k_tiles_maps, dim3(n_tiles), dim3(256), 0, s, w);

    P1RunArgs pa{};
    pa.tiles = tiles; pa.pp = sa.pp; pa.pp.range = nullptr; pa.chunk_log2 = chunk_log2; pa.w = w;
    CheckArgs ca{};
    ca.w_tgt = w_tgt; ca.scale_tgt = scale_tgt; ca.q = pk.q64; ca.auto_range = pk.auto_range; ca.w = w;
    for (int c = 0; c < 3; ++c) { ca.i0[c] = pk.i0[c]; ca.i0_out[c] = i0_out[c]; }
    ca.p99_out = p99_out; ca.scale_out = scale_out; ca.flags_out = flags_out; ca.hist_out = hist_out;
    for (int round = 0; round < (pk.auto_range ? 2 : 1); ++round) {
        pa.round = round;
        ca.round = round;
        hipLaunchKernelGGL(k_tiles_p1, dim3(dev.cus), dim3(P1_THREADS), 0, s, pa);
        hipLaunchKernelGGL(k_tiles_check, dim3(n_tiles), dim3(256), 0, s, ca);
    }
    P2RunArgs ra{};
    ra.tiles = tiles; ra.w = w;
    hipLaunchKernelGGL(k_tiles_p2, dim3(dev.cus * 8), dim3(P2_THREADS), 0, s, ra);
    return hipGetLastError();
}

}  // namespace spcn
