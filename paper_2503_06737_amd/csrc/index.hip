// Index construction on gfx950 (Section 3.1: store every point in the
// bucket of its key, one table per group of K components).
//
// Per table, the (key, id) pairs are put in (key, id) order by a stable
// least-significant-digit radix sort over the 64-bit key, 8 bits per pass:
//   hist   - one read of all keys: the 8 digit histograms of every table;
//   plan   - per table, drop the passes whose digit is the same for every key
//            (an identity permutation; SRP keys of K bits use ceil(K/8)
//            passes) and route the remaining passes between two buffers so
//            the last one lands in the index;
//   upsweep/scan/downsweep per pass - tile digit counts, their exclusive scan
//            over tiles (offset of each tile's run of each digit), and the
//            stable scatter: inside a tile, each wave ranks its 64-key rows
//            with 8 ballots per row (lanes holding the same digit), the ranks
//            are turned into tile positions through per-wave digit counters
//            in LDS, the tile is reordered in LDS and written out as
//            contiguous digit runs.
// Then bucket boundaries: heads (key differs from its predecessor) are
// counted per tile, scanned per table, and the distinct keys and the start
// offset of every bucket are written.

#include "lsh_internal.h"

namespace lsh {

constexpr int kSortThreads = 1024;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems; // 8192 keys per tile
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kPasses = 8;
constexpr int kRadix = 256;

constexpr int kHeadThreads = 256;
constexpr int kHeadItems = 16;
constexpr int kHeadTile = kHeadThreads * kHeadItems;

struct SortArgs {
    const uint64_t *kin; // input keys [L][key_ld]
    int64_t key_ld;
    int64_t n;
    int32_t L;
    uint32_t id_base;
    uint64_t *ka, *kb;   // key buffers [L][n]
    uint32_t *ia, *ib;   // id buffers [L][n] (ia = index sorted_ids)
    uint32_t *ghist;     // [L][8][256]
    int32_t *plan;       // [L][8]: -1 skip, else src | dst << 2 (0 = input, 1 = A, 2 = B)
    uint32_t *tile_hist; // [L][ntiles][256]
    int32_t ntiles;
};

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int p) { return (uint32_t)(k >> (8 * p)) & 255u; }

// ------------------------------------------------------------------ hist

__global__ __launch_bounds__(kSortThreads) void sort_hist_kernel(SortArgs a)
{
    __shared__ uint32_t h[kPasses][kRadix];
    const int t = blockIdx.y;
    for (int i = threadIdx.x; i < kPasses * kRadix; i += blockDim.x)
        (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t *k = a.kin + (int64_t)t * a.key_ld;
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + it * kSortThreads + threadIdx.x;
        const bool valid = i < a.n;
        uint64_t key = valid ? k[i] : 0;
        const uint64_t vmask = __ballot(valid);
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            // a digit shared by every valid lane (common: the zero high bytes
            // of SRP keys) is added once per wave instead of 64 times
            uint32_t dg = digit_of(key, p);
            uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
            if ((__ballot(valid && dg == d0) == vmask) && vmask == ~0ull) {
                if (lane_id() == 0)
                    atomicAdd(&h[p][d0], 64u);
            } else if (valid) {
                atomicAdd(&h[p][dg], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *g = a.ghist + (int64_t)t * kPasses * kRadix;
    for (int i = threadIdx.x; i < kPasses * kRadix; i += blockDim.x) {
        uint32_t v = (&h[0][0])[i];
        if (v)
            atomicAdd(&g[i], v);
    }
}

// ------------------------------------------------------------------ plan

__global__ __launch_bounds__(kRadix) void sort_plan_kernel(SortArgs a)
{
    const int t = blockIdx.x;
    const uint32_t *g = a.ghist + (int64_t)t * kPasses * kRadix;
    __shared__ int s_trivial[kPasses];
    if (threadIdx.x < kPasses)
        s_trivial[threadIdx.x] = 0;
    __syncthreads();
    for (int p = 0; p < kPasses; ++p)
        if ((int64_t)g[p * kRadix + threadIdx.x] == a.n)
            s_trivial[p] = 1; // one digit value holds every key: identity pass
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    bool active[kPasses];
    int P = 0;
    for (int p = 0; p < kPasses; ++p) {
        active[p] = !s_trivial[p];
        P += active[p];
    }
    if (P == 0) { // every key equal: one pass still copies keys and ids out
        active[0] = true;
        P = 1;
    }
    int i = 0, src = 0;
    for (int p = 0; p < kPasses; ++p) {
        if (!active[p]) {
            a.plan[t * kPasses + p] = -1;
            continue;
        }
        int dst = ((P - 1 - i) % 2 == 0) ? 1 : 2;
        a.plan[t * kPasses + p] = src | (dst << 2);
        src = dst;
        ++i;
    }
}

// --------------------------------------------------------------- upsweep

__device__ __forceinline__ const uint64_t *src_keys(const SortArgs &a, int sel, int t)
{
    return sel == 0 ? a.kin + (int64_t)t * a.key_ld
                    : (sel == 1 ? a.ka : a.kb) + (int64_t)t * a.n;
}

__global__ __launch_bounds__(kSortThreads) void sort_upsweep_kernel(SortArgs a, int p)
{
    const int t = blockIdx.y;
    const int pl = a.plan[t * kPasses + p];
    if (pl < 0)
        return;
    __shared__ uint32_t h[kRadix];
    for (int i = threadIdx.x; i < kRadix; i += blockDim.x)
        h[i] = 0;
    __syncthreads();
    const uint64_t *k = src_keys(a, pl & 3, t);
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + it * kSortThreads + threadIdx.x;
        if (i < a.n)
            atomicAdd(&h[digit_of(k[i], p)], 1u);
    }
    __syncthreads();
    uint32_t *th = a.tile_hist + ((int64_t)t * a.ntiles + blockIdx.x) * kRadix;
    for (int i = threadIdx.x; i < kRadix; i += blockDim.x)
        th[i] = h[i];
}

// ------------------------------------------------------------------ scan
// tile_hist[t][tile][d] <- global start of tile's run of digit d.

__global__ __launch_bounds__(kRadix) void sort_scan_kernel(SortArgs a, int p)
{
    const int t = blockIdx.x;
    if (a.plan[t * kPasses + p] < 0)
        return;
    __shared__ uint32_t s[kRadix];
    const int d = threadIdx.x;
    // exclusive scan of the global digit counts
    uint32_t c = a.ghist[((int64_t)t * kPasses + p) * kRadix + d];
    s[d] = c;
    __syncthreads();
    for (int o = 1; o < kRadix; o <<= 1) {
        uint32_t v = d >= o ? s[d - o] : 0;
        __syncthreads();
        s[d] += v;
        __syncthreads();
    }
    uint32_t run = s[d] - c;
    uint32_t *th = a.tile_hist + (int64_t)t * a.ntiles * kRadix + d;
    int tile = 0;
    for (; tile + 4 <= a.ntiles; tile += 4) {
        uint32_t v0 = th[(tile + 0) * kRadix], v1 = th[(tile + 1) * kRadix];
        uint32_t v2 = th[(tile + 2) * kRadix], v3 = th[(tile + 3) * kRadix];
        th[(tile + 0) * kRadix] = run;
        run += v0;
        th[(tile + 1) * kRadix] = run;
        run += v1;
        th[(tile + 2) * kRadix] = run;
        run += v2;
        th[(tile + 3) * kRadix] = run;
        run += v3;
    }
    for (; tile < a.ntiles; ++tile) {
        uint32_t v = th[tile * kRadix];
        th[tile * kRadix] = run;
        run += v;
    }
}

// ------------------------------------------------------------- downsweep

__global__ __launch_bounds__(kSortThreads) void sort_downsweep_kernel(SortArgs a, int p)
{
    const int t = blockIdx.y;
    const int pl = a.plan[t * kPasses + p];
    if (pl < 0)
        return;
    const int src = pl & 3, dst = pl >> 2;

    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sid[kSortTile];
    __shared__ uint32_t whist[kSortWaves][kRadix];
    __shared__ uint32_t lbase[kRadix];
    __shared__ uint32_t gbase[kRadix];

    const int tid = threadIdx.x, wid = tid / kWave, lane = lane_id();
    for (int i = tid; i < kSortWaves * kRadix; i += blockDim.x)
        (&whist[0][0])[i] = 0;
    const uint32_t *toff = a.tile_hist + ((int64_t)t * a.ntiles + blockIdx.x) * kRadix;
    for (int i = tid; i < kRadix; i += blockDim.x)
        gbase[i] = toff[i];
    __syncthreads();

    const uint64_t *kin = src_keys(a, src, t);
    const uint32_t *iin = src == 0 ? nullptr : (src == 1 ? a.ia : a.ib) + (int64_t)t * a.n;
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tile0 + (int64_t)wid * (kWave * kSortItems);

    uint64_t key[kSortItems];
    uint32_t id[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = wbase + it * kWave + lane;
        if (i < a.n) {
            key[it] = kin[i];
            id[it] = iin ? iin[i] : a.id_base + (uint32_t)i;
        } else {
            key[it] = ~0ull; // sorts last, never written out
            id[it] = 0xffffffffu;
        }
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        uint32_t dg = digit_of(key[it], p);
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        uint32_t before = __popcll(peers & lt);
        uint32_t old = whist[wid][dg];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (before == 0)
            whist[wid][dg] = old + __popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        rank[it] = old + before;
    }
    __syncthreads();
    // per digit: exclusive scan over waves, then over digits
    if (tid < kRadix) {
        uint32_t run = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            uint32_t c = whist[w][tid];
            whist[w][tid] = run;
            run += c;
        }
        lbase[tid] = run;
    }
    __syncthreads();
    // inclusive Hillis-Steele scan of the 256 digit totals (every thread
    // reaches every barrier; threads >= 256 carry no data)
    for (int o = 1; o < kRadix; o <<= 1) {
        uint32_t u = (tid < kRadix && tid >= o) ? lbase[tid - o] : 0;
        __syncthreads();
        if (tid < kRadix)
            lbase[tid] += u;
        __syncthreads();
    }
    // lbase is now inclusive; exclusive base of digit d = lbase[d] - total(d)
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        uint32_t dg = digit_of(key[it], p);
        uint32_t excl = dg == 0 ? 0 : lbase[dg - 1];
        uint32_t pos = excl + whist[wid][dg] + rank[it];
        skey[pos] = key[it];
        sid[pos] = id[it];
    }
    __syncthreads();
    uint64_t *kout = (dst == 1 ? a.ka : a.kb) + (int64_t)t * a.n;
    uint32_t *iout = (dst == 1 ? a.ia : a.ib) + (int64_t)t * a.n;
    for (int q = tid; q < kSortTile; q += kSortThreads) {
        uint32_t idv = sid[q];
        if (idv == 0xffffffffu)
            continue;
        uint64_t k = skey[q];
        uint32_t dg = digit_of(k, p);
        uint32_t excl = dg == 0 ? 0 : lbase[dg - 1];
        uint32_t g = gbase[dg] + (q - excl);
        kout[g] = k;
        iout[g] = idv;
    }
}

// ---------------------------------------------------------- bucket offsets

struct HeadArgs {
    const uint64_t *sk; // sorted keys [L][n]
    int64_t n;
    int32_t L;
    int32_t ntiles;
    uint32_t *tile_cnt; // [L][ntiles] -> exclusive base
    uint64_t *ukeys;    // [L][n]
    uint32_t *offs;     // [L][n+1]
    int64_t *nuniq;     // [L]
};

__device__ __forceinline__ bool is_head(const uint64_t *k, int64_t i)
{
    return i == 0 || k[i] != k[i - 1];
}

__global__ __launch_bounds__(kHeadThreads) void head_count_kernel(HeadArgs a)
{
    const int t = blockIdx.y;
    const uint64_t *k = a.sk + (int64_t)t * a.n;
    int64_t base = (int64_t)blockIdx.x * kHeadTile;
    uint32_t c = 0;
    for (int it = 0; it < kHeadItems; ++it) {
        int64_t i = base + it * kHeadThreads + threadIdx.x;
        if (i < a.n)
            c += is_head(k, i);
    }
    c = wave_sum(c);
    __shared__ uint32_t s[kHeadThreads / kWave];
    if (lane_id() == 0)
        s[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kHeadThreads / kWave; ++w)
            tot += s[w];
        a.tile_cnt[(int64_t)t * a.ntiles + blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(1024) void head_scan_kernel(HeadArgs a)
{
    const int t = blockIdx.x;
    uint32_t *c = a.tile_cnt + (int64_t)t * a.ntiles;
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    // each thread scans a contiguous run of tiles
    int per = (a.ntiles + 1023) / 1024;
    int lo = tid * per, hi = lo + per < a.ntiles ? lo + per : a.ntiles;
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i)
        s += c[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        uint32_t v = c[i];
        c[i] = run;
        run += v;
    }
    if (tid == 1023) {
        a.nuniq[t] = part[1023];
        a.offs[(int64_t)t * (a.n + 1) + part[1023]] = (uint32_t)a.n;
    }
}

__global__ __launch_bounds__(kHeadThreads) void head_write_kernel(HeadArgs a)
{
    constexpr int kW = kHeadThreads / kWave;
    __shared__ uint32_t pre[kHeadItems][kW];
    const int t = blockIdx.y;
    const uint64_t *k = a.sk + (int64_t)t * a.n;
    const int64_t base = (int64_t)blockIdx.x * kHeadTile;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    // item it of thread tid is position base + it*256 + tid: tile order is (it, wave, lane)
    uint64_t bal[kHeadItems];
    uint64_t key[kHeadItems];
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it) {
        int64_t i = base + it * kHeadThreads + tid;
        bool h = false;
        key[it] = 0;
        if (i < a.n) {
            key[it] = k[i];
            h = i == 0 || key[it] != k[i - 1];
        }
        bal[it] = __ballot(h);
        if (lane == 0)
            pre[it][wid] = __popcll(bal[it]);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = a.tile_cnt[(int64_t)t * a.ntiles + blockIdx.x];
        for (int it = 0; it < kHeadItems; ++it)
            for (int w = 0; w < kW; ++w) {
                uint32_t c = pre[it][w];
                pre[it][w] = run;
                run += c;
            }
    }
    __syncthreads();
    uint64_t *uk = a.ukeys + (int64_t)t * a.n;
    uint32_t *of = a.offs + (int64_t)t * (a.n + 1);
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it) {
        if ((bal[it] >> lane) & 1ull) {
            uint32_t u = pre[it][wid] + __popcll(bal[it] & lt);
            uk[u] = key[it];
            of[u] = (uint32_t)(base + it * kHeadThreads + tid);
        }
    }
}

} // namespace lsh

// ========================================================================
// host side
// ========================================================================

struct lsh_index {
    int64_t n;
    int32_t L;
    int64_t id_base;
    uint32_t *sorted_ids;
    uint64_t *ukeys;
    uint32_t *offs;
    int64_t *nuniq;
};

namespace {

struct IndexLayout {
    size_t ids, ukeys, offs, nuniq, total;
};

IndexLayout index_layout(int64_t n, int32_t L)
{
    using lsh::align_up;
    IndexLayout l;
    l.ids = 0;
    l.ukeys = l.ids + align_up((size_t)L * n * 4, 256);
    l.offs = l.ukeys + align_up((size_t)L * n * 8, 256);
    l.nuniq = l.offs + align_up((size_t)L * (n + 1) * 4, 256);
    l.total = l.nuniq + align_up((size_t)L * 8, 256);
    return l;
}

struct WsLayout {
    size_t ka, kb, ib, ghist, plan, tile_hist, tile_cnt, total;
    int ntiles, nhtiles;
};

WsLayout ws_layout(int64_t n, int32_t L)
{
    using lsh::align_up;
    WsLayout w;
    w.ntiles = (int)((n + lsh::kSortTile - 1) / lsh::kSortTile);
    w.nhtiles = (int)((n + lsh::kHeadTile - 1) / lsh::kHeadTile);
    w.ka = 0;
    w.kb = w.ka + align_up((size_t)L * n * 8, 256);
    w.ib = w.kb + align_up((size_t)L * n * 8, 256);
    w.ghist = w.ib + align_up((size_t)L * n * 4, 256);
    w.plan = w.ghist + align_up((size_t)L * lsh::kPasses * lsh::kRadix * 4, 256);
    w.tile_hist = w.plan + align_up((size_t)L * lsh::kPasses * 4, 256);
    w.tile_cnt = w.tile_hist + align_up((size_t)L * w.ntiles * lsh::kRadix * 4, 256);
    w.total = w.tile_cnt + align_up((size_t)L * (w.nhtiles > 0 ? w.nhtiles : 1) * 4, 256);
    return w;
}

} // namespace

extern "C" size_t lsh_index_bytes(int64_t n, int32_t L)
{
    if (n < 0 || L < 1)
        return 0;
    return index_layout(n, L).total;
}

extern "C" size_t lsh_build_workspace_bytes(int64_t n, int32_t L)
{
    if (n < 0 || L < 1)
        return 0;
    return ws_layout(n, L).total;
}

extern "C" lsh_status lsh_build_index(const uint64_t *keys, int64_t key_ld, int64_t n, int32_t L,
                                      int64_t id_base, void *mem, size_t mem_bytes, void *ws,
                                      size_t ws_bytes, lsh_index **out, void *stream)
{
    using namespace lsh;
    if (!out)
        LSH_FAIL(LSH_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || L < 1 || id_base < 0)
        LSH_FAIL(LSH_EINVAL, "bad n=%lld L=%d id_base=%lld", (long long)n, L, (long long)id_base);
    if (key_ld == 0)
        key_ld = n;
    if (key_ld < n)
        LSH_FAIL(LSH_EINVAL, "key_ld %lld < n %lld", (long long)key_ld, (long long)n);
    if (id_base + n > 0xfffffffell)
        LSH_FAIL(LSH_ERANGE, "ids id_base + n = %lld exceed 2^32 - 2", (long long)(id_base + n));
    if (n > 0 && !keys)
        LSH_FAIL(LSH_EINVAL, "keys is NULL");
    IndexLayout il = index_layout(n, L);
    WsLayout wl = ws_layout(n, L);
    if (!mem || mem_bytes < il.total || ((uintptr_t)mem & 255))
        LSH_FAIL(LSH_ENOMEM, "index memory needs %zu bytes (256-aligned), got %zu", il.total,
                 mem_bytes);
    if (n > 0 && (!ws || ws_bytes < wl.total || ((uintptr_t)ws & 255)))
        LSH_FAIL(LSH_ENOMEM, "build workspace needs %zu bytes (256-aligned), got %zu", wl.total,
                 ws_bytes);

    unsigned char *mb = (unsigned char *)mem;
    lsh_index *idx = new lsh_index;
    idx->n = n;
    idx->L = L;
    idx->id_base = id_base;
    idx->sorted_ids = (uint32_t *)(mb + il.ids);
    idx->ukeys = (uint64_t *)(mb + il.ukeys);
    idx->offs = (uint32_t *)(mb + il.offs);
    idx->nuniq = (int64_t *)(mb + il.nuniq);

    hipStream_t s = (hipStream_t)stream;
    auto fail = [&](const char *what, hipError_t e) {
        delete idx;
        set_error("%s: %s", what, hip_msg(e));
        return LSH_EHIP;
    };
    if (n == 0) {
        hipError_t e = hipMemsetAsync(idx->nuniq, 0, (size_t)L * 8, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(idx->offs, 0, (size_t)L * 4, s); // offs[t][0] = 0 (n+1 = 1)
        if (e != hipSuccess)
            return fail("hipMemsetAsync", e);
        *out = idx;
        return LSH_OK;
    }

    unsigned char *wb = (unsigned char *)ws;
    SortArgs sa;
    sa.kin = keys;
    sa.key_ld = key_ld;
    sa.n = n;
    sa.L = L;
    sa.id_base = (uint32_t)id_base;
    sa.ka = (uint64_t *)(wb + wl.ka);
    sa.kb = (uint64_t *)(wb + wl.kb);
    sa.ia = idx->sorted_ids;
    sa.ib = (uint32_t *)(wb + wl.ib);
    sa.ghist = (uint32_t *)(wb + wl.ghist);
    sa.plan = (int32_t *)(wb + wl.plan);
    sa.tile_hist = (uint32_t *)(wb + wl.tile_hist);
    sa.ntiles = wl.ntiles;

    hipError_t e = hipMemsetAsync(sa.ghist, 0, (size_t)L * kPasses * kRadix * 4, s);
    if (e != hipSuccess)
        return fail("hipMemsetAsync", e);
    dim3 tiles(wl.ntiles, L);
    hipLaunchKernelGGL(sort_hist_kernel, tiles, dim3(kSortThreads), 0, s, sa);
    hipLaunchKernelGGL(sort_plan_kernel, dim3(L), dim3(kRadix), 0, s, sa);
    for (int p = 0; p < kPasses; ++p) {
        hipLaunchKernelGGL(sort_upsweep_kernel, tiles, dim3(kSortThreads), 0, s, sa, p);
        hipLaunchKernelGGL(sort_scan_kernel, dim3(L), dim3(kRadix), 0, s, sa, p);
        hipLaunchKernelGGL(sort_downsweep_kernel, tiles, dim3(kSortThreads), 0, s, sa, p);
    }
    HeadArgs ha;
    ha.sk = sa.ka;
    ha.n = n;
    ha.L = L;
    ha.ntiles = wl.nhtiles;
    ha.tile_cnt = (uint32_t *)(wb + wl.tile_cnt);
    ha.ukeys = idx->ukeys;
    ha.offs = idx->offs;
    ha.nuniq = idx->nuniq;
    dim3 htiles(wl.nhtiles, L);
    hipLaunchKernelGGL(head_count_kernel, htiles, dim3(kHeadThreads), 0, s, ha);
    hipLaunchKernelGGL(head_scan_kernel, dim3(L), dim3(1024), 0, s, ha);
    hipLaunchKernelGGL(head_write_kernel, htiles, dim3(kHeadThreads), 0, s, ha);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail("index kernels", e);
    *out = idx;
    return LSH_OK;
}

extern "C" lsh_status lsh_index_get_view(const lsh_index *idx, lsh_index_view *v)
{
    if (!idx || !v)
        LSH_FAIL(LSH_EINVAL, "NULL argument");
    v->n = idx->n;
    v->L = idx->L;
    v->id_base = idx->id_base;
    v->sorted_ids = idx->sorted_ids;
    v->ukeys = idx->ukeys;
    v->offs = idx->offs;
    v->nuniq = idx->nuniq;
    return LSH_OK;
}

extern "C" void lsh_index_free(lsh_index *idx) { delete idx; }
