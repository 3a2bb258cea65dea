// Index construction on gfx950 (Section 3.1: store every point in the
// bucket of its key, one table per group of K components).
//
// The index of a table is its (key, id) pairs in (key, id) order plus the
// run heads.  Keys are 64-bit digests (E2LSH) or K sign bits (SRP), so the
// order is built most-significant-digit first:
//   1. mask    - OR and AND of every key of a table: the bits that vary;
//                the same pass counts the top B key bits per tile, a guess
//                that holds when the top bit varies (digests), and tables
//                where it does not are counted again;
//   2. msd     - the top B varying bits (B grows with n, at most 10) form the
//                segment digit: per-tile digit counts, their scan (segment
//                starts, and the list of segments too large for step 3) and
//                a stable scatter of (key, id) into 2^B segments per table;
//   3. segment - one workgroup per segment of at most 4096 keys (256 threads
//                up to 2048 keys, else 512) sorts it in LDS: 16-bit index
//                arrays ranked by the segment's varying 8-bit chunks, least
//                significant first (only the top three when more vary, unless
//                an adjacent pair shows two distinct keys that agree on them);
//   4. big     - larger segments (heavy buckets, skewed digits): a sampled
//                pivot key splits each in parallel over tiles into less /
//                equal / greater parts; less and greater parts of at most
//                4096 keys are sorted like the segments of step 3; one
//                1024-thread workgroup per segment splits the rest
//                recursively (pivot or top varying byte): parts holding a
//                single key are copied, parts of at most 8192 keys are sorted
//                in LDS;
//   5. heads   - one pass over the sorted keys: each tile counts its run
//                heads, takes the count before it from its predecessors (a
//                decoupled look-back) and writes the distinct keys and
//                bucket start offsets.
// Every scatter ranks keys stably (one ballot per digit bit gives the lanes
// of a wave that share a digit), so ids stay ascending inside a bucket.

#include "lsh_internal.h"

#include <mutex>

namespace lsh {

constexpr int kThreads = 1024;             // scatter / big-segment workgroups
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;   // 8192 keys per scatter tile
constexpr int kWaves = kThreads / kWave;
constexpr int kMsdBitsMax = 10;
constexpr int kMsdRadixMax = 1 << kMsdBitsMax;
constexpr int kRadix = 256;                // 8-bit digits below the segment digit
// keys per thread of the segment scatter (a multiple of kItems: it may rank
// several counted tiles at once; one measured fastest)
constexpr int kMsdItems = kItems;
constexpr int kMsdTile = kThreads * kMsdItems;
// Workgroups of a launch are dealt to the 8 XCDs (each with its own L2) in
// turn: workgroup i runs on XCD i % 8.
constexpr int kXcds = 8;
// workgroups per table of the digit recount (tables whose top key bit does
// not vary; for digests every workgroup exits at once)
constexpr int kMsdUpGrid = 64;
constexpr int kSegThreads = 512;
constexpr int kSegSmall = kSegThreads * kItems; // 4096: segments sorted by kSegThreads
// segments of at most 2048 keys take a 256-thread workgroup with half the
// LDS, so that four of them share a CU (two of the 4096-key ones fit)
constexpr int kSegThreadsS = 256;
constexpr int kSegTiny = kSegThreadsS * kItems; // 2048
constexpr int kSegLarge = kThreads * kItems;    // 8192: parts sorted inside the big path
constexpr int kChunks = 8;     // 8-bit chunks of a key (a segment's varying bits lie below its digit)
constexpr int kFastChunks = 3; // chunks sorted before the adjacent-pair check
constexpr int kStackMax = 16 * kRadix; // pending parts of one big segment

constexpr int kHeadThreads = 1024;
constexpr int kHeadItems = 16;
constexpr int kHeadTile = kHeadThreads * kHeadItems;

struct BuildArgs {
    const uint64_t *kin; // input keys [L][key_ld]
    int64_t key_ld;
    int64_t n;
    int32_t L;
    uint32_t id_base;
    int32_t ntiles;       // scatter tiles per table
    int32_t msd_bits;     // B
    uint64_t *tor, *tand; // [L] OR / AND of the table's keys
    uint32_t *tile_hist;  // [L][ntiles][2^B] digit counts -> global offsets
    uint32_t *ghist;      // [L][2^B] segment sizes
    uint32_t *seg_start;  // [L][2^B]
    uint64_t *ka, *kb;    // key buffers [L][n]; kb ends sorted
    uint32_t *ia, *ids;   // id buffers [L][n] (ids = the index's sorted_ids)
    uint32_t *blist;      // [L * 2^B][8]: table, segment, first tile, tiles, pivot?, #<, #=,
                          // parts handed to the LDS sorts (bit 0: <, bit 1: >)
    uint64_t *bpivot;     // [L * 2^B]: pivot key of a big segment
    uint32_t *btile;      // [maxbt][2]: big segment, tile within it
    uint32_t *tcls;       // [maxbt][4]: per tile: class counts, then class offsets
    uint32_t *bcount;     // [kCounts]: big segments, stack overflows (0 unless a bound fails),
                          // big tiles, parts of 1..2048 keys, parts of 2049..4096 keys
    uint32_t *plist;      // [2][2 * L * 2^B][3]: those parts (table, start, size)
    uint32_t *stack;      // [grid][kStackMax][3]: start, size, buffer
    uint64_t *hstat;      // [nhstat] run-head status words and counters, zeroed at the start
    int64_t nhstat;
};

constexpr int kBig = 8;    // words per big-segment entry
constexpr int kCounts = 8; // words of BuildArgs::bcount

__device__ __forceinline__ int top_shift(uint64_t vm, int bits)
{
    if (!vm)
        return 0;
    const int hb = 63 - __clzll((long long)vm);
    return hb >= bits ? hb - bits + 1 : 0;
}

// The segment digit of a table whose varying key bits (OR & ~AND over its
// keys) number 1..B: those bits, compacted in order (bit i of the digit is
// the i-th lowest varying bit).  The digit then orders the keys exactly as
// the keys do (they agree on every other bit) and separates all distinct
// keys, so each segment is one run of equal keys.  cmask is uniform.
__device__ __forceinline__ uint32_t compact_bits(uint64_t k, uint64_t cmask)
{
    uint32_t d = 0;
    for (int i = 0; cmask; ++i) {
        const int b = __builtin_ctzll(cmask);
        d |= (uint32_t)((k >> b) & 1u) << i;
        cmask &= cmask - 1;
    }
    return d;
}

// The varying bits of table t when they take the compacted digit (1..B of
// them), else 0 (the digit is then the top B bits from the highest varying one).
__device__ __forceinline__ uint64_t compact_mask(uint64_t tor, uint64_t tand, int bits)
{
    const uint64_t vm = tor & ~tand;
    return vm && __popcll(vm) <= bits ? vm : 0ull;
}

// Table t is in (key, id) order once scattered when its segment digit holds
// every varying key bit (at most B of them: the compacted digit) or no bit
// varies: each segment is then one run of equal keys, in id order (the
// scatter is stable).  Such a table is scattered straight to its final
// buffers and skips the segment sorts and the big-segment path.
__device__ __forceinline__ bool table_complete(const uint64_t *tor, const uint64_t *tand, int t,
                                               int bits)
{
    return __popcll(tor[t] & ~tand[t]) <= bits;
}

__device__ __forceinline__ bool chunk_varies(uint64_t vm, int p)
{
    return ((vm >> (8 * p)) & 255u) != 0;
}

// Inclusive sum over the lanes of a wave: shifts within rows of 16 lanes,
// then the last lane of a row broadcast to the rows above it.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true); // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true); // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true); // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true); // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); // row_bcast:31
    return x;
}

// Exclusive scan of v over threads [0, R) of the block (R <= blockDim.x,
// at most 64 waves); every thread calls it.  wsum: LDS scratch of R / 64
// words.  Within a wave by DPP; across waves every wave sums the totals of
// the waves before it the same way.
__device__ __forceinline__ uint32_t scan_excl(uint32_t v, int R, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t v0 = tid < R ? v : 0u;
    const uint32_t x = wave_incl_scan(v0);
    if (tid < R && (lane == kWave - 1 || tid == R - 1))
        wsum[w] = x;
    __syncthreads();
    const uint32_t y = lane < w && lane * kWave < R ? wsum[lane] : 0u;
    const uint32_t pre = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(y), kWave - 1);
    __syncthreads();
    return pre + x - v0;
}

// ------------------------------------------------------------------ init

__global__ __launch_bounds__(256) void build_init_kernel(BuildArgs a)
{
    const int64_t nseg = (int64_t)a.L << a.msd_bits;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nseg;
         i += (int64_t)gridDim.x * blockDim.x) {
        a.ghist[i] = 0;
        if (i < a.L) {
            a.tor[i] = 0;
            a.tand[i] = ~0ull;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nhstat;
         i += (int64_t)gridDim.x * blockDim.x)
        a.hstat[i] = 0;
    // the counters do not depend on nseg (which can be as small as 2)
    if (blockIdx.x == 0 && threadIdx.x < kCounts)
        a.bcount[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ mask

// OR / AND of a 32-bit value over the wave, the same DPP steps as
// wave_incl_scan (lanes without a source contribute the identity); the
// last lane's result is the wave's, read back as a uniform value.
template <bool OR>
__device__ __forceinline__ uint32_t wave_bits32(uint32_t x)
{
    const int id = OR ? 0 : -1;
    auto f = [](uint32_t u, int y) { return OR ? u | (uint32_t)y : u & (uint32_t)y; };
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x111, 0xf, 0xf, false)); // row_shr:1
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x112, 0xf, 0xf, false)); // row_shr:2
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x114, 0xf, 0xf, false)); // row_shr:4
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x118, 0xf, 0xf, false)); // row_shr:8
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x142, 0xa, 0xf, false)); // row_bcast:15
    x = f(x, __builtin_amdgcn_update_dpp(id, (int)x, 0x143, 0xc, 0xf, false)); // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    return ((uint64_t)wave_bits32<true>((uint32_t)(v >> 32)) << 32) |
           wave_bits32<true>((uint32_t)v);
}

__device__ __forceinline__ uint64_t wave_and64(uint64_t v)
{
    return ((uint64_t)wave_bits32<false>((uint32_t)(v >> 32)) << 32) |
           wave_bits32<false>((uint32_t)v);
}

// f(i, keys[i]) for every i < cnt, split over the block with eight loads in
// flight per thread (a single workgroup streams a whole part this way).
// Loads past the end read the last key instead (and are ignored), so that
// no load sits in a branch: the compiler then issues them together rather
// than waiting for each.
template <typename F>
__device__ __forceinline__ void for_each_key(const uint64_t *keys, uint32_t cnt, F f)
{
    const uint32_t nt = blockDim.x, tid = threadIdx.x;
    for (uint32_t base = 0; base < cnt; base += 8 * nt) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = base + u * nt + tid;
            v[u] = keys[min(i, cnt - 1u)]; // clamped: no branch around the load
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = base + u * nt + tid;
            if (i < cnt)
                f(i, v[u]);
        }
    }
}

// OR / AND of keys[0, cnt) over the block (every thread calls; all get it).
__device__ __forceinline__ void block_or_and(const uint64_t *keys, int64_t cnt, uint64_t *so,
                                             uint64_t *sa, uint64_t &vo, uint64_t &va)
{
    vo = 0;
    va = ~0ull;
    for_each_key(keys, (uint32_t)cnt, [&](uint32_t, uint64_t v) {
        vo |= v;
        va &= v;
    });
    vo = wave_or64(vo);
    va = wave_and64(va);
    const int nw = blockDim.x / kWave, wid = threadIdx.x / kWave;
    if (lane_id() == 0) {
        so[wid] = vo;
        sa[wid] = va;
    }
    __syncthreads();
    vo = 0;
    va = ~0ull;
    for (int w = 0; w < nw; ++w) {
        vo |= so[w];
        va &= sa[w];
    }
    __syncthreads();
}

// h[d] += 1 for every active lane: one add of the lane count when all
// active lanes hold the same digit (tables with few distinct keys would
// otherwise queue 64 adds on one LDS address), else one add per lane.
__device__ __forceinline__ void hist_add(uint32_t *h, uint32_t d)
{
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
    const uint64_t act = __ballot(1);
    if (__ballot(d == d0) == act) {
        if (lane_id() == __builtin_ctzll(act))
            atomicAdd(&h[d0], (uint32_t)__popcll(act));
    } else {
        atomicAdd(&h[d], 1u);
    }
}

// OR / AND of every key of a table and, guessing that the table's top key
// bit varies (true of 64-bit digests), the tile's counts of the segment
// digit key >> (64 - B).  msd_up recounts the tables where the
// guess fails (short SRP keys).
__global__ __launch_bounds__(kThreads) void mask_up_kernel(BuildArgs a)
{
    const int t = blockIdx.y;
    const int R = 1 << a.msd_bits;
    const int shift = 64 - a.msd_bits;
    __shared__ uint32_t h[kMsdRadixMax];
    __shared__ uint64_t so[kWaves], sa[kWaves];
    for (int i = threadIdx.x; i < R; i += kThreads)
        h[i] = 0;
    __syncthreads();
    const uint64_t *k = a.kin + (int64_t)t * a.key_ld;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t v[kItems];
    const bool full = base + kTile <= a.n;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = base + it * kThreads + threadIdx.x;
        v[it] = k[full ? i : min(i, a.n - 1)]; // clamped: no branch around the load
    }
    uint64_t vo = 0, va = ~0ull;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = base + it * kThreads + threadIdx.x;
        const uint64_t m = full || i < a.n ? ~0ull : 0ull;
        vo |= v[it] & m;
        va &= v[it] | ~m;
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = base + it * kThreads + threadIdx.x;
        if (full || i < a.n)
            hist_add(h, (uint32_t)(v[it] >> shift));
    }
    vo = wave_or64(vo);
    va = wave_and64(va);
    const int wid = threadIdx.x / kWave;
    if (lane_id() == 0) {
        so[wid] = vo;
        sa[wid] = va;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            so[0] |= so[w];
            sa[0] &= sa[w];
        }
        atomicOr((unsigned long long *)&a.tor[t], (unsigned long long)so[0]);
        atomicAnd((unsigned long long *)&a.tand[t], (unsigned long long)sa[0]);
    }
    uint32_t *th = a.tile_hist + ((int64_t)t * a.ntiles + blockIdx.x) * R;
    for (int i = threadIdx.x; i < R; i += kThreads)
        th[i] = h[i];
}

// ------------------------------------------------------------ segment digit

__device__ __forceinline__ bool guess_holds(const BuildArgs &a, int t)
{
    return !compact_mask(a.tor[t], a.tand[t], a.msd_bits) &&
           top_shift(a.tor[t] & ~a.tand[t], a.msd_bits) == 64 - a.msd_bits;
}

// Tables whose top key bit does not vary: count the segment digit (the top
// B varying bits) per tile.
__global__ __launch_bounds__(kThreads) void msd_up_kernel(BuildArgs a)
{
    const int t = blockIdx.y;
    if (guess_holds(a, t))
        return;
    const int R = 1 << a.msd_bits;
    __shared__ uint32_t h[kMsdRadixMax];
    const int shift = top_shift(a.tor[t] & ~a.tand[t], a.msd_bits);
    const uint64_t cmask = compact_mask(a.tor[t], a.tand[t], a.msd_bits);
    const uint64_t *k = a.kin + (int64_t)t * a.key_ld;
    // workgroups take the table's tiles in turn (the grid is capped: for
    // digest keys every workgroup exits at once)
    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        for (int i = threadIdx.x; i < R; i += blockDim.x)
            h[i] = 0;
        __syncthreads();
        const int64_t base = (int64_t)tile * kTile;
        uint64_t v[kItems];
#pragma unroll
        for (int it = 0; it < kItems; ++it)
            v[it] = k[min(base + it * kThreads + threadIdx.x, a.n - 1)];
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const int64_t i = base + it * kThreads + threadIdx.x;
            if (i < a.n)
                hist_add(h, cmask ? compact_bits(v[it], cmask)
                                  : (uint32_t)(v[it] >> shift) & (uint32_t)(R - 1));
        }
        __syncthreads();
        uint32_t *th = a.tile_hist + ((int64_t)t * a.ntiles + tile) * R;
        for (int i = threadIdx.x; i < R; i += blockDim.x)
            th[i] = h[i];
        __syncthreads();
    }
}

// ghist[t][d] <- size of segment d (the sum of the tile counts);
// tile_hist[t][tile][d] <- global start of the tile's run of digit d;
// seg_start[t][d] <- start of segment d.  Segments larger than an LDS sort
// join the big list (blist, btile) in a range the table reserves with one
// atomic add per list; the order of the tables in the lists does not matter
// (every big segment is sorted on its own).
__global__ __launch_bounds__(kMsdRadixMax) void msd_scan_kernel(BuildArgs a)
{
    const int t = blockIdx.x;
    const int R = 1 << a.msd_bits;
    // the kMsdRadixMax threads form G groups of R, one thread per digit in
    // each; group g takes tiles [g * ntiles / G, (g + 1) * ntiles / G)
    const int G = kMsdRadixMax / R;
    const int d = threadIdx.x & (R - 1), g = threadIdx.x / R;
    const int tlo = (int)((int64_t)a.ntiles * g / G), thi = (int)((int64_t)a.ntiles * (g + 1) / G);
    __shared__ uint32_t wsum[kMsdRadixMax / kWave];
    __shared__ uint32_t part[kMsdRadixMax];
    __shared__ uint32_t bres[2];
    uint32_t *th = a.tile_hist + (int64_t)t * a.ntiles * R + d;
    uint32_t c = 0;
    {
        int tile = tlo;
        for (; tile + 8 <= thi; tile += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = th[(int64_t)(tile + u) * R];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                c += v[u];
        }
        for (; tile < thi; ++tile)
            c += th[(int64_t)tile * R];
    }
    part[threadIdx.x] = c;
    __syncthreads();
    // the digit's total, and the count of its keys in the earlier groups' tiles
    uint32_t total = 0, before = 0;
    for (int q = 0; q < G; ++q) {
        const uint32_t v = part[q * R + d];
        total += v;
        before += q < g ? v : 0u;
    }
    // group 0 (threads below R) holds the digits for the scans
    const bool lead = g == 0;
    c = lead ? total : 0u;
    if (lead)
        a.ghist[(t << a.msd_bits) + d] = c;
    uint32_t run = scan_excl(c, R, wsum);
    const bool big = lead && c > (uint32_t)kSegSmall && !table_complete(a.tor, a.tand, t, a.msd_bits);
    const uint32_t ntl = big ? (c + kTile - 1) / kTile : 0u;
    const uint32_t bi = scan_excl(big ? 1u : 0u, R, wsum);
    const uint32_t ti = scan_excl(ntl, R, wsum);
    if (threadIdx.x == R - 1) {
        bres[0] = atomicAdd(&a.bcount[0], bi + (big ? 1u : 0u));
        bres[1] = atomicAdd(&a.bcount[2], ti + ntl);
    }
    if (lead)
        part[d] = run; // the digit's segment start, for the other groups
    __syncthreads();
    if (big) {
        const uint32_t b0 = bres[0] + bi, t0 = bres[1] + ti;
        uint32_t *b = a.blist + kBig * b0;
        b[0] = (uint32_t)t;
        b[1] = (uint32_t)d;
        b[2] = t0;
        b[3] = ntl;
        b[4] = 0;
        b[7] = 0;
        for (uint32_t k = 0; k < ntl; ++k) {
            a.btile[2 * (t0 + k)] = b0;
            a.btile[2 * (t0 + k) + 1] = k;
        }
    }
    if (lead)
        a.seg_start[(t << a.msd_bits) + d] = run;
    run = part[d] + before;
    int tile = tlo;
    for (; tile + 8 <= thi; tile += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = th[(int64_t)(tile + u) * R];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            th[(int64_t)(tile + u) * R] = run;
            run += v[u];
        }
    }
    for (; tile < thi; ++tile) {
        const uint32_t v = th[(int64_t)tile * R];
        th[(int64_t)tile * R] = run;
        run += v;
    }
}

// ------------------------------------------------------- stable tile scatter

// The lanes of the wave whose NB-bit digit equals this lane's digit dg (bits
// of dg at NB and above must be zero): one ballot per bit, each kept where
// this lane's bit agrees.  With m the bit sign-extended (0 or all ones), a
// half of the mask is updated as half & ~(ballot half ^ m): one three-input
// bit operation (truth table 0x90 over (half, ballot half, m)).  Four bits
// at a time: their four compares first, then two wait states before a
// compare result is read by a vector instruction.
template <int B0>
__device__ __forceinline__ void match_4bits(uint32_t dg, uint32_t &lo, uint32_t &hi)
{
    uint32_t m0, m1, m2, m3;
    uint64_t s0, s1, s2, s3;
    asm volatile("v_bfe_i32 %[m0], %[dg], %[b0], 1\n\t"
                 "v_bfe_i32 %[m1], %[dg], %[b1], 1\n\t"
                 "v_bfe_i32 %[m2], %[dg], %[b2], 1\n\t"
                 "v_bfe_i32 %[m3], %[dg], %[b3], 1\n\t"
                 "v_cmp_ne_u32_e64 %[s0], 0, %[m0]\n\t"
                 "v_cmp_ne_u32_e64 %[s1], 0, %[m1]\n\t"
                 "v_cmp_ne_u32_e64 %[s2], 0, %[m2]\n\t"
                 "v_cmp_ne_u32_e64 %[s3], 0, %[m3]"
                 : [m0] "=&v"(m0), [m1] "=&v"(m1), [m2] "=&v"(m2), [m3] "=&v"(m3),
                   [s0] "=&s"(s0), [s1] "=&s"(s1), [s2] "=&s"(s2), [s3] "=&s"(s3)
                 : [dg] "v"(dg), [b0] "n"(B0), [b1] "n"(B0 + 1), [b2] "n"(B0 + 2),
                   [b3] "n"(B0 + 3));
    asm volatile("s_nop 1\n\t"
                 "v_bitop3_b32 %[lo], %[lo], %[a0], %[m0] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[hi], %[hi], %[c0], %[m0] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[lo], %[lo], %[a1], %[m1] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[hi], %[hi], %[c1], %[m1] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[lo], %[lo], %[a2], %[m2] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[hi], %[hi], %[c2], %[m2] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[lo], %[lo], %[a3], %[m3] bitop3:0x90\n\t"
                 "v_bitop3_b32 %[hi], %[hi], %[c3], %[m3] bitop3:0x90"
                 : [lo] "+v"(lo), [hi] "+v"(hi)
                 : [m0] "v"(m0), [m1] "v"(m1), [m2] "v"(m2), [m3] "v"(m3),
                   [a0] "s"((uint32_t)s0), [c0] "s"((uint32_t)(s0 >> 32)),
                   [a1] "s"((uint32_t)s1), [c1] "s"((uint32_t)(s1 >> 32)),
                   [a2] "s"((uint32_t)s2), [c2] "s"((uint32_t)(s2 >> 32)),
                   [a3] "s"((uint32_t)s3), [c3] "s"((uint32_t)(s3 >> 32)));
}

template <int NB>
__device__ __forceinline__ void match_digit(uint32_t dg, uint32_t &lo, uint32_t &hi)
{
    static_assert(NB >= 8 && NB <= 10, "digit widths used here");
    lo = ~0u;
    hi = ~0u;
    match_4bits<0>(dg, lo, hi);
    match_4bits<4>(dg, lo, hi);
    if constexpr (NB > 8) {
        // the bits past 8 in C: the compiler fuses them the same way
#pragma unroll
        for (int b = 8; b < NB; ++b) {
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)dg, b, 1);
            const uint64_t bal = __ballot(m != 0u);
            lo &= ~((uint32_t)bal ^ m);
            hi &= ~((uint32_t)(bal >> 32) ^ m);
        }
    }
}

// Lanes below this one in a 64-lane mask given as two halves.
__device__ __forceinline__ uint32_t count_below(uint32_t lo, uint32_t hi)
{
    return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

template <int RMAX, int IT = kItems> struct ScatterLds {
    // per-wave digit counts (a wave ranks IT * 64 <= 1024 keys), then
    // per-wave prefixes inside each digit (below the tile size)
    alignas(4) uint16_t whist[kWaves][RMAX];
    uint32_t lbase[RMAX];   // first sorted position of each digit in the tile
    uint32_t goff[RMAX];    // the caller's output offset of each digit
    uint32_t wsum[RMAX / kWave];
    uint32_t count[RMAX];   // the tile's count of each digit (for the caller)
    uint16_t perm[kThreads * IT]; // tile position of the key at each sorted position
    static_assert(IT * kWave <= 1024 && kThreads * IT <= 65536, "16-bit counts");
};

// Stable scatter of one tile of 1024 * IT keys (1024 threads): keys (and
// ids, or id0 + i when ids is NULL) [0, cnt) go to kout/iout at
// goff[digit] + (rank among the tile's keys of that digit), digit = (key >>
// shift) & (2^bits - 1).  Wave w ranks rows w*IT .. w*IT+IT-1 of 64 keys;
// the lanes holding the same digit come
// from one ballot per digit bit.  Only the order is kept in LDS (the tile
// position of each sorted position); the keys are read again (from cache)
// in that order and written as contiguous digit runs, so two tiles fit in
// a CU's LDS.  On return s.count[d] holds the tile's count of digit d.
template <int RMAX, int IT = kItems, int RLOG = __builtin_ctz(RMAX)>
__device__ __forceinline__ void scatter_tile(ScatterLds<RMAX, IT> &s, const uint64_t *kin,
                                             const uint32_t *iin, uint32_t id0, int cnt,
                                             int shift, int bits, const uint32_t *goff,
                                             uint64_t *kout, uint32_t *iout,
                                             uint64_t cmask = 0)
{
    const int R = 1 << bits;
    const uint32_t dmask = (uint32_t)R - 1u;
    const int tid = threadIdx.x, wid = tid / kWave, lane = lane_id();
    for (int i = tid; i < kWaves * RMAX / 2; i += kThreads)
        ((uint32_t *)&s.whist[0][0])[i] = 0u;
    for (int i = tid; i < R; i += kThreads)
        s.goff[i] = goff[i];
    __syncthreads();

    const int wbase = wid * (kWave * IT);
    // dg[it]: the digit, then the digit | rank << 16 (rank < IT * 64).
    // Positions past the end rank after every real key of the last digit
    // (they come last in the ranking order) and are never written.  When
    // the digit lies in one 32-bit half of the key (always for the segment
    // digit of 64-bit digests) only that half is read.
    uint32_t dg[IT];
    const uint32_t *kw = (const uint32_t *)kin;
    if (cmask) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = wbase + it * kWave + lane;
            const uint64_t k = kin[min(i, cnt - 1)];
            dg[it] = compact_bits(k, cmask) | (i < cnt ? 0u : dmask);
        }
    } else if (shift >= 32 || shift + bits <= 32) {
        const int h = shift >= 32 ? 1 : 0, sh = shift - 32 * h;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = wbase + it * kWave + lane;
            // clamped load, and no select between it and a constant: the
            // load then stays out of any branch and all are issued together
            const uint32_t w = kw[2 * min(i, cnt - 1) + h];
            dg[it] = ((w >> sh) & dmask) | (i < cnt ? 0u : dmask);
        }
    } else {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = wbase + it * kWave + lane;
            const uint64_t k = kin[min(i, cnt - 1)];
            dg[it] = ((uint32_t)(k >> shift) & dmask) | (i < cnt ? 0u : dmask);
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        // digit bits at `bits` and above are zero: their ballots keep every lane
        uint32_t plo, phi;
        match_digit<RLOG>(dg[it], plo, phi);
        const uint32_t before = count_below(plo, phi);
        const uint32_t npeer = __popc(plo) + __popc(phi);
        // the first lane of each digit adds the row's count to its 16-bit
        // counter (half of a 32-bit word; a wave counts at most 1024 keys,
        // so no carry crosses into the other half); every lane then reads
        // the count including this row.  A wave's LDS operations run in
        // order.
        if (before == 0)
            __hip_atomic_fetch_add((uint32_t *)__builtin_assume_aligned(
                                       &s.whist[wid][dg[it] & ~1u], 4),
                                   npeer << (16u * (dg[it] & 1u)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        dg[it] |= ((uint32_t)s.whist[wid][dg[it]] + before - npeer) << 16;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive scan over waves; then over digits
    uint32_t tot = 0;
    if (tid < R) {
        // eight waves at a time (register budget)
#pragma unroll
        for (int w0 = 0; w0 < kWaves; w0 += 8) {
            uint32_t c[8];
#pragma unroll
            for (int w = 0; w < 8; ++w)
                c[w] = s.whist[w0 + w][tid];
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                s.whist[w0 + w][tid] = (uint16_t)tot; // prefix within the tile
                tot += c[w];
            }
        }
    }
    const uint32_t excl = scan_excl(tot, R, s.wsum);
    if (tid < R)
        s.lbase[tid] = excl;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = wbase + it * kWave + lane;
        const uint32_t d = dg[it] & 0xffffu;
        if (i < cnt)
            s.perm[s.lbase[d] + s.whist[wid][d] + (dg[it] >> 16)] = (uint16_t)i;
    }
    __syncthreads();
    // The real keys hold sorted positions [0, cnt): padding ranks last.
    // All of a thread's positions at once (clamped reads, no branch before
    // the stores), so that the reads of the keys overlap.
    {
        uint32_t pi[IT], iv[IT];
        uint64_t kv[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u)
            pi[u] = s.perm[min(u * kThreads + tid, cnt - 1)];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            kv[u] = kin[pi[u]];
            iv[u] = iin ? iin[pi[u]] : id0 + pi[u];
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int q = u * kThreads + tid;
            if (q < cnt) {
                const uint32_t d = cmask ? compact_bits(kv[u], cmask)
                                         : (uint32_t)(kv[u] >> shift) & dmask;
                const uint32_t g = s.goff[d] + ((uint32_t)q - s.lbase[d]);
                kout[g] = kv[u];
                iout[g] = iv[u];
            }
        }
    }
    // tile digit counts for the caller (lbase is exclusive, so count = next - this)
    if (tid < R) {
        // the last digit also holds the padding, which ranks after its keys
        const uint32_t nxt = tid + 1 < R ? s.lbase[tid + 1] : (uint32_t)cnt;
        s.count[tid] = nxt - s.lbase[tid];
    }
    __syncthreads();
}

// two workgroups per CU: at most 64 VGPRs (eight waves per SIMD)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void
msd_scatter_kernel(BuildArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    ScatterLds<kMsdRadixMax, kMsdItems> &s = *(ScatterLds<kMsdRadixMax, kMsdItems> *)lds;
    // Each XCD takes a contiguous range of the (table, tile) pairs in table
    // order: consecutive tiles of a table write adjacent runs of every
    // segment, and on one XCD the cache lines those runs share are completed
    // in its L2 rather than written back in parts by two.
    const int64_t ntm = (a.n + kMsdTile - 1) / kMsdTile;
    const int64_t npair = ntm * a.L;
    const int64_t chunk = (npair + kXcds - 1) / kXcds;
    const int64_t pair = (int64_t)(blockIdx.x % kXcds) * chunk + (int64_t)(blockIdx.x / kXcds);
    if (pair >= npair)
        return;
    const int t = (int)(pair / ntm);
    const int64_t tile = pair % ntm;
    const int R = 1 << a.msd_bits;
    const int shift = top_shift(a.tor[t] & ~a.tand[t], a.msd_bits);
    const uint64_t cmask = compact_mask(a.tor[t], a.tand[t], a.msd_bits);
    // kMsdTile / kTile counted tiles at once: their run of a digit starts
    // where the first tile's run starts and covers the others
    const int64_t base = (int64_t)tile * kMsdTile;
    const int cnt = (int)min((int64_t)kMsdTile, a.n - base);
    const uint32_t *goff =
        a.tile_hist + ((int64_t)t * a.ntiles + (int64_t)tile * (kMsdTile / kTile)) * R;
    // one ballot per digit bit that can be set (B at most 8, 9 or 10)
    const uint64_t *kin = a.kin + (int64_t)t * a.key_ld + base;
    const bool done = table_complete(a.tor, a.tand, t, a.msd_bits);
    uint64_t *ko = (done ? a.kb : a.ka) + (int64_t)t * a.n;
    uint32_t *io = (done ? a.ids : a.ia) + (int64_t)t * a.n;
    const uint32_t id0 = a.id_base + (uint32_t)base;
    if (a.msd_bits <= 8)
        scatter_tile<kMsdRadixMax, kMsdItems, 8>(s, kin, nullptr, id0, cnt, shift, a.msd_bits,
                                                 goff, ko, io, cmask);
    else if (a.msd_bits == 9)
        scatter_tile<kMsdRadixMax, kMsdItems, 9>(s, kin, nullptr, id0, cnt, shift, a.msd_bits,
                                                 goff, ko, io, cmask);
    else
        scatter_tile<kMsdRadixMax, kMsdItems, 10>(s, kin, nullptr, id0, cnt, shift, a.msd_bits,
                                                  goff, ko, io, cmask);
}

// ------------------------------------------------- segment sort in LDS

template <int NT> struct SegLds {
    static constexpr int S = NT * kItems;
    static constexpr int NW = NT / kWave;
    uint64_t key[S];
    uint32_t id[S];
    uint16_t ix[2][S];
    // per-wave digit counts (a wave ranks at most 512 keys), two buffers
    // used by alternate passes: a pass clears the other one for the next
    alignas(8) uint16_t whist[2][NW][kRadix];
    alignas(8) uint16_t base[NW][kRadix]; // per wave: its first position of each digit
    uint64_t so[NW], sa[NW];
    int flag;
};

// One stable counting pass of the index array src -> dst by chunk p of the
// keys, with digit counts in s.whist[buf] (zero on entry; s.whist[buf ^ 1]
// is zero on return).  Wave w ranks positions [w*rows*64, (w+1)*rows*64),
// row by row.  Two workgroup barriers: after the counts, after the scatter.
template <int NT>
__device__ __forceinline__ void seg_rank_pass(SegLds<NT> &s, const uint16_t *src, uint16_t *dst,
                                              int cnt, int rows, int p, int buf)
{
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, wid = tid / kWave, lane = lane_id();
    uint16_t (*wh)[kRadix] = s.whist[buf];
    // The other buffer's last readers (the previous pass's digit scan)
    // finished before the barrier that ended that pass; its next writers
    // (the next pass's ranking) start after this pass's last barrier.
    {
        uint32_t *z = (uint32_t *)s.whist[buf ^ 1][wid];
        z[lane] = 0u;
        z[lane + kWave] = 0u;
    }
    uint32_t ixs[kItems], dgs[kItems], rank[kItems];
    const int wbase = wid * rows * kWave;
    // All of this wave's indices, then all of their digits (byte p of the
    // key, read as a byte), with no branch between the loads so that their
    // latencies overlap.  j < NW * rows * 64 <= NT * kItems for every item,
    // also for the items at and past `rows` (which are loaded and ignored).
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int j = wbase + it * kWave + lane;
        const uint32_t ix = src[j];
        ixs[it] = j < cnt ? ix : 0u;
    }
    const uint8_t *kbytes = (const uint8_t *)s.key + p;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int j = wbase + it * kWave + lane;
        // positions past the end take digit 255 and rank after every real
        // key (they come last in the ranking order); never stored
        const uint32_t dg = kbytes[8 * ixs[it]];
        dgs[it] = j < cnt ? dg : 255u;
    }
    // Row by row, the first lane of each digit adds the row's count of it to
    // the digit's 16-bit counter (half of a 32-bit word; at most 512, so no
    // carry crosses into the other half); every lane then reads the count
    // including this row (rank = that count + lanes of the digit below it -
    // lanes of the digit in the row).  A wave's LDS operations run in order,
    // so no wait is needed between rows; the reads are made for every item
    // (past `rows` too, and ignored) so that none sits in a branch and they
    // complete together.
    int adj[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        adj[it] = 0;
        if (it < rows) {
            uint32_t plo, phi;
            match_digit<8>(dgs[it], plo, phi);
            const uint32_t before = count_below(plo, phi);
            const uint32_t npeer = __popc(plo) + __popc(phi);
            if (before == 0)
                __hip_atomic_fetch_add(
                    (uint32_t *)__builtin_assume_aligned(&wh[wid][dgs[it] & ~1u], 4),
                    npeer << (16u * (dgs[it] & 1u)), __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_WAVEFRONT);
            adj[it] = (int)before - (int)npeer;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        rank[it] = wh[wid][dgs[it]];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it)
        rank[it] += (uint32_t)adj[it];
    __syncthreads();
    // Every wave scans the 256 digit totals itself (lane l: digits 4l ..
    // 4l+3) and writes its own first position of each digit: digit start +
    // the digit's count in the waves before it.  Only this wave reads its
    // row of s.base back, so no barrier is needed before the scatter.
    {
        uint32_t c[4] = {0u, 0u, 0u, 0u}, pre[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint64_t v = *(const uint64_t *)&wh[w][4 * lane];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t x = (uint32_t)(v >> (16 * k)) & 0xffffu;
                c[k] += x;
                pre[k] += w < wid ? x : 0u;
            }
        }
        const uint32_t tot = c[0] + c[1] + c[2] + c[3];
        uint32_t e = wave_incl_scan(tot) - tot;
        uint64_t out = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            out |= (uint64_t)(e + pre[k]) << (16 * k);
            e += c[k];
        }
        *(uint64_t *)&s.base[wid][4 * lane] = out;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        if (it < rows) {
            const int j = wbase + it * kWave + lane;
            if (j < cnt)
                dst[s.base[wid][dgs[it]] + rank[it]] = (uint16_t)ixs[it];
        }
    }
    __syncthreads();
}

// Sorts the keys [0, cnt) (cnt <= NT * 8) of kin / iin by (key, id) -- ids
// ascend on entry, every pass is stable -- and writes them to kout / iout
// (which may alias kin / iin: everything is read before anything is written).
template <int NT>
__device__ __forceinline__ void seg_sort_body(SegLds<NT> &s, const uint64_t *kin,
                                              const uint32_t *iin, int cnt, uint64_t *kout,
                                              uint32_t *iout)
{
    const int tid = threadIdx.x;
    uint64_t vo = 0, va = ~0ull;
    {
        uint64_t kv[kItems];
        uint32_t iv[kItems];
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            const int j = u * NT + tid;
            kv[u] = kin[min(j, cnt - 1)]; // clamped: no branch around the loads
            iv[u] = iin[min(j, cnt - 1)];
        }
        // every slot j < NT * kItems is written (past cnt: never read), and
        // the masks take only the real keys, without a branch
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
            const int j = u * NT + tid;
            const uint64_t m = j < cnt ? ~0ull : 0ull;
            s.key[j] = kv[u];
            s.id[j] = iv[u];
            s.ix[0][j] = (uint16_t)j;
            vo |= kv[u] & m;
            va &= kv[u] | ~m;
        }
    }
    vo = wave_or64(vo);
    va = wave_and64(va);
    if (lane_id() == 0) {
        s.so[tid / kWave] = vo;
        s.sa[tid / kWave] = va;
    }
    if (tid == 0)
        s.flag = 0;
    for (int i = tid; i < (int)(sizeof(s.whist) / 4); i += NT)
        ((uint32_t *)s.whist)[i] = 0u;
    __syncthreads();
    vo = 0;
    va = ~0ull;
    for (int w = 0; w < NT / kWave; ++w) {
        vo |= s.so[w];
        va &= s.sa[w];
    }
    const uint64_t vm = vo & ~va;
    uint32_t all = 0; // bit p: chunk p varies inside the segment
    for (int p = 0; p < kChunks; ++p)
        all |= chunk_varies(vm, p) ? 1u << p : 0u;
    uint32_t fast = all; // the top kFastChunks of them
    for (int c = __popc(all) - kFastChunks; c > 0; --c)
        fast &= fast - 1;
    const int rows = (cnt + NT - 1) / NT;

    int cur = 0, npass = 0;
    for (int p = 0; p < kChunks; ++p) {
        if ((fast >> p) & 1u) {
            seg_rank_pass<NT>(s, s.ix[cur], s.ix[cur ^ 1], cnt, rows, p, npass++ & 1);
            cur ^= 1;
        }
    }
    if (fast != all) {
        // distinct keys that agree on the sorted chunks would be out of order
        uint64_t lo = 0;
        for (int p = 0; p < kChunks; ++p)
            if (((all & ~fast) >> p) & 1u)
                lo |= 0xffull << (8 * p);
        for (int j = tid + 1; j < cnt; j += NT) {
            const uint64_t x = s.key[s.ix[cur][j]], y = s.key[s.ix[cur][j - 1]];
            if (x != y && ((x ^ y) & ~lo) == 0)
                s.flag = 1;
        }
        __syncthreads();
        if (s.flag) {
            for (int j = tid; j < cnt; j += NT)
                s.ix[0][j] = (uint16_t)j;
            __syncthreads();
            cur = 0;
            for (int p = 0; p < kChunks; ++p) {
                if ((all >> p) & 1u) {
                    seg_rank_pass<NT>(s, s.ix[cur], s.ix[cur ^ 1], cnt, rows, p, npass++ & 1);
                    cur ^= 1;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int j = u * NT + tid;
        if (j < cnt) {
            const uint16_t ix = s.ix[cur][j];
            kout[j] = s.key[ix];
            iout[j] = s.id[ix];
        }
    }
    __syncthreads();
}

// Segment d of table t (blockIdx = (d, t)) when it holds LO+1 .. NT*kItems
// keys.
template <int NT, int LO>
__global__ __launch_bounds__(NT) void seg_sort_kernel(BuildArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    SegLds<NT> &s = *(SegLds<NT> *)lds;
    const int d = blockIdx.x, t = blockIdx.y;
    if (d >= (1 << a.msd_bits))
        return;
    const int e = (t << a.msd_bits) + d;
    const int cnt = (int)a.ghist[e];
    if (cnt <= LO || cnt > NT * kItems || table_complete(a.tor, a.tand, t, a.msd_bits))
        return;
    const int64_t base = (int64_t)t * a.n + a.seg_start[e];
    seg_sort_body<NT>(s, a.ka + base, a.ia + base, cnt, a.kb + base, a.ids + base);
}

// --------------------------------------------------------- big segments

// A key that fills at least 16 of 64 evenly spaced samples of keys[0, size)
// (wave 0 of the block decides; lowest lane on ties).  Returns the count
// (0 for lanes other than lane 0 of wave 0) and the key in *pivot.
__device__ __forceinline__ uint32_t sample_pivot(const uint64_t *kin, uint32_t size,
                                                 uint64_t *pivot)
{
    const int tid = threadIdx.x;
    uint32_t best = 0;
    uint64_t ks = 0;
    if (tid < kWave) {
        ks = kin[(uint64_t)tid * size / kWave];
        uint32_t c = 0;
        for (int j = 0; j < kWave; ++j) {
            const uint64_t kj = ((uint64_t)(uint32_t)__shfl((int)(ks >> 32), j, kWave) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)ks, j, kWave);
            c += kj == ks;
        }
        best = (c << 8) | (uint32_t)(kWave - 1 - tid);
        for (int o = 32; o >= 1; o >>= 1)
            best = max(best, (uint32_t)__shfl_xor((int)best, o, kWave));
        if ((uint32_t)(kWave - 1 - tid) == (best & 255u))
            *pivot = ks;
    }
    return best >> 8;
}

// Per big segment (in ka / ia after the segment scatter): the pivot, if any.
__global__ __launch_bounds__(kWave) void big_pivot_kernel(BuildArgs a)
{
    const uint32_t nb = a.bcount[0];
    for (uint32_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
        uint32_t *b = a.blist + kBig * bi;
        const int e = ((int)b[0] << a.msd_bits) + (int)b[1];
        const uint64_t *kin = a.ka + (int64_t)b[0] * a.n + a.seg_start[e];
        __shared__ uint64_t pv;
        const uint32_t c = sample_pivot(kin, a.ghist[e], &pv);
        __syncthreads();
        if (threadIdx.x == 0) {
            b[4] = c >= 16;
            a.bpivot[bi] = pv;
        }
        __syncthreads();
    }
}

// Per tile of a big segment with a pivot: counts of keys <, ==, > pivot.
__global__ __launch_bounds__(256) void big_count_kernel(BuildArgs a)
{
    const uint32_t nt = a.bcount[2];
    __shared__ uint32_t sc[256 / kWave][2];
    for (uint32_t j = blockIdx.x; j < nt; j += gridDim.x) {
        const uint32_t bi = a.btile[2 * j], k = a.btile[2 * j + 1];
        const uint32_t *b = a.blist + kBig * bi;
        if (!b[4])
            continue;
        const int e = ((int)b[0] << a.msd_bits) + (int)b[1];
        const uint32_t size = a.ghist[e];
        const uint32_t cnt = min((uint32_t)kTile, size - k * kTile);
        const uint64_t *kin = a.ka + (int64_t)b[0] * a.n + a.seg_start[e] + (int64_t)k * kTile;
        const uint64_t pivot = a.bpivot[bi];
        uint32_t nlt = 0, neq = 0;
        for_each_key(kin, cnt, [&](uint32_t, uint64_t key) {
            nlt += key < pivot;
            neq += key == pivot;
        });
        nlt = wave_sum(nlt);
        neq = wave_sum(neq);
        if (lane_id() == 0) {
            sc[threadIdx.x / kWave][0] = nlt;
            sc[threadIdx.x / kWave][1] = neq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t l = 0, q = 0;
            for (int w = 0; w < 256 / kWave; ++w) {
                l += sc[w][0];
                q += sc[w][1];
            }
            a.tcls[4 * j] = l;
            a.tcls[4 * j + 1] = q;
            a.tcls[4 * j + 2] = cnt - l - q;
        }
        __syncthreads();
    }
}

// Per big segment with a pivot: class sizes and each tile's class offsets
// (table positions: the < keys first, then the == run, then the > keys).
__global__ __launch_bounds__(kWave) void big_cscan_kernel(BuildArgs a)
{
    const uint32_t nb = a.bcount[0];
    const uint64_t lt = lanemask_lt();
    // every lane of the wave runs the same number of rounds (the ballots
    // below need the whole wave); lanes past nb do nothing
    const uint32_t rounds = (nb + gridDim.x * kWave - 1) / (gridDim.x * kWave);
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint32_t bi = (r * gridDim.x + blockIdx.x) * kWave + threadIdx.x;
        uint32_t *b = a.blist + kBig * min(bi, nb - 1u);
        const bool piv = bi < nb && b[4];
        uint32_t pst[2] = {0, 0}, pn[2] = {0, 0};
        if (piv) {
            const int e = ((int)b[0] << a.msd_bits) + (int)b[1];
            uint32_t nlt = 0, neq = 0;
            for (uint32_t k = 0; k < b[3]; ++k) {
                nlt += a.tcls[4 * (b[2] + k)];
                neq += a.tcls[4 * (b[2] + k) + 1];
            }
            uint32_t o0 = a.seg_start[e], o1 = o0 + nlt, o2 = o1 + neq;
            for (uint32_t k = 0; k < b[3]; ++k) {
                uint32_t *c = a.tcls + 4 * (b[2] + k);
                const uint32_t c0 = c[0], c1 = c[1], c2 = c[2];
                c[0] = o0;
                c[1] = o1;
                c[2] = o2;
                o0 += c0;
                o1 += c1;
                o2 += c2;
            }
            b[5] = nlt;
            b[6] = neq;
            const uint32_t size = a.ghist[e], st = a.seg_start[e];
            pst[0] = st;
            pn[0] = nlt;
            pst[1] = st + nlt + neq;
            pn[1] = size - nlt - neq;
        }
        // The < and > parts of at most 4096 keys go to the segment sorts
        // (several workgroups per CU) rather than to the big-segment sort.
        // One atomic add per wave and list reserves the wave's slots.
        uint32_t handed = 0;
        for (int q = 0; q < 2; ++q) {
            for (int cls = 0; cls < 2; ++cls) {
                const bool take = pn[q] > 0u && pn[q] <= (uint32_t)kSegSmall &&
                                  (pn[q] <= (uint32_t)kSegTiny ? 0 : 1) == cls;
                const uint64_t bal = __ballot(take);
                if (!bal)
                    continue;
                uint32_t first = 0;
                if (lane_id() == __builtin_ctzll(bal))
                    first = atomicAdd(&a.bcount[3 + cls], (uint32_t)__popcll(bal));
                first = __shfl(first, __builtin_ctzll(bal), kWave);
                if (take) {
                    const uint32_t slot = first + (uint32_t)__popcll(bal & lt);
                    uint32_t *p =
                        a.plist + 3 * ((size_t)cls * 2 * ((size_t)a.L << a.msd_bits) + slot);
                    p[0] = b[0];
                    p[1] = pst[q];
                    p[2] = pn[q];
                    handed |= 1u << q;
                }
            }
        }
        if (piv)
            b[7] = handed;
    }
}

// The < and > parts listed by big_cscan (after big_part has written them to
// kb / ids), sorted in place: class CLS 0 (1..2048 keys, 256 threads) or 1
// (2049..4096, 512 threads); workgroup g takes entries g, g + grid, ...
template <int NT, int CLS>
__global__ __launch_bounds__(NT) void part_sort_kernel(BuildArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    SegLds<NT> &s = *(SegLds<NT> *)lds;
    const uint32_t count = a.bcount[3 + CLS];
    const uint32_t *list = a.plist + 3 * (size_t)CLS * 2 * ((size_t)a.L << a.msd_bits);
    for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
        const uint32_t *p = list + 3 * (size_t)j;
        const int64_t off = (int64_t)p[0] * a.n + p[1];
        seg_sort_body<NT>(s, a.kb + off, a.ids + off, (int)p[2], a.kb + off, a.ids + off);
    }
}

// Stable 3-way partition of keys [0, cnt) around pivot: class 0 (key <
// pivot), 1 (==), 2 (>) go to kout/iout at base[class] + (rank among the
// keys of that class).  Tiles of 8192 keys in order; wave w ranks rows
// w*8 .. w*8+7 of 64 keys with two ballots; base[] (LDS) advances per tile.
__device__ __noinline__ void partition3(uint32_t (*cls)[4], const uint64_t *kin,
                                        const uint32_t *iin, uint32_t cnt, uint64_t pivot,
                                        uint32_t *base, uint64_t *kout, uint32_t *iout)
{
    const int tid = threadIdx.x, wid = tid / kWave, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    for (uint32_t t0 = 0; t0 < cnt; t0 += kTile) {
        uint32_t cl[kItems], rank[kItems], iv[kItems];
        uint64_t kv[kItems];
        uint32_t r0 = 0, r1 = 0, r2 = 0; // this wave's running class counts
        // all loads first (clamped: no branch), then the classes
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t i = t0 + wid * (kWave * kItems) + it * kWave + lane;
            kv[it] = kin[min(i, cnt - 1u)];
            iv[it] = iin[min(i, cnt - 1u)];
        }
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t i = t0 + wid * (kWave * kItems) + it * kWave + lane;
            cl[it] = i >= cnt ? 3u : kv[it] < pivot ? 0u : (kv[it] == pivot ? 1u : 2u);
        }
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t c = cl[it];
            const uint64_t b0 = __ballot(c == 0), b1 = __ballot(c == 1), b2 = __ballot(c == 2);
            const uint64_t mine = c == 0 ? b0 : (c == 1 ? b1 : b2);
            rank[it] = (c == 0 ? r0 : (c == 1 ? r1 : r2)) + __popcll(mine & lt);
            r0 += __popcll(b0);
            r1 += __popcll(b1);
            r2 += __popcll(b2);
        }
        if (lane == 0) {
            cls[wid][0] = r0;
            cls[wid][1] = r1;
            cls[wid][2] = r2;
        }
        __syncthreads();
        uint32_t p0 = 0, p1 = 0, p2 = 0; // class counts of the earlier waves
        for (int w = 0; w < wid; ++w) {
            p0 += cls[w][0];
            p1 += cls[w][1];
            p2 += cls[w][2];
        }
        const uint32_t q0 = base[0] + p0, q1 = base[1] + p1, q2 = base[2] + p2;
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t c = cl[it];
            if (c < 3) {
                const uint32_t pos = (c == 0 ? q0 : (c == 1 ? q1 : q2)) + rank[it];
                kout[pos] = kv[it];
                iout[pos] = iv[it];
            }
        }
        __syncthreads();
        if (tid < 3) {
            uint32_t tot = 0;
            for (int w = 0; w < kWaves; ++w)
                tot += cls[w][tid];
            base[tid] += tot;
        }
        __syncthreads();
    }
}

// Per tile of a big segment with a pivot: the stable 3-way scatter from
// ka / ia to kb / ids (the == run lands in its final place).  Each XCD takes
// a contiguous range of the tile list (the grid is a multiple of kXcds), so
// that consecutive tiles of a segment, which write adjacent ranges of each
// class, share their boundary cache lines in one L2.
__global__ __launch_bounds__(kThreads) void big_part_kernel(BuildArgs a)
{
    __shared__ uint32_t cls[kWaves][4];
    __shared__ uint32_t base[4];
    const uint32_t nt = a.bcount[2];
    const uint32_t chunk = (nt + kXcds - 1) / kXcds;
    const uint32_t j0 = (blockIdx.x % kXcds) * chunk, j1 = min(nt, j0 + chunk);
    for (uint32_t j = j0 + blockIdx.x / kXcds; j < j1; j += gridDim.x / kXcds) {
        const uint32_t bi = a.btile[2 * j], k = a.btile[2 * j + 1];
        const uint32_t *b = a.blist + kBig * bi;
        if (!b[4])
            continue;
        const int e = ((int)b[0] << a.msd_bits) + (int)b[1];
        const uint32_t cnt = min((uint32_t)kTile, a.ghist[e] - k * kTile);
        const int64_t tb = (int64_t)b[0] * a.n;
        const int64_t start = tb + a.seg_start[e] + (int64_t)k * kTile;
        if (threadIdx.x < 3)
            base[threadIdx.x] = a.tcls[4 * j + threadIdx.x];
        __syncthreads();
        partition3(cls, a.ka + start, a.ia + start, cnt, a.bpivot[bi], base, a.kb + tb,
                   a.ids + tb);
    }
}

struct BigLds {
    union {
        ScatterLds<kRadix> sc;
        SegLds<kThreads> sg;
    } u;
    uint32_t hist[kRadix];
    uint32_t run[kRadix];
    uint32_t wsum[kRadix / kWave];
    uint64_t so[kWaves], sa[kWaves];
    uint32_t cls[kWaves][4]; // per-wave class counts of the 3-way partition
    uint64_t pivot;
    uint32_t pivot_cnt;
    int top;
};

constexpr size_t kLdsBytes = 160 * 1024; // per CU
static_assert(sizeof(BigLds) <= kLdsBytes, "big-segment workgroup exceeds the LDS");
static_assert(4 * sizeof(SegLds<kSegThreadsS>) <= kLdsBytes, "four small sorts per CU");
static_assert(2 * sizeof(SegLds<kSegThreads>) <= kLdsBytes, "two segment sorts per CU");

// The big path calls these out of line: inlined together with the
// partition they exceed the register budget of a 1024-thread workgroup.
__device__ __noinline__ void big_seg_sort(SegLds<kThreads> &s, const uint64_t *kin,
                                          const uint32_t *iin, int cnt, uint64_t *kout,
                                          uint32_t *iout)
{
    seg_sort_body<kThreads>(s, kin, iin, cnt, kout, iout);
}

__device__ __noinline__ void big_scatter(ScatterLds<kRadix> &s, const uint64_t *kin,
                                         const uint32_t *iin, int cnt, int shift,
                                         const uint32_t *goff, uint64_t *kout, uint32_t *iout)
{
    scatter_tile<kRadix>(s, kin, iin, 0, cnt, shift, 8, goff, kout, iout);
}

// One workgroup per big segment: a stack of parts (start within the table,
// size, buffer 0 = ka/ia, 1 = kb/ids).  A part with one key is moved to
// kb/ids as it is; a part of at most kSegLarge keys is sorted in LDS into
// kb/ids; a larger one is split by its top 8 varying bits into the other
// buffer (a stable scatter, tile by tile in order) and its non-empty
// children are pushed.  Before that, a key filling at least 16 of 64 evenly
// spaced samples is split off by a stable 3-way partition (its run is final;
// the smaller and larger keys are pushed).  A segment varies in at most bits
// 0..62 and each split removes at least 8 varying bits, so a path holds at
// most 8 splits (255 pushes each) plus partitions (2 each, every one taking
// the sampled key's run out of the part), far below kStackMax.
__global__ __launch_bounds__(kThreads) void big_sort_kernel(BuildArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    BigLds &s = *(BigLds *)lds;
    const int tid = threadIdx.x;
    const uint32_t nb = a.bcount[0];
    uint32_t *stk = a.stack + (size_t)blockIdx.x * kStackMax * 3;
    for (uint32_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
        const uint32_t *b = a.blist + kBig * bi;
        const int t = (int)b[0];
        const int e = (t << a.msd_bits) + (int)b[1];
        const int64_t tb = (int64_t)t * a.n;
        if (tid == 0) {
            // a segment split around its pivot by the parallel partition
            // leaves its < and > keys in kb / ids (the == run is final);
            // any other starts whole in ka / ia
            int tp = 0;
            const uint32_t st = a.seg_start[e], size = a.ghist[e];
            if (b[4]) {
                const uint32_t nlt = b[5], neq = b[6];
                if (nlt && !(b[7] & 1u)) {
                    stk[3 * tp] = st;
                    stk[3 * tp + 1] = nlt;
                    stk[3 * tp + 2] = 1;
                    ++tp;
                }
                if (size - nlt - neq && !(b[7] & 2u)) {
                    stk[3 * tp] = st + nlt + neq;
                    stk[3 * tp + 1] = size - nlt - neq;
                    stk[3 * tp + 2] = 1;
                    ++tp;
                }
            } else {
                stk[0] = st;
                stk[1] = size;
                stk[2] = 0;
                tp = 1;
            }
            s.top = tp;
        }
        __syncthreads();
        while (true) {
            const int top = s.top;
            if (top == 0)
                break;
            const uint32_t start = stk[3 * (top - 1)];
            const uint32_t size = stk[3 * (top - 1) + 1];
            const uint32_t buf = stk[3 * (top - 1) + 2];
            __syncthreads();
            if (tid == 0)
                s.top = top - 1;
            const uint64_t *kin = (buf ? a.kb : a.ka) + tb + start;
            const uint32_t *iin = (buf ? a.ids : a.ia) + tb + start;
            uint64_t *kout = a.kb + tb + start;
            uint32_t *iout = a.ids + tb + start;
            if (size <= (uint32_t)kSegLarge) {
                big_seg_sort(s.u.sg, kin, iin, (int)size, kout, iout);
                continue;
            }
            // a key that fills at least a quarter of 64 evenly spaced samples
            // is split off by a stable 3-way partition: its run is final
            {
                const uint32_t c = sample_pivot(kin, size, &s.pivot);
                if (tid == 0)
                    s.pivot_cnt = c;
            }
            __syncthreads();
            if (s.pivot_cnt >= 16) {
                const uint64_t pivot = s.pivot;
                uint32_t nlt = 0, neq = 0;
                for_each_key(kin, size, [&](uint32_t, uint64_t k) {
                    nlt += k < pivot;
                    neq += k == pivot;
                });
                nlt = wave_sum(nlt);
                neq = wave_sum(neq);
                if (lane_id() == 0) {
                    s.cls[tid / kWave][0] = nlt;
                    s.cls[tid / kWave][1] = neq;
                }
                __syncthreads();
                nlt = neq = 0;
                for (int w = 0; w < kWaves; ++w) {
                    nlt += s.cls[w][0];
                    neq += s.cls[w][1];
                }
                __syncthreads();
                if (tid == 0) {
                    s.run[0] = 0;
                    s.run[1] = nlt;
                    s.run[2] = nlt + neq;
                }
                __syncthreads();
                uint64_t *ko = (buf ? a.ka : a.kb) + tb + start;
                uint32_t *io = (buf ? a.ia : a.ids) + tb + start;
                partition3(s.cls, kin, iin, size, pivot, s.run, ko, io);
                if (tid == 0 && s.top + 3 > kStackMax) {
                    atomicAdd(&a.bcount[1], 1u); // cannot happen (see the bound above)
                } else if (tid == 0) {
                    int tp = s.top;
                    const uint32_t ngt = size - nlt - neq;
                    if (nlt) {
                        stk[3 * tp] = start;
                        stk[3 * tp + 1] = nlt;
                        stk[3 * tp + 2] = buf ^ 1u;
                        ++tp;
                    }
                    if (buf) { // the equal run landed in ka / ia: one more move
                        stk[3 * tp] = start + nlt;
                        stk[3 * tp + 1] = neq;
                        stk[3 * tp + 2] = 0;
                        ++tp;
                    }
                    if (ngt) {
                        stk[3 * tp] = start + nlt + neq;
                        stk[3 * tp + 1] = ngt;
                        stk[3 * tp + 2] = buf ^ 1u;
                        ++tp;
                    }
                    s.top = tp;
                }
                __syncthreads();
                continue;
            }
            uint64_t vo, va;
            block_or_and(kin, size, s.so, s.sa, vo, va);
            const uint64_t vm = vo & ~va;
            if (vm == 0) { // one key: already in id order
                if (buf == 0)
                    for_each_key(kin, size, [&](uint32_t j, uint64_t k) {
                        kout[j] = k;
                        iout[j] = iin[j];
                    });
                __syncthreads();
                continue;
            }
            const int shift = top_shift(vm, 8);
            // digit counts of the whole part, then child starts
            for (int i = tid; i < kRadix; i += kThreads)
                s.hist[i] = 0;
            __syncthreads();
            for_each_key(kin, size, [&](uint32_t, uint64_t k) {
                atomicAdd(&s.hist[(uint32_t)(k >> shift) & 255u], 1u);
            });
            __syncthreads();
            const uint32_t c = tid < kRadix ? s.hist[tid] : 0u;
            const uint32_t ex = scan_excl(c, kRadix, s.wsum);
            if (tid < kRadix)
                s.run[tid] = ex;
            __syncthreads();
            // push the children: runs of consecutive children of at most
            // kSegLarge keys in total go as one part (sorting their union
            // by key orders each of them: they are already grouped by
            // digit), a larger child alone
            if (tid == 0 && s.top + kRadix > kStackMax) {
                atomicAdd(&a.bcount[1], 1u); // cannot happen (see the bound above)
            } else if (tid == 0) {
                int tp = s.top;
                uint32_t bs = 0, bn = 0; // open batch: start, size
                for (int d = 0; d <= kRadix; ++d) {
                    const uint32_t cc = d < kRadix ? s.hist[d] : 0u;
                    if (d < kRadix && cc == 0)
                        continue;
                    const bool big = cc > (uint32_t)kSegLarge;
                    if (bn && (d == kRadix || big || bn + cc > (uint32_t)kSegLarge)) {
                        stk[3 * tp] = start + bs;
                        stk[3 * tp + 1] = bn;
                        stk[3 * tp + 2] = buf ^ 1u;
                        ++tp;
                        bn = 0;
                    }
                    if (d == kRadix)
                        break;
                    if (big) {
                        stk[3 * tp] = start + s.run[d];
                        stk[3 * tp + 1] = cc;
                        stk[3 * tp + 2] = buf ^ 1u;
                        ++tp;
                    } else {
                        if (bn == 0)
                            bs = s.run[d];
                        bn += cc;
                    }
                }
                s.top = tp;
            }
            __syncthreads();
            // stable scatter into the other buffer, tile by tile in order
            uint64_t *ko = (buf ? a.ka : a.kb) + tb + start;
            uint32_t *io = (buf ? a.ia : a.ids) + tb + start;
            for (uint32_t base = 0; base < size; base += kTile) {
                const int cnt = (int)min((uint32_t)kTile, size - base);
                big_scatter(s.u.sc, kin + base, iin + base, cnt, shift, s.run, ko, io);
                if (tid < kRadix)
                    s.run[tid] += s.u.sc.count[tid];
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- bucket offsets

struct HeadArgs {
    const uint64_t *sk; // sorted keys [L][n]
    int64_t n;
    int32_t L;
    int32_t ntiles;     // head tiles per table
    uint64_t *status;   // [L][ntiles] tile status words (zero on entry)
    uint32_t *counter;  // [L][16] tile ids handed out per table (element 0 of a
                        // 64-byte line each; zero on entry)
    uint32_t *errors;   // waits that gave up (zero on entry; stays zero)
    uint64_t *ukeys;    // [L][n]
    uint32_t *offs;     // [L][n+1]
    int64_t *nuniq;     // [L]
};

// Tile status word: flag in bits 62..63 (0: not yet published, kHeadAgg: the
// tile's own head count, kHeadPre: the heads up to and including the tile),
// count in bits 0..31.
constexpr uint64_t kHeadAgg = 1ull << 62, kHeadPre = 2ull << 62;
constexpr int kSpinMax = 1 << 16; // polls of one status word (about 0.1 s)

// A 64-bit value from the lane below (wave_shr:1 on each half); lane 0
// receives `fill`.
__device__ __forceinline__ uint64_t lane_below(uint64_t x, uint64_t fill)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(
        (int)(uint32_t)fill, (int)(uint32_t)x, 0x138, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
        (int)(uint32_t)(fill >> 32), (int)(uint32_t)(x >> 32), 0x138, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lane63(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), kWave - 1);
    return ((uint64_t)hi << 32) | lo;
}

// A wave's chunk of kHeadItems rows of 64 keys, positions wb + it*64 + lane
// (loads clamped into [0, n) rather than guarded, so that none sits in a
// branch).  hb[it]: ballot of the positions (< n) that start a run.  The
// key before a position is the lane below's, for lane 0 the last lane of
// the row before, for the chunk's first row the key before the chunk: one
// load per key.
__device__ __forceinline__ void chunk_heads(const uint64_t *k, int64_t wb, int64_t n,
                                            uint64_t (&x)[kHeadItems], uint64_t (&hb)[kHeadItems])
{
    const int lane = lane_id();
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it)
        x[it] = k[min(wb + it * kWave + lane, n - 1)];
    uint64_t before = k[max(min(wb - 1, n - 1), (int64_t)0)];
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it) {
        const uint64_t prev = lane_below(x[it], before);
        const int64_t i = wb + it * kWave + lane;
        hb[it] = __ballot(i < n && (i == 0 || x[it] != prev));
        before = lane63(x[it]);
    }
}

// Run heads of every table in one pass (a decoupled look-back).  The
// workgroups of table t (blockIdx.y) take their tile ids from the table's
// counter in the order they start, so every tile a tile waits for has
// already started and runs to its end.  A tile counts its
// heads and publishes the count, then adds its predecessors' counts back to
// the first one that has published its inclusive count, publishes its own
// inclusive count and writes its distinct keys and bucket starts.  The
// status words are device-scope atomics (coherent across the XCDs' caches).
// A wait gives up after kSpinMax polls of a window and counts an error, so
// every wave exits whatever happens (by the ordering argument the count
// stays zero).
__global__ __launch_bounds__(kHeadThreads) void head_kernel(HeadArgs a)
{
    constexpr int kW = kHeadThreads / kWave;
    __shared__ uint32_t wtot[kW], s_g, s_excl;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int t = blockIdx.y;
    if (threadIdx.x == 0)
        s_g = atomicAdd(&a.counter[16 * t], 1u);
    __syncthreads();
    const int tile = (int)s_g;
    const uint64_t *k = a.sk + (int64_t)t * a.n;
    const int64_t wb = (int64_t)tile * kHeadTile + wid * (kWave * kHeadItems);
    uint64_t x[kHeadItems], hb[kHeadItems];
    chunk_heads(k, wb, a.n, x, hb);
    uint32_t tot = 0;
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it)
        tot += (uint32_t)__popcll(hb[it]);
    if (lane == 0)
        wtot[wid] = tot;
    __syncthreads();
    // wave 0 publishes the tile's count and looks back over windows of 64
    // predecessors (lane i reads tile - 1 - i; positions before tile 0 count
    // as an inclusive count of 0): it adds the counts of the lanes up to the
    // first one holding an inclusive count, once all of them are published
    if (wid == 0) {
        uint32_t agg = 0;
        for (int w = 0; w < kW; ++w)
            agg += wtot[w];
        uint64_t *st = a.status + (int64_t)t * a.ntiles;
        if (lane == 0 && tile > 0)
            __hip_atomic_store(&st[tile], kHeadAgg | agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint32_t excl = 0;
        int spin = 0;
        for (int top = tile - 1; top >= 0;) {
            const int j = top - lane;
            const uint64_t v = j >= 0 ? __hip_atomic_load(&st[j], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : kHeadPre;
            const uint64_t pre = __ballot((v >> 62) == 2), nil = __ballot((v >> 62) == 0);
            const int fp = pre ? __builtin_ctzll(pre) : kWave; // first inclusive count
            const uint64_t need = fp == kWave ? ~0ull : (2ull << fp) - 1ull;
            if (nil & need) {
                if (++spin == kSpinMax) {
                    if (lane == 0)
                        atomicAdd(a.errors, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += wave_sum(lane <= fp ? (uint32_t)v : 0u);
            if (fp < kWave)
                break;
            top -= kWave;
        }
        if (lane == 0) {
            __hip_atomic_store(&st[tile], kHeadPre | (excl + agg), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
            if (tile == a.ntiles - 1) {
                a.nuniq[t] = excl + agg;
                a.offs[(int64_t)t * (a.n + 1) + excl + agg] = (uint32_t)a.n;
            }
        }
    }
    __syncthreads();
    // heads before this wave's chunk: the tiles before, then the waves before
    uint32_t run = s_excl;
    for (int w = 0; w < wid; ++w)
        run += wtot[w];
    uint64_t *uk = a.ukeys + (int64_t)t * a.n;
    uint32_t *of = a.offs + (int64_t)t * (a.n + 1);
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int it = 0; it < kHeadItems; ++it) {
        if ((hb[it] >> lane) & 1ull) {
            const uint32_t u = run + (uint32_t)__popcll(hb[it] & lt);
            uk[u] = x[it];
            of[u] = (uint32_t)(wb + it * kWave + lane);
        }
        run += (uint32_t)__popcll(hb[it]);
    }
}

// Writes the index of an empty table set: nuniq = 0 and offs[t][0] = 0.
__global__ __launch_bounds__(256) void empty_index_kernel(int64_t *nuniq, uint32_t *offs, int L)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x) {
        nuniq[t] = 0;
        offs[t] = 0;
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
    size_t ka, kb, ia, tor, tand, tile_hist, ghist, seg_start, blist, bpivot, btile, tcls, bcount,
        plist, stack, hstat, total;
    int ntiles, nhtiles, bits, big_grid, maxbt;
};

// Segment digit width: about 2048 keys per segment, at most 2^10 segments.
// A segment sort has a fixed cost per workgroup, so at n = 1M keys per table
// 2^9 segments built faster than 2^10 (fewer, longer digit runs in the
// scatter too) and than 2^8 (more heavy segments for the big path).
int msd_bits_for(int64_t n)
{
    int b = 1;
    while (b < lsh::kMsdBitsMax && ((int64_t)2048 << b) < n)
        ++b;
    return b;
}

WsLayout ws_layout(int64_t n, int32_t L)
{
    using lsh::align_up;
    using namespace lsh;
    WsLayout w;
    w.ntiles = (int)((n + kTile - 1) / kTile);
    w.nhtiles = (int)((n + kHeadTile - 1) / kHeadTile);
    w.bits = msd_bits_for(n);
    const size_t nseg = (size_t)L << w.bits;
    // big segments: one workgroup per CU of an MI355X, each with its own stack
    w.big_grid = (int)(nseg < 256 ? nseg : 256);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align_up(bytes ? bytes : 1, 256);
        return at;
    };
    w.ka = take((size_t)L * n * 8);
    w.kb = take((size_t)L * n * 8);
    w.ia = take((size_t)L * n * 4);
    w.tor = take((size_t)L * 8);
    w.tand = take((size_t)L * 8);
    w.tile_hist = take(((size_t)L * w.ntiles << w.bits) * 4);
    w.ghist = take(nseg * 4);
    w.seg_start = take(nseg * 4);
    // tiles of the big segments: sum of ceil(c / kTile) <= L * n / kTile + (number of
    // big segments) <= L * n / kTile + L * 2^B
    w.maxbt = (int)((size_t)L * n / kTile + nseg + 1);
    w.blist = take(nseg * kBig * 4);
    w.bpivot = take(nseg * 8);
    w.btile = take((size_t)w.maxbt * 8);
    w.tcls = take((size_t)w.maxbt * 16);
    w.bcount = take(kCounts * 4);
    w.plist = take(2 * 2 * nseg * 3 * 4);
    w.stack = take((size_t)w.big_grid * kStackMax * 12);
    w.hstat = take(((size_t)L * (w.nhtiles > 0 ? w.nhtiles : 1) + 8 * (size_t)L + 1) * 8);
    w.total = o;
    return w;
}

// A build given a side stream runs its big-segment split and sort there,
// concurrently with the segment sorts on its main stream: the two touch
// disjoint segments of the sorted arrays, and the big-segment lists, pivots,
// class counts and stacks are theirs alone.  The main stream sorts the
// split's small parts after its segment sorts, once the side stream has
// partitioned them, and waits for the side stream before the run-head pass.  The fork and join events are the
// library's, one pair per device, created on first use; a build records and
// waits on them while holding the lock, so that concurrent builds do not mix
// their records.
constexpr int kMaxForkDevices = 64;
struct ForkEvents {
    hipEvent_t fork = nullptr, parted = nullptr, join = nullptr;
};
std::mutex g_fork_mu;
ForkEvents g_fork[kMaxForkDevices];

hipError_t fork_events(ForkEvents **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxForkDevices)
        return hipErrorInvalidDevice;
    ForkEvents &fe = g_fork[dev];
    if (!fe.fork && (e = hipEventCreateWithFlags(&fe.fork, hipEventDisableTiming)) != hipSuccess)
        return e;
    if (!fe.join && (e = hipEventCreateWithFlags(&fe.join, hipEventDisableTiming)) != hipSuccess)
        return e;
    if (!fe.parted &&
        (e = hipEventCreateWithFlags(&fe.parted, hipEventDisableTiming)) != hipSuccess)
        return e;
    *out = &fe;
    return hipSuccess;
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
                                      size_t ws_bytes, lsh_index **out, void *stream,
                                      void *side_stream)
{
    using namespace lsh;
    if (!out)
        LSH_FAIL(LSH_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || L < 1 || id_base < 0)
        LSH_FAIL(LSH_EINVAL, "bad n=%lld L=%d id_base=%lld", (long long)n, L, (long long)id_base);
    if (L > 65536)
        LSH_FAIL(LSH_EINVAL, "L = %d exceeds 65536 tables", L);
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
    if (lsh_status st = check_stream_device(stream); st != LSH_OK)
        return st;
    if (side_stream)
        if (lsh_status st = check_stream_device(side_stream); st != LSH_OK)
            return st;
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
        hipLaunchKernelGGL(empty_index_kernel, dim3((L + 255) / 256), dim3(256), 0, s, idx->nuniq,
                           idx->offs, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail("empty_index_kernel", e);
        *out = idx;
        return LSH_OK;
    }

    unsigned char *wb = (unsigned char *)ws;
    BuildArgs ba;
    ba.kin = keys;
    ba.key_ld = key_ld;
    ba.n = n;
    ba.L = L;
    ba.id_base = (uint32_t)id_base;
    ba.ntiles = wl.ntiles;
    ba.msd_bits = wl.bits;
    ba.tor = (uint64_t *)(wb + wl.tor);
    ba.tand = (uint64_t *)(wb + wl.tand);
    ba.tile_hist = (uint32_t *)(wb + wl.tile_hist);
    ba.ghist = (uint32_t *)(wb + wl.ghist);
    ba.seg_start = (uint32_t *)(wb + wl.seg_start);
    ba.ka = (uint64_t *)(wb + wl.ka);
    ba.kb = (uint64_t *)(wb + wl.kb);
    ba.ia = (uint32_t *)(wb + wl.ia);
    ba.ids = idx->sorted_ids;
    ba.blist = (uint32_t *)(wb + wl.blist);
    ba.bpivot = (uint64_t *)(wb + wl.bpivot);
    ba.btile = (uint32_t *)(wb + wl.btile);
    ba.tcls = (uint32_t *)(wb + wl.tcls);
    ba.bcount = (uint32_t *)(wb + wl.bcount);
    ba.plist = (uint32_t *)(wb + wl.plist);
    ba.stack = (uint32_t *)(wb + wl.stack);
    // run-head status words, the tile counters and the error count after them
    ba.hstat = (uint64_t *)(wb + wl.hstat);
    ba.nhstat = (int64_t)L * wl.nhtiles + 8 * (int64_t)L + 1;

    const size_t scatter_lds = sizeof(ScatterLds<kMsdRadixMax, kMsdItems>);
    const size_t seg_lds = sizeof(SegLds<kSegThreads>);
    const size_t segs_lds = sizeof(SegLds<kSegThreadsS>);
    const void *seg_fn = (const void *)seg_sort_kernel<kSegThreads, kSegTiny>;
    const void *segs_fn = (const void *)seg_sort_kernel<kSegThreadsS, 0>;
    const void *part_fn = (const void *)part_sort_kernel<kSegThreads, 1>;
    const void *parts_fn = (const void *)part_sort_kernel<kSegThreadsS, 0>;
    const size_t big_lds = sizeof(BigLds);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)msd_scatter_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)scatter_lds)) !=
            hipSuccess ||
        (e = hipFuncSetAttribute(seg_fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)seg_lds)) != hipSuccess ||
        (e = hipFuncSetAttribute(segs_fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)segs_lds)) != hipSuccess ||
        (e = hipFuncSetAttribute(part_fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)seg_lds)) != hipSuccess ||
        (e = hipFuncSetAttribute(parts_fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)segs_lds)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)big_sort_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)big_lds)) !=
            hipSuccess)
        return fail("hipFuncSetAttribute", e);

    const int nseg = L << wl.bits;
    dim3 tiles(wl.ntiles, L);
    hipLaunchKernelGGL(build_init_kernel, dim3((nseg + 255) / 256), dim3(256), 0, s, ba);
    hipLaunchKernelGGL(mask_up_kernel, tiles, dim3(kThreads), 0, s, ba);
    hipLaunchKernelGGL(msd_up_kernel, dim3(std::min(wl.ntiles, kMsdUpGrid), L), dim3(kThreads), 0, s,
                       ba);
    hipLaunchKernelGGL(msd_scan_kernel, dim3(L), dim3(kMsdRadixMax), 0, s, ba);
    constexpr int tpm = kMsdTile / kTile;
    const int64_t npair = (int64_t)((wl.ntiles + tpm - 1) / tpm) * L;
    hipLaunchKernelGGL(msd_scatter_kernel, dim3((unsigned)((npair + kXcds - 1) / kXcds * kXcds)),
                       dim3(kThreads), scatter_lds, s, ba);
    // Fork the big-segment path onto the side stream when one is given, a
    // segment can exceed the segment sorts (n > kSegSmall) and the main stream
    // is not being captured into a graph; otherwise everything runs on the
    // main stream, in the same order.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (side_stream && hipStreamIsCapturing(s, &cap) != hipSuccess) {
        // (the legacy stream while another stream captures): no fork, and
        // the error is cleared so that the launch check below does not see it
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;
    }
    std::unique_lock<std::mutex> fork_lock(g_fork_mu, std::defer_lock);
    ForkEvents *fe = nullptr;
    hipStream_t sb = s;
    if (side_stream && (hipStream_t)side_stream != s && n > kSegSmall &&
        cap == hipStreamCaptureStatusNone) {
        fork_lock.lock();
        if ((e = fork_events(&fe)) != hipSuccess)
            return fail("fork events", e);
        sb = (hipStream_t)side_stream;
        if ((e = hipEventRecord(fe->fork, s)) != hipSuccess ||
            (e = hipStreamWaitEvent(sb, fe->fork, 0)) != hipSuccess)
            return fail("side stream fork", e);
    }
    hipLaunchKernelGGL((seg_sort_kernel<kSegThreadsS, 0>), dim3(1 << wl.bits, L),
                       dim3(kSegThreadsS), segs_lds, s, ba);
    hipLaunchKernelGGL((seg_sort_kernel<kSegThreads, kSegTiny>), dim3(1 << wl.bits, L),
                       dim3(kSegThreads), seg_lds, s, ba);
    // The big-segment kernels walk lists built on the device, in grid-stride
    // loops.  Their grids are capped by the most work n keys per table can
    // give (segments above kSegSmall keys, their kTile tiles, two parts
    // each), so a small build (a serving insert) does not queue hundreds of
    // idle whole-CU workgroups behind other streams' work.
    const int64_t max_big = std::max<int64_t>(1, (int64_t)L * (n / (kSegSmall + 1)));
    const int64_t max_bt = std::max<int64_t>(1, (int64_t)L * (3 * n / kTile + 1));
    const int bg = (int)std::min<int64_t>(wl.big_grid, max_big);
    const int bt4 = (int)std::min<int64_t>(4 * wl.big_grid, max_bt);
    const int bt2 = (int)std::min<int64_t>(2 * wl.big_grid, max_bt);
    hipLaunchKernelGGL(big_pivot_kernel, dim3(bg), dim3(kWave), 0, sb, ba);
    hipLaunchKernelGGL(big_count_kernel, dim3(bt4), dim3(256), 0, sb, ba);
    hipLaunchKernelGGL(big_cscan_kernel, dim3(bg), dim3(kWave), 0, sb, ba);
    hipLaunchKernelGGL(big_part_kernel, dim3((bt2 + kXcds - 1) / kXcds * kXcds), dim3(kThreads), 0,
                       sb, ba);
    // the small parts are sorted on the main stream once the partition is
    // done (after the segment sorts there), the big sort on the side stream
    if (fe && ((e = hipEventRecord(fe->parted, sb)) != hipSuccess ||
               (e = hipStreamWaitEvent(s, fe->parted, 0)) != hipSuccess))
        return fail("side stream partition event", e);
    // the small parts of the split segments: as many workgroups as fit on
    // the 256 CUs at once (four and two per CU), at most two per big segment
    const int64_t parts = std::min<int64_t>(2 * nseg, 2 * max_big);
    hipLaunchKernelGGL((part_sort_kernel<kSegThreadsS, 0>),
                       dim3((int)std::min<int64_t>(parts, 4 * 256)), dim3(kSegThreadsS),
                       segs_lds, s, ba);
    hipLaunchKernelGGL((part_sort_kernel<kSegThreads, 1>),
                       dim3((int)std::min<int64_t>(parts, 2 * 256)), dim3(kSegThreads), seg_lds,
                       s, ba);
    hipLaunchKernelGGL(big_sort_kernel, dim3(bg), dim3(kThreads), big_lds, sb, ba);
    if (fe) {
        if ((e = hipGetLastError()) != hipSuccess)
            return fail("index kernels", e);
        if ((e = hipEventRecord(fe->join, sb)) != hipSuccess ||
            (e = hipStreamWaitEvent(s, fe->join, 0)) != hipSuccess)
            return fail("side stream join", e);
        fork_lock.unlock();
    }

    HeadArgs ha;
    ha.sk = ba.kb;
    ha.n = n;
    ha.L = L;
    ha.ntiles = wl.nhtiles;
    ha.status = (uint64_t *)(wb + wl.hstat);
    ha.counter = (uint32_t *)(ha.status + (size_t)L * wl.nhtiles);
    ha.errors = ha.counter + 16 * (size_t)L;
    ha.ukeys = idx->ukeys;
    ha.offs = idx->offs;
    ha.nuniq = idx->nuniq;
    hipLaunchKernelGGL(head_kernel, dim3(wl.nhtiles, L), dim3(kHeadThreads), 0, s, ha);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail("index kernels", e);
    *out = idx;
    return LSH_OK;
}

extern "C" lsh_status lsh_build_check_async(const void *ws, size_t ws_bytes, int64_t n, int32_t L,
                                            uint32_t *counts, void *stream)
{
    using namespace lsh;
    if (!counts)
        LSH_FAIL(LSH_EINVAL, "counts is NULL");
    if (n < 0 || L < 1)
        LSH_FAIL(LSH_EINVAL, "bad n=%lld L=%d", (long long)n, L);
    if (n == 0)
        return LSH_OK; // no build kernels ran; counts is not written
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const WsLayout wl = ws_layout(n, L);
    if (!ws || ws_bytes < wl.total)
        LSH_FAIL(LSH_EINVAL, "workspace needs %zu bytes, got %zu", wl.total, ws_bytes);
    const unsigned char *wb = (const unsigned char *)ws;
    // the same places lsh_build_index gives the counters
    const uint32_t *overflows = (const uint32_t *)(wb + wl.bcount) + 1;
    const uint32_t *waits =
        (const uint32_t *)((const uint64_t *)(wb + wl.hstat) + (size_t)L * wl.nhtiles) +
        16 * (size_t)L;
    if ((e = hipMemcpyAsync(&counts[0], overflows, 4, hipMemcpyDefault, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&counts[1], waits, 4, hipMemcpyDefault, s)) != hipSuccess)
        LSH_FAIL(LSH_EHIP, "lsh_build_check: %s", hip_msg(e));
    return LSH_OK;
}

extern "C" lsh_status lsh_build_check(const void *ws, size_t ws_bytes, int64_t n, int32_t L,
                                      uint32_t counts[2], void *stream)
{
    using namespace lsh;
    if (!counts)
        LSH_FAIL(LSH_EINVAL, "counts is NULL");
    counts[0] = counts[1] = 0;
    if (n < 0 || L < 1)
        LSH_FAIL(LSH_EINVAL, "bad n=%lld L=%d", (long long)n, L);
    if (n == 0)
        return LSH_OK; // no build kernels ran
    lsh_status st = lsh_build_check_async(ws, ws_bytes, n, L, counts, stream);
    if (st != LSH_OK)
        return st;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess)
        LSH_FAIL(LSH_EHIP, "lsh_build_check: %s", hip_msg(e));
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
