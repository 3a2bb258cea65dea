// Query probe and exact re-rank on gfx950.
//
// For each query (Section 3.1): look up its key in every table of every
// index segment, take the union of the bucket contents (ids below the
// watermark), score every distinct candidate by its exact distance to the
// query (Euclidean, or 1 - cos), and keep the k best by (score, id)
// (Section 6 retrieves the top-k this way).
//
// One workgroup per query (or per share, below).  Every bucket is an
// ascending id list, so the union is processed in windows of the id space
// that hold at most 2048 (one workgroup per CU) or 1024 (more) (bucket, id)
// entries: each window is gathered into LDS, sorted and deduplicated, its
// distinct ids are scored (one wave per candidate row, coalesced loads), and
// the window's (score, id) pairs are merged with the running top-k by a
// bitonic sort of 64-bit (score bits, id) keys.  Memory is bounded whatever
// the bucket sizes.
//
// Given a workspace, a batch of at most 1024 queries splits each query over
// several workgroups that take the candidate ids of their residue (id mod
// split): each bounds the same windows but gathers, sorts, dedupes and scores
// only its own ids, and leaves its top-k and candidate count in the
// workspace; query_merge_kernel then ranks the shares' entries per query.

#include <math.h>

#include <algorithm>
#include <type_traits>

#include "lsh_internal.h"

namespace lsh {

// Threads per query: 512 when the batch has at most one query per CU (a
// query then has a CU to itself), else 256.
constexpr int kQThreads = 256;
constexpr int kQThreadsSolo = 512;
constexpr int kMaxK = 64;
// a query's candidates are scored by up to kQuerySplit workgroups in batches
// of at most kSplitQueries queries (see lsh_query)
constexpr int kQuerySplit = 4;
constexpr int kSplitQueries = 1024;
constexpr int kMaxSeg = 16;
constexpr int kMaxLists = 1024;   // nseg * L

constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Per workgroup shape: cap, the (bucket, id) entries of a window; nr, the
// FP32 candidate rows a wave scores together (their loads in flight at
// once); wpe, the waves per SIMD the registers are sized for; sort_cpw, the
// chunks of 256 keys a wave holds in registers when the block sorts.  A solo query
// takes windows of 2048 entries and six rows per wave.  In a batch, windows
// of 1024 entries, three rows per wave and at most 128 VGPRs leave the LDS
// and registers for four queries per CU (two with the solo sizes), so more
// queries overlap their latency-bound phases.
template <int QT> struct QShape;
template <> struct QShape<kQThreadsSolo> {
    static constexpr int cap = 2048, nr = 6, wpe = 2, sort_cpw = 2;
};
template <> struct QShape<kQThreads> {
    static constexpr int cap = 1024, nr = 3, wpe = 4, sort_cpw = 1;
};
template <int QT> constexpr int sort_cap() { return pow2_at_least(QShape<QT>::cap + kMaxK); }

// LDS of a query workgroup: the query row, five arrays over the nl lists
// (one with nl + 1 entries), the sort buffer, the top-k and the window's ids.
template <int QT> size_t query_lds_bytes(int d, int nl)
{
    const size_t nlp = (size_t)((nl + 4) & ~3);
    return (size_t)((d * 4 + 15) & ~15) + 5 * nlp * 4 + 16 +
           (size_t)(sort_cap<QT>() + kMaxK) * 8 + (size_t)QShape<QT>::cap * 4;
}

struct QSeg {
    const uint32_t *ids;
    const uint64_t *ukeys;
    const uint32_t *offs;
    const int64_t *nuniq;
    int64_t n;
    int64_t id_end; // id_base + n: every id of the segment is below it
};

struct QueryArgs {
    QSeg seg[kMaxSeg];
    int32_t nseg, L;
    // base points
    const void *bx;
    int32_t bdt;
    const float *bscale;
    int64_t bld;
    int64_t bn;
    // queries
    const void *qx;
    int32_t qdt;
    const float *qscale;
    int64_t qld;
    int32_t d;
    const uint64_t *qkeys;
    int64_t qkey_ld;
    int32_t k;
    uint32_t watermark; // ids >= watermark are ignored (clamped to 2^32-1)
    int32_t metric;
    int32_t vec4; // FP32 base rows read as 16-byte chunks (aligned, d % 4 == 0)
    int64_t *ids;
    float *score;
    int32_t *ncand;
    // split > 1: workgroups per query; each leaves the top-k of its share of
    // the candidates in part[q][split][k] for query_merge_kernel
    int32_t split;
    uint64_t *part;
    uint32_t *pcount; // [q][split] distinct candidates of each share
};

// OCP E4M3FN -> FP32 by the gfx950 conversion instruction: exact for every
// finite pattern (subnormals included), and the NaN patterns S.1111.111 give
// NaN, as the stored value defines.
__device__ __forceinline__ float fp8_value(uint32_t b)
{
    return __builtin_amdgcn_cvt_f32_fp8((int)b, 0);
}

__device__ __forceinline__ float load_val(const void *x, int dt, const float *scale, int64_t row,
                                          int64_t ld, int32_t j)
{
    float sc = scale ? scale[row] : 1.0f;
    if (dt == LSH_F32)
        return ((const float *)x)[row * ld + j];
    if (dt == LSH_BF16)
        return sc * __uint_as_float((uint32_t)((const uint16_t *)x)[row * ld + j] << 16);
    return sc * fp8_value(((const uint8_t *)x)[row * ld + j]);
}

// Element off of a row of type DT (sc: the row's scale; 1 for FP32).
template <int DT>
__device__ __forceinline__ float load_dt(const void *x, float sc, int64_t off)
{
    if constexpr (DT == LSH_F32)
        return ((const float *)x)[off];
    if constexpr (DT == LSH_BF16)
        return sc * __uint_as_float((uint32_t)((const uint16_t *)x)[off] << 16);
    return sc * fp8_value(((const uint8_t *)x)[off]);
}

// Sums over NR candidate rows by a wave (each lane a partial sum per row):
// squared differences to the query (E2LSH) or the dot product and the row's
// squared norm (SRP).  kScoreLoads loads per lane and row are in flight at a
// time (rows of up to 1024 elements in one round trip): their indexes are
// clamped into [0, d) rather than guarded, and the lanes past d add 0.
constexpr int kScoreLoads = 16;

template <int DT, int NR>
__device__ __forceinline__ void score_rows(const QueryArgs &a, const float *qv,
                                           const int64_t (&row)[NR], float (&acc)[NR],
                                           float (&xx)[NR])
{
    const int lane = lane_id();
    float sc[NR];
    int64_t rb[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        sc[r] = DT != LSH_F32 && a.bscale ? a.bscale[row[r]] : 1.0f;
        rb[r] = row[r] * a.bld;
        acc[r] = 0.0f;
        xx[r] = 0.0f;
    }
    for (int j0 = 0; j0 < a.d; j0 += kScoreLoads * kWave) {
        float xv[NR][kScoreLoads];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < kScoreLoads; ++u)
                xv[r][u] = load_dt<DT>(a.bx, sc[r], rb[r] + min(j0 + u * kWave + lane, a.d - 1));
#pragma unroll
        for (int u = 0; u < kScoreLoads; ++u) {
            const int j = j0 + u * kWave + lane;
            const bool in = j < a.d;
            const float qj = in ? qv[j] : 0.0f;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const float x = in ? xv[r][u] : 0.0f;
                if (a.metric == LSH_E2LSH) {
                    const float df = qj - x;
                    acc[r] = fmaf(df, df, acc[r]);
                } else {
                    acc[r] = fmaf(qj, x, acc[r]);
                    xx[r] = fmaf(x, x, xx[r]);
                }
            }
        }
    }
}

// The same sums for FP32 rows read as 16-byte chunks (the base pointer
// 16-byte aligned, ld and d multiples of 4): 4 chunk loads per lane and row
// cover 1024 elements, so a wave keeps its NR rows in flight within the 63
// loads a wave can have outstanding.  Chunk indexes are clamped into the
// row; the lanes past its end add 0.
constexpr int kScoreChunks = 4;

template <int NR>
__device__ __forceinline__ void score_rows_v4(const QueryArgs &a, const float *qv,
                                              const int64_t (&row)[NR], float (&acc)[NR],
                                              float (&xx)[NR])
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int lane = lane_id();
    const int nch = a.d >> 2;
    const f4 *rp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        rp[r] = (const f4 *)((const float *)a.bx + row[r] * a.bld);
        acc[r] = 0.0f;
        xx[r] = 0.0f;
    }
    for (int c0 = 0; c0 < nch; c0 += kScoreChunks * kWave) {
        f4 xv[NR][kScoreChunks];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < kScoreChunks; ++u)
                xv[r][u] = rp[r][min(c0 + u * kWave + lane, nch - 1)];
#pragma unroll
        for (int u = 0; u < kScoreChunks; ++u) {
            const int c = c0 + u * kWave + lane;
            const bool in = c < nch;
            const f4 qc = in ? *(const f4 *)(qv + 4 * c) : f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const f4 x = in ? xv[r][u] : f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (a.metric == LSH_E2LSH) {
                        const float df = qc[e] - x[e];
                        acc[r] = fmaf(df, df, acc[r]);
                    } else {
                        acc[r] = fmaf(qc[e], x[e], acc[r]);
                        xx[r] = fmaf(x[e], x[e], xx[r]);
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *a, uint32_t lo, uint32_t hi,
                                                     uint32_t v)
{
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First index of uk[0, n) (ascending) whose key is >= key; *at gets that
// key (the search has read it) when the index is below n.  Probes are
// placed by interpolation on the key values (the bucket keys of 64-bit
// digests are spread evenly over the key range); after a probe that leaves
// more than half of the range, the next one bisects, so a search takes at
// most about twice the probes of plain bisection.
__device__ __forceinline__ int64_t lower_bound_keys(const uint64_t *uk, int64_t n, uint64_t key,
                                                    uint64_t *at)
{
    if (n == 0)
        return 0;
    uint64_t klo = uk[0], khi = uk[n - 1];
    if (key <= klo) {
        *at = klo;
        return 0;
    }
    if (key > khi)
        return n;
    int64_t lo = 0, hi = n - 1; // uk[lo] < key <= uk[hi]: the answer is in (lo, hi]
    bool bisect = false;
    while (hi - lo > 1) {
        const int64_t len = hi - lo;
        int64_t mid;
        if (bisect) {
            mid = lo + (len >> 1);
        } else {
            const double f = (double)(key - klo) / (double)(khi - klo);
            mid = lo + (int64_t)(f * (double)len);
            mid = max(lo + 1, min(hi - 1, mid));
        }
        const uint64_t km = uk[mid];
        if (km < key) {
            lo = mid;
            klo = km;
        } else {
            hi = mid;
            khi = km;
        }
        bisect = !bisect && 2 * (hi - lo) > len;
    }
    *at = khi;
    return hi;
}

// Bitonic sort of n <= 256 keys in LDS by one wave in registers: element e =
// 4 * lane + r is v[r] of the lane (keys past n sort last as ~0).  The
// network always spans 256 elements; the steps with j >= 4 exchange with
// lane ^ (j / 4), the others within the lane, and none needs a workgroup
// barrier.
__device__ __forceinline__ void wave_bitonic256(uint64_t *s, int n)
{
    const int lane = lane_id();
    uint64_t v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = 4 * lane + r;
        v[r] = e < n ? s[e] : ~0ull;
    }
#pragma unroll
    for (int k = 2; k <= 4 * kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = 4 * lane + r;
                    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v[r], j >> 2, kWave);
                    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v[r] >> 32), j >> 2, kWave);
                    const uint64_t y = ((uint64_t)hi << 32) | lo;
                    const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                    const bool y_less = y < v[r];
                    v[r] = keep_min == y_less ? y : v[r];
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if ((r & j) == 0) {
                        const bool asc = ((4 * lane + r) & k) == 0;
                        const uint64_t x = v[r], y = v[r | j];
                        const bool swap = asc ? (y < x) : (x < y);
                        v[r] = swap ? y : x;
                        v[r | j] = swap ? x : y;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = 4 * lane + r;
        if (e < n)
            s[e] = v[r];
    }
}

// Bitonic sort of n (power of two) 64-bit keys in LDS, ascending, whole
// block, one workgroup barrier per step.
__device__ void block_bitonic(uint64_t *s, int n)
{
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t x = s[i], y = s[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        s[i] = y;
                        s[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Bitonic sort of n keys (a power of two, 512 .. 256 * QW * CPW) in LDS by
// the whole block with the keys in registers: wave w holds the chunks w,
// w + QW, ... of 256 keys (key e = 256 chunk + 4 lane + r in v[c][r]).  The
// compare-exchange steps of distance below 256 stay inside a chunk and run
// in registers (lane exchanges for distances 4 .. 128, within the lane
// below 4); only the steps of distance 256 and more pass through LDS, two
// workgroup barriers each: 6 steps for 2048 keys and 10 for 4096, where the
// plain network has 66 and 78 barriers.
template <int QW, int CPW>
__device__ void block_bitonic_regs(uint64_t *s, int n)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int nch = n >> 8;
    uint64_t v[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int ch = wid + c * QW;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            v[c][r] = ch < nch ? s[256 * ch + 4 * lane + r] : 0ull;
    }
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 256) {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    if (wid + c * QW < nch) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            s[256 * (wid + c * QW) + 4 * lane + r] = v[c][r];
                    }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    if (wid + c * QW < nch) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int e = 256 * (wid + c * QW) + 4 * lane + r;
                            const uint64_t y = s[e ^ j];
                            const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                            v[c][r] = keep_min == (y < v[c][r]) ? y : v[c][r];
                        }
                    }
                __syncthreads();
            } else if (j >= 4) {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    if (wid + c * QW < nch) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int e = 256 * (wid + c * QW) + 4 * lane + r;
                            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v[c][r], j >> 2, kWave);
                            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v[c][r] >> 32), j >> 2, kWave);
                            const uint64_t y = ((uint64_t)hi << 32) | lo;
                            const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                            v[c][r] = keep_min == (y < v[c][r]) ? y : v[c][r];
                        }
                    }
            } else {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    if (wid + c * QW < nch) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if ((r & j) == 0) {
                                const bool asc = ((256 * (wid + c * QW) + 4 * lane + r) & k) == 0;
                                const uint64_t x = v[c][r], y = v[c][r | j];
                                const bool swap = asc ? (y < x) : (x < y);
                                v[c][r] = swap ? y : x;
                                v[c][r | j] = swap ? x : y;
                            }
                        }
                    }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        if (wid + c * QW < nch) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                s[256 * (wid + c * QW) + 4 * lane + r] = v[c][r];
        }
    __syncthreads();
}

// Ascending sort of n (a power of two, at most 512 * QW) keys in LDS: the
// first wave alone when n <= 256, else the whole block with the keys in
// registers, CPW chunks of 256 per wave (the batch workgroup, short of
// registers, holds one and sorts larger sets with one barrier per step).
// Every thread calls; ends with a workgroup barrier.
template <int QW, int CPW>
__device__ __forceinline__ void sort_keys(uint64_t *s, int n)
{
    if (n <= 4 * kWave) {
        if (threadIdx.x < kWave)
            wave_bitonic256(s, n);
        __syncthreads();
    } else if (n <= 256 * QW * CPW) {
        block_bitonic_regs<QW, CPW>(s, n);
    } else {
        block_bitonic(s, n);
    }
}

template <int QW>
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t *red)
{
    v = wave_sum(v);
    if (lane_id() == 0)
        red[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < QW; ++w)
        t += red[w];
    __syncthreads();
    return t;
}

template <int QW>
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, uint32_t *red)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
    if (lane_id() == 0)
        red[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < QW; ++w)
        t = max(t, red[w]);
    __syncthreads();
    return t;
}

// Exclusive prefix of v over the block (thread order); *total gets the sum.
template <int QW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *red, uint32_t *total)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o)
            incl += u;
    }
    if (lane == kWave - 1)
        red[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int w = 0; w < QW; ++w) {
        off += w < wid ? red[w] : 0;
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

constexpr int kWinBins = 256;

// The bound of a window when the rem remaining (bucket, id) entries exceed
// the capacity: with lo the smallest remaining id and [lo, hi] the range
// still in question, a histogram of the remaining ids over kWinBins equal
// parts of the range gives the largest part boundary below which at most
// kCap entries lie.  If the first part alone holds more, the range narrows
// to it and the count is repeated (at most four times: the part width falls
// 256-fold each time, and one id value has at most nl <= kCap entries, one
// per list, so a single-id part always fits).  Entries are spread over the
// threads through the prefix of the lists' remaining counts (lst_pre /
// lst_take, rewritten by the caller afterwards).
template <int QT>
__device__ void window_bound(const QueryArgs &a, int nl, uint32_t rem, const uint32_t *lst_cur,
                             const uint32_t *lst_end, uint32_t *lst_pre, uint32_t *lst_take,
                             uint32_t *hist, uint32_t *red, uint32_t *out)
{
    constexpr int QW = QT / kWave;
    constexpr int kCap = QShape<QT>::cap;
    const int tid = threadIdx.x;
    // smallest and largest remaining id (each list ascends)
    uint32_t mn = 0, mx = 0;
    for (int li = tid; li < nl; li += QT) {
        if (lst_cur[li] < lst_end[li]) {
            const int sg = li / a.L, t = li % a.L;
            const uint32_t *ids = a.seg[sg].ids + (int64_t)t * a.seg[sg].n;
            mn = max(mn, ~ids[lst_cur[li]]);
            mx = max(mx, ids[lst_end[li] - 1u]);
        }
        lst_take[li] = lst_end[li] - lst_cur[li];
    }
    const uint32_t lo = ~block_max_u32<QW>(mn, red);
    uint32_t hi = block_max_u32<QW>(mx, red);
    {
        const int per = (nl + QT - 1) / QT;
        const int l0 = tid * per, l1 = l0 + per < nl ? l0 + per : nl;
        uint32_t mine = 0;
        for (int li = l0; li < l1; ++li)
            mine += lst_take[li];
        uint32_t tot;
        uint32_t run = block_excl_scan<QW>(mine, red, &tot);
        for (int li = l0; li < l1; ++li) {
            lst_pre[li] = run;
            run += lst_take[li];
        }
    }
    __syncthreads();
    while (true) {
        // parts of width wid (64-bit: the range may span all 2^32 ids)
        const uint64_t span = (uint64_t)hi - lo + 1u;
        const uint64_t wid = (span + kWinBins - 1) / kWinBins;
        for (int i = tid; i < kWinBins; i += QT)
            hist[i] = 0;
        __syncthreads();
        for (uint32_t e = tid; e < rem; e += QT) {
            int l0 = 0, l1 = nl; // the list holding entry e: last li with pre[li] <= e
            while (l1 - l0 > 1) {
                const int mid = (l0 + l1) >> 1;
                if (lst_pre[mid] <= e)
                    l0 = mid;
                else
                    l1 = mid;
            }
            while (lst_take[l0] == 0 || lst_pre[l0] + lst_take[l0] <= e)
                ++l0;
            const int sg = l0 / a.L, t = l0 % a.L;
            const uint32_t id =
                a.seg[sg].ids[(int64_t)t * a.seg[sg].n + lst_cur[l0] + (e - lst_pre[l0])];
            if (id <= hi)
                atomicAdd(&hist[(uint32_t)(((uint64_t)id - lo) / wid)], 1u);
        }
        __syncthreads();
        if (tid < kWave) {
            // one wave scans the parts: lane l holds parts 4l .. 4l + 3
            const int lane = lane_id();
            uint32_t c[4], s4 = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                c[r] = hist[4 * lane + r];
                s4 += c[r];
            }
            uint32_t incl = s4;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t u = __shfl_up(incl, o, kWave);
                if (lane >= o)
                    incl += u;
            }
            // parts b with (entries below part b) <= kCap: the largest is the bound
            uint32_t run = incl - s4, best = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                run += c[r];
                if (run <= (uint32_t)kCap)
                    best = 4 * lane + r + 1;
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1)
                best = max(best, (uint32_t)__shfl_xor((int)best, o, kWave));
            if (lane == 0)
                red[0] = best;
        }
        __syncthreads();
        const uint32_t b = red[0];
        __syncthreads();
        if (b > 0) {
            // ids below lo + b * wid: at most kCap entries, at least the first
            // part's; never above hi + 1 (every counted id is at most hi, and
            // ids stay below 2^32 - 1, so the bound is not the all-ids mark)
            if (tid == 0)
                *out = (uint32_t)min((uint64_t)lo + b * wid, (uint64_t)hi + 1u);
            __syncthreads();
            return;
        }
        hi = (uint32_t)((uint64_t)lo + wid - 1u); // the first part alone overflows: narrow to it
    }
}

template <int QT>
__global__ __launch_bounds__(QT) __attribute__((amdgpu_waves_per_eu(QShape<QT>::wpe))) void
query_kernel(QueryArgs a)
{
    constexpr int QW = QT / kWave;
    constexpr int kCap = QShape<QT>::cap;
    constexpr int kSortCap = sort_cap<QT>();
    extern __shared__ __align__(16) unsigned char lds[];
    const int nlp = (a.nseg * a.L + 4) & ~3; // list arrays, lst_pre's extra entry included
    float *qv = (float *)lds;                                          // [d]
    uint32_t *lst_start = (uint32_t *)(lds + ((a.d * 4 + 15) & ~15));  // [nl]
    uint32_t *lst_cur = lst_start + nlp;                               // [nl]
    uint32_t *lst_end = lst_cur + nlp;                                 // [nl]
    uint32_t *lst_pre = lst_end + nlp;                                 // [nl + 1]
    uint32_t *lst_take = lst_pre + nlp;                                // [nl]
    uint64_t *sbuf = (uint64_t *)(((uintptr_t)(lst_take + nlp) + 15) & ~(uintptr_t)15); // [kSortCap]
    uint64_t *topk = sbuf + kSortCap;                                  // [kMaxK]
    uint32_t *cand = (uint32_t *)(topk + kMaxK);                       // [kCap]
    __shared__ uint32_t red[QW];
    __shared__ float s_qnorm;
    __shared__ int s_kcur;
    __shared__ uint32_t s_ncand, s_hi, s_wcount, s_ucount;
    __shared__ uint32_t s_hist[kWinBins];

    const int q = blockIdx.x / a.split, share = blockIdx.x % a.split;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int nl = a.nseg * a.L;

    // query row -> LDS, and its norm
    float part = 0.0f;
    for (int j = tid; j < a.d; j += QT) {
        float v = load_val(a.qx, a.qdt, a.qscale, q, a.qld, j);
        qv[j] = v;
        part += v * v;
    }
    part = wave_sum(part);
    if (lane == 0)
        red[wid] = __float_as_uint(part);
    __syncthreads();
    if (tid == 0) {
        float t = 0.0f;
        for (int w = 0; w < QW; ++w)
            t += __uint_as_float(red[w]);
        s_qnorm = sqrtf(t);
        s_kcur = 0;
        s_ncand = 0;
    }

    // probe: bucket of the query key in every (segment, table)
    for (int li = tid; li < nl; li += QT) {
        int sg = li / a.L, t = li % a.L;
        const QSeg &S = a.seg[sg];
        uint64_t key = a.qkeys[(int64_t)t * a.qkey_ld + q];
        const uint64_t *uk = S.ukeys + (int64_t)t * S.n;
        const int64_t nu = S.nuniq[t];
        uint64_t kat = 0;
        const int64_t lo = lower_bound_keys(uk, nu, key, &kat);
        uint32_t st = 0, en = 0;
        if (lo < nu && kat == key) {
            const uint32_t *of = S.offs + (int64_t)t * (S.n + 1);
            st = of[lo];
            en = of[lo + 1];
            // ids of a bucket ascend: drop the tail at or above the watermark
            // (none when the whole segment lies below it)
            const uint32_t *ids = S.ids + (int64_t)t * S.n;
            if (S.id_end > (int64_t)a.watermark && ids[en - 1] >= a.watermark)
                en = lower_bound_u32(ids, st, en, a.watermark);
        }
        lst_start[li] = st;
        lst_cur[li] = st;
        lst_end[li] = en;
    }
    __syncthreads();

    const float qn = s_qnorm;
    while (true) {
        // remaining entries
        uint32_t rem = 0;
        for (int li = tid; li < nl; li += QT)
            rem += lst_end[li] - lst_cur[li];
        rem = block_sum_u32<QW>(rem, red);
        if (rem == 0)
            break;
        // window [.., hi): all remaining if they fit, else an id bound whose
        // entry count fits kCap, from histograms of the remaining entries' ids
        if (tid == 0)
            s_hi = 0xffffffffu;
        __syncthreads();
        if (rem > kCap)
            window_bound<QT>(a, nl, rem, lst_cur, lst_end, lst_pre, lst_take, s_hist, red, &s_hi);
        const uint32_t hiv = s_hi;
        for (int li = tid; li < nl; li += QT) {
            int sg = li / a.L, t = li % a.L;
            const uint32_t *ids = a.seg[sg].ids + (int64_t)t * a.seg[sg].n;
            uint32_t e = hiv == 0xffffffffu ? lst_end[li]
                                            : lower_bound_u32(ids, lst_cur[li], lst_end[li], hiv);
            lst_take[li] = e - lst_cur[li];
        }
        __syncthreads();
        {
            // prefix of the per-list counts: thread owns a contiguous run of lists
            const int per = (nl + QT - 1) / QT;
            const int l0 = tid * per, l1 = l0 + per < nl ? l0 + per : nl;
            uint32_t mine = 0;
            for (int li = l0; li < l1; ++li)
                mine += lst_take[li];
            uint32_t tot;
            uint32_t run = block_excl_scan<QW>(mine, red, &tot);
            for (int li = l0; li < l1; ++li) {
                lst_pre[li] = run;
                run += lst_take[li];
            }
            if (tid == 0) {
                lst_pre[nl] = tot;
                s_wcount = tot;
            }
        }
        __syncthreads();
        const uint32_t wc = s_wcount;
        // id of window entry e (e < wc): the list holding it is the last li
        // with pre[li] <= e
        auto entry_id = [&](uint32_t e) {
            int lo = 0, hi = nl;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (lst_pre[mid] <= e)
                    lo = mid;
                else
                    hi = mid;
            }
            while (lst_take[lo] == 0 || lst_pre[lo] + lst_take[lo] <= e)
                ++lo;
            int sg = lo / a.L, t = lo % a.L;
            return a.seg[sg].ids[(int64_t)t * a.seg[sg].n + lst_cur[lo] + (e - lst_pre[lo])];
        };
        // the window's ids; a split query's workgroup keeps the ids that are
        // its own (id % split == share), compacted in order
        uint32_t wm = wc;
        if (a.split > 1) {
            constexpr int kPer = (kCap + QT - 1) / QT; // wc <= kCap
            const uint32_t per = (wc + QT - 1) / QT;
            const uint32_t e0 = (uint32_t)tid * per;
            uint32_t idv[kPer];
            uint32_t nk = 0;
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const uint32_t e = e0 + (uint32_t)i;
                idv[i] = ~0u;
                if ((uint32_t)i < per && e < wc) {
                    const uint32_t id = entry_id(e);
                    if (id % (uint32_t)a.split == (uint32_t)share) {
                        idv[i] = id;
                        ++nk;
                    }
                }
            }
            uint32_t tot;
            uint32_t pos = block_excl_scan<QW>(nk, red, &tot);
#pragma unroll
            for (int i = 0; i < kPer; ++i)
                if (idv[i] != ~0u)
                    sbuf[pos++] = idv[i];
            wm = tot;
        } else {
            for (uint32_t e = tid; e < wc; e += QT)
                sbuf[e] = entry_id(e);
        }
        int p2 = 1;
        while (p2 < (int)wm)
            p2 <<= 1;
        for (uint32_t e = wm + tid; e < (uint32_t)p2; e += QT)
            sbuf[e] = ~0ull;
        __syncthreads();
        for (int li = tid; li < nl; li += QT)
            lst_cur[li] += lst_take[li];
        sort_keys<QW, QShape<QT>::sort_cpw>(sbuf, p2);
        {
            // distinct ids, compacted in order: thread owns a contiguous run
            const int per = (p2 + QT - 1) / QT;
            const int e0 = tid * per, e1 = e0 + per < (int)wm ? e0 + per : (int)wm;
            uint32_t mine = 0;
            for (int e = e0; e < e1; ++e)
                mine += (e == 0 || sbuf[e] != sbuf[e - 1]);
            uint32_t tot;
            uint32_t pos = block_excl_scan<QW>(mine, red, &tot);
            for (int e = e0; e < e1; ++e)
                if (e == 0 || sbuf[e] != sbuf[e - 1])
                    cand[pos++] = (uint32_t)sbuf[e];
            if (tid == 0) {
                s_ucount = tot;
                s_ncand += tot;
            }
        }
        __syncthreads();
        const uint32_t uc = s_ucount;
        // score: a wave takes NR candidates c, c + QW, ... together
        // (their loads overlap); those past the end repeat c
        auto score_all = [&](auto nr_tag, auto scorer) {
            constexpr int NR = decltype(nr_tag)::value;
            for (uint32_t c = wid; c < uc; c += NR * QW) {
                int64_t row[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    row[r] = cand[c + r * QW < uc ? c + r * QW : c];
                float acc[NR], xx[NR];
                scorer(row, acc, xx);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const float ac = wave_sum(acc[r]), xs = wave_sum(xx[r]);
                    float sc;
                    if (a.metric == LSH_E2LSH) {
                        sc = sqrtf(ac);
                    } else {
                        const float xn = sqrtf(xs);
                        const float cs = (qn > 0.0f && xn > 0.0f) ? ac / (qn * xn) : 0.0f;
                        sc = 1.0f - cs;
                    }
                    if (lane == 0 && c + r * QW < uc)
                        sbuf[c + r * QW] =
                            ((uint64_t)__float_as_uint(fmaxf(sc, 0.0f)) << 32) | (uint64_t)row[r];
                }
            }
        };
        constexpr int NRV = QShape<QT>::nr;
        using nrv = std::integral_constant<int, NRV>;
        using nr2 = std::integral_constant<int, 2>;
        if (a.vec4)
            score_all(nrv{}, [&](const int64_t (&row)[NRV], float (&acc)[NRV], float (&xx)[NRV]) {
                score_rows_v4<NRV>(a, qv, row, acc, xx);
            });
        else if (a.bdt == LSH_F32)
            score_all(nr2{}, [&](const int64_t (&row)[2], float (&acc)[2], float (&xx)[2]) {
                score_rows<LSH_F32, 2>(a, qv, row, acc, xx);
            });
        else if (a.bdt == LSH_BF16)
            score_all(nr2{}, [&](const int64_t (&row)[2], float (&acc)[2], float (&xx)[2]) {
                score_rows<LSH_BF16, 2>(a, qv, row, acc, xx);
            });
        else
            score_all(nr2{}, [&](const int64_t (&row)[2], float (&acc)[2], float (&xx)[2]) {
                score_rows<LSH_FP8_E4M3FN, 2>(a, qv, row, acc, xx);
            });
        __syncthreads();
        // merge with the running top-k
        const int kc = s_kcur;
        int tot = (int)uc + kc;
        int m2 = 1;
        while (m2 < tot)
            m2 <<= 1;
        for (int e = tid; e < m2; e += QT) {
            if (e >= (int)uc)
                sbuf[e] = e < tot ? topk[e - uc] : ~0ull;
        }
        __syncthreads();
        sort_keys<QW, QShape<QT>::sort_cpw>(sbuf, m2);
        int nk = tot < a.k ? tot : a.k;
        for (int e = tid; e < nk; e += QT)
            topk[e] = sbuf[e];
        __syncthreads();
        if (tid == 0)
            s_kcur = nk;
        __syncthreads();
    }

    const int kc = s_kcur;
    if (a.split > 1) {
        // this share's top-k (entries past it are ~0, which sort last) and its
        // count of distinct candidates, for the merge kernel
        uint64_t *mp = a.part + ((int64_t)q * a.split + share) * a.k;
        for (int r = tid; r < a.k; r += QT)
            mp[r] = r < kc ? topk[r] : ~0ull;
        if (tid == 0)
            a.pcount[(int64_t)q * a.split + share] = s_ncand;
        return;
    }
    for (int r = tid; r < a.k; r += QT) {
        int64_t id = -1;
        float sc = INFINITY;
        if (r < kc) {
            id = (int64_t)(uint32_t)topk[r];
            sc = __uint_as_float((uint32_t)(topk[r] >> 32));
        }
        a.ids[(int64_t)q * a.k + r] = id;
        if (a.score)
            a.score[(int64_t)q * a.k + r] = sc;
    }
    if (tid == 0 && a.ncand)
        a.ncand[q] = (int32_t)s_ncand;
}

// The k best of a query's split * k share entries (distinct, except the ~0
// padding: the shares hold disjoint ids): entry i goes to rank
// #{j : e_j < e_i, or e_j == e_i and j < i}.  The query's candidate count is
// the sum of the shares'.  One workgroup per query, one thread per entry
// (split * k <= 256).
__global__ __launch_bounds__(256) void query_merge_kernel(const uint64_t *part,
                                                          const uint32_t *pcount, int split, int k,
                                                          int64_t *ids, float *score,
                                                          int32_t *ncand)
{
    __shared__ uint64_t e[kQuerySplit * kMaxK];
    const int q = blockIdx.x, n = split * k, i = threadIdx.x;
    if (i < n)
        e[i] = part[(int64_t)q * n + i];
    if (i == 0 && ncand) {
        uint32_t c = 0;
        for (int j = 0; j < split; ++j)
            c += pcount[(int64_t)q * split + j];
        ncand[q] = (int32_t)c;
    }
    __syncthreads();
    if (i >= n)
        return;
    const uint64_t v = e[i];
    int rank = 0;
    for (int j = 0; j < n; ++j)
        rank += (e[j] < v || (e[j] == v && j < i)) ? 1 : 0;
    if (rank < k) {
        const bool pad = v == ~0ull;
        ids[(int64_t)q * k + rank] = pad ? -1 : (int64_t)(uint32_t)v;
        if (score)
            score[(int64_t)q * k + rank] = pad ? INFINITY : __uint_as_float((uint32_t)(v >> 32));
    }
}

// Workspace of a split batch: the shares' top-k lists [nq][kQuerySplit][k],
// then their candidate counts [nq][kQuerySplit].
size_t query_ws_bytes(int64_t nq, int32_t k)
{
    if (nq < 1 || nq > kSplitQueries || k < 1 || k > kMaxK)
        return 0;
    return (size_t)nq * kQuerySplit * ((size_t)k * 8 + 4);
}

} // namespace lsh

extern "C" size_t lsh_query_workspace_bytes(int64_t nq, int32_t k)
{
    return lsh::query_ws_bytes(nq, k);
}

extern "C" lsh_status lsh_query(const lsh_index *const *segs, int32_t nseg, const lsh_points *base,
                                const lsh_points *Q, const uint64_t *qkeys, int64_t qkey_ld,
                                int32_t k, int64_t id_watermark, int32_t metric, int64_t *ids,
                                float *score, int32_t *ncand, void *workspace, size_t ws_bytes,
                                void *stream)
{
    using namespace lsh;
    if (!segs || nseg < 1 || nseg > kMaxSeg)
        LSH_FAIL(LSH_EINVAL, "need 1..%d index segments", kMaxSeg);
    if (!base || !Q || !ids)
        LSH_FAIL(LSH_EINVAL, "base, Q and ids are required");
    if (k < 1 || k > kMaxK)
        LSH_FAIL(LSH_EINVAL, "k must be in 1..%d", kMaxK);
    if (metric != LSH_E2LSH && metric != LSH_SRP)
        LSH_FAIL(LSH_EINVAL, "unknown metric %d", metric);
    lsh_status st;
    if ((st = check_points(base)) != LSH_OK || (st = check_points(Q)) != LSH_OK)
        return st;
    if (base->d != Q->d)
        LSH_FAIL(LSH_EINVAL, "base d=%d differs from query d=%d", base->d, Q->d);
    if (Q->d > 16384)
        LSH_FAIL(LSH_EINVAL, "query supports d <= 16384");
    if (Q->n == 0)
        return LSH_OK;
    if (!qkeys)
        LSH_FAIL(LSH_EINVAL, "qkeys is NULL");
    if (qkey_ld == 0)
        qkey_ld = Q->n;
    if (qkey_ld < Q->n)
        LSH_FAIL(LSH_EINVAL, "qkey_ld < number of queries");

    QueryArgs a = {};
    a.nseg = nseg;
    a.L = -1;
    int64_t maxid = 0;
    for (int s = 0; s < nseg; ++s) {
        lsh_index_view v;
        if (!segs[s] || lsh_index_get_view(segs[s], &v) != LSH_OK)
            LSH_FAIL(LSH_EINVAL, "segment %d is NULL", s);
        if (a.L < 0)
            a.L = v.L;
        if (v.L != a.L)
            LSH_FAIL(LSH_EINVAL, "segments have different L");
        a.seg[s].ids = v.sorted_ids;
        a.seg[s].ukeys = v.ukeys;
        a.seg[s].offs = v.offs;
        a.seg[s].nuniq = v.nuniq;
        a.seg[s].n = v.n;
        a.seg[s].id_end = v.id_base + v.n;
        if (v.id_base + v.n > maxid)
            maxid = v.id_base + v.n;
    }
    if ((int64_t)nseg * a.L > kMaxLists)
        LSH_FAIL(LSH_EINVAL, "nseg * L = %lld exceeds %d", (long long)nseg * a.L, kMaxLists);
    int64_t wm = id_watermark < maxid ? id_watermark : maxid;
    if (wm < 0)
        wm = 0;
    if (wm > base->n)
        LSH_FAIL(LSH_EINVAL, "indexed ids reach %lld but base holds %lld points",
                 (long long)wm, (long long)base->n);
    a.bx = base->x;
    a.bdt = base->dtype;
    a.bscale = base->row_scale;
    a.bld = base->ld;
    a.bn = base->n;
    a.qx = Q->x;
    a.qdt = Q->dtype;
    a.qscale = Q->row_scale;
    a.qld = Q->ld;
    a.d = Q->d;
    a.qkeys = qkeys;
    a.qkey_ld = qkey_ld;
    a.k = k;
    a.watermark = (uint32_t)wm;
    a.metric = metric;
    a.vec4 = base->dtype == LSH_F32 && ((uintptr_t)base->x & 15u) == 0 && base->ld % 4 == 0 &&
             Q->d % 4 == 0;
    a.ids = ids;
    a.score = score;
    a.ncand = ncand;
    // a batch that leaves CUs idle scores each query with several workgroups
    // when a workspace is given
    const int cus = device_cu_count();
    a.split = 1;
    if (workspace && Q->n <= kSplitQueries) {
        const size_t need = query_ws_bytes(Q->n, k);
        if (ws_bytes < need || ((uintptr_t)workspace & 255))
            LSH_FAIL(LSH_ENOMEM, "query workspace needs %zu bytes (256-aligned), got %zu", need,
                     ws_bytes);
        // up to four ways while the split grid keeps one workgroup per CU (the
        // 8-wave shape); batches of more queries than CUs run the 4-wave shape
        // either way and gain from halving their heaviest queries' scoring
        a.split = Q->n <= cus ? (int32_t)std::min<int64_t>(kQuerySplit, cus / Q->n) : 2;
        a.part = (uint64_t *)workspace;
        a.pcount = (uint32_t *)(a.part + (size_t)Q->n * kQuerySplit * k);
    }
    const int64_t nwg = Q->n * a.split;
    const bool solo = nwg <= cus;
    const int nl = nseg * a.L;
    const size_t lds = solo ? query_lds_bytes<kQThreadsSolo>(Q->d, nl)
                            : query_lds_bytes<kQThreads>(Q->d, nl);
    const void *fn = solo ? (const void *)query_kernel<kQThreadsSolo>
                          : (const void *)query_kernel<kQThreads>;
    LSH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (solo)
        hipLaunchKernelGGL(query_kernel<kQThreadsSolo>, dim3((unsigned)nwg), dim3(kQThreadsSolo),
                           lds, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(query_kernel<kQThreads>, dim3((unsigned)nwg), dim3(kQThreads), lds,
                           (hipStream_t)stream, a);
    LSH_LAUNCHED("query_kernel");
    if (a.split > 1) {
        hipLaunchKernelGGL(query_merge_kernel, dim3((unsigned)Q->n), dim3(256), 0,
                           (hipStream_t)stream, (const uint64_t *)a.part,
                           (const uint32_t *)a.pcount, a.split, k, ids, score, ncand);
        LSH_LAUNCHED("query_merge_kernel");
    }
    return LSH_OK;
}
