// Count-sketch and higher-order count-sketch LSH hashing on gfx950.
//
// One fused, HBM-bound kernel per call: stream the rows of X once, scatter
// every coordinate into its sketch bin (count sketch, Section 3.2 Eq. eq_cs;
// the higher-order count sketch of Eq. eqhcs is the same scatter under the
// composite bin of the per-mode hashes), discretise the m bins
// (floor((sqrt(m) y + b)/w), Definitions CS_Eucl_LSH / HCS_Eucl_LSH, or
// sgn(y), Definitions cs_consine_lsh / hcs_consine_lsh), and fold each table's
// K codes into its 64-bit bucket key (Section 3.1).
//
// Work decomposition:
//   * a workgroup of W waves shares the packed hash table (one 16-bit entry
//     per coordinate: bin << 1 | sign) in LDS, built once per workgroup from
//     h/s (CS) or from the per-mode tables (HCS);
//   * each wave owns blocks of RB consecutive rows and keeps m FP32 bins of
//     its own in LDS; a row is streamed in 16-byte chunks, chunk c of the row
//     always goes to lane c mod 64, and the next chunk group is loaded before
//     the current one is scattered (two register buffers);
//   * after a row, the wave discretises its bins (E2LSH: one lane per table;
//     SRP: one lane per component plus ballots), and stages the L keys of
//     its RB rows in LDS so the key stores leave as 8-key (64-byte) runs.
// The optional FP64 recheck recomputes, in ascending coordinate order, any
// component whose FP32 value lies within the rounding-error bound
// gamma_{c-1} * sum|terms| of a bin edge (or of zero for SRP).

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "lsh_internal.h"

namespace lsh {

constexpr int kRowsPerBlock = 8;  // RB: rows a wave hashes before writing keys
constexpr int kChunksPerLane = 4; // 16-byte chunks per lane per load group
constexpr int kMaxModes = 8;

__host__ __device__ constexpr int align16(int v) { return (v + 15) & ~15; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct HashArgs {
    const void *x;
    int64_t ld;
    int64_t n;
    int32_t d;
    const float *row_scale;
    int32_t m, K, L;
    float alpha32;  // sqrt(m) (1 for dense-style scaling, unused here)
    float inv_w32;
    float w32;
    int32_t w_pow2; // 1 when w is a power of two, so /w == *(1/w) exactly
    double alpha64, w64, inv_w64;
    const float *b;
    uint64_t *keys;
    int64_t key_ld;
    int32_t *codes;
    float *proj;
    unsigned long long *counters;
    // hash source: CS (h, s) or HCS (per-mode tables)
    int32_t hcs;
    const uint32_t *h;
    const int8_t *s;
    int32_t N;
    int32_t dk[kMaxModes], mk[kMaxModes], mode_off[kMaxModes];
    const uint32_t *hk;
    const int8_t *sk;
    // recheck support (workspace)
    const uint32_t *csr_off;
    const uint32_t *csr_idx;
    const uint32_t *cmax;
    // layout
    int32_t waves;       // waves per workgroup
    int32_t tab_bytes;   // LDS bytes of the hash table (aligned)
    int32_t mpad;        // bins per wave, padded to a multiple of 256
    int32_t wave_bytes;  // LDS bytes per wave
};

// Bin/sign entry of coordinate j: bin << 1 | (sign < 0).
__device__ __forceinline__ uint32_t table_entry(const HashArgs &a, int32_t j, bool &bad)
{
    uint32_t bin;
    uint32_t neg;
    if (!a.hcs) {
        bin = a.h[j];
        neg = a.s[j] < 0;
    } else {
        // tensor index (i_1, ..., i_N) of j, first mode fastest (Eq. eqhcs)
        int32_t rest = j;
        uint32_t stride = 1;
        bin = 0;
        neg = 0;
        for (int k = 0; k < a.N; ++k) {
            int32_t ik = rest % a.dk[k];
            rest /= a.dk[k];
            uint32_t hb = a.hk[a.mode_off[k] + ik];
            if (hb >= (uint32_t)a.mk[k]) {
                bad = true;
                hb = 0;
            }
            bin += hb * stride;
            stride *= (uint32_t)a.mk[k];
            neg ^= a.sk[a.mode_off[k] + ik] < 0;
        }
    }
    if (bin >= (uint32_t)a.m) {
        bad = true;
        bin = 0;
    }
    return (bin << 1) | neg;
}

// ----------------------------------------------------------------- decoding

template <int DT> struct Elem;
template <> struct Elem<LSH_F32> {
    using T = float;
    static constexpr int per16 = 4;
};
template <> struct Elem<LSH_BF16> {
    using T = uint16_t;
    static constexpr int per16 = 8;
};
template <> struct Elem<LSH_FP8_E4M3FN> {
    using T = uint8_t;
    static constexpr int per16 = 16;
};

// OCP E4M3FN -> FP32.  The 7 magnitude bits shifted to bits 20..26 form an
// FP32 number whose exponent is the FP8 exponent re-biased by 120 (normal
// values) or an FP32 subnormal holding mantissa * 2^-129 (FP8 subnormals);
// scaling by 2^120 restores both exactly.  (The NaN pattern is not
// special-cased: quantised data never holds it.)
__device__ __forceinline__ float fp8_to_f32(uint32_t byte)
{
    float mag = __uint_as_float((byte & 0x7fu) << 20) * 0x1.0p120f;
    return __uint_as_float(__float_as_uint(mag) | ((byte & 0x80u) << 24));
}

// Element e of a 16-byte chunk.
template <int DT> __device__ __forceinline__ float elem_value(u32x4 v, int e)
{
    uint32_t word = v[e / (Elem<DT>::per16 / 4)];
    if constexpr (DT == LSH_F32) {
        return __uint_as_float(word);
    } else if constexpr (DT == LSH_BF16) {
        return __uint_as_float((e & 1) ? (word & 0xffff0000u) : (word << 16));
    } else {
        return fp8_to_f32((word >> (8 * (e & 3))) & 0xffu);
    }
}

// Value of one element given its bit pattern in the low bits of u.
template <int DT> __device__ __forceinline__ float bits_value(uint32_t u)
{
    if constexpr (DT == LSH_F32)
        return __uint_as_float(u);
    else if constexpr (DT == LSH_BF16)
        return __uint_as_float((u & 0xffffu) << 16);
    else
        return fp8_to_f32(u & 0xffu);
}

template <int DT> __device__ __forceinline__ float scalar_value(const void *x, int64_t idx)
{
    if constexpr (DT == LSH_F32) {
        return ((const float *)x)[idx];
    } else if constexpr (DT == LSH_BF16) {
        return __uint_as_float((uint32_t)((const uint16_t *)x)[idx] << 16);
    } else {
        return fp8_to_f32(((const uint8_t *)x)[idx]);
    }
}

// --------------------------------------------------------------- LDS layout

struct WaveLds {
    float *bins;     // [mpad]
    float *absb;     // [mpad] (recheck only)
    uint64_t *stage; // [L * RB]
    uint64_t *mask;  // [ceil(m/64)] (SRP)
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------- the epilogue

// gamma_{c-1} for FP32 recursive summation of c terms, plus slack.
__device__ __forceinline__ double sum_gamma(uint32_t c)
{
    const double u = 0x1.0p-24;
    double k = c > 1 ? (double)(c - 1) : 0.0;
    return k * u / (1.0 - k * u) * (1.0 + 1e-9);
}

// Exact FP64 value of component l of row `row`, summed in ascending
// coordinate order exactly as an FP64 evaluation of the definition would.
template <int DT>
__device__ double exact_component(const HashArgs &a, const uint16_t *tab, int64_t row, double scale,
                                  int32_t l)
{
    double y = 0.0;
    uint32_t p0 = a.csr_off[l], p1 = a.csr_off[l + 1];
    for (uint32_t p = p0; p < p1; ++p) {
        uint32_t j = a.csr_idx[p];
        double xv = __dmul_rn(scale, (double)scalar_value<DT>(a.x, row * a.ld + j));
        y = __dadd_rn(y, (tab[j] & 1u) ? -xv : xv);
    }
    return y;
}

template <int DT, bool RECHECK>
__device__ __forceinline__ int32_t e2lsh_code(const HashArgs &a, const uint16_t *tab, const WaveLds &w,
                                              const float *bl, int64_t row, float scale, double gam,
                                              int32_t l, bool count, unsigned &nflag,
                                              unsigned &nchg, unsigned &nsat)
{
    float y = w.bins[l];
    double cd;
    if constexpr (!RECHECK) {
        float v = fmaf(a.alpha32 * scale, y, bl[l]);
        float c = a.w_pow2 ? floorf(v * a.inv_w32) : floorf(v / a.w32);
        cd = (double)c;
        if (a.proj && count)
            a.proj[row * a.m + l] = y * scale;
    } else {
        double y64 = (double)scale * (double)y; // exact
        double t = __dmul_rn(a.alpha64, y64);
        double b64 = (double)bl[l];
        double v = __dadd_rn(t, b64);
        double q = a.w_pow2 ? v * a.inv_w64 : v / a.w64;
        cd = floor(q);
        // distance to the nearest bin edge vs the error bound of v
        double A = (double)w.absb[l];
        double Ey = (double)scale * (A * gam * 1.0000001 + 1e-40);
        double Ev = a.alpha64 * Ey * (1.0 + 1e-12) + 1e-15 * (fabs(t) + fabs(v) + b64);
        double dist = fabs(v - a.w64 * rint(q));
        if (dist <= Ev) {
            double ye = exact_component<DT>(a, tab, row, (double)scale, l);
            double ve = __dadd_rn(__dmul_rn(a.alpha64, ye), b64);
            double ce = floor(ve / a.w64);
            if (count) {
                ++nflag;
                nchg += ce != cd;
            }
            cd = ce;
            y64 = ye;
        }
        if (a.proj && count)
            a.proj[row * a.m + l] = (float)y64;
    }
    unsigned sat = 0;
    int32_t ci = floor_to_i32(cd, sat);
    if (count)
        nsat += sat;
    return ci;
}

template <int DT, bool RECHECK>
__device__ void epilogue_e2lsh(const HashArgs &a, const uint16_t *tab, const WaveLds &w,
                               const float *bl, const uint64_t *hinit, int64_t row, int rr,
                               double gam, unsigned &nflag, unsigned &nchg, unsigned &nsat)
{
    const int lane = lane_id();
    const float scale = a.row_scale ? a.row_scale[row] : 1.0f;
    for (int t = lane; t < a.L; t += kWave) {
        const int32_t l0 = t * a.K;
        uint64_t key = e2lsh_key(a.K, hinit[2 * t], hinit[2 * t + 1], [&](int r, bool first) {
            int32_t c = e2lsh_code<DT, RECHECK>(a, tab, w, bl, row, scale, gam, l0 + r, first,
                                                nflag, nchg, nsat);
            if (first && a.codes)
                a.codes[row * a.m + l0 + r] = c;
            return c;
        });
        w.stage[t * kRowsPerBlock + rr] = key;
    }
}

template <int DT, bool RECHECK>
__device__ void epilogue_srp(const HashArgs &a, const uint16_t *tab, const WaveLds &w, int64_t row,
                             int rr, double gam, unsigned &nflag, unsigned &nchg)
{
    const int lane = lane_id();
    const float scale = a.row_scale ? a.row_scale[row] : 1.0f;
    const int ngroups = (a.m + kWave - 1) / kWave;
    for (int g = 0; g < ngroups; ++g) {
        int32_t l = g * kWave + lane;
        bool bit = false;
        if (l < a.m) {
            float y = w.bins[l];
            bit = y > 0.0f;
            double y64 = (double)scale * (double)y;
            if constexpr (RECHECK) {
                double Ey = (double)scale * ((double)w.absb[l] * gam * 1.0000001 + 1e-40);
                if (fabs(y64) <= Ey) {
                    double ye = exact_component<DT>(a, tab, row, (double)scale, l);
                    bool be = ye > 0.0;
                    ++nflag;
                    nchg += be != bit;
                    bit = be;
                    y64 = ye;
                }
            }
            if (a.codes)
                a.codes[row * a.m + l] = bit ? 1 : 0;
            if (a.proj)
                a.proj[row * a.m + l] = RECHECK ? (float)y64 : y * scale;
        }
        uint64_t bal = __ballot(bit);
        if (lane == 0)
            w.mask[g] = bal;
    }
    wave_sync();
    for (int t = lane; t < a.L; t += kWave) {
        int32_t s0 = t * a.K;
        uint64_t v = w.mask[s0 >> 6] >> (s0 & 63);
        if ((s0 & 63) + a.K > 64)
            v |= w.mask[(s0 >> 6) + 1] << (64 - (s0 & 63));
        if (a.K < 64)
            v &= (1ull << a.K) - 1ull;
        w.stage[t * kRowsPerBlock + rr] = v;
    }
}

// ------------------------------------------------------------------ kernel

template <int FAM, int DT, bool ALIGNED, bool RECHECK>
__global__ __launch_bounds__(512) void hash_kernel(HashArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint16_t *tab = (uint16_t *)lds;
    float *bl = (float *)(lds + a.tab_bytes);
    uint64_t *hinit = (uint64_t *)(lds + a.tab_bytes + align16(a.m * 4));
    unsigned char *wave_base = lds + a.tab_bytes + align16(a.m * 4) + align16(a.L * 16);

    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    const int lane = lane_id();

    // ---- prologue: hash table, shifts, per-table digest seeds, zero bins
    bool bad = false;
    for (int32_t j = tid; j < a.d; j += blockDim.x)
        tab[j] = (uint16_t)table_entry(a, j, bad);
    if (FAM == LSH_E2LSH) {
        for (int32_t l = tid; l < a.m; l += blockDim.x)
            bl[l] = a.b[l];
        for (int32_t t = tid; t < 2 * a.L; t += blockDim.x)
            hinit[t] = mix64((uint64_t)t); // = F(2*table + wide)
    }
    WaveLds w;
    unsigned char *mine = wave_base + (size_t)wid * a.wave_bytes;
    w.bins = (float *)mine;
    w.absb = (float *)(mine + a.mpad * 4);
    w.stage = (uint64_t *)(mine + (RECHECK ? 2 : 1) * a.mpad * 4);
    w.mask = w.stage + a.L * kRowsPerBlock;
    for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4) {
        *(float4 *)(w.bins + l) = make_float4(0.f, 0.f, 0.f, 0.f);
        if (RECHECK)
            *(float4 *)(w.absb + l) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (bad && a.counters)
        atomicAdd(&a.counters[3], 1ull);
    __syncthreads();

    double gam = 0.0;
    if constexpr (RECHECK)
        gam = sum_gamma(*a.cmax);

    // ---- row blocks owned by this wave
    constexpr int VEC = ALIGNED ? Elem<DT>::per16 : 1;
    const int64_t nblk = (a.n + kRowsPerBlock - 1) / kRowsPerBlock;
    const int64_t wave_gid = (int64_t)blockIdx.x * a.waves + wid;
    const int64_t wave_stride = (int64_t)gridDim.x * a.waves;
    const int32_t nchunk = a.d / VEC;                      // d % VEC == 0 when ALIGNED
    const int32_t group = kWave * kChunksPerLane;          // chunks per load group
    const int32_t ngroups = (nchunk + group - 1) / group;  // load groups per row

    unsigned nflag = 0, nchg = 0, nsat = 0;

    // cursor over (block, row in block, group)
    int64_t blk = wave_gid;
    if (blk >= nblk)
        return;
    auto rows_in = [&](int64_t bk) -> int {
        int64_t r = a.n - bk * kRowsPerBlock;
        return r < kRowsPerBlock ? (int)r : kRowsPerBlock;
    };

    using T = typename Elem<DT>::T;
    u32x4 bufA[kChunksPerLane], bufB[kChunksPerLane];

    auto load = [&](u32x4 *buf, int64_t row, int32_t g) {
        const T *xr = (const T *)a.x + row * a.ld;
#pragma unroll
        for (int i = 0; i < kChunksPerLane; ++i) {
            int32_t c = g * group + i * kWave + lane;
            if (c < nchunk) {
                if constexpr (ALIGNED) {
                    buf[i] = __builtin_nontemporal_load((const u32x4 *)(xr + (int64_t)c * VEC));
                } else {
                    uint32_t u;
                    if constexpr (DT == LSH_F32)
                        u = __float_as_uint(xr[c]);
                    else
                        u = (uint32_t)xr[c];
                    buf[i] = u32x4{u, 0u, 0u, 0u};
                }
            }
        }
    };

    auto scatter = [&](const u32x4 *buf, int32_t g) {
#pragma unroll
        for (int i = 0; i < kChunksPerLane; ++i) {
            int32_t c = g * group + i * kWave + lane;
            if (c < nchunk) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    uint32_t ent = tab[c * VEC + e];
                    float v;
                    if constexpr (ALIGNED)
                        v = elem_value<DT>(buf[i], e);
                    else
                        v = bits_value<DT>(buf[i][0]);
                    float sv = __uint_as_float(__float_as_uint(v) ^ ((ent & 1u) << 31));
                    atomicAdd(&w.bins[ent >> 1], sv);
                    if constexpr (RECHECK)
                        atomicAdd(&w.absb[ent >> 1], fabsf(v));
                }
            }
        }
    };

    int rr = 0;                    // row within block
    int32_t g = 0;                 // load group within row
    int nrows = rows_in(blk);
    load(bufA, blk * kRowsPerBlock, 0);
    bool useA = true;
    while (true) {
        // next cursor position
        int64_t nblk_i = blk;
        int nrr = rr;
        int32_t ng = g + 1;
        if (ng == ngroups) {
            ng = 0;
            ++nrr;
            if (nrr == nrows) {
                nrr = 0;
                nblk_i = blk + wave_stride;
            }
        }
        const bool have_next = nblk_i < nblk;
        if (have_next)
            load(useA ? bufB : bufA, nblk_i * kRowsPerBlock + nrr, ng);

        scatter(useA ? bufA : bufB, g);

        if (g == ngroups - 1) {
            // row complete: discretise and key
            wave_sync();
            const int64_t row = blk * kRowsPerBlock + rr;
            if constexpr (FAM == LSH_E2LSH)
                epilogue_e2lsh<DT, RECHECK>(a, tab, w, bl, hinit, row, rr, gam, nflag, nchg, nsat);
            else
                epilogue_srp<DT, RECHECK>(a, tab, w, row, rr, gam, nflag, nchg);
            wave_sync();
            for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4) {
                *(float4 *)(w.bins + l) = make_float4(0.f, 0.f, 0.f, 0.f);
                if (RECHECK)
                    *(float4 *)(w.absb + l) = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            if (rr == nrows - 1 && a.keys) {
                // block complete: write the staged keys, 8 consecutive rows per table
                const int64_t row0 = blk * kRowsPerBlock;
                for (int e = lane; e < a.L * kRowsPerBlock; e += kWave) {
                    int t = e / kRowsPerBlock, r = e % kRowsPerBlock;
                    if (r < nrows)
                        a.keys[(int64_t)t * a.key_ld + row0 + r] = w.stage[e];
                }
            }
            wave_sync();
        }
        if (!have_next)
            break;
        if (nblk_i != blk)
            nrows = rows_in(nblk_i);
        blk = nblk_i;
        rr = nrr;
        g = ng;
        useA = !useA;
    }

    if (a.counters) {
        unsigned long long f = wave_sum((unsigned long long)nflag);
        unsigned long long c = wave_sum((unsigned long long)nchg);
        unsigned long long s = wave_sum((unsigned long long)nsat);
        if (lane == 0) {
            if (f)
                atomicAdd(&a.counters[0], f);
            if (c)
                atomicAdd(&a.counters[1], c);
            if (s)
                atomicAdd(&a.counters[2], s);
        }
    }
}

} // namespace lsh

// ========================================================================
// recheck support: bin -> coordinates (ascending) of the hash, and the
// largest bin population, built on the device by one workgroup
// ========================================================================

namespace lsh {

constexpr int kCsrMaxD = 32768;

__global__ __launch_bounds__(1024) void csr_kernel(HashArgs a, uint32_t *off, uint32_t *idx,
                                                   uint32_t *cmax, int p2)
{
    extern __shared__ uint32_t skeys[];
    __shared__ uint32_t smax;
    const int tid = threadIdx.x;
    bool bad = false;
    if (tid == 0)
        smax = 0;
    for (int i = tid; i < p2; i += blockDim.x)
        skeys[i] = i < a.d ? ((table_entry(a, i, bad) >> 1) << 16) | (uint32_t)i : 0xffffffffu;
    __syncthreads();
    // bitonic sort of (bin, coordinate) pairs
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < p2; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint32_t x = skeys[i], y = skeys[ixj];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        skeys[i] = y;
                        skeys[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int p = tid; p < a.d; p += blockDim.x)
        idx[p] = skeys[p] & 0xffffu;
    auto lower = [&](uint32_t key) {
        int lo = 0, hi = a.d;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (skeys[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        return (uint32_t)lo;
    };
    for (int bin = tid; bin <= a.m; bin += blockDim.x) {
        uint32_t o = lower((uint32_t)bin << 16);
        off[bin] = o;
        if (bin < a.m) {
            uint32_t c = lower((uint32_t)(bin + 1) << 16) - o;
            atomicMax(&smax, c);
        }
    }
    __syncthreads();
    if (tid == 0)
        *cmax = smax;
}

// ========================================================================
// host side
// ========================================================================

namespace {

struct WsLayout {
    size_t cmax, off, idx, total;
};

WsLayout ws_layout(int32_t d, int32_t m)
{
    WsLayout w;
    w.cmax = 0;
    w.off = 256;
    w.idx = w.off + align_up((size_t)(m + 1) * 4, 256);
    w.total = w.idx + align_up((size_t)d * 4, 256);
    return w;
}

int esize(int dt) { return dt == LSH_F32 ? 4 : (dt == LSH_BF16 ? 2 : 1); }

template <int FAM, int DT, bool AL, bool RC>
hipError_t launch_one(const HashArgs &a, int block, size_t lds, hipStream_t st, int64_t nblk)
{
    auto k = hash_kernel<FAM, DT, AL, RC>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds);
    if (e != hipSuccess)
        return e;
    if (per_cu < 1)
        return hipErrorInvalidConfiguration;
    int64_t want = (nblk + a.waves - 1) / a.waves;
    int64_t cap = (int64_t)device_cu_count() * per_cu;
    int grid = (int)(want < cap ? want : cap);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

template <int FAM, int DT>
hipError_t launch_dt(const HashArgs &a, bool al, bool rc, int block, size_t lds, hipStream_t st,
                     int64_t nblk)
{
    if (al)
        return rc ? launch_one<FAM, DT, true, true>(a, block, lds, st, nblk)
                  : launch_one<FAM, DT, true, false>(a, block, lds, st, nblk);
    return rc ? launch_one<FAM, DT, false, true>(a, block, lds, st, nblk)
              : launch_one<FAM, DT, false, false>(a, block, lds, st, nblk);
}

template <int FAM>
hipError_t launch_fam(const HashArgs &a, int dt, bool al, bool rc, int block, size_t lds,
                      hipStream_t st, int64_t nblk)
{
    switch (dt) {
    case LSH_F32:
        return launch_dt<FAM, LSH_F32>(a, al, rc, block, lds, st, nblk);
    case LSH_BF16:
        return launch_dt<FAM, LSH_BF16>(a, al, rc, block, lds, st, nblk);
    default:
        return launch_dt<FAM, LSH_FP8_E4M3FN>(a, al, rc, block, lds, st, nblk);
    }
}

bool is_pow2(float w)
{
    int ex;
    return frexpf(w, &ex) == 0.5f;
}

} // namespace

// Validates arguments, fills the common fields of HashArgs.
lsh_status check_points(const lsh_points *p)
{
    if (!p)
        LSH_FAIL(LSH_EINVAL, "points descriptor is NULL");
    if (p->dtype < LSH_F32 || p->dtype > LSH_FP8_E4M3FN)
        LSH_FAIL(LSH_EINVAL, "unknown dtype %d", p->dtype);
    if (p->n < 0 || p->d < 1 || p->ld < p->d)
        LSH_FAIL(LSH_EINVAL, "bad shape n=%lld d=%d ld=%lld", (long long)p->n, p->d,
                 (long long)p->ld);
    if (p->n > 0 && !p->x)
        LSH_FAIL(LSH_EINVAL, "points data pointer is NULL");
    if (p->dtype != LSH_F32 && p->n > 0 && !p->row_scale)
        LSH_FAIL(LSH_EINVAL, "low-precision points need row_scale");
    if (p->dtype == LSH_F32 && p->row_scale)
        LSH_FAIL(LSH_EINVAL, "row_scale must be NULL for FP32 points");
    return LSH_OK;
}

lsh_status check_disc(const lsh_disc *c)
{
    if (!c)
        LSH_FAIL(LSH_EINVAL, "disc descriptor is NULL");
    if (c->family != LSH_E2LSH && c->family != LSH_SRP)
        LSH_FAIL(LSH_EINVAL, "unknown family %d", c->family);
    if (c->K < 1 || c->K > 64 || c->L < 1 || (int64_t)c->K * c->L != c->m)
        LSH_FAIL(LSH_EINVAL, "need 1 <= K <= 64, L >= 1, m = K*L (K=%d L=%d m=%d)", c->K, c->L,
                 c->m);
    if (c->family == LSH_E2LSH) {
        if (!(c->w > 0.0f) || !isfinite(c->w))
            LSH_FAIL(LSH_EINVAL, "w must be positive and finite");
        if (!c->b)
            LSH_FAIL(LSH_EINVAL, "E2LSH needs the shift vector b");
    }
    return LSH_OK;
}

static lsh_status hash_common(const lsh_points *pts, HashArgs a, const lsh_disc *disc,
                              const lsh_out *out, void *ws, size_t ws_bytes, void *stream)
{
    lsh_status st;
    if ((st = check_points(pts)) != LSH_OK || (st = check_disc(disc)) != LSH_OK)
        return st;
    if (disc->m > 32768)
        LSH_FAIL(LSH_EINVAL, "m = %d exceeds 32768", disc->m);
    if (!out)
        LSH_FAIL(LSH_EINVAL, "output descriptor is NULL");
    const bool rc = disc->recheck != 0;
    if (rc && pts->d > kCsrMaxD)
        LSH_FAIL(LSH_EINVAL, "recheck supports d <= %d", kCsrMaxD);
    int64_t key_ld = out->key_ld ? out->key_ld : pts->n;
    if (out->keys && key_ld < pts->n)
        LSH_FAIL(LSH_EINVAL, "key_ld %lld < n %lld", (long long)key_ld, (long long)pts->n);
    if (pts->n == 0)
        return LSH_OK;

    a.x = pts->x;
    a.ld = pts->ld;
    a.n = pts->n;
    a.d = pts->d;
    a.row_scale = pts->row_scale;
    a.m = disc->m;
    a.K = disc->K;
    a.L = disc->L;
    a.alpha64 = sqrt((double)disc->m);
    a.alpha32 = (float)a.alpha64;
    a.w32 = disc->family == LSH_E2LSH ? disc->w : 1.0f;
    a.w64 = (double)a.w32;
    a.inv_w32 = 1.0f / a.w32;
    a.inv_w64 = 1.0 / a.w64;
    a.w_pow2 = is_pow2(a.w32);
    a.b = disc->b;
    a.keys = out->keys;
    a.key_ld = key_ld;
    a.codes = out->codes;
    a.proj = out->proj;
    a.counters = (unsigned long long *)out->counters;

    const int es = esize(pts->dtype);
    const int per16 = 16 / es;
    const bool al = ((uintptr_t)pts->x % 16 == 0) && ((pts->ld * es) % 16 == 0) &&
                    (pts->d % per16 == 0);

    // LDS layout
    a.tab_bytes = align16(pts->d * 2);
    a.mpad = (int32_t)align_up((size_t)a.m, 256);
    size_t shared = (size_t)a.tab_bytes + align16(a.m * 4) + align16(a.L * 16);
    size_t per_wave = (size_t)a.mpad * 4 * (rc ? 2 : 1) + (size_t)a.L * kRowsPerBlock * 8 +
                      align16(((a.m + 63) / 64) * 8);
    a.wave_bytes = (int32_t)align_up(per_wave, 16);
    const size_t lds_max = 160 * 1024;
    const int64_t nblk = (pts->n + kRowsPerBlock - 1) / kRowsPerBlock;
    int waves = 8;
    while (waves > 1 && (shared + (size_t)waves * a.wave_bytes > lds_max || waves > nblk))
        waves >>= 1;
    size_t lds = shared + (size_t)waves * a.wave_bytes;
    if (lds > lds_max)
        LSH_FAIL(LSH_EINVAL, "d=%d, m=%d, L=%d need %zu bytes of LDS (max %zu)", pts->d, a.m, a.L,
                 lds, lds_max);
    a.waves = waves;

    hipStream_t s = (hipStream_t)stream;
    if (rc) {
        WsLayout wl = ws_layout(pts->d, a.m);
        if (!ws || ws_bytes < wl.total)
            LSH_FAIL(LSH_ENOMEM, "recheck workspace needs %zu bytes, got %zu", wl.total, ws_bytes);
        unsigned char *wb = (unsigned char *)ws;
        a.cmax = (const uint32_t *)(wb + wl.cmax);
        a.csr_off = (const uint32_t *)(wb + wl.off);
        a.csr_idx = (const uint32_t *)(wb + wl.idx);
        int p2 = 1;
        while (p2 < pts->d)
            p2 <<= 1;
        size_t clds = (size_t)p2 * 4;
        LSH_HIP(hipFuncSetAttribute((const void *)csr_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)clds));
        hipLaunchKernelGGL(csr_kernel, dim3(1), dim3(1024), clds, s, a, (uint32_t *)a.csr_off,
                           (uint32_t *)a.csr_idx, (uint32_t *)a.cmax, p2);
        LSH_LAUNCHED("csr_kernel");
    }

    hipError_t e = disc->family == LSH_E2LSH
                       ? launch_fam<LSH_E2LSH>(a, pts->dtype, al, rc, waves * kWave, lds, s, nblk)
                       : launch_fam<LSH_SRP>(a, pts->dtype, al, rc, waves * kWave, lds, s, nblk);
    if (e != hipSuccess)
        LSH_FAIL(LSH_EHIP, "hash kernel launch failed: %s", hip_msg(e));
    return LSH_OK;
}

} // namespace lsh

extern "C" size_t lsh_hash_workspace_bytes(int32_t d, int32_t m, int32_t recheck)
{
    if (!recheck || d < 1 || m < 1)
        return 0;
    return lsh::ws_layout(d, m).total;
}

extern "C" lsh_status lsh_hash_cs(const lsh_points *pts, const uint32_t *h, const int8_t *s,
                                  const lsh_disc *disc, const lsh_out *out, void *workspace,
                                  size_t ws_bytes, void *stream)
{
    if (!h || !s)
        LSH_FAIL(LSH_EINVAL, "h and s are required");
    lsh::HashArgs a = {};
    a.hcs = 0;
    a.h = h;
    a.s = s;
    return lsh::hash_common(pts, a, disc, out, workspace, ws_bytes, stream);
}

extern "C" lsh_status lsh_hash_hcs(const lsh_points *pts, int32_t N, const int32_t *d_k,
                                   const int32_t *m_k, const uint32_t *h_k, const int8_t *s_k,
                                   const lsh_disc *disc, const lsh_out *out, void *workspace,
                                   size_t ws_bytes, void *stream)
{
    if (N < 1 || N > lsh::kMaxModes || !d_k || !m_k || !h_k || !s_k)
        LSH_FAIL(LSH_EINVAL, "HCS needs 1 <= N <= %d and the per-mode tables", lsh::kMaxModes);
    lsh::HashArgs a = {};
    a.hcs = 1;
    a.N = N;
    a.hk = h_k;
    a.sk = s_k;
    int64_t D = 1, M = 1;
    int32_t o = 0;
    for (int k = 0; k < N; ++k) {
        if (d_k[k] < 1 || m_k[k] < 1)
            LSH_FAIL(LSH_EINVAL, "mode %d has d_k=%d m_k=%d", k, d_k[k], m_k[k]);
        a.dk[k] = d_k[k];
        a.mk[k] = m_k[k];
        a.mode_off[k] = o;
        o += d_k[k];
        D *= d_k[k];
        M *= m_k[k];
        if (D > (int64_t)1 << 40 || M > (int64_t)1 << 40)
            LSH_FAIL(LSH_EINVAL, "mode sizes overflow");
    }
    if (pts && D < pts->d)
        LSH_FAIL(LSH_EINVAL, "prod d_k = %lld < d = %d", (long long)D, pts->d);
    if (disc && M != disc->m)
        LSH_FAIL(LSH_EINVAL, "prod m_k = %lld != m = %d", (long long)M, disc->m);
    return lsh::hash_common(pts, a, disc, out, workspace, ws_bytes, stream);
}
