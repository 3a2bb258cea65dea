// Count-sketch and higher-order count-sketch LSH hashing on gfx950.
//
// One fused, HBM-bound kernel per call: stream the rows of X once, add every
// coordinate into its sketch bin with its sign (count sketch, Section 3.2 Eq.
// eq_cs; the higher-order count sketch of Eq. eqhcs is the same sum under the
// composite bin and sign of the per-mode hashes), discretise the m bins
// (floor((sqrt(m) y + b)/w), Definitions CS_Eucl_LSH / HCS_Eucl_LSH, or
// sgn(y), Definitions cs_consine_lsh / hcs_consine_lsh), and fold each
// table's K codes into its 64-bit bucket key (Section 3.1).
//
// Work decomposition:
//   * a workgroup of W waves shares the packed hash table (one 16-bit entry
//     per coordinate: LDS slot of its bin << 1 | sign), built once per
//     workgroup from h/s (CS) or from the per-mode tables (HCS), together
//     with the largest bin population c_max;
//   * each wave hashes blocks of RB consecutive rows.  A whole row is loaded
//     into registers with 16-byte loads (chunk c of the row in lane c mod 64)
//     -- two rows at a time when they are short, so the second row's loads
//     are in flight while the first is summed;
//   * fixed-point sums: LDS float atomics are slow on this GPU, integer ones
//     run at streaming speed.  Each row gets an exponent k from its largest
//     magnitude 2^e and c_max (k = 31 - ceil(log2(c_max + 1)) - e), every
//     term s_j x_j is scaled by 2^k, truncated to int32 and added with an LDS
//     integer atomic into the wave's bins.  No bin can overflow, the sum is
//     exact and independent of the order of the atomics (so results are
//     bit-reproducible), and y = sum * 2^-k differs from the real sum by less
//     than c * 2^-k for a bin of c terms;
//   * after a row, the wave discretises its bins (E2LSH: one lane per table,
//     bins padded one word per 16 so those reads are conflict-free; SRP: one
//     lane per component plus ballots) and stages the L keys of its RB rows
//     in LDS, so key stores leave as 8-key (64-byte) runs.
// The optional FP64 recheck recomputes, in ascending coordinate order and in
// FP64, every component whose value lies within the rigorous bound of its
// error from a bin edge (E2LSH) or from zero (SRP).

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "lsh_internal.h"

namespace lsh {

constexpr int kRowsPerBlock = 8; // RB: rows a wave hashes before writing keys
constexpr int kMaxModes = 8;

__host__ __device__ constexpr int align16(int v) { return (v + 15) & ~15; }

// LDS slot of sketch bin l: one pad word after every 16 bins, so that lanes
// reading K consecutive bins each (one lane per table) hit distinct banks.
__host__ __device__ constexpr int bin_pos(int l) { return l + (l >> 4); }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct HashArgs {
    const void *x;
    int64_t ld;
    int64_t n;
    int32_t d;
    const float *row_scale;
    int32_t m, K, L;
    float alpha32;  // sqrt(m)
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
    // layout
    int32_t waves;      // waves per workgroup
    int32_t tab_bytes;  // LDS bytes of the hash table (aligned)
    int32_t mpad;       // bin slots per wave, multiple of 256
    int32_t wave_bytes; // LDS bytes per wave
};

// Bin of coordinate j in the sketch and its sign (neg = sign < 0).
__device__ __forceinline__ uint32_t table_bin(const HashArgs &a, int32_t j, bool &bad,
                                              uint32_t &neg_out)
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
    neg_out = neg;
    return bin;
}

// Packed LDS table entry of coordinate j: LDS slot of its bin << 1 | sign bit.
__device__ __forceinline__ uint32_t table_entry(const HashArgs &a, int32_t j, bool &bad)
{
    uint32_t neg;
    uint32_t bin = table_bin(a, j, bad, neg);
    return ((uint32_t)bin_pos((int)bin) << 1) | neg;
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

// Element e of a 16-byte chunk (ALIGNED) or the single element of a chunk.
template <int DT, bool AL> __device__ __forceinline__ float chunk_value(u32x4 v, int e)
{
    if constexpr (!AL) {
        uint32_t u = v[0];
        if constexpr (DT == LSH_F32)
            return __uint_as_float(u);
        else if constexpr (DT == LSH_BF16)
            return __uint_as_float((u & 0xffffu) << 16);
        else
            return fp8_to_f32(u & 0xffu);
    } else {
        uint32_t word = v[e / (Elem<DT>::per16 / 4)];
        if constexpr (DT == LSH_F32)
            return __uint_as_float(word);
        else if constexpr (DT == LSH_BF16)
            return __uint_as_float((e & 1) ? (word & 0xffff0000u) : (word << 16));
        else
            return fp8_to_f32((word >> (8 * (e & 3))) & 0xffu);
    }
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

// ----------------------------------------------------------- wave helpers

struct WaveLds {
    int32_t *bins;   // [mpad] fixed-point sums, indexed by bin_pos
    uint64_t *stage; // [L * RB] keys of the current row block
    uint64_t *mask;  // [ceil(m/64)] SRP sign bits of the current row
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Per-row scale (1 for FP32 points), read through the scalar cache: row is
// the same in every lane.
template <int DT> __device__ __forceinline__ float row_scale_of(const HashArgs &a, int64_t row)
{
    if constexpr (DT == LSH_F32) {
        return 1.0f;
    } else {
        int64_t r = ((int64_t)__builtin_amdgcn_readfirstlane((int)(row >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)row);
        return a.row_scale[r];
    }
}

// What the epilogue needs to turn a bin's fixed-point sum into y.
struct RowFix {
    float scale;  // row scale (1 for FP32)
    float fs;     // scale * 2^-k as FP32 (may underflow for tiny rows; fast path only)
    float af;     // fs * sqrt(m) / w (fast E2LSH path)
    double s2k;   // scale * 2^-k in FP64 (exact)
    double ey;    // bound on |y - y_fp64| before the per-component term (recheck)
};

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

// ------------------------------------------------------------- the epilogue

// Code of E2LSH component l (Definition CS_Eucl_LSH): floor((sqrt(m) y + b)/w).
template <int DT, bool RECHECK>
__device__ __forceinline__ int32_t e2lsh_code(const HashArgs &a, const uint16_t *tab,
                                              const WaveLds &w, const float *bl, int64_t row,
                                              const RowFix &rf, int32_t l, bool count,
                                              unsigned &nflag, unsigned &nchg, unsigned &nsat)
{
    const int pl = bin_pos(l);
    const int32_t isum = w.bins[pl];
    double cd;
    if constexpr (!RECHECK) {
        // bl holds b / w here; the row factor sqrt(m) * scale * 2^-k / w is folded in
        float v = fmaf(rf.af, (float)isum, bl[pl]);
        cd = (double)floorf(v);
        if (a.proj && count)
            a.proj[row * a.m + l] = (float)isum * rf.fs;
    } else {
        double y64 = (double)isum * rf.s2k;
        double t = __dmul_rn(a.alpha64, y64);
        double b64 = (double)bl[pl];
        double v = __dadd_rn(t, b64);
        double q = a.w_pow2 ? v * a.inv_w64 : v / a.w64;
        cd = floor(q);
        double Ey = rf.ey + fabs(y64) * 0x1.0p-51;
        double Ev = a.alpha64 * Ey * (1.0 + 1e-12) + 0x1.0p-50 * (fabs(t) + fabs(v) + fabs(b64));
        double dist = fabs(v - a.w64 * rint(q));
        if (dist <= Ev) {
            double ye = exact_component<DT>(a, tab, row, (double)rf.scale, l);
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
                               const RowFix &rf, unsigned &nflag, unsigned &nchg, unsigned &nsat)
{
    const int lane = lane_id();
    for (int t = lane; t < a.L; t += kWave) {
        const int32_t l0 = t * a.K;
        uint64_t key = e2lsh_key(a.K, hinit[2 * t], hinit[2 * t + 1], [&](int r, bool first) {
            int32_t c = e2lsh_code<DT, RECHECK>(a, tab, w, bl, row, rf, l0 + r, first, nflag,
                                                nchg, nsat);
            if (first && a.codes)
                a.codes[row * a.m + l0 + r] = c;
            return c;
        });
        w.stage[t * kRowsPerBlock + rr] = key;
    }
}

// SRP family: bit = [y > 0] (Definition cs_consine_lsh).  The fixed-point sum
// has the sign of y except within its error bound of 0 (rechecked on request).
template <int DT, bool RECHECK>
__device__ void epilogue_srp(const HashArgs &a, const uint16_t *tab, const WaveLds &w, int64_t row,
                             int rr, const RowFix &rf, unsigned &nflag, unsigned &nchg)
{
    const int lane = lane_id();
    const int ngroups = (a.m + kWave - 1) / kWave;
    for (int g = 0; g < ngroups; ++g) {
        int32_t l = g * kWave + lane;
        bool bit = false;
        if (l < a.m) {
            const int32_t isum = w.bins[bin_pos(l)];
            bit = isum > 0;
            float yout = (float)isum * rf.fs;
            if constexpr (RECHECK) {
                double y64 = (double)isum * rf.s2k;
                double Ey = rf.ey + fabs(y64) * 0x1.0p-51;
                if (fabs(y64) <= Ey) {
                    double ye = exact_component<DT>(a, tab, row, (double)rf.scale, l);
                    bool be = ye > 0.0;
                    ++nflag;
                    nchg += be != bit;
                    bit = be;
                    y64 = ye;
                }
                yout = (float)y64;
            }
            if (a.codes)
                a.codes[row * a.m + l] = bit ? 1 : 0;
            if (a.proj)
                a.proj[row * a.m + l] = yout;
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

// CH: 16-byte chunks (ALIGNED) or single elements per lane per row; a row
// has at most 64 * CH of them.
template <int FAM, int DT, bool ALIGNED, bool RECHECK, int CH>
__global__ __launch_bounds__(512) void hash_kernel(HashArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint16_t *tab = (uint16_t *)lds;
    float *bl = (float *)(lds + a.tab_bytes);
    uint64_t *hinit = (uint64_t *)(lds + a.tab_bytes + align16(bin_pos(a.m) * 4));
    unsigned char *wave_base = lds + a.tab_bytes + align16(bin_pos(a.m) * 4) + align16(a.L * 16);
    __shared__ uint32_t s_cmax;

    const int tid = threadIdx.x;
    // wave index, made visibly uniform so the row cursor lives in SGPRs
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = lane_id();

    WaveLds w;
    unsigned char *mine = wave_base + (size_t)wid * a.wave_bytes;
    w.bins = (int32_t *)mine;
    w.stage = (uint64_t *)(mine + a.mpad * 4);
    w.mask = w.stage + a.L * kRowsPerBlock;

    // ---- prologue: zero every wave's bins; wave 0's bins first count the
    // bin populations (integer LDS atomics) to find c_max
    if (tid == 0)
        s_cmax = 0;
    for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4)
        *(int4 *)(w.bins + l) = make_int4(0, 0, 0, 0);
    __syncthreads();
    int32_t *cnt = (int32_t *)wave_base;
    bool bad = false;
    for (int32_t j = tid; j < a.d; j += blockDim.x) {
        uint32_t ent = table_entry(a, j, bad);
        tab[j] = (uint16_t)ent;
        atomicAdd(&cnt[ent >> 1], 1);
    }
    if (FAM == LSH_E2LSH) {
        // fast path: b / w (the row factor folds 1/w in); recheck: b as given
        for (int32_t l = tid; l < a.m; l += blockDim.x)
            bl[bin_pos(l)] = RECHECK ? a.b[l] : a.b[l] * a.inv_w32;
        for (int32_t t = tid; t < 2 * a.L; t += blockDim.x)
            hinit[t] = mix64((uint64_t)t); // = F(2 * table + wide)
    }
    __syncthreads();
    for (int32_t l = tid; l < a.m; l += blockDim.x)
        atomicMax(&s_cmax, (uint32_t)cnt[bin_pos(l)]);
    __syncthreads();
    for (int32_t l = tid; l < a.mpad; l += blockDim.x)
        cnt[l] = 0;
    if (bad && a.counters && tid == 0)
        atomicAdd(&a.counters[3], 1ull);
    __syncthreads();

    const uint32_t cmax = s_cmax;
    // terms are kept below 2^(31 - hr) with c_max < 2^hr: no bin overflows int32
    const int hr = cmax ? 32 - __clz(cmax) : 0;
    const int koff = 31 - hr;

    // ---- rows owned by this wave
    constexpr int VEC = ALIGNED ? Elem<DT>::per16 : 1;
    const int64_t nblk = (a.n + kRowsPerBlock - 1) / kRowsPerBlock;
    const int64_t wave_gid = (int64_t)blockIdx.x * a.waves + wid;
    const int64_t wave_stride = (int64_t)gridDim.x * a.waves;
    const int32_t nchunk = a.d / VEC; // d % VEC == 0 when ALIGNED

    unsigned nflag = 0, nchg = 0, nsat = 0;

    using T = typename Elem<DT>::T;
    using Buf = u32x4[CH];

    // Every lane issues exactly CH loads per row (chunks past the row end
    // re-read chunk 0 and are not summed), so the number of loads in flight
    // is static and each wait covers only the row being summed.
    auto load_row = [&](Buf &buf, int64_t row) {
        const T *xr = (const T *)a.x + row * a.ld;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            int32_t ch = i * kWave + lane;
            ch = ch < nchunk ? ch : 0;
            if constexpr (ALIGNED) {
                buf[i] = __builtin_nontemporal_load((const u32x4 *)(xr + (int64_t)ch * VEC));
            } else {
                uint32_t u;
                if constexpr (DT == LSH_F32)
                    u = __float_as_uint(xr[ch]);
                else
                    u = (uint32_t)xr[ch];
                buf[i] = u32x4{u, 0u, 0u, 0u};
            }
        }
    };

    constexpr int TW = VEC >= 2 ? VEC / 2 : 1; // table dwords per chunk
    auto process_row = [&](const Buf &buf, int64_t row, int rr, int nrows, int64_t row0) {
        // 1. the row's largest magnitude -> exponent e (|x| < 2^e) -> k
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i * kWave + lane < nchunk) {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    mx = fmaxf(mx, fabsf(chunk_value<DT, ALIGNED>(buf[i], e)));
            }
        }
        const uint32_t mb = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_int(wave_max(mx)));
        const int be = (int)((mb >> 23) & 0xffu);
        const int e = be == 0 ? -126 : be - 126;
        const int k = koff - e;

        // 2. signed fixed-point sums into this wave's bins
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int32_t ch = i * kWave + lane;
            if (ch < nchunk) {
                uint32_t tw[TW];
                if constexpr (VEC == 1) {
                    tw[0] = tab[ch];
                } else if constexpr (VEC == 4) {
                    uint2 v = *(const uint2 *)(tab + ch * VEC);
                    tw[0] = v.x;
                    tw[1] = v.y;
                } else {
#pragma unroll
                    for (int q = 0; q < TW / 4; ++q) {
                        u32x4 v = *(const u32x4 *)(tab + ch * VEC + q * 8);
                        tw[4 * q + 0] = v[0];
                        tw[4 * q + 1] = v[1];
                        tw[4 * q + 2] = v[2];
                        tw[4 * q + 3] = v[3];
                    }
                }
#pragma unroll
                for (int e2 = 0; e2 < VEC; ++e2) {
                    uint32_t ent = VEC == 1 ? tw[0] : (tw[e2 >> 1] >> (16 * (e2 & 1))) & 0xffffu;
                    float v = chunk_value<DT, ALIGNED>(buf[i], e2);
                    float sv = __uint_as_float(__float_as_uint(v) ^ ((ent & 1u) << 31));
                    atomicAdd(&w.bins[ent >> 1], (int32_t)ldexpf(sv, k));
                }
            }
        }

        // 3. discretise, key, stage
        wave_sync();
        RowFix rf;
        rf.scale = row_scale_of<DT>(a, row);
        rf.s2k = ldexp((double)rf.scale, -k);
        rf.fs = (float)rf.s2k;
        rf.af = rf.fs * a.alpha32 * a.inv_w32;
        if constexpr (RECHECK) {
            // truncation: each term off by < 2^-k (times the scale), a bin has
            // <= c_max terms; plus the FP64 reference's own rounding
            // (c_max^2 * 2^(e-52) bounds gamma_{c-1} * sum|terms|)
            rf.ey = (double)rf.scale * (double)cmax *
                    (ldexp(1.0, -k) + (double)cmax * ldexp(1.0, e - 51));
        } else {
            rf.ey = 0.0;
        }
        if constexpr (FAM == LSH_E2LSH)
            epilogue_e2lsh<DT, RECHECK>(a, tab, w, bl, hinit, row, rr, rf, nflag, nchg, nsat);
        else
            epilogue_srp<DT, RECHECK>(a, tab, w, row, rr, rf, nflag, nchg);
        wave_sync();
        for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4)
            *(int4 *)(w.bins + l) = make_int4(0, 0, 0, 0);
        if (rr == nrows - 1 && a.keys) {
            // block complete: write the staged keys, up to 8 consecutive rows per table
            for (int ee = lane; ee < a.L * kRowsPerBlock; ee += kWave) {
                int t = ee / kRowsPerBlock, r = ee % kRowsPerBlock;
                if (r < nrows)
                    a.keys[(int64_t)t * a.key_ld + row0 + r] = w.stage[ee];
            }
        }
        wave_sync();
    };

    for (int64_t blk = wave_gid; blk < nblk; blk += wave_stride) {
        const int64_t row0 = blk * kRowsPerBlock;
        const int nrows = (int)(a.n - row0 < kRowsPerBlock ? a.n - row0 : kRowsPerBlock);
        if constexpr (CH <= 8) {
            // two rows per step: the second row's loads overlap the first row's sums
            Buf bufA, bufB;
            for (int rr = 0; rr < nrows; rr += 2) {
                const bool two = rr + 1 < nrows;
                load_row(bufA, row0 + rr);
                load_row(bufB, row0 + rr + (two ? 1 : 0));
                process_row(bufA, row0 + rr, rr, nrows, row0);
                if (two)
                    process_row(bufB, row0 + rr + 1, rr + 1, nrows, row0);
            }
        } else {
            Buf buf;
            for (int rr = 0; rr < nrows; ++rr) {
                load_row(buf, row0 + rr);
                process_row(buf, row0 + rr, rr, nrows, row0);
            }
        }
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
    {
        uint32_t neg;
        skeys[i] = i < a.d ? (table_bin(a, i, bad, neg) << 16) | (uint32_t)i : 0xffffffffu;
    }
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

template <int FAM, int DT, bool AL, bool RC, int CH>
hipError_t launch_one(const HashArgs &a, int block, size_t lds, hipStream_t st, int64_t nblk)
{
    auto k = hash_kernel<FAM, DT, AL, RC, CH>;
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

template <int FAM, int DT, bool AL, bool RC>
hipError_t launch_ch(const HashArgs &a, int ch, int block, size_t lds, hipStream_t st, int64_t nblk)
{
    if constexpr (AL) {
        switch (ch) {
        case 1:
            return launch_one<FAM, DT, AL, RC, 1>(a, block, lds, st, nblk);
        case 2:
            return launch_one<FAM, DT, AL, RC, 2>(a, block, lds, st, nblk);
        case 4:
            return launch_one<FAM, DT, AL, RC, 4>(a, block, lds, st, nblk);
        case 8:
            return launch_one<FAM, DT, AL, RC, 8>(a, block, lds, st, nblk);
        case 16:
            return launch_one<FAM, DT, AL, RC, 16>(a, block, lds, st, nblk);
        default:
            return launch_one<FAM, DT, AL, RC, 32>(a, block, lds, st, nblk);
        }
    } else {
        if (ch <= 8)
            return launch_one<FAM, DT, AL, RC, 8>(a, block, lds, st, nblk);
        return launch_one<FAM, DT, AL, RC, 32>(a, block, lds, st, nblk);
    }
}

template <int FAM, int DT>
hipError_t launch_dt(const HashArgs &a, bool al, bool rc, int ch, int block, size_t lds,
                     hipStream_t st, int64_t nblk)
{
    if (al)
        return rc ? launch_ch<FAM, DT, true, true>(a, ch, block, lds, st, nblk)
                  : launch_ch<FAM, DT, true, false>(a, ch, block, lds, st, nblk);
    return rc ? launch_ch<FAM, DT, false, true>(a, ch, block, lds, st, nblk)
              : launch_ch<FAM, DT, false, false>(a, ch, block, lds, st, nblk);
}

template <int FAM>
hipError_t launch_fam(const HashArgs &a, int dt, bool al, bool rc, int ch, int block, size_t lds,
                      hipStream_t st, int64_t nblk)
{
    switch (dt) {
    case LSH_F32:
        return launch_dt<FAM, LSH_F32>(a, al, rc, ch, block, lds, st, nblk);
    case LSH_BF16:
        return launch_dt<FAM, LSH_BF16>(a, al, rc, ch, block, lds, st, nblk);
    default:
        return launch_dt<FAM, LSH_FP8_E4M3FN>(a, al, rc, ch, block, lds, st, nblk);
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
    if (disc->m > 16384)
        LSH_FAIL(LSH_EINVAL, "m = %d exceeds 16384", disc->m);
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
    // a row is held in registers: at most 64 * 32 chunks (16-byte chunks when
    // aligned, single elements otherwise)
    const int64_t nch = al ? pts->d / per16 : pts->d;
    int ch = 1;
    while (ch < 32 && 64 * ch < nch)
        ch <<= 1;
    if (!al && ch < 8)
        ch = 8;
    if (64 * ch < nch)
        LSH_FAIL(LSH_EINVAL, "d = %d exceeds the single-pass row size (%d elements%s)", pts->d,
                 64 * 32 * (al ? per16 : 1), al ? "" : "; rows are not 16-byte aligned");

    // LDS layout
    a.tab_bytes = align16(pts->d * 2);
    a.mpad = (int32_t)align_up((size_t)bin_pos(a.m), 256);
    size_t shared = (size_t)a.tab_bytes + align16(bin_pos(a.m) * 4) + align16(a.L * 16);
    size_t per_wave = (size_t)a.mpad * 4 + (size_t)a.L * kRowsPerBlock * 8 +
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
        uint32_t *cmax_ws = (uint32_t *)(wb + wl.cmax);
        a.csr_off = (const uint32_t *)(wb + wl.off);
        a.csr_idx = (const uint32_t *)(wb + wl.idx);
        int p2 = 1;
        while (p2 < pts->d)
            p2 <<= 1;
        size_t clds = (size_t)p2 * 4;
        LSH_HIP(hipFuncSetAttribute((const void *)csr_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)clds));
        hipLaunchKernelGGL(csr_kernel, dim3(1), dim3(1024), clds, s, a, (uint32_t *)a.csr_off,
                           (uint32_t *)a.csr_idx, cmax_ws, p2);
        LSH_LAUNCHED("csr_kernel");
    }

    hipError_t e = disc->family == LSH_E2LSH
                       ? launch_fam<LSH_E2LSH>(a, pts->dtype, al, rc, ch, waves * kWave, lds, s, nblk)
                       : launch_fam<LSH_SRP>(a, pts->dtype, al, rc, ch, waves * kWave, lds, s, nblk);
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
