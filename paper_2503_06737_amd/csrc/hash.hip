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
//   * a workgroup of W waves shares the hash table (one 32-bit entry per
//     coordinate: byte offset of its bin's LDS slot, sign in bit 31), built
//     once per workgroup from h/s (CS) or from the per-mode tables (HCS),
//     together with the largest bin population c_max; a lane keeps the
//     entries of its chunks in registers when a row has at most 1024
//     elements;
//   * each wave hashes rows of blocks of RB consecutive rows.  A row is
//     loaded into registers with 16-byte loads (chunk c of the row in lane
//     c mod 64), the wave's next row in flight while one is summed; long
//     rows are read in pieces of 1024 elements, the next piece in flight;
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
//     lane per component plus ballots) and stages the row's L keys in LDS;
//     after each block the workgroup writes them as 256-byte runs per table.
// With the FP64 recheck, a component is evaluated in FP64 from the stored
// values, in ascending coordinate order, when its FP32 value lies within the
// rigorous bound of its error from a bin edge (E2LSH) or its fixed-point sum
// within the truncation bound of zero (SRP); the other codes already equal
// the FP64 evaluation's.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "lsh_internal.h"

namespace lsh {

// RB: consecutive rows a workgroup hashes before it writes their keys; a
// table's RB keys fill two 128-byte lines
constexpr int kRowsPerBlock = 32;
constexpr int kMaxModes = 8;

__host__ __device__ constexpr int align16(int v) { return (v + 15) & ~15; }

// LDS slot of sketch bin l: one pad word after every 16 bins, so that lanes
// reading K consecutive bins each (one lane per table) hit distinct banks.
__host__ __device__ constexpr int bin_pos(int l) { return l + (l >> 4); }
// Bin slots [bin_pos(m), bin_pos(m) + 64) are per-lane trash: a lane with
// nothing to add adds there, at its own address (no same-address atomics).
constexpr int kTrashSlots = kWave;

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
    // code position of each sketch component (NULL: component l is position l)
    const uint32_t *comp_slot;
    // recheck support (workspace)
    const uint32_t *csr_off;
    const uint32_t *csr_idx;
    // layout
    int32_t waves;       // waves per workgroup
    int32_t mpad;        // bin slots per wave (bins, pad words, trash), multiple of 4
    int32_t wave_region; // LDS bytes per wave region: a power of two >= 4 * mpad
    int32_t tab_entries; // table entries: 64 * CH * VEC * pieces (rows padded to whole chunks)
    int32_t tab_off, bl_off, hinit_off, mask_off; // LDS byte offsets
    // key staging (stage_stride 0: keys are stored straight to memory):
    // key of table t for row slot i of the block is at LDS byte
    // stage_base + (t >> stage_tpc_log2) * stage_stride
    //            + ((t & (2^stage_tpc_log2 - 1)) * (RB + 1) + i) * 8
    int32_t stage_base, stage_stride, stage_tpc_log2;
    int32_t pieces; // long rows: pieces of 64 * CH chunks per row (even); 1 otherwise
};

__device__ __forceinline__ uint32_t stage_addr(const HashArgs &a, int t, int slot)
{
    const uint32_t tpc_mask = (1u << a.stage_tpc_log2) - 1u;
    return (uint32_t)a.stage_base + ((uint32_t)t >> a.stage_tpc_log2) * (uint32_t)a.stage_stride +
           (((uint32_t)t & tpc_mask) * (kRowsPerBlock + 1) + (uint32_t)slot) * 8u;
}

typedef __attribute__((address_space(3))) uint64_t lds_u64;

// Key of table t for `row` (slot `slot` of its block): staged in LDS for the
// workgroup's coalesced write-out, or stored directly.
__device__ __forceinline__ void emit_key(const HashArgs &a, int t, int64_t row, int slot,
                                         uint64_t key)
{
    if (a.stage_stride)
        *(lds_u64 *)(size_t)stage_addr(a, t, slot) = key;
    else
        a.keys[(int64_t)t * a.key_ld + row] = key;
}

// Code position of coordinate j and its sign (neg = sign < 0): the sketch
// component the coordinate adds into, then that component's position in the
// code vector (table = position / K).  Entries out of range are taken as 0
// and counted in `bad`.
__device__ __forceinline__ uint32_t table_bin(const HashArgs &a, int32_t j, uint32_t &bad,
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
                ++bad;
                hb = 0;
            }
            bin += hb * stride;
            stride *= (uint32_t)a.mk[k];
            neg ^= a.sk[a.mode_off[k] + ik] < 0;
        }
    }
    if (bin >= (uint32_t)a.m) {
        ++bad;
        bin = 0;
    }
    if (a.comp_slot) {
        bin = a.comp_slot[bin];
        if (bin >= (uint32_t)a.m) {
            ++bad;
            bin = 0;
        }
    }
    neg_out = neg;
    return bin;
}

// LDS table entry of coordinate j: byte offset of its bin's slot inside a
// wave's region, sign in bit 31.  A lane forms the LDS address of the slot
// with one v_and_or (offset bits | its wave's region base).
__device__ __forceinline__ uint32_t table_entry(const HashArgs &a, int32_t j, uint32_t &bad)
{
    uint32_t neg;
    uint32_t bin = table_bin(a, j, bad, neg);
    return ((uint32_t)bin_pos((int)bin) * 4u) | (neg << 31);
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

// OCP E4M3FN -> FP32 by the gfx950 conversion instruction (exact: every
// E4M3FN value, subnormals included, is an FP32 number).  byte 0 of w.
__device__ __forceinline__ float fp8_to_f32(uint32_t w)
{
    return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
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
        else // bytes 0-1 or 2-3 of the word as a pair: one conversion per two values
            return (e & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8((int)word, true)[e & 1]
                           : __builtin_amdgcn_cvt_pk_f32_fp8((int)word, false)[e & 1];
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

// Integer add into the LDS word at byte address addr (an address-space-3
// pointer built from the integer, so no symbol offset is added per access).
__device__ __forceinline__ void lds_add_i32(uint32_t addr, int32_t v)
{
    typedef __attribute__((address_space(3))) int32_t lds_i32;
    __atomic_fetch_add((lds_i32 *)(size_t)addr, v, __ATOMIC_RELAXED);
}

struct WaveLds {
    int32_t *bins;   // [mpad] this wave's fixed-point sums, indexed by bin_pos
    uint64_t *mask;  // [ceil(m/64)] this wave's SRP sign bits of the current row
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Maximum of a non-negative value over the wave with DPP (no LDS round
// trips): prefix maxima inside each row of 16 lanes (row_shr 1, 2, 4, 8),
// then row_bcast 15 and 31 carry them to lane 63.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
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
    float efast;  // fast path: bound on |v - v_fp64| in units of w, before the |v| term
    int32_t eunits; // fast path: bound on |sum - y 2^k / scale| in fixed-point units
};

// Fast path, counters requested: the components whose FP32 value v =
// af * sum + b/w lies within its error bound of a bin edge, so that their
// code may differ from the FP64 evaluation's.  The bound is the fixed-point
// truncation (rf.efast) plus the FP32 rounding of the sum's conversion, of
// af and of the FMA (2^-20 |v| covers them; |v| >= 2^23 is always counted).
__device__ __forceinline__ unsigned fast_near_e2lsh(const HashArgs &a, const WaveLds &w,
                                                    const float *bl, const RowFix &rf)
{
    unsigned c = 0;
    for (int32_t l = lane_id(); l < a.m; l += kWave) {
        const int pl = bin_pos(l);
        const float v = fmaf(rf.af, (float)w.bins[pl], bl[pl]);
        c += fabsf(v - rintf(v)) > rf.efast + fabsf(v) * 0x1.0p-20f ? 0u : 1u;
    }
    return c;
}

// SRP fast path: the bit of a component is certain when |sum| exceeds the
// truncation bound, else it is counted.
__device__ __forceinline__ unsigned fast_near_srp(const HashArgs &a, const WaveLds &w,
                                                  const RowFix &rf)
{
    unsigned c = 0;
    for (int32_t l = lane_id(); l < a.m; l += kWave)
        c += abs(w.bins[bin_pos(l)]) <= rf.eunits ? 1u : 0u;
    return c;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// FP64 value of component l of row `row`, summed in ascending coordinate
// order exactly as an FP64 evaluation of the definition would, by one lane.
template <int DT>
__device__ double exact_component_lane(const HashArgs &a, const uint32_t *tab, int64_t row,
                                       double scale, int32_t l)
{
    double y = 0.0;
    const uint32_t p0 = a.csr_off[l], p1 = a.csr_off[l + 1];
    for (uint32_t p = p0; p < p1; ++p) {
        const uint32_t j = a.csr_idx[p];
        const double xv = __dmul_rn(scale, (double)scalar_value<DT>(a.x, row * a.ld + j));
        y = __dadd_rn(y, (tab[j] >> 31) ? -xv : xv);
    }
    return y;
}

// A step of 64 components with more flagged ones than this evaluates them
// lane by lane, in parallel (each lane's dependent loads then overlap the
// others'); fewer are evaluated one after another by the whole wave.
constexpr int kWaveEvalMax = 16;

// FP64 value of component l (the same in every lane) of row `row`, summed
// in ascending coordinate order exactly as an FP64 evaluation of the
// definition would, by the whole wave: each lane loads one term of the bin
// (64 at a time, the coordinates from the bin table), then the terms are
// added in order through readlane.  Every term scale * x_j is exact in FP64.
template <int DT>
__device__ double exact_component_wave(const HashArgs &a, const uint32_t *tab, int64_t row,
                                       double scale, int32_t l)
{
    const int lane = lane_id();
    const uint32_t p0 = a.csr_off[l], p1 = a.csr_off[l + 1];
    double y = 0.0;
    for (uint32_t p = p0; p < p1; p += kWave) {
        const uint32_t cnt = min(p1 - p, (uint32_t)kWave);
        double t = 0.0;
        if ((uint32_t)lane < cnt) {
            const uint32_t j = a.csr_idx[p + lane];
            const double xv = __dmul_rn(scale, (double)scalar_value<DT>(a.x, row * a.ld + j));
            t = (tab[j] >> 31) ? -xv : xv;
        }
        for (uint32_t q = 0; q < cnt; ++q)
            y = __dadd_rn(y, readlane_f64(t, (int)q));
    }
    return y;
}

// ------------------------------------------------------------- the epilogue

// Fast-path code of E2LSH component l (Definition CS_Eucl_LSH):
// floor((sqrt(m) y + b)/w) in FP32; bl holds b / w and the row factor
// sqrt(m) * scale * 2^-k / w is folded into rf.af.
__device__ __forceinline__ int32_t e2lsh_code_fast(const WaveLds &w, const float *bl,
                                                   const RowFix &rf, int32_t l, bool count,
                                                   unsigned &nsat)
{
    const int pl = bin_pos(l);
    const float v = fmaf(rf.af, (float)w.bins[pl], bl[pl]);
    unsigned sat = 0;
    const int32_t ci = floor_to_i32((double)floorf(v), sat);
    if (count)
        nsat += sat;
    return ci;
}

// Recheck: the E2LSH codes of the row, lane per component, 64 components
// per step, each code written over its bin in LDS.  An FP32 screen takes
// the fast path's value v = (sqrt(m) y + b) / w and its error bound
// (rf.efast, one unit wider for the FP64 reference's own rounding; the FP32
// rounding of b / w lies inside the 2^-20 term).  Outside the bound floor(v)
// is the FP64 evaluation's code; the components of a step inside it (a NaN,
// infinite or |v| >= 2^23 value always is) are evaluated one after another
// by the whole wave in FP64 from the stored values.
template <int DT>
__device__ void recheck_e2lsh_codes(const HashArgs &a, const uint32_t *tab, const WaveLds &w,
                                    const float *bl, int64_t row, const RowFix &rf,
                                    unsigned &nflag, unsigned &nchg, unsigned &nsat)
{
    const int lane = lane_id();
    for (int32_t l0 = 0; l0 < a.m; l0 += kWave) {
        const int32_t l = l0 + lane;
        const bool in = l < a.m;
        const int pl = bin_pos(in ? l : l0);
        const int32_t isum = w.bins[pl];
        const float v32 = fmaf(rf.af, (float)isum, bl[pl] * a.inv_w32);
        double cd = (double)floorf(v32);
        double y = (double)isum * rf.s2k;
        const bool near = in && !(fabsf(v32 - rintf(v32)) >
                                  rf.efast + rf.af + fabsf(v32) * 0x1.0p-20f);
        auto take = [&](double ye) {
            const double ce = floor(__dadd_rn(__dmul_rn(a.alpha64, ye), (double)bl[pl]) / a.w64);
            ++nflag;
            nchg += ce != cd;
            cd = ce;
            y = ye;
        };
        const uint64_t flagged = __ballot(near);
        if (__popcll(flagged) > kWaveEvalMax) {
            if (near)
                take(exact_component_lane<DT>(a, tab, row, (double)rf.scale, l));
        } else {
            for (uint64_t fl = flagged; fl; fl &= fl - 1) {
                const int q = (int)__builtin_ctzll(fl);
                const double ye =
                    exact_component_wave<DT>(a, tab, row, (double)rf.scale, l0 + q);
                if (lane == q)
                    take(ye);
            }
        }
        if (in) {
            unsigned sat = 0;
            const int32_t ci = floor_to_i32(cd, sat);
            nsat += sat;
            if (a.codes)
                a.codes[row * a.m + l] = ci;
            if (a.proj)
                a.proj[row * a.m + l] = (float)y;
            w.bins[pl] = ci; // this step's bins were read above
        }
    }
}

// floor(v) as int32 in one instruction (v_cvt_flr_i32_f32); callers pass
// values well inside the int32 range.
__device__ __forceinline__ int32_t cvt_flr_i32(float v)
{
    int32_t r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Key of table t for a row whose codes are all known to lie in [-128, 127]
// (the caller's bound): code = floor(af * sum + b/w), the same FP32 value as
// the checked path, packed as two's-complement bytes with v_perm and mixed
// 8 codes per word (the narrow form of the key definition).
template <int KC>
__device__ __forceinline__ uint64_t e2lsh_narrow_key(const WaveLds &w, const float *bl,
                                                     const uint64_t *hinit, int t, float af)
{
    const int32_t l0 = t * KC;
    uint64_t h = hinit[2 * t];
#pragma unroll
    for (int q = 0; q < KC / 8; ++q) {
        uint32_t wd[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            int32_t c[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pl = bin_pos(l0 + 8 * q + 4 * hh + r);
                c[r] = cvt_flr_i32(fmaf(af, (float)w.bins[pl], bl[pl]));
            }
            const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)c[1], (uint32_t)c[0], 0x0c0c0400u);
            const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)c[3], (uint32_t)c[2], 0x0c0c0400u);
            wd[hh] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
        }
        h = mix64(h ^ (((uint64_t)wd[1] << 32) | (uint64_t)wd[0]));
    }
    return h;
}

// SRP key of table t from the signs of its K bins: bit r = [sum > 0], taken
// as med3(sum, 0, 1) and or-ed in place (two instructions per bit).
template <int KC>
__device__ __forceinline__ uint64_t srp_key(const WaveLds &w, int t)
{
    const int32_t l0 = t * KC;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int r = 0; r < KC; ++r) {
        const int32_t isum = w.bins[bin_pos(l0 + r)];
        const uint32_t bit = (uint32_t)min(max(isum, 0), 1);
        if (r < 32)
            lo |= bit << r;
        else
            hi |= bit << (r - 32);
    }
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ uint64_t srp_key_any(const HashArgs &a, const WaveLds &w, int t)
{
    const int32_t l0 = t * a.K;
    uint64_t v = 0;
    for (int r = 0; r < a.K; ++r) {
        const int32_t isum = w.bins[bin_pos(l0 + r)];
        v |= (uint64_t)(uint32_t)min(max(isum, 0), 1) << r;
    }
    return v;
}

// Fast-path table key (no recheck), K known at compile time.  Codes are
// floor(af * sum + b/w) with af = sqrt(m) * scale * 2^-k / w folded into one
// FMA; narrow tuples (all codes in [-128, 127], the common case) are packed
// four codes per dword with v_cvt_pk_u8_f32 on code + 128 (then XOR 0x80
// per byte gives the two's-complement byte of the key definition).
template <int KC>
__device__ __forceinline__ uint64_t e2lsh_fast_key(const HashArgs &a, const WaveLds &w,
                                                   const float *bl, const uint64_t *hinit, int t,
                                                   float af, int64_t row, unsigned &nsat)
{
    const int32_t l0 = t * KC;
    float c[KC];
#pragma unroll
    for (int r = 0; r < KC; ++r) {
        const int pl = bin_pos(l0 + r);
        c[r] = floorf(fmaf(af, (float)w.bins[pl], bl[pl]));
    }
    float mn = c[0], mx = c[0];
#pragma unroll
    for (int r = 1; r < KC; ++r) {
        mn = fminf(mn, c[r]);
        mx = fmaxf(mx, c[r]);
    }
    if (a.codes) {
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            unsigned s2 = 0;
            a.codes[row * a.m + l0 + r] = floor_to_i32((double)c[r], s2);
        }
    }
    if (mn >= -128.0f && mx <= 127.0f) {
        uint64_t h = hinit[2 * t];
#pragma unroll
        for (int q = 0; q < KC / 8; ++q) {
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                lo = __builtin_amdgcn_cvt_pk_u8_f32(c[8 * q + r] + 128.0f, r, lo);
                hi = __builtin_amdgcn_cvt_pk_u8_f32(c[8 * q + 4 + r] + 128.0f, r, hi);
            }
            const uint64_t W = ((uint64_t)(hi ^ 0x80808080u) << 32) | (uint64_t)(lo ^ 0x80808080u);
            h = mix64(h ^ W);
        }
        return h;
    }
    // wide tuple (rare): 32-bit codes, saturated to int32
    return e2lsh_key(KC, hinit[2 * t], hinit[2 * t + 1], [&](int r, bool first) {
        unsigned s2 = 0;
        int32_t ci = floor_to_i32((double)c[r], s2);
        if (first)
            nsat += s2;
        return ci;
    });
}

template <int DT, bool RECHECK>
__device__ void epilogue_e2lsh(const HashArgs &a, const uint32_t *tab, const WaveLds &w,
                               const float *bl, const uint64_t *hinit, int64_t row, int slot,
                               const RowFix &rf, bool narrow, unsigned &nflag, unsigned &nchg,
                               unsigned &nsat)
{
    const int lane = lane_id();
    if constexpr (RECHECK) {
        recheck_e2lsh_codes<DT>(a, tab, w, bl, row, rf, nflag, nchg, nsat);
        wave_sync();
        for (int t = lane; t < a.L; t += kWave) {
            const int32_t l0 = t * a.K;
            const uint64_t key = e2lsh_key(a.K, hinit[2 * t], hinit[2 * t + 1],
                                           [&](int r, bool) { return w.bins[bin_pos(l0 + r)]; });
            if (a.keys)
                emit_key(a, t, row, slot, key);
        }
        return;
    } else {
        if (a.counters)
            nflag += fast_near_e2lsh(a, w, bl, rf);
        if (a.proj) {
            for (int32_t l = lane; l < a.m; l += kWave)
                a.proj[row * a.m + l] = (float)w.bins[bin_pos(l)] * rf.fs;
        }
        if (narrow && !a.codes && (a.K == 16 || a.K == 8)) {
            for (int t = lane; t < a.L; t += kWave) {
                const uint64_t key = a.K == 16 ? e2lsh_narrow_key<16>(w, bl, hinit, t, rf.af)
                                               : e2lsh_narrow_key<8>(w, bl, hinit, t, rf.af);
                if (a.keys)
                    emit_key(a, t, row, slot, key);
            }
            return;
        }
        if (a.K == 16 || a.K == 8) {
            for (int t = lane; t < a.L; t += kWave) {
                uint64_t key = a.K == 16 ? e2lsh_fast_key<16>(a, w, bl, hinit, t, rf.af, row, nsat)
                                         : e2lsh_fast_key<8>(a, w, bl, hinit, t, rf.af, row, nsat);
                if (a.keys)
                    emit_key(a, t, row, slot, key);
            }
            return;
        }
    }
    for (int t = lane; t < a.L; t += kWave) {
        const int32_t l0 = t * a.K;
        uint64_t key = e2lsh_key(a.K, hinit[2 * t], hinit[2 * t + 1], [&](int r, bool first) {
            const int32_t c = e2lsh_code_fast(w, bl, rf, l0 + r, first, nsat);
            if (first && a.codes)
                a.codes[row * a.m + l0 + r] = c;
            return c;
        });
        if (a.keys)
            emit_key(a, t, row, slot, key);
    }
}

// SRP family: bit = [y > 0] (Definition cs_consine_lsh).  The fixed-point sum
// has the sign of y except within its error bound of 0 (rechecked on request).
template <int DT, bool RECHECK>
__device__ void epilogue_srp(const HashArgs &a, const uint32_t *tab, const WaveLds &w, int64_t row,
                             int slot, const RowFix &rf, unsigned &nflag, unsigned &nchg)
{
    const int lane = lane_id();
    if constexpr (!RECHECK) {
        if (a.counters)
            nflag += fast_near_srp(a, w, rf);
        if (!a.codes && !a.proj) {
            if (a.keys) {
                for (int t = lane; t < a.L; t += kWave) {
                    uint64_t v;
                    if (a.K == 16)
                        v = srp_key<16>(w, t);
                    else if (a.K == 8)
                        v = srp_key<8>(w, t);
                    else if (a.K == 32)
                        v = srp_key<32>(w, t);
                    else
                        v = srp_key_any(a, w, t);
                    emit_key(a, t, row, slot, v);
                }
            }
            return;
        }
    }
    const int ngroups = (a.m + kWave - 1) / kWave;
    // ballot of group g is kept by lane g % 64 and written out every 64 groups
    uint64_t mine = 0;
    for (int g = 0; g < ngroups; ++g) {
        int32_t l = g * kWave + lane;
        const bool in = l < a.m;
        const int32_t isum = w.bins[bin_pos(in ? l : 0)];
        bool bit = in && isum > 0;
        float yout = 0.0f;
        if (a.proj)
            yout = (float)isum * rf.fs;
        if constexpr (RECHECK) {
            // the sign is certain outside the truncation bound, widened by one
            // unit for the FP64 reference's own rounding (below one unit while
            // c_max < 2^20); the others are evaluated by the whole wave
            double y64 = (double)isum * rf.s2k;
            const bool near = in && abs(isum) <= rf.eunits + 1;
            auto take = [&](double ye) {
                const bool be = ye > 0.0;
                ++nflag;
                nchg += be != bit;
                bit = be;
                y64 = ye;
            };
            const uint64_t flagged = __ballot(near);
            if (__popcll(flagged) > kWaveEvalMax) {
                if (near)
                    take(exact_component_lane<DT>(a, tab, row, (double)rf.scale, l));
            } else {
                for (uint64_t fl = flagged; fl; fl &= fl - 1) {
                    const int q = (int)__builtin_ctzll(fl);
                    const double ye =
                        exact_component_wave<DT>(a, tab, row, (double)rf.scale, g * kWave + q);
                    if (lane == q)
                        take(ye);
                }
            }
            yout = (float)y64;
        }
        if (in) {
            if (a.codes)
                a.codes[row * a.m + l] = bit ? 1 : 0;
            if (a.proj)
                a.proj[row * a.m + l] = yout;
        }
        const uint64_t bal = __ballot(bit);
        mine = lane == (g & (kWave - 1)) ? bal : mine;
        if ((g & (kWave - 1)) == kWave - 1 || g == ngroups - 1) {
            if (lane <= (g & (kWave - 1)))
                w.mask[(g & ~(kWave - 1)) + lane] = mine;
        }
    }
    wave_sync();
    for (int t = lane; t < a.L; t += kWave) {
        int32_t s0 = t * a.K;
        uint64_t v = w.mask[s0 >> 6] >> (s0 & 63);
        if ((s0 & 63) + a.K > 64)
            v |= w.mask[(s0 >> 6) + 1] << (64 - (s0 & 63));
        if (a.K < 64)
            v &= (1ull << a.K) - 1ull;
        if (a.keys)
            emit_key(a, t, row, slot, v);
    }
}

// ------------------------------------------------------------------ kernel

template <int DT, bool ALIGNED> constexpr int ALIGNED_VEC() { return ALIGNED ? Elem<DT>::per16 : 1; }

// CH: 16-byte chunks (ALIGNED) or single elements per lane per row; a row
// has at most 64 * CH of them, unless LONG: then the row is read in
// a.pieces pieces of 64 * CH chunks, the next piece prefetched.
//
// LDS image of a workgroup (offsets in HashArgs):
//   [wave regions: waves x wave_region bytes, each holding mpad int32 bins]
//   [table: tab_entries u32] [b/w or b: bin_pos(m) floats] [digest seeds]
//   [SRP masks: waves x ceil(m/64) u64]
template <int FAM, int DT, bool ALIGNED, bool RECHECK, int CH, bool LONG>
// registers capped so that two workgroups fit per CU (the LDS limit)
__global__ __launch_bounds__(LONG ? 1024 : 512) __attribute__((amdgpu_waves_per_eu(CH * ALIGNED_VEC<DT, ALIGNED>() <= 16 ? 4 : 1)))
void hash_kernel(HashArgs a)
{
    // (the kernel has no static LDS, so this array starts at LDS address 0
    // and byte offsets into it are LDS addresses)
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t *tab = (const uint32_t *)(lds + a.tab_off);
    float *bl = (float *)(lds + a.bl_off);
    uint64_t *hinit = (uint64_t *)(lds + a.hinit_off);

    const int tid = threadIdx.x;
    // wave index, made visibly uniform so the row cursor lives in SGPRs
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = lane_id();
    constexpr int VEC = ALIGNED ? Elem<DT>::per16 : 1;

    WaveLds w;
    const uint32_t region = (uint32_t)wid * (uint32_t)a.wave_region; // this wave's base
    w.bins = (int32_t *)(lds + region);
    w.mask = (uint64_t *)(lds + a.mask_off) + (size_t)wid * ((a.m + 63) / 64);

    // ---- prologue: zero every bin; build the table (rows padded to whole
    // chunks: coordinates past d point at their lane's trash slot); count
    // the bin populations in wave 0's region to get c_max; zero again
    const int nwv = blockDim.x / kWave;
    for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4)
        *(int4 *)(w.bins + l) = make_int4(0, 0, 0, 0);
    __syncthreads();
    uint32_t bad = 0;
    uint32_t *tabw = (uint32_t *)(lds + a.tab_off);
    for (int32_t j = tid; j < a.tab_entries; j += blockDim.x) {
        uint32_t ent;
        if (j < a.d) {
            ent = table_entry(a, j, bad);
            atomicAdd((int32_t *)(lds + (ent & 0x7fffffffu)), 1);
        } else {
            ent = (uint32_t)(bin_pos(a.m) + (j / VEC) % kWave) * 4u;
        }
        tabw[j] = ent;
    }
    if (FAM == LSH_E2LSH) {
        // fast path: b / w (the row factor folds 1/w in); recheck: b as given
        for (int32_t l = tid; l < a.m; l += blockDim.x)
            bl[bin_pos(l)] = RECHECK ? a.b[l] : a.b[l] * a.inv_w32;
        for (int32_t t = tid; t < 2 * a.L; t += blockDim.x)
            hinit[t] = mix64((uint64_t)t); // = F(2 * table + wide)
    }
    __syncthreads();
    uint32_t cm = 0;
    for (int32_t l = lane; l < a.m; l += kWave)
        cm = max(cm, (uint32_t)((const int32_t *)lds)[bin_pos(l)]);
    const uint32_t cmax = wave_max_u32(cm);
    __syncthreads();
    if (wid == 0)
        for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4)
            *(int4 *)(w.bins + l) = make_int4(0, 0, 0, 0);
    // invalid hash-state entries, counted once (every workgroup sees the same)
    if (blockIdx.x == 0 && a.counters) {
        const uint32_t nb = wave_sum(bad);
        if (lane == 0 && nb)
            atomicAdd(&a.counters[3], (unsigned long long)nb);
    }
    __syncthreads();
    (void)nwv;

    // terms are kept below 2^(31 - hr) with c_max < 2^hr: no bin overflows int32
    const int hr = cmax ? 32 - __clz(cmax) : 0;
    const int koff = 31 - hr;

    // ---- rows owned by this wave
    const int32_t nchunk = a.d / VEC; // d % VEC == 0 when ALIGNED
    const uint32_t offmask = (uint32_t)a.wave_region - 1u;

    unsigned nflag = 0, nchg = 0, nsat = 0;

    using T = typename Elem<DT>::T;
    using Buf = u32x4[CH];

    // Every lane issues exactly CH loads per row (chunks past the row end
    // re-read chunk 0 and are summed into trash), so the number of loads in
    // flight is static and each wait covers only the row being summed.
    auto load_row = [&](Buf &buf, int64_t row, int32_t piece = 0) {
        const T *xr = (const T *)a.x + row * a.ld;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            int32_t ch = (piece * CH + i) * kWave + lane;
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

    // table entries of this lane's chunks: kept in registers for the whole
    // kernel when there are at most 16 per lane
    auto load_entries = [&](int i, uint32_t *tw) { // i: chunk of the row (piece * CH + i)
        const uint32_t *te = tab + (i * kWave + lane) * VEC;
        if constexpr (VEC == 1) {
            tw[0] = te[0];
        } else {
#pragma unroll
            for (int q = 0; q < VEC / 4; ++q) {
                u32x4 v = *(const u32x4 *)(te + 4 * q);
                tw[4 * q + 0] = v[0];
                tw[4 * q + 1] = v[1];
                tw[4 * q + 2] = v[2];
                tw[4 * q + 3] = v[3];
            }
        }
    };
    constexpr bool kTabRegs = !LONG && CH * VEC <= 16;
    uint32_t treg[kTabRegs ? CH * VEC : 1];
    if constexpr (kTabRegs) {
#pragma unroll
        for (int i = 0; i < CH; ++i)
            load_entries(i, treg + i * VEC);
    }

    // 3. discretise and key.  k: the bins' scale (sum = bin * 2^-k), e: the
    // row's exponent (|x| < 2^e), mb: the bits of max|x|, nres: times the
    // bins were shifted right (each loses < 1 unit of 2^-k)
    auto finish_row = [&](int64_t row, int slot, int k, int e, uint32_t mb, int nres) {
        wave_sync();
        RowFix rf;
        rf.scale = row_scale_of<DT>(a, row);
        rf.s2k = ldexp((double)rf.scale, -k);
        rf.fs = (float)rf.s2k;
        rf.af = rf.fs * a.alpha32 * a.inv_w32;
        // the truncation leaves sum within c_max + nres units of y 2^k / scale
        // (each term truncates by < 1 unit, each shift by < 1).  The FP64
        // reference's own rounding, gamma_{c-1} * sum|terms| <= c_max^2 *
        // 2^(e-52), is below one unit: 2^(e+k) = 2^(31-hr) and c_max < 2^hr
        // with hr <= 16 (c_max <= d <= 32768).
        rf.eunits = (int32_t)(cmax + (uint32_t)nres);
        rf.efast = rf.af * (float)(cmax + (uint32_t)nres + 1u) + 0x1.0p-20f;
        // every code lies in [-128, 127] when sqrt(m) * scale * c_max * max|x| / w
        // < 126: |sum| <= c_max * max|x| * 2^k (terms truncate toward zero)
        // and b/w is in [0, 1); the margin covers the FP32 rounding of the bound
        const bool narrow = a.alpha32 * rf.scale * (float)cmax * __uint_as_float(mb) * a.inv_w32 <
                            126.0f;
        if constexpr (FAM == LSH_E2LSH)
            epilogue_e2lsh<DT, RECHECK>(a, tab, w, bl, hinit, row, slot, rf, narrow, nflag, nchg,
                                        nsat);
        else
            epilogue_srp<DT, RECHECK>(a, tab, w, row, slot, rf, nflag, nchg);
        wave_sync();
        for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4)
            *(int4 *)(w.bins + l) = make_int4(0, 0, 0, 0);
        wave_sync();
    };

    auto process_row = [&](const Buf &buf, int64_t row, int slot) {
        // 1. the row's largest magnitude -> exponent e (|x| < 2^e) -> k
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < CH; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                mx = fmaxf(mx, fabsf(chunk_value<DT, ALIGNED>(buf[i], e)));
        const uint32_t mb = wave_max_u32(__float_as_uint(mx));
        const int be = (int)((mb >> 23) & 0xffu);
        const int e = be == 0 ? -126 : be - 126;
        const int k = koff - e;

        // 2. signed fixed-point sums into this wave's bins: per element one
        // v_and_or (slot address), one XOR (sign), ldexp, convert, LDS add.
        // Entries come from registers (small rows) or are read one chunk
        // ahead of the adds (LDS returns in order, so waiting for a read
        // issued before the adds does not wait for the adds).
        auto add_chunk = [&](int i, const uint32_t *tw) {
#pragma unroll
            for (int e2 = 0; e2 < VEC; ++e2) {
                const uint32_t ent = tw[e2];
                const float v = chunk_value<DT, ALIGNED>(buf[i], e2);
                const float sv = __uint_as_float(__float_as_uint(v) ^ (ent & 0x80000000u));
                lds_add_i32((ent & offmask) | region, (int32_t)ldexpf(sv, k));
            }
        };
        if constexpr (kTabRegs) {
#pragma unroll
            for (int i = 0; i < CH; ++i)
                add_chunk(i, treg + i * VEC);
        } else {
            uint32_t tw[2][VEC];
            load_entries(0, tw[0]);
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                if (i + 1 < CH)
                    load_entries(i + 1, tw[(i + 1) & 1]);
                add_chunk(i, tw[i & 1]);
            }
        }

        finish_row(row, slot, k, e, mb, 0);
    };

    // Long rows, piece p of a row: the bins' scale k follows the largest
    // exponent seen so far (e_cur); when a piece raises it, the bins are
    // shifted right by the difference first (nres counts the shifts: each
    // floors a bin by less than one unit of the new 2^-k).  Terms then stay
    // below 2^(31 - hr) as in the single-piece path.
    int e_cur = 0, nres = 0;
    uint32_t mb_row = 0;
    auto piece = [&](const Buf &buf, int32_t p) {
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < CH; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                mx = fmaxf(mx, fabsf(chunk_value<DT, ALIGNED>(buf[i], e)));
        const uint32_t mb = wave_max_u32(__float_as_uint(mx));
        const int be = (int)((mb >> 23) & 0xffu);
        const int ep = be == 0 ? -126 : be - 126;
        if (p == 0) {
            e_cur = ep;
            nres = 0;
            mb_row = mb;
        } else {
            mb_row = max(mb_row, mb);
            if (ep > e_cur) {
                const int sh = min(ep - e_cur, 31);
                wave_sync();
                for (int32_t l = lane * 4; l < a.mpad; l += kWave * 4) {
                    int4 v = *(const int4 *)(w.bins + l);
                    v.x >>= sh;
                    v.y >>= sh;
                    v.z >>= sh;
                    v.w >>= sh;
                    *(int4 *)(w.bins + l) = v;
                }
                wave_sync();
                e_cur = ep;
                ++nres;
            }
        }
        const int k = koff - e_cur;
        uint32_t tw[2][VEC];
        load_entries(p * CH, tw[0]);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i + 1 < CH)
                load_entries(p * CH + i + 1, tw[(i + 1) & 1]);
#pragma unroll
            for (int e2 = 0; e2 < VEC; ++e2) {
                const uint32_t ent = tw[i & 1][e2];
                const float v = chunk_value<DT, ALIGNED>(buf[i], e2);
                const float sv = __uint_as_float(__float_as_uint(v) ^ (ent & 0x80000000u));
                lds_add_i32((ent & offmask) | region, (int32_t)ldexpf(sv, k));
            }
        }
    };


    // Rows: the workgroup takes blocks of RB consecutive rows, blocks strided
    // by the grid; wave w of the workgroup takes rows w, w + waves, ... of
    // each block, so all waves of the GPU read one contiguous window of X
    // that slides forward.  The keys of a block are staged in LDS and, after
    // a workgroup barrier, written as 256-byte runs per table (one store
    // instruction covers two tables): storing each row's L keys straight
    // from the lanes would touch L pages and L lines per instruction.
    // Row r' (the wave's next) is loaded before row r is processed (two
    // register buffers, alternated by unrolling the loop twice: RB / waves
    // is even); every load is unconditional, rows past the end re-read row
    // n - 1.  The cursor is kept in 32-bit scalars (n < 2^30 is checked on
    // the host).  Every wave runs every block of its workgroup, so the
    // barriers are uniform.
    const int32_t n32 = (int32_t)a.n;
    const int32_t per_wave = kRowsPerBlock / a.waves;
    const int32_t nblk = (n32 + kRowsPerBlock - 1) / kRowsPerBlock;
    const bool staged = a.keys && a.stage_stride;
    auto first_row = [&](int32_t b) {
        return __builtin_amdgcn_readfirstlane(b * kRowsPerBlock + wid);
    };
    auto clamp_row = [&](int32_t r) { return r < n32 ? r : n32 - 1; };
    int32_t blk = (int32_t)blockIdx.x;
    int32_t r0 = first_row(blk);
    Buf bufA, bufB;
    load_row(bufA, clamp_row(r0));
    for (; blk < nblk; blk += (int32_t)gridDim.x) {
        const int32_t base = blk * kRowsPerBlock;
        // long rows: pieces alternate between the buffers (a.pieces is even,
        // so every row starts in bufA); the next row's first piece is loaded
        // during the current row's last one
        for (int32_t j = 0; LONG && j < per_wave; ++j) {
            const int32_t rn = j + 1 < per_wave ? r0 + a.waves : first_row(blk + (int32_t)gridDim.x);
            for (int32_t p = 0; p < a.pieces; p += 2) {
                load_row(bufB, clamp_row(r0), p + 1);
                if (r0 < n32)
                    piece(bufA, p);
                if (p + 2 < a.pieces)
                    load_row(bufA, clamp_row(r0), p + 2);
                else
                    load_row(bufA, clamp_row(rn), 0);
                if (r0 < n32)
                    piece(bufB, p + 1);
            }
            if (r0 < n32)
                finish_row(r0, r0 - base, koff - e_cur, e_cur, mb_row, nres);
            r0 = rn;
        }
        for (int32_t j = 0; !LONG && j < per_wave; j += 2) {
            const int32_t r1 = r0 + a.waves;
            load_row(bufB, clamp_row(r1));
            if (r0 < n32)
                process_row(bufA, r0, r0 - base);
            const int32_t r2 = j + 2 < per_wave ? r1 + a.waves : first_row(blk + (int32_t)gridDim.x);
            load_row(bufA, clamp_row(r2));
            if (r1 < n32)
                process_row(bufB, r1, r1 - base);
            r0 = r2;
        }
        if (staged) {
            __syncthreads();
            const int32_t total = a.L * kRowsPerBlock;
            for (int32_t q = tid; q < total; q += (int32_t)blockDim.x) {
                const int32_t t = q / kRowsPerBlock, i = q % kRowsPerBlock;
                if (base + i < n32)
                    a.keys[(int64_t)t * a.key_ld + base + i] =
                        *(const lds_u64 *)(size_t)stage_addr(a, t, i);
            }
            __syncthreads();
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
constexpr int kCsrThreads = 1024;
constexpr int kCsrWaves = kCsrThreads / kWave;
constexpr int kCsrWaveSort = 256; // largest bin whose coordinates one wave orders by rank

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    return x;
}

// Fallback for bins of more than kCsrWaveSort coordinates (a degenerate
// hash state): a bitonic sort of the (bin << 16 | coordinate) words of all
// coordinates in LDS, then each bin's start by binary search.
__device__ void csr_bitonic(const HashArgs &a, uint32_t *skeys, uint32_t *off, uint32_t *idx,
                            int p2)
{
    const int tid = threadIdx.x;
    uint32_t bad = 0, neg;
    for (int i = tid; i < p2; i += kCsrThreads)
        skeys[i] = i < a.d ? (table_bin(a, i, bad, neg) << 16) | (uint32_t)i : 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < p2; i += kCsrThreads) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t x = skeys[i], y = skeys[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        skeys[i] = y;
                        skeys[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int p = tid; p < a.d; p += kCsrThreads)
        idx[p] = skeys[p] & 0xffffu;
    for (int bin = tid; bin <= a.m; bin += kCsrThreads) {
        const uint32_t key = (uint32_t)bin << 16;
        int lo = 0, hi = a.d;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (skeys[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        off[bin] = (uint32_t)lo;
    }
}

// rank[q] += the number of the c list entries below v[q], for the first QN
// slots; eight LDS reads in flight per step (a lone read waits out the LDS
// latency), every lane reading the same address (one broadcast)
template <int QN>
__device__ __forceinline__ void csr_rank(const uint32_t *list, uint32_t c, const uint32_t *v,
                                         uint32_t *rank)
{
    uint32_t i = 0;
    for (; i + 8 <= c; i += 8) {
        uint32_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            x[u] = list[i + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < QN; ++q)
                rank[q] += x[u] < v[q] ? 1u : 0u;
    }
    for (; i < c; ++i) {
        const uint32_t x = list[i];
#pragma unroll
        for (int q = 0; q < QN; ++q)
            rank[q] += x < v[q] ? 1u : 0u;
    }
}

// The coordinates of each bin in ascending order (CSR: off[m + 1], idx[d])
// and the largest bin population, by one workgroup in LDS: a histogram of
// the bins, its exclusive scan, a placement of every coordinate at its bin's
// cursor (in any order), then each bin's coordinates put in ascending order
// by one wave (a coordinate's rank is the number of the bin's coordinates
// below it), and the list copied out.  A bin of more than kCsrWaveSort
// coordinates, or a list that does not fit beside the counts (lds_words),
// sends the table to the bitonic fallback.
// LDS: lds_words >= max(m + 1 + d, p2) words, or p2 alone.
__global__ __launch_bounds__(kCsrThreads) void csr_kernel(HashArgs a, uint32_t *off,
                                                          uint32_t *idx, uint32_t *cmax, int p2,
                                                          int lds_words)
{
    extern __shared__ uint32_t lds_csr[];
    __shared__ uint32_t wsum[kCsrWaves], wmax[kCsrWaves];
    uint32_t *cnt = lds_csr; // [m + 1]: counts, then cursors
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    uint32_t bad = 0, neg; // out-of-range entries are counted by the hash kernel
    for (int b = tid; b <= a.m; b += kCsrThreads)
        cnt[b] = 0;
    // the bins of this thread's coordinates j = tid + k * kCsrThreads, all
    // loads issued together (kept for the placement below)
    constexpr int kPer = kCsrMaxD / kCsrThreads;
    uint32_t jb[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * kCsrThreads;
        jb[k] = j < a.d ? table_bin(a, j, bad, neg) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (tid + k * kCsrThreads < a.d)
            atomicAdd(&cnt[jb[k]], 1u);
    __syncthreads();

    // exclusive scan: thread t owns bins [t * per, t * per + per)
    const int per = (a.m + kCsrThreads - 1) / kCsrThreads;
    const int b0 = tid * per;
    uint32_t tot = 0, mx = 0;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < a.m) {
            tot += cnt[b];
            mx = max(mx, cnt[b]);
        }
    }
    const uint32_t incl = wave_incl_scan_u32(tot);
    const uint32_t wm = wave_max_u32(mx);
    if (lane == kWave - 1)
        wsum[wid] = incl;
    if (lane == 0)
        wmax[wid] = wm;
    __syncthreads();
    uint32_t run = incl - tot, cm = 0;
    for (int w = 0; w < kCsrWaves; ++w) {
        run += w < wid ? wsum[w] : 0u;
        cm = max(cm, wmax[w]);
    }
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < a.m) {
            const uint32_t c = cnt[b];
            off[b] = run;
            cnt[b] = run;
            run += c;
        }
    }
    if (tid == 0) {
        off[a.m] = (uint32_t)a.d;
        *cmax = cm;
    }
    __syncthreads();
    // uniform: every thread read the same wmax
    if (cm > (uint32_t)kCsrWaveSort || a.m + 1 + a.d > lds_words) {
        csr_bitonic(a, lds_csr, off, idx, p2);
        return;
    }

    // placement at the cursors (order inside a bin still arbitrary)
    uint32_t *il = lds_csr + a.m + 1;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * kCsrThreads;
        if (j < a.d)
            il[atomicAdd(&cnt[jb[k]], 1u)] = (uint32_t)j;
    }
    __syncthreads(); // cnt[b] is now the end of bin b

    // one wave per bin: its coordinates in registers, ranked against the
    // bin's list (one broadcast LDS read per coordinate), written in order
    constexpr int Q = kCsrWaveSort / kWave;
    for (int b = wid; b < a.m; b += kCsrWaves) {
        const uint32_t o = b ? cnt[b - 1] : 0u, c = cnt[b] - o;
        if (c < 2)
            continue;
        uint32_t v[Q], rank[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t i = (uint32_t)(q * kWave + lane);
            v[q] = il[o + min(i, c - 1u)];
            rank[q] = 0;
        }
        // compares only for the slots that hold coordinates (c is uniform)
        switch ((c + kWave - 1) / kWave) {
        case 1: csr_rank<1>(il + o, c, v, rank); break;
        case 2: csr_rank<2>(il + o, c, v, rank); break;
        case 3: csr_rank<3>(il + o, c, v, rank); break;
        default: csr_rank<4>(il + o, c, v, rank); break;
        }
        wave_sync(); // every lane has read the bin before any lane writes it
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if ((uint32_t)(q * kWave + lane) < c)
                il[o + rank[q]] = v[q];
        wave_sync();
    }
    __syncthreads();
    for (int p = tid; p < a.d; p += kCsrThreads)
        idx[p] = il[p];
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

// dry: set the kernel up and size its grid without launching it, so that a
// failure is reported before any kernel of the call is enqueued.
template <int FAM, int DT, bool AL, bool RC, int CH, bool LONG = false>
hipError_t launch_one(const HashArgs &a, int block, size_t lds, hipStream_t st, int64_t nblk,
                      bool dry)
{
    auto k = hash_kernel<FAM, DT, AL, RC, CH, LONG>;
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
    int64_t want = nblk; // one block of RB rows per workgroup step
    int64_t cap = (int64_t)device_cu_count() * per_cu;
    int grid = (int)(want < cap ? want : cap);
    if (dry)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

// Chunks per lane: aligned rows of at most 256 chunks are held whole (CH =
// 1, 2 or 4); longer ones are read in pieces of 1024 elements (CH = 16 /
// elements per chunk).  Unaligned rows take 8 elements per lane, whole or
// per piece.
template <int DT, bool AL> constexpr int long_ch() { return AL ? 16 / Elem<DT>::per16 : 8; }

template <int FAM, int DT, bool AL, bool RC>
hipError_t launch_ch(const HashArgs &a, int ch, int block, size_t lds, hipStream_t st, int64_t nblk,
                     bool dry)
{
    if (a.pieces > 1)
        return launch_one<FAM, DT, AL, RC, long_ch<DT, AL>(), true>(a, block, lds, st, nblk, dry);
    if constexpr (AL) {
        switch (ch) {
        case 1:
            return launch_one<FAM, DT, AL, RC, 1>(a, block, lds, st, nblk, dry);
        case 2:
            return launch_one<FAM, DT, AL, RC, 2>(a, block, lds, st, nblk, dry);
        default:
            return launch_one<FAM, DT, AL, RC, 4>(a, block, lds, st, nblk, dry);
        }
    } else {
        return launch_one<FAM, DT, AL, RC, 8>(a, block, lds, st, nblk, dry);
    }
}

template <int FAM, int DT>
hipError_t launch_dt(const HashArgs &a, bool al, bool rc, int ch, int block, size_t lds,
                     hipStream_t st, int64_t nblk, bool dry)
{
    if (al)
        return rc ? launch_ch<FAM, DT, true, true>(a, ch, block, lds, st, nblk, dry)
                  : launch_ch<FAM, DT, true, false>(a, ch, block, lds, st, nblk, dry);
    return rc ? launch_ch<FAM, DT, false, true>(a, ch, block, lds, st, nblk, dry)
              : launch_ch<FAM, DT, false, false>(a, ch, block, lds, st, nblk, dry);
}

template <int FAM>
hipError_t launch_fam(const HashArgs &a, int dt, bool al, bool rc, int ch, int block, size_t lds,
                      hipStream_t st, int64_t nblk, bool dry)
{
    switch (dt) {
    case LSH_F32:
        return launch_dt<FAM, LSH_F32>(a, al, rc, ch, block, lds, st, nblk, dry);
    case LSH_BF16:
        return launch_dt<FAM, LSH_BF16>(a, al, rc, ch, block, lds, st, nblk, dry);
    default:
        return launch_dt<FAM, LSH_FP8_E4M3FN>(a, al, rc, ch, block, lds, st, nblk, dry);
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
    if (c->recheck < 0 || c->recheck > 2)
        LSH_FAIL(LSH_EINVAL, "recheck must be 0, 1 or 2 (got %d)", c->recheck);
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
    if (pts->n >= ((int64_t)1 << 30))
        LSH_FAIL(LSH_EINVAL, "n = %lld points: hash at most 2^30 - 1 per call", (long long)pts->n);

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
    a.comp_slot = disc->comp_slot;
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
    const int ch_whole = al ? 4 : 8; // the most a lane holds of a whole row
    while (ch < ch_whole && 64 * ch < nch)
        ch <<= 1;
    if (!al)
        ch = 8;
    a.pieces = 1;
    if (64 * ch < nch) { // read the row in pieces of 64 * ch chunks (an even count)
        ch = al ? 16 / per16 : 8;
        a.pieces = (int32_t)((nch + 64 * ch - 1) / (64 * ch));
        a.pieces += a.pieces & 1;
    }

    // LDS layout: per-wave regions of a power-of-two size (so a slot's
    // address is offset | region base), then the shared table and constants
    a.mpad = (int32_t)align_up((size_t)bin_pos(a.m) + kTrashSlots, 4);
    int region = 256;
    while (region < a.mpad * 4)
        region <<= 1;
    a.wave_region = region;
    const int vec = al ? per16 : 1;
    a.tab_entries = 64 * ch * vec * a.pieces;
    const size_t lds_max = 160 * 1024;
    const int64_t nblk = (pts->n + kRowsPerBlock - 1) / kRowsPerBlock;
    const size_t masks = (size_t)((a.m + 63) / 64) * 8;
    // key staging: ceil(L / waves) tables (rounded up to a power of two) per
    // chunk of RB + 1 keys each, chunk c in the unused tail of wave c's
    // region when it fits there, else in an area of its own
    bool stage_on = out->keys != nullptr;
    auto stage_for = [&](int wv, size_t area_off) -> size_t {
        a.stage_base = a.stage_stride = a.stage_tpc_log2 = 0;
        if (!stage_on)
            return 0;
        int lg = 0;
        while ((1 << lg) * wv < a.L)
            ++lg;
        const size_t chunk = (size_t)(1 << lg) * (kRowsPerBlock + 1) * 8;
        const size_t nchunk = (size_t)((a.L + (1 << lg) - 1) >> lg);
        a.stage_tpc_log2 = lg;
        if ((size_t)region - (size_t)a.mpad * 4 >= chunk) {
            a.stage_base = a.mpad * 4;
            a.stage_stride = region;
            return 0;
        }
        a.stage_base = (int32_t)area_off;
        a.stage_stride = (int32_t)chunk;
        return nchunk * chunk;
    };
    auto lds_for = [&](int wv) {
        size_t off = (size_t)wv * region;
        size_t tab = off;
        off += align_up((size_t)a.tab_entries * 4, 16);
        size_t blo = off;
        off += align_up((size_t)bin_pos(a.m) * 4, 16);
        size_t hio = off;
        off += align_up((size_t)a.L * 16, 16);
        size_t mo = off;
        off += (size_t)wv * masks;
        off = align_up(off, 16);
        off += stage_for(wv, off);
        a.tab_off = (int32_t)tab;
        a.bl_off = (int32_t)blo;
        a.hinit_off = (int32_t)hio;
        a.mask_off = (int32_t)mo;
        return off;
    };
    // more waves per workgroup amortise the table and build it sooner (also
    // for a few rows: waves without a row only help build it); fewer fit
    // more workgroups
    int waves = 8;
    while (waves > 1 && lds_for(waves) > lds_max)
        waves >>= 1;
    // long rows: their hash table (4 bytes per coordinate) is shared by the
    // workgroup, so sixteen waves may keep more waves resident per CU than
    // workgroups of eight that each hold a copy
    if (a.pieces > 1 && waves == 8 && lds_for(16) <= lds_max &&
        16 * (lds_max / lds_for(16)) > 8 * (lds_max / lds_for(8)))
        waves = 16;
    if (lds_for(waves) > lds_max && stage_on) {
        stage_on = false; // keys too many to stage: store them directly
        waves = 8;
        while (waves > 1 && lds_for(waves) > lds_max)
            waves >>= 1;
    }
    size_t lds = lds_for(waves);
    if (lds > lds_max)
        LSH_FAIL(LSH_EINVAL, "d=%d, m=%d, L=%d need %zu bytes of LDS (max %zu)", pts->d, a.m, a.L,
                 lds, lds_max);
    a.waves = waves;

    hipStream_t s = (hipStream_t)stream;
    auto launch_hash = [&](bool dry) {
        return disc->family == LSH_E2LSH
                   ? launch_fam<LSH_E2LSH>(a, pts->dtype, al, rc, ch, waves * kWave, lds, s, nblk, dry)
                   : launch_fam<LSH_SRP>(a, pts->dtype, al, rc, ch, waves * kWave, lds, s, nblk, dry);
    };
    hipError_t e = launch_hash(true);
    if (e != hipSuccess)
        LSH_FAIL(LSH_EHIP, "hash kernel set-up failed: %s", hip_msg(e));
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
        // recheck = 2: the workspace holds this table's CSR from an earlier call
        if (disc->recheck == 1) {
            // the rank-sort path keeps counts and list in LDS when they fit
            const size_t list_words = (size_t)a.m + 1 + (size_t)pts->d;
            const size_t lds_words =
                list_words * 4 <= 160 * 1024 ? std::max((size_t)p2, list_words) : (size_t)p2;
            const size_t clds = lds_words * 4;
            LSH_HIP(hipFuncSetAttribute((const void *)csr_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)clds));
            hipLaunchKernelGGL(csr_kernel, dim3(1), dim3(kCsrThreads), clds, s, a, (uint32_t *)a.csr_off,
                               (uint32_t *)a.csr_idx, cmax_ws, p2, (int)lds_words);
            LSH_LAUNCHED("csr_kernel");
        }
    }

    e = launch_hash(false);
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

namespace lsh {
namespace {

// Scratch of lsh_hash_cs_noalloc: the recheck's CSR of h at its largest
// (d = 32768 coordinates, m = 16384 bins), one copy per GPU for the life of
// the process.  In host code `scratch` names a host-side stand-in; only the
// address that hipGetSymbolAddress returns for the current device is used.
constexpr size_t kScratchBytes = 256 + 65792 + 131072;
static_assert(kScratchBytes >= 256 + ((16384 + 1) * 4 + 255) / 256 * 256 + kCsrMaxD * 4,
              "scratch too small for the largest recheck CSR");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up once per device.
lsh_status scratch_ptr(void **out)
{
    int dev = 0;
    LSH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        LSH_FAIL(LSH_EINVAL, "device %d is beyond the %d the static scratch supports", dev,
                 kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            LSH_FAIL(LSH_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                     hip_msg(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LSH_OK;
}

} // namespace
} // namespace lsh

extern "C" lsh_status lsh_hash_cs_noalloc(const lsh_points *pts, const uint32_t *h, const int8_t *s,
                                          const lsh_disc *disc, const lsh_out *out, void *stream)
{
    if (!h || !s)
        LSH_FAIL(LSH_EINVAL, "h and s are required");
    if (!pts || !disc)
        LSH_FAIL(LSH_EINVAL, "points and discretisation descriptors are required");
    void *ws = nullptr;
    size_t wsb = 0;
    if (disc->recheck == 2)
        LSH_FAIL(LSH_EINVAL, "recheck = 2 needs a workspace of the caller's (the static array is "
                             "shared by every call on the GPU)");
    if (disc->recheck) {
        if (pts->d < 1 || pts->d > lsh::kCsrMaxD || disc->m < 1 || disc->m > 16384)
            LSH_FAIL(LSH_EINVAL,
                     "no-allocation recheck needs 1 <= d <= %d and 1 <= m <= 16384 (d=%d m=%d)",
                     lsh::kCsrMaxD, pts->d, disc->m);
        wsb = lsh::ws_layout(pts->d, disc->m).total;
        if (wsb > lsh::kScratchBytes)
            LSH_FAIL(LSH_EINVAL, "recheck needs %zu bytes of scratch, the static array holds %zu",
                     wsb, lsh::kScratchBytes);
        lsh_status st = lsh::check_stream_device(stream);
        if (st == LSH_OK)
            st = lsh::scratch_ptr(&ws);
        if (st != LSH_OK)
            return st;
    }
    lsh::HashArgs a = {};
    a.hcs = 0;
    a.h = h;
    a.s = s;
    return lsh::hash_common(pts, a, disc, out, ws, wsb, stream);
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
