// Independent per-table sketches: L hash tables, each built from a count
// sketch (or a higher-order count sketch) of its own with K components.
//
// Section 6 of the paper builds every table from a separate small sketch
// (K components per table, L tables); the shared-sketch kernel in hash.hip
// instead splits one sketch of m = K L components into the L tables.  Here
// each coordinate j of a point adds s_t(j) x_j into bin h_t(j) of every
// table t: O(L d) additions per point against O(d) for the shared sketch.
//
// Layout and work split (gfx950, wave64):
//   * LDS holds the tables' state as one byte per (coordinate, table): the
//     bin h_t(j) < K in bits 0-5 and the sign in bit 7.  Four coordinates of
//     one table share a 32-bit word, and the words of one quad of
//     coordinates lie side by side over the tables, so lane t reads its
//     word with a conflict-free 32-bit load.
//   * One wave per point.  Lane t of group g (lane = g * Lp + t, Lp = L
//     rounded up to a power of two, G = 64 / Lp groups) owns table t's bins
//     for the coordinates of every G-th quad, so the 64 lanes add into 64
//     different bins per instruction.  For L > 32 there is one group.
//   * The bins are 64-bit fixed point: the point's values are scaled by 2^k
//     with 2^k * d * max|x| < 2^62, truncated to integers and summed with
//     64-bit LDS atomic adds.  The sum is exact in integer arithmetic and
//     independent of order; truncation leaves an error below c * 2^-k per bin
//     (c = its population), about 2^-48 * max|x| at d = 16384.  Each bin has
//     a slot for positive and one for negative terms (the byte holds
//     2 * bin + sign), so a term's LDS address is one shift-add of its byte
//     and no term is negated.
//   * The loop over a piece loads the next quad's table word and values
//     before it issues the current quad's four adds, so the adds (which
//     return nothing) never wait on a load.
//   * The point is staged in LDS as fixed-point integers in pieces of 256
//     coordinates, read by every lane of a group at the same address.
//   * Epilogue: lane t sums its groups' bins, converts them to FP64, applies
//     the row scale, and discretises in FP64: floor((sqrt(K) y + b) / w) or
//     y > 0.  The K codes form the table's key as in the shared path.
#include "lsh_internal.h"

namespace lsh {
namespace {

constexpr int kTabWavesMax = 8;
constexpr int kPiece = 256;      // coordinates staged per round
constexpr int kModesMax = 8;
constexpr size_t kTabLdsMax = 160 * 1024;

typedef __attribute__((address_space(3))) unsigned long long lds_u64;

struct TabArgs {
    const void *x;
    int64_t ld, n;
    int32_t d, lg_d;              // lg_d = ceil(log2 d)
    const float *row_scale;
    int32_t family, K, L, m, Lp, lgLp, G, nquad;
    int32_t hcs, N, mode_total;
    int32_t dk[kModesMax], mk[kModesMax], mode_off[kModesMax];
    const uint32_t *h;            // CS: [L][d]; HCS: [L][mode_total]
    const int8_t *s;
    const float *b;               // [m]
    double w64, alpha64;          // w, sqrt(K)
    uint64_t *keys;
    int64_t key_ld;
    int32_t *codes;
    float *proj;
    unsigned long long *counters;
    int32_t tab_bytes, wave_bytes, bins_words;
};

template <int DT> __device__ __forceinline__ float load_value(const void *x, int64_t idx)
{
    if constexpr (DT == LSH_F32)
        return ((const float *)x)[idx];
    else if constexpr (DT == LSH_BF16)
        return __uint_as_float((uint32_t)((const uint16_t *)x)[idx] << 16);
    else
        return __builtin_amdgcn_cvt_f32_fp8((int)((const uint8_t *)x)[idx], 0);
}

// Bin and sign of coordinate j in table t, packed as 2 * bin + sign.
// Entries out of range are taken as bin 0 and counted in `bad`.
__device__ __forceinline__ uint32_t tab_entry(const TabArgs &a, int t, int32_t j, uint32_t &bad)
{
    uint32_t bin, neg;
    if (!a.hcs) {
        const int64_t at = (int64_t)t * a.d + j;
        bin = a.h[at];
        neg = a.s[at] < 0;
    } else {
        // tensor index (i_1, ..., i_N) of j, first mode fastest (Eq. eqhcs)
        const int64_t base = (int64_t)t * a.mode_total;
        int32_t rest = j;
        uint32_t stride = 1;
        bin = 0;
        neg = 0;
        for (int k = 0; k < a.N; ++k) {
            const int32_t ik = rest % a.dk[k];
            rest /= a.dk[k];
            uint32_t hb = a.h[base + a.mode_off[k] + ik];
            if (hb >= (uint32_t)a.mk[k]) {
                ++bad;
                hb = 0;
            }
            bin += hb * stride;
            stride *= (uint32_t)a.mk[k];
            neg ^= a.s[base + a.mode_off[k] + ik] < 0;
        }
    }
    if (bin >= (uint32_t)a.K) {
        ++bad;
        bin = 0;
    }
    return 2 * bin + neg;
}

__device__ __forceinline__ float wave_max_abs(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int DT, int FAM>
__global__ __launch_bounds__(kTabWavesMax *kWave) void tables_kernel(TabArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t *tab = (uint32_t *)lds;
    unsigned char *wb = lds + a.tab_bytes + (size_t)wid * a.wave_bytes;
    int64_t *bins = (int64_t *)wb;                                  // [2K][64]
    int64_t *xq = (int64_t *)(wb + (size_t)a.bins_words * 8);       // [kPiece]
    int32_t *cstage = (int32_t *)(wb + (size_t)a.bins_words * 8);   // [Lp][K] codes (epilogue)

    // ---- table state in LDS; this wave's bins zeroed
    uint32_t bad = 0;
    for (int idx = tid; idx < a.nquad * a.Lp; idx += blockDim.x) {
        const int q = idx >> a.lgLp, t = idx & (a.Lp - 1);
        uint32_t word = 0;
        if (t < a.L)
            for (int r = 0; r < 4; ++r) {
                const int32_t j = 4 * q + r;
                if (j < a.d)
                    word |= tab_entry(a, t, j, bad) << (8 * r);
            }
        tab[idx] = word;
    }
    for (int i = lane; i < a.bins_words; i += kWave)
        bins[i] = 0;
    if (blockIdx.x == 0 && a.counters) { // out-of-range state, counted once per call
        const uint32_t nb = wave_sum(bad);
        if (lane == 0 && nb)
            atomicAdd(&a.counters[3], (unsigned long long)nb);
    }
    __syncthreads();

    const int g = lane >> a.lgLp, t = lane & (a.Lp - 1);
    // this lane's bins as an LDS-space pointer: slot r of lane l is word
    // r * 64 + l, so the 64 lanes' adds fall in 64 consecutive words of
    // each slot row and touch every bank exactly twice
    lds_u64 *mb = (lds_u64 *)(unsigned long long *)(bins + lane);
    typedef int64_t i64x2 __attribute__((ext_vector_type(2)));
    unsigned nsat = 0;

    for (int64_t row = (int64_t)blockIdx.x * nw + wid; row < a.n;
         row += (int64_t)gridDim.x * nw) {
        const int64_t rb = row * a.ld;
        float amax = 0.0f;
        for (int32_t j = lane; j < a.d; j += kWave)
            amax = fmaxf(amax, fabsf(load_value<DT>(a.x, rb + j)));
        amax = wave_max_abs(amax);
        int e = 0;
        frexpf(amax, &e); // amax < 2^e
        const int k = 62 - a.lg_d - e;

        for (int32_t base = 0; base < a.d; base += kPiece) {
#pragma unroll
            for (int c = 0; c < kPiece / kWave; ++c) {
                const int32_t j = base + lane + c * kWave;
                const float v = j < a.d ? load_value<DT>(a.x, rb + j) : 0.0f;
                xq[lane + c * kWave] = (int64_t)ldexpf(v, k);
            }
            wave_sync();
            const int q0 = base >> 2;
            const int nq = min((base + kPiece) >> 2, a.nquad) - q0; // quads in this piece
            const i64x2 *xv = (const i64x2 *)xq;
            // loads of quad qi of the piece (clamped to its last quad past the end)
            // Lanes of tables t >= L read all-zero words (bin 0, sign +) and
            // add into their own slots, which nothing reads: no lane is
            // masked off, so the adds need no branch and no wait.
            auto adds = [&](uint32_t word, i64x2 v01, i64x2 v23) {
                __atomic_fetch_add(mb + ((word & 0xffu) << 6), (unsigned long long)v01.x,
                                   __ATOMIC_RELAXED);
                __atomic_fetch_add(mb + (((word >> 8) & 0xffu) << 6), (unsigned long long)v01.y,
                                   __ATOMIC_RELAXED);
                __atomic_fetch_add(mb + (((word >> 16) & 0xffu) << 6), (unsigned long long)v23.x,
                                   __ATOMIC_RELAXED);
                __atomic_fetch_add(mb + ((word >> 24) << 6), (unsigned long long)v23.y,
                                   __ATOMIC_RELAXED);
            };
            int qi = g;
            int qc = min(qi, nq - 1);
            uint32_t wa = tab[((q0 + qc) << a.lgLp) + t];
            i64x2 a01 = xv[2 * qc], a23 = xv[2 * qc + 1];
            // two quads per trip, each loaded one step ahead of its adds
            for (; qi < nq; qi += 2 * a.G) {
                const int qb = min(qi + a.G, nq - 1);
                const uint32_t wb2 = tab[((q0 + qb) << a.lgLp) + t];
                const i64x2 b01 = xv[2 * qb], b23 = xv[2 * qb + 1];
                adds(wa, a01, a23);
                if (qi + a.G >= nq)
                    break;
                const int qa = min(qi + 2 * a.G, nq - 1);
                wa = tab[((q0 + qa) << a.lgLp) + t];
                a01 = xv[2 * qa];
                a23 = xv[2 * qa + 1];
                adds(wb2, b01, b23);
            }
            wave_sync();
        }

        // ---- epilogue: lane t of group 0 owns table t
        const double unscale =
            ldexp(1.0, -k) * (DT == LSH_F32 ? 1.0 : (double)a.row_scale[row]);
        if (g == 0 && t < a.L) {
            uint64_t key = 0;
            for (int r = 0; r < a.K; ++r) {
                int64_t sum = 0;
                for (int gg = 0; gg < a.G; ++gg) {
                    const int64_t *bb = bins + gg * a.Lp + t;
                    sum += bb[(2 * r) * kWave] - bb[(2 * r + 1) * kWave];
                }
                const double yr = (double)sum * unscale;
                if (a.proj)
                    a.proj[row * a.m + t * a.K + r] = (float)yr;
                int32_t code;
                if (FAM == LSH_E2LSH) {
                    const double v = a.alpha64 * yr + (double)a.b[t * a.K + r];
                    code = floor_to_i32(floor(v / a.w64), nsat);
                } else {
                    code = yr > 0.0 ? 1 : 0;
                    key |= (uint64_t)code << r;
                }
                if (a.codes)
                    a.codes[row * a.m + t * a.K + r] = code;
                if (FAM == LSH_E2LSH)
                    cstage[t * a.K + r] = code;
            }
            if (FAM == LSH_E2LSH)
                key = e2lsh_key(a.K, mix64((uint64_t)(2 * t)), mix64((uint64_t)(2 * t + 1)),
                                [&](int r, bool) { return cstage[t * a.K + r]; });
            if (a.keys)
                a.keys[(int64_t)t * a.key_ld + row] = key;
        }
        wave_sync();
        for (int i = lane; i < a.bins_words; i += kWave)
            bins[i] = 0;
        wave_sync();
    }
    if (a.counters && FAM == LSH_E2LSH) {
        const unsigned ns = wave_sum(nsat);
        if (lane == 0 && ns)
            atomicAdd(&a.counters[2], (unsigned long long)ns);
    }
}

int ceil_log2(int64_t v)
{
    int l = 0;
    while (((int64_t)1 << l) < v)
        ++l;
    return l;
}

template <int DT>
hipError_t launch_tables(const TabArgs &a, int waves, size_t lds, int64_t grid, hipStream_t s)
{
    const void *fn = a.family == LSH_E2LSH ? (const void *)tables_kernel<DT, LSH_E2LSH>
                                           : (const void *)tables_kernel<DT, LSH_SRP>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    if (a.family == LSH_E2LSH)
        hipLaunchKernelGGL((tables_kernel<DT, LSH_E2LSH>), dim3((unsigned)grid),
                           dim3(waves * kWave), lds, s, a);
    else
        hipLaunchKernelGGL((tables_kernel<DT, LSH_SRP>), dim3((unsigned)grid),
                           dim3(waves * kWave), lds, s, a);
    return hipGetLastError();
}

lsh_status tables_common(const lsh_points *pts, TabArgs a, const lsh_disc *disc,
                         const lsh_out *out, void *stream)
{
    lsh_status st;
    if ((st = check_points(pts)) != LSH_OK || (st = check_disc(disc)) != LSH_OK)
        return st;
    if (disc->comp_slot)
        LSH_FAIL(LSH_EINVAL, "comp_slot does not apply to per-table sketches");
    if (!out)
        LSH_FAIL(LSH_EINVAL, "output descriptor is NULL");
    const int64_t key_ld = out->key_ld ? out->key_ld : pts->n;
    if (out->keys && key_ld < pts->n)
        LSH_FAIL(LSH_EINVAL, "key_ld %lld < n %lld", (long long)key_ld, (long long)pts->n);
    if (disc->L > kWave)
        LSH_FAIL(LSH_EINVAL, "per-table sketches support L <= %d tables (L = %d)", kWave,
                 disc->L);
    if (pts->n == 0)
        return LSH_OK;
    a.x = pts->x;
    a.ld = pts->ld;
    a.n = pts->n;
    a.d = pts->d;
    a.lg_d = ceil_log2(pts->d);
    a.row_scale = pts->row_scale;
    a.family = disc->family;
    a.K = disc->K;
    a.L = disc->L;
    a.m = disc->m;
    a.lgLp = ceil_log2(disc->L);
    a.Lp = 1 << a.lgLp;
    a.G = kWave / a.Lp;
    a.nquad = (pts->d + 3) / 4;
    a.b = disc->b;
    a.w64 = disc->family == LSH_E2LSH ? (double)disc->w : 1.0;
    a.alpha64 = sqrt((double)disc->K);
    a.keys = out->keys;
    a.key_ld = key_ld;
    a.codes = out->codes;
    a.proj = out->proj;
    a.counters = (unsigned long long *)out->counters;
    a.bins_words = kWave * 2 * a.K; // [2K slots][64 lanes]
    const size_t stage = (size_t)(kPiece * 8 > a.Lp * a.K * 4 ? kPiece * 8 : a.Lp * a.K * 4);
    a.wave_bytes = (int32_t)align_up((size_t)a.bins_words * 8 + stage, 16);
    a.tab_bytes = (int32_t)align_up((size_t)a.nquad * a.Lp * 4, 16);
    int waves = kTabWavesMax;
    while (waves > 1 && (size_t)a.tab_bytes + (size_t)waves * a.wave_bytes > kTabLdsMax)
        --waves;
    const size_t lds = (size_t)a.tab_bytes + (size_t)waves * a.wave_bytes;
    if (lds > kTabLdsMax)
        LSH_FAIL(LSH_EINVAL,
                 "per-table state of d = %d coordinates x %d tables needs %zu bytes of LDS "
                 "(max %zu)",
                 pts->d, disc->L, lds, kTabLdsMax);
    const int64_t per_cu = (int64_t)(kTabLdsMax / lds);
    const int64_t want = (pts->n + waves - 1) / waves;
    const int64_t cap = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
    const int64_t grid = want < cap ? want : cap;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (pts->dtype == LSH_F32)
        e = launch_tables<LSH_F32>(a, waves, lds, grid, s);
    else if (pts->dtype == LSH_BF16)
        e = launch_tables<LSH_BF16>(a, waves, lds, grid, s);
    else
        e = launch_tables<LSH_FP8_E4M3FN>(a, waves, lds, grid, s);
    if (e != hipSuccess)
        LSH_FAIL(LSH_EHIP, "per-table hash kernel launch failed: %s", hip_msg(e));
    return LSH_OK;
}

} // namespace
} // namespace lsh

extern "C" lsh_status lsh_hash_cs_tables(const lsh_points *pts, const uint32_t *h,
                                         const int8_t *s, const lsh_disc *disc,
                                         const lsh_out *out, void *stream)
{
    if (!h || !s)
        LSH_FAIL(LSH_EINVAL, "h and s are required");
    lsh::TabArgs a = {};
    a.hcs = 0;
    a.h = h;
    a.s = s;
    return lsh::tables_common(pts, a, disc, out, stream);
}

extern "C" lsh_status lsh_hash_hcs_tables(const lsh_points *pts, int32_t N, const int32_t *d_k,
                                          const int32_t *m_k, const uint32_t *h_k,
                                          const int8_t *s_k, const lsh_disc *disc,
                                          const lsh_out *out, void *stream)
{
    if (N < 1 || N > lsh::kModesMax || !d_k || !m_k || !h_k || !s_k)
        LSH_FAIL(LSH_EINVAL, "HCS needs 1 <= N <= %d and the per-mode tables", lsh::kModesMax);
    lsh::TabArgs a = {};
    a.hcs = 1;
    a.N = N;
    a.h = h_k;
    a.s = s_k;
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
    a.mode_total = o;
    if (pts && D < pts->d)
        LSH_FAIL(LSH_EINVAL, "prod d_k = %lld < d = %d", (long long)D, pts->d);
    if (disc && M != disc->K)
        LSH_FAIL(LSH_EINVAL, "prod m_k = %lld != K = %d (each table's sketch has K components)",
                 (long long)M, disc->K);
    return lsh::tables_common(pts, a, disc, out, stream);
}
