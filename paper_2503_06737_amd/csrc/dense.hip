// Dense E2LSH / SRP on gfx950 FP32 matrix cores: the O(md) baseline
// (Section 3.1: E2LSH, Eq. datar_lsh, h(p) = floor((<r, p> + b)/w) with
// r ~ N(0, I); SRP, Definition srp, sgn(<r, p>)), m projections at once as
// Y = X R, followed by the same table-key epilogue as the sketch kernels.
//
// Tiling: a 256-thread workgroup computes a 128 x Wt tile of Y (Wt = the
// largest multiple of K not above 128, so every table lies in one tile) with
// v_mfma_f32_32x32x2f32; each wave owns a 64 x 64 quarter (2 x 2 blocks of
// 32 x 32, 64 accumulators per lane).  X and R tiles of depth 16 are staged
// in LDS (X transposed to k-major) with the next tile prefetched into
// registers while the current one is multiplied.  The workgroup index is
// remapped so that the column tiles of one row tile run back to back on the
// same XCD and share the X tile through that XCD's L2.  The epilogue spills
// the tile to LDS and turns each (row, table) into its key.

#include <math.h>

#include "lsh_internal.h"

namespace lsh {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBN = 128, kBK = 16;
constexpr int kDThreads = 256;
constexpr int kAStride = kBM + 4; // k-major X tile row stride (bank spread for the transposed store)
constexpr int kYStride = kBN + 1; // odd: the epilogue's lanes read one row each, all banks

struct DenseArgs {
    const float *x;
    int64_t ld;
    int64_t n;
    int32_t d;
    const float *R; // [d][m]
    int32_t m, K, L, family;
    int32_t tabs_per_tile, tile_w, ncol;
    int32_t xvec, rvec; // 16-byte loads allowed for X rows / R rows
    int64_t nrow_tiles, ntiles;
    float w32, inv_w32;
    int32_t w_pow2;
    const float *b;
    uint64_t *keys;
    int64_t key_ld;
    int32_t *codes;
    float *proj;
    unsigned long long *counters;
};

struct DenseSmem {
    union {
        struct {
            float a[2][kBK][kAStride];
            float b[2][kBK][kBN];
        } ld;
        float y[kBM][kYStride];
    };
    float bsh[kBN];        // the column tile's shifts b
    uint64_t seeds[kBN * 2]; // and its tables' digest seeds
};

// Epilogue shared by the dense kernels: y (the tile of X R, rows row0..,
// column tile ct) -> codes and keys, one (row, table) pair per thread and
// step.  row_factor(row) multiplies the tile's values (the row scale of
// low-precision points, 1 for FP32).
// floor(c) of an FP32 value, saturated to int32; *sat += 1 when it
// saturates (c is already integral: the saturation test needs no FP64).
__device__ __forceinline__ int32_t floorf_to_i32(float c, unsigned &sat)
{
    if (c >= 2147483648.0f) {
        ++sat;
        return 2147483647;
    }
    if (c < -2147483648.0f) {
        ++sat;
        return -2147483647 - 1;
    }
    return (int32_t)c;
}

template <typename RowFactor>
__device__ __forceinline__ void dense_epilogue(const DenseArgs &a, const float (*y)[kYStride],
                                               const float *bsh, const uint64_t *seeds,
                                               int64_t row0, int ct, RowFactor row_factor)
{
    const int tid = threadIdx.x;
    unsigned nsat = 0;
    const int npairs = kBM * a.tabs_per_tile;
    const bool outs = a.codes || a.proj;
    for (int p = tid; p < npairs; p += kDThreads) {
        const int tl = p / kBM, r = p % kBM;
        const int64_t row = row0 + r;
        const int t = ct * a.tabs_per_tile + tl;
        if (row >= a.n || t >= a.L)
            continue;
        const int c0 = tl * a.K;          // column in tile
        const int l0 = t * a.K;           // component
        const float f = row_factor(row);
        const float *yr = y[r] + c0;
        const float *br = bsh + c0;
        uint64_t key = 0;
        if (a.family == LSH_E2LSH) {
            // the narrow digest in words of 8 codes: the 8 values of a word
            // are read from LDS together (indices clamped into the table,
            // so every read is unconditional), then discretised and packed
            auto code_at = [&](float yv, float bv, unsigned &sat) {
                float v = yv * f + bv;
                float c = a.w_pow2 ? floorf(v * a.inv_w32) : floorf(v / a.w32);
                return floorf_to_i32(c, sat);
            };
            uint64_t h = seeds[2 * tl];
            bool narrow = true;
            for (int q0 = 0; q0 < a.K; q0 += 8) {
                float yv[8], bv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = min(q0 + e, a.K - 1);
                    yv[e] = yr[q];
                    bv[e] = br[q];
                }
                uint64_t W = 0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if (q0 + e < a.K) {
                        unsigned sat = 0;
                        const int32_t c = code_at(yv[e], bv[e], sat);
                        nsat += sat;
                        narrow &= (c >= -128) & (c <= 127);
                        W |= (uint64_t)(uint8_t)c << (8 * e);
                        if (outs) {
                            if (a.codes)
                                a.codes[row * a.m + l0 + q0 + e] = c;
                            if (a.proj)
                                a.proj[row * a.m + l0 + q0 + e] = yv[e] * f;
                        }
                    }
                }
                h = mix64(h ^ W);
            }
            if (narrow) {
                key = h;
            } else { // a code outside [-128, 127]: the wide digest (rare)
                unsigned sat = 0;
                key = e2lsh_key(a.K, 0, seeds[2 * tl + 1], [&](int q, bool first) {
                    return first ? 128 : code_at(yr[q], br[q], sat);
                });
            }
        } else {
            for (int q0 = 0; q0 < a.K; q0 += 8) {
                float yv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    yv[e] = yr[min(q0 + e, a.K - 1)];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if (q0 + e < a.K) {
                        const float yf = yv[e] * f;
                        const bool bit = yf > 0.0f;
                        key |= (uint64_t)bit << (q0 + e);
                        if (outs) {
                            if (a.codes)
                                a.codes[row * a.m + l0 + q0 + e] = bit ? 1 : 0;
                            if (a.proj)
                                a.proj[row * a.m + l0 + q0 + e] = yf;
                        }
                    }
                }
            }
        }
        if (a.keys)
            a.keys[(int64_t)t * a.key_ld + row] = key;
    }
    if (a.counters && nsat)
        atomicAdd(&a.counters[2], (unsigned long long)nsat);
}

// The column tile's shifts b and its tables' digest seeds F(2t), F(2t + 1)
// (E2LSH) into LDS, before the epilogue's barrier.
__device__ __forceinline__ void stage_shifts(const DenseArgs &a, float *bsh, uint64_t *seeds,
                                             int col0, int ct)
{
    if (a.family == LSH_E2LSH) {
        for (int c = threadIdx.x; c < a.tile_w; c += kDThreads)
            bsh[c] = col0 + c < a.m ? a.b[col0 + c] : 0.0f;
        for (int i = threadIdx.x; i < 2 * a.tabs_per_tile; i += kDThreads)
            seeds[i] = mix64(2ull * (uint64_t)(ct * a.tabs_per_tile) + (uint64_t)i);
    }
}

__global__ __launch_bounds__(kDThreads) void dense_kernel(DenseArgs a)
{
    __shared__ DenseSmem sm;
    // XCD-aware order: consecutive logical tiles share an XCD
    const int64_t nwg = gridDim.x;
    const int64_t per_xcd = nwg / 8;
    const int64_t lt = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (lt >= a.ntiles)
        return;
    const int64_t rt = lt / a.ncol;
    const int ct = (int)(lt % a.ncol);
    const int64_t row0 = rt * kBM;
    const int col0 = ct * a.tile_w;

    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int wr = (wid >> 1) * 64, wc = (wid & 1) * 64; // wave quarter

    // global -> register staging: X 128x16 (2 float4 per thread), R 16x128 (2 float4)
    float4 ra[2], rb[2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int idx = tid + i * kDThreads; // 0..511
            int r = idx >> 2, kq = (idx & 3) * 4;
            int64_t row = row0 + r;
            int k = k0 + kq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (row < a.n) {
                const float *p = a.x + row * a.ld + k;
                if (a.xvec && k + 3 < a.d) {
                    v = *(const float4 *)p;
                } else {
                    v.x = k + 0 < a.d ? p[0] : 0.f;
                    v.y = k + 1 < a.d ? p[1] : 0.f;
                    v.z = k + 2 < a.d ? p[2] : 0.f;
                    v.w = k + 3 < a.d ? p[3] : 0.f;
                }
            }
            ra[i] = v;
            int kk = idx >> 5, c4 = (idx & 31) * 4;
            int kr = k0 + kk, col = col0 + c4;
            float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
            if (kr < a.d) {
                const float *q = a.R + (int64_t)kr * a.m + col;
                int lim = col0 + a.tile_w < a.m ? col0 + a.tile_w : a.m;
                if (a.rvec && (col & 3) == 0 && col + 3 < lim) {
                    u = *(const float4 *)q;
                } else {
                    u.x = col + 0 < lim ? q[0] : 0.f;
                    u.y = col + 1 < lim ? q[1] : 0.f;
                    u.z = col + 2 < lim ? q[2] : 0.f;
                    u.w = col + 3 < lim ? q[3] : 0.f;
                }
            }
            rb[i] = u;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int idx = tid + i * kDThreads;
            int r = idx >> 2, kq = (idx & 3) * 4;
            sm.ld.a[buf][kq + 0][r] = ra[i].x;
            sm.ld.a[buf][kq + 1][r] = ra[i].y;
            sm.ld.a[buf][kq + 2][r] = ra[i].z;
            sm.ld.a[buf][kq + 3][r] = ra[i].w;
            int kk = idx >> 5, c4 = (idx & 31) * 4;
            *(float4 *)&sm.ld.b[buf][kk][c4] = rb[i];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[i][j][e] = 0.0f;

    const int nk = (a.d + kBK - 1) / kBK;
    gload(0);
    sstore(0);
    __syncthreads();
    const int li = lane & 31, lk = lane >> 5;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk)
            gload((kt + 1) * kBK);
#pragma unroll
        for (int ks = 0; ks < kBK / 2; ++ks) {
            const int k = ks * 2 + lk;
            float av0 = sm.ld.a[buf][k][wr + li];
            float av1 = sm.ld.a[buf][k][wr + 32 + li];
            float bv0 = sm.ld.b[buf][k][wc + li];
            float bv1 = sm.ld.b[buf][k][wc + 32 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv1, acc[1][1], 0, 0, 0);
        }
        if (kt + 1 < nk)
            sstore(buf ^ 1);
        __syncthreads();
    }

    // accumulators -> LDS tile: block (i, j), element e sits at
    // row 8*(e/4) + 4*(lane/32) + e%4, column lane%32 of the 32x32 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                int r = wr + i * 32 + 8 * (e >> 2) + 4 * lk + (e & 3);
                int c = wc + j * 32 + li;
                sm.y[r][c] = acc[i][j][e];
            }
    stage_shifts(a, sm.bsh, sm.seeds, col0, ct);
    __syncthreads();

    dense_epilogue(a, sm.y, sm.bsh, sm.seeds, row0, ct, [](int64_t) { return 1.0f; });
}


// ------------------------------------------------------------------ BF16

// Dense projection with BF16 operands on the gfx950 BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation): the same 128 x Wt tiles
// and epilogue as dense_kernel.  X holds BF16 codes with a row scale, R is
// given transposed (row l = the projection vector r_l, BF16), so both
// operands are read as 16-byte runs along k.
//
// A stage covers 128 values of k: each thread loads eight 16-byte runs of
// each operand into registers while the workgroup multiplies the previous
// stage out of LDS, so every wave keeps 16 loads in flight against 32 MFMAs
// of work (a stage of 32 left the loads' latency exposed).  The tiles sit in
// one LDS buffer, row-major with rows padded to 136 values (272 bytes), which
// spreads a quarter-wave's 16-byte reads over all banks.  Lane l reads the 8
// values k = 8 * (l / 32) .. + 7 of row (or column) l % 32 of its 32 x 32
// block for each k16 step; steps past d are skipped.
constexpr int kHK = 128;
constexpr int kHStride = kHK + 8;
constexpr int kHRuns = kBM * kHK / 8 / kDThreads; // 16-byte runs per thread and operand

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct DenseBf16Args {
    DenseArgs e;           // shapes, discretisation and outputs (x / R unused)
    const uint16_t *x;     // [n][ld] BF16 codes
    const float *scale;    // [n]
    const uint16_t *rt;    // [m][ldr] BF16
    int64_t ldr;
};

struct __align__(16) DenseBf16Smem {
    union {
        struct {
            uint16_t a[kBM][kHStride];
            uint16_t b[kBN][kHStride];
        } ld;
        float y[kBM][kYStride];
    };
    float bsh[kBN];        // the column tile's shifts b
    uint64_t seeds[kBN * 2]; // and its tables' digest seeds
};

__global__ __launch_bounds__(kDThreads) void dense_bf16_kernel(DenseBf16Args g)
{
    __shared__ DenseBf16Smem sm;
    const DenseArgs &a = g.e;
    const int64_t nwg = gridDim.x;
    const int64_t per_xcd = nwg / 8;
    const int64_t lt = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (lt >= a.ntiles)
        return;
    const int64_t rt = lt / a.ncol;
    const int ct = (int)(lt % a.ncol);
    const int64_t row0 = rt * kBM;
    const int col0 = ct * a.tile_w;
    const int lim = col0 + a.tile_w < a.m ? col0 + a.tile_w : a.m;

    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    const int wr = (wid >> 1) * 64, wc = (wid & 1) * 64;

    // global -> registers: 128 rows (columns) x 128 k of each operand, as
    // runs of 8 values
    uint4 ra[kHRuns], rb[kHRuns];
    auto run8 = [&](const uint16_t *p, int k, bool ok, bool vec) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (!ok || k >= a.d)
            return v;
        if (vec && k + 7 < a.d)
            return *(const uint4 *)p;
        uint16_t t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            t[e] = k + e < a.d ? p[e] : (uint16_t)0;
        v.x = t[0] | ((uint32_t)t[1] << 16);
        v.y = t[2] | ((uint32_t)t[3] << 16);
        v.z = t[4] | ((uint32_t)t[5] << 16);
        v.w = t[6] | ((uint32_t)t[7] << 16);
        return v;
    };
    // run i of this thread: row (column) r0 + 16 i, values kc .. kc + 7 of the stage
    const int r0 = tid >> 4, kc0 = (tid & 15) * 8;
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kHRuns; ++i) {
            const int r = r0 + 16 * i, k = k0 + kc0;
            const int64_t row = row0 + r;
            ra[i] = run8(g.x + row * a.ld + k, k, row < a.n, a.xvec);
            const int col = col0 + r;
            rb[i] = run8(g.rt + (int64_t)col * g.ldr + k, k, col < lim, a.rvec);
        }
    };
    // interior tiles (every row and column in range, 16-byte aligned runs,
    // d a multiple of 8): the address of run i is a uniform base plus this
    // lane's 32-bit offset, and only a stage that reaches past d tests k
    const bool fast = a.xvec && a.rvec && (a.d & 7) == 0 && row0 + kBM <= a.n &&
                      col0 + kBN <= a.m;
    const uint32_t xoff = (uint32_t)r0 * (uint32_t)a.ld + (uint32_t)kc0;
    const uint32_t roff = (uint32_t)r0 * (uint32_t)g.ldr + (uint32_t)kc0;
    auto gload_fast = [&](int k0, bool tail) {
#pragma unroll
        for (int i = 0; i < kHRuns; ++i) {
            const uint16_t *xa = g.x + (row0 + 16 * i) * a.ld + k0;
            const uint16_t *rb_ = g.rt + (int64_t)(col0 + 16 * i) * g.ldr + k0;
            if (!tail || k0 + kc0 < a.d) {
                ra[i] = *(const uint4 *)(xa + xoff);
                rb[i] = *(const uint4 *)(rb_ + roff);
            } else {
                ra[i] = make_uint4(0, 0, 0, 0);
                rb[i] = make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto load_stage = [&](int k0) {
        if (!fast)
            gload(k0);
        else if (k0 + kHK <= a.d)
            gload_fast(k0, false);
        else
            gload_fast(k0, true);
    };
    auto sstore = [&]() {
#pragma unroll
        for (int i = 0; i < kHRuns; ++i) {
            *(uint4 *)&sm.ld.a[r0 + 16 * i][kc0] = ra[i];
            *(uint4 *)&sm.ld.b[r0 + 16 * i][kc0] = rb[i];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[i][j][e] = 0.0f;

    const int nk = (a.d + kHK - 1) / kHK;
    const int li = lane & 31, lk = (lane >> 5) * 8;
    load_stage(0);
    for (int kt = 0; kt < nk; ++kt) {
        sstore();
        __syncthreads();
        if (kt + 1 < nk)
            load_stage((kt + 1) * kHK);
        const int nks = min(kHK, a.d - kt * kHK); // values of k in this stage
#pragma unroll
        for (int ks = 0; ks < kHK; ks += 16) {
            if (ks < nks) {
                const bf16x8 av0 = *(const bf16x8 *)&sm.ld.a[wr + li][ks + lk];
                const bf16x8 av1 = *(const bf16x8 *)&sm.ld.a[wr + 32 + li][ks + lk];
                const bf16x8 bv0 = *(const bf16x8 *)&sm.ld.b[wc + li][ks + lk];
                const bf16x8 bv1 = *(const bf16x8 *)&sm.ld.b[wc + 32 + li][ks + lk];
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av0, bv0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av0, bv1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av1, bv0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av1, bv1, acc[1][1], 0, 0, 0);
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                int r = wr + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                int c = wc + j * 32 + li;
                sm.y[r][c] = acc[i][j][e];
            }
    stage_shifts(a, sm.bsh, sm.seeds, col0, ct);
    __syncthreads();
    dense_epilogue(a, sm.y, sm.bsh, sm.seeds, row0, ct, [&](int64_t row) { return g.scale[row]; });
}

} // namespace lsh

extern "C" lsh_status lsh_hash_dense(const lsh_points *pts, const float *R, const lsh_disc *disc,
                                     const lsh_out *out, void *stream)
{
    using namespace lsh;
    lsh_status st;
    if ((st = check_points(pts)) != LSH_OK || (st = check_disc(disc)) != LSH_OK)
        return st;
    if (pts->dtype != LSH_F32)
        LSH_FAIL(LSH_EINVAL, "dense projection takes FP32 points");
    if (disc->recheck)
        LSH_FAIL(LSH_EINVAL, "recheck is not available for the dense projection");
    if (disc->comp_slot)
        LSH_FAIL(LSH_EINVAL, "comp_slot is not available for the dense projection "
                             "(permute the columns of R instead)");
    if (!R)
        LSH_FAIL(LSH_EINVAL, "R is NULL");
    if (!out)
        LSH_FAIL(LSH_EINVAL, "output descriptor is NULL");
    int64_t key_ld = out->key_ld ? out->key_ld : pts->n;
    if (out->keys && key_ld < pts->n)
        LSH_FAIL(LSH_EINVAL, "key_ld < n");
    if (pts->n == 0)
        return LSH_OK;
    DenseArgs a = {};
    a.x = (const float *)pts->x;
    a.ld = pts->ld;
    a.n = pts->n;
    a.d = pts->d;
    a.R = R;
    a.m = disc->m;
    a.K = disc->K;
    a.L = disc->L;
    a.family = disc->family;
    a.xvec = ((uintptr_t)pts->x % 16 == 0) && (pts->ld % 4 == 0);
    a.rvec = ((uintptr_t)R % 16 == 0) && (disc->m % 4 == 0);
    a.tabs_per_tile = kBN / disc->K;
    a.tile_w = a.tabs_per_tile * disc->K;
    a.ncol = (disc->L + a.tabs_per_tile - 1) / a.tabs_per_tile;
    a.nrow_tiles = (pts->n + kBM - 1) / kBM;
    a.ntiles = a.nrow_tiles * a.ncol;
    a.w32 = disc->family == LSH_E2LSH ? disc->w : 1.0f;
    a.inv_w32 = 1.0f / a.w32;
    int ex;
    a.w_pow2 = frexpf(a.w32, &ex) == 0.5f;
    a.b = disc->b;
    a.keys = out->keys;
    a.key_ld = key_ld;
    a.codes = out->codes;
    a.proj = out->proj;
    a.counters = (unsigned long long *)out->counters;
    int64_t grid = (a.ntiles + 7) / 8 * 8;
    if (grid > 0x7fffffff)
        LSH_FAIL(LSH_EINVAL, "too many tiles");
    hipLaunchKernelGGL(dense_kernel, dim3((unsigned)grid), dim3(kDThreads), 0, (hipStream_t)stream,
                       a);
    LSH_LAUNCHED("dense_kernel");
    return LSH_OK;
}

extern "C" lsh_status lsh_hash_dense_bf16(const lsh_points *pts, const uint16_t *Rt, int64_t ldr,
                                          const lsh_disc *disc, const lsh_out *out, void *stream)
{
    using namespace lsh;
    lsh_status st;
    if ((st = check_points(pts)) != LSH_OK || (st = check_disc(disc)) != LSH_OK)
        return st;
    if (pts->dtype != LSH_BF16)
        LSH_FAIL(LSH_EINVAL, "the BF16 dense projection takes BF16 points with row scales");
    if (disc->recheck)
        LSH_FAIL(LSH_EINVAL, "recheck is not available for the dense projection");
    if (disc->comp_slot)
        LSH_FAIL(LSH_EINVAL, "comp_slot is not available for the dense projection "
                             "(permute the rows of Rt instead)");
    if (!Rt)
        LSH_FAIL(LSH_EINVAL, "Rt is NULL");
    if (ldr < pts->d)
        LSH_FAIL(LSH_EINVAL, "ldr %lld < d %d", (long long)ldr, pts->d);
    if (!out)
        LSH_FAIL(LSH_EINVAL, "output descriptor is NULL");
    int64_t key_ld = out->key_ld ? out->key_ld : pts->n;
    if (out->keys && key_ld < pts->n)
        LSH_FAIL(LSH_EINVAL, "key_ld < n");
    if (pts->n == 0)
        return LSH_OK;
    DenseBf16Args g = {};
    DenseArgs &a = g.e;
    g.x = (const uint16_t *)pts->x;
    g.scale = pts->row_scale;
    g.rt = Rt;
    g.ldr = ldr;
    a.ld = pts->ld;
    a.n = pts->n;
    a.d = pts->d;
    a.m = disc->m;
    a.K = disc->K;
    a.L = disc->L;
    a.family = disc->family;
    a.xvec = ((uintptr_t)pts->x % 16 == 0) && (pts->ld % 8 == 0);
    a.rvec = ((uintptr_t)Rt % 16 == 0) && (ldr % 8 == 0);
    a.tabs_per_tile = kBN / disc->K;
    a.tile_w = a.tabs_per_tile * disc->K;
    a.ncol = (disc->L + a.tabs_per_tile - 1) / a.tabs_per_tile;
    a.nrow_tiles = (pts->n + kBM - 1) / kBM;
    a.ntiles = a.nrow_tiles * a.ncol;
    a.w32 = disc->family == LSH_E2LSH ? disc->w : 1.0f;
    a.inv_w32 = 1.0f / a.w32;
    int ex;
    a.w_pow2 = frexpf(a.w32, &ex) == 0.5f;
    a.b = disc->b;
    a.keys = out->keys;
    a.key_ld = key_ld;
    a.codes = out->codes;
    a.proj = out->proj;
    a.counters = (unsigned long long *)out->counters;
    int64_t grid = (a.ntiles + 7) / 8 * 8;
    if (grid > 0x7fffffff)
        LSH_FAIL(LSH_EINVAL, "too many tiles");
    hipLaunchKernelGGL(dense_bf16_kernel, dim3((unsigned)grid), dim3(kDThreads), 0,
                       (hipStream_t)stream, g);
    LSH_LAUNCHED("dense_bf16_kernel");
    return LSH_OK;
}
