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
constexpr int kYStride = kBN + 4;

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
};

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
    __syncthreads();

    // epilogue: one (row, table) pair per thread and step
    unsigned nsat = 0;
    const int npairs = kBM * a.tabs_per_tile;
    for (int p = tid; p < npairs; p += kDThreads) {
        const int tl = p / kBM, r = p % kBM;
        const int64_t row = row0 + r;
        const int t = ct * a.tabs_per_tile + tl;
        if (row >= a.n || t >= a.L)
            continue;
        const int c0 = tl * a.K;          // column in tile
        const int l0 = t * a.K;           // component
        uint64_t key;
        if (a.family == LSH_E2LSH) {
            key = e2lsh_key(a.K, mix64(2ull * t), mix64(2ull * t + 1), [&](int q, bool first) {
                float y = sm.y[r][c0 + q];
                float v = y + a.b[l0 + q];
                float c = a.w_pow2 ? floorf(v * a.inv_w32) : floorf(v / a.w32);
                unsigned s = 0;
                int32_t ci = floor_to_i32((double)c, s);
                if (first) {
                    nsat += s;
                    if (a.codes)
                        a.codes[row * a.m + l0 + q] = ci;
                    if (a.proj)
                        a.proj[row * a.m + l0 + q] = y;
                }
                return ci;
            });
        } else {
            key = 0;
            for (int q = 0; q < a.K; ++q) {
                float y = sm.y[r][c0 + q];
                bool bit = y > 0.0f;
                key |= (uint64_t)bit << q;
                if (a.codes)
                    a.codes[row * a.m + l0 + q] = bit ? 1 : 0;
                if (a.proj)
                    a.proj[row * a.m + l0 + q] = y;
            }
        }
        if (a.keys)
            a.keys[(int64_t)t * a.key_ld + row] = key;
    }
    if (a.counters && nsat)
        atomicAdd(&a.counters[2], (unsigned long long)nsat);
}

lsh_status check_disc(const lsh_disc *c);

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
