// Low-precision storage of points: FP32 rows -> BF16 or FP8-E4M3FN codes with
// one FP32 scale per row, the form the hashing and query calls read with
// lsh_dtype LSH_BF16 / LSH_FP8_E4M3FN.  The paper fixes no storage precision
// (its experiments are CPU-only); this is the storage of the precision path.
//
// One wave per row: a first pass takes max |x| with a wave reduction, the
// second pass (the row is then in cache) divides by the scale and rounds.
#include "lsh_internal.h"

namespace lsh {
namespace {

constexpr int kQuantWaves = 4;

__device__ __forceinline__ float wave_max_f32(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Round a binary32 value to bfloat16, nearest, ties to even (finite input).
__device__ __forceinline__ uint16_t to_bf16_rne(float v)
{
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Round v, |v| <= 448, to OCP FP8 E4M3FN (bias 7, 3 mantissa bits,
// subnormals k * 2^-9), nearest, ties to even.
__device__ __forceinline__ uint8_t to_e4m3fn_rne(float v)
{
    const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
    const float a = fabsf(v);
    uint32_t code;
    if (a < 0.015625f) {
        // below 2^-6 the grid is 2^-9; a result of 8 is 2^-6, whose code is 8
        code = (uint32_t)rintf(a * 512.0f);
    } else {
        int e;
        frexpf(a, &e);                       // a in [2^(e-1), 2^e)
        float t = rintf(ldexpf(a, 4 - e));   // a in units of its mantissa step: [8, 16]
        int be = e - 1 + 7;                  // biased exponent
        if (t == 16.0f) {
            t = 8.0f;
            ++be;
        }
        code = ((uint32_t)be << 3) | ((uint32_t)t - 8u);
    }
    return (uint8_t)(sign | code);
}

template <int DT>
__global__ __launch_bounds__(kQuantWaves *kWave) void quantize_kernel(
    const float *__restrict__ x, int64_t n, int32_t d, int64_t ldx, void *__restrict__ q,
    int64_t ldq, float *__restrict__ row_scale)
{
    const int64_t row = (int64_t)blockIdx.x * kQuantWaves + (threadIdx.x / kWave);
    if (row >= n)
        return;
    const int lane = threadIdx.x % kWave;
    const float *xr = x + row * ldx;
    float amax = 0.0f;
    for (int j = lane; j < d; j += kWave)
        amax = fmaxf(amax, fabsf(xr[j]));
    amax = wave_max_f32(amax);
    float scale;
    if (DT == LSH_BF16)
        scale = amax > 0.0f ? amax : 1.0f;
    else
        scale = amax > 0.0f ? __fdiv_rn(amax, 448.0f) : 1.0f;
    if (lane == 0)
        row_scale[row] = scale;
    if (DT == LSH_BF16) {
        uint16_t *qr = (uint16_t *)q + row * ldq;
        for (int j = lane; j < d; j += kWave)
            qr[j] = to_bf16_rne(__fdiv_rn(xr[j], scale));
    } else {
        uint8_t *qr = (uint8_t *)q + row * ldq;
        for (int j = lane; j < d; j += kWave) {
            float v = __fdiv_rn(xr[j], scale);
            v = fminf(fmaxf(v, -448.0f), 448.0f);
            qr[j] = to_e4m3fn_rne(v);
        }
    }
}

} // namespace
} // namespace lsh

extern "C" lsh_status lsh_quantize_rows(const float *x, int64_t n, int32_t d, int64_t ldx,
                                        int32_t dtype, void *q, int64_t ldq, float *row_scale,
                                        void *stream)
{
    using namespace lsh;
    if (n < 0 || d < 1 || ldx < d || ldq < d)
        LSH_FAIL(LSH_EINVAL, "bad shape n=%lld d=%d ldx=%lld ldq=%lld", (long long)n, d,
                 (long long)ldx, (long long)ldq);
    if (dtype != LSH_BF16 && dtype != LSH_FP8_E4M3FN)
        LSH_FAIL(LSH_EINVAL, "dtype %d: quantise to LSH_BF16 or LSH_FP8_E4M3FN", dtype);
    if (n == 0)
        return LSH_OK;
    if (!x || !q || !row_scale)
        LSH_FAIL(LSH_EINVAL, "x, q and row_scale are required");
    const int64_t blocks = (n + kQuantWaves - 1) / kQuantWaves;
    if (blocks > 0x7fffffff)
        LSH_FAIL(LSH_EINVAL, "n = %lld rows is too many for one call", (long long)n);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LSH_BF16)
        hipLaunchKernelGGL(quantize_kernel<LSH_BF16>, dim3((unsigned)blocks),
                           dim3(kQuantWaves * kWave), 0, s, x, n, d, ldx, q, ldq, row_scale);
    else
        hipLaunchKernelGGL(quantize_kernel<LSH_FP8_E4M3FN>, dim3((unsigned)blocks),
                           dim3(kQuantWaves * kWave), 0, s, x, n, d, ldx, q, ldq, row_scale);
    LSH_LAUNCHED("quantize_kernel");
    return LSH_OK;
}
