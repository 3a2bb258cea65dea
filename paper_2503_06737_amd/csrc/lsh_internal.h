// Internal definitions shared by the HIP sources of liblsh (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lsh.h"

namespace lsh {

constexpr int kWave = 64;

// ----------------------------------------------------------------- host side
void set_error(const char *fmt, ...);
const char *hip_msg(hipError_t e);

#define LSH_FAIL(code, ...)                                                                        \
    do {                                                                                           \
        ::lsh::set_error(__VA_ARGS__);                                                             \
        return (code);                                                                             \
    } while (0)

#define LSH_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            LSH_FAIL(LSH_EHIP, "%s failed: %s", #expr, ::lsh::hip_msg(e_));                       \
    } while (0)

// Check the launch that was just enqueued.
#define LSH_LAUNCHED(name)                                                                         \
    do {                                                                                           \
        hipError_t e_ = hipGetLastError();                                                         \
        if (e_ != hipSuccess)                                                                      \
            LSH_FAIL(LSH_EHIP, "launch of %s failed: %s", name, ::lsh::hip_msg(e_));               \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Number of compute units of the current device (cached per device).
int device_cu_count();
// LSH_OK when `stream` (NULL: the default stream) belongs to the current
// device, else LSH_EINVAL: per-device state (the static scratch array, the
// side stream of the index build) is that of the current device.
lsh_status check_stream_device(void *stream);

// Argument checks shared by the entry points (set the error message).
lsh_status check_points(const lsh_points *p);
lsh_status check_disc(const lsh_disc *c);

// -------------------------------------------------------------- device side

// SplitMix64 finaliser (Steele, Lea and Flood 2014), a bijection on 64-bit words.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Bucket key of one table from its K E2LSH codes (the digest specified in
// lsh.h): code_of(r, first_pass) returns code r; seed_narrow / seed_wide are
// F(2t) and F(2t + 1).  Narrow tuples (all codes in [-128, 127]) are packed a
// byte per code, 8 codes per word; otherwise 32 bits per code, 2 per word.
template <typename CodeOf>
__device__ __forceinline__ uint64_t e2lsh_key(int K, uint64_t seed_narrow, uint64_t seed_wide,
                                              CodeOf code_of)
{
    uint64_t h = seed_narrow, W = 0;
    bool narrow = true;
    for (int r = 0; r < K; ++r) {
        int32_t c = code_of(r, true);
        narrow &= (c >= -128) & (c <= 127);
        W |= (uint64_t)(uint8_t)c << (8 * (r & 7));
        if ((r & 7) == 7 || r == K - 1) {
            h = mix64(h ^ W);
            W = 0;
        }
    }
    if (narrow)
        return h;
    h = seed_wide;
    for (int r = 0; r < K; ++r) {
        int32_t c = code_of(r, false);
        W |= (uint64_t)(uint32_t)c << (32 * (r & 1));
        if ((r & 1) == 1 || r == K - 1) {
            h = mix64(h ^ W);
            W = 0;
        }
    }
    return h;
}

// floor() of an FP64 value, saturated to int32; *sat += 1 when it saturates.
__device__ __forceinline__ int32_t floor_to_i32(double c, unsigned &sat)
{
    if (c >= 2147483648.0) {
        ++sat;
        return 2147483647;
    }
    if (c < -2147483648.0) {
        ++sat;
        return -2147483647 - 1;
    }
    return (int32_t)c;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

} // namespace lsh
