// Error reporting and device queries shared by the liblsh entry points.
#include <stdarg.h>
#include <stdio.h>

#include "lsh_internal.h"

namespace lsh {

static thread_local char g_err[512];

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char *hip_msg(hipError_t e) { return hipGetErrorString(e); }

int device_cu_count()
{
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (cache[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0)
            cu = 256;
        cache[dev] = cu;
    }
    return cache[dev];
}

lsh_status check_stream_device(void *stream)
{
    if (!stream)
        return LSH_OK;
    int cur = 0, sd = 0;
    LSH_HIP(hipGetDevice(&cur));
    LSH_HIP(hipStreamGetDevice((hipStream_t)stream, &sd));
    if (sd != cur)
        LSH_FAIL(LSH_EINVAL, "the stream belongs to device %d but device %d is current", sd, cur);
    return LSH_OK;
}

} // namespace lsh

extern "C" const char *lsh_last_error(void) { return lsh::g_err; }

extern "C" int32_t lsh_version(void) { return 200; }
