// Host-side pieces of the codec library shared by its sources: the
// per-thread error message, device properties, argument parsing and the
// length functions of the C-ABI (include/b64.h).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>
#include <vector>

#include "b64.h"
#include "b64_internal.hpp"

namespace {

thread_local std::string t_err = "no error";

struct DevCache {
    int cus = 0;
};

std::mutex g_mu;
std::vector<DevCache> g_dev;

}  // namespace

int b64i_device_cus(int *out)
{
    int dev;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return b64i_fail(B64_HIP_ERROR, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    if (!g_dev[dev].cus) {
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return b64i_fail(B64_HIP_ERROR, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
        g_dev[dev].cus = c;
    }
    *out = g_dev[dev].cus;
    return B64_OK;
}

int b64i_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int b64i_parse_mode(int alphabet, int *mode)
{
    const int a = alphabet & 0xff;
    if (a != B64_ALPHABET_STD && a != B64_ALPHABET_URL) return b64i_fail(B64_BAD_ARG, "bad alphabet %d", a);
    if (alphabet & ~(0xff | B64_MODE_STRICT | B64_MODE_NOPAD))
        return b64i_fail(B64_BAD_ARG, "unknown mode bits 0x%x", alphabet);
    if ((alphabet & B64_MODE_STRICT) && (alphabet & B64_MODE_NOPAD))
        return b64i_fail(B64_BAD_ARG, "strict and unpadded modes cannot be combined");
    *mode = (a ? B64I_M_URL : 0) | ((alphabet & B64_MODE_STRICT) ? B64I_M_STRICT : 0) |
            ((alphabet & B64_MODE_NOPAD) ? B64I_M_NOPAD : 0);
    return B64_OK;
}

int64_t b64i_enc_len(int64_t n, int mode)
{
    if (mode & B64I_M_NOPAD) return 4 * (n / 3) + ((n % 3) ? (n % 3) + 1 : 0);
    return 4 * ((n + 2) / 3);
}

extern "C" {

const char *b64_last_error(void) { return t_err.c_str(); }

int b64_device_cus(void)
{
    int c;
    int rc = b64i_device_cus(&c);
    return rc ? rc : c;
}

int64_t b64_encoded_len(int64_t n)
{
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    return 4 * ((n + 2) / 3);
}

int64_t b64_encoded_len_mode(int64_t n, int mode)
{
    int m;
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    int rc = b64i_parse_mode(mode, &m);
    if (rc) return rc;
    return b64i_enc_len(n, m);
}

int64_t b64_decoded_max(int64_t m)
{
    if (m < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    return 3 * (m / 4);
}

int64_t b64_decoded_max_mode(int64_t m, int mode)
{
    int md;
    if (m < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    int rc = b64i_parse_mode(mode, &md);
    if (rc) return rc;
    return 3 * (m / 4) + (((md & B64I_M_NOPAD) && (m & 3) >= 2) ? (m & 3) - 1 : 0);
}

}  // extern "C"
