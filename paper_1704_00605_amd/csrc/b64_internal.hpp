// Library-internal entry points shared by the codec and the runtime sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "b64.h"
#include "b64_modes.hpp"

// Batched codec launches with a caller-built plan: unit_off (N + 1 entries,
// exclusive scan of ceil(len / 12) for encode, ceil(len / 16) for decode),
// and for decode out_len[i] = 0, err_off[i] = -1 before the call; the codec
// kernel leaves the verdicts (length, -1) or (-1, first offending index) in
// them. Message i is src[in_begin[i], in_begin[i] + in_len[i]). Enqueue only.
int b64i_encode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, const b64_tune *tune, hipStream_t s);
int b64i_decode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                        const b64_tune *tune, hipStream_t s);

// Records a failure message for b64_last_error() on this thread; returns code.
int b64i_fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Compute units of the current device (cached per device).
int b64i_device_cus(int *out);

// Alphabet/mode argument of the C-ABI -> B64I_M_* bits (B64_BAD_ARG if invalid).
int b64i_parse_mode(int alphabet, int *mode);

// Encoded length of n bytes under mode bits (with or without padding).
int64_t b64i_enc_len(int64_t n, int mode);

// Single-buffer launches (enqueue only). Decode needs n >= 1 and
// (*len_slot, *err_slot) == (0, -1) before the kernel, which leaves the
// verdict (length, -1) or (-1, first offending index) in them.
int b64i_enqueue_encode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, hipStream_t s);
int b64i_enqueue_decode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, unsigned long long *err_slot,
                        int64_t *len_slot, hipStream_t s);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return b64i_fail(B64_HIP_ERROR, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// Checks that a kernel launch was accepted.
#define LAUNCH_TRY()                                                                         \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return b64i_fail(B64_HIP_ERROR, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)
