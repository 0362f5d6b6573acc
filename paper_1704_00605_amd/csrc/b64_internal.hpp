// Library-internal entry points shared by the codec and the runtime sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "b64.h"

// Error slot value meaning "no error yet" (see b64_device.hpp).
constexpr int64_t B64I_ERR_NONE = 0x7fffffffffffffffll;

// Batched codec launches with a caller-built plan: unit_off (N + 1 entries,
// exclusive scan of ceil(len / 12) for encode, ceil(len / 16) for decode),
// and for decode out_len[i] = 0, err_off[i] = B64I_ERR_NONE before the call.
// Message i is src[in_begin[i], in_begin[i] + in_len[i]). Enqueue only.
int b64i_encode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, const b64_tune *tune, hipStream_t s);
int b64i_decode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                        const b64_tune *tune, hipStream_t s);

// Records a failure message for b64_last_error() on this thread.
int b64i_fail(int code, const char *msg);
