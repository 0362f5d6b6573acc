// gfx950 kernels and the C-ABI of the base64 codec (see include/b64.h).
//
// Kernels:
//   k_enc_single / k_dec_single   one buffer, grid-stride over 12-byte /
//                                 16-character units, one unit per lane.
//   k_plan_reduce / k_plan_scan   device planning for batches: per-message
//                                 unit counts -> exclusive scan (unit_off),
//                                 output-length and error-slot init.
//   k_enc_batch / k_dec_batch     persistent batched codec: every wave owns a
//                                 contiguous range of 64-unit groups of the
//                                 flattened unit space of all messages.
//   k_dec_batch_final             per-message verdicts.
//   k_out_offsets                 exclusive scan of output sizes.
//
// Decode errors: a lane whose unit holds a non-symbol computes the exact
// index; a wave ballot elects the first erring lane, which performs one
// atomicMin on the 64-bit error slot (Section 2: the decoder must report
// characters outside the alphabet; the smallest index is the one reported).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "b64.h"
#include "b64_device.hpp"

using namespace b64dev;

__constant__ Tables c_tab = make_tables();

// ----------------------------------------------------------- error state --
static thread_local std::string t_err = "no error";

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(B64_HIP_ERROR, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

// Checks that a kernel launch was accepted.
#define LAUNCH_TRY()                                                                         \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return fail(B64_HIP_ERROR, "kernel launch failed: %s", hipGetErrorString(e_));   \
    } while (0)

// ------------------------------------------------------------ LDS tables --
// Copies `bytes` (multiple of 4) of the constant tables into LDS.
__device__ __forceinline__ void lds_fill(uint32_t *dst, const uint8_t *src, int bytes)
{
    const uint32_t *s = (const uint32_t *)src;
    for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) dst[i] = s[i];
}

struct __attribute__((aligned(4))) u32x3 { uint32_t x, y, z; };
struct __attribute__((aligned(4))) u32x4 { uint32_t x, y, z, w; };

// ======================================================= single buffer ==

// One grid-stride step of the single-buffer encode: this lane's units are
// first + k * stride for k < UPL. Without GUARD every unit is known to be in
// range, so all UPL loads are issued before any is consumed.
template <bool ALIGNED, int UPL, bool GUARD>
__device__ __forceinline__ void enc_step(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                         int64_t first, int stride, int64_t units, const uint8_t *tab)
{
    uint32_t w[UPL][3];
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        if (!GUARD || u < units) {
            if (ALIGNED) {
                const u32x3 v = *(const u32x3 *)(src + 12 * u);
                w[k][0] = v.x; w[k][1] = v.y; w[k][2] = v.z;
            } else {
                load12(src + 12 * u, w[k][0], w[k][1], w[k][2]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        if (!GUARD || u < units) {
            uint32_t o[4];
            enc_unit(w[k][0], w[k][1], w[k][2], tab, o[0], o[1], o[2], o[3]);
            if (ALIGNED) {
                uint32_t *d = (uint32_t *)(dst + 16 * u);
                __builtin_nontemporal_store(o[0], d + 0);
                __builtin_nontemporal_store(o[1], d + 1);
                __builtin_nontemporal_store(o[2], d + 2);
                __builtin_nontemporal_store(o[3], d + 3);
            } else {
                store_words<4>(dst + 16 * u, o);
            }
        }
    }
}

// Encode src[0, n): full units [0, n / 12) in a grid-stride loop over tiles
// of blockDim * UPL units, then the final partial unit (Algorithm 1's tail)
// by one lane.
template <bool ALIGNED, int UPL>
__global__ __launch_bounds__(1024) void k_enc_single(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, int mode)
{
    __shared__ uint32_t s_tab[16];
    lds_fill(s_tab, c_tab.enc[mode & M_URL], 64);
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;

    const int64_t units = n / 12;
    const int64_t tile = (int64_t)blockDim.x * UPL;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < units; t0 += (int64_t)gridDim.x * tile) {
        if (t0 + tile <= units)
            enc_step<ALIGNED, UPL, false>(src, dst, t0 + threadIdx.x, blockDim.x, units, tab);
        else
            enc_step<ALIGNED, UPL, true>(src, dst, t0 + threadIdx.x, blockDim.x, units, tab);
    }
    const int r = (int)(n - 12 * units);
    if (r && blockIdx.x == 0 && threadIdx.x == 0)
        enc_tail(src + 12 * units, r, dst + 16 * units, tab, mode & M_NOPAD);
}

// One grid-stride step of the single-buffer decode (see enc_step). Lanes of a
// wave hold consecutive units, so the lowest erring lane of a ballot has the
// wave's smallest offset; it alone performs the atomicMin.
template <bool ALIGNED, int UPL, bool GUARD>
__device__ __forceinline__ void dec_step(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                         int64_t first, int stride, int64_t L, const uint8_t *tab,
                                         unsigned long long *err_slot)
{
    uint32_t w[UPL][4];
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        if (!GUARD || u < L) {
            if (ALIGNED) {
                const u32x4 v = *(const u32x4 *)(src + 16 * u);
                w[k][0] = v.x; w[k][1] = v.y; w[k][2] = v.z; w[k][3] = v.w;
            } else {
                load16(src + 16 * u, w[k][0], w[k][1], w[k][2], w[k][3]);
            }
        }
    }
    uint32_t bad_any = 0;
    uint32_t bad[UPL];
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        bad[k] = 0;
        if (!GUARD || u < L) {
            uint32_t o[3];
            bad[k] = dec_unit(w[k][0], w[k][1], w[k][2], w[k][3], tab, o[0], o[1], o[2]);
            bad_any |= bad[k];
            if (ALIGNED) {
                uint32_t *d = (uint32_t *)(dst + 12 * u);
                __builtin_nontemporal_store(o[0], d + 0);
                __builtin_nontemporal_store(o[1], d + 1);
                __builtin_nontemporal_store(o[2], d + 2);
            } else {
                store_words<3>(dst + 12 * u, o);
            }
        }
    }
    // rare path: some unit of this step holds a non-symbol
    if (__ballot(bad_any & INVALID)) {
#pragma unroll
        for (int k = 0; k < UPL; k++) {
            const int64_t u = first + (int64_t)k * stride;
            const bool err = (bad[k] & INVALID) != 0;
            const unsigned long long ball = __ballot(err);
            if (ball && __lane_id() == __ffsll((long long)ball) - 1) {
                const int64_t pos = 16 * u + dec_first_bad(w[k][0], w[k][1], w[k][2], w[k][3], tab);
                atomicMin(err_slot, (unsigned long long)pos);
            }
        }
    }
}

// Decode src[0, n), n >= 1. Interior units [0, L) with L = (n - 1) / 16 hold
// 16 characters that are all before the final one; unit L (1..16 characters)
// carries the padding and length rules. err_slot must hold ERR_NONE at
// launch; it ends holding the smallest offending index (or ERR_NONE). The
// lane of the final unit writes the decoded length to *len_slot when that
// unit is valid. k_dec_final turns the pair into the verdict.
template <bool ALIGNED, int UPL>
__global__ __launch_bounds__(1024) void k_dec_single(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, int mode,
                                                     unsigned long long *err_slot, int64_t *len_slot)
{
    __shared__ uint32_t s_tab[64];
    lds_fill(s_tab, c_tab.dec[mode & M_URL], 256);
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;

    const int64_t L = (n - 1) / 16;
    const int64_t tile = (int64_t)blockDim.x * UPL;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < L; t0 += (int64_t)gridDim.x * tile) {
        if (t0 + tile <= L)
            dec_step<ALIGNED, UPL, false>(src, dst, t0 + threadIdx.x, blockDim.x, L, tab, err_slot);
        else
            dec_step<ALIGNED, UPL, true>(src, dst, t0 + threadIdx.x, blockDim.x, L, tab, err_slot);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        int nout;
        const int r = (int)(n - 16 * L);
        const int idx = dec_tail(src + 16 * L, r, n, dst + 12 * L, tab, mode, &nout);
        if (idx >= 0) atomicMin(err_slot, (unsigned long long)(16 * L + idx));
        else *len_slot = 12 * L + nout;
    }
}

// Verdict of a single-buffer decode, run after k_dec_single on the same
// stream: (length, -1) or (-1, first offending index). With reset, the error
// slot is restored to ERR_NONE for the next call.
__global__ void k_dec_final(unsigned long long *err_slot, const int64_t *len_slot, int64_t *out_len,
                            int64_t *out_err, int reset)
{
    if (threadIdx.x == 0) {
        const unsigned long long e = *err_slot;
        const int64_t len = *len_slot;
        if (e == ERR_NONE) { *out_len = len; *out_err = -1; }
        else { *out_len = -1; *out_err = (int64_t)e; }
        if (reset) *err_slot = ERR_NONE;
    }
}

// Prepares an asynchronous decode's device slots: the error slot (which is
// d_err itself) to ERR_NONE, or the final verdict of an empty input.
__global__ void k_slots_init(int64_t *d_len, int64_t *d_err, int empty)
{
    if (threadIdx.x == 0) {
        *d_len = 0;
        *d_err = empty ? -1 : (int64_t)ERR_NONE;
    }
}

// ============================================================== batches ==
constexpr int PLAN_BLOCK = 256;
constexpr int PLAN_PER_THREAD = 8;
constexpr int PLAN_CHUNK = PLAN_BLOCK * PLAN_PER_THREAD;

__device__ __forceinline__ int64_t units_of(int dir, int64_t len)
{
    return dir == B64_DIR_ENCODE ? (len + 11) / 12 : (len + 15) / 16;
}

__device__ __forceinline__ int64_t enc_len_of(int64_t len, int nopad)
{
    return nopad ? 4 * (len / 3) + ((len % 3) ? (len % 3) + 1 : 0) : 4 * ((len + 2) / 3);
}

__device__ __forceinline__ int64_t dec_cap_of(int64_t len, int nopad)
{
    return 3 * (len / 4) + ((nopad && (len & 3) >= 2) ? (len & 3) - 1 : 0);
}

// Decode output slot of the batch layout: the capacity rounded up to a
// multiple of 4 so every slot starts where dst's alignment allows dword
// stores (each 16-character unit writes 12 bytes at offset 12j of its slot).
__device__ __forceinline__ int64_t dec_slot_of(int64_t len, int nopad)
{
    return (dec_cap_of(len, nopad) + 3) & ~(int64_t)3;
}

// Where the messages of a batch are. Packed form: message i is
// [begin[i], begin[i+1]) (len == nullptr, begin has N + 1 entries). Gather
// form: message i is [begin[i], begin[i] + len[i]).
struct Msgs {
    const int64_t *begin;
    const int64_t *len;
    __device__ __forceinline__ int64_t b(int64_t i) const { return begin[i]; }
    __device__ __forceinline__ int64_t n(int64_t i) const { return len ? len[i] : begin[i + 1] - begin[i]; }
};

// Block-wide exclusive scan of one int64 per thread (blockDim.x <= 1024).
__device__ int64_t block_exclusive_scan(int64_t v)
{
    __shared__ int64_t s_w[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    int64_t pre = 0;
    for (int i = 0; i < wid; i++) pre += s_w[i];
    (void)nw;
    __syncthreads();
    return pre + x - v;
}

__device__ int64_t block_sum(int64_t v)
{
    __shared__ int64_t s_w[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    int64_t t = 0;
    for (int i = 0; i < nw; i++) t += s_w[i];
    __syncthreads();
    return t;
}

// Per-chunk totals of work units.
template <int DIR>
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_reduce(Msgs msgs, int64_t N,
                                                            int64_t *__restrict__ partial)
{
    const int64_t i0 = (int64_t)blockIdx.x * PLAN_CHUNK + threadIdx.x * PLAN_PER_THREAD;
    int64_t s = 0;
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        const int64_t i = i0 + k;
        if (i < N) s += units_of(DIR, msgs.n(i));
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// unit_off = exclusive scan of units per message (N + 1 entries), plus
// per-message initialisation: encode out_len (known from the length);
// decode out_len = 0 and err_off = ERR_NONE (the atomicMin sentinel).
template <int DIR>
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_scan(
    Msgs msgs, int64_t N, const uint8_t *__restrict__ flags,
    const int64_t *__restrict__ partial, int64_t *__restrict__ unit_off,
    int64_t *__restrict__ out_len, int64_t *__restrict__ err_off)
{
    int64_t pre = 0;
    for (int64_t c = threadIdx.x; c < blockIdx.x; c += blockDim.x) pre += partial[c];
    pre = block_sum(pre);
    const int64_t i0 = (int64_t)blockIdx.x * PLAN_CHUNK + threadIdx.x * PLAN_PER_THREAD;
    int64_t u[PLAN_PER_THREAD];
    int64_t s = 0;
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        const int64_t i = i0 + k;
        u[k] = 0;
        if (i < N) {
            const int64_t len = msgs.n(i);
            const int fl = flags ? flags[i] : 0;
            u[k] = units_of(DIR, len);
            if (DIR == B64_DIR_ENCODE) {
                out_len[i] = enc_len_of(len, fl & M_NOPAD);
            } else {
                out_len[i] = 0;
                err_off[i] = (int64_t)ERR_NONE;
            }
        }
        s += u[k];
    }
    int64_t ex = pre + block_exclusive_scan(s);
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        const int64_t i = i0 + k;
        if (i < N) unit_off[i] = ex;
        if (i == N - 1) unit_off[N] = ex + u[k];
        ex += u[k];
    }
    if (N == 0 && blockIdx.x == 0 && threadIdx.x == 0) unit_off[0] = 0;
}

__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Largest m in [lo, N) with unit_off[m] <= t, given unit_off[lo] <= t <
// unit_off[N], found by the whole wave with 64-way probes. Wave-uniform.
__device__ int64_t wave_find_msg(const int64_t *__restrict__ unit_off, int64_t N, int64_t t,
                                 int64_t lo = 0)
{
    int64_t hi = N;  // unit_off[lo] <= t < unit_off[hi]
    const int lane = __lane_id();
    while (hi - lo > 1) {
        const int64_t span = hi - lo;
        const int64_t stepw = (span + 63) / 64;
        const int64_t p = lo + (int64_t)(lane + 1) * stepw;
        const bool ok = p < hi && unit_off[p] <= t;
        const unsigned long long b = __ballot(ok);
        const int c = __popcll(b);  // probes are increasing: ok holds for a prefix of lanes
        const int64_t nlo = lo + (int64_t)c * stepw;
        hi = min(hi, lo + (int64_t)(c + 1) * stepw);
        lo = nlo;
    }
    return uniform64(lo);
}

// Message of unit u when the group starting at message m spans several
// messages: counts the message ends <= u among the next 64 boundaries
// (shuffle-based binary search), advancing 64 messages at a time.
__device__ int64_t lane_find_msg(const int64_t *__restrict__ unit_off, int64_t N, int64_t m,
                                 int64_t u, bool active)
{
    const int lane = __lane_id();
    int64_t res = m;
    bool done = !active;
    int64_t base = m;
    while (true) {
        const unsigned long long pending = __ballot(!done);
        if (!pending) break;
        const int64_t idx = base + 1 + lane;
        const int64_t B = idx <= N ? unit_off[idx] : INT64_MAX;
        int c = 0;
#pragma unroll
        for (int stp = 32; stp >= 1; stp >>= 1) {
            const int64_t b = __shfl(B, c + stp - 1, 64);
            if (b <= u) c += stp;
        }
        const int64_t b63 = __shfl(B, 63, 64);
        if (c == 63 && b63 <= u) c = 64;
        if (!done && c < 64) { res = base + c; done = true; }
        base += 64;  // lanes still pending look at the next 64 boundaries
    }
    return res;
}

// What one lane works on in a batched step: unit j of message mm.
struct LaneRef {
    bool valid;
    int64_t mm, j, b, n, o;
    int fl;
};

struct BatchArgs {
    Msgs msgs;
    int64_t N, U;
    const int64_t *__restrict__ unit_off;
    const int64_t *__restrict__ out_off;
    const uint8_t *__restrict__ flags;
};

// Per-lane view of unit u, given the message m0 of a unit <= u: the
// message by a wave-wide search over the next boundaries, then its metadata.
__device__ __forceinline__ LaneRef lane_ref(const BatchArgs &a, int64_t m0, int64_t u)
{
    LaneRef r;
    r.valid = u < a.U;
    const int64_t mm = lane_find_msg(a.unit_off, a.N, m0, u, r.valid);
    r.mm = mm;
    r.j = u - a.unit_off[mm];
    r.b = a.msgs.b(mm);
    r.n = a.msgs.n(mm);
    r.o = a.out_off[mm];
    r.fl = a.flags ? a.flags[mm] : 0;
    return r;
}

// One unit of the batched encode: full 12-byte units, or the message's
// final partial unit (Algorithm 1's tail).
__device__ __forceinline__ void enc_batch_unit(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                               const LaneRef &r, bool full, const uint32_t (&w)[3],
                                               const uint8_t *tabs)
{
    const uint8_t *tab = tabs + 64 * (r.fl & M_URL);
    uint8_t *q = dst + r.o + 16 * r.j;
    if (full) {
        uint32_t o[4];
        enc_unit(w[0], w[1], w[2], tab, o[0], o[1], o[2], o[3]);
        store_words<4, true>(q, o);
    } else {
        enc_tail(src + r.b + 12 * r.j, (int)(r.n - 12 * r.j), q, tab, r.fl & M_NOPAD);
    }
}

// One unit of the batched decode: interior units (16 characters, none of
// them the message's last) or the final unit with the padding and length
// rules. Errors lower the message's err_off; the final unit's lane writes
// the decoded length when that unit is valid.
__device__ __forceinline__ void dec_batch_unit(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                               const LaneRef &r, bool interior, const uint32_t (&w)[4],
                                               const uint8_t *tabs, int64_t *__restrict__ out_len,
                                               int64_t *__restrict__ err_off)
{
    const uint8_t *tab = tabs + 256 * (r.fl & M_URL);
    uint8_t *q = dst + r.o + 12 * r.j;
    if (interior) {
        uint32_t o[3];
        const uint32_t bad = dec_unit(w[0], w[1], w[2], w[3], tab, o[0], o[1], o[2]);
        store_words<3, true>(q, o);
        if (bad & INVALID) {
            const int64_t pos = 16 * r.j + dec_first_bad(w[0], w[1], w[2], w[3], tab);
            atomicMin((unsigned long long *)&err_off[r.mm], (unsigned long long)pos);
        }
    } else {
        int nout;
        const int idx = dec_tail(src + r.b + 16 * r.j, (int)(r.n - 16 * r.j), r.n, q, tab, r.fl, &nout);
        if (idx >= 0)
            atomicMin((unsigned long long *)&err_off[r.mm], (unsigned long long)(16 * r.j + idx));
        else
            out_len[r.mm] = 12 * r.j + nout;
    }
}

// ---------------------------------------------------------------- layout 1
// One contiguous share of the 64-unit groups per wave, walked with a
// wave-uniform cursor: the message holding the wave's current group and its
// metadata, kept in scalar registers, so that groups inside one message need
// no metadata loads ahead of their data loads. Suits batches of many small
// and mid-size messages.
struct Cursor {
    int64_t m, u0, u1;  // message, its unit range [u0, u1)
    int64_t b, n, o;    // input begin, input length, output begin
    int fl;             // flags
};

__device__ __forceinline__ void cursor_load(Cursor &c, const BatchArgs &a, int64_t m)
{
    c.m = m;
    c.u0 = a.unit_off[m];
    c.u1 = a.unit_off[m + 1];
    c.b = a.msgs.b(m);
    c.n = a.msgs.n(m);
    c.o = a.out_off[m];
    c.fl = a.flags ? a.flags[m] : 0;
}

// Units gs + lane of one 64-unit group (gs < U); advances the cursor.
__device__ __forceinline__ LaneRef resolve_group(Cursor &c, const BatchArgs &a, int64_t gs)
{
    if (c.u1 <= gs) {  // the group starts in a later message
        int64_t m = c.m + 1;
        while (a.unit_off[m + 1] <= gs) m++;  // skips messages without units
        cursor_load(c, a, m);
    }
    const int64_t u = gs + __lane_id();
    if (gs + 64 <= c.u1) {  // whole group inside the cursor's message
        LaneRef r;
        r.valid = true;
        r.mm = c.m; r.j = u - c.u0; r.b = c.b; r.n = c.n; r.o = c.o; r.fl = c.fl;
        return r;
    }
    const LaneRef r = lane_ref(a, c.m, u);
    // the next group starts in the message of this group's last valid unit or later
    const unsigned long long vb = __ballot(r.valid);
    const int top = 63 - __clzll(vb);
    const int64_t last = uniform64(__shfl(r.mm, top, 64));
    if (last != c.m) cursor_load(c, a, last);
    return r;
}

// Contiguous share [g0, g1) of the 64-unit groups for the calling wave.
__device__ __forceinline__ void wave_share(int64_t U, int64_t &g0, int64_t &g1)
{
    const int64_t G = (U + 63) / 64;
    const int64_t W = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    g0 = (G * w) / W;
    g1 = (G * (w + 1)) / W;
}

template <int UPL>
__global__ __launch_bounds__(1024) void k_enc_batch_w(
    const uint8_t *__restrict__ src, Msgs msgs, int64_t N,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off,
    const uint8_t *__restrict__ flags, const int64_t *__restrict__ unit_off)
{
    __shared__ uint32_t s_tab[32];
    lds_fill(s_tab, &c_tab.enc[0][0], 128);
    __syncthreads();
    const BatchArgs a{msgs, N, unit_off[N], unit_off, out_off, flags};
    int64_t g0, g1;
    wave_share(a.U, g0, g1);
    if (g0 >= g1) return;
    Cursor c;
    cursor_load(c, a, wave_find_msg(unit_off, N, g0 * 64));
    for (int64_t g = g0; g < g1; g += UPL) {
        LaneRef r[UPL];
        uint32_t w[UPL][3];
        bool full[UPL];
#pragma unroll
        for (int k = 0; k < UPL; k++) {
            r[k].valid = false;
            full[k] = false;
            if (g + k < g1) {
                r[k] = resolve_group(c, a, (g + k) * 64);
                full[k] = r[k].valid && 12 * r[k].j + 12 <= r[k].n;
                if (full[k]) load12(src + r[k].b + 12 * r[k].j, w[k][0], w[k][1], w[k][2]);
            }
        }
#pragma unroll
        for (int k = 0; k < UPL; k++)
            if (r[k].valid) enc_batch_unit(src, dst, r[k], full[k], w[k], (const uint8_t *)s_tab);
    }
}

template <int UPL>
__global__ __launch_bounds__(1024) void k_dec_batch_w(
    const uint8_t *__restrict__ src, Msgs msgs, int64_t N,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off,
    const uint8_t *__restrict__ flags, const int64_t *__restrict__ unit_off,
    int64_t *__restrict__ out_len, int64_t *__restrict__ err_off)
{
    __shared__ uint32_t s_tab[128];
    lds_fill(s_tab, &c_tab.dec[0][0], 512);
    __syncthreads();
    const BatchArgs a{msgs, N, unit_off[N], unit_off, out_off, flags};
    int64_t g0, g1;
    wave_share(a.U, g0, g1);
    if (g0 >= g1) return;
    Cursor c;
    cursor_load(c, a, wave_find_msg(unit_off, N, g0 * 64));
    for (int64_t g = g0; g < g1; g += UPL) {
        LaneRef r[UPL];
        uint32_t w[UPL][4];
        bool interior[UPL];
#pragma unroll
        for (int k = 0; k < UPL; k++) {
            r[k].valid = false;
            interior[k] = false;
            if (g + k < g1) {
                r[k] = resolve_group(c, a, (g + k) * 64);
                interior[k] = r[k].valid && 16 * r[k].j + 16 < r[k].n;
                if (interior[k]) load16(src + r[k].b + 16 * r[k].j, w[k][0], w[k][1], w[k][2], w[k][3]);
            }
        }
#pragma unroll
        for (int k = 0; k < UPL; k++)
            if (r[k].valid)
                dec_batch_unit(src, dst, r[k], interior[k], w[k], (const uint8_t *)s_tab, out_len, err_off);
    }
}

// ---------------------------------------------------------------- layout 0
// Layout 0 (tiles): tiles of blockDim * UPL units are dealt out grid-stride,
// so the blocks in flight stream through one dense window of memory as a
// one-shot grid does. A block-wide search (bounded below by the block's
// previous tile) finds each tile's first message. A tile made of full units
// of one message runs the single-buffer step; any other tile resolves the
// message of every unit per lane. This suits batches dominated by large
// messages.
// Largest m in [lo, N) with unit_off[m] <= t, given unit_off[lo] <= t <
// unit_off[N]: all threads of the block probe blockDim.x points per round.
__device__ int64_t block_find_msg(const int64_t *__restrict__ unit_off, int64_t N, int64_t t, int64_t lo)
{
    int64_t hi = N;
    while (hi - lo > 1) {
        const int64_t stepw = (hi - lo + blockDim.x - 1) / blockDim.x;
        const int64_t p = lo + (int64_t)(threadIdx.x + 1) * stepw;
        const int ok = p < hi && unit_off[p] <= t;
        const int64_t cnt = __syncthreads_count(ok);  // probes increase: ok holds for a prefix
        const int64_t nlo = lo + cnt * stepw;
        hi = min(hi, lo + (cnt + 1) * stepw);
        lo = nlo;
    }
    return lo;
}

template <int UPL, class Fast, class General>
__device__ __forceinline__ void batch_tiles(const BatchArgs &a, Fast fast, General general, bool decode)
{
    const int64_t tile = (int64_t)blockDim.x * UPL;
    int64_t m = 0;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < a.U; t0 += (int64_t)gridDim.x * tile) {
        m = block_find_msg(a.unit_off, a.N, t0, m);
        const int64_t t1 = min(t0 + tile, a.U);
        const int64_t u0 = a.unit_off[m];
        const int64_t n = a.msgs.n(m);
        // units of message m that are full (encode: all 12 bytes in range) or
        // interior (decode: not the message's last unit)
        const int64_t full = decode ? (n - 1) / 16 : n / 12;
        if (t1 <= u0 + full) {
            fast(m, t0, t1, u0);
        } else {
#pragma unroll 1
            for (int k = 0; k < UPL; k++) general(m, t0 + (int64_t)k * blockDim.x + threadIdx.x);
        }
    }
}

template <int UPL>
__global__ __launch_bounds__(1024) void k_enc_batch_t(
    const uint8_t *__restrict__ src, Msgs msgs, int64_t N,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off,
    const uint8_t *__restrict__ flags, const int64_t *__restrict__ unit_off)
{
    __shared__ uint32_t s_tab[32];
    lds_fill(s_tab, &c_tab.enc[0][0], 128);
    __syncthreads();
    const BatchArgs a{msgs, N, unit_off[N], unit_off, out_off, flags};
    const uint8_t *tabs = (const uint8_t *)s_tab;
    auto fast = [&](int64_t m, int64_t t0, int64_t t1, int64_t u0) {
        const uint8_t *p = src + msgs.b(m);
        uint8_t *q = dst + out_off[m];
        const int fl = flags ? flags[m] : 0;
        const uint8_t *tab = tabs + 64 * (fl & M_URL);
        const int64_t j0 = t0 - u0, j1 = t1 - u0;
        const bool whole = t1 - t0 == (int64_t)blockDim.x * UPL;
        if ((((uintptr_t)p | (uintptr_t)q) & 3) == 0) {
            if (whole) enc_step<true, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab);
            else enc_step<true, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab);
        } else {
            if (whole) enc_step<false, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab);
            else enc_step<false, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab);
        }
    };
    auto general = [&](int64_t m0, int64_t u) {
        const LaneRef r = lane_ref(a, m0, u);
        if (!r.valid) return;
        const bool full = 12 * r.j + 12 <= r.n;
        uint32_t w[3];
        if (full) load12(src + r.b + 12 * r.j, w[0], w[1], w[2]);
        enc_batch_unit(src, dst, r, full, w, tabs);
    };
    batch_tiles<UPL>(a, fast, general, false);
}

template <int UPL>
__global__ __launch_bounds__(1024) void k_dec_batch_t(
    const uint8_t *__restrict__ src, Msgs msgs, int64_t N,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off,
    const uint8_t *__restrict__ flags, const int64_t *__restrict__ unit_off,
    int64_t *__restrict__ out_len, int64_t *__restrict__ err_off)
{
    __shared__ uint32_t s_tab[128];
    lds_fill(s_tab, &c_tab.dec[0][0], 512);
    __syncthreads();
    const BatchArgs a{msgs, N, unit_off[N], unit_off, out_off, flags};
    const uint8_t *tabs = (const uint8_t *)s_tab;
    auto fast = [&](int64_t m, int64_t t0, int64_t t1, int64_t u0) {
        const uint8_t *p = src + msgs.b(m);
        uint8_t *q = dst + out_off[m];
        const int fl = flags ? flags[m] : 0;
        const uint8_t *tab = tabs + 256 * (fl & M_URL);
        unsigned long long *slot = (unsigned long long *)&err_off[m];
        const int64_t j0 = t0 - u0, j1 = t1 - u0;
        const bool whole = t1 - t0 == (int64_t)blockDim.x * UPL;
        if ((((uintptr_t)p | (uintptr_t)q) & 3) == 0) {
            if (whole) dec_step<true, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot);
            else dec_step<true, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot);
        } else {
            if (whole) dec_step<false, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot);
            else dec_step<false, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot);
        }
    };
    auto general = [&](int64_t m0, int64_t u) {
        const LaneRef r = lane_ref(a, m0, u);
        if (!r.valid) return;
        const bool interior = 16 * r.j + 16 < r.n;
        uint32_t w[4];
        if (interior) load16(src + r.b + 16 * r.j, w[0], w[1], w[2], w[3]);
        dec_batch_unit(src, dst, r, interior, w, tabs, out_len, err_off);
    };
    batch_tiles<UPL>(a, fast, general, true);
}

__global__ void k_dec_batch_final(int64_t N, int64_t *__restrict__ out_len, int64_t *__restrict__ err_off)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = err_off[i];
        if (e == (int64_t)ERR_NONE) err_off[i] = -1;
        else out_len[i] = -1;
    }
}

// Exclusive scan of per-message output sizes by one workgroup.
__global__ __launch_bounds__(1024) void k_out_offsets(int dir, Msgs msgs, int64_t N,
                                                      const uint8_t *__restrict__ flags,
                                                      int64_t *__restrict__ out_off)
{
    const int64_t per = (N + blockDim.x - 1) / blockDim.x;
    const int64_t i0 = threadIdx.x * per;
    const int64_t i1 = min(N, i0 + per);
    int64_t s = 0;
    for (int64_t i = i0; i < i1; i++) {
        const int64_t len = msgs.n(i);
        const int nopad = flags ? (flags[i] & M_NOPAD) : 0;
        s += dir == B64_DIR_ENCODE ? 4 * ((len + 2) / 3) : dec_slot_of(len, nopad);
    }
    int64_t acc = block_exclusive_scan(s);
    for (int64_t i = i0; i < i1; i++) {
        out_off[i] = acc;
        const int64_t len = msgs.n(i);
        const int nopad = flags ? (flags[i] & M_NOPAD) : 0;
        acc += dir == B64_DIR_ENCODE ? 4 * ((len + 2) / 3) : dec_slot_of(len, nopad);
    }
    if (i0 < N && i1 == N) out_off[N] = acc;
    if (N == 0 && threadIdx.x == 0) out_off[0] = 0;
}

// ================================================================= host ==
namespace {

struct DevCache {
    int cus = 0;
};

std::mutex g_mu;
std::vector<DevCache> g_dev;

int device_cus(int *out)
{
    int dev;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(B64_HIP_ERROR, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    if (!g_dev[dev].cus) {
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return fail(B64_HIP_ERROR, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
        g_dev[dev].cus = c;
    }
    *out = g_dev[dev].cus;
    return B64_OK;
}

// Launch shapes of the single-buffer kernels (settable for tuning sweeps).
// Default: 512 lanes x 2 units per workgroup and one workgroup per tile
// (blocks_per_cu == 0), the fastest shape of a sweep over block {256, 512,
// 1024} x units {1, 2, 4, 8} x grid {2..64 per CU, one-shot} on MI355X for
// both directions at 1 GiB.
struct Shape {
    std::atomic<int> block{512};
    std::atomic<int> upl{2};
    std::atomic<int> blocks_per_cu{0};
};
Shape g_single[2];

// Per-thread, per-device result slots of the synchronous decode:
// [0] error slot (u64, kept at ERR_NONE between calls), [1] length written by
// the final unit, [2] verdict length, [3] verdict error offset.
struct SyncSlot {
    int dev = -1;
    unsigned long long *d = nullptr;
    int64_t *h = nullptr;
};
thread_local std::vector<SyncSlot> t_slots;

int sync_slot(SyncSlot **out)
{
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    for (auto &s : t_slots)
        if (s.dev == dev) { *out = &s; return B64_OK; }
    SyncSlot s;
    s.dev = dev;
    HIP_TRY(hipMalloc((void **)&s.d, 64));
    HIP_TRY(hipHostMalloc((void **)&s.h, 16, hipHostMallocDefault));
    unsigned long long init[4] = {ERR_NONE, 0ull, 0ull, 0ull};
    HIP_TRY(hipMemcpy(s.d, init, sizeof init, hipMemcpyHostToDevice));
    t_slots.push_back(s);
    *out = &t_slots.back();
    return B64_OK;
}

int parse_mode(int alphabet, int *mode)
{
    const int a = alphabet & 0xff;
    if (a != B64_ALPHABET_STD && a != B64_ALPHABET_URL) return fail(B64_BAD_ARG, "bad alphabet %d", a);
    if (alphabet & ~(0xff | B64_MODE_STRICT | B64_MODE_NOPAD))
        return fail(B64_BAD_ARG, "unknown mode bits 0x%x", alphabet);
    if ((alphabet & B64_MODE_STRICT) && (alphabet & B64_MODE_NOPAD))
        return fail(B64_BAD_ARG, "strict and unpadded modes cannot be combined");
    *mode = (a ? M_URL : 0) | ((alphabet & B64_MODE_STRICT) ? M_STRICT : 0) |
            ((alphabet & B64_MODE_NOPAD) ? M_NOPAD : 0);
    return B64_OK;
}

int single_grid(int dir, int64_t units, int *block, int *upl, int *grid)
{
    int cus;
    int rc = device_cus(&cus);
    if (rc) return rc;
    *block = g_single[dir].block.load();
    *upl = g_single[dir].upl.load();
    const int64_t per = (int64_t)(*block) * (*upl);
    int64_t tiles = (units + per - 1) / per;
    const int bpc = g_single[dir].blocks_per_cu.load();
    int64_t cap = bpc ? (int64_t)cus * bpc : (int64_t)INT32_MAX;
    *grid = (int)std::max<int64_t>(1, std::min(tiles, cap));
    return B64_OK;
}

template <bool A>
void launch_enc_single(int upl, int grid, int block, const uint8_t *src, int64_t n, uint8_t *dst,
                       int mode, hipStream_t s)
{
    switch (upl) {
    case 1: hipLaunchKernelGGL((k_enc_single<A, 1>), grid, block, 0, s, src, n, dst, mode); break;
    case 2: hipLaunchKernelGGL((k_enc_single<A, 2>), grid, block, 0, s, src, n, dst, mode); break;
    case 8: hipLaunchKernelGGL((k_enc_single<A, 8>), grid, block, 0, s, src, n, dst, mode); break;
    default: hipLaunchKernelGGL((k_enc_single<A, 4>), grid, block, 0, s, src, n, dst, mode); break;
    }
}

template <bool A>
void launch_dec_single(int upl, int grid, int block, const uint8_t *src, int64_t n, uint8_t *dst,
                       int mode, unsigned long long *slot, int64_t *len_slot, hipStream_t s)
{
    switch (upl) {
    case 1: hipLaunchKernelGGL((k_dec_single<A, 1>), grid, block, 0, s, src, n, dst, mode, slot, len_slot); break;
    case 2: hipLaunchKernelGGL((k_dec_single<A, 2>), grid, block, 0, s, src, n, dst, mode, slot, len_slot); break;
    case 8: hipLaunchKernelGGL((k_dec_single<A, 8>), grid, block, 0, s, src, n, dst, mode, slot, len_slot); break;
    default: hipLaunchKernelGGL((k_dec_single<A, 4>), grid, block, 0, s, src, n, dst, mode, slot, len_slot); break;
    }
}

bool aligned4(const void *a, const void *b)
{
    return (((uintptr_t)a | (uintptr_t)b) & 3) == 0;
}

int enqueue_encode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(0, n / 12, &block, &upl, &grid);
    if (rc) return rc;
    if (aligned4(src, dst)) launch_enc_single<true>(upl, grid, block, src, n, dst, mode, s);
    else launch_enc_single<false>(upl, grid, block, src, n, dst, mode, s);
    LAUNCH_TRY();
    return B64_OK;
}

// Enqueues the decode kernel of src[0, n) (n >= 1); the error slot must hold
// ERR_NONE. No verdict is formed here (see k_dec_final / k_dec_batch_final).
int enqueue_decode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, unsigned long long *slot,
                   int64_t *len_slot, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(1, (n - 1) / 16, &block, &upl, &grid);
    if (rc) return rc;
    if (aligned4(src, dst)) launch_dec_single<true>(upl, grid, block, src, n, dst, mode, slot, len_slot, s);
    else launch_dec_single<false>(upl, grid, block, src, n, dst, mode, slot, len_slot, s);
    LAUNCH_TRY();
    return B64_OK;
}

int64_t enc_len_host(int64_t n, int mode)
{
    if (mode & M_NOPAD) return 4 * (n / 3) + ((n % 3) ? (n % 3) + 1 : 0);
    return 4 * ((n + 2) / 3);
}

}  // namespace

// ================================================================ C-ABI ==
extern "C" {

const char *b64_last_error(void) { return t_err.c_str(); }

int b64_device_cus(void)
{
    int c;
    int rc = device_cus(&c);
    return rc ? rc : c;
}

int64_t b64_encoded_len(int64_t n)
{
    if (n < 0) return fail(B64_BAD_ARG, "negative length");
    return 4 * ((n + 2) / 3);
}

int64_t b64_encoded_len_mode(int64_t n, int mode)
{
    int m;
    if (n < 0) return fail(B64_BAD_ARG, "negative length");
    int rc = parse_mode(mode, &m);
    if (rc) return rc;
    return enc_len_host(n, m);
}

int64_t b64_decoded_max(int64_t m)
{
    if (m < 0) return fail(B64_BAD_ARG, "negative length");
    return 3 * (m / 4);
}

int64_t b64_decoded_max_mode(int64_t m, int mode)
{
    int md;
    if (m < 0) return fail(B64_BAD_ARG, "negative length");
    int rc = parse_mode(mode, &md);
    if (rc) return rc;
    return 3 * (m / 4) + (((md & M_NOPAD) && (m & 3) >= 2) ? (m & 3) - 1 : 0);
}

int64_t b64_encode_ex(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, void *stream)
{
    int mode;
    int rc = parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (n < 0) return fail(B64_BAD_ARG, "negative length");
    if (n == 0) return 0;
    if (!src || !dst) return fail(B64_BAD_ARG, "null buffer with n > 0");
    rc = enqueue_encode(src, n, dst, mode, (hipStream_t)stream);
    if (rc) return rc;
    return enc_len_host(n, mode);
}

int64_t b64_encode(const uint8_t *src, int64_t n, uint8_t *dst)
{
    int64_t r = b64_encode_ex(src, n, dst, B64_ALPHABET_STD, nullptr);
    if (r > 0) HIP_TRY(hipStreamSynchronize(nullptr));
    return r;
}

int64_t b64_decode_ex(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off, int alphabet,
                      void *stream)
{
    int mode;
    int rc = parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (!err_off) return fail(B64_BAD_ARG, "null err_off");
    if (n < 0) return fail(B64_BAD_ARG, "negative length");
    *err_off = -1;
    if (n == 0) return 0;
    if (!src || (!dst && n >= 4)) return fail(B64_BAD_ARG, "null buffer with n > 0");
    SyncSlot *sl;
    rc = sync_slot(&sl);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_decode(src, n, dst, mode, sl->d, (int64_t *)(sl->d + 1), s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dec_final, 1, 64, 0, s, sl->d, (const int64_t *)(sl->d + 1), (int64_t *)(sl->d + 2),
                       (int64_t *)(sl->d + 3), 1);
    LAUNCH_TRY();
    HIP_TRY(hipMemcpyAsync(sl->h, sl->d + 2, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t len = sl->h[0], err = sl->h[1];
    if (len < 0) {
        *err_off = err;
        t_err = "invalid base64 input";
        return B64_INVALID_INPUT;
    }
    return len;
}

int64_t b64_decode(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off)
{
    return b64_decode_ex(src, n, dst, err_off, B64_ALPHABET_STD, nullptr);
}

int b64_decode_async(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, int64_t *d_len,
                     int64_t *d_err, void *stream)
{
    int mode;
    int rc = parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (n < 0) return fail(B64_BAD_ARG, "negative length");
    if (!d_len || !d_err) return fail(B64_BAD_ARG, "null result slot");
    if (n > 0 && (!src || (!dst && n >= 4))) return fail(B64_BAD_ARG, "null buffer with n > 0");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_slots_init, 1, 64, 0, s, d_len, d_err, n == 0 ? 1 : 0);
    LAUNCH_TRY();
    if (n == 0) return B64_OK;
    rc = enqueue_decode(src, n, dst, mode, (unsigned long long *)d_err, d_len, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dec_final, 1, 64, 0, s, (unsigned long long *)d_err, d_len, d_len, d_err, 0);
    LAUNCH_TRY();
    return B64_OK;
}

int b64_set_single_tune(int dir, const b64_tune *t)
{
    if (dir != 0 && dir != 1) return fail(B64_BAD_ARG, "bad direction");
    if (!t) return fail(B64_BAD_ARG, "null tune");
    if (t->block) {
        if (t->block < 64 || t->block > 1024 || (t->block & 63)) return fail(B64_BAD_ARG, "bad block");
        g_single[dir].block = t->block;
    }
    if (t->units_per_lane) {
        if (t->units_per_lane != 1 && t->units_per_lane != 2 && t->units_per_lane != 4 &&
            t->units_per_lane != 8)
            return fail(B64_BAD_ARG, "units_per_lane must be 1, 2, 4 or 8");
        g_single[dir].upl = t->units_per_lane;
    }
    if (t->grid) {
        // blocks per CU; -1 selects one workgroup per tile
        if (t->grid < -1 || t->grid > 4096) return fail(B64_BAD_ARG, "blocks per CU must be -1 or 1..4096");
        g_single[dir].blocks_per_cu = t->grid < 0 ? 0 : t->grid;
    }
    return B64_OK;
}

int64_t b64_batch_workspace_bytes(int64_t N)
{
    if (N < 0) return fail(B64_BAD_ARG, "negative N");
    const int64_t chunks = (N + PLAN_CHUNK - 1) / PLAN_CHUNK;
    return 8 * (N + 1) + 8 * std::max<int64_t>(chunks, 1);
}

int b64_batch_out_offsets(int dir, const int64_t *in_off, int64_t N, int64_t *out_off,
                          const uint8_t *flags, void *stream)
{
    if (dir != B64_DIR_ENCODE && dir != B64_DIR_DECODE) return fail(B64_BAD_ARG, "bad direction");
    if (N < 0 || !in_off || !out_off) return fail(B64_BAD_ARG, "bad offsets arguments");
    Msgs msgs{in_off, nullptr};
    hipLaunchKernelGGL(k_out_offsets, 1, 1024, 0, (hipStream_t)stream, dir, msgs, N, flags, out_off);
    LAUNCH_TRY();
    return B64_OK;
}

}  // extern "C"

namespace {

// Launch shape of the batched kernels: tuned values or the defaults
// (layout 0, 512 threads x 2 units, 32 workgroups per CU: the best shape of
// the tile layout on large messages on MI355X).
int batch_shape(const b64_tune *t, int *block, int *upl, int *grid, int *layout)
{
    int cus;
    int rc = device_cus(&cus);
    if (rc) return rc;
    *layout = t ? t->layout : 0;
    const bool tiles = *layout == 0;
    *block = (t && t->block) ? t->block : (tiles ? 512 : 256);
    *upl = (t && t->units_per_lane) ? t->units_per_lane : 2;
    *grid = (t && t->grid) ? t->grid : cus * (tiles ? 32 : 8);
    if (*layout != 0 && *layout != 1) return fail(B64_BAD_ARG, "bad layout %d", *layout);
    if (*block < 64 || *block > 1024 || (*block & 63)) return fail(B64_BAD_ARG, "bad block size %d", *block);
    if (*upl != 1 && *upl != 2 && *upl != 4 && *upl != 8) return fail(B64_BAD_ARG, "bad units_per_lane %d", *upl);
    if (*grid < 1 || *grid > (1 << 20)) return fail(B64_BAD_ARG, "bad grid %d", *grid);
    return B64_OK;
}

template <int DIR>
int plan(Msgs msgs, int64_t N, const uint8_t *flags, void *ws, int64_t ws_bytes, int64_t *out_len,
         int64_t *err_off, int64_t **unit_off, hipStream_t s)
{
    if (ws_bytes < b64_batch_workspace_bytes(N) || !ws) return fail(B64_BAD_ARG, "workspace too small");
    const int64_t chunks = std::max<int64_t>(1, (N + PLAN_CHUNK - 1) / PLAN_CHUNK);
    *unit_off = (int64_t *)ws;
    int64_t *partial = (int64_t *)ws + (N + 1);
    hipLaunchKernelGGL((k_plan_reduce<DIR>), (unsigned)chunks, PLAN_BLOCK, 0, s, msgs, N, partial);
    LAUNCH_TRY();
    hipLaunchKernelGGL((k_plan_scan<DIR>), (unsigned)chunks, PLAN_BLOCK, 0, s, msgs, N, flags, partial,
                       *unit_off, out_len, err_off);
    LAUNCH_TRY();
    return B64_OK;
}

#define B64_LAUNCH_UPL(KERN, UPL, ...)                                                   \
    switch (UPL) {                                                                       \
    case 1: hipLaunchKernelGGL((KERN<1>), grid, block, 0, s, __VA_ARGS__); break;        \
    case 4: hipLaunchKernelGGL((KERN<4>), grid, block, 0, s, __VA_ARGS__); break;        \
    case 8: hipLaunchKernelGGL((KERN<8>), grid, block, 0, s, __VA_ARGS__); break;        \
    default: hipLaunchKernelGGL((KERN<2>), grid, block, 0, s, __VA_ARGS__); break;       \
    }

int launch_enc_batch(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, const int64_t *unit_off, const b64_tune *tune, hipStream_t s)
{
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    if (layout == 1) {
        B64_LAUNCH_UPL(k_enc_batch_w, upl, src, msgs, N, dst, out_off, flags, unit_off);
    } else {
        B64_LAUNCH_UPL(k_enc_batch_t, upl, src, msgs, N, dst, out_off, flags, unit_off);
    }
    LAUNCH_TRY();
    return B64_OK;
}

int launch_dec_batch(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                     const b64_tune *tune, hipStream_t s)
{
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    if (layout == 1) {
        B64_LAUNCH_UPL(k_dec_batch_w, upl, src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off);
    } else {
        B64_LAUNCH_UPL(k_dec_batch_t, upl, src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off);
    }
    LAUNCH_TRY();
    const int fb = (int)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_dec_batch_final, fb, 256, 0, s, N, out_len, err_off);
    LAUNCH_TRY();
    return B64_OK;
}

int encode_batch_any(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, int64_t *out_len, void *ws, int64_t ws_bytes,
                     const b64_tune *tune, hipStream_t s)
{
    if (N < 0) return fail(B64_BAD_ARG, "negative N");
    if (N == 0) return B64_OK;
    if (!src || !msgs.begin || !dst || !out_off || !out_len) return fail(B64_BAD_ARG, "null argument");
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    int64_t *unit_off;
    rc = plan<B64_DIR_ENCODE>(msgs, N, flags, ws, ws_bytes, out_len, nullptr, &unit_off, s);
    if (rc) return rc;
    return launch_enc_batch(src, msgs, N, dst, out_off, flags, unit_off, tune, s);
}

int decode_batch_any(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, int64_t *out_len, int64_t *err_off, void *ws,
                     int64_t ws_bytes, const b64_tune *tune, hipStream_t s)
{
    if (N < 0) return fail(B64_BAD_ARG, "negative N");
    if (N == 0) return B64_OK;
    if (!src || !msgs.begin || !dst || !out_off || !out_len || !err_off) return fail(B64_BAD_ARG, "null argument");
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    int64_t *unit_off;
    rc = plan<B64_DIR_DECODE>(msgs, N, flags, ws, ws_bytes, out_len, err_off, &unit_off, s);
    if (rc) return rc;
    return launch_dec_batch(src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off, tune, s);
}

}  // namespace

// Planned batch launches for the serving runtime: the caller supplies the
// unit prefix (and, for decode, out_len = 0 / err_off = ERR_NONE) computed on
// the host and uploaded together with the descriptors, so a serving batch is
// one upload, one codec kernel and (decode) one verdict kernel.
int b64i_encode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, const b64_tune *tune, hipStream_t s)
{
    if (N <= 0) return B64_OK;
    return launch_enc_batch(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, unit_off, tune, s);
}

int b64i_decode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                        const b64_tune *tune, hipStream_t s)
{
    if (N <= 0) return B64_OK;
    return launch_dec_batch(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, unit_off, out_len,
                            err_off, tune, s);
}

int b64i_fail(int code, const char *msg) { return fail(code, "%s", msg); }

extern "C" {

int b64_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                     const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                     void *workspace, int64_t workspace_bytes, const b64_tune *tune, void *stream)
{
    return encode_batch_any(src, Msgs{in_off, nullptr}, N, dst, out_off, flags, out_len, workspace,
                            workspace_bytes, tune, (hipStream_t)stream);
}

int b64_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                     const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                     int64_t *err_off, void *workspace, int64_t workspace_bytes,
                     const b64_tune *tune, void *stream)
{
    return decode_batch_any(src, Msgs{in_off, nullptr}, N, dst, out_off, flags, out_len, err_off,
                            workspace, workspace_bytes, tune, (hipStream_t)stream);
}

int b64_encode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, void *workspace, int64_t workspace_bytes,
                            const b64_tune *tune, void *stream)
{
    if (N > 0 && !in_len) return fail(B64_BAD_ARG, "null in_len");
    return encode_batch_any(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, out_len, workspace,
                            workspace_bytes, tune, (hipStream_t)stream);
}

int b64_decode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, int64_t *err_off, void *workspace,
                            int64_t workspace_bytes, const b64_tune *tune, void *stream)
{
    if (N > 0 && !in_len) return fail(B64_BAD_ARG, "null in_len");
    return decode_batch_any(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, out_len, err_off,
                            workspace, workspace_bytes, tune, (hipStream_t)stream);
}

int b64_encode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len, void *stream)
{
    if (N < 0 || !h_in_off || !h_out_off) return fail(B64_BAD_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> lens(N);
    for (int64_t i = 0; i < N; i++) {
        const int64_t n = h_in_off[i + 1] - h_in_off[i];
        const int fl = h_flags ? h_flags[i] : 0;
        const int mode = (fl & M_URL) | (fl & M_NOPAD);
        lens[i] = enc_len_host(n, mode);
        if (n > 0) {
            int rc = enqueue_encode(src + h_in_off[i], n, dst + h_out_off[i], mode, s);
            if (rc) return rc;
        }
    }
    if (out_len && N) HIP_TRY(hipMemcpyAsync(out_len, lens.data(), 8 * N, hipMemcpyHostToDevice, s));
    if (N) HIP_TRY(hipStreamSynchronize(s));  // lens is a local host buffer
    return B64_OK;
}

__global__ void k_each_init(int64_t N, int64_t *__restrict__ d_len, int64_t *__restrict__ d_err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        d_len[i] = 0;
        d_err[i] = (int64_t)ERR_NONE;
    }
}

int b64_decode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len,
                    int64_t *err_off, void *stream)
{
    if (N < 0 || !h_in_off || !h_out_off || !out_len || !err_off) return fail(B64_BAD_ARG, "bad arguments");
    if (N == 0) return B64_OK;
    hipStream_t s = (hipStream_t)stream;
    const int fb = (int)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_each_init, fb, 256, 0, s, N, out_len, err_off);
    LAUNCH_TRY();
    for (int64_t i = 0; i < N; i++) {
        const int64_t n = h_in_off[i + 1] - h_in_off[i];
        const int fl = h_flags ? h_flags[i] : 0;
        if (n == 0) continue;  // verdict (0, -1) comes from the init and final passes
        int rc = enqueue_decode(src + h_in_off[i], n, dst + h_out_off[i], fl & 7,
                                (unsigned long long *)(err_off + i), out_len + i, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_dec_batch_final, fb, 256, 0, s, N, out_len, err_off);
    LAUNCH_TRY();
    return B64_OK;
}

}  // extern "C"
