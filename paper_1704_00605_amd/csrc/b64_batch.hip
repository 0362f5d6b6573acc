// gfx950 kernels of the batched codec and their C-ABI (include/b64.h).
//
//   k_plan_reduce / k_plan_scan   device planning: per-message unit counts ->
//                                 exclusive scan (unit_off), output-length
//                                 and error-slot init. A decode's verdict
//                                 slots are final when its codec kernel
//                                 ends (see msg_error).
//   k_enc_batch_t / k_dec_batch_t persistent codec, tile layout: tiles of
//                                 the flattened unit space of all messages,
//                                 grid-stride.
//   k_enc_batch_w / k_dec_batch_w persistent codec, wave layout: one
//                                 contiguous range of 64-unit groups per wave.
//   k_batch_s                     staged layout: one workgroup per tile of
//                                 units, the tile's input read as aligned
//                                 16-byte chunks into LDS, its messages found
//                                 from a tile table filled by the planning
//                                 pass.
//   k_out_reduce / k_out_scan     exclusive scan of output sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "b64.h"
#include "b64_device.hpp"
#include "b64_internal.hpp"

using namespace b64dev;

static __constant__ Tables c_tab = make_tables();

constexpr int PLAN_BLOCK = 256;
constexpr int PLAN_PER_THREAD = 2;
constexpr int PLAN_CHUNK = PLAN_BLOCK * PLAN_PER_THREAD;
// Up to this many chunks (1,048,576 messages) each chunk of k_plan_scan sums
// the totals of the chunks before it itself (at most 8 loads per thread, no
// extra launch); beyond, that sum would grow with the square of the chunk
// count, so k_plan_top scans the totals first.
constexpr int64_t PLAN_DIRECT_CHUNKS = 2048;

__device__ __forceinline__ int64_t units_of(int dir, int64_t len)
{
    return dir == B64_DIR_ENCODE ? (len + 11) / 12 : (len + 15) / 16;
}

__host__ __device__ __forceinline__ int64_t enc_len_of(int64_t len, int nopad)
{
    return nopad ? 4 * (len / 3) + ((len % 3) ? (len % 3) + 1 : 0) : 4 * ((len + 2) / 3);
}

__host__ __device__ __forceinline__ int64_t dec_cap_of(int64_t len, int nopad)
{
    return 3 * (len / 4) + ((nopad && (len & 3) >= 2) ? (len & 3) - 1 : 0);
}

// Decode output slot of the batch layout: the capacity rounded up to a
// multiple of 4 so every slot starts where dst's alignment allows dword
// stores (each 16-character unit writes 12 bytes at offset 12j of its slot).
__host__ __device__ __forceinline__ int64_t dec_slot_of(int64_t len, int nopad)
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

// Tile table of the staged layout (tiles of T consecutive units of the
// flattened unit space): m[t] is the message holding tile t's first unit
// (t < W) and A[t] the input byte where that unit starts (t <= W). T == 0:
// no table. Packed batches only (a tile's input is then one byte range,
// [A[t], A[t + 1]), or up to in_off[N] for the last tile).
struct TileTab {
    int64_t T, W;
    int64_t *A, *m;
};

// One block: exclusive scan of the chunk totals, in place (batches of more
// than PLAN_DIRECT_CHUNKS chunks).
__global__ __launch_bounds__(1024) void k_plan_top(int64_t chunks, int64_t *__restrict__ partial)
{
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < chunks; base += blockDim.x) {
        const int64_t c = base + threadIdx.x;
        const int64_t v = c < chunks ? partial[c] : 0;
        const int64_t ex = block_exclusive_scan(v);
        const int64_t carry = s_carry;
        if (c < chunks) partial[c] = carry + ex;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_carry = carry + ex + v;
        __syncthreads();
    }
}

// unit_off = exclusive scan of units per message (N + 1 entries), plus
// per-message initialisation: encode out_len (known from the length);
// decode out_len = 0 and err_off = -1 (see msg_error); and
// the tile table entries of the tiles whose first unit lies in the message.
template <int DIR>
__global__ __launch_bounds__(PLAN_BLOCK) void k_plan_scan(
    Msgs msgs, int64_t N, const uint8_t *__restrict__ flags,
    const int64_t *__restrict__ partial, int64_t *__restrict__ unit_off,
    int64_t *__restrict__ out_len, int64_t *__restrict__ err_off, TileTab tt, int scanned)
{
    // units before this chunk: partial holds the chunk totals, or (scanned)
    // their exclusive prefix
    int64_t pre = 0;
    if (scanned) {
        pre = partial[blockIdx.x];
    } else {
        for (int64_t c = threadIdx.x; c < blockIdx.x; c += blockDim.x) pre += partial[c];
        pre = block_sum(pre);
    }
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
                err_off[i] = -1;
            }
        }
        s += u[k];
    }
    int64_t ex = pre + block_exclusive_scan(s);
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        const int64_t i = i0 + k;
        if (i < N) {
            unit_off[i] = ex;
            if (tt.T > 0 && u[k] > 0) {
                // tiles t with t * T in [ex, ex + u[k])
                const int64_t ub = DIR == B64_DIR_ENCODE ? 12 : 16, b = msgs.b(i);
                const int64_t te = min((ex + u[k] + tt.T - 1) / tt.T, tt.W + 1);
                for (int64_t t = (ex + tt.T - 1) / tt.T; t < te; t++) {
                    tt.A[t] = b + ub * (t * tt.T - ex);
                    if (t < tt.W) tt.m[t] = i;
                }
            }
        }
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

// Verdict slots of a batched decode, formed in place: the plan sets
// out_len = 0 and err_off = -1, which as an unsigned value is above every
// index, so atomicMin keeps the first offending index and -1 stays where
// there is none. A unit that finds an error also sets out_len to -1; the
// final unit of a valid message moves out_len from 0 to its length, which
// fails once an error has set -1, and a later error overwrites the length.
// So the slots hold the verdict when the codec kernel ends, whatever order
// the units ran in.
__device__ __forceinline__ void msg_error(int64_t *__restrict__ out_len, int64_t *__restrict__ err_off, int64_t i,
                                          int64_t pos)
{
    atomicMin((unsigned long long *)&err_off[i], (unsigned long long)pos);
    atomicExch((unsigned long long *)&out_len[i], ~0ull);
}

__device__ __forceinline__ void msg_length(int64_t *__restrict__ out_len, int64_t i, int64_t len)
{
    atomicCAS((unsigned long long *)&out_len[i], 0ull, (unsigned long long)len);
}

// One unit of the batched decode: interior units (16 characters, none of
// them the message's last) or the final unit with the padding and length
// rules, reported through msg_error / msg_length.
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
        if (bad & INVALID)
            msg_error(out_len, err_off, r.mm, 16 * r.j + dec_first_bad(w[0], w[1], w[2], w[3], tab));
    } else {
        const int res = dec_tail_inl(src + r.b + 16 * r.j, (int)(r.n - 16 * r.j), r.n, q, tab, r.fl);
        if (res >= 0) msg_error(out_len, err_off, r.mm, 16 * r.j + res);
        else msg_length(out_len, r.mm, 12 * r.j + (-1 - res));
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

// Moves the cursor to the message holding unit gs (gs < U, not before it).
__device__ __forceinline__ void cursor_seek(Cursor &c, const BatchArgs &a, int64_t gs)
{
    if (c.u1 <= gs) {  // the group starts in a later message
        int64_t m = c.m + 1;
        while (a.unit_off[m + 1] <= gs) m++;  // skips messages without units
        cursor_load(c, a, m);
    }
}

// Units gs + lane of one 64-unit group (gs < U) that holds a message boundary
// or a message's final unit. One load brings the starts of the 64 messages
// after the cursor's message m0; each lane finds its message with a 64-way
// shuffle search and loads that message's metadata (none in the cursor's
// message; units more than 64 messages past m0 take the general search). The
// cursor then moves to the message of the group's last unit, from the
// registers of the lane that holds it.
__device__ __forceinline__ LaneRef resolve_group(Cursor &c, const BatchArgs &a, int64_t gs)
{
    cursor_seek(c, a, gs);
    const int lane = __lane_id();
    const int64_t m0 = c.m;
    const int64_t idx = m0 + 1 + lane;
    const int64_t B = idx <= a.N ? a.unit_off[idx] : INT64_MAX;  // first unit of message m0 + 1 + lane
    const int64_t b63 = __shfl(B, 63, 64);
    const int64_t u = gs + lane;
    LaneRef r;
    r.valid = u < a.U;
    int cnt = 0;
#pragma unroll
    for (int stp = 32; stp >= 1; stp >>= 1) {
        const int64_t b = __shfl(B, cnt + stp - 1, 64);
        if (b <= u) cnt += stp;
    }
    if (cnt == 63 && b63 <= u) cnt = 64;
    int64_t d = cnt;  // message of unit u, relative to m0
    const bool far = r.valid && cnt == 64;
    if (__ballot(far)) {  // rare: more than 64 messages ahead
        const int64_t m2 = lane_find_msg(a.unit_off, a.N, m0 + 64, u, far);
        if (far) d = m2 - m0;
    }
    const int64_t m = m0 + d;
    const int64_t wu = __shfl(B, (int)min(max(d - 1, (int64_t)0), (int64_t)63), 64);  // start of m when 1 <= d <= 64
    const int64_t wn = __shfl(B, (int)min(d, (int64_t)63), 64);                     // start of m + 1 when d <= 63
    int64_t u0 = c.u0, u1 = c.u1;
    r.mm = m;
    r.b = c.b; r.n = c.n; r.o = c.o; r.fl = c.fl;
    if (r.valid && d > 0) {
        u0 = d <= 64 ? wu : a.unit_off[m];
        u1 = d <= 63 ? wn : a.unit_off[m + 1];
        r.b = a.msgs.b(m);
        r.n = a.msgs.n(m);
        r.o = a.out_off[m];
        r.fl = a.flags ? a.flags[m] : 0;
    }
    r.j = u - u0;
    // the next group starts in the message of this group's last valid unit or later
    const unsigned long long vb = __ballot(r.valid);
    const int top = 63 - __clzll(vb);
    const int64_t last = uniform64(__shfl(r.mm, top, 64));
    if (last != c.m) {
        c.m = last;
        c.u0 = uniform64(__shfl(u0, top, 64));
        c.u1 = uniform64(__shfl(u1, top, 64));
        c.b = uniform64(__shfl(r.b, top, 64));
        c.n = uniform64(__shfl(r.n, top, 64));
        c.o = uniform64(__shfl(r.o, top, 64));
        c.fl = __builtin_amdgcn_readfirstlane(__shfl(r.fl, top, 64));
    }
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
    for (int64_t g = g0; g < g1;) {
        // whole groups of full units inside the cursor's message: the
        // single-buffer step (no per-lane message lookup or tail branches),
        // UPL groups at a time while they fit, then one at a time
        const int64_t gs = g * 64;
        cursor_seek(c, a, gs);
        const int64_t inside = (c.u0 + c.n / 12 - gs) / 64;
        if (inside >= 1) {
            const uint8_t *p = src + c.b;
            uint8_t *q = dst + c.o;
            const MapCtx mc{(const uint8_t *)s_tab + 64 * (c.fl & M_URL)};
            const int64_t first = gs - c.u0 + __lane_id();
            const bool al = (((uintptr_t)p | (uintptr_t)q) & 3) == 0;
            if (inside >= UPL && g + UPL <= g1) {
                if (al) enc_step<true, UPL, false>(p, q, first, 64, 0, mc);
                else enc_step<false, UPL, false>(p, q, first, 64, 0, mc);
                g += UPL;
            } else {
                if (al) enc_step<true, 1, false>(p, q, first, 64, 0, mc);
                else enc_step<false, 1, false>(p, q, first, 64, 0, mc);
                g += 1;
            }
            continue;
        }
        // one group holding a message boundary or a message's final unit,
        // resolved per lane; the single-buffer step resumes after it
        const LaneRef r = resolve_group(c, a, gs);
        uint32_t w[3];
        const bool full = r.valid && 12 * r.j + 12 <= r.n;
        if (full) load12(src + r.b + 12 * r.j, w[0], w[1], w[2]);
        if (r.valid) enc_batch_unit(src, dst, r, full, w, (const uint8_t *)s_tab);
        g += 1;
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
    for (int64_t g = g0; g < g1;) {
        // whole groups of interior units inside the cursor's message: the
        // single-buffer step, UPL groups at a time while they fit, then one
        // at a time
        const int64_t gs = g * 64;
        cursor_seek(c, a, gs);
        const int64_t inside = (c.u0 + (c.n - 1) / 16 - gs) / 64;
        if (inside >= 1) {
            const uint8_t *p = src + c.b;
            uint8_t *q = dst + c.o;
            const MapCtx mc{(const uint8_t *)s_tab + 256 * (c.fl & M_URL)};
            unsigned long long *slot = (unsigned long long *)&err_off[c.m];
            int64_t *lslot = &out_len[c.m];
            const int64_t first = gs - c.u0 + __lane_id();
            const bool al = (((uintptr_t)p | (uintptr_t)q) & 3) == 0;
            if (inside >= UPL && g + UPL <= g1) {
                if (al) dec_step<true, UPL, false>(p, q, first, 64, 0, mc, slot, 0, lslot);
                else dec_step<false, UPL, false>(p, q, first, 64, 0, mc, slot, 0, lslot);
                g += UPL;
            } else {
                if (al) dec_step<true, 1, false>(p, q, first, 64, 0, mc, slot, 0, lslot);
                else dec_step<false, 1, false>(p, q, first, 64, 0, mc, slot, 0, lslot);
                g += 1;
            }
            continue;
        }
        // one group holding a message boundary or a message's final unit,
        // resolved per lane; the single-buffer step resumes after it
        const LaneRef r = resolve_group(c, a, gs);
        uint32_t w[4];
        const bool interior = r.valid && 16 * r.j + 16 < r.n;
        if (interior) load16(src + r.b + 16 * r.j, w[0], w[1], w[2], w[3]);
        if (r.valid) dec_batch_unit(src, dst, r, interior, w, (const uint8_t *)s_tab, out_len, err_off);
        g += 1;
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
    const int64_t stride = (int64_t)gridDim.x * tile;
    int64_t t0 = (int64_t)blockIdx.x * tile;
    if (t0 >= a.U) return;
    int64_t m = block_find_msg(a.unit_off, a.N, t0, 0);
    for (; t0 < a.U; t0 += stride) {
        // The next tile's search starts here: every thread probes one of the
        // blockDim.x messages after m against the next tile's first unit, and
        // the probe loads stay in flight while this tile is worked on.
        const int64_t tn = t0 + stride;
        const int64_t pi = m + 1 + threadIdx.x;
        const int ok = tn < a.U && pi < a.N && a.unit_off[pi] <= tn;
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
        // unit_off does not decrease, so the probes hold for a prefix: the
        // next tile's first message is m + (their count), unless all of them
        // hold (then a full search above the window)
        const int64_t cnt = __syncthreads_count(ok);
        m = cnt < (int64_t)blockDim.x ? m + cnt : block_find_msg(a.unit_off, a.N, tn, m + blockDim.x);
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
        const MapCtx tab{tabs + 64 * (fl & M_URL)};
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
        const MapCtx tab{tabs + 256 * (fl & M_URL)};
        unsigned long long *slot = (unsigned long long *)&err_off[m];
        int64_t *lslot = &out_len[m];
        const int64_t j0 = t0 - u0, j1 = t1 - u0;
        const bool whole = t1 - t0 == (int64_t)blockDim.x * UPL;
        if ((((uintptr_t)p | (uintptr_t)q) & 3) == 0) {
            if (whole) dec_step<true, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot, 0, lslot);
            else dec_step<true, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot, 0, lslot);
        } else {
            if (whole) dec_step<false, UPL, false>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot, 0, lslot);
            else dec_step<false, UPL, true>(p, q, j0 + threadIdx.x, blockDim.x, j1, tab, slot, 0, lslot);
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

// ---------------------------------------------------------------- layout 2
// Staged layout: one workgroup per tile of S_BLOCK * UPL consecutive units
// (grid-stride when the grid is smaller than the tile count). A packed
// batch's units tile its input without gaps, so a tile's input is the byte
// range [A[t], A[t + 1]) of the tile table whatever the message boundaries
// and alignments inside it. The workgroup reads that range as aligned 16-byte
// chunks (each holds a byte of the range, so every read lies on a page the
// buffer occupies) into LDS, in the same round as the metadata of the
// messages from the tile's first one on; each lane then finds its unit's
// message by a binary search over the staged message starts and reads its
// 12 (encode) or 16 (decode) bytes from LDS at any alignment. Tiles past the
// table or starting more than S_META messages take a per-lane path instead
// (each lane searches its unit's message and reads its bytes from global
// memory).
constexpr int S_BLOCK = 256;
constexpr int S_META = 64;  // messages one wave stages per tile

// Bytes o .. o + 15 of an LDS byte buffer (any o with o + 20 inside it).
__device__ __forceinline__ void lds_read16(const uint32_t *lds, uint32_t o, uint32_t (&w)[4])
{
    const uint32_t d = o >> 2, sh = o & 3;
    uint32_t x[5];
#pragma unroll
    for (int k = 0; k < 5; k++) x[k] = lds[d + k];
#pragma unroll
    for (int k = 0; k < 4; k++) w[k] = alignb(x[k + 1], x[k], sh);
}

// Zeroes bytes r .. 15 of w (r in 1..16).
__device__ __forceinline__ void keep_bytes(uint32_t (&w)[4], int r)
{
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int keep = r - 4 * k;
        w[k] = keep >= 4 ? w[k] : keep <= 0 ? 0u : (w[k] & ((1u << (8 * keep)) - 1u));
    }
}

// Largest m in [lo, N) with unit_off[m] <= u (unit_off[lo] <= u < unit_off[N]),
// by one lane on its own: galloping from lo (one probe when u lies in
// message lo, as in tiles inside a long message), then a binary search.
__device__ __forceinline__ int64_t lane_search_msg(const int64_t *__restrict__ unit_off, int64_t N, int64_t u,
                                                   int64_t lo)
{
    int64_t hi = N, step = 1;
    while (lo + step < N && unit_off[lo + step] <= u) {
        lo += step;
        step *= 2;
    }
    hi = min(N, lo + step);  // unit_off[lo] <= u < unit_off[hi]
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (unit_off[mid] <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int DIR, int UPL>
__global__ __launch_bounds__(S_BLOCK) void k_batch_s(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t N,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off,
    const uint8_t *__restrict__ flags, const int64_t *__restrict__ unit_off,
    const int64_t *__restrict__ tile_A, const int64_t *__restrict__ tile_m, int64_t W,
    int64_t *__restrict__ out_len, int64_t *__restrict__ err_off)
{
    constexpr bool ENC = DIR == B64_DIR_ENCODE;
    constexpr int UB = ENC ? 12 : 16;                   // input bytes per unit
    constexpr int64_t T = (int64_t)S_BLOCK * UPL;      // units per tile
    constexpr int CH = (int)((T * UB + 15) / 16 + 3);  // 16-byte chunks staged (+ misalignment, + read slack)
    constexpr int PER = (CH + S_BLOCK - 1) / S_BLOCK;
    __shared__ uint32_t s_tab[ENC ? 32 : 128];
    __shared__ uint4 s_data[CH];
    __shared__ int64_t s_u[S_META + 1], s_b[S_META + 1], s_o[S_META];
    __shared__ uint8_t s_f[S_META];
    __shared__ int s_over;
    lds_fill(s_tab, ENC ? &c_tab.enc[0][0] : &c_tab.dec[0][0], ENC ? 128 : 512);
    const int tid = threadIdx.x;
    const int64_t U = unit_off[N];
    const int64_t ntiles = (U + T - 1) / T;
    const uint8_t *tabs = (const uint8_t *)s_tab;
    const uint32_t *lds = (const uint32_t *)s_data;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();  // the previous tile's LDS reads (and the table fill) are done
        const int64_t t0 = t * T, t1 = min(t0 + T, U);
        int64_t m0;
        uintptr_t c0 = 0;
        int K = 0;
        bool staged = t < W;
        if (staged) {
            m0 = tile_m[t];
            const int64_t A = tile_A[t];
            const int64_t B = t + 1 < ntiles ? tile_A[t + 1] : in_off[N];
            // one round of loads: the messages from m0 on (one per lane of
            // wave 0, plus one more by thread 0) and the tile's input chunks
            const int64_t idx = m0 + tid;
            const bool meta = tid < S_META;
            const int64_t mu = (meta && idx <= N) ? unit_off[idx] : INT64_MAX;
            const int64_t mb = (meta && idx <= N) ? in_off[idx] : 0;
            const int64_t mo = (meta && idx < N) ? out_off[idx] : 0;
            const int mf = (meta && idx < N && flags) ? flags[idx] : 0;
            int64_t mu_x = INT64_MAX, mb_x = 0;
            if (tid == 0 && m0 + S_META <= N) {
                mu_x = unit_off[m0 + S_META];
                mb_x = in_off[m0 + S_META];
            }
            c0 = ((uintptr_t)src + (uintptr_t)A) >> 4;
            const int64_t nch = B > A ? (int64_t)((((uintptr_t)src + (uintptr_t)B - 1) >> 4) - c0) + 1 : 0;
            // chunks straight into LDS (no registers): lane l of wave w loads
            // chunk k * S_BLOCK + 64 w + l, which the load writes at 16 l past
            // its wave's LDS base
            const int wv = tid >> 6;
#pragma unroll
            for (int k = 0; k < PER; k++) {
                const int64_t i = tid + k * S_BLOCK;
                if (i < nch) {
                    const uint8_t *p = src + (int64_t)((((uintptr_t)c0 + i) << 4) - (uintptr_t)src);
                    __builtin_amdgcn_global_load_lds(
                        (const void *)p, (__attribute__((address_space(3))) void *)(s_data + k * S_BLOCK + 64 * wv), 16, 0, 0);
                }
            }
            if (meta) {
                s_u[tid] = mu;
                s_b[tid] = mb;
                s_o[tid] = mo;
                s_f[tid] = (uint8_t)mf;
            }
            if (tid == 0) {
                s_u[S_META] = mu_x;
                s_b[S_META] = mb_x;
                s_over = mu_x < t1;
            }
            __builtin_amdgcn_s_waitcnt(0);  // this wave's chunks have landed in LDS
            // messages starting before t1 (a prefix, unit_off does not
            // decrease); also the barrier for the LDS writes above
            K = __syncthreads_count(mu < t1);
            staged = !s_over;
        } else {
            m0 = block_find_msg(unit_off, N, t0, 0);
        }
#pragma unroll
        for (int k = 0; k < UPL; k++) {
            const int64_t u = t0 + (int64_t)k * S_BLOCK + tid;
            if (u >= t1) break;
            // the unit's message (index mi), its place j in it, and its bytes
            int64_t mi, j, b, n, o;
            int fl;
            uint32_t w[4];
            if (staged) {
                int lo = 0, hi = K;  // largest r < K with s_u[r] <= u
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_u[mid] <= u) lo = mid;
                    else hi = mid;
                }
                mi = m0 + lo;
                j = u - s_u[lo];
                b = s_b[lo];
                n = s_b[lo + 1] - b;
                o = s_o[lo];
                fl = s_f[lo];
                lds_read16(lds, (uint32_t)((uintptr_t)src + (uintptr_t)(b + UB * j) - (c0 << 4)), w);
            } else {  // rare: tiles past the table or starting over S_META messages
                mi = lane_search_msg(unit_off, N, u, m0);
                j = u - unit_off[mi];
                b = in_off[mi];
                n = in_off[mi + 1] - b;
                o = out_off[mi];
                fl = flags ? flags[mi] : 0;
                load_upto16(src + b + UB * j, (int)min(n - UB * j, (int64_t)UB), w);
            }
            if (ENC) {
                const uint8_t *tab = tabs + 64 * (fl & M_URL);
                uint8_t *q = dst + o + 16 * j;
                if (12 * j + 12 <= n) {
                    uint32_t oc[4];
                    enc_unit(w[0], w[1], w[2], tab, oc[0], oc[1], oc[2], oc[3]);
                    store_words<4, true>(q, oc);
                } else {
                    const int r = (int)(n - 12 * j);
                    keep_bytes(w, r);
                    enc_tail_fast(w, r, q, tab, fl & M_NOPAD);
                }
            } else {
                const uint8_t *tab = tabs + 256 * (fl & M_URL);
                uint8_t *q = dst + o + 12 * j;
                if (16 * j + 16 < n) {
                    uint32_t oc[3];
                    const uint32_t bad = dec_unit(w[0], w[1], w[2], w[3], tab, oc[0], oc[1], oc[2]);
                    store_words<3, true>(q, oc);
                    if (bad & INVALID)
                        msg_error(out_len, err_off, mi, 16 * j + dec_first_bad(w[0], w[1], w[2], w[3], tab));
                } else {
                    const int res = dec_tail_fast(w, (int)(n - 16 * j), n, q, tab, fl);
                    if (res >= 0) msg_error(out_len, err_off, mi, 16 * j + res);
                    else msg_length(out_len, mi, 12 * j + (-1 - res));
                }
            }
        }
    }
}

// Output size of message i for b64_batch_out_offsets: encoded length, or the
// decode slot (capacity rounded up to a multiple of 4).
__device__ __forceinline__ int64_t out_size_of(int dir, Msgs msgs, const uint8_t *flags, int64_t i)
{
    const int64_t len = msgs.n(i);
    const int nopad = flags ? (flags[i] & M_NOPAD) : 0;
    return dir == B64_DIR_ENCODE ? 4 * ((len + 2) / 3) : dec_slot_of(len, nopad);
}

// The output-offset scan runs in place in out_off, with no other memory:
// chunk c (PLAN_CHUNK messages) first stores its total at the index where the
// next chunk starts (or at N), a one-block pass turns those entries into
// their inclusive prefix (which is already the final out_off there), and
// every chunk then fills the rest of its range from the entry at its start.
__device__ __forceinline__ int64_t chunk_end(int64_t c, int64_t N)
{
    return std::min<int64_t>((c + 1) * PLAN_CHUNK, N);
}

// out_off[chunk_end(c)] = total output size of chunk c.
__global__ __launch_bounds__(PLAN_BLOCK) void k_out_reduce(int dir, Msgs msgs, int64_t N,
                                                          const uint8_t *__restrict__ flags,
                                                          int64_t *__restrict__ out_off)
{
    const int64_t i0 = (int64_t)blockIdx.x * PLAN_CHUNK + threadIdx.x * PLAN_PER_THREAD;
    int64_t s = 0;
    for (int k = 0; k < PLAN_PER_THREAD; k++)
        if (i0 + k < N) s += out_size_of(dir, msgs, flags, i0 + k);
    s = block_sum(s);
    if (threadIdx.x == 0) out_off[chunk_end(blockIdx.x, N)] = s;
}

// One block: inclusive scan of the chunk totals, in place.
__global__ __launch_bounds__(1024) void k_out_top(int64_t N, int64_t chunks, int64_t *__restrict__ out_off)
{
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < chunks; base += blockDim.x) {
        const int64_t c = base + threadIdx.x;
        const int64_t v = c < chunks ? out_off[chunk_end(c, N)] : 0;
        const int64_t ex = block_exclusive_scan(v);
        const int64_t carry = s_carry;
        if (c < chunks) out_off[chunk_end(c, N)] = carry + ex + v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_carry = carry + ex + v;
        __syncthreads();
    }
    if (N == 0 && threadIdx.x == 0) out_off[0] = 0;
}

// out_off[i] for the messages of chunk c, from the final entry at the chunk's
// start (0 for the first chunk); the entry at the chunk's end is already final.
__global__ __launch_bounds__(PLAN_BLOCK) void k_out_scan(int dir, Msgs msgs, int64_t N,
                                                        const uint8_t *__restrict__ flags,
                                                        int64_t *__restrict__ out_off)
{
    const int64_t c0 = (int64_t)blockIdx.x * PLAN_CHUNK;
    const int64_t pre = blockIdx.x == 0 ? 0 : out_off[c0];
    const int64_t i0 = c0 + threadIdx.x * PLAN_PER_THREAD;
    int64_t v[PLAN_PER_THREAD];
    int64_t s = 0;
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        v[k] = i0 + k < N ? out_size_of(dir, msgs, flags, i0 + k) : 0;
        s += v[k];
    }
    int64_t ex = pre + block_exclusive_scan(s);
    for (int k = 0; k < PLAN_PER_THREAD; k++) {
        const int64_t i = i0 + k;
        if (i < N && (i != c0 || blockIdx.x == 0)) out_off[i] = ex;
        ex += v[k];
    }
}

// ================================================================= host ==
// Planning workspace of a batch of N messages: unit_off (N + 1 entries), one
// partial sum per chunk of PLAN_CHUNK messages, and the staged layout's tile
// table (A: W + 1 entries, m: W entries, W = N + 4096).
constexpr int64_t plan_chunks(int64_t N) { return N > 0 ? (N + PLAN_CHUNK - 1) / PLAN_CHUNK : 1; }
constexpr int64_t tile_cap_h(int64_t N) { return N + 4096; }
constexpr int64_t batch_ws_bytes(int64_t N)
{
    return 8 * (N + 1) + 8 * plan_chunks(N) + 8 * (2 * tile_cap_h(N) + 1);
}

extern "C" {

int64_t b64_batch_workspace_bytes(int64_t N)
{
    if (N < 0) return b64i_fail(B64_BAD_ARG, "negative N");
    return batch_ws_bytes(N);
}

int b64_batch_out_offsets(int dir, const int64_t *in_off, int64_t N, int64_t *out_off,
                          const uint8_t *flags, void *stream)
{
    if (dir != B64_DIR_ENCODE && dir != B64_DIR_DECODE) return b64i_fail(B64_BAD_ARG, "bad direction");
    if (N < 0 || !in_off || !out_off) return b64i_fail(B64_BAD_ARG, "bad offsets arguments");
    hipStream_t s = (hipStream_t)stream;
    const Msgs msgs{in_off, nullptr};
    const int64_t chunks = std::max<int64_t>(1, (N + PLAN_CHUNK - 1) / PLAN_CHUNK);
    if (chunks > (int64_t)1 << 31) return b64i_fail(B64_BAD_ARG, "too many messages");
    hipLaunchKernelGGL(k_out_reduce, (unsigned)chunks, PLAN_BLOCK, 0, s, dir, msgs, N, flags, out_off);
    LAUNCH_TRY();
    hipLaunchKernelGGL(k_out_top, 1, 1024, 0, s, N, chunks, out_off);
    LAUNCH_TRY();
    hipLaunchKernelGGL(k_out_scan, (unsigned)chunks, PLAN_BLOCK, 0, s, dir, msgs, N, flags, out_off);
    LAUNCH_TRY();
    return B64_OK;
}

int b64_batch_slots(int dir, const int64_t *h_len, const uint8_t *h_flags, int64_t N, int64_t *h_need,
                    int64_t *h_out_off)
{
    if (dir != B64_DIR_ENCODE && dir != B64_DIR_DECODE) return b64i_fail(B64_BAD_ARG, "bad direction");
    if (N < 0 || (N > 0 && !h_len)) return b64i_fail(B64_BAD_ARG, "bad lengths");
    int64_t acc = 0;
    for (int64_t i = 0; i < N; i++) {
        const int64_t len = h_len[i];
        if (len < 0) return b64i_fail(B64_BAD_ARG, "negative length of message %lld", (long long)i);
        const int nopad = h_flags ? (h_flags[i] & M_NOPAD) : 0;
        if (h_need) h_need[i] = dir == B64_DIR_ENCODE ? enc_len_of(len, nopad) : dec_cap_of(len, nopad);
        if (h_out_off) h_out_off[i] = acc;
        acc += dir == B64_DIR_ENCODE ? 4 * ((len + 2) / 3) : dec_slot_of(len, nopad);
    }
    if (h_out_off) h_out_off[N] = acc;
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
    int rc = b64i_device_cus(&cus);
    if (rc) return rc;
    *layout = t ? t->layout : 0;
    const bool tiles = *layout == 0;
    *block = (t && t->block) ? t->block : (tiles ? 512 : 256);
    *upl = (t && t->units_per_lane) ? t->units_per_lane : 2;
    *grid = (t && t->grid) ? t->grid : cus * (*layout == 1 ? 8 : 32);
    if (*layout < 0 || *layout > 2) return b64i_fail(B64_BAD_ARG, "bad layout %d", *layout);
    if (*layout == 2 && *block != S_BLOCK)
        return b64i_fail(B64_BAD_ARG, "the staged layout runs %d-thread workgroups (block %d)", S_BLOCK, *block);
    if (*block < 64 || *block > 1024 || (*block & 63)) return b64i_fail(B64_BAD_ARG, "bad block size %d", *block);
    if (*upl != 1 && *upl != 2 && *upl != 4 && *upl != 8) return b64i_fail(B64_BAD_ARG, "bad units_per_lane %d", *upl);
    if (*grid < 1 || *grid > (1 << 20)) return b64i_fail(B64_BAD_ARG, "bad grid %d", *grid);
    return B64_OK;
}

// Device planning pass; fills the staged layout's tile table when the
// launch shape asks for that layout on a packed batch (tt->T > 0 then).
template <int DIR>
int plan(Msgs msgs, int64_t N, const uint8_t *flags, void *ws, int64_t ws_bytes, int64_t *out_len,
         int64_t *err_off, int64_t **unit_off, const b64_tune *tune, TileTab *tt, hipStream_t s)
{
    if (ws_bytes < b64_batch_workspace_bytes(N) || !ws) return b64i_fail(B64_BAD_ARG, "workspace too small");
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    const int64_t chunks = plan_chunks(N);
    *unit_off = (int64_t *)ws;
    int64_t *partial = (int64_t *)ws + (N + 1);
    *tt = TileTab{0, 0, nullptr, nullptr};
    if (layout == 2 && msgs.len == nullptr) {
        tt->T = (int64_t)S_BLOCK * upl;
        tt->W = tile_cap_h(N);
        tt->A = partial + chunks;
        tt->m = tt->A + tt->W + 1;
    }
    hipLaunchKernelGGL((k_plan_reduce<DIR>), (unsigned)chunks, PLAN_BLOCK, 0, s, msgs, N, partial);
    LAUNCH_TRY();
    const int scanned = chunks > PLAN_DIRECT_CHUNKS;
    if (scanned) {
        hipLaunchKernelGGL(k_plan_top, 1, 1024, 0, s, chunks, partial);
        LAUNCH_TRY();
    }
    hipLaunchKernelGGL((k_plan_scan<DIR>), (unsigned)chunks, PLAN_BLOCK, 0, s, msgs, N, flags, partial,
                       *unit_off, out_len, err_off, *tt, scanned);
    LAUNCH_TRY();
    return B64_OK;
}

#define B64_LAUNCH_STAGED(DIRV, UPL, ...)                                                        \
    switch (UPL) {                                                                               \
    case 1: hipLaunchKernelGGL((k_batch_s<DIRV, 1>), grid, S_BLOCK, 0, s, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL((k_batch_s<DIRV, 4>), grid, S_BLOCK, 0, s, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL((k_batch_s<DIRV, 8>), grid, S_BLOCK, 0, s, __VA_ARGS__); break;   \
    default: hipLaunchKernelGGL((k_batch_s<DIRV, 2>), grid, S_BLOCK, 0, s, __VA_ARGS__); break;  \
    }

#define B64_LAUNCH_UPL(KERN, UPL, ...)                                                   \
    switch (UPL) {                                                                       \
    case 1: hipLaunchKernelGGL((KERN<1>), grid, block, 0, s, __VA_ARGS__); break;        \
    case 4: hipLaunchKernelGGL((KERN<4>), grid, block, 0, s, __VA_ARGS__); break;        \
    case 8: hipLaunchKernelGGL((KERN<8>), grid, block, 0, s, __VA_ARGS__); break;        \
    default: hipLaunchKernelGGL((KERN<2>), grid, block, 0, s, __VA_ARGS__); break;       \
    }

int launch_enc_batch(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, const int64_t *unit_off, const b64_tune *tune, const TileTab &tt,
                     hipStream_t s)
{
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    if (layout == 2 && tt.T == 0) {  // no tile table (gather form): per-wave ranges instead
        layout = 1;
        upl = std::min(upl, 4);
    }
    if (layout == 2) {
        B64_LAUNCH_STAGED(B64_DIR_ENCODE, upl, src, msgs.begin, N, dst, out_off, flags, unit_off, tt.A, tt.m,
                          tt.W, nullptr, nullptr);
    } else if (layout == 1) {
        B64_LAUNCH_UPL(k_enc_batch_w, upl, src, msgs, N, dst, out_off, flags, unit_off);
    } else {
        B64_LAUNCH_UPL(k_enc_batch_t, upl, src, msgs, N, dst, out_off, flags, unit_off);
    }
    LAUNCH_TRY();
    return B64_OK;
}

int launch_dec_batch(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                     const b64_tune *tune, const TileTab &tt, hipStream_t s)
{
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    if (layout == 2 && tt.T == 0) {  // no tile table (gather form): per-wave ranges instead
        layout = 1;
        upl = std::min(upl, 4);
    }
    if (layout == 2) {
        B64_LAUNCH_STAGED(B64_DIR_DECODE, upl, src, msgs.begin, N, dst, out_off, flags, unit_off, tt.A, tt.m,
                          tt.W, out_len, err_off);
    } else if (layout == 1) {
        B64_LAUNCH_UPL(k_dec_batch_w, upl, src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off);
    } else {
        B64_LAUNCH_UPL(k_dec_batch_t, upl, src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off);
    }
    LAUNCH_TRY();
    return B64_OK;
}

int encode_batch_any(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, int64_t *out_len, void *ws, int64_t ws_bytes,
                     const b64_tune *tune, hipStream_t s)
{
    if (N < 0) return b64i_fail(B64_BAD_ARG, "negative N");
    if (N == 0) return B64_OK;
    if (!src || !msgs.begin || !dst || !out_off || !out_len) return b64i_fail(B64_BAD_ARG, "null argument");
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    int64_t *unit_off;
    TileTab tt;
    rc = plan<B64_DIR_ENCODE>(msgs, N, flags, ws, ws_bytes, out_len, nullptr, &unit_off, tune, &tt, s);
    if (rc) return rc;
    return launch_enc_batch(src, msgs, N, dst, out_off, flags, unit_off, tune, tt, s);
}

int decode_batch_any(const uint8_t *src, Msgs msgs, int64_t N, uint8_t *dst, const int64_t *out_off,
                     const uint8_t *flags, int64_t *out_len, int64_t *err_off, void *ws,
                     int64_t ws_bytes, const b64_tune *tune, hipStream_t s)
{
    if (N < 0) return b64i_fail(B64_BAD_ARG, "negative N");
    if (N == 0) return B64_OK;
    if (!src || !msgs.begin || !dst || !out_off || !out_len || !err_off) return b64i_fail(B64_BAD_ARG, "null argument");
    int block, upl, grid, layout;
    int rc = batch_shape(tune, &block, &upl, &grid, &layout);
    if (rc) return rc;
    int64_t *unit_off;
    TileTab tt;
    rc = plan<B64_DIR_DECODE>(msgs, N, flags, ws, ws_bytes, out_len, err_off, &unit_off, tune, &tt, s);
    if (rc) return rc;
    return launch_dec_batch(src, msgs, N, dst, out_off, flags, unit_off, out_len, err_off, tune, tt, s);
}

}  // namespace

// Planned batch launches for the serving runtime: the caller supplies the
// unit prefix (and, for decode, out_len = 0 / err_off = -1) computed on
// the host and uploaded together with the descriptors, so a serving batch is
// one upload and one codec kernel, which leaves the decode verdicts in place.
int b64i_encode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, const b64_tune *tune, hipStream_t s)
{
    if (N <= 0) return B64_OK;
    return launch_enc_batch(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, unit_off, tune, TileTab{}, s);
}

int b64i_decode_planned(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                        uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                        const int64_t *unit_off, int64_t *out_len, int64_t *err_off,
                        const b64_tune *tune, hipStream_t s)
{
    if (N <= 0) return B64_OK;
    return launch_dec_batch(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, unit_off, out_len,
                            err_off, tune, TileTab{}, s);
}

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

}  // extern "C"

// Device scratch of b64_decode_batch_noalloc: the planning workspace of up to
// B64_NOALLOC_MAX_MESSAGES messages. Every device the library runs on holds
// its own copy until the process ends. In host code `scratch` names a host
// stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, once per device.
constexpr int64_t SCRATCH_BYTES = (batch_ws_bytes(B64_NOALLOC_MAX_MESSAGES) + 255) / 256 * 256;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device: device address of `scratch`

int scratch_address(void **out)
{
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return b64i_fail(B64_HIP_ERROR, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return B64_OK;
}

}  // namespace

extern "C" {

int b64_decode_batch_noalloc(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                             const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                             int64_t *err_off, const b64_tune *tune, void *stream)
{
    if (N < 0) return b64i_fail(B64_BAD_ARG, "negative N");
    if (N > B64_NOALLOC_MAX_MESSAGES)
        return b64i_fail(B64_BAD_ARG, "b64_decode_batch_noalloc takes at most %d messages (got %lld)",
                         B64_NOALLOC_MAX_MESSAGES, (long long)N);
    if (N == 0) return B64_OK;
    void *ws;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return decode_batch_any(src, Msgs{in_off, nullptr}, N, dst, out_off, flags, out_len, err_off, ws,
                            SCRATCH_BYTES, tune, (hipStream_t)stream);
}

int b64_encode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, void *workspace, int64_t workspace_bytes,
                            const b64_tune *tune, void *stream)
{
    if (N > 0 && !in_len) return b64i_fail(B64_BAD_ARG, "null in_len");
    return encode_batch_any(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, out_len, workspace,
                            workspace_bytes, tune, (hipStream_t)stream);
}

int b64_decode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, int64_t *err_off, void *workspace,
                            int64_t workspace_bytes, const b64_tune *tune, void *stream)
{
    if (N > 0 && !in_len) return b64i_fail(B64_BAD_ARG, "null in_len");
    return decode_batch_any(src, Msgs{in_begin, in_len}, N, dst, out_off, flags, out_len, err_off,
                            workspace, workspace_bytes, tune, (hipStream_t)stream);
}

int b64_encode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len, void *stream)
{
    if (N < 0 || !h_in_off || !h_out_off) return b64i_fail(B64_BAD_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> lens(N);
    for (int64_t i = 0; i < N; i++) {
        const int64_t n = h_in_off[i + 1] - h_in_off[i];
        const int fl = h_flags ? h_flags[i] : 0;
        const int mode = (fl & M_URL) | (fl & M_NOPAD);
        lens[i] = b64i_enc_len(n, mode);
        if (n > 0) {
            int rc = b64i_enqueue_encode(src + h_in_off[i], n, dst + h_out_off[i], mode, s);
            if (rc) return rc;
        }
    }
    if (out_len && N) HIP_TRY(hipMemcpyAsync(out_len, lens.data(), 8 * N, hipMemcpyHostToDevice, s));
    if (N) HIP_TRY(hipStreamSynchronize(s));  // lens is a local host buffer
    return B64_OK;
}

// Result slots of the per-message decodes: (0, -1), the verdict of an empty
// message and the state each single-buffer decode forms its verdict from.
__global__ void k_each_init(int64_t N, int64_t *__restrict__ d_len, int64_t *__restrict__ d_err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        d_len[i] = 0;
        d_err[i] = -1;
    }
}

int b64_decode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len,
                    int64_t *err_off, void *stream)
{
    if (N < 0 || !h_in_off || !h_out_off || !out_len || !err_off) return b64i_fail(B64_BAD_ARG, "bad arguments");
    if (N == 0) return B64_OK;
    hipStream_t s = (hipStream_t)stream;
    const int fb = (int)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_each_init, fb, 256, 0, s, N, out_len, err_off);
    LAUNCH_TRY();
    for (int64_t i = 0; i < N; i++) {
        const int64_t n = h_in_off[i + 1] - h_in_off[i];
        const int fl = h_flags ? h_flags[i] : 0;
        if (n == 0) continue;  // verdict (0, -1) comes from the init pass
        int rc = b64i_enqueue_decode(src + h_in_off[i], n, dst + h_out_off[i], fl & 7,
                                (unsigned long long *)(err_off + i), out_len + i, s);
        if (rc) return rc;
    }
    return B64_OK;
}

}  // extern "C"
