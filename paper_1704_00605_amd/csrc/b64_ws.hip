// gfx950 whitespace-tolerant decode (Appendix B: space, line feed and
// carriage return are removed before decoding) fused into one pass, and its
// C-ABI (include/b64.h).
//
//   k_ws_init       clears the tile counter, the error slots and the tile
//                   status words.
//   k_dec_ws        one tile of the input per workgroup, tiles taken in order
//                   from an atomic counter:
//                     1. load dwords, classify every byte through one LDS
//                        table (symbol value, '=', whitespace, invalid);
//                     2. kept-byte prefix counts: per wave from ballots of the
//                        four byte positions and mbcnt, per workgroup from the
//                        wave totals;
//                     3. compact the kept class bytes into LDS;
//                     4. decoupled look-back: publish the tile's kept count
//                        and last three kept class bytes, walk back over the
//                        status words of earlier tiles to get the stripped
//                        offset P of the tile's first kept byte and the kept
//                        bytes just before it;
//                     5. decode every quad of the stripped text that ends in
//                        this tile (quads straddling tiles are completed from
//                        the carried bytes) and write its bytes at 3 * quad.
//   k_dec_ws_final  verdict from the last tile's status and the error slots.
//
// Errors are reported in the coordinates of the original input: a tile
// checks its own bytes, so it knows their original indexes. A byte outside
// the alphabet is an error wherever it is; '=' is valid only as the last one
// or two kept bytes of a stripped text whose length is a multiple of 4, which
// only the final verdict can tell; since stripping keeps order, the first '='
// in stripped order is the first in original order, so two atomicMin slots
// (original and stripped index) describe it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "b64.h"
#include "b64_device.hpp"
#include "b64_internal.hpp"

using namespace b64dev;

namespace {

// ------------------------------------------------------------- classes --
// Class byte of an input byte: its 6-bit value for a symbol of the alphabet
// (Table 1 or base64url), or one of the marks below (bit 7 set).
constexpr uint8_t C_BAD = 0x80;   // not in the alphabet, not whitespace, not '='
constexpr uint8_t C_PAD = 0xA0;   // '='
constexpr uint8_t C_WS = 0xC0;    // space, line feed, carriage return (removed)

struct WsTables {
    uint8_t cls[2][256];
};

constexpr WsTables make_ws_tables()
{
    WsTables w{};
    const Tables t = make_tables();
    for (int a = 0; a < 2; a++) {
        for (int c = 0; c < 256; c++) w.cls[a][c] = (t.dec[a][c] & INVALID) ? C_BAD : t.dec[a][c];
        w.cls[a]['='] = C_PAD;
        w.cls[a][' '] = C_WS;
        w.cls[a]['\n'] = C_WS;
        w.cls[a]['\r'] = C_WS;
    }
    return w;
}

}  // namespace

static __constant__ WsTables c_ws = make_ws_tables();

// --------------------------------------------------------- tile status --
// One 64-bit word per tile: flag (2 bits: 0 not ready, 1 aggregate of this
// tile alone, 2 inclusive prefix over tiles 0..t), kept count (38 bits) and
// the last three kept class bytes (24 bits, the most recent in the low
// byte; fewer when the count is below 3). Counts are below 2^38.
constexpr unsigned long long ST_AGG = 1ull << 62;
constexpr unsigned long long ST_INC = 2ull << 62;
constexpr int64_t WS_MAX_N = (1ll << 38) - 1;

__device__ __forceinline__ unsigned long long st_make(unsigned long long flag, uint64_t cnt, uint32_t car)
{
    return flag | (cnt << 24) | (car & 0xffffffu);
}
__device__ __forceinline__ uint64_t st_cnt(unsigned long long s) { return (s >> 24) & ((1ull << 38) - 1); }
__device__ __forceinline__ uint32_t st_car(unsigned long long s) { return (uint32_t)(s & 0xffffffu); }

// Last three kept bytes of "a then b" where b holds nb kept bytes.
__device__ __forceinline__ uint32_t car_join(uint32_t a, uint32_t b, uint64_t nb)
{
    return nb >= 3 ? b : (((a << (8 * nb)) | b) & 0xffffffu);
}

// Slots of the workspace (64-bit words): [0] tile counter, [1] first invalid
// byte (original index), [2] first '=' (original index), [3] first '='
// (stripped index); the tile status words start at word 8.
constexpr int WS_SLOT_WORDS = 8;

__global__ void k_ws_init(unsigned long long *__restrict__ ws, int64_t T)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        ws[0] = 0;
        ws[1] = ERR_NONE;
        ws[2] = ERR_NONE;
        ws[3] = ERR_NONE;
    }
    unsigned long long *st = ws + WS_SLOT_WORDS;
    for (int64_t i = i0; i < T; i += (int64_t)gridDim.x * blockDim.x) st[i] = 0;
}

__device__ __forceinline__ uint32_t load4(const uint8_t *p)
{
    const uintptr_t a = (uintptr_t)p;
    const uint32_t *d = (const uint32_t *)(a & ~(uintptr_t)3);
    const uint32_t s = (uint32_t)(a & 3);
    return s ? alignb(d[1], d[0], s) : d[0];
}

// Quad of class bytes (first byte lowest) -> 24-bit group a<<18|b<<12|c<<6|d.
__device__ __forceinline__ uint32_t quad_bits(uint32_t v)
{
    return ((v & 0x3f) << 18) | (((v >> 8) & 0x3f) << 12) | (((v >> 16) & 0x3f) << 6) | ((v >> 24) & 0x3f);
}

template <int BLOCK, int CPL, bool ALIGNED>
__global__ __launch_bounds__(BLOCK) void k_dec_ws(const uint8_t *__restrict__ src, int64_t n,
                                                  uint8_t *__restrict__ dst, int alpha,
                                                  unsigned long long *__restrict__ ws)
{
    constexpr int TILE = BLOCK * 4 * CPL;  // input bytes per tile
    constexpr int NW = BLOCK / 64;
    constexpr int E = CPL * NW;            // (k, wave) segments, at most 128
    static_assert(E <= 128, "segment scan covers at most 128 entries");
    __shared__ uint32_t s_tab[64];
    __shared__ __attribute__((aligned(16))) uint8_t s_cls[16 + TILE + 16];
    __shared__ uint32_t s_seg[E];          // kept bytes per segment, then their exclusive prefix
    __shared__ uint32_t s_tot;
    __shared__ unsigned long long s_t, s_P;

    const int tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
    lds_fill(s_tab, c_ws.cls[alpha], 256);
    if (tid == 0) s_t = atomicAdd(&ws[0], 1ull);
    __syncthreads();
    const int64_t t = (int64_t)s_t;
    const int64_t base = t * TILE;
    const uint8_t *tab = (const uint8_t *)s_tab;
    unsigned long long *status = ws + WS_SLOT_WORDS;

    // 1. load and classify; lane tid holds dwords k * BLOCK + tid (k < CPL)
    uint32_t cls[CPL], keep[CPL], pre[CPL];
    uint32_t spec = 0;
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        const int64_t off = base + 4 * ((int64_t)k * BLOCK + tid);
        uint32_t w;
        if (off + 4 <= n) {
            w = ALIGNED ? *(const uint32_t *)(src + off) : load4(src + off);
        } else {
            w = 0x20202020u;  // past the end: whitespace, removed
            for (int j = 0; j < 4; j++)
                if (off + j < n) w = (w & ~(0xffu << (8 * j))) | ((uint32_t)src[off + j] << (8 * j));
        }
        const uint32_t c = tab[w & 0xff] | ((uint32_t)tab[(w >> 8) & 0xff] << 8) |
                           ((uint32_t)tab[(w >> 16) & 0xff] << 16) | ((uint32_t)tab[w >> 24] << 24);
        cls[k] = c;
        const uint32_t x = (~c & 0x40404040u) >> 6;  // bit 8j: byte j kept
        keep[k] = (x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xf;
        spec |= c & ~(c << 1) & 0x80808080u;      // bit 7 set, bit 6 clear: invalid or '='
    }

    // 2. prefix counts of kept bytes in memory order (k, wave, lane, byte)
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        uint32_t p = 0, tot = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const unsigned long long bb = __ballot((keep[k] >> b) & 1);
            p += __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
            tot += (uint32_t)__popcll(bb);
        }
        pre[k] = p;
        if (lane == 0) s_seg[k * NW + wid] = tot;
    }
    __syncthreads();
    if (wid == 0) {
        const uint32_t a0 = 2 * lane < E ? s_seg[2 * lane] : 0u;
        const uint32_t a1 = 2 * lane + 1 < E ? s_seg[2 * lane + 1] : 0u;
        const uint32_t own = a0 + a1;
        uint32_t inc = own;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        const uint32_t ex = inc - own;
        if (2 * lane < E) s_seg[2 * lane] = ex;
        if (2 * lane + 1 < E) s_seg[2 * lane + 1] = ex + a0;
        if (lane == 63) s_tot = inc;
    }
    __syncthreads();

    // 3. compaction: kept class bytes to s_cls[16 + tile-stripped index]
    uint32_t at[CPL];
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        at[k] = s_seg[k * NW + wid] + pre[k];
        uint32_t pos = 16 + at[k];
#pragma unroll
        for (int j = 0; j < 4; j++)
            if ((keep[k] >> j) & 1) s_cls[pos++] = (uint8_t)(cls[k] >> (8 * j));
    }
    __syncthreads();
    const uint32_t ktot = s_tot;

    // 4. decoupled look-back (one lane)
    if (tid == 0) {
        uint32_t car = 0;
        for (uint32_t i = ktot > 3 ? ktot - 3 : 0; i < ktot; i++) car = (car << 8) | s_cls[16 + i];
        uint64_t P = 0;
        uint32_t before = 0;
        if (t == 0) {
            __hip_atomic_store(&status[0], st_make(ST_INC, ktot, car), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[t], st_make(ST_AGG, ktot, car), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // every earlier tile took its index before this one and publishes
            // its aggregate without waiting, so each wait below ends
            for (int64_t j = t - 1;; j--) {
                unsigned long long s;
                while (((s = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 62) == 0)
                    __builtin_amdgcn_s_sleep(1);
                before = car_join(st_car(s), before, P);
                P += st_cnt(s);
                if ((s >> 62) == 2) break;
            }
            __hip_atomic_store(&status[t], st_make(ST_INC, P + ktot, car_join(before, car, ktot)),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // carried bytes of the quad that straddles into this tile
        const int r0 = (int)(P & 3);
        for (int i = 0; i < r0; i++) s_cls[16 - r0 + i] = (uint8_t)(before >> (8 * (r0 - 1 - i)));
        s_P = P;
    }
    __syncthreads();
    const int64_t P = (int64_t)s_P;

    // rare path: invalid bytes and '=' of this tile, in original coordinates
    if (__ballot(spec != 0)) {
#pragma unroll
        for (int k = 0; k < CPL; k++) {
            const int64_t off = base + 4 * ((int64_t)k * BLOCK + tid);
            uint32_t rank = 0;
            for (int j = 0; j < 4; j++) {
                const uint32_t cb = (cls[k] >> (8 * j)) & 0xff;
                if (cb == C_BAD) atomicMin(&ws[1], (unsigned long long)(off + j));
                if (cb == C_PAD) {
                    atomicMin(&ws[2], (unsigned long long)(off + j));
                    atomicMin(&ws[3], (unsigned long long)(P + at[k] + rank));
                }
                rank += (keep[k] >> j) & 1;
            }
        }
    }

    // 5. decode the quads that end in this tile: stripped bytes
    // [P - r0, P + ktot) sit at s_cls[16 - r0 ...]
    const int r0 = (int)(P & 3);
    const int Q = (r0 + (int)ktot) >> 2;
    const int U = (Q + 3) >> 2;
    uint8_t *q0 = dst + 3 * ((P - r0) >> 2);
    for (int u = tid; u < U; u += BLOCK) {
        uint32_t v0, v1, v2, v3;
        if (r0 == 0) {
            const uint4 x = *(const uint4 *)(s_cls + 16 + 16 * u);
            v0 = x.x; v1 = x.y; v2 = x.z; v3 = x.w;
        } else {
            const uint32_t *d = (const uint32_t *)(s_cls + 12 + 16 * u);
            const uint32_t d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
            const uint32_t sh = 4 - r0;
            v0 = alignb(d1, d0, sh); v1 = alignb(d2, d1, sh); v2 = alignb(d3, d2, sh); v3 = alignb(d4, d3, sh);
        }
        const int nq = min(4, Q - 4 * u);
        uint8_t *q = q0 + 12 * (int64_t)u;
        if (nq == 4 && !((v0 | v1 | v2 | v3) & 0x80808080u)) {
            const uint32_t t0 = quad_bits(v0), t1 = quad_bits(v1), t2 = quad_bits(v2), t3 = quad_bits(v3);
            const uint32_t o[3] = {perm(t1, t0, 0x06000102u), perm(t2, t1, 0x05060001u), perm(t3, t2, 0x04050600u)};
            store_words<3, true>(q, o);
        } else {
            // a partial unit, or marks: '=' counts as 0 and the bytes it pads
            // are not written (any other placement is an error, and the
            // output of an invalid input is unspecified)
            const uint32_t vs[4] = {v0, v1, v2, v3};
            for (int i = 0; i < nq; i++) {
                const uint32_t v = vs[i];
                const uint32_t c2 = (v >> 16) & 0xff, c3 = v >> 24;
                const uint32_t tq = quad_bits(v & ~((v & 0x80808080u) >> 2) & ~(v & 0x80808080u));
                q[3 * i] = (uint8_t)(tq >> 16);
                if (!(c2 == C_PAD && c3 == C_PAD)) q[3 * i + 1] = (uint8_t)(tq >> 8);
                if (c3 != C_PAD) q[3 * i + 2] = (uint8_t)tq;
            }
        }
    }
}

// Verdict: (decoded length, -1) or (-1, first offending original index).
__global__ void k_dec_ws_final(const unsigned long long *__restrict__ ws, int64_t T, int64_t n,
                               int64_t *__restrict__ d_len, int64_t *__restrict__ d_err)
{
    if (threadIdx.x || blockIdx.x) return;
    const unsigned long long s = ws[WS_SLOT_WORDS + T - 1];
    const int64_t m = (int64_t)st_cnt(s);
    const uint32_t last = st_car(s) & 0xff;
    const unsigned long long bad = ws[1], eq_o = ws[2], eq_s = ws[3];
    bool pad_ok = true;
    int64_t pads = 0;
    if (eq_s != ERR_NONE) {
        const int64_t e = (int64_t)eq_s;
        pad_ok = (m & 3) == 0 && (e == m - 1 || (e == m - 2 && last == C_PAD));
        pads = m - e;
    }
    unsigned long long err = bad;
    if (!pad_ok && eq_o < err) err = eq_o;
    if (err == ERR_NONE && (m & 3) != 0) err = (unsigned long long)n;
    if (err != ERR_NONE) {
        *d_len = -1;
        *d_err = (int64_t)err;
    } else {
        *d_len = 3 * (m / 4) - pads;
        *d_err = -1;
    }
}

// ================================================================= host ==
namespace {

// Smallest tile of any launch shape: sizes the workspace.
constexpr int64_t WS_MIN_TILE = 256 * 4 * 2;

struct WsShape {
    int block = 512;
    int cpl = 8;
};
WsShape g_ws;

int64_t ws_tiles(int64_t n, int tile) { return (n + tile - 1) / tile; }

template <bool A>
int launch_ws(int block, int cpl, int64_t T, const uint8_t *src, int64_t n, uint8_t *dst, int alpha,
              unsigned long long *ws, hipStream_t s)
{
    const dim3 g((unsigned)T);
#define B64_WS_CASE(B, C)                                                                      \
    if (block == B && cpl == C) {                                                              \
        hipLaunchKernelGGL((k_dec_ws<B, C, A>), g, B, 0, s, src, n, dst, alpha, ws);           \
        return B64_OK;                                                                         \
    }
    B64_WS_CASE(256, 2) B64_WS_CASE(256, 4) B64_WS_CASE(256, 8)
    B64_WS_CASE(512, 2) B64_WS_CASE(512, 4) B64_WS_CASE(512, 8)
    B64_WS_CASE(1024, 2) B64_WS_CASE(1024, 4) B64_WS_CASE(1024, 8)
#undef B64_WS_CASE
    return b64i_fail(B64_BAD_ARG, "unsupported whitespace-decode shape %d x %d", block, cpl);
}

// Enqueues init, tile kernel and verdict. n >= 1.
int enqueue_ws(const uint8_t *src, int64_t n, uint8_t *dst, int alpha, int64_t *d_len, int64_t *d_err,
               unsigned long long *ws, hipStream_t s)
{
    const int block = g_ws.block, cpl = g_ws.cpl;
    const int64_t T = ws_tiles(n, (int64_t)block * 4 * cpl);
    const int ib = (int)std::min<int64_t>((T + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(k_ws_init, ib, 256, 0, s, ws, T);
    LAUNCH_TRY();
    const bool al = (((uintptr_t)src) & 3) == 0;
    int rc = al ? launch_ws<true>(block, cpl, T, src, n, dst, alpha, ws, s)
                : launch_ws<false>(block, cpl, T, src, n, dst, alpha, ws, s);
    if (rc) return rc;
    LAUNCH_TRY();
    hipLaunchKernelGGL(k_dec_ws_final, 1, 64, 0, s, ws, T, n, d_len, d_err);
    LAUNCH_TRY();
    return B64_OK;
}

int ws_alpha(int alphabet, int *alpha)
{
    int mode;
    int rc = b64i_parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (mode & (B64I_M_STRICT | B64I_M_NOPAD))
        return b64i_fail(B64_BAD_ARG, "whitespace-tolerant decode takes the alphabet only (no mode bits)");
    *alpha = mode & B64I_M_URL;
    return B64_OK;
}

// Per-thread, per-device workspace of the synchronous call (grown on demand)
// plus its verdict slots (device) and their host copy (pinned).
struct WsCache {
    int dev = -1;
    unsigned long long *d = nullptr;
    int64_t bytes = 0;
    int64_t *verdict = nullptr;  // device [len, err]
    int64_t *h = nullptr;        // pinned host [len, err]
};
thread_local std::vector<WsCache> t_ws;

}  // namespace

extern "C" {

int64_t b64_decode_ws_workspace_bytes(int64_t n)
{
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    return 8 * (WS_SLOT_WORDS + std::max<int64_t>(ws_tiles(n, WS_MIN_TILE), 1));
}

int b64_decode_ws_async(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, int64_t *d_len,
                        int64_t *d_err, void *workspace, int64_t workspace_bytes, void *stream)
{
    int alpha;
    int rc = ws_alpha(alphabet, &alpha);
    if (rc) return rc;
    if (n < 0 || n > WS_MAX_N) return b64i_fail(B64_BAD_ARG, "length outside [0, 2^38)");
    if (!d_len || !d_err) return b64i_fail(B64_BAD_ARG, "null result slot");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        const int64_t v[2] = {0, -1};
        HIP_TRY(hipMemcpyAsync(d_len, &v[0], 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_err, &v[1], 8, hipMemcpyHostToDevice, s));
        return hipStreamSynchronize(s) == hipSuccess ? B64_OK : b64i_fail(B64_HIP_ERROR, "stream sync");
    }
    if (!src || (!dst && n >= 4)) return b64i_fail(B64_BAD_ARG, "null buffer with n > 0");
    if (!workspace || workspace_bytes < b64_decode_ws_workspace_bytes(n))
        return b64i_fail(B64_BAD_ARG, "workspace smaller than b64_decode_ws_workspace_bytes(n)");
    return enqueue_ws(src, n, dst, alpha, d_len, d_err, (unsigned long long *)workspace, s);
}

int64_t b64_decode_ws(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off, int alphabet,
                      void *stream)
{
    int alpha;
    int rc = ws_alpha(alphabet, &alpha);
    if (rc) return rc;
    if (!err_off) return b64i_fail(B64_BAD_ARG, "null err_off");
    if (n < 0 || n > WS_MAX_N) return b64i_fail(B64_BAD_ARG, "length outside [0, 2^38)");
    *err_off = -1;
    if (n == 0) return 0;
    if (!src || (!dst && n >= 4)) return b64i_fail(B64_BAD_ARG, "null buffer with n > 0");
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    WsCache *c = nullptr;
    for (auto &e : t_ws)
        if (e.dev == dev) c = &e;
    if (!c) {
        t_ws.emplace_back();
        c = &t_ws.back();
        c->dev = dev;
        HIP_TRY(hipMalloc((void **)&c->verdict, 16));
        HIP_TRY(hipHostMalloc((void **)&c->h, 16, hipHostMallocDefault));
    }
    const int64_t need = b64_decode_ws_workspace_bytes(n);
    hipStream_t s = (hipStream_t)stream;
    if (c->bytes < need) {
        HIP_TRY(hipStreamSynchronize(s));
        if (c->d) HIP_TRY(hipFree(c->d));
        c->d = nullptr;
        c->bytes = 0;
        HIP_TRY(hipMalloc((void **)&c->d, need));
        c->bytes = need;
    }
    rc = enqueue_ws(src, n, dst, alpha, c->verdict, c->verdict + 1, c->d, s);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->h, c->verdict, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->h[0] < 0) {
        *err_off = c->h[1];
        return b64i_fail(B64_INVALID_INPUT, "invalid base64 input at offset %lld", (long long)c->h[1]);
    }
    return c->h[0];
}

int b64_set_ws_tune(const b64_tune *t)
{
    if (!t) return b64i_fail(B64_BAD_ARG, "null tune");
    const int block = t->block ? t->block : g_ws.block;
    const int cpl = t->units_per_lane ? t->units_per_lane : g_ws.cpl;
    if ((block != 256 && block != 512 && block != 1024) || (cpl != 2 && cpl != 4 && cpl != 8))
        return b64i_fail(B64_BAD_ARG, "whitespace-decode shape: block 256/512/1024, dwords per lane 2/4/8");
    g_ws.block = block;
    g_ws.cpl = cpl;
    return B64_OK;
}

}  // extern "C"
