// gfx950 whitespace-tolerant decode (Appendix B: space, line feed and
// carriage return are removed before decoding), and its C-ABI
// (include/b64.h). The input is cut into tiles of blockDim * 16 * CPL bytes.
//
//   k_ws_count    per tile: number of kept (non-whitespace) bytes and the
//                 last three of them, from SWAR whitespace tests, and a flag
//                 for control bytes that are not whitespace; also resets the
//                 error slots.
//   k_ws_reduce   per group of 2048 tiles: the ordered combination of their
//                 (count, last three) states.
//   k_ws_prefix   per tile: the exclusive prefix state, i.e. the stripped
//                 offset P of the tile's first kept byte and the three kept
//                 bytes just before it (an ordered scan; the operator keeps
//                 counts and the last three bytes, so it is associative).
//   k_dec_ws      per tile: compact the kept bytes into LDS (DPP wave scan
//                 of per-dword counts), put the carried bytes of the quad
//                 that straddles into the tile in front, decode every quad of
//                 the stripped text that ends in this tile through one LDS
//                 class table (its bytes go to 3 * quad index), and, when a
//                 mark (invalid byte, '=') turns up, rescan the raw tile to
//                 report it in original coordinates.
//   k_dec_ws_final verdict from the total state and the error slots.
//
// Two passes read the input (count, then decode) and no tile waits for
// another. A byte outside the alphabet is an error wherever it is; '=' is
// valid only as the last one or two kept bytes of a stripped text whose
// length is a multiple of 4, which only the final verdict can tell; since
// stripping keeps order, the first '=' in stripped order is the first in
// original order, so two atomicMin slots (original and stripped index)
// describe it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

// ----------------------------------------------------------- tile states --
// State of a run of input: kept-byte count (38 bits) and its last three kept
// bytes (24 bits, the latest in the low byte; fewer when the count is below
// 3), packed in one 64-bit word. Counts stay below 2^38.
constexpr int64_t WS_MAX_N = (1ll << 38) - 1;

struct WsSt {
    uint64_t c;
    uint32_t r;
};

// Last three kept bytes of "a then b" where b holds nb kept bytes.
__device__ __forceinline__ uint32_t car_join(uint32_t a, uint32_t b, uint64_t nb)
{
    return nb >= 3 ? b : (((a << (8 * nb)) | b) & 0xffffffu);
}
// State of run a followed by run b.
__device__ __forceinline__ WsSt st_join(WsSt a, WsSt b) { return {a.c + b.c, car_join(a.r, b.r, b.c)}; }
__device__ __forceinline__ unsigned long long st_pack(WsSt s) { return (s.c << 24) | (s.r & 0xffffffu); }
__device__ __forceinline__ WsSt st_unpack(unsigned long long w)
{
    return {(w >> 24) & (uint64_t)WS_MAX_N, (uint32_t)(w & 0xffffffu)};
}
// Bit 63 of a tile's state word (not part of the state): the tile holds a
// byte at or below 0x20 that is not whitespace.
constexpr unsigned long long WS_CTRL_FLAG = 1ull << 63;

__device__ __forceinline__ WsSt shfl_up_st(WsSt s, int d)
{
    return {(uint64_t)__shfl_up((long long)s.c, d, 64), (uint32_t)__shfl_up((int)s.r, d, 64)};
}

// Ordered inclusive scan of one state per thread over the block (blockDim a
// multiple of 64, at most 1024); *total receives the block's state.
__device__ WsSt block_scan_st(WsSt v, WsSt *total)
{
    __shared__ unsigned long long s_w[16];
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const WsSt o = shfl_up_st(v, d);
        if (lane >= d) v = st_join(o, v);
    }
    if (lane == 63) s_w[wid] = st_pack(v);
    __syncthreads();
    WsSt pre{0, 0};
    for (int i = 0; i < wid; i++) pre = st_join(pre, st_unpack(s_w[i]));
    WsSt tot{0, 0};
    for (int i = 0; i < nw; i++) tot = st_join(tot, st_unpack(s_w[i]));
    __syncthreads();
    *total = tot;
    return st_join(pre, v);
}

// Workspace (64-bit words): [0..7] slots ([1] first invalid byte, original
// index; [2] first '=', original index; [3] first '=', stripped index), then
// tile states [T], tile prefixes [T], group states [G].
constexpr int WS_SLOT_WORDS = 8;
constexpr int WS_SCAN_BLOCK = 256;
constexpr int WS_SCAN_PER = 8;
constexpr int WS_GROUP = WS_SCAN_BLOCK * WS_SCAN_PER;  // tiles per scan group

// 16 bytes at src + off (off a multiple of 16 from the tile base); bytes
// past the end read as spaces (removed).
template <bool ALIGNED>
__device__ __forceinline__ void tile_load16(const uint8_t *__restrict__ src, int64_t n, int64_t off, uint32_t (&w)[4])
{
    if (off + 16 <= n) {
        if (ALIGNED) {
            const uint32_t *p = (const uint32_t *)(src + off);
            w[0] = __builtin_nontemporal_load(p);
            w[1] = __builtin_nontemporal_load(p + 1);
            w[2] = __builtin_nontemporal_load(p + 2);
            w[3] = __builtin_nontemporal_load(p + 3);
        } else {
            load16(src + off, w[0], w[1], w[2], w[3]);
        }
        return;
    }
#pragma unroll
    for (int d = 0; d < 4; d++) {
        uint32_t x = 0x20202020u;
        for (int j = 0; j < 4; j++) {
            const int64_t o = off + 4 * d + j;
            if (o < n) x = (x & ~(0xffu << (8 * j))) | ((uint32_t)src[o] << (8 * j));
        }
        w[d] = x;
    }
}

// Kept bytes of w: bit 8j+7 set when byte j is above 0x20. On a valid input
// every byte at or below 0x20 is space, LF or CR, so this removes exactly the
// whitespace. Other bytes at or below 0x20 are invalid: the count pass flags
// their tiles (ctrl_bad), and on an invalid input the verdict does not depend
// on the counts (see k_dec_ws_final).
__device__ __forceinline__ uint32_t kept8(uint32_t w)
{
    return (((w & 0x7f7f7f7fu) + 0x5f5f5f5fu) | w) & 0x80808080u;
}

// Bit 8j+7 set when byte j of w is at or below 0x20 and is not space (0x20),
// LF (0x0A) or CR (0x0D). The byte permute serves as a lookup keyed by the
// byte values themselves: selectors 13 and above give 0xff, 12 gives 0,
// 10 copies the sign of table byte 5 (set), and 0..9 and 11 give table bytes
// or signs whose bit 0 is clear; so bit 0 of the result is set exactly for
// 10 and for 13 and above. Values 14..31 are then excluded by a compare, and
// 32 is admitted by its bit 5.
__device__ __forceinline__ uint32_t ctrl_bad(uint32_t w)
{
    const uint32_t xm = w & 0x7f7f7f7fu;
    const uint32_t kept = ((xm + 0x5f5f5f5fu) | w) & 0x80808080u;
    const uint32_t ge14 = xm + 0x72727272u;  // bit 8j+7: (byte j & 0x7f) >= 14
    const uint32_t p = perm(0x00008000u, 0u, w);
    const uint32_t ok = (w << 2) | (~ge14 & (p << 7));
    return ~kept & ~ok & 0x80808080u;
}

// Tile = BLOCK * 16 * CPL bytes; lane tid reads the 16-byte chunks
// k * BLOCK + tid (k < CPL), so memory order is (k, wave, lane, byte).
template <int BLOCK, int CPL, bool ALIGNED>
__global__ __launch_bounds__(BLOCK) void k_ws_count(const uint8_t *__restrict__ src, int64_t n,
                                                    unsigned long long *__restrict__ ws)
{
    constexpr int TILE = BLOCK * 16 * CPL;
    constexpr int NW = BLOCK / 64;
    constexpr int E = CPL * NW;
    __shared__ uint32_t s_cnt[E], s_car[E];
    const int tid = threadIdx.x, lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
    const int64_t t = blockIdx.x;
    if (t == 0 && tid == 0) {
        ws[1] = ERR_NONE;
        ws[2] = ERR_NONE;
        ws[3] = ERR_NONE;
    }
    const int64_t base = t * TILE;
    uint32_t w[CPL][4], cnt[CPL];
#pragma unroll
    for (int k = 0; k < CPL; k++) tile_load16<ALIGNED>(src, n, base + 16 * ((int64_t)k * BLOCK + tid), w[k]);
    // per segment: kept bytes, and bit 31 when it holds a control byte that
    // is not whitespace
#pragma unroll
    for (int k = 0; k < CPL; k++) {
        cnt[k] = __popc(kept8(w[k][0])) + __popc(kept8(w[k][1])) + __popc(kept8(w[k][2])) +
                 __popc(kept8(w[k][3]));
        const uint32_t bad = ctrl_bad(w[k][0]) | ctrl_bad(w[k][1]) | ctrl_bad(w[k][2]) | ctrl_bad(w[k][3]);
        uint32_t tot = __ballot(bad != 0) ? 0x80000000u : 0u;
#pragma unroll
        for (int b = 0; b < 5; b++) tot += (uint32_t)__popcll(__ballot((cnt[k] >> b) & 1)) << b;
        if (lane == 0) s_cnt[k * NW + wid] = tot;
    }
    __syncthreads();
    // the tile's last three kept bytes lie in its last (at most three)
    // non-empty segments: only the waves holding those read them out of
    // their lanes (scalar work, from the segment's last non-empty lanes)
    int need = 3;
    for (int i = E - 1; i >= 0 && need > 0; i--) {
        const uint32_t cs = s_cnt[i] & 0x7fffffffu;
        if (cs == 0) continue;
        if (i % NW == wid) {
            const int ks = i / NW;
#pragma unroll
            for (int k = 0; k < CPL; k++) {
                if (k != ks) continue;
                unsigned long long nz = __ballot(cnt[k] > 0);
                uint32_t ac = 0, ar = 0;
                while (nz && ac < 3) {
                    const int h = 63 - __clzll(nz);
                    const uint32_t x[4] = {(uint32_t)__builtin_amdgcn_readlane(w[k][0], h),
                                           (uint32_t)__builtin_amdgcn_readlane(w[k][1], h),
                                           (uint32_t)__builtin_amdgcn_readlane(w[k][2], h),
                                           (uint32_t)__builtin_amdgcn_readlane(w[k][3], h)};
                    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane(cnt[k], h);
                    // its last (up to three) kept bytes, from the top word down
                    uint32_t car = 0, nc = 0;
#pragma unroll
                    for (int i = 3; i >= 0; i--) {
                        uint32_t m = kept8(x[i]);
                        while (m && nc < 3) {
                            const int hb = 31 - __clz(m);  // bit 8j+7 of byte j
                            car |= ((x[i] >> (hb - 7)) & 0xffu) << (8 * nc);
                            m &= ~(1u << hb);
                            nc++;
                        }
                    }
                    ar = car_join(car, ar, ac);
                    ac += c;
                    nz &= ~(1ull << h);
                }
                if (lane == 0) s_car[i] = ar;
            }
        }
        need -= (int)min(cs, 3u);
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t cnt = 0;
        uint32_t ctrl = 0;
        for (int i = 0; i < E; i++) {
            cnt += s_cnt[i] & 0x7fffffffu;
            ctrl |= s_cnt[i];
        }
        uint32_t ac = 0, ar = 0;
        for (int i = E - 1; i >= 0 && ac < 3; i--) {
            const uint32_t cs = s_cnt[i] & 0x7fffffffu;
            if (cs == 0) continue;
            ar = car_join(s_car[i], ar, ac);
            ac += cs;
        }
        ws[WS_SLOT_WORDS + t] = st_pack({cnt, ar}) | ((ctrl >> 31) ? WS_CTRL_FLAG : 0ull);
    }
}

// Group g: the ordered combination of tile states [g * WS_GROUP, ...).
__global__ __launch_bounds__(WS_SCAN_BLOCK) void k_ws_reduce(unsigned long long *__restrict__ ws, int64_t T)
{
    const unsigned long long *st = ws + WS_SLOT_WORDS;
    unsigned long long *grp = ws + WS_SLOT_WORDS + 2 * T;
    const int64_t i0 = (int64_t)blockIdx.x * WS_GROUP + (int64_t)threadIdx.x * WS_SCAN_PER;
    WsSt v{0, 0};
    for (int i = 0; i < WS_SCAN_PER; i++)
        if (i0 + i < T) v = st_join(v, st_unpack(st[i0 + i]));
    WsSt tot;
    (void)block_scan_st(v, &tot);
    if (threadIdx.x == 0) grp[blockIdx.x] = st_pack(tot);
}

// Exclusive prefix state of every tile: groups before this block (an ordered
// reduction over them), then the block's own ordered scan.
__global__ __launch_bounds__(WS_SCAN_BLOCK) void k_ws_prefix(unsigned long long *__restrict__ ws, int64_t T)
{
    const unsigned long long *st = ws + WS_SLOT_WORDS;
    unsigned long long *pre = ws + WS_SLOT_WORDS + T;
    const unsigned long long *grp = ws + WS_SLOT_WORDS + 2 * T;
    const int64_t g = blockIdx.x;
    // groups [0, g): thread i combines a contiguous share, then the block scan
    // orders the shares
    const int64_t per = (g + WS_SCAN_BLOCK - 1) / WS_SCAN_BLOCK;
    WsSt gv{0, 0};
    for (int64_t j = (int64_t)threadIdx.x * per; j < min(g, (int64_t)(threadIdx.x + 1) * per); j++)
        gv = st_join(gv, st_unpack(grp[j]));
    WsSt before;
    (void)block_scan_st(gv, &before);
    const int64_t i0 = g * WS_GROUP + (int64_t)threadIdx.x * WS_SCAN_PER;
    WsSt tv[WS_SCAN_PER];
    WsSt v{0, 0};
    for (int i = 0; i < WS_SCAN_PER; i++) {
        tv[i] = i0 + i < T ? st_unpack(st[i0 + i]) : WsSt{0, 0};
        v = st_join(v, tv[i]);
    }
    WsSt tot;
    const WsSt inc = block_scan_st(v, &tot);
    (void)tot;
    // exclusive prefix of this thread's first tile: the groups before, then
    // the inclusive scan of the previous thread
    __shared__ unsigned long long s_last[16];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const WsSt prev = shfl_up_st(inc, 1);
    if (lane == 63) s_last[wid] = st_pack(inc);
    __syncthreads();
    WsSt p{0, 0};
    if (threadIdx.x > 0) p = lane > 0 ? prev : st_unpack(s_last[wid - 1]);
    WsSt run = st_join(before, p);
    for (int i = 0; i < WS_SCAN_PER; i++) {
        if (i0 + i < T) pre[i0 + i] = st_pack(run);
        run = st_join(run, tv[i]);
    }
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts
// by 1, 2, 4, 8 within each row of 16 lanes, then the last lane of a row is
// added to the next row (row_bcast:15) and lane 31 to the upper half
// (row_bcast:31). Lanes whose DPP source lies outside the row keep 0.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Quad of class bytes (first byte lowest) -> 24-bit group a<<18|b<<12|c<<6|d.
__device__ __forceinline__ uint32_t quad_bits(uint32_t v)
{
    return ((v & 0x3f) << 18) | (((v >> 8) & 0x3f) << 12) | (((v >> 16) & 0x3f) << 6) | ((v >> 24) & 0x3f);
}

// Tile = BLOCK * 16 * CPL bytes, loaded as 16-byte chunks (k * BLOCK + tid)
// and staged in LDS; counting and compaction then work on dwords
// d = k2 * BLOCK + tid (k2 < 4 * CPL), so that lanes touch consecutive LDS
// words and memory order is (k2, wave, lane, byte). The raw kept bytes are
// compacted; symbol values are looked up only when the quads are decoded, and
// marks (invalid bytes, '=') send the tile through a rescan of its raw bytes
// that reports them in original coordinates.
template <int BLOCK, int CPL, bool ALIGNED>
__global__ __launch_bounds__(BLOCK) void k_dec_ws(const uint8_t *__restrict__ src, int64_t n,
                                                  uint8_t *__restrict__ dst, int alpha,
                                                  unsigned long long *__restrict__ ws, int64_t T, int64_t t0)
{
    constexpr int TILE = BLOCK * 16 * CPL;  // input bytes per tile
    constexpr int NW = BLOCK / 64;
    constexpr int K2 = 4 * CPL;             // dwords per lane
    constexpr int E = K2 * NW;              // (k2, wave) segments
    static_assert(E <= 128, "segment scan covers at most 128 entries");
    __shared__ uint32_t s_tab[64];
    __shared__ __attribute__((aligned(16))) uint32_t s_raw[TILE / 4];      // raw tile
    // stripped text, from byte F - r0 (F in [16, 32), chosen per tile so that
    // every unit of four quads after the head starts on a 16-byte boundary),
    // with tail room for the last unit's read past a partial quad
    __shared__ uint4 s_txt4[(32 + TILE + 32) / 16];
    uint8_t *const s_txt = (uint8_t *)s_txt4;
    __shared__ uint32_t s_seg[E];          // kept bytes per segment

    const int tid = threadIdx.x, lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
    lds_fill(s_tab, c_ws.cls[alpha], 256);
    const uint8_t *tab = (const uint8_t *)s_tab;
    const int64_t t = t0 + blockIdx.x;  // tile (a launch covers tiles [t0, t0 + gridDim.x))
    const int64_t base = t * TILE;
    {
        uint32_t w[CPL][4];
#pragma unroll
        for (int k = 0; k < CPL; k++) tile_load16<ALIGNED>(src, n, base + 16 * ((int64_t)k * BLOCK + tid), w[k]);
#pragma unroll
        for (int k = 0; k < CPL; k++)
            *(uint4 *)&s_raw[4 * (k * BLOCK + tid)] = make_uint4(w[k][0], w[k][1], w[k][2], w[k][3]);
    }
    // the tile's own state (flag: a control byte other than whitespace) and
    // its exclusive prefix: stripped offset of the tile's first kept byte and
    // the kept bytes before it
    const unsigned long long own = ws[WS_SLOT_WORDS + t];
    const WsSt pf = st_unpack(ws[WS_SLOT_WORDS + T + t]);
    const int64_t P = (int64_t)pf.c;
    const int r0 = (int)(P & 3);
    // the tile's first quad is global quad qp; hq quads precede the first
    // global quad index divisible by 4 (where the units of four quads start)
    const int64_t qp = (P - r0) >> 2;
    const int hq = (int)((4 - (qp & 3)) & 3);
    const int F = 16 + ((r0 - 4 * hq) & 15);  // F - r0 + 4 * hq is a multiple of 16
    if (tid < r0) s_txt[F - r0 + tid] = (uint8_t)(pf.r >> (8 * (r0 - 1 - tid)));
    __syncthreads();

    // 1. kept bytes per dword; per-lane exclusive prefixes within the wave
    // from one DPP scan per three dwords (10-bit fields: a wave keeps at most
    // 256 bytes of a dword row)
    uint32_t xs[K2], keepm[K2], pre[K2];
#pragma unroll
    for (int k0 = 0; k0 < K2; k0 += 3) {
        uint32_t packed = 0;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int k = k0 + i;
            if (k < K2) {
                xs[k] = s_raw[k * BLOCK + tid];
                keepm[k] = kept8(xs[k]);
                packed |= (uint32_t)__popc(keepm[k]) << (10 * i);
            }
        }
        const uint32_t inc = wave_incl_sum(packed);
        const uint32_t ex = inc - packed;
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int k = k0 + i;
            if (k < K2) {
                pre[k] = (ex >> (10 * i)) & 0x3ff;
                if (lane == 0) s_seg[k * NW + wid] = (tot >> (10 * i)) & 0x3ff;
            }
        }
    }
    __syncthreads();
    // 2. exclusive prefix over the (k2, wave) segments, computed by every
    // wave (no barrier), and the tile's kept total: lane i holds segment i
    // (segments 2i and 2i + 1 when there are more than 64), scanned with DPP;
    // a segment's prefix is read out with readlane (here for the wave's own
    // segments, later by the rare rescan for any segment)
    constexpr int SPL = E > 64 ? 2 : 1;  // segments per lane
    uint32_t sa, sx, ktot;               // lane's first segment count, its exclusive prefix
    {
        const uint32_t a0 = SPL * lane < E ? s_seg[SPL * lane] : 0u;
        const uint32_t a1 = (SPL == 2 && 2 * lane + 1 < E) ? s_seg[2 * lane + 1] : 0u;
        const uint32_t sum = a0 + a1;
        const uint32_t inc = wave_incl_sum(sum);
        sx = inc - sum;
        sa = a0;
        ktot = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
    auto seg_prefix = [&](int e) -> uint32_t {  // e: wave-uniform segment index
        const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)sx, SPL == 1 ? e : e >> 1);
        return (SPL == 2 && (e & 1)) ? x + (uint32_t)__builtin_amdgcn_readlane((int)sa, e >> 1) : x;
    };
    uint32_t segpre[K2];
#pragma unroll
    for (int k = 0; k < K2; k++) segpre[k] = seg_prefix(k * NW + wid);

    // 3. compaction: kept raw bytes to s_txt[F + tile-stripped index]
#pragma unroll
    for (int k = 0; k < K2; k++) {
        const uint32_t x = xs[k], keep = keepm[k];
        uint32_t pos = F + segpre[k] + pre[k];
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (keep & (0x80u << (8 * j))) s_txt[pos++] = (uint8_t)(x >> (8 * j));
    }
    // 16 bytes of a symbol ('A', value 0) after the last kept byte: the unit
    // that reaches past the stripped text looks up no marks there
    if (tid < 16) s_txt[F + ktot + tid] = (uint8_t)'A';
    __syncthreads();

    // 4. decode the quads that end in this tile: stripped bytes
    // [P - r0, P + ktot) sit at s_txt[F - r0 ...]; quad i of the tile
    // (global quad qp + i) goes to dst + 3 * (qp + i). Units of four quads
    // start at a global quad index divisible by 4, so their 12 output bytes
    // are dword-aligned (with dst); a head unit takes the quads before the
    // first such index. Every kept byte is looked up, including those of a
    // trailing partial quad (decoded by the next tile, or left over at the end
    // of the text), so that each mark is seen by the tile that holds it.
    const int L = r0 + (int)min(ktot, (uint32_t)TILE);  // stripped bytes here
    const int64_t qcap = n / 4 - qp;                    // never past 3 * (n / 4)
    const int Q = (int)max((int64_t)0, min((int64_t)(L >> 2), qcap));  // quads decoded
    const int QC = (L + 3) >> 2;                                         // quads checked
    const int head = hq > 0 ? 1 : 0;
    const int U = head + (QC > hq ? (QC - hq + 3) >> 2 : 0);
    uint8_t *q0 = dst + 3 * qp;
    bool mark = false;
    for (int u = tid; u < U; u += BLOCK) {
        const bool hd = head && u == 0;
        const int s0 = hd ? 0 : hq + 4 * (u - head);
        const int nq = hd ? min(hq, Q) : min(4, Q - s0);           // quads to decode (may be <= 0)
        const int nb = min(hd ? 4 * hq : 16, L - 4 * s0);         // bytes to look up
        // 16 bytes from LDS byte F - r0 + 4 * s0 in one aligned read; the
        // head unit starts 4 * hq bytes before a 16-byte boundary, so its
        // quads are the last hq dwords of the chunk read
        const uint4 c = s_txt4[(F - r0 + 4 * s0) >> 4];
        uint32_t vs[4] = {c.x, c.y, c.z, c.w};
        if (hd) {
            // the head's quads; its other dwords hold a symbol, so they raise
            // no marks
            const uint32_t sym = 0x41414141u;
            if (hq == 1) {
                vs[0] = c.w; vs[1] = sym; vs[2] = sym;
            } else if (hq == 2) {
                vs[0] = c.z; vs[1] = c.w; vs[2] = sym;
            } else {
                vs[0] = c.y; vs[1] = c.z; vs[2] = c.w;
            }
            vs[3] = sym;
        }
        uint8_t *q = q0 + 3 * (int64_t)s0;
        {
            uint32_t tq[4], mk = 0;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t a = tab[vs[i] & 0xff], b = tab[(vs[i] >> 8) & 0xff];
                const uint32_t c = tab[(vs[i] >> 16) & 0xff], e = tab[vs[i] >> 24];
                mk |= a | b | c | e;
                tq[i] = (a << 18) | (b << 12) | (c << 6) | e;
            }
            if (!(mk & 0x80u)) {
                const uint32_t o[4] = {perm(tq[1], tq[0], 0x06000102u), perm(tq[2], tq[1], 0x05060001u),
                                       perm(tq[3], tq[2], 0x04050600u), 0u};
                if (nq == 4) {
                    const uint32_t o3[3] = {o[0], o[1], o[2]};
                    store_words<3, true>(q, o3);
                } else if (nq > 0) {
                    store_upto16(q, o, 3 * nq);  // the head unit, or the text's last quads here
                }
                continue;
            }
        }
        // marks (rare): '=' counts as 0 and the bytes it pads are not written
        // (any other placement is an error, and the output of an invalid input
        // is unspecified)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (4 * i < nb) {
                uint32_t cv = 0;
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (4 * i + j < nb) cv |= (uint32_t)tab[(vs[i] >> (8 * j)) & 0xff] << (8 * j);
                const uint32_t mk = cv & 0x80808080u;
                mark |= mk != 0;
                if (i < nq) {
                    const uint32_t c2 = (cv >> 16) & 0xff, c3 = cv >> 24;
                    const uint32_t tv = quad_bits(cv & ~(mk >> 2) & ~mk);
                    q[3 * i] = (uint8_t)(tv >> 16);
                    if (!(c2 == C_PAD && c3 == C_PAD)) q[3 * i + 1] = (uint8_t)(tv >> 8);
                    if (c3 != C_PAD) q[3 * i + 2] = (uint8_t)tv;
                }
            }
        }
    }

    // 5. invalid bytes and '=' in original coordinates (rare): a wave that
    // looked up a mark rescans the whole raw tile through the class table
    // (the mark may sit in any wave's raw segment), as does wave 0 when the
    // count pass flagged a control byte in this tile. The first mark of each
    // kind per lane and dword goes to its slot.
    if (__ballot(mark) != 0 || (wid == 0 && (own & WS_CTRL_FLAG))) {
#pragma unroll 1
        for (int e = 0; e < E; e++) {
            const int dw = (e / NW) * BLOCK + (e % NW) * 64 + lane;  // raw dword
            const uint32_t x = s_raw[dw];
            const uint32_t keep = kept8(x);
            const uint32_t c = __popc(keep);
            const int64_t at = P + seg_prefix(e) + (wave_incl_sum(c) - c);
            const int64_t off = base + 4 * (int64_t)dw;
            unsigned long long eb = ERR_NONE, eo = ERR_NONE, es = ERR_NONE;
            uint32_t rank = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t cb = tab[(x >> (8 * j)) & 0xff];
                if (cb == C_BAD && eb == ERR_NONE) eb = (unsigned long long)(off + j);
                if (cb == C_PAD && eo == ERR_NONE) {
                    eo = (unsigned long long)(off + j);
                    es = (unsigned long long)(at + rank);
                }
                rank += (keep >> (8 * j + 7)) & 1;
            }
            if (eb != ERR_NONE) atomicMin(&ws[1], eb);
            if (eo != ERR_NONE) {
                atomicMin(&ws[2], eo);
                atomicMin(&ws[3], es);
            }
        }
    }
}

// Verdict of an empty input: (0, -1).
__global__ void k_ws_empty(int64_t *d_len, int64_t *d_err)
{
    if (threadIdx.x == 0) {
        *d_len = 0;
        *d_err = -1;
    }
}

// Verdict: (decoded length, -1) or (-1, first offending original index).
__global__ void k_dec_ws_final(const unsigned long long *__restrict__ ws, int64_t T, int64_t n,
                               int64_t *__restrict__ d_len, int64_t *__restrict__ d_err)
{
    if (threadIdx.x || blockIdx.x) return;
    const WsSt all = st_join(st_unpack(ws[WS_SLOT_WORDS + T + T - 1]), st_unpack(ws[WS_SLOT_WORDS + T - 1]));
    const int64_t m = (int64_t)all.c;
    const uint32_t last = all.r & 0xff;
    const unsigned long long bad = ws[1], eq_o = ws[2], eq_s = ws[3];
    bool pad_ok = true;
    int64_t pads = 0;
    if (eq_s != ERR_NONE) {
        const int64_t e = (int64_t)eq_s;
        pad_ok = (m & 3) == 0 && (e == m - 1 || (e == m - 2 && last == '='));
        pads = m - e;
    }
    // With an invalid byte at i, the first '=' (if before i) is followed by a
    // kept non-'=' byte and so misplaced: the first error is min(i, first
    // '='). Without one, the counts are exact and the padding rule decides.
    unsigned long long err = bad;
    if ((bad != ERR_NONE || !pad_ok) && eq_o < err) err = eq_o;
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
constexpr int64_t WS_MIN_TILE = 256 * 16;

// Launch shape, block << 8 | chunks per lane, in one word so that a call
// always reads a pair that was set together. Default: the fastest shape of a
// sweep on MI355X (MIME text, 1.47 GB).
std::atomic<int> g_ws{256 << 8 | 2};

int64_t ws_tiles(int64_t n, int64_t tile) { return (n + tile - 1) / tile; }
int64_t ws_words(int64_t T) { return WS_SLOT_WORDS + 2 * T + (T + WS_GROUP - 1) / WS_GROUP; }

// The count pass of a tile of `chunks` 16-byte chunks. Its result does not
// depend on how the tile is split over lanes, so it takes its own shape:
// eight chunks per lane (four for the smallest tile) on as few lanes as
// cover the tile, at least one wave. With more loads in flight per lane and
// fewer lanes per tile it ran faster than the decode pass's shape (MIME
// text, 1.47 GB, 8 KiB tiles: 274 us at 256 x 2, 227 us at 64 x 8).
template <bool A>
void launch_count(int chunks, int64_t T, const uint8_t *src, int64_t n, unsigned long long *ws, hipStream_t s)
{
    const dim3 g((unsigned)T);
    switch (chunks) {
    case 256: hipLaunchKernelGGL((k_ws_count<64, 4, A>), g, 64, 0, s, src, n, ws); break;
    case 512: hipLaunchKernelGGL((k_ws_count<64, 8, A>), g, 64, 0, s, src, n, ws); break;
    case 1024: hipLaunchKernelGGL((k_ws_count<128, 8, A>), g, 128, 0, s, src, n, ws); break;
    default: hipLaunchKernelGGL((k_ws_count<256, 8, A>), g, 256, 0, s, src, n, ws); break;
    }
}

// The count pass runs 64-256 lanes per tile of 4-32 KiB (at most n / 64
// work-items, below 2^32 for any n below 2^38). The decode pass runs a
// workgroup per tile, which passes 2^32 work-items (the most one launch
// holds) above 2^36 bytes at one 16-byte chunk per lane; its tiles do not
// depend on each other, so it is launched in pieces of at most
// (2^32 - 1) / block tiles.
template <bool A>
int launch_ws(int block, int cpl, int64_t T, const uint8_t *src, int64_t n, uint8_t *dst, int alpha,
              unsigned long long *ws, hipStream_t s)
{
    const unsigned G = (unsigned)((T + WS_GROUP - 1) / WS_GROUP);
    const int64_t piece = (((int64_t)1 << 32) - 1) / block;
#define B64_WS_CASE(B, C)                                                                      \
    if (block == B && cpl == C) {                                                              \
        launch_count<A>(B * C, T, src, n, ws, s);                                              \
        hipLaunchKernelGGL(k_ws_reduce, G, WS_SCAN_BLOCK, 0, s, ws, T);                        \
        hipLaunchKernelGGL(k_ws_prefix, G, WS_SCAN_BLOCK, 0, s, ws, T);                        \
        for (int64_t t0 = 0; t0 < T; t0 += piece)                                              \
            hipLaunchKernelGGL((k_dec_ws<B, C, A>), dim3((unsigned)std::min(piece, T - t0)), B, \
                               0, s, src, n, dst, alpha, ws, T, t0);                           \
        return B64_OK;                                                                         \
    }
    B64_WS_CASE(256, 1) B64_WS_CASE(256, 2) B64_WS_CASE(256, 4) B64_WS_CASE(256, 8)
    B64_WS_CASE(512, 1) B64_WS_CASE(512, 2) B64_WS_CASE(512, 4)
    B64_WS_CASE(1024, 1) B64_WS_CASE(1024, 2)
#undef B64_WS_CASE
    return b64i_fail(B64_BAD_ARG, "unsupported whitespace-decode shape %d x %d", block, cpl);
}

// Enqueues the count, scan, decode and verdict kernels. n >= 1.
int enqueue_ws(const uint8_t *src, int64_t n, uint8_t *dst, int alpha, int64_t *d_len, int64_t *d_err,
               unsigned long long *ws, hipStream_t s)
{
    const int shape = g_ws.load();
    const int block = shape >> 8, cpl = shape & 0xff;
    const int64_t T = ws_tiles(n, (int64_t)block * 16 * cpl);
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
    return 8 * ws_words(std::max<int64_t>(ws_tiles(n, WS_MIN_TILE), 1));
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
    if (n == 0) {  // verdict (0, -1), enqueued like any other (no host wait, capturable)
        hipLaunchKernelGGL(k_ws_empty, 1, 64, 0, s, d_len, d_err);
        LAUNCH_TRY();
        return B64_OK;
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
        // kept only once both allocations succeeded
        WsCache e;
        e.dev = dev;
        hipError_t r = hipMalloc((void **)&e.verdict, 16);
        if (r == hipSuccess) r = hipHostMalloc((void **)&e.h, 16, hipHostMallocDefault);
        if (r != hipSuccess) {
            if (e.verdict) (void)hipFree(e.verdict);
            return b64i_fail(B64_HIP_ERROR, "whitespace-decode slots: %s", hipGetErrorString(r));
        }
        t_ws.push_back(e);
        c = &t_ws.back();
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
    const int cur = g_ws.load();
    const int block = t->block ? t->block : cur >> 8;
    const int cpl = t->units_per_lane ? t->units_per_lane : cur & 0xff;
    const bool ok = (block == 256 && (cpl == 1 || cpl == 2 || cpl == 4 || cpl == 8)) ||
                    (block == 512 && (cpl == 1 || cpl == 2 || cpl == 4)) ||
                    (block == 1024 && (cpl == 1 || cpl == 2));
    if (!ok)
        return b64i_fail(B64_BAD_ARG, "whitespace-decode shape: block 256 (1/2/4/8 chunks), 512 (1/2/4) "
                                      "or 1024 (1/2) with 16-byte chunks per lane");
    g_ws = block << 8 | cpl;
    return B64_OK;
}

}  // extern "C"
