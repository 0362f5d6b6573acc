// gfx950 kernels of the single-buffer codec and their C-ABI (include/b64.h).
//
//   k_enc_single  Algorithm 1 over one buffer: grid-stride over 12-byte
//                 units, one unit per lane, then the final partial unit.
//   k_dec_single  Algorithm 2 over one buffer: grid-stride over interior
//                 16-character units, then the final unit with the padding
//                 and length rules.
//   k_dec_small   one-workgroup decode of a short input, verdict included.
//   k_slots_init  sets a decode's result slots to (0, -1) before the decode
//                 kernel forms the verdict in them (streams without a cell).
//
// A decode's verdict is formed inside k_dec_single itself: with a verdict
// cell, by the workgroup that finishes last (see VerdictCell), so an
// asynchronous decode is one launch; otherwise in the caller's slots, which
// k_slots_init has set to (0, -1): an error lowers the error slot (unsigned
// atomicMin, -1 being above every index) and sets the length to -1, and the
// valid final unit moves the length from 0 to its value by compare-and-swap.

// Decode errors: a lane whose unit holds a non-symbol computes the exact
// index; a wave ballot elects the first erring lane, which performs one
// atomicMin on the 64-bit error slot (Section 2: the decoder must report
// characters outside the alphabet; the smallest index is the one reported).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "b64.h"
#include "b64_device.hpp"
#include "b64_internal.hpp"

using namespace b64dev;

static __constant__ Tables c_tab = make_tables();
static __constant__ PermMaps c_perm = make_perm_maps();
static __constant__ PairTables c_pair = make_pair_tables();

// Map context of one launch (see MapCtx): LDS tables filled by the caller.
template <int MAP>
__device__ __forceinline__ MapCtx map_ctx(const uint8_t *tab, const uint16_t *tab12, int url, bool decode)
{
    MapCtx m{};
    m.tab = tab;
    m.tab12 = tab12;
    if (MAP == 1) {
        if (!decode) {
            m.e0 = c_perm.enc_off[url][0];
            m.e1 = c_perm.enc_off[url][1];
        } else {
            m.l0 = c_perm.dec_lo[url][0]; m.l1 = c_perm.dec_lo[url][1];
            m.l2 = c_perm.dec_lo[url][2]; m.l3 = c_perm.dec_lo[url][3];
            m.h0 = c_perm.dec_hi[url][0]; m.h1 = c_perm.dec_hi[url][1];
            m.r0 = c_perm.dec_roll[url][0]; m.r1 = c_perm.dec_roll[url][1];
            m.sp = c_perm.special[url];
        }
    }
    return m;
}

// Encode src[0, n): full units [0, n / 12) in a grid-stride loop over tiles
// of blockDim * UPL units, then the final partial unit (Algorithm 1's tail)
// by one lane. AL: 0 source and destination 4-byte aligned, 1 only the
// destination, 2 a misaligned destination (written whole dwords per wave).
template <int AL, int UPL, int MAP>
__global__ __launch_bounds__(1024) void k_enc_single(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, int mode)
{
    __shared__ uint32_t s_tab[16];
    __shared__ uint32_t s_pair[MAP == 2 ? 2048 : 1];
    lds_fill(s_tab, c_tab.enc[mode & M_URL], 64);
    if (MAP == 2) lds_fill(s_pair, (const uint8_t *)c_pair.pair[mode & M_URL], 8192);
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;
    const MapCtx mc = map_ctx<MAP>(tab, (const uint16_t *)s_pair, mode & M_URL, false);

    const int64_t units = n / 12;
    const int64_t tile = (int64_t)blockDim.x * UPL;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < units; t0 += (int64_t)gridDim.x * tile) {
        if (t0 + tile <= units)
            enc_step<AL == 0, UPL, false, MAP, AL == 2>(src, dst, t0 + threadIdx.x, blockDim.x, units, mc, units);
        else
            enc_step<AL == 0, UPL, true, MAP, AL == 2>(src, dst, t0 + threadIdx.x, blockDim.x, units, mc, units);
    }
    const int r = (int)(n - 12 * units);
    if (r && blockIdx.x == 0 && threadIdx.x == 0)
        enc_tail(src + 12 * units, r, dst + 16 * units, tab, mode & M_NOPAD);
}

// Verdict cell of a one-launch decode: the workgroups of one launch meet in
// it to form the verdict without a second kernel. At rest (before and after
// every launch) it is all zero, which is also the state a static device
// array starts in, so it needs no initialisation. The first offending index
// e is kept as ERR_NONE - e under atomicMax (0 = no error yet), so that the
// resting value means "none".
struct VerdictCell {
    unsigned long long err;   // ERR_NONE - smallest offending index, or 0
    unsigned long long len;   // decoded length, written by the final unit when valid
    unsigned int done;        // workgroups finished
    unsigned int pad[3];
};
constexpr int VERDICT_CELLS = 1024;
static __device__ __align__(256) VerdictCell g_cells[VERDICT_CELLS];

// Decode src[0, n), n >= 1. Interior units [0, L) with L = (n - 1) / 16 hold
// 16 characters that are all before the final one; unit L (1..16 characters)
// carries the padding and length rules.
//   CELL == false: *len_slot and *err_slot must hold 0 and -1 at launch;
//     they end holding the verdict (length, -1) or (-1, first offending
//     index).
//   CELL == true: each workgroup keeps its smallest offending index in LDS,
//     folds it into *cell and counts itself done there; the workgroup that
//     finishes last writes the verdict (length, -1) or (-1, index) to
//     d_len / d_err and returns the cell to rest. The cell must be at rest at
//     launch and used by no other launch until this one ends.
// AL as for k_enc_single.
template <int AL, int UPL, int MAP, bool CELL>
__global__ __launch_bounds__(1024) void k_dec_single(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, int mode,
                                                     unsigned long long *err_slot, int64_t *len_slot,
                                                     VerdictCell *cell, int64_t *d_len, int64_t *d_err)
{
    __shared__ uint32_t s_tab[64];
    __shared__ unsigned long long s_err;
    lds_fill(s_tab, c_tab.dec[mode & M_URL], 256);
    if (CELL && threadIdx.x == 0) s_err = ERR_NONE;
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;
    const MapCtx mc = map_ctx<MAP>(tab, nullptr, mode & M_URL, true);
    unsigned long long *const es = CELL ? &s_err : err_slot;

    const int64_t L = (n - 1) / 16;
    const int64_t tile = (int64_t)blockDim.x * UPL;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < L; t0 += (int64_t)gridDim.x * tile) {
        if (t0 + tile <= L)
            dec_step<AL == 0, UPL, false, MAP, AL == 2>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, es, L,
                                                         CELL ? nullptr : len_slot);
        else
            dec_step<AL == 0, UPL, true, MAP, AL == 2>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, es, L,
                                                        CELL ? nullptr : len_slot);
    }
    int64_t len = -1;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int r = (int)(n - 16 * L);
        const int res = dec_tail(src + 16 * L, r, n, dst + 12 * L, tab, mode);
        if (res >= 0) {
            atomicMin(es, (unsigned long long)(16 * L + res));
            if (!CELL) atomicExch((unsigned long long *)len_slot, ~0ull);
        } else if (CELL) {
            len = 12 * L + (-1 - res);
        } else {
            atomicCAS((unsigned long long *)len_slot, 0ull, (unsigned long long)(12 * L + (-1 - res)));
        }
    }
    if constexpr (CELL) {
        __syncthreads();
        if (threadIdx.x == 0) {
            // The cell is only touched through device-scope atomics, which act
            // on one coherent copy. This workgroup's reports are waited for
            // (their returned values consumed) before it counts itself, so the
            // workgroup that counts last finds every report in the cell. No
            // release fence: that would write back this XCD's L2 on every count.
            const unsigned long long e = s_err;
            unsigned long long seen = 0;
            if (e != ERR_NONE)
                seen |= __hip_atomic_fetch_max(&cell->err, ERR_NONE - e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (len >= 0)
                seen |= __hip_atomic_exchange(&cell->len, (unsigned long long)len, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            asm volatile("" ::"v"(seen) : "memory");
            const unsigned prev = __hip_atomic_fetch_add(&cell->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == gridDim.x - 1) {
                const unsigned long long v = __hip_atomic_exchange(&cell->err, 0ull, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long l = __hip_atomic_exchange(&cell->len, 0ull, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_exchange(&cell->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v == 0) { *d_len = (int64_t)l; *d_err = -1; }
                else { *d_len = -1; *d_err = (int64_t)(ERR_NONE - v); }
            }
        }
    }
}

// Decode of a short input by one workgroup, verdict included, so that the
// whole call is one launch: the first offending index is kept in an LDS slot
// (unsigned atomicMin) and thread 0 writes (length, -1) or (-1, index) at
// the end. It takes inputs of at most SMALL_UNITS_CELL interior units (one
// pass of its 1,024 lanes x 2 units), and up to SMALL_UNITS on a stream
// without a verdict cell, where the alternative is two launches. Between
// the two, the one-launch grid of k_dec_single is faster (6.1 against
// 6.4-11.8 us for 64-256 KiB of text on MI355X).
constexpr int64_t SMALL_UNITS_CELL = 2048;
constexpr int64_t SMALL_UNITS = 16384;

template <bool ALIGNED>
__global__ __launch_bounds__(1024) void k_dec_small(const uint8_t *__restrict__ src, int64_t n,
                                                    uint8_t *__restrict__ dst, int mode,
                                                    int64_t *__restrict__ d_len, int64_t *__restrict__ d_err)
{
    __shared__ uint32_t s_tab[64];
    __shared__ unsigned long long s_err;
    __shared__ int64_t s_len;
    lds_fill(s_tab, c_tab.dec[mode & M_URL], 256);
    if (threadIdx.x == 0) s_err = ERR_NONE;
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;
    const MapCtx mc = map_ctx<0>(tab, nullptr, mode & M_URL, true);
    const int64_t L = (n - 1) / 16;
    if (threadIdx.x == 0) {
        const int res = dec_tail(src + 16 * L, (int)(n - 16 * L), n, dst + 12 * L, tab, mode);
        if (res >= 0) atomicMin(&s_err, (unsigned long long)(16 * L + res));
        s_len = 12 * L + (res >= 0 ? 0 : -1 - res);
    }
    const int64_t tile = (int64_t)blockDim.x * 2;
    for (int64_t t0 = 0; t0 < L; t0 += tile) {
        if (t0 + tile <= L)
            dec_step<ALIGNED, 2, false, 0>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, &s_err);
        else
            dec_step<ALIGNED, 2, true, 0>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, &s_err);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long e = s_err;
        if (e == ERR_NONE) { *d_len = s_len; *d_err = -1; }
        else { *d_len = -1; *d_err = (int64_t)e; }
    }
}

// Sets an asynchronous decode's result slots to (0, -1): the verdict of an
// empty input, and the state k_dec_single (without a cell) forms its
// verdict from.
__global__ void k_slots_init(int64_t *d_len, int64_t *d_err)
{
    if (threadIdx.x == 0) {
        *d_len = 0;
        *d_err = -1;
    }
}

// ================================================================= host ==
namespace {

// Launch shapes of the single-buffer kernels (settable for tuning sweeps).
// Defaults: one workgroup per tile (blocks_per_cu == 0) with 2 units per
// lane, 512 lanes to encode and 256 to decode: the fastest shapes of a sweep
// over block {256, 512, 1024} x units {1, 2, 4} x grid {8, 16, 32 per CU,
// one-shot} on MI355X at 1 GiB.
struct Shape {
    Shape(int b) : block(b) {}
    std::atomic<int> block;
    std::atomic<int> upl{2};
    std::atomic<int> blocks_per_cu{0};
    std::atomic<int> map{0};  // 0 LDS byte tables, 1 register maps, 2 (encode) LDS pair table
};
Shape g_single[2] = {512, 256};

// Per-thread, per-device verdict slots of the synchronous decode, each a
// (length, first offending index) pair written by every call: device slots d
// with the pinned pair h they are read back into, for the two-launch decode
// (its verdict is formed by atomics in device memory), and a coherent pinned
// pair hc (device address hc_dev) that the one-launch decodes write their
// verdict to directly (two plain stores, no copy back).
struct SyncSlot {
    int dev = -1;
    int64_t *d = nullptr;
    int64_t *h = nullptr;
    int64_t *hc = nullptr;
    int64_t *hc_dev = nullptr;
};
// Value of a verdict word that the decode has not written yet.
constexpr int64_t VERDICT_UNSET = INT64_MIN;
thread_local std::vector<SyncSlot> t_slots;

int sync_slot(SyncSlot **out)
{
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    for (auto &s : t_slots)
        if (s.dev == dev) { *out = &s; return B64_OK; }
    // kept only once every step succeeded (a failed step frees what it got)
    SyncSlot s;
    s.dev = dev;
    hipError_t e = hipMalloc((void **)&s.d, 64);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.h, 16, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.hc, 16, hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s.hc_dev, s.hc, 0);
    if (e != hipSuccess) {
        if (s.hc) (void)hipHostFree(s.hc);
        if (s.h) (void)hipHostFree(s.h);
        if (s.d) (void)hipFree(s.d);
        return b64i_fail(B64_HIP_ERROR, "synchronous-call slots: %s", hipGetErrorString(e));
    }
    t_slots.push_back(s);
    *out = &t_slots.back();
    return B64_OK;
}

int single_grid(int dir, int64_t units, int *block, int *upl, int *grid)
{
    int cus;
    int rc = b64i_device_cus(&cus);
    if (rc) return rc;
    *block = g_single[dir].block.load();
    *upl = g_single[dir].upl.load();
    const int64_t per = (int64_t)(*block) * (*upl);
    int64_t tiles = (units + per - 1) / per;
    const int bpc = g_single[dir].blocks_per_cu.load();
    // a launch holds fewer than 2^32 work-items; the kernels stride over the
    // tiles, so a capped grid still covers every unit
    const int64_t cap = std::min<int64_t>(bpc ? (int64_t)cus * bpc : (int64_t)INT32_MAX,
                                          (((int64_t)1 << 32) - 1) / *block);
    *grid = (int)std::max<int64_t>(1, std::min(tiles, cap));
    return B64_OK;
}

#define B64_UPL_SWITCH(KERN, A, M, ...)                                                          \
    switch (upl) {                                                                               \
    case 1: hipLaunchKernelGGL((KERN<A, 1, M>), grid, block, 0, s, __VA_ARGS__); break;          \
    case 2: hipLaunchKernelGGL((KERN<A, 2, M>), grid, block, 0, s, __VA_ARGS__); break;          \
    case 8: hipLaunchKernelGGL((KERN<A, 8, M>), grid, block, 0, s, __VA_ARGS__); break;          \
    default: hipLaunchKernelGGL((KERN<A, 4, M>), grid, block, 0, s, __VA_ARGS__); break;         \
    }

template <int A>
void launch_enc_single(int upl, int map, int grid, int block, const uint8_t *src, int64_t n, uint8_t *dst,
                       int mode, hipStream_t s)
{
    if (map == 1) {
        B64_UPL_SWITCH(k_enc_single, A, 1, src, n, dst, mode);
    } else if (map == 2) {
        B64_UPL_SWITCH(k_enc_single, A, 2, src, n, dst, mode);
    } else {
        B64_UPL_SWITCH(k_enc_single, A, 0, src, n, dst, mode);
    }
}

#define B64_UPL_SWITCH_DEC(A, M, C, ...)                                                         \
    switch (upl) {                                                                               \
    case 1: hipLaunchKernelGGL((k_dec_single<A, 1, M, C>), grid, block, 0, s, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((k_dec_single<A, 2, M, C>), grid, block, 0, s, __VA_ARGS__); break; \
    case 8: hipLaunchKernelGGL((k_dec_single<A, 8, M, C>), grid, block, 0, s, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((k_dec_single<A, 4, M, C>), grid, block, 0, s, __VA_ARGS__); break; \
    }

template <int A, bool C>
void launch_dec_single(int upl, int map, int grid, int block, const uint8_t *src, int64_t n, uint8_t *dst,
                       int mode, unsigned long long *slot, int64_t *len_slot, VerdictCell *cell,
                       int64_t *d_len, int64_t *d_err, hipStream_t s)
{
    if (map == 1) {
        B64_UPL_SWITCH_DEC(A, 1, C, src, n, dst, mode, slot, len_slot, cell, d_len, d_err);
    } else {
        B64_UPL_SWITCH_DEC(A, 0, C, src, n, dst, mode, slot, len_slot, cell, d_len, d_err);
    }
}
#undef B64_UPL_SWITCH_DEC
#undef B64_UPL_SWITCH

bool aligned4(const void *a, const void *b)
{
    return (((uintptr_t)a | (uintptr_t)b) & 3) == 0;
}

// Alignment class of a single-buffer launch (the AL template argument).
int align_class(const void *src, const void *dst)
{
    return aligned4(src, dst) ? 0 : ((uintptr_t)dst & 3) == 0 ? 1 : 2;
}

}  // namespace

int b64i_enqueue_encode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(0, n / 12, &block, &upl, &grid);
    if (rc) return rc;
    const int map = g_single[0].map.load();
    switch (align_class(src, dst)) {
    case 0: launch_enc_single<0>(upl, map, grid, block, src, n, dst, mode, s); break;
    case 1: launch_enc_single<1>(upl, map, grid, block, src, n, dst, mode, s); break;
    default: launch_enc_single<2>(upl, map, grid, block, src, n, dst, mode, s); break;
    }
    LAUNCH_TRY();
    return B64_OK;
}

// Enqueues the decode kernel of src[0, n) (n >= 1) that forms its verdict
// in *len_slot / *slot, which must hold 0 and -1.
int b64i_enqueue_decode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, unsigned long long *slot,
                        int64_t *len_slot, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(1, (n - 1) / 16, &block, &upl, &grid);
    if (rc) return rc;
    const int map = g_single[1].map.load();
    switch (align_class(src, dst)) {
    case 0:
        launch_dec_single<0, false>(upl, map, grid, block, src, n, dst, mode, slot, len_slot, nullptr, nullptr,
                                    nullptr, s);
        break;
    case 1:
        launch_dec_single<1, false>(upl, map, grid, block, src, n, dst, mode, slot, len_slot, nullptr, nullptr,
                                    nullptr, s);
        break;
    default:
        launch_dec_single<2, false>(upl, map, grid, block, src, n, dst, mode, slot, len_slot, nullptr, nullptr,
                                    nullptr, s);
        break;
    }
    LAUNCH_TRY();
    return B64_OK;
}

namespace {

// Verdict cells are handed out per (device, stream): launches on one stream
// run one after another, so a cell is back at rest before the next launch
// on its stream starts, while launches on different streams never share
// one. Streams beyond VERDICT_CELLS per device, the per-thread default
// stream (one handle for many streams), streams being captured (a graph may
// be replayed anywhere) and streams of a device other than the current one
// get no cell; their decodes take two launches.
struct CellTable {
    std::mutex mu;
    int dev = -1;
    VerdictCell *base = nullptr;
    std::vector<hipStream_t> owner;
};
std::mutex g_cells_mu;
std::vector<CellTable *> g_cell_tables;

VerdictCell *stream_cell(hipStream_t s)
{
    if (s == hipStreamPerThread) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (cs != hipStreamCaptureStatusNone) return nullptr;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (s != nullptr) {  // cells live on the current device: a stream of another takes none
        hipDevice_t sd;
        if (hipStreamGetDevice(s, &sd) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (sd != dev) return nullptr;
    }
    CellTable *t = nullptr;
    {
        std::lock_guard<std::mutex> g(g_cells_mu);
        for (CellTable *c : g_cell_tables)
            if (c->dev == dev) t = c;
        if (!t) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_cells)) != hipSuccess || !p) {
                (void)hipGetLastError();
                return nullptr;
            }
            t = new CellTable;
            t->dev = dev;
            t->base = (VerdictCell *)p;
            g_cell_tables.push_back(t);
        }
    }
    std::lock_guard<std::mutex> g(t->mu);
    for (size_t i = 0; i < t->owner.size(); i++)
        if (t->owner[i] == s) return t->base + i;
    if (t->owner.size() >= (size_t)VERDICT_CELLS) return nullptr;
    t->owner.push_back(s);
    return t->base + (t->owner.size() - 1);
}

// The counts of a verdict cell are atomics on one address, which the device
// serialises (13-16 ns apart on MI355X): a grid of G workgroups adds about
// G * 15 ns. The one-launch decode therefore keeps to the set launch shape
// only while that needs at most one workgroup per CU, then takes workgroups
// of 1,024 lanes x 4 units (64 KiB of text), up to this many. Larger inputs
// are decoded faster by the one-shot grid of small workgroups and the two
// extra launches.
constexpr int CELL_MAX_BLOCKS = 512;

int decode_two_launches(const uint8_t *src, int64_t n, uint8_t *dst, int mode, int64_t *d_len, int64_t *d_err,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_slots_init, 1, 64, 0, s, d_len, d_err);
    LAUNCH_TRY();
    return b64i_enqueue_decode(src, n, dst, mode, (unsigned long long *)d_err, d_len, s);
}

// One-workgroup decode of src[0, n) (n >= 1, at most SMALL_UNITS interior
// units) with its verdict written to d_len / d_err.
int decode_small(const uint8_t *src, int64_t n, uint8_t *dst, int mode, int64_t *d_len, int64_t *d_err,
                 hipStream_t s)
{
    if (aligned4(src, dst))
        hipLaunchKernelGGL(k_dec_small<true>, 1, 1024, 0, s, src, n, dst, mode, d_len, d_err);
    else
        hipLaunchKernelGGL(k_dec_small<false>, 1, 1024, 0, s, src, n, dst, mode, d_len, d_err);
    LAUNCH_TRY();
    return B64_OK;
}

// Decode of src[0, n) (n >= 1) with its verdict in d_len / d_err:
//   - at most SMALL_UNITS_CELL interior units: one workgroup (k_dec_small);
//   - on a stream with a verdict cell, up to 32 MiB of text: one launch of
//     k_dec_single, which forms the verdict itself;
//   - otherwise, at most SMALL_UNITS interior units: one workgroup;
//   - otherwise the slot initialisation and k_dec_single.
//   The one-launch paths write the verdict with two plain stores; given
//   `direct` (a device-visible pair, such as coherent pinned host memory)
//   they write it there instead of d_len / d_err, and *used_direct says
//   which pair holds the verdict. The two-launch path forms it by atomics on
//   d_len / d_err, which stay in device memory.
int decode_with_verdict(const uint8_t *src, int64_t n, uint8_t *dst, int mode, int64_t *d_len,
                        int64_t *d_err, hipStream_t s, int64_t *direct = nullptr, bool *used_direct = nullptr)
{
    int64_t *const l1 = direct ? direct : d_len, *const e1 = direct ? direct + 1 : d_err;
    if (used_direct) *used_direct = direct != nullptr;
    const int64_t units = (n - 1) / 16;
    if (units <= SMALL_UNITS_CELL) return decode_small(src, n, dst, mode, l1, e1, s);
    if (VerdictCell *cell = stream_cell(s)) {
        int block, upl, grid, cus;
        int rc = single_grid(1, units, &block, &upl, &grid);
        if (!rc) rc = b64i_device_cus(&cus);
        if (rc) return rc;
        if (grid > cus) {  // fewer, larger workgroups
            block = 1024;
            upl = 4;
            grid = (int)std::min<int64_t>((units + 4095) / 4096, INT32_MAX);
        }
        if (grid <= CELL_MAX_BLOCKS) {
            const int map = g_single[1].map.load();
            switch (align_class(src, dst)) {
            case 0:
                launch_dec_single<0, true>(upl, map, grid, block, src, n, dst, mode, nullptr, nullptr, cell, l1,
                                           e1, s);
                break;
            case 1:
                launch_dec_single<1, true>(upl, map, grid, block, src, n, dst, mode, nullptr, nullptr, cell, l1,
                                           e1, s);
                break;
            default:
                launch_dec_single<2, true>(upl, map, grid, block, src, n, dst, mode, nullptr, nullptr, cell, l1,
                                           e1, s);
                break;
            }
            LAUNCH_TRY();
            return B64_OK;
        }
    }
    if (units <= SMALL_UNITS) return decode_small(src, n, dst, mode, l1, e1, s);
    if (used_direct) *used_direct = false;
    return decode_two_launches(src, n, dst, mode, d_len, d_err, s);
}

}  // namespace

// ================================================================ C-ABI ==
extern "C" {

int64_t b64_encode_ex(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, void *stream)
{
    int mode;
    int rc = b64i_parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    if (n == 0) return 0;
    if (!src || !dst) return b64i_fail(B64_BAD_ARG, "null buffer with n > 0");
    rc = b64i_enqueue_encode(src, n, dst, mode, (hipStream_t)stream);
    if (rc) return rc;
    return b64i_enc_len(n, mode);
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
    int rc = b64i_parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (!err_off) return b64i_fail(B64_BAD_ARG, "null err_off");
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    *err_off = -1;
    if (n == 0) return 0;
    if (!src || (!dst && b64_decoded_max_mode(n, alphabet & ~0xff) > 0))
        return b64i_fail(B64_BAD_ARG, "null buffer with n > 0");
    SyncSlot *sl;
    rc = sync_slot(&sl);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    volatile int64_t *const hv = sl->hc;
    hv[0] = VERDICT_UNSET;
    hv[1] = VERDICT_UNSET;
    bool direct = false;
    rc = decode_with_verdict(src, n, dst, mode, sl->d, sl->d + 1, s, sl->hc_dev, &direct);
    if (rc) return rc;
    int64_t len, err;
    if (direct) {  // the verdict lands in host memory: only the wait is left
        HIP_TRY(hipStreamSynchronize(s));
        len = hv[0];
        err = hv[1];
        if (len == VERDICT_UNSET || err == VERDICT_UNSET)
            return b64i_fail(B64_HIP_ERROR, "decode finished without a verdict in host memory");
    } else {
        HIP_TRY(hipMemcpyAsync(sl->h, sl->d, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        len = sl->h[0];
        err = sl->h[1];
    }
    if (len < 0) {
        *err_off = err;
        return b64i_fail(B64_INVALID_INPUT, "invalid base64 input at offset %lld", (long long)err);
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
    int rc = b64i_parse_mode(alphabet, &mode);
    if (rc) return rc;
    if (n < 0) return b64i_fail(B64_BAD_ARG, "negative length");
    if (!d_len || !d_err) return b64i_fail(B64_BAD_ARG, "null result slot");
    if (n > 0 && (!src || (!dst && b64_decoded_max_mode(n, alphabet & ~0xff) > 0)))
        return b64i_fail(B64_BAD_ARG, "null buffer with n > 0");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(k_slots_init, 1, 64, 0, s, d_len, d_err);
        LAUNCH_TRY();
        return B64_OK;
    }
    return decode_with_verdict(src, n, dst, mode, d_len, d_err, s);
}

int b64_set_single_tune(int dir, const b64_tune *t)
{
    if (dir != 0 && dir != 1) return b64i_fail(B64_BAD_ARG, "bad direction");
    if (!t) return b64i_fail(B64_BAD_ARG, "null tune");
    // every field is checked before any is applied
    if (t->block && (t->block < 64 || t->block > 1024 || (t->block & 63)))
        return b64i_fail(B64_BAD_ARG, "bad block");
    if (t->units_per_lane && t->units_per_lane != 1 && t->units_per_lane != 2 && t->units_per_lane != 4 &&
        t->units_per_lane != 8)
        return b64i_fail(B64_BAD_ARG, "units_per_lane must be 1, 2, 4 or 8");
    // grid: blocks per CU; -1 selects one workgroup per tile
    if (t->grid && (t->grid < -1 || t->grid > 4096))
        return b64i_fail(B64_BAD_ARG, "blocks per CU must be -1 or 1..4096");
    if (t->layout < 0 || t->layout > (dir == 0 ? 2 : 1))
        return b64i_fail(B64_BAD_ARG, "map must be 0 (LDS tables), 1 (register maps) or, for encode, 2 (pair table)");
    if (t->block) g_single[dir].block = t->block;
    if (t->units_per_lane) g_single[dir].upl = t->units_per_lane;
    if (t->grid) g_single[dir].blocks_per_cu = t->grid < 0 ? 0 : t->grid;
    g_single[dir].map = t->layout;
    return B64_OK;
}

}  // extern "C"
