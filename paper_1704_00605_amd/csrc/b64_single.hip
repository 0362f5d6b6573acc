// gfx950 kernels of the single-buffer codec and their C-ABI (include/b64.h).
//
//   k_enc_single  Algorithm 1 over one buffer: grid-stride over 12-byte
//                 units, one unit per lane, then the final partial unit.
//   k_dec_single  Algorithm 2 over one buffer: grid-stride over interior
//                 16-character units, then the final unit with the padding
//                 and length rules.
//   k_dec_final   verdict (length, -1) or (-1, first offending index).
//
// Decode errors: a lane whose unit holds a non-symbol computes the exact
// index; a wave ballot elects the first erring lane, which performs one
// atomicMin on the 64-bit error slot (Section 2: the decoder must report
// characters outside the alphabet; the smallest index is the one reported).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
// by one lane.
template <bool ALIGNED, int UPL, int MAP>
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
            enc_step<ALIGNED, UPL, false, MAP>(src, dst, t0 + threadIdx.x, blockDim.x, units, mc);
        else
            enc_step<ALIGNED, UPL, true, MAP>(src, dst, t0 + threadIdx.x, blockDim.x, units, mc);
    }
    const int r = (int)(n - 12 * units);
    if (r && blockIdx.x == 0 && threadIdx.x == 0)
        enc_tail(src + 12 * units, r, dst + 16 * units, tab, mode & M_NOPAD);
}

// Decode src[0, n), n >= 1. Interior units [0, L) with L = (n - 1) / 16 hold
// 16 characters that are all before the final one; unit L (1..16 characters)
// carries the padding and length rules. err_slot must hold ERR_NONE at
// launch; it ends holding the smallest offending index (or ERR_NONE). The
// lane of the final unit writes the decoded length to *len_slot when that
// unit is valid. k_dec_final turns the pair into the verdict.
template <bool ALIGNED, int UPL, int MAP>
__global__ __launch_bounds__(1024) void k_dec_single(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, int mode,
                                                     unsigned long long *err_slot, int64_t *len_slot)
{
    __shared__ uint32_t s_tab[64];
    lds_fill(s_tab, c_tab.dec[mode & M_URL], 256);
    __syncthreads();
    const uint8_t *tab = (const uint8_t *)s_tab;
    const MapCtx mc = map_ctx<MAP>(tab, nullptr, mode & M_URL, true);

    const int64_t L = (n - 1) / 16;
    const int64_t tile = (int64_t)blockDim.x * UPL;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < L; t0 += (int64_t)gridDim.x * tile) {
        if (t0 + tile <= L)
            dec_step<ALIGNED, UPL, false, MAP>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, err_slot);
        else
            dec_step<ALIGNED, UPL, true, MAP>(src, dst, t0 + threadIdx.x, blockDim.x, L, mc, err_slot);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int r = (int)(n - 16 * L);
        const int res = dec_tail(src + 16 * L, r, n, dst + 12 * L, tab, mode);
        if (res >= 0) atomicMin(err_slot, (unsigned long long)(16 * L + res));
        else *len_slot = 12 * L + (-1 - res);
    }
}

// Decode of a short input (at most SMALL_UNITS interior units) by one
// workgroup, verdict included, so that the whole call is one launch: the
// first offending index is kept in an LDS slot (unsigned atomicMin) and
// thread 0 writes (length, -1) or (-1, index) at the end.
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
    // kept only once every step succeeded (a failed step frees what it got)
    SyncSlot s;
    s.dev = dev;
    const unsigned long long init[4] = {ERR_NONE, 0ull, 0ull, 0ull};
    hipError_t e = hipMalloc((void **)&s.d, 64);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.h, 16, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemcpy(s.d, init, sizeof init, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
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
    int64_t cap = bpc ? (int64_t)cus * bpc : (int64_t)INT32_MAX;
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

template <bool A>
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

template <bool A>
void launch_dec_single(int upl, int map, int grid, int block, const uint8_t *src, int64_t n, uint8_t *dst,
                       int mode, unsigned long long *slot, int64_t *len_slot, hipStream_t s)
{
    if (map == 1) {
        B64_UPL_SWITCH(k_dec_single, A, 1, src, n, dst, mode, slot, len_slot);
    } else {
        B64_UPL_SWITCH(k_dec_single, A, 0, src, n, dst, mode, slot, len_slot);
    }
}
#undef B64_UPL_SWITCH

bool aligned4(const void *a, const void *b)
{
    return (((uintptr_t)a | (uintptr_t)b) & 3) == 0;
}

}  // namespace

int b64i_enqueue_encode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(0, n / 12, &block, &upl, &grid);
    if (rc) return rc;
    const int map = g_single[0].map.load();
    if (aligned4(src, dst)) launch_enc_single<true>(upl, map, grid, block, src, n, dst, mode, s);
    else launch_enc_single<false>(upl, map, grid, block, src, n, dst, mode, s);
    LAUNCH_TRY();
    return B64_OK;
}

// Enqueues the decode kernel of src[0, n) (n >= 1); the error slot must hold
// ERR_NONE. No verdict is formed here (see k_dec_final).
int b64i_enqueue_decode(const uint8_t *src, int64_t n, uint8_t *dst, int mode, unsigned long long *slot,
                        int64_t *len_slot, hipStream_t s)
{
    int block, upl, grid;
    int rc = single_grid(1, (n - 1) / 16, &block, &upl, &grid);
    if (rc) return rc;
    const int map = g_single[1].map.load();
    if (aligned4(src, dst)) launch_dec_single<true>(upl, map, grid, block, src, n, dst, mode, slot, len_slot, s);
    else launch_dec_single<false>(upl, map, grid, block, src, n, dst, mode, slot, len_slot, s);
    LAUNCH_TRY();
    return B64_OK;
}

// One-launch decode of a short input (n >= 1, at most SMALL_UNITS interior
// units) with its verdict written to d_len / d_err.
int b64i_enqueue_decode_small(const uint8_t *src, int64_t n, uint8_t *dst, int mode, int64_t *d_len,
                              int64_t *d_err, hipStream_t s)
{
    if (aligned4(src, dst))
        hipLaunchKernelGGL(k_dec_small<true>, 1, 1024, 0, s, src, n, dst, mode, d_len, d_err);
    else
        hipLaunchKernelGGL(k_dec_small<false>, 1, 1024, 0, s, src, n, dst, mode, d_len, d_err);
    LAUNCH_TRY();
    return B64_OK;
}

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
    if ((n - 1) / 16 <= SMALL_UNITS) {
        rc = b64i_enqueue_decode_small(src, n, dst, mode, (int64_t *)(sl->d + 2), (int64_t *)(sl->d + 3), s);
        if (rc) return rc;
    } else {
        rc = b64i_enqueue_decode(src, n, dst, mode, sl->d, (int64_t *)(sl->d + 1), s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_dec_final, 1, 64, 0, s, sl->d, (const int64_t *)(sl->d + 1), (int64_t *)(sl->d + 2),
                           (int64_t *)(sl->d + 3), 1);
        LAUNCH_TRY();
    }
    HIP_TRY(hipMemcpyAsync(sl->h, sl->d + 2, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t len = sl->h[0], err = sl->h[1];
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
    if (n > 0 && (n - 1) / 16 <= SMALL_UNITS) {
        rc = b64i_enqueue_decode_small(src, n, dst, mode, d_len, d_err, s);
        return rc;
    }
    hipLaunchKernelGGL(k_slots_init, 1, 64, 0, s, d_len, d_err, n == 0 ? 1 : 0);
    LAUNCH_TRY();
    if (n == 0) return B64_OK;
    rc = b64i_enqueue_decode(src, n, dst, mode, (unsigned long long *)d_err, d_len, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dec_final, 1, 64, 0, s, (unsigned long long *)d_err, d_len, d_len, d_err, 0);
    LAUNCH_TRY();
    return B64_OK;
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
