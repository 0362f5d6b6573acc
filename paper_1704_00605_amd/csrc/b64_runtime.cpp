// Runtime around the codec kernels: HIP-graph capture of batched calls, a
// buddy allocator for device memory pools, and the continuous-batching
// serving loop (see include/b64.h for the contracts).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "b64.h"
#include "b64_internal.hpp"

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return b64i_fail(B64_HIP_ERROR, "%s failed: %s", what, hipGetErrorString(e));
}

#define RT_TRY(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

}  // namespace

// ===================================================================== graphs
struct b64_graph {
    int dir = 0;
    hipStream_t cap = nullptr;  // private capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int capture_batch(b64_graph *g, int dir, const uint8_t *src, const int64_t *in_off, int64_t N,
                  uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                  int64_t *err_off, void *ws, int64_t ws_bytes, const b64_tune *tune, hipGraph_t *out)
{
    RT_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    int rc;
    if (dir == B64_DIR_ENCODE)
        rc = b64_encode_batch(src, in_off, N, dst, out_off, flags, out_len, ws, ws_bytes, tune, g->cap);
    else
        rc = b64_decode_batch(src, in_off, N, dst, out_off, flags, out_len, err_off, ws, ws_bytes, tune, g->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    if (rc != B64_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    *out = graph;
    return B64_OK;
}

}  // namespace

extern "C" {

int b64_graph_create_batch(int dir, const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                           const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                           int64_t *err_off, void *workspace, int64_t workspace_bytes,
                           const b64_tune *tune, b64_graph **out)
{
    if (!out) return b64i_fail(B64_BAD_ARG, "null graph handle");
    if (dir != B64_DIR_ENCODE && dir != B64_DIR_DECODE) return b64i_fail(B64_BAD_ARG, "bad direction");
    if (N <= 0) return b64i_fail(B64_BAD_ARG, "a graph needs at least one message");
    auto *g = new b64_graph();
    g->dir = dir;
    hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    int rc = capture_batch(g, dir, src, in_off, N, dst, out_off, flags, out_len, err_off, workspace,
                           workspace_bytes, tune, &g->graph);
    if (rc == B64_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (rc != B64_OK) {
        b64_graph_destroy(g);
        return rc;
    }
    *out = g;
    return B64_OK;
}

int b64_graph_update_batch(b64_graph *g, const uint8_t *src, const int64_t *in_off, int64_t N,
                           uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                           int64_t *err_off, void *workspace, int64_t workspace_bytes,
                           const b64_tune *tune)
{
    if (!g || !g->exec) return b64i_fail(B64_BAD_ARG, "null graph");
    if (N <= 0) return b64i_fail(B64_BAD_ARG, "a graph needs at least one message");
    hipGraph_t graph = nullptr;
    int rc = capture_batch(g, g->dir, src, in_off, N, dst, out_off, flags, out_len, err_off, workspace,
                           workspace_bytes, tune, &graph);
    if (rc != B64_OK) return rc;
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    hipError_t e = hipGraphExecUpdate(g->exec, graph, &err_node, &res);
    if (e != hipSuccess || res != hipGraphExecUpdateSuccess) {
        // topology changed (e.g. a different number of planning chunks)
        (void)hipGetLastError();
        hipGraphExec_t fresh = nullptr;
        e = hipGraphInstantiate(&fresh, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        (void)hipGraphExecDestroy(g->exec);
        g->exec = fresh;
    }
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->graph = graph;
    return B64_OK;
}

int b64_graph_launch(b64_graph *g, void *stream)
{
    if (!g || !g->exec) return b64i_fail(B64_BAD_ARG, "null graph");
    RT_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return B64_OK;
}

int b64_graph_destroy(b64_graph *g)
{
    if (!g) return B64_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
    return B64_OK;
}

}  // extern "C"

// ======================================================================= pool
// Buddy allocator over [0, capacity): the capacity (rounded down to the
// minimum block) is split into power-of-two top blocks in descending size,
// so every block is aligned to its own size and its buddy is offset ^ size.
// An allocation takes the lowest free block of the smallest level that has
// one. Bookkeeping is O(1) per level: for each level a bit tree of its free
// blocks (leaf bits plus summary words, so the lowest free block is a few
// find-first-set steps away) and a count; for every minimum block a byte
// with the level + 1 of the live block that starts there. Tree containers
// had cost about 340 ns per allocation and release, which capped the
// serving loop near 3 million requests per second.
namespace {

// Set of indexes [0, n) with O(log64 n) insert, erase and lowest member.
struct BitTree {
    std::vector<std::vector<uint64_t>> lv;  // lv[0]: members; lv[i + 1]: non-zero words of lv[i]

    void init(int64_t n)
    {
        lv.clear();
        int64_t bits = n;
        do {
            const int64_t words = (bits + 63) / 64;
            lv.emplace_back((size_t)words, 0ull);
            bits = words;
        } while (bits > 1);
    }
    bool test(int64_t i) const { return (lv[0][(size_t)(i >> 6)] >> (i & 63)) & 1; }
    void insert(int64_t i)
    {
        for (auto &w : lv) {
            const bool was = w[(size_t)(i >> 6)] != 0;
            w[(size_t)(i >> 6)] |= 1ull << (i & 63);
            if (was) return;  // the summaries above already mark this word
            i >>= 6;
        }
    }
    void erase(int64_t i)
    {
        for (auto &w : lv) {
            w[(size_t)(i >> 6)] &= ~(1ull << (i & 63));
            if (w[(size_t)(i >> 6)] != 0) return;  // the word still has members
            i >>= 6;
        }
    }
    int64_t lowest() const  // -1 when empty
    {
        if (lv.back()[0] == 0) return -1;
        int64_t i = 0;
        for (size_t l = lv.size(); l-- > 0;) i = i * 64 + __builtin_ctzll(lv[l][(size_t)i]);
        return i;
    }
};

}  // namespace

struct b64_pool {
    std::mutex mu;
    int64_t minb = 256;
    int lgminb = 8;
    int64_t capacity = 0;
    int64_t used = 0;
    int64_t peak = 0;
    int maxk = 0;
    std::vector<BitTree> free_k;              // k -> free blocks of size minb << k (index = offset >> (lgminb + k))
    std::vector<int64_t> nfree;               // k -> number of free blocks
    std::vector<uint8_t> live;                // minimum block index -> 1 + level of the live block starting there, or 0
    std::vector<std::pair<int64_t, int>> tops;  // (offset, k) of top blocks
};

namespace {

int ceil_log2(int64_t x)
{
    int k = 0;
    while (((int64_t)1 << k) < x) k++;
    return k;
}

int top_k_of(const b64_pool *p, int64_t off)
{
    for (const auto &t : p->tops)
        if (off >= t.first && off < t.first + (p->minb << t.second)) return t.second;
    return -1;
}

void pool_put(b64_pool *p, int k, int64_t off)
{
    p->free_k[k].insert(off >> (p->lgminb + k));
    p->nfree[k]++;
}

void pool_take(b64_pool *p, int k, int64_t off)
{
    p->free_k[k].erase(off >> (p->lgminb + k));
    p->nfree[k]--;
}

}  // namespace

extern "C" {

int b64_pool_create(int64_t capacity, int64_t min_block, b64_pool **out)
{
    if (!out || capacity <= 0) return b64i_fail(B64_BAD_ARG, "bad pool capacity");
    if (min_block <= 0) min_block = 256;
    if (min_block & (min_block - 1)) return b64i_fail(B64_BAD_ARG, "min_block must be a power of two");
    int64_t units = capacity / min_block;
    if (units <= 0) return b64i_fail(B64_BAD_ARG, "pool capacity below one block");
    auto *p = new b64_pool();
    p->minb = min_block;
    p->lgminb = ceil_log2(min_block);
    p->capacity = units * min_block;
    p->maxk = 0;
    while (((int64_t)1 << (p->maxk + 1)) <= units) p->maxk++;
    p->free_k.resize(p->maxk + 1);
    p->nfree.assign(p->maxk + 1, 0);
    for (int k = 0; k <= p->maxk; k++) p->free_k[k].init((units >> k) + 1);
    p->live.assign((size_t)units, 0);
    int64_t off = 0;
    for (int k = p->maxk; k >= 0; k--) {
        if (units & ((int64_t)1 << k)) {
            p->tops.push_back({off, k});
            pool_put(p, k, off);
            off += min_block << k;
        }
    }
    *out = p;
    return B64_OK;
}

int b64_pool_alloc(b64_pool *p, int64_t bytes, int64_t *offset)
{
    if (!p || !offset || bytes < 0) return b64i_fail(B64_BAD_ARG, "bad pool allocation");
    if (bytes == 0) bytes = 1;
    if (bytes > p->capacity) return B64_POOL_FULL;
    const int k = ceil_log2((bytes + p->minb - 1) / p->minb);
    std::lock_guard<std::mutex> lk(p->mu);
    if (k > p->maxk) return B64_POOL_FULL;
    int j = k;
    while (j <= p->maxk && p->nfree[j] == 0) j++;
    if (j > p->maxk) return B64_POOL_FULL;
    const int64_t off = p->free_k[j].lowest() << (p->lgminb + j);
    pool_take(p, j, off);
    while (j > k) {  // split, keep the lower half
        j--;
        pool_put(p, j, off + (p->minb << j));
    }
    p->live[(size_t)(off >> p->lgminb)] = (uint8_t)(k + 1);
    p->used += p->minb << k;
    p->peak = std::max(p->peak, p->used);
    *offset = off;
    return B64_OK;
}

int b64_pool_free(b64_pool *p, int64_t offset)
{
    if (!p) return b64i_fail(B64_BAD_ARG, "null pool");
    std::lock_guard<std::mutex> lk(p->mu);
    if (offset < 0 || offset >= p->capacity || (offset & (p->minb - 1)) || p->live[(size_t)(offset >> p->lgminb)] == 0)
        return b64i_fail(B64_BAD_ARG, "offset is not a live pool block");
    int k = p->live[(size_t)(offset >> p->lgminb)] - 1;
    p->live[(size_t)(offset >> p->lgminb)] = 0;
    p->used -= p->minb << k;
    const int topk = top_k_of(p, offset);
    int64_t off = offset;
    while (k < topk) {  // merge with a free buddy
        const int64_t buddy = off ^ (p->minb << k);
        if (!p->free_k[k].test(buddy >> (p->lgminb + k))) break;
        pool_take(p, k, buddy);
        off = std::min(off, buddy);
        k++;
    }
    pool_put(p, k, off);
    return B64_OK;
}

int64_t b64_pool_free_bytes(b64_pool *p)
{
    if (!p) return b64i_fail(B64_BAD_ARG, "null pool");
    std::lock_guard<std::mutex> lk(p->mu);
    return p->capacity - p->used;
}

int64_t b64_pool_peak_bytes(b64_pool *p)
{
    if (!p) return b64i_fail(B64_BAD_ARG, "null pool");
    std::lock_guard<std::mutex> lk(p->mu);
    return p->peak;
}

int b64_pool_destroy(b64_pool *p)
{
    delete p;
    return B64_OK;
}

}  // extern "C"

// ==================================================================== serving
namespace {

using Clock = std::chrono::steady_clock;

// One in-flight batch slot: its stream, completion event, pinned staging for
// the descriptors it uploads and the verdicts it reads back, and the device
// copy of the descriptors.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int64_t *h = nullptr;   // pinned: descriptors then verdicts
    int64_t *d = nullptr;   // device: descriptors + verdict slots
    bool busy = false;
    int dir = 0;
    std::vector<int64_t> reqs;
};

// Layout (int64 words) of the descriptor block of a batch of n messages,
// packed so that one upload moves exactly what the batch needs:
// in_begin[n] | in_len[n] | out_off[n] | unit_off[n+1] | out_len[n] | err_off[n] | flags (n bytes)
struct Layout {
    int64_t n;
    int64_t in_begin() const { return 0; }
    int64_t in_len() const { return n; }
    int64_t out_off() const { return 2 * n; }
    int64_t unit_off() const { return 3 * n; }
    int64_t out_len() const { return 4 * n + 1; }
    int64_t err_off() const { return 5 * n + 1; }
    int64_t flags() const { return 6 * n + 1; }
    int64_t words() const { return 6 * n + 1 + (n + 7) / 8; }
};

struct Ready {
    int64_t req;
    double t_admit;
};

}  // namespace

extern "C" int b64_server_run(const b64_server_cfg *cfg, int64_t nreq, const double *t_arrival,
                              const uint8_t *op, const int64_t *in_begin, const int64_t *in_len,
                              const uint8_t *flags, const uint8_t *enc_src, int64_t enc_src_bytes,
                              const uint8_t *dec_src, int64_t dec_src_bytes, b64_pool *pool,
                              uint8_t *pool_base, double *t_done, int64_t *out_off, int64_t *out_len,
                              int64_t *err_off, b64_server_stats *stats)
{
    if (!cfg || nreq < 0 || !t_arrival || !op || !in_begin || !in_len || !pool || !pool_base ||
        !t_done || !out_off || !out_len || !err_off)
        return b64i_fail(B64_BAD_ARG, "null server argument");
    // every request must read inside its bank
    for (int64_t r = 0; r < nreq; r++) {
        const int64_t lim = op[r] == B64_DIR_ENCODE ? enc_src_bytes : dec_src_bytes;
        const uint8_t *bank = op[r] == B64_DIR_ENCODE ? enc_src : dec_src;
        if ((op[r] != B64_DIR_ENCODE && op[r] != B64_DIR_DECODE) || in_begin[r] < 0 || in_len[r] < 0 ||
            in_begin[r] > lim - in_len[r] || (in_len[r] > 0 && !bank) || (r && t_arrival[r] < t_arrival[r - 1]))
            return b64i_fail(B64_BAD_ARG, "request outside its bank, bad op or unsorted arrivals");
    }
    if (cfg->max_batch < 1 || cfg->streams < 1 || cfg->streams > 16 || cfg->tick_us < 0 ||
        (cfg->layout != 0 && cfg->layout != 1))
        return b64i_fail(B64_BAD_ARG, "bad server configuration");
    const int64_t B = cfg->max_batch;
    const Layout LB{B};  // largest batch: sizes the slot buffers
    const double max_s = cfg->max_seconds > 0 ? cfg->max_seconds : 600.0;
    const double tick = cfg->tick_us * 1e-6;
    b64_tune tune{cfg->block, cfg->units_per_lane, cfg->grid, cfg->layout};

    const int cus = b64_device_cus();
    if (cus <= 0) return cus < 0 ? cus : b64i_fail(B64_HIP_ERROR, "no compute units");
    std::vector<Slot> slots(cfg->streams);
    auto cleanup = [&]() {
        for (auto &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.h) (void)hipHostFree(s.h);
            if (s.d) (void)hipFree(s.d);
        }
    };
    for (auto &s : slots) {
        hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.h, 8 * LB.words(), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&s.d, 8 * LB.words());
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "server slot setup");
        }
    }
    for (int64_t r = 0; r < nreq; r++) {
        t_done[r] = -1.0;
        out_off[r] = -1;
        out_len[r] = -1;
        err_off[r] = -1;
    }
    b64_server_stats st{};
    std::deque<Ready> ready[2];
    int64_t next = 0, completed = 0;
    const auto t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    const double scale = cfg->time_scale;
    int rc = B64_OK;

    auto out_cap = [&](int64_t r) -> int64_t {
        const int64_t n = in_len[r];
        return op[r] == B64_DIR_ENCODE ? 4 * ((n + 2) / 3) : 3 * (n / 4) + 2;
    };

    auto launch_batch = [&](Slot &s, int dir, double t) -> int {
        auto &q = ready[dir];
        const int64_t n = std::min<int64_t>(B, (int64_t)q.size());
        const Layout L{n};
        s.reqs.clear();
        int64_t *h = s.h;
        int64_t u = 0;
        uint8_t *hf = (uint8_t *)(h + L.flags());
        for (int64_t i = 0; i < n; i++) {
            const int64_t r = q.front().req;
            q.pop_front();
            s.reqs.push_back(r);
            h[L.in_begin() + i] = in_begin[r];
            h[L.in_len() + i] = in_len[r];
            h[L.out_off() + i] = out_off[r];
            h[L.unit_off() + i] = u;
            u += dir == B64_DIR_ENCODE ? (in_len[r] + 11) / 12 : (in_len[r] + 15) / 16;
            h[L.out_len() + i] = 0;
            h[L.err_off() + i] = -1;
            hf[i] = flags ? flags[r] : 0;
        }
        h[L.unit_off() + n] = u;
        // grid sized from the batch (a configured grid wins): per-wave ranges
        // take about 4 groups of 64 units per wave, at most 8 workgroups per
        // CU; tiles take one workgroup per tile, at most 32 per CU
        b64_tune bt = tune;
        if (!cfg->grid) {
            int64_t want;
            if (bt.layout == 1) {
                const int64_t block = bt.block ? bt.block : 256;
                want = std::min<int64_t>(((u + 63) / 64 + 4 * (block / 64) - 1) / (4 * (block / 64)), 8 * cus);
            } else {
                const int64_t tile = (int64_t)(bt.block ? bt.block : 512) * (bt.units_per_lane ? bt.units_per_lane : 2);
                want = std::min<int64_t>((u + tile - 1) / tile, 32 * cus);
            }
            bt.grid = (int32_t)std::max<int64_t>(1, want);
        }
        int64_t *d = s.d;
        hipError_t e = hipMemcpyAsync(d, h, 8 * L.words(), hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        const uint8_t *df = (const uint8_t *)(d + L.flags());
        int r2;
        if (dir == B64_DIR_ENCODE)
            r2 = b64i_encode_planned(enc_src, d + L.in_begin(), d + L.in_len(), n, pool_base, d + L.out_off(),
                                     df, d + L.unit_off(), &bt, s.stream);
        else
            r2 = b64i_decode_planned(dec_src, d + L.in_begin(), d + L.in_len(), n, pool_base, d + L.out_off(),
                                     df, d + L.unit_off(), d + L.out_len(), d + L.err_off(), &bt, s.stream);
        if (r2 != B64_OK) return r2;
        if (dir == B64_DIR_DECODE) {
            e = hipMemcpyAsync(h + L.out_len(), d + L.out_len(), 16 * n, hipMemcpyDeviceToHost, s.stream);
            if (e != hipSuccess) return hip_fail(e, "verdict readback");
        }
        e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        s.busy = true;
        s.dir = dir;
        st.batches++;
        st.launched_requests += n;
        (void)t;
        return B64_OK;
    };
    // roctx ranges mark the three phases of the loop for a trace
    auto launch = [&](Slot &s, int dir, double t) -> int {
        roctxRangePushA(dir == B64_DIR_ENCODE ? "b64 serve: launch encode batch" : "b64 serve: launch decode batch");
        const int lrc = launch_batch(s, dir, t);
        roctxRangePop();
        return lrc;
    };

    while (completed < nreq) {
        const double t = now_s();
        if (t > max_s) {
            rc = b64i_fail(B64_TIMEOUT, "serving loop exceeded its time limit");
            break;
        }
        // 1. completions
        int inflight = 0;
        for (auto &s : slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) { inflight++; continue; }
            if (q != hipSuccess) { rc = hip_fail(q, "hipEventQuery"); break; }
            roctxRangePushA("b64 serve: complete batch");
            const double td = now_s();
            const Layout L{(int64_t)s.reqs.size()};
            for (size_t i = 0; i < s.reqs.size(); i++) {
                const int64_t r = s.reqs[i];
                t_done[r] = td;
                if (s.dir == B64_DIR_ENCODE) {
                    const int nopad = flags ? (flags[r] & B64_FLAG_NOPAD) : 0;
                    const int64_t n = in_len[r];
                    out_len[r] = nopad ? 4 * (n / 3) + ((n % 3) ? (n % 3) + 1 : 0) : 4 * ((n + 2) / 3);
                    err_off[r] = -1;
                } else {
                    out_len[r] = s.h[L.out_len() + i];
                    err_off[r] = s.h[L.err_off() + i];
                }
                if (!cfg->capture) b64_pool_free(pool, out_off[r]);
                st.bytes_in += in_len[r];
                st.bytes_out += out_len[r] > 0 ? out_len[r] : 0;
            }
            completed += (int64_t)s.reqs.size();
            s.busy = false;
            s.reqs.clear();
            roctxRangePop();
        }
        if (rc != B64_OK) break;
        st.max_inflight_batches = std::max<int64_t>(st.max_inflight_batches, inflight);
        // 2. admission in arrival order, by free pool memory
        bool blocked = false;
        const bool admitting = next < nreq && t_arrival[next] * scale <= t;
        if (admitting) roctxRangePushA("b64 serve: admit");
        while (next < nreq && t_arrival[next] * scale <= t) {
            int64_t off;
            const int64_t cap = out_cap(next);
            int a = b64_pool_alloc(pool, cap, &off);
            if (a == B64_POOL_FULL) {
                blocked = true;
                st.pool_waits++;
                break;
            }
            if (a != B64_OK) { rc = a; break; }
            out_off[next] = off;
            ready[op[next] == B64_DIR_ENCODE ? 0 : 1].push_back({next, t});
            next++;
        }
        if (admitting) roctxRangePop();
        if (rc != B64_OK) break;
        // 3. launch batches on free slots
        const bool arrivals_done = next >= nreq;
        for (int dir = 0; dir < 2; dir++) {
            while (!ready[dir].empty()) {
                const bool full = (int64_t)ready[dir].size() >= B;
                const bool due = t - ready[dir].front().t_admit >= tick;
                if (!(full || due || arrivals_done || blocked)) break;
                Slot *free_slot = nullptr;
                for (auto &s : slots)
                    if (!s.busy) { free_slot = &s; break; }
                if (!free_slot) break;
                rc = launch(*free_slot, dir, t);
                if (rc != B64_OK) break;
            }
            if (rc != B64_OK) break;
        }
        if (rc != B64_OK) break;
        // a request larger than the whole pool, or a full pool with nothing in
        // flight to release memory, can never be admitted
        if (blocked && ready[0].empty() && ready[1].empty()) {
            bool any_busy = false;
            for (auto &s : slots) any_busy |= s.busy;
            if (!any_busy) {
                rc = b64i_fail(B64_POOL_FULL, "request does not fit in the pool and nothing is in flight");
                break;
            }
        }
        if (cfg->idle_sleep_us > 0 && next < nreq && t_arrival[next] * scale > t) {
            bool any_busy = false;
            for (auto &s : slots) any_busy |= s.busy;
            if (!any_busy && ready[0].empty() && ready[1].empty())
                std::this_thread::sleep_for(std::chrono::microseconds(cfg->idle_sleep_us));
        }
    }
    st.wall_s = now_s();
    st.peak_pool_bytes = b64_pool_peak_bytes(pool);
    st.completed = completed;
    cleanup();
    if (stats) *stats = st;
    return rc;
}
