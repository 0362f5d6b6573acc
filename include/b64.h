/*
 * b64hip: base64 encoding and validating decoding on AMD Instinct MI355X
 * (gfx950), behind a plain C ABI.
 *
 * Semantics follow Muła & Lemire, "Faster Base64 Encoding and Decoding using
 * AVX2 Instructions" (arXiv 1704.00605):
 *   - alphabet: Section 2, Table 1 (standard) and the base64url variant of
 *     Section 2 (62 -> '-', 63 -> '_');
 *   - encoding: Section 2, Algorithm 1, with one '=' per leftover byte;
 *   - decoding: Section 2, Algorithm 2, where characters outside the alphabet
 *     are rejected (Section 2, and the standard quoted in Appendix B).
 * Where the paper leaves decoding lenient, this library is strict:
 *   - '=' is accepted only as the last character, or as each of the last two
 *     characters, of an input whose length is a multiple of 4;
 *   - a length that is not a multiple of 4 is an error at offset n;
 *   - the reported offset is the smallest offending index;
 *   - non-zero leftover bits in the final quad are accepted unless the strict
 *     flag (Appendix A) is requested.
 *
 * Conventions for every entry point:
 *   - Buffers named src/dst/in_off/out_off/flags/out_len/err_off/workspace
 *     are DEVICE pointers on the current HIP device, owned by the caller.
 *     The library keeps no reference after the call's GPU work ends.
 *   - Pointers documented as "host" are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the NULL stream).
 *     Calls named *_ex/_async/_batch only enqueue work on that stream unless
 *     documented otherwise; results are valid once the stream reaches them.
 *   - src and dst must not overlap. Any alignment is accepted; 4-byte
 *     aligned src and dst take the fastest path.
 *   - Lengths and offsets are int64 (inputs above 2^32 bytes are supported).
 *   - Return codes: >= 0 success (a length where documented);
 *       B64_INVALID_INPUT (-1) decode found an invalid character or length;
 *       B64_BAD_ARG (-2) null pointer with n > 0, n < 0, bad alphabet, too
 *       small workspace, bad tuning values;
 *       B64_HIP_ERROR (-3) a HIP runtime call failed;
 *       B64_POOL_FULL (-4) a pool allocation found no free block (pools);
 *       B64_TIMEOUT (-5) the serving loop hit its time limit.
 *     b64_last_error() describes the most recent failure on this thread.
 *   - Entry points allocate no device memory, except:
 *       b64_decode / b64_decode_ex: on first use on a thread and device,
 *         a 64-byte result slot and two 16-byte pinned host buffers (one of
 *         them written by the decode kernel directly), then reused;
 *       b64_decode_ws: per thread and device, its verdict slots (once) and
 *         a workspace grown to the largest input seen;
 *       b64_graph_create_batch: a private capture stream and the graph;
 *       b64_server_run: per-stream staging buffers, freed before it returns.
 *     The asynchronous and batched calls take caller-owned workspaces;
 *     b64_decode_batch_noalloc uses a static device array instead, and the
 *     single-buffer decodes a static 32 KiB array of verdict cells.
 */
#ifndef B64HIP_H
#define B64HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define B64_OK 0
#define B64_INVALID_INPUT (-1)
#define B64_BAD_ARG (-2)
#define B64_HIP_ERROR (-3)
#define B64_POOL_FULL (-4)
#define B64_TIMEOUT (-5)

/* Alphabets (Section 2): Table 1, or base64url. */
#define B64_ALPHABET_STD 0
#define B64_ALPHABET_URL 1

/* Decode/encode mode bits, OR-ed into the `alphabet` argument of the *_ex,
 * *_async and batched entry points:
 *   B64_MODE_STRICT  Appendix A: the leftover bits of a padded final quad
 *                    must be zero; a violation is an error at the index of
 *                    the character holding them (n-3 for "==", n-2 for "=").
 *   B64_MODE_NOPAD   Section 2 (padding may be omitted when the size is
 *                    known): encode writes no '='; decode accepts lengths
 *                    with n mod 4 in {0, 2, 3}, treats '=' as invalid and
 *                    reports n mod 4 == 1 as an error at offset n. */
#define B64_MODE_STRICT 0x100
#define B64_MODE_NOPAD 0x200

/* Number of characters Algorithm 1 writes for n bytes: 4 * ceil(n / 3)
 * (or 4 * floor(n / 3) + {0, 2, 3} with B64_MODE_NOPAD via b64_encoded_len_mode).
 * Pure host function; returns B64_BAD_ARG for n < 0. */
int64_t b64_encoded_len(int64_t n);
int64_t b64_encoded_len_mode(int64_t n, int mode);

/* Output capacity a decode of m characters may need: 3 * floor(m / 4)
 * (+2 for the unpadded mode's trailing partial group). Pure host function. */
int64_t b64_decoded_max(int64_t m);
int64_t b64_decoded_max_mode(int64_t m, int mode);

/* Algorithm 1 (Section 2): encode src[0, n) into dst[0, 4 * ceil(n / 3)),
 * standard alphabet, padded. Runs on the NULL stream and waits for it.
 * Returns the number of characters written. Never fails on content. */
int64_t b64_encode(const uint8_t *src, int64_t n, uint8_t *dst);

/* Algorithm 2 (Section 2) with validation: decode src[0, n) into dst, whose
 * capacity must be b64_decoded_max(n). Standard alphabet. Runs on the NULL
 * stream and waits for it. Returns the decoded length and sets *err_off = -1
 * (err_off is a HOST pointer), or returns B64_INVALID_INPUT with *err_off =
 * the first offending index (n when only the length is wrong). The contents
 * of dst are unspecified after an error. */
int64_t b64_decode(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off);

/* As b64_encode with an alphabet (plus mode bits) and a stream. Only
 * enqueues work: returns the output length immediately. */
int64_t b64_encode_ex(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, void *stream);

/* As b64_decode with an alphabet (plus mode bits) and a stream. Enqueues the
 * decode on `stream`, then waits for that stream to read back the verdict.
 * err_off is a HOST pointer. */
int64_t b64_decode_ex(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off, int alphabet,
                      void *stream);

/* Non-blocking decode. d_len and d_err are DEVICE int64 slots that receive
 * (decoded length, -1) or (-1, first offending index) when the stream
 * reaches the end of the work. Returns B64_OK once enqueued, or an argument /
 * runtime error code.
 * Launches: one for inputs up to 32 MiB of text on a stream that holds a
 * verdict cell (the last workgroup to finish forms the verdict); without a
 * cell, one up to 262,160 characters (a single workgroup); two otherwise
 * (slot set-up, decode). Each device has 1,024 verdict cells, given
 * out to the first 1,024 distinct stream handles that decode on it and kept
 * for the life of the process. Streams being captured into a graph, the
 * per-thread default stream and streams of a device other than the current
 * one get none. A cell is reused only by later work on the same stream
 * handle: a stream destroyed while its decode still runs must not have its
 * handle reused for a decode before that work ends.
 * b64_decode and b64_decode_ex take the same path on their stream. */
int b64_decode_async(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, int64_t *d_len,
                     int64_t *d_err, void *stream);

/* ------------------------------------------------------------------------
 * Whitespace-tolerant decode (Appendix B: space 0x20, line feed 0x0A and
 * carriage return 0x0D are removed before decoding, as in MIME text broken
 * into lines). The result is that of b64_decode_ex on the stripped text,
 * with one difference: *err_off / *d_err is an index into the ORIGINAL
 * input (a length error of the stripped text is reported at n). Alphabet:
 * B64_ALPHABET_STD or B64_ALPHABET_URL, no mode bits (-2 otherwise).
 * n < 2^38. dst needs capacity 3 * floor(n / 4) (the stripped length is not
 * known in advance); no byte past the decoded length is written.
 * ------------------------------------------------------------------------ */

/* Device workspace (bytes) b64_decode_ws_async needs for n input bytes:
 * about n / 256 plus 64. */
int64_t b64_decode_ws_workspace_bytes(int64_t n);

/* Asynchronous form: enqueues the decode on `stream`; the verdict lands in
 * the device slots d_len (decoded length or -1) and d_err (-1 or the first
 * offending original index). `workspace` (device, caller-owned, at least
 * b64_decode_ws_workspace_bytes(n) bytes) must not be used by another call
 * until this one completes. Returns B64_OK once enqueued. */
int b64_decode_ws_async(const uint8_t *src, int64_t n, uint8_t *dst, int alphabet, int64_t *d_len,
                        int64_t *d_err, void *workspace, int64_t workspace_bytes, void *stream);

/* Synchronous form on `stream` (NULL: default stream), with a workspace the
 * library keeps per thread and device. Returns the decoded length, or
 * B64_INVALID_INPUT with *err_off (host) = first offending original index. */
int64_t b64_decode_ws(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *err_off, int alphabet,
                      void *stream);

/* ------------------------------------------------------------------------
 * Batched forms: N messages packed back to back. Message i is
 * src[in_off[i], in_off[i+1]); in_off has N+1 non-decreasing int64 entries
 * (in_off[0] may be > 0). Its output starts at dst + out_off[i].
 * flags (nullable -> all B64_ALPHABET_STD) holds one alphabet byte per
 * message: bit 0 selects the alphabet; B64_FLAG_STRICT / B64_FLAG_NOPAD set
 * the per-message mode (decode: strict / unpadded; encode: unpadded).
 * ------------------------------------------------------------------------ */
#define B64_FLAG_URL 0x01
#define B64_FLAG_STRICT 0x02
#define B64_FLAG_NOPAD 0x04

#define B64_DIR_ENCODE 0
#define B64_DIR_DECODE 1

/* Device exclusive scan of per-message output slots (computed in place in
 * out_off, no other memory): out_off[0] = 0 and
 * out_off[i+1] - out_off[i] = 4 * ceil(len_i / 3) (encode), or the decode
 * capacity 3 * floor(len_i / 4) (+ max(0, len_i mod 4 - 1) for an unpadded
 * message) rounded up to a multiple of 4, so that every slot keeps dst's
 * 4-byte alignment. out_off has N+1 entries. Enqueued on `stream`. */
int b64_batch_out_offsets(int dir, const int64_t *in_off, int64_t N, int64_t *out_off,
                          const uint8_t *flags, void *stream);

/* Host form of the slot layout, for message lengths h_len[0, N) and
 * per-message flags h_flags (nullable; both HOST arrays): h_need[i] (nullable)
 * receives the bytes the kernels may write for message i (its encoded length
 * in its mode, or its decode capacity), h_out_off (nullable, N+1 entries) the
 * same exclusive scan b64_batch_out_offsets computes on the device. Pure host
 * function; B64_BAD_ARG for a negative length. */
int b64_batch_slots(int dir, const int64_t *h_len, const uint8_t *h_flags, int64_t N, int64_t *h_need,
                    int64_t *h_out_off);

/* Launch shape of the persistent batched kernels. A zero field means "use
 * the default". block: threads per workgroup (64..1024, multiple of 64;
 * layout 2 runs 256); units_per_lane: 12-byte (encode) / 16-character
 * (decode) units each lane carries per step (1, 2, 4 or 8); grid: workgroups
 * of the launch (0 = 32 per compute unit for layouts 0 and 2, 8 for layout
 * 1); layout: how the flattened units of all messages are shared out -
 *   0  tiles of block * units_per_lane units, grid-stride over the batch
 *      (blocks in flight cover one dense window; a tile inside one message
 *      runs the single-buffer step) - best when large messages dominate;
 *   1  one contiguous range of 64-unit groups per wave, walked with a
 *      message cursor - best for many small and mid-size messages in gather
 *      batches;
 *   2  staged tiles of 256 * units_per_lane units, one workgroup each
 *      (grid-stride when grid is smaller than the tile count, which a caller
 *      that knows the lengths can pass exactly): the planning pass records
 *      where each tile's input starts, the workgroup reads the tile's input
 *      as aligned 16-byte chunks straight into LDS and each lane takes its
 *      unit from there at any alignment - best for many small and mid-size
 *      messages in packed batches. Packed batches only: gather batches with
 *      layout 2 run layout 1. Tiles past the first N + 4096 (more than the
 *      tile table holds) or starting more than 64 messages run a slower
 *      per-lane path.
 * The autotuner picks all four per device and message-size histogram. */
typedef struct b64_tune {
    int32_t block;
    int32_t units_per_lane;
    int32_t grid;
    int32_t layout;
} b64_tune;

/* Device workspace (bytes) the batched calls need for N messages: about
 * 24 N + 64 KiB (unit offsets, partial sums, and layout 2's tile table). */
int64_t b64_batch_workspace_bytes(int64_t N);

/* Encode N messages in one persistent launch (after a device planning pass
 * over the offsets). out_off must be the scan from b64_batch_out_offsets
 * (or any per-message slots at least that large, 4-byte aligned for speed).
 * out_len[i] receives the characters written for message i. workspace is a
 * device buffer of b64_batch_workspace_bytes(N) bytes. tune may be NULL.
 * Enqueued on `stream`. */
int b64_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                     const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                     void *workspace, int64_t workspace_bytes, const b64_tune *tune, void *stream);

/* Decode N messages in one persistent launch. Per message: out_len[i] is the
 * decoded length or -1; err_off[i] is -1 or the first offending index
 * RELATIVE TO THE MESSAGE START. out_off gives capacity slots (see
 * b64_batch_out_offsets). Enqueued on `stream`. */
int b64_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                     const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                     int64_t *err_off, void *workspace, int64_t workspace_bytes,
                     const b64_tune *tune, void *stream);

/* Largest batch b64_decode_batch_noalloc accepts. */
#define B64_NOALLOC_MAX_MESSAGES (1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * b64_decode_batch without a workspace argument. Its planning workspace is a
 * static device array of the library (about 24 MiB, held by every device the
 * library runs on until the process ends), so the call allocates nothing and
 * needs no workspace; it only enqueues kernels on `stream`. N is at most
 * B64_NOALLOC_MAX_MESSAGES (B64_BAD_ARG beyond, before any work). All calls
 * on one device share that array: calls whose GPU work overlaps on one device
 * (other streams, other threads) race and must be serialised by the caller.
 * Everything else, results included, as b64_decode_batch. */
int b64_decode_batch_noalloc(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                             const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                             int64_t *err_off, const b64_tune *tune, void *stream);

/* Gather forms: message i is src[in_begin[i], in_begin[i] + in_len[i]) with
 * in_begin / in_len DEVICE arrays of N entries (messages may overlap, be in
 * any order and at any alignment); everything else as in the packed forms. */
int b64_encode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, void *workspace, int64_t workspace_bytes,
                            const b64_tune *tune, void *stream);
int b64_decode_batch_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                            int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                            int64_t *out_len, int64_t *err_off, void *workspace,
                            int64_t workspace_bytes, const b64_tune *tune, void *stream);

/* ------------------------------------------------------------------------
 * HIP graphs of batched calls: the planning and codec kernels of one
 * b64_encode_batch / b64_decode_batch (dir) are captured once and replayed
 * with a single graph launch. Arguments as for the packed batched calls; the
 * graph keeps the pointers, so the buffers must outlive it. update re-captures
 * with new pointers / N and updates the instantiated graph in place (falling
 * back to a fresh instantiation when the kernel topology changed). The graph
 * contains kernel nodes only (no memset nodes).
 * ------------------------------------------------------------------------ */
typedef struct b64_graph b64_graph;
int b64_graph_create_batch(int dir, const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                           const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                           int64_t *err_off, void *workspace, int64_t workspace_bytes,
                           const b64_tune *tune, b64_graph **out);
int b64_graph_update_batch(b64_graph *g, const uint8_t *src, const int64_t *in_off, int64_t N,
                           uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                           int64_t *err_off, void *workspace, int64_t workspace_bytes,
                           const b64_tune *tune);
int b64_graph_launch(b64_graph *g, void *stream);
int b64_graph_destroy(b64_graph *g);

/* ------------------------------------------------------------------------
 * Device memory pool (buddy allocator). The pool is host-side bookkeeping of
 * offsets in [0, capacity); the caller maps them onto its own device
 * allocation. Blocks are powers of two times min_block (a power of two,
 * default 256) and aligned to their size; an allocation takes the lowest
 * free block of the smallest size that has one. b64_pool_alloc never blocks:
 * it returns B64_POOL_FULL when no block is free, which is what drives
 * admission in the serving loop. Thread-safe. The bookkeeping takes about
 * 1.25 bytes of host memory per minimum block (40 MiB for 8 GiB at 256 B).
 * ------------------------------------------------------------------------ */
typedef struct b64_pool b64_pool;
int b64_pool_create(int64_t capacity, int64_t min_block, b64_pool **out);
int b64_pool_alloc(b64_pool *p, int64_t bytes, int64_t *offset);
int b64_pool_free(b64_pool *p, int64_t offset);
int64_t b64_pool_free_bytes(b64_pool *p);
int64_t b64_pool_peak_bytes(b64_pool *p);
int b64_pool_destroy(b64_pool *p);

/* ------------------------------------------------------------------------
 * Continuous-batching serving loop. Request r arrives at t_arrival[r] *
 * time_scale seconds after the call starts (t_arrival non-decreasing); op[r]
 * is B64_DIR_ENCODE or B64_DIR_DECODE; its input is
 * enc_src / dec_src [in_begin[r], in_begin[r] + in_len[r]) (device banks of
 * enc_src_bytes / dec_src_bytes bytes; a request outside its bank, an unknown
 * op or decreasing arrival times make the call return B64_BAD_ARG before any
 * work) and flags[r] (nullable) its per-message flags. pool_base must hold
 * the pool's capacity. Arrived requests are admitted in
 * order when the pool can hold their output (4 * ceil(n / 3) bytes to
 * encode, 3 * floor(n / 4) + 2 to decode); otherwise admission waits for
 * completed requests to release memory. Admitted requests of one direction
 * are launched together (gather form of the batched kernels, host-built
 * plan) on one of `streams` streams when max_batch are ready, when the
 * oldest has waited tick_us, or when admission is blocked; batches on
 * different streams overlap on the GPU. Completion is detected by polling
 * one event per batch. Outputs: t_done[r] (seconds since the call started,
 * host clock), out_off[r] (pool offset of the output), out_len[r] and
 * err_off[r] (the single-buffer verdict). With capture != 0 outputs are not
 * released (so callers can read them afterwards). Blocks the calling thread
 * until every request completed, the pool cannot ever admit the next
 * request (B64_POOL_FULL) or max_seconds passed (B64_TIMEOUT); in-flight
 * work is always drained before returning.
 * ------------------------------------------------------------------------ */
typedef struct b64_server_cfg {
    int32_t max_batch;      /* requests per launch and direction */
    int32_t tick_us;        /* longest wait of an admitted request before its batch launches */
    int32_t streams;        /* batches in flight (1..16) */
    int32_t capture;        /* keep outputs allocated after completion */
    int32_t idle_sleep_us;  /* sleep when nothing is in flight or ready (0 = spin) */
    int32_t block, units_per_lane, grid;  /* batched kernel launch shape (0 = default) */
    int32_t layout;         /* batched work layout, as in b64_tune (1 suits serving mixes) */
    double time_scale;      /* arrival time multiplier (1 = real time, 0 = all at once) */
    double max_seconds;     /* wall-clock limit of the call (0 = 600) */
} b64_server_cfg;

typedef struct b64_server_stats {
    int64_t completed, batches, launched_requests, pool_waits, max_inflight_batches;
    int64_t bytes_in, bytes_out, peak_pool_bytes;
    double wall_s;
} b64_server_stats;

int b64_server_run(const b64_server_cfg *cfg, int64_t nreq, const double *t_arrival,
                   const uint8_t *op, const int64_t *in_begin, const int64_t *in_len,
                   const uint8_t *flags, const uint8_t *enc_src, int64_t enc_src_bytes,
                   const uint8_t *dec_src, int64_t dec_src_bytes, b64_pool *pool,
                   uint8_t *pool_base, double *t_done, int64_t *out_off, int64_t *out_len,
                   int64_t *err_off, b64_server_stats *stats);

/* Plain per-message form of the batched calls (the baseline the batched
 * kernels are measured against): one single-buffer launch per message, all on
 * `stream`. Offsets and flags are HOST arrays here; out_len / err_off are
 * DEVICE arrays (err_off unused for encode and may be NULL). b64_encode_each
 * copies the lengths from a host buffer of its own and waits for `stream`
 * before it returns; b64_decode_each returns once its work is enqueued. */
int b64_encode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len, void *stream);
int b64_decode_each(const uint8_t *src, const int64_t *h_in_off, int64_t N, uint8_t *dst,
                    const int64_t *h_out_off, const uint8_t *h_flags, int64_t *out_len,
                    int64_t *err_off, void *stream);

/* Launch shape of the single-buffer kernels for one direction (0 encode,
 * 1 decode): block size, units per lane (1, 2, 4 or 8) and, in the `grid`
 * field, workgroups per compute unit (1..4096, or -1 for one workgroup per
 * tile, the default); zero in these fields keeps the current value. The
 * `layout` field selects the character map and is always applied:
 *   0  LDS byte tables (64 entries to encode, 256 to decode; the default);
 *   1  register maps on v_perm_b32: the range offsets of Section 4.1
 *      (Tables 4 and 5) to encode, Algorithm 3's nibble bitsets and roll
 *      table (Section 4.2) to decode;
 *   2  (encode only) an LDS table of 4096 character pairs, one lookup per
 *      12 bits (worth it with a persistent grid, which amortises its 8 KiB
 *      fill).
 * Process-wide; meant for tuning sweeps. */
int b64_set_single_tune(int dir, const b64_tune *t);

/* Launch shape of the whitespace-tolerant decode (tuning): block 256, 512 or
 * 1024 threads; units_per_lane = 16-byte input chunks per lane per tile
 * (256: 1, 2, 4 or 8; 512: 1, 2 or 4; 1024: 1 or 2); other fields ignored;
 * zero fields keep the current value. Process-wide. */
int b64_set_ws_tune(const b64_tune *t);

/* Thread-local description of the last failure (never NULL). */
const char *b64_last_error(void);

/* Library/device information: number of compute units of the current device
 * (used to size persistent grids), or B64_HIP_ERROR. */
int b64_device_cus(void);

#ifdef __cplusplus
}
#endif

#endif /* B64HIP_H */
