/*
 * Plain scalar base64 codec: the ORACLE.
 *
 * This file is test infrastructure. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it. It shares no code, table or
 * header with the GPU library; it is written from Muła & Lemire, "Faster
 * Base64 Encoding and Decoding using AVX2 Instructions" (arXiv 1704.00605):
 *
 *   - Section 2, Table 1: the 64-symbol alphabet B (value -> character).
 *   - Section 2, base64url paragraph: values 62 and 63 become '-' and '_'.
 *   - Section 2, Algorithm 1: encoding, one '=' per leftover byte.
 *   - Section 2, Algorithm 2: decoding 4 characters into 3 bytes.
 *   - Appendix B (quoted standard): characters outside the alphabet are
 *     rejected.
 *
 * Readings where the paper is silent or lenient (each is also listed in the
 * design notes of the repository):
 *   R1  '=' is not one of the 64 symbols (Table 1 caption). It is accepted only
 *       as the last character, or as each of the last two characters, of an
 *       input whose length is a multiple of 4. Anywhere else it is an invalid
 *       character at its own index (Algorithm 2 would stop silently at a '='
 *       in the middle of the stream; the strict reading rejects it).
 *   R2  A length that is not a multiple of 4 (the REQUIRE of Algorithm 2) is an
 *       error at offset n, unless an invalid character comes earlier.
 *   R3  When several characters are invalid, the smallest index is reported.
 *   R4  Non-zero leftover bits in the final quad are accepted (Appendix A says
 *       the standard does not require that check); the strict check is a
 *       separate function.
 *   R5  Each alphabet accepts only its own 64 symbols.
 *
 * Every routine here is a direct, unoptimised restatement of a definition:
 * per-group and per-character loops over 24-bit group values and their 6-bit
 * fields, with no blocking or table tricks.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_STD 0
#define ORACLE_URL 1

/* Table 1: 6-bit value v -> ASCII character, standard alphabet. */
static const char TABLE1[65] =
    "ABCDEFGHIJKLMNOPQRSTUVWXYZ"  /* 0..25  */
    "abcdefghijklmnopqrstuvwxyz"  /* 26..51 */
    "0123456789"                  /* 52..61 */
    "+/";                         /* 62, 63 */

/* The function B of Algorithm 1 for the chosen alphabet (Table 1; base64url
 * replaces 62 by '-' and 63 by '_'). */
static uint8_t oracle_B(int alphabet, unsigned v)
{
    if (alphabet == ORACLE_URL) {
        if (v == 62) return (uint8_t)'-';
        if (v == 63) return (uint8_t)'_';
    }
    return (uint8_t)TABLE1[v];
}

/* The function A of Algorithm 2 as the inverse of B: inv[ch] = v when
 * B(v) == ch, else -1. '=' is not a symbol and maps to -1 here; the padding
 * rule (R1) is applied by the decoder itself. */
static void oracle_build_A(int alphabet, int inv[256])
{
    for (int ch = 0; ch < 256; ch++) inv[ch] = -1;
    for (unsigned v = 0; v < 64; v++) inv[oracle_B(alphabet, v)] = (int)v;
}

int oracle_alphabet_ok(int alphabet) { return alphabet == ORACLE_STD || alphabet == ORACLE_URL; }

/* Exposes B and A so the tests can compare them with Tables 1, 4, 5 and 6. */
int oracle_symbol(int alphabet, int v) { return (v < 0 || v > 63) ? -1 : oracle_B(alphabet, (unsigned)v); }
int oracle_value(int alphabet, int ch)
{
    int inv[256];
    if (ch < 0 || ch > 255) return -1;
    oracle_build_A(alphabet, inv);
    return inv[ch];
}

int64_t oracle_encoded_len(int64_t n) { return n <= 0 ? 0 : 4 * ((n + 2) / 3); }

/* Encoding (Section 2, Algorithm 1). Every group of three bytes, read most
 * significant first, is one 24-bit number; its four 6-bit fields, from the
 * top, are mapped through B. A final group of r = n mod 3 bytes (1 or 2) is
 * read as a 24-bit number whose missing low bytes are zero: its first r + 1
 * fields are mapped through B and the remaining 3 - r characters are '=',
 * so the output always has 4 * ceil(n / 3) characters. Returns that number. */
static uint32_t oracle_group(const uint8_t *s, int64_t avail)
{
    uint32_t v = 0;
    for (int k = 0; k < 3; k++) v = (v << 8) | (k < avail ? s[k] : 0u);
    return v;
}

static unsigned oracle_field(uint32_t v, int k) { return (v >> (18 - 6 * k)) & 63u; }

int64_t oracle_encode(const uint8_t *s, int64_t n, uint8_t *p, int alphabet)
{
    int64_t o = 0;
    for (int64_t g = 0; g < n; g += 3) {
        const int64_t avail = n - g < 3 ? n - g : 3;
        const uint32_t v = oracle_group(s + g, avail);
        for (int k = 0; k < 4; k++) p[o++] = k <= avail ? oracle_B(alphabet, oracle_field(v, k)) : (uint8_t)'=';
    }
    return o;
}

/* R1: is character i of c[0..n) acceptable? */
static int oracle_char_ok(const uint8_t *c, int64_t n, int64_t i, const int inv[256])
{
    if (inv[c[i]] >= 0) return 1;
    if (c[i] != '=' || n % 4 != 0) return 0;
    if (i == n - 1) return 1;
    if (i == n - 2 && c[n - 1] == '=') return 1;
    return 0;
}

/* First index in [begin, end) that fails R1, or -1. */
static int64_t oracle_first_bad(const uint8_t *c, int64_t n, int64_t begin, int64_t end,
                                const int inv[256])
{
    for (int64_t i = begin; i < end; i++)
        if (!oracle_char_ok(c, n, i, inv)) return i;
    return -1;
}

/* Decoding of a validated text (Section 2, Algorithm 2): each quad of
 * characters is one 24-bit number, the values of its four characters placed
 * from the top in 6-bit fields ('=' counts as 0), and its three bytes, most
 * significant first, are the output. Quads start at qbegin, qbegin + 4, ...
 * below qend. Writes all three bytes of every quad and returns their number;
 * the caller drops one byte per trailing '='. */
static int64_t oracle_decode_quads(const uint8_t *c, int64_t qbegin, int64_t qend, uint8_t *p,
                                   const int inv[256])
{
    int64_t o = 0;
    for (int64_t i = qbegin; i < qend; i += 4) {
        uint32_t v = 0;
        for (int k = 0; k < 4; k++) v = (v << 6) | (c[i + k] == '=' ? 0u : (uint32_t)inv[c[i + k]]);
        for (int k = 0; k < 3; k++) p[o++] = (uint8_t)(v >> (16 - 8 * k));
    }
    return o;
}

/* Number of '=' ending c[0..n) (0, 1 or 2 for a validated text). */
static int64_t oracle_pads(const uint8_t *c, int64_t n)
{
    int64_t k = 0;
    while (k < 2 && k < n && c[n - 1 - k] == '=') k++;
    return k;
}

int64_t oracle_decoded_max(int64_t m) { return m <= 0 ? 0 : 3 * (m / 4); }

/* Validating decode. Returns the decoded length, or -1 with *err_off set to
 * the first offending index (R1-R3). *err_off is -1 on success. The contents
 * of p are unspecified on error. */
int64_t oracle_decode(const uint8_t *c, int64_t n, uint8_t *p, int alphabet, int64_t *err_off)
{
    int inv[256];
    int64_t bad;
    *err_off = -1;
    if (n <= 0) return 0;
    oracle_build_A(alphabet, inv);
    bad = oracle_first_bad(c, n, 0, n, inv);
    if (bad < 0 && n % 4 != 0) bad = n;
    if (bad >= 0) {
        *err_off = bad;
        return -1;
    }
    return oracle_decode_quads(c, 0, n, p, inv) - oracle_pads(c, n);
}

/* Appendix A: additional checks on the last quad. A padded final quad
 * carries bits that fall into the bytes its '=' characters drop: the low four
 * bits of the value of C[n-3] when it ends in "==", the low two bits of the
 * value of C[n-2] when it ends in one '='. They must be zero; otherwise the
 * error is reported at that character's index. Applied after oracle_decode
 * succeeds. */
int64_t oracle_decode_strict(const uint8_t *c, int64_t n, uint8_t *p, int alphabet, int64_t *err_off)
{
    int inv[256];
    int64_t len = oracle_decode(c, n, p, alphabet, err_off), pads;
    if (len < 0 || n == 0) return len;
    oracle_build_A(alphabet, inv);
    pads = oracle_pads(c, n);
    if (pads == 2 && (inv[c[n - 3]] & 15) != 0) { *err_off = n - 3; return -1; }
    if (pads == 1 && (inv[c[n - 2]] & 3) != 0) { *err_off = n - 2; return -1; }
    return len;
}

/* Section 2: padding may be omitted when the size is known. Unpadded encode:
 * Algorithm 1 without the '=' characters (2 or 3 characters for the last
 * group). */
int64_t oracle_encode_nopad(const uint8_t *s, int64_t n, uint8_t *p, int alphabet)
{
    int64_t len = oracle_encode(s, n, p, alphabet);
    while (len > 0 && p[len - 1] == '=') len--;
    return len;
}

/* Unpadded decode: the input is the padded form with its '=' removed, so its
 * length mod 4 is 0, 2 or 3; 1 is an error at offset n. '=' is invalid
 * everywhere. A trailing group of r = n mod 4 characters (2 or 3) is read as
 * a quad whose missing characters are 0, and its first r - 1 bytes are the
 * output, as for a padded final quad. */
int64_t oracle_decode_nopad(const uint8_t *c, int64_t n, uint8_t *p, int alphabet, int64_t *err_off)
{
    int inv[256];
    int64_t bad = -1, full, o, r;
    *err_off = -1;
    if (n <= 0) return 0;
    oracle_build_A(alphabet, inv);
    for (int64_t i = 0; i < n; i++)
        if (inv[c[i]] < 0) { bad = i; break; }
    if (bad < 0 && n % 4 == 1) bad = n;
    if (bad >= 0) { *err_off = bad; return -1; }
    full = n - n % 4;
    o = oracle_decode_quads(c, 0, full, p, inv);
    r = n - full;
    if (r >= 2) {
        uint32_t v = 0;
        for (int64_t k = 0; k < 4; k++) v = (v << 6) | (k < r ? (uint32_t)inv[c[full + k]] : 0u);
        for (int64_t k = 0; k < r - 1; k++) p[o++] = (uint8_t)(v >> (16 - 8 * k));
    }
    return o;
}

/* Appendix B: remove space (0x20), line feed (0x0A) and carriage return
 * (0x0D) by copying the kept bytes forward. Returns the new length. pos[k]
 * receives the original index of kept byte k when pos is not NULL. */
int64_t oracle_strip_ws(const uint8_t *a, int64_t n, uint8_t *out, int64_t *pos)
{
    int64_t q = 0;
    for (int64_t i = 0; i < n; i++) {
        uint8_t v = a[i];
        if (v == ' ' || v == '\n' || v == '\r') continue;
        if (pos) pos[q] = i;
        out[q++] = v;
    }
    return q;
}

/* Whitespace-tolerant decode: strip (Appendix B), decode, and report an error
 * offset in the coordinates of the original input. An error at the stripped
 * length (R2) maps to the original length n. */
int64_t oracle_decode_ws(const uint8_t *c, int64_t n, uint8_t *p, int alphabet, int64_t *err_off)
{
    int64_t m, len;
    uint8_t *tmp;
    int64_t *pos;
    *err_off = -1;
    if (n <= 0) return 0;
    tmp = (uint8_t *)malloc((size_t)n);
    pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!tmp || !pos) { free(tmp); free(pos); *err_off = -2; return -2; }
    m = oracle_strip_ws(c, n, tmp, pos);
    len = oracle_decode(tmp, m, p, alphabet, err_off);
    if (len < 0) *err_off = (*err_off >= m) ? n : pos[*err_off];
    free(tmp);
    free(pos);
    return len;
}

/* Batched forms: message i is src[in_off[i] .. in_off[i+1]) and its output
 * starts at dst + out_off[i]. flags[i] selects the alphabet (NULL: standard).
 * Plain loops over the single-message functions. */
void oracle_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                         const int64_t *out_off, const uint8_t *flags, int64_t *out_len)
{
    for (int64_t i = 0; i < N; i++)
        out_len[i] = oracle_encode(src + in_off[i], in_off[i + 1] - in_off[i], dst + out_off[i],
                                   flags ? flags[i] : ORACLE_STD);
}

void oracle_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                         const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                         int64_t *err_off)
{
    for (int64_t i = 0; i < N; i++)
        out_len[i] = oracle_decode(src + in_off[i], in_off[i + 1] - in_off[i], dst + out_off[i],
                                   flags ? flags[i] : ORACLE_STD, &err_off[i]);
}

/* ---- Multi-threaded wrappers, used only to time the oracle on many cores.
 * The buffer is cut at multiples of 3 bytes (encode) or 4 characters
 * (decode); each piece runs the same plain loops and the first error offset
 * is the minimum over pieces. */
typedef struct {
    const uint8_t *src;
    int64_t n, begin, end;
    uint8_t *dst;
    int alphabet, dir;
    int64_t bad, written;
} oracle_piece;

static void *oracle_piece_run(void *arg)
{
    oracle_piece *w = (oracle_piece *)arg;
    if (w->dir == 0) {
        w->written = oracle_encode(w->src + w->begin, w->end - w->begin, w->dst + (w->begin / 3) * 4,
                                   w->alphabet);
    } else {
        int inv[256];
        oracle_build_A(w->alphabet, inv);
        w->bad = oracle_first_bad(w->src, w->n, w->begin, w->end, inv);
        w->written = 0;
        /* a length that is not a multiple of 4 is an error (R2): no output */
        if (w->bad < 0 && w->n % 4 == 0)
            w->written = oracle_decode_quads(w->src, w->begin, w->end, w->dst + (w->begin / 4) * 3, inv);
    }
    return NULL;
}

static int64_t oracle_run_pieces(int dir, const uint8_t *src, int64_t n, uint8_t *dst, int alphabet,
                                 int threads, int64_t *err_off)
{
    int64_t unit = dir == 0 ? 3 : 4, units = n / unit, done = 0, total = 0, bad = -1;
    oracle_piece *w;
    pthread_t *tid;
    if (threads < 1) threads = 1;
    if (threads > 1024) threads = 1024;
    w = (oracle_piece *)calloc((size_t)threads, sizeof(*w));
    tid = (pthread_t *)calloc((size_t)threads, sizeof(*tid));
    for (int t = 0; t < threads; t++) {
        int64_t take = units / threads + (t < units % threads ? 1 : 0);
        w[t].src = src; w[t].n = n; w[t].dst = dst; w[t].alphabet = alphabet; w[t].dir = dir;
        w[t].begin = done * unit;
        done += take;
        w[t].end = (t == threads - 1) ? n : done * unit;
        w[t].bad = -1;
        pthread_create(&tid[t], NULL, oracle_piece_run, &w[t]);
    }
    for (int t = 0; t < threads; t++) {
        pthread_join(tid[t], NULL);
        if (w[t].bad >= 0 && (bad < 0 || w[t].bad < bad)) bad = w[t].bad;
        total += w[t].written;
    }
    free(w);
    free(tid);
    if (dir == 0) return total;
    if (bad < 0 && n % 4 != 0) bad = n;
    *err_off = bad;
    return bad >= 0 ? -1 : total - oracle_pads(src, n);
}

int64_t oracle_encode_mt(const uint8_t *s, int64_t n, uint8_t *p, int alphabet, int threads)
{
    int64_t unused;
    return n <= 0 ? 0 : oracle_run_pieces(0, s, n, p, alphabet, threads, &unused);
}

int64_t oracle_decode_mt(const uint8_t *c, int64_t n, uint8_t *p, int alphabet, int threads,
                         int64_t *err_off)
{
    *err_off = -1;
    return n <= 0 ? 0 : oracle_run_pieces(1, c, n, p, alphabet, threads, err_off);
}

/* Gather forms: message i is src[in_begin[i] .. in_begin[i] + in_len[i]);
 * otherwise as the packed forms above. */
void oracle_encode_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                          uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len)
{
    for (int64_t i = 0; i < N; i++)
        out_len[i] = oracle_encode(src + in_begin[i], in_len[i], dst + out_off[i],
                                   flags ? flags[i] : ORACLE_STD);
}

void oracle_decode_gather(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                          uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                          int64_t *err_off)
{
    for (int64_t i = 0; i < N; i++)
        out_len[i] = oracle_decode(src + in_begin[i], in_len[i], dst + out_off[i],
                                   flags ? flags[i] : ORACLE_STD, &err_off[i]);
}

/* ---- Multi-threaded batch wrappers, used to check very large batches in
 * seconds. The messages are cut into contiguous ranges of about equal input
 * bytes; each thread runs the plain per-message loop above over its range.
 * in_len == NULL selects the packed form (in_begin is then in_off). */
typedef struct {
    int dir;
    const uint8_t *src;
    const int64_t *in_begin, *in_len, *out_off;
    int64_t begin, end;
    uint8_t *dst;
    const uint8_t *flags;
    int64_t *out_len, *err_off;
} oracle_batch_piece;

static void *oracle_batch_piece_run(void *arg)
{
    oracle_batch_piece *w = (oracle_batch_piece *)arg;
    const int64_t b = w->begin, k = w->end - w->begin;
    const uint8_t *fl = w->flags ? w->flags + b : NULL;
    if (k <= 0) return NULL;
    if (w->in_len == NULL) {
        if (w->dir == 0)
            oracle_encode_batch(w->src, w->in_begin + b, k, w->dst, w->out_off + b, fl, w->out_len + b);
        else
            oracle_decode_batch(w->src, w->in_begin + b, k, w->dst, w->out_off + b, fl, w->out_len + b,
                                w->err_off + b);
    } else {
        if (w->dir == 0)
            oracle_encode_gather(w->src, w->in_begin + b, w->in_len + b, k, w->dst, w->out_off + b, fl,
                                 w->out_len + b);
        else
            oracle_decode_gather(w->src, w->in_begin + b, w->in_len + b, k, w->dst, w->out_off + b, fl,
                                 w->out_len + b, w->err_off + b);
    }
    return NULL;
}

static int64_t oracle_msg_len(const int64_t *in_begin, const int64_t *in_len, int64_t i)
{
    return in_len ? in_len[i] : in_begin[i + 1] - in_begin[i];
}

static void oracle_batch_pieces(int dir, const uint8_t *src, const int64_t *in_begin, const int64_t *in_len,
                                int64_t N, uint8_t *dst, const int64_t *out_off, const uint8_t *flags,
                                int64_t *out_len, int64_t *err_off, int threads)
{
    oracle_batch_piece *w;
    pthread_t *tid;
    int64_t total = 0, acc = 0, i = 0;
    if (N <= 0) return;
    if (threads < 1) threads = 1;
    if (threads > 1024) threads = 1024;
    for (int64_t j = 0; j < N; j++) total += oracle_msg_len(in_begin, in_len, j);
    w = (oracle_batch_piece *)calloc((size_t)threads, sizeof(*w));
    tid = (pthread_t *)calloc((size_t)threads, sizeof(*tid));
    for (int t = 0; t < threads; t++) {
        /* this range takes messages until its share of the bytes is reached */
        int64_t goal = (total / threads) * (t + 1);
        w[t].dir = dir; w[t].src = src; w[t].in_begin = in_begin; w[t].in_len = in_len;
        w[t].out_off = out_off; w[t].dst = dst; w[t].flags = flags; w[t].out_len = out_len;
        w[t].err_off = err_off;
        w[t].begin = i;
        if (t == threads - 1) i = N;
        else while (i < N && acc < goal) acc += oracle_msg_len(in_begin, in_len, i++);
        w[t].end = i;
        pthread_create(&tid[t], NULL, oracle_batch_piece_run, &w[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    free(w);
    free(tid);
}

void oracle_encode_batch_mt(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                            const int64_t *out_off, const uint8_t *flags, int64_t *out_len, int threads)
{
    oracle_batch_pieces(0, src, in_off, NULL, N, dst, out_off, flags, out_len, NULL, threads);
}

void oracle_decode_batch_mt(const uint8_t *src, const int64_t *in_off, int64_t N, uint8_t *dst,
                            const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                            int64_t *err_off, int threads)
{
    oracle_batch_pieces(1, src, in_off, NULL, N, dst, out_off, flags, out_len, err_off, threads);
}

void oracle_encode_gather_mt(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                             uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                             int threads)
{
    oracle_batch_pieces(0, src, in_begin, in_len, N, dst, out_off, flags, out_len, NULL, threads);
}

void oracle_decode_gather_mt(const uint8_t *src, const int64_t *in_begin, const int64_t *in_len, int64_t N,
                             uint8_t *dst, const int64_t *out_off, const uint8_t *flags, int64_t *out_len,
                             int64_t *err_off, int threads)
{
    oracle_batch_pieces(1, src, in_begin, in_len, N, dst, out_off, flags, out_len, err_off, threads);
}
