/*
 * A plain C client of the codec library: compiled with gcc against
 * include/b64.h only and linked to libb64hip.so (plus the HIP runtime for
 * device memory). It checks that the header is valid C and that the calls
 * named in it behave as declared when called from C.
 *
 *   b64_abi_client host
 *       pure-host functions and argument errors (no GPU needed);
 *   b64_abi_client gpu <payload> <text_out> <bytes_out> <pos> <byte>
 *       b64_encode of the payload on the NULL stream, b64_decode of the
 *       text, then b64_decode of the text with byte <byte> at index <pos>;
 *       writes the text and the decoded bytes and prints the returned
 *       lengths and error offsets as one line of key=value pairs.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "b64.h"

static int fails = 0;

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            fails++;                                                     \
        }                                                                \
    } while (0)

static int run_host(void)
{
    int64_t err = 0, need[5], off[6];
    const int64_t lens[5] = {0, 1, 2, 3, 17};
    const uint8_t flags[5] = {0, B64_FLAG_NOPAD, B64_FLAG_URL, 0, B64_FLAG_NOPAD};
    for (int64_t n = 0; n < 64; n++) {
        CHECK(b64_encoded_len(n) == 4 * ((n + 2) / 3));
        CHECK(b64_decoded_max(n) == 3 * (n / 4));
    }
    CHECK(b64_encoded_len(-1) == B64_BAD_ARG);
    CHECK(b64_last_error() != NULL && strlen(b64_last_error()) > 0);
    CHECK(b64_encode(NULL, 0, NULL) == 0);
    CHECK(b64_encode(NULL, 5, NULL) == B64_BAD_ARG);
    CHECK(b64_decode(NULL, 0, NULL, &err) == 0 && err == -1);
    CHECK(b64_decode(NULL, 8, NULL, &err) == B64_BAD_ARG);
    CHECK(b64_decode(NULL, 0, NULL, NULL) == B64_BAD_ARG);
    CHECK(b64_batch_slots(B64_DIR_ENCODE, lens, flags, 5, need, off) == B64_OK);
    CHECK(need[0] == 0 && need[1] == 2 && need[2] == 4 && need[3] == 4 && need[4] == 23);
    CHECK(off[0] == 0 && off[1] == 0 && off[2] == 4 && off[3] == 8 && off[4] == 12 && off[5] == 36);
    CHECK(b64_batch_slots(B64_DIR_DECODE, lens, flags, 5, need, off) == B64_OK);
    /* decode capacities 0, 0, 0, 0, 3*4 + (17 mod 4 = 1: no extra byte) */
    CHECK(need[0] == 0 && need[4] == 12 && off[5] == 12);
    CHECK(b64_batch_slots(2, lens, flags, 5, need, off) == B64_BAD_ARG);
    printf("host checks: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}

static uint8_t *read_file(const char *path, int64_t *n)
{
    FILE *f = fopen(path, "rb");
    uint8_t *buf;
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    *n = ftell(f);
    fseek(f, 0, SEEK_SET);
    buf = (uint8_t *)malloc((size_t)(*n > 0 ? *n : 1));
    if (*n > 0 && fread(buf, 1, (size_t)*n, f) != (size_t)*n) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    return buf;
}

static int write_file(const char *path, const uint8_t *p, int64_t n)
{
    FILE *f = fopen(path, "wb");
    int ok;
    if (!f) return 0;
    ok = n <= 0 || fwrite(p, 1, (size_t)n, f) == (size_t)n;
    fclose(f);
    return ok;
}

static int run_gpu(int argc, char **argv)
{
    int64_t n = 0, m, cap, dec_len, dec_err = 0, bad_len, bad_err = 0, pos;
    uint8_t *h_in, *h_text, *h_out, *d_in = NULL, *d_text = NULL, *d_out = NULL, byte;
    if (argc != 7) return 2;
    h_in = read_file(argv[2], &n);
    if (!h_in) return 2;
    pos = atoll(argv[5]);
    byte = (uint8_t)atoi(argv[6]);
    m = b64_encoded_len(n);
    cap = b64_decoded_max(m);
    if (hipMalloc((void **)&d_in, (size_t)(n > 0 ? n : 1)) != hipSuccess ||
        hipMalloc((void **)&d_text, (size_t)(m > 0 ? m : 1)) != hipSuccess ||
        hipMalloc((void **)&d_out, (size_t)(cap > 0 ? cap : 1)) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 3;
    }
    if (n > 0 && hipMemcpy(d_in, h_in, (size_t)n, hipMemcpyHostToDevice) != hipSuccess) return 3;
    CHECK(b64_encode(d_in, n, d_text) == m);
    h_text = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    h_out = (uint8_t *)malloc((size_t)(cap > 0 ? cap : 1));
    if (m > 0 && hipMemcpy(h_text, d_text, (size_t)m, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    dec_len = b64_decode(d_text, m, d_out, &dec_err);
    if (dec_len > 0 && hipMemcpy(h_out, d_out, (size_t)dec_len, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    if (pos >= 0 && pos < m && hipMemcpy(d_text + pos, &byte, 1, hipMemcpyHostToDevice) != hipSuccess) return 3;
    bad_len = b64_decode(d_text, m, d_out, &bad_err);
    if (!write_file(argv[3], h_text, m) || !write_file(argv[4], h_out, dec_len > 0 ? dec_len : 0)) return 2;
    printf("enc_len=%lld dec_len=%lld dec_err=%lld bad_len=%lld bad_err=%lld\n", (long long)m,
           (long long)dec_len, (long long)dec_err, (long long)bad_len, (long long)bad_err);
    hipFree(d_in);
    hipFree(d_text);
    hipFree(d_out);
    free(h_in);
    free(h_text);
    free(h_out);
    return fails ? 1 : 0;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && strcmp(argv[1], "host") == 0) return run_host();
    if (argc >= 2 && strcmp(argv[1], "gpu") == 0) return run_gpu(argc, argv);
    fprintf(stderr, "usage: b64_abi_client host | gpu <payload> <text_out> <bytes_out> <pos> <byte>\n");
    return 2;
}
