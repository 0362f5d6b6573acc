// Device-side building blocks of the gfx950 base64 codec.
//
// Work unit: one lane turns 12 input bytes into 16 characters (encode) or 16
// characters into 12 bytes (decode); a wave of 64 lanes therefore moves 768 or
// 1024 contiguous bytes per load instruction. This is the GPU shape of the
// paper's vector outline (Section 4: load, unpack/translate, pack, store);
// the AVX2 lane-crossing shuffles it needs on x86 have no counterpart here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "b64_modes.hpp"

namespace b64dev {

// ---------------------------------------------------------------- tables --
// Section 2, Table 1 (standard alphabet) and the base64url variant (values
// 62 and 63 become '-' and '_').
struct Tables {
    uint8_t enc[2][64];   // value -> character, per alphabet
    uint8_t dec[2][256];  // character -> value, 0x80 = not a symbol ('=' too)
};

constexpr Tables make_tables()
{
    Tables t{};
    const char std64[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/";
    for (int a = 0; a < 2; a++) {
        for (int v = 0; v < 64; v++) {
            char ch = std64[v];
            if (a == 1 && v == 62) ch = '-';
            if (a == 1 && v == 63) ch = '_';
            t.enc[a][v] = (uint8_t)ch;
        }
        for (int c = 0; c < 256; c++) t.dec[a][c] = 0x80;
        for (int v = 0; v < 64; v++) t.dec[a][t.enc[a][v]] = (uint8_t)v;
    }
    return t;
}

constexpr uint8_t INVALID = 0x80;
// "No error yet" value of an error slot; real offsets are smaller (unsigned
// atomicMin keeps the smallest).
constexpr unsigned long long ERR_NONE = 0x7fffffffffffffffull;

// Mode bits (per call or per message).
constexpr int M_URL = B64I_M_URL;
constexpr int M_STRICT = B64I_M_STRICT;
constexpr int M_NOPAD = B64I_M_NOPAD;

// -------------------------------------------------------------- byte ops --
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// (hi:lo) >> (8 * s) for s in 0..3
__device__ __forceinline__ uint32_t alignb(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}

// -------------------------------------------------------- encode (a2,a3) --
// Algorithm 1 on one triple held big-endian in the low 24 bits of v: the four
// 6-bit fields, most significant first, mapped through B (LDS table `tab`).
__device__ __forceinline__ uint32_t enc_quad(uint32_t v, const uint8_t *tab)
{
    uint32_t a = tab[v >> 18];
    uint32_t b = tab[(v >> 12) & 63];
    uint32_t c = tab[(v >> 6) & 63];
    uint32_t d = tab[v & 63];
    return a | (b << 8) | (c << 16) | (d << 24);
}

// 12 bytes (little-endian dwords w0..w2) -> 16 characters (o0..o3).
// v_perm gathers each 3-byte group into big-endian order: bytes (b0,b1,b2),
// (b3,b4,b5), (b6,b7,b8), (b9,b10,b11).
__device__ __forceinline__ void enc_unit(uint32_t w0, uint32_t w1, uint32_t w2, const uint8_t *tab,
                                         uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3)
{
    o0 = enc_quad(perm(w0, w0, 0x0c000102u), tab);
    o1 = enc_quad(perm(w0, w1, 0x0c070001u), tab);
    o2 = enc_quad(perm(w1, w2, 0x0c060700u), tab);
    o3 = enc_quad(perm(w2, w2, 0x0c010203u), tab);
}

// ----------------------------------------------------- register tails --
// Byte i (0..15) of four little-endian words, by a select chain (no
// dynamic register indexing, so no scratch memory).
__device__ __forceinline__ uint32_t byte_of(const uint32_t (&w)[4], int i)
{
    const uint32_t x = i < 4 ? w[0] : i < 8 ? w[1] : i < 12 ? w[2] : w[3];
    return (x >> (8 * (i & 3))) & 0xffu;
}

// r bytes (1..16) at p into w (zero beyond r). Only the aligned dwords that
// hold a byte of [p, p + r) are read, all in one round of predicated loads.
__device__ __forceinline__ void load_upto16(const uint8_t *p, int r, uint32_t (&w)[4])
{
    const uint32_t s = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *d = (const uint32_t *)(p - s);
    const int nd = ((int)s + r + 3) >> 2;  // 1..5
    uint32_t x[5];
#pragma unroll
    for (int k = 0; k < 5; k++) x[k] = k < nd ? d[k] : 0u;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint32_t v = s ? alignb(x[k + 1], x[k], s) : x[k];
        const int keep = r - 4 * k;  // bytes of this word inside the run
        v = keep >= 4 ? v : keep <= 0 ? 0u : (v & ((1u << (8 * keep)) - 1u));
        w[k] = v;
    }
}

// Writes c bytes (0..16) held little-endian in o to q: whole dwords when q is
// 4-byte aligned, then the partial dword; byte stores otherwise.
__device__ __forceinline__ void store_upto16(uint8_t *q, const uint32_t (&o)[4], int c)
{
    if ((((uintptr_t)q) & 3) == 0) {
        uint32_t *d = (uint32_t *)q;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (4 * k + 4 <= c) d[k] = o[k];
        const int full = c >> 2, rest = c & 3;
        if (rest) {
            const uint32_t v = full == 0 ? o[0] : full == 1 ? o[1] : full == 2 ? o[2] : o[3];
            uint8_t *e = q + 4 * full;
            if (rest & 2) { *(uint16_t *)e = (uint16_t)v; e += 2; }
            if (rest & 1) *e = (uint8_t)(rest & 2 ? v >> 16 : v);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; i++)
            if (i < c) q[i] = (uint8_t)byte_of(o, i);
    }
}

// Final partial unit of a message through the full-unit routine: r bytes
// (1..11) in w, zero beyond r, so the characters of the last group's missing
// bits come out as those of zero bits; then the positions Algorithm 1 pads
// become '=' (or are not written, unpadded). Returns the characters written.
__device__ __forceinline__ int enc_tail_fast(const uint32_t (&w)[4], int r, uint8_t *__restrict__ q,
                                             const uint8_t *tab, int nopad)
{
    uint32_t o[4];
    enc_unit(w[0], w[1], w[2], tab, o[0], o[1], o[2], o[3]);
    const int g = r / 3, rem = r - 3 * g;  // full groups, leftover bytes of the last one
    int c = 4 * g;
    if (rem) {
        // group g fills dword g: its first rem + 1 characters are real
        const uint32_t keep = (1u << (8 * (rem + 1))) - 1u;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (k == g) o[k] = (o[k] & keep) | (0x3d3d3d3du & ~keep);
        c += nopad ? rem + 1 : 4;
    }
    store_upto16(q, o, c);
    return c;
}

// The same for the r bytes (1..11) at s in global memory, group by group
// (out of line, once per message or per launch; its registers count against
// every kernel that calls it, so it stays lean rather than fast).
__device__ __noinline__ int enc_tail(const uint8_t *__restrict__ s, int r, uint8_t *__restrict__ q,
                                     const uint8_t *tab, int nopad)
{
    uint32_t w[4];
    load_upto16(s, r, w);
    uint32_t o[4] = {0u, 0u, 0u, 0u};
    int c = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int left = r - 3 * i;  // bytes from this group on
        if (left <= 0) break;
        const uint32_t v = (byte_of(w, 3 * i) << 16) | (byte_of(w, 3 * i + 1) << 8) | byte_of(w, 3 * i + 2);
        const uint32_t ch[4] = {tab[v >> 18], tab[(v >> 12) & 63], left >= 2 ? tab[(v >> 6) & 63] : (uint32_t)'=',
                                left >= 3 ? tab[v & 63] : (uint32_t)'='};
        const int emit = nopad ? (left >= 3 ? 4 : left + 1) : 4;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (j < emit) {
                const int at = c + j;  // at < 16
                const uint32_t bits = ch[j] << (8 * (at & 3));
                if (at < 4) o[0] |= bits; else if (at < 8) o[1] |= bits; else if (at < 12) o[2] |= bits; else o[3] |= bits;
            }
        }
        c += emit;
    }
    store_upto16(q, o, c);
    return c;
}

// ------------------------------------------------------ decode (a7,a9) --
// 16 characters (w0..w3) -> 12 bytes (o0..o2). Returns the OR of the 16
// looked-up values: bit 7 set means some character is not a symbol.
// Each quad (a,b,c,d) packs to the 24-bit value a<<18 | b<<12 | c<<6 | d,
// whose three bytes (most significant first) are Algorithm 2's output bytes.
__device__ __forceinline__ uint32_t dec_word(uint32_t w, const uint8_t *tab, uint32_t &t)
{
    uint32_t a = tab[w & 0xff];
    uint32_t b = tab[(w >> 8) & 0xff];
    uint32_t c = tab[(w >> 16) & 0xff];
    uint32_t d = tab[w >> 24];
    t = (a << 18) | (b << 12) | (c << 6) | d;
    return a | b | c | d;
}

__device__ __forceinline__ uint32_t dec_unit(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                             const uint8_t *tab, uint32_t &o0, uint32_t &o1,
                                             uint32_t &o2)
{
    uint32_t t0, t1, t2, t3;
    uint32_t bad = dec_word(w0, tab, t0) | dec_word(w1, tab, t1) | dec_word(w2, tab, t2) |
                   dec_word(w3, tab, t3);
    o0 = perm(t1, t0, 0x06000102u);  // t0.b2 t0.b1 t0.b0 t1.b2
    o1 = perm(t2, t1, 0x05060001u);  // t1.b1 t1.b0 t2.b2 t2.b1
    o2 = perm(t3, t2, 0x04050600u);  // t2.b0 t3.b2 t3.b1 t3.b0
    return bad;
}

// Index (0..15) of the first non-symbol among the 16 characters of a unit.
__device__ __noinline__ int dec_first_bad(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                          const uint8_t *tab)
{
    int first = 16;
#pragma unroll
    for (int k = 15; k >= 0; k--) {  // unrolled: each word picked by a constant index
        const uint32_t x = k < 4 ? w0 : k < 8 ? w1 : k < 12 ? w2 : w3;
        if (tab[(x >> (8 * (k & 3))) & 0xff] & INVALID) first = k;
    }
    return first;
}

// Final unit of a message of n characters: r characters (1..16), which are
// characters n-r .. n-1, held little-endian in w. Applies the padding rules
// ('=' only as the last one or two characters of a length divisible by 4;
// unpadded mode: '=' invalid, n mod 4 == 1 is a length error), the optional
// strict leftover-bit check (Appendix A), and writes the decoded bytes to q.
// The characters from the padding on (and past r) are read as 'A' (value
// 0), so one dec_unit gives the bytes of every group, the first non-symbol
// among the rest is the first offending index, and only the counts differ
// from an interior unit. Returns the first offending index (relative to the
// unit, r for a length error at n), or -1 - (bytes written) on success.
__device__ __forceinline__ int dec_tail_fast(const uint32_t (&w)[4], int r, int64_t n, uint8_t *__restrict__ q,
                                             const uint8_t *tab, int mode)
{
    const bool nopad = (mode & M_NOPAD) != 0;
    int pads = 0;
    if (!nopad && (n & 3) == 0 && byte_of(w, r - 1) == '=') pads = (r >= 2 && byte_of(w, r - 2) == '=') ? 2 : 1;
    const int keep = r - pads;  // characters decoded as written
    uint32_t x[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int kb = keep - 4 * k;
        const uint32_t m = kb >= 4 ? 0xffffffffu : kb <= 0 ? 0u : (1u << (8 * kb)) - 1u;
        x[k] = (w[k] & m) | (0x41414141u & ~m);
    }
    uint32_t o[4];
    o[3] = 0;
    const uint32_t bad = dec_unit(x[0], x[1], x[2], x[3], tab, o[0], o[1], o[2]);
    if (bad & INVALID) return dec_first_bad(x[0], x[1], x[2], x[3], tab);
    if (nopad ? ((n & 3) == 1) : ((n & 3) != 0)) return r;
    // Appendix A (strict): leftover bits of a padded final quad must be zero.
    if ((mode & M_STRICT) && pads == 2 && (tab[byte_of(w, r - 3)] & 15) != 0) return r - 3;
    if ((mode & M_STRICT) && pads == 1 && (tab[byte_of(w, r - 2)] & 3) != 0) return r - 2;
    const int nout = 3 * (r >> 2) - pads + ((nopad && (r & 3) >= 2) ? (r & 3) - 1 : 0);
    store_upto16(q, o, nout);
    return -1 - nout;
}

// The same for r characters at c in global memory, loaded once into
// registers. Inline form: the batched decode finishes many messages per wave,
// where a call costs more than the extra code (dec_tail below is the
// out-of-line form for once-per-launch use).
__device__ __forceinline__ int dec_tail_inl(const uint8_t *__restrict__ c, int r, int64_t n,
                                            uint8_t *__restrict__ q, const uint8_t *tab, int mode)
{
    uint32_t w[4];
    load_upto16(c, r, w);
    return dec_tail_fast(w, r, n, q, tab, mode);
}

__device__ __noinline__ int dec_tail(const uint8_t *__restrict__ c, int r, int64_t n,
                                     uint8_t *__restrict__ q, const uint8_t *tab, int mode)
{
    return dec_tail_inl(c, r, n, q, tab, mode);
}

// -------------------------------------------- register and pair maps --
// Alternatives to the LDS byte tables, chosen per launch (map 0 = LDS byte
// tables, the default):
//   map 1  the paper's vector translations with v_perm_b32 as a 4-byte-wide
//          lookup over 8-entry tables: encoding adds a per-range offset
//          (Section 4.1, Tables 4 and 5: ranges [0,26), [26,52), [52,62), 62,
//          63); decoding validates with nibble bitsets and adds an offset
//          looked up by the high nibble (Section 4.2, Algorithm 3).
//   map 2  (encode) a 4096-entry table of character pairs in LDS, one lookup
//          per 12 bits, in the spirit of the scalar table codecs the paper
//          compares against (Section 3).
// All constants are derived here from Table 1 and its base64url variant.
struct PermMaps {
    uint32_t enc_off[2][2];   // [alphabet]: offsets of range index 0..4 (bytes of a 64-bit pair)
    uint32_t dec_lo[2][4];    // [alphabet]: bitsets by low nibble 0..15
    uint32_t dec_hi[2][2];    // [alphabet]: class bit by high nibble 0..7 (8..15: 0x10)
    uint32_t dec_roll[2][2];  // [alphabet]: offset by index 0..7 (index 1: the symbol of value 63)
    uint32_t special[2];      // [alphabet]: the symbol of value 63 in all four bytes
    int consistent;           // 1 when the tables reproduce Table 1 (checked at compile time)
};

constexpr PermMaps make_perm_maps()
{
    PermMaps m{};
    const Tables t = make_tables();
    m.consistent = 1;
    for (int a = 0; a < 2; a++) {
        // encode: offsets B(v) - v, constant on each range
        const int starts[5] = {0, 26, 52, 62, 63};
        uint8_t off[8] = {};
        for (int r = 0; r < 5; r++) off[r] = (uint8_t)(t.enc[a][starts[r]] - starts[r]);
        for (int v = 0; v < 64; v++) {
            int r = (v >= 26) + (v >= 52) + (v >= 62) + (v >= 63);
            if ((uint8_t)(v + off[r]) != t.enc[a][v]) m.consistent = 0;
        }
        m.enc_off[a][0] = off[0] | (off[1] << 8) | (off[2] << 16) | ((uint32_t)off[3] << 24);
        m.enc_off[a][1] = off[4];
        // decode: the low nibbles valid under each high nibble define classes;
        // the empty class (high nibbles without symbols, 8..15 included) gets
        // bit 0x10, the others bits 0x01, 0x02, 0x04, 0x08, 0x20, 0x40, 0x80
        const uint8_t bits[7] = {0x01, 0x02, 0x04, 0x08, 0x20, 0x40, 0x80};
        uint32_t cls_set[8] = {};
        uint8_t cls_bit[8] = {};
        int ncls = 0;
        uint8_t hi[16] = {};
        for (int h = 0; h < 16; h++) {
            uint32_t set = 0;
            for (int l = 0; l < 16; l++)
                if (!(t.dec[a][(h << 4) | l] & INVALID)) set |= 1u << l;
            if (!set) { hi[h] = 0x10; continue; }
            int c = -1;
            for (int i = 0; i < ncls; i++)
                if (cls_set[i] == set) c = i;
            if (c < 0) {
                if (ncls >= 7) { m.consistent = 0; continue; }
                c = ncls++;
                cls_set[c] = set;
                cls_bit[c] = bits[c];
            }
            hi[h] = cls_bit[c];
            if (h >= 8) m.consistent = 0;  // symbols are ASCII
        }
        uint8_t lo[16] = {};
        for (int l = 0; l < 16; l++) {
            lo[l] = 0x10;
            for (int i = 0; i < ncls; i++)
                if (!(cls_set[i] & (1u << l))) lo[l] |= cls_bit[i];
        }
        for (int i = 0; i < 4; i++)
            m.dec_lo[a][i] = lo[4 * i] | (lo[4 * i + 1] << 8) | (lo[4 * i + 2] << 16) | ((uint32_t)lo[4 * i + 3] << 24);
        m.dec_hi[a][0] = hi[0] | (hi[1] << 8) | (hi[2] << 16) | ((uint32_t)hi[3] << 24);
        m.dec_hi[a][1] = hi[4] | (hi[5] << 8) | (hi[6] << 16) | ((uint32_t)hi[7] << 24);
        const uint8_t sp = t.enc[a][63];
        m.special[a] = sp * 0x01010101u;
        uint8_t roll[8] = {};
        bool set_r[8] = {};
        roll[1] = (uint8_t)(63 - sp);
        set_r[1] = true;
        for (int c = 0; c < 256; c++) {
            if ((t.dec[a][c] & INVALID) || c == sp) continue;
            const int h = c >> 4;
            if (h == 1) m.consistent = 0;
            const uint8_t r = (uint8_t)(t.dec[a][c] - c);
            if (set_r[h] && roll[h] != r) m.consistent = 0;
            roll[h] = r;
            set_r[h] = true;
        }
        m.dec_roll[a][0] = roll[0] | (roll[1] << 8) | (roll[2] << 16) | ((uint32_t)roll[3] << 24);
        m.dec_roll[a][1] = roll[4] | (roll[5] << 8) | (roll[6] << 16) | ((uint32_t)roll[7] << 24);
    }
    return m;
}
static_assert(make_perm_maps().consistent == 1, "register maps must reproduce Table 1");

// 4096 character pairs per alphabet: entry i holds B(i >> 6) then B(i & 63).
struct PairTables {
    uint16_t pair[2][4096];
};

constexpr PairTables make_pair_tables()
{
    PairTables p{};
    const Tables t = make_tables();
    for (int a = 0; a < 2; a++)
        for (int i = 0; i < 4096; i++) p.pair[a][i] = (uint16_t)(t.enc[a][i >> 6] | (t.enc[a][i & 63] << 8));
    return p;
}

// Bytewise a + b (mod 256 per byte, no carry between bytes).
__device__ __forceinline__ uint32_t byte_add(uint32_t a, uint32_t b)
{
    return ((a & 0x7f7f7f7fu) + (b & 0x7f7f7f7fu)) ^ ((a ^ b) & 0x80808080u);
}

// Bit 8j + 7 set exactly when byte j of w is zero.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t w)
{
    return ~(((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
}

// Per-launch map context: the LDS byte table (every map uses it for tails
// and error paths), the LDS pair table (map 2) and the register maps of the
// selected alphabet (map 1).
struct MapCtx {
    const uint8_t *tab;
    const uint16_t *tab12;
    uint32_t e0, e1;
    uint32_t l0, l1, l2, l3, h0, h1, r0, r1, sp;
};

// Map 1, encode: four 6-bit values (one per byte) -> four characters.
__device__ __forceinline__ uint32_t enc_map_perm(uint32_t x, uint32_t e0, uint32_t e1)
{
    // range index: how many of 26, 52, 62, 63 the value reaches (no carries:
    // values are below 64)
    const uint32_t i = (((x + 0x66666666u) >> 7) & 0x01010101u) + (((x + 0x4c4c4c4cu) >> 7) & 0x01010101u) +
                       (((x + 0x42424242u) >> 7) & 0x01010101u) + (((x + 0x41414141u) >> 7) & 0x01010101u);
    return byte_add(x, perm(e1, e0, i));
}

// Map 1, decode: four characters -> four 6-bit values (one per byte); bad
// collects nonzero bytes for characters outside the alphabet.
__device__ __forceinline__ uint32_t dec_map_perm(uint32_t x, const MapCtx &m, uint32_t &bad)
{
    const uint32_t ln = x & 0x0f0f0f0fu;
    const uint32_t hn = (x >> 4) & 0x0f0f0f0fu;
    const uint32_t l7 = ln & 0x07070707u, h7 = hn & 0x07070707u;
    const uint32_t lsel = ((ln >> 3) & 0x01010101u) * 0xffu;
    const uint32_t lb = (perm(m.l3, m.l2, l7) & lsel) | (perm(m.l1, m.l0, l7) & ~lsel);
    const uint32_t hb = perm(m.h1, m.h0, h7) | ((hn & 0x08080808u) << 1);
    bad |= lb & hb;
    const uint32_t esel = (zero_bytes(x ^ m.sp) >> 7) * 0xffu;  // bytes equal to the symbol of value 63
    const uint32_t idx = (0x01010101u & esel) | (h7 & ~esel);
    return byte_add(x, perm(m.r1, m.r0, idx));
}

template <int MAP>
__device__ __forceinline__ void enc_unit_m(uint32_t w0, uint32_t w1, uint32_t w2, const MapCtx &m,
                                           uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3)
{
    if (MAP == 0) {
        enc_unit(w0, w1, w2, m.tab, o0, o1, o2, o3);
        return;
    }
    const uint32_t g[4] = {perm(w0, w0, 0x0c000102u), perm(w0, w1, 0x0c070001u), perm(w1, w2, 0x0c060700u),
                           perm(w2, w2, 0x0c010203u)};
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t v = g[i];
        if (MAP == 1) {
            const uint32_t x = (v >> 18) | (((v >> 12) & 63) << 8) | (((v >> 6) & 63) << 16) | ((v & 63) << 24);
            o[i] = enc_map_perm(x, m.e0, m.e1);
        } else {
            o[i] = (uint32_t)m.tab12[v >> 12] | ((uint32_t)m.tab12[v & 0xfff] << 16);
        }
    }
    o0 = o[0]; o1 = o[1]; o2 = o[2]; o3 = o[3];
}

template <int MAP>
__device__ __forceinline__ uint32_t dec_unit_m(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, const MapCtx &m,
                                               uint32_t &o0, uint32_t &o1, uint32_t &o2)
{
    if (MAP == 0) return dec_unit(w0, w1, w2, w3, m.tab, o0, o1, o2);
    uint32_t bad = 0;
    const uint32_t w[4] = {w0, w1, w2, w3};
    uint32_t t[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t v = dec_map_perm(w[i], m, bad);
        t[i] = ((v & 63) << 18) | (((v >> 8) & 63) << 12) | (((v >> 16) & 63) << 6) | ((v >> 24) & 63);
    }
    o0 = perm(t[1], t[0], 0x06000102u);
    o1 = perm(t[2], t[1], 0x05060001u);
    o2 = perm(t[3], t[2], 0x04050600u);
    return bad ? INVALID : 0u;
}

// ------------------------------------------------------------ memory ops --
struct __attribute__((aligned(4))) u32x3 { uint32_t x, y, z; };
struct __attribute__((aligned(4))) u32x4 { uint32_t x, y, z, w; };

// Loads of `count` bytes from any address p read the aligned dwords that
// contain them: at offset s = p mod 4 > 0, one 4-byte-aligned 16-byte load
// at p - s (plus a dword for 16 bytes), whose last dword still holds a byte
// of [p, p + count), so every dword read lies on a page the buffer occupies.
// Pointer arithmetic (not integer casts) keeps the global address space, so
// these compile to global (not flat) loads.
__device__ __forceinline__ void load12(const uint8_t *p, uint32_t &w0, uint32_t &w1, uint32_t &w2)
{
    const uint32_t s = (uint32_t)((uintptr_t)p & 3);
    if (s == 0) {
        const u32x3 v = *(const u32x3 *)p;
        w0 = v.x; w1 = v.y; w2 = v.z;
    } else {
        const u32x4 v = *(const u32x4 *)(p - s);
        w0 = alignb(v.y, v.x, s); w1 = alignb(v.z, v.y, s); w2 = alignb(v.w, v.z, s);
    }
}

__device__ __forceinline__ void load16(const uint8_t *p, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                       uint32_t &w3)
{
    const uint32_t s = (uint32_t)((uintptr_t)p & 3);
    if (s == 0) {
        const u32x4 v = *(const u32x4 *)p;
        w0 = v.x; w1 = v.y; w2 = v.z; w3 = v.w;
    } else {
        const u32x4 v = *(const u32x4 *)(p - s);
        const uint32_t d4 = *(const uint32_t *)(p - s + 16);
        w0 = alignb(v.y, v.x, s); w1 = alignb(v.z, v.y, s); w2 = alignb(v.w, v.z, s);
        w3 = alignb(d4, v.w, s);
    }
}

// Stores of a byte run at any address: whole aligned dwords where the run
// covers them, byte/short stores for the partial dwords at either end, so no
// byte outside [q, q + 4k) is written.
__device__ __forceinline__ void store_edge_lo(uint8_t *q, uint32_t v, uint32_t nbytes)
{  // low nbytes (1..3) of v at the 4-byte aligned address q
    if (nbytes & 2) { *(uint16_t *)q = (uint16_t)v; q += 2; v >>= 16; }
    if (nbytes & 1) { q[0] = (uint8_t)v; }
}

template <int K, bool NT = false>
__device__ __forceinline__ void store_words(uint8_t *q, const uint32_t (&o)[K])
{
    const uint32_t s = (uint32_t)((uintptr_t)q & 3);
    if (s == 0) {
        uint32_t *d = (uint32_t *)q;
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (NT) __builtin_nontemporal_store(o[k], d + k);  // streamed: written once, not re-read
            else d[k] = o[k];
        }
        return;
    }
    // bytes land at offset s of the aligned window d[0 .. K]
    uint32_t *d = (uint32_t *)(q - s);
    const uint32_t sh = 4 - s;  // realign: window dword j = (o[j] : o[j-1]) >> 8*sh
    // head: high (4 - s) bytes of d[0] get the first (4 - s) bytes of o[0]
    if (s == 1) { q[0] = (uint8_t)o[0]; *(uint16_t *)(q + 1) = (uint16_t)(o[0] >> 8); }
    else if (s == 2) { *(uint16_t *)q = (uint16_t)o[0]; }
    else { q[0] = (uint8_t)o[0]; }
#pragma unroll
    for (int k = 1; k < K; k++) d[k] = alignb(o[k], o[k - 1], sh);
    // tail: low s bytes of d[K] get the last s bytes of o[K-1]
    store_edge_lo((uint8_t *)(d + K), o[K - 1] >> (8 * sh), s);
}

// K dwords' worth of bytes (K = 1 or 2) at any address p, read as the aligned
// dwords that hold them.
template <int K>
__device__ __forceinline__ void load_words(const uint8_t *p, uint32_t (&w)[K])
{
    const uint32_t s = (uint32_t)((uintptr_t)p & 3);
    const uint32_t *a = (const uint32_t *)(p - s);
    if (s == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) w[k] = a[k];
    } else {
        uint32_t v[K + 1];
#pragma unroll
        for (int k = 0; k <= K; k++) v[k] = a[k];
#pragma unroll
        for (int k = 0; k < K; k++) w[k] = alignb(v[k + 1], v[k], s);
    }
}

// Lane i gets lane i - 1's x (lane 0 gets 0): one DPP move shifting the
// whole wave by a lane, with every lane active.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}

// Stores of a wave's consecutive output runs (lane i's 4K bytes directly
// after lane i - 1's) at a destination that is not 4-byte aligned; the
// misalignment s = q & 3 is the same in every lane. Lane i writes the aligned
// window [q - s, q - s + 4K) as whole dwords in one vector store: its first
// s bytes end the run before its own, whose last word pw the caller supplies
// (the left neighbour's, by a wave shift; lane 0 recomputes it). So no
// dword is written by two waves, which on MI355X costs far more than the
// extra work: each would hold a partial dword in its XCD's L2. Only where
// the run before is not the caller's (the first unit of a buffer) does the
// lane write its head with byte/short stores (whole_head == false), and only
// at the end of the buffer's units its last s bytes (tail == true), so no byte
// outside the runs is written.
template <int K>
__device__ __forceinline__ void store_run_wave(uint8_t *q, const uint32_t (&o)[K], uint32_t pw, bool whole_head,
                                               bool tail)
{
    const uint32_t s = (uint32_t)((uintptr_t)q & 3);
    const uint32_t sh = 4 - s;
    uint32_t *d = (uint32_t *)(q - s);
    uint32_t w[K];
    w[0] = alignb(o[0], pw, sh);
#pragma unroll
    for (int k = 1; k < K; k++) w[k] = alignb(o[k], o[k - 1], sh);
    if (whole_head) {
        __builtin_nontemporal_store(w[0], d);
    } else if (s == 1) {
        q[0] = (uint8_t)o[0];
        *(uint16_t *)(q + 1) = (uint16_t)(o[0] >> 8);
    } else if (s == 2) {
        *(uint16_t *)q = (uint16_t)o[0];
    } else {
        q[0] = (uint8_t)o[0];
    }
#pragma unroll
    for (int k = 1; k < K; k++) __builtin_nontemporal_store(w[k], d + k);
    if (tail) store_edge_lo((uint8_t *)(d + K), o[K - 1] >> (8 * sh), s);
}

// ------------------------------------------------------ buffer steps --
// Copies `bytes` (multiple of 4) of the constant tables into LDS.
__device__ __forceinline__ void lds_fill(uint32_t *dst, const uint8_t *src, int bytes)
{
    const uint32_t *s = (const uint32_t *)src;
    for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) dst[i] = s[i];
}

// One grid-stride step of the encode over one buffer: this lane's units are
// first + k * stride for k < UPL. Without GUARD every unit is known to be in
// range, so all UPL loads are issued before any is consumed.
// SPLIT (the destination is not 4-byte aligned; the caller checks): every
// lane of the wave calls the step, lane l's first is the wave's first plus l,
// and the output goes through store_run_wave, with the words between lanes
// passed by a wave shift. The last s bytes of a unit are then written with
// the next unit, which must also be written by such a step: cover_end is the
// end of the run of units that these steps write, whose last unit's lane
// writes them itself. The SPLIT code is a separate instantiation because
// compiled into the same kernel as the others it costs them registers and
// speed even where it does not run.
template <bool ALIGNED, int UPL, bool GUARD, int MAP = 0, bool SPLIT = false>
__device__ __forceinline__ void enc_step(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                         int64_t first, int stride, int64_t units, const MapCtx &mc,
                                         int64_t cover_end = 0)
{
    static_assert(!(ALIGNED && SPLIT), "a split store needs a misaligned destination");
    uint32_t w[UPL][3];
    uint32_t lw[UPL];  // SPLIT, lane 0: the last input dword of the unit before its own
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        lw[k] = 0;
        if (!GUARD || u < units) {
            if (ALIGNED) {  // streamed: read once, so non-temporal
                const uint32_t *p = (const uint32_t *)(src + 12 * u);
                w[k][0] = __builtin_nontemporal_load(p);
                w[k][1] = __builtin_nontemporal_load(p + 1);
                w[k][2] = __builtin_nontemporal_load(p + 2);
            } else {
                load12(src + 12 * u, w[k][0], w[k][1], w[k][2]);
                if (SPLIT && __lane_id() == 0 && u > 0) {
                    uint32_t x[1];
                    load_words<1>(src + 12 * u - 4, x);
                    lw[k] = x[0];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        if constexpr (!SPLIT) {
            if (!GUARD || u < units) {
                uint32_t o[4];
                enc_unit_m<MAP>(w[k][0], w[k][1], w[k][2], mc, o[0], o[1], o[2], o[3]);
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
        } else {
            const bool live = !GUARD || u < units;
            uint32_t o[4] = {0, 0, 0, 0};
            if (live) enc_unit_m<MAP>(w[k][0], w[k][1], w[k][2], mc, o[0], o[1], o[2], o[3]);
            uint32_t pw = wave_shr1(o[3]);
            if (live) {
                const bool lane0 = __lane_id() == 0;
                if (lane0 && u > 0) {  // the last quad of the unit before: its last 3 bytes
                    uint32_t a, b, c;
                    enc_unit_m<MAP>(lw[k], lw[k], lw[k], mc, a, b, c, pw);
                }
                store_run_wave<4>(dst + 16 * u, o, pw, !lane0 || u > 0, u + 1 == cover_end);
            }
        }
    }
}

// One grid-stride step of the decode over one buffer (see enc_step for the
// guard, SPLIT and cover_end). Lanes of a wave hold consecutive units, so the
// lowest erring lane of a ballot has the wave's smallest offset; it alone
// performs the atomicMin (and, with bad_len, sets that length slot to -1).
template <bool ALIGNED, int UPL, bool GUARD, int MAP = 0, bool SPLIT = false>
__device__ __forceinline__ void dec_step(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                         int64_t first, int stride, int64_t L, const MapCtx &mc,
                                         unsigned long long *err_slot, int64_t cover_end = 0,
                                         int64_t *bad_len = nullptr)
{
    static_assert(!(ALIGNED && SPLIT), "a split store needs a misaligned destination");
    uint32_t w[UPL][4];
    uint32_t lw[UPL][2];  // SPLIT, lane 0: the last 8 characters of the unit before its own
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        lw[k][0] = lw[k][1] = 0;
        if (!GUARD || u < L) {
            if (ALIGNED) {  // streamed: read once, so non-temporal
                const uint32_t *p = (const uint32_t *)(src + 16 * u);
                w[k][0] = __builtin_nontemporal_load(p);
                w[k][1] = __builtin_nontemporal_load(p + 1);
                w[k][2] = __builtin_nontemporal_load(p + 2);
                w[k][3] = __builtin_nontemporal_load(p + 3);
            } else {
                load16(src + 16 * u, w[k][0], w[k][1], w[k][2], w[k][3]);
                if (SPLIT && __lane_id() == 0 && u > 0) load_words<2>(src + 16 * u - 8, lw[k]);
            }
        }
    }
    uint32_t bad_any = 0;
    uint32_t bad[UPL];
#pragma unroll
    for (int k = 0; k < UPL; k++) {
        const int64_t u = first + (int64_t)k * stride;
        bad[k] = 0;
        if constexpr (!SPLIT) {
            if (!GUARD || u < L) {
                uint32_t o[3];
                bad[k] = dec_unit_m<MAP>(w[k][0], w[k][1], w[k][2], w[k][3], mc, o[0], o[1], o[2]);
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
        } else {
            const bool live = !GUARD || u < L;
            uint32_t o[3] = {0, 0, 0};
            if (live) {
                bad[k] = dec_unit_m<MAP>(w[k][0], w[k][1], w[k][2], w[k][3], mc, o[0], o[1], o[2]);
                bad_any |= bad[k];
            }
            uint32_t pw = wave_shr1(o[2]);
            if (live) {
                const bool lane0 = __lane_id() == 0;
                if (lane0 && u > 0) {  // the last three bytes of the unit before: its last two quads
                    uint32_t a, b;
                    (void)dec_unit_m<MAP>(lw[k][0], lw[k][1], lw[k][0], lw[k][1], mc, a, b, pw);
                }
                store_run_wave<3>(dst + 12 * u, o, pw, !lane0 || u > 0, u + 1 == cover_end);
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
                const int64_t pos = 16 * u + dec_first_bad(w[k][0], w[k][1], w[k][2], w[k][3], mc.tab);
                atomicMin(err_slot, (unsigned long long)pos);
                if (bad_len) atomicExch((unsigned long long *)bad_len, ~0ull);
            }
        }
    }
}

}  // namespace b64dev
