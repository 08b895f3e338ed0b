/*
 * Plain, sequential CPU oracle of the entropy coder of the occupancy bytes: an own range
 * asymmetric numeral system (rANS) coder standing in for the closed ANS library the paper uses
 * for the geometry (Sec. 2.2 and Sec. 5: the octree's occupancy bytes are entropy coded, which
 * roughly halves their size).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code, header, table or helper with the
 * HIP path.
 *
 * The readings taken here (also listed with the design notes):
 *   A1  Model: one static table per stream over the 256 byte values, frequencies out of
 *       M = 2^12. With c_s the count of byte s among the T input bytes and P the number of
 *       distinct bytes, f_s = 1 + floor(c_s (M - P) / T) for a present byte (0 otherwise); the
 *       remainder M - sum f_s (less than P) is added to the most frequent byte (the smallest on
 *       a tie). start_s = f_0 + ... + f_{s-1}.
 *   A2  Coder: 32-bit rANS with byte-wise renormalisation (state in [L, 256 L), L = 2^23), the
 *       published byte-oriented rANS construction. The input is cut into chunks of K bytes (the
 *       last one shorter), each coded on its own from the state L: symbols taken last to first,
 *       for each one while x >= ((L >> 12) << 8) f_s a byte x mod 256 is emitted and x shifted
 *       right by 8, then x = (x / f_s) 2^12 + x mod f_s + start_s; finally the four bytes of x,
 *       least significant first. The chunk is stored as the emitted bytes in reverse order, so
 *       a decoder reads the final state (most significant byte first) and then the
 *       renormalisation bytes in the order it needs them.
 *   A3  Decoding a chunk: x from its first four bytes; per symbol, slot = x mod 2^12, s the byte
 *       with start_s <= slot < start_s + f_s, x = f_s (x >> 12) + slot - start_s, and while
 *       x < L, x = 256 x + the next byte. A chunk is accepted only if its first state is at
 *       least L (an encoder's final state always is) and it ends in the state L with every one
 *       of its bytes consumed. (So an accepted chunk never holds more than 2 bytes per symbol
 *       plus 4.)
 *
 * Every function returns a negative value on a bad argument (-1), a capacity overflow (-2) or a
 * chunk that does not decode as A3 requires (-3).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RANS_BITS 12
#define RANS_M (1u << RANS_BITS)
#define RANS_L (1u << 23)

/* A1: the frequency table of in[0..n-1]. Returns the number of distinct bytes. */
int orc_rans_table(const uint8_t *in, int64_t n, uint16_t *freq)
{
    if (n < 0 || !freq || (n > 0 && !in)) return -1;
    uint64_t cnt[256];
    memset(cnt, 0, sizeof cnt);
    for (int64_t i = 0; i < n; ++i) cnt[in[i]] += 1;
    int P = 0;
    for (int s = 0; s < 256; ++s) P += cnt[s] ? 1 : 0;
    uint32_t sum = 0;
    int most = 0;
    for (int s = 0; s < 256; ++s) {
        freq[s] = 0;
        if (cnt[s]) {
            freq[s] = (uint16_t)(1u + (uint32_t)(cnt[s] * (uint64_t)(RANS_M - (uint32_t)P) / (uint64_t)n));
            sum += freq[s];
        }
        if (cnt[s] > cnt[most]) most = s;
    }
    if (n > 0) freq[most] = (uint16_t)(freq[most] + (RANS_M - sum));
    return P;
}

int64_t orc_rans_chunks(int64_t n, int K)
{
    if (n < 0 || K < 1) return -1;
    return (n + K - 1) / K;
}

/* A2: encodes in[0..n-1] in chunks of K bytes with the table freq. off[nc + 1] receives each
 * chunk's first byte in `out` (off[nc] = total bytes); out (capacity cap, or NULL to count only)
 * the chunks one after the other. Returns the total bytes or a negative code. */
int64_t orc_rans_encode(const uint8_t *in, int64_t n, int K, const uint16_t *freq, int64_t *off,
                        uint8_t *out, int64_t cap)
{
    const int64_t nc = orc_rans_chunks(n, K);
    if (nc < 0 || !freq || !off || (n > 0 && !in)) return -1;
    uint32_t start[256];
    uint32_t acc = 0;
    for (int s = 0; s < 256; ++s) {
        start[s] = acc;
        acc += freq[s];
    }
    if (n > 0 && acc != RANS_M) return -1;
    /* a chunk's emitted bytes: at most 2 per symbol (a byte of frequency 1 costs 12 bits) + 4 */
    uint8_t *tmp = (uint8_t *)malloc((size_t)K * 2 + 4);
    if (!tmp) return -1;
    int64_t total = 0;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t b = c * K, e = (b + K <= n) ? b + K : n;
        uint32_t x = RANS_L;
        int64_t m = 0;
        for (int64_t i = e - 1; i >= b; --i) {
            const uint32_t s = in[i], f = freq[s];
            if (f == 0) {
                free(tmp);
                return -1;
            }
            const uint32_t xmax = ((RANS_L >> RANS_BITS) << 8) * f;
            while (x >= xmax) {
                tmp[m++] = (uint8_t)(x & 255u);
                x >>= 8;
            }
            x = ((x / f) << RANS_BITS) + (x % f) + start[s];
        }
        for (int k = 0; k < 4; ++k) {
            tmp[m++] = (uint8_t)(x & 255u);
            x >>= 8;
        }
        off[c] = total;
        if (out) {
            if (total + m > cap) {
                free(tmp);
                return -2;
            }
            for (int64_t k = 0; k < m; ++k) out[total + k] = tmp[m - 1 - k];
        }
        total += m;
    }
    off[nc] = total;
    free(tmp);
    return total;
}

/* A3: decodes the chunks of orc_rans_encode into out[0..n-1]. Returns 0 or a negative code. */
int orc_rans_decode(const int64_t *off, const uint8_t *data, int64_t n, int K, const uint16_t *freq,
                    uint8_t *out)
{
    const int64_t nc = orc_rans_chunks(n, K);
    if (nc < 0 || !freq || !off || (n > 0 && (!out || !data))) return -1;
    uint32_t start[257];
    uint8_t sym[RANS_M];
    uint32_t acc = 0;
    for (int s = 0; s < 256; ++s) {
        start[s] = acc;
        for (uint32_t j = 0; j < freq[s] && acc + j < RANS_M; ++j) sym[acc + j] = (uint8_t)s;
        acc += freq[s];
    }
    if (n > 0 && acc != RANS_M) return -3;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t b = c * K, e = (b + K <= n) ? b + K : n;
        const int64_t p0 = off[c], p1 = off[c + 1];
        if (p1 < p0 + 4) return -3;
        int64_t p = p0;
        uint32_t x = 0;
        for (int k = 0; k < 4; ++k) x = (x << 8) | data[p++];
        if (x < RANS_L) return -3;
        for (int64_t i = b; i < e; ++i) {
            const uint32_t slot = x & (RANS_M - 1u);
            const uint32_t s = sym[slot];
            x = freq[s] * (x >> RANS_BITS) + slot - start[s];
            while (x < RANS_L) {
                if (p >= p1) return -3;
                x = (x << 8) | data[p++];
            }
            out[i] = (uint8_t)s;
        }
        if (x != RANS_L || p != p1) return -3;
    }
    return 0;
}
