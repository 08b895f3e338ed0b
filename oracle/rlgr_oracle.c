/*
 * Plain, sequential CPU oracle of the block-parallel entropy coder of the quantized RAHT
 * coefficients (Sec. 3.4 "Quantization and Entropy Coding": run-length / adaptive Golomb-Rice
 * coding, RLGR, of independent blocks of consecutive coefficients of one channel).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code, header, table or helper with the
 * HIP path.
 *
 * The paper names the coder (Malvar's adaptive run-length / Golomb-Rice coder) and the block
 * partition, and gives no parameters. The readings taken here (also listed with the design
 * notes):
 *   G1  Blocks: channel c's Nv coefficients, in coefficient order, cut into blocks of B values
 *       (the last one shorter); block b = j * C + c covers coefficients j*B .. j*B + B - 1 of
 *       channel c. Every block is coded on its own, from the initial coder state, into a whole
 *       number of 32-bit words; bits fill a word from its most significant bit down, and the
 *       unused low bits of a block's last word are zero.
 *   G2  Coder state: two adaptive parameters held with 3 fractional bits, kp for the run mode
 *       (k = kp >> 3) and krp for the Golomb-Rice code (kr = krp >> 3), both starting at 8
 *       (k = kr = 1) and kept within 0 .. 80.
 *   G3  Run mode (k > 0): a run of zeros is sent as one 0 bit for every 2^k zeros (each one
 *       raising kp by 4), then a 1 bit and the remaining count (< 2^k) in k bits. Unless the
 *       block ends there, the nonzero value that ends the run follows as its sign bit (1 =
 *       negative) and the Golomb-Rice code of its magnitude minus one; kp then drops by 6.
 *   G4  Golomb-Rice mode (k = 0): each value v is sent as the Golomb-Rice code of
 *       u = 2v (v >= 0) or -2v - 1 (v < 0); kp rises by 3 after u = 0 and drops by 3 otherwise.
 *   G5  Golomb-Rice code of u with kr = krp >> 3: q = u >> kr ones, a 0, then the kr low bits of
 *       u; if q >= 24, 24 ones and then u in 32 bits instead (an escape for the large
 *       low-frequency coefficients, which would otherwise take up to 2^31 ones). krp then
 *       drops by 2 if q = 0 and rises by q if q > 1.
 *
 * Every function returns a negative value on a bad argument, a capacity overflow or (decoding)
 * a block whose words do not decode to exactly the block's length (with at most the last
 * word's low bits left over).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RLGR_FRAC 3
#define RLGR_PMAX 80
#define RLGR_START 8
#define RLGR_RUN_UP 4
#define RLGR_RUN_DOWN 6
#define RLGR_GR_UP 3
#define RLGR_GR_DOWN 3
#define RLGR_ESCAPE 24

/* ------------------------------------------------------------------------- bit writer */
typedef struct {
    uint32_t *w;      /* output words (NULL: count only) */
    int64_t cap;      /* words available */
    int64_t nbits;    /* bits written so far */
    int overflow;
} orc_bw;

static void bw_bit(orc_bw *b, uint32_t bit)
{
    const int64_t word = b->nbits >> 5;
    if (b->w) {
        if (word >= b->cap) {
            b->overflow = 1;
        } else {
            if ((b->nbits & 31) == 0) b->w[word] = 0;
            if (bit) b->w[word] |= 1u << (31 - (b->nbits & 31));
        }
    }
    b->nbits += 1;
}

/* the n low bits of v, most significant first */
static void bw_bits(orc_bw *b, uint64_t v, int n)
{
    for (int i = n - 1; i >= 0; --i) bw_bit(b, (uint32_t)((v >> i) & 1u));
}

static int clampp(int p) { return p < 0 ? 0 : (p > RLGR_PMAX ? RLGR_PMAX : p); }

/* G5: Golomb-Rice code of u, adapting *krp */
static void gr_put(orc_bw *b, uint64_t u, int *krp)
{
    const int kr = *krp >> RLGR_FRAC;
    const uint64_t q = u >> kr;
    if (q < RLGR_ESCAPE) {
        for (uint64_t i = 0; i < q; ++i) bw_bit(b, 1);
        bw_bit(b, 0);
        bw_bits(b, u, kr);
    } else {
        for (int i = 0; i < RLGR_ESCAPE; ++i) bw_bit(b, 1);
        bw_bits(b, u, 32);
    }
    if (q == 0) *krp = clampp(*krp - 2);
    else if (q > 1) *krp = clampp(*krp + (int)(q > RLGR_PMAX ? RLGR_PMAX : q));
}

/* Codes one block x[0..L-1] (stride `stride` between its values) into b. */
static void rlgr_block(orc_bw *b, const int32_t *x, int64_t L, int64_t stride)
{
    int kp = RLGR_START, krp = RLGR_START;
    int64_t pos = 0;
    while (pos < L) {
        int k = kp >> RLGR_FRAC;
        if (k > 0) { /* G3: run mode */
            int64_t run = 0;
            while (pos + run < L && x[(pos + run) * stride] == 0) ++run;
            while (run >= ((int64_t)1 << k)) {
                bw_bit(b, 0);
                run -= (int64_t)1 << k;
                pos += (int64_t)1 << k;
                kp = clampp(kp + RLGR_RUN_UP);
                k = kp >> RLGR_FRAC;
            }
            bw_bit(b, 1);
            bw_bits(b, (uint64_t)run, k);
            pos += run;
            if (pos == L) break;
            const int64_t v = x[pos * stride];
            pos += 1;
            bw_bit(b, v < 0 ? 1u : 0u);
            gr_put(b, (uint64_t)(v < 0 ? -v : v) - 1u, &krp);
            kp = clampp(kp - RLGR_RUN_DOWN);
        } else { /* G4: Golomb-Rice mode */
            const int64_t v = x[pos * stride];
            pos += 1;
            const uint64_t u = v >= 0 ? (uint64_t)(2 * v) : (uint64_t)(-2 * v - 1);
            gr_put(b, u, &krp);
            kp = clampp(u == 0 ? kp + RLGR_GR_UP : kp - RLGR_GR_DOWN);
        }
    }
}

/* Number of blocks of a [nv][C] coefficient matrix with blocks of B values (G1). */
int64_t orc_rlgr_blocks(int64_t nv, int C, int B)
{
    if (nv < 0 || C < 1 || B < 1) return -1;
    return (nv + B - 1) / B * C;
}

/*
 * Encodes Q [nv][C] (row-major int32) with blocks of B values. off[NB + 1] receives each block's
 * first word (off[NB] = total words); words (capacity cap) the coded blocks, one after the
 * other. Returns the total number of words, or -1 (bad argument) / -2 (capacity).
 */
int64_t orc_rlgr_encode(const int32_t *Q, int64_t nv, int C, int B, int64_t *off, uint32_t *words,
                        int64_t cap)
{
    const int64_t NB = orc_rlgr_blocks(nv, C, B);
    if (NB < 0 || !off || (nv > 0 && !Q)) return -1;
    int64_t total = 0;
    for (int64_t bi = 0; bi < NB; ++bi) {
        const int64_t j = bi / C, c = bi % C;
        const int64_t i0 = j * B, L = (i0 + B <= nv) ? B : nv - i0;
        orc_bw b = {words ? words + total : NULL, words ? cap - total : 0, 0, 0};
        rlgr_block(&b, Q + i0 * C + c, L, C);
        if (b.overflow) return -2;
        off[bi] = total;
        total += (b.nbits + 31) >> 5;
        if (words && total > cap) return -2;
    }
    off[NB] = total;
    return total;
}

/* ------------------------------------------------------------------------- bit reader */
typedef struct {
    const uint32_t *w;
    int64_t nwords;
    int64_t pos; /* bit position */
    int bad;
} orc_br;

static uint32_t br_bit(orc_br *r)
{
    const int64_t word = r->pos >> 5;
    if (word >= r->nwords) {
        r->bad = 1;
        return 0;
    }
    const uint32_t bit = (r->w[word] >> (31 - (r->pos & 31))) & 1u;
    r->pos += 1;
    return bit;
}

static uint64_t br_bits(orc_br *r, int n)
{
    uint64_t v = 0;
    for (int i = 0; i < n; ++i) v = (v << 1) | br_bit(r);
    return v;
}

static uint64_t gr_get(orc_br *r, int *krp)
{
    const int kr = *krp >> RLGR_FRAC;
    uint64_t q = 0;
    while (q < RLGR_ESCAPE && br_bit(r) == 1 && !r->bad) ++q;
    uint64_t u;
    if (q == RLGR_ESCAPE) {
        u = br_bits(r, 32);
        q = u >> kr;
    } else {
        u = (q << kr) | br_bits(r, kr);
    }
    if (q == 0) *krp = clampp(*krp - 2);
    else if (q > 1) *krp = clampp(*krp + (int)(q > RLGR_PMAX ? RLGR_PMAX : q));
    return u;
}

/* Decodes one block of L values from r into x (stride `stride`); 0, or -3 if the code does not
 * decode to exactly L values. */
static int unrlgr_block(orc_br *r, int32_t *x, int64_t L, int64_t stride)
{
    int kp = RLGR_START, krp = RLGR_START;
    int64_t pos = 0;
    while (pos < L) {
        int k = kp >> RLGR_FRAC;
        if (k > 0) {
            while (br_bit(r) == 0) {
                if (r->bad || pos + ((int64_t)1 << k) > L) return -3;
                for (int64_t i = 0; i < ((int64_t)1 << k); ++i) x[(pos + i) * stride] = 0;
                pos += (int64_t)1 << k;
                kp = clampp(kp + RLGR_RUN_UP);
                k = kp >> RLGR_FRAC;
            }
            if (r->bad) return -3;
            const int64_t run = (int64_t)br_bits(r, k);
            if (pos + run > L) return -3;
            for (int64_t i = 0; i < run; ++i) x[(pos + i) * stride] = 0;
            pos += run;
            if (pos == L) break;
            const uint32_t s = br_bit(r);
            const uint64_t m = gr_get(r, &krp) + 1u;
            if (r->bad || m > 2147483648ull || (!s && m > 2147483647ull)) return -3;
            x[pos * stride] = s ? (int32_t)(-(int64_t)m) : (int32_t)m;
            pos += 1;
            kp = clampp(kp - RLGR_RUN_DOWN);
        } else {
            const uint64_t u = gr_get(r, &krp);
            if (r->bad || u > 4294967295ull) return -3;
            x[pos * stride] = (u & 1u) ? (int32_t)(-(int64_t)((u + 1) >> 1)) : (int32_t)(u >> 1);
            pos += 1;
            kp = clampp(u == 0 ? kp + RLGR_GR_UP : kp - RLGR_GR_DOWN);
        }
    }
    /* the block's code fills exactly its words (only the last one's low bits are padding) */
    if (r->bad || ((r->pos + 31) >> 5) != r->nwords) return -3;
    return 0;
}

/* Decodes the blocks coded by orc_rlgr_encode into Q [nv][C]. Returns 0, -1 (bad argument) or
 * -3 (a block that does not decode to its length within its words). */
int orc_rlgr_decode(const int64_t *off, const uint32_t *words, int64_t nv, int C, int B, int32_t *Q)
{
    const int64_t NB = orc_rlgr_blocks(nv, C, B);
    if (NB < 0 || !off || (nv > 0 && (!Q || !words))) return -1;
    for (int64_t bi = 0; bi < NB; ++bi) {
        const int64_t j = bi / C, c = bi % C;
        const int64_t i0 = j * B, L = (i0 + B <= nv) ? B : nv - i0;
        if (off[bi + 1] < off[bi]) return -3;
        orc_br r = {words + off[bi], off[bi + 1] - off[bi], 0, 0};
        const int st = unrlgr_block(&r, Q + i0 * C + c, L, C);
        if (st) return st;
    }
    return 0;
}
