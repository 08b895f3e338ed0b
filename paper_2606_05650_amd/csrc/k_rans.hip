// Entropy coding of the occupancy bytes: an own range-ANS (rANS) coder standing in for the closed
// ANS library the paper uses for the geometry (Sec. 2.2 and Sec. 5). The paper gives no
// parameters; this coder takes these choices:
//   * one static table per stream over the 256 byte values with frequencies out of M = 2^12:
//     with c_s the count of byte s among the T input bytes and P the number of distinct bytes,
//     f_s = 1 + floor(c_s (M - P) / T) for a present byte, the remainder M - sum f_s going to the
//     most frequent byte (the smallest on a tie);
//   * 32-bit rANS with byte-wise renormalisation (state in [2^23, 2^31)), the input cut into
//     chunks of K bytes coded independently from the state 2^23; a chunk's symbols are coded
//     last to first and its bytes stored in reverse emission order (final state first, most
//     significant byte first), so that decoding reads forward;
//   * a decoder accepts a chunk only if its first state is at least 2^23 (an encoder's always
//     is) and it ends in the state 2^23 with all its bytes consumed; an accepted chunk therefore
//     holds at most 2 K + 4 bytes.
// Encode: the byte counts (LDS histograms added to device-wide counters), the table (one wave),
// then one thread per chunk codes its chunk into a scratch area, the chunks' offsets come from a
// decoupled look-back over waves of 64 chunks, and each thread copies its bytes to their place.
// Decode: one thread per chunk.
#include "gsc_device.h"

#include <cstring>

namespace gsc {

constexpr uint32_t RANS_BITS = 12, RANS_M = 1u << RANS_BITS, RANS_L = 1u << 23;
constexpr int RANS_THREADS = WAVE;  // one wave per 64 chunks
constexpr int RANS_HIST_THREADS = 256;
constexpr int RANS_HCOPIES = 8;  // LDS histograms per histogram workgroup
constexpr int RANS_HIST_BLOCKS = 4;  // 16-byte blocks per thread and round of the histogram

struct RansArgs {
    const uint8_t *in;
    uint64_t n;
    uint32_t K, nc;
    uint8_t *out;        // stream (encode) or decoded bytes (decode)
    uint64_t cap;        // encode: stream capacity; decode: input stream bytes
    const uint8_t *src;  // decode: the stream
    uint32_t *ws;        // [0] error; encode: [2..257] the byte counts
    uint64_t *status;    // look-back status of the chunk waves
    uint32_t hblocks;    // encode: histogram workgroups
    uint8_t *tmp;        // per-chunk scratch, chunk c at c * tmp_stride
    uint64_t tmp_stride;
    uint32_t stage;      // LDS bytes of a wave's staged input (encode) or stream (decode); 0: none
    int32_t *info;
};

// Chunks of at most RANS_STAGE_K bytes are coded from LDS: a wave first copies its chunks' input
// (encode) or stream bytes (decode) there with coalesced 16-byte loads, so the per-symbol loops
// hold no global load. (On gfx950 one counter tracks global loads and stores together, so a wait
// for a load inside those loops would also wait for every output store still in flight.)
constexpr uint32_t RANS_STAGE_K = 1024;

__device__ inline void rans_error(uint32_t *err, uint32_t code)
{
    atomicCAS(err, 0u, code);
}

// Workspace: the error word and the byte counts, the look-back words of the chunk waves, the
// chunks' scratch areas (256-byte aligned).
__host__ __device__ inline uint64_t rans_status_words(uint64_t nc) { return (nc + RANS_THREADS - 1) / RANS_THREADS + 1; }
__host__ __device__ inline uint64_t rans_tmp_stride(uint32_t K) { return ((uint64_t)2 * K + 4 + 15) / 16 * 16; }
// histogram workgroups: each thread counts RANS_HIST_BLOCKS 16-byte blocks per round
__host__ __device__ inline uint32_t rans_hist_blocks(uint64_t n)
{
    const uint64_t per = (uint64_t)RANS_HIST_THREADS * 16 * RANS_HIST_BLOCKS;
    const uint64_t hw = (n + per - 1) / per;
    return (uint32_t)(hw < 1 ? 1 : hw > 1024 ? 1024 : hw);
}
__host__ __device__ inline uint64_t rans_align256(uint64_t v) { return (v + 255) / 256 * 256; }
constexpr uint32_t RANS_STATUS_OFF = 1040;  // bytes: after the 258 counter words, 8-aligned
__host__ __device__ inline uint64_t rans_head_words(uint64_t nc) { return RANS_STATUS_OFF / 4 + 2 * rans_status_words(nc); }
__host__ __device__ inline uint64_t rans_tmp_off(uint64_t nc) { return rans_align256(4 * rans_head_words(nc)); }

// Stream: header, freq u16[256], offsets u32[nc + 1] (bytes into the data area), data.
__device__ inline uint64_t rans_data_off(uint32_t nc) { return sizeof(gsc_rans_header) + 512ull + 4ull * (nc + 1); }

// ---------------------------------------------------------------------------------- encode
// The info words (d_info[0..3]): the device status, n, and the stream bytes (encode, 0 on an
// error), after every other kernel of the call.
__global__ __launch_bounds__(WAVE) void k_rans_info(RansArgs a, int decode)
{
    if (threadIdx.x != 0) return;
    const uint32_t e = __hip_atomic_load(&a.ws[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.info[0] = (int32_t)e;
    a.info[1] = (int32_t)(uint32_t)a.n;
    uint64_t bytes = 0;
    if (!decode && e == 0) {
        uint32_t *tot = reinterpret_cast<uint32_t *>(a.out + sizeof(gsc_rans_header) + 512) + a.nc;
        bytes = rans_data_off(a.nc) + __hip_atomic_load(tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    a.info[2] = (int32_t)(uint32_t)(bytes & 0xFFFFFFFFu);
    a.info[3] = (int32_t)(uint32_t)(bytes >> 32);
}

__global__ __launch_bounds__(RANS_HIST_THREADS) void k_rans_hist(RansArgs a)
{
    // RANS_HCOPIES histograms per workgroup (thread t adds to copy t mod RANS_HCOPIES, the copies
    // 257 words apart so that one byte's counters lie in different banks), so that lanes holding
    // the same frequent byte seldom hit one LDS word
    __shared__ uint32_t s_h[RANS_HCOPIES][257];
    for (uint32_t i = threadIdx.x; i < RANS_HCOPIES * 257; i += RANS_HIST_THREADS) (&s_h[0][0])[i] = 0;
    __syncthreads();
    uint32_t *h = s_h[threadIdx.x % RANS_HCOPIES];
    // aligned 16-byte blocks that hold input bytes; a block reaching outside the input (only the
    // first and the last can) is read byte by byte
    const uint64_t lo = reinterpret_cast<uint64_t>(a.in), hi = lo + a.n;
    const uint64_t b0 = lo & ~15ull, nb = (hi + 15 - b0) / 16;
    // blocks k0 + u * stride (u < RANS_HIST_BLOCKS) of each round are loaded before any is counted
    const uint64_t stride = (uint64_t)gridDim.x * RANS_HIST_THREADS;
    for (uint64_t k0 = (uint64_t)blockIdx.x * RANS_HIST_THREADS + threadIdx.x; k0 < nb; k0 += RANS_HIST_BLOCKS * stride) {
        gi4 v[RANS_HIST_BLOCKS];
#pragma unroll
        for (int u = 0; u < RANS_HIST_BLOCKS; ++u) {
            const uint64_t k = k0 + u * stride, p = b0 + 16 * k;
            const bool full = k < nb && p >= lo && p + 16 <= hi;
            // (a block of the workspace stands in for one past the end or reaching outside the input)
            v[u] = *reinterpret_cast<const GAS gi4 *>(full ? p : reinterpret_cast<uint64_t>(a.ws));
        }
#pragma unroll
        for (int u = 0; u < RANS_HIST_BLOCKS; ++u) {
            const uint64_t k = k0 + u * stride, p = b0 + 16 * k;
            if (k >= nb) break;
            if (p >= lo && p + 16 <= hi) {
                const uint32_t w[4] = {(uint32_t)v[u].x, (uint32_t)v[u].y, (uint32_t)v[u].z, (uint32_t)v[u].w};
#pragma unroll
                for (int q = 0; q < 16; ++q) atomicAdd(&h[(w[q / 4] >> (8 * (q % 4))) & 255u], 1u);
            } else {
                for (uint64_t q = p < lo ? lo : p; q < p + 16 && q < hi; ++q)
                    atomicAdd(&h[*reinterpret_cast<const GAS uint8_t *>(q)], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < 256; s += RANS_HIST_THREADS) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < RANS_HCOPIES; ++q) c += s_h[q][s];
        if (c) atomicAdd(&a.ws[2 + s], c);
    }
}

// Clears the error and count words and the look-back words (encode) or the error word (decode).
__global__ __launch_bounds__(256) void k_rans_zero(uint32_t *ws, uint32_t nwords)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nwords; i += gridDim.x * 256) ws[i] = 0;
}

// One wave: the table from the byte counts, written to the stream (the header comes with the
// last chunk). An empty input gets its whole stream here.
__global__ __launch_bounds__(WAVE) void k_rans_table(RansArgs a)
{
    const uint32_t lane = lane_id();
    GAS uint16_t *tab = gp(reinterpret_cast<uint16_t *>(a.out + sizeof(gsc_rans_header)));
    if (a.nc == 0) {
        if (lane == 0) {  // an empty input: the header, a zero table and one offset
            gsc_rans_header *h = reinterpret_cast<gsc_rans_header *>(a.out);
            h->magic = GSC_RANS_MAGIC;
            h->version = GSC_VERSION;
            h->n = 0;
            h->K = a.K;
            h->nchunks = 0;
            h->total = 0;
            h->reserved = 0;
            *reinterpret_cast<uint32_t *>(a.out + sizeof(gsc_rans_header) + 512) = 0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tab[4 * lane + q] = 0;
        return;
    }
    uint32_t c[4], f[4];
    uint32_t present = 0, sum = 0;
    uint32_t best = 0, best_s = 0;  // count and byte of this lane's most frequent byte
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t s = lane * 4 + q;
        c[q] = __hip_atomic_load(&a.ws[2 + s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        present += c[q] ? 1u : 0u;
        if (c[q] > best) {
            best = c[q];
            best_s = s;
        }
    }
    uint32_t P = present;
    for (int o = 32; o > 0; o >>= 1) P += __shfl_xor(P, o, WAVE);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = c[q] ? 1u + (uint32_t)((uint64_t)c[q] * (RANS_M - P) / a.n) : 0u;
        sum += f[q];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, WAVE);
    // the most frequent byte, the smallest on a tie (lanes hold increasing bytes)
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t bc = __shfl_xor(best, o, WAVE), bs = __shfl_xor(best_s, o, WAVE);
        if (bc > best || (bc == best && bs < best_s)) {
            best = bc;
            best_s = bs;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t s = lane * 4 + q;
        tab[s] = (uint16_t)(f[q] + (s == best_s ? RANS_M - sum : 0u));
    }
}

// The encoder's table in LDS, one entry per byte value s (f its frequency, st its start):
//   x = f 2^19, the renormalisation bound;
//   y = ceil(2^(31 + l) / f) with l = ceil(log2 f): for every state x < 2^31, which is where the
//       coder divides, floor(x / f) = (x y) >> (31 + l), the multiply-high division by an
//       invariant integer of Granlund and Montgomery (1994), exact here because y < 2^32 and
//       y f - 2^(31 + l) < 2^l;
//   z = (M - f) | (31 + l) << 24: with q = floor(x / f), the coded state (q << 12) + x - q f + st
//       is x + q (M - f) + st, a 24-bit multiply-add (q < 2^19 and M - f < 2^12), whose operand
//       bits 24..31 are ignored, and the shift (31 + l) of the division is z >> 24;
//   w = st, and f itself in bits 16..28 (0 marks a byte absent from the table).
// Built by the workgroup's one wave, four bytes a lane.
__device__ inline void enc_table(const GAS uint16_t *tab, uint4 *s_enc)
{
    const uint32_t lane = lane_id();
    uint32_t f[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = tab[4 * lane + q];
        sum += f[q];
    }
    uint32_t st = wave_incl_scan(sum) - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t fq = f[q];
        const uint32_t l = fq > 1 ? 32u - (uint32_t)__clz(fq - 1) : 0u;
        const uint32_t y = fq ? (uint32_t)(((1ull << (31 + l)) + fq - 1) / fq) : 0u;
        s_enc[4 * lane + q] = make_uint4(fq << 19, y, ((RANS_M - fq) & 0xFFFFFFu) | ((31u + l) << 24),
                                         (st & 0xFFFFu) | (fq << 16));
        st += fq;
    }
}

// Reads the aligned 8-byte block at address p of the input [lo, hi). The vector load is issued
// on every path (at the valid 8-aligned address `safe` when the block reaches outside the
// input, which only the input's first and last blocks can), and such a block is then read again
// byte by byte, its other bytes zero: so no branch joins with the load still in flight.
__device__ inline uint2 in_block8(uint64_t p, uint64_t lo, uint64_t hi, uint64_t safe)
{
    const bool full = p >= lo && p + 8 <= hi;
    uint64_t v = *reinterpret_cast<const GAS uint64_t *>(full ? p : safe);
    if (!full) {
        v = 0;
        for (uint32_t q = 0; q < 8; ++q)
            if (p + q >= lo && p + q < hi) v |= (uint64_t)*reinterpret_cast<const GAS uint8_t *>(p + q) << (8 * q);
    }
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// The coding state of one chunk. Bytes are emitted low first and stored in reverse emission
// order, so the emitted bytes are written downwards from the end of the chunk's scratch area:
// acc holds the na most recent ones (acc byte 0 at the lowest address), and every complete
// 4-byte word at the top is stored as soon as it is full (top is the end of the bytes not yet
// stored, 4-aligned).
struct EncState {
    uint32_t x, na, top;
    uint64_t acc;
    bool bad;
};

// Codes one byte, given its table entry t (enc_table).
__device__ inline void enc_step(EncState &E, const uint4 &t, GAS uint32_t *tw)
{
    E.bad |= t.w < (1u << 16);  // (an absent byte: impossible with the stream's own table)
    // renormalisation: at most two bytes, since x < 2^31 and the bound is f 2^19 >= 2^19
    uint32_t x = E.x;
    const bool e1 = x >= t.x;
    const uint32_t x1 = e1 ? x >> 8 : x;
    const bool e2 = x1 >= t.x;
    const uint32_t k = (e1 ? 1u : 0u) + (e2 ? 1u : 0u);
    // the emitted bytes, low first, prepended to acc (nothing when k = 0)
    const uint32_t v = e2 ? __builtin_amdgcn_perm(0u, x, 0x0c0c0001u) : (e1 ? (x & 255u) : 0u);
    E.acc = (E.acc << (8 * k)) | v;
    E.na += k;
    x = e2 ? x1 >> 8 : x1;
    if (E.na >= 4) {
        E.top -= 4;
        tw[E.top / 4] = (uint32_t)(E.acc >> (8 * (E.na - 4)));
        E.na -= 4;
    }
    const uint32_t q = (uint32_t)(((uint64_t)x * t.y) >> (t.z >> 24));
    E.x = __umul24(q, t.z) + x + (t.w & 0xFFFFu);  // (__umul24 reads bits 0..23 of each operand)
}

// Copies the aligned 16-byte blocks that cover the addresses [lo_r, hi_r) of a buffer [lo, hi)
// to s (block i of the copy: address (lo_r & ~15) + 16 i), by the calling wave; bytes outside
// the buffer (only its first and last blocks hold any) are read one by one as zero, after a
// vector load from `safe` (16 readable bytes, 4-aligned) that keeps every path's load count
// equal. Returns the copy's first address. Four loads per lane are issued before their stores.
__device__ inline uint64_t stage_blocks(uint8_t *s, uint64_t lo_r, uint64_t hi_r, uint64_t lo, uint64_t hi,
                                        uint64_t safe)
{
    const uint32_t lane = lane_id();
    const uint64_t sb = lo_r & ~15ull;
    const uint32_t nblk = hi_r > lo_r ? (uint32_t)((hi_r - sb + 15) / 16) : 0u;
    for (uint32_t i0 = 0; i0 < nblk; i0 += 4 * WAVE) {
        gi4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + u * WAVE + lane;
            const uint64_t p = sb + 16ull * min(i, nblk - 1);
            const bool full = p >= lo && p + 16 <= hi;
            v[u] = *reinterpret_cast<const GAS gi4 *>(full ? p : safe);
            if (!full) {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
                for (uint32_t q = 0; q < 16; ++q)
                    if (p + q >= lo && p + q < hi) w[q / 4] |= (uint32_t)*reinterpret_cast<const GAS uint8_t *>(p + q) << (8 * (q % 4));
                v[u] = gi4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + u * WAVE + lane;
            if (i < nblk) *reinterpret_cast<gi4 *>(s + 16 * i) = v[u];
        }
    }
    return sb;
}

// Thread c codes chunk c into its scratch area, the wave's chunks find their offsets by
// look-back, and each thread copies its bytes to their place.
template <bool STAGED>
__global__ __launch_bounds__(RANS_THREADS) void k_rans_encode(RansArgs a)
{
    extern __shared__ gi4 s_dyn[];
    __shared__ uint4 s_enc[256];
    const GAS uint16_t *tab = gp(reinterpret_cast<const uint16_t *>(a.out + sizeof(gsc_rans_header)));
    enc_table(tab, s_enc);
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t c = blockIdx.x * RANS_THREADS + lane;
    const uint32_t S = (uint32_t)a.tmp_stride;
    GAS uint8_t *tmp = gp(a.tmp) + (uint64_t)c * S;
    EncState E;
    E.x = RANS_L;
    E.na = 0;
    E.top = S;
    E.acc = 0;
    E.bad = false;
    uint32_t m = 0;  // bytes of this chunk
    // staged: the wave's chunks are consecutive, so one copy holds all their bytes (made by every
    // lane, also those past the last chunk)
    uint8_t *s_in = reinterpret_cast<uint8_t *>(s_dyn);
    uint64_t sb = 0;
    if (STAGED) {
        const uint64_t lo = reinterpret_cast<uint64_t>(a.in), hi = lo + a.n;
        const uint64_t w0 = lo + (uint64_t)blockIdx.x * RANS_THREADS * a.K;
        sb = stage_blocks(s_in, w0, min(w0 + (uint64_t)RANS_THREADS * a.K, hi), lo, hi, reinterpret_cast<uint64_t>(a.ws));
        __syncthreads();
    }
    if (c < a.nc) {
        GAS uint32_t *tw = reinterpret_cast<GAS uint32_t *>(tmp);
        const uint64_t lo = reinterpret_cast<uint64_t>(a.in), hi = lo + a.n;
        const uint64_t b = lo + (uint64_t)c * a.K, e = min(b + a.K, hi);  // the chunk's addresses
        const uint64_t safe = reinterpret_cast<uint64_t>(a.ws);          // (8-aligned, >= 16 bytes)
        auto block8 = [&](uint64_t q) -> uint2 {
            if (STAGED) return *reinterpret_cast<const uint2 *>(s_in + (q - sb));
            return in_block8(q, lo, hi, safe);
        };
        // the chunk's 8-byte blocks from the last down, the next one loaded before this one is coded
        uint64_t p = (e - 1) & ~7ull;
        uint2 cur = block8(p);
        for (;;) {
            const bool more = p > b;
            const uint2 nxt = block8(more ? p - 8 : p);
            // the table entries of the block's eight bytes, read before any is used
            const uint32_t w[2] = {cur.x, cur.y};
            uint4 t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) t[q] = s_enc[(w[q / 4] >> (8 * (q % 4))) & 255u];
            if (p >= b && p + 8 <= e) {  // a block inside the chunk (all but its first and last)
#pragma unroll
                for (int q = 7; q >= 0; --q) enc_step(E, t[q], tw);
            } else {
#pragma unroll
                for (int q = 7; q >= 0; --q)
                    if (p + q >= b && p + q < e) enc_step(E, t[q], tw);
            }
            if (!more) break;
            p -= 8;
            cur = nxt;
        }
        // the final state, low byte emitted first (stored most significant first)
        E.acc = (E.acc << 32) | __builtin_bswap32(E.x);
        E.na += 4;
        m = S - E.top + E.na;
        if (E.na >= 4) {
            E.top -= 4;
            tw[E.top / 4] = (uint32_t)(E.acc >> (8 * (E.na - 4)));
            E.na -= 4;
        }
        if (E.na > 0) tw[E.top / 4 - 1] = (uint32_t)(E.acc << (8 * (4 - E.na)));
        if (E.bad) rans_error(a.ws, GSC_ERR_INTERNAL);  // (impossible with the stream's own table)
    }
    // the chunks' offsets: a scan over the wave, then the look-back over the waves
    uint64_t incl = m;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o, WAVE);
        if (lane >= (uint32_t)o) incl += t;
    }
    const uint64_t wave_total = __shfl(incl, WAVE - 1, WAVE);
    const uint64_t base = lookback_wave<OpSum>(a.status, 1, blockIdx.x, wave_total, reinterpret_cast<Ctrl *>(a.ws));
    const uint64_t first = base + incl - m;
    const uint64_t d0 = rans_data_off(a.nc);
    const uint64_t room = a.cap > d0 ? a.cap - d0 : 0;
    GAS uint32_t *offs = gp(reinterpret_cast<uint32_t *>(a.out + sizeof(gsc_rans_header) + 512));
    if (c < a.nc) {
        if (first + m > room || first + m > 0xFFFFFFFFull) {
            rans_error(a.ws, GSC_ERR_CAPACITY);
        } else {
            offs[c] = (uint32_t)first;
            // copy tmp[S - m, S) to the chunk's place: bytes up to the first 4-aligned destination
            // address, whole words (each from two aligned source words), then the last bytes
            const uint64_t src = reinterpret_cast<uint64_t>(a.tmp) + (uint64_t)c * S + (S - m);
            const uint64_t dst = reinterpret_cast<uint64_t>(a.out) + d0 + first;
            const uint32_t h = min(m, (uint32_t)((4u - (uint32_t)(dst & 3u)) & 3u));
            for (uint32_t k = 0; k < h; ++k)
                *reinterpret_cast<GAS uint8_t *>(dst + k) = *reinterpret_cast<const GAS uint8_t *>(src + k);
            const uint32_t nw = (m - h) / 4;
            const uint64_t s1 = src + h;
            const uint32_t dl = (uint32_t)(s1 & 3u);
            const GAS uint32_t *sw = reinterpret_cast<const GAS uint32_t *>(s1 - dl);
            GAS uint32_t *dw = reinterpret_cast<GAS uint32_t *>(dst + h);
            constexpr uint32_t CU = 8;  // words per step: the loads of a step are issued together
            uint32_t i = 0;
            if (dl == 0) {
                for (; i + CU <= nw; i += CU) {
                    uint32_t v[CU];
#pragma unroll
                    for (uint32_t u = 0; u < CU; ++u) v[u] = sw[i + u];
#pragma unroll
                    for (uint32_t u = 0; u < CU; ++u) dw[i + u] = v[u];
                }
                for (; i < nw; ++i) dw[i] = sw[i];
            } else {
                // a source word past the last whole one is read only when dl > 0, and then it still
                // starts before the end of the scratch area (which is 4-aligned)
                for (; i + CU <= nw; i += CU) {
                    uint32_t v[CU + 1];
#pragma unroll
                    for (uint32_t u = 0; u <= CU; ++u) v[u] = sw[i + u];
#pragma unroll
                    for (uint32_t u = 0; u < CU; ++u) dw[i + u] = __builtin_amdgcn_alignbyte(v[u + 1], v[u], dl);
                }
                for (; i < nw; ++i) dw[i] = __builtin_amdgcn_alignbyte(sw[i + 1], sw[i], dl);
            }
            for (uint32_t k = h + 4 * nw; k < m; ++k)
                *reinterpret_cast<GAS uint8_t *>(dst + k) = *reinterpret_cast<const GAS uint8_t *>(src + k);
        }
    }
    if (c == a.nc - 1) {  // the last chunk: the total and the header
        const uint64_t total = first + m;
        if (total <= room && total <= 0xFFFFFFFFull) {
            offs[a.nc] = (uint32_t)total;
            gsc_rans_header *hd = reinterpret_cast<gsc_rans_header *>(a.out);
            hd->magic = GSC_RANS_MAGIC;
            hd->version = GSC_VERSION;
            hd->n = a.n;
            hd->K = a.K;
            hd->nchunks = a.nc;
            hd->total = (uint32_t)total;
            hd->reserved = 0;
        }
    }
}

// ---------------------------------------------------------------------------------- decode
// The decoder's table in LDS, one word per slot of [0, M): byte | (f - 1) << 8 | (slot - start)
// << 20 of the byte whose range holds the slot. Each present byte marks its first slot; a
// running maximum over the slots (64 at a time across the wave, carried from one step to the
// next) then gives every slot its byte. Returns false (uniform) when the frequencies do not sum
// to M.
__device__ inline bool dec_table(const GAS uint16_t *tab, uint32_t *s_dec, uint32_t *s_fst)
{
    const uint32_t lane = lane_id();
    uint32_t f[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = tab[4 * lane + q];
        sum += f[q];
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (__shfl(incl, WAVE - 1, WAVE) != RANS_M) return false;
    for (uint32_t j = lane; j < RANS_M; j += WAVE) s_dec[j] = 0;
    __syncthreads();
    uint32_t st = incl - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (f[q]) s_dec[st] = 4 * lane + q + 1;
        s_fst[4 * lane + q] = f[q] | ((st & 0xFFFu) << 13);
        st += f[q];
    }
    __syncthreads();
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < RANS_M; j0 += WAVE) {
        uint32_t v = s_dec[j0 + lane];
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t t = __shfl_up(v, o, WAVE);
            if (lane >= (uint32_t)o) v = max(v, t);
        }
        v = max(v, carry);
        carry = __shfl(v, WAVE - 1, WAVE);
        const uint32_t s = v - 1, fst = s_fst[s];
        const uint32_t fs = fst & 0x1FFFu, sts = fst >> 13;
        s_dec[j0 + lane] = s | ((fs - 1) << 8) | ((j0 + lane - sts) << 20);
    }
    __syncthreads();
    return true;
}

// A 4-byte aligned word of the stream [lo, hi); bytes outside it read as zero. As in_block8, the
// word load is issued on every path (at `safe` for a word reaching outside the stream).
__device__ inline uint32_t src_word(uint64_t p, uint64_t lo, uint64_t hi, uint64_t safe)
{
    const bool full = p >= lo && p + 4 <= hi;
    uint32_t w = *reinterpret_cast<const GAS uint32_t *>(full ? p : safe);
    if (!full) {
        w = 0;
        for (uint32_t q = 0; q < 4; ++q)
            if (p + q >= lo && p + q < hi) w |= (uint32_t)*reinterpret_cast<const GAS uint8_t *>(p + q) << (8 * q);
    }
    return w;
}

// The state of one chunk's decoder: the state x, the next stream bytes in a 64-bit window (the
// next byte in the top bits; av of them), the word after them already read (nw, whose address
// follows wa), the bytes of the chunk taken (used) and a damaged-chunk flag.
struct DecState {
    uint32_t x, av, nw, used;
    uint64_t win, wa;
    bool bad;
};

// Decodes one byte; word(a) reads the aligned stream word at address a.
template <class Word>
__device__ inline uint32_t dec_step(DecState &D, const uint32_t *s_dec, uint32_t len, Word &word)
{
    if (D.av <= 4) {  // refill: at least two bytes in the window for the renormalisation
        D.win |= (uint64_t)__builtin_bswap32(D.nw) << (32 - 8 * D.av);
        D.av += 4;
        D.nw = word(D.wa);
        D.wa += 4;
    }
    const uint32_t t = s_dec[D.x & (RANS_M - 1u)];
    uint32_t x = (((t >> 8) & 0xFFFu) + 1u) * (D.x >> RANS_BITS) + (t >> 20);
    // renormalisation: the first two bytes without a branch, any further ones (a damaged stream
    // only) one at a time while the chunk has bytes left (a chunk that runs out is rejected, as a
    // decoder reading byte by byte would find)
    const uint32_t k = (x < RANS_L ? 1u : 0u) + (x < (RANS_L >> 8) ? 1u : 0u);
    x = (x << (8 * k)) | (uint32_t)((D.win >> 48) >> (16 - 8 * k));
    D.win <<= 8 * k;
    D.av -= k;
    D.used += k;
    while (x < RANS_L) {
        if (D.used >= len) {
            D.bad = true;
            break;
        }
        if (D.av == 0) {
            D.win = (uint64_t)__builtin_bswap32(D.nw) << 32;
            D.av = 4;
            D.nw = word(D.wa);
            D.wa += 4;
        }
        x = (x << 8) | (uint32_t)(D.win >> 56);
        D.win <<= 8;
        --D.av;
        ++D.used;
    }
    D.x = x;
    return t & 255u;
}

// Decodes chunk c (stream bytes [p0, p1) of the data area) into its output bytes.
template <bool STAGED>
__device__ inline void dec_chunk(const RansArgs &a, uint32_t c, uint64_t p0, uint64_t p1, uint64_t d0,
                                 const uint32_t *s_dec, const uint8_t *s_st, uint64_t sb, uint64_t se)
{
    const uint64_t lo = reinterpret_cast<uint64_t>(a.src), hi = lo + a.cap;
    const uint64_t safe = lo;
    auto word = [&](uint64_t q) -> uint32_t {
        if (STAGED) return q >= sb && q + 4 <= se ? *reinterpret_cast<const uint32_t *>(s_st + (q - sb)) : 0u;
        return src_word(q, lo, hi, safe);
    };
    const uint32_t len = (uint32_t)(p1 - p0);
    const uint64_t q0 = lo + d0 + p0;  // the chunk's first byte
    DecState D;
    D.wa = q0 & ~3ull;
    const uint32_t w0 = word(D.wa), w1 = word(D.wa + 4);
    D.wa += 8;
    const uint32_t skip = (uint32_t)(q0 & 3u);
    D.win = ((uint64_t)__builtin_bswap32(w0) << 32) | __builtin_bswap32(w1);
    D.win <<= 8 * skip;
    D.av = 8 - skip;
    D.x = (uint32_t)(D.win >> 32);
    D.win <<= 32;
    D.av -= 4;
    D.used = 4;
    D.bad = D.x < RANS_L;  // an encoder's first stored state is at least 2^23
    D.nw = word(D.wa);
    D.wa += 4;
    GAS uint8_t *ob = gp(a.out);
    const uint64_t b = (uint64_t)c * a.K, e = min(b + a.K, a.n);
    // head: bytes up to the first 4-aligned output address; body: four bytes to a word; tail
    const uint64_t oa = reinterpret_cast<uint64_t>(a.out) + b;
    const uint64_t hb = min(e - b, (uint64_t)((4u - (uint32_t)(oa & 3u)) & 3u));
    uint64_t i = b;
    for (; i < b + hb; ++i) ob[i] = (uint8_t)dec_step(D, s_dec, len, word);
    GAS uint32_t *ow = reinterpret_cast<GAS uint32_t *>(oa + hb);
    for (uint32_t j = 0; i + 4 <= e; i += 4, ++j) {
        uint32_t v = dec_step(D, s_dec, len, word);
        v |= dec_step(D, s_dec, len, word) << 8;
        v |= dec_step(D, s_dec, len, word) << 16;
        v |= dec_step(D, s_dec, len, word) << 24;
        ow[j] = v;
    }
    for (; i < e; ++i) ob[i] = (uint8_t)dec_step(D, s_dec, len, word);
    if (D.bad || D.x != RANS_L || D.used != len) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
}

// Thread c decodes chunk c. The header and table are checked by every workgroup, the chunk's
// offsets by its thread. Staged (chunks of at most RANS_STAGE_K bytes), the wave first copies
// its chunks' stream bytes to LDS and the chunk's words come from there (words outside the copy
// read as zero: only a chunk that takes more bytes than it has gets there, and it is rejected);
// a wave whose bytes do not fit the copy holds a chunk longer than an encoder writes (2 K + 4
// bytes) and is rejected whole. Otherwise the words come from global memory. The decoded bytes
// are stored four to a word (byte by byte where the chunk starts or ends inside a word).
template <bool STAGED>
__global__ __launch_bounds__(RANS_THREADS) void k_rans_decode(RansArgs a)
{
    extern __shared__ gi4 s_dyn[];
    __shared__ uint32_t s_dec[RANS_M];
    __shared__ uint32_t s_fst[256];
    const CAS gsc_rans_header *h = cp(reinterpret_cast<const gsc_rans_header *>(a.src));
    const GAS uint16_t *tab = gp(reinterpret_cast<const uint16_t *>(a.src + sizeof(gsc_rans_header)));
    const uint64_t d0 = rans_data_off(a.nc);
    const bool hdr = h->magic == GSC_RANS_MAGIC && h->n == a.n && h->K == a.K && h->nchunks == a.nc &&
                     d0 + (uint64_t)h->total <= a.cap;
    if (!hdr || !dec_table(tab, s_dec, s_fst)) {  // (uniform)
        if (threadIdx.x == 0) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
        return;
    }
    const uint32_t c = blockIdx.x * RANS_THREADS + threadIdx.x;
    const GAS uint32_t *offs = gp(reinterpret_cast<const uint32_t *>(a.src + sizeof(gsc_rans_header) + 512));
    const uint32_t cc = min(c, a.nc - 1);
    const uint64_t p0 = offs[cc], p1 = offs[cc + 1];
    const bool mine = c < a.nc;
    const bool ok = p1 >= p0 + 4 && p1 <= h->total;
    if (mine && !ok) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
    const uint64_t lo = reinterpret_cast<uint64_t>(a.src), hi = lo + a.cap;
    const uint64_t safe = lo;  // (the header: 8-aligned, 32 readable bytes)
    uint8_t *s_st = reinterpret_cast<uint8_t *>(s_dyn);
    uint64_t sb = 0, se = 0;
    if (STAGED) {
        const uint64_t rlo = mine && ok ? p0 : ~0ull, rhi = mine && ok ? p1 : 0ull;
        uint64_t wlo = rlo, whi = rhi;
        for (int o = 32; o > 0; o >>= 1) {
            wlo = min(wlo, (uint64_t)__shfl_xor(wlo, o, WAVE));
            whi = max(whi, (uint64_t)__shfl_xor(whi, o, WAVE));
        }
        if (whi > wlo && whi - wlo + 32 > a.stage) {  // (uniform)
            if (threadIdx.x == 0) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
                return;
        }
        if (whi > wlo) {
            sb = stage_blocks(s_st, lo + d0 + wlo, lo + d0 + whi, lo, hi, safe);
            se = sb + (whi + d0 + lo - sb + 15) / 16 * 16;
        }
        __syncthreads();
    }
    if (mine && ok) dec_chunk<STAGED>(a, c, p0, p1, d0, s_dec, s_st, sb, se);
}


// ------------------------------------------------------------------------------- launches
uint64_t rans_chunks(uint64_t n, uint32_t K) { return (n + K - 1) / K; }
uint64_t rans_workspace_bytes(uint64_t n, uint32_t K)
{
    const uint64_t nc = rans_chunks(n, K);
    return rans_tmp_off(nc) + nc * rans_tmp_stride(K);
}
uint64_t rans_capacity_bytes(uint64_t n, uint32_t K)
{
    const uint64_t nc = rans_chunks(n, K);
    // a symbol emits at most 2 bytes (12 bits of frequency 1, aligned to bytes), plus 4 per chunk
    return sizeof(gsc_rans_header) + 512 + 4 * (nc + 1) + 2 * n + 4 * nc;
}

// The staged kernels' LDS (static + dynamic) must fit the device's limit per workgroup.
static bool stage_fits(size_t dyn, size_t stat)
{
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    return dyn + stat <= (size_t)lim;
}

static RansArgs rans_args(uint64_t n, uint32_t K, uint32_t *ws)
{
    RansArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.K = K;
    a.nc = (uint32_t)rans_chunks(n, K);
    a.ws = ws;
    a.status = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(ws) + RANS_STATUS_OFF);
    a.hblocks = rans_hist_blocks(n);
    a.tmp = reinterpret_cast<uint8_t *>(ws) + rans_tmp_off(a.nc);
    a.tmp_stride = rans_tmp_stride(K);
    return a;
}

hipError_t launch_rans_encode(const uint8_t *in, uint64_t n, uint32_t K, uint8_t *out, uint64_t cap, void *ws,
                              int32_t *info, hipStream_t s)
{
    RansArgs a = rans_args(n, K, static_cast<uint32_t *>(ws));
    a.in = in;
    a.out = out;
    a.cap = cap;
    a.info = info;
    const uint32_t zw = (uint32_t)rans_head_words(a.nc);
    hipLaunchKernelGGL(k_rans_zero, dim3(min((zw + 255) / 256, 1024u)), dim3(256), 0, s, a.ws, zw);
    if (a.nc > 0) hipLaunchKernelGGL(k_rans_hist, dim3(a.hblocks), dim3(RANS_HIST_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_rans_table, dim3(1), dim3(WAVE), 0, s, a);
    if (a.nc > 0) {
        const dim3 g((a.nc + RANS_THREADS - 1) / RANS_THREADS);
        const uint32_t stage = (uint32_t)(RANS_THREADS * K + 32);
        if (K <= RANS_STAGE_K && stage_fits(stage, 256 * sizeof(uint4))) {
            a.stage = stage;
            hipLaunchKernelGGL(k_rans_encode<true>, g, dim3(RANS_THREADS), a.stage, s, a);
        } else {
            hipLaunchKernelGGL(k_rans_encode<false>, g, dim3(RANS_THREADS), 0, s, a);
        }
    }
    hipLaunchKernelGGL(k_rans_info, dim3(1), dim3(WAVE), 0, s, a, 0);
    return hipGetLastError();
}

hipError_t launch_rans_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t K, uint8_t *out, void *ws,
                              int32_t *info, hipStream_t s)
{
    RansArgs a = rans_args(n, K, static_cast<uint32_t *>(ws));
    a.src = in;
    a.cap = in_bytes;
    a.out = out;
    a.info = info;
    hipLaunchKernelGGL(k_rans_zero, dim3(1), dim3(256), 0, s, a.ws, 1u);
    if (a.nc > 0) {
        const dim3 g((a.nc + RANS_THREADS - 1) / RANS_THREADS);
        // an encoder's chunk holds at most 2 K + 4 bytes (two per symbol and the state)
        const uint32_t stage = (uint32_t)(RANS_THREADS * (2 * K + 8) + 32);
        if (K <= RANS_STAGE_K && stage_fits(stage, (RANS_M + 256) * sizeof(uint32_t))) {
            a.stage = stage;
            hipLaunchKernelGGL(k_rans_decode<true>, g, dim3(RANS_THREADS), a.stage, s, a);
        } else {
            hipLaunchKernelGGL(k_rans_decode<false>, g, dim3(RANS_THREADS), 0, s, a);
        }
    }
    hipLaunchKernelGGL(k_rans_info, dim3(1), dim3(WAVE), 0, s, a, 1);
    return hipGetLastError();
}

}  // namespace gsc
