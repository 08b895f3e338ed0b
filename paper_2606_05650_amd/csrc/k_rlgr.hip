// Entropy coding of the quantized coefficients (Sec. 3.4): every channel's coefficient vector,
// in coefficient order, is cut into blocks of B values, and every block is coded on its own by
// the adaptive run-length / Golomb-Rice coder the paper uses, so the blocks code in parallel.
// The paper gives no parameters; the coder follows the published method with these choices:
//   * block b = j * C + c holds coefficients j*B .. j*B + B - 1 of channel c; its code is a
//     whole number of 32-bit words, filled from the most significant bit;
//   * two adaptive parameters with 3 fractional bits, kp (run mode while kp >> 3 > 0) and krp
//     (Golomb-Rice parameter kr = krp >> 3), both starting at 8 and kept within 0..80;
//   * run mode: a 0 bit per 2^k zeros (kp += 4), then a 1 and the remaining count in k bits,
//     then, unless the block ends, the sign bit and GR(|v| - 1) of the value that ends the run
//     (kp -= 6); Golomb-Rice mode: GR(2v) or GR(-2v - 1) (kp += 3 after a zero, -= 3 otherwise);
//   * GR(u): u >> kr ones, a 0, the kr low bits; 24 ones then u in 32 bits when u >> kr >= 24;
//     krp -= 2 when u >> kr = 0, += u >> kr when it is above 1.
// A workgroup (one wave) takes one block row j: thread c codes block j * C + c. The rows pass
// through LDS in chunks of 64, so the coefficient matrix is read (encoder) and written (decoder)
// in whole rows, coalesced across the channels; each thread then walks its own column.
#include "gsc_device.h"

namespace gsc {

constexpr int RLGR_THREADS = WAVE;  // one thread per channel (C <= 64)
constexpr int RLGR_ROWS = 64;       // rows per LDS chunk
constexpr int RLGR_FRAC = 3, RLGR_PMAX = 80, RLGR_START = 8;
constexpr int RLGR_RUN_UP = 4, RLGR_RUN_DOWN = 6, RLGR_GR_UP = 3, RLGR_GR_DOWN = 3;
constexpr uint32_t RLGR_ESCAPE = 24;
static_assert(GSC_MAX_CHANNELS <= RLGR_THREADS, "one thread per channel");

__device__ inline int rl_clamp(int p) { return p < 0 ? 0 : (p > RLGR_PMAX ? RLGR_PMAX : p); }

// ------------------------------------------------------------------------------ encoder
// Bit sink: counts the bits (W = false) or also writes the words (W = true) at `out`.
template <bool W>
struct BitSink {
    uint64_t acc = 0;     // pending bits (the low nacc bits)
    uint32_t nacc = 0;
    uint64_t nbits = 0;
    GAS uint32_t *out = nullptr;
    __device__ void put(uint32_t v, uint32_t n)  // the n low bits of v (n <= 32), most significant first
    {
        if (n == 0) return;
        nbits += n;
        if (!W) return;
        acc = (acc << n) | (n == 32 ? (uint64_t)v : ((uint64_t)v & ((1ull << n) - 1ull)));
        nacc += n;
        if (nacc >= 32) {
            *out++ = (uint32_t)(acc >> (nacc - 32));
            nacc -= 32;
            acc &= nacc ? ((1ull << nacc) - 1ull) : 0ull;
        }
    }
    __device__ void flush()
    {
        if (W && nacc > 0) *out = (uint32_t)(acc << (32 - nacc));
    }
};

template <bool W>
struct RlgrEnc {
    int kp = RLGR_START, krp = RLGR_START;
    uint32_t run = 0;   // zeros of the open run segment not yet sent
    bool open = false;  // a run segment is open
    BitSink<W> bs;

    __device__ void gr(uint32_t u)
    {
        const uint32_t kr = (uint32_t)krp >> RLGR_FRAC;
        const uint32_t q = u >> kr;
        if (q < RLGR_ESCAPE) {
            bs.put(((1u << q) - 1u) << 1, q + 1);  // q ones and a zero
            bs.put(u, kr);
        } else {
            bs.put((1u << RLGR_ESCAPE) - 1u, RLGR_ESCAPE);
            bs.put(u, 32);
        }
        if (q == 0) krp = rl_clamp(krp - 2);
        else if (q > 1) krp = rl_clamp(krp + (int)min(q, (uint32_t)RLGR_PMAX));
    }
    __device__ void value(int32_t v)
    {
        if (!open && (kp >> RLGR_FRAC) == 0) {  // Golomb-Rice mode
            const uint32_t u = v >= 0 ? 2u * (uint32_t)v : 2u * (uint32_t)(-(int64_t)v) - 1u;
            gr(u);
            kp = rl_clamp(u == 0 ? kp + RLGR_GR_UP : kp - RLGR_GR_DOWN);
            return;
        }
        const uint32_t k = (uint32_t)kp >> RLGR_FRAC;  // run mode
        if (v == 0) {
            open = true;
            if (++run == (1u << k)) {
                bs.put(0, 1);
                run = 0;
                kp = rl_clamp(kp + RLGR_RUN_UP);
            }
            return;
        }
        bs.put(1, 1);
        bs.put(run, k);
        run = 0;
        open = false;
        bs.put(v < 0 ? 1u : 0u, 1);
        gr((uint32_t)(v < 0 ? -(int64_t)v : (int64_t)v) - 1u);
        kp = rl_clamp(kp - RLGR_RUN_DOWN);
    }
    __device__ void finish()
    {
        if (open) {
            bs.put(1, 1);
            bs.put(run, (uint32_t)kp >> RLGR_FRAC);
        }
        bs.flush();
    }
};

struct RlgrArgs {
    const int32_t *q;   // [nv][C]
    uint32_t nv, C, B, nb;
    uint8_t *out;       // stream: header, block table, words
    uint64_t out_cap;
    uint64_t *status;   // look-back status of the block rows (zeroed)
    uint32_t *err;      // device error word (first word of the workspace)
    int32_t *info;
};

__device__ inline GAS uint32_t *rl_table(uint8_t *out) { return gp(reinterpret_cast<uint32_t *>(out + sizeof(gsc_rlgr_header))); }
__device__ inline GAS uint32_t *rl_words(uint8_t *out, uint32_t NB)
{
    return gp(reinterpret_cast<uint32_t *>(out + sizeof(gsc_rlgr_header))) + NB + 1;
}

// Codes this thread's block of row j (count or write), streaming the rows through LDS. Each
// chunk's values are loaded into registers one chunk ahead (every load of a chunk issued before
// any is used), so the loads of chunk i + 1 are in flight while chunk i is coded. A chunk load
// is unconditional and its positions clamped: past the last chunk it re-reads the last one.
constexpr int RLGR_PER = RLGR_ROWS * RLGR_THREADS / RLGR_THREADS;  // values per thread and chunk (C <= 64)
template <bool W>
__device__ inline void rl_encode_row(const RlgrArgs &a, uint32_t j, RlgrEnc<W> &enc, int32_t *s_tile)
{
    const uint32_t tid = threadIdx.x, C = a.C;
    const uint32_t r0 = j * a.B, r1 = min(r0 + a.B, a.nv);
    const GAS int32_t *q = gp(a.q);
    int32_t v[RLGR_PER];
    auto load = [&](uint32_t rc) {
        const uint32_t nval = min((uint32_t)RLGR_ROWS, r1 - rc) * C;
        const GAS int32_t *src = q + (size_t)rc * C;
#pragma unroll
        for (int u = 0; u < RLGR_PER; ++u) v[u] = src[min(tid + (uint32_t)u * RLGR_THREADS, nval - 1)];
    };
    load(r0);  // (r0 < r1: a block row holds at least one value)
    for (uint32_t rc = r0; rc < r1; rc += RLGR_ROWS) {
        const uint32_t nr = min((uint32_t)RLGR_ROWS, r1 - rc);
        const uint32_t nval = nr * C;
        __syncthreads();  // the previous chunk is no longer read
#pragma unroll
        for (int u = 0; u < RLGR_PER; ++u) {
            const uint32_t e = tid + (uint32_t)u * RLGR_THREADS;
            if (e < nval) s_tile[e] = v[u];
        }
        __syncthreads();
        load(rc + RLGR_ROWS < r1 ? rc + RLGR_ROWS : rc);
        if (tid < C)
            for (uint32_t r = 0; r < nr; ++r) enc.value(s_tile[r * C + tid]);
    }
    if (tid < C) enc.finish();
}

// Pass 1: every block's length in words, the blocks' word offsets (an exclusive scan over the
// block rows by decoupled look-back), the block table and the header.
__global__ __launch_bounds__(RLGR_THREADS) void k_rlgr_count(RlgrArgs a)
{
    __shared__ int32_t s_tile[RLGR_ROWS * RLGR_THREADS];
    const uint32_t j = blockIdx.x, tid = threadIdx.x, C = a.C, NB = a.nb * C;
    RlgrEnc<false> enc;
    rl_encode_row<false>(a, j, enc, s_tile);
    const uint64_t words = tid < C ? (enc.bs.nbits + 31) / 32 : 0;
    uint64_t incl = words;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint64_t t = __shfl_up(incl, o, WAVE);
        if (tid >= (uint32_t)o) incl += t;
    }
    const uint64_t row_words = __shfl(incl, WAVE - 1, WAVE);
    const uint64_t base = lookback_wave<OpSum>(a.status, 1, j, row_words, reinterpret_cast<Ctrl *>(a.err));
    const uint64_t first = base + incl - words;
    // the stream's capacity (header, table, words) bounds the total
    const uint64_t room = (a.out_cap - sizeof(gsc_rlgr_header)) / 4 - (NB + 1);
    GAS uint32_t *tab = rl_table(a.out);
    if (tid < C) {
        if (first + words > room || first + words > 0xFFFFFFFFull) atomicCAS(a.err, 0u, (uint32_t)GSC_ERR_CAPACITY);
        else tab[j * C + tid] = (uint32_t)first;
    }
    if (j == a.nb - 1 && tid == 0) {
        const uint64_t total = base + row_words;
        if (total <= room && total <= 0xFFFFFFFFull) {
            tab[NB] = (uint32_t)total;
            gsc_rlgr_header *h = reinterpret_cast<gsc_rlgr_header *>(a.out);
            h->magic = GSC_RLGR_MAGIC;
            h->version = GSC_VERSION;
            h->nv = a.nv;
            h->C = C;
            h->B = a.B;
            h->nblocks = NB;
            h->total_words = (uint32_t)total;
            h->reserved = 0;
            const uint64_t bytes = sizeof(gsc_rlgr_header) + 4ull * (NB + 1 + total);
            a.info[2] = (int32_t)(uint32_t)bytes;
            a.info[3] = (int32_t)(uint32_t)(bytes >> 32);
        }
    }
}

// Pass 2: every block's code written at its offset.
__global__ __launch_bounds__(RLGR_THREADS) void k_rlgr_write(RlgrArgs a)
{
    __shared__ int32_t s_tile[RLGR_ROWS * RLGR_THREADS];
    const uint32_t j = blockIdx.x, tid = threadIdx.x, C = a.C, NB = a.nb * C;
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;  // (uniform)
    RlgrEnc<true> enc;
    if (tid < C) enc.bs.out = rl_words(a.out, NB) + rl_table(a.out)[j * C + tid];
    rl_encode_row<true>(a, j, enc, s_tile);
}

// The workspace's error word and look-back status words start at zero.
__global__ __launch_bounds__(256) void k_rlgr_zero(uint64_t *ws, uint32_t nwords)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nwords; i += gridDim.x * 256) ws[i] = 0;
}

__global__ __launch_bounds__(64) void k_rlgr_info(RlgrArgs a)
{
    if (threadIdx.x == 0) {
        if (a.nb == 0) {  // no block: the header and the one-entry table of an empty stream
            gsc_rlgr_header *h = reinterpret_cast<gsc_rlgr_header *>(a.out);
            h->magic = GSC_RLGR_MAGIC;
            h->version = GSC_VERSION;
            h->nv = 0;
            h->C = a.C;
            h->B = a.B;
            h->nblocks = 0;
            h->total_words = 0;
            h->reserved = 0;
            *rl_table(a.out) = 0;
            a.info[2] = (int32_t)(sizeof(gsc_rlgr_header) + 4);
            a.info[3] = 0;
        }
        const uint32_t e = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.info[0] = (int32_t)e;
        a.info[1] = (int32_t)a.nv;
        if (e) a.info[2] = a.info[3] = 0;
    }
}

// ------------------------------------------------------------------------------ decoder
// Bit source over one block's words [w, w + nw): a 64-bit window (cur, nxt) and the next four
// words already in flight, so that a word boundary costs no load latency.
struct BitSrc {
    const GAS uint32_t *w;
    uint32_t nw;       // words of the block
    uint32_t wi;       // index of `cur`
    uint32_t bit;      // bits of `cur` already taken (0..31)
    uint32_t cur, nxt;
    uint32_t ahead[4];  // words wi + 2 .. wi + 5
    bool bad;
    __device__ uint32_t at(uint32_t i) const { return i < nw ? w[i] : 0u; }
    __device__ void init(const GAS uint32_t *w_, uint32_t nw_)
    {
        w = w_;
        nw = nw_;
        wi = 0;
        bit = 0;
        bad = false;
        cur = at(0);
        nxt = at(1);
#pragma unroll
        for (int i = 0; i < 4; ++i) ahead[i] = at(2 + i);
    }
    __device__ void advance_word()
    {
        cur = nxt;
        nxt = ahead[0];
        ahead[0] = ahead[1];
        ahead[1] = ahead[2];
        ahead[2] = ahead[3];
        ahead[3] = at(wi + 6);
        ++wi;
    }
    __device__ uint32_t peek32() const  // the next 32 bits
    {
        return bit ? (cur << bit) | (nxt >> (32 - bit)) : cur;
    }
    __device__ void skip(uint32_t n)  // n <= 32
    {
        bit += n;
        if (bit >= 32) {
            bit -= 32;
            advance_word();
        }
        if (wi > nw || (wi == nw && bit > 0)) bad = true;  // past the block's words
    }
    __device__ uint32_t get(uint32_t n)
    {
        if (n == 0) return 0;
        const uint32_t v = peek32() >> (32 - n);
        skip(n);
        return v;
    }
    // the exact end: every value decoded, only the last word's low bits left
    __device__ bool exact_end() const { return !bad && (nw == 0 ? (wi == 0 && bit == 0) : (wi == nw - 1 && bit > 0) || (wi == nw && bit == 0)); }
};

struct RlgrDec {
    int kp = RLGR_START, krp = RLGR_START;
    uint32_t zeros = 0;       // zeros still to produce
    bool val_pending = false; // a run's terminating value follows the zeros
    uint32_t pos = 0;         // values produced
    bool bad = false;
    BitSrc bs;

    __device__ uint32_t gr()
    {
        const uint32_t kr = (uint32_t)krp >> RLGR_FRAC;
        const uint32_t ones = __clz(~bs.peek32());  // leading ones
        uint32_t q, u;
        if (ones >= RLGR_ESCAPE) {
            bs.skip(RLGR_ESCAPE);
            u = bs.get(16) << 16;
            u |= bs.get(16);
            q = u >> kr;
        } else {
            bs.skip(ones + 1);
            q = ones;
            u = (q << kr) | bs.get(kr);
        }
        if (q == 0) krp = rl_clamp(krp - 2);
        else if (q > 1) krp = rl_clamp(krp + (int)min(q, (uint32_t)RLGR_PMAX));
        return u;
    }
    // the next value of a block of L values
    __device__ int32_t next(uint32_t L)
    {
        for (;;) {
            if (zeros > 0) {
                --zeros;
                ++pos;
                return 0;
            }
            if (val_pending) {
                val_pending = false;
                const uint32_t s = bs.get(1);
                const uint32_t m = gr() + 1u;  // (wraps to 0 only for a corrupt code)
                kp = rl_clamp(kp - RLGR_RUN_DOWN);
                ++pos;
                if (m == 0 || (s ? m > 0x80000000u : m > 0x7FFFFFFFu)) bad = true;
                return s ? (int32_t)(0u - m) : (int32_t)m;
            }
            uint32_t k = (uint32_t)kp >> RLGR_FRAC;
            if (k == 0) {
                const uint32_t u = gr();
                kp = rl_clamp(u == 0 ? kp + RLGR_GR_UP : kp - RLGR_GR_DOWN);
                ++pos;
                return (u & 1u) ? (int32_t)(0u - ((u >> 1) + 1u)) : (int32_t)(u >> 1);
            }
            // a run segment: 0 bits of 2^k zeros each, a 1, the remaining count in k bits
            uint64_t z = 0;
            while (bs.get(1) == 0 && !bs.bad) {
                z += 1ull << k;
                if (pos + z > L) break;
                kp = rl_clamp(kp + RLGR_RUN_UP);
                k = (uint32_t)kp >> RLGR_FRAC;
            }
            z += bs.get(k);
            if (bs.bad || pos + z > L) {
                bad = true;
                zeros = L - pos;  // (fill the rest; the block is reported)
                val_pending = false;
                continue;
            }
            zeros = (uint32_t)z;
            val_pending = pos + z < L;
        }
    }
};

struct RlgrDecArgs {
    const uint8_t *in;
    uint64_t in_bytes;
    uint32_t nv, C, B, nb;
    int32_t *q;      // [nv][C]
    int32_t *info;
    uint32_t *err;
};

// Decodes block row j: thread c decodes block j * C + c into LDS, chunk by chunk, and the
// workgroup stores each chunk's rows.
__global__ __launch_bounds__(RLGR_THREADS) void k_rlgr_decode(RlgrDecArgs a)
{
    __shared__ int32_t s_tile[RLGR_ROWS * RLGR_THREADS];
    __shared__ uint32_t s_ok;
    const uint32_t j = blockIdx.x, tid = threadIdx.x, C = a.C, NB = a.nb * C;
    const GAS uint32_t *tab = gp(reinterpret_cast<const uint32_t *>(a.in + sizeof(gsc_rlgr_header)));
    const GAS uint32_t *words = tab + NB + 1;
    const CAS gsc_rlgr_header *h = cp(reinterpret_cast<const gsc_rlgr_header *>(a.in));
    if (tid == 0) {
        // header and table bounds (the host checked that the header and table fit in in_bytes)
        const uint32_t tw = h->total_words;
        const bool hdr = h->magic == GSC_RLGR_MAGIC && h->nv == a.nv && h->C == C && h->B == a.B && h->nblocks == NB &&
                         tab[NB] == tw && sizeof(gsc_rlgr_header) + 4ull * (NB + 1 + (uint64_t)tw) <= a.in_bytes;
        s_ok = hdr ? 1u : 0u;
        if (!hdr) atomicCAS(a.err, 0u, (uint32_t)GSC_ERR_CORRUPT_STREAM);
    }
    __syncthreads();
    if (!s_ok) return;
    const uint32_t r0 = j * a.B, r1 = min(r0 + a.B, a.nv), L = r1 - r0;
    RlgrDec dec;
    if (tid < C) {
        const uint32_t b = j * C + tid;
        const uint32_t o0 = tab[b], o1 = tab[b + 1];
        if (o1 < o0 || o1 > h->total_words) dec.bad = true;
        dec.bs.init(words + o0, dec.bad ? 0u : o1 - o0);
    }
    GAS int32_t *q = gp(a.q);
    for (uint32_t rc = r0; rc < r1; rc += RLGR_ROWS) {
        const uint32_t nr = min((uint32_t)RLGR_ROWS, r1 - rc);
        if (tid < C)
            for (uint32_t r = 0; r < nr; ++r) s_tile[r * C + tid] = dec.next(L);
        __syncthreads();
        const uint32_t nval = nr * C;
        GAS int32_t *dst = q + (size_t)rc * C;
        for (uint32_t e = tid; e < nval; e += RLGR_THREADS) dst[e] = s_tile[e];
        __syncthreads();
    }
    if (tid < C && (dec.bad || dec.bs.bad || !dec.bs.exact_end()))
        atomicCAS(a.err, 0u, (uint32_t)GSC_ERR_CORRUPT_STREAM);
}

__global__ __launch_bounds__(64) void k_rlgr_dec_info(RlgrDecArgs a)
{
    if (threadIdx.x == 0) {
        if (a.nb == 0) {  // an empty stream: only its header to check
            const gsc_rlgr_header *h = reinterpret_cast<const gsc_rlgr_header *>(a.in);
            if (h->magic != GSC_RLGR_MAGIC || h->nv != 0 || h->C != a.C || h->nblocks != 0 || h->total_words != 0)
                atomicCAS(a.err, 0u, (uint32_t)GSC_ERR_CORRUPT_STREAM);
        }
        a.info[0] = (int32_t)__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.info[1] = (int32_t)a.nv;
    }
}

// --------------------------------------------------------------------------- launches
hipError_t launch_rlgr_encode(const int32_t *q, uint32_t nv, uint32_t C, uint32_t B, uint8_t *out,
                              uint64_t out_cap, uint64_t *ws, int32_t *info, hipStream_t s)
{
    RlgrArgs a;
    a.q = q;
    a.nv = nv;
    a.C = C;
    a.B = B;
    a.nb = (nv + B - 1) / B;
    a.out = out;
    a.out_cap = out_cap;
    a.err = reinterpret_cast<uint32_t *>(ws);
    a.status = ws + 1;
    a.info = info;
    const uint32_t zw = a.nb + 1;
    hipLaunchKernelGGL(k_rlgr_zero, dim3(min((zw + 255) / 256, 1024u)), dim3(256), 0, s, ws, zw);
    if (a.nb > 0) {
        hipLaunchKernelGGL(k_rlgr_count, dim3(a.nb), dim3(RLGR_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_rlgr_write, dim3(a.nb), dim3(RLGR_THREADS), 0, s, a);
    }
    hipLaunchKernelGGL(k_rlgr_info, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rlgr_decode(const uint8_t *in, uint64_t in_bytes, uint32_t nv, uint32_t C, uint32_t B,
                              int32_t *q, uint64_t *ws, int32_t *info, hipStream_t s)
{
    RlgrDecArgs a;
    a.in = in;
    a.in_bytes = in_bytes;
    a.nv = nv;
    a.C = C;
    a.B = B;
    a.nb = (nv + B - 1) / B;
    a.q = q;
    a.info = info;
    a.err = reinterpret_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(k_rlgr_zero, dim3(1), dim3(256), 0, s, ws, 1u);
    if (a.nb > 0) hipLaunchKernelGGL(k_rlgr_decode, dim3(a.nb), dim3(RLGR_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_rlgr_dec_info, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsc
