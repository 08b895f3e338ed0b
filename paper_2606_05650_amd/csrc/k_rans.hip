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
//   * a decoder accepts a chunk only if it ends in the state 2^23 with all its bytes consumed.
// Encode: a byte histogram, the table (one wave), then one thread per chunk codes its chunk into
// a scratch area, the chunks' offsets come from a decoupled look-back over waves of 64 chunks,
// and each thread copies its bytes, reversed, to their place. Decode: one thread per chunk.
#include "gsc_device.h"

#include <cstring>

namespace gsc {

constexpr uint32_t RANS_BITS = 12, RANS_M = 1u << RANS_BITS, RANS_L = 1u << 23;
constexpr int RANS_THREADS = WAVE;  // one wave per 64 chunks
constexpr int RANS_HIST_THREADS = 256;

struct RansArgs {
    const uint8_t *in;
    uint64_t n;
    uint32_t K, nc;
    uint8_t *out;        // stream (encode) or decoded bytes (decode)
    uint64_t cap;        // encode: stream capacity; decode: input stream bytes
    const uint8_t *src;  // decode: the stream
    uint32_t *ws;        // [0] error, [1..256] histogram
    uint64_t *status;    // look-back status of the chunk waves
    uint8_t *tmp;        // per-chunk scratch, chunk c at c * tmp_stride
    uint64_t tmp_stride;
    int32_t *info;
};

__device__ inline void rans_error(uint32_t *err, uint32_t code)
{
    atomicCAS(err, 0u, code);
}

// Stream: header, freq u16[256], offsets u32[nc + 1] (bytes into the data area), data.
__device__ inline uint64_t rans_data_off(uint32_t nc) { return sizeof(gsc_rans_header) + 512ull + 4ull * (nc + 1); }

// ---------------------------------------------------------------------------------- encode
__global__ __launch_bounds__(256) void k_rans_zero(uint32_t *ws, uint32_t nwords)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nwords; i += gridDim.x * 256) ws[i] = 0;
}

__global__ __launch_bounds__(RANS_HIST_THREADS) void k_rans_hist(RansArgs a)
{
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const GAS uint8_t *in = gp(a.in);
    const uint64_t stride = (uint64_t)gridDim.x * RANS_HIST_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * RANS_HIST_THREADS + threadIdx.x; i < a.n; i += stride)
        atomicAdd(&s_h[in[i]], 1u);
    __syncthreads();
    if (s_h[threadIdx.x]) atomicAdd(&a.ws[1 + threadIdx.x], s_h[threadIdx.x]);
}

// One wave: the table from the histogram, written to the stream (the header by the last chunk).
__global__ __launch_bounds__(WAVE) void k_rans_table(RansArgs a)
{
    const uint32_t lane = lane_id();
    uint32_t c[4], f[4];
    uint32_t present = 0, sum = 0;
    uint32_t best = 0, best_s = 0;  // count and byte of this lane's most frequent byte
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t s = lane * 4 + q;
        c[q] = __hip_atomic_load(&a.ws[1 + s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    GAS uint16_t *tab = gp(reinterpret_cast<uint16_t *>(a.out + sizeof(gsc_rans_header)));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t s = lane * 4 + q;
        tab[s] = (uint16_t)(f[q] + (a.n > 0 && s == best_s ? RANS_M - sum : 0u));
    }
}

// The frequencies and starts of the stream's table in LDS (every thread of the block helps).
__device__ inline void load_table(const GAS uint16_t *tab, uint32_t *s_f, uint32_t *s_st)
{
    for (uint32_t s = threadIdx.x; s < 256; s += blockDim.x) s_f[s] = tab[s];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t s = 0; s < 256; ++s) {
            s_st[s] = acc;
            acc += s_f[s];
        }
        s_st[256] = acc;
    }
    __syncthreads();
}

// Thread c codes chunk c into its scratch area (emission order), the wave's chunks find their
// offsets by look-back, and each thread writes its bytes reversed at its offset.
__global__ __launch_bounds__(RANS_THREADS) void k_rans_encode(RansArgs a)
{
    __shared__ uint32_t s_f[256], s_st[257];
    const GAS uint16_t *tab = gp(reinterpret_cast<const uint16_t *>(a.out + sizeof(gsc_rans_header)));
    load_table(tab, s_f, s_st);
    const uint32_t lane = lane_id();
    const uint32_t c = blockIdx.x * RANS_THREADS + lane;
    uint32_t m = 0;  // bytes of this chunk
    GAS uint8_t *tmp = gp(a.tmp) + (uint64_t)c * a.tmp_stride;
    if (c < a.nc) {
        const GAS uint8_t *in = gp(a.in);
        const uint64_t b = (uint64_t)c * a.K, e = min(b + a.K, a.n);
        uint32_t x = RANS_L;
        for (uint64_t i = e; i > b; --i) {
            const uint32_t s = in[i - 1], f = s_f[s];
            if (f == 0) {  // (impossible with the stream's own table)
                rans_error(a.ws, GSC_ERR_INTERNAL);
                break;
            }
            const uint32_t xmax = ((RANS_L >> RANS_BITS) << 8) * f;
            while (x >= xmax) {
                tmp[m++] = (uint8_t)(x & 255u);
                x >>= 8;
            }
            x = ((x / f) << RANS_BITS) + (x % f) + s_st[s];
        }
        for (int k = 0; k < 4; ++k) {
            tmp[m++] = (uint8_t)(x & 255u);
            x >>= 8;
        }
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
            GAS uint8_t *dst = gp(a.out) + d0 + first;
            for (uint32_t k = 0; k < m; ++k) dst[k] = tmp[m - 1 - k];
        }
    }
    if (c == a.nc - 1) {  // the last chunk: the total and the header
        const uint64_t total = first + m;
        if (total <= room && total <= 0xFFFFFFFFull) {
            offs[a.nc] = (uint32_t)total;
            gsc_rans_header *h = reinterpret_cast<gsc_rans_header *>(a.out);
            h->magic = GSC_RANS_MAGIC;
            h->version = GSC_VERSION;
            h->n = a.n;
            h->K = a.K;
            h->nchunks = a.nc;
            h->total = (uint32_t)total;
            h->reserved = 0;
        }
    }
}

__global__ __launch_bounds__(64) void k_rans_info(RansArgs a, int decode)
{
    if (threadIdx.x != 0) return;
    if (!decode && a.nc == 0) {  // an empty input: the header, a zero table and one offset
        gsc_rans_header *h = reinterpret_cast<gsc_rans_header *>(a.out);
        h->magic = GSC_RANS_MAGIC;
        h->version = GSC_VERSION;
        h->n = 0;
        h->K = a.K;
        h->nchunks = 0;
        h->total = 0;
        h->reserved = 0;
        uint16_t *tab = reinterpret_cast<uint16_t *>(a.out + sizeof(gsc_rans_header));
        for (int s = 0; s < 256; ++s) tab[s] = 0;
        *reinterpret_cast<uint32_t *>(a.out + sizeof(gsc_rans_header) + 512) = 0;
    }
    const uint32_t e = __hip_atomic_load(&a.ws[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.info[0] = (int32_t)e;
    a.info[1] = (int32_t)(uint32_t)a.n;
    uint64_t bytes = 0;
    if (!decode && e == 0) {
        const uint32_t total = a.nc ? reinterpret_cast<const uint32_t *>(a.out + sizeof(gsc_rans_header) + 512)[a.nc] : 0u;
        bytes = rans_data_off(a.nc) + total;
    }
    a.info[2] = (int32_t)(uint32_t)(bytes & 0xFFFFFFFFu);
    a.info[3] = (int32_t)(uint32_t)(bytes >> 32);
}

// ---------------------------------------------------------------------------------- decode
// Thread c decodes chunk c. The header, table and offsets are checked first (every thread of a
// block checks the table; thread 0 the header; each thread its own offsets).
__global__ __launch_bounds__(RANS_THREADS) void k_rans_decode(RansArgs a)
{
    __shared__ uint32_t s_f[256], s_st[257];
    __shared__ uint8_t s_sym[RANS_M];
    __shared__ uint32_t s_ok;
    const GAS uint8_t *src = gp(a.src);
    const CAS gsc_rans_header *h = cp(reinterpret_cast<const gsc_rans_header *>(a.src));
    const GAS uint16_t *tab = gp(reinterpret_cast<const uint16_t *>(a.src + sizeof(gsc_rans_header)));
    load_table(tab, s_f, s_st);
    const uint64_t d0 = rans_data_off(a.nc);
    if (threadIdx.x == 0) {
        const bool hdr = h->magic == GSC_RANS_MAGIC && h->n == a.n && h->K == a.K && h->nchunks == a.nc &&
                         d0 + (uint64_t)h->total <= a.cap && s_st[256] == RANS_M;
        s_ok = hdr ? 1u : 0u;
        if (!hdr) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
    }
    __syncthreads();
    if (!s_ok) return;
    for (uint32_t s = 0; s < 256; ++s)  // the slot -> byte table (each thread a share of the slots)
        for (uint32_t j = threadIdx.x; j < s_f[s]; j += RANS_THREADS) s_sym[s_st[s] + j] = (uint8_t)s;
    __syncthreads();
    const uint32_t c = blockIdx.x * RANS_THREADS + threadIdx.x;
    if (c >= a.nc) return;
    const GAS uint32_t *offs = gp(reinterpret_cast<const uint32_t *>(a.src + sizeof(gsc_rans_header) + 512));
    const uint64_t p0 = offs[c], p1 = offs[c + 1];
    if (p1 < p0 + 4 || p1 > h->total) {
        rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
        return;
    }
    const GAS uint8_t *d = src + d0;
    uint64_t p = p0;
    uint32_t x = 0;
    for (int k = 0; k < 4; ++k) x = (x << 8) | d[p++];
    GAS uint8_t *out = gp(a.out);
    const uint64_t b = (uint64_t)c * a.K, e = min(b + a.K, a.n);
    bool bad = false;
    for (uint64_t i = b; i < e; ++i) {
        const uint32_t slot = x & (RANS_M - 1u);
        const uint32_t s = s_sym[slot];
        x = s_f[s] * (x >> RANS_BITS) + slot - s_st[s];
        while (x < RANS_L) {
            if (p >= p1) {
                bad = true;
                break;
            }
            x = (x << 8) | d[p++];
        }
        if (bad) break;
        out[i] = (uint8_t)s;
    }
    if (bad || x != RANS_L || p != p1) rans_error(a.ws, GSC_ERR_CORRUPT_STREAM);
}

// ------------------------------------------------------------------------------- launches
uint64_t rans_chunks(uint64_t n, uint32_t K) { return (n + K - 1) / K; }
uint64_t rans_tmp_stride(uint32_t K) { return ((uint64_t)2 * K + 4 + 15) / 16 * 16; }
uint64_t rans_status_words(uint64_t nc) { return (nc + RANS_THREADS - 1) / RANS_THREADS + 1; }
uint64_t rans_workspace_bytes(uint64_t n, uint32_t K)
{
    const uint64_t nc = rans_chunks(n, K);
    const uint64_t head = (257 * 4 + 7) / 8 * 8 + 8 * rans_status_words(nc);  // error + histogram, status
    return (head + 255) / 256 * 256 + nc * rans_tmp_stride(K);
}
uint64_t rans_capacity_bytes(uint64_t n, uint32_t K)
{
    const uint64_t nc = rans_chunks(n, K);
    // a symbol emits at most 2 bytes (12 bits of frequency 1, aligned to bytes), plus 4 per chunk
    return sizeof(gsc_rans_header) + 512 + 4 * (nc + 1) + 2 * n + 4 * nc;
}

static RansArgs rans_args(uint64_t n, uint32_t K, uint32_t *ws)
{
    RansArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.K = K;
    a.nc = (uint32_t)rans_chunks(n, K);
    a.ws = ws;
    a.status = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(ws) + (257 * 4 + 7) / 8 * 8);
    const uint64_t head = (257 * 4 + 7) / 8 * 8 + 8 * rans_status_words(a.nc);
    a.tmp = reinterpret_cast<uint8_t *>(ws) + (head + 255) / 256 * 256;
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
    const uint32_t zw = (uint32_t)((reinterpret_cast<uint8_t *>(a.tmp) - static_cast<uint8_t *>(ws)) / 4);
    hipLaunchKernelGGL(k_rans_zero, dim3(min((zw + 255) / 256, 1024u)), dim3(256), 0, s, static_cast<uint32_t *>(ws), zw);
    if (a.nc > 0) {
        const uint64_t hw = (n + RANS_HIST_THREADS * 16 - 1) / (RANS_HIST_THREADS * 16);
        const uint32_t hb = (uint32_t)(hw < 1024 ? hw : 1024);
        hipLaunchKernelGGL(k_rans_hist, dim3(hb), dim3(RANS_HIST_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_rans_table, dim3(1), dim3(WAVE), 0, s, a);
        hipLaunchKernelGGL(k_rans_encode, dim3((a.nc + RANS_THREADS - 1) / RANS_THREADS), dim3(RANS_THREADS), 0, s, a);
    }
    hipLaunchKernelGGL(k_rans_info, dim3(1), dim3(64), 0, s, a, 0);
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
    hipLaunchKernelGGL(k_rans_zero, dim3(1), dim3(256), 0, s, static_cast<uint32_t *>(ws), 2u);
    if (a.nc > 0)
        hipLaunchKernelGGL(k_rans_decode, dim3((a.nc + RANS_THREADS - 1) / RANS_THREADS), dim3(RANS_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_rans_info, dim3(1), dim3(64), 0, s, a, 1);
    return hipGetLastError();
}

}  // namespace gsc
