// RAHT on the GPU: prelude, forward transform (+ merge of duplicates and quantization),
// inverse transform (+ dequantization).
//
// The transform is the one of Sec. 3.1-3.3 (Eq. 1, Alg. 4-6): at binary level l = 1..3J every
// left sibling k of the active list I_l merges with its right sibling k+1,
//   [lo; hi] = [a b; -b a] [y0; y1],  a = sqrt(w0/(w0+w1)), b = sqrt(w1/(w0+w1)),
// the low-pass staying at the left entry and the high-pass at the right one. An entry i > 0 is
// removed from the active list (merged as a right sibling) exactly at level
// l_i = msb(M[i-1] xor M[i]) + 1, so I_l = {i : l_i >= l}: the pair of entry i is its nearest
// entries with level >= l_i on either side (its left partner, and the end of its own node).
//
// Tiling. A workgroup owns a tile of RT consecutive entries and performs every merge whose two
// operands lie inside the tile, all levels in LDS. A merge whose left partner lies before the
// tile, or whose right operand extends past it, is deferred: its entry is "open" and moves, with
// its partial low-pass, to the next sequence S_{k+1}. The merges among open entries are exactly
// the deferred merges (an open entry's neighbours in the active list are open too), so the same
// kernels run again on S_{k+1}, until one tile holds the whole sequence. At most 6J entries of a
// tile are open (the merges whose parent straddles one of its two boundaries: one per level).
//
// Inside a tile, a merge whose two operands lie in one 64-entry chunk depends only on merges of
// that chunk. Each wave first performs the merges of its own chunk, level by level, ordered by
// the wave's own instruction stream; then the few merges that cross chunks run level by level
// with workgroup barriers (the inverse runs the two phases in the opposite order).
#include <mutex>

#include "gsc_device.h"

namespace gsc {

static_assert(RT == RAHT_THREADS && RT % WAVE == 0, "a tile is one 64-entry chunk per wave");
static_assert(RT < 1024, "merge records pack three 10-bit positions");
// The schedule of a tile is built by RT / EPT threads, EPT entries each. The first level uses
// two entries per thread: with half as many waves per tile, all first-level tiles of a
// 1M-voxel frame fit on the GPU at once (the wave slots, not the work, limited that launch).
// The upper levels are a short chain of few tiles, where a tile's latency counts: one entry
// per thread.
constexpr int PRE_EPT1 = 2, PRE_EPT_UP = 1;
constexpr int NCHUNK = RT / WAVE;
constexpr int CROSS = NCHUNK;  // class of merges that cross chunks

// Size of the entry sequence S_k; a size beyond its allocation (impossible when every tile
// leaves at most 6J + 2 entries open) is reported and treated as empty.
// LIVE: the size may have been written during the running launch (a persistent upper-level
// launch), so it is read with a device-coherent load; otherwise it was written by an earlier
// kernel and is read through the constant address space. The sizes of S_1 and S_2 always come
// from earlier launches (the first level's schedule is a launch of its own).
template <bool LIVE = false, class FD>
__device__ inline uint32_t seq_size(FD &fd, Ctrl *ctrl, int k)
{
    const uint32_t nk = k == 1 ? cp(ctrl)->n_vox
                       : (LIVE && k >= 3) ? __builtin_amdgcn_readfirstlane(__hip_atomic_load(&ctrl->lvl_n[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                          : cp(ctrl)->lvl_n[k];
    if (nk > fd.lv[k].cap) {
        set_error(ctrl, GSC_ERR_INTERNAL);
        return 0;
    }
    return nk;
}
__device__ inline bool seq_active(uint32_t nk, int k) { return k == 1 ? nk >= 1 : nk >= 2; }

// A value that is the same in every lane, said so to the compiler, so that a loop over its bits
// runs on the scalar unit.
__device__ inline uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The rotation (a, b) = (sqrt(w0/(w0+w1)), sqrt(w1/(w0+w1))) of a merge of weights w0, w1
// (Eq. 1): FP32 division and square root, or (GSC_FLAG_FP64_WEIGHTS) FP64 rounded once to FP32.
__device__ inline float2 rotation(uint32_t w0, uint32_t w1, bool fp64)
{
    if (fp64) {
        const double sum = (double)w0 + (double)w1;
        return make_float2((float)sqrt((double)w0 / sum), (float)sqrt((double)w1 / sum));
    }
    const float f0 = (float)w0, f1 = (float)w1, sum = f0 + f1;
    return make_float2(sqrtf(f0 / sum), sqrtf(f1 / sum));
}

// Whether a frame's rotations are computed in FP64: the encoder's flag, which a decoder reads
// from the stream header (only from a stream that holds one: a shorter stream fails the header
// check, and the items that still ask here are not transformed).
template <class FD>
__device__ inline bool fp64_weights(FD &fd)
{
    if (fd.mode == MODE_DECODE)
        return fd.in_bytes >= GSC_HEADER_BYTES &&
               (cp(reinterpret_cast<const gsc_header *>(fd.in_stream))->flags & GSC_FLAG_FP64_WEIGHTS) != 0;
    return (fd.flags & GSC_FLAG_FP64_WEIGHTS) != 0;
}

// ============================================================================ prelude
// Per tile, one thread per entry: the entry's binary level l; the tile's active lists as one
// 64-bit ballot per (level, wave chunk); the entry's left partner and node end as the nearest
// set bits of its level's ballots. A merge is local when both lie inside the tile (the node may
// also end exactly at the tile end when the next entry survives to a higher level); otherwise
// the entry is open. Local merges are stored sorted by (round, class), the class being the
// wave chunk holding the whole merge or CROSS. A merge's round is one more than the rounds of the
// merges of its chunk that produced its two operands (0 for an operand not produced yet); a
// crossing merge's round is its binary level (crossing merges run after every chunk's own
// merges). The transforms take the rounds in order, so merges of a chunk that do not depend on
// one another run together, and a chunk takes as many steps as its merge tree is deep instead of
// one per binary level that holds a merge. The order of the merges that read or write any one
// entry is unchanged, so the results are the same. Open entries are compacted in order into
// S_{k+1} with a decoupled look-back whose aggregate is published as soon as the tile's open
// entries are known and whose prefix is resolved after the rest of the tile's work.
constexpr int PRE_TILES = 1;  // tiles per workgroup

// lc (first level only, or null): the codes of entries s - 1 .. s + RT of the tile starting at
// entry s, in LDS (lc[j] = code of entry s - 1 + j); otherwise they are read from the leaf codes.
template <bool LIVE, int PRE_EPT>
__device__ inline void prelude_tile(const TileMap &m, uint32_t f, int k, uint32_t tile, const uint64_t *lc = nullptr)
{
    static_assert(PRE_TILES == 1, "one tile per workgroup");
    constexpr int PRE_THREADS = RT / PRE_EPT, PRE_BLOCK = PRE_THREADS;
    constexpr int PRE_WAVES = PRE_THREADS / WAVE;
    constexpr int PRE_SEG = (SEG_N + PRE_THREADS - 1) / PRE_THREADS;  // segment counts per thread
    static_assert(PRE_EPT == 1 || PRE_EPT == 2, "one or two entries per thread");
    __shared__ uint32_t s_lvl_e;
    __shared__ uint64_t s_mask[NLVL][NCHUNK];
    __shared__ uint32_t s_cnt[SEG_N], s_fill[SEG_N];
    __shared__ uint32_t s_tmp[PRE_BLOCK / WAVE + 1];
    __shared__ uint8_t s_rdl[RT];  // round of the chunk merge that last wrote an entry
    __shared__ LbScratch<PRE_BLOCK / WAVE> s_lb;

    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    if ((uint32_t)k > fd.K) return;
    const uint32_t err = load_error(ctrl);  // (in flight while the sequence's size is read)
    const uint32_t nk = seq_size<LIVE>(fd, ctrl, k);
    if (err || !seq_active(nk, k)) return;
    auto &lv = fd.lv[k];
    const uint32_t s = tile * RT;
    if (s >= nk) return;  // uniform: the tile is past the end
    const uint32_t e = min(nk, s + RT);
    const int mlen = (int)(e - s);
    const GAS uint64_t *codes = gp((fd.mode == MODE_FWD_F32 || fd.mode == MODE_ADJ_F32) ? fd.codes_in : fd.leaf);
    const GAS uint8_t *slvl = gp(lv.s_lvl);

    // thread t holds entries j(x) = t + x PRE_THREADS, x < PRE_EPT: entry j(x) lies in wave
    // chunk w + x PRE_WAVES, and the chunk-wide steps (ballots, rounds) run once per chunk
    const uint32_t t = threadIdx.x, w = t / WAVE, lane = lane_id();
    int jj[PRE_EPT];
    uint32_t lvl[PRE_EPT];  // 0: no entry
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) jj[x] = (int)(t + x * PRE_THREADS);
    // both entries' loads before any use, at clamped positions (a load under a per-entry
    // condition would be waited for where its branch joins)
    if (k == 1) {
        uint64_t c0[PRE_EPT], c1[PRE_EPT];
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x) {
            const uint32_t i = s + (uint32_t)min(jj[x], mlen - 1);
            c0[x] = lc ? lc[i - s] : codes[i > 0 ? i - 1 : 0];
            c1[x] = lc ? lc[i - s + 1] : codes[i];
        }
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x)
            lvl[x] = jj[x] < mlen ? (s + jj[x] == 0 ? LVL_NONE : merge_level(c0[x], c1[x])) : 0u;
    } else {
        uint32_t l[PRE_EPT];
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x) l[x] = slvl[s + (uint32_t)min(jj[x], mlen - 1)];
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x) lvl[x] = jj[x] < mlen ? l[x] : 0u;
    }
    for (uint32_t q = t; q < (uint32_t)SEG_N; q += PRE_THREADS) {
        s_cnt[q] = 0;
        s_fill[q] = 0;
    }
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) s_rdl[jj[x]] = 0;
    if (t == 0)
        s_lvl_e = e < nk ? (k == 1 ? (lc ? merge_level(lc[RT], lc[RT + 1]) : merge_level(codes[e - 1], codes[e])) : slvl[e])
                         : LVL_NONE;
    // active lists of the levels that can hold a merge: an entry merges at a level of at most 3J
    // (the tile's first entry of the sequence, LVL_NONE, is in every list and is never a right
    // sibling). s_mask[q][c] has bit i set when entry i of chunk c has a level >= q. Levels are
    // below 128, so seven ballots give the bit planes of a chunk's levels; lane q compares every
    // entry's level with q on those planes (most significant bit first: an entry is below q
    // from the first bit where the two differ and q has a one) and stores the list of level q.
    static_assert(NLVL <= WAVE && LVL_NONE < 128, "one lane per level; seven bit planes");
    const uint32_t nlvl = min(3u * fd.J + 1u, (uint32_t)NLVL);
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        uint64_t plane[7];
#pragma unroll
        for (int bit = 0; bit < 7; ++bit) plane[bit] = __ballot((lvl[x] >> bit) & 1u);
        uint64_t below = 0, same = ~0ull;  // entries below lane's q; entries equal so far
#pragma unroll
        for (int bit = 6; bit >= 0; --bit) {
            const uint64_t qm = ((lane >> bit) & 1u) ? ~0ull : 0ull;
            below |= same & ~plane[bit] & qm;
            same &= ~(plane[bit] ^ qm);
        }
        if (lane >= 1 && lane < nlvl) s_mask[lane][w + x * PRE_WAVES] = ~below;
    }
    __syncthreads();

    const uint32_t lvl_e = s_lvl_e;
    bool is_local[PRE_EPT], is_open[PRE_EPT];
    int left[PRE_EPT], right[PRE_EPT];
    uint32_t cls[PRE_EPT];
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        const uint32_t wc = w + x * PRE_WAVES;  // the entry's chunk
        const uint32_t lv_ = lvl[x];
        is_local[x] = is_open[x] = false;
        left[x] = -1;
        right[x] = mlen;
        cls[x] = CROSS;
        if (jj[x] < mlen) {
            if (lv_ >= 1 && lv_ < (uint32_t)NLVL) {
                const uint64_t below = lanemask_lt();
                const uint64_t above = ~below & ~(1ull << lane);
                uint64_t mm = s_mask[lv_][wc] & below;
                if (mm) {
                    left[x] = (int)(wc * WAVE) + msb64(mm);
                } else {
                    for (int ww = (int)wc - 1; ww >= 0; --ww) {
                        const uint64_t b = s_mask[lv_][ww];
                        if (b) {
                            left[x] = ww * WAVE + msb64(b);
                            break;
                        }
                    }
                }
                mm = s_mask[lv_][wc] & above;
                if (mm) {
                    right[x] = (int)(wc * WAVE) + (__ffsll((long long)mm) - 1);
                } else {
                    for (int ww = (int)wc + 1; ww < NCHUNK; ++ww) {
                        const uint64_t b = s_mask[lv_][ww];
                        if (b) {
                            right[x] = ww * WAVE + (__ffsll((long long)b) - 1);
                            break;
                        }
                    }
                }
                is_local[x] = left[x] >= 0 && (right[x] < mlen || lvl_e > lv_);
                is_open[x] = !is_local[x];
                if (is_local[x] && left[x] / WAVE == (int)wc && (right[x] - 1) / WAVE == (int)wc) cls[x] = wc;
            } else {
                is_open[x] = true;  // entry 0 of the sequence never merges as a right sibling
            }
        }
    }
    // ---- open entries in order: ranks in the tile (the entries j(0) of all threads come before
    // the entries j(1): one scan of the two flags packed in one word), the tile's count published
    // at once (its prefix is resolved at the end, after the rest of the work)
    static_assert(PRE_THREADS < 65536, "two 16-bit counts per scanned word");
    uint32_t ptot;
    const uint32_t pex = block_excl_scan<PRE_BLOCK>((is_open[0] ? 1u : 0u) | ((PRE_EPT > 1 && is_open[PRE_EPT - 1] ? 1u : 0u) << 16), s_tmp, &ptot);
    const uint32_t total = (ptot & 0xFFFFu) + (ptot >> 16);
    uint32_t rank[PRE_EPT];
    rank[0] = pex & 0xFFFFu;
    if (PRE_EPT > 1) rank[PRE_EPT - 1] = (ptot & 0xFFFFu) + (pex >> 16);
    lookback_block_publish<OpSum>(lv.status, 1, tile, total);
    // ---- rounds: each chunk's own merges by its wave (levels ascending, no workgroup barrier).
    // A local merge's partner lies in the entry's own chunk, so the wave's chunks (one per entry
    // slot) touch disjoint entries and walk the union of their levels in one loop.
    bool mine[PRE_EPT];
    uint32_t rnd[PRE_EPT];
    uint64_t lm = 0;
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        mine[x] = is_local[x] && cls[x] != CROSS;  // (then cls is the entry's own chunk)
        rnd[x] = 0;
        lm |= mine[x] ? 1ull << lvl[x] : 0ull;
    }
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) lm |= __shfl_xor(lm, o, WAVE);
    lm = uniform64(lm);
    while (lm) {
        const uint32_t q = (uint32_t)(__ffsll((long long)lm) - 1);
        lm &= ~(1ull << q);
        uint32_t prev[PRE_EPT];
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x)
            prev[x] = mine[x] && lvl[x] == q ? max((uint32_t)s_rdl[left[x]], (uint32_t)s_rdl[jj[x]]) : 0u;
#pragma unroll
        for (int x = 0; x < PRE_EPT; ++x) {
            if (mine[x] && lvl[x] == q) {
                rnd[x] = 1u + prev[x];
                s_rdl[left[x]] = (uint8_t)rnd[x];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // ---- segment counts: a chunk's merges are counted by its own wave with ballots (only one
    // wave holds a chunk's merges; the rank in the ballot is the record's place in its segment);
    // crossing merges keep their binary level as their round (a round of their own would cost a
    // workgroup barrier per level) and are counted with LDS atomics
    uint32_t wrank[PRE_EPT];
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        wrank[x] = 0;
        uint64_t rm = mine[x] ? 1ull << rnd[x] : 0ull;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) rm |= __shfl_xor(rm, o, WAVE);
        rm = uniform64(rm);
        while (rm) {
            const uint32_t r = (uint32_t)(__ffsll((long long)rm) - 1);
            rm &= ~(1ull << r);
            const uint64_t bal = __ballot(mine[x] && rnd[x] == r);
            if (mine[x] && rnd[x] == r) wrank[x] = (uint32_t)__popcll(bal & lanemask_lt());
            if (lane == 0) s_cnt[r * NCLS + w + x * PRE_WAVES] = (uint32_t)__popcll(bal);
        }
    }
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        if (is_local[x] && cls[x] == CROSS) {
            rnd[x] = lvl[x];
            atomicAdd(&s_cnt[rnd[x] * NCLS + CROSS], 1u);
        }
    }
    __syncthreads();
    if (t < WAVE) {  // round masks of the classes: lane q tests round q
#pragma unroll
        for (uint32_t c = 0; c < (uint32_t)NCLS; ++c) {
            const uint64_t b = __ballot(s_cnt[t * NCLS + c] != 0);
            if (t == 0) gp(lv.lmask)[(size_t)tile * NCLS + c] = b;
        }
    }
    {   // segment starts: exclusive scan of the SEG_N counts (PRE_SEG per thread)
        uint32_t a[PRE_SEG], sum = 0;
#pragma unroll
        for (int q = 0; q < PRE_SEG; ++q) {
            const uint32_t i = PRE_SEG * t + q;
            a[q] = i < (uint32_t)SEG_N ? s_cnt[i] : 0u;
            sum += a[q];
        }
        uint32_t ex = group_excl_scan<PRE_BLOCK, PRE_THREADS>(sum, s_tmp, nullptr);
#pragma unroll
        for (int q = 0; q < PRE_SEG; ++q) {
            const uint32_t i = PRE_SEG * t + q;
            if (i < (uint32_t)SEG_N) s_cnt[i] = ex;
            ex += a[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        if (is_local[x]) {
            const uint32_t seg = rnd[x] * NCLS + cls[x];
            const uint32_t slot = s_cnt[seg] + (mine[x] ? wrank[x] : atomicAdd(&s_fill[seg], 1u));
            if (slot < (uint32_t)RT)
                gp(lv.rec)[(size_t)tile * RT + slot] =
                    (uint32_t)jj[x] | ((uint32_t)left[x] << 10) | ((uint32_t)right[x] << 20);
        }
    }
    for (uint32_t q = t; q < (uint32_t)LSTART_N; q += PRE_THREADS)
        gp(lv.lstart)[(size_t)tile * LSTART_N + q] = q < (uint32_t)SEG_N ? (uint16_t)s_cnt[q] : 0;

    // ---- the open entries' places in S_{k+1}
    const uint32_t base = (uint32_t)lookback_block_resolve<OpSum, PRE_BLOCK>(lv.status, 1, tile, total, ctrl, s_lb);
#pragma unroll
    for (int x = 0; x < PRE_EPT; ++x) {
        if (is_open[x]) {
            if (rank[x] < (uint32_t)OPEN_CAP) gp(lv.opos)[(size_t)tile * OPEN_CAP + rank[x]] = (uint16_t)jj[x];
            if ((uint32_t)k < fd.K) {
                auto &nx = fd.lv[k + 1];
                const uint32_t o = base + rank[x];
                if (o < nx.cap) {
                    gp(nx.s_idx)[o] = k == 1 ? s + jj[x] : gp(lv.s_idx)[s + jj[x]];
                    gp(nx.s_lvl)[o] = (uint8_t)lvl[x];
                }
            }
        }
    }
    if (t == 0) {
        if (total > open_max((int)fd.J)) set_error(ctrl, GSC_ERR_INTERNAL);
        lv.obase[tile] = base;
        lv.ocnt[tile] = min(total, (uint32_t)OPEN_CAP);
        if (e == nk) ctrl->lvl_n[k + 1] = base + total;
    }
}

// One workgroup per tile of the first level.
constexpr int PRE_BLOCK1 = RT / PRE_EPT1;
__global__ __launch_bounds__(PRE_BLOCK1) void k_prelude(TileMap m, int k)
{
    const uint32_t f = frame_of(m, blockIdx.x);
    prelude_tile<false, PRE_EPT1>(m, f, k, tile_index(m, f));
}

// The decoder's leaves and first-level schedule in one launch. A workgroup takes the RT leaves
// of one tile (two per thread, entries t and t + PRE_BLOCK1 as in the schedule) and the leaves
// just before and after the tile (threads 0 and 1): each leaf's code from the child bits on its
// path to the root (level J's bit least significant; J dependent loads of the node's child bit
// and parent, written by the octree decoding launch, the three walks of a thread interleaved),
// which is the code the level-by-level expansion produces (Alg. 2-3). The leaves' centres (and
// codes and voxel coordinates when asked for) are written, and the codes go through LDS to the
// tile's schedule (prelude_tile).
__global__ __launch_bounds__(PRE_BLOCK1) void k_dec_prelude(TileMap m)
{
    static_assert(PRE_EPT1 == 2, "two leaves per thread");
    __shared__ uint64_t s_code[RT + 2];
    const uint32_t f = frame_of(m, blockIdx.x);
    const uint32_t tile = tile_index(m, f);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    const gsc_header *hg = reinterpret_cast<const gsc_header *>(fd.in_stream);
    const CAS gsc_header *h = cp(hg);
    // (checked by the octree decoding launch, which flags a stream shorter than the header: the
    // count is read only from a stream that holds it)
    const uint32_t J = fd.J, nv = fd.in_bytes >= GSC_HEADER_BYTES ? h->n_vox : 0u;
    const uint32_t err = load_error(fd.ctrl);  // (after the header's loads: waited for with them)
    const uint32_t s = tile * RT;
    if (__builtin_amdgcn_readfirstlane(err) || s >= nv) return;
    const uint32_t t = threadIdx.x;
    const GAS uint32_t *par = gp(fd.dec_par);
    const GAS uint8_t *cbit = gp(fd.dec_cbit);
    // leaves v[0], v[1] of the tile; v[2]: s - 1 (thread 0) or s + RT (thread 1), else a repeat
    uint32_t v[3], x[3];
    uint64_t code[3];
    v[0] = s + t;
    v[1] = s + t + PRE_BLOCK1;
    v[2] = t == 0 ? (s > 0 ? s - 1 : s) : (t == 1 ? s + RT : v[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        code[i] = 0;
        x[i] = min(v[i], nv - 1);  // (a leaf past the end walks the last one's path)
    }
    uint64_t qL = 0;  // Q(L): nodes of levels 1..L-1
    for (uint32_t L = 1; L < J; ++L) qL += h->level_sizes[L];
    for (uint32_t L = J; L >= 1; --L) {
        const uint32_t size = h->level_sizes[L];
        uint64_t g[3];
        uint32_t cb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) g[i] = qL + min(x[i], size - 1);  // (clamped: never an access outside the nodes)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cb[i] = cbit[g[i]];
            x[i] = par[g[i]];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) code[i] |= (uint64_t)cb[i] << (3 * (J - L));
        if (L > 1) qL -= h->level_sizes[L - 1];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (v[i] < nv) emit_leaf(fd, hg, v[i], code[i]);
        s_code[1 + t + i * PRE_BLOCK1] = code[i];
    }
    if (t == 0) s_code[0] = code[2];
    if (t == 1) s_code[RT + 1] = code[2];
    __syncthreads();
    prelude_tile<false, PRE_EPT1>(m, f, 1, tile, s_code);
}

hipError_t launch_dec_prelude(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_prelude, dim3(m.start[m.F]), dim3(PRE_BLOCK1), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_prelude(const TileMap &m, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_prelude, dim3(m.start[m.F]), dim3(PRE_BLOCK1), 0, s, m, k);
    return hipGetLastError();
}

// ------------------------------------------------- upper levels: one persistent launch each
// The upper sequences are small and their true sizes are known only on the device (the bound of
// 6J + 2 open entries per tile is far above what real frames leave), so a launch per level and
// per worst-case tile would mostly start idle workgroups. Instead one launch of G resident
// workgroups visits the levels in order; at each level workgroup b takes the level's items
// b, b + G, ... (items over all frames of the launch, frame by frame), and the levels are
// ordered with per-workgroup phase flags. Item counts never grow from one level to the next
// (S_{k+1} is a subset of S_k's entries), so workgroups beyond a level's count leave.

// Items of level k over the frames of the launch (each frame: its tiles of S_k times np), with
// the frames' first items in s_fs[0..F]; uniform. lvl_n[k], k >= 3, is read with device-coherent
// loads: the running launch writes it (S_2's size comes from the first level's schedule launch).
__device__ inline uint32_t level_items(const TileMap &m, int k, uint32_t np, uint32_t *s_fs)
{
    if (threadIdx.x < WAVE) {
        uint32_t c = 0;
        if (threadIdx.x < m.F) {
            const CAS FrameDesc &fd = *cp(m.fd[threadIdx.x]);
            if ((uint32_t)k <= fd.K) {
                const uint32_t nk = k >= 3 ? __hip_atomic_load(&fd.ctrl->lvl_n[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                           : cp(fd.ctrl)->lvl_n[k];
                if (nk >= 2 && nk <= fd.lv[k].cap) c = (nk + RT - 1) / RT * np;
            }
        }
        const uint32_t inc = wave_incl_scan(c);
        s_fs[threadIdx.x + 1] = inc;
        if (threadIdx.x == 0) s_fs[0] = 0;
    }
    __syncthreads();
    const uint32_t total = s_fs[m.F];
    __syncthreads();  // (s_fs is read again by the caller before it is rewritten)
    return total;
}
__device__ inline uint32_t item_frame(const TileMap &m, const uint32_t *s_fs, uint32_t i)
{
    uint32_t f = 0;
    while (f + 1 < m.F && s_fs[f + 1] <= i) ++f;
    return f;
}
static_assert(GSC_MAX_BATCH <= WAVE, "one wave counts the frames' items");

// Schedules of the upper levels 2 .. kmax (the prelude of every tile of S_k, k >= 2), by the
// first Gp workgroups of a persistent launch (all resident). A level's size is known only once
// the previous level is done, so the group's workgroups wait for the previous level's producers
// (phase flags) before they count its tiles; a workgroup without a tile at a level leaves the
// group (the later levels are no larger). A workgroup that leaves releases its writes and adds
// itself to the group's counter, which reaches Gp once every level's schedule is written.
__device__ inline void up_prelude_group(const TileMap &m, int kmax, uint32_t Gp, uint32_t *s_fs, GAS uint32_t *pre_done)
{
    const CAS FrameDesc &fd0 = *cp(m.fd[0]);
    uint32_t *flags = fd0.lvl_flags;
    uint32_t phase = PHASE_PRELUDE;
    for (int k = 2; k <= kmax; ++k) {
        const uint32_t items = level_items(m, k, 1, s_fs);
        if (blockIdx.x >= items) break;
        for (uint32_t i = blockIdx.x; i < items; i += Gp) {
            const uint32_t f = item_frame(m, s_fs, i);
            prelude_tile<true, PRE_EPT_UP>(m, f, k, i - s_fs[f]);
            __syncthreads();
        }
        if (k == kmax) break;
        const uint32_t np = min(items, Gp);  // the workgroups that took an item
        level_publish(flags, ++phase);
        level_wait(flags, np, phase, fd0.ctrl);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(pre_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

uint32_t prelude_blocks(uint32_t tiles) { return ceil_div(tiles, PRE_TILES); }

// =========================================================== shared transform pieces
// A merge record (entry j | left partner l << 10 | node end r << 20, positions in the tile) as
// kept in LDS for the transforms: the slice rows of its two operands, l CH4 | j CH4 << 16
// (at most 511 * 8 < 2^16), so that a butterfly needs no multiply to address them.
__device__ inline uint32_t lds_rec(uint32_t rec, uint32_t CH4)
{
    return ((rec >> 10) & 1023u) * CH4 | (((rec & 1023u) * CH4) << 16);
}

struct TileSched {
    uint32_t tile, s, e, nk, obase, ocnt, nrec;
    int mlen;
    bool final_level;
};

// Loads the schedule of a tile of an upper level (k >= 2) into LDS: segment starts, level masks,
// open positions, voxel indices of the entries, and the records with (a, b) of every local merge.
// Returns false if the workgroup has nothing to do.
template <class FD>
__device__ inline bool load_schedule(FD &fd, Ctrl *ctrl, int k, uint32_t tile,
                                     uint32_t CH4, TileSched &ts, uint32_t *s_rec, float2 *s_ab,
                                     uint16_t *s_lst, uint16_t *s_opos, uint32_t *s_idx,
                                     unsigned long long *s_lmask)
{
    // (the size may have been written by schedule workgroups of the same launch)
    const uint32_t nk = seq_size<true>(fd, ctrl, k);
    if (!seq_active(nk, k)) return false;
    auto &lv = fd.lv[k];
    const uint32_t s = tile * RT;
    if (s >= nk) return false;
    const uint32_t tid = threadIdx.x;  // RAHT_THREADS threads, one per entry
    ts.tile = tile;
    ts.s = s;
    ts.e = min(nk, s + RT);
    ts.nk = nk;
    ts.mlen = (int)(ts.e - s);
    ts.final_level = nk <= (uint32_t)RT;
    const GAS uint16_t *lstart = gp(lv.lstart), *opos = gp(lv.opos);
    const GAS uint32_t *sidx = gp(lv.s_idx), *recs = gp(lv.rec);
    // Every load is issued at once, at clamped in-bounds slots, and none waits on another (one
    // memory round trip): the counts, the segment starts, the masks, all OPEN_CAP open
    // positions, the voxel indices and all RT record slots; slots past the tile's counts are
    // read but not used.
    static_assert(RAHT_THREADS == RT && LSTART_N <= 2 * RAHT_THREADS && OPEN_CAP <= RAHT_THREADS, "one entry per thread");
    const uint32_t obase = lv.obase[tile], ocnt = lv.ocnt[tile];
    const size_t lb = (size_t)tile * LSTART_N;
    const uint16_t ls0 = lstart[lb + tid], ls1 = lstart[lb + min(tid + (uint32_t)RT, (uint32_t)LSTART_N - 1)];
    const uint16_t op = opos[(size_t)tile * OPEN_CAP + min(tid, (uint32_t)OPEN_CAP - 1)];
    const unsigned long long lmk = gp(lv.lmask)[(size_t)tile * NCLS + min(tid, (uint32_t)NCLS - 1)];
    const uint32_t jl = min(tid, (uint32_t)ts.mlen - 1);
    const uint32_t vi = sidx[s + jl];
    const uint32_t rec = recs[(size_t)tile * RT + tid];
    const uint32_t ve = sidx[min(ts.e, nk - 1)], nv = ctrl->n_vox;
    const uint32_t vend = ts.e < nk ? ve : nv;
    ts.obase = obase;
    ts.ocnt = ocnt;
    s_lst[tid] = ls0;
    if (tid + RT < (uint32_t)LSTART_N) s_lst[tid + RT] = ls1;
    if (tid < (uint32_t)OPEN_CAP) s_opos[tid] = op;
    if (tid < (uint32_t)NCLS) s_lmask[tid] = lmk;
    // voxel indices, clamped to the frame's capacity like every row index read from the workspace
    const uint32_t cap = fd.n;
    if (tid < (uint32_t)ts.mlen) s_idx[tid] = min(vi, cap ? cap - 1 : 0u);
    if (tid == 0) s_idx[ts.mlen] = min(vend, cap);
    __syncthreads();
    ts.nrec = s_lst[SEG_N - 1];
    const bool fp64 = fp64_weights(fd);
    if (tid < ts.nrec) {
        const uint32_t q = tid;
        s_rec[q] = lds_rec(rec, CH4);
        const uint32_t ij = s_idx[rec & 1023u], il = s_idx[(rec >> 10) & 1023u], ir = s_idx[rec >> 20];
        s_ab[q] = rotation(ij - il, ir - ij, fp64);
    }
    return true;
}


// One butterfly on channels [4*c4, 4*c4+4) of merge record `rec` (in the form of lds_rec).
__device__ inline void butterfly(float4 *s_y, uint32_t C4, uint32_t rec, float2 ab, uint32_t c4,
                                 bool inverse)
{
    // rec: the LDS rows of the merge's left and right operands, already times the slice width
    // (see lds_rec)
    const uint32_t yl = rec & 0xFFFFu, yj = rec >> 16;
    const float4 y0 = s_y[yl + c4], y1 = s_y[yj + c4];
    float4 lo, hi;
    if (!inverse) {
        lo.x = ab.x * y0.x + ab.y * y1.x;
        lo.y = ab.x * y0.y + ab.y * y1.y;
        lo.z = ab.x * y0.z + ab.y * y1.z;
        lo.w = ab.x * y0.w + ab.y * y1.w;
        hi.x = -ab.y * y0.x + ab.x * y1.x;
        hi.y = -ab.y * y0.y + ab.x * y1.y;
        hi.z = -ab.y * y0.z + ab.x * y1.z;
        hi.w = -ab.y * y0.w + ab.x * y1.w;
    } else {
        lo.x = ab.x * y0.x - ab.y * y1.x;
        lo.y = ab.x * y0.y - ab.y * y1.y;
        lo.z = ab.x * y0.z - ab.y * y1.z;
        lo.w = ab.x * y0.w - ab.y * y1.w;
        hi.x = ab.y * y0.x + ab.x * y1.x;
        hi.y = ab.y * y0.y + ab.x * y1.y;
        hi.z = ab.y * y0.z + ab.x * y1.z;
        hi.w = ab.y * y0.w + ab.x * y1.w;
    }
    s_y[yl + c4] = lo;
    s_y[yj + c4] = hi;
}

// Per-thread roles: in a workgroup step, thread t handles channel chunk t % C4 of row t / C4
// (RPB rows per step); in a wave step, lane L handles chunk L % C4 of merge L / C4 (MPW
// merges per step). A slice has C4 <= max(CH4_MAX, CH4_MAX1) = 8 chunks, so RPB >= 64 and
// MPW >= 8.
struct Roles {
    uint32_t C4, RPB, row0, c4, MPW, wq, wc4, w;
    bool act, wact;
    __device__ explicit Roles(uint32_t C4_) : C4(C4_)
    {
        const uint32_t tid = threadIdx.x, lane = lane_id();
        RPB = RAHT_THREADS / C4;
        row0 = tid / C4;
        c4 = tid % C4;
        act = row0 < RPB;
        MPW = WAVE / C4;
        wq = lane / C4;
        wc4 = lane % C4;
        wact = wq < MPW;
        w = tid / WAVE;
    }
};

// The next level to visit in a mask of levels: ascending (forward) or descending (inverse).
__device__ inline uint32_t next_level(uint64_t mask, bool inverse)
{
    return inverse ? (uint32_t)msb64(mask) : (uint32_t)(__ffsll((long long)mask) - 1);
}


// Merges local to this wave's chunk, levels ascending (forward) or descending (inverse). Lane x
// holds the record range of level x in registers (read out with readlane), and each level's first
// record of a lane is loaded while the previous level runs, so a level costs one LDS round trip.
// The wave's own LDS accesses are performed in program order; the fence keeps the compiler from
// moving one level's accesses across the next level's. Only channel chunks below nch are live.
__device__ inline void wave_phase(float4 *s_y, const Roles &R, const uint32_t *s_rec,
                                  const float2 *s_ab, const uint16_t *s_lst, uint64_t mask,
                                  uint32_t nch, bool inverse, uint32_t cls)
{
    const bool live = R.wact && R.wc4 < nch;
    const uint32_t lane = lane_id();
    const uint32_t lq0 = s_lst[lane * NCLS + cls], lq1 = s_lst[lane * NCLS + cls + 1];
    mask = uniform64(mask);  // one class per wave: one mask per wave
    uint32_t x = mask ? next_level(mask, inverse) : 0u;
    uint32_t q0 = __builtin_amdgcn_readlane(lq0, x), q1 = __builtin_amdgcn_readlane(lq1, x);
    uint32_t rec = 0;
    float2 ab = make_float2(0.f, 0.f);
    if (live && q0 + R.wq < q1) {
        rec = s_rec[q0 + R.wq];
        ab = s_ab[q0 + R.wq];
    }
    while (mask) {
        mask &= ~(1ull << x);
        const uint32_t xn = mask ? next_level(mask, inverse) : 0u;
        const uint32_t q0n = __builtin_amdgcn_readlane(lq0, xn), q1n = __builtin_amdgcn_readlane(lq1, xn);
        uint32_t recn = 0;
        float2 abn = make_float2(0.f, 0.f);
        if (mask && live && q0n + R.wq < q1n) {
            recn = s_rec[q0n + R.wq];
            abn = s_ab[q0n + R.wq];
        }
        if (live && q0 + R.wq < q1) {
            butterfly(s_y, R.C4, rec, ab, R.wc4, inverse);
            for (uint32_t q = q0 + R.wq + R.MPW; q < q1; q += R.MPW)
                butterfly(s_y, R.C4, s_rec[q], s_ab[q], R.wc4, inverse);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        x = xn;
        q0 = q0n;
        q1 = q1n;
        rec = recn;
        ab = abn;
    }
}

// Merges crossing chunks: few per level (a node crosses a chunk boundary only where it holds
// one), so wave 0 performs them all, level by level in its own instruction order, and the
// workgroup waits at one barrier instead of one per level.
__device__ inline void cross_phase(float4 *s_y, const Roles &R, const uint32_t *s_rec,
                                   const float2 *s_ab, const uint16_t *s_lst, uint64_t mask,
                                   uint32_t nch, bool inverse)
{
    if (__builtin_amdgcn_readfirstlane(R.w) == 0)
        wave_phase(s_y, R, s_rec, s_ab, s_lst, mask, nch, inverse, CROSS);
    __syncthreads();
}

__device__ inline float get4(const float4 &v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Channels [4*c4, 4*c4+4) of row `row` of a row-major matrix with C columns. VEC: C % 4 == 0
// and 16-byte aligned base, one 16-byte access; otherwise element accesses guarded by C.
template <bool VEC>
__device__ inline float4 ld4(const GAS float *base, uint64_t row, uint32_t C, uint32_t c4)
{
    const GAS float *p = base + row * C + 4 * c4;
    if (VEC) return gload4(p);
    const uint32_t c = 4 * c4;
    return make_float4(c + 0 < C ? p[0] : 0.f, c + 1 < C ? p[1] : 0.f, c + 2 < C ? p[2] : 0.f,
                       c + 3 < C ? p[3] : 0.f);
}
template <bool VEC>
__device__ inline int4 ldq4(const GAS int32_t *base, uint64_t row, uint32_t C, uint32_t c4)
{
    const GAS int32_t *p = base + row * C + 4 * c4;
    if (VEC) return gload4i(p);
    const uint32_t c = 4 * c4;
    return make_int4(c + 0 < C ? p[0] : 0, c + 1 < C ? p[1] : 0, c + 2 < C ? p[2] : 0,
                     c + 3 < C ? p[3] : 0);
}
template <bool VEC>
__device__ inline void st4(GAS float *base, uint64_t row, uint32_t C, uint32_t c4, const float4 &v)
{
    GAS float *p = base + row * C + 4 * c4;
    if (VEC) {
        gstore4(p, v);
        return;
    }
    const uint32_t c = 4 * c4;
    if (c + 0 < C) p[0] = v.x;
    if (c + 1 < C) p[1] = v.y;
    if (c + 2 < C) p[2] = v.z;
    if (c + 3 < C) p[3] = v.w;
}
template <bool VEC>
__device__ inline void stq4(GAS int32_t *base, uint64_t row, uint32_t C, uint32_t c4, const int4 &v)
{
    GAS int32_t *p = base + row * C + 4 * c4;
    if (VEC) {
        gstore4i(p, v);
        return;
    }
    const uint32_t c = 4 * c4;
    if (c + 0 < C) p[0] = v.x;
    if (c + 1 < C) p[1] = v.y;
    if (c + 2 < C) p[2] = v.z;
    if (c + 3 < C) p[3] = v.w;
}

// q = sgn(y) floor(|y|/step + tau) with the exact decision of `quantize` (gsc_device.h);
// POW2: every step is a power of two, so the quotient is an exact float multiply and the decision
// a float comparison with thr = ceil_float(1 - tau).
template <bool POW2>
__device__ inline int32_t quant1(float y, float step, float inv_step, double omt, float thr)
{
    return POW2 ? quantize_pow2(y, inv_step, thr) : quantize(y, step, inv_step, omt, false);
}

constexpr int UNROLL = 8;  // independent row loads in flight per thread

// The channels of a tile are transformed in slices taken by different workgroups (see
// slice_split): on the upper levels slices of at most CH4_MAX float4 chunks (28 channels,
// 56 KB of LDS: two slices at 56 channels, measured slightly faster there than four of 16 or
// eight of 8), on the first level at most CH4_MAX1 (measured faster there: fewer, wider row
// pieces per gathered row).
constexpr uint32_t CH4_MAX = 7;
constexpr uint32_t CH4_MAX1 = 8;  // the first level: two slices of up to 32 channels (112-byte row pieces)
static_assert((RT - 1) * CH4_MAX1 < 65536u, "packed LDS rows of a merge record (lds_rec)");
__host__ __device__ inline uint32_t channel_passes(uint32_t C4, int k)
{
    const uint32_t cm = k == 1 ? CH4_MAX1 : CH4_MAX;
    return (C4 + cm - 1) / cm;
}
__host__ __device__ inline uint32_t pass_chunks(uint32_t C4, int k)
{
    const uint32_t np = channel_passes(C4, k);
    return (C4 + np - 1) / np;
}

// Loads rows j = row0, row0 + RPB, ... (< mlen) of one channel chunk into the LDS slice. The
// UNROLL loads of a batch are issued back to back: a row past the end re-reads the last valid
// row and is discarded.
template <class RowLoad>
__device__ inline void load_slice(float4 *s_y, const Roles &R, uint32_t CH4, uint32_t mlen,
                                  RowLoad rowload)
{
    for (uint32_t jb = R.row0; jb < mlen; jb += UNROLL * R.RPB) {
        float4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint32_t j = min(jb + u * R.RPB, mlen - 1);
            v[u] = rowload(j);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint32_t j = jb + u * R.RPB;
            if (j < mlen) s_y[j * CH4 + R.c4] = v[u];
        }
    }
}

// The channel slices of a tile are taken by different workgroups, one slice each: a workgroup
// makes one pass with the LDS of one slice. The NP workgroups of tile t are the blocks b,
// b + 8, ..., b + 8 (NP - 1) of a group of 8 NP blocks, which land on the same XCD (workgroups
// go to the 8 XCDs round-robin) one after the other, so the row reads of the later slices find
// the rows' cache lines in that XCD's L2.
struct SliceSplit {
    uint32_t tile, p0, p1;
};
__device__ inline SliceSplit slice_split(uint32_t local, uint32_t NP)
{
    SliceSplit h;
    const uint32_t g = local / (8 * NP), w = local % (8 * NP);
    h.tile = g * 8 + (w % 8);
    h.p0 = w / 8;
    h.p1 = h.p0 + 1;
    return h;
}
uint32_t raht_blocks(uint32_t tiles, int k, int C4)
{
    return (tiles + 7) / 8 * 8 * channel_passes((uint32_t)C4, k);
}
uint32_t channel_slices_upper(int C4) { return channel_passes((uint32_t)C4, 2); }

// ================================================= hand-over between tiling levels
// Every tiling level of a direction runs in one persistent launch, so the open entries' rows
// pass from one level to the next between workgroups of the same launch, possibly on different
// XCDs. They are written and read with device-coherent 64-bit accesses, which bypass the XCDs'
// non-coherent L2 caches, so neither side needs a cache write-back or invalidation. A producer
// waits until its stores have completed before it adds its items to its level's completion
// counter; a consumer reads the rows only after it has seen the count it needs.
__device__ inline void st_coh4(GAS float *p, const float4 &v)
{
    GAS uint64_t *q = reinterpret_cast<GAS uint64_t *>(p);
    __hip_atomic_store(q, ((uint64_t)__float_as_uint(v.y) << 32) | __float_as_uint(v.x), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, ((uint64_t)__float_as_uint(v.w) << 32) | __float_as_uint(v.z), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float4 ld_coh4(const GAS float *p)
{
    const GAS uint64_t *q = reinterpret_cast<const GAS uint64_t *>(p);
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float4(__uint_as_float((uint32_t)a), __uint_as_float((uint32_t)(a >> 32)),
                       __uint_as_float((uint32_t)b), __uint_as_float((uint32_t)(b >> 32)));
}

// Counter word w of a transform launch (DONE_FWD + k, TK_UPF, ...), in the workspace of the
// launch's first frame; the completion counters count a level's finished items over all frames.
__device__ inline GAS uint32_t *ctr_word(const TileMap &m, uint32_t w)
{
    return gp(cp(m.fd[0])->lvl_flags) + UP_GRID_MAX + w;
}
__device__ inline GAS uint32_t *done_ctr(const TileMap &m, uint32_t base, int k)
{
    return ctr_word(m, base + (uint32_t)k);
}
// Adds v items once every store of the workgroup has completed (each wave waits for its own
// stores before the barrier).
__device__ inline void done_add(GAS uint32_t *c, uint32_t v)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && v) __hip_atomic_fetch_add(c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool done_reached(const GAS uint32_t *c, uint32_t target)
{
    return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
}
// Waits (thread 0, then a barrier) until a level's counter reaches `target`. Every item a wait
// depends on comes earlier in the launch's order, each workgroup takes its items in order and
// all workgroups are resident, so the earliest unfinished item can always proceed; a spin limit
// turns a stall into GSC_ERR_INTERNAL.
__device__ inline void done_wait(const GAS uint32_t *c, uint32_t target, Ctrl *ctrl)
{
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        while (!done_reached(c, target)) {
            if (++spins > SPIN_LIMIT) {
                set_error(ctrl, GSC_ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

// The last workgroup of a transform launch to end (counted on counter word w) ends every frame's
// call (finish_frame, one wave per frame), so that a call whose last launch this is needs no
// finish launch. Each wave has waited for its memory operations (device errors are reported by
// atomics) before the workgroup is counted; what finish_frame reads was written by earlier
// launches, or is read with coherent loads (errors, level sizes), so no cache-wide acquire is
// needed. The transform's LDS (s_y) is free by then and holds the scratch.
__device__ inline void finish_if_last(const TileMap &m, uint32_t w, float4 *s_y)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    uint32_t *s_last = reinterpret_cast<uint32_t *>(s_y);
    if (threadIdx.x == 0)
        s_last[0] = __hip_atomic_fetch_add(ctr_word(m, w), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == gridDim.x;
    __syncthreads();
    if (!s_last[0]) return;
    FinishScratch *S = reinterpret_cast<FinishScratch *>(s_y + 1);
    const uint32_t wv = threadIdx.x / WAVE;
    for (uint32_t f = wv; f < m.F; f += RAHT_THREADS / WAVE) finish_frame(*cp(m.fd[f]), lane_id(), S[wv]);
}

// ------------------------------------------------------------ the upper items of a launch
// Items of upper level k (k >= 2) of frame f: the tiles of S_k times the channel slices NP. The
// sizes of levels k >= 3 are written by the schedule workgroups of the same launch, so they are
// read with device-coherent loads (never through the scalar cache), after those workgroups are done.
__device__ inline uint32_t up_frame_items(const TileMap &m, uint32_t f, int k, uint32_t NP)
{
    const CAS FrameDesc &fd = *cp(m.fd[f]);
    if ((uint32_t)k > fd.K) return 0u;
    const uint32_t nk = k >= 3 ? __hip_atomic_load(&fd.ctrl->lvl_n[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : cp(fd.ctrl)->lvl_n[k];
    return (nk >= 2 && nk <= fd.lv[k].cap) ? (nk + RT - 1) / RT * NP : 0u;
}
static_assert(GSC_MAX_BATCH <= WAVE, "one wave counts the frames' items");

// s_ucnt[k] = items of level k over the launch's frames (k = 2..kmax; s_ucnt[kmax + 1] = 0),
// counted by wave 0. Returns their sum (after a barrier). The sizes of UP_BATCH levels are
// loaded before any is used (one round trip for every level of a usual frame).
constexpr int UP_BATCH = 8;
__device__ inline uint32_t up_totals(const TileMap &m, int kmax, uint32_t NP, uint32_t *s_ucnt)
{
    if (threadIdx.x < WAVE) {
        const uint32_t lane = lane_id();
        for (int k0 = 2; k0 <= kmax; k0 += UP_BATCH) {
            uint32_t c[UP_BATCH];
#pragma unroll
            for (int q = 0; q < UP_BATCH; ++q)
                c[q] = (k0 + q <= kmax && lane < m.F) ? up_frame_items(m, lane, k0 + q, NP) : 0u;
#pragma unroll
            for (int q = 0; q < UP_BATCH; ++q) {
                if (k0 + q > kmax) break;
                const uint32_t inc = wave_incl_scan(c[q]);
                if (lane == WAVE - 1) s_ucnt[k0 + q] = inc;
            }
        }
        if (lane == 0) s_ucnt[kmax + 1 > 1 ? kmax + 1 : 1] = 0;
    }
    __syncthreads();
    uint32_t u = 0;
    for (int k = 2; k <= kmax; ++k) u += s_ucnt[k];
    return u;
}

struct UpItem {
    int k;
    uint32_t f, tile, p;
};
// Upper item g (counted over the launch's upper items) in processing order: the levels
// ascending (forward) or descending (inverse), each level frame by frame, the channel slices
// of a tile adjacent. Every wave computes the same (uniform) result.
__device__ inline UpItem up_item(const TileMap &m, int kmax, bool desc, uint32_t NP, const uint32_t *s_ucnt, uint32_t g)
{
    UpItem u;
    u.k = 0;
    u.f = u.tile = u.p = 0;
    for (int o = 0; 2 + o <= kmax; ++o) {
        const int k = desc ? kmax - o : 2 + o;
        const uint32_t c = s_ucnt[k];
        if (g < c && m.F == 1) {  // one frame: its items are the level's
            u.k = k;
            u.tile = g / NP;
            u.p = g % NP;
            return u;
        }
        if (g < c) {
            const uint32_t lane = lane_id();
            const uint32_t cf = lane < m.F ? up_frame_items(m, lane, k, NP) : 0u;
            const uint32_t inc = wave_incl_scan(cf);
            const uint64_t b = __ballot(inc > g);
            const uint32_t f = __builtin_amdgcn_readfirstlane((uint32_t)(__ffsll((long long)b) - 1));
            const uint32_t before = __builtin_amdgcn_readfirstlane((uint32_t)__shfl(inc - cf, (int)f, WAVE));
            const uint32_t local = g - before;
            u.k = k;
            u.f = f;
            u.tile = local / NP;
            u.p = local % NP;
            return u;
        }
        g -= c;
    }
    return u;
}

// ------------------------------------------------------------------ open-entry sets
// The open entries of a tile as a bit set over its RT positions (om[w] bit b: position 64 w + b)
// and the number of open entries before each word (pre[w]); the open entry whose range holds
// position j (the nearest open entry at or before j; a tile's first entry is always open) has
// index pre[w] + popcount(om[w] & bits 0..b) - 1.
struct OpenSet {
    unsigned long long *om;  // NCHUNK words
    uint32_t *pre;           // NCHUNK + 1 words
};
__device__ inline bool os_open(const OpenSet &s, uint32_t j) { return (s.om[j >> 6] >> (j & 63)) & 1ull; }
__device__ inline uint32_t os_cover(const OpenSet &s, uint32_t j)
{
    const uint32_t w = j >> 6;
    const unsigned long long upto = (2ull << (j & 63)) - 1ull;  // bits 0 .. j % 64
    return s.pre[w] + (uint32_t)__popcll(s.om[w] & upto) - 1u;
}
// Sets the bits of open positions p (one per calling thread with `on`); om must be zero.
__device__ inline void os_set(const OpenSet &s, uint32_t p, bool on)
{
    if (on) atomicOr(&s.om[p >> 6], 1ull << (p & 63));
}
// pre from om (wave 0, after the bits are set and a barrier; visible after the next barrier).
__device__ inline void os_prefix(const OpenSet &s)
{
    if (threadIdx.x < WAVE) {
        const uint32_t lane = lane_id();
        const uint32_t c = lane < (uint32_t)NCHUNK ? (uint32_t)__popcll(s.om[lane]) : 0u;
        const uint32_t inc = wave_incl_scan(c);
        if (lane <= (uint32_t)NCHUNK) s.pre[lane] = inc - c;
    }
}

// The inverse of a tile runs with the low-pass of every open entry taken as zero; the part of
// the result that the low-passes carry is added afterwards. With only the low-pass L_o of open
// entry o nonzero, every inverse butterfly hands each of its two parts sqrt(w_part / w_node) of
// its node's value (Eq. 1 with a zero high-pass), so entry j of o's range (o up to the next
// open entry) receives L_o sqrt(w_j / W_o), w_j being the entry's weight (leaves under it) and
// W_o the range's. s_L holds the low-passes of opens ob .. ob + nb - 1 (this slice's chunks);
// weight(a, b) is the number of leaves under entries a .. b - 1.
constexpr uint32_t LCAP = 32;  // open entries whose low-passes are staged in LDS at a time
template <class WeightFn>
__device__ inline void add_open_share(float4 *s_y, const Roles &R, uint32_t CH4, bool live, uint32_t mlen,
                                      const OpenSet &os, const uint16_t *s_opos, uint32_t ocnt,
                                      const float4 *s_L, uint32_t ob, uint32_t nb, bool fp64, WeightFn weight)
{
    if (!live) return;
    for (uint32_t j = R.row0; j < mlen; j += R.RPB) {
        const uint32_t o = os_cover(os, j);
        if (o < ob || o >= ob + nb) continue;
        const uint32_t p0 = s_opos[o], p1 = o + 1 < ocnt ? s_opos[o + 1] : mlen;
        const uint32_t wj = weight(j, j + 1), wo = weight(p0, p1);
        const float fac = fp64 ? (float)sqrt((double)wj / (double)wo) : sqrtf((float)wj / (float)wo);
        const float4 L = s_L[(o - ob) * CH4 + R.c4];
        float4 &y = s_y[j * CH4 + R.c4];
        y.x += fac * L.x;
        y.y += fac * L.y;
        y.z += fac * L.z;
        y.w += fac * L.w;
    }
}

// LDS arrays of an upper-level item (aliases of the first level's arrays).
struct UpArrays {
    uint32_t *rec;
    float2 *ab;
    uint16_t *lst;
    uint16_t *opos;
    uint32_t *idx;
    unsigned long long *lmask;
    OpenSet os;
    float4 *L;  // (inverse)
};

// The schedule of an item (tile of S_k, k >= 2) into LDS; false if there is nothing to do.
__device__ inline bool up_schedule(const TileMap &m, uint32_t f, int k, uint32_t tile, TileSched &ts, const UpArrays &A)
{
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    if (load_error(ctrl)) return false;
    if ((uint32_t)k > fd.K) return false;
    return load_schedule(fd, ctrl, k, tile, pass_chunks(fd.C4, k), ts, A.rec, A.ab, A.lst, A.opos, A.idx, A.lmask);
}

// The quantized (or float) coefficient rows at their voxel rows, of the entries j that `skip`
// lets through. Open entries are skipped by every caller: an open entry's coefficient is written
// by the level that completes its merge (so that every row is written exactly once in the
// launch), except at the final level, where the open entry is the sequence's first one and holds
// the DC.
template <bool VEC, bool POW2, class RowOf, class YAt, class Skip>
__device__ inline void store_coefs(const CAS FrameDesc &fd, const float *s_st, const float *s_ist, const Roles &R,
                                   uint32_t c4, uint32_t mlen, Skip skip, RowOf row_of, YAt y_at)
{
    const uint32_t C = fd.C;
    GAS float *cf = gp(fd.coef_f32);
    if (fd.mode == MODE_ENCODE) {
        const CAS Ctrl *ctrl = cp(fd.ctrl);
        uint64_t off = GSC_HEADER_BYTES, run = 0;
        for (uint32_t dd = 0; dd < fd.J; ++dd) {
            run += ctrl->hist_D[dd];
            off += run;
        }
        GAS int32_t *coef = gp(reinterpret_cast<int32_t *>(fd.stream + align_up(off, 256)));
        const double omt = 1.0 - (double)fd.tau;
        const float thr = ceil_float(omt);
        const bool deq = fd.ste == STE_FORWARD;  // float output: q * step instead of y
        float st[4], ist[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = min(4 * c4 + q, C - 1);
            st[q] = s_st[c];
            ist[q] = s_ist[c];
        }
        for (uint32_t j = R.row0; j < mlen; j += R.RPB) {
            if (skip(j)) continue;
            const float4 y = y_at(j);
            const uint64_t row = row_of(j);
            const int4 q = make_int4(quant1<POW2>(y.x, st[0], ist[0], omt, thr), quant1<POW2>(y.y, st[1], ist[1], omt, thr),
                                     quant1<POW2>(y.z, st[2], ist[2], omt, thr), quant1<POW2>(y.w, st[3], ist[3], omt, thr));
            stq4<VEC>(coef, row, C, c4, q);
            if (cf)
                st4<VEC>(cf, row, C, c4,
                         deq ? make_float4((float)q.x * st[0], (float)q.y * st[1], (float)q.z * st[2], (float)q.w * st[3])
                             : y);
        }
    } else {  // MODE_FWD_F32: float coefficient rows
        for (uint32_t j = R.row0; j < mlen; j += R.RPB) {
            if (skip(j)) continue;
            st4<VEC>(cf, row_of(j), C, c4, y_at(j));
        }
    }
}

// ============================================================== upper levels, forward
// One item (tile, channel slice p0) of S_k, k >= 2, whose schedule is in LDS: the entries'
// partial low-passes come from the rows S_{k-1}'s open entries handed over, each entry's
// coefficient row goes to its voxel's row, the open entries' partial low-passes to S_{k+1}.
template <bool VEC, bool POW2>
__device__ inline void fwd_up_item(const TileMap &m, uint32_t f, int k, uint32_t p0, const TileSched &ts,
                                   float4 *s_y, const UpArrays &A, const float *s_st, const float *s_ist)
{
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    const uint32_t C4 = fd.C4;
    const uint32_t CH4 = pass_chunks(C4, k);
    const Roles R(CH4);
    const uint32_t mlen = (uint32_t)ts.mlen;
    const uint32_t cb = p0 * CH4, nch = min(CH4, C4 - cb);
    const uint32_t c4 = cb + R.c4;  // this thread's global channel chunk
    const bool live = R.act && R.c4 < nch;
    os_set(A.os, A.opos[min(threadIdx.x, (uint32_t)OPEN_CAP - 1)], threadIdx.x < ts.ocnt);
    // ---- the entries' values of this channel slice
    if (live) {
        const GAS float *vsrc = gp(fd.lv[k - 1].vbuf);
        load_slice(s_y, R, CH4, mlen, [&](uint32_t j) { return ld_coh4(vsrc + ((size_t)(ts.s + j) * C4 + c4) * 4); });
    }
    __syncthreads();
    // ---- all local merges: within wave chunks, then across chunks (levels ascending)
    const uint64_t wmask = A.lmask[R.w], xmask = A.lmask[CROSS];
    wave_phase(s_y, R, A.rec, A.ab, A.lst, wmask, nch, false, R.w);
    __syncthreads();
    cross_phase(s_y, R, A.rec, A.ab, A.lst, xmask, nch, false);
    if (!live) return;
    store_coefs<VEC, POW2>(fd, s_st, s_ist, R, c4, mlen,
                           [&](uint32_t j) { return !ts.final_level && os_open(A.os, j); },
                           [&](uint32_t j) -> uint64_t { return A.idx[j]; },
                           [&](uint32_t j) { return s_y[j * CH4 + R.c4]; });
    if (!ts.final_level) {
        GAS float *dst = gp(fd.lv[k].vbuf);
        for (uint32_t o = R.row0; o < ts.ocnt; o += R.RPB)
            st_coh4(dst + ((size_t)(ts.obase + o) * C4 + c4) * 4, s_y[A.opos[o] * CH4 + R.c4]);
    }
}

// ============================================================== upper levels, inverse
// One item of S_k, k >= 2: coefficient rows from the entries' voxels; the tile is inverted with
// its open entries' low-passes taken as zero, then the low-passes S_{k+1} handed down (once all
// of S_{k+1}'s items are done) add their shares; the entries' synthesized values go to S_{k-1}'s
// open-entry rows.
template <bool VEC>
__device__ inline void inv_up_item(const TileMap &m, uint32_t f, int k, uint32_t p0, const TileSched &ts,
                                   float4 *s_y, const UpArrays &A, const GAS uint32_t *above_done, uint32_t above_items)
{
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    const uint32_t C = fd.C, C4 = fd.C4;
    const uint32_t CH4 = pass_chunks(C4, k);
    const Roles R(CH4);
    const uint32_t mlen = (uint32_t)ts.mlen;
    const uint32_t cb = p0 * CH4, nch = min(CH4, C4 - cb);
    const uint32_t c4 = cb + R.c4;
    const bool live = R.act && R.c4 < nch;
    const bool opens = !ts.final_level && ts.ocnt > 0;
    os_set(A.os, A.opos[min(threadIdx.x, (uint32_t)OPEN_CAP - 1)], opens && threadIdx.x < ts.ocnt);
    // ---- coefficients of every entry (the high-pass stored at it)
    if (live) {
        if (fd.mode == MODE_DECODE) {
            const gsc_header *h = reinterpret_cast<const gsc_header *>(fd.in_stream);
            const GAS int32_t *coef = gp(reinterpret_cast<const int32_t *>(fd.in_stream + h->coef_offset));
            float st[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) st[i] = 4 * c4 + i < C ? h->quant_step[4 * c4 + i] : 0.0f;
            load_slice(s_y, R, CH4, mlen, [&](uint32_t j) {
                const int4 q = ldq4<VEC>(coef, A.idx[j], C, c4);
                return make_float4((float)q.x * st[0], (float)q.y * st[1], (float)q.z * st[2], (float)q.w * st[3]);
            });
        } else {  // float coefficient rows: the straight-through forward synthesizes from its
                  // dequantized coefficients; the transform and gradient modes read the caller's
            const GAS float *fin = gp(fd.mode == MODE_ENCODE ? fd.coef_f32 : fd.attr);
            load_slice(s_y, R, CH4, mlen, [&](uint32_t j) { return ld4<VEC>(fin, A.idx[j], C, c4); });
        }
    }
    __syncthreads();
    // ---- open entries start from a zero low-pass
    if (opens) {
        os_prefix(A.os);
        if (live)
            for (uint32_t o = R.row0; o < ts.ocnt; o += R.RPB) s_y[A.opos[o] * CH4 + R.c4] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
    }
    // ---- all local merges undone: across chunks, then within chunks (levels descending)
    const uint64_t wmask = A.lmask[R.w], xmask = A.lmask[CROSS];
    cross_phase(s_y, R, A.rec, A.ab, A.lst, xmask, nch, true);
    wave_phase(s_y, R, A.rec, A.ab, A.lst, wmask, nch, true, R.w);
    __syncthreads();
    // ---- the open entries' low-passes, handed down by S_{k+1}
    if (opens) {
        done_wait(above_done, above_items, fd.ctrl);
        const GAS float *src = gp(fd.lv[k].vbuf);
        const bool fp64 = fp64_weights(fd);
        for (uint32_t ob = 0; ob < ts.ocnt; ob += LCAP) {
            const uint32_t nb = min(LCAP, ts.ocnt - ob);
            for (uint32_t q = threadIdx.x; q < nb * nch; q += RAHT_THREADS) {
                const uint32_t o = q / nch, c = q - o * nch;
                A.L[o * CH4 + c] = ld_coh4(src + ((size_t)(ts.obase + ob + o) * C4 + cb + c) * 4);
            }
            __syncthreads();
            add_open_share(s_y, R, CH4, live, mlen, A.os, A.opos, ts.ocnt, A.L, ob, nb, fp64,
                           [&](uint32_t a, uint32_t b) { return A.idx[b] - A.idx[a]; });
            __syncthreads();
        }
    }
    if (!live) return;
    GAS float *dst = gp(fd.lv[k - 1].vbuf);
    for (uint32_t j = R.row0; j < mlen; j += R.RPB) st_coh4(dst + ((size_t)(ts.s + j) * C4 + c4) * 4, s_y[j * CH4 + R.c4]);
}

// ============================================================ first level, persistent forward
// The first level carries almost all of the transform's bytes (every voxel row in, every
// coefficient row out), and a workgroup that waits first for its schedule and then for its rows
// leaves the memory system idle for much of its life. Here the workgroups are persistent:
// workgroup b takes the items (tile, channel slice) b, b + G, b + 2G, ... of the launch
// (G = gridDim.x, a multiple of 8 NP, so an item and its partner slice run at the same time on
// one XCD), and while the merges and stores of one item run, the schedule and the row loads of
// the next item are in flight in registers. The input row of every voxel's first member comes
// from the dedup kernel's table and is read two items ahead, so the next item's row addresses
// are known when its loads are issued.
// rows of a slice per thread: ceil(RT / floor(RT / CH4)), at most this for CH4 <= CH4_MAX1
__host__ __device__ constexpr int rows_per_thread_max(int ch4max)
{
    int r = 0;
    for (int c = 1; c <= ch4max; ++c) {
        const int rpb = RT / c, t = (RT + rpb - 1) / rpb;
        r = t > r ? t : r;
    }
    return r;
}
constexpr int NR1 = rows_per_thread_max((int)CH4_MAX1);
// persistent first-level workgroups per CU (as many as the LDS of a slice and the registers allow)
constexpr int PERSIST_PER_CU = 2;

struct Item1 {
    uint32_t f, tile, p, s, mlen;
    bool ok, final_level;
};

typedef const CAS FrameDesc CFrame;

// Values shared by the items of one frame, loaded when the first item of the frame is described.
struct Frame1 {
    uint32_t f;   // frame, ~0u before the first
    uint32_t nk;  // entries of S_1; 0 when the frame has nothing to transform
};

__device__ inline Item1 item1(const TileMap &m, uint32_t i, Frame1 &fc)
{
    Item1 it;  // an item that is not ok still names frame 0, so that its fields index safely
    it.f = it.tile = it.p = it.s = 0;
    it.mlen = 1;
    it.ok = it.final_level = false;
    if (i >= m.start[m.F]) return it;
    const uint32_t f = frame_of(m, i);
    CFrame *d = cp(m.fd[f]);
    if (f != fc.f) {
        // the frame's values are the same in every lane; readfirstlane says so to the compiler
        // (an atomic load's result counts as divergent), so that everything derived from them,
        // down to the descriptor pointer, stays in scalar registers
        fc.f = f;
        uint32_t nk = 0;
        if (!__builtin_amdgcn_readfirstlane(load_error(m.fd[f]->ctrl))) {
            nk = seq_size(*m.fd[f], m.fd[f]->ctrl, 1);
            if (!seq_active(nk, 1)) nk = 0;
        }
        fc.nk = __builtin_amdgcn_readfirstlane(nk);
    }
    const SliceSplit hs = slice_split(i - m.start[f], channel_passes(d->C4, 1));
    it.f = f;
    it.tile = hs.tile;
    it.p = hs.p0;
    it.s = hs.tile * RT;
    if (it.s >= fc.nk) return it;
    it.mlen = min(fc.nk, it.s + RT) - it.s;
    it.final_level = fc.nk <= (uint32_t)RT;
    it.ok = true;
    return it;
}

// One item's schedule in registers: thread t holds merge record t, word t of the segment starts
// and of the open positions (two u16 entries each) and run start t (thread 0 also the run start
// after a full tile). Everything is loaded as 32-bit words: a narrower load's value would be
// widened where the prefetch branch joins, which waits for it. Entries past the tile's counts
// are never read from LDS.
struct Sched1 {
    uint32_t rec, lst, opos, m0;
    uint64_t lm;                         // thread c < NCLS: level mask of class c
    uint32_t m_beg, m_end, obase, ocnt;  // the same in every lane (scalar loads)
};
static_assert(LSTART_N % 2 == 0 && OPEN_CAP % 2 == 0 && LSTART_N / 2 <= RT, "u16 pairs per thread");

__device__ inline void load_sched1(CFrame *d, const Item1 &it, Sched1 &S)
{
    const uint32_t tid = threadIdx.x;
    const size_t t = it.tile;
    S.rec = gp(d->lv[1].rec)[t * RT + tid];
    const GAS uint32_t *lw = reinterpret_cast<const GAS uint32_t *>(gp(d->lv[1].lstart) + t * LSTART_N);
    const GAS uint32_t *ow = reinterpret_cast<const GAS uint32_t *>(gp(d->lv[1].opos) + t * OPEN_CAP);
    S.lst = lw[min(tid, (uint32_t)LSTART_N / 2 - 1)];
    S.opos = ow[min(tid, (uint32_t)OPEN_CAP / 2 - 1)];
    // written by the prelude (and run starts by the dedup kernel), constant here: scalar loads
    S.obase = cp(d->lv[1].obase)[t];
    S.ocnt = cp(d->lv[1].ocnt)[t];
    S.lm = gp(d->lv[1].lmask)[t * NCLS + min(tid, (uint32_t)NCLS - 1)];
    // run starts (used by the encoder; the table exists in every workspace)
    S.m0 = gp(d->vh)[it.s + min(tid, it.mlen)];
    S.m_beg = cp(d->vh)[it.s];
    S.m_end = cp(d->vh)[it.s + it.mlen];
}

// Branch-free, so that every prefetched register is consumed here on every path (the compiler's
// wait analysis would otherwise leave them pending and wait for them, and for every later load,
// at their next write): threads without an entry to write store into the sink slot past the end
// of each array.
__device__ inline void commit_sched1(const Sched1 &S, const Item1 &it, uint32_t CH4, uint32_t n,
                                     bool fp64, uint32_t *s_rec, float2 *s_ab, uint32_t *s_lstw,
                                     uint32_t *s_oposw, uint32_t *s_m0, unsigned long long *s_lmask)
{
    const uint32_t tid = threadIdx.x;
    s_lmask[min(tid, (uint32_t)NCLS)] = S.lm;
    s_rec[tid] = lds_rec(S.rec, CH4);
    // (a, b) of the merge: at the first level an entry's weight is its position difference
    const uint32_t j = S.rec & 1023u, l = (S.rec >> 10) & 1023u, r = S.rec >> 20;
    s_ab[tid] = rotation(j - l, r - j, fp64);
    s_lstw[min(tid, (uint32_t)LSTART_N / 2)] = S.lst;
    s_oposw[min(tid, (uint32_t)OPEN_CAP / 2)] = S.opos;
    s_m0[tid <= it.mlen ? tid : RT + 1] = min(S.m0, n);
    if (tid == 0) s_m0[it.mlen] = min(S.m_end, n);
}

// Issues the loads of this thread's rows of an item's channel slice: chunk c4 of rows
// j = row0 + u RPB, row j of the input matrix being s_row[j] (gather) or s + j. Branch-free: a
// row past the end re-reads the tile's last row and is discarded at commit.
template <bool VEC>
__device__ inline void load_rows1(const GAS float *src, uint32_t C, const Roles &R, uint32_t c4,
                                  uint32_t mlen, bool gather, const uint32_t *s_row, uint32_t s,
                                  float4 (&D)[NR1])
{
    uint32_t row[NR1];
#pragma unroll
    for (int u = 0; u < NR1; ++u) {
        const uint32_t j = min(R.row0 + (uint32_t)u * R.RPB, mlen - 1);
        row[u] = gather ? s_row[j] : s + j;
    }
#pragma unroll
    for (int u = 0; u < NR1; ++u) D[u] = ld4<VEC>(src, row[u], C, c4);
}



// The forward transform of every tiling level in one launch. The first Gp workgroups first build
// the upper levels' schedules (up_prelude_group; Gp = the second level's tiles, at most the grid),
// which the upper levels need only at the end. Then every workgroup takes its first-level items
// (persistent and prefetching, as described above). A workgroup out of first-level items adds
// them to level 1's completion counter and takes the upper levels' items (ascending) from a
// counter; an item of level k >= 2 waits until level k - 1 is complete (all its open-entry rows
// handed over) and runs the tile as one (non-prefetching) item.
template <bool VEC, bool POW2>
__global__ __launch_bounds__(RAHT_THREADS) __attribute__((amdgpu_waves_per_eu(PERSIST_PER_CU * RAHT_THREADS / WAVE / 4))) void k_raht_fwd(TileMap m, int kmax, int finish)
{
    extern __shared__ float4 s_y[];
    __shared__ uint32_t s_rec[RT];
    __shared__ float2 s_ab[RT];
    __shared__ uint32_t s_lstw[LSTART_N / 2 + 1];   // u16 segment starts, in pairs; + sink
    __shared__ uint32_t s_oposw[OPEN_CAP / 2 + 1];  // u16 open positions, in pairs; + sink
    __shared__ uint32_t s_m0[RT + 2];               // run starts; + sink (upper items: voxel indices)
    __shared__ uint32_t s_row[RT];
    __shared__ float s_st[GSC_MAX_CHANNELS], s_ist[GSC_MAX_CHANNELS];
    __shared__ unsigned long long s_lmask[NCLS + 1];  // + sink
    __shared__ unsigned long long s_om[2][NCHUNK];    // open-entry sets of two consecutive items
    __shared__ uint32_t s_opre[NCHUNK + 1];
    __shared__ uint32_t s_ucnt[MAXK + 2];
    __shared__ uint32_t s_fs[GSC_MAX_BATCH + 1];
    __shared__ uint32_t s_tk[1];
    const uint16_t *s_lst = reinterpret_cast<const uint16_t *>(s_lstw);
    const uint16_t *s_opos = reinterpret_cast<const uint16_t *>(s_oposw);

    const uint32_t tid = threadIdx.x, items = m.start[m.F];
    // ---- the upper levels' schedules, by the first Gp workgroups
    uint32_t Gp = 0;
    if (kmax >= 2) {
        Gp = min(level_items(m, 2, 1, s_fs), gridDim.x);
        if (blockIdx.x < Gp) up_prelude_group(m, kmax, Gp, s_fs, ctr_word(m, PRE_DONE));
    }
    Frame1 fc;
    fc.f = ~0u;
    fc.nk = 0;
    // the first row of entry tid of an item (clamped where it is stored into s_row, so that
    // nothing waits for the load before then)
    auto first_row = [&](const Item1 &it) -> uint32_t {
        return gp(cp(m.fd[it.f])->first)[it.s + min(tid, it.mlen - 1)];
    };
    // row indices read from the workspace are clamped: never an access outside the input
    auto row_clamp = [&](const Item1 &it, uint32_t r) -> uint32_t {
        const uint32_t n = cp(m.fd[it.f])->n;
        return min(r, n ? n - 1 : 0u);
    };
    // the channel slice of an item: CH4 chunks per slice, nch of them in this one
    auto slice = [&](const Item1 &it, uint32_t &CH4, uint32_t &nch) {
        const uint32_t C4 = cp(m.fd[it.f])->C4;
        CH4 = pass_chunks(C4, 1);
        nch = min(CH4, C4 - it.p * CH4);
    };
    auto prefetch = [&](const Item1 &it, Sched1 &S, float4 (&D)[NR1]) {
        CFrame *d = cp(m.fd[it.f]);
        const bool enc = d->mode == MODE_ENCODE;
        uint32_t CH4, nch;
        slice(it, CH4, nch);
        const Roles R(CH4);
        load_sched1(d, it, S);
        if (R.act && R.c4 < nch)
            load_rows1<VEC>(gp(d->attr), d->C, R, it.p * CH4 + R.c4, it.mlen, enc, s_row, it.s, D);
    };
    // first-level item i goes to workgroup (Gp + i) % G: the schedule workgroups come last in the
    // round-robin, so they take one item fewer when the items do not fill the last round
    const uint32_t G = gridDim.x;
    const uint32_t b1 = blockIdx.x >= Gp ? blockIdx.x - Gp : blockIdx.x + G - Gp;  // first item
    Item1 it0 = item1(m, b1, fc);
    Item1 it1 = item1(m, b1 + G, fc);
    Sched1 S;
    float4 D[NR1];
    uint32_t F1 = 0;
    // prologue: the quantizer steps (shared by the frames of a launch) into LDS, the open-entry
    // sets cleared, the first item's rows, schedule and row loads
    if (tid < GSC_MAX_CHANNELS) {
        s_st[tid] = cp(m.fd[0])->step[tid];
        s_ist[tid] = cp(m.fd[0])->inv_step[tid];
    }
    if (tid < 2 * NCHUNK) (&s_om[0][0])[tid] = 0;
    if (it0.ok && cp(m.fd[it0.f])->mode == MODE_ENCODE) s_row[tid] = row_clamp(it0, first_row(it0));
    if (it1.ok && cp(m.fd[it1.f])->mode == MODE_ENCODE) F1 = first_row(it1);
    __syncthreads();
    if (it0.ok) prefetch(it0, S, D);

    uint32_t par = 0, n1 = 0;  // which open-entry set the current item uses; items done
    for (uint32_t i = b1; i < items; i += G, ++n1, par ^= 1u) {
        CFrame *d = cp(m.fd[it0.f]);
        const bool encode = d->mode == MODE_ENCODE;
        uint32_t CH4, nch;
        slice(it0, CH4, nch);
        const Roles R(CH4);
        const uint32_t c4 = it0.p * CH4 + R.c4;  // this thread's global channel chunk
        const bool live = it0.ok && R.act && R.c4 < nch;
        const uint32_t C = d->C, n = d->n;
        const uint32_t obase = S.obase, ocnt = S.ocnt;
        const bool dup = S.m_end - S.m_beg != it0.mlen;  // a voxel of the tile has several Gaussians
        const OpenSet os{s_om[par], s_opre};
        __syncthreads();  // the previous item is no longer read from LDS
        // ---- the current item's schedule and rows into LDS, the next item's first rows; on
        // every path, whether or not the item is ok (see commit_sched1); the item's open
        // entries into its set (the other set is cleared for the next item)
        commit_sched1(S, it0, CH4, n, fp64_weights(*d), s_rec, s_ab, s_lstw, s_oposw, s_m0, s_lmask);
        if (tid < NCHUNK) s_om[par ^ 1u][tid] = 0;
        if (it0.ok && tid < (uint32_t)OPEN_CAP / 2) {
            os_set(os, S.opos & 0xFFFFu, 2 * tid < ocnt);
            os_set(os, S.opos >> 16, 2 * tid + 1 < ocnt);
        }
        const uint32_t sink = RT * CH4;
#pragma unroll
        for (int u = 0; u < NR1; ++u) {
            const uint32_t j = R.row0 + (uint32_t)u * R.RPB;
            s_y[live && j < it0.mlen ? j * CH4 + R.c4 : sink] = D[u];
        }
        s_row[tid] = row_clamp(it1, F1);
        __syncthreads();
        // ---- prefetch: the next item's schedule and rows (issued first), then the item after it
        // and its first rows
        if (it1.ok) prefetch(it1, S, D);
        const Item1 it2 = item1(m, i + 2 * G, fc);
        if (it2.ok && cp(m.fd[it2.f])->mode == MODE_ENCODE) F1 = first_row(it2);
        // ---- the current item
        if (it0.ok) {
            const uint32_t mlen = it0.mlen, s = it0.s;
            const uint32_t nlast = n ? n - 1 : 0u;
            // this thread's rows j = row0 + t RPB sit at LDS index y0 + t ystep
            const uint32_t y0 = R.row0 * CH4 + R.c4, ystep = R.RPB * CH4;
            if (encode && dup) {
                // merge duplicates: the mean of the rows of the Gaussians in the voxel
                // (Sec. 2.1), summed in input order (the sort is stable)
                const GAS float *attr = gp(d->attr);
                const GAS uint32_t *perm = gp((d->P & 1) ? d->vals_b : d->vals_a);
                for (uint32_t j = R.row0, yi = y0; live && j < mlen; j += R.RPB, yi += ystep) {
                    const uint32_t m0 = s_m0[j], m1 = s_m0[j + 1];
                    if (m1 - m0 <= 1) continue;
                    float4 acc = s_y[yi];
                    for (uint32_t mm = m0 + 1; mm < m1; ++mm) {
                        const float4 x = ld4<VEC>(attr, min(perm[mm], nlast), C, c4);
                        acc.x += x.x;
                        acc.y += x.y;
                        acc.z += x.z;
                        acc.w += x.w;
                    }
                    const float cnt = (float)(m1 - m0);
                    acc.x /= cnt;
                    acc.y /= cnt;
                    acc.z /= cnt;
                    acc.w /= cnt;
                    s_y[yi] = acc;
                }
                __syncthreads();  // the merged rows are read by other waves' merges
            }
            if (encode && d->ste == STE_FORWARD && d->aref) {
                // the voxel means (this thread's own rows of the slice), read before any merge
                // changes them
                if (live) {
                    GAS float *ar = gp(d->aref);
                    for (uint32_t j = R.row0, yi = y0; j < mlen; j += R.RPB, yi += ystep)
                        st4<VEC>(ar, s + j, C, c4, s_y[yi]);
                }
                __syncthreads();
            }
            const uint64_t wmask = s_lmask[R.w], xmask = s_lmask[CROSS];
            wave_phase(s_y, R, s_rec, s_ab, s_lst, wmask, nch, false, R.w);
            __syncthreads();
            cross_phase(s_y, R, s_rec, s_ab, s_lst, xmask, nch, false);
            if (live) {
                const bool fl = it0.final_level;
                store_coefs<VEC, POW2>(*d, s_st, s_ist, R, c4, mlen, [&](uint32_t j) { return !fl && os_open(os, j); },
                                       [&](uint32_t j) -> uint64_t { return s + j; },
                                       [&](uint32_t j) { return s_y[j * CH4 + R.c4]; });
                if (!it0.final_level) {
                    GAS float *dst = gp(d->lv[1].vbuf);
                    const uint32_t C4 = d->C4;
                    for (uint32_t o = R.row0; o < ocnt; o += R.RPB)
                        st_coh4(dst + ((size_t)(obase + o) * C4 + c4) * 4, s_y[s_opos[o] * CH4 + R.c4]);
                }
            }
        }
        it0 = it1;
        it1 = it2;
    }
    if (kmax >= 2) {
        // ---- the upper levels, ascending
        done_add(done_ctr(m, DONE_FWD, 1), n1);  // this workgroup's first-level open rows are written
        const uint32_t NP = channel_passes(cp(m.fd[0])->C4, 2);  // every frame of a launch has the same C
        if (tid < 2 * NCHUNK) (&s_om[0][0])[tid] = 0;
        Ctrl *ctrl0 = cp(m.fd[0])->ctrl;
        // the upper levels' schedules and sizes are written (by the first Gp workgroups)
        done_wait(ctr_word(m, PRE_DONE), Gp, ctrl0);
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const uint32_t U = up_totals(m, kmax, NP, s_ucnt);
        const UpArrays A{s_rec, s_ab, reinterpret_cast<uint16_t *>(s_lstw), reinterpret_cast<uint16_t *>(s_oposw),
                         s_m0, s_lmask, OpenSet{s_om[0], s_opre}, nullptr};
        GAS uint32_t *utk = ctr_word(m, TK_UPF);
        for (;;) {
            if (tid == 0) s_tk[0] = __hip_atomic_fetch_add(utk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();  // (also: the previous item's LDS is no longer read)
            const uint32_t g = __builtin_amdgcn_readfirstlane(s_tk[0]);
            if (g >= U) break;
            const UpItem u = up_item(m, kmax, false, NP, s_ucnt, g);
            TileSched ts;
            const bool ok = up_schedule(m, u.f, u.k, u.tile, ts, A);
            // the entries' rows are handed over by level k - 1: wait until all of its items are done
            done_wait(done_ctr(m, DONE_FWD, u.k - 1), u.k == 2 ? items : s_ucnt[u.k - 1], ctrl0);
            if (ok) fwd_up_item<VEC, POW2>(m, u.f, u.k, u.p, ts, s_y, A, s_st, s_ist);
            done_add(done_ctr(m, DONE_FWD, u.k), 1);
            if (tid < NCHUNK) s_om[0][tid] = 0;
        }
    }
    if (finish) finish_if_last(m, FIN_FWD, s_y);
}

// ============================================================ upper levels, inverse (launch)
// The inverse of the upper levels kmax .. 2 in one persistent launch (all workgroups resident),
// before the first level's: with `prelude`, the first Gp workgroups first build the upper
// levels' schedules. The items run in descending level order (workgroup b takes items b, b + G,
// ...); every item inverts its tile with the open entries' low-passes taken as zero and only
// then waits for the level above, so the tiles of all levels are inverted side by side and only
// the shares of the low-passes (add_open_share) follow the levels' order.
template <bool VEC>
__global__ __launch_bounds__(RAHT_THREADS) void k_raht_inv_up(TileMap m, int kmax, int prelude)
{
    extern __shared__ float4 s_y[];
    __shared__ uint32_t s_rec[RT];
    __shared__ float2 s_ab[RT];
    __shared__ uint16_t s_lst[LSTART_N];
    __shared__ uint16_t s_opos[OPEN_CAP];
    __shared__ uint32_t s_idx[RT + 1];
    __shared__ unsigned long long s_lmask[NCLS];
    __shared__ unsigned long long s_om[NCHUNK];
    __shared__ uint32_t s_opre[NCHUNK + 1];
    __shared__ float4 s_L[LCAP * CH4_MAX];
    __shared__ uint32_t s_ucnt[MAXK + 2];
    __shared__ uint32_t s_fs[GSC_MAX_BATCH + 1];
    const uint32_t tid = threadIdx.x, G = gridDim.x;
    Ctrl *ctrl0 = cp(m.fd[0])->ctrl;
    if (tid < NCHUNK) s_om[tid] = 0;
    if (prelude) {
        const uint32_t Gp = min(level_items(m, 2, 1, s_fs), G);
        if (blockIdx.x < Gp) up_prelude_group(m, kmax, Gp, s_fs, ctr_word(m, PRE_DONE));
        done_wait(ctr_word(m, PRE_DONE), Gp, ctrl0);
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
    }
    const uint32_t NP = channel_passes(cp(m.fd[0])->C4, 2);  // every frame of a launch has the same C
    const uint32_t U = up_totals(m, kmax, NP, s_ucnt);
    const UpArrays A{s_rec, s_ab, s_lst, s_opos, s_idx, s_lmask, OpenSet{s_om, s_opre}, s_L};
    for (uint32_t g = blockIdx.x; g < U; g += G) {
        const UpItem u = up_item(m, kmax, true, NP, s_ucnt, g);
        __syncthreads();  // the previous item's LDS is no longer read
        TileSched ts;
        const bool ok = up_schedule(m, u.f, u.k, u.tile, ts, A);
        if (ok) inv_up_item<VEC>(m, u.f, u.k, u.p, ts, s_y, A, done_ctr(m, DONE_INV, u.k + 1), s_ucnt[u.k + 1]);
        done_add(done_ctr(m, DONE_INV, u.k), 1);
        if (tid < NCHUNK) s_om[tid] = 0;
    }
}

// ============================================================ first level, persistent inverse
// The same persistent, prefetching scheme for the first level of the inverse (after the upper
// levels' launch): while one item's merges are undone and its rows stored, the next item's
// schedule, coefficient rows (read as raw 32-bit words, dequantized when they are committed to
// LDS) and the low-passes of its open entries (from S_2) are in flight in registers.
// open entries per thread: ceil(OPEN_CAP / RPB) for the narrowest rows per step
constexpr int NO1 = (OPEN_CAP + RT / (int)CH4_MAX1 - 1) / (RT / (int)CH4_MAX1);

template <bool VEC>
__global__ __launch_bounds__(RAHT_THREADS) __attribute__((amdgpu_waves_per_eu(PERSIST_PER_CU * RAHT_THREADS / WAVE / 4))) void k_raht_inv(TileMap m, int finish)
{
    extern __shared__ float4 s_y[];
    __shared__ uint32_t s_rec[RT];
    __shared__ float2 s_ab[RT];
    __shared__ uint32_t s_lstw[LSTART_N / 2 + 1];   // u16 segment starts, in pairs; + sink
    __shared__ uint32_t s_oposw[OPEN_CAP / 2 + 1];  // u16 open positions, in pairs; + sink
    __shared__ uint32_t s_m0[RT + 2];               // (written by the shared commit, unused)
    __shared__ float s_st[GSC_MAX_CHANNELS];        // dequantization steps of the frame s_stf
    __shared__ unsigned long long s_lmask[NCLS + 1];  // + sink
    const uint16_t *s_lst = reinterpret_cast<const uint16_t *>(s_lstw);
    const uint16_t *s_opos = reinterpret_cast<const uint16_t *>(s_oposw);

    const uint32_t tid = threadIdx.x, G = gridDim.x, items = m.start[m.F];
    Frame1 fc;
    fc.f = ~0u;
    fc.nk = 0;
    auto slice = [&](const Item1 &it, uint32_t &CH4, uint32_t &nch) {
        const uint32_t C4 = cp(m.fd[it.f])->C4;
        CH4 = pass_chunks(C4, 1);
        nch = min(CH4, C4 - it.p * CH4);
    };
    // the coefficient rows of an item: the stream's quantized rows (decode) or float rows
    auto coef_rows = [&](CFrame *d) -> const GAS float * {
        if (d->mode == MODE_DECODE) {
            const CAS gsc_header *h = cp(reinterpret_cast<const gsc_header *>(d->in_stream));
            return reinterpret_cast<const GAS float *>(gp(d->in_stream + h->coef_offset));
        }
        return gp(d->mode == MODE_ENCODE ? d->coef_f32 : d->attr);
    };
    auto prefetch = [&](const Item1 &it, Sched1 &S, float4 (&D)[NR1], float4 (&O)[NO1]) {
        CFrame *d = cp(m.fd[it.f]);
        uint32_t CH4, nch;
        slice(it, CH4, nch);
        const Roles R(CH4);
        load_sched1(d, it, S);
        if (R.act && R.c4 < nch) {
            const uint32_t c4 = it.p * CH4 + R.c4;
            load_rows1<VEC>(coef_rows(d), d->C, R, c4, it.mlen, false, nullptr, it.s, D);
            if (!it.final_level && S.ocnt > 0) {
                const GAS float *src = gp(d->lv[1].vbuf);
#pragma unroll
                for (int u = 0; u < NO1; ++u) {
                    const uint32_t o = min(R.row0 + (uint32_t)u * R.RPB, S.ocnt - 1);
                    O[u] = gload4(src + ((size_t)(S.obase + o) * d->C4 + c4) * 4);
                }
            }
        }
    };
    Item1 it0 = item1(m, blockIdx.x, fc);
    Item1 it1 = item1(m, blockIdx.x + G, fc);
    Sched1 S;
    float4 D[NR1], O[NO1];
    uint32_t stf = ~0u;  // frame whose steps are in s_st
    if (it0.ok) prefetch(it0, S, D, O);

    for (uint32_t i = blockIdx.x; i < items; i += G) {
        CFrame *d = cp(m.fd[it0.f]);
        const bool decode = d->mode == MODE_DECODE;
        uint32_t CH4, nch;
        slice(it0, CH4, nch);
        const Roles R(CH4);
        const uint32_t c4 = it0.p * CH4 + R.c4;
        const bool live = it0.ok && R.act && R.c4 < nch;
        const uint32_t C = d->C;
        const uint32_t ocnt = S.ocnt;
        const bool has_open = it0.ok && !it0.final_level && ocnt > 0;
        if (decode && it0.f != stf) {  // the frame's dequantization steps (once per frame)
            stf = it0.f;
            const CAS gsc_header *h = cp(reinterpret_cast<const gsc_header *>(d->in_stream));
            // (read only from a stream that holds a header: a shorter one fails the header check
            // and none of its items is transformed)
            if (tid < GSC_MAX_CHANNELS) s_st[tid] = d->in_bytes >= GSC_HEADER_BYTES ? h->quant_step[tid] : 0.0f;
        }
        __syncthreads();  // the previous item is no longer read from LDS; s_st is written
        // ---- the current item's schedule and coefficient rows into LDS (branch-free, see
        // commit_sched1)
        commit_sched1(S, it0, CH4, d->n, fp64_weights(*d), s_rec, s_ab, s_lstw, s_oposw, s_m0, s_lmask);
        {
            float st[4] = {1.f, 1.f, 1.f, 1.f};
            if (decode)
#pragma unroll
                for (int q = 0; q < 4; ++q) st[q] = s_st[min(4 * c4 + q, C - 1)];
            const uint32_t sink = RT * CH4;
#pragma unroll
            for (int u = 0; u < NR1; ++u) {
                const uint32_t j = R.row0 + (uint32_t)u * R.RPB;
                float4 v = D[u];
                if (decode)
                    v = make_float4((float)__float_as_int(v.x) * st[0], (float)__float_as_int(v.y) * st[1],
                                    (float)__float_as_int(v.z) * st[2], (float)__float_as_int(v.w) * st[3]);
                s_y[live && j < it0.mlen ? j * CH4 + R.c4 : sink] = v;
            }
        }
        __syncthreads();
        // ---- open entries take the low-pass handed down by S_2 (also branch-free)
        {
            const uint32_t sink = RT * CH4;
#pragma unroll
            for (int u = 0; u < NO1; ++u) {
                const uint32_t o = R.row0 + (uint32_t)u * R.RPB;
                const bool w = live && has_open && o < ocnt;
                s_y[w ? s_opos[min(o, (uint32_t)OPEN_CAP - 1)] * CH4 + R.c4 : sink] = O[u];
            }
        }
        // ---- prefetch the next item (issued first), then the item after it
        if (it1.ok) prefetch(it1, S, D, O);
        const Item1 it2 = item1(m, i + 2 * G, fc);
        // ---- the current item: all local merges undone, across chunks, then within chunks
        if (it0.ok) {
            __syncthreads();  // the open-entry writes
            const uint64_t wmask = s_lmask[R.w], xmask = s_lmask[CROSS];
            cross_phase(s_y, R, s_rec, s_ab, s_lst, xmask, nch, true);
            wave_phase(s_y, R, s_rec, s_ab, s_lst, wmask, nch, true, R.w);
            __syncthreads();
            if (live) {
                const uint32_t mlen = it0.mlen, s = it0.s;
                const uint32_t y0 = R.row0 * CH4 + R.c4, ystep = R.RPB * CH4;
                if (d->mode == MODE_STE_BWD) {
                    // voxel gradient = synthesized rows + the added rows; each member Gaussian
                    // receives it divided by the member count (the voxel row is the members' mean)
                    GAS float *out = gp(d->attr_out);
                    const GAS float *ga = gp(d->grad_add);
                    const GAS uint32_t *vh = gp(d->vh);
                    const GAS uint32_t *perm = gp((d->P & 1) ? d->vals_b : d->vals_a);
                    const uint32_t n = d->n, nlast = n ? n - 1 : 0u;
                    for (uint32_t j = R.row0, yi = y0; j < mlen; j += R.RPB, yi += ystep) {
                        const uint32_t v = s + j;
                        const float4 a = s_y[yi];
                        const float4 b = ld4<VEC>(ga, v, C, c4);
                        const uint32_t m0 = min(vh[v], n), m1 = min(vh[v + 1], n);
                        const float cnt = (float)(m1 - m0);
                        const float4 g = make_float4((a.x + b.x) / cnt, (a.y + b.y) / cnt, (a.z + b.z) / cnt,
                                                     (a.w + b.w) / cnt);
                        for (uint32_t mm = m0; mm < m1; ++mm) st4<VEC>(out, min(perm[mm], nlast), C, c4, g);
                    }
                } else {
                    GAS float *out = gp(d->mode == MODE_ADJ_F32 ? d->coef_f32 : d->attr_out);
                    for (uint32_t j = R.row0, yi = y0; j < mlen; j += R.RPB, yi += ystep)
                        st4<VEC>(out, s + j, C, c4, s_y[yi]);
                }
            }
        }
        it0 = it1;
        it1 = it2;
    }
    if (finish) finish_if_last(m, FIN_INV, s_y);
}

// Dynamic LDS of a transform launch: the slice of RT entries of the widest tiling level, plus
// one sink slot for writes that are masked off by address rather than by branch.
size_t raht_lds_bytes(int C4)
{
    const uint32_t a = pass_chunks((uint32_t)C4, 1), b = pass_chunks((uint32_t)C4, 2);
    return ((size_t)RT * (a > b ? a : b) + 1) * sizeof(float4);
}

// Launch limits of the current device, queried once per (device, kernel, dynamic LDS) and kept
// in tables that every host thread may read and fill (guarded by one mutex).
constexpr int MAX_DEVICES = 64;
static std::mutex g_limits_mu;
static int g_cus[MAX_DEVICES];  // compute units per device, 0 = not queried yet

static int current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) dev = 0;
    return dev;
}

static uint32_t cu_count()
{
    const int dev = current_device();
    std::lock_guard<std::mutex> lock(g_limits_mu);
    if (g_cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        g_cus[dev] = v;
    }
    return (uint32_t)g_cus[dev];
}

// Workgroups of `kern` that fit on one CU at once (occupancy calculator), cached.
static uint32_t blocks_per_cu(const void *kern, int threads, size_t lds)
{
    struct Entry {
        int dev;
        const void *kern;
        size_t lds;
        int nb;
    };
    static Entry cache[64];
    static int used = 0;
    const int dev = current_device();
    std::lock_guard<std::mutex> lock(g_limits_mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].dev == dev && cache[i].kern == kern && cache[i].lds == lds) return (uint32_t)cache[i].nb;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, lds) != hipSuccess || nb < 0) nb = 0;
    if (used < 64) cache[used++] = Entry{dev, kern, lds, nb};
    return (uint32_t)nb;
}

// Workgroups of a persistent launch whose workgroups wait on one another: every one of them must
// be resident at once, so at most what the occupancy calculator allows per CU (and `per_cu_max`)
// times the CUs, a multiple of 8 (the XCDs), and at most `want`. 0 if none fits.
static uint32_t resident_grid(const void *kern, size_t lds, uint32_t per_cu_max, uint32_t want)
{
    uint32_t per_cu = blocks_per_cu(kern, RAHT_THREADS, lds);
    if (per_cu > per_cu_max) per_cu = per_cu_max;
    const uint32_t g = per_cu * cu_count() / 8 * 8;
    return want < g ? (want + 7) / 8 * 8 : g;
}

// Workgroups of a persistent first-level launch over `items` items: resident at once (as above),
// a multiple of 8 NP (an item and its partner slice, items i and i + 8 of a group of 8 NP, run
// at the same time on one XCD), and as few as give every workgroup the same number of items, up
// to one. 0 if none fits.
static uint32_t persist_grid(uint32_t items, int C4, const void *kern, size_t lds)
{
    uint32_t per_cu = blocks_per_cu(kern, RAHT_THREADS, lds);
    if (per_cu > (uint32_t)PERSIST_PER_CU) per_cu = PERSIST_PER_CU;
    const uint32_t unit = 8 * channel_passes((uint32_t)C4, 1);
    const uint32_t gmax = per_cu * cu_count() / unit * unit;
    if (gmax == 0) return 0;
    if (items <= gmax) return items;
    const uint32_t rounds = ceil_div(items, gmax);
    return ceil_div(ceil_div(items, rounds), unit) * unit;
}

hipError_t launch_raht_fwd(const TileMap &m, int kmax, bool finish, const RahtCfg &cfg, hipStream_t s)
{
    const size_t lds = raht_lds_bytes(cfg.C4);
    const void *kern = cfg.vec ? (cfg.pow2 ? reinterpret_cast<const void *>(k_raht_fwd<true, true>)
                                           : reinterpret_cast<const void *>(k_raht_fwd<true, false>))
                               : (cfg.pow2 ? reinterpret_cast<const void *>(k_raht_fwd<false, true>)
                                           : reinterpret_cast<const void *>(k_raht_fwd<false, false>));
    const uint32_t g = persist_grid(m.start[m.F], cfg.C4, kern, lds);
    if (g == 0) return hipErrorInvalidConfiguration;
    const dim3 grid(g), block(RAHT_THREADS);
    const int fin = finish ? 1 : 0;
    if (cfg.vec && cfg.pow2) hipLaunchKernelGGL((k_raht_fwd<true, true>), grid, block, lds, s, m, kmax, fin);
    else if (cfg.vec) hipLaunchKernelGGL((k_raht_fwd<true, false>), grid, block, lds, s, m, kmax, fin);
    else if (cfg.pow2) hipLaunchKernelGGL((k_raht_fwd<false, true>), grid, block, lds, s, m, kmax, fin);
    else hipLaunchKernelGGL((k_raht_fwd<false, false>), grid, block, lds, s, m, kmax, fin);
    return hipGetLastError();
}

hipError_t launch_raht_inv_up(const TileMap &m, int kmax, uint32_t items_max, bool prelude, const RahtCfg &cfg,
                              hipStream_t s)
{
    const size_t lds = raht_lds_bytes(cfg.C4);
    const void *kern = cfg.vec ? reinterpret_cast<const void *>(k_raht_inv_up<true>)
                               : reinterpret_cast<const void *>(k_raht_inv_up<false>);
    uint32_t g = resident_grid(kern, lds, 4, items_max > 0 ? items_max : 1u);
    if (g > UP_GRID_MAX) g = UP_GRID_MAX;  // (one phase flag per workgroup)
    if (g == 0) return hipErrorInvalidConfiguration;
    const dim3 grid(g), block(RAHT_THREADS);
    if (cfg.vec) hipLaunchKernelGGL((k_raht_inv_up<true>), grid, block, lds, s, m, kmax, prelude ? 1 : 0);
    else hipLaunchKernelGGL((k_raht_inv_up<false>), grid, block, lds, s, m, kmax, prelude ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_raht_inv(const TileMap &m, bool finish, const RahtCfg &cfg, hipStream_t s)
{
    const size_t lds = raht_lds_bytes(cfg.C4);
    const void *kern = cfg.vec ? reinterpret_cast<const void *>(k_raht_inv<true>)
                               : reinterpret_cast<const void *>(k_raht_inv<false>);
    const uint32_t g = persist_grid(m.start[m.F], cfg.C4, kern, lds);
    if (g == 0) return hipErrorInvalidConfiguration;
    const dim3 grid(g), block(RAHT_THREADS);
    const int fin = finish ? 1 : 0;
    if (cfg.vec) hipLaunchKernelGGL((k_raht_inv<true>), grid, block, lds, s, m, fin);
    else hipLaunchKernelGGL((k_raht_inv<false>), grid, block, lds, s, m, fin);
    return hipGetLastError();
}

}  // namespace gsc
