// RAHT on the GPU: prelude, forward transform (+ merge of duplicates and quantization),
// inverse transform (+ dequantization).
//
// The transform is the one of Sec. 3.1-3.3 (Eq. 1, Alg. 4-6): at binary level l = 1..3J every
// left sibling k of the active list I_l merges with its right sibling k+1,
//   [lo; hi] = [a b; -b a] [y0; y1],  a = sqrt(w0/(w0+w1)), b = sqrt(w1/(w0+w1)),
// the low-pass staying at the left entry and the high-pass at the right one. An entry i > 0 is
// removed from the active list (merged as a right sibling) exactly at level
// l_i = msb(M[i-1] xor M[i]) + 1, so I_l = {i : l_i >= l} and the pairs of level l are the
// entries with l_i = l and their active neighbours.
//
// Tiling. A workgroup owns a tile of RT consecutive entries and performs every merge whose two
// operands lie inside the tile, all levels in LDS. A merge whose left neighbour lies before the
// tile, or whose right operand extends past it, is deferred: its entry is "open" and moves, with
// its partial low-pass, to the next sequence S_{k+1}. The merges among open entries are exactly
// the deferred merges (an open entry's neighbours in the active list are open too), so the same
// kernels run again on S_{k+1}, until one tile holds the whole sequence. At most 6J entries of a
// tile are open (the merges whose parent straddles one of its two boundaries: one per level).
#include "gsc_device.h"

namespace gsc {

static_assert(RT < 1024, "merge records pack three 10-bit positions");
constexpr int PRE_THREADS = 256;

// Size of the entry sequence S_k; a size beyond its allocation (impossible when every tile
// leaves at most 6J + 2 entries open) is reported and treated as empty.
__device__ inline uint32_t seq_size(const FrameDesc &fd, Ctrl *ctrl, int k)
{
    const uint32_t nk = k == 1 ? ctrl->n_vox : ctrl->lvl_n[k];
    if (nk > fd.lv[k].cap) {
        set_error(ctrl, GSC_ERR_INTERNAL);
        return 0;
    }
    return nk;
}
__device__ inline bool seq_active(uint32_t nk, int k) { return k == 1 ? nk >= 1 : nk >= 2; }

// ============================================================================ prelude
// Per tile: the binary level of every entry, then the levels present, in increasing order; at
// level x every entry with l = x looks at its current neighbours in a doubly linked active
// list, records a local merge (left neighbour inside the tile, right operand ending inside the
// tile or at the next entry after it when that entry survives to a higher level) or marks
// itself open, and unlinks itself. Entries of one level are never adjacent in the active list,
// so the unlinks of a level do not conflict. Local merges are stored sorted by level; open
// entries are compacted, in order, into S_{k+1} with a decoupled look-back.
__global__ __launch_bounds__(PRE_THREADS) void k_prelude(TileMap m, int k)
{
    __shared__ uint32_t s_tile;
    __shared__ uint8_t s_lvl[RT];
    __shared__ uint8_t s_state[RT];  // 0 = untouched, 1 = local merge, 2 = open
    __shared__ int16_t s_left[RT], s_right[RT];
    __shared__ int16_t s_l[RT], s_r[RT];
    __shared__ unsigned long long s_mask;
    __shared__ uint32_t s_lcnt[NLVL], s_lfill[NLVL];
    __shared__ uint16_t s_lstart[LSTART_N];
    __shared__ uint32_t s_tmp[PRE_THREADS / WAVE + 1];
    __shared__ uint32_t s_base;
    __shared__ uint32_t s_lvl_e;

    const uint32_t f = frame_of(m, blockIdx.x);
    const FrameDesc &fd = *m.fd[f];
    Ctrl *ctrl = fd.ctrl;
    if (load_error(ctrl)) return;
    if ((uint32_t)k > fd.K) return;
    const uint32_t nk = seq_size(fd, ctrl, k);
    if (!seq_active(nk, k)) return;
    const RahtLevel &lv = fd.lv[k];
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_tile = atomicAdd(&ctrl->tile_ctr[TC_PRELUDE + k], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t s = tile * RT;
    if (s >= nk) return;
    const uint32_t e = min(nk, s + RT);
    const int mlen = (int)(e - s);
    const uint64_t *codes = (fd.mode == MODE_FWD_F32 || fd.mode == MODE_ADJ_F32) ? fd.codes_in : fd.leaf;

    for (int j = tid; j < RT; j += PRE_THREADS) {
        if (j < mlen) {
            const uint32_t i = s + j;
            s_lvl[j] = k == 1 ? (i == 0 ? LVL_NONE : merge_level(codes[i - 1], codes[i])) : lv.s_lvl[i];
        }
        s_left[j] = (int16_t)(j - 1);
        s_right[j] = (int16_t)(j + 1);
        s_state[j] = 0;
    }
    if (tid < NLVL) {
        s_lcnt[tid] = 0;
        s_lfill[tid] = 0;
    }
    if (tid == 0) {
        s_mask = 0;
        s_lvl_e = e < nk ? (k == 1 ? merge_level(codes[e - 1], codes[e]) : lv.s_lvl[e]) : LVL_NONE;
    }
    __syncthreads();
    for (int j = tid; j < mlen; j += PRE_THREADS)
        if (s_lvl[j] < NLVL) atomicOr(&s_mask, 1ull << s_lvl[j]);
    __syncthreads();
    uint64_t mask = s_mask;
    const uint32_t lvl_e = s_lvl_e;
    while (mask) {
        const uint32_t x = (uint32_t)(__ffsll((long long)mask) - 1);
        mask &= mask - 1;
        for (int j = tid; j < mlen; j += PRE_THREADS) {
            if (s_lvl[j] != x) continue;
            const int l = s_left[j], r = s_right[j];
            const bool local = (l >= 0) && (r < mlen || lvl_e > x);
            if (local) {
                s_state[j] = 1;
                s_l[j] = (int16_t)l;
                s_r[j] = (int16_t)r;
                atomicAdd(&s_lcnt[x], 1u);
            } else {
                s_state[j] = 2;
            }
            if (l >= 0) s_right[l] = (int16_t)r;
            if (r < mlen) s_left[r] = (int16_t)l;
        }
        __syncthreads();
    }
    for (int j = tid; j < mlen; j += PRE_THREADS)
        if (s_state[j] == 0) s_state[j] = 2;  // entry 0 of the sequence: never merged here
    if (tid == 0) {
        uint32_t run = 0;
        for (int x = 0; x < NLVL; ++x) {
            s_lstart[x] = (uint16_t)run;
            run += s_lcnt[x];
        }
        s_lstart[NLVL] = (uint16_t)run;
        s_lstart[NLVL + 1] = (uint16_t)run;
    }
    __syncthreads();
    for (int j = tid; j < mlen; j += PRE_THREADS) {
        if (s_state[j] != 1) continue;
        const uint32_t x = s_lvl[j];
        const uint32_t slot = s_lstart[x] + atomicAdd(&s_lfill[x], 1u);
        if (slot < (uint32_t)RT)
            lv.rec[(size_t)tile * RT + slot] =
            (uint32_t)j | ((uint32_t)s_l[j] << 10) | ((uint32_t)s_r[j] << 20);
    }
    for (int x = tid; x < LSTART_N; x += PRE_THREADS) lv.lstart[(size_t)tile * LSTART_N + x] = s_lstart[x];

    // open entries, in order: thread t owns entries 2t and 2t+1
    constexpr int EPT = RT / PRE_THREADS;
    uint32_t my = 0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int j = tid * EPT + i;
        if (j < mlen && s_state[j] == 2) ++my;
    }
    uint32_t total;
    uint32_t rank = block_excl_scan<PRE_THREADS>(my, s_tmp, &total);
    if (tid == 0) {
        if (total > open_max((int)fd.J)) set_error(ctrl, GSC_ERR_INTERNAL);
        s_base = (uint32_t)lookback<OpSum>(lv.status, 1, tile, total, ctrl);
    }
    __syncthreads();
    const uint32_t base = s_base;
    const bool has_next = (uint32_t)k < fd.K;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int j = tid * EPT + i;
        if (j < mlen && s_state[j] == 2) {
            if (rank < (uint32_t)OPEN_CAP) lv.opos[(size_t)tile * OPEN_CAP + rank] = (uint16_t)j;
            if (has_next) {
                const RahtLevel &nx = fd.lv[k + 1];
                const uint32_t o = base + rank;
                if (o < nx.cap) {
                    nx.s_idx[o] = k == 1 ? s + j : lv.s_idx[s + j];
                    nx.s_lvl[o] = s_lvl[j];
                }
            }
            ++rank;
        }
    }
    if (tid == 0) {
        lv.obase[tile] = base;
        lv.ocnt[tile] = min(total, (uint32_t)OPEN_CAP);
        if (e == nk) ctrl->lvl_n[k + 1] = base + total;
    }
}

hipError_t launch_prelude(const TileMap &m, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_prelude, dim3(m.start[m.F]), dim3(PRE_THREADS), 0, s, m, k);
    return hipGetLastError();
}

// =========================================================== shared transform pieces
struct TileSched {
    uint32_t tile, s, e, nk, obase, ocnt, nrec;
    int mlen;
    bool final_level;
};

// Loads the tile's schedule into LDS and computes (a, b) of every local merge. Returns false if
// the workgroup has nothing to do.
__device__ inline bool load_schedule(const FrameDesc &fd, Ctrl *ctrl, int k, uint32_t tile,
                                     TileSched &ts, uint32_t *s_rec, float2 *s_ab,
                                     uint16_t *s_lst, uint16_t *s_opos, uint32_t *s_idx)
{
    const uint32_t nk = seq_size(fd, ctrl, k);
    if (!seq_active(nk, k)) return false;
    const RahtLevel &lv = fd.lv[k];
    const uint32_t s = tile * RT;
    if (s >= nk) return false;
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    ts.tile = tile;
    ts.s = s;
    ts.e = min(nk, s + RT);
    ts.nk = nk;
    ts.mlen = (int)(ts.e - s);
    ts.final_level = nk <= (uint32_t)RT;
    ts.obase = lv.obase[tile];
    ts.ocnt = lv.ocnt[tile];
    for (uint32_t x = tid; x < LSTART_N; x += NT) s_lst[x] = lv.lstart[(size_t)tile * LSTART_N + x];
    for (uint32_t o = tid; o < ts.ocnt; o += NT) s_opos[o] = lv.opos[(size_t)tile * OPEN_CAP + o];
    if (k >= 2) {
        for (int j = tid; j < ts.mlen; j += NT) s_idx[j] = lv.s_idx[s + j];
        if (tid == 0) s_idx[ts.mlen] = ts.e < nk ? lv.s_idx[ts.e] : ctrl->n_vox;
    }
    __syncthreads();
    ts.nrec = s_lst[NLVL];
    for (uint32_t q = tid; q < ts.nrec; q += NT) {
        const uint32_t rec = lv.rec[(size_t)tile * RT + q];
        s_rec[q] = rec;
        const uint32_t j = rec & 1023u, l = (rec >> 10) & 1023u, r = rec >> 20;
        uint32_t ij, il, ir;
        if (k == 1) {
            ij = j;
            il = l;
            ir = r;
        } else {
            ij = s_idx[j];
            il = s_idx[l];
            ir = s_idx[r];
        }
        const float w0 = (float)(ij - il), w1 = (float)(ir - ij);
        const float sum = w0 + w1;
        s_ab[q] = make_float2(sqrtf(w0 / sum), sqrtf(w1 / sum));
    }
    return true;
}

__device__ inline uint32_t entry_index(int k, const uint32_t *s_idx, uint32_t s, int j)
{
    return k == 1 ? s + (uint32_t)j : s_idx[j];
}

__device__ inline void butterfly_level(float4 *s_y, uint32_t C4, const uint32_t *s_rec,
                                       const float2 *s_ab, uint32_t q0, uint32_t q1, bool inverse)
{
    const uint32_t n = (q1 - q0) * C4;
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) {
        const uint32_t q = q0 + t / C4, c4 = t % C4;
        const uint32_t rec = s_rec[q];
        const uint32_t j = rec & 1023u, l = (rec >> 10) & 1023u;
        const float2 ab = s_ab[q];
        const float4 y0 = s_y[l * C4 + c4], y1 = s_y[j * C4 + c4];
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
        s_y[l * C4 + c4] = lo;
        s_y[j * C4 + c4] = hi;
    }
}

__device__ inline float get4(const float4 &v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Loads channels [4*c4, 4*c4+4) of row `row` of a row-major float matrix with C columns.
__device__ inline float4 load_row4(const float *base, uint64_t row, uint32_t C, uint32_t c4,
                                   bool vec)
{
    const float *p = base + row * C + 4 * c4;
    if (vec) return *reinterpret_cast<const float4 *>(p);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t c = 4 * c4;
    if (c + 0 < C) v.x = p[0];
    if (c + 1 < C) v.y = p[1];
    if (c + 2 < C) v.z = p[2];
    if (c + 3 < C) v.w = p[3];
    return v;
}
__device__ inline void store_row4(float *base, uint64_t row, uint32_t C, uint32_t c4,
                                  const float4 &v, bool vec)
{
    float *p = base + row * C + 4 * c4;
    if (vec) {
        *reinterpret_cast<float4 *>(p) = v;
        return;
    }
    const uint32_t c = 4 * c4;
    if (c + 0 < C) p[0] = v.x;
    if (c + 1 < C) p[1] = v.y;
    if (c + 2 < C) p[2] = v.z;
    if (c + 3 < C) p[3] = v.w;
}

__device__ inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ==================================================================== forward transform
__global__ __launch_bounds__(RAHT_THREADS) void k_raht_fwd(TileMap m, int k)
{
    extern __shared__ float4 s_y[];
    __shared__ uint32_t s_rec[RT];
    __shared__ float2 s_ab[RT];
    __shared__ uint16_t s_lst[LSTART_N];
    __shared__ uint16_t s_opos[OPEN_CAP];
    __shared__ uint32_t s_idx[RT + 1];
    __shared__ uint32_t s_m0[RT + 1];
    __shared__ uint32_t s_first[RT];

    const uint32_t f = frame_of(m, blockIdx.x);
    const FrameDesc &fd = *m.fd[f];
    Ctrl *ctrl = fd.ctrl;
    if (load_error(ctrl)) return;
    if ((uint32_t)k > fd.K) return;
    TileSched ts;
    if (!load_schedule(fd, ctrl, k, blockIdx.x - m.start[f], ts, s_rec, s_ab, s_lst, s_opos, s_idx))
        return;
    const uint32_t C = fd.C, C4 = fd.C4, J = fd.J;
    const uint32_t tid = threadIdx.x;
    const uint32_t nvals = (uint32_t)ts.mlen * C4;

    // ---- load the entries' values
    if (k == 1 && fd.mode == MODE_ENCODE) {
        // merge duplicates: the mean of the rows of the Gaussians in the voxel (Sec. 2.1),
        // summed in input order (the sort is stable). The run starts and the first member's
        // row are staged in LDS so that the row loads below are independent of each other.
        const uint32_t *perm = (fd.P & 1) ? fd.vals_b : fd.vals_a;
        for (int j = tid; j <= ts.mlen; j += RAHT_THREADS) s_m0[j] = fd.vh[ts.s + j];
        __syncthreads();
        for (int j = tid; j < ts.mlen; j += RAHT_THREADS) s_first[j] = perm[s_m0[j]];
        __syncthreads();
        const bool vec = (C % 4 == 0) && aligned16(fd.attr);
        constexpr int U = 4;
        for (uint32_t t0 = tid; t0 < nvals; t0 += U * RAHT_THREADS) {
            float4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t t = t0 + u * RAHT_THREADS;
                if (t < nvals) v[u] = load_row4(fd.attr, s_first[t / C4], C, t % C4, vec);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t t = t0 + u * RAHT_THREADS;
                if (t >= nvals) break;
                const uint32_t j = t / C4, c4 = t % C4;
                const uint32_t m0 = s_m0[j], m1 = s_m0[j + 1];
                float4 acc = v[u];
                if (m1 - m0 > 1) {
                    for (uint32_t mm = m0 + 1; mm < m1; ++mm) {
                        const float4 x = load_row4(fd.attr, perm[mm], C, c4, vec);
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
                }
                s_y[j * C4 + c4] = acc;
            }
        }
    } else if (k == 1) {
        const bool vec = (C % 4 == 0) && aligned16(fd.attr);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            s_y[j * C4 + c4] = load_row4(fd.attr, ts.s + j, C, c4, vec);
        }
    } else {
        const float4 *src = reinterpret_cast<const float4 *>(fd.lv[k - 1].vbuf);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            s_y[j * C4 + c4] = src[(size_t)(ts.s + j) * C4 + c4];
        }
    }
    __syncthreads();

    // ---- all local merges, level by level (bottom-up)
    for (uint32_t x = 1; x <= 3 * J; ++x) {
        const uint32_t q0 = s_lst[x], q1 = s_lst[x + 1];
        if (q0 == q1) continue;
        butterfly_level(s_y, C4, s_rec, s_ab, q0, q1, false);
        __syncthreads();
    }

    // ---- outputs: coefficient rows of every entry (an open entry's row is rewritten by the
    // level that completes its merge), open entries' partial low-passes to S_{k+1}
    if (fd.mode == MODE_ENCODE) {
        int32_t *coef = reinterpret_cast<int32_t *>(fd.stream + (size_t)0);
        // coefficient offset from the level sizes (same formula as the header)
        uint64_t off = GSC_HEADER_BYTES, run = 0;
        for (uint32_t d = 0; d < J; ++d) {
            run += ctrl->hist_D[d];
            off += run;
        }
        coef = reinterpret_cast<int32_t *>(fd.stream + align_up(off, 256));
        const double omt = 1.0 - (double)fd.tau;
        const bool vec = (C % 4 == 0);
        float *cf = fd.coef_f32;
        const bool vecf = vec && cf && aligned16(cf);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            const float4 y = s_y[j * C4 + c4];
            const uint64_t row = entry_index(k, s_idx, ts.s, (int)j);
            int32_t q[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t c = 4 * c4 + i;
                q[i] = c < C ? quantize(get4(y, i), fd.step[c], fd.inv_step[c], omt,
                                        (fd.pow2_steps >> c) & 1ull)
                             : 0;
            }
            int32_t *p = coef + row * C + 4 * c4;
            if (vec) {
                *reinterpret_cast<int4 *>(p) = make_int4(q[0], q[1], q[2], q[3]);
            } else {
                for (int i = 0; i < 4; ++i)
                    if (4 * c4 + i < C) p[i] = q[i];
            }
            if (cf) store_row4(cf, row, C, c4, y, vecf);
        }
    } else {  // MODE_FWD_F32: float coefficient rows
        float *cf = fd.coef_f32;
        const bool vecf = (C % 4 == 0) && aligned16(cf);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            store_row4(cf, entry_index(k, s_idx, ts.s, (int)j), C, c4, s_y[j * C4 + c4], vecf);
        }
    }
    if (!ts.final_level) {
        float4 *dst = reinterpret_cast<float4 *>(fd.lv[k].vbuf);
        const uint32_t n = ts.ocnt * C4;
        for (uint32_t t = tid; t < n; t += RAHT_THREADS) {
            const uint32_t o = t / C4, c4 = t % C4;
            dst[(size_t)(ts.obase + o) * C4 + c4] = s_y[s_opos[o] * C4 + c4];
        }
    }
}

// ==================================================================== inverse transform
__global__ __launch_bounds__(RAHT_THREADS) void k_raht_inv(TileMap m, int k)
{
    extern __shared__ float4 s_y[];
    __shared__ uint32_t s_rec[RT];
    __shared__ float2 s_ab[RT];
    __shared__ uint16_t s_lst[LSTART_N];
    __shared__ uint16_t s_opos[OPEN_CAP];
    __shared__ uint32_t s_idx[RT + 1];

    const uint32_t f = frame_of(m, blockIdx.x);
    const FrameDesc &fd = *m.fd[f];
    Ctrl *ctrl = fd.ctrl;
    if (load_error(ctrl)) return;
    if ((uint32_t)k > fd.K) return;
    TileSched ts;
    if (!load_schedule(fd, ctrl, k, blockIdx.x - m.start[f], ts, s_rec, s_ab, s_lst, s_opos, s_idx))
        return;
    const uint32_t C = fd.C, C4 = fd.C4, J = fd.J;
    const uint32_t tid = threadIdx.x;
    const uint32_t nvals = (uint32_t)ts.mlen * C4;

    // ---- coefficients of every entry (the high-pass stored at it, or the DC at entry 0)
    if (fd.mode == MODE_DECODE) {
        const gsc_header *h = reinterpret_cast<const gsc_header *>(fd.in_stream);
        const int32_t *coef = reinterpret_cast<const int32_t *>(fd.in_stream + h->coef_offset);
        const bool vec = (C % 4 == 0);
        constexpr int U = 4;
        for (uint32_t t0 = tid; t0 < nvals; t0 += U * RAHT_THREADS) {
            int4 qv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t t = t0 + u * RAHT_THREADS;
                if (t >= nvals) break;
                const uint32_t j = t / C4, c4 = t % C4;
                const uint64_t row = entry_index(k, s_idx, ts.s, (int)j);
                const int32_t *p = coef + row * C + 4 * c4;
                int4 q = make_int4(0, 0, 0, 0);
                if (vec) {
                    q = *reinterpret_cast<const int4 *>(p);
                } else {
                    const uint32_t c = 4 * c4;
                    if (c + 0 < C) q.x = p[0];
                    if (c + 1 < C) q.y = p[1];
                    if (c + 2 < C) q.z = p[2];
                    if (c + 3 < C) q.w = p[3];
                }
                qv[u] = q;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t t = t0 + u * RAHT_THREADS;
                if (t >= nvals) break;
                const uint32_t j = t / C4, c4 = t % C4;
                const uint32_t c = 4 * c4;
                float4 y;
                y.x = (float)qv[u].x * (c + 0 < C ? h->quant_step[c + 0] : 0.f);
                y.y = (float)qv[u].y * (c + 1 < C ? h->quant_step[c + 1] : 0.f);
                y.z = (float)qv[u].z * (c + 2 < C ? h->quant_step[c + 2] : 0.f);
                y.w = (float)qv[u].w * (c + 3 < C ? h->quant_step[c + 3] : 0.f);
                s_y[j * C4 + c4] = y;
            }
        }
    } else {  // MODE_ADJ_F32: float coefficient rows
        const bool vec = (C % 4 == 0) && aligned16(fd.attr);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            s_y[j * C4 + c4] = load_row4(fd.attr, entry_index(k, s_idx, ts.s, (int)j), C, c4, vec);
        }
    }
    __syncthreads();
    // ---- open entries take the low-pass handed down by the next sequence
    if (!ts.final_level) {
        const float4 *src = reinterpret_cast<const float4 *>(fd.lv[k].vbuf);
        const uint32_t n = ts.ocnt * C4;
        for (uint32_t t = tid; t < n; t += RAHT_THREADS) {
            const uint32_t o = t / C4, c4 = t % C4;
            s_y[s_opos[o] * C4 + c4] = src[(size_t)(ts.obase + o) * C4 + c4];
        }
        __syncthreads();
    }
    // ---- all local merges undone, level by level (top-down)
    for (uint32_t x = 3 * J; x >= 1; --x) {
        const uint32_t q0 = s_lst[x], q1 = s_lst[x + 1];
        if (q0 == q1) continue;
        butterfly_level(s_y, C4, s_rec, s_ab, q0, q1, true);
        __syncthreads();
    }
    // ---- outputs
    if (k >= 2) {
        float4 *dst = reinterpret_cast<float4 *>(fd.lv[k - 1].vbuf);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            dst[(size_t)(ts.s + j) * C4 + c4] = s_y[j * C4 + c4];
        }
    } else {
        float *out = fd.mode == MODE_DECODE ? fd.attr_out : fd.coef_f32;
        const bool vec = (C % 4 == 0) && aligned16(out);
        for (uint32_t t = tid; t < nvals; t += RAHT_THREADS) {
            const uint32_t j = t / C4, c4 = t % C4;
            store_row4(out, ts.s + j, C, c4, s_y[j * C4 + c4], vec);
        }
    }
}

size_t raht_lds_bytes(int C4) { return (size_t)RT * C4 * sizeof(float4); }

hipError_t launch_raht_fwd(const TileMap &m, int k, int C4, hipStream_t s)
{
    const size_t lds = raht_lds_bytes(C4);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_raht_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)raht_lds_bytes(GSC_MAX_CHANNELS / 4));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_raht_fwd, dim3(m.start[m.F]), dim3(RAHT_THREADS), lds, s, m, k);
    return hipGetLastError();
}

hipError_t launch_raht_inv(const TileMap &m, int k, int C4, hipStream_t s)
{
    const size_t lds = raht_lds_bytes(C4);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_raht_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)raht_lds_bytes(GSC_MAX_CHANNELS / 4));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_raht_inv, dim3(m.start[m.F]), dim3(RAHT_THREADS), lds, s, m, k);
    return hipGetLastError();
}

}  // namespace gsc
