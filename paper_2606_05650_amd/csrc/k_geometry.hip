// Geometry kernels of the codec: per-call setup, bounding cube, voxelization + Morton codes +
// radix histograms, one-sweep radix sort passes, duplicate merge (unique), octree occupancy
// bytes for all levels in one pass, level-synchronous octree decoding, and the final
// header/info write. Every kernel takes a TileMap so that one launch serves a batch of frames.
#include "gsc_device.h"

namespace gsc {

// ====================================================================== setup / finish
// grid (blocks, F), SETUP_THREADS threads: block (b, f) zeroes its share of frame f's zero
// region (look-back status words, digit histograms); in an encode that finds the bounding cube,
// blocks 1 .. bbox_blocks(n) also take the frame's bounding-box partials (bbox_partial); block
// (0, f) builds the frame descriptor and initialises the control block. The zero region and the
// bounding-box slots come from the host's layout, so only block 0 computes it.
__device__ inline void bbox_partial(const float *pos_, uint32_t n, uint32_t b, uint32_t G, GAS uint32_t *slot);

__global__ __launch_bounds__(SETUP_THREADS) void k_setup(SetupArgs a)
{
    const uint32_t f = blockIdx.y;
    if (f >= a.count) return;
    const FrameArgs &fa = a.f[f];
    // zero the look-back status region (16-byte stores; the region is 256-byte aligned)
    if (!a.keep) {
        uint4 *z = reinterpret_cast<uint4 *>(fa.ws + fa.zero_off);
        const size_t nq = fa.zero_bytes / 16;
        const size_t stride = (size_t)gridDim.x * blockDim.x;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride)
            z[i] = make_uint4(0, 0, 0, 0);
    }
    if (a.mode == MODE_ENCODE && a.bbox_mode == 0 && !a.keep) {
        const uint32_t G = bbox_blocks(fa.n);
        if (blockIdx.x >= 1 && blockIdx.x <= G)
            bbox_partial(fa.pos, fa.n, blockIdx.x - 1, G,
                         gp(reinterpret_cast<uint32_t *>(fa.ws + fa.bbox_off)) + (size_t)(blockIdx.x - 1) * BBOX_SLOT);
    }
    if (blockIdx.x != 0) return;
    __shared__ Layout s_L;
    if (threadIdx.x == 0) make_layout((int64_t)fa.n, (int)a.J, (int)a.C, &s_L);
    __syncthreads();
    {   // the upper-level phase flags and the transforms' completion counters start at zero in
        // every call, also one that keeps the state
        uint32_t *fl = reinterpret_cast<uint32_t *>(fa.ws + s_L.lvl_flags);
        for (uint32_t i = threadIdx.x; i < UP_GRID_MAX + DONE_WORDS; i += blockDim.x) fl[i] = 0;
    }
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(fa.ws);
    FrameDesc *fd = reinterpret_cast<FrameDesc *>(fa.ws + DESC_OFF);
    __shared__ uint32_t s_prev_ok;
    if (a.keep && threadIdx.x == 0) {
        // the workspace must hold a straight-through forward of the same shape
        s_prev_ok = (fd->ste == STE_FORWARD && fd->n == fa.n && fd->J == a.J && fd->C == a.C) ? 1u : 0u;
    }
    if (!a.keep) {
        uint32_t *cw = reinterpret_cast<uint32_t *>(ctrl);
        for (uint32_t i = threadIdx.x; i < CTRL_BYTES / 4; i += blockDim.x) cw[i] = 0;
    }
    if (fa.info)
        for (uint32_t i = threadIdx.x; i < GSC_INFO_WORDS; i += blockDim.x) fa.info[i] = 0;
    __syncthreads();
    const uint32_t t = threadIdx.x;
    const Layout &L = s_L;
    if (t == 0) {
        if (a.keep) {
            if (!s_prev_ok) set_error(ctrl, GSC_ERR_INVALID_ARG);
        } else {
            ctrl->n_in = fa.n;
            if (a.mode == MODE_FWD_F32 || a.mode == MODE_ADJ_F32) ctrl->n_vox = fa.n;
        }
    }
    // the descriptor, built by several threads at once: wave 0 the per-channel steps, threads
    // 64.. the tiling levels, 96.. the octree-decoding status offsets, 128 the scalars
    if (t < GSC_MAX_CHANNELS) {
        const float st = t < a.C ? a.step[t] : 1.0f;
        fd->step[t] = st;
        int e;
        const bool p2 = frexpf(st, &e) == 0.5f;
        fd->inv_step[t] = p2 ? 1.0f / st : 0.0f;
        const uint64_t pow2 = __ballot(p2);
        if (t == 0) fd->pow2_steps = pow2;
    } else if (t >= 64 && t <= 64 + MAXK) {
        const uint32_t k = t - 64;
        RahtLevel &lv = fd->lv[k];
        if (k >= 1 && k <= L.K) {
            lv.s_idx = reinterpret_cast<uint32_t *>(fa.ws + L.s_idx[k]);
            lv.s_lvl = reinterpret_cast<uint8_t *>(fa.ws + L.s_lvl[k]);
            lv.rec = reinterpret_cast<uint32_t *>(fa.ws + L.rec[k]);
            lv.lstart = reinterpret_cast<uint16_t *>(fa.ws + L.lstart[k]);
            lv.lmask = reinterpret_cast<uint64_t *>(fa.ws + L.lmask[k]);
            lv.opos = reinterpret_cast<uint16_t *>(fa.ws + L.opos[k]);
            lv.obase = reinterpret_cast<uint32_t *>(fa.ws + L.obase[k]);
            lv.ocnt = reinterpret_cast<uint32_t *>(fa.ws + L.ocnt[k]);
            lv.status = reinterpret_cast<uint64_t *>(fa.ws + L.status[k]);
            lv.vbuf = reinterpret_cast<float *>(fa.ws + L.vbuf[k]);
            lv.tiles = L.tiles[k];
            lv.cap = L.cap[k];
        } else {
            lv.s_idx = nullptr;
            lv.s_lvl = nullptr;
            lv.rec = nullptr;
            lv.lstart = nullptr;
            lv.lmask = nullptr;
            lv.opos = nullptr;
            lv.obase = nullptr;
            lv.ocnt = nullptr;
            lv.status = nullptr;
            lv.vbuf = nullptr;
            lv.tiles = 0;
            lv.cap = 0;
        }
    } else if (t == 96) {
        fd->dec_par = reinterpret_cast<uint32_t *>(fa.ws + L.dec_par);
        fd->dec_cbit = reinterpret_cast<uint8_t *>(fa.ws + L.dec_cbit);
    } else if (t == 128) {
        fd->n = fa.n;
        fd->J = a.J;
        fd->C = a.C;
        fd->C4 = (a.C + 3) / 4;
        fd->P = L.P;
        fd->sort_bits = (uint32_t)sort_bits((int)a.J);
        fd->mode = a.mode;
        fd->ste = (a.keep && !s_prev_ok) ? STE_NONE : a.ste;
        fd->bbox_mode = a.bbox_mode;
        fd->tau = a.tau;
        for (int i = 0; i < 3; ++i) fd->bbox_min[i] = a.bbox_min[i];
        fd->cell = a.cell;
        fd->ctrl = ctrl;
        fd->zero_begin = fa.ws + L.zero_off;
        fd->zero_bytes = L.zero_bytes;
        fd->pos = fa.pos;
        fd->attr = fa.attr;
        fd->stream = fa.stream;
        fd->stream_cap = fa.stream_cap;
        fd->coef_f32 = fa.coef_f32;
        fd->codes_out = fa.codes_out;
        fd->perm_out = fa.perm_out;
        fd->voxel_of_out = fa.voxel_of_out;
        if (!a.keep) fd->flags = a.flags;  // (a kept straight-through forward keeps its flags)
        fd->in_stream = fa.in_stream;
        fd->in_bytes = fa.in_bytes;
        fd->pos_out = fa.pos_out;
        fd->vox_out = fa.vox_out;
        fd->attr_out = fa.attr_out;
        fd->info = fa.info;
        fd->codes_in = fa.codes_in;
        fd->aref = fa.aref;
        fd->grad_add = fa.grad_add;
        fd->keys_a = reinterpret_cast<uint64_t *>(fa.ws + L.keys_a);
        fd->keys_b = reinterpret_cast<uint64_t *>(fa.ws + L.keys_b);
        fd->vals_a = reinterpret_cast<uint32_t *>(fa.ws + L.vals_a);
        fd->vals_b = reinterpret_cast<uint32_t *>(fa.ws + L.vals_b);
        fd->leaf = reinterpret_cast<uint64_t *>(fa.ws + L.leaf);
        fd->vh = reinterpret_cast<uint32_t *>(fa.ws + L.vh);
        fd->first = reinterpret_cast<uint32_t *>(fa.ws + L.first);
        fd->bbox_part = reinterpret_cast<uint32_t *>(fa.ws + L.bbox_part);
        fd->lvl_flags = reinterpret_cast<uint32_t *>(fa.ws + L.lvl_flags);
        fd->sort_status = reinterpret_cast<uint32_t *>(fa.ws + L.sort_status);
        fd->sort_hist = reinterpret_cast<uint32_t *>(fa.ws + L.sort_hist);
        fd->dedup_status = reinterpret_cast<uint64_t *>(fa.ws + L.dedup_status);
        fd->occ_status = reinterpret_cast<uint64_t *>(fa.ws + L.occ_status);
        fd->dec_status = reinterpret_cast<uint64_t *>(fa.ws + L.dec_status);
        fd->sort_tiles = L.sort_tiles;
        fd->dedup_tiles = L.dedup_tiles;
        fd->occ_tiles = L.occ_tiles;
        fd->K = L.K;
    }
}

hipError_t launch_setup(const SetupArgs &a, uint32_t blocks, hipStream_t s)
{
    dim3 grid(blocks, a.count);
    hipLaunchKernelGGL(k_setup, grid, dim3(SETUP_THREADS), 0, s, a);
    return hipGetLastError();
}

// One block (one wave) per frame ends the call (finish_frame): used when the call's last launch
// is not a transform launch, which otherwise does it in its last workgroup.
__global__ __launch_bounds__(64) void k_finish(TileMap m)
{
    static_assert(WAVE == 64, "one wave per frame");
    const uint32_t f = blockIdx.x;
    if (f >= m.F) return;
    __shared__ FinishScratch S;
    finish_frame(*cp(m.fd[f]), threadIdx.x, S);
}

hipError_t launch_finish(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish, dim3(m.F), dim3(64), 0, s, m);
    return hipGetLastError();
}

// ========================================================================= bounding box
__device__ inline uint32_t f2ord(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t o)
{
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(u);
}

// The positions are read as one flat array of 3n floats in float4 chunks (chunk q holds the
// coordinates 4q .. 4q+3, whose axes are (q + i) mod 3 since 4 = 1 mod 3), in batches of
// BBOX_CHUNKS chunks: workgroup b of G takes batches b, b + G, ...; each thread issues all of a
// batch's loads at once. A workgroup (BBOX_THREADS threads, all calling) leaves its extrema in
// its own slot, words 0-5, and in word 6 whether it met a coordinate that is not finite: no
// atomics (their same-line updates serialize at the memory side), and no error word, which the
// setup kernel that runs this clears at the same time.
__device__ inline void bbox_partial(const float *pos_, uint32_t n, uint32_t b, uint32_t G, GAS uint32_t *slot)
{
    const uint64_t nf = 3ull * n;         // coordinates
    const uint64_t nq = nf / 4;            // whole float4 chunks
    const uint64_t nbatch = (nq + BBOX_CHUNKS - 1) / BBOX_CHUNKS;
    const GAS float *pos = gp(pos_);
    const bool vec = ((uintptr_t)pos_ & 15u) == 0;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (uint64_t c = b; c < nbatch; c += G) {
        const uint64_t q0 = c * BBOX_CHUNKS + threadIdx.x;
        // the chunk's first axis, (q0 + r * BBOX_THREADS) mod 3 = (q0 mod 3 + r * (BBOX_THREADS mod 3)) mod 3
        const uint32_t a00 = (uint32_t)(q0 % 3u);
        constexpr uint32_t TM3 = (uint32_t)BBOX_THREADS % 3u;
        float4 v[BBOX_F4];
        // the whole batch under one branch each: a per-load condition would wait for each load
        // where its branch joins (clamped indices: every load in bounds, nq >= 1 here)
        if (vec) {
#pragma unroll
            for (int r = 0; r < BBOX_F4; ++r) {
                const uint64_t q = q0 + (uint64_t)r * BBOX_THREADS;
                v[r] = gload4(pos + 4 * (q < nq ? q : nq - 1));
            }
        } else {
#pragma unroll
            for (int r = 0; r < BBOX_F4; ++r) {
                const uint64_t q = q0 + (uint64_t)r * BBOX_THREADS;
                const GAS float *e = pos + 4 * (q < nq ? q : nq - 1);
                v[r] = make_float4(e[0], e[1], e[2], e[3]);
            }
        }
        // axes by selects on compile-time indices: a per-element axis index into mn/mx would
        // move them to memory
#pragma unroll
        for (int r = 0; r < BBOX_F4; ++r) {
            const bool ok = q0 + (uint64_t)r * BBOX_THREADS < nq;
            const uint32_t a0 = (a00 + (uint32_t)r * TM3) % 3u;
            const float e[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bad |= ok && !isfinite(e[i]);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool mine = ok && (a0 + (uint32_t)i) % 3u == (uint32_t)a;
                    mn[a] = fminf(mn[a], mine ? e[i] : INFINITY);
                    mx[a] = fmaxf(mx[a], mine ? e[i] : -INFINITY);
                }
            }
        }
    }
    // the last nf mod 4 coordinates
    if (b == 0 && threadIdx.x < (uint32_t)(nf - 4 * nq)) {
        const uint64_t k = 4 * nq + threadIdx.x;
        const float e = pos[k];
        const uint32_t ak = (uint32_t)(k % 3u);
        bad |= !isfinite(e);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], ak == (uint32_t)a ? e : INFINITY);
            mx[a] = fmaxf(mx[a], ak == (uint32_t)a ? e : -INFINITY);
        }
    }
    // order-preserving uints (so that -0 < +0 as in an ordered comparison), reduced per wave
    // with shuffles, then across the waves in LDS
    constexpr int NW = BBOX_THREADS / WAVE;
    __shared__ uint32_t s_o[NW][7];
    const uint32_t w = threadIdx.x / WAVE;
    {
        const uint64_t bw = __ballot(bad);
        if (lane_id() == 0) s_o[w][6] = bw ? 1u : 0u;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t lo = wave_umin(f2ord(mn[a])), hi = wave_umax(f2ord(mx[a]));
        if (lane_id() == 0) {
            s_o[w][a] = lo;
            s_o[w][3 + a] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const uint32_t j = threadIdx.x;
        uint32_t o = s_o[0][j];
        for (int ww = 1; ww < NW; ++ww) o = j < 3 ? min(o, s_o[ww][j]) : max(o, s_o[ww][j]);  // (flag: max)
        slot[j] = o;
    }
}

// ===================================================== voxelize + Morton + digit histograms
// Voxelization (Sec. 2.1, Sec. 2.2 step (a)): v = min(2^J - 1, floor((p - min) / cell)) per axis
// in FP64 (bounding cube: per-axis minimum, cell = largest extent / 2^J, or 1 when the frame
// has no extent), then the Morton code of (x, y, z). The histograms of every radix digit of
// the codes are accumulated for the sort passes.
constexpr int VOX_THREADS = 512;
constexpr int VOX_PPT = 8;  // few workgroups: each adds its digit histograms into one of the copies
constexpr int VOX_TILE = VOX_THREADS * VOX_PPT;

__global__ __launch_bounds__(VOX_THREADS) void k_voxelize(TileMap m)
{
    const uint32_t f = frame_of(m, blockIdx.x);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    const uint32_t b = blockIdx.x - m.start[f];
    const uint32_t n = fd.n, J = fd.J, P = fd.P, bits = fd.sort_bits, bins = 1u << bits;
    __shared__ uint32_t s_hist[SORT_HIST_WORDS];
    const uint32_t p0 = b * VOX_TILE;
    // Every load is issued before any is used, none under a condition (a loaded value used
    // after a branch joins is waited for there), and before the error word is checked: the
    // thread's point coordinates (clamped indices; with no points, an in-bounds stand-in that is
    // never used), then the bounding-box workgroups' partial extrema (clamped slots; read but
    // unused when the caller gives the cube).
    float c[VOX_PPT][3];
    {
        const GAS float *src = n ? gp(fd.pos) : reinterpret_cast<const GAS float *>(gp(fd.bbox_part));
        const uint32_t ilast = n ? n - 1 : 0u;
#pragma unroll
        for (int r = 0; r < VOX_PPT; ++r) {
            const uint32_t i = min(p0 + r * VOX_THREADS + threadIdx.x, ilast);
#pragma unroll
            for (int a = 0; a < 3; ++a) c[r][a] = src[(size_t)i * 3 + a];
        }
    }
    for (uint32_t i = threadIdx.x; i < P * bins; i += VOX_THREADS) s_hist[i] = 0;
    {   // this workgroup's share of the sort's look-back status words (they lie outside the
        // region the setup kernel zeroes, since only an encode sorts)
        const uint32_t nb = n ? (n + VOX_TILE - 1) / VOX_TILE : 1u;
        const uint64_t nq = (uint64_t)P * (fd.sort_tiles + sort_groups(fd.sort_tiles)) * bins / 4;
        uint4 *z = reinterpret_cast<uint4 *>(fd.sort_status);
        for (uint64_t i = (uint64_t)b * VOX_THREADS + threadIdx.x; i < nq; i += (uint64_t)nb * VOX_THREADS)
            z[i] = make_uint4(0, 0, 0, 0);
    }
    const uint32_t err = load_error(ctrl);
    constexpr int NW = VOX_THREADS / WAVE;
    static_assert(BBOX_GRID_MAX <= 2 * VOX_THREADS, "two bounding-box slots per thread");
    __shared__ uint32_t s_bb[NW][7];
    {
        const uint32_t G = bbox_blocks(n);
        const GAS uint32_t *part = gp(fd.bbox_part);
        uint32_t o[7];  // minima, maxima, and whether a slot met a coordinate that is not finite
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t slot = min(threadIdx.x + h * VOX_THREADS, G - 1);
            const int4 x = gload4i(reinterpret_cast<const GAS int32_t *>(part + (size_t)slot * BBOX_SLOT));
            const uint32_t y0 = part[(size_t)slot * BBOX_SLOT + 4], y1 = part[(size_t)slot * BBOX_SLOT + 5],
                           y2 = part[(size_t)slot * BBOX_SLOT + 6];
            const uint32_t v[7] = {(uint32_t)x.x, (uint32_t)x.y, (uint32_t)x.z, (uint32_t)x.w, y0, y1, y2};
#pragma unroll
            for (int j = 0; j < 7; ++j) o[j] = h == 0 ? v[j] : (j < 3 ? min(o[j], v[j]) : max(o[j], v[j]));
        }
        const uint32_t w = threadIdx.x / WAVE;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const uint32_t r = j < 3 ? wave_umin(o[j]) : wave_umax(o[j]);
            if (lane_id() == 0) s_bb[w][j] = r;
        }
    }
    if (err) return;
    __syncthreads();
    if (fd.bbox_mode == 0) {  // (the slots are written only when the cube is found here)
        uint32_t nonfinite = 0;
        for (int ww = 0; ww < NW; ++ww) nonfinite |= s_bb[ww][6];
        if (nonfinite) {
            if (b == 0 && threadIdx.x == 0) set_error(ctrl, GSC_ERR_INVALID_ARG);
            return;
        }
    }
    double lo[3], cell;
    if (fd.bbox_mode == 0) {
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (n == 0) {
                lo[a] = 0.0;
                continue;
            }
            uint32_t omin = s_bb[0][a], omax = s_bb[0][3 + a];
            for (int ww = 1; ww < NW; ++ww) {
                omin = min(omin, s_bb[ww][a]);
                omax = max(omax, s_bb[ww][3 + a]);
            }
            lo[a] = (double)ord2f(omin);
            const double hi = (double)ord2f(omax);
            ext = fmax(ext, hi - lo[a]);
        }
        cell = ext > 0.0 ? ldexp(ext, -(int)J) : 1.0;
    } else {
        for (int a = 0; a < 3; ++a) lo[a] = fd.bbox_min[a];
        cell = fd.cell;
    }
    if (b == 0 && threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) ctrl->bbox_min[a] = lo[a];
        ctrl->cell = cell;
    }
    const double top = (double)((1u << J) - 1u);
#pragma unroll
    for (int r = 0; r < VOX_PPT; ++r) {
        const uint32_t i = p0 + r * VOX_THREADS + threadIdx.x;
        if (i >= n) continue;
        uint32_t v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double t = floor(__ddiv_rn(__dsub_rn((double)c[r][a], lo[a]), cell));
            t = t < 0.0 ? 0.0 : (t > top ? top : t);
            v[a] = (uint32_t)t;
        }
        const uint64_t key = morton3(v[0], v[1], v[2]);
        gp(fd.keys_a)[i] = key;
        for (uint32_t p = 0; p < P; ++p)
            atomicAdd(&s_hist[p * bins + ((key >> (p * bits)) & (bins - 1))], 1u);
    }
    __syncthreads();
    uint32_t *hist = fd.sort_hist + (size_t)(blockIdx.x % SORT_HIST_COPIES) * P * bins;
    for (uint32_t i = threadIdx.x; i < P * bins; i += VOX_THREADS)
        if (s_hist[i]) atomicAdd(&hist[i], s_hist[i]);
}

hipError_t launch_voxelize(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_voxelize, dim3(m.start[m.F]), dim3(VOX_THREADS), 0, s, m);
    return hipGetLastError();
}
uint32_t voxelize_blocks(uint32_t n) { return n ? ceil_div(n, VOX_TILE) : 1u; }

// ============================================================ one-sweep radix sort pass
// Stable LSD pass over digit `pass` of (key, index) pairs. Each workgroup ranks a tile of
// SORT_THREADS * KPT keys in LDS: wave w owns a contiguous 1/NW of the tile and walks it in order,
// 64 keys at a time; lanes holding the same digit are found with one ballot per digit bit and ranked
// among themselves, so equal digits keep input order. The tile's digit counts are combined
// with its predecessors' through a per-digit decoupled look-back, keys are staged in LDS in
// digit order and written out in runs.
template <int BITS>
__device__ inline uint64_t match_digit(uint32_t d)
{
    uint64_t peers = ~0ull;
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t mm = __ballot(on);
        peers &= on ? mm : ~mm;
    }
    return peers;
}

template <int KPT, int WIN, int BITS>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_pass(TileMap m, int pass)
{
    constexpr int TILE = SORT_THREADS * KPT;
    constexpr int NW = SORT_THREADS / WAVE;
    constexpr int SORT_BINS = 1 << BITS;
    __shared__ uint32_t s_wcnt[NW][SORT_BINS];
    __shared__ uint32_t s_gbase[SORT_BINS];
    __shared__ uint32_t s_lstart[SORT_BINS];
    __shared__ uint32_t s_tmp[2 * NW];
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];

    const uint32_t f = frame_of(m, blockIdx.x);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    const uint32_t n = fd.n;
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    const uint32_t tile = __builtin_amdgcn_readfirstlane(tile_index(m, f));
    const uint32_t base = tile * TILE;
    const GAS uint64_t *kin = gp((pass & 1) ? fd.keys_b : fd.keys_a);
    const GAS uint32_t *vin = gp((pass & 1) ? fd.vals_b : fd.vals_a);
    GAS uint64_t *kout = gp((pass & 1) ? fd.keys_a : fd.keys_b);
    GAS uint32_t *vout = gp((pass & 1) ? fd.vals_a : fd.vals_b);
    const uint32_t shift = (uint32_t)pass * BITS;

    // The tile's keys and indices (clamped slots, so that every load is issued at once; the
    // buffers hold at least one entry) and this thread's digit count of the frame are loaded
    // before the tile's range and the error word are checked.
    static_assert(SORT_THREADS >= SORT_BINS, "one thread per digit");
    static_assert(SORT_LB_GROUP <= (uint32_t)WIN + 1, "a group's earlier tiles fit one look-back window");
    static_assert(SORT_LB_GROUP < 32 && (uint64_t)SORT_LB_GROUP * TILE <= LB32_GSUM, "a group word's arrivals and sum fit");
    const bool dig = tid < (uint32_t)SORT_BINS;
    const uint32_t d = dig ? tid : 0u;
    uint64_t key[KPT];
    uint32_t val[KPT];
    uint32_t rank[KPT];
    const uint32_t wbase = base + w * (KPT * WAVE);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const uint32_t p = min(wbase + j * WAVE + lane, n ? n - 1 : 0u);
        key[j] = kin[p];
        val[j] = pass == 0 ? p : vin[p];
    }
    uint32_t gh = 0;  // the frame's count of digit d: the sum of its histogram copies
#pragma unroll
    for (uint32_t c = 0; c < SORT_HIST_COPIES; ++c) gh += fd.sort_hist[((size_t)c * fd.P + pass) * SORT_BINS + d];
    for (uint32_t i = tid; i < NW * SORT_BINS; i += SORT_THREADS) (&s_wcnt[0][0])[i] = 0;
    if (base >= n || load_error(ctrl)) return;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        if (wbase + j * WAVE + lane >= n) key[j] = ~0ull;  // past the end: ranked last, not written
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const uint32_t dk = (uint32_t)(key[j] >> shift) & (SORT_BINS - 1);
        const uint64_t peers = match_digit<BITS>(dk);
        const uint32_t cnt = s_wcnt[w][dk];
        __builtin_amdgcn_wave_barrier();
        const bool leader = lane == (uint32_t)(__ffsll((long long)peers) - 1);
        if (leader) s_wcnt[w][dk] = cnt + (uint32_t)__popcll(peers);
        rank[j] = cnt + (uint32_t)__popcll(peers & lanemask_lt());
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit (thread d < SORT_BINS holds digit d): wave prefixes, tile count (published at
    // once), digit start in the tile, digit start in the output
    uint32_t *status_d = fd.sort_status + (size_t)pass * fd.sort_tiles * SORT_BINS + d;
    uint32_t *gstatus_d = fd.sort_status + ((size_t)fd.P * fd.sort_tiles + (size_t)pass * sort_groups(fd.sort_tiles)) * SORT_BINS + d;
    uint32_t tile_cnt = 0, hist_excl;
    {
        if (dig) {
            uint32_t run = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = s_wcnt[ww][d];
                s_wcnt[ww][d] = run;
                run += c;
            }
            tile_cnt = run;
            lookback32_publish(status_d, gstatus_d, SORT_BINS, SORT_LB_GROUP, tile, tile_cnt);
        }
        // the exclusive scans of the frame's digit counts and of the tile's, side by side
        const uint32_t vh = dig ? gh : 0u;
        const uint32_t ih = wave_incl_scan(vh), ic = wave_incl_scan(tile_cnt);
        if (lane == WAVE - 1) {
            s_tmp[w] = ih;
            s_tmp[NW + w] = ic;
        }
        __syncthreads();
        if (tid < 2) {
            uint32_t run = 0;
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const uint32_t c = s_tmp[tid * NW + i];
                s_tmp[tid * NW + i] = run;
                run += c;
            }
        }
        __syncthreads();
        hist_excl = s_tmp[w] + ih - vh;
        if (dig) s_lstart[d] = s_tmp[NW + w] + ic - tile_cnt;
    }
    __syncthreads();
    // keys to LDS in tile-local digit order: the keys leave the registers before the look-back,
    // whose window takes their place
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const uint32_t dk = (uint32_t)(key[j] >> shift) & (SORT_BINS - 1);
        const uint32_t q = s_lstart[dk] + s_wcnt[w][dk] + rank[j];
        s_keys[q] = key[j];
        s_vals[q] = val[j];
    }
    if (dig) s_gbase[d] = hist_excl + lookback32_resolve<WIN>(status_d, gstatus_d, SORT_BINS, SORT_LB_GROUP, tile, tile_cnt, ctrl);
    __syncthreads();
    const uint32_t nvalid = min((uint32_t)TILE, n - base);
    for (uint32_t q = tid; q < nvalid; q += SORT_THREADS) {
        const uint64_t k = s_keys[q];
        const uint32_t dk = (uint32_t)(k >> shift) & (SORT_BINS - 1);
        const uint32_t o = s_gbase[dk] + (q - s_lstart[dk]);
        if (o < n) {
            kout[o] = k;
            vout[o] = s_vals[q];
        }
    }
}

template <int BITS>
static hipError_t launch_sort_pass_bits(const TileMap &m, int pass, int variant, hipStream_t s)
{
    const dim3 grid(m.start[m.F]), block(SORT_THREADS);
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_sort_pass<SORT_VARIANT[0].kpt, SORT_VARIANT[0].win, BITS>), grid, block, 0, s, m, pass); break;
    case 1: hipLaunchKernelGGL((k_sort_pass<SORT_VARIANT[1].kpt, SORT_VARIANT[1].win, BITS>), grid, block, 0, s, m, pass); break;
    case 2: hipLaunchKernelGGL((k_sort_pass<SORT_VARIANT[2].kpt, SORT_VARIANT[2].win, BITS>), grid, block, 0, s, m, pass); break;
    case 3: hipLaunchKernelGGL((k_sort_pass<SORT_VARIANT[3].kpt, SORT_VARIANT[3].win, BITS>), grid, block, 0, s, m, pass); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sort_pass(const TileMap &m, int pass, int variant, int bits, hipStream_t s)
{
    if (bits == 9) return launch_sort_pass_bits<9>(m, pass, variant, s);
    if (bits == 8) return launch_sort_pass_bits<8>(m, pass, variant, s);
    return hipErrorInvalidValue;
}

// ================================================================= unique + merge map
// Sorted keys -> occupied voxels: a run of equal keys is one voxel (Alg. 1 step 1, Unique).
// Writes the voxel codes L_J, the first sorted position of every voxel (vh, with vh[Nv] = n)
// and the input row at that position (first),
// Nv, and the histogram of new-node depths D_v (the shallowest octree depth at which voxel v
// starts a node of its own: J - floor(msb(L[v-1] xor L[v]) / 3), and 0 for v = 0), from which
// every level size follows: |L_d| = #{v : D_v <= d}.
__global__ __launch_bounds__(DEDUP_THREADS) void k_dedup(TileMap m)
{
    constexpr int NW = DEDUP_THREADS / WAVE;
    static_assert(DEDUP_KPT * NW == WAVE, "one wave scans the (row, wave) head counts");
    __shared__ uint64_t s_k[DEDUP_TILE + 1];   // s_k[1 + i] = key base + i; s_k[0] = key base - 1
    __shared__ uint32_t s_cnt[DEDUP_KPT * NW + 1];
    __shared__ uint32_t s_hist[32];
    const uint32_t f = frame_of(m, blockIdx.x);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    const uint32_t n = fd.n, J = fd.J;
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    const uint32_t tile = __builtin_amdgcn_readfirstlane(tile_index(m, f));
    const uint32_t base = tile * DEDUP_TILE;
    const GAS uint64_t *K = gp((fd.P & 1) ? fd.keys_b : fd.keys_a);  // output of the last sort pass
    const GAS uint32_t *V = gp((fd.P & 1) ? fd.vals_b : fd.vals_a);
    // striped (coalesced) loads: position i = r * DEDUP_THREADS + tid; the sorted input rows
    // are kept for the voxels' first members. They are issued at clamped positions (the buffers
    // hold at least one entry) before the tile's range and the error word are checked.
    const uint32_t last = n ? n - 1 : 0u;
    uint64_t kv[DEDUP_KPT];
    uint32_t pv[DEDUP_KPT];
#pragma unroll
    for (int r = 0; r < DEDUP_KPT; ++r) {
        const uint32_t i = min(base + r * DEDUP_THREADS + tid, last);
        kv[r] = K[i];
        pv[r] = V[i];
    }
    const uint64_t kprev = K[base > 0 ? min(base - 1, last) : 0u];
    if (tid < 32) s_hist[tid] = 0;
    if (base >= n || load_error(ctrl)) return;
    const uint32_t len = min((uint32_t)DEDUP_TILE, n - base);
#pragma unroll
    for (int r = 0; r < DEDUP_KPT; ++r) s_k[1 + r * DEDUP_THREADS + tid] = kv[r];
    if (tid == 0) s_k[0] = base > 0 ? kprev : 0ull;
    __syncthreads();
    // heads: a position starts a voxel when its key differs from the previous one
    uint32_t hbits = 0;
#pragma unroll
    for (int r = 0; r < DEDUP_KPT; ++r) {
        const uint32_t i = r * DEDUP_THREADS + tid;
        const uint64_t k = s_k[1 + i], pk = s_k[i];
        const bool first = base + i == 0;
        const bool h = i < len && (first || k != pk);
        if (h) {
            hbits |= 1u << r;
            const uint32_t D = first ? 0u : J - (uint32_t)msb64(pk ^ k) / 3u;
            atomicAdd(&s_hist[D], 1u);
        }
        const uint64_t bal = __ballot(h);
        if (lane == 0) s_cnt[r * NW + w] = (uint32_t)__popcll(bal);
    }
    __syncthreads();
    if (w == 0) {  // (row, wave) counts in position order -> exclusive offsets
        const uint32_t c = s_cnt[lane];
        const uint32_t inc = wave_incl_scan(c);
        s_cnt[lane] = inc - c;
        if (lane == WAVE - 1) s_cnt[WAVE] = inc;
    }
    __syncthreads();
    const uint32_t tile_total = s_cnt[WAVE];
    __shared__ LbScratch<DEDUP_THREADS / WAVE> s_lb;
    const uint32_t vbase = (uint32_t)lookback_block<OpSum, DEDUP_THREADS>(fd.dedup_status, 1, tile, tile_total, ctrl, s_lb);
#pragma unroll
    for (int r = 0; r < DEDUP_KPT; ++r) {
        const bool h = (hbits >> r) & 1u;
        const uint64_t bal = __ballot(h);
        if (h) {
            const uint32_t i = r * DEDUP_THREADS + tid;
            const uint32_t v = vbase + s_cnt[r * NW + w] + (uint32_t)__popcll(bal & lanemask_lt());
            if (v < n) {
                const uint64_t k = s_k[1 + i];
                gp(fd.leaf)[v] = k;
                if (fd.codes_out) gp(fd.codes_out)[v] = k;
                gp(fd.vh)[v] = base + i;
                gp(fd.first)[v] = pv[r];
            }
        }
    }
    if (fd.perm_out || fd.voxel_of_out) {
        // optional maps: the sorted order (sorted position -> input row) and, for every input
        // row, its voxel = the heads up to and including its sorted position, minus one
        GAS uint32_t *perm = gp(fd.perm_out), *vof = gp(fd.voxel_of_out);
#pragma unroll
        for (int r = 0; r < DEDUP_KPT; ++r) {
            const uint32_t i = r * DEDUP_THREADS + tid;
            const uint64_t bal = __ballot((hbits >> r) & 1u);
            if (i < len) {
                const uint32_t v = vbase + s_cnt[r * NW + w] + (uint32_t)__popcll(bal & (lanemask_lt() | (1ull << lane))) - 1u;
                if (perm) perm[base + i] = pv[r];
                if (vof && pv[r] < n) vof[pv[r]] = v;
            }
        }
    }
    if (tid < 32 && s_hist[tid]) atomicAdd(&ctrl->hist_D[tid], s_hist[tid]);
    if (tid == 0 && base + DEDUP_TILE >= n) {
        const uint32_t nv = vbase + tile_total;
        ctrl->n_vox = nv;
        fd.vh[nv] = n;
    }
}

hipError_t launch_dedup(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_dedup, dim3(m.start[m.F]), dim3(DEDUP_THREADS), 0, s, m);
    return hipGetLastError();
}

// ======================================================================== occupancy
// All occupancy bytes (Sec. 2.2 "Bitstream generation", Alg. 1 OccKernel) in one pass over the
// sorted voxel codes. Voxel v is the first leaf of its depth-d node exactly when D_v <= d; the
// byte of such a node collects bit ((L[u] >> 3(J-d-1)) & 7) of every voxel u of the node with
// D_u <= d+1 (the first leaves of its children). A tile of voxels ORs these bits in LDS per
// depth; the byte of a node that straddles tile boundaries is finished by the tile holding the
// next node's head, which learns the node's partial byte (and the node's rank) from a
// per-depth decoupled look-back over (head count, open byte).
__global__ __launch_bounds__(OCC_THREADS) void k_occupancy(TileMap m)
{
    __shared__ uint64_t s_code[OCC_TILE + 1];
    __shared__ uint32_t s_bytes[GSC_MAX_DEPTH][OCC_TILE / 4];
    __shared__ uint32_t s_carry[GSC_MAX_DEPTH];
    __shared__ uint32_t s_cnt[GSC_MAX_DEPTH];
    __shared__ uint64_t s_pref[GSC_MAX_DEPTH];
    __shared__ uint32_t s_tmp[OCC_THREADS / WAVE + 1];

    const uint32_t f = frame_of(m, blockIdx.x);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    const uint32_t J = fd.J;
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = __builtin_amdgcn_readfirstlane(tile_index(m, f));
    const uint32_t s = tile * OCC_TILE;
    // s_code[j] = L[s - 1 + j]: loaded at positions clamped to the buffer (it holds at least one
    // entry), together with the voxel count and the error word, before any of them is used
    const GAS uint64_t *leaf = gp(fd.leaf);
    constexpr int OCC_LPT = (OCC_TILE + 1 + OCC_THREADS - 1) / OCC_THREADS;
    const uint32_t lmax = fd.n ? fd.n - 1 : 0u;
    uint64_t lc[OCC_LPT];
#pragma unroll
    for (int r = 0; r < OCC_LPT; ++r) {
        const uint32_t j = min(tid + r * OCC_THREADS, (uint32_t)OCC_TILE);  // (entries past the tile: one line)
        lc[r] = leaf[min(s + j > 0 ? s + j - 1 : 0u, lmax)];
    }
    const uint32_t nv = ctrl->n_vox;
    for (uint32_t i = tid; i < GSC_MAX_DEPTH * (OCC_TILE / 4); i += OCC_THREADS)
        (&s_bytes[0][0])[i] = 0;
    if (tid < GSC_MAX_DEPTH) s_carry[tid] = 0;
    if (s >= nv || load_error(ctrl)) return;
    const uint32_t e = min(nv, s + OCC_TILE);
#pragma unroll
    for (int r = 0; r < OCC_LPT; ++r) {
        const uint32_t j = tid + r * OCC_THREADS;
        if (j < e - s + 1) s_code[j] = s + j >= 1 ? lc[r] : 0ull;
    }
    __syncthreads();

    uint32_t Dv[OCC_VPT];
    uint64_t cv[OCC_VPT];
#pragma unroll
    for (int i = 0; i < OCC_VPT; ++i) {
        const uint32_t v = s + tid * OCC_VPT + i;
        const uint32_t j = v - s + 1;
        if (v < e) {
            cv[i] = s_code[j];
            Dv[i] = v == 0 ? 0u : J - (uint32_t)msb64(s_code[j - 1] ^ cv[i]) / 3u;
        } else {
            cv[i] = 0;
            Dv[i] = 0xFFFFu;  // not a voxel: never a head, never contributes
        }
    }
    // The heads of every depth ranked at once. Voxel j = 2 t + i of the tile (thread t, slot i) is
    // a head at depth d when Dv <= d; its node's byte is number H - 1 of the tile at that depth,
    // H counting the heads up to and including it. Per wave, five ballots per slot give the bit
    // planes of the voxels' head depths (a non-voxel counts as depth 31, never a head); lane d
    // compares them with d (most significant bit first) into the wave's head masks of depth d
    // and stores their count, so one barrier and a prefix over the 16 waves replace a block scan
    // per depth.
    static_assert(OCC_VPT == 2 && GSC_MAX_DEPTH < 31 && GSC_MAX_DEPTH <= WAVE, "two slots, five planes");
    __shared__ uint32_t s_wcnt[GSC_MAX_DEPTH][OCC_THREADS / WAVE];
    const uint32_t lane = lane_id(), wv = tid / WAVE;
    uint64_t le[OCC_VPT];  // lane d < J: the wave's voxels of slot i that are heads at depth d
#pragma unroll
    for (int i = 0; i < OCC_VPT; ++i) {
        const uint32_t dv = min(Dv[i], 31u);
        uint64_t plane[5];
#pragma unroll
        for (int bit = 0; bit < 5; ++bit) plane[bit] = __ballot((dv >> bit) & 1u);
        uint64_t above = 0, same = ~0ull;  // voxels deeper than lane's d; equal so far
#pragma unroll
        for (int bit = 4; bit >= 0; --bit) {
            const uint64_t qm = ((lane >> bit) & 1u) ? ~0ull : 0ull;
            above |= same & plane[bit] & ~qm;
            same &= ~(plane[bit] ^ qm);
        }
        le[i] = ~above;
    }
    if (lane < J) s_wcnt[lane][wv] = (uint32_t)(__popcll(le[0]) + __popcll(le[1]));
    __syncthreads();
    uint32_t pre = 0, total = 0;  // lane d < J: heads of depth d in the waves before / in the tile
    if (lane < J) {
        for (uint32_t w2 = 0; w2 < OCC_THREADS / WAVE; ++w2) {
            const uint32_t c = s_wcnt[lane][w2];
            pre += w2 < wv ? c : 0u;
            total += c;
        }
        if (wv == 0) s_cnt[lane] = total;
    }
    const uint64_t lt = lanemask_lt(), me = 1ull << lane;
    for (uint32_t d = 0; d < J; ++d) {
        // (readlane returns an int: each half goes through uint32_t, so the low one is not
        // sign-extended into the high one)
        auto lane64 = [d](uint64_t v) -> uint64_t {
            return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)v, d) |
                   ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), d) << 32);
        };
        const uint64_t m0 = lane64(le[0]), m1 = lane64(le[1]);
        const uint32_t p = __builtin_amdgcn_readlane(pre, d);
        uint32_t run = p + (uint32_t)__popcll(m0 & lt) + (uint32_t)__popcll(m1 & lt);
        const uint32_t sh = 3u * (J - d - 1u);
#pragma unroll
        for (int i = 0; i < OCC_VPT; ++i) {
            run += ((i == 0 ? m0 : m1) & me) ? 1u : 0u;
            if (Dv[i] <= d + 1u) {
                const uint32_t bit = 1u << (uint32_t)((cv[i] >> sh) & 7u);
                if (run == 0) {
                    atomicOr(&s_carry[d], bit);
                } else {
                    const uint32_t k = run - 1u;
                    atomicOr(&s_bytes[d][k >> 2], bit << (8u * (k & 3u)));
                }
            }
        }
    }
    __syncthreads();
    // the stream geometry, by the last wave beside the look-backs (it depends only on the depth
    // histogram): |L_d| = hist_D[0] + ... + hist_D[d], level d's bytes start at the header size
    // plus |L_0| + ... + |L_{d-1}|; s_off[J] is the end of the occupancy bytes
    __shared__ uint64_t s_off[GSC_MAX_DEPTH + 1];
    __shared__ int s_fits;
    if (tid / WAVE == OCC_THREADS / WAVE - 1) {
        const uint32_t lane = lane_id();
        const uint32_t hd = lane <= J ? cp(ctrl)->hist_D[lane] : 0u;  // (written by the dedup kernel)
        const uint64_t size = lane < J ? (uint64_t)wave_incl_scan(hd) : 0ull;
        uint64_t incl = size;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint64_t t = __shfl_up(incl, o, WAVE);
            if (lane >= (uint32_t)o) incl += t;
        }
        const uint64_t off = GSC_HEADER_BYTES + incl - size;
        if (lane <= J) s_off[lane] = off;
        if (lane == J) {
            const uint64_t total = align_up(off, 256) + (uint64_t)cp(ctrl)->n_vox * fd.C * 4;
            s_fits = total <= fd.stream_cap;
            if (!s_fits) set_error(ctrl, GSC_ERR_CAPACITY);
        }
    }
    // one wave per depth (wave w takes depths w, w + 16, ...): the look-backs of all depths
    // proceed side by side
    for (uint32_t d = tid / WAVE; d < J; d += OCC_THREADS / WAVE) {
        const uint32_t cnt = s_cnt[d];
        const uint32_t byte = cnt ? (s_bytes[d][(cnt - 1) >> 2] >> (8u * ((cnt - 1) & 3u))) & 0xFFu
                                  : s_carry[d];
        const uint64_t agg = ((uint64_t)cnt << 8) | byte;
        // status words depth-major (depth d's words of consecutive tiles are adjacent: a round of
        // the wave's look-back reads 64 of them in four cache lines, not one line per tile)
        const uint64_t pref = lookback_wave<OpSegOr>(fd.occ_status + (size_t)d * fd.occ_tiles, 1, tile, agg, ctrl);
        if (lane_id() == 0) s_pref[d] = pref;
    }
    __syncthreads();
    if (!s_fits) return;
    const bool last = (e == nv);
    GAS uint8_t *out = gp(fd.stream);
    for (uint32_t d = 0; d < J; ++d) {
        const uint64_t pref = s_pref[d];
        const uint32_t pc = (uint32_t)(pref >> 8), por = (uint32_t)(pref & 0xFF);
        const uint32_t cnt = s_cnt[d];
        const uint64_t off = s_off[d];
        const uint32_t nw = cnt ? (last ? cnt : cnt - 1u) : 0u;
        const uint64_t lim = s_off[d + 1 < J ? d + 1 : J];  // end of level d's bytes
        for (uint32_t k = tid; k < nw; k += OCC_THREADS)
            if (off + pc + k < lim)
                out[off + pc + k] = (uint8_t)((s_bytes[d][k >> 2] >> (8u * (k & 3u))) & 0xFFu);
        if (tid == 0 && pc > 0 && (cnt > 0 || last) && off + pc - 1 < lim)
            out[off + pc - 1] = (uint8_t)(por | s_carry[d]);
    }
}

hipError_t launch_occupancy(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_occupancy, dim3(m.start[m.F]), dim3(OCC_THREADS), 0, s, m);
    return hipGetLastError();
}

// ===================================================================== octree decoding
// Decoding (Sec. 2.3, Alg. 2-3): L_0 = [0]; level d's |L_d| bytes give each parent's child
// count (population count), an exclusive prefix sum gives each parent's first child slot, and
// every parent writes (p << 3) + i for each set bit i in ascending order. The leaves are then
// turned back into voxel coordinates and voxel centres.
//
// Every level's bytes are in the stream from the start, so the decoder does not go level by
// level. Numbering the nodes of levels 1..J one after the other (level L's from
// Q(L) = |L_1| + ... + |L_{L-1}|), the first child of the node whose byte is the q-th byte of the
// stream is node P(q), the number of set bits in the bytes before it: one prefix sum over all
// bytes places every child. `k_dec_expand` writes for every node its parent's index in the
// parent's level and its child bit i (its code is the parent's code times 8 plus i);
// `k_dec_prelude` then builds each leaf's code from the child bits along its path to the root,
// most significant first, which is the code the level-by-level expansion produces.

// Header checks: everything the decoder relies on must be self-consistent and fit the caller's
// buffers. Performed by one wave, lane l checking level l's size against the next one and the
// quantizer step of channel l; returns true (in every lane) when the header is usable.
template <class FD>
__device__ inline bool header_ok_wave(FD &fd, const CAS gsc_header *h)
{
    const uint32_t lane = lane_id();
    if (fd.in_bytes < GSC_HEADER_BYTES) return false;
    if (h->magic != GSC_MAGIC || h->version != GSC_VERSION) return false;
    if (h->J != fd.J || h->C != fd.C || h->error != 0) return false;
    const uint32_t J = fd.J, C = fd.C, nv = h->n_vox;
    if (nv > fd.n) return false;
    if (h->level_sizes[J] != nv) return false;
    if (h->level_sizes[0] != (nv > 0 ? 1u : 0u)) return false;
    if (!(h->cell > 0.0)) return false;
    bool bad = false;
    uint64_t a = 0;
    if (lane < J) {
        a = h->level_sizes[lane];
        const uint64_t b = h->level_sizes[lane + 1];
        bad = b < a || b > 8 * a;
    }
    if (lane < C) {
        const float st = h->quant_step[lane];
        bad = bad || !(st > 0.0f) || !isfinite(st);
    }
    uint64_t occ = a;  // the occupancy bytes: sizes of levels 0..J-1
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) occ += __shfl_xor(occ, o, WAVE);
    if (__ballot(bad) != 0ull) return false;
    if (h->occ_offset != GSC_HEADER_BYTES || h->occ_bytes != occ) return false;
    const uint64_t co = align_up(GSC_HEADER_BYTES + occ, 256);
    if (h->coef_offset != co || h->coef_bytes != (uint64_t)nv * C * 4) return false;
    if (h->total_bytes != co + h->coef_bytes || h->total_bytes > fd.in_bytes) return false;
    return true;
}

// The level of the q-th occupancy byte and that level's first byte: levels are contiguous, so a
// scan over the (at most 21) level starts from the previous answer finds it.
struct LevelCursor {
    uint32_t d, start, end;  // level, its first byte, one past its last byte
};
__device__ inline void level_seek(const CAS gsc_header *h, uint32_t J, uint64_t q, LevelCursor &lc)
{
    while (lc.d + 1 < J && q >= lc.end) {
        ++lc.d;
        lc.start = lc.end;
        lc.end += h->level_sizes[lc.d];
    }
}

// One pass over all occupancy bytes: tile t holds bytes [t DEC_TILE, (t + 1) DEC_TILE) of the
// stream's occupancy section, striped (byte s + r DEC_THREADS + tid), and finds each byte's
// child slots with a decoupled look-back over the tiles' set-bit counts. Checks: no byte is 0,
// and the first byte of every level is the parent of the first node of the next level (its prefix
// equals Q(d + 1)), and the bytes hold exactly |L_1| + ... + |L_J| set bits.
__global__ __launch_bounds__(DEC_THREADS) void k_dec_expand(TileMap m)
{
    constexpr int NW = DEC_THREADS / WAVE;
    static_assert(DEC_PPT * NW <= WAVE, "one wave scans the (row, wave) child counts");
    __shared__ uint32_t s_cnt[WAVE + 1];
    __shared__ LbScratch<DEC_THREADS / WAVE> s_lb;
    const uint32_t f = frame_of(m, blockIdx.x);
    const CAS FrameDesc &fd = *cp(m.fd[f]);  // (not written while the kernel runs)
    Ctrl *ctrl = fd.ctrl;
    const uint32_t tile = tile_index(m, f), tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    const gsc_header *hg = reinterpret_cast<const gsc_header *>(fd.in_stream);
    const CAS gsc_header *h = cp(hg);  // (the stream is not written while it is decoded)
    // The tile's bytes are loaded before the header is checked, at positions clamped to the
    // caller's stream (a checked header's occupancy bytes lie inside it, so the clamp changes no
    // byte that is used); a stream shorter than the header fails the check and loads nothing.
    const uint64_t s = (uint64_t)tile * DEC_TILE;
    const GAS uint8_t *occ = gp(fd.in_stream + GSC_HEADER_BYTES);
    uint32_t raw[DEC_PPT];
    if (fd.in_bytes > GSC_HEADER_BYTES) {
        const uint64_t qmax = fd.in_bytes - GSC_HEADER_BYTES - 1;
#pragma unroll
        for (int r = 0; r < DEC_PPT; ++r) raw[r] = occ[min(s + r * DEC_THREADS + tid, qmax)];
    } else {
#pragma unroll
        for (int r = 0; r < DEC_PPT; ++r) raw[r] = 0u;
    }
    __shared__ int s_ok;
    if (w == 0) {
        const bool ok = header_ok_wave(fd, h);
        if (lane == 0) s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    if (!s_ok) {
        if (tile == 0 && tid == 0) set_error(ctrl, GSC_ERR_CORRUPT_STREAM);
        return;
    }
    const uint32_t J = fd.J, nv = h->n_vox;
    const uint64_t B = h->occ_bytes;
    if (tile == 0 && tid == 0) {
        ctrl->n_vox = nv;
        for (uint32_t d = 0; d <= J; ++d) ctrl->level_sizes[d] = h->level_sizes[d];
    }
    if (s >= B) return;
    uint64_t total_nodes = 0;  // |L_1| + ... + |L_J|
    for (uint32_t d = 1; d <= J; ++d) total_nodes += h->level_sizes[d];
    uint32_t bytes[DEC_PPT], wex[DEC_PPT];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < DEC_PPT; ++r) {
        const uint64_t q = s + r * DEC_THREADS + tid;
        bytes[r] = q < B ? raw[r] : 0u;
    }
#pragma unroll
    for (int r = 0; r < DEC_PPT; ++r) {
        const uint64_t q = s + r * DEC_THREADS + tid;
        if (q < B && bytes[r] == 0) bad = true;
        const uint32_t c = (uint32_t)__popc(bytes[r]);
        const uint32_t inc = wave_incl_scan(c);
        wex[r] = inc - c;
        if (lane == WAVE - 1) s_cnt[r * NW + w] = inc;
    }
    __syncthreads();
    if (w == 0) {  // (row, wave) totals in byte order -> exclusive offsets
        const uint32_t c = lane < (uint32_t)(DEC_PPT * NW) ? s_cnt[lane] : 0u;
        const uint32_t inc = wave_incl_scan(c);
        if (lane < (uint32_t)(DEC_PPT * NW)) s_cnt[lane] = inc - c;
        if (lane == WAVE - 1) s_cnt[WAVE] = inc;
    }
    __syncthreads();
    const uint32_t total = s_cnt[WAVE];
    const uint64_t base = lookback_block<OpSum, DEC_THREADS>(fd.dec_status, 1, tile, total, ctrl, s_lb);
    GAS uint32_t *par = gp(fd.dec_par);
    GAS uint8_t *cbit = gp(fd.dec_cbit);
    LevelCursor lc;
    lc.d = 0;
    lc.start = 0;
    lc.end = h->level_sizes[0];
    uint64_t q_level_next = 0;  // Q(d + 1) of the cursor's level d: nodes of levels 1..d
    uint32_t qd = 0;
#pragma unroll
    for (int r = 0; r < DEC_PPT; ++r) {
        const uint64_t q = s + r * DEC_THREADS + tid;
        if (q >= B) break;
        level_seek(h, J, q, lc);
        while (qd < lc.d) q_level_next += h->level_sizes[++qd];
        const uint64_t P = base + s_cnt[r * NW + w] + wex[r];  // set bits before byte q
        if (q == lc.start && P != q_level_next) bad = true;    // the level's first child
        if (q + 1 == B && P + (uint64_t)__popc(bytes[r]) != total_nodes) bad = true;
        const uint32_t p = (uint32_t)(q - lc.start);            // the parent's index in its level
        // the byte's children, set bits only (a wave takes as many steps as its fullest byte
        // has children, mostly one or two below the top levels, instead of eight)
        uint64_t c = P;
        for (uint32_t bits = bytes[r]; bits; bits &= bits - 1u) {
            const uint32_t i = (uint32_t)__ffs(bits) - 1u;
            if (c < total_nodes) {
                par[c] = p;
                cbit[c] = (uint8_t)i;
            } else {
                bad = true;
            }
            ++c;
        }
    }
    if (bad) set_error(ctrl, GSC_ERR_CORRUPT_STREAM);
}

hipError_t launch_dec_expand(const TileMap &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_expand, dim3(m.start[m.F]), dim3(DEC_THREADS), 0, s, m);
    return hipGetLastError();
}


}  // namespace gsc
