// Internal definitions shared by the host side and the kernels of libgsc: tile sizes, the
// per-call control block that lives at the start of every workspace, the per-frame descriptor
// the kernels read, and the workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gsc.h"

namespace gsc {

// ---------------------------------------------------------------------------- tile sizes
constexpr int WAVE = 64;

// Radix digits of 8 bits, or of 9 bits when that saves a pass over the 3J-bit codes (J = 3, 6,
// 9, 11, 12, 14, 15, 17, 18, 20, 21): 36-bit codes at J = 12 take four passes instead of five.
constexpr int SORT_BITS_MAX = 9;
constexpr int SORT_BINS_MAX = 1 << SORT_BITS_MAX;
constexpr int SORT_THREADS = 512;       // 8 waves; thread d < 2^bits also holds digit d
// Tiling variants of a sort pass (keys per thread, look-back window), chosen per call by the
// autotuner's table; the workspace is laid out for the smallest tile.
struct SortVariant {
    int kpt, win;
};
constexpr int SORT_VARIANTS = GSC_SORT_VARIANTS;
constexpr SortVariant SORT_VARIANT[SORT_VARIANTS] = {{8, 16}, {4, 16}, {12, 16}, {8, 64}};
// untuned tiling: 2048-key tiles for frames of at most 2^18 Gaussians (more workgroups for a
// small sort), 4096-key tiles above
constexpr int SORT_DEFAULT_VARIANT = 0;
constexpr int SORT_SMALL_VARIANT = 1;
constexpr uint64_t SORT_SMALL_MAX = 1ull << 18;
inline int sort_default_variant(uint64_t n) { return n <= SORT_SMALL_MAX ? SORT_SMALL_VARIANT : SORT_DEFAULT_VARIANT; }
constexpr int SORT_KPT_MIN = 4;
__host__ __device__ constexpr int sort_tile(int variant) { return SORT_THREADS * SORT_VARIANT[variant].kpt; }
// tiles per look-back group: a pass's status words are P x tiles x 2^bits tile words followed by
// P x groups x 2^bits group words
constexpr uint32_t SORT_LB_GROUP = 16;
__host__ __device__ constexpr uint32_t sort_groups(uint32_t tiles) { return (tiles + SORT_LB_GROUP - 1) / SORT_LB_GROUP; }
// histogram words of all passes: at most 8 passes of 256 digits or 7 of 512 (63-bit codes)
constexpr int SORT_HIST_WORDS = 7 * 512;
// copies of the digit histograms: the voxelize workgroup b adds into copy b mod 8 (245 device-scope
// additions per word at 1M in one copy serialize), and a sort pass sums a digit's copies
constexpr uint32_t SORT_HIST_COPIES = 8;

constexpr int DEDUP_THREADS = 512;
constexpr int DEDUP_KPT = 8;
constexpr int DEDUP_TILE = DEDUP_THREADS * DEDUP_KPT;

constexpr int OCC_THREADS = 1024;        // 16 waves: the per-depth look-backs run side by side
constexpr int OCC_VPT = 2;              // voxels per thread
constexpr int OCC_TILE = OCC_THREADS * OCC_VPT;

constexpr int DEC_THREADS = 256;
constexpr int DEC_PPT = 16;             // occupancy bytes per thread
constexpr int DEC_TILE = DEC_THREADS * DEC_PPT;

constexpr int RT = 512;                 // RAHT tile: entries (eight 64-entry wave chunks)
constexpr int RAHT_THREADS = 512;       // one wave per chunk
constexpr int OPEN_CAP = 128;           // >= 6J + 2 open entries per tile for J <= 21
constexpr int NLVL = 64;                // binary levels 1..63 fit in a 64-bit mask
constexpr uint8_t LVL_NONE = 127;       // level of entry 0: it never merges as a right sibling
constexpr int MAXK = 24;                // RAHT tiling levels (sequences S_1 .. S_MAXK)
constexpr int NCLS = RT / 64 + 1;       // merge classes: local to one wave chunk, or crossing
constexpr int SEG_N = NLVL * NCLS + 1;  // per-tile (level, class) segment starts + total
constexpr int LSTART_N = SEG_N + 1;     // padded to an even count of u16

// Upper tiling levels (k >= 2) run as one persistent launch per phase (schedules, forward,
// inverse) of at most UP_GRID_MAX workgroups, which order the levels through per-workgroup
// phase flags.
constexpr uint32_t UP_GRID_MAX = 1024;
constexpr uint32_t PHASE_PRELUDE = 0;  // flag base of the schedule launch
// Counters of the transform launches, in DONE_WORDS words after the flags, zeroed by every
// call: the finished items of every tiling level (forward: DONE_FWD + k, inverse: DONE_INV + k),
// the upper items' tickets of the forward (TK_UPF), the workgroups done with the upper levels'
// schedules (PRE_DONE), and the workgroups that have ended the first-level forward and inverse
// launches (FIN_FWD, FIN_INV).
constexpr uint32_t DONE_WORDS = 128, DONE_FWD = 0, DONE_INV = 32, TK_UPF = 80, PRE_DONE = 81, FIN_FWD = 82,
                   FIN_INV = 83;
static_assert(MAXK + 1 <= 32, "one completion counter per tiling level and direction");

// Bounding box: at most BBOX_GRID_MAX workgroups per frame (blocks 1.. of the setup launch),
// each leaving its partial minima and maxima (order-preserving uints of the floats) and a
// non-finite flag in a slot of BBOX_SLOT words, which the voxelize workgroups combine.
constexpr int BBOX_THREADS = 512;
constexpr int BBOX_F4 = 8;              // float4 chunks per thread and batch, loaded at once
constexpr uint32_t BBOX_CHUNKS = BBOX_THREADS * BBOX_F4;  // float4 chunks per batch
constexpr uint32_t BBOX_GRID_MAX = 512;
constexpr uint32_t BBOX_SLOT = 8;       // min x,y,z, max x,y,z, a coordinate not finite, 1 unused
__host__ __device__ inline uint32_t bbox_blocks(uint32_t n)
{
    if (n == 0) return 1u;
    const uint64_t batches = ((3ull * n + 3) / 4 + BBOX_CHUNKS - 1) / BBOX_CHUNKS;
    return batches < BBOX_GRID_MAX ? (uint32_t)batches : BBOX_GRID_MAX;
}

// --------------------------------------------------------------- per-call control block
// Zero-initialised by the first kernel of every call.
struct Ctrl {
    uint32_t error;              // first device error (gsc_status), 0 = ok
    uint32_t n_vox;              // Nv
    uint32_t dec_unused;
    uint32_t n_in;
    uint32_t reserved[102];
    uint32_t hist_D[32];         // voxels whose new-node depth is D, D = 0..J
    uint32_t lvl_n[MAXK + 2];    // sizes of the RAHT entry sequences, index k = 1..MAXK+1
    uint32_t level_sizes[32];    // |L_d|
    uint64_t occ_off[32];        // stream offset of level d's occupancy bytes
    uint64_t occ_bytes, coef_offset, total_bytes;
    double bbox_min[3];
    double cell;
};
constexpr size_t CTRL_BYTES = 16384;
static_assert(sizeof(Ctrl) <= CTRL_BYTES, "control block too large");


// ------------------------------------------------------------- kernel-side frame view
enum : uint32_t {
    MODE_ENCODE = 0,    // gather + average input rows, quantize coefficients into the stream
    MODE_DECODE = 1,    // dequantize from the stream, write output rows
    MODE_FWD_F32 = 2,   // float rows in, float coefficients out
    MODE_ADJ_F32 = 3,   // float coefficients in, float rows out
    MODE_STE_BWD = 4,   // gradient of the straight-through coder: float coefficient rows in,
                        // inverse transform, plus a voxel-row term, scattered to the Gaussians
};

// Straight-through coding: an encode that also writes the voxel means and the dequantized
// coefficients, then synthesizes the decoded rows with the same schedule.
enum : uint32_t { STE_NONE = 0, STE_FORWARD = 1 };

struct RahtLevel {
    uint32_t *s_idx;     // k >= 2: voxel index of each entry of S_k
    uint8_t *s_lvl;      // k >= 2: binary level of each entry
    uint32_t *rec;       // per tile: RT merge records, sorted by level
    uint16_t *lstart;    // per tile: LSTART_N starts of the (level, class) record segments
    uint64_t *lmask;     // per tile: NCLS masks, bit x of mask c set when segment (x, c) is non-empty
    uint16_t *opos;      // per tile: OPEN_CAP positions of open entries
    uint32_t *obase;     // per tile: index in S_{k+1} of its first open entry
    uint32_t *ocnt;      // per tile: open entries
    uint64_t *status;    // per tile: lookback status of the open-entry compaction
    float *vbuf;         // rows (C4 float4 each) of the entries of S_{k+1}
    uint32_t tiles;      // worst-case tiles of this level
    uint32_t cap;        // worst-case entries of S_k
};

struct FrameDesc {
    // shape and coding parameters
    uint32_t n;          // encode: Gaussians; decode / transform: voxel capacity
    uint32_t J, C, C4, P;   // depth, channels, channels/4 rounded up, sort passes
    uint32_t mode;
    uint32_t ste;        // STE_FORWARD: the workspace holds (or is building) a straight-through forward
    uint32_t bbox_mode;
    float tau;
    double bbox_min[3];
    double cell;
    float step[GSC_MAX_CHANNELS];
    float inv_step[GSC_MAX_CHANNELS];
    uint64_t pow2_steps;     // bit c set: step[c] is a power of two
    // workspace
    Ctrl *ctrl;
    uint8_t *zero_begin;
    uint64_t zero_bytes;
    // encode
    const float *pos;
    const float *attr;       // also MODE_FWD_F32 / MODE_ADJ_F32 input rows
    uint8_t *stream;
    uint64_t stream_cap;
    float *coef_f32;         // optional unquantized coefficients / transform output rows
    uint64_t *codes_out;     // optional leaf codes
    uint32_t *perm_out;      // optional stable sorted order of the Gaussians
    uint32_t *voxel_of_out;  // optional voxel of every Gaussian
    uint32_t flags;          // GSC_FLAG_* of the call (decode: taken from the stream header)
    // decode
    const uint8_t *in_stream;
    uint64_t in_bytes;
    float *pos_out;
    uint32_t *vox_out;
    float *attr_out;
    int32_t *info;           // device info words
    const uint64_t *codes_in;   // MODE_FWD_F32 / MODE_ADJ_F32: leaf codes
    float *aref;                // STE forward: voxel means of the input rows
    const float *grad_add;      // MODE_STE_BWD: gradient rows added per voxel before the scatter
    // workspace buffers
    uint64_t *keys_a, *keys_b;
    uint32_t *vals_a, *vals_b;
    uint64_t *leaf;
    uint32_t *vh;
    uint32_t *first;         // encode: input row of every voxel's first member (sorted order)
    uint32_t *bbox_part;     // encode: bounding-box workgroups' partial extrema (BBOX_SLOT each)
    uint32_t *lvl_flags;     // upper-level launches: the phase each workgroup has completed
    uint32_t *sort_status;   // P x (sort tiles + look-back groups) x 2^sort_bits
    uint32_t *sort_hist;     // SORT_HIST_COPIES x P x 2^sort_bits digit counts (zeroed by setup)
    uint32_t sort_bits;      // radix digit width (8 or 9)
    uint64_t *dedup_status;
    uint64_t *occ_status;    // occ tiles x J
    uint64_t *dec_status;    // decoder: look-back status of the occupancy-byte tiles
    uint32_t *dec_par;       // decoder: each node's parent (index in its parent's level); the
    uint8_t *dec_cbit;       //   nodes of levels 1..J one after the other; its child bit
    uint32_t sort_tiles, dedup_tiles, occ_tiles;
    uint32_t K;              // RAHT tiling levels
    RahtLevel lv[MAXK + 1];  // index 1..K
};

// Tile-to-frame map passed by value to every batched kernel: frame f owns the workgroups
// [start[f], start[f+1]) and its descriptor lives at fd[f] (inside frame f's workspace).
struct TileMap {
    uint32_t F;
    uint32_t start[GSC_MAX_BATCH + 1];
    FrameDesc *fd[GSC_MAX_BATCH];
};

// Per-frame arguments of the setup kernel (user pointers and sizes).
struct FrameArgs {
    uint32_t n;
    const float *pos;
    const float *attr;
    uint8_t *stream;
    uint64_t stream_cap;
    uint8_t *ws;
    int32_t *info;
    float *coef_f32;
    uint64_t *codes_out;
    uint32_t *perm_out;
    uint32_t *voxel_of_out;
    const uint8_t *in_stream;
    uint64_t in_bytes;
    float *pos_out;
    uint32_t *vox_out;
    float *attr_out;
    const uint64_t *codes_in;
    float *aref;
    const float *grad_add;
    // filled from the frame's layout by the host: the zero region and the bounding-box slots
    uint64_t zero_off, zero_bytes, bbox_off;
};
constexpr int SETUP_MAX = 16;
constexpr int SETUP_THREADS = BBOX_THREADS;  // the setup blocks also take the bounding-box partials
struct SetupArgs {
    uint32_t count;
    uint32_t J, C, mode, bbox_mode;
    uint32_t ste;
    uint32_t keep;       // reuse the workspace state of a previous call (no zeroing)
    uint32_t flags;      // GSC_FLAG_* (encode)
    float tau;
    double bbox_min[3];
    double cell;
    float step[GSC_MAX_CHANNELS];
    FrameArgs f[SETUP_MAX];
};

// ------------------------------------------------------------------ workspace layout
// [Ctrl][FrameDesc][sort status words][zero region: digit histograms, look-back status words][buffers ...]
constexpr size_t DESC_OFF = CTRL_BYTES;
constexpr size_t DESC_BYTES = 8192;
static_assert(sizeof(FrameDesc) <= DESC_BYTES, "descriptor too large");

struct Layout {
    size_t total;
    size_t zero_off, zero_bytes;
    size_t keys_a, keys_b, vals_a, vals_b, leaf, vh, first, bbox_part, lvl_flags;
    size_t sort_status, sort_hist, dedup_status, occ_status, dec_status, dec_par, dec_cbit;
    uint32_t dec_tiles;      // decoder: tiles of DEC_TILE occupancy bytes (all levels together)
    uint64_t dec_nodes;      // decoder: worst-case nodes of levels 1..J
    uint32_t sort_tiles, dedup_tiles, occ_tiles, P, K;
    size_t s_idx[MAXK + 1], s_lvl[MAXK + 1], rec[MAXK + 1], lstart[MAXK + 1], lmask[MAXK + 1], opos[MAXK + 1],
        obase[MAXK + 1], ocnt[MAXK + 1], status[MAXK + 1], vbuf[MAXK + 1];
    uint32_t tiles[MAXK + 1], cap[MAXK + 1];
};

__host__ __device__ inline uint32_t ceil_div(uint64_t a, uint64_t b)
{
    return (uint32_t)((a + b - 1) / b);
}
__host__ __device__ inline int sort_bits(int J)
{
    return (3 * J + 8) / 9 < (3 * J + 7) / 8 ? 9 : 8;
}
__host__ __device__ inline int sort_passes(int J) { return (3 * J + sort_bits(J) - 1) / sort_bits(J); }
__host__ __device__ inline uint32_t open_max(int J) { return 6u * (uint32_t)J + 2u; }
__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Worst-case number of octree nodes at depth d for n leaves: min(8^d, n).
__host__ __device__ inline uint64_t level_cap(int d, uint64_t n)
{
    return d >= 21 ? n : ((1ull << (3 * d)) < n ? (1ull << (3 * d)) : n);
}

// Layout of a workspace for frames of at most n entries (Gaussians or voxels) at depth J with
// C channels. Every region is 256-byte aligned. Returns false if the sizes are out of range.
__host__ __device__ inline bool make_layout(int64_t n, int J, int C, Layout *L)
{
    if (n < 0 || n > 0x7FFFFFFFll || J < 1 || J > GSC_MAX_DEPTH || C < 1 ||
        C > GSC_MAX_CHANNELS)
        return false;
    const uint64_t N = (uint64_t)(n > 0 ? n : 1);
    const int C4 = (C + 3) / 4;
    const uint32_t om = open_max(J);
    L->P = (uint32_t)sort_passes(J);
    L->sort_tiles = ceil_div(N, SORT_THREADS * SORT_KPT_MIN);
    L->dedup_tiles = ceil_div(N, DEDUP_TILE);
    L->occ_tiles = ceil_div(N, OCC_TILE);
    // RAHT tiling levels: S_1 has N entries; a tile of RT entries leaves at most 6J+2 open.
    uint32_t K = 0;
    uint64_t s = N;
    for (int k = 1; k <= MAXK; ++k) {
        L->cap[k] = (uint32_t)s;
        L->tiles[k] = ceil_div(s, RT);
        K = (uint32_t)k;
        if (s <= (uint64_t)RT) break;
        uint64_t nxt = (uint64_t)L->tiles[k] * om;
        s = nxt < s ? nxt : s;
    }
    if (L->cap[K] > (uint32_t)RT) return false;
    L->K = K;
    size_t off = DESC_OFF + DESC_BYTES;
    // the sort's status words (zeroed by the voxelize kernel of an encode, which precedes the
    // sort), then the zero region: the sort's digit histograms, every other look-back status
    // word and nothing else
    L->sort_status = off;
    off = align_up(off + (size_t)L->P * (L->sort_tiles + sort_groups(L->sort_tiles)) * ((size_t)1 << sort_bits(J)) * 4, 256);
    L->zero_off = off;
    L->sort_hist = off;
    off = align_up(off + (size_t)SORT_HIST_COPIES * L->P * ((size_t)1 << sort_bits(J)) * 4, 256);
    L->dedup_status = off;
    off = align_up(off + (size_t)L->dedup_tiles * 8, 256);
    L->occ_status = off;
    off = align_up(off + (size_t)L->occ_tiles * J * 8, 256);
    L->dec_status = off;
    uint64_t occ_cap = 0, nodes = 0;
    for (int d = 0; d < J; ++d) occ_cap += level_cap(d, N);
    for (int d = 1; d <= J; ++d) nodes += level_cap(d, N);
    L->dec_tiles = ceil_div(occ_cap, DEC_TILE);
    L->dec_nodes = nodes;
    off = align_up(off + (size_t)L->dec_tiles * 8, 256);
    for (uint32_t k = 1; k <= K; ++k) {
        L->status[k] = off;
        off = align_up(off + (size_t)L->tiles[k] * 8, 256);
    }
    L->zero_bytes = off - L->zero_off;
    // plain buffers
    L->keys_a = off; off = align_up(off + N * 8, 256);
    L->keys_b = off; off = align_up(off + N * 8, 256);
    L->vals_a = off; off = align_up(off + N * 4, 256);
    L->vals_b = off; off = align_up(off + N * 4, 256);
    L->leaf = off; off = align_up(off + N * 8, 256);
    L->vh = off; off = align_up(off + (N + 1) * 4, 256);
    L->dec_par = off; off = align_up(off + nodes * 4, 256);
    L->dec_cbit = off; off = align_up(off + nodes, 256);
    L->first = off; off = align_up(off + N * 4, 256);
    L->bbox_part = off; off = align_up(off + (size_t)BBOX_GRID_MAX * BBOX_SLOT * 4, 256);
    L->lvl_flags = off; off = align_up(off + (size_t)(UP_GRID_MAX + DONE_WORDS) * 4, 256);
    for (uint32_t k = 1; k <= K; ++k) {
        const uint32_t t = L->tiles[k];
        L->s_idx[k] = off; off = align_up(off + (size_t)L->cap[k] * 4, 256);
        L->s_lvl[k] = off; off = align_up(off + (size_t)L->cap[k], 256);
        L->rec[k] = off; off = align_up(off + (size_t)t * RT * 4, 256);
        L->lstart[k] = off; off = align_up(off + (size_t)t * LSTART_N * 2, 256);
        L->lmask[k] = off; off = align_up(off + (size_t)t * NCLS * 8, 256);
        L->opos[k] = off; off = align_up(off + (size_t)t * OPEN_CAP * 2, 256);
        L->obase[k] = off; off = align_up(off + (size_t)t * 4, 256);
        L->ocnt[k] = off; off = align_up(off + (size_t)t * 4, 256);
        const uint64_t nxt = k < K ? L->cap[k + 1] : 1;
        L->vbuf[k] = off; off = align_up(off + (size_t)nxt * C4 * 16, 256);
    }
    L->total = off;
    return true;
}

// Launch helpers (defined next to their kernels). Each returns the launch status.
hipError_t launch_setup(const SetupArgs &a, uint32_t zero_blocks, hipStream_t s);
hipError_t launch_voxelize(const TileMap &m, hipStream_t s);
hipError_t launch_sort_pass(const TileMap &m, int pass, int variant, int bits, hipStream_t s);
hipError_t launch_dedup(const TileMap &m, hipStream_t s);
hipError_t launch_occupancy(const TileMap &m, hipStream_t s);
hipError_t launch_dec_expand(const TileMap &m, hipStream_t s);
// the decoder's leaves and first-level schedule (one workgroup per first-level tile)
hipError_t launch_dec_prelude(const TileMap &m, hipStream_t s);
hipError_t launch_prelude(const TileMap &m, int k, hipStream_t s);
// Compile-time specializations of the transform kernels: vec = C % 4 == 0 and every row
// pointer 16-byte aligned; pow2 = every quantization step a power of two.
struct RahtCfg {
    int C4;
    bool vec, pow2;
};
uint32_t raht_blocks(uint32_t tiles, int k, int C4);  // first-level items of a frame
uint32_t channel_slices_upper(int C4);                // channel slices of an upper-level tile
// The forward transform of all tiling levels, with the upper levels' schedules, in one persistent
// launch; the first-level inverse (after launch_raht_inv_up). m maps the first-level items to
// frames; kmax is the largest tiling level over the frames.
// finish: the launch is the call's last and ends it (its last workgroup runs finish_frame)
hipError_t launch_raht_fwd(const TileMap &m, int kmax, bool finish, const RahtCfg &cfg, hipStream_t s);
hipError_t launch_raht_inv(const TileMap &m, bool finish, const RahtCfg &cfg, hipStream_t s);
// The upper levels' inverse (2 .. kmax; only m.F and m.fd are used) in one persistent launch,
// before launch_raht_inv; with `prelude`, the launch first builds the upper levels' schedules.
// items_max: the worst-case items of the largest upper level over the launch's frames.
hipError_t launch_raht_inv_up(const TileMap &m, int kmax, uint32_t items_max, bool prelude, const RahtCfg &cfg,
                              hipStream_t s);
hipError_t launch_finish(const TileMap &m, hipStream_t s);
// Block entropy coder (k_rlgr.hip); ws: 8 (ceil(nv / B) + 1) bytes.
// occupancy-byte rANS coder (k_rans.hip)
uint64_t rans_chunks(uint64_t n, uint32_t K);
uint64_t rans_workspace_bytes(uint64_t n, uint32_t K);
uint64_t rans_capacity_bytes(uint64_t n, uint32_t K);
hipError_t launch_rans_encode(const uint8_t *in, uint64_t n, uint32_t K, uint8_t *out, uint64_t cap, void *ws,
                              int32_t *info, hipStream_t s);
hipError_t launch_rans_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t K, uint8_t *out, void *ws,
                              int32_t *info, hipStream_t s);
// colour decorrelation (k_color.hip)
size_t color_workspace_bytes(uint32_t n);
hipError_t launch_color_forward(const float *in, float *out, uint32_t n, uint32_t C, uint32_t sh0, float *klt,
                                double *eig, double *part, int32_t *info, hipStream_t s);
hipError_t launch_color_inverse(const float *in, float *out, uint32_t n, uint32_t C, uint32_t sh0, const float *klt,
                                hipStream_t s);
hipError_t launch_rlgr_encode(const int32_t *q, uint32_t nv, uint32_t C, uint32_t B, uint8_t *out,
                              uint64_t out_cap, uint64_t *ws, int32_t *info, hipStream_t s);
hipError_t launch_rlgr_decode(const uint8_t *in, uint64_t in_bytes, uint32_t nv, uint32_t C, uint32_t B,
                              int32_t *q, uint64_t *ws, int32_t *info, hipStream_t s);

}  // namespace gsc
