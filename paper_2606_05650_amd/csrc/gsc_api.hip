// Host side of the C ABI declared in include/gsc.h: argument checks, workspace layout, and the
// launch sequence of every entry point. Nothing here allocates device memory or synchronizes.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "gsc_internal.h"

namespace gsc {
uint32_t voxelize_blocks(uint32_t n);
uint32_t prelude_blocks(uint32_t tiles);
}  // namespace gsc

using namespace gsc;

namespace {

// ------------------------------------------------------------------------ checks
gsc_status check_shape(int32_t J, int32_t C)
{
    if (J < 1 || J > GSC_MAX_DEPTH || C < 1 || C > GSC_MAX_CHANNELS) return GSC_ERR_DEPTH;
    return GSC_OK;
}

gsc_status check_params(const gsc_params *p)
{
    if (!p) return GSC_ERR_INVALID_ARG;
    gsc_status st = check_shape(p->J, p->C);
    if (st != GSC_OK) return st;
    for (int c = 0; c < p->C; ++c)
        if (!(p->quant_step[c] > 0.0f) || !isfinite(p->quant_step[c])) return GSC_ERR_INVALID_ARG;
    if (!(p->tau >= 0.0f && p->tau < 1.0f)) return GSC_ERR_INVALID_ARG;
    if (p->bbox_mode != 0 && p->bbox_mode != 1) return GSC_ERR_INVALID_ARG;
    if ((p->flags & ~GSC_FLAGS_KNOWN) != 0 || p->reserved != 0) return GSC_ERR_INVALID_ARG;
    if (p->bbox_mode == 1) {
        if (!(p->cell > 0.0) || !isfinite(p->cell)) return GSC_ERR_INVALID_ARG;
        for (int a = 0; a < 3; ++a)
            if (!isfinite(p->bbox_min[a])) return GSC_ERR_INVALID_ARG;
    }
    return GSC_OK;
}

constexpr int64_t N_LIMIT = (1ll << 30) - 1;  // sort status words hold 30-bit counts

// Device byte ranges one call touches, checked for overlaps before anything is enqueued: two
// ranges may share bytes only when neither is written. Sorted by start and swept once, keeping
// the furthest end of any range and of any written range seen so far.
struct Span {
    uintptr_t p;
    uint64_t n;
    bool w;
};
struct Spans {
    static constexpr int CAP = GSC_MAX_BATCH * 12;
    Span s[CAP];
    int k = 0;
    bool full = false;
    void add(const void *p, uint64_t n, bool w)
    {
        if (!p || n == 0) return;
        if (k == CAP) {
            full = true;
            return;
        }
        s[k++] = Span{(uintptr_t)p, n, w};
    }
    void rd(const void *p, uint64_t n) { add(p, n, false); }
    void wr(const void *p, uint64_t n) { add(p, n, true); }
    bool disjoint()
    {
        if (full) return false;
        std::sort(s, s + k, [](const Span &a, const Span &b) { return a.p < b.p; });
        uint64_t end_any = 0, end_w = 0;
        for (int i = 0; i < k; ++i) {
            const uint64_t b = (uint64_t)s[i].p, e = b + s[i].n;
            if (e < b) return false;  // wraps around the address space
            if (b < end_w || (s[i].w && b < end_any)) return false;
            end_any = std::max(end_any, e);
            if (s[i].w) end_w = std::max(end_w, e);
        }
        return true;
    }
};

uint64_t stream_capacity(int64_t n, int J, int C)
{
    uint64_t occ = 0;
    for (int d = 0; d < J; ++d) occ += level_cap(d, (uint64_t)n);
    if (n == 0) occ = 0;
    return align_up(GSC_HEADER_BYTES + occ, 256) + (uint64_t)n * (uint64_t)C * 4u;
}

// ---------------------------------------------------------------- profiling hooks
struct StageHook {
    const void *const *events = nullptr;
    int n_pairs = 0;
    uint64_t count = 0;
};
StageHook g_hooks[GSC_STAGE_COUNT];

struct StageScope {
    StageHook *h;
    hipStream_t s;
    int pair;
    StageScope(int stage, hipStream_t st) : h(&g_hooks[stage]), s(st), pair(-1)
    {
        if (h->n_pairs > 0) {
            pair = (int)(h->count++ % (uint64_t)h->n_pairs);
            (void)hipEventRecord((hipEvent_t)h->events[2 * pair], s);
        }
    }
    ~StageScope()
    {
        if (pair >= 0) (void)hipEventRecord((hipEvent_t)h->events[2 * pair + 1], s);
    }
};

// ------------------------------------------------------------------ autotuning table
// The sort tiling of an encode call is looked up by depth and by the size class (ceil(log2))
// of the largest frame of the call; entries hold variant + 1 (0 = not tuned: the default).
std::atomic<int> g_tune[GSC_MAX_DEPTH + 1][32];
thread_local int g_force_variant = -1;  // set while the tuner times a variant

int size_class(uint64_t n)
{
    int c = 0;
    while (c < 31 && (1ull << c) < n) ++c;
    return c;
}

int sort_variant_for(int J, uint64_t nmax)
{
    if (g_force_variant >= 0) return g_force_variant;
    const int v = g_tune[J][size_class(nmax)].load(std::memory_order_relaxed);
    return v > 0 ? v - 1 : sort_default_variant(nmax);
}

// ------------------------------------------------------------------- launch plumbing
struct Frame {
    Layout L;
    FrameArgs a;
};

// Builds the tile map of one kernel: frame f gets blocks(f) workgroups.
template <class Fn>
TileMap make_map(const Frame *fr, int F, Fn blocks)
{
    TileMap m;
    memset(&m, 0, sizeof(m));
    m.F = (uint32_t)F;
    m.start[0] = 0;
    for (int f = 0; f < F; ++f) {
        m.start[f + 1] = m.start[f] + blocks(fr[f]);
        m.fd[f] = reinterpret_cast<FrameDesc *>(fr[f].a.ws + DESC_OFF);
    }
    return m;
}

#define GSC_LAUNCH(expr)                                    \
    do {                                                    \
        if ((expr) != hipSuccess) return GSC_ERR_HIP;       \
    } while (0)

gsc_status run_setup(const Frame *fr, int F, const SetupArgs &proto, hipStream_t s)
{
    for (int f0 = 0; f0 < F; f0 += SETUP_MAX) {
        SetupArgs a = proto;
        a.count = (uint32_t)((F - f0) < SETUP_MAX ? (F - f0) : SETUP_MAX);
        uint64_t zmax = 0;
        uint32_t bmax = 0;  // the bounding-box workgroups of an encode that finds the cube
        const bool bbox = a.mode == MODE_ENCODE && a.bbox_mode == 0 && !a.keep;
        for (uint32_t i = 0; i < a.count; ++i) {
            const Frame &x = fr[f0 + i];
            a.f[i] = x.a;
            a.f[i].zero_off = x.L.zero_off;
            a.f[i].zero_bytes = x.L.zero_bytes;
            a.f[i].bbox_off = x.L.bbox_part;
            if (x.L.zero_bytes > zmax) zmax = x.L.zero_bytes;
            if (bbox && bbox_blocks(x.a.n) > bmax) bmax = bbox_blocks(x.a.n);
        }
        uint32_t zb = ceil_div(zmax / 16 + 1, SETUP_THREADS * 4);
        if (zb < 1) zb = 1;
        if (zb > 1024) zb = 1024;
        GSC_LAUNCH(launch_setup(a, zb > bmax + 1 ? zb : bmax + 1, s));
    }
    return GSC_OK;
}

SetupArgs make_proto(uint32_t J, uint32_t C, uint32_t mode, const gsc_params *p)
{
    SetupArgs a;
    memset(&a, 0, sizeof(a));
    a.J = J;
    a.C = C;
    a.mode = mode;
    if (p) {
        a.flags = p->flags;
        a.bbox_mode = (uint32_t)p->bbox_mode;
        a.tau = p->tau;
        for (int i = 0; i < 3; ++i) a.bbox_min[i] = p->bbox_min[i];
        a.cell = p->cell;
        for (int c = 0; c < GSC_MAX_CHANNELS; ++c) a.step[c] = c < (int)C ? p->quant_step[c] : 1.0f;
    } else {
        for (int c = 0; c < GSC_MAX_CHANNELS; ++c) a.step[c] = 1.0f;
    }
    return a;
}

int max_K(const Frame *fr, int F)
{
    int K = 0;
    for (int f = 0; f < F; ++f)
        if ((int)fr[f].L.K > K) K = (int)fr[f].L.K;
    return K;
}

// Worst-case tiles of level 2 over the frames (the largest upper level).
uint32_t upper_tiles(const Frame *fr, int F)
{
    uint32_t t = 0;
    for (int f = 0; f < F; ++f) t += fr[f].L.K >= 2 ? fr[f].L.tiles[2] : 0u;
    return t;
}

// The first level's schedule (the upper levels' schedules are built by the transform launches).
gsc_status run_prelude(const Frame *fr, int F, hipStream_t s)
{
    StageScope sc(GSC_STAGE_PRELUDE, s);
    TileMap m = make_map(fr, F, [](const Frame &x) { return x.L.K >= 1 ? prelude_blocks(x.L.tiles[1]) : 0u; });
    if (m.start[F] > 0) GSC_LAUNCH(launch_prelude(m, 1, s));
    return GSC_OK;
}

// The forward transform of every tiling level of every frame, with the upper levels' schedules:
// one persistent launch. With `last`, the launch also ends the call (the finish step) if it
// runs; *ended says whether it did.
gsc_status run_forward(const Frame *fr, int F, const RahtCfg &cfg, bool last, bool *ended, hipStream_t s)
{
    TileMap m = make_map(fr, F, [&cfg](const Frame &x) { return x.L.K >= 1 ? raht_blocks(x.L.tiles[1], 1, cfg.C4) : 0u; });
    if (m.start[F] == 0) return GSC_OK;
    StageScope sc(GSC_STAGE_RAHT_FWD1, s);
    GSC_LAUNCH(launch_raht_fwd(m, max_K(fr, F), last, cfg, s));
    *ended = last;
    return GSC_OK;
}

// The inverse: the upper levels in one launch (which first builds their schedules when `prelude`
// is set, i.e. when no forward of this workspace has built them), then the first level.
gsc_status run_inverse(const Frame *fr, int F, const RahtCfg &cfg, bool prelude, bool *ended, hipStream_t s)
{
    const int K = max_K(fr, F);
    if (K >= 2) {
        StageScope sc(GSC_STAGE_RAHT_INV_TOP, s);
        TileMap m = make_map(fr, F, [](const Frame &) { return 1u; });
        GSC_LAUNCH(launch_raht_inv_up(m, K, upper_tiles(fr, F) * channel_slices_upper(cfg.C4), prelude, cfg, s));
    }
    TileMap m = make_map(fr, F, [&cfg](const Frame &x) { return raht_blocks(x.L.tiles[1], 1, cfg.C4); });
    if (m.start[F] == 0) return GSC_OK;
    StageScope sc(GSC_STAGE_RAHT_INV1, s);
    GSC_LAUNCH(launch_raht_inv(m, true, cfg, s));  // (always a call's last launch)
    *ended = true;
    return GSC_OK;
}

// The finish step, unless the call's last transform launch has done it.
gsc_status run_finish(const Frame *fr, int F, bool ended, hipStream_t s)
{
    if (ended) return GSC_OK;
    TileMap m = make_map(fr, F, [](const Frame &) { return 1u; });
    GSC_LAUNCH(launch_finish(m, s));
    return GSC_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool all_pow2(const float *step, int C)
{
    for (int c = 0; c < C; ++c) {
        int e;
        if (frexpf(step[c], &e) != 0.5f) return false;
    }
    return true;
}

// Specialization of the transform kernels for a batch: vectorized rows when C % 4 == 0 and
// every row pointer the kernels touch is 16-byte aligned.
RahtCfg raht_cfg(const Frame *fr, int F, int C, const float *steps)
{
    RahtCfg cfg;
    cfg.C4 = (C + 3) / 4;
    cfg.vec = (C % 4 == 0);
    for (int f = 0; f < F && cfg.vec; ++f) {
        const FrameArgs &a = fr[f].a;
        cfg.vec = aligned16(a.attr) && aligned16(a.stream) && aligned16(a.coef_f32) &&
                  aligned16(a.in_stream) && aligned16(a.attr_out) && aligned16(a.aref) &&
                  aligned16(a.grad_add);
    }
    cfg.pow2 = steps ? all_pow2(steps, C) : false;
    return cfg;
}

// Encode F frames (already validated) with one launch per stage. With ste, also synthesize
// the decoded rows from the dequantized coefficients (straight-through forward).
gsc_status encode_frames(const Frame *fr, int F, const gsc_params *p, hipStream_t s, bool ste = false)
{
    StageScope whole(GSC_STAGE_ENCODE, s);
    SetupArgs proto = make_proto((uint32_t)p->J, (uint32_t)p->C, MODE_ENCODE, p);
    proto.ste = ste ? STE_FORWARD : STE_NONE;
    gsc_status st = run_setup(fr, F, proto, s);
    if (st != GSC_OK) return st;
    {
        StageScope sc(GSC_STAGE_SORT, s);
        {
            TileMap m = make_map(fr, F, [](const Frame &x) { return voxelize_blocks(x.a.n); });
            GSC_LAUNCH(launch_voxelize(m, s));
        }
        const int P = sort_passes(p->J);
        {
            uint64_t nmax = 0;
            for (int f = 0; f < F; ++f) nmax = fr[f].a.n > nmax ? fr[f].a.n : nmax;
            const int var = sort_variant_for(p->J, nmax);
            const uint32_t tile = (uint32_t)sort_tile(var);
            TileMap m = make_map(fr, F, [tile](const Frame &x) { return ceil_div(x.a.n, tile); });
            if (m.start[F] > 0)
                for (int pass = 0; pass < P; ++pass) GSC_LAUNCH(launch_sort_pass(m, pass, var, sort_bits(p->J), s));
        }
        {
            TileMap m = make_map(fr, F, [](const Frame &x) { return x.a.n ? x.L.dedup_tiles : 0u; });
            if (m.start[F] > 0) GSC_LAUNCH(launch_dedup(m, s));
        }
    }
    {
        StageScope sc(GSC_STAGE_OCCUPANCY, s);
        TileMap m = make_map(fr, F, [](const Frame &x) { return x.a.n ? x.L.occ_tiles : 0u; });
        if (m.start[F] > 0) GSC_LAUNCH(launch_occupancy(m, s));
    }
    const RahtCfg cfg = raht_cfg(fr, F, p->C, p->quant_step);
    if ((st = run_prelude(fr, F, s)) != GSC_OK) return st;
    bool ended = false;
    if ((st = run_forward(fr, F, cfg, !ste, &ended, s)) != GSC_OK) return st;
    if (ste && (st = run_inverse(fr, F, cfg, false, &ended, s)) != GSC_OK) return st;
    return run_finish(fr, F, ended, s);
}

gsc_status decode_frames(const Frame *fr, int F, int J, int C, hipStream_t s)
{
    StageScope whole(GSC_STAGE_DECODE, s);
    const SetupArgs proto = make_proto((uint32_t)J, (uint32_t)C, MODE_DECODE, nullptr);
    gsc_status st = run_setup(fr, F, proto, s);
    if (st != GSC_OK) return st;
    {
        StageScope sc(GSC_STAGE_OCTREE_DEC, s);
        {
            TileMap m = make_map(fr, F, [](const Frame &x) { return x.L.dec_tiles; });
            GSC_LAUNCH(launch_dec_expand(m, s));
        }
        {   // the leaves and the first level's schedule
            TileMap m = make_map(fr, F, [](const Frame &x) { return x.L.K >= 1 ? prelude_blocks(x.L.tiles[1]) : 0u; });
            if (m.start[F] > 0) GSC_LAUNCH(launch_dec_prelude(m, s));
        }
    }
    const RahtCfg cfg = raht_cfg(fr, F, C, nullptr);
    bool ended = false;
    if ((st = run_inverse(fr, F, cfg, true, &ended, s)) != GSC_OK) return st;
    return run_finish(fr, F, ended, s);
}

bool layout_for(int64_t n, int J, int C, Layout *L) { return make_layout(n, J, C, L); }

}  // namespace

// =============================================================================== ABI
extern "C" {

const char *gsc_status_string(gsc_status s)
{
    switch (s) {
    case GSC_OK: return "ok";
    case GSC_ERR_INVALID_ARG: return "invalid argument";
    case GSC_ERR_DEPTH: return "depth or channel count out of range";
    case GSC_ERR_WORKSPACE: return "workspace too small";
    case GSC_ERR_CAPACITY: return "output capacity too small";
    case GSC_ERR_CORRUPT_STREAM: return "corrupt stream";
    case GSC_ERR_HIP: return "HIP launch failed";
    case GSC_ERR_INTERNAL: return "internal error";
    case GSC_ERR_SCRATCH: return "frame too large for the static scratch";
    }
    return "unknown status";
}

gsc_status gsc_profile_events(int32_t stage, void *const *events, int32_t n_pairs)
{
    if (stage < 0 || stage >= GSC_STAGE_COUNT || n_pairs < 0) return GSC_ERR_INVALID_ARG;
    StageHook &h = g_hooks[stage];
    if (!events || n_pairs == 0) {
        h.events = nullptr;
        h.n_pairs = 0;
    } else {
        h.events = events;
        h.n_pairs = n_pairs;
    }
    h.count = 0;
    return GSC_OK;
}

gsc_status gsc_workspace_size(int64_t n_max, int32_t J, int32_t C, size_t *bytes)
{
    if (!bytes) return GSC_ERR_INVALID_ARG;
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    if (n_max < 0 || n_max > N_LIMIT) return GSC_ERR_INVALID_ARG;
    Layout L;
    if (!layout_for(n_max, J, C, &L)) return GSC_ERR_INVALID_ARG;
    *bytes = L.total;
    return GSC_OK;
}

gsc_status gsc_stream_capacity(int64_t n_max, int32_t J, int32_t C, size_t *bytes)
{
    if (!bytes) return GSC_ERR_INVALID_ARG;
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    if (n_max < 0 || n_max > N_LIMIT) return GSC_ERR_INVALID_ARG;
    *bytes = (size_t)stream_capacity(n_max, J, C);
    return GSC_OK;
}

}  // extern "C"

namespace {
gsc_status prepare_encode_batch(const gsc_frame_desc *frames, int32_t F, const gsc_params *params,
                                Frame *fr)
{
    if (!frames || F < 1 || F > GSC_MAX_BATCH) return GSC_ERR_INVALID_ARG;
    gsc_status st = check_params(params);
    if (st != GSC_OK) return st;
    for (int f = 0; f < F; ++f) {
        const gsc_frame_desc &d = frames[f];
        if (d.n < 0 || d.n > N_LIMIT) return GSC_ERR_INVALID_ARG;
        if (!d.d_stream || !d.d_ws || !d.d_info) return GSC_ERR_INVALID_ARG;
        if (d.n > 0 && (!d.d_pos || !d.d_attr)) return GSC_ERR_INVALID_ARG;
        if (!layout_for(d.n, params->J, params->C, &fr[f].L)) return GSC_ERR_INVALID_ARG;
        if (d.ws_bytes < fr[f].L.total) return GSC_ERR_WORKSPACE;
        if (d.stream_cap < stream_capacity(d.n, params->J, params->C)) return GSC_ERR_CAPACITY;
        FrameArgs &a = fr[f].a;
        memset(&a, 0, sizeof(a));
        a.n = (uint32_t)d.n;
        a.pos = d.d_pos;
        a.attr = d.d_attr;
        a.stream = static_cast<uint8_t *>(d.d_stream);
        a.stream_cap = d.stream_cap;
        a.ws = static_cast<uint8_t *>(d.d_ws);
        a.info = d.d_info;
    }
    static thread_local Spans sp;
    sp.k = 0;
    sp.full = false;
    const uint64_t row = (uint64_t)params->C * 4;
    for (int f = 0; f < F; ++f) {
        const gsc_frame_desc &d = frames[f];
        sp.rd(d.d_pos, (uint64_t)d.n * 12);
        sp.rd(d.d_attr, (uint64_t)d.n * row);
        sp.wr(d.d_stream, stream_capacity(d.n, params->J, params->C));
        sp.wr(d.d_ws, fr[f].L.total);
        sp.wr(d.d_info, GSC_INFO_WORDS * 4);
    }
    return sp.disjoint() ? GSC_OK : GSC_ERR_INVALID_ARG;
}
}  // namespace

extern "C" {

gsc_status gsc_encode_batch(const gsc_frame_desc *frames, int32_t F, const gsc_params *params,
                            void *stream)
{
    static thread_local Frame fr[GSC_MAX_BATCH];
    gsc_status st = prepare_encode_batch(frames, F, params, fr);
    if (st != GSC_OK) return st;
    return encode_frames(fr, F, params, static_cast<hipStream_t>(stream));
}

constexpr float SORT_TUNE_MARGIN = 0.02f;  // the autotuner keeps the default unless another is 2 % faster

gsc_status gsc_autotune(const gsc_frame_desc *frames, int32_t F, const gsc_params *params,
                        int32_t reps, int32_t *chosen, float *times_ms, void *stream)
{
    static thread_local Frame fr[GSC_MAX_BATCH];
    gsc_status st = prepare_encode_batch(frames, F, params, fr);
    if (st != GSC_OK) return st;
    if (reps < 1 || reps > 1000) return GSC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return GSC_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return GSC_ERR_HIP;
    }
    float t[SORT_VARIANTS] = {};
    for (int v = 0; v < SORT_VARIANTS && st == GSC_OK; ++v) {
        g_force_variant = v;
        st = encode_frames(fr, F, params, s);  // warm-up
        if (st == GSC_OK && hipEventRecord(e0, s) != hipSuccess) st = GSC_ERR_HIP;
        for (int r = 0; r < reps && st == GSC_OK; ++r) st = encode_frames(fr, F, params, s);
        if (st == GSC_OK && hipEventRecord(e1, s) != hipSuccess) st = GSC_ERR_HIP;
        float ms = 0.0f;
        if (st == GSC_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = GSC_ERR_HIP;
        ms /= (float)reps;
        if (times_ms) times_ms[v] = ms;
        t[v] = ms;
    }
    g_force_variant = -1;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GSC_OK) return st;
    uint64_t nmax = 0;
    for (int f = 0; f < F; ++f) nmax = fr[f].a.n > nmax ? fr[f].a.n : nmax;
    // the fastest tiling, unless it beats the size's default by less than the margin (a near
    // tie is timing noise, and the default is the tiling measured best for the size)
    int best_v = 0;
    for (int v = 1; v < SORT_VARIANTS; ++v)
        if (t[v] < t[best_v]) best_v = v;
    const int d = sort_default_variant(nmax);
    if (!(t[best_v] < (1.0f - SORT_TUNE_MARGIN) * t[d])) best_v = d;
    g_tune[params->J][size_class(nmax)].store(best_v + 1, std::memory_order_relaxed);
    if (chosen) *chosen = best_v;
    return GSC_OK;
}

gsc_status gsc_tune_set(int32_t J, int64_t n, int32_t variant)
{
    if (J < 1 || J > GSC_MAX_DEPTH || n < 0 || n > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (variant < -1 || variant >= SORT_VARIANTS) return GSC_ERR_INVALID_ARG;
    g_tune[J][size_class((uint64_t)n)].store(variant + 1, std::memory_order_relaxed);
    return GSC_OK;
}

gsc_status gsc_tune_get(int32_t J, int64_t n, int32_t *variant)
{
    if (J < 1 || J > GSC_MAX_DEPTH || n < 0 || n > N_LIMIT || !variant) return GSC_ERR_INVALID_ARG;
    *variant = sort_variant_for(J, (uint64_t)n);
    return GSC_OK;
}

gsc_status gsc_encode_frame(const float *d_pos, const float *d_attr, int64_t n,
                            const gsc_params *params, void *d_stream, size_t stream_cap,
                            void *d_ws, size_t ws_bytes, int32_t *d_info, float *d_coef_f32,
                            uint64_t *d_leaf_codes, uint32_t *d_perm, uint32_t *d_voxel_of,
                            void *stream)
{
    gsc_status st = check_params(params);
    if (st != GSC_OK) return st;
    if (n < 0 || n > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (!d_stream || !d_ws || !d_info) return GSC_ERR_INVALID_ARG;
    if (n > 0 && (!d_pos || !d_attr)) return GSC_ERR_INVALID_ARG;
    Frame fr;
    if (!layout_for(n, params->J, params->C, &fr.L)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < fr.L.total) return GSC_ERR_WORKSPACE;
    if (stream_cap < stream_capacity(n, params->J, params->C)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        const uint64_t rows = (uint64_t)n * params->C * 4;
        sp.rd(d_pos, (uint64_t)n * 12);
        sp.rd(d_attr, rows);
        sp.wr(d_stream, stream_capacity(n, params->J, params->C));
        sp.wr(d_ws, fr.L.total);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        sp.wr(d_coef_f32, rows);
        sp.wr(d_leaf_codes, (uint64_t)n * 8);
        sp.wr(d_perm, (uint64_t)n * 4);
        sp.wr(d_voxel_of, (uint64_t)n * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    memset(&fr.a, 0, sizeof(fr.a));
    fr.a.n = (uint32_t)n;
    fr.a.pos = d_pos;
    fr.a.attr = d_attr;
    fr.a.stream = static_cast<uint8_t *>(d_stream);
    fr.a.stream_cap = stream_cap;
    fr.a.ws = static_cast<uint8_t *>(d_ws);
    fr.a.info = d_info;
    fr.a.coef_f32 = d_coef_f32;
    fr.a.codes_out = d_leaf_codes;
    fr.a.perm_out = d_perm;
    fr.a.voxel_of_out = d_voxel_of;
    return encode_frames(&fr, 1, params, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ------------------------------------------------------------------ static scratch
// The workspace of gsc_encode_frame_noalloc: one array per device, part of the library's code
// object, held from the library's load on that device until the process ends. In host code
// `scratch` only names the symbol; the kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[GSC_STATIC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES];

// The current device's copy of `scratch`: looked up on the first call made with that device
// current and kept (a failed lookup is tried again by the next call). nullptr when the device
// or the lookup fails.
void *scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

gsc_status gsc_encode_frame_noalloc(const float *d_pos, const float *d_attr, int64_t n,
                                    const gsc_params *params, void *d_stream, size_t stream_cap,
                                    int32_t *d_info, float *d_coef_f32, uint64_t *d_leaf_codes,
                                    uint32_t *d_perm, uint32_t *d_voxel_of, void *stream)
{
    gsc_status st = check_params(params);
    if (st != GSC_OK) return st;
    if (n < 0 || n > N_LIMIT) return GSC_ERR_INVALID_ARG;
    Layout L;
    if (!layout_for(n, params->J, params->C, &L)) return GSC_ERR_INVALID_ARG;
    if (L.total > GSC_STATIC_SCRATCH_BYTES) return GSC_ERR_SCRATCH;
    void *ws = scratch_ptr();
    if (!ws) return GSC_ERR_HIP;
    // every region of the workspace that must start at zero is cleared by the call's setup
    // kernel, so the contents an earlier call left do not matter
    return gsc_encode_frame(d_pos, d_attr, n, params, d_stream, stream_cap, ws,
                            GSC_STATIC_SCRATCH_BYTES, d_info, d_coef_f32, d_leaf_codes, d_perm,
                            d_voxel_of, stream);
}

gsc_status gsc_decode_batch(const gsc_stream_desc *streams, int32_t F, int32_t J, int32_t C,
                            void *stream)
{
    if (!streams || F < 1 || F > GSC_MAX_BATCH) return GSC_ERR_INVALID_ARG;
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    static thread_local Frame fr[GSC_MAX_BATCH];
    for (int f = 0; f < F; ++f) {
        const gsc_stream_desc &d = streams[f];
        if (d.n_cap < 0 || d.n_cap > N_LIMIT) return GSC_ERR_INVALID_ARG;
        if (!d.d_stream || !d.d_ws || !d.d_info || !d.d_pos_out || !d.d_attr_out)
            return GSC_ERR_INVALID_ARG;
        if (!layout_for(d.n_cap, J, C, &fr[f].L)) return GSC_ERR_INVALID_ARG;
        if (d.ws_bytes < fr[f].L.total) return GSC_ERR_WORKSPACE;
        FrameArgs &a = fr[f].a;
        memset(&a, 0, sizeof(a));
        a.n = (uint32_t)d.n_cap;
        a.in_stream = static_cast<const uint8_t *>(d.d_stream);
        a.in_bytes = d.stream_bytes;
        a.ws = static_cast<uint8_t *>(d.d_ws);
        a.info = d.d_info;
        a.pos_out = d.d_pos_out;
        a.attr_out = d.d_attr_out;
    }
    static thread_local Spans sp;
    sp.k = 0;
    sp.full = false;
    for (int f = 0; f < F; ++f) {
        const gsc_stream_desc &d = streams[f];
        sp.rd(d.d_stream, d.stream_bytes);
        sp.wr(d.d_pos_out, (uint64_t)d.n_cap * 12);
        sp.wr(d.d_attr_out, (uint64_t)d.n_cap * C * 4);
        sp.wr(d.d_ws, fr[f].L.total);
        sp.wr(d.d_info, GSC_INFO_WORDS * 4);
    }
    if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    return decode_frames(fr, F, J, C, static_cast<hipStream_t>(stream));
}

gsc_status gsc_decode_frame(const void *d_stream, size_t stream_bytes, int32_t J, int32_t C,
                            int64_t n_cap, float *d_pos_out, uint32_t *d_vox_out,
                            float *d_attr_out, uint64_t *d_leaf_codes, void *d_ws,
                            size_t ws_bytes, int32_t *d_info, void *stream)
{
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    if (n_cap < 0 || n_cap > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (!d_stream || !d_ws || !d_info || !d_pos_out || !d_attr_out) return GSC_ERR_INVALID_ARG;
    Frame fr;
    if (!layout_for(n_cap, J, C, &fr.L)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < fr.L.total) return GSC_ERR_WORKSPACE;
    {
        Spans sp;
        sp.rd(d_stream, stream_bytes);
        sp.wr(d_pos_out, (uint64_t)n_cap * 12);
        sp.wr(d_vox_out, (uint64_t)n_cap * 12);
        sp.wr(d_attr_out, (uint64_t)n_cap * C * 4);
        sp.wr(d_leaf_codes, (uint64_t)n_cap * 8);
        sp.wr(d_ws, fr.L.total);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    memset(&fr.a, 0, sizeof(fr.a));
    fr.a.n = (uint32_t)n_cap;
    fr.a.in_stream = static_cast<const uint8_t *>(d_stream);
    fr.a.in_bytes = stream_bytes;
    fr.a.ws = static_cast<uint8_t *>(d_ws);
    fr.a.info = d_info;
    fr.a.pos_out = d_pos_out;
    fr.a.vox_out = d_vox_out;
    fr.a.attr_out = d_attr_out;
    fr.a.codes_out = d_leaf_codes;
    return decode_frames(&fr, 1, J, C, static_cast<hipStream_t>(stream));
}

static gsc_status raht_f32(const uint64_t *d_codes, int64_t nv, int32_t J, int32_t C,
                           const float *d_in, float *d_out, void *d_ws, size_t ws_bytes,
                           int32_t *d_info, void *stream, bool adjoint)
{
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    if (nv < 0 || nv > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (!d_ws || !d_info) return GSC_ERR_INVALID_ARG;
    if (nv > 0 && (!d_codes || !d_in || !d_out)) return GSC_ERR_INVALID_ARG;
    if (nv > 0 && (const void *)d_in == (const void *)d_out) return GSC_ERR_INVALID_ARG;
    Frame fr;
    if (!layout_for(nv, J, C, &fr.L)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < fr.L.total) return GSC_ERR_WORKSPACE;
    {
        Spans sp;
        sp.rd(d_codes, (uint64_t)nv * 8);
        sp.rd(d_in, (uint64_t)nv * C * 4);
        sp.wr(d_out, (uint64_t)nv * C * 4);
        sp.wr(d_ws, fr.L.total);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    memset(&fr.a, 0, sizeof(fr.a));
    fr.a.n = (uint32_t)nv;
    fr.a.codes_in = d_codes;
    fr.a.attr = d_in;
    fr.a.coef_f32 = d_out;
    fr.a.ws = static_cast<uint8_t *>(d_ws);
    fr.a.info = d_info;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SetupArgs proto = make_proto((uint32_t)J, (uint32_t)C, adjoint ? MODE_ADJ_F32 : MODE_FWD_F32, nullptr);
    if ((st = run_setup(&fr, 1, proto, s)) != GSC_OK) return st;
    bool ended = false;
    if (nv > 0) {
        if ((st = run_prelude(&fr, 1, s)) != GSC_OK) return st;
        const RahtCfg cfg = raht_cfg(&fr, 1, C, nullptr);
        if (adjoint)
            st = run_inverse(&fr, 1, cfg, true, &ended, s);
        else
            st = run_forward(&fr, 1, cfg, true, &ended, s);
        if (st != GSC_OK) return st;
    }
    return run_finish(&fr, 1, ended, s);
}

gsc_status gsc_ste_forward(const float *d_pos, const float *d_attr, int64_t n,
                           const gsc_params *params, void *d_stream, size_t stream_cap, void *d_ws,
                           size_t ws_bytes, int32_t *d_info, float *d_yhat, float *d_ahat,
                           float *d_aref, uint64_t *d_leaf_codes, void *stream)
{
    gsc_status st = check_params(params);
    if (st != GSC_OK) return st;
    if (n < 0 || n > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (!d_stream || !d_ws || !d_info) return GSC_ERR_INVALID_ARG;
    if (n > 0 && (!d_pos || !d_attr || !d_yhat || !d_ahat)) return GSC_ERR_INVALID_ARG;
    if (n > 0 && ((const void *)d_yhat == (const void *)d_ahat || (const void *)d_yhat == (const void *)d_attr ||
                  (const void *)d_ahat == (const void *)d_attr))
        return GSC_ERR_INVALID_ARG;
    Frame fr;
    if (!layout_for(n, params->J, params->C, &fr.L)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < fr.L.total) return GSC_ERR_WORKSPACE;
    if (stream_cap < stream_capacity(n, params->J, params->C)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        const uint64_t rows = (uint64_t)n * params->C * 4;
        sp.rd(d_pos, (uint64_t)n * 12);
        sp.rd(d_attr, rows);
        sp.wr(d_stream, stream_capacity(n, params->J, params->C));
        sp.wr(d_ws, fr.L.total);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        sp.wr(d_yhat, rows);
        sp.wr(d_ahat, rows);
        sp.wr(d_aref, rows);
        sp.wr(d_leaf_codes, (uint64_t)n * 8);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    memset(&fr.a, 0, sizeof(fr.a));
    fr.a.n = (uint32_t)n;
    fr.a.pos = d_pos;
    fr.a.attr = d_attr;
    fr.a.stream = static_cast<uint8_t *>(d_stream);
    fr.a.stream_cap = stream_cap;
    fr.a.ws = static_cast<uint8_t *>(d_ws);
    fr.a.info = d_info;
    fr.a.coef_f32 = d_yhat;
    fr.a.attr_out = d_ahat;
    fr.a.aref = d_aref;
    fr.a.codes_out = d_leaf_codes;
    return encode_frames(&fr, 1, params, static_cast<hipStream_t>(stream), true);
}

gsc_status gsc_ste_backward(int64_t n, int32_t J, int32_t C, const float *d_grad_yhat,
                            const float *d_grad_ahat, float *d_grad_attr, void *d_ws,
                            size_t ws_bytes, int32_t *d_info, void *stream)
{
    gsc_status st = check_shape(J, C);
    if (st != GSC_OK) return st;
    if (n < 0 || n > N_LIMIT) return GSC_ERR_INVALID_ARG;
    if (!d_ws || !d_info) return GSC_ERR_INVALID_ARG;
    if (n > 0 && (!d_grad_yhat || !d_grad_ahat || !d_grad_attr)) return GSC_ERR_INVALID_ARG;
    if (n > 0 && ((const void *)d_grad_attr == (const void *)d_grad_yhat ||
                  (const void *)d_grad_attr == (const void *)d_grad_ahat))
        return GSC_ERR_INVALID_ARG;
    Frame fr;
    if (!layout_for(n, J, C, &fr.L)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < fr.L.total) return GSC_ERR_WORKSPACE;
    {
        // the gradient inputs hold Nv <= n rows (Nv is known on the device only): their first
        // row is checked
        Spans sp;
        sp.rd(d_grad_yhat, (uint64_t)C * 4);
        sp.rd(d_grad_ahat, (uint64_t)C * 4);
        sp.wr(d_grad_attr, (uint64_t)n * C * 4);
        sp.wr(d_ws, fr.L.total);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    memset(&fr.a, 0, sizeof(fr.a));
    fr.a.n = (uint32_t)n;
    fr.a.attr = d_grad_yhat;
    fr.a.grad_add = d_grad_ahat;
    fr.a.attr_out = d_grad_attr;
    fr.a.ws = static_cast<uint8_t *>(d_ws);
    fr.a.info = d_info;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SetupArgs proto = make_proto((uint32_t)J, (uint32_t)C, MODE_STE_BWD, nullptr);
    proto.ste = STE_FORWARD;  // the workspace keeps holding the forward's schedule
    proto.keep = 1;
    if ((st = run_setup(&fr, 1, proto, s)) != GSC_OK) return st;
    bool ended = false;
    if (n > 0) {
        const RahtCfg cfg = raht_cfg(&fr, 1, C, nullptr);
        if ((st = run_inverse(&fr, 1, cfg, false, &ended, s)) != GSC_OK) return st;
    }
    return run_finish(&fr, 1, ended, s);
}

gsc_status gsc_raht_forward(const uint64_t *d_codes, int64_t nv, int32_t J, int32_t C,
                            const float *d_in, float *d_out, void *d_ws, size_t ws_bytes,
                            int32_t *d_info, void *stream)
{
    return raht_f32(d_codes, nv, J, C, d_in, d_out, d_ws, ws_bytes, d_info, stream, false);
}

gsc_status gsc_raht_adjoint(const uint64_t *d_codes, int64_t nv, int32_t J, int32_t C,
                            const float *d_in, float *d_out, void *d_ws, size_t ws_bytes,
                            int32_t *d_info, void *stream)
{
    return raht_f32(d_codes, nv, J, C, d_in, d_out, d_ws, ws_bytes, d_info, stream, true);
}

}  // extern "C"

// ---------------------------------------------------------------- block entropy coder
namespace {
constexpr int64_t RLGR_NV_LIMIT = (1ll << 30) - 1;
constexpr int32_t RLGR_B_MAX = 65536;

gsc_status rlgr_shape(int64_t nv, int32_t C, int32_t B)
{
    if (C < 1 || C > GSC_MAX_CHANNELS) return GSC_ERR_DEPTH;
    if (nv < 0 || nv > RLGR_NV_LIMIT || B < 1 || B > RLGR_B_MAX) return GSC_ERR_INVALID_ARG;
    return GSC_OK;
}
uint64_t rlgr_blocks(int64_t nv, int32_t C, int32_t B) { return (uint64_t)((nv + B - 1) / B) * (uint64_t)C; }
uint64_t rlgr_table_bytes(int64_t nv, int32_t C, int32_t B)
{
    return sizeof(gsc_rlgr_header) + 4ull * (rlgr_blocks(nv, C, B) + 1);
}
}  // namespace

extern "C" {

gsc_status gsc_rlgr_capacity(int64_t nv, int32_t C, int32_t B, size_t *bytes)
{
    if (!bytes) return GSC_ERR_INVALID_ARG;
    gsc_status st = rlgr_shape(nv, C, B);
    if (st != GSC_OK) return st;
    // at most 1 + 10 + 1 + 24 + 32 = 68 bits per value, and one partial word per block
    *bytes = (size_t)(rlgr_table_bytes(nv, C, B) + 4ull * (((uint64_t)nv * C * 68 + 31) / 32 + rlgr_blocks(nv, C, B)));
    return GSC_OK;
}

gsc_status gsc_rlgr_workspace_size(int64_t nv, int32_t B, size_t *bytes)
{
    if (!bytes) return GSC_ERR_INVALID_ARG;
    gsc_status st = rlgr_shape(nv, 1, B);
    if (st != GSC_OK) return st;
    *bytes = (size_t)(8ull * ((uint64_t)(nv + B - 1) / B + 1));
    return GSC_OK;
}

gsc_status gsc_rlgr_encode(const int32_t *d_q, int64_t nv, int32_t C, int32_t B, void *d_out,
                           size_t out_cap, void *d_ws, size_t ws_bytes, int32_t *d_info,
                           void *stream)
{
    gsc_status st = rlgr_shape(nv, C, B);
    if (st != GSC_OK) return st;
    if (!d_out || !d_ws || !d_info || (nv > 0 && !d_q)) return GSC_ERR_INVALID_ARG;
    size_t need = 0;
    gsc_rlgr_workspace_size(nv, B, &need);
    if (ws_bytes < need) return GSC_ERR_WORKSPACE;
    if (out_cap < rlgr_table_bytes(nv, C, B)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        sp.rd(d_q, (uint64_t)nv * C * 4);
        sp.wr(d_out, out_cap);
        sp.wr(d_ws, need);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_rlgr_encode(d_q, (uint32_t)nv, (uint32_t)C, (uint32_t)B, static_cast<uint8_t *>(d_out),
                                  out_cap, static_cast<uint64_t *>(d_ws), d_info, static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

gsc_status gsc_rlgr_decode(const void *d_in, size_t in_bytes, int64_t nv, int32_t C, int32_t B,
                           int32_t *d_q, void *d_ws, size_t ws_bytes, int32_t *d_info,
                           void *stream)
{
    gsc_status st = rlgr_shape(nv, C, B);
    if (st != GSC_OK) return st;
    if (!d_in || !d_ws || !d_info || (nv > 0 && !d_q)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < 8) return GSC_ERR_WORKSPACE;
    if (in_bytes < rlgr_table_bytes(nv, C, B)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        sp.rd(d_in, in_bytes);
        sp.wr(d_q, (uint64_t)nv * C * 4);
        sp.wr(d_ws, 8);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_rlgr_decode(static_cast<const uint8_t *>(d_in), in_bytes, (uint32_t)nv, (uint32_t)C,
                                  (uint32_t)B, d_q, static_cast<uint64_t *>(d_ws), d_info,
                                  static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

gsc_status gsc_color_workspace_size(int64_t n, size_t *bytes)
{
    if (!bytes || n < 0 || n > 0x7FFFFFFFll) return GSC_ERR_INVALID_ARG;
    *bytes = color_workspace_bytes((uint32_t)n);
    return GSC_OK;
}

static gsc_status color_shape(int64_t n, int32_t C, int32_t sh0)
{
    if (n < 0 || n > 0x7FFFFFFFll || C < 1 || C > GSC_MAX_CHANNELS || sh0 < 0 || sh0 + GSC_COLOR_SH_CHANNELS > C)
        return GSC_ERR_INVALID_ARG;
    return GSC_OK;
}

gsc_status gsc_color_forward(const float *d_attr, int64_t n, int32_t C, int32_t sh0, float *d_out,
                             float *d_klt, double *d_eig, void *d_ws, size_t ws_bytes,
                             int32_t *d_info, void *stream)
{
    gsc_status st = color_shape(n, C, sh0);
    if (st != GSC_OK) return st;
    if (!d_klt || !d_ws || !d_info || (n > 0 && (!d_attr || !d_out))) return GSC_ERR_INVALID_ARG;
    const size_t need = color_workspace_bytes((uint32_t)n);
    if (ws_bytes < need) return GSC_ERR_WORKSPACE;
    {
        Spans sp;
        sp.rd(d_attr, (uint64_t)n * C * 4);
        sp.wr(d_out, (uint64_t)n * C * 4);
        sp.wr(d_klt, GSC_COLOR_KLT_FLOATS * 4);
        sp.wr(d_eig, 3 * 15 * 8);
        sp.wr(d_ws, need);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_color_forward(d_attr, d_out, (uint32_t)n, (uint32_t)C, (uint32_t)sh0, d_klt, d_eig,
                                    static_cast<double *>(d_ws), d_info, static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

gsc_status gsc_color_inverse(const float *d_coef, int64_t n, int32_t C, int32_t sh0,
                             const float *d_klt, float *d_out, void *stream)
{
    gsc_status st = color_shape(n, C, sh0);
    if (st != GSC_OK) return st;
    if (!d_klt || (n > 0 && (!d_coef || !d_out))) return GSC_ERR_INVALID_ARG;
    {
        Spans sp;
        sp.rd(d_coef, (uint64_t)n * C * 4);
        sp.rd(d_klt, GSC_COLOR_KLT_FLOATS * 4);
        sp.wr(d_out, (uint64_t)n * C * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_color_inverse(d_coef, d_out, (uint32_t)n, (uint32_t)C, (uint32_t)sh0, d_klt,
                                    static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

static gsc_status rans_shape(int64_t n, int32_t K)
{
    if (n < 0 || n > 0x7FFFFFFFll || K < 1 || K > (1 << 20)) return GSC_ERR_INVALID_ARG;
    return GSC_OK;
}

gsc_status gsc_rans_capacity(int64_t n, int32_t K, size_t *bytes)
{
    gsc_status st = rans_shape(n, K);
    if (st != GSC_OK || !bytes) return GSC_ERR_INVALID_ARG;
    *bytes = (size_t)rans_capacity_bytes((uint64_t)n, (uint32_t)K);
    return GSC_OK;
}

gsc_status gsc_rans_workspace_size(int64_t n, int32_t K, size_t *bytes)
{
    gsc_status st = rans_shape(n, K);
    if (st != GSC_OK || !bytes) return GSC_ERR_INVALID_ARG;
    *bytes = (size_t)rans_workspace_bytes((uint64_t)n, (uint32_t)K);
    return GSC_OK;
}

gsc_status gsc_rans_encode(const void *d_in, int64_t n, int32_t K, void *d_out, size_t out_cap,
                           void *d_ws, size_t ws_bytes, int32_t *d_info, void *stream)
{
    gsc_status st = rans_shape(n, K);
    if (st != GSC_OK) return st;
    if (!d_out || !d_ws || !d_info || (n > 0 && !d_in)) return GSC_ERR_INVALID_ARG;
    if ((((uintptr_t)d_out | (uintptr_t)d_ws) & 7u) || ((uintptr_t)d_info & 3u)) return GSC_ERR_INVALID_ARG;
    const uint64_t need = rans_workspace_bytes((uint64_t)n, (uint32_t)K);
    if (ws_bytes < need) return GSC_ERR_WORKSPACE;
    const uint64_t nc = rans_chunks((uint64_t)n, (uint32_t)K);
    if (out_cap < sizeof(gsc_rans_header) + 512 + 4 * (nc + 1)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        sp.rd(d_in, (uint64_t)n);
        sp.wr(d_out, out_cap);
        sp.wr(d_ws, need);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_rans_encode(static_cast<const uint8_t *>(d_in), (uint64_t)n, (uint32_t)K,
                                  static_cast<uint8_t *>(d_out), out_cap, d_ws, d_info,
                                  static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

gsc_status gsc_rans_decode(const void *d_in, size_t in_bytes, int64_t n, int32_t K, void *d_out,
                           void *d_ws, size_t ws_bytes, int32_t *d_info, void *stream)
{
    gsc_status st = rans_shape(n, K);
    if (st != GSC_OK) return st;
    if (!d_in || !d_ws || !d_info || (n > 0 && !d_out)) return GSC_ERR_INVALID_ARG;
    if ((((uintptr_t)d_in | (uintptr_t)d_ws) & 7u) || ((uintptr_t)d_info & 3u)) return GSC_ERR_INVALID_ARG;
    if (ws_bytes < 8) return GSC_ERR_WORKSPACE;
    const uint64_t nc = rans_chunks((uint64_t)n, (uint32_t)K);
    if (in_bytes < sizeof(gsc_rans_header) + 512 + 4 * (nc + 1)) return GSC_ERR_CAPACITY;
    {
        Spans sp;
        sp.rd(d_in, in_bytes);
        sp.wr(d_out, (uint64_t)n);
        sp.wr(d_ws, 8);
        sp.wr(d_info, GSC_INFO_WORDS * 4);
        if (!sp.disjoint()) return GSC_ERR_INVALID_ARG;
    }
    GSC_LAUNCH(launch_rans_decode(static_cast<const uint8_t *>(d_in), in_bytes, (uint64_t)n, (uint32_t)K,
                                  static_cast<uint8_t *>(d_out), d_ws, d_info, static_cast<hipStream_t>(stream)));
    return GSC_OK;
}

}  // extern "C"
