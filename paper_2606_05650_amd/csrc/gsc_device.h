// Device helpers shared by the kernels: frame lookup, error flag, wave primitives,
// single-pass decoupled look-back, Morton bit spreading, and the quantizer decision.
#pragma once

#include "gsc_internal.h"

namespace gsc {

// Pointers read from a frame descriptor are generic; accesses through them compile to flat
// instructions, which also count against the LDS wait counter, so an LDS wait in a loop would
// also wait for every outstanding global store. Hot paths cast them to the global address space.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ inline GAS T *gp(T *p)
{
    return (GAS T *)p;
}
// Memory that no thread writes while a kernel runs (a frame descriptor, sizes written by earlier
// kernels) can be read through the constant address space: uniform reads then compile to scalar
// loads, which wait on the LDS/scalar counter only and so never wait for vector loads in flight.
#define CAS __attribute__((address_space(4)))
template <class T>
__device__ inline const CAS T *cp(const T *p)
{
    return (const CAS T *)p;
}
// 16-byte global accesses through clang's native vectors (HIP's float4/int4 classes cannot bind
// to global-address-space references).
typedef float gf4 __attribute__((ext_vector_type(4)));
typedef int gi4 __attribute__((ext_vector_type(4)));
__device__ inline float4 gload4(const GAS float *p)
{
    const gf4 v = *reinterpret_cast<const GAS gf4 *>(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline void gstore4(GAS float *p, const float4 &v)
{
    gf4 t;
    t.x = v.x;
    t.y = v.y;
    t.z = v.z;
    t.w = v.w;
    *reinterpret_cast<GAS gf4 *>(p) = t;
}
__device__ inline int4 gload4i(const GAS int32_t *p)
{
    const gi4 v = *reinterpret_cast<const GAS gi4 *>(p);
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ inline void gstore4i(GAS int32_t *p, const int4 &v)
{
    gi4 t;
    t.x = v.x;
    t.y = v.y;
    t.z = v.z;
    t.w = v.w;
    *reinterpret_cast<GAS gi4 *>(p) = t;
}

// ------------------------------------------------------------------------- frame lookup
__device__ inline uint32_t frame_of(const TileMap &m, uint32_t b)
{
    uint32_t f = 0;
    while (f + 1 < m.F && b >= m.start[f + 1]) ++f;
    return f;
}

// Tile of this workgroup inside its frame. Kernels with a decoupled look-back use it directly
// (no atomic tile counter: same-address atomics serialize at about 11 ns each, 11 us for a
// thousand workgroups). A tile waits only on lower tiles, and workgroups of a frame are
// dispatched to each XCD in index order, so the lowest unfinished tile is always resident;
// every wait is also bounded by SPIN_LIMIT, which turns a stall into GSC_ERR_INTERNAL.
__device__ inline uint32_t tile_index(const TileMap &m, uint32_t f) { return blockIdx.x - m.start[f]; }

__device__ inline void set_error(Ctrl *c, uint32_t code)
{
    atomicCAS(&c->error, 0u, code);
}

__device__ inline uint32_t load_error(const Ctrl *c)
{
    return __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------------- wave primitives
__device__ inline uint32_t lane_id() { return __lane_id(); }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Wave-wide minimum / maximum, returned to every lane (a workgroup-wide reduction through
// same-address LDS atomics serializes: measured 14 us for 1536 of them on 6 addresses).
__device__ inline float wave_min(float v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = fminf(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ inline float wave_max(float v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ inline uint32_t wave_umin(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = min(v, (uint32_t)__shfl_xor(v, o, WAVE));
    return v;
}
__device__ inline uint32_t wave_umax(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = max(v, (uint32_t)__shfl_xor(v, o, WAVE));
    return v;
}

// Exclusive scan over the NT threads of a block. `tmp` holds NT/64 + 1 words of LDS.
// Returns the exclusive prefix of v; *total receives the block total. Ends with a barrier.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *tmp, uint32_t *total)
{
    constexpr int NW = NT / WAVE;
    const uint32_t inc = wave_incl_scan(v);
    const uint32_t w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; ++i) {
            uint32_t t = tmp[i];
            tmp[i] = run;
            run += t;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    const uint32_t r = tmp[w] + inc - v;
    if (total) *total = tmp[NW];
    __syncthreads();
    return r;
}

// Exclusive scan within groups of GS consecutive threads (GS a multiple of 64) of an NT-thread
// block. `tmp` holds NT/64 words of LDS. Returns the exclusive prefix of v inside its group;
// *total receives the group total. Every thread of the block must call it; ends with a barrier.
template <int NT, int GS>
__device__ inline uint32_t group_excl_scan(uint32_t v, uint32_t *tmp, uint32_t *total)
{
    const uint32_t inc = wave_incl_scan(v);
    const uint32_t w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) tmp[w] = inc;
    __syncthreads();
    const uint32_t g0 = (threadIdx.x / GS) * (GS / WAVE);
    uint32_t pre = 0, tot = 0;
    for (uint32_t i = g0; i < g0 + GS / WAVE; ++i) {
        const uint32_t t = tmp[i];
        if (i < w) pre += t;
        tot += t;
    }
    if (total) *total = tot;
    __syncthreads();
    return pre + inc - v;
}

// ------------------------------------------------------------ decoupled look-back scan
// A tile publishes its aggregate, walks back over its predecessors' status words until it
// meets an inclusive prefix, then publishes its own inclusive prefix. A tile is its workgroup's
// index within the frame (tile_index): it never waits on a later tile, and a spin limit turns
// a (never expected) stall into an error.
//
// A status word carries its value in the same atomic word as its flag, and a tile uses nothing
// but those values, so relaxed device-scope atomics suffice (no cache-wide acquire/release).
// The walk issues several predecessor loads at a time (a window per thread, per wave or per
// workgroup); one dependent round costs about half a microsecond.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

// Level ordering inside a persistent launch whose workgroups are all resident. A workgroup that
// has written a level's outputs makes them visible device-wide (release: every wave writes its
// stores back past its XCD's L2) and then stores the phase number in its own flag word; a
// workgroup that reads the level waits until the flags of all np producers show the phase,
// then acquires (the XCD's L2 and the CU's L1 are invalidated, so later loads see the
// producers' data). One wave fences for the workgroup, after a workgroup barrier: a write-back
// of the L2 per wave was measured to cost more than the levels' work. One flag per workgroup: the producers never contend on a counter, and the
// consumer polls them all at once. A spin limit turns a stall into GSC_ERR_INTERNAL.
__device__ inline void level_publish(uint32_t *flags, uint32_t phase)
{
    __syncthreads();  // (workgroup scope: the other waves' stores are ordered before wave 0's fence)
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[blockIdx.x], phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
// Producers b0, b0 + 1, ... (np of them, modulo G).
__device__ inline void level_wait_range(const uint32_t *flags, uint32_t b0, uint32_t np, uint32_t G, uint32_t phase, Ctrl *ctrl)
{
    for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const uint32_t b = b0 + t < G ? b0 + t : b0 + t - G;
        uint32_t spins = 0;
        while (__hip_atomic_load(&flags[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < phase) {
            if (++spins > SPIN_LIMIT) {
                set_error(ctrl, GSC_ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // (caches shared by the workgroup)
    __syncthreads();
}
__device__ inline void level_wait(const uint32_t *flags, uint32_t np, uint32_t phase, Ctrl *ctrl)
{
    level_wait_range(flags, 0, np, np, phase, ctrl);
}

// 64-bit status word: [63:62] flag (0 none, 1 aggregate, 2 inclusive), [61:0] value.
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1ull;

__device__ inline void st_relaxed(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_relaxed(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_relaxed32(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ld_relaxed32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct OpSum {
    __device__ static uint64_t identity() { return 0; }
    __device__ static uint64_t combine(uint64_t older, uint64_t newer) { return older + newer; }
};

// (count, byte): value = count << 8 | byte. Combining appends a segment: counts add, and the
// byte restarts at the newer part when it contains a segment head (count > 0).
struct OpSegOr {
    __device__ static uint64_t identity() { return 0; }
    __device__ static uint64_t combine(uint64_t older, uint64_t newer)
    {
        const uint64_t cnt = (older >> 8) + (newer >> 8);
        const uint64_t byte = (newer >> 8) ? (newer & 0xFF) : ((older | newer) & 0xFF);
        return (cnt << 8) | byte;
    }
};

// Ordered combination of lanes [0, cnt) of a wave under Op, lane 0 being the newest value and
// higher lanes older ones; the result is returned to every lane.
template <class Op>
__device__ inline uint64_t wave_combine_ordered(uint64_t v, uint32_t cnt)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int k = 1; k < WAVE; k <<= 1) {
        const uint64_t older = __shfl_down(v, k, WAVE);
        if (lane + k < cnt) v = Op::combine(older, v);
    }
    return __shfl(v, 0, WAVE);
}

// The same look-back performed by a whole wave: each step reads the 64 nearest predecessors at
// once, so the inclusive prefix frontier advances 64 tiles per load latency. Every lane of the
// calling wave must call it; the result is returned to every lane.
template <class Op>
__device__ inline uint64_t lookback_wave(uint64_t *status, uint32_t stride, uint32_t tile,
                                         uint64_t agg, Ctrl *ctrl)
{
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0) st_relaxed(&status[0], LB_INC | agg);
        return Op::identity();
    }
    if (lane == 0) st_relaxed(&status[(size_t)tile * stride], LB_AGG | agg);
    uint64_t acc = Op::identity();
    int64_t j = (int64_t)tile - 1;  // nearest predecessor not yet combined (uniform)
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = j - (int64_t)lane;
        const uint64_t w = idx >= 0 ? ld_relaxed(&status[(size_t)idx * stride]) : (LB_INC | Op::identity());
        const uint32_t flag = (uint32_t)(w >> 62);
        const uint64_t inc_mask = __ballot(flag == 2);
        const uint64_t zero_mask = __ballot(flag == 0);
        const uint32_t cut = inc_mask ? (uint32_t)(__ffsll((long long)inc_mask) - 1) : (uint32_t)(WAVE - 1);
        const uint64_t need = cut == WAVE - 1 ? ~0ull : ((2ull << cut) - 1ull);
        const uint64_t blocked = zero_mask & need;
        // lanes before the first one that is not ready can always be combined
        const uint32_t cnt = blocked ? (uint32_t)(__ffsll((long long)blocked) - 1) : cut + 1;
        if (cnt > 0) acc = Op::combine(wave_combine_ordered<Op>(w & LB_VAL, cnt), acc);
        j -= (int64_t)cnt;
        if (!blocked) {
            if (inc_mask) break;
            continue;
        }
        if (++spins > SPIN_LIMIT) {
            if (lane == 0) set_error(ctrl, GSC_ERR_INTERNAL);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) st_relaxed(&status[(size_t)tile * stride], LB_INC | Op::combine(acc, agg));
    return acc;
}

// LDS scratch of lookback_block for a workgroup of NWV waves.
template <int NWV>
struct LbScratch {
    uint32_t inc[NWV], zero[NWV];
    uint64_t part[NWV];
};

// The look-back performed by a whole workgroup of NT threads: each round reads the NT nearest
// predecessors at once (thread t reads tile j - t), so tiles whose predecessors have all
// published their aggregates resolve in about one round per NT tiles instead of one per 64.
// Every thread of the workgroup must call it (it contains barriers); the exclusive prefix is
// returned to every thread.
// The look-back in two halves, so that a workgroup can publish its aggregate as soon as it is
// known and resolve its prefix after other work: lookback_block_publish (one store by thread 0;
// tile 0 publishes its inclusive value), then lookback_block_resolve with the same aggregate.
template <class Op>
__device__ inline void lookback_block_publish(uint64_t *status, uint32_t stride, uint32_t tile, uint64_t agg)
{
    if (threadIdx.x == 0) st_relaxed(&status[(size_t)tile * stride], (tile == 0 ? LB_INC : LB_AGG) | agg);
}

template <class Op, int NT>
__device__ inline uint64_t lookback_block_resolve(uint64_t *status, uint32_t stride, uint32_t tile,
                                                  uint64_t agg, Ctrl *ctrl, LbScratch<NT / WAVE> &sc)
{
    constexpr int NWV = NT / WAVE;
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    if (tile == 0) return Op::identity();
    uint64_t acc = Op::identity();
    int64_t j = (int64_t)tile - 1;  // nearest predecessor not yet combined (uniform)
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = j - (int64_t)tid;
        const uint64_t v = idx >= 0 ? ld_relaxed(&status[(size_t)idx * stride]) : (LB_INC | Op::identity());
        const uint32_t flag = (uint32_t)(v >> 62);
        const uint64_t inc_m = __ballot(flag == 2), zero_m = __ballot(flag == 0);
        if (lane == 0) {
            sc.inc[w] = inc_m ? w * WAVE + (uint32_t)(__ffsll((long long)inc_m) - 1) : (uint32_t)NT;
            sc.zero[w] = zero_m ? w * WAVE + (uint32_t)(__ffsll((long long)zero_m) - 1) : (uint32_t)NT;
        }
        __syncthreads();
        uint32_t first_inc = NT, first_zero = NT;
#pragma unroll
        for (int ww = 0; ww < NWV; ++ww) {
            first_inc = min(first_inc, sc.inc[ww]);
            first_zero = min(first_zero, sc.zero[ww]);
        }
        const bool found = first_inc < (uint32_t)NT;
        const uint32_t cut = found ? first_inc : (uint32_t)(NT - 1);
        const bool blocked = first_zero <= cut;
        // reads [0, cnt) are combined: up to the nearest inclusive one, or up to the first that
        // is not ready
        const uint32_t cnt = blocked ? first_zero : cut + 1;
        const uint32_t wb = w * WAVE;
        const uint32_t wcnt = cnt > wb ? min(cnt - wb, (uint32_t)WAVE) : 0u;
        const uint64_t part = wcnt ? wave_combine_ordered<Op>(v & LB_VAL, wcnt) : Op::identity();
        if (lane == 0) sc.part[w] = part;
        __syncthreads();
        uint64_t win = Op::identity();
#pragma unroll
        for (int ww = NWV - 1; ww >= 0; --ww) win = Op::combine(win, sc.part[ww]);  // older first
        acc = Op::combine(win, acc);
        j -= (int64_t)cnt;
        __syncthreads();  // scratch is rewritten by the next round
        if (!blocked) {
            if (found) break;
            continue;
        }
        if (++spins > SPIN_LIMIT) {
            if (tid == 0) set_error(ctrl, GSC_ERR_INTERNAL);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (tid == 0) st_relaxed(&status[(size_t)tile * stride], LB_INC | Op::combine(acc, agg));
    return acc;
}

template <class Op, int NT>
__device__ inline uint64_t lookback_block(uint64_t *status, uint32_t stride, uint32_t tile,
                                          uint64_t agg, Ctrl *ctrl, LbScratch<NT / WAVE> &sc)
{
    lookback_block_publish<Op>(status, stride, tile, agg);
    return lookback_block_resolve<Op, NT>(status, stride, tile, agg, ctrl, sc);
}

// 32-bit status words for the radix sort: [31:30] flag, [29:0] count (n < 2^30). A tile first
// publishes its aggregate (tile 0 its inclusive count) and adds it, with one arrival, to its
// group's word (groups of `group` tiles, at most WIN + 1); then it resolves its exclusive prefix
// from its own group's earlier tiles and the earlier groups' words, the first window of each
// loaded at once. A group word is a sum while arrivals ([29:25]) are fewer than `group`, the
// group's total once they are all in, and the inclusive count through the group's end once the
// group's last tile has resolved (it stores that only after every arrival, so that no addition
// lands on it). With every tile publishing at about the same time, a tile needs about one round
// of device-scope loads instead of t / WIN. A tile waits only on tiles of lower index.
constexpr uint32_t LB32_AGG = 1u << 30, LB32_INC = 2u << 30, LB32_VAL = (1u << 30) - 1u;
constexpr uint32_t LB32_ARRIVAL = 1u << 25, LB32_GSUM = LB32_ARRIVAL - 1u;

__device__ inline void lookback32_publish(uint32_t *status, uint32_t *gstatus, uint32_t stride, uint32_t group,
                                          uint32_t tile, uint32_t agg)
{
    st_relaxed32(&status[(size_t)tile * stride], (tile == 0 ? LB32_INC : LB32_AGG) | agg);
    __hip_atomic_fetch_add(&gstatus[(size_t)(tile / group) * stride], LB32_ARRIVAL | agg, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Loads status words hi, hi - 1, ..., down to lo (at most WIN of them; 0 past lo).
template <int WIN>
__device__ __attribute__((always_inline)) inline void lookback32_load(const uint32_t *status, uint32_t stride, int64_t hi,
                                                                     int64_t lo, uint32_t (&w)[WIN])
{
#pragma unroll
    for (int i = 0; i < WIN; ++i) w[i] = (hi - i >= lo) ? ld_relaxed32(&status[(size_t)(hi - i) * stride]) : 0u;
}

// Adds the loaded words of hi, hi - 1, ... (down to lo) to acc up to the first inclusive word
// (inc) or the first one not ready (stalled); returns the number of words added. Tile words are
// ready once published; group words (group > 0) once every arrival is in or inclusive.
template <int WIN>
__device__ __attribute__((always_inline)) inline int lookback32_take(const uint32_t (&w)[WIN], int64_t hi, int64_t lo,
                                                                    uint32_t group, uint32_t &acc, bool &inc,
                                                                    bool &stalled)
{
    int used = 0;
    bool stop = false;
    inc = stalled = false;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {  // predicated (no break) so w stays in registers
        const uint32_t flag = w[i] >> 30;
        const bool is_inc = flag == 2;
        const bool ready = group ? (is_inc || (w[i] >> 25) == group) : flag != 0;
        const uint32_t v = is_inc ? (w[i] & LB32_VAL) : group ? (w[i] & LB32_GSUM) : (w[i] & LB32_VAL);
        const bool in = !stop && hi - i >= lo;
        if (in && ready) {
            acc += v;
            ++used;
        }
        if (in && !ready) stalled = true;
        if (in && (!ready || is_inc)) {
            inc = inc || is_inc;
            stop = true;
        }
    }
    return used;
}

// Adds the values of status words hi, hi - 1, ..., lo (WIN per round, waiting for words not
// ready) to acc, or of the words down to the first inclusive one; returns true if it met an
// inclusive word (or gave up at the spin limit, with GSC_ERR_INTERNAL set).
template <int WIN>
__device__ __attribute__((always_inline)) inline bool lookback32_walk(const uint32_t *status, uint32_t stride, int64_t hi,
                                                                     int64_t lo, uint32_t group, uint32_t &acc,
                                                                     Ctrl *ctrl)
{
    int64_t j = hi;
    uint32_t spins = 0;
    while (j >= lo) {
        uint32_t w[WIN];
        lookback32_load<WIN>(status, stride, j, lo, w);
        bool inc, stalled;
        j -= lookback32_take<WIN>(w, j, lo, group, acc, inc, stalled);
        if (inc) return true;
        if (stalled) {
            if (++spins > SPIN_LIMIT) {
                set_error(ctrl, GSC_ERR_INTERNAL);
                return true;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return false;
}

template <int WIN>
__device__ __attribute__((always_inline)) inline uint32_t lookback32_resolve(uint32_t *status, uint32_t *gstatus,
                                                                            uint32_t stride, uint32_t group, uint32_t tile,
                                                                            uint32_t agg, Ctrl *ctrl)
{
    const uint32_t g = tile / group, g0 = g * group;
    uint32_t acc = 0;
    if (tile > 0) {
        // the group's earlier tiles (at most WIN) and the first window of the earlier groups, at once
        uint32_t wa[WIN], wb[WIN];
        lookback32_load<WIN>(status, stride, (int64_t)tile - 1, (int64_t)g0, wa);
        if (g > 0) lookback32_load<WIN>(gstatus, stride, (int64_t)g - 1, 0, wb);
        bool inc, stalled;
        const int ua = lookback32_take<WIN>(wa, (int64_t)tile - 1, (int64_t)g0, 0, acc, inc, stalled);
        // (in group 0 this always ends at tile 0's inclusive word)
        const bool done =
            inc || (stalled && lookback32_walk<WIN>(status, stride, (int64_t)tile - 1 - ua, (int64_t)g0, 0, acc, ctrl));
        if (!done && g > 0) {
            const int ub = lookback32_take<WIN>(wb, (int64_t)g - 1, 0, group, acc, inc, stalled);
            if (!inc) lookback32_walk<WIN>(gstatus, stride, (int64_t)g - 1 - ub, 0, group, acc, ctrl);
        }
        st_relaxed32(&status[(size_t)tile * stride], LB32_INC | (acc + agg));
    }
    if (tile - g0 == group - 1) {
        // the group's word becomes its inclusive count once every tile of the group has added to it
        uint32_t *gw = &gstatus[(size_t)g * stride];
        uint32_t spins = 0;
        while ((ld_relaxed32(gw) >> 25) != group) {
            if (++spins > SPIN_LIMIT) {
                set_error(ctrl, GSC_ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        st_relaxed32(gw, LB32_INC | (acc + agg));
    }
    return acc;
}

// ------------------------------------------------------------------------ Morton bits
// Spread the low 21 bits of v to every third bit (bit b -> bit 3b).
__device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
// Inverse of spread3: gather every third bit (bit 3b -> bit b).
__device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x ^ (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x ^ (x >> 8)) & 0x1F0000FF0000FFull;
    x = (x ^ (x >> 16)) & 0x1F00000000FFFFull;
    x = (x ^ (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}
// Code z_{J-1} y_{J-1} x_{J-1} ... z_0 y_0 x_0 (x least significant), Sec. 2.2.
__device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

__device__ inline int msb64(uint64_t x) { return 63 - __clzll((long long)x); }

// Binary level at which leaf i (i > 0) becomes a right sibling: one more than the highest bit
// in which its code differs from leaf i-1's.
__device__ inline uint8_t merge_level(uint64_t prev, uint64_t cur)
{
    return (uint8_t)(msb64(prev ^ cur) + 1);
}

// ------------------------------------------------------------------------- quantizer
// q = sgn(y) floor(|y|/step + tau), taken exactly for the given float y: the quotient is exact
// when the step is a power of two (a multiply by its exact reciprocal), else it is the
// correctly rounded FP64 quotient; floor(t + tau) is floor(t) plus one when the exact
// fractional part reaches 1 - tau (compared in FP64, where 1 - tau is exact).
__device__ inline int32_t quantize(float y, float step, float inv_step, double omt, bool pow2)
{
    const float ay = fabsf(y);
    int32_t q;
    if (pow2) {
        const float t = ay * inv_step;
        const float f = floorf(t);
        q = (int32_t)f + (((double)(t - f)) >= omt ? 1 : 0);
    } else {
        const double t = (double)ay / (double)step;
        const double f = floor(t);
        q = (int32_t)f + ((t - f) >= omt ? 1 : 0);
    }
    return y < 0.0f ? -q : q;
}

// The smallest float not below x > 0: for a float f, f >= x exactly when f >= ceil_float(x).
__device__ inline float ceil_float(double x)
{
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// The power-of-two case of `quantize` with the FP64 comparison replaced by the equivalent float
// one: the fractional part t - floor(t) is a float, so it reaches 1 - tau exactly when it reaches
// thr = ceil_float(1 - tau).
__device__ inline int32_t quantize_pow2(float y, float inv_step, float thr)
{
    const float t = fabsf(y) * inv_step;
    const float f = floorf(t);
    const int32_t q = (int32_t)f + ((t - f) >= thr ? 1 : 0);
    return y < 0.0f ? -q : q;
}

// ------------------------------------------------------------------ end of a call
// Stream geometry from the new-node depth histogram: |L_d| = #{v : D_v <= d}; level d's bytes
// start at GSC_HEADER_BYTES + sum_{d' < d} |L_d'|; the coefficients at the next multiple of 256.
struct StreamGeom {
    uint32_t level_sizes[GSC_MAX_DEPTH + 1];
    uint64_t occ_off[GSC_MAX_DEPTH + 1];
    uint64_t occ_bytes, coef_offset, total;
};
// LDS of one wave finishing one frame (indexed by depth or level: in registers it would live in
// scratch).
struct FinishScratch {
    uint32_t hist[GSC_MAX_DEPTH + 2], lvl[MAXK + 2];
    uint32_t err, nv;
    StreamGeom g;
};
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// One wave (lane t) ends frame fd's call: the device status goes to the info words and (encode)
// the stream header is written. The counters are loaded by all lanes at once and the header
// fields written in parallel: a single lane would pay one memory latency per dependent step.
__device__ inline void finish_frame(const CAS FrameDesc &fd, uint32_t t, FinishScratch &S)
{
    Ctrl *ctrl = fd.ctrl;
    const uint32_t J = fd.J, K = fd.K;
    if (t <= GSC_MAX_DEPTH) S.hist[t] = t <= J ? ctrl->hist_D[t] : 0u;
    // (the upper levels' sizes may have been written by the launch that runs this: coherent loads)
    if (t <= MAXK) S.lvl[t] = t <= K ? __hip_atomic_load(&ctrl->lvl_n[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    if (t == 0) {
        S.err = load_error(ctrl);
        S.nv = ctrl->n_vox;
    }
    wave_sync();
    const uint32_t err = S.err, nv = S.nv;
    uint64_t total = 0;
    StreamGeom &g = S.g;
    if (fd.mode == MODE_ENCODE) {
        if (t == 0) {
            uint32_t run = 0;
            uint64_t off = GSC_HEADER_BYTES;
            for (uint32_t d = 0; d <= J; ++d) {
                run += S.hist[d];
                g.level_sizes[d] = run;
                g.occ_off[d] = off;
                if (d < J) off += run;
            }
            g.occ_bytes = off - GSC_HEADER_BYTES;
            g.coef_offset = align_up(off, 256);
            g.total = g.coef_offset + (uint64_t)nv * fd.C * 4;
        }
        wave_sync();
        total = g.total;
        gsc_header *h = reinterpret_cast<gsc_header *>(fd.stream);
        for (uint32_t b = sizeof(gsc_header) + t; b < GSC_HEADER_BYTES; b += WAVE) fd.stream[b] = 0;
        for (uint64_t b = GSC_HEADER_BYTES + g.occ_bytes + t; b < g.coef_offset; b += WAVE) fd.stream[b] = 0;
        if (t < 22) h->level_sizes[t] = t <= J ? g.level_sizes[t] : 0u;
        h->quant_step[t] = t < fd.C ? fd.step[t] : 0.0f;
        if (t < 3) h->bbox_min[t] = ctrl->bbox_min[t];
        if (t == 0) {
            h->magic = GSC_MAGIC;
            h->version = GSC_VERSION;
            h->J = J;
            h->C = fd.C;
            h->n_in = fd.n;
            h->n_vox = nv;
            h->error = err;
            h->flags = fd.flags;
            h->cell = ctrl->cell;
            h->tau = fd.tau;
            h->reserved1 = 0;
            h->occ_offset = GSC_HEADER_BYTES;
            h->occ_bytes = g.occ_bytes;
            h->coef_offset = g.coef_offset;
            h->coef_bytes = (uint64_t)nv * fd.C * 4;
            h->total_bytes = g.total;
        }
    }
    if (fd.info && t == 0) {
        fd.info[0] = (int32_t)err;
        fd.info[1] = (int32_t)nv;
        fd.info[2] = (int32_t)(uint32_t)(total & 0xFFFFFFFFu);
        fd.info[3] = (int32_t)(uint32_t)(total >> 32);
        uint32_t used = 0;
        for (uint32_t k = 1; k <= K; ++k)
            if (k == 1 ? nv >= 1 : S.lvl[k] >= 2) used = k;
        fd.info[4] = (int32_t)used;
    }
}

// ------------------------------------------------------------------ decoded leaves
// Writes decoded leaf v: its voxel centre min + (coordinate + 1/2) * cell (FP64, rounded once to
// float) and, when asked for, its code and voxel coordinates.
template <class FD>
__device__ inline void emit_leaf(FD &fd, const gsc_header *h, uint32_t v, uint64_t code)
{
    if (fd.codes_out) gp(fd.codes_out)[v] = code;
    const uint32_t xyz[3] = {compact3(code), compact3(code >> 1), compact3(code >> 2)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (fd.vox_out) gp(fd.vox_out)[(size_t)v * 3 + a] = xyz[a];
        const double c = __dadd_rn(h->bbox_min[a], __dmul_rn(__dadd_rn((double)xyz[a], 0.5), h->cell));
        gp(fd.pos_out)[(size_t)v * 3 + a] = (float)c;
    }
}

}  // namespace gsc
