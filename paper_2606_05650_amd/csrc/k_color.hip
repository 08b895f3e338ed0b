// Colour decorrelation applied before the transform (Sec. 4, "Improving Compression"): every SH
// function's RGB triple goes to YUV, and each of the Y, U and V channels gets a per-frame
// Karhunen-Loeve transform over its 15 AC SH coefficients (the DC coefficients get YUV only).
// The decoder undoes both after the inverse transform. The paper gives no coefficients; this
// implementation takes these choices:
//   * YUV: the BT.601 luma weights Kr = 0.299, Kb = 0.114 and chroma ranges Umax = 0.436,
//     Vmax = 0.615 (the host builds the matrix and its inverse from these four numbers);
//   * the 48 SH channels start at column sh0: DC of R, G, B, then the 15 AC functions of R, of G
//     and of B; the output keeps that layout with YUV channels in place of colours and KLT
//     coefficients in place of functions;
//   * the KLT of a channel: eigenvectors of the covariance (about the mean) of its 15 AC values
//     over the frame's rows, in decreasing eigenvalue order, each with its largest-magnitude
//     component positive; coefficients a = E^T x, inverse x = E a; fewer than two rows: E = I.
//
// Launches: the Gram matrices of the three channels (with a constant-one feature for the sums) on
// the matrix cores, their per-block partials folded in a fixed order, the eigenvectors (FP64
// Jacobi, one wave per channel), and the per-row transform with rows staged through LDS.
#include "gsc_device.h"

namespace gsc {

typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr int COL_AC = 15;             // AC SH functions per colour
constexpr int COL_F = 16;              // features of a Gram matrix: 15 AC values and a constant 1
constexpr int COL_ENT = 3 * COL_F * COL_F;
constexpr int COL_STAT_THREADS = 512;  // 8 waves
constexpr int COL_STAT_WAVES = COL_STAT_THREADS / WAVE;
constexpr int COL_GROUPS = 16;         // 4-row MFMA groups summed in FP32 before joining the FP64 sums
constexpr int COL_UNROLL = 4;          // groups whose loads are issued together
constexpr uint32_t COL_ROWS_ALIGN = 4 * COL_GROUPS;
constexpr int COL_APPLY_ROWS = WAVE;  // rows of a chunk, one per thread
constexpr uint32_t COL_APPLY_GRID = 2048;  // workgroups of a per-row launch (eight per CU)

struct ColorArgs {
    const float *in;     // [n][C]
    float *out;          // [n][C]
    float *klt;          // [3][15][15]: E[c][i][j] = component i of basis vector j
    double *eig;         // [3][15] or null
    double *part;        // [blocks][3][16][16] Gram partial sums
    int32_t *info;
    uint32_t n, C, sh0, rows_per_wave, blocks;
    float m[9];          // (Y, U, V) = m (R, G, B), row-major
    float mi[9];         // its inverse
};

// ---------------------------------------------------------------------------- Gram matrices
// Wave w of block b takes rows [r0, r0 + rows_per_wave). Lane l feeds row 4g + l / 16 of a
// 4-row group and feature l % 16 (feature 15: the constant 1) as both operands of a 16x16x4
// FP32 MFMA, which accumulates D[i][j] += sum_k X[k][i] X[k][j] over the group's rows k; lane l
// holds D[4 (l / 16) + v][l % 16] in element v. Every COL_GROUPS groups (64 rows) the FP32 sums
// join FP64 accumulators. The 8 waves' sums are added in LDS (FP64) and the block's partial
// written out, to be summed in a fixed order by the next launch.
__global__ __launch_bounds__(COL_STAT_THREADS) void k_color_stats(ColorArgs a)
{
    __shared__ double s_p[COL_STAT_WAVES][COL_ENT];
    const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
    const uint32_t k = lane >> 4, f = lane & 15u;
    const uint32_t r0 = (blockIdx.x * COL_STAT_WAVES + w) * a.rows_per_wave;
    const uint32_t r1 = min(r0 + a.rows_per_wave, a.n);
    const GAS float *in = gp(a.in);
    const uint32_t fc = min(f, (uint32_t)COL_AC - 1);  // (feature 15 reads a valid column, replaced by 1)
    double acc64[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[c][v] = 0.0;
    for (uint32_t r = r0; r < r1; r += COL_ROWS_ALIGN) {
        mf4 acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = mf4{0.f, 0.f, 0.f, 0.f};
        for (int g = 0; g < COL_GROUPS; g += COL_UNROLL) {
            float R[COL_UNROLL], G[COL_UNROLL], B[COL_UNROLL];
            bool ok[COL_UNROLL];
#pragma unroll
            for (int u = 0; u < COL_UNROLL; ++u) {
                const uint32_t row = r + 4u * (uint32_t)(g + u) + k;
                ok[u] = row < r1;
                const GAS float *p = in + (size_t)min(row, r1 - 1) * a.C + a.sh0 + 3 + fc;
                R[u] = p[0];
                G[u] = p[COL_AC];
                B[u] = p[2 * COL_AC];
            }
#pragma unroll
            for (int u = 0; u < COL_UNROLL; ++u) {
                float x[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[c] = a.m[3 * c] * R[u] + a.m[3 * c + 1] * G[u] + a.m[3 * c + 2] * B[u];
                    if (f == 15u) x[c] = 1.f;
                    if (!ok[u]) x[c] = 0.f;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[c], x[c], acc[c], 0, 0, 0);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[c][v] += (double)acc[c][v];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) s_p[w][c * COL_F * COL_F + (4 * k + v) * COL_F + f] = acc64[c][v];
    __syncthreads();
    GAS double *part = gp(a.part) + (size_t)blockIdx.x * COL_ENT;
    for (uint32_t e = threadIdx.x; e < (uint32_t)COL_ENT; e += COL_STAT_THREADS) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < COL_STAT_WAVES; ++ww) s += s_p[ww][e];
        part[e] = s;
    }
}

// The blocks' partials folded into COL_FOLD groups (group g: blocks g, g + COL_FOLD, ..., summed
// in that order), so that the eigenvector launch adds COL_FOLD values per entry, not one per block.
constexpr int COL_FOLD = 8;
constexpr int COL_FOLD_THREADS = 256;
__global__ __launch_bounds__(COL_FOLD_THREADS) void k_color_fold(ColorArgs a)
{
    const uint32_t gid = blockIdx.x * COL_FOLD_THREADS + threadIdx.x;
    if (gid >= (uint32_t)(COL_FOLD * COL_ENT)) return;
    const uint32_t g = gid / COL_ENT, e = gid % COL_ENT;
    const GAS double *part = gp(a.part);
    double s = 0.0;
    uint32_t b = g;
    for (; b + 3 * COL_FOLD < a.blocks; b += 4 * COL_FOLD) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(b + u * COL_FOLD) * COL_ENT + e];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u];
    }
    for (; b < a.blocks; b += COL_FOLD) s += part[(size_t)b * COL_ENT + e];
    gp(a.part)[(size_t)(a.blocks + g) * COL_ENT + e] = s;  // (after the blocks' partials)
}

// ------------------------------------------------------------------------------ eigenvectors
constexpr int COL_BASIS_THREADS = 1024;
constexpr int JACOBI_SWEEPS_MAX = 30;

__device__ inline void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Cyclic Jacobi on the symmetric 16x16 matrix A (index 15 a zero padding row and column), one
// wave: each step applies 8 rotations on disjoint index pairs (round-robin order, 15 steps per
// sweep), rows first, then columns, then the eigenvector matrix V (starting as I). A rotation
// zeroes A[p][q] (the symmetric Schur decomposition of Golub and Van Loan). Sweeps stop when
// the off-diagonal energy is below 1e-26 of the diagonal's, or after JACOBI_SWEEPS_MAX.
__device__ inline void jacobi16(double (*A)[COL_F], double (*V)[COL_F], double *s_c, double *s_s, uint32_t *s_pq)
{
    const uint32_t lane = lane_id();
    for (uint32_t i = lane; i < COL_F * COL_F; i += WAVE) V[i / COL_F][i % COL_F] = (i / COL_F == i % COL_F) ? 1.0 : 0.0;
    wsync();
    for (int sweep = 0; sweep < JACOBI_SWEEPS_MAX; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (uint32_t i = lane; i < COL_F * COL_F; i += WAVE) {
            const double x = A[i / COL_F][i % COL_F];
            if (i / COL_F == i % COL_F) dia += x * x;
            else off += x * x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, WAVE);
            dia += __shfl_xor(dia, o, WAVE);
        }
        if (off <= 1e-26 * dia || off == 0.0) break;
        for (int step = 0; step < COL_F - 1; ++step) {
            if (lane < 8) {
                // players: 0 fixed, the others rotated by the step; pair i = (players[i], players[15 - i])
                auto player = [&](uint32_t j) -> uint32_t { return j == 0 ? 0u : 1u + (j - 1u + (uint32_t)step) % (COL_F - 1); };
                uint32_t p = player(lane), q = player(COL_F - 1 - lane);
                if (p > q) {
                    const uint32_t t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                const double apq = A[p][q];
                if (q < (uint32_t)COL_AC && apq != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau)) : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                s_c[lane] = c;
                s_s[lane] = s;
                s_pq[lane] = p | (q << 8);
            }
            wsync();
            // rows: (J^T A)[p][:] = c A[p][:] - s A[q][:], (J^T A)[q][:] = s A[p][:] + c A[q][:]
            {
                const uint32_t pr = lane / 8, j0 = (lane % 8) * 2;
                const uint32_t p = s_pq[pr] & 255u, q = s_pq[pr] >> 8;
                const double c = s_c[pr], s = s_s[pr];
                double ap[2], aq[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    ap[u] = A[p][j0 + u];
                    aq[u] = A[q][j0 + u];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    A[p][j0 + u] = c * ap[u] - s * aq[u];
                    A[q][j0 + u] = s * ap[u] + c * aq[u];
                }
            }
            wsync();
            // columns of A and of V: (X J)[:][p] = c X[:][p] - s X[:][q], (X J)[:][q] = s X[:][p] + c X[:][q]
            {
                const uint32_t pr = lane / 8, i0 = (lane % 8) * 2;
                const uint32_t p = s_pq[pr] & 255u, q = s_pq[pr] >> 8;
                const double c = s_c[pr], s = s_s[pr];
                double xp[4], xq[4];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    xp[u] = A[i0 + u][p];
                    xq[u] = A[i0 + u][q];
                    xp[2 + u] = V[i0 + u][p];
                    xq[2 + u] = V[i0 + u][q];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    A[i0 + u][p] = c * xp[u] - s * xq[u];
                    A[i0 + u][q] = s * xp[u] + c * xq[u];
                    V[i0 + u][p] = c * xp[2 + u] - s * xq[2 + u];
                    V[i0 + u][q] = s * xp[2 + u] + c * xq[2 + u];
                }
            }
            wsync();
        }
    }
}

// One workgroup: the folded Gram partials summed in group order (FP64), each channel's
// covariance about the mean, its eigenvectors (wave c: channel c), sorted by decreasing
// eigenvalue with the canonical sign, written as E[c] (and the eigenvalues).
__global__ __launch_bounds__(COL_BASIS_THREADS) void k_color_basis(ColorArgs a)
{
    __shared__ double s_g[COL_ENT];
    __shared__ double s_A[3][COL_F][COL_F], s_V[3][COL_F][COL_F];
    __shared__ double s_c[3][8], s_s[3][8];
    __shared__ uint32_t s_pq[3][8];
    const uint32_t t = threadIdx.x;
    const GAS double *fold = gp(a.part) + (size_t)a.blocks * COL_ENT;  // k_color_fold's groups
    if (t < (uint32_t)COL_ENT) {
        double v[COL_FOLD];
#pragma unroll
        for (int g = 0; g < COL_FOLD; ++g) v[g] = a.blocks ? fold[(size_t)g * COL_ENT + t] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < COL_FOLD; ++g) s += v[g];
        s_g[t] = s;
    }
    __syncthreads();
    const uint32_t w = t / WAVE, lane = lane_id();
    if (w >= 3) return;
    const uint32_t c = w;
    const double *G = s_g + c * COL_F * COL_F;
    const double n = (double)a.n;
    // covariance about the mean (row and column 15: the padding, zero)
    for (uint32_t e = lane; e < COL_F * COL_F; e += WAVE) {
        const uint32_t i = e / COL_F, j = e % COL_F;
        double v = 0.0;
        if (a.n >= 2 && i < (uint32_t)COL_AC && j < (uint32_t)COL_AC) {
            const double mi = G[i * COL_F + 15] / n, mj = G[j * COL_F + 15] / n;
            v = G[i * COL_F + j] / n - mi * mj;
        }
        s_A[c][i][j] = v;
    }
    wsync();
    jacobi16(s_A[c], s_V[c], s_c[c], s_s[c], s_pq[c]);
    // lane j < 15: eigenpair j's rank (decreasing eigenvalue, index order on ties) and sign
    if (lane < (uint32_t)COL_AC) {
        const uint32_t j = lane;
        const double lj = s_A[c][j][j];
        uint32_t rank = 0;
        for (uint32_t i = 0; i < (uint32_t)COL_AC; ++i) {
            const double li = s_A[c][i][i];
            rank += (li > lj || (li == lj && i < j)) ? 1u : 0u;
        }
        uint32_t im = 0;
        double best = -1.0;
        for (uint32_t i = 0; i < (uint32_t)COL_AC; ++i) {
            const double m = fabs(s_V[c][i][j]);
            if (m > best) {
                best = m;
                im = i;
            }
        }
        const double sg = s_V[c][im][j] < 0.0 ? -1.0 : 1.0;
        GAS float *E = gp(a.klt) + c * COL_AC * COL_AC;
        for (uint32_t i = 0; i < (uint32_t)COL_AC; ++i) E[i * COL_AC + rank] = (float)(sg * s_V[c][i][j]);
        if (a.eig) gp(a.eig)[c * COL_AC + rank] = a.n >= 2 ? lj : 0.0;
    }
    if (c == 0 && lane == 0 && a.info) {
        a.info[0] = 0;
        a.info[1] = (int32_t)a.n;
    }
}

// ------------------------------------------------------------------------------ per row
// A workgroup (one wave) takes the chunks of COL_APPLY_ROWS rows b, b + G, ... (G workgroups,
// a few per CU). A chunk is staged in LDS (rows padded to an odd stride, so that the threads'
// accesses to one column of their rows fall in distinct banks) from registers loaded one chunk
// ahead with coalesced loads (16-byte ones when the rows allow): the next chunk's loads are in
// flight while each thread transforms one row of the current one (forward: YUV, then
// a_c = E_c^T x_c; inverse: x_c = E_c a_c, then RGB) and the rows leave with coalesced stores.
// Columns outside the SH range are copied. The loads are unconditional at clamped positions
// (past the last chunk a workgroup re-reads its own, and never uses it).
constexpr int COL_APPLY_VPT = GSC_MAX_CHANNELS;  // values per thread and chunk (C <= 64)
template <bool INV, bool VEC>
__global__ __launch_bounds__(COL_APPLY_ROWS) __attribute__((amdgpu_waves_per_eu(VEC ? 2 : 1))) void k_color_apply(ColorArgs a)
{
    extern __shared__ float s_rows[];
    __shared__ float s_E[3 * COL_AC * COL_AC];
    const uint32_t t = threadIdx.x, C = a.C, P = C | 1u;  // padded row stride (odd)
    const uint32_t nchunk = (a.n + COL_APPLY_ROWS - 1) / COL_APPLY_ROWS;
    uint32_t ch = blockIdx.x;
    if (ch >= nchunk) return;  // (uniform: the grid has at most one workgroup per chunk)
    constexpr int NL = VEC ? COL_APPLY_VPT / 4 : COL_APPLY_VPT;  // loads per thread and chunk
    float4 r4[VEC ? NL : 1];
    float r1[VEC ? 1 : NL];
    auto load = [&](uint32_t c) {
        const uint32_t row0 = c * COL_APPLY_ROWS, nval = min((uint32_t)COL_APPLY_ROWS, a.n - row0) * C;
        const GAS float *src = gp(a.in) + (size_t)row0 * C;
        if (VEC) {  // C % 4 == 0 and 16-byte aligned rows: a float4 never straddles two rows
#pragma unroll
            for (int u = 0; u < NL; ++u) r4[u] = gload4(src + 4 * min(t + (uint32_t)u * COL_APPLY_ROWS, nval / 4 - 1));
        } else {
#pragma unroll
            for (int u = 0; u < NL; ++u) r1[u] = src[min(t + (uint32_t)u * COL_APPLY_ROWS, nval - 1)];
        }
    };
    load(ch);
    for (uint32_t i = t; i < 3u * COL_AC * COL_AC; i += COL_APPLY_ROWS) s_E[i] = gp(a.klt)[i];
    for (; ch < nchunk; ch += gridDim.x) {
        const uint32_t row0 = ch * COL_APPLY_ROWS;
        const uint32_t nr = min((uint32_t)COL_APPLY_ROWS, a.n - row0);
        const uint32_t nval = nr * C;
        __syncthreads();  // the previous chunk's rows are no longer read from LDS
        if (VEC) {
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                const uint32_t i = t + (uint32_t)u * COL_APPLY_ROWS;
                if (i < nval / 4) {
                    float *d = s_rows + ((4 * i) / C) * P + (4 * i) % C;
                    d[0] = r4[u].x;
                    d[1] = r4[u].y;
                    d[2] = r4[u].z;
                    d[3] = r4[u].w;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                const uint32_t i = t + (uint32_t)u * COL_APPLY_ROWS;
                if (i < nval) s_rows[(i / C) * P + i % C] = r1[u];
            }
        }
        __syncthreads();
        load(ch + gridDim.x < nchunk ? ch + gridDim.x : ch);  // the next chunk's rows
        if (t < nr) {
            float *x = s_rows + t * P + a.sh0;
            const float *M = INV ? a.mi : a.m;
            // DC: the 3x3 step only
            {
                const float d0 = x[0], d1 = x[1], d2 = x[2];
#pragma unroll
                for (int c = 0; c < 3; ++c) x[c] = M[3 * c] * d0 + M[3 * c + 1] * d1 + M[3 * c + 2] * d2;
            }
            float v[3][COL_AC];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < COL_AC; ++k) v[c][k] = x[3 + COL_AC * c + k];
            if (!INV) {
                // YUV per function (in place: function k's three values only), then each
                // channel's KLT
#pragma unroll
                for (int k = 0; k < COL_AC; ++k) {
                    const float r = v[0][k], g = v[1][k], b = v[2][k];
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[c][k] = M[3 * c] * r + M[3 * c + 1] * g + M[3 * c + 2] * b;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int j = 0; j < COL_AC; ++j) {
                        float s = 0.f;
#pragma unroll
                        for (int i = 0; i < COL_AC; ++i) s += s_E[(c * COL_AC + i) * COL_AC + j] * v[c][i];
                        x[3 + COL_AC * c + j] = s;
                    }
            } else {
                // each channel's KLT undone (one channel's 15 values at a time, back into v), then
                // RGB per function
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float y[COL_AC];
#pragma unroll
                    for (int i = 0; i < COL_AC; ++i) {
                        float s = 0.f;
#pragma unroll
                        for (int j = 0; j < COL_AC; ++j) s += s_E[(c * COL_AC + i) * COL_AC + j] * v[c][j];
                        y[i] = s;
                    }
#pragma unroll
                    for (int i = 0; i < COL_AC; ++i) v[c][i] = y[i];
                }
#pragma unroll
                for (int k = 0; k < COL_AC; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        x[3 + COL_AC * c + k] = M[3 * c] * v[0][k] + M[3 * c + 1] * v[1][k] + M[3 * c + 2] * v[2][k];
            }
        }
        __syncthreads();
        GAS float *dst = gp(a.out) + (size_t)row0 * C;
        if (VEC) {
            for (uint32_t i = t; i < nval / 4; i += COL_APPLY_ROWS) {
                const float *sr = s_rows + ((4 * i) / C) * P + (4 * i) % C;
                gstore4(dst + 4 * i, make_float4(sr[0], sr[1], sr[2], sr[3]));
            }
        } else {
            for (uint32_t i = t; i < nval; i += COL_APPLY_ROWS) dst[i] = s_rows[(i / C) * P + i % C];
        }
    }
}

// ------------------------------------------------------------------------------ launches
uint32_t color_rows_per_wave(uint32_t n)
{
    const uint32_t waves = 256u * COL_STAT_WAVES;  // at most 256 blocks
    uint32_t r = (n + waves - 1) / waves;
    r = (r + COL_ROWS_ALIGN - 1) / COL_ROWS_ALIGN * COL_ROWS_ALIGN;
    return r < COL_ROWS_ALIGN ? COL_ROWS_ALIGN : r;
}
uint32_t color_stat_blocks(uint32_t n)
{
    const uint32_t per_block = color_rows_per_wave(n) * COL_STAT_WAVES;
    return n == 0 ? 0u : (n + per_block - 1) / per_block;
}
size_t color_workspace_bytes(uint32_t n)
{
    return (size_t)(color_stat_blocks(n) + COL_FOLD) * COL_ENT * sizeof(double);
}

template <bool INV>
static void launch_apply(const ColorArgs &a, hipStream_t s)
{
    const bool vec = a.C % 4 == 0 && ((uintptr_t)a.in & 15u) == 0 && ((uintptr_t)a.out & 15u) == 0;
    const uint32_t chunks = (a.n + COL_APPLY_ROWS - 1) / COL_APPLY_ROWS;
    const dim3 grid(chunks < COL_APPLY_GRID ? chunks : COL_APPLY_GRID), block(COL_APPLY_ROWS);
    const size_t lds = (size_t)COL_APPLY_ROWS * (a.C | 1u) * sizeof(float);
    if (vec) hipLaunchKernelGGL((k_color_apply<INV, true>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_color_apply<INV, false>), grid, block, lds, s, a);
}

static void yuv_matrices(float *m, float *mi)
{
    // BT.601: Y = Kr R + Kg G + Kb B, U = Umax (B - Y) / (1 - Kb), V = Vmax (R - Y) / (1 - Kr)
    const double kr = 0.299, kb = 0.114, kg = 1.0 - kr - kb, umax = 0.436, vmax = 0.615;
    const double su = umax / (1.0 - kb), sv = vmax / (1.0 - kr);
    const double f[9] = {kr, kg, kb, -su * kr, -su * kg, su * (1.0 - kb), sv * (1.0 - kr), -sv * kg, -sv * kb};
    // inverse: R = Y + V / sv, B = Y + U / su, G = (Y - Kr R - Kb B) / Kg
    const double iv = 1.0 / sv, iu = 1.0 / su;
    const double r[3] = {1.0, 0.0, iv}, b[3] = {1.0, iu, 0.0};
    const double g[3] = {(1.0 - kr - kb) / kg, (-kb * iu) / kg, (-kr * iv) / kg};
    const double inv[9] = {r[0], r[1], r[2], g[0], g[1], g[2], b[0], b[1], b[2]};
    for (int i = 0; i < 9; ++i) {
        m[i] = (float)f[i];
        mi[i] = (float)inv[i];
    }
}

hipError_t launch_color_forward(const float *in, float *out, uint32_t n, uint32_t C, uint32_t sh0, float *klt,
                                double *eig, double *part, int32_t *info, hipStream_t s)
{
    ColorArgs a;
    a.in = in;
    a.out = out;
    a.klt = klt;
    a.eig = eig;
    a.part = part;
    a.info = info;
    a.n = n;
    a.C = C;
    a.sh0 = sh0;
    a.rows_per_wave = color_rows_per_wave(n);
    a.blocks = color_stat_blocks(n);
    yuv_matrices(a.m, a.mi);
    if (a.blocks > 0) {
        hipLaunchKernelGGL(k_color_stats, dim3(a.blocks), dim3(COL_STAT_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_color_fold, dim3((COL_FOLD * COL_ENT + COL_FOLD_THREADS - 1) / COL_FOLD_THREADS),
                           dim3(COL_FOLD_THREADS), 0, s, a);
    }
    hipLaunchKernelGGL(k_color_basis, dim3(1), dim3(COL_BASIS_THREADS), 0, s, a);
    if (n > 0) launch_apply<false>(a, s);
    return hipGetLastError();
}

hipError_t launch_color_inverse(const float *in, float *out, uint32_t n, uint32_t C, uint32_t sh0, const float *klt,
                                hipStream_t s)
{
    ColorArgs a;
    a.in = in;
    a.out = out;
    a.klt = const_cast<float *>(klt);
    a.eig = nullptr;
    a.part = nullptr;
    a.info = nullptr;
    a.n = n;
    a.C = C;
    a.sh0 = sh0;
    a.rows_per_wave = 0;
    a.blocks = 0;
    yuv_matrices(a.m, a.mi);
    if (n > 0) launch_apply<true>(a, s);
    return hipGetLastError();
}

}  // namespace gsc
