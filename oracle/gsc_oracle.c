/*
 * Plain, slow CPU oracle of the GS-NFS codec hot path (positions: voxelize -> Morton -> sort ->
 * unique -> per-level octree occupancy bytes; attributes: RAHT prelude -> forward RAHT ->
 * dead-zone quantization; decode: octree expansion -> Morton decode -> dequantization ->
 * inverse RAHT).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code, header, table or helper with the
 * HIP path, and nothing here is used to produce a product result.
 *
 * Arithmetic is IEEE-754 binary64, single-threaded, built with -ffp-contract=off so that no
 * multiply-add is fused. Where the paper is silent or ambiguous the reading taken is stated at
 * the function (the same list is kept with the design notes):
 *   R1  bounding cube: per-axis minimum, one cell size from the largest extent (Sec. 2.1).
 *   R2  a coordinate is quantized by floor((p - min)/cell), clamped to 2^J - 1 (Sec. 2.1).
 *   R3  duplicates are replaced by their plain arithmetic mean, summed in input order.
 *   R4  occupancy bit i <-> child code (p << 3) + i (Alg. 1 OccKernel, Alg. 3).
 *   R5  the transform runs all 3J binary levels, leaving one DC at index 0 (Sec. 3.1 footnote
 *       context: the root keeps the low-pass; Alg. 4 builds 3J levels).
 *   R6  quantization q = sgn(y) * floor(|y| / step + tau), reconstruction q * step (Sec. 3.4).
 *   R7  the voxel-depth shift of Alg. 2 is zero (voxel depth equals octree depth).
 *   R8  (differentiable extension, not in the paper) the straight-through loss measures the
 *       decoded voxel rows against the voxel means over Nv*C values, the rate proxy sums
 *       log2(1 + |yhat|/step) over every coefficient, DC included, and sgn(0) = 0.
 *
 * Every function returns a negative value on a bad argument or a capacity overflow.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DEPTH 21

/* ---------------------------------------------------------------------------------------- */
/* Morton code, Sec. 2.2 "Morton Codes": the code of (x, y, z) is the bit string                */
/* z_{J-1} y_{J-1} x_{J-1} ... z_0 y_0 x_0, x_b being the b-th least significant bit of x;      */
/* the unused high bits of the 64-bit word are zero.                                            */
/* ---------------------------------------------------------------------------------------- */
uint64_t orc_morton_encode(uint32_t x, uint32_t y, uint32_t z, int J)
{
    uint64_t m = 0;
    for (int b = 0; b < J; ++b) {
        m |= (uint64_t)((x >> b) & 1u) << (3 * b);
        m |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        m |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return m;
}

/* The code of every row of vox[n][3] (the same interleave, applied row by row). */
void orc_morton_encode_n(const uint32_t *vox, int64_t n, int J, uint64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_morton_encode(vox[3 * i], vox[3 * i + 1], vox[3 * i + 2], J);
}

/* Inverse of the interleave: every third bit, starting at bit 0 for x, 1 for y, 2 for z. */
void orc_morton_decode(uint64_t m, int J, uint32_t *xyz)
{
    uint32_t x = 0, y = 0, z = 0;
    for (int b = 0; b < J; ++b) {
        x |= (uint32_t)((m >> (3 * b)) & 1u) << b;
        y |= (uint32_t)((m >> (3 * b + 1)) & 1u) << b;
        z |= (uint32_t)((m >> (3 * b + 2)) & 1u) << b;
    }
    xyz[0] = x;
    xyz[1] = y;
    xyz[2] = z;
}

/* ---------------------------------------------------------------------------------------- */
/* Voxelization, Sec. 2.1 and Sec. 2.2 (step (a)): the cube bounding all Gaussians is split     */
/* into 2^J x 2^J x 2^J cells and every coordinate is quantized to J bits (R1, R2).             */
/* bbox_mode 0 computes bbox_min and cell from the data and returns them; bbox_mode 1 uses the  */
/* given values.                                                                                */
/* ---------------------------------------------------------------------------------------- */
int orc_voxelize(const float *pos, int64_t n, int J, int bbox_mode, double *bbox_min,
                 double *cell, uint32_t *vox)
{
    if (J < 1 || J > ORC_MAX_DEPTH || n < 0) return -1;
    if (bbox_mode == 0) {
        double mn[3] = {0.0, 0.0, 0.0}, mx[3] = {0.0, 0.0, 0.0};
        if (n > 0) {
            for (int a = 0; a < 3; ++a) mn[a] = mx[a] = (double)pos[a];
            for (int64_t i = 1; i < n; ++i)
                for (int a = 0; a < 3; ++a) {
                    double v = (double)pos[i * 3 + a];
                    if (v < mn[a]) mn[a] = v;
                    if (v > mx[a]) mx[a] = v;
                }
        }
        double ext = 0.0;
        for (int a = 0; a < 3; ++a)
            if (mx[a] - mn[a] > ext) ext = mx[a] - mn[a];
        for (int a = 0; a < 3; ++a) bbox_min[a] = mn[a];
        *cell = ext > 0.0 ? ldexp(ext, -J) : 1.0;
    } else if (!(*cell > 0.0)) {
        return -1;
    }
    const double top = (double)((1u << J) - 1u);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double t = floor(((double)pos[i * 3 + a] - bbox_min[a]) / *cell);
            if (t < 0.0) t = 0.0;
            if (t > top) t = top;
            vox[i * 3 + a] = (uint32_t)t;
        }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Sort + unique + merge, Sec. 2.2 "Voxelization" and Alg. 1 step 1: keys are sorted with their */
/* Gaussian index (a stable order: equal keys keep input order); each run of equal keys is one  */
/* occupied voxel whose attributes are the mean of the run's rows (R3).                        */
/* ---------------------------------------------------------------------------------------- */
typedef struct {
    uint64_t key;
    int64_t idx;
} orc_pair;

static int orc_pair_cmp(const void *pa, const void *pb)
{
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* keys[n] -> leaf codes L_J[nv] (sorted, unique), the sorted order perm[n] (input index of   */
/* the k-th smallest (key, index) pair), voxel_of[n] (voxel of each input row), and the      */
/* merged attributes vattr[nv][C] (mean of attr rows). Returns nv.                            */
int64_t orc_sort_merge(const uint64_t *keys, const float *attr, int64_t n, int C,
                       uint64_t *leaf, double *vattr, int64_t *perm, int64_t *voxel_of)
{
    if (n < 0 || C < 0) return -1;
    if (n == 0) return 0;
    orc_pair *p = (orc_pair *)malloc((size_t)n * sizeof(orc_pair));
    if (!p) return -2;
    for (int64_t i = 0; i < n; ++i) {
        p[i].key = keys[i];
        p[i].idx = i;
    }
    qsort(p, (size_t)n, sizeof(orc_pair), orc_pair_cmp);
    int64_t nv = 0;
    int64_t start = 0;
    for (int64_t k = 0; k <= n; ++k) {
        if (k == n || (k > 0 && p[k].key != p[k - 1].key)) {
            /* close the run [start, k) */
            leaf[nv] = p[start].key;
            if (vattr && attr) {
                for (int c = 0; c < C; ++c) {
                    double s = 0.0;
                    for (int64_t m = start; m < k; ++m) s += (double)attr[p[m].idx * C + c];
                    vattr[nv * C + c] = s / (double)(k - start);
                }
            }
            if (voxel_of)
                for (int64_t m = start; m < k; ++m) voxel_of[p[m].idx] = nv;
            ++nv;
            start = k;
        }
        if (k < n && perm) perm[k] = p[k].idx;
    }
    free(p);
    return nv;
}

/* ---------------------------------------------------------------------------------------- */
/* Octree construction, Sec. 2.2 "Octree construction" and Alg. 1 step 2:                      */
/*   L_d = Unique({ c >> 3 : c in L_{d+1} }) for d = J-1 down to 0.                            */
/* The levels are stored one after another, L_0 first; off[d] is where L_d starts and          */
/* sizes[d] = |L_d|. Returns the total node count, or a negative value if cap is exceeded.     */
/* ---------------------------------------------------------------------------------------- */
int64_t orc_octree_levels(const uint64_t *leaf, int64_t nv, int J, uint64_t *nodes, int64_t cap,
                          int64_t *off, int64_t *sizes)
{
    if (J < 1 || J > ORC_MAX_DEPTH || nv < 0) return -1;
    /* sizes bottom-up first, into a scratch copy of each level */
    uint64_t *cur = (uint64_t *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(uint64_t));
    uint64_t **lv = (uint64_t **)calloc((size_t)J + 1, sizeof(uint64_t *));
    if (!cur || !lv) {
        free(cur);
        free(lv);
        return -2;
    }
    memcpy(cur, leaf, (size_t)nv * sizeof(uint64_t));
    sizes[J] = nv;
    lv[J] = cur;
    for (int d = J - 1; d >= 0; --d) {
        int64_t m = sizes[d + 1];
        uint64_t *nxt = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
        if (!nxt) {
            for (int e = d + 1; e <= J; ++e) free(lv[e]);
            free(lv);
            return -2;
        }
        int64_t k = 0;
        for (int64_t i = 0; i < m; ++i) {
            uint64_t par = lv[d + 1][i] >> 3; /* Parent(c) = c >> 3 */
            if (k == 0 || nxt[k - 1] != par) nxt[k++] = par; /* Unique on a sorted list */
        }
        sizes[d] = k;
        lv[d] = nxt;
    }
    int64_t total = 0;
    for (int d = 0; d <= J; ++d) {
        off[d] = total;
        total += sizes[d];
    }
    int64_t rc = total;
    if (total > cap) {
        rc = -3;
    } else {
        for (int d = 0; d <= J; ++d)
            memcpy(nodes + off[d], lv[d], (size_t)sizes[d] * sizeof(uint64_t));
    }
    for (int d = 0; d <= J; ++d) free(lv[d]);
    free(lv);
    return rc;
}

/* first index k in a[0..m) with a[k] >= v (a sorted ascending) */
static int64_t orc_lower_bound(const uint64_t *a, int64_t m, uint64_t v)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* ---------------------------------------------------------------------------------------- */
/* Occupancy bytes, Sec. 2.2 "Bitstream generation" and Alg. 1 steps 3-4 (OccKernel): for     */
/* each parent p in L_d, base = p << 3; binary-search L_{d+1} for the first code >= base; scan */
/* at most 8 entries while the code is <= base + 7 and set bit (code - base) (R4). Levels are  */
/* concatenated L_0 first, each in Morton order. level_sizes[0..J] = |L_0| .. |L_J|.           */
/* Returns the number of bytes written.                                                        */
/* ---------------------------------------------------------------------------------------- */
int64_t orc_octree_encode(const uint64_t *leaf, int64_t nv, int J, int64_t *level_sizes,
                          uint8_t *occ, int64_t occ_cap)
{
    if (J < 1 || J > ORC_MAX_DEPTH || nv < 0) return -1;
    if (nv == 0) {
        for (int d = 0; d <= J; ++d) level_sizes[d] = 0;
        return 0;
    }
    int64_t cap = nv * (int64_t)(J + 1) + 1;
    uint64_t *nodes = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
    int64_t off[ORC_MAX_DEPTH + 1];
    if (!nodes) return -2;
    int64_t total = orc_octree_levels(leaf, nv, J, nodes, cap, off, level_sizes);
    if (total < 0) {
        free(nodes);
        return total;
    }
    int64_t w = 0;
    for (int d = 0; d < J; ++d) {
        const uint64_t *Ld = nodes + off[d];
        const uint64_t *Lc = nodes + off[d + 1];
        int64_t mc = level_sizes[d + 1];
        for (int64_t k = 0; k < level_sizes[d]; ++k) {
            uint64_t base = Ld[k] << 3;
            uint32_t byte = 0;
            int64_t c = orc_lower_bound(Lc, mc, base);
            for (int j = 0; j < 8 && c + j < mc; ++j)
                if (Lc[c + j] <= base + 7) byte |= 1u << (uint32_t)(Lc[c + j] - base);
            if (w >= occ_cap) {
                free(nodes);
                return -3;
            }
            occ[w++] = (uint8_t)byte;
        }
    }
    free(nodes);
    return w;
}

static int orc_popcount8(uint32_t b)
{
    int c = 0;
    for (int i = 0; i < 8; ++i) c += (b >> i) & 1u;
    return c;
}

/* ---------------------------------------------------------------------------------------- */
/* Octree decoding, Sec. 2.3 and Alg. 2-3: L_0 = [0]; for d = 0..J-1 read |L_d| bytes, count   */
/* children (population count), exclusive prefix sum, then each parent writes (parent<<3)+i  */
/* for every set bit i, in ascending i, at its offset. level_sizes is the header's metadata:  */
/* the expansion must reproduce it, else the stream is corrupt (return -4). A zero byte is    */
/* also corrupt (an internal node always has a child). Returns |L_J|.                         */
/* ---------------------------------------------------------------------------------------- */
int64_t orc_octree_decode(const uint8_t *occ, int64_t occ_bytes, const int64_t *level_sizes,
                          int J, uint64_t *leaf_out, int64_t cap)
{
    if (J < 1 || J > ORC_MAX_DEPTH) return -1;
    if (level_sizes[J] == 0) return 0;
    if (level_sizes[0] != 1) return -4;
    int64_t maxm = 1;
    for (int d = 0; d <= J; ++d)
        if (level_sizes[d] > maxm) maxm = level_sizes[d];
    if (level_sizes[J] > cap) return -3;
    uint64_t *Ld = (uint64_t *)malloc((size_t)maxm * sizeof(uint64_t));
    uint64_t *Ln = (uint64_t *)malloc((size_t)maxm * sizeof(uint64_t));
    int64_t *offs = (int64_t *)malloc((size_t)maxm * sizeof(int64_t));
    if (!Ld || !Ln || !offs) {
        free(Ld);
        free(Ln);
        free(offs);
        return -2;
    }
    int64_t M = 1, ptr = 0, rc = 0;
    Ld[0] = 0; /* implicit root */
    for (int d = 0; d < J && rc == 0; ++d) {
        if (M != level_sizes[d] || ptr + M > occ_bytes) {
            rc = -4;
            break;
        }
        const uint8_t *Occ = occ + ptr;
        ptr += M;
        int64_t run = 0;
        for (int64_t p = 0; p < M; ++p) { /* Popcount + ExclusiveScan */
            int cnt = orc_popcount8(Occ[p]);
            if (cnt == 0) rc = -4;
            offs[p] = run;
            run += cnt;
        }
        if (rc) break;
        if (run != level_sizes[d + 1] || run > maxm) {
            rc = -4;
            break;
        }
        for (int64_t p = 0; p < M; ++p) { /* expand_children_kernel */
            uint64_t base = Ld[p] << 3;
            int64_t w = offs[p];
            for (int i = 0; i < 8; ++i)
                if (Occ[p] & (1u << i)) Ln[w++] = base + (uint64_t)i;
        }
        uint64_t *t = Ld;
        Ld = Ln;
        Ln = t;
        M = run;
    }
    if (rc == 0) memcpy(leaf_out, Ld, (size_t)M * sizeof(uint64_t));
    free(Ld);
    free(Ln);
    free(offs);
    return rc == 0 ? M : rc;
}

/* ---------------------------------------------------------------------------------------- */
/* Voxel centres, Sec. 2.1: a merged Gaussian sits at the centre of its voxel,                 */
/* min_a + (v_a + 1/2) * cell, per axis (R7: the decoded voxel depth equals J).                 */
/* ---------------------------------------------------------------------------------------- */
void orc_voxel_centres(const uint64_t *leaf, int64_t nv, int J, const double *bbox_min,
                       double cell, uint32_t *vox_out, double *pos_out)
{
    for (int64_t i = 0; i < nv; ++i) {
        uint32_t v[3];
        orc_morton_decode(leaf[i], J, v);
        for (int a = 0; a < 3; ++a) {
            if (vox_out) vox_out[i * 3 + a] = v[a];
            if (pos_out) pos_out[i * 3 + a] = bbox_min[a] + ((double)v[a] + 0.5) * cell;
        }
    }
}

/* ---------------------------------------------------------------------------------------- */
/* RAHT prelude, Sec. 3.2 and Alg. 4 (non-parallel form). For l = 1..3J:                        */
/*   I_1 = (0 .. Nv-1);  I_l = I_{l-1} with the entries right after a set F_{l-1} flag removed */
/*   W_l = [I_l(2:end); Nv] - I_l                 (run-length weights, sentinel Nv)            */
/*   F_l(k) = ((M[I_l(k)] xor M[I_l(k+1)]) and (2^{3J} - 2^l)) == 0, last entry 0.            */
/* The lists of all levels are concatenated; lev_off[l-1] is where level l starts and           */
/* lev_off[3J] the total. Returns the total, or a negative value if cap is exceeded.           */
/* ---------------------------------------------------------------------------------------- */
int64_t orc_raht_prelude(const uint64_t *M, int64_t nv, int J, int64_t *I, int64_t *W,
                         uint8_t *F, int64_t *lev_off, int64_t cap)
{
    if (J < 1 || J > ORC_MAX_DEPTH || nv < 0) return -1;
    const int L = 3 * J;
    int64_t *cur = (int64_t *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(int64_t));
    uint8_t *fl = (uint8_t *)malloc((size_t)(nv > 0 ? nv : 1));
    if (!cur || !fl) {
        free(cur);
        free(fl);
        return -2;
    }
    int64_t m = nv;
    for (int64_t k = 0; k < nv; ++k) cur[k] = k;
    int64_t w = 0, rc = 0;
    const uint64_t full = (L >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << L) - 1u);
    for (int l = 1; l <= L; ++l) {
        if (l > 1) { /* I_l = I_{l-1}(not [0; F_{l-1}]) */
            int64_t k2 = 0;
            for (int64_t k = 0; k < m; ++k)
                if (k == 0 || !fl[k - 1]) cur[k2++] = cur[k];
            m = k2;
        }
        lev_off[l - 1] = w;
        const uint64_t mask = full & ~(((uint64_t)1 << l) - 1u); /* 2^{3J} - 2^l */
        for (int64_t k = 0; k < m; ++k) {
            int64_t nxt = (k + 1 < m) ? cur[k + 1] : nv;
            fl[k] = (k + 1 < m) && (((M[cur[k]] ^ M[cur[k + 1]]) & mask) == 0);
            if (w >= cap) {
                rc = -3;
                break;
            }
            I[w] = cur[k];
            W[w] = nxt - cur[k];
            F[w] = fl[k];
            ++w;
        }
        if (rc) break;
    }
    if (rc == 0) lev_off[L] = w;
    free(cur);
    free(fl);
    return rc == 0 ? w : rc;
}

/* Bound on the prelude's total list length: every level lists at most Nv entries. */
int64_t orc_raht_prelude_cap(int64_t nv, int J) { return nv * 3 * (int64_t)J; }

/* ---------------------------------------------------------------------------------------- */
/* Forward / inverse RAHT, Eq. (1) (the 2x2 butterfly) and Alg. 6, on all 3J levels (R5).      */
/* For each set flag F_l(k): i0 = I_l(k), i1 = I_l(k+1), w0 = W_l(k), w1 = W_l(k+1),            */
/*   a = sqrt(w0 / (w0 + w1)), b = sqrt(w1 / (w0 + w1));                                       */
/*   forward : Y[i0] <-  a*y0 + b*y1 ; Y[i1] <- -b*y0 + a*y1   (levels 1 .. 3J)                */
/*   inverse : Y[i0] <-  a*y0 - b*y1 ; Y[i1] <-  b*y0 + a*y1   (levels 3J .. 1)                */
/* Y is Nv x C row-major, transformed in place. Returns 0.                                     */
/* ---------------------------------------------------------------------------------------- */
static int orc_raht_apply(const uint64_t *M, int64_t nv, int J, double *Y, int C, int inverse)
{
    if (nv <= 1) return 0;
    const int L = 3 * J;
    int64_t cap = orc_raht_prelude_cap(nv, J);
    int64_t *I = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int64_t *W = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    uint8_t *F = (uint8_t *)malloc((size_t)cap);
    int64_t lev_off[3 * ORC_MAX_DEPTH + 1];
    int64_t tot = (I && W && F) ? orc_raht_prelude(M, nv, J, I, W, F, lev_off, cap) : -2;
    if (tot < 0) {
        free(I);
        free(W);
        free(F);
        return (int)tot;
    }
    for (int s = 0; s < L; ++s) {
        int l = inverse ? (L - s) : (s + 1);
        int64_t b0 = lev_off[l - 1], b1 = lev_off[l];
        for (int64_t k = b0; k + 1 < b1; ++k) {
            if (!F[k]) continue;
            int64_t i0 = I[k], i1 = I[k + 1];
            double w0 = (double)W[k], w1 = (double)W[k + 1];
            double a = sqrt(w0 / (w0 + w1)), b = sqrt(w1 / (w0 + w1));
            double *y0p = Y + i0 * C, *y1p = Y + i1 * C;
            for (int c = 0; c < C; ++c) {
                double y0 = y0p[c], y1 = y1p[c];
                if (!inverse) {
                    y0p[c] = a * y0 + b * y1;
                    y1p[c] = -b * y0 + a * y1;
                } else {
                    y0p[c] = a * y0 - b * y1;
                    y1p[c] = b * y0 + a * y1;
                }
            }
        }
    }
    free(I);
    free(W);
    free(F);
    return 0;
}

int orc_raht_forward(const uint64_t *M, int64_t nv, int J, double *Y, int C)
{
    return orc_raht_apply(M, nv, J, Y, C, 0);
}

int orc_raht_inverse(const uint64_t *M, int64_t nv, int J, double *Y, int C)
{
    return orc_raht_apply(M, nv, J, Y, C, 1);
}

/* ---------------------------------------------------------------------------------------- */
/* Dead-zone quantization, Sec. 3.4 (R6): one step per channel for every coefficient of that  */
/* channel, q = sgn(y) floor(|y|/step + tau); reconstruction y^ = q * step.                    */
/* ---------------------------------------------------------------------------------------- */
/* The quotient t = |y|/step is the correctly rounded FP64 quotient (exact when step is a    */
/* power of two). floor(t + tau) is then taken exactly, as floor(t) plus one when the        */
/* fractional part t - floor(t) (an exact difference) reaches 1 - tau, so the sum t + tau is */
/* never rounded.                                                                             */
int32_t orc_quantize1(double y, double step, double tau)
{
    double t = fabs(y) / step;
    double f = floor(t);
    double q = f + ((t - f) >= 1.0 - tau ? 1.0 : 0.0);
    if (y < 0.0) q = -q;
    if (y == 0.0) q = 0.0;
    return (int32_t)q;
}

void orc_quantize(const double *Y, int64_t nv, int C, const float *step, double tau, int32_t *Q)
{
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < C; ++c) Q[i * C + c] = orc_quantize1(Y[i * C + c], (double)step[c], tau);
}

void orc_dequantize(const int32_t *Q, int64_t nv, int C, const float *step, double *Y)
{
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < C; ++c) Y[i * C + c] = (double)Q[i * C + c] * (double)step[c];
}

/* ---------------------------------------------------------------------------------------- */
/* Whole-frame encode: voxelize -> Morton -> sort/unique/merge -> octree bytes -> RAHT ->      */
/* quantize. Outputs (caller-allocated, capacities n rows): leaf[n], level_sizes[J+1],        */
/* occ[occ_cap], Q[n*C] (row-major, Nv rows used), optional Y[n*C] (FP64 coefficients),        */
/* optional vattr[n*C] (merged attributes), bbox_min[3] and cell (in/out as in orc_voxelize). */
/* res[0] = Nv, res[1] = occupancy bytes. Returns 0 or a negative error.                      */
/* ---------------------------------------------------------------------------------------- */
int orc_encode_frame(const float *pos, const float *attr, int64_t n, int J, int C,
                     const float *step, double tau, int bbox_mode, double *bbox_min, double *cell,
                     uint64_t *leaf, int64_t *level_sizes, uint8_t *occ, int64_t occ_cap,
                     int32_t *Q, double *Y, double *vattr, int64_t *res)
{
    if (n < 0 || C < 1) return -1;
    size_t nn = (size_t)(n > 0 ? n : 1);
    uint32_t *vox = (uint32_t *)malloc(nn * 3 * sizeof(uint32_t));
    uint64_t *keys = (uint64_t *)malloc(nn * sizeof(uint64_t));
    double *A = vattr ? vattr : (double *)malloc(nn * (size_t)C * sizeof(double));
    double *Yw = Y ? Y : (double *)malloc(nn * (size_t)C * sizeof(double));
    int64_t nv = 0, nb = 0;
    int rc = -2;
    if (!vox || !keys || !A || !Yw) goto done;
    rc = orc_voxelize(pos, n, J, bbox_mode, bbox_min, cell, vox);
    if (rc) goto done;
    for (int64_t i = 0; i < n; ++i)
        keys[i] = orc_morton_encode(vox[i * 3], vox[i * 3 + 1], vox[i * 3 + 2], J);
    nv = orc_sort_merge(keys, attr, n, C, leaf, A, NULL, NULL);
    if (nv < 0) {
        rc = (int)nv;
        goto done;
    }
    nb = orc_octree_encode(leaf, nv, J, level_sizes, occ, occ_cap);
    if (nb < 0) {
        rc = (int)nb;
        goto done;
    }
    memcpy(Yw, A, (size_t)nv * (size_t)C * sizeof(double));
    rc = orc_raht_forward(leaf, nv, J, Yw, C);
    if (rc) goto done;
    orc_quantize(Yw, nv, C, step, tau, Q);
    res[0] = nv;
    res[1] = nb;
done:
    free(vox);
    free(keys);
    if (!vattr) free(A);
    if (!Y) free(Yw);
    return rc;
}

/* Whole-frame decode: octree expansion -> voxel centres -> dequantize -> inverse RAHT.        */
/* pos_out[Nv*3] (FP64 centres), vox_out[Nv*3], attr_out[Nv*C] (FP64). Returns Nv or < 0.    */
int64_t orc_decode_frame(const uint8_t *occ, int64_t occ_bytes, const int64_t *level_sizes,
                         int J, int C, const int32_t *Q, const float *step,
                         const double *bbox_min, double cell, int64_t cap, uint64_t *leaf_out,
                         uint32_t *vox_out, double *pos_out, double *attr_out)
{
    int64_t nv = orc_octree_decode(occ, occ_bytes, level_sizes, J, leaf_out, cap);
    if (nv < 0) return nv;
    orc_voxel_centres(leaf_out, nv, J, bbox_min, cell, vox_out, pos_out);
    orc_dequantize(Q, nv, C, step, attr_out);
    int rc = orc_raht_inverse(leaf_out, nv, J, attr_out, C);
    if (rc) return rc;
    return nv;
}

/* ---------------------------------------------------------------------------------------- */
/* Straight-through coding loss and its gradient: the coder of Sec. 3 (the transform of       */
/* Eq. (1) / Alg. 6 and the quantizer of Sec. 3.4) used as a differentiable layer, with the   */
/* quantizer's derivative taken as the identity (R8):                                          */
/*   a     = voxel means of the input rows (R3); a_ref = a, held constant                      */
/*   y     = T a,  yhat = Q(y) * step,  ahat = T^T yhat (the decoder's reconstruction)         */
/*   L     = 1/(Nv C) sum (ahat - a_ref)^2 + lambda sum log2(1 + |yhat| / step)                */
/*   g_ahat = 2/(Nv C) (ahat - a_ref),  g_yhat = lambda sgn(yhat) / (ln 2 (step + |yhat|))     */
/*   g_y = T g_ahat + g_yhat,  g_a = T^T g_y,  dL/dattr[i] = g_a[voxel of i] / |voxel of i|    */
/* Outputs (capacity n rows): leaf[n], voxel_of[n], aref, yhat, ahat [Nv][C], grad [n][C];    */
/* loss[0] = L, loss[1] = distortion term, loss[2] = rate term; res[0] = Nv.                  */
/* Returns 0 or a negative error.                                                             */
/* ---------------------------------------------------------------------------------------- */
int orc_ste_grad(const float *pos, const float *attr, int64_t n, int J, int C, const float *step,
                 double tau, double lambda, int bbox_mode, double *bbox_min, double *cell,
                 uint64_t *leaf, int64_t *voxel_of, double *aref, double *yhat, double *ahat,
                 double *grad, double *loss, int64_t *res)
{
    if (n < 0 || C < 1) return -1;
    loss[0] = loss[1] = loss[2] = 0.0;
    res[0] = 0;
    if (n == 0) return 0;
    uint32_t *vox = (uint32_t *)malloc((size_t)n * 3 * sizeof(uint32_t));
    uint64_t *keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    int64_t *count = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    double *G = (double *)malloc((size_t)n * (size_t)C * sizeof(double));
    int64_t nv = 0;
    size_t rows = 0;
    double inv_nc = 0.0, dist = 0.0, rate = 0.0;
    int rc = -2;
    if (!vox || !keys || !count || !G) goto done;
    rc = orc_voxelize(pos, n, J, bbox_mode, bbox_min, cell, vox);
    if (rc) goto done;
    for (int64_t i = 0; i < n; ++i)
        keys[i] = orc_morton_encode(vox[i * 3], vox[i * 3 + 1], vox[i * 3 + 2], J);
    nv = orc_sort_merge(keys, attr, n, C, leaf, aref, NULL, voxel_of);
    if (nv < 0) {
        rc = (int)nv;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) count[voxel_of[i]] += 1;
    rows = (size_t)nv * (size_t)C;

    /* y = T a, yhat = Q(y) step, ahat = T^T yhat */
    memcpy(yhat, aref, rows * sizeof(double));
    if ((rc = orc_raht_forward(leaf, nv, J, yhat, C))) goto done;
    for (int64_t v = 0; v < nv; ++v)
        for (int c = 0; c < C; ++c) {
            const double st = (double)step[c];
            yhat[v * C + c] = (double)orc_quantize1(yhat[v * C + c], st, tau) * st;
        }
    memcpy(ahat, yhat, rows * sizeof(double));
    if ((rc = orc_raht_inverse(leaf, nv, J, ahat, C))) goto done;

    /* the loss */
    inv_nc = 1.0 / ((double)nv * (double)C);
    for (size_t k = 0; k < rows; ++k) {
        const double e = ahat[k] - aref[k];
        dist += e * e;
        rate += log2(1.0 + fabs(yhat[k]) / (double)step[k % (size_t)C]);
    }
    loss[1] = dist * inv_nc;
    loss[2] = lambda * rate;
    loss[0] = loss[1] + loss[2];

    /* g_y = T g_ahat + g_yhat, g_a = T^T g_y */
    for (size_t k = 0; k < rows; ++k) G[k] = 2.0 * inv_nc * (ahat[k] - aref[k]);
    if ((rc = orc_raht_forward(leaf, nv, J, G, C))) goto done;
    for (size_t k = 0; k < rows; ++k) {
        const double yh = yhat[k], st = (double)step[k % (size_t)C];
        const double sg = yh > 0.0 ? 1.0 : (yh < 0.0 ? -1.0 : 0.0);
        G[k] += lambda * sg / (log(2.0) * (st + fabs(yh)));
    }
    if ((rc = orc_raht_inverse(leaf, nv, J, G, C))) goto done;

    /* back through the voxel mean */
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = voxel_of[i];
        for (int c = 0; c < C; ++c) grad[i * C + c] = G[v * C + c] / (double)count[v];
    }
    res[0] = nv;
done:
    free(vox);
    free(keys);
    free(count);
    free(G);
    return rc;
}
