/*
 * Self-check driver of the CPU oracle (oracle/gsc_oracle.c), built together with it under the
 * address and undefined-behaviour sanitizers by tests/test_oracle_sanitized.py. It calls every
 * exported function on small frames, including the error paths (corrupt streams, too small
 * capacities, bad arguments), and checks a few results that hold by construction (decode of
 * an encode gives back the voxels, inverse of forward gives back the rows). Any invalid access,
 * leak or undefined operation makes the sanitizers fail the run. Test infrastructure only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t orc_morton_encode(uint32_t x, uint32_t y, uint32_t z, int J);
void orc_morton_decode(uint64_t m, int J, uint32_t *xyz);
int orc_voxelize(const float *pos, int64_t n, int J, int bbox_mode, double *bbox_min,
                 double *cell, uint32_t *vox);
int64_t orc_sort_merge(const uint64_t *keys, const float *attr, int64_t n, int C,
                       uint64_t *leaf, double *vattr, int64_t *perm, int64_t *voxel_of);
int64_t orc_octree_levels(const uint64_t *leaf, int64_t nv, int J, uint64_t *nodes, int64_t cap,
                          int64_t *off, int64_t *sizes);
int64_t orc_octree_encode(const uint64_t *leaf, int64_t nv, int J, int64_t *level_sizes,
                          uint8_t *occ, int64_t occ_cap);
int64_t orc_octree_decode(const uint8_t *occ, int64_t occ_bytes, const int64_t *level_sizes,
                          int J, uint64_t *leaf_out, int64_t cap);
void orc_voxel_centres(const uint64_t *leaf, int64_t nv, int J, const double *bbox_min,
                       double cell, uint32_t *vox_out, double *pos_out);
int64_t orc_raht_prelude(const uint64_t *M, int64_t nv, int J, int64_t *I, int64_t *W,
                         uint8_t *F, int64_t *lev_off, int64_t cap);
int64_t orc_raht_prelude_cap(int64_t nv, int J);
int orc_raht_forward(const uint64_t *M, int64_t nv, int J, double *Y, int C);
int orc_raht_inverse(const uint64_t *M, int64_t nv, int J, double *Y, int C);
void orc_quantize(const double *Y, int64_t nv, int C, const float *step, double tau, int32_t *Q);
void orc_dequantize(const int32_t *Q, int64_t nv, int C, const float *step, double *Y);
int orc_encode_frame(const float *pos, const float *attr, int64_t n, int J, int C,
                     const float *step, double tau, int bbox_mode, double *bbox_min, double *cell,
                     uint64_t *leaf, int64_t *level_sizes, uint8_t *occ, int64_t occ_cap,
                     int32_t *Q, double *Y, double *vattr, int64_t *res);
int64_t orc_decode_frame(const uint8_t *occ, int64_t occ_bytes, const int64_t *level_sizes,
                         int J, int C, const int32_t *Q, const float *step,
                         const double *bbox_min, double cell, int64_t cap, uint64_t *leaf_out,
                         uint32_t *vox_out, double *pos_out, double *attr_out);
int orc_ste_grad(const float *pos, const float *attr, int64_t n, int J, int C, const float *step,
                 double tau, double lambda, int bbox_mode, double *bbox_min, double *cell,
                 uint64_t *leaf, int64_t *voxel_of, double *aref, double *yhat, double *ahat,
                 double *grad, double *loss, int64_t *res);

static int failures = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void frame(int64_t n, int J, int C, int dup)
{
    float *pos = malloc((size_t)(n ? n : 1) * 3 * sizeof(float));
    float *attr = malloc((size_t)(n ? n : 1) * C * sizeof(float));
    for (int64_t i = 0; i < n * 3; ++i) pos[i] = (float)(dup ? floor(urand() * 4) / 4 : urand());
    for (int64_t i = 0; i < n * C; ++i) attr[i] = (float)(urand() * 2 - 1);
    float step[8];
    for (int c = 0; c < C; ++c) step[c] = 1.0f / 16;
    const int64_t m = n ? n : 1;
    uint64_t *leaf = malloc((size_t)m * 8);
    int64_t sizes[22];
    const int64_t occ_cap = m * J;
    uint8_t *occ = malloc((size_t)occ_cap);
    int32_t *Q = malloc((size_t)m * C * 4);
    double *Y = malloc((size_t)m * C * 8), *va = malloc((size_t)m * C * 8);
    double bmin[3] = {0, 0, 0}, cell = 0;
    int64_t res[2] = {0, 0};
    int rc = orc_encode_frame(pos, attr, n, J, C, step, 0.5, 0, bmin, &cell, leaf, sizes, occ,
                              occ_cap, Q, Y, va, res);
    CHECK(rc == 0);
    const int64_t nv = res[0];
    /* too small an occupancy capacity is reported, not overrun */
    if (res[1] > 1) {
        int64_t r2[2];
        CHECK(orc_encode_frame(pos, attr, n, J, C, step, 0.5, 0, bmin, &cell, leaf, sizes, occ,
                               res[1] - 1, Q, NULL, NULL, r2) < 0);
    }
    uint64_t *leaf2 = malloc((size_t)m * 8);
    uint32_t *vox = malloc((size_t)m * 12);
    double *cen = malloc((size_t)m * 24), *dec = malloc((size_t)m * C * 8);
    int64_t nv2 = orc_decode_frame(occ, res[1], sizes, J, C, Q, step, bmin, cell, m, leaf2, vox,
                                   cen, dec);
    CHECK(nv2 == nv);
    for (int64_t i = 0; i < nv && nv2 == nv; ++i) CHECK(leaf2[i] == leaf[i]);
    if (nv > 1) {
        CHECK(orc_decode_frame(occ, res[1], sizes, J, C, Q, step, bmin, cell, nv - 1, leaf2, vox,
                               cen, dec) < 0); /* capacity */
        uint8_t *bad = malloc((size_t)res[1]);
        memcpy(bad, occ, (size_t)res[1]);
        bad[res[1] - 1] = 0; /* a node without children */
        CHECK(orc_octree_decode(bad, res[1], sizes, J, leaf2, m) == -4);
        CHECK(orc_octree_decode(occ, res[1] - 1, sizes, J, leaf2, m) == -4); /* truncated */
        free(bad);
    }
    /* the transform and its inverse */
    if (nv > 0) {
        double *A = malloc((size_t)nv * C * 8);
        memcpy(A, va, (size_t)nv * C * 8);
        CHECK(orc_raht_forward(leaf, nv, J, A, C) == 0);
        CHECK(orc_raht_inverse(leaf, nv, J, A, C) == 0);
        for (int64_t i = 0; i < nv * C; ++i) CHECK(fabs(A[i] - va[i]) < 1e-12);
        int64_t cap = orc_raht_prelude_cap(nv, J);
        int64_t *I = malloc((size_t)cap * 8), *W = malloc((size_t)cap * 8);
        uint8_t *F = malloc((size_t)cap);
        int64_t off[64];
        CHECK(orc_raht_prelude(leaf, nv, J, I, W, F, off, cap) > 0);
        CHECK(orc_raht_prelude(leaf, nv, J, I, W, F, off, nv - 1 > 0 ? nv - 1 : 0) < 0);
        free(I);
        free(W);
        free(F);
        int32_t *Q2 = malloc((size_t)nv * C * 4);
        double *Y2 = malloc((size_t)nv * C * 8);
        orc_quantize(Y, nv, C, step, 0.5, Q2);
        orc_dequantize(Q2, nv, C, step, Y2);
        for (int64_t i = 0; i < nv * C; ++i) CHECK(Q2[i] == Q[i]);
        free(Q2);
        free(Y2);
        free(A);
        uint64_t *nodes = malloc((size_t)(nv * (J + 1) + 1) * 8);
        int64_t lo[22], sz[22];
        CHECK(orc_octree_levels(leaf, nv, J, nodes, nv * (J + 1) + 1, lo, sz) > 0);
        CHECK(orc_octree_levels(leaf, nv, J, nodes, 1, lo, sz) < 0); /* capacity */
        free(nodes);
    }
    /* the sort with every optional output, and the straight-through gradient */
    uint64_t *keys = malloc((size_t)m * 8);
    uint32_t *v3 = malloc((size_t)m * 12);
    CHECK(orc_voxelize(pos, n, J, 0, bmin, &cell, v3) == 0);
    for (int64_t i = 0; i < n; ++i) keys[i] = orc_morton_encode(v3[3 * i], v3[3 * i + 1], v3[3 * i + 2], J);
    int64_t *perm = malloc((size_t)m * 8), *vof = malloc((size_t)m * 8);
    CHECK(orc_sort_merge(keys, attr, n, C, leaf2, va, perm, vof) == nv);
    double *aref = malloc((size_t)m * C * 8), *yh = malloc((size_t)m * C * 8);
    double *ah = malloc((size_t)m * C * 8), *gr = malloc((size_t)m * C * 8), loss[3];
    int64_t r1[1];
    CHECK(orc_ste_grad(pos, attr, n, J, C, step, 0.5, 0.01, 0, bmin, &cell, leaf2, vof, aref, yh,
                       ah, gr, loss, r1) == 0);
    CHECK(r1[0] == nv);
    uint32_t xyz[3];
    if (nv > 0) {
        orc_morton_decode(leaf[nv - 1], J, xyz);
        CHECK(orc_morton_encode(xyz[0], xyz[1], xyz[2], J) == leaf[nv - 1]);
        orc_voxel_centres(leaf, nv, J, bmin, cell, vox, cen);
    }
    free(keys);
    free(v3);
    free(perm);
    free(vof);
    free(aref);
    free(yh);
    free(ah);
    free(gr);
    free(leaf2);
    free(vox);
    free(cen);
    free(dec);
    free(pos);
    free(attr);
    free(leaf);
    free(occ);
    free(Q);
    free(Y);
    free(va);
}

int main(void)
{
    frame(0, 4, 3, 0);
    frame(1, 5, 3, 0);
    frame(2, 1, 2, 0);
    frame(300, 6, 5, 0);
    frame(500, 3, 4, 1);  /* many Gaussians per voxel */
    frame(200, 21, 3, 0); /* 63-bit codes */
    /* bad arguments */
    double bmin[3] = {0, 0, 0}, cell = 0;
    uint32_t vox[3];
    float p[3] = {0, 0, 0};
    CHECK(orc_voxelize(p, 1, 0, 0, bmin, &cell, vox) < 0);
    CHECK(orc_voxelize(p, 1, 3, 1, bmin, &cell, vox) < 0); /* given cell must be > 0 */
    CHECK(orc_octree_encode(NULL, -1, 3, NULL, NULL, 0) < 0);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle self-check ok\n");
    return 0;
}
