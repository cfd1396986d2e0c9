/*
 * CPU oracle of the interpolation-based error-bounded lossy compressor of
 * cuSZ-Hi (arXiv 2507.11165). TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the benchmark's CPU baseline call it; the product never does.
 *
 * It is the method written out plainly, one step after another, for a reader
 * to check against the paper:
 *   - error bound: Sec. 3.1 Eq. "general" and the value-range relative bound of
 *     Sec. 6.1.4;
 *   - 17^3 blocks with a stride-16 anchor grid and a 4-level hierarchy:
 *     Sec. 5.1.1;
 *   - cubic/linear spline interpolation, 1-D (dimension sequence) and
 *     multi-dimensional schemes: Sec. 5.1.2 (and the cuSZ-I background of
 *     Sec. 3.2);
 *   - sampled-block tuner: Sec. 5.1.3;
 *   - linear-scaling quantization to one-byte codes with separately stored
 *     outliers: Sec. 3.2 and Sec. 5.2.1;
 *   - Huffman encoding of the codes: Sec. 5.2.2-5.2.3 (canonical codes as in
 *     RFC 1951 Sec. 3.2.2).
 * Where the paper is silent the design notes list the reading taken; each is
 * named at the place it is used below.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off (no -ffast-math, no OpenMP).
 */
#include "hiz_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ANCHOR 16          /* anchor stride on every axis (Sec. 5.1.1) */
#define SIDE 17            /* block side including the anchors (Sec. 5.1.1) */
#define MAX_CODE_LEN 32    /* Huffman length cap (reading) */
#define MAX_N (1ull << 40) /* largest field handled */

/* Stream layout (the paper does not describe one; this is the library's own). */
#define HDR_BYTES 128
#define OFF_LEN 128
#define OFF_CHUNKS 384
#define MAGIC 0x315A4948u /* "HIZ1" */
#define VERSION 1

static const int PERM[6][3] = {
    {0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }
static int imin(int a, int b) { return a < b ? a : b; }

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Error bound                                                                */
/* ------------------------------------------------------------------------ */

/* Absolute bound epsilon. Sec. 6.1.4 states that every bound in the paper is
 * value-range relative: epsilon = eb * (max - min) (the garbled sentence is read
 * this way). The product is formed in FP64 and rounded DOWN to FP32, so the
 * FP32 bound never exceeds the requested one. */
float orc_eps(int mode, double eb, float vmin, float vmax)
{
    double e = (mode == ORC_REL) ? eb * ((double)vmax - (double)vmin) : eb;
    float f = (float)e;
    if ((double)f > e)
        f = nextafterf(f, 0.0f);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Spline stencils (Sec. 5.1.2)                                               */
/* ------------------------------------------------------------------------ */

/* Interpolation at the midpoint from the samples at -3s, -s, +s, +3s.
 * Cubic needs all four; at block edges the paper falls back to lower orders
 * (quadratic/linear); the reading ranks them cubic > quadratic > linear >
 * linear extrapolation > copy. Lagrange weights: (-1,9,9,-1)/16, (3,6,-1)/8,
 * (-1,6,3)/8, (1,1)/2, (-1,3)/2. The paper's "multiple interpolation
 * splines" (Sec. 5.1.3) add the natural cubic spline through the four
 * samples (zero second derivative at the outer two), whose value at the
 * midpoint has weights (-3,23,23,-3)/40; it falls back like the cubic. */
float orc_stencil(int spline, float a, float b, float c, float d,
                  int pa, int pc, int pd, int *rank)
{
    if (spline == ORC_CUB || spline == ORC_NAT) {
        if (pa && pc && pd) {
            *rank = 4;
            if (spline == ORC_NAT)
                return ((b + c) * 23.0f - (a + d) * 3.0f) / 40.0f;
            return ((b + c) * 9.0f - (a + d)) * 0.0625f;
        }
        if (!pa && pc && pd) {
            *rank = 3;
            return ((b * 3.0f + c * 6.0f) - d) * 0.125f;
        }
        if (pa && pc && !pd) {
            *rank = 3;
            return ((b * 6.0f + c * 3.0f) - a) * 0.125f;
        }
    }
    if (pc) {
        *rank = 2;
        return (b + c) * 0.5f;
    }
    if (pa) {
        *rank = 1;
        return b * 1.5f - a * 0.5f;
    }
    *rank = 0;
    return b;
}

/* 1-D prediction of target t along one axis with the samples at distance s. */
static float axis_pred(const float *buf, const int n[3], const int t[3], int axis,
                       int s, int spline, int *rank)
{
    const long st[3] = {(long)n[1] * n[2], n[2], 1};
    long base = ((long)t[0] * n[1] + t[1]) * n[2] + t[2];
    int tk = t[axis];
    int pa = tk - 3 * s >= 0;
    int pc = tk + s <= n[axis] - 1;
    int pd = tk + 3 * s <= n[axis] - 1;
    float a = pa ? buf[base - 3L * s * st[axis]] : 0.0f;
    float b = buf[base - (long)s * st[axis]];
    float c = pc ? buf[base + (long)s * st[axis]] : 0.0f;
    float d = pd ? buf[base + 3L * s * st[axis]] : 0.0f;
    return orc_stencil(spline, a, b, c, d, pa, pc, pd, rank);
}

/* Prediction of target t at stride s. The odd set S holds the axes on which
 * t/s is odd.
 *  - Multi-dimensional scheme (Sec. 5.1.2): interpolate along every axis of S,
 *    keep only the predictions of the highest spline order, and average them
 *    (combined in x, y, z order; three values are summed and divided by 3).
 *  - 1-D dimension-sequence scheme: the target is interpolated along the axis
 *    of S that comes last in the dimension order. */
float orc_predict(const float *buf, const int n[3], const int t[3], int s,
                  int spline, int scheme, int perm)
{
    int odd[3];
    for (int k = 0; k < 3; k++)
        odd[k] = (t[k] / s) & 1;
    if (scheme == ORC_MD) {
        float p[3] = {0, 0, 0};
        int r[3] = {-1, -1, -1};
        int best = -1;
        for (int k = 0; k < 3; k++) {
            if (!odd[k])
                continue;
            p[k] = axis_pred(buf, n, t, k, s, spline, &r[k]);
            if (r[k] > best)
                best = r[k];
        }
        float v[3];
        int m = 0;
        for (int k = 0; k < 3; k++)
            if (odd[k] && r[k] == best)
                v[m++] = p[k];
        if (m == 1)
            return v[0];
        if (m == 2)
            return (v[0] + v[1]) * 0.5f;
        return ((v[0] + v[1]) + v[2]) / 3.0f;
    }
    int axis = -1;
    for (int j = 0; j < 3; j++)
        if (odd[PERM[perm][j]])
            axis = PERM[perm][j];
    int rank;
    return axis_pred(buf, n, t, axis, s, spline, &rank);
}

/* Sub-step (1..3) in which target t of stride s is processed. The
 * multi-dimensional scheme goes 1-D -> 2-D -> 3-D targets (|S| = 1, 2, 3); the
 * dimension-sequence scheme runs one pass per axis in the given order, and a
 * target belongs to the pass of the last axis of S in that order. Targets of
 * one sub-step only read values of earlier sub-steps, levels or anchors. */
static int substep(const int t[3], int s, int scheme, int perm)
{
    int odd[3], m = 0;
    for (int k = 0; k < 3; k++) {
        odd[k] = (t[k] / s) & 1;
        m += odd[k];
    }
    if (scheme == ORC_MD)
        return m;
    int last = 0;
    for (int j = 0; j < 3; j++)
        if (odd[PERM[perm][j]])
            last = j + 1;
    return last;
}

/* ------------------------------------------------------------------------ */
/* Linear-scaling quantization (Sec. 3.2, Sec. 5.2.1)                         */
/* ------------------------------------------------------------------------ */

/* Quantize the prediction error of value x against prediction p into a one-
 * byte code 128+q with |q| <= 127; anything else, and any reconstruction that
 * FP32 rounding pushed past the bound (checked in FP64), is an outlier: code 0,
 * value kept exactly. */
static uint8_t quantize(float x, float p, float eps, float two_eb, float inv, float *xo)
{
    float diff = x - p;
    float qf = diff * inv;
    float qr = rintf(qf);
    if (!(fabsf(qr) <= 127.0f)) {
        *xo = x;
        return 0;
    }
    int q = (int)qr;
    float xr = p + ((float)q * two_eb);
    if (!(fabs((double)x - (double)xr) <= (double)eps)) {
        *xo = x;
        return 0;
    }
    *xo = xr;
    return (uint8_t)(q + 128);
}

/* ------------------------------------------------------------------------ */
/* Blocks (Sec. 5.1.1)                                                        */
/* ------------------------------------------------------------------------ */

/* Block (a,b,c) starts at 16*(a,b,c); it spans min(17, d-o) points per axis
 * (the +1 plane is shared with the next block) and owns the first
 * min(16, d-o) of them. */
typedef struct {
    uint64_t o[3];
    int n[3];
    int own[3];
} block;

static block make_block(const uint64_t dims[3], uint64_t a, uint64_t b, uint64_t c)
{
    block k;
    uint64_t ab[3] = {a, b, c};
    for (int i = 0; i < 3; i++) {
        k.o[i] = ab[i] * ANCHOR;
        uint64_t rem = dims[i] - k.o[i];
        k.n[i] = (int)(rem < SIDE ? rem : SIDE);
        k.own[i] = imin(k.n[i], ANCHOR);
    }
    return k;
}

static uint64_t gindex(const uint64_t dims[3], uint64_t x, uint64_t y, uint64_t z)
{
    return (x * dims[1] + y) * dims[2] + z;
}

#ifdef ORC_FACE_CHECK
/* Debug check of the shared faces (built only with -DORC_FACE_CHECK): a
 * block computes the points of its +1 faces itself, and those values must
 * agree bit for bit with the values every other block containing the point
 * computed (its owner's included). Each computed point is noted once per
 * block; a second note with other bits counts as a mismatch. */
static float *fc_val;
static uint8_t *fc_set;
static uint64_t fc_mismatch;

uint64_t orc_face_mismatches(void) { return fc_mismatch; }

static int fc_begin(uint64_t N)
{
    fc_mismatch = 0;
    free(fc_val);
    free(fc_set);
    fc_val = malloc(sizeof(float) * (N ? N : 1));
    fc_set = calloc(N ? N : 1, 1);
    return fc_val && fc_set;
}

static void fc_note_block(const float *buf, const block *k, const uint64_t dims[3])
{
    for (int i = 0; i < k->n[0]; i++)
        for (int j = 0; j < k->n[1]; j++)
            for (int m = 0; m < k->n[2]; m++) {
                const uint64_t g = gindex(dims, k->o[0] + i, k->o[1] + j, k->o[2] + m);
                const float v = buf[(i * k->n[1] + j) * k->n[2] + m];
                if (fc_set[g]) {
                    if (memcmp(&fc_val[g], &v, sizeof(float)) != 0)
                        fc_mismatch++;
                } else {
                    fc_set[g] = 1;
                    fc_val[g] = v;
                }
            }
}
#endif

/* Walk the levels of one block (strides 8, 4, 2, 1), sub-step by sub-step.
 * Compression (codes_in == NULL) predicts from reconstructed values, quantizes
 * and replaces each value by its reconstruction before any later target reads
 * it; decompression rebuilds each target from its code. */
static void run_levels(float *buf, const block *k, const uint8_t cfg[4][3],
                       float eps, float two_eb, float inv,
                       const uint8_t *codes_in, uint8_t *codes_out,
                       const uint64_t dims[3])
{
    for (int l = 0; l < 4; l++) {
        int s = 8 >> l;
        int spline = cfg[l][0], scheme = cfg[l][1], perm = cfg[l][2];
        for (int sub = 1; sub <= 3; sub++) {
            for (int i = 0; i < k->n[0]; i += s)
                for (int j = 0; j < k->n[1]; j += s)
                    for (int m = 0; m < k->n[2]; m += s) {
                        int t[3] = {i, j, m};
                        if (((i / s) & 1) == 0 && ((j / s) & 1) == 0 && ((m / s) & 1) == 0)
                            continue; /* coarser level or anchor */
                        if (substep(t, s, scheme, perm) != sub)
                            continue;
                        float p = orc_predict(buf, k->n, t, s, spline, scheme, perm);
                        long li = ((long)i * k->n[1] + j) * k->n[2] + m;
                        uint64_t g = gindex(dims, k->o[0] + i, k->o[1] + j, k->o[2] + m);
                        int owned = i < k->own[0] && j < k->own[1] && m < k->own[2];
                        if (codes_in == NULL) {
                            float xo;
                            uint8_t c = quantize(buf[li], p, eps, two_eb, inv, &xo);
                            buf[li] = xo;
                            if (owned)
                                codes_out[g] = c;
                        } else {
                            uint8_t c = codes_in[g];
                            if (c != 0)
                                buf[li] = p + ((float)((int)c - 128) * two_eb);
                            /* code 0: the stored outlier value is already in buf */
                        }
                    }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Tuner (Sec. 5.1.3)                                                         */
/* ------------------------------------------------------------------------ */

static void default_cfg(uint8_t cfg[4][3])
{
    for (int l = 0; l < 4; l++) {
        cfg[l][0] = ORC_CUB;
        cfg[l][1] = ORC_MD;
        cfg[l][2] = 0;
    }
}

/* Uniformly spaced full blocks with 0.2 % of the volume are sampled; each
 * level is tested with every candidate (LIN/CUB/NAT x MD/SEQ over the 6
 * dimension orders = 21) predicting from the ORIGINAL values, and the candidate with the
 * smallest aggregated error is kept per level, ties to the lower index.
 * Reading of "aggregated prediction errors": each |x - p| is counted in units
 * of 2*eps/65536, rounded to nearest and capped at 2^36 units, and summed as a
 * 64-bit integer, so the total is exact and does not depend on summation
 * order. Candidate index: spline*7 + (MD ? 0 : 1 + order).
 * A full block spans 17 points on every axis of the field, except the flat
 * axes of 2-D and 1-D fields (size 1), where it spans the one point: 2-D
 * fields (Sec. 6.1.3) are sampled in 17 x 17 blocks. */
int orc_tune(const float *x, const uint64_t dims[3], float eps,
             uint8_t cfg[4][3], uint64_t err[4][ORC_CANDS])
{
    default_cfg(cfg);
    memset(err, 0, sizeof(uint64_t) * 4 * ORC_CANDS);
    uint64_t f[3];
    int n[3];
    uint64_t vol = 1;
    for (int i = 0; i < 3; i++) {
        n[i] = dims[i] == 1 ? 1 : SIDE; /* block extent: flat axes span 1 point */
        f[i] = dims[i] == 1 ? 1 : (dims[i] >= SIDE ? (dims[i] - SIDE) / ANCHOR + 1 : 0);
        vol *= (uint64_t)n[i];
    }
    uint64_t n_full = f[0] * f[1] * f[2];
    if (n_full == 0)
        return ORC_OK;
    uint64_t N = dims[0] * dims[1] * dims[2];
    uint64_t n_s = cdiv(2 * N, 1000ull * vol); /* 0.2 % of N in full blocks */
    if (n_s < 1)
        n_s = 1;
    if (n_s > n_full)
        n_s = n_full;
    double scale = eps > 0.0f ? 65536.0 / (2.0 * (double)eps) : 65536.0;
    const double cap = 68719476736.0; /* 2^36 */
    float *buf = malloc(sizeof(float) * SIDE * SIDE * SIDE);
    if (!buf)
        return ORC_ERR_NOMEM;
    for (uint64_t j = 0; j < n_s; j++) {
        uint64_t idx = ((2 * j + 1) * n_full) / (2 * n_s);
        uint64_t c = idx % f[2], b = (idx / f[2]) % f[1], a = idx / (f[1] * f[2]);
        for (int i0 = 0; i0 < n[0]; i0++)
            for (int i1 = 0; i1 < n[1]; i1++)
                for (int i2 = 0; i2 < n[2]; i2++)
                    buf[(i0 * n[1] + i1) * n[2] + i2] =
                        x[gindex(dims, a * ANCHOR + i0, b * ANCHOR + i1, c * ANCHOR + i2)];
        for (int l = 0; l < 4; l++) {
            int s = 8 >> l;
            for (int i = 0; i < n[0]; i += s)
                for (int jj = 0; jj < n[1]; jj += s)
                    for (int m = 0; m < n[2]; m += s) {
                        if (((i / s) & 1) == 0 && ((jj / s) & 1) == 0 && ((m / s) & 1) == 0)
                            continue;
                        int t[3] = {i, jj, m};
                        float xv = buf[(i * n[1] + jj) * n[2] + m];
                        for (int cand = 0; cand < ORC_CANDS; cand++) {
                            int spline = cand / 7, r = cand % 7;
                            int scheme = r == 0 ? ORC_MD : ORC_SEQ;
                            int perm = r == 0 ? 0 : r - 1;
                            float p = orc_predict(buf, n, t, s, spline, scheme, perm);
                            float e = fabsf(xv - p);
                            double w = (double)e * scale;
                            uint64_t term = (w < cap) ? (uint64_t)(w + 0.5) : (uint64_t)cap;
                            err[l][cand] += term;
                        }
                    }
        }
    }
    free(buf);
    for (int l = 0; l < 4; l++) {
        int best = 0;
        for (int cand = 1; cand < ORC_CANDS; cand++)
            if (err[l][cand] < err[l][best])
                best = cand;
        int r = best % 7;
        cfg[l][0] = (uint8_t)(best / 7);
        cfg[l][1] = (uint8_t)(r == 0 ? ORC_MD : ORC_SEQ);
        cfg[l][2] = (uint8_t)(r == 0 ? 0 : r - 1);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Huffman codebook (Sec. 5.2.2-5.2.3)                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t w;
    int sym;
} leaf;

static int leaf_cmp(const void *pa, const void *pb)
{
    const leaf *a = pa, *b = pb;
    if (a->w != b->w)
        return a->w < b->w ? -1 : 1;
    return a->sym - b->sym;
}

/* Code lengths by the two-queue Huffman construction: leaves sorted by
 * (count, symbol) in one queue, merged nodes in a FIFO; each step merges the
 * two lightest fronts, taking the leaf when weights tie. Depth = length. */
static int huffman_lengths(const uint64_t cnt[256], uint8_t len[256])
{
    leaf lv[256];
    int n = 0;
    memset(len, 0, 256);
    for (int i = 0; i < 256; i++)
        if (cnt[i] > 0) {
            lv[n].w = cnt[i];
            lv[n].sym = i;
            n++;
        }
    if (n == 0)
        return 0;
    if (n == 1) {
        len[lv[0].sym] = 1;
        return 1;
    }
    qsort(lv, (size_t)n, sizeof(leaf), leaf_cmp);
    /* nodes 0..n-1 are the sorted leaves, n..2n-2 the merged nodes in creation order */
    uint64_t w[511];
    int parent[511];
    for (int i = 0; i < n; i++)
        w[i] = lv[i].w;
    int lq = 0, iq = n, next = n;
    for (int step = 0; step < n - 1; step++) {
        int pick[2];
        for (int h = 0; h < 2; h++) {
            int leaf_ok = lq < n;
            int int_ok = iq < next;
            if (leaf_ok && (!int_ok || w[lq] <= w[iq]))
                pick[h] = lq++;
            else
                pick[h] = iq++;
        }
        w[next] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = next;
        parent[pick[1]] = next;
        next++;
    }
    int depth[511];
    int root = next - 1;
    depth[root] = 0;
    for (int v = root - 1; v >= 0; v--)
        depth[v] = depth[parent[v]] + 1;
    int maxlen = 0;
    for (int i = 0; i < n; i++) {
        len[lv[i].sym] = (uint8_t)(depth[i] > 255 ? 255 : depth[i]);
        if (depth[i] > maxlen)
            maxlen = depth[i];
    }
    return maxlen;
}

/* Canonical codes from lengths (RFC 1951 Sec. 3.2.2): count codes per length,
 * derive the first code of each length, hand out codes in symbol order. */
static void canonical_codes(const uint8_t len[256], uint32_t code[256])
{
    uint64_t bl_count[MAX_CODE_LEN + 2] = {0};
    uint64_t next_code[MAX_CODE_LEN + 2] = {0};
    for (int i = 0; i < 256; i++)
        if (len[i])
            bl_count[len[i]]++;
    uint64_t c = 0;
    bl_count[0] = 0;
    for (int bits = 1; bits <= MAX_CODE_LEN; bits++) {
        c = (c + bl_count[bits - 1]) << 1;
        next_code[bits] = c;
    }
    for (int i = 0; i < 256; i++) {
        code[i] = 0;
        if (len[i])
            code[i] = (uint32_t)(next_code[len[i]]++);
    }
}

int orc_canonical(const uint8_t len[256], uint32_t code[256])
{
    for (int i = 0; i < 256; i++)
        if (len[i] > MAX_CODE_LEN)
            return ORC_ERR_ARG;
    canonical_codes(len, code);
    return ORC_OK;
}

/* Lengths are capped at 32 bits: while the tree is deeper, every nonzero count
 * is halved (kept >= 1) and the tree rebuilt. */
int orc_codebook(const uint64_t hist[256], uint8_t len[256], uint32_t code[256])
{
    uint64_t cnt[256];
    memcpy(cnt, hist, sizeof(cnt));
    for (;;) {
        int maxlen = huffman_lengths(cnt, len);
        if (maxlen <= MAX_CODE_LEN)
            break;
        for (int i = 0; i < 256; i++)
            if (cnt[i]) {
                cnt[i] >>= 1;
                if (cnt[i] == 0)
                    cnt[i] = 1;
            }
    }
    canonical_codes(len, code);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Chunked bit-packing                                                        */
/* ------------------------------------------------------------------------ */

/* The codes, in row-major order, are cut into chunks of `chunk` symbols. Each
 * chunk is the concatenation of its codewords, most significant bit first:
 * bit j of the chunk is bit 31-(j%32) of its word j/32; the last word is
 * zero-padded. Chunks follow each other; counts[k] = words of chunk k. */
int orc_huff_encode(const uint8_t *codes, uint64_t n, uint32_t chunk,
                    const uint8_t len[256], const uint32_t code[256],
                    uint32_t *words, uint64_t *n_words, uint32_t *counts)
{
    uint64_t nchunks = cdiv(n, chunk), w = 0;
    for (uint64_t k = 0; k < nchunks; k++) {
        uint64_t lo = k * chunk, hi = lo + chunk < n ? lo + chunk : n;
        uint64_t bit = 0;
        uint64_t start = w;
        for (uint64_t i = lo; i < hi; i++) {
            int L = len[codes[i]];
            if (L == 0)
                return ORC_ERR_ARG; /* symbol without a codeword */
            for (int b = L - 1; b >= 0; b--) {
                uint64_t wi = start + (bit >> 5);
                if ((bit & 31) == 0)
                    words[wi] = 0;
                if ((code[codes[i]] >> b) & 1u)
                    words[wi] |= 1u << (31 - (bit & 31));
                bit++;
            }
        }
        uint64_t nw = (bit + 31) / 32;
        counts[k] = (uint32_t)nw;
        w = start + nw;
    }
    *n_words = w;
    return ORC_OK;
}

/* Canonical decoding one bit at a time: extend the current code by a bit
 * until it falls into the range of codes of its length. Each chunk must use
 * exactly its stated number of words. */
int orc_huff_decode(const uint32_t *words, uint64_t n_words, const uint32_t *counts,
                    uint64_t n, uint32_t chunk, const uint8_t len[256], uint8_t *codes)
{
    uint32_t code[256];
    uint64_t bl_count[MAX_CODE_LEN + 2] = {0}, first[MAX_CODE_LEN + 2] = {0};
    uint64_t offset[MAX_CODE_LEN + 2] = {0};
    int sorted[256], ns = 0;
    for (int i = 0; i < 256; i++) {
        if (len[i] > MAX_CODE_LEN)
            return ORC_ERR_CORRUPT;
        if (len[i])
            bl_count[len[i]]++;
    }
    canonical_codes(len, code);
    /* symbols in canonical order: by length, then symbol */
    for (int L = 1; L <= MAX_CODE_LEN; L++) {
        offset[L] = (uint64_t)ns;
        for (int i = 0; i < 256; i++)
            if (len[i] == L) {
                if (ns == (int)offset[L])
                    first[L] = code[i];
                sorted[ns++] = i;
            }
    }
    if (ns == 0)
        return ORC_ERR_CORRUPT;
    uint64_t nchunks = cdiv(n, chunk), w = 0;
    for (uint64_t k = 0; k < nchunks; k++) {
        uint64_t lo = k * chunk, hi = lo + chunk < n ? lo + chunk : n;
        uint64_t start = w, nw = counts[k], bit = 0;
        if (start + nw > n_words)
            return ORC_ERR_CORRUPT;
        for (uint64_t i = lo; i < hi; i++) {
            uint64_t c = 0;
            int L = 0, found = 0;
            while (!found) {
                if (bit >= nw * 32)
                    return ORC_ERR_CORRUPT;
                uint32_t word = words[start + (bit >> 5)];
                c = (c << 1) | ((word >> (31 - (bit & 31))) & 1u);
                bit++;
                L++;
                if (L > MAX_CODE_LEN)
                    return ORC_ERR_CORRUPT;
                if (bl_count[L] && c >= first[L] && c - first[L] < bl_count[L]) {
                    codes[i] = (uint8_t)sorted[offset[L] + (c - first[L])];
                    found = 1;
                }
            }
        }
        if ((bit + 31) / 32 != nw)
            return ORC_ERR_CORRUPT;
        w = start + nw;
    }
    if (w != n_words)
        return ORC_ERR_CORRUPT;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Reordering of the codes by interpolation level (Sec. 5.1.4, Eq. reorder)   */
/* ------------------------------------------------------------------------ */

/* Interpolation level of a point: the largest l <= log2(A) = 4 such that 2^l
 * divides x, y and z (Eq. reorder). Level 4 holds the anchors, level 0 the
 * stride-1 targets. */
int orc_level(uint64_t x, uint64_t y, uint64_t z)
{
    int l = 0;
    while (l < 4 && ((x | y | z) & ((2ull << l) - 1)) == 0)
        l++;
    return l;
}

/* f(k) of Eq. reorder: f(0) = floor((d+1)/2), f(k+1) = floor((f(k)+1)/2);
 * f(-1) = d. */
static uint64_t reorder_f(uint64_t d, int k)
{
    uint64_t f = d;
    for (int i = 0; i <= k; i++)
        f = (f + 1) / 2;
    return f;
}

/* Index of point (x, y, z) in the reordered code sequence (Eq. reorder).
 * Reading: the equation as printed applies the level-0 grid's counts at
 * every level and is not a bijection for l >= 1. It is applied here on the
 * level-l grid: coordinates x/2^l, y/2^l, z/2^l, dimension sizes f(l-1)
 * (f(-1) = d), and the subtractions count the grid points of coarser levels
 * that precede the point in row-major order. prefix(l) = f_x(l) f_y(l) f_z(l)
 * is the number of points on coarser levels; the anchor level l = log2(A)
 * has prefix 0 and no subtraction. At l = 0 this is the printed formula. */
uint64_t orc_reorder_index(const uint64_t dims[3], uint64_t x, uint64_t y, uint64_t z)
{
    const int l = orc_level(x, y, z);
    const uint64_t xs = x >> l, ys = y >> l, zs = z >> l;
    const uint64_t dy = reorder_f(dims[1], l - 1), dz = reorder_f(dims[2], l - 1);
    uint64_t I = xs * dy * dz + ys * dz + zs;
    if (l == 4)
        return I;
    const uint64_t prefix =
        reorder_f(dims[0], l) * reorder_f(dims[1], l) * reorder_f(dims[2], l);
    I -= ((xs + 1) / 2) * ((dy + 1) / 2) * ((dz + 1) / 2);
    if (xs % 2 == 0)
        I -= ((ys + 1) / 2) * ((dz + 1) / 2);
    if (xs % 2 == 0 && ys % 2 == 0)
        I -= (zs + 1) / 2;
    return prefix + I;
}

/* seq[I(x,y,z)] = codes[x,y,z]. */
void orc_reorder(const uint8_t *codes, const uint64_t dims[3], uint8_t *seq)
{
    for (uint64_t x = 0; x < dims[0]; x++)
        for (uint64_t y = 0; y < dims[1]; y++)
            for (uint64_t z = 0; z < dims[2]; z++)
                seq[orc_reorder_index(dims, x, y, z)] = codes[gindex(dims, x, y, z)];
}

void orc_unreorder(const uint8_t *seq, const uint64_t dims[3], uint8_t *codes)
{
    for (uint64_t x = 0; x < dims[0]; x++)
        for (uint64_t y = 0; y < dims[1]; y++)
            for (uint64_t z = 0; z < dims[2]; z++)
                codes[gindex(dims, x, y, z)] = seq[orc_reorder_index(dims, x, y, z)];
}

/* ------------------------------------------------------------------------ */
/* Bitwise-redundancy lossless stages (Sec. 5.2.3)                            */
/* ------------------------------------------------------------------------ */
/* The input bytes are cut into chunks of LC_CHUNK bytes (the last may be
 * shorter); every chunk passes through the pipeline's stages one after the
 * other, and is stored raw when the result is not smaller than the chunk.
 * The number in a stage's name is its symbol width k in bytes; a chunk's
 * trailing bytes that do not fill a whole symbol pass through unchanged.
 *  - TCMS_k: two's complement to magnitude-sign, (w << 1) ^ (w >> (8k-1))
 *    with an arithmetic right shift, on each k-byte little-endian word.
 *  - BIT_1: bit shuffle. The chunk's bytes are taken in groups of 8; output
 *    plane p (p = 0..7) holds bit p of every input byte, input byte 8j+i of
 *    the chunk giving bit i of the plane's byte j. Planes follow each other,
 *    then the bytes left over after the last whole group.
 *  - RRE_k: a bitmap marks the words that differ from the word before (the
 *    word before the first is 0); only the marked words are kept.
 *  - RZE_k: a bitmap marks the nonzero words; only those are kept.
 * Stage output of RRE_k / RZE_k: the input length (u16), the bitmap
 * compressed recursively, the kept words, the trailing bytes. Bitmap bit i
 * is bit (i & 7) of byte i >> 3. Recursive bitmap compression (reading of
 * "compressing the bitmap recursively"): a bitmap of at most 8 bytes is
 * stored as it is; a longer one is replaced by the bitmap of its bytes that
 * differ from the byte before (the byte before the first is 0), itself
 * compressed the same way, followed by those bytes.
 * The stage details beyond the paper's sentences (chunk size, symbol order,
 * bitmap layout, recursion, raw fallback) are this implementation's reading. */

#define LC_CHUNK 16384
#define LC_MAXBUF (LC_CHUNK + LC_CHUNK / 4 + 64)

enum { ST_TCMS = 0, ST_BIT = 1, ST_RRE = 2, ST_RZE = 3 };
typedef struct {
    int op, k;
} lc_stage;

static const lc_stage TP_STAGES[3] = {{ST_TCMS, 1}, {ST_BIT, 1}, {ST_RRE, 1}};
static const lc_stage CR_STAGES[3] = {{ST_RRE, 4}, {ST_TCMS, 8}, {ST_RZE, 1}};

static uint64_t get_word(const uint8_t *p, int k)
{
    uint64_t v = 0;
    for (int b = 0; b < k; b++)
        v |= (uint64_t)p[b] << (8 * b);
    return v;
}

static void put_word(uint8_t *p, int k, uint64_t v)
{
    for (int b = 0; b < k; b++)
        p[b] = (uint8_t)(v >> (8 * b));
}

static void tcms(const uint8_t *in, int n, int k, uint8_t *out)
{
    const int bits = 8 * k, m = n / k;
    const uint64_t mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    memcpy(out, in, (size_t)n);
    for (int i = 0; i < m; i++) {
        uint64_t w = get_word(in + (size_t)i * k, k);
        uint64_t sign = (w >> (bits - 1)) & 1 ? mask : 0; /* arithmetic shift by bits-1 */
        put_word(out + (size_t)i * k, k, ((w << 1) & mask) ^ sign);
    }
}

static void tcms_inv(const uint8_t *in, int n, int k, uint8_t *out)
{
    const int bits = 8 * k, m = n / k;
    const uint64_t mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    memcpy(out, in, (size_t)n);
    for (int i = 0; i < m; i++) {
        uint64_t u = get_word(in + (size_t)i * k, k);
        uint64_t w = (u >> 1) ^ ((u & 1) ? mask : 0);
        put_word(out + (size_t)i * k, k, w & mask);
    }
}

static void bitshuffle(const uint8_t *in, int n, uint8_t *out)
{
    const int g = n / 8;
    for (int p = 0; p < 8; p++)
        for (int j = 0; j < g; j++) {
            uint8_t v = 0;
            for (int i = 0; i < 8; i++)
                v |= (uint8_t)(((in[8 * j + i] >> p) & 1) << i);
            out[p * g + j] = v;
        }
    memcpy(out + 8 * g, in + 8 * g, (size_t)(n - 8 * g));
}

static void bitshuffle_inv(const uint8_t *in, int n, uint8_t *out)
{
    const int g = n / 8;
    for (int j = 0; j < 8 * g; j++)
        out[j] = 0;
    for (int p = 0; p < 8; p++)
        for (int j = 0; j < g; j++)
            for (int i = 0; i < 8; i++)
                out[8 * j + i] |= (uint8_t)(((in[p * g + j] >> i) & 1) << p);
    memcpy(out + 8 * g, in + 8 * g, (size_t)(n - 8 * g));
}

/* Bitmap of nbytes bytes, compressed recursively; returns bytes written. */
static int bitmap_put(const uint8_t *bm, int nbytes, uint8_t *out)
{
    if (nbytes <= 8) {
        memcpy(out, bm, (size_t)nbytes);
        return nbytes;
    }
    uint8_t sub[LC_MAXBUF / 8 + 8];
    const int sb = (nbytes + 7) / 8;
    memset(sub, 0, (size_t)sb);
    for (int j = 0; j < nbytes; j++) {
        uint8_t before = j ? bm[j - 1] : 0;
        if (bm[j] != before)
            sub[j >> 3] |= (uint8_t)(1u << (j & 7));
    }
    int o = bitmap_put(sub, sb, out);
    for (int j = 0; j < nbytes; j++) {
        uint8_t before = j ? bm[j - 1] : 0;
        if (bm[j] != before)
            out[o++] = bm[j];
    }
    return o;
}

/* Inverse of bitmap_put: rebuilds nbytes bitmap bytes from in[0..avail);
 * returns the bytes read, or -1 if the input is too short. */
static int bitmap_get(const uint8_t *in, int avail, int nbytes, uint8_t *bm)
{
    if (nbytes <= 8) {
        if (avail < nbytes)
            return -1;
        memcpy(bm, in, (size_t)nbytes);
        return nbytes;
    }
    uint8_t sub[LC_MAXBUF / 8 + 8];
    const int sb = (nbytes + 7) / 8;
    int o = bitmap_get(in, avail, sb, sub);
    if (o < 0)
        return -1;
    uint8_t before = 0;
    for (int j = 0; j < nbytes; j++) {
        if ((sub[j >> 3] >> (j & 7)) & 1) {
            if (o >= avail)
                return -1;
            before = in[o++];
        }
        bm[j] = before;
    }
    return o;
}

/* RRE_k (zero_mode 0) or RZE_k (zero_mode 1) of n bytes; returns the output size. */
static int reduce(const uint8_t *in, int n, int k, int zero_mode, uint8_t *out)
{
    const int m = n / k, tail = n - m * k;
    uint8_t bm[LC_MAXBUF / 8 + 8];
    const int nb = (m + 7) / 8;
    memset(bm, 0, (size_t)nb);
    uint64_t prev = 0;
    for (int i = 0; i < m; i++) {
        uint64_t w = get_word(in + (size_t)i * k, k);
        int keep = zero_mode ? (w != 0) : (w != prev);
        if (keep)
            bm[i >> 3] |= (uint8_t)(1u << (i & 7));
        prev = w;
    }
    out[0] = (uint8_t)(n & 255);
    out[1] = (uint8_t)(n >> 8);
    int o = 2 + bitmap_put(bm, nb, out + 2);
    for (int i = 0; i < m; i++)
        if ((bm[i >> 3] >> (i & 7)) & 1) {
            memcpy(out + o, in + (size_t)i * k, (size_t)k);
            o += k;
        }
    memcpy(out + o, in + (size_t)m * k, (size_t)tail);
    return o + tail;
}

/* Inverse of reduce; returns the restored length, -1 on a malformed input. */
static int reduce_inv(const uint8_t *in, int avail, int k, int zero_mode, uint8_t *out,
                      int out_cap)
{
    if (avail < 2)
        return -1;
    const int n = in[0] | (in[1] << 8);
    if (n > out_cap)
        return -1;
    const int m = n / k, tail = n - m * k;
    uint8_t bm[LC_MAXBUF / 8 + 8];
    const int nb = (m + 7) / 8;
    int o = bitmap_get(in + 2, avail - 2, nb, bm);
    if (o < 0)
        return -1;
    o += 2;
    uint64_t prev = 0;
    for (int i = 0; i < m; i++) {
        uint64_t w;
        if ((bm[i >> 3] >> (i & 7)) & 1) {
            if (o + k > avail)
                return -1;
            w = get_word(in + o, k);
            o += k;
        } else {
            w = zero_mode ? 0 : prev;
        }
        put_word(out + (size_t)i * k, k, w);
        prev = w;
    }
    if (o + tail != avail)
        return -1;
    memcpy(out + (size_t)m * k, in + o, (size_t)tail);
    return n;
}

/* One chunk through the stages; returns the encoded size (raw if not smaller). */
static int lc_chunk_encode(const lc_stage *st, int ns, const uint8_t *in, int n, uint8_t *out)
{
    uint8_t a[LC_MAXBUF], b[LC_MAXBUF];
    memcpy(a, in, (size_t)n);
    int len = n;
    for (int i = 0; i < ns; i++) {
        if (st[i].op == ST_TCMS)
            tcms(a, len, st[i].k, b);
        else if (st[i].op == ST_BIT)
            bitshuffle(a, len, b);
        else
            len = reduce(a, len, st[i].k, st[i].op == ST_RZE, b);
        memcpy(a, b, (size_t)len);
    }
    if (len >= n) {
        memcpy(out, in, (size_t)n);
        return n;
    }
    memcpy(out, a, (size_t)len);
    return len;
}

/* Inverse of lc_chunk_encode for a chunk of n raw bytes stored in `size` bytes. */
static int lc_chunk_decode(const lc_stage *st, int ns, const uint8_t *in, int size, int n,
                           uint8_t *out)
{
    if (size == n) {
        memcpy(out, in, (size_t)n);
        return ORC_OK;
    }
    if (size > n)
        return ORC_ERR_CORRUPT;
    uint8_t a[LC_MAXBUF], b[LC_MAXBUF];
    memcpy(a, in, (size_t)size);
    int len = size;
    for (int i = ns - 1; i >= 0; i--) {
        if (st[i].op == ST_TCMS)
            tcms_inv(a, len, st[i].k, b);
        else if (st[i].op == ST_BIT)
            bitshuffle_inv(a, len, b);
        else {
            len = reduce_inv(a, len, st[i].k, st[i].op == ST_RZE, b, LC_MAXBUF);
            if (len < 0)
                return ORC_ERR_CORRUPT;
        }
        memcpy(a, b, (size_t)len);
    }
    if (len != n)
        return ORC_ERR_CORRUPT;
    memcpy(out, a, (size_t)n);
    return ORC_OK;
}

static const lc_stage *pipeline_stages(int pipe)
{
    return pipe == ORC_PIPE_TP ? TP_STAGES : CR_STAGES;
}

uint64_t orc_lc_chunks(uint64_t n) { return cdiv(n, LC_CHUNK); }

/* Chunked pipeline over n bytes: sizes[k] = stored bytes of chunk k; data
 * must hold n bytes (a chunk never stores more than its raw size). */
int orc_lc_encode(int pipe, const uint8_t *in, uint64_t n, uint32_t *sizes, uint8_t *data,
                  uint64_t *data_bytes)
{
    if (pipe != ORC_PIPE_TP && pipe != ORC_PIPE_CR)
        return ORC_ERR_ARG;
    const lc_stage *st = pipeline_stages(pipe);
    uint64_t o = 0;
    for (uint64_t c = 0; c < orc_lc_chunks(n); c++) {
        const uint64_t lo = c * LC_CHUNK;
        const int len = (int)(lo + LC_CHUNK <= n ? LC_CHUNK : n - lo);
        const int sz = lc_chunk_encode(st, 3, in + lo, len, data + o);
        sizes[c] = (uint32_t)sz;
        o += (uint64_t)sz;
    }
    *data_bytes = o;
    return ORC_OK;
}

int orc_lc_decode(int pipe, const uint32_t *sizes, const uint8_t *data, uint64_t data_bytes,
                  uint8_t *out, uint64_t n)
{
    if (pipe != ORC_PIPE_TP && pipe != ORC_PIPE_CR)
        return ORC_ERR_ARG;
    const lc_stage *st = pipeline_stages(pipe);
    uint64_t o = 0;
    for (uint64_t c = 0; c < orc_lc_chunks(n); c++) {
        const uint64_t lo = c * LC_CHUNK;
        const int len = (int)(lo + LC_CHUNK <= n ? LC_CHUNK : n - lo);
        if (sizes[c] > (uint32_t)len || o + sizes[c] > data_bytes)
            return ORC_ERR_CORRUPT;
        int rc = lc_chunk_decode(st, 3, data + o, (int)sizes[c], len, out + lo);
        if (rc)
            return rc;
        o += sizes[c];
    }
    return o == data_bytes ? ORC_OK : ORC_ERR_CORRUPT;
}

/* One stage on one buffer (tests): op 0 TCMS, 1 BIT, 2 RRE, 3 RZE; inverse
 * when inv != 0. Returns the output length or -1. */
int orc_lc_stage(int op, int k, int inv, const uint8_t *in, int n, uint8_t *out)
{
    if (n < 0 || n > LC_MAXBUF - 64)
        return -1;
    if (op == ST_TCMS) {
        if (k != 1 && k != 2 && k != 4 && k != 8)
            return -1;
        (inv ? tcms_inv : tcms)(in, n, k, out);
        return n;
    }
    if (op == ST_BIT) {
        (inv ? bitshuffle_inv : bitshuffle)(in, n, out);
        return n;
    }
    if (op == ST_RRE || op == ST_RZE) {
        if (k != 1 && k != 2 && k != 4 && k != 8)
            return -1;
        return inv ? reduce_inv(in, n, k, op == ST_RZE, out, LC_MAXBUF)
                   : reduce(in, n, k, op == ST_RZE, out);
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Stream                                                                     */
/* ------------------------------------------------------------------------ */

static void put_u16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }
static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void put_f32(uint8_t *p, float v) { memcpy(p, &v, 4); }
static void put_f64(uint8_t *p, double v) { memcpy(p, &v, 8); }
static uint16_t get_u16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
static uint32_t get_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static float get_f32(const uint8_t *p) { float v; memcpy(&v, p, 4); return v; }
static double get_f64(const uint8_t *p) { double v; memcpy(&v, p, 8); return v; }

typedef struct {
    uint64_t dims[3], N;
    int mode, flags;
    double eb;
    float eps, vmin, vmax;
    uint8_t cfg[4][3];
    uint32_t chunk;
    uint64_t n_out, payload_words, total, n_chunks, n_anchors;
    uint64_t off_anchors, off_oidx, off_oval, off_payload;
    int idx_bytes;
    int pipe;                 /* lossless pipeline (ORC_PIPE_*) */
    uint64_t n_lc, lc_bytes;  /* TP / CR: chunks and stored bytes of the last stages */
    uint64_t off_lcsizes;     /* CR: chunk-size table of the last stages */
} layout;

/* Section offsets. HF: Huffman word counts at 384, payload last. TP: the
 * last stages' chunk sizes at 384 (no Huffman sections), their data last.
 * CR: Huffman word counts at 384, then after the outliers the last stages'
 * chunk sizes and their data (the Huffman payload after those stages). */
static void compute_offsets(layout *L)
{
    const uint64_t table = L->pipe == ORC_PIPE_TP ? L->n_lc : L->n_chunks;
    L->off_anchors = align16(OFF_CHUNKS + 4 * table);
    L->off_oidx = align16(L->off_anchors + 4 * L->n_anchors);
    L->off_oval = align16(L->off_oidx + (uint64_t)L->idx_bytes * L->n_out);
    const uint64_t end_oval = L->off_oval + 4 * L->n_out;
    if (L->pipe == ORC_PIPE_HF) {
        L->off_payload = align16(end_oval);
        L->total = L->off_payload + 4 * L->payload_words;
        return;
    }
    L->off_lcsizes = L->pipe == ORC_PIPE_TP ? OFF_CHUNKS : align16(end_oval);
    L->off_payload = L->pipe == ORC_PIPE_TP ? align16(end_oval)
                                            : align16(L->off_lcsizes + 4 * L->n_lc);
    L->total = L->off_payload + L->lc_bytes;
}

static void write_header(uint8_t *o, const layout *L)
{
    memset(o, 0, HDR_BYTES);
    put_u32(o + 0, MAGIC);
    put_u16(o + 4, VERSION);
    o[6] = (uint8_t)L->mode;
    o[7] = (uint8_t)L->flags;
    put_u64(o + 8, L->dims[0]);
    put_u64(o + 16, L->dims[1]);
    put_u64(o + 24, L->dims[2]);
    put_f64(o + 32, L->eb);
    put_f32(o + 40, L->eps);
    put_f32(o + 44, L->vmin);
    put_f32(o + 48, L->vmax);
    o[52] = ANCHOR;
    o[53] = 4;
    for (int l = 0; l < 4; l++)
        for (int k = 0; k < 3; k++)
            o[56 + 3 * l + k] = L->cfg[l][k];
    put_u32(o + 68, L->chunk);
    put_u64(o + 72, L->n_out);
    put_u64(o + 80, L->payload_words);
    put_u64(o + 88, L->total);
    put_u64(o + 96, L->n_chunks);
    put_u64(o + 104, L->n_anchors);
    o[54] = (uint8_t)L->pipe;
    put_u64(o + 112, L->lc_bytes);
    put_u64(o + 120, L->n_lc);
}

/* Exact minimum and maximum; -0.0 counts as smaller than +0.0. */
static int less_total(float a, float b)
{
    if (a < b)
        return 1;
    if (a == b && signbit(a) && !signbit(b))
        return 1;
    return 0;
}

int orc_compress(const float *x, const uint64_t dims[3], int mode, double eb,
                 const orc_params *p, uint8_t **out, uint64_t *out_size,
                 orc_debug *dbg)
{
    *out = NULL;
    *out_size = 0;
    if (!x || !dims || dims[0] == 0 || dims[1] == 0 || dims[2] == 0)
        return ORC_ERR_ARG;
    if (dims[0] > MAX_N || dims[1] > MAX_N || dims[2] > MAX_N ||
        dims[0] * dims[1] > MAX_N || dims[0] * dims[1] * dims[2] > MAX_N)
        return ORC_ERR_ARG;
    if (mode != ORC_ABS && mode != ORC_REL)
        return ORC_ERR_ARG;
    if (!(eb > 0.0) || !isfinite(eb))
        return ORC_ERR_ARG;
    orc_params prm;
    if (p)
        prm = *p;
    else {
        prm.tune = 1;
        prm.chunk = 1024;
        default_cfg(prm.cfg);
        prm.pipeline = ORC_PIPE_HF;
        prm.reorder = 0;
    }
    if (prm.chunk < 256 || prm.chunk > 65536 || (prm.chunk & (prm.chunk - 1)))
        return ORC_ERR_ARG;
    if (prm.pipeline < ORC_PIPE_HF || prm.pipeline > ORC_PIPE_CR ||
        (prm.reorder != 0 && prm.reorder != 1))
        return ORC_ERR_ARG;
    for (int l = 0; l < 4; l++)
        if (prm.cfg[l][0] > 2 || prm.cfg[l][1] > 1 || prm.cfg[l][2] > 5)
            return ORC_ERR_ARG;

    const uint64_t N = dims[0] * dims[1] * dims[2];
    float vmin = x[0], vmax = x[0];
    for (uint64_t i = 0; i < N; i++) {
        if (!isfinite(x[i]))
            return ORC_ERR_NONFINITE;
        if (less_total(x[i], vmin))
            vmin = x[i];
        if (less_total(vmax, x[i]))
            vmax = x[i];
    }
    layout L;
    memset(&L, 0, sizeof(L));
    for (int i = 0; i < 3; i++)
        L.dims[i] = dims[i];
    L.N = N;
    L.mode = mode;
    L.eb = eb;
    L.vmin = vmin;
    L.vmax = vmax;
    L.chunk = prm.chunk;
    L.pipe = prm.pipeline;

    if (mode == ORC_REL && (double)vmax - (double)vmin == 0.0) {
        /* Constant field: the header and the single value. */
        L.flags = 1;
        L.eps = 0.0f;
        L.pipe = ORC_PIPE_HF;
        L.total = HDR_BYTES + 4;
        uint8_t *o = calloc(L.total, 1);
        if (!o)
            return ORC_ERR_NOMEM;
        L.n_chunks = 0;
        L.n_anchors = 0;
        default_cfg(L.cfg);
        write_header(o, &L);
        put_f32(o + HDR_BYTES, x[0]);
        *out = o;
        *out_size = L.total;
        if (dbg) {
            dbg->eps = 0.0f;
            dbg->n_out = 0;
            memset(dbg->hist, 0, sizeof(dbg->hist));
            memcpy(dbg->cfg, L.cfg, sizeof(L.cfg));
            if (dbg->recon)
                for (uint64_t i = 0; i < N; i++)
                    dbg->recon[i] = x[i];
            if (dbg->codes)
                memset(dbg->codes, 128, N);
        }
        return ORC_OK;
    }

    float eps = orc_eps(mode, eb, vmin, vmax);
    float two_eb = eps * 2.0f;
    float inv = 1.0f / two_eb;
    L.eps = eps;
    L.idx_bytes = N < (1ull << 32) ? 4 : 8;
    L.flags = L.idx_bytes == 8 ? 2 : 0;

    uint64_t tune_err[4][ORC_CANDS];
    memset(tune_err, 0, sizeof(tune_err));
    if (prm.tune) {
        int rc = orc_tune(x, dims, eps, L.cfg, tune_err);
        if (rc)
            return rc;
    } else {
        memcpy(L.cfg, prm.cfg, sizeof(L.cfg));
    }

    uint64_t nb[3];
    for (int i = 0; i < 3; i++)
        nb[i] = cdiv(dims[i], ANCHOR);
    L.n_anchors = nb[0] * nb[1] * nb[2];
    L.n_chunks = cdiv(N, prm.chunk);

    uint8_t *codes = malloc(N);
    float *anchors = malloc(sizeof(float) * L.n_anchors);
    float *buf = malloc(sizeof(float) * SIDE * SIDE * SIDE);
    if (!codes || !anchors || !buf) {
        free(codes);
        free(anchors);
        free(buf);
        return ORC_ERR_NOMEM;
    }

    /* Predict and quantize block by block; blocks are independent. */
#ifdef ORC_FACE_CHECK
    if (!fc_begin(N)) {
        free(codes);
        free(anchors);
        free(buf);
        return ORC_ERR_NOMEM;
    }
#endif
    for (uint64_t a = 0; a < nb[0]; a++)
        for (uint64_t b = 0; b < nb[1]; b++)
            for (uint64_t c = 0; c < nb[2]; c++) {
                block k = make_block(dims, a, b, c);
                for (int i = 0; i < k.n[0]; i++)
                    for (int j = 0; j < k.n[1]; j++)
                        for (int m = 0; m < k.n[2]; m++)
                            buf[(i * k.n[1] + j) * k.n[2] + m] =
                                x[gindex(dims, k.o[0] + i, k.o[1] + j, k.o[2] + m)];
                uint64_t g0 = gindex(dims, k.o[0], k.o[1], k.o[2]);
                anchors[(a * nb[1] + b) * nb[2] + c] = buf[0];
                codes[g0] = 128; /* anchors keep the zero-error code */
                run_levels(buf, &k, L.cfg, eps, two_eb, inv, NULL, codes, dims);
#ifdef ORC_FACE_CHECK
                fc_note_block(buf, &k, dims);
#endif
                if (dbg && dbg->recon)
                    for (int i = 0; i < k.own[0]; i++)
                        for (int j = 0; j < k.own[1]; j++)
                            for (int m = 0; m < k.own[2]; m++)
                                dbg->recon[gindex(dims, k.o[0] + i, k.o[1] + j, k.o[2] + m)] =
                                    buf[(i * k.n[1] + j) * k.n[2] + m];
            }
    free(buf);

    uint64_t hist[256] = {0};
    for (uint64_t i = 0; i < N; i++)
        hist[codes[i]]++;
    L.n_out = hist[0];

    uint8_t len[256];
    uint32_t code[256];
    memset(len, 0, sizeof(len));
    if (L.pipe != ORC_PIPE_TP)
        orc_codebook(hist, len, code);

    /* The lossless stage reads the codes in row-major order, or reordered by
     * level (Sec. 5.1.4, Eq. reorder) when asked. */
    uint8_t *seq = codes;
    if (prm.reorder) {
        seq = malloc(N);
        if (!seq) {
            free(codes);
            free(anchors);
            return ORC_ERR_NOMEM;
        }
        orc_reorder(codes, dims, seq);
        L.flags |= ORC_FLAG_REORDER;
    }
    /* Huffman payload (HF and CR; Sec. 5.2.2-5.2.3) */
    uint32_t *words = NULL, *counts = NULL;
    uint64_t nw = 0;
    if (L.pipe != ORC_PIPE_TP) {
        L.n_chunks = cdiv(N, prm.chunk);
        words = malloc(sizeof(uint32_t) * (N + L.n_chunks));
        counts = malloc(sizeof(uint32_t) * (L.n_chunks ? L.n_chunks : 1));
        if (words && counts)
            orc_huff_encode(seq, N, prm.chunk, len, code, words, &nw, counts);
    } else {
        L.n_chunks = 0;
        L.chunk = 0;
    }
    /* the bitwise-redundancy stages (Sec. 5.2.3): TP on the codes, CR on the
     * Huffman payload's bytes (words little-endian) */
    uint32_t *lc_sizes = NULL;
    uint8_t *lc_data = NULL;
    int fail_mem = (L.pipe != ORC_PIPE_TP && (!words || !counts));
    if (!fail_mem && L.pipe != ORC_PIPE_HF) {
        const uint8_t *lc_in = L.pipe == ORC_PIPE_TP ? seq : (const uint8_t *)words;
        const uint64_t n_in = L.pipe == ORC_PIPE_TP ? N : 4 * nw;
        L.n_lc = orc_lc_chunks(n_in);
        lc_sizes = malloc(sizeof(uint32_t) * (L.n_lc ? L.n_lc : 1));
        lc_data = malloc(n_in ? n_in : 1);
        if (lc_sizes && lc_data)
            orc_lc_encode(L.pipe, lc_in, n_in, lc_sizes, lc_data, &L.lc_bytes);
        else
            fail_mem = 1;
    }
    if (seq != codes)
        free(seq);
    if (fail_mem) {
        free(words);
        free(counts);
        free(lc_sizes);
        free(lc_data);
        free(codes);
        free(anchors);
        return ORC_ERR_NOMEM;
    }
    L.payload_words = L.pipe == ORC_PIPE_TP ? 0 : nw;
    compute_offsets(&L);

    uint8_t *o = calloc(L.total, 1);
    if (!o) {
        free(words);
        free(counts);
        free(lc_sizes);
        free(lc_data);
        free(codes);
        free(anchors);
        return ORC_ERR_NOMEM;
    }
    write_header(o, &L);
    memcpy(o + OFF_LEN, len, 256);
    for (uint64_t k = 0; k < L.n_chunks; k++)
        put_u32(o + OFF_CHUNKS + 4 * k, counts[k]);
    for (uint64_t k = 0; k < L.n_anchors; k++)
        put_f32(o + L.off_anchors + 4 * k, anchors[k]);
    /* Outliers in ascending index order with their exact values. */
    uint64_t j = 0;
    for (uint64_t i = 0; i < N; i++)
        if (codes[i] == 0) {
            if (L.idx_bytes == 4)
                put_u32(o + L.off_oidx + 4 * j, (uint32_t)i);
            else
                put_u64(o + L.off_oidx + 8 * j, i);
            put_f32(o + L.off_oval + 4 * j, x[i]);
            j++;
        }
    if (L.pipe == ORC_PIPE_HF) {
        for (uint64_t k = 0; k < nw; k++)
            put_u32(o + L.off_payload + 4 * k, words[k]);
    } else {
        for (uint64_t k = 0; k < L.n_lc; k++)
            put_u32(o + L.off_lcsizes + 4 * k, lc_sizes[k]);
        memcpy(o + L.off_payload, lc_data, L.lc_bytes);
    }
    free(lc_sizes);
    free(lc_data);

    if (dbg) {
        memcpy(dbg->hist, hist, sizeof(hist));
        memcpy(dbg->cfg, L.cfg, sizeof(L.cfg));
        memcpy(dbg->tune_err, tune_err, sizeof(tune_err));
        dbg->eps = eps;
        dbg->n_out = L.n_out;
        if (dbg->codes)
            memcpy(dbg->codes, codes, N);
    }
    free(words);
    free(counts);
    free(codes);
    free(anchors);
    *out = o;
    *out_size = L.total;
    return ORC_OK;
}

/* Parse and check the header; fills L. */
static int parse_header(const uint8_t *in, uint64_t in_size, layout *L)
{
    memset(L, 0, sizeof(*L));
    if (!in || in_size < HDR_BYTES)
        return ORC_ERR_CORRUPT;
    if (get_u32(in) != MAGIC || get_u16(in + 4) != VERSION)
        return ORC_ERR_CORRUPT;
    L->mode = in[6];
    L->flags = in[7];
    for (int i = 0; i < 3; i++)
        L->dims[i] = get_u64(in + 8 + 8 * i);
    for (int i = 0; i < 3; i++)
        if (L->dims[i] == 0 || L->dims[i] > MAX_N)
            return ORC_ERR_CORRUPT;
    if (L->dims[0] * L->dims[1] > MAX_N || L->dims[0] * L->dims[1] * L->dims[2] > MAX_N)
        return ORC_ERR_CORRUPT;
    L->N = L->dims[0] * L->dims[1] * L->dims[2];
    L->eb = get_f64(in + 32);
    L->eps = get_f32(in + 40);
    L->vmin = get_f32(in + 44);
    L->vmax = get_f32(in + 48);
    L->pipe = in[54];
    if (L->mode > 1 || (L->flags & ~7) || L->pipe > ORC_PIPE_CR)
        return ORC_ERR_CORRUPT;
    if (L->flags & 1) {
        if (L->pipe != ORC_PIPE_HF || (L->flags & ORC_FLAG_REORDER))
            return ORC_ERR_CORRUPT;
        L->total = HDR_BYTES + 4;
        if (in_size < L->total || get_u64(in + 88) != L->total)
            return ORC_ERR_CORRUPT;
        return ORC_OK;
    }
    if (in[52] != ANCHOR || in[53] != 4)
        return ORC_ERR_CORRUPT;
    for (int l = 0; l < 4; l++) {
        for (int k = 0; k < 3; k++)
            L->cfg[l][k] = in[56 + 3 * l + k];
        if (L->cfg[l][0] > 2 || L->cfg[l][1] > 1 || L->cfg[l][2] > 5)
            return ORC_ERR_CORRUPT;
    }
    L->chunk = get_u32(in + 68);
    L->n_out = get_u64(in + 72);
    L->payload_words = get_u64(in + 80);
    L->n_chunks = get_u64(in + 96);
    L->n_anchors = get_u64(in + 104);
    L->lc_bytes = get_u64(in + 112);
    L->n_lc = get_u64(in + 120);
    if (L->pipe == ORC_PIPE_TP) {
        if (L->chunk != 0 || L->n_chunks != 0 || L->payload_words != 0)
            return ORC_ERR_CORRUPT;
        if (L->n_lc != orc_lc_chunks(L->N) || L->lc_bytes > L->N)
            return ORC_ERR_CORRUPT;
    } else {
        if (L->chunk < 256 || L->chunk > 65536 || (L->chunk & (L->chunk - 1)))
            return ORC_ERR_CORRUPT;
        if (L->n_chunks != cdiv(L->N, L->chunk))
            return ORC_ERR_CORRUPT;
        if (L->payload_words > L->N + L->n_chunks)
            return ORC_ERR_CORRUPT;
        if (L->pipe == ORC_PIPE_HF && (L->n_lc != 0 || L->lc_bytes != 0))
            return ORC_ERR_CORRUPT;
        if (L->pipe == ORC_PIPE_CR && (L->n_lc != orc_lc_chunks(4 * L->payload_words) ||
                                       L->lc_bytes > 4 * L->payload_words))
            return ORC_ERR_CORRUPT;
    }
    L->idx_bytes = L->N < (1ull << 32) ? 4 : 8;
    if (((L->flags & 2) != 0) != (L->idx_bytes == 8))
        return ORC_ERR_CORRUPT;
    if (L->n_anchors != cdiv(L->dims[0], ANCHOR) * cdiv(L->dims[1], ANCHOR) *
                            cdiv(L->dims[2], ANCHOR))
        return ORC_ERR_CORRUPT;
    if (L->n_out > L->N)
        return ORC_ERR_CORRUPT;
    compute_offsets(L);
    if (get_u64(in + 88) != L->total || L->total > in_size)
        return ORC_ERR_CORRUPT;
    return ORC_OK;
}

int orc_stream_dims(const uint8_t *in, uint64_t in_size, uint64_t dims[3])
{
    layout L;
    int rc = parse_header(in, in_size, &L);
    if (rc)
        return rc;
    for (int i = 0; i < 3; i++)
        dims[i] = L.dims[i];
    return ORC_OK;
}

static int find_outlier(const uint8_t *in, const layout *L, uint64_t g, float *v)
{
    uint64_t lo = 0, hi = L->n_out;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        uint64_t idx = L->idx_bytes == 4 ? get_u32(in + L->off_oidx + 4 * mid)
                                         : get_u64(in + L->off_oidx + 8 * mid);
        if (idx == g) {
            *v = get_f32(in + L->off_oval + 4 * mid);
            return 1;
        }
        if (idx < g)
            lo = mid + 1;
        else
            hi = mid;
    }
    return 0;
}

int orc_decompress(const uint8_t *in, uint64_t in_size, float *out,
                   uint64_t out_cap, uint64_t dims_out[3], uint8_t *codes_dbg)
{
    layout L;
    int rc = parse_header(in, in_size, &L);
    if (rc)
        return rc;
    if (dims_out)
        for (int i = 0; i < 3; i++)
            dims_out[i] = L.dims[i];
    if (out_cap < L.N || !out)
        return ORC_ERR_BUFSZ;
    const uint64_t N = L.N;
    if (L.flags & 1) {
        float v = get_f32(in + HDR_BYTES);
        for (uint64_t i = 0; i < N; i++)
            out[i] = v;
        return ORC_OK;
    }
    const uint8_t *len = in + OFF_LEN;
    uint8_t *codes = malloc(N);
    uint8_t *seq = (L.flags & ORC_FLAG_REORDER) ? malloc(N) : codes;
    if (!codes || !seq) {
        free(codes);
        if (seq != codes)
            free(seq);
        return ORC_ERR_NOMEM;
    }
    rc = ORC_OK;
    /* the last stages (TP, CR): their chunk sizes, then their data */
    uint8_t *lc_out = NULL;
    if (L.pipe != ORC_PIPE_HF) {
        const uint64_t n_raw = L.pipe == ORC_PIPE_TP ? N : 4 * L.payload_words;
        uint32_t *sizes = malloc(sizeof(uint32_t) * (L.n_lc ? L.n_lc : 1));
        lc_out = L.pipe == ORC_PIPE_TP ? seq : malloc(n_raw ? n_raw : 1);
        if (!sizes || !lc_out)
            rc = ORC_ERR_NOMEM;
        for (uint64_t k = 0; !rc && k < L.n_lc; k++)
            sizes[k] = get_u32(in + L.off_lcsizes + 4 * k);
        if (!rc)
            rc = orc_lc_decode(L.pipe, sizes, in + L.off_payload, L.lc_bytes, lc_out, n_raw);
        free(sizes);
    }
    if (!rc && L.pipe != ORC_PIPE_TP) {
        /* Kraft sum must not exceed one; a single symbol has length one. */
        double kraft = 0.0;
        int nsym = 0;
        for (int i = 0; i < 256; i++)
            if (len[i]) {
                if (len[i] > MAX_CODE_LEN)
                    rc = ORC_ERR_CORRUPT;
                kraft += ldexp(1.0, -len[i]);
                nsym++;
            }
        if (nsym == 0 || (nsym == 1 && kraft != 0.5) || (nsym > 1 && kraft != 1.0))
            rc = ORC_ERR_CORRUPT;
        uint32_t *counts = malloc(sizeof(uint32_t) * (L.n_chunks ? L.n_chunks : 1));
        uint32_t *words = malloc(sizeof(uint32_t) * (L.payload_words ? L.payload_words : 1));
        if (!rc && (!counts || !words))
            rc = ORC_ERR_NOMEM;
        uint64_t sum = 0;
        for (uint64_t k = 0; !rc && k < L.n_chunks; k++) {
            counts[k] = get_u32(in + OFF_CHUNKS + 4 * k);
            sum += counts[k];
        }
        for (uint64_t k = 0; !rc && k < L.payload_words; k++)
            words[k] = L.pipe == ORC_PIPE_HF ? get_u32(in + L.off_payload + 4 * k)
                                             : get_u32(lc_out + 4 * k);
        if (!rc && sum != L.payload_words)
            rc = ORC_ERR_CORRUPT;
        if (!rc)
            rc = orc_huff_decode(words, L.payload_words, counts, N, L.chunk, len, seq);
        free(words);
        free(counts);
    }
    if (lc_out && lc_out != seq)
        free(lc_out);
    if (!rc && seq != codes)
        orc_unreorder(seq, L.dims, codes);
    if (seq != codes)
        free(seq);
    if (!rc) {
        uint64_t zeros = 0, prev = 0;
        for (uint64_t i = 0; i < N; i++)
            zeros += codes[i] == 0;
        if (zeros != L.n_out)
            rc = ORC_ERR_CORRUPT;
        for (uint64_t j = 0; !rc && j < L.n_out; j++) {
            uint64_t idx = L.idx_bytes == 4 ? get_u32(in + L.off_oidx + 4 * j)
                                            : get_u64(in + L.off_oidx + 8 * j);
            if (idx >= N || (j > 0 && idx <= prev))
                rc = ORC_ERR_CORRUPT;
            prev = idx;
        }
    }
    if (rc) {
        free(codes);
        return rc;
    }
    if (codes_dbg)
        memcpy(codes_dbg, codes, N);

    float two_eb = L.eps * 2.0f;
    uint64_t nb[3];
    for (int i = 0; i < 3; i++)
        nb[i] = cdiv(L.dims[i], ANCHOR);
    float *buf = malloc(sizeof(float) * SIDE * SIDE * SIDE);
    if (!buf) {
        free(codes);
        return ORC_ERR_NOMEM;
    }
#ifdef ORC_FACE_CHECK
    if (!fc_begin(N)) {
        free(buf);
        free(codes);
        return ORC_ERR_NOMEM;
    }
#endif
    for (uint64_t a = 0; a < nb[0] && !rc; a++)
        for (uint64_t b = 0; b < nb[1] && !rc; b++)
            for (uint64_t c = 0; c < nb[2] && !rc; c++) {
                block k = make_block(L.dims, a, b, c);
                /* Known values first: anchors (every coordinate a multiple of
                 * 16) from the anchor grid, outliers from the outlier list. */
                for (int i = 0; i < k.n[0] && !rc; i++)
                    for (int j = 0; j < k.n[1] && !rc; j++)
                        for (int m = 0; m < k.n[2] && !rc; m++) {
                            uint64_t X = k.o[0] + i, Y = k.o[1] + j, Z = k.o[2] + m;
                            float *slot = &buf[(i * k.n[1] + j) * k.n[2] + m];
                            *slot = 0.0f;
                            if (X % ANCHOR == 0 && Y % ANCHOR == 0 && Z % ANCHOR == 0) {
                                uint64_t ai = ((X / ANCHOR) * nb[1] + Y / ANCHOR) * nb[2] + Z / ANCHOR;
                                *slot = get_f32(in + L.off_anchors + 4 * ai);
                            } else if (codes[gindex(L.dims, X, Y, Z)] == 0) {
                                if (!find_outlier(in, &L, gindex(L.dims, X, Y, Z), slot))
                                    rc = ORC_ERR_CORRUPT;
                            }
                        }
                if (rc)
                    break;
                run_levels(buf, &k, L.cfg, L.eps, two_eb, 0.0f, codes, NULL, L.dims);
#ifdef ORC_FACE_CHECK
                fc_note_block(buf, &k, L.dims);
#endif
                for (int i = 0; i < k.own[0]; i++)
                    for (int j = 0; j < k.own[1]; j++)
                        for (int m = 0; m < k.own[2]; m++)
                            out[gindex(L.dims, k.o[0] + i, k.o[1] + j, k.o[2] + m)] =
                                buf[(i * k.n[1] + j) * k.n[2] + m];
            }
    free(buf);
    free(codes);
    return rc;
}
