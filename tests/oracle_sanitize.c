/*
 * Sanitizer and face-consistency driver of the CPU oracle (test
 * infrastructure). Built with -fsanitize=address,undefined and
 * -DORC_FACE_CHECK by tests/test_sanitize.py; runs the oracle over seeded
 * fields of many shapes, both bound modes, every lossless pipeline with and
 * without reordering, tuned and fixed configurations, then feeds it damaged
 * streams. Exit status 0 means: every round trip held the bound, every shared
 * face point was computed identically by every block containing it, and no
 * sanitizer fired.
 */
#include "hiz_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

/* xorshift64* (Vigna): the driver's own seeded inputs */
static uint64_t next_u64(void)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}

static double next_unit(void) { return (double)(next_u64() >> 11) / 9007199254740992.0; }

/* A smooth field (sum of sines) plus a little noise. */
static float *make_field(const uint64_t d[3])
{
    const uint64_t N = d[0] * d[1] * d[2];
    float *x = malloc(sizeof(float) * N);
    const double fx = 0.1 + next_unit(), fy = 0.1 + next_unit(), fz = 0.1 + next_unit();
    for (uint64_t i = 0; i < d[0]; i++)
        for (uint64_t j = 0; j < d[1]; j++)
            for (uint64_t k = 0; k < d[2]; k++)
                x[(i * d[1] + j) * d[2] + k] =
                    (float)(sin(fx * i) + cos(fy * j) * sin(fz * k) + 0.01 * next_unit());
    return x;
}

static int fails = 0;

static void check(int cond, const char *what, const uint64_t d[3], int pipe, int reorder)
{
    if (!cond) {
        fprintf(stderr, "FAIL %s dims %llu %llu %llu pipeline %d reorder %d\n", what,
                (unsigned long long)d[0], (unsigned long long)d[1], (unsigned long long)d[2],
                pipe, reorder);
        fails++;
    }
}

int main(void)
{
    const uint64_t shapes[][3] = {{1, 1, 1},  {1, 1, 70},  {2, 3, 65},   {17, 17, 17},
                                  {33, 20, 9}, {40, 3, 18}, {16, 16, 16}, {35, 47, 51},
                                  {65, 2, 2},  {1, 40, 33}};
    const int nshapes = (int)(sizeof(shapes) / sizeof(shapes[0]));
    for (int si = 0; si < nshapes; si++) {
        const uint64_t *d = shapes[si];
        const uint64_t N = d[0] * d[1] * d[2];
        float *x = make_field(d);
        float *y = malloc(sizeof(float) * N);
        for (int pipe = 0; pipe <= 2; pipe++)
            for (int reorder = 0; reorder <= 1; reorder++) {
                orc_params p;
                memset(&p, 0, sizeof(p));
                p.tune = (si + pipe) % 2;
                for (int l = 0; l < 4; l++) {
                    p.cfg[l][0] = (uint8_t)((l + si) % 2);
                    p.cfg[l][1] = (uint8_t)((l + pipe) % 2);
                    p.cfg[l][2] = (uint8_t)((l + si + reorder) % 6);
                }
                p.chunk = 256u << (si % 4);
                p.pipeline = pipe;
                p.reorder = reorder;
                const int mode = si % 3 ? ORC_REL : ORC_ABS;
                const double eb = si % 2 ? 1e-3 : 1e-5;
                uint8_t *z = NULL;
                uint64_t zn = 0;
                int rc = orc_compress(x, d, mode, eb, &p, &z, &zn, NULL);
                check(rc == ORC_OK, "compress", d, pipe, reorder);
                if (rc)
                    continue;
                check(orc_face_mismatches() == 0, "faces (compress)", d, pipe, reorder);
                uint64_t dd[3];
                rc = orc_decompress(z, zn, y, N, dd, NULL);
                check(rc == ORC_OK, "decompress", d, pipe, reorder);
                check(orc_face_mismatches() == 0, "faces (decompress)", d, pipe, reorder);
                float vmin = x[0], vmax = x[0];
                for (uint64_t i = 0; i < N; i++) {
                    vmin = x[i] < vmin ? x[i] : vmin;
                    vmax = x[i] > vmax ? x[i] : vmax;
                }
                const double e = mode == ORC_REL ? eb * ((double)vmax - (double)vmin) : eb;
                double worst = 0.0;
                for (uint64_t i = 0; !rc && i < N; i++) {
                    const double a = fabs((double)x[i] - (double)y[i]);
                    worst = a > worst ? a : worst;
                }
                check(worst <= e, "bound", d, pipe, reorder);
                /* damaged copies: a flipped byte, a truncation; any status, no fault */
                uint8_t *bad = malloc(zn);
                for (int t = 0; t < 24; t++) {
                    memcpy(bad, z, zn);
                    const uint64_t at = next_u64() % zn;
                    bad[at] ^= (uint8_t)(1u + next_u64() % 255u);
                    (void)orc_decompress(bad, zn - (t % 3 == 0 ? at / 2 : 0), y, N, dd, NULL);
                }
                free(bad);
                orc_free(z);
            }
        free(x);
        free(y);
    }
    /* the lossless stages on their own, every length around the chunk size */
    for (int pipe = 1; pipe <= 2; pipe++)
        for (uint64_t n = 0; n < 40000; n += 997 + 16384 * (n > 20000)) {
            uint8_t *in = malloc(n + 1), *data = malloc(n + 1), *out = malloc(n + 1);
            uint32_t *sizes = malloc(sizeof(uint32_t) * (orc_lc_chunks(n) + 1));
            for (uint64_t i = 0; i < n; i++)
                in[i] = (uint8_t)(next_unit() < 0.8 ? 128 : next_u64());
            uint64_t nb = 0;
            int rc = orc_lc_encode(pipe, in, n, sizes, data, &nb);
            rc = rc ? rc : orc_lc_decode(pipe, sizes, data, nb, out, n);
            const uint64_t dz[3] = {n, 0, 0};
            check(rc == ORC_OK && memcmp(in, out, n) == 0, "stage round trip", dz, pipe, 0);
            free(in);
            free(data);
            free(out);
            free(sizes);
        }
    printf("oracle_sanitize: %d failures\n", fails);
    return fails ? 1 : 0;
}
