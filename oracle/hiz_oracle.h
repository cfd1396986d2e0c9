/*
 * CPU oracle of the interpolation-based error-bounded compressor (cuSZ-Hi,
 * arXiv 2507.11165): a plain, single-threaded, deliberately slow C
 * implementation of what the GPU library computes.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this library: only the tests, the smoke check and the benchmark's CPU
 * baseline use it. It shares no code, header, table or constant with the GPU
 * library; both are written independently from the paper's method (Sec. 3.1
 * Eq. "general", Sec. 5.1.1-5.1.3, Sec. 5.2.1) and the readings listed in the
 * design notes.
 *
 * Floating point: IEEE FP32 with round-to-nearest-even, every binary operation
 * rounded once, no FMA contraction (build with -ffp-contract=off), denormals
 * kept, correctly rounded division. FP64 only where marked.
 */
#ifndef HIZ_ORACLE_H
#define HIZ_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_ERR_ARG = 1,
    ORC_ERR_NONFINITE = 2,
    ORC_ERR_BUFSZ = 3,
    ORC_ERR_CORRUPT = 4,
    ORC_ERR_NOMEM = 5
};

enum { ORC_ABS = 0, ORC_REL = 1 };
enum { ORC_LIN = 0, ORC_CUB = 1, ORC_NAT = 2 };
/* tuner candidates: {LIN, CUB, NAT} x {MD, SEQ over the 6 dimension orders};
 * candidate index = spline * 7 + (MD ? 0 : 1 + order) */
#define ORC_CANDS 21
enum { ORC_MD = 0, ORC_SEQ = 1 };
/* Lossless pipelines (Sec. 5.2.3): Huffman only; TCMS1-BIT1-RRE1 on the codes
 * (no Huffman, the throughput mode); Huffman then RRE4-TCMS8-RZE1 on its
 * payload (the ratio mode). */
enum { ORC_PIPE_HF = 0, ORC_PIPE_TP = 1, ORC_PIPE_CR = 2 };
/* stream flag: codes reordered by level (Sec. 5.1.4) before the lossless stage */
enum { ORC_FLAG_REORDER = 4 };

/* Per-level interpolation configuration, levels ordered by stride 8, 4, 2, 1.
 * cfg[l][0] = spline (ORC_LIN/ORC_CUB/ORC_NAT), cfg[l][1] = scheme (ORC_MD/ORC_SEQ),
 * cfg[l][2] = dimension order index 0..5 for SEQ:
 * 0 (x,y,z) 1 (x,z,y) 2 (y,x,z) 3 (y,z,x) 4 (z,x,y) 5 (z,y,x). */
typedef struct {
    int tune;              /* 1: choose cfg with the sampled-block tuner */
    uint8_t cfg[4][3];     /* used when tune == 0 */
    uint32_t chunk;        /* Huffman chunk length in symbols (power of 2, 256..65536) */
    int pipeline;          /* ORC_PIPE_* */
    int reorder;           /* 1: reorder the codes by level (Eq. reorder) first */
} orc_params;

/* Optional debug outputs of compress (any pointer may be NULL). */
typedef struct {
    uint8_t *codes;        /* N quantization codes, row-major */
    float *recon;          /* N reconstructed values x' the compressor kept */
    uint64_t hist[256];    /* code histogram */
    uint8_t cfg[4][3];     /* configuration written to the header */
    uint64_t tune_err[4][ORC_CANDS]; /* tuner error sums (when tuned) */
    float eps;             /* absolute bound actually used */
    uint64_t n_out;        /* number of outliers */
} orc_debug;

/* Error bound (Sec. 3.1 Eq. "general"; Sec. 6.1.4 value-range relative bound). */
float orc_eps(int mode, double eb, float vmin, float vmax);

/* One 1-D spline stencil at distance-s samples a=v(t-3s), b=v(t-s), c=v(t+s),
 * d=v(t+3s), with presence flags for a, c, d (Sec. 5.1.2). Returns the
 * prediction and its order rank (4 cubic, 3 quadratic, 2 linear,
 * 1 linear extrapolation, 0 copy). */
float orc_stencil(int spline, float a, float b, float c, float d,
                  int pa, int pc, int pd, int *rank);

/* Prediction of target t of a cell held in buf (extents n), computed from the
 * values currently in buf, for stride s and the given configuration. */
float orc_predict(const float *buf, const int n[3], const int t[3], int s,
                  int spline, int scheme, int perm);

/* Sampled-block tuner (Sec. 5.1.3). */
int orc_tune(const float *x, const uint64_t dims[3], float eps,
             uint8_t cfg[4][3], uint64_t err[4][ORC_CANDS]);

/* Canonical Huffman codebook from a 256-bin histogram. */
int orc_codebook(const uint64_t hist[256], uint8_t len[256], uint32_t code[256]);

/* Canonical codes from given lengths (RFC 1951 Sec. 3.2.2). */
int orc_canonical(const uint8_t len[256], uint32_t code[256]);

/* Chunked bit-packing of n codes; words must hold the worst case
 * (n*32/32 + chunks words); counts gets ceil(n/chunk) word counts. */
int orc_huff_encode(const uint8_t *codes, uint64_t n, uint32_t chunk,
                    const uint8_t len[256], const uint32_t code[256],
                    uint32_t *words, uint64_t *n_words, uint32_t *counts);
int orc_huff_decode(const uint32_t *words, uint64_t n_words, const uint32_t *counts,
                    uint64_t n, uint32_t chunk, const uint8_t len[256], uint8_t *codes);

/* Level of a point and its index in the reordered code sequence
 * (Sec. 5.1.4, Eq. reorder); reorder / unreorder the whole code array. */
int orc_level(uint64_t x, uint64_t y, uint64_t z);
uint64_t orc_reorder_index(const uint64_t dims[3], uint64_t x, uint64_t y, uint64_t z);
void orc_reorder(const uint8_t *codes, const uint64_t dims[3], uint8_t *seq);
void orc_unreorder(const uint8_t *seq, const uint64_t dims[3], uint8_t *codes);

/* Bitwise-redundancy stages (Sec. 5.2.3), chunked: n bytes -> per-chunk
 * stored sizes and concatenated chunk data (data must hold n bytes). */
uint64_t orc_lc_chunks(uint64_t n);
int orc_lc_encode(int pipe, const uint8_t *in, uint64_t n, uint32_t *sizes, uint8_t *data,
                  uint64_t *data_bytes);
int orc_lc_decode(int pipe, const uint32_t *sizes, const uint8_t *data, uint64_t data_bytes,
                  uint8_t *out, uint64_t n);
/* One stage on one buffer: op 0 TCMS, 1 BIT, 2 RRE, 3 RZE, symbol width k;
 * the inverse when inv != 0. n is at most 20480; `out` must hold 20544
 * bytes. Returns the output length, -1 on bad input. */
int orc_lc_stage(int op, int k, int inv, const uint8_t *in, int n, uint8_t *out);

/* Compress / decompress (Sec. 3.1). The stream is allocated with malloc and
 * released with orc_free. */
int orc_compress(const float *x, const uint64_t dims[3], int mode, double eb,
                 const orc_params *p, uint8_t **out, uint64_t *out_size,
                 orc_debug *dbg);
int orc_decompress(const uint8_t *in, uint64_t in_size, float *out,
                   uint64_t out_cap, uint64_t dims[3], uint8_t *codes_dbg);
/* Header fields of a stream: dims, N and whether the stream is valid enough to size. */
int orc_stream_dims(const uint8_t *in, uint64_t in_size, uint64_t dims[3]);

void orc_free(void *p);

#ifdef ORC_FACE_CHECK
/* Debug builds only: shared-face points whose values differed between the
 * blocks that computed them, over the last compress or decompress call. */
uint64_t orc_face_mismatches(void);
#endif

#ifdef __cplusplus
}
#endif
#endif
