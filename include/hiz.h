/*
 * hiz: error-bounded lossy compression of FP32 3-D fields on AMD MI355X
 * (gfx950), after the interpolation compressor cuSZ-Hi (arXiv 2507.11165).
 *
 * The library implements the problem of Sec. 3.1, Eq. "general": a compressor
 * Cmp and decompressor Dec with Z = Cmp(X), X' = Dec(Z) and
 * max_i |x_i - x'_i| <= eps for every element. The lossy stage is the anchor-
 * based, four-level spline interpolation predictor over 17^3 blocks
 * (Sec. 5.1.1-5.1.3) fused with linear-scaling quantization to one-byte codes
 * (Sec. 5.2.1); the lossless stage is Huffman coding of the codes (Sec. 5.2.2).
 *
 * Conventions shared by every entry point:
 *  - Fields are FP32, C-contiguous, shape dims = {dx, dy, dz}; element
 *    (x, y, z) is at linear index (x*dy + y)*dz + z (z fastest).
 *  - Pointers named d_* are device pointers on the context's device; the
 *    caller owns them and the library never frees or retains them past the
 *    call. Buffers passed as d_field must be 4-byte aligned, streams 16-byte
 *    aligned.
 *  - All device work is enqueued on the caller's HIP stream `stream`
 *    (0 = the default stream). Calls that return sizes or statuses
 *    synchronize that stream before returning.
 *  - No call throws; failures return a nonzero hiz_status and leave a message
 *    for hiz_last_error. Output buffers are undefined after a failure.
 *  - A context is not thread-safe: use one context per host thread.
 */
#ifndef HIZ_H
#define HIZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hiz_ctx hiz_ctx;
typedef struct ihipStream_t *hiz_stream_t; /* == hipStream_t */

typedef enum {
    HIZ_OK = 0,
    HIZ_ERR_ARG = 1,       /* invalid argument: zero dims, eb <= 0, NULL, bad params */
    HIZ_ERR_NONFINITE = 2, /* the field holds NaN or Inf */
    HIZ_ERR_BUFSZ = 3,     /* output capacity too small; *out_size holds the size needed */
    HIZ_ERR_CORRUPT = 4,   /* stream fails a structural check */
    HIZ_ERR_NOMEM = 5,     /* device or pinned allocation failed */
    HIZ_ERR_HIP = 6        /* a HIP runtime call failed */
} hiz_status;

/* Error-bound modes (Sec. 3.1; Sec. 6.1.4: the paper's bounds are relative
 * to the value range, eps = eb * (max - min)). */
typedef enum { HIZ_ABS = 0, HIZ_REL = 1 } hiz_eb_mode;

/* Interpolation choices of one level (Sec. 5.1.2). */
/* LINEAR: (1,1)/2; CUBIC: Lagrange (-1,9,9,-1)/16; NATURAL: the natural cubic
 * spline through the four samples, (-3,23,23,-3)/40 (Sec. 5.1.3, "multiple
 * interpolation splines"). Where samples are missing, CUBIC and NATURAL fall
 * back to one-sided quadratics, linear, extrapolation, copy. */
enum { HIZ_SPLINE_LINEAR = 0, HIZ_SPLINE_CUBIC = 1, HIZ_SPLINE_NATURAL = 2 };
enum { HIZ_SCHEME_MD = 0, HIZ_SCHEME_SEQ = 1 };
/* SEQ dimension orders: 0 (x,y,z) 1 (x,z,y) 2 (y,x,z) 3 (y,z,x) 4 (z,x,y) 5 (z,y,x). */

typedef struct {
    /* 1 (default): pick each level's spline and scheme with the sampled-block
     * tuner of Sec. 5.1.3 (21 candidates: 3 splines x {MD, SEQ over the 6
     * dimension orders}); 0: use `level_cfg`. */
    int tune;
    /* Per level, strides 8, 4, 2, 1: {spline, scheme, order}. */
    uint8_t level_cfg[4][3];
    /* Huffman chunk length in symbols: a power of two in [256, 65536];
     * 0 = the library's size-keyed default. Recorded in the stream. */
    uint32_t chunk;
    /* Cells along z per GPU tile (1, 2 or 4); 0 = default. Does not change the
     * output. */
    uint32_t tile_z;
    /* Lossless pipeline (Sec. 5.2.3): HIZ_PIPE_HUFFMAN (default) Huffman
     * coding of the codes; HIZ_PIPE_TP the throughput mode, the stages
     * TCMS1-BIT1-RRE1 straight on the codes (no Huffman); HIZ_PIPE_CR the
     * ratio mode, Huffman then RRE4-TCMS8-RZE1 on its payload. The stages run
     * on 16 KiB chunks; a chunk they cannot shrink is stored raw. */
    uint32_t pipeline;
    /* Codes reordered by interpolation level (Sec. 5.1.4, Eq. reorder) before
     * the lossless stage: 1 on, 0 off, -1 the pipeline's default (on for
     * HIZ_PIPE_CR, off otherwise). Recorded in the stream. */
    int32_t reorder;
} hiz_params;
enum { HIZ_PIPE_HUFFMAN = 0, HIZ_PIPE_TP = 1, HIZ_PIPE_CR = 2 };

/* Header view of a stream (host-side parse; see hiz_inspect). */
typedef struct {
    uint64_t dims[3];
    int mode;
    double eb;
    float eps;          /* absolute bound used; every |x - x'| <= eps */
    float vmin, vmax;   /* exact min and max of the input */
    int constant;       /* 1: constant field stored as one value */
    uint8_t level_cfg[4][3];
    uint32_t chunk;
    uint64_t n_outliers;
    uint64_t n_chunks;
    uint64_t payload_words;
    uint64_t total_bytes;
    int pipeline;       /* HIZ_PIPE_* */
    int reorder;        /* 1: codes reordered by level */
    uint64_t lc_bytes;  /* bytes stored by the last stages (HIZ_PIPE_TP / _CR) */
} hiz_info;

/* Create a context on HIP device `device`. `workspace_bytes` reserves device
 * scratch up front (0 = grow on demand). The context owns its workspace, code
 * buffers and tables; release it with hiz_destroy. */
hiz_status hiz_create(int device, size_t workspace_bytes, hiz_ctx **out);
void hiz_destroy(hiz_ctx *ctx);

/* Message describing the last failure on this context ("" if none). The
 * string lives until the next call on the context. */
const char *hiz_last_error(const hiz_ctx *ctx);

/* Largest stream any field of these dims can produce (every point an
 * outlier and 32-bit codewords); 0 if dims are invalid. */
uint64_t hiz_compress_bound(const uint64_t dims[3]);

/* Device workspace one field of these dims can need inside a (batched) call,
 * in either direction; a context created with the sum over a batch's fields
 * (plus 1 MiB) never grows its workspace for that batch. 0 if dims are
 * invalid. */
uint64_t hiz_workspace_bound(const uint64_t dims[3]);

/* Z = Cmp(X) (Sec. 3.1). Reads the field d_field (dims[0]*dims[1]*dims[2]
 * floats), writes the stream to d_out (capacity out_cap bytes) and its size
 * to *out_size (host memory) after synchronizing `stream`.
 * mode HIZ_REL: eps = eb * (max - min) rounded down to FP32; a field with
 * max == min is stored as a constant stream. params may be NULL (defaults).
 * Errors: HIZ_ERR_ARG, HIZ_ERR_NONFINITE, HIZ_ERR_BUFSZ (*out_size = size
 * needed), HIZ_ERR_NOMEM, HIZ_ERR_HIP. */
hiz_status hiz_compress(hiz_ctx *ctx, const float *d_field, const uint64_t dims[3],
                        hiz_eb_mode mode, double eb, const hiz_params *params,
                        void *d_out, uint64_t out_cap, uint64_t *out_size,
                        hiz_stream_t stream);

/* hiz_compress without any allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, result and errors as hiz_compress, and the
 * same stream bytes. Its workspace is a fixed 256 MiB array in device memory
 * that every GPU the library runs on holds from the library's first use
 * until the process ends (its address on the device is looked up by
 * hiz_create); the call itself makes no device, pinned or host allocation,
 * uses no HIP graph and records no profiling events. A field whose workspace
 * exceeds the array (about 1.9 bytes per point with the Huffman pipeline,
 * so up to about 512^3 points; several times more with HIZ_PIPE_CR or
 * reordering) is rejected with HIZ_ERR_ARG before any device work. Every call
 * on one GPU, from any context, shares that GPU's array: calls that overlap
 * in time on one GPU (other threads, other streams) race and must be
 * serialised by the caller. Synchronizes `stream`. */
hiz_status hiz_compress_noalloc(hiz_ctx *ctx, const float *d_field, const uint64_t dims[3],
                                hiz_eb_mode mode, double eb, const hiz_params *params,
                                void *d_out, uint64_t out_cap, uint64_t *out_size,
                                hiz_stream_t stream);

/* X' = Dec(Z) (Sec. 3.1). Reads the stream d_in (in_size bytes), writes
 * dims[0]*dims[1]*dims[2] floats to d_field (capacity field_cap elements).
 * If dims_out is not NULL it receives the field's dims. Synchronizes `stream`.
 * Errors: HIZ_ERR_CORRUPT, HIZ_ERR_BUFSZ (field_cap too small), HIZ_ERR_ARG,
 * HIZ_ERR_NOMEM, HIZ_ERR_HIP. */
hiz_status hiz_decompress(hiz_ctx *ctx, const void *d_in, uint64_t in_size,
                          float *d_field, uint64_t field_cap, uint64_t dims_out[3],
                          hiz_stream_t stream);

/* Parse the header of a stream held in HOST memory (h_stream, n bytes; the
 * first 384 bytes suffice, a prefix of the stream is enough). Checks the
 * header's internal consistency only. No device work. Errors: HIZ_ERR_CORRUPT,
 * HIZ_ERR_ARG. */
hiz_status hiz_inspect(const void *h_stream, uint64_t n, hiz_info *out);

/* ---- Batches: many independent fields per call -------------------------
 * A batch of n fields of any shapes runs each stage of the method as ONE
 * launch over the concatenated work of all fields (range and bound, tuner,
 * interpolation + quantization + histogram, codebook, encoding; or decoding,
 * outliers, reconstruction). Every field keeps its own bound, tuned level
 * configuration, histogram, codebook and chunk table, so each output stream
 * is byte-identical to what hiz_compress / hiz_decompress give for that
 * field alone. n may be 0; at most 4096.
 *
 * Arrays are host arrays of n entries (dims: 3n values, field i's dims at
 * dims[3i..3i+2]); params, when not NULL, apply to every field and their
 * tile_z is shared. Per-field failures are reported in statuses[i] (may be
 * NULL) and do not stop the other fields; the call returns HIZ_OK when every
 * field succeeded, else the first failing field's status, with a message
 * naming the field. A failure of the call itself (bad n, NULL arrays, no
 * memory, HIP error) returns before any field is processed.
 *
 * The *_submit forms only enqueue the work on `stream` and return; the batch
 * is then pending on the context until hiz_batch_finish (which waits for it)
 * and the context accepts no other call that launches work meanwhile
 * (HIZ_ERR_ARG). Decompression submit reads the stream headers first, so it
 * synchronizes `stream` once before enqueueing. Input and output buffers must
 * stay valid until hiz_batch_finish returns. */
hiz_status hiz_compress_batch(hiz_ctx *ctx, int n, const float *const *d_fields,
                              const uint64_t *dims, const int *modes, const double *ebs,
                              const hiz_params *params, void *const *d_outs,
                              const uint64_t *out_caps, uint64_t *out_sizes,
                              hiz_status *statuses, hiz_stream_t stream);
/* dims_out (3n values, may be NULL) receives each field's dims. */
hiz_status hiz_decompress_batch(hiz_ctx *ctx, int n, const void *const *d_ins,
                                const uint64_t *in_sizes, float *const *d_fields,
                                const uint64_t *field_caps, uint64_t *dims_out,
                                hiz_status *statuses, hiz_stream_t stream);
hiz_status hiz_compress_batch_submit(hiz_ctx *ctx, int n, const float *const *d_fields,
                                     const uint64_t *dims, const int *modes, const double *ebs,
                                     const hiz_params *params, void *const *d_outs,
                                     const uint64_t *out_caps, hiz_stream_t stream);
hiz_status hiz_decompress_batch_submit(hiz_ctx *ctx, int n, const void *const *d_ins,
                                       const uint64_t *in_sizes, float *const *d_fields,
                                       const uint64_t *field_caps, hiz_stream_t stream);
/* 1 when no batch is pending or the pending one has completed on the device
 * (never blocks), else 0. */
int hiz_batch_ready(hiz_ctx *ctx);
/* Wait for the pending batch. sizes[i] (may be NULL): stream bytes of field i
 * (compression; the size needed on HIZ_ERR_BUFSZ) or elements written
 * (decompression). dims (3n, may be NULL): decompressed dims. */
hiz_status hiz_batch_finish(hiz_ctx *ctx, uint64_t *sizes, uint64_t *dims,
                            hiz_status *statuses);

/* HIP-graph replay. When on, each call's launch sequence (Job-table upload,
 * every kernel, result download) is captured once per launch geometry into a
 * HIP graph and replayed by one hipGraphLaunch; calls with the same geometry
 * (field count, shapes, chunk lengths, tuner samples, outlier count for
 * decompression) reuse it. Up to 8 graphs are kept per context. Outputs do
 * not depend on this switch. Fails with HIZ_ERR_ARG while a batch is pending. */
hiz_status hiz_set_graphs(hiz_ctx *ctx, int on);
/* Graphs built and replays launched on this context so far. */
void hiz_graph_stats(const hiz_ctx *ctx, uint64_t *builds, uint64_t *replays);

/* ---- Serving: continuous batching of requests on one device -------------
 * A server owns `slots` contexts (1..16), each with its own HIP stream and a
 * workspace of an equal share of `mem_budget` bytes (0 = a quarter of the
 * device memory free at creation), allocated up front: nothing is allocated
 * while serving, and codebooks, decoder tables and code buffers stay on the
 * device. A background thread forms batches: a free slot takes the oldest
 * waiting request and, behind it in arrival order, further requests of the
 * same kind while the batch fits the slot's workspace (admission by device
 * memory, sized with hiz_workspace_bound) and holds at most `max_batch`
 * requests; requests arriving while batches run are batched onto the next
 * free slot, so batches of different slots overlap on the GPU. Each request
 * gives the same bytes (compress) or field (decompress) as a single call.
 * The caller owns every request buffer and keeps it valid until the
 * request's completion has been polled. params (may be NULL) apply to every
 * compression. Submit and poll are thread-safe. */
typedef struct hiz_server hiz_server;
enum { HIZ_OP_COMPRESS = 0, HIZ_OP_DECOMPRESS = 1 };
typedef struct {
    uint64_t id;         /* caller tag, returned in the completion */
    int op;              /* HIZ_OP_COMPRESS or HIZ_OP_DECOMPRESS */
    const void *d_in;    /* compress: FP32 field; decompress: stream */
    uint64_t in_size;    /* decompress: stream bytes */
    uint64_t dims[3];    /* compress: field dims */
    int mode;            /* compress: hiz_eb_mode */
    double eb;           /* compress: error bound */
    void *d_out;         /* compress: stream buffer; decompress: field buffer */
    uint64_t out_cap;    /* bytes (compress) or elements (decompress) */
} hiz_request;
typedef struct {
    uint64_t id;
    hiz_status status;
    uint64_t size;       /* stream bytes (compress; needed size on BUFSZ) or elements */
    double t_submit, t_start, t_done; /* seconds on hiz_server_clock */
    int batch_size;      /* requests in the batch it ran in */
    int slot;
} hiz_completion;
typedef struct {
    uint64_t submitted, completed, batches;
    int max_running;     /* most batches in flight at once */
    int slots;
    uint64_t slot_capacity;
} hiz_server_stats;

hiz_status hiz_server_create(int device, int slots, uint64_t mem_budget, int max_batch,
                             const hiz_params *params, hiz_server **out);
/* Queue one request (never blocks on the device). A request larger than a
 * slot's workspace completes with HIZ_ERR_NOMEM. */
hiz_status hiz_server_submit(hiz_server *srv, const hiz_request *req);
/* Move up to `max` completions to `out`, oldest first; returns how many. */
int hiz_server_poll(hiz_server *srv, hiz_completion *out, int max);
/* Wait until every submitted request has completed (timeout_s <= 0: no
 * limit); HIZ_ERR_HIP on timeout. Completions stay available to poll. */
hiz_status hiz_server_drain(hiz_server *srv, double timeout_s);
void hiz_server_get_stats(hiz_server *srv, hiz_server_stats *out);
/* The monotonic clock of the completion timestamps, in seconds. */
double hiz_server_clock(void);
/* Finishes every submitted request, then stops the loop and frees the slots. */
void hiz_server_destroy(hiz_server *srv);

/* Per-kernel timing of the calls made on this context while profiling is on
 * (HIP events recorded on the caller's stream around each launch). */
typedef struct {
    char name[32];
    uint64_t launches;
    double total_ms;
} hiz_kernel_stat;

void hiz_set_profiling(hiz_ctx *ctx, int on);
/* Copies up to `max` entries; returns the number of kernels seen. */
int hiz_get_profile(hiz_ctx *ctx, hiz_kernel_stat *out, int max);
void hiz_reset_profile(hiz_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
