// Internal declarations of the hiz GPU library: stream layout constants, the
// per-field job descriptor the kernels read, the per-field device state the
// kernels write, and the host-side launchers of every kernel.
#pragma once

#include "hiz.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hiz {

// ---- method constants (Sec. 5.1.1: 17^3 blocks, anchors every 16 points) ----
constexpr int kAnchor = 16;
constexpr int kSide = 17;
constexpr int kLevels = 4;      // strides 8, 4, 2, 1
constexpr int kMaxCodeLen = 32; // Huffman length cap
constexpr int kCands = 21;      // tuner candidates: {LIN, CUB, NAT} x {MD, SEQ x 6 orders}

// ---- stream layout (the paper leaves the container open; this one is ours) ----
constexpr uint32_t kMagic = 0x315A4948u; // "HIZ1"
constexpr uint16_t kVersion = 1;
constexpr int kHdrBytes = 128;
constexpr int kOffLen = 128;    // u8 code lengths [256]
constexpr int kOffChunks = 384; // u32 words per chunk [n_chunks]
// header field offsets
constexpr int H_MAGIC = 0, H_VERSION = 4, H_MODE = 6, H_FLAGS = 7, H_DIMS = 8, H_EB = 32,
              H_EPS = 40, H_MIN = 44, H_MAX = 48, H_ASTRIDE = 52, H_NLEV = 53, H_CFG = 56,
              H_CHUNK = 68, H_NOUT = 72, H_PWORDS = 80, H_TOTAL = 88, H_NCHUNKS = 96,
              H_NANCH = 104, H_PIPE = 54, H_LCBYTES = 112, H_NLC = 120;
constexpr uint8_t kFlagConst = 1, kFlagIdx64 = 2, kFlagReorder = 4;

// Lossless pipelines (Sec. 5.2.3): Huffman only; TCMS1-BIT1-RRE1 straight on
// the codes (throughput mode); Huffman, then RRE4-TCMS8-RZE1 on its payload
// (ratio mode). The bitwise-redundancy stages run on chunks of kLcChunk bytes.
enum : uint8_t { PIPE_HF = 0, PIPE_TP = 1, PIPE_CR = 2 };
constexpr int kLcChunk = 16384;
// Exact min/max (REL mode): points per work unit.
constexpr uint64_t kMmUnit = 16384;

__host__ __device__ inline uint64_t align16(uint64_t v) { return (v + 15u) & ~uint64_t(15); }
__host__ __device__ inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// ---- status bits a kernel may raise for a field ----
enum : uint32_t {
    ST_CONST = 1u,     // constant field (REL mode, max == min)
    ST_NONFINITE = 2u, // NaN/Inf in the input
    ST_OVERFLOW = 4u,  // a write would pass the output capacity
    ST_CORRUPT = 8u,   // decoder found an inconsistent stream
};

// Decoder lookup tables of one field, built once per decompression.
constexpr int kLutBits = 13;
// Decoder lookup entry for the next kLutBits payload bits: the one or two
// whole codes that fit in them. Bits 0..4: 32 - (their total length); bits
// 5..6: how many (1 or 2); bits 8..15, 16..23: the symbols in order; bits
// 24..28: the length of the first code. 0: the first code is longer than
// kLutBits bits (its length comes from `limit`).
struct DecTables {
    uint32_t lut[1 << kLutBits];
    uint32_t first[kMaxCodeLen + 2]; // first canonical code of each length
    uint32_t count[kMaxCodeLen + 2]; // codes of each length
    uint32_t index[kMaxCodeLen + 2]; // position of the first code of each length in `sorted`
    uint32_t limit[kMaxCodeLen + 2]; // first left-justified 32-bit window past the codes of each length
    uint32_t base[kMaxCodeLen + 2];  // index - first (mod 2^32): sorted[base[L] + code]
    uint8_t sorted[256];             // symbols by (length, symbol)
    uint32_t maxlen;
    uint32_t pad[3];
};

// Device-written state of one field. The first 64 bytes are what the host
// reads back after a call.
struct FieldState {
    uint32_t flags;      // ST_* bits
    uint32_t pad0;
    uint64_t total_bytes;
    uint64_t n_out;
    uint64_t zeros_seen; // decoder: code-0 count
    uint64_t payload_words;
    uint32_t kmin, kmax; // ordered keys of the exact min / max
    float vmin, vmax;
    float eps, two_eb;
    // ---- device-only ----
    float inv;
    uint32_t pad1;
    double tune_scale;
    uint8_t cfg[kLevels][3];
    uint8_t pad2[4];
    uint64_t off_oidx, off_oval, off_payload;
    uint64_t lc_bytes;   // bytes the bitwise-redundancy stages stored
    uint64_t hist[256];
    uint64_t tune_err[kLevels][kCands];
    uint32_t cb_code[256];
    uint8_t cb_len[256];
};
constexpr int kResultBytes = 64;

// Host-written, device-read description of one field of a (batched) call.
struct Job {
    const float *field;  // compress input
    float *out;          // decompress output
    uint8_t *stream;     // compress output / decompress input
    uint64_t cap;        // stream capacity (compress) or size (decompress)
    uint8_t *codes;      // N-byte code workspace
    FieldState *st;
    DecTables *dt;
    uint64_t *lb_a;      // look-back status words (encoder groups: payload words; decoder blocks)
    uint64_t *lb_b;      // look-back status words (encoder groups: outliers)
    uint64_t *woff;      // encoder: payload word offset of each chunk
    uint64_t *zoff;      // encoder: first outlier slot of each chunk
    uint2 *mm_part;      // per-unit (min, max) key partials: minmax units (REL) or tiles (ABS)
    float *crec;         // per full tile: values of its even-point grid after the coarse levels
    uint8_t *ccode;      // per full tile: codes of its owned even points (compression)
    uint64_t dims[3];
    uint64_t N;
    uint32_t nb[3];      // blocks per axis = ceil(d / 16)
    uint32_t ntz;        // tiles along z = ceil(nb[2] / tile_z)
    uint64_t n_anchors;
    uint64_t n_chunks;
    uint64_t off_anchors;
    uint32_t chunk, log2_chunk;
    int32_t mode;
    int32_t tune;
    double eb;
    uint8_t cfg_forced[kLevels][3];
    uint8_t idx_bytes;
    uint8_t pad[3];
    // prefix offsets of this field's work units in each batched work list
    uint64_t mm_begin, tune_begin, tile_begin, chunk_begin, group_begin, dblk_begin, out_begin;
    uint64_t n_mm, n_tune, n_tiles, n_groups, n_dblk;
    uint32_t n_full[3];  // full 17^3 blocks per axis (tuner sample)
    uint32_t nf[3];      // full tiles per axis: coarse slot of tile (bx, by, bz0/TZ) is
                         // (bx * nf[1] + by) * nf[2] + bz0/TZ
    uint32_t pad3;
    uint32_t n_samples;  // tuner sample size
    // decompression: section layout and bound parsed from the header
    uint64_t off_oidx, off_oval, off_payload, n_out, payload_words;
    float eps;
    uint32_t pad2;
    // lossless pipeline and code order
    uint8_t pipe;        // PIPE_*
    uint8_t reorder;     // 1: the lossless stage sees the codes reordered by level
    uint8_t tz;          // tile depth along z (1, 2 or 4 blocks)
    uint8_t pad4;
    uint32_t chunk_req;  // chunk length asked for (recorded in a constant stream's header)
    uint8_t *seq;        // codes in the order the lossless stage sees (== codes if not reordered)
    uint8_t *hpay;       // ratio mode: Huffman payload in the workspace
    uint64_t hpay_cap;   // its capacity in bytes
    uint64_t *lb_c;      // look-back status words: bitwise-redundancy chunks (stored bytes)
    uint64_t *lb_d;      // look-back status words: outlier units / bitwise-redundancy chunks (outliers)
    uint64_t lc_begin, n_lc;   // bitwise-redundancy chunks: work-list prefix, chunks (an upper
                               // bound when compressing the Huffman payload, whose size the
                               // device finds)
    uint64_t ou_begin, n_ou;   // outlier units of kLcChunk codes (compression, separate pass)
    uint64_t off_lcsizes, off_lcdata, lc_bytes; // decompression: from the header
};

// Work list shared by a launch: njobs fields and their concatenated units.
struct JobList {
    const Job *jobs;
    int njobs;
    uint64_t total; // total units of the launch's work kind
};

// Tile depths along z: 1, 2 or 4 blocks (index 0, 1, 2).
constexpr int kTileDepths = 3;

// Counters reset at the start of every call.
struct Counters {
    uint32_t enc_next;
    uint32_t dec_next;
    uint32_t lc_next;      // bitwise-redundancy chunks
    uint32_t ou_next;      // outlier units
    // per tile depth (1, 2, 4) and XCD: tiles claimed by predict / reconstruct
    uint32_t tile_next[kTileDepths][8];
    uint32_t pad[12];
};

// ---- kernel launchers (each defined next to its kernel) ----
enum WorkKind { WK_MM, WK_TUNE, WK_TILE, WK_CHUNK, WK_GROUP, WK_DBLK, WK_OUT, WK_LC, WK_OU };
constexpr int kEncGroupChunks = 64; // chunks per workgroup of the encoder's sizing pass

void launch_init_compress(const Job *d_jobs, int njobs, uint64_t max_chunks, Counters *cnt,
                          hipStream_t s);
void launch_minmax(const Job *d_jobs, int njobs, uint64_t total, int grid, hipStream_t s);
void launch_eps(const Job *d_jobs, int njobs, hipStream_t s);
void launch_tune(const Job *d_jobs, int njobs, uint64_t total, hipStream_t s);
void launch_tune_pick(const Job *d_jobs, int njobs, hipStream_t s);
// The tile kernels run over the tiles [lo, hi) of the work list, which belong
// to the njobs jobs at d_jobs (all of tile depth tile_z); ctr: their eight
// claim counters.
void launch_predict(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z, int grid,
                    uint32_t *ctr, hipStream_t s);
int predict_blocks_per_cu(int tile_z);
void launch_codebook(const Job *d_jobs, int njobs, hipStream_t s);
void launch_encode(const Job *d_jobs, int njobs, uint64_t total_chunks, uint64_t total_groups,
                   Counters *cnt, int grid, hipStream_t s);
int encode_blocks_per_cu();

void launch_fill(float *out, uint64_t n, float v, hipStream_t s);
void launch_gather_results(const Job *d_jobs, int njobs, void *d_dst, hipStream_t s);
void launch_init_decompress(const Job *d_jobs, int njobs, uint64_t max_blocks, Counters *cnt,
                            hipStream_t s);
void launch_dec_tables(const Job *d_jobs, int njobs, hipStream_t s);
// The decoder's work units are sub-blocks of kDecSub chunks, an even number
// per field, so that a workgroup of 2 * kDecSub lanes can take a pair of one
// field. `cus` picks the workgroup size: kDecSub lanes (one workgroup per
// unit) while the units fit the compute units, else 2 * kDecSub.
constexpr int kDecSub = 256;
__host__ __device__ inline uint64_t dec_subblocks(uint64_t chunks) { return 2 * cdiv(chunks, 2 * kDecSub); }
void launch_decode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, int cus, hipStream_t s);
void launch_scatter(const Job *d_jobs, int njobs, uint64_t total, hipStream_t s);
void launch_reconstruct(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z,
                        int grid, uint32_t *ctr, hipStream_t s);
// Levels of stride 8, 4, 2 of every full tile on its grid of even points
// (one wave per tile), ahead of k_predict / k_reconstruct.
void launch_coarse(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z,
                   bool compress, hipStream_t s);
// Values (4 bytes each) and codes of one tile's even-point grid.
uint64_t coarse_values_per_tile(int tile_z);
uint64_t coarse_codes_per_tile(int tile_z);
// Workspace bound over every shape of n points (a stream's field size before
// its header is read): hiz_workspace_bound of an n x 1 x 1 field plus the
// most pre-pass slots any shape of n points can have.
uint64_t workspace_bound_points(uint64_t n);
// Serving helpers (runtime.hip): pinned staging reserved for batches of up to
// n fields; decompression submit with each stream's first kOffChunks bytes
// already copied to the host (nothing waits for the device).
hiz_status ctx_reserve_pinned(hiz_ctx *c, int n);
hiz_status ctx_decompress_submit_hdrs(hiz_ctx *c, int n, const void *const *d_ins,
                                      const uint64_t *in_sizes, float *const *d_fields,
                                      const uint64_t *field_caps, hipStream_t s,
                                      const uint8_t *h_hdrs);
int reconstruct_blocks_per_cu(int tile_z);
// Bitwise-redundancy stages, reordering and outliers (k_lc.hip).
void launch_reorder(const Job *d_jobs, int njobs, uint64_t max_n, bool inverse, hipStream_t s);
void launch_outliers(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s);
void launch_lc_encode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s);
void launch_lc_decode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s);

// ---- device helpers shared by the kernels ----
#ifdef __HIPCC__
// Pointers read from a Job are generic; cast to the global address space the
// kernels' loads and stores compile to global instructions, whose completion
// is counted apart from LDS operations (a generic access is also counted with
// LDS traffic, so every LDS wait would wait for it too).
#define HIZ_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ HIZ_GLOBAL T *gmem(T *p)
{
    return (HIZ_GLOBAL T *)p;
}
// 8- and 16-byte global accesses through the compiler's own vector types (the
// HIP vector structs only work in the generic address space).
typedef float hiz_f4v __attribute__((ext_vector_type(4)));
typedef uint32_t hiz_u4v __attribute__((ext_vector_type(4)));
typedef uint32_t hiz_u2v __attribute__((ext_vector_type(2)));
// Global memory straight into LDS, no registers in between: every lane of
// the wave names its own 4-byte source, and the wave's 64 words land in order
// at dst[0..63] (dst is the same for the whole wave). The loads count as
// vector-memory loads: lds_fill_wait() retires them before a barrier makes
// the words visible to the workgroup.
__device__ __forceinline__ void lds_load_word(HIZ_GLOBAL const float *src, float *dst)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
}
// Workgroup barrier for data exchanged through LDS only: LDS operations
// retire first, global loads and stores stay in flight across it (a
// __syncthreads() would also wait for every outstanding global access, such
// as the next tile's loads issued ahead of time).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
__device__ __forceinline__ void lds_fill_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ float4 gload_f4(HIZ_GLOBAL const float *p)
{
    const hiz_f4v v = *(HIZ_GLOBAL const hiz_f4v *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 gload_u4(HIZ_GLOBAL const uint8_t *p)
{
    const hiz_u4v v = *(HIZ_GLOBAL const hiz_u4v *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
// A streamed load for data read once per call and larger than the caches
// (marked non-temporal).
__device__ __forceinline__ float4 gload_f4_nt(HIZ_GLOBAL const float *p)
{
    const hiz_f4v v = __builtin_nontemporal_load((HIZ_GLOBAL const hiz_f4v *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore_f4(HIZ_GLOBAL float *p, const float4 &v)
{
    hiz_f4v w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(HIZ_GLOBAL hiz_f4v *)p = w;
}
__device__ __forceinline__ void gstore_u4(HIZ_GLOBAL uint8_t *p, const uint4 &v)
{
    hiz_u4v w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(HIZ_GLOBAL hiz_u4v *)p = w;
}
__device__ __forceinline__ void gstore_u2(HIZ_GLOBAL uint2 *p, const uint2 &v)
{
    hiz_u2v w;
    w.x = v.x;
    w.y = v.y;
    *(HIZ_GLOBAL hiz_u2v *)p = w;
}

// Unit u of a launch's work list -> job index (binary search over prefixes).
template <WorkKind K>
__device__ inline uint64_t job_begin(const Job &j)
{
    switch (K) {
    case WK_MM: return j.mm_begin;
    case WK_TUNE: return j.tune_begin;
    case WK_TILE: return j.tile_begin;
    case WK_CHUNK: return j.chunk_begin;
    case WK_GROUP: return j.group_begin;
    case WK_DBLK: return j.dblk_begin;
    case WK_LC: return j.lc_begin;
    case WK_OU: return j.ou_begin;
    default: return j.out_begin;
    }
}

template <WorkKind K>
__device__ inline int find_job(const Job *jobs, int njobs, uint64_t u)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (job_begin<K>(jobs[mid]) <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Min/max of ordered keys over a workgroup of 256 threads; result in lane 0
// of wave 0 (other threads get partial values). `red` is 8 words of LDS.
__device__ inline void block_minmax(uint32_t &kmn, uint32_t &kmx, uint32_t *red)
{
    for (int o = 32; o > 0; o >>= 1) {
        kmn = min(kmn, (uint32_t)__shfl_xor((int)kmn, o, 64));
        kmx = max(kmx, (uint32_t)__shfl_xor((int)kmx, o, 64));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wv] = kmn;
        red[2 * wv + 1] = kmx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) {
            kmn = min(kmn, red[2 * w]);
            kmx = max(kmx, red[2 * w + 1]);
        }
    }
    __syncthreads();
}

// Reduce n (min, max) key partials with the whole workgroup (result in thread 0).
__device__ inline void reduce_partials(const uint2 *p, uint64_t n, uint32_t &kmn, uint32_t &kmx,
                                       uint32_t *red)
{
    kmn = 0xffffffffu;
    kmx = 0u;
    // 8 loads per thread in flight per round trip
    const uint64_t step = blockDim.x;
    for (uint64_t i0 = threadIdx.x; i0 < n; i0 += 8 * step) {
        uint2 v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint64_t i = i0 + k * step;
            v[k] = i < n ? p[i] : make_uint2(0xffffffffu, 0u);
        }
#pragma unroll
        for (int k = 0; k < 8; k++) {
            kmn = min(kmn, v[k].x);
            kmx = max(kmx, v[k].y);
        }
    }
    block_minmax(kmn, kmx, red);
}

// ---------------------------------------------------------------------------
// Look-back status words: [2-bit flag | 62-bit value]; flag 1 = the unit's own
// aggregate, 2 = inclusive prefix through the unit. Each unit publishes its
// aggregate, walks back over predecessors until an inclusive prefix, then
// publishes its own inclusive prefix. Units are handed out in increasing order
// by an atomic counter, so every predecessor is already running.
// ---------------------------------------------------------------------------
constexpr uint64_t LB_AGG = 1ull << 62, LB_INC = 2ull << 62, LB_MASK = (1ull << 62) - 1;

__device__ inline uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lb_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t shfl64(uint64_t v, int src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_sum64(uint64_t v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 32; o > 0; o >>= 1)
        v += shfl64(v, lane ^ o);
    return v;
}

// Exclusive prefix of unit `idx` (called by all 64 lanes of one wave). The
// wave reads the statuses of 64 predecessors per round trip; it stops at the
// nearest inclusive prefix once every unit between is at least published.
__device__ inline uint64_t lookback(uint64_t *arr, uint64_t idx, uint64_t agg)
{
    const int lane = threadIdx.x & 63;
    if (idx == 0) {
        if (lane == 0)
            lb_store(&arr[0], LB_INC | agg);
        return 0;
    }
    if (lane == 0)
        lb_store(&arr[idx], LB_AGG | agg);
    uint64_t excl = 0;
    int64_t end = (int64_t)idx;
    for (;;) {
        const int64_t j = end - 1 - lane;
        const uint64_t w = j >= 0 ? lb_load(&arr[j]) : LB_INC; // before unit 0: inclusive 0
        const uint64_t f = w >> 62;
        const uint64_t inc = __ballot(f == 2);
        const uint64_t empty = __ballot(f == 0);
        if (inc) {
            const int p = __ffsll((unsigned long long)inc) - 1;
            const uint64_t need = (p == 63) ? ~0ull : ((2ull << p) - 1);
            if ((empty & need) == 0) {
                excl += wave_sum64(lane <= p ? (w & LB_MASK) : 0);
                break;
            }
        } else if (empty == 0) {
            excl += wave_sum64(w & LB_MASK);
            end -= 64;
            continue;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0)
        lb_store(&arr[idx], LB_INC | (excl + agg));
    return excl;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = (uint32_t)__shfl_up((int)v, o, 64);
        if (lane >= o)
            v += u;
    }
    return v;
}

__device__ inline uint64_t wave_incl_scan64(uint64_t v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, o, 64);
        uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), o, 64);
        if (lane >= o)
            v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Ordered 32-bit key of a float: unsigned order == total order (-0 < +0).
__device__ inline uint32_t fkey(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float fkey_inv(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}
#endif

} // namespace hiz
