// Bitwise-redundancy lossless stages (Sec. 5.2.3), code reordering by
// interpolation level (Sec. 5.1.4, Eq. reorder) and the row-major outlier
// list of compression when the lossless stage does not see the codes in
// row-major order.
//
// Stages. A stage stream is cut into chunks of kLcChunk bytes; one workgroup
// runs one chunk through every stage of its pipeline in LDS (two ping-pong
// buffers) and stores the result, or the raw chunk when the result is not
// smaller. Chunk offsets in the stream come from a decoupled look-back over
// chunks claimed in order. Per stage, with symbol width k bytes:
//  - TCMS_k: (w << 1) ^ (w >> (8k-1)), arithmetic shift, on each k-byte word
//    (two's complement to magnitude-sign);
//  - BIT_1: bit shuffle: output plane p holds bit p of every byte, byte 8j+i
//    giving bit i of the plane's byte j (an 8x8 bit transpose per group);
//  - RRE_k / RZE_k: a bitmap marks the words that differ from the word before
//    (0 before the first) / that are nonzero, and only those are kept. The
//    stage writes its input length (u16), the bitmap compressed recursively
//    (a bitmap of at most 8 bytes as it is; a longer one as the bitmap of its
//    bytes that differ from the byte before, compressed the same way, then
//    those bytes), the kept words and the bytes after the last whole word.
// Every step is a workgroup-wide flag / scan / compaction over LDS.
#include "hiz_internal.h"

namespace hiz {

constexpr int kLcThreads = 256;
constexpr int kLcBuf = kLcChunk + kLcChunk / 4 + 64; // longest stage input or output
constexpr int kBmLevels = 6;
constexpr int kBmBytes = 3072;                        // every bitmap level of one stage

enum : int { OP_TCMS = 0, OP_BIT = 1, OP_RRE = 2, OP_RZE = 3 };
struct Stage {
    int op, k;
};

template <int P> struct Pipeline;
template <> struct Pipeline<PIPE_TP> {
    static constexpr int n = 3;
    __device__ static Stage at(int i)
    {
        return i == 0 ? Stage{OP_TCMS, 1} : i == 1 ? Stage{OP_BIT, 1} : Stage{OP_RRE, 1};
    }
};
template <> struct Pipeline<PIPE_CR> {
    static constexpr int n = 3;
    __device__ static Stage at(int i)
    {
        return i == 0 ? Stage{OP_RRE, 4} : i == 1 ? Stage{OP_TCMS, 8} : Stage{OP_RZE, 1};
    }
};

struct LcShared {
    alignas(16) uint8_t a[kLcBuf];
    alignas(16) uint8_t b[kLcBuf];
    alignas(16) uint8_t bm[kBmBytes];
    int scan[8];
    int flag;
    uint32_t id;
    uint64_t base, zbase;
};

// ---- small workgroup primitives --------------------------------------------

// Exclusive prefix of v over the workgroup; `total` gets the sum.
__device__ inline int wg_excl_scan(int v, int *tmp, int &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int incl = (int)wave_incl_scan((uint32_t)v);
    if (lane == 63)
        tmp[wv] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kLcThreads / 64; w++) {
        const int x = tmp[w];
        before += w < wv ? x : 0;
        total += x;
    }
    __syncthreads();
    return before + incl - v;
}

__device__ inline uint64_t load_word(const uint8_t *p, int k)
{
    uint64_t v = 0;
    for (int b = 0; b < k; b++)
        v |= (uint64_t)p[b] << (8 * b);
    return v;
}

__device__ inline void store_word(uint8_t *p, int k, uint64_t v)
{
    for (int b = 0; b < k; b++)
        p[b] = (uint8_t)(v >> (8 * b));
}

__device__ inline bool bit_of(const uint8_t *bm, int i) { return (bm[i >> 3] >> (i & 7)) & 1; }

// 8x8 bit transpose: byte i of v, bit p -> byte p of the result, bit i.
__device__ inline uint64_t transpose8(uint64_t x)
{
    uint64_t t;
    t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// Byte sizes of the bitmap levels of m marks; returns the top level.
__device__ inline int bitmap_levels(int m, int nb[kBmLevels], int off[kBmLevels])
{
    nb[0] = (m + 7) / 8;
    off[0] = 0;
    int L = 0;
    while (nb[L] > 8) {
        nb[L + 1] = (nb[L] + 7) / 8;
        off[L + 1] = off[L] + ((nb[L] + 15) & ~15);
        L++;
    }
    return L;
}

// Copy `cnt` elements of width w from src whose mark (bit i of marks) is set,
// in order, to dst; returns how many (same value in every thread).
__device__ int compact(const uint8_t *src, int cnt, int w, const uint8_t *marks, uint8_t *dst,
                       int *tmp)
{
    const int per = (cnt + kLcThreads - 1) / kLcThreads;
    const int i0 = min(cnt, (int)threadIdx.x * per), i1 = min(cnt, i0 + per);
    int c = 0;
    for (int i = i0; i < i1; i++)
        c += bit_of(marks, i);
    int total;
    int o = wg_excl_scan(c, tmp, total);
    for (int i = i0; i < i1; i++)
        if (bit_of(marks, i)) {
            for (int b = 0; b < w; b++)
                dst[(size_t)o * w + b] = src[(size_t)i * w + b];
            o++;
        }
    __syncthreads();
    return total;
}

// Inverse of compact: rebuild `cnt` elements of width w into dst from the
// kept elements at src; an unmarked element repeats the previous element
// (`fill` = 1, 0 before the first) or is zero (`fill` = 0). `avail` bounds the
// kept elements readable at src; returns how many were read, or -1.
__device__ int expand(const uint8_t *src, int avail, int cnt, int w, const uint8_t *marks,
                      bool fill, uint8_t *dst, int *tmp)
{
    const int per = (cnt + kLcThreads - 1) / kLcThreads;
    const int i0 = min(cnt, (int)threadIdx.x * per), i1 = min(cnt, i0 + per);
    int c = 0;
    for (int i = i0; i < i1; i++)
        c += bit_of(marks, i);
    int total;
    int r = wg_excl_scan(c, tmp, total); // kept elements before this thread's range
    if (total * w > avail)
        return -1;
    for (int i = i0; i < i1; i++) {
        const bool m = bit_of(marks, i);
        r += m;
        for (int b = 0; b < w; b++)
            dst[(size_t)i * w + b] = (m || (fill && r > 0)) ? src[(size_t)(r - 1) * w + b] : 0;
    }
    __syncthreads();
    return total;
}

// ---- stages -----------------------------------------------------------------

__device__ void st_tcms(const uint8_t *a, int n, int k, uint8_t *b, bool inv)
{
    const int m = n / k;
    for (int i = threadIdx.x; i < m; i += kLcThreads) {
        const uint64_t w = load_word(a + (size_t)i * k, k);
        uint64_t r;
        if (k == 8) {
            r = inv ? ((w >> 1) ^ (0ull - (w & 1))) : ((w << 1) ^ (uint64_t)((int64_t)w >> 63));
        } else {
            const int bits = 8 * k;
            const uint64_t mask = (1ull << bits) - 1;
            const uint64_t sign = ((w >> (bits - 1)) & 1) ? mask : 0;
            r = inv ? (((w >> 1) ^ ((w & 1) ? mask : 0)) & mask) : (((w << 1) & mask) ^ sign);
        }
        store_word(b + (size_t)i * k, k, r);
    }
    for (int i = m * k + threadIdx.x; i < n; i += kLcThreads)
        b[i] = a[i];
    __syncthreads();
}

__device__ void st_bit(const uint8_t *a, int n, uint8_t *b, bool inv)
{
    const int g = n / 8;
    for (int j = threadIdx.x; j < g; j += kLcThreads) {
        if (!inv) {
            const uint64_t t = transpose8(load_word(a + 8 * j, 8));
#pragma unroll
            for (int p = 0; p < 8; p++)
                b[p * g + j] = (uint8_t)(t >> (8 * p));
        } else {
            uint64_t v = 0;
#pragma unroll
            for (int p = 0; p < 8; p++)
                v |= (uint64_t)a[p * g + j] << (8 * p);
            store_word(b + 8 * j, 8, transpose8(v));
        }
    }
    for (int i = 8 * g + threadIdx.x; i < n; i += kLcThreads)
        b[i] = a[i];
    __syncthreads();
}

// RRE_k (zero = false) / RZE_k (zero = true) of a[0..n) into b; returns the length.
__device__ int st_reduce(const uint8_t *a, int n, int k, bool zero, uint8_t *b, LcShared &S)
{
    const int m = n / k, tail = n - m * k;
    int nb[kBmLevels], off[kBmLevels];
    const int L = bitmap_levels(m, nb, off);
    uint8_t *bm = S.bm;
    // level 0: the word marks
    for (int q = threadIdx.x; q < nb[0]; q += kLcThreads) {
        uint32_t v = 0;
        for (int i = 8 * q; i < min(m, 8 * q + 8); i++) {
            const uint64_t w = load_word(a + (size_t)i * k, k);
            const uint64_t before = i ? load_word(a + (size_t)(i - 1) * k, k) : 0;
            v |= (uint32_t)(zero ? w != 0 : w != before) << (i & 7);
        }
        bm[off[0] + q] = (uint8_t)v;
    }
    __syncthreads();
    // level l + 1: marks of the level-l bytes that differ from the byte before
    for (int l = 0; l < L; l++) {
        const uint8_t *src = bm + off[l];
        for (int q = threadIdx.x; q < nb[l + 1]; q += kLcThreads) {
            uint32_t v = 0;
            for (int j = 8 * q; j < min(nb[l], 8 * q + 8); j++)
                v |= (uint32_t)(src[j] != (j ? src[j - 1] : 0)) << (j & 7);
            bm[off[l + 1] + q] = (uint8_t)v;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b[0] = (uint8_t)(n & 255);
        b[1] = (uint8_t)(n >> 8);
    }
    int o = 2;
    for (int j = threadIdx.x; j < nb[L]; j += kLcThreads)
        b[o + j] = bm[off[L] + j];
    o += nb[L];
    __syncthreads();
    for (int l = L - 1; l >= 0; l--)
        o += compact(bm + off[l], nb[l], 1, bm + off[l + 1], b + o, S.scan);
    o += k * compact(a, m, k, bm + off[0], b + o, S.scan);
    for (int i = threadIdx.x; i < tail; i += kLcThreads)
        b[o + i] = a[(size_t)m * k + i];
    __syncthreads();
    return o + tail;
}

// Inverse of st_reduce on a[0..avail); returns the restored length or -1.
__device__ int st_reduce_inv(const uint8_t *a, int avail, int k, bool zero, uint8_t *b,
                             LcShared &S)
{
    if (avail < 2)
        return -1;
    const int n = a[0] | (a[1] << 8);
    if (n > kLcBuf)
        return -1;
    const int m = n / k, tail = n - m * k;
    int nb[kBmLevels], off[kBmLevels];
    const int L = bitmap_levels(m, nb, off);
    uint8_t *bm = S.bm;
    int pos = 2;
    if (pos + nb[L] > avail)
        return -1;
    for (int j = threadIdx.x; j < nb[L]; j += kLcThreads)
        bm[off[L] + j] = a[pos + j];
    pos += nb[L];
    __syncthreads();
    for (int l = L - 1; l >= 0; l--) {
        const int c = expand(a + pos, avail - pos, nb[l], 1, bm + off[l + 1], true, bm + off[l],
                             S.scan);
        if (c < 0)
            return -1;
        pos += c;
    }
    const int c = expand(a + pos, avail - pos, m, k, bm + off[0], !zero, b, S.scan);
    if (c < 0)
        return -1;
    pos += c * k;
    if (pos + tail != avail)
        return -1;
    for (int i = threadIdx.x; i < tail; i += kLcThreads)
        b[(size_t)m * k + i] = a[pos + i];
    __syncthreads();
    return n;
}

// The pipeline forward on S.a[0..n); the result is left in S.a, its length returned.
template <int P> __device__ int pipe_forward(LcShared &S, int n)
{
    int len = n;
    uint8_t *x = S.a, *y = S.b;
    for (int i = 0; i < Pipeline<P>::n; i++) {
        const Stage st = Pipeline<P>::at(i);
        if (st.op == OP_TCMS)
            st_tcms(x, len, st.k, y, false);
        else if (st.op == OP_BIT)
            st_bit(x, len, y, false);
        else
            len = st_reduce(x, len, st.k, st.op == OP_RZE, y, S);
        uint8_t *t = x;
        x = y;
        y = t;
    }
    if (x != S.a) {
        for (int i = threadIdx.x; i < len; i += kLcThreads)
            S.a[i] = x[i];
        __syncthreads();
    }
    return len;
}

// The pipeline backward on S.a[0..size); returns the restored length (the
// result in S.a) or -1.
template <int P> __device__ int pipe_backward(LcShared &S, int size)
{
    int len = size;
    uint8_t *x = S.a, *y = S.b;
    for (int i = Pipeline<P>::n - 1; i >= 0; i--) {
        const Stage st = Pipeline<P>::at(i);
        if (st.op == OP_TCMS)
            st_tcms(x, len, st.k, y, true);
        else if (st.op == OP_BIT)
            st_bit(x, len, y, true);
        else
            len = st_reduce_inv(x, len, st.k, st.op == OP_RZE, y, S);
        if (len < 0)
            return -1;
        uint8_t *t = x;
        x = y;
        y = t;
    }
    if (x != S.a) {
        for (int i = threadIdx.x; i < len; i += kLcThreads)
            S.a[i] = x[i];
        __syncthreads();
    }
    return len;
}

// Stage-stream input of compression: the code sequence (throughput mode) or
// the Huffman payload's bytes (ratio mode).
__device__ inline uint64_t lc_input_bytes(const Job &J, const FieldState *st)
{
    return J.pipe == PIPE_TP ? J.N : 4 * st->payload_words;
}

// Stream offsets of the stage sections: the chunk-size table and the data.
__device__ inline void lc_offsets(const Job &J, const FieldState *st, uint64_t n_lc,
                                  uint64_t &o_sizes, uint64_t &o_data)
{
    if (J.pipe == PIPE_TP) {
        o_sizes = kOffChunks;
        o_data = st->off_payload;
    } else {
        o_sizes = align16(st->off_oval + 4 * st->n_out);
        o_data = align16(o_sizes + 4 * n_lc);
    }
}

// ---- compression: one workgroup per chunk -----------------------------------
// Chunks of every job of the launch, throughput and ratio mode alike.
__global__ __launch_bounds__(kLcThreads) void k_lc_encode(const Job *__restrict__ jobs, int njobs,
                                                          uint64_t total, Counters *cnt)
{
    __shared__ LcShared S;
    const int t = threadIdx.x;
    if (t == 0)
        S.id = atomicAdd(&cnt->lc_next, 1u);
    __syncthreads();
    const uint64_t id = S.id;
    if (id >= total)
        return;
    const Job &J = jobs[find_job<WK_LC>(jobs, njobs, id)];
    const bool tp = J.pipe == PIPE_TP;
    FieldState *st = J.st;
    if (st->flags & (ST_CONST | ST_NONFINITE))
        return; // every chunk of this field returns here: nobody waits on it
    const uint64_t c = id - J.lc_begin;
    const uint64_t n_in = lc_input_bytes(J, st);
    const uint64_t n_lc = cdiv(n_in, kLcChunk);
    if (c >= n_lc)
        return; // past the end of a payload shorter than its bound
    const uint64_t lo = c * kLcChunk;
    const int n = (int)min<uint64_t>(kLcChunk, n_in - lo);
    HIZ_GLOBAL const uint8_t *src = tp ? gmem(J.seq) + lo : gmem(J.hpay) + lo;
    // raw chunk into LDS (16-byte pieces where they fit)
    const int n16 = n & ~15;
    for (int i = 16 * t; i < n16; i += 16 * kLcThreads)
        *reinterpret_cast<uint4 *>(S.a + i) = gload_u4(src + i);
    for (int i = n16 + t; i < n; i += kLcThreads)
        S.a[i] = src[i];
    __syncthreads();
    // outliers of a row-major code chunk (throughput mode, codes not reordered)
    const bool outl = tp && !J.reorder;
    int zeros = 0, zbefore = 0;
    if (outl) {
        const int per = kLcChunk / kLcThreads;
        for (int i = t * per; i < min(n, (t + 1) * per); i++)
            zeros += S.a[i] == 0;
        int zt;
        zbefore = wg_excl_scan(zeros, S.scan, zt);
        if (t < 64) {
            const uint64_t zb = lookback(J.lb_d, c, (uint64_t)zt);
            if (t == 0)
                S.zbase = zb;
        }
        __syncthreads();
        const uint64_t cap = J.cap;
        const int ib = J.idx_bytes;
        uint64_t z = S.zbase + zbefore;
        HIZ_GLOBAL uint8_t *out = gmem(J.stream);
        for (int i = t * per; i < min(n, (t + 1) * per); i++)
            if (S.a[i] == 0) {
                const uint64_t gi = lo + i;
                if (st->off_oidx + (z + 1) * ib <= cap) {
                    if (ib == 4)
                        reinterpret_cast<HIZ_GLOBAL uint32_t *>(out + st->off_oidx)[z] = (uint32_t)gi;
                    else
                        reinterpret_cast<HIZ_GLOBAL uint64_t *>(out + st->off_oidx)[z] = gi;
                }
                if (st->off_oval + (z + 1) * 4 <= cap)
                    reinterpret_cast<HIZ_GLOBAL float *>(out + st->off_oval)[z] = gmem(J.field)[gi];
                z++;
            }
        if (c == n_lc - 1 && t == 0 && S.zbase + zt != st->n_out)
            atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    }
    int len = tp ? pipe_forward<PIPE_TP>(S, n) : pipe_forward<PIPE_CR>(S, n);
    const bool raw = len >= n;
    if (raw) {
        for (int i = 16 * t; i < n16; i += 16 * kLcThreads)
            *reinterpret_cast<uint4 *>(S.a + i) = gload_u4(src + i);
        for (int i = n16 + t; i < n; i += kLcThreads)
            S.a[i] = src[i];
        len = n;
        __syncthreads();
    }
    if (t < 64) {
        const uint64_t b = lookback(J.lb_c, c, (uint64_t)len);
        if (t == 0)
            S.base = b;
    }
    __syncthreads();
    uint64_t o_sizes, o_data;
    lc_offsets(J, st, n_lc, o_sizes, o_data);
    const uint64_t cap = J.cap;
    HIZ_GLOBAL uint8_t *out = gmem(J.stream);
    const uint64_t dst = o_data + S.base;
    for (int i = t; i < len; i += kLcThreads)
        if (dst + i < cap)
            out[dst + i] = S.a[i];
    if (t == 0) {
        if (o_sizes + 4 * (c + 1) <= cap)
            reinterpret_cast<HIZ_GLOBAL uint32_t *>(out + o_sizes)[c] = (uint32_t)len;
        if (c == n_lc - 1) {
            const uint64_t lc_bytes = S.base + len;
            const uint64_t total_bytes = o_data + lc_bytes;
            st->lc_bytes = lc_bytes;
            st->total_bytes = total_bytes;
            if (H_NLC + 8 <= cap) {
                *reinterpret_cast<HIZ_GLOBAL uint64_t *>(out + H_LCBYTES) = lc_bytes;
                *reinterpret_cast<HIZ_GLOBAL uint64_t *>(out + H_NLC) = n_lc;
                *reinterpret_cast<HIZ_GLOBAL uint64_t *>(out + H_TOTAL) = total_bytes;
            }
            if (total_bytes > cap)
                atomicOr(&st->flags, (uint32_t)ST_OVERFLOW);
        }
    }
    // zero the alignment gaps around the ratio mode's sections (< 16 bytes each)
    if (!tp && c == 0 && t < 32) {
        const uint64_t a0 = t < 16 ? st->off_oval + 4 * st->n_out : o_sizes + 4 * n_lc;
        const uint64_t a1 = t < 16 ? o_sizes : o_data;
        const uint64_t g = a0 + (t & 15);
        if (g < a1 && g < cap)
            out[g] = 0;
    }
}

// ---- decompression: one workgroup per chunk ---------------------------------
__global__ __launch_bounds__(kLcThreads) void k_lc_decode(const Job *__restrict__ jobs, int njobs,
                                                          uint64_t total, Counters *cnt)
{
    __shared__ LcShared S;
    const int t = threadIdx.x;
    if (t == 0)
        S.id = atomicAdd(&cnt->lc_next, 1u);
    __syncthreads();
    const uint64_t id = S.id;
    if (id >= total)
        return;
    const Job &J = jobs[find_job<WK_LC>(jobs, njobs, id)];
    const bool tp = J.pipe == PIPE_TP;
    FieldState *st = J.st;
    const uint64_t c = id - J.lc_begin;
    const uint64_t n_raw = tp ? J.N : 4 * J.payload_words;
    const uint64_t lo = c * kLcChunk;
    const int n = (int)min<uint64_t>(kLcChunk, n_raw - lo);
    HIZ_GLOBAL const uint8_t *in = gmem(J.stream);
    const uint32_t size = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(in + J.off_lcsizes)[c];
    if (t < 64) {
        const uint64_t b = lookback(J.lb_c, c, (uint64_t)size);
        if (t == 0)
            S.base = b;
    }
    if (t == 0)
        S.flag = 0;
    __syncthreads();
    bool bad = size > (uint32_t)n || S.base + size > J.lc_bytes ||
               (c == J.n_lc - 1 && S.base + size != J.lc_bytes);
    int len = -1;
    if (!bad) {
        HIZ_GLOBAL const uint8_t *src = in + J.off_lcdata + S.base;
        for (int i = t; i < (int)size; i += kLcThreads)
            S.a[i] = src[i];
        __syncthreads();
        len = size == (uint32_t)n ? n
              : tp ? pipe_backward<PIPE_TP>(S, (int)size) : pipe_backward<PIPE_CR>(S, (int)size);
        bad = len != n;
    }
    HIZ_GLOBAL uint8_t *dst = tp ? gmem(J.seq) + lo : gmem(J.hpay) + lo;
    if (bad) {
        if (t == 0)
            atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
        for (int i = t; i < n; i += kLcThreads)
            dst[i] = 0;
        return;
    }
    const int n16 = n & ~15;
    for (int i = 16 * t; i < n16; i += 16 * kLcThreads)
        gstore_u4(dst + i, *reinterpret_cast<const uint4 *>(S.a + i));
    for (int i = n16 + t; i < n; i += kLcThreads)
        dst[i] = S.a[i];
    if (tp) {
        // code-0 count, checked against the outlier count
        int z = 0;
        for (int i = t; i < n; i += kLcThreads)
            z += S.a[i] == 0;
        for (int o = 32; o > 0; o >>= 1)
            z += __shfl_xor(z, o, 64);
        if ((t & 63) == 0 && z)
            atomicAdd((unsigned long long *)&st->zeros_seen, (unsigned long long)z);
    }
}

// ---- reordering by interpolation level (Sec. 5.1.4, Eq. reorder) -----------
// Level of a point: the largest l <= 4 with 2^l dividing every coordinate.
// Its index: points of coarser levels first (their count is the product of
// ceil(d / 2^(l+1)) over the axes), then the point's rank in row-major order
// among the level-l points, found on the grid of multiples of 2^l (sizes
// ceil(d / 2^l)) as its row-major index minus the coarser points before it.
// The anchor level is plain row-major order on the anchor grid.
__device__ inline uint64_t level_index(const Job &J, uint64_t x, uint64_t y, uint64_t z)
{
    const uint64_t any = x | y | z;
    const int l = any ? min(4, (int)__builtin_ctzll(any)) : 4;
    const uint64_t r = (1ull << l) - 1;
    const uint64_t Dy = (J.dims[1] + r) >> l, Dz = (J.dims[2] + r) >> l;
    const uint64_t xs = x >> l, ys = y >> l, zs = z >> l;
    uint64_t I = (xs * Dy + ys) * Dz + zs;
    if (l == 4)
        return I;
    const uint64_t r1 = (2ull << l) - 1;
    const uint64_t coarser = ((J.dims[0] + r1) >> (l + 1)) * ((J.dims[1] + r1) >> (l + 1)) *
                             ((J.dims[2] + r1) >> (l + 1));
    const uint64_t hy = (Dy + 1) >> 1, hz = (Dz + 1) >> 1;
    I -= ((xs + 1) >> 1) * hy * hz;
    if (!(xs & 1)) {
        I -= ((ys + 1) >> 1) * hz;
        if (!(ys & 1))
            I -= (zs + 1) >> 1;
    }
    return coarser + I;
}

// inverse = false: seq[I(x,y,z)] = codes[x,y,z]; inverse = true: the reverse.
// Threads take 4 consecutive z of a row; blockIdx.y is the job.
template <bool INV>
__global__ __launch_bounds__(256) void k_reorder(const Job *__restrict__ jobs, int njobs)
{
    const Job &J = jobs[blockIdx.y];
    if (!J.reorder || (J.st->flags & (ST_CONST | ST_NONFINITE)))
        return;
    const uint64_t dz = J.dims[2];
    const uint64_t q = (dz + 3) / 4; // 4-point pieces per row
    const uint64_t rows = J.dims[0] * J.dims[1];
    HIZ_GLOBAL uint8_t *codes = gmem(J.codes);
    HIZ_GLOBAL uint8_t *seq = gmem(J.seq);
    for (uint64_t u = blockIdx.x * 256ull + threadIdx.x; u < rows * q; u += 256ull * gridDim.x) {
        const uint64_t row = u / q, z0 = (u - row * q) * 4;
        const uint64_t x = row / J.dims[1], y = row - x * J.dims[1];
        const uint64_t g = row * dz + z0;
        const int nz = (int)min<uint64_t>(4, dz - z0);
        for (int k = 0; k < nz; k++) {
            const uint64_t I = level_index(J, x, y, z0 + k);
            if (INV)
                codes[g + k] = seq[I];
            else
                seq[I] = codes[g + k];
        }
    }
}

void launch_reorder(const Job *d_jobs, int njobs, uint64_t max_n, bool inverse, hipStream_t s)
{
    if (njobs == 0 || max_n == 0)
        return;
    uint64_t g = cdiv(cdiv(max_n, 4), 256);
    if (g > 16384)
        g = 16384;
    if (inverse)
        hipLaunchKernelGGL(k_reorder<true>, dim3((uint32_t)g, njobs), dim3(256), 0, s, d_jobs,
                           njobs);
    else
        hipLaunchKernelGGL(k_reorder<false>, dim3((uint32_t)g, njobs), dim3(256), 0, s, d_jobs,
                           njobs);
}

// ---- outliers of the row-major code array -----------------------------------
// Units of kLcChunk codes, claimed in order: count the code-0 points, take
// the outlier slot by look-back, write (index, exact value) ascending.
__global__ __launch_bounds__(256) void k_outliers(const Job *__restrict__ jobs, int njobs,
                                                  uint64_t total, Counters *cnt)
{
    __shared__ int s_scan[8];
    __shared__ uint32_t s_id;
    __shared__ uint64_t s_base;
    const int t = threadIdx.x;
    if (t == 0)
        s_id = atomicAdd(&cnt->ou_next, 1u);
    __syncthreads();
    const uint64_t id = s_id;
    if (id >= total)
        return;
    const Job &J = jobs[find_job<WK_OU>(jobs, njobs, id)];
    FieldState *st = J.st;
    if (st->flags & (ST_CONST | ST_NONFINITE))
        return;
    const uint64_t u = id - J.ou_begin;
    const uint64_t lo = u * kLcChunk;
    const int n = (int)min<uint64_t>(kLcChunk, J.N - lo);
    HIZ_GLOBAL const uint8_t *codes = gmem(J.codes) + lo;
    constexpr int per = kLcChunk / 256; // 64 codes per thread
    uint32_t w[per / 4];
    const int i0 = t * per;
    int z = 0;
    if (i0 + per <= n && ((lo + i0) & 3) == 0) {
#pragma unroll
        for (int k = 0; k < per / 4; k++) {
            w[k] = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(codes + i0)[k];
            const uint32_t v = w[k];
            z += ((v & 0xffu) == 0) + ((v & 0xff00u) == 0) + ((v & 0xff0000u) == 0) +
                 ((v & 0xff000000u) == 0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < per / 4; k++) {
            uint32_t v = 0;
            for (int b = 0; b < 4; b++) {
                const int i = i0 + 4 * k + b;
                v |= (uint32_t)(i < n ? codes[i] : 1u) << (8 * b);
            }
            w[k] = v;
            z += ((v & 0xffu) == 0) + ((v & 0xff00u) == 0) + ((v & 0xff0000u) == 0) +
                 ((v & 0xff000000u) == 0);
        }
    }
    int zt;
    const int zb = wg_excl_scan(z, s_scan, zt);
    if (t < 64) {
        const uint64_t b = lookback(J.lb_d, u, (uint64_t)zt);
        if (t == 0)
            s_base = b;
    }
    __syncthreads();
    uint64_t slot = s_base + zb;
    if (z) {
        const uint64_t cap = J.cap;
        const int ib = J.idx_bytes;
        HIZ_GLOBAL uint8_t *out = gmem(J.stream);
        for (int k = 0; k < per; k++) {
            if (((w[k >> 2] >> (8 * (k & 3))) & 0xffu) != 0)
                continue;
            const uint64_t gi = lo + i0 + k;
            if (st->off_oidx + (slot + 1) * ib <= cap) {
                if (ib == 4)
                    reinterpret_cast<HIZ_GLOBAL uint32_t *>(out + st->off_oidx)[slot] = (uint32_t)gi;
                else
                    reinterpret_cast<HIZ_GLOBAL uint64_t *>(out + st->off_oidx)[slot] = gi;
            }
            if (st->off_oval + (slot + 1) * 4 <= cap)
                reinterpret_cast<HIZ_GLOBAL float *>(out + st->off_oval)[slot] = gmem(J.field)[gi];
            slot++;
        }
    }
    if (t == 0 && u == J.n_ou - 1 && s_base + zt != st->n_out)
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
}

void launch_outliers(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s)
{
    if (total == 0)
        return;
    hipLaunchKernelGGL(k_outliers, dim3((uint32_t)total), dim3(256), 0, s, d_jobs, njobs, total,
                       cnt);
}

void launch_lc_encode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s)
{
    if (total == 0)
        return;
    hipLaunchKernelGGL(k_lc_encode, dim3((uint32_t)total), dim3(kLcThreads), 0, s, d_jobs, njobs,
                       total, cnt);
}

void launch_lc_decode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s)
{
    if (total == 0)
        return;
    hipLaunchKernelGGL(k_lc_decode, dim3((uint32_t)total), dim3(kLcThreads), 0, s, d_jobs, njobs,
                       total, cnt);
}

} // namespace hiz
