// Lossless stage: Huffman coding of the one-byte quantization codes
// (Sec. 5.2.2-5.2.3) -- codebook on the device, chunk-parallel bit-packing with
// a single-pass decoupled look-back for chunk offsets and outlier positions,
// table-driven chunk-parallel decoding, and the outlier scatter of
// decompression.
#include "hiz_internal.h"

#include <type_traits>

namespace hiz {

template <typename T> __device__ inline void put_le(uint8_t *p, T v)
{
    __builtin_memcpy(p, &v, sizeof(T));
}

// ---------------------------------------------------------------------------
// Codebook: two-queue Huffman construction over the leaves sorted by
// (count, symbol), the leaf taken first on equal weights; lengths capped at
// 32 bits by halving the counts (kept >= 1) and rebuilding; canonical codes
// as in DEFLATE (RFC 1951 Sec. 3.2.2). One workgroup per field; the
// sequential merge runs in one thread (255 steps at most).
// Also writes the header, the code lengths and the section layout, and zeroes
// the alignment gaps between sections.
// ---------------------------------------------------------------------------
__device__ void write_header(uint8_t *h, const Job &J, uint8_t flags, float eps, float vmin,
                             float vmax, const uint8_t cfg[kLevels][3], uint64_t n_out,
                             uint64_t n_chunks, uint64_t n_anchors, uint64_t total)
{
    for (int i = 0; i < kHdrBytes; i++)
        h[i] = 0;
    put_le<uint32_t>(h + H_MAGIC, kMagic);
    put_le<uint16_t>(h + H_VERSION, kVersion);
    h[H_MODE] = (uint8_t)J.mode;
    h[H_FLAGS] = flags;
    for (int k = 0; k < 3; k++)
        put_le<uint64_t>(h + H_DIMS + 8 * k, J.dims[k]);
    put_le<double>(h + H_EB, J.eb);
    put_le<float>(h + H_EPS, eps);
    put_le<float>(h + H_MIN, vmin);
    put_le<float>(h + H_MAX, vmax);
    h[H_ASTRIDE] = kAnchor;
    h[H_NLEV] = kLevels;
    for (int l = 0; l < kLevels; l++)
        for (int k = 0; k < 3; k++)
            h[H_CFG + 3 * l + k] = cfg[l][k];
    // a constant stream records the chunk length asked for, whatever the pipeline
    put_le<uint32_t>(h + H_CHUNK, (flags & kFlagConst) ? J.chunk_req : J.chunk);
    put_le<uint64_t>(h + H_NOUT, n_out);
    put_le<uint64_t>(h + H_TOTAL, total);
    put_le<uint64_t>(h + H_NCHUNKS, n_chunks);
    put_le<uint64_t>(h + H_NANCH, n_anchors);
    h[H_PIPE] = (flags & kFlagConst) ? (uint8_t)PIPE_HF : J.pipe;
}

__global__ __launch_bounds__(256) void k_codebook(const Job *__restrict__ jobs, int njobs)
{
    const Job &J = jobs[blockIdx.x];
    FieldState *st = J.st;
    __shared__ uint64_t cnt[256];
    __shared__ uint64_t key[256];
    __shared__ uint64_t w[512];
    __shared__ int16_t par[512];
    __shared__ uint8_t leafsym[256];
    __shared__ uint8_t len[256];
    __shared__ uint64_t blc[kMaxCodeLen + 2];
    __shared__ uint64_t nextc[kMaxCodeLen + 2];
    __shared__ __align__(16) uint8_t hdr[kHdrBytes];
    __shared__ int s_maxlen;
    __shared__ uint8_t s_cfg[kLevels][3];
    const int t = threadIdx.x;
    const uint32_t flags = st->flags;
    if (flags & ST_NONFINITE)
        return;
    uint8_t *out = J.stream;
    const uint64_t cap = J.cap;
    __shared__ uint32_t red[8];
    __shared__ uint32_t s_kmin, s_kmax;
    if (J.mode == 0) {
        // ABS mode: exact min/max from the prediction kernel's per-tile partials
        uint32_t kmn, kmx;
        reduce_partials(J.mm_part, J.n_tiles, kmn, kmx, red);
        if (t == 0) {
            s_kmin = kmn;
            s_kmax = kmx;
            st->kmin = kmn;
            st->kmax = kmx;
        }
    } else if (t == 0) {
        s_kmin = st->kmin;
        s_kmax = st->kmax;
    }
    __syncthreads();
    const float vmin = fkey_inv(s_kmin), vmax = fkey_inv(s_kmax);
    if (flags & ST_CONST) {
        if (t < kLevels * 3)
            s_cfg[t / 3][t % 3] = (t % 3 == 0) ? 1 : 0;
        __syncthreads();
        const uint64_t total = kHdrBytes + 4;
        if (t == 0)
            write_header(hdr, J, kFlagConst, 0.0f, vmin, vmax, s_cfg, 0, 0, 0, total);
        __syncthreads();
        if (t < kHdrBytes / 4 && 4 * (uint64_t)t + 4 <= cap)
            reinterpret_cast<uint32_t *>(out)[t] = reinterpret_cast<const uint32_t *>(hdr)[t];
        if (t == 0) {
            if (total <= cap)
                *reinterpret_cast<float *>(out + kHdrBytes) = J.field[0];
            else
                atomicOr(&st->flags, (uint32_t)ST_OVERFLOW);
            st->total_bytes = total;
            st->payload_words = 0;
            st->n_out = 0;
        }
        return;
    }

    // throughput mode: no Huffman stage, every code length 0
    cnt[t] = J.pipe == PIPE_TP ? 0 : st->hist[t];
    for (;;) {
        __syncthreads();
        const uint64_t c = cnt[t];
        // (count, symbol) as one key, 0 for an absent symbol (counts stay below
        // 2^56); the rank of a present symbol is the number of present keys
        // below its own, and key - 1 wraps an absent one past every other key
        key[t] = c ? (c << 8) | (uint64_t)t : 0;
        __syncthreads();
        int rank = 0;
        if (c) {
            const uint64_t km = key[t] - 1;
#pragma unroll 8
            for (int j = 0; j < 256; j++)
                rank += (key[j] - 1) < km;
        }
        const int n = __syncthreads_count(c != 0);
        if (c) {
            leafsym[rank] = (uint8_t)t;
            w[rank] = c;
        }
        len[t] = 0;
        __syncthreads();
        if (t == 0) {
            if (n == 1) {
                len[leafsym[0]] = 1;
            } else if (n > 1) {
                // nodes 0..n-1: sorted leaves; n..2n-2: merged nodes in creation order
                const uint64_t INF = ~0ull;
                int lq = 0, iq = n, next = n;
                uint64_t wl = w[0], wi = INF;
                for (int step = 0; step < n - 1; step++) {
                    int p0, p1;
                    uint64_t a, b;
                    if (wl <= wi) {
                        p0 = lq++;
                        a = wl;
                        wl = lq < n ? w[lq] : INF;
                    } else {
                        p0 = iq++;
                        a = wi;
                        wi = iq < next ? w[iq] : INF;
                    }
                    if (wl <= wi) {
                        p1 = lq++;
                        b = wl;
                        wl = lq < n ? w[lq] : INF;
                    } else {
                        p1 = iq++;
                        b = wi;
                        wi = iq < next ? w[iq] : INF;
                    }
                    const uint64_t sum = a + b;
                    w[next] = sum;
                    par[p0] = (int16_t)next;
                    par[p1] = (int16_t)next;
                    if (iq == next)
                        wi = sum; // the new node is the front of the empty merged queue
                    next++;
                }
            }
            s_maxlen = 0;
        }
        __syncthreads();
        if (n > 1 && t < n) {
            // depth of leaf t: parent hops up to the root (node 2n-2)
            int v = t, d = 0;
            const int root = 2 * n - 2;
            while (v != root) {
                v = par[v];
                d++;
            }
            len[leafsym[t]] = (uint8_t)min(d, 255);
            atomicMax(&s_maxlen, d);
        } else if (n == 1 && t == 0) {
            s_maxlen = 1;
        }
        __syncthreads();
        if (s_maxlen <= kMaxCodeLen)
            break;
        if (cnt[t]) {
            const uint64_t h = cnt[t] >> 1;
            cnt[t] = h ? h : 1;
        }
    }
    // canonical codes
    if (t < kMaxCodeLen + 2)
        blc[t] = 0;
    __syncthreads();
    const int L = len[t];
    if (L)
        atomicAdd((unsigned long long *)&blc[L], 1ull);
    __syncthreads();
    if (t == 0) {
        uint64_t code = 0;
        blc[0] = 0;
        for (int b = 1; b <= kMaxCodeLen; b++) {
            code = (code + blc[b - 1]) << 1;
            nextc[b] = code;
        }
    }
    __syncthreads();
    uint32_t mycode = 0;
    if (L) {
        uint32_t k = 0;
        for (int j = 0; j < t; j++)
            k += (len[j] == L);
        mycode = (uint32_t)(nextc[L] + k);
    }
    st->cb_len[t] = (uint8_t)L;
    st->cb_code[t] = mycode;
    if (kOffLen + (uint64_t)t < cap)
        out[kOffLen + t] = (uint8_t)L;

    // layout of the variable sections and the header
    const uint64_t n_out = st->hist[0];
    const uint64_t ib = J.idx_bytes;
    // the table at 384: Huffman word counts, or the stage chunk sizes (throughput mode)
    const uint64_t end_chunks = kOffChunks + 4 * (J.pipe == PIPE_TP ? J.n_lc : J.n_chunks);
    const uint64_t end_anch = J.off_anchors + 4 * J.n_anchors;
    const uint64_t o_idx = align16(end_anch);
    const uint64_t end_idx = o_idx + ib * n_out;
    const uint64_t o_val = align16(end_idx);
    const uint64_t end_val = o_val + 4 * n_out;
    const uint64_t o_pay = align16(end_val);
    if (t < kLevels * 3)
        s_cfg[t / 3][t % 3] = st->cfg[t / 3][t % 3];
    __syncthreads();
    if (t == 0) {
        st->n_out = n_out;
        st->off_oidx = o_idx;
        st->off_oval = o_val;
        st->off_payload = o_pay;
        st->vmin = vmin;
        st->vmax = vmax;
        write_header(hdr, J, (uint8_t)((ib == 8 ? kFlagIdx64 : 0) | (J.reorder ? kFlagReorder : 0)),
                     st->eps, vmin, vmax, s_cfg, n_out, J.n_chunks, J.n_anchors, 0);
    }
    __syncthreads();
    if (t < kHdrBytes / 4 && 4 * (uint64_t)t + 4 <= cap)
        reinterpret_cast<uint32_t *>(out)[t] = reinterpret_cast<const uint32_t *>(hdr)[t];
    // zero the alignment gaps (each shorter than 16 bytes)
    if (t < 64) {
        const int gap = t >> 4, k = t & 15;
        const uint64_t lo = gap == 0 ? end_chunks : gap == 1 ? end_anch : gap == 2 ? end_idx : end_val;
        const uint64_t hi = gap == 0 ? J.off_anchors : gap == 1 ? o_idx : gap == 2 ? o_val : o_pay;
        if (lo + k < hi && lo + k < cap)
            out[lo + k] = 0;
    }
}

void launch_codebook(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_codebook, dim3(njobs), dim3(256), 0, s, d_jobs, njobs);
}

// ---------------------------------------------------------------------------
// Encoder, in two passes over the codes.
//  1. k_enc_sizes: a workgroup sizes 64 consecutive chunks (codeword bits and
//     outliers per chunk), scans them, and takes one decoupled look-back over
//     the preceding groups to turn them into each chunk's payload word offset
//     and first outlier slot; it also writes the stream's chunk table and,
//     for the last group, the payload size and total stream size.
//  2. k_enc_pack: one wave per chunk, no waiting. Each lane owns a contiguous
//     run of the chunk's symbols; a wave scan of codeword lengths gives every
//     lane its bit offset, lanes OR their bits into an LDS word buffer (words
//     shared with a neighbour lane via LDS atomics), and the wave stores the
//     packed words coalesced at the chunk's offset. Outliers (code 0) are
//     written with their exact values at their slots.
// The codes are read twice; the second read mostly hits the L2/MALL and
// keeps the packing free of any cross-chunk dependency.
// ---------------------------------------------------------------------------
constexpr int kEncSeg = 1024;        // symbols packed per pass of a wave
constexpr int kEncBuf = kEncSeg + 2; // words of a wave's LDS pack buffer
constexpr int kEncWaves = 4;
constexpr int kGroupChunks = kEncGroupChunks;

__device__ inline void load_lane_codes(HIZ_GLOBAL const uint8_t *__restrict__ src, int P, int n,
                                       uint32_t r[4])
{
    // P consecutive codes (P <= 16) starting at src; n = how many are valid
    r[0] = r[1] = r[2] = r[3] = 0;
    if (n == P && (P & 3) == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (k < P / 4)
                r[k] = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(src)[k];
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (k < n)
                r[k >> 2] |= (uint32_t)src[k] << (8 * (k & 3));
    }
}

__device__ inline uint32_t code_at(const uint32_t r[4], int k)
{
    const uint32_t w = (k >> 2) == 0 ? r[0] : (k >> 2) == 1 ? r[1] : (k >> 2) == 2 ? r[2] : r[3];
    return (w >> (8 * (k & 3))) & 255u;
}

// Outlier codes (zero bytes) among the first n codes (n <= 16) of r, four
// at a time: after adding 0x7F to each byte's low seven bits, a byte's top bit
// is clear in (sum | byte) only when the byte is zero.
__device__ inline uint32_t zero_codes(const uint32_t r[4], int n)
{
    uint32_t z = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t x = r[j];
        const uint32_t m = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
        const int nb = n - 4 * j;
        const uint32_t valid = nb >= 4 ? 0xFFFFFFFFu : nb <= 0 ? 0u : (1u << (8 * nb)) - 1u;
        z += __builtin_popcount(m & valid);
    }
    return z;
}

// Inclusive scan over the wave with DPP moves: shifts by 1, 2, 4, 8 lanes
// within each row of 16 (zeros shifted in), then the last lane of row 0 (2)
// added to row 1 (3), then lane 31 to rows 2 and 3. No LDS round trips.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v)
{
    constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kBcast31, 0xc, 0xf, false);
    return (uint32_t)x;
}

// Bits and outliers of one lane's share of a segment.
__device__ inline void lane_sizes(const uint32_t r[4], int n, const uint8_t *len, uint32_t &bits,
                                  uint32_t &zeros)
{
    bits = 0;
#pragma unroll
    for (int k = 0; k < 16; k++)
        if (k < n)
            bits += len[code_at(r, k)];
    zeros = zero_codes(r, n);
}

__global__ __launch_bounds__(256) void k_enc_sizes(const Job *__restrict__ jobs, int njobs,
                                                   uint64_t total, Counters *cnt)
{
    __shared__ uint8_t len[256];
    __shared__ uint32_t s_words[kGroupChunks], s_zeros[kGroupChunks];
    __shared__ uint32_t s_gid;
    // wave and group indices read back as uniform values, so that the job
    // lookup and the job's fields go through scalar loads
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    if (t == 0)
        s_gid = atomicAdd(&cnt->enc_next, 1u);
    __syncthreads();
    const uint64_t gid = (uint32_t)__builtin_amdgcn_readfirstlane(s_gid);
    if (gid >= total)
        return;
    const Job &J = jobs[find_job<WK_GROUP>(jobs, njobs, gid)];
    FieldState *st = J.st;
    if (st->flags & (ST_CONST | ST_NONFINITE))
        return; // every group of this field returns here: nobody waits on it
    len[t] = st->cb_len[t];
    __syncthreads();
    const uint64_t g = gid - J.group_begin;
    const uint64_t cfirst = g * kGroupChunks;
    const int nc = (int)min<uint64_t>(kGroupChunks, J.n_chunks - cfirst);
    // chunks of exactly one segment (kEncSeg codes, 16 per lane)
    const bool seg1 = J.chunk == (uint32_t)kEncSeg;
    constexpr int kw = kGroupChunks / kEncWaves;
    HIZ_GLOBAL const uint8_t *seq = gmem(J.seq);
    if (seg1 && nc == kGroupChunks && ((cfirst + kGroupChunks) << J.log2_chunk) <= J.N) {
        // a whole group of one-segment chunks: the wave's kw chunks are sized
        // in an unrolled sequence with kDepth loads in flight (one load per
        // chunk would leave each chunk waiting out a full memory latency).
        // A lane's bits (<= 16 x 32) and outliers (<= 16) share one word, and
        // so do the chunk's sums (<= 2^15 bits, <= 2^10 outliers).
        constexpr int kDepth = 4;
        HIZ_GLOBAL const uint8_t *p = seq + ((cfirst + wv * kw) << J.log2_chunk) + 16 * lane;
        uint4 q[kDepth];
#pragma unroll
        for (int k = 0; k < kDepth; k++)
            q[k] = gload_u4(p + k * kEncSeg);
#pragma unroll
        for (int k = 0; k < kw; k++) {
            const uint4 v = q[k % kDepth];
            if (k + kDepth < kw)
                q[k % kDepth] = gload_u4(p + (k + kDepth) * kEncSeg);
            uint32_t r[4] = {v.x, v.y, v.z, v.w}, b, z;
            lane_sizes(r, 16, len, b, z);
            const uint32_t bz =
                (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp((z << 16) | b), 63);
            if (lane == 0) {
                s_words[wv * kw + k] = ((bz & 0xFFFFu) + 31) >> 5;
                s_zeros[wv * kw + k] = bz >> 16;
            }
        }
    } else {
        for (int k = 0; k < kw; k++) {
            const int lc = wv * kw + k;
            if (lc >= nc)
                break;
            const uint64_t c0 = (cfirst + lc) << J.log2_chunk;
            const int clen = (int)(min(c0 + J.chunk, J.N) - c0);
            uint64_t bits = 0;
            uint32_t zeros = 0;
            for (int sg = 0; sg * kEncSeg < clen; sg++) {
                const int sl = min(kEncSeg, clen - sg * kEncSeg);
                const int P = (sl + 63) / 64;
                const int n = max(0, min(P, sl - lane * P));
                uint32_t r[4], b, z;
                load_lane_codes(seq + c0 + sg * kEncSeg + lane * P, P, n, r);
                lane_sizes(r, n, len, b, z);
                bits += b;
                zeros += z;
            }
            for (int o = 32; o > 0; o >>= 1) {
                bits += shfl64(bits, lane ^ o);
                zeros += (uint32_t)__shfl_xor((int)zeros, o, 64);
            }
            if (lane == 0) {
                s_words[lc] = (uint32_t)((bits + 31) >> 5);
                s_zeros[lc] = zeros;
            }
        }
    }
    __syncthreads();
    if (wv != 0)
        return;
    const uint64_t w = lane < nc ? s_words[lane] : 0;
    const uint64_t z = lane < nc ? s_zeros[lane] : 0;
    // a group's words and outliers stay below 2^22 (chunks of at most 2^16
    // codes): 32-bit DPP scans
    const uint64_t wi = wave_incl_scan_dpp((uint32_t)w), zi = wave_incl_scan_dpp((uint32_t)z);
    const uint64_t gw = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)wi, 63);
    const uint64_t gz = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)zi, 63);
    const uint64_t wbase = lookback(J.lb_a, g, gw);
    const uint64_t zbase = lookback(J.lb_b, g, gz);
    const uint64_t cap = J.cap;
    if (lane < nc) {
        const uint64_t ck = cfirst + lane;
        gmem(J.woff)[ck] = wbase + wi - w;
        gmem(J.zoff)[ck] = zbase + zi - z;
        if (kOffChunks + 4 * (ck + 1) <= cap)
            reinterpret_cast<HIZ_GLOBAL uint32_t *>(gmem(J.stream) + kOffChunks)[ck] = (uint32_t)w;
    }
    if (lane == 0 && cfirst + nc == J.n_chunks) {
        const uint64_t pw = wbase + gw;
        st->payload_words = pw;
        if (H_TOTAL + 8 <= cap)
            *reinterpret_cast<uint64_t *>(J.stream + H_PWORDS) = pw;
        if (J.pipe == PIPE_HF) {
            // the ratio mode's stream ends after its last stages (sized there)
            const uint64_t total_bytes = st->off_payload + 4 * pw;
            st->total_bytes = total_bytes;
            if (H_TOTAL + 8 <= cap)
                *reinterpret_cast<uint64_t *>(J.stream + H_TOTAL) = total_bytes;
            if (total_bytes > cap)
                atomicOr(&st->flags, (uint32_t)ST_OVERFLOW);
        }
        if (zbase + gz != st->n_out)
            atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    }
}

// A wave-uniform 64-bit value read back from the first lane, so that the
// compiler keeps it in scalar registers. The builtin returns a signed int:
// each half goes back to uint32_t before widening, or a low half at or above
// 2^31 would be sign-extended over the high half.
__device__ __forceinline__ uint64_t uni64(uint64_t u)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    return ((uint64_t)hi << 32) | lo;
}
template <typename T> __device__ __forceinline__ T *uni_ptr(T *p)
{
    return reinterpret_cast<T *>(uni64(reinterpret_cast<uint64_t>(p)));
}

__global__ __launch_bounds__(256, 5) void k_enc_pack(const Job *__restrict__ jobs, int njobs,
                                                  uint64_t total)
{
    // per wave: (code, length) of every symbol, and the pack buffer
    __shared__ uint2 s_cl[kEncWaves][256];
    __shared__ uint32_t s_buf[kEncWaves][kEncBuf];
    // uniform wave index: the chunk loop, the job lookup and the job's fields
    // stay scalar
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint2 *cl = s_cl[wv];
    uint32_t *buf = s_buf[wv];
    for (int k = lane; k < kEncBuf; k += 64)
        buf[k] = 0;
    // values of the current job, loaded again only when the wave moves on to
    // another job
    int cur = -1;
    bool skip = false, cr = false, outl = false;
    int ib = 0;
    uint64_t o_idx = 0, o_val = 0, pay_words_cap = 0, cap = 0;
    HIZ_GLOBAL uint8_t *stream = nullptr;
    HIZ_GLOBAL uint32_t *payload = nullptr;
    HIZ_GLOBAL const float *field = nullptr;
    for (uint64_t id = (uint64_t)blockIdx.x * kEncWaves + wv; id < total;
         id += (uint64_t)gridDim.x * kEncWaves) {
        const int ji = find_job<WK_CHUNK>(jobs, njobs, id);
        const Job &J = jobs[ji];
        if (ji != cur) {
            FieldState *st = J.st;
            cur = ji;
            skip = (st->flags & (ST_CONST | ST_NONFINITE)) != 0;
            if (skip)
                continue;
            // codes left-justified in 32 bits (a symbol without a code: 0)
            for (int k = lane; k < 256; k += 64) {
                const uint32_t L = st->cb_len[k];
                cl[k] = make_uint2(L ? st->cb_code[k] << (32 - L) : 0u, L);
            }
            cap = uni64(J.cap);
            stream = uni_ptr(gmem(J.stream));
            field = uni_ptr(gmem(J.field));
            // the payload goes to the stream, or (ratio mode) to the workspace for the last stages
            cr = __builtin_amdgcn_readfirstlane((int)(J.pipe == PIPE_CR)) != 0;
            const uint64_t off_payload = uni64(st->off_payload);
            payload = cr ? reinterpret_cast<HIZ_GLOBAL uint32_t *>(gmem(J.hpay))
                         : reinterpret_cast<HIZ_GLOBAL uint32_t *>(stream + off_payload);
            payload = uni_ptr(payload);
            pay_words_cap =
                cr ? uni64(J.hpay_cap) / 4 : (cap > off_payload ? (cap - off_payload) / 4 : 0);
            // outliers here only when these codes are in row-major order
            outl = __builtin_amdgcn_readfirstlane((int)!J.reorder) != 0;
            o_idx = uni64(st->off_oidx);
            o_val = uni64(st->off_oval);
            ib = __builtin_amdgcn_readfirstlane((int)J.idx_bytes);
            wave_sync_lds();
        }
        if (skip)
            continue;
        const uint64_t ck = id - J.chunk_begin;
        const uint64_t c0 = ck << J.log2_chunk;
        const int clen = (int)(min(c0 + J.chunk, J.N) - c0);
        HIZ_GLOBAL const uint8_t *src = gmem(J.seq) + c0;
        // a chunk of exactly one segment: its codes (16 per lane) are loaded
        // together with the chunk's offsets
        const bool one = clen == kEncSeg;
        uint4 pre = make_uint4(0u, 0u, 0u, 0u);
        if (one)
            pre = gload_u4(src + 16 * lane);
        const uint64_t wbase = gmem(J.woff)[ck];
        uint64_t zpos0 = gmem(J.zoff)[ck];
        uint64_t sb = 0; // chunk-relative bit at the segment start
        for (int sg = 0; sg * kEncSeg < clen; sg++) {
            const int sl = min(kEncSeg, clen - sg * kEncSeg);
            const int P = (sl + 63) / 64;
            const int n = max(0, min(P, sl - lane * P));
            const uint64_t gfirst = c0 + (uint64_t)sg * kEncSeg + (uint64_t)lane * P;
            uint32_t r[4] = {pre.x, pre.y, pre.z, pre.w};
            if (!one)
                load_lane_codes(src + sg * kEncSeg + lane * P, P, n, r);
            // every symbol's (code, length) at once; lengths of absent
            // symbols (past n) count zero
            uint2 e[16];
            uint32_t mb = 0, mz = 0;
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const uint32_t c = code_at(r, k);
                e[k] = cl[c];
                if (k >= n)
                    e[k] = make_uint2(0u, 0u);
            }
#pragma unroll
            for (int k = 0; k < 16; k++) {
                mb += e[k].y;
                mz += (k < n) & (code_at(r, k) == 0);
            }
            // one scan for both: a lane's bits (<= 16 x 32) and outliers (<= 16)
            // share a word, and so do the segment's sums (<= 2^15, <= 2^10)
            const uint32_t incl = wave_incl_scan_dpp((mz << 16) | mb);
            const uint32_t ib_incl = incl & 0xFFFFu, iz_incl = incl >> 16;
            const uint32_t seg = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            const uint32_t seg_bits = seg & 0xFFFFu, seg_zero = seg >> 16;
            const uint64_t wseg = sb >> 5;
            // bit of this lane's first code, relative to the buffer's word 0
            uint32_t p = (uint32_t)(sb & 31) + (ib_incl - mb);
            // each code is OR-ed into the (one or two) words it covers; codes
            // are independent of one another. A left-justified code shifted
            // right by its bit offset in the word fills that word; the bits
            // shifted out (the funnel shift of code:0) start the next one. An
            // absent symbol ORs zero.
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const uint32_t cL = e[k].x, sh = p & 31;
                uint32_t *wp = buf + (p >> 5);
                atomicOr(wp, cL >> sh);
                const uint32_t lo = __builtin_amdgcn_alignbit(cL, 0u, sh);
                if (lo)
                    atomicOr(wp + 1, lo);
                p += e[k].y;
            }
            if (outl && mz) {
                uint64_t zpos = zpos0 + (iz_incl - mz);
                for (int k = 0; k < n; k++) {
                    if (code_at(r, k) != 0)
                        continue;
                    const uint64_t gi = gfirst + k;
                    if (o_idx + (zpos + 1) * ib <= cap) {
                        if (ib == 4)
                            reinterpret_cast<HIZ_GLOBAL uint32_t *>(stream + o_idx)[zpos] = (uint32_t)gi;
                        else
                            reinterpret_cast<HIZ_GLOBAL uint64_t *>(stream + o_idx)[zpos] = gi;
                    }
                    if (o_val + (zpos + 1) * 4 <= cap)
                        reinterpret_cast<HIZ_GLOBAL float *>(stream + o_val)[zpos] = field[gi];
                    zpos++;
                }
            }
            wave_sync_lds();
            const uint64_t se = sb + seg_bits;
            const uint32_t nfull = (uint32_t)((se >> 5) - wseg);
            for (uint32_t k = lane; k < nfull; k += 64) {
                const uint64_t gw = wbase + wseg + k;
                if (gw < pay_words_cap)
                    payload[gw] = buf[k];
            }
            const uint32_t partial = (se & 31) ? buf[nfull] : 0u;
            wave_sync_lds();
            for (uint32_t k = lane; k <= nfull; k += 64)
                buf[k] = 0;
            wave_sync_lds();
            if (lane == 0)
                buf[0] = partial;
            wave_sync_lds();
            sb = se;
            zpos0 += seg_zero;
        }
        if (lane == 0) {
            if (sb & 31) {
                const uint64_t gw = wbase + (sb >> 5);
                if (gw < pay_words_cap)
                    payload[gw] = buf[0];
            }
            buf[0] = 0;
        }
        wave_sync_lds();
    }
}

void launch_encode(const Job *d_jobs, int njobs, uint64_t total_chunks, uint64_t total_groups,
                   Counters *cnt, int grid, hipStream_t s)
{
    if (total_chunks == 0)
        return;
    hipLaunchKernelGGL(k_enc_sizes, dim3((uint32_t)total_groups), dim3(256), 0, s, d_jobs, njobs,
                       total_groups, cnt);
    uint64_t need = cdiv(total_chunks, kEncWaves);
    uint64_t g = need < (uint64_t)grid ? need : (uint64_t)grid;
    hipLaunchKernelGGL(k_enc_pack, dim3((uint32_t)g), dim3(64 * kEncWaves), 0, s, d_jobs, njobs,
                       total_chunks);
}

int encode_blocks_per_cu()
{
    int n = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_enc_pack, 64 * kEncWaves, 0);
    return n > 0 ? n : 1;
}

// ---------------------------------------------------------------------------
// Decompression
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_decompress(const Job *__restrict__ jobs, int njobs,
                                                         Counters *cnt)
{
    const Job &J = jobs[blockIdx.y];
    const uint32_t t = threadIdx.x;
    if (blockIdx.x == 0) {
        if (t == 0) {
            J.st->flags = 0;
            J.st->zeros_seen = 0;
            J.st->total_bytes = 0;
            J.st->n_out = J.n_out;
            J.st->payload_words = J.payload_words;
            J.st->eps = J.eps;
            J.st->two_eb = J.eps * 2.0f;
        }
        if (t < kLevels * 3)
            J.st->cfg[t / 3][t % 3] = J.cfg_forced[t / 3][t % 3];
        if (blockIdx.y == 0 && t < sizeof(Counters) / 4)
            reinterpret_cast<uint32_t *>(cnt)[t] = 0u;
    }
    for (uint64_t i = blockIdx.x * 256ull + t; i < J.n_dblk; i += 256ull * gridDim.x)
        J.lb_a[i] = 0;
    for (uint64_t i = blockIdx.x * 256ull + t; i < J.n_lc; i += 256ull * gridDim.x)
        J.lb_c[i] = 0;
}

void launch_init_decompress(const Job *d_jobs, int njobs, uint64_t max_blocks, Counters *cnt,
                            hipStream_t s)
{
    uint64_t gx = cdiv(max_blocks, 256);
    if (gx < 1)
        gx = 1;
    if (gx > 1024)
        gx = 1024;
    hipLaunchKernelGGL(k_init_decompress, dim3((uint32_t)gx, njobs), dim3(256), 0, s, d_jobs,
                       njobs, cnt);
}

// Decoder tables from the stored code lengths: canonical codes, a direct
// lookup table of up to two codes within kLutBits bits, and per-length ranges
// for longer codes. The lookup table is built by kDecTableParts workgroups
// per field, one slice each (one entry per thread); the first also writes
// the per-length tables.
constexpr int kDecTableParts = 32;

__global__ __launch_bounds__(256) void k_dec_tables(const Job *__restrict__ jobs, int njobs)
{
    const Job &J = jobs[blockIdx.y];
    DecTables *dt = J.dt;
    __shared__ uint8_t len[256];
    __shared__ uint32_t blc[kMaxCodeLen + 2];
    __shared__ uint32_t first[kMaxCodeLen + 2];
    __shared__ uint32_t index[kMaxCodeLen + 2];
    __shared__ uint8_t s_sorted[256];
    const int t = threadIdx.x;
    len[t] = gmem(J.stream)[kOffLen + t];
    if (t < kMaxCodeLen + 2)
        blc[t] = 0;
    __syncthreads();
    const int L = len[t];
    if (L >= 1 && L <= kMaxCodeLen)
        atomicAdd(&blc[L], 1u);
    __syncthreads();
    if (t == 0) {
        uint64_t code = 0;
        uint32_t idx = 0, maxlen = 0;
        blc[0] = 0;
        for (int b = 1; b <= kMaxCodeLen; b++) {
            code = (code + blc[b - 1]) << 1;
            first[b] = (uint32_t)code;
            index[b] = idx;
            idx += blc[b];
            if (blc[b])
                maxlen = (uint32_t)b;
        }
        if (blockIdx.x == 0)
            dt->maxlen = maxlen;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t <= kMaxCodeLen) {
        dt->first[t] = first[t];
        dt->count[t] = blc[t];
        dt->index[t] = index[t];
        dt->base[t] = index[t] - first[t];
        // the codes of length t end where those of length t + 1 start,
        // left-justified: (first + count) << (32 - t), saturated
        const uint64_t end = t >= 1 ? ((uint64_t)first[t] + blc[t]) << (32 - t) : 0;
        dt->limit[t] = end > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)end;
    }
    if (L >= 1 && L <= kMaxCodeLen) {
        uint32_t k = 0;
        for (int j = 0; j < t; j++)
            k += (len[j] == L);
        s_sorted[index[L] + k] = (uint8_t)t;
    }
    __syncthreads();
    if (blockIdx.x == 0)
        dt->sorted[t] = s_sorted[t];
    // this part's table entries, each by itself: the first code that
    // prefixes its index, then a second one if it fits in the rest
    constexpr uint32_t kPart = (1u << kLutBits) / kDecTableParts;
    for (uint32_t e = blockIdx.x * kPart + t; e < (blockIdx.x + 1) * kPart; e += 256) {
        uint32_t used = 0, n = 0, syms = 0, l1 = 0;
        while (n < 2) {
            uint32_t Lc = 0, sym = 0;
            for (uint32_t b = 1; b + used <= (uint32_t)kLutBits; b++) {
                const uint32_t c = (e >> (kLutBits - used - b)) & ((1u << b) - 1u);
                if (blc[b] && c - first[b] < blc[b]) {
                    Lc = b;
                    sym = s_sorted[index[b] + (c - first[b])];
                    break;
                }
            }
            if (!Lc)
                break;
            if (n == 0)
                l1 = Lc;
            syms |= sym << (8 * n);
            n++;
            used += Lc;
        }
        dt->lut[e] = n ? ((32u - used) | (n << 5) | (syms << 8) | (l1 << 24)) : 0u;
    }
}

void launch_dec_tables(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_tables, dim3(kDecTableParts, njobs), dim3(256), 0, s, d_jobs, njobs);
}

// One thread per chunk; a workgroup takes kDecChunks consecutive chunks
// (one or two sub-blocks of one field), finds its payload offset by
// look-back over the stored word counts, and each thread decodes its chunk
// sequentially with the LDS lookup table, up to two codes per table read.
constexpr int kRing = 32;      // payload words of a decoder lane's LDS ring (a power of two)
constexpr int kRowRing = 64;   // a lane's LDS output ring of codes (a power of two)
constexpr int kRowBytes = 68;  // its stride: the ring and padding (odd in words)
constexpr int kFlush = 32;     // codes a lane stores at once: one 32-byte aligned piece

template <int kDecChunks>
__global__ __launch_bounds__(kDecChunks) void k_decode(const Job *__restrict__ jobs, int njobs,
                                                       uint64_t total, Counters *cnt)
{
    static_assert(kDecChunks % kDecSub == 0 && kDecChunks >= 256, "whole sub-blocks");
    constexpr int kWaves = kDecChunks / 64;
    constexpr int kSubs = kDecChunks / kDecSub;
    __shared__ __align__(16) uint32_t lut[1 << kLutBits];
    __shared__ uint32_t limit[kMaxCodeLen + 2], base[kMaxCodeLen + 2];
    __shared__ uint8_t sorted[256];
    __shared__ uint32_t s_id, s_maxlen;
    __shared__ uint64_t s_wsum[kWaves];
    __shared__ uint64_t s_base;
    __shared__ uint32_t s_win[kDecChunks * kRing];
    __shared__ __align__(16) uint8_t s_rows[kDecChunks * kRowBytes];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0)
        s_id = atomicAdd(&cnt->dec_next, 1u);
    __syncthreads();
    // total counts sub-blocks; each field has an even number of them
    const uint64_t id = s_id;
    if (id * kSubs >= total)
        return;
    const Job &J = jobs[find_job<WK_DBLK>(jobs, njobs, id * kSubs)];
    const DecTables *dt = J.dt;
    {
        HIZ_GLOBAL const uint8_t *src = reinterpret_cast<HIZ_GLOBAL const uint8_t *>(gmem(dt->lut));
        uint4 *dst = reinterpret_cast<uint4 *>(lut);
        for (int i = t; i < (1 << kLutBits) / 4; i += kDecChunks)
            dst[i] = gload_u4(src + 16 * i);
    }
    if (t <= kMaxCodeLen) {
        limit[t] = dt->limit[t];
        base[t] = dt->base[t];
    }
    if (t < 256)
        sorted[t] = dt->sorted[t];
    if (t == 0)
        s_maxlen = dt->maxlen;
    // this workgroup's place among the field's workgroups (the look-back index)
    const uint64_t lb = (id * kSubs - J.dblk_begin) / kSubs;
    const uint64_t chunk = lb * kDecChunks + t;
    HIZ_GLOBAL const uint32_t *counts =
        reinterpret_cast<HIZ_GLOBAL const uint32_t *>(gmem(J.stream) + kOffChunks);
    // a chunk of C symbols never needs more than C words (32-bit codewords)
    uint64_t wc = chunk < J.n_chunks ? counts[chunk] : 0;
    if (wc > J.chunk) {
        atomicOr(&J.st->flags, (uint32_t)ST_CORRUPT);
        wc = J.chunk;
    }
    const uint64_t incl = wave_incl_scan64(wc);
    if (lane == 63)
        s_wsum[wv] = incl;
    __syncthreads();
    uint64_t before = 0, blk_total = 0;
    for (int k = 0; k < kWaves; k++) {
        before += (k < wv) ? s_wsum[k] : 0;
        blk_total += s_wsum[k];
    }
    if (wv == 0) {
        const uint64_t b = lookback(J.lb_a, lb, blk_total);
        if (lane == 0)
            s_base = b;
    }
    __syncthreads();
    if (chunk >= J.n_chunks)
        return;
    FieldState *st = J.st;
    const uint64_t start = s_base + before + incl - wc;
    const uint64_t pw = J.payload_words;
    if (pw == 0 || start + wc > pw) {
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
        return;
    }
    if (chunk == J.n_chunks - 1 && start + wc != pw)
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    // the payload: in the stream, or (ratio mode) restored by the last stages
    HIZ_GLOBAL const uint32_t *words =
        J.pipe == PIPE_CR ? reinterpret_cast<HIZ_GLOBAL const uint32_t *>(gmem(J.hpay))
                          : reinterpret_cast<HIZ_GLOBAL const uint32_t *>(gmem(J.stream) + J.off_payload);
    HIZ_GLOBAL uint8_t *codes = gmem(J.seq);
    const uint64_t i0 = chunk << J.log2_chunk, i1 = min(i0 + J.chunk, J.N);
    const uint32_t nsym = (uint32_t)(i1 - i0);
    const uint32_t maxlen = s_maxlen;
    const uint64_t wend = start + wc;
    // Payload words reach the decoder through a per-lane ring of kRing words
    // in LDS, filled from 16-byte aligned groups of four words. The payload
    // starts 16-byte aligned, so a group whose first word lies in the payload
    // stays inside that word's page. Relative index q counts words from
    // base0, the chunk's first word rounded down to a group; word q sits in
    // slot q % kRing of this lane's ring, at s_win[(q % kRing) * kDecChunks +
    // t], so the lanes of a wave touch consecutive words whatever slots they
    // are at. Words before the chunk's start are never taken; words past its
    // end (the next chunk's, or those of a shared line) are decoded as
    // padding, which only the tail rounds see and none of whose codes count.
    //
    // Symbols are decoded in rounds of 8 steps, the same for every lane of
    // the wave. At a round's end a lane with room for 16 more words in its
    // ring requests them into register set r % kSets (r the round), and they
    // enter the ring at the start of round r + kSets, when that set comes
    // round again: the loads have kSets - 1 rounds to arrive. Every round issues the same four
    // 16-byte loads whether or not a lane requests (a lane that does not
    // points them at one line that all such lanes share), so the wait for a
    // set covers its own loads, not the later sets'. A round takes at most 8
    // words (one per step) and reads one more ahead; a lane with fewer than
    // kLow committed words at a round's start takes its pending sets in at
    // once, then loads synchronously if it must (codes far longer than
    // usual).
    constexpr int kSets = 3;
    // committed words a lane holds at a round's start: one per step, plus
    // the word read ahead after the round's last step
    constexpr uint32_t kLow = 9;
    uint32_t *ring = s_win + t;
    // this lane's output ring of kRowRing codes; the stride is odd in
    // words, so lanes at the same position write different banks
    uint8_t *row = s_rows + t * kRowBytes;
    const uint64_t base0 = start & ~3ull;
    const uint32_t r0 = (uint32_t)(start - base0);
    // payload words from base0 on (at least 1: start < pw), capped
    const uint32_t pwr = (uint32_t)min(pw - base0, (uint64_t)0x7FFFFFF0u);
    const uint32_t pwr4 = (pwr + 3u) & ~3u;
    HIZ_GLOBAL const uint32_t *wb = words + base0;
    HIZ_GLOBAL const uint8_t *shared_line = reinterpret_cast<HIZ_GLOBAL const uint8_t *>(gmem(dt->lut));
    // the group of words q..q+3, or the shared line when not wanted or past the payload
    auto group = [&](uint32_t q, bool live) __attribute__((always_inline)) -> uint4 {
        return gload_u4(live && q < pwr ? reinterpret_cast<HIZ_GLOBAL const uint8_t *>(wb + q) : shared_line);
    };
    // words q..q+15 (q a multiple of 16) into their slots
    auto put16 = [&](uint32_t q, const uint4 (&g)[4]) __attribute__((always_inline)) {
        uint32_t *r = ring + (q & 16u) * kDecChunks;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            r[(4 * k + 0) * kDecChunks] = g[k].x;
            r[(4 * k + 1) * kDecChunks] = g[k].y;
            r[(4 * k + 2) * kDecChunks] = g[k].z;
            r[(4 * k + 3) * kDecChunks] = g[k].w;
        }
    };
    static_assert(kRing == 32, "the ring holds two sets of 16 words");
    {
        uint4 g0[4], g1[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            g0[k] = group(4 * k, true);
            g1[k] = group(16 + 4 * k, true);
        }
        put16(0, g0);
        put16(16, g1);
    }
    // words up to wp are in the ring, up to wq in the ring or requested; rp
    // is the next word the bit buffer takes; wp, wq and the sets' first
    // words stay multiples of 16
    uint32_t wp = kRing, wq = kRing, rp;
    uint4 pre[kSets][4];
    uint32_t pq[kSets];
    bool pend[kSets];
#pragma unroll
    for (int s = 0; s < kSets; s++) {
        pq[s] = 0;
        pend[s] = false;
    }
    uint32_t zeros = 0;
    bool bad = false;
    // Ends of the code ranges of the lengths past the table (kLutBits + 1 ..
    // maxlen - 1), left-justified, less one (all ones for the lengths not
    // used): the same for every lane, kept in scalar registers. A code
    // longer than the table has length kLutBits + 1 plus the number of these
    // its window is above.
    uint32_t lim[kMaxCodeLen - kLutBits - 1], base3[3];
#pragma unroll
    for (int k = 0; k < kMaxCodeLen - kLutBits - 1; k++) {
        const int Lk = kLutBits + 1 + k;
        lim[k] = __builtin_amdgcn_readfirstlane((uint32_t)Lk < maxlen ? limit[Lk] - 1u : 0xFFFFFFFFu);
    }
#pragma unroll
    for (int k = 0; k < 3; k++)
        base3[k] = __builtin_amdgcn_readfirstlane(base[kLutBits + 1 + k]);
    // Bit buffer: the next nb (32..63 before a step) payload bits, first bit
    // at the top of hi, then lo; zeros below them. The word after the buffer
    // waits in nextw, so a refill never waits for LDS; rp counts words taken
    // out of the ring. e is the table entry of the buffer's first kLutBits
    // bits, read a step ahead.
    uint32_t hi = ring[(r0 & (kRing - 1)) * kDecChunks], lo = ring[((r0 + 1) & (kRing - 1)) * kDecChunks],
             nextw = ring[((r0 + 2) & (kRing - 1)) * kDecChunks];
    rp = r0 + 3;
    // the ring word at rp, read a step ahead: a refill takes it as the new
    // nextw. It is read right after the step's table read, so the wait for
    // the entry at the next step's start leaves it in flight
    uint32_t nw = ring[(rp & (kRing - 1)) * kDecChunks];
    int nb = 64;
    uint32_t e = lut[hi >> (32 - kLutBits)];
    uint32_t pos = 0, flushed = 0; // codes decoded (padding past the end included) / stored
    uint32_t cb = 0, ub = 0;       // tail rounds: bits taken so far / by the chunk's own codes
    bool tail = false;             // the same for the whole wave
    // One step: the one or two codes of entry e. It shifts the buffer by
    // their length, reads the next entry straight from the shifted buffer (an
    // entry takes at most kLutBits of the 32 or more valid bits), writes the
    // two symbol bytes at the lane's output position (a second byte past the
    // entry's count is overwritten later) and advances by the count, then
    // refills by masks when fewer than 32 bits remain. When some lane of the
    // wave holds a code longer than the table (SLOW, decided for the wave),
    // that lane takes the code's length from the range ends and its symbol
    // from the sorted table first, and every lane reads its next entry after
    // the refill. Past the chunk's last code the steps decode
    // padding; in the tail rounds ub keeps the bits the chunk's own codes
    // took, and only the chunk's own codes can be invalid.
    auto step_as = [&](auto tail_tag, auto slow_tag) __attribute__((always_inline)) {
        constexpr bool TAIL = decltype(tail_tag)::value;
        constexpr bool SLOW = decltype(slow_tag)::value;
        const bool slow = SLOW && e == 0u;
        if (SLOW && slow) {
            // the three lengths past the table first (their sorted-table
            // bases are in scalar registers); longer codes only when some
            // lane of the wave holds one
            uint32_t L = kLutBits + 1 + (hi > lim[0] ? 1u : 0u) + (hi > lim[1] ? 1u : 0u) +
                         (hi > lim[2] ? 1u : 0u);
            uint32_t bL = hi > lim[0] ? (hi > lim[1] ? base3[2] : base3[1]) : base3[0];
            if (__builtin_expect(__any(hi > lim[2]), 0)) {
#pragma unroll
                for (int k = 3; k < kMaxCodeLen - kLutBits - 1; k++)
                    L += hi > lim[k] ? 1u : 0u;
                if (L > kLutBits + 3 && L <= kMaxCodeLen)
                    bL = base[L];
            }
            uint32_t sym = 0;
            if (L > maxlen) {
                bad = bad || !TAIL || pos < nsym;
                L = 1;
            } else {
                sym = sorted[(bL + (hi >> (32 - L))) & 255u];
            }
            if (L == 32) {
                // the entry can shift by at most 31: take one bit here
                hi = __builtin_amdgcn_alignbit(hi, lo, 31u);
                lo <<= 1;
                nb -= 1;
                if (TAIL)
                    cb += 1;
                L = 31;
            }
            e = (32u - L) | (1u << 5) | (sym << 8) | (L << 24);
        }
        const uint32_t tb = (0u - e) & 31u; // bits the entry's codes take
        hi = __builtin_amdgcn_alignbit(hi, lo, e);
        lo <<= tb;
        nb -= (int)tb;
        // refill: m is all ones when fewer than 32 bits remain
        auto refill = [&]() __attribute__((always_inline)) {
            const uint32_t m = (uint32_t)((nb - 32) >> 31);
            hi |= (nextw >> nb) & m;
            lo = (__builtin_amdgcn_alignbit(nextw, 0u, (uint32_t)nb) & m) | (lo & ~m);
            nb += (int)(m & 32u);
            nextw = (nw & m) | (nextw & ~m);
            rp -= m;
        };
        // with no long code in the wave at least 19 bits remain after the
        // shift, so the next entry is read before the refill; otherwise
        // after it
        uint32_t en = 0;
        if (!SLOW)
            en = lut[hi >> (32 - kLutBits)];
        else
            refill();
        row[pos & (kRowRing - 1)] = (uint8_t)(e >> 8);
        row[(pos + 1) & (kRowRing - 1)] = (uint8_t)(e >> 16);
        const uint32_t n = (e >> 5) & 3u;
        if (TAIL) {
            // a second code past the chunk's end is padding: only the first counts
            ub = pos < nsym ? cb + ((pos + n > nsym) ? (e >> 24) : tb) : ub;
            cb += tb;
        }
        pos += n;
        if (!SLOW)
            refill();
        else
            en = lut[hi >> (32 - kLutBits)];
        nw = ring[(rp & (kRing - 1)) * kDecChunks];
        e = en;
    };
    auto step = [&](auto tail_tag) __attribute__((always_inline)) {
        if (__builtin_expect(__any(e == 0u), 0))
            step_as(tail_tag, std::true_type{});
        else
            step_as(tail_tag, std::false_type{});
    };
    auto zbytes = [](uint32_t w, uint32_t valid) -> uint32_t {
        // 0x80 in each byte of w that is zero, then only the valid bytes
        const uint32_t z = ~(((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w | 0x7F7F7F7Fu);
        const uint32_t msk = valid >= 4 ? 0xFFFFFFFFu : ((1u << (8 * valid)) - 1u);
        return (uint32_t)__builtin_popcount(z & msk);
    };
    // One round: set S's words, requested at the end of the round kSets
    // rounds back, enter the ring; the ring is topped up if it runs low; 8
    // steps; a lane holding kFlush codes, or its chunk's last ones, stores
    // them from its output ring, counting code-0 bytes on the way; set S is
    // requested again.
    auto round = [&](auto set_tag) __attribute__((always_inline)) {
        constexpr int S = decltype(set_tag)::value;
        if (pend[S]) {
            put16(pq[S], pre[S]);
            wp += 16;
            pend[S] = false;
        }
        if (__builtin_expect(__any(wp - rp < kLow), 0)) {
            // the pending sets in request order, then a synchronous load
#pragma unroll
            for (int i = 1; i < kSets; i++) {
                const int S2 = (S + i) % kSets;
                if (wp - rp < kLow && pend[S2]) {
                    put16(pq[S2], pre[S2]);
                    wp += 16;
                    pend[S2] = false;
                }
            }
            if (wp - rp < kLow) {
                uint4 g[4];
#pragma unroll
                for (int k = 0; k < 4; k++)
                    g[k] = group(wq + 4 * k, true);
                put16(wq, g);
                wq += 16;
                wp += 16;
            }
        }
        // tail rounds from the first round in which some lane may reach its end
        if (!tail && __any(pos + 16 >= nsym)) {
            tail = true;
            cb = 32u * (rp - r0 - 1) - (uint32_t)nb;
        }
        if (tail) {
#pragma unroll
            for (int k = 0; k < 8; k++)
                step(std::true_type{});
        } else {
#pragma unroll
            for (int k = 0; k < 8; k++)
                step(std::false_type{});
        }
        // a round decodes at most 16 codes, so a lane holds fewer than
        // kFlush + 16 unstored codes at a round's end and one store per
        // round keeps up; each store is one whole 32-byte aligned piece of
        // the chunk's codes (the chunk's last piece may be shorter)
        static_assert(kFlush + 16 + 1 <= kRowRing, "the output ring holds a round's codes");
        if (flushed < nsym && (pos >= flushed + kFlush || pos >= nsym)) {
            const uint8_t *rb = row + (flushed & (kRowRing - 1));
            const uint32_t *rw = reinterpret_cast<const uint32_t *>(rb);
            uint32_t w[kFlush / 4];
#pragma unroll
            for (int k = 0; k < kFlush / 4; k++)
                w[k] = rw[k];
            const uint32_t cnt = min((uint32_t)kFlush, nsym - flushed);
            const uint64_t o = i0 + flushed;
            if (cnt == kFlush) {
#pragma unroll
                for (int k = 0; k < kFlush / 16; k++)
                    gstore_u4(codes + o + 16 * k, make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]));
#pragma unroll
                for (int k = 0; k < kFlush / 4; k++)
                    zeros += zbytes(w[k], 4);
            } else {
                for (uint32_t k = 0; k < cnt; k++)
                    codes[o + k] = rb[k];
#pragma unroll
                for (int k = 0; k < kFlush / 4; k++)
                    zeros += zbytes(w[k], cnt > 4u * k ? cnt - 4u * k : 0u);
            }
            flushed += kFlush;
        }
        // request, at the round's end, where any wait it needs is for LDS
        // work that the next step waits for anyway: words up to wq - rp + 16
        // fit the ring. The four groups are loaded from one base address at
        // offsets 0, 16, 32 and 48 bytes, each offset capped so that the
        // group starts inside the payload (a capped group repeats an earlier
        // one: its words are past the payload's end and only decoded as
        // padding); a lane that does not request, or whose words are all
        // past the payload, reads the shared line
        const bool want = wq - rp <= kRing - 16;
        {
            const bool live = want && wq < pwr;
            HIZ_GLOBAL const uint8_t *src =
                live ? reinterpret_cast<HIZ_GLOBAL const uint8_t *>(wb + wq) : shared_line;
            const uint32_t cap = live ? 4u * min(12u, pwr4 - 4u - wq) : 48u;
            pre[S][0] = gload_u4(src);
#pragma unroll
            for (int k = 1; k < 4; k++)
                pre[S][k] = gload_u4(src + min(16u * k, cap));
        }
        pq[S] = wq;
        pend[S] = want;
        wq += want ? 16u : 0u;
    };
    // rounds, the same for every lane of the wave, until every lane has
    // stored its chunk; unrolled by kSets so that each set is a fixed group
    // of registers, with no exit between them (a lane past its chunk's end
    // decodes padding and stores nothing), so that the loop is entered from
    // one place only and each set's wait counts the later sets' loads
    static_assert(kSets == 3, "the loop below runs three sets");
#pragma nounroll
    while (__any(flushed < nsym)) {
        round(std::integral_constant<int, 0>{});
        round(std::integral_constant<int, 1>{});
        round(std::integral_constant<int, 2>{});
    }
    // bits taken by the chunk's codes
    const uint64_t used = tail ? (uint64_t)ub : 32ull * (rp - r0 - 1) - (uint64_t)nb;
    if (bad || (used + 31) / 32 != wc)
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    if (zeros)
        atomicAdd((unsigned long long *)&st->zeros_seen, (unsigned long long)zeros);
}

void launch_decode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, int cus, hipStream_t s)
{
    if (total == 0)
        return;
    // one workgroup of kDecSub lanes per compute unit while the sub-blocks
    // fit the device; past that, workgroups of two sub-blocks share one
    // table among twice the lanes (one workgroup per compute unit either
    // way, by their LDS)
    if (total <= (uint64_t)cus)
        hipLaunchKernelGGL(k_decode<kDecSub>, dim3((uint32_t)total), dim3(kDecSub), 0, s, d_jobs,
                           njobs, total, cnt);
    else
        hipLaunchKernelGGL(k_decode<2 * kDecSub>, dim3((uint32_t)(total / 2)), dim3(2 * kDecSub), 0,
                           s, d_jobs, njobs, total, cnt);
}

// Outliers go to their positions in the output before reconstruction reads
// them; indices must ascend and stay inside the field.
__global__ __launch_bounds__(256) void k_scatter(const Job *__restrict__ jobs, int njobs,
                                                 uint64_t total)
{
    for (uint64_t u = blockIdx.x * 256ull + threadIdx.x; u < total; u += 256ull * gridDim.x) {
        const Job &J = jobs[find_job<WK_OUT>(jobs, njobs, u)];
        const uint64_t i = u - J.out_begin;
        HIZ_GLOBAL const uint8_t *ip = gmem(J.stream) + J.off_oidx;
        uint64_t idx, prev = 0;
        if (J.idx_bytes == 4) {
            idx = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(ip)[i];
            if (i)
                prev = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(ip)[i - 1];
        } else {
            idx = reinterpret_cast<HIZ_GLOBAL const uint64_t *>(ip)[i];
            if (i)
                prev = reinterpret_cast<HIZ_GLOBAL const uint64_t *>(ip)[i - 1];
        }
        if (idx >= J.N || (i && prev >= idx)) {
            atomicOr(&J.st->flags, (uint32_t)ST_CORRUPT);
            continue;
        }
        gmem(J.out)[idx] = reinterpret_cast<HIZ_GLOBAL const float *>(gmem(J.stream) + J.off_oval)[i];
    }
}

void launch_scatter(const Job *d_jobs, int njobs, uint64_t total, hipStream_t s)
{
    if (total == 0)
        return;
    uint64_t g = cdiv(total, 256);
    if (g > 8192)
        g = 8192;
    hipLaunchKernelGGL(k_scatter, dim3((uint32_t)g), dim3(256), 0, s, d_jobs, njobs, total);
}

} // namespace hiz
