// Lossless stage: Huffman coding of the one-byte quantization codes
// (Sec. 5.2.2-5.2.3) -- codebook on the device, chunk-parallel bit-packing with
// a single-pass decoupled look-back for chunk offsets and outlier positions,
// table-driven chunk-parallel decoding, and the outlier scatter of
// decompression.
#include "hiz_internal.h"

namespace hiz {

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

__device__ uint64_t lookback(uint64_t *arr, uint64_t idx, uint64_t agg)
{
    if (idx == 0) {
        lb_store(&arr[0], LB_INC | agg);
        return 0;
    }
    lb_store(&arr[idx], LB_AGG | agg);
    uint64_t excl = 0, j = idx - 1;
    for (;;) {
        const uint64_t w = lb_load(&arr[j]);
        const uint64_t f = w >> 62;
        if (f == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += w & LB_MASK;
        if (f == 2 || j == 0)
            break;
        j--;
    }
    lb_store(&arr[idx], LB_INC | (excl + agg));
    return excl;
}

__device__ inline uint64_t shfl64(uint64_t v, int src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
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
    put_le<uint32_t>(h + H_CHUNK, J.chunk);
    put_le<uint64_t>(h + H_NOUT, n_out);
    put_le<uint64_t>(h + H_TOTAL, total);
    put_le<uint64_t>(h + H_NCHUNKS, n_chunks);
    put_le<uint64_t>(h + H_NANCH, n_anchors);
}

__global__ __launch_bounds__(256) void k_codebook(const Job *__restrict__ jobs, int njobs)
{
    const Job &J = jobs[blockIdx.x];
    FieldState *st = J.st;
    __shared__ uint64_t cnt[256];
    __shared__ uint64_t w[512];
    __shared__ int16_t par[512];
    __shared__ uint8_t dep[512];
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
    const float vmin = fkey_inv(st->kmin), vmax = fkey_inv(st->kmax);
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

    cnt[t] = st->hist[t];
    for (;;) {
        __syncthreads();
        const uint64_t c = cnt[t];
        int rank = 0;
        if (c) {
            for (int j = 0; j < 256; j++) {
                const uint64_t cj = cnt[j];
                rank += (cj != 0) & ((cj < c) | ((cj == c) & (j < t)));
            }
        }
        const int n = __syncthreads_count(c != 0);
        if (c) {
            leafsym[rank] = (uint8_t)t;
            w[rank] = c;
        }
        len[t] = 0;
        __syncthreads();
        if (t == 0) {
            int maxlen = 0;
            if (n == 1) {
                len[leafsym[0]] = 1;
                maxlen = 1;
            } else if (n > 1) {
                int lq = 0, iq = n, next = n;
                for (int step = 0; step < n - 1; step++) {
                    int p0, p1;
                    if (lq < n && (iq >= next || w[lq] <= w[iq]))
                        p0 = lq++;
                    else
                        p0 = iq++;
                    if (lq < n && (iq >= next || w[lq] <= w[iq]))
                        p1 = lq++;
                    else
                        p1 = iq++;
                    w[next] = w[p0] + w[p1];
                    par[p0] = (int16_t)next;
                    par[p1] = (int16_t)next;
                    next++;
                }
                const int root = next - 1;
                dep[root] = 0;
                for (int v = root - 1; v >= 0; v--)
                    dep[v] = (uint8_t)(dep[par[v]] + 1);
                for (int i = 0; i < n; i++) {
                    len[leafsym[i]] = dep[i];
                    maxlen = max(maxlen, (int)dep[i]);
                }
            }
            s_maxlen = maxlen;
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
    const uint64_t end_chunks = kOffChunks + 4 * J.n_chunks;
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
        write_header(hdr, J, ib == 8 ? kFlagIdx64 : 0, st->eps, vmin, vmax, s_cfg, n_out,
                     J.n_chunks, J.n_anchors, 0);
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
// Encoder. One wave per chunk; chunks are taken in increasing order from an
// atomic counter. Each lane owns a contiguous run of the chunk's symbols; a
// wave scan of codeword lengths gives every lane its bit offset, lanes OR
// their bits into an LDS word buffer (shared boundary words with atomics),
// and the wave stores the packed words coalesced. The chunk's payload offset
// and its first outlier slot come from the look-back over preceding chunks,
// so codes are read once and every section is written in place.
// ---------------------------------------------------------------------------
constexpr int kEncSeg = 1024;            // symbols packed per pass
constexpr int kEncBuf = kEncSeg + 2;     // words of the LDS pack buffer
constexpr int kEncWaves = 4;

__device__ inline void load_lane_codes(const uint8_t *__restrict__ src, int P, int n,
                                       uint32_t r[4])
{
    // P consecutive codes (P <= 16) starting at src; n = how many are valid
    r[0] = r[1] = r[2] = r[3] = 0;
    if (n == P && (P & 3) == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (k < P / 4)
                r[k] = reinterpret_cast<const uint32_t *>(src)[k];
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

__global__ __launch_bounds__(256) void k_encode(const Job *__restrict__ jobs, int njobs,
                                                uint64_t total, Counters *cnt)
{
    __shared__ uint32_t s_code[kEncWaves][256];
    __shared__ uint8_t s_len[kEncWaves][256];
    __shared__ uint32_t s_buf[kEncWaves][kEncBuf];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *code = s_code[wv];
    uint8_t *len = s_len[wv];
    uint32_t *buf = s_buf[wv];
    for (int k = lane; k < kEncBuf; k += 64)
        buf[k] = 0;
    int cur = -1;
    for (;;) {
        uint32_t id = 0;
        if (lane == 0)
            id = atomicAdd(&cnt->enc_next, 1u);
        id = (uint32_t)__shfl((int)id, 0, 64);
        if (id >= total)
            break;
        const int ji = find_job<WK_CHUNK>(jobs, njobs, id);
        const Job &J = jobs[ji];
        FieldState *st = J.st;
        if (st->flags & (ST_CONST | ST_NONFINITE))
            continue;
        if (ji != cur) {
            for (int k = lane; k < 256; k += 64) {
                code[k] = st->cb_code[k];
                len[k] = st->cb_len[k];
            }
            cur = ji;
            wave_sync_lds();
        }
        const uint64_t ck = id - J.chunk_begin;
        const uint64_t c0 = ck << J.log2_chunk;
        const uint64_t c1 = min(c0 + J.chunk, J.N);
        const int clen = (int)(c1 - c0);
        const int nseg = (clen + kEncSeg - 1) / kEncSeg;
        const uint8_t *src = J.codes + c0;

        // pass 1: chunk totals (bits, outliers)
        uint32_t r[4];
        uint64_t lbits = 0;
        uint32_t lzero = 0;
        for (int sg = 0; sg < nseg; sg++) {
            const int sl = min(kEncSeg, clen - sg * kEncSeg);
            const int P = (sl + 63) / 64;
            const int n = max(0, min(P, sl - lane * P));
            load_lane_codes(src + sg * kEncSeg + lane * P, P, n, r);
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k < n) {
                    const uint32_t c = code_at(r, k);
                    lbits += len[c];
                    lzero += (c == 0);
                }
            }
        }
        uint64_t tbits = lbits;
        uint32_t tzero = lzero;
        for (int o = 32; o > 0; o >>= 1) {
            tbits += shfl64(tbits, lane ^ o);
            tzero += (uint32_t)__shfl_xor((int)tzero, o, 64);
        }
        const uint64_t twords = (tbits + 31) >> 5;
        uint64_t excl = 0;
        if (lane < 2)
            excl = lookback(lane == 0 ? J.lb_a : J.lb_b, ck, lane == 0 ? twords : (uint64_t)tzero);
        const uint64_t wbase = shfl64(excl, 0);
        const uint64_t obase = shfl64(excl, 1);

        const uint64_t cap = J.cap;
        uint32_t *payload = reinterpret_cast<uint32_t *>(J.stream + st->off_payload);
        const uint64_t pay_words_cap =
            cap > st->off_payload ? (cap - st->off_payload) / 4 : 0;
        const uint64_t o_idx = st->off_oidx, o_val = st->off_oval;
        const int ib = J.idx_bytes;

        // pass 2: pack segment by segment
        uint64_t sb = 0;      // chunk-relative bit at the segment start
        uint64_t zrun = 0;    // outliers before the segment
        for (int sg = 0; sg < nseg; sg++) {
            const int sl = min(kEncSeg, clen - sg * kEncSeg);
            const int P = (sl + 63) / 64;
            const int n = max(0, min(P, sl - lane * P));
            const uint64_t gfirst = c0 + (uint64_t)sg * kEncSeg + (uint64_t)lane * P;
            load_lane_codes(src + sg * kEncSeg + lane * P, P, n, r);
            uint32_t mb = 0, mz = 0;
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k < n) {
                    const uint32_t c = code_at(r, k);
                    mb += len[c];
                    mz += (c == 0);
                }
            }
            const uint32_t ib_incl = wave_incl_scan(mb);
            const uint32_t iz_incl = wave_incl_scan(mz);
            const uint32_t seg_bits = (uint32_t)__shfl((int)ib_incl, 63, 64);
            const uint32_t seg_zero = (uint32_t)__shfl((int)iz_incl, 63, 64);
            const uint64_t wb = sb >> 5;
            // bit offset of this lane relative to word wb
            uint32_t orel = (uint32_t)(sb & 31) + (ib_incl - mb);
            uint32_t cw = orel >> 5, sh = orel & 31, curw = 0;
            uint64_t zpos = obase + zrun + (iz_incl - mz);
            for (int k = 0; k < n; k++) {
                const uint32_t c = code_at(r, k);
                const uint32_t L = len[c], cd = code[c];
                if (sh + L < 32) {
                    curw |= cd << (32 - sh - L);
                    sh += L;
                } else if (sh + L == 32) {
                    curw |= cd;
                    atomicOr(&buf[cw], curw);
                    cw++;
                    curw = 0;
                    sh = 0;
                } else {
                    const uint32_t rr = sh + L - 32;
                    curw |= cd >> rr;
                    atomicOr(&buf[cw], curw);
                    cw++;
                    curw = cd << (32 - rr);
                    sh = rr;
                }
                if (c == 0) {
                    const uint64_t gi = gfirst + k;
                    if (o_idx + (zpos + 1) * ib <= cap) {
                        if (ib == 4)
                            reinterpret_cast<uint32_t *>(J.stream + o_idx)[zpos] = (uint32_t)gi;
                        else
                            reinterpret_cast<uint64_t *>(J.stream + o_idx)[zpos] = gi;
                    }
                    if (o_val + (zpos + 1) * 4 <= cap)
                        reinterpret_cast<float *>(J.stream + o_val)[zpos] = J.field[gi];
                    zpos++;
                }
            }
            if (sh > 0)
                atomicOr(&buf[cw], curw);
            wave_sync_lds();
            const uint64_t se = sb + seg_bits;
            const uint32_t nfull = (uint32_t)((se >> 5) - wb);
            for (uint32_t k = lane; k < nfull; k += 64) {
                const uint64_t gw = wbase + wb + k;
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
            zrun += seg_zero;
        }
        // last partial word of the chunk
        if (lane == 0) {
            if (sb & 31) {
                const uint64_t gw = wbase + (sb >> 5);
                if (gw < pay_words_cap)
                    payload[gw] = buf[0];
            }
            buf[0] = 0;
            if (kOffChunks + 4 * (ck + 1) <= cap)
                reinterpret_cast<uint32_t *>(J.stream + kOffChunks)[ck] = (uint32_t)twords;
            if (ck == J.n_chunks - 1) {
                const uint64_t pw = wbase + twords;
                const uint64_t total_bytes = st->off_payload + 4 * pw;
                st->payload_words = pw;
                st->total_bytes = total_bytes;
                if (H_TOTAL + 8 <= cap) {
                    *reinterpret_cast<uint64_t *>(J.stream + H_PWORDS) = pw;
                    *reinterpret_cast<uint64_t *>(J.stream + H_TOTAL) = total_bytes;
                }
                if (total_bytes > cap)
                    atomicOr(&st->flags, (uint32_t)ST_OVERFLOW);
                if (obase + tzero != st->n_out)
                    atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
            }
        }
        wave_sync_lds();
    }
}

void launch_encode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, int grid,
                   hipStream_t s)
{
    if (total == 0)
        return;
    uint64_t need = cdiv(total, kEncWaves);
    uint64_t g = need < (uint64_t)grid ? need : (uint64_t)grid;
    hipLaunchKernelGGL(k_encode, dim3((uint32_t)g), dim3(64 * kEncWaves), 0, s, d_jobs, njobs,
                       total, cnt);
}

int encode_blocks_per_cu()
{
    int n = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_encode, 64 * kEncWaves, 0);
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
// lookup table for codes up to kLutBits bits and per-length ranges for the
// longer ones.
__global__ __launch_bounds__(256) void k_dec_tables(const Job *__restrict__ jobs, int njobs)
{
    const Job &J = jobs[blockIdx.x];
    DecTables *dt = J.dt;
    __shared__ uint8_t len[256];
    __shared__ uint32_t blc[kMaxCodeLen + 2];
    __shared__ uint32_t first[kMaxCodeLen + 2];
    __shared__ uint32_t index[kMaxCodeLen + 2];
    const int t = threadIdx.x;
    len[t] = J.stream[kOffLen + t];
    if (t < kMaxCodeLen + 2)
        blc[t] = 0;
    for (int i = t; i < (1 << kLutBits); i += 256)
        dt->lut[i] = 0;
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
        dt->maxlen = maxlen;
    }
    __syncthreads();
    if (t <= kMaxCodeLen) {
        dt->first[t] = first[t];
        dt->count[t] = blc[t];
        dt->index[t] = index[t];
    }
    if (L >= 1 && L <= kMaxCodeLen) {
        uint32_t k = 0;
        for (int j = 0; j < t; j++)
            k += (len[j] == L);
        const uint32_t code = first[L] + k;
        dt->sorted[index[L] + k] = (uint8_t)t;
        if (L <= kLutBits) {
            const uint32_t lo = code << (kLutBits - L), hi = (code + 1) << (kLutBits - L);
            for (uint32_t e = lo; e < hi && e < (1u << kLutBits); e++)
                dt->lut[e] = (uint16_t)((L << 8) | t);
        }
    }
}

void launch_dec_tables(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_tables, dim3(njobs), dim3(256), 0, s, d_jobs, njobs);
}

// One thread per chunk; a workgroup takes 256 consecutive chunks, finds its
// payload offset by look-back over the stored word counts, and each thread
// decodes its chunk sequentially with the LDS lookup table.
constexpr int kDecChunks = 256;

__global__ __launch_bounds__(256) void k_decode(const Job *__restrict__ jobs, int njobs,
                                                uint64_t total, Counters *cnt)
{
    __shared__ uint16_t lut[1 << kLutBits];
    __shared__ uint32_t first[kMaxCodeLen + 2], count[kMaxCodeLen + 2], index[kMaxCodeLen + 2];
    __shared__ uint8_t sorted[256];
    __shared__ uint32_t s_id, s_maxlen;
    __shared__ uint64_t s_wsum[4];
    __shared__ uint64_t s_base;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0)
        s_id = atomicAdd(&cnt->dec_next, 1u);
    __syncthreads();
    const uint64_t id = s_id;
    if (id >= total)
        return;
    const Job &J = jobs[find_job<WK_DBLK>(jobs, njobs, id)];
    const DecTables *dt = J.dt;
    for (int i = t; i < (1 << kLutBits); i += 256)
        lut[i] = dt->lut[i];
    if (t <= kMaxCodeLen) {
        first[t] = dt->first[t];
        count[t] = dt->count[t];
        index[t] = dt->index[t];
    }
    sorted[t] = dt->sorted[t];
    if (t == 0)
        s_maxlen = dt->maxlen;
    const uint64_t lb = id - J.dblk_begin;
    const uint64_t chunk = lb * kDecChunks + t;
    const uint32_t *counts = reinterpret_cast<const uint32_t *>(J.stream + kOffChunks);
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
    for (int k = 0; k < 4; k++) {
        before += (k < wv) ? s_wsum[k] : 0;
        blk_total += s_wsum[k];
    }
    if (t == 0)
        s_base = lookback(J.lb_a, lb, blk_total);
    __syncthreads();
    if (chunk >= J.n_chunks)
        return;
    FieldState *st = J.st;
    const uint64_t start = s_base + before + incl - wc;
    const uint64_t pw = J.payload_words;
    if (start + wc > pw) {
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
        return;
    }
    if (chunk == J.n_chunks - 1 && start + wc != pw)
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    const uint32_t *words = reinterpret_cast<const uint32_t *>(J.stream + J.off_payload);
    const uint64_t i0 = chunk << J.log2_chunk, i1 = min(i0 + J.chunk, J.N);
    const uint32_t maxlen = s_maxlen;
    uint64_t wpos = start;
    const uint64_t wend = start + wc;
    uint64_t buf = 0;
    int nb = 0;
    uint64_t used = 0;
    uint32_t pack = 0, zeros = 0;
    bool bad = false;
    uint64_t i = i0;
    for (; i < i1; i++) {
        if (nb < 32) {
            const uint32_t wd = wpos < wend ? words[wpos] : 0u;
            wpos++;
            buf |= (uint64_t)wd << (32 - nb);
            nb += 32;
        }
        const uint32_t e = lut[buf >> (64 - kLutBits)];
        uint32_t L, sym;
        if (e) {
            L = e >> 8;
            sym = e & 255u;
        } else {
            sym = 0;
            for (L = kLutBits + 1; L <= maxlen; L++) {
                const uint32_t c = (uint32_t)(buf >> (64 - L));
                if (c - first[L] < count[L]) {
                    sym = sorted[index[L] + (c - first[L])];
                    break;
                }
            }
            if (L > maxlen) {
                bad = true;
                break;
            }
        }
        buf <<= L;
        nb -= (int)L;
        used += L;
        zeros += (sym == 0);
        pack |= sym << (8 * (i & 3));
        if ((i & 3) == 3) {
            *reinterpret_cast<uint32_t *>(J.codes + i - 3) = pack;
            pack = 0;
        }
    }
    if (!bad && (i1 & 3)) {
        for (uint64_t k = i1 & ~uint64_t(3); k < i1; k++)
            J.codes[k] = (uint8_t)(pack >> (8 * (k & 3)));
    }
    if (bad || (used + 31) / 32 != wc)
        atomicOr(&st->flags, (uint32_t)ST_CORRUPT);
    if (zeros)
        atomicAdd((unsigned long long *)&st->zeros_seen, (unsigned long long)zeros);
}

void launch_decode(const Job *d_jobs, int njobs, uint64_t total, Counters *cnt, hipStream_t s)
{
    if (total == 0)
        return;
    hipLaunchKernelGGL(k_decode, dim3((uint32_t)total), dim3(kDecChunks), 0, s, d_jobs, njobs,
                       total, cnt);
}

// Outliers go to their positions in the output before reconstruction reads
// them; indices must ascend and stay inside the field.
__global__ __launch_bounds__(256) void k_scatter(const Job *__restrict__ jobs, int njobs,
                                                 uint64_t total)
{
    for (uint64_t u = blockIdx.x * 256ull + threadIdx.x; u < total; u += 256ull * gridDim.x) {
        const Job &J = jobs[find_job<WK_OUT>(jobs, njobs, u)];
        const uint64_t i = u - J.out_begin;
        const uint8_t *ip = J.stream + J.off_oidx;
        uint64_t idx, prev = 0;
        if (J.idx_bytes == 4) {
            idx = reinterpret_cast<const uint32_t *>(ip)[i];
            if (i)
                prev = reinterpret_cast<const uint32_t *>(ip)[i - 1];
        } else {
            idx = reinterpret_cast<const uint64_t *>(ip)[i];
            if (i)
                prev = reinterpret_cast<const uint64_t *>(ip)[i - 1];
        }
        if (idx >= J.N || (i && prev >= idx)) {
            atomicOr(&J.st->flags, (uint32_t)ST_CORRUPT);
            continue;
        }
        J.out[idx] = reinterpret_cast<const float *>(J.stream + J.off_oval)[i];
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
