// Preparation kernels of compression: state reset, exact min/max of the field,
// the absolute error bound (Sec. 3.1 Eq. "general", Sec. 6.1.4) and the
// sampled-block tuner (Sec. 5.1.3).
#include "hiz_internal.h"

namespace hiz {

// ---------------------------------------------------------------------------
// Reset of per-field state and look-back flags (a fill kernel rather than
// hipMemsetAsync so that the sequence can be captured in a HIP graph).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_compress(const Job *__restrict__ jobs, int njobs,
                                                       Counters *cnt)
{
    const Job &J = jobs[blockIdx.y];
    FieldState *st = J.st;
    const uint32_t t = threadIdx.x;
    if (blockIdx.x == 0) {
        st->hist[t] = 0;
        if (t < kLevels * kCands)
            (&st->tune_err[0][0])[t] = 0;
        if (t == 0) {
            st->flags = 0u;
            st->n_out = 0;
            st->payload_words = 0;
            st->total_bytes = 0;
            st->zeros_seen = 0;
        }
        if (blockIdx.y == 0 && t < sizeof(Counters) / 4)
            reinterpret_cast<uint32_t *>(cnt)[t] = 0u;
    }
    for (uint64_t i = blockIdx.x * 256ull + t; i < J.n_groups; i += 256ull * gridDim.x) {
        J.lb_a[i] = 0;
        J.lb_b[i] = 0;
    }
    // look-back words of the last stages' chunks and of the outlier units
    for (uint64_t i = blockIdx.x * 256ull + t; i < J.n_lc; i += 256ull * gridDim.x)
        J.lb_c[i] = 0;
    const uint64_t nd = J.n_ou > J.n_lc ? J.n_ou : J.n_lc;
    for (uint64_t i = blockIdx.x * 256ull + t; i < nd; i += 256ull * gridDim.x)
        J.lb_d[i] = 0;
}

void launch_init_compress(const Job *d_jobs, int njobs, uint64_t max_chunks, Counters *cnt,
                          hipStream_t s)
{
    uint64_t gx = cdiv(max_chunks, 256);
    if (gx < 1)
        gx = 1;
    if (gx > 1024)
        gx = 1024;
    hipLaunchKernelGGL(k_init_compress, dim3((uint32_t)gx, njobs), dim3(256), 0, s, d_jobs, njobs,
                       cnt);
}

// ---------------------------------------------------------------------------
// Exact min/max (REL mode): ordered 32-bit keys reduced with atomics, so the
// result does not depend on the order of reduction; NaN/Inf raise a flag.
// ---------------------------------------------------------------------------

__device__ inline uint32_t wave_min_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__global__ __launch_bounds__(256) void k_minmax(const Job *__restrict__ jobs, int njobs,
                                                uint64_t total)
{
    __shared__ uint32_t red[8];
    const uint32_t t = threadIdx.x;
    for (uint64_t u = blockIdx.x; u < total; u += gridDim.x) {
        const Job &J = jobs[find_job<WK_MM>(jobs, njobs, u)];
        const uint64_t lu = u - J.mm_begin;
        const uint64_t lo = lu * kMmUnit;
        const uint64_t hi = min(lo + kMmUnit, J.N);
        HIZ_GLOBAL const float *f = gmem(J.field);
        uint32_t kmn = 0xffffffffu, kmx = 0u;
        bool bad = false;
        const bool vec = ((reinterpret_cast<uintptr_t>(f) & 15u) == 0) && (hi - lo == kMmUnit);
        if (vec) {
            // all 16 loads of a thread in flight before any is used: one
            // memory round trip per unit; streamed (the field is larger than
            // the caches, so nothing of it would be found there later)
            HIZ_GLOBAL const float *fb = f + lo;
            constexpr int K = (int)(kMmUnit / 4 / 256);
            float4 q4[K];
#pragma unroll
            for (int k = 0; k < K; k++)
                q4[k] = gload_f4_nt(fb + 4 * (k * 256 + t));
#pragma unroll
            for (int k = 0; k < K; k++) {
                const float4 q = q4[k];
                float e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    bad |= !isfinite(e[i]);
                    uint32_t key = fkey(e[i]);
                    kmn = min(kmn, key);
                    kmx = max(kmx, key);
                }
            }
        } else {
            for (uint64_t i = lo + t; i < hi; i += 256) {
                float e = f[i];
                bad |= !isfinite(e);
                uint32_t key = fkey(e);
                kmn = min(kmn, key);
                kmx = max(kmx, key);
            }
        }
        if (__any(bad) && (t & 63) == 0)
            atomicOr(&J.st->flags, (uint32_t)ST_NONFINITE);
        block_minmax(kmn, kmx, red);
        if (t == 0)
            gstore_u2(gmem(J.mm_part) + lu, make_uint2(kmn, kmx));
    }
}

void launch_minmax(const Job *d_jobs, int njobs, uint64_t total, int grid, hipStream_t s)
{
    if (total == 0)
        return;
    uint64_t g = total < (uint64_t)grid ? total : (uint64_t)grid;
    hipLaunchKernelGGL(k_minmax, dim3((uint32_t)g), dim3(256), 0, s, d_jobs, njobs, total);
}

// ---------------------------------------------------------------------------
// Error bound: eps = eb (ABS) or eb * (max - min) (REL), formed in FP64 and
// rounded down to FP32 so that it never exceeds the requested bound.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eps(const Job *__restrict__ jobs, int njobs)
{
    __shared__ uint32_t red[8];
    const Job &J = jobs[blockIdx.x];
    FieldState *st = J.st;
    double e = J.eb;
    if (J.mode == 1) {
        uint32_t kmn, kmx;
        reduce_partials(J.mm_part, J.n_mm, kmn, kmx, red);
        if (threadIdx.x != 0)
            return;
        st->kmin = kmn;
        st->kmax = kmx;
        if (st->flags & ST_NONFINITE)
            return;
        const float vmin = fkey_inv(kmn), vmax = fkey_inv(kmx);
        st->vmin = vmin;
        st->vmax = vmax;
        const double range = (double)vmax - (double)vmin;
        if (range == 0.0) {
            st->flags |= ST_CONST;
            return;
        }
        e = J.eb * range;
    } else if (threadIdx.x != 0) {
        return;
    }
    float f = (float)e;
    if ((double)f > e)
        f = nextafterf(f, 0.0f);
    st->eps = f;
    st->two_eb = f * 2.0f;
    st->inv = 1.0f / st->two_eb;
    st->tune_scale = f > 0.0f ? 65536.0 / (2.0 * (double)f) : 65536.0;
}

void launch_eps(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_eps, dim3(njobs), dim3(256), 0, s, d_jobs, njobs);
}

// ---------------------------------------------------------------------------
// Tuner (Sec. 5.1.3). Full 17^3 blocks with 0.2 % of the volume are sampled at
// even spacing. Every level is tested with the 21 candidates {LIN, CUB, NAT}
// x {MD, SEQ over the 6 dimension orders}, predicting from ORIGINAL values; the
// candidate with the smallest aggregated |x - p| wins per level (ties: lower
// index). Each |x - p| is counted in units of 2*eps/65536, rounded and capped
// at 2^36, and summed as a 64-bit integer, so the totals are exact and do not
// depend on the reduction order.
//
// Work balance follows the paper's idea of giving the expensive fine levels
// more thread blocks: per sample, one block tests strides 8 and 4, two
// blocks share stride 2 and six share stride 1. Unlike the paper, each block
// tests all 21 candidates on its share of targets, because the candidates
// reuse the same per-axis stencils.
// ---------------------------------------------------------------------------
constexpr int kTuneParts = 9;

__constant__ int8_t c_perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// 1-D spline stencil (Sec. 5.1.2): Lagrange weights at the midpoint from the
// samples at -3s, -s, +s, +3s; lower orders where samples are missing. With
// all four samples, spline 2 is the natural cubic spline through them (zero
// second derivative at the outer samples): weights (-3, 23, 23, -3) / 40.
__device__ __forceinline__ float stencil_1d(float a, float b, float c, float d, bool pa, bool pc,
                                            bool pd, int spline, int &rank)
{
    const bool cub = spline != 0;
    if (cub && pa && pc && pd) {
        rank = 4;
        if (spline == 2)
            return ((b + c) * 23.0f - (a + d) * 3.0f) / 40.0f;
        return ((b + c) * 9.0f - (a + d)) * 0.0625f;
    }
    if (cub && pc && pd) {
        rank = 3;
        return ((b * 3.0f + c * 6.0f) - d) * 0.125f;
    }
    if (cub && pa && pc) {
        rank = 3;
        return ((b * 6.0f + c * 3.0f) - a) * 0.125f;
    }
    if (pc) {
        rank = 2;
        return (b + c) * 0.5f;
    }
    if (pa) {
        rank = 1;
        return b * 1.5f - a * 0.5f;
    }
    rank = 0;
    return b;
}

// Mean of the predictions of maximal rank, combined in x, y, z order.
__device__ __forceinline__ float md_combine(const float p[3], const int r[3], int mask)
{
    int best = -1;
    for (int k = 0; k < 3; k++)
        if ((mask >> k) & 1)
            best = max(best, r[k]);
    bool u0 = (mask & 1) && r[0] == best, u1 = (mask & 2) && r[1] == best,
         u2 = (mask & 4) && r[2] == best;
    int m = (int)u0 + (int)u1 + (int)u2;
    float first = u0 ? p[0] : (u1 ? p[1] : p[2]);
    float second = u0 ? (u1 ? p[1] : p[2]) : p[2];
    if (m == 1)
        return first;
    if (m == 2)
        return (first + second) * 0.5f;
    return ((p[0] + p[1]) + p[2]) / 3.0f;
}

__device__ __forceinline__ uint64_t tune_term(float x, float p, double scale)
{
    float e = fabsf(x - p);
    double w = (double)e * scale;
    const double cap = 68719476736.0; // 2^36
    return (w < cap) ? (uint64_t)(w + 0.5) : (uint64_t)cap;
}

__device__ inline uint64_t wave_sum_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        lo = (uint32_t)__shfl_xor((int)lo, o, 64);
        hi = (uint32_t)__shfl_xor((int)hi, o, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Accumulate the 21 candidate error sums of the targets [g0, g1) of the
// stride-s grid of a block held in LDS (strides 17*17, 17, 1) whose extent on
// axis k is E[k] (17, or 1 on a flat axis).
__device__ void tune_level(const float *__restrict__ blk, const int E[3], int s, int g0, int g1,
                           double scale, uint64_t acc[kCands])
{
    const int Gx = E[0] == 1 ? 1 : 16 / s + 1, Gy = E[1] == 1 ? 1 : 16 / s + 1,
              Gz = E[2] == 1 ? 1 : 16 / s + 1;
    for (int g = g0 + (int)threadIdx.x; g < g1; g += blockDim.x) {
        int iz = g % Gz, r = g / Gz, iy = r % Gy, ix = r / Gy;
        int mask = (ix & 1) | ((iy & 1) << 1) | ((iz & 1) << 2);
        if (mask == 0)
            continue;
        int t[3] = {ix * s, iy * s, iz * s};
        const int st[3] = {kSide * kSide, kSide, 1};
        int li = (t[0] * kSide + t[1]) * kSide + t[2];
        float pl[3] = {0, 0, 0}, pc3[3] = {0, 0, 0}, pn[3] = {0, 0, 0};
        int rl[3] = {-1, -1, -1}, rc[3] = {-1, -1, -1}, rn[3] = {-1, -1, -1};
        for (int k = 0; k < 3; k++) {
            if (!((mask >> k) & 1))
                continue;
            int tk = t[k];
            bool pa = tk - 3 * s >= 0, pcp = tk + s <= E[k] - 1, pd = tk + 3 * s <= E[k] - 1;
            float b = blk[li - s * st[k]];
            float a = pa ? blk[li - 3 * s * st[k]] : 0.0f;
            float c = pcp ? blk[li + s * st[k]] : 0.0f;
            float d = pd ? blk[li + 3 * s * st[k]] : 0.0f;
            pl[k] = stencil_1d(a, b, c, d, pa, pcp, pd, 0, rl[k]);
            pc3[k] = stencil_1d(a, b, c, d, pa, pcp, pd, 1, rc[k]);
            pn[k] = stencil_1d(a, b, c, d, pa, pcp, pd, 2, rn[k]);
        }
        float x = blk[li];
        acc[0] += tune_term(x, md_combine(pl, rl, mask), scale);
        acc[7] += tune_term(x, md_combine(pc3, rc, mask), scale);
        acc[14] += tune_term(x, md_combine(pn, rn, mask), scale);
        for (int perm = 0; perm < 6; perm++) {
            int axis = -1;
            for (int j = 0; j < 3; j++)
                if ((mask >> c_perm[perm][j]) & 1)
                    axis = c_perm[perm][j];
            float vl = axis == 0 ? pl[0] : (axis == 1 ? pl[1] : pl[2]);
            float vc = axis == 0 ? pc3[0] : (axis == 1 ? pc3[1] : pc3[2]);
            float vn = axis == 0 ? pn[0] : (axis == 1 ? pn[1] : pn[2]);
            acc[1 + perm] += tune_term(x, vl, scale);
            acc[8 + perm] += tune_term(x, vc, scale);
            acc[15 + perm] += tune_term(x, vn, scale);
        }
    }
}

__device__ void tune_flush(FieldState *st, int level, uint64_t acc[kCands], uint64_t *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = 0; c < kCands; c++) {
        uint64_t v = wave_sum_u64(acc[c]);
        if (lane == 0)
            red[wave * kCands + c] = v;
        acc[c] = 0;
    }
    __syncthreads();
    if (threadIdx.x < kCands) {
        uint64_t v = 0;
        for (int w = 0; w < nw; w++)
            v += red[w * kCands + threadIdx.x];
        if (v)
            atomicAdd((unsigned long long *)&st->tune_err[level][threadIdx.x],
                      (unsigned long long)v);
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_tune(const Job *__restrict__ jobs, int njobs,
                                              uint64_t total)
{
    __shared__ float blk[kSide * kSide * kSide];
    __shared__ uint64_t red[4 * kCands];
    const uint64_t u = blockIdx.x;
    if (u >= total)
        return;
    const Job &J = jobs[find_job<WK_TUNE>(jobs, njobs, u)];
    FieldState *st = J.st;
    if (st->flags & (ST_CONST | ST_NONFINITE))
        return;
    const uint64_t lu = u - J.tune_begin;
    const uint64_t j = lu / kTuneParts;
    const int part = (int)(lu % kTuneParts);
    const uint64_t n_full = (uint64_t)J.n_full[0] * J.n_full[1] * J.n_full[2];
    const uint64_t idx = ((2 * j + 1) * n_full) / (2 * (uint64_t)J.n_samples);
    const uint64_t bc = idx % J.n_full[2], bb = (idx / J.n_full[2]) % J.n_full[1],
                   ba = idx / ((uint64_t)J.n_full[1] * J.n_full[2]);
    const uint64_t dy = J.dims[1], dz = J.dims[2];
    // a full block spans 17 points per axis, 1 on a flat axis (2-D / 1-D fields)
    const int E[3] = {J.dims[0] == 1 ? 1 : kSide, J.dims[1] == 1 ? 1 : kSide,
                      J.dims[2] == 1 ? 1 : kSide};
    for (int i = threadIdx.x; i < kSide * kSide * kSide; i += blockDim.x) {
        int z = i % kSide, r = i / kSide, y = r % kSide, x = r / kSide;
        if (x < E[0] && y < E[1] && z < E[2])
            blk[i] = gmem(J.field)[((ba * kAnchor + x) * dy + (bb * kAnchor + y)) * dz +
                                   bc * kAnchor + z];
    }
    __syncthreads();
    auto targets = [&](int s) {
        const int g = 16 / s + 1;
        return (E[0] == 1 ? 1 : g) * (E[1] == 1 ? 1 : g) * (E[2] == 1 ? 1 : g);
    };
    const double scale = st->tune_scale;
    uint64_t acc[kCands];
    for (int c = 0; c < kCands; c++)
        acc[c] = 0;
    if (part == 0) {
        tune_level(blk, E, 8, 0, targets(8), scale, acc);
        tune_flush(st, 0, acc, red);
        tune_level(blk, E, 4, 0, targets(4), scale, acc);
        tune_flush(st, 1, acc, red);
    } else if (part <= 2) {
        const int G3 = targets(2), h = part - 1;
        tune_level(blk, E, 2, h * G3 / 2, (h + 1) * G3 / 2, scale, acc);
        tune_flush(st, 2, acc, red);
    } else {
        const int G3 = targets(1), h = part - 3;
        tune_level(blk, E, 1, h * G3 / 6, (h + 1) * G3 / 6, scale, acc);
        tune_flush(st, 3, acc, red);
    }
}

void launch_tune(const Job *d_jobs, int njobs, uint64_t total, hipStream_t s)
{
    if (total == 0)
        return;
    hipLaunchKernelGGL(k_tune, dim3((uint32_t)total), dim3(256), 0, s, d_jobs, njobs, total);
}

// Per-level argmin (ties to the lower candidate), or the forced/default
// configuration when the tuner is off or no full block exists.
// One wave per field: each lane loads one candidate's error of every level at
// once, and a wave argmin picks the smallest error, the lower candidate on
// equal errors (the first in candidate order).
__global__ __launch_bounds__(64) void k_tune_pick(const Job *__restrict__ jobs, int njobs)
{
    static_assert(kCands <= 64, "one lane per candidate");
    const Job &J = jobs[blockIdx.x];
    FieldState *st = J.st;
    const int lane = threadIdx.x;
    const bool measured = J.tune && J.n_samples > 0;
    uint64_t err[kLevels];
#pragma unroll
    for (int l = 0; l < kLevels; l++)
        err[l] = measured && lane < kCands ? st->tune_err[l][lane] : ~0ull;
#pragma unroll
    for (int l = 0; l < kLevels; l++) {
        uint64_t e = err[l];
        int c = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t e2 = shfl64(e, lane ^ o);
            const int c2 = __shfl_xor(c, o, 64);
            if (e2 < e || (e2 == e && c2 < c)) {
                e = e2;
                c = c2;
            }
        }
        if (lane != 0)
            continue;
        uint8_t sp, sc, pm;
        if (measured) {
            const int r = c % 7;
            sp = (uint8_t)(c / 7);
            sc = (uint8_t)(r == 0 ? 0 : 1);
            pm = (uint8_t)(r == 0 ? 0 : r - 1);
        } else if (J.tune) {
            sp = 1;
            sc = 0;
            pm = 0;
        } else {
            sp = J.cfg_forced[l][0];
            sc = J.cfg_forced[l][1];
            pm = J.cfg_forced[l][2];
        }
        st->cfg[l][0] = sp;
        st->cfg[l][1] = sc;
        st->cfg[l][2] = pm;
    }
}

void launch_tune_pick(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_tune_pick, dim3(njobs), dim3(64), 0, s, d_jobs, njobs);
}

// ---------------------------------------------------------------------------
// Constant-field decompression: every element gets the stored value.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(float *out, uint64_t n, float v)
{
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += 256ull * gridDim.x)
        out[i] = v;
}

void launch_fill(float *out, uint64_t n, float v, hipStream_t s)
{
    uint64_t g = cdiv(n, 256);
    if (g > 4096)
        g = 4096;
    if (g < 1)
        g = 1;
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)g), dim3(256), 0, s, out, n, v);
}

// ---------------------------------------------------------------------------
// The first bytes of every job's state, packed for one device-to-host copy.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather_results(const Job *__restrict__ jobs, int njobs,
                                                        uint32_t *__restrict__ dst)
{
    constexpr int W = kResultBytes / 4;
    const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
    if (i >= (uint64_t)njobs * W)
        return;
    const int j = (int)(i / W), w = (int)(i % W);
    dst[i] = reinterpret_cast<const uint32_t *>(jobs[j].st)[w];
}

void launch_gather_results(const Job *d_jobs, int njobs, void *d_dst, hipStream_t s)
{
    const uint64_t n = (uint64_t)njobs * (kResultBytes / 4);
    hipLaunchKernelGGL(k_gather_results, dim3((uint32_t)cdiv(n, 256)), dim3(256), 0, s, d_jobs,
                       njobs, static_cast<uint32_t *>(d_dst));
}

} // namespace hiz
