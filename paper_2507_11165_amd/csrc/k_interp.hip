// Level-wise spline interpolation over 17^3 blocks (Sec. 5.1.1-5.1.2), fused
// with linear-scaling quantization and the code histogram (compression) or
// with reconstruction from codes (decompression).
//
// GPU design. A workgroup owns a tile of TZ consecutive blocks along z
// (1 x 1 x TZ blocks, 17 x 17 x (16*TZ+1) points with the shared +1 faces).
// The tile's values live in LDS for the whole level walk; every target of a
// sub-step is independent of the others in that sub-step, so the workgroup
// sweeps a sub-step in parallel and synchronizes between sub-steps. Targets on
// the face shared by two blocks of a tile are computed once: their stencils
// never leave the face, so they equal what each block would compute alone,
// and z-stencils stop at the block's own faces exactly as in a lone block.
// Workgroups are persistent: each walks a contiguous run of tiles handed to
// its XCD (blockIdx % 8), so neighbouring tiles that share halo faces are read
// through the same L2. The code histogram is kept in LDS across all tiles of a
// workgroup and flushed once.
#include "hiz_internal.h"

namespace hiz {

__constant__ int8_t c_perm_i[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                      {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

template <int TZ> struct TileShape {
    static constexpr int EZ = 16 * TZ + 1;   // points along z incl. the far face
    static constexpr int PZ = EZ;            // LDS pitch of a z row (odd: spreads banks)
    static constexpr int PX = kSide * PZ;    // LDS stride of x
    static constexpr int NV = kSide * PX;    // values in the tile
    static constexpr int OZ = 16 * TZ;       // owned points along z (full tile)
    static constexpr int NC = 16 * 16 * OZ;  // owned codes
    static constexpr int NROW = kSide * kSide;
};

struct Geo {
    int ex, ey, ez;       // tile extents (<= 17, 17, 16*TZ+1)
    int ownx, owny, ownz; // owned extents
};

struct QParams {
    float eps, two_eb, inv;
};

// 1-D spline stencil (Sec. 5.1.2) along a line of LDS stride `st` at index li.
__device__ __forceinline__ float stencil_lds(const float *__restrict__ v, int li, int st, int s,
                                             bool pa, bool pc, bool pd, bool cub, int &rank)
{
    const float b = v[li - s * st];
    if (cub && pa && pc && pd) {
        const float a = v[li - 3 * s * st], c = v[li + s * st], d = v[li + 3 * s * st];
        rank = 4;
        return ((b + c) * 9.0f - (a + d)) * 0.0625f;
    }
    if (cub && pc && pd) {
        const float c = v[li + s * st], d = v[li + 3 * s * st];
        rank = 3;
        return ((b * 3.0f + c * 6.0f) - d) * 0.125f;
    }
    if (cub && pa && pc) {
        const float a = v[li - 3 * s * st], c = v[li + s * st];
        rank = 3;
        return ((b * 6.0f + c * 3.0f) - a) * 0.125f;
    }
    if (pc) {
        const float c = v[li + s * st];
        rank = 2;
        return (b + c) * 0.5f;
    }
    if (pa) {
        const float a = v[li - 3 * s * st];
        rank = 1;
        return b * 1.5f - a * 0.5f;
    }
    rank = 0;
    return b;
}

// Prediction of target (x,y,z) at stride S with odd-axis mask M.
// axis < 0: multi-dimensional scheme (mean of the highest-order predictions
// along the axes of M, in x, y, z order); otherwise 1-D along `axis`.
template <int TZ, int S, int M>
__device__ __forceinline__ float predict(const float *__restrict__ v, int li, int x, int y, int z,
                                         const Geo &g, int axis, bool cub)
{
    using TS = TileShape<TZ>;
    float px = 0.f, py = 0.f, pz = 0.f;
    int rx = -1, ry = -1, rz = -1;
    const bool want_x = (M & 1) && (axis < 0 || axis == 0);
    const bool want_y = (M & 2) && (axis < 0 || axis == 1);
    const bool want_z = (M & 4) && (axis < 0 || axis == 2);
    if (want_x)
        px = stencil_lds(v, li, TS::PX, S, x >= 3 * S, x + S < g.ex, x + 3 * S < g.ex, cub, rx);
    if (want_y)
        py = stencil_lds(v, li, TS::PZ, S, y >= 3 * S, y + S < g.ey, y + 3 * S < g.ey, cub, ry);
    if (want_z) {
        // z stencils stop at the faces of the target's own block
        const int hi = min((z & ~15) + 16, g.ez - 1);
        pz = stencil_lds(v, li, 1, S, (z & 15) >= 3 * S, z + S <= hi, z + 3 * S <= hi, cub, rz);
    }
    if (axis >= 0)
        return axis == 0 ? px : (axis == 1 ? py : pz);
    if (M == 1)
        return px;
    if (M == 2)
        return py;
    if (M == 4)
        return pz;
    const int best = max(rx, max(ry, rz));
    const bool ux = (M & 1) && rx == best, uy = (M & 2) && ry == best,
               uz = (M & 4) && rz == best;
    const int m = (int)ux + (int)uy + (int)uz;
    const float first = ux ? px : (uy ? py : pz);
    const float second = ux ? (uy ? py : pz) : pz;
    if (m == 1)
        return first;
    if (m == 2)
        return (first + second) * 0.5f;
    return ((px + py) + pz) / 3.0f;
}

// Linear-scaling quantization (code = 128 + q, |q| <= 127; else outlier code 0
// with the exact value kept). The FP64 check guarantees |x - x'| <= eps after
// FP32 rounding of the reconstruction.
__device__ __forceinline__ uint8_t quantize(float xv, float p, const QParams &q, float &xo)
{
    const float diff = xv - p;
    const float qf = diff * q.inv;
    const float qr = rintf(qf);
    uint8_t code = 0;
    xo = xv;
    if (fabsf(qr) <= 127.0f) {
        const int qi = (int)qr;
        const float xr = p + ((float)qi * q.two_eb);
        if (fabs((double)xv - (double)xr) <= (double)q.eps) {
            code = (uint8_t)(qi + 128);
            xo = xr;
        }
    }
    return code;
}

// One pattern of a sub-step: targets whose odd-axis mask is M at stride S.
template <int TZ, int S, int M, bool COMP>
__device__ __forceinline__ void pattern(float *__restrict__ v, uint8_t *__restrict__ cb,
                                        const uint8_t *__restrict__ cl, const Geo &g, int axis,
                                        bool cub, const QParams &q)
{
    using TS = TileShape<TZ>;
    constexpr int CX = (M & 1) ? 8 / S : 8 / S + 1;
    constexpr int CY = (M & 2) ? 8 / S : 8 / S + 1;
    constexpr int CZ = (M & 4) ? 8 * TZ / S : 8 * TZ / S + 1;
    constexpr int TOT = CX * CY * CZ;
    for (int i = threadIdx.x; i < TOT; i += blockDim.x) {
        const int iz = i % CZ, r = i / CZ, iy = r % CY, ix = r / CY;
        const int x = ((M & 1) ? 2 * ix + 1 : 2 * ix) * S;
        const int y = ((M & 2) ? 2 * iy + 1 : 2 * iy) * S;
        const int z = ((M & 4) ? 2 * iz + 1 : 2 * iz) * S;
        if (x >= g.ex || y >= g.ey || z >= g.ez)
            continue;
        const int li = x * TS::PX + y * TS::PZ + z;
        const float p = predict<TZ, S, M>(v, li, x, y, z, g, axis, cub);
        if (COMP) {
            float xo;
            const uint8_t code = quantize(v[li], p, q, xo);
            v[li] = xo;
            if (x < g.ownx && y < g.owny && z < g.ownz)
                cb[(x * 16 + y) * TS::OZ + z] = code;
        } else {
            const uint8_t c = cl[li];
            if (c != 0)
                v[li] = p + ((float)((int)c - 128) * q.two_eb);
        }
    }
}

template <int TZ, int S, bool COMP>
__device__ __forceinline__ void dispatch(int M, float *v, uint8_t *cb, const uint8_t *cl,
                                         const Geo &g, int axis, bool cub, const QParams &q)
{
    switch (M) {
    case 1: pattern<TZ, S, 1, COMP>(v, cb, cl, g, axis, cub, q); break;
    case 2: pattern<TZ, S, 2, COMP>(v, cb, cl, g, axis, cub, q); break;
    case 3: pattern<TZ, S, 3, COMP>(v, cb, cl, g, axis, cub, q); break;
    case 4: pattern<TZ, S, 4, COMP>(v, cb, cl, g, axis, cub, q); break;
    case 5: pattern<TZ, S, 5, COMP>(v, cb, cl, g, axis, cub, q); break;
    case 6: pattern<TZ, S, 6, COMP>(v, cb, cl, g, axis, cub, q); break;
    default: pattern<TZ, S, 7, COMP>(v, cb, cl, g, axis, cub, q); break;
    }
}

// One level (stride S) in three sub-steps. MD: 1-D, then 2-D, then 3-D
// targets. SEQ(order): pass j handles the targets whose last odd axis in the
// order is the j-th, interpolating along that axis.
template <int TZ, int S, bool COMP>
__device__ void level(float *v, uint8_t *cb, const uint8_t *cl, const Geo &g, const uint8_t *cfg,
                      const QParams &q)
{
    const bool cub = cfg[0] != 0;
    const bool md = cfg[1] == 0;
    const int perm = cfg[2];
    for (int sub = 1; sub <= 3; sub++) {
        for (int M = 1; M <= 7; M++) {
            int axis = -1;
            if (md) {
                if (__popc(M) != sub)
                    continue;
            } else {
                int last = -1;
                for (int j = 0; j < 3; j++)
                    if ((M >> c_perm_i[perm][j]) & 1)
                        last = j;
                if (last != sub - 1)
                    continue;
                axis = c_perm_i[perm][sub - 1];
            }
            dispatch<TZ, S, COMP>(M, v, cb, cl, g, axis, cub, q);
        }
        __syncthreads();
    }
}

template <int TZ, bool COMP>
__device__ void walk_levels(float *v, uint8_t *cb, const uint8_t *cl, const Geo &g,
                            const uint8_t (*cfg)[3], const QParams &q)
{
    level<TZ, 8, COMP>(v, cb, cl, g, cfg[0], q);
    level<TZ, 4, COMP>(v, cb, cl, g, cfg[1], q);
    level<TZ, 2, COMP>(v, cb, cl, g, cfg[2], q);
    level<TZ, 1, COMP>(v, cb, cl, g, cfg[3], q);
}

// Tile u of job J -> geometry and global row offsets (into LDS `rowoff`).
template <int TZ>
__device__ __forceinline__ Geo tile_geometry(const Job &J, uint64_t lt, uint64_t &ox, uint64_t &oy,
                                             uint64_t &oz, uint32_t &bx, uint32_t &by,
                                             uint32_t &bz0)
{
    const uint64_t tz = lt % J.ntz, r = lt / J.ntz;
    by = (uint32_t)(r % J.nb[1]);
    bx = (uint32_t)(r / J.nb[1]);
    bz0 = (uint32_t)(tz * TZ);
    ox = (uint64_t)bx * kAnchor;
    oy = (uint64_t)by * kAnchor;
    oz = (uint64_t)bz0 * kAnchor;
    Geo g;
    g.ex = (int)min<uint64_t>(kSide, J.dims[0] - ox);
    g.ey = (int)min<uint64_t>(kSide, J.dims[1] - oy);
    g.ez = (int)min<uint64_t>(16 * TZ + 1, J.dims[2] - oz);
    g.ownx = min(g.ex, 16);
    g.owny = min(g.ey, 16);
    g.ownz = (int)min<uint64_t>(16 * TZ, J.dims[2] - oz);
    return g;
}

__device__ __forceinline__ void xcd_range(uint64_t total, uint64_t &first, uint64_t &end,
                                          uint64_t &step)
{
    const uint32_t G = gridDim.x, b = blockIdx.x;
    if (G >= 8 && (G & 7) == 0) {
        const uint32_t xcd = b & 7, l = b >> 3;
        const uint64_t lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
        first = lo + l;
        end = hi;
        step = G >> 3;
    } else {
        first = b;
        end = total;
        step = G;
    }
}

// ---------------------------------------------------------------------------
// Compression: predict + quantize + histogram, persistent over tiles.
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(256) void k_predict(const Job *__restrict__ jobs, int njobs,
                                                 uint64_t total)
{
    using TS = TileShape<TZ>;
    __shared__ float v[TS::NV];
    __shared__ __align__(16) uint8_t cb[TS::NC];
    __shared__ uint64_t rowoff[TS::NROW];
    __shared__ uint32_t hist[256];
    __shared__ uint8_t cfg[kLevels][3];
    __shared__ QParams qp;
    __shared__ uint32_t skip;

    const int t = threadIdx.x;
    hist[t] = 0;
    int cur = -1;
    uint64_t first, end, step;
    xcd_range(total, first, end, step);
    for (uint64_t u = first; u < end; u += step) {
        const int ji = find_job<WK_TILE>(jobs, njobs, u);
        const Job &J = jobs[ji];
        if (ji != cur) {
            __syncthreads();
            if (cur >= 0) {
                const uint32_t h = hist[t];
                if (h)
                    atomicAdd((unsigned long long *)&jobs[cur].st->hist[t], (unsigned long long)h);
            }
            hist[t] = 0;
            if (t == 0) {
                const FieldState *st = J.st;
                skip = st->flags & (ST_CONST | ST_NONFINITE);
                qp.eps = st->eps;
                qp.two_eb = st->two_eb;
                qp.inv = st->inv;
            }
            if (t < kLevels * 3)
                cfg[t / 3][t % 3] = J.st->cfg[t / 3][t % 3];
            cur = ji;
            __syncthreads();
        }
        if (skip)
            continue;
        uint64_t ox, oy, oz;
        uint32_t bx, by, bz0;
        const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
        const uint64_t dy = J.dims[1], dz = J.dims[2];
        for (int r = t; r < TS::NROW; r += blockDim.x) {
            const int x = r / kSide, y = r % kSide;
            rowoff[r] = ((ox + x) * dy + (oy + y)) * dz + oz;
        }
        __syncthreads();
        // load the tile (with its +1 faces) into LDS
        const bool abs_mode = J.mode == 0;
        uint32_t kmn = 0xffffffffu, kmx = 0u;
        bool bad = false;
        for (int i = t; i < TS::NROW * TS::EZ; i += blockDim.x) {
            const int z = i % TS::EZ, r = i / TS::EZ;
            const int y = r % kSide, x = r / kSide;
            if (x < g.ex && y < g.ey && z < g.ez) {
                const float val = J.field[rowoff[r] + z];
                v[x * TS::PX + y * TS::PZ + z] = val;
                if (abs_mode) {
                    bad |= !isfinite(val);
                    const uint32_t k = fkey(val);
                    kmn = min(kmn, k);
                    kmx = max(kmx, k);
                }
            }
        }
        if (abs_mode) {
            for (int o = 32; o > 0; o >>= 1) {
                kmn = min(kmn, (uint32_t)__shfl_xor((int)kmn, o, 64));
                kmx = max(kmx, (uint32_t)__shfl_xor((int)kmx, o, 64));
            }
            const int anybad = __any(bad);
            if ((t & 63) == 0) {
                atomicMin(&J.st->kmin, kmn);
                atomicMax(&J.st->kmax, kmx);
                if (anybad)
                    atomicOr(&J.st->flags, (uint32_t)ST_NONFINITE);
            }
        }
        // anchors owned by this tile: local (0, 0, 16j)
        if (t < TZ && 16 * t < g.ownz) {
            cb[t * 16] = 128;
            const uint64_t ai = ((uint64_t)bx * J.nb[1] + by) * J.nb[2] + bz0 + t;
            const uint64_t off = J.off_anchors + 4 * ai;
            if (off + 4 <= J.cap)
                *reinterpret_cast<float *>(J.stream + off) = J.field[rowoff[0] + 16 * t];
        }
        __syncthreads();
        walk_levels<TZ, true>(v, cb, nullptr, g, cfg, qp);
        // codes of owned points -> global, histogram in LDS
        if (g.ownz == TS::OZ && (dz & 3) == 0) {
            for (int i = t; i < 16 * 16 * TS::OZ / 4; i += blockDim.x) {
                const int w = i % (TS::OZ / 4), r = i / (TS::OZ / 4);
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny) {
                    const uint32_t c4 = *reinterpret_cast<const uint32_t *>(&cb[r * TS::OZ + 4 * w]);
                    *reinterpret_cast<uint32_t *>(J.codes + rowoff[x * kSide + y] + 4 * w) = c4;
                    atomicAdd(&hist[c4 & 255], 1u);
                    atomicAdd(&hist[(c4 >> 8) & 255], 1u);
                    atomicAdd(&hist[(c4 >> 16) & 255], 1u);
                    atomicAdd(&hist[c4 >> 24], 1u);
                }
            }
        } else {
            for (int i = t; i < 16 * 16 * TS::OZ; i += blockDim.x) {
                const int z = i % TS::OZ, r = i / TS::OZ;
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny && z < g.ownz) {
                    const uint8_t c = cb[r * TS::OZ + z];
                    J.codes[rowoff[x * kSide + y] + z] = c;
                    atomicAdd(&hist[c], 1u);
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (cur >= 0) {
        const uint32_t h = hist[t];
        if (h)
            atomicAdd((unsigned long long *)&jobs[cur].st->hist[t], (unsigned long long)h);
    }
}

template <int TZ> static void launch_predict_t(const Job *d_jobs, int njobs, uint64_t total,
                                              int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_predict<TZ>, dim3(grid), dim3(256), 0, s, d_jobs, njobs, total);
}

void launch_predict(const Job *d_jobs, int njobs, uint64_t total, int tile_z, int grid,
                    hipStream_t s)
{
    if (total == 0)
        return;
    if (tile_z == 1)
        launch_predict_t<1>(d_jobs, njobs, total, grid, s);
    else if (tile_z == 4)
        launch_predict_t<4>(d_jobs, njobs, total, grid, s);
    else
        launch_predict_t<2>(d_jobs, njobs, total, grid, s);
}

int predict_blocks_per_cu(int tile_z)
{
    int n = 0;
    if (tile_z == 1)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_predict<1>, 256, 0);
    else if (tile_z == 4)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_predict<4>, 256, 0);
    else
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_predict<2>, 256, 0);
    return n > 0 ? n : 1;
}

// ---------------------------------------------------------------------------
// Decompression: rebuild the tile from codes, anchors and outliers.
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(256) void k_reconstruct(const Job *__restrict__ jobs, int njobs,
                                                     uint64_t total)
{
    using TS = TileShape<TZ>;
    __shared__ float v[TS::NV];
    __shared__ uint8_t cl[TS::NV];
    __shared__ uint64_t rowoff[TS::NROW];
    __shared__ uint8_t cfg[kLevels][3];
    __shared__ QParams qp;

    const int t = threadIdx.x;
    int cur = -1;
    uint64_t first, end, step;
    xcd_range(total, first, end, step);
    for (uint64_t u = first; u < end; u += step) {
        const int ji = find_job<WK_TILE>(jobs, njobs, u);
        const Job &J = jobs[ji];
        if (ji != cur) {
            __syncthreads();
            if (t == 0) {
                qp.eps = J.st->eps;
                qp.two_eb = J.st->two_eb;
                qp.inv = 0.f;
            }
            if (t < kLevels * 3)
                cfg[t / 3][t % 3] = J.st->cfg[t / 3][t % 3];
            cur = ji;
            __syncthreads();
        }
        uint64_t ox, oy, oz;
        uint32_t bx, by, bz0;
        const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
        const uint64_t dy = J.dims[1], dz = J.dims[2];
        for (int r = t; r < TS::NROW; r += blockDim.x) {
            const int x = r / kSide, y = r % kSide;
            rowoff[r] = ((ox + x) * dy + (oy + y)) * dz + oz;
        }
        __syncthreads();
        const float *anchors = reinterpret_cast<const float *>(J.stream + J.off_anchors);
        for (int i = t; i < TS::NROW * TS::EZ; i += blockDim.x) {
            const int z = i % TS::EZ, r = i / TS::EZ;
            const int y = r % kSide, x = r / kSide;
            if (x < g.ex && y < g.ey && z < g.ez) {
                const int li = x * TS::PX + y * TS::PZ + z;
                const uint64_t gi = rowoff[r] + z;
                const uint8_t c = J.codes[gi];
                cl[li] = c;
                if ((x & 15) == 0 && (y & 15) == 0 && (z & 15) == 0) {
                    const uint64_t ai = ((uint64_t)(bx + (x >> 4)) * J.nb[1] + (by + (y >> 4))) *
                                            J.nb[2] +
                                        bz0 + (z >> 4);
                    v[li] = anchors[ai];
                } else if (c == 0) {
                    v[li] = J.out[gi]; // outlier value scattered beforehand
                }
            }
        }
        __syncthreads();
        walk_levels<TZ, false>(v, nullptr, cl, g, cfg, qp);
        for (int i = t; i < 16 * 16 * TS::OZ; i += blockDim.x) {
            const int z = i % TS::OZ, r = i / TS::OZ;
            const int y = r % 16, x = r / 16;
            if (x < g.ownx && y < g.owny && z < g.ownz)
                J.out[rowoff[x * kSide + y] + z] = v[x * TS::PX + y * TS::PZ + z];
        }
        __syncthreads();
    }
}

template <int TZ> static void launch_reconstruct_t(const Job *d_jobs, int njobs, uint64_t total,
                                                  int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_reconstruct<TZ>, dim3(grid), dim3(256), 0, s, d_jobs, njobs, total);
}

void launch_reconstruct(const Job *d_jobs, int njobs, uint64_t total, int tile_z, int grid,
                        hipStream_t s)
{
    if (total == 0)
        return;
    if (tile_z == 1)
        launch_reconstruct_t<1>(d_jobs, njobs, total, grid, s);
    else if (tile_z == 4)
        launch_reconstruct_t<4>(d_jobs, njobs, total, grid, s);
    else
        launch_reconstruct_t<2>(d_jobs, njobs, total, grid, s);
}

int reconstruct_blocks_per_cu(int tile_z)
{
    int n = 0;
    if (tile_z == 1)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_reconstruct<1>, 256, 0);
    else if (tile_z == 4)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_reconstruct<4>, 256, 0);
    else
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_reconstruct<2>, 256, 0);
    return n > 0 ? n : 1;
}

} // namespace hiz
