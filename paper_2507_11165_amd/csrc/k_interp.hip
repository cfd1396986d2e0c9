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

#include <type_traits>

namespace hiz {

// axis orders of the sequential scheme (32-bit entries: read with scalar
// loads, which do not wait for vector-memory loads in flight)
__constant__ int32_t c_perm_i[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                       {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// A tile of 1 x 1 x TZ blocks of edge BS (+1 shared face per axis) in LDS.
// BS = 16 is the method's block; BS = 8 is the grid of its even points, on
// which the levels of stride 8, 4, 2 are the same computation at half the
// coordinates (strides 4, 2, 1).
template <int TZ, int BS = 16> struct TileShape {
    static constexpr int SIDE = BS + 1;      // points per block edge incl. the face
    static constexpr int EZ = BS * TZ + 1;   // points along z incl. the far face
    static constexpr int PZ = EZ;            // LDS pitch of a z row (odd: spreads banks)
    static constexpr int PX = SIDE * PZ;     // LDS stride of x
    static constexpr int NV = SIDE * PX;     // values in the tile
    static constexpr int OZ = BS * TZ;       // owned points along z (full tile)
    static constexpr int NC = BS * BS * OZ;  // owned codes
    static constexpr int NROW = SIDE * SIDE;
};

struct Geo {
    int ex, ey, ez;       // tile extents (<= 17, 17, 16*TZ+1)
    int ownx, owny, ownz; // owned extents
};

struct QParams {
    float eps, two_eb, inv;
};

// Compile-time loop over I = B..E-1 (each iteration sees a constant index).
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Four-sample midpoint value of the cubic splines (CUB = 1: Lagrange
// (-1, 9, 9, -1) / 16; CUB = 2: the natural cubic spline through the samples,
// zero second derivative at the outer two, (-3, 23, 23, -3) / 40).
template <int CUB> __device__ __forceinline__ float mid4(float a, float b, float c, float d)
{
    if constexpr (CUB == 2)
        return ((b + c) * 23.0f - (a + d) * 3.0f) / 40.0f;
    else
        return ((b + c) * 9.0f - (a + d)) * 0.0625f;
}

// 1-D spline stencil (Sec. 5.1.2) from the samples a = v(t-3s), b = v(t-s),
// c = v(t+s), d = v(t+3s): the spline's midpoint value (CUB: 0 linear,
// 1 cubic, 2 natural cubic); where samples are missing the order drops to
// quadratic (one side), linear, linear extrapolation or copy. Rank: 4 cubic,
// 3 quadratic, 2 linear, 1 extrapolation, 0 copy. Presence known at compile
// time (interior of full blocks).
template <int CUB, bool PA, bool PC, bool PD>
__device__ __forceinline__ float stencil_ct(float a, float b, float c, float d, int &rank)
{
    if constexpr (CUB && PA && PC && PD) {
        rank = 4;
        return mid4<CUB>(a, b, c, d);
    } else if constexpr (CUB && !PA && PC && PD) {
        rank = 3;
        return ((b * 3.0f + c * 6.0f) - d) * 0.125f;
    } else if constexpr (CUB && PA && PC && !PD) {
        rank = 3;
        return ((b * 6.0f + c * 3.0f) - a) * 0.125f;
    } else if constexpr (PC) {
        rank = 2;
        return (b + c) * 0.5f;
    } else if constexpr (PA) {
        rank = 1;
        return b * 1.5f - a * 0.5f;
    } else {
        rank = 0;
        return b;
    }
}

// The same stencil with presence known only at run time, evaluated without
// branches (every candidate is formed, the applicable one selected; samples
// that are missing are never selected).
template <int CUB>
__device__ __forceinline__ float stencil_rt(float a, float b, float c, float d, bool pa, bool pc,
                                            bool pd, int &rank)
{
    const float vl = (b + c) * 0.5f;
    const float ve = b * 1.5f - a * 0.5f;
    float v = pc ? vl : (pa ? ve : b);
    int r = pc ? 2 : (pa ? 1 : 0);
    if constexpr (CUB) {
        const float vc = mid4<CUB>(a, b, c, d);
        const float vqr = ((b * 3.0f + c * 6.0f) - d) * 0.125f;
        const float vql = ((b * 6.0f + c * 3.0f) - a) * 0.125f;
        const bool full = pa && pc && pd, right = !pa && pc && pd, left = pa && pc && !pd;
        v = full ? vc : (right ? vqr : (left ? vql : v));
        r = full ? 4 : ((right || left) ? 3 : r);
    }
    rank = r;
    return v;
}

// Multi-dimensional combination over the odd axes in mask M: keep the
// predictions of the highest rank and average them in x, y, z order.
template <int M>
__device__ __forceinline__ float md_combine(float px, float py, float pz, int rx, int ry, int rz)
{
    if constexpr (M == 1)
        return px;
    else if constexpr (M == 2)
        return py;
    else if constexpr (M == 4)
        return pz;
    else {
        const int best = max((M & 1) ? rx : -1, max((M & 2) ? ry : -1, (M & 4) ? rz : -1));
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
}

// Linear-scaling quantization (code = 128 + q, |q| <= 127; else outlier code 0
// with the exact value kept). The FP64 check guarantees |x - x'| <= eps after
// FP32 rounding of the reconstruction.
__device__ __forceinline__ uint8_t quantize(float xv, float p, const QParams &q, float &xo)
{
    // the same operations as the definition, evaluated without branches
    const float diff = xv - p;
    const float qf = diff * q.inv;
    const float qr = rintf(qf);
    const bool inrange = fabsf(qr) <= 127.0f;
    const int qi = (int)(inrange ? qr : 0.0f);
    const float xr = p + ((float)qi * q.two_eb);
    const bool ok = inrange && fabs((double)xv - (double)xr) <= (double)q.eps;
    xo = ok ? xr : xv;
    return ok ? (uint8_t)(qi + 128) : (uint8_t)0;
}

// 1-D stencil across the line direction at LDS index li along an axis of
// stride st, for a target whose coordinate on that axis is `c` in a block
// spanning [lo, hi] on that axis (run-time presence; branch-free).
// Samples of a cross-axis stencil: the presence of the samples depends only on
// the target's coordinate on that axis, which is the same for every target of
// a line, so the flags are fixed per line and the loads can be issued early.
struct CrossSamples {
    float a, b, c, d;
};
struct CrossFlags {
    bool pa, pc, pd;
};
template <bool FULL>
__device__ __forceinline__ CrossFlags cross_flags(int c, int lo, int hi, int S)
{
    return CrossFlags{c - 3 * S >= lo, FULL || c + S <= hi, c + 3 * S <= hi};
}
__device__ __forceinline__ CrossSamples cross_load(const float *__restrict__ v, int li, int st,
                                                   int S, const CrossFlags &f)
{
    CrossSamples r;
    r.b = v[li - S * st];
    r.a = v[f.pa ? li - 3 * S * st : li - S * st];
    const int ic = f.pc ? li + S * st : li - S * st;
    r.c = v[ic];
    r.d = v[f.pd ? li + 3 * S * st : ic];
    return r;
}
// 1-D stencil across the line direction from its samples (missing samples
// are never selected).
template <int CUB, bool FULL>
__device__ __forceinline__ float cross_eval(const CrossSamples &s, const CrossFlags &f, int &rank)
{
    if constexpr (FULL) {
        // inside a full block a target always has its +s neighbour
        const float vl = (s.b + s.c) * 0.5f;
        if constexpr (CUB) {
            const float vc = mid4<CUB>(s.a, s.b, s.c, s.d);
            const float vqr = ((s.b * 3.0f + s.c * 6.0f) - s.d) * 0.125f;
            const float vql = ((s.b * 6.0f + s.c * 3.0f) - s.a) * 0.125f;
            const float v1 = f.pa ? vql : vl;
            const float v2 = f.pa ? vc : vqr;
            rank = f.pd ? (f.pa ? 4 : 3) : (f.pa ? 3 : 2);
            return f.pd ? v2 : v1;
        } else {
            rank = 2;
            return vl;
        }
    } else {
        return stencil_rt<CUB>(s.a, s.b, s.c, s.d, f.pa, f.pc, f.pd, rank);
    }
}

// One line of targets: along axis A (0 x, 1 y, 2 z) at stride S inside one
// block, through (x0, y0, z0) whose A-coordinate is the block start; the
// targets sit at odd multiples of S along A, the knowns at even multiples.
// The four samples of the line stencil slide along the line in registers, so
// each target costs one new LDS read plus, for the multi-dimensional scheme,
// stencils along the other odd axes (MB/MC: the first/second other axis in
// x, y, z order is odd and used). nA: extent of the block along A (17 for
// full blocks). The stride is a run-time value so that one compact code path
// serves every level.
template <int TZ, int A, int MB, int MC, int CUB, bool COMP, bool FULL, int BS>
__device__ __forceinline__ void do_line(float *__restrict__ v, uint8_t *__restrict__ cb,
                                        const uint8_t *__restrict__ cl, const Geo &g, int x0,
                                        int y0, int z0, int nA, int S, const QParams &q)
{
    using TS = TileShape<TZ, BS>;
    constexpr int B = (A == 0) ? 1 : 0;
    constexpr int C = (A == 2) ? 1 : 2;
    constexpr int stA = A == 0 ? TS::PX : (A == 1 ? TS::PZ : 1);
    constexpr int stB = B == 0 ? TS::PX : TS::PZ;
    constexpr int stC = C == 1 ? TS::PZ : 1;
    constexpr int M = (1 << A) | (MB << B) | (MC << C);
    const int K = (BS / 2) >> __builtin_ctz(S);
    const int last = nA - 1;
    const int li0 = x0 * TS::PX + y0 * TS::PZ + z0;
    // block bounds of the cross axes
    const int cB = B == 0 ? x0 : y0;
    const int cC = C == 1 ? y0 : z0;
    const int hiB = (B == 0 ? g.ex : g.ey) - 1;
    int loC = 0, hiC;
    if constexpr (C == 2) {
        loC = cC & ~(BS - 1);
        hiC = min(loC + BS, g.ez - 1);
    } else {
        hiC = g.ey - 1;
    }
    const CrossFlags fB = cross_flags<FULL>(cB, 0, hiB, S);
    const CrossFlags fC = cross_flags<FULL>(cC, loC, hiC, S);
    float a = 0.f;
    float b = v[li0];
    float c = v[li0 + min(2 * S, last) * stA];
    float d = v[li0 + min(4 * S, last) * stA];
    // loads of the first target; every later target's loads are issued one
    // iteration ahead, so LDS latency overlaps the previous target's work
    int lin = li0 + min(S, last) * stA;
    float xn = 0.f;
    uint8_t cn = 0;
    if constexpr (COMP)
        xn = v[lin];
    else
        cn = cl[lin];
    CrossSamples sB{}, sC{};
    if constexpr (MB)
        sB = cross_load(v, lin, stB, S, fB);
    if constexpr (MC)
        sC = cross_load(v, lin, stC, S, fC);
#pragma unroll 1
    for (int k = 0; k < K; k++) {
        const int tpos = (2 * k + 1) * S;
        if (!FULL && tpos > last)
            break;
        const int li = lin;
        const float xv = xn;
        const uint8_t cc = cn;
        const CrossSamples tB = sB, tC = sC;
        // next target's loads (in bounds even past the line's end)
        lin = li0 + min(tpos + 2 * S, last) * stA;
        if constexpr (COMP)
            xn = v[lin];
        else
            cn = cl[lin];
        if constexpr (MB)
            sB = cross_load(v, lin, stB, S, fB);
        if constexpr (MC)
            sC = cross_load(v, lin, stC, S, fC);
        const bool pa = k > 0, pc = FULL || (2 * k + 2) * S <= last,
                   pd = (2 * k + 4) * S <= last;
        int rA;
        float pA;
        if (CUB && pa && pc && pd) {
            rA = 4;
            pA = mid4<CUB>(a, b, c, d);
        } else {
            pA = stencil_rt<CUB>(a, b, c, d, pa, pc, pd, rA);
        }
        float p;
        if constexpr (M == (1 << A)) {
            p = pA;
        } else {
            float pB = 0.f, pC = 0.f;
            int rB = -1, rC = -1;
            if constexpr (MB)
                pB = cross_eval<CUB, FULL>(tB, fB, rB);
            if constexpr (MC)
                pC = cross_eval<CUB, FULL>(tC, fC, rC);
            const float px = A == 0 ? pA : pB;
            const int rx = A == 0 ? rA : rB;
            const float py = A == 1 ? pA : (B == 1 ? pB : pC);
            const int ry = A == 1 ? rA : (B == 1 ? rB : rC);
            const float pz = A == 2 ? pA : pC;
            const int rz = A == 2 ? rA : rC;
            p = md_combine<M>(px, py, pz, rx, ry, rz);
        }
        // slide the window: the next target's +3s sample
        a = b;
        b = c;
        c = d;
        d = v[li0 + min((2 * k + 6) * S, last) * stA];
        const int x = A == 0 ? tpos : x0;
        const int y = A == 1 ? tpos : y0;
        const int z = A == 2 ? z0 + tpos : z0;
        if constexpr (COMP) {
            float xo;
            const uint8_t code = quantize(xv, p, q, xo);
            v[li] = xo;
            const bool own = x < g.ownx && y < g.owny && z < g.ownz;
            cb[own ? (x * BS + y) * TS::OZ + z : TS::NC] = code;
        } else {
            if (cc != 0)
                v[li] = p + ((float)((int)cc - 128) * q.two_eb);
            // code 0: the exact outlier value is already in place
        }
    }
}

enum : int { M_EVEN = 0, M_ODD = 1, M_ALL = 2 };

// Coordinates of a mode in [0, n - 1] at stride S = 2^ls (shifts, no division).
__device__ __forceinline__ int mode_count(int mode, int n, int ls)
{
    if (mode == M_EVEN)
        return ((n - 1) >> (ls + 1)) + 1;
    if (mode == M_ODD)
        return n - 1 >= (1 << ls) ? ((n - 1 - (1 << ls)) >> (ls + 1)) + 1 : 0;
    return ((n - 1) >> ls) + 1;
}
__device__ __forceinline__ int mode_coord(int mode, int i, int S)
{
    return mode == M_EVEN ? 2 * i * S : (mode == M_ODD ? (2 * i + 1) * S : i * S);
}

// quotient n / d for n, d < 2^16 with a multiply (m = floor((2^32 - 1) / d) + 1)
__device__ __forceinline__ uint32_t qdiv(uint32_t n, uint32_t d, uint32_t m)
{
    return d == 1 ? n : __umulhi(n, m);
}
// The multipliers of every divisor a line group can have (line counts per
// cross axis up to 17 and 16 * 4 + 1, and their products), built at compile
// time so that no division runs on the device.
constexpr int kMagicMax = kSide * (16 * 4 + 1);
struct MagicTable {
    uint32_t m[kMagicMax + 1];
};
constexpr MagicTable make_magic_table()
{
    MagicTable t{};
    for (int d = 0; d <= kMagicMax; d++)
        t.m[d] = d <= 1 ? 0u : (uint32_t)(0xffffffffu / (uint32_t)d + 1u);
    return t;
}
__constant__ MagicTable c_magic = make_magic_table();
// d is the same for the whole workgroup: the lookup is a scalar load, which
// does not wait for the vector-memory loads in flight
__device__ __forceinline__ uint32_t qmagic(uint32_t d)
{
    return c_magic.m[__builtin_amdgcn_readfirstlane(d)];
}
template <int V> constexpr int kLog2 = V <= 1 ? 0 : 1 + kLog2<V / 2>;

// A group of lines of one kind: axis A plus which cross axes are odd and
// interpolated (MD), with the coordinate modes of the two cross axes.
struct LineGroup {
    int kind;        // template instance, see run_line
    int A, modeB, modeC;
    int cntB, cntC, ncell, lines;
    uint32_t mC, mBC; // magic multipliers for / cntC and / (cntB * cntC)
};

__device__ __forceinline__ LineGroup make_group(int kind, int A, int modeB, int modeC, int S,
                                                int ls, const Geo &g, int TZ, int lbs)
{
    LineGroup G;
    G.kind = kind;
    G.A = A;
    G.modeB = modeB;
    G.modeC = modeC;
    const int nB = A == 0 ? g.ey : g.ex;
    const int nC = A == 2 ? g.ey : g.ez;
    G.cntB = mode_count(modeB, nB, ls);
    G.cntC = mode_count(modeC, nC, ls);
    if (A == 2)
        G.ncell = g.ez - 1 >= S ? min(TZ, ((g.ez - 1 - S) >> lbs) + 1) : 0;
    else
        G.ncell = 1;
    if ((A == 0 && g.ex - 1 < S) || (A == 1 && g.ey - 1 < S))
        G.ncell = 0;
    G.lines = G.cntB * G.cntC * G.ncell;
    G.mC = qmagic((uint32_t)G.cntC);
    G.mBC = qmagic((uint32_t)(G.cntB * G.cntC));
    return G;
}

// kinds: 0..2 plain lines along z, y, x; 3 along x with y odd (MD xy);
// 4 along z with x odd (MD xz); 5 along z with y odd (MD yz); 6 along z with x
// and y odd (MD xyz).
template <int TZ, int CUB, bool COMP, bool FULL, int BS>
__device__ __forceinline__ void run_line(const LineGroup &G, int l, int S, float *v, uint8_t *cb,
                                         const uint8_t *cl, const Geo &g, const QParams &q)
{
    const uint32_t nbc = (uint32_t)(G.cntB * G.cntC);
    const uint32_t cell = qdiv((uint32_t)l, nbc, G.mBC);
    const uint32_t rem = (uint32_t)l - cell * nbc;
    const uint32_t iB = qdiv(rem, (uint32_t)G.cntC, G.mC);
    const uint32_t iC = rem - iB * (uint32_t)G.cntC;
    const int cB = mode_coord(G.modeB, (int)iB, S);
    const int cC = mode_coord(G.modeC, (int)iC, S);
    if (G.A == 2) {
        const int z0 = BS * (int)cell;
        const int nA = FULL ? BS + 1 : min(BS + 1, g.ez - z0);
        switch (G.kind) {
        case 0: do_line<TZ, 2, 0, 0, CUB, COMP, FULL, BS>(v, cb, cl, g, cB, cC, z0, nA, S, q); break;
        case 4: do_line<TZ, 2, 1, 0, CUB, COMP, FULL, BS>(v, cb, cl, g, cB, cC, z0, nA, S, q); break;
        case 5: do_line<TZ, 2, 0, 1, CUB, COMP, FULL, BS>(v, cb, cl, g, cB, cC, z0, nA, S, q); break;
        default: do_line<TZ, 2, 1, 1, CUB, COMP, FULL, BS>(v, cb, cl, g, cB, cC, z0, nA, S, q); break;
        }
    } else if (G.A == 1) {
        do_line<TZ, 1, 0, 0, CUB, COMP, FULL, BS>(v, cb, cl, g, cB, 0, cC, FULL ? BS + 1 : g.ey, S,
                                                  q);
    } else if (G.kind == 3) {
        do_line<TZ, 0, 1, 0, CUB, COMP, FULL, BS>(v, cb, cl, g, 0, cB, cC, FULL ? BS + 1 : g.ex, S,
                                                  q);
    } else {
        do_line<TZ, 0, 0, 0, CUB, COMP, FULL, BS>(v, cb, cl, g, 0, cB, cC, FULL ? BS + 1 : g.ex, S,
                                                  q);
    }
}

// The finest level (stride 1) inside a full tile of blocks of BS (16: the
// method's blocks; 8: the pre-pass's even-point grid, whose stride 1 is the
// stride-2 level), where 7 of every 8 targets sit: the line has its full
// BS + 1 points, so its BS / 2 targets, their window of knowns and the
// presence of every line sample are fixed at compile time. All samples are
// read up front at constant offsets from the line's start and the targets
// run unrolled; only the cross-axis sample presence (fixed per line) is a
// run-time choice. Arithmetic is the same as in do_line, operation for
// operation.
// KB, KE: the line's targets KB..KE-1 (a half line when a sub-step has too
// few lines to fill the workgroup), with the knowns their stencils read.
template <int TZ, int A, int MB, int MC, int CUB, bool COMP, int BS = 16, int KB = 0,
          int KE = BS / 2>
__device__ __forceinline__ void do_line_s1(float *__restrict__ v, uint8_t *__restrict__ cb,
                                           const uint8_t *__restrict__ cl, const Geo &g, int x0,
                                           int y0, int z0, const QParams &q)
{
    constexpr int NT = BS / 2; // targets of a full line
    static_assert(0 <= KB && KB < KE && KE <= NT, "targets of one line");
    constexpr int JB = KB > 0 ? KB - 1 : 0, JE = KE < NT ? KE + 1 : NT; // knowns JB..JE
    using TS = TileShape<TZ, BS>;
    constexpr int B = (A == 0) ? 1 : 0;
    constexpr int C = (A == 2) ? 1 : 2;
    constexpr int stA = A == 0 ? TS::PX : (A == 1 ? TS::PZ : 1);
    constexpr int stB = B == 0 ? TS::PX : TS::PZ;
    constexpr int stC = C == 1 ? TS::PZ : 1;
    constexpr int M = (1 << A) | (MB << B) | (MC << C);
    const int li0 = x0 * TS::PX + y0 * TS::PZ + z0;
    const float *vl = v + li0;
    // cross-axis sample presence, fixed along the line
    const int cB = B == 0 ? x0 : y0;
    const int cC = C == 1 ? y0 : z0;
    const int loC = C == 2 ? (cC & ~(BS - 1)) : 0;
    const CrossFlags fB = cross_flags<true>(cB, 0, TS::SIDE - 1, 1);
    const CrossFlags fC = cross_flags<true>(cC, loC, loC + BS, 1);
    const int oBa = fB.pa ? -3 * stB : -stB, oBd = fB.pd ? 3 * stB : stB;
    const int oCa = fC.pa ? -3 * stC : -stC, oCd = fC.pd ? 3 * stC : stC;
    // codes: owned lines write at a fixed step, others to the dummy slot
    constexpr int cstep = A == 0 ? BS * TS::OZ : (A == 1 ? TS::OZ : 1);
    bool own;
    int cbase;
    if constexpr (A == 2) {
        own = x0 < g.ownx && y0 < g.owny;
        cbase = (x0 * BS + y0) * TS::OZ + z0;
    } else if constexpr (A == 1) {
        own = x0 < g.ownx && z0 < g.ownz;
        cbase = x0 * BS * TS::OZ + z0;
    } else {
        own = y0 < g.owny && z0 < g.ownz;
        cbase = y0 * TS::OZ + z0;
    }
    const int cb0 = own ? cbase : TS::NC;
    const int cst = own ? cstep : 0;
    float w[NT + 1];
#pragma unroll
    for (int j = JB; j <= JE; j++)
        w[j] = vl[2 * j * stA];
    float xv[NT];
    uint8_t cc[NT];
#pragma unroll
    for (int k = KB; k < KE; k++) {
        xv[k] = vl[(2 * k + 1) * stA];
        if constexpr (!COMP)
            cc[k] = cl[li0 + (2 * k + 1) * stA];
    }
    // Cross-axis samples of target k, read one target ahead: the next
    // target's reads are issued before this target's value is written back,
    // so that their latency overlaps this target's arithmetic (no target of a
    // sub-step reads another's result, so the order is free).
    struct XS {
        CrossSamples b, c;
    };
    auto load_cross = [&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        const int li = li0 + (2 * k + 1) * stA;
        XS r{};
        if constexpr (MB) {
            r.b.b = v[li - stB];
            r.b.a = v[li + oBa];
            r.b.c = v[li + stB];
            r.b.d = v[li + oBd];
        }
        if constexpr (MC) {
            r.c.b = v[li - stC];
            r.c.a = v[li + oCa];
            r.c.c = v[li + stC];
            r.c.d = v[li + oCd];
        }
        return r;
    };
    XS xs[NT];
    if constexpr (M != (1 << A))
        xs[KB] = load_cross(std::integral_constant<int, KB>{});
    static_for<KB, KE>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int tpos = 2 * k + 1;
        const int li = li0 + tpos * stA;
        if constexpr (M != (1 << A) && k + 1 < KE)
            xs[k + 1] = load_cross(std::integral_constant<int, (k + 1 < KE ? k + 1 : k)>{});
        int rA;
        const float pA = stencil_ct<CUB, (k > 0), true, (k < NT - 1)>(
            k > 0 ? w[k > 0 ? k - 1 : 0] : 0.f, w[k], w[k + 1],
            k < NT - 1 ? w[k < NT - 1 ? k + 2 : NT] : 0.f, rA);
        float p;
        if constexpr (M == (1 << A)) {
            p = pA;
        } else {
            float pB = 0.f, pC = 0.f;
            int rB = -1, rC = -1;
            if constexpr (MB)
                pB = cross_eval<CUB, true>(xs[k].b, fB, rB);
            if constexpr (MC)
                pC = cross_eval<CUB, true>(xs[k].c, fC, rC);
            const float px = A == 0 ? pA : pB;
            const int rx = A == 0 ? rA : rB;
            const float py = A == 1 ? pA : (B == 1 ? pB : pC);
            const int ry = A == 1 ? rA : (B == 1 ? rB : rC);
            const float pz = A == 2 ? pA : pC;
            const int rz = A == 2 ? rA : rC;
            p = md_combine<M>(px, py, pz, rx, ry, rz);
        }
        if constexpr (COMP) {
            float xo;
            const uint8_t code = quantize(xv[k], p, q, xo);
            v[li] = xo;
            cb[cb0 + tpos * cst] = code;
        } else {
            // code 0: the exact outlier value already in place is kept
            const uint8_t c8 = cc[k];
            v[li] = c8 != 0 ? p + ((float)((int)c8 - 128) * q.two_eb) : xv[k];
        }
    });
}

// Half of a line of three-dimensional targets (sub-step 3 of the MD scheme,
// whose lines number half the workgroup or fewer): the first or second half
// of its targets.
template <int TZ, int CUB, bool COMP, int BS>
__device__ __forceinline__ void run_half_line_s1(const LineGroup &G, int l, int half, float *v,
                                                 uint8_t *cb, const uint8_t *cl, const Geo &g,
                                                 const QParams &q)
{
    const uint32_t nbc = (uint32_t)(G.cntB * G.cntC);
    const uint32_t cell = qdiv((uint32_t)l, nbc, G.mBC);
    const uint32_t rem = (uint32_t)l - cell * nbc;
    const uint32_t iB = qdiv(rem, (uint32_t)G.cntC, G.mC);
    const uint32_t iC = rem - iB * (uint32_t)G.cntC;
    const int cB = mode_coord(G.modeB, (int)iB, 1);
    const int cC = mode_coord(G.modeC, (int)iC, 1);
    const int z0 = BS * (int)cell;
    constexpr int H = BS / 4;
    if (half == 0)
        do_line_s1<TZ, 2, 1, 1, CUB, COMP, BS, 0, H>(v, cb, cl, g, cB, cC, z0, q);
    else
        do_line_s1<TZ, 2, 1, 1, CUB, COMP, BS, H, 2 * H>(v, cb, cl, g, cB, cC, z0, q);
}

template <int TZ, int CUB, bool COMP, int BS>
__device__ __forceinline__ void run_line_s1(const LineGroup &G, int l, float *v, uint8_t *cb,
                                            const uint8_t *cl, const Geo &g, const QParams &q)
{
    const uint32_t nbc = (uint32_t)(G.cntB * G.cntC);
    const uint32_t cell = qdiv((uint32_t)l, nbc, G.mBC);
    const uint32_t rem = (uint32_t)l - cell * nbc;
    const uint32_t iB = qdiv(rem, (uint32_t)G.cntC, G.mC);
    const uint32_t iC = rem - iB * (uint32_t)G.cntC;
    const int cB = mode_coord(G.modeB, (int)iB, 1);
    const int cC = mode_coord(G.modeC, (int)iC, 1);
    if (G.A == 2) {
        const int z0 = BS * (int)cell;
        switch (G.kind) {
        case 0: do_line_s1<TZ, 2, 0, 0, CUB, COMP, BS>(v, cb, cl, g, cB, cC, z0, q); break;
        case 4: do_line_s1<TZ, 2, 1, 0, CUB, COMP, BS>(v, cb, cl, g, cB, cC, z0, q); break;
        case 5: do_line_s1<TZ, 2, 0, 1, CUB, COMP, BS>(v, cb, cl, g, cB, cC, z0, q); break;
        default: do_line_s1<TZ, 2, 1, 1, CUB, COMP, BS>(v, cb, cl, g, cB, cC, z0, q); break;
        }
    } else if (G.A == 1) {
        do_line_s1<TZ, 1, 0, 0, CUB, COMP, BS>(v, cb, cl, g, cB, 0, cC, q);
    } else if (G.kind == 3) {
        do_line_s1<TZ, 0, 1, 0, CUB, COMP, BS>(v, cb, cl, g, 0, cB, cC, q);
    } else {
        do_line_s1<TZ, 0, 0, 0, CUB, COMP, BS>(v, cb, cl, g, 0, cB, cC, q);
    }
}

// One level (stride S) in three sub-steps, each a set of line groups swept in
// parallel by the workgroup, with a barrier between sub-steps.
// MD: 1-D, then 2-D, then 3-D targets. SEQ(order): pass j interpolates along
// the j-th axis of the order every target whose last odd axis (in that order)
// is that axis; axes earlier in the order take every multiple of S, later
// ones even multiples only.
template <int TZ, int CUB, bool COMP, bool FULL, int BS>
__device__ __forceinline__ void level_lines(float *v, uint8_t *cb, const uint8_t *cl, const Geo &g,
                                            int S, bool md, int perm, const QParams &q)
{
    // workgroup size: 256 threads for blocks of 16, one wave for the
    // even-point grid (a constant, so no load of the launch size waits on
    // the vector-memory loads in flight)
    constexpr int NT = BS == 16 ? 256 : 64;
    const int ls = __builtin_ctz(S);
    for (int sub = 1; sub <= 3; sub++) {
        LineGroup G0, G1, G2;
        int ng;
        if (md) {
            if (sub == 1) {
                G0 = make_group(0, 2, M_EVEN, M_EVEN, S, ls, g, TZ, kLog2<BS>);
                G1 = make_group(1, 1, M_EVEN, M_EVEN, S, ls, g, TZ, kLog2<BS>);
                G2 = make_group(2, 0, M_EVEN, M_EVEN, S, ls, g, TZ, kLog2<BS>);
                ng = 3;
            } else if (sub == 2) {
                G0 = make_group(3, 0, M_ODD, M_EVEN, S, ls, g, TZ, kLog2<BS>);
                G1 = make_group(4, 2, M_ODD, M_EVEN, S, ls, g, TZ, kLog2<BS>);
                G2 = make_group(5, 2, M_EVEN, M_ODD, S, ls, g, TZ, kLog2<BS>);
                ng = 3;
            } else {
                G0 = make_group(6, 2, M_ODD, M_ODD, S, ls, g, TZ, kLog2<BS>);
                G1 = G0;
                G2 = G0;
                ng = 1;
            }
        } else {
            // uniform index: scalar loads of the table
            perm = __builtin_amdgcn_readfirstlane(perm);
            const int A = c_perm_i[perm][sub - 1];
            const int B = A == 0 ? 1 : 0, C = A == 2 ? 1 : 2;
            // an axis placed before A in the order may be odd or even
            bool earlyB = false, earlyC = false;
            for (int j = 0; j < sub - 1; j++) {
                earlyB |= c_perm_i[perm][j] == B;
                earlyC |= c_perm_i[perm][j] == C;
            }
            const int modeB = earlyB ? M_ALL : M_EVEN;
            const int modeC = earlyC ? M_ALL : M_EVEN;
            G0 = make_group(A == 2 ? 0 : (A == 1 ? 1 : 2), A, modeB, modeC, S, ls, g, TZ, kLog2<BS>);
            G1 = G0;
            G2 = G0;
            ng = 1;
        }
        const int n0 = G0.lines;
        const int n1 = n0 + (ng > 1 ? G1.lines : 0);
        const int n2 = n1 + (ng > 2 ? G2.lines : 0);
        if (FULL && S == 1) {
            if constexpr (FULL) {
                if (md && sub == 3 && 2 * n0 <= NT) {
                    // three-dimensional targets: half lines, one per thread
                    if ((int)threadIdx.x < 2 * n0)
                        run_half_line_s1<TZ, CUB, COMP, BS>(G0, threadIdx.x >> 1, threadIdx.x & 1,
                                                            v, cb, cl, g, q);
                } else
                for (int i = threadIdx.x; i < n2; i += NT) {
                    if (i < n0)
                        run_line_s1<TZ, CUB, COMP, BS>(G0, i, v, cb, cl, g, q);
                    else if (i < n1)
                        run_line_s1<TZ, CUB, COMP, BS>(G1, i - n0, v, cb, cl, g, q);
                    else
                        run_line_s1<TZ, CUB, COMP, BS>(G2, i - n1, v, cb, cl, g, q);
                }
            }
        } else {
            for (int i = threadIdx.x; i < n2; i += NT) {
                if (i < n0)
                    run_line<TZ, CUB, COMP, FULL, BS>(G0, i, S, v, cb, cl, g, q);
                else if (i < n1)
                    run_line<TZ, CUB, COMP, FULL, BS>(G1, i - n0, S, v, cb, cl, g, q);
                else
                    run_line<TZ, CUB, COMP, FULL, BS>(G2, i - n1, S, v, cb, cl, g, q);
            }
        }
        lds_barrier();
    }
}

template <int TZ, bool COMP, int BS = 16>
__device__ __forceinline__ void level(float *v, uint8_t *cb, const uint8_t *cl, const Geo &g, int S,
                                      const uint8_t *cfg, const QParams &q)
{
    const int spline = cfg[0];
    const bool md = cfg[1] == 0;
    const int perm = cfg[2];
    const bool full = g.ex == BS + 1 && g.ey == BS + 1 && g.ez == BS * TZ + 1;
    if (spline == 2) {
        if (full)
            level_lines<TZ, 2, COMP, true, BS>(v, cb, cl, g, S, md, perm, q);
        else
            level_lines<TZ, 2, COMP, false, BS>(v, cb, cl, g, S, md, perm, q);
    } else if (spline == 1) {
        if (full)
            level_lines<TZ, 1, COMP, true, BS>(v, cb, cl, g, S, md, perm, q);
        else
            level_lines<TZ, 1, COMP, false, BS>(v, cb, cl, g, S, md, perm, q);
    } else {
        if (full)
            level_lines<TZ, 0, COMP, true, BS>(v, cb, cl, g, S, md, perm, q);
        else
            level_lines<TZ, 0, COMP, false, BS>(v, cb, cl, g, S, md, perm, q);
    }
}

// Levels of stride 8, 4, 2, 1 in order (coarse to fine).
template <int TZ, bool COMP>
__device__ __forceinline__ void walk_levels(float *v, uint8_t *cb, const uint8_t *cl, const Geo &g,
                                            const uint8_t (*cfg)[3], const QParams &q)
{
#pragma unroll 1
    for (int l = 0; l < kLevels; l++)
        level<TZ, COMP>(v, cb, cl, g, 8 >> l, cfg[l], q);
}

// Tile u of job J -> geometry and global row offsets (into LDS `rowoff`).
template <int TZ>
__device__ __forceinline__ Geo tile_geometry(const Job &J, uint64_t lt, uint64_t &ox, uint64_t &oy,
                                             uint64_t &oz, uint32_t &bx, uint32_t &by,
                                             uint32_t &bz0)
{
    // a launch holds fewer than 2^32 tiles: 32-bit division
    const uint32_t l = (uint32_t)lt;
    const uint32_t tz = l % J.ntz, r = l / J.ntz;
    by = r % J.nb[1];
    bx = r / J.nb[1];
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

// Tiles whose owned points all lie inside the field (only a far face may be
// missing, where the field ends): their coarse levels run in the pre-pass.
template <int TZ> __device__ __forceinline__ bool prepass_tile(const Geo &g)
{
    return g.ownx == 16 && g.owny == 16 && g.ownz == 16 * TZ;
}

// Tiles handed out on demand. Each XCD (workgroups are dealt to the eight
// XCDs round-robin by blockIdx) owns a contiguous eighth of the tile list, so
// tiles that share halo faces meet in the same L2, and its workgroups claim
// tiles one at a time from a counter: a workgroup that meets slower tiles
// (partial ones at the field's faces) simply takes fewer. A workgroup whose
// own eighth is exhausted goes on to the other XCDs' eighths, so an eighth
// that holds more partial tiles does not hold up the launch. Thread 0 asks
// for the next tile while the current one is processed; the index goes
// through a two-slot LDS buffer so that it never overwrites the one some
// wave is still reading. The claims are made by the first lane of the last
// wave, which issues no global stores of its own: reading a claim's result
// then waits only for that wave's loads (long done), not for the tile's
// output stores still draining.
constexpr int kClaimThread = 192;
constexpr int kStoreThreads = 192; // threads of a tile's output stores
struct TileQueue {
    uint64_t base;  // first tile of the launch's range
    uint64_t total; // tiles in the range
    uint32_t *ctr;  // eight counters, one per eighth
    int home;      // this workgroup's XCD
    int k;         // eighths tried so far (thread 0)
    uint32_t ask;  // outstanding claim on eighth (home + k) & 7 (thread 0)
};
__device__ __forceinline__ uint64_t eighth_lo(uint64_t total, int x) { return total * x / 8; }
__device__ __forceinline__ TileQueue tile_queue(uint64_t lo, uint64_t hi, uint32_t *ctr)
{
    TileQueue q;
    q.base = lo;
    q.total = hi - lo;
    q.ctr = ctr;
    q.home = (gridDim.x >= 8 && (gridDim.x & 7) == 0) ? (int)(blockIdx.x & 7) : 0;
    q.k = 0;
    q.ask = 0;
    if (threadIdx.x == kClaimThread)
        q.ask = atomicAdd(&q.ctr[q.home], 1u);
    return q;
}
// Claiming thread: resolve the outstanding claim into a tile index (the
// range's end = none left) and ask for the following one.
__device__ __forceinline__ uint64_t next_tile(TileQueue &q)
{
    while (q.k < 8) {
        const int x = (q.home + q.k) & 7;
        const uint64_t lo = eighth_lo(q.total, x), hi = eighth_lo(q.total, x + 1);
        if (lo + q.ask < hi) {
            // an eighth is dealt from its end: the tiles cut by the field's
            // far faces (slower: all four levels, general line code) gather
            // there and go first instead of holding up the end of the launch
            const uint64_t u = hi - 1 - q.ask;
            q.ask = atomicAdd(&q.ctr[x], 1u);
            return q.base + u;
        }
        q.k++;
        if (q.k < 8)
            q.ask = atomicAdd(&q.ctr[(q.home + q.k) & 7], 1u);
    }
    return q.base + q.total;
}
__device__ __forceinline__ uint64_t claim_tile(TileQueue &q, uint64_t *slot, int it)
{
    if (threadIdx.x == kClaimThread)
        slot[it & 1] = next_tile(q);
    lds_barrier();
    // the same for every lane: job lookups and job fields go to scalar loads
    // (the builtin returns a signed int: both halves go back to uint32_t
    // before widening, so that the low half is never sign-extended)
    const uint64_t u = slot[it & 1];
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Tile I/O. Values go from global memory straight into LDS, every load of
// the tile in flight at once. For codes each thread issues all of its global
// loads before it writes any of them to LDS, so a tile costs one memory round
// trip rather than one per element; rows are read as 16-byte pieces where
// the field's rows are 16-byte aligned (dz a multiple of 16).
// ---------------------------------------------------------------------------
// LDS words dst[(x * SIDE + y) * PZ + z], e < N, from global offsets
// base + x * sx + y * sy + z * sz. Wave w of NW issues loads w, w + NW, ...
// (64 words each); a lane's coordinates and offset advance incrementally. In
// a partial tile (full false) words outside the extents ex, ey, ez take the
// value at base and are never read.
template <int N, int PZ, int SIDE, int NW>
__device__ __forceinline__ void lds_fill_tile(float *__restrict__ dst,
                                              HIZ_GLOBAL const float *__restrict__ src,
                                              uint64_t base, uint64_t sx, uint64_t sy, uint64_t sz,
                                              bool full, int ex, int ey, int ez)
{
    constexpr int NJ = (N + 63) / 64;
    constexpr int STEP = 64 * NW, DR = STEP / PZ, DZ = STEP % PZ;
    static_assert(DR < SIDE, "one step crosses at most one row of rows");
    const int wave = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int e0 = 64 * wave + lane;
    int z = e0 % PZ, r = e0 / PZ;
    int y = r % SIDE, x = r / SIDE;
    uint64_t off = base + (uint64_t)x * sx + (uint64_t)y * sy + (uint64_t)z * sz;
    // offset steps (unsigned wrap-around where a step goes backwards)
    const uint64_t d0 = (uint64_t)DR * sy + (uint64_t)DZ * sz;
    const uint64_t dzw = sy - (uint64_t)PZ * sz;
    const uint64_t dyw = sx - (uint64_t)SIDE * sy;
#pragma unroll 2
    for (int j = wave; j < NJ; j += NW) {
        const bool in = full || (x < ex && y < ey && z < ez);
        if (N % 64 == 0 || j < NJ - 1 || 64 * j + lane < N)
            lds_load_word(src + (in ? off : base), dst + 64 * j);
        z += DZ;
        y += DR;
        off += d0;
        if (z >= PZ) {
            z -= PZ;
            y += 1;
            off += dzw;
        }
        if (y >= SIDE) {
            y -= SIDE;
            x += 1;
            off += dyw;
        }
    }
}

// Extremes (as order keys) and finiteness of the tile's values in LDS.
template <int TZ>
__device__ __forceinline__ void scan_tile_values(const float *__restrict__ v, const Geo &g,
                                                 uint32_t &kmn, uint32_t &kmx, bool &bad)
{
    using TS = TileShape<TZ>;
    for (int e = threadIdx.x; e < TS::NV; e += 256) {
        const int r = e / TS::PZ, z = e - r * TS::PZ;
        const int x = r / kSide, y = r - x * kSide;
        if (x < g.ex && y < g.ey && z < g.ez) {
            const float val = v[e];
            bad |= !isfinite(val);
            const uint32_t k = fkey(val);
            kmn = min(kmn, k);
            kmx = max(kmx, k);
        }
    }
}

// Codes of the whole tile region (with faces) into LDS, any alignment: each
// thread issues 8 byte loads before it writes any of them.
template <int TZ>
__device__ __forceinline__ void load_tile_codes(uint8_t *__restrict__ cl,
                                                HIZ_GLOBAL const uint8_t *__restrict__ codes,
                                                uint64_t base, uint64_t sx, uint64_t dz,
                                                const Geo &g)
{
    using TS = TileShape<TZ>;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma nounroll
    for (int i0 = 0; i0 < TS::NV; i0 += 256 * 8) {
        uint8_t b[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int e = i0 + tid + 256 * k;
            const int z = e % TS::PZ, r = e / TS::PZ;
            const int y = r % kSide, x = r / kSide;
            const bool in = e < TS::NV && x < g.ex && y < g.ey && z < g.ez;
            b[k] = codes[in ? base + (uint64_t)x * sx + (uint64_t)y * dz + z : base];
        }
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int e = i0 + tid + 256 * k;
            if (e < TS::NV)
                cl[e] = b[k];
        }
    }
}

// A full tile's even-point grid after the coarse levels (values, and for
// compression the codes of its owned points) replaces the raw values in the
// tile: its loads are issued ahead of the tile's own loads (coarse_fetch) and
// written into LDS once the tile is there (coarse_place).
template <int TZ, int NT> struct CoarseRegs {
    using TC = TileShape<TZ, 8>;
    static constexpr int IV = (TC::NV + NT - 1) / NT;
    static constexpr int IC = (TC::NC / 4 + NT - 1) / NT; // 4-byte words
    float val[IV];
    uint32_t code[IC];
};
template <int TZ, int NT>
__device__ __forceinline__ void coarse_fetch(CoarseRegs<TZ, NT> &r, int tid,
                                             HIZ_GLOBAL const float *__restrict__ crec,
                                             HIZ_GLOBAL const uint8_t *__restrict__ ccode)
{
    using TC = TileShape<TZ, 8>;
    static_assert(TC::NC % 4 == 0 && TC::OZ % 4 == 0, "code words hold 4 points of a row");
#pragma unroll
    for (int k = 0; k < r.IV; k++) {
        const int i = tid + NT * k;
        r.val[k] = crec[i < TC::NV ? i : 0];
    }
    if (ccode) {
        HIZ_GLOBAL const uint32_t *cw = reinterpret_cast<HIZ_GLOBAL const uint32_t *>(ccode);
#pragma unroll
        for (int k = 0; k < r.IC; k++) {
            const int i = tid + NT * k;
            r.code[k] = cw[i < TC::NC / 4 ? i : 0];
        }
    }
}
template <int TZ, int NT>
__device__ __forceinline__ void coarse_place(const CoarseRegs<TZ, NT> &r, int tid,
                                             float *__restrict__ v, uint8_t *__restrict__ cb)
{
    using TF = TileShape<TZ>;
    using TC = TileShape<TZ, 8>;
    // LDS addresses are recomputed per tile, not kept (or spilled) across the tile loop
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int k = 0; k < r.IV; k++) {
        const int i = tid + NT * k;
        if (i < TC::NV) {
            const int zc = i % TC::PZ, q = i / TC::PZ;
            const int yc = q % TC::SIDE, xc = q / TC::SIDE;
            v[2 * xc * TF::PX + 2 * yc * TF::PZ + 2 * zc] = r.val[k];
        }
    }
    if (cb) {
#pragma unroll
        for (int k = 0; k < r.IC; k++) {
            const int i = 4 * (tid + NT * k);
            if (i < TC::NC) {
                const int zc = i % TC::OZ, q = i / TC::OZ;
                const int yc = q % 8, xc = q / 8;
                uint8_t *c = cb + (2 * xc * 16 + 2 * yc) * TF::OZ + 2 * zc;
#pragma unroll
                for (int b = 0; b < 4; b++)
                    c[2 * b] = (uint8_t)(r.code[k] >> (8 * b));
            }
        }
    }
}

// A tile's values (and, for a full tile, its coarse-grid results) fetched
// into registers while the previous tile is computed. Rows of the tile are
// read as 16-byte pieces (thread t holds pieces t + 256 k, a piece being four
// consecutive z of one (x, y) row) plus the far z face one point per row;
// this needs rows that start 16-byte aligned and tiles that hold every piece
// (the tile's z extent at least 16 * TZ). Other tiles are loaded straight
// into LDS when they are placed. Used where the registers fit next to the
// levels' (tiles of one or two blocks).
template <int TZ> struct TileRegs {
    static constexpr int NP = kSide * kSide * 4 * TZ; // pieces
    static constexpr int IP = (NP + 255) / 256;
    static constexpr int NF = kSide * kSide; // far-face points
    static constexpr int IF = (NF + 255) / 256;
    float4 piece[IP];
    float face[IF];
    CoarseRegs<TZ, 256> cr;
    bool vec; // pieces fetched (else the tile is loaded when placed)
};
template <int TZ> constexpr bool kPrefetchTiles = TZ <= 2;

template <int TZ>
__device__ __forceinline__ void tile_fetch(TileRegs<TZ> &f, const Job &J, uint64_t u, int tid)
{
    using TS = TileShape<TZ>;
    using TR = TileRegs<TZ>;
    // the lane's coordinate sequence depends on the thread index alone: made
    // opaque here so that it is recomputed per tile rather than hoisted out
    // of the tile loop into dozens of long-lived registers
    asm volatile("" : "+v"(tid));
    uint64_t ox, oy, oz;
    uint32_t bx, by, bz0;
    const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
    const uint64_t dy = J.dims[1], dz = J.dims[2];
    const uint64_t sx = dy * dz, base = (ox * dy + oy) * dz + oz;
    const bool full = g.ex == kSide && g.ey == kSide && g.ez == TS::EZ;
    f.vec = (dz & 3) == 0 && (reinterpret_cast<uintptr_t>(J.field) & 15) == 0 &&
            g.ez >= 16 * TZ;
    if (J.crec && prepass_tile<TZ>(g)) {
        const uint64_t ci = ((uint64_t)bx * J.nf[1] + by) * J.nf[2] + bz0 / TZ;
        coarse_fetch<TZ, 256>(f.cr, tid, gmem(J.crec) + ci * TileShape<TZ, 8>::NV,
                              gmem(J.ccode) + ci * TileShape<TZ, 8>::NC);
    }
    if (!f.vec)
        return;
    HIZ_GLOBAL const float *field = gmem(J.field);
    // piece t + 256 k: row r = t / (4 TZ) + k * 64 / TZ, z = 4 * (t % (4 TZ))
    constexpr int RS = 64 / TZ, DX = RS / kSide, DY = RS % kSide;
    int r = tid / (4 * TZ);
    int y = r % kSide, x = r / kSide;
    uint64_t off = base + (uint64_t)x * sx + (uint64_t)y * dz + 4 * (tid % (4 * TZ));
    const uint64_t d0 = DX * sx + DY * dz, dyw = sx - kSide * dz;
#pragma unroll
    for (int k = 0; k < TR::IP; k++) {
        const bool in = (k < TR::IP - 1 || tid + 256 * k < TR::NP) &&
                        (full || (x < g.ex && y < g.ey));
        f.piece[k] = gload_f4(field + (in ? off : base));
        x += DX;
        y += DY;
        off += d0;
        if (y >= kSide) {
            y -= kSide;
            x += 1;
            off += dyw;
        }
    }
    // far face: row t + 256 k, z = 16 TZ
#pragma unroll
    for (int k = 0; k < TR::IF; k++) {
        const int rr = tid + 256 * k;
        const int fy = rr % kSide, fx = rr / kSide;
        const bool in = rr < TR::NF && fx < g.ex && fy < g.ey && g.ez == TS::EZ;
        f.face[k] = field[in ? base + (uint64_t)fx * sx + (uint64_t)fy * dz + 16 * TZ : base];
    }
}

// The fetched tile into LDS (rows outside a partial tile's extent receive
// values that are never read); a tile that was not fetched loads here.
template <int TZ>
__device__ __forceinline__ void tile_place(const TileRegs<TZ> &f, float *__restrict__ v,
                                           const Job &J, uint64_t base, uint64_t sx, uint64_t dz,
                                           const Geo &g, int tid)
{
    using TS = TileShape<TZ>;
    using TR = TileRegs<TZ>;
    // LDS addresses are recomputed per tile, not kept (or spilled) across the tile loop
    asm volatile("" : "+v"(tid));
    if (f.vec) {
#pragma unroll
        for (int k = 0; k < TR::IP; k++) {
            const int i = tid + 256 * k;
            if (k < TR::IP - 1 || i < TR::NP) {
                float *p = v + (i / (4 * TZ)) * TS::PZ + 4 * (i % (4 * TZ));
                p[0] = f.piece[k].x;
                p[1] = f.piece[k].y;
                p[2] = f.piece[k].z;
                p[3] = f.piece[k].w;
            }
        }
#pragma unroll
        for (int k = 0; k < TR::IF; k++) {
            const int rr = tid + 256 * k;
            if (rr < TR::NF)
                v[rr * TS::PZ + 16 * TZ] = f.face[k];
        }
    } else {
        lds_fill_tile<TS::NV, TS::PZ, kSide, 4>(v, gmem(J.field), base, sx, dz, 1,
                                                g.ex == kSide && g.ey == kSide && g.ez == TS::EZ,
                                                g.ex, g.ey, g.ez);
        lds_fill_wait();
    }
}

// ---------------------------------------------------------------------------
// Compression: predict + quantize + histogram, persistent over tiles. Where
// the tile fits in registers, the next tile's loads are issued before this
// tile's levels run, so the levels hide their latency; otherwise each tile
// is loaded straight into LDS before its levels.
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(256, 3) void k_predict(const Job *__restrict__ jobs, int njobs,
                                                 uint64_t lo, uint64_t total, uint32_t *ctr)
{
    using TS = TileShape<TZ>;
    constexpr bool PF = kPrefetchTiles<TZ>;
    __shared__ float v[TS::NV];
    __shared__ __align__(16) uint8_t cb[TS::NC + 16]; // + a dummy slot for faces
    __shared__ uint32_t hist[256];
    __shared__ uint8_t cfg[kLevels][3];
    __shared__ QParams qp;
    __shared__ uint32_t skip;
    __shared__ uint32_t red[8];

    __shared__ uint64_t s_tile[2];

    const int t = threadIdx.x;
    hist[t] = 0;
    int cur = -1;
    // the thread index passes through an empty asm so that index arithmetic
    // of the unrolled fetches is redone per tile rather than kept in registers
    int ftid = t;
    asm volatile("" : "+v"(ftid));
    TileRegs<TZ> f;
    TileQueue tq = tile_queue(lo, total, ctr);
    uint64_t u = claim_tile(tq, s_tile, 0);
    if (PF && u < total)
        tile_fetch<TZ>(f, jobs[find_job<WK_TILE>(jobs, njobs, u)], u, ftid);
    for (int it = 1; u < total; it++) {
        // every wave is done with the previous tile's LDS past this point
        const uint64_t un = claim_tile(tq, s_tile, it);
        const int ji = find_job<WK_TILE>(jobs, njobs, u);
        const Job &J = jobs[ji];
        if (ji != cur) {
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
            lds_barrier();
        }
        if (skip) {
            if (PF && un < total)
                tile_fetch<TZ>(f, jobs[find_job<WK_TILE>(jobs, njobs, un)], un, ftid);
            u = un;
            continue;
        }
        uint64_t ox, oy, oz;
        uint32_t bx, by, bz0;
        const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
        const uint64_t dy = J.dims[1], dz = J.dims[2];
        const uint64_t sx = dy * dz, base = (ox * dy + oy) * dz + oz;
        const bool abs_mode = J.mode == 0;
        // the coarse levels of this tile ran ahead on its even-point grid
        const bool coarse = J.crec && prepass_tile<TZ>(g);
        // the tile (with its +1 faces) into LDS
        if constexpr (PF) {
            tile_place<TZ>(f, v, J, base, sx, dz, g, ftid);
        } else {
            if (coarse) {
                const uint64_t ci = ((uint64_t)bx * J.nf[1] + by) * J.nf[2] + bz0 / TZ;
                coarse_fetch<TZ, 256>(f.cr, ftid, gmem(J.crec) + ci * TileShape<TZ, 8>::NV,
                                      gmem(J.ccode) + ci * TileShape<TZ, 8>::NC);
            }
            lds_fill_tile<TS::NV, TS::PZ, kSide, 4>(v, gmem(J.field), base, sx, dz, 1,
                                                    g.ex == kSide && g.ey == kSide &&
                                                        g.ez == TS::EZ,
                                                    g.ex, g.ey, g.ez);
            lds_fill_wait();
        }
        // anchors owned by this tile: local (0, 0, 16j), stored raw from the
        // tile in LDS (the levels never write them)
        if (t < TZ && 16 * t < g.ownz)
            cb[t * 16] = 128;
        lds_barrier();
        if (abs_mode) {
            uint32_t kmn = 0xffffffffu, kmx = 0u;
            bool bad = false;
            scan_tile_values<TZ>(v, g, kmn, kmx, bad);
            if (__any(bad) && (t & 63) == 0)
                atomicOr(&J.st->flags, (uint32_t)ST_NONFINITE);
            block_minmax(kmn, kmx, red);
            if (t == 0)
                gstore_u2(gmem(J.mm_part) + (u - J.tile_begin), make_uint2(kmn, kmx));
        }
        if (coarse) {
            coarse_place<TZ, 256>(f.cr, ftid, v, cb);
            lds_barrier();
        }
        // the next tile's loads fly while this tile's levels run
        if (PF && un < total)
            tile_fetch<TZ>(f, jobs[find_job<WK_TILE>(jobs, njobs, un)], un, ftid);
        if (t < TZ && 16 * t < g.ownz) {
            const uint64_t ai = ((uint64_t)bx * J.nb[1] + by) * J.nb[2] + bz0 + t;
            const uint64_t off = J.off_anchors + 4 * ai;
            if (off + 4 <= J.cap)
                *reinterpret_cast<HIZ_GLOBAL float *>(gmem(J.stream) + off) = v[16 * t];
        }
        if (coarse)
            level<TZ, true>(v, cb, nullptr, g, 1, cfg[kLevels - 1], qp);
        else
            walk_levels<TZ, true>(v, cb, nullptr, g, cfg, qp);
        // codes of owned points -> global, histogram in LDS
        if (g.ownz == TS::OZ && (dz & 15) == 0) {
            for (int i = t; t < kStoreThreads && i < 16 * 16 * TZ; i += kStoreThreads) {
                const int w = i % TZ, r = i / TZ;
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny) {
                    const uint4 c16 = *reinterpret_cast<const uint4 *>(&cb[r * TS::OZ + 16 * w]);
                    gstore_u4(gmem(J.codes) + base + x * sx + y * dz + 16 * w, c16);
                    const uint32_t cw[4] = {c16.x, c16.y, c16.z, c16.w};
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        atomicAdd(&hist[cw[j] & 255], 1u);
                        atomicAdd(&hist[(cw[j] >> 8) & 255], 1u);
                        atomicAdd(&hist[(cw[j] >> 16) & 255], 1u);
                        atomicAdd(&hist[cw[j] >> 24], 1u);
                    }
                }
            }
        } else {
            for (int i = t; t < kStoreThreads && i < 16 * 16 * TS::OZ; i += kStoreThreads) {
                const int z = i % TS::OZ, r = i / TS::OZ;
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny && z < g.ownz) {
                    const uint8_t c = cb[r * TS::OZ + z];
                    gmem(J.codes)[base + x * sx + y * dz + z] = c;
                    atomicAdd(&hist[c], 1u);
                }
            }
        }
        u = un;
    }
    __syncthreads();
    if (cur >= 0) {
        const uint32_t h = hist[t];
        if (h)
            atomicAdd((unsigned long long *)&jobs[cur].st->hist[t], (unsigned long long)h);
    }
}

template <int TZ> static void launch_predict_t(const Job *d_jobs, int njobs, uint64_t lo,
                                              uint64_t hi, int grid, uint32_t *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_predict<TZ>, dim3(grid), dim3(256), 0, s, d_jobs, njobs, lo, hi, ctr);
}

void launch_predict(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z, int grid,
                    uint32_t *ctr, hipStream_t s)
{
    if (hi <= lo)
        return;
    if (tile_z == 1)
        launch_predict_t<1>(d_jobs, njobs, lo, hi, grid, ctr, s);
    else if (tile_z == 4)
        launch_predict_t<4>(d_jobs, njobs, lo, hi, grid, ctr, s);
    else
        launch_predict_t<2>(d_jobs, njobs, lo, hi, grid, ctr, s);
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

// A tile's codes (and anchors, and for a pre-pass tile its coarse-grid
// values) fetched into registers while the previous tile is reconstructed:
// rows of the tile as 16-byte pieces (thread t holds pieces t + 256 k, a piece
// being 16 consecutive z of one (x, y) row) and the far z face one code per
// row. Needs rows that start 16-byte aligned (dz a multiple of 16) and tiles
// that hold every piece; other tiles load their codes when placed.
template <int TZ> struct CodeRegs {
    static constexpr int NP = kSide * kSide * TZ; // pieces
    static constexpr int IP = (NP + 255) / 256;
    static constexpr int NF = kSide * kSide;
    static constexpr int IF = (NF + 255) / 256;
    static constexpr int NA = 4 * (TZ + 1); // anchors of the tile region
    uint4 piece[IP];
    uint32_t face[IF];
    float anchor;
    CoarseRegs<TZ, 256> cr;
    bool vec;
};

// whether a 32-bit word holds a zero byte
__device__ __forceinline__ bool has_zero_byte(uint32_t w)
{
    return ((w - 0x01010101u) & ~w & 0x80808080u) != 0;
}

template <int TZ>
__device__ __forceinline__ void code_fetch(CodeRegs<TZ> &f, const Job &J, uint64_t u, int tid)
{
    using TS = TileShape<TZ>;
    using CR = CodeRegs<TZ>;
    // opaque per tile: the unrolled index arithmetic is not hoisted out of the
    // tile loop into long-lived registers
    asm volatile("" : "+v"(tid));
    uint64_t ox, oy, oz;
    uint32_t bx, by, bz0;
    const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
    const uint64_t dy = J.dims[1], dz = J.dims[2];
    const uint64_t sx = dy * dz, base = (ox * dy + oy) * dz + oz;
    const bool full = g.ex == kSide && g.ey == kSide && g.ez == TS::EZ;
    if (J.crec && prepass_tile<TZ>(g)) {
        const uint64_t ci = ((uint64_t)bx * J.nf[1] + by) * J.nf[2] + bz0 / TZ;
        coarse_fetch<TZ, 256>(f.cr, tid, gmem(J.crec) + ci * TileShape<TZ, 8>::NV, nullptr);
    }
    // anchors of the tile region: every coordinate a multiple of 16
    {
        const int x = 16 * (tid & 1), y = 16 * ((tid >> 1) & 1), z = 16 * (tid >> 2);
        const bool in = tid < CR::NA && x < g.ex && y < g.ey && z < g.ez;
        const uint64_t ai = ((uint64_t)(bx + (x >> 4)) * J.nb[1] + (by + (y >> 4))) * J.nb[2] +
                            bz0 + (z >> 4);
        HIZ_GLOBAL const float *anchors =
            reinterpret_cast<HIZ_GLOBAL const float *>(gmem(J.stream) + J.off_anchors);
        f.anchor = anchors[in ? ai : 0];
    }
    f.vec = (dz & 15) == 0 && g.ez >= 16 * TZ;
    if (!f.vec)
        return;
    HIZ_GLOBAL const uint8_t *codes = gmem(J.codes);
    // piece t + 256 k: row r = t / TZ + k * 256 / TZ, z = 16 * (t % TZ)
    constexpr int RS = 256 / TZ, DX = RS / kSide, DY = RS % kSide;
    int r = tid / TZ;
    int y = r % kSide, x = r / kSide;
    uint64_t off = base + (uint64_t)x * sx + (uint64_t)y * dz + 16 * (tid % TZ);
    const uint64_t d0 = DX * sx + DY * dz, dyw = sx - kSide * dz;
#pragma unroll
    for (int k = 0; k < CR::IP; k++) {
        const bool in = (k < CR::IP - 1 || tid + 256 * k < CR::NP) &&
                        (full || (x < g.ex && y < g.ey));
        f.piece[k] = gload_u4(codes + (in ? off : base));
        x += DX;
        y += DY;
        off += d0;
        if (y >= kSide) {
            y -= kSide;
            x += 1;
            off += dyw;
        }
    }
#pragma unroll
    for (int k = 0; k < CR::IF; k++) {
        const int rr = tid + 256 * k;
        const int fy = rr % kSide, fx = rr / kSide;
        const bool in = rr < CR::NF && fx < g.ex && fy < g.ey && g.ez == TS::EZ;
        f.face[k] = codes[in ? base + (uint64_t)fx * sx + (uint64_t)fy * dz + 16 * TZ : base];
    }
}

// The fetched codes into LDS and the anchors into the value tile; returns
// whether this thread saw a zero code (a possible outlier). A tile that was
// not fetched loads its codes here.
template <int TZ>
__device__ __forceinline__ bool code_place(const CodeRegs<TZ> &f, uint8_t *__restrict__ cl,
                                           float *__restrict__ v, const Job &J, uint64_t base,
                                           uint64_t sx, uint64_t dz, const Geo &g, int tid)
{
    using TS = TileShape<TZ>;
    using CR = CodeRegs<TZ>;
    if (tid < CR::NA) {
        const int x = 16 * (tid & 1), y = 16 * ((tid >> 1) & 1), z = 16 * (tid >> 2);
        if (x < g.ex && y < g.ey && z < g.ez)
            v[x * TS::PX + y * TS::PZ + z] = f.anchor;
    }
    if (!f.vec) {
        load_tile_codes<TZ>(cl, gmem(J.codes), base, sx, dz, g);
        return true;
    }
    bool zero = false;
#pragma unroll
    for (int k = 0; k < CR::IP; k++) {
        const int i = tid + 256 * k;
        if (k < CR::IP - 1 || i < CR::NP) {
            uint8_t *p = cl + (i / TZ) * TS::PZ + 16 * (i % TZ);
            const uint32_t w[4] = {f.piece[k].x, f.piece[k].y, f.piece[k].z, f.piece[k].w};
#pragma unroll
            for (int j = 0; j < 16; j++)
                p[j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
            zero |= has_zero_byte(w[0]) | has_zero_byte(w[1]) | has_zero_byte(w[2]) |
                    has_zero_byte(w[3]);
        }
    }
#pragma unroll
    for (int k = 0; k < CR::IF; k++) {
        const int rr = tid + 256 * k;
        if (rr < CR::NF) {
            cl[rr * TS::PZ + 16 * TZ] = (uint8_t)f.face[k];
            zero |= (f.face[k] & 255u) == 0;
        }
    }
    return zero;
}

// ---------------------------------------------------------------------------
// Decompression: rebuild the tile from codes, anchors and outliers,
// persistent over tiles; the next tile's codes are fetched into registers
// before this tile's levels run, so the levels hide their latency.
// ---------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(256, 3) void k_reconstruct(const Job *__restrict__ jobs, int njobs,
                                                     uint64_t lo, uint64_t total, uint32_t *ctr)
{
    using TS = TileShape<TZ>;
    __shared__ float v[TS::NV];
    __shared__ uint8_t cl[TS::NV];
    __shared__ uint8_t cfg[kLevels][3];
    __shared__ QParams qp;
    __shared__ uint64_t s_tile[2];
    __shared__ uint32_t s_zero;

    const int t = threadIdx.x;
    int cur = -1;
    int ftid = t;
    asm volatile("" : "+v"(ftid));
    CodeRegs<TZ> f;
    TileQueue tq = tile_queue(lo, total, ctr);
    uint64_t u = claim_tile(tq, s_tile, 0);
    if (u < total)
        code_fetch<TZ>(f, jobs[find_job<WK_TILE>(jobs, njobs, u)], u, ftid);
    for (int it = 1; u < total; it++) {
        // every wave is done with the previous tile's LDS past this point
        const uint64_t un = claim_tile(tq, s_tile, it);
        const int ji = find_job<WK_TILE>(jobs, njobs, u);
        const Job &J = jobs[ji];
        if (ji != cur) {
            if (t == 0) {
                qp.eps = J.st->eps;
                qp.two_eb = J.st->two_eb;
                qp.inv = 0.f;
            }
            if (t < kLevels * 3)
                cfg[t / 3][t % 3] = J.st->cfg[t / 3][t % 3];
            cur = ji;
        }
        if (t == 0)
            s_zero = 0;
        uint64_t ox, oy, oz;
        uint32_t bx, by, bz0;
        const Geo g = tile_geometry<TZ>(J, u - J.tile_begin, ox, oy, oz, bx, by, bz0);
        const uint64_t dy = J.dims[1], dz = J.dims[2];
        const uint64_t sx = dy * dz, base = (ox * dy + oy) * dz + oz;
        const bool coarse = J.crec && prepass_tile<TZ>(g);
        lds_barrier();
        const bool zero = code_place<TZ>(f, cl, v, J, base, sx, dz, g, ftid);
        if (__any(zero) && (t & 63) == 0)
            s_zero = 1;
        lds_barrier();
        // outliers (code 0, anchors excluded): their exact values were
        // scattered into the output beforehand; only tiles holding a zero code
        // look, 8 loads per thread in flight
        if (s_zero) {
            constexpr int NE = TS::NV;
#pragma nounroll
            for (int i0 = 0; i0 < NE; i0 += 256 * 8) {
                float ov[8];
                bool hit[8];
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const int e = i0 + t + 256 * k;
                    const int z = e % TS::PZ, r = e / TS::PZ;
                    const int y = r % kSide, x = r / kSide;
                    hit[k] = e < NE && x < g.ex && y < g.ey && z < g.ez && cl[e] == 0 &&
                             !((x & 15) == 0 && (y & 15) == 0 && (z & 15) == 0);
                    ov[k] = hit[k] ? gmem(J.out)[base + (uint64_t)x * sx + (uint64_t)y * dz + z]
                                   : 0.f;
                }
#pragma unroll
                for (int k = 0; k < 8; k++)
                    if (hit[k])
                        v[i0 + t + 256 * k] = ov[k];
            }
            lds_barrier();
        }
        if (coarse) {
            coarse_place<TZ, 256>(f.cr, ftid, v, nullptr);
            lds_barrier();
        }
        // the next tile's loads fly while this tile's levels run
        if (un < total)
            code_fetch<TZ>(f, jobs[find_job<WK_TILE>(jobs, njobs, un)], un, ftid);
        if (coarse)
            level<TZ, false>(v, nullptr, cl, g, 1, cfg[kLevels - 1], qp);
        else
            walk_levels<TZ, false>(v, nullptr, cl, g, cfg, qp);
        if (g.ownz == TS::OZ && (dz & 3) == 0 && (reinterpret_cast<uintptr_t>(J.out) & 15) == 0) {
            for (int i = t; t < kStoreThreads && i < 16 * 16 * 4 * TZ; i += kStoreThreads) {
                const int w = i % (4 * TZ), r = i / (4 * TZ);
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny) {
                    const float *vp = v + x * TS::PX + y * TS::PZ + 4 * w;
                    gstore_f4(gmem(J.out) + base + (uint64_t)x * sx + (uint64_t)y * dz + 4 * w,
                              make_float4(vp[0], vp[1], vp[2], vp[3]));
                }
            }
        } else {
            for (int i = t; t < kStoreThreads && i < 16 * 16 * TS::OZ; i += kStoreThreads) {
                const int z = i % TS::OZ, r = i / TS::OZ;
                const int y = r % 16, x = r / 16;
                if (x < g.ownx && y < g.owny && z < g.ownz)
                    gmem(J.out)[base + (uint64_t)x * sx + (uint64_t)y * dz + z] =
                        v[x * TS::PX + y * TS::PZ + z];
            }
        }
        u = un;
    }
}

template <int TZ> static void launch_reconstruct_t(const Job *d_jobs, int njobs, uint64_t lo,
                                                  uint64_t hi, int grid, uint32_t *ctr,
                                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_reconstruct<TZ>, dim3(grid), dim3(256), 0, s, d_jobs, njobs, lo, hi, ctr);
}

void launch_reconstruct(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z,
                        int grid, uint32_t *ctr, hipStream_t s)
{
    if (hi <= lo)
        return;
    if (tile_z == 1)
        launch_reconstruct_t<1>(d_jobs, njobs, lo, hi, grid, ctr, s);
    else if (tile_z == 4)
        launch_reconstruct_t<4>(d_jobs, njobs, lo, hi, grid, ctr, s);
    else
        launch_reconstruct_t<2>(d_jobs, njobs, lo, hi, grid, ctr, s);
}

// ---------------------------------------------------------------------------
// Coarse levels (strides 8, 4, 2) of every tile whose owned points all lie in
// the field, one wave per tile, on the tile's grid of even points: up to
// 9 x 9 x (8 TZ + 1) values, the same computation as in the full tile at half
// the coordinates (strides 4, 2, 1); a line's samples exist in the half grid
// exactly when they exist in the full one.
// Many tiles per CU are in flight at once, so the serial chain of nine
// sub-steps per tile overlaps across tiles instead of holding a full tile's
// LDS. The results (values, and codes of the owned points for compression)
// go to per-tile workspace slots for k_predict / k_reconstruct to overlay.
// Tiles cut short inside their owned points are left to the full kernels,
// which run all four levels.
// ---------------------------------------------------------------------------
template <int TZ, bool COMP>
__global__ __launch_bounds__(64) void k_coarse(const Job *__restrict__ jobs, int njobs,
                                               uint64_t lo, uint64_t total)
{
    using TC = TileShape<TZ, 8>;
    constexpr int IV = (TC::NV + 63) / 64;
    __shared__ float v[TC::NV];
    __shared__ __align__(16) uint8_t cb[TC::NC + 16];
    __shared__ uint8_t cl[COMP ? 1 : TC::NV];
    __shared__ uint8_t cfg[kLevels][3];
    __shared__ QParams qp;
    const int t = threadIdx.x;
    // tiles from the end of the list first: those cut by the field's far
    // faces (slower, general line code) gather there and start early rather
    // than form the launch's tail
    for (uint64_t w = blockIdx.x; w < total - lo; w += gridDim.x) {
        const uint64_t u = total - 1 - w;
        const Job &J = jobs[find_job<WK_TILE>(jobs, njobs, u)];
        const FieldState *st = J.st;
        if (COMP && (st->flags & (ST_CONST | ST_NONFINITE)))
            continue;
        uint64_t ox, oy, oz;
        uint32_t bx, by, bz0;
        const uint64_t lt = u - J.tile_begin;
        const Geo gf = tile_geometry<TZ>(J, lt, ox, oy, oz, bx, by, bz0);
        if (!prepass_tile<TZ>(gf))
            continue;
        // the even-point grid: extents 8 or 9 per axis (8 TZ or 8 TZ + 1 along
        // z), every owned point inside
        const Geo gc = {(gf.ex + 1) / 2, (gf.ey + 1) / 2, (gf.ez + 1) / 2, 8, 8, TC::OZ};
        const bool cfull = gc.ex == TC::SIDE && gc.ey == TC::SIDE && gc.ez == TC::EZ;
        __syncthreads();
        if (t == 0) {
            qp.eps = st->eps;
            qp.two_eb = st->two_eb;
            qp.inv = COMP ? st->inv : 0.f;
        }
        if (t < kLevels * 3)
            cfg[t / 3][t % 3] = st->cfg[t / 3][t % 3];
        const uint64_t dy = J.dims[1], dz = J.dims[2];
        auto gidx = [&](int i) -> uint64_t {
            const int zc = i % TC::PZ, r = i / TC::PZ;
            const int yc = r % TC::SIDE, xc = r / TC::SIDE;
            return ((ox + 2 * xc) * dy + (oy + 2 * yc)) * dz + oz + 2 * zc;
        };
        // the lane index is opaque so its arithmetic is not kept across tiles
        int tid = t;
        asm volatile("" : "+v"(tid));
        constexpr int B = 8;
        if constexpr (COMP) {
            // the even points straight into LDS, all in flight at once
            lds_fill_tile<TC::NV, TC::PZ, TC::SIDE, 1>(v, gmem(J.field), (ox * dy + oy) * dz + oz,
                                                       2 * dy * dz, 2 * dz, 2, cfull, gc.ex, gc.ey,
                                                       gc.ez);
            if (t < TZ)
                cb[8 * t] = 128; // anchors (0, 0, 8j)
        } else {
            // codes; anchors from the stream; outliers scattered into the output
            HIZ_GLOBAL const uint8_t *codes = gmem(J.codes);
            HIZ_GLOBAL const float *out = gmem(J.out);
            HIZ_GLOBAL const float *anchors =
                reinterpret_cast<HIZ_GLOBAL const float *>(gmem(J.stream) + J.off_anchors);
#pragma nounroll
            for (int i0 = 0; i0 < TC::NV; i0 += 64 * B) {
                uint32_t c[B];
#pragma unroll
                for (int k = 0; k < B; k++) {
                    const int i = i0 + tid + 64 * k;
                    const int zc = i % TC::PZ, r = i / TC::PZ;
                    const int yc = r % TC::SIDE, xc = r / TC::SIDE;
                    const bool in = i < TC::NV && xc < gc.ex && yc < gc.ey && zc < gc.ez;
                    c[k] = codes[gidx(in ? i : 0)];
                }
                float ov[B];
#pragma unroll
                for (int k = 0; k < B; k++) {
                    const int i = i0 + tid + 64 * k;
                    const int zc = i % TC::PZ, r = i / TC::PZ;
                    const int yc = r % TC::SIDE, xc = r / TC::SIDE;
                    const bool in = i < TC::NV && xc < gc.ex && yc < gc.ey && zc < gc.ez;
                    const bool anchor = (xc & 7) == 0 && (yc & 7) == 0 && (zc & 7) == 0;
                    const uint64_t ai = ((uint64_t)(bx + (xc >> 3)) * J.nb[1] + (by + (yc >> 3))) *
                                            J.nb[2] +
                                        bz0 + (zc >> 3);
                    ov[k] = 0.f;
                    if (in && anchor)
                        ov[k] = anchors[ai];
                    else if (in && c[k] == 0)
                        ov[k] = out[gidx(i)];
                }
#pragma unroll
                for (int k = 0; k < B; k++) {
                    const int i = i0 + tid + 64 * k;
                    if (i < TC::NV) {
                        cl[i] = (uint8_t)c[k];
                        v[i] = ov[k];
                    }
                }
            }
        }
        lds_fill_wait();
        __syncthreads();
#pragma unroll 1
        for (int l = 0; l < kLevels - 1; l++) {
            if constexpr (COMP)
                level<TZ, true, 8>(v, cb, nullptr, gc, 4 >> l, cfg[l], qp);
            else
                level<TZ, false, 8>(v, nullptr, cl, gc, 4 >> l, cfg[l], qp);
        }
        const uint64_t ci = ((uint64_t)bx * J.nf[1] + by) * J.nf[2] + bz0 / TZ;
        HIZ_GLOBAL float *crec = gmem(J.crec) + ci * TC::NV;
        for (int i = t; i < TC::NV; i += 64)
            crec[i] = v[i];
        if constexpr (COMP) {
            HIZ_GLOBAL uint8_t *cc = gmem(J.ccode) + ci * TC::NC;
            for (int i = t; i < TC::NC / 16; i += 64)
                gstore_u4(cc + 16 * i, *reinterpret_cast<const uint4 *>(&cb[16 * i]));
        }
    }
}

template <int TZ>
static void launch_coarse_t(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, bool compress,
                            hipStream_t s)
{
    const uint64_t n = hi - lo;
    const uint32_t g = (uint32_t)(n < (1u << 30) ? n : (1u << 30));
    if (compress)
        hipLaunchKernelGGL((k_coarse<TZ, true>), dim3(g), dim3(64), 0, s, d_jobs, njobs, lo, hi);
    else
        hipLaunchKernelGGL((k_coarse<TZ, false>), dim3(g), dim3(64), 0, s, d_jobs, njobs, lo, hi);
}

void launch_coarse(const Job *d_jobs, int njobs, uint64_t lo, uint64_t hi, int tile_z,
                   bool compress, hipStream_t s)
{
    if (hi <= lo)
        return;
    if (tile_z == 1)
        launch_coarse_t<1>(d_jobs, njobs, lo, hi, compress, s);
    else if (tile_z == 4)
        launch_coarse_t<4>(d_jobs, njobs, lo, hi, compress, s);
    else
        launch_coarse_t<2>(d_jobs, njobs, lo, hi, compress, s);
}

uint64_t coarse_values_per_tile(int tile_z)
{
    return tile_z == 1 ? TileShape<1, 8>::NV : (tile_z == 4 ? TileShape<4, 8>::NV : TileShape<2, 8>::NV);
}

uint64_t coarse_codes_per_tile(int tile_z)
{
    return tile_z == 1 ? TileShape<1, 8>::NC : (tile_z == 4 ? TileShape<4, 8>::NC : TileShape<2, 8>::NC);
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
