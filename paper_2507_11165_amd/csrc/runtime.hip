// Host runtime of the hiz library: context and device workspace, job
// descriptors, the launch sequence of compression and decompression, stream
// header parsing, per-kernel profiling, and the C ABI declared in hiz.h.
#include "hiz.h"
#include "hiz_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace hiz;

namespace {

constexpr uint64_t kMaxN = 1ull << 40;

struct KStat {
    std::string name;
    uint64_t launches = 0;
    double ms = 0.0;
};

struct Pending {
    int stat;
    hipEvent_t a, b;
};

} // namespace

struct hiz_ctx {
    int device = 0;
    int cus = 0;
    void *ws = nullptr;
    size_t ws_size = 0;
    uint8_t *pinned = nullptr;
    size_t pinned_size = 0;
    std::string err;
    bool profiling = false;
    std::vector<KStat> stats;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> events;
    size_t next_event = 0;
    int pred_bpc[5] = {0, 0, 0, 0, 0};
    int rec_bpc[5] = {0, 0, 0, 0, 0};
    int enc_bpc = 0;
};

namespace {

hiz_status fail(hiz_ctx *c, hiz_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    return st;
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((ctx), HIZ_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

uint64_t pow2ceil(uint64_t v)
{
    uint64_t p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

int ilog2(uint64_t v)
{
    int l = 0;
    while ((1ull << l) < v)
        l++;
    return l;
}

// Huffman chunk length keyed by field size: enough chunks to keep every
// decoder lane busy, never below 256 or above 1024 symbols.
uint32_t default_chunk(uint64_t N)
{
    uint64_t c = pow2ceil(cdiv(N, 131072));
    return (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(256, c));
}

constexpr int kDefaultTileZ = 2;

// ---- profiling ----
hipEvent_t take_event(hiz_ctx *c)
{
    if (c->next_event == c->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        c->events.push_back(e);
    }
    return c->events[c->next_event++];
}

int stat_index(hiz_ctx *c, const char *name)
{
    for (size_t i = 0; i < c->stats.size(); i++)
        if (c->stats[i].name == name)
            return (int)i;
    KStat k;
    k.name = name;
    c->stats.push_back(k);
    return (int)c->stats.size() - 1;
}

struct Scope {
    hiz_ctx *c;
    hipStream_t s;
    Pending p;
    bool on;
    Scope(hiz_ctx *c_, hipStream_t s_, const char *name) : c(c_), s(s_), on(c_->profiling)
    {
        if (on) {
            p.stat = stat_index(c, name);
            p.a = take_event(c);
            p.b = take_event(c);
            on = p.a && p.b;
            if (on)
                hipEventRecord(p.a, s);
        }
    }
    ~Scope()
    {
        if (on) {
            hipEventRecord(p.b, s);
            c->pending.push_back(p);
        }
    }
};

void collect_profile(hiz_ctx *c)
{
    for (const Pending &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->stats[p.stat].launches++;
            c->stats[p.stat].ms += ms;
        }
    }
    c->pending.clear();
    c->next_event = 0;
}

// ---- workspace ----
struct Arena {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes)
    {
        uint64_t o = (off + 255) & ~uint64_t(255);
        off = o + bytes;
        return o;
    }
};

hiz_status ensure_ws(hiz_ctx *c, uint64_t bytes)
{
    if (bytes <= c->ws_size)
        return HIZ_OK;
    if (c->ws) {
        hipDeviceSynchronize();
        hipFree(c->ws);
        c->ws = nullptr;
        c->ws_size = 0;
    }
    uint64_t want = bytes + bytes / 8 + (1u << 20);
    if (hipMalloc(&c->ws, want) != hipSuccess) {
        c->ws = nullptr;
        hipGetLastError();
        return fail(c, HIZ_ERR_NOMEM, "cannot allocate %llu bytes of device workspace",
                    (unsigned long long)want);
    }
    c->ws_size = want;
    return HIZ_OK;
}

hiz_status ensure_pinned(hiz_ctx *c, uint64_t bytes)
{
    if (bytes <= c->pinned_size)
        return HIZ_OK;
    if (c->pinned)
        hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_size = 0;
    uint64_t want = std::max<uint64_t>(bytes, 64 * 1024);
    if (hipHostMalloc((void **)&c->pinned, want, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        hipGetLastError();
        return fail(c, HIZ_ERR_NOMEM, "cannot allocate %llu bytes of pinned memory",
                    (unsigned long long)want);
    }
    c->pinned_size = want;
    return HIZ_OK;
}

bool debug_on()
{
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("HIZ_DEBUG");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}

int predict_grid(hiz_ctx *c, int tz, uint64_t total, bool rec)
{
    int *cache = rec ? c->rec_bpc : c->pred_bpc;
    if (!cache[tz]) {
        cache[tz] = rec ? reconstruct_blocks_per_cu(tz) : predict_blocks_per_cu(tz);
        if (debug_on())
            fprintf(stderr, "[hiz] %s tile_z=%d: %d CUs x %d workgroups per CU\n",
                    rec ? "reconstruct" : "predict", tz, c->cus, cache[tz]);
    }
    uint64_t g = (uint64_t)c->cus * cache[tz];
    if (g >= 8)
        g &= ~uint64_t(7);
    if (total < g)
        g = total;
    return (int)std::max<uint64_t>(1, g);
}

// ---- header parsing (host) ----
template <typename T> T get_le(const uint8_t *p)
{
    T v;
    memcpy(&v, p, sizeof(T));
    return v;
}

struct Parsed {
    hiz_info info;
    uint64_t N;
    int idx_bytes;
    uint64_t off_anchors, off_oidx, off_oval, off_payload;
    float const_value;
};

hiz_status parse_header(hiz_ctx *c, const uint8_t *h, uint64_t n, uint64_t in_size, Parsed *P)
{
    memset(P, 0, sizeof(*P));
    hiz_info &I = P->info;
    if (n < (uint64_t)kHdrBytes || in_size < (uint64_t)kHdrBytes)
        return fail(c, HIZ_ERR_CORRUPT, "stream shorter than its header");
    if (get_le<uint32_t>(h + H_MAGIC) != kMagic || get_le<uint16_t>(h + H_VERSION) != kVersion)
        return fail(c, HIZ_ERR_CORRUPT, "bad magic or version");
    I.mode = h[H_MODE];
    const uint8_t flags = h[H_FLAGS];
    if (I.mode > 1 || (flags & ~3))
        return fail(c, HIZ_ERR_CORRUPT, "bad mode or flags");
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        I.dims[k] = get_le<uint64_t>(h + H_DIMS + 8 * k);
        if (I.dims[k] == 0 || I.dims[k] > kMaxN)
            return fail(c, HIZ_ERR_CORRUPT, "bad dims");
        if (N > kMaxN / I.dims[k])
            return fail(c, HIZ_ERR_CORRUPT, "field too large");
        N *= I.dims[k];
    }
    P->N = N;
    I.eb = get_le<double>(h + H_EB);
    I.eps = get_le<float>(h + H_EPS);
    I.vmin = get_le<float>(h + H_MIN);
    I.vmax = get_le<float>(h + H_MAX);
    I.total_bytes = get_le<uint64_t>(h + H_TOTAL);
    if (flags & kFlagConst) {
        I.constant = 1;
        if (I.total_bytes != kHdrBytes + 4u || in_size < I.total_bytes)
            return fail(c, HIZ_ERR_CORRUPT, "bad constant stream");
        if (n >= kHdrBytes + 4u)
            P->const_value = get_le<float>(h + kHdrBytes);
        return HIZ_OK;
    }
    if (h[H_ASTRIDE] != kAnchor || h[H_NLEV] != kLevels)
        return fail(c, HIZ_ERR_CORRUPT, "bad anchor stride or level count");
    for (int l = 0; l < kLevels; l++) {
        for (int k = 0; k < 3; k++)
            I.level_cfg[l][k] = h[H_CFG + 3 * l + k];
        if (I.level_cfg[l][0] > 1 || I.level_cfg[l][1] > 1 || I.level_cfg[l][2] > 5)
            return fail(c, HIZ_ERR_CORRUPT, "bad level configuration");
    }
    I.chunk = get_le<uint32_t>(h + H_CHUNK);
    if (I.chunk < 256 || I.chunk > 65536 || (I.chunk & (I.chunk - 1)))
        return fail(c, HIZ_ERR_CORRUPT, "bad chunk length");
    I.n_outliers = get_le<uint64_t>(h + H_NOUT);
    I.payload_words = get_le<uint64_t>(h + H_PWORDS);
    I.n_chunks = get_le<uint64_t>(h + H_NCHUNKS);
    const uint64_t n_anchors = get_le<uint64_t>(h + H_NANCH);
    P->idx_bytes = N < (1ull << 32) ? 4 : 8;
    if (((flags & kFlagIdx64) != 0) != (P->idx_bytes == 8))
        return fail(c, HIZ_ERR_CORRUPT, "bad index width flag");
    if (I.n_chunks != cdiv(N, I.chunk))
        return fail(c, HIZ_ERR_CORRUPT, "bad chunk count");
    if (n_anchors != cdiv(I.dims[0], kAnchor) * cdiv(I.dims[1], kAnchor) * cdiv(I.dims[2], kAnchor))
        return fail(c, HIZ_ERR_CORRUPT, "bad anchor count");
    if (I.n_outliers > N || I.payload_words > N + I.n_chunks)
        return fail(c, HIZ_ERR_CORRUPT, "bad outlier or payload size");
    P->off_anchors = align16(kOffChunks + 4 * I.n_chunks);
    P->off_oidx = align16(P->off_anchors + 4 * n_anchors);
    P->off_oval = align16(P->off_oidx + (uint64_t)P->idx_bytes * I.n_outliers);
    P->off_payload = align16(P->off_oval + 4 * I.n_outliers);
    if (I.total_bytes != P->off_payload + 4 * I.payload_words || I.total_bytes > in_size)
        return fail(c, HIZ_ERR_CORRUPT, "stream size does not match its header");
    if (n >= (uint64_t)kOffChunks) {
        // the code lengths must form a complete prefix code (one symbol: length 1)
        const uint8_t *len = h + kOffLen;
        uint64_t kraft = 0; // in units of 2^-32
        int nsym = 0;
        for (int i = 0; i < 256; i++) {
            if (!len[i])
                continue;
            if (len[i] > kMaxCodeLen)
                return fail(c, HIZ_ERR_CORRUPT, "code length above 32");
            kraft += 1ull << (32 - len[i]);
            nsym++;
        }
        if (nsym == 0 || (nsym == 1 && kraft != (1ull << 31)) || (nsym > 1 && kraft != (1ull << 32)))
            return fail(c, HIZ_ERR_CORRUPT, "code lengths do not form a complete prefix code");
    }
    return HIZ_OK;
}

bool valid_cfg(const uint8_t cfg[4][3])
{
    for (int l = 0; l < 4; l++)
        if (cfg[l][0] > 1 || cfg[l][1] > 1 || cfg[l][2] > 5)
            return false;
    return true;
}

} // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

hiz_status hiz_create(int device, size_t workspace_bytes, hiz_ctx **out)
{
    if (!out)
        return HIZ_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        hipGetLastError();
        return HIZ_ERR_ARG;
    }
    hiz_ctx *c = new (std::nothrow) hiz_ctx();
    if (!c)
        return HIZ_ERR_NOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess) {
        delete c;
        return HIZ_ERR_HIP;
    }
    if (workspace_bytes && ensure_ws(c, workspace_bytes) != HIZ_OK) {
        delete c;
        return HIZ_ERR_NOMEM;
    }
    if (ensure_pinned(c, 64 * 1024) != HIZ_OK) {
        hipFree(c->ws);
        delete c;
        return HIZ_ERR_NOMEM;
    }
    *out = c;
    return HIZ_OK;
}

void hiz_destroy(hiz_ctx *c)
{
    if (!c)
        return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (hipEvent_t e : c->events)
        hipEventDestroy(e);
    if (c->ws)
        hipFree(c->ws);
    if (c->pinned)
        hipHostFree(c->pinned);
    delete c;
}

const char *hiz_last_error(const hiz_ctx *c) { return c ? c->err.c_str() : "no context"; }

uint64_t hiz_compress_bound(const uint64_t dims[3])
{
    if (!dims)
        return 0;
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        if (dims[k] == 0 || dims[k] > kMaxN || N > kMaxN / dims[k])
            return 0;
        N *= dims[k];
    }
    const uint64_t chunks = cdiv(N, 256);
    const uint64_t anchors = cdiv(dims[0], kAnchor) * cdiv(dims[1], kAnchor) * cdiv(dims[2], kAnchor);
    // header, lengths, chunk table, anchors, outlier indices (8 B) and values,
    // payload of 32-bit codewords plus one padding word per chunk, section gaps
    return kOffChunks + 4 * chunks + 4 * anchors + 12 * N + 4 * (N + chunks) + 64;
}

void hiz_set_profiling(hiz_ctx *c, int on)
{
    if (c)
        c->profiling = on != 0;
}

int hiz_get_profile(hiz_ctx *c, hiz_kernel_stat *out, int max)
{
    if (!c)
        return 0;
    for (int i = 0; i < max && i < (int)c->stats.size(); i++) {
        memset(&out[i], 0, sizeof(out[i]));
        strncpy(out[i].name, c->stats[i].name.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = c->stats[i].launches;
        out[i].total_ms = c->stats[i].ms;
    }
    return (int)c->stats.size();
}

void hiz_reset_profile(hiz_ctx *c)
{
    if (c)
        c->stats.clear();
}

hiz_status hiz_compress(hiz_ctx *c, const float *d_field, const uint64_t dims[3],
                        hiz_eb_mode mode, double eb, const hiz_params *params, void *d_out,
                        uint64_t out_cap, uint64_t *out_size, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    c->err.clear();
    if (!d_field || !dims || !d_out || !out_size)
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    *out_size = 0;
    if (mode != HIZ_ABS && mode != HIZ_REL)
        return fail(c, HIZ_ERR_ARG, "bad error-bound mode");
    if (!(eb > 0.0) || !std::isfinite(eb))
        return fail(c, HIZ_ERR_ARG, "error bound must be finite and positive");
    if ((reinterpret_cast<uintptr_t>(d_field) & 3) || (reinterpret_cast<uintptr_t>(d_out) & 15))
        return fail(c, HIZ_ERR_ARG, "field must be 4-byte and stream 16-byte aligned");
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        if (dims[k] == 0 || dims[k] > kMaxN || N > kMaxN / dims[k])
            return fail(c, HIZ_ERR_ARG, "bad dims");
        N *= dims[k];
    }
    hiz_params p;
    memset(&p, 0, sizeof(p));
    p.tune = 1;
    for (int l = 0; l < 4; l++)
        p.level_cfg[l][0] = HIZ_SPLINE_CUBIC;
    if (params)
        p = *params;
    if (!valid_cfg(p.level_cfg))
        return fail(c, HIZ_ERR_ARG, "bad level configuration");
    uint32_t chunk = p.chunk ? p.chunk : default_chunk(N);
    if (chunk < 256 || chunk > 65536 || (chunk & (chunk - 1)))
        return fail(c, HIZ_ERR_ARG, "chunk must be a power of two in [256, 65536]");
    int tz = p.tile_z ? (int)p.tile_z : kDefaultTileZ;
    if (tz != 1 && tz != 2 && tz != 4)
        return fail(c, HIZ_ERR_ARG, "tile_z must be 1, 2 or 4");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));

    Job J;
    memset(&J, 0, sizeof(J));
    J.field = d_field;
    J.stream = static_cast<uint8_t *>(d_out);
    J.cap = out_cap;
    for (int k = 0; k < 3; k++) {
        J.dims[k] = dims[k];
        J.nb[k] = (uint32_t)cdiv(dims[k], kAnchor);
        J.n_full[k] = dims[k] >= (uint64_t)kSide ? (uint32_t)((dims[k] - kSide) / kAnchor + 1) : 0;
    }
    J.N = N;
    J.ntz = (uint32_t)cdiv(J.nb[2], tz);
    J.n_anchors = (uint64_t)J.nb[0] * J.nb[1] * J.nb[2];
    J.chunk = chunk;
    J.log2_chunk = (uint32_t)ilog2(chunk);
    J.n_chunks = cdiv(N, chunk);
    J.off_anchors = align16(kOffChunks + 4 * J.n_chunks);
    J.mode = mode;
    J.tune = p.tune ? 1 : 0;
    J.eb = eb;
    memcpy(J.cfg_forced, p.level_cfg, sizeof(J.cfg_forced));
    J.idx_bytes = N < (1ull << 32) ? 4 : 8;
    J.n_mm = mode == HIZ_REL ? cdiv(N, 16384) : 0;
    const uint64_t n_full = (uint64_t)J.n_full[0] * J.n_full[1] * J.n_full[2];
    if (J.tune && n_full > 0) {
        uint64_t ns = std::max<uint64_t>(1, cdiv(2 * N, 1000ull * 4913ull));
        J.n_samples = (uint32_t)std::min<uint64_t>(ns, n_full);
    }
    J.n_tune = (uint64_t)J.n_samples * 9;
    J.n_tiles = (uint64_t)J.nb[0] * J.nb[1] * J.ntz;

    Arena A;
    const uint64_t o_job = A.take(sizeof(Job));
    const uint64_t o_st = A.take(sizeof(FieldState));
    const uint64_t o_cnt = A.take(sizeof(Counters));
    const uint64_t o_codes = A.take(N);
    J.n_groups = cdiv(J.n_chunks, kEncGroupChunks);
    const uint64_t o_lba = A.take(8 * J.n_groups);
    const uint64_t o_lbb = A.take(8 * J.n_groups);
    const uint64_t o_woff = A.take(8 * J.n_chunks);
    const uint64_t o_zoff = A.take(8 * J.n_chunks);
    const uint64_t o_mm = A.take(8 * std::max<uint64_t>(J.n_mm, J.n_tiles));
    hiz_status rc = ensure_ws(c, A.off);
    if (rc)
        return rc;
    rc = ensure_pinned(c, sizeof(Job) + kResultBytes + 256);
    if (rc)
        return rc;
    uint8_t *ws = static_cast<uint8_t *>(c->ws);
    J.st = reinterpret_cast<FieldState *>(ws + o_st);
    J.codes = ws + o_codes;
    J.lb_a = reinterpret_cast<uint64_t *>(ws + o_lba);
    J.lb_b = reinterpret_cast<uint64_t *>(ws + o_lbb);
    J.mm_part = reinterpret_cast<uint2 *>(ws + o_mm);
    J.woff = reinterpret_cast<uint64_t *>(ws + o_woff);
    J.zoff = reinterpret_cast<uint64_t *>(ws + o_zoff);
    Job *d_job = reinterpret_cast<Job *>(ws + o_job);
    Counters *d_cnt = reinterpret_cast<Counters *>(ws + o_cnt);
    memcpy(c->pinned, &J, sizeof(J));
    uint8_t *h_res = c->pinned + ((sizeof(Job) + 255) & ~size_t(255));

    HIP_TRY(c, hipMemcpyAsync(d_job, c->pinned, sizeof(Job), hipMemcpyHostToDevice, s));
    {
        Scope sc(c, s, "init");
        launch_init_compress(d_job, 1, J.n_groups, d_cnt, s);
    }
    if (J.n_mm) {
        Scope sc(c, s, "minmax");
        launch_minmax(d_job, 1, J.n_mm, c->cus * 8, s);
    }
    {
        Scope sc(c, s, "eps");
        launch_eps(d_job, 1, s);
    }
    if (J.n_tune) {
        Scope sc(c, s, "tune");
        launch_tune(d_job, 1, J.n_tune, s);
    }
    {
        Scope sc(c, s, "tune_pick");
        launch_tune_pick(d_job, 1, s);
    }
    {
        Scope sc(c, s, "predict_quant");
        launch_predict(d_job, 1, J.n_tiles, tz, predict_grid(c, tz, J.n_tiles, false), s);
    }
    {
        Scope sc(c, s, "codebook");
        launch_codebook(d_job, 1, s);
    }
    {
        if (!c->enc_bpc) {
            c->enc_bpc = encode_blocks_per_cu();
            if (debug_on())
                fprintf(stderr, "[hiz] encode: %d CUs x %d workgroups per CU\n", c->cus,
                        c->enc_bpc);
        }
        Scope sc(c, s, "encode");
        launch_encode(d_job, 1, J.n_chunks, J.n_groups, d_cnt, c->cus * c->enc_bpc, s);
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(h_res, J.st, kResultBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->profiling)
        collect_profile(c);
    FieldState res;
    memcpy(&res, h_res, kResultBytes);
    if (res.flags & ST_NONFINITE)
        return fail(c, HIZ_ERR_NONFINITE, "field holds NaN or Inf");
    if (res.flags & ST_CORRUPT)
        return fail(c, HIZ_ERR_HIP, "internal consistency check failed");
    *out_size = res.total_bytes;
    if ((res.flags & ST_OVERFLOW) || res.total_bytes > out_cap)
        return fail(c, HIZ_ERR_BUFSZ, "output needs %llu bytes, capacity is %llu",
                    (unsigned long long)res.total_bytes, (unsigned long long)out_cap);
    return HIZ_OK;
}

hiz_status hiz_inspect(const void *h_stream, uint64_t n, hiz_info *out)
{
    if (!h_stream || !out)
        return HIZ_ERR_ARG;
    Parsed P;
    // only the header is checked: the bytes given may be a prefix of the stream
    hiz_status rc =
        parse_header(nullptr, static_cast<const uint8_t *>(h_stream), n, ~uint64_t(0), &P);
    if (rc)
        return rc;
    *out = P.info;
    return HIZ_OK;
}

hiz_status hiz_decompress(hiz_ctx *c, const void *d_in, uint64_t in_size, float *d_field,
                          uint64_t field_cap, uint64_t dims_out[3], hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    c->err.clear();
    if (!d_in || !d_field)
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    if ((reinterpret_cast<uintptr_t>(d_field) & 3) || (reinterpret_cast<uintptr_t>(d_in) & 15))
        return fail(c, HIZ_ERR_ARG, "field must be 4-byte and stream 16-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    hiz_status rc = ensure_pinned(c, 4096);
    if (rc)
        return rc;
    const uint64_t nh = std::min<uint64_t>(in_size, kOffChunks);
    if (nh < (uint64_t)kHdrBytes)
        return fail(c, HIZ_ERR_CORRUPT, "stream shorter than its header");
    HIP_TRY(c, hipMemcpyAsync(c->pinned, d_in, nh, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    Parsed P;
    rc = parse_header(c, c->pinned, nh, in_size, &P);
    if (rc)
        return rc;
    if (P.info.constant == 0 && nh < (uint64_t)kOffChunks)
        return fail(c, HIZ_ERR_CORRUPT, "stream shorter than its tables");
    if (dims_out)
        for (int k = 0; k < 3; k++)
            dims_out[k] = P.info.dims[k];
    if (field_cap < P.N)
        return fail(c, HIZ_ERR_BUFSZ, "field needs %llu elements", (unsigned long long)P.N);
    if (P.info.constant) {
        {
            Scope sc(c, s, "fill");
            launch_fill(d_field, P.N, P.const_value, s);
        }
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamSynchronize(s));
        if (c->profiling)
            collect_profile(c);
        return HIZ_OK;
    }
    const int tz = kDefaultTileZ;
    Job J;
    memset(&J, 0, sizeof(J));
    J.out = d_field;
    J.stream = const_cast<uint8_t *>(static_cast<const uint8_t *>(d_in));
    J.cap = in_size;
    for (int k = 0; k < 3; k++) {
        J.dims[k] = P.info.dims[k];
        J.nb[k] = (uint32_t)cdiv(J.dims[k], kAnchor);
    }
    J.N = P.N;
    J.ntz = (uint32_t)cdiv(J.nb[2], tz);
    J.n_anchors = (uint64_t)J.nb[0] * J.nb[1] * J.nb[2];
    J.chunk = P.info.chunk;
    J.log2_chunk = (uint32_t)ilog2(J.chunk);
    J.n_chunks = P.info.n_chunks;
    J.off_anchors = P.off_anchors;
    J.mode = P.info.mode;
    J.eb = P.info.eb;
    memcpy(J.cfg_forced, P.info.level_cfg, sizeof(J.cfg_forced));
    J.idx_bytes = (uint8_t)P.idx_bytes;
    J.n_tiles = (uint64_t)J.nb[0] * J.nb[1] * J.ntz;
    J.n_dblk = cdiv(J.n_chunks, 256);
    J.off_oidx = P.off_oidx;
    J.off_oval = P.off_oval;
    J.off_payload = P.off_payload;
    J.n_out = P.info.n_outliers;
    J.payload_words = P.info.payload_words;
    J.eps = P.info.eps;

    Arena A;
    const uint64_t o_job = A.take(sizeof(Job));
    const uint64_t o_st = A.take(sizeof(FieldState));
    const uint64_t o_cnt = A.take(sizeof(Counters));
    const uint64_t o_dt = A.take(sizeof(DecTables));
    const uint64_t o_codes = A.take(J.N);
    const uint64_t o_lba = A.take(8 * J.n_dblk);
    rc = ensure_ws(c, A.off);
    if (rc)
        return rc;
    rc = ensure_pinned(c, sizeof(Job) + kResultBytes + 256);
    if (rc)
        return rc;
    uint8_t *ws = static_cast<uint8_t *>(c->ws);
    J.st = reinterpret_cast<FieldState *>(ws + o_st);
    J.dt = reinterpret_cast<DecTables *>(ws + o_dt);
    J.codes = ws + o_codes;
    J.lb_a = reinterpret_cast<uint64_t *>(ws + o_lba);
    Job *d_job = reinterpret_cast<Job *>(ws + o_job);
    Counters *d_cnt = reinterpret_cast<Counters *>(ws + o_cnt);
    memcpy(c->pinned, &J, sizeof(J));
    uint8_t *h_res = c->pinned + ((sizeof(Job) + 255) & ~size_t(255));

    HIP_TRY(c, hipMemcpyAsync(d_job, c->pinned, sizeof(Job), hipMemcpyHostToDevice, s));
    {
        Scope sc(c, s, "init_dec");
        launch_init_decompress(d_job, 1, J.n_dblk, d_cnt, s);
    }
    {
        Scope sc(c, s, "dec_tables");
        launch_dec_tables(d_job, 1, s);
    }
    {
        Scope sc(c, s, "decode");
        launch_decode(d_job, 1, J.n_dblk, d_cnt, s);
    }
    if (J.n_out) {
        Scope sc(c, s, "scatter");
        launch_scatter(d_job, 1, J.n_out, s);
    }
    {
        Scope sc(c, s, "reconstruct");
        launch_reconstruct(d_job, 1, J.n_tiles, tz, predict_grid(c, tz, J.n_tiles, true), s);
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(h_res, J.st, kResultBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->profiling)
        collect_profile(c);
    FieldState res;
    memcpy(&res, h_res, kResultBytes);
    if ((res.flags & ST_CORRUPT) || res.zeros_seen != J.n_out)
        return fail(c, HIZ_ERR_CORRUPT, "stream failed a decoding check");
    return HIZ_OK;
}

} // extern "C"
