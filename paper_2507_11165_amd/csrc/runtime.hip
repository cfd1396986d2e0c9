// Host runtime of the hiz library: context and device workspace, job
// descriptors, the launch sequence of (batched) compression and
// decompression, HIP-graph replay of that sequence, stream header parsing,
// per-kernel profiling, and the C ABI declared in hiz.h.
//
// Every call, single or batched, builds one Job per field and runs each stage
// of the method as ONE launch over the concatenated work units of all its
// fields (work-list prefixes in the Job table), so a batch of many uneven
// fields costs the same number of launches as a single field.
#include "hiz.h"
#include "hiz_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace hiz;

namespace {

constexpr uint64_t kMaxN = 1ull << 40;
constexpr int kMaxBatch = 4096;  // fields per batched call
constexpr int kGraphSlots = 8;   // instantiated graphs kept per context

struct KStat {
    std::string name;
    uint64_t launches = 0;
    double ms = 0.0;
};

struct Pending {
    int stat;
    hipEvent_t a, b;
};

// Launch geometry of one enqueued sequence: equal keys replay the same graph
// (the Job table itself is re-uploaded by the graph's first node).
struct GraphKey {
    int kind; // 0 compress, 1 decompress
    int njobs;
    uint64_t v[24];
    const void *ws;
    const void *pinned;
};

struct GraphSlot {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};

// The batch most recently enqueued on a context, until hiz_batch_finish.
struct Batch {
    bool pending = false;
    int kind = 0;                      // 0 compress, 1 decompress
    int n = 0;                         // caller fields
    int njobs = 0;                     // fields with device work
    std::vector<int> field;            // job -> caller field
    std::vector<hiz_status> status;    // caller field -> status known before launch
    std::vector<uint64_t> size;        // caller field -> bytes (compress) / elements (decompress)
    std::vector<uint64_t> cap;         // caller field -> output capacity
    std::vector<uint64_t> dims;        // caller field -> dims parsed from the header (decompress)
    std::vector<uint64_t> n_out;       // job -> outliers named by the header (decompress)
    std::vector<std::string> msg;      // caller field -> message of a failure before launch
    hipStream_t s = nullptr;
    uint8_t *h_res = nullptr;          // pinned: njobs x kResultBytes
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
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    GraphSlot gslot[kGraphSlots];
    uint64_t gclock = 0;
    uint64_t graph_builds = 0, graph_replays = 0;
    hipEvent_t done = nullptr;
    hipEvent_t chain = nullptr; // end event of the previous timed launch of the current sequence
    Batch batch;
    uint8_t *scratch = nullptr; // this device's copy of the allocation-free call's scratch array
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

std::string fmt_msg(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return buf;
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

// Launch defaults of a field: Huffman chunk length and tile depth, read off
// a table measured once on an MI355X by paper_2507_11165_amd/tune_table.py
// (compress + decompress of one field per shape, chunk length and tile
// depth). Each row holds a measured shape and its pick: the chunk length with
// the highest compress + decompress throughput among those whose compression
// ratio is within 1 % of the best ratio, and the fastest tile depth for it. A
// field takes the row nearest to it in (log N, log dz); a tile depth above the
// field's block count along z is lowered to it.
struct LaunchRow {
    uint64_t dims[3];
    uint32_t chunk;
    int tz;
};
constexpr LaunchRow kLaunchTable[] = {
    {{64, 64, 64}, 1024, 1},     {{128, 128, 128}, 1024, 2}, {{192, 192, 192}, 1024, 4},
    {{256, 256, 256}, 1024, 2},  {{100, 500, 500}, 1024, 2}, {{384, 384, 384}, 1024, 2},
    {{512, 512, 512}, 1024, 2},  {{384, 96, 48}, 1024, 1},   {{48, 96, 384}, 1024, 2},
};

struct LaunchDefaults {
    uint32_t chunk;
    int tz;
};

LaunchDefaults default_launch(const uint64_t dims[3])
{
    const double n = std::log2((double)dims[0] * (double)dims[1] * (double)dims[2]);
    const double z = std::log2((double)dims[2]);
    const LaunchRow *best = &kLaunchTable[0];
    double bd = 1e300;
    for (const LaunchRow &r : kLaunchTable) {
        const double rn = std::log2((double)r.dims[0] * (double)r.dims[1] * (double)r.dims[2]);
        const double rz = std::log2((double)r.dims[2]);
        const double d = (n - rn) * (n - rn) + (z - rz) * (z - rz);
        if (d < bd) {
            bd = d;
            best = &r;
        }
    }
    LaunchDefaults L{best->chunk, best->tz};
    const uint64_t nbz = cdiv(dims[2], kAnchor);
    while (L.tz > 1 && (uint64_t)L.tz > nbz)
        L.tz >>= 1;
    return L;
}

int depth_index(int tz) { return tz == 1 ? 0 : tz == 2 ? 1 : 2; }

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

// HIP events around one launch on the launch stream; off while a graph is
// being captured (events would become graph nodes). Within a launch sequence
// (chained scopes, back to back on one stream) a launch's start event is the
// previous launch's end event, so each launch records one event.
struct Scope {
    hiz_ctx *c;
    hipStream_t s;
    Pending p;
    bool on, chained;
    Scope(hiz_ctx *c_, hipStream_t s_, const char *name, bool allow = true, bool chained_ = false)
        : c(c_), s(s_), on(c_->profiling && allow), chained(chained_)
    {
        if (on) {
            p.stat = stat_index(c, name);
            p.a = chained && c->chain ? c->chain : take_event(c);
            p.b = take_event(c);
            on = p.a && p.b;
            if (on && p.a != c->chain)
                hipEventRecord(p.a, s);
        }
    }
    ~Scope()
    {
        if (on) {
            hipEventRecord(p.b, s);
            c->pending.push_back(p);
            if (chained)
                c->chain = p.b;
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

// ---- graphs ----
void drop_graphs(hiz_ctx *c)
{
    for (GraphSlot &g : c->gslot) {
        if (g.exec)
            hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.used = 0;
    }
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
        drop_graphs(c);
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
    if (c->pinned) {
        hipDeviceSynchronize();
        drop_graphs(c);
        hipHostFree(c->pinned);
    }
    c->pinned = nullptr;
    c->pinned_size = 0;
    uint64_t want = std::max<uint64_t>(bytes + bytes / 4, 64 * 1024);
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

int encode_grid(hiz_ctx *c)
{
    if (!c->enc_bpc) {
        c->enc_bpc = encode_blocks_per_cu();
        if (debug_on())
            fprintf(stderr, "[hiz] encode: %d CUs x %d workgroups per CU\n", c->cus, c->enc_bpc);
    }
    return c->cus * c->enc_bpc;
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
    uint64_t off_lcsizes, n_lc; // last stages: chunk-size table and chunk count
    float const_value;
};

// Checks a stream header; `msg` receives the reason of a failure.
hiz_status parse_header(std::string *msg, const uint8_t *h, uint64_t n, uint64_t in_size,
                        Parsed *P)
{
#define BAD(text)                                                                                 \
    do {                                                                                          \
        if (msg)                                                                                  \
            *msg = text;                                                                          \
        return HIZ_ERR_CORRUPT;                                                                   \
    } while (0)
    memset(P, 0, sizeof(*P));
    hiz_info &I = P->info;
    if (n < (uint64_t)kHdrBytes || in_size < (uint64_t)kHdrBytes)
        BAD("stream shorter than its header");
    if (get_le<uint32_t>(h + H_MAGIC) != kMagic || get_le<uint16_t>(h + H_VERSION) != kVersion)
        BAD("bad magic or version");
    I.mode = h[H_MODE];
    const uint8_t flags = h[H_FLAGS];
    I.pipeline = h[H_PIPE];
    I.reorder = (flags & kFlagReorder) ? 1 : 0;
    if (I.mode > 1 || (flags & ~7) || I.pipeline > PIPE_CR)
        BAD("bad mode, flags or pipeline");
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        I.dims[k] = get_le<uint64_t>(h + H_DIMS + 8 * k);
        if (I.dims[k] == 0 || I.dims[k] > kMaxN)
            BAD("bad dims");
        if (N > kMaxN / I.dims[k])
            BAD("field too large");
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
        if (I.pipeline != PIPE_HF || I.reorder)
            BAD("bad constant stream");
        if (I.total_bytes != kHdrBytes + 4u || in_size < I.total_bytes)
            BAD("bad constant stream");
        if (n >= kHdrBytes + 4u)
            P->const_value = get_le<float>(h + kHdrBytes);
        return HIZ_OK;
    }
    if (h[H_ASTRIDE] != kAnchor || h[H_NLEV] != kLevels)
        BAD("bad anchor stride or level count");
    for (int l = 0; l < kLevels; l++) {
        for (int k = 0; k < 3; k++)
            I.level_cfg[l][k] = h[H_CFG + 3 * l + k];
        if (I.level_cfg[l][0] > 2 || I.level_cfg[l][1] > 1 || I.level_cfg[l][2] > 5)
            BAD("bad level configuration");
    }
    I.chunk = get_le<uint32_t>(h + H_CHUNK);
    I.n_outliers = get_le<uint64_t>(h + H_NOUT);
    I.payload_words = get_le<uint64_t>(h + H_PWORDS);
    I.n_chunks = get_le<uint64_t>(h + H_NCHUNKS);
    I.lc_bytes = get_le<uint64_t>(h + H_LCBYTES);
    P->n_lc = get_le<uint64_t>(h + H_NLC);
    const uint64_t n_anchors = get_le<uint64_t>(h + H_NANCH);
    if (I.pipeline == PIPE_TP) {
        // no Huffman stage: the stages run on the N code bytes
        if (I.chunk != 0 || I.n_chunks != 0 || I.payload_words != 0)
            BAD("bad throughput-mode header");
        if (P->n_lc != cdiv(N, kLcChunk) || I.lc_bytes > N)
            BAD("bad stage section size");
    } else {
        if (I.chunk < 256 || I.chunk > 65536 || (I.chunk & (I.chunk - 1)))
            BAD("bad chunk length");
        if (I.n_chunks != cdiv(N, I.chunk))
            BAD("bad chunk count");
        if (I.payload_words > N + I.n_chunks)
            BAD("bad payload size");
        if (I.pipeline == PIPE_HF && (P->n_lc != 0 || I.lc_bytes != 0))
            BAD("bad stage section size");
        if (I.pipeline == PIPE_CR &&
            (P->n_lc != cdiv(4 * I.payload_words, kLcChunk) || I.lc_bytes > 4 * I.payload_words))
            BAD("bad stage section size");
    }
    P->idx_bytes = N < (1ull << 32) ? 4 : 8;
    if (((flags & kFlagIdx64) != 0) != (P->idx_bytes == 8))
        BAD("bad index width flag");
    if (n_anchors != cdiv(I.dims[0], kAnchor) * cdiv(I.dims[1], kAnchor) * cdiv(I.dims[2], kAnchor))
        BAD("bad anchor count");
    if (I.n_outliers > N)
        BAD("bad outlier count");
    // sections: HF payload last; TP stage sizes at 384, stage data last; CR
    // Huffman word counts at 384, stage sizes and data after the outliers
    const uint64_t table = I.pipeline == PIPE_TP ? P->n_lc : I.n_chunks;
    P->off_anchors = align16(kOffChunks + 4 * table);
    P->off_oidx = align16(P->off_anchors + 4 * n_anchors);
    P->off_oval = align16(P->off_oidx + (uint64_t)P->idx_bytes * I.n_outliers);
    const uint64_t end_oval = P->off_oval + 4 * I.n_outliers;
    uint64_t total;
    if (I.pipeline == PIPE_HF) {
        P->off_payload = align16(end_oval);
        total = P->off_payload + 4 * I.payload_words;
    } else {
        P->off_lcsizes = I.pipeline == PIPE_TP ? (uint64_t)kOffChunks : align16(end_oval);
        P->off_payload = I.pipeline == PIPE_TP ? align16(end_oval)
                                               : align16(P->off_lcsizes + 4 * P->n_lc);
        total = P->off_payload + I.lc_bytes;
    }
    if (I.total_bytes != total || I.total_bytes > in_size)
        BAD("stream size does not match its header");
    if (I.pipeline == PIPE_TP)
        return HIZ_OK;
    if (n >= (uint64_t)kOffChunks) {
        // the code lengths must form a complete prefix code (one symbol: length 1)
        const uint8_t *len = h + kOffLen;
        uint64_t kraft = 0; // in units of 2^-32
        int nsym = 0;
        for (int i = 0; i < 256; i++) {
            if (!len[i])
                continue;
            if (len[i] > kMaxCodeLen)
                BAD("code length above 32");
            kraft += 1ull << (32 - len[i]);
            nsym++;
        }
        if (nsym == 0 || (nsym == 1 && kraft != (1ull << 31)) || (nsym > 1 && kraft != (1ull << 32)))
            BAD("code lengths do not form a complete prefix code");
    }
    return HIZ_OK;
#undef BAD
}

bool valid_cfg(const uint8_t cfg[4][3])
{
    for (int l = 0; l < 4; l++)
        if (cfg[l][0] > 2 || cfg[l][1] > 1 || cfg[l][2] > 5)
            return false;
    return true;
}

// Shared parameters of a call (NULL = defaults) and its tile shape; on a
// failure `msg` names the bad parameter.
hiz_status check_params(const hiz_params *params, hiz_params &p, int &tz, const char *&msg)
{
    memset(&p, 0, sizeof(p));
    p.tune = 1;
    for (int l = 0; l < 4; l++)
        p.level_cfg[l][0] = HIZ_SPLINE_CUBIC;
    p.reorder = -1;
    if (params)
        p = *params;
    msg = "";
    if (!valid_cfg(p.level_cfg)) {
        msg = "bad level configuration";
        return HIZ_ERR_ARG;
    }
    if (p.chunk && (p.chunk < 256 || p.chunk > 65536 || (p.chunk & (p.chunk - 1)))) {
        msg = "chunk must be a power of two in [256, 65536]";
        return HIZ_ERR_ARG;
    }
    // 0: each field's tile depth from the launch table
    tz = (int)p.tile_z;
    if (tz != 0 && tz != 1 && tz != 2 && tz != 4) {
        msg = "tile_z must be 0, 1, 2 or 4";
        return HIZ_ERR_ARG;
    }
    if (p.pipeline > HIZ_PIPE_CR) {
        msg = "pipeline must be HIZ_PIPE_HUFFMAN, HIZ_PIPE_TP or HIZ_PIPE_CR";
        return HIZ_ERR_ARG;
    }
    if (p.reorder < -1 || p.reorder > 1) {
        msg = "reorder must be -1, 0 or 1";
        return HIZ_ERR_ARG;
    }
    if (p.reorder < 0)
        p.reorder = p.pipeline == HIZ_PIPE_CR ? 1 : 0;
    return HIZ_OK;
}

hiz_status resolve_params(hiz_ctx *c, const hiz_params *params, hiz_params &p, int &tz)
{
    const char *msg = "";
    hiz_status rc = check_params(params, p, tz, msg);
    return rc ? fail(c, rc, "%s", msg) : HIZ_OK;
}

// Tiles whose owned points all lie inside the field (their coarse levels run
// in the pre-pass), per axis: a block starting at 16b qualifies when
// 16b + 16 <= d.
void set_full_tiles(Job &J, int tz)
{
    J.nf[0] = (uint32_t)(J.dims[0] / kAnchor);
    J.nf[1] = (uint32_t)(J.dims[1] / kAnchor);
    J.nf[2] = (uint32_t)(J.dims[2] / kAnchor / (uint64_t)tz);
}

uint64_t full_tiles(const Job &J) { return (uint64_t)J.nf[0] * J.nf[1] * J.nf[2]; }

// Geometry and parameters of one field to compress; device pointers are
// filled in by the caller once the workspace is laid out.
hiz_status plan_compress(const float *d_field, const uint64_t dims[3], int mode, double eb,
                         const hiz_params &p, int tz, void *d_out, uint64_t out_cap, Job &J,
                         const char *&msg)
{
    if (!d_field || !dims || !d_out) {
        msg = "NULL argument";
        return HIZ_ERR_ARG;
    }
    if (mode != HIZ_ABS && mode != HIZ_REL) {
        msg = "bad error-bound mode";
        return HIZ_ERR_ARG;
    }
    if (!(eb > 0.0) || !std::isfinite(eb)) {
        msg = "error bound must be finite and positive";
        return HIZ_ERR_ARG;
    }
    if ((reinterpret_cast<uintptr_t>(d_field) & 3) || (reinterpret_cast<uintptr_t>(d_out) & 15)) {
        msg = "field must be 4-byte and stream 16-byte aligned";
        return HIZ_ERR_ARG;
    }
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        if (dims[k] == 0 || dims[k] > kMaxN || N > kMaxN / dims[k]) {
            msg = "bad dims";
            return HIZ_ERR_ARG;
        }
        N *= dims[k];
    }
    const LaunchDefaults dl = default_launch(dims);
    const uint32_t chunk = p.chunk ? p.chunk : dl.chunk;
    if (!tz)
        tz = dl.tz;
    memset(&J, 0, sizeof(J));
    J.field = d_field;
    J.stream = static_cast<uint8_t *>(d_out);
    J.cap = out_cap;
    for (int k = 0; k < 3; k++) {
        J.dims[k] = dims[k];
        J.nb[k] = (uint32_t)cdiv(dims[k], kAnchor);
        // full blocks per axis: 17 points, or the single point of a flat axis
        J.n_full[k] = dims[k] == 1 ? 1
                      : dims[k] >= (uint64_t)kSide ? (uint32_t)((dims[k] - kSide) / kAnchor + 1)
                                                   : 0;
    }
    J.N = N;
    J.tz = (uint8_t)tz;
    J.ntz = (uint32_t)cdiv(J.nb[2], tz);
    J.n_anchors = (uint64_t)J.nb[0] * J.nb[1] * J.nb[2];
    J.chunk = chunk;
    J.chunk_req = chunk;
    J.log2_chunk = (uint32_t)ilog2(chunk);
    J.n_chunks = cdiv(N, chunk);
    J.off_anchors = align16(kOffChunks + 4 * J.n_chunks);
    J.mode = mode;
    J.tune = p.tune ? 1 : 0;
    J.eb = eb;
    memcpy(J.cfg_forced, p.level_cfg, sizeof(J.cfg_forced));
    J.idx_bytes = N < (1ull << 32) ? 4 : 8;
    J.n_mm = mode == HIZ_REL ? cdiv(N, kMmUnit) : 0;
    const uint64_t n_full = (uint64_t)J.n_full[0] * J.n_full[1] * J.n_full[2];
    if (J.tune && n_full > 0) {
        // Sec. 5.1.3: about 0.2 % of the points, in whole full blocks
        uint64_t vol = 1;
        for (int k = 0; k < 3; k++)
            vol *= dims[k] == 1 ? 1 : (uint64_t)kSide;
        uint64_t ns = std::max<uint64_t>(1, cdiv(2 * N, 1000ull * vol));
        J.n_samples = (uint32_t)std::min<uint64_t>(ns, n_full);
    }
    J.n_tune = (uint64_t)J.n_samples * 9;
    J.n_tiles = (uint64_t)J.nb[0] * J.nb[1] * J.ntz;
    J.n_groups = cdiv(J.n_chunks, kEncGroupChunks);
    set_full_tiles(J, tz);
    J.pipe = (uint8_t)p.pipeline;
    J.reorder = (uint8_t)(p.reorder ? 1 : 0);
    if (J.pipe == PIPE_TP) {
        // no Huffman stage; the stage chunk sizes take the table at 384
        J.chunk = 0;
        J.log2_chunk = 0;
        J.n_chunks = 0;
        J.n_groups = 0;
        J.n_lc = cdiv(N, kLcChunk);
        J.off_anchors = align16(kOffChunks + 4 * J.n_lc);
    } else if (J.pipe == PIPE_CR) {
        // the payload (at most one 32-bit word per code plus a padding word
        // per chunk) waits in the workspace for the last stages
        J.hpay_cap = 4 * (N + J.n_chunks);
        J.n_lc = cdiv(J.hpay_cap, kLcChunk);
    }
    // outliers in row-major order need their own pass when the lossless stage
    // sees the codes reordered
    J.n_ou = J.reorder ? cdiv(N, kLcChunk) : 0;
    return HIZ_OK;
}

// Geometry of one field to decompress from its parsed header.
void plan_decompress(const Parsed &P, const void *d_in, uint64_t in_size, float *d_field, int tz,
                     Job &J)
{
    memset(&J, 0, sizeof(J));
    J.out = d_field;
    J.stream = const_cast<uint8_t *>(static_cast<const uint8_t *>(d_in));
    J.cap = in_size;
    for (int k = 0; k < 3; k++) {
        J.dims[k] = P.info.dims[k];
        J.nb[k] = (uint32_t)cdiv(J.dims[k], kAnchor);
    }
    J.N = P.N;
    J.tz = (uint8_t)tz;
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
    J.n_dblk = dec_subblocks(J.n_chunks);
    set_full_tiles(J, tz);
    J.off_oidx = P.off_oidx;
    J.off_oval = P.off_oval;
    J.off_payload = P.off_payload;
    J.n_out = P.info.n_outliers;
    J.payload_words = P.info.payload_words;
    J.eps = P.info.eps;
    J.pipe = (uint8_t)P.info.pipeline;
    J.reorder = (uint8_t)P.info.reorder;
    J.n_lc = P.n_lc;
    J.off_lcsizes = P.off_lcsizes;
    J.off_lcdata = P.off_payload;
    J.lc_bytes = P.info.lc_bytes;
    if (J.pipe == PIPE_CR)
        J.hpay_cap = 4 * J.payload_words;
}

// Totals of one enqueued sequence (also the graph key's payload).
struct Totals {
    uint64_t mm = 0, tune = 0, tiles = 0, chunks = 0, groups = 0, dblk = 0, out = 0;
    uint64_t max_groups = 0, max_dblk = 0;
    uint64_t lc = 0, ou = 0;   // stage chunks, outlier units
    uint64_t max_n = 0;        // largest field (reordering launch)
    bool reorder = false;      // some field's codes are reordered
    uint64_t max_clear = 0;    // longest look-back array any field clears at the start
    // per tile depth (jobs ordered by depth): jobs [jlo, jhi) with tiles [tlo, thi)
    int jlo[kTileDepths] = {0, 0, 0}, jhi[kTileDepths] = {0, 0, 0};
    uint64_t tlo[kTileDepths] = {0, 0, 0}, thi[kTileDepths] = {0, 0, 0};
};

// Lay out the workspace for `jobs`, set their prefixes and device pointers,
// and stage the Job table in pinned memory. Returns the device addresses of
// the Job table, the counters and the result block.
struct Layout {
    Job *d_jobs;
    Counters *d_cnt;
    uint8_t *d_res;
    uint8_t *h_res;
    const void *h_jobs; // host copy of the Job table the sequence uploads
};

// Workspace sections of one field (offsets from the workspace base).
struct Sections {
    uint64_t st, codes, crec, ccode, dt, lba, lbb, woff, zoff, mm, seq, hpay, lbc, lbd;
};

// Take one field's sections from the arena and add its work units to the
// launch totals (its work-list prefixes are the totals before it).
void take_sections(Arena &A, Job &J, bool decompress, Totals &T, Sections &o)
{
    const int tz = J.tz;
    memset(&o, 0, sizeof(o));
    o.st = A.take(sizeof(FieldState));
    o.codes = A.take(J.N);
    // the code sequence of the lossless stage, the ratio mode's payload, and
    // the look-back words of the stage chunks and outlier units
    o.seq = J.reorder ? A.take(J.N) : 0;
    o.hpay = J.pipe == PIPE_CR ? A.take(J.hpay_cap) : 0;
    o.lbc = A.take(8 * J.n_lc);
    o.lbd = A.take(8 * std::max(J.n_lc, J.n_ou));
    J.lc_begin = T.lc;
    J.ou_begin = T.ou;
    T.lc += J.n_lc;
    T.ou += J.n_ou;
    T.max_n = std::max(T.max_n, J.N);
    T.reorder = T.reorder || J.reorder;
    T.max_clear = std::max(T.max_clear, std::max(J.n_lc, J.n_ou));
    o.crec = A.take(4 * coarse_values_per_tile(tz) * full_tiles(J));
    o.ccode = decompress ? 0 : A.take(coarse_codes_per_tile(tz) * full_tiles(J));
    if (decompress) {
        o.dt = A.take(sizeof(DecTables));
        o.lba = A.take(8 * J.n_dblk);
        J.tile_begin = T.tiles;
        J.dblk_begin = T.dblk;
        J.out_begin = T.out;
        T.tiles += J.n_tiles;
        T.dblk += J.n_dblk;
        T.out += J.n_out;
        T.max_dblk = std::max(T.max_dblk, J.n_dblk);
    } else {
        o.lba = A.take(8 * J.n_groups);
        o.lbb = A.take(8 * J.n_groups);
        o.woff = A.take(8 * J.n_chunks);
        o.zoff = A.take(8 * J.n_chunks);
        o.mm = A.take(8 * std::max<uint64_t>(J.n_mm, J.n_tiles));
        J.mm_begin = T.mm;
        J.tune_begin = T.tune;
        J.tile_begin = T.tiles;
        J.chunk_begin = T.chunks;
        J.group_begin = T.groups;
        T.mm += J.n_mm;
        T.tune += J.n_tune;
        T.tiles += J.n_tiles;
        T.chunks += J.n_chunks;
        T.groups += J.n_groups;
        T.max_groups = std::max(T.max_groups, J.n_groups);
    }
}

// Device pointers of one field's sections in the workspace at `ws`.
void bind_sections(uint8_t *ws, Job &J, bool decompress, const Sections &o)
{
    J.st = reinterpret_cast<FieldState *>(ws + o.st);
    J.codes = ws + o.codes;
    J.seq = J.reorder ? ws + o.seq : J.codes;
    J.hpay = J.pipe == PIPE_CR ? ws + o.hpay : nullptr;
    J.lb_c = reinterpret_cast<uint64_t *>(ws + o.lbc);
    J.lb_d = reinterpret_cast<uint64_t *>(ws + o.lbd);
    J.crec = reinterpret_cast<float *>(ws + o.crec);
    J.ccode = decompress ? nullptr : ws + o.ccode;
    J.lb_a = reinterpret_cast<uint64_t *>(ws + o.lba);
    if (decompress) {
        J.dt = reinterpret_cast<DecTables *>(ws + o.dt);
    } else {
        J.lb_b = reinterpret_cast<uint64_t *>(ws + o.lbb);
        J.woff = reinterpret_cast<uint64_t *>(ws + o.woff);
        J.zoff = reinterpret_cast<uint64_t *>(ws + o.zoff);
        J.mm_part = reinterpret_cast<uint2 *>(ws + o.mm);
    }
}

bool totals_fit(const Totals &T)
{
    return T.groups <= 0xffffffffull && T.dblk <= 0xffffffffull && T.tune <= 0xffffffffull &&
           T.tiles <= 0xffffffffull && T.lc <= 0xffffffffull && T.ou <= 0xffffffffull;
}

// Per-depth job and tile ranges of a Job table ordered by tile depth.
void depth_ranges(const Job *jobs, int nj, Totals &T)
{
    for (int d = 0; d < kTileDepths; d++) {
        T.jlo[d] = T.jhi[d] = 0;
        T.tlo[d] = T.thi[d] = 0;
    }
    int j = 0;
    for (int d = 0; d < kTileDepths; d++) {
        T.jlo[d] = j;
        T.tlo[d] = j < nj ? jobs[j].tile_begin : T.tiles;
        while (j < nj && depth_index(jobs[j].tz) == d)
            j++;
        T.jhi[d] = j;
        T.thi[d] = j < nj ? jobs[j].tile_begin : T.tiles;
    }
}

// Stable order of a call's jobs by tile depth, so that each depth's jobs and
// tiles are contiguous (one launch of the tile kernels per depth); `field`
// and `extra` (when not empty) follow the jobs.
void order_by_depth(std::vector<Job> &jobs, std::vector<int> &field, std::vector<uint64_t> &extra)
{
    const size_t n = jobs.size();
    std::vector<size_t> idx(n);
    for (size_t i = 0; i < n; i++)
        idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        return depth_index(jobs[a].tz) < depth_index(jobs[b].tz);
    });
    std::vector<Job> j2(n);
    std::vector<int> f2(n);
    std::vector<uint64_t> e2(extra.empty() ? 0 : n);
    for (size_t i = 0; i < n; i++) {
        j2[i] = jobs[idx[i]];
        f2[i] = field[idx[i]];
        if (!extra.empty())
            e2[i] = extra[idx[i]];
    }
    jobs.swap(j2);
    field.swap(f2);
    if (!extra.empty())
        extra.swap(e2);
}

hiz_status layout(hiz_ctx *c, std::vector<Job> &jobs, bool decompress, Totals &T, Layout &L)
{
    const int nj = (int)jobs.size();
    Arena A;
    const uint64_t o_jobs = A.take(sizeof(Job) * nj);
    const uint64_t o_cnt = A.take(sizeof(Counters));
    const uint64_t o_res = A.take((uint64_t)kResultBytes * nj);
    std::vector<Sections> o(nj);
    T = Totals();
    for (int j = 0; j < nj; j++)
        take_sections(A, jobs[j], decompress, T, o[j]);
    depth_ranges(jobs.data(), nj, T);
    if (!totals_fit(T))
        return fail(c, HIZ_ERR_ARG, "batch too large for one launch");
    hiz_status rc = ensure_ws(c, A.off);
    if (rc)
        return rc;
    const uint64_t job_bytes = ((sizeof(Job) * nj + 255) & ~uint64_t(255));
    rc = ensure_pinned(c, job_bytes + (uint64_t)kResultBytes * nj + 256);
    if (rc)
        return rc;
    uint8_t *ws = static_cast<uint8_t *>(c->ws);
    for (int j = 0; j < nj; j++)
        bind_sections(ws, jobs[j], decompress, o[j]);
    memcpy(c->pinned, jobs.data(), sizeof(Job) * nj);
    L.d_jobs = reinterpret_cast<Job *>(ws + o_jobs);
    L.d_cnt = reinterpret_cast<Counters *>(ws + o_cnt);
    L.d_res = ws + o_res;
    L.h_res = c->pinned + job_bytes;
    L.h_jobs = c->pinned;
    return HIZ_OK;
}

// The launch sequence of compression (Sec. 5: range and bound, tuner,
// interpolation + quantization + histogram, codebook, encoding) for all jobs.
// Claim counters of the tile kernels of one depth (a device address).
uint32_t *depth_counters(const Layout &L, int d)
{
    return reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(L.d_cnt) +
                                        offsetof(Counters, tile_next)) + 8 * d;
}

void enqueue_compress(hiz_ctx *c, const Layout &L, int nj, const Totals &T, hipStream_t s,
                      bool prof)
{
    hipMemcpyAsync(L.d_jobs, L.h_jobs, sizeof(Job) * nj, hipMemcpyHostToDevice, s);
    c->chain = nullptr;
    {
        Scope sc(c, s, "init", prof, true);
        launch_init_compress(L.d_jobs, nj, std::max(T.max_groups, T.max_clear), L.d_cnt, s);
    }
    if (T.mm) {
        Scope sc(c, s, "minmax", prof, true);
        launch_minmax(L.d_jobs, nj, T.mm, c->cus * 8, s);
    }
    {
        Scope sc(c, s, "eps", prof, true);
        launch_eps(L.d_jobs, nj, s);
    }
    if (T.tune) {
        Scope sc(c, s, "tune", prof, true);
        launch_tune(L.d_jobs, nj, T.tune, s);
    }
    {
        Scope sc(c, s, "tune_pick", prof, true);
        launch_tune_pick(L.d_jobs, nj, s);
    }
    // the tile kernels: one launch per tile depth present
    for (int d = 0; d < kTileDepths; d++) {
        if (T.thi[d] <= T.tlo[d])
            continue;
        const int tz = 1 << d;
        const Job *dj = L.d_jobs + T.jlo[d];
        const int nd = T.jhi[d] - T.jlo[d];
        {
            Scope sc(c, s, "coarse", prof, true);
            launch_coarse(dj, nd, T.tlo[d], T.thi[d], tz, true, s);
        }
        {
            Scope sc(c, s, "predict_quant", prof, true);
            launch_predict(dj, nd, T.tlo[d], T.thi[d], tz,
                           predict_grid(c, tz, T.thi[d] - T.tlo[d], false), depth_counters(L, d),
                           s);
        }
    }
    if (T.reorder) {
        Scope sc(c, s, "reorder", prof, true);
        launch_reorder(L.d_jobs, nj, T.max_n, false, s);
    }
    {
        Scope sc(c, s, "codebook", prof, true);
        launch_codebook(L.d_jobs, nj, s);
    }
    if (T.chunks) {
        Scope sc(c, s, "encode", prof, true);
        launch_encode(L.d_jobs, nj, T.chunks, T.groups, L.d_cnt, encode_grid(c), s);
    }
    if (T.ou) {
        Scope sc(c, s, "outliers", prof, true);
        launch_outliers(L.d_jobs, nj, T.ou, L.d_cnt, s);
    }
    if (T.lc) {
        Scope sc(c, s, "lc_encode", prof, true);
        launch_lc_encode(L.d_jobs, nj, T.lc, L.d_cnt, s);
    }
    c->chain = nullptr;
    launch_gather_results(L.d_jobs, nj, L.d_res, s);
    hipMemcpyAsync(L.h_res, L.d_res, (size_t)kResultBytes * nj, hipMemcpyDeviceToHost, s);
}

// The launch sequence of decompression (decode, outliers, reconstruction).
void enqueue_decompress(hiz_ctx *c, const Layout &L, int nj, const Totals &T, hipStream_t s,
                        bool prof)
{
    hipMemcpyAsync(L.d_jobs, L.h_jobs, sizeof(Job) * nj, hipMemcpyHostToDevice, s);
    c->chain = nullptr;
    {
        Scope sc(c, s, "init_dec", prof, true);
        launch_init_decompress(L.d_jobs, nj, std::max(T.max_dblk, T.max_clear), L.d_cnt, s);
    }
    if (T.dblk) {
        Scope sc(c, s, "dec_tables", prof, true);
        launch_dec_tables(L.d_jobs, nj, s);
    }
    if (T.lc) {
        Scope sc(c, s, "lc_decode", prof, true);
        launch_lc_decode(L.d_jobs, nj, T.lc, L.d_cnt, s);
    }
    if (T.dblk) {
        Scope sc(c, s, "decode", prof, true);
        launch_decode(L.d_jobs, nj, T.dblk, L.d_cnt, c->cus, s);
    }
    if (T.reorder) {
        Scope sc(c, s, "unreorder", prof, true);
        launch_reorder(L.d_jobs, nj, T.max_n, true, s);
    }
    if (T.out) {
        Scope sc(c, s, "scatter", prof, true);
        launch_scatter(L.d_jobs, nj, T.out, s);
    }
    for (int d = 0; d < kTileDepths; d++) {
        if (T.thi[d] <= T.tlo[d])
            continue;
        const int tz = 1 << d;
        const Job *dj = L.d_jobs + T.jlo[d];
        const int nd = T.jhi[d] - T.jlo[d];
        {
            Scope sc(c, s, "coarse_rec", prof, true);
            launch_coarse(dj, nd, T.tlo[d], T.thi[d], tz, false, s);
        }
        {
            Scope sc(c, s, "reconstruct", prof, true);
            launch_reconstruct(dj, nd, T.tlo[d], T.thi[d], tz,
                               predict_grid(c, tz, T.thi[d] - T.tlo[d], true),
                               depth_counters(L, d), s);
        }
    }
    c->chain = nullptr;
    launch_gather_results(L.d_jobs, nj, L.d_res, s);
    hipMemcpyAsync(L.h_res, L.d_res, (size_t)kResultBytes * nj, hipMemcpyDeviceToHost, s);
}

// Run the sequence eagerly, or replay (building on first use) the HIP graph of
// this launch geometry. Graph replay re-reads the Job table from the same
// pinned buffer, so only the geometry has to match.
hiz_status enqueue(hiz_ctx *c, int kind, const Layout &L, int nj, const Totals &T,
                   hipStream_t s)
{
    if (!c->graphs) {
        if (kind == 0)
            enqueue_compress(c, L, nj, T, s, true);
        else
            enqueue_decompress(c, L, nj, T, s, true);
        HIP_TRY(c, hipGetLastError());
        return HIZ_OK;
    }
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.kind = kind;
    key.njobs = nj;
    const uint64_t v[24] = {T.mm,       T.tune,    T.tiles,    T.chunks,  T.groups, T.dblk,
                            T.out,      T.max_groups, T.max_dblk, (uint64_t)c->cus, T.lc, T.ou,
                            (uint64_t)T.jlo[0], (uint64_t)T.jlo[1], (uint64_t)T.jlo[2],
                            (uint64_t)T.jhi[0], (uint64_t)T.jhi[1], (uint64_t)T.jhi[2],
                            T.tlo[0],   T.tlo[1],  T.tlo[2],   T.thi[0],  T.thi[1], T.thi[2]};
    memcpy(key.v, v, sizeof(v));
    key.ws = c->ws;
    key.pinned = c->pinned;
    // occupancy queries stay outside the capture
    for (int tz = 1; tz <= 4; tz *= 2)
        predict_grid(c, tz, 1, kind == 1);
    encode_grid(c);
    GraphSlot *hit = nullptr;
    for (GraphSlot &g : c->gslot)
        if (g.exec && memcmp(&g.key, &key, sizeof(key)) == 0)
            hit = &g;
    if (!hit) {
        if (!c->cap_stream)
            HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        GraphSlot *victim = &c->gslot[0];
        for (GraphSlot &g : c->gslot)
            if (!g.exec || g.used < victim->used)
                victim = &g;
        if (victim->exec) {
            hipGraphExecDestroy(victim->exec);
            victim->exec = nullptr;
        }
        HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        if (kind == 0)
            enqueue_compress(c, L, nj, T, c->cap_stream, false);
        else
            enqueue_decompress(c, L, nj, T, c->cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess || !g) {
            hipGetLastError();
            return fail(c, HIZ_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&victim->exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
            victim->exec = nullptr;
            hipGetLastError();
            return fail(c, HIZ_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        victim->key = key;
        hit = victim;
        c->graph_builds++;
    }
    hit->used = ++c->gclock;
    {
        Scope sc(c, s, kind == 0 ? "graph_compress" : "graph_decompress");
        HIP_TRY(c, hipGraphLaunch(hit->exec, s));
    }
    c->graph_replays++;
    return HIZ_OK;
}

void begin_batch(hiz_ctx *c, int kind, int n, hipStream_t s)
{
    Batch &B = c->batch;
    B.kind = kind;
    B.n = n;
    B.njobs = 0;
    B.field.clear();
    B.status.assign(n, HIZ_OK);
    B.size.assign(n, 0);
    B.cap.assign(n, 0);
    B.dims.assign(3 * (size_t)n, 0);
    B.n_out.clear();
    B.msg.assign(n, std::string());
    B.s = s;
    B.h_res = nullptr;
}

// A submission that failed after enqueueing part of its work: let that work
// drain so that nothing still reads the context's buffers.
hiz_status abandon(hiz_ctx *c, hipStream_t s, hiz_status rc)
{
    std::string keep = c->err;
    hipStreamSynchronize(s);
    hipGetLastError();
    c->err = keep;
    return rc;
}

hiz_status mark_submitted(hiz_ctx *c)
{
    if (!c->done)
        HIP_TRY(c, hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    HIP_TRY(c, hipEventRecord(c->done, c->batch.s));
    c->batch.pending = true;
    return HIZ_OK;
}

hiz_status submit_compress(hiz_ctx *c, int n, const float *const *d_fields, const uint64_t *dims,
                           const int *modes, const double *ebs, const hiz_params *params,
                           void *const *d_outs, const uint64_t *caps, hipStream_t s)
{
    c->err.clear();
    if (n < 0 || n > kMaxBatch)
        return fail(c, HIZ_ERR_ARG, "batch size must be in [0, %d]", kMaxBatch);
    if (n > 0 && (!d_fields || !dims || !modes || !ebs || !d_outs || !caps))
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    if (c->batch.pending)
        return fail(c, HIZ_ERR_ARG, "the previous batch on this context is not finished");
    hiz_params p;
    int tz;
    hiz_status rc = resolve_params(c, params, p, tz);
    if (rc)
        return rc;
    HIP_TRY(c, hipSetDevice(c->device));
    begin_batch(c, 0, n, s);
    Batch &B = c->batch;
    std::vector<Job> jobs;
    jobs.reserve(n);
    for (int i = 0; i < n; i++) {
        Job J;
        B.cap[i] = caps[i];
        const char *m = "";
        B.status[i] = plan_compress(d_fields[i], dims + 3 * i, modes[i], ebs[i], p, tz, d_outs[i],
                                    caps[i], J, m);
        if (B.status[i])
            B.msg[i] = m;
        if (B.status[i] == HIZ_OK) {
            jobs.push_back(J);
            B.field.push_back(i);
        }
    }
    B.njobs = (int)jobs.size();
    if (B.njobs) {
        std::vector<uint64_t> none;
        order_by_depth(jobs, B.field, none);
        Totals T;
        Layout L;
        rc = layout(c, jobs, false, T, L);
        if (rc)
            return abandon(c, s, rc);
        B.h_res = L.h_res;
        rc = enqueue(c, 0, L, B.njobs, T, s);
        if (rc)
            return abandon(c, s, rc);
    }
    rc = mark_submitted(c);
    return rc ? abandon(c, s, rc) : rc;
}

// h_hdrs (may be NULL): host copies of the first kOffChunks bytes of every
// stream (fewer when a stream is shorter), read by the caller beforehand; then
// nothing here waits for the device.
hiz_status submit_decompress(hiz_ctx *c, int n, const void *const *d_ins,
                             const uint64_t *in_sizes, float *const *d_fields,
                             const uint64_t *field_caps, hipStream_t s,
                             const uint8_t *h_hdrs = nullptr)
{
    c->err.clear();
    if (n < 0 || n > kMaxBatch)
        return fail(c, HIZ_ERR_ARG, "batch size must be in [0, %d]", kMaxBatch);
    if (n > 0 && (!d_ins || !in_sizes || !d_fields || !field_caps))
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    if (c->batch.pending)
        return fail(c, HIZ_ERR_ARG, "the previous batch on this context is not finished");
    HIP_TRY(c, hipSetDevice(c->device));
    begin_batch(c, 1, n, s);
    Batch &B = c->batch;
    // headers and code-length tables of every stream, in one synchronization
    hiz_status rc = ensure_pinned(c, (uint64_t)kOffChunks * std::max(n, 1));
    if (rc)
        return rc;
    std::vector<uint64_t> nh(n, 0);
    for (int i = 0; i < n; i++) {
        if (!d_ins[i] || !d_fields[i]) {
            B.status[i] = HIZ_ERR_ARG;
            B.msg[i] = "NULL argument";
            continue;
        }
        if ((reinterpret_cast<uintptr_t>(d_fields[i]) & 3) ||
            (reinterpret_cast<uintptr_t>(d_ins[i]) & 15)) {
            B.status[i] = HIZ_ERR_ARG;
            B.msg[i] = "field must be 4-byte and stream 16-byte aligned";
            continue;
        }
        nh[i] = std::min<uint64_t>(in_sizes[i], kOffChunks);
        if (nh[i] < (uint64_t)kHdrBytes) {
            B.status[i] = HIZ_ERR_CORRUPT;
            B.msg[i] = "stream shorter than its header";
            continue;
        }
        if (h_hdrs)
            memcpy(c->pinned + (uint64_t)kOffChunks * i, h_hdrs + (uint64_t)kOffChunks * i, nh[i]);
        else if (hipMemcpyAsync(c->pinned + (uint64_t)kOffChunks * i, d_ins[i], nh[i],
                                hipMemcpyDeviceToHost, s) != hipSuccess)
            return abandon(c, s, fail(c, HIZ_ERR_HIP, "cannot read the header of stream %d", i));
    }
    if (!h_hdrs)
        HIP_TRY(c, hipStreamSynchronize(s));
    std::vector<Parsed> P(n);
    std::vector<Job> jobs;
    for (int i = 0; i < n; i++) {
        if (B.status[i])
            continue;
        B.cap[i] = field_caps[i];
        hiz_status st = parse_header(&B.msg[i], c->pinned + (uint64_t)kOffChunks * i, nh[i],
                                     in_sizes[i], &P[i]);
        if (st == HIZ_OK && !P[i].info.constant && nh[i] < (uint64_t)kOffChunks) {
            st = HIZ_ERR_CORRUPT;
            B.msg[i] = "stream shorter than its tables";
        }
        if (st == HIZ_OK && field_caps[i] < P[i].N) {
            st = HIZ_ERR_BUFSZ;
            B.msg[i] = fmt_msg("field needs %llu elements", (unsigned long long)P[i].N);
        }
        B.status[i] = st;
        B.size[i] = P[i].N;
        if (st == HIZ_OK || st == HIZ_ERR_BUFSZ)
            for (int k = 0; k < 3; k++)
                B.dims[3 * i + k] = P[i].info.dims[k];
    }
    // constant streams: one fill each (their device work is done here)
    for (int i = 0; i < n; i++) {
        if (B.status[i] || !P[i].info.constant)
            continue;
        Scope sc(c, s, "fill");
        launch_fill(d_fields[i], P[i].N, P[i].const_value, s);
    }
    for (int i = 0; i < n; i++) {
        if (B.status[i] || P[i].info.constant)
            continue;
        Job J;
        plan_decompress(P[i], d_ins[i], in_sizes[i], d_fields[i],
                        default_launch(P[i].info.dims).tz, J);
        jobs.push_back(J);
        B.field.push_back(i);
        B.n_out.push_back(J.n_out);
    }
    if (hipGetLastError() != hipSuccess)
        return abandon(c, s, fail(c, HIZ_ERR_HIP, "fill launch failed"));
    B.njobs = (int)jobs.size();
    if (B.njobs) {
        order_by_depth(jobs, B.field, B.n_out);
        Totals T;
        Layout L;
        rc = layout(c, jobs, true, T, L);
        if (rc)
            return abandon(c, s, rc);
        B.h_res = L.h_res;
        rc = enqueue(c, 1, L, B.njobs, T, s);
        if (rc)
            return abandon(c, s, rc);
    }
    rc = mark_submitted(c);
    return rc ? abandon(c, s, rc) : rc;
}

// Wait for the pending batch and turn its device results into per-field
// statuses and sizes. Returns the first failing field's status.
hiz_status finish(hiz_ctx *c, uint64_t *sizes, uint64_t *dims, hiz_status *statuses)
{
    Batch &B = c->batch;
    if (!B.pending)
        return fail(c, HIZ_ERR_ARG, "no batch is pending on this context");
    B.pending = false;
    HIP_TRY(c, hipEventSynchronize(c->done));
    if (c->profiling)
        collect_profile(c);
    for (int j = 0; j < B.njobs; j++) {
        const int i = B.field[j];
        FieldState res;
        memcpy(&res, B.h_res + (size_t)kResultBytes * j, kResultBytes);
        if (B.kind == 0) {
            if (res.flags & ST_NONFINITE) {
                B.status[i] = HIZ_ERR_NONFINITE;
                B.msg[i] = "field holds NaN or Inf";
                continue;
            }
            if (res.flags & ST_CORRUPT) {
                B.status[i] = HIZ_ERR_HIP;
                B.msg[i] = "internal consistency check failed";
                continue;
            }
            B.size[i] = res.total_bytes;
            if ((res.flags & ST_OVERFLOW) || res.total_bytes > B.cap[i]) {
                B.status[i] = HIZ_ERR_BUFSZ;
                B.msg[i] = fmt_msg("output needs %llu bytes, capacity is %llu",
                                   (unsigned long long)res.total_bytes,
                                   (unsigned long long)B.cap[i]);
            }
        } else if ((res.flags & ST_CORRUPT) || res.zeros_seen != B.n_out[j]) {
            B.status[i] = HIZ_ERR_CORRUPT;
            B.msg[i] = "stream failed a decoding check";
        }
    }
    hiz_status first = HIZ_OK;
    for (int i = 0; i < B.n; i++) {
        if (sizes)
            sizes[i] = B.size[i];
        if (dims)
            for (int k = 0; k < 3; k++)
                dims[3 * i + k] = B.dims[3 * i + k];
        if (statuses)
            statuses[i] = B.status[i];
        if (B.status[i] && first == HIZ_OK) {
            first = B.status[i];
            if (B.n == 1)
                c->err = B.msg[i];
            else
                c->err = fmt_msg("field %d: %s", i, B.msg[i].c_str());
        }
    }
    return first;
}


// ---- allocation-free compression -------------------------------------------
// The workspace of hiz_compress_noalloc: a fixed array in device memory that
// every GPU running the library holds once, from the code object's load until
// the process ends. In host code `scratch` names a host-side stand-in, never
// the device memory: the address each device holds it at is looked up once
// per device (hiz_create, with that device current) and only that address is
// used afterwards.
constexpr uint64_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `device` (resolved once).
hiz_status resolve_scratch(int device, uint8_t **out)
{
    if (device < 0 || device >= kMaxDevices)
        return HIZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hipGetLastError();
            return HIZ_ERR_HIP;
        }
        g_scratch_ptr[device] = static_cast<uint8_t *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return HIZ_OK;
}

// One compression through the scratch array: the same plan, layout and launch
// sequence as hiz_compress, with no device, pinned or heap allocation (the
// Job table goes up from the pinned block the context allocated at creation,
// and profiling and graphs are skipped).
hiz_status compress_noalloc(hiz_ctx *c, const float *d_field, const uint64_t dims[3], int mode,
                            double eb, const hiz_params *params, void *d_out, uint64_t out_cap,
                            uint64_t *out_size, hipStream_t s)
{
    c->err.clear();
    if (c->batch.pending)
        return fail(c, HIZ_ERR_ARG, "the previous batch on this context is not finished");
    if (!c->scratch)
        return fail(c, HIZ_ERR_HIP, "the scratch array's device address is not known");
    hiz_params p;
    int tz;
    hiz_status rc = resolve_params(c, params, p, tz);
    if (rc)
        return rc;
    HIP_TRY(c, hipSetDevice(c->device));
    Job J;
    const char *m = "";
    rc = plan_compress(d_field, dims, mode, eb, p, tz, d_out, out_cap, J, m);
    if (rc)
        return fail(c, rc, "%s", m);
    // the same sections as a one-field batch, laid out from the scratch base
    Arena A;
    const uint64_t o_jobs = A.take(sizeof(Job));
    const uint64_t o_cnt = A.take(sizeof(Counters));
    const uint64_t o_res = A.take(kResultBytes);
    Totals T;
    Sections o;
    take_sections(A, J, false, T, o);
    depth_ranges(&J, 1, T);
    if (!totals_fit(T))
        return fail(c, HIZ_ERR_ARG, "field too large for one launch");
    if (A.off > kScratchBytes)
        return fail(c, HIZ_ERR_ARG,
                    "field needs %llu bytes of workspace; the allocation-free call holds at most "
                    "%llu (use hiz_compress)",
                    (unsigned long long)A.off, (unsigned long long)kScratchBytes);
    const uint64_t job_bytes = (sizeof(Job) + 255) & ~uint64_t(255);
    if (job_bytes + kResultBytes > c->pinned_size)
        return fail(c, HIZ_ERR_ARG, "the context's staging block is too small");
    bind_sections(c->scratch, J, false, o);
    memcpy(c->pinned, &J, sizeof(Job));
    Layout L;
    L.d_jobs = reinterpret_cast<Job *>(c->scratch + o_jobs);
    L.d_cnt = reinterpret_cast<Counters *>(c->scratch + o_cnt);
    L.d_res = c->scratch + o_res;
    L.h_res = c->pinned + job_bytes;
    L.h_jobs = c->pinned;
    enqueue_compress(c, L, 1, T, s, false);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(s));
    FieldState res;
    memcpy(&res, L.h_res, kResultBytes);
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
    // set-up for hiz_compress_noalloc: the scratch array's address on this
    // device, launch-grid queries, and room for any error message, so that
    // the call itself allocates nothing
    if (resolve_scratch(device, &c->scratch) != HIZ_OK) {
        hipFree(c->ws);
        hipHostFree(c->pinned);
        delete c;
        return HIZ_ERR_HIP;
    }
    for (int tz = 1; tz <= 4; tz *= 2)
        predict_grid(c, tz, 1, false);
    encode_grid(c);
    c->err.reserve(512);
    *out = c;
    return HIZ_OK;
}

void hiz_destroy(hiz_ctx *c)
{
    if (!c)
        return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    drop_graphs(c);
    for (hipEvent_t e : c->events)
        hipEventDestroy(e);
    if (c->done)
        hipEventDestroy(c->done);
    if (c->cap_stream)
        hipStreamDestroy(c->cap_stream);
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
    // payload of 32-bit codewords plus one padding word per chunk, the ratio
    // mode's stage chunk sizes, section gaps
    return kOffChunks + 4 * chunks + 4 * anchors + 12 * N + 4 * (N + chunks) +
           4 * cdiv(4 * (N + chunks), kLcChunk) + 96;
}

uint64_t hiz_workspace_bound(const uint64_t dims[3])
{
    if (!dims)
        return 0;
    uint64_t N = 1;
    for (int k = 0; k < 3; k++) {
        if (dims[k] == 0 || dims[k] > kMaxN || N > kMaxN / dims[k])
            return 0;
        N *= dims[k];
    }
    // the largest layout either direction can take: shortest chunks, one-block
    // tiles, and one 256-byte alignment gap per workspace section
    const uint64_t chunks = cdiv(N, 256);
    const uint64_t groups = cdiv(chunks, kEncGroupChunks);
    const uint64_t tiles = cdiv(dims[0], kAnchor) * cdiv(dims[1], kAnchor) * cdiv(dims[2], kAnchor);
    const uint64_t mm = std::max<uint64_t>(cdiv(N, kMmUnit), tiles);
    const uint64_t per_job = sizeof(Job) + kResultBytes + sizeof(FieldState) + 12 * 256;
    // per-tile coarse-level slots (values and codes of the even-point grid)
    uint64_t coarse = 0;
    for (int tz = 1; tz <= 4; tz *= 2) {
        const uint64_t nt = (dims[0] / kAnchor) * (dims[1] / kAnchor) * (dims[2] / kAnchor / tz);
        coarse = std::max(coarse, nt * (4 * coarse_values_per_tile(tz) + coarse_codes_per_tile(tz)));
    }
    // the lossless pipelines: reordered code sequence, the ratio mode's
    // payload, stage and outlier-unit look-back words (with their gaps)
    const uint64_t lc = cdiv(4 * (N + chunks), kLcChunk);
    const uint64_t pipes = N + 4 * (N + chunks) + 16 * lc + 4 * 256;
    const uint64_t comp = per_job + N + 16 * groups + 16 * chunks + 8 * mm + coarse + pipes;
    const uint64_t dec = per_job + sizeof(DecTables) + N + 8 * dec_subblocks(chunks) + coarse + pipes;
    return std::max(comp, dec);
}

} // extern "C"

namespace hiz {
// Pinned staging of a context for batches of up to n fields, allocated now so
// that no later call of that size reallocates it.
hiz_status ctx_reserve_pinned(hiz_ctx *c, int n)
{
    const uint64_t jobs = ((sizeof(Job) * (uint64_t)n + 255) & ~uint64_t(255)) +
                          (uint64_t)kResultBytes * n + 256;
    return ensure_pinned(c, std::max<uint64_t>(jobs, (uint64_t)kOffChunks * n));
}

// Decompression submit with the streams' header bytes already on the host.
hiz_status ctx_decompress_submit_hdrs(hiz_ctx *c, int n, const void *const *d_ins,
                                      const uint64_t *in_sizes, float *const *d_fields,
                                      const uint64_t *field_caps, hipStream_t s,
                                      const uint8_t *h_hdrs)
{
    return submit_decompress(c, n, d_ins, in_sizes, d_fields, field_caps, s, h_hdrs);
}

uint64_t workspace_bound_points(uint64_t n)
{
    const uint64_t d[3] = {n, 1, 1};
    const uint64_t b = hiz_workspace_bound(d);
    if (b == 0)
        return 0;
    // a tile of 16 x 16 x 16 tz owned points has one slot
    uint64_t coarse = 0;
    for (int tz = 1; tz <= 4; tz *= 2)
        coarse = std::max<uint64_t>(coarse, n / (4096ull * tz) * (4 * coarse_values_per_tile(tz) +
                                                                 coarse_codes_per_tile(tz)));
    return b + coarse;
}
} // namespace hiz

extern "C" {

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

hiz_status hiz_set_graphs(hiz_ctx *c, int on)
{
    if (!c)
        return HIZ_ERR_ARG;
    if (c->batch.pending)
        return fail(c, HIZ_ERR_ARG, "a batch is pending on this context");
    c->graphs = on != 0;
    return HIZ_OK;
}

void hiz_graph_stats(const hiz_ctx *c, uint64_t *builds, uint64_t *replays)
{
    if (builds)
        *builds = c ? c->graph_builds : 0;
    if (replays)
        *replays = c ? c->graph_replays : 0;
}

hiz_status hiz_compress(hiz_ctx *c, const float *d_field, const uint64_t dims[3],
                        hiz_eb_mode mode, double eb, const hiz_params *params, void *d_out,
                        uint64_t out_cap, uint64_t *out_size, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    if (!out_size || !dims)
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    *out_size = 0;
    const int m = (int)mode;
    void *outs[1] = {d_out};
    hiz_status rc = submit_compress(c, 1, &d_field, dims, &m, &eb, params, outs, &out_cap,
                                    reinterpret_cast<hipStream_t>(stream));
    return rc ? rc : finish(c, out_size, nullptr, nullptr);
}

hiz_status hiz_compress_noalloc(hiz_ctx *c, const float *d_field, const uint64_t dims[3],
                                hiz_eb_mode mode, double eb, const hiz_params *params, void *d_out,
                                uint64_t out_cap, uint64_t *out_size, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    if (!out_size || !dims)
        return fail(c, HIZ_ERR_ARG, "NULL argument");
    *out_size = 0;
    return compress_noalloc(c, d_field, dims, (int)mode, eb, params, d_out, out_cap, out_size,
                            reinterpret_cast<hipStream_t>(stream));
}

hiz_status hiz_decompress(hiz_ctx *c, const void *d_in, uint64_t in_size, float *d_field,
                          uint64_t field_cap, uint64_t dims_out[3], hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    hiz_status rc = submit_decompress(c, 1, &d_in, &in_size, &d_field, &field_cap,
                                      reinterpret_cast<hipStream_t>(stream));
    if (rc)
        return rc;
    uint64_t dims[3] = {0, 0, 0};
    rc = finish(c, nullptr, dims, nullptr);
    if (dims_out && dims[0])
        memcpy(dims_out, dims, sizeof(dims));
    return rc;
}

hiz_status hiz_compress_batch_submit(hiz_ctx *c, int n, const float *const *d_fields,
                                     const uint64_t *dims, const int *modes, const double *ebs,
                                     const hiz_params *params, void *const *d_outs,
                                     const uint64_t *out_caps, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    return submit_compress(c, n, d_fields, dims, modes, ebs, params, d_outs, out_caps,
                           reinterpret_cast<hipStream_t>(stream));
}

hiz_status hiz_decompress_batch_submit(hiz_ctx *c, int n, const void *const *d_ins,
                                       const uint64_t *in_sizes, float *const *d_fields,
                                       const uint64_t *field_caps, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    return submit_decompress(c, n, d_ins, in_sizes, d_fields, field_caps,
                             reinterpret_cast<hipStream_t>(stream));
}

int hiz_batch_ready(hiz_ctx *c)
{
    if (!c || !c->batch.pending)
        return 1;
    return hipEventQuery(c->done) == hipSuccess ? 1 : 0;
}

hiz_status hiz_batch_finish(hiz_ctx *c, uint64_t *sizes, uint64_t *dims, hiz_status *statuses)
{
    if (!c)
        return HIZ_ERR_ARG;
    return finish(c, sizes, dims, statuses);
}

hiz_status hiz_compress_batch(hiz_ctx *c, int n, const float *const *d_fields,
                              const uint64_t *dims, const int *modes, const double *ebs,
                              const hiz_params *params, void *const *d_outs,
                              const uint64_t *out_caps, uint64_t *out_sizes,
                              hiz_status *statuses, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    hiz_status rc = submit_compress(c, n, d_fields, dims, modes, ebs, params, d_outs, out_caps,
                                    reinterpret_cast<hipStream_t>(stream));
    return rc ? rc : finish(c, out_sizes, nullptr, statuses);
}

hiz_status hiz_decompress_batch(hiz_ctx *c, int n, const void *const *d_ins,
                                const uint64_t *in_sizes, float *const *d_fields,
                                const uint64_t *field_caps, uint64_t *dims_out,
                                hiz_status *statuses, hiz_stream_t stream)
{
    if (!c)
        return HIZ_ERR_ARG;
    hiz_status rc = submit_decompress(c, n, d_ins, in_sizes, d_fields, field_caps,
                                      reinterpret_cast<hipStream_t>(stream));
    return rc ? rc : finish(c, nullptr, dims_out, statuses);
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

} // extern "C"
