// C-ABI of the library: handle, emulated CGEMM orchestration, TTGT tensor
// contraction planner, permute, FP64 reductions and the test entry points.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "gather.hpp"

using namespace qce;

// ---------------------------------------------------------------------------
// Scratch of qce_cgemm_emulated_noalloc: a fixed array in every GPU's copy of
// the library, held until the process ends.  Host code never uses the
// array's name as an address: its device address is looked up once per
// device (qce_create, with that device current) and kept in
// g_scratch_ptr.  It holds one GEMM's panels, split-k partial tiles and
// statistics records, all written before they are read, so nothing in it
// needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the scratch on `device`, which must be current.
hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

namespace {
// A GEMM recorded for a grouped launch.  Operands as the panel writer reads
// them (P[r][l] = kcontig ? x[l + r*ld] : x[r + l*ld], conjugated if conj),
// each a caller pointer or, when ws >= 0, a byte offset into the group's
// temporaries at the start of the workspace (a permuted copy).
struct GroupOperand {
    const float2 *ptr = nullptr;
    int64_t ld = 1;
    bool kcontig = false, conj = false;
    int64_t ws = -1;
};
struct GroupItem {
    int mode = QCE_MODE_AUTO;  // AUTO (statistics), FP16X2_SCALED (statistics) or a forced mode
    GroupOperand a, b;
    int64_t m = 0, n = 0, k = 0;
    float2 alpha{1.f, 0.f}, beta{0.f, 0.f};
    float2 *C = nullptr;  // or c_ws >= 0: a temporary
    int64_t ldc = 1, c_ws = -1;
    int count = 1;                  // batch entries
    int64_t sa = 0, sb = 0, sc = 0;  // elements between entries
    int64_t index = 0;              // first decision index (qce_cgemm_grouped: caller order)
};
// A permute run before (operands) or after (outputs) a group's GEMMs.
struct GroupPermute {
    const float2 *src = nullptr;
    int64_t src_ws = -1;
    float2 *dst = nullptr;
    int64_t dst_ws = -1;
    PermDesc d;
    int64_t total = 0;
    bool identity = false;
};
}  // namespace

struct qce_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    qce_mode mode = QCE_MODE_AUTO;
    double t = 0.1, t3 = 0.0;
    // size policy (Sec. 4.3) calibrated on gfx950: statistics pay off from
    // min(m, n, k) = 512 (the paper's A100 values are 2048 and 512)
    int64_t auto_min = 512, emul_min = 512;
    DevState *st = nullptr;        // device
    DevState *dec_base = nullptr;  // decisions of the last call (st, or a batch's states in the workspace)
    int dec_count = 1;
    double *fid_partials = nullptr;  // device, kFidBlocks * 4
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = true;
    bool have_decision = false;
    bool last_on_device = false;
    qce_decision last_host{};
    char err[512] = {0};
    // opt-in timing (qce_set_timing)
    bool timing = false;
    int32_t tag = 0;
    int *mode_log = nullptr;  // device ring of selected modes, kLogCap entries
    int64_t n_calls = 0;      // GEMM calls issued (ring position)
    int64_t first_unresolved_call = 0;
    struct Rec {
        int32_t tag;
        int kind;   // qce_phase for non-GEMM spans; -1 GEMM kernel span; -2 call marker
        int cls;    // GEMM kernel class (mode of the kernel template) for kind == -1
        int fixed;  // mode known on the host, else -1 (look up the device log)
        int64_t call;
        hipEvent_t a, b;
        bool resolved;
        double ms;
        int phase;  // resolved phase
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    // grouped small contractions (qce_group_begin / qce_group_end)
    bool grouping = false;
    bool fused_gather = true;  // permute fused into the split (qce_contract)
    bool smallk = true;        // short-k narrow GEMMs split on load (no panel pass)
    bool gemm_policy = false;  // the size policy also applies to the CGEMM entry points in AUTO mode
    bool group_gemms = true;   // panel-path contractions recorded in groups (grouped launch)
    int gemm_tile = 0;         // panel GEMM tile: 64, 128, or 0 for the tuned table
    std::vector<qce::SmallItem> pending;
    char *grp_dev = nullptr;   // descriptor arena on the device
    char *grp_host = nullptr;  // its pinned host mirror (source of the copies)
    size_t grp_cap = 0, grp_used = 0;
    std::vector<std::pair<char *, char *>> grp_old;  // outgrown arenas, freed at destroy
    // panel-path GEMMs of qce_contract recorded in the open group, their
    // permutes and the bytes of their temporaries
    std::vector<GroupItem> gitems;
    std::vector<GroupPermute> gpre, gpost;
    size_t gtemp = 0;
    int64_t gentries = 0;            // batch entries of gitems that take statistics
    unsigned int *gqueue = nullptr;  // device, kGroupQueueWords zeroed tile counters of the grouped GEMM
    // decisions of the last grouped call in caller order: state index (>= 0)
    // or -1 - index into dec_host (entries that took no statistics)
    std::vector<int64_t> dec_map;
    std::vector<qce_decision> dec_host;
};

namespace {

constexpr int kFidBlocks = 512;
constexpr int kLogCap = 1 << 15;

// ---- timing helpers -------------------------------------------------------
hipEvent_t ev_get(qce_handle *h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipEvent_t span_begin(qce_handle *h) {
    if (!h->timing) return nullptr;
    hipEvent_t e = ev_get(h);
    if (e && hipEventRecord(e, h->stream) != hipSuccess) {
        h->pool.push_back(e);
        return nullptr;
    }
    return e;
}

void span_end(qce_handle *h, hipEvent_t a, int kind, int cls = 0, int fixed = -1, int64_t call = -1) {
    if (!a) return;
    hipEvent_t b = ev_get(h);
    if (!b || hipEventRecord(b, h->stream) != hipSuccess) {
        h->pool.push_back(a);
        if (b) h->pool.push_back(b);
        return;
    }
    h->recs.push_back({h->tag, kind, cls, fixed, call, a, b, false, 0.0, 0});
}

bool class_matches(int cls, int mode) {
    if (cls == QCE_MODE_FP16X2) return mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED;
    return cls == mode;
}

int class_phase(int cls) {
    return (cls == QCE_MODE_FP16X2 || cls == QCE_MODE_FP16X2_SCALED) ? QCE_PHASE_GEMM_FP16X2
         : cls == QCE_MODE_BF16X3 ? QCE_PHASE_GEMM_BF16X3 : QCE_PHASE_GEMM_FP32;
}

// Synchronise and turn pending records into (phase, ms).
hipError_t resolve_timing(qce_handle *h) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    std::vector<int> log;
    bool need_log = false;
    for (auto &r : h->recs)
        if (!r.resolved && r.fixed < 0 && (r.kind == -1 || r.kind == -2)) need_log = true;
    if (need_log && h->mode_log) {
        log.resize(kLogCap);
        e = hipMemcpy(log.data(), h->mode_log, sizeof(int) * kLogCap, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
    }
    for (auto &r : h->recs) {
        if (r.resolved) continue;
        int mode = r.fixed;
        if (mode < 0 && (r.kind == -1 || r.kind == -2))
            mode = (r.call >= 0 && !log.empty()) ? log[r.call % kLogCap] : QCE_MODE_FP32;
        if (r.kind == -2) {
            r.phase = -1 - mode;  // call marker: encodes the mode
            r.ms = 0.0;
        } else {
            float ms = 0.f;
            if (r.a && r.b) (void)hipEventElapsedTime(&ms, r.a, r.b);
            r.ms = ms;
            // cls < 0: one launch that ran the mode it read from the device flag
            r.phase = r.kind >= 0 ? r.kind
                    : r.cls < 0 ? class_phase(mode)
                    : (class_matches(r.cls, mode) ? class_phase(r.cls) : QCE_PHASE_GEMM_SKIPPED);
        }
        if (r.a) h->pool.push_back(r.a);
        if (r.b) h->pool.push_back(r.b);
        r.a = r.b = nullptr;
        r.resolved = true;
    }
    h->first_unresolved_call = h->n_calls;
    return hipSuccess;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

qce_status fail(qce_handle *h, qce_status s, const char *fmt, ...) {
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->err, sizeof(h->err), fmt, ap);
        va_end(ap);
    }
    return s;
}

#define QCE_HIP(h, expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((h), QCE_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

bool parse_mode(const char *s, qce_mode *m) {
    std::string v(s);
    for (auto &c : v) c = (char)tolower(c);
    if (v == "auto") *m = QCE_MODE_AUTO;
    else if (v == "fp16x2" || v == "fp16tcec") *m = QCE_MODE_FP16X2;
    else if (v == "fp16x2s" || v == "fp16x2_scaled") *m = QCE_MODE_FP16X2_SCALED;
    else if (v == "bf16x3") *m = QCE_MODE_BF16X3;
    else if (v == "fp32") *m = QCE_MODE_FP32;
    else return false;
    return true;
}

bool parse_double(const char *s, double *out) {
    char *end = nullptr;
    double v = strtod(s, &end);
    if (end == s || *end != '\0') return false;
    *out = v;
    return true;
}

bool parse_i64(const char *s, int64_t *out) {
    char *end = nullptr;
    long long v = strtoll(s, &end, 10);
    if (end == s || *end != '\0') return false;
    *out = v;
    return true;
}

// Make sure the handle workspace holds `bytes`.
// The decision records of a batched call live in the workspace: once it is
// freed or replaced they are gone.
void forget_batch_decisions(qce_handle *h) {
    if (h->dec_base != h->st || !h->dec_map.empty()) {
        h->dec_map.clear();
        h->dec_host.clear();
        h->dec_base = h->st;
        h->dec_count = 1;
        h->have_decision = false;
    }
}

qce_status ensure_ws(qce_handle *h, size_t bytes) {
    if (bytes <= h->ws_bytes) return QCE_SUCCESS;
    if (!h->ws_owned)
        return fail(h, QCE_ERR_ALLOC, "caller workspace of %zu bytes, %zu needed", h->ws_bytes, bytes);
    if (h->ws) {
        QCE_HIP(h, hipStreamSynchronize(h->stream));
        QCE_HIP(h, hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
        forget_batch_decisions(h);
    }
    size_t want = bytes + bytes / 8;
    want = (want + 4095) & ~(size_t)4095;
    if (hipMalloc(&h->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        return fail(h, QCE_ERR_ALLOC, "hipMalloc of %zu bytes failed", want);
    }
    h->ws_bytes = want;
    return QCE_SUCCESS;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A GEMM operand as the panel writer sees it: P[r][l] = kcontig ? x[l + r*ld]
// : x[r + l*ld], conjugated if conj.
struct OperandView {
    const float2 *ptr;
    int64_t ld;
    bool kcontig;
    bool conj;
    // set: the operand is read through this bit map by the split (ptr is
    // the whole tensor, contiguous; ld = rows, kcontig = conj = false)
    const GatherMap *gm = nullptr;
};

// Both operands into panels in one launch when neither is read through a
// bit map and they are small (below 2^24 elements in all: there the launch
// overhead is the split's main cost); else one launch per operand.
hipError_t split_operand(const OperandView &v, int64_t rows, int64_t k, char *panels, const DevState *st,
                         int which, int forced_mode, hipStream_t s, int nb, int64_t xstride, int64_t pstride);
hipError_t split_operands(const OperandView &a, const OperandView &b, int64_t m, int64_t n, int64_t k,
                          char *panA, char *panB, const DevState *st, int forced_mode, hipStream_t s, int nb,
                          int64_t sa, int64_t sb, int64_t pa, int64_t pb) {
    if (a.gm || b.gm || (double)(m + n) * (double)k * (double)nb > (double)(int64_t(1) << 24)) {
        hipError_t e = split_operand(a, m, k, panA, st, 0, forced_mode, s, nb, sa, pa);
        if (e != hipSuccess) return e;
        return split_operand(b, n, k, panB, st, 1, forced_mode, s, nb, sb, pb);
    }
    SplitJob ja{}, jb{};
    const OperandView *v[2] = {&a, &b};
    SplitJob *j[2] = {&ja, &jb};
    for (int w = 0; w < 2; ++w) {
        SplitJob &q = *j[w];
        q.x = v[w]->ptr;
        q.ldx = v[w]->ld;
        q.kcontig = v[w]->kcontig;
        q.conj = v[w]->conj;
        q.rows = w ? n : m;
        q.k = k;
        q.panels = w ? panB : panA;
        q.st = st;
        q.which = w;
        q.forced_mode = forced_mode;
        q.shift = 0;
        q.batch = nb;
        q.xstride = w ? sb : sa;
        q.pstride = w ? pb : pa;
        q.blocks = split_job_blocks(q.rows, k, q.kcontig);
    }
    return launch_split_pair(ja, jb, s);
}

// Split one operand into panels (the mode and shift from the device state
// when st is set).
hipError_t split_operand(const OperandView &v, int64_t rows, int64_t k, char *panels, const DevState *st,
                         int which, int forced_mode, hipStream_t s, int nb, int64_t xstride, int64_t pstride) {
    if (v.gm) {
        if (nb != 1 || (int64_t(1) << v.gm->nr) != rows || (int64_t(1) << v.gm->nk) != k)
            return hipErrorInvalidValue;
        return launch_split_gather(v.ptr, *v.gm, panels, st, which, forced_mode, 0, s);
    }
    return launch_split_panels(v.ptr, v.ld, v.kcontig, v.conj, rows, k, panels, st, which, forced_mode, 0, s, nb,
                               xstride, pstride);
}

MatDesc stored_desc(const OperandView &v, int64_t rows, int64_t k) {
    // the stored column-major matrix behind the view
    if (v.kcontig) return MatDesc{v.ptr, k, rows, v.ld};
    return MatDesc{v.ptr, rows, k, v.ld};
}

// A batch of equally shaped GEMMs: entry z uses A + z*sa, B + z*sb,
// C + z*sc (elements); count 1 is one GEMM.
struct Batch {
    int count = 1;
    int64_t sa = 0, sb = 0, sc = 0;
};

// Workspace of one (batched) GEMM: panels of every entry, split-k partial
// tiles, and for a batch the per-entry device states.
struct CgemmWs {
    size_t pa = 0, pb = 0, panels = 0, partial = 0, states = 0, records = 0, total = 0;
};
CgemmWs cgemm_ws_layout(int64_t m, int64_t n, int64_t k, int count) {
    CgemmWs w;
    if (k == 0) return w;
    if (irregular_shape(m, n, k)) {
        w.total = align256(direct_ws_bytes(m, n, k, count));
        return w;
    }
    w.pa = align256(panel_bytes(m, k));
    w.pb = align256(panel_bytes(n, k));
    w.panels = (w.pa + w.pb) * (size_t)count;
    w.partial = align256(gemm_partial_bytes(m, n, k, count) * (size_t)count);
    w.states = count > 1 ? align256(sizeof(DevState) * (size_t)count) : 0;
    // statistics block records (bounded over every leading dimension)
    w.records = align256(sizeof(StatsRecord) * (size_t)(stats_blocks_bound(m, k) + stats_blocks_bound(k, n)) *
                         (size_t)count);
    w.total = w.panels + w.partial + w.states + w.records;
    return w;
}

// The emulated CGEMM of one GEMM (or a batch of them): C = alpha * PA * PB^T
// + beta * C where PA (m x k) and PB (n x k) are the panel views.  `ws` holds
// the panel buffers (cgemm_ws_layout).
qce_status cgemm_core(qce_handle *h, int mode, const OperandView &a, const OperandView &b,
                      int64_t m, int64_t n, int64_t k, float2 alpha, float2 beta, float2 *C,
                      int64_t ldc, char *ws, const Batch &bt = Batch{}) {
    hipStream_t s = h->stream;
    const int beta_zero = beta.x == 0.f && beta.y == 0.f;
    const bool batched = bt.count > 1;
    h->dec_base = h->st;
    h->dec_count = bt.count;  // host-side records (forced / irregular / k == 0) hold for every entry
    h->dec_map.clear();
    h->dec_host.clear();
    if (k == 0) {
        hipEvent_t e0 = span_begin(h);
        QCE_HIP(h, launch_scale_c(C, m, n, ldc, beta, beta_zero, s, bt.count, bt.sc));
        span_end(h, e0, QCE_PHASE_OTHER);
        h->have_decision = true;
        h->last_on_device = false;
        h->last_host = qce_decision{};
        h->last_host.mode = QCE_MODE_FP32;
        return QCE_SUCCESS;
    }
    if (irregular_shape(m, n, k)) {
        if (a.gm || b.gm) return fail(h, QCE_ERR_INVALID_VALUE, "bit-map operands need a matrix-core shape");
        DirectArgs d{};
        d.A = a.ptr;
        d.lda = a.ld;
        d.a_kcontig = a.kcontig;
        d.a_conj = a.conj;
        d.B = b.ptr;
        d.ldb = b.ld;
        d.b_kcontig = b.kcontig;
        d.b_conj = b.conj;
        d.m = m;
        d.n = n;
        d.k = k;
        d.C = C;
        d.ldc = ldc;
        d.alpha = alpha;
        d.beta = beta;
        d.beta_zero = beta_zero;
        d.partial = reinterpret_cast<float2 *>(ws);
        d.batch = bt.count;
        d.bsA = bt.sa;
        d.bsB = bt.sb;
        d.bsC = bt.sc;
        hipEvent_t e0 = span_begin(h);
        QCE_HIP(h, launch_direct(d, s));
        span_end(h, e0, QCE_PHASE_GEMM_IRREGULAR);
        h->have_decision = true;
        h->last_on_device = false;
        h->last_host = qce_decision{};
        h->last_host.mode = QCE_MODE_FP32;
        for (int o = 0; o < 2; ++o) {
            h->last_host.n2[o] = -1;
            h->last_host.emax[o] = INT32_MIN;
        }
        return QCE_SUCCESS;
    }
    // keep the device mode log from wrapping over unresolved timing records
    if (h->timing && h->n_calls - h->first_unresolved_call >= kLogCap / 2)
        QCE_HIP(h, resolve_timing(h));
    const int64_t call = h->n_calls++;
    const int slot = (int)(call % kLogCap);
    int *log = h->timing && !batched ? h->mode_log : nullptr;

    const CgemmWs wl = cgemm_ws_layout(m, n, k, bt.count);
    char *panA = ws;
    char *panB = panA + wl.pa * (size_t)bt.count;
    char *part = ws + wl.panels;
    DevState *dst = batched ? reinterpret_cast<DevState *>(ws + wl.panels + wl.partial) : h->st;
    StatsRecord *rec = reinterpret_cast<StatsRecord *>(ws + wl.panels + wl.partial + wl.states);
    h->dec_base = dst;
    MatDesc da = stored_desc(a, m, k), db = stored_desc(b, n, k);
    da.bstride = bt.sa;
    db.bstride = bt.sb;
    GemmArgs g{};
    g.batch = bt.count;
    g.bsA = (int64_t)wl.pa;
    g.bsB = (int64_t)wl.pb;
    g.bsC = bt.sc;
    g.panelsA = panA;
    g.panelsB = panB;
    g.m = m;
    g.n = n;
    g.k = k;
    g.C = C;
    g.ldc = ldc;
    g.alpha = alpha;
    g.beta = beta;
    g.beta_zero = beta_zero;
    g.partial = gemm_partial_bytes(m, n, k, bt.count) ? reinterpret_cast<float2 *>(part) : nullptr;
    g.tile = h->gemm_tile;
    const int nb = bt.count;
    if (h->smallk && !a.gm && !b.gm && smallk_shape(m, n, k)) {
        // short k, narrow C: split on load, no panel pass
        SmallKArgs q{};
        q.A = a.ptr;
        q.lda = a.ld;
        q.a_kcontig = a.kcontig;
        q.a_conj = a.conj;
        q.B = b.ptr;
        q.ldb = b.ld;
        q.b_kcontig = b.kcontig;
        q.b_conj = b.conj;
        q.m = m;
        q.n = n;
        q.k = k;
        q.C = C;
        q.ldc = ldc;
        q.alpha = alpha;
        q.beta = beta;
        q.beta_zero = beta_zero;
        q.batch = nb;
        q.bsA = bt.sa;
        q.bsB = bt.sb;
        q.bsC = bt.sc;
        const bool stats = mode == QCE_MODE_AUTO || mode == QCE_MODE_FP16X2_SCALED;
        if (stats) {
            // the statistics launch only: every workgroup of the short-k
            // kernel takes the decision from the records itself
            hipEvent_t e0 = span_begin(h);
            QCE_HIP(h, launch_stats(da, db, dst, rec, h->t, h->t3, mode == QCE_MODE_AUTO ? -1 : QCE_MODE_FP16X2_SCALED,
                                    log, slot, s, nb, false, &q.sel));
            span_end(h, e0, QCE_PHASE_STATS);
            q.st = nullptr;
            q.select_here = 1;
            q.forced_mode = -1;
        } else {
            q.st = nullptr;
            q.forced_mode = mode;
        }
        hipEvent_t eg = span_begin(h);
        QCE_HIP(h, launch_smallk(q, s));
        if (batched) {
            span_end(h, eg, QCE_PHASE_GEMM_BATCHED);
        } else if (mode == QCE_MODE_AUTO) {
            span_end(h, eg, -1, -1, -1, call);
            if (h->timing) h->recs.push_back({h->tag, -2, 0, -1, call, nullptr, nullptr, false, 0.0, 0});
        } else {
            const int cls = mode == QCE_MODE_BF16X3 ? QCE_MODE_BF16X3
                          : mode == QCE_MODE_FP32 ? QCE_MODE_FP32 : QCE_MODE_FP16X2;
            span_end(h, eg, -1, cls, mode, call);
            if (h->timing) h->recs.push_back({h->tag, -2, 0, mode, call, nullptr, nullptr, false, 0.0, 0});
        }
        h->have_decision = true;
        h->last_on_device = stats;
        if (!stats) {
            h->last_host = qce_decision{};
            h->last_host.mode = mode;
            for (int o = 0; o < 2; ++o) {
                h->last_host.n2[o] = -1;
                h->last_host.emax[o] = INT32_MIN;
            }
        }
        return QCE_SUCCESS;
    }
    if (mode == QCE_MODE_AUTO || mode == QCE_MODE_FP16X2_SCALED) {
        hipEvent_t e0 = span_begin(h);
        QCE_HIP(h, launch_stats(da, db, dst, rec, h->t, h->t3, mode == QCE_MODE_AUTO ? -1 : QCE_MODE_FP16X2_SCALED,
                                log, slot, s, nb));
        span_end(h, e0, QCE_PHASE_STATS);
        hipEvent_t e1 = span_begin(h);
        QCE_HIP(h, split_operands(a, b, m, n, k, panA, panB, dst, 0, s, nb, bt.sa, bt.sb, (int64_t)wl.pa,
                                  (int64_t)wl.pb));
        span_end(h, e1, QCE_PHASE_SPLIT);
        g.st = dst;
        g.forced_mode = -1;
        hipEvent_t eg = span_begin(h);
        QCE_HIP(h, launch_gemm(g, -1, s));
        if (batched) {
            span_end(h, eg, QCE_PHASE_GEMM_BATCHED);
        } else {
            span_end(h, eg, -1, -1, -1, call);
            if (h->timing) h->recs.push_back({h->tag, -2, 0, -1, call, nullptr, nullptr, false, 0.0, 0});
        }
        h->have_decision = true;
        h->last_on_device = true;
    } else {
        hipEvent_t e1 = span_begin(h);
        QCE_HIP(h, split_operands(a, b, m, n, k, panA, panB, nullptr, mode, s, nb, bt.sa, bt.sb, (int64_t)wl.pa,
                                  (int64_t)wl.pb));
        span_end(h, e1, QCE_PHASE_SPLIT);
        g.st = nullptr;
        g.forced_mode = mode;
        const int cls = mode == QCE_MODE_BF16X3 ? QCE_MODE_BF16X3
                      : mode == QCE_MODE_FP32 ? QCE_MODE_FP32 : QCE_MODE_FP16X2;
        hipEvent_t eg = span_begin(h);
        QCE_HIP(h, launch_gemm(g, cls, s));
        span_end(h, eg, -1, cls, mode, call);
        if (h->timing) h->recs.push_back({h->tag, -2, 0, mode, call, nullptr, nullptr, false, 0.0, 0});
        h->have_decision = true;
        h->last_on_device = false;
        h->last_host = qce_decision{};
        h->last_host.mode = mode;
        for (int o = 0; o < 2; ++o) {
            h->last_host.n2[o] = -1;
            h->last_host.emax[o] = INT32_MIN;
        }
    }
    return QCE_SUCCESS;
}

// Size policy of qce_contract in AUTO mode (Sec. 4.3): statistics for
// min(m, n, k) >= auto_min, and for output-dominated GEMMs too (k >= 64,
// min(m, n) >= auto_min, m n k >= 8 auto_min^3: there the FP32 products
// take longer than writing C, so the emulation pays while the statistics
// read only the small operands); BF16X3 for min(m, n, k) >= emul_min;
// otherwise FP32.
int policy_mode(const qce_handle *h, int64_t m, int64_t n, int64_t k) {
    const int64_t mn = std::min(std::min(m, n), k);
    if (mn >= h->auto_min) return QCE_MODE_AUTO;
    const double a = (double)h->auto_min;
    if (k >= 64 && std::min(m, n) >= h->auto_min && (double)m * (double)n * (double)k >= 8.0 * a * a * a)
        return QCE_MODE_AUTO;
    if (mn >= h->emul_min) return QCE_MODE_BF16X3;
    return QCE_MODE_FP32;
}

// The mode of a CGEMM entry-point call: the handle's mode, or in AUTO mode
// with the CGEMM size policy switched on, the size policy's choice.
int gemm_mode(const qce_handle *h, int64_t m, int64_t n, int64_t k) {
    return h->mode == QCE_MODE_AUTO && h->gemm_policy ? policy_mode(h, m, n, k) : h->mode;
}

size_t cgemm_ws_bytes(int64_t m, int64_t n, int64_t k, int count = 1) {
    return cgemm_ws_layout(m, n, k, count).total;
}

bool valid_op(int op) { return op == QCE_OP_N || op == QCE_OP_T || op == QCE_OP_C; }

// --- permute planning -----------------------------------------------------

// Build the merged permutation descriptor: output axis d is input axis
// perm[d] of a row-major tensor with extents ext.
qce_status plan_permute(qce_handle *h, int rank, const int64_t *ext, const int32_t *perm,
                        PermDesc &d, int64_t &total, bool &identity) {
    std::vector<int64_t> istr(rank);
    int64_t s = 1;
    for (int a = rank - 1; a >= 0; --a) {
        istr[a] = s;
        s *= ext[a];
    }
    total = s;
    std::vector<int64_t> oe, os;
    for (int a = 0; a < rank; ++a) {
        const int64_t e = ext[perm[a]];
        if (e == 1) continue;
        const int64_t st = istr[perm[a]];
        if (!oe.empty() && os.back() == st * e) {
            oe.back() *= e;
            os.back() = st;
        } else {
            oe.push_back(e);
            os.push_back(st);
        }
    }
    identity = oe.size() <= 1 && (os.empty() || os[0] == 1);
    if ((int)oe.size() > kMaxRank)
        return fail(h, QCE_ERR_NOT_SUPPORTED, "permutation needs %zu merged axes (max %d)", oe.size(), kMaxRank);
    memset(&d, 0, sizeof(d));
    d.rank = (int)oe.size();
    d.pow2 = 1;
    for (int a = 0; a < d.rank; ++a) {
        d.ext[a] = oe[a];
        d.istride[a] = os[a];
        int lg = 0;
        while ((int64_t(1) << lg) < oe[a]) ++lg;
        d.log2ext[a] = lg;
        if ((int64_t(1) << lg) != oe[a]) d.pow2 = 0;
    }
    return QCE_SUCCESS;
}

qce_status run_permute(qce_handle *h, int rank, const int64_t *ext, const int32_t *perm,
                       const float2 *x, float2 *y) {
    PermDesc d;
    int64_t total = 0;
    bool identity = false;
    qce_status st = plan_permute(h, rank, ext, perm, d, total, identity);
    if (st != QCE_SUCCESS) return st;
    if (total == 0) return QCE_SUCCESS;
    if (identity) {
        hipEvent_t e0 = span_begin(h);
        QCE_HIP(h, hipMemcpyAsync(y, x, (size_t)total * sizeof(float2), hipMemcpyDeviceToDevice, h->stream));
        span_end(h, e0, QCE_PHASE_PERMUTE);
        return QCE_SUCCESS;
    }
    hipEvent_t e0 = span_begin(h);
    QCE_HIP(h, launch_permute(x, y, total, d, h->stream));
    span_end(h, e0, QCE_PHASE_PERMUTE);
    return QCE_SUCCESS;
}

// Grouped small contractions: the descriptor of C[lc] = sum A[la] B[lb]
// when the contraction is an irregular shape small enough for one thread per
// output element (false otherwise, or when its dimensions do not fit).
constexpr int64_t kSmallMaxSum = 1024, kSmallMaxOut = int64_t(1) << 22, kSmallMaxWork = int64_t(1) << 24;

template <class ExtOf>
bool small_item(const qce_tensor *a, const int32_t *la, const qce_tensor *b, const int32_t *lb,
                const qce_tensor *c, const int32_t *lc, const std::vector<int32_t> &K, ExtOf ext_of,
                int64_t m, int64_t n, int64_t k, int64_t nc, SmallItem &it) {
    if (!irregular_shape(m, n, k) || k > kSmallMaxSum || nc > kSmallMaxOut || nc * k > kSmallMaxWork)
        return false;
    auto stride_in = [](const qce_tensor *t, const int32_t *l, int32_t lab) -> int64_t {
        int64_t s = 1;
        for (int i = t->rank - 1; i >= 0; --i) {
            if (l[i] == lab) return s;
            s *= t->extents[i];
        }
        return 0;  // label not in the tensor
    };
    struct Dim {
        int64_t e, sa, sb;
    };
    // outer -> inner, merging a dimension into the one outside it when both
    // operands step through them contiguously
    auto push = [](std::vector<Dim> &v, Dim d) {
        if (d.e == 1) return;
        if (!v.empty() && v.back().sa == d.sa * d.e && v.back().sb == d.sb * d.e) {
            v.back().e *= d.e;
            v.back().sa = d.sa;
            v.back().sb = d.sb;
        } else {
            v.push_back(d);
        }
    };
    std::vector<Dim> out, sum;
    for (int i = 0; i < c->rank; ++i) push(out, Dim{c->extents[i], stride_in(a, la, lc[i]), stride_in(b, lb, lc[i])});
    for (int32_t lab : K) push(sum, Dim{ext_of(lab), stride_in(a, la, lab), stride_in(b, lb, lab)});
    if ((int)out.size() > kSmallOut || (int)sum.size() > kSmallSum) return false;
    it.n_out = nc;
    it.n_sum = k;
    it.nd_out = (int)out.size();
    it.nd_sum = (int)sum.size();
    for (int d = 0; d < it.nd_out; ++d) {
        it.out_ext[d] = out[d].e;
        it.out_sa[d] = out[d].sa;
        it.out_sb[d] = out[d].sb;
    }
    for (int t = 0; t < it.nd_sum; ++t) {  // fastest first
        const Dim &d = sum[sum.size() - 1 - t];
        it.sum_ext[t] = d.e;
        it.sum_sa[t] = d.sa;
        it.sum_sb[t] = d.sb;
    }
    return true;
}

// The bit map of an operand whose row bit t sits at stride 2^rsh[t] and k
// bit t at 2^ksh[t] in its tensor, with the split's 64 x 64 tile bits (the
// low six of each index) listed by increasing stride.
GatherMap gather_map_from_shifts(int nr, int nk, const int8_t *rsh, const int8_t *ksh) {
    GatherMap g;
    g.nr = nr;
    g.nk = nk;
    for (int t = 0; t < nr && t < 32; ++t) g.rsh[t] = rsh[t];
    for (int t = 0; t < nk && t < 32; ++t) g.ksh[t] = ksh[t];
    std::vector<std::pair<int, int>> tb;  // (stride exponent, tile position)
    for (int t = 0; t < std::min(6, nr); ++t) tb.emplace_back(g.rsh[t], t);
    for (int t = 0; t < std::min(6, nk); ++t) tb.emplace_back(g.ksh[t], 6 + t);
    std::sort(tb.begin(), tb.end());
    g.nt = (int)tb.size();
    for (int i = 0; i < g.nt; ++i) {
        g.tsh[i] = (int8_t)tb[i].first;
        g.tpos[i] = (int8_t)tb[i].second;
    }
    return g;
}

// `need` bytes of the group descriptor arena: hp in its pinned host mirror
// (filled by the caller, then copied to dp on the stream), dp on the device.
// The arena is reused from its start only after the stream has drained it,
// and never grown during stream capture.
qce_status grp_reserve(qce_handle *h, size_t need, char *&hp, char *&dp) {
    need = align256(need);
    if (h->grp_used + need > h->grp_cap) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        QCE_HIP(h, hipStreamIsCapturing(h->stream, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(h, QCE_ERR_ALLOC, "group descriptor space full during stream capture "
                                          "(run the work once before capturing, then qce_group_reset)");
        QCE_HIP(h, hipStreamSynchronize(h->stream));  // earlier copies and launches are done
        if (need > h->grp_cap) {
            if (h->grp_dev) h->grp_old.push_back({h->grp_dev, h->grp_host});
            h->grp_dev = nullptr;
            h->grp_host = nullptr;
            const size_t cap = std::max<size_t>(size_t(1) << 20, 4 * need);
            if (hipMalloc(&h->grp_dev, cap) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void **>(&h->grp_host), cap, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                if (h->grp_dev) (void)hipFree(h->grp_dev);
                h->grp_dev = nullptr;
                h->grp_host = nullptr;
                h->grp_cap = 0;
                return fail(h, QCE_ERR_ALLOC, "group descriptor space of %zu bytes", cap);
            }
            h->grp_cap = cap;
        }
        h->grp_used = 0;
    }
    hp = h->grp_host + h->grp_used;
    dp = h->grp_dev + h->grp_used;
    h->grp_used += need;
    return QCE_SUCCESS;
}

qce_status run_group_permute(qce_handle *h, const GroupPermute &p, char *ws) {
    if (p.total == 0) return QCE_SUCCESS;
    const float2 *src = p.src_ws >= 0 ? reinterpret_cast<const float2 *>(ws + p.src_ws) : p.src;
    float2 *dst = p.dst_ws >= 0 ? reinterpret_cast<float2 *>(ws + p.dst_ws) : p.dst;
    hipEvent_t e0 = span_begin(h);
    if (p.identity)
        QCE_HIP(h, hipMemcpyAsync(dst, src, (size_t)p.total * sizeof(float2), hipMemcpyDeviceToDevice, h->stream));
    else
        QCE_HIP(h, launch_permute(src, dst, p.total, p.d, h->stream));
    span_end(h, e0, QCE_PHASE_PERMUTE);
    return QCE_SUCCESS;
}

// The GEMMs of a group in one launch per phase: operand permutes, one
// statistics launch (every entry that selects its mode), one split launch
// (both operands of every entry), one persistent grouped GEMM launch (and
// one split-k sum launch), output permutes.  Workspace: the temporaries
// (temp_bytes, offsets used by the items and permutes) | decision states of
// every entry that takes statistics | per item: panels of A, of B, partial
// tiles, statistics records.  Items must be matrix-core shapes with k > 0.
// first_state (optional) receives each item's first decision state index
// (states at h->dec_base afterwards), -1 for items without statistics.
qce_status run_group_gemms(qce_handle *h, std::vector<GroupItem> &items, const std::vector<GroupPermute> &pre,
                           const std::vector<GroupPermute> &post, size_t temp_bytes,
                           std::vector<int64_t> *first_state = nullptr) {
    const int count = (int)items.size();
    if (first_state) first_state->assign(items.size(), -1);
    if (count == 0 && pre.empty() && post.empty()) return QCE_SUCCESS;
    std::vector<GroupGemmEntry> ents(count);
    int64_t n_states = 0;
    for (int i = 0; i < count; ++i) {
        const GroupItem &it = items[i];
        if (it.m <= 0 || it.n <= 0 || it.k <= 0 || irregular_shape(it.m, it.n, it.k) || it.count < 1)
            return fail(h, QCE_ERR_INTERNAL, "grouped GEMM entry of shape %lld x %lld x %lld", (long long)it.m,
                        (long long)it.n, (long long)it.k);
        GemmArgs &g = ents[i].g;
        g = GemmArgs{};
        g.m = it.m;
        g.n = it.n;
        g.k = it.k;
        g.ldc = it.ldc;
        g.alpha = it.alpha;
        g.beta = it.beta;
        g.beta_zero = it.beta.x == 0.f && it.beta.y == 0.f;
        g.batch = it.count;
        g.bsA = (int64_t)align256(panel_bytes(it.m, it.k));
        g.bsB = (int64_t)align256(panel_bytes(it.n, it.k));
        g.bsC = it.sc;
        if (it.mode == QCE_MODE_AUTO || it.mode == QCE_MODE_FP16X2_SCALED) n_states += it.count;
    }
    if (n_states > kMaxBatch + 1)
        return fail(h, QCE_ERR_NOT_SUPPORTED, "%lld grouped entries take statistics (at most %d)",
                    (long long)n_states, kMaxBatch + 1);
    const int tile = count ? gemm_group_tile(ents.data(), count, h->gemm_tile) : 128;
    if (count) gemm_group_shape(ents.data(), count, tile);
    struct Off {
        size_t pa, pb, part, rec;
        int64_t st;  // first state index, -1: no statistics
    };
    std::vector<Off> off(count);
    size_t total = align256(temp_bytes);
    const size_t states_off = total;
    total += align256(sizeof(DevState) * (size_t)n_states);
    int64_t si = 0;
    for (int i = 0; i < count; ++i) {
        const GroupItem &it = items[i];
        const GemmArgs &g = ents[i].g;
        Off &o = off[i];
        const bool stats = it.mode == QCE_MODE_AUTO || it.mode == QCE_MODE_FP16X2_SCALED;
        o.st = stats ? si : -1;
        if (stats) si += it.count;
        o.pa = total;
        total += (size_t)g.bsA * (size_t)it.count;
        o.pb = total;
        total += (size_t)g.bsB * (size_t)it.count;
        o.part = total;
        if (ents[i].nsplit > 1) total += align256((size_t)g.bsPartial * sizeof(float2) * (size_t)it.count);
        o.rec = total;
        if (stats)
            total += align256(sizeof(StatsRecord) *
                              (size_t)(stats_blocks_bound(it.m, it.k) + stats_blocks_bound(it.k, it.n)) *
                              (size_t)it.count);
    }
    DeviceGuard dg(h->device);
    qce_status rs = ensure_ws(h, total);
    if (rs != QCE_SUCCESS) return rs;
    char *ws = static_cast<char *>(h->ws);
    DevState *states = reinterpret_cast<DevState *>(ws + states_off);
    auto resolve = [&](const GroupOperand &v) {
        return v.ws >= 0 ? reinterpret_cast<const float2 *>(ws + v.ws) : v.ptr;
    };
    std::vector<GroupStatsEntry> sents;
    std::vector<SplitJob> jobs;
    int64_t stat_blocks = 0, split_blocks = 0, selects = 0;
    for (int i = 0; i < count; ++i) {
        const GroupItem &it = items[i];
        GemmArgs &g = ents[i].g;
        const Off &o = off[i];
        const float2 *pa = resolve(it.a), *pb = resolve(it.b);
        g.panelsA = ws + o.pa;
        g.panelsB = ws + o.pb;
        g.C = it.c_ws >= 0 ? reinterpret_cast<float2 *>(ws + it.c_ws) : it.C;
        g.partial = ents[i].nsplit > 1 ? reinterpret_cast<float2 *>(ws + o.part) : nullptr;
        DevState *dst = o.st >= 0 ? states + o.st : nullptr;
        g.st = dst;
        g.forced_mode = dst ? -1 : it.mode;
        if (dst) {
            MatDesc da = it.a.kcontig ? MatDesc{pa, it.k, it.m, it.a.ld, it.sa} : MatDesc{pa, it.m, it.k, it.a.ld, it.sa};
            MatDesc db = it.b.kcontig ? MatDesc{pb, it.k, it.n, it.b.ld, it.sb} : MatDesc{pb, it.n, it.k, it.b.ld, it.sb};
            GroupStatsEntry se;
            if (stats_group_entry(da, db, dst, reinterpret_cast<StatsRecord *>(ws + o.rec), h->t, h->t3,
                                  it.mode == QCE_MODE_AUTO ? -1 : QCE_MODE_FP16X2_SCALED, it.count, se) != hipSuccess)
                return fail(h, QCE_ERR_NOT_SUPPORTED, "statistics of a %lld x %lld x %lld grouped entry",
                            (long long)it.m, (long long)it.n, (long long)it.k);
            se.block_start = stat_blocks;
            stat_blocks += (int64_t)(se.args.blocks_a + se.args.blocks_b) * se.batch;
            se.select_start = selects;
            selects += se.batch;
            sents.push_back(se);
        }
        for (int w = 0; w < 2; ++w) {
            const GroupOperand &v = w ? it.b : it.a;
            SplitJob j{};
            j.x = w ? pb : pa;
            j.ldx = v.ld;
            j.kcontig = v.kcontig;
            j.conj = v.conj;
            j.rows = w ? it.n : it.m;
            j.k = it.k;
            j.panels = ws + (w ? o.pb : o.pa);
            j.st = dst;
            j.which = w;
            j.forced_mode = it.mode;
            j.shift = 0;
            j.batch = it.count;
            j.xstride = w ? it.sb : it.sa;
            j.pstride = w ? g.bsB : g.bsA;
            j.blocks = split_job_blocks(j.rows, j.k, j.kcontig);
            j.block_start = split_blocks;
            split_blocks += j.blocks * j.batch;
            jobs.push_back(j);
        }
    }
    int64_t total_tiles = 0, total_red = 0;
    if (count) gemm_group_schedule(ents.data(), count, total_tiles, total_red);
    // descriptors: statistics entries | split jobs | GEMM entries
    const size_t b0 = align256(sizeof(GroupStatsEntry) * sents.size());
    const size_t b1 = align256(sizeof(SplitJob) * jobs.size());
    const size_t b2 = align256(sizeof(GroupGemmEntry) * ents.size());
    char *hp = nullptr, *dp = nullptr;
    if (count) {
        rs = grp_reserve(h, b0 + b1 + b2, hp, dp);
        if (rs != QCE_SUCCESS) return rs;
        if (!sents.empty()) memcpy(hp, sents.data(), sizeof(GroupStatsEntry) * sents.size());
        memcpy(hp + b0, jobs.data(), sizeof(SplitJob) * jobs.size());
        memcpy(hp + b0 + b1, ents.data(), sizeof(GroupGemmEntry) * ents.size());
        QCE_HIP(h, hipMemcpyAsync(dp, hp, b0 + b1 + b2, hipMemcpyHostToDevice, h->stream));
    }
    for (const GroupPermute &p : pre) {
        rs = run_group_permute(h, p, ws);
        if (rs != QCE_SUCCESS) return rs;
    }
    if (count) {
        if (!sents.empty()) {
            hipEvent_t e0 = span_begin(h);
            QCE_HIP(h, launch_stats_grouped(reinterpret_cast<const GroupStatsEntry *>(dp), (int)sents.size(),
                                            stat_blocks, selects, h->stream));
            span_end(h, e0, QCE_PHASE_STATS);
        }
        hipEvent_t e1 = span_begin(h);
        QCE_HIP(h, launch_split_grouped(reinterpret_cast<const SplitJob *>(dp + b0), (int)jobs.size(), split_blocks,
                                        h->stream));
        span_end(h, e1, QCE_PHASE_SPLIT);
        hipEvent_t e2 = span_begin(h);
        QCE_HIP(h, launch_gemm_grouped(reinterpret_cast<const GroupGemmEntry *>(dp + b0 + b1), count, total_tiles,
                                       total_red, tile, h->gqueue, h->stream));
        span_end(h, e2, QCE_PHASE_GEMM_BATCHED);
    }
    for (const GroupPermute &p : post) {
        rs = run_group_permute(h, p, ws);
        if (rs != QCE_SUCCESS) return rs;
    }
    // the group's decision states (forget_batch_decisions resets them when
    // the workspace changes)
    h->dec_base = states;
    h->dec_map.clear();
    h->dec_host.clear();
    h->dec_count = 1;
    h->have_decision = false;
    h->last_on_device = false;
    if (first_state)
        for (int i = 0; i < count; ++i) (*first_state)[i] = off[i].st;
    return QCE_SUCCESS;
}

bool checked_numel(int rank, const int64_t *ext, int64_t &n) {
    n = 1;
    for (int a = 0; a < rank; ++a) {
        if (ext[a] < 1) return false;
        if (n > INT64_MAX / ext[a]) return false;
        n *= ext[a];
    }
    return true;
}

}  // namespace

extern "C" {

const char *qce_status_string(qce_status s) {
    switch (s) {
    case QCE_SUCCESS: return "QCE_SUCCESS";
    case QCE_ERR_INVALID_VALUE: return "QCE_ERR_INVALID_VALUE";
    case QCE_ERR_NOT_SUPPORTED: return "QCE_ERR_NOT_SUPPORTED";
    case QCE_ERR_ALLOC: return "QCE_ERR_ALLOC";
    case QCE_ERR_HIP: return "QCE_ERR_HIP";
    case QCE_ERR_INTERNAL: return "QCE_ERR_INTERNAL";
    }
    return "QCE_ERR_UNKNOWN";
}

const char *qce_last_error(const qce_handle *h) { return h ? h->err : "null handle"; }

qce_status qce_create(qce_handle **out, int device) {
    if (!out) return QCE_ERR_INVALID_VALUE;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return QCE_ERR_INVALID_VALUE;
    qce_handle *h = new qce_handle();
    h->device = device;
    if (const char *v = getenv("QCE_MODE")) {
        if (!parse_mode(v, &h->mode)) { delete h; return QCE_ERR_INVALID_VALUE; }
    }
    if (const char *v = getenv("QCE_UNDERFLOW_TOL")) {
        if (!parse_double(v, &h->t) || !(h->t >= 0 && h->t <= 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
    }
    if (const char *v = getenv("QCE_BF16X3_TOL")) {
        if (!parse_double(v, &h->t3) || !(h->t3 >= 0 && h->t3 <= 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
    }
    if (const char *v = getenv("QCE_AUTO_MIN_DIM")) {
        if (!parse_i64(v, &h->auto_min) || h->auto_min < 0) { delete h; return QCE_ERR_INVALID_VALUE; }
    }
    if (const char *v = getenv("QCE_EMUL_MIN_DIM")) {
        if (!parse_i64(v, &h->emul_min) || h->emul_min < 0) { delete h; return QCE_ERR_INVALID_VALUE; }
    }
    if (const char *v = getenv("QCE_FUSED_GATHER")) {
        int64_t f = 0;
        if (!parse_i64(v, &f) || (f != 0 && f != 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
        h->fused_gather = f == 1;
    }
    if (const char *v = getenv("QCE_SMALLK")) {
        int64_t f = 0;
        if (!parse_i64(v, &f) || (f != 0 && f != 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
        h->smallk = f == 1;
    }
    if (const char *v = getenv("QCE_GEMM_SIZE_POLICY")) {
        int64_t f = 0;
        if (!parse_i64(v, &f) || (f != 0 && f != 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
        h->gemm_policy = f == 1;
    }
    if (const char *v = getenv("QCE_GROUPED_GEMM")) {
        int64_t f = 0;
        if (!parse_i64(v, &f) || (f != 0 && f != 1)) { delete h; return QCE_ERR_INVALID_VALUE; }
        h->group_gemms = f == 1;
    }
    if (h->emul_min > h->auto_min) { delete h; return QCE_ERR_INVALID_VALUE; }
    DeviceGuard g(device);
    auto release = [h]() {
        if (h->st) (void)hipFree(h->st);
        if (h->fid_partials) (void)hipFree(h->fid_partials);
        if (h->mode_log) (void)hipFree(h->mode_log);
        if (h->gqueue) (void)hipFree(h->gqueue);
        delete h;
    };
    if (hipMalloc(&h->st, sizeof(DevState)) != hipSuccess ||
        hipMalloc(&h->fid_partials, sizeof(double) * 4 * kFidBlocks) != hipSuccess ||
        hipMalloc(&h->mode_log, sizeof(int) * kLogCap) != hipSuccess ||
        hipMalloc(&h->gqueue, sizeof(unsigned int) * kGroupQueueWords) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return QCE_ERR_ALLOC;
    }
    if (scratch_init(device) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return QCE_ERR_HIP;
    }
    if (hipMemset(h->st, 0, sizeof(DevState)) != hipSuccess ||
        hipMemset(h->gqueue, 0, sizeof(unsigned int) * kGroupQueueWords) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        release();
        return QCE_ERR_HIP;
    }
    h->dec_base = h->st;
    *out = h;
    return QCE_SUCCESS;
}

qce_status qce_destroy(qce_handle *h) {
    if (!h) return QCE_SUCCESS;
    DeviceGuard g(h->device);
    qce_status rc = QCE_SUCCESS;
    if (hipStreamSynchronize(h->stream) != hipSuccess) rc = QCE_ERR_HIP;
    if (h->ws && h->ws_owned) (void)hipFree(h->ws);
    for (auto &r : h->recs) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    (void)hipFree(h->st);
    (void)hipFree(h->fid_partials);
    (void)hipFree(h->mode_log);
    (void)hipFree(h->gqueue);
    if (h->grp_dev) (void)hipFree(h->grp_dev);
    if (h->grp_host) (void)hipHostFree(h->grp_host);
    for (auto &pr : h->grp_old) {
        (void)hipFree(pr.first);
        (void)hipHostFree(pr.second);
    }
    delete h;
    return rc;
}

qce_status qce_set_stream(qce_handle *h, void *stream) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    hipStream_t ns = static_cast<hipStream_t>(stream);
    if (ns != h->stream) QCE_HIP(h, hipStreamSynchronize(h->stream));
    h->stream = ns;
    return QCE_SUCCESS;
}

qce_status qce_set_mode(qce_handle *h, qce_mode m) {
    if (!h || (int)m < QCE_MODE_FP16X2 || (int)m > QCE_MODE_AUTO) return QCE_ERR_INVALID_VALUE;
    h->mode = m;
    return QCE_SUCCESS;
}

qce_status qce_get_mode(const qce_handle *h, qce_mode *m) {
    if (!h || !m) return QCE_ERR_INVALID_VALUE;
    *m = h->mode;
    return QCE_SUCCESS;
}

qce_status qce_set_underflow_tolerance(qce_handle *h, double t, double t3) {
    if (!h || !(t >= 0 && t <= 1) || !(t3 >= 0 && t3 <= 1)) return QCE_ERR_INVALID_VALUE;
    h->t = t;
    h->t3 = t3;
    return QCE_SUCCESS;
}

qce_status qce_set_size_policy(qce_handle *h, int64_t auto_min, int64_t emul_min) {
    if (!h || emul_min < 0 || emul_min > auto_min) return QCE_ERR_INVALID_VALUE;
    h->auto_min = auto_min;
    h->emul_min = emul_min;
    return QCE_SUCCESS;
}

qce_status qce_set_gemm_tile(qce_handle *h, int32_t tile) {
    if (!h || (tile != 0 && tile != 64 && tile != 128)) return QCE_ERR_INVALID_VALUE;
    h->gemm_tile = tile;
    return QCE_SUCCESS;
}

qce_status qce_set_gemm_size_policy(qce_handle *h, int32_t enable) {
    if (!h || (enable != 0 && enable != 1)) return QCE_ERR_INVALID_VALUE;
    h->gemm_policy = enable == 1;
    return QCE_SUCCESS;
}

qce_status qce_get_size_policy(const qce_handle *h, int64_t *auto_min, int64_t *emul_min) {
    if (!h || !auto_min || !emul_min) return QCE_ERR_INVALID_VALUE;
    *auto_min = h->auto_min;
    *emul_min = h->emul_min;
    return QCE_SUCCESS;
}

qce_status qce_set_workspace(qce_handle *h, void *ptr, size_t bytes) {
    if (!h || (ptr == nullptr) != (bytes == 0)) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    if (h->ws && h->ws_owned) {
        QCE_HIP(h, hipStreamSynchronize(h->stream));
        QCE_HIP(h, hipFree(h->ws));
    }
    h->ws = ptr;
    h->ws_bytes = bytes;
    h->ws_owned = ptr == nullptr;
    forget_batch_decisions(h);
    return QCE_SUCCESS;
}

size_t qce_cgemm_workspace_size(int64_t m, int64_t n, int64_t k) {
    if (m <= 0 || n <= 0 || k < 0) return 0;
    return cgemm_ws_bytes(m, n, k);
}

size_t qce_cgemm_batched_workspace_size(int64_t m, int64_t n, int64_t k, int64_t batch) {
    if (m <= 0 || n <= 0 || k < 0 || batch <= 0 || batch > kMaxBatch) return 0;
    return cgemm_ws_bytes(m, n, k, (int)batch);
}

namespace {
// Argument checks shared by the single-GEMM entry points; QCE_SUCCESS with
// *noop set when there is nothing to do.
qce_status cgemm_check(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n, int64_t k,
                       const qce_c32 *A, int64_t lda, const qce_c32 *B, int64_t ldb, const qce_c32 *C,
                       int64_t ldc, bool *noop) {
    *noop = false;
    if (!valid_op(opA) || !valid_op(opB)) return fail(h, QCE_ERR_INVALID_VALUE, "bad op");
    if (m < 0 || n < 0 || k < 0) return fail(h, QCE_ERR_INVALID_VALUE, "negative size");
    const int64_t arows = opA == QCE_OP_N ? m : k, brows = opB == QCE_OP_N ? k : n;
    if (lda < std::max<int64_t>(1, arows) || ldb < std::max<int64_t>(1, brows) ||
        ldc < std::max<int64_t>(1, m))
        return fail(h, QCE_ERR_INVALID_VALUE, "leading dimension too small");
    if (m == 0 || n == 0) {
        *noop = true;
        return QCE_SUCCESS;
    }
    if (!C || (k > 0 && (!A || !B))) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
         reinterpret_cast<uintptr_t>(C)) & 7)
        return fail(h, QCE_ERR_INVALID_VALUE, "pointer not 8-byte aligned");
    return QCE_SUCCESS;
}
}  // namespace

qce_status qce_cgemm_emulated(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                              int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                              const qce_c32 *B, int64_t ldb, const qce_c32 *beta, qce_c32 *C,
                              int64_t ldc) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    bool noop = false;
    qce_status st = cgemm_check(h, opA, opB, m, n, k, A, lda, B, ldb, C, ldc, &noop);
    if (st != QCE_SUCCESS || noop) return st;
    DeviceGuard g(h->device);
    const float2 al = alpha ? make_float2(alpha->re, alpha->im) : make_float2(1.f, 0.f);
    const float2 be = beta ? make_float2(beta->re, beta->im) : make_float2(0.f, 0.f);
    st = ensure_ws(h, cgemm_ws_bytes(m, n, k));
    if (st != QCE_SUCCESS) return st;
    OperandView va{reinterpret_cast<const float2 *>(A), lda, opA != QCE_OP_N, opA == QCE_OP_C};
    OperandView vb{reinterpret_cast<const float2 *>(B), ldb, opB == QCE_OP_N, opB == QCE_OP_C};
    return cgemm_core(h, gemm_mode(h, m, n, k), va, vb, m, n, k, al, be, reinterpret_cast<float2 *>(C), ldc,
                      static_cast<char *>(h->ws));
}

size_t qce_noalloc_scratch_bytes(void) { return kScratchBytes; }

qce_status qce_cgemm_emulated_noalloc(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                                      int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                                      const qce_c32 *B, int64_t ldb, const qce_c32 *beta, qce_c32 *C,
                                      int64_t ldc) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    bool noop = false;
    qce_status st = cgemm_check(h, opA, opB, m, n, k, A, lda, B, ldb, C, ldc, &noop);
    if (st != QCE_SUCCESS || noop) return st;
    const size_t need = cgemm_ws_bytes(m, n, k);
    if (need > kScratchBytes)
        return fail(h, QCE_ERR_INVALID_VALUE,
                    "a %lld x %lld x %lld GEMM needs %zu bytes of scratch; the fixed scratch holds %zu",
                    (long long)m, (long long)n, (long long)k, need, kScratchBytes);
    void *ws = scratch_ptr(h->device);
    if (!ws) return fail(h, QCE_ERR_INTERNAL, "no scratch address for device %d", h->device);
    DeviceGuard g(h->device);
    const float2 al = alpha ? make_float2(alpha->re, alpha->im) : make_float2(1.f, 0.f);
    const float2 be = beta ? make_float2(beta->re, beta->im) : make_float2(0.f, 0.f);
    OperandView va{reinterpret_cast<const float2 *>(A), lda, opA != QCE_OP_N, opA == QCE_OP_C};
    OperandView vb{reinterpret_cast<const float2 *>(B), ldb, opB == QCE_OP_N, opB == QCE_OP_C};
    // no timing records here: a new event could allocate
    const bool timing = h->timing;
    h->timing = false;
    st = cgemm_core(h, gemm_mode(h, m, n, k), va, vb, m, n, k, al, be, reinterpret_cast<float2 *>(C), ldc,
                    static_cast<char *>(ws));
    h->timing = timing;
    return st;
}

qce_status qce_cgemm_strided_batched(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                                     int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                                     int64_t strideA, const qce_c32 *B, int64_t ldb, int64_t strideB,
                                     const qce_c32 *beta, qce_c32 *C, int64_t ldc, int64_t strideC,
                                     int64_t batch) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (!valid_op(opA) || !valid_op(opB)) return fail(h, QCE_ERR_INVALID_VALUE, "bad op");
    if (m < 0 || n < 0 || k < 0 || batch < 0) return fail(h, QCE_ERR_INVALID_VALUE, "negative size");
    if (batch > kMaxBatch) return fail(h, QCE_ERR_INVALID_VALUE, "batch %lld > %d", (long long)batch, kMaxBatch);
    const int64_t arows = opA == QCE_OP_N ? m : k, brows = opB == QCE_OP_N ? k : n;
    if (lda < std::max<int64_t>(1, arows) || ldb < std::max<int64_t>(1, brows) ||
        ldc < std::max<int64_t>(1, m))
        return fail(h, QCE_ERR_INVALID_VALUE, "leading dimension too small");
    if (strideA < 0 || strideB < 0 || strideC < 0) return fail(h, QCE_ERR_INVALID_VALUE, "negative stride");
    if (batch > 1 && m > 0 && n > 0 && strideC < ldc * (n - 1) + m)
        return fail(h, QCE_ERR_INVALID_VALUE, "C entries overlap (strideC too small)");
    if (m == 0 || n == 0 || batch == 0) return QCE_SUCCESS;
    if (!C || (k > 0 && (!A || !B))) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
         reinterpret_cast<uintptr_t>(C)) & 7)
        return fail(h, QCE_ERR_INVALID_VALUE, "pointer not 8-byte aligned");
    DeviceGuard g(h->device);
    const float2 al = alpha ? make_float2(alpha->re, alpha->im) : make_float2(1.f, 0.f);
    const float2 be = beta ? make_float2(beta->re, beta->im) : make_float2(0.f, 0.f);
    qce_status st = ensure_ws(h, cgemm_ws_bytes(m, n, k, (int)batch));
    if (st != QCE_SUCCESS) return st;
    OperandView va{reinterpret_cast<const float2 *>(A), lda, opA != QCE_OP_N, opA == QCE_OP_C};
    OperandView vb{reinterpret_cast<const float2 *>(B), ldb, opB == QCE_OP_N, opB == QCE_OP_C};
    Batch bt;
    bt.count = (int)batch;
    bt.sa = strideA;
    bt.sb = strideB;
    bt.sc = strideC;
    return cgemm_core(h, gemm_mode(h, m, n, k), va, vb, m, n, k, al, be, reinterpret_cast<float2 *>(C), ldc,
                      static_cast<char *>(h->ws), bt);
}

qce_status qce_cgemm_grouped(qce_handle *h, int64_t count, const qce_gemm_desc *descs) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (count < 0 || count > kMaxBatch + 1)
        return fail(h, QCE_ERR_INVALID_VALUE, "group of %lld GEMMs (0..%d)", (long long)count, kMaxBatch + 1);
    if (count == 0) return QCE_SUCCESS;
    if (!descs) return fail(h, QCE_ERR_INVALID_VALUE, "null descriptor array");
    std::vector<char> noop((size_t)count, 0);
    for (int64_t i = 0; i < count; ++i) {
        const qce_gemm_desc &d = descs[i];
        bool nop = false;
        qce_status st = cgemm_check(h, d.opA, d.opB, d.m, d.n, d.k, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, &nop);
        if (st != QCE_SUCCESS) {
            char msg[sizeof(h->err)];
            snprintf(msg, sizeof(msg), "%s", h->err);
            return fail(h, st, "entry %lld: %s", (long long)i, msg);
        }
        noop[(size_t)i] = nop;
    }
    DeviceGuard g(h->device);
    std::vector<GroupItem> items;
    std::vector<int64_t> direct;  // irregular shapes and k == 0: their own kernels
    for (int64_t i = 0; i < count; ++i) {
        if (noop[(size_t)i]) continue;
        const qce_gemm_desc &d = descs[i];
        if (d.k == 0 || irregular_shape(d.m, d.n, d.k)) {
            direct.push_back(i);
            continue;
        }
        GroupItem it;
        it.mode = gemm_mode(h, d.m, d.n, d.k);
        it.a = GroupOperand{reinterpret_cast<const float2 *>(d.A), d.lda, d.opA != QCE_OP_N, d.opA == QCE_OP_C, -1};
        it.b = GroupOperand{reinterpret_cast<const float2 *>(d.B), d.ldb, d.opB == QCE_OP_N, d.opB == QCE_OP_C, -1};
        it.m = d.m;
        it.n = d.n;
        it.k = d.k;
        it.alpha = make_float2(d.alpha.re, d.alpha.im);
        it.beta = make_float2(d.beta.re, d.beta.im);
        it.C = reinterpret_cast<float2 *>(d.C);
        it.ldc = d.ldc;
        it.index = i;
        items.push_back(it);
    }
    // the workspace use of these ends before the group's, in stream order
    for (int64_t i : direct) {
        const qce_gemm_desc &d = descs[i];
        qce_status st = ensure_ws(h, cgemm_ws_bytes(d.m, d.n, d.k));
        if (st != QCE_SUCCESS) return st;
        OperandView va{reinterpret_cast<const float2 *>(d.A), d.lda, d.opA != QCE_OP_N, d.opA == QCE_OP_C};
        OperandView vb{reinterpret_cast<const float2 *>(d.B), d.ldb, d.opB == QCE_OP_N, d.opB == QCE_OP_C};
        st = cgemm_core(h, h->mode, va, vb, d.m, d.n, d.k, make_float2(d.alpha.re, d.alpha.im),
                        make_float2(d.beta.re, d.beta.im), reinterpret_cast<float2 *>(d.C), d.ldc,
                        static_cast<char *>(h->ws));
        if (st != QCE_SUCCESS) return st;
    }
    std::vector<int64_t> first;
    qce_status st = run_group_gemms(h, items, {}, {}, 0, &first);
    if (st != QCE_SUCCESS) return st;
    // decision records in the caller's order
    if (items.empty()) h->dec_base = h->st;
    h->dec_map.assign((size_t)count, 0);
    h->dec_host.clear();
    qce_decision hostrec{};
    hostrec.mode = QCE_MODE_FP32;  // irregular shapes, k == 0, empty outputs: FP32, no statistics
    for (int o = 0; o < 2; ++o) {
        hostrec.n2[o] = -1;
        hostrec.emax[o] = INT32_MIN;
    }
    for (int64_t i = 0; i < count; ++i) {
        h->dec_host.push_back(hostrec);
        h->dec_map[(size_t)i] = -(int64_t)h->dec_host.size();
    }
    for (size_t j = 0; j < items.size(); ++j) {
        if (first[j] >= 0) {
            h->dec_map[(size_t)items[j].index] = first[j];
        } else {
            h->dec_host[(size_t)items[j].index].mode = items[j].mode;
        }
    }
    h->dec_count = (int)count;
    h->have_decision = true;
    h->last_on_device = false;
    return QCE_SUCCESS;
}

qce_status qce_get_last_decision(qce_handle *h, qce_decision *out) {
    if (!h || !out) return QCE_ERR_INVALID_VALUE;
    if (!h->have_decision) return fail(h, QCE_ERR_INVALID_VALUE, "no GEMM has run on this handle");
    if (!h->dec_map.empty()) return qce_get_batch_decision(h, (int64_t)h->dec_map.size() - 1, out);
    DeviceGuard g(h->device);
    QCE_HIP(h, hipStreamSynchronize(h->stream));
    if (h->last_on_device) {
        QCE_HIP(h, hipMemcpy(out, &h->dec_base->last, sizeof(qce_decision), hipMemcpyDeviceToHost));
    } else {
        *out = h->last_host;
    }
    return QCE_SUCCESS;
}

qce_status qce_get_batch_decision(qce_handle *h, int64_t index, qce_decision *out) {
    if (!h || !out) return QCE_ERR_INVALID_VALUE;
    if (!h->have_decision) return fail(h, QCE_ERR_INVALID_VALUE, "no GEMM has run on this handle");
    if (index < 0 || index >= h->dec_count)
        return fail(h, QCE_ERR_INVALID_VALUE, "entry %lld of a batch of %d", (long long)index, h->dec_count);
    DeviceGuard g(h->device);
    QCE_HIP(h, hipStreamSynchronize(h->stream));
    if (!h->dec_map.empty()) {
        const int64_t w = h->dec_map[(size_t)index];
        if (w >= 0)
            QCE_HIP(h, hipMemcpy(out, &h->dec_base[w].last, sizeof(qce_decision), hipMemcpyDeviceToHost));
        else
            *out = h->dec_host[(size_t)(-1 - w)];
        return QCE_SUCCESS;
    }
    if (h->last_on_device) {
        QCE_HIP(h, hipMemcpy(out, &h->dec_base[index].last, sizeof(qce_decision), hipMemcpyDeviceToHost));
    } else {
        *out = h->last_host;
    }
    return QCE_SUCCESS;
}

qce_status qce_expstats(qce_handle *h, const qce_c32 *X, int64_t rows, int64_t cols, int64_t ld,
                        qce_decision *out) {
    if (!h || !out) return QCE_ERR_INVALID_VALUE;
    if (rows < 0 || cols < 0 || ld < std::max<int64_t>(1, rows) || (rows * cols > 0 && !X))
        return fail(h, QCE_ERR_INVALID_VALUE, "bad matrix");
    DeviceGuard g(h->device);
    hipStream_t s = h->stream;
    MatDesc a{reinterpret_cast<const float2 *>(X), rows, cols, ld, 0};
    MatDesc none{nullptr, 0, 0, 1, 0};
    if (rows == 0 || cols == 0) {
        *out = qce_decision{};
        out->emax[0] = out->emax[1] = INT32_MIN;
        out->stats_taken = 1;
        return QCE_SUCCESS;
    }
    qce_status sts = ensure_ws(h, stats_record_bytes(a, none));
    if (sts != QCE_SUCCESS) return sts;
    QCE_HIP(h, launch_stats(a, none, h->st, static_cast<StatsRecord *>(h->ws), h->t, h->t3, -1, nullptr, 0, s));
    QCE_HIP(h, hipStreamSynchronize(s));
    QCE_HIP(h, hipMemcpy(out, &h->st->last, sizeof(qce_decision), hipMemcpyDeviceToHost));
    return QCE_SUCCESS;
}

qce_status qce_split(qce_handle *h, qce_mode mode, int32_t shift, const qce_c32 *x, int64_t n,
                     uint16_t *planes) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (mode != QCE_MODE_FP16X2 && mode != QCE_MODE_BF16X3)
        return fail(h, QCE_ERR_NOT_SUPPORTED, "split is defined for FP16X2 and BF16X3");
    if (n < 0 || (n > 0 && (!x || !planes))) return fail(h, QCE_ERR_INVALID_VALUE, "bad buffers");
    if (mode == QCE_MODE_BF16X3 && shift != 0) return fail(h, QCE_ERR_INVALID_VALUE, "BF16X3 takes no shift");
    DeviceGuard g(h->device);
    QCE_HIP(h, launch_split_planar(mode, shift, reinterpret_cast<const float2 *>(x), n, planes, h->stream));
    return QCE_SUCCESS;
}

size_t qce_panel_bytes(qce_mode mode, int64_t rows, int64_t k) {
    if (rows <= 0 || k <= 0) return 0;
    const size_t per = mode == QCE_MODE_BF16X3 ? 12 : (mode == QCE_MODE_FP16X2 || mode == QCE_MODE_FP16X2_SCALED ||
                                                         mode == QCE_MODE_FP32) ? 8 : 0;
    return (size_t)round_up(rows, kPanelRows) * (size_t)round_up(k, kKPad) * per;
}

namespace {
qce_status panel_mode_check(qce_handle *h, qce_mode mode, int32_t shift) {
    if (mode != QCE_MODE_FP16X2 && mode != QCE_MODE_FP16X2_SCALED && mode != QCE_MODE_BF16X3 &&
        mode != QCE_MODE_FP32)
        return fail(h, QCE_ERR_INVALID_VALUE, "panels are written for FP16X2, FP16X2_SCALED, BF16X3 or FP32");
    if (mode != QCE_MODE_FP16X2_SCALED && shift != 0)
        return fail(h, QCE_ERR_INVALID_VALUE, "only FP16X2_SCALED takes a shift");
    if (shift < -150 || shift > 150) return fail(h, QCE_ERR_INVALID_VALUE, "shift out of range");
    return QCE_SUCCESS;
}
}  // namespace

qce_status qce_split_panels(qce_handle *h, qce_mode mode, int32_t shift, int32_t layout, int32_t conj,
                            const qce_c32 *X, int64_t rows, int64_t k, int64_t ld, void *panels) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    qce_status st = panel_mode_check(h, mode, shift);
    if (st != QCE_SUCCESS) return st;
    if (layout != 0 && layout != 1) return fail(h, QCE_ERR_INVALID_VALUE, "layout is 0 or 1");
    if (rows < 0 || k < 0) return fail(h, QCE_ERR_INVALID_VALUE, "negative size");
    if (rows == 0 || k == 0) return QCE_SUCCESS;
    if (ld < (layout == 0 ? rows : k)) return fail(h, QCE_ERR_INVALID_VALUE, "leading dimension too small");
    if (!X || !panels) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    if ((reinterpret_cast<uintptr_t>(X) & 7) || (reinterpret_cast<uintptr_t>(panels) & 15))
        return fail(h, QCE_ERR_INVALID_VALUE, "misaligned pointer");
    DeviceGuard g(h->device);
    QCE_HIP(h, launch_split_panels(reinterpret_cast<const float2 *>(X), ld, layout, conj != 0, rows, k, panels,
                                   nullptr, 0, mode, shift, h->stream));
    return QCE_SUCCESS;
}

qce_status qce_split_panels_bitmap(qce_handle *h, qce_mode mode, int32_t shift, const qce_c32 *X, int32_t nr,
                                   int32_t nk, const int32_t *rsh, const int32_t *ksh, void *panels) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    qce_status st = panel_mode_check(h, mode, shift);
    if (st != QCE_SUCCESS) return st;
    if (nr < 5 || nk < 4 || nr > 31 || nk > 31 || nr + nk > 40)
        return fail(h, QCE_ERR_INVALID_VALUE, "need 5 <= nr, 4 <= nk, nr, nk <= 31, nr + nk <= 40");
    if (!X || !panels || !rsh || !ksh) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    if ((reinterpret_cast<uintptr_t>(X) & 7) || (reinterpret_cast<uintptr_t>(panels) & 15))
        return fail(h, QCE_ERR_INVALID_VALUE, "misaligned pointer");
    int8_t r8[32], k8[32];
    for (int t = 0; t < nr; ++t) r8[t] = (int8_t)std::max(-1, std::min(127, rsh[t]));
    for (int t = 0; t < nk; ++t) k8[t] = (int8_t)std::max(-1, std::min(127, ksh[t]));
    const GatherMap gm = gather_map_from_shifts(nr, nk, r8, k8);
    if (!gather_map_valid(gm))
        return fail(h, QCE_ERR_INVALID_VALUE, "rsh and ksh are not a permutation of 0..nr+nk-1");
    DeviceGuard g(h->device);
    QCE_HIP(h, launch_split_gather(reinterpret_cast<const float2 *>(X), gm, panels, nullptr, 0, mode, shift,
                                   h->stream));
    return QCE_SUCCESS;
}

qce_status qce_permute(qce_handle *h, const qce_tensor *x, const void *X, const int32_t *perm,
                       void *Y) {
    if (!h || !x || x->rank < 0 || (x->rank > 0 && (!x->extents || !perm)))
        return QCE_ERR_INVALID_VALUE;
    if (x->rank > 64) return fail(h, QCE_ERR_NOT_SUPPORTED, "rank above 64");
    int64_t n = 0;
    if (!checked_numel(x->rank, x->extents, n)) return fail(h, QCE_ERR_INVALID_VALUE, "bad extents");
    std::vector<char> seen(x->rank, 0);
    for (int a = 0; a < x->rank; ++a) {
        if (perm[a] < 0 || perm[a] >= x->rank || seen[perm[a]])
            return fail(h, QCE_ERR_INVALID_VALUE, "not a permutation");
        seen[perm[a]] = 1;
    }
    if (!X || !Y) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    DeviceGuard g(h->device);
    return run_permute(h, x->rank, x->extents, perm, static_cast<const float2 *>(X),
                       static_cast<float2 *>(Y));
}

qce_status qce_accumulate_f64(qce_handle *h, const qce_c32 *src, double *acc2) {
    if (!h || !src || !acc2) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    hipEvent_t e0 = span_begin(h);
    QCE_HIP(h, launch_accumulate_f64(reinterpret_cast<const float2 *>(src), acc2, h->stream));
    span_end(h, e0, QCE_PHASE_OTHER);
    return QCE_SUCCESS;
}

qce_status qce_accumulate_n_f64(qce_handle *h, const qce_c32 *src, int64_t n, double *acc2) {
    if (!h || !acc2 || n < 0 || (n > 0 && !src)) return QCE_ERR_INVALID_VALUE;
    if (n == 0) return QCE_SUCCESS;
    DeviceGuard g(h->device);
    const int nb = (int)std::min<int64_t>(kFidBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipEvent_t e0 = span_begin(h);
    QCE_HIP(h, launch_accumulate_n_f64(reinterpret_cast<const float2 *>(src), n, h->fid_partials, nb, acc2,
                                       h->stream));
    span_end(h, e0, QCE_PHASE_OTHER);
    return QCE_SUCCESS;
}

qce_status qce_fidelity_f64(qce_handle *h, const qce_c32 *a, const qce_c32 *b, int64_t n,
                            double *out4) {
    if (!h || !out4 || n < 0 || (n > 0 && (!a || !b))) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    int nb = (int)std::min<int64_t>(kFidBlocks, std::max<int64_t>(1, (n + 255) / 256));
    QCE_HIP(h, launch_fidelity_f64(reinterpret_cast<const float2 *>(a), reinterpret_cast<const float2 *>(b),
                                   n, h->fid_partials, nb, out4, h->stream));
    return QCE_SUCCESS;
}

// ---------------------------------------------------------------------------
// Tensor contraction by TTGT.
// ---------------------------------------------------------------------------
qce_status qce_contract(qce_handle *h, const qce_tensor *a, const void *A, const int32_t *la,
                        const qce_tensor *b, const void *B, const int32_t *lb,
                        const qce_tensor *c, void *C, const int32_t *lc) {
    if (!h || !a || !b || !c) return QCE_ERR_INVALID_VALUE;
    const int ra = a->rank, rb = b->rank, rc = c->rank;
    if (ra < 0 || rb < 0 || rc < 0 || ra > 64 || rb > 64 || rc > 64)
        return fail(h, QCE_ERR_INVALID_VALUE, "bad rank");
    if ((ra && (!a->extents || !la)) || (rb && (!b->extents || !lb)) || (rc && (!c->extents || !lc)))
        return fail(h, QCE_ERR_INVALID_VALUE, "missing extents or labels");
    int64_t na, nb_, nc;
    if (!checked_numel(ra, a->extents, na) || !checked_numel(rb, b->extents, nb_) ||
        !checked_numel(rc, c->extents, nc))
        return fail(h, QCE_ERR_INVALID_VALUE, "bad extents");
    if (!A || !B || !C) return fail(h, QCE_ERR_INVALID_VALUE, "null pointer");
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(C)) & 7)
        return fail(h, QCE_ERR_INVALID_VALUE, "pointer not 8-byte aligned");
    auto find = [](const int32_t *l, int r, int32_t x) {
        for (int i = 0; i < r; ++i)
            if (l[i] == x) return i;
        return -1;
    };
    auto unique = [&](const int32_t *l, int r) {
        for (int i = 0; i < r; ++i)
            if (find(l, i, l[i]) >= 0) return false;
        return true;
    };
    if (!unique(la, ra) || !unique(lb, rb) || !unique(lc, rc))
        return fail(h, QCE_ERR_INVALID_VALUE, "duplicate label within a tensor");
    std::vector<int32_t> K, FA, FB, BT;  // labels in A's / B's order
    for (int i = 0; i < ra; ++i) {
        const int jb = find(lb, rb, la[i]), jc = find(lc, rc, la[i]);
        if (jb >= 0) {
            if (a->extents[i] != b->extents[jb]) return fail(h, QCE_ERR_INVALID_VALUE, "extent mismatch");
            if (jc >= 0) {
                if (c->extents[jc] != a->extents[i]) return fail(h, QCE_ERR_INVALID_VALUE, "extent mismatch");
                BT.push_back(la[i]);
            } else {
                K.push_back(la[i]);
            }
        } else {
            if (jc < 0) return fail(h, QCE_ERR_NOT_SUPPORTED, "label %d summed over one input", la[i]);
            if (c->extents[jc] != a->extents[i]) return fail(h, QCE_ERR_INVALID_VALUE, "extent mismatch");
            FA.push_back(la[i]);
        }
    }
    for (int i = 0; i < rb; ++i) {
        if (find(la, ra, lb[i]) >= 0) continue;
        const int jc = find(lc, rc, lb[i]);
        if (jc < 0) return fail(h, QCE_ERR_NOT_SUPPORTED, "label %d summed over one input", lb[i]);
        if (c->extents[jc] != b->extents[i]) return fail(h, QCE_ERR_INVALID_VALUE, "extent mismatch");
        FB.push_back(lb[i]);
    }
    if ((int)(FA.size() + FB.size() + BT.size()) != rc)
        return fail(h, QCE_ERR_INVALID_VALUE, "output label not in any input");

    auto ext_of = [&](int32_t lab) -> int64_t {
        int i = find(la, ra, lab);
        if (i >= 0) return a->extents[i];
        return b->extents[find(lb, rb, lab)];
    };
    auto prod = [&](const std::vector<int32_t> &ls) {
        int64_t p = 1;
        for (int32_t x : ls) p *= ext_of(x);
        return p;
    };
    // Inside a group (qce_group_begin): a contraction the GEMM path would send
    // to the irregular-shape kernel, and small enough, is recorded and runs at
    // qce_group_end in one launch with the group's other small contractions.
    if (h->grouping) {
        SmallItem it{};
        if (small_item(a, la, b, lb, c, lc, K, ext_of, prod(FA), prod(FB), prod(K), nc, it)) {
            it.A = static_cast<const float2 *>(A);
            it.B = static_cast<const float2 *>(B);
            it.C = static_cast<float2 *>(C);
            h->pending.push_back(it);
            return QCE_SUCCESS;
        }
    }
    // batch labels (in A, B and C): one independent GEMM per value, outermost
    // everywhere, in the order C lists them
    std::vector<int32_t> BO;
    for (int i = 0; i < rc; ++i)
        if (std::find(BT.begin(), BT.end(), lc[i]) != BT.end()) BO.push_back(lc[i]);
    const int nbt = (int)BO.size();
    const int64_t kk = prod(K), ma = prod(FA), nb = prod(FB), count = prod(BO);
    bool bt_front = true;
    for (int i = 0; i < nbt; ++i)
        if (lc[i] != BO[i]) bt_front = false;

    // Output: C row-major with labels lc = [BO][rest].  Per batch entry the
    // rest is, as a column-major matrix, m x n when rest = [free labels of
    // the "GEMM-B" operand][free labels of the "GEMM-A" operand].  Try both
    // roles; otherwise compute into a temporary [BO][FB (B order)][FA (A
    // order)] and permute.
    const int32_t *lcr = lc + nbt;
    const int rcr = rc - nbt;
    auto is_set_block = [&](int off, int len, const std::vector<int32_t> &set) {
        if (len != (int)set.size()) return false;
        for (int i = 0; i < len; ++i)
            if (std::find(set.begin(), set.end(), lcr[off + i]) == set.end()) return false;
        return true;
    };
    bool swap = false, out_perm = false;
    std::vector<int32_t> SA, SB;  // free-label order required of GEMM-A / GEMM-B operand
    if (bt_front && is_set_block(rcr - (int)FA.size(), (int)FA.size(), FA) && is_set_block(0, (int)FB.size(), FB)) {
        SA.assign(lcr + rcr - FA.size(), lcr + rcr);
        SB.assign(lcr, lcr + FB.size());
    } else if (bt_front && is_set_block(rcr - (int)FB.size(), (int)FB.size(), FB) &&
               is_set_block(0, (int)FA.size(), FA)) {
        swap = true;
        SA.assign(lcr + rcr - FB.size(), lcr + rcr);
        SB.assign(lcr, lcr + FA.size());
    } else {
        out_perm = true;
        SA = FA;
        SB = FB;
    }
    // GEMM-A = (swap ? B : A), GEMM-B = the other.
    const int32_t *lx = swap ? lb : la, *ly = swap ? la : lb;
    const int rx = swap ? rb : ra, ry = swap ? ra : rb;
    const void *X = swap ? B : A, *Y = swap ? A : B;
    const int64_t *ex = swap ? b->extents : a->extents, *ey = swap ? a->extents : b->extents;
    const int64_t m = swap ? nb : ma, n = swap ? ma : nb;

    // Does operand (labels l) hold [BO][K][F] or [BO][F][K] with the given
    // orders?  0: [K][F], 1: [F][K], -1: neither
    auto layout = [&](const int32_t *l, int r, const std::vector<int32_t> &korder,
                      const std::vector<int32_t> &forder) -> int {
        for (int i = 0; i < nbt; ++i)
            if (l[i] != BO[i]) return -1;
        const int32_t *q = l + nbt;
        const int rq = r - nbt;
        bool kf = true, fk = true;
        const int nk = (int)korder.size(), nf = (int)forder.size();
        for (int i = 0; i < rq; ++i) {
            if (i < nk ? q[i] != korder[i] : q[i] != forder[i - nk]) kf = false;
            if (i < nf ? q[i] != forder[i] : q[i] != korder[i - nf]) fk = false;
        }
        return kf ? 0 : (fk ? 1 : -1);
    };
    auto korder_of = [&](const int32_t *l, int r) {
        std::vector<int32_t> ko;
        for (int i = 0; i < r; ++i)
            if (std::find(K.begin(), K.end(), l[i]) != K.end()) ko.push_back(l[i]);
        return ko;
    };
    // choose the K order (from X or from Y) that permutes fewer elements
    std::vector<int32_t> kx = korder_of(lx, rx), ky = korder_of(ly, ry);
    int64_t sx = 1, sy = 1;
    for (int i = 0; i < rx; ++i) sx *= ex[i];
    for (int i = 0; i < ry; ++i) sy *= ey[i];
    auto cost = [&](const std::vector<int32_t> &ko) {
        int64_t c0 = 0;
        if (layout(lx, rx, ko, SA) < 0) c0 += sx;
        if (layout(ly, ry, ko, SB) < 0) c0 += sy;
        return c0;
    };
    std::vector<int32_t> korder = cost(kx) <= cost(ky) ? kx : ky;
    int lay_x = layout(lx, rx, korder, SA), lay_y = layout(ly, ry, korder, SB);

    // Permute fused into the split (every extent 2, no batch labels, a
    // matrix-core shape): an operand in neither [K][F] nor [F][K] order is
    // read by the split kernel through its bit permutation, one read
    // instead of a permuted copy plus a read.  The kernel loads 64 x 64
    // tiles whose bits are the last six labels of the F order and of the K
    // order; the longest run of the operand's own last labels inside the
    // tile is read contiguously.  Where a run is below 2^5 elements the
    // six tile K labels are picked greedily, each time the next label of
    // the operand with the shorter run; an operand left with a run below
    // 2^3 elements (64 bytes) is permuted as before.
    bool gx = false, gy = false;
    GatherMap gmx, gmy;
    bool fuse = nbt == 0 && h->fused_gather && !irregular_shape(m, n, kk) && (lay_x < 0 || lay_y < 0) &&
                SA.size() <= 31 && SB.size() <= 31 && K.size() <= 31;
    for (int i = 0; fuse && i < ra; ++i) fuse = a->extents[i] == 2;
    for (int i = 0; fuse && i < rb; ++i) fuse = b->extents[i] == 2;
    if (fuse) {
        auto in_last6 = [](const std::vector<int32_t> &v, int32_t lab) {
            for (size_t i = v.size() > 6 ? v.size() - 6 : 0; i < v.size(); ++i)
                if (v[i] == lab) return true;
            return false;
        };
        auto run_of = [&](const int32_t *l, int r, const std::vector<int32_t> &F,
                          const std::vector<int32_t> &ko) {
            int run = 0;
            for (int i = r - 1; i >= 0 && (in_last6(F, l[i]) || in_last6(ko, l[i])); --i) ++run;
            return run;
        };
        constexpr int kMinRun = 3, kGoodRun = 5;
        if ((lay_x < 0 && run_of(lx, rx, SA, korder) < kGoodRun) ||
            (lay_y < 0 && run_of(ly, ry, SB, korder) < kGoodRun)) {
            std::vector<int32_t> tk;
            auto in_tk = [&](int32_t lab) { return std::find(tk.begin(), tk.end(), lab) != tk.end(); };
            // index in l of the operand's next label outside the tile, if a
            // K label (-1: a full run, or capped by an F label)
            auto next_k = [&](const int32_t *l, int r, const std::vector<int32_t> &F, int &run) {
                run = 0;
                for (int i = r - 1; i >= 0; --i) {
                    if (in_last6(F, l[i]) || in_tk(l[i])) {
                        ++run;
                        continue;
                    }
                    return std::find(K.begin(), K.end(), l[i]) != K.end() ? i : -1;
                }
                return -1;
            };
            while (tk.size() < std::min<size_t>(6, K.size())) {
                int run_x = 0, run_y = 0;
                const int ix = next_k(lx, rx, SA, run_x), iy = next_k(ly, ry, SB, run_y);
                if (ix >= 0 && (iy < 0 || run_x <= run_y)) tk.push_back(lx[ix]);
                else if (iy >= 0) tk.push_back(ly[iy]);
                else break;
            }
            std::vector<int32_t> ko;
            for (int32_t lab : korder)
                if (!in_tk(lab)) ko.push_back(lab);
            for (int32_t lab : korder)
                if (in_tk(lab)) ko.push_back(lab);
            korder = ko;
            lay_x = layout(lx, rx, korder, SA);
            lay_y = layout(ly, ry, korder, SB);
        }
        // P[r][l]: r's bit t is label F[|F| - 1 - t], l's bit t is label
        // korder[|K| - 1 - t]; a label at position i of l holds stride 2^(r-1-i)
        auto make_map = [&](const int32_t *l, int r, const std::vector<int32_t> &F) {
            const int nr = (int)F.size(), nk = (int)korder.size();
            int8_t rsh[32], ksh[32];
            for (int t = 0; t < nr; ++t) rsh[t] = (int8_t)(r - 1 - find(l, r, F[nr - 1 - t]));
            for (int t = 0; t < nk; ++t) ksh[t] = (int8_t)(r - 1 - find(l, r, korder[nk - 1 - t]));
            return gather_map_from_shifts(nr, nk, rsh, ksh);
        };
        if (lay_x < 0 && run_of(lx, rx, SA, korder) >= kMinRun) {
            gmx = make_map(lx, rx, SA);
            gx = gather_map_valid(gmx);
        }
        if (lay_y < 0 && run_of(ly, ry, SB, korder) >= kMinRun) {
            gmy = make_map(ly, ry, SB);
            gy = gather_map_valid(gmy);
        }
    }

    // A full contraction (every label summed, every extent 2) of two
    // tensors in different label orders: one pass reads the permuted
    // operand through the tile of its bit permutation and sums the
    // products (no permuted copy).
    if (h->fused_gather && nbt == 0 && FA.empty() && FB.empty() && kk > 1 && (lay_x < 0) != (lay_y < 0)) {
        bool two = true;
        for (int i = 0; two && i < ra; ++i) two = a->extents[i] == 2;
        for (int i = 0; two && i < rb; ++i) two = b->extents[i] == 2;
        const bool px = lay_x < 0;
        const int32_t *lp = px ? lx : ly;
        const int rp = px ? rx : ry;
        std::vector<int32_t> perm;
        for (int32_t lab : korder) perm.push_back(find(lp, rp, lab));
        PermDesc d;
        int64_t total = 0;
        bool identity = false;
        if (two && rp == (int)korder.size() &&
            plan_permute(h, rp, px ? ex : ey, perm.data(), d, total, identity) == QCE_SUCCESS && !identity) {
            const int64_t parts = permuted_dot_partials(d);
            if (parts > 0) {
                DeviceGuard g(h->device);
                qce_status st = ensure_ws(h, align256((size_t)parts * sizeof(float2)));
                if (st != QCE_SUCCESS) return st;
                h->dec_base = h->st;
                h->dec_count = 1;
                h->dec_map.clear();
                h->dec_host.clear();
                hipEvent_t e0 = span_begin(h);
                QCE_HIP(h, launch_permuted_dot(static_cast<const float2 *>(px ? X : Y),
                                               static_cast<const float2 *>(px ? Y : X), d,
                                               static_cast<float2 *>(h->ws), static_cast<float2 *>(C),
                                               h->stream));
                span_end(h, e0, QCE_PHASE_GEMM_IRREGULAR);
                h->have_decision = true;
                h->last_on_device = false;
                h->last_host = qce_decision{};
                h->last_host.mode = QCE_MODE_FP32;
                for (int o = 0; o < 2; ++o) {
                    h->last_host.n2[o] = -1;
                    h->last_host.emax[o] = INT32_MIN;
                }
                return QCE_SUCCESS;
            }
        }
    }

    int mode = h->mode;
    if (mode == QCE_MODE_AUTO) mode = policy_mode(h, m, n, kk);
    // Inside a group, a GEMM of the panel path is recorded too: it runs at
    // qce_group_end with the group's other such GEMMs, one launch per phase
    // (its permutes run there as well, into temporaries of the group).
    const bool takes_stats = mode == QCE_MODE_AUTO || mode == QCE_MODE_FP16X2_SCALED;
    if (h->grouping && h->group_gemms && !gx && !gy && kk > 0 && m > 0 && n > 0 && !irregular_shape(m, n, kk) &&
        !(h->smallk && smallk_shape(m, n, kk)) && count >= 1 && count <= kMaxBatch &&
        (!takes_stats || h->gentries + count <= kMaxBatch + 1)) {
        GroupItem it;
        it.mode = mode;
        std::vector<GroupPermute> pre;
        size_t temp = h->gtemp;  // end of the group's temporaries
        auto operand = [&](int lay, const int32_t *l, int r, const int64_t *e, const void *src, int64_t rows,
                           const std::vector<int32_t> &forder, GroupOperand &v) -> qce_status {
            if (lay == 0) {  // [K][F]: column-major rows x k
                v = GroupOperand{static_cast<const float2 *>(src), std::max<int64_t>(1, rows), false, false, -1};
                return QCE_SUCCESS;
            }
            if (lay == 1) {  // [F][K]: column-major k x rows
                v = GroupOperand{static_cast<const float2 *>(src), std::max<int64_t>(1, kk), true, false, -1};
                return QCE_SUCCESS;
            }
            // permuted to [BO][K][F] in a temporary first
            std::vector<int32_t> perm;
            for (int32_t lab : BO) perm.push_back(find(l, r, lab));
            for (int32_t lab : korder) perm.push_back(find(l, r, lab));
            for (int32_t lab : forder) perm.push_back(find(l, r, lab));
            GroupPermute p;
            qce_status ps = plan_permute(h, r, e, perm.data(), p.d, p.total, p.identity);
            if (ps != QCE_SUCCESS) return ps;
            p.src = static_cast<const float2 *>(src);
            p.dst_ws = (int64_t)temp;
            temp += align256((size_t)p.total * sizeof(float2));
            v = GroupOperand{nullptr, std::max<int64_t>(1, rows), false, false, p.dst_ws};
            pre.push_back(p);
            return QCE_SUCCESS;
        };
        qce_status ps = operand(lay_x, lx, rx, ex, X, m, SA, it.a);
        if (ps == QCE_SUCCESS) ps = operand(lay_y, ly, ry, ey, Y, n, SB, it.b);
        if (ps != QCE_SUCCESS) return ps;
        GroupPermute post;
        if (out_perm) {
            // the GEMM writes [BO][SB][SA] (row-major) into a temporary, then
            // the permute to lc
            std::vector<int32_t> tl(BO);
            tl.insert(tl.end(), SB.begin(), SB.end());
            tl.insert(tl.end(), SA.begin(), SA.end());
            std::vector<int64_t> te;
            for (int32_t lab : tl) te.push_back(ext_of(lab));
            std::vector<int32_t> perm;
            for (int i = 0; i < rc; ++i) perm.push_back(find(tl.data(), rc, lc[i]));
            ps = plan_permute(h, rc, te.data(), perm.data(), post.d, post.total, post.identity);
            if (ps != QCE_SUCCESS) return ps;
            it.c_ws = (int64_t)temp;
            post.src_ws = it.c_ws;
            post.dst = static_cast<float2 *>(C);
            temp += align256((size_t)nc * 8);
        } else {
            it.C = static_cast<float2 *>(C);
        }
        it.m = m;
        it.n = n;
        it.k = kk;
        it.ldc = std::max<int64_t>(1, m);
        it.count = (int)count;
        it.sa = kk * m;
        it.sb = kk * n;
        it.sc = m * n;
        h->gitems.push_back(it);
        for (const GroupPermute &q : pre) h->gpre.push_back(q);
        if (out_perm) h->gpost.push_back(post);
        h->gtemp = temp;
        if (takes_stats) h->gentries += count;
        return QCE_SUCCESS;
    }

    // workspace: panels | permuted X | permuted Y | temporary C
    const int chunk = (int)std::min<int64_t>(std::max<int64_t>(count, 1), kMaxBatch);
    size_t off = align256(cgemm_ws_bytes(m, n, kk, chunk));
    const size_t offx = off;
    if (lay_x < 0 && !gx) off += align256((size_t)sx * 8);
    const size_t offy = off;
    if (lay_y < 0 && !gy) off += align256((size_t)sy * 8);
    const size_t offc = off;
    if (out_perm) off += align256((size_t)nc * 8);
    DeviceGuard g(h->device);
    qce_status st = ensure_ws(h, off);
    if (st != QCE_SUCCESS) return st;
    char *ws = static_cast<char *>(h->ws);

    auto permute_to_kf = [&](const int32_t *l, int r, const int64_t *e, const void *src,
                             const std::vector<int32_t> &forder, void *dst) -> qce_status {
        std::vector<int32_t> perm;
        for (int32_t lab : BO) perm.push_back(find(l, r, lab));
        for (int32_t lab : korder) perm.push_back(find(l, r, lab));
        for (int32_t lab : forder) perm.push_back(find(l, r, lab));
        return run_permute(h, r, e, perm.data(), static_cast<const float2 *>(src),
                           reinterpret_cast<float2 *>(dst));
    };
    OperandView vx, vy;
    if (gx) {
        vx = OperandView{static_cast<const float2 *>(X), m, false, false, &gmx};
    } else if (lay_x < 0) {
        st = permute_to_kf(lx, rx, ex, X, SA, ws + offx);
        if (st != QCE_SUCCESS) return st;
        vx = OperandView{reinterpret_cast<const float2 *>(ws + offx), std::max<int64_t>(1, m), false, false};
    } else if (lay_x == 0) {  // [K][F]: column-major m x k
        vx = OperandView{static_cast<const float2 *>(X), std::max<int64_t>(1, m), false, false};
    } else {  // [F][K]: column-major k x m
        vx = OperandView{static_cast<const float2 *>(X), std::max<int64_t>(1, kk), true, false};
    }
    if (gy) {
        vy = OperandView{static_cast<const float2 *>(Y), n, false, false, &gmy};
    } else if (lay_y < 0) {
        st = permute_to_kf(ly, ry, ey, Y, SB, ws + offy);
        if (st != QCE_SUCCESS) return st;
        vy = OperandView{reinterpret_cast<const float2 *>(ws + offy), std::max<int64_t>(1, n), false, false};
    } else if (lay_y == 0) {  // [K][F]: rows j contiguous: P[j][l] = y[j + l*n]
        vy = OperandView{static_cast<const float2 *>(Y), std::max<int64_t>(1, n), false, false};
    } else {  // [F][K]: P[j][l] = y[l + j*k]
        vy = OperandView{static_cast<const float2 *>(Y), std::max<int64_t>(1, kk), true, false};
    }
    float2 *Cg = out_perm ? reinterpret_cast<float2 *>(ws + offc) : static_cast<float2 *>(C);
    // batch entries in launches of at most kMaxBatch
    for (int64_t z0 = 0; z0 < std::max<int64_t>(count, 1); z0 += chunk) {
        Batch bt;
        bt.count = (int)std::min<int64_t>(chunk, std::max<int64_t>(count, 1) - z0);
        bt.sa = kk * m;
        bt.sb = kk * n;
        bt.sc = m * n;
        OperandView cx = vx, cy = vy;
        cx.ptr += z0 * bt.sa;
        cy.ptr += z0 * bt.sb;
        st = cgemm_core(h, mode, cx, cy, m, n, kk, make_float2(1.f, 0.f), make_float2(0.f, 0.f),
                        Cg + z0 * bt.sc, std::max<int64_t>(1, m), ws, bt);
        if (st != QCE_SUCCESS) return st;
    }
    if (out_perm) {
        // temporary has labels [BO][SB][SA] (row-major); permute to lc
        std::vector<int32_t> tl(BO);
        tl.insert(tl.end(), SB.begin(), SB.end());
        tl.insert(tl.end(), SA.begin(), SA.end());
        std::vector<int64_t> te;
        for (int32_t lab : tl) te.push_back(ext_of(lab));
        std::vector<int32_t> perm;
        for (int i = 0; i < rc; ++i) perm.push_back(find(tl.data(), rc, lc[i]));
        st = run_permute(h, rc, te.data(), perm.data(), Cg, static_cast<float2 *>(C));
        if (st != QCE_SUCCESS) return st;
    }
    return QCE_SUCCESS;
}

qce_status qce_group_begin(qce_handle *h) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (h->grouping) return fail(h, QCE_ERR_INVALID_VALUE, "a group is already open");
    h->grouping = true;
    h->pending.clear();
    h->gitems.clear();
    h->gpre.clear();
    h->gpost.clear();
    h->gtemp = 0;
    h->gentries = 0;
    return QCE_SUCCESS;
}

qce_status qce_group_end(qce_handle *h) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (!h->grouping) return fail(h, QCE_ERR_INVALID_VALUE, "no group is open");
    h->grouping = false;
    DeviceGuard g(h->device);
    // the recorded panel-path GEMMs (grouped launches)
    if (!h->gitems.empty()) {
        std::vector<GroupItem> items;
        std::vector<GroupPermute> pre, post;
        items.swap(h->gitems);
        pre.swap(h->gpre);
        post.swap(h->gpost);
        const size_t temp = h->gtemp;
        h->gtemp = 0;
        h->gentries = 0;
        qce_status gs = run_group_gemms(h, items, pre, post, temp);
        if (gs != QCE_SUCCESS) {
            h->pending.clear();
            return gs;
        }
    }
    const int count = (int)h->pending.size();
    if (count == 0) return QCE_SUCCESS;
    std::vector<int64_t> starts(count + 1, 0);
    for (int i = 0; i < count; ++i) starts[i + 1] = starts[i] + (h->pending[i].n_out + 255) / 256;
    const size_t bi = align256(sizeof(SmallItem) * (size_t)count);
    const size_t need = bi + align256(sizeof(int64_t) * (size_t)(count + 1));
    char *hp = nullptr, *dp = nullptr;
    qce_status rs = grp_reserve(h, need, hp, dp);
    if (rs != QCE_SUCCESS) {
        h->pending.clear();
        return rs;
    }
    memcpy(hp, h->pending.data(), sizeof(SmallItem) * (size_t)count);
    memcpy(hp + bi, starts.data(), sizeof(int64_t) * (size_t)(count + 1));
    h->pending.clear();
    hipEvent_t e0 = span_begin(h);
    QCE_HIP(h, hipMemcpyAsync(dp, hp, need, hipMemcpyHostToDevice, h->stream));
    QCE_HIP(h, launch_group(reinterpret_cast<const SmallItem *>(dp), reinterpret_cast<const int64_t *>(dp + bi),
                            count, starts[count], h->stream));
    span_end(h, e0, QCE_PHASE_GEMM_IRREGULAR);
    return QCE_SUCCESS;
}

qce_status qce_group_reset(qce_handle *h, size_t reserve_bytes) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    if (h->grouping) return fail(h, QCE_ERR_INVALID_VALUE, "a group is open");
    DeviceGuard g(h->device);
    QCE_HIP(h, hipStreamSynchronize(h->stream));
    if (reserve_bytes > h->grp_cap) {
        if (h->grp_dev) h->grp_old.push_back({h->grp_dev, h->grp_host});
        h->grp_dev = nullptr;
        h->grp_host = nullptr;
        h->grp_cap = 0;
        if (hipMalloc(&h->grp_dev, reserve_bytes) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&h->grp_host), reserve_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            if (h->grp_dev) (void)hipFree(h->grp_dev);
            h->grp_dev = nullptr;
            h->grp_host = nullptr;
            return fail(h, QCE_ERR_ALLOC, "group descriptor space of %zu bytes", reserve_bytes);
        }
        h->grp_cap = reserve_bytes;
    }
    h->grp_used = 0;
    return QCE_SUCCESS;
}

qce_status qce_set_timing(qce_handle *h, int enable) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    h->timing = enable != 0;
    return QCE_SUCCESS;
}

qce_status qce_set_timing_tag(qce_handle *h, int32_t tag) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    h->tag = tag;
    return QCE_SUCCESS;
}

qce_status qce_reset_timing(qce_handle *h) {
    if (!h) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    QCE_HIP(h, resolve_timing(h));
    h->recs.clear();
    return QCE_SUCCESS;
}

qce_status qce_get_timing(qce_handle *h, int32_t tag, qce_timing *out) {
    if (!h || !out) return QCE_ERR_INVALID_VALUE;
    DeviceGuard g(h->device);
    QCE_HIP(h, resolve_timing(h));
    *out = qce_timing{};
    for (const auto &r : h->recs) {
        if (tag >= 0 && r.tag != tag) continue;
        if (r.kind == -2) {
            const int mode = -1 - r.phase;
            if (mode >= 0 && mode < 4) out->gemms_by_mode[mode]++;
            continue;
        }
        if (r.phase < 0 || r.phase >= QCE_NUM_PHASES) continue;
        out->ms[r.phase] += r.ms;
        out->count[r.phase]++;
    }
    return QCE_SUCCESS;
}

}  // extern "C"
