// Host runtime and C ABI of the GPU library (see include/bemc.h).
#include "bemc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bemc_internal.h"
#include "server.h"

using namespace bemc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return BEMC_OK;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(BEMC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t dev_alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

template <typename T>
void dev_free(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace


// Device buffers of one evaluation: point ordering, near-pair list and its regrouping,
// element-chunk partial sums, counters.  The context owns one set that grows on demand;
// the allocation-free entry point uses a fixed set carved from a static device array.
struct EvalWork {
    OrderWork ow{};
    int64_t ow_cap = 0;              // points
    NearPair* near = nullptr;
    unsigned long long near_cap = 0;  // pairs
    NearWork nw{};
    int64_t nw_pts = 0;
    unsigned long long nw_pairs = 0;
    int nw_rows = 0;
    double* partial = nullptr;
    size_t partial_cap = 0;  // doubles
    DevCounters* ctr = nullptr;
};

namespace {
// Buffers of the allocation-free entry point, one set per device, carved from that device's
// static scratch array (noalloc.hip) when the first context on the device is created.
// Nothing is allocated: the set only holds addresses inside the array.
struct NoAllocSet {
    bool tried = false;
    int status = BEMC_OK;
    std::string msg;
    EvalWork w{};
};
std::mutex g_noalloc_mu;
NoAllocSet g_noalloc[kNoAllocMaxDevices];

// `device` must be current.  Returns BEMC_OK and the device's set, or the set-up error.
int noalloc_set(int device, NoAllocSet** out)
{
    *out = nullptr;
    if (device < 0 || device >= kNoAllocMaxDevices) return BEMC_E_LIMIT;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocSet& S = g_noalloc[device];
    *out = &S;
    if (S.tried) return S.status;
    S.tried = true;
    void* base = nullptr;
    const hipError_t e = noalloc_scratch(device, &base);
    if (e != hipSuccess) {
        S.status = BEMC_E_DEVICE;
        S.msg = std::string("address of the allocation-free workspace: ") + hipGetErrorString(e);
        return S.status;
    }
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + 255) & ~size_t(255);
        void* q = p + off;
        off += bytes;
        return q;
    };
    const size_t P = (size_t)kNoAllocMaxPoints, C = (size_t)kNoAllocMaxNearPairs;
    EvalWork& W = S.w;
    W.ctr = static_cast<DevCounters*>(take(sizeof(DevCounters)));
    W.ow.keys_in = static_cast<uint32_t*>(take(P * 4));
    W.ow.keys_out = static_cast<uint32_t*>(take(P * 4));
    W.ow.idx_in = static_cast<uint32_t*>(take(P * 4));
    W.ow.perm = static_cast<uint32_t*>(take(P * 4));
    W.ow.temp = take(kNoAllocTempBytes);
    W.ow.temp_bytes = kNoAllocTempBytes;
    W.ow.bbox = static_cast<double*>(take(6 * 1024 * 8));
    W.ow.pts = static_cast<double*>(take(3 * P * 8));
    W.ow.res = static_cast<double*>(take(4 * P * 8));  // phi and the three field rows
    W.ow_cap = (int64_t)P;
    W.near = static_cast<NearPair*>(take(C * sizeof(NearPair)));
    W.near_cap = C;
    W.nw.count = static_cast<uint32_t*>(take(P * 4));
    W.nw.start = static_cast<uint32_t*>(take(P * 4));
    W.nw.cursor = static_cast<uint32_t*>(take(P * 4));
    W.nw.grouped = static_cast<NearPair*>(take(C * sizeof(NearPair)));
    W.nw.origin = static_cast<uint32_t*>(take(C * 4));
    W.nw.sorted = static_cast<NearPair*>(take(C * sizeof(NearPair)));
    W.nw.slot = static_cast<uint32_t*>(take(C * 4));
    W.nw.res = static_cast<double*>(take(C * 4 * 8));
    W.nw.cost = static_cast<uint8_t*>(take(C));
    W.nw.order = static_cast<uint32_t*>(take(C * 4));
    W.nw.opair = static_cast<NearPair*>(take(C * sizeof(NearPair)));
    W.nw.buckets = static_cast<uint32_t*>(take(3 * kCostClasses * 4));
    W.nw.temp = take(kNoAllocTempBytes);
    W.nw.temp_bytes = kNoAllocTempBytes;
    W.nw_pts = (int64_t)P;
    W.nw_pairs = C;
    W.nw_rows = 4;
    W.partial = static_cast<double*>(take(kNoAllocPartialDoubles * 8));
    W.partial_cap = kNoAllocPartialDoubles;
    if (off > kNoAllocScratchBytes || order_temp_bytes((int64_t)P) > kNoAllocTempBytes ||
        near_scan_temp_bytes((int64_t)P) > kNoAllocTempBytes) {
        S.status = BEMC_E_LIMIT;
        S.msg = "the allocation-free workspace layout does not fit its array";
        W = EvalWork{};
        return S.status;
    }
    return BEMC_OK;
}
}  // namespace

// Record of one enqueued evaluation: pinned copies of its counters and its events.  A
// small ring of them lets evaluations be in flight while the host goes on.
struct CallRec {
    DevCounters* h_ctr = nullptr;   // counters at the end of the call (pinned)
    DevCounters* d_ctr = nullptr;   // h_ctr's device address: the call's last kernel writes it
    DevCounters* h_list = nullptr;  // counters after the near-pair list pass (pinned)
    hipEvent_t ev_list = nullptr, ev_far0 = nullptr, ev_far1 = nullptr, ev_near1 = nullptr, ev_done = nullptr;
    bool pending = false;
    int mode = 0;
    int64_t pairs = 0, node_ints = 0;  // node_ints < 0: counted on the device
    unsigned long long cap = 0;
};

struct bemc_context {
    int device = 0;
    int tri_rule = 33, rect_gl_n = 7, max_depth = 24;  // rect_gl_n < 0: Table B with -rect_gl_n points
    double near_dr = 3.0;

    // rule tables (device)
    double *d_tri = nullptr, *d_rect = nullptr;
    int nt = 0, nr = 0;
    // rule choice by distance ratio: level tables and limits
    bool dr_rules = false;
    double tri_dr[3] = { 100.0, 25.0, 10.0 }, rect_dr[3] = { 150.0, 40.0, 15.0 };
    double *d_lv_tri = nullptr, *d_lv_rect = nullptr;
    int lv_tri_off[5] = { 0, 0, 0, 0, 0 }, lv_rect_off[5] = { 0, 0, 0, 0, 0 };
    LevelRules levels() const;

    // elements (device)
    int64_t n_tri = 0, n_rect = 0, ne = 0;
    std::vector<double> h_area, h_L;  // host copies
    double* d_nrec = nullptr;  // near-walk records, packed on the device from the arrays below
    double *d_geom = nullptr, *d_cen = nullptr, *d_thr2 = nullptr, *d_frame = nullptr, *d_loc = nullptr,
           *d_L = nullptr, *d_area = nullptr, *d_nrm = nullptr, *d_q = nullptr, *d_qc = nullptr;
    int n_rhs = 0;
    bool have_geometry = false;

    // evaluation buffers and the near-pair list policy
    EvalWork w{};
    bool near_grow = true;  // the list grows to each evaluation's near-pair count
    // The collocation product's near stage depends on the geometry and the rules only (its
    // records are unit-density potentials; the densities are applied when the sums are
    // formed): after one product, the near-pair list, its order and those records stay in the
    // work buffers, and the next product with the same geometry and rules reuses them.  Any
    // change of geometry or rules, any reallocation of those buffers and any other evaluation
    // on them ends this.
    bool colloc_cached = false;
    int ensure_order(int64_t n);
    int ensure_near_capacity(unsigned long long need);
    int ensure_near_work(int64_t n, int rows);
    int ensure_partial(size_t need);
    void free_work();

    // evaluations in flight
    static constexpr int kCallRing = 4;
    CallRec rec[kCallRing];
    int rec_next = 0, rec_last = -1;
    hipStream_t last_stream = nullptr;
    int sticky = BEMC_OK;  // an error found in an earlier call, reported once
    std::string sticky_msg;
    int last_status = BEMC_OK;  // of the last finished call (OK or BEMC_W_ON_SURFACE)
    bemc_stats last{};
    int finish(int i);          // wait for record i and fold it into last / sticky
    void poll_finished();       // fold every finished record (no waiting)
    int drain();                // wait for every pending record

    bemc::Server* server = nullptr;

    int set_rules_tables();
    Elements elements() const;
    RuleTables rules() const;
    // mode kNearEval: phi, E at points; kNearColloc: out (= phi) [n_rhs][ne] at centroids;
    // kNearGrad: G (= phi) [6][n] at points.  noalloc: use the fixed buffers in W.
    int run(int mode, const double* pts, int64_t n, int precision, int rhs, int n_rhs_colloc, double* phi,
            double* E, hipStream_t s, EvalWork& W, bool noalloc);
};

Elements bemc_context::elements() const
{
    Elements e{};
    e.geom = d_geom; e.cen = d_cen; e.thr2 = d_thr2; e.frame = d_frame; e.loc = d_loc; e.nrec = d_nrec; e.L = d_L;
    e.area = d_area; e.nrm = d_nrm; e.q = d_q; e.ne = ne; e.n_tri = (int)n_tri; e.n_rhs = n_rhs;
    return e;
}

RuleTables bemc_context::rules() const
{
    RuleTables r{};
    r.tri = d_tri; r.rect = d_rect; r.nt = nt; r.nr = nr;
    return r;
}

namespace {
void pack_tri(const std::vector<TriNode>& tn, std::vector<double>& t64)
{
    for (const auto& n : tn) {
        t64.push_back(n.la); t64.push_back(n.lb); t64.push_back(n.lc); t64.push_back(n.w);
    }
}
void pack_rect(const std::vector<RectNode>& rn, std::vector<double>& r64)
{
    for (const auto& n : rn) {
        r64.push_back(n.x); r64.push_back(n.y); r64.push_back(n.w); r64.push_back(0.0);
    }
}
bool rect_rule_nodes(int spec, std::vector<RectNode>& rn)
{
    return spec > 0 ? rectangle_gauss_rule(spec, rn) : rectangle_table_rule(-spec, rn);
}
// a node table on the device
int upload_table(const std::vector<double>& t64, double** d64)
{
    dev_free(*d64);
    HIP_TRY(dev_alloc(d64, t64.size()));
    HIP_TRY(hipMemcpy(*d64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice));
    return BEMC_OK;
}
}  // namespace

int bemc_context::set_rules_tables()
{
    std::vector<TriNode> tn;
    std::vector<RectNode> rn;
    if (!triangle_rule(tri_rule, tn)) return fail(BEMC_E_INVALID_ARG, "unknown triangle rule %d", tri_rule);
    if (!rect_rule_nodes(rect_gl_n, rn)) return fail(BEMC_E_INVALID_ARG, "invalid rectangle rule %d", rect_gl_n);
    HIP_TRY(hipSetDevice(device));
    if (drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    std::vector<double> t64, r64;
    pack_tri(tn, t64);
    pack_rect(rn, r64);
    int rc = upload_table(t64, &d_tri);
    if (rc) return rc;
    if ((rc = upload_table(r64, &d_rect))) return rc;
    nt = (int)tn.size();
    nr = (int)rn.size();
    // levels of the distance-ratio rule choice: 7 / 12 / 19 / tri_rule and B2 / B3 / B4 / rect rule
    std::vector<double> lt, lr;
    const int tl[3] = { 7, 12, 19 }, rl[3] = { 7, 12, 17 };
    lv_tri_off[0] = lv_rect_off[0] = 0;
    for (int l = 0; l < 4; ++l) {
        std::vector<TriNode> a;
        std::vector<RectNode> b;
        if (l < 3) {
            triangle_rule(tl[l], a);
            rectangle_table_rule(rl[l], b);
        } else {
            a = tn;
            b = rn;
        }
        pack_tri(a, lt);
        pack_rect(b, lr);
        lv_tri_off[l + 1] = lv_tri_off[l] + (int)a.size();
        lv_rect_off[l + 1] = lv_rect_off[l] + (int)b.size();
    }
    if ((rc = upload_table(lt, &d_lv_tri))) return rc;
    if ((rc = upload_table(lr, &d_lv_rect))) return rc;
    return ok();
}

LevelRules bemc_context::levels() const
{
    LevelRules L{};
    L.tab.tri = d_lv_tri; L.tab.rect = d_lv_rect;
    L.tab.nt = lv_tri_off[4]; L.tab.nr = lv_rect_off[4];
    for (int i = 0; i < 5; ++i) { L.tri_off[i] = lv_tri_off[i]; L.rect_off[i] = lv_rect_off[i]; }
    for (int i = 0; i < 3; ++i) {
        L.tri_c[i] = (tri_dr[i] / near_dr) * (tri_dr[i] / near_dr);
        L.rect_c[i] = (rect_dr[i] / near_dr) * (rect_dr[i] / near_dr);
    }
    return L;
}

// ------------------------------------------------------------ evaluation buffers ---
namespace {
void free_order(OrderWork& ow)
{
    dev_free(ow.keys_in); dev_free(ow.keys_out); dev_free(ow.idx_in); dev_free(ow.perm);
    if (ow.temp) (void)hipFree(ow.temp);
    ow.temp = nullptr;
    dev_free(ow.bbox); dev_free(ow.pts); dev_free(ow.res);
}
}  // namespace

void bemc_context::free_work()
{
    colloc_cached = false;
    free_order(w.ow);
    w.ow_cap = 0;
    dev_free(w.near);
    w.near_cap = 0;
    near_work_free(w.nw);
    w.nw_pts = 0;
    w.nw_pairs = 0;
    w.nw_rows = 0;
    dev_free(w.partial);
    w.partial_cap = 0;
}

// Buffers are only replaced once every evaluation in flight has finished (drain first).
int bemc_context::ensure_order(int64_t n)
{
    if (n <= w.ow_cap && order_temp_bytes(n) <= w.ow.temp_bytes) return ok();
    n = std::max(n, w.ow_cap);
    if (drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    free_order(w.ow);
    w.ow_cap = 0;
    const size_t m = (size_t)n;
    w.ow.temp_bytes = order_temp_bytes(n);
    if (dev_alloc(&w.ow.keys_in, m) || dev_alloc(&w.ow.keys_out, m) || dev_alloc(&w.ow.idx_in, m) ||
        dev_alloc(&w.ow.perm, m) || hipMalloc(&w.ow.temp, std::max<size_t>(w.ow.temp_bytes, 1)) ||
        dev_alloc(&w.ow.bbox, 6 * 1024) || dev_alloc(&w.ow.pts, 3 * m) || dev_alloc(&w.ow.res, 6 * m)) {
        (void)hipGetLastError();
        free_order(w.ow);
        return fail(BEMC_E_OUT_OF_MEMORY, "point-ordering workspace for %lld points", (long long)n);
    }
    w.ow_cap = n;
    return ok();
}

int bemc_context::ensure_near_work(int64_t n, int rows)
{
    if (n <= w.nw_pts && w.near_cap <= w.nw_pairs && rows <= w.nw_rows && near_scan_temp_bytes(n) <= w.nw.temp_bytes)
        return ok();
    const int64_t np = std::max(n, w.nw_pts);
    const unsigned long long pairs = std::max(w.near_cap, w.nw_pairs);
    const int nrw = std::max(rows, w.nw_rows);
    if (drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    colloc_cached = false;
    near_work_free(w.nw);
    w.nw_pts = 0;
    w.nw_pairs = 0;
    w.nw_rows = 0;
    if (near_work_alloc(w.nw, np, pairs, nrw) != hipSuccess)
        return fail(BEMC_E_OUT_OF_MEMORY, "near-field work buffers for %llu pairs", pairs);
    w.nw_pts = np;
    w.nw_pairs = pairs;
    w.nw_rows = nrw;
    return ok();
}

int bemc_context::ensure_near_capacity(unsigned long long need)
{
    if (need <= w.near_cap) return ok();
    if (need > kMaxNearPairs) return fail(BEMC_E_LIMIT, "%llu near pairs exceed the 2^32 - 1 limit", need);
    unsigned long long cap = std::max<unsigned long long>(need, 1ull << 20);
    cap = std::min(cap + cap / 4, kMaxNearPairs);
    if (drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    colloc_cached = false;
    dev_free(w.near);
    w.near_cap = 0;
    if (dev_alloc(&w.near, (size_t)cap) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BEMC_E_OUT_OF_MEMORY, "near-pair list of %llu entries", cap);
    }
    w.near_cap = cap;
    return ok();
}

int bemc_context::ensure_partial(size_t need)
{
    if (need <= w.partial_cap) return ok();
    if (drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    dev_free(w.partial);
    w.partial_cap = 0;
    if (dev_alloc(&w.partial, need) != hipSuccess) {
        (void)hipGetLastError();
        return BEMC_E_OUT_OF_MEMORY;  // the caller falls back to one chunk
    }
    w.partial_cap = need;
    return ok();
}

// -------------------------------------------------------- evaluations in flight ---
int bemc_context::finish(int i)
{
    CallRec& r = rec[i];
    if (!r.pending) return BEMC_OK;
    r.pending = false;
    const hipError_t e = hipEventSynchronize(r.ev_done);
    if (e != hipSuccess) {
        sticky = BEMC_E_DEVICE;
        sticky_msg = std::string("an evaluation failed on the device: ") + hipGetErrorString(e);
        return BEMC_E_DEVICE;
    }
    const DevCounters& c = *r.h_ctr;
    float far_ms = 0.f, near_ms = 0.f;
    (void)hipEventElapsedTime(&far_ms, r.ev_far0, r.ev_far1);
    (void)hipEventElapsedTime(&near_ms, r.ev_far1, r.ev_near1);
    last = bemc_stats{};
    last.pairs = r.pairs;
    last.node_interactions = r.node_ints >= 0 ? r.node_ints : (int64_t)c.node_ints;
    last.near_pairs = (int64_t)c.near_count;
    last.leaves = (int64_t)c.leaves;
    last.cap_hits = (int64_t)c.cap_hits;
    last.on_surface = (int64_t)c.on_surface;
    last.max_depth = (int64_t)c.max_depth;
    last.near_capacity = (int64_t)r.cap;
    last.far_ms = far_ms;
    last.near_ms = near_ms;
    last.node_interactions_pair_rule = r.node_ints >= 0 ? r.node_ints : (int64_t)c.node_ints_pair;
    last_status = (r.mode != kNearColloc && c.on_surface) ? BEMC_W_ON_SURFACE : BEMC_OK;
    char buf[256];
    if (c.near_count > r.cap) {
        snprintf(buf, sizeof buf,
                 "an evaluation found %llu near pairs but the near-pair list holds %llu: its near field is "
                 "incomplete (raise bemc_set_near_capacity or let the list grow)",
                 c.near_count, r.cap);
        sticky = BEMC_E_LIMIT;
        sticky_msg = buf;
    } else if (c.visit_limit_hits) {
        snprintf(buf, sizeof buf, "%llu near pairs hit the subdivision visit limit", c.visit_limit_hits);
        sticky = BEMC_E_LIMIT;
        sticky_msg = buf;
    }
    return BEMC_OK;
}

void bemc_context::poll_finished()
{
    for (int i = 0; i < kCallRing; ++i)
        if (rec[i].pending && hipEventQuery(rec[i].ev_done) == hipSuccess) (void)finish(i);
}

int bemc_context::drain()
{
    int rc = BEMC_OK;
    // oldest first, so that `last` ends with the latest call
    for (int k = 1; k <= kCallRing; ++k) {
        const int i = (rec_next + k - 1) % kCallRing;
        if (rec[i].pending && finish(i)) rc = BEMC_E_DEVICE;
    }
    return rc;
}

// The pipeline of one evaluation, enqueued on `s`:
//   Morton ordering of the points (field and gradient);
//   near-pair list (near_list_kernel: classification with box culling, compaction);
//   far field (near pairs excluded by the same test), element-chunk reduction;
//   near-list regrouping, FP64 near field, ordered per-point sums, unordering;
//   counters to pinned host memory (written by the last kernel).
// Growing list (default): the host reads the list pass's pair count after the far field is
// enqueued and, if the list was too short, grows it and repeats the list pass (never the
// far field), then enqueues the near field and returns.  Fixed list, and the buffers of the
// allocation-free entry point: no host wait at all; an overflow is reported by
// bemc_query_stats and the next call.
int bemc_context::run(int mode, const double* pts, int64_t n, int precision, int rhs, int n_rhs_colloc, double* phi,
                      double* E, hipStream_t s, EvalWork& W, bool noalloc)
{
    HIP_TRY(hipSetDevice(device));
    const bool colloc = mode == kNearColloc;
    const bool grad = mode == kNearGrad;
    const int64_t npts = colloc ? ne : n;
    const int near_rows = colloc ? 1 : (grad ? 6 : 4);
    // errors found in finished earlier calls are reported first, once
    poll_finished();
    if (sticky) {
        const int rc = sticky;
        sticky = BEMC_OK;
        return fail(rc, "%s", sticky_msg.c_str());
    }
    // buffers (the growing ones only change once nothing is in flight)
    if (!noalloc) {
        if (!colloc) {
            int rc = ensure_order(n);
            if (rc) return rc;
        }
        if (W.near_cap == 0) {
            int rc = ensure_near_capacity(std::max<unsigned long long>(1ull << 20, (unsigned long long)npts * 8));
            if (rc) return rc;
        }
        int rc = ensure_near_work(npts, near_rows);
        if (rc) return rc;
    }
    // a field or gradient evaluation in these buffers overwrites the collocation near stage
    const bool own_work = &W == &w;
    if (!colloc && own_work) colloc_cached = false;
    const bool reuse_near = colloc && own_work && colloc_cached;
    // element split: many more workgroups than resident slots, so that the dispatcher
    // balances the tail; the chunk partial sums are reduced in fixed order
    const int64_t blocks = (npts + 511) / 512;  // nominal 512 points per workgroup (256-768 in fact)
    int n_split = (int)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, (kSplitTargetBlocks + blocks - 1) / blocks));
    n_split = (int)std::min<int64_t>(n_split, std::max<int64_t>(1, ne / 16));  // chunks of >= 16 elements
    const int64_t rows = colloc ? n_rhs_colloc : (grad ? 6 : 4);
    if (n_split > 1) {
        const size_t need = (size_t)n_split * (size_t)rows * (size_t)npts;
        if (noalloc) {
            while (n_split > 1 && (size_t)n_split * (size_t)rows * (size_t)npts > W.partial_cap) --n_split;
        } else if (ensure_partial(need)) {
            n_split = 1;  // not enough memory for the chunks: one chunk
        }
    }
    // the call record (waits only if the ring is full of calls in flight)
    const int ri = rec_next;
    if (rec[ri].pending && finish(ri)) return fail(BEMC_E_DEVICE, "%s", sticky_msg.c_str());
    rec_next = (rec_next + 1) % kCallRing;
    CallRec& R = rec[ri];
    if (rec_last >= 0 && last_stream != s) HIP_TRY(hipStreamWaitEvent(s, rec[rec_last].ev_done, 0));

    double* user_phi = phi;
    double* user_E = E;
    const bool ordered = !colloc && n > kOrderMinPoints;  // Morton order of the points
    if (!colloc) {
        if (ordered) {
            HIP_TRY(order_points(pts, n, W.ow, s));
            pts = W.ow.pts;
        }
        phi = W.ow.res;
        E = E ? W.ow.res + n : nullptr;
    }
    double* G = grad ? phi : nullptr;
    if (grad) phi = E = nullptr;

    Elements el = elements();
    if (colloc) { el.q = d_qc; el.n_rhs = n_rhs_colloc; }
    const double* lpts = colloc ? d_cen : pts;
    // the counters and the near stage's order clears in one launch (a list regrowth below
    // reallocates the latter, and the near stage then clears them itself); a collocation
    // product that reuses the near stage keeps the counters of the product that formed it
    bool order_cleared = true;
    if (!reuse_near) {
        HIP_TRY(clear_call(W.ctr, W.nw, npts, s));
        HIP_TRY(launch_near_list(lpts, npts, el, W.near, W.near_cap, W.ctr, s));
    }
    const bool read_count = near_grow && !noalloc && !reuse_near;
    if (read_count) {
        HIP_TRY(hipMemcpyAsync(R.h_list, W.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(R.ev_list, s));
    }

    FarArgs fa{};
    fa.el = el; fa.rules = rules();
    fa.pts = pts; fa.n = npts; fa.rhs = rhs; fa.n_rhs = n_rhs_colloc; fa.K = coulomb_constant();
    fa.phi = phi; fa.E = E; fa.G = G;
    fa.elem_begin = 0; fa.elem_end = ne; fa.n_split = n_split; fa.chunk = (ne + n_split - 1) / n_split;
    fa.partial = n_split > 1 ? W.partial : nullptr;
    fa.near_list = W.near; fa.near_cap = W.near_cap; fa.ctr = W.ctr;
    fa.dr_rules = (dr_rules && !colloc) ? 1 : 0;
    fa.lv = levels();
    HIP_TRY(hipEventRecord(R.ev_far0, s));
    HIP_TRY(colloc ? launch_far_colloc(fa, precision, s)
                   : (grad ? launch_far_grad(fa, precision, s) : launch_far_eval(fa, precision, s)));
    HIP_TRY(hipEventRecord(R.ev_far1, s));  // far_ms: the far-field kernel alone
    // (field and gradient: the chunks are added with the near sums at the end)
    if (n_split > 1 && colloc) HIP_TRY(launch_reduce_chunks(W.partial, n_split, rows, npts, fa.K, phi, s));

    if (read_count) {
        // the far field runs meanwhile; the list pass finished long before it
        HIP_TRY(hipEventSynchronize(R.ev_list));
        const unsigned long long found = R.h_list->near_count;
        if (found > W.near_cap) {  // grow the list and list again
            int rc = ensure_near_capacity(found);
            if (rc) return rc;
            if ((rc = ensure_near_work(npts, near_rows))) return rc;
            order_cleared = false;
            HIP_TRY(launch_reset_near_count(W.ctr, s));
            HIP_TRY(launch_near_list(lpts, npts, el, W.near, W.near_cap, W.ctr, s));
        }
    }

    NearArgs na{};
    na.el = el; na.rules = fa.rules; na.pts = colloc ? nullptr : pts; na.n = npts; na.rhs = rhs;
    na.n_rhs = n_rhs_colloc; na.K = fa.K; na.phi = phi; na.E = E; na.G = G; na.near_cap = W.near_cap;
    na.ctr = W.ctr; na.near_dr2 = near_dr * near_dr; na.max_depth = max_depth; na.visit_limit = 1ll << 22;
    na.near_list = W.near; na.slot = W.nw.slot; na.order = W.nw.order; na.opair = W.nw.opair;
    na.walk_end = near_walk_end(W.nw); na.heavy_end = near_heavy_end(W.nw); na.deep = 1;
    na.res = W.nw.res;
    if (!reuse_near) {
        HIP_TRY(near_order(W.near, W.ctr, W.near_cap, npts, lpts, el, W.nw, order_cleared, s));
        HIP_TRY(launch_near(na, mode, s));
    }
    if (colloc) {
        HIP_TRY(near_reduce(W.nw, npts, mode, phi, E, G, el.q, ne, n_rhs_colloc, fa.K, W.ctr, R.d_ctr, s));
    } else {
        // far field (chunk sums) + near sums, back to the caller's order, in one pass
        const int orows = grad ? 6 : (user_E ? 4 : 1);
        HIP_TRY(near_finish(W.nw, npts, mode, orows, n_split > 1 ? W.partial : nullptr, n_split, (int)rows,
                            W.ow.res, fa.K, ordered ? W.ow.perm : nullptr, user_phi, grad ? user_phi + n : user_E,
                            W.ctr, R.d_ctr, s));
    }
    HIP_TRY(hipEventRecord(R.ev_near1, s));
    // the counters: written by that last kernel into the pinned record (one launch fewer per
    // call), else copied here
    if (!R.d_ctr) HIP_TRY(hipMemcpyAsync(R.h_ctr, W.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(R.ev_done, s));
    if (colloc && own_work) colloc_cached = true;  // later products are ordered after this one
    R.pending = true;
    R.mode = mode;
    R.pairs = npts * ne;
    R.node_ints = fa.dr_rules ? -1 : npts * (n_tri * (int64_t)nt + n_rect * (int64_t)nr);
    R.cap = W.near_cap;
    rec_last = ri;
    last_stream = s;
    return ok();
}

// ======================================================================= C ABI ====
extern "C" {

const char* bemc_last_error(void) { return g_last_error.c_str(); }

double bemc_coulomb_constant(void) { return coulomb_constant(); }

int bemc_rule_size(int tri_rule)
{
    std::vector<TriNode> t;
    return triangle_rule(tri_rule, t) ? (int)t.size() : -1;
}

int bemc_create(int device, bemc_handle* out)
{
    if (!out) return fail(BEMC_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(BEMC_E_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(BEMC_E_INVALID_ARG, "device %d of %d", device, ndev);
    bemc_context* h = new bemc_context();
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete h; return fail(BEMC_E_DEVICE, "hipSetDevice(%d)", device); }
    int rc = h->set_rules_tables();
    if (rc) { bemc_destroy(h); return rc; }
    NoAllocSet* na = nullptr;
    (void)noalloc_set(device, &na);  // once per device; a failure is reported by bemc_eval_noalloc
    if (dev_alloc(&h->w.ctr, 1) != hipSuccess) {
        bemc_destroy(h);
        return fail(BEMC_E_OUT_OF_MEMORY, "counter buffers");
    }
    for (auto& r : h->rec) {
        if (hipHostMalloc(reinterpret_cast<void**>(&r.h_ctr), sizeof(DevCounters), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&r.h_list), sizeof(DevCounters), hipHostMallocDefault) != hipSuccess) {
            bemc_destroy(h);
            return fail(BEMC_E_OUT_OF_MEMORY, "pinned counter buffers");
        }
        // without a device address the host copies the counters itself (and the failed call's
        // error must not be reported by the next launch's hipGetLastError)
        if (hipHostGetDevicePointer(reinterpret_cast<void**>(&r.d_ctr), r.h_ctr, 0) != hipSuccess) {
            r.d_ctr = nullptr;
            (void)hipGetLastError();
        }
        for (hipEvent_t* e : { &r.ev_list, &r.ev_far0, &r.ev_far1, &r.ev_near1, &r.ev_done })
            if (hipEventCreate(e) != hipSuccess) { bemc_destroy(h); return fail(BEMC_E_DEVICE, "hipEventCreate"); }
    }
    *out = h;
    return ok();
}

static void free_elements(bemc_context* h)
{
    dev_free(h->d_geom); dev_free(h->d_cen); dev_free(h->d_thr2); dev_free(h->d_frame); dev_free(h->d_loc);
    dev_free(h->d_nrec);
    dev_free(h->d_L); dev_free(h->d_area); dev_free(h->d_nrm); dev_free(h->d_q); dev_free(h->d_qc);
    h->n_rhs = 0;
    h->have_geometry = false;
}

int bemc_destroy(bemc_handle h)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (h->server) bemc_server_stop(h);
    (void)hipSetDevice(h->device);
    (void)h->drain();
    (void)hipDeviceSynchronize();
    free_elements(h);
    dev_free(h->d_tri); dev_free(h->d_rect);
    dev_free(h->d_lv_tri); dev_free(h->d_lv_rect);
    h->free_work();
    dev_free(h->w.ctr);
    for (auto& r : h->rec) {
        if (r.h_ctr) (void)hipHostFree(r.h_ctr);
        if (r.h_list) (void)hipHostFree(r.h_list);
        for (hipEvent_t e : { r.ev_list, r.ev_far0, r.ev_far1, r.ev_near1, r.ev_done })
            if (e) (void)hipEventDestroy(e);
    }
    delete h;
    return ok();
}

int bemc_set_rules(bemc_handle h, int tri_rule, int rect_gl_n, double near_dr, int max_depth)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "rules cannot change while serving");
    h->colloc_cached = false;
    // the far-field sums expand r^2 about the element's centroid, whose rounding is bounded
    // for DR >= 2 (in FP32 by about 9 ulp of r^2)
    if (!(near_dr >= 2.0) || !std::isfinite(near_dr)) return fail(BEMC_E_INVALID_ARG, "near_dr must be >= 2");
    if (max_depth < 0 || max_depth > 30) return fail(BEMC_E_INVALID_ARG, "max_depth must be in 0..30");
    std::vector<TriNode> t;
    if (!triangle_rule(tri_rule, t)) return fail(BEMC_E_INVALID_ARG, "unknown triangle rule %d", tri_rule);
    {
        std::vector<RectNode> rn;
        if (rect_gl_n == 0 || rect_gl_n > 16 || (rect_gl_n < 0 && !rectangle_table_rule(-rect_gl_n, rn)))
            return fail(BEMC_E_INVALID_ARG, "rectangle rule must be 1..16 (Gauss n x n) or -4/-7/-12/-17/-33 (Table B)");
        const int nr = rect_gl_n > 0 ? rect_gl_n * rect_gl_n : (int)rn.size();
        if (h->dr_rules && ((int)t.size() < kMinDrTriNodes || nr < kMinDrRectNodes))
            return fail(BEMC_E_INVALID_ARG, "with the rule choice by distance ratio enabled, the rules must have at "
                        "least %d (triangle) and %d (rectangle) points", kMinDrTriNodes, kMinDrRectNodes);
    }
    const int old_t = h->tri_rule, old_r = h->rect_gl_n;
    h->tri_rule = tri_rule;
    h->rect_gl_n = rect_gl_n;
    int rc = h->set_rules_tables();
    if (rc) { h->tri_rule = old_t; h->rect_gl_n = old_r; return rc; }
    const double old_dr = h->near_dr;
    h->near_dr = near_dr;
    h->max_depth = max_depth;
    if (h->have_geometry && old_dr != near_dr) {  // thresholds (near_dr L)^2 depend on near_dr
        std::vector<double> thr(h->h_L.size());
        for (size_t i = 0; i < thr.size(); ++i) thr[i] = (near_dr * h->h_L[i]) * (near_dr * h->h_L[i]);
        HIP_TRY(hipSetDevice(h->device));
        if (h->drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
        HIP_TRY(hipMemcpy(h->d_thr2, thr.data(), thr.size() * 8, hipMemcpyHostToDevice));
        HIP_TRY(launch_pack_near_records(h->elements(), h->d_nrec, nullptr));
        HIP_TRY(hipDeviceSynchronize());
    }
    return ok();
}

int bemc_upload_geometry(bemc_handle h, const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
                         void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "geometry cannot change while serving");
    h->colloc_cached = false;
    if (n_tri < 0 || n_rect < 0) return fail(BEMC_E_INVALID_ARG, "negative element count");
    if ((n_tri > 0 && !tri) || (n_rect > 0 && !rect)) return fail(BEMC_E_INVALID_ARG, "null geometry pointer");
    const int64_t ne = n_tri + n_rect;
    if (ne >= (1ll << 31)) return fail(BEMC_E_LIMIT, "too many elements (%lld)", (long long)ne);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    std::vector<double> geom(9 * (size_t)ne), cen(3 * (size_t)ne), thr2((size_t)ne), frame(9 * (size_t)ne),
        loc(9 * (size_t)ne, 0.0), L((size_t)ne), area((size_t)ne), nrm(3 * (size_t)ne);
    auto at = [ne](std::vector<double>& v, int comp, int64_t e) -> double& { return v[(size_t)comp * ne + e]; };
    for (int64_t e = 0; e < ne; ++e) {
        const bool is_tri = e < n_tri;
        const double* g = is_tri ? tri + 9 * e : rect + 9 * (e - n_tri);
        for (int c = 0; c < 9; ++c) {
            if (!std::isfinite(g[c])) return fail(BEMC_E_NONFINITE, "element %lld has a non-finite coordinate", (long long)e);
            at(geom, c, e) = g[c];
        }
        double C[3], N[3], F1[3], a, Lh;  // F1: first in-plane axis of the element frame
        if (is_tri) {
            const double *A = g, *B = g + 3, *Cv = g + 6;
            const double u[3] = { B[0] - A[0], B[1] - A[1], B[2] - A[2] };
            const double v[3] = { Cv[0] - A[0], Cv[1] - A[1], Cv[2] - A[2] };
            const double w[3] = { Cv[0] - B[0], Cv[1] - B[1], Cv[2] - B[2] };
            N[0] = u[1] * v[2] - u[2] * v[1];
            N[1] = u[2] * v[0] - u[0] * v[2];
            N[2] = u[0] * v[1] - u[1] * v[0];
            const double n2 = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            a = 0.5 * n2;
            const double la = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            const double lb = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double lc = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            Lh = (la + lb + lc) / 3.0;  // Sec. 2: L = (a + b + c) / 3
            if (!(a > 0.0) || !(la > 0.0 && lb > 0.0 && lc > 0.0))
                return fail(BEMC_E_DEGENERATE_ELEMENT, "triangle %lld has zero area", (long long)e);
            for (int c = 0; c < 3; ++c) {
                C[c] = (A[c] + B[c] + Cv[c]) / 3.0;
                N[c] /= n2;
                F1[c] = u[c] / lc;  // along B - A
            }
        } else {
            const double *P0 = g, *e1 = g + 3, *e2 = g + 6;
            const double la = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            const double lb = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
            if (!(la > 0.0 && lb > 0.0)) return fail(BEMC_E_DEGENERATE_ELEMENT, "rectangle %lld has a zero side", (long long)e);
            const double dp = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
            if (std::fabs(dp) > 1e-10 * la * lb)
                return fail(BEMC_E_NOT_RECTANGLE, "rectangle %lld: sides not orthogonal", (long long)e);
            N[0] = e1[1] * e2[2] - e1[2] * e2[1];
            N[1] = e1[2] * e2[0] - e1[0] * e2[2];
            N[2] = e1[0] * e2[1] - e1[1] * e2[0];
            const double n2 = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            a = la * lb;
            if (!(a > 0.0) || !(n2 > 0.0))  // sides so short that the area or the normal underflows
                return fail(BEMC_E_DEGENERATE_ELEMENT, "rectangle %lld has zero area", (long long)e);
            Lh = 0.5 * (la + lb);  // mean of the four sides
            for (int c = 0; c < 3; ++c) {
                C[c] = P0[c] + 0.5 * e1[c] + 0.5 * e2[c];  // Eq. 3.2: Q_cen
                N[c] /= n2;
                F1[c] = e2[c] / lb;  // along the second side
            }
        }
        // element frame: F1, F2 = N x F1 in the plane, N the normal
        const double F2[3] = { N[1] * F1[2] - N[2] * F1[1], N[2] * F1[0] - N[0] * F1[2], N[0] * F1[1] - N[1] * F1[0] };
        for (int c = 0; c < 3; ++c) {
            at(cen, c, e) = C[c];
            at(nrm, c, e) = N[c];
            at(frame, c, e) = F1[c];
            at(frame, 3 + c, e) = F2[c];
            at(frame, 6 + c, e) = N[c];
        }
        auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
        if (is_tri) {  // in-plane coordinates of the vertices relative to the centroid
            for (int m = 0; m < 3; ++m) {
                const double d[3] = { g[3 * m] - C[0], g[3 * m + 1] - C[1], g[3 * m + 2] - C[2] };
                at(loc, 2 * m, e) = dot(d, F1);
                at(loc, 2 * m + 1, e) = dot(d, F2);
                at(loc, 6 + m, e) = dot(d, N);  // rounding-level height: the frame of a sliver
                                                 // is known only to eps x aspect ratio
            }
        } else {  // half sides: e1 / 2 = gamma F1 + beta F2, e2 / 2 = alpha F1
            const double h1[3] = { 0.5 * g[3], 0.5 * g[4], 0.5 * g[5] };
            at(loc, 0, e) = dot(h1, F1);
            at(loc, 1, e) = dot(h1, F2);
            at(loc, 2, e) = 0.5 * std::sqrt(dot(g + 6, g + 6));
            // the corner P0 - c in the frame (c is the rounded centroid, so this is not exactly
            // -e1/2 - e2/2, and the plane may pass beside c by a rounding of the coordinates),
            // and the sides' rounding-level heights
            const double d0[3] = { g[0] - C[0], g[1] - C[1], g[2] - C[2] };
            at(loc, 3, e) = dot(d0, F1);
            at(loc, 4, e) = dot(d0, F2);
            at(loc, 5, e) = dot(d0, N);
            at(loc, 6, e) = dot(g + 3, N);
            at(loc, 7, e) = dot(g + 6, N);
        }
        area[(size_t)e] = a;
        L[(size_t)e] = Lh;
        thr2[(size_t)e] = (h->near_dr * Lh) * (h->near_dr * Lh);
    }

    HIP_TRY(hipSetDevice(h->device));
    if (h->drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    HIP_TRY(hipStreamSynchronize(s));
    free_elements(h);
    h->n_tri = n_tri;
    h->n_rect = n_rect;
    h->ne = ne;
    if (dev_alloc(&h->d_geom, geom.size()) || dev_alloc(&h->d_cen, cen.size()) || dev_alloc(&h->d_thr2, thr2.size()) ||
        dev_alloc(&h->d_frame, frame.size()) || dev_alloc(&h->d_loc, loc.size()) || dev_alloc(&h->d_L, L.size()) ||
        dev_alloc(&h->d_area, area.size()) || dev_alloc(&h->d_nrm, nrm.size()) ||
        dev_alloc(&h->d_nrec, (size_t)std::max<int64_t>(ne, 1) * kNearRec)) {
        (void)hipGetLastError();
        free_elements(h);
        return fail(BEMC_E_OUT_OF_MEMORY, "element arrays for %lld elements", (long long)ne);
    }
    HIP_TRY(hipMemcpyAsync(h->d_geom, geom.data(), geom.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_cen, cen.data(), cen.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_thr2, thr2.data(), thr2.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_frame, frame.data(), frame.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_loc, loc.data(), loc.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_L, L.data(), L.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_area, area.data(), area.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->d_nrm, nrm.data(), nrm.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_pack_near_records(h->elements(), h->d_nrec, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->h_area = area;
    h->h_L = L;
    h->have_geometry = true;
    return ok();
}

int bemc_upload_densities(bemc_handle h, const double* sigma, int n_rhs, int sigma_on_device, void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry) return fail(BEMC_E_NO_GEOMETRY, "upload the geometry first");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "densities cannot change while serving");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(BEMC_E_INVALID_ARG, "n_rhs must be in 1..%d", kMaxRhs);
    if (!sigma && h->ne > 0) return fail(BEMC_E_INVALID_ARG, "sigma is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t cnt = (size_t)n_rhs * (size_t)h->ne;
    if (!sigma_on_device)
        for (size_t i = 0; i < cnt; ++i)
            if (!std::isfinite(sigma[i])) return fail(BEMC_E_NONFINITE, "sigma[%zu] is not finite", i);
    HIP_TRY(hipSetDevice(h->device));
    if (h->drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    HIP_TRY(hipStreamSynchronize(s));
    dev_free(h->d_q);
    h->n_rhs = 0;
    if (dev_alloc(&h->d_q, cnt) != hipSuccess) { (void)hipGetLastError(); return fail(BEMC_E_OUT_OF_MEMORY, "charges"); }
    double* d_sig = nullptr;
    if (sigma_on_device) {
        d_sig = const_cast<double*>(sigma);
    } else {
        if (dev_alloc(&d_sig, cnt) != hipSuccess) { (void)hipGetLastError(); return fail(BEMC_E_OUT_OF_MEMORY, "sigma staging"); }
        HIP_TRY(hipMemcpyAsync(d_sig, sigma, cnt * 8, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(launch_charges(d_sig, h->d_area, h->d_q, h->ne, n_rhs, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!sigma_on_device) dev_free(d_sig);
    h->n_rhs = n_rhs;
    return ok();
}

int bemc_eval(bemc_handle h, const double* pts, int64_t n, int precision, int rhs, double* phi, double* E,
              void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry || h->n_rhs == 0) return fail(BEMC_E_NO_GEOMETRY, "geometry and densities must be uploaded");
    if (n < 0) return fail(BEMC_E_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (n >= (1ll << 31)) return fail(BEMC_E_LIMIT, "n >= 2^31");
    if (!pts || !phi) return fail(BEMC_E_INVALID_ARG, "null point or output pointer");
    if (precision != BEMC_FP64 && precision != BEMC_MIXED) return fail(BEMC_E_INVALID_ARG, "precision %d", precision);
    if (rhs < 0 || rhs >= h->n_rhs) return fail(BEMC_E_INVALID_ARG, "rhs %d of %d", rhs, h->n_rhs);
    return h->run(kNearEval, pts, n, precision, rhs, 1, phi, E, reinterpret_cast<hipStream_t>(stream), h->w, false);
}

int bemc_eval_noalloc(bemc_handle h, const double* pts, int64_t n, int precision, int rhs, double* phi, double* E,
                      void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry || h->n_rhs == 0) return fail(BEMC_E_NO_GEOMETRY, "geometry and densities must be uploaded");
    if (n < 0) return fail(BEMC_E_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (n > kNoAllocMaxPoints)
        return fail(BEMC_E_LIMIT, "%lld points exceed the %lld of the allocation-free workspace", (long long)n,
                    (long long)kNoAllocMaxPoints);
    if (!pts || !phi) return fail(BEMC_E_INVALID_ARG, "null point or output pointer");
    if (precision != BEMC_FP64 && precision != BEMC_MIXED) return fail(BEMC_E_INVALID_ARG, "precision %d", precision);
    if (rhs < 0 || rhs >= h->n_rhs) return fail(BEMC_E_INVALID_ARG, "rhs %d of %d", rhs, h->n_rhs);
    HIP_TRY(hipSetDevice(h->device));
    NoAllocSet* S = nullptr;
    const int rc = noalloc_set(h->device, &S);
    if (rc) return fail(rc, "%s", S ? S->msg.c_str() : "device index out of range");
    if (order_temp_bytes(n) > S->w.ow.temp_bytes || near_scan_temp_bytes(n) > S->w.nw.temp_bytes)
        return fail(BEMC_E_LIMIT, "sort workspace for %lld points exceeds the allocation-free workspace", (long long)n);
    return h->run(kNearEval, pts, n, precision, rhs, 1, phi, E, reinterpret_cast<hipStream_t>(stream), S->w, true);
}

int bemc_eval_gradient(bemc_handle h, const double* pts, int64_t n, int precision, int rhs, double* G, void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry || h->n_rhs == 0) return fail(BEMC_E_NO_GEOMETRY, "geometry and densities must be uploaded");
    if (n < 0) return fail(BEMC_E_INVALID_ARG, "n < 0");
    if (n == 0) return ok();
    if (n >= (1ll << 31)) return fail(BEMC_E_LIMIT, "n >= 2^31");
    if (!pts || !G) return fail(BEMC_E_INVALID_ARG, "null point or output pointer");
    if (precision != BEMC_FP64 && precision != BEMC_MIXED) return fail(BEMC_E_INVALID_ARG, "precision %d", precision);
    if (rhs < 0 || rhs >= h->n_rhs) return fail(BEMC_E_INVALID_ARG, "rhs %d of %d", rhs, h->n_rhs);
    return h->run(kNearGrad, pts, n, precision, rhs, 1, G, nullptr, reinterpret_cast<hipStream_t>(stream), h->w,
                  false);
}

int bemc_collocation_matvec(bemc_handle h, const double* sigma, int n_rhs, int precision, double* out, void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry) return fail(BEMC_E_NO_GEOMETRY, "geometry must be uploaded");
    if (n_rhs < 1 || n_rhs > kMaxRhs) return fail(BEMC_E_INVALID_ARG, "n_rhs must be in 1..%d", kMaxRhs);
    if (!sigma || !out) return fail(BEMC_E_INVALID_ARG, "null pointer");
    if (precision != BEMC_FP64 && precision != BEMC_MIXED) return fail(BEMC_E_INVALID_ARG, "precision %d", precision);
    if (h->server) return fail(BEMC_E_INVALID_ARG, "collocation while serving is not supported");
    if (h->ne == 0) return ok();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(h->device));
    // charges q = sigma * area of these densities, kept apart from the evaluation densities;
    // the buffer is shared by the calls on the context, so this one waits for the last
    if (!h->d_qc && dev_alloc(&h->d_qc, (size_t)kMaxRhs * (size_t)h->ne) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BEMC_E_OUT_OF_MEMORY, "collocation charges");
    }
    if (h->rec_last >= 0 && h->last_stream != s) HIP_TRY(hipStreamWaitEvent(s, h->rec[h->rec_last].ev_done, 0));
    HIP_TRY(launch_charges(sigma, h->d_area, h->d_qc, h->ne, n_rhs, s));
    return h->run(kNearColloc, nullptr, h->ne, precision, 0, n_rhs, out, nullptr, s, h->w, false);
}

int bemc_solve_densities(bemc_handle h, const double* potential, double* sigma, double tol, int max_iter,
                         int restart, int precision, bemc_solve_info* info, void* stream)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (!h->have_geometry) return fail(BEMC_E_NO_GEOMETRY, "geometry must be uploaded");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "not while serving");
    if (!potential || !sigma) return fail(BEMC_E_INVALID_ARG, "null pointer");
    if (!(tol > 0.0) || max_iter < 1 || restart < 1 || restart > 200)
        return fail(BEMC_E_INVALID_ARG, "tol > 0, max_iter >= 1, restart in 1..200 required");
    if (precision != BEMC_FP64 && precision != BEMC_MIXED && precision != BEMC_MIXED_REFINE)
        return fail(BEMC_E_INVALID_ARG, "precision %d", precision);
    if (info) *info = bemc_solve_info{};
    if (h->ne == 0) return ok();
    HIP_TRY(hipSetDevice(h->device));
    std::string err;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int rc = precision == BEMC_MIXED_REFINE
                       ? bemc::solve_refined(h, h->elements(), potential, sigma, tol, max_iter, restart, info, s, err)
                       : bemc::solve_gmres(h, h->elements(), potential, sigma, tol, max_iter, restart, precision, info,
                                           s, err);
    if (rc) return fail(rc, "%s", err.c_str());
    return ok();
}

int bemc_set_dr_rules(bemc_handle h, int enable, const double* tri_dr, const double* rect_dr)
{
    if (!h) return fail(BEMC_E_INVALID_ARG, "null handle");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "rules cannot change while serving");
    h->colloc_cached = false;
    double t[3] = { 100.0, 25.0, 10.0 }, r[3] = { 150.0, 40.0, 15.0 };
    if (tri_dr) std::copy(tri_dr, tri_dr + 3, t);
    if (rect_dr) std::copy(rect_dr, rect_dr + 3, r);
    for (const double* v : { t, r })
        if (!(v[0] >= v[1] && v[1] >= v[2] && v[2] >= h->near_dr) || !std::isfinite(v[0]))
            return fail(BEMC_E_INVALID_ARG, "limits must be finite, decreasing and >= near_dr");
    // the levels must get finer in order: a wavefront runs the finest level one of its
    // pairs needs, which must then be at least as accurate as every lane's own choice
    if (enable && (h->nt < kMinDrTriNodes || h->nr < kMinDrRectNodes))
        return fail(BEMC_E_INVALID_ARG, "the rule choice by distance ratio needs rules of at least %d (triangle) "
                    "and %d (rectangle) points, finer than its 19-point and Table B4 levels", kMinDrTriNodes,
                    kMinDrRectNodes);
    h->dr_rules = enable != 0;
    std::copy(t, t + 3, h->tri_dr);
    std::copy(r, r + 3, h->rect_dr);
    return ok();
}

int bemc_set_near_capacity(bemc_handle h, int64_t pairs, int grow)
{
    if (!h || pairs < 1) return fail(BEMC_E_INVALID_ARG, "invalid capacity");
    if ((unsigned long long)pairs > kMaxNearPairs) return fail(BEMC_E_LIMIT, "capacity above 2^32 - 1 pairs");
    HIP_TRY(hipSetDevice(h->device));
    if (h->drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    h->colloc_cached = false;
    dev_free(h->w.near);
    h->w.near_cap = 0;
    if (dev_alloc(&h->w.near, (size_t)pairs) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BEMC_E_OUT_OF_MEMORY, "near-pair list of %lld entries", (long long)pairs);
    }
    h->w.near_cap = (unsigned long long)pairs;
    h->near_grow = grow != 0;
    return ok();
}

int bemc_query_stats(bemc_handle h, bemc_stats* out)
{
    if (!h || !out) return fail(BEMC_E_INVALID_ARG, "null argument");
    (void)hipSetDevice(h->device);
    (void)h->drain();
    *out = h->last;
    if (h->sticky) {
        const int rc = h->sticky;
        h->sticky = BEMC_OK;
        return fail(rc, "%s", h->sticky_msg.c_str());
    }
    if (h->last_status == BEMC_W_ON_SURFACE) {
        g_last_error = "some field points of the last evaluation lie on an element";
        return BEMC_W_ON_SURFACE;
    }
    return ok();
}

// ----------------------------------------------------------------- serving -------
int bemc_server_start(bemc_handle h, const bemc_server_config* cfg)
{
    if (!h || !cfg) return fail(BEMC_E_INVALID_ARG, "null argument");
    if (!h->have_geometry || h->n_rhs == 0) return fail(BEMC_E_NO_GEOMETRY, "geometry and densities must be uploaded");
    if (h->server) return fail(BEMC_E_INVALID_ARG, "server already running");
    HIP_TRY(hipSetDevice(h->device));
    if (h->drain()) return fail(BEMC_E_DEVICE, "an earlier evaluation failed");
    ServerEnv env{};
    env.device = h->device;
    env.el = h->elements();
    env.rules = h->rules();
    env.near_dr = h->near_dr;
    env.max_depth = h->max_depth;
    env.n_tri = h->n_tri;
    env.n_rect = h->n_rect;
    env.dr_rules = h->dr_rules ? 1 : 0;
    env.lv = h->levels();
    std::string err;
    bemc::Server* s = bemc::Server::create(env, *cfg, err);
    if (!s) return fail(BEMC_E_INVALID_ARG, "%s", err.c_str());
    h->server = s;
    return ok();
}

int bemc_server_submit(bemc_handle h, const double* pts_host, int64_t n, double* phi_host, double* E_host,
                       uint64_t* ticket)
{
    if (!h || !h->server) return fail(BEMC_E_INVALID_ARG, "server not running");
    if (!ticket || (n > 0 && (!pts_host || !phi_host)) || n < 0) return fail(BEMC_E_INVALID_ARG, "bad query arguments");
    std::string err;
    int rc = h->server->submit(pts_host, n, phi_host, E_host, ticket, err);
    if (rc) return fail(rc, "%s", err.c_str());
    return ok();
}

int bemc_server_poll(bemc_handle h, uint64_t ticket, bemc_query_info* info)
{
    if (!h || !h->server || !info) return fail(BEMC_E_INVALID_ARG, "server not running");
    if (!h->server->poll(ticket, info)) return fail(BEMC_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    return ok();
}

int bemc_server_wait(bemc_handle h, uint64_t ticket, double timeout_s, bemc_query_info* info)
{
    if (!h || !h->server) return fail(BEMC_E_INVALID_ARG, "server not running");
    bemc_query_info tmp{};
    bemc_query_info* inf = info ? info : &tmp;
    const int rc = h->server->wait(ticket, timeout_s, inf);
    if (rc == 1) return fail(BEMC_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (rc == 2) return fail(BEMC_E_INVALID_ARG, "timeout");
    if (inf->status != BEMC_OK) return fail(inf->status, "query failed: %s", h->server->last_error().c_str());
    return ok();
}

int bemc_server_stop(bemc_handle h)
{
    if (!h || !h->server) return fail(BEMC_E_INVALID_ARG, "server not running");
    h->server->stop();
    delete h->server;
    h->server = nullptr;
    return ok();
}

}  // extern "C"
