// Continuous-batching query server.
//
// Geometry and densities stay resident; each free stream slot takes the longest prefix of
// a waiting queue (arrival order) whose points fit into one batch and whose device memory
// fits what the memory budget has left, runs one far-field launch over all of them (split
// over element chunks when the batch is small, with a fixed-order reduction of the
// chunks), the FP64 near field, and copies the results back.  Slots on different streams
// overlap on the device; queries arriving while batches run are admitted as soon as a slot
// and memory are free.  Optionally short queries have a queue and a slot of their own (the
// other slots take them only when no long query waits).
//
// Memory: one device allocation made at start (the budget, at most twice what full batches
// on every stream need) is handed out per batch by a first-fit list on the host; a batch
// takes a block for its per-point buffers and one for its near-pair list when it is admitted
// and gives both back when it completes; the list is sized from the near-pair density of the
// batches before it (16 pairs per point at first, then 1.25 x the density seen, raised at
// once and lowered slowly).  The whole
// batch is enqueued at admission.  When its list pass found more near pairs than the list
// holds, the completed batch's far field is kept, the list grows (a larger block) and only
// the list pass and the near stage run again; a growth that does not fit waits while
// another batch is running and will give memory back, and otherwise takes its block outside
// the arena (stream-ordered), so at most one batch at a time exceeds the budget, by its
// list.  No scheduler step waits on the device.
#include "server.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace bemc {

namespace {
// Workgroups per far-field launch: many times the resident capacity, so that every
// workgroup is short and a batch on another stream gets compute units within a few ms.
constexpr int kWavesTarget = 16 * 1024;
constexpr int kMaxServeSplit = 1024;  // element chunks of one serving launch
constexpr int kSlotSplit = 256;       // partial-sum rows of a batch: kSlotSplit x max_batch_points
constexpr int kPointsPerBlock = 512;  // nominal points per workgroup for sizing the split (the
                                       // far kernels hold 256-768, by precision and rule)
constexpr size_t kGranule = 256;

size_t up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }
}  // namespace

// ---------------------------------------------------------------------- arena -----
hipError_t Arena::init(size_t bytes)
{
    bytes = up(bytes);
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(&base_), bytes);
    if (e != hipSuccess) {
        base_ = nullptr;
        return e;
    }
    size_ = bytes;
    used_ = 0;
    free_.clear();
    free_[0] = bytes;
    return hipSuccess;
}

void Arena::destroy()
{
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
    size_ = used_ = 0;
    free_.clear();
}

size_t Arena::take(size_t bytes)
{
    bytes = up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        return off;
    }
    return kNone;
}

void Arena::give(size_t off, size_t bytes)
{
    if (off == kNone) return;
    bytes = up(std::max<size_t>(bytes, 1));
    used_ -= std::min(used_, bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
        it->second += next->second;
        free_.erase(next);
    }
    if (it != free_.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            free_.erase(it);
        }
    }
}

// --------------------------------------------------------------------- server -----
double Server::now() const
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count() - t0_;
}

Server* Server::create(const ServerEnv& env, const bemc_server_config& cfg, std::string& err)
{
    Server* s = new Server();
    if (!s->init(env, cfg, err)) {
        s->stop();
        delete s;
        return nullptr;
    }
    return s;
}

int Server::split_for(int64_t n) const
{
    const int64_t blocks = (n + kPointsPerBlock - 1) / kPointsPerBlock;
    // Element chunks: enough workgroups to fill the chip, and short ones for a small batch
    // so that it finishes soon even while long batches hold most of the compute units;
    // partial sums bounded by max_split_ x max_batch_points rows of 4; chunks of at least 64
    // elements.
    const int64_t cap = (int64_t)max_split_ * cfg_.max_batch_points / std::max<int64_t>(1, n);
    return (int)std::max<int64_t>(
        1, std::min({ kWavesTarget / std::max<int64_t>(1, blocks), cap, env_.el.ne / 64, (int64_t)kMaxServeSplit }));
}

unsigned long long Server::initial_near(int64_t n, bool base) const
{
    const double pairs = std::ceil((base ? 16.0 : pairs_per_point_) * (double)n);
    return (unsigned long long)std::min<double>(std::max<double>(4096.0, pairs), (double)kMaxNearPairs);
}

// points, far results, far + near results, partial sums for the batch's element chunks, the
// near stage's per-point segments and scan workspace
size_t Server::fix_bytes(int64_t n) const
{
    const int ns = split_for(n);
    return up((size_t)n * 8 * 3) + 2 * up((size_t)n * 8 * 4) + (ns > 1 ? up((size_t)ns * 4 * 8 * (size_t)n) : 0) +
           3 * up((size_t)n * 4) + up(near_scan_temp_bytes(std::max<int64_t>(n, 1)));
}

// the near-pair list, its regrouping, cost order and result records (4 rows)
size_t Server::pair_bytes(int64_t, unsigned long long pairs)
{
    const size_t p = (size_t)pairs;
    return up(p * sizeof(NearPair)) * 4 + up(p * 4) * 3 + up(p) + up(p * 4 * 8) + up(3 * kCostClasses * 4);
}

void Server::carve_fix(Slot& s)
{
    const int64_t n = s.n;
    char* p = arena_.base() + s.fix_off;
    auto take = [&](size_t b) { char* q = p; p += up(b); return q; };
    s.d_pts = reinterpret_cast<double*>(take((size_t)n * 8 * 3));
    s.d_far = reinterpret_cast<double*>(take((size_t)n * 8 * 4));
    s.d_out = reinterpret_cast<double*>(take((size_t)n * 8 * 4));
    s.d_partial = s.n_split > 1 ? reinterpret_cast<double*>(take((size_t)s.n_split * 4 * 8 * (size_t)n)) : nullptr;
    s.nw.count = reinterpret_cast<uint32_t*>(take((size_t)n * 4));
    s.nw.start = reinterpret_cast<uint32_t*>(take((size_t)n * 4));
    s.nw.cursor = reinterpret_cast<uint32_t*>(take((size_t)n * 4));
    s.nw.temp_bytes = near_scan_temp_bytes(std::max<int64_t>(n, 1));
    s.nw.temp = take(s.nw.temp_bytes);
}

// the near-pair arrays of a list of s.near_cap pairs in the block at base (pair_bytes of it)
void Server::carve_pairs(Slot& s, char* base)
{
    const size_t c = (size_t)s.near_cap;
    char* p = base;
    auto take = [&](size_t b) { char* q = p; p += up(b); return q; };
    s.d_near = reinterpret_cast<NearPair*>(take(c * sizeof(NearPair)));
    s.nw.grouped = reinterpret_cast<NearPair*>(take(c * sizeof(NearPair)));
    s.nw.sorted = reinterpret_cast<NearPair*>(take(c * sizeof(NearPair)));
    s.nw.origin = reinterpret_cast<uint32_t*>(take(c * 4));
    s.nw.slot = reinterpret_cast<uint32_t*>(take(c * 4));
    s.nw.order = reinterpret_cast<uint32_t*>(take(c * 4));
    s.nw.opair = reinterpret_cast<NearPair*>(take(c * sizeof(NearPair)));
    s.nw.cost = reinterpret_cast<uint8_t*>(take(c));
    s.nw.res = reinterpret_cast<double*>(take(c * 4 * 8));
    s.nw.buckets = reinterpret_cast<uint32_t*>(take(3 * kCostClasses * 4));
}

void Server::release(Slot& s)
{
    arena_.give(s.fix_off, s.fix_bytes);
    arena_.give(s.pair_off, s.pair_bytes);
    if (s.spill) (void)hipFreeAsync(s.spill, s.stream);
    s.spill = nullptr;
    s.fix_off = s.pair_off = Arena::kNone;
    s.fix_bytes = s.pair_bytes = 0;
    s.near_cap = 0;
}

bool Server::init(const ServerEnv& env, const bemc_server_config& cfg, std::string& err)
{
    env_ = env;
    cfg_ = cfg;
    t0_ = 0.0;
    t0_ = now();
    if (cfg.max_batch_points < 1 || cfg.max_batch_points >= (1ll << 31) || cfg.n_streams < 1 || cfg.n_streams > 8 ||
        (cfg.precision != BEMC_FP64 && cfg.precision != BEMC_MIXED) || cfg.small_query_points < 0) {
        err = "invalid server configuration";
        return false;
    }
    const int64_t M = cfg.max_batch_points;
    const int64_t blocks = (M + kPointsPerBlock - 1) / kPointsPerBlock;
    max_split_ = (int)std::max<int64_t>(1, std::min<int64_t>(kSlotSplit, kWavesTarget / std::max<int64_t>(1, blocks)));
    const size_t full = fix_bytes(M) + pair_bytes(M, initial_near(M, true));
    if (full > cfg.mem_budget_bytes) {
        err = "memory budget too small for one batch of max_batch_points";
        return false;
    }
    if (hipSetDevice(env.device) != hipSuccess) { err = "hipSetDevice"; return false; }
    // the budget, but no more than twice what full batches on every stream need (room for
    // near-list growth)
    const size_t arena = std::min<size_t>(cfg.mem_budget_bytes, 2 * full * (size_t)cfg.n_streams);
    if (arena_.init(arena) != hipSuccess) {
        (void)hipGetLastError();
        err = "out of device memory for the batch arena";
        return false;
    }
    slots_.resize((size_t)cfg.n_streams);
    for (auto& s : slots_) {
        bool okk = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_ctr), sizeof(DevCounters)) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_pts), (size_t)M * 3 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_out), (size_t)M * 4 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_ctr), sizeof(DevCounters), hipHostMallocDefault) == hipSuccess;
        if (!okk) {
            (void)hipGetLastError();
            err = "out of device or pinned memory for the batch slots";
            return false;
        }
    }
    if (cfg.small_query_points > 0 && slots_.size() >= 2) slots_.back().small_only = true;
    thread_ = std::thread([this] { loop(); });
    return true;
}

Server::~Server() { stop(); }

std::string Server::last_error()
{
    std::lock_guard<std::mutex> lk(mu_);
    return err_;
}

int Server::submit(const double* pts, int64_t n, double* phi, double* E, uint64_t* ticket, std::string& err)
{
    if (n > cfg_.max_batch_points) {
        err = "query larger than max_batch_points";
        return BEMC_E_ADMISSION;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) {
        err = "server is stopping";
        return BEMC_E_INVALID_ARG;
    }
    Query q{};
    q.id = next_id_++;
    q.pts = pts;
    q.n = n;
    q.phi = phi;
    q.E = E;
    q.info.submit_s = now();
    q.info.batch_id = -1;
    q.small = cfg_.small_query_points > 0 && n <= cfg_.small_query_points;
    queries_.emplace(q.id, q);
    (q.small ? waiting_small_ : waiting_).push_back(q.id);
    *ticket = q.id;
    cv_.notify_one();
    return BEMC_OK;
}

bool Server::poll(uint64_t ticket, bemc_query_info* info)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = queries_.find(ticket);
    if (it == queries_.end()) return false;
    *info = it->second.info;
    return true;
}

int Server::wait(uint64_t ticket, double timeout_s, bemc_query_info* info)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = queries_.find(ticket);
    if (it == queries_.end()) return 1;
    auto pred = [&] { return queries_[ticket].info.done != 0; };
    if (timeout_s < 0) {
        done_cv_.wait(lk, pred);
    } else if (!done_cv_.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        *info = queries_[ticket].info;
        return 2;
    }
    *info = queries_[ticket].info;
    queries_.erase(ticket);  // delivered: the record is released
    return 0;
}

void Server::stop()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stopping_ = true;
        cv_.notify_all();
    }
    if (thread_.joinable()) thread_.join();
    (void)hipSetDevice(env_.device);
    for (auto& s : slots_) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.d_ctr) (void)hipFree(s.d_ctr);
        if (s.h_pts) (void)hipHostFree(s.h_pts);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.h_ctr) (void)hipHostFree(s.h_ctr);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        s = Slot{};
    }
    slots_.clear();
    arena_.destroy();
}

// The near stage of the batch in s (its list holds near_cap pairs): the far field is
// copied to the output, the near pairs regrouped and ordered, the near field added in
// fixed order, the results and counters copied to pinned memory, the completion event.
bool Server::near_stage(Slot& s, std::string& err)
{
    const int64_t n = s.n, ne = env_.el.ne;
    const double K = coulomb_constant();
    NearArgs na{};
    na.el = env_.el;
    na.rules = env_.rules;
    na.pts = s.d_pts;
    na.n = n;
    na.rhs = 0;
    na.n_rhs = 1;
    na.K = K;
    na.phi = s.d_out;
    na.E = s.d_out + n;
    na.near_list = s.d_near;
    na.near_cap = s.near_cap;
    na.slot = s.nw.slot;
    na.order = s.nw.order;
    na.opair = s.nw.opair;
    na.walk_end = near_walk_end(s.nw);
    na.heavy_end = near_heavy_end(s.nw);
    // depth first only: the breadth-first walk needs more registers than a finished far-field
    // wave of another stream frees, so its workgroups would wait for a long batch to drain
    na.deep = 0;
    na.res = s.nw.res;
    na.ctr = s.d_ctr;
    na.near_dr2 = env_.near_dr * env_.near_dr;
    na.max_depth = env_.max_depth;
    na.visit_limit = 1ll << 22;
    // d_out = the far field (the element-chunk partial sums, or d_far with one chunk) + the near
    // field; both stay, so a repeated near stage starts from them again
    hipError_t e = near_order(s.d_near, s.d_ctr, s.near_cap, n, s.d_pts, env_.el, s.nw, false, s.stream);
    if (e == hipSuccess) e = launch_near(na, kNearEval, s.stream);
    if (e == hipSuccess)
        e = near_finish(s.nw, n, kNearEval, 4, s.n_split > 1 ? s.d_partial : nullptr, s.n_split, 4, s.d_far, K,
                        nullptr, s.d_out, s.d_out + n, s.d_ctr, nullptr, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out, s.d_out, (size_t)n * 4 * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_ctr, s.d_ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    s.state = kRun;
    return true;
}

// The whole batch, enqueued at admission (its blocks are taken): copy-in, near-pair list,
// far field (chunk partial sums, or the far results with one chunk), near stage.
bool Server::launch(Slot& s, std::string& err)
{
    const int64_t n = s.n;
    // pack points SoA into pinned staging
    int64_t off = 0;
    for (uint64_t id : s.queries) {
        Query& q = queries_[id];
        for (int64_t i = 0; i < q.n; ++i) {
            s.h_pts[off + i] = q.pts[3 * i];
            s.h_pts[n + off + i] = q.pts[3 * i + 1];
            s.h_pts[2 * n + off + i] = q.pts[3 * i + 2];
        }
        off += q.n;
    }
    const int64_t ne = env_.el.ne;
    const double K = coulomb_constant();
    hipError_t e = hipMemcpyAsync(s.d_pts, s.h_pts, (size_t)n * 3 * 8, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = launch_zero_counters(s.d_ctr, s.stream);
    if (e == hipSuccess) e = launch_near_list(s.d_pts, n, env_.el, s.d_near, s.near_cap, s.d_ctr, s.stream);
    FarArgs fa{};
    fa.el = env_.el;
    fa.rules = env_.rules;
    fa.pts = s.d_pts;
    fa.n = n;
    fa.rhs = 0;
    fa.n_rhs = 1;
    fa.K = K;
    fa.phi = s.d_far;
    fa.E = s.d_far + n;
    fa.partial = s.n_split > 1 ? s.d_partial : nullptr;
    fa.elem_begin = 0;
    fa.elem_end = ne;
    fa.n_split = s.n_split;
    fa.chunk = (ne + s.n_split - 1) / s.n_split;
    fa.near_list = s.d_near;
    fa.near_cap = s.near_cap;
    fa.ctr = s.d_ctr;
    fa.dr_rules = env_.dr_rules;
    fa.lv = env_.lv;
    if (e == hipSuccess) e = launch_far_eval(fa, cfg_.precision, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    return near_stage(s, err);
}

// The batch's list overflowed (its stream is idle): give back the list's block, take one
// for 1.25 x the pairs found, list again and repeat the near stage.  Returns 1 when the block
// does not fit now (the batch waits), < 0 on an error.
int Server::grow(Slot& s, std::string& err)
{
    const unsigned long long found = s.h_ctr->near_count;
    if (found > kMaxNearPairs) {
        err = "near pairs of a batch exceed 2^32 - 1";
        return BEMC_E_LIMIT;
    }
    arena_.give(s.pair_off, s.pair_bytes);
    s.pair_off = Arena::kNone;
    s.pair_bytes = 0;
    if (s.spill) (void)hipFreeAsync(s.spill, s.stream);
    s.spill = nullptr;
    const unsigned long long cap = std::min(found + found / 4, kMaxNearPairs);
    const size_t b = pair_bytes(s.n, cap);
    const size_t off = arena_.take(b);
    s.near_cap = cap;  // before carving: the arrays are laid out for it
    if (off != Arena::kNone) {
        s.pair_off = off;
        s.pair_bytes = b;
        carve_pairs(s, arena_.base() + off);
    } else {
        bool running = false;
        for (auto& o : slots_) running |= (&o != &s && o.state == kRun);
        if (running) {
            s.near_cap = 0;  // no list while it waits (the count to grow to stays in h_ctr)
            s.state = kGrow;
            return 1;  // another batch will give memory back
        }
        // nothing can give memory back: this batch alone goes beyond the budget, by its list
        if (hipMallocAsync(reinterpret_cast<void**>(&s.spill), b, s.stream) != hipSuccess) {
            (void)hipGetLastError();
            s.spill = nullptr;
            err = "out of device memory for a batch's near-pair list";
            return BEMC_E_OUT_OF_MEMORY;
        }
        carve_pairs(s, s.spill);
    }
    hipError_t e = launch_reset_near_stage(s.d_ctr, s.stream);  // the near stage runs again from pair 0
    if (e == hipSuccess) e = launch_near_list(s.d_pts, s.n, env_.el, s.d_near, s.near_cap, s.d_ctr, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return BEMC_E_DEVICE;
    }
    if (!near_stage(s, err)) return BEMC_E_DEVICE;
    return 0;
}

// Every query of the batch ends with `status`; the batch's blocks are given back.
void Server::fail_batch(Slot& s, int status, const std::string& err)
{
    (void)hipStreamSynchronize(s.stream);  // nothing of the batch may still use its blocks
    release(s);
    std::lock_guard<std::mutex> lk(mu_);
    err_ = err;
    for (uint64_t id : s.queries) {
        Query& q = queries_[id];
        q.info.status = status;
        q.info.done = 1;
        q.info.end_s = now();
    }
    s.state = kIdle;
    s.queries.clear();
    done_cv_.notify_all();
}

void Server::complete(Slot& s)
{
    const int64_t n = s.n;
    if (n > 0) {  // the list size of the next batches follows the near-pair density seen
        const double want = 1.25 * (double)s.h_ctr->near_count / (double)n;
        pairs_per_point_ = want > pairs_per_point_ ? want : std::max(16.0, 0.99 * pairs_per_point_ + 0.01 * want);
    }
    std::vector<uint64_t> ids;
    {
        std::lock_guard<std::mutex> lk(mu_);
        ids = s.queries;
    }
    int64_t off = 0;
    for (uint64_t id : ids) {
        Query* q;
        {
            std::lock_guard<std::mutex> lk(mu_);
            q = &queries_[id];
        }
        for (int64_t i = 0; i < q->n; ++i) {
            q->phi[i] = s.h_out[off + i];
            if (q->E) {
                q->E[3 * i] = s.h_out[n + off + i];
                q->E[3 * i + 1] = s.h_out[2 * n + off + i];
                q->E[3 * i + 2] = s.h_out[3 * n + off + i];
            }
        }
        off += q->n;
    }
    release(s);
    const double t = now();
    std::lock_guard<std::mutex> lk(mu_);
    for (uint64_t id : ids) {
        Query& q = queries_[id];
        q.info.status = s.h_ctr->visit_limit_hits ? BEMC_E_LIMIT : BEMC_OK;
        q.info.done = 1;
        q.info.end_s = t;
    }
    s.state = kIdle;
    s.queries.clear();
    done_cv_.notify_all();
}

void Server::loop()
{
    (void)hipSetDevice(env_.device);
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
        bool progressed = false;
        // completions, list growths (outside the lock: they copy results and enqueue)
        for (auto& s : slots_) {
            const bool finished = s.state == kRun && hipEventQuery(s.done) == hipSuccess;
            if (!finished && s.state != kGrow) continue;
            lk.unlock();
            if (s.n > 0 && s.h_ctr->near_count > s.near_cap) {  // the list overflowed
                std::string err;
                const int rc = grow(s, err);
                if (rc < 0) fail_batch(s, rc, err);
                progressed |= rc != 1;
            } else {
                complete(s);
                progressed = true;
            }
            lk.lock();
        }
        // admissions: each free slot takes the longest prefix of its queue that fits one
        // batch and the memory left
        for (auto& s : slots_) {
            if (s.state != kIdle) continue;
            std::deque<uint64_t>* wq = s.small_only ? &waiting_small_ : (waiting_.empty() ? &waiting_small_ : &waiting_);
            if (wq->empty()) continue;
            // points of the longest prefix within max_batch_points, then shortened until its
            // blocks fit the arena
            int64_t pts = 0;
            size_t k = 0;
            for (; k < wq->size(); ++k) {
                const int64_t qn = queries_[(*wq)[k]].n;
                if (pts + qn > cfg_.max_batch_points) break;
                pts += qn;
            }
            size_t fo = Arena::kNone, po = Arena::kNone, fb = 0, pb = 0;
            unsigned long long cap = 0;
            auto fits = [&](bool base) {
                fb = fix_bytes(pts);
                cap = initial_near(pts, base);
                pb = pair_bytes(pts, cap);
                fo = arena_.take(fb);
                po = fo == Arena::kNone ? Arena::kNone : arena_.take(pb);
                if (po != Arena::kNone) return true;
                arena_.give(fo, fb);
                fo = Arena::kNone;
                return false;
            };
            while (k > 0 && pts > 0 && !fits(false)) pts -= queries_[(*wq)[--k]].n;
            if (k == 0) {
                // not even the first query with the density seen: with nothing in flight that
                // could give memory back, it starts with the base list (which always fits)
                bool busy = false;
                for (auto& o : slots_) busy |= o.state != kIdle;
                if (busy) continue;  // the first query waits for memory
                k = 1;
                pts = queries_[wq->front()].n;
                if (!fits(true)) continue;  // (unreachable: one base batch fits the arena)
            }
            s.queries.assign(wq->begin(), wq->begin() + (std::ptrdiff_t)k);
            wq->erase(wq->begin(), wq->begin() + (std::ptrdiff_t)k);
            s.n = pts;
            s.batch_id = next_batch_++;
            const double t = now();
            for (uint64_t id : s.queries) {
                Query& q = queries_[id];
                q.info.start_s = t;
                q.info.batch_id = s.batch_id;
                q.info.batch_points = pts;
            }
            progressed = true;
            std::string err;
            if (pts == 0) {  // only empty queries: nothing to run
                std::memset(s.h_ctr, 0, sizeof(DevCounters));
                s.state = kRun;
                if (hipEventRecord(s.done, s.stream) == hipSuccess) continue;
                err = "hipEventRecord";
            } else {
                s.fix_off = fo; s.fix_bytes = fb;
                s.pair_off = po; s.pair_bytes = pb;
                s.n_split = split_for(pts);
                s.near_cap = cap;
                carve_fix(s);
                carve_pairs(s, arena_.base() + po);
                if (launch(s, err)) continue;
            }
            lk.unlock();
            fail_batch(s, BEMC_E_DEVICE, err);
            lk.lock();
        }
        bool any_busy = false;
        for (auto& s : slots_) any_busy |= s.state != kIdle;
        if (stopping_ && waiting_.empty() && waiting_small_.empty() && !any_busy) break;
        if (!progressed) cv_.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 2000));
    }
}

}  // namespace bemc
