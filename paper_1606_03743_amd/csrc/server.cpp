// Continuous-batching query server.
//
// Geometry and densities stay resident; each free stream slot takes the longest prefix of
// a waiting queue (arrival order) whose points fit into one batch, runs one far-field
// launch over all of them (split over element chunks when the batch is small, with a
// fixed-order reduction of the chunks), the FP64 near field, and copies the results back.
// Slots on different streams overlap on the device; queries arriving while batches run
// are admitted as soon as a slot is free.  Optionally short queries have a queue and a
// slot of their own (the other slots take them only when no long query waits).
#include "server.h"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace bemc {

namespace {
// Workgroups per far-field launch: many times the resident capacity, so that every
// workgroup is short and a batch on another stream gets compute units within a few ms.
constexpr int kWavesTarget = 16 * 1024;
constexpr int kMaxServeSplit = 1024;  // element chunks of one serving launch
constexpr int kSlotSplit = 256;       // partial-sum rows of a slot: kSlotSplit x max_batch_points
constexpr int kPointsPerBlock = 512;  // nominal points per workgroup for sizing the split (the
                                       // far kernels hold 256-768, by precision and rule)
}  // namespace

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
    const unsigned long long near0 = (unsigned long long)std::max<int64_t>(1 << 16, 16 * M);
    // points, results, partial sums, near list (+ its regrouping and 4 result rows) and
    // the per-point near-field segments
    const size_t slot_bytes = (size_t)M * 8 * (3 + 1 + 3 + 4 * (size_t)max_split_) + (size_t)M * 12 +
                              near0 * (3 * sizeof(NearPair) + 8 + 4 * sizeof(double)) + 4096;
    int n_slots = (int)std::min<size_t>((size_t)cfg.n_streams, cfg.mem_budget_bytes / slot_bytes);
    if (n_slots < 1) {
        err = "memory budget too small for one batch slot";
        return false;
    }
    if (hipSetDevice(env.device) != hipSuccess) { err = "hipSetDevice"; return false; }
    slots_.resize((size_t)n_slots);
    for (auto& s : slots_) {
        bool okk = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_pts), (size_t)M * 3 * 8) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_phi), (size_t)M * 8) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_E), (size_t)M * 3 * 8) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_partial), (size_t)M * 4 * 8 * max_split_) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_near), near0 * sizeof(NearPair)) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_ctr), sizeof(DevCounters)) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_pts), (size_t)M * 3 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_out), (size_t)M * 4 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_ctr), sizeof(DevCounters), hipHostMallocDefault) == hipSuccess &&
                   near_work_alloc(s.nw, M, near0, 4) == hipSuccess;
        if (!okk) {
            (void)hipGetLastError();
            err = "out of device or pinned memory for the batch slots";
            return false;
        }
        s.near_cap = near0;
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
        if (s.d_pts) (void)hipFree(s.d_pts);
        if (s.d_phi) (void)hipFree(s.d_phi);
        if (s.d_E) (void)hipFree(s.d_E);
        if (s.d_partial) (void)hipFree(s.d_partial);
        if (s.d_near) (void)hipFree(s.d_near);
        near_work_free(s.nw);
        if (s.d_ctr) (void)hipFree(s.d_ctr);
        if (s.h_pts) (void)hipHostFree(s.h_pts);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.h_ctr) (void)hipHostFree(s.h_ctr);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        s = Slot{};
    }
    slots_.clear();
}

// Enqueue the batch held by slot s (its queries and point count are set).
bool Server::launch(Slot& s, std::string& err)
{
    const int64_t n = s.n;
    if (s.near_cap == 0 || !s.d_near || !s.nw.count) {  // a failed regrowth left no near-field buffers
        err = "batch slot has no near-pair buffers";
        return false;
    }
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
    const int64_t blocks = (n + kPointsPerBlock - 1) / kPointsPerBlock;
    // Element chunks: enough workgroups to fill the chip, and short ones for a small batch
    // so that it finishes soon even while long batches hold most of the compute units;
    // bounded by the partial-sum buffer (max_split_ x max_batch_points rows of 4) and by
    // chunks of at least 64 elements.
    const int64_t cap = (int64_t)max_split_ * cfg_.max_batch_points / std::max<int64_t>(1, n);
    const int n_split = (int)std::max<int64_t>(
        1, std::min({ kWavesTarget / blocks, cap, env_.el.ne / 64, (int64_t)kMaxServeSplit }));
    const int64_t ne = env_.el.ne;
    const int64_t chunk = (ne + n_split - 1) / n_split;
    const double K = coulomb_constant();
    hipError_t e = hipMemcpyAsync(s.d_pts, s.h_pts, (size_t)n * 3 * 8, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = launch_zero_counters(s.d_ctr, s.stream);
    FarArgs fa{};
    fa.el = env_.el;
    fa.rules = env_.rules;
    fa.pts = s.d_pts;
    fa.n = n;
    fa.rhs = 0;
    fa.n_rhs = 1;
    fa.K = K;
    fa.phi = s.d_phi;
    fa.E = s.d_E;
    fa.partial = n_split > 1 ? s.d_partial : nullptr;
    fa.elem_begin = 0;
    fa.elem_end = ne;
    fa.n_split = n_split;
    fa.chunk = chunk;
    fa.near_list = s.d_near;
    fa.near_cap = s.near_cap;
    fa.ctr = s.d_ctr;
    fa.dr_rules = env_.dr_rules;
    fa.lv = env_.lv;
    if (e == hipSuccess) e = launch_near_list(s.d_pts, n, env_.el, s.d_near, s.near_cap, s.d_ctr, s.stream);
    if (e == hipSuccess) e = launch_far_eval(fa, cfg_.precision, s.stream);
    if (e == hipSuccess && n_split > 1) e = launch_reduce_split(s.d_partial, n_split, n, K, s.d_phi, s.d_E, s.stream);
    NearArgs na{};
    na.el = env_.el;
    na.rules = env_.rules;
    na.pts = s.d_pts;
    na.n = n;
    na.rhs = 0;
    na.n_rhs = 1;
    na.K = K;
    na.phi = s.d_phi;
    na.E = s.d_E;
    na.near_list = s.d_near;
    na.near_cap = s.near_cap;
    na.slot = s.nw.slot;
    na.res = s.nw.res;
    na.ctr = s.d_ctr;
    na.near_dr2 = env_.near_dr * env_.near_dr;
    na.max_depth = env_.max_depth;
    na.visit_limit = 1ll << 22;
    if (e == hipSuccess) e = near_order(s.d_near, s.d_ctr, s.near_cap, n, s.nw, s.stream);
    if (e == hipSuccess) e = launch_near(na, kNearEval, s.stream);
    if (e == hipSuccess)
        e = near_reduce(s.nw, n, kNearEval, s.d_phi, s.d_E, nullptr, env_.el.q, ne, 1, K, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out, s.d_phi, (size_t)n * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out + n, s.d_E, (size_t)n * 3 * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_ctr, s.d_ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    return true;
}

void Server::complete(Slot& s)
{
    const int64_t n = s.n;
    if (s.h_ctr->near_count > s.near_cap) {
        // near-pair list overflowed: grow it and run the batch again (synchronously)
        const unsigned long long cap = s.h_ctr->near_count + s.h_ctr->near_count / 4;
        (void)hipFree(s.d_near);
        s.d_near = nullptr;
        if (cap > kMaxNearPairs || hipMalloc(reinterpret_cast<void**>(&s.d_near), cap * sizeof(NearPair)) != hipSuccess ||
            near_work_alloc(s.nw, cfg_.max_batch_points, cap, 4) != hipSuccess) {
            (void)hipGetLastError();
            s.near_cap = 0;
        } else {
            s.near_cap = cap;
        }
        std::string err;
        bool relaunched = false;
        if (s.near_cap) {
            std::lock_guard<std::mutex> lk(mu_);
            relaunched = launch(s, err);
        }
        if (relaunched && hipEventSynchronize(s.done) == hipSuccess && s.h_ctr->near_count <= s.near_cap) {
            // fall through to the scatter below
        } else {
            std::lock_guard<std::mutex> lk(mu_);
            err_ = "near-pair list could not be grown";
            for (uint64_t id : s.queries) {
                Query& q = queries_[id];
                q.info.status = BEMC_E_OUT_OF_MEMORY;
                q.info.done = 1;
                q.info.end_s = now();
            }
            s.busy = false;
            s.queries.clear();
            done_cv_.notify_all();
            return;
        }
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
    const double t = now();
    std::lock_guard<std::mutex> lk(mu_);
    for (uint64_t id : ids) {
        Query& q = queries_[id];
        q.info.status = s.h_ctr->visit_limit_hits ? BEMC_E_LIMIT : BEMC_OK;
        q.info.done = 1;
        q.info.end_s = t;
    }
    s.busy = false;
    s.queries.clear();
    done_cv_.notify_all();
}

void Server::loop()
{
    (void)hipSetDevice(env_.device);
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
        bool progressed = false;
        // completions
        for (auto& s : slots_) {
            if (!s.busy) continue;
            if (hipEventQuery(s.done) == hipSuccess) {
                lk.unlock();
                complete(s);
                lk.lock();
                progressed = true;
            }
        }
        // admissions: each free slot takes the longest prefix of its queue that fits
        for (auto& s : slots_) {
            if (s.busy) continue;
            std::deque<uint64_t>* wq = s.small_only ? &waiting_small_ : (waiting_.empty() ? &waiting_small_ : &waiting_);
            if (wq->empty()) continue;
            int64_t pts = 0;
            s.queries.clear();
            while (!wq->empty()) {
                Query& q = queries_[wq->front()];
                if (pts + q.n > cfg_.max_batch_points) break;
                pts += q.n;
                s.queries.push_back(q.id);
                wq->pop_front();
            }
            if (s.queries.empty()) continue;
            s.n = pts;
            s.batch_id = next_batch_++;
            const double t = now();
            for (uint64_t id : s.queries) {
                Query& q = queries_[id];
                q.info.start_s = t;
                q.info.batch_id = s.batch_id;
                q.info.batch_points = pts;
            }
            s.busy = true;
            std::string err;
            bool launched;
            if (pts == 0) {
                launched = true;  // only empty queries: nothing to run
                (void)hipEventRecord(s.done, s.stream);
                std::memset(s.h_ctr, 0, sizeof(DevCounters));
            } else {
                launched = launch(s, err);
            }
            if (!launched) {
                err_ = err;
                for (uint64_t id : s.queries) {
                    Query& q = queries_[id];
                    q.info.status = BEMC_E_DEVICE;
                    q.info.done = 1;
                    q.info.end_s = now();
                }
                s.busy = false;
                s.queries.clear();
                done_cv_.notify_all();
            }
            progressed = true;
        }
        bool any_busy = false;
        for (auto& s : slots_) any_busy |= s.busy;
        if (stopping_ && waiting_.empty() && waiting_small_.empty() && !any_busy) break;
        if (!progressed) cv_.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 2000));
    }
}

}  // namespace bemc
