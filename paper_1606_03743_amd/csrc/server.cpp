// Continuous-batching query server.
//
// Geometry and densities stay resident; each free stream slot takes the longest prefix of
// a waiting queue (arrival order) whose points fit into one batch and whose device memory
// fits what the budget has left, runs one far-field launch over all of them (split over
// element chunks when the batch is small, with a fixed-order reduction of the chunks), the
// FP64 near field, and copies the results back.  Slots on different streams overlap on
// the device; queries arriving while batches run are admitted as soon as a slot and memory
// are free.  Optionally short queries have a queue and a slot of their own (the other slots
// take them only when no long query waits).
//
// Memory: each batch allocates its buffers on its own stream (stream-ordered allocation
// from the device's pool) when it is admitted and releases them when it completes; the
// scheduler accounts their bytes against the budget.  A batch runs in two phases: the
// near-pair list pass, the far field and the chunk reduction are enqueued at admission;
// once the list pass's pair count has reached the host (about a millisecond later, while
// the far field runs), the near stage is enqueued -- after growing the batch's list on its
// own stream when it was too short.  No host wait stalls the other slots, and the far
// field is never repeated.
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
constexpr size_t kNearPairBytes = sizeof(NearPair) + kNearWorkBytesPerPair + 4 * sizeof(double);

template <typename T>
hipError_t alloc_async(T** p, size_t count, hipMemPool_t pool, hipStream_t s)
{
    return hipMallocFromPoolAsync(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T), pool, s);
}
template <typename T>
void free_async(T*& p, hipStream_t s)
{
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
}
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

unsigned long long Server::initial_near(int64_t n) const
{
    return (unsigned long long)std::max<int64_t>(4096, 16 * n);
}

// points, potential and field, element-chunk partial sums, near-pair list with its
// regrouping, cost order and result records, per-point segments and scan workspace
size_t Server::batch_bytes(int64_t n, unsigned long long near_pairs) const
{
    const int ns = split_for(n);
    return (size_t)n * 8 * (3 + 1 + 3) + (ns > 1 ? (size_t)ns * 4 * 8 * (size_t)n : 0) +
           near_pairs * sizeof(NearPair) + near_work_bytes(n, near_pairs, 4);
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
    if (batch_bytes(M, initial_near(M)) > cfg.mem_budget_bytes) {
        err = "memory budget too small for one batch of max_batch_points";
        return false;
    }
    if (hipSetDevice(env.device) != hipSuccess) { err = "hipSetDevice"; return false; }
    // the server's own memory pool: released batch memory stays in it (up to the budget)
    // instead of going back to the driver at every synchronisation, and memory released on
    // one stream is reused on another only once that release has completed (no dependency
    // between the streams is ever inserted: a short batch never waits for a long one)
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = env.device;
    if (hipMemPoolCreate(&pool_, &props) != hipSuccess) {
        (void)hipGetLastError();
        pool_ = nullptr;
        err = "could not create the batch memory pool";
        return false;
    }
    uint64_t thr = cfg.mem_budget_bytes;
    int no = 0;
    if (hipMemPoolSetAttribute(pool_, hipMemPoolAttrReleaseThreshold, &thr) != hipSuccess ||
        hipMemPoolSetAttribute(pool_, hipMemPoolReuseAllowInternalDependencies, &no) != hipSuccess) {
        (void)hipGetLastError();
        err = "could not configure the batch memory pool";
        return false;
    }
    slots_.resize((size_t)cfg.n_streams);
    for (auto& s : slots_) {
        bool okk = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&s.listed, hipEventDisableTiming) == hipSuccess &&
                   hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess &&
                   hipMalloc(reinterpret_cast<void**>(&s.d_ctr), sizeof(DevCounters)) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_pts), (size_t)M * 3 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_out), (size_t)M * 4 * 8, hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_ctr), sizeof(DevCounters), hipHostMallocDefault) == hipSuccess &&
                   hipHostMalloc(reinterpret_cast<void**>(&s.h_list), sizeof(DevCounters), hipHostMallocDefault) == hipSuccess;
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
        if (s.stream) {
            free_batch(s);
            (void)hipStreamSynchronize(s.stream);
        }
        if (s.d_ctr) (void)hipFree(s.d_ctr);
        if (s.h_pts) (void)hipHostFree(s.h_pts);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.h_ctr) (void)hipHostFree(s.h_ctr);
        if (s.h_list) (void)hipHostFree(s.h_list);
        if (s.listed) (void)hipEventDestroy(s.listed);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        s = Slot{};
    }
    slots_.clear();
    if (pool_) (void)hipMemPoolDestroy(pool_);  // every allocation of it has been released
    pool_ = nullptr;
}

bool Server::alloc_batch(Slot& s, std::string& err)
{
    const int64_t n = s.n;
    s.n_split = split_for(n);
    s.near_cap = initial_near(n);
    hipError_t e = alloc_async(&s.d_pts, (size_t)n * 3, pool_, s.stream);
    if (e == hipSuccess) e = alloc_async(&s.d_phi, (size_t)n, pool_, s.stream);
    if (e == hipSuccess) e = alloc_async(&s.d_E, (size_t)n * 3, pool_, s.stream);
    if (e == hipSuccess && s.n_split > 1)
        e = alloc_async(&s.d_partial, (size_t)s.n_split * 4 * (size_t)n, pool_, s.stream);
    if (e == hipSuccess) e = alloc_async(&s.d_near, (size_t)s.near_cap, pool_, s.stream);
    if (e == hipSuccess) e = near_work_alloc_async(s.nw, n, s.near_cap, 4, pool_, s.stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        err = std::string("batch buffers: ") + hipGetErrorString(e);
        free_batch(s);
        return false;
    }
    s.bytes = batch_bytes(n, s.near_cap);
    mem_used_ += s.bytes;
    return true;
}

void Server::free_batch(Slot& s)
{
    free_async(s.d_pts, s.stream);
    free_async(s.d_phi, s.stream);
    free_async(s.d_E, s.stream);
    free_async(s.d_partial, s.stream);
    free_async(s.d_near, s.stream);
    near_work_free_async(s.nw, s.stream);
    mem_used_ -= std::min(mem_used_, s.bytes);
    s.bytes = 0;
    s.near_cap = 0;
}

// Phase 1, enqueued at admission: copy-in, near-pair list pass (its count copied to the
// host and marked by s.listed), far field and chunk reduction.
bool Server::launch_far(Slot& s, std::string& err)
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
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_list, s.d_ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.listed, s.stream);
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
    if (e == hipSuccess && s.n_split > 1)
        e = launch_reduce_split(s.d_partial, s.n_split, n, K, s.d_phi, s.d_E, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    s.state = kFar;
    return true;
}

// Phase 2, once the list pass's count is on the host: grow the list on the batch's stream
// if it was too short (and list again; the far field stays), then regrouping, near field,
// ordered sums, copy-out.  Returns 1 when the grown list does not fit the memory left while
// another batch is in its near stage (the batch waits for it), < 0 on an error.
int Server::near_stage(Slot& s, std::string& err)
{
    const int64_t n = s.n;
    const unsigned long long found = s.h_list->near_count;
    hipError_t e = hipSuccess;
    if (found > s.near_cap) {
        if (found > kMaxNearPairs) {
            err = "near pairs of a batch exceed 2^32 - 1";
            return BEMC_E_LIMIT;
        }
        const unsigned long long cap = std::min(found + found / 4, kMaxNearPairs);
        const size_t grown = batch_bytes(n, cap);
        const size_t extra = grown - std::min(grown, s.bytes);
        if (mem_used_ + extra > cfg_.mem_budget_bytes) {
            // wait while another batch is in its near stage: it completes without further
            // memory and releases its buffers.  Otherwise (the other batches in flight are
            // waiting for their own pair counts or growths) grow beyond the budget: then this
            // batch is in its near stage and the others wait for it, so at most one batch at a
            // time exceeds the budget and no two batches wait for each other.
            bool draining = false;
            for (auto& o : slots_) draining |= (&o != &s && o.state == kNear);
            if (draining) return 1;
        }
        free_async(s.d_near, s.stream);
        near_work_free_async(s.nw, s.stream);
        e = alloc_async(&s.d_near, (size_t)cap, pool_, s.stream);
        if (e == hipSuccess) e = near_work_alloc_async(s.nw, n, cap, 4, pool_, s.stream);
        mem_used_ += extra;
        s.bytes = grown;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            err = std::string("near-pair list could not be grown: ") + hipGetErrorString(e);
            s.near_cap = 0;
            return BEMC_E_OUT_OF_MEMORY;
        }
        s.near_cap = cap;
        e = launch_reset_near_count(s.d_ctr, s.stream);
        if (e == hipSuccess) e = launch_near_list(s.d_pts, n, env_.el, s.d_near, s.near_cap, s.d_ctr, s.stream);
    }
    const int64_t ne = env_.el.ne;
    const double K = coulomb_constant();
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
    na.order = s.nw.order;
    na.res = s.nw.res;
    na.ctr = s.d_ctr;
    na.near_dr2 = env_.near_dr * env_.near_dr;
    na.max_depth = env_.max_depth;
    na.visit_limit = 1ll << 22;
    if (e == hipSuccess) e = near_order(s.d_near, s.d_ctr, s.near_cap, n, s.d_pts, env_.el, s.nw, s.stream);
    if (e == hipSuccess) e = launch_near(na, kNearEval, s.stream);
    if (e == hipSuccess)
        e = near_reduce(s.nw, n, kNearEval, s.d_phi, s.d_E, nullptr, env_.el.q, ne, 1, K, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out, s.d_phi, (size_t)n * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out + n, s.d_E, (size_t)n * 3 * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_ctr, s.d_ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return BEMC_E_DEVICE;
    }
    s.state = kNear;
    return 0;
}

// Every query of the batch ends with `status`; the batch's buffers are released.
void Server::fail_batch(Slot& s, int status, const std::string& err)
{
    (void)hipStreamSynchronize(s.stream);  // nothing of the batch may still use its buffers
    free_batch(s);
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
    free_batch(s);
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
        // completions and second phases (outside the lock: they copy results and enqueue)
        for (auto& s : slots_) {
            if (s.state == kNear && hipEventQuery(s.done) == hipSuccess) {
                lk.unlock();
                complete(s);
                lk.lock();
                progressed = true;
            } else if (s.state == kFar && hipEventQuery(s.listed) == hipSuccess) {
                lk.unlock();
                std::string err;
                const int rc = near_stage(s, err);
                if (rc < 0) fail_batch(s, rc, err);
                lk.lock();
                progressed |= rc != 1;
            }
        }
        // admissions: each free slot takes the longest prefix of its queue that fits one
        // batch and the memory left
        for (auto& s : slots_) {
            if (s.state != kIdle) continue;
            std::deque<uint64_t>* wq = s.small_only ? &waiting_small_ : (waiting_.empty() ? &waiting_small_ : &waiting_);
            if (wq->empty()) continue;
            int64_t pts = 0;
            size_t k = 0;
            for (; k < wq->size(); ++k) {
                const int64_t qn = queries_[(*wq)[k]].n;
                if (pts + qn > cfg_.max_batch_points) break;
                if (pts + qn > 0 && mem_used_ + batch_bytes(pts + qn, initial_near(pts + qn)) > cfg_.mem_budget_bytes) break;
                pts += qn;
            }
            if (k == 0) continue;  // the first query waits for memory
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
                s.state = kNear;
                if (hipEventRecord(s.done, s.stream) == hipSuccess) continue;
                err = "hipEventRecord";
            } else if (alloc_batch(s, err) && launch_far(s, err)) {
                continue;
            }
            lk.unlock();
            fail_batch(s, err.rfind("batch buffers", 0) == 0 ? BEMC_E_OUT_OF_MEMORY : BEMC_E_DEVICE, err);
            lk.lock();
        }
        bool any_busy = false;
        for (auto& s : slots_) any_busy |= s.state != kIdle;
        if (stopping_ && waiting_.empty() && waiting_small_.empty() && !any_busy) break;
        if (!progressed) cv_.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 2000));
    }
}

}  // namespace bemc
