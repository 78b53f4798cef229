// Continuous-batching query server (host scheduler thread + HIP streams).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bemc.h"
#include "bemc_internal.h"

namespace bemc {

// Device memory of the batches in flight: one allocation made when the server starts,
// handed out and taken back by a first-fit list of free blocks on the host (scheduler thread
// only; 256-byte granules).  No HIP allocation call is made per batch.
class Arena {
public:
    static constexpr size_t kNone = ~size_t(0);
    hipError_t init(size_t bytes);
    void destroy();
    size_t take(size_t bytes);              // offset of a block, or kNone
    void give(size_t off, size_t bytes);    // bytes as passed to take
    char* base() const { return base_; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }

private:
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, coalesced
};

struct ServerEnv {
    int device;
    Elements el;
    RuleTables rules;
    double near_dr;
    int max_depth;
    int64_t n_tri, n_rect;
    int dr_rules;   // rule choice by distance ratio (queries are particle tracks: already coherent)
    LevelRules lv;
};

class Server {
public:
    static Server* create(const ServerEnv& env, const bemc_server_config& cfg, std::string& err);
    ~Server();
    int submit(const double* pts, int64_t n, double* phi, double* E, uint64_t* ticket, std::string& err);
    bool poll(uint64_t ticket, bemc_query_info* info);
    int wait(uint64_t ticket, double timeout_s, bemc_query_info* info);  // 0 ok, 1 unknown, 2 timeout
    void stop();
    std::string last_error();

private:
    struct Query {
        uint64_t id;
        const double* pts;
        int64_t n;
        double* phi;
        double* E;
        bool small;
        bemc_query_info info;
    };
    enum SlotState { kIdle = 0, kRun = 1, kGrow = 2 };
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        int state = kIdle;  // kRun: enqueued up to the completion event; kGrow: its near-pair
                            // list overflowed and waits for memory to grow
        // arena blocks of the batch: per-point buffers and the per-pair near buffers
        size_t fix_off = Arena::kNone, fix_bytes = 0, pair_off = Arena::kNone, pair_bytes = 0;
        char* spill = nullptr;  // a grown list's block outside the arena (nothing could give
                                // memory back): stream-ordered allocation, released with the batch
        double *d_pts = nullptr;   // [3][n]
        double *d_far = nullptr;   // [4][n] far field (phi, E) of a one-chunk batch (else the
                                   // partial sums hold it); kept for a repeated near stage
        double *d_out = nullptr;   // [4][n] far + near
        double *d_partial = nullptr;
        NearPair* d_near = nullptr;
        unsigned long long near_cap = 0;
        NearWork nw{};  // per-point segments and per-pair results (near_cap pairs, 4 rows)
        DevCounters* d_ctr = nullptr;                 // kept for the server's lifetime
        double *h_pts = nullptr, *h_out = nullptr;    // pinned staging: [3][M] in, [4][M] out
        DevCounters* h_ctr = nullptr;
        bool small_only = false;  // serves the short-query class only
        int64_t batch_id = -1;
        int64_t n = 0;
        int n_split = 1;
        std::vector<uint64_t> queries;
    };

    Server() = default;
    bool init(const ServerEnv& env, const bemc_server_config& cfg, std::string& err);
    void loop();
    int split_for(int64_t n) const;                     // element chunks of a batch of n points
    size_t fix_bytes(int64_t n) const;                  // per-point buffers of a batch
    static size_t pair_bytes(int64_t n, unsigned long long pairs);  // near list and its buffers
    // near-pair list of a new batch (base: the first estimate, 16 pairs per point)
    unsigned long long initial_near(int64_t n, bool base = false) const;
    void carve_fix(Slot& s);
    void carve_pairs(Slot& s, char* base);
    void release(Slot& s);                              // the batch's arena blocks
    bool launch(Slot& s, std::string& err);             // the whole batch, at admission
    bool near_stage(Slot& s, std::string& err);         // (again) after a list growth
    int grow(Slot& s, std::string& err);                // 0 enqueued, 1 waits for memory, < 0 error
    void complete(Slot& s);
    void fail_batch(Slot& s, int status, const std::string& err);
    double now() const;

    ServerEnv env_{};
    bemc_server_config cfg_{};
    int max_split_ = 64;
    Arena arena_;  // device memory of the batches in flight (scheduler thread only)
    double pairs_per_point_ = 16.0;  // near-pair list of a new batch per point: 1.25 x the
                                     // density seen (up at once, down slowly; scheduler thread)
    std::vector<Slot> slots_;
    std::mutex mu_;
    std::condition_variable cv_;       // scheduler wake-up
    std::condition_variable done_cv_;  // query completion
    std::deque<uint64_t> waiting_;        // long queries (all queries with one class)
    std::deque<uint64_t> waiting_small_;  // short queries (small_query_points > 0)
    std::unordered_map<uint64_t, Query> queries_;
    uint64_t next_id_ = 1;
    int64_t next_batch_ = 0;
    bool stopping_ = false;
    std::thread thread_;
    std::string err_;
    double t0_ = 0.0;
};

}  // namespace bemc
