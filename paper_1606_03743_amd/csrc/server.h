// Continuous-batching query server (host scheduler thread + HIP streams).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bemc.h"
#include "bemc_internal.h"

namespace bemc {

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
    enum SlotState { kIdle = 0, kFar = 1, kNear = 2 };
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t listed = nullptr;  // the near-pair list pass's count has reached h_list
        hipEvent_t done = nullptr;
        int state = kIdle;  // kFar: far field enqueued, near-pair count pending; kNear: near field enqueued
        // buffers of the batch in flight: stream-ordered allocations, released at completion
        double *d_pts = nullptr, *d_phi = nullptr, *d_E = nullptr, *d_partial = nullptr;
        NearPair* d_near = nullptr;
        unsigned long long near_cap = 0;
        NearWork nw{};  // per-point segments and per-pair results (near_cap pairs, 4 rows)
        size_t bytes = 0;  // device bytes accounted to the batch
        DevCounters* d_ctr = nullptr;                 // kept for the server's lifetime
        double *h_pts = nullptr, *h_out = nullptr;    // pinned staging: [3][M] in, [4][M] out
        DevCounters *h_ctr = nullptr, *h_list = nullptr;
        bool small_only = false;  // serves the short-query class only
        int64_t batch_id = -1;
        int64_t n = 0;
        int n_split = 1;
        std::vector<uint64_t> queries;
    };

    Server() = default;
    bool init(const ServerEnv& env, const bemc_server_config& cfg, std::string& err);
    void loop();
    int split_for(int64_t n) const;                  // element chunks of a batch of n points
    size_t batch_bytes(int64_t n, unsigned long long near_pairs) const;
    unsigned long long initial_near(int64_t n) const;  // near-pair list of a new batch
    bool alloc_batch(Slot& s, std::string& err);     // stream-ordered, on the slot's stream
    void free_batch(Slot& s);                        // stream-ordered
    bool launch_far(Slot& s, std::string& err);      // copy-in, list pass, far field
    int near_stage(Slot& s, std::string& err);       // 0 enqueued, 1 deferred (memory), < 0 error
    void complete(Slot& s);
    void fail_batch(Slot& s, int status, const std::string& err);
    double now() const;

    ServerEnv env_{};
    bemc_server_config cfg_{};
    int max_split_ = 64;
    size_t mem_used_ = 0;  // device bytes of the batches in flight (scheduler thread only)
    hipMemPool_t pool_ = nullptr;  // the batches' buffers (stream-ordered allocations)
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
