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
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        double *d_pts = nullptr, *d_phi = nullptr, *d_E = nullptr, *d_partial = nullptr;
        double *h_pts = nullptr, *h_out = nullptr;  // pinned staging: [3][M] in, [4][M] out
        NearPair* d_near = nullptr;
        unsigned long long near_cap = 0;
        NearWork nw{};  // per-point segments and per-pair results (near_cap pairs, 4 rows)
        DevCounters *d_ctr = nullptr, *h_ctr = nullptr;
        bool busy = false;
        bool small_only = false;  // serves the short-query class only
        int64_t batch_id = -1;
        int64_t n = 0;
        std::vector<uint64_t> queries;
    };

    Server() = default;
    bool init(const ServerEnv& env, const bemc_server_config& cfg, std::string& err);
    void loop();
    bool launch(Slot& s, std::string& err);
    void complete(Slot& s);
    double now() const;

    ServerEnv env_{};
    bemc_server_config cfg_{};
    int max_split_ = 64;
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
