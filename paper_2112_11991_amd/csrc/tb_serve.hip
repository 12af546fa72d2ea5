// tb_serve.hip -- the continuous-batching request loop (host code only).
//
// Requests (a resident series and a chunk of templates, Sec. 5's per-DM-trial
// x template work) arrive over time.  The loop is a client of the plan's own
// calls: tb_search_templates admits a request and spreads its waves over the
// plan's lanes, tb_poll sees it finish, tb_get_candidates copies its records
// and tb_release hands its buffers back to the plan's pools.  It computes no
// part of the search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <deque>
#include <numeric>
#include <thread>
#include <vector>

#include "tb_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Running {
    uint32_t idx;  // position in the caller's request array
    int64_t rid;
};

double seconds_since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

}  // namespace

extern "C" tb_status tb_serve(tb_plan_t plan, const tb_serve_request* req, uint32_t count, double time_scale,
                              uint32_t flags, tb_candidate* out, uint64_t capacity, tb_serve_result* res,
                              uint32_t stats[2])
{
    if (!plan || (count && (!req || !res)) || (capacity && !out) || !(time_scale > 0.0) ||
        !std::isfinite(time_scale) || (flags & ~(uint32_t)TB_SERVE_SATURATE))
        return TB_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < count; ++i)
        if (!std::isfinite(req[i].t_arrival_s) || req[i].t_arrival_s < 0.0 || (req[i].count && !req[i].templates))
            return TB_ERR_INVALID_ARG;
    const bool saturate = flags & TB_SERVE_SATURATE;
    const uint64_t ring = tb::plan_ring_capacity(plan);

    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return req[a].t_arrival_s < req[b].t_arrival_s; });
    for (uint32_t i = 0; i < count; ++i) res[i] = tb_serve_result{-1.0, -1.0, 0, 0, 0, TB_ERR_NOT_READY, 0};

    std::deque<uint32_t> waiting;
    std::vector<Running> running;
    uint32_t next = 0, max_in_flight = 0, budget_waits = 0;
    uint64_t used = 0;
    tb_status failure = TB_OK;
    const auto t0 = Clock::now();
    auto due = [&](uint32_t i) { return saturate ? 0.0 : req[i].t_arrival_s * time_scale; };

    // Copies a finished request's records and releases it.
    auto finish = [&](const Running& r) -> tb_status {
        tb_serve_result& o = res[r.idx];
        o.t_done_s = seconds_since(t0);
        uint64_t total = 0;
        const uint64_t room = capacity - used;
        tb_status st = tb_get_candidates(plan, r.rid, room ? out + used : nullptr, room, &total, 1);
        if (st != TB_OK && st != TB_ERR_OVERFLOW) {
            tb_release(plan, r.rid);
            return st;
        }
        const uint64_t kept = st == TB_ERR_OVERFLOW ? std::min(total, ring) : total;
        o.cand_offset = used;
        o.n_copied = std::min(kept, room);
        o.n_total = total;
        o.status = (st == TB_ERR_OVERFLOW || o.n_copied < total) ? TB_ERR_OVERFLOW : TB_OK;
        used += o.n_copied;
        return tb_release(plan, r.rid);
    };

    while (failure == TB_OK && (next < count || !waiting.empty() || !running.empty())) {
        const double now = seconds_since(t0);
        while (next < count && due(order[next]) <= now) waiting.push_back(order[next++]);

        // admission in arrival order while the budget allows
        while (!waiting.empty()) {
            const uint32_t i = waiting.front();
            int64_t rid = -1;
            tb_status st = tb_search_templates(plan, req[i].series_id, req[i].templates, req[i].count,
                                               req[i].first_template_id, &rid);
            if (st == TB_ERR_BUDGET && !running.empty()) {
                ++budget_waits;
                break;
            }
            if (st != TB_OK) {
                res[i].status = st;
                failure = st;
                break;
            }
            res[i].t_admit_s = seconds_since(t0);
            running.push_back(Running{i, rid});
            waiting.pop_front();
        }
        max_in_flight = std::max<uint32_t>(max_in_flight, (uint32_t)running.size());
        if (failure != TB_OK) break;

        bool progressed = false;
        for (size_t k = 0; k < running.size();) {
            tb_status st = tb_poll(plan, running[k].rid);
            if (st == TB_ERR_NOT_READY) {
                ++k;
                continue;
            }
            const Running r = running[k];
            running.erase(running.begin() + (ptrdiff_t)k);
            st = st == TB_OK ? finish(r) : (tb_release(plan, r.rid), st);
            if (st != TB_OK) {
                res[r.idx].status = st;
                failure = st;
                break;
            }
            progressed = true;
        }
        if (failure != TB_OK || progressed) continue;
        if (running.empty() && waiting.empty() && next < count) {
            // idle until the next arrival: sleep most of the gap, then spin
            const double gap = due(order[next]) - seconds_since(t0);
            if (gap > 2e-3) std::this_thread::sleep_for(std::chrono::duration<double>(gap - 1e-3));
        } else {
            std::this_thread::yield();
        }
    }
    // on failure: wait for and release whatever is still in flight
    for (const Running& r : running) tb_release(plan, r.rid);
    if (stats) {
        stats[0] = max_in_flight;
        stats[1] = budget_waits;
    }
    return failure;
}
