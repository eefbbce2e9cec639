// server.hip -- a request loop over one resident data graph.
//
// Queries arrive one at a time (cstm_server_submit).  The server admits them in
// arrival order while the device-memory bound of their CSTs fits the budget
// (cstm_cst_estimate, doubled for the block cache's power-of-two rounding),
// builds admitted CSTs on builder threads with a stream each, and hands every
// built CST to the next free enumeration lane: a lane takes all CSTs built so
// far (up to max_batch) and counts them in one persistent launch on its own
// stream.  With two or more lanes a new batch starts while a long one is still
// running, so requests that arrive while others are on the GPU overlap with
// them.  Each request's count is available as soon as its batch ends; its CST
// is then freed and its charge returned to admission.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    int32_t k = 0;
    int32_t qlabel[CSTM_MAX_K] = {};
    std::vector<int32_t> qedges;
    uint64_t limit = 0;
    uint64_t charge = 0;
    cstm_cst* cst = nullptr;
    bool built = false, done = false;
    cstm_request_result res{};
};

}  // namespace

struct cstm_server {
    cstm_ctx* ctx = nullptr;
    const cstm_graph* g = nullptr;
    uint64_t budget = 0;
    int max_batch = 256;
    int64_t batch_wait_us = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request*> pending;  // submitted, not admitted
    std::deque<Request*> ready;    // built, not launched
    uint64_t next_id = 1;
    uint64_t in_use = 0;
    int unbuilt = 0;               // admitted requests still being built
    int busy_lanes = 0;
    bool closing = false;
    cstm_server_stats st{};
    std::vector<hipStream_t> streams;
    std::vector<std::thread> threads;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void finish(Request* r, cstm_status status, uint64_t count) {
        if (r->cst) {
            cstm_cst_free(r->cst);
            r->cst = nullptr;
        }
        std::lock_guard<std::mutex> lk(mu);
        r->res.done = 1;
        r->res.status = status;
        r->res.count = status == CSTM_OK ? count : 0;
        r->res.done_s = now();
        in_use -= r->charge;
        r->charge = 0;
        r->done = true;
        if (status == CSTM_OK) st.completed++;
        else st.failed++;
        cv.notify_all();
    }

    void build_loop(hipStream_t s) {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            Request* r = nullptr;
            cstm_status refuse = CSTM_OK;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    cv.wait(lk, [&] { return !pending.empty() || closing; });
                    if (pending.empty()) {
                        cv.notify_all();
                        return;
                    }
                    r = pending.front();
                    if (r->charge == 0) {
                        uint64_t est = 0;
                        cstm_status e = cstm_cst_estimate(g, r->k, r->qlabel, (int32_t)(r->qedges.size() / 2),
                                                          r->qedges.data(), &est);
                        if (e != CSTM_OK) refuse = e;
                        else r->charge = 2 * est + 1;
                    }
                    if (refuse == CSTM_OK && r->charge > budget) refuse = CSTM_ENOMEM;
                    if (refuse != CSTM_OK) {
                        pending.pop_front();
                        r->charge = 0;
                        break;
                    }
                    // admission in arrival order: the head request waits until it fits
                    if (in_use + r->charge <= budget) {
                        pending.pop_front();
                        in_use += r->charge;
                        if (in_use > st.peak_bytes) st.peak_bytes = in_use;
                        unbuilt++;
                        r->res.admit_s = now();
                        break;
                    }
                    cv.wait(lk);
                }
            }
            if (refuse != CSTM_OK) {
                finish(r, refuse, 0);
                continue;
            }
            cstm_cst* c = nullptr;
            cstm_status e = cstm_cst_build(ctx, g, r->k, r->qlabel, (int32_t)(r->qedges.size() / 2),
                                           r->qedges.data(), s, &c);
            if (e != CSTM_OK) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    unbuilt--;
                }
                finish(r, e, 0);
                continue;
            }
            std::lock_guard<std::mutex> lk(mu);
            unbuilt--;
            r->cst = c;
            r->built = true;
            r->res.built_s = now();
            // the build's temporaries are back in the pool: from here on the
            // request holds only its CST's arena (doubled for the block
            // cache's rounding)
            const uint64_t kept = 2 * (std::max(c->bytes, c->mem_bytes) + sizeof(CstDev) + 65536) + 1;
            if (kept < r->charge) {
                in_use -= r->charge - kept;
                r->charge = kept;
            }
            ready.push_back(r);
            cv.notify_all();
        }
    }

    void lane_loop(int lane, hipStream_t s) {
        (void)hipSetDevice(ctx->device);
        std::vector<Request*> batch;
        std::vector<cstm_cst*> csts;
        std::vector<uint64_t> counts, limits;
        bool builds_in_flight = false;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return !ready.empty() || (closing && pending.empty() && unbuilt == 0); });
                if (ready.empty()) {
                    cv.notify_all();
                    return;
                }
                // Under load (another lane already running) a short wait lets more
                // built CSTs join this launch; an idle server launches at once.
                if (batch_wait_us > 0 && busy_lanes > 0 && (int)ready.size() < max_batch &&
                    (!pending.empty() || unbuilt > 0)) {
                    const auto until = Clock::now() + std::chrono::microseconds(batch_wait_us);
                    cv.wait_until(lk, until, [&] { return (int)ready.size() >= max_batch || busy_lanes == 0; });
                    if (ready.empty()) continue;  // another lane took them meanwhile
                }
                batch.clear();
                while (!ready.empty() && (int)batch.size() < max_batch) {
                    batch.push_back(ready.front());
                    ready.pop_front();
                }
                // builds still to come share the CUs with this launch
                builds_in_flight = !pending.empty() || unbuilt > 0;
                busy_lanes++;
                if (busy_lanes > st.max_overlap) st.max_overlap = busy_lanes;
                st.launches++;
                st.batched += batch.size();
            }
            const double t_launch = now();
            csts.clear();
            limits.clear();
            bool any_limit = false;
            for (Request* r : batch) {
                csts.push_back(r->cst);
                limits.push_back(r->limit);
                any_limit |= r->limit != 0;
                r->res.batch_size = (int32_t)batch.size();
                r->res.lane = lane;
                r->res.launch_s = t_launch;
            }
            counts.assign(batch.size(), 0);
            cstm_enum_stats es{};
            cstm_status e = cstm_guard([&] {
                EnumOpts o;
                o.limits = any_limit ? limits.data() : nullptr;
                o.deadline_ms = ctx->tune.deadline_ms;
                o.force_hbm = true;  // admission charged the CSTs, not partition images
                if (builds_in_flight) o.wgs_per_cu = ctx->tune.serve_wgs_per_cu;
                cstm_enumerate_run(ctx, (int)csts.size(), csts.data(), 0, nullptr, 0, counts.data(), nullptr, o, s, &es);
            });
            {
                std::lock_guard<std::mutex> lk(mu);
                busy_lanes--;
                if (e == CSTM_OK) {
                    st.kernel_ms += es.kernel_ms;
                    st.extensions += es.extensions;
                    st.edge_checks += es.edge_checks;
                    st.pushed += es.pushed;
                    st.summed += es.summed;
                    st.chunks += es.chunks;
                }
            }
            for (size_t i = 0; i < batch.size(); ++i) finish(batch[i], e, counts[i]);
        }
    }
};

extern "C" cstm_status cstm_server_create(cstm_ctx* ctx, const cstm_graph* g, uint64_t mem_budget, int32_t lanes,
                                          int32_t builders, int32_t max_batch, int32_t batch_wait_us,
                                          cstm_server** out) {
    cstm_server* srv = nullptr;
    cstm_status st = cstm_guard([&] {
        CSTM_REQUIRE(ctx && g && out, CSTM_EINVAL, "NULL argument");
        *out = nullptr;
        CSTM_REQUIRE(g->ctx == ctx, CSTM_EINVAL, "graph belongs to another context");
        if (lanes <= 0) lanes = 2;
        if (builders <= 0) builders = 2;
        if (max_batch <= 0) max_batch = 256;
        CSTM_REQUIRE(lanes <= 16 && builders <= 64, CSTM_EINVAL, "at most 16 lanes and 64 builders");
        CSTM_REQUIRE(mem_budget > 0, CSTM_EINVAL, "memory budget must be positive");
        // every lane's launch borrows a task-ring workspace: charged once, up front
        const uint64_t rings = (uint64_t)lanes * (uint64_t)cstm_hbm_workspace_bytes(max_batch);
        CSTM_REQUIRE(mem_budget > rings, CSTM_ENOMEM,
                     "memory budget does not cover the lanes' task rings (" + std::to_string(rings) + " bytes)");
        HIP_TRY(hipSetDevice(ctx->device));
        srv = new cstm_server();
        srv->ctx = ctx;
        srv->g = g;
        srv->budget = mem_budget - rings;
        srv->max_batch = max_batch;
        srv->batch_wait_us = batch_wait_us < 0 ? 0 : batch_wait_us;
        srv->t0 = Clock::now();
        for (int i = 0; i < builders + lanes; ++i) {
            hipStream_t s = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));  // default priority
            srv->streams.push_back(s);
        }
        for (int i = 0; i < builders; ++i) srv->threads.emplace_back([srv, i] { srv->build_loop(srv->streams[i]); });
        for (int i = 0; i < lanes; ++i)
            srv->threads.emplace_back([srv, i, builders] { srv->lane_loop(i, srv->streams[builders + i]); });
        *out = srv;
    });
    if (st != CSTM_OK && srv) {
        cstm_server_destroy(srv);
    }
    return st;
}

extern "C" cstm_status cstm_server_submit(cstm_server* srv, int32_t k, const int32_t* qlabel, int32_t m_q,
                                          const int32_t* qedges, uint64_t limit, uint64_t* ticket) {
    return cstm_guard([&] {
        CSTM_REQUIRE(srv && ticket, CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(k >= 1 && k <= CSTM_MAX_K && qlabel, CSTM_EINVAL, "query size k must be in 1..32");
        CSTM_REQUIRE(m_q >= 0 && m_q <= CSTM_MAX_K * (CSTM_MAX_K - 1) / 2 && (m_q == 0 || qedges), CSTM_EINVAL,
                     "bad query edge array");
        auto r = std::make_unique<Request>();
        r->k = k;
        for (int u = 0; u < k; ++u) r->qlabel[u] = qlabel[u];
        r->qedges.assign(qedges, qedges + 2 * (size_t)m_q);
        r->limit = limit;
        std::lock_guard<std::mutex> lk(srv->mu);
        CSTM_REQUIRE(!srv->closing, CSTM_EINVAL, "server is shutting down");
        r->id = srv->next_id++;
        r->res.submit_s = srv->now();
        r->res.status = CSTM_OK;
        *ticket = r->id;
        srv->pending.push_back(r.get());
        srv->reqs.emplace(r->id, std::move(r));
        srv->st.submitted++;
        srv->cv.notify_all();
    });
}

static cstm_status take_result(cstm_server* srv, uint64_t ticket, double timeout_s, bool block,
                               cstm_request_result* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(srv && out, CSTM_EINVAL, "NULL argument");
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        CSTM_REQUIRE(it != srv->reqs.end(), CSTM_EINVAL, "unknown ticket (never issued, or its result was taken)");
        Request* r = it->second.get();
        if (block && !r->done) {
            auto pred = [&] { return r->done; };
            if (timeout_s > 0) srv->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
            else srv->cv.wait(lk, pred);
        }
        *out = r->res;
        out->done = r->done ? 1 : 0;
        if (r->done) srv->reqs.erase(it);  // a finished result is handed out once
    });
}

extern "C" cstm_status cstm_server_poll(cstm_server* srv, uint64_t ticket, cstm_request_result* out) {
    return take_result(srv, ticket, 0.0, false, out);
}

extern "C" cstm_status cstm_server_wait(cstm_server* srv, uint64_t ticket, double timeout_s,
                                        cstm_request_result* out) {
    return take_result(srv, ticket, timeout_s, true, out);
}

extern "C" cstm_status cstm_server_get_stats(cstm_server* srv, cstm_server_stats* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(srv && out, CSTM_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        *out = srv->st;
        out->in_use_bytes = srv->in_use;
        out->admission_bytes = srv->budget;
    });
}

extern "C" void cstm_server_destroy(cstm_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->closing = true;
        srv->cv.notify_all();
    }
    for (auto& t : srv->threads) t.join();
    for (auto& kv : srv->reqs)
        if (kv.second->cst) cstm_cst_free(kv.second->cst);
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    delete srv;
}
