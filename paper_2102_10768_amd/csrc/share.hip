// Host-core share of the matching tasks (Algorithm 3, Section V-C).
//
// The root candidates of a CST are cut into runs (the first split of
// Algorithm 2: runs of root candidates have disjoint search spaces).  Each
// run's workload is the sum of c_root(v) over its root candidates (the
// workload DP of Section V-C).  Runs are handed out in root order by the rule
// of Algorithm 3: a run goes to the host cores when the host's workload with
// it stays below delta times the workload handed out so far (counting it);
// otherwise it goes to the GPU.  The GPU enumerates its runs with the
// HBM-resident kernel while host threads run a plain backtracking search over
// a host copy of the CST lists for theirs; the count is the sum.
#include <atomic>
#include <chrono>
#include <exception>
#include <thread>

#include "internal.h"

namespace {

// The CST lists in host memory, indexed by position in the matching order.
struct HostCst {
    int k = 0;
    int par[CSTM_MAX_K] = {};
    uint32_t same[CSTM_MAX_K] = {};  // earlier positions with the same label
    std::vector<int32_t> gid[CSTM_MAX_K];
    std::vector<int64_t> toff[CSTM_MAX_K];  // position >= 1: per parent candidate
    std::vector<int32_t> tadj[CSTM_MAX_K];  // candidate indices into this position
    struct Nt {
        int from = 0;
        std::vector<int64_t> off;  // per candidate of position `from`
        std::vector<int32_t> gid;  // data-vertex ids, ascending within each list
    };
    std::vector<Nt> nt[CSTM_MAX_K];  // by later position
};

template <class T>
void fetch(std::vector<T>& dst, const T* src, int64_t n, hipStream_t s) {
    dst.resize((size_t)std::max<int64_t>(n, 0));
    if (n > 0) HIP_TRY(hipMemcpyAsync(dst.data(), src, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s));
}

void copy_to_host(const cstm_cst* c, HostCst& H, hipStream_t s) {
    const CstDev& D = c->host_desc;
    H.k = c->k;
    for (int i = 0; i < c->k; ++i) {
        const int u = c->order[i];
        H.par[i] = D.pos[i].par;
        H.same[i] = D.pos[i].same_mask;
        fetch(H.gid[i], c->cand[u], c->ncand[u], s);
        if (i > 0) {
            const int p = c->parent[u];
            fetch(H.toff[i], c->tree[u].off, c->ncand[p] + 1, s);
            fetch(H.tadj[i], c->tree[u].adj, c->tree[u].entries, s);
        }
    }
    for (const EdgeLists& el : c->nt) {
        HostCst::Nt n;
        n.from = el.from;
        fetch(n.off, el.off, c->ncand[c->order[el.from]] + 1, s);
        fetch(n.gid, el.adj_gid, el.entries, s);
        H.nt[el.to].push_back(std::move(n));
    }
    HIP_TRY(hipStreamSynchronize(s));
}

// Embeddings of the CST whose root is candidate r: depth-first over the
// matching order, extending position d from the tree list of its parent's
// candidate, rejecting a data vertex used by an earlier position of the same
// label or missing from a non-tree list of an earlier neighbour.
uint64_t count_from_root(const HostCst& H, int64_t r, const std::atomic<bool>& stop) {
    const int k = H.k;
    if (k == 1) return 1;
    int32_t x[CSTM_MAX_K], g[CSTM_MAX_K];
    int64_t cur[CSTM_MAX_K], end[CSTM_MAX_K];
    x[0] = (int32_t)r;
    g[0] = H.gid[0][(size_t)r];
    auto open = [&](int d) {
        const int64_t px = x[H.par[d]];
        cur[d] = H.toff[d][(size_t)px];
        end[d] = H.toff[d][(size_t)px + 1];
    };
    uint64_t cnt = 0, steps = 0;
    int d = 1;
    open(1);
    while (d >= 1) {
        if (cur[d] == end[d]) {
            --d;
            continue;
        }
        if ((++steps & 0xFFFFF) == 0 && stop.load(std::memory_order_relaxed)) return cnt;
        const int32_t idx = H.tadj[d][(size_t)cur[d]++];
        const int32_t v = H.gid[d][(size_t)idx];
        bool ok = true;
        for (uint32_t m = H.same[d]; m && ok; m &= m - 1) ok = g[__builtin_ctz(m)] != v;
        for (const HostCst::Nt& n : H.nt[d]) {
            if (!ok) break;
            const int64_t a = n.off[(size_t)x[n.from]], b = n.off[(size_t)x[n.from] + 1];
            ok = std::binary_search(n.gid.begin() + a, n.gid.begin() + b, v);
        }
        if (!ok) continue;
        if (d == k - 1) {
            ++cnt;
            continue;
        }
        x[d] = idx;
        g[d] = v;
        ++d;
        open(d);
    }
    return cnt;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" cstm_status cstm_enumerate_shared(cstm_cst* cst, double delta, int64_t n_runs, int32_t host_threads,
                                             uint64_t* count_out, cstm_share_stats* st_out, void* stream) {
    cstm_share_stats st{};
    uint64_t count = 0;
    cstm_status status = cstm_guard([&] {
        CSTM_REQUIRE(cst && count_out, CSTM_EINVAL, "NULL argument");
        CSTM_REQUIRE(delta >= 0.0 && delta <= 1.0, CSTM_EINVAL, "delta must lie in [0, 1]");
        CSTM_REQUIRE(n_runs >= 0, CSTM_EINVAL, "negative run count");
        CSTM_REQUIRE(host_threads >= 0 && host_threads <= 256, CSTM_EINVAL, "host_threads must lie in [0, 256]");
        HIP_TRY(hipSetDevice(cst->ctx->device));
        hipStream_t s = stream ? (hipStream_t)stream : cst->stream;
        st.delta = delta;
        if (host_threads == 0) host_threads = (int32_t)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        st.host_threads = host_threads;
        if (cst->empty) return;
        cstm_cst_workload_run(cst);
        const std::vector<uint64_t>& w = cst->root_w;
        const int64_t nr = (int64_t)w.size();
        if (nr == 0) return;
        const int64_t runs = std::min<int64_t>(nr, n_runs > 0 ? n_runs : 1024);
        // Algorithm 3 over the runs, in root order.  Weights are exact
        // integers (each c_root saturates at 2^64 - 1); the running sums are
        // 128-bit, and only the comparison with delta times the total is
        // taken in long double (64-bit significand).
        std::vector<int64_t> dev_ranges, host_ranges;
        unsigned __int128 wc = 0, wf = 0;
        for (int64_t i = 0; i < runs; ++i) {
            const int64_t lo = i * nr / runs, hi = (i + 1) * nr / runs;
            unsigned __int128 wr = 0;
            for (int64_t r = lo; r < hi; ++r) wr += w[(size_t)r];
            const bool to_host = (long double)(wc + wr) < (long double)delta * (long double)(wc + wf + wr);
            std::vector<int64_t>& dst = to_host ? host_ranges : dev_ranges;
            if (to_host) {
                wc += wr;
                ++st.groups_host;
            } else {
                wf += wr;
                ++st.groups_device;
            }
            if (!dst.empty() && dst.back() == lo) dst.back() = hi;  // merge with the previous run
            else {
                dst.push_back(lo);
                dst.push_back(hi);
            }
        }
        const unsigned __int128 u64max = ~(uint64_t)0;
        st.w_host = (uint64_t)(wc > u64max ? u64max : wc);
        st.w_device = (uint64_t)(wf > u64max ? u64max : wf);
        const auto t0 = std::chrono::steady_clock::now();
        // the GPU's runs, launched from a thread of their own so that the host
        // search overlaps them
        std::exception_ptr dev_err;
        uint64_t dev_count = 0;
        std::atomic<bool> stop{false};
        std::thread dev([&] {
            try {
                HIP_TRY(hipSetDevice(cst->ctx->device));
                EnumOpts o;
                o.deadline_ms = cst->ctx->tune.deadline_ms;
                o.root_ranges = dev_ranges.data();
                o.n_ranges = (int64_t)dev_ranges.size() / 2;
                cstm_cst* one[1] = {cst};
                cstm_enumerate_run(cst->ctx, 1, one, 0, nullptr, 0, &dev_count, nullptr, o, s);
                st.device_ms = ms_since(t0);
            } catch (...) {
                dev_err = std::current_exception();
                stop.store(true);
            }
        });
        std::exception_ptr host_err;
        std::atomic<uint64_t> host_count{0};
        try {
            if (!host_ranges.empty()) {
                HostCst H;
                hipStream_t cs = nullptr;
                HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                try {
                    copy_to_host(cst, H, cs);
                } catch (...) {
                    (void)hipStreamDestroy(cs);
                    throw;
                }
                HIP_TRY(hipStreamDestroy(cs));
                st.copy_ms = ms_since(t0);
                // work items: at most 16 root candidates each, taken in order
                std::vector<std::pair<int64_t, int64_t>> items;
                for (size_t i = 0; i < host_ranges.size(); i += 2)
                    for (int64_t lo = host_ranges[i]; lo < host_ranges[i + 1]; lo += 16)
                        items.push_back({lo, std::min<int64_t>(lo + 16, host_ranges[i + 1])});
                std::atomic<size_t> next{0};
                std::vector<std::thread> pool;
                auto worker = [&] {
                    uint64_t mine = 0;
                    for (size_t j; !stop.load(std::memory_order_relaxed) && (j = next.fetch_add(1)) < items.size();)
                        for (int64_t r = items[j].first; r < items[j].second; ++r) mine += count_from_root(H, r, stop);
                    host_count.fetch_add(mine);
                };
                try {
                    for (int t = 0; t < host_threads; ++t) pool.emplace_back(worker);
                } catch (...) {
                    stop.store(true);
                    for (auto& th : pool) th.join();
                    throw;
                }
                for (auto& th : pool) th.join();
                st.host_ms = ms_since(t0);
            }
        } catch (...) {
            host_err = std::current_exception();
        }
        dev.join();
        if (dev_err) std::rethrow_exception(dev_err);
        if (host_err) std::rethrow_exception(host_err);
        st.count_host = host_count.load();
        st.count_device = dev_count;
        st.wall_ms = ms_since(t0);
        count = st.count_host + st.count_device;
    });
    if (count_out) *count_out = count;
    if (st_out) *st_out = st;
    return status;
}
