// context.hip -- context, device memory and error reporting.
#include <cstring>

#include "internal.h"

static thread_local std::string g_last_error;

void cstm_set_error(const std::string& msg) { g_last_error = msg; }

extern "C" const char* cstm_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* cstm_version(void) { return "cstm 0.1 gfx950"; }

// ---------------------------------------------------------------- device memory

// Device blocks up to 256 MB come from power-of-two size classes and go back
// to a per-context cache when freed, so repeated CST builds do not pay for
// hipMalloc/hipFree (hipFree also waits for the whole device).  Callers free a
// block only after the work that used it has completed on its stream.
static constexpr int kMaxPooledClass = 28;  // 256 MB

void* cstm_ctx::dmalloc(size_t bytes) {
    void* p = nullptr;
    if (alloc) {
        p = alloc(bytes, user);
        if (!p) throw CstmError{CSTM_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
        return p;
    }
    std::lock_guard<std::mutex> lk(pool_mu);
    int cls = 8;
    while (cls <= kMaxPooledClass && (size_t(1) << cls) < bytes) ++cls;
    if (cls <= kMaxPooledClass) {
        if (pool.size() <= (size_t)cls) pool.resize(cls + 1);
        if (!pool[cls].empty()) {
            p = pool[cls].back();
            pool[cls].pop_back();
            return p;
        }
        bytes = size_t(1) << cls;
    } else {
        cls = -1;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        release_pool();  // give cached blocks back and try once more
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw CstmError{CSTM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
        }
    }
    block_class[p] = cls;
    return p;
}

void cstm_ctx::dfree(void* p) {
    if (!p) return;
    if (free_fn) {
        free_fn(p, user);
        return;
    }
    std::lock_guard<std::mutex> lk(pool_mu);
    auto it = block_class.find(p);
    if (it != block_class.end() && it->second >= 0) {
        pool[it->second].push_back(p);
        return;
    }
    if (it != block_class.end()) block_class.erase(it);
    (void)hipFree(p);
}

void cstm_ctx::release_pool() {
    for (auto& bin : pool) {
        for (void* p : bin) {
            block_class.erase(p);
            (void)hipFree(p);
        }
        bin.clear();
    }
}

void* cstm_ctx::ws_acquire(size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(ws_mu);
        size_t best = ws_free.size();
        for (size_t i = 0; i < ws_free.size(); ++i)
            if (ws_free[i].second >= bytes && (best == ws_free.size() || ws_free[i].second < ws_free[best].second))
                best = i;
        if (best < ws_free.size()) {
            void* p = ws_free[best].first;
            ws_free.erase(ws_free.begin() + (long)best);
            return p;
        }
    }
    size_t want = bytes + bytes / 4;
    void* p = dmalloc(want);
    std::lock_guard<std::mutex> lk(ws_mu);
    ws_all.push_back(p);
    ws_sizes[p] = want;
    return p;
}

void cstm_ctx::ws_release(void* p) {
    std::lock_guard<std::mutex> lk(ws_mu);
    ws_free.push_back({p, ws_sizes[p]});
}

void DevArena::release(void* p) {
    for (size_t i = 0; i < blocks.size(); ++i) {
        if (blocks[i] == p) {
            ctx->dfree(p);
            blocks[i] = blocks.back();
            blocks.pop_back();
            sizes[i] = sizes.back();
            sizes.pop_back();
            return;
        }
    }
}

void DevArena::clear() {
    if (!ctx) return;
    for (void* p : blocks) ctx->dfree(p);
    blocks.clear();
    sizes.clear();
}

// ---------------------------------------------------------------- context API

static void apply_defaults(cstm_ctx* c) {
    cstm_tune& t = c->tune;
    if (t.waves_per_wg <= 0) t.waves_per_wg = 4;
    if (t.waves_per_wg > 16) t.waves_per_wg = 16;
    if (t.wgs_per_cu <= 0) t.wgs_per_cu = 4;
    int64_t state = 256 + (int64_t)t.waves_per_wg * 64;
    int64_t max_budget = (c->lds_per_wg - state) & ~int64_t(15);
    if (t.part_budget_bytes == 0) {
        // share the LDS of one CU between wgs_per_cu workgroups
        int64_t per = (int64_t)(160 * 1024) / t.wgs_per_cu - state;
        if (per > max_budget) per = max_budget;
        t.part_budget_bytes = (uint64_t)(per & ~int64_t(15));
    }
    if ((int64_t)t.part_budget_bytes > max_budget) t.part_budget_bytes = (uint64_t)max_budget;
    if (t.max_list_len < 0) t.max_list_len = 0;
    if (t.max_replication == 0) t.max_replication = 16;  // negative: no limit
    if (t.enum_mode < CSTM_MODE_AUTO || t.enum_mode > CSTM_MODE_HBM) t.enum_mode = CSTM_MODE_AUTO;
    if (t.deadline_ms < 0) t.deadline_ms = 0;
    if (t.hbm_wgs_per_cu <= 0) t.hbm_wgs_per_cu = 2;
    if (t.hbm_donate_period == 0) t.hbm_donate_period = 64;
    if (t.hbm_flat_max == 0) t.hbm_flat_max = 2048;
    if (t.hbm_donate_last_min <= 0) t.hbm_donate_last_min = 4096;
    if (t.last_level_sum == 0) t.last_level_sum = 1;
    if (t.hbm_donate_min <= 0) t.hbm_donate_min = 16;
    if (t.hbm_idle_ms <= 0) t.hbm_idle_ms = 30000;
    if (t.order_rule < 0 || t.order_rule > 1) t.order_rule = 0;
    if (t.serve_wgs_per_cu <= 0) t.serve_wgs_per_cu = 2;
}

extern "C" cstm_status cstm_ctx_create(int device, cstm_alloc_fn alloc, cstm_free_fn free_fn, void* user,
                                       const cstm_tune* tune, cstm_ctx** out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(out, CSTM_EINVAL, "out is NULL");
        *out = nullptr;
        CSTM_REQUIRE((alloc == nullptr) == (free_fn == nullptr), CSTM_EINVAL, "alloc and free must be given together");
        int ndev = 0;
        HIP_TRY(hipGetDeviceCount(&ndev));
        CSTM_REQUIRE(device >= 0 && device < ndev, CSTM_EINVAL, "device index out of range");
        HIP_TRY(hipSetDevice(device));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, device));
        CSTM_REQUIRE(prop.warpSize == CSTM_WAVE, CSTM_EDEVICE, "expected 64-wide wavefronts");
        cstm_ctx* c = new cstm_ctx();
        c->device = device;
        c->alloc = alloc;
        c->free_fn = free_fn;
        c->user = user;
        c->num_cus = prop.multiProcessorCount;
        c->lds_per_wg = (int64_t)prop.sharedMemPerBlock;
        if (tune) c->tune = *tune;
        apply_defaults(c);
        try {
            cstm_noalloc_init(device);  // this device's address of the no-allocation scratch array
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

extern "C" void cstm_ctx_destroy(cstm_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (void* p : ctx->ws_all) ctx->dfree(p);
    {
        std::lock_guard<std::mutex> lk(ctx->pool_mu);
        ctx->release_pool();
    }
    delete ctx;
}

extern "C" cstm_status cstm_ctx_get_tune(const cstm_ctx* ctx, cstm_tune* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(ctx && out, CSTM_EINVAL, "NULL argument");
        *out = ctx->tune;
    });
}

extern "C" cstm_status cstm_ctx_set_tune(cstm_ctx* ctx, const cstm_tune* tune) {
    return cstm_guard([&] {
        CSTM_REQUIRE(ctx && tune, CSTM_EINVAL, "NULL argument");
        ctx->tune = *tune;
        apply_defaults(ctx);
    });
}

extern "C" cstm_status cstm_ctx_lds_bytes(const cstm_ctx* ctx, int64_t* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(ctx && out, CSTM_EINVAL, "NULL argument");
        *out = ctx->lds_per_wg;
    });
}

extern "C" cstm_status cstm_ctx_last_enum_stats(const cstm_ctx* ctx, cstm_enum_stats* out) {
    return cstm_guard([&] {
        CSTM_REQUIRE(ctx && out, CSTM_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(const_cast<cstm_ctx*>(ctx)->ws_mu);
        *out = ctx->last_enum;
    });
}
