// Batched independent PFC instances (C ABI in include/pfc_batch.h): one solver context and
// one HIP stream per instance, and a pool of host threads that hands the instances out,
// largest first, for each time step.  Host code only; the device work is the solver's.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pfc_batch.h"
#include "pfc_internal.h"

struct pfc_batch {
    std::vector<pfc_ctx*> ctx;
    std::vector<hipStream_t> streams;
    std::vector<int> order;              // instance indices, largest grid first
    std::vector<std::thread> pool;
    int device = 0;

    std::mutex m;
    std::condition_variable cv_work, cv_done;
    long generation = 0;                 // one per pfc_batch_step call
    int busy = 0;                        // workers still running the current step
    bool quit = false;
    std::atomic<int> next{0};            // next position in `order` to hand out

    // arguments of the current step
    double* const* phis = nullptr;
    pfc_step_stats* st = nullptr;
    pfc_status* status = nullptr;

    std::string err;
};

namespace {

void worker(pfc_batch* b) {
    (void)hipSetDevice(b->device);
    long seen = 0;
    const int n = (int)b->ctx.size();
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(b->m);
            b->cv_work.wait(lk, [&] { return b->quit || b->generation != seen; });
            if (b->quit) return;
            seen = b->generation;
        }
        for (;;) {
            const int k = b->next.fetch_add(1);
            if (k >= n) break;
            const int i = b->order[k];
            b->status[i] = pfc_step(b->ctx[i], b->phis[i], &b->st[i]);
        }
        std::lock_guard<std::mutex> lk(b->m);
        if (--b->busy == 0) b->cv_done.notify_one();
    }
}

void teardown(pfc_batch* b) {
    {
        std::lock_guard<std::mutex> lk(b->m);
        b->quit = true;
    }
    b->cv_work.notify_all();
    for (std::thread& t : b->pool)
        if (t.joinable()) t.join();
    for (pfc_ctx* c : b->ctx)
        if (c) pfc_destroy(c);
    for (hipStream_t s : b->streams)
        if (s) (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

pfc_status pfc_batch_create(int count, const pfc_grid* grids, const pfc_model* models, const pfc_opts* opts,
                            int workers, pfc_batch** out) {
    if (!out) return PFC_EINVAL;
    *out = nullptr;
    if (count < 1 || !grids || !models || !opts || workers < 1 || workers > 64) return PFC_EINVAL;
    pfc_batch* b = new pfc_batch();
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return PFC_EHIP;
    }
    b->ctx.assign(count, nullptr);
    b->streams.assign(count, nullptr);
    pfc_status s = PFC_OK;
    for (int i = 0; i < count && s == PFC_OK; ++i) {
        if (hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) != hipSuccess) {
            s = PFC_EHIP;
            break;
        }
        s = pfc_create(&grids[i], &models[i], &opts[i], b->streams[i], &b->ctx[i]);
    }
    if (s != PFC_OK) {
        teardown(b);
        delete b;
        return s;
    }
    b->order.resize(count);
    for (int i = 0; i < count; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        const auto cells = [&](int i) { return (long)grids[i].n[0] * grids[i].n[1] * (grids[i].dim == 3 ? grids[i].n[2] : 1); };
        return cells(x) > cells(y);
    });
    const int nw = std::min(workers, count);
    for (int w = 0; w < nw; ++w) b->pool.emplace_back(worker, b);
    *out = b;
    return PFC_OK;
}

void pfc_batch_destroy(pfc_batch* b) {
    if (!b) return;
    teardown(b);
    delete b;
}

const char* pfc_batch_last_error(const pfc_batch* b) { return b ? b->err.c_str() : "null batch"; }

pfc_status pfc_batch_step(pfc_batch* b, double* const* phis, pfc_step_stats* st, pfc_status* status) {
    if (!b) return PFC_EINVAL;
    const int n = (int)b->ctx.size();
    if (!phis || !st || !status) {
        b->err = "bad argument";
        return PFC_EINVAL;
    }
    for (int i = 0; i < n; ++i)
        if (!phis[i]) {
            b->err = "null field for instance " + std::to_string(i);
            return PFC_EINVAL;
        }
    {
        std::lock_guard<std::mutex> lk(b->m);
        b->phis = phis;
        b->st = st;
        b->status = status;
        b->next.store(0);
        b->busy = (int)b->pool.size();
        b->generation++;
    }
    b->cv_work.notify_all();
    {
        std::unique_lock<std::mutex> lk(b->m);
        b->cv_done.wait(lk, [&] { return b->busy == 0; });
    }
    for (int i = 0; i < n; ++i)
        if (status[i] != PFC_OK) {
            b->err = "instance " + std::to_string(i) + ": " + pfc_last_error(b->ctx[i]);
            return status[i];
        }
    return PFC_OK;
}

pfc_status pfc_batch_reset(pfc_batch* b) {
    if (!b) return PFC_EINVAL;
    for (pfc_ctx* c : b->ctx) {
        const pfc_status s = pfc_reset(c);
        if (s != PFC_OK) return s;
    }
    return PFC_OK;
}

pfc_status pfc_batch_attach_net(pfc_batch* b, pfc_net* net, const double* scales, const double* dt_range) {
    if (!b) return PFC_EINVAL;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        const pfc_status s = pfc_attach_net(b->ctx[i], net, scales, dt_range);
        if (s != PFC_OK) {
            b->err = "instance " + std::to_string(i) + ": " + pfc_last_error(b->ctx[i]);
            return s;
        }
    }
    return PFC_OK;
}

pfc_status pfc_batch_instance(pfc_batch* b, int i, pfc_ctx** out) {
    if (!b || !out || i < 0 || i >= (int)b->ctx.size()) return PFC_EINVAL;
    *out = b->ctx[i];
    return PFC_OK;
}

}  // extern "C"
