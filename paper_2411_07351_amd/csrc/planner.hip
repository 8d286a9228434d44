// Native planner pool: plans made (and their lane-view programs copied to a
// device) on threads of the library, so that a request loop in any language
// only submits and polls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "fht.h"

namespace {

struct Task {
    int64_t ticket;
    int32_t rows, cols;
    int32_t dtype;
    int32_t split;
    uint32_t qmask;
    bool has_sched;
    fht_schedule sched;
};

struct Result {
    fht_status status;
    fht_plan plan;
};

// Plans per batched copy of the uploader.
constexpr size_t kUploadGroup = 32;

}  // namespace

// Worker threads only plan (host code); one uploader thread, the only one
// that calls HIP, copies the programs of up to kUploadGroup finished plans in
// one allocation and one copy: small allocations and copies from many threads
// serialise inside the HIP runtime.
struct fht_planner_s {
    int device = -1;
    std::mutex mu;
    std::condition_variable cv, up_cv;
    std::deque<Task> queue;                           // to plan
    std::deque<std::pair<int64_t, fht_plan>> up;     // planned, to copy
    std::unordered_set<int64_t> pending;              // queued, planning or copying
    std::unordered_map<int64_t, Result> done;
    int64_t next = 0;
    bool stop = false, up_stop = false;
    std::vector<std::thread> workers;
    std::thread uploader;

    void finish(int64_t ticket, Result r)  // with mu held
    {
        pending.erase(ticket);
        done.emplace(ticket, r);
    }

    void work()
    {
        for (;;) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop) return;
                t = queue.front();
                queue.pop_front();
            }
            Result r{FHT_OK, nullptr};
            r.status = fht_plan_create(&r.plan, t.rows, t.cols, t.dtype, t.split, t.qmask,
                                       t.has_sched ? &t.sched : nullptr);
            std::lock_guard<std::mutex> lk(mu);
            if (r.status == FHT_OK && device >= 0) {
                up.emplace_back(t.ticket, r.plan);
                up_cv.notify_one();
            } else {
                finish(t.ticket, r);
            }
        }
    }

    void upload()
    {
        fht_status dev_status = FHT_OK;
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n <= device) dev_status = FHT_ENODEV;
        else if (hipSetDevice(device) != hipSuccess) dev_status = FHT_EHIP;
        std::vector<std::pair<int64_t, fht_plan>> jobs;
        std::vector<fht_plan> plans;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                up_cv.wait(lk, [&] { return up_stop || !up.empty(); });
                if (up_stop) return;
                // the plans finished so far, a bounded number at a time so that
                // plans become ready while others are still being planned
                const size_t k = std::min(up.size(), kUploadGroup);
                jobs.assign(up.begin(), up.begin() + k);
                up.erase(up.begin(), up.begin() + k);
            }
            plans.clear();
            for (const auto &j : jobs) plans.push_back(j.second);
            fht_status all = dev_status;
            if (all == FHT_OK)
                all = fht_plan_upload_programs_many(plans.data(), static_cast<int32_t>(plans.size()));
            std::vector<Result> res;
            for (const auto &j : jobs) {
                Result r{all, j.second};
                // on a failure, find the plans that fail on their own
                if (r.status != FHT_OK && dev_status == FHT_OK)
                    r.status = fht_plan_upload_programs(r.plan);
                if (r.status != FHT_OK) {
                    fht_plan_destroy(r.plan);
                    r.plan = nullptr;
                }
                res.push_back(r);
            }
            std::lock_guard<std::mutex> lk(mu);
            for (size_t k = 0; k < jobs.size(); ++k) finish(jobs[k].first, res[k]);
        }
    }
};

extern "C" {

fht_status fht_planner_create(int32_t threads, int32_t device, fht_planner *out)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    if (threads < 1 || threads > 256 || device < -1) return FHT_EINVAL;
    fht_planner p = new (std::nothrow) fht_planner_s;
    if (!p) return FHT_ENOMEM;
    p->device = device;
    try {
        for (int i = 0; i < threads; ++i) p->workers.emplace_back([p] { p->work(); });
        if (device >= 0) p->uploader = std::thread([p] { p->upload(); });
    } catch (...) {
        fht_planner_destroy(p);
        return FHT_ENOMEM;
    }
    *out = p;
    return FHT_OK;
}

fht_status fht_planner_submit(fht_planner pl, int32_t rows, int32_t cols, int32_t dtype,
                              int32_t split, uint32_t quadrant_mask,
                              const fht_schedule *sched, int64_t *ticket)
{
    if (!pl || !ticket) return FHT_EINVAL;
    Task t{};
    t.rows = rows;
    t.cols = cols;
    t.dtype = dtype;
    t.split = split;
    t.qmask = quadrant_mask;
    t.has_sched = sched != nullptr;
    if (sched) t.sched = *sched;
    try {
        std::lock_guard<std::mutex> lk(pl->mu);
        t.ticket = pl->next;
        pl->queue.push_back(t);
        try {
            pl->pending.insert(t.ticket);
        } catch (...) {
            pl->queue.pop_back();
            throw;
        }
        ++pl->next;
    } catch (...) {
        return FHT_ENOMEM;
    }
    pl->cv.notify_one();
    *ticket = t.ticket;
    return FHT_OK;
}

int32_t fht_planner_poll(fht_planner pl, int64_t ticket, fht_plan *plan, fht_status *status)
{
    if (!pl || !plan || !status) return -1;
    std::lock_guard<std::mutex> lk(pl->mu);
    auto it = pl->done.find(ticket);
    if (it == pl->done.end()) return pl->pending.count(ticket) ? 0 : -1;
    *plan = it->second.plan;
    *status = it->second.status;
    pl->done.erase(it);
    return 1;
}

void fht_planner_destroy(fht_planner pl)
{
    if (!pl) return;
    {
        std::lock_guard<std::mutex> lk(pl->mu);
        pl->stop = true;
        pl->queue.clear();  // submitted, not started: never made
    }
    pl->cv.notify_all();
    for (std::thread &w : pl->workers)
        if (w.joinable()) w.join();
    {
        std::lock_guard<std::mutex> lk(pl->mu);
        pl->up_stop = true;
    }
    pl->up_cv.notify_all();
    if (pl->uploader.joinable()) pl->uploader.join();
    for (auto &j : pl->up) fht_plan_destroy(j.second);  // planned, never copied
    for (auto &kv : pl->done) fht_plan_destroy(kv.second.plan);
    delete pl;
}

}  // extern "C"
