// C ABI of the dyadic-pattern fast Hough transform (declared in include/fht.h).
//
// A plan holds, for the two lane orientations of an R x C image (lanes =
// rows for quadrants V+/V-, lanes = columns for H+/H-), the fused-pass tile
// programs made by the planner, concatenated into one header table, one op
// table and one work-item list per launch.  Launch p runs pass p of every
// selected quadrant that has one; pass 0 reads the image, the last pass of a
// quadrant writes its output, and passes in between ping-pong through the
// workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fht.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace {

using fht::JobDesc;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t acc_bytes(fht_dtype d) { return d == FHT_F64 ? 8 : 4; }

struct DevTables {
    int device = -1;
    int32_t *hdrs = nullptr;
    int32_t *ops = nullptr;
    std::vector<int32_t *> items;  // per launch
};

void free_tables(DevTables &t)
{
    if (t.hdrs) (void)hipFree(t.hdrs);
    if (t.ops) (void)hipFree(t.ops);
    for (int32_t *p : t.items)
        if (p) (void)hipFree(p);
    t = DevTables{};
}

template <typename T>
hipError_t upload(const std::vector<T> &host, T **dev)
{
    *dev = nullptr;
    if (host.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dev), host.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
}

fht_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return FHT_OK;
    if (e == hipErrorOutOfMemory) return FHT_ENOMEM;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return FHT_ENODEV;
    return FHT_EHIP;
}

}  // namespace

struct fht_plan_s {
    int32_t R = 0, C = 0;
    fht_dtype dtype = FHT_U8;
    fht_split split = FHT_SPLIT_S;
    uint32_t qmask = 0;
    fht::AxisPlan axis[2];
    int npass[4] = {0, 0, 0, 0};
    size_t out_off[4] = {0, 0, 0, 0};
    size_t out_elems = 0;
    size_t ws_off[4][2] = {};
    size_t ws_bytes = 0;
    // Combined tables: programs of both views, all passes.
    std::vector<int32_t> hdrs, ops;
    std::vector<std::vector<int32_t>> items;  // per launch: {prog, job, s0, 0}
    std::vector<std::vector<int>> jobs_q;     // per launch: quadrant of each job slot
    std::vector<int> lds_bytes;               // per launch
    int threads = 256;                        // per workgroup
    // prog_base[v][p]: index of the first program of view v, pass p.
    std::vector<int> prog_base[2];
    std::mutex mu;
    std::deque<DevTables> dev;  // stable addresses: launches hold pointers into it

    ~fht_plan_s()
    {
        for (DevTables &t : dev) {
            int cur = 0;
            if (hipGetDevice(&cur) == hipSuccess && t.device >= 0) (void)hipSetDevice(t.device);
            free_tables(t);
            (void)hipSetDevice(cur);
        }
    }

    int view_of(int q) const { return q >> 1; }

    // Device tables for the current device, uploading them on first use.
    fht_status tables(const DevTables **out)
    {
        int d = -1;
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return hip_status(e);
        std::lock_guard<std::mutex> lk(mu);
        for (const DevTables &t : dev)
            if (t.device == d) {
                *out = &t;
                return FHT_OK;
            }
        DevTables t;
        t.device = d;
        e = upload(hdrs, &t.hdrs);
        if (e == hipSuccess) e = upload(ops, &t.ops);
        for (size_t p = 0; e == hipSuccess && p < items.size(); ++p) {
            int32_t *ptr = nullptr;
            e = upload(items[p], &ptr);
            t.items.push_back(ptr);
        }
        if (e != hipSuccess) {
            free_tables(t);
            return hip_status(e);
        }
        dev.push_back(t);
        *out = &dev.back();
        return FHT_OK;
    }
};

struct fht_batch_s {
    fht_dtype dtype = FHT_U8;
    int device = -1;
    size_t ws_bytes = 0;
    int32_t *hdrs = nullptr;
    int32_t *ops = nullptr;
    JobDesc *jobs = nullptr;
    std::vector<int32_t *> items;
    std::vector<int> n_items;
    std::vector<int> lds_bytes;
    int threads = 256;

    ~fht_batch_s()
    {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (device >= 0) (void)hipSetDevice(device);
        if (hdrs) (void)hipFree(hdrs);
        if (ops) (void)hipFree(ops);
        if (jobs) (void)hipFree(jobs);
        for (int32_t *p : items)
            if (p) (void)hipFree(p);
        if (have) (void)hipSetDevice(cur);
    }
};

extern "C" {

const char *fht_status_string(fht_status s)
{
    switch (s) {
    case FHT_OK: return "ok";
    case FHT_EINVAL: return "invalid argument";
    case FHT_EDTYPE: return "unsupported or mixed dtype";
    case FHT_ENOMEM: return "out of memory";
    case FHT_EHIP: return "HIP runtime error";
    case FHT_EBUSY: return "over budget";
    case FHT_ENODEV: return "no HIP device";
    }
    return "unknown status";
}

fht_status fht_plan_create(fht_plan *out, int32_t rows, int32_t cols, fht_dtype dtype,
                           fht_split split, uint32_t quadrant_mask, const fht_schedule *sched)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    if (rows < 1 || cols < 1 || rows > 65536 || cols > 65536) return FHT_EINVAL;
    if (quadrant_mask == 0 || quadrant_mask > 15) return FHT_EINVAL;
    if (split != FHT_SPLIT_S && split != FHT_SPLIT_T) return FHT_EINVAL;
    if (dtype != FHT_U8 && dtype != FHT_F32 && dtype != FHT_F64) return FHT_EDTYPE;

    fht::Schedule sc;
    if (sched) {
        if (sched->s_tile) sc.s_tile = sched->s_tile;
        if (sched->s_tile_first) sc.s_tile_first = sched->s_tile_first;
        if (sched->threads) sc.threads = sched->threads;
        if (sched->first_levels) sc.first_levels = sched->first_levels;
        if (sched->max_levels) sc.max_levels = sched->max_levels;
        if (sched->lds_budget) sc.lds_budget = sched->lds_budget;
        if (sched->t_tile) sc.t_tile = sched->t_tile;
    }
    if (sc.s_tile < fht::kChunk || sc.s_tile > fht::kMaxTarget || sc.s_tile % fht::kChunk ||
        sc.s_tile_first < fht::kChunk || sc.s_tile_first > fht::kMaxTarget ||
        sc.s_tile_first % fht::kChunk || sc.first_levels < 1 ||
        (sc.threads != 256 && sc.threads != 512 && sc.threads != 1024) ||
        sc.first_levels > fht::kMaxFirstLevels || sc.max_levels < 1 || sc.max_levels > fht::kMaxSteps ||
        sc.lds_budget < 1024 || sc.lds_budget > 65536 || sc.t_tile < 0 || sc.t_tile > 4096)
        return FHT_EINVAL;

    fht_plan_s *p = new (std::nothrow) fht_plan_s;
    if (!p) return FHT_ENOMEM;
    try {
        p->R = rows;
        p->C = cols;
        p->dtype = dtype;
        p->split = split;
        p->qmask = quadrant_mask;
        p->threads = sc.threads;
        const int eb = static_cast<int>(acc_bytes(dtype));
        // uint8 images: first-pass sums of at most 64 lanes fit 16 bits in LDS.
        const int first_eb = dtype == FHT_U8 ? 2 : eb;
        for (int v = 0; v < 2; ++v) {
            const bool used = quadrant_mask & (3u << (2 * v));
            if (!used) continue;
            const int W = v == 0 ? rows : cols, H = v == 0 ? cols : rows;
            std::string err;
            if (!fht::plan_axis(W, H, static_cast<int>(split), first_eb, eb, sc, &p->axis[v],
                                &err)) {
                delete p;
                return FHT_EINVAL;
            }
        }
        // Output and workspace layout.
        size_t off = 0, ws = 0;
        int nlaunch = 0;
        for (int q = 0; q < 4; ++q) {
            if (!(quadrant_mask & (1u << q))) continue;
            const fht::AxisPlan &ax = p->axis[q >> 1];
            const size_t wh = static_cast<size_t>(ax.W) * ax.H;
            p->out_off[q] = off;
            off += wh;
            p->npass[q] = static_cast<int>(ax.passes.size());
            nlaunch = std::max(nlaunch, p->npass[q]);
            const int nbuf = std::min(p->npass[q] - 1, 2);
            for (int b = 0; b < nbuf; ++b) {
                p->ws_off[q][b] = ws;
                ws += align_up(wh * eb, 256);
            }
        }
        p->out_elems = off;
        p->ws_bytes = ws;
        // Concatenate the program tables of both views.
        for (int v = 0; v < 2; ++v) {
            for (const fht::Pass &ps : p->axis[v].passes) {
                const int op_base = static_cast<int>(p->ops.size() / 4);
                p->prog_base[v].push_back(static_cast<int>(p->hdrs.size() / fht::kHdrInts));
                for (size_t i = 0; i < ps.hdrs.size(); i += fht::kHdrInts) {
                    p->hdrs.insert(p->hdrs.end(), ps.hdrs.begin() + i,
                                   ps.hdrs.begin() + i + fht::kHdrInts);
                    p->hdrs[p->hdrs.size() - fht::kHdrInts] += op_base;
                }
                p->ops.insert(p->ops.end(), ps.ops.begin(), ps.ops.end());
            }
        }
        // Per-launch work lists: job slot j of launch l is the j-th selected
        // quadrant that still has a pass l.
        p->items.resize(nlaunch);
        p->jobs_q.resize(nlaunch);
        p->lds_bytes.assign(nlaunch, 0);
        for (int l = 0; l < nlaunch; ++l) {
            for (int q = 0; q < 4; ++q) {
                if (!(quadrant_mask & (1u << q)) || p->npass[q] <= l) continue;
                const int v = q >> 1;
                const int job = static_cast<int>(p->jobs_q[l].size());
                p->jobs_q[l].push_back(q);
                const fht::Pass &ps = p->axis[v].passes[l];
                for (size_t i = 0; i < ps.items.size(); i += 4) {
                    p->items[l].push_back(ps.items[i] + p->prog_base[v][l]);
                    p->items[l].push_back(job);
                    p->items[l].push_back(ps.items[i + 2]);
                    p->items[l].push_back(0);
                }
                p->lds_bytes[l] = std::max(p->lds_bytes[l], ps.max_lds_elems * (l == 0 ? first_eb : eb));
            }
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return FHT_ENOMEM;
    }
    *out = p;
    return FHT_OK;
}

void fht_plan_destroy(fht_plan plan) { delete plan; }

size_t fht_plan_out_elems(fht_plan plan) { return plan ? plan->out_elems : 0; }

int64_t fht_plan_out_offset(fht_plan plan, int32_t q)
{
    if (!plan || q < 0 || q > 3 || !(plan->qmask & (1u << q))) return -1;
    return static_cast<int64_t>(plan->out_off[q]);
}

size_t fht_plan_workspace_bytes(fht_plan plan) { return plan ? plan->ws_bytes : 0; }

int32_t fht_plan_num_launches(fht_plan plan)
{
    return plan ? static_cast<int32_t>(plan->items.size()) : 0;
}

fht_status fht_plan_upload(fht_plan plan)
{
    if (!plan) return FHT_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    const DevTables *t = nullptr;
    return plan->tables(&t);
}

static fht_status forward_one(fht_plan plan, const DevTables *t, size_t l, const void *d_img,
                              void *d_out, void *d_ws, void *stream)
{
    const size_t eb = acc_bytes(plan->dtype);
    const fht::Dt dt = static_cast<fht::Dt>(plan->dtype);
    char *ws = static_cast<char *>(d_ws);
    char *out = static_cast<char *>(d_out);
    fht::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.items = reinterpret_cast<const int4 *>(t->items[l]);
    a.hdrs = t->hdrs;
    a.ops = reinterpret_cast<const int4 *>(t->ops);
    a.jobs = nullptr;
    a.ws = nullptr;
    for (size_t j = 0; j < plan->jobs_q[l].size(); ++j) {
        const int q = plan->jobs_q[l][j];
        const fht::AxisPlan &ax = plan->axis[q >> 1];
        const bool final = static_cast<int>(l) == plan->npass[q] - 1;
        JobDesc &jd = a.inl[j];
        jd.src = (l == 0) ? d_img : ws + plan->ws_off[q][(l - 1) & 1];
        jd.dst = final ? out + plan->out_off[q] * eb : ws + plan->ws_off[q][l & 1];
        jd.H = ax.H;
        jd.ld = plan->C;
        jd.flags = ((q >> 1) ? fht::JF_COLS : 0) | ((q & 1) ? fht::JF_MIRROR : 0) |
                   (final ? fht::JF_FINAL : 0);
    }
    const int nitems = static_cast<int>(plan->items[l].size() / 4);
    const hipError_t e = fht::launch_pass(dt, l == 0, a, nitems, plan->lds_bytes[l],
                                          plan->threads, static_cast<hipStream_t>(stream));
    return hip_status(e);
}

static fht_status forward_checks(fht_plan plan, const void *d_img, void *d_out, void *d_ws,
                                 const DevTables **t)
{
    if (!plan || !d_img || !d_out) return FHT_EINVAL;
    if (plan->ws_bytes && !d_ws) return FHT_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    return plan->tables(t);
}

fht_status fht_forward(fht_plan plan, const void *d_img, void *d_out, void *d_ws, void *stream)
{
    const DevTables *t = nullptr;
    fht_status st = forward_checks(plan, d_img, d_out, d_ws, &t);
    for (size_t l = 0; st == FHT_OK && l < plan->items.size(); ++l)
        st = forward_one(plan, t, l, d_img, d_out, d_ws, stream);
    return st;
}

fht_status fht_forward_launch(fht_plan plan, int32_t launch, const void *d_img, void *d_out,
                              void *d_ws, void *stream)
{
    const DevTables *t = nullptr;
    fht_status st = forward_checks(plan, d_img, d_out, d_ws, &t);
    if (st != FHT_OK) return st;
    if (launch < 0 || launch >= static_cast<int32_t>(plan->items.size())) return FHT_EINVAL;
    return forward_one(plan, t, static_cast<size_t>(launch), d_img, d_out, d_ws, stream);
}

fht_status fht_batch_create(fht_batch *out, const fht_plan *plans, int32_t n,
                            const void *const *d_imgs, void *const *d_outs)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    if (!plans || !d_imgs || !d_outs || n < 1) return FHT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !d_imgs[i] || !d_outs[i]) return FHT_EINVAL;
    for (int i = 1; i < n; ++i)
        if (plans[i]->dtype != plans[0]->dtype || plans[i]->split != plans[0]->split)
            return FHT_EDTYPE;
    for (int i = 1; i < n; ++i)
        if (plans[i]->threads != plans[0]->threads) return FHT_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return FHT_ENODEV;

    fht_batch_s *b = new (std::nothrow) fht_batch_s;
    if (!b) return FHT_ENOMEM;
    b->dtype = plans[0]->dtype;
    b->threads = plans[0]->threads;
    const size_t eb = acc_bytes(b->dtype);
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_status(e);
    }
    try {
        // Distinct plans share one copy of their tables.
        std::vector<fht_plan> uniq;
        std::vector<int> hdr_base, op_base;
        std::vector<int32_t> hdrs, ops;
        auto table_of = [&](fht_plan p) {
            for (size_t u = 0; u < uniq.size(); ++u)
                if (uniq[u] == p) return static_cast<int>(u);
            uniq.push_back(p);
            hdr_base.push_back(static_cast<int>(hdrs.size() / fht::kHdrInts));
            op_base.push_back(static_cast<int>(ops.size() / 4));
            for (size_t i = 0; i < p->hdrs.size(); i += fht::kHdrInts) {
                hdrs.insert(hdrs.end(), p->hdrs.begin() + i, p->hdrs.begin() + i + fht::kHdrInts);
                hdrs[hdrs.size() - fht::kHdrInts] += op_base.back();
            }
            ops.insert(ops.end(), p->ops.begin(), p->ops.end());
            return static_cast<int>(uniq.size() - 1);
        };
        size_t nlaunch = 0;
        for (int i = 0; i < n; ++i) nlaunch = std::max(nlaunch, plans[i]->items.size());
        std::vector<std::vector<int32_t>> items(nlaunch);
        std::vector<JobDesc> jobs;
        b->lds_bytes.assign(nlaunch, 0);
        size_t ws = 0;
        for (int i = 0; i < n; ++i) {
            const fht_plan p = plans[i];
            const int u = table_of(p);
            const size_t ws_base = ws;
            ws += align_up(p->ws_bytes, 256);
            for (size_t l = 0; l < p->items.size(); ++l) {
                std::vector<int> slot;
                for (size_t j = 0; j < p->jobs_q[l].size(); ++j) {
                    const int q = p->jobs_q[l][j];
                    const fht::AxisPlan &ax = p->axis[q >> 1];
                    const bool final = static_cast<int>(l) == p->npass[q] - 1;
                    JobDesc jd;
                    std::memset(&jd, 0, sizeof(jd));
                    int flags = ((q >> 1) ? fht::JF_COLS : 0) | ((q & 1) ? fht::JF_MIRROR : 0) |
                                (final ? fht::JF_FINAL : 0);
                    if (l == 0) {
                        jd.src = d_imgs[i];
                    } else {
                        jd.src = reinterpret_cast<const void *>(ws_base + p->ws_off[q][(l - 1) & 1]);
                        flags |= fht::JF_SRC_WS;
                    }
                    if (final) {
                        jd.dst = static_cast<char *>(d_outs[i]) + p->out_off[q] * eb;
                    } else {
                        jd.dst = reinterpret_cast<void *>(ws_base + p->ws_off[q][l & 1]);
                        flags |= fht::JF_DST_WS;
                    }
                    jd.H = ax.H;
                    jd.ld = p->C;
                    jd.flags = flags;
                    slot.push_back(static_cast<int>(jobs.size()));
                    jobs.push_back(jd);
                }
                const std::vector<int32_t> &src = p->items[l];
                for (size_t k = 0; k < src.size(); k += 4) {
                    const int prog = src[k];
                    // rebase the program index from the plan's table to the batch's
                    items[l].push_back(prog + hdr_base[u]);
                    items[l].push_back(slot[src[k + 1]]);
                    items[l].push_back(src[k + 2]);
                    items[l].push_back(0);
                }
                b->lds_bytes[l] = std::max(b->lds_bytes[l], p->lds_bytes[l]);
            }
        }
        b->ws_bytes = ws;
        e = upload(hdrs, &b->hdrs);
        if (e == hipSuccess) e = upload(ops, &b->ops);
        if (e == hipSuccess) e = upload(jobs, &b->jobs);
        for (size_t l = 0; e == hipSuccess && l < nlaunch; ++l) {
            int32_t *ptr = nullptr;
            e = upload(items[l], &ptr);
            b->items.push_back(ptr);
            b->n_items.push_back(static_cast<int>(items[l].size() / 4));
        }
        if (e != hipSuccess) {
            delete b;
            return hip_status(e);
        }
    } catch (const std::bad_alloc &) {
        delete b;
        return FHT_ENOMEM;
    }
    *out = b;
    return FHT_OK;
}

size_t fht_batch_workspace_bytes(fht_batch batch) { return batch ? batch->ws_bytes : 0; }

int32_t fht_batch_num_launches(fht_batch batch)
{
    return batch ? static_cast<int32_t>(batch->items.size()) : 0;
}

static fht_status batch_one(fht_batch batch, size_t l, void *d_ws, void *stream)
{
    fht::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.items = reinterpret_cast<const int4 *>(batch->items[l]);
    a.hdrs = batch->hdrs;
    a.ops = reinterpret_cast<const int4 *>(batch->ops);
    a.jobs = batch->jobs;
    a.ws = static_cast<char *>(d_ws);
    const hipError_t e = fht::launch_pass(static_cast<fht::Dt>(batch->dtype), l == 0, a,
                                          batch->n_items[l], batch->lds_bytes[l], batch->threads,
                                          static_cast<hipStream_t>(stream));
    return hip_status(e);
}

fht_status fht_batch_run(fht_batch batch, void *d_ws, void *stream)
{
    if (!batch) return FHT_EINVAL;
    if (batch->ws_bytes && !d_ws) return FHT_EINVAL;
    fht_status st = FHT_OK;
    for (size_t l = 0; st == FHT_OK && l < batch->items.size(); ++l)
        st = batch_one(batch, l, d_ws, stream);
    return st;
}

fht_status fht_batch_run_launch(fht_batch batch, int32_t launch, void *d_ws, void *stream)
{
    if (!batch) return FHT_EINVAL;
    if (batch->ws_bytes && !d_ws) return FHT_EINVAL;
    if (launch < 0 || launch >= static_cast<int32_t>(batch->items.size())) return FHT_EINVAL;
    return batch_one(batch, static_cast<size_t>(launch), d_ws, stream);
}

void fht_batch_destroy(fht_batch batch) { delete batch; }

int32_t fht_plan_num_passes(fht_plan plan, int32_t v)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v)))) return -1;
    return static_cast<int32_t>(plan->axis[v].passes.size());
}

fht_status fht_plan_pass_tables(fht_plan plan, int32_t v, int32_t pass, const int32_t **hdrs,
                                int32_t *n_progs, const int32_t **ops, int32_t *n_ops,
                                const int32_t **items, int32_t *n_items, int32_t *s_tile)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v)))) return FHT_EINVAL;
    const fht::AxisPlan &ax = plan->axis[v];
    if (pass < 0 || pass >= static_cast<int32_t>(ax.passes.size())) return FHT_EINVAL;
    const fht::Pass &ps = ax.passes[pass];
    if (hdrs) *hdrs = ps.hdrs.data();
    if (n_progs) *n_progs = static_cast<int32_t>(ps.hdrs.size() / fht::kHdrInts);
    if (ops) *ops = ps.ops.data();
    if (n_ops) *n_ops = static_cast<int32_t>(ps.ops.size() / 4);
    if (items) *items = ps.items.data();
    if (n_items) *n_items = static_cast<int32_t>(ps.items.size() / 4);
    if (s_tile) *s_tile = ps.S;
    return FHT_OK;
}

}  // extern "C"
