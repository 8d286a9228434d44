// C ABI of the dyadic-pattern fast Hough transform (declared in include/fht.h).
//
// A plan holds, for the two lane orientations of an R x C image (lanes =
// rows for quadrants V+/V-, lanes = columns for H+/H-), the fused-pass tile
// programs made by the planner, concatenated into one header table and one
// entry table, plus a list of launches.  Pass p of every selected quadrant
// runs in the launches of level p (one per element-type combination: the two
// orientations of a non-square image may differ); pass 0 reads the image, the
// last pass of a quadrant writes its output, and passes in between ping-pong
// through the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <tuple>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fht.h"
#include "kernels.hpp"
#include "plan.hpp"

// Workspace of fht_forward_noalloc, for callers that cannot allocate device
// memory.  The runtime gives every device its own copy when it loads this
// code object; it lives until the process ends.  Host code must not pass the
// array's name to a kernel (on the host it only stands for the symbol): it
// uses the device address hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) unsigned char scratch[FHT_NOALLOC_WS_BYTES];

namespace {

using fht::Combo;
using fht::JobDesc;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes of an output (and workspace) element.
size_t acc_bytes(fht_dtype d) { return d == FHT_F64 ? 8 : 4; }

fht_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return FHT_OK;
    if (e == hipErrorOutOfMemory) return FHT_ENOMEM;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return FHT_ENODEV;
    return FHT_EHIP;
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

// uint8 images keep 16-bit sums while nodes are at most this wide.
constexpr int kNarrowWidth = 257;

// Tree levels per adjoint gather launch.
constexpr int kAdjointFuse = 3;

// Output rows of a gather pass in the order its launch takes them, by the
// lowest source row they read: the rows of a node's descendants (several
// levels down) at the same relative slope read the same source rows at
// different shifts, and consecutive rows of the order share a workgroup.
std::vector<int32_t> gather_order(const fht::AdjointPass &ap)
{
    const int W = static_cast<int>(ap.offs.size()) - 1;
    std::vector<int32_t> key(W), order(W);
    for (int x = 0; x < W; ++x) {
        int lo = INT32_MAX;
        for (int i = ap.offs[x]; i < ap.offs[x + 1]; ++i) lo = std::min(lo, ap.terms[2 * i]);
        key[x] = lo;
        order[x] = x;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    return order;
}

// The fused final adjoint launch needs at least this many 64 x 64 tiles (one
// per compute unit); below, the last gathers and the combine run apart.
constexpr int64_t kFinalMinTiles = 256;

// Element types of pass p of an axis plan (see fht::Combo); `pair` selects
// the quadrant-pair form.
Combo pass_combo(fht_dtype dt, const fht::AxisPlan &ax, size_t p, bool pair)
{
    const bool final = p + 1 == ax.passes.size();
    if (pair) {
        if (p == 0) return final ? Combo::P_U8_FIRST_FINAL : Combo::P_U8_FIRST;
        if (ax.passes[p].max_root_w <= kNarrowWidth)
            return final ? Combo::P_U16_MID_FINAL : Combo::P_U16_MID;
        return Combo::P_I32;
    }
    if (dt == FHT_F32) return p == 0 ? Combo::F32_FIRST : Combo::F32_LATER;
    if (dt == FHT_F64) return p == 0 ? Combo::F64_FIRST : Combo::F64_LATER;
    const bool narrow_out = ax.passes[p].max_root_w <= kNarrowWidth;
    if (p == 0) return final ? Combo::U8_U16_I32 : Combo::U8_U16_U16;
    const bool narrow_in = ax.passes[p - 1].max_root_w <= kNarrowWidth;
    if (!narrow_in) return Combo::I32_I32_I32;
    if (!narrow_out) return Combo::U16_I32_I32;
    return final ? Combo::U16_U16_I32 : Combo::U16_U16_U16;
}

// A job slot of a plan launch: quadrant q, or the pair q, q + 1 of one lane view.
struct JobRef {
    int q = 0;
    bool pair = false;
};

// One kernel launch: the work items of one level and one type combination.
struct Launch {
    int level = 0;
    Combo combo = Combo::I32_I32_I32;
    int lds_bytes = 0;
    int threads = 256;
    std::vector<int32_t> items;  // {program, job slot, first position, first entry}
    std::vector<JobRef> jobs;    // plan launches: what each job slot runs
    std::string kernel;          // plan launches: the kernel's template signature
};

// The signature of the kernel a launch runs, as profilers print it.
std::string kernel_name(Combo c, int threads, bool table)
{
    const char *src = "int", *lds = "int", *dst = "int";
    bool first = false, pair = false;
    switch (c) {
    case Combo::U8_U16_U16: src = "unsigned char"; lds = dst = "unsigned short"; first = true; break;
    case Combo::U8_U16_I32: src = "unsigned char"; lds = "unsigned short"; first = true; break;
    case Combo::U16_U16_U16: src = lds = dst = "unsigned short"; break;
    case Combo::U16_U16_I32: src = lds = "unsigned short"; break;
    case Combo::U16_I32_I32: src = "unsigned short"; break;
    case Combo::I32_I32_I32: break;
    case Combo::F32_FIRST: first = true; [[fallthrough]];
    case Combo::F32_LATER: src = lds = dst = "float"; break;
    case Combo::F64_FIRST: first = true; [[fallthrough]];
    case Combo::F64_LATER: src = lds = dst = "double"; break;
    case Combo::P_U8_FIRST: src = "unsigned char"; lds = dst = "unsigned int"; first = pair = true; break;
    case Combo::P_U8_FIRST_FINAL: src = "unsigned char"; lds = "unsigned int"; first = pair = true; break;
    case Combo::P_U16_MID: src = lds = dst = "unsigned int"; pair = true; break;
    case Combo::P_U16_MID_FINAL: src = lds = "unsigned int"; pair = true; break;
    case Combo::P_I32: src = "unsigned int"; lds = "HIP_vector_type<unsigned int, 2u>"; pair = true; break;
    }
    return "fht_pass_kernel<" + std::to_string(threads) + ", " + src + ", " + lds + ", " + dst +
           ", " + (first ? "true" : "false") + ", " + (table ? "true" : "false") + ", " +
           (pair ? "true" : "false") + ">";
}

// Program memory of lane views that left the plan cache.  hipFree waits for
// the whole device, so blocks are not freed one by one as views leave the
// cache (a burst of fresh plans in a full cache would stall every stream once
// per eviction); they are collected and freed together once they pass
// kRetireBytes.
constexpr size_t kRetireBytes = size_t(64) << 20;

struct Retired {
    std::mutex mu;
    std::vector<std::pair<int, void *>> blocks;  // (device, pointer)
    size_t bytes = 0;
};

Retired &retired()
{
    static Retired *r = new Retired;  // never destroyed (see axis_cache)
    return *r;
}

void retire(int device, void *p, size_t bytes)
{
    std::vector<std::pair<int, void *>> now;
    {
        Retired &r = retired();
        std::lock_guard<std::mutex> lk(r.mu);
        r.blocks.emplace_back(device, p);
        r.bytes += bytes;
        if (r.bytes < kRetireBytes) return;
        now.swap(r.blocks);
        r.bytes = 0;
    }
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (const auto &b : now) {
        (void)hipSetDevice(b.first);
        (void)hipFree(b.second);
    }
    if (have) (void)hipSetDevice(cur);
}

// Device memory of `bytes` bytes, retired (on its own device) with the last
// view using it.
std::shared_ptr<void> device_block(void *p, int device, size_t bytes)
{
    return std::shared_ptr<void>(p, [device, bytes](void *q) { retire(device, q, bytes); });
}

// Batched program copies on one device: a non-blocking stream and two pinned
// staging buffers that host copies and DMA alternate between (made on first
// use, kept until the process ends).
constexpr size_t kStageBytes = size_t(4) << 20;

struct CopyLane {
    std::mutex mu;
    hipStream_t stream = nullptr;
    void *stage[2] = {nullptr, nullptr};
    hipEvent_t free[2] = {nullptr, nullptr};  // the last copy out of stage[b] is done

    hipError_t init()
    {
        hipError_t e = hipSuccess;
        if (!stream) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        for (int b = 0; b < 2 && e == hipSuccess; ++b) {
            if (!stage[b]) e = hipHostMalloc(&stage[b], kStageBytes, 0);
            if (e == hipSuccess && !free[b]) e = hipEventCreateWithFlags(&free[b], hipEventDisableTiming);
        }
        return e;
    }
};

// Image sink into a host vector.
struct VecSink {
    std::vector<int32_t> v;
    void put(const int32_t *p, size_t n) { v.insert(v.end(), p, p + n); }
    void zeros(size_t n) { v.resize(v.size() + n, 0); }
};

// Image sink that writes a device range through a lane's staging buffers:
// host writes fill one buffer while the DMA empties the other.  The lane's
// mutex must be held from the first write to finish().
struct StagedSink {
    CopyLane &L;
    char *dev;
    size_t at = 0, fill = 0, flushes = 0;
    int b = 0;
    hipError_t e = hipSuccess;

    void bytes(const void *p, size_t n)
    {
        const char *c = static_cast<const char *>(p);
        while (n && e == hipSuccess) {
            const size_t m = std::min(n, kStageBytes - fill);
            char *s = static_cast<char *>(L.stage[b]) + fill;
            if (c) {
                std::memcpy(s, c, m);
                c += m;
            } else {
                std::memset(s, 0, m);
            }
            fill += m;
            n -= m;
            if (fill == kStageBytes) flush();
        }
    }
    void put(const int32_t *p, size_t n) { bytes(p, n * sizeof(int32_t)); }
    void zeros(size_t n) { bytes(nullptr, n * sizeof(int32_t)); }
    void pad_to(size_t align)
    {
        const size_t pos = at + fill;
        bytes(nullptr, align_up(pos, align) - pos);
    }

    void flush()
    {
        if (!fill || e != hipSuccess) return;
        e = hipMemcpyAsync(dev + at, L.stage[b], fill, hipMemcpyHostToDevice, L.stream);
        if (e == hipSuccess) e = hipEventRecord(L.free[b], L.stream);
        at += fill;
        fill = 0;
        b ^= 1;
        // buffer b was last emptied by the flush before this one
        if (e == hipSuccess && ++flushes >= 2) e = hipEventSynchronize(L.free[b]);
    }

    hipError_t finish()
    {
        flush();
        const hipError_t s = hipStreamSynchronize(L.stream);
        return e != hipSuccess ? e : s;
    }
};

CopyLane &copy_lane(int d)
{
    static std::mutex m;
    static std::map<int, CopyLane *> *lanes = new std::map<int, CopyLane *>;
    std::lock_guard<std::mutex> lk(m);
    CopyLane *&l = (*lanes)[d];
    if (!l) l = new CopyLane;
    return *l;
}

// Device copy of one lane view's tile programs.
struct DevProgs {
    int device = -1;
    int32_t *hdrs = nullptr;  // after the entries, in the same block
    int4 *ops = nullptr;
    std::shared_ptr<void> mem;  // the block (may hold other views' programs too)
};

// One lane view's tile programs, shared by every plan with the same lane
// count, schedule and element rule and H at least the widest position window
// (see fht::retile_items), with their device copies (uploaded on first use on
// each device, freed with the last plan that uses them).  `plan.passes[p].items`
// are for H = min(H, kMaxTarget); plans keep their own items.
struct ViewProgs {
    fht::AxisPlan plan;
    std::mutex mu;
    std::deque<DevProgs> dev;

    // Device copy on device d, or null (with mu held).
    const DevProgs *find(int d) const
    {
        for (const DevProgs &x : dev)
            if (x.device == d) return &x;
        return nullptr;
    }

    bool on_device(int d)
    {
        std::lock_guard<std::mutex> lk(mu);
        return find(d) != nullptr;
    }

    // The device image, written to `out` (put(ints, n), zeros(n)): every
    // pass's entries (program headers point at them by index), spare zero
    // entries (the first pass fetches entries [first, first + 64) of a
    // program before it knows its length), then the headers.  *n_ops: ints
    // before the headers.
    template <typename Sink>
    void write_image(Sink &out, size_t *n_ops) const
    {
        size_t ops = 0;
        for (const fht::Pass &ps : plan.passes) {
            out.put(ps.ops.data(), ps.ops.size());
            ops += ps.ops.size();
        }
        out.zeros(4 * fht::kEntryPrefetch);
        *n_ops = ops + 4 * fht::kEntryPrefetch;
        int op_base = 0;
        for (const fht::Pass &ps : plan.passes) {
            int32_t h[fht::kHdrInts];
            for (size_t i = 0; i < ps.hdrs.size(); i += fht::kHdrInts) {
                std::copy(ps.hdrs.begin() + i, ps.hdrs.begin() + i + fht::kHdrInts, h);
                h[fht::kHdrFirst] += op_base;
                out.put(h, fht::kHdrInts);
            }
            op_base += static_cast<int>(ps.ops.size() / 4);
        }
    }

    size_t image_ints() const
    {
        size_t n = 4 * fht::kEntryPrefetch;
        for (const fht::Pass &ps : plan.passes) n += ps.ops.size() + ps.hdrs.size();
        return n;
    }

    // Records a copy of image() at `at` (16-byte aligned) in block `mem` on
    // device d, unless one is there already.
    const DevProgs *adopt(int d, int32_t *at, size_t n_ops, const std::shared_ptr<void> &mem)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (const DevProgs *x = find(d)) return x;
        DevProgs x;
        x.device = d;
        x.ops = reinterpret_cast<int4 *>(at);
        x.hdrs = at + n_ops;
        x.mem = mem;
        dev.push_back(x);
        return &dev.back();
    }

    fht_status device_progs(const DevProgs **out)
    {
        int d = -1;
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return hip_status(e);
        {
            std::lock_guard<std::mutex> lk(mu);
            if ((*out = find(d))) return FHT_OK;
        }
        size_t n_ops = 0;
        VecSink img;
        img.v.reserve(image_ints());
        write_image(img, &n_ops);
        int32_t *o = nullptr;
        e = upload(img.v, &o);
        if (e != hipSuccess) {
            if (o) (void)hipFree(o);
            return hip_status(e);
        }
        *out = adopt(d, o, n_ops, device_block(o, d, img.v.size() * sizeof(int32_t)));
        return FHT_OK;
    }

    // First program of pass p in the concatenated tables.
    int prog_base(size_t p) const
    {
        int b = 0;
        for (size_t i = 0; i < p; ++i) b += static_cast<int>(plan.passes[i].hdrs.size() / fht::kHdrInts);
        return b;
    }

    // Device entry index of the first entry of program `prog` of pass p.
    int first_entry(size_t p, int prog) const
    {
        int b = 0;
        for (size_t i = 0; i < p; ++i) b += static_cast<int>(plan.passes[i].ops.size() / 4);
        return b + plan.passes[p].hdrs[static_cast<size_t>(prog) * fht::kHdrInts];
    }
};

struct DevTables {
    int device = -1;
    const DevProgs *views[2] = {nullptr, nullptr};
    int32_t *items_blob = nullptr;              // every launch's items, one allocation
    std::vector<int32_t *> items;               // per launch, into items_blob
    bool adj_up = false;                         // adjoint tables uploaded (first adjoint call)
    int32_t *adj_offs[2] = {nullptr, nullptr};   // fused adjoint passes per lane view
    int32_t *adj_terms[2] = {nullptr, nullptr};
    size_t bytes = 0;                            // device bytes of the tables above
};

// Retires a plan's device tables (see retire: a plan destroyed while other
// work runs does not wait for the device).
void free_tables(DevTables &t)
{
    const size_t share = t.bytes / 5 + 1;  // the retire threshold only needs a rough size
    for (int32_t *p : t.adj_offs)
        if (p) retire(t.device, p, share);
    for (int32_t *p : t.adj_terms)
        if (p) retire(t.device, p, share);
    if (t.items_blob) retire(t.device, t.items_blob, share);
    t = DevTables{};
}

// Process-wide cache of lane-view programs: a view of W lanes is planned once
// per schedule, element rule and min(H, kMaxTarget).  Bounded by the bytes of
// the cached host tables, least recently used first out.
struct AxisKey {
    int W, H, split, narrow, wide, narrow_w, transition;
    int s_tile, s_tile_first, first_levels, max_levels, lds_budget, t_tile;
    bool operator<(const AxisKey &o) const
    {
        return std::tie(W, H, split, narrow, wide, narrow_w, transition, s_tile, s_tile_first,
                        first_levels, max_levels, lds_budget, t_tile) <
               std::tie(o.W, o.H, o.split, o.narrow, o.wide, o.narrow_w, o.transition, o.s_tile,
                        o.s_tile_first, o.first_levels, o.max_levels, o.lds_budget, o.t_tile);
    }
};

struct AxisCache {
    std::mutex mu;
    std::list<std::pair<AxisKey, std::shared_ptr<ViewProgs>>> lru;
    std::map<AxisKey, decltype(lru)::iterator> index;
    size_t bytes = 0;
    size_t capacity = size_t(256) << 20;
};

AxisCache &axis_cache()
{
    // never destroyed: its device tables must not be freed after the HIP
    // runtime has shut down at process exit
    static AxisCache *c = new AxisCache;
    return *c;
}

size_t table_bytes(const fht::AxisPlan &ax)
{
    size_t b = 0;
    for (const fht::Pass &ps : ax.passes) b += (ps.hdrs.size() + ps.ops.size() + ps.items.size()) * 4;
    return b;
}

// The view's programs, and the work items of each pass for height H.
std::shared_ptr<ViewProgs> plan_view(int W, int H, int split, const fht::ElemRule &rule,
                                     const fht::Schedule &sc,
                                     std::vector<std::vector<int32_t>> *items)
{
    const int Hk = std::min(H, fht::kMaxTarget);
    const AxisKey key{W, Hk, split, rule.narrow_bytes, rule.wide_bytes, rule.narrow_width,
                      rule.transition_bytes, sc.s_tile, sc.s_tile_first, sc.first_levels,
                      sc.max_levels, sc.lds_budget, sc.t_tile};
    AxisCache &c = axis_cache();
    std::shared_ptr<ViewProgs> hit;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.index.find(key);
        if (it != c.index.end()) {
            c.lru.splice(c.lru.begin(), c.lru, it->second);
            hit = it->second->second;
        }
    }
    if (!hit) {
        auto made = std::make_shared<ViewProgs>();
        std::string err;
        if (!fht::plan_axis(W, Hk, split, rule, sc, &made->plan, &err)) return nullptr;
        // views pushed out of the cache are destroyed after the lock is released
        std::vector<std::shared_ptr<ViewProgs>> dropped;
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.index.find(key);
        if (it != c.index.end()) {
            hit = it->second->second;  // planned meanwhile by another thread
        } else {
            hit = made;
            c.lru.emplace_front(key, hit);
            c.index[key] = c.lru.begin();
            c.bytes += table_bytes(hit->plan);
            while (c.bytes > c.capacity && c.lru.size() > 1) {
                c.bytes -= table_bytes(c.lru.back().second->plan);
                c.index.erase(c.lru.back().first);
                dropped.push_back(std::move(c.lru.back().second));
                c.lru.pop_back();
            }
        }
    }
    items->clear();
    if (H == Hk) {
        for (const fht::Pass &ps : hit->plan.passes) items->push_back(ps.items);
    } else {
        fht::AxisPlan shape;  // passes with programs counted but not copied
        for (const fht::Pass &ps : hit->plan.passes) {
            fht::Pass q;
            q.S = ps.S;
            q.hdrs.resize(ps.hdrs.size());
            shape.passes.push_back(std::move(q));
        }
        fht::retile_items(&shape, H);
        for (fht::Pass &ps : shape.passes) items->push_back(std::move(ps.items));
    }
    return hit;
}

}  // namespace

struct fht_plan_s {
    int32_t R = 0, C = 0;
    fht_dtype dtype = FHT_U8;
    fht_split split = FHT_SPLIT_S;
    uint32_t qmask = 0;
    int threads = 512, threads_first = 256;
    std::shared_ptr<ViewProgs> view[2];            // programs of lane view v (shared)
    int vW[2] = {0, 0}, vH[2] = {0, 0};            // lanes and positions of view v
    std::vector<std::vector<int32_t>> vitems[2];   // work items of view v, pass p
    int npass[4] = {0, 0, 0, 0};
    size_t out_off[4] = {0, 0, 0, 0};
    size_t out_elems = 0;
    size_t ws_off[4][2] = {};
    size_t ws_bytes = 0;
    std::vector<Launch> launches;    // in level order
    // Adjoint (float plans).  Its gather tables are built on first use (a
    // forward-only caller never pays for them); the pass counts and the
    // workspace layout are known at creation.
    bool adj_view[2] = {false, false};  // lane views with an adjoint
    int adj_npass[2] = {0, 0};          // fused gather passes per lane view
    bool adj_built = false;          // guarded by mu
    fht::AdjointAxis adj[2];         // adjoint steps per lane view
    std::vector<fht::AdjointPass> adjp[2];          // the steps fused into gather passes
    std::vector<size_t> adjp_offs[2], adjp_terms[2];  // where pass p starts in the tables
    size_t adj_ws_off[4][2] = {};
    size_t adj_ws_bytes = 0;
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
        for (int v = 0; v < 2; ++v) {
            if (!view[v]) continue;
            const fht_status st = view[v]->device_progs(&t.views[v]);
            if (st != FHT_OK) return st;
        }
        {
            // one allocation and one copy for all launches (fewer runtime calls)
            std::vector<int32_t> all;
            std::vector<size_t> at;
            for (const Launch &L : launches) {
                at.push_back(all.size());
                all.insert(all.end(), L.items.begin(), L.items.end());
            }
            e = upload(all, &t.items_blob);
            t.bytes += all.size() * sizeof(int32_t);
            for (size_t l = 0; l < launches.size(); ++l)
                t.items.push_back(t.items_blob ? t.items_blob + at[l] : nullptr);
        }
        if (e != hipSuccess) {
            free_tables(t);
            return hip_status(e);
        }
        dev.push_back(t);
        *out = &dev.back();
        return FHT_OK;
    }

    // Device tables already uploaded to device d, or null (never uploads).
    const DevTables *find_tables(int d)
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const DevTables &t : dev)
            if (t.device == d) return &t;
        return nullptr;
    }

    const fht::AxisPlan &ax(int v) const { return view[v]->plan; }

    // The adjoint's host tables (caller holds mu).
    void build_adjoint()
    {
        if (adj_built) return;
        for (int v = 0; v < 2; ++v) {
            if (!adj_view[v]) continue;
            adj[v] = fht::plan_adjoint_axis(v == 0 ? R : C, static_cast<int>(split));
            adjp[v] = fht::fuse_adjoint(adj[v], v == 0 ? C : R, kAdjointFuse);
            size_t ob = 0, tb = 0;
            for (const fht::AdjointPass &ap : adjp[v]) {
                adjp_offs[v].push_back(ob);
                adjp_terms[v].push_back(tb);
                ob += 2 * ap.offs.size() - 1;  // offsets, then the row order
                tb += ap.terms.size() / 2;
            }
        }
        adj_built = true;
    }

    void adjoint_host()
    {
        std::lock_guard<std::mutex> lk(mu);
        build_adjoint();
    }

    // ... and their copy in `t` (device tables of the current device).
    fht_status adjoint_tables(const DevTables *t)
    {
        std::lock_guard<std::mutex> lk(mu);
        build_adjoint();
        DevTables &dt = const_cast<DevTables &>(*t);  // guarded by mu, like its creation
        if (dt.adj_up) return FHT_OK;
        hipError_t e = hipSuccess;
        for (int v = 0; e == hipSuccess && v < 2; ++v) {
            std::vector<int32_t> offs, terms;
            for (const fht::AdjointPass &ap : adjp[v]) {
                offs.insert(offs.end(), ap.offs.begin(), ap.offs.end());
                const std::vector<int32_t> order = gather_order(ap);
                offs.insert(offs.end(), order.begin(), order.end());
                terms.insert(terms.end(), ap.terms.begin(), ap.terms.end());
            }
            e = upload(offs, &dt.adj_offs[v]);
            if (e == hipSuccess) e = upload(terms, &dt.adj_terms[v]);
            dt.bytes += (offs.size() + terms.size()) * sizeof(int32_t);
        }
        if (e != hipSuccess) {
            for (int v = 0; v < 2; ++v) {
                if (dt.adj_offs[v]) (void)hipFree(dt.adj_offs[v]);
                if (dt.adj_terms[v]) (void)hipFree(dt.adj_terms[v]);
                dt.adj_offs[v] = dt.adj_terms[v] = nullptr;
            }
            return hip_status(e);
        }
        dt.adj_up = true;
        return FHT_OK;
    }

    bool narrow(int v, size_t p) const { return ax(v).passes[p].max_root_w <= kNarrowWidth; }

    // Pass p of lane view v runs both quadrants of the view as pairs: uint8
    // images with both quadrants selected, while the pass keeps 16-bit sums
    // and in the pass that outgrows them.
    bool pair_pass(int v, size_t p) const
    {
        return dtype == FHT_U8 && ((qmask >> (2 * v)) & 3u) == 3u &&
               (p == 0 || narrow(v, p) || narrow(v, p - 1));
    }

    // Pass p leaves pair rows (16-bit sums packed in 32 bits) in the workspace.
    bool pair_rows(int v, size_t p) const { return pair_pass(v, p) && (p == 0 || narrow(v, p)); }

    // The job of slot r in its pass `level`; workspace offsets are absolute
    // (ws != null) or relative to the workspace (ws == null, batch tables).
    // Pair rows live in the buffers of the pair's positive-slope quadrant.
    JobDesc job(JobRef r, int level, const void *img, void *out, char *ws, size_t ws_base,
                const DevProgs *const *progs) const
    {
        JobDesc jd;
        std::memset(&jd, 0, sizeof(jd));
        const int q = r.q, v = q >> 1;
        const bool final = level == npass[q] - 1;
        jd.hdrs = progs[v]->hdrs;
        jd.ops = progs[v]->ops;
        int flags = (v ? fht::JF_COLS : 0) | (final ? fht::JF_FINAL : 0);
        if (r.pair)
            flags |= fht::JF_PAIR;
        else if (q & 1)
            flags |= fht::JF_MIRROR;
        auto ws_ptr = [&](int qq, int buf) {
            const size_t off = ws_base + ws_off[qq][buf];
            return ws ? static_cast<void *>(ws + off) : reinterpret_cast<void *>(off);
        };
        if (level == 0) {
            jd.src = img;
        } else {
            jd.src = ws_ptr(pair_rows(v, level - 1) ? (q & ~1) : q, (level - 1) & 1);
            if (!ws) flags |= fht::JF_SRC_WS;
        }
        if (final) {
            jd.dst = static_cast<char *>(out) + out_off[q] * acc_bytes(dtype);
            if (r.pair) jd.dst2 = static_cast<char *>(out) + out_off[q + 1] * acc_bytes(dtype);
        } else if (r.pair && !pair_rows(v, level)) {
            // the pass that outgrows 16 bits splits the pairs into two row sets
            jd.dst = ws_ptr(q, level & 1);
            jd.dst2 = ws_ptr(q + 1, level & 1);
            if (!ws) flags |= fht::JF_DST_WS;
        } else {
            jd.dst = ws_ptr(q, level & 1);
            if (!ws) flags |= fht::JF_DST_WS;
        }
        jd.H = vH[v];
        jd.ld = C;
        jd.flags = flags;
        return jd;
    }
};

// A batch's device work list lives in one table blob: jobs, then the items of
// every launch, each 256-byte aligned (the programs are the lane views').
// The blob is built in host memory; it goes to device memory the library
// allocates (fht_batch_create) or the caller provides (fht_batch_upload).
struct fht_batch_s {
    fht_dtype dtype = FHT_U8;
    int device = -1;
    size_t ws_bytes = 0;
    std::vector<char> blob;
    size_t off_jobs = 0;
    struct Pending {            // a job, made when the device is known
        fht_plan plan;
        JobRef ref;
        int level;
        const void *img;
        void *out;
        size_t ws_base;
    };
    std::vector<Pending> pending;
    std::vector<std::pair<void *, size_t>> images;  // device image and its bytes, per image
    std::vector<size_t> off_items;  // per launch
    char *dev = nullptr;            // device copy of the blob (null until uploaded)
    bool owns = false;              // dev was allocated by the library
    std::vector<Launch> launches;

    ~fht_batch_s()
    {
        if (!owns || !dev) return;
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (device >= 0) (void)hipSetDevice(device);
        (void)hipFree(dev);
        if (have) (void)hipSetDevice(cur);
    }
};

namespace {

bool valid_threads(int t) { return t == 256 || t == 512; }

fht_status make_schedule(const fht_schedule *sched, fht::Schedule *sc)
{
    if (sched) {
        if (sched->s_tile) sc->s_tile = sched->s_tile;
        if (sched->s_tile_first) sc->s_tile_first = sched->s_tile_first;
        if (sched->threads) sc->threads = sched->threads;
        if (sched->threads_first) sc->threads_first = sched->threads_first;
        if (sched->first_levels) sc->first_levels = sched->first_levels;
        if (sched->max_levels) sc->max_levels = sched->max_levels;
        if (sched->lds_budget) sc->lds_budget = sched->lds_budget;
        if (sched->t_tile) sc->t_tile = sched->t_tile < 0 ? 0 : sched->t_tile;
    }
    if (sc->s_tile < fht::kChunk || sc->s_tile > fht::kMaxTarget || sc->s_tile % fht::kChunk ||
        sc->s_tile_first < fht::kChunk || sc->s_tile_first > fht::kMaxTarget ||
        sc->s_tile_first % fht::kChunk || !valid_threads(sc->threads) ||
        !valid_threads(sc->threads_first) || sc->first_levels < 1 ||
        sc->first_levels > fht::kMaxFirstLevels || sc->max_levels < 1 ||
        sc->max_levels > fht::kMaxSteps || sc->lds_budget < 1024 || sc->lds_budget > 163840 ||
        sc->t_tile < 0 || sc->t_tile > 4096)
        return FHT_EINVAL;
    return FHT_OK;
}

// Launch l of the plan for n same-shape images (image b at b strides, in bytes).
fht_status forward_one(fht_plan plan, const DevTables *t, size_t l, const void *d_img,
                       void *d_out, void *d_ws, void *stream, int n = 1, int64_t img_stride = 0,
                       int64_t out_stride = 0)
{
    const Launch &L = plan->launches[l];
    fht::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.items = reinterpret_cast<const int4 *>(t->items[l]);
    a.img_stride = img_stride;
    a.out_stride = out_stride;
    a.ws_stride = static_cast<int64_t>(align_up(plan->ws_bytes, 256));
    for (size_t j = 0; j < L.jobs.size(); ++j)
        a.inl[j] = plan->job(L.jobs[j], L.level, d_img, d_out, static_cast<char *>(d_ws), 0,
                             t->views);
    const int nitems = static_cast<int>(L.items.size() / 4);
    return hip_status(fht::launch_pass(L.combo, a, nitems, L.lds_bytes, L.threads,
                                       static_cast<hipStream_t>(stream), n));
}

fht_status forward_checks(fht_plan plan, const void *d_img, void *d_out, void *d_ws,
                          const DevTables **t)
{
    if (!plan || !d_img || !d_out) return FHT_EINVAL;
    if (plan->ws_bytes && !d_ws) return FHT_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    return plan->tables(t);
}

fht_status batch_one(fht_batch batch, size_t l, void *d_ws, void *stream)
{
    const Launch &L = batch->launches[l];
    fht::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.items = reinterpret_cast<const int4 *>(batch->dev + batch->off_items[l]);
    a.jobs = reinterpret_cast<const JobDesc *>(batch->dev + batch->off_jobs);
    a.ws = static_cast<char *>(d_ws);
    const int nitems = static_cast<int>(L.items.size() / 4);
    return hip_status(fht::launch_pass(L.combo, a, nitems, L.lds_bytes, L.threads,
                                       static_cast<hipStream_t>(stream)));
}

// Fault injection (fht_debug_fail_next): the next `g_fail_count` enqueue calls
// return `g_fail_code` without enqueuing anything.
std::atomic<int> g_fail_count{0};
std::atomic<int> g_fail_code{0};

bool injected_failure(fht_status *st)
{
    int c = g_fail_count.load();
    while (c > 0) {
        if (g_fail_count.compare_exchange_weak(c, c - 1)) {
            *st = static_cast<fht_status>(g_fail_code.load());
            return true;
        }
    }
    return false;
}

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxScratchDevices];  // device d's copy of `scratch`, once looked up

// Address of device d's scratch (d current), looked up on the first call on
// that device.  Allocates nothing.
fht_status scratch_on(int d, void **out)
{
    if (d < 0 || d >= kMaxScratchDevices) return FHT_ENODEV;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[d]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!p) return FHT_EHIP;
        g_scratch_at[d] = p;
    }
    *out = g_scratch_at[d];
    return FHT_OK;
}

// Host half of batch creation: the batch's launches and table blob.  The
// work items go in now; the jobs, which point at each lane view's device
// programs, are written by finish_jobs once the device is known.
void batch_prepare(fht_batch_s *b, const fht_plan *plans, int32_t n, const void *const *d_imgs,
                   void *const *d_outs)
{
    // Batch launches keyed by (level, combination, workgroup size), in level
    // order: plans made with other workgroup sizes (the autotuner picks a
    // schedule per size class) get launches of their own.  A launch takes the
    // largest LDS size of its items.
    std::map<std::tuple<int, int, int>, size_t> key;
    size_t ws = 0;
    for (int i = 0; i < n; ++i) {
        const fht_plan p = plans[i];
        const size_t ws_base = ws;
        ws += align_up(p->ws_bytes, 256);
        for (const Launch &L : p->launches) {
            const auto k = std::make_tuple(L.level, static_cast<int>(L.combo), L.threads);
            auto found = key.find(k);
            if (found == key.end()) {
                found = key.emplace(k, b->launches.size()).first;
                b->launches.emplace_back();
                b->launches.back().level = L.level;
                b->launches.back().combo = L.combo;
                b->launches.back().threads = L.threads;
            }
            Launch &B = b->launches[found->second];
            const int slot0 = static_cast<int>(b->pending.size());
            for (const JobRef &r : L.jobs)
                b->pending.push_back({p, r, L.level, d_imgs[i], d_outs[i], ws_base});
            const size_t at = B.items.size();
            B.items.resize(at + L.items.size());
            int32_t *dst = B.items.data() + at;
            for (size_t k4 = 0; k4 < L.items.size(); k4 += 4) {
                dst[k4] = L.items[k4];
                dst[k4 + 1] = slot0 + L.items[k4 + 1];
                dst[k4 + 2] = L.items[k4 + 2];
                dst[k4 + 3] = L.items[k4 + 3];
            }
            B.lds_bytes = std::max(B.lds_bytes, L.lds_bytes);
        }
    }
    std::stable_sort(b->launches.begin(), b->launches.end(),
                     [](const Launch &x, const Launch &y) { return x.level < y.level; });
    b->ws_bytes = ws;

    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    b->off_jobs = place(b->pending.size() * sizeof(JobDesc));
    for (const Launch &L : b->launches) b->off_items.push_back(place(L.items.size() * sizeof(int32_t)));
    b->blob.resize(std::max<size_t>(off, 256));
    for (size_t l = 0; l < b->launches.size(); ++l) {
        const std::vector<int32_t> &items = b->launches[l].items;
        if (!items.empty())
            std::memcpy(b->blob.data() + b->off_items[l], items.data(), items.size() * sizeof(int32_t));
    }
}

// Writes the batch's jobs into its blob for the current device, uploading the
// lane views' programs there on first use.
fht_status finish_jobs(fht_batch_s *b)
{
    JobDesc *jobs = reinterpret_cast<JobDesc *>(b->blob.data() + b->off_jobs);
    fht_plan last = nullptr;
    const DevProgs *progs[2] = {nullptr, nullptr};
    for (size_t j = 0; j < b->pending.size(); ++j) {
        const fht_batch_s::Pending &pj = b->pending[j];
        if (pj.plan != last) {
            for (int v = 0; v < 2; ++v) {
                progs[v] = nullptr;
                if (!pj.plan->view[v]) continue;
                const fht_status st = pj.plan->view[v]->device_progs(&progs[v]);
                if (st != FHT_OK) return st;
            }
            last = pj.plan;
        }
        const JobDesc jd = pj.plan->job(pj.ref, pj.level, pj.img, pj.out, nullptr, pj.ws_base, progs);
        std::memcpy(jobs + j, &jd, sizeof(jd));
    }
    return FHT_OK;
}

fht_status batch_checks(const fht_plan *plans, int32_t n, const void *const *d_imgs,
                        void *const *d_outs)
{
    if (!plans || !d_imgs || !d_outs || n < 1) return FHT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !d_imgs[i] || !d_outs[i]) return FHT_EINVAL;
    for (int i = 1; i < n; ++i)
        if (plans[i]->dtype != plans[0]->dtype || plans[i]->split != plans[0]->split)
            return FHT_EDTYPE;
    return FHT_OK;
}

}  // namespace

extern "C" {

const char *fht_status_string(int32_t s)
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

fht_status fht_plan_create(fht_plan *out, int32_t rows, int32_t cols, int32_t dtype_arg,
                           int32_t split_arg, uint32_t quadrant_mask, const fht_schedule *sched)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    if (rows < 1 || cols < 1 || rows > 65536 || cols > 65536) return FHT_EINVAL;
    if (quadrant_mask == 0 || quadrant_mask > 15) return FHT_EINVAL;
    if (split_arg != FHT_SPLIT_S && split_arg != FHT_SPLIT_T) return FHT_EINVAL;
    if (dtype_arg != FHT_U8 && dtype_arg != FHT_F32 && dtype_arg != FHT_F64) return FHT_EDTYPE;
    const fht_dtype dtype = static_cast<fht_dtype>(dtype_arg);
    const fht_split split = static_cast<fht_split>(split_arg);
    fht::Schedule sc;
    if (make_schedule(sched, &sc) != FHT_OK) return FHT_EINVAL;

    fht_plan_s *p = new (std::nothrow) fht_plan_s;
    if (!p) return FHT_ENOMEM;
    try {
        p->R = rows;
        p->C = cols;
        p->dtype = dtype;
        p->split = split;
        p->qmask = quadrant_mask;
        p->threads = sc.threads;
        p->threads_first = sc.threads_first;
        const int eb = static_cast<int>(acc_bytes(dtype));
        fht::ElemRule rule;
        rule.narrow_bytes = dtype == FHT_U8 ? 2 : eb;
        rule.wide_bytes = eb;
        rule.narrow_width = dtype == FHT_U8 ? kNarrowWidth : 0;
        for (int v = 0; v < 2; ++v) {
            if (!(quadrant_mask & (3u << (2 * v)))) continue;
            const int W = v == 0 ? rows : cols, H = v == 0 ? cols : rows;
            // both quadrants of a uint8 view run as 16-bit pairs: 4-byte LDS elements
            fht::ElemRule vrule = rule;
            if (dtype == FHT_U8 && ((quadrant_mask >> (2 * v)) & 3u) == 3u) {
                vrule.narrow_bytes = 4;
                vrule.transition_bytes = 8;
            }
            p->view[v] = plan_view(W, H, static_cast<int>(split), vrule, sc, &p->vitems[v]);
            if (!p->view[v]) {
                delete p;
                return FHT_EINVAL;
            }
            p->vW[v] = W;
            p->vH[v] = H;
        }
        // Output and workspace layout (workspace rows are sized for the widest
        // element type any pass stores).
        size_t off = 0, ws = 0;
        int nlevels = 0;
        for (int q = 0; q < 4; ++q) {
            if (!(quadrant_mask & (1u << q))) continue;
            const int v = q >> 1;
            const size_t wh = static_cast<size_t>(p->vW[v]) * p->vH[v];
            p->out_off[q] = off;
            off += wh;
            p->npass[q] = static_cast<int>(p->ax(v).passes.size());
            nlevels = std::max(nlevels, p->npass[q]);
            const int nbuf = std::min(p->npass[q] - 1, 2);
            for (int b = 0; b < nbuf; ++b) {
                p->ws_off[q][b] = ws;
                ws += align_up(wh * eb, 256);
            }
        }
        p->out_elems = off;
        p->ws_bytes = ws;
        // Adjoint steps and their ping-pong buffers (float plans).
        if (dtype != FHT_U8) {
            for (int v = 0; v < 2; ++v) {
                if (!(quadrant_mask & (3u << (2 * v)))) continue;
                // one gather pass per kAdjointFuse levels of the order tree
                p->adj_view[v] = true;
                const int levels = fht::make_tree_height(v == 0 ? rows : cols);
                p->adj_npass[v] = (levels + kAdjointFuse - 1) / kAdjointFuse;
            }
            size_t aws = 0;
            for (int q = 0; q < 4; ++q) {
                if (!(quadrant_mask & (1u << q))) continue;
                const int npass = p->adj_npass[q >> 1];
                const size_t wh = static_cast<size_t>(rows) * cols;
                for (int b = 0; b < std::min(npass, 2); ++b) {
                    p->adj_ws_off[q][b] = aws;
                    aws += align_up(wh * eb, 256);
                }
            }
            p->adj_ws_bytes = aws;
        }
        // Launches: level by level, one per type combination; job slot j of a
        // launch is its j-th quadrant.
        for (int l = 0; l < nlevels; ++l) {
            std::vector<size_t> level_launches;
            for (int q = 0; q < 4; ++q) {
                if (!(quadrant_mask & (1u << q)) || p->npass[q] <= l) continue;
                const int v = q >> 1;
                const bool pair = p->pair_pass(v, l);
                if (pair && (q & 1)) continue;  // run by the pair job of q - 1
                const fht::Pass &ps = p->ax(v).passes[l];
                const std::vector<int32_t> &items = p->vitems[v][l];
                const int prog_base = p->view[v]->prog_base(l);
                const Combo combo = pass_combo(dtype, p->ax(v), l, pair);
                Launch *L = nullptr;
                for (size_t k : level_launches)
                    if (p->launches[k].combo == combo) L = &p->launches[k];
                if (!L) {
                    level_launches.push_back(p->launches.size());
                    p->launches.emplace_back();
                    L = &p->launches.back();
                    L->level = l;
                    L->combo = combo;
                    L->threads = l == 0 ? sc.threads_first : sc.threads;
                    L->kernel = kernel_name(combo, L->threads, false);
                }
                const int job = static_cast<int>(L->jobs.size());
                L->jobs.push_back(JobRef{q, pair});
                L->items.reserve(L->items.size() + items.size());
                for (size_t i = 0; i < items.size(); i += 4) {
                    L->items.push_back(items[i] + prog_base);
                    L->items.push_back(job);
                    L->items.push_back(items[i + 2]);
                    L->items.push_back(p->view[v]->first_entry(l, items[i]));
                }
                L->lds_bytes = std::max(L->lds_bytes, ps.max_lds_elems * ps.elem_bytes);
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
    return plan ? static_cast<int32_t>(plan->launches.size()) : 0;
}

fht_status fht_plan_launch_info(fht_plan plan, int32_t launch, int32_t *level,
                                int64_t *bytes_in, int64_t *bytes_out, int32_t *n_items)
{
    if (!plan || launch < 0 || launch >= static_cast<int32_t>(plan->launches.size()))
        return FHT_EINVAL;
    const Launch &L = plan->launches[launch];
    int in_b = 4, out_b = 4;
    switch (L.combo) {
    case Combo::U8_U16_U16: in_b = 1; out_b = 2; break;
    case Combo::U8_U16_I32: in_b = 1; out_b = 4; break;
    case Combo::U16_U16_U16: in_b = 2; out_b = 2; break;
    case Combo::U16_U16_I32: in_b = 2; out_b = 4; break;
    case Combo::U16_I32_I32: in_b = 2; out_b = 4; break;
    case Combo::I32_I32_I32: in_b = 4; out_b = 4; break;
    case Combo::F32_FIRST: case Combo::F32_LATER: in_b = 4; out_b = 4; break;
    case Combo::F64_FIRST: case Combo::F64_LATER: in_b = 8; out_b = 8; break;
    case Combo::P_U8_FIRST: in_b = 1; out_b = 2; break;
    case Combo::P_U8_FIRST_FINAL: in_b = 1; out_b = 4; break;
    case Combo::P_U16_MID: in_b = 2; out_b = 2; break;
    case Combo::P_U16_MID_FINAL: in_b = 2; out_b = 4; break;
    case Combo::P_I32: in_b = 2; out_b = 4; break;
    }
    int64_t bin = 0, bout = 0;
    bool image_counted = false;
    for (const JobRef &r : L.jobs) {
        const int64_t wh = static_cast<int64_t>(plan->vW[r.q >> 1]) * plan->vH[r.q >> 1];
        for (int c = 0; c < (r.pair ? 2 : 1); ++c) {
            if (L.level == 0) {
                // every quadrant of a launch reads the same image; count it once
                if (!image_counted) bin += static_cast<int64_t>(plan->R) * plan->C * in_b;
                image_counted = true;
            } else {
                bin += wh * in_b;
            }
            bout += wh * out_b;
        }
    }
    if (level) *level = L.level;
    if (bytes_in) *bytes_in = bin;
    if (bytes_out) *bytes_out = bout;
    if (n_items) *n_items = static_cast<int32_t>(L.items.size() / 4);
    return FHT_OK;
}

const char *fht_plan_launch_kernel(fht_plan plan, int32_t launch)
{
    if (!plan || launch < 0 || launch >= static_cast<int32_t>(plan->launches.size())) return nullptr;
    return plan->launches[launch].kernel.c_str();
}

fht_status fht_plan_upload(fht_plan plan)
{
    if (!plan) return FHT_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    const DevTables *t = nullptr;
    return plan->tables(&t);
}

fht_status fht_plan_upload_programs(fht_plan plan)
{
    if (!plan) return FHT_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    for (int v = 0; v < 2; ++v) {
        if (!plan->view[v]) continue;
        const DevProgs *p = nullptr;
        const fht_status st = plan->view[v]->device_progs(&p);
        if (st != FHT_OK) return st;
    }
    return FHT_OK;
}

fht_status fht_plan_upload_programs_many(const fht_plan *plans, int32_t n)
{
    if (n < 0 || (n > 0 && !plans)) return FHT_EINVAL;
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i]) return FHT_EINVAL;
    int count = 0, d = -1;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return FHT_ENODEV;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_status(e);
    try {
        // distinct lane views without a copy on this device
        std::vector<std::shared_ptr<ViewProgs>> views;
        for (int32_t i = 0; i < n; ++i)
            for (int v = 0; v < 2; ++v) {
                const std::shared_ptr<ViewProgs> &vp = plans[i]->view[v];
                if (vp && std::find(views.begin(), views.end(), vp) == views.end() &&
                    !vp->on_device(d))
                    views.push_back(vp);
            }
        if (views.empty()) return FHT_OK;
        // every view's image (256-byte aligned) in one allocation, written
        // through the staging buffers in one pass
        std::vector<size_t> n_ops(views.size()), off(views.size());
        size_t total = 0;
        for (size_t k = 0; k < views.size(); ++k) {
            off[k] = total;
            total += align_up(views[k]->image_ints() * sizeof(int32_t), 256);
        }
        void *block = nullptr;
        e = hipMalloc(&block, total);
        if (e != hipSuccess) return hip_status(e);
        const std::shared_ptr<void> mem = device_block(block, d, total);
        {
            CopyLane &L = copy_lane(d);
            std::lock_guard<std::mutex> lk(L.mu);
            if ((e = L.init()) != hipSuccess) return hip_status(e);
            StagedSink out{L, static_cast<char *>(block)};
            for (size_t k = 0; k < views.size(); ++k) {
                out.pad_to(256);
                views[k]->write_image(out, &n_ops[k]);
            }
            if ((e = out.finish()) != hipSuccess) return hip_status(e);
        }
        for (size_t k = 0; k < views.size(); ++k)
            views[k]->adopt(d, reinterpret_cast<int32_t *>(static_cast<char *>(block) + off[k]),
                            n_ops[k], mem);
    } catch (const std::bad_alloc &) {
        return FHT_ENOMEM;
    }
    return FHT_OK;
}

fht_status fht_forward(fht_plan plan, const void *d_img, void *d_out, void *d_ws, void *stream)
{
    const DevTables *t = nullptr;
    fht_status st = forward_checks(plan, d_img, d_out, d_ws, &t);
    if (st == FHT_OK && injected_failure(&st)) return st;
    for (size_t l = 0; st == FHT_OK && l < plan->launches.size(); ++l)
        st = forward_one(plan, t, l, d_img, d_out, d_ws, stream);
    return st;
}

fht_status fht_forward_noalloc(fht_plan plan, const void *d_img, void *d_out, void *stream)
{
    if (!plan || !d_img || !d_out) return FHT_EINVAL;
    if (plan->ws_bytes > FHT_NOALLOC_WS_BYTES) return FHT_EINVAL;
    int n = 0, d = -1;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return FHT_ENODEV;
    const hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_status(e);
    const DevTables *t = plan->find_tables(d);
    if (!t) return FHT_EINVAL;  // tables not on this device: fht_plan_upload allocates them
    void *ws = nullptr;
    fht_status st = FHT_OK;
    if (plan->ws_bytes) st = scratch_on(d, &ws);
    if (st == FHT_OK && injected_failure(&st)) return st;
    // every workspace element is written before it is read: nothing to clear
    for (size_t l = 0; st == FHT_OK && l < plan->launches.size(); ++l)
        st = forward_one(plan, t, l, d_img, d_out, ws, stream);
    return st;
}

size_t fht_plan_workspace_bytes_many(fht_plan plan, int32_t n)
{
    if (!plan || n < 1) return 0;
    return plan->ws_bytes ? static_cast<size_t>(n) * align_up(plan->ws_bytes, 256) : 0;
}

fht_status fht_forward_many(fht_plan plan, int32_t n, const void *d_imgs, int64_t img_stride,
                            void *d_outs, int64_t out_stride, void *d_ws, void *stream)
{
    if (n < 1 || n > 65535 || img_stride < 0 || out_stride < 0) return FHT_EINVAL;
    const DevTables *t = nullptr;
    fht_status st = forward_checks(plan, d_imgs, d_outs, d_ws, &t);
    if (st == FHT_OK && injected_failure(&st)) return st;
    for (size_t l = 0; st == FHT_OK && l < plan->launches.size(); ++l)
        st = forward_one(plan, t, l, d_imgs, d_outs, d_ws, stream, n, img_stride, out_stride);
    return st;
}

fht_status fht_forward_launch(fht_plan plan, int32_t launch, const void *d_img, void *d_out,
                              void *d_ws, void *stream)
{
    const DevTables *t = nullptr;
    fht_status st = forward_checks(plan, d_img, d_out, d_ws, &t);
    if (st != FHT_OK) return st;
    if (launch < 0 || launch >= static_cast<int32_t>(plan->launches.size())) return FHT_EINVAL;
    if (injected_failure(&st)) return st;
    return forward_one(plan, t, static_cast<size_t>(launch), d_img, d_out, d_ws, stream);
}

fht_status fht_batch_prepare(fht_batch *out, const fht_plan *plans, int32_t n,
                             const void *const *d_imgs, void *const *d_outs)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    const fht_status st = batch_checks(plans, n, d_imgs, d_outs);
    if (st != FHT_OK) return st;
    fht_batch_s *b = new (std::nothrow) fht_batch_s;
    if (!b) return FHT_ENOMEM;
    b->dtype = plans[0]->dtype;
    try {
        batch_prepare(b, plans, n, d_imgs, d_outs);
        const size_t px_bytes = b->dtype == FHT_U8 ? 1 : acc_bytes(b->dtype);
        for (int32_t i = 0; i < n; ++i)
            b->images.emplace_back(const_cast<void *>(d_imgs[i]),
                                   static_cast<size_t>(plans[i]->R) * plans[i]->C * px_bytes);
    } catch (const std::bad_alloc &) {
        delete b;
        return FHT_ENOMEM;
    }
    *out = b;
    return FHT_OK;
}

fht_status fht_batch_copy_images(fht_batch batch, const void *const *srcs, void *stream)
{
    if (!batch || !srcs) return FHT_EINVAL;
    for (size_t i = 0; i < batch->images.size(); ++i) {
        if (!srcs[i]) continue;
        const hipError_t e = hipMemcpyAsync(batch->images[i].first, srcs[i], batch->images[i].second,
                                            hipMemcpyDefault, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_status(e);
    }
    return FHT_OK;
}

size_t fht_batch_tables_bytes(fht_batch batch) { return batch ? batch->blob.size() : 0; }

fht_status fht_batch_upload(fht_batch batch, void *d_tables, size_t bytes, void *stream)
{
    if (!batch || !d_tables || bytes < batch->blob.size() || batch->owns) return FHT_EINVAL;
    fht_status st = FHT_OK;
    if (injected_failure(&st)) return st;
    hipError_t e = hipGetDevice(&batch->device);
    if (e != hipSuccess) return hip_status(e);
    st = finish_jobs(batch);
    if (st != FHT_OK) return st;
    e = hipMemcpyAsync(d_tables, batch->blob.data(), batch->blob.size(), hipMemcpyHostToDevice,
                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_status(e);
    batch->dev = static_cast<char *>(d_tables);
    return FHT_OK;
}

fht_status fht_batch_upload_staged(fht_batch batch, void *d_tables, size_t bytes, void *h_staging,
                                   void *stream)
{
    if (!batch || !d_tables || !h_staging || bytes < batch->blob.size() || batch->owns)
        return FHT_EINVAL;
    fht_status st = FHT_OK;
    if (injected_failure(&st)) return st;
    hipError_t e = hipGetDevice(&batch->device);
    if (e != hipSuccess) return hip_status(e);
    st = finish_jobs(batch);
    if (st != FHT_OK) return st;
    std::memcpy(h_staging, batch->blob.data(), batch->blob.size());
    e = hipMemcpyAsync(d_tables, h_staging, batch->blob.size(), hipMemcpyHostToDevice,
                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_status(e);
    batch->dev = static_cast<char *>(d_tables);
    return FHT_OK;
}

fht_status fht_batch_create(fht_batch *out, const fht_plan *plans, int32_t n,
                            const void *const *d_imgs, void *const *d_outs)
{
    if (!out) return FHT_EINVAL;
    *out = nullptr;
    fht_status st = batch_checks(plans, n, d_imgs, d_outs);
    if (st != FHT_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return FHT_ENODEV;
    fht_batch b = nullptr;
    st = fht_batch_prepare(&b, plans, n, d_imgs, d_outs);
    if (st != FHT_OK) return st;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) {
        st = finish_jobs(b);
        if (st != FHT_OK) {
            delete b;
            return st;
        }
    }
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&b->dev), b->blob.size());
    if (e == hipSuccess) {
        b->owns = true;
        e = hipMemcpy(b->dev, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        delete b;
        return hip_status(e);
    }
    *out = b;
    return FHT_OK;
}

size_t fht_batch_workspace_bytes(fht_batch batch) { return batch ? batch->ws_bytes : 0; }

int32_t fht_batch_num_launches(fht_batch batch)
{
    return batch ? static_cast<int32_t>(batch->launches.size()) : 0;
}

fht_status fht_batch_run(fht_batch batch, void *d_ws, void *stream)
{
    if (!batch || !batch->dev) return FHT_EINVAL;
    if (batch->ws_bytes && !d_ws) return FHT_EINVAL;
    fht_status st = FHT_OK;
    if (injected_failure(&st)) return st;
    for (size_t l = 0; st == FHT_OK && l < batch->launches.size(); ++l)
        st = batch_one(batch, l, d_ws, stream);
    return st;
}

fht_status fht_batch_run_launch(fht_batch batch, int32_t launch, void *d_ws, void *stream)
{
    if (!batch || !batch->dev) return FHT_EINVAL;
    if (batch->ws_bytes && !d_ws) return FHT_EINVAL;
    if (launch < 0 || launch >= static_cast<int32_t>(batch->launches.size())) return FHT_EINVAL;
    fht_status st = FHT_OK;
    if (injected_failure(&st)) return st;
    return batch_one(batch, static_cast<size_t>(launch), d_ws, stream);
}

void fht_batch_destroy(fht_batch batch) { delete batch; }

fht_status fht_plan_work(fht_plan plan, int64_t *adds_tree, int64_t *adds_executed)
{
    if (!plan) return FHT_EINVAL;
    int64_t tree = 0, done = 0;
    for (int q = 0; q < 4; ++q) {
        if (!(plan->qmask & (1u << q))) continue;
        const int v = q >> 1;
        const fht::AxisPlan &ax = plan->ax(v);
        // Theorem 1's count: every non-leaf node of width w merges w rows of H
        const fht::Tree tr = fht::make_tree(plan->vW[v], ax.split);
        for (const fht::Node &n : tr.nodes)
            if (n.w > 1) tree += static_cast<int64_t>(n.w) * plan->vH[v];
        // what the kernels add: whole 64-position chunks of every merge entry
        for (size_t p = 0; p < ax.passes.size(); ++p) {
            const fht::Pass &ps = ax.passes[p];
            const std::vector<int32_t> &items = plan->vitems[v][p];
            for (size_t i = 0; i < items.size(); i += 4) {
                const int32_t *h = ps.hdrs.data() + static_cast<size_t>(items[i]) * fht::kHdrInts;
                int64_t merges = 0;
                for (int k = 0; k < h[fht::kHdrSteps]; ++k) merges += h[fht::kHdrStepCounts + k];
                if (h[fht::kHdrStoreMerge]) merges += h[fht::kHdrStores];  // stores that add
                merges += h[fht::kHdrLoadMerges];
                done += merges * h[fht::kHdrChunks] * fht::kChunk;
            }
        }
    }
    if (adds_tree) *adds_tree = tree;
    if (adds_executed) *adds_executed = done;
    return FHT_OK;
}

size_t fht_plan_adjoint_workspace_bytes(fht_plan plan) { return plan ? plan->adj_ws_bytes : 0; }

int32_t fht_plan_adjoint_num_passes(fht_plan plan, int32_t v)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v))) || plan->dtype == FHT_U8)
        return -1;
    return plan->adj_npass[v];
}

fht_status fht_plan_adjoint_pass(fht_plan plan, int32_t v, int32_t pass, int32_t *levels,
                                 const int32_t **offs, const int32_t **terms, int32_t *n_terms)
{
    if (fht_plan_adjoint_num_passes(plan, v) <= pass || pass < 0) return FHT_EINVAL;
    plan->adjoint_host();
    const fht::AdjointPass &ap = plan->adjp[v][pass];
    if (levels) *levels = ap.levels;
    if (offs) *offs = ap.offs.data();
    if (terms) *terms = ap.terms.data();
    if (n_terms) *n_terms = static_cast<int32_t>(ap.terms.size() / 2);
    return FHT_OK;
}

fht_status fht_plan_adjoint_tasks(fht_plan plan, int32_t v, const int32_t **tasks,
                                  int32_t *levels, int32_t *lanes)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v)))) return FHT_EINVAL;
    if (plan->dtype == FHT_U8) return FHT_EDTYPE;
    plan->adjoint_host();
    const fht::AdjointAxis &ax = plan->adj[v];
    if (tasks) *tasks = ax.tasks.data();
    if (levels) *levels = ax.levels;
    if (lanes) *lanes = ax.W;
    return FHT_OK;
}

size_t fht_plan_adjoint_workspace_bytes_many(fht_plan plan, int32_t n)
{
    if (!plan || n < 1) return 0;
    return plan->adj_ws_bytes ? static_cast<size_t>(n) * align_up(plan->adj_ws_bytes, 256) : 0;
}

fht_status fht_adjoint_many(fht_plan plan, int32_t n, const void *d_gouts, int64_t gout_stride,
                            void *d_gimgs, int64_t gimg_stride, void *d_ws, void *stream)
{
    if (!plan || !d_gouts || !d_gimgs) return FHT_EINVAL;
    if (n < 1 || n > 65535 || gout_stride < 0 || gimg_stride < 0) return FHT_EINVAL;
    if (plan->dtype == FHT_U8) return FHT_EDTYPE;
    if (plan->adj_ws_bytes && !d_ws) return FHT_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return FHT_ENODEV;
    const DevTables *t = nullptr;
    fht_status st = plan->tables(&t);
    if (st != FHT_OK) return st;
    if (injected_failure(&st)) return st;
    st = plan->adjoint_tables(t);
    if (st != FHT_OK) return st;
    const fht::Real real = plan->dtype == FHT_F64 ? fht::Real::F64 : fht::Real::F32;
    const size_t eb = acc_bytes(plan->dtype);
    const int64_t ws_stride = static_cast<int64_t>(align_up(plan->adj_ws_bytes, 256));
    hipStream_t hs = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(d_ws);
    const char *gout = static_cast<const char *>(d_gouts);
    // Every quadrant's passes but its last run as gather launches; the last
    // ones run in the final launch, which also sums into the image gradient,
    // when its 64 x 64 tiles give every compute unit one; otherwise the last
    // gathers run as their own launch and a combine launch adds up.
    int max_passes = 0;
    for (int q = 0; q < 4; ++q)
        if (plan->qmask & (1u << q))
            max_passes = std::max(max_passes, plan->adj_npass[q >> 1]);
    const int64_t tiles = static_cast<int64_t>((plan->R + 63) / 64) * ((plan->C + 63) / 64) * n;
    const bool fuse_last = tiles >= kFinalMinTiles;
    const int gathers = fuse_last ? max_passes - 1 : max_passes;
    for (int k = 0; k < gathers; ++k) {
        fht::AdjArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src_stride = k == 0 ? gout_stride : ws_stride;
        a.dst_stride = ws_stride;
        int nj = 0, max_w = 0, max_h = 0;
        for (int q = 0; q < 4; ++q) {
            if (!(plan->qmask & (1u << q))) continue;
            const int v = q >> 1;
            const fht::AdjointAxis &ax = plan->adj[v];
            if (plan->adj_npass[v] <= (fuse_last ? k + 1 : k)) continue;
            fht::AdjJob &j = a.job[nj++];
            j.src = k == 0 ? static_cast<const void *>(gout + plan->out_off[q] * eb)
                           : static_cast<const void *>(ws + plan->adj_ws_off[q][(k - 1) & 1]);
            j.dst = ws + plan->adj_ws_off[q][k & 1];
            j.offs = t->adj_offs[v] + plan->adjp_offs[v][k];
            j.order = j.offs + ax.W + 1;
            j.terms = reinterpret_cast<const int2 *>(t->adj_terms[v]) + plan->adjp_terms[v][k];
            j.W = ax.W;
            j.H = (q >> 1) ? plan->R : plan->C;
            j.mirror_in = (k == 0 && (q & 1)) ? 1 : 0;
            max_w = std::max(max_w, ax.W);
            max_h = std::max(max_h, j.H);
        }
        const hipError_t e = fht::launch_adjoint_step(real, a, nj, max_w, hs, n, max_h);
        if (e != hipSuccess) return hip_status(e);
    }
    if (!fuse_last) {
        fht::CombineArgs c;
        std::memset(&c, 0, sizeof(c));
        c.R = plan->R;
        c.C = plan->C;
        c.dst = d_gimgs;
        c.dst_stride = gimg_stride;
        for (int q = 0; q < 4; ++q) {
            if (!(plan->qmask & (1u << q))) continue;
            const int L = plan->adj_npass[q >> 1];
            // after the steps a negative-slope quadrant is in the mirrored frame
            c.src[q] = L > 0 ? static_cast<const void *>(ws + plan->adj_ws_off[q][(L - 1) & 1])
                             : static_cast<const void *>(gout + plan->out_off[q] * eb);
            c.src_stride[q] = L > 0 ? ws_stride : gout_stride;
            c.mirror[q] = (L > 0 && (q & 1)) ? 1 : 0;
        }
        return hip_status(fht::launch_adjoint_combine(real, c, hs, n));
    }
    fht::FinalArgs c;
    std::memset(&c, 0, sizeof(c));
    c.R = plan->R;
    c.C = plan->C;
    c.dst = d_gimgs;
    c.dst_stride = gimg_stride;
    for (int q = 0; q < 4; ++q) {
        if (!(plan->qmask & (1u << q))) continue;
        const int v = q >> 1;
        const int L = plan->adj_npass[v];
        fht::FinalJob &f = c.q[q];
        if (L == 0) {  // no tree levels: the lane gradient is the output gradient
            f.src = gout + plan->out_off[q] * eb;
            f.src_stride = gout_stride;
            continue;
        }
        // pass L - 1 reads the output gradient (L = 1, at mirrored positions
        // for negative slopes) or the rows pass L - 2 wrote
        f.src = L == 1 ? static_cast<const void *>(gout + plan->out_off[q] * eb)
                       : static_cast<const void *>(ws + plan->adj_ws_off[q][(L - 2) & 1]);
        f.src_stride = L == 1 ? gout_stride : ws_stride;
        f.offs = t->adj_offs[v] + plan->adjp_offs[v][L - 1];
        f.terms = reinterpret_cast<const int2 *>(t->adj_terms[v]) + plan->adjp_terms[v][L - 1];
        f.in_mirror = (L == 1 && (q & 1)) ? 1 : 0;
        // after its passes a negative-slope quadrant is in the mirrored frame
        f.out_mirror = (q & 1) ? 1 : 0;
    }
    return hip_status(fht::launch_adjoint_final(real, c, hs, n));
}

fht_status fht_adjoint(fht_plan plan, const void *d_gout, void *d_gimg, void *d_ws, void *stream)
{
    return fht_adjoint_many(plan, 1, d_gout, 0, d_gimg, 0, d_ws, stream);
}

size_t fht_peaks_workspace_bytes(int32_t capacity)
{
    if (capacity < 1) return 0;
    return 256 + static_cast<size_t>(capacity) * sizeof(uint64_t);
}

fht_status fht_peaks(fht_plan plan, const void *d_out, int32_t k, int32_t radius,
                     double min_value, int32_t capacity, void *d_ws, fht_peak *d_peaks,
                     int32_t *d_found, void *stream)
{
    if (!plan || !d_out || !d_ws || !d_peaks || !d_found) return FHT_EINVAL;
    if (k < 1 || k > 4096 || radius < 0 || radius > 64 || capacity < k || capacity > (1 << 26))
        return FHT_EINVAL;
    if (plan->out_elems >= 0xffffffffull) return FHT_EINVAL;
    static_assert(sizeof(fht_peak) == sizeof(fht::PeakOut), "peak layout");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return FHT_ENODEV;
    fht_status st = FHT_OK;
    if (injected_failure(&st)) return st;
    fht::PeakArgs a;
    std::memset(&a, 0, sizeof(a));
    const size_t eb = acc_bytes(plan->dtype);
    size_t max_elems = 0;
    for (int q = 0; q < 4; ++q) {
        if (!(plan->qmask & (1u << q))) continue;
        const int v = q >> 1;
        const int j = a.nq++;
        a.src[j] = static_cast<const char *>(d_out) + plan->out_off[q] * eb;
        a.W[j] = plan->vW[v];
        a.H[j] = plan->vH[v];
        a.base[j] = plan->out_off[q];
        a.quadrant[j] = q;
        max_elems = std::max(max_elems, static_cast<size_t>(plan->vW[v]) * plan->vH[v]);
    }
    a.radius = radius;
    a.min_value = min_value;
    a.k = k;
    a.capacity = capacity;
    a.counter = static_cast<uint32_t *>(d_ws);
    a.keys = reinterpret_cast<uint64_t *>(static_cast<char *>(d_ws) + 256);
    a.flat = d_out;
    a.out = reinterpret_cast<fht::PeakOut *>(d_peaks);
    a.n_found = d_found;
    const fht::PeakElem elem = plan->dtype == FHT_U8    ? fht::PeakElem::I32
                               : plan->dtype == FHT_F32 ? fht::PeakElem::F32
                                                        : fht::PeakElem::F64;
    return hip_status(fht::launch_peaks(elem, a, max_elems, static_cast<hipStream_t>(stream)));
}

void fht_debug_fail_next(int32_t code, int32_t count)
{
    g_fail_code.store(code);
    g_fail_count.store(count > 0 && code != FHT_OK ? count : 0);
}

int32_t fht_plan_num_passes(fht_plan plan, int32_t v)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v)))) return -1;
    return static_cast<int32_t>(plan->ax(v).passes.size());
}

fht_status fht_plan_pass_tables(fht_plan plan, int32_t v, int32_t pass, const int32_t **hdrs,
                                int32_t *n_progs, const int32_t **ops, int32_t *n_ops,
                                const int32_t **items, int32_t *n_items, int32_t *s_tile)
{
    if (!plan || v < 0 || v > 1 || !(plan->qmask & (3u << (2 * v)))) return FHT_EINVAL;
    const fht::AxisPlan &ax = plan->ax(v);
    if (pass < 0 || pass >= static_cast<int32_t>(ax.passes.size())) return FHT_EINVAL;
    const fht::Pass &ps = ax.passes[pass];
    const std::vector<int32_t> &its = plan->vitems[v][pass];
    if (hdrs) *hdrs = ps.hdrs.data();
    if (n_progs) *n_progs = static_cast<int32_t>(ps.hdrs.size() / fht::kHdrInts);
    if (ops) *ops = ps.ops.data();
    if (n_ops) *n_ops = static_cast<int32_t>(ps.ops.size() / 4);
    if (items) *items = its.data();
    if (n_items) *n_items = static_cast<int32_t>(its.size() / 4);
    if (s_tile) *s_tile = ps.S;
    return FHT_OK;
}

}  // extern "C"
