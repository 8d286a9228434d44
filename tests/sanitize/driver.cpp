// Host-side exercise of libfht's C ABI for the sanitizer builds (AddressSanitizer
// + UndefinedBehaviorSanitizer, and ThreadSanitizer): plan creation for many
// shapes, dtypes, splits, quadrant masks and schedules (and rejected
// arguments), every host-side query, batches prepared in host memory, the
// planner pool fed and polled from several threads, and fault injection from
// several threads.  No device is needed or touched: the pool runs with device
// -1 and nothing is uploaded.  Exit status 0 means every check held; the
// sanitizers abort the process on a finding.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "fht.h"

namespace {

int g_fail = 0;

void check(bool ok, const char *what, int a = 0, int b = 0)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s (%d, %d)\n", what, a, b);
        ++g_fail;
    }
}

void queries(fht_plan p, int R, int C)
{
    const size_t n = fht_plan_out_elems(p);
    size_t sum = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t off = fht_plan_out_offset(p, q);
        if (off >= 0) sum += static_cast<size_t>(R) * C;
    }
    check(sum == n, "out elems", R, C);
    (void)fht_plan_workspace_bytes(p);
    (void)fht_plan_workspace_bytes_many(p, 3);
    const int nl = fht_plan_num_launches(p);
    for (int l = 0; l < nl; ++l) {
        int32_t level = 0, items = 0;
        int64_t bi = 0, bo = 0;
        check(fht_plan_launch_info(p, l, &level, &bi, &bo, &items) == FHT_OK, "launch info", l);
        check(fht_plan_launch_kernel(p, l) != nullptr, "launch kernel", l);
    }
    check(fht_plan_launch_info(p, nl, nullptr, nullptr, nullptr, nullptr) == FHT_EINVAL,
          "launch info past the end");
    int64_t tree = 0, exec = 0;
    check(fht_plan_work(p, &tree, &exec) == FHT_OK && exec >= tree, "work");
    for (int v = 0; v < 2; ++v) {
        const int np = fht_plan_num_passes(p, v);
        for (int k = 0; k < np; ++k) {
            const int32_t *h, *o, *it;
            int32_t nh, no, ni, s;
            check(fht_plan_pass_tables(p, v, k, &h, &nh, &o, &no, &it, &ni, &s) == FHT_OK,
                  "pass tables", v, k);
            // touch every entry (reads past a table's end show up here)
            long acc = 0;
            for (int i = 0; i < nh * FHT_HDR_INTS; ++i) acc += h[i];
            for (int i = 0; i < no * 4; ++i) acc += o[i];
            for (int i = 0; i < ni * 4; ++i) acc += it[i];
            check(acc != 0x7fffffff, "tables");
        }
        const int na = fht_plan_adjoint_num_passes(p, v);
        for (int k = 0; k < na; ++k) {
            int32_t lv = 0, nt = 0;
            const int32_t *offs, *terms;
            if (fht_plan_adjoint_pass(p, v, k, &lv, &offs, &terms, &nt) == FHT_OK) {
                long acc = 0;
                for (int i = 0; i < nt * 2; ++i) acc += terms[i];
                check(acc >= 0, "adjoint terms");
            }
        }
        const int32_t *tasks;
        int32_t lv = 0, lanes = 0;
        if (fht_plan_adjoint_tasks(p, v, &tasks, &lv, &lanes) == FHT_OK) {
            long acc = 0;
            for (int i = 0; i < lv * lanes * 4; ++i) acc += tasks[i];
            check(acc >= 0, "adjoint tasks");
        }
    }
}

void plans_and_batches()
{
    const int shapes[][2] = {{1, 1}, {1, 9}, {9, 1}, {2, 3}, {61, 47}, {257, 70}, {300, 513},
                             {1021, 17}, {5, 4096}, {4097, 3}, {20000, 2}};
    fht_schedule scheds[3] = {{0, 0, 0, 0, 0, 0, 0, 0},
                              {64, 2, 2, 8192, 0, 64, 256, 256},
                              {256, 6, 7, 65536, 8, 64, 512, 512}};
    std::vector<fht_plan> keep;
    for (const auto &sh : shapes)
        for (int dt = 0; dt < 3; ++dt)
            for (int split = 0; split < 2; ++split)
                for (int si = 0; si < 3; ++si) {
                    const uint32_t mask = (si == 1) ? 5u : (si == 2 ? 10u : 15u);
                    fht_plan p = nullptr;
                    const fht_status st = fht_plan_create(&p, sh[0], sh[1], dt,
                                                          split, mask,
                                                          si ? &scheds[si] : nullptr);
                    check(st == FHT_OK, "plan create", sh[0], sh[1]);
                    if (st != FHT_OK) continue;
                    queries(p, sh[0], sh[1]);
                    if (dt == 0 && split == 0 && si == 0) keep.push_back(p);
                    else fht_plan_destroy(p);
                }
    // rejected arguments
    fht_plan p = nullptr;
    check(fht_plan_create(&p, 0, 5, FHT_U8, FHT_SPLIT_S, 15, nullptr) == FHT_EINVAL, "rows 0");
    check(fht_plan_create(&p, 5, 70000, FHT_U8, FHT_SPLIT_S, 15, nullptr) == FHT_EINVAL, "cols");
    check(fht_plan_create(&p, 5, 5, 9, FHT_SPLIT_S, 15, nullptr) ==
              FHT_EDTYPE, "dtype");
    check(fht_plan_create(&p, 5, 5, FHT_U8, FHT_SPLIT_S, 16, nullptr) == FHT_EINVAL, "mask");
    check(fht_plan_create(&p, 5, 5, FHT_U8, 7, 15, nullptr) == FHT_EINVAL, "split");
    check(fht_plan_create(&p, 5, 5, -3, FHT_SPLIT_S, 15, nullptr) == FHT_EDTYPE, "dtype < 0");
    fht_schedule bad{96, 0, 0, 0, 0, 0, 0, 0};
    check(fht_plan_create(&p, 5, 5, FHT_U8, FHT_SPLIT_S, 15, &bad) == FHT_EINVAL, "schedule");
    check(p == nullptr, "no plan on failure");
    // batches in host memory (no upload): fake device addresses are only stored
    std::vector<const void *> imgs;
    std::vector<void *> outs;
    for (size_t i = 0; i < keep.size(); ++i) {
        imgs.push_back(reinterpret_cast<const void *>(0x100000 * (i + 1)));
        outs.push_back(reinterpret_cast<void *>(0x40000000 + 0x100000 * (i + 1)));
    }
    fht_batch b = nullptr;
    check(fht_batch_prepare(&b, keep.data(), static_cast<int32_t>(keep.size()), imgs.data(),
                            outs.data()) == FHT_OK, "batch prepare");
    if (b) {
        check(fht_batch_tables_bytes(b) > 0, "tables bytes");
        check(fht_batch_num_launches(b) > 0, "batch launches");
        (void)fht_batch_workspace_bytes(b);
        check(fht_batch_run(b, nullptr, nullptr) != FHT_OK, "run before upload fails");
        fht_batch_destroy(b);
    }
    check(fht_batch_prepare(&b, keep.data(), 0, imgs.data(), outs.data()) == FHT_EINVAL, "empty");
    for (fht_plan q : keep) fht_plan_destroy(q);
    fht_plan_destroy(nullptr);
    fht_batch_destroy(nullptr);
}

void planner_pool(int threads, int submitters, int per_thread)
{
    fht_planner pool = nullptr;
    check(fht_planner_create(threads, -1, &pool) == FHT_OK, "pool create");
    if (!pool) return;
    std::atomic<int> made{0}, failed{0};
    std::vector<std::thread> th;
    for (int k = 0; k < submitters; ++k)
        th.emplace_back([&, k] {
            std::mt19937 rng(1234 + k);
            std::vector<int64_t> tickets;
            for (int i = 0; i < per_thread; ++i) {
                const int R = 1 + static_cast<int>(rng() % 700), C = 1 + static_cast<int>(rng() % 700);
                const int rows = (i % 9 == 8) ? -1 : R;  // some bad requests
                int64_t t = -1;
                if (fht_planner_submit(pool, rows, C, i % 3,
                                       i & 1, 15, nullptr, &t) == FHT_OK)
                    tickets.push_back(t);
            }
            // poll half of them to completion; leave the rest to destroy
            for (size_t i = 0; i < tickets.size() / 2; ++i) {
                fht_plan p = nullptr;
                fht_status st = FHT_OK;
                int r;
                while ((r = fht_planner_poll(pool, tickets[i], &p, &st)) == 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                check(r == 1, "poll");
                if (st == FHT_OK) {
                    ++made;
                    fht_plan_destroy(p);
                } else {
                    ++failed;
                    check(p == nullptr, "failed plan is null");
                }
                check(fht_planner_poll(pool, tickets[i], &p, &st) == -1, "ticket forgotten");
            }
        });
    for (auto &t : th) t.join();
    check(made > 0 && failed > 0, "pool made and rejected plans", made, failed);
    fht_planner_destroy(pool);  // frees what no poll took
}

void fault_injection_threads()
{
    std::vector<std::thread> th;
    for (int k = 0; k < 4; ++k)
        th.emplace_back([k] {
            for (int i = 0; i < 2000; ++i) {
                fht_debug_fail_next(-4, (i + k) % 3);
                (void)fht_status_string(-(i % 9));
            }
        });
    for (auto &t : th) t.join();
    fht_debug_fail_next(FHT_OK, 0);
}

}  // namespace

int main()
{
    plans_and_batches();
    planner_pool(8, 4, 60);
    planner_pool(1, 2, 20);
    fault_injection_threads();
    // a pool destroyed at once, with its queue full
    fht_planner pool = nullptr;
    if (fht_planner_create(4, -1, &pool) == FHT_OK) {
        int64_t t;
        for (int i = 0; i < 200; ++i)
            fht_planner_submit(pool, 300 + i, 200, FHT_U8, FHT_SPLIT_S, 15, nullptr, &t);
        fht_planner_destroy(pool);
    }
    std::printf("sanitizer driver: %s\n", g_fail ? "FAILED" : "ok");
    return g_fail ? 1 : 0;
}
