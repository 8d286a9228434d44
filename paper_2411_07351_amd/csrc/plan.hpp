// Host-side planner: the computation-order tree of Alg. 1 and the fused-pass
// tile programs the gfx950 kernels execute.  Pure C++, no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fht {

constexpr int kHdrInts = 32;     // ints per tile-program header
constexpr int kMaxSteps = 24;    // header slots for per-step op counts (8 + k < 32)

// [.] of Alg. 1: nearest integer to num / den (num >= 0, den > 0), ties to even.
int64_t round_half_even(int64_t num, int64_t den);

// Left width of Split(w) (Sec. 3): floor(w/2) for Split_S, the largest power
// of two below w for Split_T.
int split_left(int w, int split);

// A node of the computation-order tree G (proof of Theorem 1): the lane range
// [a, a + w) with children Split(w); height = ceil(log2 w).
struct Node {
    int a = 0, w = 1, w0 = 0;
    int left = -1, right = -1;
    int height = 0;
};

struct Tree {
    int W = 0, split = 0;
    std::vector<Node> nodes;  // nodes[0] is the root
};

Tree make_tree(int W, int split);

struct Schedule {
    int s_tile = 128;
    int first_levels = 5;
    int max_levels = 6;
    int lds_budget = 64 * 1024;
    int t_tile = 0;           // 0: try 64, 32, 16, 8
};

// One fused pass: from the frontier of level lin (maximal nodes of height
// <= lin) to the frontier of level lout.
struct Pass {
    int lin = 0, lout = 0;
    int t_tile = 0;
    int max_lds_elems = 0;
    std::vector<int32_t> hdrs;   // kHdrInts per program
    std::vector<int32_t> ops;    // 4 per op
    std::vector<int32_t> items;  // 4 per work item
};

struct AxisPlan {
    int W = 0, H = 0, split = 0, S = 0;
    std::vector<Pass> passes;
};

// Plans the passes for W lanes of H positions.  elem_bytes is the size of the
// accumulator element (4 or 8).  Returns false and sets *err on failure.
bool plan_axis(int W, int H, int split, int elem_bytes, const Schedule &sched,
               AxisPlan *out, std::string *err);

}  // namespace fht
