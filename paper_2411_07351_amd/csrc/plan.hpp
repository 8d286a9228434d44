// Host-side planner: the computation-order tree of Alg. 1 and the fused-pass
// tile programs the gfx950 kernels execute.  Pure C++, no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fht {

constexpr int kHdrInts = 32;     // ints per tile-program header
constexpr int kHdrFirst = 0;     // index of the program's first entry in its pass
constexpr int kHdrLoads = 1;     // load entries
constexpr int kHdrStores = 2;    // store entries
constexpr int kHdrSteps = 3;     // merge steps run in LDS
constexpr int kHdrLds = 4;       // LDS elements
constexpr int kHdrEntries = 5;   // all entries
constexpr int kHdrLevelIn = 6;   // level the pass starts from
constexpr int kHdrHeight = 7;    // height of the pass root
constexpr int kHdrStepCounts = 8;  // slots 8 .. 23: entries of each LDS merge step
constexpr int kMaxSteps = 16;
constexpr int kHdrLoadEnd = 24;  // first pass: largest end of a lane's padded load window
constexpr int kHdrSTile = 25;    // positions per work item of this pass
constexpr int kHdrChunks = 26;   // chunks K every entry of the program covers
constexpr int kHdrStoreMerge = 27;  // 1: the stores add the root's last merge (see emit_tile)
constexpr int kHdrLoadMerges = 28;  // load-merge entries (step 1 read from the source rows)
constexpr int kHdrElemBytes = 29;   // LDS element bytes of the pass
constexpr int kHdrLaneBase = 30;    // lanes added to every row the entries name (see share_tile)
constexpr int kChunk = 64;       // positions per chunk (one wavefront access)
constexpr int kMaxFirstLevels = 6;  // first-pass roots have at most 64 lanes
constexpr int kMaxTarget = 256;     // widest row window a schedule may ask for
constexpr int kMaxChunks = 4;       // chunks per entry the kernels are built for
constexpr int kEntryPrefetch = 64;  // entries a kernel may read from a program's first one

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

// Height of the order tree of W lanes, ceil(log2 W), for either split.
int make_tree_height(int W);

// Row windows are tiled in 64-position chunks; a pass picks the largest
// position tile whose widest window fits its target width.
struct Schedule {
    int s_tile = 192;         // target window width, later passes
    int s_tile_first = 128;   // target window width, first pass
    int first_levels = 5;
    int max_levels = 3;
    int lds_budget = 64 * 1024;
    int t_tile = 16;          // 0: the largest of 32, 16, 8, 4 that fits
    int threads = 512;        // threads per workgroup of later passes: 256 or 512
    int threads_first = 512;  // threads per workgroup of the first pass
};

// One fused pass: from the frontier of level lin (maximal nodes of height
// <= lin) to the frontier of level lout.
struct Pass {
    int lin = 0, lout = 0;
    int t_tile = 0;
    int S = 0;                   // positions per work item
    int widest = 0;              // widest row window
    int max_root_w = 0;          // widest node this pass produces
    int elem_bytes = 4;          // LDS element size
    int max_lds_elems = 0;
    bool fits = true;            // every program respects the kernel's prefetch limits
    std::vector<int32_t> hdrs;   // kHdrInts per program
    std::vector<int32_t> ops;    // 4 per op
    std::vector<int32_t> items;  // 4 per work item
};

struct AxisPlan {
    int W = 0, H = 0, split = 0;
    std::vector<Pass> passes;
};

// LDS element size of a pass as a function of the widest nodes it reads and
// produces: `narrow_bytes` while the output width is at most `narrow_width`,
// `transition_bytes` (if set) for the pass that crosses it, else `wide_bytes`
// (uint8 images: 16-bit sums up to 257 lanes, then 32-bit; quadrant pairs keep
// two sums per element).
struct ElemRule {
    int narrow_bytes = 4, wide_bytes = 4, narrow_width = 0, transition_bytes = 0;
    int bytes_for(int in_width, int out_width) const
    {
        if (out_width <= narrow_width) return narrow_bytes;
        if (transition_bytes && in_width <= narrow_width) return transition_bytes;
        return wide_bytes;
    }
};

// Plans the passes for W lanes of H positions.  Returns false and sets *err
// on failure.
bool plan_axis(int W, int H, int split, const ElemRule &rule, const Schedule &sched,
               AxisPlan *out, std::string *err);

// Tile programs depend on H only through the position tile, which is
// min(H, a width fixed by the schedule and the slope tiles) <= kMaxTarget: a
// plan made for any H >= kMaxTarget serves every such H once its work items
// are regenerated.  Moves `ax` to height H >= kMaxTarget.
void retile_items(AxisPlan *ax, int H);

// Gather steps of the adjoint (back-projection) of Alg. 1, top down.  Step k
// takes the gradients of the frontier of level L - k (L = root height) to
// those of level L - k - 1; in every step, output row x is
//   g_out[x][s] = sum_{j < n} g_in[p0 + j][(s - (right ? r0 + j : 0)) mod H]
// with tasks[(k W + x) 4 ..] = {p0, n, r0, right}.  Rows of a node sit at its
// lane range, as in the forward direction.
struct AdjointAxis {
    int W = 0, levels = 0;
    std::vector<int32_t> tasks;  // levels x W x 4
};

AdjointAxis plan_adjoint_axis(int W, int split);

// The adjoint's steps fused into gathers of up to `max_levels` levels each
// (top down): pass p maps the gradients of one frontier to those `levels`
// levels further down, in one launch,
//   g_out[x][s] = sum_{i in [offs[x], offs[x+1])} g_in[row_i][(s - shift_i) mod H],
// with terms[2 i] = row_i, terms[2 i + 1] = shift_i mod H: the composition
// of the single steps (shifts add along each path; the preimages partition
// the rows, so no term repeats).
struct AdjointPass {
    int levels = 0;
    std::vector<int32_t> offs;   // W + 1
    std::vector<int32_t> terms;  // 2 per term
};

std::vector<AdjointPass> fuse_adjoint(const AdjointAxis &ax, int H, int max_levels);

}  // namespace fht
