// Launch interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fht {

// One (image, quadrant, pass) job of a launch.
struct JobDesc {
    const void *src;  // image (first pass) or the previous pass's [W][H] rows
    void *dst;        // next pass's [W][H] rows or the final output
    int32_t H;        // positions per lane
    int32_t ld;       // image row stride in elements (first pass only)
    int32_t flags;    // JF_* bits
    int32_t pad;
};

enum : int32_t {
    JF_COLS = 1,        // lanes are image columns (quadrants H+ and H-)
    JF_MIRROR = 2,      // negative slopes: positions are mirrored y -> (H - y) mod H
    JF_FINAL = 4,       // dst is the final output (stored un-mirrored)
    JF_SRC_WS = 8,      // src is an offset into the launch workspace
    JF_DST_WS = 16,     // dst is an offset into the launch workspace
};

constexpr int kInlineJobs = 4;

struct PassArgs {
    const int4 *items;     // {program, job, first position, 0}
    const int32_t *hdrs;   // 32 ints per program
    const int4 *ops;       // row operations
    const JobDesc *jobs;   // device job table, or null to use inl
    char *ws;              // workspace base for JF_*_WS offsets
    JobDesc inl[kInlineJobs];
};

enum class Dt { U8 = 0, F32 = 1, F64 = 2 };

// Enqueues one fused pass of `n_items` work items with `threads` (256, 512
// or 1024) threads per workgroup.  from_image selects the first-pass loader
// (reads the image of dtype dt), otherwise the pass reads accumulator rows.
// Returns the launch status.
hipError_t launch_pass(Dt dt, bool from_image, const PassArgs &args, int n_items,
                       int lds_bytes, int threads, hipStream_t stream);

}  // namespace fht
