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

// Element types of one fused pass: what it reads (the image in a first pass,
// the previous pass's rows otherwise), what it keeps in LDS, what it writes.
// uint8 images keep 16-bit sums while nodes are at most 257 lanes wide
// (255 * 257 < 2^16), so those intermediates move half the bytes.
enum class Combo {
    U8_U16_U16,    // first pass, uint8 image, 16-bit rows out
    U8_U16_I32,    // first pass, uint8 image, final int32 output
    U16_U16_U16,   // later pass, 16-bit in and out
    U16_U16_I32,   // later pass, 16-bit in, final int32 output
    U16_I32_I32,   // later pass, 16-bit in, 32-bit sums
    I32_I32_I32,   // later pass, 32-bit
    F32_FIRST,     // first pass, float32 image
    F32_LATER,
    F64_FIRST,     // first pass, float64 image
    F64_LATER,
};

// Enqueues one fused pass of `n_items` work items with `threads` (256 or
// 512) threads per workgroup.  Returns the launch status.
hipError_t launch_pass(Combo combo, const PassArgs &args, int n_items, int lds_bytes, int threads,
                       hipStream_t stream);

}  // namespace fht
