// Launch interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fht {

// One (image, quadrant or quadrant pair, pass) job of a launch.
struct JobDesc {
    const void *src;       // image (first pass) or the previous pass's [W][H] rows
    void *dst;             // next pass's [W][H] rows or the final output
    void *dst2;            // pair jobs: rows or output of the negative-slope quadrant
    const int32_t *hdrs;   // tile-program headers of this job's lane view (32 ints each)
    const int4 *ops;       // their row entries
    int32_t H;             // positions per lane
    int32_t ld;            // image row stride in elements (first pass only)
    int32_t flags;         // JF_* bits
    int32_t pad;
};

enum : int32_t {
    JF_COLS = 1,        // lanes are image columns (quadrants H+ and H-)
    JF_MIRROR = 2,      // negative slopes: positions are mirrored y -> (H - y) mod H
    JF_FINAL = 4,       // dst is the final output (stored un-mirrored)
    JF_SRC_WS = 8,      // src is an offset into the launch workspace
    JF_DST_WS = 16,     // dst is an offset into the launch workspace
    JF_PAIR = 32,       // the job runs both quadrants of a lane view as pairs
                        // (positive slope low, mirrored negative slope high)
};

constexpr int kInlineJobs = 4;

struct PassArgs {
    const int4 *items;     // {program of the job's view, job, first position, first entry}
    const JobDesc *jobs;   // device job table, or null to use inl
    char *ws;              // workspace base for JF_*_WS offsets
    // Same-shape image batches (grid.y = image b, inline jobs only): image b's
    // image, output and workspace sit b strides (bytes) after image 0's.
    int64_t img_stride, out_stride, ws_stride;
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
    // Quadrant pairs (JF_PAIR): the positive- and negative-slope quadrants of
    // one lane view share the order tree and every program, so one work item
    // runs both, adding 16-bit pairs with one 32-bit add (no carry crosses
    // the halves: each stays below 2^16 while nodes are at most 257 wide).
    P_U8_FIRST,        // first pass, uint8 image, pair rows out
    P_U8_FIRST_FINAL,  // first pass, two final int32 outputs
    P_U16_MID,         // later pass, pair rows in and out
    P_U16_MID_FINAL,   // later pass, pair rows in, two final int32 outputs
    P_I32,             // the pass that outgrows 16 bits: pair rows in, 32-bit pairs in
                       // LDS, two int32 row sets (or final outputs) out
};

// Enqueues one fused pass of `n_items` work items with `threads` (256 or
// 512) threads per workgroup, for `n_images` same-shape images (see
// PassArgs strides).  Returns the launch status.
hipError_t launch_pass(Combo combo, const PassArgs &args, int n_items, int lds_bytes, int threads,
                       hipStream_t stream, int n_images = 1);

// Adjoint (back-projection).  One fused gather pass of one quadrant: rows of
// the gradient of one frontier to those of a frontier several levels down
// (see fht::AdjointPass for the term format).
struct AdjJob {
    const void *src;       // [W][H] gradient rows in (the output gradient in pass 0)
    void *dst;             // [W][H] gradient rows out
    const int32_t *offs;   // W + 1 term offsets
    const int32_t *order;  // the W output rows in launch order (a permutation of 0 .. W - 1)
    const int2 *terms;     // {source row, shift mod H}
    int32_t W, H;
    int32_t mirror_in;     // read src at mirrored positions (pass 0 of V-/H-)
    int32_t pad;
};

struct AdjArgs {
    AdjJob job[kInlineJobs];
    // same-shape image batches (grid.z = image): bytes between images
    int64_t src_stride, dst_stride;
};

// Sum of the quadrants' lane gradients into the image gradient (R x C):
// quadrants 0/1 have lanes = rows, 2/3 lanes = columns; `mirror` reads the
// positions at (H - y) mod H.
struct CombineArgs {
    const void *src[kInlineJobs];  // null: quadrant absent
    int32_t mirror[kInlineJobs];
    int32_t R, C;
    void *dst;
    // same-shape image batches (grid.z = image): bytes between images of each
    // source and of the destination
    int64_t src_stride[kInlineJobs], dst_stride;
};

// The last gather pass of every quadrant fused with the sum into the image
// gradient (R x C): one job per quadrant.
struct FinalJob {
    const void *src;        // rows the quadrant's last pass reads; null: quadrant absent
    const int32_t *offs;    // W + 1 term offsets of that pass; null: no tree levels (W = 1),
                            // the lane gradient is src itself
    const int2 *terms;      // {source row, shift mod H}
    int64_t src_stride;     // bytes between images of a same-shape batch
    int32_t in_mirror;      // src is read at mirrored positions (the last pass is the first)
    int32_t out_mirror;     // the quadrant's lane gradient is in the mirrored frame
};

struct FinalArgs {
    FinalJob q[kInlineJobs];  // quadrants 0..3 (lanes = rows for 0/1, columns for 2/3)
    int32_t R, C;
    void *dst;
    int64_t dst_stride;
};

enum class Real { F32, F64 };

// Peak finding over the quadrant outputs of one image.
struct PeakOut {
    float value;
    int32_t quadrant, t, s;
};

struct PeakArgs {
    const void *src[kInlineJobs];  // quadrant outputs [W][H], present ones first
    int32_t W[kInlineJobs], H[kInlineJobs];
    uint64_t base[kInlineJobs];    // flat output index of each quadrant's first element
    int32_t quadrant[kInlineJobs];
    int32_t nq;
    int32_t radius;
    double min_value;
    int32_t k, capacity;
    uint32_t *counter;             // workspace: candidate count
    uint64_t *keys;                // workspace: candidate keys (flat output index)
    const void *flat;              // the whole output (flat index 0)
    PeakOut *out;                  // k peaks, strongest first
    int32_t *n_found;              // [0] peaks written, [1] candidates found
};

enum class PeakElem { I32, F32, F64 };

hipError_t launch_peaks(PeakElem elem, const PeakArgs &args, size_t max_elems, hipStream_t stream);

// max_h: the largest H of the jobs (rows of up to 512 positions go in one
// round of loads).
hipError_t launch_adjoint_step(Real real, const AdjArgs &args, int n_jobs, int max_w,
                               hipStream_t stream, int n_images = 1, int max_h = 0);
hipError_t launch_adjoint_final(Real real, const FinalArgs &args, hipStream_t stream,
                                int n_images = 1);
hipError_t launch_adjoint_combine(Real real, const CombineArgs &args, hipStream_t stream,
                                  int n_images = 1);

}  // namespace fht
