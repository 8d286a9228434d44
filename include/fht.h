/*
 * fht.h - C ABI of the MI355X (gfx950) dyadic-pattern fast Hough transform.
 *
 * The transform is FHT2D of Kazimirov, Nikolaev, Rybakova and Terekhin,
 * "Generalization of Brady-Yong Algorithm for Fast Hough Transform to Arbitrary
 * Image Size" (arXiv 2411.07351), Sec. 3, Alg. 1: the image is split into two
 * column ranges of widths Split(w) (Split_S = floor/ceil halves, the FHT2DS
 * rule; Split_T = largest power of two on the left, the paper's FHT2DT rule),
 * both halves are transformed recursively, and row t of the result is the sum
 * of row [t k_0] of the left result and row [t k_1] of the right result
 * circularly shifted by t - [t k_1], with k_P = (w_P - 1)/(w - 1) and [.] the
 * nearest integer (ties to even, computed exactly).  Every output is therefore
 * a sum along a dyadic pattern of Alg. 2, wrapped mod the image height.
 *
 * Quadrants.  For a row-major image of R rows and C columns four lane-major
 * views A[x][y] are transformed:
 *   q0 "V+": lanes x = image rows (W = R), positions y = columns (H = C), shift +1
 *   q1 "V-": same lanes, shift -1 (negative slopes)
 *   q2 "H+": lanes x = image columns (W = C), positions y = rows (H = R), shift +1
 *   q3 "H-": same lanes, shift -1
 * Output q is out_q[t][s] = sum_x A[x][(s + sign_q * pat_{W,t}(x)) mod H],
 * t in [0, W), s in [0, H), row-major W x H.  The selected quadrants are
 * stored back to back in q order in one output buffer.
 *
 * Types.  FHT_U8 images give int32 outputs (exact: 255 W < 2^31); FHT_F32
 * gives float32; FHT_F64 gives float64.
 *
 * Memory and ownership.  All image, output and workspace pointers are device
 * pointers (HIP) that the caller allocates and owns.  A plan owns its host
 * tables and the device copies of them; it is immutable after creation and may
 * be shared by threads and streams.  Calls that use the same workspace must not
 * overlap.  The library allocates device memory only for plan tables
 * (fht_plan_upload, or the first fht_forward of a plan on a device) and for
 * batch tables (fht_batch_create).
 *
 * Errors.  No call aborts or throws.  Arguments are checked before anything
 * is enqueued; launches are asynchronous on the given stream, so a device fault
 * surfaces at the caller's next synchronisation.
 */
#ifndef FHT_H_
#define FHT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FHT_OK = 0,
    FHT_EINVAL = -1,  /* bad size, null pointer, bad quadrant mask or schedule */
    FHT_EDTYPE = -2,  /* unknown dtype or mixed dtypes in one batch */
    FHT_ENOMEM = -3,  /* host or device allocation failed */
    FHT_EHIP = -4,    /* a HIP runtime call or kernel launch failed */
    FHT_EBUSY = -5,   /* request does not fit the stated budget (serving admission) */
    FHT_ENODEV = -6   /* no HIP device is available */
} fht_status;

typedef enum { FHT_U8 = 0, FHT_F32 = 1, FHT_F64 = 2 } fht_dtype;

/* Sec. 3: FHT2DS (Split_S, floor/ceil halves) and FHT2DT (Split_T). */
typedef enum { FHT_SPLIT_S = 0, FHT_SPLIT_T = 1 } fht_split;

typedef struct fht_plan_s *fht_plan;
typedef struct fht_batch_s *fht_batch;
typedef struct fht_planner_s *fht_planner;

/*
 * Tiling of the fused passes (not in the paper: the paper's recursion runs one
 * level at a time).  Zero in a field means "library default".
 *   s_tile        widest row window of a later pass, in positions (64, 128,
 *                 192 or 256); the pass takes the largest position tile that fits
 *   first_levels  tree levels fused in the first pass (1..6)
 *   max_levels    tree levels fused in each later pass (1..16)
 *   lds_budget    LDS bytes a work item may use (1024..163840)
 *   t_tile        slope rows per work item in later passes, halved while the
 *                 pass does not fit the LDS budget (-1: start from 32)
 *   s_tile_first  widest row window of the first pass (64..256, multiple of 64)
 *   threads       threads per workgroup of later passes: 256 or 512
 *   threads_first threads per workgroup of the first pass: 256 or 512
 */
typedef struct {
    int32_t s_tile;
    int32_t first_levels;
    int32_t max_levels;
    int32_t lds_budget;
    int32_t t_tile;
    int32_t s_tile_first;
    int32_t threads;
    int32_t threads_first;
} fht_schedule;

/* Human-readable name of a status code (an fht_status value; static storage,
 * "unknown status" for any other value). */
const char *fht_status_string(int32_t s);

/*
 * Build a plan for rows x cols images of the given dtype (an fht_dtype value)
 * and split rule (an fht_split value; Sec. 3, Alg. 1).  Enumerated arguments
 * of this ABI are passed as int32_t, so any value a caller passes is checked
 * rather than being outside its enumeration.  quadrant_mask bit q selects
 * output q (1..15).  sched may be NULL.  Host-only: needs no GPU.  On success
 * *out owns the plan.
 * Errors: FHT_EINVAL (rows or cols < 1 or > 65536, mask 0 or > 15, bad
 * schedule), FHT_EDTYPE, FHT_ENOMEM.
 */
fht_status fht_plan_create(fht_plan *out, int32_t rows, int32_t cols, int32_t dtype,
                           int32_t split, uint32_t quadrant_mask, const fht_schedule *sched);

/* Frees host and device tables of a plan; NULL is ignored.  The caller
 * must make sure no enqueued work still uses the plan.  Device memory (of
 * plans, and of lane-view programs the process-wide program cache drops) is
 * released in groups of at least 64 MiB, because each release waits for the
 * device: destroying a plan does not stall the streams. */
void fht_plan_destroy(fht_plan plan);

/* Elements of the output buffer: sum over selected q of W_q * H_q. */
size_t fht_plan_out_elems(fht_plan plan);

/* Element offset of quadrant q in the output buffer, or -1 if not selected. */
int64_t fht_plan_out_offset(fht_plan plan, int32_t q);

/* Bytes of device workspace fht_forward needs (0 if none). */
size_t fht_plan_workspace_bytes(fht_plan plan);

/* Number of kernel launches one fht_forward enqueues. */
int32_t fht_plan_num_launches(fht_plan plan);

/*
 * Launch `launch` of fht_forward: its pass level, the algorithmic bytes it must
 * move for one image (every element it reads once plus every element it
 * writes once: the image or the previous pass's rows, then the next pass's rows
 * or the output; uint8 images keep 16-bit rows while nodes are at most 257
 * lanes wide) and its number of work items.  Any pointer may be NULL.
 * Errors: FHT_EINVAL.
 */
fht_status fht_plan_launch_info(fht_plan plan, int32_t launch, int32_t *level,
                                int64_t *bytes_in, int64_t *bytes_out, int32_t *n_items);

/* Inspection (tests and tools; not needed to run the transform).
 * Additions of the plan's forward transform, summed over its quadrants:
 * *adds_tree is the count of Alg. 1 (every non-leaf node of width w of the
 * order tree adds w rows of H positions: Theorem 1's f(n) for n x n);
 * *adds_executed is what the fused kernels add, whole 64-position chunks of
 * every merge including the halo positions of their tiles.  Host only; either
 * pointer may be NULL.  Errors: FHT_EINVAL. */
fht_status fht_plan_work(fht_plan plan, int64_t *adds_tree, int64_t *adds_executed);

/* The signature of the kernel launch `launch` of fht_forward runs, as
 * profilers print it (without its namespace and arguments), valid while the
 * plan lives; NULL for a bad index. */
const char *fht_plan_launch_kernel(fht_plan plan, int32_t launch);

/* Copy the plan's tables to the current HIP device (idempotent).  Needed only
 * before capturing fht_forward into a HIP graph.  Errors: FHT_ENODEV, FHT_ENOMEM,
 * FHT_EHIP. */
fht_status fht_plan_upload(fht_plan plan);
/* Copy only the plan's lane-view programs to the current HIP device
 * (idempotent; programs are shared by every plan of the same lane count):
 * what batches (fht_batch_create, fht_batch_upload) read, without the plan's
 * own work items, which only fht_forward uses.  A server can call it on a
 * planner thread so that its loop never waits for the copy.  Errors:
 * FHT_EINVAL, FHT_ENODEV, FHT_ENOMEM, FHT_EHIP. */
fht_status fht_plan_upload_programs(fht_plan plan);
/* The same for n plans at once: the programs of all their lane views not yet
 * on the current device go in one device allocation and one copy, through
 * two 4 MiB pinned staging buffers and a non-blocking stream of the library
 * (so the copy never waits for work on other streams).  The block is freed
 * with the last view in it.  Errors: FHT_EINVAL (n < 0, or a null plan),
 * FHT_ENODEV, FHT_ENOMEM, FHT_EHIP; on an error no view is marked as copied. */
fht_status fht_plan_upload_programs_many(const fht_plan *plans, int32_t n);

/*
 * Planner pool: plans (fht_plan_create) made on `threads` worker threads of
 * the library, and, for device >= 0, their lane-view programs copied to that
 * HIP device by one more thread of the pool, up to 32 finished plans per
 * fht_plan_upload_programs_many (small copies from many threads serialise
 * inside the HIP runtime).  A request loop only submits and polls: it never
 * runs the planner, holds no lock of its own language's runtime while plans
 * are made, and never waits for the copies.  device -1 plans on the host only.
 *   fht_planner_create  threads in [1, 256].  Errors: FHT_EINVAL, FHT_ENOMEM.
 *   fht_planner_submit  queues one plan (arguments as fht_plan_create; the
 *                       schedule, if any, is copied) and returns its ticket
 *                       (0, 1, 2, ... in submission order).  Errors: FHT_EINVAL,
 *                       FHT_ENOMEM.  Bad plan arguments are reported by the poll.
 *   fht_planner_poll    1 once the ticket's plan is finished: *status is what
 *                       making (and copying) it returned and *plan the plan,
 *                       owned by the caller from then on (NULL unless *status
 *                       is FHT_OK); the ticket is then forgotten.  0 while it
 *                       is queued or being made, -1 for a null argument or a
 *                       ticket never issued or already taken.
 *   fht_planner_destroy drops queued plans, waits for those being made and the
 *                       copy under way, frees the plans no poll took (finished
 *                       or waiting for their copy), and joins the threads;
 *                       NULL is ignored.
 * Submit and poll may be called from any threads.  With device >= 0 the
 * uploader allocates device memory and copies on its own stream while plans
 * arrive: a HIP graph captured meanwhile in global capture mode on another
 * thread fails, so capture with thread-local mode or while no plan is made.
 */
fht_status fht_planner_create(int32_t threads, int32_t device, fht_planner *out);
fht_status fht_planner_submit(fht_planner planner, int32_t rows, int32_t cols, int32_t dtype,
                              int32_t split, uint32_t quadrant_mask, const fht_schedule *sched,
                              int64_t *ticket);
int32_t fht_planner_poll(fht_planner planner, int64_t ticket, fht_plan *plan, fht_status *status);
void fht_planner_destroy(fht_planner planner);

/*
 * Forward transform of one image (Alg. 1 for every selected quadrant).
 *   d_img  device, row-major rows x cols of the plan's dtype (uint8/float/double)
 *   d_out  device, fht_plan_out_elems elements (int32 for FHT_U8, else the dtype)
 *   d_ws   device, fht_plan_workspace_bytes bytes (may be NULL when that is 0)
 *   stream HIP stream (hipStream_t) or NULL for the null stream
 * Asynchronous.  Errors: FHT_EINVAL (null pointers), FHT_ENODEV, FHT_EHIP.
 */
fht_status fht_forward(fht_plan plan, const void *d_img, void *d_out, void *d_ws, void *stream);

/*
 * fht_forward without allocating, for callers that cannot call hipMalloc:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * device allocation.  The workspace is the library's own static device
 * scratch of FHT_NOALLOC_WS_BYTES bytes (64 MiB: 32 bytes per pixel covers
 * about 2 Mpx, e.g. 1448 x 1448), one copy per device, held until the
 * process ends.  The plan's tables must already be on the current device
 * (fht_plan_upload, or an earlier fht_forward there); this call allocates
 * nothing.  Every call on one device shares that device's scratch, so calls
 * that overlap on one device (other streams, other threads) race and give
 * wrong results; the scratch keeps the last call's contents, and since every
 * element is written before it is read nothing needs clearing.
 *   d_img, d_out, stream  as fht_forward
 * Errors: FHT_EINVAL (null pointers, fht_plan_workspace_bytes(plan) above
 * FHT_NOALLOC_WS_BYTES, tables not uploaded to the current device),
 * FHT_ENODEV, FHT_EHIP.
 */
#define FHT_NOALLOC_WS_BYTES ((size_t)64 * 1024 * 1024)
fht_status fht_forward_noalloc(fht_plan plan, const void *d_img, void *d_out, void *stream);

/*
 * fht_forward for n same-shape images at once (one launch per fused pass for
 * all of them): image b is read at d_imgs + b * img_stride and its output
 * written at d_outs + b * out_stride (strides in bytes, >= 0, multiples of
 * the element sizes).  d_ws holds fht_plan_workspace_bytes_many(plan, n)
 * bytes.  n in 1..65535.  Errors: as fht_forward, FHT_EINVAL for bad n or
 * strides.
 */
size_t fht_plan_workspace_bytes_many(fht_plan plan, int32_t n);
fht_status fht_forward_many(fht_plan plan, int32_t n, const void *d_imgs, int64_t img_stride,
                            void *d_outs, int64_t out_stride, void *d_ws, void *stream);

/* Enqueues only launch `launch` (0 <= launch < fht_plan_num_launches) of
 * fht_forward, with the same arguments.  Running launches 0, 1, ... in order
 * on one stream equals fht_forward; it lets a caller time or interleave the
 * fused passes.  Errors: as fht_forward, FHT_EINVAL for a bad index. */
fht_status fht_forward_launch(fht_plan plan, int32_t launch, const void *d_img, void *d_out,
                              void *d_ws, void *stream);

/*
 * Batched forward over n images of possibly different sizes (one plan each,
 * all of one dtype and split, with any schedules): one launch per fused pass,
 * element types and workgroup size for the whole batch instead of per image.  fht_batch_create binds the device pointers and builds
 * the batch's device work list; fht_batch_run enqueues it (it may be captured
 * into a HIP graph).  d_ws must hold fht_batch_workspace_bytes bytes.
 *   plans  host array of n plans (each must outlive the batch)
 *   d_imgs host array of n device image pointers
 *   d_outs host array of n device output pointers (fht_plan_out_elems each)
 * Errors: FHT_EINVAL, FHT_EDTYPE (dtypes or splits differ), FHT_ENOMEM,
 * FHT_EHIP.
 */
fht_status fht_batch_create(fht_batch *out, const fht_plan *plans, int32_t n,
                            const void *const *d_imgs, void *const *d_outs);
size_t fht_batch_workspace_bytes(fht_batch batch);
int32_t fht_batch_num_launches(fht_batch batch);
fht_status fht_batch_run(fht_batch batch, void *d_ws, void *stream);
/* One launch of fht_batch_run (0 <= launch < fht_batch_num_launches). */
fht_status fht_batch_run_launch(fht_batch batch, int32_t launch, void *d_ws, void *stream);
/* Frees the batch and, for fht_batch_create, its device tables (a device
 * synchronisation point).  A batch whose tables went to caller memory with
 * fht_batch_upload frees host memory only. */
void fht_batch_destroy(fht_batch batch);

/*
 * The same batch in two halves, for callers that must not allocate or
 * synchronise the device while other work runs (a serving loop):
 * fht_batch_prepare builds the work list in host memory only (same arguments
 * and errors as fht_batch_create, no FHT_ENODEV); fht_batch_tables_bytes is the
 * size of its device tables; fht_batch_upload enqueues their copy into
 * caller-owned device memory d_tables (at least that many bytes, 256-byte
 * aligned) on `stream`.  fht_batch_run on that stream (or one ordered after
 * it) then runs the batch.  The caller keeps d_tables alive while the batch
 * runs, and destroys the batch only after the copy has completed (the copy
 * reads the batch's host memory).  A batch can be uploaded once; fht_batch_run
 * before the upload returns FHT_EINVAL.
 * Errors of fht_batch_upload: FHT_EINVAL (null, too small, already owning
 * tables), FHT_EHIP.
 */
fht_status fht_batch_prepare(fht_batch *out, const fht_plan *plans, int32_t n,
                             const void *const *d_imgs, void *const *d_outs);
size_t fht_batch_tables_bytes(fht_batch batch);
fht_status fht_batch_upload(fht_batch batch, void *d_tables, size_t bytes, void *stream);
/* fht_batch_upload through caller-owned pinned host memory h_staging (at
 * least fht_batch_tables_bytes bytes, from hipHostMalloc or a pinned
 * allocator): the tables are written there and copied from there, so the copy
 * is asynchronous (from pageable memory the runtime waits for it).  The caller
 * keeps h_staging, like d_tables, alive until the copy has completed.  Errors:
 * those of fht_batch_upload, and FHT_EINVAL for a null h_staging. */
fht_status fht_batch_upload_staged(fht_batch batch, void *d_tables, size_t bytes,
                                   void *h_staging, void *stream);

/* Enqueues on `stream` the copies of the batch's images from srcs[i], one
 * entry per image of the batch (host memory, pinned for an asynchronous copy,
 * or device memory; NULL: image i is in place already) to the device images the batch was made with, rows x cols
 * pixels of its dtype each, in one call for the whole batch.  srcs must stay
 * valid and unchanged until the stream has passed the copies.  Errors:
 * FHT_EINVAL, FHT_EHIP (copies enqueued before the failing one stay). */
fht_status fht_batch_copy_images(fht_batch batch, const void *const *srcs, void *stream);

/*
 * Adjoint (back-projection) of fht_forward for float32/float64 plans: the
 * image gradient of a scalar function of the output, given its output
 * gradient.  With out_q[t][s] = sum_x A_q[x][(s + sigma_q pat_t(x)) mod H]
 * (Alg. 2 patterns; A_q the lane view of quadrant q, sigma = +1 for V+/H+,
 * -1 for V-/H-), it computes
 *   gimg = sum_q view_q^T ( g_q[x][y] = sum_t gout_q[t][(y - sigma_q pat_t(x)) mod H] )
 * by running the merges of Alg. 1 backwards, up to three tree levels per
 * gather launch; the last gather of every quadrant runs in one final launch
 * that also sums the quadrants into d_gimg.
 *   d_gout device, fht_plan_out_elems elements in fht_forward's output layout
 *   d_gimg device, rows x cols, overwritten
 *   d_ws   device, fht_plan_adjoint_workspace_bytes bytes (NULL when 0)
 * Asynchronous.  Errors: FHT_EDTYPE (uint8 plan), FHT_EINVAL, FHT_ENODEV,
 * FHT_ENOMEM, FHT_EHIP.
 */
size_t fht_plan_adjoint_workspace_bytes(fht_plan plan);
/* Inspection (tests and tools; not needed to run the transform).
 * Host view of the adjoint's gather steps of lane view v (0: lanes are rows,
 * 1: columns), valid while the plan lives: *levels steps of *lanes tasks of 4
 * ints {p0, n, r0, right}; step k, row x:
 *   g_out[x][s] = sum_{j<n} g_in[p0 + j][(s - (right ? r0 + j : 0)) mod H].
 * Errors: FHT_EINVAL, FHT_EDTYPE (uint8 plan). */
fht_status fht_plan_adjoint_tasks(fht_plan plan, int32_t v, const int32_t **tasks,
                                  int32_t *levels, int32_t *lanes);
/* Inspection (tests and tools; not needed to run the transform).
 * The gather launches fht_adjoint runs for lane view v: those steps composed
 * a few levels at a time.  fht_plan_adjoint_num_passes returns their number
 * (-1 for a bad view or a uint8 plan); pass `pass` covers *levels steps:
 *   g_out[x][s] = sum_{i in [offs[x], offs[x+1])} g_in[terms[2i]][(s - terms[2i+1]) mod H]
 * with offs holding lanes + 1 entries and shifts already reduced mod H.
 * Pointers are valid while the plan lives.  Errors: FHT_EINVAL. */
int32_t fht_plan_adjoint_num_passes(fht_plan plan, int32_t v);
fht_status fht_plan_adjoint_pass(fht_plan plan, int32_t v, int32_t pass, int32_t *levels,
                                 const int32_t **offs, const int32_t **terms, int32_t *n_terms);
fht_status fht_adjoint(fht_plan plan, const void *d_gout, void *d_gimg, void *d_ws, void *stream);
/* fht_adjoint for n same-shape images: output gradient b at d_gouts +
 * b * gout_stride, image gradient b at d_gimgs + b * gimg_stride (bytes);
 * d_ws holds fht_plan_adjoint_workspace_bytes_many(plan, n) bytes.  n in
 * 1..65535.  Errors: as fht_adjoint. */
size_t fht_plan_adjoint_workspace_bytes_many(fht_plan plan, int32_t n);
fht_status fht_adjoint_many(fht_plan plan, int32_t n, const void *d_gouts, int64_t gout_stride,
                            void *d_gimgs, int64_t gimg_stride, void *d_ws, void *stream);

/*
 * Peak finding on the quadrant outputs of one image (the step after the
 * transform: a straight segment concentrates on one output, Sec. 3).
 * A candidate is an output out_q[t][s] >= min_value that is a strict maximum
 * of its (2 radius + 1)^2 window in (t, s) of quadrant q (s wraps mod H, t is
 * clipped to [0, W)); an equal neighbour earlier in the flat output order
 * wins the tie.  The k strongest candidates (value descending, then flat
 * output index ascending) go to d_peaks.
 *   d_out     device, the plan's output (fht_forward layout, NaN-free)
 *   k         1..4096 peaks wanted; radius 0..64; capacity k..2^26 candidates kept
 *   d_ws      device, fht_peaks_workspace_bytes(capacity) bytes
 *   d_peaks   device, k fht_peak records (value as float)
 *   d_found   device, 2 int32: peaks written, candidates found (more than
 *             capacity means some were dropped: raise min_value or capacity)
 * Asynchronous.  Errors: FHT_EINVAL, FHT_ENODEV, FHT_EHIP.
 */
typedef struct fht_peak {
    float value;
    int32_t quadrant, t, s;
} fht_peak;
size_t fht_peaks_workspace_bytes(int32_t capacity);
fht_status fht_peaks(fht_plan plan, const void *d_out, int32_t k, int32_t radius,
                     double min_value, int32_t capacity, void *d_ws, fht_peak *d_peaks,
                     int32_t *d_found, void *stream);

/*
 * Fault injection for tests of error handling: the next `count` calls that
 * enqueue device work (fht_forward, fht_forward_noalloc, fht_forward_many,
 * fht_forward_launch, fht_adjoint, fht_adjoint_many, fht_peaks,
 * fht_batch_upload, fht_batch_upload_staged, fht_batch_run, fht_batch_run_launch) return
 * `code` (an fht_status value) after checking their
 * arguments and before enqueuing anything.  count <= 0 or code == FHT_OK
 * disarms it.  Process-wide; safe to call from any thread.
 */
void fht_debug_fail_next(int32_t code, int32_t count);

/*
 * Inspection (tests and tools; not needed to run the transform).
 * Host view of a plan's tables, for inspection and tests of the planner.
 * Quadrant view v = 0 (lanes are image rows) or 1 (lanes are image columns).
 * fht_plan_num_passes returns the number of fused passes of view v (or -1).
 * fht_plan_pass_tables returns pointers into the plan (valid while it lives):
 *   hdrs  n_progs x FHT_HDR_INTS ints: [0] first entry, [1] loads, [2] stores,
 *         [3] merge steps in LDS, [4] LDS elements, [5] all entries, [6] level in,
 *         [7] height of the pass root, [8 + k] entries of LDS merge step k,
 *         [24] first pass: end of the padded load windows, [25] positions per item,
 *         [26] chunks k of every entry, [27] 1 if the stores add (the root's
 *         last merge), [28] load-merges, [29] LDS element bytes, [30] lane base:
 *         added to every src and dst row the program's entries name (programs
 *         of pass roots of equal widths share entries)
 *   ops   4 ints each, every entry covering k whole 64-position chunks, in the
 *         order loads, load-merges, merge steps, stores:
 *         load  {lds, src row, position offset, k}: lds[d+c] = src[row][(s0+off+c) mod H]
 *         load-merge {lds dst, src row a, src row b, off | r << 16}:
 *               lds[d+c] = src[a][(s0+off+c) mod H] + src[b][(s0+off+r+c) mod H]
 *         merge {lds dst, lds src0, lds src1, k}:  lds[d+c] = lds[a+c] + lds[b+c]
 *         store {lds, dst row, limit, src1}: dst[row][s0+c] = lds[d+c] (+ lds[src1+c]
 *               when [27] is set), c < limit, s0+c < H
 *   items 4 ints each: {program, 0, first position, 0}
 *   s_tile positions per item of this pass.
 */
#define FHT_HDR_INTS 32
int32_t fht_plan_num_passes(fht_plan plan, int32_t v);
fht_status fht_plan_pass_tables(fht_plan plan, int32_t v, int32_t pass,
                                const int32_t **hdrs, int32_t *n_progs,
                                const int32_t **ops, int32_t *n_ops,
                                const int32_t **items, int32_t *n_items,
                                int32_t *s_tile);

#ifdef __cplusplus
}
#endif

#endif /* FHT_H_ */
