// gfx950 kernels of the dyadic-pattern fast Hough transform.
//
// One launch executes one fused pass of Alg. 1 for many work items.  A work
// item (one workgroup of 4 or 8 wavefronts) runs a planner-made program:
// it loads the rows its slope tile needs into LDS, runs the merge steps of
// Alg. 1 (row t of a node = row t0 of the left child + row t1 of the right
// child rotated by t - t1) in LDS, and writes its output rows back.  The
// stores do the root's last merge on the way out, and a pass whose rows reach
// LDS through registers does its first merge on the way in (load-merges), so
// neither level's rows pass through LDS: LDS writes are the scarcest LDS
// bandwidth on this chip.
// The rotation is folded into LDS addresses, so every merge is a contiguous
// vector add over K whole 64-position chunks: one position per lane, which
// keeps LDS accesses bank-conflict free and HBM accesses coalesced.  This is
// a memory-bound integer or float add: no MFMA.
//
// Instruction economy.  K is fixed per program, so each row costs three
// address additions and 3K LDS accesses.  Row descriptors reach a wavefront
// 64 at a time through one vector load and are broadcast with readlane (a
// scalar load per row would share the LDS wait counter and serialise the
// rows); the next merge step's descriptors are fetched while the current step
// runs.  Later passes load HBM rows straight into LDS (global_load_lds_dword),
// all of a wavefront's rows in flight at once.
#include "kernels.hpp"
#include "plan.hpp"  // program header layout (host and device agree on it)

#include <type_traits>

namespace fht {

namespace {

// Read-only tables, read through the constant address space so that the
// compiler uses scalar loads for wave-uniform indices (item and header).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)(p);
}

struct E4 { int x, y, z, w; };
__device__ __forceinline__ E4 ld4(cptr<int32_t> t, int i)
{
    return E4{t[4 * i], t[4 * i + 1], t[4 * i + 2], t[4 * i + 3]};
}

__device__ __forceinline__ int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

template <bool TABLE>
__device__ __forceinline__ JobDesc pick_job(const PassArgs &a, int j)
{
    if constexpr (TABLE) {
        cptr<JobDesc> p = as_const(a.jobs) + j;
        JobDesc d;
        d.src = p->src;
        d.dst = p->dst;
        d.dst2 = p->dst2;
        d.hdrs = p->hdrs;
        d.ops = p->ops;
        d.H = p->H;
        d.ld = p->ld;
        d.flags = p->flags;
        d.pad = 0;
        return d;
    }
    switch (j) {
    case 0: return a.inl[0];
    case 1: return a.inl[1];
    case 2: return a.inl[2];
    default: return a.inl[3];
    }
}

// p mod H for p >= 0; ONE promises p < 2 H (one conditional subtraction, no
// division), which the callers check once per row or item.
template <bool ONE>
__device__ __forceinline__ int wrap(int p, int H)
{
    if constexpr (ONE)
        return p >= H ? p - H : p;
    else
        return p % H;
}

// Descriptors of this wavefront's entries g + NW * lane of a table of n entries.
template <int NW>
__device__ __forceinline__ int4 fetch_desc(const int4 *ent, int n, int g, int lane)
{
    const int idx = g + NW * lane;
    return idx < n ? ent[idx] : make_int4(0, 0, 0, 0);
}

template <int NW>
__device__ __forceinline__ int group_size(int n, int g)
{
    return min(64, (n - g + NW - 1) / NW);
}

// Merges of one group: entries {dst, src0, src1, K}, lds[dst + c] = lds[src0 + c] + lds[src1 + c].
template <int K, typename TL>
__device__ __forceinline__ void merge_group(TL *lds, const int4 &mine, int m, int lane)
{
    int j = 0;
    for (; j + 2 <= m; j += 2) {
        TL *d0 = lds + rl(mine.x, j) + lane, *d1 = lds + rl(mine.x, j + 1) + lane;
        const TL *a0 = lds + rl(mine.y, j) + lane, *a1 = lds + rl(mine.y, j + 1) + lane;
        const TL *b0 = lds + rl(mine.z, j) + lane, *b1 = lds + rl(mine.z, j + 1) + lane;
        TL x0[K], y0[K], x1[K], y1[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            x0[k] = a0[64 * k];
            y0[k] = b0[64 * k];
            x1[k] = a1[64 * k];
            y1[k] = b1[64 * k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            d0[64 * k] = static_cast<TL>(x0[k] + y0[k]);
            d1[64 * k] = static_cast<TL>(x1[k] + y1[k]);
        }
    }
    if (j < m) {
        TL *d0 = lds + rl(mine.x, j) + lane;
        const TL *a0 = lds + rl(mine.y, j) + lane, *b0 = lds + rl(mine.z, j) + lane;
        TL x0[K], y0[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            x0[k] = a0[64 * k];
            y0[k] = b0[64 * k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) d0[64 * k] = static_cast<TL>(x0[k] + y0[k]);
    }
}

// A source element as an LDS element: pair rows (two 16-bit sums in 32 bits)
// become two 32-bit sums when the LDS holds 32-bit pairs.
template <typename TL, typename TS>
__device__ __forceinline__ TL widen(TS v)
{
    if constexpr (std::is_same<TL, uint2>::value)
        return make_uint2(static_cast<uint32_t>(v) & 0xffffu, static_cast<uint32_t>(v) >> 16);
    else
        return static_cast<TL>(v);
}

// Later-pass loads {dst, row, offset, K}: lds[dst + c] = src[row][(s0 + offset + c) mod H].
// Rows go straight from HBM into 32-bit LDS elements when the LDS type is
// 32-bit (global_load_lds_dword; the 16-bit form zero-extends each lane's
// value into its dword, which widens 16-bit rows on the way); other rows go
// through registers, four rows of loads in flight before their LDS writes.
// ONE: every row window wraps around at most once (H >= 64 K).
template <int K, int NW, typename TS, typename TL, bool ONE>
__device__ __forceinline__ void load_rows_impl(TL *lds, const int4 *ent, int n, const TS *src,
                                               int H, int s0, int wave, int lane)
{
    for (int g = wave; g < n; g += 64 * NW) {
        const int4 mine = fetch_desc<NW>(ent, n, g, lane);
        const int m = group_size<NW>(n, g);
        if constexpr (sizeof(TL) == 4 && (sizeof(TS) == 4 || sizeof(TS) == 2)) {
            for (int j = 0; j < m; ++j) {
                int base = s0 + rl(mine.z, j);
                if (base >= H) base %= H;
                const TS *rowp = src + static_cast<size_t>(rl(mine.y, j)) * H;
                TL *dst = lds + rl(mine.x, j);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const TS *gp = rowp + static_cast<uint32_t>(wrap<ONE>(base + 64 * k + lane, H));
                    auto *g1 = (const __attribute__((address_space(1))) void *)(gp);
                    auto *l3 = (__attribute__((address_space(3))) void *)(dst + 64 * k);
                    if constexpr (sizeof(TS) == 2)
                        __builtin_amdgcn_global_load_lds(g1, l3, 2, 0, 0);
                    else
                        __builtin_amdgcn_global_load_lds(g1, l3, 4, 0, 0);
                }
            }
        } else {
            constexpr int R = 4;
            for (int j0 = 0; j0 < m; j0 += R) {
                TL v[R][K];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int j = min(j0 + r, m - 1);
                    int base = s0 + rl(mine.z, j);
                    if (base >= H) base %= H;
                    const TS *rowp = src + static_cast<size_t>(rl(mine.y, j)) * H;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        v[r][k] = widen<TL>(rowp[static_cast<uint32_t>(wrap<ONE>(base + 64 * k + lane, H))]);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (j0 + r < m) {
                        TL *dst = lds + rl(mine.x, j0 + r) + lane;
#pragma unroll
                        for (int k = 0; k < K; ++k) dst[64 * k] = v[r][k];
                    }
                }
            }
        }
    }
}

// Load-merges {dst, row a, row b, offset | r << 16} (step 1 of a later pass,
// read from the source rows instead of LDS copies of them):
//   lds[dst + c] = src[a][(s0 + offset + c) mod H] + src[b][(s0 + offset + r + c) mod H]
// Four entries' loads are in flight before their LDS writes.
template <int K, int NW, typename TS, typename TL, bool ONE>
__device__ __forceinline__ void load_merge_impl(TL *lds, const int4 *ent, int n, const TS *src,
                                                int H, int s0, int wave, int lane)
{
    constexpr int R = 4;
    for (int g = wave; g < n; g += 64 * NW) {
        const int4 mine = fetch_desc<NW>(ent, n, g, lane);
        const int m = group_size<NW>(n, g);
        for (int j0 = 0; j0 < m; j0 += R) {
            TS a[R][K], b[R][K];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = min(j0 + r, m - 1);
                const uint32_t offs = static_cast<uint32_t>(rl(mine.w, j));
                int ba = s0 + static_cast<int>(offs & 0xffffu);
                if (ba >= H) ba %= H;
                int bb = ba + static_cast<int>(offs >> 16);
                if (bb >= H) bb %= H;
                const TS *pa = src + static_cast<size_t>(rl(mine.y, j)) * H;
                const TS *pb = src + static_cast<size_t>(rl(mine.z, j)) * H;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    a[r][k] = pa[static_cast<uint32_t>(wrap<ONE>(ba + 64 * k + lane, H))];
                    b[r][k] = pb[static_cast<uint32_t>(wrap<ONE>(bb + 64 * k + lane, H))];
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (j0 + r < m) {
                    TL *dst = lds + rl(mine.x, j0 + r) + lane;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        dst[64 * k] = static_cast<TL>(widen<TL>(a[r][k]) + widen<TL>(b[r][k]));
                }
            }
        }
    }
}

template <int K, int NW, typename TS, typename TL>
__device__ __forceinline__ void load_merges(TL *lds, const int4 *ent, int n, const TS *src, int H,
                                            int s0, int wave, int lane)
{
    if (H >= 64 * K)
        load_merge_impl<K, NW, TS, TL, true>(lds, ent, n, src, H, s0, wave, lane);
    else
        load_merge_impl<K, NW, TS, TL, false>(lds, ent, n, src, H, s0, wave, lane);
}

template <int K, int NW, typename TS, typename TL>
__device__ __forceinline__ void load_rows(TL *lds, const int4 *ent, int n, const TS *src, int H,
                                          int s0, int wave, int lane)
{
    if (H >= 64 * K)
        load_rows_impl<K, NW, TS, TL, true>(lds, ent, n, src, H, s0, wave, lane);
    else
        load_rows_impl<K, NW, TS, TL, false>(lds, ent, n, src, H, s0, wave, lane);
}

// First-pass loads: the lanes of the pass root (at most 64, one descriptor
// {dst, lane, window start, K} each, in lane order) times their K-chunk
// position windows, read from the image.  Lanes are image rows (positions
// contiguous in memory) or image columns (lanes contiguous in memory); the
// thread mapping follows the contiguous direction so that loads coalesce.
//   rows: wavefront w takes lanes w + NW i, two lanes at a time
//   cols: thread t takes lane t % XW and positions t / XW + k * (threads / XW)
// Every thread issues a batch of loads (clamped in bounds) before their LDS
// writes, so they are in flight together.  With PAIR every element is
// (value at y) | (value at the mirrored position (H - y) mod H) << 16: the
// positive- and negative-slope quadrants together.  ONE: the windows wrap
// around at most once (load_end <= H).
constexpr int ROWS_AT_ONCE = 4;  // lanes per wavefront whose loads are in flight together
constexpr int COLS_AT_ONCE = 8;  // positions per thread whose loads are in flight together

template <typename TL, typename TSrc, bool PAIR>
__device__ __forceinline__ TL image_elem(TSrc a, TSrc b)
{
    if constexpr (PAIR)
        return static_cast<TL>(a) | (static_cast<TL>(b) << 16);
    else
        return static_cast<TL>(a);
}

// `pre` is entry `lane` of the program, fetched early (see fht_pass_kernel).
__device__ __forceinline__ int4 lane_entry(const int4 &pre, int src_lane)
{
    const int a = src_lane << 2;
    return make_int4(__builtin_amdgcn_ds_bpermute(a, pre.x), __builtin_amdgcn_ds_bpermute(a, pre.y),
                     __builtin_amdgcn_ds_bpermute(a, pre.z), __builtin_amdgcn_ds_bpermute(a, pre.w));
}

template <int K, int NW, typename TSrc, typename TL, bool PAIR, bool ONE>
__device__ __forceinline__ void load_image_impl(TL *lds, const int4 &pre, int nl, int load_end,
                                                const TSrc *img, const JobDesc &job, int s0,
                                                int wave, int lane)
{
    const int H = job.H;
    const size_t ld = static_cast<size_t>(job.ld);
    const bool mirror = !PAIR && (job.flags & JF_MIRROR);
    if (job.flags & JF_COLS) {
        const int XW = nl <= 32 ? 32 : 64;
        const int x = threadIdx.x % XW, pstep = 64 * NW / XW;
        const bool xin = x < nl;
        const int4 mine = lane_entry(pre, xin ? x : nl - 1);
        const int wend = mine.z + 64 * K;
        const TSrc *colp = img + mine.y;
        constexpr int U = COLS_AT_ONCE;
        for (int p0 = threadIdx.x / XW; p0 < load_end; p0 += pstep * U) {
            TSrc a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = min(p0 + u * pstep, load_end - 1);
                const int y = wrap<ONE>(s0 + p, H);
                const int ym = y != 0 ? H - y : 0;
                a[u] = colp[(mirror ? ym : y) * ld];
                if constexpr (PAIR) b[u] = colp[ym * ld];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + u * pstep;
                if (xin && p < load_end && p >= mine.z && p < wend)
                    lds[mine.x + p - mine.z] = image_elem<TL, TSrc, PAIR>(a[u], b[u]);
            }
        }
    } else {
        // lanes >= nl hold other entries; only lanes < nl are read (readlane)
        const int4 mine = pre;
        // RW lanes per wavefront at a time (wavefront w takes lanes w + NW i)
        constexpr int RW = ROWS_AT_ONCE;
        for (int x0 = wave; x0 < nl; x0 += RW * NW) {
            TSrc a[RW * K], b[RW * K];
#pragma unroll
            for (int q = 0; q < RW * K; ++q) {
                const int x = min(x0 + (q / K) * NW, nl - 1);
                const int k = q % K;
                const int y = wrap<ONE>(s0 + rl(mine.z, x) + 64 * k + lane, H);
                const int ym = y != 0 ? H - y : 0;
                const TSrc *rowp = img + static_cast<size_t>(rl(mine.y, x)) * ld;
                a[q] = rowp[mirror ? ym : y];
                if constexpr (PAIR) b[q] = rowp[ym];
            }
#pragma unroll
            for (int q = 0; q < RW * K; ++q) {
                const int xr = x0 + (q / K) * NW;
                const int k = q % K;
                if (xr < nl) lds[rl(mine.x, xr) + 64 * k + lane] = image_elem<TL, TSrc, PAIR>(a[q], b[q]);
            }
        }
    }
}

template <int K, int NW, typename TSrc, typename TL, bool PAIR>
__device__ __forceinline__ void load_image(TL *lds, const int4 &pre, int nl, int load_end,
                                           const TSrc *img, const JobDesc &job, int s0, int wave,
                                           int lane)
{
    if (load_end <= job.H)
        load_image_impl<K, NW, TSrc, TL, PAIR, true>(lds, pre, nl, load_end, img, job, s0, wave, lane);
    else
        load_image_impl<K, NW, TSrc, TL, PAIR, false>(lds, pre, nl, load_end, img, job, s0, wave, lane);
}

// Stores {src, row, limit, src1}: dst[row][s0 + c] = lds[src + c] for
// c < limit and s0 + c < H, plus lds[src1 + c] when MERGE (the pass root's
// last merge, done on the way out); the final output of a negative-slope
// quadrant is written back in un-mirrored position order.
// The two sums of a pair element: 16-bit halves of 32 bits, or the
// components of a 32-bit pair.
template <typename TL>
__device__ __forceinline__ uint32_t pair_lo(TL v)
{
    if constexpr (std::is_same<TL, uint2>::value) return v.x;
    else return static_cast<uint32_t>(v) & 0xffffu;
}

template <typename TL>
__device__ __forceinline__ uint32_t pair_hi(TL v)
{
    if constexpr (std::is_same<TL, uint2>::value) return v.y;
    else return static_cast<uint32_t>(v) >> 16;
}

template <int K, int NW, typename TL, typename TD, bool PAIR_OUT, bool MERGE, bool STREAM>
__device__ __forceinline__ void store_rows_impl(const TL *lds, const int4 *ent, int n, TD *dst,
                                                TD *dst2, int H, int s0, bool unmirror, int wave,
                                                int lane)
{
    for (int g = wave; g < n; g += 64 * NW) {
        const int4 mine = fetch_desc<NW>(ent, n, g, lane);
        const int m = group_size<NW>(n, g);
        for (int j = 0; j < m; ++j) {
            const int lim = min(rl(mine.z, j), H - s0);
            const TL *srcp = lds + rl(mine.x, j) + lane;
            const size_t row = static_cast<size_t>(rl(mine.y, j)) * H;
            TD *rowp = dst + row;
            TL v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = srcp[64 * k];
            if constexpr (MERGE) {
                const TL *src1 = lds + rl(mine.w, j) + lane;
                TL w[K];
#pragma unroll
                for (int k = 0; k < K; ++k) w[k] = src1[64 * k];
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] = static_cast<TL>(v[k] + w[k]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = 64 * k + lane;
                if (c < lim) {
                    const int s = s0 + c;
                    const int sm = s != 0 ? H - s : 0;
                    if constexpr (!STREAM) {
                        if constexpr (PAIR_OUT) {
                            rowp[s] = static_cast<TD>(pair_lo(v[k]));
                            dst2[row + (unmirror ? sm : s)] = static_cast<TD>(pair_hi(v[k]));
                        } else {
                            rowp[unmirror ? sm : s] = static_cast<TD>(v[k]);
                        }
                    } else if constexpr (PAIR_OUT) {
                        __builtin_nontemporal_store(static_cast<TD>(pair_lo(v[k])), rowp + s);
                        __builtin_nontemporal_store(static_cast<TD>(pair_hi(v[k])),
                                                    dst2 + row + (unmirror ? sm : s));
                    } else {
                        __builtin_nontemporal_store(static_cast<TD>(v[k]), rowp + (unmirror ? sm : s));
                    }
                }
            }
        }
    }
}

// With PAIR_OUT each pair is split into two int32 rows: the positive-slope
// sum to dst, the negative-slope sum (mirrored frame) to dst2, stored at the
// un-mirrored position when `unmirror` (the final output).
// Stores stream past the caches (rows are written once and not re-read by
// their pass), except, with `cached`, the final outputs of job-table
// launches: a batch's int32 outputs then go through L2, which merges the
// partial lines of neighbouring tiles and of the reversed negative-slope rows
// (the widening pass of a 64-image batch 8 % faster; per-image launches, whose
// last pass ends with every dirty line written back, are slower that way).
template <int K, int NW, typename TL, typename TD, bool PAIR_OUT, bool MERGE, bool CACHED_FINAL>
__device__ __forceinline__ void store_rows(const TL *lds, const int4 *ent, int n, TD *dst,
                                           TD *dst2, int H, int s0, bool unmirror, int wave,
                                           int lane, bool final_out)
{
    if constexpr (CACHED_FINAL) {
        if (final_out) {
            store_rows_impl<K, NW, TL, TD, PAIR_OUT, MERGE, false>(lds, ent, n, dst, dst2, H, s0,
                                                                    unmirror, wave, lane);
            return;
        }
    }
    store_rows_impl<K, NW, TL, TD, PAIR_OUT, MERGE, true>(lds, ent, n, dst, dst2, H, s0, unmirror,
                                                           wave, lane);
}
template <int NT, int K, typename TSrc, typename TL, typename TD, bool FROM_IMAGE, bool PAIR,
          bool TABLE>
__device__ __forceinline__ void run_item(TL *lds, cptr<int32_t> hdr, const int4 *ent,
                                         const int4 &pre, const JobDesc &job, const char *src,
                                         char *dst, char *dst2, int s0)
{
    constexpr int NW = NT / 64;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nload = hdr[kHdrLoads], nstore = hdr[kHdrStores], nsteps = hdr[kHdrSteps];
    const int H = job.H;
    constexpr bool PAIR_OUT = PAIR && sizeof(TD) == 4 && std::is_signed<TD>::value;

    // Programs of pass roots of equal widths share their entries; the lane
    // base moves the rows they name to this program's root.
    {
        const int64_t lb = hdr[kHdrLaneBase];
        const int64_t src_row = FROM_IMAGE ? ((job.flags & JF_COLS) ? 1 : job.ld) : H;
        src += lb * src_row * static_cast<int64_t>(sizeof(TSrc));
        dst += lb * H * static_cast<int64_t>(sizeof(TD));
        if constexpr (PAIR_OUT) dst2 += lb * H * static_cast<int64_t>(sizeof(TD));
    }

    // load-merge entries: the planner emits them only for LDS elements of
    // other than 4 bytes (4-byte rows are loaded straight into LDS instead)
    constexpr bool LOAD_MERGE = !FROM_IMAGE && sizeof(TL) != 4;
    const int nlm = LOAD_MERGE ? hdr[kHdrLoadMerges] : 0;

    // Descriptors of the first merge step, fetched before the loads.
    const int4 *step_ent = ent + nload + nlm;
    int cnt = nsteps > 0 ? hdr[kHdrStepCounts] : 0;
    int4 cur = fetch_desc<NW>(step_ent, cnt, wave, lane);

    if constexpr (FROM_IMAGE) {
        load_image<K, NW, TSrc, TL, PAIR>(lds, pre, nload, hdr[kHdrLoadEnd],
                                          reinterpret_cast<const TSrc *>(src), job, s0, wave, lane);
    } else {
        load_rows<K, NW, TSrc, TL>(lds, ent, nload, reinterpret_cast<const TSrc *>(src), H, s0,
                                   wave, lane);
        if constexpr (LOAD_MERGE)
            load_merges<K, NW, TSrc, TL>(lds, ent + nload, nlm, reinterpret_cast<const TSrc *>(src),
                                         H, s0, wave, lane);
        __builtin_amdgcn_s_waitcnt(0);  // direct-to-LDS loads have landed
    }

    for (int k = 0; k < nsteps; ++k) {
        __syncthreads();
        const int4 *next_ent = step_ent + cnt;
        const int next_cnt = k + 1 < nsteps ? hdr[kHdrStepCounts + k + 1] : 0;
        const int4 nxt = fetch_desc<NW>(next_ent, next_cnt, wave, lane);
        if (wave < cnt) merge_group<K, TL>(lds, cur, group_size<NW>(cnt, wave), lane);
        for (int g = wave + 64 * NW; g < cnt; g += 64 * NW)
            merge_group<K, TL>(lds, fetch_desc<NW>(step_ent, cnt, g, lane), group_size<NW>(cnt, g),
                               lane);
        step_ent = next_ent;
        cnt = next_cnt;
        cur = nxt;
    }
    __syncthreads();

    const bool final_out = (job.flags & JF_FINAL) != 0;
    const bool unmirror = final_out && (PAIR_OUT || (job.flags & JF_MIRROR));
    // int32 outputs of job-table launches are stored through L2 (see store_rows)
    constexpr bool CACHED = TABLE && std::is_same<TD, int32_t>::value;
    if (hdr[kHdrStoreMerge])  // the stores add the root's last merge
        store_rows<K, NW, TL, TD, PAIR_OUT, true, CACHED>(
            lds, step_ent, nstore, reinterpret_cast<TD *>(dst), reinterpret_cast<TD *>(dst2), H, s0,
            unmirror, wave, lane, final_out);
    else
        store_rows<K, NW, TL, TD, PAIR_OUT, false, CACHED>(
            lds, step_ent, nstore, reinterpret_cast<TD *>(dst), reinterpret_cast<TD *>(dst2), H, s0,
            unmirror, wave, lane, final_out);
}

// TSrc / TL / TD: element types read, kept in LDS and written (see Combo).
// TABLE: jobs come from a device table (batches) instead of kernel arguments.
//
// Workgroup b runs item (b mod 8) * ceil(n / 8) + b / 8: workgroups are
// dealt to the eight XCDs round robin, so this gives each XCD a contiguous
// range of items and neighbouring tiles, which read overlapping rows, share
// an L2.
template <int NT, typename TSrc, typename TL, typename TD, bool FROM_IMAGE, bool TABLE, bool PAIR>
__global__ void __launch_bounds__(NT) fht_pass_kernel(PassArgs args, int n_items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TL *lds = reinterpret_cast<TL *>(smem_raw);

    const int per_xcd = (n_items + 7) / 8;
    const int it = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (it >= n_items) return;
    const E4 item = ld4(as_const(reinterpret_cast<const int32_t *>(args.items)), it);
    const JobDesc job = pick_job<TABLE>(args, item.y);
    cptr<int32_t> hdr = as_const(job.hdrs) + static_cast<size_t>(item.x) * kHdrInts;
    // The item names its program's first entry, so the first pass fetches
    // its load entries (one per lane of the root, at most 64) together with
    // the header instead of after it; the tables end with spare entries, so
    // this never reads past them.
    const int4 *ent = job.ops + item.w;
    int4 pre = make_int4(0, 0, 0, 0);
    if constexpr (FROM_IMAGE) pre = ent[threadIdx.x & 63];

    const char *src = static_cast<const char *>(job.src);
    if (job.flags & JF_SRC_WS) src = args.ws + reinterpret_cast<uintptr_t>(job.src);
    char *dst = static_cast<char *>(job.dst);
    char *dst2 = static_cast<char *>(job.dst2);
    if (job.flags & JF_DST_WS) {
        dst = args.ws + reinterpret_cast<uintptr_t>(job.dst);
        dst2 = args.ws + reinterpret_cast<uintptr_t>(job.dst2);
    }
    if constexpr (!TABLE) {
        // image blockIdx.y of a same-shape batch
        const int64_t b = blockIdx.y;
        src += b * (FROM_IMAGE ? args.img_stride : args.ws_stride);
        const int64_t od = b * ((job.flags & JF_FINAL) ? args.out_stride : args.ws_stride);
        dst += od;
        dst2 += od;
    }
    switch (hdr[kHdrChunks]) {
    case 1: run_item<NT, 1, TSrc, TL, TD, FROM_IMAGE, PAIR, TABLE>(lds, hdr, ent, pre, job, src, dst, dst2, item.z); break;
    case 2: run_item<NT, 2, TSrc, TL, TD, FROM_IMAGE, PAIR, TABLE>(lds, hdr, ent, pre, job, src, dst, dst2, item.z); break;
    case 3: run_item<NT, 3, TSrc, TL, TD, FROM_IMAGE, PAIR, TABLE>(lds, hdr, ent, pre, job, src, dst, dst2, item.z); break;
    default: run_item<NT, 4, TSrc, TL, TD, FROM_IMAGE, PAIR, TABLE>(lds, hdr, ent, pre, job, src, dst, dst2, item.z); break;
    }
}

template <int NT, typename TSrc, typename TL, typename TD, bool FROM_IMAGE, bool PAIR>
hipError_t launch_nt(const PassArgs &args, int n_items, int lds_bytes, hipStream_t stream,
                     int n_images)
{
    const dim3 grid((n_items + 7) / 8 * 8, n_images), block(NT);
    if (args.jobs)
        fht_pass_kernel<NT, TSrc, TL, TD, FROM_IMAGE, true, PAIR><<<grid, block, lds_bytes, stream>>>(args, n_items);
    else
        fht_pass_kernel<NT, TSrc, TL, TD, FROM_IMAGE, false, PAIR><<<grid, block, lds_bytes, stream>>>(args, n_items);
    return hipGetLastError();
}

template <typename TSrc, typename TL, typename TD, bool FROM_IMAGE, bool PAIR = false>
hipError_t launch_typed(const PassArgs &args, int n_items, int lds_bytes, int threads,
                        hipStream_t stream, int n_images)
{
    if (threads == 512)
        return launch_nt<512, TSrc, TL, TD, FROM_IMAGE, PAIR>(args, n_items, lds_bytes, stream,
                                                              n_images);
    return launch_nt<256, TSrc, TL, TD, FROM_IMAGE, PAIR>(args, n_items, lds_bytes, stream,
                                                          n_images);
}

}  // namespace

hipError_t launch_pass(Combo combo, const PassArgs &args, int n, int lds, int threads,
                       hipStream_t stream, int n_images)
{
    if (n <= 0 || n_images <= 0) return hipSuccess;
    switch (combo) {
    case Combo::U8_U16_U16: return launch_typed<uint8_t, uint16_t, uint16_t, true>(args, n, lds, threads, stream, n_images);
    case Combo::U8_U16_I32: return launch_typed<uint8_t, uint16_t, int32_t, true>(args, n, lds, threads, stream, n_images);
    case Combo::U16_U16_U16: return launch_typed<uint16_t, uint16_t, uint16_t, false>(args, n, lds, threads, stream, n_images);
    case Combo::U16_U16_I32: return launch_typed<uint16_t, uint16_t, int32_t, false>(args, n, lds, threads, stream, n_images);
    case Combo::U16_I32_I32: return launch_typed<uint16_t, int32_t, int32_t, false>(args, n, lds, threads, stream, n_images);
    case Combo::I32_I32_I32: return launch_typed<int32_t, int32_t, int32_t, false>(args, n, lds, threads, stream, n_images);
    case Combo::F32_FIRST: return launch_typed<float, float, float, true>(args, n, lds, threads, stream, n_images);
    case Combo::F32_LATER: return launch_typed<float, float, float, false>(args, n, lds, threads, stream, n_images);
    case Combo::F64_FIRST: return launch_typed<double, double, double, true>(args, n, lds, threads, stream, n_images);
    case Combo::F64_LATER: return launch_typed<double, double, double, false>(args, n, lds, threads, stream, n_images);
    case Combo::P_U8_FIRST: return launch_typed<uint8_t, uint32_t, uint32_t, true, true>(args, n, lds, threads, stream, n_images);
    case Combo::P_U8_FIRST_FINAL: return launch_typed<uint8_t, uint32_t, int32_t, true, true>(args, n, lds, threads, stream, n_images);
    case Combo::P_U16_MID: return launch_typed<uint32_t, uint32_t, uint32_t, false, true>(args, n, lds, threads, stream, n_images);
    case Combo::P_U16_MID_FINAL: return launch_typed<uint32_t, uint32_t, int32_t, false, true>(args, n, lds, threads, stream, n_images);
    case Combo::P_I32: return launch_typed<uint32_t, uint2, int32_t, false, true>(args, n, lds, threads, stream, n_images);
    }
    return hipErrorInvalidValue;
}

}  // namespace fht
