// gfx950 kernels of the adjoint (back-projection) of the dyadic-pattern fast
// Hough transform.
//
// The transform is linear: out[t][s] = sum_x A[x][(s + pat_t(x)) mod H] for
// every quadrant view A (Sec. 3; negative slopes run in a mirrored position
// frame).  Its adjoint sends an output gradient G back along the same
// patterns.  It is computed by running the merges of Alg. 1 backwards: each
// lane row of a child gathers the contiguous range of parent rows that read
// it, the right child's rows rotated back by the shift they were given.
// Several levels go in one launch as a gather over the composed terms (about
// 2^levels rows per output row, adjacent rows sharing them in L2).  The last
// gather of every quadrant runs in one final launch that also adds the
// quadrants' lane gradients into the image gradient, transposing the
// column-lane quadrants through LDS, so the last lane gradients never go to
// memory; where that launch would have too few tiles to fill the chip (one
// small image), the last gathers run as their own launch and a combine
// launch adds the lane gradients.  Memory-bound gathers: no MFMA.
#include "kernels.hpp"

namespace fht {

namespace {

constexpr int kRowsPerBlock = 8;  // one wavefront per output row
constexpr int kLoadsAtOnce = 32;  // loads of a wavefront in flight together

// CH: 64-position chunks of a row per round of loads (4, or 8 for rows of
// up to 512 positions, which then take one round instead of two); terms
// whose loads are in flight together: kLoadsAtOnce / CH.  The rows go in the
// job's order: rows that read the same source rows (the descendants of one
// node at the same relative slope) share a workgroup, and so its L1.
template <typename T, int CH>
__global__ void __launch_bounds__(64 * kRowsPerBlock) adj_step_kernel(AdjArgs args)
{
    constexpr int kTermsAtOnce = kLoadsAtOnce / CH;
    const AdjJob &job = args.job[blockIdx.y];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * kRowsPerBlock + wave;
    if (slot >= job.W) return;
    const int x = job.order[slot];
    const int H = job.H;
    const int64_t b = blockIdx.z;  // image of a same-shape batch
    const T *src = reinterpret_cast<const T *>(static_cast<const char *>(job.src) + b * args.src_stride);
    T *dst = reinterpret_cast<T *>(static_cast<char *>(job.dst) + b * args.dst_stride) +
             static_cast<size_t>(x) * H;
    const bool mirror = job.mirror_in != 0;
    const int t0 = job.offs[x], t1 = job.offs[x + 1];
    // The row's terms reach the wavefront 64 at a time through one vector
    // load and are broadcast with readlane, so no load waits per term.
    const int m0 = min(64, t1 - t0);
    const int2 first = lane < m0 ? job.terms[t0 + lane] : make_int2(0, 0);
    // terms times up to CH 64-position chunks of loads in flight together
    // (three fused levels give about eight terms per row); the last round of
    // a row takes only the chunks it covers
    for (int s0 = 0; s0 < H; s0 += 64 * CH) {
        const int nu = min(CH, (H - s0 + 63) >> 6);
        T acc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) acc[u] = T(0);
        for (int tb = t0; tb < t1; tb += 64) {
            const int m = min(64, t1 - tb);
            const int2 mine = tb == t0 ? first : (lane < m ? job.terms[tb + lane] : make_int2(0, 0));
            for (int j0 = 0; j0 < m; j0 += kTermsAtOnce) {
                T v[kTermsAtOnce][CH];
#pragma unroll
                for (int jj = 0; jj < kTermsAtOnce; ++jj) {
                    const int j = min(j0 + jj, m - 1);
                    const int rowi = __builtin_amdgcn_readlane(mine.x, j);
                    const int sh = __builtin_amdgcn_readlane(mine.y, j);
                    const T *row = src + static_cast<size_t>(rowi) * H;
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        if (u >= nu) break;
                        const int s = min(s0 + 64 * u + lane, H - 1);
                        int y = s - sh;
                        if (y < 0) y += H;
                        if (mirror && y != 0) y = H - y;
                        v[jj][u] = row[y];
                    }
                }
#pragma unroll
                for (int jj = 0; jj < kTermsAtOnce; ++jj)
                    if (j0 + jj < m) {
#pragma unroll
                        for (int u = 0; u < CH; ++u)
                            if (u < nu) acc[u] += v[jj][u];
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int s = s0 + 64 * u + lane;
            if (s < H) __builtin_nontemporal_store(acc[u], dst + s);
        }
    }
}

constexpr int kTile = 64;

// Lane gradient of quadrant job `a` (positive slope) plus that of `b` (the
// negative slope of the same lane view, mirrored frame) at lane x (uniform
// across the wavefront) and position p (per lane): the view's last gather,
// the terms of row x shared by both quadrants.
template <typename T>
__device__ __forceinline__ T view_gather(const FinalJob &a, const FinalJob &b, int x, int H, int p,
                                         int lane)
{
    const T *sa = static_cast<const T *>(a.src), *sb = static_cast<const T *>(b.src);
    const int pa = p;
    const int pb = (b.out_mirror && p != 0) ? H - p : p;
    const FinalJob &t = sa ? a : b;
    if (!t.offs) {  // no tree levels: the lane gradient is the output gradient
        T v = T(0);
        if (sa) v += sa[static_cast<size_t>(x) * H + pa];
        if (sb) v += sb[static_cast<size_t>(x) * H + pb];
        return v;
    }
    constexpr int TA = 8;  // terms whose loads (two quadrants each) are in flight together
    const int t0 = t.offs[x], t1 = t.offs[x + 1];
    T acc = T(0);
    for (int tb = t0; tb < t1; tb += 64) {
        const int m = min(64, t1 - tb);
        const int2 mine = lane < m ? t.terms[tb + lane] : make_int2(0, 0);
        for (int j0 = 0; j0 < m; j0 += TA) {
            T va[TA], vb[TA];
#pragma unroll
            for (int jj = 0; jj < TA; ++jj) {
                const int j = min(j0 + jj, m - 1);
                const size_t row = static_cast<size_t>(__builtin_amdgcn_readlane(mine.x, j)) * H;
                const int sh = __builtin_amdgcn_readlane(mine.y, j);
                int ya = pa - sh, yb = pb - sh;
                if (ya < 0) ya += H;
                if (yb < 0) yb += H;
                if (a.in_mirror && ya != 0) ya = H - ya;
                if (b.in_mirror && yb != 0) yb = H - yb;
                va[jj] = sa ? sa[row + ya] : T(0);
                vb[jj] = sb ? sb[row + yb] : T(0);
            }
#pragma unroll
            for (int jj = 0; jj < TA; ++jj)
                if (j0 + jj < m) acc += va[jj] + vb[jj];
        }
    }
    return acc;
}

// view_gather for NR rows x0 + r xstep (r < nrows <= NR, uniform across the
// wavefront) at once: each round issues the loads of TA terms of every row
// (two quadrants each), so NR times as many loads are in flight as in the
// single-row form.  Rows of more than 64 terms (Split_T's wide fan-in) take
// the single-row form.
template <typename T, int NR>
__device__ __forceinline__ void view_gather_rows(const FinalJob &a, const FinalJob &b, int x0,
                                                 int xstep, int nrows, int H, int p, int lane,
                                                 T (&out)[NR])
{
    const T *sa = static_cast<const T *>(a.src), *sb = static_cast<const T *>(b.src);
    const FinalJob &t = sa ? a : b;
    const int pa = p;
    const int pb = (b.out_mirror && p != 0) ? H - p : p;
    if (!t.offs) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            out[r] = r < nrows ? view_gather<T>(a, b, x0 + r * xstep, H, p, lane) : T(0);
        return;
    }
    int t0[NR], m[NR];
    int mmax = 0;
    bool small = true;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int x = x0 + (r < nrows ? r : 0) * xstep;
        t0[r] = t.offs[x];
        m[r] = r < nrows ? t.offs[x + 1] - t0[r] : 0;
        mmax = max(mmax, m[r]);
        small = small && m[r] <= 64;
    }
    if (!small) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            out[r] = r < nrows ? view_gather<T>(a, b, x0 + r * xstep, H, p, lane) : T(0);
        return;
    }
    int2 mine[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        mine[r] = lane < m[r] ? t.terms[t0[r] + lane] : make_int2(0, 0);
    constexpr int TA = 4;
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = T(0);
    for (int j0 = 0; j0 < mmax; j0 += TA) {
        T va[NR][TA], vb[NR][TA];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int jj = 0; jj < TA; ++jj) {
                // a term past the row's last repeats the last one (in bounds); it is not added
                const int j = min(j0 + jj, max(m[r] - 1, 0));
                const size_t row = static_cast<size_t>(__builtin_amdgcn_readlane(mine[r].x, j)) * H;
                const int sh = __builtin_amdgcn_readlane(mine[r].y, j);
                int ya = pa - sh, yb = pb - sh;
                if (ya < 0) ya += H;
                if (yb < 0) yb += H;
                if (a.in_mirror && ya != 0) ya = H - ya;
                if (b.in_mirror && yb != 0) yb = H - yb;
                va[r][jj] = sa ? sa[row + ya] : T(0);
                vb[r][jj] = sb ? sb[row + yb] : T(0);
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int jj = 0; jj < TA; ++jj)
                if (j0 + jj < m[r]) acc[r] += va[r][jj] + vb[r][jj];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r] = acc[r];
}


// grad[i][j] = sum over present quadrants of their lane gradient at (i, j):
// q0/q1 read g[i][j'] (lanes are rows), q2/q3 read g[j][i'] (lanes are
// columns), primes marking mirrored positions where asked.  A block covers a
// 64 x 64 tile; column-lane quadrants are staged transposed in LDS.
template <typename T>
__global__ void __launch_bounds__(256) adj_combine_kernel(CombineArgs args)
{
    __shared__ T tile[kTile][kTile + 1];
    constexpr int KR = kTile / 4;  // rows per thread
    const int R = args.R, C = args.C;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    const int tj = threadIdx.x & 63, ti = threadIdx.x >> 6;  // 64 x 4 threads
    const int64_t b = blockIdx.z;  // image of a same-shape batch
    auto source = [&](int q) -> const T * {
        return args.src[q] ? reinterpret_cast<const T *>(static_cast<const char *>(args.src[q]) +
                                                         b * args.src_stride[q])
                           : nullptr;
    };
    // Row-lane quadrants: every load of the thread is issued before the adds.
    const T *g0 = source(0), *g1 = source(1);
    const int j = j0 + tj;
    T acc[KR];
    {
        const int jc = min(j, C - 1);
        const int jj0 = (args.mirror[0] && jc != 0) ? C - jc : jc;
        const int jj1 = (args.mirror[1] && jc != 0) ? C - jc : jc;
        T v0[KR], v1[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const size_t row = static_cast<size_t>(min(i0 + ti + 4 * k, R - 1)) * C;
            v0[k] = g0 ? g0[row + jj0] : T(0);
            v1[k] = g1 ? g1[row + jj1] : T(0);
        }
#pragma unroll
        for (int k = 0; k < KR; ++k) acc[k] = v0[k] + v1[k];
    }
    // Column-lane quadrants: both are staged, summed, as tile[a][c] =
    // g[j0 + a][i'(i0 + c)] with threads along c, then read transposed.
    const T *g2 = source(2), *g3 = source(3);
    if (g2 || g3) {  // uniform across the block
        const int c = threadIdx.x & 63;
        const int i = min(i0 + c, R - 1);
        const int ii2 = (args.mirror[2] && i != 0) ? R - i : i;
        const int ii3 = (args.mirror[3] && i != 0) ? R - i : i;
        T v2[KR], v3[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const size_t row = static_cast<size_t>(min(j0 + ti + 4 * k, C - 1)) * R;
            v2[k] = g2 ? g2[row + ii2] : T(0);
            v3[k] = g3 ? g3[row + ii3] : T(0);
        }
#pragma unroll
        for (int k = 0; k < KR; ++k) tile[ti + 4 * k][c] = v2[k] + v3[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; ++k) acc[k] += tile[tj][ti + 4 * k];
    }
    T *out = reinterpret_cast<T *>(static_cast<char *>(args.dst) + b * args.dst_stride);
    if (j < C) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int i = i0 + ti + 4 * k;
            if (i < R) out[static_cast<size_t>(i) * C + j] = acc[k];
        }
    }
}

// grad[i][j] = sum over present quadrants of their lane gradient at (i, j),
// each computed here by its last gather: q0/q1 at lane i, position j'
// (lanes are rows), q2/q3 at lane j, position i' (lanes are columns), primes
// marking mirrored positions.  A block of eight wavefronts covers a 64 x 64
// tile; each wavefront gathers eight rows of each lane view, one position
// per lane, and the column-lane rows are staged in LDS and read transposed.
template <typename T>
__global__ void __launch_bounds__(512) adj_final_kernel(FinalArgs args)
{
    __shared__ T tile[kTile][kTile + 1];
    constexpr int KR = kTile / 8;  // rows per wavefront
    const int R = args.R, C = args.C;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t b = blockIdx.z;  // image of a same-shape batch
    FinalJob q[kInlineJobs];
#pragma unroll
    for (int k = 0; k < kInlineJobs; ++k) {
        q[k] = args.q[k];
        if (q[k].src) q[k].src = static_cast<const char *>(q[k].src) + b * q[k].src_stride;
    }
    // rows wave + 8 k of the tile, four at a time (k = 4 g + r)
    constexpr int NR = 4;
    T acc[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) acc[k] = T(0);
    if (q[0].src || q[1].src) {  // uniform across the block
        const int jc = min(j0 + lane, C - 1);
#pragma unroll
        for (int g = 0; g < KR / NR; ++g) {
            const int x0 = i0 + wave + 8 * NR * g;
            const int n = x0 < R ? min(NR, (R - 1 - x0) / 8 + 1) : 0;
            T v[NR];
            if (n > 0) {
                view_gather_rows<T, NR>(q[0], q[1], x0, 8, n, C, jc, lane, v);
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[NR * g + r] = v[r];
            }
        }
    }
    if (q[2].src || q[3].src) {
        const int ic = min(i0 + lane, R - 1);
#pragma unroll
        for (int g = 0; g < KR / NR; ++g) {
            const int x0 = j0 + wave + 8 * NR * g;
            const int n = x0 < C ? min(NR, (C - 1 - x0) / 8 + 1) : 0;
            T v[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = T(0);
            if (n > 0) view_gather_rows<T, NR>(q[2], q[3], x0, 8, n, R, ic, lane, v);
#pragma unroll
            for (int r = 0; r < NR; ++r) tile[wave + 8 * (NR * g + r)][lane] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; ++k) acc[k] += tile[lane][wave + 8 * k];
    }
    T *out = reinterpret_cast<T *>(static_cast<char *>(args.dst) + b * args.dst_stride);
    const int j = j0 + lane;
    if (j < C) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int i = i0 + wave + 8 * k;
            if (i < R) out[static_cast<size_t>(i) * C + j] = acc[k];
        }
    }
}

}  // namespace

hipError_t launch_adjoint_step(Real real, const AdjArgs &args, int n_jobs, int max_w,
                               hipStream_t stream, int n_images, int max_h)
{
    if (n_jobs <= 0 || max_w <= 0 || n_images <= 0) return hipSuccess;
    const dim3 grid((max_w + kRowsPerBlock - 1) / kRowsPerBlock, n_jobs, n_images),
        block(64 * kRowsPerBlock);
    const bool wide = max_h > 256;  // rows of 257..512 positions: one round of 8 chunks
    if (real == Real::F64) {
        if (wide) adj_step_kernel<double, 8><<<grid, block, 0, stream>>>(args);
        else adj_step_kernel<double, 4><<<grid, block, 0, stream>>>(args);
    } else {
        if (wide) adj_step_kernel<float, 8><<<grid, block, 0, stream>>>(args);
        else adj_step_kernel<float, 4><<<grid, block, 0, stream>>>(args);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_combine(Real real, const CombineArgs &args, hipStream_t stream,
                                  int n_images)
{
    if (n_images <= 0) return hipSuccess;
    const dim3 grid((args.C + kTile - 1) / kTile, (args.R + kTile - 1) / kTile, n_images),
        block(256);
    if (real == Real::F64)
        adj_combine_kernel<double><<<grid, block, 0, stream>>>(args);
    else
        adj_combine_kernel<float><<<grid, block, 0, stream>>>(args);
    return hipGetLastError();
}

hipError_t launch_adjoint_final(Real real, const FinalArgs &args, hipStream_t stream,
                                int n_images)
{
    if (n_images <= 0) return hipSuccess;
    const dim3 grid((args.C + kTile - 1) / kTile, (args.R + kTile - 1) / kTile, n_images),
        block(512);
    if (real == Real::F64)
        adj_final_kernel<double><<<grid, block, 0, stream>>>(args);
    else
        adj_final_kernel<float><<<grid, block, 0, stream>>>(args);
    return hipGetLastError();
}

}  // namespace fht
