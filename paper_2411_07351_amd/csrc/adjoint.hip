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
// 2^levels rows per output row, adjacent rows sharing them in L2).  A final
// launch adds the quadrants' lane gradients into the image gradient,
// transposing the column-lane quadrants through LDS.  Memory-bound gathers:
// no MFMA.
#include "kernels.hpp"

namespace fht {

namespace {

constexpr int kRowsPerBlock = 4;  // one wavefront per output row

template <typename T>
__global__ void __launch_bounds__(256) adj_step_kernel(AdjArgs args)
{
    const AdjJob &job = args.job[blockIdx.y];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x * kRowsPerBlock + wave;
    if (x >= job.W) return;
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
    // four terms times up to four 64-position chunks of loads in flight
    // together; the last group of a row takes only the chunks it covers
    for (int s0 = 0; s0 < H; s0 += 256) {
        const int nu = min(4, (H - s0 + 63) >> 6);
        T acc[4] = {T(0), T(0), T(0), T(0)};
        for (int tb = t0; tb < t1; tb += 64) {
            const int m = min(64, t1 - tb);
            const int2 mine = tb == t0 ? first : (lane < m ? job.terms[tb + lane] : make_int2(0, 0));
            for (int j0 = 0; j0 < m; j0 += 4) {
                T v[4][4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int j = min(j0 + jj, m - 1);
                    const int rowi = __builtin_amdgcn_readlane(mine.x, j);
                    const int sh = __builtin_amdgcn_readlane(mine.y, j);
                    const T *row = src + static_cast<size_t>(rowi) * H;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (u >= nu) break;
                        const int s = min(s0 + 64 * u + lane, H - 1);
                        int y = s - sh;
                        if (y < 0) y += H;
                        if (mirror && y != 0) y = H - y;
                        v[jj][u] = row[y];
                    }
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    if (j0 + jj < m) {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (u < nu) acc[u] += v[jj][u];
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + 64 * u + lane;
            if (s < H) __builtin_nontemporal_store(acc[u], dst + s);
        }
    }
}

constexpr int kTile = 64;

// grad[i][j] = sum over present quadrants of their lane gradient at (i, j):
// q0/q1 read g[i][j'] (lanes are rows), q2/q3 read g[j][i'] (lanes are
// columns), primes marking mirrored positions where asked.  A block covers a
// 64 x 64 tile; column-lane quadrants are staged transposed in LDS.
template <typename T>
__global__ void __launch_bounds__(256) adj_combine_kernel(CombineArgs args)
{
    __shared__ T tile[kTile][kTile + 1];
    const int R = args.R, C = args.C;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    const int tj = threadIdx.x & 63, ti = threadIdx.x >> 6;  // 64 x 4 threads
    T acc[kTile / 4];
#pragma unroll
    for (int k = 0; k < kTile / 4; ++k) acc[k] = T(0);
    const int j = j0 + tj;
    const int64_t b = blockIdx.z;  // image of a same-shape batch
    for (int q = 0; q < 2; ++q) {
        const T *g = args.src[q] ? reinterpret_cast<const T *>(static_cast<const char *>(args.src[q]) +
                                                               b * args.src_stride[q])
                                 : nullptr;
        if (!g || j >= C) continue;
        const int jj = (args.mirror[q] && j != 0) ? C - j : j;
#pragma unroll
        for (int k = 0; k < kTile / 4; ++k) {
            const int i = i0 + ti + 4 * k;
            if (i < R) acc[k] += g[static_cast<size_t>(i) * C + jj];
        }
    }
    for (int q = 2; q < 4; ++q) {
        const T *g = args.src[q] ? reinterpret_cast<const T *>(static_cast<const char *>(args.src[q]) +
                                                               b * args.src_stride[q])
                                 : nullptr;
        if (!g) continue;  // uniform across the block
        // stage g[j0 + a][i'(i0 + b)] as tile[a][b], threads along b
        const int b = threadIdx.x & 63;
        const int i = i0 + b;
        const int ii = (args.mirror[q] && i != 0) ? R - i : i;
        for (int a = threadIdx.x >> 6; a < kTile; a += 4) {
            const int jr = j0 + a;
            tile[a][b] = (jr < C && i < R) ? g[static_cast<size_t>(jr) * R + ii] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTile / 4; ++k) acc[k] += tile[tj][ti + 4 * k];
        __syncthreads();
    }
    T *out = reinterpret_cast<T *>(static_cast<char *>(args.dst) + b * args.dst_stride);
    if (j < C) {
#pragma unroll
        for (int k = 0; k < kTile / 4; ++k) {
            const int i = i0 + ti + 4 * k;
            if (i < R) out[static_cast<size_t>(i) * C + j] = acc[k];
        }
    }
}

}  // namespace

hipError_t launch_adjoint_step(Real real, const AdjArgs &args, int n_jobs, int max_w,
                               hipStream_t stream, int n_images)
{
    if (n_jobs <= 0 || max_w <= 0 || n_images <= 0) return hipSuccess;
    const dim3 grid((max_w + kRowsPerBlock - 1) / kRowsPerBlock, n_jobs, n_images), block(256);
    if (real == Real::F64)
        adj_step_kernel<double><<<grid, block, 0, stream>>>(args);
    else
        adj_step_kernel<float><<<grid, block, 0, stream>>>(args);
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

}  // namespace fht
