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
constexpr int kTermsAtOnce = 8;   // terms whose loads are in flight together

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
    // eight terms times up to four 64-position chunks of loads in flight
    // together (three fused levels give about eight terms per row); the last
    // group of a row takes only the chunks it covers
    for (int s0 = 0; s0 < H; s0 += 256) {
        const int nu = min(4, (H - s0 + 63) >> 6);
        T acc[4] = {T(0), T(0), T(0), T(0)};
        for (int tb = t0; tb < t1; tb += 64) {
            const int m = min(64, t1 - tb);
            const int2 mine = tb == t0 ? first : (lane < m ? job.terms[tb + lane] : make_int2(0, 0));
            for (int j0 = 0; j0 < m; j0 += kTermsAtOnce) {
                T v[kTermsAtOnce][4];
#pragma unroll
                for (int jj = 0; jj < kTermsAtOnce; ++jj) {
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
                for (int jj = 0; jj < kTermsAtOnce; ++jj)
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
