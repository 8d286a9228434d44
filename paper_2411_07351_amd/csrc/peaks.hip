// gfx950 kernels of peak finding on the quadrant Hough images: strict local
// maxima (ties broken by position) above a floor, then the k strongest.
//
// A straight segment in the image concentrates its pixels on one output
// J_q[t][s] (the pattern of slope t through shift s, Sec. 3), so lines are
// found as isolated maxima.  Neighbourhoods are (2 radius + 1)^2 windows in
// (t, s) of one quadrant: s wraps around (lines wrap, Alg. 1), t does not.
#include "kernels.hpp"

namespace fht {

namespace {

__device__ __forceinline__ uint32_t order_bits(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float from_order_bits(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void peaks_clear_kernel(uint32_t *counter) { if (threadIdx.x == 0) counter[0] = 0; }

// One thread per output element of one quadrant (grid.y = quadrant slot).
template <typename T>
__global__ void __launch_bounds__(256) peaks_nms_kernel(PeakArgs a)
{
    const int qi = blockIdx.y;
    const T *img = static_cast<const T *>(a.src[qi]);
    const int W = a.W[qi], H = a.H[qi];
    const size_t n = static_cast<size_t>(W) * H;
    const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const T v = img[e];
    if (static_cast<double>(v) < a.min_value) return;
    const int t = static_cast<int>(e / H), s = static_cast<int>(e % H);
    const int r = a.radius;
    for (int dt = -r; dt <= r; ++dt) {
        const int tt = t + dt;
        if (tt < 0 || tt >= W) continue;
        for (int ds = -r; ds <= r; ++ds) {
            if (dt == 0 && ds == 0) continue;
            int ss = s + ds;
            ss = ((ss % H) + H) % H;
            const size_t f = static_cast<size_t>(tt) * H + ss;
            if (f == e) continue;  // the window wrapped onto the element itself
            const T u = img[f];
            // strict maximum; equal neighbours earlier in the row-major order win
            if (u > v || (u == v && f < e)) return;
        }
    }
    const uint32_t slot = atomicAdd(a.counter, 1u);
    if (slot < static_cast<uint32_t>(a.capacity)) {
        const uint64_t idx = a.base[qi] + e;
        a.keys[slot] = (static_cast<uint64_t>(order_bits(static_cast<float>(v))) << 32) |
                       (0xffffffffull - idx);
    }
}

constexpr int kSelThreads = 1024;

// The k largest keys (value, then smaller output index) by k rounds of a
// workgroup argmax; each round removes its winner.
__global__ void __launch_bounds__(kSelThreads) peaks_select_kernel(PeakArgs a)
{
    __shared__ uint64_t best[kSelThreads / 64];
    const uint32_t total = a.counter[0];
    const int m = static_cast<int>(min(total, static_cast<uint32_t>(a.capacity)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int found = 0;
    for (int round = 0; round < a.k; ++round) {
        uint64_t mine = 0;
        for (int i = threadIdx.x; i < m; i += kSelThreads) mine = max(mine, a.keys[i]);
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(mine, off, 64);
            mine = max(mine, o);
        }
        if (lane == 0) best[wave] = mine;
        __syncthreads();
        uint64_t top = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) top = max(top, best[w]);
        __syncthreads();
        if (top == 0) break;
        // remove the winner (keys are unique: they hold the output index)
        for (int i = threadIdx.x; i < m; i += kSelThreads)
            if (a.keys[i] == top) a.keys[i] = 0;
        if (threadIdx.x == 0) {
            const uint64_t idx = 0xffffffffull - (top & 0xffffffffull);
            int q = 0;
            for (int j = 1; j < a.nq; ++j)
                if (idx >= a.base[j]) q = j;
            const uint64_t rel = idx - a.base[q];
            PeakOut p;
            p.value = from_order_bits(static_cast<uint32_t>(top >> 32));
            p.quadrant = a.quadrant[q];
            p.t = static_cast<int32_t>(rel / a.H[q]);
            p.s = static_cast<int32_t>(rel % a.H[q]);
            a.out[round] = p;
        }
        ++found;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.n_found[0] = found;
        a.n_found[1] = static_cast<int32_t>(min(total, 0x7fffffffu));
    }
}

}  // namespace

hipError_t launch_peaks(PeakElem elem, const PeakArgs &args, int max_elems, hipStream_t stream)
{
    peaks_clear_kernel<<<1, 64, 0, stream>>>(args.counter);
    if (max_elems > 0) {
        const dim3 grid((max_elems + 255) / 256, args.nq), block(256);
        switch (elem) {
        case PeakElem::I32: peaks_nms_kernel<int32_t><<<grid, block, 0, stream>>>(args); break;
        case PeakElem::F32: peaks_nms_kernel<float><<<grid, block, 0, stream>>>(args); break;
        case PeakElem::F64: peaks_nms_kernel<double><<<grid, block, 0, stream>>>(args); break;
        }
    }
    peaks_select_kernel<<<1, kSelThreads, 0, stream>>>(args);
    return hipGetLastError();
}

}  // namespace fht
