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

// A candidate's key is its quadrant slot (bits 48..) and its index in that
// quadrant: quadrants are stored in q order, so keys order candidates by their
// flat output index.
constexpr uint64_t kNoKey = ~0ull;
constexpr int kKeySlotShift = 48;

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
    if (slot < static_cast<uint32_t>(a.capacity))
        a.keys[slot] = (static_cast<uint64_t>(qi) << kKeySlotShift) | e;
}

template <typename T>
__device__ __forceinline__ double key_value(const PeakArgs &a, uint64_t key)
{
    const int qi = static_cast<int>(key >> kKeySlotShift);
    const size_t e = key & ((1ull << kKeySlotShift) - 1);
    const void *src = qi == 0 ? a.src[0] : qi == 1 ? a.src[1] : qi == 2 ? a.src[2] : a.src[3];
    return static_cast<double>(static_cast<const T *>(src)[e]);
}

// (value, key) beats (bv, bk): larger value, then smaller flat index.  Every
// output type converts to double exactly, so the order is the values' own.
__device__ __forceinline__ bool beats(double v, uint64_t k, double bv, uint64_t bk)
{
    return bk == kNoKey || v > bv || (v == bv && k < bk);
}

constexpr int kSelThreads = 1024;

// The k strongest candidates (value descending, then flat output index
// ascending) by k rounds of a workgroup argmax; each round removes its
// winner.
template <typename T>
__global__ void __launch_bounds__(kSelThreads) peaks_select_kernel(PeakArgs a)
{
    __shared__ double best_v[kSelThreads / 64];
    __shared__ uint64_t best_k[kSelThreads / 64];
    const uint32_t total = a.counter[0];
    const int m = static_cast<int>(min(total, static_cast<uint32_t>(a.capacity)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int found = 0;
    for (int round = 0; round < a.k; ++round) {
        double bv = 0.0;
        uint64_t bk = kNoKey;
        for (int i = threadIdx.x; i < m; i += kSelThreads) {
            const uint64_t k = a.keys[i];
            if (k == kNoKey) continue;
            const double v = key_value<T>(a, k);
            if (beats(v, k, bv, bk)) {
                bv = v;
                bk = k;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const uint64_t ok = __shfl_xor(bk, off, 64);
            if (ok != kNoKey && beats(ov, ok, bv, bk)) {
                bv = ov;
                bk = ok;
            }
        }
        if (lane == 0) {
            best_v[wave] = bv;
            best_k[wave] = bk;
        }
        __syncthreads();
        double tv = 0.0;
        uint64_t tk = kNoKey;
        for (int w = 0; w < kSelThreads / 64; ++w)
            if (best_k[w] != kNoKey && beats(best_v[w], best_k[w], tv, tk)) {
                tv = best_v[w];
                tk = best_k[w];
            }
        __syncthreads();
        if (tk == kNoKey) break;
        // remove the winner (keys are unique: they hold the output index)
        for (int i = threadIdx.x; i < m; i += kSelThreads)
            if (a.keys[i] == tk) a.keys[i] = kNoKey;
        if (threadIdx.x == 0) {
            const int qi = static_cast<int>(tk >> kKeySlotShift);
            const uint64_t e = tk & ((1ull << kKeySlotShift) - 1);
            const int H = qi == 0 ? a.H[0] : qi == 1 ? a.H[1] : qi == 2 ? a.H[2] : a.H[3];
            PeakOut p;
            p.value = static_cast<float>(tv);
            p.quadrant = qi == 0 ? a.quadrant[0] : qi == 1 ? a.quadrant[1]
                       : qi == 2 ? a.quadrant[2] : a.quadrant[3];
            p.t = static_cast<int32_t>(e / H);
            p.s = static_cast<int32_t>(e % H);
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

hipError_t launch_peaks(PeakElem elem, const PeakArgs &args, size_t max_elems, hipStream_t stream)
{
    if (max_elems > (static_cast<size_t>(0x7fffffff) * 256)) return hipErrorInvalidValue;
    peaks_clear_kernel<<<1, 64, 0, stream>>>(args.counter);
    const dim3 grid(static_cast<unsigned>((max_elems + 255) / 256), args.nq), block(256);
    switch (elem) {
    case PeakElem::I32:
        if (max_elems > 0) peaks_nms_kernel<int32_t><<<grid, block, 0, stream>>>(args);
        peaks_select_kernel<int32_t><<<1, kSelThreads, 0, stream>>>(args);
        break;
    case PeakElem::F32:
        if (max_elems > 0) peaks_nms_kernel<float><<<grid, block, 0, stream>>>(args);
        peaks_select_kernel<float><<<1, kSelThreads, 0, stream>>>(args);
        break;
    case PeakElem::F64:
        if (max_elems > 0) peaks_nms_kernel<double><<<grid, block, 0, stream>>>(args);
        peaks_select_kernel<double><<<1, kSelThreads, 0, stream>>>(args);
        break;
    }
    return hipGetLastError();
}

}  // namespace fht
