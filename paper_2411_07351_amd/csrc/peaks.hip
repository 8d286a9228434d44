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

// A candidate's key is its flat output index (quadrants are stored in q
// order, so keys order candidates by quadrant, then slope, then shift).
constexpr uint64_t kNoKey = ~0ull;

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
        a.keys[slot] = a.base[qi] + e;
}

// (value, key) beats (bv, bk): larger value, then smaller flat index.  Every
// output type converts to double exactly, so the order is the values' own.
__device__ __forceinline__ bool beats(double v, uint64_t k, double bv, uint64_t bk)
{
    return bk == kNoKey || v > bv || (v == bv && k < bk);
}

constexpr int kSelThreads = 1024;
constexpr int kSortCap = 8192;  // candidates sorted in LDS at once (k <= 4096 of them wanted)

// Order-preserving 64-bit image of a value (larger value, larger image; -0
// and +0 are one value, as in the comparison above).
__device__ __forceinline__ uint64_t ordered(double v)
{
    if (v == 0.0) v = 0.0;
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ bool before(uint64_t va, uint64_t ka, uint64_t vb, uint64_t kb)
{
    return va > vb || (va == vb && ka < kb);
}

// The selection's view of the arguments, in scalars: a candidate's quadrant
// slot follows from comparing its key with the slots' first flat indices
// (slots past the last present one start at the largest key), never from
// indexing the argument arrays by a per-lane slot, which would copy them to
// scratch memory.
template <typename T>
struct SelView {
    const T *flat;
    uint64_t b0, b1, b2, b3;
    int h0, h1, h2, h3, q0, q1, q2, q3;

    __device__ explicit SelView(const PeakArgs &a)
        : flat(static_cast<const T *>(a.flat)), b0(a.base[0]),
          b1(a.nq > 1 ? a.base[1] : kNoKey), b2(a.nq > 2 ? a.base[2] : kNoKey),
          b3(a.nq > 3 ? a.base[3] : kNoKey), h0(a.H[0]), h1(a.H[1]), h2(a.H[2]), h3(a.H[3]),
          q0(a.quadrant[0]), q1(a.quadrant[1]), q2(a.quadrant[2]), q3(a.quadrant[3]) {}

    __device__ __forceinline__ double value(uint64_t key) const
    {
        return static_cast<double>(flat[key]);
    }

    // Slot s holds the keys from b_s on, and b1 <= b2 <= b3: a key at or past
    // b3 is past b2 and b1 too, so the fields follow by adding differences
    // (a chain of selects would become an indexed load of this object).
    __device__ __forceinline__ PeakOut peak(uint64_t key, double v) const
    {
        const int i1 = key >= b1, i2 = key >= b2, i3 = key >= b3;
        const uint64_t base = b0 + i1 * (b1 - b0) + i2 * (b2 - b1) + i3 * (b3 - b2);
        const uint64_t e = key - base;
        const int H = h0 + i1 * (h1 - h0) + i2 * (h2 - h1) + i3 * (h3 - h2);
        PeakOut p;
        p.value = static_cast<float>(v);
        p.quadrant = q0 + i1 * (q1 - q0) + i2 * (q2 - q1) + i3 * (q3 - q2);
        p.t = static_cast<int32_t>(e / H);
        p.s = static_cast<int32_t>(e % H);
        return p;
    }
};

// The k strongest candidates (value descending, then flat output index
// ascending).  At most kSortCap candidates: all of them are sorted in LDS
// (bitonic).  More: a radix select over the values' ordered images (8 bits
// a round) finds the k-th largest value first, and only the candidates at or
// above it are sorted; if those are still too many (a tie at that value
// spanning thousands of candidates), k rounds of a workgroup argmax, each
// removing its winner, pick them instead.
template <typename T>
__global__ void __launch_bounds__(kSelThreads) peaks_select_kernel(PeakArgs a)
{
    __shared__ uint64_t sv[kSortCap], sk[kSortCap];
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sh_prefix, sh_mask;
    __shared__ uint32_t sh_kk, sh_count;
    __shared__ double best_v[kSelThreads / 64];
    __shared__ uint64_t best_k[kSelThreads / 64];
    const uint32_t total = a.counter[0];
    const int m = static_cast<int>(min(total, static_cast<uint32_t>(a.capacity)));
    const int k = min(a.k, m);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const SelView<T> view(a);
    uint64_t *keys = a.keys;
    PeakOut *out = a.out;

    // threshold: the ordered value of the k-th largest candidate (every
    // candidate when they all fit)
    uint64_t thr = 0;
    if (m > kSortCap) {
        if (tid == 0) {
            sh_prefix = 0;
            sh_mask = 0;
            sh_kk = static_cast<uint32_t>(k);
        }
        for (int shift = 56; shift >= 0; shift -= 8) {
            for (int b = tid; b < 256; b += kSelThreads) hist[b] = 0;
            __syncthreads();
            const uint64_t prefix = sh_prefix, mask = sh_mask;
            for (int i = tid; i < m; i += kSelThreads) {
                const uint64_t ov = ordered(view.value(keys[i]));
                if ((ov & mask) == prefix) atomicAdd(&hist[(ov >> shift) & 255], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t kk = sh_kk;
                for (int b = 255; b >= 0; --b) {
                    if (kk <= hist[b]) {
                        sh_prefix = prefix | (static_cast<uint64_t>(b) << shift);
                        sh_mask = mask | (0xffull << shift);
                        break;
                    }
                    kk -= hist[b];
                }
                sh_kk = kk;
            }
            __syncthreads();
        }
        thr = sh_prefix;
    }
    // collect the candidates at or above the threshold
    if (tid == 0) sh_count = 0;
    __syncthreads();
    for (int i = tid; i < m; i += kSelThreads) {
        const uint64_t key = keys[i];
        const uint64_t ov = ordered(view.value(key));
        if (ov >= thr) {
            const uint32_t slot = atomicAdd(&sh_count, 1u);
            if (slot < static_cast<uint32_t>(kSortCap)) {
                sv[slot] = ov;
                sk[slot] = key;
            }
        }
    }
    __syncthreads();
    const uint32_t got = sh_count;
    int found = 0;
    if (got <= static_cast<uint32_t>(kSortCap)) {
        // bitonic sort of the collected candidates, padded to a power of two
        // with entries that sort last
        int n = 1;
        while (n < static_cast<int>(got)) n <<= 1;
        for (int i = static_cast<int>(got) + tid; i < n; i += kSelThreads) {
            sv[i] = 0;
            sk[i] = kNoKey;
        }
        __syncthreads();
        for (int size = 2; size <= n; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = tid; i < n / 2; i += kSelThreads) {
                    const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t vl = sv[lo], kl = sk[lo], vh = sv[hi], kh = sk[hi];
                    if (before(vh, kh, vl, kl) == up) {
                        sv[lo] = vh;
                        sk[lo] = kh;
                        sv[hi] = vl;
                        sk[hi] = kl;
                    }
                }
                __syncthreads();
            }
        }
        for (int i = tid; i < k; i += kSelThreads) out[i] = view.peak(sk[i], view.value(sk[i]));
        found = k;
    } else {
        for (int round = 0; round < k; ++round) {
            double bv = 0.0;
            uint64_t bk = kNoKey;
            for (int i = tid; i < m; i += kSelThreads) {
                const uint64_t kx = keys[i];
                if (kx == kNoKey) continue;
                const double v = view.value(kx);
                if (beats(v, kx, bv, bk)) {
                    bv = v;
                    bk = kx;
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
            for (int i = tid; i < m; i += kSelThreads)
                if (keys[i] == tk) keys[i] = kNoKey;
            if (tid == 0) out[round] = view.peak(tk, tv);
            ++found;
            __syncthreads();
        }
    }
    if (tid == 0) {
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
