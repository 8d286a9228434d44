// gfx950 kernels of the dyadic-pattern fast Hough transform.
//
// One launch executes one fused pass of Alg. 1 for many work items.  A work
// item (one workgroup) runs a planner-made program: it loads the rows its
// slope tile needs from HBM into LDS, runs the merge steps of Alg. 1 (row t
// of a node = row t0 of the left child + row t1 of the right child rotated by
// t - t1) entirely in LDS, and writes its output rows back.  The rotation is
// folded into LDS addresses, so every merge is a contiguous vector add;
// waves take whole rows and lanes take consecutive positions, which keeps LDS
// accesses bank-conflict free and HBM accesses coalesced.  This is a
// memory-bound integer or float add: no MFMA.
#include "kernels.hpp"

namespace fht {

namespace {

template <bool TABLE>
__device__ __forceinline__ JobDesc pick_job(const PassArgs &a, int j)
{
    if constexpr (TABLE) return a.jobs[j];
    switch (j) {
    case 0: return a.inl[0];
    case 1: return a.inl[1];
    case 2: return a.inl[2];
    default: return a.inl[3];
    }
}

// TABLE: jobs come from a device table (batches) instead of kernel arguments.
template <typename TSrc, typename TAcc, bool FROM_IMAGE, bool TABLE>
__global__ void __launch_bounds__(kBlockThreads) fht_pass_kernel(PassArgs args)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TAcc *lds = reinterpret_cast<TAcc *>(smem_raw);

    const int4 item = args.items[blockIdx.x];
    const int32_t *hdr = args.hdrs + static_cast<size_t>(item.x) * 32;
    const int first = hdr[0], nload = hdr[1], nstore = hdr[2], nsteps = hdr[3];
    const JobDesc job = pick_job<TABLE>(args, item.y);
    const int H = job.H;
    const int s0 = item.z;
    const int4 *ops = args.ops + first;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    constexpr int nw = kBlockThreads / 64;

    const char *src = static_cast<const char *>(job.src);
    if (job.flags & JF_SRC_WS) src = args.ws + reinterpret_cast<uintptr_t>(job.src);
    char *dst = static_cast<char *>(job.dst);
    if (job.flags & JF_DST_WS) dst = args.ws + reinterpret_cast<uintptr_t>(job.dst);

    // Load phase: lds[d + c] = src[row][(s0 + off + c) mod H].
    for (int i = wave; i < nload; i += nw) {
        const int4 op = ops[i];
        int base = s0 + op.z;
        if (base >= H) base %= H;
        for (int c = lane; c < op.w; c += 64) {
            int pos = base + c;
            if (pos >= H) pos -= H;
            if (pos >= H) pos %= H;
            TAcc v;
            if constexpr (FROM_IMAGE) {
                int y = pos;
                if ((job.flags & JF_MIRROR) && y != 0) y = H - y;
                const size_t addr = (job.flags & JF_COLS)
                                        ? static_cast<size_t>(y) * job.ld + op.y
                                        : static_cast<size_t>(op.y) * job.ld + y;
                v = static_cast<TAcc>(reinterpret_cast<const TSrc *>(src)[addr]);
            } else {
                v = reinterpret_cast<const TAcc *>(src)[static_cast<size_t>(op.y) * H + pos];
            }
            lds[op.x + c] = v;
        }
    }

    // Merge steps of Alg. 1: lds[d + c] = lds[a + c] + lds[b + c].
    int k0 = nload;
    for (int k = 0; k < nsteps; ++k) {
        __syncthreads();
        const int cnt = hdr[8 + k];
        for (int i = wave; i < cnt; i += nw) {
            const int4 op = ops[k0 + i];
            for (int c = lane; c < op.w; c += 64)
                lds[op.x + c] = lds[op.y + c] + lds[op.z + c];
        }
        k0 += cnt;
    }
    __syncthreads();

    // Store phase: dst[row][s0 + c] for s0 + c < H (final output un-mirrored).
    const int limit = H - s0;
    const bool unmirror = (job.flags & JF_FINAL) && (job.flags & JF_MIRROR);
    TAcc *out = reinterpret_cast<TAcc *>(dst);
    for (int i = wave; i < nstore; i += nw) {
        const int4 op = ops[k0 + i];
        const int n = op.w < limit ? op.w : limit;
        TAcc *row = out + static_cast<size_t>(op.y) * H;
        for (int c = lane; c < n; c += 64) {
            int s = s0 + c;
            if (unmirror && s != 0) s = H - s;
            row[s] = lds[op.x + c];
        }
    }
}

}  // namespace

template <typename TSrc, typename TAcc>
hipError_t launch_typed(bool from_image, const PassArgs &args, int n_items, int lds_bytes,
                        hipStream_t stream)
{
    const dim3 grid(n_items), block(kBlockThreads);
    const bool table = args.jobs != nullptr;
    if (from_image) {
        if (table)
            fht_pass_kernel<TSrc, TAcc, true, true><<<grid, block, lds_bytes, stream>>>(args);
        else
            fht_pass_kernel<TSrc, TAcc, true, false><<<grid, block, lds_bytes, stream>>>(args);
    } else {
        if (table)
            fht_pass_kernel<TAcc, TAcc, false, true><<<grid, block, lds_bytes, stream>>>(args);
        else
            fht_pass_kernel<TAcc, TAcc, false, false><<<grid, block, lds_bytes, stream>>>(args);
    }
    return hipGetLastError();
}

hipError_t launch_pass(Dt dt, bool from_image, const PassArgs &args, int n_items,
                       int lds_bytes, hipStream_t stream)
{
    if (n_items <= 0) return hipSuccess;
    switch (dt) {
    case Dt::U8: return launch_typed<uint8_t, int32_t>(from_image, args, n_items, lds_bytes, stream);
    case Dt::F32: return launch_typed<float, float>(from_image, args, n_items, lds_bytes, stream);
    case Dt::F64: return launch_typed<double, double>(from_image, args, n_items, lds_bytes, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fht
