// Small-state kernel: one workgroup runs a whole gate list on a state that
// fits in LDS (2^n amplitudes, n <= 13 for complex128 and n <= 14 for
// complex64 in 128 KiB).  Used for the merge booster's sub-states (Sec. 4.4:
// entanglement-free gate blocks simulated on small sub-state vectors) and for
// batching many small circuits into one launch (one workgroup per circuit).
#include "device.hpp"

namespace qs {

namespace {

constexpr int kSmallThreads = 512;
constexpr uint32_t kSmallLdsBytes = 128u * 1024u;

template <typename R, int K>
__device__ __forceinline__ void small_dense(c2_t<R> *s, int n, const GateDesc &g, const QS_CONST R *m)
{
    using V = c2_t<R>;
    constexpr int D = 1 << K;
    const uint64_t ng = 1ull << (n - K);
    uint32_t offq[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        uint32_t o = 0;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if ((r >> t) & 1) o |= 1u << g.q[t];
        offq[r] = o;
    }
    for (uint64_t grp = threadIdx.x; grp < ng; grp += blockDim.x) {
        const uint32_t base = (uint32_t)insert_zeros<K>(grp, g.sorted);
        V v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = s[base | offq[c]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc = cmul(ldc<R>(m, (uint64_t)(r * D)), v[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac(acc, ldc<R>(m, (uint64_t)(r * D + c)), v[c]);
            s[base | offq[r]] = acc;
        }
    }
}

template <typename R>
__device__ __forceinline__ void run_small(const SmallItem &it)
{
    using V = c2_t<R>;
    extern __shared__ char smem_raw[];
    V *s = reinterpret_cast<V *>(smem_raw);
    const int n = (int)it.n;
    const uint32_t len = 1u << n;
    V *gstate = reinterpret_cast<V *>(it.state);
    const QS_CONST R *tables = as_const(reinterpret_cast<const R *>(it.tables));
    const GateDesc *gates = it.gates;
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        if (it.init) {
            V v;
            v.x = i == 0 ? R(1) : R(0);
            v.y = R(0);
            s[i] = v;
        } else {
            s[i] = gstate[i];
        }
    }
    __syncthreads();
    for (uint32_t gi = 0; gi < it.ngates; ++gi) {
        const GateDesc g = gates[gi];
        const QS_CONST R *m = tables + 2 * g.table;
        if (g.diag) {
            for (uint32_t x = threadIdx.x; x < len; x += blockDim.x) {
                uint32_t y = 0;
                for (uint32_t t = 0; t < g.k; ++t) y |= ((x >> g.q[t]) & 1u) << t;
                s[x] = cmul(s[x], ldc<R>(m, y));
            }
        } else {
            switch (g.k) {
            case 1: small_dense<R, 1>(s, n, g, m); break;
            case 2: small_dense<R, 2>(s, n, g, m); break;
            case 3: small_dense<R, 3>(s, n, g, m); break;
            case 4: small_dense<R, 4>(s, n, g, m); break;
            case 5: small_dense<R, 5>(s, n, g, m); break;
            default: small_dense<R, 6>(s, n, g, m); break;
            }
        }
        __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) gstate[i] = s[i];
}

template <typename R>
__global__ __launch_bounds__(kSmallThreads) void k_small(const SmallItem *__restrict__ items)
{
    run_small<R>(items[blockIdx.x]);
}

// Items addressed by pointer (kernel argument), one workgroup each: circuits
// of different contexts batched into one launch without a shared device list.
template <typename R>
__global__ __launch_bounds__(kSmallThreads) void k_small_ptrs(SmallPtrs P)
{
    run_small<R>(*P.item[blockIdx.x]);
}

}  // namespace

int small_max_qubits(bool c128) { return c128 ? 13 : 14; }

template <typename R>
hipError_t launch_small_batch(const SmallItem *items_dev, uint32_t count, uint32_t max_n, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const uint32_t bytes = (uint32_t)sizeof(c2_t<R>) << max_n;
    if (bytes > kSmallLdsBytes) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_small<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kSmallLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    k_small<R><<<count, kSmallThreads, bytes, s>>>(items_dev);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_small_ptrs(const SmallPtrs &P, uint32_t count, uint32_t max_n, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    if (count > (uint32_t)kSmallBatchMax) return hipErrorInvalidValue;
    const uint32_t bytes = (uint32_t)sizeof(c2_t<R>) << max_n;
    if (bytes > kSmallLdsBytes) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_small_ptrs<R>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    k_small_ptrs<R><<<count, kSmallThreads, bytes, s>>>(P);
    return hipGetLastError();
}

template hipError_t launch_small_ptrs<double>(const SmallPtrs &, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_small_ptrs<float>(const SmallPtrs &, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_small_batch<double>(const SmallItem *, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_small_batch<float>(const SmallItem *, uint32_t, uint32_t, hipStream_t);

}  // namespace qs
