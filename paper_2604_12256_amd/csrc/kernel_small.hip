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

// Each thread owns the amplitudes i = tid + u * blockDim (u < kPer) and
// computes their new values from the LDS state (output-stationary): for a
// dense gate, out[i] = sum_c M[r(i)][c] s[base(i) | off(c)] where r(i)
// collects the gate-qubit bits of i; all outputs are computed before any is
// written back (one barrier), so register use does not grow with 2^k.
template <typename R>
__device__ __forceinline__ void run_small(const SmallItem &it)
{
    using V = c2_t<R>;
    constexpr int kPer = (kSmallLdsBytes / sizeof(V)) / kSmallThreads;  // 16 (c128) / 32 (c64)
    extern __shared__ char smem_raw[];
    V *s = reinterpret_cast<V *>(smem_raw);
    const int n = (int)it.n;
    const uint32_t len = 1u << n;
    V *gstate = reinterpret_cast<V *>(it.state);
    const R *tables = reinterpret_cast<const R *>(it.tables);
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
        const GateDesc *g = it.gates + gi;
        const uint32_t k = g->k;
        const R *m = tables + 2 * g->table;
        uint32_t gmask = 0;
        for (uint32_t t = 0; t < k; ++t) gmask |= 1u << g->q[t];
        if (g->diag) {
            for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
                uint32_t y = 0;
                for (uint32_t t = 0; t < k; ++t) y |= ((i >> g->q[t]) & 1u) << t;
                s[i] = cmul(s[i], ldc<R>(m, y));
            }
        } else {
            const uint32_t d = 1u << k;
            V out[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const uint32_t i = threadIdx.x + (uint32_t)u * blockDim.x;
                if (i < len) {
                    uint32_t r = 0;
                    for (uint32_t t = 0; t < k; ++t) r |= ((i >> g->q[t]) & 1u) << t;
                    const uint32_t base = i & ~gmask;
                    V acc;
                    acc.x = R(0);
                    acc.y = R(0);
                    for (uint32_t c = 0; c < d; ++c) {
                        uint32_t o = base;
                        for (uint32_t t = 0; t < k; ++t)
                            if ((c >> t) & 1u) o |= 1u << g->q[t];
                        cmac(acc, ldc<R>(m, (uint64_t)r * d + c), s[o]);
                    }
                    out[u] = acc;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const uint32_t i = threadIdx.x + (uint32_t)u * blockDim.x;
                if (i < len) s[i] = out[u];
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
