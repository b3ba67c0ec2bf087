// Measurement on the state vector: the projective model in which the
// operator M_i^j keeps the amplitudes whose qubit j is i (the paper's
// measurement background, Sec. 2).  Three operations:
//
// * collapse of one qubit to an outcome, renormalised (one pass);
// * shot sampling by the inverse of the cumulative distribution in logical
//   index order, for caller-supplied uniforms (a marginal over the top
//   logical qubits picks the block, then one workgroup per needed block
//   scans it);
// * expectation values of Z strings, <psi| Z_S |psi> = sum_x |a_x|^2 (-1)^|x & S|.
//
// Every sum is FP64 in a fixed order, so results are deterministic.
#include <algorithm>

#include "device.hpp"

namespace qs {

namespace {

constexpr int kBlock = 256;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_collapse(c2_t<R> *__restrict__ a, uint64_t len, uint64_t bit,
                                                     uint64_t want, R scale)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < len; x += stride) {
        c2_t<R> v;
        if ((x & bit) == want) {
            v = a[x];
            v.x *= scale;
            v.y *= scale;
        } else {
            v.x = (R)0;
            v.y = (R)0;
        }
        a[x] = v;
    }
}

// One workgroup per needed block of 2^nlow consecutive logical indices.
// Thread t owns the segment [t 2^seg, (t+1) 2^seg) of the block; segment
// sums and their prefix are formed in a fixed order, then every shot of the
// block finds its segment by bisection and its index by a sequential scan.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_sample(const c2_t<R> *__restrict__ a, SampleArgs S,
                                                   const uint64_t *__restrict__ tabs,
                                                   const uint64_t *__restrict__ bases,
                                                   const uint64_t *__restrict__ ids,
                                                   const uint32_t *__restrict__ start,
                                                   const double *__restrict__ resid, uint64_t *__restrict__ out)
{
    __shared__ uint64_t tl[512], th[512];
    __shared__ double P[kBlock];
    for (int i = threadIdx.x; i < 512; i += kBlock) {
        tl[i] = tabs[i];
        th[i] = tabs[512 + i];
    }
    __syncthreads();
    const uint32_t bi = blockIdx.x;
    const uint64_t base = bases[bi];
    const uint32_t t = threadIdx.x;
    const uint64_t L = 1ull << S.seg_log2;
    auto prob = [&](uint64_t w) {
        const c2_t<R> v = a[base | tl[w & 511] | th[w >> 9]];
        const double re = (double)v.x, im = (double)v.y;
        return re * re + im * im;
    };
    double s = 0.0;
    if (t < S.nthr)
        for (uint64_t k = 0; k < L; ++k) s += prob(((uint64_t)t << S.seg_log2) + k);
    P[t] = s;
    __syncthreads();
    if (t == 0) {
        double acc = 0.0;
        for (int i = 0; i < S.nthr; ++i) {
            acc += P[i];
            P[i] = acc;
        }
    }
    __syncthreads();
    const int nthr = S.nthr;
    for (uint32_t j = start[bi] + t; j < start[bi + 1]; j += kBlock) {
        double r = resid[j];
        int seg;
        if (!(r < P[nthr - 1])) {
            // rounding put the target past this block's own total: take the
            // last segment with mass, and in it the last amplitude with mass
            seg = nthr - 1;
            while (seg > 0 && !(P[seg] > P[seg - 1])) --seg;
            r = P[seg];
        } else {
            int lo = 0, hi = nthr - 1;  // smallest i with P[i] > r
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (P[mid] > r) hi = mid;
                else lo = mid + 1;
            }
            seg = lo;
        }
        double acc = seg ? P[seg - 1] : 0.0;
        const uint64_t w0 = (uint64_t)seg << S.seg_log2;
        uint64_t pick = w0, last_pos = w0;
        bool found = false;
        for (uint64_t k = 0; k < L; ++k) {
            const double p = prob(w0 + k);
            if (p > 0.0) last_pos = w0 + k;
            acc += p;
            if (acc > r) {
                pick = w0 + k;
                found = true;
                break;
            }
        }
        if (!found) pick = last_pos;
        out[j] = (ids[bi] << S.nlow) | pick;
    }
}

constexpr uint32_t kZBlocks = 2048;

// The sign (-1)^popcount(x & m) splits into a per-lane factor (the six lane
// bits of x, fixed for the whole launch since the stride is a multiple of
// 64) and a wave-uniform one (the bits above), computed once per iteration
// in scalar registers: two FP64 operations per mask and amplitude.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_expect_z_partial(const c2_t<R> *__restrict__ a, uint64_t len, ZArgs Z,
                                                             double *__restrict__ part)
{
    __shared__ double sh[kBlock];
    double acc[kZMasksPerLaunch], lane_sign[kZMasksPerLaunch];
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int k = 0; k < kZMasksPerLaunch; ++k) {
        acc[k] = 0.0;
        lane_sign[k] = (__popc(lane & (uint32_t)Z.m[k] & 63u) & 1) ? -1.0 : 1.0;
    }
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    // first index of this wave's 64 consecutive amplitudes (wave-uniform)
    uint64_t xw = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u);
    xw = wave_uniform_u64(xw);
    for (; xw < len; xw += stride) {
        double p = 0.0;
        if (xw + lane < len) {  // states below 64 amplitudes fill part of one wave
            const c2_t<R> v = a[xw + lane];
            const double re = (double)v.x, im = (double)v.y;
            p = re * re + im * im;
        }
#pragma unroll
        for (int k = 0; k < kZMasksPerLaunch; ++k)
            if (k < Z.nm) {
                const double us = (__popcll(xw & Z.m[k]) & 1) ? -p : p;  // wave-uniform sign
                acc[k] = fma(lane_sign[k], us, acc[k]);
            }
    }
    for (int k = 0; k < Z.nm; ++k) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < kZMasksPerLaunch; ++u)
            if (u == k) v = acc[u];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int h = kBlock / 2; h >= 1; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(uint64_t)blockIdx.x * Z.nm + k] = sh[0];
        __syncthreads();
    }
}

// One workgroup per mask: fixed strided sums over the partials, then a
// fixed tree.
__global__ __launch_bounds__(kBlock) void k_expect_z_final(const double *__restrict__ part, uint32_t nblocks,
                                                           int nm, double *__restrict__ out)
{
    __shared__ double sh[kBlock];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) acc += part[(uint64_t)b * nm + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
}

uint32_t grid_for(uint64_t len)
{
    uint64_t b = (len + kBlock - 1) / kBlock;
    if (b > (1ull << 20)) b = 1ull << 20;
    return (uint32_t)(b ? b : 1);
}

}  // namespace

template <typename R>
hipError_t launch_collapse(void *state, int n, int phys_qubit, int outcome, double scale, hipStream_t s)
{
    if (phys_qubit < 0 || phys_qubit >= n || (outcome != 0 && outcome != 1)) return hipErrorInvalidValue;
    const uint64_t len = 1ull << n, bit = 1ull << phys_qubit;
    k_collapse<R><<<grid_for(len), kBlock, 0, s>>>((c2_t<R> *)state, len, bit, outcome ? bit : 0ull, (R)scale);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sample(const void *state, const SampleArgs &S, uint32_t nblocks, const uint64_t *tabs,
                         const uint64_t *bases, const uint64_t *ids, const uint32_t *start, const double *resid,
                         uint64_t *out, hipStream_t s)
{
    if (nblocks == 0) return hipSuccess;
    if (S.nlow < 0 || S.nlow > 18 || S.nthr < 1 || S.nthr > kBlock || S.seg_log2 < 0 ||
        ((uint64_t)S.nthr << S.seg_log2) != (1ull << S.nlow))
        return hipErrorInvalidValue;
    k_sample<R><<<nblocks, kBlock, 0, s>>>((const c2_t<R> *)state, S, tabs, bases, ids, start, resid, out);
    return hipGetLastError();
}

size_t expect_z_scratch_bytes() { return (size_t)kZBlocks * kZMasksPerLaunch * sizeof(double); }

template <typename R>
hipError_t launch_expect_z(const void *state, int n, const ZArgs &Z, double *out, double *scratch, hipStream_t s)
{
    if (Z.nm < 1 || Z.nm > kZMasksPerLaunch) return hipErrorInvalidValue;
    const uint64_t len = 1ull << n;
    uint32_t nb = (uint32_t)std::min<uint64_t>(kZBlocks, (len + kBlock - 1) / kBlock);
    k_expect_z_partial<R><<<nb, kBlock, 0, s>>>((const c2_t<R> *)state, len, Z, scratch);
    k_expect_z_final<<<Z.nm, kBlock, 0, s>>>(scratch, nb, Z.nm, out);
    return hipGetLastError();
}

#define QS_INSTANTIATE_MEASURE(R)                                                                          \
    template hipError_t launch_collapse<R>(void *, int, int, int, double, hipStream_t);                  \
    template hipError_t launch_sample<R>(const void *, const SampleArgs &, uint32_t, const uint64_t *,    \
                                         const uint64_t *, const uint64_t *, const uint32_t *,            \
                                         const double *, uint64_t *, hipStream_t);                       \
    template hipError_t launch_expect_z<R>(const void *, int, const ZArgs &, double *, double *, hipStream_t);
QS_INSTANTIATE_MEASURE(double)
QS_INSTANTIATE_MEASURE(float)

}  // namespace qs
