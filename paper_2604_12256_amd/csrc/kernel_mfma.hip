// Dense k-qubit gate (k = 3, 4, 5) on the matrix cores: a batched GEMM.
//
// For every group of 2^k amplitudes that differ only in the gate's qubits
// (Sec. 2.2), y = U x.  Written in real arithmetic on interleaved (re, im)
// vectors, y_r = M_r x_r with the 2^(k+1) x 2^(k+1) real matrix
//   M_r[2r][2c] = Re U[r][c],  M_r[2r][2c+1] = -Im U[r][c],
//   M_r[2r+1][2c] = Im U[r][c], M_r[2r+1][2c+1] = Re U[r][c],
// so a wave computes Y = M_r X for 16 groups at once (X: 2^(k+1) x 16) with
// 16x16x4 MFMA steps: complex64 states on FP32 MFMA, complex128 on FP64 MFMA.
//
// Operand layout of the 16x16x4 MFMA (one block): lane l = j + 16 q holds
// A[j][q] and B[q][j] of each k-step.  Accumulator v of lane l holds
// D[4q + v][j] for the FP32 instruction and D[4v + q][j] for the FP64 one
// (output groups of 4 rows vs 1 row per lane block).  Every lane keeps its
// slice of M_r in registers for the whole launch.
#include "device.hpp"

namespace qs {

namespace {

constexpr int kMfmaThreads = 256;

template <typename R> struct Mfma;
template <> struct Mfma<float> {
    static constexpr bool kRowsPerLaneContiguous = true;   // D[4q + v][j]
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    static constexpr bool kRowsPerLaneContiguous = false;  // D[4v + q][j]
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename R, int K>
__global__ __launch_bounds__(kMfmaThreads) void k_dense_mfma(c2_t<R> *__restrict__ a, const R *__restrict__ mr,
                                                             uint64_t nbatches, GateDesc g)
{
    using V = c2_t<R>;
    using acc_t = typename Mfma<R>::acc_t;
    constexpr int D = 2 << K;   // real dimension
    constexpr int T = D / 16;   // 16-row output tiles
    constexpr int S = D / 4;    // k-steps of 4
    const uint32_t lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;

    R areg[T][S];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int s = 0; s < S; ++s) areg[t][s] = mr[(16 * t + j) * D + 4 * s + q];

    // amplitude offset of matrix index c (bit t of c <-> qubit q[t])
    auto off = [&](int c) {
        uint64_t o = 0;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if ((c >> t) & 1) o |= 1ull << g.q[t];
        return o;
    };
    // B row 4s + q is part q%2 of amplitude 2s + q/2: a wave-uniform offset
    // (matrix index 2s) plus the lane's bit for q/2 (gate qubit 0); offsets
    // count scalar parts (R), so a lane loads only the part it uses.
    const uint64_t lane_in = ((uint64_t)(q >> 1) << g.q[0]) * 2 + (q & 1);
    // Output amplitudes written by this lane, two per tile:
    //  rows 16t + 4q + v (FP32): amplitudes 8t + 2q + {0, 1}, (re, im) = (v0, v1), (v2, v3);
    //  rows 16t + 4v + q (FP64): lane holds re (q even) or im (q odd) of amplitudes
    //  8t + 2v + q/2; the partner lane l ^ 16 holds the other part, so even-q lanes
    //  write v = 0, 1 and odd-q lanes v = 2, 3.
    uint64_t out_off[T][2];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (Mfma<R>::kRowsPerLaneContiguous) {
            out_off[t][0] = off(8 * t + 2 * (int)q);
            out_off[t][1] = off(8 * t + 2 * (int)q + 1);
        } else {
            const int v0 = (q & 1) ? 2 : 0;
            out_off[t][0] = off(8 * t + 2 * v0 + (int)(q >> 1));
            out_off[t][1] = off(8 * t + 2 * (v0 + 1) + (int)(q >> 1));
        }
    }

    const R *ap = reinterpret_cast<const R *>(a);
    auto load_b = [&](uint64_t bb, R *bv) {
        const uint64_t base2 = insert_zeros<K>(bb * 16 + j, g.sorted) * 2 + lane_in;
#pragma unroll
        for (int s = 0; s < S; ++s) bv[s] = ap[base2 + off(2 * s) * 2];
    };
    const uint64_t wave = ((uint64_t)blockIdx.x * kMfmaThreads + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kMfmaThreads) >> 6;
    // the next batch's operands are loaded while this batch's products run
    constexpr bool kPrefetch = true;
    R bv[S], bn[S];
    if (wave < nbatches) load_b(wave, bv);
    for (uint64_t b = wave; b < nbatches; b += nwaves) {
        if constexpr (kPrefetch) {
            if (b + nwaves < nbatches) load_b(b + nwaves, bn);
        }
        const uint64_t base = insert_zeros<K>(b * 16 + j, g.sorted);
        acc_t acc[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            acc[t] = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int s = 0; s < S; ++s) acc[t] = Mfma<R>::mma(areg[t][s], bv[s], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            V y0, y1;
            if (Mfma<R>::kRowsPerLaneContiguous) {
                y0.x = acc[t][0];
                y0.y = acc[t][1];
                y1.x = acc[t][2];
                y1.y = acc[t][3];
            } else {
                R mine[4], other[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    mine[v] = acc[t][v];
                    other[v] = __shfl_xor(mine[v], 16, 64);
                }
                if ((q & 1) == 0) {  // own = re, partner = im; amplitudes of v = 0, 1
                    y0.x = mine[0];
                    y0.y = other[0];
                    y1.x = mine[1];
                    y1.y = other[1];
                } else {             // own = im, partner = re; amplitudes of v = 2, 3
                    y0.x = other[2];
                    y0.y = mine[2];
                    y1.x = other[3];
                    y1.y = mine[3];
                }
            }
            a[base | out_off[t][0]] = y0;
            a[base | out_off[t][1]] = y1;
        }
        if constexpr (kPrefetch) {
#pragma unroll
            for (int s = 0; s < S; ++s) bv[s] = bn[s];
        } else if (b + nwaves < nbatches) {
            load_b(b + nwaves, bv);
        }
    }
}

}  // namespace

template <typename R>
hipError_t launch_dense_mfma(void *state, int n, const GateDesc &g, const void *mat, hipStream_t s)
{
    const int k = (int)g.k;
    if (k < 3 || k > 5 || n < k + 4) return hipErrorInvalidValue;
    const uint64_t nbatches = 1ull << (n - k - 4);
    const uint64_t waves_per_block = kMfmaThreads / 64;
    uint64_t blocks = (nbatches + waves_per_block - 1) / waves_per_block;
    if (blocks > 8192) blocks = 8192;
    auto *a = (c2_t<R> *)state;
    auto *m = (const R *)mat;
    if (k == 3) k_dense_mfma<R, 3><<<(uint32_t)blocks, kMfmaThreads, 0, s>>>(a, m, nbatches, g);
    else if (k == 4) k_dense_mfma<R, 4><<<(uint32_t)blocks, kMfmaThreads, 0, s>>>(a, m, nbatches, g);
    else k_dense_mfma<R, 5><<<(uint32_t)blocks, kMfmaThreads, 0, s>>>(a, m, nbatches, g);
    return hipGetLastError();
}

template hipError_t launch_dense_mfma<float>(void *, int, const GateDesc &, const void *, hipStream_t);
template hipError_t launch_dense_mfma<double>(void *, int, const GateDesc &, const void *, hipStream_t);

}  // namespace qs
