// Device-side helpers and the launch interface between the executor and the
// kernels.  gfx950 (CDNA4) only: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace qs {

// Read-only data every lane of a wave reads at the same address (gate
// matrices, stage programs) is addressed through the constant address space,
// so the compiler issues scalar loads for it.
#define QS_CONST __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ const QS_CONST T *as_const(const T *p)
{
    return (const QS_CONST T *)(p);
}

// Complex entry i of an interleaved (re, im) real array, in any address space.
template <typename R, typename P>
__device__ __forceinline__ auto ldc(P m, uint64_t i)
{
    using V = typename std::conditional<sizeof(R) == 8, double2, float2>::type;
    V v;
    v.x = m[2 * i];
    v.y = m[2 * i + 1];
    return v;
}

// Interleaved complex amplitude: double2 (complex128) or float2 (complex64).
template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };
template <typename R> using c2_t = typename C2<R>::T;

template <typename V>
__device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += m * a
template <typename V>
__device__ __forceinline__ void cmac(V &acc, V m, V a)
{
    acc.x = fma(m.x, a.x, acc.x);
    acc.x = fma(-m.y, a.y, acc.x);
    acc.y = fma(m.x, a.y, acc.y);
    acc.y = fma(m.y, a.x, acc.y);
}

// A 64-bit value every lane of the wave holds, moved to scalar registers.
// The builtin returns a signed 32-bit int: each half is taken back as
// unsigned before widening, so that a low half with bit 31 set (indices of
// 2^31 and above) does not sign-extend into the high half.
__device__ __forceinline__ uint64_t wave_uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// Scatter the low bits of x to the set bit positions of mask (bit-deposit).
__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t mask)
{
    uint64_t r = 0;
    while (mask) {
        const uint64_t low = mask & (~mask + 1);
        if (x & 1) r |= low;
        x >>= 1;
        mask &= mask - 1;
    }
    return r;
}

// Insert a zero bit at each of the ascending positions pos[0..k-1].
template <int K>
__device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const int *pos)
{
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const uint64_t lo = g & ((1ull << pos[t]) - 1);
        g = ((g >> pos[t]) << (pos[t] + 1)) | lo;
    }
    return g;
}

struct GateDesc {            // one gate of a small-state program / full-pass op
    uint32_t diag;           // 1: table is a 2^k diagonal (k <= 24); else a dense 2^k x 2^k matrix (k <= 6)
    uint32_t k;
    int32_t q[24];           // matrix bit t <-> qubit q[t]
    int32_t sorted[6];       // dense: q ascending
    uint64_t table;          // offset (complex entries) in the table arena
};

struct SmallItem {           // one circuit of a batched small-state launch
    void *state;             // buffer holding 2^n amplitudes
    const GateDesc *gates;   // device program
    const void *tables;      // device table arena (same dtype as the state)
    uint32_t n, ngates, init;
    uint32_t pad;
};

constexpr int kSmallBatchMax = 128;
struct SmallPtrs {           // kernel-argument list of items for one batched launch
    const SmallItem *item[kSmallBatchMax];
};

// ---- launchers (return hipError_t of the launch) ---------------------------
template <typename R> hipError_t launch_init(void *state, int n, hipStream_t s);
template <typename R> hipError_t launch_dense(void *state, int n, const GateDesc &g, const void *mat, hipStream_t s);
template <typename R> hipError_t launch_dense_mfma(void *state, int n, const GateDesc &g, const void *mat, hipStream_t s);
template <typename R> hipError_t launch_diag_q(void *state, int n, int k, const int *q, const void *table, hipStream_t s);
template <typename R> hipError_t launch_kron(void *dst, const void *lo, int nlo, const void *hi, int nhi, hipStream_t s);
template <typename R> hipError_t launch_perm(void *dst, const void *src, int n, const int *perm, hipStream_t s);
// in-place exchange of physical bits lo[k] <-> hi[k] (lo < 6 <= hi)
template <typename R> hipError_t launch_swap_bits(void *state, int n, const int *lo, const int *hi, int npairs,
                                                  hipStream_t s);
template <typename RA, typename RB> hipError_t launch_inner_perm(const void *a, const void *b, int n, const int *map,
                                                                 double *out, double *scratch, hipStream_t s);
template <typename R> hipError_t launch_gather(const void *state, const uint64_t *idx, uint64_t m, double *out, hipStream_t s);
// marginal over the physical qubits q[0..nq): out[2^nq] doubles (device), scratch as sized by marginal_scratch_bytes
template <typename R> hipError_t launch_marginal(const void *state, int n, const int *q, int nq, double *out,
                                                 double *scratch, hipStream_t s);
size_t marginal_scratch_bytes(int n, const int *q, int nq);  // q ascending, as passed to launch_marginal
// out[y] = in[b(y)], bit t of y at bit where[t] of b (device arrays of 2^nq doubles)
hipError_t launch_permute_bins(const double *in, double *out, int nq, const int *where, hipStream_t s);
template <typename RA, typename RB> hipError_t launch_inner(const void *a, const void *b, int n, double *out,
                                                            double *scratch, hipStream_t s);
size_t inner_scratch_bytes(int n);
template <typename R> hipError_t launch_small_batch(const SmallItem *items_dev, uint32_t count, uint32_t max_n,
                                                    hipStream_t s);
template <typename R> hipError_t launch_small_ptrs(const SmallPtrs &P, uint32_t count, uint32_t max_n,
                                                   hipStream_t s);
int small_max_qubits(bool c128);

// Stage kernel: program built by the executor (see kernel_stage.hip).
// LDS slot swizzle of the stage kernel's transpose buffer (linear over XOR):
// 16-byte slots (complex128) fold local-index bits 4..15 into bits 0..3,
// 8-byte slots (complex64) fold bits 5..14 into bits 0..4, so that local bit
// l lands on slot bit l mod 4 (resp. l mod 5).  The host writes the
// swizzled byte offsets of each register set into the stage program.
__host__ __device__ inline uint32_t stage_swizzle(uint32_t i, bool c64)
{
    return c64 ? i ^ (((i >> 5) ^ (i >> 10)) & 31u) : i ^ (((i >> 4) ^ (i >> 8) ^ (i >> 12)) & 15u);
}
constexpr int kStageHeaderWords = 160;   // program header incl. neutral offsets at [128, 128 + 2^RB)
constexpr int kStagePhaseWords = 16;     // phase header before its register offsets

struct StageLaunch {
    void *state;
    const uint32_t *prog;    // device program words
    const void *tables;      // device table arena
    int n, C, nphases;
    uint64_t nchunks;
    uint64_t xbits = 0;      // bits OR-ed into the wave-uniform base for selectors only (the
                             // outer qubits of a host-memory offload window, at bits >= n)
    // tensor product formed on load: when kron_lo is set, the chunk is read as
    // kron_lo[x mod 2^kron_nlo] * kron_hi[x >> kron_nlo] instead of state[x]
    const void *kron_lo = nullptr, *kron_hi = nullptr;
    int kron_nlo = 0;
    // the program holds quadratic-phase operators: launched on the kernel
    // variant that has them (the others keep the register allocation of the
    // kernel without)
    bool quad = false;
};
template <typename R> hipError_t launch_stage(const StageLaunch &L, hipStream_t s);

// One stage of each of several independent states in one launch (kernel
// argument, so no device allocation): job j owns workgroups
// first_block[j] .. first_block[j + 1] - 1, one chunk each.  Every job's
// program uses the launch's chunk size C and has nchunks = its block count.
constexpr uint32_t kStageJobsMax = 64;
struct StageJob {
    void *state;
    const uint32_t *prog;
    const void *tables;
    const void *kron_lo, *kron_hi;  // as in StageLaunch (kron_lo NULL: read the state)
    int32_t kron_nlo, pad;
};
struct StageJobs {
    uint32_t n;
    uint32_t first_block[kStageJobsMax + 1];
    StageJob job[kStageJobsMax];
};
template <typename R> hipError_t launch_stage_multi(const StageJobs &J, int C, bool quad, hipStream_t s);

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s);
// host-memory offload: window v (outer qubits fixed) between the mapped host
// state and a device window; rows of row_bytes, 2^S windows interleaved
hipError_t launch_window_copy(void *dst, const void *src, uint64_t window_bytes, uint64_t row_bytes, int S,
                              uint64_t v, bool to_host, hipStream_t s);

// ---- measurement (kernels_measure.hip) ----
// Inverse-CDF sampling inside blocks of 2^nlow consecutive logical indices:
// nthr threads each own 2^seg_log2 of them (nthr << seg_log2 == 2^nlow).
// The physical address of within-block offset w is
// base | tabs[w & 511] | tabs[512 + (w >> 9)] (nlow <= 18).
struct SampleArgs {
    int32_t nlow, seg_log2, nthr, pad;
};
constexpr int kZMasksPerLaunch = 16;
struct ZArgs {
    uint64_t m[kZMasksPerLaunch];   // physical qubit masks of the Z strings
    int32_t nm, pad;
};
template <typename R> hipError_t launch_collapse(void *state, int n, int phys_qubit, int outcome, double scale,
                                                 hipStream_t s);
template <typename R> hipError_t launch_sample(const void *state, const SampleArgs &S, uint32_t nblocks,
                                               const uint64_t *tabs, const uint64_t *bases, const uint64_t *ids,
                                               const uint32_t *start, const double *resid, uint64_t *out,
                                               hipStream_t s);
size_t expect_z_scratch_bytes();
template <typename R> hipError_t launch_expect_z(const void *state, int n, const ZArgs &Z, double *out,
                                                 double *scratch, hipStream_t s);

}  // namespace qs
