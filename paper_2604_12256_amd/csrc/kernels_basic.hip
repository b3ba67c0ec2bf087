// Full-pass kernels: state initialisation, dense gate apply on the VALU,
// diagonal phase apply, tensor product, qubit permutation, reductions,
// amplitude gather, inner product and a plain copy (bandwidth reference).
//
// Every full pass streams the state once from HBM and once back; these
// kernels are bound by HBM bandwidth (8 TB/s on MI355X), so each thread
// touches whole 16-byte (complex128) or 8-byte (complex64) amplitudes with
// consecutive lanes on consecutive addresses wherever the gate allows.
#include "device.hpp"

namespace qs {

namespace {

constexpr int kBlock = 256;

// Grids hold at most 2^22 workgroups (2^30 work-items, inside the 32-bit
// dispatch size); kernels loop over the rest with a grid stride, so states
// of more than 2^32 amplitudes (33 and 34 qubits in complex128 fit in HBM)
// run with the same kernels.  Up to 30 qubits no grid reaches the cap.
constexpr uint64_t kMaxBlocks = 1ull << 22;

uint32_t blocks_for(uint64_t work, uint64_t per_block)
{
    uint64_t b = (work + per_block - 1) / per_block;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (uint32_t)(b ? b : 1);
}

// |0...0>: zero fill with amplitude 0 set to 1 (a kernel, not a memset, so
// that the op can be captured in a graph).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(c2_t<R> *__restrict__ a, uint64_t len)
{
    using V = c2_t<R>;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * 4;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock * 4 + threadIdx.x; i0 < len; i0 += stride) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kBlock;
            if (i < len) {
                V v;
                v.x = i == 0 ? R(1) : R(0);
                v.y = R(0);
                a[i] = v;
            }
        }
    }
}

// Dense k-qubit gate, one thread per group of 2^k amplitudes (Sec. 2.2: the
// 2^k amplitudes that differ only in the gate's qubits are multiplied by the
// gate matrix).  The matrix index is uniform across the wave.
template <typename R, int K>
__global__ __launch_bounds__(kBlock) void k_dense(c2_t<R> *__restrict__ a, const c2_t<R> *__restrict__ mg,
                                                  uint64_t ngroups, GateDesc g)
{
    using V = c2_t<R>;
    const QS_CONST R *m = as_const(reinterpret_cast<const R *>(mg));
    constexpr int D = 1 << K;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t grp = (uint64_t)blockIdx.x * kBlock + threadIdx.x; grp < ngroups; grp += stride) {
        const uint64_t base = insert_zeros<K>(grp, g.sorted);
        uint64_t off[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            uint64_t o = 0;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if ((r >> t) & 1) o |= 1ull << g.q[t];
            off[r] = base | o;
        }
        V v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = a[off[c]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc = cmul(ldc<R>(m, (uint64_t)(r * D)), v[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac(acc, ldc<R>(m, (uint64_t)(r * D + c)), v[c]);
            a[off[r]] = acc;
        }
    }
}

// Six-qubit dense gate: a block stages four groups of 64 amplitudes in LDS
// and every thread computes one output amplitude (one matrix row), so no
// thread holds a whole group in registers.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense6(c2_t<R> *__restrict__ a, const R *__restrict__ m, uint64_t ngroups,
                                                   GateDesc g)
{
    using V = c2_t<R>;
    __shared__ V tile[kBlock];
    const uint32_t r = threadIdx.x & 63;
    // the loop bound is uniform across the workgroup (barriers inside)
    for (uint64_t g0 = (uint64_t)blockIdx.x * (kBlock / 64); g0 < ngroups; g0 += (uint64_t)gridDim.x * (kBlock / 64)) {
        const uint64_t grp = g0 + threadIdx.x / 64;
        const bool valid = grp < ngroups;
        uint64_t mine = 0;
        if (valid) {
            mine = insert_zeros<6>(grp, g.sorted);
#pragma unroll
            for (int t = 0; t < 6; ++t)
                if ((r >> t) & 1) mine |= 1ull << g.q[t];
            tile[threadIdx.x] = a[mine];
        }
        __syncthreads();
        if (valid) {
            const V *in = tile + (threadIdx.x & ~63u);
            V acc = cmul(ldc<R>(m, (uint64_t)r * 64), in[0]);
            for (int c = 1; c < 64; ++c) cmac(acc, ldc<R>(m, (uint64_t)r * 64 + c), in[c]);
            a[mine] = acc;
        }
        __syncthreads();  // the tile is reused by the next groups
    }
}

// Diagonal of 2^k entries over the qubits q[0..k): a[x] *= T[y], y collects
// bit q[t] of x into bit t (Sec. 4.5: one complex multiply per amplitude).
struct DiagArgs {
    int32_t k;
    int32_t q[24];
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag(c2_t<R> *__restrict__ a, const c2_t<R> *__restrict__ T,
                                                 uint64_t len, DiagArgs d)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * 2;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * 2; i0 < len; i0 += stride) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint64_t x = i0 + u;
            if (x >= len) return;
            uint32_t y = 0;
            for (int t = 0; t < d.k; ++t) y |= (uint32_t)((x >> d.q[t]) & 1) << t;
            a[x] = cmul(a[x], T[y]);
        }
    }
}

// Tensor product (Alg. 5 tensorProduct): dst[(i_hi << nlo) | i_lo] = lo[i_lo] hi[i_hi].
template <typename R>
__global__ __launch_bounds__(kBlock) void k_kron(c2_t<R> *__restrict__ dst, const c2_t<R> *__restrict__ lo,
                                                 const c2_t<R> *__restrict__ hi, int nlo, uint64_t len)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * 4;
    for (uint64_t x0 = (uint64_t)blockIdx.x * kBlock * 4 + threadIdx.x; x0 < len; x0 += stride) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t x = x0 + (uint64_t)u * kBlock;
            if (x < len) dst[x] = cmul(lo[x & ((1ull << nlo) - 1)], hi[x >> nlo]);
        }
    }
}

// Qubit permutation (Sec. 2.3): dst[pi(x)] = src[x], pi moves source bit p to
// destination bit perm[p].  Out of place.
struct PermArgs {
    int32_t n;
    int32_t perm[40];
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_perm(c2_t<R> *__restrict__ dst, const c2_t<R> *__restrict__ src,
                                                 uint64_t len, PermArgs p)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < len; x += stride) {
        uint64_t y = 0;
        for (int b = 0; b < p.n; ++b) y |= ((x >> b) & 1ull) << p.perm[b];
        dst[y] = src[x];
    }
}

// Qubit reordering in place (Sec. 2.3, Eq. of the swap gate): exchanges
// physical bits lo[k] <-> hi[k] for every pair, i.e. a[sigma(x)] = a[x].  A
// tile holds every combination of the low bits and the high bits of the
// pairs (<= 12 bits), so the tile maps onto itself: it is read into LDS with
// the low bits contiguous and written back permuted, also with the low bits
// contiguous -- both sides coalesced, no second state buffer.
struct SwapArgs {
    int32_t npairs, tbits;
    int32_t lo[6], hi[6];
    uint64_t tilemask, outmask;
    uint64_t ntiles;
};

__device__ __forceinline__ uint32_t extract_bits(uint64_t x, uint64_t mask)
{
    uint32_t r = 0;
    int k = 0;
    while (mask) {
        const int p = __builtin_ctzll(mask);
        r |= (uint32_t)((x >> p) & 1ull) << k++;
        mask &= mask - 1;
    }
    return r;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_swap_bits(c2_t<R> *__restrict__ a, SwapArgs S)
{
    using V = c2_t<R>;
    extern __shared__ char smem_raw[];
    V *lds = reinterpret_cast<V *>(smem_raw);
    const uint32_t ntile = 1u << S.tbits;
    for (uint64_t t = blockIdx.x; t < S.ntiles; t += gridDim.x) {  // uniform across the workgroup
        const uint64_t base = deposit(t, S.outmask);
        for (uint32_t i = threadIdx.x; i < ntile; i += kBlock) lds[i] = a[base | deposit(i, S.tilemask)];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < ntile; i += kBlock) {
            const uint64_t y = base | deposit(i, S.tilemask);
            uint64_t x = y;
            for (int k = 0; k < S.npairs; ++k)
                if (((y >> S.lo[k]) ^ (y >> S.hi[k])) & 1ull) x ^= (1ull << S.lo[k]) | (1ull << S.hi[k]);
            a[y] = lds[extract_bits(x, S.tilemask)];
        }
        __syncthreads();  // the LDS tile is reused by the next tile
    }
}

// <a|b> with b stored under another qubit layout: element i of a pairs with
// element pi(i) of b (bit p of i -> bit map[p]).
template <typename RA, typename RB>
__global__ __launch_bounds__(kBlock) void k_inner_perm_partial(const c2_t<RA> *__restrict__ a,
                                                               const c2_t<RB> *__restrict__ b, uint64_t len,
                                                               PermArgs P, double2 *__restrict__ part)
{
    __shared__ double sre[kBlock], sim[kBlock];
    double re = 0.0, im = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < len; x += stride) {
        uint64_t y = 0;
        for (int p = 0; p < P.n; ++p) y |= ((x >> p) & 1ull) << P.perm[p];
        const double ar = (double)a[x].x, ai = (double)a[x].y;
        const double br = (double)b[y].x, bi = (double)b[y].y;
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sre[0], sim[0]);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_gather(const c2_t<R> *__restrict__ a, const uint64_t *__restrict__ idx,
                                                   uint64_t m, double2 *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const c2_t<R> v = a[idx[i]];
        out[i] = make_double2((double)v.x, (double)v.y);
    }
}

// Marginal probabilities, deterministic: one wave per (bin y, z segment) sums
// |a_x|^2 over x = deposit(y, S) | deposit(z, ~S) for z in the segment, each
// lane in increasing z, then a fixed butterfly over the lanes; a second
// kernel adds the segments in order.
struct MargArgs {
    uint64_t smask;
    int32_t nq, pad;
    int32_t sorted[24];     // marginal qubits, ascending
    uint64_t zseg;          // z values per segment
    uint32_t nseg;
    uint32_t contig;        // every selected qubit at or above log2(zseg), zseg a multiple of 256:
                            // a segment is one contiguous run of amplitudes
};

// deposit(z, ~S) for ascending S: insert a zero bit at every position of S.
__device__ __forceinline__ uint64_t spread_out(uint64_t z, const MargArgs &M)
{
    for (int t = 0; t < M.nq; ++t) {
        const uint64_t lo = z & ((1ull << M.sorted[t]) - 1);
        z = ((z >> M.sorted[t]) << (M.sorted[t] + 1)) | lo;
    }
    return z;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_marg_partial(const c2_t<R> *__restrict__ a, MargArgs M,
                                                         double *__restrict__ part)
{
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nbins = 1ull << M.nq;
    if (wave >= nbins * M.nseg) return;
    const uint64_t y = wave % nbins, seg = wave / nbins;
    const uint64_t xy = deposit(y, M.smask);
    double acc = 0.0;
    const uint64_t z0 = seg * M.zseg;
    if (M.contig) {
        // the segment is the run xy | spread_out(z0) + [0, zseg): each lane
        // takes two neighbouring amplitudes per step, two steps in flight
        const c2_t<R> *p = a + (xy | spread_out(z0, M));
        double acc1 = 0.0;
        for (uint64_t i = 2 * lane; i < M.zseg; i += 256) {
            const c2_t<R> u0 = p[i], u1 = p[i + 1], u2 = p[i + 128], u3 = p[i + 129];
            acc += (double)u0.x * (double)u0.x + (double)u0.y * (double)u0.y;
            acc += (double)u1.x * (double)u1.x + (double)u1.y * (double)u1.y;
            acc1 += (double)u2.x * (double)u2.x + (double)u2.y * (double)u2.y;
            acc1 += (double)u3.x * (double)u3.x + (double)u3.y * (double)u3.y;
        }
        acc += acc1;
    } else {
        for (uint64_t z = z0 + lane; z < z0 + M.zseg; z += 64) {
            const c2_t<R> v = a[xy | spread_out(z, M)];
            const double re = (double)v.x, im = (double)v.y;
            acc += re * re + im * im;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) part[seg * nbins + y] = acc;
}

// Marginal over a qubit set that includes some of the low six qubits: each
// wave reads contiguous runs of 64 amplitudes (lane = low six address bits),
// so every lane accumulates the bin its lane bits select.  Wave w takes one
// value yh of the selected high qubits and a segment of the unselected high
// bits; afterwards the lanes of a bin (differing only in unselected low bits)
// are combined by a fixed butterfly.  Bin bit order: ascending qubits (the
// selected low qubits first, then yh).
struct MargLaneArgs {
    uint32_t sl;            // selected low qubits (mask over bits 0..5)
    int32_t kl, kh;         // counts of selected low / high qubits
    int32_t shi[24];        // selected high qubits, ascending
    uint64_t zseg;          // unselected-high values per segment
    uint32_t nseg;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_marg_partial_lanes(const c2_t<R> *__restrict__ a, MargLaneArgs M,
                                                               double *__restrict__ part)
{
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nyh = 1ull << M.kh;
    if (wave >= nyh * M.nseg) return;  // whole waves (the wave index is uniform)
    const uint64_t yh = wave % nyh, seg = wave / nyh;
    uint64_t base = 0;
    for (int t = 0; t < M.kh; ++t) base |= ((yh >> t) & 1ull) << M.shi[t];
    double acc = 0.0;
    const uint64_t z0 = seg * M.zseg;
#pragma unroll 4
    for (uint64_t z = z0; z < z0 + M.zseg; ++z) {
        // z over the unselected high bits: zeros inserted at the selected
        // high qubits (wave-uniform)
        uint64_t hz = z;
        for (int t = 0; t < M.kh; ++t) {
            const int p = M.shi[t] - 6;
            hz = ((hz >> p) << (p + 1)) | (hz & ((1ull << p) - 1));
        }
        const c2_t<R> v = a[base | (hz << 6) | lane];
        const double re = (double)v.x, im = (double)v.y;
        acc += re * re + im * im;
    }
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (!((M.sl >> b) & 1u)) acc += __shfl_xor(acc, 1 << b, 64);
    if ((lane & ~M.sl & 63u) == 0) {
        uint32_t yl = 0;
        for (int b = 0, t = 0; b < 6; ++b)
            if ((M.sl >> b) & 1u) yl |= ((lane >> b) & 1u) << t++;
        const uint64_t bin = (uint64_t)yl | (yh << M.kl);
        part[seg * (1ull << (M.kl + M.kh)) + bin] = acc;
    }
}

// Few bins, many segments: one block per bin, fixed strided sums then a
// fixed tree.
__global__ __launch_bounds__(kBlock) void k_marg_final_block(const double *__restrict__ part, uint64_t nbins,
                                                             uint32_t nseg, double *__restrict__ out)
{
    __shared__ double sh[kBlock];
    const uint64_t y = blockIdx.x;
    double acc = 0.0;
    for (uint32_t g = threadIdx.x; g < nseg; g += kBlock) acc += part[(uint64_t)g * nbins + y];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[y] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_marg_final(const double *__restrict__ part, uint64_t nbins,
                                                       uint32_t nseg, double *__restrict__ out)
{
    const uint64_t y = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (y >= nbins) return;
    double s = 0.0;
    for (uint32_t g = 0; g < nseg; ++g) s += part[(uint64_t)g * nbins + y];
    out[y] = s;
}

// <a|b> in FP64: every block sums a fixed strided sequence per thread, then
// a fixed tree over the block; a second kernel adds the block results in a
// fixed tree.
constexpr uint32_t kInnerBlocks = 2048;

template <typename RA, typename RB>
__global__ __launch_bounds__(kBlock) void k_inner_partial(const c2_t<RA> *__restrict__ a,
                                                          const c2_t<RB> *__restrict__ b, uint64_t len,
                                                          double2 *__restrict__ part)
{
    __shared__ double sre[kBlock], sim[kBlock];
    double re = 0.0, im = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < len; x += stride) {
        const double ar = (double)a[x].x, ai = (double)a[x].y;
        const double br = (double)b[x].x, bi = (double)b[x].y;
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sre[0], sim[0]);
}

__global__ __launch_bounds__(kBlock) void k_inner_final(const double2 *__restrict__ part, uint32_t n,
                                                        double *__restrict__ out)
{
    __shared__ double sre[kBlock], sim[kBlock];
    double re = 0.0, im = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        re += part[i].x;
        im += part[i].y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sre[0];
        out[1] = sim[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * 4;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock * 4 + threadIdx.x; i < n16; i += stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * kBlock < n16) v[u] = src[i + u * kBlock];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * kBlock < n16) dst[i + u * kBlock] = v[u];
    }
}

}  // namespace

template <typename R>
hipError_t launch_init(void *state, int n, hipStream_t s)
{
    const uint64_t len = 1ull << n;
    k_init<R><<<blocks_for(len, kBlock * 4), kBlock, 0, s>>>((c2_t<R> *)state, len);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dense(void *state, int n, const GateDesc &g, const void *mat, hipStream_t s)
{
    const int k = (int)g.k;
    if (k < 1 || k > 6 || k > n) return hipErrorInvalidValue;
    const uint64_t ng = 1ull << (n - k);
    const uint32_t nb = blocks_for(ng, kBlock);
    auto *a = (c2_t<R> *)state;
    auto *m = (const c2_t<R> *)mat;
    switch (k) {
    case 1: k_dense<R, 1><<<nb, kBlock, 0, s>>>(a, m, ng, g); break;
    case 2: k_dense<R, 2><<<nb, kBlock, 0, s>>>(a, m, ng, g); break;
    case 3: k_dense<R, 3><<<nb, kBlock, 0, s>>>(a, m, ng, g); break;
    case 4: k_dense<R, 4><<<nb, kBlock, 0, s>>>(a, m, ng, g); break;
    case 5: k_dense<R, 5><<<nb, kBlock, 0, s>>>(a, m, ng, g); break;
    default:
        k_dense6<R><<<blocks_for(ng, kBlock / 64), kBlock, 0, s>>>(a, (const R *)mat, ng, g);
        break;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_diag_q(void *state, int n, int k, const int *q, const void *table, hipStream_t s)
{
    if (k < 1 || k > 24 || k > n) return hipErrorInvalidValue;
    DiagArgs d{};
    d.k = k;
    for (int t = 0; t < k; ++t) d.q[t] = q[t];
    const uint64_t len = 1ull << n;
    k_diag<R><<<blocks_for(len, kBlock * 2), kBlock, 0, s>>>((c2_t<R> *)state, (const c2_t<R> *)table, len, d);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_kron(void *dst, const void *lo, int nlo, const void *hi, int nhi, hipStream_t s)
{
    const uint64_t len = 1ull << (nlo + nhi);
    k_kron<R><<<blocks_for(len, kBlock * 4), kBlock, 0, s>>>((c2_t<R> *)dst, (const c2_t<R> *)lo,
                                                         (const c2_t<R> *)hi, nlo, len);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_perm(void *dst, const void *src, int n, const int *perm, hipStream_t s)
{
    if (n < 1 || n > 40) return hipErrorInvalidValue;
    PermArgs p{};
    p.n = n;
    for (int b = 0; b < n; ++b) p.perm[b] = perm[b];
    const uint64_t len = 1ull << n;
    k_perm<R><<<blocks_for(len, kBlock), kBlock, 0, s>>>((c2_t<R> *)dst, (const c2_t<R> *)src, len, p);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gather(const void *state, const uint64_t *idx, uint64_t m, double *out, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    k_gather<R><<<blocks_for(m, kBlock), kBlock, 0, s>>>((const c2_t<R> *)state, idx, m, (double2 *)out);
    return hipGetLastError();
}

namespace {
void marg_shape(int n, int nq, uint64_t *zseg, uint32_t *nseg)
{
    const uint64_t nz = 1ull << (n - nq);
    // aim for >= 2^16 waves in flight when the bins alone give fewer
    uint64_t seg = 1;
    const uint64_t nbins = 1ull << nq;
    while (nbins * seg < (1ull << 16) && nz / (seg * 2) >= 256) seg *= 2;
    *nseg = (uint32_t)seg;
    *zseg = nz / seg;
}
}  // namespace

// Segments of the lane-contiguous marginal: enough waves to fill the chip
// (2^15), each sweeping at least 64 runs.
void marg_lane_shape(int n, int kh, uint64_t *zseg, uint32_t *nseg)
{
    const uint64_t nz = 1ull << (n - 6 - kh);
    uint64_t seg = 1;
    while ((seg << kh) < (1ull << 15) && nz / (seg * 2) >= 64) seg *= 2;
    *nseg = (uint32_t)seg;
    *zseg = nz / seg;
}

bool marg_by_lanes(int n, const int *q, int nq)
{
    return n >= 8 && nq > 0 && q[0] < 6 && (n - 6) > 0;
}

size_t marginal_scratch_bytes(int n, const int *q, int nq)
{
    uint64_t zseg;
    uint32_t nseg;
    if (marg_by_lanes(n, q, nq)) {
        int kh = 0;
        for (int t = 0; t < nq; ++t) kh += q[t] >= 6;
        marg_lane_shape(n, kh, &zseg, &nseg);
    } else {
        marg_shape(n, nq, &zseg, &nseg);
    }
    return (size_t)nseg * (1ull << nq) * sizeof(double);
}

template <typename R>
hipError_t launch_marginal(const void *state, int n, const int *q, int nq, double *out, double *scratch,
                           hipStream_t s)
{
    if (nq < 0 || nq > n || nq > 20) return hipErrorInvalidValue;
    MargArgs M{};
    for (int t = 0; t < nq; ++t) {
        M.smask |= 1ull << q[t];
        M.sorted[t] = q[t];
        if (t && q[t] <= q[t - 1]) return hipErrorInvalidValue;  // callers pass ascending qubits
    }
    M.nq = nq;
    // y bit t <-> qubit q[t]: deposit() fills ascending positions, so the
    // bins come out in ascending-qubit order; the executor passes q sorted and
    // reorders on the host.
    const uint64_t nbins = 1ull << nq;
    uint32_t nseg;
    if (marg_by_lanes(n, q, nq)) {  // low qubits selected: lane-contiguous reads
        MargLaneArgs L{};
        for (int t = 0; t < nq; ++t) {
            if (q[t] < 6) {
                L.sl |= 1u << q[t];
                ++L.kl;
            } else {
                L.shi[L.kh++] = q[t];
            }
        }
        marg_lane_shape(n, L.kh, &L.zseg, &L.nseg);
        nseg = L.nseg;
        const uint64_t waves = (1ull << L.kh) * L.nseg;
        if (waves * 64 > kMaxBlocks * kBlock) return hipErrorInvalidValue;  // one wave per unit, no grid stride
        k_marg_partial_lanes<R><<<blocks_for(waves * 64, kBlock), kBlock, 0, s>>>((const c2_t<R> *)state, L, scratch);
    } else {
        marg_shape(n, nq, &M.zseg, &M.nseg);
        M.contig = (nq == 0 || (1ull << q[0]) >= M.zseg) && M.zseg % 256 == 0 ? 1u : 0u;
        nseg = M.nseg;
        const uint64_t waves = nbins * M.nseg;
        if (waves * 64 > kMaxBlocks * kBlock) return hipErrorInvalidValue;  // one wave per unit, no grid stride
        k_marg_partial<R><<<blocks_for(waves * 64, kBlock), kBlock, 0, s>>>((const c2_t<R> *)state, M, scratch);
    }
    if (nseg >= 64)
        k_marg_final_block<<<(uint32_t)nbins, kBlock, 0, s>>>(scratch, nbins, nseg, out);
    else
        k_marg_final<<<blocks_for(nbins, kBlock), kBlock, 0, s>>>(scratch, nbins, nseg, out);
    return hipGetLastError();
}

// Host-memory offload: copies window v of the state between the host (mapped
// pinned memory, read or written by the GPU over the host link) and a device
// window.  In 16-byte units: the window is rows of 2^r units; window unit
// i = (row << r) | off is state unit ((row << S | v) << r) | off.
__global__ __launch_bounds__(kBlock) void k_window_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                        uint64_t units, uint32_t r, uint32_t S, uint64_t v,
                                                        uint32_t to_host)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t omask = (1ull << r) - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < units; i += stride) {
        const uint64_t h = ((((i >> r) << S) | v) << r) | (i & omask);
        if (to_host) dst[h] = src[i];
        else dst[i] = src[h];
    }
}

hipError_t launch_window_copy(void *dst, const void *src, uint64_t window_bytes, uint64_t row_bytes, int S,
                              uint64_t v, bool to_host, hipStream_t s)
{
    if (row_bytes < 16 || (row_bytes & (row_bytes - 1)) || window_bytes % row_bytes || S < 0 || S > 40)
        return hipErrorInvalidValue;
    const uint64_t units = window_bytes / 16;
    const uint32_t r = (uint32_t)__builtin_ctzll(row_bytes / 16);
    k_window_copy<<<blocks_for(units, kBlock * 8), kBlock, 0, s>>>((uint4 *)dst, (const uint4 *)src, units, r,
                                                                  (uint32_t)S, v, to_host ? 1u : 0u);
    return hipGetLastError();
}

// out[y] = in[b(y)] with bit t of y moved to bit where[t] of b: marginal bins
// from ascending physical order into the caller's qubit order.
struct BinPerm {
    int32_t where[24];
    int32_t nq, pad;
};

__global__ __launch_bounds__(kBlock) void k_permute_bins(const double *__restrict__ in, double *__restrict__ out,
                                                         BinPerm P)
{
    const uint64_t y = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (y >= (1ull << P.nq)) return;
    uint64_t b = 0;
    for (int t = 0; t < P.nq; ++t) b |= ((y >> t) & 1ull) << P.where[t];
    out[y] = in[b];
}

hipError_t launch_permute_bins(const double *in, double *out, int nq, const int *where, hipStream_t s)
{
    if (nq < 0 || nq > 24) return hipErrorInvalidValue;
    BinPerm P{};
    P.nq = nq;
    for (int t = 0; t < nq; ++t) {
        if (where[t] < 0 || where[t] >= nq) return hipErrorInvalidValue;
        P.where[t] = where[t];
    }
    k_permute_bins<<<blocks_for(1ull << nq, kBlock), kBlock, 0, s>>>(in, out, P);
    return hipGetLastError();
}

size_t inner_scratch_bytes(int n)
{
    (void)n;
    return kInnerBlocks * sizeof(double2);
}

template <typename RA, typename RB>
hipError_t launch_inner(const void *a, const void *b, int n, double *out, double *scratch, hipStream_t s)
{
    const uint64_t len = 1ull << n;
    uint32_t nb = blocks_for(len, kBlock * 8);
    if (nb > kInnerBlocks) nb = kInnerBlocks;
    k_inner_partial<RA, RB><<<nb, kBlock, 0, s>>>((const c2_t<RA> *)a, (const c2_t<RB> *)b, len,
                                                  (double2 *)scratch);
    k_inner_final<<<1, kBlock, 0, s>>>((const double2 *)scratch, nb, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_swap_bits(void *state, int n, const int *lo, const int *hi, int npairs, hipStream_t s)
{
    if (npairs < 0 || npairs > 6 || n < 1 || n > 40) return hipErrorInvalidValue;
    if (npairs == 0) return hipSuccess;
    const int low = n < 6 ? n : 6;
    SwapArgs S{};
    S.npairs = npairs;
    uint64_t tm = (1ull << low) - 1;
    for (int k = 0; k < npairs; ++k) {
        if (lo[k] < 0 || lo[k] >= low || hi[k] < low || hi[k] >= n) return hipErrorInvalidValue;
        S.lo[k] = lo[k];
        S.hi[k] = hi[k];
        tm |= 1ull << hi[k];
    }
    S.tilemask = tm;
    S.tbits = __builtin_popcountll(tm);
    S.outmask = ((n >= 64) ? ~0ull : ((1ull << n) - 1)) & ~tm;
    S.ntiles = 1ull << (n - S.tbits);
    const size_t lds = sizeof(c2_t<R>) << S.tbits;
    k_swap_bits<R><<<blocks_for(S.ntiles, 1), kBlock, lds, s>>>((c2_t<R> *)state, S);
    return hipGetLastError();
}

template <typename RA, typename RB>
hipError_t launch_inner_perm(const void *a, const void *b, int n, const int *map, double *out, double *scratch,
                             hipStream_t s)
{
    const uint64_t len = 1ull << n;
    PermArgs P{};
    P.n = n;
    for (int p = 0; p < n; ++p) P.perm[p] = map[p];
    uint32_t nb = blocks_for(len, kBlock * 8);
    if (nb > kInnerBlocks) nb = kInnerBlocks;
    k_inner_perm_partial<RA, RB><<<nb, kBlock, 0, s>>>((const c2_t<RA> *)a, (const c2_t<RB> *)b, len, P,
                                                       (double2 *)scratch);
    k_inner_final<<<1, kBlock, 0, s>>>((const double2 *)scratch, nb, out);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s)
{
    // one workgroup per 16 KiB (no grid-stride loop below 64 GiB): the
    // fastest of the copy forms measured on MI355X (5.64 TB/s on 16 GiB,
    // against 5.14 TB/s with a 2^14-workgroup grid stride)
    const uint64_t n16 = bytes / 16;
    const uint32_t nb = blocks_for(n16, kBlock * 4);
    k_copy<<<nb, kBlock, 0, s>>>((uint4 *)dst, (const uint4 *)src, n16);
    return hipGetLastError();
}

#define QS_INST(R)                                                                                       \
    template hipError_t launch_init<R>(void *, int, hipStream_t);                                       \
    template hipError_t launch_dense<R>(void *, int, const GateDesc &, const void *, hipStream_t);      \
    template hipError_t launch_diag_q<R>(void *, int, int, const int *, const void *, hipStream_t);     \
    template hipError_t launch_kron<R>(void *, const void *, int, const void *, int, hipStream_t);      \
    template hipError_t launch_perm<R>(void *, const void *, int, const int *, hipStream_t);            \
    template hipError_t launch_gather<R>(const void *, const uint64_t *, uint64_t, double *, hipStream_t); \
    template hipError_t launch_marginal<R>(const void *, int, const int *, int, double *, double *, hipStream_t); \
    template hipError_t launch_swap_bits<R>(void *, int, const int *, const int *, int, hipStream_t);
QS_INST(double)
QS_INST(float)
template hipError_t launch_inner<double, double>(const void *, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_inner<double, float>(const void *, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_inner<float, double>(const void *, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_inner<float, float>(const void *, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_inner_perm<double, double>(const void *, const void *, int, const int *, double *, double *,
                                                      hipStream_t);
template hipError_t launch_inner_perm<double, float>(const void *, const void *, int, const int *, double *, double *,
                                                     hipStream_t);
template hipError_t launch_inner_perm<float, double>(const void *, const void *, int, const int *, double *, double *,
                                                     hipStream_t);
template hipError_t launch_inner_perm<float, float>(const void *, const void *, int, const int *, double *, double *,
                                                    hipStream_t);

}  // namespace qs
