// Cache-blocked stage kernel (block-by-block scheme, Alg. 2; the "all-in-one"
// branch of the adaptive simulator, Alg. 5).
//
// One workgroup owns one chunk of 2^C amplitudes at a time: the amplitudes
// whose local qubits (C physical bit positions, always including bits 0..5
// so that every wave reads 1 KiB / 512 B contiguous runs) vary and whose
// global qubits are fixed by the chunk id.  The chunk is read from HBM once,
// every gate of the stage is applied on chip, and it is written back once.
//
// On chip the chunk lives in VGPRs: each thread holds 2^RB amplitudes (RB = 4
// for complex128, 5 for complex64), indexed by RB "register" local bits; the
// other local bits give the thread id.  The stage is cut into register
// phases; a phase applies fused dense operators on register bits and
// diagonal operators on any bits (non-register bits are constants per
// thread).  Between phases whose register sets differ, the chunk goes through
// LDS once (write in the old mapping, read in the new one).
//
// Program words (built on the host; read with wave-uniform loads):
//   header  [0] C  [1] n  [2] nphases  [3] RB  [4,5] local mask  [6,7] global mask
//           [8 + i] physical bit of local bit i (i < C)   [32 + p] word offset of phase p
//           [128 + j] LDS byte offset of register j in the load/store mapping
//   phase   [0] nops  [1] non-register local mask  [2] register local mask
//           [3] number of wave bits of the thread id (thread-id bits 6, 7, ...)
//           [4..7] local bit of thread-id bit i (bytes; bits 0..5 are the lane bits)
//           [8, 9] physical bit of wave bit i (bytes)
//           [16 + j] LDS byte offset of register j (swizzled; j < 2^RB)
//           [16 + 2^RB + 16 o ...] op o (a 64-byte record)
//   op      [0] type (bits 0-7: 1 dense, 2 diagonal, 3 quadratic phase) | register mask (bits of the
//           register tile the operator acts on) << 8 | selector count << 16 (5 bits) |
//           bit fields F << 21 (3 bits) | selectors wave-uniform << 24 |
//           log2 of the table bytes per selector value << 25
//           [1,2] table byte offset
//           F = 0: [3..9] selector sources (bytes): 0x80 | b is lane bit b of the
//           thread id, any other value the physical position of a chunk or wave bit
//           F > 0 (wave-uniform selectors on runs of consecutive positions):
//           [3 + f] field f: first physical position | width << 16, the fields
//           filling the selector from bit 0 up
//   A dense op's table holds 2^nsel matrices of (2^k)^2 entries, a diagonal
//   op's 2^nsel blocks of 2^k factors (k = popcount of the register mask).
//   A quadratic-phase op: [3] word offset (from the program start) of its
//   block of complex FP64 factors, [4], [6], [7] entry offsets in the block of
//   its low chunk rows, high chunk rows and register-pair factors, [5]
//   h | nhi << 8 (the chunk-index bits of the low and the high rows); see
//   quad_op.  Only the kernel variant with quadratic-phase operators runs them.
#include "device.hpp"

namespace qs {

namespace {

constexpr int kStageMaxThreads = 512;
constexpr uint32_t kStageLdsBytes = 128u * 1024u;

template <typename R> __device__ __forceinline__ uint32_t swz(uint32_t i)
{
    return stage_swizzle(i, sizeof(R) == 4);
}

__device__ __forceinline__ uint32_t byte_at(const QS_CONST uint32_t *w, int i)
{
    return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu;
}

struct __attribute__((aligned(64))) OpRec {
    uint32_t w[16];
};

__device__ __forceinline__ OpRec load_rec(const QS_CONST uint32_t *p)
{
    OpRec r;
#pragma unroll
    for (int i = 0; i < 16; ++i) r.w[i] = p[i];
    return r;
}

// Selector value of an op record: bit u from selector source byte u (a lane
// bit of the thread id, or a bit of the wave-uniform base `ub`).  Up to
// twelve sources come from the record held in scalar registers; wider
// diagonals read theirs from memory.
template <bool LANE>
__device__ __forceinline__ uint32_t sel_bit(uint32_t b, uint64_t ub, uint32_t tid)
{
    if (LANE && (b & 0x80u)) return (tid >> (b & 63u)) & 1u;
    return (uint32_t)(ub >> (b & 63u)) & 1u;
}

template <bool LANE>
__device__ __forceinline__ uint32_t gather_sel(const OpRec &r, const QS_CONST uint32_t *rec, uint32_t nsel,
                                               uint64_t ub, uint32_t tid)
{
    if (nsel == 0) return 0;
    if (nsel <= 4) {
        uint32_t sel = sel_bit<LANE>(r.w[3] & 0xffu, ub, tid);
        if (nsel > 1) {
            sel |= sel_bit<LANE>((r.w[3] >> 8) & 0xffu, ub, tid) << 1;
            if (nsel > 2) {
                sel |= sel_bit<LANE>((r.w[3] >> 16) & 0xffu, ub, tid) << 2;
                if (nsel > 3) sel |= sel_bit<LANE>(r.w[3] >> 24, ub, tid) << 3;
            }
        }
        return sel;
    }
    uint32_t sel = 0;
    if (nsel <= 12) {  // sources in record words 3..5, loaded with the record
#pragma unroll
        for (uint32_t u = 0; u < 12; ++u)
            if (u < nsel) sel |= sel_bit<LANE>((r.w[3 + u / 4] >> (8 * (u % 4))) & 0xffu, ub, tid) << u;
        return sel;
    }
    for (uint32_t u = 0; u < nsel; ++u) sel |= sel_bit<LANE>(byte_at(rec + 3, (int)u), ub, tid) << u;
    return sel;
}

template <int RB>
__device__ __forceinline__ uint64_t reg_phys_offset(int j, const uint64_t *regphys)
{
    uint64_t o = 0;
#pragma unroll
    for (int b = 0; b < RB; ++b)
        if ((j >> b) & 1) o |= regphys[b];
    return o;
}

// Dense operator on the register bits of MASK; m holds (2^k)^2 entries,
// bit t of its index <-> t-th set bit of MASK.  One- and two-bit operators
// are applied in place with no register copies: every output first
// accumulates all its terms except the real part of its diagonal
// coefficient; then each output's last FMA reads its own input for the last
// time and may take over that input's registers.
template <typename R, int RB, int MASK, typename MP>
__device__ __forceinline__ void apply_dense(c2_t<R> *amp, MP m)
{
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;
    constexpr int NR = 1 << RB;
#pragma unroll
    for (int outer = 0; outer < NR; ++outer) {
        if (outer & MASK) continue;
        int idx[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            int x = outer, bit = 0;
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if ((MASK >> b) & 1) {
                    if ((c >> bit) & 1) x |= 1 << b;
                    ++bit;
                }
            idx[c] = x;
        }
        if constexpr (K > 2) {
            // whole-tile operator: copies are negligible beside its (2^k)^2
            // products, and fewer values stay live
            c2_t<R> v[D];
#pragma unroll
            for (int c = 0; c < D; ++c) v[c] = amp[idx[c]];
#pragma unroll
            for (int r = 0; r < D; ++r) {
                c2_t<R> acc = cmul(ldc<R>(m, (uint64_t)(r * D)), v[0]);
#pragma unroll
                for (int c = 1; c < D; ++c) cmac(acc, ldc<R>(m, (uint64_t)(r * D + c)), v[c]);
                amp[idx[r]] = acc;
            }
            continue;
        }
        R ar[D], ai[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            // diagonal coefficient's imaginary part first (starts the sums)
            const R dim = ldc<R>(m, (uint64_t)(r * D + r)).y;
            ar[r] = -dim * amp[idx[r]].y;
            ai[r] = dim * amp[idx[r]].x;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if (c == r) continue;
                const c2_t<R> w = ldc<R>(m, (uint64_t)(r * D + c));
                ar[r] = fma(w.x, amp[idx[c]].x, ar[r]);
                ar[r] = fma(-w.y, amp[idx[c]].y, ar[r]);
                ai[r] = fma(w.x, amp[idx[c]].y, ai[r]);
                ai[r] = fma(w.y, amp[idx[c]].x, ai[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const R dre = ldc<R>(m, (uint64_t)(r * D + r)).x;
            amp[idx[r]].x = fma(dre, amp[idx[r]].x, ar[r]);
            amp[idx[r]].y = fma(dre, amp[idx[r]].y, ai[r]);
        }
    }
}

// Diagonal operator on the register bits of MASK: register j is multiplied by
// t[bits of j under MASK] (in place: the two products that need the other
// part are formed first, each final FMA is its input's last use).
template <typename R, int RB, int MASK, typename MP>
__device__ __forceinline__ void apply_diag(c2_t<R> *amp, MP t)
{
    constexpr int NR = 1 << RB;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        int idx = 0, bit = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if ((MASK >> b) & 1) {
                if ((j >> b) & 1) idx |= 1 << bit;
                ++bit;
            }
        const c2_t<R> w = ldc<R>(t, (uint64_t)idx);
        const R pr = -w.y * amp[j].y, pi = w.y * amp[j].x;
        amp[j].x = fma(w.x, amp[j].x, pr);
        amp[j].y = fma(w.x, amp[j].y, pi);
    }
}

template <typename R, int RB, int M = 0, typename MP>
__device__ __forceinline__ void dispatch_diag(uint32_t mask, c2_t<R> *amp, MP t)
{
    if constexpr (M < (1 << RB)) {
        if (mask == (uint32_t)M) apply_diag<R, RB, M, MP>(amp, t);
        else dispatch_diag<R, RB, M + 1, MP>(mask, amp, t);
    } else {
        __builtin_unreachable();  // every mask below 2^RB is handled above
    }
}

template <typename R, int RB, typename MP>
__device__ __forceinline__ void dispatch_dense(uint32_t mask, c2_t<R> *amp, MP m)
{
    constexpr int FULL = (1 << RB) - 1;
    switch (mask) {
    case 1: apply_dense<R, RB, 1, MP>(amp, m); break;
    case 2: apply_dense<R, RB, 2, MP>(amp, m); break;
    case 4: apply_dense<R, RB, 4, MP>(amp, m); break;
    case 8: apply_dense<R, RB, 8, MP>(amp, m); break;
    case 3: apply_dense<R, RB, 3, MP>(amp, m); break;
    case 5: apply_dense<R, RB, 5, MP>(amp, m); break;
    case 6: apply_dense<R, RB, 6, MP>(amp, m); break;
    case 9: apply_dense<R, RB, 9, MP>(amp, m); break;
    case 10: apply_dense<R, RB, 10, MP>(amp, m); break;
    case 12: apply_dense<R, RB, 12, MP>(amp, m); break;
    case FULL: apply_dense<R, RB, FULL, MP>(amp, m); break;
    default:
        if constexpr (RB == 5) {
            switch (mask) {
            case 16: apply_dense<R, RB, 16, MP>(amp, m); break;
            case 17: apply_dense<R, RB, 17, MP>(amp, m); break;
            case 18: apply_dense<R, RB, 18, MP>(amp, m); break;
            case 20: apply_dense<R, RB, 20, MP>(amp, m); break;
            case 24: apply_dense<R, RB, 24, MP>(amp, m); break;
            default: __builtin_unreachable();
            }
        } else {
            // the host encodes only the masks above (stage_dense_mask_ok)
            __builtin_unreachable();
        }
        break;
    }
}

// Local index of thread-id bits under a phase's thread map (map bytes packed
// in t0..t2: byte i = local bit of thread-id bit i), branch-free.
__device__ __forceinline__ uint32_t thread_local_base(uint32_t tid, uint32_t t0, uint32_t t1, uint32_t t2,
                                                      int nbits)
{
    const uint32_t t[3] = {t0, t1, t2};
    uint32_t lb = 0;
#pragma unroll
    for (int i = 0; i < 12; ++i)
        if (i < nbits) lb |= ((tid >> i) & 1u) << ((t[i / 4] >> (8 * (i % 4))) & 0xffu);
    return lb;
}

// Moves the chunk between two register/thread mappings through LDS.  The
// thread and register parts of a local index have disjoint bits, so the
// swizzled slot is swz(lb) ^ swz(r): a per-thread term and a wave-uniform
// one, the latter read from the program (byte offsets of each register).
typedef __attribute__((address_space(3))) char lds_byte_t;

template <typename R, int RB>
__device__ __forceinline__ void transpose(c2_t<R> *amp, uint32_t lds_base, uint32_t old_lb,
                                          const QS_CONST uint32_t *old_off, uint32_t new_lb,
                                          const QS_CONST uint32_t *new_off)
{
    constexpr int NR = 1 << RB;
    using V = c2_t<R>;
    struct alignas(2 * sizeof(R)) pair_t {
        R x, y;
    };
    typedef __attribute__((address_space(3))) pair_t lds_v_t;
    __syncthreads();
    // LDS byte address = (base | per-thread term) ^ wave-uniform term; the
    // base of the dynamic LDS is 0 here (the kernel has no static LDS), so
    // OR and XOR do not carry into it.  (The empty asm keeps the per-thread
    // term opaque, so that the compiler does not expand the swizzle again
    // per element.)
    uint32_t wb = lds_base | (swz<R>(old_lb) * (uint32_t)sizeof(V));
    asm volatile("" : "+v"(wb));
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        lds_v_t *p = reinterpret_cast<lds_v_t *>((uintptr_t)(wb ^ old_off[j]));
        p->x = amp[j].x;
        p->y = amp[j].y;
    }
    __syncthreads();
    uint32_t rb = lds_base | (swz<R>(new_lb) * (uint32_t)sizeof(V));
    asm volatile("" : "+v"(rb));
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const lds_v_t *p = reinterpret_cast<const lds_v_t *>((uintptr_t)(rb ^ new_off[j]));
        amp[j].x = p->x;
        amp[j].y = p->y;
    }
}

// Quadratic-phase operator (op type 3): amplitude x is multiplied by
// e^{i phi(x)}, phi(x) = c + sum a_q x_q + sum b_qp x_q x_p over the buffer's
// qubits, formed in FP64 (also for complex64 states, whose amplitudes take
// one FP32 rounding per operator).  Its block of complex FP64
// unit factors (in the program words) holds, for the chunk's share, rows
// selected by the low and the high half of the chunk index: lane l < C forms
// B_l = e^{i beta_l} (the coefficient the chunk bits give local bit l) as the
// product of its two row entries, and a wave product over the other lanes
// forms the chunk bits' own factor E.  A thread starts from its table entry
// (constant and thread-bit terms) times E, takes in B of each set thread bit,
// and walks its 2^RB amplitudes in Gray-code order with a running product:
// flipping register bit b multiplies by G_b = e^{i(a_b + thread and chunk
// terms of b)} (or its conjugate) and by the pair factors with the register
// bits already set.
template <typename R, int RB>
__device__ __forceinline__ void quad_op(c2_t<R> *amp, const OpRec &rec, const uint32_t *Pg, uint64_t chunk,
                                        uint32_t tid, int C, uint32_t rmask, uint32_t t0, uint32_t t1, uint32_t t2)
{
    using V = c2_t<double>;
    constexpr int NR = 1 << RB;
    const int h = (int)(rec.w[5] & 0xffu), nhi = (int)((rec.w[5] >> 8) & 0xffu);
    const int ncl = C + nhi + 1, nch = C + 1;
    const int lane = (int)(tid & 63u);
    const uint64_t glo = chunk & ((1ull << h) - 1), ghi = chunk >> h;
    const V *blk = reinterpret_cast<const V *>(Pg + rec.w[3]);
    const V *tlo = blk + rec.w[4] + glo * (uint64_t)ncl;
    const V *thi = blk + rec.w[6] + ghi * (uint64_t)nch;
    const V one{1.0, 0.0};
    const V vlo = lane < ncl ? tlo[lane] : one;
    const V vhi = lane < nch ? thi[lane] : one;
    const V B = cmul(vlo, vhi);
    V p = one;
    if (lane >= C && lane < C + nhi && ((ghi >> (lane - C)) & 1ull)) p = vlo;
    if (lane == C + nhi) p = vlo;
    if (lane == C) p = cmul(p, vhi);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) p = cmul(p, V{__shfl_xor(p.x, off), __shfl_xor(p.y, off)});

    const int nt = C - RB;
    const V *row = blk + (size_t)tid * (1 + RB);
    const V *qm = blk + rec.w[7];
    V F = cmul(row[0], p);
    for (int i = 0; i < nt; ++i) {
        const uint32_t w = i < 4 ? t0 : i < 8 ? t1 : t2;
        const int j = (int)((w >> (8 * (i & 3))) & 0xffu);
        const V f2 = cmul(F, V{__shfl(B.x, j), __shfl(B.y, j)});
        if ((tid >> i) & 1u) F = f2;
    }
    V G[RB];
    uint32_t rm = rmask;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int j = __builtin_ctz(rm);
        rm &= rm - 1u;
        G[b] = cmul(row[1 + b], V{__shfl(B.x, j), __shfl(B.y, j)});
    }
    V Q = F;
    amp[0] = cmul(amp[0], c2_t<R>{(R)Q.x, (R)Q.y});
#pragma unroll
    for (int k = 1; k < NR; ++k) {
        const int g = k ^ (k >> 1), b = __builtin_ctz(k), prev = g ^ (1 << b);
        const bool set = (g >> b) & 1;
        V f = set ? G[b] : V{G[b].x, -G[b].y};
#pragma unroll
        for (int b2 = 0; b2 < RB; ++b2) {
            if (b2 == b || !((prev >> b2) & 1)) continue;
            const int lo = b < b2 ? b : b2, hi = b < b2 ? b2 : b;
            const V q = qm[lo * (2 * RB - lo - 1) / 2 + (hi - lo - 1)];
            f = cmul(f, set ? q : V{q.x, -q.y});
        }
        Q = cmul(Q, f);
        amp[g] = cmul(amp[g], c2_t<R>{(R)Q.x, (R)Q.y});
    }
}

// The chunks first, first + step, ... below nchunks of one stage program.
// With klo set, the chunk is the tensor product klo (x) khi formed on load
// (Alg. 7's merge of the booster's two halves, without writing and re-reading
// the product): amplitude x = klo[x mod 2^knlo] * khi[x >> knlo].
template <typename R, int RB, bool QD>
__device__ __forceinline__ void stage_chunks(c2_t<R> *__restrict__ state, const uint32_t *__restrict__ Pg,
                                             const c2_t<R> *__restrict__ tables, uint64_t first, uint64_t nchunks,
                                             uint64_t step, uint64_t xbits, const c2_t<R> *__restrict__ klo,
                                             const c2_t<R> *__restrict__ khi, int knlo)
{
    using V = c2_t<R>;
    const QS_CONST uint32_t *P = as_const(Pg);
    const QS_CONST char *ctables = reinterpret_cast<const QS_CONST char *>(as_const(reinterpret_cast<const R *>(tables)));
    const char *rtables = reinterpret_cast<const char *>(tables);
    constexpr int NR = 1 << RB;
    extern __shared__ char smem_raw[];
    const uint32_t lds = (uint32_t)(uintptr_t)(lds_byte_t *)smem_raw;  // LDS byte address of the buffer

    const int C = (int)P[0];
    const int nph = (int)P[2];
    const uint64_t Lmask = (uint64_t)P[4] | ((uint64_t)P[5] << 32);
    const uint64_t Gmask = (uint64_t)P[6] | ((uint64_t)P[7] << 32);
    const uint32_t tid = threadIdx.x;
    // wave index in a scalar register (the asm keeps the compiler from
    // turning the uniform bit tests below back into per-lane code)
    uint32_t wave;
    asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(wave) : "v"(tid));
    wave >>= 6;
    const uint32_t all_local = (1u << C) - 1;
    const uint32_t neutral_nonr = (1u << (C - RB)) - 1;
    const uint32_t neutral_r = all_local & ~neutral_nonr;
    const QS_CONST uint32_t *const neutral_off = P + 128;
    uint64_t regphys[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) regphys[b] = 1ull << P[8 + C - RB + b];
    const uint64_t tphys = deposit(tid, Lmask);
    // load/store mapping: thread-id bit i <-> local bit i (packed like a phase's map)
    uint32_t neutral_t[3] = {0, 0, 0};
    for (int i = 0; i < C - RB; ++i) neutral_t[i / 4] |= (uint32_t)i << (8 * (i % 4));

    V amp[NR];
    // chunk bits at their physical positions: deposited once, then advanced
    // by a masked add (the bits outside the mask are set, so that carries run
    // through them)
    const uint64_t cstep = deposit(step, Gmask);
    uint64_t cbase = deposit(first, Gmask);
    for (uint64_t chunk = first; chunk < nchunks; chunk += step, cbase = ((cbase | ~Gmask) + cstep) & Gmask) {
        // chunk bits, thread bits and register bits are disjoint: each
        // amplitude is a per-thread pointer plus a wave-uniform offset
        V *const pt = state + (cbase | tphys);
        if (klo) {
            const uint64_t lomask = (1ull << knlo) - 1;
            const uint64_t base = cbase | tphys;
            uint64_t rbits = 0;
#pragma unroll
            for (int b = 0; b < RB; ++b) rbits |= regphys[b];
            if (!(rbits & lomask)) {
                // register bits all in the high factor: one low factor per thread
                const V lo = klo[base & lomask];
#pragma unroll
                for (int j = 0; j < NR; ++j) amp[j] = cmul(lo, khi[(base | reg_phys_offset<RB>(j, regphys)) >> knlo]);
            } else if (!(rbits >> knlo)) {
                // register bits all in the low factor: one high factor per thread
                const V hi = khi[base >> knlo];
#pragma unroll
                for (int j = 0; j < NR; ++j) amp[j] = cmul(klo[(base | reg_phys_offset<RB>(j, regphys)) & lomask], hi);
            } else {
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const uint64_t x = base | reg_phys_offset<RB>(j, regphys);
                    amp[j] = cmul(klo[x & lomask], khi[x >> knlo]);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < NR; ++j) amp[j] = pt[reg_phys_offset<RB>(j, regphys)];
        }
        // current mapping: register mask and thread-map words (workgroup-uniform)
        uint32_t cur_lb = tid, cur_r = neutral_r;
        uint32_t cur_t0 = neutral_t[0], cur_t1 = neutral_t[1], cur_t2 = neutral_t[2];
        const QS_CONST uint32_t *cur_off = neutral_off;
        for (int p = 0; p < nph; ++p) {
            const QS_CONST uint32_t *ph = P + P[32 + p];
            const uint32_t nops = ph[0], rmask = ph[2];
            const uint32_t t0 = ph[4], t1 = ph[5], t2 = ph[6];
            if (rmask != cur_r || t0 != cur_t0 || t1 != cur_t1 || t2 != cur_t2) {
                const uint32_t lb = thread_local_base(tid, t0, t1, t2, C - RB);
                transpose<R, RB>(amp, lds, cur_lb, cur_off, lb, ph + 16);
                cur_lb = lb;
                cur_r = rmask;
                cur_t0 = t0;
                cur_t1 = t1;
                cur_t2 = t2;
                cur_off = ph + 16;
            }
            // wave-uniform base: chunk bits and the wave bits of the thread id
            // at their physical positions, and any bits beyond the buffer
            // (outer qubits of an offload window)
            uint64_t ub = cbase | xbits;
            const uint32_t nwave = ph[3];
            for (uint32_t i = 0; i < nwave; ++i)
                ub |= (uint64_t)((wave >> i) & 1u) << byte_at(ph + 8, (int)i);
            const QS_CONST uint32_t *recs = ph + 16 + NR;
            auto apply_op = [&](const OpRec &rec, uint32_t o) __attribute__((always_inline)) {
                const uint32_t head = rec.w[0];
                if constexpr (QD) {
                    if ((head & 0xffu) == 3u) {
                        quad_op<R, RB>(amp, rec, Pg, chunk, tid, C, rmask, t0, t1, t2);
                        return;
                    }
                }
                const uint32_t mask = (head >> 8) & 0xffu, nsel = (head >> 16) & 0x1fu, shift = head >> 25;
                const uint64_t toff = (uint64_t)rec.w[1] | ((uint64_t)rec.w[2] << 32);
                if ((head >> 24) & 1u) {
                    uint32_t sel;
                    const uint32_t nfield = (head >> 21) & 7u;
                    if (nfield) {
                        sel = 0;
                        uint32_t u = 0;
#pragma unroll
                        for (uint32_t f = 0; f < 6; ++f)
                            if (f < nfield) {
                                const uint32_t d = rec.w[3 + f], w = d >> 16;
                                sel |= ((uint32_t)(ub >> (d & 63u)) & ((1u << w) - 1u)) << u;
                                u += w;
                            }
                    } else {
                        sel = gather_sel<false>(rec, recs + 16 * o, nsel, ub, tid);
                    }
                    const QS_CONST R *m = reinterpret_cast<const QS_CONST R *>(ctables + toff + ((uint64_t)sel << shift));
                    if ((head & 0xffu) == 1u) dispatch_dense<R, RB>(mask, amp, m);
                    else dispatch_diag<R, RB>(mask, amp, m);
                } else {
                    const uint32_t sel = gather_sel<true>(rec, recs + 16 * o, nsel, ub, tid);
                    const R *m = reinterpret_cast<const R *>(rtables + toff + ((uint64_t)sel << shift));
                    if ((head & 0xffu) == 1u) dispatch_dense<R, RB>(mask, amp, m);
                    else dispatch_diag<R, RB>(mask, amp, m);
                }
            };
            OpRec cur = load_rec(recs);
            for (uint32_t o = 0; o < nops; o += 2) {
                OpRec second;
                if (o + 1 < nops) second = load_rec(recs + 16 * (o + 1));
                apply_op(cur, o);
                if (o + 2 < nops) cur = load_rec(recs + 16 * (o + 2));
                if (o + 1 < nops) apply_op(second, o + 1);
            }
        }
        if (cur_r != neutral_r || cur_t0 != neutral_t[0] || cur_t1 != neutral_t[1] || cur_t2 != neutral_t[2])
            transpose<R, RB>(amp, lds, cur_lb, cur_off, tid, neutral_off);
#pragma unroll
        for (int j = 0; j < NR; ++j) pt[reg_phys_offset<RB>(j, regphys)] = amp[j];
        __syncthreads();  // LDS reuse by the next chunk
    }
}

template <typename R, int RB, bool QD>
__global__ __launch_bounds__(kStageMaxThreads) void k_stage(c2_t<R> *__restrict__ state,
                                                            const uint32_t *__restrict__ Pg,
                                                            const c2_t<R> *__restrict__ tables,
                                                            uint64_t nchunks, uint64_t xbits,
                                                            const c2_t<R> *__restrict__ klo,
                                                            const c2_t<R> *__restrict__ khi, int knlo)
{
    stage_chunks<R, RB, QD>(state, Pg, tables, blockIdx.x, nchunks, gridDim.x, xbits, klo, khi, knlo);
}

// Stages of several independent states (one stage program each, same chunk
// size) in one launch: workgroup b runs chunk b - first_block[j] of job j,
// where job j is the last with first_block[j] <= b.
template <typename R, int RB, bool QD>
__global__ __launch_bounds__(kStageMaxThreads) void k_stage_multi(const StageJobs J)
{
    const uint32_t b = blockIdx.x;
    uint32_t lo = 0, hi = J.n;  // first_block[lo] <= b < first_block[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (J.first_block[mid] <= b) lo = mid;
        else hi = mid;
    }
    const StageJob &job = J.job[lo];
    const uint64_t chunk = b - J.first_block[lo];
    stage_chunks<R, RB, QD>((c2_t<R> *)job.state, job.prog, (const c2_t<R> *)job.tables, chunk, chunk + 1, 1, 0,
                            (const c2_t<R> *)job.kron_lo, (const c2_t<R> *)job.kron_hi, job.kron_nlo);
}

template <typename R, int RB, bool QD> hipError_t stage_lds_attr()
{
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)k_stage<R, RB, QD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kStageLdsBytes);
    // the batched kernel with quadratic-phase operators exists for complex128
    // only (in complex64 it would need scratch memory)
    if constexpr (!QD || sizeof(R) == 8)
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_stage_multi<R, RB, QD>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStageLdsBytes);
    done = e == hipSuccess;
    return e;
}

}  // namespace

template <typename R>
hipError_t launch_stage(const StageLaunch &L, hipStream_t s)
{
    constexpr int RB = sizeof(R) == 8 ? 4 : 5;
    const int C = L.C;
    if (C < RB + 6 || C > 16) return hipErrorInvalidValue;
    const uint32_t threads = 1u << (C - RB);
    const uint32_t lds = (uint32_t)sizeof(c2_t<R>) << C;
    if (threads > (uint32_t)kStageMaxThreads || lds > kStageLdsBytes) return hipErrorInvalidValue;
    hipError_t e = L.quad ? stage_lds_attr<R, RB, true>() : stage_lds_attr<R, RB, false>();
    if (e != hipSuccess) return e;
    // at most 2^15 workgroups: on large states each walks several chunks, so
    // its set-up (thread bases, mapping tables) is paid once per several
    // chunks (measured best on MI355X against one chunk per workgroup and
    // against fewer, longer-lived workgroups)
    uint64_t grid = L.nchunks;
    if (grid > (1ull << 15)) grid = 1ull << 15;
    if (L.kron_lo && (L.kron_nlo < 1 || L.kron_nlo >= L.n || !L.kron_hi)) return hipErrorInvalidValue;
    if (L.quad) {
        k_stage<R, RB, true><<<(uint32_t)grid, threads, lds, s>>>(
            (c2_t<R> *)L.state, L.prog, (const c2_t<R> *)L.tables, L.nchunks, L.xbits, (const c2_t<R> *)L.kron_lo,
            (const c2_t<R> *)L.kron_hi, L.kron_nlo);
        return hipGetLastError();
    }
        k_stage<R, RB, false><<<(uint32_t)grid, threads, lds, s>>>(
            (c2_t<R> *)L.state, L.prog, (const c2_t<R> *)L.tables, L.nchunks, L.xbits, (const c2_t<R> *)L.kron_lo,
            (const c2_t<R> *)L.kron_hi, L.kron_nlo);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stage_multi(const StageJobs &J, int C, bool quad, hipStream_t s)
{
    constexpr int RB = sizeof(R) == 8 ? 4 : 5;
    if (C < RB + 6 || C > 16 || J.n == 0 || J.n > kStageJobsMax) return hipErrorInvalidValue;
    const uint32_t threads = 1u << (C - RB);
    const uint32_t lds = (uint32_t)sizeof(c2_t<R>) << C;
    if (threads > (uint32_t)kStageMaxThreads || lds > kStageLdsBytes) return hipErrorInvalidValue;
    for (uint32_t j = 0; j < J.n; ++j)
        if (J.first_block[j + 1] <= J.first_block[j] || J.job[j].state == nullptr || J.job[j].prog == nullptr)
            return hipErrorInvalidValue;
    if (J.first_block[0] != 0) return hipErrorInvalidValue;
    if constexpr (sizeof(R) == 8) {
        if (quad) {
            hipError_t e = stage_lds_attr<R, RB, true>();
            if (e != hipSuccess) return e;
            k_stage_multi<R, RB, true><<<J.first_block[J.n], threads, lds, s>>>(J);
            return hipGetLastError();
        }
    } else if (quad) {
        return hipErrorInvalidValue;
    }
    hipError_t e = stage_lds_attr<R, RB, false>();
    if (e != hipSuccess) return e;
    k_stage_multi<R, RB, false><<<J.first_block[J.n], threads, lds, s>>>(J);
    return hipGetLastError();
}

template hipError_t launch_stage<double>(const StageLaunch &, hipStream_t);
template hipError_t launch_stage<float>(const StageLaunch &, hipStream_t);
template hipError_t launch_stage_multi<double>(const StageJobs &, int, bool, hipStream_t);
template hipError_t launch_stage_multi<float>(const StageJobs &, int, bool, hipStream_t);

}  // namespace qs
