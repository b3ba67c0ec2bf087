// C ABI of the simulator and the executor that runs a plan on the device
// (adaptive simulation, Alg. 5: tensor product, fused diagonal, dense gate,
// chunk-wise stage; Alg. 1 when no optimisation is enabled).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "device.hpp"
#include "ir.hpp"
#include "qsim355.h"

using qs::cplx;

namespace {

struct Prepared {
    sim_op_kind kind;
    int buffer = 0, nb = 0;
    qs::GateDesc gd{};          // DENSE / DIAG
    int lo = 0, hi = 0;         // KRON sources
    int npairs = 0;             // PERM: exchanged physical bit pairs
    int plo[6] = {0}, phi[6] = {0};
    size_t prog_off = 0;        // STAGE: word offset of its program
    int C = 0, nph = 0;
    uint64_t nchunks = 0;
    int outer_lo = 0, outer_n = 0, pass_ops = 0;  // WINDOW (host-memory offload pass)
    bool init_window = false;
    bool small = false;         // STAGE run by the small-state kernel
    bool mfma = false;          // DENSE on the matrix cores (table holds the real-ified matrix)
    uint32_t item = 0;          // index of its SmallItem
    uint32_t batch = 0;         // ops of the batch starting here (0 = inside a batch)
    bool fused = false;         // KRON formed by the next stage's chunk loads (not launched)
    bool kron = false;          // STAGE: its chunks are the tensor product of buffers klo, khi
    int klo = 0, khi = 0;
    bool quad = false;          // STAGE: has quadratic-phase operators (kernel variant with them)
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

hipError_t grow(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

const char *kNullCtx = "null context";

}  // namespace

// ---- allocation-free outputs ------------------------------------------------
// Device scratch for callers that cannot allocate (sim_probabilities_noalloc):
// one array per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address (it is a host-side stand-in): the
// device address comes from hipGetSymbolAddress, once per device, at
// sim_create.
namespace {
constexpr size_t kNoAllocScratchBytes = 24ull << 20;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

struct sim_plan {
    qs::Plan plan;
};

struct sim_ctx {
    int n = 0;
    sim_dtype dtype = SIM_C128;
    qs::Options opt;
    void *state = nullptr;
    uint64_t state_bytes = 0;
    hipStream_t stream = nullptr;
    int device = 0;

    std::vector<qs::Operator> gates;
    qs::Plan plan;
    bool loaded = false, ran = false;
    // logical -> physical qubit map of the state the last run produced: the
    // plan's layout after sim_run, the identity after a batched small-state
    // run (which applies the input gates in logical order)
    std::vector<int> layout;

    DevBuf tables, prog, gdesc, items, scratch, io;
    std::vector<DevBuf> subbufs;          // booster sub-states (index = buffer id)
    std::vector<Prepared> prep;
    std::vector<qs::SmallItem> host_items;
    bool small_whole = false;              // whole circuit as one small-state item (batched runs)
    size_t small_whole_item = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // host-memory offload: the state lives in `host`; `state` holds two
    // device windows of 2^window amplitudes; copies run on h2d / d2h
    void *host = nullptr;
    void *host_dev = nullptr;              // the same memory as the device addresses it
    uint64_t host_bytes = 0;
    int window = 0;
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr}, ev_out[2] = {nullptr, nullptr};
    hipEvent_t ev_pass = nullptr;
    bool timing_pending = false;
    bool profiling = false, profiled = false;
    std::vector<hipEvent_t> op_ev;       // 2 per plan op when profiling
    sim_run_stats stats{};
    std::string err;

    size_t amp_bytes() const { return dtype == SIM_C128 ? 16 : 8; }
    void *buf(int id) { return id == 0 ? state : subbufs[id].p; }
};

namespace {

sim_status fail(sim_ctx *c, sim_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

sim_status hip_fail(sim_ctx *c, hipError_t e, const char *where)
{
    return fail(c, SIM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr, where)                         \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

bool convert_gates(const sim_gate *gates, uint64_t ng, int n, std::vector<qs::Operator> &out, std::string *err)
{
    out.clear();
    out.reserve(ng);
    for (uint64_t i = 0; i < ng; ++i) {
        std::string e;
        qs::Operator op = qs::gate_operator(gates[i], n, &e);
        if (!e.empty()) {
            *err = "gate " + std::to_string(i) + ": " + e;
            return false;
        }
        out.push_back(std::move(op));
    }
    return true;
}

// Device form of a quadratic-phase operator in one register phase (the
// kernel side is quad_op in kernel_stage.hip): one block of complex FP64 unit
// factors (appended to `block`; the caller stores it in the program words, so
// that it keeps FP64 for complex64 states too).  First the per-thread rows, indexed by the thread id:
// e^{i(c + form on the thread bits)}, then for each register bit b
// e^{i(a_b + sum over set thread bits t of b(t, b))}; then e^{i b(b, b')} for
// the register-bit pairs b < b'.  Then the chunk rows: the chunk bits are the
// buffer's global qubits in ascending order, and the chunk index g splits
// into its low h bits and the rest.  Low row g_lo: e^{i beta_j(g_lo)} for the
// C local bits j, e^{i gamma_l(g_lo)} for the high chunk bits hi_l (gamma_l =
// sum over set low bits i of b(i, hi_l)), then e^{i phi(g_lo)}; high row g_hi:
// e^{i beta_j(g_hi)} for j < C, then e^{i phi(g_hi)}, with beta_j(g) the sum
// over set chunk bits i of b(i, j) and phi(g) the form on the chunk bits
// alone.  A row is the row of g without its top bit times that bit's factors
// (one complex multiply per entry); the phase column is summed as an angle.
// Returns the entry offsets of the low and the high rows in the block,
// h | (number of high bits) << 8, and the entry offset of the pair factors.
static std::array<uint32_t, 4> encode_quad(const qs::KOp &k, int C, int n, int reg_bits, uint32_t rmask,
                                                 const std::vector<int> &tmap, const std::vector<int> &local,
                                                 uint64_t L, std::vector<cplx> &tables)
{
    auto B = [&](int q, int p) { return q < p ? k.qb[(size_t)q * n + p] : k.qb[(size_t)p * n + q]; };
    const size_t start = tables.size();
    // register bit b <-> the b-th set bit of the register mask (local index)
    int regloc[8], nr = 0;
    for (int i = 0; i < C; ++i)
        if ((rmask >> i) & 1) regloc[nr++] = i;
    if (nr != reg_bits) throw std::runtime_error("encode_quad: register mask");
    const int nt = C - reg_bits;
    for (uint64_t tid = 0; tid < (1ull << nt); ++tid) {
        double e = k.qc;
        for (int i = 0; i < nt; ++i) {
            if (!((tid >> i) & 1)) continue;
            const int qi = local[tmap[i]];
            e += k.qa[qi];
            for (int i2 = i + 1; i2 < nt; ++i2)
                if ((tid >> i2) & 1) e += B(qi, local[tmap[i2]]);
        }
        tables.push_back(std::polar(1.0, e));
        for (int b = 0; b < reg_bits; ++b) {
            const int qb = local[regloc[b]];
            double u = k.qa[qb];
            for (int i = 0; i < nt; ++i)
                if ((tid >> i) & 1) u += B(local[tmap[i]], qb);
            tables.push_back(std::polar(1.0, u));
        }
    }
    const uint32_t pairs = (uint32_t)(tables.size() - start);
    for (int b = 0; b < reg_bits; ++b)
        for (int b2 = b + 1; b2 < reg_bits; ++b2)
            tables.push_back(std::polar(1.0, B(local[regloc[b]], local[regloc[b2]])));
    std::vector<int> gpos;
    for (int q = 0; q < n; ++q)
        if (!((L >> q) & 1)) gpos.push_back(q);
    const int nG = (int)gpos.size(), h = (nG + 1) / 2, nhi = nG - h;
    auto rows = [&](int first, int nb, bool cross) {
        const int ncol = C + (cross ? nhi : 0) + 1;
        const size_t at = tables.size();
        tables.resize(at + ((size_t)ncol << nb), cplx(1.0, 0.0));
        std::vector<double> phi((size_t)1 << nb, 0.0);
        std::vector<cplx> f(ncol - 1);
        for (int t = 0; t < nb; ++t) {
            const int qt = gpos[first + t];
            for (int j = 0; j < C; ++j) f[j] = std::polar(1.0, B(qt, local[j]));
            if (cross)
                for (int l = 0; l < nhi; ++l) f[C + l] = std::polar(1.0, B(qt, gpos[h + l]));
            for (uint64_t g = 1ull << t; g < (2ull << t); ++g) {
                const uint64_t g0 = g ^ (1ull << t);
                cplx *row = &tables[at + g * ncol];
                const cplx *prev = &tables[at + g0 * ncol];
                for (int c = 0; c < ncol - 1; ++c) row[c] = prev[c] * f[c];
                double d = k.qa[qt];
                for (int i = 0; i < t; ++i)
                    if ((g0 >> i) & 1) d += B(gpos[first + i], qt);
                phi[g] = phi[g0] + d;
            }
        }
        for (uint64_t g = 0; g < (1ull << nb); ++g) tables[at + g * ncol + ncol - 1] = std::polar(1.0, phi[g]);
        return (uint32_t)(at - start);
    };
    const uint32_t lo = rows(0, h, true);
    const uint32_t hi = rows(h, nhi, false);
    return {lo, hi, (uint32_t)h | ((uint32_t)nhi << 8), pairs};
}

// Program words of one stage (layout documented in kernel_stage.hip).
// amp_bytes: bytes of one table entry on the device (16 complex128, 8 complex64).
void encode_stage(const qs::PlanOp &st, int reg_bits, uint32_t amp_bytes, std::vector<uint32_t> &w,
                  std::vector<cplx> &tables)
{
    const int C = (int)st.local.size(), n = st.buffer_qubits;
    const int NR = 1 << reg_bits;
    const bool c64 = amp_bytes == 8;
    const uint32_t amp_shift = c64 ? 3u : 4u;
    if (st.phases.size() > 96) throw std::runtime_error("encode_stage: too many phases");
    const size_t base = w.size();
    w.resize(base + qs::kStageHeaderWords, 0);
    uint64_t L = 0;
    int local_of[64];
    for (int q = 0; q < 64; ++q) local_of[q] = -1;
    for (int i = 0; i < C; ++i) {
        L |= 1ull << st.local[i];
        local_of[st.local[i]] = i;
    }
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    const uint64_t G = all & ~L;
    // swizzled LDS byte offsets of the register part of a local index
    auto reg_offsets = [&](uint32_t rmask, uint32_t *dst) {
        int pos[8], nb = 0;
        for (int i = 0; i < C; ++i)
            if ((rmask >> i) & 1) pos[nb++] = i;
        for (int j = 0; j < NR; ++j) {
            uint32_t r = 0;
            for (int b = 0; b < nb; ++b)
                if ((j >> b) & 1) r |= 1u << pos[b];
            dst[j] = qs::stage_swizzle(r, c64) << amp_shift;
        }
    };
    w[base + 0] = (uint32_t)C;
    w[base + 1] = (uint32_t)n;
    w[base + 2] = (uint32_t)st.phases.size();
    w[base + 3] = (uint32_t)reg_bits;
    w[base + 4] = (uint32_t)L;
    w[base + 5] = (uint32_t)(L >> 32);
    w[base + 6] = (uint32_t)G;
    w[base + 7] = (uint32_t)(G >> 32);
    for (int i = 0; i < C; ++i) w[base + 8 + i] = (uint32_t)st.local[i];
    {
        const uint32_t neutral_r = ((1u << C) - 1) & ~((1u << (C - reg_bits)) - 1);
        reg_offsets(neutral_r, &w[base + 128]);
    }
    std::vector<uint32_t> qwords;                    // FP64 blocks of quadratic-phase operators
    std::vector<std::pair<size_t, size_t>> qpatch;  // (op word in w, block offset in qwords)
    for (size_t p = 0; p < st.phases.size(); ++p) {
        const qs::Phase &ph = st.phases[p];
        w[base + 32 + p] = (uint32_t)(w.size() - base);
        const size_t pb = w.size();
        w.resize(pb + qs::kStagePhaseWords + NR + 16 * ph.ops.size(), 0);
        uint32_t rmask = 0;
        for (int i : ph.reg) rmask |= 1u << i;
        const uint32_t nonr = ((1u << C) - 1) & ~rmask;
        if ((int)ph.tmap.size() != C - reg_bits) throw std::runtime_error("encode_stage: bad thread map");
        const int nwave = C - reg_bits - 6;
        if (nwave < 0 || nwave > 8) throw std::runtime_error("encode_stage: bad thread count");
        w[pb + 0] = (uint32_t)ph.ops.size();
        w[pb + 1] = nonr;
        w[pb + 2] = rmask;
        w[pb + 3] = (uint32_t)nwave;
        for (size_t i = 0; i < ph.tmap.size(); ++i) w[pb + 4 + i / 4] |= (uint32_t)ph.tmap[i] << (8 * (i % 4));
        // physical bit of each wave bit of the thread id (thread-id bits 6, 7, ...)
        for (int i = 0; i < nwave; ++i)
            w[pb + 8 + i / 4] |= (uint32_t)st.local[ph.tmap[6 + i]] << (8 * (i % 4));
        reg_offsets(rmask, &w[pb + qs::kStagePhaseWords]);
        std::vector<int> reg_phys;
        for (int i : ph.reg) reg_phys.push_back(st.local[i]);
        int tid_bit_of_local[64];
        for (int i = 0; i < 64; ++i) tid_bit_of_local[i] = -1;
        for (size_t i = 0; i < ph.tmap.size(); ++i) tid_bit_of_local[ph.tmap[i]] = (int)i;
        for (size_t o = 0; o < ph.ops.size(); ++o) {
            const qs::KOp &k = ph.ops[o];
            uint32_t *op = &w[pb + qs::kStagePhaseWords + NR + 16 * o];
            const uint64_t toff = tables.size();
            if (k.type == qs::KOp::QUAD) {
                std::vector<cplx> blk;
                const auto offs = encode_quad(k, C, n, reg_bits, rmask, ph.tmap, st.local, L, blk);
                op[0] = 3u;
                op[4] = offs[0];
                op[5] = offs[2];
                op[6] = offs[1];
                op[7] = offs[3];
                // word offset of the block, set once the phases are laid out
                qpatch.push_back({(size_t)(op - w.data()) + 3, qwords.size()});
                const size_t at = qwords.size();
                qwords.resize(at + 4 * blk.size());
                std::memcpy(&qwords[at], blk.data(), blk.size() * sizeof(cplx));
                continue;
            }
            uint32_t mask = 0;
            std::vector<int> sel;
            if (k.type == qs::KOp::DENSE) {
                mask = k.reg_mask;
                // the stage kernel applies dense operators on one or two
                // register bits or on the whole register tile
                const int kr = __builtin_popcount(mask);
                if (mask >= (1u << reg_bits) || !(kr == 1 || kr == 2 || kr == reg_bits))
                    throw std::runtime_error("encode_stage: unsupported register mask");
                sel = k.sel;
                tables.insert(tables.end(), k.table.begin(), k.table.end());
            } else {
                // diagonal: register bits of the index -> mask, the other bits
                // select a block of 2^|mask| factors (table [sel][register part])
                std::vector<int> regbit_of(k.dq.size(), -1), selbit_of(k.dq.size(), -1);
                for (size_t t = 0; t < k.dq.size(); ++t) {
                    int b = -1;
                    for (int u = 0; u < reg_bits; ++u)
                        if (reg_phys[u] == k.dq[t]) b = u;
                    if (b >= 0) {
                        mask |= 1u << b;
                        regbit_of[t] = b;
                    } else {
                        selbit_of[t] = (int)sel.size();
                        sel.push_back(k.dq[t]);
                    }
                }
                const int km = __builtin_popcount(mask);
                std::vector<int> rank(reg_bits, -1);  // register bit -> bit of the register part
                for (int u = 0, r = 0; u < reg_bits; ++u)
                    if ((mask >> u) & 1) rank[u] = r++;
                if (sel.size() > 24) throw std::runtime_error("encode_stage: diagonal too wide");
                std::vector<cplx> tab((size_t)1 << (sel.size() + km));
                for (uint64_t sv = 0; sv < (1ull << sel.size()); ++sv)
                    for (uint64_t jm = 0; jm < (1ull << km); ++jm) {
                        uint64_t y = 0;
                        for (size_t t = 0; t < k.dq.size(); ++t) {
                            const uint64_t bit = regbit_of[t] >= 0 ? (jm >> rank[regbit_of[t]]) & 1
                                                                   : (sv >> selbit_of[t]) & 1;
                            y |= bit << t;
                        }
                        tab[(sv << km) | jm] = k.table[y];
                    }
                tables.insert(tables.end(), tab.begin(), tab.end());
            }
            if (sel.size() > 28) throw std::runtime_error("encode_stage: too many selector bits");
            // selector source bytes: a lane bit of the thread id (0x80 | bit), or
            // the physical position of a chunk or wave bit (wave-uniform)
            bool uni = true;
            uint32_t nfield = 0;
            std::vector<std::pair<int, int>> fields;
            for (int q : sel)
                if (local_of[q] >= 0 && tid_bit_of_local[local_of[q]] >= 0 && tid_bit_of_local[local_of[q]] < 6)
                    uni = false;
            if (uni && sel.size() > 1) {
                // wave-uniform selectors in ascending physical order (the
                // table's blocks permuted to match), so that selectors on
                // consecutive bits are read as one bit field
                std::vector<int> order(sel.size());
                for (size_t t = 0; t < sel.size(); ++t) order[t] = (int)t;
                std::sort(order.begin(), order.end(), [&](int x, int y) { return sel[x] < sel[y]; });
                std::vector<int> rank(sel.size());
                for (size_t t = 0; t < sel.size(); ++t) rank[order[t]] = (int)t;
                const int kmb = __builtin_popcount(mask);
                const size_t blk = k.type == qs::KOp::DENSE ? (1ull << (2 * kmb)) : (1ull << kmb);
                const size_t nblk = 1ull << sel.size();
                std::vector<cplx> perm(blk * nblk);
                for (size_t bi = 0; bi < nblk; ++bi) {
                    size_t bo = 0;
                    for (size_t t = 0; t < sel.size(); ++t) bo |= ((bi >> t) & 1ull) << rank[t];
                    std::copy(tables.begin() + toff + bi * blk, tables.begin() + toff + (bi + 1) * blk,
                              perm.begin() + bo * blk);
                }
                std::copy(perm.begin(), perm.end(), tables.begin() + toff);
                std::vector<int> sorted(sel.size());
                for (size_t t = 0; t < sel.size(); ++t) sorted[rank[t]] = sel[t];
                sel.swap(sorted);
            }
            if (uni && !sel.empty()) {
                // bit fields: runs of consecutive physical positions (at most
                // five; more and the kernel reads the source bytes one by one)
                std::vector<std::pair<int, int>> runs;
                for (int q : sel) {
                    if (!runs.empty() && runs.back().first + runs.back().second == q) ++runs.back().second;
                    else runs.push_back({q, 1});
                }
                if (runs.size() <= 6) nfield = (uint32_t)runs.size();
                fields = runs;
            }
            for (size_t t = 0; t < sel.size() && !nfield; ++t) {
                const int q = sel[t];
                uint32_t code = (uint32_t)q;
                if (local_of[q] >= 0) {
                    const int tb = tid_bit_of_local[local_of[q]];
                    if (tb < 0) throw std::runtime_error("encode_stage: selector on a register bit");
                    if (tb < 6) {
                        code = 0x80u | (uint32_t)tb;
                        uni = false;
                    }
                }
                op[3 + t / 4] |= code << (8 * (t % 4));
            }
            for (uint32_t f = 0; f < nfield; ++f)
                op[3 + f] = (uint32_t)fields[f].first | ((uint32_t)fields[f].second << 16);
            const int km = __builtin_popcount(mask);
            const uint32_t shift = (k.type == qs::KOp::DENSE ? 2u * (uint32_t)km : (uint32_t)km) + amp_shift;
            op[0] = (k.type == qs::KOp::DENSE ? 1u : 2u) | (mask << 8) | ((uint32_t)sel.size() << 16) |
                    (nfield << 21) | ((uni ? 1u : 0u) << 24) | (shift << 25);
            const uint64_t tbytes = toff * amp_bytes;
            op[1] = (uint32_t)tbytes;
            op[2] = (uint32_t)(tbytes >> 32);
        }
    }
    if (!qwords.empty()) {
        // the FP64 blocks follow the phases, 16-byte aligned in the program
        // buffer (its device copy starts at a 256-byte boundary)
        while (w.size() & 3) w.push_back(0);
        const size_t at = w.size();
        w.insert(w.end(), qwords.begin(), qwords.end());
        for (const auto &pq : qpatch) w[pq.first] = (uint32_t)(at + pq.second - base);
    }
}

qs::GateDesc desc_of(const qs::Operator &g, uint64_t toff)
{
    qs::GateDesc d{};
    d.diag = g.diag ? 1u : 0u;
    d.k = (uint32_t)g.k();
    for (int t = 0; t < g.k() && t < 24; ++t) d.q[t] = g.q[t];
    if (!g.diag) {
        std::vector<int> s = g.q;
        std::sort(s.begin(), s.end());
        for (int t = 0; t < g.k() && t < 6; ++t) d.sorted[t] = s[t];
    }
    d.table = toff;
    return d;
}

template <typename R>
std::vector<qs::c2_t<R>> to_device_precision(const std::vector<cplx> &v)
{
    std::vector<qs::c2_t<R>> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        out[i].x = (R)v[i].real();
        out[i].y = (R)v[i].imag();
    }
    return out;
}

// Uploads every table and program of the plan and prepares the launches.
sim_status prepare(sim_ctx *c)
{
    const qs::Plan &P = c->plan;
    std::vector<cplx> tables;
    std::vector<uint32_t> prog;
    std::vector<qs::GateDesc> gdesc;
    std::vector<qs::SmallItem> items;
    std::vector<size_t> item_gate_off;
    c->prep.clear();
    // sub-state buffers
    c->subbufs.resize(P.buffer_qubits.size());
    for (size_t b = 1; b < P.buffer_qubits.size(); ++b) {
        hipError_t e = grow(c->subbufs[b], c->amp_bytes() << P.buffer_qubits[b]);
        if (e != hipSuccess) return hip_fail(c, e, "sub-state allocation");
    }
    const int small_max = qs::small_max_qubits(c->dtype == SIM_C128);
    for (const qs::PlanOp &op : P.ops) {
        Prepared p;
        p.kind = op.kind;
        p.buffer = op.buffer;
        p.nb = op.buffer_qubits;
        switch (op.kind) {
        case SIM_OP_INIT:
            break;
        case SIM_OP_KRON:
            p.lo = op.src_lo;
            p.hi = op.src_hi;
            break;
        case SIM_OP_DENSE:
        case SIM_OP_DIAG: {
            const uint64_t toff = tables.size();
            const int k = op.op.k();
            // fused gates on the matrix cores from k = 4 (FP64) / k = 3 (FP32;
            // the FP64 three-qubit gate measured faster on the VALU kernel)
            const int kmin = c->dtype == SIM_C64 ? 3 : 4;
            if (!op.op.diag && k >= kmin && k <= 5 && op.buffer_qubits >= k + 4) {
                // real-ified 2^(k+1) x 2^(k+1) matrix for the MFMA kernel,
                // stored as consecutive pairs of reals
                const int d = 1 << k, D = 2 * d;
                std::vector<double> mr((size_t)D * D);
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) {
                        const cplx u = op.op.m[(size_t)r * d + c];
                        mr[(size_t)(2 * r) * D + 2 * c] = u.real();
                        mr[(size_t)(2 * r) * D + 2 * c + 1] = -u.imag();
                        mr[(size_t)(2 * r + 1) * D + 2 * c] = u.imag();
                        mr[(size_t)(2 * r + 1) * D + 2 * c + 1] = u.real();
                    }
                for (size_t i = 0; i < mr.size(); i += 2) tables.push_back(cplx(mr[i], mr[i + 1]));
                p.mfma = true;
            } else {
                tables.insert(tables.end(), op.op.m.begin(), op.op.m.end());
            }
            p.gd = desc_of(op.op, toff);
            break;
        }
        case SIM_OP_WINDOW:
            p.outer_lo = op.outer_lo;
            p.outer_n = op.outer_n;
            p.pass_ops = op.pass_ops;
            p.init_window = op.init_window;
            break;
        case SIM_OP_PERM: {
            // a product of exchanges of low bits (< 6) with high bits
            const int low = std::min(6, op.buffer_qubits);
            for (int q = 0; q < op.buffer_qubits; ++q) {
                const int d = op.perm[q];
                if (d == q) continue;
                if (op.perm[d] != q) return fail(c, SIM_E_UNSUPPORTED, "permutation is not a product of swaps");
                if (q < low) {
                    if (d < low || p.npairs >= 6) return fail(c, SIM_E_UNSUPPORTED, "unsupported permutation");
                    p.plo[p.npairs] = q;
                    p.phi[p.npairs] = d;
                    ++p.npairs;
                } else if (d >= low) {
                    return fail(c, SIM_E_UNSUPPORTED, "unsupported permutation");
                }
            }
            break;
        }
        case SIM_OP_STAGE: {
            const bool whole = (int)op.local.size() == op.buffer_qubits;
            if (whole && op.buffer_qubits <= small_max && op.phases.empty() && !c->window) {
                p.small = true;
                qs::SmallItem it{};
                it.n = (uint32_t)op.buffer_qubits;
                it.ngates = (uint32_t)op.gates.size();
                it.init = 0;
                item_gate_off.push_back(gdesc.size());
                for (const qs::Operator &g : op.gates) {
                    gdesc.push_back(desc_of(g, tables.size()));
                    tables.insert(tables.end(), g.m.begin(), g.m.end());
                }
                p.item = (uint32_t)items.size();
                it.state = c->buf(op.buffer);
                items.push_back(it);
            } else {
                p.prog_off = prog.size();
                p.C = (int)op.local.size();
                p.nph = (int)op.phases.size();
                p.nchunks = 1ull << (op.buffer_qubits - p.C);
                encode_stage(op, c->opt.reg_bits, c->dtype == SIM_C64 ? 8u : 16u, prog, tables);
                for (const qs::Phase &ph : op.phases)
                    for (const qs::KOp &k : ph.ops) p.quad |= k.type == qs::KOp::QUAD;
            }
            break;
        }
        default:
            return fail(c, SIM_E_UNSUPPORTED, "plan op kind not executable");
        }
        c->prep.push_back(p);
    }
    // the whole circuit as one small-state item, for batched launches of
    // many small circuits (sim_run_batch)
    c->small_whole = c->n <= small_max && !c->window;
    if (c->small_whole) {
        qs::SmallItem it{};
        it.n = (uint32_t)c->n;
        it.ngates = (uint32_t)c->gates.size();
        it.init = 1;
        it.state = c->state;
        item_gate_off.push_back(gdesc.size());
        for (const qs::Operator &g : c->gates) {
            gdesc.push_back(desc_of(g, tables.size()));
            tables.insert(tables.end(), g.m.begin(), g.m.end());
        }
        c->small_whole_item = items.size();
        items.push_back(it);
    }
    // batches of consecutive small runs on distinct buffers
    for (size_t i = 0; i < c->prep.size();) {
        if (!c->prep[i].small) {
            ++i;
            continue;
        }
        size_t j = i;
        std::vector<int> seen;
        while (j < c->prep.size() && c->prep[j].small &&
               std::find(seen.begin(), seen.end(), c->prep[j].buffer) == seen.end()) {
            seen.push_back(c->prep[j].buffer);
            ++j;
        }
        c->prep[i].batch = (uint32_t)(j - i);
        i = j;
    }
    // the booster's last tensor product (into the full state) is formed by the
    // next stage while it loads its chunks: the product is never written to
    // HBM and read back
    for (size_t i = 0; i + 1 < c->prep.size(); ++i) {
        Prepared &k = c->prep[i], &st = c->prep[i + 1];
        if (k.kind == SIM_OP_KRON && k.buffer == 0 && st.kind == SIM_OP_STAGE && st.buffer == 0 && !st.small &&
            !c->window) {
            k.fused = true;
            st.kron = true;
            st.klo = k.lo;
            st.khi = k.hi;
        }
    }
    // upload
    const size_t amp = c->amp_bytes();
    HIPCHK(c, grow(c->tables, std::max<size_t>(tables.size() * amp, 256)), "table allocation");
    HIPCHK(c, grow(c->prog, std::max<size_t>(prog.size() * 4, 256)), "program allocation");
    HIPCHK(c, grow(c->gdesc, std::max<size_t>(gdesc.size() * sizeof(qs::GateDesc), 256)), "gate allocation");
    HIPCHK(c, grow(c->items, std::max<size_t>(items.size() * sizeof(qs::SmallItem), 256)), "item allocation");
    for (size_t i = 0; i < items.size(); ++i) {
        items[i].gates = (const qs::GateDesc *)c->gdesc.p + item_gate_off[i];
        items[i].tables = c->tables.p;
    }
    if (!tables.empty()) {
        if (c->dtype == SIM_C128) {
            auto t = to_device_precision<double>(tables);
            HIPCHK(c, hipMemcpyAsync(c->tables.p, t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice, c->stream),
                   "table upload");
            HIPCHK(c, hipStreamSynchronize(c->stream), "table upload");
        } else {
            auto t = to_device_precision<float>(tables);
            HIPCHK(c, hipMemcpyAsync(c->tables.p, t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice, c->stream),
                   "table upload");
            HIPCHK(c, hipStreamSynchronize(c->stream), "table upload");
        }
    }
    if (!prog.empty())
        HIPCHK(c, hipMemcpyAsync(c->prog.p, prog.data(), prog.size() * 4, hipMemcpyHostToDevice, c->stream),
               "program upload");
    if (!gdesc.empty())
        HIPCHK(c, hipMemcpyAsync(c->gdesc.p, gdesc.data(), gdesc.size() * sizeof(qs::GateDesc), hipMemcpyHostToDevice,
                                 c->stream),
               "gate upload");
    if (!items.empty())
        HIPCHK(c, hipMemcpyAsync(c->items.p, items.data(), items.size() * sizeof(qs::SmallItem), hipMemcpyHostToDevice,
                                 c->stream),
               "item upload");
    HIPCHK(c, hipStreamSynchronize(c->stream), "upload");
    c->host_items = items;
    return SIM_OK;
}

// One op of a host-memory offload pass on a device window (qubits are window
// bits; xbits carries the window's outer qubits at bits W and above for the
// stage kernel's selectors).
template <typename R>
hipError_t launch_window_op(sim_ctx *c, const Prepared &p, void *buf, uint64_t xbits)
{
    const size_t amp = c->amp_bytes();
    switch (p.kind) {
    case SIM_OP_STAGE: {
        qs::StageLaunch L;
        L.state = buf;
        L.prog = (const uint32_t *)c->prog.p + p.prog_off;
        L.tables = c->tables.p;
        L.n = p.nb;
        L.C = p.C;
        L.nphases = p.nph;
        L.nchunks = p.nchunks;
        L.xbits = xbits;
        L.quad = p.quad;
        return qs::launch_stage<R>(L, c->stream);
    }
    case SIM_OP_DENSE:
        if (p.mfma)
            return qs::launch_dense_mfma<R>(buf, p.nb, p.gd, (const char *)c->tables.p + p.gd.table * amp, c->stream);
        return qs::launch_dense<R>(buf, p.nb, p.gd, (const char *)c->tables.p + p.gd.table * amp, c->stream);
    case SIM_OP_DIAG:
        return qs::launch_diag_q<R>(buf, p.nb, (int)p.gd.k, p.gd.q, (const char *)c->tables.p + p.gd.table * amp,
                                    c->stream);
    default:
        return hipErrorInvalidValue;
    }
}

// Host-memory offload: every pass streams the 2^S windows of the state
// (outer qubits fixed, rows of 2^lo amplitudes with a stride of 2^(lo+S))
// through two device buffers: window v is read on the h2d stream while
// window v - 1 is computed and window v - 2 written back on the d2h stream.
template <typename R>
sim_status execute_offload(sim_ctx *c)
{
    const size_t amp = c->amp_bytes();
    const int N = c->n, W = c->window;
    char *win[2] = {(char *)c->state, (char *)c->state + (amp << W)};
    bool first_pass = true;
    for (size_t i = 0; i < c->prep.size();) {
        const Prepared &w = c->prep[i];
        if (w.kind != SIM_OP_WINDOW) return fail(c, SIM_E_UNSUPPORTED, "offload plan: op outside a window pass");
        const int lo = w.outer_lo, S = w.outer_n, m = w.pass_ops;
        if (S != N - W || lo < 0 || lo + S > N || i + (size_t)m >= c->prep.size())
            return fail(c, SIM_E_UNSUPPORTED, "offload plan: bad window pass");
        const uint64_t nwin = 1ull << S;
        const size_t width = amp << lo;  // row bytes: windows are rows of 2^lo amplitudes
        // the windows of this pass overlap every window of the previous one:
        // the first read waits for the last write-back of that pass
        if (!first_pass) HIPCHK(c, hipStreamWaitEvent(c->h2d, c->ev_pass, 0), "wait");
        for (uint64_t v = 0; v < nwin; ++v) {
            const int b = (int)(v & 1);
            char *dbuf = win[b];
            if (w.init_window) {
                HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_out[b], 0), "wait");
                if (v == 0) HIPCHK(c, qs::launch_init<R>(dbuf, W, c->stream), "window init");
                else HIPCHK(c, hipMemsetAsync(dbuf, 0, amp << W, c->stream), "window init");
            } else {
                HIPCHK(c, hipStreamWaitEvent(c->h2d, c->ev_out[b], 0), "wait");
                HIPCHK(c, qs::launch_window_copy(dbuf, c->host_dev, amp << W, width, S, v, false, c->h2d),
                       "window read");
                HIPCHK(c, hipEventRecord(c->ev_in[b], c->h2d), "event record");
                HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_in[b], 0), "wait");
            }
            for (int k = 1; k <= m; ++k) {
                const hipError_t e = launch_window_op<R>(c, c->prep[i + k], dbuf, v << W);
                if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
            }
            HIPCHK(c, hipEventRecord(c->ev_done[b], c->stream), "event record");
            HIPCHK(c, hipStreamWaitEvent(c->d2h, c->ev_done[b], 0), "wait");
            HIPCHK(c, qs::launch_window_copy(c->host_dev, dbuf, amp << W, width, S, v, true, c->d2h), "window write");
            HIPCHK(c, hipEventRecord(c->ev_out[b], c->d2h), "event record");
        }
        HIPCHK(c, hipEventRecord(c->ev_pass, c->d2h), "event record");
        first_pass = false;
        i += (size_t)m + 1;
    }
    // the run ends when the last write-back has landed
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_pass, 0), "wait");
    return SIM_OK;
}

// One prepared op of a resident-state plan on stream st.  hipErrorNotSupported
// marks an op kind this path does not execute.
template <typename R>
hipError_t launch_op(sim_ctx *c, size_t i, hipStream_t st)
{
    const size_t amp = c->amp_bytes();
    const Prepared &p = c->prep[i];
    switch (p.kind) {
    case SIM_OP_INIT:
        return qs::launch_init<R>(c->buf(p.buffer), p.nb, st);
    case SIM_OP_KRON: {
        if (p.fused) return hipSuccess;  // formed by the next stage's loads
        const int nlo = c->plan.buffer_qubits[p.lo], nhi = c->plan.buffer_qubits[p.hi];
        return qs::launch_kron<R>(c->buf(p.buffer), c->buf(p.lo), nlo, c->buf(p.hi), nhi, st);
    }
    case SIM_OP_DENSE:
        if (p.mfma)
            return qs::launch_dense_mfma<R>(c->buf(p.buffer), p.nb, p.gd, (const char *)c->tables.p + p.gd.table * amp,
                                            st);
        return qs::launch_dense<R>(c->buf(p.buffer), p.nb, p.gd, (const char *)c->tables.p + p.gd.table * amp, st);
    case SIM_OP_PERM:
        return qs::launch_swap_bits<R>(c->buf(p.buffer), p.nb, p.plo, p.phi, p.npairs, st);
    case SIM_OP_DIAG:
        return qs::launch_diag_q<R>(c->buf(p.buffer), p.nb, (int)p.gd.k, p.gd.q,
                                    (const char *)c->tables.p + p.gd.table * amp, st);
    case SIM_OP_STAGE:
        if (p.small) {
            if (!p.batch) return hipSuccess;  // launched with the first op of its batch
            uint32_t maxn = 0;
            for (uint32_t u = 0; u < p.batch; ++u) maxn = std::max<uint32_t>(maxn, c->prep[i + u].nb);
            return qs::launch_small_batch<R>((const qs::SmallItem *)c->items.p + p.item, p.batch, maxn, st);
        } else {
            qs::StageLaunch L;
            L.state = c->buf(p.buffer);
            L.prog = (const uint32_t *)c->prog.p + p.prog_off;
            L.tables = c->tables.p;
            L.n = p.nb;
            L.C = p.C;
            L.nphases = p.nph;
            L.nchunks = p.nchunks;
            if (p.kron) {
                L.kron_lo = c->buf(p.klo);
                L.kron_hi = c->buf(p.khi);
                L.kron_nlo = c->plan.buffer_qubits[p.klo];
            }
            L.quad = p.quad;
            return qs::launch_stage<R>(L, st);
        }
    default:
        return hipErrorNotSupported;
    }
}

template <typename R>
sim_status execute(sim_ctx *c)
{
    if (c->window) return execute_offload<R>(c);
    for (size_t i = 0; i < c->prep.size(); ++i) {
        if (c->profiling) HIPCHK(c, hipEventRecord(c->op_ev[2 * i], c->stream), "event record");
        const hipError_t e = launch_op<R>(c, i, c->stream);
        if (e == hipErrorNotSupported) return fail(c, SIM_E_UNSUPPORTED, "plan op kind not executable");
        if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
        if (c->profiling) HIPCHK(c, hipEventRecord(c->op_ev[2 * i + 1], c->stream), "event record");
    }
    return SIM_OK;
}

// Several resident-state plans on one stream, their full-state stages
// launched together: every state runs its ops one by one up to its next
// full-state stage; then the states waiting at a stage (grouped by chunk
// size, up to 64 per launch) run that stage in one launch, one workgroup per
// chunk.  Every chunk computes exactly what the state's own stage launch
// computes for it.
template <typename R>
sim_status execute_staged_batch(sim_ctx *const *cs, uint32_t n, hipStream_t st)
{
    std::vector<size_t> cur(n, 0);
    // complex64 stages with quadratic-phase operators run one state per
    // launch (the batched kernel has no complex64 variant with them)
    auto batched = [](const Prepared &p) {
        return p.kind == SIM_OP_STAGE && !p.small && p.buffer == 0 && !(sizeof(R) == 4 && p.quad);
    };
    for (;;) {
        bool left = false;
        for (uint32_t k = 0; k < n; ++k) {
            sim_ctx *c = cs[k];
            while (cur[k] < c->prep.size() && !batched(c->prep[cur[k]])) {
                const hipError_t e = launch_op<R>(c, cur[k], st);
                if (e == hipErrorNotSupported) return fail(c, SIM_E_UNSUPPORTED, "plan op kind not executable");
                if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
                ++cur[k];
            }
            left |= cur[k] < c->prep.size();
        }
        if (!left) return SIM_OK;
        // states waiting at a full-state stage, by chunk size
        std::vector<uint32_t> wait;
        for (uint32_t k = 0; k < n; ++k)
            if (cur[k] < cs[k]->prep.size()) wait.push_back(k);
        std::stable_sort(wait.begin(), wait.end(), [&](uint32_t a, uint32_t b) {
            return cs[a]->prep[cur[a]].C < cs[b]->prep[cur[b]].C;
        });
        for (size_t w0 = 0; w0 < wait.size();) {
            const int C = cs[wait[w0]]->prep[cur[wait[w0]]].C;
            qs::StageJobs J{};
            size_t w = w0;
            uint64_t blocks = 0;
            bool quad = false;
            while (w < wait.size() && J.n < qs::kStageJobsMax) {
                sim_ctx *c = cs[wait[w]];
                const Prepared &p = c->prep[cur[wait[w]]];
                if (p.C != C || blocks + p.nchunks > 0x7fffffffull) break;
                J.first_block[J.n] = (uint32_t)blocks;
                J.job[J.n].state = c->buf(0);
                J.job[J.n].prog = (const uint32_t *)c->prog.p + p.prog_off;
                J.job[J.n].tables = c->tables.p;
                J.job[J.n].kron_lo = p.kron ? c->buf(p.klo) : nullptr;
                J.job[J.n].kron_hi = p.kron ? c->buf(p.khi) : nullptr;
                J.job[J.n].kron_nlo = p.kron ? c->plan.buffer_qubits[p.klo] : 0;
                quad |= p.quad;
                blocks += p.nchunks;
                ++J.n;
                ++w;
            }
            J.first_block[J.n] = (uint32_t)blocks;
            const hipError_t e = qs::launch_stage_multi<R>(J, C, quad, st);
            if (e != hipSuccess) return hip_fail(cs[wait[w0]], e, "batched stage launch");
            for (size_t u = w0; u < w; ++u) ++cur[wait[u]];
            w0 = w;
        }
    }
}

void fill_stats(const qs::Plan &P, uint64_t n_gates, sim_run_stats *s)
{
    s->n_gates = n_gates;
    s->n_ops = P.stats.n_ops;
    s->full_passes = P.stats.full_passes;
    s->write_passes = P.stats.write_passes;
    s->n_stages = P.stats.n_stages;
    s->n_dense = P.stats.n_dense;
    s->n_diag = P.stats.n_diag;
    s->n_kron = P.stats.n_kron;
    s->n_perm = P.stats.n_perm;
    s->n_subruns = P.stats.n_subruns;
    s->plan_ms = P.stats.plan_ms;
    s->algorithmic_bytes = P.stats.bytes;
    s->flops = P.stats.flops;
    s->est_ms = P.stats.est_ms;
    s->offload_passes = P.stats.offload_passes;
    s->window_qubits = (uint64_t)P.opt.window_qubits;
    s->pcie_bytes = P.stats.pcie_bytes;
}

// Marginal of an offloaded state: its top-qubit slices of 2^W amplitudes
// pass through the device one after the other; each slice's marginal over
// the selected qubits below W goes to the host and is added, slice by slice
// in order, into the bins its top bits select (deterministic).
sim_status offload_marginal(sim_ctx *c, const std::vector<int> &ph, double *out)
{
    const int N = c->n, W = c->window, nq = (int)ph.size();
    const size_t amp = c->amp_bytes();
    std::vector<int> inner;
    for (int q : ph)
        if (q < W) inner.push_back(q);
    std::sort(inner.begin(), inner.end());
    const int ki = (int)inner.size();
    const size_t nib = 1ull << ki;
    const size_t scr = qs::marginal_scratch_bytes(W, inner.data(), ki);
    HIPCHK(c, grow(c->scratch, scr + nib * 8 + 64), "scratch allocation");
    double *dbins = (double *)((char *)c->scratch.p + ((scr + 63) / 64) * 64);
    std::vector<double> bins(nib);
    std::fill(out, out + (1ull << nq), 0.0);
    for (uint64_t v = 0; v < (1ull << (N - W)); ++v) {
        HIPCHK(c, hipMemcpyAsync(c->state, (const char *)c->host + (v * amp << W), amp << W, hipMemcpyHostToDevice,
                                 c->stream),
               "slice read");
        const hipError_t e =
            c->dtype == SIM_C128
                ? qs::launch_marginal<double>(c->state, W, inner.data(), ki, dbins, (double *)c->scratch.p, c->stream)
                : qs::launch_marginal<float>(c->state, W, inner.data(), ki, dbins, (double *)c->scratch.p, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "marginal");
        HIPCHK(c, hipMemcpyAsync(bins.data(), dbins, nib * 8, hipMemcpyDeviceToHost, c->stream), "copy out");
        HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
        for (size_t yb = 0; yb < nib; ++yb) {
            size_t y = 0;
            for (int t = 0; t < nq; ++t) {
                uint64_t bit;
                if (ph[t] < W) bit = (yb >> (std::find(inner.begin(), inner.end(), ph[t]) - inner.begin())) & 1;
                else bit = (v >> (ph[t] - W)) & 1;
                y |= (size_t)bit << t;
            }
            out[y] += bins[yb];
        }
    }
    return SIM_OK;
}

}  // namespace

extern "C" {

const char *sim_version(void) { return "qsim355 0.1 (gfx950)"; }

sim_status sim_device_copy(void *dst, const void *src, uint64_t bytes, void *stream)
{
    if (!dst || !src || (bytes % 16)) return SIM_E_INVAL;
    return qs::launch_copy(dst, src, bytes, (hipStream_t)stream) == hipSuccess ? SIM_OK : SIM_E_DEVICE;
}

sim_status sim_create(uint32_t n_qubits, sim_dtype dtype, const sim_options *opts, sim_ctx **out)
{
    if (!out || !opts) return SIM_E_INVAL;
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 36) return SIM_E_INVAL;
    if (dtype != SIM_C128 && dtype != SIM_C64) return SIM_E_INVAL;
    if (!opts->dev_state) return SIM_E_INVAL;
    // a stage chunk spans at least one full wave of register tiles (2^(rb+6))
    // and at most one 512-thread workgroup of them (2^(rb+9))
    const uint32_t rb = dtype == SIM_C128 ? 4u : 5u;
    if (opts->C && (opts->C < rb + 6 || opts->C > rb + 9)) return SIM_E_INVAL;
    const uint64_t need = (dtype == SIM_C128 ? 16ull : 8ull) << n_qubits;
    if (opts->host_state) {
        // host-memory offload: the state is in host memory, the device
        // buffer holds two windows
        if (opts->host_state_bytes < need) return SIM_E_NOMEM;
        if (!(opts->opt & SIM_OPT_STAGES)) return SIM_E_UNSUPPORTED;
    } else if (opts->dev_state_bytes < need) {
        return SIM_E_NOMEM;
    }
    sim_ctx *c = new (std::nothrow) sim_ctx();
    if (!c) return SIM_E_NOMEM;
    c->n = (int)n_qubits;
    c->dtype = dtype;
    c->opt = qs::resolve_options(opts, dtype, (int)n_qubits);
    c->state = opts->dev_state;
    c->state_bytes = opts->dev_state_bytes;
    c->stream = (hipStream_t)opts->stream;
    if (opts->host_state) {
        c->host = opts->host_state;
        c->host_bytes = opts->host_state_bytes;
        c->window = c->opt.window_qubits;
        // a window holds at least one stage chunk
        if (c->window < std::max<int>((int)c->opt.C, 6 + c->opt.reg_bits)) {
            delete c;
            return SIM_E_NOMEM;
        }
    }
    if (hipGetDevice(&c->device) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess || noalloc_scratch_setup(c->device) != hipSuccess) {
        if (c->ev0) hipEventDestroy(c->ev0);
        if (c->ev1) hipEventDestroy(c->ev1);
        delete c;
        return SIM_E_DEVICE;
    }
    if (c->window) {
        bool ok = hipHostGetDevicePointer(&c->host_dev, c->host, 0) == hipSuccess &&
                  hipStreamCreateWithFlags(&c->h2d, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&c->d2h, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_pass, hipEventDisableTiming) == hipSuccess;
        for (int b = 0; b < 2 && ok; ++b)
            ok = hipEventCreateWithFlags(&c->ev_in[b], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&c->ev_done[b], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&c->ev_out[b], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            sim_destroy(c);
            return SIM_E_DEVICE;
        }
    }
    *out = c;
    return SIM_OK;
}

sim_status sim_load_circuit(sim_ctx *c, const sim_gate *gates, uint64_t n_gates)
{
    if (!c) return SIM_E_INVAL;
    if (!gates && n_gates) return fail(c, SIM_E_INVAL, "gates is NULL");
    std::vector<qs::Operator> ops;
    std::string err;
    if (!convert_gates(gates, n_gates, c->n, ops, &err)) return fail(c, SIM_E_INVAL, err);
    qs::Plan plan;
    plan.n = c->n;
    plan.dtype = c->dtype;
    plan.opt = c->opt;
    try {
        qs::build_plan(plan, ops);
    } catch (const std::exception &ex) {
        return fail(c, SIM_E_UNSUPPORTED, std::string("planner: ") + ex.what());
    }
    std::swap(c->plan, plan);
    std::swap(c->gates, ops);
    sim_status s;
    try {
        s = prepare(c);
    } catch (const std::exception &ex) {
        s = fail(c, SIM_E_UNSUPPORTED, std::string("prepare: ") + ex.what());
    }
    if (s != SIM_OK) {  // keep the old circuit
        std::swap(c->plan, plan);
        std::swap(c->gates, ops);
        if (c->loaded) prepare(c);
        return s;
    }
    c->loaded = true;
    c->ran = false;
    fill_stats(c->plan, c->gates.size(), &c->stats);
    // a tensor product formed on load skips one write and one read of the state
    for (const Prepared &p : c->prep)
        if (p.fused) {
            c->stats.algorithmic_bytes -= 2.0 * (double)(c->amp_bytes() << c->n);
            c->stats.write_passes -= 1;
        }
    return SIM_OK;
}

sim_status sim_run_async(sim_ctx *c)
{
    if (!c) return SIM_E_INVAL;
    if (!c->loaded) return fail(c, SIM_E_STATE, "no circuit loaded");
    if (c->profiling && !c->window) {
        while (c->op_ev.size() < 2 * c->prep.size()) {
            hipEvent_t ev;
            HIPCHK(c, hipEventCreate(&ev), "event create");
            c->op_ev.push_back(ev);
        }
    }
    c->profiled = c->profiling && !c->window;
    HIPCHK(c, hipEventRecord(c->ev0, c->stream), "event record");
    sim_status s = c->dtype == SIM_C128 ? execute<double>(c) : execute<float>(c);
    if (s != SIM_OK) return s;
    HIPCHK(c, hipEventRecord(c->ev1, c->stream), "event record");
    c->timing_pending = true;
    c->ran = true;
    c->layout = c->plan.layout;
    return SIM_OK;
}

sim_status sim_run(sim_ctx *c)
{
    sim_status s = sim_run_async(c);
    if (s != SIM_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1), "event time");
    c->stats.run_ms = ms;
    c->timing_pending = false;
    return SIM_OK;
}

sim_status sim_amplitudes(sim_ctx *c, const uint64_t *idx, uint64_t m, double *out)
{
    if (!c) return SIM_E_INVAL;
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if (!out && m) return fail(c, SIM_E_INVAL, "out is NULL");
    const uint64_t len = 1ull << c->n;
    const std::vector<int> &lay = c->layout;
    bool identity = true;
    for (int q = 0; q < c->n; ++q) identity &= (lay[q] == q);
    // logical -> physical index, one table lookup per byte of the index
    const int nbytes = (c->n + 7) / 8;
    std::vector<uint64_t> spread(identity ? 0 : (size_t)nbytes * 256);
    for (int b = 0; b < (int)spread.size() / 256; ++b)
        for (uint32_t v = 0; v < 256; ++v) {
            uint64_t y = 0;
            for (int t = 0; t < 8 && 8 * b + t < c->n; ++t)
                if ((v >> t) & 1) y |= 1ull << lay[8 * b + t];
            spread[256 * b + v] = y;
        }
    auto phys = [&](uint64_t x) {
        if (identity) return x;
        uint64_t y = 0;
        for (int b = 0; b < nbytes; ++b) y |= spread[256 * b + ((x >> (8 * b)) & 255)];
        return y;
    };
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    if (c->window) {
        // offload: the final state is in host memory (logical = physical order)
        if (idx)
            for (uint64_t i = 0; i < m; ++i)
                if (idx[i] >= len) return fail(c, SIM_E_INVAL, "amplitude index out of range");
        if (!idx && m != len) return fail(c, SIM_E_INVAL, "idx NULL requires n == 2^N");
        for (uint64_t i = 0; i < m; ++i) {
            const uint64_t x = idx ? idx[i] : i;
            if (c->dtype == SIM_C128) {
                out[2 * i] = ((const double *)c->host)[2 * x];
                out[2 * i + 1] = ((const double *)c->host)[2 * x + 1];
            } else {
                out[2 * i] = ((const float *)c->host)[2 * x];
                out[2 * i + 1] = ((const float *)c->host)[2 * x + 1];
            }
        }
        return SIM_OK;
    }
    const uint64_t kBatch = 1ull << 22;
    if (!idx) {
        if (m != len) return fail(c, SIM_E_INVAL, "idx NULL requires n == 2^N");
        if (identity && c->dtype == SIM_C128) {
            HIPCHK(c, hipMemcpy(out, c->state, len * 16, hipMemcpyDeviceToHost), "copy out");
            return SIM_OK;
        }
    } else {
        for (uint64_t i = 0; i < m; ++i)
            if (idx[i] >= len) return fail(c, SIM_E_INVAL, "amplitude index out of range");
    }
    std::vector<uint64_t> hidx;
    for (uint64_t s0 = 0; s0 < m; s0 += kBatch) {
        const uint64_t cnt = std::min(kBatch, m - s0);
        hidx.resize(cnt);
        for (uint64_t i = 0; i < cnt; ++i) hidx[i] = phys(idx ? idx[s0 + i] : s0 + i);
        HIPCHK(c, grow(c->io, cnt * (8 + 16)), "io allocation");
        uint64_t *didx = (uint64_t *)c->io.p;
        double *dout = (double *)((char *)c->io.p + cnt * 8);
        HIPCHK(c, hipMemcpyAsync(didx, hidx.data(), cnt * 8, hipMemcpyHostToDevice, c->stream), "index upload");
        hipError_t e = c->dtype == SIM_C128 ? qs::launch_gather<double>(c->state, didx, cnt, dout, c->stream)
                                            : qs::launch_gather<float>(c->state, didx, cnt, dout, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "gather");
        HIPCHK(c, hipMemcpyAsync(out + 2 * s0, dout, cnt * 16, hipMemcpyDeviceToHost, c->stream), "copy out");
        HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    }
    return SIM_OK;
}

sim_status sim_probabilities(sim_ctx *c, const uint32_t *qubits, uint32_t nq, double *out)
{
    if (!c) return SIM_E_INVAL;
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
    if (nq > 16 || (int)nq > c->n) return fail(c, SIM_E_INVAL, "at most 16 qubits");
    if (nq && !qubits) return fail(c, SIM_E_INVAL, "qubits is NULL");
    std::vector<int> ph(nq);
    for (uint32_t t = 0; t < nq; ++t) {
        if ((int)qubits[t] >= c->n) return fail(c, SIM_E_INVAL, "qubit out of range");
        for (uint32_t u = 0; u < t; ++u)
            if (qubits[u] == qubits[t]) return fail(c, SIM_E_INVAL, "duplicate qubit");
        ph[t] = c->layout[qubits[t]];
    }
    if (c->window) return offload_marginal(c, ph, out);
    std::vector<int> sorted = ph;
    std::sort(sorted.begin(), sorted.end());
    const size_t nbins = 1ull << nq;
    const size_t scr = qs::marginal_scratch_bytes(c->n, sorted.data(), (int)nq);
    HIPCHK(c, grow(c->scratch, scr + nbins * 8 + 64), "scratch allocation");
    double *dout = (double *)((char *)c->scratch.p + ((scr + 63) / 64) * 64);
    hipError_t e = c->dtype == SIM_C128
                       ? qs::launch_marginal<double>(c->state, c->n, sorted.data(), (int)nq, dout,
                                                     (double *)c->scratch.p, c->stream)
                       : qs::launch_marginal<float>(c->state, c->n, sorted.data(), (int)nq, dout,
                                                    (double *)c->scratch.p, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "marginal");
    std::vector<double> bins(nbins);
    HIPCHK(c, hipMemcpyAsync(bins.data(), dout, nbins * 8, hipMemcpyDeviceToHost, c->stream), "copy out");
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    // bin bit u <-> sorted[u]; output bit t <-> ph[t]
    std::vector<int> where(nq);
    for (uint32_t t = 0; t < nq; ++t)
        where[t] = (int)(std::find(sorted.begin(), sorted.end(), ph[t]) - sorted.begin());
    for (size_t y = 0; y < nbins; ++y) {
        size_t b = 0;
        for (uint32_t t = 0; t < nq; ++t) b |= ((y >> t) & 1ull) << where[t];
        out[y] = bins[b];
    }
    return SIM_OK;
}

sim_status sim_probabilities_noalloc(sim_ctx *c, const uint32_t *qubits, uint32_t nq, double *out)
{
    if (!c) return SIM_E_INVAL;
    if (c->window) return fail(c, SIM_E_UNSUPPORTED, "not available for a state in host memory");
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
    if (nq > 16 || (int)nq > c->n) return fail(c, SIM_E_INVAL, "at most 16 qubits");
    if (nq && !qubits) return fail(c, SIM_E_INVAL, "qubits is NULL");
    int ph[16], sorted[16], where[16];
    for (uint32_t t = 0; t < nq; ++t) {
        if ((int)qubits[t] >= c->n) return fail(c, SIM_E_INVAL, "qubit out of range");
        for (uint32_t u = 0; u < t; ++u)
            if (qubits[u] == qubits[t]) return fail(c, SIM_E_INVAL, "duplicate qubit");
        ph[t] = c->layout[qubits[t]];
        sorted[t] = ph[t];
    }
    std::sort(sorted, sorted + nq);
    for (uint32_t t = 0; t < nq; ++t) where[t] = (int)(std::find(sorted, sorted + nq, ph[t]) - sorted);
    char *base = (char *)noalloc_scratch(c->device);
    if (!base) return fail(c, SIM_E_STATE, "no scratch on this device (context created elsewhere?)");
    // scratch layout: per-segment partial bins | bins (ascending physical
    // order) | bins in the caller's qubit order
    const size_t nbins = 1ull << nq;
    const size_t part = qs::marginal_scratch_bytes(c->n, sorted, (int)nq);
    const size_t off_bins = (part + 255) / 256 * 256;
    const size_t off_out = off_bins + (nbins * 8 + 255) / 256 * 256;
    const size_t need = off_out + nbins * 8;
    if (need > kNoAllocScratchBytes)
        return fail(c, SIM_E_UNSUPPORTED, "marginal needs " + std::to_string(need) +
                                              " bytes of scratch, above the static maximum of " +
                                              std::to_string(kNoAllocScratchBytes));
    double *bins = (double *)(base + off_bins), *dout = (double *)(base + off_out);
    hipError_t e = c->dtype == SIM_C128
                       ? qs::launch_marginal<double>(c->state, c->n, sorted, (int)nq, bins, (double *)base, c->stream)
                       : qs::launch_marginal<float>(c->state, c->n, sorted, (int)nq, bins, (double *)base, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "marginal");
    HIPCHK(c, qs::launch_permute_bins(bins, dout, (int)nq, where, c->stream), "bin order");
    HIPCHK(c, hipMemcpyAsync(out, dout, nbins * 8, hipMemcpyDeviceToHost, c->stream), "copy out");
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    return SIM_OK;
}

// ---- measurement ----------------------------------------------------------

sim_status sim_measure(sim_ctx *c, uint32_t qubit, double u, uint32_t *outcome, double *prob)
{
    if (!c) return SIM_E_INVAL;
    if (c->window) return fail(c, SIM_E_UNSUPPORTED, "not available for a state in host memory");
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if ((int)qubit >= c->n) return fail(c, SIM_E_INVAL, "qubit out of range");
    if (!(u >= 0.0 && u < 1.0)) return fail(c, SIM_E_INVAL, "u must lie in [0, 1)");
    double bins[2];
    sim_status st = sim_probabilities(c, &qubit, 1, bins);
    if (st != SIM_OK) return st;
    const double total = bins[0] + bins[1];
    if (!(total > 0.0)) return fail(c, SIM_E_STATE, "state has zero norm");
    const int m = u < bins[0] / total ? 0 : 1;
    const double pm = bins[m];
    const double scale = 1.0 / std::sqrt(pm);
    hipError_t e = c->dtype == SIM_C128 ? qs::launch_collapse<double>(c->state, c->n, c->layout[qubit], m, scale,
                                                                      c->stream)
                                        : qs::launch_collapse<float>(c->state, c->n, c->layout[qubit], m, scale,
                                                                     c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "collapse");
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    if (outcome) *outcome = (uint32_t)m;
    if (prob) *prob = pm / total;
    return SIM_OK;
}

sim_status sim_sample(sim_ctx *c, const double *u, uint64_t n_shots, uint64_t *out)
{
    if (!c) return SIM_E_INVAL;
    if (c->window) return fail(c, SIM_E_UNSUPPORTED, "not available for a state in host memory");
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if (n_shots == 0) return SIM_OK;
    if (!u || !out) return fail(c, SIM_E_INVAL, "u or out is NULL");
    if (n_shots > (1ull << 31)) return fail(c, SIM_E_INVAL, "at most 2^31 shots per call");
    for (uint64_t i = 0; i < n_shots; ++i)
        if (!(u[i] >= 0.0 && u[i] < 1.0)) return fail(c, SIM_E_INVAL, "every u must lie in [0, 1)");
    const int n = c->n;
    const int K = n >= 9 ? std::min(16, n - 8) : 0;  // top logical qubits resolved by a marginal
    const int nlow = n - K;
    std::vector<uint32_t> top(K);
    for (int t = 0; t < K; ++t) top[t] = (uint32_t)(nlow + t);
    std::vector<double> bins((size_t)1 << K);
    sim_status st = sim_probabilities(c, top.data(), (uint32_t)K, bins.data());
    if (st != SIM_OK) return st;
    std::vector<double> C(bins.size());
    double acc = 0.0;
    for (size_t b = 0; b < bins.size(); ++b) C[b] = (acc += bins[b]);
    const double T = acc;
    if (!(T > 0.0)) return fail(c, SIM_E_STATE, "state has zero norm");
    size_t last_pos = 0;
    for (size_t b = 0; b < bins.size(); ++b)
        if (bins[b] > 0.0) last_pos = b;
    // block and residual per shot; the block is the first whose cumulative
    // mass exceeds u T
    std::vector<uint64_t> blk(n_shots);
    std::vector<double> res(n_shots);
    for (uint64_t i = 0; i < n_shots; ++i) {
        const double t = u[i] * T;
        size_t b = (size_t)(std::upper_bound(C.begin(), C.end(), t) - C.begin());
        if (b >= C.size()) {
            b = last_pos;
            res[i] = bins[b];  // past every block: the block's last amplitude with mass
        } else {
            res[i] = t - (b ? C[b - 1] : 0.0);
        }
        blk[i] = b;
    }
    // shots grouped by block (counting sort, stable)
    std::vector<uint32_t> count(bins.size() + 1, 0), order(n_shots);
    for (uint64_t i = 0; i < n_shots; ++i) ++count[blk[i] + 1];
    for (size_t b = 0; b < bins.size(); ++b) count[b + 1] += count[b];
    for (uint64_t i = 0; i < n_shots; ++i) order[count[blk[i]]++] = (uint32_t)i;
    std::vector<uint64_t> ids, bases;
    std::vector<uint32_t> start;
    std::vector<double> rs(n_shots);
    for (uint64_t j = 0; j < n_shots; ++j) {
        const uint64_t b = blk[order[j]];
        if (ids.empty() || ids.back() != b) {
            ids.push_back(b);
            start.push_back((uint32_t)j);
            uint64_t base = 0;
            for (int t = 0; t < K; ++t) base |= ((b >> t) & 1ull) << c->layout[nlow + t];
            bases.push_back(base);
        }
        rs[j] = res[order[j]];
    }
    start.push_back((uint32_t)n_shots);
    std::vector<uint64_t> tabs(1024, 0);
    for (uint32_t w = 0; w < 512; ++w)
        for (int q = 0; q < 9; ++q) {
            if (q < nlow && ((w >> q) & 1)) tabs[w] |= 1ull << c->layout[q];
            if (9 + q < nlow && ((w >> q) & 1)) tabs[512 + w] |= 1ull << c->layout[9 + q];
        }
    qs::SampleArgs S{};
    S.nlow = nlow;
    S.nthr = nlow >= 8 ? 256 : (1 << nlow);
    S.seg_log2 = nlow >= 8 ? nlow - 8 : 0;
    const size_t nb = ids.size();
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_tabs = 0, o_bases = o_tabs + al(1024 * 8), o_ids = o_bases + al(nb * 8),
                 o_start = o_ids + al(nb * 8), o_res = o_start + al((nb + 1) * 4), o_out = o_res + al(n_shots * 8),
                 total = o_out + al(n_shots * 8);
    HIPCHK(c, grow(c->io, total), "sample buffers");
    char *d = (char *)c->io.p;
    HIPCHK(c, hipMemcpyAsync(d + o_tabs, tabs.data(), 1024 * 8, hipMemcpyHostToDevice, c->stream), "upload");
    HIPCHK(c, hipMemcpyAsync(d + o_bases, bases.data(), nb * 8, hipMemcpyHostToDevice, c->stream), "upload");
    HIPCHK(c, hipMemcpyAsync(d + o_ids, ids.data(), nb * 8, hipMemcpyHostToDevice, c->stream), "upload");
    HIPCHK(c, hipMemcpyAsync(d + o_start, start.data(), (nb + 1) * 4, hipMemcpyHostToDevice, c->stream), "upload");
    HIPCHK(c, hipMemcpyAsync(d + o_res, rs.data(), n_shots * 8, hipMemcpyHostToDevice, c->stream), "upload");
    hipError_t e = c->dtype == SIM_C128
                       ? qs::launch_sample<double>(c->state, S, (uint32_t)nb, (const uint64_t *)(d + o_tabs),
                                                   (const uint64_t *)(d + o_bases), (const uint64_t *)(d + o_ids),
                                                   (const uint32_t *)(d + o_start), (const double *)(d + o_res),
                                                   (uint64_t *)(d + o_out), c->stream)
                       : qs::launch_sample<float>(c->state, S, (uint32_t)nb, (const uint64_t *)(d + o_tabs),
                                                  (const uint64_t *)(d + o_bases), (const uint64_t *)(d + o_ids),
                                                  (const uint32_t *)(d + o_start), (const double *)(d + o_res),
                                                  (uint64_t *)(d + o_out), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sample");
    std::vector<uint64_t> sorted_out(n_shots);
    HIPCHK(c, hipMemcpyAsync(sorted_out.data(), d + o_out, n_shots * 8, hipMemcpyDeviceToHost, c->stream),
           "copy out");
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    for (uint64_t j = 0; j < n_shots; ++j) out[order[j]] = sorted_out[j];
    return SIM_OK;
}

sim_status sim_expect_z(sim_ctx *c, const uint64_t *masks, uint32_t n_masks, double *out)
{
    if (!c) return SIM_E_INVAL;
    if (c->window) return fail(c, SIM_E_UNSUPPORTED, "not available for a state in host memory");
    if (!c->ran) return fail(c, SIM_E_STATE, "sim_run has not completed");
    if (n_masks == 0) return SIM_OK;
    if (!masks || !out) return fail(c, SIM_E_INVAL, "masks or out is NULL");
    const uint64_t all = c->n >= 64 ? ~0ull : ((1ull << c->n) - 1);
    for (uint32_t i = 0; i < n_masks; ++i)
        if (masks[i] & ~all) return fail(c, SIM_E_INVAL, "mask names a qubit out of range");
    const size_t scr = qs::expect_z_scratch_bytes();
    HIPCHK(c, grow(c->scratch, scr + 64 * 8 + 256), "scratch allocation");
    double *dout = (double *)((char *)c->scratch.p + ((scr + 255) / 256) * 256);
    for (uint32_t i0 = 0; i0 < n_masks; i0 += qs::kZMasksPerLaunch) {
        qs::ZArgs Z{};
        Z.nm = (int32_t)std::min<uint32_t>(qs::kZMasksPerLaunch, n_masks - i0);
        for (int k = 0; k < Z.nm; ++k) {
            uint64_t pm = 0;
            for (int q = 0; q < c->n; ++q)
                if ((masks[i0 + k] >> q) & 1) pm |= 1ull << c->layout[q];
            Z.m[k] = pm;
        }
        hipError_t e = c->dtype == SIM_C128
                           ? qs::launch_expect_z<double>(c->state, c->n, Z, dout, (double *)c->scratch.p, c->stream)
                           : qs::launch_expect_z<float>(c->state, c->n, Z, dout, (double *)c->scratch.p, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "expectation");
        HIPCHK(c, hipMemcpyAsync(out + i0, dout, Z.nm * 8, hipMemcpyDeviceToHost, c->stream), "copy out");
        HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    }
    return SIM_OK;
}

sim_status sim_expect_diagonal(sim_ctx *c, const uint32_t *qubits, uint32_t nq, const double *f, double *out)
{
    if (!c) return SIM_E_INVAL;
    if (!f || !out) return fail(c, SIM_E_INVAL, "f or out is NULL");
    std::vector<double> bins((size_t)1 << std::min<uint32_t>(nq, 16));
    sim_status st = sim_probabilities(c, qubits, nq, bins.data());
    if (st != SIM_OK) return st;
    double acc = 0.0;
    for (size_t y = 0; y < bins.size(); ++y) acc += bins[y] * f[y];
    *out = acc;
    return SIM_OK;
}

sim_status sim_inner(sim_ctx *a, sim_ctx *b, double *out)
{
    if (!a || !b) return SIM_E_INVAL;
    if (!out) return fail(a, SIM_E_INVAL, "out is NULL");
    if (a->n != b->n) return fail(a, SIM_E_INVAL, "qubit counts differ");
    if (!a->ran || !b->ran) return fail(a, SIM_E_STATE, "both contexts must have run");
    if (a->window || b->window) return fail(a, SIM_E_UNSUPPORTED, "not available for a state in host memory");
    HIPCHK(a, hipStreamSynchronize(b->stream), "synchronize");
    if (a->layout != b->layout) {
        // element i of a (physical) is logical x = pa^-1(i); b holds it at pb(x)
        std::vector<int> inv_a(a->n), map(a->n);
        for (int q = 0; q < a->n; ++q) inv_a[a->layout[q]] = q;
        for (int p = 0; p < a->n; ++p) map[p] = b->layout[inv_a[p]];
        const size_t scr = qs::inner_scratch_bytes(a->n);
        HIPCHK(a, grow(a->scratch, scr + 64), "scratch allocation");
        double *dout = (double *)((char *)a->scratch.p + scr);
        hipError_t e;
        double *sp = (double *)a->scratch.p;
        if (a->dtype == SIM_C128 && b->dtype == SIM_C128)
            e = qs::launch_inner_perm<double, double>(a->state, b->state, a->n, map.data(), dout, sp, a->stream);
        else if (a->dtype == SIM_C128)
            e = qs::launch_inner_perm<double, float>(a->state, b->state, a->n, map.data(), dout, sp, a->stream);
        else if (b->dtype == SIM_C128)
            e = qs::launch_inner_perm<float, double>(a->state, b->state, a->n, map.data(), dout, sp, a->stream);
        else
            e = qs::launch_inner_perm<float, float>(a->state, b->state, a->n, map.data(), dout, sp, a->stream);
        if (e != hipSuccess) return hip_fail(a, e, "inner product");
        HIPCHK(a, hipMemcpyAsync(out, dout, 16, hipMemcpyDeviceToHost, a->stream), "copy out");
        HIPCHK(a, hipStreamSynchronize(a->stream), "synchronize");
        return SIM_OK;
    }
    const size_t scr = qs::inner_scratch_bytes(a->n);
    HIPCHK(a, grow(a->scratch, scr + 64), "scratch allocation");
    double *dout = (double *)((char *)a->scratch.p + scr);
    hipError_t e;
    if (a->dtype == SIM_C128 && b->dtype == SIM_C128)
        e = qs::launch_inner<double, double>(a->state, b->state, a->n, dout, (double *)a->scratch.p, a->stream);
    else if (a->dtype == SIM_C128)
        e = qs::launch_inner<double, float>(a->state, b->state, a->n, dout, (double *)a->scratch.p, a->stream);
    else if (b->dtype == SIM_C128)
        e = qs::launch_inner<float, double>(a->state, b->state, a->n, dout, (double *)a->scratch.p, a->stream);
    else
        e = qs::launch_inner<float, float>(a->state, b->state, a->n, dout, (double *)a->scratch.p, a->stream);
    if (e != hipSuccess) return hip_fail(a, e, "inner product");
    HIPCHK(a, hipMemcpyAsync(out, dout, 16, hipMemcpyDeviceToHost, a->stream), "copy out");
    HIPCHK(a, hipStreamSynchronize(a->stream), "synchronize");
    return SIM_OK;
}

sim_status sim_stats(const sim_ctx *c, sim_run_stats *out)
{
    if (!c || !out) return SIM_E_INVAL;
    sim_ctx *m = const_cast<sim_ctx *>(c);
    if (m->timing_pending && hipEventQuery(m->ev1) == hipSuccess) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, m->ev0, m->ev1) == hipSuccess) m->stats.run_ms = ms;
        m->timing_pending = false;
    }
    *out = c->stats;
    return SIM_OK;
}

sim_status sim_set_profiling(sim_ctx *c, uint32_t enable)
{
    if (!c) return SIM_E_INVAL;
    c->profiling = enable != 0;
    return SIM_OK;
}

sim_status sim_op_timings(sim_ctx *c, sim_op_timing *out, uint64_t cap, uint64_t *n)
{
    if (!c || !n) return SIM_E_INVAL;
    *n = c->prep.size();
    if (!c->profiled) return fail(c, SIM_E_STATE, "no profiled run");
    HIPCHK(c, hipStreamSynchronize(c->stream), "synchronize");
    for (size_t i = 0; i < c->prep.size() && i < cap; ++i) {
        out[i].kind = c->plan.ops[i].kind;
        out[i].buffer = (uint32_t)c->plan.ops[i].buffer;
        out[i].flops = c->plan.ops[i].flops;
        out[i].bytes = c->plan.ops[i].bytes;
        // a tensor product formed by the next stage's loads: no bytes of its
        // own, and that stage reads the two factors instead of the state
        if (c->prep[i].fused) out[i].bytes = 0;
        if (c->prep[i].kron) out[i].bytes -= (double)(c->amp_bytes() << c->prep[i].nb);
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->op_ev[2 * i], c->op_ev[2 * i + 1]), "event time");
        out[i].ms = ms;
    }
    return SIM_OK;
}

const char *sim_last_error(const sim_ctx *c) { return c ? c->err.c_str() : kNullCtx; }

sim_status sim_device_bytes(const sim_ctx *c, uint64_t *out)
{
    if (!c || !out) return SIM_E_INVAL;
    uint64_t total = 0;
    for (const DevBuf *b : {&c->tables, &c->prog, &c->gdesc, &c->items, &c->scratch, &c->io}) total += b->bytes;
    for (const DevBuf &b : c->subbufs) total += b.bytes;
    *out = total;
    return SIM_OK;
}

sim_status sim_destroy(sim_ctx *c)
{
    if (!c) return SIM_E_INVAL;
    hipStreamSynchronize(c->stream);
    if (c->h2d) hipStreamSynchronize(c->h2d);
    if (c->d2h) hipStreamSynchronize(c->d2h);
    for (int b = 0; b < 2; ++b)
        for (hipEvent_t ev : {c->ev_in[b], c->ev_done[b], c->ev_out[b]})
            if (ev) hipEventDestroy(ev);
    if (c->ev_pass) hipEventDestroy(c->ev_pass);
    if (c->h2d) hipStreamDestroy(c->h2d);
    if (c->d2h) hipStreamDestroy(c->d2h);
    for (DevBuf *b : {&c->tables, &c->prog, &c->gdesc, &c->items, &c->scratch, &c->io})
        if (b->p) hipFree(b->p);
    for (DevBuf &b : c->subbufs)
        if (b.p) hipFree(b.p);
    for (hipEvent_t ev : c->op_ev) hipEventDestroy(ev);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    delete c;
    return SIM_OK;
}

sim_status sim_run_batch(sim_ctx *const *ctxs, uint32_t n_ctx, void *stream)
{
    if (!ctxs && n_ctx) return SIM_E_INVAL;
    if (n_ctx == 0) return SIM_OK;
    for (uint32_t i = 0; i < n_ctx; ++i) {
        sim_ctx *c = ctxs[i];
        if (!c) return SIM_E_INVAL;
        if (!c->loaded) return fail(c, SIM_E_STATE, "no circuit loaded");
        if (c->window) return fail(c, SIM_E_UNSUPPORTED, "host-memory offload contexts cannot be batched");
        if (c->dtype != ctxs[0]->dtype) return fail(c, SIM_E_INVAL, "batched contexts must share the dtype");
        for (uint32_t j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(c, SIM_E_INVAL, "a context appears twice in the batch");
    }
    hipStream_t s = stream ? (hipStream_t)stream : ctxs[0]->stream;
    std::vector<sim_ctx *> small, staged;
    for (uint32_t i = 0; i < n_ctx; ++i) (ctxs[i]->small_whole ? small : staged).push_back(ctxs[i]);
    for (size_t i0 = 0; i0 < small.size(); i0 += qs::kSmallBatchMax) {
        const uint32_t cnt = (uint32_t)std::min<size_t>(qs::kSmallBatchMax, small.size() - i0);
        qs::SmallPtrs P{};
        uint32_t maxn = 0;
        for (uint32_t u = 0; u < cnt; ++u) {
            sim_ctx *c = small[i0 + u];
            P.item[u] = (const qs::SmallItem *)c->items.p + c->small_whole_item;
            maxn = std::max<uint32_t>(maxn, (uint32_t)c->n);
        }
        hipError_t e = ctxs[0]->dtype == SIM_C128 ? qs::launch_small_ptrs<double>(P, cnt, maxn, s)
                                                  : qs::launch_small_ptrs<float>(P, cnt, maxn, s);
        if (e != hipSuccess) return hip_fail(ctxs[0], e, "batched launch");
    }
    if (!staged.empty()) {
        const sim_status st = ctxs[0]->dtype == SIM_C128
                                  ? execute_staged_batch<double>(staged.data(), (uint32_t)staged.size(), s)
                                  : execute_staged_batch<float>(staged.data(), (uint32_t)staged.size(), s);
        if (st != SIM_OK) return st;
    }
    for (sim_ctx *c : small) {
        c->layout.resize(c->n);
        for (int q = 0; q < c->n; ++q) c->layout[q] = q;
    }
    for (sim_ctx *c : staged) c->layout = c->plan.layout;
    for (uint32_t i = 0; i < n_ctx; ++i) {
        ctxs[i]->ran = true;
        ctxs[i]->timing_pending = false;
        ctxs[i]->profiled = false;
    }
    return SIM_OK;
}

// ---- host-only planning ----------------------------------------------------

sim_status sim_plan_build(uint32_t n_qubits, sim_dtype dtype, const sim_options *opts, const sim_gate *gates,
                          uint64_t n_gates, sim_plan **out)
{
    if (!out) return SIM_E_INVAL;
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 36 || (dtype != SIM_C128 && dtype != SIM_C64)) return SIM_E_INVAL;
    if (!gates && n_gates) return SIM_E_INVAL;
    std::vector<qs::Operator> ops;
    std::string err;
    if (!convert_gates(gates, n_gates, (int)n_qubits, ops, &err)) return SIM_E_INVAL;
    sim_plan *p = new (std::nothrow) sim_plan();
    if (!p) return SIM_E_NOMEM;
    p->plan.n = (int)n_qubits;
    p->plan.dtype = dtype;
    p->plan.opt = qs::resolve_options(opts, dtype, (int)n_qubits);
    try {
        qs::build_plan(p->plan, ops);
    } catch (const std::exception &) {
        delete p;
        return SIM_E_UNSUPPORTED;
    }
    *out = p;
    return SIM_OK;
}

uint64_t sim_plan_num_ops(const sim_plan *p) { return p ? p->plan.ops.size() : 0; }

namespace {
// Physical bit of qubit q of op i: ops inside a host-memory offload pass
// name window bits.
struct WindowMap {
    int lo = 0, n = 0, nq = 0;
    bool on = false;
    int operator()(int q) const { return on ? qs::window_to_physical(q, lo, n, nq) : q; }
};
WindowMap window_map(const qs::Plan &P, uint64_t i)
{
    WindowMap m;
    for (uint64_t j = 0; j < P.ops.size() && j < i; ++j)
        if (P.ops[j].kind == SIM_OP_WINDOW && j + (uint64_t)P.ops[j].pass_ops >= i) {
            m.on = true;
            m.lo = P.ops[j].outer_lo;
            m.n = P.ops[j].outer_n;
            m.nq = P.n;
        }
    return m;
}
}  // namespace

sim_status sim_plan_get_op(const sim_plan *p, uint64_t i, sim_plan_op *op, double *payload)
{
    if (!p || !op || i >= p->plan.ops.size()) return SIM_E_INVAL;
    const qs::PlanOp &o = p->plan.ops[i];
    std::memset(op, 0, sizeof(*op));
    op->kind = o.kind;
    op->buffer = (uint32_t)o.buffer;
    op->buffer_qubits = (uint32_t)o.buffer_qubits;
    op->src_lo = (uint32_t)o.src_lo;
    op->src_hi = (uint32_t)o.src_hi;
    const WindowMap wm = window_map(p->plan, i);
    if (wm.on) op->buffer_qubits = (uint32_t)p->plan.n;  // reported on the full state
    if (o.kind == SIM_OP_WINDOW) {
        op->nq = (uint32_t)o.pass_ops;
        op->qubits[0] = (uint32_t)o.outer_lo;
        op->qubits[1] = (uint32_t)o.outer_n;
        op->qubits[2] = o.init_window ? 1u : 0u;
    } else if (o.kind == SIM_OP_DENSE || o.kind == SIM_OP_DIAG) {
        op->nq = (uint32_t)o.op.q.size();
        for (size_t t = 0; t < o.op.q.size() && t < 32; ++t) op->qubits[t] = (uint32_t)wm(o.op.q[t]);
        op->payload_len = o.op.m.size();
        if (payload)
            for (size_t t = 0; t < o.op.m.size(); ++t) {
                payload[2 * t] = o.op.m[t].real();
                payload[2 * t + 1] = o.op.m[t].imag();
            }
    } else if (o.kind == SIM_OP_STAGE) {
        op->nq = (uint32_t)o.gates.size();
        op->local_qubits = (uint32_t)o.local.size();
        for (size_t t = 0; t < o.local.size() && t < 32; ++t) op->qubits[t] = (uint32_t)wm(o.local[t]);
        op->n_phases = (uint32_t)o.phases.size();
    } else if (o.kind == SIM_OP_PERM) {
        op->nq = (uint32_t)o.perm.size();
        for (size_t t = 0; t < o.perm.size() && t < 32; ++t) op->qubits[t] = (uint32_t)o.perm[t];
    }
    return SIM_OK;
}

sim_status sim_plan_stage_gate(const sim_plan *p, uint64_t op_index, uint64_t i, sim_plan_gate *g, double *payload)
{
    if (!p || !g || op_index >= p->plan.ops.size()) return SIM_E_INVAL;
    const qs::PlanOp &o = p->plan.ops[op_index];
    if (o.kind != SIM_OP_STAGE || i >= o.gates.size()) return SIM_E_INVAL;
    const qs::Operator &x = o.gates[i];
    const WindowMap wm = window_map(p->plan, op_index);
    std::memset(g, 0, sizeof(*g));
    g->diagonal = x.diag ? 1 : 0;
    g->nq = (uint32_t)x.q.size();
    for (size_t t = 0; t < x.q.size() && t < 16; ++t) g->qubits[t] = (uint32_t)wm(x.q[t]);
    g->payload_len = x.m.size();
    if (payload)
        for (size_t t = 0; t < x.m.size(); ++t) {
            payload[2 * t] = x.m[t].real();
            payload[2 * t + 1] = x.m[t].imag();
        }
    return SIM_OK;
}

sim_status sim_plan_stage_kernel_op(const sim_plan *p, uint64_t op_index, uint64_t i, sim_plan_gate *g,
                                    double *payload)
{
    if (!p || !g || op_index >= p->plan.ops.size()) return SIM_E_INVAL;
    const qs::PlanOp &o = p->plan.ops[op_index];
    if (o.kind != SIM_OP_STAGE) return SIM_E_INVAL;
    const WindowMap wm = window_map(p->plan, op_index);
    for (const qs::Phase &ph : o.phases) {
        if (i >= ph.ops.size()) {
            i -= ph.ops.size();
            continue;
        }
        const qs::KOp &k = ph.ops[i];
        std::memset(g, 0, sizeof(*g));
        if (k.type == qs::KOp::QUAD) {
            // (code, angle) pairs: code -1 the constant, q * 64 + q the
            // linear term of qubit q, q * 64 + p (q < p) the pair term
            std::vector<std::pair<double, double>> terms{{-1.0, k.qc}};
            const int nb = o.buffer_qubits;
            for (int q = 0; q < nb; ++q) {
                if (k.qa[q] != 0.0) terms.push_back({(double)(wm(q) * 64 + wm(q)), k.qa[q]});
                for (int p2 = q + 1; p2 < nb; ++p2) {
                    const double v = k.qb[(size_t)q * nb + p2];
                    const int a = std::min(wm(q), wm(p2)), bq = std::max(wm(q), wm(p2));
                    if (v != 0.0) terms.push_back({(double)(a * 64 + bq), v});
                }
            }
            g->diagonal = 2;
            g->payload_len = terms.size();
            if (payload)
                for (size_t t = 0; t < terms.size(); ++t) {
                    payload[2 * t] = terms[t].first;
                    payload[2 * t + 1] = terms[t].second;
                }
            return SIM_OK;
        }
        if (k.type == qs::KOp::DIAG) {
            g->diagonal = 1;
            g->nq = (uint32_t)k.dq.size();
            for (int q : k.dq)
                for (int b : ph.reg)
                    if (o.local[b] == q) g->n_register++;
            for (size_t t = 0; t < k.dq.size() && t < 16; ++t) g->qubits[t] = (uint32_t)wm(k.dq[t]);
            g->payload_len = k.table.size();
            if (payload)
                for (size_t t = 0; t < k.table.size(); ++t) {
                    payload[2 * t] = k.table[t].real();
                    payload[2 * t + 1] = k.table[t].imag();
                }
            return SIM_OK;
        }
        std::vector<int> q;
        for (int b = 0; b < (int)ph.reg.size(); ++b)
            if ((k.reg_mask >> b) & 1) q.push_back(o.local[ph.reg[b]]);
        const int kr = (int)q.size(), ks = (int)k.sel.size();
        for (int t : k.sel) q.push_back(t);
        g->diagonal = 0;
        g->nq = (uint32_t)q.size();
        g->n_register = (uint32_t)kr;
        for (size_t t = 0; t < q.size() && t < 16; ++t) g->qubits[t] = (uint32_t)wm(q[t]);
        const uint64_t D = 1ull << (kr + ks), dr = 1ull << kr;
        g->payload_len = D * D;
        if (payload) {
            for (uint64_t t = 0; t < 2 * D * D; ++t) payload[t] = 0.0;
            for (uint64_t sel = 0; sel < (1ull << ks); ++sel)
                for (uint64_t r = 0; r < dr; ++r)
                    for (uint64_t c = 0; c < dr; ++c) {
                        const cplx v = k.table[sel * dr * dr + r * dr + c];
                        const uint64_t R = r | (sel << kr), Cc = c | (sel << kr);
                        payload[2 * (R * D + Cc)] = v.real();
                        payload[2 * (R * D + Cc) + 1] = v.imag();
                    }
        }
        return SIM_OK;
    }
    return SIM_E_INVAL;
}

sim_status sim_plan_layout(const sim_plan *p, uint32_t *phys)
{
    if (!p || !phys) return SIM_E_INVAL;
    for (size_t q = 0; q < p->plan.layout.size(); ++q) phys[q] = (uint32_t)p->plan.layout[q];
    return SIM_OK;
}

sim_status sim_plan_stats(const sim_plan *p, sim_run_stats *out)
{
    if (!p || !out) return SIM_E_INVAL;
    std::memset(out, 0, sizeof(*out));
    fill_stats(p->plan, 0, out);
    return SIM_OK;
}

sim_status sim_plan_counters(const sim_plan *p, uint64_t *dd_visits, uint64_t *booster_gates, uint64_t *booster_groups)
{
    if (!p) return SIM_E_INVAL;
    if (dd_visits) *dd_visits = p->plan.stats.dd_visits;
    if (booster_gates) *booster_gates = p->plan.stats.booster_gates;
    if (booster_groups) *booster_groups = p->plan.stats.booster_groups;
    return SIM_OK;
}

sim_status sim_plan_destroy(sim_plan *p)
{
    if (!p) return SIM_E_INVAL;
    delete p;
    return SIM_OK;
}

}  // extern "C"
