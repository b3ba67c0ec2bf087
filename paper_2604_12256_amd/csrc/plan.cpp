// Host optimiser: builds the execution plan of a circuit.
//
// Pass order follows the swarm optimisation of Sec. 4.2 (Alg. 4) on one
// device (no rank level):
//   merge booster (Sec. 4.4, Alg. 6-7) -> diagonal detector (Sec. 4.5, Alg. 8)
//   -> gate block search with limit C (cache-blocked stages, Alg. 2)
//   -> gate block search with limit F and fusion inside every block.
// Every pass keeps the state the circuit defines (Alg. 1) up to rounding.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <exception>
#include <stdexcept>
#include <thread>

#include "ir.hpp"

namespace qs {

namespace {

int popc(uint64_t x) { return __builtin_popcountll(x); }

// Cost model of one stage-kernel operator: device microseconds per 2^30
// amplitudes, measured on MI355X as the increment per operator inside
// compute-bound stages (chunk 2^12 complex128 / 2^13 complex64).  Dense
// operators on three or more register bits run as the whole register tile
// (4 bits complex128, 5 bits complex64).
double op_cost(bool diag, int dense_qubits, bool c64)
{
    if (diag) return c64 ? 145.0 : 265.0;
    if (dense_qubits <= 1) return c64 ? 247.0 : 286.0;
    if (dense_qubits == 2) return c64 ? 478.0 : 652.0;
    return c64 ? 9510.0 : 7570.0;
}

// Diagonal table operators, by shape: table width w (qubits), k of them
// register bits (2^k entries per thread), and whether a selector is a lane
// bit (every lane loads its own entries) or all selectors are wave-uniform
// (scalar loads).  Microseconds per 2^30 amplitudes, measured on MI355X as
// the increment per operator in stages of 20 and 60 such operators.
double diag_cost(int w, int k, bool lane, bool c64)
{
    static const double u128[4] = {172.0, 292.0, 354.0, 360.0}, l128[4] = {265.0, 374.0, 387.0, 444.0};
    static const double u64[4] = {147.0, 162.0, 211.0, 226.0}, l64[4] = {155.0, 222.0, 225.0, 258.0};
    static const double r128[6] = {0.0, 25.0, 45.0, 220.0, 420.0, 420.0}, r64[6] = {0.0, 5.0, 10.0, 15.0, 20.0, 25.0};
    const int sel = w - k;
    const int b = sel <= 2 ? 0 : sel <= 6 ? 1 : sel <= 10 ? 2 : 3;
    const double base = c64 ? (lane ? l64[b] : u64[b]) : (lane ? l128[b] : u128[b]);
    return base + (c64 ? r64[std::min(k, 5)] : r128[std::min(k, 5)]);
}

// A quadratic-phase operator (the product of many diagonals on one or two
// qubits, applied as one phase form, in FP64): microseconds per 2^30
// amplitudes.
constexpr double kQuadCostC64 = 600.0;
double quad_cost(bool c64) { return c64 ? kQuadCostC64 : 1200.0; }
// The stage kernel variant with quadratic-phase operators runs the stage's
// other work this much slower; the fixed part of a stage pass (loads,
// stores, transposes) in the same units as the operator costs.
constexpr double kQuadVariantPenalty = 0.06, kStageFixedUs = 2500.0;

// Device seconds of one stage-kernel operator on `amps` amplitudes, in a
// phase whose register bits sit at the physical qubits `reg` and whose lane
// bits at `lane` (bit masks).
double kop_seconds(const KOp &k, int reg_bits, double amps, bool c64, uint64_t reg, uint64_t lane)
{
    const double scale = amps / 1073741824.0 * 1e-6;
    if (k.type == KOp::QUAD) return scale * quad_cost(c64);
    if (k.type == KOp::DIAG) {
        int kr = 0;
        bool ln = false;
        for (int q : k.dq) {
            kr += (int)((reg >> q) & 1);
            ln |= ((lane >> q) & 1) != 0;
        }
        return scale * diag_cost((int)k.dq.size(), kr, ln, c64);
    }
    const int kr = __builtin_popcount(k.reg_mask);
    return scale * op_cost(false, kr >= 3 ? reg_bits : kr, c64);
}

// Floating-point operations per amplitude: a dense k-qubit operator does 2^k
// complex multiply-adds (8 flops each), a diagonal one complex multiply (6).
double op_flops(bool diag, int dense_qubits) { return diag ? 6.0 : 8.0 * double(1 << dense_qubits); }

// A quadratic phase: the running product that forms each amplitude's factor
// and its application, one complex multiply each.
constexpr double kQuadFlops = 12.0;

}  // namespace

Options resolve_options(const sim_options *o, sim_dtype dtype, int n)
{
    Options r;
    if (o) {
        r.opt = o->opt;
        r.C = o->C;
        r.F = o->F ? o->F : 5;
        r.D = o->D ? o->D : 10;
        r.B = o->B ? o->B : 4;
        r.force_fuse_k = o->force_fuse_k;
    }
    r.reg_bits = dtype == SIM_C128 ? 4 : 5;
    // Every stage keeps the lowest physical qubits local so that a wave's
    // loads and stores come in contiguous runs of whole 128-byte cache lines:
    // 8 complex128 or 16 complex64 amplitudes.  Fewer fixed qubits leave more
    // room in the local set (on the 30-qubit layered circuit 15 passes
    // instead of 21 with six fixed qubits, measured 9% faster on MI355X);
    // runs of half a line measured slower.
    r.fixed_low = (o && o->L) ? (int)std::min<uint32_t>(o->L, 6) : (dtype == SIM_C128 ? 3 : 4);
    // Default chunk: 2^12 complex128 / 2^13 complex64 amplitudes (64 KiB), so two
    // workgroups share a CU and one's HBM load/store overlaps the other's compute.
    if (r.C == 0) r.C = dtype == SIM_C128 ? 12 : 13;
    if (r.F > 6) r.F = 6;
    if (r.D > 20) r.D = 20;
    if (r.D < 1) r.D = 1;
    if (r.B < 1) r.B = 1;
    if (o && o->host_state) {
        // host-memory offload: windows of the state pass through the device;
        // the merge booster (sub-states) and qubit reordering (permutation
        // passes) are not used in this mode
        r.window_qubits = offload_window_qubits(o->dev_state_bytes, dtype == SIM_C128 ? 16 : 8, n);
        r.opt &= ~(uint32_t)(SIM_OPT_BOOST | SIM_OPT_REMAP);
    }
    return r;
}

int offload_window_qubits(uint64_t dev_bytes, uint64_t amp_bytes, int nq)
{
    int W = 0;
    while (W + 1 <= nq - 1 && (2 * amp_bytes << (W + 1)) <= dev_bytes) ++W;
    return (2 * amp_bytes << W) <= dev_bytes ? W : 0;
}

// ---------------------------------------------------------------------------
// Merge booster, divide component (Alg. 6).  The division is a binary
// halving of the qubit count: a part larger than div_size splits into its
// floor half and its ceiling half, in that order, and the parts that need no
// split are the leaves, listed left to right.  An explicit work list (next
// part at the back) yields them in that order.
void divider(int n, int div_size, std::vector<int> &que)
{
    std::vector<int> todo{n};
    while (!todo.empty()) {
        const int part = todo.back();
        todo.pop_back();
        if (part <= div_size || part < 2) {
            que.push_back(part);
            continue;
        }
        todo.push_back(part - part / 2);  // ceiling half: visited second
        todo.push_back(part / 2);         // floor half: visited first
    }
}

// ---------------------------------------------------------------------------
// Diagonal detector (Alg. 8).  Readings where the listing is silent or
// inconsistent:
//  * a run holding a single diagonal is emitted unchanged (the listing only
//    emits runs of two or more);
//  * a non-diagonal gate is deferred to the unprocessed list when it touches
//    a qubit of an earlier diagonal of the run OR a qubit of an already
//    deferred gate, so two non-commuting gates are never reordered;
//  * deferring marks every qubit of the deferred gate in the stop table;
//  * a diagonal stops the run when it touches a marked qubit or when the union
//    of the run's qubits would exceed D (the practical upper bound of
//    Sec. 4.5); the scan then restarts at that gate.
// The fused table is the product of the members' diagonals on the ascending
// union of their qubits.
std::vector<Operator> diagonal_detector(int n, int D, const std::vector<Operator> &in, uint64_t *visits)
{
    (void)n;
    std::vector<Operator> res;
    res.reserve(in.size());
    uint64_t placed = 0;
    size_t it = 0;
    while (it < in.size()) {
        const Operator &g = in[it];
        if (!g.diag) {
            res.push_back(g);
            ++placed;
            ++it;
            continue;
        }
        std::vector<size_t> diag_list{it};
        std::vector<size_t> u_list;
        uint64_t stop = 0, dep = g.mask(), uni = g.mask();
        size_t f = it + 1;
        for (; f < in.size(); ++f) {
            const Operator &h = in[f];
            const uint64_t hm = h.mask();
            if (!h.diag) {
                if (hm & (dep | stop)) {
                    stop |= hm;
                    u_list.push_back(f);
                } else {
                    res.push_back(h);
                    ++placed;
                }
            } else {
                if ((hm & stop) || popc(uni | hm) > D) break;
                dep |= hm;
                uni |= hm;
                diag_list.push_back(f);
            }
        }
        if (diag_list.size() == 1) {
            res.push_back(g);
        } else {
            std::vector<int> qs;
            for (int q = 0; q < 64; ++q)
                if ((uni >> q) & 1) qs.push_back(q);
            std::vector<const Operator *> members;
            for (size_t idx : diag_list) members.push_back(&in[idx]);
            res.push_back(diag_product(qs, members));
        }
        placed += diag_list.size();
        for (size_t idx : u_list) res.push_back(in[idx]);
        placed += u_list.size();
        it = f;
    }
    if (visits) *visits = placed;
    return res;
}

namespace {

// Qubits a gate needs in registers (and hence local) inside a stage: those on
// which it is not block diagonal.  A dense gate selecting its block by more
// than two qubits, or a 3+ qubit dense gate selecting by any, keeps all its
// qubits (the stage kernel takes at most two block-selecting bits, and
// lane-bit selection only for 1- and 2-bit operators).
uint64_t tile_need(const Operator &g)
{
    uint64_t need = need_mask(g);
    if (!g.diag && (popc(g.mask() & ~need) > 2 || (popc(need) > 2 && (g.mask() & ~need)))) need = g.mask();
    return need;
}

// ---------------------------------------------------------------------------
// Plan assembly helpers.

struct Builder {
    Plan &plan;
    const Options &o;

    double amp_bytes() const { return plan.dtype == SIM_C128 ? 16.0 : 8.0; }

    void add_full_pass_op(int buffer, int nb, const Operator &g)
    {
        PlanOp op;
        op.kind = g.diag ? SIM_OP_DIAG : SIM_OP_DENSE;
        op.buffer = buffer;
        op.buffer_qubits = nb;
        op.op = g;
        const double amps = std::ldexp(1.0, nb);
        op.flops = op_flops(g.diag, g.k()) * amps;
        op.bytes = 2.0 * amps * amp_bytes();
        plan.ops.push_back(std::move(op));
    }

    // Fusion inside one phase: greedy merging of consecutive gates into one
    // operator while the fused operator costs no more FMA per amplitude than
    // its members applied one by one (cost-based fusion with the register
    // tile as the size limit).  A fused dense operator acts on 1, 2 or all r
    // register bits (the kernel's code paths) and may select its block by at
    // most two non-register qubits; selection by a lane bit is only allowed
    // for 1- and 2-bit operators (their matrices are then loaded per lane).
    void fuse_phase(Phase &ph, const std::vector<const Operator *> &gates, const std::vector<int> &reg_phys,
                    uint64_t lane_phys, uint64_t local_phys, double *flops_per_amp, bool reg_diags_to_z)
    {
        const int r = (int)reg_phys.size();
        auto regbit = [&](int phys) {
            for (int b = 0; b < r; ++b)
                if (reg_phys[b] == phys) return b;
            return -1;
        };
        const int kTmaxLane = 2, kTmaxUniform = 4;
        const bool fuse = (o.opt & SIM_OPT_FUSE) != 0;  // without it every gate is its own kernel op
        const uint32_t full = (1u << r) - 1;
        auto kernel_mask = [&](uint32_t S) { return popc(S) >= 3 ? full : S; };
        const bool c64 = plan.dtype == SIM_C64;
        auto dense_cost = [&](uint32_t S) { return op_cost(false, popc(kernel_mask(S)), c64); };
        auto lane_sel = [&](const std::vector<int> &T) {
            for (int t : T)
                if ((lane_phys >> t) & 1) return true;
            return false;
        };
        struct Block {
            bool open = false;
            uint32_t S = 0;
            std::vector<int> T;
            Operator acc;
            double indiv = 0;
        } F;
        auto qlist = [&](uint32_t S, const std::vector<int> &T) {
            std::vector<int> l;
            for (int b = 0; b < r; ++b)
                if ((S >> b) & 1) l.push_back(reg_phys[b]);
            for (int t : T) l.push_back(t);
            return l;
        };
        auto push_diag = [&](const std::vector<int> &q, const std::vector<cplx> &table) {
            KOp k;
            k.type = KOp::DIAG;
            k.dq = q;
            k.table = table;
            *flops_per_amp += op_flops(true, 0);
            ph.ops.push_back(std::move(k));
        };
        auto emit = [&](Block &B) {
            if (!B.open) return;
            if (B.acc.diag) {
                push_diag(B.acc.q, B.acc.m);
            } else {
                KOp k;
                k.type = KOp::DENSE;
                const uint32_t km = kernel_mask(B.S);
                if (km != B.S) B.acc = embed(B.acc, qlist(km, B.T));
                k.reg_mask = km;
                k.sel = B.T;
                const int ks = popc(km);
                std::vector<int> fixed_pos;
                for (size_t u = 0; u < B.T.size(); ++u) fixed_pos.push_back(ks + (int)u);
                for (uint64_t sel = 0; sel < (1ull << B.T.size()); ++sel) {
                    std::vector<cplx> blk = sub_block(B.acc, fixed_pos, sel);
                    k.table.insert(k.table.end(), blk.begin(), blk.end());
                }
                *flops_per_amp += op_flops(false, ks);
                ph.ops.push_back(std::move(k));
            }
            B = Block();
        };
        // Several blocks stay open at once, one per disjoint set of register
        // qubits; they may share selector qubits only, so open blocks commute
        // and a gate can join the block that owns its register qubits even
        // when other blocks were opened after it.  A gate bridging two blocks
        // closes them.
        std::vector<Block> open;
        // Diagonal gates commute with each other, and with every open block
        // whose content is diagonal on their qubits.  With fusion on, they are
        // collected into one diagonal Z per phase (register qubits S, selector
        // qubits T), which keeps that property for every open block: a gate
        // joining Z first closes the blocks owning its register qubits, and a
        // dense gate on a register qubit of Z emits Z first.  Z is emitted when
        // its selectors would exceed kZsel (the kernel keeps up to 12 selector
        // sources in registers) or its table 2^kZmax entries, and at the end of
        // the phase.  One table lookup and one complex multiply per amplitude
        // then serve every diagonal of the phase.
        Block Z;
        struct ZMember {
            const Operator *g;
            uint32_t S;           // register bits
            std::vector<int> T;   // selector qubits
            uint64_t tmask;       // selector qubits as a mask
        };
        std::vector<ZMember> zmem;
        // a chunk reads the slice of a table its chunk bits select: at most
        // kZloc chunk-local table qubits keep that slice (16 KiB) in L1
        const int kZsel = 12, kZmax = 14, kZloc = c64 ? 11 : 10;
        auto member_sets = [&](const std::vector<ZMember> &ms, uint32_t *S, std::vector<int> *T) {
            *S = 0;
            T->clear();
            for (const ZMember &m : ms) {
                *S |= m.S;
                for (int x : m.T)
                    if (std::find(T->begin(), T->end(), x) == T->end()) T->push_back(x);
            }
        };
        // Packs commuting diagonal members into as few tables as the caps
        // allow (at most kZsel selectors, 2^kZmax entries, kZloc chunk-local
        // qubits): a table starts from the widest unplaced member and grows
        // by the member that adds the fewest new qubits, so gates inside the
        // table's qubits join first.  Members commute, so order is free.
        auto emit_members = [&](std::vector<ZMember> &ms) {
            const size_t nm = ms.size();
            std::vector<char> used(nm, 0);
            size_t left = nm;
            // members all on one or two qubits: one quadratic-phase operator
            // when it costs less than the tables they pack into
            bool quad = fuse && (o.opt & SIM_OPT_QUAD) && o.window_qubits == 0 && nm > 1;
            for (size_t i = 0; i < nm && quad; ++i) quad = ms[i].g->diag && ms[i].g->k() <= 2;
            std::vector<KOp> packed;
            double packed_us = 0;
            auto fits = [&](uint32_t S, uint64_t T) {
                return popc(T) <= kZsel && popc(S) + popc(T) <= kZmax &&
                       popc(S) + popc(T & local_phys) <= kZloc;
            };
            while (left) {
                size_t seed = nm;
                for (size_t i = 0; i < nm; ++i)
                    if (!used[i] && (seed == nm || popc(ms[i].S) + popc(ms[i].tmask) >
                                                       popc(ms[seed].S) + popc(ms[seed].tmask)))
                        seed = i;
                uint32_t S = ms[seed].S;
                uint64_t T = ms[seed].tmask;
                std::vector<size_t> grp{seed};
                used[seed] = 1;
                --left;
                while (left) {
                    size_t best = nm;
                    int best_add = 1 << 30;
                    for (size_t i = 0; i < nm && best_add > 0; ++i) {
                        if (used[i]) continue;
                        const int add = popc(ms[i].S & ~S) + popc(ms[i].tmask & ~T);
                        if (add < best_add && fits(S | ms[i].S, T | ms[i].tmask)) {
                            best = i;
                            best_add = add;
                        }
                    }
                    if (best == nm) break;
                    S |= ms[best].S;
                    T |= ms[best].tmask;
                    used[best] = 1;
                    --left;
                    grp.push_back(best);
                }
                std::sort(grp.begin(), grp.end());
                std::vector<int> tl;
                for (int q = 0; q < 64; ++q)
                    if ((T >> q) & 1) tl.push_back(q);
                KOp k;
                k.type = KOp::DIAG;
                k.dq = qlist(S, tl);
                for (size_t i : grp) k.members.push_back(*ms[i].g);
                packed_us += diag_cost((int)k.dq.size(), popc(S), (T & lane_phys) != 0, c64);
                packed.push_back(std::move(k));
            }
            if (quad && quad_cost(c64) < packed_us) {
                KOp k;
                k.type = KOp::QUAD;
                for (size_t i = 0; i < nm; ++i) k.members.push_back(*ms[i].g);
                k.alt = std::move(packed);
                k.alt_us = packed_us;
                *flops_per_amp += kQuadFlops;
                ph.ops.push_back(std::move(k));
            } else {
                for (KOp &k : packed) {
                    *flops_per_amp += op_flops(true, 0);
                    ph.ops.push_back(std::move(k));
                }
            }
            ms.clear();
        };
        auto emit_z = [&]() {
            emit_members(zmem);
            Z = Block();
        };
        auto z_add = [&](const Operator &g, uint32_t gS, const std::vector<int> &gT) {
            uint64_t tm = 0;
            for (int x : gT) {
                tm |= 1ull << x;
                if (std::find(Z.T.begin(), Z.T.end(), x) == Z.T.end()) Z.T.push_back(x);
            }
            Z.open = true;
            Z.S |= gS;
            zmem.push_back({&g, gS, gT, tm});
        };
        // the members of Z on any of the register bits `bits` leave Z (a dense
        // gate on those bits follows them; the rest of Z commutes with it)
        auto z_take = [&](uint32_t bits) {
            std::vector<ZMember> taken, kept;
            for (ZMember &m : zmem) (m.S & bits ? taken : kept).push_back(std::move(m));
            zmem.swap(kept);
            member_sets(zmem, &Z.S, &Z.T);
            Z.open = !zmem.empty();
            return taken;
        };
        auto close_all_owning = [&](uint32_t S, const std::vector<int> &T) {
            for (size_t i = 0; i < open.size();) {
                bool hit = (open[i].S & S) != 0;
                // a selector of the new gate that is a register qubit of a block
                // (never, selectors are non-register) or a register qubit of the
                // gate that is a selector of a block: the block uses it as a
                // control, which does not commute with the gate
                for (int t : open[i].T)
                    for (int b = 0; b < r; ++b)
                        if (((S >> b) & 1) && reg_phys[b] == t) hit = true;
                (void)T;
                if (hit) {
                    emit(open[i]);
                    open.erase(open.begin() + i);
                } else {
                    ++i;
                }
            }
        };
        for (const Operator *gp : gates) {
            const Operator &g = *gp;
            uint32_t gS = 0;
            std::vector<int> gT;
            for (int x : g.q) {
                int b = regbit(x);
                if (b >= 0) gS |= 1u << b;
                else gT.push_back(x);
            }
            if (g.diag && g.k() > 3) {  // a wide diagonal (diagonal detector output)
                close_all_owning(gS, gT);
                if (fuse) z_add(g, gS, gT);
                else push_diag(g.q, g.m);  // its own table
                continue;
            }
            // diagonals of Z on g's register bits precede g
            std::vector<ZMember> P;
            if (fuse && !g.diag && (gS & Z.S)) P = z_take(gS);
            const double gcost = g.diag ? op_cost(true, 0, c64) : dense_cost(gS);
            // blocks owning a register qubit of g
            std::vector<size_t> own;
            for (size_t i = 0; i < open.size(); ++i)
                if (open[i].S & gS) own.push_back(i);
            if (fuse && own.size() == 1) {
                Block &B = open[own[0]];
                const uint32_t S2 = B.S | gS;
                std::vector<int> T2 = B.T;
                for (int x : gT)
                    if (std::find(T2.begin(), T2.end(), x) == T2.end()) T2.push_back(x);
                const bool diag2 = B.acc.diag && g.diag;
                const double fused = diag2 ? op_cost(true, 0, c64) : dense_cost(S2);
                const bool sel_ok = diag2 ? (int)T2.size() <= kTmaxUniform
                                          : (lane_sel(T2) ? ((int)T2.size() <= kTmaxLane && popc(kernel_mask(S2)) <= 2)
                                                          : (int)T2.size() <= kTmaxUniform);
                // a register qubit g adds to B must not be another block's selector
                bool clash = false;
                for (size_t i = 0; i < open.size(); ++i) {
                    if (i == own[0]) continue;
                    for (int t : open[i].T)
                        for (int b = 0; b < r; ++b)
                            if (((gS >> b) & 1) && reg_phys[b] == t) clash = true;
                }
                if (!clash && sel_ok && fused <= B.indiv + gcost + 1e-9) {
                    if (!P.empty()) {  // the whole table goes first, packed (it commutes with every open block)
                        for (ZMember &m : P) zmem.push_back(std::move(m));
                        P.clear();
                        emit_z();
                    }
                    std::vector<int> l2 = qlist(S2, T2);
                    if (l2 != B.acc.q) B.acc = embed(B.acc, l2);
                    apply_left(B.acc, g);
                    B.S = S2;
                    B.T = T2;
                    B.indiv += gcost;
                    continue;
                }
            }
            // g starts a block of its own: close every block it does not commute with
            close_all_owning(gS, gT);
            if (fuse && g.diag && (gS == 0 || reg_diags_to_z)) {
                z_add(g, gS, gT);
                continue;
            }
            const bool alone_ok = g.diag ? (int)gT.size() <= kTmaxUniform
                                         : (lane_sel(gT) ? ((int)gT.size() <= kTmaxLane && popc(kernel_mask(gS)) <= 2)
                                                         : (int)gT.size() <= kTmaxUniform);
            if (!alone_ok) {
                if (g.diag) {
                    push_diag(g.q, g.m);
                    continue;
                }
                throw std::runtime_error("fuse_phase: dense gate needs more register bits");
            }
            Block nb;
            nb.open = true;
            nb.S = gS;
            nb.T = gT;
            nb.indiv = gcost;
            if (!P.empty()) {
                // fold the diagonals g follows into g's block when that costs no
                // more than a table op of their own
                uint32_t pS;
                std::vector<int> pT;
                member_sets(P, &pS, &pT);
                const uint32_t S2 = gS | pS;
                std::vector<int> T2 = gT;
                for (int x : pT)
                    if (std::find(T2.begin(), T2.end(), x) == T2.end()) T2.push_back(x);
                const bool ok = (lane_sel(T2) ? ((int)T2.size() <= kTmaxLane && popc(kernel_mask(S2)) <= 2)
                                              : (int)T2.size() <= kTmaxUniform) &&
                                dense_cost(S2) <= gcost + op_cost(true, 0, c64) + 1e-9;
                if (ok) {
                    std::vector<const Operator *> pm;
                    for (const ZMember &m : P) pm.push_back(m.g);
                    const std::vector<int> l2 = qlist(S2, T2);
                    nb.acc = embed(diag_product(l2, pm), l2);
                    apply_left(nb.acc, g);
                    nb.S = S2;
                    nb.T = T2;
                    P.clear();
                } else {  // the whole table goes first, packed
                    for (ZMember &m : P) zmem.push_back(std::move(m));
                    P.clear();
                    emit_z();
                    nb.acc = embed(g, qlist(gS, gT));
                }
            } else {
                nb.acc = embed(g, qlist(gS, gT));
            }
            if (!fuse || gS == 0) {  // no fusion, or a phase on non-register bits only: emit now
                emit(nb);
                continue;
            }
            open.push_back(std::move(nb));
        }
        for (Block &B : open) emit(B);
        emit_z();
    }

    // LDS bank order of a phase's lane bits.  The stage kernel's transposes
    // write and read 16-byte (complex128) or 8-byte (complex64) slots at a
    // swizzled local index whose low slot bits take local bit l to bit
    // l mod M (M = 4 for complex128, 5 for complex64).  The lanes the LDS
    // serves together then hit distinct banks when lane bits 0..M-1 sit on
    // local bits of residues 0..M-1 in that order (this holds whether the
    // LDS serves 8 or 16 lanes of a 16-byte access per cycle).  Reorders
    // the lane bits (the first six thread-id bits) toward that pattern; a
    // wave bit no gate of the phase uses may replace a lane bit, which never
    // makes a wave-uniform selector lane-varying.
    void order_lanes_for_lds(std::vector<int> &t, const std::vector<int> &uses) const
    {
        const int M = plan.dtype == SIM_C128 ? 4 : 5;  // slot bits of the swizzle: 16-byte or 8-byte slots
        const int nl = 6;
        if ((int)t.size() < nl) return;
        std::vector<int> L(t.begin(), t.begin() + nl), W(t.begin() + nl, t.end());
        std::vector<int> head(M, -1);
        std::vector<bool> placed(nl, false);
        for (int want = 0; want < M; ++want)
            for (int i = 0; i < nl; ++i)
                if (!placed[i] && L[i] % M == want) {
                    head[want] = i;
                    placed[i] = true;
                    break;
                }
        for (int want = 0; want < M; ++want) {
            if (head[want] >= 0) continue;
            int w = -1, x = -1;
            for (int j = 0; j < (int)W.size() && w < 0; ++j)
                if (W[j] % M == want && uses[W[j]] == 0) w = j;
            for (int i = 0; i < nl; ++i)  // the most-used unplaced lane bit leaves
                if (!placed[i] && (x < 0 || uses[L[i]] > uses[L[x]])) x = i;
            if (w < 0 || x < 0) continue;
            std::swap(L[x], W[w]);
            head[want] = x;
            placed[x] = true;
        }
        std::vector<int> out;
        for (int want = 0; want < M; ++want) {
            int i = head[want];
            if (i < 0)  // residue unavailable: any unplaced lane bit holds the slot
                for (int j = 0; j < nl; ++j)
                    if (!placed[j]) {
                        i = j;
                        placed[j] = true;
                        break;
                    }
            out.push_back(L[i]);
        }
        for (int i = 0; i < nl; ++i)
            if (!placed[i]) out.push_back(L[i]);
        out.insert(out.end(), W.begin(), W.end());
        t.swap(out);
    }

    // Register phases of one stage: gate block search with limit r on the
    // qubits each gate needs in registers, over the stage's gate list (the
    // same search as the stage partition, one level down the memory
    // hierarchy).  At most kMaxPhases phases; the gates beyond are returned.
    static constexpr int kMaxPhases = 96;

    std::vector<int> make_phases(PlanOp &st, const std::vector<Operator> &all, const std::vector<int> &idx,
                                 double *flops)
    {
        const int r = o.reg_bits, C = (int)st.local.size();
        int local_of[64];
        for (int q = 0; q < 64; ++q) local_of[q] = -1;
        for (int i = 0; i < C; ++i) local_of[st.local[i]] = i;
        std::vector<int> rem = idx;
        std::vector<int> prev;
        for (int b = 0; b < r; ++b) prev.push_back(C - r + b);  // load mapping
        double fpa = 0;
        while (!rem.empty() && (int)st.phases.size() < kMaxPhases) {
            uint64_t R = 0, blocked = 0;  // R over local bit indices
            std::vector<int> take, left;
            for (int gi : rem) {
                const Operator &g = all[gi];
                const uint64_t qs = g.mask();
                if (qs & blocked) {
                    blocked |= qs;
                    left.push_back(gi);
                    continue;
                }
                uint64_t nd = 0;
                const uint64_t need = tile_need(g);
                for (int q = 0; q < 64; ++q)
                    if ((need >> q) & 1) {
                        if (local_of[q] < 0) throw std::runtime_error("make_phases: qubit not local");
                        nd |= 1ull << local_of[q];
                    }
                if (popc(R | nd) <= r) {
                    R |= nd;
                    take.push_back(gi);
                } else {
                    blocked |= qs;
                    left.push_back(gi);
                }
            }
            if (take.empty()) throw std::runtime_error("make_phases: no progress");
            for (int b : prev)  // keep previous register bits where free
                if (popc(R) < r) R |= 1ull << b;
            for (int i = C - 1; i >= 0 && popc(R) < r; --i) R |= 1ull << i;
            Phase ph;
            for (int i = 0; i < C; ++i)
                if ((R >> i) & 1) ph.reg.push_back(i);
            std::vector<int> reg_phys;
            for (int i : ph.reg) reg_phys.push_back(st.local[i]);
            // thread-id bits: the non-register local bits least used by this
            // phase's gates become lane bits, so that the bits selecting a
            // fused block or indexing a diagonal table are wave-uniform
            // whenever possible (scalar loads instead of per-lane loads)
            std::vector<int> uses(C, 0);
            for (int gi : take)
                for (int q : all[gi].q)
                    if (local_of[q] >= 0 && !((R >> local_of[q]) & 1)) uses[local_of[q]]++;
            for (int i = 0; i < C; ++i)
                if (!((R >> i) & 1)) ph.tmap.push_back(i);
            std::stable_sort(ph.tmap.begin(), ph.tmap.end(), [&](int a, int b) { return uses[a] < uses[b]; });
            order_lanes_for_lds(ph.tmap, uses);
            uint64_t lane_phys = 0;
            for (int i = 0; i < 6 && i < (int)ph.tmap.size(); ++i) lane_phys |= 1ull << st.local[ph.tmap[i]];
            std::vector<const Operator *> tg;
            for (int gi : take) {
                tg.push_back(&all[gi]);
                st.gates.push_back(all[gi]);
            }
            // narrow diagonals on register qubits either open blocks that a
            // later dense gate can absorb, or join the phase's diagonal table
            // (better when many share a register qubit): both are built, and
            // the table form is kept when it is cheaper by the cost model
            // without adding operators (per-operator overheads the marginal
            // costs miss made more, lighter operators slower on the
            // 30-qubit layered circuit)
            const double amps = std::ldexp(1.0, st.buffer_qubits);
            const bool c64 = plan.dtype == SIM_C64;
            Phase alt = ph;
            double f0 = 0, f1 = 0, t0 = 0, t1 = 0;
            uint64_t local_m = 0;
            for (int q : st.local) local_m |= 1ull << q;
            fuse_phase(ph, tg, reg_phys, lane_phys, local_m, &f0, false);
            uint64_t reg_m = 0;
            for (int q : reg_phys) reg_m |= 1ull << q;
            for (const KOp &k : ph.ops) t0 += kop_seconds(k, r, amps, c64, reg_m, lane_phys);
            if (o.opt & SIM_OPT_FUSE) {
                fuse_phase(alt, tg, reg_phys, lane_phys, local_m, &f1, true);
                for (const KOp &k : alt.ops) t1 += kop_seconds(k, r, amps, c64, reg_m, lane_phys);
                if (t1 < t0 && alt.ops.size() <= ph.ops.size()) {
                    ph = std::move(alt);
                    t0 = t1;
                    f0 = f1;
                }
            }
            fpa += f0;
            st.est_s += t0;
            st.phases.push_back(std::move(ph));
            prev = st.phases.back().reg;
            rem.swap(left);
        }
        // Quadratic-phase operators run on a kernel variant whose other work
        // is slower (its register allocation; measured on MI355X): a stage
        // keeps them only when they save more than that costs over the stage,
        // else each goes back to the tables it replaced.
        {
            const double scale = std::ldexp(1.0, st.buffer_qubits) / 1073741824.0 * 1e-6;
            double save = 0, quad_us = 0;
            int nquad = 0;
            for (const Phase &ph : st.phases)
                for (const KOp &k : ph.ops)
                    if (k.type == KOp::QUAD) {
                        save += k.alt_us - quad_cost(plan.dtype == SIM_C64);
                        quad_us += quad_cost(plan.dtype == SIM_C64);
                        ++nquad;
                    }
            const double other_us = st.est_s / scale - quad_us + kStageFixedUs;
            if (nquad && save < kQuadVariantPenalty * other_us) {
                for (Phase &ph : st.phases) {
                    std::vector<KOp> ops;
                    for (KOp &k : ph.ops) {
                        if (k.type != KOp::QUAD) {
                            ops.push_back(std::move(k));
                            continue;
                        }
                        fpa += op_flops(true, 0) * (double)k.alt.size() - kQuadFlops;
                        for (KOp &t : k.alt) ops.push_back(std::move(t));
                    }
                    ph.ops.swap(ops);
                }
                st.est_s += scale * save;
            } else {
                // a phase of quadratic-phase operators alone on the load
                // mapping's register bits takes the load mapping's thread
                // order too (the operator reads any order), so the chunk
                // needs no transpose into or out of it
                const uint64_t neutral = ((1ull << r) - 1) << (C - r);
                for (Phase &ph : st.phases) {
                    bool only = !ph.ops.empty();
                    uint64_t R = 0;
                    for (KOp &k : ph.ops) {
                        k.alt.clear();
                        only &= k.type == KOp::QUAD;
                    }
                    for (int i : ph.reg) R |= 1ull << i;
                    if (only && R == neutral)
                        for (int i = 0; i < C - r; ++i) ph.tmap[i] = i;
                }
            }
        }
        *flops += fpa;
        return rem;
    }

    // Gate block search with limit C over the gates of one buffer (Alg. 4,
    // GBSA(N, C)): greedy DAG frontier; a gate joins the open stage when none
    // of its qubits is blocked and its locally-needed qubits fit; otherwise all
    // its qubits become blocked.  Diagonal gates and block-selecting (control)
    // qubits need not be local: inside a chunk the other bits are constants.
    // One greedy stage (gate block search with limit C) over the remaining
    // gates: the local set starts with the always-local low bits; a gate
    // joins when none of its qubits is blocked and the qubits it needs fit.
    struct Masks {
        std::vector<uint64_t> qs, nd;   // per gate: all qubits, qubits needed locally
    };

    static uint64_t permute_mask(uint64_t m, const std::vector<int> &sigma)
    {
        uint64_t out = 0;
        for (size_t q = 0; q < sigma.size(); ++q)
            if ((m >> q) & 1) out |= 1ull << sigma[q];
        return out;
    }

    void greedy_stage(const Masks &M, const std::vector<int> &rem, int C, int low, int r, uint64_t *Lout,
                      std::vector<int> *take, std::vector<int> *left, uint64_t avail = ~0ull) const
    {
        uint64_t L = (1ull << low) - 1;
        uint64_t blocked = 0;
        for (int gi : rem) {
            const uint64_t qs = M.qs[gi];
            const uint64_t nd = M.nd[gi];
            if ((qs & blocked) || popc(nd) > r || (nd & ~avail)) {
                blocked |= qs;
                if (left) left->push_back(gi);
                continue;
            }
            if (popc(L | nd) <= C) {
                L |= nd;
                if (take) take->push_back(gi);
            } else {
                blocked |= qs;
                if (left) left->push_back(gi);
            }
        }
        *Lout = L;
    }

    // The greedy frontier with a fixed local set L: a gate is taken when none
    // of its qubits is blocked, the qubits it needs are in L and fit the
    // register tile; otherwise all its qubits become blocked.  Counts the
    // gates taken (stopping once every qubit in `live` is blocked) or collects
    // them; `wanted` gathers the global qubits whose absence turned a gate
    // away that was not blocked otherwise.
    size_t frontier(const Masks &M, const std::vector<int> &rem, uint64_t L, int r, uint64_t live,
                    std::vector<int> *take, std::vector<int> *left, uint64_t *wanted = nullptr) const
    {
        uint64_t blocked = 0;
        size_t n = 0;
        for (size_t i = 0; i < rem.size(); ++i) {
            const int gi = rem[i];
            const uint64_t qs = M.qs[gi], nd = M.nd[gi];
            if ((qs & blocked) || (nd & ~L) || popc(nd) > r) {
                if (wanted && !(qs & blocked) && popc(nd) <= r) *wanted |= nd & ~L;
                blocked |= qs;
                if (left) left->push_back(gi);
                if (!left && (blocked & live) == live) break;
                continue;
            }
            ++n;
            if (take) take->push_back(gi);
        }
        return n;
    }

    // Local search on a stage's local set (the gate block search chooses the
    // local qubits in gate order; the choice decides how far the stage gets):
    // swap one local qubit above the always-local low bits for a global qubit
    // that a turned-away gate wanted, whenever the frontier then takes more
    // gates, until no swap helps (at most kMaxEvals frontier evaluations).
    // Frontier count on a contiguous copy of the remaining gates' masks.
    static size_t frontier_count(const std::vector<uint64_t> &qs, const std::vector<uint64_t> &nd, uint64_t L,
                                 int r, uint64_t live, uint64_t *wanted)
    {
        uint64_t blocked = 0;
        size_t n = 0;
        for (size_t i = 0; i < qs.size(); ++i) {
            if ((qs[i] & blocked) || (nd[i] & ~L) || popc(nd[i]) > r) {
                if (!(qs[i] & blocked) && popc(nd[i]) <= r) *wanted |= nd[i] & ~L;
                blocked |= qs[i];
                if ((blocked & live) == live) break;
                continue;
            }
            ++n;
        }
        return n;
    }

    uint64_t refine_local(const Masks &M, const std::vector<int> &rem, uint64_t L, int low, int r, int nb) const
    {
        constexpr int kMaxEvals = 300;
        std::vector<uint64_t> qs(rem.size()), nd(rem.size());
        uint64_t live = 0;
        for (size_t i = 0; i < rem.size(); ++i) {
            qs[i] = M.qs[rem[i]];
            nd[i] = M.nd[rem[i]];
            live |= qs[i];
        }
        uint64_t wanted = 0;
        size_t best = frontier_count(qs, nd, L, r, live, &wanted);
        int evals = 1;
        bool improved = true;
        while (improved && evals < kMaxEvals) {
            improved = false;
            for (int a = low; a < nb && !improved && evals < kMaxEvals; ++a) {
                if (!((L >> a) & 1)) continue;
                for (int b = low; b < nb && evals < kMaxEvals; ++b) {
                    if (((L >> b) & 1) || !((wanted >> b) & 1)) continue;
                    const uint64_t L2 = (L & ~(1ull << a)) | (1ull << b);
                    uint64_t w2 = 0;
                    const size_t c = frontier_count(qs, nd, L2, r, live, &w2);
                    ++evals;
                    if (c > best) {
                        best = c;
                        L = L2;
                        wanted = w2;
                        improved = true;
                        break;
                    }
                }
            }
        }
        return L;
    }

    // Gates consumed by the next `horizon` greedy stages.
    size_t lookahead(const Masks &M, std::vector<int> rem, int C, int low, int r, int horizon) const
    {
        size_t consumed = 0;
        for (int h = 0; h < horizon && !rem.empty(); ++h) {
            if (popc(M.nd[rem.front()]) > r) {
                rem.erase(rem.begin());
                ++consumed;
                continue;
            }
            uint64_t L;
            std::vector<int> take, left;
            greedy_stage(M, rem, C, low, r, &L, &take, &left);
            consumed += take.size();
            rem.swap(left);
        }
        return consumed;
    }

    static void swap_qubits(Operator &g, const std::vector<int> &sigma)
    {
        for (int &q : g.q) q = sigma[q];
    }

    // Qubit reordering (Sec. 2.3): the low physical bits are local in every
    // stage (coalescing), so qubits that the coming gates need often should
    // sit there.  Candidate: swap the least-needed low bits with the
    // most-needed high bits of a window of upcoming gates; accepted when the
    // lookahead consumes enough more gates in the same number of stages to
    // repay the permutation pass.  Free when the state is still |0...0>.
    bool maybe_remap(std::vector<Operator> &pg, Masks &M, const std::vector<int> &rem, int nb, int C, int low,
                     int r)
    {
        const int kWindow = 400, kHorizon = 6;
        std::vector<double> freq(nb, 0.0);
        int cnt = 0;
        for (int gi : rem) {
            if (cnt++ >= kWindow) break;
            const uint64_t nd = M.nd[gi];
            for (int q = 0; q < nb; ++q)
                if ((nd >> q) & 1) freq[q] += 1.0;
        }
        std::vector<int> lows, highs;
        // the in-place permutation pass exchanges bits below 6 with bits at 6
        // or above (its tile holds the low six bits and the partners)
        for (int q = 0; q < low; ++q) lows.push_back(q);
        for (int q = std::max(low, 6); q < nb; ++q) highs.push_back(q);
        std::stable_sort(lows.begin(), lows.end(), [&](int a, int b) { return freq[a] < freq[b]; });
        std::stable_sort(highs.begin(), highs.end(), [&](int a, int b) { return freq[a] > freq[b]; });
        std::vector<int> sigma(nb);
        for (int q = 0; q < nb; ++q) sigma[q] = q;
        int pairs = 0;
        for (size_t i = 0; i < lows.size() && i < highs.size(); ++i) {
            if (freq[highs[i]] <= freq[lows[i]] + 1.0) break;
            sigma[lows[i]] = highs[i];
            sigma[highs[i]] = lows[i];
            ++pairs;
        }
        if (!pairs) return false;
        const size_t c0 = lookahead(M, rem, C, low, r, kHorizon);
        Masks T = M;
        for (int gi : rem) {
            T.qs[gi] = permute_mask(M.qs[gi], sigma);
            T.nd[gi] = permute_mask(M.nd[gi], sigma);
        }
        const size_t c1 = lookahead(T, rem, C, low, r, kHorizon);
        bool fresh = false;
        for (auto it = plan.ops.rbegin(); it != plan.ops.rend(); ++it)
            if (it->buffer == 0) {
                fresh = it->kind == SIM_OP_INIT;
                break;
            }
        // stages saved over the horizon ~ kHorizon * (1 - c0 / c1); the in-place
        // permutation pass costs about three stage passes on MI355X (measured:
        // 18.9 ms against 6.8 ms for a plain 16 GiB copy pass)
        const double saved = c1 > 0 ? kHorizon * (1.0 - double(c0) / double(c1)) : 0.0;
        if (!(c1 > c0 && (fresh || saved >= 3.0))) return false;
        M.qs.swap(T.qs);
        M.nd.swap(T.nd);
        for (int gi : rem) swap_qubits(pg[gi], sigma);
        std::vector<int> &lay = plan.layout;  // logical -> physical
        for (int &p : lay) p = sigma[p];
        if (!fresh) {
            PlanOp op;
            op.kind = SIM_OP_PERM;
            op.buffer = 0;
            op.buffer_qubits = nb;
            op.perm = sigma;  // source bit p -> destination bit sigma[p] (a product of swaps)
            const double amps = std::ldexp(1.0, nb);
            op.bytes = 2.0 * amps * amp_bytes();
            plan.stats.full_passes += 1;
            plan.stats.bytes += op.bytes;
            plan.stats.n_perm += 1;
            plan.ops.push_back(std::move(op));
        }
        return true;
    }

    // Cache-blocked stages over the buffer.  In window mode (host-memory
    // offload) the gates may also name bits at and above nb (the outer bits
    // of the pass, fixed per window): they can only select blocks or index
    // diagonals, so a gate that needs one locally, or a full-pass gate that
    // touches one, ends the pass; the gates not taken are returned (indices
    // into `gates`, in circuit order).
    std::vector<int> stages(int buffer, int nb, const std::vector<Operator> &gates, bool window = false)
    {
        const int C = std::min<int>((int)o.C, nb), r = o.reg_bits;
        const int low = std::min(o.fixed_low, C);
        // gates on physical qubits of the buffer (the full state may be remapped)
        std::vector<Operator> pg = gates;
        if (buffer == 0)
            for (Operator &g : pg)
                for (int &q : g.q) q = plan.layout[q];
        std::vector<int> rem(gates.size());
        for (size_t i = 0; i < gates.size(); ++i) rem[i] = (int)i;
        Masks M;
        M.qs.resize(pg.size());
        M.nd.resize(pg.size());
        for (size_t i = 0; i < pg.size(); ++i) {
            M.qs[i] = pg[i].mask();
            M.nd[i] = tile_need(pg[i]);
        }
        const double nb_amps = std::ldexp(1.0, nb);
        const bool remap = buffer == 0 && (o.opt & SIM_OPT_REMAP) && nb > C && !window;
        const uint64_t avail = nb >= 64 ? ~0ull : ((1ull << nb) - 1);
        while (!rem.empty()) {
            if (remap) maybe_remap(pg, M, rem, nb, C, low, r);
            const Operator &first = pg[rem.front()];
            if (popc(M.nd[rem.front()]) > r) {  // beyond the register tile: one full pass
                if (M.qs[rem.front()] & ~avail) break;  // on an outer bit: not in this pass
                add_full_pass_op(buffer, nb, first);
                account_full_pass(buffer, nb, first);
                rem.erase(rem.begin());
                continue;
            }
            uint64_t L;
            std::vector<int> take, left;
            greedy_stage(M, rem, C, low, r, &L, &take, &left, avail);
            for (int q = 0; q < nb && popc(L) < C; ++q) L |= 1ull << q;
            if (nb > C) {
                L = refine_local(M, rem, L, low, r, nb);
                take.clear();
                left.clear();
                frontier(M, rem, L, r, ~0ull, &take, &left);
            }
            if (take.empty()) break;  // window mode: every frontier gate needs an outer bit
            PlanOp st;
            st.kind = SIM_OP_STAGE;
            st.buffer = buffer;
            st.buffer_qubits = nb;
            for (int q = 0; q < nb; ++q)
                if ((L >> q) & 1) st.local.push_back(q);
            double fpa = 0;
            std::vector<int> over = make_phases(st, pg, take, &fpa);
            st.flops = fpa * nb_amps;
            st.bytes = 2.0 * nb_amps * amp_bytes();
            plan.stats.flops += st.flops;
            if (buffer == 0) {
                plan.stats.full_passes += 1;
                plan.stats.bytes += 2.0 * nb_amps * amp_bytes();
                plan.stats.n_stages += 1;
            } else {
                plan.stats.n_subruns += 1;
            }
            plan.ops.push_back(std::move(st));
            if (!over.empty()) {  // phase cap hit: the rest goes back, in circuit order
                left.insert(left.end(), over.begin(), over.end());
                std::sort(left.begin(), left.end());
            }
            rem.swap(left);
        }
        if (!rem.empty() && !window) throw std::runtime_error("stage partition made no progress");
        return rem;
    }

    // Host-memory offload (the state lives in host memory; the device holds
    // two windows of 2^W amplitudes).  A pass fixes S = N - W outer qubits, a
    // contiguous range of bit positions, so that every window is a 2D block
    // of the state (rows of 2^lo amplitudes); inside the pass the outer
    // qubits are constants of the window, read only by selectors and
    // diagonal tables.  The range is chosen so that the gate frontier runs
    // furthest before a gate needs one of its qubits locally; the pass's
    // stages are the cache-blocked stages of the window, and it ends when
    // every frontier gate needs an outer qubit.  The first pass creates
    // |0...0> in the windows instead of reading them.
    void offload(const std::vector<Operator> &in)
    {
        const int N = plan.n, W = o.window_qubits, S = N - W;
        const int lo_min = std::min(7, W);
        std::vector<Operator> gates = in;
        if (o.opt & SIM_OPT_DIAG) {
            uint64_t v = 0;
            gates = diagonal_detector(N, (int)o.D, gates, &v);
            plan.stats.dd_visits += v;
        }
        std::vector<uint64_t> qs(gates.size()), nd(gates.size());
        for (size_t i = 0; i < gates.size(); ++i) {
            qs[i] = gates[i].mask();
            nd[i] = tile_need(gates[i]);
        }
        std::vector<int> rem(gates.size());
        for (size_t i = 0; i < gates.size(); ++i) rem[i] = (int)i;
        const double amp = amp_bytes(), scale = std::ldexp(1.0, S);
        const uint64_t all = (N >= 64) ? ~0ull : ((1ull << N) - 1);
        bool first = true;
        while (first || !rem.empty()) {
            // outer range: the frontier takes the most gates before it stops;
            // ranges at bit 7 or above first (rows of at least 128
            // amplitudes), then any range above the always-local low bits
            int best_lo = N - S;
            size_t best = 0;
            for (const int floor_lo : {lo_min, std::min(lo_min, o.fixed_low)}) {
                for (int lo = N - S; lo >= floor_lo; --lo) {
                    const uint64_t R = ((1ull << S) - 1) << lo;
                    uint64_t blocked = 0;
                    size_t n = 0;
                    for (size_t i = 0; i < rem.size() && i < 4000; ++i) {
                        const int g = rem[i];
                        if ((qs[g] & blocked) || (nd[g] & R) || (popc(nd[g]) > o.reg_bits && (qs[g] & R))) {
                            blocked |= qs[g];
                            if ((blocked & all) == all) break;
                            continue;
                        }
                        ++n;
                    }
                    if (n > best) {
                        best = n;
                        best_lo = lo;
                    }
                }
                if (best > 0 || rem.empty()) break;
            }
            if (!rem.empty() && best == 0)
                throw std::runtime_error("offload: every outer range holds a qubit the next gates need");
            std::vector<Operator> wg;
            wg.reserve(rem.size());
            for (int g : rem) {
                Operator w = gates[g];
                for (int &q : w.q) q = physical_to_window(q, best_lo, S, N);
                wg.push_back(std::move(w));
            }
            PlanOp win;
            win.kind = SIM_OP_WINDOW;
            win.buffer = 0;
            win.buffer_qubits = N;
            win.outer_lo = best_lo;
            win.outer_n = S;
            win.init_window = first;
            const size_t mark = plan.ops.size();
            plan.ops.push_back(std::move(win));
            const PlanStats before = plan.stats;
            const std::vector<int> left = stages(0, W, wg, true);
            // a window op is one pass over the whole state on the device
            plan.stats.bytes = before.bytes + (plan.stats.bytes - before.bytes) * scale;
            plan.stats.flops = before.flops + (plan.stats.flops - before.flops) * scale;
            for (size_t i = mark + 1; i < plan.ops.size(); ++i) {
                plan.ops[i].bytes *= scale;
                plan.ops[i].flops *= scale;
            }
            plan.ops[mark].pass_ops = (int)(plan.ops.size() - mark - 1);
            if (!rem.empty() && left.size() == rem.size()) throw std::runtime_error("offload: pass made no progress");
            plan.stats.offload_passes += 1;
            // every window is written back; all but the first pass read them first
            plan.stats.pcie_bytes += (first ? 1.0 : 2.0) * std::ldexp(1.0, N) * amp;
            std::vector<int> next;
            next.reserve(left.size());
            for (int i : left) next.push_back(rem[i]);
            rem.swap(next);
            first = false;
        }
    }

    void account_full_pass(int buffer, int nb, const Operator &g)
    {
        const double amps = std::ldexp(1.0, nb);
        if (buffer != 0) {
            plan.stats.n_subruns += 1;
            return;
        }
        plan.stats.full_passes += 1;
        plan.stats.bytes += 2.0 * amps * amp_bytes();
        plan.stats.flops += op_flops(g.diag, g.k()) * amps;
        if (g.diag) plan.stats.n_diag += 1;
        else plan.stats.n_dense += 1;
    }

    // Gate block search with limit F and fusion (Alg. 4, GBSA(N, F, GB, 1)):
    // blocks of at most F qubits; a block is fused into one operator when that
    // costs no more than its members (or always, with force_fuse_k).
    void fused_passes(int buffer, int nb, const std::vector<Operator> &gates)
    {
        const int F = o.force_fuse_k ? (int)o.force_fuse_k : (int)o.F;
        std::vector<const Operator *> rem;
        for (const Operator &g : gates) rem.push_back(&g);
        while (!rem.empty()) {
            uint64_t U = 0, blocked = 0;
            std::vector<const Operator *> take, left;
            for (const Operator *g : rem) {
                const uint64_t qs = g->mask();
                if (qs & blocked) {
                    blocked |= qs;
                    left.push_back(g);
                    continue;
                }
                if (popc(U | qs) <= F || take.empty()) {
                    U |= qs;
                    take.push_back(g);
                } else {
                    blocked |= qs;
                    left.push_back(g);
                }
            }
            // full-pass cost of the members one by one vs fused: the state is
            // read and written once per op, so fusing saves passes; dense
            // arithmetic grows as 2^k (cost model: passes dominate up to F).
            bool all_diag = true;
            for (const Operator *g : take) all_diag &= g->diag;
            std::vector<int> ql;
            for (int q = 0; q < 64; ++q)
                if ((U >> q) & 1) ql.push_back(q);
            if (take.size() == 1) {
                add_full_pass_op(buffer, nb, *take[0]);
                account_full_pass(buffer, nb, *take[0]);
            } else {
                Operator acc;
                acc.q = ql;
                acc.diag = all_diag;
                if (all_diag) acc.m.assign(1ull << ql.size(), cplx(1.0, 0.0));
                else {
                    const uint64_t d = 1ull << ql.size();
                    acc.m.assign(d * d, cplx(0.0, 0.0));
                    for (uint64_t i = 0; i < d; ++i) acc.m[i * d + i] = 1.0;
                }
                for (const Operator *g : take) apply_left(acc, *g);
                add_full_pass_op(buffer, nb, acc);
                account_full_pass(buffer, nb, acc);
            }
            rem.swap(left);
        }
    }

    // Estimated device time of an op (cost model of the adaptive simulator).
    // A stage: HBM time at the measured copy rate (5.1 TB/s) and compute time
    // (its operators plus a fixed per-chunk part: loads, stores, transposes)
    // overlap, the smaller contributing a fifth (measured on MI355X).  Full
    // passes: the larger of HBM and arithmetic time.  Plus a launch overhead.
    static double est_seconds(const PlanOp &op)
    {
        if (op.kind == SIM_OP_STAGE) {
            const double amps = std::ldexp(1.0, op.buffer_qubits);
            const bool c64 = op.bytes < 24.0 * amps;  // 2 x 8 B per amplitude
            const double mem = op.bytes / 5.1e12;
            const double comp = op.est_s + (c64 ? 1.5e-3 : 2.5e-3) * amps / 1073741824.0;
            return std::max(mem, comp) + 0.2 * std::min(mem, comp) + 4e-6;
        }
        return std::max(op.bytes / 5.1e12, op.flops / 55e12) + 4e-6;
    }

    // Executes the gates of one buffer with the enabled passes.  With cache
    // blocking on, the diagonal detector's fused tables may block more stage
    // boundaries than they save (diagonals fuse into neighbouring dense blocks
    // for free inside a stage), so both lowerings are built and the cheaper
    // one by the cost model is kept.
    void lower(int buffer, int nb, std::vector<Operator> gates)
    {
        if ((o.opt & SIM_OPT_DIAG) && (o.opt & SIM_OPT_STAGES)) {
            const size_t mark = plan.ops.size();
            // the detector's lowering is built on a copy of the plan on a
            // second thread while this one builds the plain lowering
            Plan alt = plan;
            uint64_t v = 0;
            std::exception_ptr err;
            std::thread th([&] {
                try {
                    Builder b2{alt, o};
                    b2.lower_gates(buffer, nb, diagonal_detector(nb, (int)o.D, gates, &v));
                } catch (...) {
                    err = std::current_exception();
                }
            });
            try {
                lower_gates(buffer, nb, gates);
            } catch (...) {
                th.join();
                throw;
            }
            th.join();
            if (err) std::rethrow_exception(err);
            double t_dd = 0, t_plain = 0;
            for (size_t i = mark; i < alt.ops.size(); ++i) t_dd += est_seconds(alt.ops[i]);
            for (size_t i = mark; i < plan.ops.size(); ++i) t_plain += est_seconds(plan.ops[i]);
            if (t_dd <= t_plain) {  // a tie keeps the detector: fewer, wider table members
                plan.ops.swap(alt.ops);
                plan.stats = alt.stats;
                plan.layout = alt.layout;
            }
            plan.stats.dd_visits += v;
            return;
        }
        if (o.opt & SIM_OPT_DIAG) {
            uint64_t v = 0;
            gates = diagonal_detector(nb, (int)o.D, gates, &v);
            plan.stats.dd_visits += v;
        }
        lower_gates(buffer, nb, std::move(gates));
    }

    void lower_gates(int buffer, int nb, std::vector<Operator> gates)
    {
        if (gates.empty()) return;
        const bool small = buffer != 0 && nb <= (plan.dtype == SIM_C128 ? 13 : 14);
        if ((o.opt & SIM_OPT_STAGES) && small) {
            // the whole sub-state is one chunk: one launch runs its gate list
            PlanOp st;
            st.kind = SIM_OP_STAGE;
            st.buffer = buffer;
            st.buffer_qubits = nb;
            for (int q = 0; q < nb; ++q) st.local.push_back(q);
            st.gates = std::move(gates);
            plan.stats.n_subruns += 1;
            plan.ops.push_back(std::move(st));
            return;
        }
        // a stage chunk holds at least one wave (64 threads of 2^reg_bits amplitudes)
        if ((o.opt & SIM_OPT_STAGES) && nb >= 6 + o.reg_bits) {
            stages(buffer, nb, gates);
        } else if (o.opt & SIM_OPT_FUSE) {
            fused_passes(buffer, nb, gates);
        } else {
            for (const Operator &g : gates) {
                add_full_pass_op(buffer, nb, g);
                account_full_pass(buffer, nb, g);
            }
        }
    }

    void init_op(int buffer, int nb)
    {
        PlanOp op;
        op.kind = SIM_OP_INIT;
        op.buffer = buffer;
        op.buffer_qubits = nb;
        op.bytes = std::ldexp(1.0, nb) * amp_bytes();
        plan.ops.push_back(std::move(op));
        if (buffer == 0) {
            plan.stats.write_passes += 1;
            plan.stats.bytes += std::ldexp(1.0, nb) * amp_bytes();
        }
    }

    // Merge booster (Alg. 7) with these readings: groups are contiguous qubit
    // ranges starting at qubit 0 (the listing counts from 1); the gate block
    // of a group takes every gate whose qubits lie inside the group and that
    // no earlier, untaken gate shares a qubit with (so the block is a prefix
    // of the remaining circuit restricted to the group, and the group stays
    // unentangled from the rest while it runs); an unpaired trailing group is
    // carried to the next round unchanged (the listing would drop it); the
    // division size is ceil(N / B) as in the listing.
    std::vector<Operator> booster(const std::vector<Operator> &gates)
    {
        const int n = plan.n;
        std::vector<int> que;
        divider(n, (n + (int)o.B - 1) / (int)o.B, que);
        if (que.size() <= 1) {
            init_op(0, n);
            return gates;
        }
        struct Group { int lo, len, buffer; };
        std::vector<Group> groups;
        int acc = 0;
        for (int len : que) {
            Group g{acc, len, (int)plan.buffer_qubits.size()};
            plan.buffer_qubits.push_back(len);
            groups.push_back(g);
            init_op(g.buffer, len);
            acc += len;
        }
        plan.stats.booster_groups += groups.size();
        std::vector<Operator> rest = gates;
        std::vector<char> taken(rest.size(), 0);
        while (true) {
            // generation step for every group of this round
            for (const Group &G : groups) {
                const uint64_t gm = (G.len >= 64 ? ~0ull : ((1ull << G.len) - 1)) << G.lo;
                uint64_t blocked = 0;
                std::vector<Operator> block;
                for (size_t i = 0; i < rest.size(); ++i) {
                    if (taken[i]) continue;
                    const uint64_t qs = rest[i].mask();
                    if ((qs & ~gm) || (qs & blocked)) {
                        blocked |= qs;
                        continue;
                    }
                    taken[i] = 1;
                    Operator local = rest[i];
                    for (int &q : local.q) q -= G.lo;
                    block.push_back(std::move(local));
                }
                plan.stats.booster_gates += block.size();
                lower(G.buffer, G.len, std::move(block));
            }
            if (groups.size() == 1) break;
            // merge step: pairs (0,1), (2,3), ...; an odd last group carries over
            std::vector<Group> next;
            for (size_t i = 0; i + 1 < groups.size(); i += 2) {
                const Group &A = groups[i], &Bg = groups[i + 1];
                Group M{A.lo, A.len + Bg.len, 0};
                if (M.len == plan.n) M.buffer = 0;
                else {
                    M.buffer = (int)plan.buffer_qubits.size();
                    plan.buffer_qubits.push_back(M.len);
                }
                PlanOp k;
                k.kind = SIM_OP_KRON;
                k.buffer = M.buffer;
                k.buffer_qubits = M.len;
                k.src_lo = A.buffer;
                k.src_hi = Bg.buffer;
                k.bytes = std::ldexp(1.0, M.len) * amp_bytes();
                k.flops = 6.0 * std::ldexp(1.0, M.len);
                plan.ops.push_back(std::move(k));
                if (M.buffer == 0) {
                    plan.stats.write_passes += 1;
                    plan.stats.bytes += std::ldexp(1.0, M.len) * amp_bytes();
                    plan.stats.n_kron += 1;
                }
                next.push_back(M);
            }
            if (groups.size() & 1) next.push_back(groups.back());
            groups.swap(next);
            if (groups.size() == 1 && groups[0].buffer == 0) break;
        }
        std::vector<Operator> left;
        for (size_t i = 0; i < rest.size(); ++i)
            if (!taken[i]) left.push_back(rest[i]);
        return left;
    }
};

}  // namespace

namespace {

// True for the exact two-qubit exchange |ab> -> |ba> (entries exactly 0 and 1).
bool is_swap(const Operator &g)
{
    if (g.k() != 2 || g.diag) return false;
    for (uint64_t r = 0; r < 4; ++r)
        for (uint64_t c = 0; c < 4; ++c) {
            const uint64_t sr = ((r & 1) << 1) | (r >> 1);
            if (g.at(r, c) != cplx(c == sr ? 1.0 : 0.0, 0.0)) return false;
        }
    return true;
}

// Qubit relabelling (Sec. 2.3: a swap only changes which index bit holds a
// qubit, so the gates after it are re-indexed): with remapping enabled a SWAP
// gate moves no data.  pi[q] is the label logical qubit q carries after the
// swaps seen so far; later gates act on the relabelled qubits.
std::vector<Operator> relabel_swaps(const std::vector<Operator> &gates, int n, std::vector<int> &pi)
{
    pi.resize(n);
    for (int q = 0; q < n; ++q) pi[q] = q;
    std::vector<Operator> out;
    out.reserve(gates.size());
    for (const Operator &g : gates) {
        if (is_swap(g)) {
            std::swap(pi[g.q[0]], pi[g.q[1]]);
            continue;
        }
        out.push_back(g);
        for (int &q : out.back().q) q = pi[q];
    }
    return out;
}

}  // namespace

// Phase form of a product of diagonals on one or two qubits (entries of unit
// modulus): with c = arg d(00), a diagonal d on qubits (q, p) has phase
// c + (arg d(10) - c) x_q + (arg d(01) - c) x_p
//   + (arg d(11) - arg d(10) - arg d(01) + c) x_q x_p
// (entry index bit t <-> qubit t of the gate), and the phases of a product
// add up.
static void quad_coefficients(KOp &k, int n)
{
    k.qc = 0;
    k.qa.assign(n, 0.0);
    k.qb.assign((size_t)n * n, 0.0);
    for (const Operator &g : k.members) {
        const double c = std::arg(g.m[0]);
        k.qc += c;
        if (g.k() == 1) {
            k.qa[g.q[0]] += std::arg(g.m[1]) - c;
            continue;
        }
        const double d1 = std::arg(g.m[1]), d2 = std::arg(g.m[2]), d3 = std::arg(g.m[3]);
        k.qa[g.q[0]] += d1 - c;
        k.qa[g.q[1]] += d2 - c;
        const int lo = std::min(g.q[0], g.q[1]), hi = std::max(g.q[0], g.q[1]);
        k.qb[(size_t)lo * n + hi] += d3 - d1 - d2 + c;
    }
    k.members.clear();
}

void build_plan(Plan &plan, const std::vector<Operator> &gates)
{
    auto t0 = std::chrono::steady_clock::now();
    plan.ops.clear();
    plan.stats = PlanStats();
    plan.buffer_qubits.assign(1, plan.n);
    plan.layout.resize(plan.n);
    for (int q = 0; q < plan.n; ++q) plan.layout[q] = q;
    std::vector<int> pi;
    const bool relabel = (plan.opt.opt & SIM_OPT_REMAP) &&
                         std::any_of(gates.begin(), gates.end(), [](const Operator &g) { return is_swap(g); });
    std::vector<Operator> relabelled;
    if (relabel) relabelled = relabel_swaps(gates, plan.n, pi);
    const std::vector<Operator> &in = relabel ? relabelled : gates;
    Builder b{plan, plan.opt};
    std::vector<Operator> rest;
    if (plan.opt.window_qubits > 0) {
        b.offload(in);
    } else {
        if (plan.opt.opt & SIM_OPT_BOOST) {
            rest = b.booster(in);
        } else {
            b.init_op(0, plan.n);
            rest = in;
        }
        b.lower(0, plan.n, std::move(rest));
    }
    for (PlanOp &op : plan.ops)  // tables of the accumulated diagonals of the kept lowering
        for (Phase &ph : op.phases)
            for (KOp &k : ph.ops)
                if (k.type == KOp::QUAD) {
                    quad_coefficients(k, op.buffer_qubits);
                } else if (!k.members.empty()) {
                    std::vector<const Operator *> ms;
                    for (const Operator &g : k.members) ms.push_back(&g);
                    k.table = diag_product(k.dq, ms).m;
                    k.members.clear();
                }
    if (relabel) {  // logical q carries label pi[q], which sits at bit layout[pi[q]]
        std::vector<int> lay(plan.n);
        for (int q = 0; q < plan.n; ++q) lay[q] = plan.layout[pi[q]];
        plan.layout.swap(lay);
    }
    plan.stats.n_ops = plan.ops.size();
    for (const PlanOp &op : plan.ops)
        if (op.buffer == 0 && op.kind != SIM_OP_WINDOW) plan.stats.est_ms += 1e3 * Builder::est_seconds(op);
    plan.stats.est_ms += 1e3 * plan.stats.pcie_bytes / 50e9;  // host link, one direction at a time
    auto t1 = std::chrono::steady_clock::now();
    plan.stats.plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace qs
