// Internal representation shared by the host optimiser, the executor and the
// C ABI.  Host-only C++17; no HIP types here.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qsim355.h"

namespace qs {

using cplx = std::complex<double>;

constexpr int kMaxGateQubits = 6;

// A linear operator on an ordered qubit list: bit t of the row/column index
// is qubit q[t] of the buffer it acts on.  `diag` operators store only the
// 2^k diagonal; dense ones store the 2^k x 2^k matrix row-major.
struct Operator {
    std::vector<int> q;
    bool diag = false;
    std::vector<cplx> m;

    int k() const { return (int)q.size(); }
    uint64_t mask() const {
        uint64_t s = 0;
        for (int x : q) s |= 1ull << x;
        return s;
    }
    cplx at(uint64_t r, uint64_t c) const {
        if (diag) return r == c ? m[r] : cplx(0.0, 0.0);
        return m[(r << q.size()) + c];
    }
};

// Qubits on which the operator is not block diagonal (the qubits a stage must
// hold locally); on the others it only selects a block, like a control.
uint64_t need_mask(const Operator &op);
// True when every off-diagonal entry is exactly zero.
bool is_diagonal(const Operator &op);
// The operator on the superset list `to` (every qubit of op.q must be in to).
Operator embed(const Operator &op, const std::vector<int> &to);
// Product of diagonal operators (every qubit of each in `to`), as a diagonal
// on the list `to`; members multiply in list order.
Operator diag_product(const std::vector<int> &to, const std::vector<const Operator *> &ds);
// Returns b * a (a applied first); result on the union of their qubit lists
// (a's qubits first, then b's new ones, in order).
Operator compose(const Operator &a, const Operator &b);
// Left-multiplies `acc` (on list acc.q) in place by `g`, whose qubits must all
// be in acc.q.
void apply_left(Operator &acc, const Operator &g);
// Block of a dense operator with the qubits in `fixed_pos` (indices into q)
// pinned to the bits of `sel`; result acts on the remaining qubits in order.
std::vector<cplx> sub_block(const Operator &op, const std::vector<int> &fixed_pos, uint64_t sel);

// Validated input gate with its textbook matrix.
Operator gate_operator(const sim_gate &g, int n_qubits, std::string *err);

// ---------------------------------------------------------------------------
// Plan

// One op executed by the stage kernel on the registers of a phase.
struct KOp {
    enum Type : uint32_t { DENSE = 1, DIAG = 2, QUAD = 3 } type;
    uint32_t reg_mask = 0;            // DENSE: register bits acted on
    std::vector<int> sel;             // physical qubits selecting the block (DENSE)
    std::vector<int> dq;              // DIAG: physical qubits of the table index (bit t <-> dq[t])
    std::vector<cplx> table;          // DENSE: 2^|sel| blocks of (2^k)^2; DIAG: 2^|dq| entries
    // DIAG built from several diagonals: the members, multiplied into `table`
    // once the plan is final (planning compares lowerings before that)
    std::vector<Operator> members;
    // QUAD: a diagonal whose phase is a quadratic form of the index bits,
    // phi(x) = qc + sum_q qa[q] x_q + sum_{q<p} qb[q * n + p] x_q x_p over the
    // buffer's n physical qubits (the product of members on one or two
    // qubits: every such diagonal of unit modulus has this form exactly)
    double qc = 0;
    std::vector<double> qa, qb;
    // QUAD while planning: the diagonal tables it replaces, and their cost
    // (microseconds per 2^30 amplitudes), in case the stage keeps tables
    std::vector<KOp> alt;
    double alt_us = 0;
};

struct Phase {
    std::vector<int> reg;             // local bit index of register bit b
    std::vector<int> tmap;            // local bit index of thread-id bit i (lanes = i < 6)
    std::vector<KOp> ops;
};

struct PlanOp {
    sim_op_kind kind;
    int buffer = 0;                   // 0 = full state
    int buffer_qubits = 0;
    int src_lo = 0, src_hi = 0;       // KRON
    Operator op;                      // DENSE / DIAG (physical qubits of the buffer)
    std::vector<int> perm;            // PERM: destination bit of source bit p
    // STAGE
    std::vector<int> local;           // physical local qubits, ascending; local bit i <-> local[i]
    std::vector<Operator> gates;      // the stage's operators in execution order (semantic)
    std::vector<Phase> phases;        // kernel program
    double flops = 0;                 // floating-point operations of the op
    double bytes = 0;                 // algorithmic HBM bytes of the op
    double est_s = 0;                 // STAGE: modelled device seconds of its operators
    // WINDOW (host-memory offload pass): the next pass_ops ops run on each
    // window of the state whose outer qubits [outer_lo, outer_lo + outer_n)
    // are fixed; their qubits are window bits (physical bit p below outer_lo
    // stays p, one above the range becomes p - outer_n, and the outer bits
    // sit at W, W + 1, ... where only selectors may read them)
    int outer_lo = 0, outer_n = 0, pass_ops = 0;
    bool init_window = false;         // the windows start as |0...0> instead of being read
};

struct PlanStats {
    uint64_t full_passes = 0, write_passes = 0, n_stages = 0, n_dense = 0, n_diag = 0,
             n_kron = 0, n_perm = 0, n_subruns = 0, n_ops = 0;
    double bytes = 0, flops = 0, plan_ms = 0, est_ms = 0;
    uint64_t dd_visits = 0, booster_gates = 0, booster_groups = 0;
    uint64_t offload_passes = 0;
    double pcie_bytes = 0;
};

struct Options {
    uint32_t opt = 0, C = 0, F = 5, D = 10, B = 4, force_fuse_k = 0;
    int reg_bits = 4;                 // register bits per thread in a stage
    int fixed_low = 6;                // physical bits every stage keeps local (coalescing; set per dtype)
    int window_qubits = 0;            // host-memory offload: qubits of a device window (0 = off)
};

struct Plan {
    int n = 0;
    sim_dtype dtype = SIM_C128;
    Options opt;
    std::vector<int> buffer_qubits;   // [0] = n; booster sub-states after
    std::vector<PlanOp> ops;
    std::vector<int> layout;          // logical qubit -> physical bit at the end
    PlanStats stats;
};

// Fills the defaults of the options for a dtype.
Options resolve_options(const sim_options *o, sim_dtype dtype, int n);
// Builds the plan (all host passes).  Throws std::runtime_error on failure.
void build_plan(Plan &plan, const std::vector<Operator> &gates);

// Host-memory offload: physical bit of window bit w of a pass whose outer
// range is [lo, lo + n) in a state of `nq` qubits (window bits at and above
// nq - n name the outer bits, in order).
inline int window_to_physical(int w, int lo, int n, int nq)
{
    const int W = nq - n;
    if (w >= W) return lo + (w - W);
    return w < lo ? w : w + n;
}
inline int physical_to_window(int p, int lo, int n, int nq)
{
    const int W = nq - n;
    if (p < lo) return p;
    if (p < lo + n) return W + (p - lo);
    return p - n;
}
// Window qubits for a device work area of `dev_bytes` holding two windows
// (at most nq - 1); 0 if not even one qubit fits.
int offload_window_qubits(uint64_t dev_bytes, uint64_t amp_bytes, int nq);

// Passes, exposed for the plan builder and its tests.
std::vector<Operator> diagonal_detector(int n, int D, const std::vector<Operator> &in, uint64_t *visits);
void divider(int n, int div_size, std::vector<int> &que);

}  // namespace qs
