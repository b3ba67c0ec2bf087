// Gate library and operator algebra of the host optimiser (FP64).
//
// The paper names the gates it uses (Z, CP, RZZ in Sec. 3 and 4.5; RX, H, RY in
// Sec. 4.5; CNOT and RZ in Sec. 5.1) but prints no matrices; the textbook ones
// are used.  Matrix layout follows Sec. 2.2: bit t of the row/column index is
// qubit q[t].
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "ir.hpp"

namespace qs {

namespace {

int arity(uint32_t kind, uint32_t nq)
{
    switch (kind) {
    case SIM_G_MATRIX: case SIM_G_DIAG: return (int)nq;
    case SIM_G_CZ: case SIM_G_CNOT: case SIM_G_CPHASE: case SIM_G_RZZ: case SIM_G_SWAP: return 2;
    default: return 1;
    }
}

}  // namespace

Operator gate_operator(const sim_gate &g, int n, std::string *err)
{
    Operator op;
    if (g.kind >= SIM_G_NKINDS) { *err = "unknown gate kind"; return op; }
    const int k = arity(g.kind, g.nq);
    if (k < 1 || k > kMaxGateQubits || (int)g.nq != k) { *err = "bad qubit count for gate kind"; return op; }
    for (int t = 0; t < k; ++t) {
        if ((int)g.q[t] >= n) { *err = "qubit index out of range"; return op; }
        for (int u = 0; u < t; ++u)
            if (g.q[u] == g.q[t]) { *err = "duplicate qubit in gate"; return op; }
        op.q.push_back((int)g.q[t]);
    }
    const int d = 1 << k;
    const double th = g.theta, c = std::cos(th / 2), s = std::sin(th / 2), r2 = std::sqrt(0.5);
    const cplx I(0.0, 1.0);
    auto dense = [&](std::initializer_list<cplx> v) { op.diag = false; op.m.assign(v); };
    auto diagv = [&](std::initializer_list<cplx> v) { op.diag = true; op.m.assign(v); };
    switch (g.kind) {
    case SIM_G_MATRIX: {
        if (!g.data) { *err = "MATRIX gate without data"; return op; }
        op.diag = false;
        op.m.resize((size_t)d * d);
        for (int i = 0; i < d * d; ++i) op.m[i] = cplx(g.data[2 * i], g.data[2 * i + 1]);
        // unitarity: |M^H M - I| <= 1e-10 entrywise
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                cplx acc = 0;
                for (int r = 0; r < d; ++r) acc += std::conj(op.m[r * d + a]) * op.m[r * d + b];
                if (std::abs(acc - (a == b ? 1.0 : 0.0)) > 1e-10) { *err = "MATRIX gate is not unitary"; return op; }
            }
        if (is_diagonal(op)) {
            std::vector<cplx> dv(d);
            for (int i = 0; i < d; ++i) dv[i] = op.m[(size_t)i * d + i];
            op.m = dv;
            op.diag = true;
        }
        break;
    }
    case SIM_G_DIAG:
        if (!g.data) { *err = "DIAG gate without data"; return op; }
        op.diag = true;
        op.m.resize(d);
        for (int i = 0; i < d; ++i) {
            op.m[i] = cplx(g.data[2 * i], g.data[2 * i + 1]);
            if (std::abs(std::abs(op.m[i]) - 1.0) > 1e-10) { *err = "DIAG entry is not of unit modulus"; return op; }
        }
        break;
    case SIM_G_H: dense({r2, r2, r2, -r2}); break;
    case SIM_G_X: dense({0, 1, 1, 0}); break;
    case SIM_G_Y: dense({0, -I, I, 0}); break;
    case SIM_G_Z: diagv({1, -1}); break;
    case SIM_G_S: diagv({1, I}); break;
    case SIM_G_T: diagv({1, cplx(r2, r2)}); break;
    case SIM_G_SX: dense({cplx(0.5, 0.5), cplx(0.5, -0.5), cplx(0.5, -0.5), cplx(0.5, 0.5)}); break;
    case SIM_G_RX: dense({c, -I * s, -I * s, c}); break;
    case SIM_G_RY: dense({c, -s, s, c}); break;
    case SIM_G_RZ: diagv({cplx(c, -s), cplx(c, s)}); break;
    case SIM_G_CZ: diagv({1, 1, 1, -1}); break;
    case SIM_G_CPHASE: diagv({1, 1, 1, cplx(std::cos(th), std::sin(th))}); break;
    case SIM_G_RZZ: diagv({cplx(c, -s), cplx(c, s), cplx(c, s), cplx(c, -s)}); break;
    case SIM_G_CNOT:  // index = b(control) + 2 b(target)
        dense({1, 0, 0, 0,  0, 0, 0, 1,  0, 0, 1, 0,  0, 1, 0, 0});
        break;
    case SIM_G_SWAP:
        dense({1, 0, 0, 0,  0, 0, 1, 0,  0, 1, 0, 0,  0, 0, 0, 1});
        break;
    default: *err = "unknown gate kind"; return op;
    }
    return op;
}

bool is_diagonal(const Operator &op)
{
    if (op.diag) return true;
    const uint64_t d = 1ull << op.q.size();
    for (uint64_t r = 0; r < d; ++r)
        for (uint64_t c = 0; c < d; ++c)
            if (r != c && op.m[r * d + c] != cplx(0.0, 0.0)) return false;
    return true;
}

uint64_t need_mask(const Operator &op)
{
    if (op.diag) return 0;
    const int k = op.k();
    const uint64_t d = 1ull << k;
    uint64_t need = 0;
    for (int t = 0; t < k; ++t) {
        bool blockdiag = true;
        for (uint64_t r = 0; r < d && blockdiag; ++r)
            for (uint64_t c = 0; c < d; ++c)
                if ((((r ^ c) >> t) & 1) && op.m[r * d + c] != cplx(0.0, 0.0)) { blockdiag = false; break; }
        if (!blockdiag) need |= 1ull << op.q[t];
    }
    return need;
}

Operator embed(const Operator &op, const std::vector<int> &to)
{
    const int k = op.k(), K = (int)to.size();
    std::vector<int> pos(k);
    uint64_t inmask = 0;
    for (int t = 0; t < k; ++t) {
        int p = -1;
        for (int u = 0; u < K; ++u)
            if (to[u] == op.q[t]) p = u;
        if (p < 0) throw std::runtime_error("embed: qubit not in target list");
        pos[t] = p;
        inmask |= 1ull << p;
    }
    auto sub = [&](uint64_t x) {
        uint64_t r = 0;
        for (int t = 0; t < k; ++t) r |= ((x >> pos[t]) & 1ull) << t;
        return r;
    };
    Operator out;
    out.q = to;
    const uint64_t D = 1ull << K;
    if (op.diag) {
        out.diag = true;
        out.m.resize(D);
        for (uint64_t x = 0; x < D; ++x) out.m[x] = op.m[sub(x)];
        return out;
    }
    out.diag = false;
    out.m.assign(D * D, cplx(0.0, 0.0));
    for (uint64_t r = 0; r < D; ++r)
        for (uint64_t c = 0; c < D; ++c)
            if ((r & ~inmask) == (c & ~inmask)) out.m[r * D + c] = op.m[(sub(r) << k) + sub(c)];
    return out;
}

void apply_left(Operator &acc, const Operator &g)
{
    const int K = acc.k(), k = g.k();
    std::vector<int> pos(k);
    for (int t = 0; t < k; ++t) {
        pos[t] = -1;
        for (int u = 0; u < K; ++u)
            if (acc.q[u] == g.q[t]) pos[t] = u;
        if (pos[t] < 0) throw std::runtime_error("apply_left: qubit not in accumulator");
    }
    const uint64_t D = 1ull << K, d = 1ull << k;
    if (acc.diag && g.diag) {
        for (uint64_t x = 0; x < D; ++x) {
            uint64_t r = 0;
            for (int t = 0; t < k; ++t) r |= ((x >> pos[t]) & 1ull) << t;
            acc.m[x] *= g.m[r];
        }
        return;
    }
    if (acc.diag) {  // promote to dense
        std::vector<cplx> full(D * D, cplx(0.0, 0.0));
        for (uint64_t x = 0; x < D; ++x) full[x * D + x] = acc.m[x];
        acc.m.swap(full);
        acc.diag = false;
    }
    uint64_t gmask = 0;
    std::vector<uint64_t> off(d);
    for (uint64_t r = 0; r < d; ++r) {
        uint64_t o = 0;
        for (int t = 0; t < k; ++t)
            if ((r >> t) & 1) o |= 1ull << pos[t];
        off[r] = o;
    }
    for (int t = 0; t < k; ++t) gmask |= 1ull << pos[t];
    std::vector<cplx> v(d), w(d);
    // every column of acc is a state of K qubits; apply g to it
    for (uint64_t col = 0; col < D; ++col)
        for (uint64_t base = 0; base < D; ++base) {
            if (base & gmask) continue;
            for (uint64_t c = 0; c < d; ++c) v[c] = acc.m[(base | off[c]) * D + col];
            for (uint64_t r = 0; r < d; ++r) {
                cplx s = 0;
                for (uint64_t c = 0; c < d; ++c) s += g.at(r, c) * v[c];
                w[r] = s;
            }
            for (uint64_t r = 0; r < d; ++r) acc.m[(base | off[r]) * D + col] = w[r];
        }
}

namespace {

// out (a diagonal on `to`) *= d, entry by entry; d's index is the OR of a part
// from the low `lo` bits of the entry index and a part from the high bits
void diag_multiply_into(Operator &out, const Operator &d)
{
    const int K = out.k(), lo = K / 2, hi = K - lo;
    std::vector<int> pos(d.k());
    for (int t = 0; t < d.k(); ++t) {
        pos[t] = -1;
        for (int u = 0; u < K; ++u)
            if (out.q[u] == d.q[t]) pos[t] = u;
        if (pos[t] < 0) throw std::runtime_error("diag_product: qubit not in target list");
    }
    std::vector<uint32_t> tl(1u << lo), th(1u << hi);
    for (uint32_t x = 0; x < (1u << lo); ++x) {
        uint32_t r = 0;
        for (int t = 0; t < d.k(); ++t)
            if (pos[t] < lo) r |= ((x >> pos[t]) & 1u) << t;
        tl[x] = r;
    }
    for (uint32_t x = 0; x < (1u << hi); ++x) {
        uint32_t r = 0;
        for (int t = 0; t < d.k(); ++t)
            if (pos[t] >= lo) r |= ((x >> (pos[t] - lo)) & 1u) << t;
        th[x] = r;
    }
    const cplx *dm = d.m.data();
    for (uint32_t xh = 0; xh < (1u << hi); ++xh) {
        const uint32_t rh = th[xh];
        cplx *row = out.m.data() + ((uint64_t)xh << lo);
        for (uint32_t xl = 0; xl < (1u << lo); ++xl) {
            const cplx a = row[xl], b = dm[rh | tl[xl]];
            row[xl] = cplx(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
        }
    }
}

}  // namespace

Operator diag_product(const std::vector<int> &to, const std::vector<const Operator *> &ds)
{
    const int K = (int)to.size();
    if (K > 30) throw std::runtime_error("diag_product: too many qubits");
    for (const Operator *d : ds)
        if (!d->diag) throw std::runtime_error("diag_product: member not diagonal");
    Operator out;
    out.q = to;
    out.diag = true;
    out.m.assign(1ull << K, cplx(1.0, 0.0));
    // narrow members are first multiplied into partial products on at most
    // kP qubits (small tables), so a full-size pass is paid per partial
    // product rather than per member
    const int kP = 8;
    if (K <= kP || ds.size() < 4) {
        for (const Operator *d : ds) diag_multiply_into(out, *d);
        return out;
    }
    std::vector<std::vector<int>> pq;
    std::vector<std::vector<const Operator *>> pm;
    for (const Operator *d : ds) {
        if (d->k() >= kP) {
            diag_multiply_into(out, *d);
            continue;
        }
        int best = -1;
        size_t best_size = 0;
        for (size_t p = 0; p < pq.size(); ++p) {
            std::vector<int> u = pq[p];
            for (int x : d->q)
                if (std::find(u.begin(), u.end(), x) == u.end()) u.push_back(x);
            if ((int)u.size() <= kP && (best < 0 || u.size() < best_size)) {
                best = (int)p;
                best_size = u.size();
            }
        }
        if (best < 0) {
            pq.emplace_back(d->q.begin(), d->q.end());
            pm.push_back({d});
        } else {
            for (int x : d->q)
                if (std::find(pq[best].begin(), pq[best].end(), x) == pq[best].end()) pq[best].push_back(x);
            pm[best].push_back(d);
        }
    }
    for (size_t p = 0; p < pq.size(); ++p) {
        Operator part;
        part.q = pq[p];
        part.diag = true;
        part.m.assign(1ull << pq[p].size(), cplx(1.0, 0.0));
        for (const Operator *d : pm[p]) diag_multiply_into(part, *d);
        diag_multiply_into(out, part);
    }
    return out;
}

Operator compose(const Operator &a, const Operator &b)
{
    std::vector<int> u = a.q;
    for (int x : b.q) {
        bool have = false;
        for (int y : u) have |= (x == y);
        if (!have) u.push_back(x);
    }
    Operator acc = embed(a, u);
    apply_left(acc, b);
    return acc;
}

std::vector<cplx> sub_block(const Operator &op, const std::vector<int> &fixed_pos, uint64_t sel)
{
    const int k = op.k();
    uint64_t fmask = 0, fval = 0;
    for (size_t u = 0; u < fixed_pos.size(); ++u) {
        fmask |= 1ull << fixed_pos[u];
        fval |= ((sel >> u) & 1ull) << fixed_pos[u];
    }
    std::vector<int> free_pos;
    for (int t = 0; t < k; ++t)
        if (!((fmask >> t) & 1)) free_pos.push_back(t);
    const int kf = (int)free_pos.size();
    const uint64_t df = 1ull << kf;
    auto expand = [&](uint64_t x) {
        uint64_t r = fval;
        for (int t = 0; t < kf; ++t) r |= ((x >> t) & 1ull) << free_pos[t];
        return r;
    };
    std::vector<cplx> out(df * df);
    for (uint64_t r = 0; r < df; ++r)
        for (uint64_t c = 0; c < df; ++c) out[r * df + c] = op.at(expand(r), expand(c));
    return out;
}

}  // namespace qs
