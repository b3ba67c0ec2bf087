/*
 * Plain complex128 full-state simulator -- TEST INFRASTRUCTURE ONLY.
 *
 * This is the oracle the GPU path is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * What it computes (paper, Sec. 2.1-2.2, Eq. (1) and Alg. 1):
 *   the state |psi> = sum_i a_i |i>, i in [0, 2^N), each a_i a pair of IEEE
 *   binary64 numbers; start at |0...0>; apply every gate of the circuit in
 *   input order, one full pass over the state per gate (gate-by-gate scheme).
 *   Qubit j is bit j of the amplitude index (Sec. 2.2: U_j acts on the pairs
 *   that differ only in bit j).  For a k-qubit gate on the ordered list
 *   q[0..k-1], bit t of the gate matrix's row/column index is bit q[t] of the
 *   amplitude index; an ascending list reproduces the two-qubit layout of
 *   Sec. 2.2 (higher qubit = most significant matrix bit).
 *
 * Every gate, diagonal ones included, goes through the same dense
 * gather / matrix-vector / scatter loop: no special cases.
 *
 * Build: gcc -O3 -fopenmp -ffp-contract=off (no fused multiply-add, so the
 * rounding of each product and sum is the plain IEEE one).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Gate kinds (oracle-private numbering). */
enum {
    OG_MATRIX = 0, /* explicit 2^k x 2^k complex matrix, row-major, (re,im) */
    OG_DIAG = 1,   /* explicit 2^k diagonal, (re,im)                        */
    OG_H, OG_X, OG_Y, OG_Z, OG_S, OG_T, OG_SX,
    OG_RX, OG_RY, OG_RZ,
    OG_CZ, OG_CNOT, OG_CPHASE, OG_RZZ, OG_SWAP,
    OG_NKINDS
};

typedef struct {
    int32_t kind;
    int32_t nq;
    int32_t q[6];
    double theta;
    const double *data;
} og_gate;

#define OG_MAXK 6

static int og_arity(int kind, int nq)
{
    switch (kind) {
    case OG_MATRIX: case OG_DIAG: return nq;
    case OG_CZ: case OG_CNOT: case OG_CPHASE: case OG_RZZ: case OG_SWAP: return 2;
    default: return 1;
    }
}

/*
 * The textbook matrix of a gate (the paper names the gates but prints no
 * matrices).  M is 2^k x 2^k complex, row-major, interleaved (re, im).
 * Returns 0 on success, -1 for an unknown kind or bad arity.
 */
int og_gate_matrix(const og_gate *g, double *M)
{
    int k = og_arity(g->kind, g->nq);
    if (k < 1 || k > OG_MAXK || g->nq != k) return -1;
    int d = 1 << k;
    memset(M, 0, sizeof(double) * 2 * d * d);
#define RE(r, c) M[2 * ((r) * d + (c))]
#define IM(r, c) M[2 * ((r) * d + (c)) + 1]
    double th = g->theta, c = cos(th / 2), s = sin(th / 2), r2 = 1.0 / sqrt(2.0);
    switch (g->kind) {
    case OG_MATRIX:
        if (!g->data) return -1;
        memcpy(M, g->data, sizeof(double) * 2 * d * d);
        break;
    case OG_DIAG:
        if (!g->data) return -1;
        for (int i = 0; i < d; ++i) { RE(i, i) = g->data[2 * i]; IM(i, i) = g->data[2 * i + 1]; }
        break;
    case OG_H: RE(0, 0) = r2; RE(0, 1) = r2; RE(1, 0) = r2; RE(1, 1) = -r2; break;
    case OG_X: RE(0, 1) = 1; RE(1, 0) = 1; break;
    case OG_Y: IM(0, 1) = -1; IM(1, 0) = 1; break;
    case OG_Z: RE(0, 0) = 1; RE(1, 1) = -1; break;
    case OG_S: RE(0, 0) = 1; IM(1, 1) = 1; break;
    case OG_T: RE(0, 0) = 1; RE(1, 1) = r2; IM(1, 1) = r2; break;
    case OG_SX: /* square root of X: (1/2) [[1+i, 1-i], [1-i, 1+i]] */
        RE(0, 0) = 0.5; IM(0, 0) = 0.5; RE(0, 1) = 0.5; IM(0, 1) = -0.5;
        RE(1, 0) = 0.5; IM(1, 0) = -0.5; RE(1, 1) = 0.5; IM(1, 1) = 0.5;
        break;
    case OG_RX: /* exp(-i theta X / 2) */
        RE(0, 0) = c; IM(0, 1) = -s; IM(1, 0) = -s; RE(1, 1) = c; break;
    case OG_RY: /* exp(-i theta Y / 2) */
        RE(0, 0) = c; RE(0, 1) = -s; RE(1, 0) = s; RE(1, 1) = c; break;
    case OG_RZ: /* exp(-i theta Z / 2) */
        RE(0, 0) = c; IM(0, 0) = -s; RE(1, 1) = c; IM(1, 1) = s; break;
    case OG_CZ: RE(0, 0) = 1; RE(1, 1) = 1; RE(2, 2) = 1; RE(3, 3) = -1; break;
    case OG_CNOT: /* q[0] control = matrix bit 0, q[1] target = matrix bit 1 */
        RE(0, 0) = 1; RE(2, 2) = 1; RE(1, 3) = 1; RE(3, 1) = 1; break;
    case OG_CPHASE: /* diag(1, 1, 1, e^{i theta}) */
        RE(0, 0) = 1; RE(1, 1) = 1; RE(2, 2) = 1; RE(3, 3) = cos(th); IM(3, 3) = sin(th); break;
    case OG_RZZ: /* exp(-i theta Z(x)Z / 2): e^{-i theta/2} on even parity */
        RE(0, 0) = c; IM(0, 0) = -s; RE(1, 1) = c; IM(1, 1) = s;
        RE(2, 2) = c; IM(2, 2) = s; RE(3, 3) = c; IM(3, 3) = -s; break;
    case OG_SWAP: RE(0, 0) = 1; RE(1, 2) = 1; RE(2, 1) = 1; RE(3, 3) = 1; break;
    default: return -1;
    }
#undef RE
#undef IM
    return 0;
}

static int og_check(int n, const og_gate *g)
{
    int k = og_arity(g->kind, g->nq);
    if (g->kind < 0 || g->kind >= OG_NKINDS || k < 1 || k > OG_MAXK || g->nq != k || k > n) return -1;
    for (int t = 0; t < k; ++t) {
        if (g->q[t] < 0 || g->q[t] >= n) return -1;
        for (int u = 0; u < t; ++u)
            if (g->q[u] == g->q[t]) return -1;
    }
    return 0;
}

/* Apply one gate: the 2^N x 2^N lift of M, by gather / multiply / scatter. */
static void og_apply_one(int n, const og_gate *g, const double *M, double *a)
{
    int k = g->nq, d = 1 << k;
    int sorted[OG_MAXK];
    for (int t = 0; t < k; ++t) sorted[t] = g->q[t];
    for (int t = 1; t < k; ++t)             /* insertion sort, ascending */
        for (int u = t; u > 0 && sorted[u - 1] > sorted[u]; --u) {
            int tmp = sorted[u]; sorted[u] = sorted[u - 1]; sorted[u - 1] = tmp;
        }
    /* offset of matrix index r: bit t of r goes to amplitude bit q[t] */
    uint64_t off[1 << OG_MAXK];
    for (int r = 0; r < d; ++r) {
        uint64_t o = 0;
        for (int t = 0; t < k; ++t)
            if ((r >> t) & 1) o |= (uint64_t)1 << g->q[t];
        off[r] = o;
    }
    int64_t groups = (int64_t)1 << (n - k);
#pragma omp parallel for schedule(static) if (groups >= 65536)
    for (int64_t grp = 0; grp < groups; ++grp) {
        /* base index: insert a zero at every target position, low to high */
        uint64_t base = (uint64_t)grp;
        for (int t = 0; t < k; ++t) {
            uint64_t lo = base & (((uint64_t)1 << sorted[t]) - 1);
            base = ((base >> sorted[t]) << (sorted[t] + 1)) | lo;
        }
        double vr[1 << OG_MAXK], vi[1 << OG_MAXK];
        for (int c = 0; c < d; ++c) {
            vr[c] = a[2 * (base | off[c])];
            vi[c] = a[2 * (base | off[c]) + 1];
        }
        for (int r = 0; r < d; ++r) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < d; ++c) {
                double mr = M[2 * (r * d + c)], mi = M[2 * (r * d + c) + 1];
                sr += mr * vr[c] - mi * vi[c];
                si += mr * vi[c] + mi * vr[c];
            }
            a[2 * (base | off[r])] = sr;
            a[2 * (base | off[r]) + 1] = si;
        }
    }
}

/* Apply gates[0..ng) in order to the state a (2^n complex, interleaved). */
int og_apply(int n, const og_gate *gates, int64_t ng, double *a)
{
    if (n < 0 || n > 40) return -1;
    double M[2 * (1 << OG_MAXK) * (1 << OG_MAXK)];
    for (int64_t i = 0; i < ng; ++i) {
        if (og_check(n, &gates[i]) != 0) return -1;
        if (og_gate_matrix(&gates[i], M) != 0) return -1;
        og_apply_one(n, &gates[i], M, a);
    }
    return 0;
}

/* |0...0> followed by the circuit. */
int og_run(int n, const og_gate *gates, int64_t ng, double *a)
{
    if (n < 0 || n > 40) return -1;
    int64_t len = (int64_t)2 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i) a[i] = 0.0;
    a[0] = 1.0;
    return og_apply(n, gates, ng, a);
}

/* Pairwise (recursive halving) sum of |a_i|^2 over [lo, hi). */
static double og_pairwise_norm(const double *a, int64_t lo, int64_t hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += a[2 * i] * a[2 * i] + a[2 * i + 1] * a[2 * i + 1];
        return s;
    }
    int64_t mid = lo + (hi - lo) / 2;
    return og_pairwise_norm(a, lo, mid) + og_pairwise_norm(a, mid, hi);
}

double og_norm(int n, const double *a)
{
    int64_t len = (int64_t)1 << n;
    /* split the top of the recursion across threads; the tree is the same */
    int levels = n < 6 ? 0 : 6;
    int64_t parts = (int64_t)1 << levels, step = len >> levels;
    double part[64];
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < parts; ++p) part[p] = og_pairwise_norm(a, p * step, (p + 1) * step);
    for (int l = levels; l > 0; --l)
        for (int64_t p = 0; p < ((int64_t)1 << (l - 1)); ++p) part[p] = part[2 * p] + part[2 * p + 1];
    return part[0];
}

/* <a|b> = sum conj(a_i) b_i, pairwise over the same tree as og_norm. */
static void og_pairwise_inner(const double *a, const double *b, int64_t lo, int64_t hi, double *re, double *im)
{
    if (hi - lo <= 8) {
        double sr = 0.0, si = 0.0;
        for (int64_t i = lo; i < hi; ++i) {
            double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
            sr += ar * br + ai * bi;
            si += ar * bi - ai * br;
        }
        *re = sr; *im = si;
        return;
    }
    int64_t mid = lo + (hi - lo) / 2;
    double r1, i1, r2, i2;
    og_pairwise_inner(a, b, lo, mid, &r1, &i1);
    og_pairwise_inner(a, b, mid, hi, &r2, &i2);
    *re = r1 + r2; *im = i1 + i2;
}

void og_inner(int n, const double *a, const double *b, double *out)
{
    int64_t len = (int64_t)1 << n;
    int levels = n < 6 ? 0 : 6;
    int64_t parts = (int64_t)1 << levels, step = len >> levels;
    double pr[64], pi[64];
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < parts; ++p) og_pairwise_inner(a, b, p * step, (p + 1) * step, &pr[p], &pi[p]);
    for (int l = levels; l > 0; --l)
        for (int64_t p = 0; p < ((int64_t)1 << (l - 1)); ++p) {
            pr[p] = pr[2 * p] + pr[2 * p + 1];
            pi[p] = pi[2 * p] + pi[2 * p + 1];
        }
    out[0] = pr[0]; out[1] = pi[0];
}

/*
 * Marginal distribution over the qubit list S (the measurement background of
 * Sec. 2, an unnumbered subsection between Sec. 2.3 and Sec. 2.4):
 * P[y] = sum over x with bit S[t] of x equal to bit t of y of |a_x|^2.
 * The index range is cut into a fixed number of equal parts (independent of
 * the thread count), each summed into its own bins in index order, and the
 * parts are combined in part order: the result does not depend on
 * OMP_NUM_THREADS.
 */
int og_marginal(int n, const double *a, const int32_t *S, int ns, double *out)
{
    if (ns < 0 || ns > 24 || ns > n) return -1;
    for (int t = 0; t < ns; ++t) {
        if (S[t] < 0 || S[t] >= n) return -1;
        for (int u = 0; u < t; ++u) if (S[u] == S[t]) return -1;
    }
    int64_t nb = (int64_t)1 << ns, len = (int64_t)1 << n;
    int64_t parts = ns <= 20 ? 16 : 1;
    if (parts > len) parts = len;
    double *bins = (double *)calloc((size_t)(parts * nb), sizeof(double));
    if (!bins) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < parts; ++p) {
        int64_t lo = len * p / parts, hi = len * (p + 1) / parts;
        double *mine = bins + p * nb;
        for (int64_t x = lo; x < hi; ++x) {
            int64_t y = 0;
            for (int t = 0; t < ns; ++t) y |= (int64_t)((x >> S[t]) & 1) << t;
            mine[y] += a[2 * x] * a[2 * x] + a[2 * x + 1] * a[2 * x + 1];
        }
    }
    for (int64_t y = 0; y < nb; ++y) {
        double s = 0.0;
        for (int64_t p = 0; p < parts; ++p) s += bins[p * nb + y];
        out[y] = s;
    }
    free(bins);
    return 0;
}

int og_num_threads(void) { return omp_get_max_threads(); }
void og_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
