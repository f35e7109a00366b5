/*
 * FP64 CPU oracle for the amplitude-pairing state-vector method.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header or table with the GPU
 * library: gate matrices, the pair loop, expectations and gradients are all
 * written out here on their own.
 *
 * What it follows (QVecOpt, arXiv 2508.15545):
 *   - state: a dense vector of 2^n complex amplitudes, 16 bytes each in
 *     double precision (Sec. II, Eq. 1-2);
 *   - a one-qubit gate on qubit k updates every pair (i, i XOR 2^k) by the
 *     2x2 matrix (Sec. III.A, Eq. 5). The pairs are enumerated the way the
 *     paper describes: scan i in order, act only when bit k of i is 0, so
 *     each pair is visited exactly once and 2^(n-1) pairs are updated;
 *   - two-qubit gates touch groups of four amplitudes (Sec. III.C says such
 *     gates only mix amplitudes within these groups): the quadruple
 *     {i, i^2^a, i^2^b, i^2^a^2^b} with bits a, b of i equal to 0;
 *   - the result must equal the dense product of Eq. 3-4 (the method changes
 *     neither the logic nor the accuracy, Sec. V), which the tests check.
 *
 * Readings where the paper is silent (gate matrices, qubit order, the 4x4
 * basis order, expectation and gradient definitions) are listed in the design
 * notes; they are: qubit k = bit k of the index; 4x4 index m = bit(t0) +
 * 2 bit(t1); OpenQASM-2 gate matrices; <psi|H|psi> for Pauli sums; gradients
 * of that expectation by the adjoint method, parameter shift and central
 * finite differences.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fcx-limited-range sv_oracle.c -o liboracle.so -lm
 * (-fcx-limited-range makes complex products the textbook (ac-bd, ad+bc)
 * formula instead of a libgcc call with infinity recovery.)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Op codes: the oracle's own numbering (the Python wrapper maps names). */
enum {
    OR_H = 0, OR_X, OR_Y, OR_Z, OR_S, OR_SDG, OR_T, OR_TDG,
    OR_RX, OR_RY, OR_RZ, OR_P, OR_U3, OR_MAT1,
    OR_CX, OR_CZ, OR_CP, OR_SWAP, OR_MAT2,
    OR_NOPS
};

/* One gate of a circuit as the wrapper hands it over. */
typedef struct {
    int32_t op;
    int32_t q0, q1;        /* target (1q) / (control, target) / (t0, t1) */
    int32_t param_index;   /* gradient slot, -1 if fixed */
    double p[32];          /* angles, or the matrix as (re, im) pairs */
} or_gate;

static uint64_t pair_updates = 0; /* Table I invariant: pairs touched */

uint64_t or_pair_updates(void) { return pair_updates; }
void or_reset_pair_updates(void) { pair_updates = 0; }

/* ------------------------------------------------------------ matrices --- */

/* 2x2 matrix of a one-qubit op (row-major, m[2r+c]). Returns 0 on success. */
static int one_qubit_matrix(int op, const double* p, cplx m[4])
{
    const double r2 = 1.0 / sqrt(2.0);
    double c, s;
    switch (op) {
    case OR_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return 0;
    case OR_X: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return 0;
    case OR_Y: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; return 0;
    case OR_Z: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; return 0;
    case OR_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; return 0;
    case OR_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; return 0;
    case OR_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * M_PI / 4); return 0;
    case OR_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(-I * M_PI / 4); return 0;
    case OR_RX: /* exp(-i theta X / 2) */
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; return 0;
    case OR_RY: /* exp(-i theta Y / 2) */
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c; m[1] = -s; m[2] = s; m[3] = c; return 0;
    case OR_RZ: /* exp(-i theta Z / 2) */
        m[0] = cexp(-I * p[0] / 2); m[1] = 0; m[2] = 0; m[3] = cexp(I * p[0] / 2); return 0;
    case OR_P:
        m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * p[0]); return 0;
    case OR_U3: /* U3(theta, phi, lambda), OpenQASM 2 */
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c;
        m[1] = -cexp(I * p[2]) * s;
        m[2] = cexp(I * p[1]) * s;
        m[3] = cexp(I * (p[1] + p[2])) * c;
        return 0;
    case OR_MAT1:
        for (int e = 0; e < 4; e++) m[e] = p[2 * e] + I * p[2 * e + 1];
        return 0;
    default:
        return -1;
    }
}

int or_gate_matrix(const or_gate* g, double* out /* 2*dim*dim */)
{
    cplx m[16];
    int dim = 2;
    if (g->op < OR_CX) {
        if (one_qubit_matrix(g->op, g->p, m)) return -1;
    } else {
        /* 4x4 in the basis m = bit(q0) + 2 bit(q1) */
        dim = 4;
        for (int e = 0; e < 16; e++) m[e] = 0;
        switch (g->op) {
        case OR_CX: /* control q0, target q1: flip bit 1 of m when bit 0 is 1 */
            m[0 * 4 + 0] = 1; m[2 * 4 + 2] = 1; m[1 * 4 + 3] = 1; m[3 * 4 + 1] = 1; break;
        case OR_CZ:
            m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1; break;
        case OR_CP:
            m[0] = 1; m[5] = 1; m[10] = 1; m[15] = cexp(I * g->p[0]); break;
        case OR_SWAP:
            m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[15] = 1; break;
        case OR_MAT2:
            for (int e = 0; e < 16; e++) m[e] = g->p[2 * e] + I * g->p[2 * e + 1];
            break;
        default:
            return -1;
        }
    }
    for (int e = 0; e < dim * dim; e++) { out[2 * e] = creal(m[e]); out[2 * e + 1] = cimag(m[e]); }
    return dim;
}

/* --------------------------------------------------------- application --- */

/* Eq. 5: for every i with bit k = 0 (and every control bit = 1), update the
 * pair (a_i, a_{i^2^k}) by u. */
void or_apply_1q(cplx* a, int n, int k, const cplx u[4], uint64_t ctrl_mask)
{
    const int64_t N = (int64_t)1 << n;
    const uint64_t bit = (uint64_t)1 << k;
    uint64_t count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count)
    for (int64_t i = 0; i < N; i++) {
        if ((uint64_t)i & bit) continue;                      /* visited from its partner */
        if (((uint64_t)i & ctrl_mask) != ctrl_mask) continue;  /* control not satisfied */
        const uint64_t j = (uint64_t)i ^ bit;
        const cplx x = a[i], y = a[j];
        a[i] = u[0] * x + u[1] * y;
        a[j] = u[2] * x + u[3] * y;
        count++;
    }
    pair_updates += count;
}

/* Two-qubit gate: every quadruple with bits a, b of i equal to 0. */
void or_apply_2q(cplx* s, int n, int qa, int qb, const cplx u[16])
{
    const int64_t N = (int64_t)1 << n;
    const uint64_t ba = (uint64_t)1 << qa, bb = (uint64_t)1 << qb;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        if ((uint64_t)i & (ba | bb)) continue;
        const uint64_t idx[4] = {(uint64_t)i, (uint64_t)i | ba, (uint64_t)i | bb, (uint64_t)i | ba | bb};
        cplx v[4], w[4];
        for (int c = 0; c < 4; c++) v[c] = s[idx[c]];
        for (int r = 0; r < 4; r++) {
            w[r] = 0;
            for (int c = 0; c < 4; c++) w[r] += u[4 * r + c] * v[c];
        }
        for (int r = 0; r < 4; r++) s[idx[r]] = w[r];
    }
}

static void conj_transpose(const cplx* m, cplx* out, int dim)
{
    for (int r = 0; r < dim; r++)
        for (int c = 0; c < dim; c++) out[r * dim + c] = conj(m[c * dim + r]);
}

/* Apply one gate (or its inverse when dagger != 0). */
int or_apply_gate(cplx* s, int n, const or_gate* g, int dagger)
{
    double buf[32];
    cplx m[16], md[16];
    const int dim = or_gate_matrix(g, buf);
    if (dim < 0) return -1;
    for (int e = 0; e < dim * dim; e++) m[e] = buf[2 * e] + I * buf[2 * e + 1];
    if (dagger) {
        conj_transpose(m, md, dim);
        memcpy(m, md, sizeof(cplx) * dim * dim);
    }
    if (dim == 2) {
        or_apply_1q(s, n, g->q0, m, 0);
    } else if (g->op == OR_CX) {
        /* X on the target, restricted to control = 1 */
        const cplx x[4] = {0, 1, 1, 0};
        or_apply_1q(s, n, g->q1, x, (uint64_t)1 << g->q0);
    } else {
        or_apply_2q(s, n, g->q0, g->q1, m);
    }
    return 0;
}

int or_run(cplx* s, int n, const or_gate* gates, int n_gates)
{
    for (int l = 0; l < n_gates; l++)
        if (or_apply_gate(s, n, &gates[l], 0)) return -1;
    return 0;
}

int or_run_inverse(cplx* s, int n, const or_gate* gates, int n_gates)
{
    for (int l = n_gates - 1; l >= 0; l--)
        if (or_apply_gate(s, n, &gates[l], 1)) return -1;
    return 0;
}

void or_set_basis(cplx* s, int n, uint64_t x)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) s[i] = 0;
    s[x] = 1;
}

/* ---------------------------------------------------------- reductions --- */

/* Pairwise (cascade) summation of v[0..len): a range of more than 8 terms
 * is the sum of its two halves (the first has len / 2 terms), 8 or fewer
 * are added left to right. */
static double pairwise_rec(const double* v, int64_t len)
{
    if (len <= 8) {
        double t = 0;
        for (int64_t i = 0; i < len; i++) t += v[i];
        return t;
    }
    const int64_t h = len / 2;
    return pairwise_rec(v, h) + pairwise_rec(v + h, len - h);
}

/* The same tree for long ranges, with the 64 subtrees six levels down
 * summed on OpenMP threads and then joined in the tree's own order: every
 * node is still the sum of its two children, so the result is identical to
 * pairwise_rec's. */
double or_pairwise_sum(const double* v, int64_t len)
{
    enum { DEPTH = 6, LEAVES = 1 << DEPTH };
    if (len < ((int64_t)1 << 16)) return pairwise_rec(v, len);
    int64_t off[LEAVES], cnt[LEAVES];
    off[0] = 0;
    cnt[0] = len;
    for (int d = 0; d < DEPTH; d++) {      /* split every node of level d */
        const int nodes = 1 << d;
        for (int k = nodes - 1; k >= 0; k--) {
            const int64_t o = off[k], c = cnt[k], h = c / 2;
            off[2 * k] = o;
            cnt[2 * k] = h;
            off[2 * k + 1] = o + h;
            cnt[2 * k + 1] = c - h;
        }
    }
    double part[LEAVES];
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < LEAVES; k++) part[k] = pairwise_rec(v + off[k], cnt[k]);
    for (int nodes = LEAVES / 2; nodes >= 1; nodes /= 2)   /* join level by level */
        for (int k = 0; k < nodes; k++) part[k] = part[2 * k] + part[2 * k + 1];
    return part[0];
}

/* P|j> for the Pauli string (x_mask, z_mask): i^{#Y} (-1)^{|j & z|} |j ^ x>. */
static cplx pauli_phase(uint64_t j, uint64_t xm, uint64_t zm)
{
    static const cplx ipow[4] = {1, I, -1, -I};
    const int ny = __builtin_popcountll(xm & zm) & 3;
    const int sign = __builtin_popcountll(j & zm) & 1;
    return sign ? -ipow[ny] : ipow[ny];
}

/* <a|P|b> = sum_j conj(a_{j^x}) phase(j) b_j, summed pairwise; complex. */
static cplx pauli_inner(const cplx* a, const cplx* b, int n, uint64_t xm, uint64_t zm, double* tmp_re, double* tmp_im)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; j++) {
        const cplx t = conj(a[(uint64_t)j ^ xm]) * pauli_phase((uint64_t)j, xm, zm) * b[j];
        tmp_re[j] = creal(t);
        tmp_im[j] = cimag(t);
    }
    return or_pairwise_sum(tmp_re, N) + I * or_pairwise_sum(tmp_im, N);
}

/* f = <psi|H|psi> for H = sum_t coeff_t P_t. Returns NAN on allocation failure. */
double or_expect(const cplx* s, int n, int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm)
{
    const int64_t N = (int64_t)1 << n;
    double* re = malloc(sizeof(double) * N);
    double* im = malloc(sizeof(double) * N);
    double* per_term = malloc(sizeof(double) * (n_terms > 0 ? n_terms : 1));
    if (!re || !im || !per_term) { free(re); free(im); free(per_term); return NAN; }
    for (int t = 0; t < n_terms; t++)
        per_term[t] = coeff[t] * creal(pauli_inner(s, s, n, xm[t], zm[t], re, im));
    const double f = or_pairwise_sum(per_term, n_terms);
    free(re); free(im); free(per_term);
    return f;
}

/* out = H s */
int or_apply_pauli_sum(const cplx* s, cplx* out, int n, int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm)
{
    const int64_t N = (int64_t)1 << n;
    for (int64_t i = 0; i < N; i++) out[i] = 0;
    for (int t = 0; t < n_terms; t++) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < N; j++) {
            /* (P s)_{j^x} gets phase(j) s_j */
            out[(uint64_t)j ^ xm[t]] += coeff[t] * pauli_phase((uint64_t)j, xm[t], zm[t]) * s[j];
        }
    }
    return 0;
}

/* ------------------------------------------------------------ gradients --- */

/* Generator G of a trainable gate U = exp(-i theta G / 2) as a Pauli string. */
static int generator(const or_gate* g, uint64_t* xm, uint64_t* zm)
{
    const uint64_t b = (uint64_t)1 << g->q0;
    switch (g->op) {
    case OR_RX: *xm = b; *zm = 0; return 0;
    case OR_RY: *xm = b; *zm = b; return 0;
    case OR_RZ: *xm = 0; *zm = b; return 0;
    default: return -1;
    }
}

/*
 * Adjoint differentiation of f(theta) = <psi|H|psi>, psi = U_L..U_1 |x0>.
 * phi = psi, lam = H psi; for l = L..1:
 *   if U_l = exp(-i theta G / 2) is trainable: d f / d theta += Im <lam|G|phi>
 *   phi <- U_l^dag phi;  lam <- U_l^dag lam.
 * (d/dtheta of U_l is (-i G/2) U_l, and 2 Re <lam|(-i G/2)|phi> = Im <lam|G|phi>.)
 * grad must hold n_params zeros on entry. Returns f, or NAN on failure.
 */
double or_adjoint_grad(int n, uint64_t x0, const or_gate* gates, int n_gates,
                       int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm,
                       double* grad, int n_params)
{
    const int64_t N = (int64_t)1 << n;
    cplx* phi = malloc(sizeof(cplx) * N);
    cplx* lam = malloc(sizeof(cplx) * N);
    double* re = malloc(sizeof(double) * N);
    double* im = malloc(sizeof(double) * N);
    double f = NAN;
    if (!phi || !lam || !re || !im) goto done;
    or_set_basis(phi, n, x0);
    if (or_run(phi, n, gates, n_gates)) goto done;
    or_apply_pauli_sum(phi, lam, n, n_terms, coeff, xm, zm);
    f = creal(pauli_inner(phi, lam, n, 0, 0, re, im));
    for (int l = n_gates - 1; l >= 0; l--) {
        const or_gate* g = &gates[l];
        if (g->param_index >= 0) {
            uint64_t gx, gz;
            if (g->param_index >= n_params || generator(g, &gx, &gz)) { f = NAN; goto done; }
            grad[g->param_index] += cimag(pauli_inner(lam, phi, n, gx, gz, re, im));
        }
        or_apply_gate(phi, n, g, 1);
        or_apply_gate(lam, n, g, 1);
    }
done:
    free(phi); free(lam); free(re); free(im);
    return f;
}

static double circuit_value(cplx* s, int n, uint64_t x0, const or_gate* gates, int n_gates,
                            int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm)
{
    or_set_basis(s, n, x0);
    if (or_run(s, n, gates, n_gates)) return NAN;
    return or_expect(s, n, n_terms, coeff, xm, zm);
}

/*
 * Parameter-shift rule, per gate occurrence: for U = exp(-i theta P / 2) with
 * a Pauli P, d f / d theta = [f(theta + pi/2) - f(theta - pi/2)] / 2 exactly.
 * Only the gates whose index appears in `which` (n_which of them, or all
 * trainable gates when which == NULL) are shifted. grad must be zeroed.
 */
int or_param_shift_grad(int n, uint64_t x0, const or_gate* gates, int n_gates,
                        int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm,
                        double* grad, int n_params, const int32_t* which, int n_which)
{
    const int64_t N = (int64_t)1 << n;
    cplx* s = malloc(sizeof(cplx) * N);
    or_gate* work = malloc(sizeof(or_gate) * (n_gates > 0 ? n_gates : 1));
    if (!s || !work) { free(s); free(work); return -1; }
    memcpy(work, gates, sizeof(or_gate) * n_gates);
    for (int l = 0; l < n_gates; l++) {
        const int p = gates[l].param_index;
        if (p < 0) continue;
        if (p >= n_params) { free(s); free(work); return -1; }
        if (which) {
            int hit = 0;
            for (int w = 0; w < n_which; w++) hit |= (which[w] == p);
            if (!hit) continue;
        }
        const double th = gates[l].p[0];
        work[l].p[0] = th + M_PI / 2;
        const double fp = circuit_value(s, n, x0, work, n_gates, n_terms, coeff, xm, zm);
        work[l].p[0] = th - M_PI / 2;
        const double fm = circuit_value(s, n, x0, work, n_gates, n_terms, coeff, xm, zm);
        work[l].p[0] = th;
        grad[p] += 0.5 * (fp - fm);
    }
    free(s); free(work);
    return 0;
}

/* Central finite differences in each parameter (all occurrences shifted). */
int or_finite_diff_grad(int n, uint64_t x0, const or_gate* gates, int n_gates,
                        int n_terms, const double* coeff, const uint64_t* xm, const uint64_t* zm,
                        double* grad, int n_params, double h, const int32_t* which, int n_which)
{
    const int64_t N = (int64_t)1 << n;
    cplx* s = malloc(sizeof(cplx) * N);
    or_gate* work = malloc(sizeof(or_gate) * (n_gates > 0 ? n_gates : 1));
    if (!s || !work) { free(s); free(work); return -1; }
    const int count = which ? n_which : n_params;
    for (int w = 0; w < count; w++) {
        const int p = which ? which[w] : w;
        if (p < 0 || p >= n_params) { free(s); free(work); return -1; }
        double fpm[2];
        for (int side = 0; side < 2; side++) {
            memcpy(work, gates, sizeof(or_gate) * n_gates);
            for (int l = 0; l < n_gates; l++)
                if (work[l].param_index == p) work[l].p[0] += side == 0 ? h : -h;
            fpm[side] = circuit_value(s, n, x0, work, n_gates, n_terms, coeff, xm, zm);
        }
        grad[p] = (fpm[0] - fpm[1]) / (2 * h);
    }
    free(s); free(work);
    return 0;
}

/* Threads the OpenMP loops use (the CPU-baseline reports it). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int k) { if (k > 0) omp_set_num_threads(k); }
#else
int or_num_threads(void) { return 1; }
void or_set_threads(int k) { (void)k; }
#endif
