/*
 * CPU reference ("oracle") for variational-circuit expectation values.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no source with the GPU library: it builds its own gate matrices from their
 * definitions and applies one gate at a time to a dense complex128 vector.
 *
 * What it computes (paper, Sec. 1 and Sec. 3): a circuit of gate tensors
 * acting on the state |0...0>, and the expectation value <psi|H|psi> of an
 * operator H given in factorized form (a weighted sum of Pauli strings, never
 * a dense 2^n x 2^n matrix), plus the gradient of that expectation value with
 * respect to the circuit parameters (Sec. 3, forward value and full gradient
 * of a transverse-field Ising Hamiltonian).  The "causality-simplified
 * contraction" named as future work in Sec. 4 is realised as light cones:
 * each term is evaluated on the sub-circuit that can influence it.
 *
 * Readings of points the paper leaves open (all listed with the design notes):
 *   - qubit q is bit q of the amplitude index;
 *   - RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2);
 *   - CZ = diag(1,1,1,-1); CNOT(q0=control, q1=target) flips the target when
 *     the control is 1; a two-qubit matrix acts on j = 2*bit(q0) + bit(q1);
 *   - U1 is a caller-given 2x2 matrix (row-major);
 *   - Pauli action: X|b> = |1-b>, Y|b> = i(-1)^b |1-b>, Z|b> = (-1)^b |b>;
 *   - light cone of a term: start from the term's qubits, walk the gates
 *     backwards, and add both qubits of every two-qubit gate that touches the
 *     set; a gate is in the cone if it touches the set at its time.
 *
 * The pin of each entry point is listed in this package's __init__.py.
 *
 * Gate-kind codes are the shared interchange format: RX=0 RY=1 RZ=2 CZ=3
 * CNOT=4 U1=5.  Return codes: 0 ok, -1 invalid input, -2 out of memory.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { K_RX = 0, K_RY = 1, K_RZ = 2, K_CZ = 3, K_CNOT = 4, K_U1 = 5 };

#define OK 0
#define EINVAL_ (-1)
#define ENOMEM_ (-2)

/* ------------------------------------------------------------------------ */
/* gate matrices, built from their definitions                               */
/* ------------------------------------------------------------------------ */

/* exp(-i t P / 2) = cos(t/2) I - i sin(t/2) P for a Pauli P. */
static void rotation_matrix(int kind, double t, cplx u[2][2]) {
    const double c = cos(0.5 * t), s = sin(0.5 * t);
    /* Pauli matrices */
    const cplx X[2][2] = {{0, 1}, {1, 0}};
    const cplx Y[2][2] = {{0, -I}, {I, 0}};
    const cplx Z[2][2] = {{1, 0}, {0, -1}};
    const cplx(*P)[2] = kind == K_RX ? X : kind == K_RY ? Y : Z;
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 2; ++k) u[r][k] = (r == k ? c : 0.0) - I * s * P[r][k];
}

static void two_qubit_matrix(int kind, cplx u[4][4]) {
    memset(u, 0, sizeof(cplx) * 16);
    if (kind == K_CZ) {
        u[0][0] = 1; u[1][1] = 1; u[2][2] = 1; u[3][3] = -1;
    } else { /* CNOT, control = first qubit (high bit of j), target = second */
        u[0][0] = 1; u[1][1] = 1; u[2][3] = 1; u[3][2] = 1;
    }
}

/* ------------------------------------------------------------------------ */
/* gate application on a dense vector                                        */
/* ------------------------------------------------------------------------ */

static void apply_1q(int n, cplx* psi, int q, cplx u[2][2]) {
    const int64_t N = (int64_t)1 << n;
    const int64_t bit = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if (x & bit) continue;
        const cplx a = psi[x], b = psi[x | bit];
        psi[x] = u[0][0] * a + u[0][1] * b;
        psi[x | bit] = u[1][0] * a + u[1][1] * b;
    }
}

static void apply_2q(int n, cplx* psi, int qa, int qb, cplx u[4][4]) {
    const int64_t N = (int64_t)1 << n;
    const int64_t ba = (int64_t)1 << qa, bb = (int64_t)1 << qb;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        if ((x & ba) || (x & bb)) continue;
        int64_t idx[4];
        cplx v[4];
        for (int j = 0; j < 4; ++j) {
            idx[j] = x | ((j & 2) ? ba : 0) | ((j & 1) ? bb : 0);
            v[j] = psi[idx[j]];
        }
        for (int r = 0; r < 4; ++r) {
            cplx acc = 0;
            for (int j = 0; j < 4; ++j) acc += u[r][j] * v[j];
            psi[idx[r]] = acc;
        }
    }
}

typedef struct {
    int n, n_gates;
    const uint8_t* kind;
    const int32_t* q0;
    const int32_t* q1;
    const int32_t* param;
    const double* angle;
    const double* mat; /* [n_gates*8] re,im interleaved, row-major 2x2 (U1 only); may be NULL */
} circuit_t;

/* max_n bounds n for the dense entry points; light-cone entry points allow wide circuits. */
static int check_circuit(const circuit_t* c, int n_params, int max_n) {
    if (c->n < 1 || c->n > max_n || c->n_gates < 0) return EINVAL_;
    for (int g = 0; g < c->n_gates; ++g) {
        const int k = c->kind[g];
        if (c->q0[g] < 0 || c->q0[g] >= c->n) return EINVAL_;
        if (k == K_CZ || k == K_CNOT) {
            if (c->q1[g] < 0 || c->q1[g] >= c->n || c->q1[g] == c->q0[g]) return EINVAL_;
        } else if (k == K_RX || k == K_RY || k == K_RZ) {
            if (c->param[g] >= n_params) return EINVAL_;
        } else if (k == K_U1) {
            if (!c->mat) return EINVAL_;
        } else {
            return EINVAL_;
        }
    }
    return OK;
}

/* Angle of gate g: theta[param] when parameterised, else the fixed angle.
 * shift_gate/shift add a displacement to one gate occurrence (parameter shift). */
static double gate_angle(const circuit_t* c, const double* theta, int g, int shift_gate, double shift) {
    double t = c->param[g] >= 0 ? theta[c->param[g]] : c->angle[g];
    if (g == shift_gate) t += shift;
    return t;
}

static void run_gates(const circuit_t* c, const double* theta, int shift_gate, double shift, cplx* psi) {
    const int64_t N = (int64_t)1 << c->n;
    memset(psi, 0, sizeof(cplx) * (size_t)N);
    psi[0] = 1.0;
    for (int g = 0; g < c->n_gates; ++g) {
        const int k = c->kind[g];
        if (k == K_RX || k == K_RY || k == K_RZ) {
            cplx u[2][2];
            rotation_matrix(k, gate_angle(c, theta, g, shift_gate, shift), u);
            apply_1q(c->n, psi, c->q0[g], u);
        } else if (k == K_U1) {
            cplx u[2][2];
            for (int r = 0; r < 2; ++r)
                for (int j = 0; j < 2; ++j)
                    u[r][j] = c->mat[g * 8 + (r * 2 + j) * 2] + I * c->mat[g * 8 + (r * 2 + j) * 2 + 1];
            apply_1q(c->n, psi, c->q0[g], u);
        } else {
            cplx u[4][4];
            two_qubit_matrix(k, u);
            apply_2q(c->n, psi, c->q0[g], c->q1[g], u);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pauli-string expectation values                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n_terms;
    const double* coeff;
    const int32_t* term_off;
    const int32_t* qubits;
    const uint8_t* paulis;
} hamiltonian_t;

static int check_hamiltonian(const hamiltonian_t* h, int n) {
    if (h->n_terms < 0) return EINVAL_;
    for (int t = 0; t < h->n_terms; ++t) {
        const int a = h->term_off[t], b = h->term_off[t + 1];
        if (b < a) return EINVAL_;
        for (int k = a; k < b; ++k) {
            const int q = h->qubits[k], p = h->paulis[k];
            if (q < 0 || q >= n) return EINVAL_;
            if (p != 'X' && p != 'Y' && p != 'Z') return EINVAL_;
            for (int k2 = a; k2 < k; ++k2)
                if (h->qubits[k2] == q) return EINVAL_;
        }
    }
    return OK;
}

/* <psi| P |psi> for one Pauli string, as sum_y conj(psi[z(y)]) * k(y) * psi[y],
 * where P|y> = k(y) |z(y)> is built factor by factor from the single-qubit
 * actions.  Summed in fixed chunks (each chunk in long double, chunks added in
 * index order) so the result does not depend on the thread count. */
#define CHUNK ((int64_t)1 << 14)
static cplx pauli_expect(int n, const cplx* psi, int len, const int32_t* qs, const uint8_t* ps) {
    const int64_t N = (int64_t)1 << n;
    const int64_t n_chunks = (N + CHUNK - 1) / CHUNK;
    long double* pr = (long double*)malloc(sizeof(long double) * (size_t)n_chunks);
    long double* pi = (long double*)malloc(sizeof(long double) * (size_t)n_chunks);
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        long double sr = 0, si = 0;
        const int64_t end = (ch + 1) * CHUNK < N ? (ch + 1) * CHUNK : N;
        for (int64_t y = ch * CHUNK; y < end; ++y) {
            int64_t z = y;
            cplx k = 1.0;
            for (int j = 0; j < len; ++j) {
                const int q = qs[j];
                const int b = (int)((y >> q) & 1);
                if (ps[j] == 'X') {
                    z ^= (int64_t)1 << q;
                } else if (ps[j] == 'Y') {
                    z ^= (int64_t)1 << q;
                    k *= b ? -I : I;
                } else {
                    k *= b ? -1.0 : 1.0;
                }
            }
            const cplx term = conj(psi[z]) * k * psi[y];
            sr += creal(term);
            si += cimag(term);
        }
        pr[ch] = sr;
        pi[ch] = si;
    }
    long double sr = 0, si = 0;
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        sr += pr[ch];
        si += pi[ch];
    }
    free(pr);
    free(pi);
    return (double)sr + I * (double)si;
}

/* Per-term values <P_t> (real and imaginary parts) and the weighted total. */
static void hamiltonian_expect(int n, const cplx* psi, const hamiltonian_t* h, double* term_re, double* term_im,
                               double* total) {
    long double acc = 0;
    for (int t = 0; t < h->n_terms; ++t) {
        const int a = h->term_off[t], b = h->term_off[t + 1];
        const cplx v = pauli_expect(n, psi, b - a, h->qubits + a, h->paulis + a);
        if (term_re) term_re[t] = creal(v);
        if (term_im) term_im[t] = cimag(v);
        acc += (long double)h->coeff[t] * (long double)creal(v);
    }
    *total = (double)acc;
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                     */
/* ------------------------------------------------------------------------ */

#define CIRCUIT_ARGS                                                                                 \
    int n, int n_gates, const uint8_t *kind, const int32_t *q0, const int32_t *q1, const int32_t *param, \
        const double *angle, const double *mat, int n_params
#define CIRCUIT_INIT {n, n_gates, kind, q0, q1, param, angle, mat}
#define HAM_ARGS \
    int n_terms, const double *coeff, const int32_t *term_off, const int32_t *qubits, const uint8_t *paulis
#define HAM_INIT {n_terms, coeff, term_off, qubits, paulis}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Final state |psi(theta)> = U_G ... U_1 |0...0>, written as 2^n (re, im) pairs. */
int oracle_statevector(CIRCUIT_ARGS, const double* theta, double* psi_out) {
    const circuit_t c = CIRCUIT_INIT;
    if (check_circuit(&c, n_params, 40) != OK) return EINVAL_;
    run_gates(&c, theta, -1, 0.0, (cplx*)psi_out);
    return OK;
}

/* <psi|H|psi> for a given state; per-term <P_t> (may be NULL). */
int oracle_expect_state(int n, const double* psi, HAM_ARGS, double* term_re, double* term_im, double* total) {
    const hamiltonian_t h = HAM_INIT;
    if (n < 1 || n > 40 || check_hamiltonian(&h, n) != OK) return EINVAL_;
    hamiltonian_expect(n, (const cplx*)psi, &h, term_re, term_im, total);
    return OK;
}

static int expect_shifted(const circuit_t* c, const double* theta, int shift_gate, double shift, const hamiltonian_t* h,
                          cplx* work, double* out) {
    run_gates(c, theta, shift_gate, shift, work);
    hamiltonian_expect(c->n, work, h, NULL, NULL, out);
    return OK;
}

/* <psi(theta)|H|psi(theta)> by the dense state vector; theta is [batch, n_params]. */
int oracle_expect(CIRCUIT_ARGS, HAM_ARGS, const double* theta, int batch, double* out) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 40) != OK || check_hamiltonian(&h, n) != OK || batch < 1) return EINVAL_;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << n));
    if (!psi) return ENOMEM_;
    for (int b = 0; b < batch; ++b) expect_shifted(&c, theta + (size_t)b * n_params, -1, 0.0, &h, psi, out + b);
    free(psi);
    return OK;
}

/* Gradient by the parameter-shift rule, gate occurrence by gate occurrence:
 * for a rotation exp(-i t P/2), dE/dt = [E(t + pi/2) - E(t - pi/2)] / 2, and a
 * parameter used by several gates collects the sum over its occurrences. */
int oracle_grad_psr(CIRCUIT_ARGS, HAM_ARGS, const double* theta, double* grad) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 40) != OK || check_hamiltonian(&h, n) != OK) return EINVAL_;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << n));
    if (!psi) return ENOMEM_;
    for (int j = 0; j < n_params; ++j) grad[j] = 0.0;
    for (int g = 0; g < n_gates; ++g) {
        if (param[g] < 0 || !(kind[g] == K_RX || kind[g] == K_RY || kind[g] == K_RZ)) continue;
        double ep, em;
        expect_shifted(&c, theta, g, +M_PI / 2, &h, psi, &ep);
        expect_shifted(&c, theta, g, -M_PI / 2, &h, psi, &em);
        grad[param[g]] += 0.5 * (ep - em);
    }
    free(psi);
    return OK;
}

/* Parameter-shift derivative for a subset of parameters only (idx[k] in [0, n_params)). */
int oracle_grad_psr_subset(CIRCUIT_ARGS, HAM_ARGS, const double* theta, int n_idx, const int32_t* idx, double* grad) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 40) != OK || check_hamiltonian(&h, n) != OK) return EINVAL_;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << n));
    if (!psi) return ENOMEM_;
    for (int k = 0; k < n_idx; ++k) {
        grad[k] = 0.0;
        for (int g = 0; g < n_gates; ++g) {
            if (param[g] != idx[k]) continue;
            double ep, em;
            expect_shifted(&c, theta, g, +M_PI / 2, &h, psi, &ep);
            expect_shifted(&c, theta, g, -M_PI / 2, &h, psi, &em);
            grad[k] += 0.5 * (ep - em);
        }
    }
    free(psi);
    return OK;
}

/* Central finite difference [E(theta + h e_j) - E(theta - h e_j)] / (2h) for listed parameters. */
int oracle_grad_fd(CIRCUIT_ARGS, HAM_ARGS, const double* theta, double step, int n_idx, const int32_t* idx,
                   double* grad) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 40) != OK || check_hamiltonian(&h, n) != OK || step == 0.0) return EINVAL_;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << n));
    double* th = (double*)malloc(sizeof(double) * (size_t)(n_params > 0 ? n_params : 1));
    if (!psi || !th) {
        free(psi);
        free(th);
        return ENOMEM_;
    }
    for (int k = 0; k < n_idx; ++k) {
        double ep, em;
        memcpy(th, theta, sizeof(double) * (size_t)n_params);
        th[idx[k]] = theta[idx[k]] + step;
        expect_shifted(&c, th, -1, 0.0, &h, psi, &ep);
        th[idx[k]] = theta[idx[k]] - step;
        expect_shifted(&c, th, -1, 0.0, &h, psi, &em);
        grad[k] = (ep - em) / (2.0 * step);
    }
    free(psi);
    free(th);
    return OK;
}

/* ------------------------------------------------------------------------ */
/* light cones                                                               */
/* ------------------------------------------------------------------------ */

/* Backward closure for one term: in_set[q] = 1 for the cone's qubits, in_cone[g] = 1
 * for the gates that touch the set at their time. */
static void light_cone(const circuit_t* c, int len, const int32_t* qs, uint8_t* in_set, uint8_t* in_cone) {
    memset(in_set, 0, (size_t)c->n);
    for (int j = 0; j < len; ++j) in_set[qs[j]] = 1;
    for (int g = c->n_gates - 1; g >= 0; --g) {
        const int k = c->kind[g];
        in_cone[g] = 0;
        if (k == K_CZ || k == K_CNOT) {
            if (in_set[c->q0[g]] || in_set[c->q1[g]]) {
                in_set[c->q0[g]] = 1;
                in_set[c->q1[g]] = 1;
                in_cone[g] = 1;
            }
        } else if (in_set[c->q0[g]]) {
            in_cone[g] = 1;
        }
    }
}

/* Canonical light-cone qubit sets, ascending, term by term: set t is
 * set_qubits[set_off[t] .. set_off[t+1]).  cap bounds the total entries;
 * returns -3 when it would be exceeded. */
int oracle_lightcone_sets(CIRCUIT_ARGS, HAM_ARGS, int32_t* set_off, int32_t* set_qubits, int cap) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 1 << 24) != OK || check_hamiltonian(&h, n) != OK) return EINVAL_;
    uint8_t* in_set = (uint8_t*)malloc((size_t)n);
    uint8_t* in_cone = (uint8_t*)malloc((size_t)(n_gates > 0 ? n_gates : 1));
    int pos = 0;
    set_off[0] = 0;
    for (int t = 0; t < n_terms; ++t) {
        light_cone(&c, term_off[t + 1] - term_off[t], qubits + term_off[t], in_set, in_cone);
        for (int q = 0; q < n; ++q) {
            if (!in_set[q]) continue;
            if (pos >= cap) {
                free(in_set);
                free(in_cone);
                return -3;
            }
            set_qubits[pos++] = q;
        }
        set_off[t + 1] = pos;
    }
    free(in_set);
    free(in_cone);
    return OK;
}

/* <H> term by term, each term on its own light cone with the dense simulator:
 * the cone's qubits are relabelled 0..s-1 in ascending order, the in-cone
 * gates are kept in their original order, and <P_t> is evaluated there.
 * term_vals[t] = <P_t> (without the coefficient); max_cone bounds s. */
int oracle_expect_lightcone(CIRCUIT_ARGS, HAM_ARGS, const double* theta, int max_cone, double* term_vals,
                            double* total) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 1 << 24) != OK || check_hamiltonian(&h, n) != OK) return EINVAL_;
    uint8_t* in_set = (uint8_t*)malloc((size_t)n);
    uint8_t* in_cone = (uint8_t*)malloc((size_t)(n_gates > 0 ? n_gates : 1));
    int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* sk = (uint8_t*)malloc((size_t)(n_gates > 0 ? n_gates : 1));
    int32_t* sq0 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_gates > 0 ? n_gates : 1));
    int32_t* sq1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_gates > 0 ? n_gates : 1));
    int32_t* sp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_gates > 0 ? n_gates : 1));
    double* sa = (double*)malloc(sizeof(double) * (size_t)(n_gates > 0 ? n_gates : 1));
    double* sm = (double*)malloc(sizeof(double) * 8 * (size_t)(n_gates > 0 ? n_gates : 1));
    int32_t tq[64];
    int rc = OK;
    long double acc = 0;
    for (int t = 0; t < n_terms && rc == OK; ++t) {
        const int a = term_off[t], b = term_off[t + 1];
        light_cone(&c, b - a, qubits + a, in_set, in_cone);
        int s = 0;
        for (int q = 0; q < n; ++q) label[q] = in_set[q] ? s++ : -1;
        if (s > max_cone || b - a > 64) {
            rc = -3;
            break;
        }
        if (s == 0) { /* identity term */
            if (term_vals) term_vals[t] = 1.0;
            acc += (long double)coeff[t];
            continue;
        }
        int sg = 0;
        for (int g = 0; g < n_gates; ++g) {
            if (!in_cone[g]) continue;
            sk[sg] = kind[g];
            sq0[sg] = label[q0[g]];
            sq1[sg] = (kind[g] == K_CZ || kind[g] == K_CNOT) ? label[q1[g]] : -1;
            sp[sg] = param[g];
            sa[sg] = angle[g];
            if (mat) memcpy(sm + 8 * (size_t)sg, mat + 8 * (size_t)g, sizeof(double) * 8);
            else memset(sm + 8 * (size_t)sg, 0, sizeof(double) * 8);
            ++sg;
        }
        for (int k = a; k < b; ++k) tq[k - a] = label[qubits[k]];
        const circuit_t sub = {s, sg, sk, sq0, sq1, sp, sa, sm};
        cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << s));
        if (!psi) {
            rc = ENOMEM_;
            break;
        }
        run_gates(&sub, theta, -1, 0.0, psi);
        const cplx v = pauli_expect(s, psi, b - a, tq, paulis + a);
        free(psi);
        if (term_vals) term_vals[t] = creal(v);
        acc += (long double)coeff[t] * (long double)creal(v);
    }
    if (rc == OK) *total = (double)acc;
    free(in_set);
    free(in_cone);
    free(label);
    free(sk);
    free(sq0);
    free(sq1);
    free(sp);
    free(sa);
    free(sm);
    return rc;
}

/* Parameter-shift gradient with every term evaluated on its canonical light
 * cone (Sec. 3's full gradient of <H>; Sec. 4's causality-based contraction).
 * A gate outside a term's cone cannot change that term, so for each listed
 * parameter idx[k] and every gate g that uses it, only the terms whose cone
 * contains g are re-evaluated, on their cones, with g's angle shifted by
 * +-pi/2: grad[k] = sum of c_t (<P_t>(+) - <P_t>(-)) / 2.  max_cone bounds the
 * cone size. */
int oracle_grad_psr_lightcone(CIRCUIT_ARGS, HAM_ARGS, const double* theta, int max_cone, int n_idx,
                              const int32_t* idx, double* grad) {
    const circuit_t c = CIRCUIT_INIT;
    const hamiltonian_t h = HAM_INIT;
    if (check_circuit(&c, n_params, 1 << 24) != OK || check_hamiltonian(&h, n) != OK) return EINVAL_;
    for (int k = 0; k < n_idx; ++k) {
        if (idx[k] < 0 || idx[k] >= n_params) return EINVAL_;
        grad[k] = 0.0;
    }
    const size_t ng = (size_t)(n_gates > 0 ? n_gates : 1);
    uint8_t* in_set = (uint8_t*)malloc((size_t)n);
    uint8_t* in_cone = (uint8_t*)malloc(ng);
    int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* sk = (uint8_t*)malloc(ng);
    int32_t* sq0 = (int32_t*)malloc(sizeof(int32_t) * ng);
    int32_t* sq1 = (int32_t*)malloc(sizeof(int32_t) * ng);
    int32_t* sp = (int32_t*)malloc(sizeof(int32_t) * ng);
    double* sa = (double*)malloc(sizeof(double) * ng);
    double* sm = (double*)malloc(sizeof(double) * 8 * ng);
    int32_t tq[64];
    int rc = OK;
    for (int t = 0; t < n_terms && rc == OK; ++t) {
        const int a = term_off[t], b = term_off[t + 1];
        if (b == a) continue; /* identity: no dependence on the parameters */
        light_cone(&c, b - a, qubits + a, in_set, in_cone);
        int s = 0;
        for (int q = 0; q < n; ++q) label[q] = in_set[q] ? s++ : -1;
        if (s > max_cone || b - a > 64) {
            rc = -3;
            break;
        }
        int sg = 0;
        for (int g = 0; g < n_gates; ++g) {
            if (!in_cone[g]) continue;
            sk[sg] = kind[g];
            sq0[sg] = label[q0[g]];
            sq1[sg] = (kind[g] == K_CZ || kind[g] == K_CNOT) ? label[q1[g]] : -1;
            sp[sg] = param[g];
            sa[sg] = angle[g];
            if (mat) memcpy(sm + 8 * (size_t)sg, mat + 8 * (size_t)g, sizeof(double) * 8);
            else memset(sm + 8 * (size_t)sg, 0, sizeof(double) * 8);
            ++sg;
        }
        for (int k = a; k < b; ++k) tq[k - a] = label[qubits[k]];
        const circuit_t sub = {s, sg, sk, sq0, sq1, sp, sa, sm};
        cplx* psi = (cplx*)malloc(sizeof(cplx) * ((size_t)1 << s));
        if (!psi) {
            rc = ENOMEM_;
            break;
        }
        for (int g = 0; g < sg; ++g) {
            if (sp[g] < 0 || !(sk[g] == K_RX || sk[g] == K_RY || sk[g] == K_RZ)) continue;
            for (int k = 0; k < n_idx; ++k) {
                if (idx[k] != sp[g]) continue;
                run_gates(&sub, theta, g, +M_PI / 2, psi);
                const double ep = creal(pauli_expect(s, psi, b - a, tq, paulis + a));
                run_gates(&sub, theta, g, -M_PI / 2, psi);
                const double em = creal(pauli_expect(s, psi, b - a, tq, paulis + a));
                grad[k] += coeff[t] * 0.5 * (ep - em);
            }
        }
        free(psi);
    }
    free(in_set);
    free(in_cone);
    free(label);
    free(sk);
    free(sq0);
    free(sq1);
    free(sp);
    free(sa);
    free(sm);
    return rc;
}
