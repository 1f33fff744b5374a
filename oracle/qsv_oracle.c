/*
 * qsv_oracle.c -- plain, slow, FP64 CPU oracle for the state-vector hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, header,
 * table or helper with the GPU library; the two meet only through the seeded
 * circuit descriptions produced by the input generators.
 *
 * Every routine is the plain definition from the paper, written out gate by gate
 * in double-precision complex arithmetic (C99 `double complex`), parallelised
 * only by an OpenMP loop over independent amplitude groups:
 *   - state vector and normalisation ............ Eq. 1 (Section 1)
 *   - single-target gate application ............. Eq. 2 (Section 2.1)
 *   - Kronecker-embedded gate action ............. Eq. 3 (Section 2.2), for k targets
 *   - canonical gate set and rotations ........... Eq. 4 (Section 3)
 *   - outcome probabilities ...................... Eq. 1 and Eq. 18 (Section 9.1)
 *   - Pauli-string expectation ................... <psi|P|psi>, P a tensor product of
 *                                                  Pauli matrices (definition)
 * Qubit t is bit t of the amplitude index.  For a k-target gate, bit j of the
 * local (row/column) index belongs to targets[j].
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

#define OR_MAX_K 10

/* ------------------------------------------------------------------ Eq. 1 */
int or_init_zero(cplx* psi, int n)
{
    if (n < 1 || n > 36 || !psi) return -1;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
    return 0;
}

static int targets_ok(int n, int k, const int* t)
{
    if (k < 1 || k > OR_MAX_K || k > n) return 0;
    for (int j = 0; j < k; ++j) {
        if (t[j] < 0 || t[j] >= n) return 0;
        for (int i = 0; i < j; ++i)
            if (t[i] == t[j]) return 0;
    }
    return 1;
}

/* ------------------------------------------------------- Eq. 2 / Eq. 3
 * Apply the dense 2^k x 2^k matrix U (row-major, U[r*d + c]) to the targets.
 * For every index b whose target bits are all clear, the 2^k amplitudes
 * psi[b + off(r)], off(r) = sum_j bit_j(r) * 2^targets[j], form a vector v and
 * are replaced by U v.  For k = 1 this is exactly Eq. 2; in general it is the
 * action of the Kronecker-embedded operator of Eq. 3 on the target subspace.   */
int or_apply(cplx* psi, int n, int k, const int* targets, const cplx* U)
{
    if (!psi || !U || !targets || !targets_ok(n, k, targets)) return -1;
    const int d = 1 << k;
    int64_t off[1 << OR_MAX_K];
    for (int r = 0; r < d; ++r) {
        int64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((r >> j) & 1) o += (int64_t)1 << targets[j];
        off[r] = o;
    }
    /* target positions in ascending order, for inserting zero bits */
    int s[OR_MAX_K];
    for (int j = 0; j < k; ++j) s[j] = targets[j];
    for (int a = 1; a < k; ++a)
        for (int b = a; b > 0 && s[b - 1] > s[b]; --b) {
            int tmp = s[b]; s[b] = s[b - 1]; s[b - 1] = tmp;
        }
    const int64_t G = (int64_t)1 << (n - k);
#pragma omp parallel
    {
        cplx v[1 << OR_MAX_K], w[1 << OR_MAX_K];
#pragma omp for schedule(static)
        for (int64_t g = 0; g < G; ++g) {
            int64_t b = g;
            for (int j = 0; j < k; ++j) {
                const int p = s[j];
                const int64_t low = b & (((int64_t)1 << p) - 1);
                b = ((b >> p) << (p + 1)) | low;
            }
            for (int r = 0; r < d; ++r) v[r] = psi[b + off[r]];
            for (int r = 0; r < d; ++r) {
                cplx acc = 0.0;
                for (int c = 0; c < d; ++c) acc += U[(int64_t)r * d + c] * v[c];
                w[r] = acc;
            }
            for (int r = 0; r < d; ++r) psi[b + off[r]] = w[r];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ Eq. 4
 * Canonical gates.  Rotations R_P(theta) = exp(-i theta P / 2) =
 * cos(theta/2) I - i sin(theta/2) P.  U3 follows the OpenQASM 2 convention
 * [[cos(t/2), -e^{i l} sin(t/2)], [e^{i p} sin(t/2), e^{i(p+l)} cos(t/2)]].
 * Two- and three-qubit gates are written as their action on basis states,
 * local bit 0 = first listed qubit: CNOT(c, t) flips t when c = 1;
 * TOFFOLI(c1, c2, t) flips t when c1 = c2 = 1; SWAP exchanges the two bits;
 * CZ negates |11>.   Returns 0 and sets *k, or -1 for an unknown name.        */
static void set_identity(cplx* U, int d)
{
    for (int i = 0; i < d * d; ++i) U[i] = 0.0;
    for (int i = 0; i < d; ++i) U[i * d + i] = 1.0;
}

int or_gate_matrix(const char* name, const double* p, int* k, cplx* U)
{
    const double r2 = 1.0 / sqrt(2.0);
    if (!strcmp(name, "I")) { *k = 1; set_identity(U, 2); return 0; }
    if (!strcmp(name, "X")) { *k = 1; U[0] = 0; U[1] = 1; U[2] = 1; U[3] = 0; return 0; }
    if (!strcmp(name, "Y")) { *k = 1; U[0] = 0; U[1] = -I; U[2] = I; U[3] = 0; return 0; }
    if (!strcmp(name, "Z")) { *k = 1; U[0] = 1; U[1] = 0; U[2] = 0; U[3] = -1; return 0; }
    if (!strcmp(name, "H")) { *k = 1; U[0] = r2; U[1] = r2; U[2] = r2; U[3] = -r2; return 0; }
    if (!strcmp(name, "S")) { *k = 1; U[0] = 1; U[1] = 0; U[2] = 0; U[3] = I; return 0; }
    if (!strcmp(name, "SDG")) { *k = 1; U[0] = 1; U[1] = 0; U[2] = 0; U[3] = -I; return 0; }
    if (!strcmp(name, "T")) { *k = 1; U[0] = 1; U[1] = 0; U[2] = 0; U[3] = cexp(I * M_PI / 4); return 0; }
    if (!strcmp(name, "TDG")) { *k = 1; U[0] = 1; U[1] = 0; U[2] = 0; U[3] = cexp(-I * M_PI / 4); return 0; }
    if (!strcmp(name, "RX")) {
        const double c = cos(p[0] / 2), s = sin(p[0] / 2);
        *k = 1; U[0] = c; U[1] = -I * s; U[2] = -I * s; U[3] = c; return 0;
    }
    if (!strcmp(name, "RY")) {
        const double c = cos(p[0] / 2), s = sin(p[0] / 2);
        *k = 1; U[0] = c; U[1] = -s; U[2] = s; U[3] = c; return 0;
    }
    if (!strcmp(name, "RZ")) {
        *k = 1; U[0] = cexp(-I * p[0] / 2); U[1] = 0; U[2] = 0; U[3] = cexp(I * p[0] / 2); return 0;
    }
    if (!strcmp(name, "U3")) {
        const double c = cos(p[0] / 2), s = sin(p[0] / 2);
        *k = 1;
        U[0] = c;
        U[1] = -cexp(I * p[2]) * s;
        U[2] = cexp(I * p[1]) * s;
        U[3] = cexp(I * (p[1] + p[2])) * c;
        return 0;
    }
    if (!strcmp(name, "CNOT") || !strcmp(name, "CZ") || !strcmp(name, "SWAP")) {
        *k = 2;
        for (int i = 0; i < 16; ++i) U[i] = 0.0;
        for (int col = 0; col < 4; ++col) {
            const int b0 = col & 1, b1 = (col >> 1) & 1;
            int row = col;
            cplx amp = 1.0;
            if (!strcmp(name, "CNOT") && b0) row = col ^ 2;
            if (!strcmp(name, "CZ") && b0 && b1) amp = -1.0;
            if (!strcmp(name, "SWAP")) row = (b0 << 1) | b1;
            U[row * 4 + col] = amp;
        }
        return 0;
    }
    if (!strcmp(name, "TOFFOLI")) {
        *k = 3;
        for (int i = 0; i < 64; ++i) U[i] = 0.0;
        for (int col = 0; col < 8; ++col) {
            const int row = ((col & 3) == 3) ? (col ^ 4) : col;
            U[row * 8 + col] = 1.0;
        }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------- Eq. 1 normalisation
 * sum_k |alpha_k|^2.  Each thread sums a fixed contiguous block with Neumaier's
 * compensated summation; block sums are combined in block order the same way.  */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum* a, double x)
{
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

#define OR_BLOCKS 256
double or_norm2(const cplx* psi, int n)
{
    const int64_t N = (int64_t)1 << n;
    double part[OR_BLOCKS];
#pragma omp parallel for schedule(static)
    for (int b = 0; b < OR_BLOCKS; ++b) {
        const int64_t lo = N * b / OR_BLOCKS, hi = N * (b + 1) / OR_BLOCKS;
        nsum a = {0.0, 0.0};
        for (int64_t i = lo; i < hi; ++i) {
            const double re = creal(psi[i]), im = cimag(psi[i]);
            nadd(&a, re * re + im * im);
        }
        part[b] = a.s + a.c;
    }
    nsum tot = {0.0, 0.0};
    for (int b = 0; b < OR_BLOCKS; ++b) nadd(&tot, part[b]);
    return tot.s + tot.c;
}

/* --------------------------------------------- outcome probabilities
 * out[o] = sum over k with (bit qubits[j] of k) == (bit j of o) of |alpha_k|^2.
 * m == n with qubits = (0..n-1) gives the full distribution.                   */
int or_probs(const cplx* psi, int n, const int* qubits, int m, double* out)
{
    if (m < 1 || m > n || !psi || !qubits || !out) return -1;
    for (int j = 0; j < m; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return -1;
        for (int i = 0; i < j; ++i) if (qubits[i] == qubits[j]) return -1;
    }
    const int64_t N = (int64_t)1 << n, M = (int64_t)1 << m;
    nsum* acc = (nsum*)calloc((size_t)M, sizeof(nsum));
    if (!acc) return -1;
    for (int64_t k = 0; k < N; ++k) {
        int64_t o = 0;
        for (int j = 0; j < m; ++j) o |= ((k >> qubits[j]) & 1) << j;
        const double re = creal(psi[k]), im = cimag(psi[k]);
        nadd(&acc[o], re * re + im * im);
    }
    for (int64_t o = 0; o < M; ++o) out[o] = acc[o].s + acc[o].c;
    free(acc);
    return 0;
}

/* ------------------------------------------------ Pauli-string expectation
 * P = prod_j sigma_{paulis[j]}(qubits[j]).  Acting on a basis state,
 *   X|b> = |1-b>,  Z|b> = (-1)^b |b>,  Y|b> = i (-1)^b |1-b>,
 * so P|k> = i^{nY} (-1)^{popcount(k & zy)} |k xor xy>, with xy the X/Y positions
 * and zy the Z/Y positions.  Hence
 *   <psi|P|psi> = sum_k conj(psi[k xor xy]) * i^{nY} * (-1)^{popcount(k & zy)} * psi[k].
 * Writes the real and imaginary parts (the latter ~0 for a normalised psi).     */
int or_pauli_expval(const cplx* psi, int n, int nq, const int* qubits, const char* paulis,
                    double* re_out, double* im_out)
{
    int64_t xy = 0, zy = 0;
    int ny = 0;
    for (int j = 0; j < nq; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return -1;
        const int64_t bit = (int64_t)1 << qubits[j];
        if ((xy | zy) & bit) return -1;           /* repeated qubit */
        switch (paulis[j]) {
        case 'I': break;
        case 'X': xy |= bit; break;
        case 'Y': xy |= bit; zy |= bit; ++ny; break;
        case 'Z': zy |= bit; break;
        default: return -1;
        }
    }
    cplx iny = 1.0;
    for (int j = 0; j < ny; ++j) iny *= I;
    const int64_t N = (int64_t)1 << n;
    double pre[OR_BLOCKS], pim[OR_BLOCKS];
#pragma omp parallel for schedule(static)
    for (int b = 0; b < OR_BLOCKS; ++b) {
        const int64_t lo = N * b / OR_BLOCKS, hi = N * (b + 1) / OR_BLOCKS;
        nsum ar = {0.0, 0.0}, ai = {0.0, 0.0};
        for (int64_t k = lo; k < hi; ++k) {
            const double sign = (__builtin_popcountll((uint64_t)(k & zy)) & 1) ? -1.0 : 1.0;
            const cplx term = conj(psi[k ^ xy]) * iny * sign * psi[k];
            nadd(&ar, creal(term));
            nadd(&ai, cimag(term));
        }
        pre[b] = ar.s + ar.c;
        pim[b] = ai.s + ai.c;
    }
    nsum tr = {0.0, 0.0}, ti = {0.0, 0.0};
    for (int b = 0; b < OR_BLOCKS; ++b) { nadd(&tr, pre[b]); nadd(&ti, pim[b]); }
    *re_out = tr.s + tr.c;
    *im_out = ti.s + ti.c;
    return 0;
}

/* <a|b> = sum_k conj(a_k) b_k, combined like or_norm2 (used for the fidelity
 * |<psi_ref|psi>|^2 of the paper's Table 3).                                     */
void or_inner(const cplx* a, const cplx* b, int n, double* re_out, double* im_out)
{
    const int64_t N = (int64_t)1 << n;
    double pre[OR_BLOCKS], pim[OR_BLOCKS];
#pragma omp parallel for schedule(static)
    for (int blk = 0; blk < OR_BLOCKS; ++blk) {
        const int64_t lo = N * blk / OR_BLOCKS, hi = N * (blk + 1) / OR_BLOCKS;
        nsum ar = {0.0, 0.0}, ai = {0.0, 0.0};
        for (int64_t k = lo; k < hi; ++k) {
            const cplx t = conj(a[k]) * b[k];
            nadd(&ar, creal(t));
            nadd(&ai, cimag(t));
        }
        pre[blk] = ar.s + ar.c;
        pim[blk] = ai.s + ai.c;
    }
    nsum tr = {0.0, 0.0}, ti = {0.0, 0.0};
    for (int blk = 0; blk < OR_BLOCKS; ++blk) { nadd(&tr, pre[blk]); nadd(&ti, pim[blk]); }
    *re_out = tr.s + tr.c;
    *im_out = ti.s + ti.c;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
