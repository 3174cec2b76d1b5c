/*
 * Plain FP64 CPU oracle for the state-vector gate engine.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. The GPU product path never links, imports or calls it.
 *
 * What it computes (De Raedt et al., "Massive Parallel Quantum Computer Simulator"):
 *   - the state of L qubits is 2^L complex amplitudes a(x_{L-1}...x_0); qubit 0 is the least
 *     significant bit of the index (Sec. II.A, Eq. STAT2);
 *   - every gate is an in-place update of pairs of amplitudes whose indices differ only in the
 *     target bit (Sec. III.A, Eqs. NUM2-NUM8).
 * Storage: interleaved (re, im) doubles, amplitude i at a[2i], a[2i+1].
 * Each loop visits every index once, in increasing order; no blocking, no fusion, no reordering.
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add), optional OpenMP over the index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops use (1 without OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define BIT(i, q) (((i) >> (q)) & 1ULL)

/* Eq. NUM2: Hadamard on qubit j. a'(..0_j..) = (a(..0_j..) + a(..1_j..))/sqrt2,
 *                                 a'(..1_j..) = (a(..0_j..) - a(..1_j..))/sqrt2. */
void or_hadamard(double *a, int L, int j)
{
    const int64_t D = (int64_t)1 << L;
    const double s = 1.0 / sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, j)) continue;
        int64_t k = i | ((int64_t)1 << j);
        double x0r = a[2 * i], x0i = a[2 * i + 1], x1r = a[2 * k], x1i = a[2 * k + 1];
        a[2 * i] = s * (x0r + x1r);
        a[2 * i + 1] = s * (x0i + x1i);
        a[2 * k] = s * (x0r - x1r);
        a[2 * k + 1] = s * (x0i - x1i);
    }
}

/* Eq. NUM3: the paper's X = exp(i pi S^x / 2) on qubit j.
 *   a'(..0_j..) = (a(..0_j..) + i a(..1_j..))/sqrt2,  a'(..1_j..) = (a(..1_j..) + i a(..0_j..))/sqrt2.
 * inverse != 0 applies the conjugate transpose (i -> -i), the paper's X-bar. */
void or_xrot(double *a, int L, int j, int inverse)
{
    const int64_t D = (int64_t)1 << L;
    const double s = 1.0 / sqrt(2.0);
    const double g = inverse ? -1.0 : 1.0; /* coefficient of i */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, j)) continue;
        int64_t k = i | ((int64_t)1 << j);
        double x0r = a[2 * i], x0i = a[2 * i + 1], x1r = a[2 * k], x1i = a[2 * k + 1];
        /* i * (xr + i xi) = -xi + i xr */
        a[2 * i] = s * (x0r - g * x1i);
        a[2 * i + 1] = s * (x0i + g * x1r);
        a[2 * k] = s * (x1r - g * x0i);
        a[2 * k + 1] = s * (x1i + g * x0r);
    }
}

/* Eq. NUM4: the paper's Y = exp(i pi S^y / 2) on qubit j.
 *   a'(..0_j..) = (a(..0_j..) + a(..1_j..))/sqrt2,  a'(..1_j..) = (a(..1_j..) - a(..0_j..))/sqrt2.
 * inverse != 0 applies the transpose (the matrix is real), the paper's Y-bar. */
void or_yrot(double *a, int L, int j, int inverse)
{
    const int64_t D = (int64_t)1 << L;
    const double s = 1.0 / sqrt(2.0);
    const double g = inverse ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, j)) continue;
        int64_t k = i | ((int64_t)1 << j);
        double x0r = a[2 * i], x0i = a[2 * i + 1], x1r = a[2 * k], x1i = a[2 * k + 1];
        a[2 * i] = s * (x0r + g * x1r);
        a[2 * i + 1] = s * (x0i + g * x1i);
        a[2 * k] = s * (x1r - g * x0r);
        a[2 * k + 1] = s * (x1i - g * x0i);
    }
}

/* Eq. NUM5 (phase shift R(phi) on qubit j) and Eq. COMM5 (controlled phase shift): amplitudes whose
 * bit j is 1 and whose control bits (cmask) are all 1 are multiplied by e^{i phi}; all others are
 * left unchanged. */
void or_phase(double *a, int L, int j, uint64_t cmask, double phi)
{
    const int64_t D = (int64_t)1 << L;
    const double c = cos(phi), s = sin(phi);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (!BIT(i, j) || (((uint64_t)i & cmask) != cmask)) continue;
        double xr = a[2 * i], xi = a[2 * i + 1];
        a[2 * i] = c * xr - s * xi;
        a[2 * i + 1] = c * xi + s * xr;
    }
}

/* Eq. NUM6 (CNOT, one control) and Eq. NUM8 (Toffoli, two controls): for every index whose control
 * bits are all 1 and whose target bit k is 0, swap its amplitude with that of the index with bit k
 * set. No arithmetic. cmask == 0 gives the plain bit flip (Pauli X). */
void or_cnot(double *a, int L, uint64_t cmask, int k)
{
    const int64_t D = (int64_t)1 << L;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, k) || (((uint64_t)i & cmask) != cmask)) continue;
        int64_t m = i | ((int64_t)1 << k);
        double tr = a[2 * i], ti = a[2 * i + 1];
        a[2 * i] = a[2 * m];
        a[2 * i + 1] = a[2 * m + 1];
        a[2 * m] = tr;
        a[2 * m + 1] = ti;
    }
}

/* Eq. NUM7: controlled-V(phi), V = (1/2)[[1+e^{i phi}, 1-e^{i phi}], [1-e^{i phi}, 1+e^{i phi}]],
 * applied to target k on the indices whose control bits (cmask) are 1. */
void or_cv(double *a, int L, uint64_t cmask, int k, double phi)
{
    const int64_t D = (int64_t)1 << L;
    const double er = cos(phi), ei = sin(phi);
    const double pr = 0.5 * (1.0 + er), pi = 0.5 * ei;   /* (1 + e^{i phi}) / 2 */
    const double mr = 0.5 * (1.0 - er), mi = -0.5 * ei;  /* (1 - e^{i phi}) / 2 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, k) || (((uint64_t)i & cmask) != cmask)) continue;
        int64_t m = i | ((int64_t)1 << k);
        double x0r = a[2 * i], x0i = a[2 * i + 1], x1r = a[2 * m], x1i = a[2 * m + 1];
        a[2 * i] = (pr * x0r - pi * x0i) + (mr * x1r - mi * x1i);
        a[2 * i + 1] = (pr * x0i + pi * x0r) + (mr * x1i + mi * x1r);
        a[2 * m] = (mr * x0r - mi * x0i) + (pr * x1r - pi * x1i);
        a[2 * m + 1] = (mr * x0i + mi * x0r) + (pr * x1i + pi * x1r);
    }
}

/* The common form of Eqs. NUM2-NUM8: a 2x2 unitary u (row-major, (re, im) pairs:
 * u = {u00r, u00i, u01r, u01i, u10r, u10i, u11r, u11i}) on target j, restricted to indices whose
 * control bits (cmask) are all 1:
 *   a'(..0_j..) = u00 a(..0_j..) + u01 a(..1_j..),   a'(..1_j..) = u10 a(..0_j..) + u11 a(..1_j..). */
void or_unitary(double *a, int L, int j, uint64_t cmask, const double *u)
{
    const int64_t D = (int64_t)1 << L;
    const double u00r = u[0], u00i = u[1], u01r = u[2], u01i = u[3];
    const double u10r = u[4], u10i = u[5], u11r = u[6], u11i = u[7];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (BIT(i, j) || (((uint64_t)i & cmask) != cmask)) continue;
        int64_t m = i | ((int64_t)1 << j);
        double x0r = a[2 * i], x0i = a[2 * i + 1], x1r = a[2 * m], x1i = a[2 * m + 1];
        a[2 * i] = (u00r * x0r - u00i * x0i) + (u01r * x1r - u01i * x1i);
        a[2 * i + 1] = (u00r * x0i + u00i * x0r) + (u01r * x1i + u01i * x1r);
        a[2 * m] = (u10r * x0r - u10i * x0i) + (u11r * x1r - u11i * x1i);
        a[2 * m + 1] = (u10r * x0i + u10i * x0r) + (u11r * x1i + u11i * x1r);
    }
}

/* Quantum swap of qubits p and q (a permutation, no arithmetic): the amplitude of every index with
 * bit p = 1, bit q = 0 is exchanged with that of the index with the two bits the other way round. */
void or_swap(double *a, int L, int p, int q)
{
    const int64_t D = (int64_t)1 << L;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        if (!(BIT(i, p) == 1 && BIT(i, q) == 0)) continue;
        int64_t m = (i & ~((int64_t)1 << p)) | ((int64_t)1 << q);
        double tr = a[2 * i], ti = a[2 * i + 1];
        a[2 * i] = a[2 * m];
        a[2 * i + 1] = a[2 * m + 1];
        a[2 * m] = tr;
        a[2 * m + 1] = ti;
    }
}

/* A dense k-qubit gate: for every index b whose bits at qubits[0..k-1] are all 0, gather the 2^k
 * amplitudes v[r] = a(b + sum_s bit_s(r) 2^{qubits[s]}), form w = U v (U is 2^k x 2^k, row-major,
 * interleaved complex; matrix index bit s <-> qubits[s]) and scatter w back. */
void or_dense(double *a, int L, int k, const int *qubits, const double *U)
{
    const int64_t D = (int64_t)1 << L;
    const int K = 1 << k;
    uint64_t qmask = 0;
    for (int s = 0; s < k; ++s) qmask |= 1ULL << qubits[s];
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * 2 * K);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * K);
#pragma omp for schedule(static)
        for (int64_t b = 0; b < D; ++b) {
            if ((uint64_t)b & qmask) continue;
            for (int r = 0; r < K; ++r) {
                int64_t x = b;
                for (int s = 0; s < k; ++s)
                    if ((r >> s) & 1) x |= (int64_t)1 << qubits[s];
                idx[r] = x;
                v[2 * r] = a[2 * x];
                v[2 * r + 1] = a[2 * x + 1];
            }
            for (int r = 0; r < K; ++r) {
                double sr = 0.0, si = 0.0;
                for (int c = 0; c < K; ++c) {
                    double ur = U[2 * (r * K + c)], ui = U[2 * (r * K + c) + 1];
                    sr += ur * v[2 * c] - ui * v[2 * c + 1];
                    si += ur * v[2 * c + 1] + ui * v[2 * c];
                }
                a[2 * idx[r]] = sr;
                a[2 * idx[r] + 1] = si;
            }
        }
        free(v);
        free(idx);
    }
}

/* Probabilities p_i = |a_i|^2 (Sec. II.A: the probability of observing basis state i). */
void or_probs(const double *a, int L, double *p)
{
    const int64_t D = (int64_t)1 << L;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i)
        p[i] = a[2 * i] * a[2 * i] + a[2 * i + 1] * a[2 * i + 1];
}

/* Pairwise (recursive halving) sum of p[0..n-1]. */
static double pairwise(const double *p, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += p[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise(p, h) + pairwise(p + h, n - h);
}

/* Eq. STAT1: sum_i |a_i|^2, summed pairwise over the index. */
double or_norm(const double *a, int L)
{
    const int64_t D = (int64_t)1 << L;
    double *p = (double *)malloc(sizeof(double) * D);
    if (!p) return -1.0;
    or_probs(a, L, p);
    double s = pairwise(p, D);
    free(p);
    return s;
}

/* Eq. Shor7: <Q_i> = sum_k p_k k_i for every qubit i (k_i = bit i of k). Each qubit's sum runs
 * pairwise over the probabilities of the indices with that bit set. */
void or_marginals(const double *a, int L, double *q)
{
    const int64_t D = (int64_t)1 << L;
    double *p = (double *)malloc(sizeof(double) * D);
    double *sel = (double *)malloc(sizeof(double) * (D / 2 + 1));
    or_probs(a, L, p);
    for (int b = 0; b < L; ++b) {
        int64_t m = 0;
        for (int64_t i = 0; i < D; ++i)
            if (BIT(i, b)) sel[m++] = p[i];
        q[b] = pairwise(sel, m);
    }
    free(p);
    free(sel);
}

/* Sec. V (Shor's algorithm): the conditional operation that computes f(x) = y^x mod G into the
 * f-register, written as the permutation |x>|z> -> |x>|z XOR f(x)> of basis states (x = the bits
 * xf .. xf+xq-1 of the index, z = the bits ff .. ff+fq-1). The powers come from their definition,
 * f(0) = 1 mod G and f(x+1) = f(x) y mod G; then every pair of indices the map exchanges is swapped
 * once, from its smaller index. */
void or_modexp(double *a, int L, int xf, int xq, int ff, int fq, uint64_t y, uint64_t G)
{
    const int64_t D = (int64_t)1 << L;
    const int64_t X = (int64_t)1 << xq;
    uint64_t *f = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)X);
    f[0] = 1 % G;
    for (int64_t x = 1; x < X; ++x) f[x] = (f[x - 1] * (y % G)) % G;
    (void)fq;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
        const int64_t x = (i >> xf) & (X - 1);
        const int64_t m = i ^ (int64_t)(f[x] << ff);
        if (m <= i) continue;
        double tr = a[2 * i], ti = a[2 * i + 1];
        a[2 * i] = a[2 * m];
        a[2 * i + 1] = a[2 * m + 1];
        a[2 * m] = tr;
        a[2 * m + 1] = ti;
    }
    free(f);
}
