/*
 * hf_oracle.c -- plain, slow, FP64 CPU oracle for the screened two-electron Fock build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file;
 * it exists so that tests, the smoke check and the bench's CPU baseline have an
 * independent reference.  It shares no code, header, table or constant generator with the
 * HIP library.
 *
 * What is computed (Background section, "Hartree--Fock" paragraph and its kernel listing:
 * a loop over unique (ij|kl) quartets of contracted s Gaussians, four nested loops over the
 * Gaussian primitives accumulating the primitive integral built from the Boys function F0,
 * then six atomic updates of the Fock matrix, Coulomb with factor 4 and exchange with
 * factor -1, reading a symmetric density):
 *
 *   primitive   g_a(r) = (2 a / pi)^(3/4) exp(-a |r - A|^2), contracted phi = sum_a c_a g_a
 *   product     p = a + b, mu = a b / p, P = (a A + b B) / p,
 *               K_ab = w_a w_b exp(-mu |A - B|^2),  w_a = c_a (2 a / pi)^(3/4)
 *   integral    (ab|cd) = 2 pi^(5/2) / (p q sqrt(p + q)) K_ab K_cd F0(rho |P - Q|^2),
 *               rho = p q / (p + q)        (the listing's dkl * f0t * sqrt(aijkl) term)
 *   Boys        F_m(t) = int_0^1 u^(2m) exp(-t u^2) du
 *   Schwarz     Q_ij = sqrt((ij|ij)); a quartet is kept iff Q_ij Q_kl >= tau
 *   Fock        G_ij = sum_kl D_kl [ s(ij,kl) (ij|kl) - 1/2 s(ik,jl) (ik|jl) ]
 *   energy      E2 = 1/2 sum_ij D_ij G_ij
 *
 * The unique-quartet scatter (hfo_fock) is the rearrangement of the plain definition that
 * keeps the listing's factors 4 and -1: with v = (ij|kl) * deg (deg halves once for each of
 * i = j, k = l, ij = kl),
 *   F_ij += 4 D_kl v,  F_kl += 4 D_ij v,
 *   F_ik -= D_jl v,    F_il -= D_jk v,   F_jk -= D_il v,   F_jl -= D_ik v,
 * followed by G = (F + F^T) / 2.  hfo_fock_bruteforce and hfo_fock_element evaluate the
 * plain definition directly and pin the scatter.
 *
 * The nuclear gradient (hfo_grad) differentiates E2 = sum_unique Gamma_ijkl (ij|kl),
 * Gamma = deg (4 D_ij D_kl - D_ik D_jl - D_il D_jk), with the screening decisions held
 * fixed; the derivative of one primitive integral uses F0 and F1 (dF0/dt = -F1).  The
 * paper has no gradient; this is the derivative of the functional above.  hfo_grad_pair is
 * the same contraction for the pairing sum_ij W_ij G_ij with a fixed W (the derivative
 * through the G output), with Gamma replaced by its polarisation B(X, D).
 *
 * Readings where the paper is silent: normalised primitives with the coefficients used as
 * given (no contraction renormalisation); contracted Schwarz bounds in FP64 with a
 * "keep iff >= tau" test and no primitive-level screening; G symmetrised as (F + F^T)/2;
 * E2 as above; atomics target F only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HFO_PI 3.14159265358979323846264338327950288

/* ---------------------------------------------------------------- Boys function */

/* F_m(t) by its Kummer series  F_m(t) = exp(-t) sum_k (2t)^k / [(2m+1)(2m+3)...(2m+2k+1)].
 * Every term is positive, so there is no cancellation; it is used for t <= 100 and the
 * large-t limit (2m-1)!! / 2^(m+1) sqrt(pi / t^(2m+1)) beyond (the neglected part is below
 * exp(-100) relative). */
double hfo_boys_series(int m, double t)
{
    if (t > 100.0) {
        double df = 1.0;                       /* (2m-1)!! */
        for (int i = 1; i <= m; ++i) df *= (double)(2 * i - 1);
        return df / pow(2.0, (double)(m + 1)) * sqrt(HFO_PI / pow(t, 2.0 * m + 1.0));
    }
    double term = 1.0 / (2.0 * m + 1.0);
    double sum = term;
    for (int k = 1; k < 2000; ++k) {
        term *= 2.0 * t / (2.0 * m + 2.0 * k + 1.0);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return exp(-t) * sum;
}

/* F0(t) = (1/2) sqrt(pi / t) erf(sqrt t), F0(0) = 1: the closed form, used inside the integrals. */
double hfo_boys0(double t)
{
    if (t < 1e-15) return 1.0 - t / 3.0;
    double st = sqrt(t);
    return 0.5 * sqrt(HFO_PI) / st * erf(st);
}

/* F1(t): series below t = 1, closed form (F0 - exp(-t)) / (2t) at and above (the two terms
 * differ by at least half of F0 there, so the subtraction loses under one digit). */
double hfo_boys1(double t)
{
    if (t < 1.0) return hfo_boys_series(1, t);
    return (hfo_boys0(t) - exp(-t)) / (2.0 * t);
}

/* ---------------------------------------------------------------- basis */

static void prim_weights(int g, const double *exps, const double *coefs, double *w)
{
    for (int a = 0; a < g; ++a) w[a] = coefs[a] * pow(2.0 * exps[a] / HFO_PI, 0.75);
}

/* Overlap <phi_A | phi_B> of two contracted s functions. */
double hfo_overlap(const double *A, const double *B, int g, const double *exps, const double *coefs)
{
    double w[16];
    prim_weights(g, exps, coefs, w);
    double ab2 = 0.0;
    for (int x = 0; x < 3; ++x) ab2 += (A[x] - B[x]) * (A[x] - B[x]);
    double s = 0.0;
    for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) {
            double p = exps[a] + exps[b];
            s += w[a] * w[b] * pow(HFO_PI / p, 1.5) * exp(-exps[a] * exps[b] / p * ab2);
        }
    return s;
}

/* Contracted (AB|CD): the four nested primitive loops of the kernel listing. */
double hfo_eri(const double *A, const double *B, const double *C, const double *D,
               int g, const double *exps, const double *coefs)
{
    double w[16];
    prim_weights(g, exps, coefs, w);
    double ab2 = 0.0, cd2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        cd2 += (C[x] - D[x]) * (C[x] - D[x]);
    }
    double eri = 0.0;
    for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) {
            double p = exps[a] + exps[b];
            double Kab = w[a] * w[b] * exp(-exps[a] * exps[b] / p * ab2);
            double P[3];
            for (int x = 0; x < 3; ++x) P[x] = (exps[a] * A[x] + exps[b] * B[x]) / p;
            for (int c = 0; c < g; ++c)
                for (int d = 0; d < g; ++d) {
                    double q = exps[c] + exps[d];
                    double Kcd = w[c] * w[d] * exp(-exps[c] * exps[d] / q * cd2);
                    double Q[3], pq2 = 0.0;
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (exps[c] * C[x] + exps[d] * D[x]) / q;
                        pq2 += (P[x] - Q[x]) * (P[x] - Q[x]);
                    }
                    double rho = p * q / (p + q);
                    double pref = 2.0 * pow(HFO_PI, 2.5) / (p * q * sqrt(p + q));
                    eri += pref * Kab * Kcd * hfo_boys0(rho * pq2);
                }
        }
    return eri;
}

/* Gradient of one contracted (AB|CD) with respect to the four centres, each scaled by
 * gamma and added into gA, gB, gC, gD (3 components each).  Per primitive quartet, with
 * E = pref K_ab K_cd:
 *   d/dA = E [ -2 mu_ab (A-B) F0 - 2 rho (a/p) (P-Q) F1 ]
 *   d/dB = E [ +2 mu_ab (A-B) F0 - 2 rho (b/p) (P-Q) F1 ]
 *   d/dC = E [ -2 mu_cd (C-D) F0 + 2 rho (c/q) (P-Q) F1 ]
 *   d/dD = E [ +2 mu_cd (C-D) F0 + 2 rho (d/q) (P-Q) F1 ]                                 */
static void eri_grad(const double *A, const double *B, const double *C, const double *D,
                     int g, const double *exps, const double *w, double gamma,
                     double *gA, double *gB, double *gC, double *gD)
{
    double ab2 = 0.0, cd2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        cd2 += (C[x] - D[x]) * (C[x] - D[x]);
    }
    for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) {
            double p = exps[a] + exps[b];
            double muab = exps[a] * exps[b] / p;
            double Kab = w[a] * w[b] * exp(-muab * ab2);
            double P[3];
            for (int x = 0; x < 3; ++x) P[x] = (exps[a] * A[x] + exps[b] * B[x]) / p;
            for (int c = 0; c < g; ++c)
                for (int d = 0; d < g; ++d) {
                    double q = exps[c] + exps[d];
                    double mucd = exps[c] * exps[d] / q;
                    double Kcd = w[c] * w[d] * exp(-mucd * cd2);
                    double Q[3], pq2 = 0.0;
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (exps[c] * C[x] + exps[d] * D[x]) / q;
                        pq2 += (P[x] - Q[x]) * (P[x] - Q[x]);
                    }
                    double rho = p * q / (p + q);
                    double E = gamma * 2.0 * pow(HFO_PI, 2.5) / (p * q * sqrt(p + q)) * Kab * Kcd;
                    double T = rho * pq2;
                    double f0 = hfo_boys0(T), f1 = hfo_boys1(T);
                    for (int x = 0; x < 3; ++x) {
                        double pqx = P[x] - Q[x];
                        gA[x] += E * (-2.0 * muab * (A[x] - B[x]) * f0 - 2.0 * rho * (exps[a] / p) * pqx * f1);
                        gB[x] += E * (+2.0 * muab * (A[x] - B[x]) * f0 - 2.0 * rho * (exps[b] / p) * pqx * f1);
                        gC[x] += E * (-2.0 * mucd * (C[x] - D[x]) * f0 + 2.0 * rho * (exps[c] / q) * pqx * f1);
                        gD[x] += E * (+2.0 * mucd * (C[x] - D[x]) * f0 + 2.0 * rho * (exps[d] / q) * pqx * f1);
                    }
                }
        }
}

/* ---------------------------------------------------------------- Schwarz */

static inline int64_t pidx(int64_t i, int64_t j)
{
    if (i < j) { int64_t t = i; i = j; j = t; }
    return i * (i + 1) / 2 + j;
}

/* Q[ij] = sqrt((ij|ij)) for every pair i >= j, at index i(i+1)/2 + j. */
void hfo_schwarz(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                 int nthreads, double *Q)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            const double *A = xyz + 3 * i, *B = xyz + 3 * j;
            Q[pidx(i, j)] = sqrt(hfo_eri(A, B, A, B, g, exps, coefs));
        }
}

static double quartet_deg(int64_t i, int64_t j, int64_t k, int64_t l, int64_t ij, int64_t kl)
{
    double deg = 1.0;
    if (i == j) deg *= 0.5;
    if (k == l) deg *= 0.5;
    if (ij == kl) deg *= 0.5;
    return deg;
}

/* ---------------------------------------------------------------- Fock build */

/* Unique-quartet build over bra pairs with canonical index in [bra_begin, bra_end)
 * (the whole build when the range is [0, n(n+1)/2)).  F (n*n) receives G, e2 receives
 * E2 computed from that G, nsurv the number of quartets kept.  Q may be NULL (computed
 * here) or the array from hfo_schwarz.  Returns 0, or -1 when memory runs out. */
int hfo_fock(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
             const double *dens, double tau, const double *Qin, int nthreads,
             int64_t bra_begin, int64_t bra_end, double *F, double *e2, int64_t *nsurv)
{
    const int64_t npair = n * (n + 1) / 2;
    double *Q = (double *)Qin;
    int ownQ = 0;
    if (!Q) {
        Q = (double *)malloc(sizeof(double) * (size_t)npair);
        if (!Q) return -1;
        hfo_schwarz(n, xyz, g, exps, coefs, nthreads, Q);
        ownQ = 1;
    }
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)npair * 2);
    if (!pi) { if (ownQ) free(Q); return -1; }
    for (int64_t i = 0, p = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j, ++p) { pi[2 * p] = i; pi[2 * p + 1] = j; }
    if (bra_begin < 0) bra_begin = 0;
    if (bra_end > npair) bra_end = npair;

    memset(F, 0, sizeof(double) * (size_t)(n * n));
    int64_t count = 0;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(+ : count)
#endif
    {
        double *Fp = (double *)calloc((size_t)(n * n), sizeof(double));
        if (!Fp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t ij = bra_begin; ij < bra_end; ++ij) {
                const int64_t i = pi[2 * ij], j = pi[2 * ij + 1];
                for (int64_t kl = 0; kl <= ij; ++kl) {
                    if (Q[ij] * Q[kl] < tau) continue;
                    const int64_t k = pi[2 * kl], l = pi[2 * kl + 1];
                    double eri = hfo_eri(xyz + 3 * i, xyz + 3 * j, xyz + 3 * k, xyz + 3 * l, g, exps, coefs);
                    double v = eri * quartet_deg(i, j, k, l, ij, kl);
                    Fp[i * n + j] += 4.0 * dens[k * n + l] * v;
                    Fp[k * n + l] += 4.0 * dens[i * n + j] * v;
                    Fp[i * n + k] -= dens[j * n + l] * v;
                    Fp[i * n + l] -= dens[j * n + k] * v;
                    Fp[j * n + k] -= dens[i * n + l] * v;
                    Fp[j * n + l] -= dens[i * n + k] * v;
                    ++count;
                }
            }
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int64_t x = 0; x < n * n; ++x) F[x] += Fp[x];
            free(Fp);
        }
    }
    free(pi);
    if (ownQ) free(Q);
    if (failed) return -1;
    /* G = (F + F^T) / 2 and E2 = 1/2 sum D o G */
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < i; ++j) {
            double s = 0.5 * (F[i * n + j] + F[j * n + i]);
            F[i * n + j] = s;
            F[j * n + i] = s;
        }
    for (int64_t x = 0; x < n * n; ++x) e += dens[x] * F[x];
    *e2 = 0.5 * e;
    if (nsurv) *nsurv = count;
    return 0;
}

/* One element of G straight from the plain definition:
 *   G_ij = sum_kl D_kl [ s(ij,kl) (ij|kl) - 1/2 s(ik,jl) (ik|jl) ].
 * Q is the array from hfo_schwarz. */
double hfo_fock_element(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                        const double *dens, double tau, const double *Q, int nthreads,
                        int64_t i, int64_t j)
{
    double acc = 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for reduction(+ : acc) schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < n; ++k)
        for (int64_t l = 0; l < n; ++l) {
            const double *A = xyz + 3 * i, *B = xyz + 3 * j, *C = xyz + 3 * k, *D = xyz + 3 * l;
            if (Q[pidx(i, j)] * Q[pidx(k, l)] >= tau)
                acc += dens[k * n + l] * hfo_eri(A, B, C, D, g, exps, coefs);
            if (Q[pidx(i, k)] * Q[pidx(j, l)] >= tau)
                acc -= 0.5 * dens[k * n + l] * hfo_eri(A, C, B, D, g, exps, coefs);
        }
    return acc;
}

/* Every element of G from the plain definition (O(n^4) integrals; for tiny n). */
int hfo_fock_bruteforce(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                        const double *dens, double tau, double *F, double *e2)
{
    const int64_t npair = n * (n + 1) / 2;
    double *Q = (double *)malloc(sizeof(double) * (size_t)npair);
    if (!Q) return -1;
    hfo_schwarz(n, xyz, g, exps, coefs, 1, Q);
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            F[i * n + j] = hfo_fock_element(n, xyz, g, exps, coefs, dens, tau, Q, 1, i, j);
        }
    for (int64_t x = 0; x < n * n; ++x) e += dens[x] * F[x];
    *e2 = 0.5 * e;
    free(Q);
    return 0;
}

/* dE2/dR (n*3) over the unique quartets kept by the screen, also returning E2 and the
 * number of quartets kept.  Returns 0, or -1 when memory runs out. */
int hfo_grad(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
             const double *dens, double tau, const double *Qin, int nthreads,
             double *grad, double *e2, int64_t *nsurv)
{
    const int64_t npair = n * (n + 1) / 2;
    double *Q = (double *)Qin;
    int ownQ = 0;
    if (!Q) {
        Q = (double *)malloc(sizeof(double) * (size_t)npair);
        if (!Q) return -1;
        hfo_schwarz(n, xyz, g, exps, coefs, nthreads, Q);
        ownQ = 1;
    }
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)npair * 2);
    if (!pi) { if (ownQ) free(Q); return -1; }
    for (int64_t i = 0, p = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j, ++p) { pi[2 * p] = i; pi[2 * p + 1] = j; }
    double w[16];
    prim_weights(g, exps, coefs, w);
    memset(grad, 0, sizeof(double) * (size_t)(3 * n));
    double energy = 0.0;
    int64_t count = 0;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(+ : energy, count)
#endif
    {
        double *gp = (double *)calloc((size_t)(3 * n), sizeof(double));
        if (!gp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t ij = 0; ij < npair; ++ij) {
                const int64_t i = pi[2 * ij], j = pi[2 * ij + 1];
                for (int64_t kl = 0; kl <= ij; ++kl) {
                    if (Q[ij] * Q[kl] < tau) continue;
                    const int64_t k = pi[2 * kl], l = pi[2 * kl + 1];
                    double gam = quartet_deg(i, j, k, l, ij, kl) *
                                 (4.0 * dens[i * n + j] * dens[k * n + l] - dens[i * n + k] * dens[j * n + l] -
                                  dens[i * n + l] * dens[j * n + k]);
                    const double *A = xyz + 3 * i, *B = xyz + 3 * j, *C = xyz + 3 * k, *D = xyz + 3 * l;
                    energy += gam * hfo_eri(A, B, C, D, g, exps, coefs);
                    eri_grad(A, B, C, D, g, exps, w, gam, gp + 3 * i, gp + 3 * j, gp + 3 * k, gp + 3 * l);
                    ++count;
                }
            }
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int64_t x = 0; x < 3 * n; ++x) grad[x] += gp[x];
            free(gp);
        }
    }
    free(pi);
    if (ownQ) free(Q);
    if (failed) return -1;
    if (e2) *e2 = energy;
    if (nsurv) *nsurv = count;
    return 0;
}

/* Gradient of the pairing L = sum_ij W_ij G_ij(R) of a fixed matrix W with the forward's G,
 * the screening decisions held fixed (used for the derivative through the G output).  In
 * unique-quartet form L = sum_unique B (ij|kl) with B the polarisation of 2 Gamma in which one
 * density is replaced by X:
 *   B = deg (4 (X_ij D_kl + D_ij X_kl) - (X_ik D_jl + D_ik X_jl) - (X_il D_jk + D_il X_jk)),
 * so X = W gives dL/dR, X = D / 2 gives dE2/dR, and X = W + (g/2) D gives both at once. */
int hfo_grad_pair(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                  const double *dens, const double *xdens, double tau, const double *Qin, int nthreads,
                  double *grad)
{
    const int64_t npair = n * (n + 1) / 2;
    double *Q = (double *)Qin;
    int ownQ = 0;
    if (!Q) {
        Q = (double *)malloc(sizeof(double) * (size_t)npair);
        if (!Q) return -1;
        hfo_schwarz(n, xyz, g, exps, coefs, nthreads, Q);
        ownQ = 1;
    }
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)npair * 2);
    if (!pi) { if (ownQ) free(Q); return -1; }
    for (int64_t i = 0, p = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j, ++p) { pi[2 * p] = i; pi[2 * p + 1] = j; }
    double w[16];
    prim_weights(g, exps, coefs, w);
    memset(grad, 0, sizeof(double) * (size_t)(3 * n));
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *gp = (double *)calloc((size_t)(3 * n), sizeof(double));
        if (!gp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t ij = 0; ij < npair; ++ij) {
                const int64_t i = pi[2 * ij], j = pi[2 * ij + 1];
                for (int64_t kl = 0; kl <= ij; ++kl) {
                    if (Q[ij] * Q[kl] < tau) continue;
                    const int64_t k = pi[2 * kl], l = pi[2 * kl + 1];
                    const double *X = xdens, *D = dens;
                    const double b = quartet_deg(i, j, k, l, ij, kl) *
                                     (4.0 * (X[i * n + j] * D[k * n + l] + D[i * n + j] * X[k * n + l]) -
                                      (X[i * n + k] * D[j * n + l] + D[i * n + k] * X[j * n + l]) -
                                      (X[i * n + l] * D[j * n + k] + D[i * n + l] * X[j * n + k]));
                    const double *A = xyz + 3 * i, *B = xyz + 3 * j, *C = xyz + 3 * k, *E = xyz + 3 * l;
                    eri_grad(A, B, C, E, g, exps, w, b, gp + 3 * i, gp + 3 * j, gp + 3 * k, gp + 3 * l);
                }
            }
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int64_t x = 0; x < 3 * n; ++x) grad[x] += gp[x];
            free(gp);
        }
    }
    free(pi);
    if (ownQ) free(Q);
    return failed ? -1 : 0;
}

int hfo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
