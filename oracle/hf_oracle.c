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
 * Per-atom bases (the *_atoms entry points and hfo_eri4) give every atom its own exponents
 * and coefficients; the formulas above take each centre's own exponents (the kernel listing
 * passes one exponent and one coefficient array for all atoms, which is the special case of
 * identical rows).
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

/* A basis description is (g, exps, coefs, astride): atom i carries the contraction
 * exps[i * astride + a], coefs[i * astride + a], a < g.  astride = 0 gives every atom the
 * same contraction (the kernel listing's single exponent and coefficient arrays);
 * astride = g gives each atom its own (per-atom bases).  The primitive formulas above hold
 * for any exponent on any centre. */

static void prim_weights(int g, const double *exps, const double *coefs, double *w)
{
    for (int a = 0; a < g; ++a) w[a] = coefs[a] * pow(2.0 * exps[a] / HFO_PI, 0.75);
}

/* w for every atom of a basis description (one row when astride = 0); NULL when out of memory. */
static double *atom_weights(int64_t n, int g, const double *exps, const double *coefs, int64_t astride)
{
    const int64_t rows = astride ? n : 1;
    double *w = (double *)malloc(sizeof(double) * (size_t)(rows * g));
    if (!w) return NULL;
    for (int64_t i = 0; i < rows; ++i) prim_weights(g, exps + i * astride, coefs + i * astride, w + i * g);
    return w;
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

/* Contracted (AB|CD): the four nested primitive loops of the kernel listing, each centre
 * with its own exponents e* and weights w*. */
static double eri_core(const double *A, const double *B, const double *C, const double *D, int g,
                       const double *eA, const double *wA, const double *eB, const double *wB,
                       const double *eC, const double *wC, const double *eD, const double *wD)
{
    double ab2 = 0.0, cd2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        cd2 += (C[x] - D[x]) * (C[x] - D[x]);
    }
    double eri = 0.0;
    for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) {
            double p = eA[a] + eB[b];
            double Kab = wA[a] * wB[b] * exp(-eA[a] * eB[b] / p * ab2);
            double P[3];
            for (int x = 0; x < 3; ++x) P[x] = (eA[a] * A[x] + eB[b] * B[x]) / p;
            for (int c = 0; c < g; ++c)
                for (int d = 0; d < g; ++d) {
                    double q = eC[c] + eD[d];
                    double Kcd = wC[c] * wD[d] * exp(-eC[c] * eD[d] / q * cd2);
                    double Q[3], pq2 = 0.0;
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (eC[c] * C[x] + eD[d] * D[x]) / q;
                        pq2 += (P[x] - Q[x]) * (P[x] - Q[x]);
                    }
                    double rho = p * q / (p + q);
                    double pref = 2.0 * pow(HFO_PI, 2.5) / (p * q * sqrt(p + q));
                    eri += pref * Kab * Kcd * hfo_boys0(rho * pq2);
                }
        }
    return eri;
}

/* Contracted (AB|CD) with one contraction on all four centres. */
double hfo_eri(const double *A, const double *B, const double *C, const double *D,
               int g, const double *exps, const double *coefs)
{
    double w[16];
    prim_weights(g, exps, coefs, w);
    return eri_core(A, B, C, D, g, exps, w, exps, w, exps, w, exps, w);
}

/* Contracted (AB|CD) with a contraction of its own on each centre (eX, cX: g values each). */
double hfo_eri4(const double *A, const double *B, const double *C, const double *D, int g,
                const double *eA, const double *cA, const double *eB, const double *cB,
                const double *eC, const double *cC, const double *eD, const double *cD)
{
    double wA[16], wB[16], wC[16], wD[16];
    prim_weights(g, eA, cA, wA);
    prim_weights(g, eB, cB, wB);
    prim_weights(g, eC, cC, wC);
    prim_weights(g, eD, cD, wD);
    return eri_core(A, B, C, D, g, eA, wA, eB, wB, eC, wC, eD, wD);
}

/* Gradient of one contracted (AB|CD) with respect to the four centres, each scaled by
 * gamma and added into gA, gB, gC, gD (3 components each).  Per primitive quartet, with
 * E = pref K_ab K_cd:
 *   d/dA = E [ -2 mu_ab (A-B) F0 - 2 rho (a/p) (P-Q) F1 ]
 *   d/dB = E [ +2 mu_ab (A-B) F0 - 2 rho (b/p) (P-Q) F1 ]
 *   d/dC = E [ -2 mu_cd (C-D) F0 + 2 rho (c/q) (P-Q) F1 ]
 *   d/dD = E [ +2 mu_cd (C-D) F0 + 2 rho (d/q) (P-Q) F1 ]                                 */
static void eri_grad(const double *A, const double *B, const double *C, const double *D, int g,
                     const double *eA, const double *wA, const double *eB, const double *wB,
                     const double *eC, const double *wC, const double *eD, const double *wD, double gamma,
                     double *gA, double *gB, double *gC, double *gD)
{
    double ab2 = 0.0, cd2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        cd2 += (C[x] - D[x]) * (C[x] - D[x]);
    }
    for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) {
            double p = eA[a] + eB[b];
            double muab = eA[a] * eB[b] / p;
            double Kab = wA[a] * wB[b] * exp(-muab * ab2);
            double P[3];
            for (int x = 0; x < 3; ++x) P[x] = (eA[a] * A[x] + eB[b] * B[x]) / p;
            for (int c = 0; c < g; ++c)
                for (int d = 0; d < g; ++d) {
                    double q = eC[c] + eD[d];
                    double mucd = eC[c] * eD[d] / q;
                    double Kcd = wC[c] * wD[d] * exp(-mucd * cd2);
                    double Q[3], pq2 = 0.0;
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (eC[c] * C[x] + eD[d] * D[x]) / q;
                        pq2 += (P[x] - Q[x]) * (P[x] - Q[x]);
                    }
                    double rho = p * q / (p + q);
                    double E = gamma * 2.0 * pow(HFO_PI, 2.5) / (p * q * sqrt(p + q)) * Kab * Kcd;
                    double T = rho * pq2;
                    double f0 = hfo_boys0(T), f1 = hfo_boys1(T);
                    for (int x = 0; x < 3; ++x) {
                        double pqx = P[x] - Q[x];
                        gA[x] += E * (-2.0 * muab * (A[x] - B[x]) * f0 - 2.0 * rho * (eA[a] / p) * pqx * f1);
                        gB[x] += E * (+2.0 * muab * (A[x] - B[x]) * f0 - 2.0 * rho * (eB[b] / p) * pqx * f1);
                        gC[x] += E * (-2.0 * mucd * (C[x] - D[x]) * f0 + 2.0 * rho * (eC[c] / q) * pqx * f1);
                        gD[x] += E * (+2.0 * mucd * (C[x] - D[x]) * f0 + 2.0 * rho * (eD[d] / q) * pqx * f1);
                    }
                }
        }
}

/* (ij|kl) of atoms i, j, k, l under a basis description with weights W (atom_weights). */
static double eri_atoms(const double *xyz, int g, const double *exps, const double *W, int64_t astride,
                        int64_t i, int64_t j, int64_t k, int64_t l)
{
    const int64_t s = astride, sw = astride ? g : 0;
    return eri_core(xyz + 3 * i, xyz + 3 * j, xyz + 3 * k, xyz + 3 * l, g,
                    exps + i * s, W + i * sw, exps + j * s, W + j * sw,
                    exps + k * s, W + k * sw, exps + l * s, W + l * sw);
}

static void eri_grad_atoms(const double *xyz, int g, const double *exps, const double *W, int64_t astride,
                           int64_t i, int64_t j, int64_t k, int64_t l, double gamma, double *grad)
{
    const int64_t s = astride, sw = astride ? g : 0;
    eri_grad(xyz + 3 * i, xyz + 3 * j, xyz + 3 * k, xyz + 3 * l, g,
             exps + i * s, W + i * sw, exps + j * s, W + j * sw,
             exps + k * s, W + k * sw, exps + l * s, W + l * sw, gamma,
             grad + 3 * i, grad + 3 * j, grad + 3 * k, grad + 3 * l);
}

/* ---------------------------------------------------------------- Schwarz */

static inline int64_t pidx(int64_t i, int64_t j)
{
    if (i < j) { int64_t t = i; i = j; j = t; }
    return i * (i + 1) / 2 + j;
}

/* Q[ij] = sqrt((ij|ij)) for every pair i >= j, at index i(i+1)/2 + j. */
static int schwarz_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                     int64_t astride, int nthreads, double *Q)
{
    double *W = atom_weights(n, g, exps, coefs, astride);
    if (!W) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) Q[pidx(i, j)] = sqrt(eri_atoms(xyz, g, exps, W, astride, i, j, i, j));
    free(W);
    return 0;
}

void hfo_schwarz(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                 int nthreads, double *Q)
{
    (void)schwarz_s(n, xyz, g, exps, coefs, 0, nthreads, Q);
}

/* Per-atom bases: exps and coefs hold g values per atom (n * g). */
int hfo_schwarz_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                      int nthreads, double *Q)
{
    return schwarz_s(n, xyz, g, exps, coefs, g, nthreads, Q);
}

static double quartet_deg(int64_t i, int64_t j, int64_t k, int64_t l, int64_t ij, int64_t kl)
{
    double deg = 1.0;
    if (i == j) deg *= 0.5;
    if (k == l) deg *= 0.5;
    if (ij == kl) deg *= 0.5;
    return deg;
}

/* Q from the caller, or computed (*own set when the caller must free it); NULL when out of memory. */
static double *schwarz_or(const double *Qin, int64_t n, const double *xyz, int g, const double *exps,
                          const double *coefs, int64_t astride, int nthreads, int *own)
{
    *own = 0;
    if (Qin) return (double *)Qin;
    double *Q = (double *)malloc(sizeof(double) * (size_t)(n * (n + 1) / 2));
    if (!Q) return NULL;
    if (schwarz_s(n, xyz, g, exps, coefs, astride, nthreads, Q) != 0) { free(Q); return NULL; }
    *own = 1;
    return Q;
}

/* (i, j) of every canonical pair index i(i+1)/2 + j. */
static int64_t *pair_list(int64_t n)
{
    const int64_t npair = n * (n + 1) / 2;
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)npair * 2);
    if (!pi) return NULL;
    for (int64_t i = 0, p = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j, ++p) { pi[2 * p] = i; pi[2 * p + 1] = j; }
    return pi;
}

/* ---------------------------------------------------------------- Fock build */

/* Unique-quartet build over bra pairs with canonical index in [bra_begin, bra_end)
 * (the whole build when the range is [0, n(n+1)/2)).  F (n*n) receives G, e2 receives
 * E2 computed from that G, nsurv the number of quartets kept.  Q may be NULL (computed
 * here) or the array from hfo_schwarz.  Returns 0, or -1 when memory runs out. */
static int fock_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs, int64_t astride,
                  const double *dens, double tau, const double *Qin, int nthreads,
                  int64_t bra_begin, int64_t bra_end, double *F, double *e2, int64_t *nsurv)
{
    const int64_t npair = n * (n + 1) / 2;
    int ownQ = 0;
    double *Q = schwarz_or(Qin, n, xyz, g, exps, coefs, astride, nthreads, &ownQ);
    if (!Q) return -1;
    int64_t *pi = pair_list(n);
    double *W = atom_weights(n, g, exps, coefs, astride);
    if (!pi || !W) { free(pi); free(W); if (ownQ) free(Q); return -1; }
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
                    double eri = eri_atoms(xyz, g, exps, W, astride, i, j, k, l);
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
    free(W);
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

int hfo_fock(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
             const double *dens, double tau, const double *Qin, int nthreads,
             int64_t bra_begin, int64_t bra_end, double *F, double *e2, int64_t *nsurv)
{
    return fock_s(n, xyz, g, exps, coefs, 0, dens, tau, Qin, nthreads, bra_begin, bra_end, F, e2, nsurv);
}

int hfo_fock_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                   const double *dens, double tau, const double *Qin, int nthreads,
                   int64_t bra_begin, int64_t bra_end, double *F, double *e2, int64_t *nsurv)
{
    return fock_s(n, xyz, g, exps, coefs, g, dens, tau, Qin, nthreads, bra_begin, bra_end, F, e2, nsurv);
}

/* One element of G straight from the plain definition:
 *   G_ij = sum_kl D_kl [ s(ij,kl) (ij|kl) - 1/2 s(ik,jl) (ik|jl) ].
 * Q is the array from hfo_schwarz.  Returns NAN when out of memory. */
static double fock_element_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                             int64_t astride, const double *dens, double tau, const double *Q, int nthreads,
                             int64_t i, int64_t j)
{
    double *W = atom_weights(n, g, exps, coefs, astride);
    if (!W) return NAN;
    double acc = 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for reduction(+ : acc) schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < n; ++k)
        for (int64_t l = 0; l < n; ++l) {
            if (Q[pidx(i, j)] * Q[pidx(k, l)] >= tau)
                acc += dens[k * n + l] * eri_atoms(xyz, g, exps, W, astride, i, j, k, l);
            if (Q[pidx(i, k)] * Q[pidx(j, l)] >= tau)
                acc -= 0.5 * dens[k * n + l] * eri_atoms(xyz, g, exps, W, astride, i, k, j, l);
        }
    free(W);
    return acc;
}

double hfo_fock_element(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                        const double *dens, double tau, const double *Q, int nthreads,
                        int64_t i, int64_t j)
{
    return fock_element_s(n, xyz, g, exps, coefs, 0, dens, tau, Q, nthreads, i, j);
}

double hfo_fock_element_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                              const double *dens, double tau, const double *Q, int nthreads,
                              int64_t i, int64_t j)
{
    return fock_element_s(n, xyz, g, exps, coefs, g, dens, tau, Q, nthreads, i, j);
}

/* Every element of G from the plain definition (O(n^4) integrals; for tiny n). */
static int fock_bruteforce_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                             int64_t astride, const double *dens, double tau, double *F, double *e2)
{
    const int64_t npair = n * (n + 1) / 2;
    double *Q = (double *)malloc(sizeof(double) * (size_t)npair);
    if (!Q) return -1;
    if (schwarz_s(n, xyz, g, exps, coefs, astride, 1, Q) != 0) { free(Q); return -1; }
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            F[i * n + j] = fock_element_s(n, xyz, g, exps, coefs, astride, dens, tau, Q, 1, i, j);
        }
    for (int64_t x = 0; x < n * n; ++x) e += dens[x] * F[x];
    *e2 = 0.5 * e;
    free(Q);
    return 0;
}

int hfo_fock_bruteforce(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                        const double *dens, double tau, double *F, double *e2)
{
    return fock_bruteforce_s(n, xyz, g, exps, coefs, 0, dens, tau, F, e2);
}

int hfo_fock_bruteforce_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                              const double *dens, double tau, double *F, double *e2)
{
    return fock_bruteforce_s(n, xyz, g, exps, coefs, g, dens, tau, F, e2);
}

/* dE2/dR (n*3) over the unique quartets kept by the screen, also returning E2 and the
 * number of quartets kept.  Returns 0, or -1 when memory runs out. */
static int grad_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs, int64_t astride,
                  const double *dens, double tau, const double *Qin, int nthreads,
                  double *grad, double *e2, int64_t *nsurv)
{
    const int64_t npair = n * (n + 1) / 2;
    int ownQ = 0;
    double *Q = schwarz_or(Qin, n, xyz, g, exps, coefs, astride, nthreads, &ownQ);
    if (!Q) return -1;
    int64_t *pi = pair_list(n);
    double *W = atom_weights(n, g, exps, coefs, astride);
    if (!pi || !W) { free(pi); free(W); if (ownQ) free(Q); return -1; }
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
                    energy += gam * eri_atoms(xyz, g, exps, W, astride, i, j, k, l);
                    eri_grad_atoms(xyz, g, exps, W, astride, i, j, k, l, gam, gp);
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
    free(W);
    if (ownQ) free(Q);
    if (failed) return -1;
    if (e2) *e2 = energy;
    if (nsurv) *nsurv = count;
    return 0;
}

int hfo_grad(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
             const double *dens, double tau, const double *Qin, int nthreads,
             double *grad, double *e2, int64_t *nsurv)
{
    return grad_s(n, xyz, g, exps, coefs, 0, dens, tau, Qin, nthreads, grad, e2, nsurv);
}

int hfo_grad_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                   const double *dens, double tau, const double *Qin, int nthreads,
                   double *grad, double *e2, int64_t *nsurv)
{
    return grad_s(n, xyz, g, exps, coefs, g, dens, tau, Qin, nthreads, grad, e2, nsurv);
}

/* Gradient of the pairing L = sum_ij W_ij G_ij(R) of a fixed matrix W with the forward's G,
 * the screening decisions held fixed (used for the derivative through the G output).  In
 * unique-quartet form L = sum_unique B (ij|kl) with B the polarisation of 2 Gamma in which one
 * density is replaced by X:
 *   B = deg (4 (X_ij D_kl + D_ij X_kl) - (X_ik D_jl + D_ik X_jl) - (X_il D_jk + D_il X_jk)),
 * so X = W gives dL/dR, X = D / 2 gives dE2/dR, and X = W + (g/2) D gives both at once. */
static int grad_pair_s(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                       int64_t astride, const double *dens, const double *xdens, double tau, const double *Qin,
                       int nthreads, double *grad)
{
    const int64_t npair = n * (n + 1) / 2;
    int ownQ = 0;
    double *Q = schwarz_or(Qin, n, xyz, g, exps, coefs, astride, nthreads, &ownQ);
    if (!Q) return -1;
    int64_t *pi = pair_list(n);
    double *W = atom_weights(n, g, exps, coefs, astride);
    if (!pi || !W) { free(pi); free(W); if (ownQ) free(Q); return -1; }
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
                    eri_grad_atoms(xyz, g, exps, W, astride, i, j, k, l, b, gp);
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
    free(W);
    if (ownQ) free(Q);
    return failed ? -1 : 0;
}

int hfo_grad_pair(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                  const double *dens, const double *xdens, double tau, const double *Qin, int nthreads,
                  double *grad)
{
    return grad_pair_s(n, xyz, g, exps, coefs, 0, dens, xdens, tau, Qin, nthreads, grad);
}

int hfo_grad_pair_atoms(int64_t n, const double *xyz, int g, const double *exps, const double *coefs,
                        const double *dens, const double *xdens, double tau, const double *Qin, int nthreads,
                        double *grad)
{
    return grad_pair_s(n, xyz, g, exps, coefs, g, dens, xdens, tau, Qin, nthreads, grad);
}

/* ---------------------------------------------------------------- one-electron integrals */

/* For the self-consistent field around the two-electron build (not part of the paper's
 * kernel, which computes the electron-repulsion term only): overlap S, kinetic energy T and
 * nuclear attraction V of contracted s functions, from the standard closed forms of s
 * Gaussians (p = a + b, mu = a b / p, P = (a A + b B) / p, R = |A - B|):
 *   S_ab = w_a w_b (pi / p)^(3/2) exp(-mu R^2)
 *   T_ab = mu (3 - 2 mu R^2) S_ab
 *   V_ab = - sum_C Z_C w_a w_b (2 pi / p) exp(-mu R^2) F0(p |P - C|^2)
 * Per-atom rows (astride = g) as the *_atoms functions.  S, T, V are n x n, symmetric. */
int hfo_one_electron_atoms(int64_t n, const double *xyz, const double *Z, int g, const double *exps,
                           const double *coefs, double *S, double *T, double *V)
{
    double *W = atom_weights(n, g, exps, coefs, g);
    if (!W) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            const double *A = xyz + 3 * i, *B = xyz + 3 * j;
            const double *ea = exps + i * g, *eb = exps + j * g, *wa = W + i * g, *wb = W + j * g;
            double r2 = 0.0;
            for (int x = 0; x < 3; ++x) r2 += (A[x] - B[x]) * (A[x] - B[x]);
            double s = 0.0, t = 0.0, v = 0.0;
            for (int a = 0; a < g; ++a)
                for (int b = 0; b < g; ++b) {
                    double p = ea[a] + eb[b], mu = ea[a] * eb[b] / p;
                    double K = wa[a] * wb[b] * exp(-mu * r2);
                    double sab = K * pow(HFO_PI / p, 1.5);
                    s += sab;
                    t += mu * (3.0 - 2.0 * mu * r2) * sab;
                    double P[3];
                    for (int x = 0; x < 3; ++x) P[x] = (ea[a] * A[x] + eb[b] * B[x]) / p;
                    for (int64_t c = 0; c < n; ++c) {
                        double pc2 = 0.0;
                        for (int x = 0; x < 3; ++x) pc2 += (P[x] - xyz[3 * c + x]) * (P[x] - xyz[3 * c + x]);
                        v -= Z[c] * K * (2.0 * HFO_PI / p) * hfo_boys0(p * pc2);
                    }
                }
            S[i * n + j] = S[j * n + i] = s;
            T[i * n + j] = T[j * n + i] = t;
            V[i * n + j] = V[j * n + i] = v;
        }
    free(W);
    return 0;
}

int hfo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
