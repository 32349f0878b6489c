// Internal declarations of the self-consistent field around the two-electron build.
#pragma once

#include "hfk_internal.hpp"

namespace hfk {

constexpr int kDiisMax = 8;   // Fock matrices kept for the DIIS extrapolation

// Workspace of the SCF, appended after the per-atom Fock layout (offsets from the start).
struct ScfLayout {
    size_t S, H, X, F, G, Fx, A, C, T1, T2;   // n x n FP64 (column-major where it matters)
    size_t eps, evw;                          // [n] eigenvalues, [n] eigensolver scratch
    size_t info, scal;                        // eigensolver status; device scalars (E_nn, E2, |err|max)
    size_t Z;                                 // [n] nuclear charges
    size_t diisF, diisE;                      // [kDiisMax][n*n]
    size_t rocws;                             // linear-algebra library scratch
    size_t rocws_bytes;
    size_t total;
};

ScfLayout make_scf_layout(size_t base, int64_t n);

struct ScfResult {
    double energy;
    int iterations;
    int converged;
};

// Runs the SCF on `st` (waits for it whenever the host needs a number).  The Fock layout L
// (per-atom bases, workgroups set) and the uploaded Basis b come from the caller; dens holds
// the guess when use_guess is set and receives the final density.  Returns HFK_OK or a
// status with its message in msg.
hfk_status run_scf(const Layout &L, const Basis &b, char *ws, const ScfLayout &SL, const double *xyz,
                   const double *charges_host, int nocc, double tau, int prec, int strat, int max_iter,
                   double e_tol, double d_tol, double *dens, bool use_guess, double *eps_out, ScfResult *res,
                   hipStream_t st, char *msg, size_t msglen);

}  // namespace hfk
