/*
 * hfk.h -- C ABI of the MI355X (gfx950) two-electron Fock build library, libhfk.so.
 *
 * The operation (Background section, "Hartree--Fock" paragraph and its kernel listing):
 * for a system of atoms, each carrying one contracted s-type Gaussian built from the same
 * primitives (exponents xpnt, coefficients coef), loop over the unique electron-repulsion
 * quartets (ij|kl) that pass the Schwarz screen Q_ij Q_kl >= tau, Q_ij = sqrt((ij|ij)),
 * evaluate each from its primitive quartets with the Boys function F0, and scatter the
 * Coulomb (factor 4) and exchange (factor -1) contributions into the Fock matrix read
 * against the density, under the 8-fold permutational symmetry of the integrals.  The
 * library returns the symmetrised two-electron matrix
 *     G_ij = sum_kl D_kl [ s(ij,kl) (ij|kl) - 1/2 s(ik,jl) (ik|jl) ]
 * and the two-electron energy E2 = 1/2 sum_ij D_ij G_ij.
 *
 * Conventions shared by every entry point:
 *   - Units: bohr in, hartree out.  Every matrix is FP64, row-major, contiguous.
 *   - Pointers without a _host suffix are DEVICE pointers (memory of the current HIP
 *     device).  Pointers with _host are host memory read during the call.
 *   - The caller owns every buffer.  The library never allocates, frees or retains caller
 *     memory: its scratch comes from the caller's workspace, whose size the matching
 *     *_workspace_bytes call returns (a bound that depends only on the sizes passed).
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the null stream)
 *     and the call returns without waiting for it, except hfk_read_stats.
 *   - Arguments are validated on the host before any HIP call; an invalid call enqueues
 *     nothing.  A non-zero hfk_status is returned on failure and hfk_last_error() gives a
 *     thread-local message.  No C++ exception crosses this interface.
 *   - The density must be symmetric (the kernel listing reads dens as a symmetric matrix:
 *     the Coulomb scatter uses D_kl for both orders of k and l, the exchange reads D_ik,
 *     D_jl, D_il and D_jk for one order each).  The library does not check it unless debug
 *     mode is on (hfk_set_debug), in which case a density that is not symmetric is refused
 *     with HFK_ENOTSYM before any build work.
 *   - Calls that share a workspace must not overlap in time (same stream, or ordered).
 */
#ifndef HFK_H
#define HFK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hfk_status {
    HFK_OK = 0,
    HFK_EINVAL = 1,        /* an argument is out of range or a required pointer is NULL */
    HFK_ENOMEM = 2,        /* the workspace is smaller than *_workspace_bytes asked for */
    HFK_EHIP = 3,          /* a HIP runtime call failed (message holds the HIP error) */
    HFK_EUNSUPPORTED = 4,  /* valid but outside what this library version supports (sizes, device) */
    HFK_ENOTSYM = 5        /* debug mode only: a density is not symmetric within the debug tolerance */
} hfk_status;

typedef enum hfk_precision {
    HFK_FP64 = 0,   /* every step in FP64 */
    HFK_MIXED = 1   /* primitive integrals and Boys function in FP32; Schwarz bounds, the
                       contraction into the Fock matrix, the energy and the gradient
                       accumulation in FP64 */
} hfk_precision;

/* Accumulation strategy of the forward build (chosen by hfk_tune or passed explicitly). */
typedef enum hfk_strategy {
    HFK_STRATEGY_AUTO = 0,     /* library default, or the tuned choice once hfk_tune ran */
    HFK_STRATEGY_PRIVATE = 1,  /* each workgroup owns an FP64 copy of F; summed at the end */
    HFK_STRATEGY_ATOMIC = 2,   /* workgroups flush their LDS rows into one F with atomics */
    HFK_STRATEGY_DETERMINISTIC = 3   /* every sum in a fixed order: repeated builds with the same
                                        inputs on the same device agree bit for bit.  Static
                                        block schedule, private copies of F and of the ket
                                        vectors, per-wave LDS rows.  Up to 1024 atoms (hfk_fock and
                                        hfk_fock_atoms; HFK_EUNSUPPORTED above); slower than the
                                        other strategies and never chosen by the tuner */
} hfk_strategy;

/* Arguments accept up to HFK_MAX_NGAUSS primitives per function; the kernels are built for
 * up to HFK_BUILT_NGAUSS (more returns HFK_EUNSUPPORTED). */
enum { HFK_MAX_NGAUSS = 8, HFK_BUILT_NGAUSS = 6 };

/* Counters of the last build that used a workspace, read back by hfk_read_stats. */
typedef struct hfk_stats {
    int64_t natoms;          /* atoms (basis functions) */
    int64_t pairs;           /* n(n+1)/2 */
    int64_t sig_pairs;       /* pairs with Q_ij * max Q >= tau */
    int64_t quartets;        /* unique quartets kept by the screen (ij >= kl) */
    int64_t work_items;      /* items of the persistent quartet kernel */
    int32_t strategy;        /* hfk_strategy actually used */
    int32_t groups;          /* persistent workgroups launched */
    int32_t precision;       /* hfk_precision used */
    int32_t variant;         /* quartet-kernel variant used (hfk_set_config) */
    int32_t tile_items;      /* items (1024 kets each) per block of the single-molecule
                                kernels, or items (256 kets) per block of the batched one */
    int32_t group_bras;      /* bras per group whose blocks are numbered ket-block-major */
    int32_t ket_copies;      /* copies of the ket-side Coulomb vector (= groups: one per
                                workgroup, plain read-modify-writes; fewer: shared, atomics) */
    int32_t reserved;
} hfk_stats;

/* Workspace size (bytes) for hfk_fock / hfk_fock_grad on `natoms` atoms with `ngauss`
 * primitives per atom at `precision`; with_grad != 0 adds what hfk_fock_grad needs.
 * Uses the current device's compute-unit count.  Errors: HFK_EINVAL for natoms < 1,
 * ngauss outside [1, HFK_MAX_NGAUSS], an unknown precision or a NULL bytes_out. */
hfk_status hfk_workspace_bytes(int64_t natoms, int32_t ngauss, int32_t precision,
                               int32_t with_grad, size_t *bytes_out);

/* Forward Fock build: the Background section's kernel (listing of the Hartree--Fock
 * kernel), over all unique screened quartets.
 *   natoms           n >= 1
 *   xyz              [n*3] atom positions (bohr)
 *   ngauss           primitives per contracted function, 1..HFK_MAX_NGAUSS
 *   exps_host        [ngauss] primitive exponents, each > 0 and finite (host memory)
 *   coefs_host       [ngauss] contraction coefficients, finite (host memory); the
 *                    primitives are normalised, the coefficients are used as given
 *   dens             [n*n] symmetric density D
 *   tau              Schwarz threshold, finite and >= 0 (a quartet is kept iff
 *                    Q_ij Q_kl >= tau)
 *   precision        hfk_precision
 *   strategy         hfk_strategy (HFK_STRATEGY_AUTO for the default)
 *   fock             [n*n] output G (overwritten)
 *   e2               [1] output E2 (device, overwritten)
 *   workspace        device scratch of at least hfk_workspace_bytes(...) bytes, 256-byte
 *                    aligned; its contents on entry do not matter
 * Errors: HFK_EINVAL (arguments), HFK_ENOMEM (workspace too small), HFK_EUNSUPPORTED
 * (n above what one workgroup's LDS rows hold, or ngauss above HFK_BUILT_NGAUSS),
 * HFK_EHIP (launch failure). */
hfk_status hfk_fock(int64_t natoms, const double *xyz, int32_t ngauss,
                    const double *exps_host, const double *coefs_host,
                    const double *dens, double tau, int32_t precision, int32_t strategy,
                    double *fock, double *e2,
                    void *workspace, size_t workspace_bytes, void *stream);

/* hfk_fock for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same build with the atomics
 * strategy, whose scratch is a static device array of 64 MiB inside the library instead
 * of a caller workspace.  The call allocates nothing (no hipMalloc, no library routine that
 * allocates).  Every GPU the library runs on holds its own copy of that array until the
 * process ends; every call on a GPU shares that GPU's copy, so calls that overlap in time on
 * one GPU race (serialise them, e.g. on one stream).  Each call clears what it needs.
 *   Arguments and outputs as hfk_fock, without strategy and workspace.
 * Errors as hfk_fock; HFK_EUNSUPPORTED when the system needs more scratch than the array
 * holds (about 256 atoms with 3 primitives per function, fewer with more primitives). */
hfk_status hfk_fock_noalloc(int64_t natoms, const double *xyz, int32_t ngauss,
                            const double *exps_host, const double *coefs_host,
                            const double *dens, double tau, int32_t precision,
                            double *fock, double *e2, void *stream);

/* Backward of the forward outputs (G, E2) for upstream (g_fock, g_e2).  The paper has no
 * gradient; this is the derivative of what the forward defines, with the screening
 * decisions held fixed.  With W = (g_fock + g_fock^T)/2 (0 if g_fock is NULL) and
 * X = W + (g_e2 / 2) D:
 *   d_xyz  = sum_unique B_ijkl d(ij|kl)/dR,
 *            B = deg (4 (X_ij D_kl + D_ij X_kl) - (X_ik D_jl + D_ik X_jl) - (X_il D_jk + D_il X_jk)),
 *            which for g_fock = NULL is g_e2 * dE2/dR with Gamma = deg (4 D_ij D_kl - D_ik D_jl
 *            - D_il D_jk)
 *   d_dens = g_e2 G + G(W): dE2/dD = G (E2 is a symmetric bilinear form in D) and the map
 *            D -> G is linear and self-adjoint, so the pull-back of W is a Fock build with W
 *            as the density (run here when g_fock is given)
 * Inputs as hfk_fock plus
 *   g_e2     [1] upstream dL/dE2 (device)
 *   g_fock   [n*n] upstream dL/dG (device) or NULL
 *   fock_in  [n*n] G from the forward call on the same inputs; may be NULL when d_dens is
 * Outputs
 *   d_xyz    [n*3] (overwritten)
 *   d_dens   [n*n] or NULL (not computed)
 *   e2_out   [1] or NULL: E2 recomputed as sum_unique Gamma (ij|kl)
 * The workspace must be sized with with_grad != 0.  Errors as hfk_fock; HFK_EINVAL if
 * d_dens is given without fock_in. */
hfk_status hfk_fock_grad(int64_t natoms, const double *xyz, int32_t ngauss,
                         const double *exps_host, const double *coefs_host,
                         const double *dens, double tau, int32_t precision,
                         const double *g_e2, const double *g_fock, const double *fock_in,
                         double *d_xyz, double *d_dens, double *e2_out,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Per-atom bases: every atom carries a contracted s function of its own (all with ngauss
 * primitives), for instance hydrogen and helium in one system.  The integrals are those of
 * hfk_fock with each centre's own exponents and weights: the Gaussian product and the
 * primitive integral of the Background section hold for any exponent on any centre, and
 * one basis on every atom (the kernel listing) is the case of identical rows.
 * Workspace size for hfk_fock_atoms (with_grad = 0) or hfk_fock_grad_atoms (with_grad != 0);
 * arguments and errors as hfk_workspace_bytes. */
hfk_status hfk_workspace_bytes_atoms(int64_t natoms, int32_t ngauss, int32_t precision, int32_t with_grad,
                                     size_t *bytes_out);

/* Forward Fock build with per-atom bases.  Arguments, outputs and errors as hfk_fock except
 *   exps_host    [natoms*ngauss] row i: the exponents of atom i, each > 0 and finite (host)
 *   coefs_host   [natoms*ngauss] row i: the contraction coefficients of atom i, finite (host)
 *   workspace    at least hfk_workspace_bytes_atoms(...) bytes
 * Every row is validated on the host before any device work (HFK_EINVAL names the atom).
 * The rows are copied into the workspace before the call returns, so the host arrays may be
 * reused at once.  Only the hybrid form of the quartet kernel is built for this call
 * (hfk_set_config's variant does not apply); strategy and workgroups per CU follow
 * hfk_fock. */
hfk_status hfk_fock_atoms(int64_t natoms, const double *xyz, int32_t ngauss,
                          const double *exps_host, const double *coefs_host,
                          const double *dens, double tau, int32_t precision, int32_t strategy,
                          double *fock, double *e2,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Backward of hfk_fock_atoms: arguments, outputs and errors as hfk_fock_grad, with the
 * per-atom rows of hfk_fock_atoms; the workspace is sized by hfk_workspace_bytes_atoms with
 * with_grad != 0.  The pull-back of g_fock is a Fock build with per-atom bases. */
hfk_status hfk_fock_grad_atoms(int64_t natoms, const double *xyz, int32_t ngauss,
                               const double *exps_host, const double *coefs_host,
                               const double *dens, double tau, int32_t precision,
                               const double *g_e2, const double *g_fock, const double *fock_in,
                               double *d_xyz, double *d_dens, double *e2_out,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Self-consistent field around the two-electron build (closed shell).  The paper's kernel
 * is the electron-repulsion term of the Fock operator; this is the loop on either side of
 * it: core Hamiltonian H = T + V of contracted s functions with nuclear charges, symmetric
 * orthogonalisation X = S^(-1/2), F = H + G(D) with G from the screened build (per-atom
 * bases), energy E = 1/2 sum D o (H + F) + E_nn, orbitals of X F X, D = 2 C_occ C_occ^T
 * (the nocc lowest orbitals), DIIS on X (F D S - S D F) X over the last 8 iterations, until
 * |E - E_prev| < e_tol and max |X (F D S - S D F) X| < d_tol, or max_iter Fock builds.
 * Workspace size for hfk_scf; arguments and errors as hfk_workspace_bytes_atoms. */
hfk_status hfk_scf_workspace_bytes(int64_t natoms, int32_t ngauss, int32_t precision, size_t *bytes_out);

/*   natoms .. coefs_host   as hfk_fock_atoms (device xyz, host per-atom rows)
 *   charges_host     [natoms] nuclear charges Z, finite and >= 0 (host)
 *   nocc             doubly occupied orbitals, 0 .. natoms
 *   tau, precision   of the two-electron builds; strategy as hfk_fock (DETERMINISTIC makes
 *                    the whole loop repeat bit for bit)
 *   max_iter         >= 1; e_tol, d_tol > 0
 *   dens             [n*n] device: the starting density when use_guess != 0 (else the core
 *                    Hamiltonian's orbitals start), and on return the density of the last
 *                    build, whose energy is *energy_host
 *   orb_energies     [n] device or NULL: orbital energies of the final F, ascending
 *   energy_host, iterations_host, converged_host   host outputs (Fock builds taken; 1 when
 *                    both tolerances were met)
 *   workspace        hfk_scf_workspace_bytes(...) bytes, 256-byte aligned
 * The call waits for `stream` whenever the loop needs a number on the host and returns when
 * the loop has ended.  Dense products and eigenproblems run in rocBLAS and rocSOLVER with
 * their scratch taken from the workspace (HFK_ENOMEM if their own query asks for more).
 * Errors as hfk_fock_atoms; HFK_EUNSUPPORTED for a (nearly) singular overlap matrix; HFK_EHIP
 * also when an eigensolve does not converge (a Fock matrix or guess density with NaN or Inf). */
hfk_status hfk_scf(int64_t natoms, const double *xyz, const double *charges_host, int32_t ngauss,
                   const double *exps_host, const double *coefs_host, int32_t nocc, double tau,
                   int32_t precision, int32_t strategy, int32_t max_iter, double e_tol, double d_tol,
                   double *dens, int32_t use_guess, double *orb_energies, double *energy_host,
                   int32_t *iterations_host, int32_t *converged_host,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Workspace size for hfk_fock_batched over `nmol` molecules whose atom ranges are
 * atom_off_host[m] .. atom_off_host[m+1] (CSR, host memory, nondecreasing, starting at 0).
 * with_grad != 0 adds the gradient accumulators. */
hfk_status hfk_batched_workspace_bytes(int64_t nmol, const int64_t *atom_off_host,
                                       int32_t ngauss, int32_t precision, int32_t with_grad,
                                       size_t *bytes_out);

/* Ragged batch of independent molecules in one persistent launch.
 *   xyz          [sum n, 3] positions of all molecules, molecule m at rows
 *                atom_off_host[m] .. atom_off_host[m+1]
 *   dens_packed  the molecules' n_m x n_m densities stored one after another
 *                (molecule m starts at sum_{m'<m} n_m'^2)
 *   fock_packed  output, same packing as dens_packed
 *   e2           [nmol] output energies
 *   d_xyz        [sum n, 3] output dE2/dR, or NULL for a forward-only call
 * Each molecule needs 1 <= n_m <= 128 atoms (its matrices stay in LDS).
 * Errors as hfk_fock; HFK_EUNSUPPORTED for a molecule above 128 atoms. */
hfk_status hfk_fock_batched(int64_t nmol, const int64_t *atom_off_host, const double *xyz,
                            int32_t ngauss, const double *exps_host, const double *coefs_host,
                            const double *dens_packed, double tau, int32_t precision,
                            double *fock_packed, double *e2, double *d_xyz,
                            void *workspace, size_t workspace_bytes, void *stream);

/* Ragged batches with per-atom bases (see hfk_fock_atoms): workspace size, arguments and
 * errors as hfk_batched_workspace_bytes. */
hfk_status hfk_batched_workspace_bytes_atoms(int64_t nmol, const int64_t *atom_off_host,
                                             int32_t ngauss, int32_t precision, int32_t with_grad,
                                             size_t *bytes_out);

/* hfk_fock_batched with per-atom bases:
 *   exps_host    [sum n * ngauss] row a: the exponents of stacked atom a (molecule m's atoms
 *                are rows atom_off_host[m] .. atom_off_host[m+1]), each > 0 and finite
 *   coefs_host   [sum n * ngauss] the matching contraction coefficients, finite
 * Every row is validated on the host and copied into the workspace before the call returns.
 * Other arguments, outputs and errors as hfk_fock_batched; the workspace is sized by
 * hfk_batched_workspace_bytes_atoms. */
hfk_status hfk_fock_batched_atoms(int64_t nmol, const int64_t *atom_off_host, const double *xyz,
                                  int32_t ngauss, const double *exps_host, const double *coefs_host,
                                  const double *dens_packed, double tau, int32_t precision,
                                  double *fock_packed, double *e2, double *d_xyz,
                                  void *workspace, size_t workspace_bytes, void *stream);

/* Waits for `stream`, then copies the counters of the last build made with `workspace`
 * into *out.  Errors: HFK_EINVAL for NULL arguments, HFK_EHIP. */
hfk_status hfk_read_stats(const void *workspace, void *stream, hfk_stats *out);

/* The counters of the last successful build call made on this thread (hfk_fock*,
 * hfk_fock_grad*, hfk_fock_batched*): waits for that call's stream and reads its workspace,
 * which must still be allocated.  Errors: HFK_EINVAL for NULL out or when this thread has
 * made no build call, HFK_EHIP. */
hfk_status hfk_last_stats(hfk_stats *out);

/* Debug mode, process-wide, off by default.  While it is on, every call that takes a
 * density (hfk_fock*, hfk_fock_grad* for dens and g_fock, hfk_fock_batched* per molecule,
 * hfk_scf for a guess density) first checks it on the device, waits for `stream`, and
 * refuses it before any build work:
 *   HFK_EINVAL    an entry is NaN or infinite;
 *   HFK_ENOTSYM   some |D_ij - D_ji| > sym_tol * max_ij |D_ij| (per molecule for batches;
 *                 the message names the largest difference, and the first molecule).
 * sym_tol must be finite and >= 0 (0 asks for exact symmetry).  Errors: HFK_EINVAL. */
hfk_status hfk_set_debug(int32_t on, double sym_tol);

/* Autotuner of the forward build.  Times hfk_fock on the given system on `stream` and
 * searches the launch configuration one dimension at a time, starting from the untuned
 * default and keeping a candidate only when it beats the best so far:
 *   persistent workgroups per compute unit 1..6 (capped at what fits on a CU),
 *   quartet-tile shape: items per block {1, 2, 4, 8, 16} x bras per group {256 .. 4096},
 *   ket-side Coulomb vectors {one per workgroup, 8 shared, 32 shared},
 *   accumulation strategy {ATOMIC, PRIVATE}, quartet-kernel variant {hybrid, direct}.
 * The result is kept for the rest of the process under (device architecture, precision,
 * size bucket ceil(log2 natoms)) and written to cache_path as JSON when cache_path is not
 * NULL (with every other tuned entry of the process).  best_out (may be NULL) receives the
 * chosen hfk_strategy.  Inputs and workspace as hfk_fock (fock and e2 are overwritten).
 * Waits for `stream`.  Errors as hfk_fock. */
hfk_status hfk_tune(int64_t natoms, const double *xyz, int32_t ngauss,
                    const double *exps_host, const double *coefs_host,
                    const double *dens, double tau, int32_t precision,
                    double *fock, double *e2, void *workspace, size_t workspace_bytes,
                    void *stream, const char *cache_path, int32_t *best_out);

/* Autotuner of the batched path: times hfk_fock_batched on the given batch, one dimension
 * at a time from the untuned default: waves per workgroup {8, 4}, persistent workgroups per
 * compute unit 1..4, items (256 kets) per block {auto, 8, 16, 32, 64, 128}, and the
 * accumulation strategy {shared: blocks of a molecule added to G with atomics; owned:
 * molecules up to a work bound run whole in one workgroup and are stored without atomics,
 * bound {2^14, 2^16, 2^18} quartets}.  Keeps the fastest for the rest of the process under (device
 * architecture, precision), writes the table to cache_path when it is not NULL, and
 * returns the chosen workgroups per CU in best_gpc_out (may be NULL).  Arguments as
 * hfk_fock_batched (outputs overwritten). */
hfk_status hfk_tune_batched(int64_t nmol, const int64_t *atom_off_host, const double *xyz,
                            int32_t ngauss, const double *exps_host, const double *coefs_host,
                            const double *dens_packed, double tau, int32_t precision,
                            double *fock_packed, double *e2, double *d_xyz,
                            void *workspace, size_t workspace_bytes, void *stream,
                            const char *cache_path, int32_t *best_gpc_out);

/* Loads a table written by hfk_tune / hfk_tune_batched (JSON); entries for another device
 * architecture are kept but not used on this one.  Errors: HFK_EINVAL (NULL, unreadable,
 * not such a table, or an entry out of range). */
hfk_status hfk_load_tuning(const char *cache_path);

/* Forgets every tuned entry of the process (the untuned defaults apply again). */
hfk_status hfk_clear_tuning(void);

/* Process-wide override of the launch configuration of hfk_fock, for tuning and tests:
 *   variant          0 = every primitive quartet evaluates the Boys function in place,
 *                    1 = near/far split with per-wave compaction of near-field quartets,
 *                   -1 = library choice (default: tuned value, else 1)
 *   groups_per_cu    persistent workgroups per compute unit, 1..6, or 0 for the default
 *                    (also the gradient kernel's count of hfk_fock_grad, capped at what fits)
 * Errors: HFK_EINVAL for values outside these sets. */
hfk_status hfk_set_config(int32_t variant, int32_t groups_per_cu);

/* Process-wide override of the quartet-tile shape of hfk_fock and hfk_fock_atoms (and of
 * the gradient kernel and pull-back build of hfk_fock_grad; not of the deterministic
 * strategy), for tuning and tests:
 *   tile_items     items of 1024 kets per block of one bra, 1..16 (0: library choice)
 *   group_bras     bras per group whose blocks are numbered ket-block-major: 256, 512,
 *                  1024, 2048 or 4096 (0: library choice)
 *   ket_copies     copies of the ket-side Coulomb vector: 1..1024 shared copies updated
 *                  with atomics (workgroup w uses copy w mod ket_copies), 0 for one per
 *                  workgroup with plain updates (fewer, shared, when they exceed the memory
 *                  budget), or -1 for the library's choice
 * hfk_set_shape(0, 0, -1) returns to the library's choices.  Errors: HFK_EINVAL for values
 * outside these sets. */
hfk_status hfk_set_shape(int32_t tile_items, int32_t group_bras, int32_t ket_copies);

/* Process-wide override of the batched launch, for tuning and tests; 0 keeps the library's
 * choice:
 *   groups_per_cu  persistent workgroups per compute unit, 1..4 (capped at what fits)
 *   block_items    items of 256 kets per fetched block of a shared molecule, 1..1024
 *   owned_bound    -1: every molecule is split into blocks (shared accumulation);
 *                  k > 0: molecules with at most k unique quartets before screening run
 *                  whole in one workgroup and store G and the gradient without atomics
 *   waves          waves per workgroup, 4 or 8
 * hfk_set_batched_config(0, 0, 0, 0) returns to the library's choices.  Errors: HFK_EINVAL
 * for values outside these sets. */
hfk_status hfk_set_batched_config(int32_t groups_per_cu, int32_t block_items, int64_t owned_bound, int32_t waves);

/* Kernel timing for measurement tools: while enabled, every call records a pair of HIP
 * events on its stream around each launch of its quartet kernel (the dominant kernel: the
 * forward, gradient or batched kernel; a gradient call with g_fock records its pull-back
 * build too).  hfk_profile_read
 * waits for the recorded events, returns the summed duration in milliseconds and the
 * number of launches timed, and clears the record.  Process-wide; not thread-safe against
 * concurrent builds.  Errors: HFK_EINVAL (NULL outputs), HFK_EHIP. */
hfk_status hfk_profile_enable(int32_t on);
hfk_status hfk_profile_read(double *total_ms, int64_t *launches);

/* Message of the last failing call on this thread ("" if none). */
const char *hfk_last_error(void);

/* Library version string. */
const char *hfk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HFK_H */
