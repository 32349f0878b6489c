// Internal declarations of libhfk: workspace layout, basis tables, launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hfk.h"

namespace hfk {

constexpr int kMaxG = HFK_MAX_NGAUSS;
constexpr int kMaxG2 = kMaxG * kMaxG;

// Pairs are ordered by (Q band, spatial cell of the pair centre): band b holds
// 2^(1-(b+1)/R) <= Q < 2^(1-b/R) with R bands per octave; within a band, cells follow a
// Morton curve over the bounding box (kCellBits per axis), so 64 consecutive kets sit
// close together in space.  Wide bands (two octaves) put more pairs in a band, so a
// wave's kets are closer together and fewer waves straddle the near/far switch, for a
// few more kets that fail the lane-level screen at the end of a bra's prefix.
constexpr double kBandsPerOctave = 0.5;
constexpr int kNumBands = 128;
constexpr int kCellBits = 4;
constexpr int kNumCells = 1 << (3 * kCellBits);
constexpr int kNumBuckets = kNumBands * kNumCells;

// Boys function table of H(T) = erf(sqrt T)/sqrt T = (2/sqrt(pi)) F0(T) about T_k = k h,
// k = 0 .. kBoysGrid-1: row k holds c_n with H(T) ~ sum_n c_n (T - T_k)^n for |T - T_k| <= h/2.
// FP64 rows are of degree 5, the Chebyshev economisation of the degree-7 Taylor row (whose
// coefficients are (2/sqrt(pi)) (-1)^n F_n(T_k) / n!): on the interval the dropped degree-6
// and degree-7 terms are replaced by their lower-degree Chebyshev parts, which leaves an
// error near 2e-14 where the degree-5 Taylor row would leave 5e-13.  Six coefficients are 48
// bytes, three 16-byte LDS reads.
constexpr int kBoysOrder = 6;          // coefficients used (degree 5)
constexpr int kBoysStride = 6;         // row length (48 bytes: 16-byte aligned rows)
constexpr double kBoysH = 1.0 / 12.0;  // grid spacing
constexpr double kBoysInvH = 12.0;
constexpr double kTswitch = 32.0;      // above this H(T) = T^(-1/2) to < 1e-15 relative
constexpr double kSqrtSwitchInvH = 19.595917942265423;   // sqrt(kTswitch / h) = sqrt(384)
constexpr int kBoysGrid = 393;         // covers [0, 32.75): rows up to kTswitch / h and 8 more
// The FP32 paths use a finer grid with a shorter expansion: degree 3 at h = 1/16 leaves a
// Taylor remainder below 1e-8 relative (under FP32 rounding), and a row of four
// coefficients is one 16-byte LDS read.  The rows are computed in FP64 and rounded once.
constexpr int kBoysOrderF = 4;
constexpr int kBoysStrideF = 4;
constexpr double kBoysHF = 0.0625;
constexpr double kBoysInvHF = 16.0;
constexpr double kSqrtSwitchInvHF = 22.627416997969522;   // sqrt(kTswitch / hF) = sqrt(512)
constexpr int kBoysGridF = 536;        // covers [0, 33.5)

// Table geometry of each precision (rows, coefficients per row, grid spacing).
template <typename R> struct BoysGrid;
// Gradient tables.  FP64: since g(T) = -(4/sqrt(pi)) F1(T) = 2 H'(T), one row of H of
// degree 7 (kBoysOrderG coefficients) gives both: its value, and its derivative, which is
// exactly the degree-6 Taylor expansion of g about the same point; rows of kBoysStrideG
// values (a pad: 72-byte rows of 18 dwords start on 32 different banks).  FP32: H's and g's
// rows of degree 3 in two tables of 16-byte rows (g's at a constant offset, within
// ds_read_b128's 16-bit offset), since the derivative of a degree-3 row would leave g at
// degree 2, short of FP32 accuracy.  pair_stride: values per row step; g_off: g's row after
// H's (-1: derived); table_len: values in all.
constexpr int kBoysOrderG = 8;
constexpr int kBoysStrideG = 9;
template <> struct BoysGrid<double> {
    static constexpr int rows = kBoysGrid, stride = kBoysStride, order = kBoysOrder, pair_stride = kBoysStrideG;
    static constexpr int g_off = -1, table_len = rows * pair_stride;
    static constexpr double h = kBoysH, inv_h = kBoysInvH, sqrt_sw_inv_h = kSqrtSwitchInvH;
};
template <> struct BoysGrid<float> {
    static constexpr int rows = kBoysGridF, stride = kBoysStrideF, order = kBoysOrderF, pair_stride = 4;
    static constexpr int g_off = rows * stride, table_len = 2 * rows * stride;
    static constexpr double h = kBoysHF, inv_h = kBoysInvHF, sqrt_sw_inv_h = kSqrtSwitchInvHF;
};

constexpr int kWave = 64;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupThreads = kWave * kWavesPerGroup;
constexpr int kKetsPerItem = kGroupThreads;   // one 64-ket chunk per wave per item
// Single-molecule items: (bra, kItemKets kets); each wave takes kWaveKets of them and runs
// them as kSubChunks 64-lane chunks.
constexpr int kSubChunks = 4;
constexpr int kWaveKets = kWave * kSubChunks;
constexpr int kItemKets = kWavesPerGroup * kWaveKets;
constexpr int kBlockItems = 16;  // items per dynamically fetched block of the quartet kernels
// Batched kernel: items of kKetsPerItem kets are cut into units of one wave's 64 kets; the
// workgroup has 4 or 8 waves (set at launch, at most kBatchMaxThreads threads); the bra table
// holds kBBra values per primitive pair (Px Py Pz S, mu S, fa S, fb S, fa fb S, fb^2 S, pad).
constexpr int kUnitsPerItem = kKetsPerItem / kWave;
constexpr int kBatchMaxThreads = 512;
constexpr int kBBra = 12;
// Gradient bra weights per primitive pair of the single-molecule tables.
constexpr int kGW = 8;
// Single-molecule blocks: kTileItems items of one bra (twice as many with FP32 ket data).
// Bras are taken kGroupBras at a time and their blocks are numbered ket-block-major (block
// K of every bra of the group, then block K+1), so the workgroups running at the same
// moment read the same few thousand kets and the ket table is served from L2 instead of
// streaming past it.  Four FP64 items (4096 kets, 1.5 MB of ket data) fit next to the rest
// in an XCD's 4 MB L2: fabric reads per launch at 512 atoms are 30 GB against 105 GB with
// eight items and 220 GB with sixteen; two or three items cut reads further but flush rows
// more often and run slower.  The FP32 ket table is half the size, and eight items are the
// faster choice there.
constexpr int kTileItems = 4;
constexpr int kGroupBras = 1024;
// Bras per group are a power of two in [kMinGroupBras, kMaxGroupBras] (tuned); the group
// tables are sized for the smallest.
constexpr int kMinGroupBras = 256;
constexpr int kMaxGroupBras = 4096;
constexpr int kMaxTileItems = 16;

// Device-side counters written by the build and read back by hfk_read_stats.
struct DevHeader {
    unsigned long long qmax_bits;   // max Q as the bit pattern of a positive double
    int sig_pairs;
    int pad0;
    long long items;
    unsigned long long quartets;
    double centroid[3];
    double bmin[3];
    double bmax[3];
    int strategy;
    int groups;
    int precision;
    int natoms;
    int variant;
    int max_bucket;                 // most pairs in one (band, cell) bucket (fixed pair order only)
    unsigned long long next_block;  // work counter of the quartet kernels (blocks of items)
    long long blocks;               // blocks of the single-molecule kernels (empty ones included)
    int tile;                       // launch shape of the last build (for the stats)
    int group_bras;
    int ket_copies;
    int pad1;
    // batched block table: owned-molecule blocks, shared blocks, items per shared block
    long long bt_own;
    long long bt_sh;
    long long bsz;
    // debug check of the density (hfk_set_debug): bit patterns of non-negative doubles
    unsigned long long dchk_asym;   // max |D_ij - D_ji| (single molecule)
    unsigned long long dchk_max;    // max |D_ij| (single molecule)
    unsigned long long dchk_ratio;  // max over molecules of max|D_ij - D_ji| / max|D_ij| (batched)
    unsigned long long dchk_bad;    // non-finite entries
    int dchk_mol;                   // first molecule over the tolerance (batched), or INT_MAX
    int dchk_badmol;                // first molecule with a non-finite entry (batched), or INT_MAX
};

// Basis constants shared by every pair, computed on the host from exps/coefs and passed
// by value.  ab = a * g + b indexes a primitive pair.  With per-atom bases, aexp and aw
// point at device rows [n][g] of exponents and weights (primitive a on atom i at
// i * g + a) and alpha/w are unused; for one basis on every atom they are NULL.
struct Basis {
    int g;
    int g2;
    double alpha[kMaxG];
    double w[kMaxG];            // c_a (2 alpha_a / pi)^(3/4)
    const double *aexp;
    const double *aw;
};

// Per primitive pair / quartet constants, in device memory (written by a setup kernel).
struct BasisDev {
    double p[kMaxG2];           // alpha_a + alpha_b
    double mu[kMaxG2];          // alpha_a alpha_b / p
    double fa[kMaxG2];          // alpha_a / p
    double fb[kMaxG2];          // alpha_b / p
    double pi32[kMaxG2];        // (pi / p)^(3/2)
    double rho[kMaxG2 * kMaxG2];    // p q / (p + q), [ab * g2 + cd]
    double srho[kMaxG2 * kMaxG2];   // sqrt(rho)
    double r2sw[kMaxG2 * kMaxG2];   // kTswitch / rho: |P-Q|^2 beyond which the far field is exact
    double rs[3 * kMaxG2 * kMaxG2];     // (rho, sqrt(rho), kTswitch / rho) interleaved
    float rs_f[3 * kMaxG2 * kMaxG2];
    double rsn[3 * kMaxG2 * kMaxG2];    // (kTswitch / rho, rho / h, sqrt(rho / h)): T on the table grid
    float rsn_f[3 * kMaxG2 * kMaxG2];   // the same on the FP32 grid (h = kBoysHF)
    double rsg[4 * kMaxG2 * kMaxG2];    // (kTswitch / rho, rho / h, sqrt(rho / h), (rho / h)^(3/2))
    float rsg_f[4 * kMaxG2 * kMaxG2];   // the same on the FP32 grid
    float rho_f[kMaxG2 * kMaxG2];
    float srho_f[kMaxG2 * kMaxG2];
    float r2sw_f[kMaxG2 * kMaxG2];
};

// Workspace layout of the single-molecule path.  Every offset is 256-byte aligned.
struct Layout {
    int64_t n, npair, pcap;     // pcap = npair rounded up to 64, plus one spare chunk
    int g, g2, groups;          // groups: persistent workgroups the buffers are sized for
    int tile;                   // items per block (kTileItems, doubled for FP32 ket data; tuned)
    int gshift;                 // log2 of the bras per group (tuned)
    int kcopies;                // ket-side Coulomb vectors requested (0: one per workgroup)
    bool private_ok;            // per-workgroup copies of F fit the memory budget
    size_t hdr, basis, boys, boys_f;
    size_t q_unsorted, bucket_of, bucket_cnt, bucket_off, bucket_cur;
    size_t pk, pl, pq, pd;                 // sorted pair tables
    size_t prim;                           // [5][g2][pcap] doubles: Px, Py, Pz, S, |P|^2 (+ kTswitch/p per-atom)
    size_t prim_f;                         // [4][g2][pcap] floats (mixed) (+ kTswitch/p per-atom)
    bool atoms;                            // per-atom bases: the tables below are present
    size_t arow;                           // [2][n][g] exponents and weights of every atom
    size_t bip, bip_f;                     // [pcap][g2] kTswitch/p of every bra primitive pair
    size_t pmu, pfa;                       // per-atom gradient: [g2][pcap] mu and a/p of the ket pairs
    size_t bgw, bgw_f;                     // gradient: [pcap][g2][kGW] bra weights mu S, fa S, fb S, fa fb S, fb^2 S
    size_t bra, bra_f;                     // [pcap][g2][8] Px Py Pz S -2Px -2Py -2Pz |P|^2 (wave-uniform bra data)
    size_t boys_g, boys_g_f;               // gradient tables: H of degree 7 (FP64), g(T) = -(4/sqrt(pi)) F1(T) (FP32 grid)
    size_t nitems, lim, item_off, scan_tmp;
    size_t gcnt, goff;                     // per bra group: blocks, and their exclusive prefix
    int64_t ngroups;                       // bra groups of 2^gshift bras
    int64_t ngroups_cap;                   // groups the tables hold (groups of kMinGroupBras)
    size_t fpriv;                          // [groups][n*n] or [n*n]
    size_t jcol;                           // [jcopies][pcap] ket-side Coulomb vectors
    int jcopies;                           // copies of the ket vector (one per workgroup while they fit)
    size_t fsum;                           // [n*n]
    size_t e2part;                         // partial energies
    size_t xw;                             // gradient with dL/dG: W and X, [2][n*n]
    size_t e2tmp;                          // one double of scratch
    size_t grad;                           // [groups][n*3] gradient accumulators
    size_t total;
};

// compact: the layout of the allocation-free call (one F for the atomics strategy, at most
// kCompactKetCopies shared ket vectors).
constexpr int kCompactKetCopies = 8;
Layout make_layout(int64_t n, int g, int prec, int with_grad, int groups, bool atoms = false, bool compact = false);
// Ket-side Coulomb vectors a build uses: one per workgroup within the memory budget, or the
// requested number of shared copies when that is smaller.
inline int effective_copies(const Layout &L)
{
    int c = L.jcopies < L.groups ? L.jcopies : L.groups;
    if (L.kcopies > 0 && L.kcopies < c) c = L.kcopies;
    return c;
}

// Sets the quartet-tile shape of a layout: items per block, bras per group (a power of two
// in [kMinGroupBras, kMaxGroupBras]) and the requested ket-side Coulomb vector copies.
void set_shape(Layout &L, int tile, int group_bras, int ket_copies);

// Workspace layout of the batched path.
struct BLayout {
    int64_t nmol, ptot, ntot, pcap;
    int64_t tri;                // sum of n (n + 1) / 2: entries of the packed triangles
    int g, g2, nmax;
    size_t hdr, basis, boys, boys_f, boys_g, boys_g_f;
    size_t mol_n, mol_aoff, mol_poff, mol_doff, mol_toff, cent, qmax;
    size_t q, bucket_of, bcnt, boff, bcur;
    size_t pk, pl, pm, pq, pd, prim, prim_f, bra, bra_f;
    size_t nitems, lim, klo, item_off, scan_tmp;
    size_t facc, gacc;
    size_t mol_i0, mol_i1;              // per molecule: first and end item
    size_t cnt_own, cnt_sh, off_own, off_sh;   // per molecule: blocks of each kind and their prefix
    bool atoms;                 // per-atom bases: ket component 4 is kTswitch/p, tables below
    size_t arow;                // [2][sum n][g] exponents and weights of every atom
    size_t bip, bip_f;          // [pcap][g2] kTswitch/p of the bra pairs
    size_t kmu, kfa;            // per-atom gradient: [g2][pcap] ket mu and a/p
    size_t total;
};

BLayout make_blayout(int64_t nmol, const int64_t *atom_off, int g, int with_grad, bool atoms = false);
size_t batched_smem_bytes(int nmax, int prec);
// Launch configuration of the batched kernel: block_items 0 = automatic (total items /
// (8 x workgroups), clamped to [16, 64]); owned_bound > 0: molecules with at most that many
// unique quartets before screening run whole in one workgroup (plain stores), -1: none.
struct BatchedShape {
    int gpc;
    int block_items;
    long long owned_bound;
    int waves;                  // waves per workgroup (4 or 8)
};
// Copies the per-molecule tables (atom counts, offsets) into the workspace and waits for
// the copies (their host staging ends with the call).
hipError_t upload_batch_tables(const BLayout &L, char *ws, const int64_t *atom_off_host, hipStream_t st);
hipError_t launch_batched(const BLayout &L, const Basis &b, char *ws, const int64_t *atom_off_host, const double *xyz,
                          const double *dens, double tau, int prec, double *fock, double *e2, double *d_xyz,
                          int groups, const BatchedShape &shape, hipStream_t st);
int batched_resident_groups(int g, int prec, bool grad, bool atoms, int nmax, int waves);
// Debug check of densities on the device (results in the header's dchk fields, which the
// first launch clears): one row-major n x n matrix, or nmol matrices at mol_doff with sizes
// mol_n (device arrays), each compared against tol times its own largest entry.
hipError_t launch_dens_check(DevHeader *hdr, int64_t n, const double *dens, hipStream_t st);
hipError_t launch_dens_check_batched(DevHeader *hdr, int64_t nmol, const long long *mol_doff, const int *mol_n,
                                     const double *dens, double tol, hipStream_t st);
// Pads the batched pair tables (four-component ket table, plus kTswitch/p with per-atom
// bases; kmu/kfa: per-atom gradient tables or NULL) past the last pair.
hipError_t launch_pair_pad(const DevHeader *hdr, int64_t pcap, int g2, bool atoms, int *pk, int *pl, double *pq,
                           double *pd, double *prim, float *prim_f, double *kmu, double *kfa, hipStream_t st);

int device_cu_count();

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error; all enqueue on `st`.
hipError_t launch_setup(const Basis &b, BasisDev *bd, double *boys, double *boys_f, double *boys_g,
                        double *boys_g_f, DevHeader *hdr, int64_t n, const double *xyz, hipStream_t st);
hipError_t launch_zero_counter(unsigned long long *p, hipStream_t st);
// fixed_order: pairs within a (band, cell) bucket by pair index (deterministic strategy)
// instead of the order an atomic cursor hands out.  That mode waits for the stream once to
// read the largest bucket and returns hipErrorNotSupported, before sorting, when it holds
// more than kMaxFixedBucket pairs.
constexpr int kMaxFixedBucket = 4096;
hipError_t launch_pairs(const Layout &L, const Basis &b, char *ws, const double *xyz, const double *dens,
                        double tau, hipStream_t st, bool fixed_order = false);
hipError_t launch_fock(const Layout &L, const Basis &b, char *ws, const double *dens, double tau,
                       int prec, int strategy, int variant, double *fock, double *e2, hipStream_t st);
size_t fock_smem_bytes(int64_t n, int prec, int variant);
int fock_resident_groups(int g, int prec, int variant, int64_t n, bool atoms = false, bool det = false);
// Events around the quartet kernel when profiling is enabled (no-ops otherwise).
void profile_begin(hipStream_t st);
void profile_end(hipStream_t st);

hipError_t launch_header_info(char *hdr, int strategy, int groups, int precision, int variant,
                              hipStream_t st, int tile = 0, int group_bras = 0, int ket_copies = 0);
hipError_t launch_scan(const long long *in, int64_t m, long long *out, long long *tmp, long long *total,
                       hipStream_t st);
// Gradient kernel and its reductions.  xdens: X of the two-density contraction (see
// hfk_fock_grad), or NULL for g_e2 * dE2/dR.  d_dens here is g_e2 * fock_in only; the
// caller adds G(W) for an upstream dL/dG.
hipError_t launch_grad(const Layout &L, const Basis &b, char *ws, const double *xyz, const double *dens,
                       double tau, int prec, const double *g_e2, const double *xdens, const double *fock_in,
                       double *d_xyz, double *d_dens, double *e2_out, hipStream_t st);
// W = (gF + gF^T)/2 and X = W + (g_e2/2) D into xw[0 .. n*n) and xw[n*n .. 2 n*n).
hipError_t launch_make_xw(int64_t n, const double *dens, const double *g_fock, const double *g_e2, double *xw,
                          hipStream_t st);
// y += g_e2 * x over m values.
hipError_t launch_axpy_dev(int64_t m, const double *g_e2, const double *x, double *y, hipStream_t st);
size_t grad_smem_bytes(int64_t n, int prec);
int grad_resident_groups(int g, int prec, int64_t n, bool atoms);

}  // namespace hfk
