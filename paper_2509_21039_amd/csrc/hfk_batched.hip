// Ragged batches of independent molecules in one persistent launch, forward Fock build and
// (optionally) the nuclear gradient fused into the same primitive loop.
//
// Pairs of every molecule are prepared in one pass and stored in (molecule, Q band) order;
// a bra's kets are the molecule's pairs up to its screen limit (t <= s keeps each quartet
// once).  Items of 256 kets are numbered molecule by molecule.  Workgroups fetch blocks from
// a global counter through a block table with two kinds of blocks:
//   owned:  all items of one molecule (molecules up to a tuned work bound), fetched first;
//   shared: up to bsz consecutive items of one molecule.
// A workgroup keeps the current molecule's whole two-electron matrix in LDS (lower
// triangle, the symmetrisation G = (F + F^T)/2 folded in: F_xy and F_yx land in the same
// slot) and its n x 3 gradient.  At the end of an owned block they are stored as they are
// (no other workgroup touches that molecule); at the end of a shared block they are added
// to the global accumulators with atomics.  Per primitive quartet the loop forms E(r) (the integral) and
// W(r) = E'(r)/r (its radial derivative) from the same r^2, so the forward result and the
// gradient come out of one pass over the quartets.
//
// Per-atom bases (kAtoms): pair bounds and tables come from the atom rows; the ket table's
// component 4 and a per-bra uniform array hold kTswitch / p, whose sum is the quartet's
// switch radius^2, and near steps derive rho from it (as in the single-molecule kernels).
#include <string.h>

#include <vector>

#include "hfk_device.hpp"

namespace hfk {

struct BArgs {
    const DevHeader *hdr;
    const BasisDev *bd;
    const double *tabH;
    const double *tabH_f;   // rows of the FP32 grid (FP64 values)
    const double *tabG;
    const double *tabG_f;
    const int *pk;
    const int *pl;
    const int *pm;
    const double *pq;
    const double *pd;
    const double *prim;
    const float *prim_f;
    const double *bra;
    const float *bra_f;
    const double *bip;      // per-atom bases: [pcap][g2] kTswitch / p of the bra pairs (and FP32)
    const float *bip_f;
    const double *kmu;      // per-atom gradient: [g2][pcap] ket mu and a/p
    const double *kfa;
    const long long *item_off;
    const int *lim;
    const int *klo;
    const int *mol_n;
    const long long *mol_aoff;
    const long long *mol_doff;
    const long long *mol_toff;
    const double *xyz;
    const double *dens;
    double *facc;        // packed lower triangles, molecule m at mol_toff[m]
    double *gacc;        // [sum n][3]
    const long long *off_own;   // [nmol + 1] exclusive prefix of owned blocks per molecule
    const long long *off_sh;    // [nmol + 1] exclusive prefix of shared blocks per molecule
    const long long *mol_i0;    // [nmol] first item of each molecule
    const long long *mol_i1;    // [nmol] end of its items
    int nmol;
    unsigned long long *quartets;
    unsigned long long *next_block;
    int64_t pcap;
    double tau;
    int nmax;
};

template <typename R> struct BPrec;
template <> struct BPrec<double> {
    static __device__ const double *prim(const BArgs &a) { return a.prim; }
    static __device__ const double *bra(const BArgs &a) { return a.bra; }
    static __device__ const double *bip(const BArgs &a) { return a.bip; }
    static __device__ const double *rsg(const BasisDev *bd) { return bd->rsg; }
};
template <> struct BPrec<float> {
    static __device__ const float *prim(const BArgs &a) { return a.prim_f; }
    static __device__ const float *bra(const BArgs &a) { return a.bra_f; }
    static __device__ const float *bip(const BArgs &a) { return a.bip_f; }
    static __device__ const float *rsg(const BasisDev *bd) { return bd->rsg_f; }
};

__device__ inline int tri(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

// Last m in [0, nmol) with off[m] <= p: the molecule whose range of a prefix sum holds p
// (molecules with an empty range share their offset with the next one and are skipped).
__device__ inline int mol_of(const long long *__restrict__ off, int nmol, long long p)
{
    int lo = 0, hi = nmol - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ pair preparation

__global__ void k_b_mol(int nmol, const int *__restrict__ nm, const long long *__restrict__ aoff,
                        const double *__restrict__ xyz, double *__restrict__ cent, unsigned long long *__restrict__ qmax)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol) return;
    double c[3] = {0, 0, 0};
    for (int i = 0; i < nm[m]; ++i)
        for (int d = 0; d < 3; ++d) c[d] += xyz[3 * (aoff[m] + i) + d];
    for (int d = 0; d < 3; ++d) cent[3 * m + d] = c[d] / nm[m];
    qmax[m] = 0;
}

__global__ __launch_bounds__(256) void k_b_pair_q(Basis b, const BasisDev *__restrict__ bd, int nmol,
                                                  const long long *__restrict__ poff,
                                                  const long long *__restrict__ aoff,
                                                  const double *__restrict__ cent, const double *__restrict__ xyz,
                                                  long long ptot, double *__restrict__ qout,
                                                  unsigned long long *__restrict__ qmax)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ptot) return;
    const int m = mol_of(poff, nmol, p);
    int64_t i, j;
    pair_of_index(p - poff[m], i, j);
    const double *c = cent + 3 * m;
    const double *xa = xyz + 3 * (aoff[m] + i), *xb = xyz + 3 * (aoff[m] + j);
    double A[3] = {xa[0] - c[0], xa[1] - c[1], xa[2] - c[2]};
    double B[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
    double px[kMaxG2], py[kMaxG2], pz[kMaxG2], ps[kMaxG2], pp[kMaxG2];
    double s = 0.0;
    if (b.aexp) {
        pair_prims_atoms(b, aoff[m] + i, aoff[m] + j, A, B, px, py, pz, ps, pp);
        for (int ab = 0; ab < b.g2; ++ab)
            for (int cd = 0; cd < b.g2; ++cd) {
                const double dx = px[ab] - px[cd], dy = py[ab] - py[cd], dz = pz[ab] - pz[cd];
                const double rho = pp[ab] * pp[cd] / (pp[ab] + pp[cd]);
                s += ps[ab] * ps[cd] * sqrt(rho) * erf_over_sqrt(rho * (dx * dx + dy * dy + dz * dz));
            }
    } else {
        pair_prims(b, bd, A, B, px, py, pz, ps);
        for (int ab = 0; ab < b.g2; ++ab)
            for (int cd = 0; cd < b.g2; ++cd) {
                const double dx = px[ab] - px[cd], dy = py[ab] - py[cd], dz = pz[ab] - pz[cd];
                s += ps[ab] * ps[cd] * bd->srho[ab * b.g2 + cd] *
                     erf_over_sqrt(bd->rho[ab * b.g2 + cd] * (dx * dx + dy * dy + dz * dz));
            }
    }
    const double q = sqrt(s);
    qout[p] = q;
    atomicMax(&qmax[m], (unsigned long long)__double_as_longlong(q));
}

__global__ __launch_bounds__(256) void k_b_bucket_count(int nmol, const long long *__restrict__ poff, long long ptot,
                                                        double tau, const unsigned long long *__restrict__ qmax,
                                                        const double *__restrict__ q, int *__restrict__ bucket_of,
                                                        long long *__restrict__ cnt)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ptot) return;
    const int m = mol_of(poff, nmol, p);
    const double qm = __longlong_as_double((long long)qmax[m]);
    const double qp = q[p];
    int bk = -1;
    if (qp * qm >= tau && qp > 0.0) {
        bk = m * kNumBands + q_band(qp);
        atomicAdd((unsigned long long *)&cnt[bk], 1ULL);
    }
    bucket_of[p] = bk;
}

__global__ __launch_bounds__(256) void k_b_cursors(const long long *__restrict__ off, long long nb, int *__restrict__ cur,
                                                   DevHeader *__restrict__ hdr)
{
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) cur[b] = (int)off[b];
    if (b == 0) {
        hdr->sig_pairs = (int)off[nb];
        hdr->quartets = 0;
    }
}

__global__ __launch_bounds__(256) void k_b_pair_scatter(
    Basis b, const BasisDev *__restrict__ bd, int nmol, const long long *__restrict__ poff,
    const long long *__restrict__ aoff, const long long *__restrict__ doff, const int *__restrict__ nm,
    const double *__restrict__ cent, const double *__restrict__ xyz, const double *__restrict__ dens, long long ptot,
    int64_t pcap, const double *__restrict__ q, const int *__restrict__ bucket_of, int *__restrict__ cur,
    int *__restrict__ pk, int *__restrict__ pl, int *__restrict__ pm, double *__restrict__ pq, double *__restrict__ pd,
    double *__restrict__ prim, float *__restrict__ prim_f, double *__restrict__ bra, float *__restrict__ bra_f,
    double *__restrict__ bip, float *__restrict__ bip_f, double *__restrict__ kmu, double *__restrict__ kfa)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ptot) return;
    const int bk = bucket_of[p];
    if (bk < 0) return;
    const int pos = atomicAdd(&cur[bk], 1);
    const int m = bk / kNumBands;
    int64_t i, j;
    pair_of_index(p - poff[m], i, j);
    const double *c = cent + 3 * m;
    const double *xa = xyz + 3 * (aoff[m] + i), *xb = xyz + 3 * (aoff[m] + j);
    double A[3] = {xa[0] - c[0], xa[1] - c[1], xa[2] - c[2]};
    double B[3] = {xb[0] - c[0], xb[1] - c[1], xb[2] - c[2]};
    double px[kMaxG2], py[kMaxG2], pz[kMaxG2], ps[kMaxG2], pp[kMaxG2], mu[kMaxG2], fa[kMaxG2];
    if (b.aexp)
        pair_prims_atoms(b, aoff[m] + i, aoff[m] + j, A, B, px, py, pz, ps, pp, mu, fa);
    else
        pair_prims(b, bd, A, B, px, py, pz, ps);
    pk[pos] = (int)i;
    pl[pos] = (int)j;
    pm[pos] = m;
    pq[pos] = q[p];
    pd[pos] = dens[doff[m] + i * nm[m] + j];
    const int g2 = b.g2;
    for (int ab = 0; ab < g2; ++ab) {
        prim[(0 * g2 + ab) * pcap + pos] = px[ab];
        prim[(1 * g2 + ab) * pcap + pos] = py[ab];
        prim[(2 * g2 + ab) * pcap + pos] = pz[ab];
        prim[(3 * g2 + ab) * pcap + pos] = ps[ab];
        prim_f[(0 * g2 + ab) * pcap + pos] = (float)px[ab];
        prim_f[(1 * g2 + ab) * pcap + pos] = (float)py[ab];
        prim_f[(2 * g2 + ab) * pcap + pos] = (float)pz[ab];
        prim_f[(3 * g2 + ab) * pcap + pos] = (float)ps[ab];
        // bra row: centre, charge and the charge weighted by mu and by the fractions
        // fa = a/p, fb = b/p of the primitive pair (the gradient's bra weights)
        double *ba = bra + ((int64_t)pos * g2 + ab) * kBBra;
        float *bf = bra_f + ((int64_t)pos * g2 + ab) * kBBra;
        const double m_ab = b.aexp ? mu[ab] : bd->mu[ab];
        const double fa_ab = b.aexp ? fa[ab] : bd->fa[ab];
        const double fb_ab = b.aexp ? 1.0 - fa[ab] : bd->fb[ab];
        const double row[kBBra] = {px[ab], py[ab], pz[ab], ps[ab], m_ab * ps[ab], fa_ab * ps[ab], fb_ab * ps[ab],
                                   fa_ab * fb_ab * ps[ab], fb_ab * fb_ab * ps[ab], 0.0, 0.0, 0.0};
        for (int c = 0; c < kBBra; ++c) {
            ba[c] = row[c];
            bf[c] = (float)row[c];
        }
    }
    if (bip) {
        for (int ab = 0; ab < g2; ++ab) {
            const double sw = kTswitch / pp[ab];
            prim[(4 * g2 + ab) * pcap + pos] = sw;
            prim_f[(4 * g2 + ab) * pcap + pos] = (float)sw;
            bip[(int64_t)pos * g2 + ab] = sw;
            bip_f[(int64_t)pos * g2 + ab] = (float)sw;
        }
    }
    if (kmu) {
        for (int ab = 0; ab < g2; ++ab) {
            kmu[(int64_t)ab * pcap + pos] = mu[ab];
            kfa[(int64_t)ab * pcap + pos] = fa[ab];
        }
    }
}

__global__ void k_b_pad(const DevHeader *__restrict__ hdr, int64_t pcap, int *__restrict__ pm)
{
    const int64_t pos = hdr->sig_pairs + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos < pcap) pm[pos] = 0;
}

// Ket range of every bra s: kets t in [klo_s, lim_s), klo_s the first pair of its molecule,
// lim_s = min(s + 1, end of the molecule's band holding tau / Q_s).
__global__ __launch_bounds__(256) void k_b_limits(const DevHeader *__restrict__ hdr, double tau,
                                                  const double *__restrict__ pq, const int *__restrict__ pm,
                                                  const long long *__restrict__ boff, long long *__restrict__ nitems,
                                                  int *__restrict__ lims, int *__restrict__ klo, int64_t pcap)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= pcap) return;
    long long ni = 0;
    if (s < hdr->sig_pairs) {
        const int m = pm[s];
        const long long start = boff[(long long)m * kNumBands];
        const double thr = tau / pq[s];
        long long bend;
        if (thr <= 0.0) {
            bend = boff[(long long)(m + 1) * kNumBands];
        } else {
            // band 0 is open-ended: a threshold above its edges still ends there
            const int bt = q_band(thr);
            bend = boff[(long long)m * kNumBands + bt + 1];
        }
        const long long lim = bend < s + 1 ? bend : s + 1;
        const long long cnt = lim > start ? lim - start : 0;
        ni = (cnt + kKetsPerItem - 1) / kKetsPerItem;
        lims[s] = (int)lim;
        klo[s] = (int)start;
    } else {
        lims[s] = 0;
        klo[s] = 0;
    }
    nitems[s] = ni;
}

// Block table of the quartet kernel.  Per molecule: its item range, and either one owned
// block (all its items; molecules with at most owned_bound unique quartets before the
// screen, P (P + 1) / 2 with P = n (n + 1) / 2) or ceil(items / bsz) shared blocks.
// bsz = block_items, or (0: automatic) total items / (8 x workgroups) clamped to
// [kBlockItems, 4 kBlockItems]: big batches get fewer fetches and molecule switches, small
// ones keep enough blocks to spread.
__global__ __launch_bounds__(256) void k_b_blocks(DevHeader *__restrict__ hdr, int64_t nmol,
                                                  const int *__restrict__ nm, const long long *__restrict__ boff,
                                                  const long long *__restrict__ item_off, int block_items,
                                                  long long owned_bound, int groups, long long *__restrict__ mi0,
                                                  long long *__restrict__ mi1, long long *__restrict__ cnt_own,
                                                  long long *__restrict__ cnt_sh)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long bsz = block_items;
    if (bsz <= 0) {
        bsz = hdr->items / (8LL * (long long)groups);
        bsz = bsz < kBlockItems ? kBlockItems : (bsz > 4 * kBlockItems ? 4 * kBlockItems : bsz);
    }
    if (m == 0) hdr->bsz = bsz;
    if (m >= nmol) return;
    const long long i0 = item_off[boff[m * kNumBands]], i1 = item_off[boff[(m + 1) * kNumBands]];
    mi0[m] = i0;
    mi1[m] = i1;
    const long long n = nm[m], P = n * (n + 1) / 2;
    const bool own = owned_bound > 0 && P * (P + 1) / 2 <= owned_bound;
    cnt_own[m] = own && i1 > i0 ? 1 : 0;
    cnt_sh[m] = own ? 0 : (i1 - i0 + bsz - 1) / bsz;
}

// ------------------------------------------------------------------ fused quartet kernel

// Work within a block.  A block is a range of items of one molecule (all of them for an
// owned block).  Each item (bra s, 256 kets) is cut into four units of 64 kets, and the
// waves of the workgroup take the block's units round-robin, each on its own: a wave walks
// its units in item order, keeps its bra's data while the bra stays the same, and folds its
// bra-side sums into LDS when the bra changes.  The waves meet only at the start and the
// end of a block (LDS cleared, then the molecule's accumulators written out), so a bra with
// few kets occupies one wave, not the workgroup.  The wave count per workgroup is set at
// launch (blockDim.x / 64): with a large molecule's triangle in LDS few workgroups fit on a
// CU, and wider ones keep the SIMDs supplied.
//
// Gradient contraction.  With P_ab = A + fb (B - A) and Q_cd = C + fd (D - C) (fa = a/p,
// fb = b/p, fc = c/q, fd = d/q), the separation splits into atom vectors,
//     P - Q = R_AC + fb R_BA - fd R_DC,   R_AC = A - C, R_BA = B - A, R_DC = D - C,
// so the W terms of the derivatives need only scalar sums of w = S_ab S_cd W(r) weighted by
// the fractions: per primitive quartet the lane adds S_cd E, mu_cd S_cd E, S_cd W, fd S_cd W,
// fc S_cd W and fc fd S_cd W (one FMA each), and once per bra primitive pair these are
// folded with the bra's weights (S, mu S, fa S, fb S, fa fb S, fb^2 S from the bra table).
// Every weighted sum is accumulated directly (no difference of two sums), so FP32 partial
// sums keep their relative accuracy.  Per kept quartet, with Gamma the density factor:
//   dA = Gamma [ -2 AB sum mu S S E + R_AC sum fa w + R_BA sum fa fb w - R_DC sum fa fd w ]
//   dB = Gamma [ +2 AB sum mu S S E + R_AC sum fb w + R_BA sum fb^2 w - R_DC sum fb fd w ]
//   dC = Gamma [ -2 CD sum mu_cd S S E - R_AC sum fc w - R_BA sum fc fb w + R_DC sum fc fd w ]
//   dD = -(dA + dB + dC)
template <int G, typename R, bool kGrad, bool kAtoms = false>
__global__ __launch_bounds__(kBatchMaxThreads) void k_batched(BArgs a)
{
    constexpr int G2 = G * G;
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const int nmax = a.nmax;
    using BG = BoysGrid<R>;
    // the Boys table first (16-byte aligned rows), then the molecule's accumulators
    R *tHG = (R *)smem;
    double *Lt = (double *)(tHG + BG::table_len);  // [nmax (nmax+1) / 2]
    double *lg = Lt + nmax * (nmax + 1) / 2;                   // [3 nmax]
    const int nthr = (int)blockDim.x, tid = threadIdx.x, lane = tid % kWave;
    // the wave index through readfirstlane, so that everything derived from it (the unit
    // loop, the bra walk) is known to be wave-uniform and stays in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int nwaves = nthr / kWave;
    const int S = a.hdr->sig_pairs;
    const BasisDev *bd = a.bd;
    // grid-scaled rows (argument T' = T / h) from the FP64 rows (one rounding for FP32):
    // coefficient m of H times h^m sqrt(h) kE, of g times h^m h^(3/2) kW (FP32 only; FP64
    // takes g from the derivative of H's degree-7 row)
    {
        // FP64: the degree-7 rows of H (tabG); FP32: H's and g's rows on the FP32 grid
        const double *gH = sizeof(R) == 8 ? a.tabG : a.tabH_f, *gG = a.tabG_f;
        for (int x = tid; x < BG::table_len; x += nthr) {
            int k, c;
            bool isg;
            if constexpr (sizeof(R) == 8) {   // H's rows of degree 7, padded
                k = x / BG::pair_stride;
                c = x % BG::pair_stride;
                isg = false;
            } else {                          // H's rows, then g's
                isg = x >= BG::g_off;
                const int y = isg ? x - BG::g_off : x;
                k = y / BG::stride;
                c = y % BG::stride;
            }
            const int order = sizeof(R) == 8 ? kBoysOrderG : BG::stride;
            const int rowlen = sizeof(R) == 8 ? kBoysStrideG : BG::stride;
            double v = 0.0;   // the pad
            if (c < order) {
                double sc = sqrt(BG::h);
                for (int e = 0; e < c; ++e) sc *= BG::h;
                v = isg ? gG[k * rowlen + c] * sc * BG::h * (double)GradScale<R>::kW
                        : gH[k * rowlen + c] * sc * (double)GradScale<R>::kE;
            }
            tHG[x] = (R)v;
        }
    }
    unsigned long long kept = 0;
    __shared__ long long blk_at;
    __shared__ int s_first;
    // blocks from a global counter through the block table: owned blocks first (whole
    // molecules), then shared blocks of bsz items, until both kinds are exhausted
    const long long bt_own = a.hdr->bt_own, bt_all = bt_own + a.hdr->bt_sh, bsz = a.hdr->bsz;
    const R *prim = BPrec<R>::prim(a);
    const cptr<R> rsg = (cptr<R>)BPrec<R>::rsg(bd);
    const cptr<double> cmu = (cptr<double>)bd->mu;
    const cptr<double> cfa = (cptr<double>)bd->fa;
    const cptr<double> cfb = (cptr<double>)bd->fb;
    for (;;) {
    __syncthreads();
    if (tid == 0) blk_at = (long long)atomicAdd(a.next_block, 1ULL);
    __syncthreads();
    const long long blk = blk_at;
    if (blk >= bt_all) break;
    const bool owned = blk < bt_own;
    const int mol = owned ? mol_of(a.off_own, a.nmol, blk) : mol_of(a.off_sh, a.nmol, blk - bt_own);
    long long m0 = a.mol_i0[mol];
    if (!owned) m0 += (blk - bt_own - a.off_sh[mol]) * bsz;
    const long long m1 = owned || m0 + bsz > a.mol_i1[mol] ? a.mol_i1[mol] : m0 + bsz;
    const int nm = a.mol_n[mol];
    const long long aoff = a.mol_aoff[mol], doff = a.mol_doff[mol], toff = a.mol_toff[mol];
    const int ntri = nm * (nm + 1) / 2;
    for (int x = tid; x < ntri; x += nthr) Lt[x] = 0.0;
    if (kGrad)
        for (int x = tid; x < 3 * nm; x += nthr) lg[x] = 0.0;
    if (tid == 0) {
        // the bra of item m0: the last s with item_off[s] <= m0
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.item_off[mid] <= m0) lo = mid; else hi = mid - 1;
        }
        s_first = lo;
    }
    __syncthreads();
    {
    int s = s_first, curbra = -1;
    int bi = 0, bj = 0, lim = 0, klo = 0;
    double qs = 0.0, ds = 0.0, Ax = 0.0, Ay = 0.0, Az = 0.0, Bx = 0.0, By = 0.0, Bz = 0.0;
    double jb = 0.0, gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
    // folds this wave's bra-side sums into the LDS accumulators
    auto flush_bra = [&]() {
        const double w = wave_sum(jb);
        if (lane == 0 && w != 0.0) atomicAdd(&Lt[tri(bi, bj)], 4.0 * w);
        jb = 0.0;
        if (kGrad) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double wa = wave_sum(gA[c]), wb = wave_sum(gB[c]);
                if (lane == 0) {
                    atomicAdd(&lg[3 * bi + c], wa);
                    atomicAdd(&lg[3 * bj + c], wb);
                }
                gA[c] = gB[c] = 0.0;
            }
        }
    };
    const long long nunits = (m1 - m0) * kUnitsPerItem;
    for (long long u = wave; u < nunits; u += nwaves) {
        const long long m = m0 + u / kUnitsPerItem;
        while (a.item_off[s + 1] <= m) ++s;
        if (s != curbra) {
            if (curbra >= 0) flush_bra();
            curbra = s;
            bi = a.pk[s];
            bj = a.pl[s];
            qs = a.pq[s];
            ds = a.pd[s];
            lim = a.lim[s];
            klo = a.klo[s];
            const double *xa = a.xyz + 3 * (aoff + bi), *xb = a.xyz + 3 * (aoff + bj);
            Ax = xa[0]; Ay = xa[1]; Az = xa[2];
            Bx = xb[0]; By = xb[1]; Bz = xb[2];
        }
        const long long t0 = klo + (m - a.item_off[s]) * kKetsPerItem + (u % kUnitsPerItem) * kWave;
        if (t0 >= lim) continue;
        const long long tk = t0 + lane;
        const bool valid = (tk < lim) && (qs * a.pq[tk] >= a.tau);
        const long long t = valid ? tk : S;   // lanes without a kept quartet read the first pad entry
        const cptr<R> bra = (cptr<R>)(BPrec<R>::bra(a) + (int64_t)s * kBBra * G2);
        const cptr<R> bipp = kAtoms ? (cptr<R>)(BPrec<R>::bip(a) + (int64_t)s * G2) : nullptr;
        const int k = a.pk[t], l = a.pl[t];

        // forward: eri; gradient: sX = sum mu_ab S S E, sZ = sum mu_cd S S E and the
        // fraction-weighted sums of w (names: weights of bra, then ket)
        R eri = R(0), sX = R(0), sZ = R(0);
        R wA = R(0), wAB = R(0), wB = R(0), wBB = R(0), wAD = R(0), wBD = R(0), wC = R(0), wCB = R(0), wCD = R(0);
#pragma unroll 1
        for (int cb = 0; cb < G; ++cb) {
            R kx[G], ky[G], kz[G], ks[G], kp[G];
            R kms[G], kds[G], kcs[G], kcds[G];   // S_cd times mu_cd, fd, fc, fc fd
            // buffer loads of the ket table: component and this cb's rows in the resource,
            // the row as a scalar offset, the ket as a 32-bit lane offset
            const unsigned tb = (unsigned)t * (unsigned)sizeof(R);
            auto ld = [&](int c, int d) {
                return ket_load<R>(ket_rows(prim, (int64_t)c * G2 + cb * G, a.pcap, G), tb,
                                  (int)((int64_t)d * a.pcap * (int64_t)sizeof(R)));
            };
#pragma unroll
            for (int d = 0; d < G; ++d) {
                kx[d] = ld(0, d);
                ky[d] = ld(1, d);
                kz[d] = ld(2, d);
                ks[d] = ld(3, d);
                kp[d] = kAtoms ? ld(4, d) : R(0);
            }
            if (kGrad) {
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    const int cd = cb * G + d;
                    double mu, fc;
                    if constexpr (kAtoms) {
                        mu = a.kmu[(int64_t)cd * a.pcap + t];
                        fc = a.kfa[(int64_t)cd * a.pcap + t];
                    } else {
                        mu = cmu[cd];
                        fc = cfa[cd];
                    }
                    const double fd = kAtoms ? 1.0 - fc : cfb[cd];
                    kms[d] = (R)mu * ks[d];
                    kcs[d] = (R)fc * ks[d];
                    kds[d] = (R)fd * ks[d];
                    kcds[d] = (R)(fc * fd) * ks[d];
                }
            }
#pragma unroll 1
            for (int ab = 0; ab < G2; ++ab) {
                // every scalar of this bra primitive in one batch of scalar loads:
                // Px Py Pz S mu*S fa*S fb*S fa*fb*S fb^2*S, and the switch data
                const cptr<R> bp = bra + kBBra * ab;
                R b[kGrad ? 9 : 4], u[4 * G], bsw = R(0);
#pragma unroll
                for (int c = 0; c < (kGrad ? 9 : 4); ++c) b[c] = bp[c];
                if constexpr (kAtoms) {
                    bsw = bipp[ab];
                    asm volatile("" ::"s"(bsw));
                } else {
                    const cptr<R> up = rsg + 4 * (ab * G2 + cb * G);
#pragma unroll
                    for (int c = 0; c < 4 * G; ++c) u[c] = up[c];
#pragma unroll
                    for (int c = 0; c < 4 * G; ++c) asm volatile("" ::"s"(u[c]));
                }
                const R px = b[0], py = b[1], pz = b[2];
                R U = R(0), Y = R(0), X0 = R(0), X1 = R(0), Xc = R(0), Xcd = R(0);
                // every lane's separation and far-field E, W first (independent across d:
                // their reciprocal square roots issue back to back), then the near lanes
                // overwrite theirs from the table under exec masks
                R r2[G], E[G], W[G];
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    const R dx = px - kx[d], dy = py - ky[d], dz = pz - kz[d];
                    r2[d] = dx * dx + dy * dy + dz * dz;
                    const R y = GradScale<R>::e_far(r2[d]);
                    E[d] = y;
                    W[d] = kGrad ? GradScale<R>::w_far(y) : R(0);
                }
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    // switch radius^2 kTswitch / rho (per-atom bases: sum of the stored halves)
                    const R sw = kAtoms ? bsw + kp[d] : u[4 * d];
                    if (r2[d] < sw) {
                        // (rho/h, sqrt(rho/h), (rho/h)^(3/2)) from the table, or from sw
                        R q1, q2, q3;
                        if constexpr (kAtoms) {
                            q2 = rsqrt_r(sw) * R(BG::sqrt_sw_inv_h);
                            q1 = q2 * q2;
                            q3 = q1 * q2;
                        } else {
                            q1 = u[4 * d + 1];
                            q2 = u[4 * d + 2];
                            q3 = u[4 * d + 3];
                        }
                        // sqrt(h) H and h^(3/2) g at T' = T / h on the table grid
                        R dd;
                        const unsigned off = boys_row<R, BG::pair_stride>(r2[d], q1, dd);
                        if constexpr (sizeof(R) == 8) {
                            // degree-7 rows of H; g = 2 H': W on the grid is (2 kW / kE) dE/dd
                            double de;
                            E[d] = q2 * boys_eval_d(tHG, off, dd, de);
                            if (kGrad) W[d] = q3 * (R(2.0 * GradScale<R>::kW / GradScale<R>::kE) * de);
                        } else {
                            E[d] = q2 * boys_eval<R>(tHG, off, dd);
                            if (kGrad) W[d] = q3 * boys_eval<R>(tHG + BG::g_off, off, dd);
                        }
                    }
                }
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    U = fma(ks[d], E[d], U);
                    if (kGrad) {
                        Y = fma(kms[d], E[d], Y);
                        X0 = fma(ks[d], W[d], X0);
                        X1 = fma(kds[d], W[d], X1);
                        Xc = fma(kcs[d], W[d], Xc);
                        Xcd = fma(kcds[d], W[d], Xcd);
                    }
                }
                eri = fma(b[3], U, eri);
                if (kGrad) {
                    sX = fma(b[4], U, sX);
                    sZ = fma(b[3], Y, sZ);
                    wA = fma(b[5], X0, wA);
                    wAB = fma(b[7], X0, wAB);
                    wB = fma(b[6], X0, wB);
                    wBB = fma(b[8], X0, wBB);
                    wAD = fma(b[5], X1, wAD);
                    wBD = fma(b[6], X1, wBD);
                    wC = fma(b[3], Xc, wC);
                    wCB = fma(b[6], Xc, wCB);
                    wCD = fma(b[3], Xcd, wCD);
                }
            }
        }
        {
            // back from the accumulators' scales (E times kE, W times kW)
            constexpr R iE = R(1) / GradScale<R>::kE, iW = R(1) / GradScale<R>::kW;
            eri *= iE;
            if (kGrad) {
                sX *= iE; sZ *= iE;
                wA *= iW; wAB *= iW; wB *= iW; wBB *= iW; wAD *= iW; wBD *= iW; wC *= iW; wCB *= iW; wCD *= iW;
            }
        }
        if (valid) {
            ++kept;
            double deg = 1.0;
            if (bi == bj) deg *= 0.5;
            if (k == l) deg *= 0.5;
            if (t == s) deg *= 0.5;
            const double v = (double)eri * deg;
            const double *Dm = a.dens + doff;
            const double Dik = Dm[bi * nm + k], Dil = Dm[bi * nm + l];
            const double Djk = Dm[bj * nm + k], Djl = Dm[bj * nm + l];
            const double dt = a.pd[t];
            jb = fma(dt, v, jb);
            atomicAdd(&Lt[tri(k, l)], 4.0 * ds * v);
            atomicAdd(&Lt[tri(bi, k)], -Djl * v);
            atomicAdd(&Lt[tri(bi, l)], -Djk * v);
            atomicAdd(&Lt[tri(bj, k)], -Dil * v);
            atomicAdd(&Lt[tri(bj, l)], -Dik * v);
            if (kGrad) {
                const double gam = deg * (4.0 * ds * dt - Dik * Djl - Dil * Djk);
                const double *xc = a.xyz + 3 * (aoff + k), *xd = a.xyz + 3 * (aoff + l);
                const double A[3] = {Ax, Ay, Az}, B[3] = {Bx, By, Bz};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double rac = A[c] - xc[c], rba = B[c] - A[c], rdc = xd[c] - xc[c];
                    const double GA = gam * (2.0 * rba * (double)sX + rac * (double)wA + rba * (double)wAB -
                                             rdc * (double)wAD);
                    const double GB = gam * (-2.0 * rba * (double)sX + rac * (double)wB + rba * (double)wBB -
                                             rdc * (double)wBD);
                    const double GC = gam * (2.0 * rdc * (double)sZ - rac * (double)wC - rba * (double)wCB +
                                             rdc * (double)wCD);
                    gA[c] += GA;
                    gB[c] += GB;
                    atomicAdd(&lg[3 * k + c], GC);
                    atomicAdd(&lg[3 * l + c], -(GA + GB + GC));
                }
            }
        }
    }
    if (curbra >= 0) flush_bra();
    }
    __syncthreads();
    if (owned) {
        // the molecule's only block: store the accumulators as they are
        for (int x = tid; x < ntri; x += nthr) a.facc[toff + x] = Lt[x];
        if (kGrad)
            for (int x = tid; x < 3 * nm; x += nthr) a.gacc[3 * aoff + x] = lg[x];
    } else {
        for (int x = tid; x < ntri; x += nthr) {
            const double v = Lt[x];
            if (v != 0.0) atomicAdd(&a.facc[toff + x], v);
        }
        if (kGrad) {
            for (int x = tid; x < 3 * nm; x += nthr) {
                const double v = lg[x];
                if (v != 0.0) atomicAdd(&a.gacc[3 * aoff + x], v);
            }
        }
    }
    }
    for (int off = 32; off > 0; off >>= 1) kept += __shfl_xor(kept, off, 64);
    if (lane == 0 && kept) atomicAdd(a.quartets, kept);
}

// G from the folded lower triangle and E2 = 1/2 sum D o G, one block per molecule.
__global__ __launch_bounds__(256) void k_b_final(const int *__restrict__ mol_n, const long long *__restrict__ doff,
                                                 const long long *__restrict__ toff, const double *__restrict__ facc,
                                                 const double *__restrict__ dens, double *__restrict__ fock,
                                                 double *__restrict__ e2)
{
    __shared__ double red[256];
    const int m = blockIdx.x;
    const int n = mol_n[m];
    const double *L = facc + toff[m];
    double e = 0.0;
    for (int x = threadIdx.x; x < n * n; x += 256) {
        const int i = x / n, j = x % n;
        const double v = i == j ? L[tri(i, i)] : 0.5 * L[tri(i, j)];
        fock[doff[m] + x] = v;
        e += dens[doff[m] + x] * v;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) e2[m] = 0.5 * red[0];
}

__global__ void k_b_fill(double *__restrict__ p, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.0;
}

__global__ void k_b_fill_ll(long long *__restrict__ p, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0;
}

__global__ void k_b_copy(const double *__restrict__ s, int64_t m, double *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) d[i] = s[i];
}

// ------------------------------------------------------------------ host side

template <int G, typename R, bool GR, bool AT>
static int bres(size_t smem, int threads)
{
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched<G, R, GR, AT>, threads, smem) == hipSuccess
               ? nb
               : 0;
}

template <typename R, bool GR, bool AT>
static int bres_g(int g, size_t smem, int threads)
{
    switch (g) {
    case 1: return bres<1, R, GR, AT>(smem, threads);
    case 2: return bres<2, R, GR, AT>(smem, threads);
    case 3: return bres<3, R, GR, AT>(smem, threads);
    case 4: return bres<4, R, GR, AT>(smem, threads);
    case 5: return bres<5, R, GR, AT>(smem, threads);
    default: return bres<6, R, GR, AT>(smem, threads);
    }
}

// Workgroups of the batched kernel (`waves` waves each) that fit on one CU at once (0 if the
// runtime cannot tell).
int batched_resident_groups(int g, int prec, bool grad, bool atoms, int nmax, int waves)
{
    const size_t smem = batched_smem_bytes(nmax, prec);
    const int th = waves * kWave;
    if (prec == HFK_MIXED) {
        if (grad) return atoms ? bres_g<float, true, true>(g, smem, th) : bres_g<float, true, false>(g, smem, th);
        return atoms ? bres_g<float, false, true>(g, smem, th) : bres_g<float, false, false>(g, smem, th);
    }
    if (grad) return atoms ? bres_g<double, true, true>(g, smem, th) : bres_g<double, true, false>(g, smem, th);
    return atoms ? bres_g<double, false, true>(g, smem, th) : bres_g<double, false, false>(g, smem, th);
}

size_t batched_smem_bytes(int nmax, int prec)
{
    return sizeof(double) * ((size_t)nmax * (nmax + 1) / 2 + 3 * (size_t)nmax) +
           (prec == HFK_MIXED ? sizeof(float) * BoysGrid<float>::table_len
                              : sizeof(double) * BoysGrid<double>::table_len);
}

BLayout make_blayout(int64_t nmol, const int64_t *atom_off, int g, int with_grad, bool atoms)
{
    BLayout L;
    memset(&L, 0, sizeof(L));
    L.nmol = nmol;
    L.atoms = atoms;
    L.g = g;
    L.g2 = g * g;
    long long ptot = 0, ntot = 0, tri = 0, nmax = 0;
    for (int64_t m = 0; m < nmol; ++m) {
        const long long n = atom_off[m + 1] - atom_off[m];
        ptot += n * (n + 1) / 2;
        tri += n * (n + 1) / 2;
        ntot += n;
        nmax = n > nmax ? n : nmax;
    }
    L.ptot = ptot;
    L.ntot = ntot;
    L.tri = tri;
    L.nmax = (int)nmax;
    L.pcap = ((ptot + 63) / 64) * 64 + 64;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t PC = (size_t)L.pcap, g2 = (size_t)L.g2, NM = (size_t)nmol;
    const size_t NB = NM * kNumBands;
    L.hdr = take(sizeof(DevHeader));
    L.basis = take(sizeof(BasisDev));
    L.boys = take(sizeof(double) * kBoysGrid * kBoysStride);
    L.boys_f = take(sizeof(double) * kBoysGridF * kBoysStrideF);
    L.boys_g = take(sizeof(double) * kBoysGrid * kBoysStrideG);
    L.boys_g_f = take(sizeof(double) * kBoysGridF * kBoysStrideF);
    L.mol_n = take(sizeof(int) * NM);
    L.mol_aoff = take(sizeof(long long) * (NM + 1));
    L.mol_poff = take(sizeof(long long) * (NM + 1));
    L.mol_doff = take(sizeof(long long) * (NM + 1));
    L.mol_toff = take(sizeof(long long) * (NM + 1));
    L.cent = take(sizeof(double) * 3 * NM);
    L.qmax = take(sizeof(unsigned long long) * NM);
    L.q = take(sizeof(double) * (size_t)ptot);
    L.bucket_of = take(sizeof(int) * (size_t)ptot);
    L.bcnt = take(sizeof(long long) * NB);
    L.boff = take(sizeof(long long) * (NB + 1));
    L.bcur = take(sizeof(int) * NB);
    L.pk = take(sizeof(int) * PC);
    L.pl = take(sizeof(int) * PC);
    L.pm = take(sizeof(int) * PC);
    L.pq = take(sizeof(double) * PC);
    L.pd = take(sizeof(double) * PC);
    L.prim = take(sizeof(double) * (atoms ? 5 : 4) * g2 * PC);   // Px, Py, Pz, S (, kTswitch/p)
    L.prim_f = take(sizeof(float) * (atoms ? 5 : 4) * g2 * PC);
    if (atoms) {
        L.arow = take(sizeof(double) * 2 * (size_t)ntot * (size_t)g);
        L.bip = take(sizeof(double) * g2 * PC);
        L.bip_f = take(sizeof(float) * g2 * PC);
        if (with_grad) {
            L.kmu = take(sizeof(double) * g2 * PC);
            L.kfa = take(sizeof(double) * g2 * PC);
        }
    }
    L.bra = take(sizeof(double) * kBBra * g2 * PC);
    L.bra_f = take(sizeof(float) * kBBra * g2 * PC);
    L.nitems = take(sizeof(long long) * PC);
    L.lim = take(sizeof(int) * PC);
    L.klo = take(sizeof(int) * PC);
    L.item_off = take(sizeof(long long) * (PC + 1));
    const size_t scan_n = PC > NB ? PC : NB;
    L.scan_tmp = take(sizeof(long long) * ((scan_n + 1023) / 1024 + 1));
    L.facc = take(sizeof(double) * (size_t)tri);
    L.gacc = with_grad ? take(sizeof(double) * 3 * (size_t)ntot) : 0;
    L.mol_i0 = take(sizeof(long long) * NM);
    L.mol_i1 = take(sizeof(long long) * NM);
    L.cnt_own = take(sizeof(long long) * NM);
    L.cnt_sh = take(sizeof(long long) * NM);
    L.off_own = take(sizeof(long long) * (NM + 1));
    L.off_sh = take(sizeof(long long) * (NM + 1));
    L.total = o;
    return L;
}

hipError_t upload_batch_tables(const BLayout &L, char *ws, const int64_t *atom_off_host, hipStream_t st)
{
    const int64_t nmol = L.nmol;
    std::vector<int> nm(nmol);
    std::vector<long long> aoff(nmol + 1), poff(nmol + 1), doff(nmol + 1), toff(nmol + 1);
    aoff[0] = poff[0] = doff[0] = toff[0] = 0;
    for (int64_t m = 0; m < nmol; ++m) {
        const long long n = atom_off_host[m + 1] - atom_off_host[m];
        nm[m] = (int)n;
        aoff[m + 1] = atom_off_host[m + 1];
        poff[m + 1] = poff[m] + n * (n + 1) / 2;
        doff[m + 1] = doff[m] + n * n;
        toff[m + 1] = toff[m] + n * (n + 1) / 2;
    }
    hipError_t e = hipMemcpyAsync(ws + L.mol_n, nm.data(), sizeof(int) * nmol, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.mol_aoff, aoff.data(), sizeof(long long) * (nmol + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.mol_poff, poff.data(), sizeof(long long) * (nmol + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.mol_doff, doff.data(), sizeof(long long) * (nmol + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.mol_toff, toff.data(), sizeof(long long) * (nmol + 1), hipMemcpyHostToDevice, st);
    // the host vectors end with this call: wait until the copies have consumed them
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t launch_batched(const BLayout &L, const Basis &b, char *ws, const int64_t *atom_off_host, const double *xyz,
                          const double *dens, double tau, int prec, double *fock, double *e2, double *d_xyz,
                          int groups, const BatchedShape &shape, hipStream_t st)
{
    (void)atom_off_host;
    const int64_t nmol = L.nmol;
    hipError_t e = hipSuccess;
    DevHeader *hdr = (DevHeader *)(ws + L.hdr);
    const BasisDev *bd = (const BasisDev *)(ws + L.basis);
    const int *d_n = (const int *)(ws + L.mol_n);
    const long long *d_aoff = (const long long *)(ws + L.mol_aoff);
    const long long *d_poff = (const long long *)(ws + L.mol_poff);
    const long long *d_doff = (const long long *)(ws + L.mol_doff);
    const long long *d_toff = (const long long *)(ws + L.mol_toff);
    double *cent = (double *)(ws + L.cent);
    unsigned long long *qmax = (unsigned long long *)(ws + L.qmax);
    const unsigned nbp = (unsigned)((L.ptot + 255) / 256);
    const long long NB = (long long)nmol * kNumBands;
    long long *bcnt = (long long *)(ws + L.bcnt);
    long long *boff = (long long *)(ws + L.boff);
    int *bcur = (int *)(ws + L.bcur);
    hipLaunchKernelGGL(k_b_mol, dim3((unsigned)((nmol + 127) / 128)), dim3(128), 0, st, (int)nmol, d_n, d_aoff, xyz,
                       cent, qmax);
    hipLaunchKernelGGL(k_b_pair_q, dim3(nbp), dim3(256), 0, st, b, bd, (int)nmol, d_poff, d_aoff, cent, xyz, L.ptot,
                       (double *)(ws + L.q), qmax);
    hipLaunchKernelGGL(k_b_fill_ll, dim3((unsigned)((NB + 255) / 256)), dim3(256), 0, st, bcnt, (int64_t)NB);
    hipLaunchKernelGGL(k_b_bucket_count, dim3(nbp), dim3(256), 0, st, (int)nmol, d_poff, L.ptot, tau, qmax,
                       (const double *)(ws + L.q), (int *)(ws + L.bucket_of), bcnt);
    e = launch_scan(bcnt, NB, boff, (long long *)(ws + L.scan_tmp), nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_cursors, dim3((unsigned)((NB + 255) / 256)), dim3(256), 0, st, boff, NB, bcur, hdr);
    hipLaunchKernelGGL(k_b_pair_scatter, dim3(nbp), dim3(256), 0, st, b, bd, (int)nmol, d_poff, d_aoff, d_doff, d_n,
                       cent, xyz, dens, L.ptot, L.pcap, (const double *)(ws + L.q), (const int *)(ws + L.bucket_of), bcur,
                       (int *)(ws + L.pk), (int *)(ws + L.pl), (int *)(ws + L.pm), (double *)(ws + L.pq),
                       (double *)(ws + L.pd), (double *)(ws + L.prim), (float *)(ws + L.prim_f), (double *)(ws + L.bra),
                       (float *)(ws + L.bra_f), L.atoms ? (double *)(ws + L.bip) : nullptr,
                       L.atoms ? (float *)(ws + L.bip_f) : nullptr, L.kmu ? (double *)(ws + L.kmu) : nullptr,
                       L.kmu ? (double *)(ws + L.kfa) : nullptr);
    const unsigned nbc = (unsigned)((L.pcap + 255) / 256);
    e = launch_pair_pad(hdr, L.pcap, L.g2, L.atoms, (int *)(ws + L.pk), (int *)(ws + L.pl), (double *)(ws + L.pq),
                        (double *)(ws + L.pd), (double *)(ws + L.prim), (float *)(ws + L.prim_f),
                        L.kmu ? (double *)(ws + L.kmu) : nullptr, L.kmu ? (double *)(ws + L.kfa) : nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_pad, dim3(nbc), dim3(256), 0, st, hdr, L.pcap, (int *)(ws + L.pm));
    hipLaunchKernelGGL(k_b_limits, dim3(nbc), dim3(256), 0, st, hdr, tau, (const double *)(ws + L.pq),
                       (const int *)(ws + L.pm), boff, (long long *)(ws + L.nitems), (int *)(ws + L.lim),
                       (int *)(ws + L.klo), L.pcap);
    e = launch_scan((const long long *)(ws + L.nitems), L.pcap, (long long *)(ws + L.item_off),
                    (long long *)(ws + L.scan_tmp), &hdr->items, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_blocks, dim3((unsigned)((nmol + 255) / 256)), dim3(256), 0, st, hdr, (int64_t)nmol, d_n,
                       (const long long *)boff, (const long long *)(ws + L.item_off), shape.block_items,
                       shape.owned_bound, groups, (long long *)(ws + L.mol_i0), (long long *)(ws + L.mol_i1),
                       (long long *)(ws + L.cnt_own), (long long *)(ws + L.cnt_sh));
    e = launch_scan((const long long *)(ws + L.cnt_own), nmol, (long long *)(ws + L.off_own),
                    (long long *)(ws + L.scan_tmp), &hdr->bt_own, st);
    if (e == hipSuccess)
        e = launch_scan((const long long *)(ws + L.cnt_sh), nmol, (long long *)(ws + L.off_sh),
                        (long long *)(ws + L.scan_tmp), &hdr->bt_sh, st);
    if (e != hipSuccess) return e;

    const long long tri = L.tri;
    hipLaunchKernelGGL(k_b_fill, dim3((unsigned)((tri + 255) / 256)), dim3(256), 0, st, (double *)(ws + L.facc),
                       (int64_t)tri);
    const bool grad = d_xyz != nullptr;
    if (grad)
        hipLaunchKernelGGL(k_b_fill, dim3((unsigned)((3 * L.ntot + 255) / 256)), dim3(256), 0, st,
                           (double *)(ws + L.gacc), (int64_t)(3 * L.ntot));
    BArgs a;
    a.hdr = hdr;
    a.bd = bd;
    a.tabH = (const double *)(ws + L.boys);
    a.tabH_f = (const double *)(ws + L.boys_f);
    a.tabG = (const double *)(ws + L.boys_g);
    a.tabG_f = (const double *)(ws + L.boys_g_f);
    a.pk = (const int *)(ws + L.pk);
    a.pl = (const int *)(ws + L.pl);
    a.pm = (const int *)(ws + L.pm);
    a.pq = (const double *)(ws + L.pq);
    a.pd = (const double *)(ws + L.pd);
    a.prim = (const double *)(ws + L.prim);
    a.prim_f = (const float *)(ws + L.prim_f);
    a.bra = (const double *)(ws + L.bra);
    a.bra_f = (const float *)(ws + L.bra_f);
    a.bip = L.atoms ? (const double *)(ws + L.bip) : nullptr;
    a.bip_f = L.atoms ? (const float *)(ws + L.bip_f) : nullptr;
    a.kmu = L.kmu ? (const double *)(ws + L.kmu) : nullptr;
    a.kfa = L.kmu ? (const double *)(ws + L.kfa) : nullptr;
    a.item_off = (const long long *)(ws + L.item_off);
    a.lim = (const int *)(ws + L.lim);
    a.klo = (const int *)(ws + L.klo);
    a.mol_n = d_n;
    a.mol_aoff = d_aoff;
    a.mol_doff = d_doff;
    a.mol_toff = d_toff;
    a.xyz = xyz;
    a.dens = dens;
    a.facc = (double *)(ws + L.facc);
    a.gacc = grad ? (double *)(ws + L.gacc) : nullptr;
    a.quartets = &hdr->quartets;
    a.next_block = &hdr->next_block;
    a.off_own = (const long long *)(ws + L.off_own);
    a.off_sh = (const long long *)(ws + L.off_sh);
    a.mol_i0 = (const long long *)(ws + L.mol_i0);
    a.mol_i1 = (const long long *)(ws + L.mol_i1);
    a.nmol = (int)nmol;
    a.pcap = L.pcap;
    a.tau = tau;
    a.nmax = L.nmax;
    const size_t smem = batched_smem_bytes(L.nmax, prec);
    const int threads = (shape.waves == 8 ? 8 : 4) * kWave;
    {
        const hipError_t ez = launch_zero_counter(a.next_block, st);
        if (ez != hipSuccess) return ez;
    }
    profile_begin(st);
    if (grad && L.atoms && !L.kmu) return hipErrorInvalidValue;   // per-atom gradient tables missing
#define HFK_B_LAUNCH(GG, RR, GR)                                                                         \
    do {                                                                                                 \
        if (L.atoms)                                                                                     \
            hipLaunchKernelGGL((k_batched<GG, RR, GR, true>), dim3(groups), dim3(threads), smem, st, a); \
        else                                                                                             \
            hipLaunchKernelGGL((k_batched<GG, RR, GR, false>), dim3(groups), dim3(threads), smem, st, a); \
    } while (0)
    if (prec == HFK_MIXED) {
        if (grad) {
            switch (b.g) {
            case 1: HFK_B_LAUNCH(1, float, true); break;
            case 2: HFK_B_LAUNCH(2, float, true); break;
            case 3: HFK_B_LAUNCH(3, float, true); break;
            case 4: HFK_B_LAUNCH(4, float, true); break;
            case 5: HFK_B_LAUNCH(5, float, true); break;
            default: HFK_B_LAUNCH(6, float, true); break;
            }
        } else {
            switch (b.g) {
            case 1: HFK_B_LAUNCH(1, float, false); break;
            case 2: HFK_B_LAUNCH(2, float, false); break;
            case 3: HFK_B_LAUNCH(3, float, false); break;
            case 4: HFK_B_LAUNCH(4, float, false); break;
            case 5: HFK_B_LAUNCH(5, float, false); break;
            default: HFK_B_LAUNCH(6, float, false); break;
            }
        }
    } else {
        if (grad) {
            switch (b.g) {
            case 1: HFK_B_LAUNCH(1, double, true); break;
            case 2: HFK_B_LAUNCH(2, double, true); break;
            case 3: HFK_B_LAUNCH(3, double, true); break;
            case 4: HFK_B_LAUNCH(4, double, true); break;
            case 5: HFK_B_LAUNCH(5, double, true); break;
            default: HFK_B_LAUNCH(6, double, true); break;
            }
        } else {
            switch (b.g) {
            case 1: HFK_B_LAUNCH(1, double, false); break;
            case 2: HFK_B_LAUNCH(2, double, false); break;
            case 3: HFK_B_LAUNCH(3, double, false); break;
            case 4: HFK_B_LAUNCH(4, double, false); break;
            case 5: HFK_B_LAUNCH(5, double, false); break;
            default: HFK_B_LAUNCH(6, double, false); break;
            }
        }
    }
#undef HFK_B_LAUNCH
    profile_end(st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_final, dim3((unsigned)nmol), dim3(256), 0, st, d_n, d_doff, d_toff,
                       (const double *)(ws + L.facc), dens, fock, e2);
    if (grad)
        hipLaunchKernelGGL(k_b_copy, dim3((unsigned)((3 * L.ntot + 255) / 256)), dim3(256), 0, st,
                           (const double *)(ws + L.gacc), (int64_t)(3 * L.ntot), d_xyz);
    return hipGetLastError();
}

}  // namespace hfk
