// Ragged batches of independent molecules in one persistent launch, forward Fock build and
// (optionally) the nuclear gradient fused into the same primitive loop.
//
// Pairs of every molecule are prepared in one pass and stored in (molecule, Q band) order;
// a bra's kets are the molecule's pairs up to its screen limit (t <= s keeps each quartet
// once).  Items of 256 kets are numbered molecule by molecule; workgroups fetch blocks of
// consecutive items from a global counter.  A workgroup keeps the current molecule's whole
// two-electron matrix in LDS (lower triangle, the symmetrisation G = (F + F^T)/2 folded in:
// F_xy and F_yx land in the same slot) and its n x 3 gradient, and flushes both with
// global atomics when the molecule or the block changes.  Per primitive quartet the loop forms E(r) (the integral) and
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
    const float *tabH_f;
    const double *tabG;
    const float *tabG_f;
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
    const double *kmu;      // per-atom gradient: [g2][pcap] ket mu and a/p, [pcap][g2][2] bra
    const double *kfa;
    const double *bmf;
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
    static __device__ const double *tabH(const BArgs &a) { return a.tabH; }
    static __device__ const double *tabG(const BArgs &a) { return a.tabG; }
    static __device__ const double *rsg(const BasisDev *bd) { return bd->rsg; }
};
template <> struct BPrec<float> {
    static __device__ const float *prim(const BArgs &a) { return a.prim_f; }
    static __device__ const float *bra(const BArgs &a) { return a.bra_f; }
    static __device__ const float *bip(const BArgs &a) { return a.bip_f; }
    static __device__ const float *tabH(const BArgs &a) { return a.tabH_f; }
    static __device__ const float *tabG(const BArgs &a) { return a.tabG_f; }
    static __device__ const float *rsg(const BasisDev *bd) { return bd->rsg_f; }
};

__device__ inline int tri(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

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
    double *__restrict__ bip, float *__restrict__ bip_f, double *__restrict__ kmu, double *__restrict__ kfa,
    double *__restrict__ bmf)
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
        double *ba = bra + ((int64_t)pos * g2 + ab) * 8;
        float *bf = bra_f + ((int64_t)pos * g2 + ab) * 8;
        const double p2 = px[ab] * px[ab] + py[ab] * py[ab] + pz[ab] * pz[ab];
        ba[0] = px[ab]; ba[1] = py[ab]; ba[2] = pz[ab]; ba[3] = ps[ab];
        ba[4] = -2.0 * px[ab]; ba[5] = -2.0 * py[ab]; ba[6] = -2.0 * pz[ab]; ba[7] = p2;
        bf[0] = (float)px[ab]; bf[1] = (float)py[ab]; bf[2] = (float)pz[ab]; bf[3] = (float)ps[ab];
        bf[4] = (float)ba[4]; bf[5] = (float)ba[5]; bf[6] = (float)ba[6]; bf[7] = (float)p2;
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
            bmf[((int64_t)pos * g2 + ab) * 2] = mu[ab];
            bmf[((int64_t)pos * g2 + ab) * 2 + 1] = fa[ab];
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

// ------------------------------------------------------------------ fused quartet kernel

template <int G, typename R, bool kGrad, bool kAtoms = false>
__global__ __launch_bounds__(kGroupThreads) void k_batched(BArgs a)
{
    constexpr int G2 = G * G;
    extern __shared__ double smem[];
    const int nmax = a.nmax;
    double *Lt = smem;                                         // [nmax (nmax+1) / 2]
    double *lg = Lt + nmax * (nmax + 1) / 2;                   // [3 nmax]
    R *tH = (R *)(lg + 3 * nmax);
    R *tG = tH + kBoysGrid * kBoysStride;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const long long M = a.hdr->items;
    const int S = a.hdr->sig_pairs;
    const BasisDev *bd = a.bd;
    // grid-scaled rows (argument T' = T / h): coefficient m of H times h^m sqrt(h), of g times
    // h^m h^(3/2), built from the FP64 rows
    for (int x = tid; x < kBoysGrid * kBoysStride; x += kGroupThreads) {
        const int m = x % kBoysStride;
        double sc = sqrt(kBoysH);
        for (int e = 0; e < m; ++e) sc *= kBoysH;
        tH[x] = (R)(a.tabH[x] * sc);
        tG[x] = (R)(a.tabG[x] * sc * kBoysH);
    }
    unsigned long long kept = 0;
    __shared__ long long blk_at;
    // blocks of bsz consecutive items, fetched from a global counter until exhausted: at least
    // kBlockItems, and up to four times that while every workgroup still gets eight blocks
    // or more (fewer fetches and molecule switches; 2000 clusters: 751 ms against 766 ms
    // with blocks of 16)
    long long bsz = M / (8LL * (long long)gridDim.x);
    bsz = bsz < kBlockItems ? kBlockItems : (bsz > 4 * kBlockItems ? 4 * kBlockItems : bsz);
    for (;;) {
    __syncthreads();
    if (tid == 0) blk_at = (long long)atomicAdd(a.next_block, 1ULL);
    __syncthreads();
    const long long m0 = blk_at * bsz;
    if (m0 >= M) break;
    const long long m1 = m0 + bsz < M ? m0 + bsz : M;
    int s;
    {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.item_off[mid] <= m0) lo = mid; else hi = mid - 1;
        }
        s = lo;
    }
    const R *prim = BPrec<R>::prim(a);
    const cptr<R> rsg = (cptr<R>)BPrec<R>::rsg(bd);
    const cptr<double> cmu = (cptr<double>)bd->mu;
    const cptr<double> cfa = (cptr<double>)bd->fa;
    const cptr<double> cfb = (cptr<double>)bd->fb;
    int curmol = -1, curbra = -1;
    int nm = 0;
    long long aoff = 0, doff = 0, toff = 0;
    int bi = 0, bj = 0, lim = 0, klo = 0;
    double qs = 0.0, ds = 0.0, ABx = 0.0, ABy = 0.0, ABz = 0.0;
    double jb = 0.0, gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};

    for (long long m = m0; m <= m1; ++m) {
        if (m < m1) {
            while (a.item_off[s + 1] <= m) ++s;
        }
        const int mol = m < m1 ? a.pm[s] : -1;
        const bool newbra = (m == m1) || (s != curbra);
        if (newbra && curbra >= 0) {
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
            curbra = -1;
        }
        if (m == m1 || mol != curmol) {
            __syncthreads();
            if (curmol >= 0) {
                const int nt = nm * (nm + 1) / 2;
                for (int x = tid; x < nt; x += kGroupThreads) {
                    const double v = Lt[x];
                    if (v != 0.0) atomicAdd(&a.facc[toff + x], v);
                }
                if (kGrad) {
                    for (int x = tid; x < 3 * nm; x += kGroupThreads) {
                        const double v = lg[x];
                        if (v != 0.0) atomicAdd(&a.gacc[3 * aoff + x], v);
                    }
                }
            }
            __syncthreads();
            if (m == m1) break;
            curmol = mol;
            nm = a.mol_n[mol];
            aoff = a.mol_aoff[mol];
            doff = a.mol_doff[mol];
            toff = a.mol_toff[mol];
            for (int x = tid; x < nm * (nm + 1) / 2; x += kGroupThreads) Lt[x] = 0.0;
            for (int x = tid; x < 3 * nm; x += kGroupThreads) lg[x] = 0.0;
            __syncthreads();
        }
        if (curbra != s) {
            curbra = s;
            bi = a.pk[s];
            bj = a.pl[s];
            qs = a.pq[s];
            ds = a.pd[s];
            lim = a.lim[s];
            klo = a.klo[s];
            ABx = a.xyz[3 * (aoff + bi)] - a.xyz[3 * (aoff + bj)];
            ABy = a.xyz[3 * (aoff + bi) + 1] - a.xyz[3 * (aoff + bj) + 1];
            ABz = a.xyz[3 * (aoff + bi) + 2] - a.xyz[3 * (aoff + bj) + 2];
        }
        const long long t0 = klo + (m - a.item_off[s]) * kKetsPerItem + (long long)wave * kWave;
        if (t0 >= lim) continue;
        const long long tk = t0 + lane;
        const bool valid = (tk < lim) && (qs * a.pq[tk] >= a.tau);
        const long long t = valid ? tk : S;   // lanes without a kept quartet read the first pad entry
        const cptr<R> bra = (cptr<R>)(BPrec<R>::bra(a) + (int64_t)s * 8 * G2);
        const cptr<R> bipp = kAtoms ? (cptr<R>)(BPrec<R>::bip(a) + (int64_t)s * G2) : nullptr;
        const cptr<double> bmfp = (kAtoms && kGrad) ? (cptr<double>)(a.bmf + (int64_t)s * 2 * G2) : nullptr;
        const int k = a.pk[t], l = a.pl[t];

        R sX = R(0), eri = R(0);
        R sYa[3] = {R(0), R(0), R(0)}, sYb[3] = {R(0), R(0), R(0)};
        double kC[3] = {0.0, 0.0, 0.0};
        double CD[3] = {0.0, 0.0, 0.0};
        if (kGrad) {
#pragma unroll
            for (int c = 0; c < 3; ++c) CD[c] = a.xyz[3 * (aoff + k) + c] - a.xyz[3 * (aoff + l) + c];
        }
#pragma unroll 1
        for (int cb = 0; cb < G; ++cb) {
            R kx[G], ky[G], kz[G], ks[G], kp[G];
            R Uc[G], Vc[G][3];
            // buffer loads of the ket table: component base, primitive pair as a scalar
            // offset, ket as a 32-bit lane offset
            const unsigned tb = (unsigned)t * (unsigned)sizeof(R);
            auto ld = [&](int c, int cd) {
                const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(prim + (int64_t)c * G2 * a.pcap), (short)0, (int)(G2 * a.pcap * (int64_t)sizeof(R)),
                    0x00020000);
                const int so = (int)((int64_t)cd * a.pcap * (int64_t)sizeof(R));
                if constexpr (sizeof(R) == 8)
                    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rc, (int)tb, so, 0));
                else
                    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)tb, so, 0));
            };
#pragma unroll
            for (int d = 0; d < G; ++d) {
                const int cd = cb * G + d;
                kx[d] = ld(0, cd);
                ky[d] = ld(1, cd);
                kz[d] = ld(2, cd);
                ks[d] = ld(3, cd);
                kp[d] = kAtoms ? ld(4, cd) : R(0);
                Uc[d] = R(0);
                Vc[d][0] = Vc[d][1] = Vc[d][2] = R(0);
            }
#pragma unroll 1
            for (int ab = 0; ab < G2; ++ab) {
                // every scalar of this bra primitive in one batch of scalar loads
                const cptr<R> bp = bra + 8 * ab;
                R b[4], u[4 * G], bsw = R(0);
                double bmu = 0.0, bfa = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) b[c] = bp[c];
                if constexpr (kAtoms) {
                    bsw = bipp[ab];
                    if constexpr (kGrad) {
                        bmu = bmfp[2 * ab];
                        bfa = bmfp[2 * ab + 1];
                    }
                    asm volatile("" ::"s"(bsw));
                } else {
                    const cptr<R> up = rsg + 4 * (ab * G2 + cb * G);
#pragma unroll
                    for (int c = 0; c < 4 * G; ++c) u[c] = up[c];
#pragma unroll
                    for (int c = 0; c < 4 * G; ++c) asm volatile("" ::"s"(u[c]));
                }
                const R px = b[0], py = b[1], pz = b[2], sab = b[3];
                R U = R(0), V0 = R(0), V1 = R(0), V2 = R(0);
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    const R dx = px - kx[d], dy = py - ky[d], dz = pz - kz[d];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    // switch radius^2 kTswitch / rho (per-atom bases: sum of the stored halves)
                    const R sw = kAtoms ? bsw + kp[d] : u[4 * d];
                    const bool near = r2 < sw;
                    R E, W = R(0);
                    if (__builtin_amdgcn_ballot_w64(near)) {
                        // (rho/h, sqrt(rho/h), (rho/h)^(3/2)) from the table, or from sw
                        R q1, q2, q3;
                        if constexpr (kAtoms) {
                            q2 = rsqrt_r(sw) * R(kSqrtSwitchInvH);
                            q1 = q2 * q2;
                            q3 = q1 * q2;
                        } else {
                            q1 = u[4 * d + 1];
                            q2 = u[4 * d + 2];
                            q3 = u[4 * d + 3];
                        }
                        // T' = T / h on the table grid; sqrt(h) H and h^(3/2) g, or their far
                        // forms T'^(-1/2) and -T'^(-3/2)
                        const R Ts = r2 * q1;
                        const R y = rsqrt_r(Ts);
                        const R Tc = fmin(Ts, R(kBoysGrid - 4));
                        const R kd = rint(Tc);
                        const R dd = Tc - kd;
                        const unsigned off = __umul24((unsigned)(int)kd, (unsigned)(kBoysStride * sizeof(R)));
                        const R *ch = (const R *)((const char *)tH + off);
                        R vh = ch[6];
#pragma unroll
                        for (int m = 5; m >= 0; --m) vh = vh * dd + ch[m];
                        E = q2 * (near ? vh : y);
                        if (kGrad) {
                            const R *cg = (const R *)((const char *)tG + off);
                            R vg = cg[6];
#pragma unroll
                            for (int m = 5; m >= 0; --m) vg = vg * dd + cg[m];
                            W = q3 * (near ? vg : -(y * y * y));
                        }
                    } else {
                        const R y = rsqrt_r(r2);
                        E = y;
                        if (kGrad) W = -(y * y * y);
                    }
                    U += ks[d] * E;
                    if (kGrad) {
                        const R wk = ks[d] * W, wb = sab * W;
                        V0 += wk * dx;
                        V1 += wk * dy;
                        V2 += wk * dz;
                        Uc[d] += sab * E;
                        Vc[d][0] += wb * dx;
                        Vc[d][1] += wb * dy;
                        Vc[d][2] += wb * dz;
                    }
                }
                const R su = sab * U;
                eri += su;
                if (kGrad) {
                    R fa, fb;
                    if constexpr (kAtoms) {
                        sX += (R)bmu * su;
                        fa = (R)bfa * sab;
                        fb = sab - fa;
                    } else {
                        sX += (R)cmu[ab] * su;
                        fa = (R)cfa[ab] * sab;
                        fb = (R)cfb[ab] * sab;
                    }
                    sYa[0] += fa * V0; sYa[1] += fa * V1; sYa[2] += fa * V2;
                    sYb[0] += fb * V0; sYb[1] += fb * V1; sYb[2] += fb * V2;
                }
            }
            if (kGrad) {
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    const int cd = cb * G + d;
                    const double sc = (double)ks[d];
                    double kmu, kfa;
                    if constexpr (kAtoms) {
                        kmu = a.kmu[(int64_t)cd * a.pcap + t];
                        kfa = a.kfa[(int64_t)cd * a.pcap + t];
                    } else {
                        kmu = cmu[cd];
                        kfa = cfa[cd];
                    }
                    const double mu2 = -2.0 * kmu * sc * (double)Uc[d];
                    const double fc = kfa * sc;
#pragma unroll
                    for (int c = 0; c < 3; ++c) kC[c] += mu2 * CD[c] - fc * (double)Vc[d][c];
                }
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
                const double AB[3] = {ABx, ABy, ABz};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double GA = gam * (-2.0 * AB[c] * (double)sX + (double)sYa[c]);
                    const double GB = gam * (2.0 * AB[c] * (double)sX + (double)sYb[c]);
                    const double GC = gam * kC[c];
                    gA[c] += GA;
                    gB[c] += GB;
                    atomicAdd(&lg[3 * k + c], GC);
                    atomicAdd(&lg[3 * l + c], -(GA + GB + GC));
                }
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

size_t batched_smem_bytes(int nmax, int prec)
{
    return sizeof(double) * ((size_t)nmax * (nmax + 1) / 2 + 3 * (size_t)nmax) +
           2 * (size_t)kBoysGrid * kBoysStride * (prec == HFK_MIXED ? sizeof(float) : sizeof(double));
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
    L.boys_f = take(sizeof(float) * kBoysGrid * kBoysStride);
    L.boys_g = take(sizeof(double) * kBoysGrid * kBoysStride);
    L.boys_g_f = take(sizeof(float) * kBoysGrid * kBoysStride);
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
            L.bmf = take(sizeof(double) * 2 * g2 * PC);
        }
    }
    L.bra = take(sizeof(double) * 8 * g2 * PC);
    L.bra_f = take(sizeof(float) * 8 * g2 * PC);
    L.nitems = take(sizeof(long long) * PC);
    L.lim = take(sizeof(int) * PC);
    L.klo = take(sizeof(int) * PC);
    L.item_off = take(sizeof(long long) * (PC + 1));
    const size_t scan_n = PC > NB ? PC : NB;
    L.scan_tmp = take(sizeof(long long) * ((scan_n + 1023) / 1024 + 1));
    L.facc = take(sizeof(double) * (size_t)tri);
    L.gacc = with_grad ? take(sizeof(double) * 3 * (size_t)ntot) : 0;
    L.total = o;
    return L;
}

hipError_t launch_batched(const BLayout &L, const Basis &b, char *ws, const int64_t *atom_off_host, const double *xyz,
                          const double *dens, double tau, int prec, double *fock, double *e2, double *d_xyz,
                          int groups, hipStream_t st)
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
    if (e != hipSuccess) return e;

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
                       L.kmu ? (double *)(ws + L.kfa) : nullptr, L.kmu ? (double *)(ws + L.bmf) : nullptr);
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

    long long tri = 0;
    for (int64_t m = 0; m < nmol; ++m) tri += (long long)nm[m] * (nm[m] + 1) / 2;
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
    a.tabH_f = (const float *)(ws + L.boys_f);
    a.tabG = (const double *)(ws + L.boys_g);
    a.tabG_f = (const float *)(ws + L.boys_g_f);
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
    a.bmf = L.kmu ? (const double *)(ws + L.bmf) : nullptr;
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
    a.pcap = L.pcap;
    a.tau = tau;
    a.nmax = L.nmax;
    const size_t smem = batched_smem_bytes(L.nmax, prec);
    {
        const hipError_t ez = launch_zero_counter(a.next_block, st);
        if (ez != hipSuccess) return ez;
    }
    profile_begin(st);
    if (grad && L.atoms && !L.kmu) return hipErrorInvalidValue;   // per-atom gradient tables missing
#define HFK_B_LAUNCH(GG, RR, GR)                                                                         \
    do {                                                                                                 \
        if (L.atoms)                                                                                     \
            hipLaunchKernelGGL((k_batched<GG, RR, GR, true>), dim3(groups), dim3(kGroupThreads), smem, st, a); \
        else                                                                                             \
            hipLaunchKernelGGL((k_batched<GG, RR, GR, false>), dim3(groups), dim3(kGroupThreads), smem, st, a); \
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
