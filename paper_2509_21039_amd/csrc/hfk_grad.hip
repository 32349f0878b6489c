// Backward of the two-electron energy: dE2/dR for every atom, contracting derivative
// integrals with density products over the same screened unique quartets as the forward
// build (screening decisions held fixed), and dE2/dD = G.
//
//   E2 = sum_unique Gamma (ij|kl),   Gamma = deg (4 D_ij D_kl - D_ik D_jl - D_il D_jk)
//   (ab|cd) = S_ab S_cd E(r),  E(r) = erf(sqrt(rho) r)/r = sqrt(rho) H(T),  T = rho r^2,
//   W(r) = E'(r)/r = rho^(3/2) g(T),  g(T) = -(4/sqrt(pi)) F1(T)
//   d(ab|cd)/dA = S_ab S_cd [ -2 mu_ab (A-B) E + (a/p) (P-Q) W ]
//   d(ab|cd)/dB = S_ab S_cd [ +2 mu_ab (A-B) E + (b/p) (P-Q) W ]
//   d(ab|cd)/dC = S_ab S_cd [ -2 mu_cd (C-D) E - (c/q) (P-Q) W ]
//   d(ab|cd)/dD = -(dA + dB + dC)            (translation invariance)
// Beyond the switch E = 1/r and W = -1/r^3 exactly; below it both come from Taylor tables.
// With P = A + fb (B - A) and Q = C + fd (D - C) (fa = a/p, fb = b/p, fc = c/q, fd = d/q) the
// separation is P - Q = R_AC + fb R_BA - fd R_DC, so the W terms need only scalar sums of
// w = S_ab S_cd W weighted by the fractions (sum fa w, fa fb w, fa fd w, fb w, fb^2 w,
// fb fd w, fc w, fc fb w, fc fd w), each accumulated directly: the lane adds S_cd E,
// mu_cd S_cd E, S_cd W, fd S_cd W, fc S_cd W and fc fd S_cd W per primitive quartet and folds
// them once per bra primitive pair with the bra's weights (mu S, fa S, fb S, fa fb S, fb^2 S,
// stored per pair), and the atom vectors enter once per quartet in FP64.
//
// Per-atom bases (kAtoms): mu, a/p and rho differ per primitive pair and quartet.  The
// switch radius^2 kTswitch / rho is the sum of the stored kTswitch / p of bra and ket (as in
// the forward kernel); near steps derive sqrt(rho/h), rho/h and (rho/h)^(3/2) from it with
// one reciprocal square root; the bra's (mu, a/p) come through scalar loads and the ket's
// from two SoA tables read once per ket primitive pair.
//
// Work decomposition as in the forward kernel (items of 1024 kets of one bra, blocks of
// items fetched from a global counter in the same bra-group numbering, taken from its end
// so that the largest blocks start first, 256 kets per wave packed
// into full 64-lane chunks after the screen).  Bra-atom gradients accumulate in
// registers and are reduced across the wave when the bra changes; ket-atom gradients go to
// an LDS copy of the n x 3 gradient; each workgroup writes its copy out once.
#include "hfk_device.hpp"

namespace hfk {

struct GradArgs {
    const DevHeader *hdr;
    const BasisDev *bd;
    const double *tabH;
    const double *tabH_f;   // rows of the FP32 grid (FP64 values)
    const double *tabG;
    const double *tabG_f;
    const int *pk;
    const int *pl;
    const double *pq;
    const double *pd;
    const double *prim;
    const float *prim_f;
    const double *bra;
    const float *bra_f;
    const double *bip;      // per-atom bases: [pcap][g2] kTswitch / p of the bra pairs (and FP32 copy)
    const float *bip_f;
    const double *kmu;      // per-atom bases: [g2][pcap] mu and a/p of the ket pairs
    const double *kfa;
    const double *bgw;      // [pcap][g2][kGW] bra weights mu S, fa S, fb S, fa fb S, fb^2 S (and FP32 copy)
    const float *bgw_f;
    const long long *item_off;
    const long long *goff;      // [ngroups + 1] block offsets of the bra groups
    int64_t ngroups;
    int gshift;                 // log2 of the bras per group
    int tile;               // items per block
    const int *lim;
    const double *dens;
    const double *xdens;    // X of the two-density contraction, or NULL (Gamma from D alone)
    const double *xyz;
    double *gpriv;      // [groups][n*3]
    double *epart;      // [groups]
    unsigned long long *next_block;
    int64_t pcap;
    double tau;
    int n;
};

template <typename R> struct GPrec;
template <> struct GPrec<double> {
    static __device__ const double *prim(const GradArgs &a) { return a.prim; }
    static __device__ const double *bra(const GradArgs &a) { return a.bra; }
    static __device__ const double *bip(const GradArgs &a) { return a.bip; }
    static __device__ const double *bgw(const GradArgs &a) { return a.bgw; }
    static __device__ const double *rsg(const BasisDev *bd) { return bd->rsg; }
    static __device__ double rsqrt(double x) { return rsqrt_fp64(x); }
};
template <> struct GPrec<float> {
    static __device__ const float *prim(const GradArgs &a) { return a.prim_f; }
    static __device__ const float *bra(const GradArgs &a) { return a.bra_f; }
    static __device__ const float *bip(const GradArgs &a) { return a.bip_f; }
    static __device__ const float *bgw(const GradArgs &a) { return a.bgw_f; }
    static __device__ const float *rsg(const BasisDev *bd) { return bd->rsg_f; }
    static __device__ float rsqrt(float x) { return rsqrt_fp32(x); }
};

template <int G, typename R, bool kAtoms = false>
// One-basis FP64 kernels with up to three primitives are held to 128 VGPRs (four waves per
// SIMD); the compiler then spills a few registers outside the quartet loop only.  The others
// keep the register count they need.
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu((kAtoms || G > 3) ? 1 : 4)))
void k_grad(GradArgs a)
{
    constexpr int G2 = G * G;
    constexpr int kPComp = sizeof(R) == 8 ? 5 : 4;   // ket component holding kTswitch / p
    // FP64 forms |P-Q|^2 from the expanded table entries (4 operations, centroid-centred
    // coordinates keep the cancellation near 1e-13 bohr^2); FP32 subtracts the centres
    constexpr bool kExpand = sizeof(R) == 8;
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const int n = a.n;
    using BG = BoysGrid<R>;
    // the Boys table first (16-byte aligned rows), then the gradient partials
    R *tHG = (R *)smem;
    double *lg = (double *)(tHG + BG::table_len);   // [n*3]
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int gid = blockIdx.x;
    const long long M = a.hdr->items;
    const int S = a.hdr->sig_pairs;
    const BasisDev *bd = a.bd;
    __shared__ int wperm[kWavesPerGroup][kWaveKets];
    __shared__ long long blk_at;
    for (int x = tid; x < 3 * n; x += kGroupThreads) lg[x] = 0.0;
    // grid-scaled rows (argument T' = T / h) from the FP64 rows (one rounding for FP32):
    // coefficient m of H times h^m sqrt(h) kE, of g times h^m h^(3/2) kW (FP32 only; FP64
    // takes g from the derivative of H's degree-7 row)
    {
        // FP64: the degree-7 rows of H (tabG); FP32: H's and g's rows on the FP32 grid
        const double *gH = sizeof(R) == 8 ? a.tabG : a.tabH_f, *gG = a.tabG_f;
        for (int x = tid; x < BG::table_len; x += kGroupThreads) {
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
    __syncthreads();

    double eacc = 0.0;
    // blocks (bra group, ket block K, bra) fetched from a global counter until exhausted
    const long long NB = a.hdr->blocks;
    (void)M;
    for (;;) {
    __syncthreads();
    if (tid == 0) blk_at = (long long)atomicAdd(a.next_block, 1ULL);
    __syncthreads();
    if (blk_at >= NB) break;
    // taken from the end of the numbering: the bras are in Q-bucket order with kets t <= s,
    // so the last blocks hold the most kets; starting with them leaves the small ones for
    // the tail (he128: -1.2% FP64 and -3.3% mixed kernel time; the forward kernel keeps the
    // forward order, where the reverse measured 0.2% slower at 512 atoms)
    const long long blk = NB - 1 - blk_at;
    {
        int s;
        long long m0, m1;
        {
            // group: the last g with goff[g] <= blk; within it K-major over the group's bras
            int64_t lo = 0, hi = a.ngroups - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (a.goff[mid] <= blk) lo = mid; else hi = mid - 1;
            }
            const long long local = blk - a.goff[lo];
            s = (int)((lo << a.gshift) + (local & ((1LL << a.gshift) - 1)));
            if (s >= S) continue;
            const long long i1 = a.item_off[s + 1];
            m0 = a.item_off[s] + (local >> a.gshift) * a.tile;
            if (m0 >= i1) continue;
            m1 = m0 + a.tile < i1 ? m0 + a.tile : i1;
        }
        const R *prim = GPrec<R>::prim(a);
        const cptr<R> rsg = (cptr<R>)GPrec<R>::rsg(bd);
        const cptr<double> cmu = (cptr<double>)bd->mu;
        const cptr<double> cfa = (cptr<double>)bd->fa;
        const cptr<double> cfb = (cptr<double>)bd->fb;
        int cur = -1, bi = 0, bj = 0, lim = 0;
        double qs = 0.0, ds = 0.0;
        double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
        for (long long m = m0; m <= m1; ++m) {
            if (m < m1) {
                while (a.item_off[s + 1] <= m) ++s;
            }
            if (m == m1 || s != cur) {
                if (cur >= 0) {
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
                if (m == m1) break;
                cur = s;
                bi = a.pk[s];
                bj = a.pl[s];
                qs = a.pq[s];
                ds = a.pd[s];
                lim = a.lim[s];
            }
            const long long wbase = (m - a.item_off[s]) * kItemKets + (long long)wave * kWaveKets;
            if (wbase >= lim) continue;
            int *perm = wperm[wave];
            const int nvalid = pack_kets(wbase, lane, perm,
                                         [&](long long t) { return t < lim && qs * a.pq[t] >= a.tau; });
            if (nvalid == 0) continue;
            for (int c0 = 0; c0 < nvalid; c0 += kWave) {
                const bool valid = c0 + lane < nvalid;
                const long long t = valid ? perm[c0 + lane] : S;   // S: first pad entry
                const cptr<R> bra = (cptr<R>)(GPrec<R>::bra(a) + (int64_t)s * 8 * G2);
                const cptr<R> bipp = kAtoms ? (cptr<R>)(GPrec<R>::bip(a) + (int64_t)s * G2) : nullptr;
                const cptr<R> bwp = (cptr<R>)(GPrec<R>::bgw(a) + (int64_t)s * kGW * G2);

                // eri; sX = sum mu_ab S S E, sZ = sum mu_cd S S E; fraction-weighted sums of
                // w = S S W (names: weights of bra, then ket)
                R eri = R(0), sX = R(0), sZ = R(0);
                R wA = R(0), wAB = R(0), wB = R(0), wBB = R(0), wAD = R(0), wBD = R(0), wC = R(0), wCB = R(0),
                  wCD = R(0);
                const int k = a.pk[t], l = a.pl[t];
    #pragma unroll 1
                for (int cb = 0; cb < G; ++cb) {
                    R kx[G], ky[G], kz[G], ks[G], kp[G], kq[G];
                    R kms[G], kds[G], kcs[G], kcds[G];   // S_cd times mu_cd, fd, fc, fc fd
                    // buffer loads of the ket table: component and this cb's rows in the
                    // resource, the row as a scalar offset, the ket as a 32-bit lane offset
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
                        kp[d] = kAtoms ? ld(kPComp, d) : R(0);
                        kq[d] = kExpand ? ld(4, d) : R(0);
                    }
                    // ket weights (mu_cd, fd, fc, fc fd): per lane for per-atom bases, else
                    // uniform scalars
                    R kw[4 * G];
#pragma unroll
                    for (int d = 0; d < G; ++d) {
                        const int cd = cb * G + d;
                        if constexpr (kAtoms) {
                            const double mu = a.kmu[(int64_t)cd * a.pcap + t];
                            const double fc = a.kfa[(int64_t)cd * a.pcap + t];
                            const double fd = 1.0 - fc;
                            kms[d] = (R)mu * ks[d];
                            kcs[d] = (R)fc * ks[d];
                            kds[d] = (R)fd * ks[d];
                            kcds[d] = (R)(fc * fd) * ks[d];
                        } else {
                            const double mu = cmu[cd], fc = cfa[cd], fd = cfb[cd];
                            kw[4 * d] = (R)mu;
                            kw[4 * d + 1] = (R)fd;
                            kw[4 * d + 2] = (R)fc;
                            kw[4 * d + 3] = (R)(fc * fd);
                        }
                    }
#pragma unroll 1
                    for (int ab = 0; ab < G2; ++ab) {
                        // every scalar of this bra primitive in one batch of scalar loads: the
                        // centre and charge, the weights mu S, fa S, fb S, fa fb S, fb^2 S, and
                        // the switch data
                        const cptr<R> bp = bra + 8 * ab;
                        const cptr<R> wp = bwp + kGW * ab;
                        R b[8], bw[5], u[4 * G], bsw = R(0);
#pragma unroll
                        for (int c = 0; c < (kExpand ? 8 : 4); ++c) b[c] = bp[c];
#pragma unroll
                        for (int c = 0; c < 5; ++c) bw[c] = wp[c];
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
                        const R px = b[0], py = b[1], pz = b[2], sab = b[3];
                        R U = R(0), Y = R(0), X0 = R(0), X1 = R(0), Xc = R(0), Xcd = R(0);
                        // every lane's separation and far-field E, W first (independent across
                        // d: their reciprocal square roots issue back to back), then the near lanes
                        // overwrite theirs from the table under exec masks
                        R r2[G], E[G], W[G];
#pragma unroll
                        for (int d = 0; d < G; ++d) {
                            if (kExpand) {
                                r2[d] = fma(b[4], kx[d], fma(b[5], ky[d], fma(b[6], kz[d], kq[d] + b[7])));
                            } else {
                                const R dx = px - kx[d], dy = py - ky[d], dz = pz - kz[d];
                                r2[d] = dx * dx + dy * dy + dz * dz;
                            }
                            const R y = GradScale<R>::e_far(r2[d]);
                            E[d] = y;
                            W[d] = GradScale<R>::w_far(y);
                        }
#pragma unroll
                        for (int d = 0; d < G; ++d) {
                            const R sw = kAtoms ? bsw + kp[d] : u[4 * d];
                            if (r2[d] < sw) {
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
                                R dd;
                                const unsigned off = boys_row<R, BG::pair_stride>(r2[d], q1, dd);
                                if constexpr (sizeof(R) == 8) {
                                    double de;
                                    E[d] = q2 * boys_eval_d(tHG, off, dd, de);
                                    W[d] = q3 * (R(2.0 * GradScale<R>::kW / GradScale<R>::kE) * de);
                                } else {
                                    E[d] = q2 * boys_eval<R>(tHG, off, dd);
                                    W[d] = q3 * boys_eval<R>(tHG + BG::g_off, off, dd);
                                }
                            }
                        }
#pragma unroll
                        for (int d = 0; d < G; ++d) {
                            if constexpr (kAtoms) {
                                U = fma(ks[d], E[d], U);
                                Y = fma(kms[d], E[d], Y);
                                X0 = fma(ks[d], W[d], X0);
                                X1 = fma(kds[d], W[d], X1);
                                Xc = fma(kcs[d], W[d], Xc);
                                Xcd = fma(kcds[d], W[d], Xcd);
                            } else {
                                const R T = ks[d] * E[d], V = ks[d] * W[d];
                                U += T;
                                Y = fma(kw[4 * d], T, Y);
                                X0 += V;
                                X1 = fma(kw[4 * d + 1], V, X1);
                                Xc = fma(kw[4 * d + 2], V, Xc);
                                Xcd = fma(kw[4 * d + 3], V, Xcd);
                            }
                        }
                        eri = fma(sab, U, eri);
                        sX = fma(bw[0], U, sX);
                        sZ = fma(sab, Y, sZ);
                        wA = fma(bw[1], X0, wA);
                        wAB = fma(bw[3], X0, wAB);
                        wB = fma(bw[2], X0, wB);
                        wBB = fma(bw[4], X0, wBB);
                        wAD = fma(bw[1], X1, wAD);
                        wBD = fma(bw[2], X1, wBD);
                        wC = fma(sab, Xc, wC);
                        wCB = fma(bw[2], Xc, wCB);
                        wCD = fma(sab, Xcd, wCD);
                    }
                }
                {
                    // back from the accumulators' scales (E times kE, W times kW)
                    constexpr R iE = R(1) / GradScale<R>::kE, iW = R(1) / GradScale<R>::kW;
                    eri *= iE; sX *= iE; sZ *= iE;
                    wA *= iW; wAB *= iW; wB *= iW; wBB *= iW; wAD *= iW; wBD *= iW; wC *= iW; wCB *= iW; wCD *= iW;
                }
                if (valid) {
                    double deg = 1.0;
                    if (bi == bj) deg *= 0.5;
                    if (k == l) deg *= 0.5;
                    if (t == s) deg *= 0.5;
                    const double *Di = a.dens + (int64_t)bi * n, *Dj = a.dens + (int64_t)bj * n;
                    const double dt = a.pd[t];
                    const double gE = deg * (4.0 * ds * dt - Di[k] * Dj[l] - Di[l] * Dj[k]);
                    double gam = gE;
                    if (a.xdens) {
                        // B(X, D): the polarisation of 2 Gamma with one density replaced by X
                        const double *Xi = a.xdens + (int64_t)bi * n, *Xj = a.xdens + (int64_t)bj * n;
                        const double xs = Xi[bj], xt = a.xdens[(int64_t)k * n + l];
                        gam = deg * (4.0 * (xs * dt + ds * xt) - (Xi[k] * Dj[l] + Di[k] * Xj[l]) -
                                     (Xi[l] * Dj[k] + Di[l] * Xj[k]));
                    }
                    const double *xa = a.xyz + 3 * bi, *xb = a.xyz + 3 * bj;
                    const double *xc = a.xyz + 3 * k, *xd = a.xyz + 3 * l;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        // P - Q = R_AC + fb R_BA - fd R_DC
                        const double rac = xa[c] - xc[c], rba = xb[c] - xa[c], rdc = xd[c] - xc[c];
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
                    eacc += gE * (double)eri;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    }
    // energy partial of the workgroup
    __shared__ double ered[kWavesPerGroup];
    const double ew = wave_sum(eacc);
    if (lane == 0) ered[wave] = ew;
    __syncthreads();
    double *gp = a.gpriv + (int64_t)gid * 3 * n;
    for (int x = tid; x < 3 * n; x += kGroupThreads) gp[x] = lg[x];
    if (tid == 0) {
        double e = 0.0;
        for (int w = 0; w < kWavesPerGroup; ++w) e += ered[w];
        a.epart[gid] = e;
    }
}

// d_xyz = g_e2 * sum over workgroups; E2 = sum of partials (fixed order); d_dens = g_e2 * G.
// d_xyz = scale * sum of the workgroup partials; scale = g_e2[0], or 1 when g_e2 is NULL
// (the two-density contraction already carries it).
// Sum of the workgroups' gradient copies: a workgroup takes kRedOut consecutive outputs, each
// in kRedSlices interleaved slices of the copies (coalesced rows, many loads in flight), and
// adds the slices in a fixed order.
constexpr int kRedOut = 16, kRedSlices = 16;
static_assert(kRedOut * kRedSlices == 256, "one 256-thread workgroup");
__global__ __launch_bounds__(256) void k_grad_reduce(const double *__restrict__ gpriv, int groups, int64_t m,
                                                     const double *__restrict__ g_e2, double *__restrict__ d_xyz)
{
    __shared__ double part[kRedSlices][kRedOut];
    const int o = threadIdx.x % kRedOut, sl = threadIdx.x / kRedOut;
    const int64_t x = (int64_t)blockIdx.x * kRedOut + o;
    double s = 0.0;
    if (x < m) {
        for (int gph = sl; gph < groups; gph += kRedSlices) s += gpriv[(int64_t)gph * m + x];
    }
    part[sl][o] = s;
    __syncthreads();
    if (sl == 0 && x < m) {
        double t = part[0][o];
        for (int k = 1; k < kRedSlices; ++k) t += part[k][o];
        d_xyz[x] = g_e2 ? g_e2[0] * t : t;
    }
}

__global__ __launch_bounds__(256) void k_make_xw(int64_t n, const double *__restrict__ dens,
                                                 const double *__restrict__ gf, const double *__restrict__ g_e2,
                                                 double *__restrict__ w, double *__restrict__ x)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n * n) return;
    const int64_t i = p / n, j = p % n;
    const double wv = 0.5 * (gf[p] + gf[j * n + i]);
    w[p] = wv;
    x[p] = wv + 0.5 * g_e2[0] * dens[p];
}

hipError_t launch_make_xw(int64_t n, const double *dens, const double *g_fock, const double *g_e2, double *xw,
                          hipStream_t st)
{
    const int64_t n2 = n * n;
    hipLaunchKernelGGL(k_make_xw, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n, dens, g_fock, g_e2, xw,
                       xw + n2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_axpy_dev(int64_t m, const double *__restrict__ g_e2,
                                                  const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) y[p] += g_e2[0] * x[p];
}

hipError_t launch_axpy_dev(int64_t m, const double *g_e2, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy_dev, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, g_e2, x, y);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_grad_energy(const double *__restrict__ epart, int groups,
                                                     double *__restrict__ e2)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < groups; b += 256) s += epart[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *e2 = red[0];
}

__global__ __launch_bounds__(256) void k_scale_copy(const double *__restrict__ src, int64_t m,
                                                    const double *__restrict__ g_e2, double *__restrict__ dst)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) dst[x] = g_e2[0] * src[x];
}

size_t grad_smem_bytes(int64_t n, int prec)
{
    return sizeof(double) * 3 * (size_t)n +
           (prec == HFK_MIXED ? sizeof(float) * BoysGrid<float>::table_len
                              : sizeof(double) * BoysGrid<double>::table_len);
}

template <int G, typename R>
static int grad_res(bool atoms, size_t smem)
{
    int nb = 0;
    const hipError_t e = atoms ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grad<G, R, true>, kGroupThreads, smem)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grad<G, R, false>, kGroupThreads, smem);
    return e == hipSuccess ? nb : 0;
}

// Workgroups of the gradient kernel that fit on one CU at once (registers and LDS); 0 if the
// runtime cannot tell.
int grad_resident_groups(int g, int prec, int64_t n, bool atoms)
{
    const size_t smem = grad_smem_bytes(n, prec);
    if (prec == HFK_MIXED) {
        switch (g) {
        case 1: return grad_res<1, float>(atoms, smem);
        case 2: return grad_res<2, float>(atoms, smem);
        case 3: return grad_res<3, float>(atoms, smem);
        case 4: return grad_res<4, float>(atoms, smem);
        case 5: return grad_res<5, float>(atoms, smem);
        default: return grad_res<6, float>(atoms, smem);
        }
    }
    switch (g) {
    case 1: return grad_res<1, double>(atoms, smem);
    case 2: return grad_res<2, double>(atoms, smem);
    case 3: return grad_res<3, double>(atoms, smem);
    case 4: return grad_res<4, double>(atoms, smem);
    case 5: return grad_res<5, double>(atoms, smem);
    default: return grad_res<6, double>(atoms, smem);
    }
}

template <int G, typename R>
static hipError_t launch_grad_t(const GradArgs &a, int groups, size_t smem, bool atoms, hipStream_t st)
{
    const hipError_t ez = launch_zero_counter(a.next_block, st);
    if (ez != hipSuccess) return ez;
    profile_begin(st);
    if (atoms)
        hipLaunchKernelGGL((k_grad<G, R, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    else
        hipLaunchKernelGGL((k_grad<G, R, false>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    profile_end(st);
    return hipGetLastError();
}

hipError_t launch_grad(const Layout &L, const Basis &b, char *ws, const double *xyz, const double *dens,
                       double tau, int prec, const double *g_e2, const double *xdens, const double *fock_in,
                       double *d_xyz, double *d_dens, double *e2_out, hipStream_t st)
{
    GradArgs a;
    a.hdr = (const DevHeader *)(ws + L.hdr);
    a.bd = (const BasisDev *)(ws + L.basis);
    a.tabH = (const double *)(ws + L.boys);
    a.tabH_f = (const double *)(ws + L.boys_f);
    a.tabG = (const double *)(ws + L.boys_g);
    a.tabG_f = (const double *)(ws + L.boys_g_f);
    a.pk = (const int *)(ws + L.pk);
    a.pl = (const int *)(ws + L.pl);
    a.pq = (const double *)(ws + L.pq);
    a.pd = (const double *)(ws + L.pd);
    a.prim = (const double *)(ws + L.prim);
    a.prim_f = (const float *)(ws + L.prim_f);
    a.bra = (const double *)(ws + L.bra);
    a.bra_f = (const float *)(ws + L.bra_f);
    const bool at = L.atoms && L.pmu;
    a.bip = at ? (const double *)(ws + L.bip) : nullptr;
    a.bip_f = at ? (const float *)(ws + L.bip_f) : nullptr;
    a.kmu = at ? (const double *)(ws + L.pmu) : nullptr;
    a.kfa = at ? (const double *)(ws + L.pfa) : nullptr;
    a.bgw = (const double *)(ws + L.bgw);
    a.bgw_f = (const float *)(ws + L.bgw_f);
    a.item_off = (const long long *)(ws + L.item_off);
    a.lim = (const int *)(ws + L.lim);
    a.goff = (const long long *)(ws + L.goff);
    a.ngroups = L.ngroups;
    a.gshift = L.gshift;
    a.tile = L.tile;
    a.dens = dens;
    a.xdens = xdens;
    a.xyz = xyz;
    a.gpriv = (double *)(ws + L.grad);
    a.epart = (double *)(ws + L.grad) + (size_t)L.groups * 3 * L.n;
    a.next_block = &((DevHeader *)(ws + L.hdr))->next_block;
    a.pcap = L.pcap;
    a.tau = tau;
    a.n = (int)L.n;
    const size_t smem = grad_smem_bytes(L.n, prec);
    hipError_t err;
    if (prec == HFK_MIXED) {
        switch (b.g) {
        case 1: err = launch_grad_t<1, float>(a, L.groups, smem, at, st); break;
        case 2: err = launch_grad_t<2, float>(a, L.groups, smem, at, st); break;
        case 3: err = launch_grad_t<3, float>(a, L.groups, smem, at, st); break;
        case 4: err = launch_grad_t<4, float>(a, L.groups, smem, at, st); break;
        case 5: err = launch_grad_t<5, float>(a, L.groups, smem, at, st); break;
        default: err = launch_grad_t<6, float>(a, L.groups, smem, at, st); break;
        }
    } else {
        switch (b.g) {
        case 1: err = launch_grad_t<1, double>(a, L.groups, smem, at, st); break;
        case 2: err = launch_grad_t<2, double>(a, L.groups, smem, at, st); break;
        case 3: err = launch_grad_t<3, double>(a, L.groups, smem, at, st); break;
        case 4: err = launch_grad_t<4, double>(a, L.groups, smem, at, st); break;
        case 5: err = launch_grad_t<5, double>(a, L.groups, smem, at, st); break;
        default: err = launch_grad_t<6, double>(a, L.groups, smem, at, st); break;
        }
    }
    if (err != hipSuccess) return err;
    const int64_t m = 3 * L.n;
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((m + kRedOut - 1) / kRedOut)), dim3(256), 0, st, a.gpriv,
                       L.groups, m, xdens ? nullptr : g_e2, d_xyz);
    if (e2_out) hipLaunchKernelGGL(k_grad_energy, dim3(1), dim3(256), 0, st, a.epart, L.groups, e2_out);
    if (d_dens) {
        const int64_t n2 = L.n * L.n;
        hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, fock_in, n2, g_e2,
                           d_dens);
    }
    return hipGetLastError();
}

}  // namespace hfk
