// Forward Fock build on one GPU: the unique-quartet loop with the primitive contraction
// and the six-way scatter of the Hartree--Fock kernel (Background section, kernel
// listing), re-designed for CDNA4.
//
// Work decomposition.  Significant pairs are stored in Q-bucketed order (t = 0 .. S-1),
// so the kets kept by the screen for a bra s form a prefix t < lim_s (t <= s keeps each
// unordered quartet once; a lane-level test Q_s Q_t >= tau handles the partial bucket).
// An item is (bra s, 1024 consecutive kets).  Persistent workgroups fetch blocks of up to
// kTileItems items of one bra from a global counter (the cost per item varies with the
// bra's surroundings, and static ranges left a long tail of slow workgroups).  Blocks are
// numbered ket-block-major within groups of bras (1024 unless tuned), so the workgroups running
// together read the same kets, which then come from L2.  Each of a workgroup's four waves
// takes 256 kets of an item and runs them as 64-lane chunks, one ket per lane; the bra's
// primitive data are wave-uniform.  In the hybrid form the wave first packs the kets that
// pass the screen (ballot + lane count, order kept so loads stay coalesced) into full
// chunks.
//
// Accumulation (replacing one global FP64 atomic per update):
//   F_ij += 4 D_kl v   per-lane register, reduced across the wave when the bra changes
//   F_kl += 4 D_ij v   coalesced read-modify-write of a per-workgroup vector over kets
//                      (atomics into shared copies when per-workgroup ones exceed the budget)
//   F_ik, F_il, F_jk, F_jl -= ...   LDS atomics into copies of rows i and j of F, flushed
//                      to a per-workgroup copy of F (or with global atomics) once per bra
// and a final kernel sums the copies, symmetrises and forms E2.
//
// Deterministic strategy (kDet): the same arithmetic with every sum taken in a fixed order,
// so repeated builds agree bit for bit.  Blocks are dealt out by a static grid stride
// instead of the global counter and every workgroup owns its copy of F and of the ket
// vector.  Within a workgroup each wave stages its exchange updates (k, l, v) in LDS; at the
// end of every item the waves apply them to rows i and j one wave after the other (a wave's
// atomic adds within one instruction are applied by the LDS in a fixed lane order), and the
// F_ij partial sums of the four waves are added in wave order.  The final kernels sum the
// workgroup copies in workgroup order.
#include "hfk_device.hpp"

namespace hfk {

struct FockArgs {
    const DevHeader *hdr;
    const BasisDev *bd;
    const double *boys;
    const double *boys_f;   // rows of the FP32 grid (FP64 values, rounded once into LDS)
    const int *pk;
    const int *pl;
    const double *pq;
    const double *pd;
    const double *prim;
    const float *prim_f;
    const double *bra;
    const float *bra_f;
    const double *bip;          // per-atom bases: [pcap][g2] kTswitch / p of the bra primitive pairs
    const float *bip_f;
    const long long *item_off;
    const long long *goff;      // [ngroups + 1] block offsets of the bra groups
    int64_t ngroups;
    int gshift;                 // log2 of the bras per group
    int tile;                   // items per block
    const int *lim;
    const double *dens;
    double *fpriv;
    double *jcol;       // [jcopies][pcap]
    unsigned long long *quartets;
    unsigned long long *next_block;
    int64_t pcap;
    double tau;
    int n;
    int strategy;
    int jcopies;        // ket vectors: one per workgroup if equal to the grid, else shared (atomics)
};

template <typename R> struct Prec;
template <> struct Prec<double> {
    static __device__ const double *prim(const FockArgs &a) { return a.prim; }
    static __device__ const double *bra(const FockArgs &a) { return a.bra; }
    static __device__ const double *bip(const FockArgs &a) { return a.bip; }
    static __device__ const double *boys(const FockArgs &a) { return a.boys; }
    static __device__ const double *rho(const BasisDev *bd) { return bd->rho; }
    static __device__ const double *srho(const BasisDev *bd) { return bd->srho; }
    static __device__ const double *r2sw(const BasisDev *bd) { return bd->r2sw; }
    static __device__ const double *rs(const BasisDev *bd) { return bd->rs; }
    static __device__ const double *rsn(const BasisDev *bd) { return bd->rsn; }
    static __device__ double rsqrt(double x) { return rsqrt_fp64(x); }
    // The hybrid kernel's FP64 accumulator carries -2 times the sum, which lets the Newton
    // step of the reciprocal square root fold into the product: with the hardware estimate
    // y, y1 = y (3 - x y^2) / 2 and -2 s y1 = (s y) (x y^2 - 3).  The far-field term of a
    // primitive quartet is returned as the two factors a = s y and b = x y^2 - 3 (three
    // operations after rsq; the accumulating FMA makes four), so that near lanes can replace
    // both before the one FMA that adds the term.
    static constexpr double kAccScale = -2.0;
    static __device__ void far_split(double s, double x, double &a, double &b)
    {
        const double y = __builtin_amdgcn_rsq(x);
        a = s * y;
        b = fma(x, y * y, -3.0);
    }
};
template <> struct Prec<float> {
    static __device__ const float *prim(const FockArgs &a) { return a.prim_f; }
    static __device__ const float *bra(const FockArgs &a) { return a.bra_f; }
    static __device__ const float *bip(const FockArgs &a) { return a.bip_f; }
    static __device__ const double *boys(const FockArgs &a) { return a.boys_f; }
    static __device__ const float *rho(const BasisDev *bd) { return bd->rho_f; }
    static __device__ const float *srho(const BasisDev *bd) { return bd->srho_f; }
    static __device__ const float *r2sw(const BasisDev *bd) { return bd->r2sw_f; }
    static __device__ const float *rs(const BasisDev *bd) { return bd->rs_f; }
    static __device__ const float *rsn(const BasisDev *bd) { return bd->rsn_f; }
    static __device__ float rsqrt(float x) { return rsqrt_fp32(x); }
    static constexpr float kAccScale = 1.0f;   // no Newton step in FP32
    static __device__ void far_split(float s, float x, float &a, float &b) { a = s; b = rsqrt_fp32(x); }
};

// Polynomial of the table row nearest to T (T below the switch, so the row exists).
template <typename R>
__device__ inline R boys_nearest_row(R T, const R *__restrict__ tab)
{
    using BG = BoysGrid<R>;
    const int k = (int)(T * R(BG::inv_h) + R(0.5));
    const R d = T - (R)k * R(BG::h);
    const R *c = tab + k * BG::stride;
    R v = c[BG::order - 1];
#pragma unroll
    for (int m = BG::order - 2; m >= 0; --m) v = v * d + c[m];
    return v;
}

// H(T) = erf(sqrt T)/sqrt T: table row below the switch, T^(-1/2) above it (both
// evaluated, one selected).
template <typename R>
__device__ inline R boys_h(R T, const R *__restrict__ tab)
{
    const R far = Prec<R>::rsqrt(fmax(T, R(1e-30)));
    const R Tc = fmin(T, R(kTswitch + 0.5));
    const R v = boys_nearest_row<R>(Tc, tab);
    return T < R(kTswitch) ? v : far;
}

// The lane's ket primitives are consumed in blocks of G (fixed c, all d), so only G of
// them occupy registers at a time; the bra primitive pair ab runs in the middle loop.

// Contracted (bra | ket) for one lane, every primitive quartet evaluated in place.
// (ab|cd) = S_ab S_cd sqrt(rho) H(rho |P - Q|^2).
template <int G, typename R>
__device__ inline R quartet_eri_direct(const R *__restrict__ lbra, const R *__restrict__ prim, int64_t pcap,
                                       int64_t t, const R *__restrict__ lrs, const R *__restrict__ tab)
{
    constexpr int G2 = G * G;
    R eri = R(0);
#pragma unroll 1
    for (int cb = 0; cb < G; ++cb) {
        R kx[G], ky[G], kz[G], ks[G];
#pragma unroll
        for (int d = 0; d < G; ++d) {
            const int cd = cb * G + d;
            kx[d] = prim[(int64_t)(0 * G2 + cd) * pcap + t];
            ky[d] = prim[(int64_t)(1 * G2 + cd) * pcap + t];
            kz[d] = prim[(int64_t)(2 * G2 + cd) * pcap + t];
            ks[d] = prim[(int64_t)(3 * G2 + cd) * pcap + t];
        }
#pragma unroll 1
        for (int ab = 0; ab < G2; ++ab) {
            const R px = lbra[4 * ab], py = lbra[4 * ab + 1], pz = lbra[4 * ab + 2];
            R acc = R(0);
#pragma unroll
            for (int d = 0; d < G; ++d) {
                const int x = ab * G2 + cb * G + d;
                const R dx = px - kx[d], dy = py - ky[d], dz = pz - kz[d];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R h = boys_h<R>(r2 * lrs[2 * x], tab);
                acc += (ks[d] * lrs[2 * x + 1]) * h;
            }
            eri += lbra[4 * ab + 3] * acc;
        }
    }
    return eri;
}

// kAccScale sqrt(h) H(T) for a lane below the switch radius (the table is scaled to match).
template <typename R>
__device__ inline R boys_near(R r2, R rsh, const R *__restrict__ tab)
{
    R d;
    const unsigned off = boys_row<R>(r2, rsh, d);
    return boys_eval<R>(tab, off, d);
}

// Contracted (bra | ket), far field first: for one bra primitive pair a lane forms |P-Q|^2
// of its G ket primitive pairs and their far-field terms S_cd / |P-Q| (exact beyond the
// switch radius; the G reciprocal square roots issue back to back); then, under exec masks,
// lanes below the switch radius replace a term by S_cd sqrt(rho/h) * sqrt(h) H(T) from the
// grid table (a wave with no near lane, the common case once kets are spatially sorted, skips
// the table part, and only near lanes read the table from LDS); the terms are added last, in
// one branch-free run of FMAs.  Far values of near lanes (|P-Q|^2 may be zero or round
// below it) are discarded, never added.  Lanes without a kept quartet point at a pad entry
// (centres 1e6 bohr away, zero weight), so they are never near and add nothing.  Uniform data come through scalar loads issued together
// at the top of each bra primitive: (Px, Py, Pz, S, -2Px, -2Py, -2Pz, |P|^2) and, per
// primitive quartet, (switch radius^2, rho/h, sqrt(rho/h)).
// FP64 forms |P-Q|^2 as |P|^2 + |Q|^2 - 2 P.Q (4 operations; with centroid-centred
// coordinates the cancellation stays near 1e-13 bohr^2 absolute); FP32 subtracts the
// centres directly, which its precision needs.  The FP64 accumulator holds -2 times the sum
// (kAccScale; the near-branch table is scaled to match), which saves one operation in each
// Newton step of the reciprocal square root; the result is scaled back once per quartet.
// Per-atom bases (kAtoms): rho = p q / (p + q) differs per quartet, so the scalar combo
// table gives way to kTswitch / p of the bra (uniform, bip) and of the ket (last ket
// component): their sum is kTswitch / rho, the switch radius^2 itself, so the test costs
// one add; only the near branch needs sqrt(rho / h) = sqrt(kTswitch / h) / sqrt(that sum)
// (one reciprocal square root); the far field S_cd / |P-Q| does not depend on rho at all.
template <int G, typename R, bool kAtoms = false>
__device__ inline R quartet_eri_hybrid(cptr<R> bra, const R *__restrict__ prim, int64_t pcap, unsigned t,
                                       cptr<R> rsn, const R *__restrict__ tab, cptr<R> bip = nullptr)
{
    constexpr int G2 = G * G;
    constexpr bool kExpand = sizeof(R) == 8;
    constexpr int kPComp = kExpand ? 5 : 4;   // ket component holding kTswitch / p (per-atom bases)
    // FP32 with up to three primitives loads the next cb's ket data while it works on this one
    // (the kernel has registers to spare: he1024 mixed 209.6 -> 203.2 ms); FP64 would drop from
    // five to four waves per SIMD for it and run slower (he512 67.9 -> 73.5 ms), so it loads
    // each cb at its start
    constexpr bool kPrefetch = sizeof(R) == 4 && G <= 3;
    constexpr int kSlots = kPrefetch ? 2 : 1;
    R eri = R(0);
    R kx[kSlots][G], ky[kSlots][G], kz[kSlots][G], ks[kSlots][G], kq[kSlots][G], kp[kSlots][G];
    // buffer loads: one resource per component over the G rows of a cb, the row as a scalar
    // offset and the ket as a 32-bit lane offset (no 64-bit address math per lane)
    const unsigned tb = t * (unsigned)sizeof(R);
    auto load_cb = [&](int cbl, int slot) {
        auto ld = [&](int c, int d) {
            return ket_load<R>(ket_rows(prim, (int64_t)c * G2 + cbl * G, pcap, G), tb,
                               (int)((int64_t)d * pcap * (int64_t)sizeof(R)));
        };
#pragma unroll
        for (int d = 0; d < G; ++d) {
            kx[slot][d] = ld(0, d);
            ky[slot][d] = ld(1, d);
            kz[slot][d] = ld(2, d);
            ks[slot][d] = ld(3, d);
            kq[slot][d] = kExpand ? ld(4, d) : R(0);
            kp[slot][d] = kAtoms ? ld(kPComp, d) : R(0);
        }
    };
    constexpr int kCbUnroll = kPrefetch ? G : 1;   // the slots must be compile-time indices
    if constexpr (kPrefetch) load_cb(0, 0);
#pragma unroll kCbUnroll
    for (int cb = 0; cb < G; ++cb) {
        const int cur = kPrefetch ? (cb & 1) : 0;
        if constexpr (kPrefetch) {
            if (cb + 1 < G) load_cb(cb + 1, cur ^ 1);
        } else {
            load_cb(cb, 0);
        }
#pragma unroll 1
        for (int ab = 0; ab < G2; ++ab) {
            const cptr<R> bp = bra + 8 * ab;
            R b[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) b[c] = bp[c];
            R acc = R(0);
            if constexpr (kAtoms) {
                const R bi = bip[ab];
                asm volatile("" ::"s"(bi));
                R r2[G], fa[G], fb[G];
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    if (kExpand) {
                        r2[d] = fma(b[4], kx[cur][d], fma(b[5], ky[cur][d], fma(b[6], kz[cur][d], kq[cur][d] + b[7])));
                    } else {
                        const R dx = b[0] - kx[cur][d], dy = b[1] - ky[cur][d], dz = b[2] - kz[cur][d];
                        r2[d] = dx * dx + dy * dy + dz * dz;
                    }
                    Prec<R>::far_split(ks[cur][d], r2[d], fa[d], fb[d]);
                }
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    const R sw = bi + kp[cur][d];   // kTswitch / rho
                    if (r2[d] < sw) {
                        const R y = rsqrt_r(sw) * R(BoysGrid<R>::sqrt_sw_inv_h);   // sqrt(rho / h)
                        fa[d] = ks[cur][d] * y;
                        fb[d] = boys_near<R>(r2[d], y * y, tab);
                    }
                }
#pragma unroll
                for (int d = 0; d < G; ++d) acc = fma(fa[d], fb[d], acc);
            } else {
                const cptr<R> up = rsn + 3 * (ab * G2 + cb * G);
                R u[3 * G];
#pragma unroll
                for (int c = 0; c < 3 * G; ++c) u[c] = up[c];
                // keep every uniform load in one batch at the top (not sunk into the branches)
#pragma unroll
                for (int c = 0; c < 3 * G; ++c) asm volatile("" ::"s"(u[c]));
                R r2[G], fa[G], fb[G];
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    if (kExpand) {
                        r2[d] = fma(b[4], kx[cur][d], fma(b[5], ky[cur][d], fma(b[6], kz[cur][d], kq[cur][d] + b[7])));
                    } else {
                        const R dx = b[0] - kx[cur][d], dy = b[1] - ky[cur][d], dz = b[2] - kz[cur][d];
                        r2[d] = dx * dx + dy * dy + dz * dz;
                    }
                    Prec<R>::far_split(ks[cur][d], r2[d], fa[d], fb[d]);
                }
#pragma unroll
                for (int d = 0; d < G; ++d) {
                    if (r2[d] < u[3 * d]) {
                        fa[d] = ks[cur][d] * u[3 * d + 2];
                        fb[d] = boys_near<R>(r2[d], u[3 * d + 1], tab);
                    }
                }
#pragma unroll
                for (int d = 0; d < G; ++d) acc = fma(fa[d], fb[d], acc);
            }
            eri += b[3] * acc;
        }
    }
    return eri * (R(1) / Prec<R>::kAccScale);
}

// LDS carve-up of the quartet kernel (bytes, 16-byte aligned pieces).
template <typename R> struct FockSmem {
    static constexpr int kCombos = kMaxG2 * kMaxG2 / 16;                    // g <= 4 here: 256 combos
    static constexpr size_t tab_bytes = sizeof(R) * BoysGrid<R>::rows * BoysGrid<R>::stride;
    static constexpr size_t uni_bytes = 4 * sizeof(R) * 16 + 2 * sizeof(R) * kCombos;   // bra, (rho, srho)
    // deterministic strategy: per wave, kWaveKets staged updates (v, then k and l)
    static constexpr size_t stage_bytes = kWavesPerGroup * kWaveKets * (sizeof(double) + 2 * sizeof(int));
    static size_t total(int n, bool split, bool det = false)
    {
        return sizeof(double) * 2 * (size_t)n + tab_bytes + (split ? 0 : uni_bytes) + (det ? stage_bytes : 0);
    }
};

template <int G, typename R, bool kSplit, bool kAtoms = false, bool kDet = false>
__global__ __launch_bounds__(kGroupThreads) void k_fock(FockArgs a)
{
    constexpr int G2 = G * G;
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const int n = a.n;
    // the table first, so its row addresses need no base register
    char *sp = (char *)smem;
    R *tab = (R *)sp;                       // Boys table (grid-scaled for the hybrid form)
    sp += FockSmem<R>::tab_bytes;
    double *rowi = (double *)sp;
    double *rowj = rowi + n;
    sp += sizeof(double) * 2 * (size_t)n;
    R *lbra = (R *)sp;                      // direct form: [G2][4] Px, Py, Pz, S of the current bra
    R *luni = lbra + 4 * 16;                // direct form: (rho, sqrt rho) per primitive quartet
    // deterministic strategy: staged exchange updates of each wave (the hybrid form has no
    // direct-form slots, so they start at the same place)
    double *stv = (double *)sp;                                   // [waves][kWaveKets] v
    int *stk = (int *)(stv + kWavesPerGroup * kWaveKets);         // [waves][kWaveKets] k
    int *stl = stk + kWavesPerGroup * kWaveKets;                  // [waves][kWaveKets] l
    __shared__ double jbs[kWavesPerGroup];
    __shared__ int bra_at[2];
    __shared__ double bra_qd[2];
    __shared__ int wperm[kWavesPerGroup][kWaveKets];

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int gid = blockIdx.x, ng = gridDim.x;
    const long long M = a.hdr->items;
    const int S = a.hdr->sig_pairs;
    const BasisDev *bd = a.bd;

    {
        // the rows of this precision's grid, from FP64 values (one rounding for FP32); the
        // hybrid form scales coefficient m by h^m sqrt(h) and the accumulator's scale
        using BG = BoysGrid<R>;
        const double *gtab = Prec<R>::boys(a);
        for (int x = tid; x < BG::rows * BG::stride; x += kGroupThreads) {
            const int m = x % BG::stride;
            double sc = 1.0;
            if (kSplit) {
                sc = sqrt(BG::h) * (double)Prec<R>::kAccScale;
                for (int e = 0; e < m; ++e) sc *= BG::h;
            }
            tab[x] = (R)(gtab[x] * sc);
        }
    }
    if (!kSplit) {
        for (int x = tid; x < G2 * G2; x += kGroupThreads) {
            luni[2 * x] = Prec<R>::rho(bd)[x];
            luni[2 * x + 1] = Prec<R>::srho(bd)[x];
        }
    }
    const cptr<R> crs = (cptr<R>)Prec<R>::rsn(bd);
    const bool jshared = a.jcopies < ng;
    double *jcol = a.jcol + (int64_t)(gid % a.jcopies) * a.pcap;
    const bool priv = kDet || a.strategy == HFK_STRATEGY_PRIVATE;
    double *fp = priv ? a.fpriv + (int64_t)gid * n * n : a.fpriv;
    if (priv) {
        for (int64_t x = tid; x < (int64_t)n * n; x += kGroupThreads) fp[x] = 0.0;
    }
    if (!jshared) {
        for (int64_t x = tid; x < S; x += kGroupThreads) jcol[x] = 0.0;
    }
    __syncthreads();
    const R *prim = Prec<R>::prim(a);
    unsigned long long kept = 0;
    __shared__ long long blk_at;
    const long long NB = a.hdr->blocks;
    (void)M;
    // blocks (bra group, ket block K, bra) fetched from a global counter until exhausted, or
    // dealt out by a static grid stride (deterministic strategy)
    for (long long it = 0;; ++it) {
    if (!kDet && tid == 0) blk_at = (long long)atomicAdd(a.next_block, 1ULL);
    __syncthreads();
    const long long blk = kDet ? (long long)gid + it * ng : blk_at;
    __syncthreads();
    if (blk >= NB) break;
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
        if (m0 >= i1) continue;   // this bra has fewer blocks than the group's longest
        m1 = m0 + a.tile < i1 ? m0 + a.tile : i1;
    }
    int cur = -1, bi = 0, bj = 0;
    double qs = 0.0, ds = 0.0, jb = 0.0;
    int lim = 0;

    for (long long m = m0; m <= m1; ++m) {
        if (m < m1) {
            while (a.item_off[s + 1] <= m) ++s;
        }
        if (m == m1 || s != cur) {
            if (cur >= 0) {
                // flush the finished bra: F_ij from the wave partial sums, then rows i, j
                const double w = wave_sum(jb);
                if constexpr (kDet) {
                    // the four wave sums in wave order
                    if (lane == 0) jbs[wave] = w;
                    __syncthreads();
                    if (tid == 0) {
                        double sw = jbs[0];
#pragma unroll
                        for (int wv = 1; wv < kWavesPerGroup; ++wv) sw += jbs[wv];
                        if (sw != 0.0) rowi[bj] += 4.0 * sw;
                    }
                } else {
                    if (lane == 0 && w != 0.0) atomicAdd(&rowi[bj], 4.0 * w);
                }
                jb = 0.0;
                __syncthreads();
                double *fi = fp + (int64_t)bi * n, *fj = fp + (int64_t)bj * n;
                if (priv) {
                    if (bi == bj) {
                        for (int c = tid; c < n; c += kGroupThreads) fi[c] += rowi[c] + rowj[c];
                    } else {
                        for (int c = tid; c < n; c += kGroupThreads) {
                            fi[c] += rowi[c];
                            fj[c] += rowj[c];
                        }
                    }
                } else {
                    for (int c = tid; c < n; c += kGroupThreads) {
                        const double vi = rowi[c], vj = rowj[c];
                        if (vi != 0.0) atomicAdd(&fi[c], vi);
                        if (vj != 0.0) atomicAdd(&fj[c], vj);
                    }
                }
                __syncthreads();
            }
            if (m == m1) break;
            const R *br = Prec<R>::bra(a) + (int64_t)s * 8 * G2;
            if (!kSplit && tid < 4 * G2) lbra[tid] = br[8 * (tid / 4) + tid % 4];
            if (tid == 0) {
                bra_at[0] = a.pk[s];
                bra_at[1] = a.pl[s];
                bra_qd[0] = a.pq[s];
                bra_qd[1] = a.pd[s];
            }
            for (int c = tid; c < n; c += kGroupThreads) {
                rowi[c] = 0.0;
                rowj[c] = 0.0;
            }
            __syncthreads();
            cur = s;
            bi = bra_at[0];
            bj = bra_at[1];
            qs = bra_qd[0];
            ds = bra_qd[1];
            lim = a.lim[s];
        }
        const long long wbase = (m - a.item_off[s]) * kItemKets + (long long)wave * kWaveKets;
        if constexpr (!kDet) {
            if (wbase >= lim) continue;
        }
        // one 64-lane chunk: ket t per lane (valid: kept by the screen), scatter of v
        // (deterministic strategy: the exchange updates are staged at position `slot`)
        auto chunk = [&](int t, bool valid, int slot) {
            R eri;
            if (kSplit)
                eri = quartet_eri_hybrid<G, R, kAtoms>(
                    (cptr<R>)(Prec<R>::bra(a) + (int64_t)s * 8 * G2), prim, a.pcap, (unsigned)t, crs, tab,
                    kAtoms ? (cptr<R>)(Prec<R>::bip(a) + (int64_t)s * G2) : nullptr);
            else
                eri = quartet_eri_direct<G, R>(lbra, prim, a.pcap, t, luni, tab);
            const int k = a.pk[t], l = a.pl[t];
            double deg = 1.0;
            if (bi == bj) deg *= 0.5;
            if (k == l) deg *= 0.5;
            if (t == s) deg *= 0.5;
            const double v = valid ? (double)eri * deg : 0.0;
            jb = fma(a.pd[t], v, jb);
            if (valid) {
                ++kept;
                if (jshared)
                    atomicAdd(&jcol[t], 4.0 * ds * v);
                else
                    jcol[t] += 4.0 * ds * v;
                if constexpr (kDet) {
                    stv[wave * kWaveKets + slot] = v;
                    stk[wave * kWaveKets + slot] = k;
                    stl[wave * kWaveKets + slot] = l;
                } else {
                    const double *Di = a.dens + (int64_t)bi * n;
                    const double *Dj = a.dens + (int64_t)bj * n;
                    atomicAdd(&rowi[k], -Dj[l] * v);
                    atomicAdd(&rowi[l], -Dj[k] * v);
                    atomicAdd(&rowj[k], -Di[l] * v);
                    atomicAdd(&rowj[l], -Di[k] * v);
                }
            }
        };
        if constexpr (kDet) {
            int nvalid = 0;
            if (wbase < lim) {
                int *perm = wperm[wave];
                nvalid = pack_kets(wbase, lane, perm, [&](long long t) { return t < lim && qs * a.pq[t] >= a.tau; });
                for (int c0 = 0; c0 < nvalid; c0 += kWave) {
                    const bool valid = c0 + lane < nvalid;
                    chunk(valid ? perm[c0 + lane] : S, valid, c0 + lane);
                }
            }
            // every wave's updates are staged; apply them wave after wave
            __syncthreads();
            const double *Di = a.dens + (int64_t)bi * n;
            const double *Dj = a.dens + (int64_t)bj * n;
            for (int wv = 0; wv < kWavesPerGroup; ++wv) {
                if (wave == wv) {
                    for (int e = lane; e < nvalid; e += kWave) {
                        const double v = stv[wave * kWaveKets + e];
                        const int k = stk[wave * kWaveKets + e], l = stl[wave * kWaveKets + e];
                        atomicAdd(&rowi[k], -Dj[l] * v);
                        atomicAdd(&rowi[l], -Dj[k] * v);
                        atomicAdd(&rowj[k], -Di[l] * v);
                        atomicAdd(&rowj[l], -Di[k] * v);
                    }
                }
                __syncthreads();
            }
        } else if (kSplit) {
            // keep the screened kets of this wave's 256, in order, packed into full chunks
            int *perm = wperm[wave];
            const int nvalid = pack_kets(wbase, lane, perm,
                                         [&](long long t) { return t < lim && qs * a.pq[t] >= a.tau; });
            if (nvalid == 0) continue;
            for (int c0 = 0; c0 < nvalid; c0 += kWave) {
                const bool valid = c0 + lane < nvalid;
                chunk(valid ? perm[c0 + lane] : S, valid, 0);   // S: first pad entry
            }
            __builtin_amdgcn_wave_barrier();
        } else {
            for (int c = 0; c < kSubChunks; ++c) {
                const long long t0 = wbase + c * kWave;
                if (t0 >= lim) break;
                const long long t = t0 + lane;   // < S + 64 <= pcap: padded tables
                chunk((int)t, t < lim && qs * a.pq[t] >= a.tau, 0);
            }
        }
    }
    }
    // survivors: one atomic per wave
    for (int off = 32; off > 0; off >>= 1) kept += __shfl_xor(kept, off, 64);
    if (lane == 0 && kept) atomicAdd(a.quartets, kept);
}

// ------------------------------------------------------------------ final reduction

__global__ __launch_bounds__(256) void k_sum_private(const double *__restrict__ fpriv, int groups, int64_t n2,
                                                     double *__restrict__ fsum)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n2) return;
    double s = 0.0;
    for (int gph = 0; gph < groups; ++gph) s += fpriv[(int64_t)gph * n2 + x];
    fsum[x] = s;
}

__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src, int64_t m, double *__restrict__ dst)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) dst[x] = src[x];
}

__global__ __launch_bounds__(256) void k_fill(double *__restrict__ p, int64_t m, double v)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) p[x] = v;
}

// F_kl += sum over the copies of the ket-side Coulomb vector (each t is a distinct pair).
__global__ __launch_bounds__(256) void k_jcol_scatter(const DevHeader *__restrict__ hdr,
                                                      const double *__restrict__ jcol, int groups,
                                                      int64_t pcap, const int *__restrict__ pk,
                                                      const int *__restrict__ pl, int n,
                                                      double *__restrict__ fsum)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= hdr->sig_pairs) return;
    double s = 0.0;
    for (int gph = 0; gph < groups; ++gph) s += jcol[(int64_t)gph * pcap + t];
    fsum[(int64_t)pk[t] * n + pl[t]] += s;
}

// G = (F + F^T)/2 and per-block partial sums of D o G.
__global__ __launch_bounds__(256) void k_symmetrise(const double *__restrict__ fsum,
                                                    const double *__restrict__ dens, int n,
                                                    double *__restrict__ fock, double *__restrict__ part)
{
    __shared__ double red[256];
    const int64_t n2 = (int64_t)n * n;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (x < n2) {
        const int64_t i = x / n, j = x % n;
        const double gv = 0.5 * (fsum[x] + fsum[j * n + i]);
        fock[x] = gv;
        e = dens[x] * gv;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// E2 = 1/2 sum of the partials (one block, fixed order).
__global__ __launch_bounds__(256) void k_energy(const double *__restrict__ part, int nb, double scale,
                                                double *__restrict__ e2)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *e2 = scale * red[0];
}

template <int G, typename R>
static hipError_t launch_fock_t(const FockArgs &a, int groups, int variant, bool atoms, hipStream_t st)
{
    // the direct form keeps a bra's primitive data in LDS slots sized for g <= 4; per-atom
    // bases and the deterministic strategy run the hybrid form only
    const bool det = a.strategy == HFK_STRATEGY_DETERMINISTIC;
    const bool split = G > 4 || variant != 0 || atoms || det;
    const size_t smem = FockSmem<R>::total(a.n, split, det);
    const hipError_t ez = launch_zero_counter(a.next_block, st);
    if (ez != hipSuccess) return ez;
    profile_begin(st);
    if (det) {
        if (atoms)
            hipLaunchKernelGGL((k_fock<G, R, true, true, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
        else
            hipLaunchKernelGGL((k_fock<G, R, true, false, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    } else if (atoms) {
        hipLaunchKernelGGL((k_fock<G, R, true, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    } else if constexpr (G > 4) {
        hipLaunchKernelGGL((k_fock<G, R, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    } else {
        if (split)
            hipLaunchKernelGGL((k_fock<G, R, true>), dim3(groups), dim3(kGroupThreads), smem, st, a);
        else
            hipLaunchKernelGGL((k_fock<G, R, false>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    }
    profile_end(st);
    return hipGetLastError();
}

template <int G, typename R>
static int resident_t(bool split, size_t smem, bool atoms, bool det)
{
    int nb = 0;
    hipError_t e;
    if (det) {
        e = atoms ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, true, true, true>, kGroupThreads,
                                                                 smem)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, true, false, true>, kGroupThreads,
                                                                 smem);
    } else if (atoms) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, true, true>, kGroupThreads, smem);
    } else if constexpr (G > 4) {
        (void)split;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, true>, kGroupThreads, smem);
    } else {
        e = split ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, true>, kGroupThreads, smem)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fock<G, R, false>, kGroupThreads, smem);
    }
    return e == hipSuccess ? nb : 0;
}

// Workgroups of the quartet kernel that fit on one CU at once (registers and LDS); 0 if
// the runtime cannot tell.  Persistent workgroups beyond this would only queue.
int fock_resident_groups(int g, int prec, int variant, int64_t n, bool atoms, bool det)
{
    const bool split = variant != 0 || atoms || det;
    const size_t smem = prec == HFK_MIXED ? FockSmem<float>::total((int)n, split, det)
                                          : FockSmem<double>::total((int)n, split, det);
    if (prec == HFK_MIXED) {
        switch (g) {
        case 1: return resident_t<1, float>(split, smem, atoms, det);
        case 2: return resident_t<2, float>(split, smem, atoms, det);
        case 3: return resident_t<3, float>(split, smem, atoms, det);
        case 4: return resident_t<4, float>(split, smem, atoms, det);
        case 5: return resident_t<5, float>(true, smem, atoms, det);
        default: return resident_t<6, float>(true, smem, atoms, det);
        }
    }
    switch (g) {
    case 1: return resident_t<1, double>(split, smem, atoms, det);
    case 2: return resident_t<2, double>(split, smem, atoms, det);
    case 3: return resident_t<3, double>(split, smem, atoms, det);
    case 4: return resident_t<4, double>(split, smem, atoms, det);
    case 5: return resident_t<5, double>(true, smem, atoms, det);
    default: return resident_t<6, double>(true, smem, atoms, det);
    }
}

size_t fock_smem_bytes(int64_t n, int prec, int variant)
{
    return prec == HFK_MIXED ? FockSmem<float>::total((int)n, variant != 0)
                             : FockSmem<double>::total((int)n, variant != 0);
}

hipError_t launch_fock(const Layout &L, const Basis &b, char *ws, const double *dens, double tau, int prec,
                       int strategy, int variant, double *fock, double *e2, hipStream_t st)
{
    DevHeader *hdr = (DevHeader *)(ws + L.hdr);
    FockArgs a;
    a.hdr = hdr;
    a.bd = (const BasisDev *)(ws + L.basis);
    a.boys = (const double *)(ws + L.boys);
    a.boys_f = (const double *)(ws + L.boys_f);
    a.pk = (const int *)(ws + L.pk);
    a.pl = (const int *)(ws + L.pl);
    a.pq = (const double *)(ws + L.pq);
    a.pd = (const double *)(ws + L.pd);
    a.prim = (const double *)(ws + L.prim);
    a.prim_f = (const float *)(ws + L.prim_f);
    a.bra = (const double *)(ws + L.bra);
    a.bra_f = (const float *)(ws + L.bra_f);
    a.bip = L.atoms ? (const double *)(ws + L.bip) : nullptr;
    a.bip_f = L.atoms ? (const float *)(ws + L.bip_f) : nullptr;
    a.item_off = (const long long *)(ws + L.item_off);
    a.lim = (const int *)(ws + L.lim);
    a.goff = (const long long *)(ws + L.goff);
    a.ngroups = L.ngroups;
    a.gshift = L.gshift;
    a.tile = L.tile;
    a.dens = dens;
    a.fpriv = (double *)(ws + L.fpriv);
    a.jcol = (double *)(ws + L.jcol);
    a.quartets = &hdr->quartets;
    a.next_block = &hdr->next_block;
    a.pcap = L.pcap;
    a.tau = tau;
    a.n = (int)L.n;
    a.strategy = strategy;
    a.jcopies = effective_copies(L);
    if (a.jcopies < L.groups) {
        // shared ket vectors are cleared before the launch (workgroups clear private ones)
        const int64_t nj = (int64_t)a.jcopies * L.pcap;
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((nj + 255) / 256)), dim3(256), 0, st, a.jcol, nj, 0.0);
    }
    const int64_t n2 = L.n * L.n;
    const unsigned nb2 = (unsigned)((n2 + 255) / 256);
    if (strategy == HFK_STRATEGY_ATOMIC)
        hipLaunchKernelGGL(k_fill, dim3(nb2), dim3(256), 0, st, a.fpriv, n2, 0.0);
    hipError_t err = hipSuccess;
    const int g = b.g;
    const bool at = L.atoms;
    if (prec == HFK_MIXED) {
        switch (g) {
        case 1: err = launch_fock_t<1, float>(a, L.groups, variant, at, st); break;
        case 2: err = launch_fock_t<2, float>(a, L.groups, variant, at, st); break;
        case 3: err = launch_fock_t<3, float>(a, L.groups, variant, at, st); break;
        case 4: err = launch_fock_t<4, float>(a, L.groups, variant, at, st); break;
        case 5: err = launch_fock_t<5, float>(a, L.groups, 1, at, st); break;
        default: err = launch_fock_t<6, float>(a, L.groups, 1, at, st); break;
        }
    } else {
        switch (g) {
        case 1: err = launch_fock_t<1, double>(a, L.groups, variant, at, st); break;
        case 2: err = launch_fock_t<2, double>(a, L.groups, variant, at, st); break;
        case 3: err = launch_fock_t<3, double>(a, L.groups, variant, at, st); break;
        case 4: err = launch_fock_t<4, double>(a, L.groups, variant, at, st); break;
        case 5: err = launch_fock_t<5, double>(a, L.groups, 1, at, st); break;
        default: err = launch_fock_t<6, double>(a, L.groups, 1, at, st); break;
        }
    }
    if (err != hipSuccess) return err;
    double *fsum = (double *)(ws + L.fsum);
    if (strategy == HFK_STRATEGY_PRIVATE || strategy == HFK_STRATEGY_DETERMINISTIC)
        hipLaunchKernelGGL(k_sum_private, dim3(nb2), dim3(256), 0, st, a.fpriv, L.groups, n2, fsum);
    else
        hipLaunchKernelGGL(k_copy, dim3(nb2), dim3(256), 0, st, a.fpriv, n2, fsum);
    hipLaunchKernelGGL(k_jcol_scatter, dim3((unsigned)((L.pcap + 255) / 256)), dim3(256), 0, st, hdr, a.jcol,
                       a.jcopies, L.pcap, a.pk, a.pl, a.n, fsum);
    double *part = (double *)(ws + L.e2part);
    hipLaunchKernelGGL(k_symmetrise, dim3(nb2), dim3(256), 0, st, fsum, dens, a.n, fock, part);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, part, (int)nb2, 0.5, e2);
    return hipGetLastError();
}

}  // namespace hfk
