// Forward Fock build on one GPU: the unique-quartet loop with the primitive contraction
// and the six-way scatter of the Hartree--Fock kernel (Background section, kernel
// listing), re-designed for CDNA4.
//
// Work decomposition.  Significant pairs are stored in Q-bucketed order (t = 0 .. S-1),
// so the kets kept by the screen for a bra s form a prefix t < lim_s (t <= s keeps each
// unordered quartet once; a lane-level test Q_s Q_t >= tau handles the partial bucket).
// An item is (bra s, 256 consecutive kets); items are numbered bra by bra and every
// persistent workgroup takes one contiguous range of them, so a workgroup stays on one
// bra for many items.  Each of its four waves takes 64 kets of an item, one per lane;
// the bra's primitive data are wave-uniform.
//
// Accumulation (replacing one global FP64 atomic per update):
//   F_ij += 4 D_kl v   per-lane register, reduced across the wave when the bra changes
//   F_kl += 4 D_ij v   coalesced read-modify-write of a per-workgroup vector over kets
//   F_ik, F_il, F_jk, F_jl -= ...   LDS atomics into copies of rows i and j of F, flushed
//                      to a per-workgroup copy of F (or with global atomics) once per bra
// and a final kernel sums the copies, symmetrises and forms E2.
#include "hfk_device.hpp"

namespace hfk {

struct FockArgs {
    const DevHeader *hdr;
    const BasisDev *bd;
    const double *boys;
    const float *boys_f;
    const int *pk;
    const int *pl;
    const double *pq;
    const double *pd;
    const double *prim;
    const float *prim_f;
    const long long *item_off;
    const int *lim;
    const double *dens;
    double *fpriv;
    double *jcol;
    unsigned long long *quartets;
    int64_t pcap;
    double tau;
    int n;
    int strategy;
};

template <typename R> struct Prec;
template <> struct Prec<double> {
    static __device__ const double *prim(const FockArgs &a) { return a.prim; }
    static __device__ const double *boys(const FockArgs &a) { return a.boys; }
    static __device__ const double *rho(const BasisDev *bd) { return bd->rho; }
    static __device__ const double *srho(const BasisDev *bd) { return bd->srho; }
    static __device__ double rsqrt(double x) { return rsqrt_fp64(x); }
};
template <> struct Prec<float> {
    static __device__ const float *prim(const FockArgs &a) { return a.prim_f; }
    static __device__ const float *boys(const FockArgs &a) { return a.boys_f; }
    static __device__ const float *rho(const BasisDev *bd) { return bd->rho_f; }
    static __device__ const float *srho(const BasisDev *bd) { return bd->srho_f; }
    static __device__ float rsqrt(float x) { return rsqrt_fp32(x); }
};

// H(T) = erf(sqrt T)/sqrt T: Taylor expansion about the nearest grid point below the
// switch, T^(-1/2) above it (both evaluated, one selected: no divergence).
template <typename R>
__device__ inline R boys_h(R T, const R *__restrict__ tab)
{
    const R far = Prec<R>::rsqrt(T > R(1e-30) ? T : R(1e-30));
    const R Tc = T < R(kTswitch + 0.5) ? T : R(kTswitch + 0.5);
    const int k = (int)(Tc * R(kBoysInvH) + R(0.5));
    const R d = T - (R)k * R(kBoysH);
    const R *c = tab + k * kBoysStride;
    R v = c[6];
    v = v * d + c[5];
    v = v * d + c[4];
    v = v * d + c[3];
    v = v * d + c[2];
    v = v * d + c[1];
    v = v * d + c[0];
    return T < R(kTswitch) ? v : far;
}

// Contracted (bra | ket) for one lane: bra primitives are wave-uniform (LDS), the ket's
// are the lane's own.  (ab|cd) = S_ab S_cd sqrt(rho) H(rho |P - Q|^2).
template <int G, typename R>
__device__ inline R quartet_eri(const R *__restrict__ bx, const R *__restrict__ by,
                                const R *__restrict__ bz, const R *__restrict__ bs,
                                const R (&kx)[G * G], const R (&ky)[G * G], const R (&kz)[G * G],
                                const R (&ks)[G * G], const R *__restrict__ rho,
                                const R *__restrict__ srho, const R *__restrict__ tab)
{
    constexpr int G2 = G * G;
    R eri = R(0);
#pragma unroll
    for (int ab = 0; ab < G2; ++ab) {
        const R px = bx[ab], py = by[ab], pz = bz[ab];
        R acc = R(0);
#pragma unroll
        for (int cd = 0; cd < G2; ++cd) {
            const R dx = px - kx[cd], dy = py - ky[cd], dz = pz - kz[cd];
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R T = r2 * rho[ab * G2 + cd];
            const R h = boys_h<R>(T, tab);
            acc += (ks[cd] * srho[ab * G2 + cd]) * h;
        }
        eri += bs[ab] * acc;
    }
    return eri;
}

template <int G, typename R>
__global__ __launch_bounds__(kGroupThreads) void k_fock(FockArgs a)
{
    constexpr int G2 = G * G;
    extern __shared__ double smem[];
    const int n = a.n;
    double *rowi = smem;
    double *rowj = smem + n;
    R *tab = (R *)(smem + 2 * n);
    __shared__ R bra_p[4][G2];
    __shared__ int bra_at[2];
    __shared__ double bra_qd[2];

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int gid = blockIdx.x, ng = gridDim.x;
    const long long M = a.hdr->items;
    const int S = a.hdr->sig_pairs;
    const long long m0 = M * gid / ng, m1 = M * (gid + 1) / ng;
    const BasisDev *bd = a.bd;

    const R *gtab = Prec<R>::boys(a);
    for (int x = tid; x < kBoysGrid * kBoysStride; x += kGroupThreads) tab[x] = gtab[x];
    double *jcol = a.jcol + (int64_t)gid * a.pcap;
    double *fp = a.strategy == HFK_STRATEGY_PRIVATE ? a.fpriv + (int64_t)gid * n * n : a.fpriv;
    if (a.strategy == HFK_STRATEGY_PRIVATE) {
        for (int64_t x = tid; x < (int64_t)n * n; x += kGroupThreads) fp[x] = 0.0;
    }
    for (int64_t x = tid; x < S; x += kGroupThreads) jcol[x] = 0.0;
    __syncthreads();
    if (m0 >= m1) return;

    // bra of the first item: the last s with item_off[s] <= m0
    int s;
    {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.item_off[mid] <= m0) lo = mid; else hi = mid - 1;
        }
        s = lo;
    }
    const R *prim = Prec<R>::prim(a);
    const R *rho = Prec<R>::rho(bd);
    const R *srho = Prec<R>::srho(bd);
    int cur = -1, bi = 0, bj = 0;
    double qs = 0.0, ds = 0.0, jb = 0.0;
    unsigned long long kept = 0;
    int lim = 0;

    for (long long m = m0; m <= m1; ++m) {
        if (m < m1) {
            while (a.item_off[s + 1] <= m) ++s;
        }
        if (m == m1 || s != cur) {
            if (cur >= 0) {
                // flush the finished bra: F_ij from the wave partial sums, then rows i, j
                const double w = wave_sum(jb);
                if (lane == 0 && w != 0.0) atomicAdd(&rowi[bj], 4.0 * w);
                jb = 0.0;
                __syncthreads();
                if (a.strategy == HFK_STRATEGY_PRIVATE) {
                    double *fi = fp + (int64_t)bi * n, *fj = fp + (int64_t)bj * n;
                    if (bi == bj) {
                        for (int c = tid; c < n; c += kGroupThreads) fi[c] += rowi[c] + rowj[c];
                    } else {
                        for (int c = tid; c < n; c += kGroupThreads) {
                            fi[c] += rowi[c];
                            fj[c] += rowj[c];
                        }
                    }
                } else {
                    double *fi = fp + (int64_t)bi * n, *fj = fp + (int64_t)bj * n;
                    for (int c = tid; c < n; c += kGroupThreads) {
                        const double vi = rowi[c], vj = rowj[c];
                        if (vi != 0.0) atomicAdd(&fi[c], vi);
                        if (vj != 0.0) atomicAdd(&fj[c], vj);
                    }
                }
                __syncthreads();
            }
            if (m == m1) break;
            // load the new bra
            if (tid < 4 * G2) {
                const int c = tid / G2, ab = tid % G2;
                bra_p[c][ab] = prim[(int64_t)(c * G2 + ab) * a.pcap + s];
            }
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
        const long long t0 = (m - a.item_off[s]) * kKetsPerItem + (long long)wave * kWave;
        if (t0 >= lim) continue;
        const long long t = t0 + lane;   // < S + 64 <= pcap: padded tables
        const bool in = t < lim;
        const double qt = a.pq[t];
        const bool valid = in && (qs * qt >= a.tau);
        R kx[G2], ky[G2], kz[G2], ks[G2];
#pragma unroll
        for (int cd = 0; cd < G2; ++cd) {
            kx[cd] = prim[(int64_t)(0 * G2 + cd) * a.pcap + t];
            ky[cd] = prim[(int64_t)(1 * G2 + cd) * a.pcap + t];
            kz[cd] = prim[(int64_t)(2 * G2 + cd) * a.pcap + t];
            ks[cd] = prim[(int64_t)(3 * G2 + cd) * a.pcap + t];
        }
        const R eri = quartet_eri<G, R>(bra_p[0], bra_p[1], bra_p[2], bra_p[3], kx, ky, kz, ks, rho, srho, tab);
        const int k = a.pk[t], l = a.pl[t];
        double deg = 1.0;
        if (bi == bj) deg *= 0.5;
        if (k == l) deg *= 0.5;
        if (t == s) deg *= 0.5;
        const double v = valid ? (double)eri * deg : 0.0;
        jb = fma(a.pd[t], v, jb);
        if (valid) {
            ++kept;
            jcol[t] += 4.0 * ds * v;
            const double *Di = a.dens + (int64_t)bi * n;
            const double *Dj = a.dens + (int64_t)bj * n;
            atomicAdd(&rowi[k], -Dj[l] * v);
            atomicAdd(&rowi[l], -Dj[k] * v);
            atomicAdd(&rowj[k], -Di[l] * v);
            atomicAdd(&rowj[l], -Di[k] * v);
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

// F_kl += sum over workgroups of the ket-side Coulomb vector (each t is a distinct pair).
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
static hipError_t launch_fock_t(const FockArgs &a, int groups, size_t smem, hipStream_t st)
{
    profile_begin(st);
    hipLaunchKernelGGL((k_fock<G, R>), dim3(groups), dim3(kGroupThreads), smem, st, a);
    profile_end(st);
    return hipGetLastError();
}

hipError_t launch_fock(const Layout &L, const Basis &b, char *ws, const double *dens, double tau, int prec,
                       int strategy, double *fock, double *e2, hipStream_t st)
{
    DevHeader *hdr = (DevHeader *)(ws + L.hdr);
    FockArgs a;
    a.hdr = hdr;
    a.bd = (const BasisDev *)(ws + L.basis);
    a.boys = (const double *)(ws + L.boys);
    a.boys_f = (const float *)(ws + L.boys_f);
    a.pk = (const int *)(ws + L.pk);
    a.pl = (const int *)(ws + L.pl);
    a.pq = (const double *)(ws + L.pq);
    a.pd = (const double *)(ws + L.pd);
    a.prim = (const double *)(ws + L.prim);
    a.prim_f = (const float *)(ws + L.prim_f);
    a.item_off = (const long long *)(ws + L.item_off);
    a.lim = (const int *)(ws + L.lim);
    a.dens = dens;
    a.fpriv = (double *)(ws + L.fpriv);
    a.jcol = (double *)(ws + L.jcol);
    a.quartets = &hdr->quartets;
    a.pcap = L.pcap;
    a.tau = tau;
    a.n = (int)L.n;
    a.strategy = strategy;
    const int64_t n2 = L.n * L.n;
    const unsigned nb2 = (unsigned)((n2 + 255) / 256);
    if (strategy == HFK_STRATEGY_ATOMIC)
        hipLaunchKernelGGL(k_fill, dim3(nb2), dim3(256), 0, st, a.fpriv, n2, 0.0);
    const size_t smem = (size_t)(2 * L.n) * sizeof(double) +
                        (size_t)kBoysGrid * kBoysStride * (prec == HFK_MIXED ? sizeof(float) : sizeof(double));
    hipError_t err = hipSuccess;
    const int g = b.g;
    if (prec == HFK_MIXED) {
        switch (g) {
        case 1: err = launch_fock_t<1, float>(a, L.groups, smem, st); break;
        case 2: err = launch_fock_t<2, float>(a, L.groups, smem, st); break;
        case 3: err = launch_fock_t<3, float>(a, L.groups, smem, st); break;
        default: err = launch_fock_t<4, float>(a, L.groups, smem, st); break;
        }
    } else {
        switch (g) {
        case 1: err = launch_fock_t<1, double>(a, L.groups, smem, st); break;
        case 2: err = launch_fock_t<2, double>(a, L.groups, smem, st); break;
        case 3: err = launch_fock_t<3, double>(a, L.groups, smem, st); break;
        default: err = launch_fock_t<4, double>(a, L.groups, smem, st); break;
        }
    }
    if (err != hipSuccess) return err;
    double *fsum = (double *)(ws + L.fsum);
    if (strategy == HFK_STRATEGY_PRIVATE)
        hipLaunchKernelGGL(k_sum_private, dim3(nb2), dim3(256), 0, st, a.fpriv, L.groups, n2, fsum);
    else
        hipLaunchKernelGGL(k_copy, dim3(nb2), dim3(256), 0, st, a.fpriv, n2, fsum);
    hipLaunchKernelGGL(k_jcol_scatter, dim3((unsigned)((L.pcap + 255) / 256)), dim3(256), 0, st, hdr, a.jcol,
                       L.groups, L.pcap, a.pk, a.pl, a.n, fsum);
    double *part = (double *)(ws + L.e2part);
    hipLaunchKernelGGL(k_symmetrise, dim3(nb2), dim3(256), 0, st, fsum, dens, a.n, fock, part);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, part, (int)nb2, 0.5, e2);
    return hipGetLastError();
}

}  // namespace hfk
