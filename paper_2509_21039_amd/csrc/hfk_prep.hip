// Setup and pair preparation for the Fock build: basis constants, Boys table, Schwarz
// bounds, the Q-bucketed pair order and the work items of the quartet kernel.
#include "hfk_device.hpp"

namespace hfk {

// ------------------------------------------------------------------ setup

// Basis constants per primitive pair and quartet; zeroes the header; centroid of xyz.
__global__ __launch_bounds__(256) void k_setup(Basis b, BasisDev *__restrict__ bd,
                                               DevHeader *__restrict__ hdr, int64_t n,
                                               const double *__restrict__ xyz)
{
    const int t = threadIdx.x;
    const int g = b.g, g2 = b.g2;
    for (int ab = t; ab < g2; ab += blockDim.x) {
        const int a = ab / g, c = ab % g;
        const double p = b.alpha[a] + b.alpha[c];
        bd->p[ab] = p;
        bd->mu[ab] = b.alpha[a] * b.alpha[c] / p;
        bd->fa[ab] = b.alpha[a] / p;
        bd->fb[ab] = b.alpha[c] / p;
        bd->pi32[ab] = pow(kPi / p, 1.5);
    }
    for (int x = t; x < g2 * g2; x += blockDim.x) {
        const int ab = x / g2, cd = x % g2;
        const double p = b.alpha[ab / g] + b.alpha[ab % g];
        const double q = b.alpha[cd / g] + b.alpha[cd % g];
        const double rho = p * q / (p + q);
        bd->rho[x] = rho;
        bd->srho[x] = sqrt(rho);
        bd->r2sw[x] = kTswitch / rho;
        bd->rho_f[x] = (float)rho;
        bd->rs[3 * x] = rho;
        bd->rs[3 * x + 1] = sqrt(rho);
        bd->rs[3 * x + 2] = kTswitch / rho;
        bd->rs_f[3 * x] = (float)rho;
        bd->rs_f[3 * x + 1] = (float)sqrt(rho);
        bd->rs_f[3 * x + 2] = (float)(kTswitch / rho);
        bd->rsn[3 * x] = kTswitch / rho;
        bd->rsn[3 * x + 1] = rho * kBoysInvH;
        bd->rsn[3 * x + 2] = sqrt(rho * kBoysInvH);
        bd->rsn_f[3 * x] = (float)(kTswitch / rho);
        bd->rsn_f[3 * x + 1] = (float)(rho * kBoysInvHF);
        bd->rsn_f[3 * x + 2] = (float)sqrt(rho * kBoysInvHF);
        {
            const double r = rho * kBoysInvH, sr = sqrt(r);
            bd->rsg[4 * x] = kTswitch / rho;
            bd->rsg[4 * x + 1] = r;
            bd->rsg[4 * x + 2] = sr;
            bd->rsg[4 * x + 3] = r * sr;
            const double rf = rho * kBoysInvHF, srf = sqrt(rf);
            bd->rsg_f[4 * x] = (float)(kTswitch / rho);
            bd->rsg_f[4 * x + 1] = (float)rf;
            bd->rsg_f[4 * x + 2] = (float)srf;
            bd->rsg_f[4 * x + 3] = (float)(rf * srf);
        }
        bd->srho_f[x] = (float)sqrt(rho);
        bd->r2sw_f[x] = (float)(kTswitch / rho);
    }
    // centroid and bounding box (block reductions, one block)
    __shared__ double red[3][256], rmin[3][256], rmax[3][256];
    double s0 = 0, s1 = 0, s2 = 0;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = t; i < n; i += blockDim.x) {
        s0 += xyz[3 * i];
        s1 += xyz[3 * i + 1];
        s2 += xyz[3 * i + 2];
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], xyz[3 * i + c]);
            hi[c] = fmax(hi[c], xyz[3 * i + c]);
        }
    }
    red[0][t] = s0; red[1][t] = s1; red[2][t] = s2;
    for (int c = 0; c < 3; ++c) {
        rmin[c][t] = lo[c];
        rmax[c][t] = hi[c];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int c = 0; c < 3; ++c) {
                red[c][t] += red[c][t + w];
                rmin[c][t] = fmin(rmin[c][t], rmin[c][t + w]);
                rmax[c][t] = fmax(rmax[c][t], rmax[c][t + w]);
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int c = 0; c < 3; ++c) {
            hdr->bmin[c] = rmin[c][0];
            hdr->bmax[c] = rmax[c][0];
        }
        hdr->qmax_bits = 0;
        hdr->sig_pairs = 0;
        hdr->items = 0;
        hdr->quartets = 0;
        hdr->max_bucket = 0;
        hdr->centroid[0] = red[0][0] / (double)n;
        hdr->centroid[1] = red[1][0] / (double)n;
        hdr->centroid[2] = red[2][0] / (double)n;
        hdr->natoms = (int)n;
    }
}

// Boys tables.  Row k of `tg` holds (2/sqrt(pi)) (-1)^m F_m(k h) / m!, m = 0..7 (Taylor
// coefficients of H(T) = erf(sqrt T)/sqrt T about T_k, rows of kBoysStrideG: the FP64 gradient
// kernels take g(T) = -(4/sqrt(pi)) F1(T) = 2 H'(T) from its derivative); row k of `tab` is its
// degree-5 Chebyshev economisation on [T_k - h/2, T_k + h/2] (the forward kernels' rows).  On
// the FP32 grid (spacing kBoysHF, kBoysOrderF coefficients, still in FP64) `tab_f` holds H's
// Taylor rows and `tg_f` g's, -(4/sqrt(pi)) (-1)^m F_{m+1}(k h) / m!.  The highest order
// comes from its positive Kummer series (no cancellation), the lower ones from the downward
// recursion F_m = (2T F_{m+1} + e^-T) / (2m + 1), which is stable in that direction (one
// series per row instead of one per order: each term of a series is a division).
__device__ inline void boys_rows(double T, int order, int stride, double *v, double *w)
{
    double fm[kBoysOrderG + 1];
    const double et = exp(-T);
    {
        const int m = order;
        double term = 1.0 / (2.0 * m + 1.0), sum = term;
        for (int i = 1; i < 400; ++i) {
            term *= 2.0 * T / (2.0 * m + 2.0 * i + 1.0);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        fm[m] = et * sum;
    }
    for (int m = order - 1; m >= 0; --m) fm[m] = (2.0 * T * fm[m + 1] + et) / (2.0 * m + 1.0);
    double fact = 1.0;
    for (int m = 0; m < stride; ++m) {
        v[m] = 0.0;
        if (w) w[m] = 0.0;
        if (m < order) {
            if (m > 0) fact *= (double)m;
            const double sgn = (m & 1) ? -1.0 : 1.0;
            v[m] = kTwoOverSqrtPi * sgn * fm[m] / fact;
            if (w) w[m] = -2.0 * kTwoOverSqrtPi * sgn * fm[m + 1] / fact;
        }
    }
}

__global__ void k_boys_table(double *__restrict__ tab, double *__restrict__ tab_f, double *__restrict__ tg,
                             double *__restrict__ tg_f)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kBoysGrid) {
        double *t7 = tg + k * kBoysStrideG;
        boys_rows(k * kBoysH, kBoysOrderG, kBoysStrideG, t7, nullptr);
        // economise to degree 5 in u = (T - T_k) / r, r = h/2 (b_m = c_m r^m): drop T7(u)/64
        // and T6(u)/32 from the expansion, keeping the lower-degree parts of u^7 and u^6
        //   u^7 = (T7 + 112 u^5 - 56 u^3 + 7 u) / 64,   u^6 = (T6 + 48 u^4 - 18 u^2 + 1) / 32
        static_assert(kBoysOrder == 6 && kBoysOrderG == 8, "degree-7 rows economised to degree 5");
        const double r = 0.5 * kBoysH;
        double b[8], rm = 1.0;
        for (int m = 0; m < 8; ++m) {
            b[m] = t7[m] * rm;
            rm *= r;
        }
        b[5] += b[7] * (112.0 / 64.0);
        b[3] -= b[7] * (56.0 / 64.0);
        b[1] += b[7] * (7.0 / 64.0);
        b[4] += b[6] * (48.0 / 32.0);
        b[2] -= b[6] * (18.0 / 32.0);
        b[0] += b[6] * (1.0 / 32.0);
        rm = 1.0;
        for (int m = 0; m < kBoysStride; ++m) {
            tab[k * kBoysStride + m] = b[m] / rm;
            rm *= r;
        }
    }
    if (k < kBoysGridF)
        boys_rows(k * kBoysHF, kBoysOrderF, kBoysStrideF, tab_f + k * kBoysStrideF, tg_f + k * kBoysStrideF);
}

hipError_t launch_setup(const Basis &b, BasisDev *bd, double *boys, double *boys_f, double *boys_g,
                        double *boys_g_f, DevHeader *hdr, int64_t n, const double *xyz, hipStream_t st)
{
    static_assert(kBoysGridF >= kBoysGrid, "one thread per row of the longer table");
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, b, bd, hdr, n, xyz);
    hipLaunchKernelGGL(k_boys_table, dim3((kBoysGridF + 63) / 64), dim3(64), 0, st, boys, boys_f, boys_g,
                       boys_g_f);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pairs

// Schwarz bound of every pair i >= j: Q_ij = sqrt((ij|ij)) in FP64, each primitive
// quartet as S_ab S_cd sqrt(rho) H(rho |P-Q|^2) with H(T) = erf(sqrt T)/sqrt T.
__global__ __launch_bounds__(256) void k_pair_q(Basis b, const BasisDev *__restrict__ bd,
                                                DevHeader *__restrict__ hdr, int64_t n,
                                                const double *__restrict__ xyz,
                                                double *__restrict__ qout)
{
    const int64_t npair = n * (n + 1) / 2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double q = 0.0;
    if (p < npair) {
        int64_t i, j;
        pair_of_index(p, i, j);
        const double c0 = hdr->centroid[0], c1 = hdr->centroid[1], c2 = hdr->centroid[2];
        double A[3] = {xyz[3 * i] - c0, xyz[3 * i + 1] - c1, xyz[3 * i + 2] - c2};
        double B[3] = {xyz[3 * j] - c0, xyz[3 * j + 1] - c1, xyz[3 * j + 2] - c2};
        double px[kMaxG2], py[kMaxG2], pz[kMaxG2], ps[kMaxG2], pp[kMaxG2];
        double s = 0.0;
        if (b.aexp) {
            // per-atom bases: rho of every primitive quartet from the pair exponents
            pair_prims_atoms(b, i, j, A, B, px, py, pz, ps, pp);
            for (int ab = 0; ab < b.g2; ++ab)
                for (int cd = 0; cd < b.g2; ++cd) {
                    const double dx = px[ab] - px[cd], dy = py[ab] - py[cd], dz = pz[ab] - pz[cd];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double rho = pp[ab] * pp[cd] / (pp[ab] + pp[cd]);
                    s += ps[ab] * ps[cd] * sqrt(rho) * erf_over_sqrt(rho * r2);
                }
        } else {
            pair_prims(b, bd, A, B, px, py, pz, ps);
            for (int ab = 0; ab < b.g2; ++ab)
                for (int cd = 0; cd < b.g2; ++cd) {
                    const double dx = px[ab] - px[cd], dy = py[ab] - py[cd], dz = pz[ab] - pz[cd];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    s += ps[ab] * ps[cd] * bd->srho[ab * b.g2 + cd] * erf_over_sqrt(bd->rho[ab * b.g2 + cd] * r2);
                }
        }
        q = sqrt(s);
        qout[p] = q;
    }
    // block max, then one atomic per block (positive doubles order like their bit patterns)
    __shared__ double red[256];
    red[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&hdr->qmax_bits, (unsigned long long)__double_as_longlong(red[0]));
}

// Morton index of the cell holding point c inside the bounding box.
__device__ inline int morton_cell(const double *c, const DevHeader *__restrict__ hdr)
{
    constexpr int side = 1 << kCellBits;
    int code = 0;
    for (int d = 0; d < 3; ++d) {
        const double ext = hdr->bmax[d] - hdr->bmin[d];
        int u = ext > 0.0 ? (int)((c[d] - hdr->bmin[d]) / ext * side) : 0;
        u = u < 0 ? 0 : (u >= side ? side - 1 : u);
        for (int b = 0; b < kCellBits; ++b) code |= ((u >> b) & 1) << (3 * b + d);
    }
    return code;
}

__global__ __launch_bounds__(256) void k_bucket_count(int64_t n, double tau, const DevHeader *__restrict__ hdr,
                                                      const double *__restrict__ xyz,
                                                      const double *__restrict__ q, int *__restrict__ bucket_of,
                                                      long long *__restrict__ cnt)
{
    const int64_t npair = n * (n + 1) / 2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    const double qmax = __longlong_as_double((long long)hdr->qmax_bits);
    const double qp = q[p];
    int b = -1;
    if (qp * qmax >= tau && qp > 0.0) {
        int64_t i, j;
        pair_of_index(p, i, j);
        const double c[3] = {0.5 * (xyz[3 * i] + xyz[3 * j]), 0.5 * (xyz[3 * i + 1] + xyz[3 * j + 1]),
                             0.5 * (xyz[3 * i + 2] + xyz[3 * j + 2])};
        b = q_band(qp) * kNumCells + morton_cell(c, hdr);
        atomicAdd((unsigned long long *)&cnt[b], 1ULL);
    }
    bucket_of[p] = b;
}

// Bucket offsets -> cursors (int) and the significant-pair total.
__global__ __launch_bounds__(256) void k_bucket_cursors(const long long *__restrict__ off, int *__restrict__ cur,
                                                        DevHeader *__restrict__ hdr)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < kNumBuckets) cur[b] = (int)off[b];
    if (b == 0) hdr->sig_pairs = (int)off[kNumBuckets];
}

// Writes every significant pair at its bucketed position: atoms, Q, D_kl and the SoA
// primitive-pair table {Px, Py, Pz, S} (FP64 and FP32), centred on the centroid.  With
// per-atom bases (bip != NULL) the ket tables gain kTswitch / p as their last component
// (FP64 component 5, FP32 component 4) and bip/bip_f receive it per bra primitive pair:
// the two add up to kTswitch / rho of the quartet.
__global__ __launch_bounds__(256) void k_pair_scatter(Basis b, const BasisDev *__restrict__ bd,
                                                      const DevHeader *__restrict__ hdr, int64_t n,
                                                      int64_t pcap, const double *__restrict__ xyz,
                                                      const double *__restrict__ dens,
                                                      const double *__restrict__ q,
                                                      const int *__restrict__ bucket_of,
                                                      int *__restrict__ cur, int *__restrict__ pk,
                                                      int *__restrict__ pl, double *__restrict__ pq,
                                                      double *__restrict__ pd, double *__restrict__ prim,
                                                      float *__restrict__ prim_f, double *__restrict__ bra,
                                                      float *__restrict__ bra_f, double *__restrict__ bip,
                                                      float *__restrict__ bip_f, double *__restrict__ kmu,
                                                      double *__restrict__ kfa, double *__restrict__ bgw,
                                                      float *__restrict__ bgw_f,
                                                      const int *__restrict__ slot)
{
    const int64_t npair = n * (n + 1) / 2;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p;
    int pos;
    if (slot) {
        // fixed order: thread x writes position x, holding pair slot[x]
        if (x >= hdr->sig_pairs) return;
        pos = (int)x;
        p = slot[x];
    } else {
        // order within a bucket as the atomic cursor hands out places
        p = x;
        if (p >= npair) return;
        const int bk = bucket_of[p];
        if (bk < 0) return;
        pos = atomicAdd(&cur[bk], 1);
    }
    int64_t i, j;
    pair_of_index(p, i, j);
    const double c0 = hdr->centroid[0], c1 = hdr->centroid[1], c2 = hdr->centroid[2];
    double A[3] = {xyz[3 * i] - c0, xyz[3 * i + 1] - c1, xyz[3 * i + 2] - c2};
    double B[3] = {xyz[3 * j] - c0, xyz[3 * j + 1] - c1, xyz[3 * j + 2] - c2};
    double px[kMaxG2], py[kMaxG2], pz[kMaxG2], ps[kMaxG2], pp[kMaxG2], mu[kMaxG2], fa[kMaxG2];
    if (b.aexp)
        pair_prims_atoms(b, i, j, A, B, px, py, pz, ps, pp, mu, fa);
    else
        pair_prims(b, bd, A, B, px, py, pz, ps);
    pk[pos] = (int)i;
    pl[pos] = (int)j;
    pq[pos] = q[p];
    pd[pos] = dens[i * n + j];
    const int g2 = b.g2;
    for (int ab = 0; ab < g2; ++ab) {
        prim[(0 * g2 + ab) * pcap + pos] = px[ab];
        prim[(1 * g2 + ab) * pcap + pos] = py[ab];
        prim[(2 * g2 + ab) * pcap + pos] = pz[ab];
        prim[(3 * g2 + ab) * pcap + pos] = ps[ab];
        prim[(4 * g2 + ab) * pcap + pos] = px[ab] * px[ab] + py[ab] * py[ab] + pz[ab] * pz[ab];
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
        bf[4] = (float)(-2.0 * px[ab]); bf[5] = (float)(-2.0 * py[ab]); bf[6] = (float)(-2.0 * pz[ab]);
        bf[7] = (float)p2;
    }
    if (bip) {
        for (int ab = 0; ab < g2; ++ab) {
            const double ip = kTswitch / pp[ab];
            prim[(5 * g2 + ab) * pcap + pos] = ip;
            prim_f[(4 * g2 + ab) * pcap + pos] = (float)ip;
            bip[(int64_t)pos * g2 + ab] = ip;
            bip_f[(int64_t)pos * g2 + ab] = (float)ip;
        }
    }
    if (kmu) {
        // per-atom gradient: mu and a/p of every ket primitive pair
        for (int ab = 0; ab < g2; ++ab) {
            kmu[(int64_t)ab * pcap + pos] = mu[ab];
            kfa[(int64_t)ab * pcap + pos] = fa[ab];
        }
    }
    if (bgw) {
        // gradient: the bra weights mu S, fa S, fb S, fa fb S, fb^2 S of every primitive pair
        for (int ab = 0; ab < g2; ++ab) {
            const double m_ab = b.aexp ? mu[ab] : bd->mu[ab];
            const double fa_ab = b.aexp ? fa[ab] : bd->fa[ab];
            const double fb_ab = b.aexp ? 1.0 - fa[ab] : bd->fb[ab];
            const double row[kGW] = {m_ab * ps[ab], fa_ab * ps[ab], fb_ab * ps[ab], fa_ab * fb_ab * ps[ab],
                                     fb_ab * fb_ab * ps[ab], 0.0, 0.0, 0.0};
            double *w = bgw + ((int64_t)pos * g2 + ab) * kGW;
            float *wf = bgw_f + ((int64_t)pos * g2 + ab) * kGW;
            for (int c = 0; c < kGW; ++c) {
                w[c] = row[c];
                wf[c] = (float)row[c];
            }
        }
    }
}

// Fixed pair order (deterministic strategy): every significant pair's index into its
// bucket's range (in any order), then each bucket's range sorted by pair index, so the
// bucketed order is a function of the inputs alone.
__global__ __launch_bounds__(256) void k_slot_fill(int64_t npair, const int *__restrict__ bucket_of,
                                                   int *__restrict__ cur, int *__restrict__ slot)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    const int bk = bucket_of[p];
    if (bk >= 0) slot[atomicAdd(&cur[bk], 1)] = (int)p;
}

__global__ __launch_bounds__(256) void k_bucket_max(const long long *__restrict__ off, DevHeader *__restrict__ hdr)
{
    __shared__ int red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    red[threadIdx.x] = b < kNumBuckets ? (int)(off[b + 1] - off[b]) : 0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&hdr->max_bucket, red[0]);
}

__global__ __launch_bounds__(256) void k_slot_sort(const long long *__restrict__ off, int *__restrict__ slot)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= kNumBuckets) return;
    const long long lo = off[b], hi = off[b + 1];
    // insertion sort of one bucket (buckets hold tens of pairs)
    for (long long x = lo + 1; x < hi; ++x) {
        const int v = slot[x];
        long long y = x - 1;
        while (y >= lo && slot[y] > v) {
            slot[y + 1] = slot[y];
            --y;
        }
        slot[y + 1] = v;
    }
}

// Pads the tail chunk of the sorted tables with harmless entries (atom 0, zero weight,
// centres 1e6 bohr away) so that lanes past the last pair, or lanes pointed at the first
// pad entry, read defined memory and land in the far branch with a zero integral.
// Ket table components: Px Py Pz S always; p2: FP64 component 4 holds |P|^2; swc / swc_f:
// the FP64 / FP32 component holding kTswitch/p of per-atom bases (-1: none), padded with
// 1 so that the switch radius stays far below the pad distance.  kmu/kfa (per-atom
// gradient tables, or NULL) are zeroed there too.
__global__ void k_pair_pad(const DevHeader *__restrict__ hdr, int64_t pcap, int g2, bool p2, int swc, int swc_f,
                           int *__restrict__ pk, int *__restrict__ pl, double *__restrict__ pq,
                           double *__restrict__ pd, double *__restrict__ prim, float *__restrict__ prim_f,
                           double *__restrict__ kmu, double *__restrict__ kfa)
{
    const int64_t s = hdr->sig_pairs;
    const int64_t pos = s + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= pcap) return;
    pk[pos] = 0;
    pl[pos] = 0;
    pq[pos] = 0.0;
    pd[pos] = 0.0;
    for (int ab = 0; ab < g2; ++ab) {
        for (int c = 0; c < 4; ++c) {
            prim[(c * g2 + ab) * pcap + pos] = c < 3 ? 1e6 : 0.0;
            prim_f[(c * g2 + ab) * pcap + pos] = c < 3 ? 1e6f : 0.0f;
        }
        if (p2) prim[(4 * g2 + ab) * pcap + pos] = 3e12;
        if (swc >= 0) prim[((int64_t)swc * g2 + ab) * pcap + pos] = 1.0;
        if (swc_f >= 0) prim_f[((int64_t)swc_f * g2 + ab) * pcap + pos] = 1.0f;
        if (kmu) {
            kmu[(int64_t)ab * pcap + pos] = 0.0;
            kfa[(int64_t)ab * pcap + pos] = 0.0;
        }
    }
}

hipError_t launch_pair_pad(const DevHeader *hdr, int64_t pcap, int g2, bool atoms, int *pk, int *pl, double *pq,
                           double *pd, double *prim, float *prim_f, double *kmu, double *kfa, hipStream_t st)
{
    // the batched tables hold the four-component ket table, plus kTswitch/p as component 4
    // (FP64 and FP32) with per-atom bases
    hipLaunchKernelGGL(k_pair_pad, dim3((unsigned)((pcap + 255) / 256)), dim3(256), 0, st, hdr, pcap, g2, false,
                       atoms ? 4 : -1, atoms ? 4 : -1, pk, pl, pq, pd, prim, prim_f, kmu, kfa);
    return hipGetLastError();
}

// Ket range of every bra s (in bucketed order): kets t < lim_s with
// lim_s = min(s + 1, end of the band holding tau / Q_s); items of kItemKets kets.
__global__ __launch_bounds__(256) void k_limits(const DevHeader *__restrict__ hdr, double tau,
                                                const double *__restrict__ pq,
                                                const long long *__restrict__ boff,
                                                long long *__restrict__ nitems, int *__restrict__ lims,
                                                int64_t pcap)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = hdr->sig_pairs;
    if (s >= pcap) return;
    long long ni = 0;
    if (s < S) {
        const double thr = tau / pq[s];
        int64_t bend;
        if (thr <= 0.0) {
            bend = S;
        } else {
            // band 0 is open-ended (every Q above its lower edge), so a threshold above the
            // largest band edge still lands there; the lane-level test finishes the job
            const int bt = q_band(thr);
            bend = bt + 1 >= kNumBands ? S : boff[(bt + 1) * kNumCells];
        }
        const int64_t lim = bend < s + 1 ? bend : s + 1;
        ni = (lim + kItemKets - 1) / kItemKets;
        lims[s] = (int)lim;
    } else {
        lims[s] = 0;
    }
    nitems[s] = ni;
}

// ------------------------------------------------------------------ exclusive scan (int64)

constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const long long *__restrict__ in, int64_t m,
                                                            long long *__restrict__ bsum)
{
    __shared__ long long red[kScanBlock];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    red[threadIdx.x] = i < m ? in[i] : 0;
    __syncthreads();
    for (int w = kScanBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Exclusive scan of the block sums in one block (nb <= 1024 * 16).
__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(long long *__restrict__ bsum, int nb)
{
    __shared__ long long part[kScanBlock];
    const int t = threadIdx.x;
    const int per = (nb + kScanBlock - 1) / kScanBlock;
    long long s = 0;
    for (int i = 0; i < per; ++i) {
        const int x = t * per + i;
        if (x < nb) s += bsum[x];
    }
    part[t] = s;
    __syncthreads();
    for (int w = 1; w < kScanBlock; w <<= 1) {
        long long v = (t >= w) ? part[t - w] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = part[t] - s;
    for (int i = 0; i < per; ++i) {
        const int x = t * per + i;
        if (x < nb) {
            const long long v = bsum[x];
            bsum[x] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const long long *__restrict__ in, int64_t m,
                                                           const long long *__restrict__ bsum,
                                                           long long *__restrict__ out,
                                                           long long *__restrict__ total)
{
    __shared__ long long part[kScanBlock];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + t;
    const long long v = i < m ? in[i] : 0;
    part[t] = v;
    __syncthreads();
    for (int w = 1; w < kScanBlock; w <<= 1) {
        long long u = (t >= w) ? part[t - w] : 0;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    const long long excl = bsum[blockIdx.x] + part[t] - v;
    if (i < m) out[i] = excl;
    if (i == m - 1) {
        out[m] = excl + v;
        if (total) *total = excl + v;
    }
}

hipError_t launch_scan(const long long *in, int64_t m, long long *out, long long *tmp, long long *total,
                       hipStream_t st)
{
    const int nb = (int)((m + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, st, in, m, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanBlock), 0, st, in, m, tmp, out, total);
    return hipGetLastError();
}

__global__ void k_header_info(DevHeader *hdr, int strategy, int groups, int precision, int variant, int tile,
                              int group_bras, int ket_copies)
{
    hdr->strategy = strategy;
    hdr->groups = groups;
    hdr->precision = precision;
    hdr->variant = variant;
    hdr->tile = tile >= 0 ? tile : (int)hdr->bsz;   // batched: the block size its table used
    hdr->group_bras = group_bras;
    hdr->ket_copies = ket_copies;
}

hipError_t launch_header_info(char *hdr, int strategy, int groups, int precision, int variant, hipStream_t st,
                              int tile, int group_bras, int ket_copies)
{
    hipLaunchKernelGGL(k_header_info, dim3(1), dim3(1), 0, st, (DevHeader *)hdr, strategy, groups, precision,
                       variant, tile, group_bras, ket_copies);
    return hipGetLastError();
}

// ------------------------------------------------------------------ debug check of the density

__global__ void k_dchk_reset(DevHeader *hdr)
{
    hdr->dchk_asym = 0;
    hdr->dchk_max = 0;
    hdr->dchk_ratio = 0;
    hdr->dchk_bad = 0;
    hdr->dchk_mol = 0x7fffffff;
    hdr->dchk_badmol = 0x7fffffff;
}

// Non-negative doubles order like their bit patterns, so atomicMax on the patterns is a max.
__device__ inline void atomic_max_nonneg(unsigned long long *p, double v)
{
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// One matrix, any size: grid-stride over its entries, block maxima, then atomics.
__global__ __launch_bounds__(256) void k_dens_check(int64_t n, const double *__restrict__ D,
                                                    DevHeader *__restrict__ hdr)
{
    __shared__ double ra[256], rm[256];
    __shared__ unsigned long long rb[256];
    double asym = 0.0, mx = 0.0;
    unsigned long long bad = 0;
    const int64_t n2 = n * n;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n2; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x / n, j = x - i * n;
        const double v = D[x];
        if (!isfinite(v)) {
            ++bad;
            continue;
        }
        mx = fmax(mx, fabs(v));
        const double w = D[j * n + i];
        if (isfinite(w)) asym = fmax(asym, fabs(v - w));
    }
    ra[threadIdx.x] = asym;
    rm[threadIdx.x] = mx;
    rb[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ra[threadIdx.x] = fmax(ra[threadIdx.x], ra[threadIdx.x + w]);
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
            rb[threadIdx.x] += rb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomic_max_nonneg(&hdr->dchk_asym, ra[0]);
        atomic_max_nonneg(&hdr->dchk_max, rm[0]);
        if (rb[0]) atomicAdd(&hdr->dchk_bad, rb[0]);
    }
}

// Many small matrices: one block per molecule (grid-stride over molecules), each judged
// against tol times its own largest entry.
__global__ __launch_bounds__(256) void k_dens_check_batched(int64_t nmol, const long long *__restrict__ doff,
                                                            const int *__restrict__ nmv,
                                                            const double *__restrict__ D, double tol,
                                                            DevHeader *__restrict__ hdr)
{
    __shared__ double ra[256], rm[256];
    __shared__ unsigned long long rb[256];
    for (int64_t m = blockIdx.x; m < nmol; m += gridDim.x) {
        const int64_t n = nmv[m];
        const double *Dm = D + doff[m];
        double asym = 0.0, mx = 0.0;
        unsigned long long bad = 0;
        for (int64_t x = threadIdx.x; x < n * n; x += blockDim.x) {
            const int64_t i = x / n, j = x - i * n;
            const double v = Dm[x];
            if (!isfinite(v)) {
                ++bad;
                continue;
            }
            mx = fmax(mx, fabs(v));
            const double w = Dm[j * n + i];
            if (isfinite(w)) asym = fmax(asym, fabs(v - w));
        }
        ra[threadIdx.x] = asym;
        rm[threadIdx.x] = mx;
        rb[threadIdx.x] = bad;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ra[threadIdx.x] = fmax(ra[threadIdx.x], ra[threadIdx.x + w]);
                rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
                rb[threadIdx.x] += rb[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (rb[0]) {
                atomicAdd(&hdr->dchk_bad, rb[0]);
                atomicMin(&hdr->dchk_badmol, (int)m);
            }
            const double a = ra[0], b = rm[0];
            if (a > tol * b) {
                atomicMin(&hdr->dchk_mol, (int)m);
                atomic_max_nonneg(&hdr->dchk_ratio, b > 0.0 ? a / b : a);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_dens_check(DevHeader *hdr, int64_t n, const double *dens, hipStream_t st)
{
    hipLaunchKernelGGL(k_dchk_reset, dim3(1), dim3(1), 0, st, hdr);
    const int64_t nb = (n * n + 255) / 256;
    hipLaunchKernelGGL(k_dens_check, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, st, n, dens, hdr);
    return hipGetLastError();
}

hipError_t launch_dens_check_batched(DevHeader *hdr, int64_t nmol, const long long *mol_doff, const int *mol_n,
                                     const double *dens, double tol, hipStream_t st)
{
    hipLaunchKernelGGL(k_dchk_reset, dim3(1), dim3(1), 0, st, hdr);
    hipLaunchKernelGGL(k_dens_check_batched, dim3((unsigned)(nmol < 4096 ? nmol : 4096)), dim3(256), 0, st, nmol,
                       mol_doff, mol_n, dens, tol, hdr);
    return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long *__restrict__ p)
{
    if (threadIdx.x == 0) *p = 0ULL;
}

// Zeroes a work counter with a kernel (stream-ordered, no memset node).
hipError_t launch_zero_counter(unsigned long long *p, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p);
    return hipGetLastError();
}

__global__ void k_fill_i64(long long *__restrict__ p, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0;
}

// Blocks of every bra group: 2^gshift x the largest block count of its bras (bras with
// fewer blocks leave empty slots, skipped by the kernels).
// One workgroup per group of bras: the largest block count of its bras (a block-wide max).
__global__ __launch_bounds__(256) void k_group_blocks(const DevHeader *__restrict__ hdr,
                                                      const long long *__restrict__ nitems, int64_t ngroups,
                                                      int gshift, int tile, long long *__restrict__ gcnt)
{
    __shared__ long long red[256];
    const int64_t g = blockIdx.x;   // the grid is exactly ngroups workgroups
    const int tid = threadIdx.x;
    const int64_t S = hdr->sig_pairs;
    const int64_t gb = (int64_t)1 << gshift;
    long long nb = 0;
    for (int64_t s = g * gb + tid; s < (g + 1) * gb && s < S; s += blockDim.x) {
        const long long b = (nitems[s] + tile - 1) / tile;
        nb = b > nb ? b : nb;
    }
    red[tid] = nb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = red[tid + w] > red[tid] ? red[tid + w] : red[tid];
        __syncthreads();
    }
    if (tid == 0) gcnt[g] = red[0] * gb;
}

hipError_t launch_pairs(const Layout &L, const Basis &b, char *ws, const double *xyz, const double *dens,
                        double tau, hipStream_t st, bool fixed_order)
{
    DevHeader *hdr = (DevHeader *)(ws + L.hdr);
    const BasisDev *bd = (const BasisDev *)(ws + L.basis);
    const int64_t np = L.npair;
    const int bs = 256;
    const unsigned nbp = (unsigned)((np + bs - 1) / bs);
    long long *cnt = (long long *)(ws + L.bucket_cnt);
    long long *off = (long long *)(ws + L.bucket_off);
    int *cur = (int *)(ws + L.bucket_cur);
    hipLaunchKernelGGL(k_fill_i64, dim3((kNumBuckets + 255) / 256), dim3(256), 0, st, cnt, (int64_t)kNumBuckets);
    hipLaunchKernelGGL(k_pair_q, dim3(nbp), dim3(bs), 0, st, b, bd, hdr, L.n, xyz, (double *)(ws + L.q_unsorted));
    hipLaunchKernelGGL(k_bucket_count, dim3(nbp), dim3(bs), 0, st, L.n, tau, hdr, xyz,
                       (const double *)(ws + L.q_unsorted), (int *)(ws + L.bucket_of), cnt);
    hipError_t e = launch_scan(cnt, kNumBuckets, off, (long long *)(ws + L.scan_tmp), nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_cursors, dim3((kNumBuckets + 255) / 256), dim3(256), 0, st, off, cur, hdr);
    // fixed order: the pair of every position first (the item counts' storage is free until
    // the limits are computed below)
    int *slot = fixed_order ? (int *)(ws + L.nitems) : nullptr;
    if (fixed_order) {
        hipLaunchKernelGGL(k_bucket_max, dim3((kNumBuckets + 255) / 256), dim3(256), 0, st, off, hdr);
        int hmax = 0;
        e = hipMemcpyAsync(&hmax, &hdr->max_bucket, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (hmax > kMaxFixedBucket) return hipErrorNotSupported;
        hipLaunchKernelGGL(k_slot_fill, dim3(nbp), dim3(bs), 0, st, np, (const int *)(ws + L.bucket_of), cur, slot);
        hipLaunchKernelGGL(k_slot_sort, dim3((kNumBuckets + 255) / 256), dim3(256), 0, st, off, slot);
    }
    hipLaunchKernelGGL(k_pair_scatter, dim3(nbp), dim3(bs), 0, st, b, bd, hdr, L.n, L.pcap, xyz, dens,
                       (const double *)(ws + L.q_unsorted), (const int *)(ws + L.bucket_of), cur,
                       (int *)(ws + L.pk), (int *)(ws + L.pl), (double *)(ws + L.pq), (double *)(ws + L.pd),
                       (double *)(ws + L.prim), (float *)(ws + L.prim_f), (double *)(ws + L.bra),
                       (float *)(ws + L.bra_f), L.atoms ? (double *)(ws + L.bip) : nullptr,
                       L.atoms ? (float *)(ws + L.bip_f) : nullptr, L.pmu ? (double *)(ws + L.pmu) : nullptr,
                       L.pmu ? (double *)(ws + L.pfa) : nullptr, L.bgw ? (double *)(ws + L.bgw) : nullptr,
                       L.bgw ? (float *)(ws + L.bgw_f) : nullptr, slot);
    hipLaunchKernelGGL(k_pair_pad, dim3((unsigned)((L.pcap + 255) / 256)), dim3(256), 0, st, hdr, L.pcap, L.g2,
                       true, L.atoms ? 5 : -1, L.atoms ? 4 : -1,
                       (int *)(ws + L.pk), (int *)(ws + L.pl), (double *)(ws + L.pq), (double *)(ws + L.pd),
                       (double *)(ws + L.prim), (float *)(ws + L.prim_f), L.pmu ? (double *)(ws + L.pmu) : nullptr,
                       L.pmu ? (double *)(ws + L.pfa) : nullptr);
    hipLaunchKernelGGL(k_limits, dim3((unsigned)((L.pcap + 255) / 256)), dim3(256), 0, st, hdr, tau,
                       (const double *)(ws + L.pq), off, (long long *)(ws + L.nitems), (int *)(ws + L.lim),
                       L.pcap);
    e = launch_scan((const long long *)(ws + L.nitems), L.pcap, (long long *)(ws + L.item_off),
                    (long long *)(ws + L.scan_tmp), &hdr->items, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_blocks, dim3((unsigned)L.ngroups), dim3(256), 0, st, hdr,
                       (const long long *)(ws + L.nitems), L.ngroups, L.gshift, L.tile, (long long *)(ws + L.gcnt));
    return launch_scan((const long long *)(ws + L.gcnt), L.ngroups, (long long *)(ws + L.goff),
                       (long long *)(ws + L.scan_tmp), &hdr->blocks, st);
}

}  // namespace hfk
