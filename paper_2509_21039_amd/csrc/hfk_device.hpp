// Device helpers shared by the libhfk kernels.
#pragma once

#include "hfk_internal.hpp"

namespace hfk {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoOverSqrtPi = 1.12837916709551257389615890312154517;

// H(T) = erf(sqrt T) / sqrt T with H(0) = 2/sqrt(pi): the reduced Boys function
// (2/sqrt(pi)) F0(T).  Accurate library erf; used off the hot path (Schwarz bounds).
__device__ inline double erf_over_sqrt(double T)
{
    if (T < 1e-12) return kTwoOverSqrtPi * (1.0 - T / 3.0);
    const double s = sqrt(T);
    return erf(s) / s;
}

// Gaussian product of the primitives of atoms A and B (coordinates already centred):
// P_ab = (a A + b B)/p and S_ab = w_a w_b exp(-mu |A-B|^2) (pi/p)^(3/2), the charge of
// the product distribution, for every primitive pair ab = a*g + b.
__device__ inline void pair_prims(const Basis &b, const BasisDev *__restrict__ bd, const double *A,
                                  const double *B, double *px, double *py, double *pz, double *ps)
{
    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    const double ab2 = dx * dx + dy * dy + dz * dz;
    for (int ab = 0; ab < b.g2; ++ab) {
        const int a = ab / b.g, c = ab % b.g;
        const double fa = bd->fa[ab], fb = bd->fb[ab];
        px[ab] = fa * A[0] + fb * B[0];
        py[ab] = fa * A[1] + fb * B[1];
        pz[ab] = fa * A[2] + fb * B[2];
        ps[ab] = b.w[a] * b.w[c] * exp(-bd->mu[ab] * ab2) * bd->pi32[ab];
    }
}

// Per-atom bases: the same for atoms i (at A) and j (at B) with exponents and weights from
// the atom rows, plus p = alpha_a + alpha_b of every primitive pair (a on i, b on j).
__device__ inline void pair_prims_atoms(const Basis &b, int64_t i, int64_t j, const double *A, const double *B,
                                        double *px, double *py, double *pz, double *ps, double *pp,
                                        double *pmu = nullptr, double *pfa = nullptr)
{
    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    const double ab2 = dx * dx + dy * dy + dz * dz;
    const double *ei = b.aexp + i * b.g, *ej = b.aexp + j * b.g;
    const double *wi = b.aw + i * b.g, *wj = b.aw + j * b.g;
    for (int ab = 0; ab < b.g2; ++ab) {
        const int a = ab / b.g, c = ab % b.g;
        const double p = ei[a] + ej[c];
        const double fa = ei[a] / p, fb = ej[c] / p;
        px[ab] = fa * A[0] + fb * B[0];
        py[ab] = fa * A[1] + fb * B[1];
        pz[ab] = fa * A[2] + fb * B[2];
        ps[ab] = wi[a] * wj[c] * exp(-(ei[a] * ej[c] / p) * ab2) * pow(kPi / p, 1.5);
        pp[ab] = p;
        if (pmu) {
            pmu[ab] = ei[a] * ej[c] / p;
            pfa[ab] = fa;
        }
    }
}

// Reciprocal square root in FP64: the hardware estimate (relative error ~5e-8) refined by
// one Newton step, y (1 + e/2) with e = 1 - x y^2, leaving ~1.5 e^2 ~ 4e-15.
__device__ inline double rsqrt_fp64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, 0.5, y);
}

__device__ inline float rsqrt_fp32(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ inline double rsqrt_r(double x) { return rsqrt_fp64(x); }
__device__ inline float rsqrt_r(float x) { return rsqrt_fp32(x); }

// Far field of the gradient kernels: E(r) = 1/r and W(r) = E'(r)/r = -1/r^3 from x = r^2,
// scaled for the kernels' accumulators.  FP64: the estimate y of x^(-1/2) takes one Newton
// step folded into the product, e = y (x y^2 - 3) = -2 y1 (error ~1.5 (5e-8)^2), so E is carried
// times kE = -2 and W = e^3 = -8 y1^3 times kW = 8; the near-branch tables are scaled to match
// and the sums scaled back once per quartet.  FP32 has no Newton step: E = y, W = -y^3.
template <typename R> struct GradScale;
template <> struct GradScale<double> {
    static constexpr double kE = -2.0, kW = 8.0;
    static __device__ double e_far(double x)
    {
        const double y = __builtin_amdgcn_rsq(x);
        return y * fma(x, y * y, -3.0);
    }
    static __device__ double w_far(double e) { return e * e * e; }
};
template <> struct GradScale<float> {
    static constexpr float kE = 1.0f, kW = 1.0f;
    static __device__ float e_far(float x) { return rsqrt_fp32(x); }
    static __device__ float w_far(float e) { return -(e * e * e); }
};

// Table row of a lane below the switch radius, from r2 = |P-Q|^2 and rsh = rho/h:
// T' = r2 rsh on the grid of this precision.  Adding the rounding constant 1.5 2^52 (FP32:
// 1.5 2^23) in the FMA that forms T' rounds it to the nearest row, whose index is then read
// off the sum's encoding (no separate round and convert).  Returns the row's byte offset (rows
// of kRowLen values) and d = T' - row from one more FMA.
// The row needs no clamp: a caller takes this branch only for r2 < sw, where the switch
// radius^2 sw = kTswitch / rho and rsh come from the same rho (per-atom bases derive rsh
// from sw itself), so T' < kTswitch / h up to a few roundings and the row is at most
// kTswitch / h = 384 (FP32: 512), below the table's rows; r2 is a sum of squares, or in the
// expanded FP64 form below zero by rounding only (~1e-12 bohr^2), so the row is at least 0.
template <typename R, int kRowLen = BoysGrid<R>::stride>
__device__ inline unsigned boys_row(R r2, R rsh, R &d)
{
    using BG = BoysGrid<R>;
    constexpr unsigned kRowBytes = kRowLen * sizeof(R);
    static_assert(BG::rows > kTswitch * BG::inv_h, "rows up to kTswitch / h");
    if constexpr (sizeof(R) == 8) {
        constexpr double kRound = 6755399441055744.0;   // 1.5 * 2^52
        const double sum = fma(r2, rsh, kRound);
        d = fma(r2, rsh, -(sum - kRound));
        // the low 32 bits of the sum's encoding are the row
        return __umul24((unsigned)__double_as_longlong(sum), kRowBytes);
    } else {
        constexpr float kRound = 12582912.0f;           // 1.5 * 2^23
        const float sum = fmaf(r2, rsh, kRound);
        d = fmaf(r2, rsh, -(sum - kRound));
        // the sum is 1.5 2^23 + row, whose encoding is 0x4B400000 + row
        return (__float_as_uint(sum) - 0x4B400000u) * kRowBytes;
    }
}

// The row's polynomial at d (Horner).  FP64 rows are 48 bytes and FP32 rows 16 bytes, on
// 16-byte boundaries: three LDS reads and one.
template <typename R>
__device__ inline R boys_eval(const R *__restrict__ tab, unsigned off, R d)
{
    const R *c = (const R *)((const char *)tab + off);
    if constexpr (sizeof(R) == 8) {
        // degree-5 rows of 48 bytes on 16-byte boundaries: three LDS reads
        static_assert(BoysGrid<double>::order == 6 && BoysGrid<double>::stride == 6, "degree-5 rows");
        const double2 c01 = ((const double2 *)c)[0], c23 = ((const double2 *)c)[1], c45 = ((const double2 *)c)[2];
        R v = c45.y;
        v = v * d + c45.x;
        v = v * d + c23.y;
        v = v * d + c23.x;
        v = v * d + c01.y;
        v = v * d + c01.x;
        return v;
    } else {
        static_assert(BoysGrid<float>::order == 4 && BoysGrid<float>::stride == 4, "degree-3 rows of 16 bytes");
        const float4 r = *(const float4 *)c;
        return fmaf(fmaf(fmaf(r.w, d, r.z), d, r.y), d, r.x);
    }
}

// Value and derivative in d of a degree-7 FP64 row (kBoysOrderG coefficients) by joint
// Horner steps: p = p d + c_m, q = q d + p.
__device__ inline double boys_eval_d(const double *__restrict__ tab, unsigned off, double d, double &dp)
{
    static_assert(kBoysOrderG == 8, "degree-7 rows");
    const double *c = (const double *)((const char *)tab + off);
    double p = c[7], q = p;
    p = fma(p, d, c[6]);
    q = fma(q, d, p);
    p = fma(p, d, c[5]);
    q = fma(q, d, p);
    p = fma(p, d, c[4]);
    q = fma(q, d, p);
    p = fma(p, d, c[3]);
    q = fma(q, d, p);
    p = fma(p, d, c[2]);
    q = fma(q, d, p);
    p = fma(p, d, c[1]);
    q = fma(q, d, p);
    p = fma(p, d, c[0]);
    dp = q;
    return p;
}

// Wave-uniform tables read through the constant address space are fetched with scalar
// loads (they are never written while a kernel runs).
template <typename T> using cptr = const __attribute__((address_space(4))) T *;

// Buffer loads from an SoA table [C][g2][pcap] with the ket t as a 32-bit lane offset.  A
// resource covers `rows` consecutive primitive-pair rows of one component starting at row
// first_row (the 64-bit part of the address lives in the resource base), and the row within
// it is the scalar offset d * pcap * sizeof(R): every offset and the record count stay below
// 2^31 for tables of up to 2^31 / (rows * sizeof(R)) pairs, whatever the number of
// components and primitive pairs in front.
template <typename R>
__device__ inline __amdgpu_buffer_rsrc_t ket_rows(const R *tab, int64_t first_row, int64_t pcap, int rows)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(tab + first_row * pcap), (short)0,
                                             (int)((int64_t)rows * pcap * (int64_t)sizeof(R)), 0x00020000);
}

template <typename R>
__device__ inline R ket_load(__amdgpu_buffer_rsrc_t rc, unsigned voff, int soff)
{
    if constexpr (sizeof(R) == 8)
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rc, (int)voff, soff, 0));
    else
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)voff, soff, 0));
}

// Pair index p = i(i+1)/2 + j (i >= j) back to (i, j).
__device__ inline void pair_of_index(int64_t p, int64_t &i, int64_t &j)
{
    int64_t r = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > p) --r;
    while ((r + 1) * (r + 2) / 2 <= p) ++r;
    i = r;
    j = p - r * (r + 1) / 2;
}

// Q band: floor((1 - log2 q) * bands per octave), clamped; larger Q -> smaller band.
__device__ inline int q_band(double q)
{
    const double x = (1.0 - log2(q)) * (double)kBandsPerOctave;
    if (!(x < (double)(kNumBands - 1))) return kNumBands - 1;
    return x < 0.0 ? 0 : (int)x;
}

// Wave-wide sum (64 lanes) of a double through cross-lane shuffles.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int lane_id() { return (int)__lane_id(); }

// Packs this wave's kets t = base + r * 64 + lane (r < kSubChunks) for which keep(t) holds
// into perm[0 .. count), in ascending order (ballot + lane count, no atomics), and returns
// the wave-uniform count.
template <typename Keep>
__device__ inline int pack_kets(long long base, int lane, int *__restrict__ perm, Keep keep)
{
    int count = 0;
#pragma unroll
    for (int r = 0; r < kSubChunks; ++r) {
        const long long t = base + r * kWave + lane;
        const bool ok = keep(t);
        const unsigned long long mk = __builtin_amdgcn_ballot_w64(ok);
        if (ok)
            perm[count + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u))] =
                (int)t;
        count += (int)__popcll(mk);
    }
    __builtin_amdgcn_wave_barrier();
    return count;
}

}  // namespace hfk
