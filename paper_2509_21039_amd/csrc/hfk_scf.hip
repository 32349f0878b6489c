// Closed-shell self-consistent field around the two-electron build: the loop on either side
// of the paper's kernel (which computes the electron-repulsion term of the Fock operator).
//
//   H = T + V (one-electron integrals of contracted s functions, kernels below)
//   X = S^(-1/2) (symmetric orthogonalisation)
//   repeat: G = G(D) (the screened two-electron build), F = H + G,
//           E = 1/2 sum D o (H + F) + E_nn,
//           e = X (F D S - S D F) X (the commutator in the orthonormal basis),
//           F_x = DIIS extrapolation over the last kDiisMax (F, e),
//           eigenvectors C' of X F_x X, C = X C', D = 2 C_occ C_occ^T (Aufbau)
//   until |E - E_prev| < e_tol and max |e| < d_tol.
//
// The integral kernels and the two-electron build are this library's; the dense products
// and the symmetric eigenproblems go to rocBLAS and rocSOLVER, whose scratch comes from the
// caller's workspace.  Matrices are n x n FP64 with leading dimension n; every one that is
// symmetric reads the same in either storage order, and the products are taken column-major.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "hfk_device.hpp"
#include "hfk_scf.hpp"

namespace hfk {

// ------------------------------------------------------------------ one-electron integrals

// S and H = T + V for every i >= j (written to both triangles).  For primitives a (atom i)
// and b (atom j): p = a + b, mu = a b / p, K = w_a w_b exp(-mu R^2),
//   S_ab = K (pi/p)^(3/2),  T_ab = mu (3 - 2 mu R^2) S_ab,
//   V_ab = - sum_C Z_C K (2 pi / p) F0(p |P - C|^2),  F0(t) = (sqrt(pi)/2) erf(sqrt t)/sqrt t.
// A primitive product whose K (2 pi / p) is below 1e-17 skips the nucleus loop: its term is
// at most 1e-17 times the total nuclear charge (F0 <= 1).
__global__ __launch_bounds__(256) void k_one_electron(int64_t n, int g, const double *__restrict__ xyz,
                                                      const double *__restrict__ Z,
                                                      const double *__restrict__ aexp,
                                                      const double *__restrict__ aw, double *__restrict__ S,
                                                      double *__restrict__ H)
{
    const int64_t npair = n * (n + 1) / 2;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npair) return;
    int64_t i, j;
    pair_of_index(q, i, j);
    const double A[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    const double B[3] = {xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2]};
    const double r2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    double s = 0.0, t = 0.0, v = 0.0;
    for (int a = 0; a < g; ++a)
        for (int c = 0; c < g; ++c) {
            const double ea = aexp[i * g + a], eb = aexp[j * g + c];
            const double p = ea + eb, mu = ea * eb / p;
            const double K = aw[i * g + a] * aw[j * g + c] * exp(-mu * r2);
            const double sab = K * pow(kPi / p, 1.5);
            s += sab;
            t += mu * (3.0 - 2.0 * mu * r2) * sab;
            const double kv = K * (2.0 * kPi / p);
            if (fabs(kv) < 1e-17) continue;
            const double P[3] = {(ea * A[0] + eb * B[0]) / p, (ea * A[1] + eb * B[1]) / p,
                                 (ea * A[2] + eb * B[2]) / p};
            double vz = 0.0;
            for (int64_t cc = 0; cc < n; ++cc) {
                const double dx = P[0] - xyz[3 * cc], dy = P[1] - xyz[3 * cc + 1], dz = P[2] - xyz[3 * cc + 2];
                vz += Z[cc] * erf_over_sqrt(p * (dx * dx + dy * dy + dz * dz));
            }
            v -= kv * 0.5 * sqrt(kPi) * vz;
        }
    S[i * n + j] = S[j * n + i] = s;
    H[i * n + j] = H[j * n + i] = t + v;
}

// E_nn = sum_{A > B} Z_A Z_B / R_AB (one block, fixed order).
__global__ __launch_bounds__(256) void k_enuc(int64_t n, const double *__restrict__ xyz, const double *__restrict__ Z,
                                              double *__restrict__ out)
{
    __shared__ double red[256];
    double e = 0.0;
    for (int64_t a = threadIdx.x; a < n; a += 256)
        for (int64_t b = 0; b < a; ++b) {
            const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                         dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            e += Z[a] * Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------ small dense helpers

// W(:, k) = U(:, k) / sqrt(s_k) (column-major).
__global__ __launch_bounds__(256) void k_scale_cols(int64_t n, const double *__restrict__ U,
                                                    const double *__restrict__ s, double *__restrict__ W)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n * n) W[x] = U[x] / sqrt(s[x / n]);
}

__global__ __launch_bounds__(256) void k_add(int64_t m, const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ c)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) c[x] = a[x] + b[x];
}

// Out = A - A^T.
__global__ __launch_bounds__(256) void k_antisym(int64_t n, const double *__restrict__ A, double *__restrict__ out)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * n) return;
    const int64_t r = x % n, c = x / n;
    out[x] = A[x] - A[r * n + c];
}

// The numbers the host needs after each build, in one launch of 3 + kDiisMax blocks, each a
// fixed-order block reduction (so repeated runs agree bit for bit):
//   out[0] = <D, H>, out[1] = <D, F>, out[2] = max |e|,
//   out[3 + k] = <e, e_k> for every history slot k set in `filled` (0 for the others).
__global__ __launch_bounds__(256) void k_scf_scalars(int64_t n2, const double *__restrict__ D,
                                                     const double *__restrict__ H, const double *__restrict__ F,
                                                     const double *__restrict__ e, const double *__restrict__ hist,
                                                     unsigned filled, double *__restrict__ out)
{
    __shared__ double red[256];
    const int q = blockIdx.x;   // uniform over the block: an early return keeps every barrier whole
    const bool mx = q == 2;
    const double *a = q < 2 ? D : e;
    const double *b = q == 0 ? H : (q == 1 ? F : (q == 2 ? e : hist + (int64_t)(q - 3) * n2));
    if (q >= 3 && !((filled >> (q - 3)) & 1u)) {
        if (threadIdx.x == 0) out[q] = 0.0;
        return;
    }
    double v = 0.0;
    for (int64_t x = threadIdx.x; x < n2; x += 256) v = mx ? fmax(v, fabs(a[x])) : fma(a[x], b[x], v);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] = mx ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
}

struct Coefs {
    double c[kDiisMax];
    int slot[kDiisMax];
    int m;
};

// out = sum_i c_i F[slot_i] (the DIIS combination).
__global__ __launch_bounds__(256) void k_lincomb(int64_t n2, Coefs cf, const double *__restrict__ hist,
                                                 double *__restrict__ out)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n2) return;
    double s = 0.0;
    for (int i = 0; i < cf.m; ++i) s += cf.c[i] * hist[(int64_t)cf.slot[i] * n2 + x];
    out[x] = s;
}

// ------------------------------------------------------------------ layout

ScfLayout make_scf_layout(size_t base, int64_t n)
{
    ScfLayout L;
    size_t o = base;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t n2 = (size_t)n * (size_t)n * sizeof(double);
    L.S = take(n2);
    L.H = take(n2);
    L.X = take(n2);
    L.F = take(n2);
    L.G = take(n2);
    L.Fx = take(n2);
    L.A = take(n2);
    L.C = take(n2);
    L.T1 = take(n2);
    L.T2 = take(n2);
    L.eps = take(sizeof(double) * (size_t)n);
    L.evw = take(sizeof(double) * (size_t)n);
    L.info = take(sizeof(int));
    L.scal = take(sizeof(double) * 32);
    L.Z = take(sizeof(double) * (size_t)n);
    L.diisF = take(n2 * kDiisMax);
    L.diisE = take(n2 * kDiisMax);
    // the eigensolver's scratch grows like n^2 (checked against the library's own query)
    L.rocws_bytes = 4 * n2 + ((size_t)64 << 20);
    L.rocws = take(L.rocws_bytes);
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ the loop

namespace {

struct Ctx {
    rocblas_handle h = nullptr;   // the calling thread's handle for the current device
    hipStream_t st = nullptr;
    int64_t n = 0;
    char *msg = nullptr;
    size_t msglen = 0;
};

// One rocBLAS handle per calling thread and device, created on the first SCF call and kept
// for the life of the thread: creating one per call cost time on every call, and handles are
// not shared between threads.  Each call sets its stream and its workspace before any use.
// The handles are never destroyed (so teardown order at process exit does not matter).
rocblas_handle thread_handle()
{
    thread_local std::vector<rocblas_handle> handles;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    if ((int)handles.size() <= dev) handles.resize(dev + 1, nullptr);
    if (!handles[dev] && rocblas_create_handle(&handles[dev]) != rocblas_status_success) handles[dev] = nullptr;
    return handles[dev];
}

hfk_status say(Ctx &c, hfk_status s, const char *what)
{
    snprintf(c.msg, c.msglen, "%s", what);
    return s;
}

unsigned blocks(int64_t m) { return (unsigned)((m + 255) / 256); }

// C = op(A) op(B) (column-major n x n, inner dimension k).
bool gemm(Ctx &c, bool ta, bool tb, rocblas_int k, const double *A, const double *B, double *C, double alpha = 1.0)
{
    const double beta = 0.0;
    const rocblas_int n = (rocblas_int)c.n;
    return rocblas_dgemm(c.h, ta ? rocblas_operation_transpose : rocblas_operation_none,
                         tb ? rocblas_operation_transpose : rocblas_operation_none, n, n, k, &alpha, A,
                         ta ? k : n, B, tb ? n : k, &beta, C, n) == rocblas_status_success;
}

// Orbitals of Fx: A = X Fx X, eigenpairs (eps ascending, vectors in A), C = X A, and when
// dens is given D = 2 C_occ C_occ^T.
hfk_status diagonalise(Ctx &c, const ScfLayout &SL, char *ws, const double *Fx, int nocc, double *dens)
{
    double *X = (double *)(ws + SL.X), *A = (double *)(ws + SL.A), *C = (double *)(ws + SL.C);
    double *T1 = (double *)(ws + SL.T1);
    if (!gemm(c, false, false, (rocblas_int)c.n, Fx, X, T1) || !gemm(c, false, false, (rocblas_int)c.n, X, T1, A))
        return say(c, HFK_EHIP, "dgemm failed");
    if (rocsolver_dsyevd(c.h, rocblas_evect_original, rocblas_fill_lower, (rocblas_int)c.n, A, (rocblas_int)c.n,
                         (double *)(ws + SL.eps), (double *)(ws + SL.evw), (rocblas_int *)(ws + SL.info)) !=
        rocblas_status_success)
        return say(c, HFK_EHIP, "dsyevd failed");
    if (!gemm(c, false, false, (rocblas_int)c.n, X, A, C)) return say(c, HFK_EHIP, "dgemm failed");
    if (dens) {
        // D = 2 C(:, 0:nocc) C(:, 0:nocc)^T
        const double two = 2.0, zero = 0.0;
        const rocblas_int n = (rocblas_int)c.n;
        if (rocblas_dgemm(c.h, rocblas_operation_none, rocblas_operation_transpose, n, n, (rocblas_int)nocc, &two, C,
                          n, C, n, &zero, dens, n) != rocblas_status_success)
            return say(c, HFK_EHIP, "dgemm failed");
    }
    return HFK_OK;
}

// The status the last symmetric eigensolve left in the workspace (waits for the stream):
// a positive value means it did not converge, as with a matrix that holds NaN or Inf.
hfk_status info_status(Ctx &c, int info)
{
    if (info == 0) return HFK_OK;
    snprintf(c.msg, c.msglen, "dsyevd did not converge (info = %d)", info);
    return HFK_EHIP;
}

hfk_status solver_info(Ctx &c, char *ws, const ScfLayout &SL)
{
    int info = 0;
    if (hipMemcpyAsync(&info, ws + SL.info, sizeof(int), hipMemcpyDeviceToHost, c.st) != hipSuccess ||
        hipStreamSynchronize(c.st) != hipSuccess)
        return say(c, HFK_EHIP, "eigensolver status copy failed");
    return info_status(c, info);
}

// Solves the (m+1) x (m+1) DIIS system by Gaussian elimination with partial pivoting;
// false if it is singular.
bool diis_solve(const std::vector<double> &B, int m, std::vector<double> &coef)
{
    const int N = m + 1;
    std::vector<double> M((size_t)N * (N + 1));
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) M[i * (N + 1) + j] = (i < m && j < m) ? B[i * kDiisMax + j] : (i == m && j == m ? 0.0 : -1.0);
        M[i * (N + 1) + N] = i == m ? -1.0 : 0.0;
    }
    for (int col = 0; col < N; ++col) {
        int piv = col;
        for (int r = col + 1; r < N; ++r)
            if (fabs(M[r * (N + 1) + col]) > fabs(M[piv * (N + 1) + col])) piv = r;
        if (fabs(M[piv * (N + 1) + col]) < 1e-300) return false;
        if (piv != col)
            for (int k = 0; k <= N; ++k) std::swap(M[col * (N + 1) + k], M[piv * (N + 1) + k]);
        for (int r = 0; r < N; ++r) {
            if (r == col) continue;
            const double f = M[r * (N + 1) + col] / M[col * (N + 1) + col];
            for (int k = col; k <= N; ++k) M[r * (N + 1) + k] -= f * M[col * (N + 1) + k];
        }
    }
    coef.assign(m, 0.0);
    for (int i = 0; i < m; ++i) coef[i] = M[i * (N + 1) + N] / M[i * (N + 1) + i];
    return true;
}

}  // namespace

hfk_status run_scf(const Layout &L, const Basis &b, char *ws, const ScfLayout &SL, const double *xyz,
                   const double *charges_host, int nocc, double tau, int prec, int strat, int max_iter,
                   double e_tol, double d_tol, double *dens, bool use_guess, double *eps_out, ScfResult *res,
                   hipStream_t st, char *msg, size_t msglen)
{
    Ctx c;
    c.st = st;
    c.n = L.n;
    c.msg = msg;
    c.msglen = msglen;
    const int64_t n = L.n, n2 = n * n;
    c.h = thread_handle();
    if (!c.h) return say(c, HFK_EHIP, "rocblas_create_handle failed");
    if (rocblas_set_stream(c.h, st) != rocblas_status_success) return say(c, HFK_EHIP, "rocblas_set_stream failed");
    (void)rocblas_set_pointer_mode(c.h, rocblas_pointer_mode_host);
    {
        // the library scratch comes from the workspace: its own size query first (with the
        // real buffers, which a query does not touch)
        size_t need = 0;
        const double one = 1.0, zero = 0.0;
        const rocblas_int ni = (rocblas_int)n;
        double *qa = (double *)(ws + SL.A), *qb = (double *)(ws + SL.T1), *qc = (double *)(ws + SL.T2);
        (void)rocblas_start_device_memory_size_query(c.h);
        (void)rocsolver_dsyevd(c.h, rocblas_evect_original, rocblas_fill_lower, ni, qa, ni, (double *)(ws + SL.eps),
                               (double *)(ws + SL.evw), (rocblas_int *)(ws + SL.info));
        (void)rocblas_dgemm(c.h, rocblas_operation_none, rocblas_operation_none, ni, ni, ni, &one, qa, ni, qb, ni, &zero,
                            qc, ni);
        if (rocblas_stop_device_memory_size_query(c.h, &need) != rocblas_status_success)
            return say(c, HFK_EHIP, "rocblas memory size query failed");
        if (need > SL.rocws_bytes) return say(c, HFK_ENOMEM, "linear-algebra scratch exceeds its workspace share");
        if (rocblas_set_workspace(c.h, ws + SL.rocws, SL.rocws_bytes) != rocblas_status_success)
            return say(c, HFK_EHIP, "rocblas_set_workspace failed");
    }
    double *S = (double *)(ws + SL.S), *H = (double *)(ws + SL.H), *X = (double *)(ws + SL.X);
    double *F = (double *)(ws + SL.F), *G = (double *)(ws + SL.G), *Fx = (double *)(ws + SL.Fx);
    double *A = (double *)(ws + SL.A), *T1 = (double *)(ws + SL.T1), *T2 = (double *)(ws + SL.T2);
    double *Z = (double *)(ws + SL.Z), *scal = (double *)(ws + SL.scal), *eps = (double *)(ws + SL.eps);
    double *hF = (double *)(ws + SL.diisF), *hE = (double *)(ws + SL.diisE);
    hipError_t e = hipMemcpyAsync(Z, charges_host, sizeof(double) * n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return say(c, HFK_EHIP, "charges copy failed");
    hipLaunchKernelGGL(k_one_electron, dim3(blocks(n * (n + 1) / 2)), dim3(256), 0, st, n, b.g, xyz, Z, b.aexp,
                       b.aw, S, H);
    hipLaunchKernelGGL(k_enuc, dim3(1), dim3(256), 0, st, n, xyz, Z, scal);
    if ((e = hipGetLastError()) != hipSuccess) return say(c, HFK_EHIP, "integral launch failed");
    double enn = 0.0;
    if (hipMemcpyAsync(&enn, scal, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return say(c, HFK_EHIP, "nuclear repulsion copy failed");

    // X = S^(-1/2) = U s^(-1/2) U^T
    hfk_status s_ok = HFK_OK;
    if (hipMemcpyAsync(A, S, sizeof(double) * n2, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return say(c, HFK_EHIP, "copy failed");
    if (rocsolver_dsyevd(c.h, rocblas_evect_original, rocblas_fill_lower, (rocblas_int)n, A, (rocblas_int)n, eps,
                         (double *)(ws + SL.evw), (rocblas_int *)(ws + SL.info)) != rocblas_status_success)
        return say(c, HFK_EHIP, "dsyevd failed");
    {
        std::vector<double> s(n);
        if (hipMemcpyAsync(s.data(), eps, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return say(c, HFK_EHIP, "eigenvalue copy failed");
        if ((s_ok = solver_info(c, ws, SL)) != HFK_OK) return s_ok;
        if (!(s[0] > 1e-12 * s[n - 1])) return say(c, HFK_EUNSUPPORTED, "overlap matrix is (nearly) singular");
    }
    hipLaunchKernelGGL(k_scale_cols, dim3(blocks(n2)), dim3(256), 0, st, n, A, eps, T1);
    if (!gemm(c, false, true, (rocblas_int)n, T1, A, X)) return say(c, HFK_EHIP, "dgemm failed");

    if (!use_guess && (s_ok = diagonalise(c, SL, ws, H, nocc, dens)) != HFK_OK) return s_ok;

    std::vector<double> B((size_t)kDiisMax * kDiisMax, 0.0);
    std::vector<int> age(kDiisMax, -1);   // iteration that filled each slot, -1 empty
    double e_old = 0.0, E = 0.0;
    bool have_old = false, conv = false;
    int it = 0;
    double *e2tmp = scal + 1;
    for (it = 1; it <= max_iter; ++it) {
        // G(D), F = H + G
        hipError_t ef = launch_pairs(L, b, ws, xyz, dens, tau, st, strat == HFK_STRATEGY_DETERMINISTIC);
        if (ef == hipSuccess) ef = launch_fock(L, b, ws, dens, tau, prec, strat, 1, G, e2tmp, st);
        if (ef != hipSuccess) return say(c, HFK_EHIP, "Fock build failed");
        hipLaunchKernelGGL(k_add, dim3(blocks(n2)), dim3(256), 0, st, n2, H, G, F);
        // e = X (F D S - S D F) X into the history slot of the oldest entry
        int slot = 0;
        for (int k = 0; k < kDiisMax; ++k)
            if (age[k] < age[slot]) slot = k;
        double *ek = hE + (int64_t)slot * n2;
        if (!gemm(c, false, false, (rocblas_int)n, F, dens, T1) || !gemm(c, false, false, (rocblas_int)n, T1, S, T2))
            return say(c, HFK_EHIP, "dgemm failed");
        hipLaunchKernelGGL(k_antisym, dim3(blocks(n2)), dim3(256), 0, st, n, T2, T1);
        if (!gemm(c, false, false, (rocblas_int)n, T1, X, T2) || !gemm(c, false, false, (rocblas_int)n, X, T2, ek))
            return say(c, HFK_EHIP, "dgemm failed");
        if (hipMemcpyAsync(hF + (int64_t)slot * n2, F, sizeof(double) * n2, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return say(c, HFK_EHIP, "copy failed");
        age[slot] = it;
        // E = 1/2 (<D, H> + <D, F>) + E_nn, max |e| and the new row of the DIIS matrix, read
        // back with one wait
        unsigned filled = 0;
        for (int k = 0; k < kDiisMax; ++k)
            if (age[k] >= 0) filled |= 1u << k;
        hipLaunchKernelGGL(k_scf_scalars, dim3(3 + kDiisMax), dim3(256), 0, st, n2, dens, H, F, ek, hE, filled,
                           scal + 8);
        // with the status of the last eigensolve: the one whose orbitals gave this density
        double sc[3 + kDiisMax];
        int info = 0;
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sc, scal + 8, sizeof(sc), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&info, ws + SL.info, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return say(c, HFK_EHIP, "scalar copy failed");
        if ((s_ok = info_status(c, info)) != HFK_OK) return s_ok;
        E = 0.5 * (sc[0] + sc[1]) + enn;
        const double emax = sc[2];
        for (int k = 0; k < kDiisMax; ++k)
            if (age[k] >= 0) B[slot * kDiisMax + k] = B[k * kDiisMax + slot] = sc[3 + k];
        if (have_old && fabs(E - e_old) < e_tol && emax < d_tol) {
            conv = true;
            break;
        }
        // the last build allowed: its density is the one whose energy is E (no further
        // eigensolve, which could also leave a failed solve behind the returned density)
        if (it == max_iter) break;
        // DIIS over the filled slots (oldest first), else F itself
        std::vector<int> order;
        for (int k = 0; k < kDiisMax; ++k)
            if (age[k] >= 0) order.push_back(k);
        std::sort(order.begin(), order.end(), [&](int x, int y) { return age[x] < age[y]; });
        const double *Fuse = F;
        if (order.size() >= 2) {
            const int m = (int)order.size();
            std::vector<double> Bm((size_t)kDiisMax * kDiisMax, 0.0), coef;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) Bm[i * kDiisMax + j] = B[order[i] * kDiisMax + order[j]];
            if (diis_solve(Bm, m, coef)) {
                Coefs cf;
                cf.m = m;
                for (int i = 0; i < m; ++i) {
                    cf.c[i] = coef[i];
                    cf.slot[i] = order[i];
                }
                hipLaunchKernelGGL(k_lincomb, dim3(blocks(n2)), dim3(256), 0, st, n2, cf, hF, Fx);
                Fuse = Fx;
            }
        }
        if ((s_ok = diagonalise(c, SL, ws, Fuse, nocc, dens)) != HFK_OK) return s_ok;
        e_old = E;
        have_old = true;
    }
    if (it > max_iter) it = max_iter;
    // orbital energies of the final F (the density stays the one that built it)
    if ((s_ok = diagonalise(c, SL, ws, F, nocc, nullptr)) != HFK_OK) return s_ok;
    if (eps_out && hipMemcpyAsync(eps_out, eps, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return say(c, HFK_EHIP, "eigenvalue copy failed");
    if (hipStreamSynchronize(st) != hipSuccess) return say(c, HFK_EHIP, "stream sync failed");
    if ((s_ok = solver_info(c, ws, SL)) != HFK_OK) return s_ok;
    res->energy = E;
    res->iterations = it;
    res->converged = conv ? 1 : 0;
    return HFK_OK;
}

}  // namespace hfk
