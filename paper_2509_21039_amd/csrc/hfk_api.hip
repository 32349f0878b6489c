// Host side of the libhfk C ABI: validation, workspace layout and launch sequencing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hfk_internal.hpp"
#include "hfk_scf.hpp"

namespace hfk {

static thread_local char g_err[512];

static hfk_status fail(hfk_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

static hfk_status hip_fail(hipError_t e, const char *where)
{
    return fail(HFK_EHIP, "%s: %s", where, hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// Per-workgroup copies of F are used while they stay within this many bytes in total.
constexpr double kPrivateBudget = 16.0e9;
// Ket-side Coulomb vectors: one per workgroup within this budget, else fewer copies that
// workgroups share through atomics.
constexpr double kJcolBudget = 8.0e9;

Layout make_layout(int64_t n, int g, int prec, int with_grad, int groups, bool atoms)
{
    Layout L;
    memset(&L, 0, sizeof(L));
    L.n = n;
    L.atoms = atoms;
    L.tile = prec == HFK_MIXED ? 2 * kTileItems : kTileItems;
    L.private_ok = (double)groups * (double)n * (double)n * 8.0 <= kPrivateBudget;
    L.npair = n * (n + 1) / 2;
    L.pcap = ((L.npair + 63) / 64) * 64 + 64;
    L.g = g;
    L.g2 = g * g;
    L.groups = groups;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t P = (size_t)L.npair, PC = (size_t)L.pcap, g2 = (size_t)L.g2;
    L.hdr = take(sizeof(DevHeader));
    L.basis = take(sizeof(BasisDev));
    L.boys = take(sizeof(double) * kBoysGrid * kBoysStride);
    L.boys_f = take(sizeof(float) * kBoysGrid * kBoysStride);
    L.q_unsorted = take(sizeof(double) * P);
    L.bucket_of = take(sizeof(int) * P);
    L.bucket_cnt = take(sizeof(long long) * kNumBuckets);
    L.bucket_off = take(sizeof(long long) * (kNumBuckets + 1));
    L.bucket_cur = take(sizeof(int) * kNumBuckets);
    L.pk = take(sizeof(int) * PC);
    L.pl = take(sizeof(int) * PC);
    L.pq = take(sizeof(double) * PC);
    L.pd = take(sizeof(double) * PC);
    L.prim = take(sizeof(double) * (atoms ? 6 : 5) * g2 * PC);   // Px, Py, Pz, S, |P|^2 (, 1/p)
    L.prim_f = take(sizeof(float) * (atoms ? 5 : 4) * g2 * PC);
    if (atoms) {
        L.arow = take(sizeof(double) * 2 * (size_t)n * (size_t)g);
        L.bip = take(sizeof(double) * g2 * PC);
        L.bip_f = take(sizeof(float) * g2 * PC);
        if (with_grad) {
            L.pmu = take(sizeof(double) * g2 * PC);
            L.pfa = take(sizeof(double) * g2 * PC);
            L.bmf = take(sizeof(double) * 2 * g2 * PC);
        }
    }
    L.bra = take(sizeof(double) * 8 * g2 * PC);
    L.bra_f = take(sizeof(float) * 8 * g2 * PC);
    L.boys_g = take(sizeof(double) * kBoysGrid * kBoysStride);
    L.boys_g_f = take(sizeof(float) * kBoysGrid * kBoysStride);
    L.nitems = take(sizeof(long long) * PC);
    L.lim = take(sizeof(int) * PC);
    L.item_off = take(sizeof(long long) * (PC + 1));
    L.ngroups = (L.pcap + kGroupBras - 1) / kGroupBras;
    L.gcnt = take(sizeof(long long) * (size_t)(L.ngroups + 1));
    L.goff = take(sizeof(long long) * (size_t)(L.ngroups + 1));
    L.scan_tmp = take(sizeof(long long) * (((PC > (size_t)kNumBuckets ? PC : (size_t)kNumBuckets) + 1023) / 1024 + 1));
    const size_t n2 = (size_t)(n * n);
    L.fpriv = take(sizeof(double) * n2 * (size_t)(L.private_ok ? groups : 1));
    {
        const double fit = kJcolBudget / (8.0 * (double)PC);
        L.jcopies = fit >= (double)groups ? groups : (fit >= 1.0 ? (int)fit : 1);
    }
    L.jcol = take(sizeof(double) * PC * (size_t)L.jcopies);
    L.fsum = take(sizeof(double) * n2);
    L.e2part = take(sizeof(double) * ((n2 + 255) / 256 + 256));
    L.grad = with_grad ? take(sizeof(double) * 3 * (size_t)n * (size_t)groups + sizeof(double) * 4096) : 0;
    L.xw = with_grad ? take(sizeof(double) * 2 * n2) : 0;
    L.e2tmp = take(sizeof(double));
    L.total = o;
    return L;
}

constexpr int kMaxGroupsPerCU = 6;
// Kernels are instantiated for 1 .. kMaxBuiltG primitives per atom.
constexpr int kMaxBuiltG = HFK_BUILT_NGAUSS;
static int g_cfg_variant = -1;
static int g_cfg_gpc = 0;

// Workgroups the buffers are sized for (the most any configuration launches).
static int groups_cap(int cus) { return (cus > 0 ? cus : 256) * kMaxGroupsPerCU; }

// need_dens: the call reads a density (every build does; the SCF makes its own)
static hfk_status check_common(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps,
                               const double *coefs, const double *dens, double tau, int32_t precision,
                               bool need_dens = true)
{
    if (natoms < 1) return fail(HFK_EINVAL, "natoms must be >= 1 (got %lld)", (long long)natoms);
    if (ngauss < 1 || ngauss > HFK_MAX_NGAUSS)
        return fail(HFK_EINVAL, "ngauss must be in [1, %d] (got %d)", HFK_MAX_NGAUSS, (int)ngauss);
    if (!xyz) return fail(HFK_EINVAL, "xyz is NULL");
    if (need_dens && !dens) return fail(HFK_EINVAL, "dens is NULL");
    if (!exps) return fail(HFK_EINVAL, "exps_host is NULL");
    if (!coefs) return fail(HFK_EINVAL, "coefs_host is NULL");
    for (int a = 0; a < ngauss; ++a) {
        if (!(exps[a] > 0.0) || !isfinite(exps[a]))
            return fail(HFK_EINVAL, "exps_host[%d] must be finite and > 0 (got %g)", a, exps[a]);
        if (!isfinite(coefs[a])) return fail(HFK_EINVAL, "coefs_host[%d] is not finite", a);
    }
    if (!isfinite(tau) || tau < 0.0) return fail(HFK_EINVAL, "tau must be finite and >= 0 (got %g)", tau);
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    return HFK_OK;
}

// Per-atom rows: every exponent finite and > 0, every coefficient finite.
static hfk_status check_rows(int64_t natoms, int32_t ngauss, const double *exps, const double *coefs)
{
    for (int64_t x = 0; x < natoms * ngauss; ++x) {
        if (!(exps[x] > 0.0) || !isfinite(exps[x]))
            return fail(HFK_EINVAL, "exps_host[%lld] (atom %lld) must be finite and > 0 (got %g)", (long long)x,
                        (long long)(x / ngauss), exps[x]);
        if (!isfinite(coefs[x]))
            return fail(HFK_EINVAL, "coefs_host[%lld] (atom %lld) is not finite", (long long)x,
                        (long long)(x / ngauss));
    }
    return HFK_OK;
}

static Basis make_basis(int32_t ngauss, const double *exps, const double *coefs)
{
    Basis b;
    memset(&b, 0, sizeof(b));
    b.g = ngauss;
    b.g2 = ngauss * ngauss;
    for (int a = 0; a < ngauss; ++a) {
        b.alpha[a] = exps[a];
        b.w[a] = coefs[a] * pow(2.0 * exps[a] / 3.14159265358979323846, 0.75);
    }
    return b;
}

// n above which rows i and j of F no longer fit in one workgroup's LDS next to the Boys table
constexpr int64_t kMaxAtoms = 6144;
// n above which the gradient kernel's LDS copy of dE2/dR (n x 3) and its two tables no longer fit
constexpr int64_t kMaxGradAtoms = 4096;
constexpr int kGradGroupsPerCU = 2;
// Items per block of the gradient kernel: eight (he512 FP64 184 ms against 191 with four;
// its per-item work is about 2.4 times the forward's, so fewer row flushes matter more
// than the smaller ket working set).
constexpr int kGradTileItems = 8;
// Largest system of the deterministic strategy: every workgroup needs its own copies of F
// and of the ket vector within the workspace budgets, and four wave copies of rows i, j in LDS.
constexpr int64_t kMaxDetAtoms = 1024;

// Deterministic strategy: every workgroup must own a copy of F and of the ket vector.
static hfk_status det_groups(Layout &L)
{
    if (!L.private_ok) return fail(HFK_EUNSUPPORTED, "private copies of F do not fit for the deterministic strategy");
    if (L.jcopies < L.groups) L.groups = L.jcopies;
    return HFK_OK;
}
// Largest molecule of a batch (its triangle of F and its gradient stay in LDS).
constexpr int kMaxBatchAtomsApi = 128;
static int g_cfg_batch_gpc = 0;
static int g_tuned_batch_gpc = 0;

// Tuned strategy per (precision, size class); 0 = not tuned.
static std::mutex g_tune_mu;

static int size_class(int64_t n) { return n <= 128 ? 0 : n <= 384 ? 1 : n <= 768 ? 2 : 3; }

struct TunedConfig {
    int strategy;      // 0 = not tuned
    int variant;
    int gpc;
};
static TunedConfig g_tuned_cfg[2][4];

// The configuration before any tuning.  Timed over whole calls (side kernels included) on
// MI355X for He 64 to 1024 and H/He 128, FP64 and mixed: ATOMIC was the faster strategy at
// every size (the per-workgroup copies of F and their summation cost more than the atomics
// they save), and small systems ran fastest with fewer workgroups per CU (2 at 64 atoms,
// 4 at 128, the most that fit above).
static TunedConfig default_config(int64_t n)
{
    return TunedConfig{HFK_STRATEGY_ATOMIC, 1, n <= 64 ? 2 : (n <= 128 ? 4 : 6)};
}

static TunedConfig pick_config(int32_t strategy, int32_t precision, int64_t n, int32_t ngauss)
{
    TunedConfig c;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        c = g_tuned_cfg[precision][size_class(n)];
    }
    if (c.strategy == 0) c = default_config(n);
    if (strategy == HFK_STRATEGY_PRIVATE || strategy == HFK_STRATEGY_ATOMIC) c.strategy = strategy;
    if (g_cfg_variant >= 0) c.variant = g_cfg_variant;
    if (g_cfg_gpc > 0) c.gpc = g_cfg_gpc;
    if (ngauss > 4) c.variant = 1;   // the direct form is built for g <= 4 only
    if (strategy == HFK_STRATEGY_DETERMINISTIC) {
        // a fixed configuration, independent of tuning and overrides (capped at residency)
        c = TunedConfig{HFK_STRATEGY_DETERMINISTIC, 1, kMaxGroupsPerCU};
    }
    return c;
}

// ------------------------------------------------------------------ kernel timing

static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;
static hipEvent_t g_prof_open = nullptr;

void profile_begin(hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    g_prof_open = e;
}

void profile_end(hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || !g_prof_open) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    g_prof_events.emplace_back(g_prof_open, e);
    g_prof_open = nullptr;
}

}  // namespace hfk

using namespace hfk;

extern "C" {

const char *hfk_last_error(void) { return g_err; }

hfk_status hfk_set_config(int32_t variant, int32_t groups_per_cu)
{
    g_err[0] = 0;
    if (variant < -1 || variant > 1) return fail(HFK_EINVAL, "variant must be -1, 0 or 1 (got %d)", (int)variant);
    if (groups_per_cu < 0 || groups_per_cu > kMaxGroupsPerCU)
        return fail(HFK_EINVAL, "groups_per_cu must be in [0, %d] (got %d)", kMaxGroupsPerCU, (int)groups_per_cu);
    g_cfg_variant = variant;
    g_cfg_gpc = groups_per_cu;
    return HFK_OK;
}

hfk_status hfk_profile_enable(int32_t on)
{
    g_err[0] = 0;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return HFK_OK;
}

hfk_status hfk_profile_read(double *total_ms, int64_t *launches)
{
    g_err[0] = 0;
    if (!total_ms || !launches) return fail(HFK_EINVAL, "total_ms and launches must not be NULL");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double sum = 0.0;
    int64_t cnt = 0;
    hfk_status st = HFK_OK;
    for (auto &p : g_prof_events) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess && st == HFK_OK) st = hip_fail(e, "event timing");
        sum += ms;
        ++cnt;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_prof_events.clear();
    *total_ms = sum;
    *launches = cnt;
    return st;
}

const char *hfk_version(void) { return "hfk 0.1 (gfx950)"; }

hfk_status hfk_workspace_bytes(int64_t natoms, int32_t ngauss, int32_t precision, int32_t with_grad,
                               size_t *bytes_out)
{
    g_err[0] = 0;
    if (!bytes_out) return fail(HFK_EINVAL, "bytes_out is NULL");
    if (natoms < 1) return fail(HFK_EINVAL, "natoms must be >= 1 (got %lld)", (long long)natoms);
    if (ngauss < 1 || ngauss > HFK_MAX_NGAUSS)
        return fail(HFK_EINVAL, "ngauss must be in [1, %d] (got %d)", HFK_MAX_NGAUSS, (int)ngauss);
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    const Layout L = make_layout(natoms, ngauss, precision, with_grad, groups_cap(device_cu_count()));
    *bytes_out = L.total;
    return HFK_OK;
}

hfk_status hfk_fock(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                    const double *coefs_host, const double *dens, double tau, int32_t precision,
                    int32_t strategy, double *fock, double *e2, void *workspace, size_t workspace_bytes,
                    void *stream)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    if (!fock) return fail(HFK_EINVAL, "fock is NULL");
    if (!e2) return fail(HFK_EINVAL, "e2 is NULL");
    if (!workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (strategy < HFK_STRATEGY_AUTO || strategy > HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EINVAL, "unknown strategy %d", (int)strategy);
    if (strategy == HFK_STRATEGY_DETERMINISTIC && natoms > kMaxDetAtoms)
        return fail(HFK_EUNSUPPORTED, "the deterministic strategy supports natoms <= %lld", (long long)kMaxDetAtoms);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    Layout L = make_layout(natoms, ngauss, precision, 0, groups_cap(cus));
    if (workspace_bytes < L.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
    const TunedConfig cfg = pick_config(strategy, precision, natoms, ngauss);
    int strat = cfg.strategy;
    if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
    {
        // no more persistent workgroups than fit on a CU at once
        const bool det = strat == HFK_STRATEGY_DETERMINISTIC;
        const int fit = fock_resident_groups(ngauss, precision, cfg.variant, natoms, false, det);
        L.groups = cus * (fit > 0 && cfg.gpc > fit ? fit : cfg.gpc);
        if (det) {
            hfk_status sd = det_groups(L);
            if (sd != HFK_OK) return sd;
        }
    }
    const Basis b = make_basis(ngauss, exps_host, coefs_host);
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys),
                                (float *)(ws + L.boys_f), (double *)(ws + L.boys_g),
                                (float *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = launch_pairs(L, b, ws, xyz, dens, tau, st, strat == HFK_STRATEGY_DETERMINISTIC);
    if (e == hipErrorNotSupported && strat == HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EUNSUPPORTED, "deterministic strategy: more than %d pairs share one (Q band, cell) bucket",
                    kMaxFixedBucket);
    if (e != hipSuccess) return hip_fail(e, "pair launch");
    e = launch_fock(L, b, ws, dens, tau, precision, strat, cfg.variant, fock, e2, st);
    if (e != hipSuccess) return hip_fail(e, "fock launch");
    e = launch_header_info(ws + L.hdr, strat, L.groups, precision, cfg.variant, st);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    return HFK_OK;
}

}  // extern "C"

// Per-atom bases: exponents and weights of every atom, [2][n][g], copied to the workspace,
// and the Basis that points the kernels at them.  The staging vector is pageable host memory
// that ends with this call, so the copy is waited for here rather than trusting the runtime
// to have read it when hipMemcpyAsync returns (the wait also covers work queued before it).
static hipError_t upload_rows(double *arow, int64_t natoms, int32_t ngauss, const double *exps,
                              const double *coefs, hipStream_t st, Basis *b)
{
    const size_t ng = (size_t)natoms * (size_t)ngauss;
    std::vector<double> rows(2 * ng);
    for (size_t x = 0; x < ng; ++x) {
        rows[x] = exps[x];
        rows[ng + x] = coefs[x] * pow(2.0 * exps[x] / 3.14159265358979323846, 0.75);
    }
    memset(b, 0, sizeof(*b));
    b->g = ngauss;
    b->g2 = ngauss * ngauss;
    for (int a = 0; a < ngauss; ++a) b->alpha[a] = 1.0;   // the one-basis tables stay finite, unused
    b->aexp = arow;
    b->aw = arow + ng;
    const hipError_t e = hipMemcpyAsync(arow, rows.data(), sizeof(double) * 2 * ng, hipMemcpyHostToDevice, st);
    return e != hipSuccess ? e : hipStreamSynchronize(st);
}

extern "C" {

hfk_status hfk_workspace_bytes_atoms(int64_t natoms, int32_t ngauss, int32_t precision, int32_t with_grad,
                                     size_t *bytes_out)
{
    g_err[0] = 0;
    if (!bytes_out) return fail(HFK_EINVAL, "bytes_out is NULL");
    if (natoms < 1) return fail(HFK_EINVAL, "natoms must be >= 1 (got %lld)", (long long)natoms);
    if (ngauss < 1 || ngauss > HFK_MAX_NGAUSS)
        return fail(HFK_EINVAL, "ngauss must be in [1, %d] (got %d)", HFK_MAX_NGAUSS, (int)ngauss);
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    if (with_grad && natoms > kMaxGradAtoms)
        return fail(HFK_EUNSUPPORTED, "gradient supports natoms <= %lld", (long long)kMaxGradAtoms);
    const Layout L = make_layout(natoms, ngauss, precision, with_grad, groups_cap(device_cu_count()), true);
    *bytes_out = L.total;
    return HFK_OK;
}

hfk_status hfk_fock_atoms(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                          const double *coefs_host, const double *dens, double tau, int32_t precision,
                          int32_t strategy, double *fock, double *e2, void *workspace, size_t workspace_bytes,
                          void *stream)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    s = check_rows(natoms, ngauss, exps_host, coefs_host);
    if (s != HFK_OK) return s;
    if (!fock) return fail(HFK_EINVAL, "fock is NULL");
    if (!e2) return fail(HFK_EINVAL, "e2 is NULL");
    if (!workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (strategy < HFK_STRATEGY_AUTO || strategy > HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EINVAL, "unknown strategy %d", (int)strategy);
    if (strategy == HFK_STRATEGY_DETERMINISTIC && natoms > kMaxDetAtoms)
        return fail(HFK_EUNSUPPORTED, "the deterministic strategy supports natoms <= %lld", (long long)kMaxDetAtoms);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    Layout L = make_layout(natoms, ngauss, precision, 0, groups_cap(cus), true);
    if (workspace_bytes < L.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
    TunedConfig cfg = pick_config(strategy, precision, natoms, ngauss);
    cfg.variant = 1;   // per-atom bases run the hybrid form only
    int strat = cfg.strategy;
    if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
    {
        const bool det = strat == HFK_STRATEGY_DETERMINISTIC;
        const int fit = fock_resident_groups(ngauss, precision, 1, natoms, true, det);
        L.groups = cus * (fit > 0 && cfg.gpc > fit ? fit : cfg.gpc);
        if (det) {
            hfk_status sd = det_groups(L);
            if (sd != HFK_OK) return sd;
        }
    }
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    Basis b;
    hipError_t e = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
    if (e != hipSuccess) return hip_fail(e, "basis rows copy");
    e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (float *)(ws + L.boys_f),
                     (double *)(ws + L.boys_g), (float *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz,
                     st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = launch_pairs(L, b, ws, xyz, dens, tau, st, strat == HFK_STRATEGY_DETERMINISTIC);
    if (e == hipErrorNotSupported && strat == HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EUNSUPPORTED, "deterministic strategy: more than %d pairs share one (Q band, cell) bucket",
                    kMaxFixedBucket);
    if (e != hipSuccess) return hip_fail(e, "pair launch");
    e = launch_fock(L, b, ws, dens, tau, precision, strat, 1, fock, e2, st);
    if (e != hipSuccess) return hip_fail(e, "fock launch");
    e = launch_header_info(ws + L.hdr, strat, L.groups, precision, 1, st);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    return HFK_OK;
}

hfk_status hfk_scf_workspace_bytes(int64_t natoms, int32_t ngauss, int32_t precision, size_t *bytes_out)
{
    g_err[0] = 0;
    if (!bytes_out) return fail(HFK_EINVAL, "bytes_out is NULL");
    if (natoms < 1) return fail(HFK_EINVAL, "natoms must be >= 1 (got %lld)", (long long)natoms);
    if (ngauss < 1 || ngauss > HFK_MAX_NGAUSS)
        return fail(HFK_EINVAL, "ngauss must be in [1, %d] (got %d)", HFK_MAX_NGAUSS, (int)ngauss);
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    const Layout L = make_layout(natoms, ngauss, precision, 0, groups_cap(device_cu_count()), true);
    *bytes_out = make_scf_layout(L.total, natoms).total;
    return HFK_OK;
}

hfk_status hfk_scf(int64_t natoms, const double *xyz, const double *charges_host, int32_t ngauss,
                   const double *exps_host, const double *coefs_host, int32_t nocc, double tau, int32_t precision,
                   int32_t strategy, int32_t max_iter, double e_tol, double d_tol, double *dens, int32_t use_guess,
                   double *orb_energies, double *energy_host, int32_t *iterations_host, int32_t *converged_host,
                   void *workspace, size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, nullptr, tau, precision, false);
    if (s != HFK_OK) return s;
    s = check_rows(natoms, ngauss, exps_host, coefs_host);
    if (s != HFK_OK) return s;
    if (!charges_host) return fail(HFK_EINVAL, "charges_host is NULL");
    for (int64_t a = 0; a < natoms; ++a)
        if (!isfinite(charges_host[a]) || charges_host[a] < 0.0)
            return fail(HFK_EINVAL, "charges_host[%lld] must be finite and >= 0", (long long)a);
    if (nocc < 0 || nocc > natoms) return fail(HFK_EINVAL, "nocc must be in [0, natoms] (got %d)", (int)nocc);
    if (max_iter < 1) return fail(HFK_EINVAL, "max_iter must be >= 1 (got %d)", (int)max_iter);
    if (!(e_tol > 0.0) || !(d_tol > 0.0) || !isfinite(e_tol) || !isfinite(d_tol))
        return fail(HFK_EINVAL, "e_tol and d_tol must be finite and > 0");
    if (!dens) return fail(HFK_EINVAL, "dens is NULL");
    if (!energy_host || !iterations_host || !converged_host)
        return fail(HFK_EINVAL, "energy_host, iterations_host and converged_host must not be NULL");
    if (!workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (strategy < HFK_STRATEGY_AUTO || strategy > HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EINVAL, "unknown strategy %d", (int)strategy);
    if (strategy == HFK_STRATEGY_DETERMINISTIC && natoms > kMaxDetAtoms)
        return fail(HFK_EUNSUPPORTED, "the deterministic strategy supports natoms <= %lld", (long long)kMaxDetAtoms);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    Layout L = make_layout(natoms, ngauss, precision, 0, groups_cap(cus), true);
    const ScfLayout SL = make_scf_layout(L.total, natoms);
    if (workspace_bytes < SL.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, SL.total);
    TunedConfig cfg = pick_config(strategy, precision, natoms, ngauss);
    cfg.variant = 1;
    int strat = cfg.strategy;
    if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
    {
        const bool det = strat == HFK_STRATEGY_DETERMINISTIC;
        const int fit = fock_resident_groups(ngauss, precision, 1, natoms, true, det);
        L.groups = cus * (fit > 0 && cfg.gpc > fit ? fit : cfg.gpc);
        if (det) {
            hfk_status sd = det_groups(L);
            if (sd != HFK_OK) return sd;
        }
    }
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    Basis b;
    hipError_t e = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
    if (e != hipSuccess) return hip_fail(e, "basis rows copy");
    e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (float *)(ws + L.boys_f),
                     (double *)(ws + L.boys_g), (float *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz,
                     st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    ScfResult r;
    char msg[256];
    msg[0] = 0;
    s = run_scf(L, b, ws, SL, xyz, charges_host, nocc, tau, precision, strat, max_iter, e_tol, d_tol, dens,
                use_guess != 0, orb_energies, &r, st, msg, sizeof(msg));
    if (s != HFK_OK) return fail(s, "scf: %s", msg);
    *energy_host = r.energy;
    *iterations_host = r.iterations;
    *converged_host = r.converged;
    return HFK_OK;
}

hfk_status hfk_read_stats(const void *workspace, void *stream, hfk_stats *out)
{
    g_err[0] = 0;
    if (!workspace || !out) return fail(HFK_EINVAL, "workspace and out must not be NULL");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    DevHeader h;
    e = hipMemcpy(&h, workspace, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "header copy");
    memset(out, 0, sizeof(*out));
    out->natoms = h.natoms;
    out->pairs = (int64_t)h.natoms * (h.natoms + 1) / 2;
    out->sig_pairs = h.sig_pairs;
    out->quartets = (int64_t)h.quartets;
    out->work_items = h.items;
    out->strategy = h.strategy;
    out->groups = h.groups;
    out->precision = h.precision;
    out->variant = h.variant;
    return HFK_OK;
}

// hfk_fock_grad and hfk_fock_grad_atoms (atoms: exps/coefs are per-atom rows).
static hfk_status fock_grad_impl(bool atoms, int64_t natoms, const double *xyz, int32_t ngauss,
                                 const double *exps_host, const double *coefs_host, const double *dens, double tau,
                                 int32_t precision, const double *g_e2, const double *g_fock, const double *fock_in,
                                 double *d_xyz, double *d_dens, double *e2_out, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    if (atoms) {
        s = check_rows(natoms, ngauss, exps_host, coefs_host);
        if (s != HFK_OK) return s;
    }
    if (!g_e2) return fail(HFK_EINVAL, "g_e2 is NULL");
    if (!d_xyz) return fail(HFK_EINVAL, "d_xyz is NULL");
    if (d_dens && !fock_in) return fail(HFK_EINVAL, "d_dens needs fock_in");
    if (!workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (natoms > kMaxGradAtoms)
        return fail(HFK_EUNSUPPORTED, "gradient supports natoms <= %lld", (long long)kMaxGradAtoms);
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    Layout L = make_layout(natoms, ngauss, precision, 1, groups_cap(cus), atoms);
    if (workspace_bytes < L.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
    L.groups = cus * kGradGroupsPerCU;
    const int fwd_tile = L.tile;
    L.tile = kGradTileItems;   // the gradient kernel's blocks (the pull-back build below uses fwd_tile)
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    Basis b;
    if (atoms) {
        const hipError_t eu = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
        if (eu != hipSuccess) return hip_fail(eu, "basis rows copy");
    } else {
        b = make_basis(ngauss, exps_host, coefs_host);
    }
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (float *)(ws + L.boys_f),
                                (double *)(ws + L.boys_g), (float *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr),
                                natoms, xyz, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = launch_pairs(L, b, ws, xyz, dens, tau, st);
    if (e != hipSuccess) return hip_fail(e, "pair launch");
    const int64_t n2 = natoms * natoms;
    double *xw = (double *)(ws + L.xw);
    if (g_fock) {
        e = launch_make_xw(natoms, dens, g_fock, g_e2, xw, st);
        if (e != hipSuccess) return hip_fail(e, "W/X launch");
    }
    e = launch_grad(L, b, ws, xyz, dens, tau, precision, g_e2, g_fock ? xw + n2 : nullptr, fock_in, d_xyz,
                    g_fock ? nullptr : d_dens, e2_out, st);
    if (e != hipSuccess) return hip_fail(e, "gradient launch");
    if (g_fock && d_dens) {
        // d_dens = G(W) + g_e2 G: a Fock build with W as the density (the pair tables are
        // rebuilt around W; the screen depends on the geometry only), then the axpy
        Layout LW = L;
        LW.tile = fwd_tile;
        e = launch_pairs(LW, b, ws, xyz, xw, tau, st);
        if (e != hipSuccess) return hip_fail(e, "pair launch (W)");
        TunedConfig cfg = pick_config(HFK_STRATEGY_AUTO, precision, natoms, ngauss);
        if (atoms) cfg.variant = 1;   // per-atom bases run the hybrid form only
        int strat = cfg.strategy;
        if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
        Layout LF = LW;
        const int fit = fock_resident_groups(ngauss, precision, cfg.variant, natoms, atoms);
        LF.groups = cus * (fit > 0 && cfg.gpc > fit ? fit : cfg.gpc);
        e = launch_fock(LF, b, ws, xw, tau, precision, strat, cfg.variant, d_dens, (double *)(ws + L.e2tmp), st);
        if (e != hipSuccess) return hip_fail(e, "Fock launch (W)");
        e = launch_axpy_dev(n2, g_e2, fock_in, d_dens, st);
        if (e != hipSuccess) return hip_fail(e, "axpy launch");
    }
    e = launch_header_info(ws + L.hdr, 0, L.groups, precision, -1, st);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    return HFK_OK;
}

hfk_status hfk_fock_grad(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                         const double *coefs_host, const double *dens, double tau, int32_t precision,
                         const double *g_e2, const double *g_fock, const double *fock_in, double *d_xyz,
                         double *d_dens, double *e2_out, void *workspace, size_t workspace_bytes, void *stream)
{
    return fock_grad_impl(false, natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision, g_e2, g_fock,
                          fock_in, d_xyz, d_dens, e2_out, workspace, workspace_bytes, stream);
}

hfk_status hfk_fock_grad_atoms(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                               const double *coefs_host, const double *dens, double tau, int32_t precision,
                               const double *g_e2, const double *g_fock, const double *fock_in, double *d_xyz,
                               double *d_dens, double *e2_out, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    return fock_grad_impl(true, natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision, g_e2, g_fock,
                          fock_in, d_xyz, d_dens, e2_out, workspace, workspace_bytes, stream);
}

static hfk_status check_batch(int64_t nmol, const int64_t *atom_off)
{
    if (nmol < 1) return fail(HFK_EINVAL, "nmol must be >= 1 (got %lld)", (long long)nmol);
    if (!atom_off) return fail(HFK_EINVAL, "atom_off_host is NULL");
    if (atom_off[0] != 0) return fail(HFK_EINVAL, "atom_off_host[0] must be 0");
    for (int64_t m = 0; m < nmol; ++m) {
        const int64_t n = atom_off[m + 1] - atom_off[m];
        if (n < 1) return fail(HFK_EINVAL, "molecule %lld has %lld atoms (needs >= 1)", (long long)m, (long long)n);
        if (n > kMaxBatchAtomsApi)
            return fail(HFK_EUNSUPPORTED, "molecule %lld has %lld atoms; the batched path holds at most %d",
                        (long long)m, (long long)n, kMaxBatchAtomsApi);
    }
    return HFK_OK;
}

static hfk_status batched_ws_impl(bool atoms, int64_t nmol, const int64_t *atom_off_host, int32_t ngauss,
                                  int32_t precision, int32_t with_grad, size_t *bytes_out)
{
    g_err[0] = 0;
    if (!bytes_out) return fail(HFK_EINVAL, "bytes_out is NULL");
    if (ngauss < 1 || ngauss > HFK_MAX_NGAUSS)
        return fail(HFK_EINVAL, "ngauss must be in [1, %d] (got %d)", HFK_MAX_NGAUSS, (int)ngauss);
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    hfk_status s = check_batch(nmol, atom_off_host);
    if (s != HFK_OK) return s;
    *bytes_out = make_blayout(nmol, atom_off_host, ngauss, with_grad, atoms).total;
    return HFK_OK;
}

hfk_status hfk_batched_workspace_bytes(int64_t nmol, const int64_t *atom_off_host, int32_t ngauss,
                                       int32_t precision, int32_t with_grad, size_t *bytes_out)
{
    return batched_ws_impl(false, nmol, atom_off_host, ngauss, precision, with_grad, bytes_out);
}

hfk_status hfk_batched_workspace_bytes_atoms(int64_t nmol, const int64_t *atom_off_host, int32_t ngauss,
                                             int32_t precision, int32_t with_grad, size_t *bytes_out)
{
    return batched_ws_impl(true, nmol, atom_off_host, ngauss, precision, with_grad, bytes_out);
}

// hfk_fock_batched and hfk_fock_batched_atoms (atoms: exps/coefs are per-atom rows over the
// stacked atoms of the batch).
static hfk_status fock_batched_impl(bool atoms, int64_t nmol, const int64_t *atom_off_host, const double *xyz,
                                    int32_t ngauss, const double *exps_host, const double *coefs_host,
                                    const double *dens_packed, double tau, int32_t precision, double *fock_packed,
                                    double *e2, double *d_xyz, void *workspace, size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    hfk_status s = check_batch(nmol, atom_off_host);
    if (s != HFK_OK) return s;
    s = check_common(atom_off_host[nmol], xyz, ngauss, exps_host, coefs_host, dens_packed, tau, precision);
    if (s != HFK_OK) return s;
    if (atoms) {
        s = check_rows(atom_off_host[nmol], ngauss, exps_host, coefs_host);
        if (s != HFK_OK) return s;
    }
    if (!fock_packed) return fail(HFK_EINVAL, "fock_packed is NULL");
    if (!e2) return fail(HFK_EINVAL, "e2 is NULL");
    if (!workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const BLayout L = make_blayout(nmol, atom_off_host, ngauss, d_xyz != nullptr, atoms);
    if (workspace_bytes < L.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    Basis b;
    if (atoms) {
        const hipError_t eu = upload_rows((double *)(ws + L.arow), atom_off_host[nmol], ngauss, exps_host,
                                          coefs_host, st, &b);
        if (eu != hipSuccess) return hip_fail(eu, "basis rows copy");
    } else {
        b = make_basis(ngauss, exps_host, coefs_host);
    }
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (float *)(ws + L.boys_f),
                                (double *)(ws + L.boys_g), (float *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr),
                                atom_off_host[nmol], xyz, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    const int gpc = g_cfg_batch_gpc > 0 ? g_cfg_batch_gpc : g_tuned_batch_gpc > 0 ? g_tuned_batch_gpc : 2;
    e = launch_batched(L, b, ws, atom_off_host, xyz, dens_packed, tau, precision, fock_packed, e2, d_xyz, cus * gpc, st);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    e = launch_header_info(ws + L.hdr, 0, cus * gpc, precision, -1, st);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    return HFK_OK;
}

hfk_status hfk_fock_batched(int64_t nmol, const int64_t *atom_off_host, const double *xyz, int32_t ngauss,
                            const double *exps_host, const double *coefs_host, const double *dens_packed,
                            double tau, int32_t precision, double *fock_packed, double *e2, double *d_xyz,
                            void *workspace, size_t workspace_bytes, void *stream)
{
    return fock_batched_impl(false, nmol, atom_off_host, xyz, ngauss, exps_host, coefs_host, dens_packed, tau,
                             precision, fock_packed, e2, d_xyz, workspace, workspace_bytes, stream);
}

hfk_status hfk_fock_batched_atoms(int64_t nmol, const int64_t *atom_off_host, const double *xyz, int32_t ngauss,
                                  const double *exps_host, const double *coefs_host, const double *dens_packed,
                                  double tau, int32_t precision, double *fock_packed, double *e2, double *d_xyz,
                                  void *workspace, size_t workspace_bytes, void *stream)
{
    return fock_batched_impl(true, nmol, atom_off_host, xyz, ngauss, exps_host, coefs_host, dens_packed, tau,
                             precision, fock_packed, e2, d_xyz, workspace, workspace_bytes, stream);
}

// ------------------------------------------------------------------ autotuner

static double time_fock_ms(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps,
                           const double *coefs, const double *dens, double tau, int32_t precision, int32_t strategy,
                           double *fock, double *e2, void *ws, size_t wsb, hipStream_t st, int reps, hfk_status *err)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        *err = fail(HFK_EHIP, "event create");
        return 0.0;
    }
    double best = 1e300;
    for (int r = 0; r <= reps; ++r) {
        (void)hipEventRecord(e0, st);
        hfk_status s = hfk_fock(natoms, xyz, ngauss, exps, coefs, dens, tau, precision, strategy, fock, e2, ws, wsb, st);
        (void)hipEventRecord(e1, st);
        if (s != HFK_OK) {
            *err = s;
            break;
        }
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            *err = fail(HFK_EHIP, "event timing");
            break;
        }
        if (r > 0 && ms < best) best = ms;     // the first run warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

static hfk_status write_tuning(const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f) return fail(HFK_EINVAL, "cannot write %s", path);
    fprintf(f, "{\n  \"format\": \"hfk-tuning-1\",\n  \"entries\": [\n");
    bool first = true;
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < 4; ++c) {
            const TunedConfig &t = g_tuned_cfg[p][c];
            if (!t.strategy) continue;
            fprintf(f, "%s    {\"precision\": %d, \"size_class\": %d, \"strategy\": %d, \"variant\": %d, \"gpc\": %d}",
                    first ? "" : ",\n", p, c, t.strategy, t.variant, t.gpc);
            first = false;
        }
    fprintf(f, "\n  ],\n  \"batched_gpc\": %d\n}\n", g_tuned_batch_gpc);
    fclose(f);
    return HFK_OK;
}

hfk_status hfk_tune(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                    const double *coefs_host, const double *dens, double tau, int32_t precision, double *fock,
                    double *e2, void *workspace, size_t workspace_bytes, void *stream, const char *cache_path,
                    int32_t *best_out)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    const int save_var = g_cfg_variant, save_gpc = g_cfg_gpc;
    const int strategies[2] = {HFK_STRATEGY_PRIVATE, HFK_STRATEGY_ATOMIC};
    const int variants[2] = {1, 0};
    const int gpcs[4] = {3, 4, 5, 6};
    TunedConfig best{0, 1, 2};
    double best_ms = 1e300;
    hfk_status err = HFK_OK;
    for (int si = 0; si < 2 && err == HFK_OK; ++si)
        for (int vi = 0; vi < (ngauss > 4 ? 1 : 2) && err == HFK_OK; ++vi)
            for (int gi = 0; gi < 4 && err == HFK_OK; ++gi) {
                g_cfg_variant = variants[vi];
                g_cfg_gpc = gpcs[gi];
                const double ms = time_fock_ms(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision,
                                               strategies[si], fock, e2, workspace, workspace_bytes,
                                               (hipStream_t)stream, 2, &err);
                if (err == HFK_OK && ms < best_ms) {
                    best_ms = ms;
                    best = TunedConfig{strategies[si], variants[vi], gpcs[gi]};
                }
            }
    g_cfg_variant = save_var;
    g_cfg_gpc = save_gpc;
    if (err != HFK_OK) return err;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned_cfg[precision][size_class(natoms)] = best;
    }
    if (best_out) *best_out = best.strategy;
    if (cache_path) return write_tuning(cache_path);
    return HFK_OK;
}

hfk_status hfk_tune_batched(int64_t nmol, const int64_t *atom_off_host, const double *xyz, int32_t ngauss,
                            const double *exps_host, const double *coefs_host, const double *dens_packed, double tau,
                            int32_t precision, double *fock_packed, double *e2, double *d_xyz, void *workspace,
                            size_t workspace_bytes, void *stream, const char *cache_path, int32_t *best_gpc_out)
{
    g_err[0] = 0;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(HFK_EHIP, "event create");
    const int save = g_cfg_batch_gpc;
    int best = 2;
    double best_ms = 1e300;
    hfk_status err = HFK_OK;
    for (int gpc = 1; gpc <= 3 && err == HFK_OK; ++gpc) {
        g_cfg_batch_gpc = gpc;
        for (int r = 0; r < 3 && err == HFK_OK; ++r) {
            (void)hipEventRecord(e0, st);
            err = hfk_fock_batched(nmol, atom_off_host, xyz, ngauss, exps_host, coefs_host, dens_packed, tau,
                                   precision, fock_packed, e2, d_xyz, workspace, workspace_bytes, stream);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (err == HFK_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                err = fail(HFK_EHIP, "event timing");
            if (err == HFK_OK && r > 0 && ms < best_ms) {
                best_ms = ms;
                best = gpc;
            }
        }
    }
    g_cfg_batch_gpc = save;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != HFK_OK) return err;
    g_tuned_batch_gpc = best;
    if (best_gpc_out) *best_gpc_out = best;
    if (cache_path) return write_tuning(cache_path);
    return HFK_OK;
}

static bool json_int(const char *obj, const char *key, int *out)
{
    char pat[64];
    snprintf(pat, sizeof(pat), "\"%s\"", key);
    const char *p = strstr(obj, pat);
    if (!p) return false;
    p = strchr(p + strlen(pat), ':');
    if (!p) return false;
    return sscanf(p + 1, " %d", out) == 1;
}

hfk_status hfk_load_tuning(const char *cache_path)
{
    g_err[0] = 0;
    if (!cache_path) return fail(HFK_EINVAL, "cache_path is NULL");
    FILE *f = fopen(cache_path, "r");
    if (!f) return fail(HFK_EINVAL, "cannot read %s", cache_path);
    std::vector<char> buf;
    char tmp[4096];
    size_t got;
    while ((got = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    fclose(f);
    buf.push_back(0);
    const char *txt = buf.data();
    if (!strstr(txt, "\"hfk-tuning-1\"")) return fail(HFK_EINVAL, "%s is not an hfk tuning table", cache_path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const char *p = strchr(txt, '{'); p; p = strchr(p + 1, '{')) {
        const char *end = strchr(p, '}');
        if (!end) break;
        std::string obj(p, end - p + 1);
        int prec, cls, strat, var, gpc;
        if (json_int(obj.c_str(), "precision", &prec) && json_int(obj.c_str(), "size_class", &cls) &&
            json_int(obj.c_str(), "strategy", &strat) && json_int(obj.c_str(), "variant", &var) &&
            json_int(obj.c_str(), "gpc", &gpc)) {
            if (prec < 0 || prec > 1 || cls < 0 || cls > 3 || strat < 1 || strat > 2 || var < 0 || var > 1 ||
                gpc < 1 || gpc > kMaxGroupsPerCU)
                return fail(HFK_EINVAL, "bad entry in %s", cache_path);
            g_tuned_cfg[prec][cls] = TunedConfig{strat, var, gpc};
        }
    }
    int bg = 0;
    if (json_int(txt, "batched_gpc", &bg) && bg >= 1 && bg <= 3) g_tuned_batch_gpc = bg;
    return HFK_OK;
}

}  // extern "C"
