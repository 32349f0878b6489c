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

static double bits_to_double(unsigned long long b)
{
    double d;
    memcpy(&d, &b, sizeof(d));
    return d;
}

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

Layout make_layout(int64_t n, int g, int prec, int with_grad, int groups, bool atoms, bool compact)
{
    Layout L;
    memset(&L, 0, sizeof(L));
    L.n = n;
    L.atoms = atoms;
    L.tile = prec == HFK_MIXED ? 2 * kTileItems : kTileItems;
    L.gshift = 10;   // kGroupBras
    L.kcopies = 0;
    L.private_ok = !compact && (double)groups * (double)n * (double)n * 8.0 <= kPrivateBudget;
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
    L.boys_f = take(sizeof(double) * kBoysGridF * kBoysStrideF);
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
        }
    }
    if (with_grad) {
        L.bgw = take(sizeof(double) * kGW * g2 * PC);
        L.bgw_f = take(sizeof(float) * kGW * g2 * PC);
    }
    L.bra = take(sizeof(double) * 8 * g2 * PC);
    L.bra_f = take(sizeof(float) * 8 * g2 * PC);
    L.boys_g = take(sizeof(double) * kBoysGrid * kBoysStrideG);
    L.boys_g_f = take(sizeof(double) * kBoysGridF * kBoysStrideF);
    L.nitems = take(sizeof(long long) * PC);
    L.lim = take(sizeof(int) * PC);
    L.item_off = take(sizeof(long long) * (PC + 1));
    L.ngroups = (L.pcap + kGroupBras - 1) / kGroupBras;
    L.ngroups_cap = (L.pcap + kMinGroupBras - 1) / kMinGroupBras;
    L.gcnt = take(sizeof(long long) * (size_t)(L.ngroups_cap + 1));
    L.goff = take(sizeof(long long) * (size_t)(L.ngroups_cap + 1));
    L.scan_tmp = take(sizeof(long long) * (((PC > (size_t)kNumBuckets ? PC : (size_t)kNumBuckets) + 1023) / 1024 + 1));
    const size_t n2 = (size_t)(n * n);
    L.fpriv = take(sizeof(double) * n2 * (size_t)(L.private_ok ? groups : 1));
    {
        const double fit = kJcolBudget / (8.0 * (double)PC);
        L.jcopies = fit >= (double)groups ? groups : (fit >= 1.0 ? (int)fit : 1);
        if (compact && L.jcopies > kCompactKetCopies) L.jcopies = kCompactKetCopies;
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

void set_shape(Layout &L, int tile, int group_bras, int ket_copies)
{
    L.tile = tile;
    int sh = 0;
    while ((1 << sh) < group_bras) ++sh;
    L.gshift = sh;
    L.ngroups = (L.pcap + (1LL << sh) - 1) >> sh;
    L.kcopies = ket_copies;
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
// n above which the gradient kernel's LDS copy of dE2/dR (n x 3) and its Boys tables no longer fit
constexpr int64_t kMaxGradAtoms = 4096;
constexpr int kGradGroupsPerCU = 4;
constexpr int kDefaultKetCopies = 8;   // untuned default: shared ket-side Coulomb vectors
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
// Pairs of all molecules of a batch: the ket table's buffer resources cover G rows of
// pcap values (G <= 6 FP64: 48 bytes per pair), which must stay below 2^31 bytes.
constexpr int64_t kMaxBatchPairs = 40000000;
constexpr int kMaxBatchGroupsPerCU = 4;

// ------------------------------------------------------------------ launch configuration

// One launch configuration of the single-molecule forward build.
struct TunedConfig {
    int strategy;      // 0 = not set
    int variant;
    int gpc;           // persistent workgroups per CU
    int tile;          // items per block
    int gbras;         // bras per group
    int kcopies;       // ket-side Coulomb vectors (0: one per workgroup)
};

// One launch configuration of the batched path.
struct BatchedConfig {
    int gpc;                // 0 = not set
    int block_items;        // 0 = automatic
    long long owned_bound;  // -1 = no owned molecules
    int waves;              // waves per workgroup: 4 or 8
};

// Size bucket of the tuning table: ceil(log2 n).
static int size_bucket(int64_t n)
{
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

// Architecture name of the current device (gcnArchName up to the first ':'), cached per device.
static std::string device_arch()
{
    static std::mutex mu;
    static std::vector<std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    if ((int)names.size() <= dev) names.resize(dev + 1);
    if (names[dev].empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
        std::string a(prop.gcnArchName);
        const size_t c = a.find(':');
        names[dev] = c == std::string::npos ? a : a.substr(0, c);
    }
    return names[dev];
}

struct TuneEntry {
    std::string arch;
    int precision;
    int bucket;
    TunedConfig cfg;
};
struct BatchedEntry {
    std::string arch;
    int precision;
    BatchedConfig cfg;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tuned;
static std::vector<BatchedEntry> g_tuned_b;

// Process-wide overrides (hfk_set_config, hfk_set_shape, hfk_set_batched_config).
static int g_cfg_tile = 0, g_cfg_gbras = 0, g_cfg_kcopies = -1;
static BatchedConfig g_cfg_b{0, 0, 0, 0};
// The candidate being timed by a tuner on this thread (takes precedence over everything).
static thread_local const TunedConfig *g_force = nullptr;
static thread_local const BatchedConfig *g_force_b = nullptr;

// The configuration before any tuning.  Timed over whole calls (side kernels included) on
// MI355X for He 64 to 1024 and H/He 128, FP64 and mixed: ATOMIC was the faster strategy at
// every size (the per-workgroup copies of F and their summation cost more than the atomics
// they save), and small systems ran fastest with fewer workgroups per CU (2 at 64 atoms,
// 4 at 128, the most that fit above).  Blocks of four items of 1024 kets (eight with the
// FP32 ket table, half the size), groups of 1024 bras, one ket vector per workgroup.
static TunedConfig default_config(int64_t n, int precision)
{
    // eight shared ket-side Coulomb vectors: they stay cached where one per workgroup does
    // not (he512 FP64 68.0 against 69.2 ms, he1024 mixed 210.0 against 221.2 ms, he128 2.12
    // against 2.19 ms)
    return TunedConfig{HFK_STRATEGY_ATOMIC, 1, n <= 64 ? 2 : (n <= 128 ? 4 : 6),
                       precision == HFK_MIXED ? 2 * kTileItems : kTileItems, kGroupBras, kDefaultKetCopies};
}

// Before tuning: eight-wave workgroups, two per CU (the LDS holds two molecules' triangles
// up to 96 atoms), automatic block size, every molecule in shared blocks.
static BatchedConfig default_batched_config() { return BatchedConfig{2, 0, -1, 8}; }

static bool lookup_tuned(const std::string &arch, int precision, int bucket, TunedConfig *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry &e : g_tuned)
        if (e.arch == arch && e.precision == precision && e.bucket == bucket) {
            *out = e.cfg;
            return true;
        }
    return false;
}

static TunedConfig pick_config(int32_t strategy, int32_t precision, int64_t n, int32_t ngauss)
{
    TunedConfig c = default_config(n, precision);
    if (g_force) {
        c = *g_force;
    } else {
        TunedConfig t;
        if (lookup_tuned(device_arch(), precision, size_bucket(n), &t)) c = t;
        if (strategy == HFK_STRATEGY_PRIVATE || strategy == HFK_STRATEGY_ATOMIC) c.strategy = strategy;
        if (g_cfg_variant >= 0) c.variant = g_cfg_variant;
        if (g_cfg_gpc > 0) c.gpc = g_cfg_gpc;
        if (g_cfg_tile > 0) c.tile = g_cfg_tile;
        if (g_cfg_gbras > 0) c.gbras = g_cfg_gbras;
        if (g_cfg_kcopies >= 0) c.kcopies = g_cfg_kcopies;
    }
    if (ngauss > 4) c.variant = 1;   // the direct form is built for g <= 4 only
    if (strategy == HFK_STRATEGY_DETERMINISTIC) {
        // a fixed configuration, independent of tuning and overrides (capped at residency)
        c = TunedConfig{HFK_STRATEGY_DETERMINISTIC, 1, kMaxGroupsPerCU,
                        precision == HFK_MIXED ? 2 * kTileItems : kTileItems, kGroupBras, 0};
    }
    return c;
}

static BatchedConfig pick_batched_config(int32_t precision)
{
    BatchedConfig c = default_batched_config();
    if (g_force_b) return *g_force_b;
    {
        const std::string arch = device_arch();
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const BatchedEntry &e : g_tuned_b)
            if (e.arch == arch && e.precision == precision) c = e.cfg;
    }
    if (g_cfg_b.gpc > 0) c.gpc = g_cfg_b.gpc;
    if (g_cfg_b.block_items > 0) c.block_items = g_cfg_b.block_items;
    if (g_cfg_b.owned_bound != 0) c.owned_bound = g_cfg_b.owned_bound;
    if (g_cfg_b.waves > 0) c.waves = g_cfg_b.waves;
    return c;
}

// ------------------------------------------------------------------ debug mode

static bool g_debug = false;
static double g_debug_tol = 0.0;

// Debug check of one n x n density (hfk_set_debug): waits for the stream.
static hfk_status debug_check(char *ws_hdr, int64_t n, const double *dens, hipStream_t st, const char *what)
{
    if (!g_debug) return HFK_OK;
    DevHeader *hdr = (DevHeader *)ws_hdr;
    hipError_t e = launch_dens_check(hdr, n, dens, st);
    DevHeader h;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, hdr, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "density check");
    if (h.dchk_bad) return fail(HFK_EINVAL, "%s has %llu non-finite entries", what, (unsigned long long)h.dchk_bad);
    const double asym = bits_to_double(h.dchk_asym);
    const double mx = bits_to_double(h.dchk_max);
    if (asym > g_debug_tol * mx)
        return fail(HFK_ENOTSYM, "%s is not symmetric: max |D_ij - D_ji| = %.3e, max |D_ij| = %.3e, tolerance %.3e",
                    what, asym, mx, g_debug_tol);
    return HFK_OK;
}

// ------------------------------------------------------------------ static scratch

// Scratch of the allocation-free entry point (hfk_fock_noalloc): device memory that every
// GPU the library runs on holds from module load until the process ends.  In host code the
// array's name is only a stand-in; its device address comes from hipGetSymbolAddress, once
// per device with that device current, and only that address is ever passed to kernels or
// copies.  Every call on a GPU shares that GPU's copy: calls that overlap in time on one GPU
// race, and each call clears what it needs (counters, accumulators) before use.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;   // per device

static hfk_status static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (uintptr_t)p % 256 != 0) return fail(HFK_EHIP, "static scratch has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HFK_OK;
}

// ------------------------------------------------------------------ last build of this thread

static thread_local const void *g_last_ws = nullptr;
static thread_local void *g_last_stream = nullptr;

static void note_last(const void *ws, void *stream)
{
    g_last_ws = ws;
    g_last_stream = stream;
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

}  // extern "C"

// hfk_fock, and (compact) hfk_fock_noalloc: the workspace is then the static scratch, laid
// out for the atomics strategy with a few shared ket vectors.
static hfk_status fock_one_basis(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                                 const double *coefs_host, const double *dens, double tau, int32_t precision,
                                 int32_t strategy, double *fock, double *e2, void *workspace, size_t workspace_bytes,
                                 void *stream, bool compact)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    if (!fock) return fail(HFK_EINVAL, "fock is NULL");
    if (!e2) return fail(HFK_EINVAL, "e2 is NULL");
    if (!compact && !workspace) return fail(HFK_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(HFK_EINVAL, "workspace must be 256-byte aligned");
    if (strategy < HFK_STRATEGY_AUTO || strategy > HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EINVAL, "unknown strategy %d", (int)strategy);
    if (strategy == HFK_STRATEGY_DETERMINISTIC && natoms > kMaxDetAtoms)
        return fail(HFK_EUNSUPPORTED, "the deterministic strategy supports natoms <= %lld", (long long)kMaxDetAtoms);
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    if (ngauss > kMaxBuiltG) return fail(HFK_EUNSUPPORTED, "ngauss above %d is not built in this version", kMaxBuiltG);
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    Layout L = make_layout(natoms, ngauss, precision, 0, groups_cap(cus), false, compact);
    if (compact) {
        if (L.total > kStaticScratchBytes)
            return fail(HFK_EUNSUPPORTED,
                        "this system needs %zu bytes of scratch; the allocation-free call holds %zu (about 256 atoms "
                        "with 3 primitives per function)",
                        L.total, kStaticScratchBytes);
        s = static_scratch(&workspace);
        if (s != HFK_OK) return s;
        workspace_bytes = kStaticScratchBytes;
    }
    if (workspace_bytes < L.total)
        return fail(HFK_ENOMEM, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
    TunedConfig cfg = pick_config(strategy, precision, natoms, ngauss);
    if (compact) {
        // the scratch is laid out for atomics and the layout's shared ket vectors
        cfg.strategy = HFK_STRATEGY_ATOMIC;
        cfg.kcopies = 0;
    }
    int strat = cfg.strategy;
    if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
    set_shape(L, cfg.tile, cfg.gbras, cfg.kcopies);
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
    s = debug_check(ws + L.hdr, natoms, dens, st, "dens");
    if (s != HFK_OK) return s;
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys),
                                (double *)(ws + L.boys_f), (double *)(ws + L.boys_g),
                                (double *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = launch_pairs(L, b, ws, xyz, dens, tau, st, strat == HFK_STRATEGY_DETERMINISTIC);
    if (e == hipErrorNotSupported && strat == HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EUNSUPPORTED, "deterministic strategy: more than %d pairs share one (Q band, cell) bucket",
                    kMaxFixedBucket);
    if (e != hipSuccess) return hip_fail(e, "pair launch");
    e = launch_fock(L, b, ws, dens, tau, precision, strat, cfg.variant, fock, e2, st);
    if (e != hipSuccess) return hip_fail(e, "fock launch");
    e = launch_header_info(ws + L.hdr, strat, L.groups, precision, cfg.variant, st, L.tile, 1 << L.gshift,
                           effective_copies(L));
    if (e != hipSuccess) return hip_fail(e, "header launch");
    note_last(workspace, stream);
    return HFK_OK;
}

extern "C" {

hfk_status hfk_fock(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                    const double *coefs_host, const double *dens, double tau, int32_t precision,
                    int32_t strategy, double *fock, double *e2, void *workspace, size_t workspace_bytes,
                    void *stream)
{
    return fock_one_basis(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision, strategy, fock, e2,
                          workspace, workspace_bytes, stream, false);
}

hfk_status hfk_fock_noalloc(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                            const double *coefs_host, const double *dens, double tau, int32_t precision,
                            double *fock, double *e2, void *stream)
{
    return fock_one_basis(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision, HFK_STRATEGY_ATOMIC,
                          fock, e2, nullptr, 0, stream, true);
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
    set_shape(L, cfg.tile, cfg.gbras, cfg.kcopies);
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
    s = debug_check(ws + L.hdr, natoms, dens, st, "dens");
    if (s != HFK_OK) return s;
    Basis b;
    hipError_t e = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
    if (e != hipSuccess) return hip_fail(e, "basis rows copy");
    e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (double *)(ws + L.boys_f),
                     (double *)(ws + L.boys_g), (double *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz,
                     st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = launch_pairs(L, b, ws, xyz, dens, tau, st, strat == HFK_STRATEGY_DETERMINISTIC);
    if (e == hipErrorNotSupported && strat == HFK_STRATEGY_DETERMINISTIC)
        return fail(HFK_EUNSUPPORTED, "deterministic strategy: more than %d pairs share one (Q band, cell) bucket",
                    kMaxFixedBucket);
    if (e != hipSuccess) return hip_fail(e, "pair launch");
    e = launch_fock(L, b, ws, dens, tau, precision, strat, 1, fock, e2, st);
    if (e != hipSuccess) return hip_fail(e, "fock launch");
    e = launch_header_info(ws + L.hdr, strat, L.groups, precision, 1, st, L.tile, 1 << L.gshift,
                           effective_copies(L));
    if (e != hipSuccess) return hip_fail(e, "header launch");
    note_last(workspace, stream);
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
    set_shape(L, cfg.tile, cfg.gbras, cfg.kcopies);
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
    if (use_guess) {
        s = debug_check(ws + L.hdr, natoms, dens, st, "guess density");
        if (s != HFK_OK) return s;
    }
    Basis b;
    hipError_t e = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
    if (e != hipSuccess) return hip_fail(e, "basis rows copy");
    e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (double *)(ws + L.boys_f),
                     (double *)(ws + L.boys_g), (double *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr), natoms, xyz,
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
    out->tile_items = h.tile;
    out->group_bras = h.group_bras;
    out->ket_copies = h.ket_copies;
    return HFK_OK;
}

hfk_status hfk_last_stats(hfk_stats *out)
{
    if (!out) return fail(HFK_EINVAL, "out is NULL");
    if (!g_last_ws) return fail(HFK_EINVAL, "no build call has been made on this thread");
    return hfk_read_stats(g_last_ws, g_last_stream, out);
}

hfk_status hfk_set_debug(int32_t on, double sym_tol)
{
    g_err[0] = 0;
    if (!isfinite(sym_tol) || sym_tol < 0.0)
        return fail(HFK_EINVAL, "sym_tol must be finite and >= 0 (got %g)", sym_tol);
    g_debug = on != 0;
    g_debug_tol = sym_tol;
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
    {
        // as many persistent workgroups as fit on a CU, up to kGradGroupsPerCU (or the count
        // hfk_set_config asks for)
        const int fit = grad_resident_groups(ngauss, precision, natoms, atoms);
        const int want = g_cfg_gpc > 0 ? g_cfg_gpc : kGradGroupsPerCU;
        L.groups = cus * (fit > 0 && fit < want ? fit : want);
    }
    // the gradient kernel's blocks: eight items, groups of 1024 bras, unless hfk_set_shape
    // asks for another shape (the pull-back build below takes the forward's shape)
    set_shape(L, g_cfg_tile > 0 ? g_cfg_tile : kGradTileItems, g_cfg_gbras > 0 ? g_cfg_gbras : kGroupBras, 0);
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    s = debug_check(ws + L.hdr, natoms, dens, st, "dens");
    if (s != HFK_OK) return s;
    Basis b;
    if (atoms) {
        const hipError_t eu = upload_rows((double *)(ws + L.arow), natoms, ngauss, exps_host, coefs_host, st, &b);
        if (eu != hipSuccess) return hip_fail(eu, "basis rows copy");
    } else {
        b = make_basis(ngauss, exps_host, coefs_host);
    }
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (double *)(ws + L.boys_f),
                                (double *)(ws + L.boys_g), (double *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr),
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
        TunedConfig cfg = pick_config(HFK_STRATEGY_AUTO, precision, natoms, ngauss);
        if (atoms) cfg.variant = 1;   // per-atom bases run the hybrid form only
        int strat = cfg.strategy;
        if (strat == HFK_STRATEGY_PRIVATE && !L.private_ok) strat = HFK_STRATEGY_ATOMIC;
        Layout LW = L;
        set_shape(LW, cfg.tile, cfg.gbras, cfg.kcopies);
        e = launch_pairs(LW, b, ws, xyz, xw, tau, st);
        if (e != hipSuccess) return hip_fail(e, "pair launch (W)");
        Layout LF = LW;
        const int fit = fock_resident_groups(ngauss, precision, cfg.variant, natoms, atoms);
        LF.groups = cus * (fit > 0 && cfg.gpc > fit ? fit : cfg.gpc);
        e = launch_fock(LF, b, ws, xw, tau, precision, strat, cfg.variant, d_dens, (double *)(ws + L.e2tmp), st);
        if (e != hipSuccess) return hip_fail(e, "Fock launch (W)");
        e = launch_axpy_dev(n2, g_e2, fock_in, d_dens, st);
        if (e != hipSuccess) return hip_fail(e, "axpy launch");
    }
    e = launch_header_info(ws + L.hdr, 0, L.groups, precision, -1, st, L.tile, 1 << L.gshift, 0);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    note_last(workspace, stream);
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
    int64_t pairs = 0;
    for (int64_t m = 0; m < nmol; ++m) {
        const int64_t n = atom_off[m + 1] - atom_off[m];
        pairs += n * (n + 1) / 2;
    }
    if (pairs > kMaxBatchPairs)
        return fail(HFK_EUNSUPPORTED, "the batch has %lld atom pairs; one call holds at most %lld",
                    (long long)pairs, (long long)kMaxBatchPairs);
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
    hipError_t e = launch_setup(b, (BasisDev *)(ws + L.basis), (double *)(ws + L.boys), (double *)(ws + L.boys_f),
                                (double *)(ws + L.boys_g), (double *)(ws + L.boys_g_f), (DevHeader *)(ws + L.hdr),
                                atom_off_host[nmol], xyz, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    e = upload_batch_tables(L, ws, atom_off_host, st);
    if (e != hipSuccess) return hip_fail(e, "batch tables copy");
    if (g_debug) {
        DevHeader *hdr = (DevHeader *)(ws + L.hdr);
        e = launch_dens_check_batched(hdr, nmol, (const long long *)(ws + L.mol_doff), (const int *)(ws + L.mol_n),
                                      dens_packed, g_debug_tol, st);
        DevHeader h;
        if (e == hipSuccess) e = hipMemcpyAsync(&h, hdr, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "density check");
        if (h.dchk_bad)
            return fail(HFK_EINVAL, "dens_packed has %llu non-finite entries (first in molecule %d)",
                        (unsigned long long)h.dchk_bad, h.dchk_badmol);
        if (h.dchk_mol != 0x7fffffff)
            return fail(HFK_ENOTSYM,
                        "the density of molecule %d is not symmetric (largest max |D_ij - D_ji| / max |D_ij| over "
                        "the molecules outside the tolerance: %.3e, tolerance %.3e)",
                        h.dchk_mol, bits_to_double(h.dchk_ratio), g_debug_tol);
    }
    const BatchedConfig bc = pick_batched_config(precision);
    int gpc = bc.gpc;
    {
        const int fit = batched_resident_groups(ngauss, precision, d_xyz != nullptr, atoms, L.nmax, bc.waves);
        if (fit > 0 && gpc > fit) gpc = fit;
    }
    const BatchedShape shape{gpc, bc.block_items, bc.owned_bound, bc.waves};
    e = launch_batched(L, b, ws, atom_off_host, xyz, dens_packed, tau, precision, fock_packed, e2, d_xyz, cus * gpc,
                       shape, st);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    e = launch_header_info(ws + L.hdr, 0, cus * gpc, precision, -1, st, -1, 0, 0);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    note_last(workspace, stream);
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

}  // extern "C"

// ------------------------------------------------------------------ autotuner

// Best of `reps` timed calls after one untimed call (HIP events on the stream).
template <typename Call>
static double time_call_ms(Call call, hipStream_t st, int reps, hfk_status *err)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        *err = fail(HFK_EHIP, "event create");
        return 0.0;
    }
    double best = 1e300;
    for (int r = 0; r <= reps; ++r) {
        (void)hipEventRecord(e0, st);
        const hfk_status s = call();
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
        if (r > 0 && ms < best) best = ms;     // the first call warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// A candidate replaces the best so far only when it is faster by more than this fraction
// (back-to-back timings of one configuration agree to about 0.3%).
constexpr double kTuneMargin = 0.005;

static hfk_status write_tuning(const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f) return fail(HFK_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    fprintf(f, "{\n  \"format\": \"hfk-tuning-2\",\n  \"entries\": [\n");
    for (size_t x = 0; x < g_tuned.size(); ++x) {
        const TuneEntry &t = g_tuned[x];
        fprintf(f,
                "    {\"arch\": \"%s\", \"precision\": %d, \"size_bucket\": %d, \"strategy\": %d, \"variant\": %d, "
                "\"gpc\": %d, \"tile_items\": %d, \"group_bras\": %d, \"ket_copies\": %d}%s\n",
                t.arch.c_str(), t.precision, t.bucket, t.cfg.strategy, t.cfg.variant, t.cfg.gpc, t.cfg.tile,
                t.cfg.gbras, t.cfg.kcopies, x + 1 < g_tuned.size() ? "," : "");
    }
    fprintf(f, "  ],\n  \"batched\": [\n");
    for (size_t x = 0; x < g_tuned_b.size(); ++x) {
        const BatchedEntry &t = g_tuned_b[x];
        fprintf(f,
                "    {\"arch\": \"%s\", \"precision\": %d, \"gpc\": %d, \"block_items\": %d, \"owned_bound\": %lld, "
                "\"waves\": %d}%s\n",
                t.arch.c_str(), t.precision, t.cfg.gpc, t.cfg.block_items, t.cfg.owned_bound, t.cfg.waves,
                x + 1 < g_tuned_b.size() ? "," : "");
    }
    fprintf(f, "  ]\n}\n");
    fclose(f);
    return HFK_OK;
}

static void store_tuned(const std::string &arch, int precision, int bucket, const TunedConfig &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TuneEntry &e : g_tuned)
        if (e.arch == arch && e.precision == precision && e.bucket == bucket) {
            e.cfg = c;
            return;
        }
    g_tuned.push_back(TuneEntry{arch, precision, bucket, c});
}

static void store_tuned_b(const std::string &arch, int precision, const BatchedConfig &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (BatchedEntry &e : g_tuned_b)
        if (e.arch == arch && e.precision == precision) {
            e.cfg = c;
            return;
        }
    g_tuned_b.push_back(BatchedEntry{arch, precision, c});
}

extern "C" {

hfk_status hfk_tune(int64_t natoms, const double *xyz, int32_t ngauss, const double *exps_host,
                    const double *coefs_host, const double *dens, double tau, int32_t precision, double *fock,
                    double *e2, void *workspace, size_t workspace_bytes, void *stream, const char *cache_path,
                    int32_t *best_out)
{
    g_err[0] = 0;
    hfk_status s = check_common(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision);
    if (s != HFK_OK) return s;
    if (natoms > kMaxAtoms) return fail(HFK_EUNSUPPORTED, "natoms above %lld", (long long)kMaxAtoms);
    hipStream_t st = (hipStream_t)stream;
    const int cus = device_cu_count();
    if (cus <= 0) return fail(HFK_EHIP, "no HIP device");
    const Layout L0 = make_layout(natoms, ngauss, precision, 0, groups_cap(cus));
    hfk_status err = HFK_OK;
    TunedConfig best = default_config(natoms, precision);
    if (ngauss > 4) best.variant = 1;
    TunedConfig cand;
    auto run = [&]() {
        return hfk_fock(natoms, xyz, ngauss, exps_host, coefs_host, dens, tau, precision, HFK_STRATEGY_AUTO, fock,
                        e2, workspace, workspace_bytes, stream);
    };
    auto timed = [&](const TunedConfig &c) {
        cand = c;
        g_force = &cand;
        const double ms = time_call_ms(run, st, 2, &err);
        g_force = nullptr;
        return ms;
    };
    double best_ms = timed(best);
    // one dimension at a time, each candidate against the best so far
    auto try_dim = [&](auto set, const int *vals, int nv) {
        for (int x = 0; x < nv && err == HFK_OK; ++x) {
            TunedConfig c = best;
            set(c, vals[x]);
            if (memcmp(&c, &best, sizeof(c)) == 0) continue;
            const double ms = timed(c);
            if (err == HFK_OK && ms < best_ms * (1.0 - kTuneMargin)) {
                best_ms = ms;
                best = c;
            }
        }
    };
    const int strategies[2] = {HFK_STRATEGY_ATOMIC, HFK_STRATEGY_PRIVATE};
    const int variants[2] = {1, 0};
    const int gpcs[6] = {1, 2, 3, 4, 5, 6};
    const int tiles[5] = {1, 2, 4, 8, 16};
    const int gbras[5] = {256, 512, 1024, 2048, 4096};
    const int kcopies[3] = {0, 8, 32};
    try_dim([](TunedConfig &c, int v) { c.strategy = v; }, strategies, L0.private_ok ? 2 : 1);
    if (ngauss <= 4) try_dim([](TunedConfig &c, int v) { c.variant = v; }, variants, 2);
    {
        // workgroups per CU up to what fits on a CU (more would only queue)
        const int fit = fock_resident_groups(ngauss, precision, best.variant, natoms, false, false);
        try_dim([](TunedConfig &c, int v) { c.gpc = v; }, gpcs, fit > 0 && fit < 6 ? fit : 6);
    }
    try_dim([](TunedConfig &c, int v) { c.tile = v; }, tiles, 5);
    try_dim([](TunedConfig &c, int v) { c.gbras = v; }, gbras, 5);
    try_dim([](TunedConfig &c, int v) { c.kcopies = v; }, kcopies, 3);
    // the first dimensions again, against the final shape
    try_dim([](TunedConfig &c, int v) { c.gpc = v; }, gpcs, 6);
    try_dim([](TunedConfig &c, int v) { c.tile = v; }, tiles, 5);
    if (err != HFK_OK) return err;
    store_tuned(device_arch(), precision, size_bucket(natoms), best);
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
    if (precision != HFK_FP64 && precision != HFK_MIXED)
        return fail(HFK_EINVAL, "precision must be HFK_FP64 or HFK_MIXED (got %d)", (int)precision);
    hipStream_t st = (hipStream_t)stream;
    hfk_status err = HFK_OK;
    BatchedConfig best = default_batched_config();
    BatchedConfig cand;
    auto run = [&]() {
        return hfk_fock_batched(nmol, atom_off_host, xyz, ngauss, exps_host, coefs_host, dens_packed, tau, precision,
                                fock_packed, e2, d_xyz, workspace, workspace_bytes, stream);
    };
    auto timed = [&](const BatchedConfig &c) {
        cand = c;
        g_force_b = &cand;
        const double ms = time_call_ms(run, st, 2, &err);
        g_force_b = nullptr;
        return ms;
    };
    double best_ms = timed(best);
    auto try_dim = [&](auto set, const long long *vals, int nv) {
        for (int x = 0; x < nv && err == HFK_OK; ++x) {
            BatchedConfig c = best;
            set(c, vals[x]);
            if (memcmp(&c, &best, sizeof(c)) == 0) continue;
            const double ms = timed(c);
            if (err == HFK_OK && ms < best_ms * (1.0 - kTuneMargin)) {
                best_ms = ms;
                best = c;
            }
        }
    };
    const long long gpcs[4] = {1, 2, 3, 4};
    const long long items[6] = {0, 8, 16, 32, 64, 128};
    const long long owned[4] = {-1, 1LL << 14, 1LL << 16, 1LL << 18};
    const long long waves[2] = {8, 4};
    try_dim([](BatchedConfig &c, long long v) { c.waves = (int)v; }, waves, 2);
    try_dim([](BatchedConfig &c, long long v) { c.gpc = (int)v; }, gpcs, 4);
    try_dim([](BatchedConfig &c, long long v) { c.block_items = (int)v; }, items, 6);
    try_dim([](BatchedConfig &c, long long v) { c.owned_bound = v; }, owned, 4);
    try_dim([](BatchedConfig &c, long long v) { c.gpc = (int)v; }, gpcs, 4);
    if (err != HFK_OK) return err;
    store_tuned_b(device_arch(), precision, best);
    if (best_gpc_out) *best_gpc_out = best.gpc;
    if (cache_path) return write_tuning(cache_path);
    return HFK_OK;
}

}  // extern "C"

static bool json_ll(const char *obj, const char *key, long long *out)
{
    char pat[64];
    snprintf(pat, sizeof(pat), "\"%s\"", key);
    const char *p = strstr(obj, pat);
    if (!p) return false;
    p = strchr(p + strlen(pat), ':');
    if (!p) return false;
    return sscanf(p + 1, " %lld", out) == 1;
}

static bool json_str(const char *obj, const char *key, std::string *out)
{
    char pat[64];
    snprintf(pat, sizeof(pat), "\"%s\"", key);
    const char *p = strstr(obj, pat);
    if (!p) return false;
    p = strchr(p + strlen(pat), ':');
    if (!p) return false;
    p = strchr(p, '"');
    if (!p) return false;
    const char *q = strchr(p + 1, '"');
    if (!q) return false;
    out->assign(p + 1, q - p - 1);
    return true;
}

static bool is_pow2_in(long long v, long long lo, long long hi)
{
    return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

extern "C" {

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
    if (!strstr(txt, "\"hfk-tuning-2\"")) return fail(HFK_EINVAL, "%s is not an hfk tuning table", cache_path);
    const char *bat = strstr(txt, "\"batched\"");
    std::vector<TuneEntry> single;
    std::vector<BatchedEntry> batched;
    for (const char *p = strchr(txt, '{'); p; p = strchr(p + 1, '{')) {
        if (p == txt) continue;   // the outer object
        const char *end = strchr(p, '}');
        if (!end) break;
        const std::string obj(p, end - p + 1);
        const char *o = obj.c_str();
        std::string arch;
        long long prec, v[6];
        if (!json_str(o, "arch", &arch) || !json_ll(o, "precision", &prec) || prec < 0 || prec > 1)
            return fail(HFK_EINVAL, "bad entry in %s", cache_path);
        if (bat && p > bat) {
            if (!json_ll(o, "gpc", &v[0]) || !json_ll(o, "block_items", &v[1]) || !json_ll(o, "owned_bound", &v[2]) ||
                !json_ll(o, "waves", &v[3]) || v[0] < 1 || v[0] > kMaxBatchGroupsPerCU || v[1] < 0 || v[1] > 1024 ||
                v[2] == 0 || v[2] < -1 || (v[3] != 4 && v[3] != 8))
                return fail(HFK_EINVAL, "bad batched entry in %s", cache_path);
            batched.push_back(BatchedEntry{arch, (int)prec, BatchedConfig{(int)v[0], (int)v[1], v[2], (int)v[3]}});
        } else {
            long long bucket;
            if (!json_ll(o, "size_bucket", &bucket) || !json_ll(o, "strategy", &v[0]) || !json_ll(o, "variant", &v[1]) ||
                !json_ll(o, "gpc", &v[2]) || !json_ll(o, "tile_items", &v[3]) || !json_ll(o, "group_bras", &v[4]) ||
                !json_ll(o, "ket_copies", &v[5]) || bucket < 0 || bucket > 62 || v[0] < 1 || v[0] > 2 || v[1] < 0 ||
                v[1] > 1 || v[2] < 1 || v[2] > kMaxGroupsPerCU || v[3] < 1 || v[3] > kMaxTileItems ||
                !is_pow2_in(v[4], kMinGroupBras, kMaxGroupBras) || v[5] < 0 || v[5] > 1024)
                return fail(HFK_EINVAL, "bad entry in %s", cache_path);
            single.push_back(TuneEntry{arch, (int)prec, (int)bucket,
                                       TunedConfig{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5]}});
        }
    }
    for (const TuneEntry &e : single) store_tuned(e.arch, e.precision, e.bucket, e.cfg);
    for (const BatchedEntry &e : batched) store_tuned_b(e.arch, e.precision, e.cfg);
    return HFK_OK;
}

hfk_status hfk_clear_tuning(void)
{
    g_err[0] = 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_tuned_b.clear();
    return HFK_OK;
}

hfk_status hfk_set_shape(int32_t tile_items, int32_t group_bras, int32_t ket_copies)
{
    g_err[0] = 0;
    if (tile_items < 0 || tile_items > kMaxTileItems)
        return fail(HFK_EINVAL, "tile_items must be in [0, %d] (got %d)", kMaxTileItems, (int)tile_items);
    if (group_bras != 0 && !is_pow2_in(group_bras, kMinGroupBras, kMaxGroupBras))
        return fail(HFK_EINVAL, "group_bras must be 0 or a power of two in [%d, %d] (got %d)", kMinGroupBras,
                    kMaxGroupBras, (int)group_bras);
    if (ket_copies < -1 || ket_copies > 1024)
        return fail(HFK_EINVAL, "ket_copies must be in [-1, 1024] (got %d)", (int)ket_copies);
    g_cfg_tile = tile_items;
    g_cfg_gbras = group_bras;
    g_cfg_kcopies = ket_copies;
    return HFK_OK;
}

hfk_status hfk_set_batched_config(int32_t groups_per_cu, int32_t block_items, int64_t owned_bound, int32_t waves)
{
    g_err[0] = 0;
    if (waves != 0 && waves != 4 && waves != 8)
        return fail(HFK_EINVAL, "waves must be 0, 4 or 8 (got %d)", (int)waves);
    if (groups_per_cu < 0 || groups_per_cu > kMaxBatchGroupsPerCU)
        return fail(HFK_EINVAL, "groups_per_cu must be in [0, %d] (got %d)", kMaxBatchGroupsPerCU, (int)groups_per_cu);
    if (block_items < 0 || block_items > 1024)
        return fail(HFK_EINVAL, "block_items must be in [0, 1024] (got %d)", (int)block_items);
    if (owned_bound < -1) return fail(HFK_EINVAL, "owned_bound must be -1, 0 or > 0 (got %lld)", (long long)owned_bound);
    g_cfg_b = BatchedConfig{groups_per_cu, block_items, (long long)owned_bound, waves};
    return HFK_OK;
}

}  // extern "C"
