// VALU throughput probe for MI355X: cycles per wave-wide instruction of the operations the
// quartet kernels are built from (FP64 FMA and multiply, FP32 FMA, v_rsq_f64, v_rsq_f32
// between conversions, and the far step's reciprocal square root with its folded Newton
// step).  Every mode runs eight independent dependency chains per lane, 8 waves per SIMD, and
// is timed with HIP events; cycles are reported at the 2.4 GHz engine clock and at the clock
// measured during the launch (thread 0's shader-clock ticks over its constant-rate ticks).
// Each thread writes one output element at its global index (grid sized to the buffer).
//
//     valu_probe            prints one JSON line
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(double *out, double a, double b, unsigned long long *clk)
{
    double v[kChains];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c0 = 0, w0 = 0;
    if (gid == 0) {
        c0 = clock64();        // shader clock counter
        w0 = wall_clock64();   // constant-rate counter
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 1.0 + 1e-3 * (gid + c);
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (MODE == 0) {
                v[c] = fma(v[c], v[(c + 1) % kChains], v[(c + 2) % kChains]);   // FP64 FMA
            } else if constexpr (MODE == 1) {
                v[c] = v[c] * a;                                                   // FP64 multiply
            } else if constexpr (MODE == 2) {
                v[c] = (double)fmaf((float)v[c], (float)a, (float)b);              // FP32 FMA
            } else if constexpr (MODE == 3) {
                v[c] = __builtin_amdgcn_rsq(v[c]);                                 // v_rsq_f64
            } else if constexpr (MODE == 4) {
                const double y = __builtin_amdgcn_rsq(v[c]);                       // 4 FMA + 1 rsq
                v[c] = fma(fma(fma(fma(y, a, b), a, b), a, b), a, v[c]);
            } else if constexpr (MODE == 5) {
                const double y = __builtin_amdgcn_rsq(v[c]);                       // rsq + Newton
                v[c] = fma(y * y, v[c], -3.0) * y + b;
            } else {
                const double y = (double)__builtin_amdgcn_rsqf((float)v[c]);       // cvt, rsq32, cvt + Newton
                v[c] = fma(y * y, v[c], -3.0) * y + b;
            }
        }
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[gid] = s;
    if (gid == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - w0;
    }
}

template <int MODE>
float run(double *out, int blocks, unsigned long long *clk)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
    hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, out, 0.999999, 1e-9, clk);
    float ms = -1.0f;
    if (hipEventRecord(e0) == hipSuccess) {
        hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, out, 0.999999, 1e-9, clk);
        if (hipEventRecord(e1) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
            (void)hipEventElapsedTime(&ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

int main()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
    const int cus = p.multiProcessorCount;
    const int blocks = cus * 8;   // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    double *out = nullptr;
    unsigned long long *clk = nullptr;
    if (hipMalloc(&out, sizeof(double) * blocks * 256) != hipSuccess) return 1;
    if (hipMalloc(&clk, 2 * sizeof(unsigned long long)) != hipSuccess) return 1;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess) wall_khz = 0;
    const char *names[] = {"fma_f64", "mul_f64", "fma_f32", "rsq_f64", "4fma_f64+rsq_f64", "rsq_f64+newton",
                           "cvt+rsq_f32+cvt+newton"};
    float t[7];
    double mhz[7];
    unsigned long long c[2];
    auto clock_mhz = [&]() {
        // engine clock during the last launch: shader-clock ticks over constant-rate ticks
        if (hipMemcpy(c, clk, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess || c[1] == 0 || wall_khz <= 0)
            return 0.0;
        return (double)c[0] / ((double)c[1] / (wall_khz * 1e3)) / 1e6;
    };
    t[0] = run<0>(out, blocks, clk); mhz[0] = clock_mhz();
    t[1] = run<1>(out, blocks, clk); mhz[1] = clock_mhz();
    t[2] = run<2>(out, blocks, clk); mhz[2] = clock_mhz();
    t[3] = run<3>(out, blocks, clk); mhz[3] = clock_mhz();
    t[4] = run<4>(out, blocks, clk); mhz[4] = clock_mhz();
    t[5] = run<5>(out, blocks, clk); mhz[5] = clock_mhz();
    t[6] = run<6>(out, blocks, clk); mhz[6] = clock_mhz();
    const double steps = (double)kIters * kChains * (blocks * 4.0) / (cus * 4.0);   // per SIMD
    printf("{\"probe\": \"valu\", \"cus\": %d, \"cycles_per_step_at_2400MHz\": {", cus);
    for (int m = 0; m < 7; ++m)
        printf("%s\"%s\": %.2f", m ? ", " : "", names[m], t[m] * 1e-3 * 2.4e9 / steps);
    printf("}, \"cycles_per_step_at_measured_clock\": {");
    for (int m = 0; m < 7; ++m)
        printf("%s\"%s\": %.2f", m ? ", " : "", names[m], t[m] * 1e-3 * mhz[m] * 1e6 / steps);
    printf("}, \"measured_clock_mhz\": [");
    for (int m = 0; m < 7; ++m) printf("%s%.0f", m ? ", " : "", mhz[m]);
    printf("]}\n");
    (void)hipFree(clk);
    (void)hipFree(out);
    for (int m = 0; m < 7; ++m)
        if (t[m] < 0) return 1;
    return 0;
}
