// VALU throughput probe for MI355X: cycles per wave-wide instruction of the operations the
// quartet kernels are built from (FP64 FMA and multiply, FP32 FMA, v_rsq_f64, v_rsq_f32
// between conversions, and the far step's reciprocal square root with its folded Newton
// step).  Every mode runs eight independent dependency chains per lane, 8 waves per SIMD, and
// is timed with HIP events; cycles are reported at the 2.4 GHz engine clock.  Each thread
// writes one output element at its global index (grid sized to the buffer).
//
//     valu_probe            prints one JSON line
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(double *out, double a, double b)
{
    double v[kChains];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
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
}

template <int MODE>
float run(double *out, int blocks)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
    hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, out, 0.999999, 1e-9);
    float ms = -1.0f;
    if (hipEventRecord(e0) == hipSuccess) {
        hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, out, 0.999999, 1e-9);
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
    if (hipMalloc(&out, sizeof(double) * blocks * 256) != hipSuccess) return 1;
    const char *names[] = {"fma_f64", "mul_f64", "fma_f32", "rsq_f64", "4fma_f64+rsq_f64", "rsq_f64+newton",
                           "cvt+rsq_f32+cvt+newton"};
    float t[7];
    t[0] = run<0>(out, blocks);
    t[1] = run<1>(out, blocks);
    t[2] = run<2>(out, blocks);
    t[3] = run<3>(out, blocks);
    t[4] = run<4>(out, blocks);
    t[5] = run<5>(out, blocks);
    t[6] = run<6>(out, blocks);
    const double steps = (double)kIters * kChains * (blocks * 4.0) / (cus * 4.0);   // per SIMD
    printf("{\"probe\": \"valu\", \"cus\": %d, \"cycles_per_step_at_2400MHz\": {", cus);
    for (int m = 0; m < 7; ++m)
        printf("%s\"%s\": %.2f", m ? ", " : "", names[m], t[m] * 1e-3 * 2.4e9 / steps);
    printf("}}\n");
    (void)hipFree(out);
    for (int m = 0; m < 7; ++m)
        if (t[m] < 0) return 1;
    return 0;
}
