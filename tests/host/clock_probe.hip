// Test instrument: the shader clock while the each-pair-once FP64 force pass
// runs.  The kernel below is the library's own workgroup body (this file
// includes its source) with lane 0 of each workgroup reading s_memtime (the
// shader clock) and s_memrealtime (a constant 100 MHz counter) before and
// after it; their ratio over a workgroup is the clock it ran at.  Built into
// tests/host/libclockprobe.so by the package build; used by the GPU tests
// and the clock profile only, never by the library.
#include "kernels_mutual.hip"

#include <vector>

namespace nb {
namespace {

template <int KMT, int KMW>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual_clocked(
    const double* __restrict__ pos, const double* __restrict__ gm, int64_t n, MutualTail tl,
    MutualMap map, double* __restrict__ part, unsigned long long* __restrict__ clk)
{
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int g, r, half, xslot;
    mt_lookup(map, tl, blockIdx.x, g, r, half, xslot);
    mutual_unit<KMT, KMW, 0>(pos, gm, n, n, 0, g, r, part, tl, half, xslot);
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        unsigned long long* o = clk + 4 * (int64_t)blockIdx.x;
        o[0] = c0;
        o[1] = c1;
        o[2] = t0;
        o[3] = t1;
    }
}

}  // namespace
}  // namespace nb

// batches x per_batch back-to-back launches of the (4, 4) pass on n bodies
// (host positions pos_host[3n] and G m gm_host[n]).  Per batch: the event
// time per launch (us), and over the workgroups of the batch's last launch
// the mean, minimum and maximum shader clock (GHz).  Returns 0 on success.
extern "C" __attribute__((visibility("default"))) int clock_probe_force(const double* pos_host, const double* gm_host, int64_t n,
                                 int batches, int per_batch, double* us_per_launch,
                                 double* sclk_mean, double* sclk_min, double* sclk_max)
{
    using namespace nb;
    if (n < 1 || batches < 1 || per_batch < 1) return 1;
    const MutualTail tl = mutual_tail(n, 4, 4);
    const int64_t pairs = (int64_t)tl.R * (tl.R + 1) / 2;
    const int grid = (int)(tl.F + 2 * (pairs - tl.F));
    const int slots = mutual_slots(n, 4, 4);
    double *pos = nullptr, *gm = nullptr, *part = nullptr;
    unsigned long long* clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    std::vector<unsigned long long> h((size_t)grid * 4);
    if (hipMalloc(&pos, 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&gm, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&part, (size_t)slots * 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&clk, (size_t)grid * 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemcpy(pos, pos_host, 3 * n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(gm, gm_host, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = 2;
    }
    for (int b = 0; rc == 0 && b < batches; ++b) {
        if (hipEventRecord(e0, nullptr) != hipSuccess) { rc = 3; break; }
        for (int k = 0; k < per_batch; ++k)
            hipLaunchKernelGGL((k_force_mutual_clocked<4, 4>), dim3(grid), dim3(256), 0, nullptr,
                               pos, gm, n, tl, mutual_map(tl, grid), part, clk);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess) { rc = 4; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (hipMemcpy(h.data(), clk, h.size() * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost) != hipSuccess) { rc = 5; break; }
        double cyc = 0.0, ticks = 0.0, lo = 1e30, hi = 0.0;
        for (int w = 0; w < grid; ++w) {
            const double c = (double)(h[4 * w + 1] - h[4 * w]);
            const double t = (double)(h[4 * w + 3] - h[4 * w + 2]);
            if (t <= 0.0) continue;
            cyc += c;
            ticks += t;
            const double f = 0.1 * c / t;
            lo = f < lo ? f : lo;
            hi = f > hi ? f : hi;
        }
        us_per_launch[b] = 1e3 * ms / per_batch;
        sclk_mean[b] = ticks > 0.0 ? 0.1 * cyc / ticks : 0.0;
        sclk_min[b] = lo;
        sclk_max[b] = hi;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (pos) (void)hipFree(pos);
    if (gm) (void)hipFree(gm);
    if (part) (void)hipFree(part);
    if (clk) (void)hipFree(clk);
    return rc;
}
