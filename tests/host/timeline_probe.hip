// Test instrument: when each wave of the each-pair-once FP64 force pass
// (shape (4, 4)) enters, starts its sweep (sources and targets staged), ends
// it, and exits, in the 100 MHz s_memrealtime counter, with the CU and SIMD
// it ran on (HW_ID, XCC_ID).  The kernel below is the library's own
// workgroup body (this file includes its source) with its marks defined to
// record these times; built into tests/host/libtimelineprobe.so by the
// package build; used by the GPU tests and the timeline profile only, never
// by the library.
#include <hip/hip_runtime.h>
#include <cstdint>

// per wave: entry, sweep start, sweep end, exit, HW_ID, XCC_ID, unit, unused
__device__ unsigned long long* g_timeline = nullptr;
#define NB_MUTUAL_MARK(k)                                                                   \
    do {                                                                                    \
        const unsigned long long ts_ = __builtin_amdgcn_s_memrealtime();                    \
        unsigned long long* r_ = g_timeline;                                                \
        if (r_ && (threadIdx.x & 63) == 0)                                                  \
            r_[((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 8 + (k)] = ts_;             \
    } while (0)
#include "kernels_mutual.hip"

namespace nb {
namespace {

__global__ __launch_bounds__(256) void k_force_mutual_timeline(
    const double* __restrict__ pos, const double* __restrict__ gm, int64_t n, MutualTail tl,
    MutualMap map, double* __restrict__ part)
{
    NB_MUTUAL_MARK(0);
    int g, r, half, xslot;
    mt_lookup(map, tl, blockIdx.x, g, r, half, xslot);
    mutual_unit<4, 4, 0>(pos, gm, n, n, 0, g, r, part, tl, half, xslot);
    NB_MUTUAL_MARK(3);
    unsigned long long* o = g_timeline;
    if (o && (threadIdx.x & 63) == 0) {
        o += ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 8;
        o[4] = __builtin_amdgcn_s_getreg(63492);   // HW_ID (32 bits)
        o[5] = __builtin_amdgcn_s_getreg(63508);   // XCC_ID (32 bits)
        o[6] = (unsigned long long)((int64_t)g * 1000000 + (int64_t)r * 10 + (half + 1));
    }
}

}  // namespace
}  // namespace nb

// `warm` unrecorded launches, then one recorded launch of the (4, 4) pass on
// n bodies (host positions pos_host[3n], G m gm_host[n]); out[grid * 32]
// receives the records (8 per wave, 4 waves per workgroup), *grid_out the
// workgroup count, *us_out the recorded launch's event time.  Returns 0 on
// success, 1 on bad arguments or a too small out, 2 on a HIP error.
extern "C" __attribute__((visibility("default"))) int timeline_probe_force(
    const double* pos_host, const double* gm_host, int64_t n, int warm,
    unsigned long long* out, int64_t out_len, int* grid_out, double* us_out)
{
    using namespace nb;
    if (n < 1 || warm < 0 || !out || !grid_out || !us_out) return 1;
    const MutualTail tl = mutual_tail(n, 4, 4);
    const int64_t pairs = (int64_t)tl.R * (tl.R + 1) / 2;
    const int64_t grid = tl.F + 2 * (pairs - tl.F);
    *grid_out = (int)grid;
    if (grid * 32 > out_len) return 1;
    const int slots = mutual_slots(n, 4, 4);
    double *pos = nullptr, *gm = nullptr, *part = nullptr;
    unsigned long long* rec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 2;
    const size_t rec_bytes = (size_t)grid * 32 * sizeof(unsigned long long);
    unsigned long long* none = nullptr;
    float ms = 0.f;
    if (hipMalloc(&pos, 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&gm, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&part, (size_t)slots * 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&rec, rec_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        goto done;
    if (hipMemcpy(pos, pos_host, 3 * n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(gm, gm_host, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(rec, 0, rec_bytes) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_timeline), &none, sizeof(none)) != hipSuccess)
        goto done;
    for (int k = 0; k < warm; ++k)
        hipLaunchKernelGGL(k_force_mutual_timeline, dim3((unsigned)grid), dim3(256), 0, nullptr,
                           pos, gm, n, tl, mutual_map(tl, grid), part);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_timeline), &rec, sizeof(rec)) != hipSuccess ||
        hipEventRecord(e0, nullptr) != hipSuccess)
        goto done;
    hipLaunchKernelGGL(k_force_mutual_timeline, dim3((unsigned)grid), dim3(256), 0, nullptr, pos,
                       gm, n, tl, mutual_map(tl, grid), part);
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipMemcpy(out, rec, rec_bytes, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_timeline), &none, sizeof(none)) != hipSuccess)
        goto done;
    *us_out = 1e3 * ms;
    rc = 0;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(pos);
    (void)hipFree(gm);
    (void)hipFree(part);
    (void)hipFree(rec);
    return rc;
}
