// Small systems (n <= kSmallMax): one workgroup of 1024 lanes keeps the
// whole state in LDS and executes consecutive launches of the
// kick-drift-kick loop of Eqs. (3)-(4) without leaving the kernel.
//
// Below a few hundred bodies a force pass is a few microseconds of work
// spread over far fewer wavefronts than the chip holds, so the multi-kernel
// path is bound by launch and inter-kernel gaps.  Here each step costs one
// pair sweep plus two workgroup barriers:
//  * lane (slice s, target p) with s = tid / n sums Eq. (1) over the source
//    slice [s L, (s+1) L), L = ceil(n / S), into LDS partials;
//  * after a barrier, lane e < 3n adds the S partials of component e in
//    ascending slice order (fixed order: deterministic) and applies the
//    half kicks and the drift to the LDS copy of (r, v);
//  * the state goes back to global memory at the end of the launch.
// The pair arithmetic is the one of the multi-CU force pass: the FP64 form
// with the refined FP32 reciprocal square root, or, in the split form,
// sources [0, n_major) with one Newton step and FP64 accumulation and the
// light sources as FP32 block sums entering a Kahan-compensated FP32 sum.
#include "common.hpp"
#include "pair_math.hpp"

namespace nb {
namespace {

using namespace pm;

constexpr int kThreads = 1024;
constexpr int kBlkS = 16;          // FP32 block length of the light-source sums
constexpr int64_t kSegment = 4096; // launch indices per kernel launch

struct __attribute__((aligned(32))) SBody {
    double x, y, z, gm;
};

template <bool SPLIT>
__global__ __launch_bounds__(kThreads) void k_run_small(
    const double* __restrict__ pos_in, double* __restrict__ pos_out, double* __restrict__ vel,
    const double* __restrict__ mass, int n, int S, const int64_t* __restrict__ nmaj_ptr, double G,
    double dt, int64_t i0, int64_t i1, int64_t steps, double* __restrict__ acc,
    double* __restrict__ traj, uint32_t* __restrict__ flags)
{
    __shared__ SBody body[kSmallMax];
    __shared__ float gm32[kSmallMax];
    __shared__ double lvel[3 * kSmallMax];
    __shared__ double part[3 * kThreads];   // S * 3n <= 3 * 1024

    const int tid = threadIdx.x;
    const int m3 = 3 * n;
    const bool run = steps > 0;
    const int nm = SPLIT ? (int)*nmaj_ptr : n;
    double* bd = reinterpret_cast<double*>(body);

    for (int j = tid; j < n; j += kThreads) {
        SBody b;
        b.x = pos_in[j];
        b.y = pos_in[n + j];
        b.z = pos_in[2 * n + j];
        b.gm = G * mass[j];
        body[j] = b;
        gm32[j] = (float)b.gm;
    }
    if (run)
        for (int e = tid; e < m3; e += kThreads) lvel[e] = vel[e];
    __syncthreads();

    const int s = tid / n;
    const int p = tid - s * n;
    const bool active = s < S;
    const int L = (n + S - 1) / S;
    const int jb = active ? min(s * L, n) : 0;
    const int je = active ? min(jb + L, n) : 0;
    const int jm = SPLIT ? max(jb, min(nm, je)) : je;
    const double hdt = 0.5 * dt;
    const PolyConst c = {vreg_const(1.875), vreg_const(1.5)};
    bool bad = false;

    for (int64_t i = i0; i <= i1; ++i) {
        if (active) {
            const SBody t = body[p];
            double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll 4
            for (int j = jb; j < jm; ++j) {
                const SBody b = body[j];
                const double dx = b.x - t.x;
                const double dy = b.y - t.y;
                const double dz = b.z - t.z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                double f = SPLIT ? gm_rinv3_newton1(r2, b.gm) : gm_rinv3_f64(r2, b.gm, c);
                f = (j == p) ? 0.0 : f;
                ax = __builtin_fma(f, dx, ax);
                ay = __builtin_fma(f, dy, ay);
                az = __builtin_fma(f, dz, az);
            }
            if (SPLIT) {
                float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
                for (int b0 = jm; b0 < je; b0 += kBlkS) {
                    const int b1 = min(b0 + kBlkS, je);
                    float bx = 0.f, by = 0.f, bz = 0.f;
                    for (int j = b0; j < b1; ++j) {
                        const SBody b = body[j];
                        const float dx = (float)(b.x - t.x);
                        const float dy = (float)(b.y - t.y);
                        const float dz = (float)(b.z - t.z);
                        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                        const float y = __builtin_amdgcn_rsqf(r2);
                        float w = gm32[j] * (y * y * y);
                        w = (j == p) ? 0.f : w;
                        bx = __builtin_fmaf(w, dx, bx);
                        by = __builtin_fmaf(w, dy, by);
                        bz = __builtin_fmaf(w, dz, bz);
                    }
                    kahan_add(sx, cx, bx);
                    kahan_add(sy, cy, by);
                    kahan_add(sz, cz, bz);
                }
                ax += (double)sx - (double)cx;
                ay += (double)sy - (double)cy;
                az += (double)sz - (double)cz;
            }
            double* ps = part + s * m3;
            ps[p] = ax;
            ps[n + p] = ay;
            ps[2 * n + p] = az;
        }
        __syncthreads();
        const bool close = i > 0;
        const bool open = i < steps;
        for (int e = tid; e < m3; e += kThreads) {
            double a = 0.0;
            for (int q = 0; q < S; ++q) a += part[q * m3 + e];
            bool fin = __builtin_isfinite(a);
            if (acc) acc[e] = a;
            if (run) {
                double v = lvel[e];
                if (close) v = v + hdt * a;
                if (open) {
                    v = v + hdt * a;
                    const int k = e / n;
                    const int q = e - k * n;
                    const double r = bd[4 * q + k] + dt * v;
                    fin = fin && __builtin_isfinite(r);
                    bd[4 * q + k] = r;
                    if (traj) traj[(i - i0) * m3 + e] = r;
                }
                fin = fin && __builtin_isfinite(v);
                lvel[e] = v;
            }
            bad = bad || !fin;
        }
        __syncthreads();
    }

    if (run) {
        for (int e = tid; e < m3; e += kThreads) {
            const int k = e / n;
            const int q = e - k * n;
            if (pos_out) pos_out[e] = bd[4 * q + k];
            vel[e] = lvel[e];
        }
    }
    if (bad && flags) atomicOr(flags, 1u);
}

}  // namespace

int small_slices(int64_t n, const Tile& t)
{
    if (n < 1 || n > kSmallMax) return 0;
    int64_t S = t.chunks < 1 ? 1 : t.chunks;
    S = S < n ? S : n;
    const int64_t cap = kThreads / n;
    return (int)(S < cap ? S : cap);
}

hipError_t launch_run_small(int precision, const Tile& tile, const double* pos_in,
                            double* pos_out, double* vel, const double* mass, int64_t n,
                            const int64_t* nmaj, double G, double dt, int64_t i0, int64_t i1,
                            int64_t steps, double* acc, double* traj, uint32_t* flags,
                            hipStream_t s)
{
    const int S = small_slices(n, tile);
    if (tile.variant != 3 || S < 1 || i0 < 0 || i1 < i0 || (steps > 0 && (!vel || i1 > steps)) ||
        (precision == 1 && !nmaj) || (acc && steps > 0))
        return hipErrorInvalidValue;
    if (steps > 0 && !pos_out && !traj) return hipErrorInvalidValue;
    const double* rin = pos_in;
    for (int64_t a = i0; a <= i1; a += kSegment) {
        const int64_t b = (a + kSegment - 1 < i1) ? a + kSegment - 1 : i1;
        double* tr = traj ? traj + (a - i0) * 3 * n : nullptr;
        // a launch that stores nothing but the trajectory hands its last
        // position on through the trajectory buffer
        const bool last = (b == i1);
        double* rout = pos_out;
        if (precision == 0)
            hipLaunchKernelGGL(k_run_small<false>, dim3(1), dim3(kThreads), 0, s, rin, rout, vel,
                               mass, (int)n, S, nmaj, G, dt, a, b, steps, acc, tr, flags);
        else
            hipLaunchKernelGGL(k_run_small<true>, dim3(1), dim3(kThreads), 0, s, rin, rout, vel,
                               mass, (int)n, S, nmaj, G, dt, a, b, steps, acc, tr, flags);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (!last) rin = rout ? rout : tr + (b - a) * 3 * n;
    }
    return hipSuccess;
}

}  // namespace nb
