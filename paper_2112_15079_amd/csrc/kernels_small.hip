// Small systems (n <= kSmallMax): one workgroup of 1024 lanes keeps the
// whole state on chip and executes consecutive launches of the
// kick-drift-kick loop of Eqs. (3)-(4) without leaving the kernel.
//
// Below a few hundred bodies a force pass is a few microseconds of work
// spread over far fewer wavefronts than the chip holds, so the multi-kernel
// path is bound by launch and inter-kernel gaps.  Here each step costs one
// pair sweep plus two workgroup barriers:
//  * lane (slice s, target p), s = tid / n, sums Eq. (1) over slice s of its
//    sources into LDS partials;
//  * after a barrier, lane e (< 3n, and e + 1024) adds the S partials of
//    component e in ascending slice order (fixed order: deterministic) and
//    applies the half kicks and the drift; velocities stay in registers,
//    positions in LDS;
//  * the state goes back to global memory at the end of the launch.
//
// Sources are visited in rotated order so that no lane ever meets its own
// body and the self pair needs no mask: each mass class (all bodies in the
// FP64 form; [0, n_major) and [n_major, n) in the split form) is stored
// twice in a row in LDS, and target p walks its own class starting just
// after itself (c0 + p + 1, ..., wrapping through the second copy) and any
// other class from its start.  Lanes of a wavefront read consecutive LDS
// words (no bank conflicts).
//
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

// One mass class as seen from a lane: LDS indices base + k for the lane's
// slice k in [kb, ke).
struct Span {
    int base, kb, ke;
};

// Class [c0, c0 + len) stored twice from LDS index d0; `slice` of S slices
// of the lane's visiting order (own class: skip itself).
__device__ __forceinline__ Span class_span(int p, int c0, int len, int d0, int longest,
                                           int slice, int S)
{
    const bool own = (p >= c0) && (p < c0 + len);
    const int count = own ? len - 1 : len;
    const int L = (longest + S - 1) / S;
    Span sp;
    sp.base = d0 + (own ? (p - c0) + 1 : 0);
    sp.kb = min(slice * L, count);
    sp.ke = min(sp.kb + L, count);
    return sp;
}

template <bool SPLIT>
__global__ __launch_bounds__(kThreads) void k_run_small(
    const double* pos_in, double* pos_out, double* __restrict__ vel,   // pos_in may be pos_out
    const double* __restrict__ mass, int n, int S, const int64_t* __restrict__ nmaj_ptr, double G,
    double dt, int64_t i0, int64_t i1, int64_t steps, double* __restrict__ acc,
    double* __restrict__ traj, uint32_t* __restrict__ flags)
{
    __shared__ double lx[2 * kSmallMax], ly[2 * kSmallMax], lz[2 * kSmallMax];
    __shared__ double lg[2 * kSmallMax];
    __shared__ float lg32[2 * kSmallMax];
    __shared__ double part[3 * kThreads];   // S * 3n <= 3 * 1024

    const int tid = threadIdx.x;
    const int m3 = 3 * n;
    const bool run = steps > 0;
    const int nm = SPLIT ? (int)*nmaj_ptr : n;   // FP64-class bodies [0, nm)
    const int nl = n - nm;                       // FP32-class bodies [nm, n)
    // LDS index of the first copy of body q, and the distance to the second
    auto slot = [&](int q) { return q < nm ? q : 2 * nm + (q - nm); };
    auto period = [&](int q) { return q < nm ? nm : nl; };

    for (int q = tid; q < n; q += kThreads) {
        const int a = slot(q), b = a + period(q);
        const double x = pos_in[q], y = pos_in[n + q], z = pos_in[2 * n + q];
        const double g = G * mass[q];
        lx[a] = x; lx[b] = x;
        ly[a] = y; ly[b] = y;
        lz[a] = z; lz[b] = z;
        lg[a] = g; lg[b] = g;
        lg32[a] = (float)g; lg32[b] = (float)g;
    }
    double v0 = 0.0, v1 = 0.0;
    if (run) {
        if (tid < m3) v0 = vel[tid];
        if (tid + kThreads < m3) v1 = vel[tid + kThreads];
    }
    __syncthreads();

    const int s = tid / n;
    const int p = tid - s * n;
    const bool active = s < S;
    const int ps = slot(p);
    // longest visiting order per class over all lanes (sets the slice length)
    const Span A = class_span(p, 0, nm, 0, nl > 0 ? nm : nm - 1, s, S);
    const Span B = class_span(p, nm, nl, 2 * nm, nm > 0 ? nl : nl - 1, s, S);
    const double hdt = 0.5 * dt;
    const PolyConst c = {vreg_const(1.875), vreg_const(1.5)};
    bool bad = false;

    for (int64_t i = i0; i <= i1; ++i) {
        if (active) {
            const double tx = lx[ps], ty = ly[ps], tz = lz[ps];
            double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll 4
            for (int k = A.kb; k < A.ke; ++k) {
                const int j = A.base + k;
                const double dx = lx[j] - tx;
                const double dy = ly[j] - ty;
                const double dz = lz[j] - tz;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double f = SPLIT ? gm_rinv3_newton1(r2, lg[j]) : gm_rinv3_f64(r2, lg[j], c);
                ax = __builtin_fma(f, dx, ax);
                ay = __builtin_fma(f, dy, ay);
                az = __builtin_fma(f, dz, az);
            }
            if (SPLIT) {
                float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
                for (int k0 = B.kb; k0 < B.ke; k0 += kBlkS) {
                    const int k1 = min(k0 + kBlkS, B.ke);
                    float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll 4
                    for (int k = k0; k < k1; ++k) {
                        const int j = B.base + k;
                        const float dx = (float)(lx[j] - tx);
                        const float dy = (float)(ly[j] - ty);
                        const float dz = (float)(lz[j] - tz);
                        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                        const float y = __builtin_amdgcn_rsqf(r2);
                        const float w = lg32[j] * (y * y * y);
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
            double* pp = part + s * m3;
            pp[p] = ax;
            pp[n + p] = ay;
            pp[2 * n + p] = az;
        }
        __syncthreads();
        const bool close = i > 0;
        const bool open = i < steps;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + h * kThreads;
            if (e >= m3) break;
            double a = 0.0;
            for (int q = 0; q < S; ++q) a += part[q * m3 + e];
            bool fin = __builtin_isfinite(a);
            if (acc) acc[e] = a;
            if (run) {
                double v = h ? v1 : v0;
                if (close) v = v + hdt * a;
                if (open) {
                    v = v + hdt * a;
                    const int k = e / n;
                    const int q = e - k * n;
                    double* plane = k == 0 ? lx : (k == 1 ? ly : lz);
                    const int sa = slot(q);
                    const double r = plane[sa] + dt * v;
                    fin = fin && __builtin_isfinite(r);
                    plane[sa] = r;
                    plane[sa + period(q)] = r;
                    if (traj) traj[(i - i0) * m3 + e] = r;
                }
                fin = fin && __builtin_isfinite(v);
                if (h) v1 = v; else v0 = v;
            }
            bad = bad || !fin;
        }
        __syncthreads();
    }

    if (run) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + h * kThreads;
            if (e >= m3) break;
            const int k = e / n;
            const int q = e - k * n;
            const double* plane = k == 0 ? lx : (k == 1 ? ly : lz);
            if (pos_out) pos_out[e] = plane[slot(q)];
            vel[e] = h ? v1 : v0;
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
        if (precision == 0)
            hipLaunchKernelGGL(k_run_small<false>, dim3(1), dim3(kThreads), 0, s, rin, pos_out,
                               vel, mass, (int)n, S, nmaj, G, dt, a, b, steps, acc, tr, flags);
        else
            hipLaunchKernelGGL(k_run_small<true>, dim3(1), dim3(kThreads), 0, s, rin, pos_out,
                               vel, mass, (int)n, S, nmaj, G, dt, a, b, steps, acc, tr, flags);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // a launch that stores nothing but the trajectory hands its last
        // position on through the trajectory buffer
        if (b < i1) rin = pos_out ? pos_out : tr + (b - a) * 3 * n;
    }
    return hipSuccess;
}

}  // namespace nb
