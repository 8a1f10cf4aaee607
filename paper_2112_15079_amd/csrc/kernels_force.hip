// Force pass of Eq. (1): a_p = sum_{j != p} G m_j (r_j - r_p) / |r_j - r_p|^3.
//
// gfx950 design (vector ALU bound, no MFMA: the pair sum is not a dense
// contraction):
//  * positions and masses are structure-of-arrays planes, so the per-target
//    and per-source loads are unit-stride;
//  * a workgroup stages one tile of 64*waves sources in LDS as packed
//    (x, y, z, G m) doubles; every lane of a wavefront reads the same source,
//    so each LDS read is a broadcast;
//  * each lane keeps `tpl` targets and their accumulators in registers, so one
//    LDS read feeds tpl pair evaluations;
//  * the source range is split into chunks (grid.y) to give small systems
//    enough workgroups for 256 CUs; chunk partials are summed in a fixed
//    order by the step epilogue, so results are deterministic;
//  * the self pair is masked only in the tiles that overlap the workgroup's
//    own targets.
#include "common.hpp"
#include "pair_math.hpp"

namespace nb {
namespace {

using namespace pm;

struct __attribute__((aligned(32))) Src {
    double x, y, z, gm;
};

// Padding source for the ragged last tile: massless and far away, so its
// term is an exact zero without a branch.
constexpr double kPad = 1.0e18;

template <int T>
struct Targets {
    double x[T], y[T], z[T];
    int id[T];
};

// `pos` points at the system's first body; planes are `stride` apart.
template <int T, int NT>
__device__ __forceinline__ void load_targets(Targets<T>& tg, const double* __restrict__ pos,
                                             int64_t stride, int64_t n, int64_t base, int tid)
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = base + (int64_t)t * NT + tid;
        const int64_t q = p < n ? p : n - 1;
        tg.id[t] = (int)p;
        tg.x[t] = pos[q];
        tg.y[t] = pos[stride + q];
        tg.z[t] = pos[2 * stride + q];
    }
}

// Light sources of the split form (j >= small_from) carry G m as an FP32
// value in the low half of the gm slot (see small_gm), saving a conversion
// per pair in the FP32 sweep.
__device__ __forceinline__ Src load_source(const double* __restrict__ pos,
                                           const double* __restrict__ mass, int64_t stride,
                                           int64_t j, int64_t jend, double G,
                                           int64_t small_from = INT64_MAX)
{
    Src s;
    if (j < jend) {
        s.x = pos[j];
        s.y = pos[stride + j];
        s.z = pos[2 * stride + j];
        const double gm = G * mass[j];
        s.gm = j < small_from ? gm
                              : __builtin_bit_cast(double, (uint64_t)__builtin_bit_cast(uint32_t, (float)gm));
    } else {
        s.x = kPad;
        s.y = kPad;
        s.z = kPad;
        s.gm = 0.0;
    }
    return s;
}

// ---------------------------------------------------------------------------
// FP64 sweep over sources [jb, je) of the LDS tile.
template <int T, bool MASK, bool NEWTON1>
__device__ __forceinline__ void sweep_f64(const Src* __restrict__ tile, int jb, int je, int j0,
                                          const Targets<T>& tg, double (&ax)[T], double (&ay)[T],
                                          double (&az)[T], const PolyConst& c32)
{
#pragma unroll 4
    for (int jj = jb; jj < je; ++jj) {
        const Src s = tile[jj];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const double dx = s.x - tg.x[t];
            const double dy = s.y - tg.y[t];
            const double dz = s.z - tg.z[t];
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            double f = NEWTON1 ? gm_rinv3_newton1(r2, s.gm) : gm_rinv3_f64(r2, s.gm, c32);
            if (MASK) f = (j0 + jj == tg.id[t]) ? 0.0 : f;
            ax[t] = __builtin_fma(f, dx, ax[t]);
            ay[t] = __builtin_fma(f, dy, ay[t]);
            az[t] = __builtin_fma(f, dz, az[t]);
        }
    }
}

// FP32 sweep for light sources: FP64 displacement, then the term in FP32;
// the terms of each block of kBlk sources are added in FP32 and each block
// sum enters a Kahan-compensated FP32 running sum.
constexpr int kBlk = 16;

template <int T>
struct Kahan {
    float sx[T], sy[T], sz[T], cx[T], cy[T], cz[T];
};


__device__ __forceinline__ float small_gm(double slot)
{
    return __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(uint64_t, slot));
}

template <int T, bool MASK>
__device__ __forceinline__ void sweep_small(const Src* __restrict__ tile, int jb, int je, int j0,
                                            const Targets<T>& tg, Kahan<T>& k)
{
    for (int b0 = jb; b0 < je; b0 += kBlk) {
        const int b1 = (b0 + kBlk < je) ? b0 + kBlk : je;
        float bx[T], by[T], bz[T];
#pragma unroll
        for (int t = 0; t < T; ++t) { bx[t] = 0.f; by[t] = 0.f; bz[t] = 0.f; }
#pragma unroll 4
        for (int jj = b0; jj < b1; ++jj) {
            const Src s = tile[jj];
            const float gm = small_gm(s.gm);
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const float dx = (float)(s.x - tg.x[t]);
                const float dy = (float)(s.y - tg.y[t]);
                const float dz = (float)(s.z - tg.z[t]);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                const float y = __builtin_amdgcn_rsqf(r2);
                float w = gm * (y * y * y);
                if (MASK) w = (j0 + jj == tg.id[t]) ? 0.f : w;
                bx[t] = __builtin_fmaf(w, dx, bx[t]);
                by[t] = __builtin_fmaf(w, dy, by[t]);
                bz[t] = __builtin_fmaf(w, dz, bz[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            kahan_add(k.sx[t], k.cx[t], bx[t]);
            kahan_add(k.sy[t], k.cy[t], by[t]);
            kahan_add(k.sz[t], k.cz[t], bz[t]);
        }
    }
}

// ---------------------------------------------------------------------------
// One workgroup: targets [tb0, tb0 + NT*T), sources [jbeg, jend) of a system
// of n bodies whose planes start at pos/mass/part_c and are `stride` apart.
template <int T, int W, bool SPLIT>
__device__ __forceinline__ void force_block(const double* __restrict__ pos,
                                            const double* __restrict__ mass, int64_t stride,
                                            int64_t n, int64_t n_major, double G, int64_t tb0,
                                            int64_t jbeg, int64_t jend,
                                            double* __restrict__ part_c)
{
    constexpr int NT = 64 * W;
    __shared__ Src tile[NT];
    const int tid = threadIdx.x;

    Targets<T> tg;
    load_targets<T, NT>(tg, pos, stride, n, tb0, tid);
    double ax[T], ay[T], az[T];
    Kahan<T> k;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
        k.sx[t] = 0.f; k.sy[t] = 0.f; k.sz[t] = 0.f;
        k.cx[t] = 0.f; k.cy[t] = 0.f; k.cz[t] = 0.f;
    }
    const int64_t tend = tb0 + (int64_t)NT * T;
    const PolyConst c32 = {vreg_const(1.875), vreg_const(1.5)};

    const int64_t small_from = SPLIT ? n_major : INT64_MAX;
    Src next = load_source(pos, mass, stride, jbeg + tid, jend, G, small_from);
    for (int64_t j0 = jbeg; j0 < jend; j0 += NT) {
        __syncthreads();
        tile[tid] = next;
        __syncthreads();
        if (j0 + NT < jend)
            next = load_source(pos, mass, stride, j0 + NT + tid, jend, G, small_from);
        const bool diag = (j0 < tend) && (tb0 < j0 + NT);
        const int j0i = (int)j0;
        if (!SPLIT) {
            if (diag) sweep_f64<T, true, false>(tile, 0, NT, j0i, tg, ax, ay, az, c32);
            else      sweep_f64<T, false, false>(tile, 0, NT, j0i, tg, ax, ay, az, c32);
        } else {
            int64_t jm64 = n_major - j0;
            const int jm = jm64 <= 0 ? 0 : (jm64 >= NT ? NT : (int)jm64);
            if (jm == NT) {
                if (diag) sweep_f64<T, true, true>(tile, 0, NT, j0i, tg, ax, ay, az, c32);
                else      sweep_f64<T, false, true>(tile, 0, NT, j0i, tg, ax, ay, az, c32);
            } else if (jm == 0) {
                if (diag) sweep_small<T, true>(tile, 0, NT, j0i, tg, k);
                else      sweep_small<T, false>(tile, 0, NT, j0i, tg, k);
            } else {
                sweep_f64<T, true, true>(tile, 0, jm, j0i, tg, ax, ay, az, c32);
                sweep_small<T, true>(tile, jm, NT, j0i, tg, k);
            }
        }
    }

#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = tb0 + (int64_t)t * NT + tid;
        if (p < n) {
            double vx = ax[t], vy = ay[t], vz = az[t];
            if (SPLIT) {
                vx += (double)k.sx[t] - (double)k.cx[t];
                vy += (double)k.sy[t] - (double)k.cy[t];
                vz += (double)k.sz[t] - (double)k.cz[t];
            }
            __builtin_nontemporal_store(vx, &part_c[p]);
            __builtin_nontemporal_store(vy, &part_c[stride + p]);
            __builtin_nontemporal_store(vz, &part_c[2 * stride + p]);
        }
    }
}

// ---------------------------------------------------------------------------
// Scalar-operand variant.  Every lane of a wavefront needs the same source,
// so the source coordinates and G m are fetched once per wavefront into
// scalar registers (one s_load_dwordx16 brings 8 consecutive values of a
// plane through the scalar data cache) and enter the vector instructions as
// scalar operands: no LDS staging, no barriers, no per-lane copies.  The
// mass plane is pre-multiplied by G (gm).
constexpr int kSGroup = 8;

template <int T, bool MASK, bool NEWTON1>
__device__ __forceinline__ void pair_f64(double sx, double sy, double sz, double sg, int64_t j,
                                         const Targets<T>& tg, double (&ax)[T], double (&ay)[T],
                                         double (&az)[T], const PolyConst& c)
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const double dx = sx - tg.x[t];
        const double dy = sy - tg.y[t];
        const double dz = sz - tg.z[t];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        double f = NEWTON1 ? gm_rinv3_newton1(r2, sg) : gm_rinv3_f64(r2, sg, c);
        if (MASK) f = (j == tg.id[t]) ? 0.0 : f;
        ax[t] = __builtin_fma(f, dx, ax[t]);
        ay[t] = __builtin_fma(f, dy, ay[t]);
        az[t] = __builtin_fma(f, dz, az[t]);
    }
}

template <int T, bool MASK>
__device__ __forceinline__ void pair_small(double sx, double sy, double sz, double sg, int64_t j,
                                           const Targets<T>& tg, float (&bx)[T], float (&by)[T],
                                           float (&bz)[T])
{
    const float gm = (float)sg;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const float dx = (float)(sx - tg.x[t]);
        const float dy = (float)(sy - tg.y[t]);
        const float dz = (float)(sz - tg.z[t]);
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        const float y = __builtin_amdgcn_rsqf(r2);
        float w = gm * (y * y * y);
        if (MASK) w = (j == tg.id[t]) ? 0.f : w;
        bx[t] = __builtin_fmaf(w, dx, bx[t]);
        by[t] = __builtin_fmaf(w, dy, by[t]);
        bz[t] = __builtin_fmaf(w, dz, bz[t]);
    }
}

template <int T>
__device__ __forceinline__ void kahan_flush(Kahan<T>& k, float (&bx)[T], float (&by)[T],
                                            float (&bz)[T])
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        kahan_add(k.sx[t], k.cx[t], bx[t]);
        kahan_add(k.sy[t], k.cy[t], by[t]);
        kahan_add(k.sz[t], k.cz[t], bz[t]);
        bx[t] = 0.f; by[t] = 0.f; bz[t] = 0.f;
    }
}

// One workgroup of W wavefronts.  SHARE = false (variant 1): each wave owns
// its own targets (lane l of the group holds tb0 + t*64*W + l, as in the LDS
// variant) and sweeps all sources [jbeg, jend).  SHARE = true (variant 2):
// all waves share the targets [tb0, tb0 + 64*T) (lane l holds tb0 + t*64 + l)
// and split the sources into W contiguous runs; the W partial sums are added
// in wave order through LDS, so one partial per group reaches global memory.
// out(comp, p, a) receives the sum over [jbeg, jend) of component comp of
// target p's acceleration, once per (comp, p < n).
template <int T, int W, bool SPLIT, bool SHARE, class Out>
__device__ __forceinline__ void force_block_s(const double* __restrict__ pos,
                                              const double* __restrict__ gm, int64_t stride,
                                              int64_t n, int64_t n_major, int64_t tb0,
                                              int64_t jbeg, int64_t jend, Out&& out)
{
    constexpr int TS = SHARE ? 64 : 64 * W;   // stride between a lane's targets
    const int lane = SHARE ? (threadIdx.x & 63) : threadIdx.x;
    const int wave = SHARE ? (threadIdx.x >> 6) : 0;
    Targets<T> tg;
    load_targets<T, TS>(tg, pos, stride, n, tb0, lane);
    double ax[T], ay[T], az[T];
    Kahan<T> k;
    float bx[T], by[T], bz[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
        k.sx[t] = 0.f; k.sy[t] = 0.f; k.sz[t] = 0.f;
        k.cx[t] = 0.f; k.cy[t] = 0.f; k.cz[t] = 0.f;
        bx[t] = 0.f; by[t] = 0.f; bz[t] = 0.f;
    }
    const PolyConst c32 = {vreg_const(1.875), vreg_const(1.5)};
    const int64_t tend = tb0 + (int64_t)TS * T;
    const double* __restrict__ px = pos;
    const double* __restrict__ py = pos + stride;
    const double* __restrict__ pz = pos + 2 * stride;

    // this wave's run of sources (a multiple of kSGroup long, except the last)
    constexpr int NW = SHARE ? W : 1;
    const int64_t span = jend - jbeg;
    const int64_t run = ((span + NW - 1) / NW + kSGroup - 1) / kSGroup * kSGroup;
    const int64_t wb = jbeg + (int64_t)wave * run;
    const int64_t we = (wb + run < jend) ? wb + run : jend;

    int small_groups = 0;
    int64_t j = wb;
    for (; j + kSGroup <= we; j += kSGroup) {
        double xs[kSGroup], ys[kSGroup], zs[kSGroup], gs[kSGroup];
#pragma unroll
        for (int u = 0; u < kSGroup; ++u) {
            xs[u] = px[j + u];
            ys[u] = py[j + u];
            zs[u] = pz[j + u];
            gs[u] = gm[j + u];
        }
        const bool diag = (j < tend) && (tb0 < j + kSGroup);
        if (!SPLIT || j + kSGroup <= n_major) {
            if (diag) {
#pragma unroll
                for (int u = 0; u < kSGroup; ++u)
                    pair_f64<T, true, SPLIT>(xs[u], ys[u], zs[u], gs[u], j + u, tg, ax, ay, az, c32);
            } else {
#pragma unroll
                for (int u = 0; u < kSGroup; ++u)
                    pair_f64<T, false, SPLIT>(xs[u], ys[u], zs[u], gs[u], j + u, tg, ax, ay, az, c32);
            }
        } else if (j >= n_major) {
            if (diag) {
#pragma unroll
                for (int u = 0; u < kSGroup; ++u)
                    pair_small<T, true>(xs[u], ys[u], zs[u], gs[u], j + u, tg, bx, by, bz);
            } else {
#pragma unroll
                for (int u = 0; u < kSGroup; ++u)
                    pair_small<T, false>(xs[u], ys[u], zs[u], gs[u], j + u, tg, bx, by, bz);
            }
            // a compensated add every kBlk small sources
            if (++small_groups == kBlk / kSGroup) {
                kahan_flush(k, bx, by, bz);
                small_groups = 0;
            }
        } else {
            for (int u = 0; u < kSGroup; ++u) {
                if (j + u < n_major)
                    pair_f64<T, true, true>(xs[u], ys[u], zs[u], gs[u], j + u, tg, ax, ay, az, c32);
                else
                    pair_small<T, true>(xs[u], ys[u], zs[u], gs[u], j + u, tg, bx, by, bz);
            }
        }
    }
    for (; j < we; ++j) {
        const double sx = px[j], sy = py[j], sz = pz[j], sg = gm[j];
        if (!SPLIT || j < n_major)
            pair_f64<T, true, SPLIT>(sx, sy, sz, sg, j, tg, ax, ay, az, c32);
        else
            pair_small<T, true>(sx, sy, sz, sg, j, tg, bx, by, bz);
    }
    if (SPLIT) {
        kahan_flush(k, bx, by, bz);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            ax[t] += (double)k.sx[t] - (double)k.cx[t];
            ay[t] += (double)k.sy[t] - (double)k.cy[t];
            az[t] += (double)k.sz[t] - (double)k.cz[t];
        }
    }

    if (SHARE && W > 1) {
        __shared__ double red[W][3 * T][64];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            red[wave][3 * t + 0][lane] = ax[t];
            red[wave][3 * t + 1][lane] = ay[t];
            red[wave][3 * t + 2][lane] = az[t];
        }
        __syncthreads();
        // wave w finishes component rows w, w + W, ...; waves summed in order
        for (int row = wave; row < 3 * T; row += W) {
            double s = red[0][row][lane];
            for (int w = 1; w < W; ++w) s += red[w][row][lane];
            const int t = row / 3, comp = row % 3;
            const int64_t p = tb0 + (int64_t)t * 64 + lane;
            if (p < n) out(comp, p, s);
        }
    } else {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int64_t p = tb0 + (int64_t)t * TS + lane;
            if (p < n) {
                out(0, p, ax[t]);
                out(1, p, ay[t]);
                out(2, p, az[t]);
            }
        }
    }
}

// Store into the chunk-partial planes (plane stride `stride`).
struct PartStore {
    double* __restrict__ part_c;
    int64_t stride;
    __device__ __forceinline__ void operator()(int comp, int64_t p, double a) const
    {
        __builtin_nontemporal_store(a, &part_c[comp * stride + p]);
    }
};

template <int T, int W, bool SPLIT, bool SHARE>
__global__ __launch_bounds__(64 * W) void k_force_s(const double* __restrict__ pos,
                                                    const double* __restrict__ gm, int64_t n,
                                                    const int64_t* __restrict__ nmaj,
                                                    int64_t chunk_len, double* __restrict__ part)
{
    const int64_t n_major = SPLIT ? nmaj[0] : 0;
    const int64_t tb0 = (int64_t)blockIdx.x * (SHARE ? 64 : 64 * W) * T;
    const int64_t c = blockIdx.y;
    const int64_t jbeg = c * chunk_len;
    const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;
    force_block_s<T, W, SPLIT, SHARE>(pos, gm, n, n, n_major, tb0, jbeg, jend,
                                      PartStore{part + c * 3 * n, n});
}

// Whole step in one launch (variant 4): the waves of a workgroup split all n
// sources of its 64*T targets (as variant 2 with a single chunk), reduce
// through LDS in wave order, and the same threads apply the step's kicks and
// drift (the arithmetic of k_step for one chunk).  pos_in and pos_out are
// different buffers.
struct StepKdk {
    const double* __restrict__ pos_in;
    double* __restrict__ pos_out;
    double* __restrict__ vel;
    double* __restrict__ acc;
    uint32_t* __restrict__ flags;
    int64_t n;
    double hdt, dt;
    int mode;
    __device__ __forceinline__ void operator()(int comp, int64_t p, double a) const
    {
        const int64_t e = comp * n + p;
        bool finite = __builtin_isfinite(a);
        if (mode & kStoreAcc) acc[e] = a;
        if (mode & (kClose | kOpen)) {
            double v = vel[e];
            if (mode & kClose) v = v + hdt * a;
            if (mode & kOpen) {
                v = v + hdt * a;
                const double r = pos_in[e] + dt * v;
                finite = finite && __builtin_isfinite(r);
                pos_out[e] = r;
            }
            finite = finite && __builtin_isfinite(v);
            vel[e] = v;
        }
        if (!finite && flags) atomicOr(flags, 1u);
    }
};

template <int T, int W, bool SPLIT>
__global__ __launch_bounds__(64 * W) void k_step_fused(const double* __restrict__ pos_in,
                                                       const double* __restrict__ gm, int64_t n,
                                                       const int64_t* __restrict__ nmaj,
                                                       StepKdk kdk)
{
    const int64_t n_major = SPLIT ? nmaj[0] : 0;
    const int64_t tb0 = (int64_t)blockIdx.x * 64 * T;
    force_block_s<T, W, SPLIT, true>(pos_in, gm, n, n, n_major, tb0, 0, n, kdk);
}

template <int T, int W, bool SPLIT, bool SHARE>
__global__ __launch_bounds__(64 * W) void k_force_s_batched(const double* __restrict__ pos,
                                                            const double* __restrict__ gm,
                                                            int64_t n_total,
                                                            const BatchUnit* __restrict__ units,
                                                            int64_t num_units,
                                                            const int64_t* __restrict__ nmaj,
                                                            double* __restrict__ part)
{
    constexpr int GR = SHARE ? kSGroup * W : kSGroup;
    for (int64_t u = blockIdx.x; u < num_units; u += gridDim.x) {
        const BatchUnit w = units[u];
        const int64_t n_major = SPLIT ? nmaj[w.sys] : 0;
        const int64_t n = w.n;
        const int64_t chunk_len = ((n + w.chunks - 1) / w.chunks + GR - 1) / GR * GR;
        const int64_t jbeg = (int64_t)w.chunk * chunk_len;
        const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;
        const int64_t tb0 = (int64_t)w.tblock * (SHARE ? 64 : 64 * W) * T;
        force_block_s<T, W, SPLIT, SHARE>(pos + w.body0, gm + w.body0, n_total, n, n_major, tb0,
                                          jbeg, jend,
                                          PartStore{part + (int64_t)w.chunk * 3 * n_total + w.body0,
                                                    n_total});
        if (SHARE && W > 1) __syncthreads();   // the LDS reduction buffer is reused
    }
}

template <int T, int W, bool SPLIT>
__global__ __launch_bounds__(64 * W) void k_force(const double* __restrict__ pos,
                                                  const double* __restrict__ mass, int64_t n,
                                                  const int64_t* __restrict__ nmaj,
                                                  int64_t chunk_len, double G,
                                                  double* __restrict__ part)
{
    constexpr int NT = 64 * W;
    const int64_t n_major = SPLIT ? nmaj[0] : 0;
    const int64_t tb0 = (int64_t)blockIdx.x * NT * T;
    const int64_t c = blockIdx.y;
    const int64_t jbeg = c * chunk_len;
    const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;
    force_block<T, W, SPLIT>(pos, mass, n, n, n_major, G, tb0, jbeg, jend, part + c * 3 * n);
}

// Batched: a persistent grid walks a list of work units (system, target
// block, chunk), sorted by decreasing cost on the host.  Systems are
// contiguous sub-ranges of the concatenated planes (stride n_total).
template <int T, int W, bool SPLIT>
__global__ __launch_bounds__(64 * W) void k_force_batched(const double* __restrict__ pos,
                                                          const double* __restrict__ mass,
                                                          int64_t n_total, double G,
                                                          const BatchUnit* __restrict__ units,
                                                          int64_t num_units,
                                                          const int64_t* __restrict__ nmaj,
                                                          double* __restrict__ part)
{
    constexpr int NT = 64 * W;
    for (int64_t u = blockIdx.x; u < num_units; u += gridDim.x) {
        const BatchUnit w = units[u];
        const int64_t n_major = SPLIT ? nmaj[w.sys] : 0;
        const int64_t n = w.n;
        const int64_t chunk_len = ((n + w.chunks - 1) / w.chunks + NT - 1) / NT * NT;
        const int64_t jbeg = (int64_t)w.chunk * chunk_len;
        const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;
        const int64_t tb0 = (int64_t)w.tblock * NT * T;
        force_block<T, W, SPLIT>(pos + w.body0, mass + w.body0, n_total, n, n_major, G, tb0,
                                 jbeg, jend, part + (int64_t)w.chunk * 3 * n_total + w.body0);
        __syncthreads();   // the LDS tile is reused by the next unit
    }
}


}  // namespace

bool tile_supported(const Tile& t)
{
    if (t.variant == 3) return t.tpl == 1 && t.waves == 16 && t.chunks >= 1 && t.chunks <= kMaxChunks;
    if (t.variant == 5) return mutual_shape_supported(t.tpl, t.waves) && t.chunks == 1;
    if (t.variant == 4)   // (16 waves of 64 would exceed the register file: spills)
        return (t.tpl == 1 || t.tpl == 2) && (t.waves == 2 || t.waves == 4 || t.waves == 8) &&
               t.chunks == 1;
    const bool tpl_ok = t.tpl == 1 || t.tpl == 2 || t.tpl == 4;
    const bool w_ok = t.waves == 1 || t.waves == 2 || t.waves == 4 || t.waves == 8;
    return tpl_ok && w_ok && t.chunks >= 1 && t.chunks <= kMaxChunks &&
           (t.variant >= 0 && t.variant <= 2);
}

int64_t chunk_length(int64_t n, const Tile& t)
{
    if (t.variant == 4) return n;
    if (t.variant == 3) {
        const int64_t S = small_slices(n, t) < 1 ? 1 : small_slices(n, t);
        return (n + S - 1) / S;
    }
    const int64_t tw = t.variant == 2 ? (int64_t)kSGroup * t.waves
                     : t.variant == 1 ? (int64_t)kSGroup : tile_width(t);
    const int64_t per = (n + t.chunks - 1) / t.chunks;
    return (per + tw - 1) / tw * tw;
}

template <int T, int W>
static hipError_t launch_tw(int precision, int variant, const double* pos, const double* mass,
                            const double* gm, int64_t n, const int64_t* nmaj, double G,
                            int64_t chunk_len, int chunks, double* part, hipStream_t s)
{
    constexpr int NT = 64 * W;
    if (variant == 1 || variant == 2) {
        const int64_t tpb = (variant == 2 ? 64 : NT) * T;
        const dim3 g1((unsigned)((n + tpb - 1) / tpb), (unsigned)chunks);
        if (variant == 1 && precision == 0)
            hipLaunchKernelGGL((k_force_s<T, W, false, false>), g1, dim3(NT), 0, s, pos, gm, n,
                               nmaj, chunk_len, part);
        else if (variant == 1)
            hipLaunchKernelGGL((k_force_s<T, W, true, false>), g1, dim3(NT), 0, s, pos, gm, n,
                               nmaj, chunk_len, part);
        else if (precision == 0)
            hipLaunchKernelGGL((k_force_s<T, W, false, true>), g1, dim3(NT), 0, s, pos, gm, n,
                               nmaj, chunk_len, part);
        else
            hipLaunchKernelGGL((k_force_s<T, W, true, true>), g1, dim3(NT), 0, s, pos, gm, n,
                               nmaj, chunk_len, part);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((n + (int64_t)NT * T - 1) / ((int64_t)NT * T)), (unsigned)chunks);
    if (precision == 0)
        hipLaunchKernelGGL((k_force<T, W, false>), grid, dim3(NT), 0, s, pos, mass, n, nmaj,
                           chunk_len, G, part);
    else
        hipLaunchKernelGGL((k_force<T, W, true>), grid, dim3(NT), 0, s, pos, mass, n, nmaj,
                           chunk_len, G, part);
    return hipGetLastError();
}

template <int T, int W>
static hipError_t launch_batched_tw(int precision, int variant, const double* pos,
                                    const double* mass, const double* gm, int64_t n_total,
                                    double G, const BatchUnit* units, int64_t num_units,
                                    const int64_t* nmaj, int grid, double* part, hipStream_t s)
{
    constexpr int NT = 64 * W;
    if (variant == 1 || variant == 2) {
        if (variant == 1 && precision == 0)
            hipLaunchKernelGGL((k_force_s_batched<T, W, false, false>), dim3(grid), dim3(NT), 0, s,
                               pos, gm, n_total, units, num_units, nmaj, part);
        else if (variant == 1)
            hipLaunchKernelGGL((k_force_s_batched<T, W, true, false>), dim3(grid), dim3(NT), 0, s,
                               pos, gm, n_total, units, num_units, nmaj, part);
        else if (precision == 0)
            hipLaunchKernelGGL((k_force_s_batched<T, W, false, true>), dim3(grid), dim3(NT), 0, s,
                               pos, gm, n_total, units, num_units, nmaj, part);
        else
            hipLaunchKernelGGL((k_force_s_batched<T, W, true, true>), dim3(grid), dim3(NT), 0, s,
                               pos, gm, n_total, units, num_units, nmaj, part);
        return hipGetLastError();
    }
    if (precision == 0)
        hipLaunchKernelGGL((k_force_batched<T, W, false>), dim3(grid), dim3(NT), 0, s, pos, mass,
                           n_total, G, units, num_units, nmaj, part);
    else
        hipLaunchKernelGGL((k_force_batched<T, W, true>), dim3(grid), dim3(NT), 0, s, pos, mass,
                           n_total, G, units, num_units, nmaj, part);
    return hipGetLastError();
}

#define NB_TILE_CASES(X) \
    X(1, 1) X(1, 2) X(1, 4) X(1, 8) X(2, 1) X(2, 2) X(2, 4) X(2, 8) X(4, 1) X(4, 2) X(4, 4) X(4, 8)

int effective_chunks(int64_t n, const Tile& t)
{
    if (t.variant == 5) return mutual_slots(n, t.tpl, t.waves);
    const int64_t L = chunk_length(n, t);
    return (int)((n + L - 1) / L);
}

hipError_t launch_force(int precision, const Tile& tile, const double* pos, const double* mass,
                        const double* gm, int64_t n, const int64_t* nmaj, double G, double* part,
                        hipStream_t s)
{
    if (tile.variant == 5)
        return launch_force_mutual(precision, tile.tpl, tile.waves, pos, gm, n, nmaj, part, s);
    if ((tile.variant != 0 && !gm) || tile.variant >= 3) return hipErrorInvalidValue;
    const int64_t L = chunk_length(n, tile);
    const int chunks = effective_chunks(n, tile);
#define NB_CASE(TT, WW)                                                                  \
    if (tile.tpl == TT && tile.waves == WW)                                              \
        return launch_tw<TT, WW>(precision, tile.variant, pos, mass, gm, n, nmaj, G, L, chunks, \
                                 part, s);
    NB_TILE_CASES(NB_CASE)
#undef NB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_force_batched(int precision, const Tile& tile, const double* pos,
                                const double* mass, const double* gm, int64_t n_total, double G,
                                const BatchUnit* units, int64_t num_units, const int64_t* nmaj,
                                int grid, double* part, hipStream_t s)
{
    if ((tile.variant != 0 && !gm) || tile.variant >= 3) return hipErrorInvalidValue;
#define NB_CASE(TT, WW)                                                                   \
    if (tile.tpl == TT && tile.waves == WW)                                               \
        return launch_batched_tw<TT, WW>(precision, tile.variant, pos, mass, gm, n_total, G, \
                                         units, num_units, nmaj, grid, part, s);
    NB_TILE_CASES(NB_CASE)
#undef NB_CASE
    return hipErrorInvalidValue;
}

template <int T, int W>
static hipError_t step_fused_tw(int precision, const double* pos_in, const double* gm, int64_t n,
                                const int64_t* nmaj, const StepKdk& kdk, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 64 * T - 1) / (64 * T)));
    if (precision == 0)
        hipLaunchKernelGGL((k_step_fused<T, W, false>), grid, dim3(64 * W), 0, s, pos_in, gm, n,
                           nmaj, kdk);
    else
        hipLaunchKernelGGL((k_step_fused<T, W, true>), grid, dim3(64 * W), 0, s, pos_in, gm, n,
                           nmaj, kdk);
    return hipGetLastError();
}

hipError_t launch_step_fused(int precision, const Tile& tile, const double* pos_in,
                             double* pos_out, double* vel, const double* gm, int64_t n,
                             const int64_t* nmaj, double dt, int mode, double* acc,
                             uint32_t* flags, hipStream_t s)
{
    if (tile.variant != 4 || !gm || (precision == 1 && !nmaj) ||
        ((mode & kStoreAcc) && !acc) || ((mode & (kClose | kOpen)) && !vel) ||
        ((mode & kOpen) && (!pos_out || pos_out == pos_in)))
        return hipErrorInvalidValue;
    const StepKdk kdk{pos_in, pos_out, vel, acc, flags, n, 0.5 * dt, dt, mode};
#define NB_CASE(TT, WW) \
    if (tile.tpl == TT && tile.waves == WW) return step_fused_tw<TT, WW>(precision, pos_in, gm, n, nmaj, kdk, s);
    NB_CASE(1, 2) NB_CASE(1, 4) NB_CASE(1, 8) NB_CASE(2, 2) NB_CASE(2, 4) NB_CASE(2, 8)
#undef NB_CASE
    return hipErrorInvalidValue;
}

}  // namespace nb
