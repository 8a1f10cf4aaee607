// Force pass of Eq. (1) with each unordered pair evaluated once (Newton's
// third law; tile variant 5): the pair's factor f = |d|^-3 serves both
// a_i += G m_j f d and a_j -= G m_i f d.  In FP64 that is about 23 vector
// instructions per unordered pair with four targets per lane, against 2 x 17
// for the two ordered pairs.
//
// Bodies are cut into blocks of 64 and the blocks into "ranges" of kMM = 4.
// Workgroup (g, r), r >= g, takes range g as its targets and range r as its
// sources, whose four blocks it stages in LDS.  Each of its KMW waves holds
// KMT target blocks of range g (one body of each per lane); see MutualShape
// for how the waves split the (target block, source block) tiles between
// them.  In phase p wave w works on source block (w + p) mod 4, so in every
// phase the waves touch different source blocks.
//
// Within a tile, each row of 16 lanes meets each group of 16 sources in turn
// (sub-phase q: group (row + q) mod 4) and, within a group, lane c pairs with
// source (c + k) mod 16 at step k; the reaction sum of that source travels with
// it from lane to lane inside the row (a DPP rotation, no LDS round trip), so
// after 16 steps each lane holds the reactions on its starting source, which
// it adds to the block's reaction sums in LDS (in a fixed order: the result
// is deterministic).
// Tiles below the diagonal (source block < target block) are skipped; on the
// diagonal the tile is evaluated one way only, over all 63 other sources.
//
// Split form (SPLIT): bodies are in class order, the n_major heavy ones
// first.  A wave whose target blocks start below the first block free of
// heavy bodies evaluates its tiles in FP64 as above (both directions, so the
// reactions of heavy targets on light sources and every term of a heavy
// source are FP64).  Every other tile pairs light targets with light sources
// and is evaluated in FP32: FP64 displacement rounded to FP32, FP32 rsqrt,
// FP32 terms both ways; the 16 terms of one sub-phase (a block of 16 sources
// for a target, of 16 targets for a reaction) are summed in FP32 and each
// block sum is added to the FP64 accumulators.
//
// Output: one partial per (body, range) in the chunk layout of the other force
// passes, so the ordinary step epilogue adds them in slot order.  Workgroup
// (g, r), r > g, writes its targets' accelerations to slot r and the reactions
// on its sources to slot g; workgroup (g, g) adds the two for each of its
// bodies and writes slot g.  A body of range R thus receives slot s < R as a
// source, slot s > R as a target and slot R from the diagonal workgroup:
// every slot exactly once.  An ensemble runs the same workgroups per system,
// listed as units (system, g, r), on planes spanning all systems.
#include "common.hpp"
#include "pair_math.hpp"

namespace nb {
namespace {

using namespace pm;

constexpr int kMM = 4;   // blocks per range (source blocks per workgroup, target blocks too)

// Padding bodies: massless, far away and at distinct points, so every term
// they take part in is a finite zero (or goes to a body that is not stored).
constexpr double kPadBase = 1.0e18;
constexpr double kPadStep = 1.0e13;

struct Body {
    double x, y, z, gm;
};

// Body i of a system of n bodies whose coordinate planes are `stride` apart.
__device__ __forceinline__ Body load_body(const double* __restrict__ pos,
                                          const double* __restrict__ gm, int64_t n,
                                          int64_t stride, int64_t i)
{
    Body b;
    if (i < n) {
        b.x = pos[i];
        b.y = pos[stride + i];
        b.z = pos[2 * stride + i];
        b.gm = gm[i];
    } else {
        b.x = kPadBase + kPadStep * (double)i;
        b.y = kPadBase;
        b.z = kPadBase;
        b.gm = 0.0;
    }
    return b;
}

// Rotation of a double within each row of 16 lanes: lane c receives the value
// of lane (c + 1) mod 16 (DPP row_ror by 15, on both 32-bit halves).
__device__ __forceinline__ double row_next(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x12F, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x12F, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ float row_next32(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x12F,
                                                              0xF, 0xF, true));
}

// The FP32 form of tile_sweep (light targets, light sources): per target the
// 16 terms of a sub-phase are summed in FP32 and the sum is added to the
// FP64 accumulator; the reaction of a row travels as FP32 and its 16-term sum
// is added to the FP64 reaction sums in LDS.
template <int KMT, int NSYM, bool DIAG>
__device__ __forceinline__ void tile_sweep32(const double* __restrict__ sx,
                                             const double* __restrict__ sy,
                                             const double* __restrict__ sz,
                                             const float* __restrict__ sgf,
                                             double* __restrict__ ra, int lane,
                                             const Body (&tg)[KMT], const float (&tgf)[KMT],
                                             double (&ax)[KMT], double (&ay)[KMT],
                                             double (&az)[KMT])
{
    constexpr bool kReact = NSYM > 0;
    const int row = lane >> 4;
    const int col = lane & 15;
    for (int q = 0; q < 4; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;
        float bx[KMT], by[KMT], bz[KMT];
#pragma unroll
        for (int t = 0; t < KMT; ++t) { bx[t] = 0.f; by[t] = 0.f; bz[t] = 0.f; }
        float rx = 0.f, ry = 0.f, rz = 0.f;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int jj = 32 * grp + col + k;
            const double jx = sx[jj], jy = sy[jj], jz = sz[jj];
            const float jg = sgf[jj];
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                if (t > NSYM || (t == NSYM && !DIAG)) continue;
                if (t == NSYM && q == 0 && k == 0) continue;   // the target itself
                const float dx = (float)(jx - tg[t].x);
                const float dy = (float)(jy - tg[t].y);
                const float dz = (float)(jz - tg[t].z);
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                const float y = __builtin_amdgcn_rsqf(r2);
                const float f = y * y * y;   // |d|^-3
                const float fi = jg * f;
                bx[t] = __builtin_fmaf(fi, dx, bx[t]);
                by[t] = __builtin_fmaf(fi, dy, by[t]);
                bz[t] = __builtin_fmaf(fi, dz, bz[t]);
                if (t < NSYM) {
                    const float fj = tgf[t] * f;
                    rx = __builtin_fmaf(-fj, dx, rx);
                    ry = __builtin_fmaf(-fj, dy, ry);
                    rz = __builtin_fmaf(-fj, dz, rz);
                }
            }
            if (kReact) {
                rx = row_next32(rx);
                ry = row_next32(ry);
                rz = row_next32(rz);
            }
        }
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            ax[t] += (double)bx[t];
            ay[t] += (double)by[t];
            az[t] += (double)bz[t];
        }
        if (kReact) {
            ra[home] += (double)rx;
            ra[64 + home] += (double)ry;
            ra[128 + home] += (double)rz;
        }
    }
}

// One tile sweep: the KMT targets of this lane (target blocks I0 .. I0+KMT-1)
// against one source block J staged in LDS as four groups of 16 sources,
// each stored twice in a row (s*[32*grp + i], i < 32).  Targets t < NSYM lie
// below J (both directions), target NSYM is J itself if DIAG (one direction,
// without the self pair), the rest lie above J (nothing to do).  Lane (row R,
// column c) pairs with source 16*grp + (c + k) mod 16 at step k of sub-phase
// q, grp = (R + q) mod 4; the reaction on that source rotates within the row
// (DPP, no LDS round trip) and after 16 steps is added to the block's
// reaction sums in LDS (`ra`, three planes of 64).  Rows work on different
// groups, so these adds never collide.
template <int KMT, int NSYM, bool DIAG>
__device__ __forceinline__ void tile_sweep(const double* __restrict__ sx,
                                           const double* __restrict__ sy,
                                           const double* __restrict__ sz,
                                           const double* __restrict__ sg,
                                           double* __restrict__ ra, int lane,
                                           const Body (&tg)[KMT], double (&ax)[KMT],
                                           double (&ay)[KMT], double (&az)[KMT],
                                           const PolyConst& c)
{
    constexpr bool kReact = NSYM > 0;
    const int row = lane >> 4;
    const int col = lane & 15;
    for (int q = 0; q < 4; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;     // the source this lane starts (and ends) with
        double rx = 0.0, ry = 0.0, rz = 0.0;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int jj = 32 * grp + col + k;
            const double jx = sx[jj], jy = sy[jj], jz = sz[jj], jg = sg[jj];
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                if (t > NSYM || (t == NSYM && !DIAG)) continue;
                if (t == NSYM && q == 0 && k == 0) continue;   // the target itself
                const double dx = jx - tg[t].x;
                const double dy = jy - tg[t].y;
                const double dz = jz - tg[t].z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double f = gm_rinv3_f64(r2, 1.0, c);   // |d|^-3
                const double fi = jg * f;
                ax[t] = __builtin_fma(fi, dx, ax[t]);
                ay[t] = __builtin_fma(fi, dy, ay[t]);
                az[t] = __builtin_fma(fi, dz, az[t]);
                if (t < NSYM) {   // reaction on the source
                    const double fj = tg[t].gm * f;
                    rx = __builtin_fma(-fj, dx, rx);
                    ry = __builtin_fma(-fj, dy, ry);
                    rz = __builtin_fma(-fj, dz, rz);
                }
            }
            if (kReact) {
                rx = row_next(rx);
                ry = row_next(ry);
                rz = row_next(rz);
            }
        }
        if (kReact) {
            ra[home] += rx;
            ra[64 + home] += ry;
            ra[128 + home] += rz;
        }
    }
}

// Workgroup shapes: KMW waves, KMT target blocks per wave.  With KMT * KMW =
// kMM each wave holds its own target blocks and visits all four source
// blocks; with KMW = kMM and KMT > 1, KMT waves spaced kMM / KMT apart hold
// the same target blocks and split the source blocks between them, and
// their partial sums are added at the end in wave order.  In phase p wave w
// works on source block (w + p) mod kMM, so no two waves share one.
template <int KMT, int KMW>
struct MutualShape {
    static constexpr int kSets = kMM / KMT;          // target sets (of KMT blocks)
    static constexpr int kShare = KMT * KMW / kMM;   // waves per target set
    static constexpr int kPhases = kMM / kShare;     // source blocks per wave
    static_assert(kSets * KMT == kMM && kShare * kMM == KMT * KMW, "tile the range");
    static_assert(kShare == 1 || KMW == kMM, "waves sharing targets are kMM / KMT apart");
};

template <int KMT>
__device__ __forceinline__ void sweep_dispatch(int d, const double* px, const double* py,
                                               const double* pz, const double* pg, double* ra,
                                               int lane, const Body (&tg)[KMT],
                                               double (&ax)[KMT], double (&ay)[KMT],
                                               double (&az)[KMT], const PolyConst& c)
{
    // d = J - I0: targets I0 + t < J for t < d, I0 + d == J
    if (d >= KMT) {
        tile_sweep<KMT, KMT, false>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
        return;
    }
    switch (d) {
    case 0: tile_sweep<KMT, 0, true>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c); break;
    case 1: tile_sweep<KMT, (KMT > 1 ? 1 : 0), true>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c); break;
    case 2: tile_sweep<KMT, (KMT > 2 ? 2 : 0), true>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c); break;
    case 3: tile_sweep<KMT, (KMT > 3 ? 3 : 0), true>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c); break;
    default: break;
    }
}

template <int KMT>
__device__ __forceinline__ void sweep_dispatch32(int d, const double* px, const double* py,
                                                 const double* pz, const float* pg, double* ra,
                                                 int lane, const Body (&tg)[KMT],
                                                 const float (&tgf)[KMT], double (&ax)[KMT],
                                                 double (&ay)[KMT], double (&az)[KMT])
{
    if (d >= KMT) {
        tile_sweep32<KMT, KMT, false>(px, py, pz, pg, ra, lane, tg, tgf, ax, ay, az);
        return;
    }
    switch (d) {
    case 0: tile_sweep32<KMT, 0, true>(px, py, pz, pg, ra, lane, tg, tgf, ax, ay, az); break;
    case 1: tile_sweep32<KMT, (KMT > 1 ? 1 : 0), true>(px, py, pz, pg, ra, lane, tg, tgf, ax, ay, az); break;
    case 2: tile_sweep32<KMT, (KMT > 2 ? 2 : 0), true>(px, py, pz, pg, ra, lane, tg, tgf, ax, ay, az); break;
    case 3: tile_sweep32<KMT, (KMT > 3 ? 3 : 0), true>(px, py, pz, pg, ra, lane, tg, tgf, ax, ay, az); break;
    default: break;
    }
}

// Workgroup (g, r) of a system of n bodies: pos, gm and part start at the
// system's first body, coordinate and partial planes are `stride` apart
// (partial slot c of component k of body i at part[(3c + k) stride + i]).
template <int KMT, int KMW, bool SPLIT>
__device__ __forceinline__ void mutual_unit(const double* __restrict__ pos,
                                            const double* __restrict__ gm, int64_t n,
                                            int64_t stride, int64_t n_major, int g, int r,
                                            double* __restrict__ part)
{
    using Shape = MutualShape<KMT, KMW>;
    __shared__ double sx[kMM][128], sy[kMM][128], sz[kMM][128], sg[kMM][128];
    __shared__ float sgf[SPLIT ? kMM : 1][128];
    __shared__ double racc[kMM][3][64];
    __shared__ double comb[Shape::kShare > 1 ? Shape::kShare - 1 : 1][Shape::kSets][KMT][3][64];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int set = w % Shape::kSets;   // this wave's target set
    const int h = w / Shape::kSets;     // its rank among the waves sharing the set
    const int nb = (int)((n + 63) / 64);
    const int I0 = g * kMM + set * KMT;   // this wave's target blocks I0 .. I0 + KMT - 1
    const int J0 = r * kMM;               // the workgroup's source blocks J0 .. J0 + 3
    const int64_t plane = 3 * stride;

    Body tg[KMT];
    double ax[KMT], ay[KMT], az[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        tg[t] = load_body(pos, gm, n, stride, (int64_t)(I0 + t) * 64 + lane);
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
    }

    // stage the source blocks (wave w: blocks w, w + KMW, ...): four groups
    // of 16, each twice in a row
    for (int jb = w; jb < kMM; jb += KMW) {
        const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
        const Body b = load_body(pos, gm, n, stride, j);
        const int a0 = 32 * (lane >> 4) + (lane & 15);
        sx[jb][a0] = b.x; sx[jb][a0 + 16] = b.x;
        sy[jb][a0] = b.y; sy[jb][a0 + 16] = b.y;
        sz[jb][a0] = b.z; sz[jb][a0 + 16] = b.z;
        sg[jb][a0] = b.gm; sg[jb][a0 + 16] = b.gm;
        if (SPLIT) {
            sgf[jb][a0] = (float)b.gm;
            sgf[jb][a0 + 16] = (float)b.gm;
        }
        racc[jb][0][lane] = 0.0;
        racc[jb][1][lane] = 0.0;
        racc[jb][2][lane] = 0.0;
    }
    float tgf[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) tgf[t] = (float)tg[t].gm;
    // split form: waves whose target blocks start below the first block
    // free of heavy bodies stay in FP64
    const bool fp32 = SPLIT && I0 >= (int)((n_major + 63) / 64);
    __syncthreads();

    if (fp32) {
        for (int p = 0; p < Shape::kPhases; ++p) {
            const int jb = (w + p) % kMM;
            const int J = J0 + jb;
            if (J < nb && J >= I0)
                sweep_dispatch32<KMT>(J - I0, sx[jb], sy[jb], sz[jb], sgf[SPLIT ? jb : 0],
                                      &racc[jb][0][0], lane, tg, tgf, ax, ay, az);
            __syncthreads();
        }
    } else {
        const PolyConst c = {vreg_const(1.875), vreg_const(1.5)};
        for (int p = 0; p < Shape::kPhases; ++p) {
            const int jb = (w + p) % kMM;
            const int J = J0 + jb;
            if (J < nb && J >= I0)
                sweep_dispatch<KMT>(J - I0, sx[jb], sy[jb], sz[jb], sg[jb], &racc[jb][0][0],
                                    lane, tg, ax, ay, az, c);
            __syncthreads();
        }
    }

    if (Shape::kShare > 1) {
        // the target sums of the waves sharing a set (one buffer per set and
        // rank), added in wave order
        if (h > 0) {
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                comb[h - 1][set][t][0][lane] = ax[t];
                comb[h - 1][set][t][1][lane] = ay[t];
                comb[h - 1][set][t][2][lane] = az[t];
            }
        }
        __syncthreads();
        if (h == 0) {
            for (int o = 0; o < Shape::kShare - 1; ++o) {
#pragma unroll
                for (int t = 0; t < KMT; ++t) {
                    ax[t] += comb[o][set][t][0][lane];
                    ay[t] += comb[o][set][t][1][lane];
                    az[t] += comb[o][set][t][2][lane];
                }
            }
        }
    }

    if (r > g) {
        // targets' partials to slot r, the sources' reactions to slot g
        if (h == 0) {
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                const int64_t i = (int64_t)(I0 + t) * 64 + lane;
                if (i < n) {
                    double* pt = part + (int64_t)r * plane;
                    pt[i] = ax[t];
                    pt[stride + i] = ay[t];
                    pt[2 * stride + i] = az[t];
                }
            }
        }
        for (int jb = w; jb < kMM; jb += KMW) {
            const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
            if (j < n) {
                double* ps = part + (int64_t)g * plane;
                ps[j] = racc[jb][0][lane];
                ps[stride + j] = racc[jb][1][lane];
                ps[2 * stride + j] = racc[jb][2][lane];
            }
        }
    } else if (h == 0) {
        // the diagonal workgroup: targets and sources are the same blocks;
        // each body's partial and the reaction on it, added in that order
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int64_t i = (int64_t)(I0 + t) * 64 + lane;
            const int jb = set * KMT + t;
            if (i < n) {
                double* pt = part + (int64_t)g * plane;
                pt[i] = ax[t] + racc[jb][0][lane];
                pt[stride + i] = ay[t] + racc[jb][1][lane];
                pt[2 * stride + i] = az[t] + racc[jb][2][lane];
            }
        }
    }
}

template <int KMT, int KMW, bool SPLIT>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual(const double* __restrict__ pos,
                                                           const double* __restrict__ gm,
                                                           int64_t n,
                                                           const int64_t* __restrict__ nmaj,
                                                           int ranges, double* __restrict__ part)
{
    // blockIdx.x enumerates the pairs (g, r), r >= g, row by row: row g
    // starts at S(g) = g*ranges - g(g-1)/2; g from the quadratic's root,
    // corrected by at most a step either way for rounding
    const int64_t bid = blockIdx.x;
    const double R2 = 2.0 * ranges + 1.0;
    int g = (int)((R2 - __builtin_sqrt(R2 * R2 - 8.0 * (double)bid)) * 0.5);
    g = g < 0 ? 0 : (g > ranges - 1 ? ranges - 1 : g);
    auto row_start = [&](int64_t x) { return x * ranges - x * (x - 1) / 2; };
    if (g > 0 && row_start(g) > bid) --g;
    if (g < ranges - 1 && row_start(g + 1) <= bid) ++g;
    const int r = (int)(bid - row_start(g)) + g;
    mutual_unit<KMT, KMW, SPLIT>(pos, gm, n, n, SPLIT ? nmaj[0] : 0, g, r, part);
}

// The ensemble: one workgroup per unit (system, g = tblock, r = chunk) of the
// work list; the partial planes span all systems (stride n_total).
template <int KMT, int KMW, bool SPLIT>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual_batched(
    const double* __restrict__ pos, const double* __restrict__ gm, int64_t n_total,
    const BatchUnit* __restrict__ units, const int64_t* __restrict__ nmaj,
    double* __restrict__ part)
{
    const BatchUnit u = units[blockIdx.x];
    mutual_unit<KMT, KMW, SPLIT>(pos + u.body0, gm + u.body0, u.n, n_total,
                                 SPLIT ? nmaj[u.sys] : 0, u.tblock, u.chunk, part + u.body0);
}

}  // namespace

int mutual_ranges(int64_t n) { return (int)((((n + 63) / 64) + kMM - 1) / kMM); }

bool mutual_shape_supported(int tpl, int waves)
{
    return (tpl == 1 && waves == 4) || (tpl == 2 && waves == 2) || (tpl == 2 && waves == 4) ||
           (tpl == 4 && waves == 4);
}

template <bool SPLIT>
static void launch_mutual_shape(int tpl, int waves, dim3 grid, const double* pos, const double* gm,
                                int64_t n, const int64_t* nmaj, int ranges, double* part,
                                hipStream_t s)
{
    const dim3 block((unsigned)(64 * waves));
    if (tpl == 1)
        hipLaunchKernelGGL((k_force_mutual<1, 4, SPLIT>), grid, block, 0, s, pos, gm, n, nmaj,
                           ranges, part);
    else if (tpl == 2 && waves == 2)
        hipLaunchKernelGGL((k_force_mutual<2, 2, SPLIT>), grid, block, 0, s, pos, gm, n, nmaj,
                           ranges, part);
    else if (tpl == 2)
        hipLaunchKernelGGL((k_force_mutual<2, 4, SPLIT>), grid, block, 0, s, pos, gm, n, nmaj,
                           ranges, part);
    else
        hipLaunchKernelGGL((k_force_mutual<4, 4, SPLIT>), grid, block, 0, s, pos, gm, n, nmaj,
                           ranges, part);
}

template <bool SPLIT>
static void launch_mutual_batched_shape(int tpl, int waves, dim3 grid, const double* pos,
                                        const double* gm, int64_t n_total, const BatchUnit* units,
                                        const int64_t* nmaj, double* part, hipStream_t s)
{
    const dim3 block((unsigned)(64 * waves));
    if (tpl == 1)
        hipLaunchKernelGGL((k_force_mutual_batched<1, 4, SPLIT>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else if (tpl == 2 && waves == 2)
        hipLaunchKernelGGL((k_force_mutual_batched<2, 2, SPLIT>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else if (tpl == 2)
        hipLaunchKernelGGL((k_force_mutual_batched<2, 4, SPLIT>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else
        hipLaunchKernelGGL((k_force_mutual_batched<4, 4, SPLIT>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
}

hipError_t launch_force_mutual_batched(int precision, int tpl, int waves, const double* pos,
                                       const double* gm, int64_t n_total, const BatchUnit* units,
                                       int64_t num_units, const int64_t* nmaj, double* part,
                                       hipStream_t s)
{
    if (!gm || !units || num_units < 1 || !mutual_shape_supported(tpl, waves) ||
        (precision != 0 && !nmaj))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)num_units);
    if (precision == 0)
        launch_mutual_batched_shape<false>(tpl, waves, grid, pos, gm, n_total, units, nullptr,
                                           part, s);
    else
        launch_mutual_batched_shape<true>(tpl, waves, grid, pos, gm, n_total, units, nmaj, part,
                                          s);
    return hipGetLastError();
}

hipError_t launch_force_mutual(int precision, int tpl, int waves, const double* pos,
                               const double* gm, int64_t n, const int64_t* nmaj, double* part,
                               hipStream_t s)
{
    if (!gm || n < 1 || !mutual_shape_supported(tpl, waves) || (precision != 0 && !nmaj))
        return hipErrorInvalidValue;
    const int64_t ranges = mutual_ranges(n);
    const dim3 grid((unsigned)(ranges * (ranges + 1) / 2));
    if (precision == 0)
        launch_mutual_shape<false>(tpl, waves, grid, pos, gm, n, nullptr, (int)ranges, part, s);
    else
        launch_mutual_shape<true>(tpl, waves, grid, pos, gm, n, nmaj, (int)ranges, part, s);
    return hipGetLastError();
}

}  // namespace nb
