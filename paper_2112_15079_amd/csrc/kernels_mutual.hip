// Force pass of Eq. (1) with each unordered pair evaluated once (Newton's
// third law; tile variant 5): the pair's factor f = |d|^-3 serves both
// a_i += G m_j f d and a_j -= G m_i f d.  (The adjoint's transpose-Jacobian
// pass with the same schedule follows at the end of the file.)  In FP64 that is about 23 vector
// instructions per unordered pair with four targets per lane, against 2 x 17
// for the two ordered pairs.
//
// Bodies are cut into blocks of 64 and the blocks into "ranges" of kMM = 4.
// Workgroup (g, r), r >= g, takes range g as its targets and range r as its
// sources and stages the four blocks of each in LDS (each body loaded once
// per workgroup).  Each of its KMW waves then holds KMT target blocks of
// range g in registers (one body of each per lane); see MutualShape
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
//
// The last round (single systems, shape (4, 4)): the pass takes about one
// period per ceil(pairs / 256) rounds of workgroups, one per CU per round.
// When the pairs past the last whole round are few (at most 128), those
// pairs are each run as two workgroups of half the work, so the partly
// filled round costs half a period: a half holds all four target blocks
// (four per lane) against all four source blocks, one per wave, over two
// of the four sub-phases (0-1, 2-3), at the whole pair's cost per pair.
// Both halves reach every target and every source, so the second half
// writes its target sums and its reactions to extra slots.  The split pairs
// are those on the super-diagonals r - g = 1 .. D - 1 and the first kD of
// r - g = D; the extra slots of pair (g, g + d) are R + d - 1 (reactions)
// and R + D + d - 1 (targets), and the diagonal workgroup of each range
// writes zeros to the extra slots that no split pair fills, so every body
// still receives each of its R + 2D slots exactly once.
#include "common.hpp"
#include "pair_math.hpp"

// Marks for the test instruments (tests/host), which define the macro
// before including this file; in the library it expands to nothing.
#ifndef NB_MUTUAL_MARK
#define NB_MUTUAL_MARK(k)
#endif

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

// A source block in LDS: four groups of 16 sources; group grp holds the x,
// y, z and G m planes of 32 entries each (its 16 sources twice in a row) at
// kGrp * grp + 32 * plane, so that one base address with immediate offsets
// reaches all four planes of a group.
constexpr int kGrp = 128;
constexpr int kSrcBlock = 4 * kGrp;

__device__ __forceinline__ void stage_source(double* __restrict__ sb, int lane, const Body& b)
{
    const int a0 = kGrp * (lane >> 4) + (lane & 15);
    sb[a0] = b.x; sb[a0 + 16] = b.x;
    sb[a0 + 32] = b.y; sb[a0 + 48] = b.y;
    sb[a0 + 64] = b.z; sb[a0 + 80] = b.z;
    sb[a0 + 96] = b.gm; sb[a0 + 112] = b.gm;
}

// The FP32 form of tile_sweep (light targets, light sources): per target the
// 16 terms of a sub-phase are summed in FP32 and the sum is added to the
// FP64 accumulator; the reaction of a row travels as FP32 and its 16-term sum
// is added to the FP64 reaction sums in LDS.
template <int KMT, int NSYM, bool DIAG, int Q0 = 0, int Q1 = 4>
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
    for (int q = Q0; q < Q1; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;
        float bx[KMT], by[KMT], bz[KMT];
#pragma unroll
        for (int t = 0; t < KMT; ++t) { bx[t] = 0.f; by[t] = 0.f; bz[t] = 0.f; }
        float rx = 0.f, ry = 0.f, rz = 0.f;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int jj = kGrp * grp + col + k;
            const double jx = sx[jj], jy = sy[jj], jz = sz[jj];
            const float jg = sgf[32 * grp + col + k];
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

// Kahan's compensated addition of the FP32 product a * b: s + a b with the
// rounding error carried in c (the product rounded once, inside the FMA).
__device__ __forceinline__ void kahan_fma(float& s, float& c, float a, float b)
{
    const float y = __builtin_fmaf(a, b, -c);
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Per-lane FP32 Kahan sums of the three components.
struct Kahan3 {
    float s[3], c[3];
};

__device__ __forceinline__ void k3_zero(Kahan3& k)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) { k.s[i] = 0.f; k.c[i] = 0.f; }
}

// The compensated split form (precision 2): the FP64 displacement d and
// squared distance r2; |d|^-3 = y^3 from the FP32 reciprocal square root y0
// of float(r2) refined by one Newton step in FP64, y = y0 (1 + e / 2),
// e = 1 - r2 y0^2 (for every pair); a light source's term on a target (a
// light target's reaction on a source) rounded to FP32 as
// float(G m f) * float(d) and added to an FP32 Kahan sum; a heavy body's
// term added in FP64.  MIXED: bodies of either class may meet in this tile
// (class by index: below n_major is heavy); otherwise every body is light
// and only the FP32 sums are kept.  The target sums (ka) run over the whole
// sweep of the workgroup; each reaction's (16 targets of a row) is added to
// the FP64 reaction sums in LDS as s - c.  Tile geometry as tile_sweep.
template <int KMT, int NSYM, bool DIAG, bool MIXED, int Q0 = 0, int Q1 = 4>
__device__ __forceinline__ void tile_sweep_comp(const double* __restrict__ sx,
                                                const double* __restrict__ sy,
                                                const double* __restrict__ sz,
                                                const double* __restrict__ sg,
                                                double* __restrict__ ra, int lane,
                                                const Body (&tg)[KMT], const bool (&theavy)[KMT],
                                                int64_t jbase, int64_t n_major,
                                                double (&ax)[KMT], double (&ay)[KMT],
                                                double (&az)[KMT], Kahan3 (&ka)[KMT])
{
    constexpr bool kReact = NSYM > 0;
    const int row = lane >> 4;
    const int col = lane & 15;
    for (int q = Q0; q < Q1; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;
        double rx = 0.0, ry = 0.0, rz = 0.0;
        Kahan3 kr;
        k3_zero(kr);
#pragma unroll 2
        for (int k = 0; k < 16; ++k) {
            const int jj = kGrp * grp + col + k;
            const double jx = sx[jj], jy = sy[jj], jz = sz[jj], jg = sg[jj];
            const bool jheavy = MIXED && jbase + 16 * grp + ((col + k) & 15) < n_major;
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                if (t > NSYM || (t == NSYM && !DIAG)) continue;
                if (t == NSYM && q == 0 && k == 0) continue;   // the target itself
                const double dx = jx - tg[t].x;
                const double dy = jy - tg[t].y;
                const double dz = jz - tg[t].z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double y0 = (double)__builtin_amdgcn_rsqf((float)r2);
                const double e = __builtin_fma(-r2, y0 * y0, 1.0);
                const double y = __builtin_fma(y0 * e, 0.5, y0);
                const double f = y * y * y;   // |d|^-3
                const float dx32 = (float)dx, dy32 = (float)dy, dz32 = (float)dz;
                const double fi = jg * f;
                if (MIXED) {
                    const double wi = jheavy ? fi : 0.0;
                    const float fi32 = jheavy ? 0.f : (float)fi;
                    ax[t] = __builtin_fma(wi, dx, ax[t]);
                    ay[t] = __builtin_fma(wi, dy, ay[t]);
                    az[t] = __builtin_fma(wi, dz, az[t]);
                    kahan_fma(ka[t].s[0], ka[t].c[0], fi32, dx32);
                    kahan_fma(ka[t].s[1], ka[t].c[1], fi32, dy32);
                    kahan_fma(ka[t].s[2], ka[t].c[2], fi32, dz32);
                } else {
                    const float fi32 = (float)fi;
                    kahan_fma(ka[t].s[0], ka[t].c[0], fi32, dx32);
                    kahan_fma(ka[t].s[1], ka[t].c[1], fi32, dy32);
                    kahan_fma(ka[t].s[2], ka[t].c[2], fi32, dz32);
                }
                if (t < NSYM) {   // reaction on the source
                    const double fj = tg[t].gm * f;
                    if (MIXED) {
                        const double wj = theavy[t] ? fj : 0.0;
                        const float fj32 = theavy[t] ? 0.f : (float)fj;
                        rx = __builtin_fma(-wj, dx, rx);
                        ry = __builtin_fma(-wj, dy, ry);
                        rz = __builtin_fma(-wj, dz, rz);
                        kahan_fma(kr.s[0], kr.c[0], -fj32, dx32);
                        kahan_fma(kr.s[1], kr.c[1], -fj32, dy32);
                        kahan_fma(kr.s[2], kr.c[2], -fj32, dz32);
                    } else {
                        const float fj32 = (float)fj;
                        kahan_fma(kr.s[0], kr.c[0], -fj32, dx32);
                        kahan_fma(kr.s[1], kr.c[1], -fj32, dy32);
                        kahan_fma(kr.s[2], kr.c[2], -fj32, dz32);
                    }
                }
            }
            if (kReact) {
                if (MIXED) {
                    rx = row_next(rx);
                    ry = row_next(ry);
                    rz = row_next(rz);
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    kr.s[i] = row_next32(kr.s[i]);
                    kr.c[i] = row_next32(kr.c[i]);
                }
            }
        }
        if (kReact) {
            ra[home] += rx + ((double)kr.s[0] - (double)kr.c[0]);
            ra[64 + home] += ry + ((double)kr.s[1] - (double)kr.c[1]);
            ra[128 + home] += rz + ((double)kr.s[2] - (double)kr.c[2]);
        }
    }
}

// One tile sweep: the KMT targets of this lane (target blocks I0 .. I0+KMT-1)
// against one source block J staged in LDS as four groups of 16 sources,
// each stored twice in a row (s*[kGrp*grp + i], i < 32).  Targets t < NSYM lie
// below J (both directions), target NSYM is J itself if DIAG (one direction,
// without the self pair), the rest lie above J (nothing to do).  Lane (row R,
// column c) pairs with source 16*grp + (c + k) mod 16 at step k of sub-phase
// q, grp = (R + q) mod 4; the reaction on that source rotates within the row
// (DPP, no LDS round trip) and after 16 steps is added to the block's
// reaction sums in LDS (`ra`, three planes of 64).  Rows work on different
// groups, so these adds never collide.
template <int KMT, int NSYM, bool DIAG, int Q0 = 0, int Q1 = 4>
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
    for (int q = Q0; q < Q1; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;     // the source this lane starts (and ends) with
        double rx = 0.0, ry = 0.0, rz = 0.0;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int jj = kGrp * grp + col + k;
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

template <int KMT, bool MIXED>
__device__ __forceinline__ void sweep_dispatch_comp(int d, const double* px, const double* py,
                                                    const double* pz, const double* pg,
                                                    double* ra, int lane, const Body (&tg)[KMT],
                                                    const bool (&th)[KMT], int64_t jbase,
                                                    int64_t n_major, double (&ax)[KMT],
                                                    double (&ay)[KMT], double (&az)[KMT],
                                                    Kahan3 (&ka)[KMT])
{
    if (d >= KMT) {
        tile_sweep_comp<KMT, KMT, false, MIXED>(px, py, pz, pg, ra, lane, tg, th, jbase, n_major,
                                                ax, ay, az, ka);
        return;
    }
    switch (d) {
    case 0: tile_sweep_comp<KMT, 0, true, MIXED>(px, py, pz, pg, ra, lane, tg, th, jbase, n_major, ax, ay, az, ka); break;
    case 1: tile_sweep_comp<KMT, (KMT > 1 ? 1 : 0), true, MIXED>(px, py, pz, pg, ra, lane, tg, th, jbase, n_major, ax, ay, az, ka); break;
    case 2: tile_sweep_comp<KMT, (KMT > 2 ? 2 : 0), true, MIXED>(px, py, pz, pg, ra, lane, tg, th, jbase, n_major, ax, ay, az, ka); break;
    case 3: tile_sweep_comp<KMT, (KMT > 3 ? 3 : 0), true, MIXED>(px, py, pz, pg, ra, lane, tg, th, jbase, n_major, ax, ay, az, ka); break;
    default: break;
    }
}

// The compensated split form's sweep of one tile by a wave holding target
// blocks I0 .. I0 + KT - 1 (light: no heavy body among them or the sources).
template <int KT>
__device__ __forceinline__ void sweep_comp(bool light, int d, int I0, int J, int lane,
                                           const double* px, const double* py, const double* pz,
                                           const double* pg, double* ra, const Body (&tg)[KT],
                                           int64_t n_major, double (&ax)[KT], double (&ay)[KT],
                                           double (&az)[KT], Kahan3 (&ka)[KT])
{
    bool th[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) th[t] = (int64_t)(I0 + t) * 64 + lane < n_major;
    if (light)
        sweep_dispatch_comp<KT, false>(d, px, py, pz, pg, ra, lane, tg, th, (int64_t)J * 64,
                                       n_major, ax, ay, az, ka);
    else
        sweep_dispatch_comp<KT, true>(d, px, py, pz, pg, ra, lane, tg, th, (int64_t)J * 64,
                                      n_major, ax, ay, az, ka);
}

// Which workgroups run whole range pairs and which run halves (see the top
// of the file).  D = 0: every pair whole.
struct MutualTail {
    int R;    // ranges
    int F;    // workgroups running whole pairs (a multiple of 256 when D > 0)
    int D;    // split pairs lie on super-diagonals 1 .. D
    int kD;   // ... on super-diagonal D only those with g < kD
};

// Split pairs in row g: (g, g + 1) .. (g, g + s(g)).
__host__ __device__ inline int mt_split_in_row(const MutualTail& t, int g)
{
    if (t.D == 0) return 0;
    const int a = t.D - 1 < t.R - 1 - g ? t.D - 1 : t.R - 1 - g;
    return a + (g < t.kD ? 1 : 0);
}

// Whole pairs in rows 0 .. g-1 (each row: R - y pairs, s(y) of them split).
__host__ __device__ inline int64_t mt_row_start(const MutualTail& t, int g)
{
    int64_t c = (int64_t)g * t.R - (int64_t)g * (g - 1) / 2;
    if (t.D == 0) return c;
    const int a = g < t.R - t.D + 1 ? g : t.R - t.D + 1;   // rows holding all D - 1
    c -= (int64_t)(t.D - 1) * a;
    for (int y = a; y < g; ++y) c -= t.R - 1 - y;
    c -= g < t.kD ? g : t.kD;
    return c;
}

// Workgroup bid -> pair (g, r) and half (-1: whole; 0, 1: the halves of a
// split pair, the second writing its reactions to extra slot xslot).
__host__ __device__ inline void mt_decode(const MutualTail& tl, int64_t bid, int& g, int& r,
                                          int& half, int& xslot)
{
    if (bid >= tl.F) {   // the halves of the split pairs, super-diagonal by super-diagonal
        const int64_t h = bid - tl.F;
        int u = (int)(h >> 1), d = 1;
        while (d < tl.D && u >= tl.R - d) {
            u -= tl.R - d;
            ++d;
        }
        g = u;
        r = u + d;
        half = (int)(h & 1);
        xslot = tl.R + d - 1;
        return;
    }
    // the whole pairs (g, r), r >= g, row by row without the split ones: row
    // g from the quadratic's root for the full triangle (row start
    // g R - g(g-1)/2), then the last row starting at or before bid
    const double R2 = 2.0 * tl.R + 1.0;
    g = (int)((R2 - __builtin_sqrt(R2 * R2 - 8.0 * (double)bid)) * 0.5);
    g = g < 0 ? 0 : (g > tl.R - 1 ? tl.R - 1 : g);
    while (g > 0 && mt_row_start(tl, g) > bid) --g;
    while (g < tl.R - 1 && mt_row_start(tl, g + 1) <= bid) ++g;
    const int idx = (int)(bid - mt_row_start(tl, g));
    r = idx == 0 ? g : g + mt_split_in_row(tl, g) + idx;
    half = -1;
    xslot = 0;
}

// Whether range pair (g, g + d), 1 <= d <= D, is split into halves.
__host__ __device__ inline bool mt_is_split(const MutualTail& tl, int g, int d)
{
    return g >= 0 && g + d <= tl.R - 1 && (d < tl.D || g < tl.kD);
}

// The decode above listed by the host for passes of at most kMapMax
// workgroups over at most 64 ranges, and handed over in the kernel's
// arguments: a workgroup then reads its entry with one load, where the
// closed form's scalar arithmetic (about 350 instructions) would delay its
// first staging loads (0.6 us of a 46 us pass at 10,425 bodies, measured).
// Entry b: g | r << 6 | (half + 1) << 12; a half's extra slot is R + r - g - 1.
// count 0: the kernel runs the closed form.
constexpr int kMapMax = 1536;
struct MutualMap {
    int32_t count;
    uint16_t e[kMapMax];
};

// Workgroup bid's pair from the list when it holds one, else by the closed form.
__device__ __forceinline__ void mt_lookup(const MutualMap& map, const MutualTail& tl, int64_t bid,
                                          int& g, int& r, int& half, int& xslot)
{
    if (map.count > 0) {
        const uint32_t v = __builtin_amdgcn_readfirstlane((uint32_t)map.e[bid]);
        g = (int)(v & 63u);
        r = (int)((v >> 6) & 63u);
        half = (int)(v >> 12) - 1;
        xslot = half >= 0 ? tl.R + (r - g) - 1 : 0;
    } else {
        mt_decode(tl, bid, g, r, half, xslot);
    }
}

// Half `half` of the split pair (g, r), r > g, by sub-phases: the four
// target blocks of range g (four per lane) against source block 4r + w in
// wave w, over sub-phases Q0 .. Q1 - 1 (half 0: 0 and 1, half 1: 2 and 3),
// so each half has the whole pair's per-pair cost and half its tiles.  Both
// halves reach every target and every source: half 0 writes the targets'
// sums to slot r and the reactions to slot g, half 1 to the extra slots
// R + D + d - 1 and R + d - 1 (xslot).  The LDS arrays are the whole pair's.
template <int PREC, int Q0, int Q1>
__device__ __forceinline__ void mutual_half_body(const double* __restrict__ pos,
                                                 const double* __restrict__ gm, int64_t n,
                                                 int64_t n_major, const MutualTail& tl, int g,
                                                 int r, int xslot, double* __restrict__ part,
                                                 double (*src)[kSrcBlock], float (*sgf)[128],
                                                 double (*racc)[3][64], double* cbuf)
{
    constexpr int KMT = 4;
    constexpr bool SPLIT = PREC == 1;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nb = (int)((n + 63) / 64);
    const int I0 = g * kMM;
    const int J = r * kMM + w;
    const int64_t plane = 3 * n;

    double ax[KMT], ay[KMT], az[KMT];
    Kahan3 ka[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
        k3_zero(ka[t]);
    }
    // wave w stages target block I0 + w and source block J
    double (*tst)[4][64] = reinterpret_cast<double (*)[4][64]>(cbuf);
    {
        const Body a = load_body(pos, gm, n, n, (int64_t)(I0 + w) * 64 + lane);
        const Body b = load_body(pos, gm, n, n, (int64_t)J * 64 + lane);
        tst[w][0][lane] = a.x;
        tst[w][1][lane] = a.y;
        tst[w][2][lane] = a.z;
        tst[w][3][lane] = a.gm;
        stage_source(src[w], lane, b);
        if (SPLIT) {
            const int a0 = 32 * (lane >> 4) + (lane & 15);
            sgf[w][a0] = (float)b.gm;
            sgf[w][a0 + 16] = (float)b.gm;
        }
        racc[w][0][lane] = 0.0;
        racc[w][1][lane] = 0.0;
        racc[w][2][lane] = 0.0;
    }
    const bool fp32 = PREC != 0 && I0 >= (int)((n_major + 63) / 64);
    __syncthreads();
    NB_MUTUAL_MARK(1);
    Body tg[KMT];
    float tgf[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        tg[t] = Body{tst[t][0][lane], tst[t][1][lane], tst[t][2][lane], tst[t][3][lane]};
        tgf[t] = (float)tg[t].gm;
    }
    if (J < nb) {   // r > g: J - I0 >= 4, every tile both ways
        const double* sb = src[w];
        if constexpr (PREC == 2) {
            bool th[KMT];
#pragma unroll
            for (int t = 0; t < KMT; ++t) th[t] = (int64_t)(I0 + t) * 64 + lane < n_major;
            if (fp32)
                tile_sweep_comp<KMT, KMT, false, false, Q0, Q1>(sb, sb + 32, sb + 64, sb + 96,
                                                                &racc[w][0][0], lane, tg, th,
                                                                (int64_t)J * 64, n_major, ax, ay,
                                                                az, ka);
            else
                tile_sweep_comp<KMT, KMT, false, true, Q0, Q1>(sb, sb + 32, sb + 64, sb + 96,
                                                               &racc[w][0][0], lane, tg, th,
                                                               (int64_t)J * 64, n_major, ax, ay,
                                                               az, ka);
        } else if (PREC == 1 && fp32) {
            tile_sweep32<KMT, KMT, false, Q0, Q1>(sb, sb + 32, sb + 64, sgf[SPLIT ? w : 0],
                                                  &racc[w][0][0], lane, tg, tgf, ax, ay, az);
        } else {
            tile_sweep<KMT, KMT, false, Q0, Q1>(sb, sb + 32, sb + 64, sb + 96, &racc[w][0][0],
                                                lane, tg, ax, ay, az,
                                                PolyConst{vreg_const(1.875), vreg_const(1.5)});
        }
    }
    NB_MUTUAL_MARK(2);
    if (PREC == 2) {
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            ax[t] += (double)ka[t].s[0] - (double)ka[t].c[0];
            ay[t] += (double)ka[t].s[1] - (double)ka[t].c[1];
            az[t] += (double)ka[t].s[2] - (double)ka[t].c[2];
        }
    }
    // the four waves' target sums, added in wave order (the buffer held the
    // staged targets: every wave has read them before this barrier)
    __syncthreads();
    double (*comb)[KMT][3][64] = reinterpret_cast<double (*)[KMT][3][64]>(cbuf);
    if (w > 0) {
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            comb[w - 1][t][0][lane] = ax[t];
            comb[w - 1][t][1][lane] = ay[t];
            comb[w - 1][t][2][lane] = az[t];
        }
    }
    __syncthreads();
    const bool second = Q0 > 0;
    if (w == 0) {
        for (int o = 0; o < 3; ++o) {
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                ax[t] += comb[o][t][0][lane];
                ay[t] += comb[o][t][1][lane];
                az[t] += comb[o][t][2][lane];
            }
        }
        const int tslot = second ? xslot + tl.D : r;
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int64_t i = (int64_t)(I0 + t) * 64 + lane;
            if (i < n) {
                double* pt = part + (int64_t)tslot * plane;
                __builtin_nontemporal_store(ax[t], &pt[i]);
                __builtin_nontemporal_store(ay[t], &pt[n + i]);
                __builtin_nontemporal_store(az[t], &pt[2 * n + i]);
            }
        }
    }
    const int64_t j = (int64_t)J * 64 + lane;
    if (j < n) {
        double* ps = part + (int64_t)(second ? xslot : g) * plane;
        __builtin_nontemporal_store(racc[w][0][lane], &ps[j]);
        __builtin_nontemporal_store(racc[w][1][lane], &ps[n + j]);
        __builtin_nontemporal_store(racc[w][2][lane], &ps[2 * n + j]);
    }
}

// Workgroup (g, r) of a system of n bodies: pos, gm and part start at the
// system's first body, coordinate and partial planes are `stride` apart
// (partial slot c of component k of body i at part[(3c + k) stride + i]).
// half >= 0 runs that half of a split pair instead (single systems, stride
// n, shape (4, 4)); the diagonal workgroup zero-fills the extra slots of
// `tl` that no split pair writes.
template <int KMT, int KMW, int PREC>
__device__ __forceinline__ void mutual_unit(const double* __restrict__ pos,
                                            const double* __restrict__ gm, int64_t n,
                                            int64_t stride, int64_t n_major, int g, int r,
                                            double* __restrict__ part, const MutualTail& tl,
                                            int half, int xslot)
{
    using Shape = MutualShape<KMT, KMW>;
    constexpr bool SPLIT = PREC == 1;   // the FP32 tiles (light sources' G m as floats)
    __shared__ double src[kMM][kSrcBlock];
    __shared__ float sgf[SPLIT ? kMM : 1][128];
    __shared__ double racc[kMM][3][64];
    // the range's target blocks at the start, the waves' target sums at the end
    constexpr int kCombD = (Shape::kShare > 1 ? Shape::kShare - 1 : 1) * Shape::kSets * KMT * 3 * 64;
    constexpr int kTgtD = kMM * 4 * 64;
    __shared__ double cbuf[kCombD > kTgtD ? kCombD : kTgtD];
    double (*comb)[Shape::kSets][KMT][3][64] =
        reinterpret_cast<double (*)[Shape::kSets][KMT][3][64]>(cbuf);
    if constexpr (KMT == 4 && KMW == 4) {
        static_assert(sizeof(cbuf) >= 3 * 4 * 3 * 64 * sizeof(double), "half-pair sums fit");
        if (half == 0) {
            mutual_half_body<PREC, 0, 2>(pos, gm, n, n_major, tl, g, r, xslot, part, src,
                                         SPLIT ? sgf : nullptr, racc, cbuf);
            return;
        }
        if (half == 1) {
            mutual_half_body<PREC, 2, 4>(pos, gm, n, n_major, tl, g, r, xslot, part, src,
                                         SPLIT ? sgf : nullptr, racc, cbuf);
            return;
        }
    }

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int set = w % Shape::kSets;   // this wave's target set
    const int h = w / Shape::kSets;     // its rank among the waves sharing the set
    const int nb = (int)((n + 63) / 64);
    const int I0 = g * kMM + set * KMT;   // this wave's target blocks I0 .. I0 + KMT - 1
    const int J0 = r * kMM;               // the workgroup's source blocks J0 .. J0 + 3
    const int64_t plane = 3 * stride;

    double ax[KMT], ay[KMT], az[KMT];
    Kahan3 ka[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
        k3_zero(ka[t]);
    }

    // stage the range's target blocks and its source blocks (wave w: blocks
    // w, w + KMW, ...): the targets as planes of 64, the sources in four
    // groups of 16, each twice in a row.  Each wave then reads its own target
    // blocks from LDS: one global load of a body per workgroup, not per wave.
    double (*tst)[4][64] = reinterpret_cast<double (*)[4][64]>(cbuf);
    for (int jb = w; jb < kMM; jb += KMW) {
        const Body a = load_body(pos, gm, n, stride, (int64_t)(g * kMM + jb) * 64 + lane);
        const Body b = load_body(pos, gm, n, stride, (int64_t)(J0 + jb) * 64 + lane);
        tst[jb][0][lane] = a.x;
        tst[jb][1][lane] = a.y;
        tst[jb][2][lane] = a.z;
        tst[jb][3][lane] = a.gm;
        stage_source(src[jb], lane, b);
        if (SPLIT) {
            const int a0 = 32 * (lane >> 4) + (lane & 15);
            sgf[jb][a0] = (float)b.gm;
            sgf[jb][a0 + 16] = (float)b.gm;
        }
        racc[jb][0][lane] = 0.0;
        racc[jb][1][lane] = 0.0;
        racc[jb][2][lane] = 0.0;
    }
    // split form: waves whose target blocks start below the first block
    // free of heavy bodies stay in FP64
    const bool fp32 = PREC != 0 && I0 >= (int)((n_major + 63) / 64);
    __syncthreads();
    NB_MUTUAL_MARK(1);   // sources and targets staged, the sweep begins
    Body tg[KMT];
    float tgf[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        const int tb = set * KMT + t;
        tg[t] = Body{tst[tb][0][lane], tst[tb][1][lane], tst[tb][2][lane], tst[tb][3][lane]};
        tgf[t] = (float)tg[t].gm;
    }

    if constexpr (PREC == 2) {
        for (int p = 0; p < Shape::kPhases; ++p) {
            const int jb = (w + p) % kMM;
            const int J = J0 + jb;
            if (J < nb && J >= I0)
                sweep_comp<KMT>(fp32, J - I0, I0, J, lane, src[jb], src[jb] + 32, src[jb] + 64,
                                src[jb] + 96,
                                &racc[jb][0][0], tg, n_major, ax, ay, az, ka);
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            ax[t] += (double)ka[t].s[0] - (double)ka[t].c[0];
            ay[t] += (double)ka[t].s[1] - (double)ka[t].c[1];
            az[t] += (double)ka[t].s[2] - (double)ka[t].c[2];
        }
    } else if (fp32) {
        for (int p = 0; p < Shape::kPhases; ++p) {
            const int jb = (w + p) % kMM;
            const int J = J0 + jb;
            if (J < nb && J >= I0)
                sweep_dispatch32<KMT>(J - I0, src[jb], src[jb] + 32, src[jb] + 64, sgf[SPLIT ? jb : 0],
                                      &racc[jb][0][0], lane, tg, tgf, ax, ay, az);
            __syncthreads();
        }
    } else {
        const PolyConst c = {vreg_const(1.875), vreg_const(1.5)};
        for (int p = 0; p < Shape::kPhases; ++p) {
            const int jb = (w + p) % kMM;
            const int J = J0 + jb;
            if (J < nb && J >= I0)
                sweep_dispatch<KMT>(J - I0, src[jb], src[jb] + 32, src[jb] + 64, src[jb] + 96,
                                    &racc[jb][0][0],
                                    lane, tg, ax, ay, az, c);
            __syncthreads();
        }
    }

    NB_MUTUAL_MARK(2);   // the sweep done
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
                    __builtin_nontemporal_store(ax[t], &pt[i]);
                    __builtin_nontemporal_store(ay[t], &pt[stride + i]);
                    __builtin_nontemporal_store(az[t], &pt[2 * stride + i]);
                }
            }
        }
        for (int jb = w; jb < kMM; jb += KMW) {
            const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
            if (j < n) {
                double* ps = part + (int64_t)g * plane;
                __builtin_nontemporal_store(racc[jb][0][lane], &ps[j]);
                __builtin_nontemporal_store(racc[jb][1][lane], &ps[stride + j]);
                __builtin_nontemporal_store(racc[jb][2][lane], &ps[2 * stride + j]);
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
                __builtin_nontemporal_store(ax[t] + racc[jb][0][lane], &pt[i]);
                __builtin_nontemporal_store(ay[t] + racc[jb][1][lane], &pt[stride + i]);
                __builtin_nontemporal_store(az[t] + racc[jb][2][lane], &pt[2 * stride + i]);
                // extra slot R + d - 1 (reactions) is written by the split
                // pair (g - d, g), R + D + d - 1 (targets) by the split pair
                // (g, g + d); zeros where the pair is whole
                for (int d = 1; d <= tl.D; ++d) {
                    if (!mt_is_split(tl, g - d, d)) {
                        double* pz = part + (int64_t)(tl.R + d - 1) * plane;
                        __builtin_nontemporal_store(0.0, &pz[i]);
                        __builtin_nontemporal_store(0.0, &pz[stride + i]);
                        __builtin_nontemporal_store(0.0, &pz[2 * stride + i]);
                    }
                    if (!mt_is_split(tl, g, d)) {
                        double* pz = part + (int64_t)(tl.R + tl.D + d - 1) * plane;
                        __builtin_nontemporal_store(0.0, &pz[i]);
                        __builtin_nontemporal_store(0.0, &pz[stride + i]);
                        __builtin_nontemporal_store(0.0, &pz[2 * stride + i]);
                    }
                }
            }
        }
    }
}

template <int KMT, int KMW, int PREC>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual(const double* __restrict__ pos,
                                                           const double* __restrict__ gm,
                                                           int64_t n,
                                                           const int64_t* __restrict__ nmaj,
                                                           MutualTail tl, MutualMap map,
                                                           double* __restrict__ part)
{
    int g, r, half, xslot;
    mt_lookup(map, tl, blockIdx.x, g, r, half, xslot);
    mutual_unit<KMT, KMW, PREC>(pos, gm, n, n, PREC != 0 ? nmaj[0] : 0, g, r, part, tl, half,
                                xslot);
}

// The ensemble: one workgroup per unit (system, g = tblock, r = chunk) of the
// work list; the partial planes span all systems (stride n_total).
template <int KMT, int KMW, int PREC>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual_batched(
    const double* __restrict__ pos, const double* __restrict__ gm, int64_t n_total,
    const BatchUnit* __restrict__ units, const int64_t* __restrict__ nmaj,
    double* __restrict__ part)
{
    const BatchUnit u = units[blockIdx.x];
    const MutualTail whole{u.chunks, 0, 0, 0};
    mutual_unit<KMT, KMW, PREC>(pos + u.body0, gm + u.body0, u.n, n_total,
                                PREC != 0 ? nmaj[u.sys] : 0, u.tblock, u.chunk, part + u.body0,
                                whole, -1, 0);
}

// ---------------------------------------------------------------------------
// The transpose Jacobian of Eq. (1) (the adjoint's inner pass) with each
// unordered pair evaluated once.  For a cotangent u on the accelerations and
// the pair (q, j), d = r_j - r_q, K(d) = I/|d|^3 - 3 d d^T/|d|^5:
//   body q gains  G K(d) w,      w = m_q u_j - m_j u_q,
//   body j gains -G K(d) w       (K is even in d, w odd in the pair),
// and in the mass gradient q gains -G u_j.d/|d|^3, j gains +G u_q.d/|d|^3.
// The pass runs on lam (u = c lam) and scales by G c at the store, as the
// one-way pass does.  Schedule as the force pass above, the last round's
// pairs of shape (4, 4) split into sub-phase halves the same way: the four
// reaction sums (three position components, the mass term) travel along the
// row with their source.  Partial slot c of plane k (0..2: position gradient,
// 3: mass gradient) of body i at part[(4c + k) n + i]; slot r holds workgroup
// (g, r)'s target sums, slot g its reactions, a second half's go to the
// extra slots of its pair, so a body receives each of its R + 2D slots
// exactly once.

struct VBody {
    double x, y, z, m, ux, uy, uz;
};

// Padding bodies are massless, far away, at distinct points and carry no
// cotangent, so every term they take part in is zero or is not stored.
__device__ __forceinline__ VBody load_vbody(const double* __restrict__ pos,
                                            const double* __restrict__ mass,
                                            const double* __restrict__ lam, int64_t n, int64_t i)
{
    VBody b;
    if (i < n) {
        b.x = pos[i];
        b.y = pos[n + i];
        b.z = pos[2 * n + i];
        b.m = mass[i];
        b.ux = lam[i];
        b.uy = lam[n + i];
        b.uz = lam[2 * n + i];
    } else {
        b.x = kPadBase + kPadStep * (double)i;
        b.y = kPadBase;
        b.z = kPadBase;
        b.m = 0.0;
        b.ux = 0.0;
        b.uy = 0.0;
        b.uz = 0.0;
    }
    return b;
}

// The staged source blocks: per block four groups of 16 sources; group grp
// holds the planes x, y, z, m, ux, uy, uz of 32 entries each (its 16 sources
// twice in a row) at kVGrp * grp + 32 * plane, one base address with
// immediate offsets for all seven.
constexpr int kVGrp = 7 * 32;

struct VSrc {
    double s[kMM][4 * kVGrp];
};

struct VAcc {
    double x, y, z, g;
};

// One tile (KMT target blocks of a wave against source block jb), the
// geometry of tile_sweep: targets t < NSYM both ways, t == NSYM one way when
// DIAG (the diagonal block, its own body skipped), t > NSYM not at all;
// sub-phases Q0 .. Q1 - 1.
template <int KMT, int NSYM, bool DIAG, int Q0 = 0, int Q1 = 4>
__device__ __forceinline__ void vjp_tile(const VSrc& S, int jb, double* __restrict__ ra, int lane,
                                         const VBody (&tg)[KMT], VAcc (&o)[KMT])
{
    constexpr bool kReact = NSYM > 0;
    const int row = lane >> 4;
    const int col = lane & 15;
    for (int q = Q0; q < Q1; ++q) {
        const int grp = (row + q) & 3;
        const int home = 16 * grp + col;
        double rx = 0.0, ry = 0.0, rz = 0.0, rg = 0.0;
#pragma unroll 2
        for (int k = 0; k < 16; ++k) {
            const double* sj = &S.s[jb][kVGrp * grp + col + k];
            const double jx = sj[0], jy = sj[32], jz = sj[64], jm = sj[96];
            const double jux = sj[128], juy = sj[160], juz = sj[192];
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                if (t > NSYM || (t == NSYM && !DIAG)) continue;
                if (t == NSYM && q == 0 && k == 0) continue;   // the target itself
                const double dx = jx - tg[t].x;
                const double dy = jy - tg[t].y;
                const double dz = jz - tg[t].z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double y = rinv_f64(r2);
                const double y2 = y * y;
                const double i3 = y * y2;
                const double i5 = i3 * y2;
                const double wx = __builtin_fma(-jm, tg[t].ux, tg[t].m * jux);
                const double wy = __builtin_fma(-jm, tg[t].uy, tg[t].m * juy);
                const double wz = __builtin_fma(-jm, tg[t].uz, tg[t].m * juz);
                const double dw = __builtin_fma(dz, wz, __builtin_fma(dy, wy, dx * wx));
                const double c = 3.0 * dw * i5;
                o[t].x = __builtin_fma(-c, dx, __builtin_fma(wx, i3, o[t].x));
                o[t].y = __builtin_fma(-c, dy, __builtin_fma(wy, i3, o[t].y));
                o[t].z = __builtin_fma(-c, dz, __builtin_fma(wz, i3, o[t].z));
                const double ujd = __builtin_fma(juz, dz, __builtin_fma(juy, dy, jux * dx));
                o[t].g = __builtin_fma(ujd, i3, o[t].g);
                if (t < NSYM) {   // the reaction on the source
                    rx = __builtin_fma(c, dx, __builtin_fma(-wx, i3, rx));
                    ry = __builtin_fma(c, dy, __builtin_fma(-wy, i3, ry));
                    rz = __builtin_fma(c, dz, __builtin_fma(-wz, i3, rz));
                    const double uqd =
                        __builtin_fma(tg[t].uz, dz, __builtin_fma(tg[t].uy, dy, tg[t].ux * dx));
                    rg = __builtin_fma(-uqd, i3, rg);
                }
            }
            if (kReact) {
                rx = row_next(rx);
                ry = row_next(ry);
                rz = row_next(rz);
                rg = row_next(rg);
            }
        }
        if (kReact) {
            ra[home] += rx;
            ra[64 + home] += ry;
            ra[128 + home] += rz;
            ra[192 + home] += rg;
        }
    }
}

template <int KMT>
__device__ __forceinline__ void vjp_tile_dispatch(int d, const VSrc& S, int jb, double* ra,
                                                  int lane, const VBody (&tg)[KMT],
                                                  VAcc (&o)[KMT])
{
    // d = J - I0: targets I0 + t < J for t < d, I0 + d == J
    if (d >= KMT) {
        vjp_tile<KMT, KMT, false>(S, jb, ra, lane, tg, o);
        return;
    }
    switch (d) {
    case 0: vjp_tile<KMT, 0, true>(S, jb, ra, lane, tg, o); break;
    case 1: vjp_tile<KMT, (KMT > 1 ? 1 : 0), true>(S, jb, ra, lane, tg, o); break;
    case 2: vjp_tile<KMT, (KMT > 2 ? 2 : 0), true>(S, jb, ra, lane, tg, o); break;
    case 3: vjp_tile<KMT, (KMT > 3 ? 3 : 0), true>(S, jb, ra, lane, tg, o); break;
    default: break;
    }
}

template <int KMT, int KMW>
__global__ __launch_bounds__(64 * KMW) void k_vjp_mutual(const double* __restrict__ pos,
                                                         const double* __restrict__ mass,
                                                         const double* __restrict__ lam,
                                                         double gc, int64_t n, MutualTail tl,
                                                         double* __restrict__ part)
{
    using Shape = MutualShape<KMT, KMW>;
    // the waves' partial sums reuse the staged sources' space once the sweep
    // is done (36 KB of LDS in all, four workgroups per CU; shape (4, 4)
    // stages its targets as well: 50 KB, three per CU)
    using Comb = double[Shape::kShare > 1 ? Shape::kShare - 1 : 1][Shape::kSets][KMT][4][64];
    static_assert(sizeof(Comb) <= sizeof(VSrc), "the sums fit in the sources' space");
    __shared__ double smem[sizeof(VSrc) / sizeof(double)];
    __shared__ double racc[kMM][4][64];
    VSrc& S = *reinterpret_cast<VSrc*>(smem);
    Comb& comb = *reinterpret_cast<Comb*>(smem);

    // shape (4, 4): the pairs past the last whole round run as halves by
    // sub-phases, as in the force pass (the second half's target sums and
    // reactions in the extra slots R + D + d - 1 and R + d - 1)
    int g, r, half, xslot;
    mt_decode(tl, blockIdx.x, g, r, half, xslot);

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int set = w % Shape::kSets;
    const int h = w / Shape::kSets;
    const int nb = (int)((n + 63) / 64);
    const int I0 = g * kMM + set * KMT;
    const int J0 = r * kMM;
    const int64_t plane = 4 * n;

    // shape (4, 4): the four waves hold the same four target blocks, so the
    // range's targets are staged in LDS too (each body loaded once per
    // workgroup, not once per wave); the other shapes load their own
    constexpr bool kShareTargets = KMT == 4 && KMW == 4;
    __shared__ double tst[kShareTargets ? kMM : 1][7][64];
    VBody tg[KMT];
    VAcc o[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        if (!kShareTargets) tg[t] = load_vbody(pos, mass, lam, n, (int64_t)(I0 + t) * 64 + lane);
        o[t] = VAcc{0.0, 0.0, 0.0, 0.0};
    }
    for (int jb = w; jb < kMM; jb += KMW) {
        if (kShareTargets) {
            const VBody a = load_vbody(pos, mass, lam, n, (int64_t)(g * kMM + jb) * 64 + lane);
            const double v[7] = {a.x, a.y, a.z, a.m, a.ux, a.uy, a.uz};
#pragma unroll
            for (int pl = 0; pl < 7; ++pl) tst[jb][pl][lane] = v[pl];
        }
        const VBody b = load_vbody(pos, mass, lam, n, (int64_t)(J0 + jb) * 64 + lane);
        double* sb = &S.s[jb][kVGrp * (lane >> 4) + (lane & 15)];
        const double v[7] = {b.x, b.y, b.z, b.m, b.ux, b.uy, b.uz};
#pragma unroll
        for (int pl = 0; pl < 7; ++pl) {
            sb[32 * pl] = v[pl];
            sb[32 * pl + 16] = v[pl];
        }
        for (int k = 0; k < 4; ++k) racc[jb][k][lane] = 0.0;
    }
    __syncthreads();
    if (kShareTargets) {
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int tb = set * KMT + t;
            tg[t] = VBody{tst[tb][0][lane], tst[tb][1][lane], tst[tb][2][lane], tst[tb][3][lane],
                          tst[tb][4][lane], tst[tb][5][lane], tst[tb][6][lane]};
        }
    }
    for (int p = 0; p < Shape::kPhases; ++p) {
        const int jb = (w + p) % kMM;
        const int J = J0 + jb;
        if (J < nb && J >= I0) {
            if constexpr (KMT == 4 && KMW == 4) {   // a half: r > g, so J - I0 >= 4
                if (half == 0)
                    vjp_tile<4, 4, false, 0, 2>(S, jb, &racc[jb][0][0], lane, tg, o);
                else if (half == 1)
                    vjp_tile<4, 4, false, 2, 4>(S, jb, &racc[jb][0][0], lane, tg, o);
                else
                    vjp_tile_dispatch<KMT>(J - I0, S, jb, &racc[jb][0][0], lane, tg, o);
            } else {
                vjp_tile_dispatch<KMT>(J - I0, S, jb, &racc[jb][0][0], lane, tg, o);
            }
        }
        __syncthreads();
    }

    if (Shape::kShare > 1) {   // the sums of the waves sharing a target set, in wave order
        if (h > 0) {
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                comb[h - 1][set][t][0][lane] = o[t].x;
                comb[h - 1][set][t][1][lane] = o[t].y;
                comb[h - 1][set][t][2][lane] = o[t].z;
                comb[h - 1][set][t][3][lane] = o[t].g;
            }
        }
        __syncthreads();
        if (h == 0) {
            for (int k = 0; k < Shape::kShare - 1; ++k) {
#pragma unroll
                for (int t = 0; t < KMT; ++t) {
                    o[t].x += comb[k][set][t][0][lane];
                    o[t].y += comb[k][set][t][1][lane];
                    o[t].z += comb[k][set][t][2][lane];
                    o[t].g += comb[k][set][t][3][lane];
                }
            }
        }
    }

    if (r > g) {   // targets' sums to slot r, the sources' reactions to slot g
        const int tslot = half == 1 ? xslot + tl.D : r;
        const int rslot = half == 1 ? xslot : g;
        if (h == 0) {
#pragma unroll
            for (int t = 0; t < KMT; ++t) {
                const int64_t i = (int64_t)(I0 + t) * 64 + lane;
                if (i < n) {
                    double* pt = part + (int64_t)tslot * plane;
                    __builtin_nontemporal_store(gc * o[t].x, &pt[i]);
                    __builtin_nontemporal_store(gc * o[t].y, &pt[n + i]);
                    __builtin_nontemporal_store(gc * o[t].z, &pt[2 * n + i]);
                    __builtin_nontemporal_store(-gc * o[t].g, &pt[3 * n + i]);
                }
            }
        }
        for (int jb = w; jb < kMM; jb += KMW) {
            const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
            if (j < n) {
                double* ps = part + (int64_t)rslot * plane;
                __builtin_nontemporal_store(gc * racc[jb][0][lane], &ps[j]);
                __builtin_nontemporal_store(gc * racc[jb][1][lane], &ps[n + j]);
                __builtin_nontemporal_store(gc * racc[jb][2][lane], &ps[2 * n + j]);
                __builtin_nontemporal_store(-gc * racc[jb][3][lane], &ps[3 * n + j]);
            }
        }
    } else if (h == 0) {   // the diagonal: each body's sum and the reaction on it
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int64_t i = (int64_t)(I0 + t) * 64 + lane;
            const int jb = set * KMT + t;
            if (i < n) {
                double* pt = part + (int64_t)g * plane;
                __builtin_nontemporal_store(gc * (o[t].x + racc[jb][0][lane]), &pt[i]);
                __builtin_nontemporal_store(gc * (o[t].y + racc[jb][1][lane]), &pt[n + i]);
                __builtin_nontemporal_store(gc * (o[t].z + racc[jb][2][lane]), &pt[2 * n + i]);
                __builtin_nontemporal_store(-gc * (o[t].g + racc[jb][3][lane]), &pt[3 * n + i]);
                // zeros in the extra slots of the pairs (g - d, g), (g, g + d)
                // that are not split
                for (int d = 1; d <= tl.D; ++d) {
                    for (int e = 0; e < 2; ++e) {
                        if (mt_is_split(tl, e == 0 ? g - d : g, d)) continue;
                        double* pz = part + (int64_t)(tl.R + (e == 0 ? 0 : tl.D) + d - 1) * plane;
                        __builtin_nontemporal_store(0.0, &pz[i]);
                        __builtin_nontemporal_store(0.0, &pz[n + i]);
                        __builtin_nontemporal_store(0.0, &pz[2 * n + i]);
                        __builtin_nontemporal_store(0.0, &pz[3 * n + i]);
                    }
                }
            }
        }
    }
}

}  // namespace

int mutual_ranges(int64_t n) { return (int)((((n + 63) / 64) + kMM - 1) / kMM); }

// CUs of the device the split of the last round is laid out for (results
// do not depend on the device).
static constexpr int64_t kMutualCUs = 256;

static MutualTail mutual_tail(int64_t n, int tpl, int waves)
{
    MutualTail t;
    t.R = mutual_ranges(n);
    const int64_t U = (int64_t)t.R * (t.R + 1) / 2;
    const int64_t rem = U % kMutualCUs;
    t.F = (int)U;
    t.D = 0;
    t.kD = 0;
    // split only the pairs past the last whole round, when their halves fit
    // in one round and they are off the diagonal
    if (tpl != 4 || waves != 4 || U > 64 * kMutualCUs || rem == 0 || 2 * rem > kMutualCUs ||
        rem > U - t.R)
        return t;
    int64_t left = rem;
    int d = 1;
    while (left > t.R - d) {
        left -= t.R - d;
        ++d;
    }
    t.D = d;
    t.kD = (int)left;
    t.F = (int)(U - rem);
    return t;
}

int mutual_slots(int64_t n, int tpl, int waves)
{
    const MutualTail t = mutual_tail(n, tpl, waves);
    return t.R + 2 * t.D;
}

bool mutual_shape_supported(int tpl, int waves)
{
    return (tpl == 1 && waves == 4) || (tpl == 2 && waves == 2) || (tpl == 2 && waves == 4) ||
           (tpl == 4 && waves == 4);
}

// The kernel-argument list of a pass's decode (count 0 where it does not
// fit), kept per host thread for the last shape of the split.
static const MutualMap& mutual_map(const MutualTail& tl, int64_t grid)
{
    thread_local MutualTail last{-1, -1, -1, -1};
    thread_local MutualMap m{};
    if (last.R == tl.R && last.F == tl.F && last.D == tl.D && last.kD == tl.kD) return m;
    m.count = 0;
    if (tl.R <= 64 && grid <= kMapMax) {
        for (int64_t b = 0; b < grid; ++b) {
            int g, r, half, xslot;
            mt_decode(tl, b, g, r, half, xslot);
            m.e[b] = (uint16_t)(g | (r << 6) | ((half + 1) << 12));
        }
        m.count = (int32_t)grid;
    }
    last = tl;
    return m;
}

template <int PREC>
static void launch_mutual_shape(int tpl, int waves, dim3 grid, const double* pos, const double* gm,
                                int64_t n, const int64_t* nmaj, const MutualTail& tl,
                                double* part, hipStream_t s)
{
    const dim3 block((unsigned)(64 * waves));
    const MutualMap& map = mutual_map(tl, (int64_t)grid.x);
    if (tpl == 1)
        hipLaunchKernelGGL((k_force_mutual<1, 4, PREC>), grid, block, 0, s, pos, gm, n, nmaj,
                           tl, map, part);
    else if (tpl == 2 && waves == 2)
        hipLaunchKernelGGL((k_force_mutual<2, 2, PREC>), grid, block, 0, s, pos, gm, n, nmaj,
                           tl, map, part);
    else if (tpl == 2)
        hipLaunchKernelGGL((k_force_mutual<2, 4, PREC>), grid, block, 0, s, pos, gm, n, nmaj,
                           tl, map, part);
    else
        hipLaunchKernelGGL((k_force_mutual<4, 4, PREC>), grid, block, 0, s, pos, gm, n, nmaj,
                           tl, map, part);
}

template <int PREC>
static void launch_mutual_batched_shape(int tpl, int waves, dim3 grid, const double* pos,
                                        const double* gm, int64_t n_total, const BatchUnit* units,
                                        const int64_t* nmaj, double* part, hipStream_t s)
{
    const dim3 block((unsigned)(64 * waves));
    if (tpl == 1)
        hipLaunchKernelGGL((k_force_mutual_batched<1, 4, PREC>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else if (tpl == 2 && waves == 2)
        hipLaunchKernelGGL((k_force_mutual_batched<2, 2, PREC>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else if (tpl == 2)
        hipLaunchKernelGGL((k_force_mutual_batched<2, 4, PREC>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
    else
        hipLaunchKernelGGL((k_force_mutual_batched<4, 4, PREC>), grid, block, 0, s, pos, gm,
                           n_total, units, nmaj, part);
}

hipError_t launch_force_mutual_batched(int precision, int tpl, int waves, const double* pos,
                                       const double* gm, int64_t n_total, const BatchUnit* units,
                                       int64_t num_units, const int64_t* nmaj, double* part,
                                       hipStream_t s)
{
    if (!gm || !units || num_units < 1 || !mutual_shape_supported(tpl, waves) ||
        precision < 0 || precision > 2 || (precision != 0 && !nmaj))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)num_units);
    if (precision == 0)
        launch_mutual_batched_shape<0>(tpl, waves, grid, pos, gm, n_total, units, nullptr, part,
                                       s);
    else if (precision == 1)
        launch_mutual_batched_shape<1>(tpl, waves, grid, pos, gm, n_total, units, nmaj, part, s);
    else
        launch_mutual_batched_shape<2>(tpl, waves, grid, pos, gm, n_total, units, nmaj, part, s);
    return hipGetLastError();
}

hipError_t launch_force_mutual(int precision, int tpl, int waves, const double* pos,
                               const double* gm, int64_t n, const int64_t* nmaj, double* part,
                               hipStream_t s)
{
    if (!gm || n < 1 || !mutual_shape_supported(tpl, waves) || precision < 0 || precision > 2 ||
        (precision != 0 && !nmaj))
        return hipErrorInvalidValue;
    const MutualTail tl = mutual_tail(n, tpl, waves);
    const int64_t pairs = (int64_t)tl.R * (tl.R + 1) / 2;
    const dim3 grid((unsigned)(tl.F + 2 * (pairs - tl.F)));   // whole pairs, then halves
    if (precision == 0)
        launch_mutual_shape<0>(tpl, waves, grid, pos, gm, n, nullptr, tl, part, s);
    else if (precision == 1)
        launch_mutual_shape<1>(tpl, waves, grid, pos, gm, n, nmaj, tl, part, s);
    else
        launch_mutual_shape<2>(tpl, waves, grid, pos, gm, n, nmaj, tl, part, s);
    return hipGetLastError();
}

hipError_t launch_vjp_mutual(int tpl, int waves, const double* pos, const double* mass,
                             const double* lam, double cu, int64_t n, double G, double* part,
                             hipStream_t s)
{
    if (n < 1 || n > kMutualMaxN || !mutual_shape_supported(tpl, waves))
        return hipErrorInvalidValue;
    const MutualTail tl = mutual_tail(n, tpl, waves);
    const int64_t U = (int64_t)tl.R * (tl.R + 1) / 2;
    const dim3 grid((unsigned)(tl.F + 2 * (U - tl.F)));
    const dim3 block((unsigned)(64 * waves));
    const double gc = G * cu;
    if (tpl == 1)
        hipLaunchKernelGGL((k_vjp_mutual<1, 4>), grid, block, 0, s, pos, mass, lam, gc, n, tl, part);
    else if (tpl == 2 && waves == 2)
        hipLaunchKernelGGL((k_vjp_mutual<2, 2>), grid, block, 0, s, pos, mass, lam, gc, n, tl, part);
    else if (tpl == 2)
        hipLaunchKernelGGL((k_vjp_mutual<2, 4>), grid, block, 0, s, pos, mass, lam, gc, n, tl, part);
    else
        hipLaunchKernelGGL((k_vjp_mutual<4, 4>), grid, block, 0, s, pos, mass, lam, gc, n, tl, part);
    return hipGetLastError();
}

}  // namespace nb
