// Force pass of Eq. (1) with each unordered pair evaluated once (Newton's
// third law; tile variant 5, FP64): the pair's factor f = |d|^-3 serves both
// a_i += G m_j f d and a_j -= G m_i f d, about 21 vector instructions for two
// ordered pairs instead of 2 x 17.
//
// Bodies are cut into blocks of 64 and the blocks into "ranges" of kMM = 4.
// Workgroup (g, r), r >= g, takes range g as its targets and range r as its
// sources: KMW waves, wave w holding target blocks KMT*w .. KMT*w + KMT-1 of
// range g (one body of each per lane), KMT * KMW = 4.  The four source blocks
// are staged in LDS; in phase t wave w works on source block (w + t) mod 4, so
// in every phase the waves touch different source blocks, and after four
// phases every (target block, source block) tile has been visited once.
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
// Output: one partial per (body, range) in the chunk layout of the other force
// passes, so the ordinary step epilogue adds them in slot order.  Workgroup
// (g, r), r > g, writes its targets' accelerations to slot r and the reactions
// on its sources to slot g; workgroup (g, g) adds the two for each of its
// bodies and writes slot g.  A body of range R thus receives slot s < R as a
// source, slot s > R as a target and slot R from the diagonal workgroup:
// every slot exactly once.
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

enum TileType { kNone = 0, kDiag = 1, kSym = 2 };

struct Body {
    double x, y, z, gm;
};

__device__ __forceinline__ Body load_body(const double* __restrict__ pos,
                                          const double* __restrict__ gm, int64_t n, int64_t i)
{
    Body b;
    if (i < n) {
        b.x = pos[i];
        b.y = pos[n + i];
        b.z = pos[2 * n + i];
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

// One tile: the KMT targets of this lane against the source block staged in
// LDS as four groups of 16 sources, each stored twice in a row
// (s*[32*grp + i], i < 32).  Lane (row R, column c) pairs with source
// 16*grp + (c + k) mod 16 at step k of sub-phase q, grp = (R + q) mod 4; the
// reaction on that source rotates within the row (DPP, no LDS round trip) and
// after 16 steps is added to the block's reaction sums in LDS (`ra`, three
// planes of 64).  Rows work on different groups, so these adds never collide.
template <int KMT, int TY0, int TY1>
__device__ __forceinline__ void tile_sweep(const double* __restrict__ sx,
                                           const double* __restrict__ sy,
                                           const double* __restrict__ sz,
                                           const double* __restrict__ sg,
                                           double* __restrict__ ra, int lane,
                                           const Body (&tg)[KMT], double (&ax)[KMT],
                                           double (&ay)[KMT], double (&az)[KMT],
                                           const PolyConst& c)
{
    constexpr bool kReact = (TY0 == kSym) || (KMT > 1 && TY1 == kSym);
    constexpr int TY[2] = {TY0, TY1};
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
                if (TY[t] == kNone) continue;
                if (TY[t] == kDiag && q == 0 && k == 0) continue;   // the target itself
                const double dx = jx - tg[t].x;
                const double dy = jy - tg[t].y;
                const double dz = jz - tg[t].z;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const double f = gm_rinv3_f64(r2, 1.0, c);   // |d|^-3
                const double fi = jg * f;
                ax[t] = __builtin_fma(fi, dx, ax[t]);
                ay[t] = __builtin_fma(fi, dy, ay[t]);
                az[t] = __builtin_fma(fi, dz, az[t]);
                if (TY[t] == kSym) {   // reaction on the source
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

template <int KMT, int KMW>
__global__ __launch_bounds__(64 * KMW) void k_force_mutual(const double* __restrict__ pos,
                                                           const double* __restrict__ gm,
                                                           int64_t n, int ranges,
                                                           double* __restrict__ part)
{
    static_assert(KMT * KMW == kMM, "a wave's target blocks tile the range");
    __shared__ double sx[kMM][128], sy[kMM][128], sz[kMM][128], sg[kMM][128];
    __shared__ double racc[kMM][3][64];

    // blockIdx.x enumerates the pairs (g, r), r >= g, row by row
    int g = 0, r = (int)blockIdx.x;
    while (g < ranges - 1 && r >= ranges - g) {
        r -= ranges - g;
        ++g;
    }
    r += g;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nb = (int)((n + 63) / 64);
    const int I0 = g * kMM + w * KMT;   // this wave's target blocks I0 .. I0 + KMT - 1
    const int J0 = r * kMM;             // the workgroup's source blocks J0 .. J0 + 3
    const int64_t plane = 3 * n;

    // stage the source blocks (wave w: blocks w, w + KMW, ...): four groups
    // of 16, each twice in a row
    for (int jb = w; jb < kMM; jb += KMW) {
        const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
        const Body b = load_body(pos, gm, n, j);
        const int a0 = 32 * (lane >> 4) + (lane & 15);
        sx[jb][a0] = b.x; sx[jb][a0 + 16] = b.x;
        sy[jb][a0] = b.y; sy[jb][a0 + 16] = b.y;
        sz[jb][a0] = b.z; sz[jb][a0 + 16] = b.z;
        sg[jb][a0] = b.gm; sg[jb][a0 + 16] = b.gm;
        racc[jb][0][lane] = 0.0;
        racc[jb][1][lane] = 0.0;
        racc[jb][2][lane] = 0.0;
    }
    Body tg[KMT];
    double ax[KMT], ay[KMT], az[KMT];
#pragma unroll
    for (int t = 0; t < KMT; ++t) {
        tg[t] = load_body(pos, gm, n, (int64_t)(I0 + t) * 64 + lane);
        ax[t] = 0.0; ay[t] = 0.0; az[t] = 0.0;
    }
    const PolyConst c = {vreg_const(1.875), vreg_const(1.5)};
    __syncthreads();

    for (int phase = 0; phase < kMM; ++phase) {
        const int jb = (w + phase) % kMM;
        const int J = J0 + jb;
        int ty[2] = {kNone, kNone};
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int I = I0 + t;
            ty[t] = (I >= nb || J >= nb || I > J) ? kNone : (I == J ? kDiag : kSym);
        }
        const double* px = sx[jb];
        const double* py = sy[jb];
        const double* pz = sz[jb];
        const double* pg = sg[jb];
        double* ra = &racc[jb][0][0];
        if (KMT == 1) {
            if (ty[0] == kSym)
                tile_sweep<KMT, kSym, kNone>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
            else if (ty[0] == kDiag)
                tile_sweep<KMT, kDiag, kNone>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
        } else {
            if (ty[0] == kSym && ty[1] == kSym)
                tile_sweep<KMT, kSym, kSym>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
            else if (ty[0] == kSym && ty[1] == kDiag)
                tile_sweep<KMT, kSym, kDiag>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
            else if (ty[0] == kDiag)   // (the second target block then lies above J)
                tile_sweep<KMT, kDiag, kNone>(px, py, pz, pg, ra, lane, tg, ax, ay, az, c);
            // (kSym, kNone) and (kNone, kDiag) cannot occur: the wave's blocks
            // are consecutive, and a block past the last body implies J <= I0.
        }
        __syncthreads();
    }

    if (r > g) {
        // targets' partials to slot r, the sources' reactions to slot g
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int64_t i = (int64_t)(I0 + t) * 64 + lane;
            if (i < n) {
                double* pt = part + (int64_t)r * plane;
                pt[i] = ax[t];
                pt[n + i] = ay[t];
                pt[2 * n + i] = az[t];
            }
        }
        for (int jb = w; jb < kMM; jb += KMW) {
            const int64_t j = (int64_t)(J0 + jb) * 64 + lane;
            if (j < n) {
                double* ps = part + (int64_t)g * plane;
                ps[j] = racc[jb][0][lane];
                ps[n + j] = racc[jb][1][lane];
                ps[2 * n + j] = racc[jb][2][lane];
            }
        }
    } else {
        // the diagonal workgroup: targets and sources are the same blocks;
        // each body's partial and the reaction on it, added in that order
#pragma unroll
        for (int t = 0; t < KMT; ++t) {
            const int64_t i = (int64_t)(I0 + t) * 64 + lane;
            const int jb = w * KMT + t;
            if (i < n) {
                double* pt = part + (int64_t)g * plane;
                pt[i] = ax[t] + racc[jb][0][lane];
                pt[n + i] = ay[t] + racc[jb][1][lane];
                pt[2 * n + i] = az[t] + racc[jb][2][lane];
            }
        }
    }
}

}  // namespace

int mutual_ranges(int64_t n) { return (int)((((n + 63) / 64) + kMM - 1) / kMM); }

bool mutual_shape_supported(int tpl, int waves) { return (tpl == 1 && waves == 4) || (tpl == 2 && waves == 2); }

hipError_t launch_force_mutual(int tpl, int waves, const double* pos, const double* gm, int64_t n,
                               double* part, hipStream_t s)
{
    if (!gm || n < 1 || !mutual_shape_supported(tpl, waves)) return hipErrorInvalidValue;
    const int64_t ranges = mutual_ranges(n);
    const dim3 grid((unsigned)(ranges * (ranges + 1) / 2));
    if (tpl == 1)
        hipLaunchKernelGGL((k_force_mutual<1, 4>), grid, dim3(256), 0, s, pos, gm, n, (int)ranges, part);
    else
        hipLaunchKernelGGL((k_force_mutual<2, 2>), grid, dim3(128), 0, s, pos, gm, n, (int)ranges, part);
    return hipGetLastError();
}

}  // namespace nb
