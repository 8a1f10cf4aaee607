// Shared declarations of the HIP library: the tile shape, the per-launch
// argument blocks and the host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

// Shape of one force launch.  A workgroup of 64*waves lanes owns
// 64*waves*tpl consecutive targets; lane l of the group handles targets
// base + t*64*waves + l for t < tpl, so every target plane is loaded and
// stored with unit stride.  The source range is split into `chunks`
// contiguous pieces (grid.y), each summed separately; the step epilogue adds
// the pieces in a fixed order, so results do not depend on scheduling.
struct Tile {
    int tpl;          // targets per lane: 1, 2, 4
    int waves;        // wavefronts per workgroup: 1, 2, 4, 8
    int chunks;       // source chunks, 1..64
    int variant = 0;  // 0: sources staged in LDS; 1: sources as scalar operands;
                      // 2: as 1, with the waves of a group splitting the sources;
                      // 3: one workgroup runs whole steps (n <= kSmallMax, tpl = 1,
                      //    waves = 16, chunks = source slices per target);
                      // 4: as 2 over all sources (chunks = 1) with the step's kicks
                      //    and drift in the same kernel (tpl 1, 2; waves 2, 4, 8);
                      // 5: each unordered pair once ((tpl, waves) = (1, 4),
                      //    (2, 2), (2, 4), (4, 4); chunks = 1: the pass writes
                      //    mutual_slots(n, tpl, waves) partials)
};

constexpr int kMaxChunks = 64;
// Largest system the single-workgroup variant holds in LDS.
constexpr int kSmallMax = 512;

// Source tile width (bodies staged in LDS per pass) = lanes of a workgroup.
inline int tile_width(const Tile& t) { return 64 * t.waves; }

// Targets owned by one workgroup: variants 0 and 1 spread 64*waves lanes
// over distinct targets; in variant 2 the waves share 64*tpl targets and
// split the sources among themselves.
inline int64_t targets_per_block(const Tile& t)
{
    return (int64_t)64 * t.tpl * (t.variant == 2 ? 1 : t.waves);
}

bool tile_supported(const Tile& t);

// Length of each source chunk: a multiple of the tile width so that only the
// very last tile of the last chunk holds padding.
int64_t chunk_length(int64_t n, const Tile& t);
// Chunks actually used for n bodies (<= t.chunks).
int effective_chunks(int64_t n, const Tile& t);

// ----- force pass (Eq. (1)) ------------------------------------------------
// part[c*3n + k*n + p] receives the chunk-c partial of component k of a_p.
// Split form: sources [0, n_major) are accumulated in FP64 with a single
// Newton-refined reciprocal square root, sources [n_major, n) in FP32 with
// Kahan compensation.
// nmaj: device pointer to the number of FP64-class sources (split form only).
// gm: G * mass plane (required by variant 1; the LDS variant scales on load).
hipError_t launch_force(int precision, const Tile& tile, const double* pos, const double* mass,
                        const double* gm, int64_t n, const int64_t* nmaj, double G, double* part,
                        hipStream_t s);

// Batched form: `units` work items of (system, target block, chunk), see
// kernels_force.hip.
struct BatchUnit {
    int64_t body0;     // first body of the system
    int32_t n;         // bodies in the system
    int32_t sys;       // system index (split form: nmaj[sys] FP64-class sources first)
    int32_t tblock;    // target block within the system
    int32_t chunk;     // chunk index
    int32_t chunks;    // chunks of this system
    int32_t pad;
};
hipError_t launch_force_batched(int precision, const Tile& tile, const double* pos,
                                const double* mass, const double* gm, int64_t n_total, double G,
                                const BatchUnit* units, int64_t num_units, const int64_t* nmaj,
                                int grid, double* part, hipStream_t s);

// ----- each pair once (variant 5, FP64 or split) -------------------------------
// Ranges of 4 blocks of 64 bodies; the pass writes one partial per range and
// body (slot order = range order), plus the extra slots of a split last round,
// summed by the ordinary step epilogue.
int mutual_ranges(int64_t n);
// Partial slots of a single system's pass: the ranges, plus the extra slots
// of the split last round (shape (4, 4) only).
int mutual_slots(int64_t n, int tpl, int waves);
// Largest single system the each-pair-once passes take (one partial slot per
// range of 256 bodies: 512 at the largest).
constexpr int64_t kMutualMaxN = 131072;
// The adjoint's transpose-Jacobian pass with each unordered pair once: four
// partial planes per slot (position gradient, mass gradient), one slot per
// range (mutual_ranges(n)), in the layout launch_vjp_reduce sums.
hipError_t launch_vjp_mutual(int tpl, int waves, const double* pos, const double* mass,
                             const double* lam, double cu, int64_t n, double G, double* part,
                             hipStream_t s);
bool mutual_shape_supported(int tpl, int waves);
hipError_t launch_force_mutual(int precision, int tpl, int waves, const double* pos,
                               const double* gm, int64_t n, const int64_t* nmaj, double* part,
                               hipStream_t s);
// The ensemble's each-pair-once pass: one workgroup per unit (system,
// g = tblock, r = chunk, ranges = chunks); partials of stride n_total.
hipError_t launch_force_mutual_batched(int precision, int tpl, int waves, const double* pos,
                                       const double* gm, int64_t n_total, const BatchUnit* units,
                                       int64_t num_units, const int64_t* nmaj, double* part,
                                       hipStream_t s);

// ----- small systems: one workgroup, whole steps (variant 3) ----------------
// Source slices per target actually used for n bodies (0 if n > kSmallMax).
int small_slices(int64_t n, const Tile& t);
// Launch indices i0..i1 of a run of `steps` steps (i = 0..steps; launch i is
// the force pass at r_i, the closing half kick for i > 0 and, for i < steps,
// the opening half kick and the drift), state read from pos_in / vel and
// written back to pos_out / vel at the end (pos_in == pos_out allowed).
// acc != NULL (only with steps = 0): store a(r) in acc.  traj != NULL: the
// position after each drift of launch i goes to traj + (i - i0) * 3n.
// Split form (precision 1): sources [0, *nmaj) are the FP64 class.
hipError_t launch_run_small(int precision, const Tile& tile, const double* pos_in,
                            double* pos_out, double* vel, const double* mass, int64_t n,
                            const int64_t* nmaj, double G, double dt, int64_t i0, int64_t i1,
                            int64_t steps, double* acc, double* traj, uint32_t* flags,
                            hipStream_t s);

// ----- step epilogue (Eqs. (3)-(4) as kick-drift-kick) -----------------------
enum StepMode : int {
    kStoreAcc = 1,   // write a to acc
    kClose = 2,      // v += dt/2 a  (closing half kick of the step that ends here)
    kOpen = 4,       // v += dt/2 a; r_out = r_in + dt v  (next step's kick + drift)
};

// One launch of the step loop with a variant-4 tile: Eq. (1) at pos_in and
// the mode's updates, in one kernel (pos_out != pos_in).
hipError_t launch_step_fused(int precision, const Tile& tile, const double* pos_in,
                             double* pos_out, double* vel, const double* gm, int64_t n,
                             const int64_t* nmaj, double dt, int mode, double* acc,
                             uint32_t* flags, hipStream_t s);
// a_p = sum_{c < chunks_of(p)} part[c][.][p] in ascending c, then the mode's
// updates.  chunks_of(p) = chunks, or body_chunks[p] when that is not NULL.
hipError_t launch_step(const double* part, int chunks, const int8_t* body_chunks, int64_t n,
                       double* vel, const double* pos_in, double* pos_out, double* acc,
                       double dt, int mode, uint32_t* flags, hipStream_t s);
// out[k * nt + q] = sum_{c < chunks} part[c][k][t0 + q] in ascending c, for
// the targets t0 .. t0 + nt - 1 of an n-body system (a share of the targets).
hipError_t launch_shard_sum(const double* part, int chunks, int64_t n, int64_t t0, int64_t nt,
                            double* out, hipStream_t s);

// ----- fourth-order Runge-Kutta (the alternative integrator of Sec. 2) ---------
// Stage s = 1..4 after the force pass at the stage position (pos for s = 1,
// rs otherwise): sums the chunk partials, accumulates the slopes in sr, sv
// and writes the next stage's position / velocity into rs, vs, or, for
// s = 4, the step's result into pos, vel.
hipError_t launch_rk4_stage(const double* part, int chunks, int64_t n, int stage, double dt,
                            double* pos, double* vel, double* rs, double* vs, double* sr,
                            double* sv, uint32_t* flags, hipStream_t s);

// ----- split form: class order -------------------------------------------------
// Stable partition of each system's bodies into mass >= threshold first:
// perm[body0 + i] = original index of the i-th body in class order, and
// nmaj[k] = number of FP64-class bodies of system k.  offsets: device array of
// num_systems + 1 body offsets, or NULL for one system of n_single bodies.
hipError_t launch_partition(const double* mass, const int64_t* offsets, int num_systems,
                            int64_t n_single, double threshold, int32_t* perm, int64_t* nmaj,
                            hipStream_t s);
hipError_t launch_gather(const int32_t* perm, int64_t n, const double* src3, double* dst3,
                         int planes, hipStream_t s);
hipError_t launch_scatter(const int32_t* perm, int64_t n, const double* src3, double* dst3,
                          int planes, hipStream_t s);

// ----- diagnostics -------------------------------------------------------------
// rows[p] = -G m_p / 2 sum_{j != p} m_j / |r_j - r_p| (compensated): source
// chunks (at most max_chunks; part holds 2 n doubles per chunk) merged in
// chunk order.
hipError_t launch_potential_rows(const double* pos, const double* mass, int64_t n, double G,
                                 double* part, int max_chunks, double* rows, hipStream_t s);
hipError_t launch_energy_finish(const double* rows, const double* vel, const double* mass,
                                int64_t n, double* out, hipStream_t s);
hipError_t launch_momenta(const double* pos, const double* vel, const double* mass, int64_t n,
                          double* out, hipStream_t s);

// ----- adjoint (transpose of the Jacobian of Eq. (1)) ------------------------------
// Source chunks of the transpose-Jacobian pass: multiples of 8 sources
// (the last LDS tile of a chunk may be partly used), at most t.chunks.
int64_t vjp_chunk_length(int64_t n, const Tile& t);
int vjp_chunks(int64_t n, const Tile& t);
// Chunk partials of (J^T u, M^T u) for the cotangent u = cu * lam on the
// accelerations (variant-0 tiles, tpl <= 2, waves <= 4), vjp_chunks of them.
hipError_t launch_vjp(const Tile& tile, const double* pos, const double* mass, const double* lam,
                      double cu, int64_t n, double G, double* part, hipStream_t s);
// lam_r += sum of chunk partials (planes 0..2), g_m += plane 3; then, if
// drift, lam_v += dt * lam_r (the adjoint of the drift before this pass).
hipError_t launch_vjp_reduce(const double* part, int chunks, int64_t n, double* lam_r,
                             double* g_m, double* lam_v, double dt, bool drift, hipStream_t s);
// u = c * lam_v
hipError_t launch_scale(const double* x, double c, int64_t m, double* y, hipStream_t s);
// y += c * x
hipError_t launch_axpy(const double* x, double c, int64_t m, double* y, hipStream_t s);
hipError_t launch_fill(double* y, double v, int64_t m, hipStream_t s);

}  // namespace nb
