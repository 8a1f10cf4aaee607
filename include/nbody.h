/*
 * nbody.h - C ABI of the MI355X (gfx950) direct-sum N-body library.
 *
 * The method (Zhu, "N-body Simulations of the Solar System with CPU-based
 * Parallel Methods"):
 *   Eq. (1)       a_p = sum_{j != p} G m_j (r_j - r_p) / |r_j - r_p|^3
 *   Eqs. (3)-(4)  velocity Verlet: r_{i+1} = r_i + v_i dt + a_i dt^2 / 2,
 *                 v_{i+1} = v_i + (a_i + a_{i+1}) dt / 2.
 *
 * Conventions shared by every entry point
 *   - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     unless the name ends in _host.  All floating point is IEEE double.
 *   - Layout is structure of arrays with plane stride n:
 *       pos[0..n) = x, pos[n..2n) = y, pos[2n..3n) = z   (same for vel, acc,
 *       gradients); mass[0..n).
 *   - Units are the caller's; G must be in those units.  No softening: the
 *     self pair j = p is excluded by index, and two distinct bodies at the
 *     same point give non-finite values, as Eq. (1) does.  In the split
 *     form, squared separations must lie inside the FP32 normal range
 *     (1e-37 .. 1e37 in the caller's units): its reciprocal square root is
 *     seeded in FP32 and refined in FP64.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; results are ready when the stream is.
 *   - Ownership: the caller owns every buffer.  Scratch memory is the
 *     caller's `workspace` of at least nbody_workspace_bytes(...) bytes
 *     (256-byte aligned); the library allocates no device memory.  It keeps
 *     only its tile-shape table, up to 64 captured step graphs and up to 8
 *     ensemble work lists (least recently used dropped first, after waiting
 *     for the device), all released by nbody_reset_caches().  A captured
 *     graph bakes in the addresses of the buffers it ran on; a later call
 *     with the same buffers replays it.
 *   - Errors: arguments are validated before anything is enqueued; a bad
 *     argument returns NBODY_EINVAL (nothing enqueued), a short workspace
 *     NBODY_EWORKSPACE, a HIP failure NBODY_EHIP.  nbody_last_error() gives
 *     a message for the calling thread.  Device faults surface at the
 *     caller's next synchronisation.  No C++ exception crosses this ABI.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NBODY_OK = 0,
    NBODY_EINVAL = 1,        /* bad argument; nothing enqueued */
    NBODY_EUNSUPPORTED = 2,  /* valid but not supported (e.g. n too large) */
    NBODY_EWORKSPACE = 3,    /* workspace NULL or smaller than required */
    NBODY_EHIP = 4           /* a HIP runtime call failed */
} nbody_status;

typedef enum {
    /* FP64 throughout; r^-3 to full FP64 accuracy. */
    NBODY_FP64 = 0,
    /* Split precision: FP64 displacement, kicks, drifts and accumulation of
     * sources with mass >= small_mass; 1/|r|^3 from an FP32 reciprocal
     * square root refined by one FP64 Newton step for those sources;
     * sources lighter than small_mass are summed in FP32 with Kahan
     * compensation.  As run: where the each-pair-once pass (tile variant 5)
     * runs, a pair of two light bodies is evaluated wholly in FP32 (FP32
     * displacement, squared distance and reciprocal square root, no Newton
     * step) and its terms summed in blocks of 16 in FP32, each block added
     * to an FP64 sum; every other pair as in NBODY_FP64.  The one-way passes
     * form light sources' terms in FP32 and add blocks of 16 to a Kahan sum.
     * Faster than NBODY_FP64. */
    NBODY_SPLIT = 1,
    /* Split precision exactly as the split form is specified: FP64
     * displacement, squared distance, kicks and drifts; for every pair
     * 1/|r|^3 = y^3 with y the FP32 reciprocal square root of float(r^2)
     * refined by one FP64 Newton step; terms of sources with mass >=
     * small_mass accumulated in FP64, terms of lighter sources rounded to
     * FP32 (float(G m y^3) * float(d)) and accumulated in FP32 with Kahan
     * compensation (per workgroup of the each-pair-once pass, whose partial
     * sums are then added in FP64).  Runs in the each-pair-once pass only:
     * single systems of at most 131,072 bodies, ensembles of systems of at
     * most 10,240; NBODY_EUNSUPPORTED beyond.  Slower than NBODY_FP64 (about
     * twice the instructions per pair). */
    NBODY_SPLIT_COMPENSATED = 2
} nbody_precision;

typedef enum {
    NBODY_OP_ACCEL = 0,
    NBODY_OP_RUN = 1,
    NBODY_OP_ADJOINT = 2,
    NBODY_OP_BATCHED = 3,
    NBODY_OP_ENERGY = 4,
    NBODY_OP_RK4 = 5,
    /* nbody_verlet_checkpoints and nbody_verlet_adjoint_from_checkpoints
     * (the adjoint's workspace without its checkpoints) */
    NBODY_OP_ADJOINT_SWEEP = 6,
    /* nbody_accel_shard (n_total = the system's n; precision NBODY_FP64) */
    NBODY_OP_ACCEL_SHARD = 7
} nbody_op;

/* Bytes of workspace that `op` needs.  n_total: bodies (for BATCHED, the sum
 * over systems); num_systems: systems (1 unless BATCHED); steps and
 * checkpoint_every: only used by ADJOINT.  Returns 0 for invalid input. */
size_t nbody_workspace_bytes(int32_t op, int64_t n_total, int32_t num_systems,
                             int64_t steps, int64_t checkpoint_every,
                             int32_t precision);

/* Eq. (1): acc_out[3n] = accelerations of all n bodies at positions pos.
 * vel, dt and steps are accepted for a uniform argument block and ignored
 * (vel may be NULL).  precision: nbody_precision; small_mass is the split
 * threshold in mass units (ignored for NBODY_FP64).  n >= 1. */
int32_t nbody_accel(const double* pos, const double* vel, const double* mass,
                    int64_t n, double G, double dt, int64_t steps,
                    double* acc_out, int32_t precision, double small_mass,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Eq. (1) for a contiguous share of the targets: acc_out[3 * nt] (planes of
 * stride nt) = the FP64 accelerations of bodies t0 .. t0 + nt - 1 of the
 * n-body system at pos, each summed over all n sources.  This is one GPU's
 * force pass when the targets of a system are split among several GPUs that
 * each hold every source position (the Sec. 3 decomposition: each process
 * owns part of the bodies and needs all positions every step).  The pass is
 * the one-way kernel (sources split into chunks, partials summed in a fixed
 * chunk order), so the result is deterministic; it agrees with nbody_accel
 * to rounding, not bit for bit.  0 <= t0, 1 <= nt, t0 + nt <= n.  Workspace:
 * op NBODY_OP_ACCEL_SHARD for n.  Errors as nbody_accel; nothing is enqueued
 * on an invalid argument. */
int32_t nbody_accel_shard(const double* pos, const double* mass, int64_t n, double G,
                          int64_t t0, int64_t nt, double* acc_out,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Eqs. (3)-(4): advance (pos, vel) in place by `steps` velocity-Verlet steps
 * of size dt.  a(r_0) is computed first, then one evaluation of Eq. (1) per
 * step, so a run of n steps followed by one of m steps equals one run of
 * n + m steps bit for bit.  steps = 0 is a no-op.  The step sequence is the
 * kick-drift-kick form, which is Eqs. (3)-(4) rearranged (a_{i+1} is reused
 * as the next step's a_i).  Sets the non-finite flag read by
 * nbody_get_flags when any r, v or a stops being finite. */
int32_t nbody_verlet_run(double* pos, double* vel, const double* mass,
                         int64_t n, double G, double dt, int64_t steps,
                         int32_t precision, double small_mass,
                         void* workspace, size_t workspace_bytes, void* stream);

/* nbody_verlet_run for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same run, bit for bit, with no workspace argument.  Its
 * scratch memory (partials, G m, the second position buffer, the split
 * form's class-ordered copies, the flags word) is a static 32 MiB device
 * array that each GPU the library runs on holds until the process ends;
 * its address is looked up once per device.  Runs whose scratch would
 * exceed 32 MiB (about 20,000 bodies) return NBODY_EUNSUPPORTED with
 * nothing enqueued.  Every launch is enqueued directly on `stream` (no
 * captured graphs, which allocate), so a caller may itself capture the call;
 * the call allocates nothing and frees nothing.  Calls on one GPU share its
 * scratch: calls that overlap in time on that GPU (two streams, two host
 * threads) race and must not be made.  The non-finite flag is cleared at
 * the start of each call and not reported. */
int32_t nbody_verlet_run_static(double* pos, double* vel, const double* mass,
                                int64_t n, double G, double dt, int64_t steps,
                                int32_t precision, double small_mass, void* stream);

/* The classical fourth-order Runge-Kutta method, the higher-order
 * alternative to velocity Verlet that Sec. 2 names, for r' = v, v' = a(r)
 * with a from Eq. (1): advance (pos, vel) in place by `steps` steps of size
 * dt, four evaluations of Eq. (1) per step (at r, and at the three stage
 * positions r + dt/2 kr1, r + dt/2 kr2, r + dt kr3); (r, v) += dt/6 (k1 +
 * 2 k2 + 2 k3 + k4).  Not symplectic: its energy error grows with time,
 * as O(dt^4).  Arguments, precision, workspace (op NBODY_OP_RK4) and the
 * non-finite flag as for nbody_verlet_run; steps = 0 is a no-op and runs
 * chain bit for bit. */
int32_t nbody_rk4_run(double* pos, double* vel, const double* mass,
                      int64_t n, double G, double dt, int64_t steps,
                      int32_t precision, double small_mass,
                      void* workspace, size_t workspace_bytes, void* stream);

/* Gradient of a scalar loss L(r_T, v_T) of the FP64 run of Eqs. (3)-(4)
 * started from (pos0, vel0) with masses `mass`: the exact discrete adjoint
 * of the step map (reverse sweep, one Jacobian-transpose product of Eq. (1)
 * per step).  Inputs grad_posT = dL/dr_T, grad_velT = dL/dv_T ([3n] each).
 * Outputs grad_pos0, grad_vel0 ([3n]) and grad_mass ([n]); pos_out/vel_out
 * ([3n], may be NULL) receive r_T, v_T.  The forward run is stored every
 * checkpoint_every steps and recomputed segment by segment during the
 * reverse sweep; the library recomputes the next segment on a second stream
 * of its own (default priority) while `stream` sweeps the current one, and
 * every piece of that work is ordered before later work on `stream`.
 * Calls on one device enqueue one at a time.  Inputs are not modified.
 * checkpoint_every >= 1. */
int32_t nbody_verlet_adjoint(const double* pos0, const double* vel0, const double* mass,
                             int64_t n, double G, double dt, int64_t steps,
                             int64_t checkpoint_every,
                             const double* grad_posT, const double* grad_velT,
                             double* grad_pos0, double* grad_vel0, double* grad_mass,
                             double* pos_out, double* vel_out,
                             void* workspace, size_t workspace_bytes, void* stream);

/* The two halves of nbody_verlet_adjoint, for callers that run the forward
 * trajectory anyway (an autograd forward pass) and take its gradient later:
 * nbody_verlet_checkpoints runs the FP64 forward run of nbody_verlet_adjoint
 * from (pos0, vel0), storing (r, v) at steps 0, K, 2K, ... and at `steps`
 * into `checkpoints` (a DEVICE buffer of (ceil(steps / K) + 1) * 6n doubles,
 * record k = r_kK in doubles [6nk, 6nk + 3n) and v_kK in the next 3n; the
 * last record holds the final state) and the final state into pos_out /
 * vel_out (may be NULL); nbody_verlet_adjoint_from_checkpoints runs the
 * reverse sweep of nbody_verlet_adjoint from such a buffer (unchanged, and
 * the same n, G, dt, steps, K and masses).  Their results equal
 * nbody_verlet_adjoint's bit for bit.  Workspace: nbody_workspace_bytes with
 * op NBODY_OP_ADJOINT_SWEEP.  K = checkpoint_every >= 1. */
int32_t nbody_verlet_checkpoints(const double* pos0, const double* vel0, const double* mass,
                                 int64_t n, double G, double dt, int64_t steps,
                                 int64_t checkpoint_every, double* checkpoints,
                                 double* pos_out, double* vel_out,
                                 void* workspace, size_t workspace_bytes, void* stream);
int32_t nbody_verlet_adjoint_from_checkpoints(const double* checkpoints, const double* mass,
                                              int64_t n, double G, double dt, int64_t steps,
                                              int64_t checkpoint_every,
                                              const double* grad_posT, const double* grad_velT,
                                              double* grad_pos0, double* grad_vel0,
                                              double* grad_mass, void* workspace,
                                              size_t workspace_bytes, void* stream);

/* Eqs. (3)-(4) for num_systems independent systems in one launch per step.
 * System k owns bodies [offsets_host[k], offsets_host[k+1]) of the
 * concatenated SoA arrays (plane stride = offsets_host[num_systems]); bodies
 * of different systems do not interact.  offsets_host is a HOST array of
 * num_systems + 1 non-decreasing values starting at 0; every system has at
 * least one body.  The step loop is captured into a HIP graph on first use
 * and replayed.  Tile: the one nbody_autotune_batched chose, else each pair
 * once (variant 5, (4, 4)) when every system has at most 10,240 bodies and
 * sum n_k^2 / sum n_k >= 2,048, else the one-way heuristic; a variant-5 tile
 * with a system of more than 10,240 bodies gives way to the one-way
 * heuristic. */
int32_t nbody_verlet_run_batched(double* pos, double* vel, const double* mass,
                                 const int64_t* offsets_host, int32_t num_systems,
                                 double G, double dt, int64_t steps,
                                 int32_t precision, double small_mass,
                                 void* workspace, size_t workspace_bytes, void* stream);

/* Sec. 2 accuracy measure: out[0] = kinetic sum m|v|^2/2, out[1] = potential
 * -sum_{i<j} G m_i m_j / |r_i - r_j|, out[2] = total.  `out` is a DEVICE
 * array of 3 doubles.  FP64 with compensated sums; deterministic. */
int32_t nbody_energy(const double* pos, const double* vel, const double* mass,
                     int64_t n, double G, double* out,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Total linear and angular momentum: out[0..3) = sum m v,
 * out[3..6) = sum m r x v (DEVICE array of 6 doubles, compensated). */
int32_t nbody_momenta(const double* pos, const double* vel, const double* mass,
                      int64_t n, double* out, void* stream);

/* Flags set by the last runs on this workspace (bit 0: a non-finite r, v or
 * a was produced).  Synchronises `stream`.  clear != 0 resets them. */
int32_t nbody_get_flags(void* workspace, void* stream, int32_t clear, int32_t* flags_host);

/* Tile shape of the force pass: targets per lane (1, 2, 4), waves per
 * workgroup (1, 2, 4, 8), source chunks (1..64) and how sources reach the
 * lanes (variant 0: staged through LDS; 1: read once per wavefront into
 * scalar registers; 2: as 1, the waves of a workgroup sharing targets and
 * splitting the sources; the adjoint pass supports variants 0, 1 and 5
 * and defaults to 1 below 4,500 bodies, to 5 in shape (4, 4) from there).
 * Variant 3 (kind 0 only, n <= 512, targets_per_lane = 1, waves = 16):
 * one workgroup holds the system in LDS and runs whole steps, force pass,
 * reduction and kick-drift-kick, in one launch; chunks is then the number
 * of source slices per target (capped at 1024 / n).  The heuristic picks it
 * for n <= 160.
 * Variant 4 (kind 0 only, targets_per_lane 1 or 2, waves 2, 4 or 8, chunks
 * 1): the waves of a workgroup split all sources of its targets, and the
 * same kernel applies the step's kicks and drift, so a step is one launch.
 * The heuristic picks it for 160 < n <= 512.
 * Variant 5 (kinds 0 and 1; (targets_per_lane, waves) = (1, 4), (2, 2), (2, 4) or
 * (4, 4); chunks 1): each unordered pair is evaluated once and the reaction
 * is added to the source (Newton's third law applied to Eq. (1)); in the
 * split form pairs of light bodies are evaluated in FP32 both ways and every
 * pair of a target block holding a heavy body in FP64.  The pass writes one
 * partial per range of 256 bodies and is accepted for n <= 131,072 (the
 * workspace of nbody_accel, nbody_verlet_run, nbody_rk4_run and
 * nbody_verlet_adjoint holds ceil(n / 256) partial slots, or a few more
 * for a split last round (below), up to that size:
 * 1.6 GB at n = 131,072).  With (4, 4), when the range pairs past the last
 * whole round of 256 workgroups are few (at most 128, of at most 16,384
 * pairs), each of them runs as two workgroups over half of the sub-phases
 * each, and extra slots take the second halves' target sums and reactions
 * (47 slots at n = 10,425); the transpose-Jacobian pass (kind 1, variant 5,
 * shape (4, 4)) splits its last round the same way.  Results stay bitwise
 * repeatable.  The heuristic picks (4, 4) from n = 4,096 (FP64) or 8,000
 * (split) up to n = 131,072, and for kind 1 from n = 4,500. */
typedef struct {
    int32_t targets_per_lane;
    int32_t waves;
    int32_t chunks;
    int32_t variant;
} nbody_tile;

/* The tile shape the library will use for (kind, precision, n): the tuned
 * one if nbody_autotune ran for that size class, else a heuristic.
 * kind: 0 = force pass, 1 = adjoint pass, 2 = batched ensemble (n is
 * ignored; chunks are chosen per system; without a tuned tile this reports
 * the one-way heuristic, while a run may take variant 5 from its system
 * sizes, see nbody_verlet_run_batched). */
int32_t nbody_get_tile(int32_t kind, int32_t precision, int64_t n, nbody_tile* tile_host);

/* Force a tile shape for (kind, precision, n's size class); shapes outside
 * the supported set return NBODY_EINVAL. */
int32_t nbody_set_tile(int32_t kind, int32_t precision, int64_t n, const nbody_tile* tile_host);

/* Time candidate tile shapes for (kind, precision) on the caller's data with
 * HIP events and keep the fastest for n's size class.  pos and mass as for
 * nbody_accel; synchronises `stream`.  best_host (may be NULL) receives the
 * winner and best_ms_host (may be NULL) its time per force pass. */
int32_t nbody_autotune(int32_t kind, int32_t precision, const double* pos, const double* mass,
                       int64_t n, double G, double small_mass,
                       void* workspace, size_t workspace_bytes, void* stream,
                       nbody_tile* best_host, double* best_ms_host);

/* As nbody_autotune for the batched ensemble: times the ensemble's force pass
 * and its epilogue (one launch each over all systems) for candidate tile
 * shapes, variant 5 among them when every system has at most 10,240 bodies,
 * and keeps the fastest for kind 2.  offsets_host as for nbody_verlet_run_batched.
 * Synchronises `stream`. */
int32_t nbody_autotune_batched(int32_t precision, const double* pos, const double* mass,
                               const int64_t* offsets_host, int32_t num_systems, double G,
                               double small_mass, void* workspace, size_t workspace_bytes,
                               void* stream, nbody_tile* best_host, double* best_ms_host);

/* Average duration (ms) of one force pass (kind 0: Eq. (1) for `precision`;
 * kind 1: the adjoint's transpose-Jacobian pass) over `reps` back-to-back
 * launches with the current tile shape, timed by HIP events recorded on
 * `stream` around the force kernels only.  Inputs as for nbody_accel (kind 1
 * uses a constant cotangent).  Synchronises `stream`. */
int32_t nbody_time_force(int32_t kind, int32_t precision, const double* pos, const double* mass,
                         int64_t n, double G, double small_mass, int32_t reps,
                         void* workspace, size_t workspace_bytes, void* stream,
                         double* ms_per_pass_host);

/* Drops captured graphs, ensemble work lists and tuned tile shapes; waits
 * for the devices those graphs ran on first. */
void nbody_reset_caches(void);

/* Message describing the calling thread's last failure ("" if none). */
const char* nbody_last_error(void);

/* Library version string. */
const char* nbody_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
