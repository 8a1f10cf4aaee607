// O(N) kernels around the force pass: the kick-drift-kick step epilogue that
// realises Eqs. (3)-(4), the class-order gather/scatter of the split form,
// and the diagnostics of Sec. 2 (energy, momenta).
#include "common.hpp"
#include "pair_math.hpp"
#include "reduce.hpp"

namespace nb {
namespace {

using namespace pm;

constexpr int kBlock = 256;

// Sum the chunk partials of a_p in a fixed order (below), then apply the
// half kicks and the drift:
//   kClose: v += dt/2 a                         (v_{i+1}, end of step i)
//   kOpen:  v += dt/2 a;  r_out = r_in + dt v   (v_{i+3/2}, r_{i+2})
// Eqs. (3)-(4) follow: r_{i+1} = r_i + dt (v_i + dt/2 a_i) and
// v_{i+1} = v_i + dt/2 a_i + dt/2 a_{i+1}.
// GS threads per (body, component) sum the partials (chunk_sum); the state
// the epilogue reads is loaded before the partials, so its latency overlaps
// theirs.
// PER_BODY: an ensemble's per-body partial counts (body_chunks) instead of
// one count for every body.
template <int GS, bool PER_BODY>
__global__ __launch_bounds__(kBlock) void k_step(const double* __restrict__ part, int chunks,
                                                 const int8_t* __restrict__ body_chunks,
                                                 int64_t n, double* __restrict__ vel,
                                                 const double* __restrict__ pos_in,
                                                 double* __restrict__ pos_out,
                                                 double* __restrict__ acc, double hdt, double dt,
                                                 int mode, uint32_t* __restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = t / GS;   // k * n + p
    const int sub = (int)(t % GS);
    const bool live = i < 3 * n;
    const int64_t ii = live ? i : 0;
    const int64_t p = ii % n;
    const int C = PER_BODY ? (int)body_chunks[p] : chunks;
    const bool head = live && sub == 0;
    const double v0 = (head && (mode & (kClose | kOpen))) ? vel[i] : 0.0;
    const double r0 = (head && (mode & kOpen)) ? pos_in[i] : 0.0;
    const double a = chunk_sum<GS>(part, C, 3 * n, ii, sub, live);
    if (!head) return;
    bool finite = __builtin_isfinite(a);
    if (mode & kStoreAcc) acc[i] = a;
    if (mode & (kClose | kOpen)) {
        double v = v0;
        if (mode & kClose) v = v + hdt * a;
        if (mode & kOpen) {
            v = v + hdt * a;
            const double r = r0 + dt * v;
            finite = finite && __builtin_isfinite(r);
            pos_out[i] = r;
        }
        finite = finite && __builtin_isfinite(v);
        vel[i] = v;
    }
    if (!finite && flags) atomicOr(flags, 1u);
}

// The accelerations of targets t0 .. t0 + nt - 1 from the chunk partials of
// a pass over those targets (GS threads per (component, target) element,
// summed by chunk_sum), into planes of stride nt.
template <int GS>
__global__ __launch_bounds__(kBlock) void k_shard_sum(const double* __restrict__ part,
                                                      int chunks, int64_t n, int64_t t0,
                                                      int64_t nt, double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t e = t / GS;   // k * nt + q
    const int sub = (int)(t % GS);
    const bool live = e < 3 * nt;
    const int64_t ee = live ? e : 0;
    const int64_t k = ee / nt;
    const int64_t q = ee - k * nt;
    const double a = chunk_sum<GS>(part, chunks, 3 * n, k * n + t0 + q, sub, live);
    if (live && sub == 0) out[e] = a;
}

// Classical fourth-order Runge-Kutta (r' = v, v' = a(r)): stage s's
// acceleration a (the chunk partials of the force pass at the stage position,
// summed in ascending chunk order) and the stage velocity give the slopes
// (kr, kv); sr, sv accumulate kr1 + 2 kr2 + 2 kr3 and kv1 + 2 kv2 + 2 kv3;
//   s = 1: kr = v,  next stage at (r + dt/2 kr, v + dt/2 kv)
//   s = 2: kr = vs, next stage at (r + dt/2 kr, v + dt/2 kv)
//   s = 3: kr = vs, next stage at (r + dt kr,   v + dt kv)
//   s = 4: kr = vs, r += dt/6 (sr + kr), v += dt/6 (sv + kv).
template <int GS>
__global__ __launch_bounds__(kBlock) void k_rk4_stage(const double* __restrict__ part, int chunks,
                                                      int64_t n, int stage, double dt,
                                                      double* __restrict__ pos,
                                                      double* __restrict__ vel,
                                                      double* __restrict__ rs,
                                                      double* __restrict__ vs,
                                                      double* __restrict__ sr,
                                                      double* __restrict__ sv,
                                                      uint32_t* __restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = t / GS;
    const int sub = (int)(t % GS);
    const bool live = i < 3 * n;
    const int64_t ii = live ? i : 0;
    const bool head = live && sub == 0;
    double p0 = 0.0, v0 = 0.0, vs0 = 0.0, sr0 = 0.0, sv0 = 0.0;
    if (head) {
        p0 = pos[i];
        v0 = vel[i];
        if (stage > 1) {
            vs0 = vs[i];
            sr0 = sr[i];
            sv0 = sv[i];
        }
    }
    const double a = chunk_sum<GS>(part, chunks, 3 * n, ii, sub, live);
    if (!head) return;
    bool finite = __builtin_isfinite(a);
    const double kr = (stage == 1) ? v0 : vs0;
    if (stage < 4) {
        if (stage == 1) {
            sr[i] = kr;
            sv[i] = a;
        } else {
            sr[i] = sr0 + 2.0 * kr;
            sv[i] = sv0 + 2.0 * a;
        }
        const double h = (stage == 3) ? dt : 0.5 * dt;
        const double r = p0 + h * kr;
        const double v = v0 + h * a;
        finite = finite && __builtin_isfinite(r) && __builtin_isfinite(v);
        rs[i] = r;
        vs[i] = v;
    } else {
        const double h6 = dt / 6.0;
        const double r = p0 + h6 * (sr0 + kr);
        const double v = v0 + h6 * (sv0 + a);
        finite = finite && __builtin_isfinite(r) && __builtin_isfinite(v);
        pos[i] = r;
        vel[i] = v;
    }
    if (!finite && flags) atomicOr(flags, 1u);
}

__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* __restrict__ perm, int64_t n,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst, int planes)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    for (int k = 0; k < planes; ++k) dst[(int64_t)k * n + i] = src[(int64_t)k * n + j];
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ perm, int64_t n,
                                                    const double* __restrict__ src,
                                                    double* __restrict__ dst, int planes)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    for (int k = 0; k < planes; ++k) dst[(int64_t)k * n + j] = src[(int64_t)k * n + i];
}

// Stable partition of each system into mass >= thr first (one workgroup per
// system): a count pass, then a block-wide scan per 1024-body slice.
constexpr int kPart = 1024;

__global__ __launch_bounds__(kPart) void k_partition(const double* __restrict__ mass,
                                                     const int64_t* __restrict__ offsets,
                                                     int64_t n_single, double thr,
                                                     int32_t* __restrict__ perm,
                                                     int64_t* __restrict__ nmaj)
{
    __shared__ int scan[kPart];
    const int tid = threadIdx.x;
    const int64_t b0 = offsets ? offsets[blockIdx.x] : 0;
    const int64_t b1 = offsets ? offsets[blockIdx.x + 1] : n_single;

    int cnt = 0;
    for (int64_t i = b0 + tid; i < b1; i += kPart) cnt += (mass[i] >= thr) ? 1 : 0;
    scan[tid] = cnt;
    __syncthreads();
    for (int w = kPart / 2; w > 0; w >>= 1) {
        if (tid < w) scan[tid] += scan[tid + w];
        __syncthreads();
    }
    const int64_t total = scan[0];
    __syncthreads();

    int64_t base_major = 0, base_small = total;
    for (int64_t c0 = b0; c0 < b1; c0 += kPart) {
        const int64_t i = c0 + tid;
        const bool valid = i < b1;
        const int f = (valid && mass[i] >= thr) ? 1 : 0;
        scan[tid] = f;
        __syncthreads();
        for (int off = 1; off < kPart; off <<= 1) {
            const int v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int excl = scan[tid] - f;          // majors before tid in this slice
        const int chunk_major = scan[kPart - 1];
        if (valid) {
            if (f) perm[b0 + base_major + excl] = (int32_t)i;
            else   perm[b0 + base_small + (tid - excl)] = (int32_t)i;
        }
        const int64_t nvalid = (b1 - c0 < kPart) ? (b1 - c0) : kPart;
        base_major += chunk_major;
        base_small += nvalid - chunk_major;
        __syncthreads();
    }
    if (tid == 0) nmaj[blockIdx.x] = total;
}

// ---------------------------------------------------------------------------
// Diagnostics.  Neumaier-compensated sums; fixed summation order.
struct CSum {
    double s, c;
};

__device__ __forceinline__ void cadd(CSum& a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
    else                      a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void cmerge(CSum& a, const CSum& b)
{
    cadd(a, b.s);
    cadd(a, b.c);
}

constexpr int kRowTile = 256;

// Row sums of the pair potential of Sec. 2 over one chunk of sources, each
// unordered pair once: S_c(p) = sum_{j in chunk c, j > p} m_j / |r_j - r_p|,
// compensated, stored as (s, c) in part[2c][p], part[2c + 1][p] (grid.y =
// chunks of chunk_len; a chunk wholly below the row block has nothing to do).
__global__ __launch_bounds__(kRowTile) void k_potential_rows(const double* __restrict__ pos,
                                                             const double* __restrict__ mass,
                                                             int64_t n, int64_t chunk_len,
                                                             double* __restrict__ part)
{
    __shared__ double sx[kRowTile], sy[kRowTile], sz[kRowTile], sm[kRowTile];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kRowTile + tid;
    const int64_t q = p < n ? p : n - 1;
    const double px = pos[q], py = pos[n + q], pz = pos[2 * n + q];
    const int64_t je0 = (int64_t)(blockIdx.y + 1) * chunk_len;
    const int64_t je = je0 < n ? je0 : n;
    const int64_t row0 = (int64_t)blockIdx.x * kRowTile;
    // sources j > p only: start at the row block's first row + 1 at the earliest
    const int64_t jb = (int64_t)blockIdx.y * chunk_len > row0 + 1 ? (int64_t)blockIdx.y * chunk_len
                                                                  : row0 + 1;
    CSum acc = {0.0, 0.0};
    for (int64_t j0 = jb; j0 < je; j0 += kRowTile) {
        const int64_t j = j0 + tid;
        __syncthreads();
        if (j < je) {
            sx[tid] = pos[j];
            sy[tid] = pos[n + j];
            sz[tid] = pos[2 * n + j];
            sm[tid] = mass[j];
        }
        __syncthreads();
        const int cnt = (je - j0 < kRowTile) ? (int)(je - j0) : kRowTile;
        for (int jj = 0; jj < cnt; ++jj) {
            if (j0 + jj <= q) continue;
            const double dx = sx[jj] - px, dy = sy[jj] - py, dz = sz[jj] - pz;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            cadd(acc, sm[jj] * rinv_f64(r2));
        }
    }
    if (p < n) {
        part[(int64_t)(2 * blockIdx.y) * n + p] = acc.s;
        part[(int64_t)(2 * blockIdx.y + 1) * n + p] = acc.c;
    }
}

// rows[p] = -G m_p * (the chunk sums merged in chunk order); sum_p rows[p] is
// the pair potential (each unordered pair once).
__global__ __launch_bounds__(kBlock) void k_potential_merge(const double* __restrict__ part,
                                                            int chunks, const double* __restrict__ mass,
                                                            int64_t n, double G,
                                                            double* __restrict__ rows)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    CSum m = {0.0, 0.0};
    for (int c = 0; c < chunks; ++c)
        cmerge(m, CSum{part[(int64_t)(2 * c) * n + p], part[(int64_t)(2 * c + 1) * n + p]});
    rows[p] = -G * mass[p] * (m.s + m.c);
}

constexpr int kRed = 1024;

__device__ void block_reduce(CSum* sh, CSum v, int nvals)
{
    // Writes the combined value of all threads' v into sh[0]; fixed order.
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = kRed / 2; w > 0; w >>= 1) {
        if (tid < w) {
            CSum a = sh[tid];
            cmerge(a, sh[tid + w]);
            sh[tid] = a;
        }
        __syncthreads();
    }
    (void)nvals;
}

__global__ __launch_bounds__(kRed) void k_energy_finish(const double* __restrict__ rows,
                                                        const double* __restrict__ vel,
                                                        const double* __restrict__ mass,
                                                        int64_t n, double* __restrict__ out)
{
    __shared__ CSum sh[kRed];
    const int tid = threadIdx.x;
    CSum kin = {0.0, 0.0}, pot = {0.0, 0.0};
    for (int64_t i = tid; i < n; i += kRed) {
        const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        cadd(kin, 0.5 * mass[i] * (vx * vx + vy * vy + vz * vz));
        cadd(pot, rows[i]);
    }
    block_reduce(sh, kin, kRed);
    const CSum K = sh[0];
    __syncthreads();
    block_reduce(sh, pot, kRed);
    const CSum U = sh[0];
    if (tid == 0) {
        const double k = K.s + K.c, u = U.s + U.c;
        CSum e = {0.0, 0.0};
        cadd(e, k);
        cadd(e, u);
        out[0] = k;
        out[1] = u;
        out[2] = e.s + e.c;
    }
}

__global__ __launch_bounds__(kRed) void k_momenta(const double* __restrict__ pos,
                                                  const double* __restrict__ vel,
                                                  const double* __restrict__ mass, int64_t n,
                                                  double* __restrict__ out)
{
    __shared__ CSum sh[kRed];
    const int tid = threadIdx.x;
    CSum c[6];
    for (int k = 0; k < 6; ++k) c[k] = {0.0, 0.0};
    for (int64_t i = tid; i < n; i += kRed) {
        const double rx = pos[i], ry = pos[n + i], rz = pos[2 * n + i];
        const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        const double m = mass[i];
        cadd(c[0], m * vx);
        cadd(c[1], m * vy);
        cadd(c[2], m * vz);
        cadd(c[3], m * (ry * vz - rz * vy));
        cadd(c[4], m * (rz * vx - rx * vz));
        cadd(c[5], m * (rx * vy - ry * vx));
    }
    for (int k = 0; k < 6; ++k) {
        block_reduce(sh, c[k], kRed);
        if (tid == 0) out[k] = sh[0].s + sh[0].c;
        __syncthreads();
    }
}

}  // namespace

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_step(const double* part, int chunks, const int8_t* body_chunks, int64_t n,
                       double* vel, const double* pos_in, double* pos_out, double* acc,
                       double dt, int mode, uint32_t* flags, hipStream_t s)
{
    // four threads per element for 16 to 95 partials of a single system; one
    // below that, from 96 partials (the each-pair-once pass on large systems)
    // and for an ensemble's per-body counts, where each load of a wavefront
    // then reads 512 contiguous bytes of one partial plane (measured faster)
    if (body_chunks)
        hipLaunchKernelGGL((k_step<1, true>), dim3(blocks_for(3 * n, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, body_chunks, n, vel, pos_in, pos_out, acc, 0.5 * dt, dt,
                           mode, flags);
    else if (chunks >= 16 && chunks < 96)
        hipLaunchKernelGGL((k_step<4, false>), dim3(blocks_for(12 * n, kBlock)), dim3(kBlock), 0,
                           s, part, chunks, body_chunks, n, vel, pos_in, pos_out, acc, 0.5 * dt,
                           dt, mode, flags);
    else
        hipLaunchKernelGGL((k_step<1, false>), dim3(blocks_for(3 * n, kBlock)), dim3(kBlock), 0,
                           s, part, chunks, body_chunks, n, vel, pos_in, pos_out, acc, 0.5 * dt,
                           dt, mode, flags);
    return hipGetLastError();
}

hipError_t launch_shard_sum(const double* part, int chunks, int64_t n, int64_t t0, int64_t nt,
                            double* out, hipStream_t s)
{
    if (chunks >= 16 && chunks < 96)
        hipLaunchKernelGGL(k_shard_sum<4>, dim3(blocks_for(12 * nt, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, t0, nt, out);
    else
        hipLaunchKernelGGL(k_shard_sum<1>, dim3(blocks_for(3 * nt, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, t0, nt, out);
    return hipGetLastError();
}

hipError_t launch_rk4_stage(const double* part, int chunks, int64_t n, int stage, double dt,
                            double* pos, double* vel, double* rs, double* vs, double* sr,
                            double* sv, uint32_t* flags, hipStream_t s)
{
    if (stage < 1 || stage > 4) return hipErrorInvalidValue;
    if (chunks >= 16)
        hipLaunchKernelGGL(k_rk4_stage<4>, dim3(blocks_for(12 * n, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, stage, dt, pos, vel, rs, vs, sr, sv, flags);
    else
        hipLaunchKernelGGL(k_rk4_stage<1>, dim3(blocks_for(3 * n, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, stage, dt, pos, vel, rs, vs, sr, sv, flags);
    return hipGetLastError();
}

hipError_t launch_partition(const double* mass, const int64_t* offsets, int num_systems,
                            int64_t n_single, double threshold, int32_t* perm, int64_t* nmaj,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_partition, dim3((unsigned)num_systems), dim3(kPart), 0, s, mass, offsets,
                       n_single, threshold, perm, nmaj);
    return hipGetLastError();
}

hipError_t launch_gather(const int32_t* perm, int64_t n, const double* src, double* dst,
                         int planes, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, perm, n, src,
                       dst, planes);
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* perm, int64_t n, const double* src, double* dst,
                          int planes, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, perm, n, src,
                       dst, planes);
    return hipGetLastError();
}

hipError_t launch_potential_rows(const double* pos, const double* mass, int64_t n, double G,
                                 double* part, int max_chunks, double* rows, hipStream_t s)
{
    // source chunks of whole tiles until about 1024 workgroups have work (half
    // of the (row block, chunk) grid lies below the diagonal)
    const int64_t row_blocks = blocks_for(n, kRowTile);
    int64_t c = (2048 + row_blocks - 1) / row_blocks;
    c = c < 1 ? 1 : (c > max_chunks ? max_chunks : c);
    const int64_t per = (n + c - 1) / c;
    const int64_t chunk_len = (per + kRowTile - 1) / kRowTile * kRowTile;
    const int chunks = (int)((n + chunk_len - 1) / chunk_len);
    hipLaunchKernelGGL(k_potential_rows, dim3((unsigned)row_blocks, (unsigned)chunks),
                       dim3(kRowTile), 0, s, pos, mass, n, chunk_len, part);
    hipLaunchKernelGGL(k_potential_merge, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, part,
                       chunks, mass, n, G, rows);
    return hipGetLastError();
}

hipError_t launch_energy_finish(const double* rows, const double* vel, const double* mass,
                                int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(kRed), 0, s, rows, vel, mass, n, out);
    return hipGetLastError();
}

hipError_t launch_momenta(const double* pos, const double* vel, const double* mass, int64_t n,
                          double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_momenta, dim3(1), dim3(kRed), 0, s, pos, vel, mass, n, out);
    return hipGetLastError();
}

}  // namespace nb
