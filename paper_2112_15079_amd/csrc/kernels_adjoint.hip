// Transpose of the Jacobian of Eq. (1), the inner operation of the discrete
// adjoint of the velocity-Verlet trajectory.
//
// With d_qj = r_j - r_q and the tidal tensor K(d) = I/|d|^3 - 3 d d^T/|d|^5
// (symmetric, even in d), the Jacobian blocks of Eq. (1) are
//   d a_p/d r_q = G m_q K(d_pq)  (q != p),   d a_p/d r_p = -sum_j G m_j K(d_pj),
//   d a_p/d m_q = G d_pq / |d_pq|^3.
// For a cotangent u on the accelerations this gives, per body q,
//   (J^T u)_q = G sum_{j != q} K(d_qj) (m_q u_j - m_j u_q)
//   (M^T u)_q = -G sum_{j != q} u_j . d_qj / |d_qj|^3,
// one all-pairs pass over (r, m, u) with the same tiling as the force pass.
#include "common.hpp"
#include "pair_math.hpp"
#include "reduce.hpp"

namespace nb {
namespace {

using namespace pm;

struct __attribute__((aligned(64))) ASrc {
    double x, y, z, m, ux, uy, uz, pad;
};

constexpr double kPad = 1.0e18;

// Sources [0, cnt) of the LDS tile (cnt is the same for the whole workgroup).
template <int T, int W, bool MASK>
__device__ __forceinline__ void vjp_sweep(const ASrc* __restrict__ tile, int cnt, int j0,
                                          const double (&qx)[T], const double (&qy)[T],
                                          const double (&qz)[T], const double (&qm)[T],
                                          const double (&ux)[T], const double (&uy)[T],
                                          const double (&uz)[T], const int (&qid)[T],
                                          double (&ox)[T], double (&oy)[T], double (&oz)[T],
                                          double (&og)[T])
{
#pragma unroll 2
    for (int jj = 0; jj < cnt; ++jj) {
        const ASrc s = tile[jj];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const double dx = s.x - qx[t];
            const double dy = s.y - qy[t];
            const double dz = s.z - qz[t];
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const double y = rinv_f64(r2);
            const double y2 = y * y;
            double i3 = y * y2;
            double i5 = i3 * y2;
            if (MASK) {
                const bool self = (j0 + jj == qid[t]);
                i3 = self ? 0.0 : i3;
                i5 = self ? 0.0 : i5;
            }
            // w = m_q u_j - m_j u_q
            const double wx = __builtin_fma(-s.m, ux[t], qm[t] * s.ux);
            const double wy = __builtin_fma(-s.m, uy[t], qm[t] * s.uy);
            const double wz = __builtin_fma(-s.m, uz[t], qm[t] * s.uz);
            const double dw = __builtin_fma(dz, wz, __builtin_fma(dy, wy, dx * wx));
            const double c = 3.0 * dw * i5;
            ox[t] = __builtin_fma(-c, dx, __builtin_fma(wx, i3, ox[t]));
            oy[t] = __builtin_fma(-c, dy, __builtin_fma(wy, i3, oy[t]));
            oz[t] = __builtin_fma(-c, dz, __builtin_fma(wz, i3, oz[t]));
            const double ud = __builtin_fma(s.uz, dz, __builtin_fma(s.uy, dy, s.ux * dx));
            og[t] = __builtin_fma(ud, i3, og[t]);
        }
    }
}

// part[c*4n + k*n + q]: chunk-c partials of G (K (m_q u_j - m_j u_q)) (k < 3)
// and of -G u_j . d / |d|^3 (k = 3), for the cotangent u = cu * lam.
template <int T, int W>
__global__ __launch_bounds__(64 * W) void k_vjp(const double* __restrict__ pos,
                                                const double* __restrict__ mass,
                                                const double* __restrict__ lam, double cu,
                                                int64_t n, int64_t chunk_len, double G,
                                                double* __restrict__ part)
{
    constexpr int NT = 64 * W;
    __shared__ ASrc tile[NT];
    const int tid = threadIdx.x;
    const int64_t tb0 = (int64_t)blockIdx.x * NT * T;
    const int64_t c = blockIdx.y;
    const int64_t jbeg = c * chunk_len;
    const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;

    double qx[T], qy[T], qz[T], qm[T], ux[T], uy[T], uz[T];
    double ox[T], oy[T], oz[T], og[T];
    int qid[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = tb0 + (int64_t)t * NT + tid;
        const int64_t q = p < n ? p : n - 1;
        qid[t] = (int)p;
        qx[t] = pos[q]; qy[t] = pos[n + q]; qz[t] = pos[2 * n + q];
        qm[t] = mass[q];
        ux[t] = cu * lam[q]; uy[t] = cu * lam[n + q]; uz[t] = cu * lam[2 * n + q];
        ox[t] = 0.0; oy[t] = 0.0; oz[t] = 0.0; og[t] = 0.0;
    }
    const int64_t tend = tb0 + (int64_t)NT * T;
    for (int64_t j0 = jbeg; j0 < jend; j0 += NT) {
        const int64_t j = j0 + tid;
        ASrc s;
        if (j < jend) {
            s.x = pos[j]; s.y = pos[n + j]; s.z = pos[2 * n + j];
            s.m = mass[j];
            s.ux = cu * lam[j]; s.uy = cu * lam[n + j]; s.uz = cu * lam[2 * n + j];
        } else {
            s.x = kPad; s.y = kPad; s.z = kPad;
            s.m = 0.0; s.ux = 0.0; s.uy = 0.0; s.uz = 0.0;
        }
        s.pad = 0.0;
        __syncthreads();
        tile[tid] = s;
        __syncthreads();
        // chunks are multiples of 8 sources, not of the tile width: the last
        // tile of a chunk is swept only over its valid sources
        const int cnt = (int)((jend - j0) < NT ? (jend - j0) : NT);
        const bool diag = (j0 < tend) && (tb0 < j0 + NT);
        if (diag) vjp_sweep<T, W, true>(tile, cnt, (int)j0, qx, qy, qz, qm, ux, uy, uz, qid, ox, oy, oz, og);
        else      vjp_sweep<T, W, false>(tile, cnt, (int)j0, qx, qy, qz, qm, ux, uy, uz, qid, ox, oy, oz, og);
    }
    double* pc = part + c * 4 * n;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = tb0 + (int64_t)t * NT + tid;
        if (p < n) {
            __builtin_nontemporal_store(G * ox[t], &pc[p]);
            __builtin_nontemporal_store(G * oy[t], &pc[n + p]);
            __builtin_nontemporal_store(G * oz[t], &pc[2 * n + p]);
            __builtin_nontemporal_store(-G * og[t], &pc[3 * n + p]);
        }
    }
}

// Scalar-operand form (tile variant 1): every lane of a wavefront needs the
// same source, so the wave reads kVG sources at a time from the planes at a
// uniform index (scalar loads; no LDS, no barriers) and sweeps its chunk.
// The product is linear in the cotangent, so it runs on lam and the outputs
// are scaled by cu.
constexpr int kVG = 4;

template <int T, bool MASK>
__device__ __forceinline__ void vjp_pair(double sx, double sy, double sz, double sm, double sux,
                                         double suy, double suz, int64_t j, const double (&qx)[T],
                                         const double (&qy)[T], const double (&qz)[T],
                                         const double (&qm)[T], const double (&ux)[T],
                                         const double (&uy)[T], const double (&uz)[T],
                                         const int64_t (&qid)[T], double (&ox)[T],
                                         double (&oy)[T], double (&oz)[T], double (&og)[T])
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const double dx = sx - qx[t];
        const double dy = sy - qy[t];
        const double dz = sz - qz[t];
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const double y = rinv_f64(r2);
        const double y2 = y * y;
        double i3 = y * y2;
        double i5 = i3 * y2;
        if (MASK) {
            const bool self = (j == qid[t]);
            i3 = self ? 0.0 : i3;
            i5 = self ? 0.0 : i5;
        }
        const double wx = __builtin_fma(-sm, ux[t], qm[t] * sux);
        const double wy = __builtin_fma(-sm, uy[t], qm[t] * suy);
        const double wz = __builtin_fma(-sm, uz[t], qm[t] * suz);
        const double dw = __builtin_fma(dz, wz, __builtin_fma(dy, wy, dx * wx));
        const double c = 3.0 * dw * i5;
        ox[t] = __builtin_fma(-c, dx, __builtin_fma(wx, i3, ox[t]));
        oy[t] = __builtin_fma(-c, dy, __builtin_fma(wy, i3, oy[t]));
        oz[t] = __builtin_fma(-c, dz, __builtin_fma(wz, i3, oz[t]));
        const double ud = __builtin_fma(suz, dz, __builtin_fma(suy, dy, sux * dx));
        og[t] = __builtin_fma(ud, i3, og[t]);
    }
}

template <int T, int W>
__global__ __launch_bounds__(64 * W) void k_vjp_s(const double* __restrict__ pos,
                                                  const double* __restrict__ mass,
                                                  const double* __restrict__ lam, double cu,
                                                  int64_t n, int64_t chunk_len, double G,
                                                  double* __restrict__ part)
{
    constexpr int NT = 64 * W;
    const int tid = threadIdx.x;
    const int64_t tb0 = (int64_t)blockIdx.x * NT * T;
    const int64_t c = blockIdx.y;
    const int64_t jbeg = c * chunk_len;
    const int64_t jend = (jbeg + chunk_len < n) ? jbeg + chunk_len : n;

    double qx[T], qy[T], qz[T], qm[T], ux[T], uy[T], uz[T];
    double ox[T], oy[T], oz[T], og[T];
    int64_t qid[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = tb0 + (int64_t)t * NT + tid;
        const int64_t q = p < n ? p : n - 1;
        qid[t] = p;
        qx[t] = pos[q]; qy[t] = pos[n + q]; qz[t] = pos[2 * n + q];
        qm[t] = mass[q];
        ux[t] = lam[q]; uy[t] = lam[n + q]; uz[t] = lam[2 * n + q];
        ox[t] = 0.0; oy[t] = 0.0; oz[t] = 0.0; og[t] = 0.0;
    }
    const int64_t tend = tb0 + (int64_t)NT * T;
    int64_t j = jbeg;
    for (; j + kVG <= jend; j += kVG) {   // whole groups: contiguous scalar loads
        double xs[kVG], ys[kVG], zs[kVG], ms[kVG], uxs[kVG], uys[kVG], uzs[kVG];
#pragma unroll
        for (int u = 0; u < kVG; ++u) {
            xs[u] = pos[j + u]; ys[u] = pos[n + j + u]; zs[u] = pos[2 * n + j + u];
            ms[u] = mass[j + u];
            uxs[u] = lam[j + u]; uys[u] = lam[n + j + u]; uzs[u] = lam[2 * n + j + u];
        }
        if ((j < tend) && (tb0 < j + kVG)) {
#pragma unroll
            for (int u = 0; u < kVG; ++u)
                vjp_pair<T, true>(xs[u], ys[u], zs[u], ms[u], uxs[u], uys[u], uzs[u], j + u, qx,
                                  qy, qz, qm, ux, uy, uz, qid, ox, oy, oz, og);
        } else {
#pragma unroll
            for (int u = 0; u < kVG; ++u)
                vjp_pair<T, false>(xs[u], ys[u], zs[u], ms[u], uxs[u], uys[u], uzs[u], j + u, qx,
                                   qy, qz, qm, ux, uy, uz, qid, ox, oy, oz, og);
        }
    }
    for (; j < jend; ++j)   // the chunk's ragged end
        vjp_pair<T, true>(pos[j], pos[n + j], pos[2 * n + j], mass[j], lam[j], lam[n + j],
                          lam[2 * n + j], j, qx, qy, qz, qm, ux, uy, uz, qid, ox, oy, oz, og);
    double* pc = part + c * 4 * n;
    const double gc = G * cu;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t p = tb0 + (int64_t)t * NT + tid;
        if (p < n) {
            __builtin_nontemporal_store(gc * ox[t], &pc[p]);
            __builtin_nontemporal_store(gc * oy[t], &pc[n + p]);
            __builtin_nontemporal_store(gc * oz[t], &pc[2 * n + p]);
            __builtin_nontemporal_store(-gc * og[t], &pc[3 * n + p]);
        }
    }
}

constexpr int kBlock = 256;

// lam_r += sum of the chunk partials of planes 0..2, g_m += plane 3; then,
// when `drift` is set, the adjoint of the drift that precedes this force pass
// in the reverse sweep: lam_v += dt lam_r.  GS threads per (plane, body)
// element sum the partials in a fixed order (chunk_sum: deterministic); the
// values the update reads are loaded before the partials.
template <int GS>
__global__ __launch_bounds__(kBlock) void k_vjp_reduce(const double* __restrict__ part,
                                                       int chunks, int64_t n,
                                                       double* __restrict__ lam_r,
                                                       double* __restrict__ g_m,
                                                       double* __restrict__ lam_v, double dt,
                                                       int drift)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = t / GS;   // k * n + q, k = 0..3
    const int sub = (int)(t % GS);
    const bool live = i < 4 * n;
    const int64_t ii = live ? i : 0;
    const bool head = live && sub == 0;
    const bool plane_r = i < 3 * n;
    double r0 = 0.0, v0 = 0.0, m0 = 0.0;
    if (head) {
        if (plane_r) {
            r0 = lam_r[i];
            if (drift) v0 = lam_v[i];
        } else {
            m0 = g_m[i - 3 * n];
        }
    }
    const double a = chunk_sum<GS>(part, chunks, 4 * n, ii, sub, live);
    if (!head) return;
    if (plane_r) {
        const double r = r0 + a;
        lam_r[i] = r;
        if (drift) lam_v[i] = __builtin_fma(dt, r, v0);
    } else {
        g_m[i - 3 * n] = m0 + a;
    }
}

__global__ __launch_bounds__(kBlock) void k_scale(const double* __restrict__ x, double c,
                                                  int64_t m, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) y[i] = c * x[i];
}

__global__ __launch_bounds__(kBlock) void k_axpy(const double* __restrict__ x, double c,
                                                 int64_t m, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) y[i] = __builtin_fma(c, x[i], y[i]);
}

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ y, double v, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) y[i] = v;
}

}  // namespace

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int T, int W>
static hipError_t vjp_tw(const double* pos, const double* mass, const double* lam, double cu,
                         int64_t n, int64_t L, int chunks, double G, double* part, hipStream_t s)
{
    constexpr int NT = 64 * W;
    const dim3 grid((unsigned)((n + (int64_t)NT * T - 1) / ((int64_t)NT * T)), (unsigned)chunks);
    hipLaunchKernelGGL((k_vjp<T, W>), grid, dim3(NT), 0, s, pos, mass, lam, cu, n, L, G, part);
    return hipGetLastError();
}

template <int T, int W>
static hipError_t vjp_s_tw(const double* pos, const double* mass, const double* lam, double cu,
                           int64_t n, int64_t L, int chunks, double G, double* part, hipStream_t s)
{
    constexpr int NT = 64 * W;
    const dim3 grid((unsigned)((n + (int64_t)NT * T - 1) / ((int64_t)NT * T)), (unsigned)chunks);
    hipLaunchKernelGGL((k_vjp_s<T, W>), grid, dim3(NT), 0, s, pos, mass, lam, cu, n, L, G, part);
    return hipGetLastError();
}

static constexpr int64_t kVjpGranule = 8;

int64_t vjp_chunk_length(int64_t n, const Tile& t)
{
    const int64_t per = (n + t.chunks - 1) / t.chunks;
    return (per + kVjpGranule - 1) / kVjpGranule * kVjpGranule;
}

int vjp_chunks(int64_t n, const Tile& t)
{
    if (t.variant == 5) return mutual_slots(n, t.tpl, t.waves);   // each pair once
    const int64_t L = vjp_chunk_length(n, t);
    return (int)((n + L - 1) / L);
}

hipError_t launch_vjp(const Tile& tile, const double* pos, const double* mass, const double* lam,
                      double cu, int64_t n, double G, double* part, hipStream_t s)
{
    if (tile.variant == 5)
        return launch_vjp_mutual(tile.tpl, tile.waves, pos, mass, lam, cu, n, G, part, s);
    if (tile.variant != 0 && tile.variant != 1) return hipErrorInvalidValue;
    const int64_t L = vjp_chunk_length(n, tile);
    const int chunks = vjp_chunks(n, tile);
#define NB_CASE(TT, WW)                                                                 \
    if (tile.tpl == TT && tile.waves == WW)                                             \
        return tile.variant == 1 ? vjp_s_tw<TT, WW>(pos, mass, lam, cu, n, L, chunks, G, part, s) \
                                 : vjp_tw<TT, WW>(pos, mass, lam, cu, n, L, chunks, G, part, s);
    NB_CASE(1, 1) NB_CASE(1, 2) NB_CASE(1, 4) NB_CASE(2, 1) NB_CASE(2, 2) NB_CASE(2, 4)
#undef NB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_vjp_reduce(const double* part, int chunks, int64_t n, double* lam_r,
                             double* g_m, double* lam_v, double dt, bool drift, hipStream_t s)
{
    if (chunks >= 16)
        hipLaunchKernelGGL(k_vjp_reduce<4>, dim3(blocks_for(16 * n, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, lam_r, g_m, lam_v, dt, drift ? 1 : 0);
    else
        hipLaunchKernelGGL(k_vjp_reduce<1>, dim3(blocks_for(4 * n, kBlock)), dim3(kBlock), 0, s,
                           part, chunks, n, lam_r, g_m, lam_v, dt, drift ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_scale(const double* x, double c, int64_t m, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, s, x, c, m, y);
    return hipGetLastError();
}

hipError_t launch_axpy(const double* x, double c, int64_t m, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, s, x, c, m, y);
    return hipGetLastError();
}

hipError_t launch_fill(double* y, double v, int64_t m, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, s, y, v, m);
    return hipGetLastError();
}

}  // namespace nb
