/*
 * Plain FP64 CPU oracle for the direct-sum N-body method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or constant with the HIP
 * library and is written to be checked against the paper by eye, not to be
 * fast.
 *
 * What it follows:
 *   accel      Eq. (1): a_p = sum_{j != p} G m_j (r_j - r_p) / |r_j - r_p|^3,
 *              terms in ascending j, compensated accumulation (accel_targets:
 *              the same sum for a list of targets).
 *   verlet     Eqs. (3)-(4), velocity Verlet, taken literally, one force
 *              evaluation per step (a_{i+1} is kept as the next a_i).
 *   energy     Sec. 2: total energy (kinetic + pair potential) is the accuracy
 *              measure of a run.
 *   momenta    total linear and angular momentum (invariants of Eq. (1)).
 *   euler      the first-order scheme Sec. 2 rejects (negative control only).
 *   rk4        the classical fourth-order Runge-Kutta method Sec. 2 names as
 *              the alternative to velocity Verlet.
 *   vjp        the transpose of the Jacobian of Eq. (1) applied to a
 *              cotangent, from the Jacobian blocks written out one by one.
 *   adjoint    reverse-mode chain rule through the literal Eqs. (3)-(4) map.
 *   tangent    forward-mode derivative of the literal Eqs. (3)-(4) map, by
 *              dual numbers carried through every arithmetic operation.
 *
 * Every function is pinned by the CPU tests to something other than itself
 * (closed forms, invariants, extended precision, worked examples, finite
 * differences, other derivations); none is left unpinned.
 *
 * Layout: structure of arrays, pos[0..n) = x, pos[n..2n) = y, pos[2n..3n) = z,
 * likewise vel, acc and the cotangents; mass[0..n).  All double precision.
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* threads                                                                   */
/* ------------------------------------------------------------------------ */

void oracle_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated summation                                            */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } csum;

static void cs_add(csum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double cs_val(const csum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Eq. (1)                                                                   */
/* ------------------------------------------------------------------------ */

/* One target of Eq. (1): sum over j != p, in ascending j, of the terms
 * G m_j d / (r2 * sqrt(r2)), d = r_j - r_p, each term in plain FP64.  The
 * sum is the exact sum of Eq. (1), accumulated with Neumaier compensation so
 * that its rounding error stays at a few ulp of sum |term| whatever the
 * number of bodies: a plain running sum drifts by up to ~1e-13 relative when
 * one close parent dominates 10^4 tiny asteroid terms.  No softening:
 * coincident distinct bodies give non-finite values. */
static void accel_one(int64_t n, double G, const double* x, const double* y, const double* z,
                      const double* mass, int64_t p, double* out)
{
    csum ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == p) continue;
        double dx = x[j] - x[p];
        double dy = y[j] - y[p];
        double dz = z[j] - z[p];
        double r2 = dx * dx + dy * dy + dz * dz;
        double r = sqrt(r2);
        double s = G * mass[j] / (r2 * r);
        cs_add(&ax, s * dx);
        cs_add(&ay, s * dy);
        cs_add(&az, s * dz);
    }
    out[0] = cs_val(&ax);
    out[1] = cs_val(&ay);
    out[2] = cs_val(&az);
}

/* Eq. (1) for all bodies.  Each target's sum is serial, so the result does
 * not depend on the thread count. */
void oracle_accel(int64_t n, double G, const double* pos, const double* mass, double* acc)
{
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n; ++p) {
        double a[3];
        accel_one(n, G, pos, pos + n, pos + 2 * n, mass, p, a);
        acc[p] = a[0];
        acc[n + p] = a[1];
        acc[2 * n + p] = a[2];
    }
}

/* Eq. (1) for the listed targets only: acc[3*k + c] for target idx[k],
 * component c (for sampled checks at large n). */
void oracle_accel_targets(int64_t n, double G, const double* pos, const double* mass,
                          const int64_t* idx, int64_t count, double* acc)
{
    int64_t k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < count; ++k)
        accel_one(n, G, pos, pos + n, pos + 2 * n, mass, idx[k], acc + 3 * k);
}

/* ------------------------------------------------------------------------ */
/* Eqs. (3)-(4)                                                               */
/* ------------------------------------------------------------------------ */

/* Velocity Verlet, literally:
 *   r_{i+1} = r_i + v_i dt + (1/2) a_i dt^2
 *   v_{i+1} = v_i + (1/2) (a_i + a_{i+1}) dt,   a_{i+1} = A(r_{i+1}).
 * pos and vel are updated in place.  If traj is not NULL it receives r_0 ..
 * r_steps ((steps+1) * 3n doubles).  Returns 0, or -1 on allocation failure. */
int oracle_verlet(int64_t n, double G, double dt, int64_t steps,
                  double* pos, double* vel, const double* mass, double* traj)
{
    int64_t m = 3 * n;
    double* a0 = (double*)malloc(sizeof(double) * m);
    double* a1 = (double*)malloc(sizeof(double) * m);
    if (!a0 || !a1) { free(a0); free(a1); return -1; }
    oracle_accel(n, G, pos, mass, a0);
    if (traj) memcpy(traj, pos, sizeof(double) * m);
    for (int64_t i = 0; i < steps; ++i) {
        for (int64_t k = 0; k < m; ++k)
            pos[k] = pos[k] + vel[k] * dt + 0.5 * a0[k] * dt * dt;
        oracle_accel(n, G, pos, mass, a1);
        for (int64_t k = 0; k < m; ++k)
            vel[k] = vel[k] + 0.5 * (a0[k] + a1[k]) * dt;
        double* t = a0; a0 = a1; a1 = t;
        if (traj) memcpy(traj + (i + 1) * m, pos, sizeof(double) * m);
    }
    free(a0);
    free(a1);
    return 0;
}

/* Explicit Euler, the first-order scheme the paper rejects in Sec. 2:
 * r_{i+1} = r_i + v_i dt,  v_{i+1} = v_i + a_i dt.  Negative control only. */
int oracle_euler(int64_t n, double G, double dt, int64_t steps,
                 double* pos, double* vel, const double* mass)
{
    int64_t m = 3 * n;
    double* a = (double*)malloc(sizeof(double) * m);
    if (!a) return -1;
    for (int64_t i = 0; i < steps; ++i) {
        oracle_accel(n, G, pos, mass, a);
        for (int64_t k = 0; k < m; ++k) {
            pos[k] = pos[k] + vel[k] * dt;
            vel[k] = vel[k] + a[k] * dt;
        }
    }
    free(a);
    return 0;
}

/* The classical fourth-order Runge-Kutta method, the higher-order
 * alternative Sec. 2 names, applied to the first-order system r' = v,
 * v' = A(r):
 *   k1 = (v,            A(r))
 *   k2 = (v + dt/2 kv1, A(r + dt/2 kr1))
 *   k3 = (v + dt/2 kv2, A(r + dt/2 kr2))
 *   k4 = (v + dt kv3,   A(r + dt kr3))
 *   (r, v) += dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * Four force evaluations per step. */
int oracle_rk4(int64_t n, double G, double dt, int64_t steps,
               double* pos, double* vel, const double* mass)
{
    int64_t m = 3 * n;
    double* buf = (double*)malloc(sizeof(double) * m * 10);
    if (!buf) return -1;
    double *kr1 = buf, *kv1 = buf + m, *kr2 = buf + 2 * m, *kv2 = buf + 3 * m;
    double *kr3 = buf + 4 * m, *kv3 = buf + 5 * m, *kr4 = buf + 6 * m, *kv4 = buf + 7 * m;
    double *rs = buf + 8 * m;   /* the stage position */
    for (int64_t i = 0; i < steps; ++i) {
        for (int64_t k = 0; k < m; ++k) kr1[k] = vel[k];
        oracle_accel(n, G, pos, mass, kv1);
        for (int64_t k = 0; k < m; ++k) {
            kr2[k] = vel[k] + 0.5 * dt * kv1[k];
            rs[k] = pos[k] + 0.5 * dt * kr1[k];
        }
        oracle_accel(n, G, rs, mass, kv2);
        for (int64_t k = 0; k < m; ++k) {
            kr3[k] = vel[k] + 0.5 * dt * kv2[k];
            rs[k] = pos[k] + 0.5 * dt * kr2[k];
        }
        oracle_accel(n, G, rs, mass, kv3);
        for (int64_t k = 0; k < m; ++k) {
            kr4[k] = vel[k] + dt * kv3[k];
            rs[k] = pos[k] + dt * kr3[k];
        }
        oracle_accel(n, G, rs, mass, kv4);
        for (int64_t k = 0; k < m; ++k) {
            pos[k] = pos[k] + dt / 6.0 * (kr1[k] + 2.0 * kr2[k] + 2.0 * kr3[k] + kr4[k]);
            vel[k] = vel[k] + dt / 6.0 * (kv1[k] + 2.0 * kv2[k] + 2.0 * kv3[k] + kv4[k]);
        }
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                                */
/* ------------------------------------------------------------------------ */

/* out[0] = kinetic sum_i m_i |v_i|^2 / 2, out[1] = potential
 * -sum_{i<j} G m_i m_j / |r_i - r_j|, out[2] = their sum.  Every sum is
 * Neumaier-compensated; rows are summed in ascending order. */
void oracle_energy(int64_t n, double G, const double* pos, const double* vel,
                   const double* mass, double* out)
{
    const double* x = pos;
    const double* y = pos + n;
    const double* z = pos + 2 * n;
    double* row = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        csum r = {0.0, 0.0};
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = x[j] - x[i];
            double dy = y[j] - y[i];
            double dz = z[j] - z[i];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            cs_add(&r, -G * mass[i] * mass[j] / d);
        }
        row[i] = cs_val(&r);
    }
    csum pot = {0.0, 0.0}, kin = {0.0, 0.0};
    for (i = 0; i < n; ++i) {
        cs_add(&pot, row[i]);
        double v2 = vel[i] * vel[i] + vel[n + i] * vel[n + i] + vel[2 * n + i] * vel[2 * n + i];
        cs_add(&kin, 0.5 * mass[i] * v2);
    }
    free(row);
    out[0] = cs_val(&kin);
    out[1] = cs_val(&pot);
    csum tot = {0.0, 0.0};
    cs_add(&tot, out[0]);
    cs_add(&tot, out[1]);
    out[2] = cs_val(&tot);
}

/* P = sum m v, L = sum m r x v (compensated). */
void oracle_momenta(int64_t n, const double* pos, const double* vel, const double* mass,
                    double* P, double* L)
{
    csum p[3] = {{0, 0}, {0, 0}, {0, 0}}, l[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t i = 0; i < n; ++i) {
        double rx = pos[i], ry = pos[n + i], rz = pos[2 * n + i];
        double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        double m = mass[i];
        cs_add(&p[0], m * vx);
        cs_add(&p[1], m * vy);
        cs_add(&p[2], m * vz);
        cs_add(&l[0], m * (ry * vz - rz * vy));
        cs_add(&l[1], m * (rz * vx - rx * vz));
        cs_add(&l[2], m * (rx * vy - ry * vx));
    }
    for (int k = 0; k < 3; ++k) { P[k] = cs_val(&p[k]); L[k] = cs_val(&l[k]); }
}

/* ------------------------------------------------------------------------ */
/* Transpose of the Jacobian of Eq. (1)                                       */
/* ------------------------------------------------------------------------ */

/* Tidal block K(d) = I/|d|^3 - 3 d d^T/|d|^5, written into k[9] (row major). */
static void tidal(double dx, double dy, double dz, double* k)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    double r = sqrt(r2);
    double i3 = 1.0 / (r2 * r);
    double i5 = i3 / r2;
    double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            k[3 * a + b] = (a == b ? i3 : 0.0) - 3.0 * d[a] * d[b] * i5;
}

/* For a cotangent u on the accelerations:
 *   out_r[q] = sum_p (d a_p / d r_q)^T u_p,  out_m[q] = sum_p u_p . d a_p / d m_q,
 * with the Jacobian blocks of Eq. (1):
 *   d a_p / d r_q = G m_q K(r_q - r_p)               (q != p)
 *   d a_p / d r_p = -sum_{j != p} G m_j K(r_j - r_p)
 *   d a_p / d m_q = G (r_q - r_p) / |r_q - r_p|^3     (q != p), 0 for q = p.
 * K is symmetric, so (d a_p / d r_q)^T = d a_p / d r_q. */
void oracle_vjp(int64_t n, double G, const double* pos, const double* mass,
                const double* u, double* out_r, double* out_m)
{
    const double* x = pos;
    const double* y = pos + n;
    const double* z = pos + 2 * n;
    int64_t q;
#pragma omp parallel for schedule(static)
    for (q = 0; q < n; ++q) {
        double k[9];
        double o[3] = {0.0, 0.0, 0.0};
        double gm = 0.0;
        /* off-diagonal blocks: p != q contributes (G m_q K(r_q - r_p)) u_p */
        for (int64_t p = 0; p < n; ++p) {
            if (p == q) continue;
            double dx = x[q] - x[p], dy = y[q] - y[p], dz = z[q] - z[p];
            tidal(dx, dy, dz, k);
            double up[3] = {u[p], u[n + p], u[2 * n + p]};
            for (int a = 0; a < 3; ++a)
                o[a] += G * mass[q] * (k[3 * a + 0] * up[0] + k[3 * a + 1] * up[1] + k[3 * a + 2] * up[2]);
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            gm += G * (up[0] * dx + up[1] * dy + up[2] * dz) / (r2 * r);
        }
        /* diagonal block: -(sum_j G m_j K(r_j - r_q)) u_q */
        double uq[3] = {u[q], u[n + q], u[2 * n + q]};
        for (int64_t j = 0; j < n; ++j) {
            if (j == q) continue;
            tidal(x[j] - x[q], y[j] - y[q], z[j] - z[q], k);
            for (int a = 0; a < 3; ++a)
                o[a] -= G * mass[j] * (k[3 * a + 0] * uq[0] + k[3 * a + 1] * uq[1] + k[3 * a + 2] * uq[2]);
        }
        out_r[q] = o[0];
        out_r[n + q] = o[1];
        out_r[2 * n + q] = o[2];
        out_m[q] = gm;
    }
}

/* ------------------------------------------------------------------------ */
/* Reverse mode through Eqs. (3)-(4)                                          */
/* ------------------------------------------------------------------------ */

/* Gradient of a scalar L(r_n, v_n) with respect to (r_0, v_0, m) for the
 * literal Eqs. (3)-(4) map of oracle_verlet.  Inputs lam_r = dL/dr_n,
 * lam_v = dL/dv_n.  The forward trajectory r_0..r_n is stored whole.
 *
 * Forward step i:  r_{i+1} = r_i + dt v_i + dt^2/2 a_i
 *                  a_{i+1} = A(r_{i+1}; m)
 *                  v_{i+1} = v_i + dt/2 (a_i + a_{i+1}),   a_0 = A(r_0; m).
 * Reverse step i (bar = adjoint), given rb = bar r_{i+1}, vb = bar v_{i+1},
 * ab = bar a_{i+1} (the part already collected from step i+1):
 *   ab  += dt/2 vb                      (a_{i+1} in v_{i+1})
 *   rb  += J(r_{i+1})^T ab,  mb += M(r_{i+1})^T ab   (a_{i+1} = A(r_{i+1}))
 *   bar a_i  = dt/2 vb + dt^2/2 rb      (a_i in v_{i+1} and r_{i+1})
 *   bar v_i  = vb + dt rb,  bar r_i = rb
 * and finally bar r_0 += J(r_0)^T bar a_0, mb += M(r_0)^T bar a_0. */
int oracle_adjoint(int64_t n, double G, double dt, int64_t steps,
                   const double* pos0, const double* vel0, const double* mass,
                   const double* lam_r, const double* lam_v,
                   double* g_r0, double* g_v0, double* g_m)
{
    int64_t m = 3 * n;
    size_t tsz = sizeof(double) * (size_t)m * (size_t)(steps + 1);
    double* traj = (double*)malloc(tsz);
    double* p = (double*)malloc(sizeof(double) * m);
    double* v = (double*)malloc(sizeof(double) * m);
    double* rb = (double*)malloc(sizeof(double) * m);
    double* vb = (double*)malloc(sizeof(double) * m);
    double* ab = (double*)malloc(sizeof(double) * m);
    double* jr = (double*)malloc(sizeof(double) * m);
    double* jm = (double*)malloc(sizeof(double) * (size_t)n);
    if (!traj || !p || !v || !rb || !vb || !ab || !jr || !jm) {
        free(traj); free(p); free(v); free(rb); free(vb); free(ab); free(jr); free(jm);
        return -1;
    }
    memcpy(p, pos0, sizeof(double) * m);
    memcpy(v, vel0, sizeof(double) * m);
    oracle_verlet(n, G, dt, steps, p, v, mass, traj);

    memcpy(rb, lam_r, sizeof(double) * m);
    memcpy(vb, lam_v, sizeof(double) * m);
    memset(ab, 0, sizeof(double) * m);
    for (int64_t q = 0; q < n; ++q) g_m[q] = 0.0;

    for (int64_t i = steps - 1; i >= 0; --i) {
        const double* r1 = traj + (i + 1) * m;
        for (int64_t k = 0; k < m; ++k) ab[k] += 0.5 * dt * vb[k];
        oracle_vjp(n, G, r1, mass, ab, jr, jm);
        for (int64_t k = 0; k < m; ++k) rb[k] += jr[k];
        for (int64_t q = 0; q < n; ++q) g_m[q] += jm[q];
        for (int64_t k = 0; k < m; ++k) {
            double a_i = 0.5 * dt * vb[k] + 0.5 * dt * dt * rb[k];
            vb[k] = vb[k] + dt * rb[k];
            ab[k] = a_i;
        }
    }
    oracle_vjp(n, G, traj, mass, ab, jr, jm);
    for (int64_t k = 0; k < m; ++k) g_r0[k] = rb[k] + jr[k];
    for (int64_t k = 0; k < m; ++k) g_v0[k] = vb[k];
    for (int64_t q = 0; q < n; ++q) g_m[q] += jm[q];

    free(traj); free(p); free(v); free(rb); free(vb); free(ab); free(jr); free(jm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward mode through Eqs. (3)-(4) by dual numbers                          */
/* ------------------------------------------------------------------------ */

typedef struct { double v, d; } dual;

static dual d_add(dual a, dual b) { dual r = {a.v + b.v, a.d + b.d}; return r; }
static dual d_sub(dual a, dual b) { dual r = {a.v - b.v, a.d - b.d}; return r; }
static dual d_mul(dual a, dual b) { dual r = {a.v * b.v, a.d * b.v + a.v * b.d}; return r; }
static dual d_div(dual a, dual b)
{
    dual r = {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
    return r;
}
static dual d_sqrt(dual a)
{
    double s = sqrt(a.v);
    dual r = {s, a.d / (2.0 * s)};
    return r;
}
static dual d_const(double c) { dual r = {c, 0.0}; return r; }

static void dual_accel(int64_t n, dual G, const dual* pos, const dual* mass, dual* acc)
{
    const dual* x = pos;
    const dual* y = pos + n;
    const dual* z = pos + 2 * n;
    int64_t p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < n; ++p) {
        dual ax = d_const(0), ay = d_const(0), az = d_const(0);
        for (int64_t j = 0; j < n; ++j) {
            if (j == p) continue;
            dual dx = d_sub(x[j], x[p]);
            dual dy = d_sub(y[j], y[p]);
            dual dz = d_sub(z[j], z[p]);
            dual r2 = d_add(d_add(d_mul(dx, dx), d_mul(dy, dy)), d_mul(dz, dz));
            dual r = d_sqrt(r2);
            dual s = d_div(d_mul(G, mass[j]), d_mul(r2, r));
            ax = d_add(ax, d_mul(s, dx));
            ay = d_add(ay, d_mul(s, dy));
            az = d_add(az, d_mul(s, dz));
        }
        acc[p] = ax;
        acc[n + p] = ay;
        acc[2 * n + p] = az;
    }
}

/* Carries (value, directional derivative) pairs through the literal
 * Eqs. (3)-(4) loop.  Inputs: r_0, v_0, m and a direction (dr_0, dv_0, dm).
 * Outputs: r_n, v_n and their directional derivatives. */
int oracle_tangent(int64_t n, double G, double dt, int64_t steps,
                   const double* pos0, const double* vel0, const double* mass,
                   const double* dpos0, const double* dvel0, const double* dmass,
                   double* pos_out, double* vel_out, double* dpos_out, double* dvel_out)
{
    int64_t m = 3 * n;
    dual* p = (dual*)malloc(sizeof(dual) * m);
    dual* v = (dual*)malloc(sizeof(dual) * m);
    dual* ms = (dual*)malloc(sizeof(dual) * (size_t)n);
    dual* a0 = (dual*)malloc(sizeof(dual) * m);
    dual* a1 = (dual*)malloc(sizeof(dual) * m);
    if (!p || !v || !ms || !a0 || !a1) {
        free(p); free(v); free(ms); free(a0); free(a1);
        return -1;
    }
    for (int64_t k = 0; k < m; ++k) {
        p[k].v = pos0[k]; p[k].d = dpos0[k];
        v[k].v = vel0[k]; v[k].d = dvel0[k];
    }
    for (int64_t q = 0; q < n; ++q) { ms[q].v = mass[q]; ms[q].d = dmass[q]; }
    dual Gd = d_const(G), h = d_const(dt), half = d_const(0.5);
    dual hh = d_mul(half, d_mul(h, h));
    dual hhalf = d_mul(half, h);
    dual_accel(n, Gd, p, ms, a0);
    for (int64_t i = 0; i < steps; ++i) {
        for (int64_t k = 0; k < m; ++k)
            p[k] = d_add(d_add(p[k], d_mul(v[k], h)), d_mul(a0[k], hh));
        dual_accel(n, Gd, p, ms, a1);
        for (int64_t k = 0; k < m; ++k)
            v[k] = d_add(v[k], d_mul(hhalf, d_add(a0[k], a1[k])));
        dual* t = a0; a0 = a1; a1 = t;
    }
    for (int64_t k = 0; k < m; ++k) {
        pos_out[k] = p[k].v; dpos_out[k] = p[k].d;
        vel_out[k] = v[k].v; dvel_out[k] = v[k].d;
    }
    free(p); free(v); free(ms); free(a0); free(a1);
    return 0;
}
