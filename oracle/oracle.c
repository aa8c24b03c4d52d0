/*
 * FP64 CPU oracle for the Hermite block-step direct N-body method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product library never links, loads or calls it, and it shares no source
 * with the HIP path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FMA contraction, so every product and sum rounds as written).
 *
 * Conventions (Portegies Zwart et al., "A parallel gravitational N-body
 * kernel", Sect. 2.1):
 *   G = 1, N-body units.  Arrays are structure-of-arrays: x[0*n + i] is the
 *   x component of particle i, x[1*n + i] the y component, x[2*n + i] the z
 *   component.  Outputs for an active list are laid out the same way with
 *   n_act in place of n.
 *
 * Readings of the paper used here (each one also listed in the design notes):
 *   - Eq. (Force) prints r_i - r_j, which would be repulsive; gravity is
 *     attractive, so the pair vector is r_ij = x_j - x_i.
 *   - Plummer softening: R^2 = |r_ij|^2 + eps^2, used in a, k and phi alike.
 *   - The jerk k = da/dt is not printed; it is the exact time derivative of
 *     the softened acceleration along the predicted motion.
 *   - The potential is not in the paper; phi_i = -sum_{j != i} m_j / R.
 *   - Aarseth's criterion (Eq. timestep) is evaluated with the end-of-step
 *     quantities |a_1|, |a2_1| (a2_1 = a2 + a3 dt), |k_1|, |a3|.
 *   - Time steps are powers of two: the criterion is rounded down to a
 *     power of two; a step may shrink at any time, may at most double, and
 *     only doubles when the current time is a multiple of the doubled step;
 *     steps are capped at dt_max and an error is raised below dt_min.
 *   - Initial steps: eta_s |a| / |k| rounded down to a power of two.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_DTMIN (-5)
#define ORACLE_E_NONFINITE (-6)
#define ORACLE_E_INVAL (-1)

/* Threads the OpenMP loops of this library use. */
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

/* ---------------------------------------------------------------------- */
/* Pairwise sums (Sect. 2.1, Eq. Force; jerk and potential as read above). */

/* Acceleration, jerk and potential on particle i from every j != i in
 * [j_begin, j_end), j ascending, plain FP64. */
static void pair_sum(int64_t n, const double *m, const double *x, const double *v,
                     double eps2, int64_t i, int64_t j_begin, int64_t j_end,
                     double acc[3], double jerk[3], double *pot) {
    const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
    const double vxi = v[i], vyi = v[n + i], vzi = v[2 * n + i];
    double ax = 0.0, ay = 0.0, az = 0.0;
    double kx = 0.0, ky = 0.0, kz = 0.0;
    double ph = 0.0;
    for (int64_t j = j_begin; j < j_end; ++j) {
        if (j == i) continue;
        const double dx = x[j] - xi, dy = x[n + j] - yi, dz = x[2 * n + j] - zi;
        const double dvx = v[j] - vxi, dvy = v[n + j] - vyi, dvz = v[2 * n + j] - vzi;
        const double r2 = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(r2);
        const double rinv2 = rinv * rinv;
        const double mr3 = m[j] * rinv * rinv2;          /* m_j / R^3            */
        const double rv = dx * dvx + dy * dvy + dz * dvz; /* r_ij . v_ij          */
        const double c = 3.0 * rv * rinv2;                /* 3 (r.v) / R^2        */
        ax += mr3 * dx;
        ay += mr3 * dy;
        az += mr3 * dz;
        kx += mr3 * (dvx - c * dx);
        ky += mr3 * (dvy - c * dy);
        kz += mr3 * (dvz - c * dz);
        ph -= m[j] * rinv;
    }
    acc[0] = ax; acc[1] = ay; acc[2] = az;
    jerk[0] = kx; jerk[1] = ky; jerk[2] = kz;
    *pot = ph;
}

/* a, k, phi on the active particles act[0..n_act) from all n particles.
 * acc, jerk: [3][n_act]; pot: [n_act] or NULL.  OpenMP over active i only:
 * each i's sum runs j-ascending in one thread, so results do not depend on
 * the thread count. */
void oracle_force(int64_t n, const double *m, const double *x, const double *v, double eps,
                  int64_t n_act, const int32_t *act, double *acc, double *jerk, double *pot) {
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_act; ++q) {
        double a[3], k[3], p;
        pair_sum(n, m, x, v, eps2, (int64_t)act[q], 0, n, a, k, &p);
        for (int d = 0; d < 3; ++d) {
            acc[d * n_act + q] = a[d];
            jerk[d * n_act + q] = k[d];
        }
        if (pot) pot[q] = p;
    }
}

/* The paper's j-parallel partition (Sect. 3, Flowchart) emulated on one CPU:
 * the j range is cut into p contiguous slices of ceil(n/p); each slice gives a
 * partial sum, and the partials are added in slice order. */
void oracle_force_sliced(int64_t n, const double *m, const double *x, const double *v,
                         double eps, int64_t p, int64_t n_act, const int32_t *act,
                         double *acc, double *jerk, double *pot) {
    const double eps2 = eps * eps;
    const int64_t w = (n + p - 1) / p;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_act; ++q) {
        double at[3] = {0, 0, 0}, kt[3] = {0, 0, 0}, pt = 0.0;
        for (int64_t s = 0; s < p; ++s) {
            int64_t b = s * w, e = b + w;
            if (b > n) b = n;
            if (e > n) e = n;
            double a[3], k[3], ph;
            pair_sum(n, m, x, v, eps2, (int64_t)act[q], b, e, a, k, &ph);
            for (int d = 0; d < 3; ++d) { at[d] += a[d]; kt[d] += k[d]; }
            pt += ph;
        }
        for (int d = 0; d < 3; ++d) {
            acc[d * n_act + q] = at[d];
            jerk[d * n_act + q] = kt[d];
        }
        if (pot) pot[q] = pt;
    }
}

/* Sums of the absolute pair terms on each active particle, the scale that
 * rounding errors of any summation order are measured against:
 * out[0][q] = sum m_j |r_ij| / R^3 (acceleration), out[1][q] = sum of
 * |jerk term|, out[2][q] = sum m_j / R (potential).  out: [3][n_act]. */
void oracle_force_abs(int64_t n, const double *m, const double *x, const double *v, double eps,
                      int64_t n_act, const int32_t *act, double *out) {
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = act[q];
        double sa = 0.0, sk = 0.0, sp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            const double dvx = v[j] - v[i], dvy = v[n + j] - v[n + i], dvz = v[2 * n + j] - v[2 * n + i];
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            const double rinv = 1.0 / sqrt(r2);
            const double mr3 = m[j] * rinv * rinv * rinv;
            const double c = 3.0 * (dx * dvx + dy * dvy + dz * dvz) * rinv * rinv;
            const double wx = dvx - c * dx, wy = dvy - c * dy, wz = dvz - c * dz;
            sa += mr3 * sqrt(dx * dx + dy * dy + dz * dz);
            sk += mr3 * sqrt(wx * wx + wy * wy + wz * wz);
            sp += m[j] * rinv;
        }
        out[q] = sa;
        out[n_act + q] = sk;
        out[2 * n_act + q] = sp;
    }
}

/* ---------------------------------------------------------------------- */
/* Perturber lists (Sect. 3.1): for each star the stars whose force on it  */
/* exceeds a threshold, in the order a serial sweep over the particles    */
/* identifies them, at most cap of them (the paper's code keeps 256).     */

/* For active particle i = act[q]: every j != i with
 * m_j / (|x_j - x_i|^2 + eps^2) > thr, in ascending j, the first cap of them
 * in lists[q * cap ...] and -1 in the rest of the row; counts[q] = the
 * number of j that pass, also beyond cap.  R^2 is formed as
 * ((dx dx + dy dy) + dz dz) + eps^2, each operation rounded. */
void oracle_perturbers(int64_t n, const double *m, const double *x, double eps, double thr, int64_t n_act,
                       const int32_t *act, int32_t cap, int32_t *lists, int32_t *counts) {
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = act[q];
        int32_t found = 0;
        for (int32_t s = 0; s < cap; ++s) lists[q * cap + s] = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            if (m[j] / r2 > thr) {
                if (found < cap) lists[q * cap + found] = (int32_t)j;
                ++found;
            }
        }
        counts[q] = found;
    }
}

/* ---------------------------------------------------------------------- */
/* Hermite predictor (Sect. 2.1, predictor equations).                    */

void oracle_predict(int64_t n, const double *x, const double *v, const double *a,
                    const double *k, const double *t, double t_pred, double *xp, double *vp) {
    for (int64_t i = 0; i < n; ++i) {
        const double h = t_pred - t[i];
        for (int d = 0; d < 3; ++d) {
            const int64_t o = d * n + i;
            xp[o] = x[o] + v[o] * h + a[o] * h * h / 2.0 + k[o] * h * h * h / 6.0;
            vp[o] = v[o] + a[o] * h + k[o] * h * h / 2.0;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Hermite corrector (Sect. 2.1, corrector equations) for one particle.
 * a0, k0: values at the start of the step; a1, k1: recomputed at the
 * predicted time; Delta a = a0 - a1.  Outputs the corrected x, v and the
 * estimated second and third derivatives of the acceleration (a2, a3). */
void oracle_correct_one(double h, const double a0[3], const double k0[3], const double a1[3],
                        const double k1[3], const double xp[3], const double vp[3], double x[3],
                        double v[3], double a2[3], double a3[3]) {
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    for (int d = 0; d < 3; ++d) {
        const double da = a0[d] - a1[d];
        a2[d] = -6.0 * da / h2 - (4.0 * k0[d] + 2.0 * k1[d]) / h;
        a3[d] = 12.0 * da / h3 + 6.0 * (k0[d] + k1[d]) / h2;
        x[d] = xp[d] + a2[d] * h4 / 24.0 + a3[d] * h5 / 120.0;
        v[d] = vp[d] + a2[d] * h3 / 6.0 + a3[d] * h4 / 24.0;
    }
}

static double norm3(const double u[3]) { return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

/* Aarseth's criterion (Sect. 2.1, Eq. timestep) with the end-of-step values:
 * a1, k1 recomputed at the new time, a2 propagated to the new time
 * (a2 + a3 h), a3 constant over the step. */
double oracle_aarseth_dt(double eta, const double a1[3], const double k1[3], const double a2[3],
                         const double a3[3], double h) {
    double a2p[3];
    for (int d = 0; d < 3; ++d) a2p[d] = a2[d] + a3[d] * h;
    const double na = norm3(a1), nk = norm3(k1), na2 = norm3(a2p), na3 = norm3(a3);
    const double den = nk * na3 + na2 * na2;
    if (den == 0.0) return INFINITY; /* no higher derivatives: no limit */
    return sqrt(eta * (na * na2 + nk * nk) / den);
}

/* Largest power of two not above x (x > 0, finite), exactly. */
double oracle_pow2_floor(double x) {
    int e;
    (void)frexp(x, &e); /* x = f * 2^e, f in [0.5, 1) */
    return ldexp(1.0, e - 1);
}

/* Block-step quantisation of a new step (power of two, commensurate with the
 * current time t_now).  Returns the new step; sets *status to ORACLE_E_DTMIN
 * when the result falls below dt_min, ORACLE_E_NONFINITE for a NaN or
 * non-positive criterion. */
double oracle_quantize(double dt_raw, double dt_old, double t_now, double dt_max, double dt_min,
                       int *status) {
    if (isnan(dt_raw) || !isfinite(dt_old)) {
        *status = ORACLE_E_NONFINITE;
        return dt_old;
    }
    if (!(dt_raw > 0.0)) {
        *status = ORACLE_E_DTMIN;
        return dt_old;
    }
    /* an unbounded criterion (no force, no jerk) asks for the largest step */
    double dt_new = isinf(dt_raw) ? dt_max : oracle_pow2_floor(dt_raw);
    if (dt_new < dt_old) {
        /* shrink: t_now is a multiple of dt_old, hence of any smaller power of two */
    } else if (dt_new >= 2.0 * dt_old && fmod(t_now, 2.0 * dt_old) == 0.0) {
        dt_new = 2.0 * dt_old;
    } else {
        dt_new = dt_old;
    }
    if (dt_new > dt_max) dt_new = dt_max;
    if (dt_new < dt_min) *status = ORACLE_E_DTMIN;
    return dt_new;
}

/* Initial step at t = 0: eta_s |a| / |k| rounded down to a power of two and
 * capped at dt_max. */
double oracle_initial_dt(double eta_s, const double a[3], const double k[3], double dt_max,
                         double dt_min, int *status) {
    const double na = norm3(a), nk = norm3(k);
    double dt;
    if (nk == 0.0) {
        dt = dt_max;
    } else {
        const double raw = eta_s * na / nk;
        if (!(raw > 0.0) || !isfinite(raw)) {
            *status = (raw == 0.0) ? ORACLE_E_DTMIN : ORACLE_E_NONFINITE;
            return dt_min;
        }
        dt = oracle_pow2_floor(raw);
    }
    if (dt > dt_max) dt = dt_max;
    if (dt < dt_min) *status = ORACLE_E_DTMIN;
    return dt;
}

/* ---------------------------------------------------------------------- */
/* Block-step integrator (Sect. 2.1, the per-step item list).             */

/* Start: a, k of every particle from x, v; t_i = 0; dt_i from the initial
 * rule.  Returns ORACLE_OK or an error. */
int oracle_start(int64_t n, const double *m, const double *x, const double *v, double eps,
                 double eta_s, double dt_max, double dt_min, double *a, double *k, double *t,
                 double *dt) {
    int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!all) return ORACLE_E_INVAL;
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    oracle_force(n, m, x, v, eps, n, all, a, k, NULL);
    free(all);
    int status = ORACLE_OK;
    for (int64_t i = 0; i < n; ++i) {
        double ai[3] = {a[i], a[n + i], a[2 * n + i]};
        double ki[3] = {k[i], k[n + i], k[2 * n + i]};
        t[i] = 0.0;
        dt[i] = oracle_initial_dt(eta_s, ai, ki, dt_max, dt_min, &status);
    }
    return status;
}

/* Next block time and the block itself (ascending indices). */
int64_t oracle_select(int64_t n, const double *t, const double *dt, double *t_sys, int32_t *act) {
    double tmin = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        const double ti = t[i] + dt[i];
        if (ti < tmin) tmin = ti;
    }
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] == tmin) act[c++] = (int32_t)i;
    *t_sys = tmin;
    return c;
}

/* One block step.  work must hold 13*n doubles.  act (n ints) receives the
 * block.  Returns the block size, or a negative error code; *t_sys receives
 * the new block time. */
int64_t oracle_block_step(int64_t n, const double *m, double *x, double *v, double *a,
                          double *k, double *t, double *dt, double eps, double eta,
                          double dt_max, double dt_min, double *work, int32_t *act,
                          double *t_sys_out) {
    double t_sys;
    const int64_t nb = oracle_select(n, t, dt, &t_sys, act);
    double *xp = work, *vp = work + 3 * n;
    double *a1 = work + 6 * n, *k1 = a1 + 3 * nb;
    oracle_predict(n, x, v, a, k, t, t_sys, xp, vp);
    oracle_force(n, m, xp, vp, eps, nb, act, a1, k1, NULL);
    int status = ORACLE_OK;
    for (int64_t q = 0; q < nb; ++q) {
        const int64_t i = act[q];
        const double h = t_sys - t[i];
        double a0v[3], k0v[3], a1v[3], k1v[3], xpv[3], vpv[3], xn[3], vn[3], a2[3], a3[3];
        for (int d = 0; d < 3; ++d) {
            a0v[d] = a[d * n + i];
            k0v[d] = k[d * n + i];
            a1v[d] = a1[d * nb + q];
            k1v[d] = k1[d * nb + q];
            xpv[d] = xp[d * n + i];
            vpv[d] = vp[d * n + i];
        }
        oracle_correct_one(h, a0v, k0v, a1v, k1v, xpv, vpv, xn, vn, a2, a3);
        const double raw = oracle_aarseth_dt(eta, a1v, k1v, a2, a3, h);
        const double dtn = oracle_quantize(raw, dt[i], t_sys, dt_max, dt_min, &status);
        for (int d = 0; d < 3; ++d) {
            if (!isfinite(xn[d]) || !isfinite(vn[d])) status = ORACLE_E_NONFINITE;
            x[d * n + i] = xn[d];
            v[d * n + i] = vn[d];
            a[d * n + i] = a1v[d];
            k[d * n + i] = k1v[d];
        }
        t[i] = t_sys;
        dt[i] = dtn;
    }
    *t_sys_out = t_sys;
    return status == ORACLE_OK ? nb : (int64_t)status;
}

/* Advance block steps until the block time reaches t_end (which must be a
 * multiple of dt_max, so every particle is synchronised there) or max_steps
 * have been taken.  Returns the number of block steps, or a negative error;
 * *n_int receives the number of pairwise interactions (block size * n summed
 * over steps) and *t_reached the last block time. */
int64_t oracle_run(int64_t n, const double *m, double *x, double *v, double *a, double *k,
                   double *t, double *dt, double eps, double eta, double dt_max, double dt_min,
                   double t_end, int64_t max_steps, double *n_int, double *t_reached) {
    double *work = (double *)malloc(sizeof(double) * (size_t)(13 * n));
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!work || !act) {
        free(work);
        free(act);
        return ORACLE_E_INVAL;
    }
    int64_t steps = 0;
    double ni = 0.0, ts = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] > ts) ts = t[i];
    while (ts < t_end && steps < max_steps) {
        const int64_t nb = oracle_block_step(n, m, x, v, a, k, t, dt, eps, eta, dt_max, dt_min,
                                             work, act, &ts);
        if (nb < 0) {
            steps = nb;
            break;
        }
        ni += (double)nb * (double)n;
        ++steps;
    }
    free(work);
    free(act);
    *n_int = ni;
    *t_reached = ts;
    return steps;
}

/* ---------------------------------------------------------------------- */
/* Diagnostics: softened energy, linear and angular momentum.             */

void oracle_diagnostics(int64_t n, const double *m, const double *x, const double *v, double eps,
                        double out[8] /* KE, PE, Px, Py, Pz, Lx, Ly, Lz */) {
    const double eps2 = eps * eps;
    double ke = 0.0, pe = 0.0;
    double p[3] = {0, 0, 0}, l[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double xi[3] = {x[i], x[n + i], x[2 * n + i]};
        const double vi[3] = {v[i], v[n + i], v[2 * n + i]};
        ke += 0.5 * m[i] * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
        for (int d = 0; d < 3; ++d) p[d] += m[i] * vi[d];
        l[0] += m[i] * (xi[1] * vi[2] - xi[2] * vi[1]);
        l[1] += m[i] * (xi[2] * vi[0] - xi[0] * vi[2]);
        l[2] += m[i] * (xi[0] * vi[1] - xi[1] * vi[0]);
    }
    /* per-particle potentials in parallel, then summed in index order so
     * the result does not depend on the number of threads */
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            s -= m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        if (phi) phi[i] = s;
    }
    for (int64_t i = 0; i < n && phi; ++i) pe += 0.5 * m[i] * phi[i];
    free(phi);
    out[0] = ke;
    out[1] = pe;
    out[2] = p[0]; out[3] = p[1]; out[4] = p[2];
    out[5] = l[0]; out[6] = l[1]; out[7] = l[2];
}
