/*
 * CPU oracle: trajectories of one Paul-trapped ion plus one atom.
 * TEST INFRASTRUCTURE ONLY (see iat_oracle.h).  Plain FP64 C, libm, OpenMP over
 * trajectories.  Written for readability against the paper, not for speed.
 */
#include "iat_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NY 12

/* ---------------------------------------------------------------------------
 * Dormand-Prince 5(4) coefficients, as published by Dormand & Prince (1980),
 * J. Comput. Appl. Math. 6:19 (also Hairer, Norsett & Wanner, Solving ODEs I,
 * Table II.5.2).  This is the pair behind ode45, which the paper's integrator
 * follows (model paragraph after Eq. (1)).
 * ------------------------------------------------------------------------- */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
/* fifth-order weights (= last row of A, so the pair is FSAL) */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
/* embedded fourth-order weights */
static const double DP_BH[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

void orc_tableau(double A[49], double b[7], double bhat[7], double c[7])
{
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 7; ++j) A[i * 7 + j] = (j < 6) ? DP_A[i][j] : 0.0;
        b[i] = DP_B[i];
        bhat[i] = DP_BH[i];
        c[i] = DP_C[i];
    }
}

typedef void (*rhs_fn)(const void* ctx, double tau, const double* y, double* dy);

/*
 * One attempted Dormand-Prince step of size h from (tau, y) for an n-dimensional
 * system.  k is a 7*n array whose first row holds k1 = f(tau, y) on entry.
 * Stages: Y_s = y + h sum_{j<s} a_sj k_j,  k_s = f(tau + c_s h, Y_s).
 * y5 = y + h sum_j b_j k_j (fifth order).  If err != NULL the last stage
 * k7 = f(tau + h, y5) is evaluated (first same as last) and
 * err = h sum_j (b_j - bhat_j) k_j.
 */
static void dp5_attempt(int n, rhs_fn f, const void* ctx, double tau, const double* y, double h,
                        double* k, double* ytmp, double* y5, double* err)
{
    for (int s = 1; s < 6; ++s) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += DP_A[s][j] * k[j * n + i];
            ytmp[i] = y[i] + h * acc;
        }
        f(ctx, tau + DP_C[s] * h, ytmp, &k[s * n]);
    }
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += DP_B[j] * k[j * n + i];
        y5[i] = y[i] + h * acc;
    }
    if (err) {
        f(ctx, tau + DP_C[6] * h, y5, &k[6 * n]);
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 7; ++j) acc += (DP_B[j] - DP_BH[j]) * k[j * n + i];
            err[i] = h * acc;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Equations of motion from Eq. (1), in internal units: length a0, mass m_e,
 * time tau = Omega t.  Energies scale by 1/Omega^2, so C4' = C4/Omega^2 and
 * C8' = C8/Omega^2; the trap acceleration of the ion along axis k becomes
 * -(a_k + 2 q_k cos(tau + phase0)) r_{i,k} / 4.
 * ------------------------------------------------------------------------- */
typedef struct {
    double m_a, m_i, C4, C8;     /* internal units */
    double a[3], q[3], phase0;
} sys_int;

static void traj_rhs(const void* ctx, double tau, const double* y, double* dy)
{
    const sys_int* S = (const sys_int*)ctx;
    double d[3] = {y[0] - y[3], y[1] - y[4], y[2] - y[5]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r4 = r2 * r2, r6 = r4 * r2, r10 = r6 * r4;
    /* V = C8/r^8 - C4/r^4 ; force on the atom F = -(dV/dr) d/r = (8 C8/r^10 - 4 C4/r^6) d */
    double s = 8.0 * S->C8 / r10 - 4.0 * S->C4 / r6;
    double cs = cos(tau + S->phase0);
    for (int k = 0; k < 3; ++k) {
        double F = s * d[k];
        double kappa = (S->a[k] + 2.0 * S->q[k] * cs) / 4.0;
        dy[k] = y[6 + k];
        dy[3 + k] = y[9 + k];
        dy[6 + k] = F / S->m_a;
        dy[9 + k] = -F / S->m_i - kappa * y[3 + k];
    }
}

static void make_sys(const orc_problem* p, sys_int* S)
{
    double w2 = p->omega * p->omega;
    double C8 = p->C4 * p->C4 / (4.0 * p->De);
    S->m_a = p->m_atom;
    S->m_i = p->m_ion;
    S->C4 = p->C4 / w2;
    S->C8 = C8 / w2;
    for (int k = 0; k < 3; ++k) {
        S->a[k] = p->a[k];
        S->q[k] = p->q[k];
    }
    S->phase0 = p->phase0;
}

/* right-hand side in atomic units (time t, not tau), for the pins */
void orc_rhs_au(const orc_problem* p, double t, const double y[12], double dydt[12])
{
    sys_int S;
    make_sys(p, &S);
    double yi[NY], dyi[NY];
    for (int k = 0; k < 6; ++k) {
        yi[k] = y[k];
        yi[6 + k] = y[6 + k] / p->omega;
    }
    traj_rhs(&S, p->omega * t, yi, dyi);
    for (int k = 0; k < 6; ++k) {
        dydt[k] = dyi[k] * p->omega;
        dydt[6 + k] = dyi[6 + k] * p->omega * p->omega;
    }
}

/* separation |r_a - r_i| and the sign carrier d . (v_a - v_i) of its rate */
static double separation(const double* y)
{
    double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}
static double radial_rate_sign(const double* y)
{
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += (y[k] - y[3 + k]) * (y[6 + k] - y[9 + k]);
    return s;
}

/* The exit sphere.  Head-on runs start the ion at the trap centre, so the sphere the atom starts
 * on is the separation r0.  Thermal runs (Fig. 3 caption) start the atom on the sphere of radius
 * r0 about the trap centre with the ion displaced from it; the separation may then begin above r0
 * and a grazing atom never cross it from inside, so they stop when the atom leaves that sphere. */
static double exit_radius(const orc_problem* p, const double* y)
{
    if (!p->exit_centre) return separation(y);
    return sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
}
static double exit_rate_sign(const orc_problem* p, const double* y)
{
    if (!p->exit_centre) return radial_rate_sign(y);
    return y[0] * y[6] + y[1] * y[7] + y[2] * y[8];
}

/* relative energy 1/2 mu |v_a - v_i|^2 + V(r), internal units */
static double relative_energy(const sys_int* S, const double* y)
{
    double mu = S->m_a * S->m_i / (S->m_a + S->m_i);
    double v2 = 0.0;
    for (int k = 0; k < 3; ++k) v2 += (y[6 + k] - y[9 + k]) * (y[6 + k] - y[9 + k]);
    double r = separation(y);
    double r4 = r * r * r * r;
    return 0.5 * mu * v2 + S->C8 / (r4 * r4) - S->C4 / r4;
}

/* ion energy of Eq. (1) (kinetic + trap terms), a.u. */
double orc_ion_energy(const orc_problem* p, const double y[12], double t)
{
    double ke = 0.0, pe = 0.0;
    double cs = cos(p->omega * t + p->phase0);
    for (int k = 0; k < 3; ++k) {
        ke += 0.5 * p->m_ion * y[9 + k] * y[9 + k];
        pe += (p->a[k] + 2.0 * p->q[k] * cs) * p->m_ion * p->omega * p->omega * y[3 + k] * y[3 + k] / 8.0;
    }
    return ke + pe;
}

/* scattering angle and momentum transfer (Fig. 1 caption), ion heating */
void orc_observables(const orc_problem* p, const double y_init[12], const double y_fin[12],
                     double t_fin, double* angle, double* q_transfer, double* dE_ion)
{
    const double* vi = y_init + 6;
    const double* vf = y_fin + 6;
    double cx = vi[1] * vf[2] - vi[2] * vf[1];
    double cy = vi[2] * vf[0] - vi[0] * vf[2];
    double cz = vi[0] * vf[1] - vi[1] * vf[0];
    double dot = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
    /* arccos(v_i.v_f / (|v_i||v_f|)) written in its well-conditioned atan2 form */
    *angle = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
    double dv0 = vf[0] - vi[0], dv1 = vf[1] - vi[1], dv2 = vf[2] - vi[2];
    *q_transfer = p->m_atom * sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
    *dE_ion = orc_ion_energy(p, y_fin, t_fin) - orc_ion_energy(p, y_init, 0.0);
}

/* ---------------------------------------------------------------------------
 * Exit location.  The accepted step (tau, y) -> y(tau + h) carried the separation
 * from r_prev <= r0 to r_new > r0.  The crossing step size h* in (0, h] is found
 * by four secant iterations on g(h*) = r(RK5(y, h*)) - r0, each a fresh fifth-order
 * step from y; the first secant point is the linear interpolation between the step
 * ends.  The last evaluated step is the final state.
 * ------------------------------------------------------------------------- */
static double exit_locate(const orc_problem* p, const sys_int* S, double tau, const double* y, const double* k1,
                          double h, double r_prev, double r_new, double r0, double* yf, int64_t* nrhs)
{
    double k[7 * NY], ytmp[NY], y5[NY];
    double x0 = 0.0, g0 = r_prev - r0, x1 = h, g1 = r_new - r0;
    for (int it = 0; it < 4; ++it) {
        double x2 = (g1 != g0) ? x1 - g1 * (x1 - x0) / (g1 - g0) : x1;
        if (x2 < 0.0) x2 = 0.0;
        if (x2 > h) x2 = h;
        memcpy(k, k1, sizeof(double) * NY);
        dp5_attempt(NY, traj_rhs, S, tau, y, x2, k, ytmp, y5, NULL);
        *nrhs += 5;
        double g2 = exit_radius(p, y5) - r0;
        x0 = x1;
        g0 = g1;
        x1 = x2;
        g1 = g2;
        memcpy(yf, y5, sizeof(y5));
    }
    return x1;
}

/* ---------------------------------------------------------------------------
 * One trajectory.
 * Error test: err = max_k |e_k| / (atol + rtol max(|y_k|, |y5_k|)); accept iff err <= 1.
 * Step factor: min(5, max(0.2, 0.9 err^(-1/5))) (5 when err = 0), capped at 1 right
 * after a rejection; h <= hmax and the last step lands exactly on tau_max.
 * After each accepted step: bounce test (periapsis of the relative motion inside
 * r_b), bound-state test, exit test.
 * ------------------------------------------------------------------------- */
static int integrate_impl(const orc_problem* p, orc_result* R, double* hrec, int64_t cap)
{
    sys_int S;
    make_sys(p, &S);
    const double W = p->omega;
    const double tau_max = p->t_max * W;
    const double h0 = p->h0 > 0 ? p->h0 : 2.0 * M_PI * 1e-3;
    const double hmax = p->hmax > 0 ? p->hmax : 2.0 * M_PI / 8.0;
    const double hmin = p->hmin > 0 ? p->hmin : 1e-6 * h0;
    const double r_m = pow(p->C4 / (2.0 * p->De), 0.25);
    const double r_b = p->r_bounce_over_rm * r_m;
    const double r_floor = 0.1 * r_m;
    const double r0 = p->r0;

    double y[NY], y5[NY], err[NY], ytmp[NY], k[7 * NY], yend[NY];
    for (int kx = 0; kx < 6; ++kx) {
        y[kx] = p->y0[kx];
        y[6 + kx] = p->y0[6 + kx] / W;
    }
    memset(R, 0, sizeof(*R));
    uint32_t status = 0;
    int64_t n_acc = 0, n_rej = 0, nrhs = 0;
    int32_t nb = 0;
    double tau = 0.0, tau_first = 0.0, tau_last = 0.0;
    int rec_overflow = 0;

    /* start-of-run check of the asymptotic-start condition 10|V(r0)| < E */
    {
        double e_kin = 0.0;
        for (int kx = 0; kx < 3; ++kx) e_kin += 0.5 * p->m_atom * p->y0[6 + kx] * p->y0[6 + kx];
        double r = separation(p->y0);
        double r4 = r * r * r * r;
        double C8 = p->C4 * p->C4 / (4.0 * p->De);
        double V = C8 / (r4 * r4) - p->C4 / r4;
        if (!(10.0 * fabs(V) < e_kin)) status |= ORC_WARN_R0;
    }

    int finite0 = 1;
    for (int kx = 0; kx < NY; ++kx) finite0 &= isfinite(y[kx]);
    if (!finite0) {
        status |= ORC_NONFINITE;
        memcpy(yend, y, sizeof(y));
        goto done;
    }

    traj_rhs(&S, tau, y, k);
    nrhs = 1;
    double h = h0 < hmax ? h0 : hmax;
    int last_rejected = 0;
    double r_prev = separation(y), s_prev = radial_rate_sign(y), e_prev = exit_radius(p, y);

    for (;;) {
        if (p->max_steps > 0 && n_acc >= p->max_steps) {
            status |= ORC_MAX_STEPS;
            break;
        }
        int final_step = 0;
        if (h >= tau_max - tau) {
            h = tau_max - tau;
            final_step = 1;
        }
        if (!final_step && h < hmin) {
            status |= ORC_H_UNDERFLOW;
            break;
        }
        dp5_attempt(NY, traj_rhs, &S, tau, y, h, k, ytmp, y5, err);
        nrhs += 6;
        double en = 0.0;
        for (int i = 0; i < NY; ++i) {
            double sc = p->atol + p->rtol * fmax(fabs(y[i]), fabs(y5[i]));
            double ratio = fabs(err[i]) / sc;
            if (ratio > en || isnan(ratio)) en = ratio;
        }
        if (en <= 1.0) {
            n_acc++;
            int finite = 1;
            for (int i = 0; i < NY; ++i) finite &= isfinite(y5[i]);
            if (!finite) {
                status |= ORC_NONFINITE;
                break;
            }
            double tau_new = final_step ? tau_max : tau + h;
            double r_new = separation(y5), s_new = radial_rate_sign(y5);
            if (s_prev < 0.0 && s_new >= 0.0 && fmin(r_prev, r_new) < r_b) {
                if (nb == 0) tau_first = tau_new;
                tau_last = tau_new;
                nb++;
            }
            if (relative_energy(&S, y5) < 0.0) status |= ORC_BOUND_SEEN;
            if (r_new < r_floor) {
                memcpy(y, y5, sizeof(y));
                tau = tau_new;
                status |= ORC_R_UNDERFLOW;
                if (hrec) { if (n_acc <= cap) hrec[n_acc - 1] = h; else rec_overflow = 1; }
                break;
            }
            double e_new = exit_radius(p, y5);
            if (e_prev <= r0 && e_new > r0 && exit_rate_sign(p, y5) > 0.0) {
                double hs = exit_locate(p, &S, tau, y, k, h, e_prev, e_new, r0, yend, &nrhs);
                /* the located exit step, followed by the full size of that step */
                if (hrec) { if (n_acc < cap) { hrec[n_acc - 1] = hs; hrec[n_acc] = h; } else rec_overflow = 1; }
                tau = tau + hs;
                status |= ORC_EXITED;
                memcpy(y, yend, sizeof(y));
                break;
            }
            if (hrec) { if (n_acc <= cap) hrec[n_acc - 1] = h; else rec_overflow = 1; }
            memcpy(y, y5, sizeof(y));
            memcpy(k, &k[6 * NY], sizeof(double) * NY);
            tau = tau_new;
            r_prev = r_new;
            s_prev = s_new;
            e_prev = e_new;
            if (final_step) {
                status |= ORC_TMAX;
                break;
            }
            double fac = (en == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(en, -0.2)));
            if (last_rejected) fac = fmin(1.0, fac);
            h = fmin(hmax, h * fac);
            last_rejected = 0;
        } else {
            n_rej++;
            double fac = isnan(en) ? 0.2 : fmax(0.2, 0.9 * pow(en, -0.2));
            h = h * fac;
            last_rejected = 1;
        }
    }
    memcpy(yend, y, sizeof(y));

done:
    if (nb >= 2 || (status & ORC_TMAX)) status |= ORC_COMPLEX;
    for (int kx = 0; kx < 6; ++kx) {
        R->y_final[kx] = yend[kx];
        R->y_final[6 + kx] = yend[6 + kx] * W;
    }
    R->tau_final = tau;
    R->t_dwell = tau / W;
    R->t_first = tau_first / W;
    R->t_last = tau_last / W;
    R->n_bounce = nb;
    R->status = status;
    R->n_accept = n_acc;
    R->n_reject = n_rej;
    R->n_rhs = nrhs;
    orc_observables(p, p->y0, R->y_final, R->t_dwell, &R->angle, &R->q_transfer, &R->dE_ion);
    return rec_overflow ? -1 : 0;
}

int orc_integrate(const orc_problem* p, orc_result* r) { return integrate_impl(p, r, NULL, 0); }

int orc_integrate_record(const orc_problem* p, orc_result* r, double* h, int64_t cap)
{
    return integrate_impl(p, r, h, cap);
}

void orc_integrate_batch(int64_t n, const orc_problem* p, orc_result* r, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) integrate_impl(&p[i], &r[i], NULL, 0);
}

/* ---------------------------------------------------------------------------
 * Initial conditions (head-on-run paragraph): ion at rest at the trap centre,
 * atom on the sphere of radius r0 in direction (theta, phi), moving radially
 * inward with E = 1/2 m_a v0^2.
 * ------------------------------------------------------------------------- */
void orc_headon_state(double theta, double phi, double E, double m_atom, double r0, double y0[12])
{
    double n[3] = {sin(theta) * cos(phi), sin(theta) * sin(phi), cos(theta)};
    double v0 = sqrt(2.0 * E / m_atom);
    for (int k = 0; k < 3; ++k) {
        y0[k] = r0 * n[k];
        y0[3 + k] = 0.0;
        y0[6 + k] = -v0 * n[k];
        y0[9 + k] = 0.0;
    }
}

/* cell-centred grid on the octant (Fig. 1): theta_j = (j+1/2)(pi/2)/n_theta,
   phi_k = (k+1/2)(pi/2)/n_phi, id = j*n_phi + k */
void orc_grid_angles(int64_t id, int n_theta, int n_phi, double* theta, double* phi)
{
    int64_t j = id / n_phi, kk = id % n_phi;
    *theta = ((double)j + 0.5) * (M_PI / 2.0) / (double)n_theta;
    *phi = ((double)kk + 0.5) * (M_PI / 2.0) / (double)n_phi;
}

/* ---------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplications with the
 * Weyl-sequence key schedule.
 * ------------------------------------------------------------------------- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/*
 * Sweep draws for trajectory id: counter blocks (id, 0, 0, 0) and (id, 1, 0, 0)
 * under key (seed, 0) give uniforms u0..u7.  Direction uniform on the sphere
 * (cos theta = 1 - 2 u0, phi = 2 pi u1), RF phase 2 pi u2 (phase paragraph of the
 * Fig. 4 discussion), E log-uniform from u3, q uniform from u4, De log-uniform
 * from u5 -- or, for E, q, De given as lists, the cell digits of id mod the
 * number of cells (species slowest, De fastest).
 */
void orc_sweep_draw(int64_t id, const orc_sweep* s, double* cos_theta, double* phi, double* phase0,
                    double* E, double* qx, double* De, int32_t* species)
{
    uint64_t key[2] = {s->seed, 0};
    uint64_t c0[4] = {(uint64_t)id, 0, 0, 0}, c1[4] = {(uint64_t)id, 1, 0, 0};
    uint64_t b0[4], b1[4];
    orc_philox4x64_10(c0, key, b0);
    orc_philox4x64_10(c1, key, b1);
    double u[8] = {u01(b0[0]), u01(b0[1]), u01(b0[2]), u01(b0[3]),
                   u01(b1[0]), u01(b1[1]), u01(b1[2]), u01(b1[3])};
    int64_t nE = s->n_E > 0 ? s->n_E : 1, nq = s->n_q > 0 ? s->n_q : 1, nD = s->n_De > 0 ? s->n_De : 1;
    int64_t ncell = (int64_t)s->n_species * nE * nq * nD;
    int64_t c = id % ncell;
    int64_t iD = c % nD;
    c /= nD;
    int64_t iq = c % nq;
    c /= nq;
    int64_t iE = c % nE;
    c /= nE;
    int64_t isp = c;
    *cos_theta = 1.0 - 2.0 * u[0];
    *phi = 2.0 * M_PI * u[1];
    *phase0 = 2.0 * M_PI * u[2];
    *E = s->n_E > 0 ? s->E[iE] : s->E_lo * pow(s->E_hi / s->E_lo, u[3]);
    *qx = s->n_q > 0 ? s->q[iq] : s->q_lo + (s->q_hi - s->q_lo) * u[4];
    *De = s->n_De > 0 ? s->De[iD] : s->De_lo * pow(s->De_hi / s->De_lo, u[5]);
    *species = s->species[isp];
}

/* Box-Muller (G. E. P. Box and M. E. Muller, Ann. Math. Stat. 29, 610 (1958)): from uniforms u in
 * [0, 1) and v, r = sqrt(-2 ln(1 - u)) gives the normals r cos(2 pi v) and r sin(2 pi v). */
void orc_thermal_normals(int64_t id, uint64_t seed, double z[10])
{
    uint64_t key[2] = {seed, 0};
    for (int b = 0; b < 3; ++b) {
        uint64_t c[4] = {(uint64_t)id, (uint64_t)(2 + b), 0, 0}, o[4];
        orc_philox4x64_10(c, key, o);
        for (int m = 0; m < 2; ++m) {
            int j = 2 * (2 * b + m);
            if (j >= 10) break;
            double r = sqrt(-2.0 * log(1.0 - u01(o[2 * m])));
            double a = 2.0 * M_PI * u01(o[2 * m + 1]);
            z[j] = r * cos(a);
            z[j + 1] = r * sin(a);
        }
    }
}

/* ---------------------------------------------------------------------------
 * Fixed-step order test on y' = lam y or x'' = -x, for the pins.
 * ------------------------------------------------------------------------- */
static void rhs_exp(const void* ctx, double t, const double* y, double* dy)
{
    (void)t;
    dy[0] = (*(const double*)ctx) * y[0];
}
static void rhs_sho(const void* ctx, double t, const double* y, double* dy)
{
    (void)ctx;
    (void)t;
    dy[0] = y[1];
    dy[1] = -y[0];
}

double orc_fixed_step_error(int kind, double lam, double t_end, int n_steps)
{
    int n = kind == 0 ? 1 : 2;
    rhs_fn f = kind == 0 ? rhs_exp : rhs_sho;
    double y[2] = {1.0, 0.0}, y5[2], ytmp[2], err[2], k[14];
    double h = t_end / n_steps, t = 0.0;
    f(&lam, t, y, k);
    for (int s = 0; s < n_steps; ++s) {
        dp5_attempt(n, f, &lam, t, y, h, k, ytmp, y5, err);
        for (int i = 0; i < n; ++i) {
            y[i] = y5[i];
            k[i] = k[6 * n + i];
        }
        t += h;
    }
    if (kind == 0) return y[0] - exp(lam * t_end);
    return fmax(fabs(y[0] - cos(t_end)), fabs(y[1] + sin(t_end)));
}
