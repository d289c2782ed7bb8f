/*
 * CPU oracle, part 2: sensitivities of the observables.  TEST INFRASTRUCTURE ONLY.
 *
 * Tangent-linear of the discrete accepted-step map by internal differentiation: the primal is
 * run once (adaptive, recording its accepted step sizes), then the augmented system
 *   y' = f(tau, y),  Y_j' = J(tau, y) Y_j + b_j(tau, y)
 * (12 columns of the stability matrix, one column per model parameter q_x and De) is replayed
 * with the same Runge-Kutta scheme and the recorded steps.  At an exit the crossing time moves
 * with the state; first order: dh* = -(grad g . Y)/(grad g . f) with g = |r_a - r_i| - r0.
 *
 * Frozen-step central differences replay the same recorded steps for perturbed parameters and
 * locate the exit afresh (secant from the last step start), as in the primal run.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "iat_oracle.h"

#define NY 12
#define NCOL 14            /* 12 state columns + q_x + De */
#define NAUG (NY + NY * NCOL)

/* Dormand-Prince 5(4) coefficients (Dormand & Prince 1980), typed again here so that this
   file stands alone. */
static const double C_[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double A_[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
static const double B_[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0};

typedef struct {
    double m_a, m_i, C4, C8, De;   /* internal units (C4, C8 divided by Omega^2; De in a.u.) */
    double a[3], q[3], qr[3], phase0;
    int ncol;                      /* tangent columns carried (0 = primal only) */
} tsys;

static void make_tsys(const orc_problem* p, const double q_ratio[3], tsys* S)
{
    double w2 = p->omega * p->omega;
    S->m_a = p->m_atom;
    S->m_i = p->m_ion;
    S->C4 = p->C4 / w2;
    S->C8 = p->C4 * p->C4 / (4.0 * p->De) / w2;
    S->De = p->De;
    for (int k = 0; k < 3; ++k) {
        S->a[k] = p->a[k];
        S->q[k] = p->q[k];
        S->qr[k] = q_ratio[k];
    }
    S->phase0 = p->phase0;
    S->ncol = NCOL;
}

/* primal right-hand side of Eq. (1), internal units (the same formulas as iat_oracle.c) */
static void primal_rhs(const tsys* S, double tau, const double* y, double* dy)
{
    double d[3] = {y[0] - y[3], y[1] - y[4], y[2] - y[5]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r4 = r2 * r2, r6 = r4 * r2, r10 = r6 * r4;
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

/*
 * Augmented right-hand side.  With d = r_a - r_i, rho = |d|^2, s(rho) = 8 C8 rho^-5 - 4 C4 rho^-3:
 * the Jacobian of the force F = s d with respect to d is H = s I + 2 s'(rho) d d^T, so a tangent
 * column (dr_a, dr_i, dv_a, dv_i) moves as
 *   dr_a' = dv_a, dr_i' = dv_i, dv_a' = H (dr_a - dr_i)/m_a, dv_i' = -H (dr_a - dr_i)/m_i - kappa o dr_i
 * plus, for the parameter columns, the explicit derivative of f:
 *   q_x: dv_i,k' += -(q_ratio_k cos(tau + phase0)/2) r_i,k
 *   De : dv_a' += (ds/dDe) d/m_a, dv_i' -= (ds/dDe) d/m_i, ds/dDe = -8 C8 rho^-5 / De.
 */
static void aug_rhs(const void* ctx, double tau, const double* Y, double* dY)
{
    const tsys* S = (const tsys*)ctx;
    primal_rhs(S, tau, Y, dY);
    if (S->ncol == 0) return;
    double d[3] = {Y[0] - Y[3], Y[1] - Y[4], Y[2] - Y[5]};
    double rho = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double s = 8.0 * S->C8 / pow(rho, 5) - 4.0 * S->C4 / pow(rho, 3);
    double sp = -40.0 * S->C8 / pow(rho, 6) + 12.0 * S->C4 / pow(rho, 4);
    double H[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a][b] = (a == b ? s : 0.0) + 2.0 * sp * d[a] * d[b];
    double cs = cos(tau + S->phase0);
    double kappa[3];
    for (int k = 0; k < 3; ++k) kappa[k] = (S->a[k] + 2.0 * S->q[k] * cs) / 4.0;
    double dsdDe = -8.0 * S->C8 / pow(rho, 5) / S->De;
    for (int c = 0; c < S->ncol; ++c) {
        const double* T = Y + NY + NY * c;
        double* dT = dY + NY + NY * c;
        double dd[3] = {T[0] - T[3], T[1] - T[4], T[2] - T[5]};
        for (int a = 0; a < 3; ++a) {
            double Hd = H[a][0] * dd[0] + H[a][1] * dd[1] + H[a][2] * dd[2];
            dT[a] = T[6 + a];
            dT[3 + a] = T[9 + a];
            dT[6 + a] = Hd / S->m_a;
            dT[9 + a] = -Hd / S->m_i - kappa[a] * T[3 + a];
        }
        if (c == 12) {
            for (int k = 0; k < 3; ++k) dT[9 + k] += -(S->qr[k] * cs / 2.0) * Y[3 + k];
        } else if (c == 13) {
            for (int k = 0; k < 3; ++k) {
                dT[6 + k] += dsdDe * d[k] / S->m_a;
                dT[9 + k] -= dsdDe * d[k] / S->m_i;
            }
        }
    }
}

/* fifth-order Dormand-Prince step of an n-dimensional system (no error estimate) */
static void rk5_step(int n, const tsys* S, double tau, const double* y, double h, double* out)
{
    double* k = (double*)malloc(sizeof(double) * 6 * n);
    double* yt = (double*)malloc(sizeof(double) * n);
    aug_rhs(S, tau, y, k);
    for (int s = 1; s < 6; ++s) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += A_[s][j] * k[j * n + i];
            yt[i] = y[i] + h * acc;
        }
        aug_rhs(S, tau + C_[s] * h, yt, &k[s * n]);
    }
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += B_[j] * k[j * n + i];
        out[i] = y[i] + h * acc;
    }
    free(k);
    free(yt);
}

static double sep(const double* y)
{
    double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

/* primal record: accepted steps, and for an exit also the full size of the exit step */
typedef struct {
    orc_result res;
    double* h;
    int64_t n;          /* accepted steps (the last one is the located exit step if exited) */
    double h_exit_full;
    int exited;
} record;

static int primal_record(const orc_problem* p, record* R)
{
    orc_result r0;
    orc_integrate(p, &r0);
    int64_t cap = r0.n_accept + 2;
    R->h = (double*)malloc(sizeof(double) * cap);
    if (orc_integrate_record(p, &R->res, R->h, cap) != 0) return -1;
    R->n = R->res.n_accept;
    R->exited = (R->res.status & ORC_EXITED) != 0;
    R->h_exit_full = R->exited ? R->h[R->n] : 0.0;
    return 0;
}

/* head-on start and its derivatives with respect to theta, phi, E (internal units) */
static void headon_internal(const orc_problem* p, double theta, double phi, double E, double y[12],
                            double dth[12], double dph[12], double dE[12])
{
    double st = sin(theta), ct = cos(theta), sp = sin(phi), cp = cos(phi);
    double n[3] = {st * cp, st * sp, ct};
    double nt[3] = {ct * cp, ct * sp, -st};
    double np[3] = {-st * sp, st * cp, 0.0};
    double v0 = sqrt(2.0 * E / p->m_atom) / p->omega;
    double dv0 = v0 / (2.0 * E);
    for (int k = 0; k < 12; ++k) y[k] = dth[k] = dph[k] = dE[k] = 0.0;
    for (int k = 0; k < 3; ++k) {
        y[k] = p->r0 * n[k];
        y[6 + k] = -v0 * n[k];
        dth[k] = p->r0 * nt[k];
        dth[6 + k] = -v0 * nt[k];
        dph[k] = p->r0 * np[k];
        dph[6 + k] = -v0 * np[k];
        dE[6 + k] = -dv0 * n[k];
    }
}

/* ion energy of Eq. (1) in a.u. from an internal state at internal time tau */
static double ion_energy_int(const orc_problem* p, const double* y, double tau)
{
    double ke = 0.0, pe = 0.0, w = p->omega, cs = cos(tau + p->phase0);
    for (int k = 0; k < 3; ++k) {
        double v = y[9 + k] * w;
        ke += 0.5 * p->m_ion * v * v;
        pe += (p->a[k] + 2.0 * p->q[k] * cs) * p->m_ion * w * w * y[3 + k] * y[3 + k] / 8.0;
    }
    return ke + pe;
}

/* observables from the internal final state, the start velocity (a.u.) and tau_f */
static void obs_of(const orc_problem* p, const double* vi_au, const double* yf, double tau_f, double out[3])
{
    double vf[3] = {yf[6] * p->omega, yf[7] * p->omega, yf[8] * p->omega};
    double cx = vi_au[1] * vf[2] - vi_au[2] * vf[1];
    double cy = vi_au[2] * vf[0] - vi_au[0] * vf[2];
    double cz = vi_au[0] * vf[1] - vi_au[1] * vf[0];
    double dot = vi_au[0] * vf[0] + vi_au[1] * vf[1] + vi_au[2] * vf[2];
    out[0] = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
    double d0 = vf[0] - vi_au[0], d1 = vf[1] - vi_au[1], d2 = vf[2] - vi_au[2];
    out[1] = p->m_atom * sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    out[2] = ion_energy_int(p, yf, tau_f);   /* E_ion(0) = 0 for the head-on start */
}

int orc_tangent(const orc_problem* p0, double theta, double phi, double E, const double q_ratio[3],
                double dobs[15], double phi_out[144], double* ftle)
{
    if (p0->exit_centre) return -2;   /* head-on problems only */
    orc_problem p = *p0;
    double y0[12], dth[12], dph[12], dEy[12];
    headon_internal(&p, theta, phi, E, y0, dth, dph, dEy);
    for (int k = 0; k < 12; ++k) p.y0[k] = k < 6 ? y0[k] : y0[k] * p.omega;
    record R;
    if (primal_record(&p, &R) != 0) return -1;
    tsys S;
    make_tsys(&p, q_ratio, &S);
    double* Y = (double*)calloc(NAUG, sizeof(double));
    double* Yn = (double*)calloc(NAUG, sizeof(double));
    memcpy(Y, y0, sizeof(y0));
    for (int c = 0; c < 12; ++c) Y[NY + NY * c + c] = 1.0;   /* Phi(0) = I */
    double tau = 0.0;
    int64_t nsteps = R.n;
    for (int64_t s = 0; s < nsteps; ++s) {
        rk5_step(NAUG, &S, tau, Y, R.h[s], Yn);
        memcpy(Y, Yn, sizeof(double) * NAUG);
        tau = (s == nsteps - 1 && (R.res.status & ORC_TMAX)) ? p.t_max * p.omega : tau + R.h[s];
    }
    /* FTLE input: Phi at the final time, before the exit-time correction */
    for (int a = 0; a < 12; ++a)
        for (int c = 0; c < 12; ++c) phi_out[a * 12 + c] = Y[NY + NY * c + a];
    *ftle = 0.0;
    double f[12];
    primal_rhs(&S, tau, Y, f);
    if (R.exited) {
        double r = sep(Y);
        double g[12] = {0};
        for (int k = 0; k < 3; ++k) {
            g[k] = (Y[k] - Y[3 + k]) / r;
            g[3 + k] = -g[k];
        }
        double gf = 0.0;
        for (int k = 0; k < 12; ++k) gf += g[k] * f[k];
        for (int c = 0; c < NCOL; ++c) {
            double* T = Y + NY + NY * c;
            double gT = 0.0;
            for (int k = 0; k < 12; ++k) gT += g[k] * T[k];
            double dh = -gT / gf;
            for (int k = 0; k < 12; ++k) T[k] += f[k] * dh;
            /* the crossing time moves by dh: kept in the spare slot below */
            Yn[c] = dh;
        }
    } else {
        for (int c = 0; c < NCOL; ++c) Yn[c] = 0.0;
    }
    /* d(obs)/d(y_f) and d(obs)/d(tau_f) by differentiating the observable formulas */
    double vi[3] = {y0[6] * p.omega, y0[7] * p.omega, y0[8] * p.omega};
    double vf[3] = {Y[6] * p.omega, Y[7] * p.omega, Y[8] * p.omega};
    double c3[3] = {vi[1] * vf[2] - vi[2] * vf[1], vi[2] * vf[0] - vi[0] * vf[2], vi[0] * vf[1] - vi[1] * vf[0]};
    double Sn = sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
    double D = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
    double den = Sn * Sn + D * D;
    double ch[3] = {c3[0] / Sn, c3[1] / Sn, c3[2] / Sn};
    /* dS/dvf = ch x vi ; dS/dvi = vf x ch ; dD/dvf = vi ; dD/dvi = vf */
    double dS_dvf[3] = {ch[1] * vi[2] - ch[2] * vi[1], ch[2] * vi[0] - ch[0] * vi[2], ch[0] * vi[1] - ch[1] * vi[0]};
    double dS_dvi[3] = {vf[1] * ch[2] - vf[2] * ch[1], vf[2] * ch[0] - vf[0] * ch[2], vf[0] * ch[1] - vf[1] * ch[0]};
    double dang_dvf[3], dang_dvi[3];
    for (int k = 0; k < 3; ++k) {
        dang_dvf[k] = (D * dS_dvf[k] - Sn * vi[k]) / den;
        dang_dvi[k] = (D * dS_dvi[k] - Sn * vf[k]) / den;
    }
    double dv[3] = {vf[0] - vi[0], vf[1] - vi[1], vf[2] - vi[2]};
    double ndv = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double dq_dvf[3] = {p.m_atom * dv[0] / ndv, p.m_atom * dv[1] / ndv, p.m_atom * dv[2] / ndv};
    /* dE_ion = E_ion(y_f, tau_f): gradient in internal state units, and in tau_f */
    double cs = cos(tau + p.phase0), sn = sin(tau + p.phase0), w = p.omega;
    double dE_dy[12] = {0};
    double dE_dtau = 0.0, dE_dq = 0.0;
    for (int k = 0; k < 3; ++k) {
        dE_dy[3 + k] = (p.a[k] + 2.0 * p.q[k] * cs) * p.m_ion * w * w * Y[3 + k] / 4.0;
        dE_dy[9 + k] = p.m_ion * w * w * Y[9 + k];
        dE_dtau += -2.0 * p.q[k] * sn * p.m_ion * w * w * Y[3 + k] * Y[3 + k] / 8.0;
        dE_dq += 2.0 * q_ratio[k] * cs * p.m_ion * w * w * Y[3 + k] * Y[3 + k] / 8.0;
    }
    /* columns: dy_f/dp for p = theta, phi, E from Phi (corrected) times dy0/dp; q, De directly */
    const double* dy0[3] = {dth, dph, dEy};
    for (int pi = 0; pi < 5; ++pi) {
        double col[12], dtau = 0.0;
        if (pi < 3) {
            for (int a = 0; a < 12; ++a) {
                col[a] = 0.0;
                for (int c = 0; c < 12; ++c) col[a] += Y[NY + NY * c + a] * dy0[pi][c];
            }
            for (int c = 0; c < 12; ++c) dtau += Yn[c] * dy0[pi][c];
        } else {
            int c = pi == 3 ? 12 : 13;
            for (int a = 0; a < 12; ++a) col[a] = Y[NY + NY * c + a];
            dtau = Yn[c];
        }
        double da = 0.0, dq = 0.0, de = 0.0;
        for (int k = 0; k < 3; ++k) {
            da += dang_dvf[k] * w * col[6 + k];
            dq += dq_dvf[k] * w * col[6 + k];
        }
        for (int k = 0; k < 12; ++k) de += dE_dy[k] * col[k];
        de += dE_dtau * dtau;
        if (pi < 3) {   /* explicit dependence through the start velocity */
            for (int k = 0; k < 3; ++k) {
                double dvi = dy0[pi][6 + k] * w;
                da += dang_dvi[k] * dvi;
                dq -= dq_dvf[k] * dvi;
            }
        }
        if (pi == 3) de += dE_dq;
        dobs[0 * 5 + pi] = da;
        dobs[1 * 5 + pi] = dq;
        dobs[2 * 5 + pi] = de;
    }
    free(Y);
    free(Yn);
    free(R.h);
    return 0;
}

/* frozen-step replay of the primal for perturbed parameters; returns the observables */
static int replay_obs(const orc_problem* p, const record* R, double theta, double phi, double E, double out[3])
{
    double y[12], dth[12], dph[12], dEy[12], yn[12];
    headon_internal(p, theta, phi, E, y, dth, dph, dEy);
    tsys S;
    double qr[3] = {0, 0, 0};
    make_tsys(p, qr, &S);
    S.ncol = 0;
    double tau = 0.0;
    int64_t whole = R->exited ? R->n - 1 : R->n;
    for (int64_t s = 0; s < whole; ++s) {
        rk5_step(NY, &S, tau, y, R->h[s], yn);
        memcpy(y, yn, sizeof(y));
        tau = (s == whole - 1 && (R->res.status & ORC_TMAX)) ? p->t_max * p->omega : tau + R->h[s];
    }
    if (R->exited) {
        /* fresh exit location from the last step start, as in the primal run */
        double hf = R->h_exit_full;
        rk5_step(NY, &S, tau, y, hf, yn);
        double x0 = 0.0, g0 = sep(y) - p->r0, x1 = hf, g1 = sep(yn) - p->r0, yt[12];
        for (int it = 0; it < 4; ++it) {
            double x2 = (g1 != g0) ? x1 - g1 * (x1 - x0) / (g1 - g0) : x1;
            if (x2 < 0.0) x2 = 0.0;
            if (x2 > hf) x2 = hf;
            rk5_step(NY, &S, tau, y, x2, yt);
            double g2 = sep(yt) - p->r0;
            x0 = x1;
            g0 = g1;
            x1 = x2;
            g1 = g2;
        }
        memcpy(y, yt, sizeof(y));
        tau += x1;
    }
    double vi[3] = {0, 0, 0}, y0[12];
    headon_internal(p, theta, phi, E, y0, dth, dph, dEy);
    for (int k = 0; k < 3; ++k) vi[k] = y0[6 + k] * p->omega;
    obs_of(p, vi, y, tau, out);
    return 0;
}

int orc_fd(const orc_problem* p0, double theta, double phi, double E, const double q_ratio[3], double rel_h,
           double dobs[15])
{
    if (p0->exit_centre) return -2;   /* head-on problems only */
    orc_problem p = *p0;
    double y0[12], dth[12], dph[12], dEy[12];
    headon_internal(&p, theta, phi, E, y0, dth, dph, dEy);
    for (int k = 0; k < 12; ++k) p.y0[k] = k < 6 ? y0[k] : y0[k] * p.omega;
    record R;
    if (primal_record(&p, &R) != 0) return -1;
    double qx = p.q[0] / (q_ratio[0] != 0.0 ? q_ratio[0] : 1.0);
    double base[5] = {theta, phi, E, qx, p.De};
    double ref[5] = {1.0, 1.0, fabs(E), fmax(fabs(qx), 0.1), fabs(p.De)};
    for (int pi = 0; pi < 5; ++pi) {
        double h = rel_h * fmax(fabs(base[pi]), ref[pi]);
        double o[2][3];
        for (int sgn = 0; sgn < 2; ++sgn) {
            double v[5];
            memcpy(v, base, sizeof(v));
            v[pi] += sgn == 0 ? h : -h;
            orc_problem q = p;
            for (int k = 0; k < 3; ++k) q.q[k] = v[3] * q_ratio[k];
            q.De = v[4];
            replay_obs(&q, &R, v[0], v[1], v[2], o[sgn]);
        }
        for (int k = 0; k < 3; ++k) dobs[k * 5 + pi] = (o[0][k] - o[1][k]) / (2.0 * h);
    }
    free(R.h);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Frozen-step central differences in extended precision, Richardson-extrapolated.
 *
 * The replay of the recorded accepted steps is a smooth map of the parameters, but evaluated in
 * FP64 it carries round-off that the collision amplifies (~1e-11 of the observables), so a central
 * difference of step h has a round-off floor of that over h on top of its O(h^2) truncation.  The
 * same replay in the x87 extended format (64-bit significand, ~2^11 times less round-off) lowers
 * that floor, and Richardson's extrapolation (4 D(h/2) - D(h))/3 of the central quotients D cancels
 * their h^2 term, leaving O(h^4).  Every operation of the replay (start state, Runge-Kutta stages,
 * exit secant, observables) is carried out in long double here, with its own exact-ratio tableau.
 * ------------------------------------------------------------------------- */
typedef long double ldbl;

static const ldbl LC_[7] = {0.0L, 1.0L / 5.0L, 3.0L / 10.0L, 4.0L / 5.0L, 8.0L / 9.0L, 1.0L, 1.0L};
static const ldbl LA_[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0L / 5.0L, 0, 0, 0, 0},
    {3.0L / 40.0L, 9.0L / 40.0L, 0, 0, 0},
    {44.0L / 45.0L, -56.0L / 15.0L, 32.0L / 9.0L, 0, 0},
    {19372.0L / 6561.0L, -25360.0L / 2187.0L, 64448.0L / 6561.0L, -212.0L / 729.0L, 0},
    {9017.0L / 3168.0L, -355.0L / 33.0L, 46732.0L / 5247.0L, 49.0L / 176.0L, -5103.0L / 18656.0L},
};
static const ldbl LB_[6] = {35.0L / 384.0L, 0.0L, 500.0L / 1113.0L, 125.0L / 192.0L, -2187.0L / 6784.0L,
                            11.0L / 84.0L};

typedef struct {
    ldbl w, m_a, m_i, C4, C8;      /* C4, C8 divided by Omega^2 */
    ldbl a[3], q[3], phase0, r0;
} lsys;

/* the system at parameters (q_x, De), everything else from the problem */
static void make_lsys(const orc_problem* p, ldbl qx, const double q_ratio[3], ldbl De, lsys* S)
{
    S->w = p->omega;
    ldbl w2 = S->w * S->w;
    S->m_a = p->m_atom;
    S->m_i = p->m_ion;
    S->C4 = (ldbl)p->C4 / w2;
    S->C8 = (ldbl)p->C4 * (ldbl)p->C4 / (4.0L * De) / w2;
    for (int k = 0; k < 3; ++k) {
        S->a[k] = p->a[k];
        S->q[k] = qx * (ldbl)q_ratio[k];
    }
    S->phase0 = p->phase0;
    S->r0 = p->r0;
}

static void rhs_ld(const lsys* S, ldbl tau, const ldbl* y, ldbl* dy)
{
    ldbl d[3] = {y[0] - y[3], y[1] - y[4], y[2] - y[5]};
    ldbl r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    ldbl r4 = r2 * r2, r6 = r4 * r2, r10 = r6 * r4;
    ldbl s = 8.0L * S->C8 / r10 - 4.0L * S->C4 / r6;
    ldbl cs = cosl(tau + S->phase0);
    for (int k = 0; k < 3; ++k) {
        ldbl F = s * d[k];
        ldbl kappa = (S->a[k] + 2.0L * S->q[k] * cs) / 4.0L;
        dy[k] = y[6 + k];
        dy[3 + k] = y[9 + k];
        dy[6 + k] = F / S->m_a;
        dy[9 + k] = -F / S->m_i - kappa * y[3 + k];
    }
}

static void rk5_ld(const lsys* S, ldbl tau, const ldbl* y, ldbl h, ldbl* out)
{
    ldbl k[6][NY], yt[NY];
    rhs_ld(S, tau, y, k[0]);
    for (int s = 1; s < 6; ++s) {
        for (int i = 0; i < NY; ++i) {
            ldbl acc = 0.0L;
            for (int j = 0; j < s; ++j) acc += LA_[s][j] * k[j][i];
            yt[i] = y[i] + h * acc;
        }
        rhs_ld(S, tau + LC_[s] * h, yt, k[s]);
    }
    for (int i = 0; i < NY; ++i) {
        ldbl acc = 0.0L;
        for (int j = 0; j < 6; ++j) acc += LB_[j] * k[j][i];
        out[i] = y[i] + h * acc;
    }
}

static ldbl sep_ld(const ldbl* y)
{
    ldbl d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
    return sqrtl(d0 * d0 + d1 * d1 + d2 * d2);
}

/* observables (angle, q_transfer, dE_ion) of the frozen-step replay at parameters v */
static void replay_obs_ld(const orc_problem* p, const record* R, const double q_ratio[3], const ldbl v[5],
                          ldbl out[3])
{
    lsys S;
    make_lsys(p, v[3], q_ratio, v[4], &S);
    ldbl n[3] = {sinl(v[0]) * cosl(v[1]), sinl(v[0]) * sinl(v[1]), cosl(v[0])};
    ldbl v0 = sqrtl(2.0L * v[2] / S.m_a);     /* a.u. */
    ldbl y[NY], yn[NY], vi[3];
    for (int k = 0; k < 3; ++k) {
        y[k] = S.r0 * n[k];
        y[3 + k] = 0.0L;
        vi[k] = -v0 * n[k];
        y[6 + k] = vi[k] / S.w;
        y[9 + k] = 0.0L;
    }
    ldbl tau = 0.0L;
    int64_t whole = R->exited ? R->n - 1 : R->n;
    for (int64_t s = 0; s < whole; ++s) {
        rk5_ld(&S, tau, y, R->h[s], yn);
        memcpy(y, yn, sizeof(y));
        tau = (s == whole - 1 && (R->res.status & ORC_TMAX)) ? (ldbl)p->t_max * S.w : tau + R->h[s];
    }
    if (R->exited) {
        ldbl hf = R->h_exit_full, yt[NY];
        rk5_ld(&S, tau, y, hf, yn);
        ldbl x0 = 0.0L, g0 = sep_ld(y) - S.r0, x1 = hf, g1 = sep_ld(yn) - S.r0;
        for (int it = 0; it < 4; ++it) {
            ldbl x2 = (g1 != g0) ? x1 - g1 * (x1 - x0) / (g1 - g0) : x1;
            if (x2 < 0.0L) x2 = 0.0L;
            if (x2 > hf) x2 = hf;
            rk5_ld(&S, tau, y, x2, yt);
            ldbl g2 = sep_ld(yt) - S.r0;
            x0 = x1;
            g0 = g1;
            x1 = x2;
            g1 = g2;
        }
        memcpy(y, yt, sizeof(y));
        tau += x1;
    }
    ldbl vf[3] = {y[6] * S.w, y[7] * S.w, y[8] * S.w};
    ldbl cx = vi[1] * vf[2] - vi[2] * vf[1], cy = vi[2] * vf[0] - vi[0] * vf[2], cz = vi[0] * vf[1] - vi[1] * vf[0];
    out[0] = atan2l(sqrtl(cx * cx + cy * cy + cz * cz), vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2]);
    ldbl d0 = vf[0] - vi[0], d1 = vf[1] - vi[1], d2 = vf[2] - vi[2];
    out[1] = S.m_a * sqrtl(d0 * d0 + d1 * d1 + d2 * d2);
    ldbl cs = cosl(tau + S.phase0), e = 0.0L;
    for (int k = 0; k < 3; ++k) {
        ldbl u = y[9 + k] * S.w;
        e += 0.5L * S.m_i * u * u + (S.a[k] + 2.0L * S.q[k] * cs) * S.m_i * S.w * S.w * y[3 + k] * y[3 + k] / 8.0L;
    }
    out[2] = e;                      /* E_ion(0) = 0 for the head-on start */
}

int orc_fd_richardson(const orc_problem* p0, double theta, double phi, double E, const double q_ratio[3],
                      double rel_h, double dobs[15])
{
    if (p0->exit_centre) return -2;   /* head-on problems only */
    orc_problem p = *p0;
    double y0[12], dth[12], dph[12], dEy[12];
    headon_internal(&p, theta, phi, E, y0, dth, dph, dEy);
    for (int k = 0; k < 12; ++k) p.y0[k] = k < 6 ? y0[k] : y0[k] * p.omega;
    record R;
    if (primal_record(&p, &R) != 0) return -1;
    double qx = p.q[0] / (q_ratio[0] != 0.0 ? q_ratio[0] : 1.0);
    ldbl base[5] = {theta, phi, E, qx, p.De};
    double ref[5] = {1.0, 1.0, fabs(E), fmax(fabs(qx), 0.1), fabs(p.De)};
    for (int pi = 0; pi < 5; ++pi) {
        ldbl h = (ldbl)rel_h * (ldbl)fmax(fabs((double)base[pi]), ref[pi]);
        ldbl D[2][3];
        for (int lev = 0; lev < 2; ++lev) {
            ldbl hl = lev == 0 ? h : h / 2.0L, o[2][3];
            for (int sgn = 0; sgn < 2; ++sgn) {
                ldbl v[5];
                for (int j = 0; j < 5; ++j) v[j] = base[j];
                v[pi] += sgn == 0 ? hl : -hl;
                replay_obs_ld(&p, &R, q_ratio, v, o[sgn]);
            }
            for (int k = 0; k < 3; ++k) D[lev][k] = (o[0][k] - o[1][k]) / (2.0L * hl);
        }
        for (int k = 0; k < 3; ++k) dobs[k * 5 + pi] = (double)((4.0L * D[1][k] - D[0][k]) / 3.0L);
    }
    free(R.h);
    return 0;
}
