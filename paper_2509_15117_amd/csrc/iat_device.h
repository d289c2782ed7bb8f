// Device side of libiat: one lane integrates one trajectory with its whole FP64 state in
// registers.  Shared by the plain and the persistent kernels, so a trajectory id gives the
// same bits whichever kernel or lane runs it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iat.h"

namespace iat {

// ---------------------------------------------------------------------------------------
// Dormand & Prince (1980) 5(4) pair, J. Comput. Appl. Math. 6:19 (the ode45 pair the paper
// cites for its integrator).  a_sj, the fifth-order weights b_j (= last row, FSAL) and the
// error weights e_j = b_j - bhat_j.
// ---------------------------------------------------------------------------------------
constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                 a54 = -212.0 / 729.0;
constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                 a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                 b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
constexpr double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0,
                 e5 = -17253.0 / 339200.0, e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;

// Second-order (Runge-Kutta-Nystrom) form.  Because the position derivative is the
// velocity, the stage positions are X_s = x + c_s h v + h^2 sum_j (A^2)_sj F_j and the
// fifth-order position is x + h v + h^2 sum_j (bA)_j F_j, where F_j are the stage
// accelerations.  Only the six accelerations per stage are kept, not twelve derivatives.
// The position error h sum_j e_j V_j reduces to h^2 sum_j (eA)_j F_j since sum_j e_j = 0.
constexpr double p31 = a32 * a21;
constexpr double p41 = a42 * a21 + a43 * a31, p42 = a43 * a32;
constexpr double p51 = a52 * a21 + a53 * a31 + a54 * a41, p52 = a53 * a32 + a54 * a42,
                 p53 = a54 * a43;
constexpr double p61 = a62 * a21 + a63 * a31 + a64 * a41 + a65 * a51,
                 p62 = a63 * a32 + a64 * a42 + a65 * a52, p63 = a64 * a43 + a65 * a53,
                 p64 = a65 * a54;
constexpr double q1 = b3 * a31 + b4 * a41 + b5 * a51 + b6 * a61,
                 q2 = b3 * a32 + b4 * a42 + b5 * a52 + b6 * a62,
                 q3 = b4 * a43 + b5 * a53 + b6 * a63, q4 = b5 * a54 + b6 * a64, q5 = b6 * a65;
constexpr double r1 = e3 * a31 + e4 * a41 + e5 * a51 + e6 * a61 + e7 * b1,
                 r2 = e3 * a32 + e4 * a42 + e5 * a52 + e6 * a62,
                 r3 = e4 * a43 + e5 * a53 + e6 * a63 + e7 * b3,
                 r4 = e5 * a54 + e6 * a64 + e7 * b4, r5 = e6 * a65 + e7 * b5, r6 = e7 * b6;

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---------------------------------------------------------------------------------------
// Launch parameters (kernel argument block), all in internal units where it matters.
// ---------------------------------------------------------------------------------------
struct KParams {
    // system
    double omega, m_ion;
    double a_x, q_x, a_ratio[3], q_ratio[3];
    double E, De, phase0;
    int32_t species, n_species;
    double r0, r0sq, tau_max;
    double rtol, atol, h0, hmax, hmin;
    double r_bounce_over_rm, rb_ratio2;
    double inv_mi, kA[3];        // 1/m_i and a_k/4
    int64_t max_steps;
    double sp_m[IAT_MAX_SPECIES], sp_C4[IAT_MAX_SPECIES];
    // batch
    int64_t n;
    const double *theta, *phi, *E_arr, *qx_arr, *De_arr, *phase_arr, *y0;
    const int32_t* sp_arr;
    iat_gen gen;
    // outputs
    double *angle, *q_transfer, *dE_ion, *t_dwell, *t_first, *t_last;
    int32_t* n_bounce;
    uint32_t* status;
    int64_t *n_accept, *n_reject, *n_rhs;
    double* y_final;
    uint64_t* stats;
    int32_t refill_every;
};

// Species table lookup by select (no dynamic indexing into the kernel-argument block).
__device__ __forceinline__ double species_mass(const KParams& P, int sp)
{
    double m = P.sp_m[0];
#pragma unroll
    for (int s = 1; s < IAT_MAX_SPECIES; ++s) m = (sp == s) ? P.sp_m[s] : m;
    return m;
}
__device__ __forceinline__ double species_C4(const KParams& P, int sp)
{
    double c = P.sp_C4[0];
#pragma unroll
    for (int s = 1; s < IAT_MAX_SPECIES; ++s) c = (sp == s) ? P.sp_C4[s] : c;
    return c;
}
template <typename T>
__device__ __forceinline__ T pick8(const T* a, int64_t idx)
{
    T r = a[0];
#pragma unroll
    for (int s = 1; s < 8; ++s) r = (idx == s) ? a[s] : r;
    return r;
}

// Physical parameters of one trajectory.
struct TrajParams {
    double sin_t, cos_t, sin_p, cos_p;  // direction of the start point
    double E, qx, De, phase0;
    int32_t sp;
};

// Per-lane constants of the equations of motion (internal units).  Values that are the same
// for every trajectory of a launch (1/m_i, a_k, q ratios) are read from KParams instead.
struct Lane {
    double inv_ma;
    double c8x8, c4x4;      // 8 C8', 4 C4'  (C' = C / Omega^2)
    double qx_half;         // q_x / 2: kappa_k(tau) = a_k/4 + (q_x/2) q_ratio_k cos(tau + phase0)
    double phase0;
    double rm2;             // r_m^2
    double half_mu;         // reduced mass / 2
};

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds, Weyl key schedule.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__device__ __forceinline__ double unit_double(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Trajectory id -> physical parameters (GRID / SWEEP / ARRAYS generators, see iat.h).
__device__ inline void traj_params(const KParams& P, int64_t i, TrajParams& t)
{
    const int64_t gid = P.gen.id0 + i;
    double theta = 0.0, phi = 0.0;
    t.E = P.E;
    t.qx = P.q_x;
    t.De = P.De;
    t.phase0 = P.phase0;
    t.sp = P.species;
    if (P.gen.kind == IAT_GEN_GRID) {
        const int64_t j = gid / P.gen.n_phi, k = gid % P.gen.n_phi;
        theta = ((double)j + 0.5) * (kTwoPi / 4.0) / (double)P.gen.n_theta;
        phi = ((double)k + 0.5) * (kTwoPi / 4.0) / (double)P.gen.n_phi;
    } else if (P.gen.kind == IAT_GEN_SWEEP) {
        uint64_t b0[4] = {(uint64_t)gid, 0, 0, 0}, b1[4] = {(uint64_t)gid, 1, 0, 0};
        philox4x64(b0, P.gen.seed, 0);
        philox4x64(b1, P.gen.seed, 0);
        const int64_t nE = P.gen.n_E > 0 ? P.gen.n_E : 1, nq = P.gen.n_q > 0 ? P.gen.n_q : 1,
                      nD = P.gen.n_De > 0 ? P.gen.n_De : 1;
        int64_t c = gid % ((int64_t)P.gen.n_species * nE * nq * nD);
        const int64_t iD = c % nD;
        c /= nD;
        const int64_t iq = c % nq;
        c /= nq;
        const int64_t iE = c % nE;
        c /= nE;
        theta = acos(1.0 - 2.0 * unit_double(b0[0]));
        phi = kTwoPi * unit_double(b0[1]);
        t.phase0 = kTwoPi * unit_double(b0[2]);
        t.E = P.gen.n_E > 0 ? pick8(P.gen.E, iE) : P.gen.E_lo * pow(P.gen.E_hi / P.gen.E_lo, unit_double(b0[3]));
        t.qx = P.gen.n_q > 0 ? pick8(P.gen.q, iq) : P.gen.q_lo + (P.gen.q_hi - P.gen.q_lo) * unit_double(b1[0]);
        t.De = P.gen.n_De > 0 ? pick8(P.gen.De, iD)
                              : P.gen.De_lo * pow(P.gen.De_hi / P.gen.De_lo, unit_double(b1[1]));
        t.sp = pick8(P.gen.species, c);
    } else {
        if (P.theta) theta = P.theta[i];
        if (P.phi) phi = P.phi[i];
        if (P.E_arr) t.E = P.E_arr[i];
        if (P.qx_arr) t.qx = P.qx_arr[i];
        if (P.De_arr) t.De = P.De_arr[i];
        if (P.phase_arr) t.phase0 = P.phase_arr[i];
        if (P.sp_arr) t.sp = P.sp_arr[i];
    }
    t.sin_t = sin(theta);
    t.cos_t = cos(theta);
    t.sin_p = sin(phi);
    t.cos_p = cos(phi);
}

// Start state in atomic units: the given y0, else the head-on start.
__device__ inline void start_state_au(const KParams& P, int64_t i, const TrajParams& t, double y[12])
{
    if (P.y0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = P.y0[(int64_t)k * P.n + i];
        return;
    }
    const double n0 = t.sin_t * t.cos_p, n1 = t.sin_t * t.sin_p, n2 = t.cos_t;
    const double v0 = sqrt(2.0 * t.E / species_mass(P, t.sp));
    y[0] = P.r0 * n0;
    y[1] = P.r0 * n1;
    y[2] = P.r0 * n2;
    y[6] = -v0 * n0;
    y[7] = -v0 * n1;
    y[8] = -v0 * n2;
#pragma unroll
    for (int k = 3; k < 6; ++k) {
        y[k] = 0.0;
        y[6 + k] = 0.0;
    }
}

__device__ inline void lane_consts(const KParams& P, const TrajParams& t, Lane& L)
{
    const double ma = species_mass(P, t.sp), mi = P.m_ion;
    const double w2 = P.omega * P.omega;
    const double C4 = species_C4(P, t.sp);
    const double C8 = C4 * C4 / (4.0 * t.De);
    L.inv_ma = 1.0 / ma;
    L.c8x8 = 8.0 * (C8 / w2);
    L.c4x4 = 4.0 * (C4 / w2);
    L.qx_half = 0.5 * t.qx;
    L.phase0 = t.phase0;
    L.rm2 = sqrt(C4 / (2.0 * t.De));
    L.half_mu = 0.5 * (ma * mi / (ma + mi));
}

// ---------------------------------------------------------------------------------------
// Equations of motion (Eq. (1)) in internal units.  d = r_a - r_i, u = 1/|d|^2;
// force on the atom F = (8 C8' u^5 - 4 C4' u^3) d; atom a = F/m_a; ion a = -F/m_i - kappa o r_i
// with kappa_k = (a_k + 2 q_k cos(tau + phase0))/4.  `cs` is cos(tau + phase0).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void accel(const KParams& P, const Lane& L, double cs, const double X[6], double A[6])
{
    const double d0 = X[0] - X[3], d1 = X[1] - X[4], d2 = X[2] - X[5];
    const double rho = d0 * d0 + d1 * d1 + d2 * d2;
    const double u = 1.0 / rho;
    const double u2 = u * u;
    const double s = u2 * u * (L.c8x8 * u2 - L.c4x4);
    const double qc = L.qx_half * cs;
    const double F0 = s * d0, F1 = s * d1, F2 = s * d2;
    A[0] = F0 * L.inv_ma;
    A[1] = F1 * L.inv_ma;
    A[2] = F2 * L.inv_ma;
    A[3] = -F0 * P.inv_mi - (P.kA[0] + qc * P.q_ratio[0]) * X[3];
    A[4] = -F1 * P.inv_mi - (P.kA[1] + qc * P.q_ratio[1]) * X[4];
    A[5] = -F2 * P.inv_mi - (P.kA[2] + qc * P.q_ratio[2]) * X[5];
}

// cos and sin of a stage offset 0 <= d <= pi/4 (steps never exceed an eighth of the RF
// period): Maclaurin series through d^16 and d^17; the first omitted terms are below 3e-18.
__device__ __forceinline__ void small_sincos(double d, double& c, double& s)
{
    constexpr double f2 = 1.0 / 2, f3 = f2 / 3, f4 = f3 / 4, f5 = f4 / 5, f6 = f5 / 6, f7 = f6 / 7,
                     f8 = f7 / 8, f9 = f8 / 9, f10 = f9 / 10, f11 = f10 / 11, f12 = f11 / 12,
                     f13 = f12 / 13, f14 = f13 / 14, f15 = f14 / 15, f16 = f15 / 16, f17 = f16 / 17;
    const double z = d * d;
    double pc = f16;
    pc = pc * z - f14;
    pc = pc * z + f12;
    pc = pc * z - f10;
    pc = pc * z + f8;
    pc = pc * z - f6;
    pc = pc * z + f4;
    pc = pc * z - f2;
    c = pc * z + 1.0;
    double ps = f17;
    ps = ps * z - f15;
    ps = ps * z + f13;
    ps = ps * z - f11;
    ps = ps * z + f9;
    ps = ps * z - f7;
    ps = ps * z + f5;
    ps = ps * z - f3;
    s = d + d * (ps * z);
}

// cos(theta + d) from cos/sin(theta) and the stage offset d
__device__ __forceinline__ double cos_shift(double cb, double sb, double d)
{
    double c, s;
    small_sincos(d, c, s);
    return cb * c - sb * s;
}

// One Dormand-Prince step of size h from (tau, x, v) with F1 = accel(tau, x).
// Always produces the fifth-order (x5, v5).  With fsal it also evaluates the last stage
// F7 = accel(tau + h, x5) and returns the max-norm error ratio
//   en = max_k |err_k| / (atol + rtol max(|y_k|, |y5_k|))   (NaN if anything is non-finite);
// without it (exit re-steps) it returns 0 after five new evaluations.
__device__ __forceinline__ double dp5_step(const KParams& P, const Lane& L, bool fsal, double tau, double h,
                                           const double x[6], const double v[6], const double F1[6],
                                           double x5[6], double v5[6], double F7[6])
{
    const double hh = h * h;
    double sb, cb;
    sincos(tau + L.phase0, &sb, &cb);
    double F2[6], F3[6], F4[6], F5[6], F6[6], X[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = x[k] + (c2 * h) * v[k];
    accel(P, L, cos_shift(cb, sb, c2 * h), X, F2);
    // stage velocities are not needed: only positions enter the accelerations
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = x[k] + (c3 * h) * v[k] + hh * (p31 * F1[k]);
    accel(P, L, cos_shift(cb, sb, c3 * h), X, F3);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = x[k] + (c4 * h) * v[k] + hh * (p41 * F1[k] + p42 * F2[k]);
    accel(P, L, cos_shift(cb, sb, c4 * h), X, F4);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        X[k] = x[k] + (c5 * h) * v[k] + hh * (p51 * F1[k] + p52 * F2[k] + p53 * F3[k]);
    accel(P, L, cos_shift(cb, sb, c5 * h), X, F5);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        X[k] = x[k] + h * v[k] + hh * (p61 * F1[k] + p62 * F2[k] + p63 * F3[k] + p64 * F4[k]);
    const double cs_end = cos_shift(cb, sb, h);
    accel(P, L, cs_end, X, F6);
    double ex[6], ev[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        x5[k] = x[k] + h * v[k] + hh * (q1 * F1[k] + q2 * F2[k] + q3 * F3[k] + q4 * F4[k] + q5 * F5[k]);
        v5[k] = v[k] + h * (b1 * F1[k] + b3 * F3[k] + b4 * F4[k] + b5 * F5[k] + b6 * F6[k]);
        ex[k] = hh * (r1 * F1[k] + r2 * F2[k] + r3 * F3[k] + r4 * F4[k] + r5 * F5[k] + r6 * F6[k]);
        ev[k] = h * (e1 * F1[k] + e3 * F3[k] + e4 * F4[k] + e5 * F5[k] + e6 * F6[k]);
    }
    if (!fsal) return 0.0;
    accel(P, L, cs_end, x5, F7);
#pragma unroll
    for (int k = 0; k < 6; ++k) ev[k] += h * (e7 * F7[k]);
    // max_k |err_k| / sc_k located by cross-multiplication (sc_k > 0), then one division
    double num = 0.0, den = 1.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double yk = k < 6 ? x[k] : v[k - 6];
        const double y5k = k < 6 ? x5[k] : v5[k - 6];
        const double ek = fabs(k < 6 ? ex[k] : ev[k - 6]);
        const double sc = P.atol + P.rtol * fmax(fabs(yk), fabs(y5k));
        bad |= !(ek <= 1.0e300) || !(sc <= 1.0e300);
        const bool gt = ek * den > num * sc;
        num = gt ? ek : num;
        den = gt ? sc : den;
    }
    return bad ? __builtin_nan("") : num / den;
}

// Trajectory state carried across steps.  mode 0: stepping; mode 1..4: the lane is locating
// the exit crossing (secant iterate mode), holding the step start y_n in x, v, F1.
struct Traj {
    double x[6], v[6], F1[6];
    double tau, h;
    double rho_prev, s_prev;     // separation^2 and sign carrier of d(separation)/dt at y_n
    double sx1, sg1;             // secant: latest iterate (the previous one is in rho_prev/s_prev)
    double tau_first, tau_last;
    int32_t nacc, nrej, nrhs, nb;
    uint32_t status, mode;
    bool last_rej, done;
    Lane L;
};

__device__ __forceinline__ double sep2(const double x[6])
{
    const double d0 = x[0] - x[3], d1 = x[1] - x[4], d2 = x[2] - x[5];
    return d0 * d0 + d1 * d1 + d2 * d2;
}
__device__ __forceinline__ double radial_sign(const double x[6], const double v[6])
{
    return (x[0] - x[3]) * (v[0] - v[3]) + (x[1] - x[4]) * (v[1] - v[4]) + (x[2] - x[5]) * (v[2] - v[5]);
}

__device__ inline void traj_start(const KParams& P, int64_t i, Traj& T)
{
    TrajParams tp;
    traj_params(P, i, tp);
    lane_consts(P, tp, T.L);
    double y[12];
    start_state_au(P, i, tp, y);
    T.status = 0;
    {   // asymptotic-start condition 10 |V(r0)| < E (head-on-run paragraph)
        const double ma = species_mass(P, tp.sp);
        const double ek = 0.5 * ma * (y[6] * y[6] + y[7] * y[7] + y[8] * y[8]);
        const double C4 = species_C4(P, tp.sp), C8 = C4 * C4 / (4.0 * tp.De);
        const double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2, r4 = r2 * r2;
        const double V = C8 / (r4 * r4) - C4 / r4;
        if (!(10.0 * fabs(V) < ek)) T.status |= IAT_ST_WARN_R0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        T.x[k] = y[k];
        T.v[k] = y[6 + k] / P.omega;
    }
    T.tau = 0.0;
    T.tau_first = T.tau_last = 0.0;
    T.sx1 = T.sg1 = 0.0;
    T.nacc = T.nrej = 0;
    T.nb = 0;
    T.mode = 0;
    T.last_rej = false;
    T.done = false;
    double fin = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) fin += T.x[k] + T.v[k];
    if (!__builtin_isfinite(fin)) {
        T.status |= IAT_ST_NONFINITE;
        T.done = true;
        T.nrhs = 0;
        T.h = 0.0;
        T.rho_prev = T.s_prev = 0.0;
        return;
    }
    accel(P, T.L, cos(T.L.phase0), T.x, T.F1);
    T.nrhs = 1;
    T.h = P.h0 < P.hmax ? P.h0 : P.hmax;
    T.rho_prev = sep2(T.x);
    T.s_prev = radial_sign(T.x, T.v);
}

// One attempted step plus the events of an accepted step, or one secant iterate of the exit
// location.  Exit location: once an accepted step y_n -> y_{n+1} carries the separation across
// r0 outward, four secant iterations on g(h*) = |r(RK5(y_n, h*))| - r0 follow, each a fresh
// step from y_n, starting from the linear interpolation between the step ends; the last
// iterate is the final state.
__device__ __forceinline__ void traj_advance(const KParams& P, Traj& T)
{
    double h;
    bool fin = false;
    const bool exiting = T.mode != 0;
    if (exiting) {
        const double x0 = T.rho_prev, g0 = T.s_prev, x1 = T.sx1, g1 = T.sg1;
        h = (g1 != g0) ? x1 - g1 * (x1 - x0) / (g1 - g0) : x1;
        h = h < 0.0 ? 0.0 : (h > T.h ? T.h : h);
    } else {
        if (T.nacc >= P.max_steps) {
            T.status |= IAT_ST_MAX_STEPS;
            T.done = true;
            return;
        }
        h = T.h;
        if (h >= P.tau_max - T.tau) {
            h = P.tau_max - T.tau;
            fin = true;
        }
        if (!fin && h < P.hmin) {
            T.status |= IAT_ST_H_UNDERFLOW;
            T.done = true;
            return;
        }
    }
    double x5[6], v5[6], F7[6];
    const double en = dp5_step(P, T.L, !exiting, T.tau, h, T.x, T.v, T.F1, x5, v5, F7);
    if (exiting) {
        T.nrhs += 5;
        const double g2 = sqrt(sep2(x5)) - P.r0;
        T.rho_prev = T.sx1;
        T.s_prev = T.sg1;
        T.sx1 = h;
        T.sg1 = g2;
        if (++T.mode > 4) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                T.x[k] = x5[k];
                T.v[k] = v5[k];
            }
            T.tau = T.tau + h;
            T.status |= IAT_ST_EXITED;
            T.done = true;
        }
        return;
    }
    T.nrhs += 6;
    if (en <= 1.0) {
        T.nacc++;
        double fs = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) fs += x5[k] + v5[k];
        if (!__builtin_isfinite(fs)) {
            T.status |= IAT_ST_NONFINITE;
            T.done = true;
            return;
        }
        const double tau_new = fin ? P.tau_max : T.tau + h;
        const double rho_new = sep2(x5), s_new = radial_sign(x5, v5);
        // bounce: periapsis of the relative motion inside r_b
        if (T.s_prev < 0.0 && s_new >= 0.0 && fmin(T.rho_prev, rho_new) < T.L.rm2 * P.rb_ratio2) {
            if (T.nb == 0) T.tau_first = tau_new;
            T.tau_last = tau_new;
            T.nb++;
        }
        // bound-state test: 1/2 mu v_rel^2 + C8'/rho^4 - C4'/rho^2 < 0 (rho = r^2), taken
        // multiplied through by rho^4 > 0 so that no division is needed
        {
            const double w0 = v5[0] - v5[3], w1 = v5[1] - v5[4], w2 = v5[2] - v5[5];
            const double rho2 = rho_new * rho_new;
            if (T.L.half_mu * (w0 * w0 + w1 * w1 + w2 * w2) * (rho2 * rho2) + 0.125 * T.L.c8x8 -
                    0.25 * T.L.c4x4 * rho2 < 0.0)
                T.status |= IAT_ST_BOUND_SEEN;
        }
        if (rho_new < 0.01 * T.L.rm2) {   // separation below 0.1 r_m: integration broken
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                T.x[k] = x5[k];
                T.v[k] = v5[k];
            }
            T.tau = tau_new;
            T.status |= IAT_ST_R_UNDERFLOW;
            T.done = true;
            return;
        }
        if (T.rho_prev <= P.r0sq && rho_new > P.r0sq && s_new > 0.0) {
            // keep y_n; the next four calls are the secant iterates (x0, g0) -> (rho_prev, s_prev)
            T.mode = 1;
            T.s_prev = sqrt(T.rho_prev) - P.r0;
            T.rho_prev = 0.0;
            T.sx1 = h;
            T.sg1 = sqrt(rho_new) - P.r0;
            T.h = h;
            return;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            T.x[k] = x5[k];
            T.v[k] = v5[k];
            T.F1[k] = F7[k];
        }
        T.tau = tau_new;
        T.rho_prev = rho_new;
        T.s_prev = s_new;
        if (fin) {
            T.status |= IAT_ST_TMAX;
            T.done = true;
            T.h = h;
            return;
        }
        double fac = en == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * exp2(-0.2 * log2(en))));
        if (T.last_rej) fac = fmin(1.0, fac);
        T.h = fmin(P.hmax, h * fac);
        T.last_rej = false;
    } else {
        T.nrej++;
        const double fac = (en != en) ? 0.2 : fmax(0.2, 0.9 * exp2(-0.2 * log2(en)));
        T.h = h * fac;
        T.last_rej = true;
    }
}

// Ion energy of Eq. (1) (kinetic + trap terms) in atomic units at internal time tau.
__device__ __forceinline__ double ion_energy_au(const KParams& P, double qx, double phase0, const double y[12],
                                                double tau)
{
    const double cs = cos(tau + phase0);
    double ke = 0.0, pe = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ke += y[9 + k] * y[9 + k];
        pe += (P.a_x * P.a_ratio[k] + 2.0 * (qx * P.q_ratio[k]) * cs) * y[3 + k] * y[3 + k];
    }
    return 0.5 * P.m_ion * ke + pe * (P.m_ion * P.omega * P.omega / 8.0);
}

// Write the observables of trajectory i (outputs are in atomic units).
__device__ inline void traj_finish(const KParams& P, int64_t i, const Traj& T)
{
    TrajParams tp;
    traj_params(P, i, tp);
    double y0[12];
    start_state_au(P, i, tp, y0);
    double yf[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        yf[k] = T.x[k];
        yf[6 + k] = T.v[k] * P.omega;
    }
    uint32_t st = T.status;
    if (T.nb >= 2 || (st & IAT_ST_TMAX)) st |= IAT_ST_COMPLEX;
    const double* vi = y0 + 6;
    const double* vf = yf + 6;
    const double cx = vi[1] * vf[2] - vi[2] * vf[1];
    const double cy = vi[2] * vf[0] - vi[0] * vf[2];
    const double cz = vi[0] * vf[1] - vi[1] * vf[0];
    const double dot = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
    P.angle[i] = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
    const double dv0 = vf[0] - vi[0], dv1 = vf[1] - vi[1], dv2 = vf[2] - vi[2];
    P.q_transfer[i] = species_mass(P, tp.sp) * sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
    P.dE_ion[i] = ion_energy_au(P, tp.qx, tp.phase0, yf, T.tau) - ion_energy_au(P, tp.qx, tp.phase0, y0, 0.0);
    const double inv_w = 1.0 / P.omega;
    P.t_dwell[i] = T.tau * inv_w;
    if (P.t_first) P.t_first[i] = T.tau_first * inv_w;
    if (P.t_last) P.t_last[i] = T.tau_last * inv_w;
    P.n_bounce[i] = T.nb;
    P.status[i] = st;
    if (P.n_accept) P.n_accept[i] = T.nacc;
    if (P.n_reject) P.n_reject[i] = T.nrej;
    if (P.n_rhs) P.n_rhs[i] = T.nrhs;
    if (P.y_final) {
#pragma unroll
        for (int k = 0; k < 12; ++k) P.y_final[(int64_t)k * P.n + i] = yf[k];
    }
}

}  // namespace iat
