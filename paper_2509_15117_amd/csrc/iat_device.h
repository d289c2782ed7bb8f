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

// The Nystrom tableau as one object.  Where a kernel's step uses kTab directly the coefficients
// become instruction literals; a 64-bit literal has to be rebuilt in scalar registers at every use
// (two scalar moves, each a wave issue slot), so the latency-bound four-lane tail instead holds a
// copy in vector registers for the whole kernel (tab_in_registers).  The values are the same, so
// the step gives the same bits either way.
struct Tab {
    double c2, c3, c4, c5;
    double p31, p41, p42, p51, p52, p53, p61, p62, p63, p64;
    double q1, q2, q3, q4, q5;
    double b1, b3, b4, b5, b6;
    double r1, r2, r3, r4, r5, r6;
    double e1, e3, e4, e5, e6, e7;
};
constexpr Tab kTab = {c2,  c3,  c4,  c5,  p31, p41, p42, p51, p52, p53, p61, p62, p63, p64, q1, q2, q3, q4,
                      q5,  b1,  b3,  b4,  b5,  b6,  r1,  r2,  r3,  r4,  r5,  r6,  e1, e3, e4, e5, e6, e7};

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
    const int64_t* id0_dev;      // device offset added to gen.id0, or NULL
    iat_gen gen;
    // outputs
    double *angle, *q_transfer, *dE_ion, *t_dwell, *t_first, *t_last;
    int32_t* n_bounce;
    uint32_t* status;
    int64_t *n_accept, *n_reject, *n_rhs;
    double* y_final;
    uint64_t* stats;
    int32_t refill_every;
    int64_t budget;              // attempted steps before suspension (0: never)
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

// Global id of the batch's first trajectory: gen.id0, plus the device-side offset when one is given
// (one captured call replayed over successive chunks).
__device__ __forceinline__ int64_t batch_id0(const KParams& P) { return P.gen.id0 + (P.id0_dev ? *P.id0_dev : 0); }

// Trajectory id -> physical parameters (GRID / SWEEP / ARRAYS generators, see iat.h).
__device__ inline void traj_params(const KParams& P, int64_t i, TrajParams& t)
{
    const int64_t gid = batch_id0(P) + i;
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
    } else if (P.gen.kind == IAT_GEN_SWEEP || P.gen.kind == IAT_GEN_THERMAL) {
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

// Nine standard normals of a thermal start: Box-Muller on Philox blocks (id, 2..4, 0, 0).
__device__ inline void thermal_normals(const KParams& P, int64_t gid, double z[10])
{
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        uint64_t c[4] = {(uint64_t)gid, (uint64_t)(2 + b), 0, 0};
        philox4x64(c, P.gen.seed, 0);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (2 * (2 * b + m) >= 10) break;
            const double r = sqrt(-2.0 * log(1.0 - unit_double(c[2 * m])));
            double sn, cs;
            sincospi(2.0 * unit_double(c[2 * m + 1]), &sn, &cs);
            z[2 * (2 * b + m)] = r * cs;
            z[2 * (2 * b + m) + 1] = r * sn;
        }
    }
}

// Start state in atomic units: the given y0, the thermal start, else the head-on start.
__device__ inline void start_state_au(const KParams& P, int64_t i, const TrajParams& t, double y[12])
{
    if (P.y0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) y[k] = P.y0[(int64_t)k * P.n + i];
        return;
    }
    if (P.gen.kind == IAT_GEN_THERMAL) {
        double z[10];
        thermal_normals(P, batch_id0(P) + i, z);
        const double n0 = t.sin_t * t.cos_p, n1 = t.sin_t * t.sin_p, n2 = t.cos_t;
        const double sa = sqrt(t.E / species_mass(P, t.sp));
        double v0 = sa * z[0], v1 = sa * z[1], v2 = sa * z[2];
        if (v0 * n0 + v1 * n1 + v2 * n2 >= 0.0) {
            v0 = -v0;
            v1 = -v1;
            v2 = -v2;
        }
        const double w = t.qx * P.omega / (2.0 * sqrt(2.0));
        const double sv = sqrt(P.gen.T_ion / P.m_ion), sx = sv / w;
        y[0] = P.r0 * n0;
        y[1] = P.r0 * n1;
        y[2] = P.r0 * n2;
        y[6] = v0;
        y[7] = v1;
        y[8] = v2;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            y[3 + k] = sx * z[3 + k];
            y[9 + k] = sv * z[6 + k];
        }
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
// Per-component expressions.  Every arithmetic expression of a step is written once here and
// used by both forms of the step: one lane per trajectory (all 12 components in one lane) and
// four lanes per trajectory (lane k of a quad holds the atom and ion components of axis k).
// With contraction decided per source expression, both forms produce the same bits.
// ---------------------------------------------------------------------------------------

// 1/x by the hardware reciprocal refined with two Newton steps (x > 0, normal).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double dot3(double a0, double a1, double a2, double b0, double b1, double b2)
{
    return a0 * b0 + a1 * b1 + a2 * b2;
}

// Equations of motion (Eq. (1)) in internal units.  d = r_a - r_i, u = 1/|d|^2; the force on
// the atom is F = s d with s = 8 C8' u^5 - 4 C4' u^3; atom acceleration F/m_a; ion acceleration
// -F/m_i - kappa_k r_i,k with kappa_k = (a_k + 2 q_k cos(tau + phase0))/4 = kA_k + qc qr_k,
// qc = (q_x/2) cos(tau + phase0).
__device__ __forceinline__ double force_scale_rr(const Lane& L, double rr)
{
    const double u = recip(rr);
    const double u2 = u * u;
    return u2 * u * (L.c8x8 * u2 - L.c4x4);
}
__device__ __forceinline__ double force_scale(const Lane& L, double d0, double d1, double d2)
{
    return force_scale_rr(L, dot3(d0, d1, d2, d0, d1, d2));
}
__device__ __forceinline__ double acc_atom(const Lane& L, double s, double dk) { return (s * dk) * L.inv_ma; }
__device__ __forceinline__ double acc_ion(double inv_mi, double s, double dk, double kA, double qc, double qr,
                                          double xi)
{
    return -(s * dk) * inv_mi - (kA + qc * qr) * xi;
}

// A copy of the tableau in vector registers: the empty asm statements make each value opaque, so
// the compiler keeps it in a register instead of folding it back into literals.
__device__ __forceinline__ Tab tab_in_registers()
{
    Tab t = kTab;
#define IAT_PIN(f) asm volatile("" : "+v"(t.f))
    IAT_PIN(c2); IAT_PIN(c3); IAT_PIN(c4); IAT_PIN(c5);
    IAT_PIN(p31); IAT_PIN(p41); IAT_PIN(p42); IAT_PIN(p51); IAT_PIN(p52); IAT_PIN(p53);
    IAT_PIN(p61); IAT_PIN(p62); IAT_PIN(p63); IAT_PIN(p64);
    IAT_PIN(q1); IAT_PIN(q2); IAT_PIN(q3); IAT_PIN(q4); IAT_PIN(q5);
    IAT_PIN(b1); IAT_PIN(b3); IAT_PIN(b4); IAT_PIN(b5); IAT_PIN(b6);
    IAT_PIN(r1); IAT_PIN(r2); IAT_PIN(r3); IAT_PIN(r4); IAT_PIN(r5); IAT_PIN(r6);
    IAT_PIN(e1); IAT_PIN(e3); IAT_PIN(e4); IAT_PIN(e5); IAT_PIN(e6); IAT_PIN(e7);
#undef IAT_PIN
    return t;
}

// Stage positions X_s = x + c_s h v + h^2 sum_j (A^2)_sj F_j, fifth-order solution and error.
__device__ __forceinline__ double stage2(double x, double v, double h, const Tab& T = kTab)
{
    return x + (T.c2 * h) * v;
}
__device__ __forceinline__ double stage3(double x, double v, double h, double hh, double f1, const Tab& T = kTab)
{
    return x + (T.c3 * h) * v + hh * (T.p31 * f1);
}
__device__ __forceinline__ double stage4(double x, double v, double h, double hh, double f1, double f2,
                                         const Tab& T = kTab)
{
    return x + (T.c4 * h) * v + hh * (T.p41 * f1 + T.p42 * f2);
}
__device__ __forceinline__ double stage5(double x, double v, double h, double hh, double f1, double f2, double f3,
                                         const Tab& T = kTab)
{
    return x + (T.c5 * h) * v + hh * (T.p51 * f1 + T.p52 * f2 + T.p53 * f3);
}
__device__ __forceinline__ double stage6(double x, double v, double h, double hh, double f1, double f2, double f3,
                                         double f4, const Tab& T = kTab)
{
    return x + h * v + hh * (T.p61 * f1 + T.p62 * f2 + T.p63 * f3 + T.p64 * f4);
}
__device__ __forceinline__ double sol_x(double x, double v, double h, double hh, double f1, double f2, double f3,
                                        double f4, double f5, const Tab& T = kTab)
{
    return x + h * v + hh * (T.q1 * f1 + T.q2 * f2 + T.q3 * f3 + T.q4 * f4 + T.q5 * f5);
}
__device__ __forceinline__ double sol_v(double v, double h, double f1, double f3, double f4, double f5, double f6,
                                        const Tab& T = kTab)
{
    return v + h * (T.b1 * f1 + T.b3 * f3 + T.b4 * f4 + T.b5 * f5 + T.b6 * f6);
}
__device__ __forceinline__ double err_x(double hh, double f1, double f2, double f3, double f4, double f5, double f6,
                                        const Tab& T = kTab)
{
    return hh * (T.r1 * f1 + T.r2 * f2 + T.r3 * f3 + T.r4 * f4 + T.r5 * f5 + T.r6 * f6);
}
__device__ __forceinline__ double err_v(double h, double f1, double f3, double f4, double f5, double f6, double f7,
                                        const Tab& T = kTab)
{
    const double e = h * (T.e1 * f1 + T.e3 * f3 + T.e4 * f4 + T.e5 * f5 + T.e6 * f6);
    return e + h * (T.e7 * f7);
}
// |err_k| / (atol + rtol max(|y_k|, |y5_k|)) with a refined hardware reciprocal
__device__ __forceinline__ double err_ratio(double e, double y, double y5, double rtol, double atol)
{
    const double sc = atol + rtol * fmax(fabs(y), fabs(y5));
    double r = __builtin_amdgcn_rcp(sc);
    r = fma(r, fma(-sc, r, 1.0), r);
    return fabs(e) * r;
}
__device__ __forceinline__ bool ratio_bad(double r) { return !(r <= 1.0e300); }
__device__ __forceinline__ bool is_finite(double x) { return __builtin_isfinite(x); }

// fma(a, b, c); A3: as the three-address instruction.  For a chain whose addends are constants kept in
// registers the compiler otherwise picks the two-address accumulate form and copies the constant into
// the accumulator before every step of the chain (the latency-bound solo level takes A3; the other
// kernels keep the compiler's choice, which holds their register count).  Same value either way.
template <bool A3>
__device__ __forceinline__ double fma3(double a, double b, double c)
{
    if constexpr (A3) {
        double r;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
        return r;
    } else {
        return fma(a, b, c);
    }
}

// cos and sin of a stage offset 0 <= d <= pi/4 (steps never exceed an eighth of the RF
// period): Maclaurin series through d^16 and d^17; the first omitted terms are below 3e-18.
template <bool A3 = false>
__device__ __forceinline__ void small_sincos(double d, double& c, double& s)
{
    constexpr double f2 = 1.0 / 2, f3 = f2 / 3, f4 = f3 / 4, f5 = f4 / 5, f6 = f5 / 6, f7 = f6 / 7,
                     f8 = f7 / 8, f9 = f8 / 9, f10 = f9 / 10, f11 = f10 / 11, f12 = f11 / 12,
                     f13 = f12 / 13, f14 = f13 / 14, f15 = f14 / 15, f16 = f15 / 16, f17 = f16 / 17;
    const double z = d * d;
    double pc = f16;
    pc = fma3<A3>(pc, z, -f14);
    pc = fma3<A3>(pc, z, f12);
    pc = fma3<A3>(pc, z, -f10);
    pc = fma3<A3>(pc, z, f8);
    pc = fma3<A3>(pc, z, -f6);
    pc = fma3<A3>(pc, z, f4);
    pc = fma3<A3>(pc, z, -f2);
    c = fma3<A3>(pc, z, 1.0);
    double ps = f17;
    ps = fma3<A3>(ps, z, -f15);
    ps = fma3<A3>(ps, z, f13);
    ps = fma3<A3>(ps, z, -f11);
    ps = fma3<A3>(ps, z, f9);
    ps = fma3<A3>(ps, z, -f7);
    ps = fma3<A3>(ps, z, f5);
    ps = fma3<A3>(ps, z, -f3);
    s = d + d * (ps * z);
}

// sin and cos of an RF phase 0 <= x < 1.6e6: Cody-Waite reduction x = k pi/2 + r with pi/2
// split into P1 + P2 + P3 (33, 33 and 53 significant bits, so k P1 and k P2 are exact for
// |k| < 2^20), then the Maclaurin polynomials on |r| <= pi/4 and the quadrant k mod 4.
__device__ __forceinline__ double phase_reduce(double x, double& k)
{
    constexpr double kTwoOverPi = 0.63661977236758134308;
    constexpr double P1 = 0x1.921fb54400000p+0, P2 = 0x1.0b4611a600000p-34, P3 = 0x1.3198a2e037073p-69;
    k = rint(x * kTwoOverPi);
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    return fma(-k, P3, r);
}
// sin, cos of x = k pi/2 + r from cos r, sin r
__device__ __forceinline__ void phase_quadrant(double k, double cr, double sr, double& s, double& c)
{
    const int q = ((int)k) & 3;
    const double a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;   // sin, cos up to sign
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}
__device__ __forceinline__ void phase_sincos(double x, double& s, double& c)
{
    double k;
    const double r = phase_reduce(x, k);
    double cr, sr;
    small_sincos(r, cr, sr);
    phase_quadrant(k, cr, sr, s, c);
}

// en^(-1/5) for en >= 1e-4: single-precision estimate from the hardware log2/exp2, refined by
// two Newton steps on g(y) = en y^5 - 1 (the relative error goes 1e-7 -> 3e-14 -> rounding).
__device__ __forceinline__ double inv_fifth_root(double en)
{
    const float ef = (float)en;
    double y = (double)__builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(ef));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y2 = y * y;
        const double t = fma(-en, y2 * y2 * y, 1.0);
        y = fma(0.2 * y, t, y);
    }
    return y;
}

// cos(theta + d) from cos/sin(theta) and cos/sin(d)
__device__ __forceinline__ double cos_comb(double cb, double sb, double c, double s) { return cb * c - sb * s; }
// cos(theta + d) from cos/sin(theta) and the stage offset d
__device__ __forceinline__ double cos_shift(double cb, double sb, double d)
{
    double c, s;
    small_sincos(d, c, s);
    return cos_comb(cb, sb, c, s);
}

// Cosines of the RF phase at the stage times tau + c_s h (s = 2..6; stage 7 shares c = 1).
struct StageCos {
    double c2, c3, c4, c5, c6;
};
__device__ __forceinline__ StageCos stage_cos(double tau, double phase0, double h)
{
    double sb, cb;
    phase_sincos(tau + phase0, sb, cb);
    StageCos C;
    C.c2 = cos_shift(cb, sb, c2 * h);
    C.c3 = cos_shift(cb, sb, c3 * h);
    C.c4 = cos_shift(cb, sb, c4 * h);
    C.c5 = cos_shift(cb, sb, c5 * h);
    C.c6 = cos_shift(cb, sb, h);
    return C;
}

// bound-state test 1/2 mu v_rel^2 + C8'/rho^4 - C4'/rho^2 < 0 (rho = r^2), multiplied through
// by rho^4 > 0 so that no division is needed
__device__ __forceinline__ bool bound_state(const Lane& L, double rho, double w2)
{
    const double rho2 = rho * rho;
    return L.half_mu * w2 * (rho2 * rho2) + 0.125 * L.c8x8 - 0.25 * L.c4x4 * rho2 < 0.0;
}

// Step factors min(5, max(0.2, 0.9 en^(-1/5))), capped at 1 right after a rejection; below
// en = 1.8e-4 the factor is 5 whatever en is ((0.9/5)^5 = 1.89e-4).
__device__ __forceinline__ double step_factor(double en, bool last_rej)
{
    const double fac = en < 1.8e-4 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * inv_fifth_root(en)));
    return last_rej ? fmin(1.0, fac) : fac;
}
__device__ __forceinline__ double reject_factor(double en)
{
    return (en != en) ? 0.2 : fmax(0.2, 0.9 * inv_fifth_root(en));
}

// ---------------------------------------------------------------------------------------
// Trajectory state carried across steps.  mode 0: stepping; mode 1..4: the trajectory is
// locating its exit crossing (secant iterate mode), holding the step start y_n.
// The scalar part is the same for both forms; the vector part is 12 components (one lane)
// or the 4 components of one axis (four lanes).
// ---------------------------------------------------------------------------------------
struct Scal {
    double tau, h;
    double rho_prev, s_prev;     // separation^2 and the sign carrier of its rate at y_n
    double sx1, sg1;             // secant: latest iterate (the previous one sits in rho_prev/s_prev)
    double tau_first, tau_last;
    int32_t nacc, nrej, nrhs, nb;
    uint32_t status, mode;
    int32_t last_rej, done;
};

__device__ inline void scal_init(const KParams& P, Scal& S)
{
    S.tau = 0.0;
    S.tau_first = S.tau_last = 0.0;
    S.sx1 = S.sg1 = 0.0;
    S.nacc = S.nrej = 0;
    S.nrhs = 0;
    S.nb = 0;
    S.mode = 0;
    S.last_rej = 0;
    S.done = 0;
    S.h = P.h0 < P.hmax ? P.h0 : P.hmax;
    S.rho_prev = S.s_prev = 0.0;
}

// asymptotic-start condition 10 |V(r0)| < E (head-on-run paragraph), on the a.u. start state
__device__ inline bool warn_r0(const KParams& P, const TrajParams& tp, const double y[12])
{
    const double ma = species_mass(P, tp.sp);
    const double ek = 0.5 * ma * (y[6] * y[6] + y[7] * y[7] + y[8] * y[8]);
    const double C4 = species_C4(P, tp.sp), C8 = C4 * C4 / (4.0 * tp.De);
    const double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2, r4 = r2 * r2;
    const double V = C8 / (r4 * r4) - C4 / r4;
    return !(10.0 * fabs(V) < ek);
}

// The launch constants a step reads.  Where a kernel is short of scalar registers the compiler
// reloads them from the kernel-argument block at every use (a scalar load and its wait); the
// latency-bound four-lane tail keeps a copy in vector registers instead (step_k_in_registers).
struct StepK {
    double r0, r0sq, tau_max, rtol, atol, hmax, hmin, rb_ratio2;
    int64_t max_steps;
};
__device__ __forceinline__ StepK step_k(const KParams& P)
{
    StepK k;
    k.r0 = P.r0;
    k.r0sq = P.r0sq;
    k.tau_max = P.tau_max;
    k.rtol = P.rtol;
    k.atol = P.atol;
    k.hmax = P.hmax;
    k.hmin = P.hmin;
    k.rb_ratio2 = P.rb_ratio2;
    k.max_steps = P.max_steps;
    return k;
}
__device__ __forceinline__ StepK step_k_in_registers(const KParams& P)
{
    StepK k = step_k(P);
    asm volatile("" : "+v"(k.r0), "+v"(k.r0sq), "+v"(k.tau_max), "+v"(k.rtol), "+v"(k.atol));
    asm volatile("" : "+v"(k.hmax), "+v"(k.hmin), "+v"(k.rb_ratio2), "+v"(k.max_steps));
    return k;
}

// A branch condition of the step, as is, or (UNI) as a wave-uniform value for kernels in which every
// lane of the wave holds the same scalar state: a ballot turns it into a scalar condition, so the
// branch needs no exec-mask bookkeeping.  The value of the condition is the same either way.
template <bool UNI>
__device__ __forceinline__ bool cond(bool c)
{
    if constexpr (UNI)
        return __builtin_amdgcn_ballot_w64(c) != 0;
    else
        return c;
}
// The lanes of the wave on which one comparison holds.  ANDs and ORs of these masks are, lane by lane,
// the masks of the ANDs and ORs of the comparisons; the ballot of a single comparison is that
// comparison's own lane mask, while the ballot of a combined condition first turns it into a vector
// value and back.
__device__ __forceinline__ uint64_t lanes(bool c) { return __builtin_amdgcn_ballot_w64(c); }

// Step prologue shared by both forms: picks h and handles the stops that precede a step.
// Returns false when the trajectory stopped.
template <bool UNI = false>
__device__ __forceinline__ bool step_prologue(const StepK& K, Scal& S, double& h, bool& fin)
{
    fin = false;
    if (cond<UNI>(S.mode != 0)) {
        const double x0 = S.rho_prev, g0 = S.s_prev, x1 = S.sx1, g1 = S.sg1;
        h = (g1 != g0) ? x1 - g1 * (x1 - x0) / (g1 - g0) : x1;
        h = h < 0.0 ? 0.0 : (h > S.h ? S.h : h);
        return true;
    }
    if (cond<UNI>(S.nacc >= K.max_steps)) {
        S.status |= IAT_ST_MAX_STEPS;
        S.done = 1;
        return false;
    }
    h = S.h;
    if (cond<UNI>(h >= K.tau_max - S.tau)) {
        h = K.tau_max - S.tau;
        fin = true;
    }
    if (cond<UNI>(!fin && h < K.hmin)) {
        S.status |= IAT_ST_H_UNDERFLOW;
        S.done = 1;
        return false;
    }
    return true;
}

// What an attempted (or secant) step decided.
enum StepOutcome { OUT_SECANT_CONT = 0, OUT_SECANT_DONE, OUT_REJECT, OUT_NONFINITE, OUT_ACCEPT, OUT_STOP_RFLOOR,
                   OUT_ENTER_EXIT, OUT_TMAX };

// Where a trajectory leaves.  Head-on runs stop when the atom-ion separation crosses r0 outward
// (the ion starts at the centre, so that sphere is the start sphere).  Thermal runs (Fig. 3)
// displace the ion from the centre, so the separation can start above r0 and a grazing atom would
// never cross it from inside; they stop when the atom leaves the sphere of radius r0 about the
// trap centre on which it started.  The choice is a compile-time parameter (CE = centre exit) so
// the head-on kernels carry none of it.
// Exit geometry of CE runs: e = |r_atom|^2 and its rate sign r_atom . v_atom.

// Bookkeeping after a step, shared by both forms.  rho_new, s_new, w2: separation^2, its rate sign
// and the relative speed^2 of the new state; e_prev, e_new, se_new: the exit geometry of the step
// start and of the new state when CE (else the separation is the exit geometry); fin: final step.
// In secant mode only the exit radius of the new state is used.
template <bool CE = false, bool UNI = false>
__device__ __forceinline__ StepOutcome step_epilogue(const StepK& K, Scal& S, const Lane& L, double h, bool fin,
                                                     double en, bool finite, double rho_new, double s_new,
                                                     double w2, double e_prev = 0.0, double e_new = 0.0,
                                                     double se_new = 0.0)
{
    if (cond<UNI>(S.mode != 0)) {
        S.nrhs += 5;
        const double g2 = sqrt(CE ? e_new : rho_new) - K.r0;
        S.rho_prev = S.sx1;
        S.s_prev = S.sg1;
        S.sx1 = h;
        S.sg1 = g2;
        if (cond<UNI>(++S.mode > 4)) {
            S.tau = S.tau + h;
            S.status |= IAT_ST_EXITED;
            S.done = 1;
            return OUT_SECANT_DONE;
        }
        return OUT_SECANT_CONT;
    }
    S.nrhs += 6;
    if (cond<UNI>(!(en <= 1.0))) {
        S.nrej++;
        S.h = h * reject_factor(en);
        S.last_rej = 1;
        return OUT_REJECT;
    }
    S.nacc++;
    if (cond<UNI>(!finite)) {
        S.status |= IAT_ST_NONFINITE;
        S.done = 1;
        return OUT_NONFINITE;
    }
    const double tau_new = fin ? K.tau_max : S.tau + h;
    // bounce: periapsis of the relative motion inside r_b
    if (cond<UNI>(S.s_prev < 0.0 && s_new >= 0.0 && fmin(S.rho_prev, rho_new) < L.rm2 * K.rb_ratio2)) {
        if (S.nb == 0) S.tau_first = tau_new;
        S.tau_last = tau_new;
        S.nb++;
    }
    if (cond<UNI>(bound_state(L, rho_new, w2))) S.status |= IAT_ST_BOUND_SEEN;
    if (cond<UNI>(rho_new < 0.01 * L.rm2)) {   // separation below 0.1 r_m: integration broken
        S.tau = tau_new;
        S.status |= IAT_ST_R_UNDERFLOW;
        S.done = 1;
        return OUT_STOP_RFLOOR;
    }
    const double ex_prev = CE ? e_prev : S.rho_prev, ex_new = CE ? e_new : rho_new;
    if (cond<UNI>(ex_prev <= K.r0sq && ex_new > K.r0sq && (CE ? se_new : s_new) > 0.0)) {
        // keep y_n; the next four steps are secant iterates, (x0, g0) kept in (rho_prev, s_prev)
        S.mode = 1;
        S.s_prev = sqrt(ex_prev) - K.r0;
        S.rho_prev = 0.0;
        S.sx1 = h;
        S.sg1 = sqrt(ex_new) - K.r0;
        S.h = h;
        return OUT_ENTER_EXIT;
    }
    S.tau = tau_new;
    S.rho_prev = rho_new;
    S.s_prev = s_new;
    if (cond<UNI>(fin)) {
        S.status |= IAT_ST_TMAX;
        S.done = 1;
        S.h = h;
        return OUT_TMAX;
    }
    S.h = fmin(K.hmax, h * step_factor(en, S.last_rej != 0));
    S.last_rej = 0;
    return OUT_ACCEPT;
}

// ---------------------------------------------------------------------------------------
// One lane per trajectory.
// ---------------------------------------------------------------------------------------
struct Traj1 {
    double x[6], v[6], F1[6];   // r_atom, r_ion ; v_atom, v_ion ; accelerations at y_n
    Scal S;
    Lane L;
};

__device__ __forceinline__ void accel1(const KParams& P, const Lane& L, double cs, const double X[6], double A[6])
{
    const double d0 = X[0] - X[3], d1 = X[1] - X[4], d2 = X[2] - X[5];
    const double s = force_scale(L, d0, d1, d2);
    const double qc = L.qx_half * cs;
    A[0] = acc_atom(L, s, d0);
    A[1] = acc_atom(L, s, d1);
    A[2] = acc_atom(L, s, d2);
    A[3] = acc_ion(P.inv_mi, s, d0, P.kA[0], qc, P.q_ratio[0], X[3]);
    A[4] = acc_ion(P.inv_mi, s, d1, P.kA[1], qc, P.q_ratio[1], X[4]);
    A[5] = acc_ion(P.inv_mi, s, d2, P.kA[2], qc, P.q_ratio[2], X[5]);
}

// Runs once per trajectory.
// ---------------------------------------------------------------------------------------
// Per-call work buffer, structure of arrays over the n trajectories of a call:
//   D[0..11]  internal state x[6] (r_atom, r_ion), v[6] (v_atom, v_ion): the start state on
//             entry to the integration kernels, the final state on exit
//   D[12..18] lane constants (inv_ma, c8x8, c4x4, qx_half, phase0, rm2, half_mu)
//   D[19..21] tau, tau_first, tau_last (final)
//   I[0..4]   nacc, nrej, nrhs, n_bounce, status
// A setup kernel fills the start, the integration kernels only load, step and store, and an
// observables kernel turns the final state into the outputs, so the step loops carry nothing
// but the step.
// ---------------------------------------------------------------------------------------
struct Work {
    double* D;
    int32_t* I;
    int64_t n;
    __device__ __forceinline__ double& d(int f, int64_t i) const { return D[(int64_t)f * n + i]; }
    __device__ __forceinline__ int32_t& k(int f, int64_t i) const { return I[(int64_t)f * n + i]; }
};
constexpr int kWorkDoubles = 22, kWorkInts = 5;

__device__ inline void work_setup(const KParams& P, const Work& W, int64_t i)
{
    TrajParams tp;
    traj_params(P, i, tp);
    Lane L;
    lane_consts(P, tp, L);
    double y[12];
    start_state_au(P, i, tp, y);
    for (int k = 0; k < 6; ++k) {
        W.d(k, i) = y[k];
        W.d(6 + k, i) = y[6 + k] / P.omega;
    }
    W.d(12, i) = L.inv_ma;
    W.d(13, i) = L.c8x8;
    W.d(14, i) = L.c4x4;
    W.d(15, i) = L.qx_half;
    W.d(16, i) = L.phase0;
    W.d(17, i) = L.rm2;
    W.d(18, i) = L.half_mu;
    W.k(4, i) = (int32_t)(warn_r0(P, tp, y) ? IAT_ST_WARN_R0 : 0u);
}

__device__ __forceinline__ void work_lane(const Work& W, int64_t i, Lane& L)
{
    L.inv_ma = W.d(12, i);
    L.c8x8 = W.d(13, i);
    L.c4x4 = W.d(14, i);
    L.qx_half = W.d(15, i);
    L.phase0 = W.d(16, i);
    L.rm2 = W.d(17, i);
    L.half_mu = W.d(18, i);
}

__device__ __forceinline__ void work_store_scal(const Work& W, int64_t i, const Scal& S)
{
    W.d(19, i) = S.tau;
    W.d(20, i) = S.tau_first;
    W.d(21, i) = S.tau_last;
    W.k(0, i) = S.nacc;
    W.k(1, i) = S.nrej;
    W.k(2, i) = S.nrhs;
    W.k(3, i) = S.nb;
    W.k(4, i) = (int32_t)S.status;
}

__device__ inline void traj1_start(const KParams& P, const Work& W, int64_t i, Traj1& T)
{
    work_lane(W, i, T.L);
    scal_init(P, T.S);
    T.S.status = (uint32_t)W.k(4, i);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        T.x[k] = W.d(k, i);
        T.v[k] = W.d(6 + k, i);
        fin = fin && is_finite(T.x[k]) && is_finite(T.v[k]);
    }
    if (!fin) {
        T.S.status |= IAT_ST_NONFINITE;
        T.S.done = 1;
        return;
    }
    double s0, c0;
    phase_sincos(T.L.phase0, s0, c0);
    accel1(P, T.L, c0, T.x, T.F1);
    T.S.nrhs = 1;
    const double d0 = T.x[0] - T.x[3], d1 = T.x[1] - T.x[4], d2 = T.x[2] - T.x[5];
    T.S.rho_prev = dot3(d0, d1, d2, d0, d1, d2);
    T.S.s_prev = dot3(d0, d1, d2, T.v[0] - T.v[3], T.v[1] - T.v[4], T.v[2] - T.v[5]);
}

__device__ __forceinline__ void traj1_store(const Work& W, int64_t i, const Traj1& T)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        W.d(k, i) = T.x[k];
        W.d(6 + k, i) = T.v[k];
    }
    work_store_scal(W, i, T.S);
}

// One attempted step (or secant iterate) of a one-lane trajectory.
template <bool CE = false>
__device__ __forceinline__ void traj1_advance(const KParams& P, Traj1& T)
{
    const StepK K = step_k(P);
    double h;
    bool fin;
    if (!step_prologue(K, T.S, h, fin)) return;
    const bool exiting = T.S.mode != 0;
    const double hh = h * h;
    const StageCos C = stage_cos(T.S.tau, T.L.phase0, h);
    double F2[6], F3[6], F4[6], F5[6], F6[6], X[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = stage2(T.x[k], T.v[k], h);
    accel1(P, T.L, C.c2, X, F2);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = stage3(T.x[k], T.v[k], h, hh, T.F1[k]);
    accel1(P, T.L, C.c3, X, F3);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = stage4(T.x[k], T.v[k], h, hh, T.F1[k], F2[k]);
    accel1(P, T.L, C.c4, X, F4);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = stage5(T.x[k], T.v[k], h, hh, T.F1[k], F2[k], F3[k]);
    accel1(P, T.L, C.c5, X, F5);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = stage6(T.x[k], T.v[k], h, hh, T.F1[k], F2[k], F3[k], F4[k]);
    accel1(P, T.L, C.c6, X, F6);
    double x5[6], v5[6], ex[6], F7[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        x5[k] = sol_x(T.x[k], T.v[k], h, hh, T.F1[k], F2[k], F3[k], F4[k], F5[k]);
        v5[k] = sol_v(T.v[k], h, T.F1[k], F3[k], F4[k], F5[k], F6[k]);
        ex[k] = err_x(hh, T.F1[k], F2[k], F3[k], F4[k], F5[k], F6[k]);
    }
    double en = 0.0;
    bool finite = true;
    if (!exiting) {
        accel1(P, T.L, C.c6, x5, F7);
        bool bad = false;
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double ev = err_v(h, T.F1[k], F3[k], F4[k], F5[k], F6[k], F7[k]);
            const double rx = err_ratio(ex[k], T.x[k], x5[k], K.rtol, K.atol);
            const double rv = err_ratio(ev, T.v[k], v5[k], K.rtol, K.atol);
            bad = bad || ratio_bad(rx) || ratio_bad(rv);
            m = fmax(m, fmax(rx, rv));
            finite = finite && is_finite(x5[k]) && is_finite(v5[k]);
        }
        en = bad ? __builtin_nan("") : m;
    }
    const double d0 = x5[0] - x5[3], d1 = x5[1] - x5[4], d2 = x5[2] - x5[5];
    const double w0 = v5[0] - v5[3], w1 = v5[1] - v5[4], w2 = v5[2] - v5[5];
    const double rho_new = dot3(d0, d1, d2, d0, d1, d2);
    const double s_new = dot3(d0, d1, d2, w0, w1, w2);
    const double ww = dot3(w0, w1, w2, w0, w1, w2);
    double e_prev = 0.0, e_new = 0.0, se_new = 0.0;
    if (CE) {
        e_prev = dot3(T.x[0], T.x[1], T.x[2], T.x[0], T.x[1], T.x[2]);
        e_new = dot3(x5[0], x5[1], x5[2], x5[0], x5[1], x5[2]);
        se_new = dot3(x5[0], x5[1], x5[2], v5[0], v5[1], v5[2]);
    }
    const StepOutcome o = step_epilogue<CE>(K, T.S, T.L, h, fin, en, finite, rho_new, s_new, ww, e_prev, e_new, se_new);
    if (o == OUT_SECANT_DONE || o == OUT_STOP_RFLOOR) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            T.x[k] = x5[k];
            T.v[k] = v5[k];
        }
    } else if (o == OUT_ACCEPT || o == OUT_TMAX) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            T.x[k] = x5[k];
            T.v[k] = v5[k];
            T.F1[k] = F7[k];
        }
    }
}

// ---------------------------------------------------------------------------------------
// Four lanes per trajectory: lane k = 0, 1, 2 of an aligned quad holds axis k (atom and ion
// position, velocity and stage accelerations); lane 3 shadows axis 2.  Values shared across
// axes (separation, radial rate, error norm) are gathered with quad DPP moves and evaluated
// with the same expressions as the one-lane form, so both give the same bits.  Every branch
// depends on quad-uniform values only, so the four lanes of a quad stay converged.
// ---------------------------------------------------------------------------------------
// Lane SRC of each quad to the whole quad: two 32-bit quad-permute moves.  ROW: the caller's quad is
// lanes 0-3 and the only live lanes of its row of 16 (one trajectory per wave), so the row
// broadcast of lane SRC does the same in one 64-bit move.
template <int SRC, bool ROW = false>
__device__ __forceinline__ double quad_bcast(double v)
{
    if constexpr (ROW) {
        const int64_t x = __builtin_bit_cast(int64_t, v);
        const int64_t y = __builtin_amdgcn_mov_dpp(x, 0x150 + SRC, 0xF, 0xF, false);
        return __builtin_bit_cast(double, y);
    } else {
        constexpr int ctrl = SRC | (SRC << 2) | (SRC << 4) | (SRC << 6);
        const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
        return __hiloint2double(hi, lo);
    }
}
__device__ __forceinline__ double quad_max(double v)
{
    constexpr int x1 = 1 | (0 << 2) | (3 << 4) | (2 << 6), x2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
    double o = __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), x1, 0xF, 0xF, false),
                                __builtin_amdgcn_mov_dpp(__double2loint(v), x1, 0xF, 0xF, false));
    v = fmax(v, o);
    o = __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), x2, 0xF, 0xF, false),
                         __builtin_amdgcn_mov_dpp(__double2loint(v), x2, 0xF, 0xF, false));
    return fmax(v, o);
}
__device__ __forceinline__ int quad_or(int v)
{
    constexpr int x1 = 1 | (0 << 2) | (3 << 4) | (2 << 6), x2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
    v |= __builtin_amdgcn_mov_dpp(v, x1, 0xF, 0xF, false);
    return v | __builtin_amdgcn_mov_dpp(v, x2, 0xF, 0xF, false);
}

// Stage cosines for the four-lane form: the values of stage_cos, with its six polynomial
// evaluations (the phase remainder and the five stage offsets) shared out over the quad's lanes
// in two rounds and gathered with quad moves.

template <bool ROW = false>
__device__ __forceinline__ StageCos stage_cos4q(double tau, double phase0, double h, bool l0, double cl, double cl2)
{
    double k;
    const double r = phase_reduce(tau + phase0, k);
    // every lane reduces the phase: without this the compiler moves the reduction into a branch taken
    // by lane 0 alone, and a quad then runs the lane cases one after another
    asm volatile("" ::"v"(r));
    const double a1 = l0 ? r : cl * h;
    const double a2 = cl2 * h;
    double cA, sA, cB, sB;
    small_sincos(a1, cA, sA);
    small_sincos(a2, cB, sB);
    double sb, cb;
    phase_quadrant(k, quad_bcast<0, ROW>(cA), quad_bcast<0, ROW>(sA), sb, cb);
    StageCos C;
    C.c2 = cos_comb(cb, sb, quad_bcast<1, ROW>(cA), quad_bcast<1, ROW>(sA));
    C.c3 = cos_comb(cb, sb, quad_bcast<2, ROW>(cA), quad_bcast<2, ROW>(sA));
    C.c4 = cos_comb(cb, sb, quad_bcast<3, ROW>(cA), quad_bcast<3, ROW>(sA));
    C.c5 = cos_comb(cb, sb, quad_bcast<0, ROW>(cB), quad_bcast<0, ROW>(sB));
    C.c6 = cos_comb(cb, sb, quad_bcast<1, ROW>(cB), quad_bcast<1, ROW>(sB));
    return C;
}

template <bool ROW = false>
__device__ __forceinline__ StageCos stage_cos4(double tau, double phase0, double h, const Tab& T = kTab)
{
    // per-lane offset coefficients, so each argument is one product: a1 = c_l h (lanes 1..3, lane 0
    // takes the phase remainder), a2 = c5 h (lanes 0, 2) or 1.0 h = h (lanes 1, 3)
    const int l = __lane_id() & 3;
    const double cl = l == 1 ? T.c2 : (l == 2 ? T.c3 : T.c4);
    const double cl2 = (l & 1) ? 1.0 : T.c5;
    return stage_cos4q<ROW>(tau, phase0, h, l == 0, cl, cl2);
}

struct Traj4 {
    double xa, xi, va, vi, F1a, F1i;   // this lane's axis
    Scal S;
    Lane L;
};

// Per-lane constants of the four-lane form.  A kernel that steps many times computes them once and
// holds them in registers (quad_consts<true>); evaluated at each use, the compiler may turn their
// lane-dependent selects into a table in private memory.
struct Quad4 {
    int k;            // this lane's axis (lane 3 shadows axis 2)
    bool l0;          // lane 0: evaluates the series of the phase remainder
    double kA, qr;    // a_k / 4 and q_k / q_x of the axis
    double cl, cl2;   // stage-cosine offsets of the lane's two series: c2, c3, c4 (lanes 1..3) and c5 or 1
};
template <bool PIN>
__device__ __forceinline__ Quad4 quad_consts(const KParams& P, const Tab& T)
{
    const int l = __lane_id() & 3;
    Quad4 Q;
    Q.k = min(l, 2);
    Q.l0 = l == 0;
    Q.kA = Q.k == 0 ? P.kA[0] : (Q.k == 1 ? P.kA[1] : P.kA[2]);
    Q.qr = Q.k == 0 ? P.q_ratio[0] : (Q.k == 1 ? P.q_ratio[1] : P.q_ratio[2]);
    Q.cl = l == 1 ? T.c2 : (l == 2 ? T.c3 : T.c4);
    Q.cl2 = (l & 1) ? 1.0 : T.c5;
    if (PIN) asm volatile("" : "+v"(Q.kA), "+v"(Q.qr), "+v"(Q.cl), "+v"(Q.cl2));
    return Q;
}

__device__ __forceinline__ int quad_axis() { return min((int)(__lane_id() & 3), 2); }

template <bool ROW = false>
__device__ __forceinline__ void accel4q(const KParams& P, const Lane& L, double kA, double qr, double cs, double Xa,
                                        double Xi, double& Aa, double& Ai)
{
    const double dk = Xa - Xi;
    const double d0 = quad_bcast<0, ROW>(dk), d1 = quad_bcast<1, ROW>(dk), d2 = quad_bcast<2, ROW>(dk);
    const double s = force_scale(L, d0, d1, d2);
    const double qc = L.qx_half * cs;
    Aa = acc_atom(L, s, dk);
    Ai = acc_ion(P.inv_mi, s, dk, kA, qc, qr, Xi);
}
template <bool ROW = false>
__device__ __forceinline__ void accel4(const KParams& P, const Lane& L, int k, double cs, double Xa, double Xi,
                                       double& Aa, double& Ai)
{
    const double kA = k == 0 ? P.kA[0] : (k == 1 ? P.kA[1] : P.kA[2]);
    const double qr = k == 0 ? P.q_ratio[0] : (k == 1 ? P.q_ratio[1] : P.q_ratio[2]);
    accel4q<ROW>(P, L, kA, qr, cs, Xa, Xi, Aa, Ai);
}

// Start of a four-lane trajectory from the work buffer (same bits as traj1_start).
__device__ inline void traj4_start(const KParams& P, const Work& W, int64_t i, Traj4& T)
{
    const int k = quad_axis();
    work_lane(W, i, T.L);
    scal_init(P, T.S);
    T.S.status = (uint32_t)W.k(4, i);
    T.xa = W.d(k, i);
    T.xi = W.d(3 + k, i);
    T.va = W.d(6 + k, i);
    T.vi = W.d(9 + k, i);
    T.F1a = T.F1i = 0.0;
    const int nonfin = quad_or((is_finite(T.xa) && is_finite(T.xi) && is_finite(T.va) && is_finite(T.vi)) ? 0 : 1);
    if (nonfin) {
        T.S.status |= IAT_ST_NONFINITE;
        T.S.done = 1;
        return;
    }
    double s0, c0;
    phase_sincos(T.L.phase0, s0, c0);
    accel4(P, T.L, k, c0, T.xa, T.xi, T.F1a, T.F1i);
    T.S.nrhs = 1;
    const double dk = T.xa - T.xi, wk = T.va - T.vi;
    const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
    const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
    T.S.rho_prev = dot3(d0, d1, d2, d0, d1, d2);
    T.S.s_prev = dot3(d0, d1, d2, w0, w1, w2);
}

// Everything a step of the four-lane form computes before its bookkeeping (the four-lane counterpart of
// Step8): this lane's axis of the fifth-order state and of the FSAL acceleration, the error norm and the
// geometry of the new state.
struct Step4 {
    double x5a, x5i, v5a, v5i, F7a, F7i, en;
    bool finite;
    double rho_new, s_new, ww, e_prev, e_new, se_new;
};
template <bool CE, bool ROW>
__device__ __forceinline__ Step4 traj4_trial(const KParams& P, const StepK& K, const Traj4& T, const Tab& B,
                                             const Quad4& Q, double h, bool exiting)
{
    const double hh = h * h;
    const StageCos C = stage_cos4q<ROW>(T.S.tau, T.L.phase0, h, Q.l0, Q.cl, Q.cl2);
    double F2a, F2i, F3a, F3i, F4a, F4i, F5a, F5i, F6a, F6i;
    accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c2, stage2(T.xa, T.va, h, B), stage2(T.xi, T.vi, h, B), F2a, F2i);
    accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c3, stage3(T.xa, T.va, h, hh, T.F1a, B), stage3(T.xi, T.vi, h, hh, T.F1i, B), F3a, F3i);
    accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c4, stage4(T.xa, T.va, h, hh, T.F1a, F2a, B), stage4(T.xi, T.vi, h, hh, T.F1i, F2i, B), F4a,
           F4i);
    accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c5, stage5(T.xa, T.va, h, hh, T.F1a, F2a, F3a, B),
           stage5(T.xi, T.vi, h, hh, T.F1i, F2i, F3i, B), F5a, F5i);
    accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c6, stage6(T.xa, T.va, h, hh, T.F1a, F2a, F3a, F4a, B),
           stage6(T.xi, T.vi, h, hh, T.F1i, F2i, F3i, F4i, B), F6a, F6i);
    Step4 R;
    R.x5a = sol_x(T.xa, T.va, h, hh, T.F1a, F2a, F3a, F4a, F5a, B);
    R.x5i = sol_x(T.xi, T.vi, h, hh, T.F1i, F2i, F3i, F4i, F5i, B);
    R.v5a = sol_v(T.va, h, T.F1a, F3a, F4a, F5a, F6a, B);
    R.v5i = sol_v(T.vi, h, T.F1i, F3i, F4i, F5i, F6i, B);
    R.en = 0.0;
    R.F7a = R.F7i = 0.0;
    R.finite = true;
    if (!exiting) {
        accel4q<ROW>(P, T.L, Q.kA, Q.qr, C.c6, R.x5a, R.x5i, R.F7a, R.F7i);
        const double ra = err_ratio(err_x(hh, T.F1a, F2a, F3a, F4a, F5a, F6a, B), T.xa, R.x5a, K.rtol, K.atol);
        const double ri = err_ratio(err_x(hh, T.F1i, F2i, F3i, F4i, F5i, F6i, B), T.xi, R.x5i, K.rtol, K.atol);
        const double rva = err_ratio(err_v(h, T.F1a, F3a, F4a, F5a, F6a, R.F7a, B), T.va, R.v5a, K.rtol, K.atol);
        const double rvi = err_ratio(err_v(h, T.F1i, F3i, F4i, F5i, F6i, R.F7i, B), T.vi, R.v5i, K.rtol, K.atol);
        const int bad = quad_or((ratio_bad(ra) || ratio_bad(ri) || ratio_bad(rva) || ratio_bad(rvi)) ? 1 : 0);
        const int nonfin =
            quad_or((is_finite(R.x5a) && is_finite(R.x5i) && is_finite(R.v5a) && is_finite(R.v5i)) ? 0 : 1);
        const double m = quad_max(fmax(fmax(ra, rva), fmax(ri, rvi)));
        R.en = bad ? __builtin_nan("") : m;
        R.finite = nonfin == 0;
    }
    const double dk = R.x5a - R.x5i, wk = R.v5a - R.v5i;
    const double d0 = quad_bcast<0, ROW>(dk), d1 = quad_bcast<1, ROW>(dk), d2 = quad_bcast<2, ROW>(dk);
    const double w0 = quad_bcast<0, ROW>(wk), w1 = quad_bcast<1, ROW>(wk), w2 = quad_bcast<2, ROW>(wk);
    R.rho_new = dot3(d0, d1, d2, d0, d1, d2);
    R.s_new = dot3(d0, d1, d2, w0, w1, w2);
    R.ww = dot3(w0, w1, w2, w0, w1, w2);
    R.e_prev = R.e_new = R.se_new = 0.0;
    if (CE) {
        const double p0 = quad_bcast<0, ROW>(T.xa), p1 = quad_bcast<1, ROW>(T.xa), p2 = quad_bcast<2, ROW>(T.xa);
        const double a0 = quad_bcast<0, ROW>(R.x5a), a1 = quad_bcast<1, ROW>(R.x5a), a2 = quad_bcast<2, ROW>(R.x5a);
        const double u0 = quad_bcast<0, ROW>(R.v5a), u1 = quad_bcast<1, ROW>(R.v5a), u2 = quad_bcast<2, ROW>(R.v5a);
        R.e_prev = dot3(p0, p1, p2, p0, p1, p2);
        R.e_new = dot3(a0, a1, a2, a0, a1, a2);
        R.se_new = dot3(a0, a1, a2, u0, u1, u2);
    }
    return R;
}

// Bookkeeping of the four-lane form: the shared epilogue and the state update it decides.
template <bool CE>
__device__ __forceinline__ StepOutcome traj4_finish(const StepK& K, Traj4& T, double h, bool fin, const Step4& R)
{
    const StepOutcome o = step_epilogue<CE>(K, T.S, T.L, h, fin, R.en, R.finite, R.rho_new, R.s_new, R.ww, R.e_prev,
                                            R.e_new, R.se_new);
    // selects, not branches: with branches the compiler keeps R in private memory
    const bool fsal = o == OUT_ACCEPT || o == OUT_TMAX;
    const bool moved = fsal || o == OUT_SECANT_DONE || o == OUT_STOP_RFLOOR;
    T.xa = moved ? R.x5a : T.xa;
    T.xi = moved ? R.x5i : T.xi;
    T.va = moved ? R.v5a : T.va;
    T.vi = moved ? R.v5i : T.vi;
    T.F1a = fsal ? R.F7a : T.F1a;
    T.F1i = fsal ? R.F7i : T.F1i;
    return o;
}

// One attempted step of the four-lane form.  Returns the StepOutcome, or -1 when the trajectory
// stopped before stepping (step cap, step underflow); h_used receives the step size tried.
template <bool CE = false, bool ROW = false>
__device__ __forceinline__ int traj4_step_k(const KParams& P, const StepK& K, Traj4& T, double& h_used,
                                            const Tab& B)
{
    double h;
    bool fin;
    h_used = 0.0;
    if (!step_prologue(K, T.S, h, fin)) return -1;
    h_used = h;
    const Step4 R = traj4_trial<CE, ROW>(P, K, T, B, quad_consts<false>(P, B), h, T.S.mode != 0);
    return (int)traj4_finish<CE>(K, T, h, fin, R);
}

template <bool CE = false>
__device__ __forceinline__ int traj4_step(const KParams& P, Traj4& T, double& h_used, const Tab& B = kTab)
{
    return traj4_step_k<CE>(P, step_k(P), T, h_used, B);
}

template <bool CE = false>
__device__ __forceinline__ void traj4_advance(const KParams& P, Traj4& T, const Tab& B = kTab)
{
    double h;
    (void)traj4_step<CE>(P, T, h, B);
}
template <bool CE = false, bool ROW = false>
__device__ __forceinline__ void traj4_advance_k(const KParams& P, const StepK& K, Traj4& T, const Tab& B)
{
    double h;
    (void)traj4_step_k<CE, ROW>(P, K, T, h, B);
}

// One step of the four-lane form for the lanes that call it (every quad of them a running trajectory),
// the common cases first.  When every calling quad is on an ordinary step (stepping mode, under the step
// cap, not the final step, h above its floor) and none of them, once the step is tried, is accepted with
// an event (periapsis inside r_b, separation floor, exit crossing, non-finite state), each quad is either
// accepted or rejected with the plain updates of step_epilogue for those cases.  Otherwise every calling
// quad takes the general path (the same step, the same bits).
template <bool CE = false>
__device__ __forceinline__ void traj4_step_fast(const KParams& P, const StepK& K, Traj4& T, const Tab& B,
                                                const Quad4& Q)
{
    Scal& S = T.S;
    const bool plain = (S.mode == 0) & (S.nacc < K.max_steps) & !(S.h >= K.tau_max - S.tau) & !(S.h < K.hmin);
    bool general = __builtin_amdgcn_ballot_w64(!plain) != 0;
    double h = S.h;
    bool fin = false;
    if (general && !step_prologue(K, S, h, fin)) return;
    const Step4 R = traj4_trial<CE, false>(P, K, T, B, Q, h, S.mode != 0);
    const bool acc = R.en <= 1.0;
    if (!general) {
        const double ex_prev = CE ? R.e_prev : S.rho_prev, ex_new = CE ? R.e_new : R.rho_new;
        const bool bounce =
            (S.s_prev < 0.0) & (R.s_new >= 0.0) & (fmin(S.rho_prev, R.rho_new) < T.L.rm2 * K.rb_ratio2);
        const bool floor = R.rho_new < 0.01 * T.L.rm2;
        const bool crossing = (ex_prev <= K.r0sq) & (ex_new > K.r0sq) & ((CE ? R.se_new : R.s_new) > 0.0);
        general = __builtin_amdgcn_ballot_w64(acc & (!R.finite | bounce | floor | crossing)) != 0;
    }
    if (general) {
        (void)traj4_finish<CE>(K, T, h, fin, R);
        return;
    }
    S.nrhs += 6;
    // both step factors before the branch, so that they share the one root of en
    const double h_acc = fmin(K.hmax, h * step_factor(R.en, S.last_rej != 0));
    const double h_rej = h * reject_factor(R.en);
    if (acc) {
        S.nacc++;
        S.status |= bound_state(T.L, R.rho_new, R.ww) ? (uint32_t)IAT_ST_BOUND_SEEN : 0u;
        S.tau = S.tau + h;
        S.rho_prev = R.rho_new;
        S.s_prev = R.s_new;
        S.h = h_acc;
        S.last_rej = 0;
        T.xa = R.x5a;
        T.xi = R.x5i;
        T.va = R.v5a;
        T.vi = R.v5i;
        T.F1a = R.F7a;
        T.F1i = R.F7i;
    } else {
        S.nrej++;
        S.h = h_rej;
        S.last_rej = 1;
    }
}

// ---------------------------------------------------------------------------------------
// Outputs.
// ---------------------------------------------------------------------------------------
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

// Observables of trajectory i from its final state in the work buffer (outputs in a.u.).
__device__ inline void work_observe(const KParams& P, const Work& W, int64_t i)
{
    TrajParams tp;
    traj_params(P, i, tp);
    double y0[12];
    start_state_au(P, i, tp, y0);
    double yf[12];
    for (int k = 0; k < 6; ++k) {
        yf[k] = W.d(k, i);
        yf[6 + k] = W.d(6 + k, i) * P.omega;
    }
    const double tau = W.d(19, i);
    const int32_t nb = W.k(3, i);
    uint32_t st = (uint32_t)W.k(4, i);
    if (nb >= 2 || (st & IAT_ST_TMAX)) st |= IAT_ST_COMPLEX;
    const double* vi = y0 + 6;
    const double* vf = yf + 6;
    const double cx = vi[1] * vf[2] - vi[2] * vf[1];
    const double cy = vi[2] * vf[0] - vi[0] * vf[2];
    const double cz = vi[0] * vf[1] - vi[1] * vf[0];
    const double dot = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
    P.angle[i] = atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
    const double dv0 = vf[0] - vi[0], dv1 = vf[1] - vi[1], dv2 = vf[2] - vi[2];
    P.q_transfer[i] = species_mass(P, tp.sp) * sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
    P.dE_ion[i] = ion_energy_au(P, tp.qx, tp.phase0, yf, tau) - ion_energy_au(P, tp.qx, tp.phase0, y0, 0.0);
    const double inv_w = 1.0 / P.omega;
    P.t_dwell[i] = tau * inv_w;
    if (P.t_first) P.t_first[i] = W.d(20, i) * inv_w;
    if (P.t_last) P.t_last[i] = W.d(21, i) * inv_w;
    P.n_bounce[i] = nb;
    P.status[i] = st;
    if (P.n_accept) P.n_accept[i] = W.k(0, i);
    if (P.n_reject) P.n_reject[i] = W.k(1, i);
    if (P.n_rhs) P.n_rhs[i] = W.k(2, i);
    if (P.y_final) {
        for (int k = 0; k < 12; ++k) P.y_final[(int64_t)k * P.n + i] = yf[k];
    }
}

// ---------------------------------------------------------------------------------------
// Suspended trajectories (continuation records), structure of arrays of capacity cap:
// doubles [26][cap]: x[6], v[6], F1[6], tau, h, rho_prev, s_prev, sx1, sg1, tau_first, tau_last;
// int32 [8][cap]: nacc, nrej, nrhs, nb, status, mode, last_rej, (pad); int64 [cap]: id.
// ---------------------------------------------------------------------------------------
struct Cont {
    double* d;
    int32_t* n;
    int64_t* id;
    int64_t cap;
    unsigned long long* count;   // records written
    unsigned long long* head;    // records taken by the resuming kernel
};

__device__ inline void cont_save(const Cont& C, int64_t slot, int64_t i, const Traj1& T)
{
    const int64_t c = C.cap;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        C.d[(0 + k) * c + slot] = T.x[k];
        C.d[(6 + k) * c + slot] = T.v[k];
        C.d[(12 + k) * c + slot] = T.F1[k];
    }
    const Scal& S = T.S;
    C.d[18 * c + slot] = S.tau;
    C.d[19 * c + slot] = S.h;
    C.d[20 * c + slot] = S.rho_prev;
    C.d[21 * c + slot] = S.s_prev;
    C.d[22 * c + slot] = S.sx1;
    C.d[23 * c + slot] = S.sg1;
    C.d[24 * c + slot] = S.tau_first;
    C.d[25 * c + slot] = S.tau_last;
    C.n[0 * c + slot] = S.nacc;
    C.n[1 * c + slot] = S.nrej;
    C.n[2 * c + slot] = S.nrhs;
    C.n[3 * c + slot] = S.nb;
    C.n[4 * c + slot] = (int32_t)S.status;
    C.n[5 * c + slot] = (int32_t)S.mode;
    C.n[6 * c + slot] = S.last_rej;
    C.id[slot] = i;
}

__device__ inline void cont_load4(const KParams& P, const Work& W, const Cont& C, int64_t slot, int k, Traj4& T,
                                  int64_t& i)
{
    const int64_t c = C.cap;
    i = C.id[slot];
    (void)P;
    T.xa = C.d[(0 + k) * c + slot];
    T.xi = C.d[(3 + k) * c + slot];
    T.va = C.d[(6 + k) * c + slot];
    T.vi = C.d[(9 + k) * c + slot];
    T.F1a = C.d[(12 + k) * c + slot];
    T.F1i = C.d[(15 + k) * c + slot];
    Scal& S = T.S;
    S.tau = C.d[18 * c + slot];
    S.h = C.d[19 * c + slot];
    S.rho_prev = C.d[20 * c + slot];
    S.s_prev = C.d[21 * c + slot];
    S.sx1 = C.d[22 * c + slot];
    S.sg1 = C.d[23 * c + slot];
    S.tau_first = C.d[24 * c + slot];
    S.tau_last = C.d[25 * c + slot];
    S.nacc = C.n[0 * c + slot];
    S.nrej = C.n[1 * c + slot];
    S.nrhs = C.n[2 * c + slot];
    S.nb = C.n[3 * c + slot];
    S.status = (uint32_t)C.n[4 * c + slot];
    S.mode = (uint32_t)C.n[5 * c + slot];
    S.last_rej = C.n[6 * c + slot];
    S.done = 0;
    work_lane(W, i, T.L);
}

// The record of a four-lane trajectory (the layout of cont_save): lanes 0..2 of the quad write
// their axis, lane 0 the scalar state and the id.
__device__ inline void cont_save4(const Cont& C, int64_t slot, int64_t i, const Traj4& T, int lane_in_quad)
{
    const int64_t c = C.cap;
    if (lane_in_quad < 3) {
        const int k = lane_in_quad;
        C.d[(0 + k) * c + slot] = T.xa;
        C.d[(3 + k) * c + slot] = T.xi;
        C.d[(6 + k) * c + slot] = T.va;
        C.d[(9 + k) * c + slot] = T.vi;
        C.d[(12 + k) * c + slot] = T.F1a;
        C.d[(15 + k) * c + slot] = T.F1i;
    }
    if (lane_in_quad != 0) return;
    const Scal& S = T.S;
    C.d[18 * c + slot] = S.tau;
    C.d[19 * c + slot] = S.h;
    C.d[20 * c + slot] = S.rho_prev;
    C.d[21 * c + slot] = S.s_prev;
    C.d[22 * c + slot] = S.sx1;
    C.d[23 * c + slot] = S.sg1;
    C.d[24 * c + slot] = S.tau_first;
    C.d[25 * c + slot] = S.tau_last;
    C.n[0 * c + slot] = S.nacc;
    C.n[1 * c + slot] = S.nrej;
    C.n[2 * c + slot] = S.nrhs;
    C.n[3 * c + slot] = S.nb;
    C.n[4 * c + slot] = (int32_t)S.status;
    C.n[5 * c + slot] = (int32_t)S.mode;
    C.n[6 * c + slot] = S.last_rej;
    C.id[slot] = i;
}

__device__ __forceinline__ void traj4_store(const Work& W, int64_t i, const Traj4& T, int lane_in_quad)
{
    if (lane_in_quad < 3) {
        W.d(lane_in_quad, i) = T.xa;
        W.d(3 + lane_in_quad, i) = T.xi;
        W.d(6 + lane_in_quad, i) = T.va;
        W.d(9 + lane_in_quad, i) = T.vi;
    }
    if (lane_in_quad == 0) work_store_scal(W, i, T.S);
}

// ---------------------------------------------------------------------------------------
// Eight lanes per trajectory, for the solo level (one trajectory per wave).  Lanes 0, 1, 2 of the
// octet hold the atom's coordinate 0, 1, 2 and lanes 7, 6, 5 the ion's, so that the half-row mirror
// pairs every lane with the same axis of the other body; lanes 3 and 4 shadow axis 2.  The ion lanes
// keep their position, velocity and accelerations negated: the separation d_k = X_atom,k - X_ion,k is
// then the sum of a lane's value and its partner's in every lane (negation is exact, so the sum rounds
// as the difference does in the other forms).  Each lane carries one coordinate, so the stage sums,
// the fifth-order solution and the error estimate take half the instructions of the four-lane form,
// and the six small-angle series of the stage cosines run in one round; every value is formed by the
// same expression as in the other forms, so the bits are the same.
// ---------------------------------------------------------------------------------------
struct Traj8 {
    double x, v, F1;   // this lane's coordinate (negated on ion lanes)
    double m;          // this lane's inverse mass: 1/m_a on atom lanes, 1/m_i on ion lanes
    Scal S;
    Lane L;
};

__device__ __forceinline__ int oct_lane() { return (int)(__lane_id() & 7); }
__device__ __forceinline__ bool oct_atom() { return oct_lane() < 4; }
__device__ __forceinline__ int oct_axis()
{
    const int l = oct_lane();
    return l < 4 ? min(l, 2) : min(7 - l, 2);
}

// the other body's same axis: lane 7 - l of the half row (two 32-bit half-row-mirror moves)
__device__ __forceinline__ double oct_partner(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x141, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x141, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// max(a, b) as the one instruction, for operands that are never NaN: fmax first quiets a signalling NaN
// in an operand that a lane move brought in, one more instruction per such operand.
__device__ __forceinline__ double max_num(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// Maximum over the octet of values that are never NaN.
__device__ __forceinline__ double oct_max(double v)
{
    constexpr int x1 = 1 | (0 << 2) | (3 << 4) | (2 << 6), x2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
    v = max_num(v, oct_partner(v));
    v = max_num(v, __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), x1, 0xF, 0xF, false),
                                    __builtin_amdgcn_mov_dpp(__double2loint(v), x1, 0xF, 0xF, false)));
    return max_num(v, __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), x2, 0xF, 0xF, false),
                                       __builtin_amdgcn_mov_dpp(__double2loint(v), x2, 0xF, 0xF, false)));
}
__device__ __forceinline__ int oct_or(int v)
{
    return quad_or(v | __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
}

// Per-lane constants of the eight-lane form, set once per kernel and held in registers.
struct Oct {
    bool atom;        // lanes 0..3: the atom's side of the half-row mirror
    bool l0;          // lane 0: evaluates the series of the phase remainder
    double kA, qr;    // ion lanes, axis k: a_k / 4 and q_k / q_x; +0 on atom lanes
    double cl;        // lanes 1..5: the offset coefficient c2, c3, c4, c5, 1 of this lane's stage series
};
__device__ __forceinline__ Oct oct_consts(const KParams& P, const Tab& T)
{
    const int l = oct_lane(), ax = oct_axis();
    Oct O;
    O.atom = l < 4;
    O.l0 = l == 0;
    // the trap acts on the ion only: +0 on the atom's lanes (then K = kA + qc qr is +0 there)
    O.kA = O.atom ? 0.0 : (ax == 0 ? P.kA[0] : (ax == 1 ? P.kA[1] : P.kA[2]));
    O.qr = O.atom ? 0.0 : (ax == 0 ? P.q_ratio[0] : (ax == 1 ? P.q_ratio[1] : P.q_ratio[2]));
    O.cl = l == 1 ? T.c2 : (l == 2 ? T.c3 : (l == 3 ? T.c4 : (l == 4 ? T.c5 : 1.0)));
    // opaque values: the compiler keeps them in registers instead of re-deriving them per step
    asm volatile("" : "+v"(O.kA), "+v"(O.qr), "+v"(O.cl));
    return O;
}

// Stage cosines for the eight-lane form: the values of stage_cos.  Lanes 0..5 each evaluate one of the
// six small-angle series in a single round (lane 0 the phase remainder, lanes 1..5 the offsets c2 h,
// c3 h, c4 h, c5 h and h); the quadrant of lane 0's result goes to every lane, each of lanes 1..5
// combines it with its own offset, and row broadcasts gather the five cosines.
__device__ __forceinline__ StageCos stage_cos8(double tau, double phase0, double h, const Oct& O)
{
    double k;
    const double r = phase_reduce(tau + phase0, k);
    asm volatile("" ::"v"(r));
    const double a = O.l0 ? r : O.cl * h;
    double c, s;
    small_sincos<true>(a, c, s);
    double sb, cb;
    phase_quadrant(k, quad_bcast<0, true>(c), quad_bcast<0, true>(s), sb, cb);
    const double cs = cos_comb(cb, sb, c, s);
    StageCos C;
    C.c2 = quad_bcast<1, true>(cs);
    C.c3 = quad_bcast<2, true>(cs);
    C.c4 = quad_bcast<3, true>(cs);
    C.c5 = quad_bcast<4, true>(cs);
    C.c6 = quad_bcast<5, true>(cs);
    return C;
}

// Separation at a stage position X (negated on ion lanes): this lane's component d_k = X + partner,
// the three components in every lane and |d|^2 by the expression of the other forms.
struct Sep8 {
    double dk, d0, d1, d2, rr;
};
__device__ __forceinline__ Sep8 sep8(double X)
{
    Sep8 D;
    D.dk = X + oct_partner(X);
    D.d0 = quad_bcast<0, true>(D.dk);
    D.d1 = quad_bcast<1, true>(D.dk);
    D.d2 = quad_bcast<2, true>(D.dk);
    D.rr = dot3(D.d0, D.d1, D.d2, D.d0, D.d1, D.d2);
    return D;
}

// Acceleration of this lane's coordinate at stage position X with separation D, with the bits of acc_atom
// and acc_ion in one expression: with t = s d_k and m = 1/m_a (atom lanes) or 1/m_i (ion lanes),
//   atom:  (s d_k) / m_a                  = fma(t, m, -0)        (adding -0 leaves every product as is)
//   ion:   -acc_ion = -fma(-t, m, K X)    = fma(t, m, -(K X))    (X = -x_ion; rounding is sign-symmetric)
// where K = kA + qc qr and K X is rounded as the product K x_ion of the other forms.  The addend is
// fma(K, X, +0) on every lane: the rounded product K X when that is not zero, and +0 when it is, so on the
// atom lanes (K = +0) it is the -0 of the atom's expression.  On an ion lane an exactly zero K X thus
// enters as -0 where the other forms add +0, which changes the result only when t m is an exact -0 as
// well: the sign of an exactly zero acceleration.
__device__ __forceinline__ double accel8(const Lane& L, const Oct& O, double m, double cs, double X, const Sep8& D)
{
    const double s = force_scale_rr(L, D.rr);
    const double qc = L.qx_half * cs;
    const double kx = fma(O.kA + qc * O.qr, X, 0.0);
    return fma(s * D.dk, m, -kx);
}
__device__ __forceinline__ double accel8(const Lane& L, const Oct& O, double m, double cs, double X)
{
    return accel8(L, O, m, cs, X, sep8(X));
}

// Everything a step of the eight-lane form computes before its bookkeeping: the fifth-order state, the
// acceleration there (FSAL; not in secant mode), the error norm and the geometry of the new state.
// SECANT: the step may be a secant iterate (then `exiting` says whether it is); without it the
// error-norm part runs unconditionally.
struct Step8 {
    double x5, v5, F7, en;
    bool finite;
    uint64_t nonfin;    // lanes(non-finite new state): 0 exactly when `finite`
    double rho_new, s_new, ww, e_prev, e_new, se_new;
};
template <bool CE, bool SECANT>
__device__ __forceinline__ Step8 traj8_trial(const KParams& P, const StepK& K, const Traj8& T, const Tab& B,
                                             const Oct& O, double h, bool exiting)
{
    const double hh = h * h;
    const StageCos C = stage_cos8(T.S.tau, T.L.phase0, h, O);
    const double F2 = accel8(T.L, O, T.m, C.c2, stage2(T.x, T.v, h, B));
    const double F3 = accel8(T.L, O, T.m, C.c3, stage3(T.x, T.v, h, hh, T.F1, B));
    const double F4 = accel8(T.L, O, T.m, C.c4, stage4(T.x, T.v, h, hh, T.F1, F2, B));
    const double F5 = accel8(T.L, O, T.m, C.c5, stage5(T.x, T.v, h, hh, T.F1, F2, F3, B));
    const double F6 = accel8(T.L, O, T.m, C.c6, stage6(T.x, T.v, h, hh, T.F1, F2, F3, F4, B));
    Step8 R;
    R.x5 = sol_x(T.x, T.v, h, hh, T.F1, F2, F3, F4, F5, B);
    R.v5 = sol_v(T.v, h, T.F1, F3, F4, F5, F6, B);
    const Sep8 D = sep8(R.x5);
    R.en = 0.0;
    R.F7 = 0.0;
    R.finite = true;
    R.nonfin = 0;
    if (!SECANT || cond<true>(!exiting)) {
        R.F7 = accel8(T.L, O, T.m, C.c6, R.x5, D);
        const double rx = err_ratio(err_x(hh, T.F1, F2, F3, F4, F5, F6, B), T.x, R.x5, K.rtol, K.atol);
        const double rv = err_ratio(err_v(h, T.F1, F3, F4, F5, F6, R.F7, B), T.v, R.v5, K.rtol, K.atol);
        // every octet of the wave holds the same trajectory: a wave ballot is the octet's OR
        const bool bad = (lanes(ratio_bad(rx)) | lanes(ratio_bad(rv))) != 0;
        R.nonfin = lanes(!is_finite(R.x5)) | lanes(!is_finite(R.v5));
        // a NaN ratio makes the step bad, and then the maximum is not used
        const double m = oct_max(fmax(rx, rv));
        R.en = bad ? __builtin_nan("") : m;
        R.finite = R.nonfin == 0;
    }
    const double wk = R.v5 + oct_partner(R.v5);
    const double w0 = quad_bcast<0, true>(wk), w1 = quad_bcast<1, true>(wk), w2 = quad_bcast<2, true>(wk);
    R.rho_new = D.rr;
    R.s_new = dot3(D.d0, D.d1, D.d2, w0, w1, w2);
    R.ww = dot3(w0, w1, w2, w0, w1, w2);
    R.e_prev = R.e_new = R.se_new = 0.0;
    if (CE) {
        const double p0 = quad_bcast<0, true>(T.x), p1 = quad_bcast<1, true>(T.x), p2 = quad_bcast<2, true>(T.x);
        const double a0 = quad_bcast<0, true>(R.x5), a1 = quad_bcast<1, true>(R.x5), a2 = quad_bcast<2, true>(R.x5);
        const double u0 = quad_bcast<0, true>(R.v5), u1 = quad_bcast<1, true>(R.v5), u2 = quad_bcast<2, true>(R.v5);
        R.e_prev = dot3(p0, p1, p2, p0, p1, p2);
        R.e_new = dot3(a0, a1, a2, a0, a1, a2);
        R.se_new = dot3(a0, a1, a2, u0, u1, u2);
    }
    return R;
}

// Bookkeeping of the eight-lane form: the shared epilogue and the state update it decides.
template <bool CE>
__device__ __forceinline__ void traj8_finish(const StepK& K, Traj8& T, double h, bool fin, const Step8& R)
{
    const StepOutcome o = step_epilogue<CE, true>(K, T.S, T.L, h, fin, R.en, R.finite, R.rho_new, R.s_new, R.ww,
                                                  R.e_prev, R.e_new, R.se_new);
    const bool moved = o == OUT_SECANT_DONE || o == OUT_STOP_RFLOOR || o == OUT_ACCEPT || o == OUT_TMAX;
    T.x = moved ? R.x5 : T.x;
    T.v = moved ? R.v5 : T.v;
    T.F1 = (o == OUT_ACCEPT || o == OUT_TMAX) ? R.F7 : T.F1;
}

// One attempted step (or secant iterate) of the eight-lane form, any mode.
template <bool CE>
__device__ __forceinline__ void traj8_advance(const KParams& P, const StepK& K, Traj8& T, const Tab& B, const Oct& O)
{
    double h;
    bool fin;
    if (!step_prologue<true>(K, T.S, h, fin)) return;
    const Step8 R = traj8_trial<CE, true>(P, K, T, B, O, h, T.S.mode != 0);
    traj8_finish<CE>(K, T, h, fin, R);
}

// Steps of the eight-lane form, the common cases in a loop of their own.  Almost every step is an
// ordinary one (stepping mode, under the step cap, not the final step, h above its floor) that is either
// rejected or accepted with nothing crossed (no periapsis inside r_b, no separation floor, no exit
// crossing, finite state).  For these the prologue and epilogue reduce to one uniform test each and the
// plain updates below, which are what step_prologue and step_epilogue do in these cases.  At the first
// step that is not such a step the loop ends with the state as it was before that step, and the general
// path takes the step again from there (same inputs, same bits); the trial's results never leave the
// loop, so no register carries them past its exits.  `iters` counts the attempted steps (and stops).
template <bool CE>
__device__ __forceinline__ void traj8_run(const KParams& P, const StepK& K, Traj8& T, const Tab& B, const Oct& O,
                                          uint64_t& iters)
{
    Scal& S = T.S;
    // the loop never changes the mode: stepping mode is tested once
    for (bool stepping = lanes(S.mode == 0) != 0; stepping;) {
        const uint64_t plain =
            lanes(S.nacc < K.max_steps) & lanes(!(S.h >= K.tau_max - S.tau)) & lanes(!(S.h < K.hmin));
        if (plain == 0) break;
        const double h = S.h;
        const Step8 R = traj8_trial<CE, false>(P, K, T, B, O, h, false);
        const uint64_t acc = lanes(R.en <= 1.0);
        const double ex_prev = CE ? R.e_prev : S.rho_prev, ex_new = CE ? R.e_new : R.rho_new;
        const uint64_t bounce = lanes(S.s_prev < 0.0) & lanes(R.s_new >= 0.0) &
                                lanes(fmin(S.rho_prev, R.rho_new) < T.L.rm2 * K.rb_ratio2);
        const uint64_t floor = lanes(R.rho_new < 0.01 * T.L.rm2);
        const uint64_t crossing =
            lanes(ex_prev <= K.r0sq) & lanes(ex_new > K.r0sq) & lanes((CE ? R.se_new : R.s_new) > 0.0);
        const uint64_t event = acc & (R.nonfin | bounce | floor | crossing);
        if (event != 0) break;
        ++iters;
        S.nrhs += 6;
        if (acc != 0) {
            S.nacc++;
            S.status |= bound_state(T.L, R.rho_new, R.ww) ? (uint32_t)IAT_ST_BOUND_SEEN : 0u;
            S.tau = S.tau + h;
            S.rho_prev = R.rho_new;
            S.s_prev = R.s_new;
            S.h = fmin(K.hmax, h * step_factor(R.en, S.last_rej != 0));
            S.last_rej = 0;
            T.x = R.x5;
            T.v = R.v5;
            T.F1 = R.F7;
        } else {
            S.nrej++;
            S.h = h * reject_factor(R.en);
            S.last_rej = 1;
        }
    }
    ++iters;
    traj8_advance<CE>(P, K, T, B, O);
}

// A record of the continuation layout (cont_save) into the eight-lane form.
__device__ inline void cont_load8(const Work& W, const Cont& C, int64_t slot, bool atom, int ax, Traj8& T, int64_t& i)
{
    const int64_t c = C.cap;
    i = C.id[slot];
    const int comp = atom ? ax : 3 + ax;
    const double x = C.d[(0 + comp) * c + slot], v = C.d[(6 + comp) * c + slot], f = C.d[(12 + comp) * c + slot];
    T.x = atom ? x : -x;
    T.v = atom ? v : -v;
    T.F1 = atom ? f : -f;
    Scal& S = T.S;
    S.tau = C.d[18 * c + slot];
    S.h = C.d[19 * c + slot];
    S.rho_prev = C.d[20 * c + slot];
    S.s_prev = C.d[21 * c + slot];
    S.sx1 = C.d[22 * c + slot];
    S.sg1 = C.d[23 * c + slot];
    S.tau_first = C.d[24 * c + slot];
    S.tau_last = C.d[25 * c + slot];
    S.nacc = C.n[0 * c + slot];
    S.nrej = C.n[1 * c + slot];
    S.nrhs = C.n[2 * c + slot];
    S.nb = C.n[3 * c + slot];
    S.status = (uint32_t)C.n[4 * c + slot];
    S.mode = (uint32_t)C.n[5 * c + slot];
    S.last_rej = C.n[6 * c + slot];
    S.done = 0;
    work_lane(W, i, T.L);
}

// Final state into the work buffer: lanes 0..2 the atom's coordinates, lanes 7..5 the ion's (sign
// restored), lane 0 the scalar state.
__device__ __forceinline__ void traj8_store(const Work& W, int64_t i, const Traj8& T, int l)
{
    if (l < 3) {
        W.d(l, i) = T.x;
        W.d(6 + l, i) = T.v;
    } else if (l >= 5) {
        W.d(3 + (7 - l), i) = -T.x;
        W.d(9 + (7 - l), i) = -T.v;
    }
    if (l == 0) work_store_scal(W, i, T.S);
}

}  // namespace iat
