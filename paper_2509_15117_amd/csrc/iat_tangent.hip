// Tangent-linear of the accepted-step map and iat_integrate_tangent.
//
// Internal differentiation: each tangent column obeys the same Runge-Kutta scheme, with the
// primal's step sizes, applied to  dY' = J(tau, y) dY + b(tau, y).  One wave per trajectory:
// quad c (4 lanes, one per axis) carries column c of the 12 x 12 stability matrix (c < 12) or the
// forcing column of q_x (c = 12) or De (c = 13) next to the four-lane primal, which every quad
// evaluates identically (same bits as iat_integrate).  Quads 14 and 15 shadow column 13.
// A per-trajectory kernel then applies the chain rule to the observables and computes the
// finite-time Lyapunov exponent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "iat_device.h"
#include "iat_host.h"

namespace iat {

constexpr int kCols = 14;

// Tangent of the accelerations at one stage, next to the primal ones (same expressions as
// accel4 for the primal).  With u = 1/rho and s(rho) = 8 C8' rho^-5 - 4 C4' rho^-3:
//   (H dd)_k = s dd_k + 2 s'(rho) d_k (d . dd),   s' = u^4 (3 (4C4') - 5 (8C8') u^2),
//   dA_a = (H dd)/m_a,  dA_i = -(H dd)/m_i - kappa o dX_i,
// forcing of q_x: dA_i,k += -(q_ratio_k cos/2) X_i,k; of De: ds/dDe = -(8C8') u^5 / De.
__device__ __forceinline__ void accel4_tan(const KParams& P, const Lane& L, int k, int col, double inv_De,
                                           double ffac, double cs, double Xa, double Xi, double tXa, double tXi,
                                           double& Aa, double& Ai, double& tAa, double& tAi)
{
    const double dk = Xa - Xi;
    const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
    const double s = force_scale(L, d0, d1, d2);
    const double qc = L.qx_half * cs;
    const double kA = k == 0 ? P.kA[0] : (k == 1 ? P.kA[1] : P.kA[2]);
    const double qr = k == 0 ? P.q_ratio[0] : (k == 1 ? P.q_ratio[1] : P.q_ratio[2]);
    Aa = acc_atom(L, s, dk);
    Ai = acc_ion(P.inv_mi, s, dk, kA, qc, qr, Xi);
    const double u = recip(dot3(d0, d1, d2, d0, d1, d2));
    const double u2 = u * u;
    const double sp = u2 * u2 * (3.0 * L.c4x4 - 5.0 * L.c8x8 * u2);
    const double tdk = tXa - tXi;
    const double t0 = quad_bcast<0>(tdk), t1 = quad_bcast<1>(tdk), t2 = quad_bcast<2>(tdk);
    const double Hd = s * tdk + 2.0 * sp * dk * dot3(d0, d1, d2, t0, t1, t2);
    tAa = Hd * L.inv_ma;
    tAi = -Hd * P.inv_mi - (kA + qc * qr) * tXi;
    if (col == 12) tAi += ffac * (-(qr * (0.5 * cs)) * Xi);
    if (col == 13) {
        const double Fd = (-L.c8x8 * u2 * u2 * u * inv_De) * dk * ffac;
        tAa += Fd * L.inv_ma;
        tAi -= Fd * P.inv_mi;
    }
}

struct Tan4 {
    double xa, xi, va, vi, F1a, F1i;   // tangent column, this lane's axis
    int exp2s;                         // the column is stored scaled by 2^-exp2s
    double ffac;                       // forcing scale 2^-exp2s
};

__device__ __forceinline__ void tan_rescale(Tan4& D)
{
    const double m = quad_max(fmax(fmax(fabs(D.xa), fabs(D.xi)), fmax(fmax(fabs(D.va), fabs(D.vi)),
                                                                      fmax(fabs(D.F1a), fabs(D.F1i)))));
    if (m > 0x1.0p+400) {
        D.xa = ldexp(D.xa, -400);
        D.xi = ldexp(D.xi, -400);
        D.va = ldexp(D.va, -400);
        D.vi = ldexp(D.vi, -400);
        D.F1a = ldexp(D.F1a, -400);
        D.F1i = ldexp(D.F1i, -400);
        D.ffac = ldexp(D.ffac, -400);
        D.exp2s += 400;
    }
}

// One attempted step of the four-lane primal with its tangent column.  Returns through the
// tangent arguments the column at the step end (only committed by the caller's logic below).
__device__ __forceinline__ void tan4_advance(const KParams& P, const StepK& K, Traj4& T, Tan4& D, int col,
                                             double inv_De, double& ex_xa, double& ex_xi, double& ex_va,
                                             double& ex_vi)
{
    double h;
    bool fin;
    if (!step_prologue(K, T.S, h, fin)) return;
    const bool exiting = T.S.mode != 0;
    const int k = quad_axis();
    const double hh = h * h;
    const StageCos C = stage_cos4(T.S.tau, T.L.phase0, h);
    double F2a, F2i, F3a, F3i, F4a, F4i, F5a, F5i, F6a, F6i;
    double G2a, G2i, G3a, G3i, G4a, G4i, G5a, G5i, G6a, G6i;
    const double ff = D.ffac;
    accel4_tan(P, T.L, k, col, inv_De, ff, C.c2, stage2(T.xa, T.va, h), stage2(T.xi, T.vi, h),
               stage2(D.xa, D.va, h), stage2(D.xi, D.vi, h), F2a, F2i, G2a, G2i);
    accel4_tan(P, T.L, k, col, inv_De, ff, C.c3, stage3(T.xa, T.va, h, hh, T.F1a), stage3(T.xi, T.vi, h, hh, T.F1i),
               stage3(D.xa, D.va, h, hh, D.F1a), stage3(D.xi, D.vi, h, hh, D.F1i), F3a, F3i, G3a, G3i);
    accel4_tan(P, T.L, k, col, inv_De, ff, C.c4, stage4(T.xa, T.va, h, hh, T.F1a, F2a),
               stage4(T.xi, T.vi, h, hh, T.F1i, F2i), stage4(D.xa, D.va, h, hh, D.F1a, G2a),
               stage4(D.xi, D.vi, h, hh, D.F1i, G2i), F4a, F4i, G4a, G4i);
    accel4_tan(P, T.L, k, col, inv_De, ff, C.c5, stage5(T.xa, T.va, h, hh, T.F1a, F2a, F3a),
               stage5(T.xi, T.vi, h, hh, T.F1i, F2i, F3i), stage5(D.xa, D.va, h, hh, D.F1a, G2a, G3a),
               stage5(D.xi, D.vi, h, hh, D.F1i, G2i, G3i), F5a, F5i, G5a, G5i);
    accel4_tan(P, T.L, k, col, inv_De, ff, C.c6, stage6(T.xa, T.va, h, hh, T.F1a, F2a, F3a, F4a),
               stage6(T.xi, T.vi, h, hh, T.F1i, F2i, F3i, F4i), stage6(D.xa, D.va, h, hh, D.F1a, G2a, G3a, G4a),
               stage6(D.xi, D.vi, h, hh, D.F1i, G2i, G3i, G4i), F6a, F6i, G6a, G6i);
    const double x5a = sol_x(T.xa, T.va, h, hh, T.F1a, F2a, F3a, F4a, F5a);
    const double x5i = sol_x(T.xi, T.vi, h, hh, T.F1i, F2i, F3i, F4i, F5i);
    const double v5a = sol_v(T.va, h, T.F1a, F3a, F4a, F5a, F6a);
    const double v5i = sol_v(T.vi, h, T.F1i, F3i, F4i, F5i, F6i);
    const double y5a = sol_x(D.xa, D.va, h, hh, D.F1a, G2a, G3a, G4a, G5a);
    const double y5i = sol_x(D.xi, D.vi, h, hh, D.F1i, G2i, G3i, G4i, G5i);
    const double w5a = sol_v(D.va, h, D.F1a, G3a, G4a, G5a, G6a);
    const double w5i = sol_v(D.vi, h, D.F1i, G3i, G4i, G5i, G6i);
    double en = 0.0, F7a = 0.0, F7i = 0.0, G7a = 0.0, G7i = 0.0;
    bool finite = true;
    if (!exiting) {
        accel4_tan(P, T.L, k, col, inv_De, ff, C.c6, x5a, x5i, y5a, y5i, F7a, F7i, G7a, G7i);
        const double ra = err_ratio(err_x(hh, T.F1a, F2a, F3a, F4a, F5a, F6a), T.xa, x5a, K.rtol, K.atol);
        const double ri = err_ratio(err_x(hh, T.F1i, F2i, F3i, F4i, F5i, F6i), T.xi, x5i, K.rtol, K.atol);
        const double rva = err_ratio(err_v(h, T.F1a, F3a, F4a, F5a, F6a, F7a), T.va, v5a, K.rtol, K.atol);
        const double rvi = err_ratio(err_v(h, T.F1i, F3i, F4i, F5i, F6i, F7i), T.vi, v5i, K.rtol, K.atol);
        const int bad = quad_or((ratio_bad(ra) || ratio_bad(ri) || ratio_bad(rva) || ratio_bad(rvi)) ? 1 : 0);
        const int nonfin =
            quad_or((is_finite(x5a) && is_finite(x5i) && is_finite(v5a) && is_finite(v5i)) ? 0 : 1);
        const double m = quad_max(fmax(fmax(ra, rva), fmax(ri, rvi)));
        en = bad ? __builtin_nan("") : m;
        finite = nonfin == 0;
    }
    const double dk = x5a - x5i, wk = v5a - v5i;
    const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
    const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
    const double rho_new = dot3(d0, d1, d2, d0, d1, d2);
    const double s_new = dot3(d0, d1, d2, w0, w1, w2);
    const double ww = dot3(w0, w1, w2, w0, w1, w2);
    const StepOutcome o = step_epilogue(K, T.S, T.L, h, fin, en, finite, rho_new, s_new, ww);
    if (o == OUT_SECANT_CONT || o == OUT_SECANT_DONE) {
        // tangent of the latest secant iterate RK5(y_n, h*) with h* frozen
        ex_xa = y5a;
        ex_xi = y5i;
        ex_va = w5a;
        ex_vi = w5i;
    }
    if (o == OUT_SECANT_DONE || o == OUT_STOP_RFLOOR) {
        T.xa = x5a;
        T.xi = x5i;
        T.va = v5a;
        T.vi = v5i;
        D.xa = (o == OUT_SECANT_DONE) ? ex_xa : y5a;
        D.xi = (o == OUT_SECANT_DONE) ? ex_xi : y5i;
        D.va = (o == OUT_SECANT_DONE) ? ex_va : w5a;
        D.vi = (o == OUT_SECANT_DONE) ? ex_vi : w5i;
    } else if (o == OUT_ACCEPT || o == OUT_TMAX) {
        T.xa = x5a;
        T.xi = x5i;
        T.va = v5a;
        T.vi = v5i;
        T.F1a = F7a;
        T.F1i = F7i;
        D.xa = y5a;
        D.xi = y5i;
        D.va = w5a;
        D.vi = w5i;
        D.F1a = G7a;
        D.F1i = G7i;
        tan_rescale(D);
    }
}

// Per-trajectory tangent scratch: 14 columns x (12 corrected entries + exit-time shift + exponent)
struct TanOut {
    double* col;     // [n][14][13]
    int32_t* ex;     // [n][14]
    double* Phi;     // [n][144] or NULL (uncorrected stability matrix, row-major, scaled per column)
};

__global__ void __launch_bounds__(256) k_tangent(KParams P, Work W, TanOut O)
{
    const int lane = __lane_id();
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;   // one wave per trajectory
    if (i >= P.n) return;
    const int q = lane >> 2;
    const int col = q < kCols ? q : kCols - 1;
    const int k = quad_axis();
    const int kk = lane & 3;
    Traj4 T;
    work_lane(W, i, T.L);
    scal_init(P, T.S);
    T.S.status = (uint32_t)W.k(4, i);
    T.xa = W.d(k, i);
    T.xi = W.d(3 + k, i);
    T.va = W.d(6 + k, i);
    T.vi = W.d(9 + k, i);
    const int nonfin = quad_or((is_finite(T.xa) && is_finite(T.xi) && is_finite(T.va) && is_finite(T.vi)) ? 0 : 1);
    Tan4 D;
    D.exp2s = 0;
    D.ffac = 1.0;
    D.xa = (col == k) ? 1.0 : 0.0;
    D.xi = (col == 3 + k) ? 1.0 : 0.0;
    D.va = (col == 6 + k) ? 1.0 : 0.0;
    D.vi = (col == 9 + k) ? 1.0 : 0.0;
    TrajParams tp;
    traj_params(P, i, tp);
    const double inv_De = 1.0 / tp.De;
    if (nonfin) {
        T.S.status |= IAT_ST_NONFINITE;
        T.S.done = 1;
    } else {
        double s0, c0;
        phase_sincos(T.L.phase0, s0, c0);
        accel4_tan(P, T.L, k, col, inv_De, 1.0, c0, T.xa, T.xi, D.xa, D.xi, T.F1a, T.F1i, D.F1a, D.F1i);
        T.S.nrhs = 1;
        const double dk = T.xa - T.xi, wk = T.va - T.vi;
        const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
        const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
        T.S.rho_prev = dot3(d0, d1, d2, d0, d1, d2);
        T.S.s_prev = dot3(d0, d1, d2, w0, w1, w2);
    }
    double ex_xa = 0.0, ex_xi = 0.0, ex_va = 0.0, ex_vi = 0.0;
    const StepK K = step_k_in_registers(P);      // latency-bound: launch constants held in registers
    while (!T.S.done) tan4_advance(P, K, T, D, col, inv_De, ex_xa, ex_xi, ex_va, ex_vi);
    // uncorrected stability matrix (columns 0..11), scaled by 2^-exp2s per column
    if (O.Phi && q < 12 && kk < 3) {
        double* Ph = O.Phi + (size_t)i * 144;
        Ph[(0 + k) * 12 + col] = D.xa;
        Ph[(3 + k) * 12 + col] = D.xi;
        Ph[(6 + k) * 12 + col] = D.va;
        Ph[(9 + k) * 12 + col] = D.vi;
    }
    // exit-time correction: dh = -(d . dd)/(d . w), dY += f(y_f) dh
    double dh = 0.0;
    if (T.S.status & IAT_ST_EXITED) {
        double s1, c1;
        phase_sincos(T.S.tau + T.L.phase0, s1, c1);
        double Aa, Ai, tAa, tAi;
        accel4_tan(P, T.L, k, col, inv_De, D.ffac, c1, T.xa, T.xi, D.xa, D.xi, Aa, Ai, tAa, tAi);
        const double dk = T.xa - T.xi, wk = T.va - T.vi, tdk = D.xa - D.xi;
        const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
        const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
        const double t0 = quad_bcast<0>(tdk), t1 = quad_bcast<1>(tdk), t2 = quad_bcast<2>(tdk);
        dh = -dot3(d0, d1, d2, t0, t1, t2) / dot3(d0, d1, d2, w0, w1, w2);
        D.xa += T.va * dh;
        D.xi += T.vi * dh;
        D.va += Aa * dh;
        D.vi += Ai * dh;
    }
    if (q < kCols && kk < 3) {
        double* c = O.col + ((size_t)i * kCols + col) * 13;
        c[0 + k] = D.xa;
        c[3 + k] = D.xi;
        c[6 + k] = D.va;
        c[9 + k] = D.vi;
        if (k == 0) {
            c[12] = dh;
            O.ex[(size_t)i * kCols + col] = D.exp2s;
        }
    }
    if (lane == 0) {
        // the primal's final state, for the observables
        W.d(19, i) = T.S.tau;
        W.d(20, i) = T.S.tau_first;
        W.d(21, i) = T.S.tau_last;
        W.k(0, i) = T.S.nacc;
        W.k(1, i) = T.S.nrej;
        W.k(2, i) = T.S.nrhs;
        W.k(3, i) = T.S.nb;
        W.k(4, i) = (int32_t)T.S.status;
    }
    if (q == 0 && kk < 3) {
        W.d(k, i) = T.xa;
        W.d(3 + k, i) = T.xi;
        W.d(6 + k, i) = T.va;
        W.d(9 + k, i) = T.vi;
    }
}

// Eigenvalues of a symmetric 12 x 12 matrix by cyclic Jacobi rotations: on return the diagonal
// of A holds them.
__device__ void sym12_jacobi(double A[144])
{
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 12; ++p) {
            diag += A[p * 13] * A[p * 13];
            for (int r = p + 1; r < 12; ++r) off += A[p * 12 + r] * A[p * 12 + r];
        }
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < 11; ++p)
            for (int r = p + 1; r < 12; ++r) {
                const double apr = A[p * 12 + r];
                if (apr == 0.0) continue;
                const double theta = (A[r * 13] - A[p * 13]) / (2.0 * apr);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int m = 0; m < 12; ++m) {
                    const double amp = A[m * 12 + p], amr = A[m * 12 + r];
                    A[m * 12 + p] = c * amp - s * amr;
                    A[m * 12 + r] = s * amp + c * amr;
                }
                for (int m = 0; m < 12; ++m) {
                    const double apm = A[p * 12 + m], arm = A[r * 12 + m];
                    A[p * 12 + m] = c * apm - s * arm;
                    A[r * 12 + m] = s * apm + c * arm;
                }
            }
    }
}
__device__ double sym12_max_eig(double A[144])
{
    sym12_jacobi(A);
    double mx = A[0];
    for (int p = 1; p < 12; ++p) mx = fmax(mx, A[p * 13]);
    return mx;
}

// Chain rule to the observables and the FTLE, one thread per trajectory.
__global__ void __launch_bounds__(128) k_tangent_post(KParams P, Work W, TanOut O, double* dobs, double* ftle,
                                                      double* lyap, int32_t* phi_exp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    TrajParams tp;
    traj_params(P, i, tp);
    const double w = P.omega;
    // head-on start and its derivatives in internal units
    const double st = tp.sin_t, ct = tp.cos_t, sp = tp.sin_p, cp = tp.cos_p;
    const double n[3] = {st * cp, st * sp, ct}, nt[3] = {ct * cp, ct * sp, -st}, np_[3] = {-st * sp, st * cp, 0.0};
    const double ma = species_mass(P, tp.sp);
    const double v0 = sqrt(2.0 * tp.E / ma) / w, dv0 = v0 / (2.0 * tp.E);
    double dy0[3][12];
    for (int a = 0; a < 12; ++a) dy0[0][a] = dy0[1][a] = dy0[2][a] = 0.0;
    for (int k = 0; k < 3; ++k) {
        dy0[0][k] = P.r0 * nt[k];
        dy0[0][6 + k] = -v0 * nt[k];
        dy0[1][k] = P.r0 * np_[k];
        dy0[1][6 + k] = -v0 * np_[k];
        dy0[2][6 + k] = -dv0 * n[k];
    }
    double yf[12];
    for (int a = 0; a < 12; ++a) yf[a] = W.d(a, i);
    const double tau = W.d(19, i);
    const double* C = O.col + (size_t)i * kCols * 13;
    const int32_t* E = O.ex + (size_t)i * kCols;
    // observable gradients (a.u. velocities), as derived from the observable formulas
    double vi[3], vf[3];
    for (int k = 0; k < 3; ++k) {
        vi[k] = -v0 * n[k] * w;
        vf[k] = yf[6 + k] * w;
    }
    const double c3[3] = {vi[1] * vf[2] - vi[2] * vf[1], vi[2] * vf[0] - vi[0] * vf[2], vi[0] * vf[1] - vi[1] * vf[0]};
    const double Sn = sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
    const double D = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
    const double den = Sn * Sn + D * D;
    double ch[3];
    for (int k = 0; k < 3; ++k) ch[k] = c3[k] / Sn;
    const double dS_dvf[3] = {ch[1] * vi[2] - ch[2] * vi[1], ch[2] * vi[0] - ch[0] * vi[2], ch[0] * vi[1] - ch[1] * vi[0]};
    const double dS_dvi[3] = {vf[1] * ch[2] - vf[2] * ch[1], vf[2] * ch[0] - vf[0] * ch[2], vf[0] * ch[1] - vf[1] * ch[0]};
    double dang_dvf[3], dang_dvi[3], dq_dvf[3];
    const double dv[3] = {vf[0] - vi[0], vf[1] - vi[1], vf[2] - vi[2]};
    const double ndv = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int k = 0; k < 3; ++k) {
        dang_dvf[k] = (D * dS_dvf[k] - Sn * vi[k]) / den;
        dang_dvi[k] = (D * dS_dvi[k] - Sn * vf[k]) / den;
        dq_dvf[k] = ma * dv[k] / ndv;
    }
    double sn1, cs1;
    phase_sincos(tau + tp.phase0, sn1, cs1);
    double dE_dy[12];
    for (int a = 0; a < 12; ++a) dE_dy[a] = 0.0;
    double dE_dtau = 0.0, dE_dq = 0.0;
    const double mw2 = P.m_ion * w * w;
    for (int k = 0; k < 3; ++k) {
        const double ak = P.a_x * P.a_ratio[k], qk = tp.qx * P.q_ratio[k];
        dE_dy[3 + k] = (ak + 2.0 * qk * cs1) * mw2 * yf[3 + k] / 4.0;
        dE_dy[9 + k] = mw2 * yf[9 + k];
        dE_dtau += -2.0 * qk * sn1 * mw2 * yf[3 + k] * yf[3 + k] / 8.0;
        dE_dq += 2.0 * P.q_ratio[k] * cs1 * mw2 * yf[3 + k] * yf[3 + k] / 8.0;
    }
    double* out = dobs + (size_t)i * 15;
    for (int pi = 0; pi < 5; ++pi) {
        double colv[12], dtau = 0.0;
        for (int a = 0; a < 12; ++a) colv[a] = 0.0;
        if (pi < 3) {
            for (int c = 0; c < 12; ++c) {
                if (dy0[pi][c] == 0.0) continue;
                const double sc = ldexp(dy0[pi][c], E[c]);
                for (int a = 0; a < 12; ++a) colv[a] += C[c * 13 + a] * sc;
                dtau += C[c * 13 + 12] * sc;
            }
        } else {
            const int c = pi == 3 ? 12 : 13;
            for (int a = 0; a < 12; ++a) colv[a] = ldexp(C[c * 13 + a], E[c]);
            dtau = ldexp(C[c * 13 + 12], E[c]);
        }
        double da = 0.0, dq = 0.0, de = 0.0;
        for (int k = 0; k < 3; ++k) {
            da += dang_dvf[k] * w * colv[6 + k];
            dq += dq_dvf[k] * w * colv[6 + k];
        }
        for (int a = 0; a < 12; ++a) de += dE_dy[a] * colv[a];
        de += dE_dtau * dtau;
        if (pi < 3)
            for (int k = 0; k < 3; ++k) {
                const double dvi = dy0[pi][6 + k] * w;
                da += dang_dvi[k] * dvi;
                dq -= dq_dvf[k] * dvi;
            }
        if (pi == 3) de += dE_dq;
        out[0 * 5 + pi] = da;
        out[1 * 5 + pi] = dq;
        out[2 * 5 + pi] = de;
    }
    // FTLE = ln sigma_max(Phi(t_f, 0)) / t_f with Phi from the uncorrected columns
    if (ftle || lyap || phi_exp) {
        int emax = E[0];
        for (int c = 1; c < 12; ++c) emax = max(emax, E[c]);
        if (phi_exp) phi_exp[i] = emax;
        if (ftle || lyap) {
            double Ph[144], M[144];
            if (O.Phi) {
                for (int a = 0; a < 144; ++a) Ph[a] = O.Phi[(size_t)i * 144 + a];
            }
            double big = 0.0;
            for (int a = 0; a < 12; ++a)
                for (int c = 0; c < 12; ++c) {
                    Ph[a * 12 + c] = ldexp(Ph[a * 12 + c], E[c] - emax);
                    big = fmax(big, fabs(Ph[a * 12 + c]));
                }
            const double sc = big > 0.0 ? 1.0 / big : 1.0;
            for (int a = 0; a < 144; ++a) Ph[a] *= sc;
            for (int a = 0; a < 12; ++a)
                for (int b = 0; b < 12; ++b) {
                    double s = 0.0;
                    for (int m = 0; m < 12; ++m) s += Ph[m * 12 + a] * Ph[m * 12 + b];
                    M[a * 12 + b] = s;
                }
            const double t_f = tau / w;
            const double ln2 = 0.69314718055994530942;
            if (ftle) ftle[i] = (0.5 * log(sym12_max_eig(M)) - log(sc) + emax * ln2) / t_f;
            if (lyap) {
                // Lyapunov spectrum of D Phi D^-1, D = sqrt(mass) per coordinate (canonical scaling,
                // in which Phi is symplectic: the exponents pair as lambda, -lambda)
                const double ra = sqrt(ma), ri = sqrt(P.m_ion);
                double dsc[12];
                for (int k = 0; k < 3; ++k) {
                    dsc[k] = dsc[6 + k] = ra;
                    dsc[3 + k] = dsc[9 + k] = ri;
                }
                double big2 = 0.0;
                for (int a = 0; a < 12; ++a)
                    for (int c = 0; c < 12; ++c) {
                        Ph[a * 12 + c] *= dsc[a] / dsc[c];
                        big2 = fmax(big2, fabs(Ph[a * 12 + c]));
                    }
                const double sc2 = big2 > 0.0 ? 1.0 / big2 : 1.0;
                for (int a = 0; a < 144; ++a) Ph[a] *= sc2;
                for (int a = 0; a < 12; ++a)
                    for (int b = 0; b < 12; ++b) {
                        double s = 0.0;
                        for (int m = 0; m < 12; ++m) s += Ph[m * 12 + a] * Ph[m * 12 + b];
                        M[a * 12 + b] = s;
                    }
                sym12_jacobi(M);
                double ev[12];
                for (int a = 0; a < 12; ++a) ev[a] = M[a * 13];
                for (int a = 1; a < 12; ++a)          // descending
                    for (int b = a; b > 0 && ev[b] > ev[b - 1]; --b) {
                        const double t = ev[b];
                        ev[b] = ev[b - 1];
                        ev[b - 1] = t;
                    }
                for (int a = 0; a < 12; ++a)
                    lyap[(size_t)i * 12 + a] = ev[a] > 0.0
                        ? (0.5 * log(ev[a]) - log(sc) - log(sc2) + emax * ln2) / t_f
                        : __builtin_nan("");
            }
        }
    }
    if (O.Phi) {
        // report the stability matrix on the common scale 2^phi_exp
        int emax = E[0];
        for (int c = 1; c < 12; ++c) emax = max(emax, E[c]);
        for (int a = 0; a < 12; ++a)
            for (int c = 0; c < 12; ++c)
                O.Phi[(size_t)i * 144 + a * 12 + c] = ldexp(O.Phi[(size_t)i * 144 + a * 12 + c], E[c] - emax);
    }
}

}  // namespace iat

using namespace iat;

extern "C" int iat_integrate_tangent(const iat_system* sys, const iat_species* species, int n_species,
                                     const iat_batch* batch, const iat_obs* obs, double* dobs_dp, double* ftle,
                                     double* lyap, double* Phi_out, const iat_launch* launch, void* stream)
{
    int rc = validate_common(sys, species, n_species, batch);
    if (rc) return rc;
    if (batch->y0) return set_error(IAT_ENOTSUP, "tangent: only head-on starts (y0 == NULL) have (theta, phi, E)");
    if (batch->gen.kind == IAT_GEN_THERMAL)
        return set_error(IAT_ENOTSUP, "tangent: thermal starts are not parameterised by (theta, phi, E)");
    if (!obs) return set_error(IAT_EINVAL, "obs is NULL");
    if (batch->n > 0 &&
        (!obs->angle || !obs->q_transfer || !obs->dE_ion || !obs->t_dwell || !obs->n_bounce || !obs->status || !dobs_dp))
        return set_error(IAT_EINVAL, "tangent: obs outputs and dobs_dp are required");
    (void)launch;
    if (batch->n == 0) return 0;
    KParams P;
    fill_params(P, sys, species, n_species, batch);
    fill_outputs(P, obs);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = batch->n;
    const size_t work_bytes = (size_t)n * (kWorkDoubles * sizeof(double) + kWorkInts * sizeof(int32_t));
    const size_t col_bytes = (size_t)n * kCols * 13 * sizeof(double);
    const size_t ex_bytes = (size_t)n * kCols * sizeof(int32_t);
    const size_t phi_bytes = (size_t)n * 144 * sizeof(double);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const bool own_phi = Phi_out == nullptr && (ftle != nullptr || lyap != nullptr);
    const size_t bytes = up(work_bytes) + up(col_bytes) + up(ex_bytes) + (own_phi ? up(phi_bytes) : 0);
    void* ws = nullptr;
    if (hipMallocAsync(&ws, bytes, st) != hipSuccess) return set_error(IAT_EHIP, "hipMallocAsync of %zu bytes failed", bytes);
    char* base = (char*)ws;
    Work W;
    W.n = n;
    W.D = (double*)base;
    W.I = (int32_t*)(W.D + (size_t)kWorkDoubles * n);
    TanOut O;
    O.col = (double*)(base + up(work_bytes));
    O.ex = (int32_t*)(base + up(work_bytes) + up(col_bytes));
    O.Phi = own_phi ? (double*)(base + up(work_bytes) + up(col_bytes) + up(ex_bytes)) : Phi_out;
    launch_setup(P, W, st);
    const int64_t lanes = n * 64;
    hipLaunchKernelGGL(k_tangent, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, P, W, O);
    hipLaunchKernelGGL(k_tangent_post, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, P, W, O, dobs_dp, ftle,
                       lyap, (int32_t*)nullptr);
    launch_observe(P, W, st);
    if (hipFreeAsync(ws, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return 0;
}
