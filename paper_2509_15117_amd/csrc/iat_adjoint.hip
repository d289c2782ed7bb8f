// Discrete adjoint of the accepted-step map (iat_adjoint).
//
// The gradient of J = sum_k obs_bar_k obs_k with respect to (theta, phi, E, q_x, De) is the
// transpose of the tangent-linear of the same discrete map: every accepted Runge-Kutta step is
// differentiated with its step size frozen, the exit time by the event condition |d| = r0.
//
//   1. scan      : record count per trajectory from its accepted-step count (a prior
//                  iat_integrate of the same batch) -> exclusive offsets.
//   2. forward   : the four-lane primal again (same bits as iat_integrate), storing a checkpoint
//                  (state, FSAL acceleration, time, next trial step) every 256 committed steps and
//                  the state before the final (exit or t_max) step with that step's size.
//   3. seed      : one lane per trajectory: dJ/dy_f and dJ/dtau_f from the observable formulas,
//                  projected on the exit event; the explicit dependence of J on the start velocity
//                  and on q_x is kept aside.
//   4. order     : the differentiable trajectories sorted into descending buckets of log2 of their
//                  committed steps; the reverse kernel's quads take them from this queue in order,
//                  longest first, so the longest reverse sweeps start at once and the short ones fill
//                  in around them (no static striding of trajectories over quads).
//   5. reverse   : four lanes per trajectory.  The final step, then each segment from the last:
//                  recompute the segment from its checkpoint (states kept in per-quad scratch), and
//                  apply the step adjoints backwards.  For one step of the Nystrom form
//                    X_s = x + c_s h v + h^2 sum_j P_sj F_j,  F_s = a(tau + c_s h, X_s),
//                    x' = x + h v + h^2 sum_j Q_j F_j,        v' = v + h sum_j B_j F_j,
//                  the adjoints are Fbar_s = h^2 Q_s lx + h B_s lv + h^2 sum_{r>s} P_rs Xbar_r and
//                  Xbar_s = J_s^T Fbar_s (s = 6..1), then lx += sum_s Xbar_s and
//                  lv += h lx + h sum_s c_s Xbar_s; q_x and De collect (da/dp)^T Fbar_s.
//                  Adjoints that pass 2^400 are rescaled (exponent tracked per trajectory).
//   6. post      : chain rule through the head-on start (theta, phi, E) and the explicit terms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "iat_device.h"
#include "iat_host.h"

namespace iat {

constexpr int kSeg = 256;          // committed steps between checkpoints
constexpr int kRec = 24;           // doubles per record: lanes 0..2 hold 6 values of their axis, lane 3 (tau, h)
constexpr int kScr = 8;            // doubles per lane per recomputed step: x_a, x_i, v_a, v_i, F1_a, F1_i, tau, h
constexpr int kSkip = -1;
constexpr int kReplayFailed = -1;  // exponent value that marks a failed recomputation
constexpr int kBuckets = 64;       // queue buckets: floor(log2(committed steps + 1))
// control words of the reverse kernel's queue: [0] next queue position, [1] queue length,
// [2, 2 + kBuckets) bucket sizes, [2 + kBuckets, 2 + 2 kBuckets) bucket fill cursors
constexpr int kCtlWords = 2 + 2 * kBuckets;

struct AdjBuf {
    int64_t* off;        // [n + 1] first record of each trajectory (exclusive scan of the counts)
    double* rec;         // [total][kRec]
    int64_t cap;         // records available
    double* lam;         // [12][n] adjoint of the state (seed, then at the start)
    double* acc;         // [3][n] q_x and De adjoint sums, exponent of the 2^400 rescaling
    double* expl;        // [8][n] explicit terms (unscaled): 5 parameters, then dJ/dv_atom(0) (a.u.)
    int32_t* info;       // [2][n] committed steps, state (1 = ok, kSkip = skipped)
    double* scr;         // per-quad scratch [kSeg][kScr][lanes]
    int64_t lanes;       // 4 x resident quads of the reverse kernel
    int64_t* order;      // [n] queue of the reverse kernel: trajectory indices, longest bucket first
    unsigned long long* ctl;   // [kCtlWords] queue control words (zeroed by the scan kernel)
};

// ---------------------------------------------------------------------------------------
// 1. offsets: records = accepted/256 + 2 (checkpoints 0..J and the final step) for trajectories
// that exited or reached t_max; 0 otherwise.  Exact exclusive scan over every trajectory (one block,
// contiguous chunks per thread), off[n] = the total.  Trajectory i owns records [off[i], off[i+1]);
// the forward pass skips every trajectory whose range ends beyond cap, so no record is ever written
// at or past cap.  ctl, if not NULL, receives the zeroed queue control words.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_adj_scan(const int64_t* n_accept, const uint32_t* status, int64_t n,
                                                   int64_t* off, unsigned long long* ctl)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    if (ctl && t < kCtlWords) ctl[t] = 0ull;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = min(n, t * per), hi = min(n, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) {
        const bool ok = (status[i] & (IAT_ST_EXITED | IAT_ST_TMAX)) != 0 && n_accept[i] >= 0;
        s += ok ? n_accept[i] / kSeg + 2 : 0;
    }
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int j = 0; j < 1024; ++j) {
            const int64_t v = part[j];
            part[j] = run;
            run += v;
        }
        off[n] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        const bool ok = (status[i] & (IAT_ST_EXITED | IAT_ST_TMAX)) != 0 && n_accept[i] >= 0;
        off[i] = run;
        run += ok ? n_accept[i] / kSeg + 2 : 0;
    }
}

__device__ __forceinline__ void rec_store(double* r, int lane4, double xa, double xi, double va, double vi, double fa,
                                          double fi, double tau, double h)
{
    if (lane4 < 3) {
        r[lane4 * 6 + 0] = xa;
        r[lane4 * 6 + 1] = xi;
        r[lane4 * 6 + 2] = va;
        r[lane4 * 6 + 3] = vi;
        r[lane4 * 6 + 4] = fa;
        r[lane4 * 6 + 5] = fi;
    } else {
        r[18] = tau;
        r[19] = h;
    }
}

// ---------------------------------------------------------------------------------------
// 2. forward pass with checkpoints, one quad per trajectory
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adj_forward(KParams P, Work W, AdjBuf B)
{
    const int lane4 = __lane_id() & 3;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    if (i >= P.n) return;
    const int64_t m = B.off[i + 1] - B.off[i];
    if (m < 2 || B.off[i + 1] > B.cap) {     // no records, or they do not fit the workspace
        if (lane4 == 0) {
            B.info[i] = 0;
            B.info[P.n + i] = kSkip;
        }
        return;
    }
    double* R = B.rec + B.off[i] * kRec;
    const Tab TB = tab_in_registers();     // latency-bound: coefficients held in registers
    Traj4 T;
    traj4_start(P, W, i, T);
    bool ok = true;
    int32_t ncom = 0;
    if (ok && !T.S.done) rec_store(R, lane4, T.xa, T.xi, T.va, T.vi, T.F1a, T.F1i, T.S.tau, T.S.h);
    double fxa = 0, fxi = 0, fva = 0, fvi = 0, ffa = 0, ffi = 0, ftau = 0, fh = 0;
    while (!T.S.done) {
        const double xa = T.xa, xi = T.xi, va = T.va, vi = T.vi, fa = T.F1a, fi = T.F1i, tau = T.S.tau;
        double h;
        const int o = traj4_step(P, T, h, TB);
        if (o == OUT_ACCEPT) {
            ++ncom;
            if (ncom % kSeg == 0) {
                const int64_t j = ncom / kSeg;
                if (j <= m - 2) {
                    if (ok) rec_store(R + j * kRec, lane4, T.xa, T.xi, T.va, T.vi, T.F1a, T.F1i, T.S.tau, T.S.h);
                } else {
                    ok = false;      // more steps than the accepted count promised
                }
            }
        } else if (o == OUT_TMAX || o == OUT_SECANT_DONE) {
            fxa = xa;
            fxi = xi;
            fva = va;
            fvi = vi;
            ffa = fa;
            ffi = fi;
            ftau = tau;
            fh = h;
        }
    }
    const bool good = ok && (T.S.status & (IAT_ST_EXITED | IAT_ST_TMAX)) &&
                      !(T.S.status & (IAT_ST_NONFINITE | IAT_ST_R_UNDERFLOW | IAT_ST_H_UNDERFLOW | IAT_ST_MAX_STEPS));
    if (good) rec_store(R + (m - 1) * kRec, lane4, fxa, fxi, fva, fvi, ffa, ffi, ftau, fh);
    traj4_store(W, i, T, lane4);      // final state, time and counters (as iat_integrate)
    if (lane4 == 0) {
        B.info[i] = ncom;
        B.info[P.n + i] = good ? 1 : kSkip;
    }
}

// ---------------------------------------------------------------------------------------
// 3. seed: dJ/dy_f (internal units) projected on the exit event, explicit terms aside
// ---------------------------------------------------------------------------------------
struct StartDeriv {
    double dy[3][12];    // d y0 / d(theta, phi, E), internal units
    double dvi[3][3];    // d v_atom(0) / d(theta, phi, E), a.u.
};

__device__ inline void start_derivatives(const KParams& P, const TrajParams& tp, StartDeriv& S)
{
    const double w = P.omega;
    const double st = tp.sin_t, ct = tp.cos_t, sp = tp.sin_p, cp = tp.cos_p;
    const double n[3] = {st * cp, st * sp, ct}, nt[3] = {ct * cp, ct * sp, -st}, np_[3] = {-st * sp, st * cp, 0.0};
    const double ma = species_mass(P, tp.sp);
    const double v0 = sqrt(2.0 * tp.E / ma) / w, dv0 = v0 / (2.0 * tp.E);
    for (int p = 0; p < 3; ++p)
        for (int a = 0; a < 12; ++a) S.dy[p][a] = 0.0;
    for (int k = 0; k < 3; ++k) {
        S.dy[0][k] = P.r0 * nt[k];
        S.dy[0][6 + k] = -v0 * nt[k];
        S.dy[1][k] = P.r0 * np_[k];
        S.dy[1][6 + k] = -v0 * np_[k];
        S.dy[2][6 + k] = -dv0 * n[k];
    }
    for (int p = 0; p < 3; ++p)
        for (int k = 0; k < 3; ++k) S.dvi[p][k] = S.dy[p][6 + k] * w;
}

__global__ void __launch_bounds__(128) k_adj_seed(KParams P, Work W, AdjBuf B, const double* obs_bar)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    double lam[12];
    for (int a = 0; a < 12; ++a) lam[a] = 0.0;
    double ex[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (B.info[P.n + i] == 1) {
        TrajParams tp;
        traj_params(P, i, tp);
        Lane L;
        lane_consts(P, tp, L);
        const double w = P.omega;
        const double ga = obs_bar[3 * i + 0], gq = obs_bar[3 * i + 1], ge = obs_bar[3 * i + 2];
        double y0[12];
        start_state_au(P, i, tp, y0);
        double yf[12];
        for (int a = 0; a < 12; ++a) yf[a] = W.d(a, i);
        const double tau = W.d(19, i);
        const uint32_t st = (uint32_t)W.k(4, i);
        double vi[3], vf[3];
        for (int k = 0; k < 3; ++k) {
            vi[k] = y0[6 + k];
            vf[k] = yf[6 + k] * w;
        }
        // angle = atan2(|vi x vf|, vi . vf), q = m_a |vf - vi|, dE = E_ion(tau_f) - E_ion(0)
        const double c3[3] = {vi[1] * vf[2] - vi[2] * vf[1], vi[2] * vf[0] - vi[0] * vf[2],
                              vi[0] * vf[1] - vi[1] * vf[0]};
        const double Sn = sqrt(c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
        const double D = vi[0] * vf[0] + vi[1] * vf[1] + vi[2] * vf[2];
        const double den = Sn * Sn + D * D;
        double ch[3];
        for (int k = 0; k < 3; ++k) ch[k] = c3[k] / Sn;
        const double dS_dvf[3] = {ch[1] * vi[2] - ch[2] * vi[1], ch[2] * vi[0] - ch[0] * vi[2],
                                  ch[0] * vi[1] - ch[1] * vi[0]};
        const double dS_dvi[3] = {vf[1] * ch[2] - vf[2] * ch[1], vf[2] * ch[0] - vf[0] * ch[2],
                                  vf[0] * ch[1] - vf[1] * ch[0]};
        const double dv[3] = {vf[0] - vi[0], vf[1] - vi[1], vf[2] - vi[2]};
        const double ndv = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const double ma = species_mass(P, tp.sp);
        double dang_dvf[3], dang_dvi[3], dq_dvf[3];
        for (int k = 0; k < 3; ++k) {
            dang_dvf[k] = (D * dS_dvf[k] - Sn * vi[k]) / den;
            dang_dvi[k] = (D * dS_dvi[k] - Sn * vf[k]) / den;
            dq_dvf[k] = ma * dv[k] / ndv;
        }
        double sn1, cs1;
        phase_sincos(tau + tp.phase0, sn1, cs1);
        const double mw2 = P.m_ion * w * w;
        double dE_dtau = 0.0, dE_dq = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double ak = P.a_x * P.a_ratio[k], qk = tp.qx * P.q_ratio[k];
            lam[3 + k] = ge * ((ak + 2.0 * qk * cs1) * mw2 * yf[3 + k] / 4.0);
            lam[9 + k] = ge * (P.m_ion * (yf[9 + k] * w) * w);
            lam[6 + k] = (ga * dang_dvf[k] + gq * dq_dvf[k]) * w;
            dE_dtau += -2.0 * qk * sn1 * mw2 * yf[3 + k] * yf[3 + k] / 8.0;
            dE_dq += 2.0 * P.q_ratio[k] * cs1 * mw2 * yf[3 + k] * yf[3 + k] / 8.0;
        }
        if (st & IAT_ST_EXITED) {
            // the exit time moves with the state: |d|^2 = r0^2 at tau_f
            double X[6], A[6];
            for (int a = 0; a < 6; ++a) X[a] = yf[a];
            accel1(P, L, cs1, X, A);
            double lf = 0.0;
            for (int a = 0; a < 6; ++a) lf += lam[a] * yf[6 + a] + lam[6 + a] * A[a];
            double dd = 0.0;
            double d[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = yf[k] - yf[3 + k];
                dd += d[k] * (yf[6 + k] - yf[9 + k]);
            }
            const double mu = (lf + ge * dE_dtau) / dd;
            for (int k = 0; k < 3; ++k) {
                lam[k] -= mu * d[k];
                lam[3 + k] += mu * d[k];
            }
        }
        StartDeriv S;
        start_derivatives(P, tp, S);
        for (int k = 0; k < 3; ++k) ex[5 + k] = ga * dang_dvi[k] - gq * dq_dvf[k];
        for (int p = 0; p < 3; ++p)
            for (int k = 0; k < 3; ++k) ex[p] += ex[5 + k] * S.dvi[p][k];
        ex[3] = ge * dE_dq;
    }
    for (int a = 0; a < 12; ++a) B.lam[(int64_t)a * P.n + i] = lam[a];
    for (int p = 0; p < 8; ++p) B.expl[(int64_t)p * P.n + i] = ex[p];
}

// ---------------------------------------------------------------------------------------
// 4. queue of the reverse sweep: differentiable trajectories by descending bucket of
// floor(log2(committed steps + 1)); within a bucket in arrival order (the order only decides which
// quad runs a trajectory, never its bits: each quad recomputes from the records alone)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int step_bucket(int32_t ncom)
{
    return 63 - __clzll((unsigned long long)ncom + 1ull);
}

__global__ void __launch_bounds__(256) k_adj_order_count(int64_t n, AdjBuf B)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || B.info[n + i] != 1) return;
    atomicAdd(&B.ctl[2 + step_bucket(B.info[i])], 1ull);
}

__global__ void __launch_bounds__(256) k_adj_order_fill(int64_t n, AdjBuf B)
{
    __shared__ unsigned long long start[kBuckets];
    const int t = threadIdx.x;
    if (t < kBuckets) {
        unsigned long long s = 0;
        for (int b = t + 1; b < kBuckets; ++b) s += B.ctl[2 + b];
        start[t] = s;
        if (blockIdx.x == 0 && t == 0) B.ctl[1] = s + B.ctl[2];
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + t;
    if (i >= n || B.info[n + i] != 1) return;
    const int b = step_bucket(B.info[i]);
    B.order[start[b] + atomicAdd(&B.ctl[2 + kBuckets + b], 1ull)] = i;
}

// ---------------------------------------------------------------------------------------
// 5. reverse sweep
// ---------------------------------------------------------------------------------------
// Xbar = J^T Fbar at one stage for this lane's axis:  with u = Fbar_a/m_a - Fbar_i/m_i,
// Xbar_a = G u, Xbar_i = -G u - kappa Fbar_i, G = s I + 2 s'(rho) d d^T; q_x and De pick up
// (da/dq_x)^T Fbar and (da/dDe)^T Fbar (this lane's share, summed over the axes at the end).
__device__ __forceinline__ void stage_adjoint(const KParams& P, const Lane& L, int k, double cs, double inv_De,
                                              double Xa, double Xi, double Fba, double Fbi, double& Xba, double& Xbi,
                                              double& pq, double& pD)
{
    const double dk = Xa - Xi;
    const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
    const double u = recip(dot3(d0, d1, d2, d0, d1, d2));
    const double u2 = u * u;
    const double s = u2 * u * (L.c8x8 * u2 - L.c4x4);
    const double sp = u2 * u2 * (3.0 * L.c4x4 - 5.0 * L.c8x8 * u2);
    const double wk = Fba * L.inv_ma - Fbi * P.inv_mi;
    const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
    const double Gw = s * wk + 2.0 * sp * dk * dot3(d0, d1, d2, w0, w1, w2);
    const double qc = L.qx_half * cs;
    const double kA = k == 0 ? P.kA[0] : (k == 1 ? P.kA[1] : P.kA[2]);
    const double qr = k == 0 ? P.q_ratio[0] : (k == 1 ? P.q_ratio[1] : P.q_ratio[2]);
    Xba = Gw;
    Xbi = -Gw - (kA + qc * qr) * Fbi;
    pq += Fbi * (-(qr * (0.5 * cs)) * Xi);
    pD += (-L.c8x8 * u2 * u2 * u * inv_De) * dk * wk;
}

struct Adj4 {
    double xa, xi, va, vi;   // adjoint of this lane's axis of the state
    double pq, pD;           // parameter adjoints (this lane's share)
    int e2;                  // everything above is scaled by 2^-e2
};

// Adjoint of one committed step taken from (x, v, F1) at tau with step h.
__device__ inline void step_adjoint(const KParams& P, const Lane& L, int k, double inv_De, double xa, double xi,
                                    double va, double vi, double F1a, double F1i, double tau, double h, Adj4& A)
{
    const double hh = h * h;
    double sb, cb;
    phase_sincos(tau + L.phase0, sb, cb);
    const double cs2 = cos_shift(cb, sb, c2 * h), cs3 = cos_shift(cb, sb, c3 * h), cs4 = cos_shift(cb, sb, c4 * h),
                 cs5 = cos_shift(cb, sb, c5 * h), cs6 = cos_shift(cb, sb, h);
    // stage positions (as in the primal step)
    double F2a, F2i, F3a, F3i, F4a, F4i, F5a, F5i;
    const double X2a = stage2(xa, va, h), X2i = stage2(xi, vi, h);
    accel4(P, L, k, cs2, X2a, X2i, F2a, F2i);
    const double X3a = stage3(xa, va, h, hh, F1a), X3i = stage3(xi, vi, h, hh, F1i);
    accel4(P, L, k, cs3, X3a, X3i, F3a, F3i);
    const double X4a = stage4(xa, va, h, hh, F1a, F2a), X4i = stage4(xi, vi, h, hh, F1i, F2i);
    accel4(P, L, k, cs4, X4a, X4i, F4a, F4i);
    const double X5a = stage5(xa, va, h, hh, F1a, F2a, F3a), X5i = stage5(xi, vi, h, hh, F1i, F2i, F3i);
    accel4(P, L, k, cs5, X5a, X5i, F5a, F5i);
    const double X6a = stage6(xa, va, h, hh, F1a, F2a, F3a, F4a), X6i = stage6(xi, vi, h, hh, F1i, F2i, F3i, F4i);
    // reverse over the stages
    const double lxa = A.xa, lxi = A.xi, lva = A.va, lvi = A.vi;
    double B6a, B6i, B5a, B5i, B4a, B4i, B3a, B3i, B2a, B2i, B1a, B1i;
    stage_adjoint(P, L, k, cs6, inv_De, X6a, X6i, h * b6 * lva, h * b6 * lvi, B6a, B6i, A.pq, A.pD);
    stage_adjoint(P, L, k, cs5, inv_De, X5a, X5i, hh * q5 * lxa + h * b5 * lva, hh * q5 * lxi + h * b5 * lvi, B5a, B5i,
                  A.pq, A.pD);
    stage_adjoint(P, L, k, cs4, inv_De, X4a, X4i, hh * (q4 * lxa + p64 * B6a) + h * b4 * lva,
                  hh * (q4 * lxi + p64 * B6i) + h * b4 * lvi, B4a, B4i, A.pq, A.pD);
    stage_adjoint(P, L, k, cs3, inv_De, X3a, X3i, hh * (q3 * lxa + p53 * B5a + p63 * B6a) + h * b3 * lva,
                  hh * (q3 * lxi + p53 * B5i + p63 * B6i) + h * b3 * lvi, B3a, B3i, A.pq, A.pD);
    stage_adjoint(P, L, k, cs2, inv_De, X2a, X2i, hh * (q2 * lxa + p42 * B4a + p52 * B5a + p62 * B6a),
                  hh * (q2 * lxi + p42 * B4i + p52 * B5i + p62 * B6i), B2a, B2i, A.pq, A.pD);
    stage_adjoint(P, L, k, cb, inv_De, xa, xi,
                  hh * (q1 * lxa + p31 * B3a + p41 * B4a + p51 * B5a + p61 * B6a) + h * b1 * lva,
                  hh * (q1 * lxi + p31 * B3i + p41 * B4i + p51 * B5i + p61 * B6i) + h * b1 * lvi, B1a, B1i, A.pq,
                  A.pD);
    A.xa = lxa + (B1a + B2a + B3a + B4a + B5a + B6a);
    A.xi = lxi + (B1i + B2i + B3i + B4i + B5i + B6i);
    A.va = lva + h * lxa + h * (c2 * B2a + c3 * B3a + c4 * B4a + c5 * B5a + B6a);
    A.vi = lvi + h * lxi + h * (c2 * B2i + c3 * B3i + c4 * B4i + c5 * B5i + B6i);
    // keep the adjoint inside the exponent range
    const double m = quad_max(fmax(fmax(fabs(A.xa), fabs(A.xi)), fmax(fabs(A.va), fabs(A.vi))));
    if (m > 0x1.0p+400) {
        A.xa = ldexp(A.xa, -400);
        A.xi = ldexp(A.xi, -400);
        A.va = ldexp(A.va, -400);
        A.vi = ldexp(A.vi, -400);
        A.pq = ldexp(A.pq, -400);
        A.pD = ldexp(A.pD, -400);
        A.e2 += 400;
    }
}

__device__ __forceinline__ double quad_sum3(double v)
{
    const double a = quad_bcast<0>(v), b = quad_bcast<1>(v), c = quad_bcast<2>(v);
    return (a + b) + c;
}

// Reverse sweep of trajectory i by one quad: the final step, then each segment from the last, recomputed
// from its checkpoint into the quad's scratch (lanes gl of B.scr) and swept backwards.
__device__ inline void reverse_trajectory(const KParams& P, const Work& W, const AdjBuf& B, const StepK& K, int64_t i,
                                          int k, int lane4, int64_t gl)
{
    Lane L;
    work_lane(W, i, L);
    TrajParams tp;
    traj_params(P, i, tp);
    const double inv_De = 1.0 / tp.De;
    const int64_t m = B.off[i + 1] - B.off[i];
    const double* R = B.rec + B.off[i] * kRec;
    const int32_t ncom = B.info[i];
    Adj4 A;
    A.xa = B.lam[(int64_t)k * P.n + i];
    A.xi = B.lam[(int64_t)(3 + k) * P.n + i];
    A.va = B.lam[(int64_t)(6 + k) * P.n + i];
    A.vi = B.lam[(int64_t)(9 + k) * P.n + i];
    A.pq = A.pD = 0.0;
    A.e2 = 0;
    {   // the final step
        const double* r = R + (m - 1) * kRec;
        step_adjoint(P, L, k, inv_De, r[k * 6 + 0], r[k * 6 + 1], r[k * 6 + 2], r[k * 6 + 3], r[k * 6 + 4],
                     r[k * 6 + 5], r[18], r[19], A);
    }
    for (int32_t j = ncom / kSeg; j >= 0; --j) {
        const int32_t cnt = min(kSeg, ncom - j * kSeg);
        if (cnt <= 0) continue;
        // recompute the segment from its checkpoint, keeping each committed step's start
        const double* r = R + (int64_t)j * kRec;
        Traj4 T;
        T.L = L;
        scal_init(P, T.S);
        T.xa = r[k * 6 + 0];
        T.xi = r[k * 6 + 1];
        T.va = r[k * 6 + 2];
        T.vi = r[k * 6 + 3];
        T.F1a = r[k * 6 + 4];
        T.F1i = r[k * 6 + 5];
        T.S.tau = r[18];
        T.S.h = r[19];
        T.S.nacc = 0;
        {
            const double dk = T.xa - T.xi, wk = T.va - T.vi;
            const double d0 = quad_bcast<0>(dk), d1 = quad_bcast<1>(dk), d2 = quad_bcast<2>(dk);
            const double w0 = quad_bcast<0>(wk), w1 = quad_bcast<1>(wk), w2 = quad_bcast<2>(wk);
            T.S.rho_prev = dot3(d0, d1, d2, d0, d1, d2);
            T.S.s_prev = dot3(d0, d1, d2, w0, w1, w2);
        }
        int32_t c = 0;
        int guard = 0;
        while (c < cnt && !T.S.done && guard < 64 * kSeg) {
            double* sl = B.scr + (int64_t)c * kScr * B.lanes + gl;
            sl[0 * B.lanes] = T.xa;
            sl[1 * B.lanes] = T.xi;
            sl[2 * B.lanes] = T.va;
            sl[3 * B.lanes] = T.vi;
            sl[4 * B.lanes] = T.F1a;
            sl[5 * B.lanes] = T.F1i;
            sl[6 * B.lanes] = T.S.tau;
            double h;
            const int o = traj4_step_k(P, K, T, h, kTab);
            sl[7 * B.lanes] = h;
            if (o == OUT_ACCEPT) ++c;
            ++guard;
        }
        if (c != cnt) {      // the recomputation did not retrace the forward pass
            A.e2 = kReplayFailed;
            break;
        }
        for (int32_t s = c - 1; s >= 0; --s) {
            const double* sl = B.scr + (int64_t)s * kScr * B.lanes + gl;
            step_adjoint(P, L, k, inv_De, sl[0], sl[1 * B.lanes], sl[2 * B.lanes], sl[3 * B.lanes],
                         sl[4 * B.lanes], sl[5 * B.lanes], sl[6 * B.lanes], sl[7 * B.lanes], A);
        }
    }
    // adjoint at the start, parameter sums over the three axes
    if (lane4 < 3) {
        B.lam[(int64_t)k * P.n + i] = A.xa;
        B.lam[(int64_t)(3 + k) * P.n + i] = A.xi;
        B.lam[(int64_t)(6 + k) * P.n + i] = A.va;
        B.lam[(int64_t)(9 + k) * P.n + i] = A.vi;
    }
    const double pq = quad_sum3(lane4 < 3 ? A.pq : 0.0), pD = quad_sum3(lane4 < 3 ? A.pD : 0.0);
    if (lane4 == 0) {
        B.acc[i] = pq;
        B.acc[P.n + i] = pD;
        B.acc[2 * P.n + i] = (double)A.e2;
        if (A.e2 == kReplayFailed) B.info[P.n + i] = kSkip;
    }
}

__global__ void __launch_bounds__(256) k_adj_reverse(KParams P, Work W, AdjBuf B)
{
    const int lane = __lane_id();
    const int lane4 = lane & 3;
    const int k = quad_axis();
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;     // resident quad
    const int64_t gl = q * 4 + lane4;
    const bool leader = lane4 == 0;
    const uint64_t lt = (lane & ~3) == 0 ? 0ull : (~0ull >> (64 - (lane & ~3)));
    const StepK K = step_k_in_registers(P);     // latency-bound: launch constants held in registers
    const unsigned long long queued = B.ctl[1];
    // Every lane of the wave stays in this loop until no quad of the wave has work, so the loop's
    // exit and the queue hand-out below are wave-uniform: quads that need a trajectory take queue
    // positions by ballot rank from one atomic of the wave.  (A per-quad exit around a lane-0 atomic
    // and a shuffle lets the compiler run the shuffle of the three other lanes ahead of their
    // leader's atomic, so those lanes would keep re-reading a stale position.)
    bool need = gl < B.lanes;                   // quads beyond the scratch take no work
    bool active = false;
    int64_t i = -1;
    for (;;) {
        const uint64_t mask = __ballot(need && leader);
        if (mask) {
            const int first = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0ull;
            if (lane == first) base = atomicAdd(&B.ctl[0], (unsigned long long)__popcll(mask));
            base = __shfl(base, first, 64);
            if (need) {
                const unsigned long long pos = base + (unsigned long long)__popcll(mask & lt);
                active = pos < queued;
                i = active ? B.order[pos] : -1;
                need = false;          // a quad past the end of the queue takes no more work
            }
        }
        if (!__any(active)) break;
        if (active) {
            reverse_trajectory(P, W, B, K, i, k, lane4, gl);
            active = false;
            need = true;
        }
    }
}

// ---------------------------------------------------------------------------------------
// 5. chain rule through the head-on start, explicit terms, skipped trajectories
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_adj_post(KParams P, AdjBuf B, double* p_bar, double* y0_bar)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    double* o = p_bar + 5 * i;
    if (B.info[P.n + i] != 1) {
        for (int p = 0; p < 5; ++p) o[p] = __builtin_nan("");
        if (y0_bar)
            for (int a = 0; a < 12; ++a) y0_bar[12 * i + a] = __builtin_nan("");
        P.status[i] |= IAT_ST_ADJ_SKIPPED;
        return;
    }
    TrajParams tp;
    traj_params(P, i, tp);
    StartDeriv S;
    start_derivatives(P, tp, S);
    const int e2 = (int)B.acc[2 * P.n + i];
    for (int p = 0; p < 3; ++p) {
        double s = 0.0;
        for (int a = 0; a < 12; ++a) s += S.dy[p][a] * B.lam[(int64_t)a * P.n + i];
        o[p] = ldexp(s, e2) + B.expl[(int64_t)p * P.n + i];
    }
    o[3] = ldexp(B.acc[i], e2) + B.expl[3 * P.n + i];
    o[4] = ldexp(B.acc[P.n + i], e2) + B.expl[4 * P.n + i];
    if (y0_bar) {
        // gradient with respect to the start state in a.u. (positions a0, velocities a.u.)
        const double inv_w = 1.0 / P.omega;
        for (int a = 0; a < 6; ++a) y0_bar[12 * i + a] = ldexp(B.lam[(int64_t)a * P.n + i], e2);
        for (int a = 6; a < 12; ++a) y0_bar[12 * i + a] = ldexp(B.lam[(int64_t)a * P.n + i], e2) * inv_w;
        for (int k = 0; k < 3; ++k) y0_bar[12 * i + 6 + k] += B.expl[(int64_t)(5 + k) * P.n + i];
    }
}

// resident quads of the reverse kernel (and so its scratch size)
int64_t reverse_quads(int64_t n)
{
    int n_cu = 0;
    if (device_state(&n_cu) != 0 || n_cu < 1) n_cu = 256;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_adj_reverse, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t q = (int64_t)n_cu * per_cu * 64;
    return std::max<int64_t>(64, std::min<int64_t>(q, ((n + 63) / 64) * 64));
}

struct AdjLayout {
    size_t off, work, lam, acc, expl, info, order, ctl, scr, rec, total_fixed;
    int64_t lanes;
};

AdjLayout adj_layout(int64_t n)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    AdjLayout L;
    L.lanes = 4 * reverse_quads(n);
    size_t o = 0;
    L.off = o;
    o += up((size_t)(n + 1) * sizeof(int64_t));
    L.work = o;
    o += up((size_t)n * (kWorkDoubles * sizeof(double) + kWorkInts * sizeof(int32_t)));
    L.lam = o;
    o += up((size_t)n * 12 * sizeof(double));
    L.acc = o;
    o += up((size_t)n * 3 * sizeof(double));
    L.expl = o;
    o += up((size_t)n * 8 * sizeof(double));
    L.info = o;
    o += up((size_t)n * 2 * sizeof(int32_t));
    L.order = o;
    o += up((size_t)n * sizeof(int64_t));
    L.ctl = o;
    o += up((size_t)kCtlWords * sizeof(unsigned long long));
    L.scr = o;
    o += up((size_t)L.lanes * kSeg * kScr * sizeof(double));
    L.rec = o;
    L.total_fixed = o;
    return L;
}

}  // namespace iat

using namespace iat;

static int adj_check(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch,
                     const iat_obs* obs)
{
    int rc = validate_common(sys, species, n_species, batch);
    if (rc) return rc;
    if (batch->y0) return set_error(IAT_ENOTSUP, "adjoint: only head-on starts (y0 == NULL) have (theta, phi, E)");
    if (batch->gen.kind == IAT_GEN_THERMAL)
        return set_error(IAT_ENOTSUP, "adjoint: thermal starts are not parameterised by (theta, phi, E)");
    if (!obs) return set_error(IAT_EINVAL, "obs is NULL");
    if (batch->n > 0 && (!obs->n_accept || !obs->status))
        return set_error(IAT_EINVAL, "adjoint: obs.n_accept and obs.status of the batch's iat_integrate run are required");
    return 0;
}

extern "C" int iat_adjoint_workspace_bytes(const iat_system* sys, const iat_species* species, int n_species,
                                           const iat_batch* batch, const iat_obs* obs, size_t* bytes, void* stream)
{
    int rc = adj_check(sys, species, n_species, batch, obs);
    if (rc) return rc;
    if (!bytes) return set_error(IAT_EINVAL, "bytes is NULL");
    const int64_t n = batch->n;
    if (n == 0) {
        *bytes = 0;
        return 0;
    }
    hipStream_t st = (hipStream_t)stream;
    AdjLayout Lo = adj_layout(n);
    int64_t* off = nullptr;
    if (hipMallocAsync((void**)&off, (size_t)(n + 1) * sizeof(int64_t), st) != hipSuccess)
        return set_error(IAT_EHIP, "hipMallocAsync failed");
    hipLaunchKernelGGL(k_adj_scan, dim3(1), dim3(1024), 0, st, (const int64_t*)obs->n_accept,
                       (const uint32_t*)obs->status, n, off, (unsigned long long*)nullptr);
    int64_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFreeAsync(off, st);
    if (e != hipSuccess) return set_error(IAT_EHIP, "reading the record count failed: %s", hipGetErrorString(e));
    *bytes = Lo.total_fixed + (size_t)total * kRec * sizeof(double);
    return 0;
}

extern "C" int iat_adjoint(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch,
                           const iat_obs* obs, const double* obs_bar, double* p_bar, double* y0_bar, void* ws,
                           size_t ws_bytes,
                           const iat_launch* launch, void* stream)
{
    int rc = adj_check(sys, species, n_species, batch, obs);
    if (rc) return rc;
    (void)launch;
    const int64_t n = batch->n;
    if (n == 0) return 0;
    if (!obs_bar || !p_bar) return set_error(IAT_EINVAL, "adjoint: obs_bar and p_bar are required");
    KParams P;
    fill_params(P, sys, species, n_species, batch);
    fill_outputs(P, obs);
    hipStream_t st = (hipStream_t)stream;
    const AdjLayout Lo = adj_layout(n);
    void* own = nullptr;
    size_t bytes = ws_bytes;
    if (!ws) {
        rc = iat_adjoint_workspace_bytes(sys, species, n_species, batch, obs, &bytes, stream);
        if (rc) return rc;
        if (hipMallocAsync(&own, bytes, st) != hipSuccess)
            return set_error(IAT_EHIP, "hipMallocAsync of %zu bytes failed", bytes);
        ws = own;
    } else if (ws_bytes < Lo.total_fixed) {
        return set_error(IAT_EWORKSPACE, "adjoint workspace of %zu bytes is below the fixed part (%zu bytes)", ws_bytes,
                         Lo.total_fixed);
    }
    char* base = (char*)ws;
    AdjBuf B;
    B.off = (int64_t*)(base + Lo.off);
    B.lam = (double*)(base + Lo.lam);
    B.acc = (double*)(base + Lo.acc);
    B.expl = (double*)(base + Lo.expl);
    B.info = (int32_t*)(base + Lo.info);
    B.scr = (double*)(base + Lo.scr);
    B.order = (int64_t*)(base + Lo.order);
    B.ctl = (unsigned long long*)(base + Lo.ctl);
    B.rec = (double*)(base + Lo.rec);
    B.cap = (int64_t)((bytes - Lo.total_fixed) / (kRec * sizeof(double)));
    B.lanes = Lo.lanes;
    Work W;
    W.n = n;
    W.D = (double*)(base + Lo.work);
    W.I = (int32_t*)(W.D + (size_t)kWorkDoubles * n);
    hipLaunchKernelGGL(k_adj_scan, dim3(1), dim3(1024), 0, st, (const int64_t*)obs->n_accept,
                       (const uint32_t*)obs->status, n, B.off, B.ctl);
    launch_setup(P, W, st);
    hipLaunchKernelGGL(k_adj_forward, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, st, P, W, B);
    hipLaunchKernelGGL(k_adj_seed, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, P, W, B, obs_bar);
    hipLaunchKernelGGL(k_adj_order_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, B);
    hipLaunchKernelGGL(k_adj_order_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, B);
    hipLaunchKernelGGL(k_adj_reverse, dim3((unsigned)(Lo.lanes / 256 + (Lo.lanes % 256 ? 1 : 0))), dim3(256), 0, st,
                       P, W, B);
    hipLaunchKernelGGL(k_adj_post, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, P, B, p_bar, y0_bar);
    if (own && hipFreeAsync(own, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return 0;
}
