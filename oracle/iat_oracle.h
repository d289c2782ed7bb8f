/*
 * CPU oracle for batched classical integration of one Paul-trapped ion plus one atom.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 re-statement of the method
 * used to check the HIP library: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant with
 * the library (paper_2509_15117_amd/csrc) and includes nothing from it.
 *
 * Physics (the paper's Eq. (1) and the model paragraph that follows it):
 *   H = 1/2 m_a v_a^2 + 1/2 m_i v_i^2 + V(|r_a - r_i|)
 *       + sum_k (a_k + 2 q_k cos(Omega t + phase0)) m_i Omega^2 r_{i,k}^2 / 8,
 *   V(r) = C8/r^8 - C4/r^4,  C4 = alpha/2,  C8 = C4^2/(4 De) (well depth De).
 * Integrator: Dormand-Prince 5(4) (the ode45 pair the paper cites), FSAL, advancing
 * with the fifth-order solution; max-norm mixed error test; standard step controller.
 * Run: head-on start on the r0 sphere (head-on-run paragraph), stop when the
 * separation crosses r0 outward or at t_max.
 * Observables: scattering angle and momentum transfer as defined in the Fig. 1
 * caption; bounce count; ion energy change; dwell time; complex flag.
 *
 * Every physical input is in atomic units (a0, m_e, E_h, hbar/E_h).  Internally the
 * integration runs in length a0, mass m_e and time tau = Omega t.
 */
#ifndef IAT_ORACLE_H
#define IAT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status bits (same meaning as the library's, numbered independently here) */
#define ORC_COMPLEX      (1u << 0)   /* n_bounce >= 2 or stopped at t_max           */
#define ORC_BOUND_SEEN   (1u << 1)   /* relative energy < 0 at some accepted step    */
#define ORC_EXITED       (1u << 2)   /* separation crossed r0 outward (normal end)   */
#define ORC_TMAX         (1u << 8)
#define ORC_H_UNDERFLOW  (1u << 9)
#define ORC_NONFINITE    (1u << 10)
#define ORC_MAX_STEPS    (1u << 11)
#define ORC_R_UNDERFLOW  (1u << 12)
#define ORC_WARN_R0      (1u << 13)

typedef struct {
    double m_ion, m_atom;        /* m_e                                            */
    double C4, De;               /* E_h a0^4 ; E_h                                  */
    double omega;                /* RF angular frequency, 1/(a.u. time)             */
    double a[3], q[3];           /* Mathieu parameters per axis                     */
    double phase0;               /* RF phase at t = 0                               */
    double r0;                   /* exit sphere radius, a0                          */
    double t_max;                /* a.u. time                                       */
    double rtol, atol;           /* on the internal state (a0, a0 per unit tau)     */
    double h0, hmax, hmin;       /* internal time; <= 0 selects the defaults        */
    double r_bounce_over_rm;     /* periapsis threshold for a bounce, units of r_m  */
    int64_t max_steps;           /* accepted-step cap; 0 = none                     */
    double y0[12];               /* r_atom, r_ion, v_atom, v_ion (a.u.)             */
    int64_t exit_centre;         /* 0: stop when the atom-ion separation leaves r0
                                    (head-on runs); 1: when the atom leaves the sphere
                                    of radius r0 about the trap centre (thermal runs) */
} orc_problem;

typedef struct {
    double angle, q_transfer, dE_ion, t_dwell, t_first, t_last;   /* a.u.          */
    int32_t n_bounce;
    uint32_t status;
    int64_t n_accept, n_reject, n_rhs;
    double tau_final;            /* internal time at the end                        */
    double y_final[12];          /* a.u.                                            */
} orc_result;

/* integration */
int  orc_integrate(const orc_problem* p, orc_result* r);
void orc_integrate_batch(int64_t n, const orc_problem* p, orc_result* r, int nthreads);
/* Same as orc_integrate, also recording the accepted step sizes (internal time):
   h[0 .. n_accept-2] are the whole accepted steps, h[n_accept-1] the last one (the
   located exit step when the run exited, and then h[n_accept] is the full size of the step
   that crossed r0).  Returns -1 if cap is too small. */
int  orc_integrate_record(const orc_problem* p, orc_result* r, double* h, int64_t cap);

/* initial conditions */
void orc_headon_state(double theta, double phi, double E, double m_atom, double r0, double y0[12]);
void orc_grid_angles(int64_t id, int n_theta, int n_phi, double* theta, double* phi);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

typedef struct {
    uint64_t seed;
    int32_t n_species, n_E, n_q, n_De;     /* list lengths; 0 for E, q, De = range   */
    int32_t species[8];
    double E[8], q[8], De[8];
    double E_lo, E_hi, q_lo, q_hi, De_lo, De_hi;
} orc_sweep;
void orc_sweep_draw(int64_t id, const orc_sweep* s, double* cos_theta, double* phi, double* phase0,
                    double* E, double* qx, double* De, int32_t* species);

/* thermal runs (Fig. 3): nine standard normals z[0..8] of trajectory id by Box-Muller on the
 * Philox blocks (id, 2..4, 0, 0) under key (seed, 0); z[9] is drawn and unused */
void orc_thermal_normals(int64_t id, uint64_t seed, double z[10]);

/* observables from an initial and a final state (a.u.) */
void orc_observables(const orc_problem* p, const double y_init[12], const double y_fin[12],
                     double t_fin, double* angle, double* q_transfer, double* dE_ion);
double orc_ion_energy(const orc_problem* p, const double y[12], double t);

/* pieces exposed for the pins */
void orc_tableau(double A[49], double b[7], double bhat[7], double c[7]);
void orc_rhs_au(const orc_problem* p, double t, const double y[12], double dydt[12]);
/* fixed-step Dormand-Prince integration of a scalar test equation:
   kind 0: y' = lam*y (y(0)=1);  kind 1: harmonic oscillator x''=-x (x=1,v=0).
   Returns the global error at t_end after n_steps equal steps. */
double orc_fixed_step_error(int kind, double lam, double t_end, int n_steps);

/* tangent-linear of the discrete accepted-step map (internal differentiation,
   frozen step sequence) and its frozen-step finite-difference counterpart.
   Parameter order p = (theta, phi, E, q_x, De); head-on problems only.
   dobs[3*5]: d(angle, q_transfer, dE_ion)/dp;  phi_out[144]: Phi(t_f, 0) with
   rows/cols in the r_atom, r_ion, v_atom, v_ion order (internal units).
   q_ratio gives dq_k/dq_x per axis.  Returns 0 on success, -2 for a thermal-run problem. */
int orc_tangent(const orc_problem* p, double theta, double phi, double E, const double q_ratio[3],
                double dobs[15], double phi_out[144], double* ftle);
int orc_fd(const orc_problem* p, double theta, double phi, double E, const double q_ratio[3],
           double rel_h, double dobs[15]);
/* the same frozen-step central differences with the replay in extended precision (long double),
   extrapolated from steps h and h/2 by Richardson's (4 D(h/2) - D(h)) / 3 */
int orc_fd_richardson(const orc_problem* p, double theta, double phi, double E, const double q_ratio[3],
                      double rel_h, double dobs[15]);

#ifdef __cplusplus
}
#endif
#endif
