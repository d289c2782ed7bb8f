/*
 * libiat -- batched classical trajectories of one Paul-trapped ion plus one atom on
 * AMD Instinct MI355X (gfx950).  C ABI: plain structs, pointers and sizes.
 *
 * Model (the paper's Eq. (1) and the model paragraph after it): Newton's equations for
 * the 12 positions and velocities of an ion (mass m_i) in the time-dependent trap
 *   U_trap = sum_k (a_k + 2 q_k cos(Omega t + phase0)) m_i Omega^2 r_{i,k}^2 / 8
 * interacting with an atom (mass m_a) through V(r) = C8/r^8 - C4/r^4, C4 = alpha/2.
 * C8 is fixed by the well depth De: C8 = C4^2/(4 De), so V(r_m) = -De at
 * r_m = (C4/(2 De))^(1/4).  Integrated by the adaptive Dormand-Prince 5(4) pair the paper
 * cites.  Head-on start (head-on-run paragraph): ion at rest at the trap centre, atom on the
 * sphere of radius r0 moving radially inward with E = m_a v0^2 / 2.  A trajectory ends when
 * the ion-atom separation crosses r0 outward (thermal runs: when the atom leaves the sphere of
 * radius r0 about the trap centre), or at t_max.
 *
 * Units: every physical input and output is in atomic units (a0, m_e, E_h, hbar/E_h);
 * angles in radians.  Integration runs internally in length a0 and time tau = Omega t;
 * rtol/atol apply to that internal state (positions in a0, velocities in a0 per unit tau)
 * and h0/hmax/hmin are in units of tau.
 *
 * Memory: pointers are DEVICE pointers unless documented as host.  Output arrays are
 * caller-allocated, length n, structure-of-arrays.  y_final and y0 are 12 x n,
 * component-major (element k of trajectory j at [k*n + j]), component order
 * r_atom(3), r_ion(3), v_atom(3), v_ion(3).
 * Streams: `stream` is a hipStream_t passed as void*; every call enqueues work on it and
 * returns without synchronising, except where documented (phase timing through
 * iat_launch.kernel_ms, sizing of the adjoint workspace, iat_fp64_peak).  NULL means the
 * default stream.  Calls allocate their scratch stream-ordered (hipMallocAsync/hipFreeAsync)
 * from the device's default pool, so they can be captured in a HIP graph.
 * Errors: 0 = OK, IAT_EINVAL = bad argument (nothing enqueued), IAT_EHIP = HIP runtime
 * error while enqueueing, IAT_EWORKSPACE = workspace too small, IAT_ENOTSUP = unsupported
 * option.  iat_last_error() returns a thread-local message for the last nonzero return.
 * Numerical trouble in a trajectory is never an error return: it sets status bits.
 */
#ifndef IAT_H
#define IAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IAT_EINVAL (-1)
#define IAT_EHIP (-2)
#define IAT_EWORKSPACE (-3)
#define IAT_ENOTSUP (-4)

/* per-trajectory status bits */
#define IAT_ST_COMPLEX      (1u << 0)  /* >= 2 bounces, or still bound at t_max (Fig. 1 text:
                                          a direct collision is a single bounce)            */
#define IAT_ST_BOUND_SEEN   (1u << 1)  /* relative energy < 0 at some accepted step (the
                                          negative-energy bound state of the Eq. (2) text)  */
#define IAT_ST_EXITED       (1u << 2)  /* crossed the exit sphere outward: the normal end  */
#define IAT_ST_TMAX         (1u << 8)  /* reached t_max                                     */
#define IAT_ST_H_UNDERFLOW  (1u << 9)  /* step size fell below hmin                         */
#define IAT_ST_NONFINITE    (1u << 10) /* non-finite state                                  */
#define IAT_ST_MAX_STEPS    (1u << 11) /* accepted-step cap reached                         */
#define IAT_ST_R_UNDERFLOW  (1u << 12) /* separation below 0.1 r_m (integration broken)     */
#define IAT_ST_WARN_R0      (1u << 13) /* start violates 10|V(r0)| < E (head-on-run text)   */
#define IAT_ST_ADJ_SKIPPED  (1u << 14) /* adjoint not computed (no exit or t_max end, or its
                                          checkpoints did not fit the workspace): NaN       */

#define IAT_MAX_SPECIES 8
#define IAT_MAX_STEPS_LIMIT (1LL << 28)   /* largest accepted-step cap (range of the step counters) */

/* One atomic species: mass (m_e) and C4 = alpha/2 (a.u.). */
typedef struct {
    double m_atom;
    double C4;
} iat_species;

/* Trap, per-batch defaults and integrator settings (host struct, copied at call time). */
typedef struct {
    double m_ion;             /* m_e                                                    */
    double omega_rf;          /* Omega, 1/(a.u. time)                                   */
    double a_x, q_x;          /* default Mathieu parameters of the x axis               */
    double a_ratio[3];        /* a_k = a_x * a_ratio[k]; ring trap (1, 1, -2)           */
    double q_ratio[3];        /* q_k = q_x * q_ratio[k]; ring trap (1, 1, -2)           */
    double E;                 /* default collision energy, E_h                          */
    double De;                /* default well depth, E_h                                */
    double phase0;            /* default RF phase Omega t0 at t = 0                     */
    int32_t species;          /* default species index                                  */
    int32_t reserved0;
    double r0;                /* start/exit sphere radius, a0                           */
    double t_max;             /* a.u. time                                              */
    double rtol, atol;        /* error tolerances on the internal state                 */
    double h0, hmax, hmin;    /* tau units; 0 -> 2pi*1e-3, 2pi/8, 1e-6*h0               */
    double r_bounce_over_rm;  /* bounce = periapsis inside this many r_m; 0 -> 1        */
    int64_t max_steps;        /* accepted-step cap (status MAX_STEPS); 0 = no cap short of
                                 IAT_MAX_STEPS_LIMIT; above the limit: IAT_EINVAL         */
} iat_system;

enum { IAT_GEN_ARRAYS = 0, IAT_GEN_GRID = 1, IAT_GEN_SWEEP = 2, IAT_GEN_THERMAL = 3 };

/* How trajectory ids map to parameters.
 *  GRID : cell-centred (theta, phi) grid on the octant (Fig. 1),
 *         theta_j = (j+1/2)(pi/2)/n_theta, phi_k = (k+1/2)(pi/2)/n_phi, id = j*n_phi + k;
 *         E, q_x, De, phase0, species from iat_system.
 *  SWEEP: Philox4x64-10 (Salmon et al., SC'11) blocks (id, 0, 0, 0) and (id, 1, 0, 0) under
 *         key (seed, 0) give uniforms u0..u7 = (x >> 11) 2^-53; cos(theta) = 1 - 2 u0,
 *         phi = 2 pi u1, phase0 = 2 pi u2 (random RF phase of the Fig. 4 runs);
 *         E = E_lo (E_hi/E_lo)^u3 or a list, q_x = q_lo + (q_hi - q_lo) u4 or a list,
 *         De = De_lo (De_hi/De_lo)^u5 or a list.  Lists are indexed by the mixed-radix
 *         digits of cell = id mod (n_species * n_E' * n_q' * n_De') with species slowest
 *         and De fastest (n' = max(n, 1)).
 *  THERMAL: the thermal runs of Fig. 3.  Species, q_x, De, phase0 and the start point as for
 *         SWEEP, with E (list or range) the bath energy k_B T.  Blocks (id, 2..4, 0, 0) give
 *         uniforms w0..w11 and Box-Muller normals z_{2m} = sqrt(-2 ln(1 - w_{2m})) cos(2 pi w_{2m+1}),
 *         z_{2m+1} = the same with sin.  Atom at r0 n on the sphere, velocity
 *         sqrt(k_B T / m_a) (z0, z1, z2), negated when it does not point inward (n . v >= 0);
 *         ion drawn from the thermal distribution at k_B T_ion in the isotropic harmonic trap
 *         omega = q_x Omega / 2^(3/2): position sqrt(k_B T_ion / (m_i omega^2)) (z3, z4, z5),
 *         velocity sqrt(k_B T_ion / m_i) (z6, z7, z8).  A thermal trajectory ends when the atom
 *         crosses the sphere of radius r0 about the trap centre outward (the sphere it started
 *         on; the separation from the displaced ion may start above r0).  y0 must be NULL.
 *  ARRAYS: per-trajectory device arrays in iat_batch (NULL entries take the defaults). */
typedef struct {
    int32_t kind;
    int32_t n_theta, n_phi;
    int32_t n_species;
    int32_t species[IAT_MAX_SPECIES];
    int32_t n_E, n_q, n_De;
    int32_t reserved0;
    double E[8], q[8], De[8];
    double E_lo, E_hi, q_lo, q_hi, De_lo, De_hi;
    uint64_t seed;
    int64_t id0;              /* global id of this call's first trajectory (streaming)  */
    double T_ion;             /* THERMAL: k_B T of the ion's initial distribution (E_h)  */
} iat_gen;

typedef struct {
    int64_t n;                               /* number of trajectories (>= 0)         */
    const double *theta, *phi, *E, *q_x, *De, *phase0;  /* ARRAYS mode, device, or NULL */
    const int32_t* species;                  /* ARRAYS mode, device, or NULL          */
    const double* y0;                        /* 12 x n start states (a.u.), or NULL:
                                                overrides the head-on start (any mode) */
    const int64_t* id0_dev;                  /* device int64, or NULL: added to gen.id0 when the
                                                kernels run, so that one call captured in a HIP
                                                graph can be replayed over successive chunks of a
                                                sweep (the caller keeps grid ids inside the grid;
                                                BOXCOUNT refuses it)                      */
    iat_gen gen;
} iat_batch;

/* Outputs (device, length n, caller-allocated).  Required: angle, q_transfer, dE_ion,
 * t_dwell, n_bounce, status.  Optional (NULL = not written): the rest.
 *   angle      = atan2(|v_i x v_f|, v_i . v_f) of the atom's initial/final velocity,
 *                i.e. arccos(v_i.v_f/(v_i v_f)) (Fig. 1 caption)
 *   q_transfer = m_a |v_f - v_i| (Fig. 1 caption)
 *   dE_ion     = E_ion(t_f) - E_ion(0), E_ion = ion kinetic + trap terms of Eq. (1)
 *   t_dwell    = t_f; t_bounce_first/last = time of the first/last bounce (0 if none)  */
typedef struct {
    double *angle, *q_transfer, *dE_ion, *t_dwell, *t_bounce_first, *t_bounce_last;
    int32_t* n_bounce;
    uint32_t* status;
    int64_t *n_accept, *n_reject, *n_rhs;
    double* y_final;
} iat_obs;

enum { IAT_KERNEL_PLAIN = 1, IAT_KERNEL_PERSISTENT = 2 };

/* Launch shape.  kernel: PLAIN = one lane per trajectory, one launch per batch;
 * PERSISTENT = resident grid whose lanes refill from a device work queue; trajectories that
 * outlive step_budget continue four lanes per trajectory in a second kernel, and the last ones
 * running there finish in a third, one trajectory per wave (see tail_budget).  All kernels give
 * the same bits for the same trajectory.
 * Zero fields take defaults.  stats, if not NULL, is a device uint64[11] to which the
 * call ADDS: [0] RHS evaluations, [1] accepted steps, [2] rejected steps,
 * [3] trajectories finished, [4] issued step slots (one-lane kernels: wave iterations x 64;
 * four-lane kernels: wave iterations x trajectories per wave), [5] useful step slots (attempted
 * steps), [6] RHS evaluations performed inside the four-lane tail kernel, [7] trajectories
 * finished by it, [8] RHS evaluations performed inside the one-per-wave solo kernel,
 * [9] trajectories finished by it; and whose [10] it raises (atomic max) to
 * (attempted steps << 34) | global id of the longest trajectory the call finished (attempted steps
 * = accepted + rejected, clamped to 2^30 - 1; the global id is gen.id0 + index for GRID, SWEEP and
 * THERMAL batches and the index for ARRAYS batches, modulo 2^34): the batch's critical path.
 * kernel_ms, if not NULL, is HOST float[5] that receives the durations of the call's phases on
 * its stream (setup, main integration kernel, four-lane tail kernel, solo kernel, observables),
 * measured with HIP events; the call then waits for its work to finish before returning. */
typedef struct {
    int32_t kernel;
    int32_t block;            /* threads per block: 64, 128, 192 or 256                */
    int32_t blocks_per_cu;    /* PERSISTENT: resident blocks per CU (0 = occupancy max) */
    int32_t refill_every;     /* PERSISTENT: attempted steps between refills (>= 1)    */
    int32_t step_budget;      /* PERSISTENT: attempted steps after which an unfinished
                                 trajectory is suspended and finished by four lanes (one
                                 per axis) to cut the latency of long-lived complexes;
                                 0 = default (20000), -1 = never                         */
    int32_t max_suspended;    /* PERSISTENT: at most this many trajectories are suspended in
                                 one call (continuation records of 248 B each, allocated
                                 with the call's workspace); the others finish in the
                                 one-lane kernel.  0 = min(n, 2^23)                      */
    int32_t tail_budget;      /* PERSISTENT: when a trajectory in the four-lane tail is
                                 suspended again and finished alone in its wave (at most
                                 min(max_suspended, 2^16) of them per call; the others stay
                                 in the tail).  0 = default: once at most 4 per compute unit
                                 (the solo level's waves) of the trajectories that entered the
                                 tail are still running or waiting there; > 0: after this many
                                 attempted steps in the tail; -1 = never                  */
    int32_t reserved;         /* must be 0                                                */
    uint64_t* stats;
    float* kernel_ms;
} iat_launch;

/* Integrate a batch (the paper's head-on runs: model paragraph, head-on-run paragraph,
 * observables of the Fig. 1 caption).  ckpt_ws/ckpt_bytes: reserved, pass NULL/0 (iat_adjoint
 * stores its own checkpoints).  Returns 0 or an error code. */
int iat_integrate(const iat_system* sys, const iat_species* species /* host */, int n_species,
                  const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                  void* ckpt_ws, size_t ckpt_bytes, void* stream);

/* Allocation-free variant of iat_integrate, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as iat_integrate (the same bits per trajectory), except:
 *  - the call's workspace (queue counters, work buffer, continuation records) is a fixed array
 *    inside the library, about 21 MiB per GPU, held from the library's first use on that GPU
 *    until the process ends; the call allocates and frees nothing;
 *  - n <= IAT_NOALLOC_MAX_N (larger: IAT_EINVAL, nothing enqueued); at most 32768 trajectories per
 *    call are suspended to the four-lane tail and 4096 of those to the solo level, the others
 *    finish in the kernel that runs them (same bits);
 *  - launch.kernel_ms must be NULL (phase timing creates events and waits);
 *  - every call on one GPU uses that GPU's one array, which keeps the last call's contents (each
 *    call clears the counters it uses with a fill kernel): calls that can overlap in time on one
 *    GPU (different streams, or different threads) race and must not be issued; calls ordered in
 *    one stream are safe;
 *  - the first call on a device resolves the array's device address (hipGetSymbolAddress): make it
 *    outside stream capture. */
#define IAT_NOALLOC_MAX_N 65536
int iat_integrate_noalloc(const iat_system* sys, const iat_species* species /* host */, int n_species,
                          const iat_batch* batch, const iat_obs* obs, const iat_launch* launch, void* stream);

/* Reductions of a batch's outputs (the ensemble quantities of Figs. 3 and 4, and the fractal
 * structure of Fig. 1).  obs needs dE_ion, n_bounce and status.  out is device memory; CELLS, both W0 histograms and
 * the LIFETIME counts ADD to it (zero it first to start), so chunks of one sweep accumulate;
 * BOXCOUNT overwrites it.
 * IAT_REDUCE_CELLS (SWEEP batches): per cell c (cell = id mod n_cells), out[5c..5c+4] =
 *   (count, complex count, sum dE_ion, sum dE_ion^2, sum n_bounce); sums run in a fixed order.
 * IAT_REDUCE_W0_HIST: per species slot s of the sweep list (slot 0 otherwise), 64 bins of
 *   log10(E/W0) over [-3, 3] (clamped), out[(s*64 + b)*2 + {0,1}] = (total, complex) counts, W0 from
 *   Eq. (2) with omega = (Omega/2) sqrt(a_x + q_x^2/2); then out[n_slots*128 + b], b < 256: counts of
 *   sign(dE) log10(1 + |dE|/(k_B 1 nK)) over +-log10(1 + 1e8) (clamped).
 * IAT_REDUCE_W0_HIST_BOUND: as W0_HIST, with out[(s*64 + b)*2 + 1] counting the trajectories that
 *   reached the negative-energy bound state (IAT_ST_BOUND_SEEN; the temporary atom-ion bound state of
 *   the Eq. (2) text) instead of IAT_ST_COMPLEX.
 * IAT_REDUCE_BOXCOUNT (a whole square power-of-two GRID batch): box-counting dimensions of the
 *   complex-forming set.  For boxes of s = 2^k cells, N_set(k) = boxes holding a complex cell and
 *   N_bnd(k) = boxes holding both kinds; out[0] = D_boundary, out[1] = D_set (least-squares slopes
 *   of log N against log(1/s) over s = 2..64), out[2+2k] = N_set(k), out[3+2k] = N_bnd(k), k = 0..log2(side);
 *   side 2..32768; NaN slopes when fewer than two levels have boxes.
 * IAT_REDUCE_LIFETIME (the complex survival of Fig. 2; obs also needs t_bounce_first and
 *   t_bounce_last): per species slot s (as for W0_HIST), out[98*s + b], b < 96: exited complexes
 *   (>= 2 bounces) by log10((t_last - t_first bounce)/1 us) over [-2, 4] (clamped);
 *   out[98*s + 96]: complexes still bound at t_max or at the step cap (censored, alive
 *   throughout); out[98*n_slots + s] = the power-law exponent alpha of the survival fraction,
 *   S(t) ~ t^-alpha, least squares of log S against log t over bin edges t >= 20 us, from the
 *   accumulated counts (overwritten by every call; NaN below two points).
 */
#define IAT_REDUCE_CELLS 1
#define IAT_REDUCE_W0_HIST 2
#define IAT_REDUCE_BOXCOUNT 3
#define IAT_REDUCE_LIFETIME 4
#define IAT_REDUCE_W0_HIST_BOUND 5
int iat_reduce(const iat_system* sys, const iat_species* species, int n_species,
               const iat_batch* batch, const iat_obs* obs, int kind, double* out, void* stream);

/* Tangent-linear of the accepted-step map (internal differentiation: the tangent columns
 * obey the same Runge-Kutta scheme with the primal's step sequence).  Per trajectory:
 * dobs_dp[15*n] = d(angle, q_transfer, dE_ion)/d(theta, phi, E, q_x, De), laid out
 * [j*15 + 5*i + p]; ftle[n] = ln(sigma_max(Phi(t_f, 0)))/t_f (per a.u. time), Phi the
 * 12x12 stability matrix of the internal state; lyap[12*n] or NULL: the finite-time Lyapunov
 * spectrum ln(sigma_k(D Phi D^-1))/t_f, descending, D = sqrt(mass) on each coordinate (the
 * canonical scaling in which Phi is symplectic, so the exponents pair as +-lambda up to the
 * integrator's truncation error); exponents whose sigma_k^2 falls below ~1e-15 sigma_max^2 are
 * set by rounding (their pairs are the reliable values), and NaN where sigma_k^2 rounds to <= 0;
 * Phi_out[144*n] (row-major per trajectory, internal units) or NULL.  Columns that grow past
 * 2^400 are rescaled as they go
 * (exponents tracked per column); Phi_out holds Phi * 2^-e with e the largest column exponent,
 * so e = 0 and Phi_out = Phi unless the stretching passed 2^400 (long-lived complexes), and ftle
 * and lyap account for e.  Head-on GRID/SWEEP/ARRAYS batches only; y0 and THERMAL batches are
 * rejected (IAT_ENOTSUP).
 * Workspace: one device allocation of n*(22*8 + 5*4 + 14*13*8 + 14*4 [+ 144*8 when Phi_out is
 * NULL and ftle or lyap is not]) bytes, stream-ordered on the given stream. */
int iat_integrate_tangent(const iat_system* sys, const iat_species* species, int n_species,
                          const iat_batch* batch, const iat_obs* obs, double* dobs_dp, double* ftle,
                          double* lyap, double* Phi_out, const iat_launch* launch, void* stream);

/* Discrete adjoint of the accepted-step map (the sensitivities of the scattering observables of
 * the Fig. 1 caption to the start and model parameters).  Per trajectory j:
 *   p_bar[5*j + p] = d/dp sum_k obs_bar[3*j + k] obs_k,   obs = (angle, q_transfer, dE_ion),
 *   p = (theta, phi, E, q_x, De),
 * the exact derivative of the same discrete map that iat_integrate_tangent differentiates
 * (accepted steps with their sizes frozen, the exit time moved by the event |r_a - r_i| = r0).
 * obs must hold the iat_integrate outputs of this same batch: n_accept (device int64[n]) sizes
 * the checkpoints (one every 256 accepted steps, 192 bytes each), status selects the
 * trajectories (exited or t_max); the call sets IAT_ST_ADJ_SKIPPED in obs.status and writes NaN
 * to p_bar for the others, and for any trajectory whose checkpoints do not fit ws.
 * obs_bar: device double[3*n]; p_bar: device double[5*n]; y0_bar: device double[12*n] or NULL,
 * receiving dJ/dy0 for the start state in a.u. (atom and ion positions in a0, velocities in a.u.;
 * the explicit dependence of the angle and q on the start velocity included).
 * ws/ws_bytes: device workspace of at least iat_adjoint_workspace_bytes() bytes; ws = NULL makes
 * the call size (one stream synchronisation) and allocate it itself, stream-ordered.
 * Head-on GRID/SWEEP/ARRAYS batches only (y0 batches: IAT_ENOTSUP).  Gradients that pass the
 * double range come out as +-inf. */
int iat_adjoint(const iat_system* sys, const iat_species* species, int n_species,
                const iat_batch* batch, const iat_obs* obs, const double* obs_bar, double* p_bar,
                double* y0_bar, void* ws, size_t ws_bytes, const iat_launch* launch, void* stream);

/* Device workspace bytes iat_adjoint needs for this batch (reads obs.n_accept and obs.status of
 * its iat_integrate run on the stream and synchronises it). */
int iat_adjoint_workspace_bytes(const iat_system* sys, const iat_species* species, int n_species,
                                const iat_batch* batch, const iat_obs* obs, size_t* bytes, void* stream);

/* Device workspace of one call, for callers that budget device memory before it (the integration,
 * reduction and adjoint of the batched trajectories above; the calls themselves allocate and free
 * what they need, stream-ordered, unless a workspace is passed in).  which:
 *   IAT_WS_INTEGRATE  bytes iat_integrate allocates for this batch and launch (launch may be NULL:
 *                     defaults): 256 B of counters, the work buffer (196 B per trajectory) and the
 *                     continuation records of the tail and solo levels (248 B each); host only;
 *   IAT_WS_REDUCE     bytes iat_reduce of kind reduce_kind allocates for this batch (CELLS: partial
 *                     sums per cell and slice; BOXCOUNT: level flags; the histogram kinds: 0); host only;
 *   IAT_WS_ADJOINT    as iat_adjoint_workspace_bytes (reads obs of the forward run on `stream` and
 *                     synchronises it).
 * obs and stream are used by IAT_WS_ADJOINT only, reduce_kind by IAT_WS_REDUCE only.  Writes *bytes
 * (host); returns the validation errors of the call it sizes, IAT_EINVAL for an unknown `which`. */
#define IAT_WS_INTEGRATE 1
#define IAT_WS_REDUCE 2
#define IAT_WS_ADJOINT 3
int iat_workspace_bytes(int which, const iat_system* sys, const iat_species* species, int n_species,
                        const iat_batch* batch, const iat_obs* obs, const iat_launch* launch, int reduce_kind,
                        size_t* bytes, void* stream);

/* Diagnostics: the FP64 rate this GPU sustains on independent FMAs (eight chains per lane,
 * n_threads lanes, a multiple of 256, `iters` x 64 FMAs each), timed with HIP events on the
 * stream; writes TFLOP/s to *tflops (host).  scratch: device double[n_threads] (written).  The
 * call waits for its kernel.  Not part of the method: the measured denominator next to the
 * published FP64 vector peak. */
int iat_fp64_peak(double* scratch, int64_t n_threads, int iters, double* tflops, void* stream);

const char* iat_last_error(void);
/* Library version string. */
const char* iat_version(void);
/* Forget cached device attributes and trim the memory that the library's stream-ordered
 * allocations left in each device's default pool; safe to call at exit. */
void iat_release(void);

#ifdef __cplusplus
}
#endif
#endif
