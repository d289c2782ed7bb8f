// Batch integration kernels of libiat and the iat_integrate entry point.
//
// PLAIN      : one lane per trajectory; a wave runs until its slowest lane has finished.
// PERSISTENT : a resident grid; whenever lanes finish, the wave takes as many new ids from a
//              device counter as it has free lanes (one atomic per wave, ids handed out by
//              ballot rank), so long-lived complexes do not hold idle lanes hostage.
// Both call the same device step (iat_device.h): a trajectory gives identical bits in both.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "iat_device.h"
#include "iat_host.h"

#include <algorithm>

namespace iat {

constexpr int64_t kDefaultBudget = 20000;        // attempted steps before a trajectory moves to 4 lanes
constexpr int64_t kMaxSuspended = 1 << 23;       // continuation records per call (248 B each)

__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ uint64_t wave_max(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

struct LaneStats {
    uint64_t rhs = 0, acc = 0, rej = 0, done = 0, useful = 0;
};

__device__ __forceinline__ void flush_stats(uint64_t* stats, const LaneStats& s, uint64_t issued)
{
    if (!stats) return;
    const uint64_t r = wave_sum(s.rhs), a = wave_sum(s.acc), j = wave_sum(s.rej), d = wave_sum(s.done),
                   u = wave_sum(s.useful);
    if (__lane_id() == 0) {
        atomicAdd((unsigned long long*)&stats[0], (unsigned long long)r);
        atomicAdd((unsigned long long*)&stats[1], (unsigned long long)a);
        atomicAdd((unsigned long long*)&stats[2], (unsigned long long)j);
        atomicAdd((unsigned long long*)&stats[3], (unsigned long long)d);
        atomicAdd((unsigned long long*)&stats[4], (unsigned long long)issued);
        atomicAdd((unsigned long long*)&stats[5], (unsigned long long)u);
    }
}

__global__ void __launch_bounds__(256) k_setup(KParams P, Work W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) work_setup(P, W, i);
}

__global__ void __launch_bounds__(256) k_observe(KParams P, Work W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.n) work_observe(P, W, i);
}

__global__ void __launch_bounds__(256) k_integrate_plain(KParams P, Work W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    LaneStats st;
    uint64_t iters = 0;
    if (i < P.n) {
        Traj1 T;
        traj1_start(P, W, i, T);
        while (!T.S.done) {
            traj1_advance(P, T);
            ++iters;
        }
        traj1_store(W, i, T);
        st.rhs = T.S.nrhs;
        st.acc = T.S.nacc;
        st.rej = T.S.nrej;
        st.done = 1;
        st.useful = T.S.nacc + T.S.nrej;
    }
    // every lane of the wave is issued for as many steps as its slowest lane needed
    flush_stats(P.stats, st, 64ull * wave_max(iters));
}

// Persistent refill kernel.  A trajectory that has used `budget` attempted steps without
// finishing is suspended into the continuation records (while slots last) and its lane takes
// new work; k_integrate_tail finishes the suspended ones four lanes per trajectory.
__global__ void __launch_bounds__(256) k_integrate_persistent(KParams P, Work W, unsigned long long* queue, Cont C)
{
    const int lane = __lane_id();
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    LaneStats st;
    uint64_t iters = 0;
    Traj1 T;
    int64_t i = -1;
    bool active = false, need = true, may_suspend = P.budget > 0;
    for (;;) {
        // hand out new ids to the lanes that need one: one atomic per wave
        const uint64_t mask = __ballot(need);
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(mask));
            base = __shfl(base, leader, 64);
            if (need) {
                i = (int64_t)(base + __popcll(mask & lanemask_lt));
                active = i < P.n;
                if (active) traj1_start(P, W, i, T);
                need = false;
            }
        }
        if (!__any(active)) break;
        for (int k = 0; k < P.refill_every; ++k) {
            if (active && !T.S.done) traj1_advance(P, T);
        }
        iters += P.refill_every;
        if (active) {
            if (T.S.done) {
                traj1_store(W, i, T);
                st.rhs += T.S.nrhs;
                st.acc += T.S.nacc;
                st.rej += T.S.nrej;
                st.done += 1;
                st.useful += T.S.nacc + T.S.nrej;
                active = false;
                need = true;
            } else if (may_suspend && T.S.nacc + T.S.nrej >= P.budget) {
                const unsigned long long slot = atomicAdd(C.count, 1ull);
                if ((int64_t)slot < C.cap) {
                    cont_save(C, (int64_t)slot, i, T);
                    st.useful += T.S.nacc + T.S.nrej;
                    active = false;
                    need = true;
                } else {
                    may_suspend = false;
                }
            }
        }
    }
    flush_stats(P.stats, st, 64ull * iters);
}

// Finishes suspended trajectories with four lanes each (one per axis): the per-step latency of
// a long-lived complex is what bounds a batch's wall time.
__global__ void __launch_bounds__(256) k_integrate_tail(KParams P, Work W, Cont C)
{
    const int lane = __lane_id();
    const int qlead = lane & ~3;
    const bool leader = (lane & 3) == 0;
    const uint64_t lt = (qlead == 0) ? 0ull : (~0ull >> (64 - qlead));
    const int k = quad_axis();
    unsigned long long cnt = *C.count;
    const int64_t total = (int64_t)(cnt < (unsigned long long)C.cap ? cnt : (unsigned long long)C.cap);
    LaneStats st;
    uint64_t iters = 0;
    Traj4 T;
    int64_t i = -1;
    int32_t resumed_at = 0, resumed_rhs = 0;
    uint64_t tail_rhs = 0, tail_done = 0;
    bool active = false, need = true;
    for (;;) {
        const uint64_t mask = __ballot(need && leader);
        if (mask) {
            const int first = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(C.head, (unsigned long long)__popcll(mask));
            base = __shfl(base, first, 64);
            if (need) {
                const int64_t slot = (int64_t)(base + __popcll(mask & lt));
                active = slot < total;
                if (active) {
                    cont_load4(P, W, C, slot, k, T, i);
                    resumed_at = T.S.nacc + T.S.nrej;
                    resumed_rhs = T.S.nrhs;
                }
                need = false;
            }
        }
        if (!__any(active)) break;
        if (active && !T.S.done) traj4_advance(P, T);
        ++iters;
        if (active && T.S.done) {
            traj4_store(W, i, T, lane & 3);
            if (leader) {
                st.rhs += T.S.nrhs;
                st.acc += T.S.nacc;
                st.rej += T.S.nrej;
                st.done += 1;
                st.useful += T.S.nacc + T.S.nrej - resumed_at;
                tail_rhs += (uint64_t)(T.S.nrhs - resumed_rhs);
                tail_done += 1;
            }
            active = false;
            need = true;
        }
    }
    // a wave carries 16 trajectories: 16 step slots per iteration
    flush_stats(P.stats, st, 0ull);
    if (P.stats) {
        const uint64_t tr = wave_sum(tail_rhs), td = wave_sum(tail_done);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&P.stats[4], (unsigned long long)(16ull * iters));
            atomicAdd((unsigned long long*)&P.stats[6], (unsigned long long)tr);
            atomicAdd((unsigned long long*)&P.stats[7], (unsigned long long)td);
        }
    }
}

__global__ void k_reset_counters(unsigned long long* q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
}

}  // namespace iat

// ------------------------------------------------------------------------------- host side
namespace iat {

static thread_local char g_err[1024];

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

const char* last_error() { return g_err; }

namespace {
constexpr int kMaxDevices = 64;
int g_n_cu[kMaxDevices];
std::mutex g_mu;
}  // namespace

// Compute-unit count of the current device (cached).
int device_state(int* n_cu, unsigned long long** unused)
{
    (void)unused;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(IAT_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_n_cu[dev] == 0 &&
        hipDeviceGetAttribute(&g_n_cu[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return set_error(IAT_EHIP, "hipDeviceGetAttribute failed");
    if (n_cu) *n_cu = g_n_cu[dev];
    return 0;
}

void release_devices() {}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int validate_common(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch)
{
    if (!sys || !species || !batch) return set_error(IAT_EINVAL, "NULL sys, species or batch");
    if (n_species < 1 || n_species > IAT_MAX_SPECIES)
        return set_error(IAT_EINVAL, "n_species must be in [1, %d]", IAT_MAX_SPECIES);
    for (int s = 0; s < n_species; ++s)
        if (!finite_pos(species[s].m_atom) || !finite_pos(species[s].C4))
            return set_error(IAT_EINVAL, "species %d: m_atom and C4 must be finite and > 0", s);
    if (!finite_pos(sys->m_ion) || !finite_pos(sys->omega_rf))
        return set_error(IAT_EINVAL, "m_ion and omega_rf must be finite and > 0");
    if (!finite_pos(sys->r0) || !finite_pos(sys->t_max)) return set_error(IAT_EINVAL, "r0 and t_max must be > 0");
    if (!finite_pos(sys->rtol) || !finite_pos(sys->atol)) return set_error(IAT_EINVAL, "rtol and atol must be > 0");
    if (sys->h0 < 0 || sys->hmax < 0 || sys->hmin < 0 || sys->r_bounce_over_rm < 0 || sys->max_steps < 0)
        return set_error(IAT_EINVAL, "h0, hmax, hmin, r_bounce_over_rm and max_steps must be >= 0");
    if (sys->t_max * sys->omega_rf + std::fabs(sys->phase0) > 1.5e6)
        return set_error(IAT_EINVAL, "Omega t_max must stay below 1.5e6 RF radians (phase reduction range)");
    if (sys->hmax > kTwoPi / 8.0)
        return set_error(IAT_EINVAL, "hmax must not exceed pi/4 (an eighth of the RF period in tau units)");
    if (!std::isfinite(sys->a_x) || !std::isfinite(sys->q_x) || !std::isfinite(sys->phase0))
        return set_error(IAT_EINVAL, "a_x, q_x and phase0 must be finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(sys->a_ratio[k]) || !std::isfinite(sys->q_ratio[k]))
            return set_error(IAT_EINVAL, "a_ratio and q_ratio must be finite");
    if (sys->species < 0 || sys->species >= n_species) return set_error(IAT_EINVAL, "default species out of range");
    if (batch->n < 0) return set_error(IAT_EINVAL, "batch n < 0");
    const iat_gen& g = batch->gen;
    if (g.kind == IAT_GEN_GRID) {
        if (g.n_theta < 1 || g.n_phi < 1) return set_error(IAT_EINVAL, "grid n_theta and n_phi must be >= 1");
        if (g.id0 < 0 || g.id0 + batch->n > (int64_t)g.n_theta * g.n_phi)
            return set_error(IAT_EINVAL, "grid ids [id0, id0 + n) exceed n_theta * n_phi");
    } else if (g.kind == IAT_GEN_SWEEP) {
        if (g.n_species < 1 || g.n_species > IAT_MAX_SPECIES)
            return set_error(IAT_EINVAL, "sweep n_species must be in [1, %d]", IAT_MAX_SPECIES);
        for (int s = 0; s < g.n_species; ++s)
            if (g.species[s] < 0 || g.species[s] >= n_species)
                return set_error(IAT_EINVAL, "sweep species[%d] out of range", s);
        if (g.n_E < 0 || g.n_E > 8 || g.n_q < 0 || g.n_q > 8 || g.n_De < 0 || g.n_De > 8)
            return set_error(IAT_EINVAL, "sweep list lengths must be in [0, 8]");
        for (int k = 0; k < g.n_E; ++k)
            if (!finite_pos(g.E[k])) return set_error(IAT_EINVAL, "sweep E list entries must be > 0");
        for (int k = 0; k < g.n_De; ++k)
            if (!finite_pos(g.De[k])) return set_error(IAT_EINVAL, "sweep De list entries must be > 0");
        for (int k = 0; k < g.n_q; ++k)
            if (!std::isfinite(g.q[k])) return set_error(IAT_EINVAL, "sweep q list entries must be finite");
        if (g.n_E == 0 && !(finite_pos(g.E_lo) && finite_pos(g.E_hi) && g.E_hi >= g.E_lo))
            return set_error(IAT_EINVAL, "sweep E range needs 0 < E_lo <= E_hi");
        if (g.n_De == 0 && !(finite_pos(g.De_lo) && finite_pos(g.De_hi) && g.De_hi >= g.De_lo))
            return set_error(IAT_EINVAL, "sweep De range needs 0 < De_lo <= De_hi");
        if (g.n_q == 0 && !(std::isfinite(g.q_lo) && std::isfinite(g.q_hi) && g.q_hi >= g.q_lo))
            return set_error(IAT_EINVAL, "sweep q range needs q_lo <= q_hi");
        if (g.id0 < 0) return set_error(IAT_EINVAL, "id0 must be >= 0");
    } else if (g.kind == IAT_GEN_ARRAYS) {
        if (!batch->y0 && (!batch->theta || !batch->phi))
            return set_error(IAT_EINVAL, "ARRAYS batches need theta and phi, or y0");
    } else {
        return set_error(IAT_EINVAL, "unknown generator kind %d", g.kind);
    }
    if (!batch->E && !finite_pos(sys->E) && !batch->y0 && g.kind != IAT_GEN_SWEEP)
        return set_error(IAT_EINVAL, "collision energy E must be > 0");
    if (!batch->De && !finite_pos(sys->De) && !(g.kind == IAT_GEN_SWEEP))
        return set_error(IAT_EINVAL, "well depth De must be > 0");
    return 0;
}

void fill_params(KParams& P, const iat_system* sys, const iat_species* species, int n_species,
                 const iat_batch* batch)
{
    std::memset(&P, 0, sizeof(P));
    P.omega = sys->omega_rf;
    P.m_ion = sys->m_ion;
    P.a_x = sys->a_x;
    P.q_x = sys->q_x;
    for (int k = 0; k < 3; ++k) {
        P.a_ratio[k] = sys->a_ratio[k];
        P.q_ratio[k] = sys->q_ratio[k];
    }
    P.E = sys->E;
    P.De = sys->De;
    P.phase0 = sys->phase0;
    P.species = sys->species;
    P.n_species = n_species;
    P.r0 = sys->r0;
    P.r0sq = sys->r0 * sys->r0;
    P.tau_max = sys->t_max * sys->omega_rf;
    P.rtol = sys->rtol;
    P.atol = sys->atol;
    P.h0 = sys->h0 > 0 ? sys->h0 : kTwoPi * 1e-3;
    P.hmax = sys->hmax > 0 ? sys->hmax : kTwoPi / 8.0;
    P.hmin = sys->hmin > 0 ? sys->hmin : 1e-6 * P.h0;
    P.r_bounce_over_rm = sys->r_bounce_over_rm > 0 ? sys->r_bounce_over_rm : 1.0;
    P.rb_ratio2 = P.r_bounce_over_rm * P.r_bounce_over_rm;
    P.inv_mi = 1.0 / sys->m_ion;
    for (int k = 0; k < 3; ++k) P.kA[k] = 0.25 * (sys->a_x * sys->a_ratio[k]);
    P.max_steps = sys->max_steps > 0 ? sys->max_steps : IAT_DEFAULT_MAX_STEPS;
    for (int s = 0; s < n_species; ++s) {
        P.sp_m[s] = species[s].m_atom;
        P.sp_C4[s] = species[s].C4;
    }
    P.n = batch->n;
    P.theta = batch->theta;
    P.phi = batch->phi;
    P.E_arr = batch->E;
    P.qx_arr = batch->q_x;
    P.De_arr = batch->De;
    P.phase_arr = batch->phase0;
    P.sp_arr = batch->species;
    P.y0 = batch->y0;
    P.gen = batch->gen;
}

void fill_outputs(KParams& P, const iat_obs* obs)
{
    P.angle = obs->angle;
    P.q_transfer = obs->q_transfer;
    P.dE_ion = obs->dE_ion;
    P.t_dwell = obs->t_dwell;
    P.t_first = obs->t_bounce_first;
    P.t_last = obs->t_bounce_last;
    P.n_bounce = obs->n_bounce;
    P.status = obs->status;
    P.n_accept = obs->n_accept;
    P.n_reject = obs->n_reject;
    P.n_rhs = obs->n_rhs;
    P.y_final = obs->y_final;
}

// Optional phase timing with HIP events on the call's stream (launch.kernel_ms).
PhaseTimer::PhaseTimer(float* out, hipStream_t st) : out_(out), st_(st)
{
    if (!out_) return;
    for (int k = 0; k < 5; ++k)
        if (hipEventCreate(&ev_[k]) != hipSuccess) ev_[k] = nullptr;
}
void PhaseTimer::mark(int k)
{
    if (out_ && ev_[k]) (void)hipEventRecord(ev_[k], st_);
}
int PhaseTimer::finish()
{
    if (!out_) return 0;
    int rc = 0;
    if (hipEventSynchronize(ev_[4]) != hipSuccess) rc = set_error(IAT_EHIP, "timing: hipEventSynchronize failed");
    for (int k = 0; k < 4 && rc == 0; ++k)
        if (hipEventElapsedTime(&out_[k], ev_[k], ev_[k + 1]) != hipSuccess)
            rc = set_error(IAT_EHIP, "timing: hipEventElapsedTime failed");
    return rc;
}
PhaseTimer::~PhaseTimer()
{
    if (!out_) return;
    for (int k = 0; k < 5; ++k)
        if (ev_[k]) (void)hipEventDestroy(ev_[k]);
}

int resolve_launch(const iat_launch* launch, iat_launch* out)
{
    iat_launch L{};
    if (launch) L = *launch;
    if (L.kernel == 0) L.kernel = IAT_KERNEL_PERSISTENT;
    if (L.kernel != IAT_KERNEL_PLAIN && L.kernel != IAT_KERNEL_PERSISTENT)
        return set_error(IAT_EINVAL, "launch.kernel must be IAT_KERNEL_PLAIN or IAT_KERNEL_PERSISTENT");
    if (L.block == 0) L.block = 256;
    if (L.block < 64 || L.block > 256 || L.block % 64 != 0)
        return set_error(IAT_EINVAL, "launch.block must be 64, 128, 192 or 256");
    if (L.blocks_per_cu < 0) return set_error(IAT_EINVAL, "launch.blocks_per_cu must be >= 0");
    if (L.refill_every == 0) L.refill_every = 1;
    if (L.refill_every < 1 || L.refill_every > 4096)
        return set_error(IAT_EINVAL, "launch.refill_every must be in [1, 4096]");
    if (L.step_budget < -1) return set_error(IAT_EINVAL, "launch.step_budget must be >= -1");
    *out = L;
    return 0;
}

}  // namespace iat

using namespace iat;

namespace iat {
void launch_setup(const KParams& P, const Work& W, hipStream_t st)
{
    hipLaunchKernelGGL(k_setup, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, W);
}
void launch_observe(const KParams& P, const Work& W, hipStream_t st)
{
    hipLaunchKernelGGL(k_observe, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, W);
}
}  // namespace iat

extern "C" int iat_integrate(const iat_system* sys, const iat_species* species, int n_species,
                             const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                             void* ckpt_ws, size_t ckpt_bytes, void* stream)
{
    int rc = validate_common(sys, species, n_species, batch);
    if (rc) return rc;
    if (!obs) return set_error(IAT_EINVAL, "obs is NULL");
    if (batch->n > 0 &&
        (!obs->angle || !obs->q_transfer || !obs->dE_ion || !obs->t_dwell || !obs->n_bounce || !obs->status))
        return set_error(IAT_EINVAL, "obs: angle, q_transfer, dE_ion, t_dwell, n_bounce and status are required");
    if (ckpt_ws || ckpt_bytes)
        return set_error(IAT_ENOTSUP, "checkpointing is done by iat_adjoint itself; pass NULL/0");
    iat_launch L;
    rc = resolve_launch(launch, &L);
    if (rc) return rc;
    if (batch->n == 0) return 0;
    KParams P;
    fill_params(P, sys, species, n_species, batch);
    fill_outputs(P, obs);
    P.stats = L.stats;
    P.refill_every = L.refill_every;
    hipStream_t st = (hipStream_t)stream;
    int n_cu = 0;
    rc = device_state(&n_cu, nullptr);
    if (rc) return rc;
    const int64_t n = batch->n;
    if (n > (int64_t)0x7fffffff * 256) return set_error(IAT_EINVAL, "batch too large for one launch");
    const unsigned nblk = (unsigned)((n + 255) / 256);
    P.budget = 0;
    int64_t cap = 0;
    if (L.kernel == IAT_KERNEL_PERSISTENT) {
        P.budget = L.step_budget > 0 ? L.step_budget : (L.step_budget == 0 ? kDefaultBudget : 0);
        cap = P.budget > 0 ? std::min<int64_t>(n, kMaxSuspended) : 0;
    }
    // one stream-ordered block: queue counters | work buffer | continuation records
    const size_t rec = 26 * sizeof(double) + 8 * sizeof(int32_t) + sizeof(int64_t);
    const size_t work_bytes = (size_t)n * (kWorkDoubles * sizeof(double) + kWorkInts * sizeof(int32_t));
    const size_t bytes = 256 + ((work_bytes + 255) / 256) * 256 + (size_t)cap * rec;
    void* ws = nullptr;
    if (hipMallocAsync(&ws, bytes, st) != hipSuccess) return set_error(IAT_EHIP, "hipMallocAsync of %zu bytes failed", bytes);
    unsigned long long* q = (unsigned long long*)ws;
    Work W;
    W.n = n;
    W.D = (double*)((char*)ws + 256);
    W.I = (int32_t*)(W.D + (size_t)kWorkDoubles * n);
    Cont C;
    C.count = q + 1;
    C.head = q + 2;
    C.cap = cap;
    C.d = (double*)((char*)ws + 256 + ((work_bytes + 255) / 256) * 256);
    C.n = (int32_t*)(C.d + 26 * cap);
    C.id = (int64_t*)(C.n + 8 * cap);
    PhaseTimer timer(L.kernel_ms, st);
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, q, 4);
    timer.mark(0);
    hipLaunchKernelGGL(k_setup, dim3(nblk), dim3(256), 0, st, P, W);
    timer.mark(1);
    if (L.kernel == IAT_KERNEL_PLAIN) {
        hipLaunchKernelGGL(k_integrate_plain, dim3((unsigned)((n + L.block - 1) / L.block)), dim3(L.block), 0, st, P, W);
    } else {
        int per_cu = L.blocks_per_cu;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_integrate_persistent, L.block,
                                                             0) != hipSuccess || per_cu < 1)
                per_cu = 1;
        }
        int64_t blocks = (int64_t)n_cu * per_cu;
        const int64_t need = (n + L.block - 1) / L.block;
        if (blocks > need) blocks = need;
        hipLaunchKernelGGL(k_integrate_persistent, dim3((unsigned)blocks), dim3(L.block), 0, st, P, W, q, C);
        timer.mark(2);
        if (cap > 0) {
            int per_cu4 = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu4, (const void*)k_integrate_tail, 256, 0) !=
                    hipSuccess || per_cu4 < 1)
                per_cu4 = 1;
            int64_t blocks4 = (int64_t)n_cu * per_cu4;
            const int64_t need4 = (4 * cap + 255) / 256;
            if (blocks4 > need4) blocks4 = need4;
            hipLaunchKernelGGL(k_integrate_tail, dim3((unsigned)blocks4), dim3(256), 0, st, P, W, C);
        }
    }
    if (L.kernel == IAT_KERNEL_PLAIN) timer.mark(2);
    timer.mark(3);
    hipLaunchKernelGGL(k_observe, dim3(nblk), dim3(256), 0, st, P, W);
    timer.mark(4);
    if (hipFreeAsync(ws, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return timer.finish();
}

extern "C" const char* iat_last_error(void) { return iat::last_error(); }
extern "C" const char* iat_version(void) { return "libiat 0.1 (gfx950)"; }
extern "C" void iat_release(void) { iat::release_devices(); }
