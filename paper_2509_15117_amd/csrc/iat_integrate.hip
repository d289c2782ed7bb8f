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

namespace iat {

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

__global__ void __launch_bounds__(256) k_integrate_plain(KParams P)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    LaneStats st;
    uint64_t iters = 0;
    if (i < P.n) {
        Traj T;
        traj_start(P, i, T);
        while (!T.done) {
            traj_advance(P, T);
            ++iters;
        }
        traj_finish(P, i, T);
        st.rhs = T.nrhs;
        st.acc = T.nacc;
        st.rej = T.nrej;
        st.done = 1;
        st.useful = T.nacc + T.nrej;
    }
    // every lane of the wave is issued for as many steps as its slowest lane needed
    flush_stats(P.stats, st, 64ull * wave_max(iters));
}

__global__ void __launch_bounds__(256) k_integrate_persistent(KParams P, unsigned long long* queue)
{
    const int lane = __lane_id();
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    LaneStats st;
    uint64_t iters = 0;
    Traj T;
    int64_t i = -1;
    bool active = false, need = true;
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
                if (active) traj_start(P, i, T);
                need = false;
            }
        }
        if (!__any(active)) break;
        for (int k = 0; k < P.refill_every; ++k) {
            if (active && !T.done) traj_advance(P, T);
        }
        iters += P.refill_every;
        if (active && T.done) {
            traj_finish(P, i, T);
            st.rhs += T.nrhs;
            st.acc += T.nacc;
            st.rej += T.nrej;
            st.done += 1;
            st.useful += T.nacc + T.nrej;
            active = false;
            need = true;
        }
    }
    flush_stats(P.stats, st, 64ull * iters);
}

__global__ void k_reset_counter(unsigned long long* q) { *q = 0ull; }

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
constexpr int kQueueSlots = 256;
struct DeviceState {
    unsigned long long* queues = nullptr;
    std::atomic<unsigned> next{0};
    int n_cu = 0;
};
DeviceState g_dev[kMaxDevices];
std::mutex g_mu;
}  // namespace

int device_state(int* n_cu, unsigned long long** queue_slot)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(IAT_EHIP, "hipGetDevice failed");
    DeviceState& d = g_dev[dev];
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!d.queues) {
            void* p = nullptr;
            if (hipMalloc(&p, sizeof(unsigned long long) * kQueueSlots) != hipSuccess)
                return set_error(IAT_EHIP, "hipMalloc of the work-queue counters failed");
            d.queues = (unsigned long long*)p;
            if (hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                return set_error(IAT_EHIP, "hipDeviceGetAttribute failed");
        }
    }
    if (n_cu) *n_cu = d.n_cu;
    if (queue_slot) *queue_slot = d.queues + (d.next.fetch_add(1) % kQueueSlots);
    return 0;
}

void release_devices()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& d : g_dev) {
        if (d.queues) (void)hipFree(d.queues);
        d.queues = nullptr;
    }
}

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
    *out = L;
    return 0;
}

}  // namespace iat

using namespace iat;

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
    if (L.kernel == IAT_KERNEL_PLAIN) {
        const int64_t blocks = (batch->n + L.block - 1) / L.block;
        if (blocks > 0x7fffffffLL) return set_error(IAT_EINVAL, "batch too large for one launch");
        hipLaunchKernelGGL(k_integrate_plain, dim3((unsigned)blocks), dim3(L.block), 0, st, P);
    } else {
        int n_cu = 0;
        unsigned long long* q = nullptr;
        rc = device_state(&n_cu, &q);
        if (rc) return rc;
        int per_cu = L.blocks_per_cu;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_integrate_persistent, L.block,
                                                             0) != hipSuccess || per_cu < 1)
                per_cu = 1;
        }
        int64_t blocks = (int64_t)n_cu * per_cu;
        const int64_t need = (batch->n + L.block - 1) / L.block;
        if (blocks > need) blocks = need;
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, q);
        hipLaunchKernelGGL(k_integrate_persistent, dim3((unsigned)blocks), dim3(L.block), 0, st, P, q);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return 0;
}

extern "C" const char* iat_last_error(void) { return iat::last_error(); }
extern "C" const char* iat_version(void) { return "libiat 0.1 (gfx950)"; }
extern "C" void iat_release(void) { iat::release_devices(); }
