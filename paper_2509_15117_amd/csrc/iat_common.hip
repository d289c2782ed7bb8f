// Host-side helpers shared by the libiat entry points: error strings, per-device attributes,
// argument validation, kernel parameter blocks, launch shapes and phase timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "iat_device.h"
#include "iat_host.h"

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
int device_state(int* n_cu)
{
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

// Forget the cached device attributes and hand the memory that the stream-ordered allocations of
// this library left in each device's default pool back to the runtime.
void release_devices()
{
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    for (int d = 0; d < kMaxDevices; ++d) {
        if (g_n_cu[d] == 0) continue;
        g_n_cu[d] = 0;
        hipMemPool_t pool;
        if (hipSetDevice(d) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess)
            (void)hipMemPoolTrimTo(pool, 0);
    }
    if (have_cur) (void)hipSetDevice(cur);
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
    if (sys->max_steps > IAT_MAX_STEPS_LIMIT)
        return set_error(IAT_EINVAL, "max_steps %lld is above the limit of the step counters (%lld)",
                         (long long)sys->max_steps, (long long)IAT_MAX_STEPS_LIMIT);
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
    } else if (g.kind == IAT_GEN_SWEEP || g.kind == IAT_GEN_THERMAL) {
        if (g.kind == IAT_GEN_THERMAL) {
            if (!(g.T_ion >= 0.0) || !std::isfinite(g.T_ion))
                return set_error(IAT_EINVAL, "thermal T_ion must be finite and >= 0");
            if (batch->y0) return set_error(IAT_EINVAL, "thermal batches draw their own start states (y0 must be NULL)");
            const bool qpos = g.n_q > 0 ? true : g.q_lo > 0.0;
            for (int k = 0; k < g.n_q; ++k) if (!(g.q[k] > 0.0)) return set_error(IAT_EINVAL, "thermal q_x must be > 0");
            if (!qpos) return set_error(IAT_EINVAL, "thermal q_x must be > 0 (it sets the ion's trap frequency)");
        }
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
    if (!batch->E && !finite_pos(sys->E) && !batch->y0 && g.kind != IAT_GEN_SWEEP && g.kind != IAT_GEN_THERMAL)
        return set_error(IAT_EINVAL, "collision energy E must be > 0");
    if (!batch->De && !finite_pos(sys->De) && !(g.kind == IAT_GEN_SWEEP || g.kind == IAT_GEN_THERMAL))
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
    P.max_steps = sys->max_steps > 0 ? sys->max_steps : IAT_MAX_STEPS_LIMIT;
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
    P.id0_dev = batch->id0_dev;
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
    for (int k = 0; k < kMarks; ++k)
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
    if (hipEventSynchronize(ev_[kMarks - 1]) != hipSuccess)
        rc = set_error(IAT_EHIP, "timing: hipEventSynchronize failed");
    for (int k = 0; k + 1 < kMarks && rc == 0; ++k)
        if (hipEventElapsedTime(&out_[k], ev_[k], ev_[k + 1]) != hipSuccess)
            rc = set_error(IAT_EHIP, "timing: hipEventElapsedTime failed");
    return rc;
}
PhaseTimer::~PhaseTimer()
{
    if (!out_) return;
    for (int k = 0; k < kMarks; ++k)
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
    if (L.max_suspended < 0) return set_error(IAT_EINVAL, "launch.max_suspended must be >= 0");
    if (L.tail_budget < -1) return set_error(IAT_EINVAL, "launch.tail_budget must be >= -1");
    if (L.reserved != 0) return set_error(IAT_EINVAL, "launch.reserved must be 0");
    *out = L;
    return 0;
}

}  // namespace iat

extern "C" int iat_workspace_bytes(int which, const iat_system* sys, const iat_species* species, int n_species,
                                   const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                                   int reduce_kind, size_t* bytes, void* stream)
{
    using namespace iat;
    if (!bytes) return set_error(IAT_EINVAL, "bytes is NULL");
    switch (which) {
    case IAT_WS_INTEGRATE:
        return integrate_ws_bytes(sys, species, n_species, batch, launch, bytes);
    case IAT_WS_REDUCE: {
        const int rc = validate_common(sys, species, n_species, batch);
        return rc ? rc : reduce_ws_bytes(batch, reduce_kind, bytes);
    }
    case IAT_WS_ADJOINT:
        return iat_adjoint_workspace_bytes(sys, species, n_species, batch, obs, bytes, stream);
    default:
        return set_error(IAT_EINVAL, "unknown workspace kind %d", which);
    }
}
