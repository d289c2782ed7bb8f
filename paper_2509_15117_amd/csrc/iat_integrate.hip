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
constexpr int64_t kMaxSolo = 1 << 16;            // records of the solo level per call
constexpr int kTailSteps = 4;                    // steps per turn of the four-lane tail kernel's loop (a power of 2)

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
    uint64_t longest = 0;     // (attempted steps << 34) | global id of the longest trajectory finished
};

// The longest trajectory of a call, packed so that one atomic max keeps it: attempted steps (clamped
// to 30 bits) above the trajectory's global id (34 bits; generated batches number from gen.id0).
__device__ __forceinline__ uint64_t longest_key(const KParams& P, int64_t i, int32_t nacc, int32_t nrej)
{
    int64_t steps = (int64_t)nacc + (int64_t)nrej;
    steps = steps < 0 ? 0 : (steps > 0x3fffffff ? 0x3fffffff : steps);
    const int64_t gid = (P.gen.kind == IAT_GEN_ARRAYS ? 0 : batch_id0(P)) + i;
    return ((uint64_t)steps << 34) | ((uint64_t)gid & 0x3ffffffffull);
}

__device__ __forceinline__ void flush_stats(uint64_t* stats, const LaneStats& s, uint64_t issued)
{
    if (!stats) return;
    const uint64_t r = wave_sum(s.rhs), a = wave_sum(s.acc), j = wave_sum(s.rej), d = wave_sum(s.done),
                   u = wave_sum(s.useful), lg = wave_max(s.longest);
    if (__lane_id() == 0) {
        atomicAdd((unsigned long long*)&stats[0], (unsigned long long)r);
        atomicAdd((unsigned long long*)&stats[1], (unsigned long long)a);
        atomicAdd((unsigned long long*)&stats[2], (unsigned long long)j);
        atomicAdd((unsigned long long*)&stats[3], (unsigned long long)d);
        atomicAdd((unsigned long long*)&stats[4], (unsigned long long)issued);
        atomicAdd((unsigned long long*)&stats[5], (unsigned long long)u);
        if (lg) atomicMax((unsigned long long*)&stats[10], (unsigned long long)lg);
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

template <bool CE>
__global__ void __launch_bounds__(256) k_integrate_plain(KParams P, Work W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    LaneStats st;
    uint64_t iters = 0;
    if (i < P.n) {
        Traj1 T;
        traj1_start(P, W, i, T);
        while (!T.S.done) {
            traj1_advance<CE>(P, T);
            ++iters;
        }
        traj1_store(W, i, T);
        st.rhs = T.S.nrhs;
        st.acc = T.S.nacc;
        st.rej = T.S.nrej;
        st.done = 1;
        st.useful = T.S.nacc + T.S.nrej;
        if (P.stats) st.longest = longest_key(P, i, T.S.nacc, T.S.nrej);
    }
    // every lane of the wave is issued for as many steps as its slowest lane needed
    flush_stats(P.stats, st, 64ull * wave_max(iters));
}

// Persistent refill kernel.  A trajectory that has used `budget` attempted steps without
// finishing is suspended into the continuation records (while slots last) and its lane takes
// new work; k_integrate_tail finishes the suspended ones four lanes per trajectory.
template <bool CE>
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
            if (active && !T.S.done) traj1_advance<CE>(P, T);
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
                if (P.stats) {
                    const uint64_t key = longest_key(P, i, T.S.nacc, T.S.nrej);
                    st.longest = key > st.longest ? key : st.longest;
                }
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
// a long-lived complex is what bounds a batch's wall time.  QUADS trajectories share a wave.
// Trajectories move on to k_integrate_solo, which finishes them one per wave so that the longest
// complexes run without wave or SIMD neighbours, by one of two rules: with budget2 > 0, after
// budget2 more attempted steps here; with pop_limit > 0, once at most pop_limit of the records this
// kernel resumes are still running or waiting (`gone` counts the finished and moved ones), i.e. once
// the solo level's waves can hold them all.  A trajectory is moved (suspended again into C2, while
// its slots last) after the step it is on, and its quad takes new work.  Counters: stats[si] RHS
// evaluations and stats[si + 1] trajectories finished in this kernel.
template <bool CE, int QUADS>
__device__ __forceinline__ void tail_run(const KParams& P, const Work& W, const Cont& C, const Cont& C2,
                                         int budget2, int64_t pop_limit, unsigned long long* gone, int si)
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
    bool active = false, need = (lane >> 2) < QUADS, may_suspend = (budget2 > 0 || pop_limit > 0) && C2.cap > 0;
    bool few_left = false;       // pop_limit rule: the remaining population fits the solo level
    const Tab B = tab_in_registers();
    const StepK K = step_k_in_registers(P);
    const Quad4 Q = quad_consts<true>(P, B);
    // The hand-out, population and suspension checks run once per turn of kTailSteps steps (a quad whose
    // trajectory ends early in a turn idles for the rest of it), in one loop: as a loop nested in the
    // step loop they cost the kernel registers.
    for (;;) {
        if ((iters & (kTailSteps - 1)) == 0) {
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
            // every lane reads the counter in the same load, so the flag is wave-uniform
            if (pop_limit > 0 && may_suspend && !few_left && (iters & 63) == 0)
                few_left =
                    total - (int64_t)__hip_atomic_load(gone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= pop_limit;
        }
        if (active && !T.S.done) traj4_step_fast<CE>(P, K, T, B, Q);
        ++iters;
        if ((iters & (kTailSteps - 1)) != 0) continue;
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
                if (pop_limit > 0) atomicAdd(gone, 1ull);
                if (P.stats) {
                    const uint64_t key = longest_key(P, i, T.S.nacc, T.S.nrej);
                    st.longest = key > st.longest ? key : st.longest;
                }
            }
            active = false;
            need = (lane >> 2) < QUADS;
        } else if (active && may_suspend &&
                   (budget2 > 0 ? T.S.nacc + T.S.nrej - resumed_at >= budget2 : few_left)) {
            // quad-uniform: the whole quad holds the same scalar state
            unsigned long long s2 = 0;
            if (leader) s2 = atomicAdd(C2.count, 1ull);
            s2 = __shfl(s2, qlead, 64);
            if ((int64_t)s2 < C2.cap) {
                cont_save4(C2, (int64_t)s2, i, T, lane & 3);
                if (leader) {
                    st.useful += T.S.nacc + T.S.nrej - resumed_at;
                    tail_rhs += (uint64_t)(T.S.nrhs - resumed_rhs);
                    if (pop_limit > 0) atomicAdd(gone, 1ull);
                }
                active = false;
                need = true;   // a quad that suspends is one of the wave's QUADS quads
            } else {
                may_suspend = false;
            }
        }
    }
    flush_stats(P.stats, st, 0ull);
    if (P.stats) {
        const uint64_t tr = wave_sum(tail_rhs), td = wave_sum(tail_done);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&P.stats[4], (unsigned long long)QUADS * iters);
            atomicAdd((unsigned long long*)&P.stats[si], (unsigned long long)tr);
            atomicAdd((unsigned long long*)&P.stats[si + 1], (unsigned long long)td);
        }
    }
}

template <bool CE>
__global__ void __launch_bounds__(256) k_integrate_tail(KParams P, Work W, Cont C, Cont C2, int budget2,
                                                        int64_t pop_limit, unsigned long long* gone)
{
    tail_run<CE, 16>(P, W, C, C2, budget2, pop_limit, gone, 6);
}

// 64-bit value of the wave's first active lane, as a wave-uniform (scalar) value
__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The solo level: one trajectory per wave, eight lanes per trajectory (every octet of the wave runs a
// copy of it, so the whole wave follows one control path and its branches are uniform), launched in
// blocks of four waves, one block per compute unit, so that the dispatcher puts one wave on each SIMD.
// Each wave takes records from C one at a time.  Counters: stats[8] RHS evaluations and stats[9]
// trajectories finished here.
template <bool CE>
__global__ void __launch_bounds__(256) k_integrate_solo(KParams P, Work W, Cont C)
{
    const int lane = __lane_id();
    const int l = lane & 7;
    const bool atom = l < 4;
    const int ax = atom ? min(l, 2) : min(7 - l, 2);
    const unsigned long long cnt = *C.count;
    const int64_t total = (int64_t)(cnt < (unsigned long long)C.cap ? cnt : (unsigned long long)C.cap);
    const Tab B = tab_in_registers();
    const StepK K = step_k_in_registers(P);
    const Oct O = oct_consts(P, B);
    LaneStats st;
    uint64_t iters = 0, solo_rhs = 0, solo_done = 0;
    for (;;) {
        unsigned long long slot = 0;
        if (lane == 0) slot = atomicAdd(C.head, 1ull);
        slot = first_lane_u64(slot);
        if ((int64_t)slot >= total) break;
        Traj8 T;
        int64_t i;
        cont_load8(W, C, (int64_t)slot, atom, ax, T, i);
        T.m = atom ? T.L.inv_ma : P.inv_mi;
        const int32_t resumed_at = T.S.nacc + T.S.nrej, resumed_rhs = T.S.nrhs;
        while (!__builtin_amdgcn_readfirstlane(T.S.done)) traj8_run<CE>(P, K, T, B, O, iters);
        if (lane < 8) traj8_store(W, i, T, l);
        if (lane == 0) {
            st.rhs += T.S.nrhs;
            st.acc += T.S.nacc;
            st.rej += T.S.nrej;
            st.done += 1;
            st.useful += T.S.nacc + T.S.nrej - resumed_at;
            solo_rhs += (uint64_t)(T.S.nrhs - resumed_rhs);
            solo_done += 1;
            if (P.stats) {
                const uint64_t key = longest_key(P, i, T.S.nacc, T.S.nrej);
                st.longest = key > st.longest ? key : st.longest;
            }
        }
    }
    flush_stats(P.stats, st, 0ull);
    if (P.stats && lane == 0) {
        atomicAdd((unsigned long long*)&P.stats[4], (unsigned long long)iters);
        atomicAdd((unsigned long long*)&P.stats[8], (unsigned long long)solo_rhs);
        atomicAdd((unsigned long long*)&P.stats[9], (unsigned long long)solo_done);
    }
}

__global__ void k_reset_counters(unsigned long long* q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
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

namespace iat {

// One call's device workspace: queue counters | work buffer (n trajectories) | continuation records
// of the four-lane tail (cap) | continuation records of the solo level (cap2).
constexpr size_t kRecBytes = 26 * sizeof(double) + 8 * sizeof(int32_t) + sizeof(int64_t);
constexpr size_t kWorkBytesPerTraj = kWorkDoubles * sizeof(double) + kWorkInts * sizeof(int32_t);
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t workspace_bytes(int64_t n, int64_t cap, int64_t cap2)
{
    return 256 + round256((size_t)n * kWorkBytesPerTraj) + (size_t)(cap + cap2) * kRecBytes;
}

// Largest batch of the allocation-free entry point, and its continuation-record limits (a trajectory
// that finds no free record keeps running where it is, with the same bits).
constexpr int64_t kNoAllocMaxN = 1 << 16;
constexpr int64_t kNoAllocMaxSuspended = 1 << 15;
constexpr int64_t kNoAllocMaxSolo = 1 << 12;
constexpr size_t kScratchBytes = workspace_bytes(kNoAllocMaxN, kNoAllocMaxSuspended, kNoAllocMaxSolo);

// Validated arguments of an integration call and the launch shape they resolve to.
struct IntegrateCall {
    KParams P;
    iat_launch L;
    int64_t n = 0, cap = 0, cap2 = 0;
    int budget2 = 0;
    bool pop_rule = false;       // move to the solo level once the tail's population fits it
    bool ce = false;
};

// sizing: only the workspace is wanted (obs may be NULL, nothing is launched)
static int integrate_prepare(const iat_system* sys, const iat_species* species, int n_species,
                             const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                             int64_t suspended_limit, int64_t solo_limit, IntegrateCall& c, bool sizing = false)
{
    int rc = validate_common(sys, species, n_species, batch);
    if (rc) return rc;
    if (!obs && !sizing) return set_error(IAT_EINVAL, "obs is NULL");
    if (obs && batch->n > 0 &&
        (!obs->angle || !obs->q_transfer || !obs->dE_ion || !obs->t_dwell || !obs->n_bounce || !obs->status))
        return set_error(IAT_EINVAL, "obs: angle, q_transfer, dE_ion, t_dwell, n_bounce and status are required");
    rc = resolve_launch(launch, &c.L);
    if (rc) return rc;
    c.n = batch->n;
    if (c.n > (int64_t)0x7fffffff * 256) return set_error(IAT_EINVAL, "batch too large for one launch");
    fill_params(c.P, sys, species, n_species, batch);
    if (obs) fill_outputs(c.P, obs);
    c.P.stats = c.L.stats;
    c.P.refill_every = c.L.refill_every;
    c.P.budget = 0;
    c.cap = 0;
    if (c.L.kernel == IAT_KERNEL_PERSISTENT) {
        c.P.budget = c.L.step_budget > 0 ? c.L.step_budget : (c.L.step_budget == 0 ? kDefaultBudget : 0);
        const int64_t lim = c.L.max_suspended > 0 ? std::min<int64_t>(c.L.max_suspended, suspended_limit)
                                                  : suspended_limit;
        c.cap = c.P.budget > 0 ? std::min<int64_t>(c.n, lim) : 0;
    }
    // second level: trajectories still running in the four-lane tail finish one per wave in
    // k_integrate_solo, moved there after tail_budget steps, or (default) once the tail's
    // remaining population fits the solo level's waves
    c.budget2 = c.L.tail_budget > 0 ? c.L.tail_budget : 0;
    c.pop_rule = c.L.tail_budget == 0;
    c.cap2 = (c.cap > 0 && (c.budget2 > 0 || c.pop_rule)) ? std::min<int64_t>(c.cap, solo_limit) : 0;
    if (c.cap2 == 0) {
        c.budget2 = 0;
        c.pop_rule = false;
    }
    // thermal runs leave through the start sphere about the trap centre (CE kernels)
    c.ce = batch->gen.kind == IAT_GEN_THERMAL;
    return 0;
}

// Enqueues the whole call on `st` over the workspace `ws` of workspace_bytes(n, cap, cap2) bytes.
// Returns the first launch error (0 if none); the caller reports it.
static hipError_t integrate_enqueue(IntegrateCall& c, void* ws, int n_cu, hipStream_t st, PhaseTimer& timer)
{
    KParams& P = c.P;
    const iat_launch& L = c.L;
    const int64_t n = c.n, cap = c.cap, cap2 = c.cap2;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    unsigned long long* q = (unsigned long long*)ws;
    const size_t work_bytes = (size_t)n * kWorkBytesPerTraj;
    Work W;
    W.n = n;
    W.D = (double*)((char*)ws + 256);
    W.I = (int32_t*)(W.D + (size_t)kWorkDoubles * n);
    Cont C;
    C.count = q + 1;
    C.head = q + 2;
    C.cap = cap;
    C.d = (double*)((char*)ws + 256 + round256(work_bytes));
    C.n = (int32_t*)(C.d + 26 * cap);
    C.id = (int64_t*)(C.n + 8 * cap);
    Cont C2;
    C2.count = q + 3;
    C2.head = q + 4;
    C2.cap = cap2;
    C2.d = (double*)(C.id + cap);
    C2.n = (int32_t*)(C2.d + 26 * cap2);
    C2.id = (int64_t*)(C2.n + 8 * cap2);
    // the counters start at zero (a fill kernel, not a memset node, so that the call can be captured)
    unsigned long long* gone = q + 5;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, q, 6);
    timer.mark(0);
    hipLaunchKernelGGL(k_setup, dim3(nblk), dim3(256), 0, st, P, W);
    timer.mark(1);
    hipError_t launch_err = hipSuccess;
    const bool ce = c.ce;
    const void* k_plain = ce ? (const void*)k_integrate_plain<true> : (const void*)k_integrate_plain<false>;
    const void* k_pers = ce ? (const void*)k_integrate_persistent<true> : (const void*)k_integrate_persistent<false>;
    const void* k_tail = ce ? (const void*)k_integrate_tail<true> : (const void*)k_integrate_tail<false>;
    const void* k_solo = ce ? (const void*)k_integrate_solo<true> : (const void*)k_integrate_solo<false>;
    if (L.kernel == IAT_KERNEL_PLAIN) {
        void* args[] = {&P, &W};
        launch_err = hipLaunchKernel(k_plain, dim3((unsigned)((n + L.block - 1) / L.block)), dim3(L.block), args, 0, st);
        timer.mark(2);
        timer.mark(3);
    } else {
        int per_cu = L.blocks_per_cu;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pers, L.block, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
        }
        int64_t blocks = (int64_t)n_cu * per_cu;
        const int64_t need = (n + L.block - 1) / L.block;
        if (blocks > need) blocks = need;
        void* args[] = {&P, &W, &q, &C};
        launch_err = hipLaunchKernel(k_pers, dim3((unsigned)blocks), dim3(L.block), args, 0, st);
        timer.mark(2);
        if (cap > 0) {
            int per_cu4 = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu4, k_tail, 256, 0) != hipSuccess || per_cu4 < 1)
                per_cu4 = 1;
            int64_t blocks4 = (int64_t)n_cu * per_cu4;
            const int64_t need4 = (4 * cap + 255) / 256;
            if (blocks4 > need4) blocks4 = need4;
            // the solo level's waves: one per SIMD (k_integrate_solo's launch below)
            int64_t pop_limit = c.pop_rule ? std::min<int64_t>((int64_t)n_cu * 4, cap2) : 0;
            void* args4[] = {&P, &W, &C, &C2, &c.budget2, &pop_limit, &gone};
            const hipError_t e4 = hipLaunchKernel(k_tail, dim3((unsigned)blocks4), dim3(256), args4, 0, st);
            if (launch_err == hipSuccess) launch_err = e4;
        }
        timer.mark(3);
        if (cap2 > 0) {
            // one wave per SIMD: blocks of four waves, at most one block per compute unit, so that the
            // survivors run without wave or SIMD neighbours
            const int64_t waves1 = std::min<int64_t>((int64_t)n_cu * 4, cap2);
            const int64_t blocks1 = (waves1 + 3) / 4;
            void* args1[] = {&P, &W, &C2};
            const hipError_t e1 = hipLaunchKernel(k_solo, dim3((unsigned)blocks1), dim3(256), args1, 0, st);
            if (launch_err == hipSuccess) launch_err = e1;
        }
    }
    timer.mark(4);
    hipLaunchKernelGGL(k_observe, dim3(nblk), dim3(256), 0, st, P, W);
    timer.mark(5);
    return launch_err;
}

// The allocation-free entry point's workspace: one array per device, resolved to a device address
// once per device with hipGetSymbolAddress (the array's name is not a device address in host code).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

static int scratch_address(void** out)
{
    constexpr int kMaxDev = 64;
    static void* addr[kMaxDev] = {};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
        return set_error(IAT_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(IAT_EHIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return 0;
}

int integrate_ws_bytes(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch,
                       const iat_launch* launch, size_t* bytes)
{
    IntegrateCall c;
    const int rc = integrate_prepare(sys, species, n_species, batch, nullptr, launch, kMaxSuspended, kMaxSolo, c, true);
    if (rc) return rc;
    *bytes = c.n == 0 ? 0 : workspace_bytes(c.n, c.cap, c.cap2);
    return 0;
}

}  // namespace iat

extern "C" int iat_integrate(const iat_system* sys, const iat_species* species, int n_species,
                             const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                             void* ckpt_ws, size_t ckpt_bytes, void* stream)
{
    if (ckpt_ws || ckpt_bytes)
        return set_error(IAT_ENOTSUP, "checkpointing is done by iat_adjoint itself; pass NULL/0");
    IntegrateCall c;
    int rc = integrate_prepare(sys, species, n_species, batch, obs, launch, kMaxSuspended, kMaxSolo, c);
    if (rc) return rc;
    if (c.n == 0) return 0;
    int n_cu = 0;
    rc = device_state(&n_cu);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = workspace_bytes(c.n, c.cap, c.cap2);
    void* ws = nullptr;
    if (hipMallocAsync(&ws, bytes, st) != hipSuccess) return set_error(IAT_EHIP, "hipMallocAsync of %zu bytes failed", bytes);
    PhaseTimer timer(c.L.kernel_ms, st);
    const hipError_t launch_err = integrate_enqueue(c, ws, n_cu, st, timer);
    if (hipFreeAsync(ws, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_err;
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return timer.finish();
}

extern "C" int iat_integrate_noalloc(const iat_system* sys, const iat_species* species, int n_species,
                                     const iat_batch* batch, const iat_obs* obs, const iat_launch* launch,
                                     void* stream)
{
    IntegrateCall c;
    int rc = integrate_prepare(sys, species, n_species, batch, obs, launch, kNoAllocMaxSuspended, kNoAllocMaxSolo, c);
    if (rc) return rc;
    if (c.n > kNoAllocMaxN)
        return set_error(IAT_EINVAL, "iat_integrate_noalloc: n = %lld is above its limit of %lld trajectories",
                         (long long)c.n, (long long)kNoAllocMaxN);
    if (c.L.kernel_ms)
        return set_error(IAT_EINVAL, "iat_integrate_noalloc: phase timing (launch.kernel_ms) is not available");
    if (c.n == 0) return 0;
    int n_cu = 0;
    rc = device_state(&n_cu);
    if (rc) return rc;
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    PhaseTimer timer(nullptr, st);
    const hipError_t launch_err = integrate_enqueue(c, ws, n_cu, st, timer);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_err;
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return 0;
}

extern "C" const char* iat_last_error(void) { return iat::last_error(); }
extern "C" const char* iat_version(void) { return "libiat 0.1 (gfx950)"; }
extern "C" void iat_release(void) { iat::release_devices(); }
