// Ensemble reductions of a batch's outputs (iat_reduce).
//
// CELLS     : per sweep cell c (cell = id mod n_cells): count, complex count, sum dE, sum dE^2,
//             sum n_bounce.  Sums run in a fixed order (per-cell partials over fixed id slices,
//             then the partials in slice order), so results do not depend on scheduling.
// W0_HIST   : per species, 64 bins of log10(E/W0) over [-3, 3] (total, complex), W0 from Eq. (2)
//             with omega = (Omega/2) sqrt(a_x + q_x^2/2); and 256 bins of the heating
//             sign(dE) log10(1 + |dE|/(k_B 1 nK)).  Integer counts accumulate exactly.
//             W0_HIST_BOUND: the same with the second column counting trajectories that reached the
//             negative-energy bound state (Eq. (2) text) instead of the complex flag.
// BOXCOUNT  : box-counting dimensions of the complex-forming set of a GRID batch: for box sizes
//             s = 2^k, the number of boxes holding complex cells (occupied) and holding both kinds
//             (boundary); slopes of log N(s) against log(1/s) by least squares.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "iat_device.h"
#include "iat_host.h"

namespace iat {

constexpr int kSlices = 64;
constexpr double kNanoKelvin = 3.1668115634556e-15;   // k_B x 1 nK in hartree (CODATA 2018)

struct RedIn {
    const double* dE;
    const int32_t* nb;
    const uint32_t* status;
    int64_t n, id0;
    const int64_t* id0_dev;      // device offset added to id0, or NULL
    const double *t_first, *t_last;
};

// complex lifetimes (t_last - t_first bounce): 96 bins of log10(lifetime / 1 us) over [-2, 4]
constexpr int kLifeBins = 96, kLifeSlot = kLifeBins + 2;     // + censored count + spare
constexpr double kLifeLo = -2.0, kLifeHi = 4.0;
constexpr double kAuTimeMicro = 2.4188843265857e-11;           // atomic unit of time in microseconds

__host__ __device__ __forceinline__ int64_t cell_count(const iat_gen& g)
{
    const int64_t nE = g.n_E > 0 ? g.n_E : 1, nq = g.n_q > 0 ? g.n_q : 1, nD = g.n_De > 0 ? g.n_De : 1;
    return (int64_t)g.n_species * nE * nq * nD;
}

// thread (cell, slice): fixed-order sums over the ids of that cell within the slice
__global__ void k_reduce_cells(KParams P, RedIn R, double* part, int64_t ncell)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell * kSlices) return;
    const int64_t c = t / kSlices, j = t % kSlices;
    // local index i has global id id0 + i and cell (id0 + i) mod ncell
    const int64_t id0 = R.id0 + (R.id0_dev ? *R.id0_dev : 0);
    int64_t first = (c - id0 % ncell + ncell) % ncell;       // smallest local i of cell c
    const int64_t per = (R.n + kSlices - 1) / kSlices;
    const int64_t lo = j * per, hi = min(R.n, lo + per);
    int64_t i = first;
    if (i < lo) i += ((lo - i + ncell - 1) / ncell) * ncell;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (; i < hi; i += ncell) {
        const double e = R.dE[i];
        s0 += 1.0;
        s1 += (R.status[i] & IAT_ST_COMPLEX) ? 1.0 : 0.0;
        s2 += e;
        s3 += e * e;
        s4 += (double)R.nb[i];
    }
    double* o = part + (c * kSlices + j) * 5;
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
    o[3] = s3;
    o[4] = s4;
}

__global__ void k_reduce_cells_final(const double* part, int64_t ncell, double* out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int f = 0; f < 5; ++f) {
        double s = 0.0;
        for (int j = 0; j < kSlices; ++j) s += part[(c * kSlices + j) * 5 + f];
        out[c * 5 + f] += s;
    }
}

// Eq. (2): W0 = (8/(3 pi)) (m_a/(m_i + m_a))^(5/3) (m_i^2 omega^4 C4 / q_x^2)^(1/3),
// omega = (Omega/2) sqrt(a_x + q_x^2/2)  (a.u.)
__device__ __forceinline__ double w0_eq2(double m_a, double m_i, double C4, double Omega, double a_x, double q_x)
{
    const double om = 0.5 * Omega * sqrt(a_x + 0.5 * q_x * q_x);
    const double om2 = om * om;
    return (8.0 / (3.0 * 3.14159265358979323846)) * pow(m_a / (m_i + m_a), 5.0 / 3.0) *
           cbrt(m_i * m_i * om2 * om2 * C4 / (q_x * q_x));
}

__global__ void __launch_bounds__(256) k_reduce_hist(KParams P, RedIn R, double* out, int nsp, uint32_t cmask)
{
    __shared__ double hw[IAT_MAX_SPECIES * 64 * 2];
    __shared__ double hh[256];
    for (int t = threadIdx.x; t < nsp * 128; t += blockDim.x) hw[t] = 0.0;
    for (int t = threadIdx.x; t < 256; t += blockDim.x) hh[t] = 0.0;
    __syncthreads();
    const double X = log10(1.0 + 1.0e8);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R.n; i += (int64_t)gridDim.x * blockDim.x) {
        TrajParams tp;
        traj_params(P, i, tp);
        const double W0 = w0_eq2(species_mass(P, tp.sp), P.m_ion, species_C4(P, tp.sp), P.omega, P.a_x, tp.qx);
        double xb = (log10(tp.E / W0) + 3.0) / 6.0 * 64.0;
        int b = (int)floor(xb);
        b = b < 0 ? 0 : (b > 63 ? 63 : b);
        // species slot = position of tp.sp in the sweep's species list (or 0)
        int slot = 0;
#pragma unroll
        for (int s = 0; s < IAT_MAX_SPECIES; ++s)
            slot = (s < P.gen.n_species && P.gen.species[s] == tp.sp) ? s : slot;
        if (P.gen.kind != IAT_GEN_SWEEP && P.gen.kind != IAT_GEN_THERMAL) slot = 0;
        atomicAdd(&hw[(slot * 64 + b) * 2 + 0], 1.0);
        if (R.status[i] & cmask) atomicAdd(&hw[(slot * 64 + b) * 2 + 1], 1.0);
        const double e = R.dE[i];
        const double x = (e < 0.0 ? -1.0 : 1.0) * log10(1.0 + fabs(e) / kNanoKelvin);
        int hb = (int)floor((x + X) / (2.0 * X) * 256.0);
        hb = hb < 0 ? 0 : (hb > 255 ? 255 : hb);
        atomicAdd(&hh[hb], 1.0);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nsp * 128; t += blockDim.x)
        if (hw[t] != 0.0) atomicAdd(&out[t], hw[t]);
    for (int t = threadIdx.x; t < 256; t += blockDim.x)
        if (hh[t] != 0.0) atomicAdd(&out[nsp * 128 + t], hh[t]);
}

// Box counting on a side x side grid (side a power of two) as a pyramid of box flags: bit 0 = the box
// holds a complex-forming cell, bit 1 = all its cells are complex-forming.  Level 0 reads the status
// words; level k merges 2 x 2 boxes of level k-1.  Counts are reduced per wave before the atomic.
__device__ __forceinline__ void count_box(uint8_t f, unsigned long long* counts, int k, bool live)
{
    const bool occ = live && (f & 1), bnd = live && (f & 1) && !(f & 2);
    const unsigned long long mo = __ballot(occ), mb = __ballot(bnd);
    if ((threadIdx.x & 63) == 0) {
        if (mo) atomicAdd(&counts[2 * k + 0], (unsigned long long)__popcll(mo));
        if (mb) atomicAdd(&counts[2 * k + 1], (unsigned long long)__popcll(mb));
    }
}

__global__ void k_box_level0(const uint32_t* status, int64_t n, uint8_t* flags, unsigned long long* counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    uint8_t f = 0;
    if (live) {
        f = (status[i] & IAT_ST_COMPLEX) ? 3 : 0;
        flags[i] = f;
    }
    count_box(f, counts, 0, live);
}

__global__ void k_box_level(const uint8_t* prev, int side_prev, uint8_t* next, int k, unsigned long long* counts)
{
    const int side = side_prev >> 1;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = b < (int64_t)side * side;
    uint8_t f = 0;
    if (live) {
        const int r = (int)(b / side), c = (int)(b % side);
        const int64_t p0 = (int64_t)(2 * r) * side_prev + 2 * c, p1 = p0 + side_prev;
        const uint8_t a = prev[p0], bb = prev[p0 + 1], cc = prev[p1], d = prev[p1 + 1];
        f = (uint8_t)(((a | bb | cc | d) & 1) | (a & bb & cc & d & 2));
        next[b] = f;
    }
    count_box(f, counts, k, live);
}

// Lifetime histogram per species slot: exited complexes by log10 lifetime; complexes still bound at
// t_max or at the step cap go to the censored counter (their lifetime is only bounded below).
__global__ void __launch_bounds__(256) k_reduce_life(KParams P, RedIn R, double* out, int nsp)
{
    __shared__ double h[IAT_MAX_SPECIES * kLifeSlot];
    for (int t = threadIdx.x; t < nsp * kLifeSlot; t += blockDim.x) h[t] = 0.0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R.n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t st = R.status[i];
        if (!(st & IAT_ST_COMPLEX)) continue;
        int slot = 0;
        if (P.gen.kind == IAT_GEN_SWEEP || P.gen.kind == IAT_GEN_THERMAL) {
            TrajParams tp;
            traj_params(P, i, tp);
#pragma unroll
            for (int s = 0; s < IAT_MAX_SPECIES; ++s)
                slot = (s < P.gen.n_species && P.gen.species[s] == tp.sp) ? s : slot;
        }
        if ((st & IAT_ST_EXITED) && R.nb[i] >= 2) {
            const double x = log10((R.t_last[i] - R.t_first[i]) * kAuTimeMicro);
            int b = (int)floor((x - kLifeLo) / (kLifeHi - kLifeLo) * kLifeBins);
            b = b < 0 ? 0 : (b > kLifeBins - 1 ? kLifeBins - 1 : b);
            atomicAdd(&h[slot * kLifeSlot + b], 1.0);
        } else if (st & (IAT_ST_TMAX | IAT_ST_MAX_STEPS)) {
            atomicAdd(&h[slot * kLifeSlot + kLifeBins], 1.0);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nsp * kLifeSlot; t += blockDim.x)
        if (h[t] != 0.0) atomicAdd(&out[t], h[t]);
}

// Survival S(t) = fraction of complexes alive at the lower edge t of each bin (censored ones alive
// throughout); power-law exponent = -(LSQ slope of log S against log t) over edges t >= 20 us.
__global__ void k_life_fit(double* out, int nsp)
{
    const int slot = threadIdx.x;
    if (slot >= nsp) return;
    const double* h = out + slot * kLifeSlot;
    double total = h[kLifeBins];
    for (int b = 0; b < kLifeBins; ++b) total += h[b];
    double cum = h[kLifeBins], sx = 0, sy = 0, sxx = 0, sxy = 0;
    int m = 0;
    const double tmin = log10(20.0);
    for (int b = kLifeBins - 1; b >= 0; --b) {
        cum += h[b];
        const double lt = kLifeLo + b * (kLifeHi - kLifeLo) / kLifeBins;      // log10 of the lower edge
        if (lt < tmin || total <= 0.0 || cum <= 0.0) continue;
        const double x = lt * 2.30258509299404568402, y = log(cum / total);
        sx += x;
        sy += y;
        sxx += x * x;
        sxy += x * y;
        ++m;
    }
    out[nsp * kLifeSlot + slot] = m >= 2 ? -(m * sxy - sx * sy) / (m * sxx - sx * sx) : __builtin_nan("");
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0ull;
}

// least-squares slopes of log N(s) vs log(1/s) over s = 2^kmin .. 2^kmax
__global__ void k_boxcount_fit(const unsigned long long* counts, int levels, int kmin, int kmax, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int w = 0; w < 2; ++w) {
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        int m = 0;
        for (int k = kmin; k <= kmax && k < levels; ++k) {
            const double N = (double)counts[2 * k + w];
            if (N <= 0.0) continue;
            const double x = -k * 0.69314718055994530942, y = log(N);
            sx += x;
            sy += y;
            sxx += x * x;
            sxy += x * y;
            ++m;
        }
        // w = 0 counts occupied boxes (D_set, out[1]); w = 1 boundary boxes (D_boundary, out[0])
        out[1 - w] = m >= 2 ? (m * sxy - sx * sy) / (m * sxx - sx * sx) : __builtin_nan("");
    }
    for (int k = 0; k < levels; ++k) {
        out[2 + 2 * k] = (double)counts[2 * k];
        out[3 + 2 * k] = (double)counts[2 * k + 1];
    }
}

}  // namespace iat

namespace iat {

// Device bytes of the CELLS partial sums (per cell and slice: count, complexes and three sums).
static size_t cells_part_bytes(int64_t ncell) { return (size_t)ncell * kSlices * 5 * sizeof(double); }
// BOXCOUNT buffer: level counters, then one flag byte per cell of the current level and of the next.
static void box_layout(int64_t n, size_t& cbytes, size_t& fbytes, size_t& gbytes)
{
    cbytes = 256;
    fbytes = (size_t)n;
    gbytes = (size_t)n / 4 + 1;
}

// The batch conditions of the reductions that need them (EINVAL otherwise).
static int reduce_check(const iat_batch* batch, int kind)
{
    const iat_gen& g = batch->gen;
    if (kind == IAT_REDUCE_CELLS && g.kind != IAT_GEN_SWEEP && g.kind != IAT_GEN_THERMAL)
        return set_error(IAT_EINVAL, "reduce CELLS needs a SWEEP or THERMAL batch");
    if (kind == IAT_REDUCE_BOXCOUNT) {
        if (g.kind != IAT_GEN_GRID || g.id0 != 0 || batch->id0_dev || batch->n != (int64_t)g.n_theta * g.n_phi)
            return set_error(IAT_EINVAL, "reduce BOXCOUNT needs a whole GRID batch");
        const int nt = g.n_theta;
        if (nt != g.n_phi || nt < 2 || (nt & (nt - 1)) != 0 || nt > 32768)
            return set_error(IAT_EINVAL, "reduce BOXCOUNT needs a square power-of-two grid, side 2..32768");
    }
    return 0;
}

int reduce_ws_bytes(const iat_batch* batch, int kind, size_t* bytes)
{
    size_t c = 0, f = 0, g = 0;
    if (batch->n > 0) {
        const int rc = reduce_check(batch, kind);
        if (rc) return rc;
    }
    switch (kind) {
    case IAT_REDUCE_CELLS:
        *bytes = batch->n == 0 ? 0 : cells_part_bytes(cell_count(batch->gen));
        return 0;
    case IAT_REDUCE_BOXCOUNT:
        box_layout(batch->n, c, f, g);
        *bytes = batch->n == 0 ? 0 : c + f + g;
        return 0;
    case IAT_REDUCE_W0_HIST:
    case IAT_REDUCE_W0_HIST_BOUND:
    case IAT_REDUCE_LIFETIME:
        *bytes = 0;          // these accumulate straight into `out`
        return 0;
    default:
        return set_error(IAT_EINVAL, "unknown reduce kind %d", kind);
    }
}

}  // namespace iat

using namespace iat;

extern "C" int iat_reduce(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch,
                          const iat_obs* obs, int kind, double* out, void* stream)
{
    int rc = validate_common(sys, species, n_species, batch);
    if (rc) return rc;
    if (!obs || !out) return set_error(IAT_EINVAL, "reduce: obs and out are required");
    if (batch->n > 0 && (!obs->dE_ion || !obs->status || !obs->n_bounce))
        return set_error(IAT_EINVAL, "reduce: obs.dE_ion, obs.n_bounce and obs.status are required");
    KParams P;
    fill_params(P, sys, species, n_species, batch);
    RedIn R{obs->dE_ion, obs->n_bounce, obs->status, batch->n, batch->gen.id0, batch->id0_dev,
            obs->t_bounce_first, obs->t_bounce_last};
    hipStream_t st = (hipStream_t)stream;
    if (batch->n == 0) return 0;
    rc = reduce_check(batch, kind);
    if (rc) return rc;
    if (kind == IAT_REDUCE_CELLS) {
        const int64_t ncell = cell_count(batch->gen);
        void* part = nullptr;
        const size_t bytes = cells_part_bytes(ncell);
        if (hipMallocAsync(&part, bytes, st) != hipSuccess) return set_error(IAT_EHIP, "hipMallocAsync failed");
        const int64_t threads = ncell * kSlices;
        hipLaunchKernelGGL(k_reduce_cells, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, P, R,
                           (double*)part, ncell);
        hipLaunchKernelGGL(k_reduce_cells_final, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, st,
                           (const double*)part, ncell, out);
        if (hipFreeAsync(part, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    } else if (kind == IAT_REDUCE_W0_HIST || kind == IAT_REDUCE_W0_HIST_BOUND) {
        const int nsp = (batch->gen.kind == IAT_GEN_SWEEP || batch->gen.kind == IAT_GEN_THERMAL) ? batch->gen.n_species : 1;
        const int64_t blocks = std::min<int64_t>((batch->n + 255) / 256, 4096);
        const uint32_t cmask = kind == IAT_REDUCE_W0_HIST ? IAT_ST_COMPLEX : IAT_ST_BOUND_SEEN;
        hipLaunchKernelGGL(k_reduce_hist, dim3((unsigned)blocks), dim3(256), 0, st, P, R, out, nsp, cmask);
    } else if (kind == IAT_REDUCE_LIFETIME) {
        if (!obs->t_bounce_first || !obs->t_bounce_last)
            return set_error(IAT_EINVAL, "reduce LIFETIME needs obs.t_bounce_first and obs.t_bounce_last");
        const int nsp = (batch->gen.kind == IAT_GEN_SWEEP || batch->gen.kind == IAT_GEN_THERMAL) ? batch->gen.n_species : 1;
        const int64_t blocks = std::min<int64_t>((batch->n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_reduce_life, dim3((unsigned)blocks), dim3(256), 0, st, P, R, out, nsp);
        hipLaunchKernelGGL(k_life_fit, dim3(1), dim3(64), 0, st, out, nsp);
    } else if (kind == IAT_REDUCE_BOXCOUNT) {
        const iat_gen& g = batch->gen;
        const int nt = g.n_theta;
        int levels = 0;
        while ((1 << levels) <= nt) ++levels;
        size_t cbytes, fbytes, gbytes;
        box_layout(batch->n, cbytes, fbytes, gbytes);
        void* buf = nullptr;
        if (hipMallocAsync(&buf, cbytes + fbytes + gbytes, st) != hipSuccess)
            return set_error(IAT_EHIP, "hipMallocAsync failed");
        unsigned long long* cnt = (unsigned long long*)buf;
        uint8_t* fa = (uint8_t*)buf + cbytes;
        uint8_t* fb = fa + fbytes;
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, cnt, 2 * levels);
        hipLaunchKernelGGL(k_box_level0, dim3((unsigned)((batch->n + 255) / 256)), dim3(256), 0, st,
                           (const uint32_t*)obs->status, batch->n, fa, cnt);
        for (int k = 1; k < levels; ++k) {
            const int side_prev = nt >> (k - 1);
            const int64_t boxes = (int64_t)(side_prev / 2) * (side_prev / 2);
            hipLaunchKernelGGL(k_box_level, dim3((unsigned)((boxes + 255) / 256)), dim3(256), 0, st,
                               (const uint8_t*)fa, side_prev, fb, k, cnt);
            std::swap(fa, fb);
        }
        const int kmin = 1, kmax = std::min(6, levels - 1);
        hipLaunchKernelGGL(k_boxcount_fit, dim3(1), dim3(1), 0, st, (const unsigned long long*)cnt, levels, kmin, kmax,
                           out);
        if (hipFreeAsync(buf, st) != hipSuccess) return set_error(IAT_EHIP, "hipFreeAsync failed");
    } else {
        return set_error(IAT_EINVAL, "unknown reduce kind %d", kind);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(IAT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return 0;
}
