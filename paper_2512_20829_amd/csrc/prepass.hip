// Per-trajectory prepass, bucket bounds, record permutation and the
// per-trajectory normaliser of the conservative deposition mode.
#include "internal.hpp"
#include "kernels.hpp"
#include "prepass.hpp"

namespace flp {

// Per-trajectory prepass of trajectory i of one snapshot on a Cartesian
// mesh, written at global index gi (prepass_traj with the mesh's keyer).
template <typename R, int D>
__device__ inline void prepass_one(const TrajDev& t, const MeshDev& m, const PhysDev& ph, const float* hfac,
                                   int deposit, int64_t i, int64_t gi, uint32_t key_base, uint32_t sentinel,
                                   uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, double* qd,
                                   unsigned long long& skipped, unsigned long long& nosup)
{
    prepass_traj<R, D>(t, LatticeKey<D>{m}, ph, hfac, deposit, i, gi, key_base, sentinel, keys, vals, rpos, rw, qd,
                       skipped, nosup);
}

// Trajectories per thread of the prepass kernels: each trajectory is one
// long dependent binary64 chain, and several per thread give the scheduler
// independent chains to interleave (0.317 -> 0.150 ms for 2M trajectories
// from one to four).
constexpr int kPrepassPerThread = 4;
static_assert(kPrepassPerThread < 8, "wave_count_sum takes per-lane counts below 8");

// kPrepassPerThread trajectories of one snapshot per thread, blockDim apart.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_prepass(TrajDev t, MeshDev m, PhysDev ph, const float* hfac,
                                                 int deposit, uint32_t* keys, uint32_t* vals,
                                                 double4* rpos, R* rw, double* qd,
                                                 unsigned long long* stats)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kPrepassPerThread + threadIdx.x;
    const uint32_t sentinel = (uint32_t)kClasses * (uint32_t)m.ntiles;
    unsigned long long skipped = 0, nosup = 0;   // counts over the thread's trajectories
#pragma unroll
    for (int u = 0; u < kPrepassPerThread; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        if (i < t.count)
            prepass_one<R, D>(t, m, ph, hfac, deposit, i, i, 0u, sentinel, keys, vals, rpos, rw, qd, skipped, nosup);
    }
    wave_count_sum(stats, ST_SKIPPED, (unsigned)skipped);
    wave_count_sum(stats, ST_NOSUPPORT, (unsigned)nosup);
}

// kPrepassPerThread trajectories of a batch of snapshots per thread,
// blockDim apart: trajectories of snapshot s occupy global indices
// [item.base, item.base + count) and their keys the bucket range
// [item.key_base, item.key_base + kClasses * ntiles).
template <typename R, int D>
__global__ __launch_bounds__(256) void k_prepass_batch(const BatchItem* items, int nsnap, int64_t total,
                                                       uint32_t sentinel, uint32_t* keys, uint32_t* vals,
                                                       double4* rpos, R* rw, unsigned long long* stats)
{
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x * kPrepassPerThread + threadIdx.x;
    unsigned long long skipped = 0, nosup = 0;   // counts over the thread's trajectories
#pragma unroll
    for (int u = 0; u < kPrepassPerThread; ++u) {
        const int64_t gi = g0 + (int64_t)u * blockDim.x;
        if (gi < total) {
            int lo = 0, hi = nsnap - 1;      // last item with base <= gi
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (items[mid].base <= gi)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const BatchItem& it = items[lo];
            prepass_one<R, D>(it.t, it.g.m, it.ph, it.hfac, 0, gi - it.base, gi, it.key_base, sentinel, keys, vals,
                              rpos, rw, nullptr, skipped, nosup);
        }
    }
    wave_count_sum(stats, ST_SKIPPED, (unsigned)skipped);
    wave_count_sum(stats, ST_NOSUPPORT, (unsigned)nosup);
}

// Largest non-empty neighbourhood class, read off the bucket bounds.
__global__ void k_max_class(const uint32_t* bstart, int ntiles, unsigned long long* stats)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long mc = 0;
    for (int k = 0; k < kClasses; ++k)
        if (bstart[(int64_t)k * ntiles] != bstart[(int64_t)(k + 1) * ntiles]) mc = (unsigned long long)k;
    stats[ST_MAXCLASS] = mc;
}

// Largest non-empty class over the snapshots of a batch (one wave).
__global__ void k_max_class_batch(const BatchItem* items, int nsnap, const uint32_t* bstart,
                                  unsigned long long* stats)
{
    unsigned long long mc = 0;
    for (int s = threadIdx.x; s < nsnap; s += kWave) {
        const uint32_t* b = bstart + items[s].key_base;
        const int64_t nt = items[s].g.m.ntiles;
        for (int k = 0; k < kClasses; ++k)
            if (b[k * nt] != b[(k + 1) * nt] && (unsigned long long)k > mc) mc = (unsigned long long)k;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(mc, o, kWave);
        mc = t > mc ? t : mc;
    }
    if (threadIdx.x == 0) stats[ST_MAXCLASS] = mc;
}

// Bucket starts from sorted keys: bstart[b] = first position with key >= b
// (binary search), one thread per bucket b in [0, nb].
__global__ void k_bucket_bounds(const uint32_t* keys, int64_t n, uint32_t nb, uint32_t* bstart)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > (int64_t)nb) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    bstart[b] = (uint32_t)lo;
}

template <typename R>
__global__ void k_permute(const uint32_t* order, int64_t n, const double4* rpos_u, const R* rw_u,
                          double4* rpos, R* rw, int copy_w)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = order[p];
    rpos[p] = rpos_u[i];
    if (copy_w) {
        // whole records in 16-byte words
        constexpr int NQ = (int)(kRecW * sizeof(R) / sizeof(uint4));
        const uint4* src = reinterpret_cast<const uint4*>(rw_u + (int64_t)i * kRecW);
        uint4* dst = reinterpret_cast<uint4*>(rw + p * kRecW);
#pragma unroll
        for (int k = 0; k < NQ; ++k) dst[k] = src[k];
    }
}

constexpr int kZTab = 64;

// Deposition normaliser Z_i = sum over the cells in reach of the kernel
// factors, one half wave per valid trajectory (sorted order; the half waves
// of a workgroup take trajectories in turn), written into its weight record as
// {1/h, Q/(h Z)} (the 1/h factors cancel); with Z = 0 the record becomes a
// delta record {0, Q} flagged by 1/h < 0.  Per-axis factors of the cells in
// the trajectory's support box go to LDS (same binary64 offsets and the same
// inclusion test as the gather), lanes sweep the rows, and a fixed butterfly
// reduces the half wave.  The support box is swept in blocks of
// at most kZTab cells per axis.  Within a block, a cell (jx, jy, jz) is
// included iff (S0[jx] + S1[jy]) + S2[jz] <= c^2, evaluated in the working
// precision exactly as the gather does.  Floating-point addition is monotone,
// so on every row (jy, jz) the included cells are those whose S0 does not
// exceed a threshold: a prefix of the block's S0 values in ascending order.
// The block's S0 values are therefore ranked once, their factors E0 summed
// in binary64 in that order, and each row costs one binary search instead of
// one test per cell.  This holds for any shape of S0 (also across the
// periodic wrap of a support that spans a whole axis).
template <typename R>
struct NormLds {
    R S[3][kZTab];
    R E[3][kZTab];
    R Ss[kZTab];               // S0 of the block in ascending order
    double Pf[kZTab + 1];      // Pf[k] = sum of E0 over the k smallest S0
    R Es[kZTab];
};
// Waves per workgroup of the normaliser; each half wave (kNormLanes lanes)
// takes trajectories p = 2 (wave id) + half, + all half waves, ... with its
// own LDS tables, so the workgroups are few and long-lived rather than one
// short one per trajectory.  A support box spans about 2 c h |det J| / w
// cells per axis (tens), so half a wave covers an axis table in one pass
// and the two halves of a wave work on two trajectories at once.
constexpr int kNormWaves = 4;
constexpr int kNormLanes = 32;
constexpr int kNormPerWave = kWave / kNormLanes;
constexpr int kNormRanksPerLane = kZTab / kNormLanes;
static_assert(kZTab % kNormLanes == 0 && kWave % kNormLanes == 0, "ranks and half waves tile evenly");

template <typename R, int D>
__global__ __launch_bounds__(kWave * kNormWaves) void k_deposit_norm(MeshDev m, PhysDev ph, const uint32_t* nvalid,
                                                                    const uint32_t* order, const double* qd,
                                                                    int64_t N, double4* rpos, R* rw,
                                                                    unsigned long long* stats)
{
    constexpr int C = D + 1;
    constexpr int NL = kNormLanes;
    __shared__ NormLds<R> lds[kNormWaves][kNormPerWave];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int sub = lane / NL, sl = lane % NL;
    R (*S)[kZTab] = lds[wave][sub].S;
    R (*E)[kZTab] = lds[wave][sub].E;
    R* Ss = lds[wave][sub].Ss;
    double* Pf = lds[wave][sub].Pf;
    R* Es = lds[wave][sub].Es;
    const int64_t nv = (int64_t)*nvalid;
    const int64_t stride = (int64_t)gridDim.x * kNormWaves * kNormPerWave;
    for (int64_t p0 = ((int64_t)blockIdx.x * kNormWaves + wave) * kNormPerWave; p0 < nv; p0 += stride) {
        const int64_t p = p0 + sub;
        if (p < nv) {
            double4 P = rpos[p];
            double x[3] = {P.x, P.y, P.z};
            double inv_h = P.w;
            double h = 1.0 / inv_h;
            double rc = ph.cutoff * h * (1.0 + kSupportMargin);
            R c2;
            {
                R c = (R)ph.cutoff;
                c2 = c * c;
            }
            int64_t lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
            for (int a = 0; a < D; ++a) {
                double flo = (x[a] - rc - m.lo[a]) / m.w[a] - 0.5 - 1e-9;
                double fhi = (x[a] + rc - m.lo[a]) / m.w[a] - 0.5 + 1e-9;
                flo = fmin(fmax(flo, -4.0e15), 4.0e15);
                fhi = fmin(fmax(fhi, -4.0e15), 4.0e15);
                int64_t ilo = (int64_t)ceil(flo), ihi = (int64_t)floor(fhi);
                if (m.periodic[a]) {
                    if (ihi - ilo + 1 >= m.n[a]) { ilo = 0; ihi = m.n[a] - 1; }
                } else {
                    ilo = ilo < 0 ? 0 : ilo;
                    ihi = ihi >= m.n[a] ? m.n[a] - 1 : ihi;
                }
                lo[a] = ilo;
                cnt[a] = ihi - ilo + 1;
                if (cnt[a] < 0) cnt[a] = 0;
            }
            double z = 0.0;
            for (int64_t bz = 0; bz < cnt[2]; bz += kZTab)
            for (int64_t by = 0; by < cnt[1]; by += kZTab)
            for (int64_t bx = 0; bx < cnt[0]; bx += kZTab) {
                int64_t b0[3] = {bx, by, bz};
                int len[3];
                for (int a = 0; a < 3; ++a) {
                    int64_t l = cnt[a] - b0[a];
                    len[a] = (int)(l < kZTab ? l : kZTab);
                }
                wave_sync();
                for (int a = 0; a < D; ++a) {
                    for (int j = sl; j < len[a]; j += NL) {
                        int64_t ci = lo[a] + b0[a] + j;
                        if (m.periodic[a]) ci = posmod(ci, m.n[a]);
                        axis_factor<R>(m, a, ci, x[a], inv_h, S[a][j], E[a][j]);
                    }
                }
                if (D == 2 && sl == 0) { S[2][0] = 0; E[2][0] = 1; }
                wave_sync();
                // rank of each S0 (ties broken by index): a permutation of 0..len0-1
                for (int j = sl; j < len[0]; j += NL) {
                    const R v = S[0][j];
                    int r = 0;
                    for (int i = 0; i < len[0]; ++i) {
                        const R u = S[0][i];
                        r += (u < v || (u == v && i < j)) ? 1 : 0;
                    }
                    Ss[r] = v;
                    Es[r] = E[0][j];
                }
                wave_sync();
                // prefix sums of E0 in rank order: lane sl owns ranks
                // kNormRanksPerLane sl .. + kNormRanksPerLane - 1
                {
                    double e[kNormRanksPerLane], part = 0.0;
#pragma unroll
                    for (int q = 0; q < kNormRanksPerLane; ++q) {
                        const int r = kNormRanksPerLane * sl + q;
                        e[q] = r < len[0] ? (double)Es[r] : 0.0;
                        part += e[q];
                    }
                    double incl = part;
#pragma unroll
                    for (int o = 1; o < NL; o <<= 1) {
                        double t = __shfl_up(incl, o, NL);
                        if (sl >= o) incl += t;
                    }
                    double run = incl - part;
                    if (sl == 0) Pf[0] = 0.0;
#pragma unroll
                    for (int q = 0; q < kNormRanksPerLane; ++q) {
                        const int r = kNormRanksPerLane * sl + q;
                        run += e[q];
                        if (r < len[0]) Pf[r + 1] = run;
                    }
                }
                wave_sync();
                const int n0 = len[0];
                const R smin = Ss[0];
                const int64_t rows = (int64_t)len[1] * (D == 3 ? len[2] : 1);
                for (int64_t j = sl; j < rows; j += NL) {
                    const int jy = (int)(j % len[1]);
                    const int jz = (int)(j / len[1]);
                    const R sy = S[1][jy], sz = S[2][jz];
                    // number of ranks k with (Ss[k] + sy) + sz <= c^2 (a prefix)
                    R s = smin + sy;
                    if (D == 3) s = s + sz;
                    if (!(s <= c2)) continue;
                    int klo = 1, khi = n0;
                    while (klo < khi) {
                        const int mid = (klo + khi + 1) >> 1;
                        R t = Ss[mid - 1] + sy;
                        if (D == 3) t = t + sz;
                        if (t <= c2)
                            klo = mid;
                        else
                            khi = mid - 1;
                    }
                    z += Pf[klo] * ((double)E[1][jy] * (double)E[2][jz]);
                }
            }
#pragma unroll
            for (int o = NL / 2; o > 0; o >>= 1) z += __shfl_xor(z, o, NL);
            if (sl == 0) {
                // K_ci / Z_i = E_ci / z_i with z_i = sum_c E_ci (the 1/h factors cancel)
                uint32_t i = order[p];
                R* w = rw + p * kRecW;
                if (z > 0.0) {
                    w[0] = (R)inv_h;
                    for (int k = 0; k < C; ++k) w[1 + k] = (R)(qd[(int64_t)k * N + i] / z);
                } else {
                    w[0] = (R)0;
                    for (int k = 0; k < C; ++k) w[1 + k] = (R)qd[(int64_t)k * N + i];
                    rpos[p].w = -inv_h;
                    atomicAdd(&stats[ST_ZERO], 1ull);
                }
            }
        }
        wave_sync();   // the tables are rewritten for the next trajectory
    }
}

// ---------------------------------------------------------------- launchers
template <typename R, int D>
hipError_t launch_prepass(const TrajDev& t, const MeshDev& m, const PhysDev& ph, const float* hfac,
                          int deposit, uint32_t* keys, uint32_t* vals, double4* rpos, R* rw,
                          double* qd, unsigned long long* stats, hipStream_t s)
{
    if (t.count == 0) return hipSuccess;
    const int64_t per_block = 256 * kPrepassPerThread;
    unsigned nb = (unsigned)((t.count + per_block - 1) / per_block);
    FLA_LAUNCH((k_prepass<R, D>), dim3(nb), dim3(256), 0, s, t, m, ph, hfac, deposit, keys, vals,
                       rpos, rw, qd, stats);
    return hipGetLastError();
}

hipError_t launch_bucket_bounds(const uint32_t* keys, int64_t n, uint32_t nb, uint32_t* bstart,
                                hipStream_t s)
{
    unsigned g = (unsigned)(((int64_t)nb + 1 + 255) / 256);
    FLA_LAUNCH(k_bucket_bounds, dim3(g), dim3(256), 0, s, keys, n, nb, bstart);
    return hipGetLastError();
}

hipError_t launch_max_class(const uint32_t* bstart, int ntiles, unsigned long long* stats, hipStream_t s)
{
    FLA_LAUNCH(k_max_class, dim3(1), dim3(64), 0, s, bstart, ntiles, stats);
    return hipGetLastError();
}

hipError_t launch_max_class_batch(const BatchItem* items, int nsnap, const uint32_t* bstart,
                                  unsigned long long* stats, hipStream_t s)
{
    FLA_LAUNCH(k_max_class_batch, dim3(1), dim3(kWave), 0, s, items, nsnap, bstart, stats);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_permute(const uint32_t* order, int64_t n, const double4* rpos_u, const R* rw_u,
                          double4* rpos, R* rw, int copy_w, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = (unsigned)((n + 255) / 256);
    FLA_LAUNCH((k_permute<R>), dim3(g), dim3(256), 0, s, order, n, rpos_u, rw_u, rpos, rw, copy_w);
    return hipGetLastError();
}

template <typename R, int D>
hipError_t launch_deposit_norm(const MeshDev& m, const PhysDev& ph, const uint32_t* nvalid,
                               const uint32_t* order, const double* qd, int64_t N, double4* rpos, R* rw,
                               unsigned long long* stats, hipStream_t s)
{
    if (N == 0) return hipSuccess;
    const int64_t want = (N + kNormWaves * kNormPerWave - 1) / (kNormWaves * kNormPerWave);
    const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
    FLA_LAUNCH((k_deposit_norm<R, D>), dim3(grid), dim3(kWave * kNormWaves), 0, s, m, ph, nvalid, order,
                       qd, N, rpos, rw, stats);
    return hipGetLastError();
}

template <typename R, int D>
hipError_t launch_prepass_batch(const BatchItem* items, int nsnap, int64_t total, uint32_t sentinel, uint32_t* keys,
                                uint32_t* vals, double4* rpos, R* rw, unsigned long long* stats, hipStream_t s)
{
    if (total == 0) return hipSuccess;
    const int64_t per_block = 256 * kPrepassPerThread;
    unsigned nb = (unsigned)((total + per_block - 1) / per_block);
    FLA_LAUNCH((k_prepass_batch<R, D>), dim3(nb), dim3(256), 0, s, items, nsnap, total, sentinel, keys, vals,
                       rpos, rw, stats);
    return hipGetLastError();
}

#define FLP_INST(R, D)                                                                              \
    template hipError_t launch_prepass_batch<R, D>(const BatchItem*, int, int64_t, uint32_t, uint32_t*, \
                                                   uint32_t*, double4*, R*, unsigned long long*,     \
                                                   hipStream_t);                                     \
    template hipError_t launch_prepass<R, D>(const TrajDev&, const MeshDev&, const PhysDev&,        \
                                             const float*, int, uint32_t*, uint32_t*, double4*, R*, \
                                             double*, unsigned long long*, hipStream_t);            \
    template hipError_t launch_deposit_norm<R, D>(const MeshDev&, const PhysDev&, const uint32_t*,  \
                                                  const uint32_t*, const double*, int64_t,          \
                                                  double4*, R*, unsigned long long*, hipStream_t);
FLP_INST(float, 2)
FLP_INST(float, 3)
FLP_INST(double, 2)
FLP_INST(double, 3)
template hipError_t launch_permute<float>(const uint32_t*, int64_t, const double4*, const float*, double4*,
                                          float*, int, hipStream_t);
template hipError_t launch_permute<double>(const uint32_t*, int64_t, const double4*, const double*,
                                           double4*, double*, int, hipStream_t);

}  // namespace flp
