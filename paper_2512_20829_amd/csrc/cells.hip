// FLA projection on general meshes: the cells are points (their centroids)
// with volumes, as on an unstructured finite-volume mesh.  The estimator
// (eqs. kernel-estimator, kernel, smoothing-length, coupling-terms-kernel)
// needs nothing of a cell but the point where it is evaluated, and the mesh
// enters the result only through the per-cell factor n_hat of App. A
// (eq. mv-scal: proportional to the cell volume).
//
// Spatial index (built once per mesh): a rectilinear grid of buckets whose
// per-axis edges sit at quantiles of the centroid coordinates, so that the
// buckets of a stretched or clustered mesh hold similar numbers of cells;
// cells sorted by bucket.  Trajectories are keyed by home bucket and
// neighbourhood class (distance in buckets to the farthest bucket their
// cutoff sphere reaches) and sorted, as on the Cartesian mesh.
//
// Gather: one wave per work item of up to kCellsPerItem cells of one bucket,
// each lane owning kCellsPerLane cells.  The wave walks the records of the
// buckets within reach class by class; records are wave-uniform and come
// through scalar loads, a record whose cutoff sphere misses the bounding box
// of the wave's cells is skipped as a whole, and each lane evaluates its
// pairs with the binary64 offsets and the inclusion test of the Cartesian
// gather (so both paths, and the oracle, take the same decisions).
#include "internal.hpp"
#include "kernels.hpp"
#include "prepass.hpp"

namespace flp {

// Number of interior edges e[1..nb-1] that are <= p: the bucket of p along
// one axis, clamped to [0, nb - 1].
__device__ inline int bucket_of(const double* e, int nb, double p)
{
    int l = 0, r = nb - 1;
    while (l < r) {
        const int mid = (l + r + 1) >> 1;
        if (e[mid] <= p)
            l = mid;
        else
            r = mid - 1;
    }
    return l;
}

// Histogram of the centroid coordinates per axis (kCellsHistBins equal bins
// over [lo, hi]) and validation: a centroid outside the box or not finite, or
// a volume that is negative or not finite, counts in *bad.
__global__ void k_cells_hist(int dim, int64_t M, const double* x0, const double* x1, const double* x2, double lo0,
                             double lo1, double lo2, double hi0, double hi1, double hi2, uint32_t* hist, uint32_t* bad,
                             const double* vol)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    const double* xs[3] = {x0, x1, x2};
    const double los[3] = {lo0, lo1, lo2}, his[3] = {hi0, hi1, hi2};
    bool ok = !vol || (isfinite(vol[c]) && vol[c] >= 0.0);
    for (int a = 0; a < dim; ++a) {
        const double x = xs[a][c];
        if (!(x >= los[a] && x <= his[a])) {       // also rejects NaN
            ok = false;
            continue;
        }
        double f = (x - los[a]) / (his[a] - los[a]) * (double)kCellsHistBins;
        int bin = (int)fmin(fmax(floor(f), 0.0), (double)(kCellsHistBins - 1));
        atomicAdd(&hist[(int64_t)a * kCellsHistBins + bin], 1u);
    }
    if (!ok) atomicAdd(bad, 1u);
}

hipError_t launch_cells_hist(int dim, int64_t M, const double* const* xc, const double* lo, const double* hi,
                             uint32_t* hist, uint32_t* bad, const double* vol, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    const int64_t blocks = (M + 255) / 256;
    FLA_LAUNCH(k_cells_hist, dim3((unsigned)blocks), dim3(256), 0, s, dim, M, xc[0], xc[1],
                       dim == 3 ? xc[2] : xc[0], lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], hist, bad, vol);
    return hipGetLastError();
}

// Bucket key (linear bucket index, axis 0 fastest) and identity value of each cell.
__global__ void k_cells_key(CellGridDev g, int64_t M, const double* x0, const double* x1, const double* x2,
                            uint32_t* keys, uint32_t* vals)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    const double* xs[3] = {x0, x1, x2};
    int64_t lin = 0, stride = 1;
    for (int a = 0; a < g.dim; ++a) {
        lin += stride * bucket_of(g.edges[a], g.nb[a], xs[a][c]);
        stride *= g.nb[a];
    }
    keys[c] = (uint32_t)lin;
    vals[c] = (uint32_t)c;
}

hipError_t launch_cells_key(const CellGridDev& g, int64_t M, const double* const* xc, uint32_t* keys, uint32_t* vals,
                            hipStream_t s)
{
    if (M == 0) return hipSuccess;
    const int64_t blocks = (M + 255) / 256;
    FLA_LAUNCH(k_cells_key, dim3((unsigned)blocks), dim3(256), 0, s, g, M, xc[0], xc[1],
                       g.dim == 3 ? xc[2] : xc[0], keys, vals);
    return hipGetLastError();
}

// Centroids and volumes in bucket order, and the permutation back.
__global__ void k_cells_sorted(int dim, int64_t M, const uint32_t* order, const double* x0, const double* x1,
                               const double* x2, const double* vol, double* s0, double* s1, double* s2, double* vs,
                               uint32_t* perm)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const uint32_t c = order[p];
    s0[p] = x0[c];
    s1[p] = x1[c];
    if (dim == 3) s2[p] = x2[c];
    if (vol) vs[p] = vol[c];
    perm[p] = c;
}

hipError_t launch_cells_sorted(int dim, int64_t M, const uint32_t* order, const double* const* xc, const double* vol,
                               double* const* xs, double* vs, uint32_t* perm, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    const int64_t blocks = (M + 255) / 256;
    FLA_LAUNCH(k_cells_sorted, dim3((unsigned)blocks), dim3(256), 0, s, dim, M, order, xc[0], xc[1],
                       dim == 3 ? xc[2] : xc[0], vol, xs[0], xs[1], dim == 3 ? xs[2] : xs[0], vs, perm);
    return hipGetLastError();
}

// Sort key of a trajectory on the bucket grid: home bucket and the largest
// per-axis distance in buckets (circular on periodic axes; a support that
// spans a whole periodic axis counts as the axis's bucket count) from the
// home bucket to a bucket that can hold a centroid within rc.  The support
// interval is widened by 1e-12 of |x| + rc + L, far more than the rounding of
// x -+ rc and of the periodic wrap.  Returns false when the interval misses
// a closed box (every centroid lies in the box).
template <int D>
struct BucketKey {
    const CellGridDev& g;
    __device__ uint32_t stride() const { return (uint32_t)g.nbuckets; }
    __device__ bool operator()(const double* x, double rc, int64_t& bl, int& reach) const
    {
        int hb[3] = {0, 0, 0};
        reach = 0;
        bool support = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int nb = g.nb[a];
            const double* e = g.edges[a];
            const double sl = 1e-12 * (fabs(x[a]) + rc + g.L[a]);
            const double plo = x[a] - rc - sl, phi = x[a] + rc + sl;
            int ra;
            if (g.periodic[a]) {
                const double xw = x[a] - floor((x[a] - g.lo[a]) / g.L[a]) * g.L[a];
                hb[a] = bucket_of(e, nb, xw);
                if (!(phi - plo < g.L[a])) {
                    ra = nb;
                } else {
                    const double lw = plo - floor((plo - g.lo[a]) / g.L[a]) * g.L[a];
                    const double hw = phi - floor((phi - g.lo[a]) / g.L[a]) * g.L[a];
                    const int blo = bucket_of(e, nb, lw), bhi = bucket_of(e, nb, hw);
                    int dl = hb[a] - blo, dr = bhi - hb[a];
                    dl = dl < 0 ? dl + nb : dl;
                    dr = dr < 0 ? dr + nb : dr;
                    ra = dl > dr ? dl : dr;
                }
            } else {
                if (phi < g.lo[a] || plo > g.hi[a]) support = false;
                const double xc = fmin(fmax(x[a], g.lo[a]), g.hi[a]);
                hb[a] = bucket_of(e, nb, xc);
                const int blo = bucket_of(e, nb, fmax(plo, g.lo[a])), bhi = bucket_of(e, nb, fmin(phi, g.hi[a]));
                ra = hb[a] - blo;
                if (bhi - hb[a] > ra) ra = bhi - hb[a];
            }
            if (ra < 0) ra = 0;
            if (ra > kClasses) ra = kClasses;
            if (ra > reach) reach = ra;
        }
        bl = hb[0] + (int64_t)g.nb[0] * (hb[1] + (int64_t)g.nb[1] * hb[2]);
        return support;
    }
};

constexpr int kCellsPrepassPerThread = 4;

template <typename R, int D>
__global__ __launch_bounds__(256) void k_cells_prepass(TrajDev t, CellGridDev g, PhysDev ph, const float* hfac,
                                                       uint32_t* keys, uint32_t* vals, double4* rpos, R* rw,
                                                       unsigned long long* stats)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kCellsPrepassPerThread + threadIdx.x;
    const uint32_t sentinel = (uint32_t)kClasses * (uint32_t)g.nbuckets;
    unsigned long long skipped = 0, nosup = 0;
    const BucketKey<D> key{g};
#pragma unroll
    for (int u = 0; u < kCellsPrepassPerThread; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        if (i < t.count)
            prepass_traj<R, D>(t, key, ph, hfac, 0, i, i, 0u, sentinel, keys, vals, rpos, rw, nullptr, skipped,
                               nosup);
    }
    wave_count_sum(stats, ST_SKIPPED, (unsigned)skipped);
    wave_count_sum(stats, ST_NOSUPPORT, (unsigned)nosup);
}

template <typename R, int D>
hipError_t launch_cells_prepass(const TrajDev& t, const CellGridDev& g, const PhysDev& ph, const float* hfac,
                                uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, unsigned long long* stats,
                                hipStream_t s)
{
    if (t.count == 0) return hipSuccess;
    const int64_t per = 256 * kCellsPrepassPerThread;
    const int64_t blocks = (t.count + per - 1) / per;
    FLA_LAUNCH((k_cells_prepass<R, D>), dim3((unsigned)blocks), dim3(256), 0, s, t, g, ph, hfac, keys, vals,
                       rpos, rw, stats);
    return hipGetLastError();
}

// Buckets within reach r of bucket b along one axis, as at most two runs
// [s, e] (a periodic axis wraps; a reach that covers the axis lists every
// bucket once).
__device__ inline int axis_runs(int b, int r, int nb, int periodic, int* s, int* e)
{
    if (periodic) {
        if (2 * r + 1 >= nb) {
            s[0] = 0;
            e[0] = nb - 1;
            return 1;
        }
        const int lo = b - r, hi = b + r;
        if (lo < 0) {
            s[0] = lo + nb;
            e[0] = nb - 1;
            s[1] = 0;
            e[1] = hi;
            return 2;
        }
        if (hi >= nb) {
            s[0] = lo;
            e[0] = nb - 1;
            s[1] = 0;
            e[1] = hi - nb;
            return 2;
        }
        s[0] = lo;
        e[0] = hi;
        return 1;
    }
    s[0] = b - r < 0 ? 0 : b - r;
    e[0] = b + r > nb - 1 ? nb - 1 : b + r;
    return 1;
}

__device__ inline double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline double uniform(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Running sums of one lane's cells: binary64 directly, binary32 in blocks
// folded into a compensated (hi, lo) pair.
template <typename R, int C> struct CellSums;
template <int C> struct CellSums<double, C> {
    double den[kCellsPerLane], num[kCellsPerLane][C];
    __device__ void zero()
    {
#pragma unroll
        for (int u = 0; u < kCellsPerLane; ++u) {
            den[u] = 0.0;
#pragma unroll
            for (int k = 0; k < C; ++k) num[u][k] = 0.0;
        }
    }
    __device__ void fold() {}
    __device__ double total_den(int u) const { return den[u]; }
    __device__ double total_num(int u, int k) const { return num[u][k]; }
};
template <int C> struct CellSums<float, C> {
    float den[kCellsPerLane], num[kCellsPerLane][C];            // current block
    float dhi[kCellsPerLane], dlo[kCellsPerLane];
    float nhi[kCellsPerLane][C], nlo[kCellsPerLane][C];
    __device__ void zero()
    {
#pragma unroll
        for (int u = 0; u < kCellsPerLane; ++u) {
            den[u] = dhi[u] = dlo[u] = 0.0f;
#pragma unroll
            for (int k = 0; k < C; ++k) num[u][k] = nhi[u][k] = nlo[u][k] = 0.0f;
        }
    }
    __device__ static void two_sum(float& hi, float& lo, float b)
    {
#pragma clang fp contract(off)
        const float s = hi + b;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (b - bb);
        hi = s;
        lo += err;
    }
    __device__ void fold()
    {
#pragma unroll
        for (int u = 0; u < kCellsPerLane; ++u) {
            two_sum(dhi[u], dlo[u], den[u]);
            den[u] = 0.0f;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                two_sum(nhi[u][k], nlo[u][k], num[u][k]);
                num[u][k] = 0.0f;
            }
        }
    }
    __device__ double total_den(int u) const { return (double)dhi[u] + (double)dlo[u]; }
    __device__ double total_num(int u, int k) const { return (double)nhi[u][k] + (double)nlo[u][k]; }
};

// records accumulated in binary32 before a fold into the compensated sums
constexpr int kCellsFoldEvery = 16;

template <typename R, int D, bool COUNT>
__global__ __launch_bounds__(256) void k_cells_gather(CellsGatherArgs a)
{
    constexpr int C = D + 1;
    constexpr int CPL = kCellsPerLane;
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int item = xcd_remap(blockIdx.x, gridDim.x) * (int)(blockDim.x / kWave) + wave;
    if (item >= a.nwork) return;
    const int4 wk = a.work[item];
    const int b = wk.x, first = wk.y, ncell = wk.z;
    int bc[3];
    bc[0] = b % a.g.nb[0];
    bc[1] = (b / a.g.nb[0]) % a.g.nb[1];
    bc[2] = D == 3 ? b / (a.g.nb[0] * a.g.nb[1]) : 0;

    double xc[CPL][3];
    bool act[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int k = u * kWave + lane;
        act[u] = k < ncell;
        const int p = first + (act[u] ? k : 0);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) xc[u][ax] = a.xc[ax][p];
    }
    // bounding box of the wave's cells: centre and half extent per axis
    double cb[3], eh[3];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        double lo = xc[0][ax], hi = xc[0][ax];
#pragma unroll
        for (int u = 1; u < CPL; ++u) {
            lo = fmin(lo, xc[u][ax]);
            hi = fmax(hi, xc[u][ax]);
        }
        lo = uniform(wave_min(lo));
        hi = uniform(wave_max(hi));
        cb[ax] = 0.5 * (lo + hi);
        eh[ax] = 0.5 * (hi - lo) * (1.0 + 1e-12) + 1e-300;
    }
    const float cf = (float)a.cutoff;
    const float c2f = cf * cf;
    double c2d;
    {
#pragma clang fp contract(off)
        c2d = a.cutoff * a.cutoff;
    }

    CellSums<R, C> acc;
    acc.zero();
    uint32_t np[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) np[u] = 0;
    int since_fold = 0;

    const int nbk = a.g.nbuckets;
    const R* rw = (const R*)a.rw;
    for (int k = 0; k < kClasses; ++k) {
        const uint32_t* bs = a.bstart + (int64_t)k * nbk;
        if (bs[0] == bs[nbk]) continue;
        const int r = (k == kClasses - 1) ? (1 << 28) : k;
        int xs[2], xe[2], ys[2], ye[2], zs[2], ze[2];
        const int nx = axis_runs(bc[0], r, a.g.nb[0], a.g.periodic[0], xs, xe);
        const int ny = axis_runs(bc[1], r, a.g.nb[1], a.g.periodic[1], ys, ye);
        int nz = 1;
        zs[0] = ze[0] = 0;
        if (D == 3) nz = axis_runs(bc[2], r, a.g.nb[2], a.g.periodic[2], zs, ze);
        for (int iz = 0; iz < nz; ++iz)
            for (int z = zs[iz]; z <= ze[iz]; ++z)
                for (int iy = 0; iy < ny; ++iy)
                    for (int y = ys[iy]; y <= ye[iy]; ++y) {
                        const int row = (z * a.g.nb[1] + y) * a.g.nb[0];
                        for (int ix = 0; ix < nx; ++ix) {
                            const uint32_t j0 = __builtin_amdgcn_readfirstlane(bs[row + xs[ix]]);
                            const uint32_t j1 = __builtin_amdgcn_readfirstlane(bs[row + xe[ix] + 1]);
                            for (uint32_t j = j0; j < j1; ++j) {
                                const double4 rp = a.rpos[j];
                                // skip a record whose cutoff sphere misses the wave's box
                                double gap2 = 0.0;
                                const double rx[3] = {rp.x, rp.y, rp.z};
#pragma unroll
                                for (int ax = 0; ax < D; ++ax) {
                                    double d = rx[ax] - cb[ax];
                                    if (a.g.periodic[ax]) d = min_image(d, a.g.L[ax]);
                                    const double gp = fabs(d) - eh[ax];
                                    if (gp > 0.0) gap2 += gp * gp;
                                }
                                if (gap2 * (rp.w * rp.w) > a.filt2) continue;
                                R w[C + 1];     // 1/h, then q_k/h
#pragma unroll
                                for (int q = 0; q <= C; ++q) w[q] = rw[(int64_t)j * kRecW + q];
#pragma unroll
                                for (int u = 0; u < CPL; ++u) {
                                    R s[3];
#pragma unroll
                                    for (int ax = 0; ax < D; ++ax) {
                                        double d;
                                        {
#pragma clang fp contract(off)
                                            d = xc[u][ax] - rx[ax];
                                        }
                                        if (a.g.periodic[ax]) d = min_image(d, a.g.L[ax]);
                                        s[ax] = (R)scaled_sq(d, rp.w);
                                    }
                                    R sum;
                                    {
#pragma clang fp contract(off)
                                        sum = s[0] + s[1];
                                        if (D == 3) sum = sum + s[2];
                                    }
                                    bool inc;
                                    if constexpr (sizeof(R) == 4)
                                        inc = sum <= c2f;
                                    else
                                        inc = sum <= c2d;
                                    inc = inc && act[u];
                                    if (inc) {
                                        const R e = gauss_factor(sum);
                                        acc.den[u] += e * w[0];
#pragma unroll
                                        for (int q = 0; q < C; ++q) acc.num[u][q] += e * w[1 + q];
                                        if (COUNT) np[u] += 1;
                                    }
                                }
                                if (sizeof(R) == 4 && ++since_fold == kCellsFoldEvery) {
                                    acc.fold();
                                    since_fold = 0;
                                }
                            }
                        }
                    }
    }
    acc.fold();

    unsigned long long wave_pairs = 0;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        if (!act[u]) continue;
        const int p = first + u * kWave + lane;
        const uint32_t cell = a.perm[p];
        const double den = acc.total_den(u);
        double f;
        {
#pragma clang fp contract(off)
            f = -a.scale * (a.use_vol ? a.vol[p] : 1.0);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const double S = den > 0.0 ? f * (acc.total_num(u, q) / den) : 0.0;
            ((R*)a.out[q])[cell] = (R)S;
        }
        if (a.den) ((R*)a.den)[cell] = (R)den;
        if (COUNT) {
            if (a.pairs) a.pairs[cell] = np[u];
            wave_pairs += np[u];
        }
    }
    if (COUNT) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wave_pairs += __shfl_xor(wave_pairs, o, kWave);
        if (lane == 0 && wave_pairs) atomicAdd(&a.stats[ST_PAIRS], wave_pairs);
    }
}

template <typename R, int D>
hipError_t launch_cells_gather(const CellsGatherArgs& a, bool count, hipStream_t s)
{
    if (a.nwork == 0) return hipSuccess;
    constexpr int kWavesPerBlock = 4;
    const int blocks = (a.nwork + kWavesPerBlock - 1) / kWavesPerBlock;
    if (count)
        FLA_LAUNCH((k_cells_gather<R, D, true>), dim3(blocks), dim3(kWave * kWavesPerBlock), 0, s, a);
    else
        FLA_LAUNCH((k_cells_gather<R, D, false>), dim3(blocks), dim3(kWave * kWavesPerBlock), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_cells_prepass<float, 2>(const TrajDev&, const CellGridDev&, const PhysDev&, const float*,
                                                   uint32_t*, uint32_t*, double4*, float*, unsigned long long*,
                                                   hipStream_t);
template hipError_t launch_cells_prepass<float, 3>(const TrajDev&, const CellGridDev&, const PhysDev&, const float*,
                                                   uint32_t*, uint32_t*, double4*, float*, unsigned long long*,
                                                   hipStream_t);
template hipError_t launch_cells_prepass<double, 2>(const TrajDev&, const CellGridDev&, const PhysDev&, const float*,
                                                    uint32_t*, uint32_t*, double4*, double*, unsigned long long*,
                                                    hipStream_t);
template hipError_t launch_cells_prepass<double, 3>(const TrajDev&, const CellGridDev&, const PhysDev&, const float*,
                                                    uint32_t*, uint32_t*, double4*, double*, unsigned long long*,
                                                    hipStream_t);
template hipError_t launch_cells_gather<float, 2>(const CellsGatherArgs&, bool, hipStream_t);
template hipError_t launch_cells_gather<float, 3>(const CellsGatherArgs&, bool, hipStream_t);
template hipError_t launch_cells_gather<double, 2>(const CellsGatherArgs&, bool, hipStream_t);
template hipError_t launch_cells_gather<double, 3>(const CellsGatherArgs&, bool, hipStream_t);

}  // namespace flp
