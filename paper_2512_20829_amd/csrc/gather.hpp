// Cell-centric gather of the Nadaraya-Watson numerator and denominator
// (eqs. kernel-estimator, kernel and coupling-terms-kernel; App. B steps
// 1c, 1d, 2a, 2c) with the epilogue fused in.  No atomics touch the fields:
// every cell is owned by exactly one lane of one wave, and each lane visits
// the trajectories of its tile in a fixed order, so results are bitwise
// reproducible.
//
// Work decomposition (one workgroup of four 64-lane waves per part of a tile
// in 3-D: half the tile, cut across x, by default, or the whole tile; two
// waves per tile in 2-D; the waves take the candidate chunks in turn and
// their partial sums are added in wave order at the end; the workgroups are
// persistent and take their XCD's parts in heaviest-first order, k_gather):
//  * a tile is TE^D cells, split into 2^D sub-blocks of SB^D cells; lane l
//    owns the cell with in-block coordinates lc(l) in every sub-block of its
//    workgroup;
//  * candidate trajectories come from the buckets (class k, home tile) of
//    the neighbourhood of the tile: a class-k trajectory reaches at most k
//    tiles from its home tile (the last class spans whole axes);
//  * a conservative binary64 sphere/box test compacts candidates into an
//    LDS list (order preserved with wave ballots);
//  * per batch of 64 candidates the lanes build, in LDS, the per-axis factors
//    s = (d/h)^2 and e = exp(-s/2) for the cell centres of the workgroup on
//    every axis (the Gaussian is separable on a Cartesian mesh), plus the
//    per-half minima of s, in straight-line code (the minimum image and the
//    delta records take one branch per axis);
//  * every lane then walks the batch: a sub-block is visited only if the
//    minima admit a pair there (an exact, wave-uniform skip); a pair costs
//    2 adds, 1 compare, 2 multiplies, 1 select and C+1 multiply-adds; in
//    binary32 the C channel multiply-adds of a sub-block run as one
//    4x4x1 matrix instruction, and the 3-D plan-1 loop takes four records
//    per step under the union of their skips (records that reach no cell
//    of a visited pair of sub-blocks add exact zeros; the unions come from
//    two lane permutations of the masks);
//  * binary32 partial sums of one batch are folded into compensated
//    (TwoSum) totals, binary64 sums need no compensation.
//
// The tile part a workgroup owns is its shape: half a tile along x (the 3-D
// default, TP = 2) or the whole tile (TP = 1; always in 2-D).  Plan codes
// plan + kGatherPlans * shape select both (fla_autotune times them all).
//
// This header holds the kernels and their launchers; the units
// gather_{f32,f64}_{2d,3d}.hip instantiate them per precision and dimension,
// so that they compile in parallel.
#pragma once
#include "internal.hpp"
#include "kernels.hpp"

namespace flp {

// Gather mode of the Nadaraya-Watson estimator on any mesh (uniform or
// rectilinear axes); FLA_NW itself assumes uniform axes.
constexpr int kNwGeneral = 2;

constexpr int kCap = 2 * kWave;

typedef float F4 __attribute__((ext_vector_type(4)));

// A value that is the same on every lane, moved to scalar registers (the
// vector unit computes binary64 and binary32 values into vector registers).
__device__ inline double uniform_value(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline float uniform_value(float v)
{
    return __int_as_float((int)__builtin_amdgcn_readfirstlane((unsigned)__float_as_int(v)));
}

template <typename R> __device__ inline R r_inf();
template <> __device__ inline float r_inf<float>() { return __builtin_inff(); }
template <> __device__ inline double r_inf<double>() { return __builtin_inf(); }

template <typename R>
__device__ inline void two_sum_acc(R& hi, R& lo, R p)
{
    R s = hi + p;
    R bp = s - hi;
    R err = (hi - (s - bp)) + (p - bp);
    hi = s;
    lo += err;
}

// waves per workgroup (all work on one tile): four in 3-D; two in 2-D, whose
// tiles have twice the cells per axis and whose staging tables are larger
template <int D> struct GatherWaves { static constexpr int value = D == 3 ? 4 : 2; };

// Workgroups per tile (the shape).  With TP = 2 (3-D only) each workgroup
// owns one half of the tile along x (4 of its 8 sub-blocks), which halves
// the registers of its sums and its staging space, so that more workgroups
// share a compute unit, at the cost of scanning and staging every candidate
// once per half.  (Along x: the inclusion sum is ((s_x + s_y) + s_z), so
// sub-blocks paired along z still share their partial sum s_x + s_y.)
__host__ __device__ constexpr int tile_parts(int D, int shape) { return D == 3 && shape == 0 ? 2 : 1; }

// Waves per SIMD the register allocation is held to.
template <typename R, int D, int TP> struct GatherOcc {
    static constexpr int value = sizeof(R) == 4 ? (TP == 2 ? 3 : 2) : 1;
};

template <typename R, int D, int TP>
struct GatherLds {
    using R4 = typename V4<R>::T;
    using R2 = typename V2<R>::T;
    static constexpr int SB = Geo<D>::SB, NA = D + 2;
    static constexpr int NT = TP == 2 ? D - 1 : D;   // axes staged for both halves (split: y, z)
    uint32_t cand[kCap];               // compacted candidate record indices
    R4 tab[kWave][NT][SB];             // {s, e} at in-block position l and l + SB
    R2 tabs[kWave][TP == 2 ? SB : 1];  // split axis x: {s, e} of the owned half
    R wts[kWave][NA];                  // {1/h, q/h ...} of each staged record
    int mask[kWave];                   // sub-blocks holding at least one included pair
};

// Per-axis factors of one record for the tile at tile coordinates tc, whose
// cell centres are xcs: tab[a][l] = {s, e} at in-block positions l and
// l + SB of axis a, with s = (d/h)^2 (binary64 rounded to R) and
// e = exp(-s/2); with the split, axis x is staged for the owned half
// only, tabs[l] = {s, e} at position soff + l.  A delta record (1/h < 0) has
// factor 1 at its home cell and 0 elsewhere.  Returns the visit mask of the
// workgroup's sub-blocks: bit b is set iff the sum of the per-axis minima of
// s over sub-block b passes the cutoff (sums are monotone in each term, so
// no sub-block holding an included pair is skipped).
template <typename R, int D, int TP>
__device__ __forceinline__ int stage_record(const MeshDev& m, const double (*xcs)[Geo<D>::TE], const int* tc,
                                            const int soff, const double4 P, const R c2,
                                            typename V4<R>::T (*tab)[Geo<D>::SB], typename V2<R>::T* tabs)
{
    using G = Geo<D>;
    constexpr int TE = G::TE, SB = G::SB, NP = 2 * SB, NSB = G::NSB / TP;
    using R4 = typename V4<R>::T;
    using R2 = typename V2<R>::T;
    double x[3] = {P.x, P.y, P.z};
    const bool delta = P.w < 0.0;
    const double inv_h = delta ? -P.w : P.w;
    R mn[3][2];
    // Straight-line code per axis (the positions are independent chains);
    // the minimum image and the delta records take one branch per axis.
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const bool one = TP == 2 && a == 0;   // one half of this axis, at soff
        const int np = one ? SB : NP;
        double d[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            // positions l and l + SB of the sub-blocks, or soff + l
            const int pp = one ? soff + p : p;
            d[p] = (p < np) ? xcs[a][pp] - x[a] : 0.0;
        }
        if (m.periodic[a]) {
            // centres of cells beyond the mesh are NaN, ignored by fmax
            double dm = 0.0;
#pragma unroll
            for (int p = 0; p < NP; ++p) dm = fmax(dm, fabs(d[p]));
            const double L = m.L[a];
            if (dm > 0.5 * L) {
                if (dm < L) {
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
#pragma clang fp contract(off)
                        const double w = d[p] > 0.0 ? d[p] - L : d[p] + L;
                        d[p] = fabs(d[p]) <= 0.5 * L ? d[p] : w;
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < NP; ++p) d[p] = min_image(d[p], L);
                }
            }
        }
        // s = (d/h)^2 rounded to R, e = exp(-s/2); a NaN centre gives a NaN s,
        // which never passes the test and is ignored by the minima
        R sv[NP], ev[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            sv[p] = (R)scaled_sq(d[p], inv_h);
            ev[p] = gauss_factor(sv[p]);
        }
        if (delta) {
            // whole amount into the home cell: factor 1 there, 0 elsewhere
            const int64_t hcell = home_index(m, a, x[a]);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int pp = one ? soff + p : p;
                const bool home = (int64_t)tc[a] * TE + pp == hcell;
                sv[p] = home ? (R)0 : r_inf<R>();
                ev[p] = home ? (R)1 : (R)0;
            }
        }
        R mlo = r_inf<R>(), mhi = r_inf<R>();
#pragma unroll
        for (int l = 0; l < SB; ++l) {
            if (one) {
                R2 t2;
                t2.x = sv[l];
                t2.y = ev[l];
                tabs[l] = t2;
            } else {
                R4 t4;
                t4.x = sv[l];
                t4.y = ev[l];
                t4.z = sv[l + SB];
                t4.w = ev[l + SB];
                tab[TP == 2 ? a - 1 : a][l] = t4;
                mhi = fmin(mhi, sv[l + SB]);
            }
            mlo = fmin(mlo, sv[l]);
        }
        mn[a][0] = mlo;
        mn[a][1] = mhi;
    }
    // visit mask: the sub-block can hold an included pair (the sum of
    // the per-axis minima passes; binary32/64 sums are monotone in each
    // term, so the skip never drops an included pair)
    int mk = 0;
#pragma unroll
    for (int b = 0; b < NSB; ++b) {
        // sub-block bits: (x, y, z), or (y, z) with x split
        const int bx = TP == 2 ? 0 : b & 1;
        const int by = TP == 2 ? b & 1 : (b >> 1) & 1;
        const int bz = TP == 2 ? (b >> 1) & 1 : (b >> 2) & 1;
        R smin = mn[0][bx] + mn[1][by];
        if (D == 3) smin = smin + mn[2][bz];
        mk |= (smin <= c2) ? (1 << b) : 0;
    }
    return mk;
}

// Rows of home tiles that the tile at tile coordinates tc must consider for
// neighbourhood class k: the home tiles within k tiles of tc on every axis
// (the last class: whole axes), in rows along x, ordered z, then y; along x
// the home tiles of a row are contiguous in the sorted order (one run, or two
// across a periodic wrap, with tile ranges runs[q]).
struct ClassRows {
    uint32_t kb;        // first bucket of the class
    int lo_t[3], cnt_t[3];
    int runs[2][2];
    int nruns, nrows;
};

template <int D>
__device__ __forceinline__ void class_rows(const MeshDev& m, const int* tc, int k, ClassRows& cr)
{
    cr.kb = (uint32_t)k * (uint32_t)m.ntiles;
    const int r = (k == kClasses - 1) ? (1 << 28) : k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= D) {
            cr.lo_t[a] = 0;
            cr.cnt_t[a] = 1;
            continue;
        }
        int nt = m.nt[a];
        if (2 * (int64_t)r + 1 >= nt) {
            cr.lo_t[a] = 0;
            cr.cnt_t[a] = nt;
        } else if (m.periodic[a]) {
            cr.lo_t[a] = tc[a] - r;
            cr.cnt_t[a] = 2 * r + 1;
        } else {
            int l0 = tc[a] - r < 0 ? 0 : tc[a] - r;
            int l1 = tc[a] + r >= nt ? nt - 1 : tc[a] + r;
            cr.lo_t[a] = l0;
            cr.cnt_t[a] = l1 - l0 + 1;
        }
    }
    const int x0 = cr.lo_t[0], x1 = cr.lo_t[0] + cr.cnt_t[0] - 1;
    cr.nruns = 1;
    if (x0 < 0) {
        cr.runs[0][0] = x0 + m.nt[0];
        cr.runs[0][1] = m.nt[0] - 1;
        cr.runs[1][0] = 0;
        cr.runs[1][1] = x1;
        cr.nruns = 2;
    } else if (x1 >= m.nt[0]) {
        cr.runs[0][0] = x0;
        cr.runs[0][1] = m.nt[0] - 1;
        cr.runs[1][0] = 0;
        cr.runs[1][1] = x1 - m.nt[0];
        cr.nruns = 2;
    } else {
        cr.runs[0][0] = x0;
        cr.runs[0][1] = x1;
        cr.runs[1][0] = 0;
        cr.runs[1][1] = -1;
    }
    cr.nrows = cr.cnt_t[1] * cr.cnt_t[2];
}

// First bucket of row `row` of a class.
template <int D>
__device__ __forceinline__ uint32_t row_bucket(const MeshDev& m, const ClassRows& cr, int row)
{
    const int jz = row / cr.cnt_t[1], jy = row - jz * cr.cnt_t[1];
    int hz = cr.lo_t[2] + jz;
    if (D == 3) hz = (int)posmod(hz, m.nt[2]);
    const int hy = (int)posmod(cr.lo_t[1] + jy, m.nt[1]);
    return cr.kb + (uint32_t)m.nt[0] * ((uint32_t)hy + (uint32_t)m.nt[1] * (uint32_t)hz);
}

// Calls fn(s0, s1) for every non-empty run [s0, s1) of sorted records that
// the tile at tile coordinates tc must consider, class by class, row by row
// (class_rows).  The bucket bounds of up to 64 rows are fetched at once, one
// row per lane, and read back with readlane, so the rows do not wait on one
// scalar load each.
template <int D, typename F>
__device__ __forceinline__ void for_each_run(const MeshDev& m, const uint32_t* bstart, const int* tc,
                                             const int lane, F&& fn)
{
    for (int k = 0; k < kClasses; ++k) {
        const uint32_t kb = (uint32_t)k * (uint32_t)m.ntiles;
        if (bstart[kb] == bstart[kb + m.ntiles]) continue;
        ClassRows cr;
        class_rows<D>(m, tc, k, cr);
        for (int g0 = 0; g0 < cr.nrows; g0 += kWave) {
            // lane j fetches the bounds of row g0 + j
            uint32_t b00 = 0, b01 = 0, b10 = 0, b11 = 0;
            const int row = g0 + lane;
            if (row < cr.nrows) {
                const uint32_t rowb = row_bucket<D>(m, cr, row);
                b00 = bstart[rowb + cr.runs[0][0]];
                b01 = bstart[rowb + cr.runs[0][1] + 1];
                if (cr.nruns == 2) {
                    b10 = bstart[rowb + cr.runs[1][0]];
                    b11 = bstart[rowb + cr.runs[1][1] + 1];
                }
            }
            // runs in order: row by row, the runs of a row in x order
            const int nr = cr.nrows - g0 < kWave ? cr.nrows - g0 : kWave;
            for (int j = 0; j < nr * cr.nruns; ++j) {
                const int jr = cr.nruns == 2 ? j >> 1 : j;
                const bool second = cr.nruns == 2 && (j & 1);
                const uint32_t a0 = __builtin_amdgcn_readlane(b00, jr), a1 = __builtin_amdgcn_readlane(b01, jr);
                const uint32_t c0 = __builtin_amdgcn_readlane(b10, jr), c1 = __builtin_amdgcn_readlane(b11, jr);
                const uint32_t s0 = second ? c0 : a0, s1 = second ? c1 : a1;
                if (s0 < s1) fn(s0, s1);
            }
        }
    }
}

// Conservative test of one record against the tile: a delta record (1/h < 0)
// belongs to the tile of its home cell; any other record passes if the
// scaled binary64 distance from its position to the tile's box of cell
// centres (mid bmid, half-widths bhalf; axes where the box spans half a
// periodic box or more are not tested) is within filt2.
template <int D>
__device__ __forceinline__ bool candidate_ok(const MeshDev& m, const double4 P, const int* tc, const double* bmid,
                                             const double* bhalf, const bool* faxis, double filt2)
{
    constexpr int TE = Geo<D>::TE;
    double x[3] = {P.x, P.y, P.z};
    if (P.w < 0.0) {
        bool ok = true;
#pragma unroll
        for (int a = 0; a < D; ++a) ok = ok && (home_index(m, a, x[a]) / TE == tc[a]);
        return ok;
    }
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (!faxis[a]) continue;
        double d = fabs(axis_offset(m, a, bmid[a], x[a])) - bhalf[a];
        if (d > 0.0) {
            double u = d * P.w;
            acc += u * u;
        }
    }
    return acc <= filt2;
}

// The work of one workgroup: every cell of its part `work % TP` of tile
// `work / TP` of the mesh of g.
template <typename R, int D, int MODE, bool COUNT, int PLAN, int TP>
__device__ __forceinline__ void gather_tile(const GatherArgs& g, const int work)
{
    constexpr int kGatherWaves = GatherWaves<D>::value;
    using G = Geo<D>;
    static_assert(TP == 1 || D == 3, "tiles are split along x in 3-D only");
    constexpr int TE = G::TE, SB = G::SB, NSB = G::NSB / TP, C = D + 1, NA = C + 1;
    constexpr int NT = GatherLds<R, D, TP>::NT;
    constexpr bool kComp = sizeof(R) == 4;
    using R4 = typename V4<R>::T;
    using R2 = typename V2<R>::T;
    using L = GatherLds<R, D, TP>;
    static_assert(sizeof(L) * kGatherWaves >= sizeof(R) * kGatherWaves * NSB * NA * kWave,
                  "reduction buffer must fit in the staging space");
    __shared__ L lds[kGatherWaves];
    __shared__ double xcs[D][TE];

    const MeshDev& m = g.m;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    L& my = lds[wave];
    const int tile = work / TP;
    const int soff = (TP == 2) ? (work % TP) * SB : 0;   // first owned cell of the tile along x
    int tc[3];
    tc[0] = tile % m.nt[0];
    tc[1] = (tile / m.nt[0]) % m.nt[1];
    tc[2] = (D == 3) ? tile / (m.nt[0] * m.nt[1]) : 0;
    // a part lying wholly beyond the mesh has no cells (uniform over the workgroup)
    if (TP == 2 && (int64_t)tc[0] * TE + soff >= m.n[0]) return;

    // kNwGeneral takes any mesh (rectilinear axes read their edges); the
    // other modes assume uniform axes and compute the centres
    constexpr bool kGeneral = MODE == kNwGeneral;
    if (threadIdx.x < D * TE) {
        int a = threadIdx.x / TE, p = threadIdx.x % TE;
        int64_t idx = (int64_t)tc[a] * TE + p;
        xcs[a][p] = idx < m.n[a] ? (kGeneral ? cell_centre(m, a, idx) : uniform_centre(m, a, idx))
                                 : __builtin_nan("");
    }
    int lc[3];
    if (D == 3) {
        lc[0] = lane & 3;
        lc[1] = (lane >> 2) & 3;
        lc[2] = lane >> 4;
    } else {
        lc[0] = lane & 7;
        lc[1] = lane >> 3;
        lc[2] = 0;
    }
    R c2;
    {
        R c = (R)g.cutoff;
        c2 = uniform_value(c * c);
    }
    // conservative tile box of cell centres for the candidate filter: on
    // uniform axes from the formula (extrapolated past the last cell), on
    // rectilinear axes from the existing centres in the table.  (The box
    // decides which records are staged, hence where the binary32 partial
    // sums are folded: a uniform axis gets the same box in either mode, so
    // a uniform snapshot of a batch that also holds rectilinear ones keeps
    // the bits of its own call.)
    if (kGeneral) __syncthreads();
    double bmid[3] = {0, 0, 0}, bhalf[3] = {0, 0, 0};
    bool faxis[3] = {false, false, false};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const bool one = TP == 2 && a == 0;
        double f, l;
        if (kGeneral && m.edges[a]) {
            const int p0 = one ? soff : 0;
            int p1 = p0 + (one ? SB : TE) - 1;
            const int last = (int)(m.n[a] - 1 - (int64_t)tc[a] * TE);
            if (p1 > last) p1 = last;
            f = xcs[a][p0];
            l = xcs[a][p1];
        } else {
            const int64_t c0 = (int64_t)tc[a] * TE + (one ? soff : 0);
            f = uniform_centre(m, a, c0);
            l = uniform_centre(m, a, c0 + (one ? SB : TE) - 1);
        }
        bmid[a] = uniform_value(0.5 * (f + l));
        bhalf[a] = uniform_value(0.5 * (l - f));
        faxis[a] = !(m.periodic[a] && 4.0 * bhalf[a] >= m.L[a]);
    }

    // Binary32: the C source channels of a sub-block are accumulated on the
    // matrix unit (see `sub` below), the denominator on the vector unit.
    constexpr bool kMfma = sizeof(R) == 4;
    R part[NSB][NA];
    R hi[NSB][NA];
    R lo[NSB][NA];
    F4 acc[NSB];
#pragma unroll
    for (int b = 0; b < NSB; ++b) {
        acc[b] = F4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            part[b][k] = 0;
            hi[b][k] = 0;
            lo[b][k] = 0;
        }
    }
    // included pairs per sub-block of this lane (counted calls only)
    uint32_t cntb[NSB];
#pragma unroll
    for (int b = 0; b < NSB; ++b) cntb[b] = 0;
    const uint64_t ltmask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();

    // ---- one batch of n <= 64 staged candidates of this wave
    auto process = [&](int n) {
        wave_sync();
        if (lane < n) {
            uint32_t p = my.cand[lane];
            double4 P = g.rpos[p];
            const R* w = (const R*)g.rw + (size_t)p * kRecW;
#pragma unroll
            for (int k = 0; k < NA; ++k) my.wts[lane][k] = w[k];
            my.mask[lane] = stage_record<R, D, TP>(m, xcs, tc, soff, P, c2, my.tab[lane], my.tabs[lane]);
        }
        wave_sync();
        // every lane keeps the mask of one staged record (read with readlane,
        // no LDS round trip)
        const int maskv = (lane < n) ? my.mask[lane] : 0;
        // union of the masks of records 4q .. 4q + 3, on the lanes of quad q
        int mask4 = maskv | __builtin_amdgcn_mov_dpp(maskv, 0xB1, 0xF, 0xF, false);
        mask4 = mask4 | __builtin_amdgcn_mov_dpp(mask4, 0x4E, 0xF, 0xF, false);
        // one sub-block of one record: the per-pair inclusion test, then the
        // denominator multiply-add and the C channel multiply-adds.  In
        // binary32 the channels go to one v_mfma_f32_4x4x1_16b_f32: with A
        // broadcast from lanes 0..3 (cbsz 4, abid 0) it forms, in every
        // 4-lane block, the outer product of the record's channel weights
        // (lane m of A holds q_m/h) and the four lanes' kernel weights (B),
        // so that register k of lane l accumulates channel k of the lane's
        // cell: the layout of the vector path, with 4 multiply-adds per lane
        // moved off the vector unit.
        auto sub = [&](int b, const R4* t, const R2& ts, const R* wv, float wq, bool live = true) {
            R s, ew;
            if constexpr (TP == 2) {
                // x split: ts holds the owned half of x, t the y and z tables
                const int by = b & 1, bz = (b >> 1) & 1;
                s = ts.x + (by ? t[0].z : t[0].x);
                ew = ts.y * (by ? t[0].w : t[0].y);
                s = s + (bz ? t[1].z : t[1].x);
                ew = ew * (bz ? t[1].w : t[1].y);
            } else {
                const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
                s = (bx ? t[0].z : t[0].x) + (by ? t[1].z : t[1].x);
                ew = (bx ? t[0].w : t[0].y) * (by ? t[1].w : t[1].y);
                if constexpr (D == 3) {
                    s = s + (bz ? t[2].z : t[2].x);
                    ew = ew * (bz ? t[2].w : t[2].y);
                }
            }
            bool in = s <= c2;
            ew = in ? ew : (R)0;
            if constexpr (kMfma) {
                part[b][0] = fma(ew, wv[0], part[b][0]);
                acc[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(wq, (float)ew, acc[b], 4, 0, 0);
            } else {
#pragma unroll
                for (int k = 0; k < NA; ++k) part[b][k] = fma(ew, wv[k], part[b][k]);
            }
            if (COUNT) cntb[b] += (in && live) ? 1u : 0u;
        };
        // x split, sub-block b = by + 2 bz: the pair (by, 0), (by, 1) shares
        // s_x + s_y and e_x e_y
        auto pre = [&](int by, const R4* t, const R2& ts, R& sxy, R& exy) {
            sxy = ts.x + (by ? t[0].z : t[0].x);
            exy = ts.y * (by ? t[0].w : t[0].y);
        };
        auto fin = [&](int b, int bz, R sxy, R exy, const R4* t, const R* wv, float wq, bool live) {
            const R s = sxy + (bz ? t[1].z : t[1].x);
            R ew = exy * (bz ? t[1].w : t[1].y);
            const bool in = s <= c2;
            ew = in ? ew : (R)0;
            if constexpr (kMfma) {
                part[b][0] = fma(ew, wv[0], part[b][0]);
                acc[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(wq, (float)ew, acc[b], 4, 0, 0);
            } else {
#pragma unroll
                for (int k = 0; k < NA; ++k) part[b][k] = fma(ew, wv[k], part[b][k]);
            }
            if (COUNT) cntb[b] += (in && live) ? 1u : 0u;
        };
        // PLAN sets the granularity of the wave-uniform skips of a record that
        // reaches the workgroup's part: 0 one branch per sub-block, 1 per
        // pair of sub-blocks along z (3-D), 2 per half tile (whole tiles
        // have 8 sub-blocks; with the x split the part has 4, so 2 and 3
        // coincide), 3 none (every sub-block evaluated, masked by the pair
        // test); in 2-D, 1 and 2 evaluate the whole tile.  All plans add the
        // same products; a skipped sub-block only saves additions of zero.
        auto accumulate = [&](int e, const R4* t, const R2& ts, const R* wv, float wq) {
            const int mk = __builtin_amdgcn_readlane(maskv, e);
            if (mk == 0) return;
            if (PLAN == 3 || (D == 2 && PLAN != 0) || (PLAN == 2 && NSB == 4)) {
#pragma unroll
                for (int b = 0; b < NSB; ++b) sub(b, t, ts, wv, wq);
            } else if (PLAN == 2) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (mk & (0x0F << (4 * h))) {
#pragma unroll
                        for (int b = 4 * h; b < 4 * h + 4; ++b) sub(b, t, ts, wv, wq);
                    }
            } else if (PLAN == 1) {
#pragma unroll
                for (int q = 0; q < NSB / 2; ++q)
                    if (mk & (((1 << (NSB / 2)) | 1) << q)) {
                        sub(q, t, ts, wv, wq);
                        sub(q + NSB / 2, t, ts, wv, wq);
                    }
            } else {
#pragma unroll
                for (int b = 0; b < NSB; ++b)
                    if (mk & (1 << b)) sub(b, t, ts, wv, wq);
            }
        };
        // weights of staged record e: {1/h, q/h ...} on every lane, and, for
        // the matrix unit, q_m/h on lane m < C of each 4-lane group (0 on the
        // others)
        const int wm = lane & 3;
        auto load_w = [&](int e, R* w, float& wq) {
            if constexpr (kMfma) {
                w[0] = my.wts[e][0];
                wq = wm < C ? (float)my.wts[e][1 + (wm < C ? wm : 0)] : 0.0f;
            } else {
#pragma unroll
                for (int k = 0; k < NA; ++k) w[k] = my.wts[e][k];
                wq = 0.0f;
            }
        };
        // factors of staged record e at the lane's cells
        auto load_t = [&](int e, R4* t, R2& ts) {
#pragma unroll
            for (int a = 0; a < NT; ++a) t[a] = my.tab[e][a][lc[TP == 2 ? a + 1 : a]];
            if (TP == 2) ts = my.tabs[e][lc[0]];
        };
        R4 tA[NT], tB[NT];
        R2 hA, hB;
        R wA[NA], wB[NA];
        float qA, qB;
        if (PLAN == 1 && D == 3 && kMfma) {
            // Four records per step.  A pair of sub-blocks is evaluated for
            // all four records when any of them reaches it: a record that
            // reaches no cell there adds exact zeros (its kernel weights are
            // 0 on every lane), so the sums are those of one record at a
            // time, while the tests and branches are shared by four records
            // and the four independent chains fill the issue slots.  Slots
            // past the batch end repeat record e with zero weights and are
            // not counted as pairs.
            R4 tC[NT], tD[NT];
            R2 hC, hD;
            R wC[NA], wD[NA];
            float qC, qD;
            for (int e = 0; e < n; e += 4) {
                const bool l1 = e + 1 < n, l2 = e + 2 < n, l3 = e + 3 < n;
                const int e1 = l1 ? e + 1 : e;
                const int e2 = l2 ? e + 2 : e;
                const int e3 = l3 ? e + 3 : e;
                load_t(e, tA, hA);
                load_t(e1, tB, hB);
                load_t(e2, tC, hC);
                load_t(e3, tD, hD);
                load_w(e, wA, qA);
                load_w(e1, wB, qB);
                load_w(e2, wC, qC);
                load_w(e3, wD, qD);
                if (!l1) {
#pragma unroll
                    for (int k = 0; k < NA; ++k) wB[k] = 0;
                    qB = 0.0f;
                }
                if (!l2) {
#pragma unroll
                    for (int k = 0; k < NA; ++k) wC[k] = 0;
                    qC = 0.0f;
                }
                if (!l3) {
#pragma unroll
                    for (int k = 0; k < NA; ++k) wD[k] = 0;
                    qD = 0.0f;
                }
                const int mk = __builtin_amdgcn_readlane(mask4, e);
                if (mk == 0) continue;
                if constexpr (TP == 2) {
#pragma unroll
                    for (int q = 0; q < NSB / 2; ++q) {
                        const bool m0 = (mk >> q) & 1, m1 = (mk >> (q + NSB / 2)) & 1;
                        if (!(m0 || m1)) continue;
                        R sxy[4], exy[4];
                        pre(q, tA, hA, sxy[0], exy[0]);
                        pre(q, tB, hB, sxy[1], exy[1]);
                        pre(q, tC, hC, sxy[2], exy[2]);
                        pre(q, tD, hD, sxy[3], exy[3]);
                        if (m0) {
                            fin(q, 0, sxy[0], exy[0], tA, wA, qA, true);
                            fin(q, 0, sxy[1], exy[1], tB, wB, qB, l1);
                            fin(q, 0, sxy[2], exy[2], tC, wC, qC, l2);
                            fin(q, 0, sxy[3], exy[3], tD, wD, qD, l3);
                        }
                        if (m1) {
                            fin(q + NSB / 2, 1, sxy[0], exy[0], tA, wA, qA, true);
                            fin(q + NSB / 2, 1, sxy[1], exy[1], tB, wB, qB, l1);
                            fin(q + NSB / 2, 1, sxy[2], exy[2], tC, wC, qC, l2);
                            fin(q + NSB / 2, 1, sxy[3], exy[3], tD, wD, qD, l3);
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int q = 0; q < NSB / 2; ++q)
                    if (mk & (((1 << (NSB / 2)) | 1) << q)) {
                        sub(q, tA, hA, wA, qA);
                        sub(q + NSB / 2, tA, hA, wA, qA);
                        sub(q, tB, hB, wB, qB, l1);
                        sub(q + NSB / 2, tB, hB, wB, qB, l1);
                        sub(q, tC, hC, wC, qC, l2);
                        sub(q + NSB / 2, tC, hC, wC, qC, l2);
                        sub(q, tD, hD, wD, qD, l3);
                        sub(q + NSB / 2, tD, hD, wD, qD, l3);
                    }
            }
        } else {
            // one record at a time; the factors of the next record are read
            // while the current one is accumulated
            load_t(0, tA, hA);
            load_w(0, wA, qA);
            for (int e = 0; e < n; e += 2) {
                if (e + 1 < n) {
                    load_t(e + 1, tB, hB);
                    load_w(e + 1, wB, qB);
                }
                accumulate(e, tA, hA, wA, qA);
                if (e + 1 >= n) break;
                if (e + 2 < n) {
                    load_t(e + 2, tA, hA);
                    load_w(e + 2, wA, qA);
                }
                accumulate(e + 1, tB, hB, wB, qB);
            }
        }
        if (kComp) {
#pragma unroll
            for (int b = 0; b < NSB; ++b) {
                two_sum_acc(hi[b][0], lo[b][0], part[b][0]);
                part[b][0] = 0;
#pragma unroll
                for (int k = 1; k < NA; ++k) {
                    two_sum_acc(hi[b][k], lo[b][k], kMfma ? (R)acc[b][k - 1] : part[b][k]);
                    part[b][k] = 0;
                }
                acc[b] = F4{0.f, 0.f, 0.f, 0.f};
            }
        }
        wave_sync();
    };

    int ncand = 0;
    uint32_t chunk = 0;          // chunks of 64 candidates are dealt round-robin to the waves
    for_each_run<D>(m, g.bstart, tc, lane, [&](const uint32_t s0, const uint32_t s1) {
        // this wave's chunks of the run: base0, base0 + 4*64, ...
        const uint32_t nch = (s1 - s0 + kWave - 1) / kWave;
        const uint32_t first = (uint32_t)((wave - (int)(chunk % kGatherWaves) + kGatherWaves) % kGatherWaves);
        chunk += nch;
        double4 Pn = make_double4(0, 0, 0, 0);
        if (first < nch && s0 + first * kWave + lane < s1) Pn = g.rpos[s0 + first * kWave + lane];
        for (uint32_t c = first; c < nch; c += kGatherWaves) {
            const uint32_t base = s0 + c * kWave;
            uint32_t p = base + lane;
            double4 P = Pn;
            const uint32_t pn = base + kGatherWaves * kWave + lane;
            if (pn < s1) Pn = g.rpos[pn];
            const bool ok = p < s1 && candidate_ok<D>(m, P, tc, bmid, bhalf, faxis, g.filt2);
            uint64_t bal = __ballot(ok);
            if (ok) my.cand[ncand + __popcll(bal & ltmask)] = p;
            ncand += __popcll(bal);
            if (ncand >= kWave) {
                process(kWave);
                int rem = ncand - kWave;
                uint32_t mv = (lane < rem) ? my.cand[kWave + lane] : 0u;
                wave_sync();
                if (lane < rem) my.cand[lane] = mv;
                ncand = rem;
            }
        }
    });
    if (ncand > 0) process(ncand);

    // ---- fixed-order reduction of the waves' partial sums through LDS
    __syncthreads();
    R* red = reinterpret_cast<R*>(lds);   // [wave][b][k][lane]
#pragma unroll
    for (int b = 0; b < NSB; ++b)
#pragma unroll
        for (int k = 0; k < NA; ++k)
            red[((wave * NSB + b) * NA + k) * kWave + lane] = kComp ? hi[b][k] + lo[b][k] : part[b][k];
    __syncthreads();

    // linear index of the lane's cell in sub-block b; false beyond the mesh
    auto cell_of = [&](int b, int64_t& lin) {
        int64_t cidx[3] = {0, 0, 0};
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            int half;
            if (TP == 2)
                half = a == 0 ? soff : ((b >> (a > 0 ? a - 1 : 0)) & 1) * SB;
            else
                half = ((b >> a) & 1) * SB;
            cidx[a] = (int64_t)tc[a] * TE + half + lc[a];
            inside = inside && cidx[a] < m.n[a];
        }
        lin = cidx[0] + (int64_t)m.n[0] * (cidx[1] + (int64_t)m.n[1] * cidx[2]);
        return inside;
    };

    // ---- epilogue: divide (NW) or scale by 1/V_c (deposition), sign, scale
    for (int b = wave; b < NSB; b += kGatherWaves) {
        int64_t lin;
        if (!cell_of(b, lin)) continue;
        double tot[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            double acc = 0.0;
            for (int v = 0; v < kGatherWaves; ++v) acc += (double)red[((v * NSB + b) * NA + k) * kWave + lane];
            tot[k] = acc;
        }
        double den = tot[0];
        double cs = g.cell_scale ? (double)((const R*)g.cell_scale)[lin] : 1.0;
        double f = -g.scale * cs;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            double val;
            if (MODE != FLA_DEPOSIT)
                val = (den > 0.0) ? f * (tot[1 + k] / den) : 0.0;
            else
                val = f * tot[1 + k] / m.vol;
            ((R*)g.out[k])[lin] = (R)val;
        }
        if (g.den) ((R*)g.den)[lin] = (R)den;
    }
    if (COUNT) {
        // every wave holds counts for all of the workgroup's cells (the
        // waves split the candidates, not the cells); integer sums do not
        // depend on the order of the atomic additions
        unsigned long long npairs = 0;
#pragma unroll
        for (int b = 0; b < NSB; ++b) {
            npairs += cntb[b];
            int64_t lin;
            if (g.pairs && cntb[b] && cell_of(b, lin)) atomicAdd(&g.pairs[lin], cntb[b]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) npairs += __shfl_xor(npairs, o, kWave);
        if (lane == 0 && npairs) atomicAdd(&g.stats[ST_PAIRS], npairs);
    }
}

// Slot b of the launch belongs to XCD b % kXcds and computes the work item
// order[xcd_remap(b)] (the heaviest items of each XCD first).  Without a
// queue every workgroup takes its own slot; with one, the workgroups (as many
// as the compute units hold) take their XCD's slots x, x + kXcds, ... in
// order from that XCD's counter until they pass the end, so a workgroup that
// finishes early starts the next item at once (128^3: 4.93 -> 4.80 ms).  Which
// workgroup computes an item does not change its results.
template <typename R, int D, int MODE, bool COUNT, int PLAN, int TP>
static __global__ __launch_bounds__(kWave * GatherWaves<D>::value, (GatherOcc<R, D, TP>::value)) void k_gather(GatherArgs g)
{
    const int total = g.m.ntiles * TP;
    if (!g.queue) {
        int w = xcd_remap(blockIdx.x, total);
        if (g.order) w = g.order[w];
        gather_tile<R, D, MODE, COUNT, PLAN, TP>(g, w);
        return;
    }
    __shared__ int s_slot;
    const int x = blockIdx.x % kXcds;
    for (;;) {
        __syncthreads();   // every lane has read the previous slot
        if (threadIdx.x == 0) s_slot = x + kXcds * (int)atomicAdd(&g.queue[x], 1u);
        __syncthreads();
        const int slot = s_slot;
        if (slot >= total) break;
        int w = xcd_remap(slot, total);
        if (g.order) w = g.order[w];
        gather_tile<R, D, MODE, COUNT, PLAN, TP>(g, w);
    }
}

// Estimated work of every tile: the number of candidate records its scan
// visits (the bucket sizes over its class neighbourhoods).  One wave per
// tile, a row per lane.
template <int D>
static __global__ __launch_bounds__(256) void k_tile_cost(GatherArgs g)
{
    const MeshDev& m = g.m;
    const int tile = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int lane = threadIdx.x % kWave;
    if (tile >= m.ntiles) return;   // whole waves
    int tc[3];
    tc[0] = tile % m.nt[0];
    tc[1] = (tile / m.nt[0]) % m.nt[1];
    tc[2] = (D == 3) ? tile / (m.nt[0] * m.nt[1]) : 0;
    uint32_t c = 0;
    for (int k = 0; k < kClasses; ++k) {
        const uint32_t kb = (uint32_t)k * (uint32_t)m.ntiles;
        if (g.bstart[kb] == g.bstart[kb + m.ntiles]) continue;
        ClassRows cr;
        class_rows<D>(m, tc, k, cr);
        for (int row = lane; row < cr.nrows; row += kWave) {
            const uint32_t rowb = row_bucket<D>(m, cr, row);
            for (int q = 0; q < cr.nruns; ++q)
                c += g.bstart[rowb + cr.runs[q][1] + 1] - g.bstart[rowb + cr.runs[q][0]];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (lane == 0) g.tile_cost[tile] = c;
}

// Work order of the single-snapshot gather.  Workgroups are dealt
// round-robin over the XCDs and xcd_remap gives each XCD a contiguous range
// of slots; inside its range (one workgroup of this kernel per XCD) the work
// units are placed in descending classes of their tile's cost (four classes
// per power of two), so that the heaviest tiles start first and the light
// ones fill the end.  The order inside a class is immaterial: a work unit's
// results do not depend on the slot that computes it.
constexpr int kOrderBins = 33 * 4;
static __global__ __launch_bounds__(1024) void k_tile_order(const uint32_t* __restrict__ cost, int nunits, int zs,
                                                     int* __restrict__ order)
{
    __shared__ uint32_t cnt[kOrderBins];
    const int x = blockIdx.x;
    const int q = nunits / kXcds, rem = nunits % kXcds;
    const int s0 = x * q + (x < rem ? x : rem), n = q + (x < rem ? 1 : 0);
    auto bin = [](uint32_t c) {
        const int b = 32 - __clz(c);   // 0 for c = 0, else 1 + floor(log2 c)
        const int sub = b >= 3 ? (int)((c >> (b - 3)) & 3u) : 0;
        return b * 4 + sub;
    };
    for (int i = threadIdx.x; i < kOrderBins; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&cnt[bin(cost[(s0 + i) / zs])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = kOrderBins - 1; b >= 0; --b) {
            const uint32_t t = cnt[b];
            cnt[b] = acc;
            acc += t;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t pos = atomicAdd(&cnt[bin(cost[(s0 + i) / zs])], 1u);
        order[s0 + pos] = s0 + i;
    }
}

// Work item of workgroup `bid` of a batch of `nwork` items.  Workgroups are
// dealt round-robin over the XCDs in launch order; in every full chunk of
// kXcds * chunk items, XCD x receives the `chunk` consecutive items
// x * chunk ... x * chunk + chunk - 1, so neighbouring tiles of one snapshot
// share an L2 while the chunks still start in work-list order.
static __device__ inline int batch_work_item(int bid, int nwork, int chunk)
{
    const int span = kXcds * chunk;
    const int c = bid / span, off = bid % span;
    if ((c + 1) * span > nwork) return bid;
    return c * span + (off % kXcds) * chunk + off / kXcds;
}

// Persistent workgroups over the work items of a batch, one (snapshot,
// tile part) at a time.  The snapshots are stored in work-list order:
// items[s].tile_base is the first work item of snapshot s.  Slot b of the
// ordered launch (batch_work_item) belongs to XCD b % kXcds; each XCD has
// its own counter (queue[x], zeroed before the launch), from which its
// workgroups take that XCD's slots x, x + kXcds, ... in order until they
// pass the end.  Every item is taken exactly once, by a workgroup of the XCD
// the ordered launch gives it, and a workgroup that finishes early takes the
// next one instead of waiting for the dispatcher (on the 64-snapshot batch
// 37.5 against 38.4 ms).  Which workgroup computes an item does not change
// its results.
template <typename R, int D, int MODE, bool COUNT, int PLAN, int TP>
static __global__ __launch_bounds__(kWave * GatherWaves<D>::value, (GatherOcc<R, D, TP>::value)) void k_gather_batch(
    const BatchItem* __restrict__ items, int nsnap, int nwork, int chunk, uint32_t* __restrict__ queue)
{
    __shared__ int s_slot;
    const int total = nwork * TP;
    const int x = blockIdx.x % kXcds;
    for (;;) {
        __syncthreads();   // every lane has read the previous slot
        if (threadIdx.x == 0) s_slot = x + kXcds * (int)atomicAdd(&queue[x], 1u);
        __syncthreads();
        const int slot = s_slot;
        if (slot >= total) break;
        const int u = batch_work_item(slot, total, chunk);
        const int j = u / TP;         // tile-level work item
        int lo = 0, hi = nsnap - 1;   // last snapshot whose first work item is <= j
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].tile_base <= j)
                lo = mid;
            else
                hi = mid - 1;
        }
        gather_tile<R, D, MODE, COUNT, PLAN, TP>(items[lo].g, (j - items[lo].tile_base) * TP + u % TP);
    }
}

template <typename R, int D, int MODE, bool COUNT, int TP>
static void launch_plan(const GatherArgs& g, int plan, dim3 grid, dim3 block, hipStream_t s)
{
    switch (plan) {
    case 1: FLA_LAUNCH((k_gather<R, D, MODE, COUNT, 1, TP>), grid, block, 0, s, g); break;
    case 2: FLA_LAUNCH((k_gather<R, D, MODE, COUNT, 2, TP>), grid, block, 0, s, g); break;
    case 3: FLA_LAUNCH((k_gather<R, D, MODE, COUNT, 3, TP>), grid, block, 0, s, g); break;
    default: FLA_LAUNCH((k_gather<R, D, MODE, COUNT, 0, TP>), grid, block, 0, s, g); break;
    }
}

// Workgroups that the compute units hold at once (waves per SIMD from the
// register budget, 4 SIMDs per unit).
template <typename R, int D, int TP>
static int64_t resident_workgroups(int ncu)
{
    return (int64_t)(ncu > 0 ? ncu : 1) * GatherOcc<R, D, TP>::value * 4 / GatherWaves<D>::value;
}

template <typename R, int D, int MODE, bool COUNT, int TP>
static void launch_batch_plan(const BatchItem* items, int nsnap, int nwork, int chunk, int plan, uint32_t* queue,
                              int ncu, hipStream_t s)
{
    // as many workgroups as the compute units hold, at most one per item
    int64_t nb = resident_workgroups<R, D, TP>(ncu);
    const int64_t total = (int64_t)nwork * TP;
    if (nb > total) nb = total;
    if (nb < 1) nb = 1;
    dim3 grid((unsigned)nb), block(kWave * GatherWaves<D>::value);
    switch (plan) {
    case 1: FLA_LAUNCH((k_gather_batch<R, D, MODE, COUNT, 1, TP>), grid, block, 0, s, items, nsnap, nwork, chunk, queue); break;
    case 2: FLA_LAUNCH((k_gather_batch<R, D, MODE, COUNT, 2, TP>), grid, block, 0, s, items, nsnap, nwork, chunk, queue); break;
    case 3: FLA_LAUNCH((k_gather_batch<R, D, MODE, COUNT, 3, TP>), grid, block, 0, s, items, nsnap, nwork, chunk, queue); break;
    default: FLA_LAUNCH((k_gather_batch<R, D, MODE, COUNT, 0, TP>), grid, block, 0, s, items, nsnap, nwork, chunk, queue); break;
    }
}

template <typename R, int D, int TP>
static void launch_batch_shape(const BatchItem* items, int nsnap, int nwork, int chunk, bool count, int plan,
                               bool general, uint32_t* queue, int ncu, hipStream_t s)
{
    if (general) {
        if (count)
            launch_batch_plan<R, D, kNwGeneral, true, TP>(items, nsnap, nwork, chunk, plan, queue, ncu, s);
        else
            launch_batch_plan<R, D, kNwGeneral, false, TP>(items, nsnap, nwork, chunk, plan, queue, ncu, s);
    } else {
        if (count)
            launch_batch_plan<R, D, FLA_NW, true, TP>(items, nsnap, nwork, chunk, plan, queue, ncu, s);
        else
            launch_batch_plan<R, D, FLA_NW, false, TP>(items, nsnap, nwork, chunk, plan, queue, ncu, s);
    }
}

// plan_code = plan + kGatherPlans * shape (shape 1: whole tiles, 3-D only)
template <typename R, int D>
hipError_t launch_gather_batch(const BatchItem* items, int nsnap, int nwork, int chunk, bool count, int plan_code,
                               bool general, uint32_t* queue, int ncu, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    const int plan = plan_code % kGatherPlans, shape = plan_code / kGatherPlans;
    // the XCD counters start at zero (a fill kernel: the launch may be captured)
    hipError_t e = launch_fill_u32(queue, kXcds, 0u, s);
    if (e != hipSuccess) return e;
    if constexpr (D == 3) {
        if (tile_parts(D, shape) == 2) {
            launch_batch_shape<R, D, 2>(items, nsnap, nwork, chunk, count, plan, general, queue, ncu, s);
            return hipGetLastError();
        }
    }
    launch_batch_shape<R, D, 1>(items, nsnap, nwork, chunk, count, plan, general, queue, ncu, s);
    return hipGetLastError();
}

template <typename R, int D, int TP>
static hipError_t launch_gather_shape(const GatherArgs& g, int mode, bool count, int plan, hipStream_t s)
{
    if (g.order) {
        FLA_LAUNCH(k_tile_cost<D>, dim3((unsigned)((g.m.ntiles + 3) / 4)), dim3(256), 0, s, g);
        FLA_LAUNCH(k_tile_order, dim3(kXcds), dim3(1024), 0, s, (const uint32_t*)g.tile_cost, g.m.ntiles * TP, TP,
                   g.order);
    }
    int64_t nb = (int64_t)g.m.ntiles * TP;
    if (g.queue) {
        // as many workgroups as the compute units hold at once; the XCD
        // counters start at zero (a fill kernel: the launch may be captured)
        const int64_t fit = resident_workgroups<R, D, TP>(g.ncu);
        if (fit < nb) nb = fit;
        hipError_t e = launch_fill_u32(g.queue, kXcds, 0u, s);
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)nb), block(kWave * GatherWaves<D>::value);
    const bool general = g.m.edges[0] || g.m.edges[1] || g.m.edges[2];
    if (mode == FLA_NW && general) {
        if (count)
            launch_plan<R, D, kNwGeneral, true, TP>(g, plan, grid, block, s);
        else
            launch_plan<R, D, kNwGeneral, false, TP>(g, plan, grid, block, s);
    } else if (mode == FLA_NW) {
        if (count)
            launch_plan<R, D, FLA_NW, true, TP>(g, plan, grid, block, s);
        else
            launch_plan<R, D, FLA_NW, false, TP>(g, plan, grid, block, s);
    } else {
        if (count)
            launch_plan<R, D, FLA_DEPOSIT, true, TP>(g, plan, grid, block, s);
        else
            launch_plan<R, D, FLA_DEPOSIT, false, TP>(g, plan, grid, block, s);
    }
    return hipGetLastError();
}

template <typename R, int D>
hipError_t launch_gather(const GatherArgs& g, int mode, bool count, int plan_code, hipStream_t s)
{
    if (g.m.ntiles <= 0) return hipSuccess;
    const int plan = plan_code % kGatherPlans, shape = plan_code / kGatherPlans;
    if constexpr (D == 3) {
        if (tile_parts(D, shape) == 2) return launch_gather_shape<R, D, 2>(g, mode, count, plan, s);
    }
    return launch_gather_shape<R, D, 1>(g, mode, count, plan, s);
}

}  // namespace flp
