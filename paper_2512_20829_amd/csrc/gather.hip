// Cell-centric gather of the Nadaraya-Watson numerator and denominator
// (eqs. kernel-estimator, kernel and coupling-terms-kernel; App. B steps
// 1c, 1d, 2a, 2c) with the epilogue fused in.  No atomics touch the fields:
// every cell is owned by exactly one lane of one wave, and each lane visits
// the trajectories of its tile in a fixed order, so results are bitwise
// reproducible.
//
// Work decomposition (one 64-lane wave per tile):
//  * a tile is TE^D cells, split into 2^D sub-blocks of SB^D cells; lane l
//    owns the cell with in-block coordinates lc(l) in every sub-block;
//  * candidate trajectories come from the buckets (class k, home tile) of
//    the neighbourhood of the tile: a class-k trajectory reaches at most k
//    tiles from its home tile (the last class spans whole axes);
//  * a conservative binary64 sphere/box test compacts candidates into an
//    LDS list (order preserved with wave ballots);
//  * per batch of 64 candidates the lanes build, in LDS, the per-axis factors
//    s = (d/h)^2 and e = exp(-s/2) for the TE cell centres of the tile on
//    every axis (the Gaussian is separable on a Cartesian mesh), plus the
//    per-half minima of s;
//  * every lane then walks the batch: a sub-block is visited only if the
//    minima admit a pair there (an exact, wave-uniform skip); a pair costs
//    2 adds, 1 compare, 2 multiplies, 1 select and C+1 multiply-adds;
//  * binary32 partial sums of one batch are folded into compensated
//    (TwoSum) totals, binary64 sums need no compensation.
#include "internal.hpp"
#include "kernels.hpp"

namespace flp {

constexpr int kCap = 2 * kWave;

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

template <typename R, int D, int MODE, bool COUNT>
__global__ __launch_bounds__(64) void k_gather(GatherArgs g)
{
    using G = Geo<D>;
    constexpr int TE = G::TE, SB = G::SB, NSB = G::NSB, C = D + 1, NA = C + 1;
    constexpr bool kComp = sizeof(R) == 4;
    using R4 = typename V4<R>::T;
    __shared__ uint32_t cand[kCap];
    __shared__ R4 tab[kWave][D][SB];
    __shared__ R mins[kWave][D][2];
    __shared__ R wts[kWave][NA];
    __shared__ double xcs[D][TE];

    const MeshDev& m = g.m;
    const int lane = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, m.ntiles);
    int tc[3];
    tc[0] = tile % m.nt[0];
    tc[1] = (tile / m.nt[0]) % m.nt[1];
    tc[2] = (D == 3) ? tile / (m.nt[0] * m.nt[1]) : 0;

    if (lane < D * TE) {
        int a = lane / TE, p = lane % TE;
        xcs[a][p] = cell_centre(m, a, (int64_t)tc[a] * TE + p);
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
        c2 = c * c;
    }
    // conservative tile box of cell centres for the candidate filter
    double bmid[3] = {0, 0, 0}, bhalf[3] = {0, 0, 0};
    bool faxis[3] = {false, false, false};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double f = cell_centre(m, a, (int64_t)tc[a] * TE);
        double l = cell_centre(m, a, (int64_t)tc[a] * TE + TE - 1);
        bmid[a] = 0.5 * (f + l);
        bhalf[a] = 0.5 * (l - f);
        faxis[a] = !(m.periodic[a] && 4.0 * bhalf[a] >= m.L[a]);
    }

    R part[NSB][NA];
    R hi[NSB][NA];
    R lo[NSB][NA];
#pragma unroll
    for (int b = 0; b < NSB; ++b)
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            part[b][k] = 0;
            hi[b][k] = 0;
            lo[b][k] = 0;
        }
    unsigned long long npairs = 0;
    const uint64_t ltmask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();

    // ---- one batch of L <= 64 candidates: tables, then accumulation
    auto process = [&](int L) {
        __syncthreads();
        if (lane < L) {
            uint32_t p = cand[lane];
            double4 P = g.rpos[p];
            const R* w = (const R*)g.rw + (size_t)p * kRecW;
#pragma unroll
            for (int k = 0; k < NA; ++k) wts[lane][k] = w[k];
            double x[3] = {P.x, P.y, P.z};
            bool delta = P.w < 0.0;
            double inv_h = delta ? -P.w : P.w;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int64_t hcell = delta ? home_index(m, a, x[a]) : -1;
                R mlo = r_inf<R>(), mhi = r_inf<R>();
#pragma unroll
                for (int l = 0; l < SB; ++l) {
                    R s[2], e[2];
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        int pp = l + hh * SB;
                        int64_t idx = (int64_t)tc[a] * TE + pp;
                        if (idx >= m.n[a]) {
                            s[hh] = r_inf<R>();
                            e[hh] = 0;
                        } else if (delta) {
                            bool home = idx == hcell;
                            s[hh] = home ? (R)0 : r_inf<R>();
                            e[hh] = home ? (R)1 : (R)0;
                        } else {
                            double d = axis_offset(m, a, xcs[a][pp], x[a]);
                            R sr = (R)scaled_sq(d, inv_h);
                            s[hh] = sr;
                            e[hh] = exp((R)-0.5 * sr);
                        }
                    }
                    R4 t4;
                    t4.x = s[0];
                    t4.y = e[0];
                    t4.z = s[1];
                    t4.w = e[1];
                    tab[lane][a][l] = t4;
                    mlo = fmin(mlo, s[0]);
                    mhi = fmin(mhi, s[1]);
                }
                mins[lane][a][0] = mlo;
                mins[lane][a][1] = mhi;
            }
        }
        __syncthreads();
        for (int e = 0; e < L; ++e) {
            R mn[3][2];
            R4 t[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                mn[a][0] = mins[e][a][0];
                mn[a][1] = mins[e][a][1];
                t[a] = tab[e][a][lc[a]];
            }
            R wv[NA];
#pragma unroll
            for (int k = 0; k < NA; ++k) wv[k] = wts[e][k];
#pragma unroll
            for (int b = 0; b < NSB; ++b) {
                const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
                R smin = mn[0][bx] + mn[1][by];
                if (D == 3) smin = smin + mn[2][bz];
                if (smin <= c2) {
                    R s = (bx ? t[0].z : t[0].x) + (by ? t[1].z : t[1].x);
                    R ew = (bx ? t[0].w : t[0].y) * (by ? t[1].w : t[1].y);
                    if (D == 3) {
                        s = s + (bz ? t[2].z : t[2].x);
                        ew = ew * (bz ? t[2].w : t[2].y);
                    }
                    bool in = s <= c2;
                    ew = in ? ew : (R)0;
#pragma unroll
                    for (int k = 0; k < NA; ++k) part[b][k] = fma(ew, wv[k], part[b][k]);
                    if (COUNT) npairs += in ? 1ull : 0ull;
                }
            }
        }
        if (kComp) {
#pragma unroll
            for (int b = 0; b < NSB; ++b)
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    two_sum_acc(hi[b][k], lo[b][k], part[b][k]);
                    part[b][k] = 0;
                }
        }
    };

    int ncand = 0;
    const int ntl = m.ntiles;
    for (int k = 0; k < kClasses; ++k) {
        const uint32_t kb = (uint32_t)k * (uint32_t)ntl;
        if (g.bstart[kb] == g.bstart[kb + ntl]) continue;
        const int r = (k == kClasses - 1) ? (1 << 28) : k;
        int lo_t[3], cnt_t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a >= D) {
                lo_t[a] = 0;
                cnt_t[a] = 1;
                continue;
            }
            int nt = m.nt[a];
            if (2 * (int64_t)r + 1 >= nt) {
                lo_t[a] = 0;
                cnt_t[a] = nt;
            } else if (m.periodic[a]) {
                lo_t[a] = tc[a] - r;
                cnt_t[a] = 2 * r + 1;
            } else {
                int l0 = tc[a] - r < 0 ? 0 : tc[a] - r;
                int l1 = tc[a] + r >= nt ? nt - 1 : tc[a] + r;
                lo_t[a] = l0;
                cnt_t[a] = l1 - l0 + 1;
            }
        }
        for (int jz = 0; jz < cnt_t[2]; ++jz) {
            int hz = lo_t[2] + jz;
            if (D == 3) hz = (int)posmod(hz, m.nt[2]);
            for (int jy = 0; jy < cnt_t[1]; ++jy) {
                int hy = (int)posmod(lo_t[1] + jy, m.nt[1]);
                int x0 = lo_t[0], x1 = lo_t[0] + cnt_t[0] - 1;
                int runs[2][2];
                int nruns = 1;
                if (x0 < 0) {
                    runs[0][0] = x0 + m.nt[0];
                    runs[0][1] = m.nt[0] - 1;
                    runs[1][0] = 0;
                    runs[1][1] = x1;
                    nruns = 2;
                } else if (x1 >= m.nt[0]) {
                    runs[0][0] = x0;
                    runs[0][1] = m.nt[0] - 1;
                    runs[1][0] = 0;
                    runs[1][1] = x1 - m.nt[0];
                    nruns = 2;
                } else {
                    runs[0][0] = x0;
                    runs[0][1] = x1;
                }
                const uint32_t rowb = kb + (uint32_t)m.nt[0] * ((uint32_t)hy + (uint32_t)m.nt[1] * (uint32_t)hz);
                for (int q = 0; q < nruns; ++q) {
                    const uint32_t s0 = g.bstart[rowb + runs[q][0]];
                    const uint32_t s1 = g.bstart[rowb + runs[q][1] + 1];
                    for (uint32_t base = s0; base < s1; base += kWave) {
                        uint32_t p = base + lane;
                        bool ok = false;
                        if (p < s1) {
                            double4 P = g.rpos[p];
                            double x[3] = {P.x, P.y, P.z};
                            if (P.w < 0.0) {
                                ok = true;
#pragma unroll
                                for (int a = 0; a < D; ++a) ok = ok && (home_index(m, a, x[a]) / TE == tc[a]);
                            } else {
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
                                ok = acc <= g.filt2;
                            }
                        }
                        uint64_t bal = __ballot(ok);
                        if (ok) cand[ncand + __popcll(bal & ltmask)] = p;
                        ncand += __popcll(bal);
                        if (ncand >= kWave) {
                            process(kWave);
                            __syncthreads();
                            int rem = ncand - kWave;
                            uint32_t mv = (lane < rem) ? cand[kWave + lane] : 0u;
                            __syncthreads();
                            if (lane < rem) cand[lane] = mv;
                            ncand = rem;
                        }
                    }
                }
            }
        }
    }
    if (ncand > 0) process(ncand);

    // ---- epilogue: divide (NW) or scale by 1/V_c (deposition), sign, scale
#pragma unroll
    for (int b = 0; b < NSB; ++b) {
        int64_t cidx[3] = {0, 0, 0};
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cidx[a] = (int64_t)tc[a] * TE + ((b >> a) & 1) * SB + lc[a];
            inside = inside && cidx[a] < m.n[a];
        }
        if (!inside) continue;
        int64_t lin = cidx[0] + (int64_t)m.n[0] * (cidx[1] + (int64_t)m.n[1] * cidx[2]);
        R den = kComp ? hi[b][0] + lo[b][0] : part[b][0];
        double cs = g.cell_scale ? (double)((const R*)g.cell_scale)[lin] : 1.0;
        double f = -g.scale * cs;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            R num = kComp ? hi[b][1 + k] + lo[b][1 + k] : part[b][1 + k];
            double val;
            if (MODE == FLA_NW)
                val = (den > (R)0) ? f * ((double)num / (double)den) : 0.0;
            else
                val = f * (double)num / m.vol;
            ((R*)g.out[k])[lin] = (R)val;
        }
        if (g.den) ((R*)g.den)[lin] = den;
    }
    if (COUNT) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) npairs += __shfl_xor(npairs, o, kWave);
        if (lane == 0 && npairs) atomicAdd(&g.stats[ST_PAIRS], npairs);
    }
}

template <typename R, int D>
hipError_t launch_gather(const GatherArgs& g, int mode, bool count, hipStream_t s)
{
    dim3 grid((unsigned)g.m.ntiles), block(kWave);
    if (mode == FLA_NW) {
        if (count)
            hipLaunchKernelGGL((k_gather<R, D, FLA_NW, true>), grid, block, 0, s, g);
        else
            hipLaunchKernelGGL((k_gather<R, D, FLA_NW, false>), grid, block, 0, s, g);
    } else {
        if (count)
            hipLaunchKernelGGL((k_gather<R, D, FLA_DEPOSIT, true>), grid, block, 0, s, g);
        else
            hipLaunchKernelGGL((k_gather<R, D, FLA_DEPOSIT, false>), grid, block, 0, s, g);
    }
    return hipGetLastError();
}

template hipError_t launch_gather<float, 2>(const GatherArgs&, int, bool, hipStream_t);
template hipError_t launch_gather<float, 3>(const GatherArgs&, int, bool, hipStream_t);
template hipError_t launch_gather<double, 2>(const GatherArgs&, int, bool, hipStream_t);
template hipError_t launch_gather<double, 3>(const GatherArgs&, int, bool, hipStream_t);

}  // namespace flp
