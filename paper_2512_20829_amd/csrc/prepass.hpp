// Record emission of the per-trajectory prepass, shared by the prepass
// kernels and the trajectory producer (which emits the same records from
// the state it has just integrated).
#pragma once

#include "internal.hpp"
#include "kernels.hpp"

namespace flp {

// Adds the sum over the wave of the per-lane counts c (0 <= c < 8) to
// stats[slot]: one ballot per bit and one atomic per wave.
__device__ inline void wave_count_sum(unsigned long long* stats, int slot, unsigned c)
{
    const unsigned long long n = (unsigned long long)__popcll(__ballot(c & 1u)) +
                                 2ull * (unsigned long long)__popcll(__ballot(c & 2u)) +
                                 4ull * (unsigned long long)__popcll(__ballot(c & 4u));
    if ((threadIdx.x % kWave) == 0 && n) atomicAdd(&stats[slot], n);
}

// Sort key of a trajectory on a Cartesian mesh: its home tile (linear tile
// index) and neighbourhood class (the largest distance in tiles, per axis,
// from the home tile to a tile holding a cell centre within rc; circular on
// periodic axes, where a support spanning the whole axis counts as the
// axis's tile count).  Returns false when no cell centre of a closed box is
// within reach.
template <int D>
struct LatticeKey {
    const MeshDev& m;
    __device__ uint32_t stride() const { return (uint32_t)m.ntiles; }
    __device__ bool operator()(const double* x, double rc, int64_t& tl, int& reach) const
    {
        constexpr int TE = Geo<D>::TE;
        int64_t ht[3] = {0, 0, 0};
        reach = 0;
        bool support = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            int64_t hc, ilo, ihi;
            if (m.edges[a]) {
                // rectilinear axis: the home cell and the cells whose centres
                // can lie within rc by binary search, over the periodic
                // extension on a periodic axis (index i of period k is
                // i + k n); the support interval is widened by 1e-12 of
                // |x| + rc + L, far more than the rounding of x -+ rc and of
                // the wrap
                const double* e = m.edges[a];
                const int n = m.n[a];
                const double sl = 1e-12 * (fabs(x[a]) + rc + m.L[a]);
                const double plo = x[a] - rc - sl, phi = x[a] + rc + sl;
                if (m.periodic[a]) {
                    const double kx = fmin(fmax(floor((x[a] - m.lo[a]) / m.L[a]), -1.0e12), 1.0e12);
                    const double kl = fmin(fmax(floor((plo - m.lo[a]) / m.L[a]), -1.0e12), 1.0e12);
                    const double kh = fmin(fmax(floor((phi - m.lo[a]) / m.L[a]), -1.0e12), 1.0e12);
                    hc = edge_cell(e, n, x[a] - kx * m.L[a]) + (int64_t)kx * n;
                    ilo = centre_at_or_above(e, n, plo - kl * m.L[a]) + (int64_t)kl * n;
                    ihi = centre_at_or_below(e, n, phi - kh * m.L[a]) + (int64_t)kh * n;
                } else {
                    hc = edge_cell(e, n, x[a]);
                    ilo = centre_at_or_above(e, n, plo);
                    ihi = centre_at_or_below(e, n, phi);
                }
            } else {
                // home cell by division, exactly as the gather's home_index; the
                // support bounds (they only choose the bucket class) by a
                // multiply with 1/w, widened by 1e-9 plus 1e-15 of the quotient,
                // far more than the few ulps by which the product can differ
                double g = floor((x[a] - m.lo[a]) / m.w[a]);
                g = fmin(fmax(g, -4.0e15), 4.0e15);
                hc = (int64_t)g;
                const double iw = 1.0 / m.w[a];
                const double qlo = (x[a] - rc - m.lo[a]) * iw, qhi = (x[a] + rc - m.lo[a]) * iw;
                double flo = qlo - 0.5 - (1e-9 + 1e-15 * fabs(qlo));
                double fhi = qhi - 0.5 + (1e-9 + 1e-15 * fabs(qhi));
                flo = fmin(fmax(flo, -4.0e15), 4.0e15);
                fhi = fmin(fmax(fhi, -4.0e15), 4.0e15);
                ilo = (int64_t)ceil(flo);
                ihi = (int64_t)floor(fhi);
            }
            int64_t ra;
            if (m.periodic[a]) {
                // tile distances are circular: the last tile of an axis whose
                // cell count is not a multiple of TE is short, so wrapped cells
                // are mapped back into [0, n) before taking their tile
                int64_t wrapped = posmod(hc, m.n[a]);
                int64_t sh = wrapped - hc;
                hc = wrapped;
                ilo += sh;
                ihi += sh;
                ht[a] = hc / TE;
                if (ilo > ihi) {
                    support = false;
                    ra = 0;
                } else if (ihi - ilo + 1 >= m.n[a]) {
                    ra = m.nt[a];
                } else {
                    int64_t tl = posmod(ilo, m.n[a]) / TE, tr = posmod(ihi, m.n[a]) / TE;
                    int64_t dl = ilo > hc ? 0 : posmod(ht[a] - tl, m.nt[a]);
                    int64_t dr = ihi < hc ? 0 : posmod(tr - ht[a], m.nt[a]);
                    ra = dl > dr ? dl : dr;
                }
            } else {
                hc = hc < 0 ? 0 : (hc >= m.n[a] ? m.n[a] - 1 : hc);
                ilo = ilo < 0 ? 0 : ilo;
                ihi = ihi >= m.n[a] ? m.n[a] - 1 : ihi;
                if (ilo > ihi) support = false;
                ht[a] = hc / TE;
                int64_t tlo = floordiv(ilo, TE), thi = floordiv(ihi, TE);
                ra = ht[a] - tlo;
                if (thi - ht[a] > ra) ra = thi - ht[a];
            }
            if (ra < 0) ra = 0;
            if (ra > kClasses) ra = kClasses;
            if ((int)ra > reach) reach = (int)ra;
        }
        tl = ht[0] + (int64_t)m.nt[0] * (ht[1] + (int64_t)m.nt[1] * ht[2]);
        return support;
    }
};

// Emits the prepass records of one trajectory of one snapshot (index i of
// count N), written at global index gi, from its binary64 position x,
// Jacobian J, initial number density n0 and source terms phi: the sort key
// (key_base + neighbourhood class * key.stride() + home tile or bucket from
// the keyer `key`, or `sentinel`), the
// unsorted position record {x, y, z, 1/h} and weight record {1/h, q/h}, with
// h = h0 |det J| fac and q = n0/|det J| phi (or, in deposition mode, the
// binary64 amounts Q = q V_seed |det J| to qd).  ok: the inputs are valid.
// Adds 1 to `skipped` / `nosup` when the trajectory is skipped or reaches no
// cell centre.
template <typename R, int D, typename K>
__device__ inline void emit_records(const K& key, const PhysDev& ph, double fac, int deposit, int64_t N, int64_t i,
                                    int64_t gi, uint32_t key_base, uint32_t sentinel, const double* x, const double* J,
                                    double n0, const double* phi_in, bool ok, double seed_volume, uint32_t* keys,
                                    uint32_t* vals, double4* rpos, R* rw, double* qd, unsigned long long& skipped,
                                    unsigned long long& nosup)
{
    constexpr int C = D + 1;
    double det = det_rn<D>(J);
    double adet = fabs(det);
    ok = ok && isfinite(n0) && isfinite(det) && det != 0.0 && isfinite(fac) && fac > 0.0;
    double h, n, phi[4] = {0, 0, 0, 0};
    {
#pragma clang fp contract(off)
        h = ph.h0 * adet;
        h = h * fac;
    }
    n = n0 / adet;
    if (ok)
#pragma unroll
        for (int k = 0; k < C; ++k) phi[k] = phi_in[k];
    if (ok) {
        ok = isfinite(h) && h > 0.0 && isfinite(n);
#pragma unroll
        for (int k = 0; k < C; ++k) ok = ok && isfinite(phi[k]);
    }
    uint32_t skey = sentinel;
    if (!ok) {
        skipped += 1;
    } else {
        double inv_h = 1.0 / h;
        double rc = ph.cutoff * h * (1.0 + kSupportMargin);
        int64_t tl = 0;
        int reach = 0;
        const bool support = key(x, rc, tl, reach);
        // In deposition mode a trajectory that reaches no cell centre still
        // deposits its whole amount into its home cell, so it is kept.
        if (!support) nosup += 1;
        if (support || deposit) {
            int cls = !support ? 0 : (reach < kClasses - 1 ? reach : kClasses - 1);
            skey = key_base + (uint32_t)cls * key.stride() + (uint32_t)tl;
        }
        rpos[gi] = make_double4(x[0], x[1], x[2], inv_h);
        // the weight record is built in registers and stored whole (16-byte stores)
        R w[kRecW];
#pragma unroll
        for (int k = 0; k < kRecW; ++k) w[k] = (R)0;
        w[0] = (R)inv_h;
        if (deposit) {
            double sc = seed_volume * adet;
#pragma unroll
            for (int k = 0; k < C; ++k) qd[(int64_t)k * N + i] = (n * phi[k]) * sc;
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) w[1 + k] = (R)(inv_h * (n * phi[k]));
        }
        static_assert(kRecW * sizeof(R) % sizeof(uint4) == 0, "weight records are whole 16-byte words");
        uint4* wd = reinterpret_cast<uint4*>(rw + gi * kRecW);
        const uint4* ws = reinterpret_cast<const uint4*>(w);
#pragma unroll
        for (int k = 0; k < (int)(kRecW * sizeof(R) / sizeof(uint4)); ++k) wd[k] = ws[k];
    }
    keys[gi] = skey;
    vals[gi] = (uint32_t)gi;
}

// Per-trajectory prepass of trajectory i of one snapshot, written at global
// index gi: loads the inputs, forms the droplet source terms and emits the
// records keyed by `key` (emit_records).
template <typename R, int D, typename K>
__device__ inline void prepass_traj(const TrajDev& t, const K& key, const PhysDev& ph, const float* hfac,
                                    int deposit, int64_t i, int64_t gi, uint32_t key_base, uint32_t sentinel,
                                    uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, double* qd,
                                    unsigned long long& skipped, unsigned long long& nosup)
{
    const int64_t N = t.count;
    double x[3] = {0, 0, 0}, J[9], v[3], ug[3];
    // every input is read, then tested with non-short-circuit ands, so that
    // the loads issue together instead of one test's branch at a time
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = t.x[a][i];
        v[a] = (double)((const R*)t.v[a])[i];
        ug[a] = (double)((const R*)t.ug[a])[i];
    }
#pragma unroll
    for (int e = 0; e < D * D; ++e) J[e] = t.J[(int64_t)e * N + i];
    const double r = (double)((const R*)t.r)[i];
    const double n0 = t.n0 ? t.n0[i] : t.n0_scalar;
    const double fac = hfac ? (double)hfac[i] : 1.0;
    int fin = isfinite(r);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        fin &= isfinite(x[a]);
        fin &= isfinite(v[a]);
        fin &= isfinite(ug[a]);
    }
#pragma unroll
    for (int e = 0; e < D * D; ++e) fin &= isfinite(J[e]);
    const bool ok = fin != 0;
    double phi[4] = {0, 0, 0, 0};
    if (ok) droplet_phi<D>(r, v, ug, ph, phi);
    emit_records<R, D>(key, ph, fac, deposit, N, i, gi, key_base, sentinel, x, J, n0, phi, ok, t.seed_volume, keys,
                       vals, rpos, rw, qd, skipped, nosup);
}

// The records of one trajectory keyed on a Cartesian mesh.
template <typename R, int D>
__device__ inline void prepass_emit(const MeshDev& m, const PhysDev& ph, double fac, int deposit, int64_t N, int64_t i,
                                    int64_t gi, uint32_t key_base, uint32_t sentinel, const double* x, const double* J,
                                    double n0, const double* phi_in, bool ok, double seed_volume, uint32_t* keys,
                                    uint32_t* vals, double4* rpos, R* rw, double* qd, unsigned long long& skipped,
                                    unsigned long long& nosup)
{
    emit_records<R, D>(LatticeKey<D>{m}, ph, fac, deposit, N, i, gi, key_base, sentinel, x, J, n0, phi_in, ok,
                       seed_volume, keys, vals, rpos, rw, qd, skipped, nosup);
}

}  // namespace flp
