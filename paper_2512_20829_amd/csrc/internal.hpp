// Internal declarations of the gfx950 FLA projection library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flaproj.h"

namespace flp {

constexpr int kWave = 64;
constexpr int kClasses = 16;         // neighbourhood classes (reach 0..14 tiles, 15 = whole axes)
constexpr int kXcds = 8;             // XCDs per MI355X
constexpr int kRecW = 8;             // reals per weight record: w0, wq[0..C-1], padding
constexpr double kSupportMargin = 1e-5;  // relative widening of conservative support tests

// Tile geometry of the gather: a tile is TE^D cells processed by one wave,
// split into 2^D sub-blocks of SB^D cells; each lane owns one cell per sub-block.
template <int D> struct Geo;
template <> struct Geo<3> { static constexpr int TE = 8, SB = 4, NSB = 8; };
template <> struct Geo<2> { static constexpr int TE = 16, SB = 8, NSB = 4; };

struct MeshDev {
    int dim;
    int n[3];
    int periodic[3];
    int te;          // tile edge in cells
    int nt[3];       // tiles per axis
    int ntiles;
    int64_t M;
    double lo[3];
    double hi[3];
    double w[3];     // cell width (hi - lo)/n, computed on the host
    double L[3];     // box length hi - lo
    double vol;      // cell volume (uniform axes)
    // rectilinear axes: n[a] + 1 increasing cell edges (device, binary64),
    // NULL for a uniform axis; cell centres at the edge midpoints
    const double* edges[3];
};

struct TrajDev {
    int64_t count;
    const double* x[3];
    const double* J;
    const void* v[3];
    const void* ug[3];
    const void* r;
    const double* n0;
    double n0_scalar;
    double seed_volume;
};

struct PhysDev {
    double rho_d, mu, delta, h0, cutoff, scale;
};

// Launch log: when g_trace is nonzero (FLA_TRACE set in the environment
// when a context is created) every kernel launch is reported on stderr with
// its grid, block, LDS bytes and stream before it is enqueued.
extern int g_trace;
void trace_launch(const char* kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s);
#define FLA_LAUNCH(kern, grid, block, lds, stream, ...)                                           \
    do {                                                                                          \
        if (::flp::g_trace) ::flp::trace_launch(#kern, dim3(grid), dim3(block), (size_t)(lds), (stream)); \
        hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);                          \
    } while (0)

// statistics slots (device int64 array)
enum StatSlot { ST_TRAJ = 0, ST_SKIPPED, ST_NOSUPPORT, ST_PAIRS, ST_OUTSIDE, ST_ZERO, ST_MAXCLASS, ST_N };

// ---------------------------------------------------------------------------
// Exact-arithmetic helpers: binary64 operations whose rounding must not be
// altered by multiply-add contraction (they decide which pairs are included).
// ---------------------------------------------------------------------------
// Centre of cell i on a uniform axis.
__device__ inline double uniform_centre(const MeshDev& m, int a, int64_t i)
{
#pragma clang fp contract(off)
    double t = ((double)i + 0.5) * m.w[a];
    return m.lo[a] + t;
}

// Centre of cell i on a uniform or a rectilinear axis.
__device__ inline double cell_centre(const MeshDev& m, int a, int64_t i)
{
#pragma clang fp contract(off)
    if (m.edges[a]) {
        const double* e = m.edges[a];
        return 0.5 * (e[i] + e[i + 1]);
    }
    double t = ((double)i + 0.5) * m.w[a];
    return m.lo[a] + t;
}

// Rectilinear axes.  The cell holding p: the last edge e[i] <= p, clamped
// to [0, n - 1].
__device__ inline int64_t edge_cell(const double* e, int n, double p)
{
    int l = 0, r = n - 1;
    while (l < r) {
        const int mid = (l + r + 1) >> 1;
        if (e[mid] <= p)
            l = mid;
        else
            r = mid - 1;
    }
    return l;
}
// The first cell whose centre is >= p (n if none), and the last cell whose
// centre is <= p (-1 if none), over one period of the axis.
__device__ inline int64_t centre_at_or_above(const double* e, int n, double p)
{
    int l = 0, r = n;
    while (l < r) {
        const int mid = (l + r) >> 1;
        double c;
        {
#pragma clang fp contract(off)
            c = 0.5 * (e[mid] + e[mid + 1]);
        }
        if (c >= p)
            r = mid;
        else
            l = mid + 1;
    }
    return l;
}
__device__ inline int64_t centre_at_or_below(const double* e, int n, double p)
{
    int l = -1, r = n - 1;
    while (l < r) {
        const int mid = (l + r + 1) >> 1;
        double c;
        {
#pragma clang fp contract(off)
            c = 0.5 * (e[mid] + e[mid + 1]);
        }
        if (c <= p)
            l = mid;
        else
            r = mid - 1;
    }
    return l;
}

// Minimum image d - L rint(d/L) of an offset d on a periodic axis of length
// L, with the division only for |d| >= L.  For |d| < L the rounded quotient
// lies in [0, 1] in magnitude and exceeds 1/2 exactly when |d| > L/2: the
// binary64 numbers above 1/2 start at 1/2 + 2^-53, the midpoint 1/2 + 2^-54
// rounds to the even 1/2, and L/2 < L (1/2 + 2^-54) < succ(L/2), so for a
// binary64 d the test d/L > 1/2 + 2^-54 is d > L/2.  Hence rint(d/L) is 1
// for d > L/2, -1 for d < -L/2 and 0 otherwise (rint(1/2) = 0), and the
// result is d - L, d + L or d, each rounded once as in d - L*rint(d/L).
__device__ inline double min_image(double d, double L)
{
#pragma clang fp contract(off)
    const double ad = fabs(d);
    if (ad <= 0.5 * L) return d;
    if (ad < L) return d > 0.0 ? d - L : d + L;
    double k = rint(d / L);
    double s = L * k;
    return d - s;
}

// offset from point xp to centre xc along axis a; minimum image on periodic axes
__device__ inline double axis_offset(const MeshDev& m, int a, double xc, double xp)
{
#pragma clang fp contract(off)
    double d = xc - xp;
    if (m.periodic[a]) d = min_image(d, m.L[a]);
    return d;
}

__device__ inline double scaled_sq(double d, double inv_h)
{
#pragma clang fp contract(off)
    double u = d * inv_h;
    return u * u;
}

template <int D> __device__ inline double det_rn(const double* J);
template <> __device__ inline double det_rn<2>(const double* J)
{
#pragma clang fp contract(off)
    double p = J[0] * J[3];
    double q = J[1] * J[2];
    return p - q;
}
template <> __device__ inline double det_rn<3>(const double* J)
{
#pragma clang fp contract(off)
    double m0 = J[4] * J[8] - J[5] * J[7];
    double m1 = J[3] * J[8] - J[5] * J[6];
    double m2 = J[3] * J[7] - J[4] * J[6];
    double t0 = J[0] * m0;
    double t1 = J[1] * m1;
    double t2 = J[2] * m2;
    return (t0 - t1) + t2;
}

// exp(-s/2) of one axis: binary32 as exp2 of a pre-scaled argument (the
// hardware exponential; relative error a few 1e-7 for s <= 16), binary64 from
// the library.
__device__ inline float gauss_factor(float s) { return __builtin_amdgcn_exp2f(s * -0.72134752044448170368f); }
__device__ inline double gauss_factor(double s) { return exp(-0.5 * s); }

// Per-axis factors of the separable Gaussian for the cell centre with index
// ci on axis a and a trajectory at coordinate xp with bandwidth 1/inv_h:
//   s = (d/h)^2 in binary64, rounded to the working precision R,
//   e = exp(-s/2) in R.
// The product of e over the axes is exp(-|x_c - x_i|^2 / (2 h^2)); the sum of
// s over the axes (in R, axis order) decides inclusion against cutoff^2.
template <typename R>
__device__ inline void axis_factor(const MeshDev& m, int a, int64_t ci, double xp, double inv_h, R& s, R& e)
{
    double d = axis_offset(m, a, cell_centre(m, a, ci), xp);
    R sr = (R)scaled_sq(d, inv_h);
    s = sr;
    e = gauss_factor(sr);
}

// Droplet source channels of one droplet (in T; binary64 for the projection):
//   m = 4/3 pi rho r^3, tau = 2 rho r^2/(9 mu), F = m (ug - v)/tau,
//   mdot = 4 pi rho r^2 * delta/(2 r), phi = [mdot, F + mdot v]   (eqs. 3-5, 9)
template <int D, typename T>
__device__ inline void droplet_phi_t(T r, const T* v, const T* ug, const PhysDev& ph, T* phi)
{
    constexpr T kPi = (T)3.14159265358979323846;
    const T rho = (T)ph.rho_d;
    T m = ((T)4.0 / (T)3.0) * kPi * rho * r * r * r;
    T tau = (T)2.0 * rho * r * r / ((T)9.0 * (T)ph.mu);
    T rdot = (T)ph.delta / ((T)2.0 * r);
    T mdot = (T)4.0 * kPi * rho * r * r * rdot;
    phi[0] = mdot;
    const T m_tau = m / tau;   // one division for the D drag components
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T F = m_tau * (ug[a] - v[a]);
        phi[1 + a] = F + mdot * v[a];
    }
}

template <int D>
__device__ inline void droplet_phi(double r, const double* v, const double* ug, const PhysDev& ph, double* phi)
{
    droplet_phi_t<D, double>(r, v, ug, ph, phi);
}

// Floor division for possibly negative integers.
__device__ inline int64_t floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}
// a mod b in [0, b) for b > 0.  Indices within one period of [0, b) (all
// positions inside or next to the box) take no 64-bit division, which is a
// long instruction sequence on this hardware.
__device__ inline int64_t posmod(int64_t a, int64_t b)
{
    if (a >= 0 && a < b) return a;
    if (a < 0 && a >= -b) return a + b;
    if (a >= b && a - b < b) return a - b;
    int64_t r = a % b;
    return r < 0 ? r + b : r;
}

// Cell index of coordinate x on axis a: floor((x - lo)/w), wrapped on a periodic
// axis, clamped to the box on a closed one (the trajectory's home cell).
__device__ inline int64_t home_index(const MeshDev& m, int a, double x)
{
    double g = floor((x - m.lo[a]) / m.w[a]);
    g = fmin(fmax(g, -4.0e15), 4.0e15);
    int64_t k = (int64_t)g;
    if (m.periodic[a]) return posmod(k, m.n[a]);
    return k < 0 ? 0 : (k >= m.n[a] ? m.n[a] - 1 : k);
}

// Block remapping so that each XCD (workgroups are dealt round-robin over
// the XCDs) receives a contiguous range of tiles.
__device__ inline int xcd_remap(int bid, int nblocks)
{
    int q = nblocks / kXcds, rem = nblocks % kXcds;
    int x = bid % kXcds, j = bid / kXcds;
    return x * q + (x < rem ? x : rem) + j;
}

// Wave-level LDS synchronisation: orders this wave's LDS accesses across lanes
// without a workgroup barrier.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };
template <typename R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

// ---------------------------------------------------------------------------
// host-side helpers shared by the translation units
// ---------------------------------------------------------------------------
struct Workspace;

hipError_t launch_exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* tmp, int64_t tmp_words,
                                     hipStream_t s);
int64_t scan_tmp_words(int64_t n);

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                            int64_t n, int key_bits, uint32_t* hist, int64_t hist_words,
                            uint32_t* scan_tmp, int64_t scan_tmp_words_, hipStream_t s,
                            bool* result_in_alt);
int64_t radix_hist_words(int64_t n);

}  // namespace flp
