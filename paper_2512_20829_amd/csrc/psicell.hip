// PSI-CELL box counting (eqs. vol-avg-discrete and coupling-terms-definition)
// and small fill kernels.
//
// The sum over the particles of a cell is made order-independent by exact
// integer arithmetic: a first pass finds max |phi_k| per channel, each phi is
// then quantised to a multiple of 2^-e_k with e_k chosen so that
// count * max|phi_k| * 2^e_k <= 2^62 (no partial sum can overflow int64),
// and the integers are added with 64-bit atomics.  The quantisation error of
// one particle is at most 2^-(e_k+1), i.e. relative to the largest |phi|
// about count * 2^-63.  One HBM pass for the bound plus one for the sums.
#include "internal.hpp"
#include "kernels.hpp"

namespace flp {

template <typename R, int D>
__device__ inline bool psi_particle(const PsiArgs& a, int64_t p, int64_t& cell, double* phi)
{
    const MeshDev& m = a.m;
    int64_t lin = 0, stride = 1;
    double v[3], ug[3];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        double x = a.p.x[ax][p];
        if (!isfinite(x)) return false;
        double g = floor((x - m.lo[ax]) / m.w[ax]);
        if (!(fabs(g) < 9.0e15)) return false;
        int64_t k = (int64_t)g;
        if (m.periodic[ax]) {
            k = posmod(k, m.n[ax]);
        } else if (k < 0 || k >= m.n[ax]) {
            if (k == m.n[ax] && x == m.hi[ax])
                k = m.n[ax] - 1;
            else
                return false;
        }
        lin += k * stride;
        stride *= m.n[ax];
        v[ax] = (double)((const R*)a.p.v[ax])[p];
        ug[ax] = (double)((const R*)a.p.ug[ax])[p];
        if (!isfinite(v[ax]) || !isfinite(ug[ax])) return false;
    }
    double r = (double)((const R*)a.p.r)[p];
    if (!isfinite(r)) return false;
    droplet_phi<D>(r, v, ug, a.ph, phi);
#pragma unroll
    for (int k = 0; k < D + 1; ++k)
        if (!isfinite(phi[k])) return false;
    cell = lin;
    return true;
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_psi_bound(PsiArgs a)
{
    constexpr int C = D + 1;
    double mx[C];
#pragma unroll
    for (int k = 0; k < C; ++k) mx[k] = 0.0;
    unsigned long long outside = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.p.count; p += stride) {
        int64_t c;
        double phi[4];
        if (psi_particle<R, D>(a, p, c, phi)) {
#pragma unroll
            for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], fabs(phi[k]));
        } else {
            ++outside;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        outside += __shfl_xor(outside, o, kWave);
#pragma unroll
        for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], __shfl_xor(mx[k], o, kWave));
    }
    if ((threadIdx.x % kWave) == 0) {
        if (outside) atomicAdd(&a.stats[ST_OUTSIDE], outside);
#pragma unroll
        for (int k = 0; k < C; ++k)
            if (mx[k] > 0.0) atomicMax(&a.maxbits[k], (unsigned long long)__double_as_longlong(mx[k]));
    }
}

template <int D>
__global__ void k_psi_scale(PsiArgs a)
{
    constexpr int C = D + 1;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double n = (double)(a.p.count > 0 ? a.p.count : 1);
    for (int k = 0; k < C; ++k) {
        double mx = __longlong_as_double((long long)a.maxbits[k]);
        int e = 0;
        if (mx > 0.0) {
            int ex;
            frexp(mx * n, &ex);          // mx * n < 2^ex
            e = 62 - ex;
            if (e > 1000) e = 1000;
        }
        a.qscale[k] = ldexp(1.0, e);
    }
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_psi_accum(PsiArgs a)
{
    constexpr int C = D + 1;
    const int64_t M = a.m.M;
    double qs[C];
#pragma unroll
    for (int k = 0; k < C; ++k) qs[k] = a.qscale[k];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.p.count; p += stride) {
        int64_t c;
        double phi[4];
        if (!psi_particle<R, D>(a, p, c, phi)) continue;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            long long qv = llrint(phi[k] * qs[k]);
            atomicAdd(&a.acc[(int64_t)k * M + c], (unsigned long long)qv);
        }
        atomicAdd(&a.counts[c], 1u);
    }
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_psi_finalize(PsiArgs a)
{
    constexpr int C = D + 1;
    const int64_t M = a.m.M;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    double cs = a.cell_scale ? (double)((const R*)a.cell_scale)[c] : 1.0;
    double f = -(a.weight / a.m.vol) * cs;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        double sum = (double)(long long)a.acc[(int64_t)k * M + c] / a.qscale[k];
        ((R*)a.out[k])[c] = (R)(f * sum);
    }
    if (a.den) ((R*)a.den)[c] = (R)a.counts[c];
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(unsigned int* p, int64_t n, unsigned int v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
template <typename R>
__global__ void k_fill_real(R* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (R)0;
}

static unsigned grid_for(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_fill_real(R* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_real<R>), dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
template hipError_t launch_fill_real<float>(float*, int64_t, hipStream_t);
template hipError_t launch_fill_real<double>(double*, int64_t, hipStream_t);

template <typename R, int D>
hipError_t launch_psicell(const PsiArgs& a, hipStream_t s)
{
    constexpr int C = D + 1;
    hipError_t e = launch_fill_u64(a.acc, (int64_t)C * a.m.M, 0ull, s);
    if (e == hipSuccess) e = launch_fill_u32(a.counts, a.m.M, 0u, s);
    if (e == hipSuccess) e = launch_fill_u64(a.maxbits, C, 0ull, s);
    if (e != hipSuccess) return e;
    // enough waves to stream HBM: 8 blocks of 256 per CU
    unsigned g = grid_for(a.p.count);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL((k_psi_bound<R, D>), dim3(g), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_psi_scale<D>), dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL((k_psi_accum<R, D>), dim3(g), dim3(256), 0, s, a);
    unsigned gm = (unsigned)((a.m.M + 255) / 256);
    hipLaunchKernelGGL((k_psi_finalize<R, D>), dim3(gm), dim3(256), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_psicell<float, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<float, 3>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<double, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<double, 3>(const PsiArgs&, hipStream_t);

}  // namespace flp
