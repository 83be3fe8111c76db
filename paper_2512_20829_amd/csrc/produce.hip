// Trajectory producer: droplets advanced over one carrier time step in an
// analytic gas field, fused with the prepass so that the advanced position
// and Jacobian go straight from registers into the projection's records.
//
// Per droplet (eqs. Stokes-drag, evap-model and Jacobian-evolution in
// dimensional form, tau = 2 rho r^2/(9 mu)):
//   x' = v,  v' = (u(x) - v)/tau,  r' = delta/(2 r),
//   J' = K,  K' = (grad u(x) J - K)/tau,
// together with the droplet's contributions Q' = [mdot, F + mdot v]
// (F = m (u - v)/tau, mdot = 4 pi rho r^2 r'), integrated by the classical
// fourth-order Runge-Kutta method over `substeps` equal substeps: every
// substep's contributions are formed from the stage derivatives and summed
// over the step (App. B steps 1a-1b).  The step's source rates Q/dt enter the
// estimator in place of the instantaneous ones.  Binary64 throughout, one
// droplet per thread, contraction off, so that the operations are those of
// the written method.
#include "internal.hpp"
#include "kernels.hpp"
#include "prepass.hpp"

namespace flp {

// u(x) and grad u(x) (row a: du_a/dx_b) of the gas field.
template <int D>
__device__ inline void flow_eval(const FlowDev& f, const double* x, double* u, double* gu)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = f.u0[a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
            u[a] += f.G[a * 3 + b] * x[b];
            gu[a * D + b] = f.G[a * 3 + b];
        }
    }
    const double w = 2.0 * 3.14159265358979323846 * f.k, U = f.U;
    if (D == 2 && f.kind == FLA_FLOW_TAYLOR_GREEN) {
        double sx, cx, sy, cy;
        sincos(w * x[0], &sx, &cx);
        sincos(w * x[1], &sy, &cy);
        u[0] += U * sx * cy;
        u[1] -= U * cx * sy;
        gu[0] += U * w * cx * cy;
        gu[1] -= U * w * sx * sy;
        gu[2] += U * w * sx * sy;
        gu[3] -= U * w * cx * cy;
    } else if (D == 3 && f.kind == FLA_FLOW_ABC) {
        const double A = f.abc[0], B = f.abc[1], C = f.abc[2];
        double sx, cx, sy, cy, sz, cz;
        sincos(w * x[0] + f.phase[0], &sx, &cx);
        sincos(w * x[1] + f.phase[1], &sy, &cy);
        sincos(w * x[D - 1] + f.phase[2], &sz, &cz);
        u[0] += U * (A * sz + C * cy);
        u[1] += U * (B * sx + A * cz);
        u[D - 1] += U * (C * sy + B * cx);
        gu[0 * D + 1] -= U * C * w * sy;
        gu[0 * D + D - 1] += U * A * w * cz;
        gu[1 * D + 0] += U * B * w * cx;
        gu[1 * D + D - 1] -= U * A * w * sz;
        gu[(D - 1) * D + 0] -= U * B * w * sx;
        gu[(D - 1) * D + 1] += U * C * w * cy;
    }
}

// Time derivative of the state y = [x, v, r, J, K, Q].
template <int D>
__device__ inline void producer_rhs(const FlowDev& f, const PhysDev& ph, const double* y, double* dy)
{
#pragma clang fp contract(off)
    constexpr int OJ = 2 * D + 1, OK = OJ + D * D, OQ = OK + D * D;
    double u[3], gu[9];
    flow_eval<D>(f, y, u, gu);
    const double r = y[2 * D];
    const double rho = ph.rho_d;
    const double tau = 2.0 * rho * r * r / (9.0 * ph.mu);
    const double m = (4.0 / 3.0) * 3.14159265358979323846 * rho * r * r * r;
    const double rdot = ph.delta / (2.0 * r);
    const double mdot = 4.0 * 3.14159265358979323846 * rho * r * r * rdot;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dy[a] = y[D + a];
        dy[D + a] = (u[a] - y[D + a]) / tau;
    }
    dy[2 * D] = rdot;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            double gJ = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) gJ += gu[a * D + c] * y[OJ + c * D + b];
            dy[OJ + a * D + b] = y[OK + a * D + b];
            dy[OK + a * D + b] = (gJ - y[OK + a * D + b]) / tau;
        }
    dy[OQ] = mdot;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double F = m * (u[a] - y[D + a]) / tau;
        dy[OQ + 1 + a] = F + mdot * y[D + a];
    }
}

// Held to 256 registers so that two waves share a SIMD (the binary64 RK4
// chains are long; a few bytes of spill): 1.64 -> 1.35 ms for 2M droplets
// in 3-D; at 168 registers the spills made it twice as slow.
template <typename R, int D>
__global__ __launch_bounds__(256, 2) void k_produce(ProduceArgs p, MeshDev m, PhysDev ph, const float* hfac, int deposit,
                                                 uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, double* qd,
                                                 unsigned long long* stats)
{
#pragma clang fp contract(off)
    constexpr int C = D + 1, NY = 2 * D + 1 + 2 * D * D + C;
    constexpr int OJ = 2 * D + 1, OK = OJ + D * D, OQ = OK + D * D;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t sentinel = (uint32_t)kClasses * (uint32_t)m.ntiles;
    unsigned long long skipped = 0, nosup = 0;
    if (i < p.count) {
        const int64_t N = p.count;
        double y[NY];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            y[a] = p.x[a][i];
            y[D + a] = p.v[a][i];
        }
        y[2 * D] = p.r[i];
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            y[OJ + e] = p.J[(int64_t)e * N + i];
            y[OK + e] = p.dJ[(int64_t)e * N + i];
        }
#pragma unroll
        for (int k = 0; k < C; ++k) y[OQ + k] = 0.0;
        bool ok = true;
#pragma unroll
        for (int e = 0; e < NY; ++e) ok = ok && isfinite(y[e]);
        const double r0 = y[2 * D];
        ok = ok && r0 > 0.0 && r0 * r0 + ph.delta * p.dt > 0.0;
        const double h = p.dt / (double)p.substeps;
        if (ok) {
            double acc[NY], yt[NY], k[NY];
            for (int s = 0; s < p.substeps; ++s) {
                // k1
                producer_rhs<D>(p.flow, ph, y, k);
#pragma unroll
                for (int e = 0; e < NY; ++e) {
                    acc[e] = k[e];
                    yt[e] = y[e] + 0.5 * h * k[e];
                }
                // k2
                producer_rhs<D>(p.flow, ph, yt, k);
#pragma unroll
                for (int e = 0; e < NY; ++e) {
                    acc[e] = acc[e] + 2.0 * k[e];
                    yt[e] = y[e] + 0.5 * h * k[e];
                }
                // k3
                producer_rhs<D>(p.flow, ph, yt, k);
#pragma unroll
                for (int e = 0; e < NY; ++e) {
                    acc[e] = acc[e] + 2.0 * k[e];
                    yt[e] = y[e] + h * k[e];
                }
                // k4
                producer_rhs<D>(p.flow, ph, yt, k);
#pragma unroll
                for (int e = 0; e < NY; ++e) y[e] = y[e] + (h / 6.0) * (acc[e] + k[e]);
            }
#pragma unroll
            for (int e = 0; e < NY; ++e) ok = ok && isfinite(y[e]);
            ok = ok && y[2 * D] > 0.0;
        }
        double phi[4] = {0, 0, 0, 0};
        if (ok)
#pragma unroll
            for (int k = 0; k < C; ++k) phi[k] = y[OQ + k] / p.dt;
        if (ok && p.update) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                p.x[a][i] = y[a];
                p.v[a][i] = y[D + a];
            }
            p.r[i] = y[2 * D];
#pragma unroll
            for (int e = 0; e < D * D; ++e) {
                p.J[(int64_t)e * N + i] = y[OJ + e];
                p.dJ[(int64_t)e * N + i] = y[OK + e];
            }
        }
        if (p.phibar)
#pragma unroll
            for (int k = 0; k < C; ++k) p.phibar[(int64_t)k * N + i] = phi[k];
        double xe[3] = {y[0], y[1], D == 3 ? y[2] : 0.0};
        const double n0 = p.n0 ? p.n0[i] : p.n0_scalar;
        const double fac = hfac ? (double)hfac[i] : 1.0;
        prepass_emit<R, D>(m, ph, fac, deposit, N, i, i, 0u, sentinel, xe, y + OJ, n0, phi, ok, p.seed_volume, keys,
                           vals, rpos, rw, qd, skipped, nosup);
    }
    wave_count_sum(stats, ST_SKIPPED, (unsigned)skipped);
    wave_count_sum(stats, ST_NOSUPPORT, (unsigned)nosup);
}

template <typename R, int D>
hipError_t launch_produce(const ProduceArgs& p, const MeshDev& m, const PhysDev& ph, const float* hfac, int deposit,
                          uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, double* qd, unsigned long long* stats,
                          hipStream_t s)
{
    if (p.count <= 0) return hipSuccess;
    const unsigned g = (unsigned)((p.count + 255) / 256);
    FLA_LAUNCH((k_produce<R, D>), dim3(g), dim3(256), 0, s, p, m, ph, hfac, deposit, keys, vals, rpos, rw, qd,
                       stats);
    return hipGetLastError();
}

#define FLP_PINST(R, D)                                                                                          \
    template hipError_t launch_produce<R, D>(const ProduceArgs&, const MeshDev&, const PhysDev&, const float*, int, \
                                             uint32_t*, uint32_t*, double4*, R*, double*, unsigned long long*,     \
                                             hipStream_t);
FLP_PINST(float, 2)
FLP_PINST(float, 3)
FLP_PINST(double, 2)
FLP_PINST(double, 3)

}  // namespace flp
