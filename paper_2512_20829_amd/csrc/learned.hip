// Learned bandwidth correction: features, the 5-64-64-1 network on bf16
// MFMA, the gradient of a loss through the estimator with respect to the
// smoothing lengths, the network backward, Adam and the relative-L2 loss.
//
// The correction multiplies h_i = h0 |det J_i| (eq. smoothing-length) by
// g_i = exp(s_max tanh o_i), s_max = ln 4, where o_i is the network output
// for the features
//   f = [log s1, log s2, log s3, log(n/n0) = -log|det J|, log(1 + N_nbr)]
// (s_k the singular values of J, largest first; N_nbr the valid trajectories
// with home cell in the 3^d block around the trajectory's home cell).
// Inputs z = (f - mu)/sd and the first hidden layer are rounded to bf16 for
// the MFMA (v_mfma_f32_16x16x16_bf16, fp32 accumulation); weights are the
// fp32 master copy rounded to bf16 when staged in LDS.
//
// MFMA fragment layout used throughout (16x16x16, wave64):
//   A (16x16, row m, col k):  lane l holds A[l % 16][4 (l / 16) + j], j < 4
//   B (16x16, row k, col n):  lane l holds B[4 (l / 16) + j][l % 16]
//   D (16x16):                lane l holds D[4 (l / 16) + j][l % 16]
// Trajectories are the N dimension, so a layer's D fragment for a 16-row
// block of hidden units is the next layer's B fragment for that K block.
#include "internal.hpp"
#include "kernels.hpp"
#include "learned.hpp"

namespace flp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (unsigned short)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_val(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float round_bf16(float f) { return bf16_val(bf16_bits(f)); }

// Logistic function from the hardware base-2 exponential and reciprocal
// (each within about one binary32 ulp; the activations are rounded to bf16
// for the next layer, 2^-8 relative, so the difference from the correctly
// rounded form is immaterial).
__device__ inline float sigmoid_f(float a)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a * -1.44269504088896340736f));
}
__device__ inline float silu_f(float a) { return a * sigmoid_f(a); }
__device__ inline float dsilu_f(float a)
{
    const float s = sigmoid_f(a);
    return s * (1.0f + a * (1.0f - s));
}

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline bf16x4 load4(const unsigned short* p)
{
    bf16x4 v;
    v.x = (short)p[0];
    v.y = (short)p[1];
    v.z = (short)p[2];
    v.w = (short)p[3];
    return v;
}
__device__ inline bf16x4 load4s(const unsigned short* p, int stride)
{
    bf16x4 v;
    v.x = (short)p[0];
    v.y = (short)p[stride];
    v.z = (short)p[2 * stride];
    v.w = (short)p[3 * stride];
    return v;
}

// Validity and binary64 terms shared with the prepass (same checks, factor 1).
template <typename R, int D>
__device__ inline bool load_terms(const TrajDev& t, int64_t i, double* x, double* J, double& det)
{
    const int64_t N = t.count;
    // every input is read, then tested with non-short-circuit ands, so that
    // the loads issue together instead of one test's branch at a time
    double v[3], ug[3];
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
    det = det_rn<D>(J);
    int fin = isfinite(r);
    fin &= isfinite(n0);
    fin &= isfinite(det);
    fin &= det != 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        fin &= isfinite(x[a]);
        fin &= isfinite(v[a]);
        fin &= isfinite(ug[a]);
    }
#pragma unroll
    for (int e = 0; e < D * D; ++e) fin &= isfinite(J[e]);
    return fin != 0;
}

// Singular values of J (largest first) from the eigenvalues of J^T J: the
// closed form for a symmetric 3x3 matrix, O. K. Smith, "Eigenvalues of a
// symmetric 3 x 3 matrix", Communications of the ACM 4(4), 168 (1961): with
// q = tr(A)/3 and p^2 = (|A - qI|_F^2)/6, the eigenvalues are
// q + 2p cos(phi + 2 pi k/3), phi = acos(det((A - qI)/p)/2)/3 (the
// trigonometric solution of the characteristic cubic).  The middle one
// comes from the trace and the smallest singular value from
// |det J| / (s1 s2), both free of the cubic's cancellation.
template <int D>
__device__ inline void singular_values(const double* J, double adet, double* s)
{
    if (D == 2) {
        double a = J[0] * J[0] + J[2] * J[2];
        double b = J[0] * J[1] + J[2] * J[3];
        double c = J[1] * J[1] + J[3] * J[3];
        double tr = a + c, df = a - c;
        double l1 = 0.5 * (tr + sqrt(df * df + 4.0 * b * b));
        s[0] = sqrt(l1);
        s[1] = adet / s[0];
        s[2] = 1.0;
        return;
    }
    double A[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) A[p][q] = J[0 * 3 + p] * J[0 * 3 + q] + J[1 * 3 + p] * J[1 * 3 + q] + J[2 * 3 + p] * J[2 * 3 + q];
    double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double qm = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    double l1, l2;
    if (p1 == 0.0) {
        double d0 = A[0][0], d1 = A[1][1], d2 = A[2][2];
        double hi = fmax(d0, fmax(d1, d2)), lo = fmin(d0, fmin(d1, d2));
        l1 = hi;
        l2 = d0 + d1 + d2 - hi - lo;
    } else {
        double p2 = (A[0][0] - qm) * (A[0][0] - qm) + (A[1][1] - qm) * (A[1][1] - qm) + (A[2][2] - qm) * (A[2][2] - qm) + 2.0 * p1;
        double p = sqrt(p2 / 6.0);
        const double ip = 1.0 / p;
        double B[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) B[a][b] = (A[a][b] - (a == b ? qm : 0.0)) * ip;
        double r = 0.5 * (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                          B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]));
        r = fmin(1.0, fmax(-1.0, r));
        double phi = acos(r) / 3.0;
        l1 = qm + 2.0 * p * cos(phi);
        double l3 = qm + 2.0 * p * cos(phi + 2.0943951023931954923);
        l2 = 3.0 * qm - l1 - l3;
    }
    s[0] = sqrt(fmax(l1, 0.0));
    s[1] = sqrt(fmax(l2, 0.0));
    s[2] = adet / (s[0] * s[1]);
}

// ---------------------------------------------------------------- counts and features
// One trajectory per thread (2 and 4 per thread, blockDim apart with all
// loads issued first, were slower).  The pass counts the valid trajectories
// (the prepass's validity) per home cell with integer atomics and, from the
// J it has loaded, forms the four features that do not need the counts: the
// binary64 singular values and det J, standardised and rounded to bf16 as
// the oracle forms them.  Its 16-byte record per trajectory is
// {z0 z1, z2 z3, home cell, valid << 16}, with zeros and kNoHome for an
// invalid trajectory; the network kernel replaces the home cell by z4, the
// standardised log(1 + neighbour count), once the counts are box-summed.
constexpr uint32_t kNoHome = 0xFFFFFFFFu;
template <typename R, int D>
__global__ __launch_bounds__(256) void k_home_count(TrajDev t, MeshDev m, const float* __restrict__ theta,
                                                    unsigned int* __restrict__ cnt, uint4* __restrict__ zb,
                                                    float* __restrict__ zout, float* __restrict__ fraw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = t.count;
    if (i >= N) return;
    double x[3], J[9], det;
    const bool ok = load_terms<R, D>(t, i, x, J, det);
    uint4 rec = make_uint4(0u, 0u, kNoHome, 0u);
    float f[4] = {0, 0, 0, 0};
    if (ok) {
        int64_t c = 0, st = 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            c += home_index(m, a, x[a]) * st;
            st *= m.n[a];
        }
        atomicAdd(&cnt[c], 1u);
        const double adet = fabs(det);
        double s[3];
        singular_values<D>(J, adet, s);
        // binary64 features and standardisation: z is rounded to bf16 for the
        // network, so it is formed as exactly as the oracle forms it
        const double fd[4] = {log(s[0]), log(s[1]), D == 3 ? log(s[2]) : 0.0, -log(adet)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (fraw) fraw[(int64_t)k * N + i] = (float)fd[k];
            f[k] = (float)((fd[k] - (double)theta[kOffMu + k]) / (double)theta[kOffSd + k]);
        }
        rec = make_uint4(bf16_bits(f[0]) | ((uint32_t)bf16_bits(f[1]) << 16),
                         bf16_bits(f[2]) | ((uint32_t)bf16_bits(f[3]) << 16), (uint32_t)c, 1u << 16);
    } else if (fraw) {
#pragma unroll
        for (int k = 0; k < 4; ++k) fraw[(int64_t)k * N + i] = __builtin_nanf("");
    }
    zb[i] = rec;
    if (zout)
#pragma unroll
        for (int k = 0; k < 4; ++k) zout[(int64_t)k * N + i] = ok ? round_bf16(f[k]) : 0.0f;
}

// One axis of the 3^D box sum of the per-cell counts: out[c] = in[c - s] +
// in[c] + in[c + s] along axis a (stride s), wrapping on a periodic axis
// (on an axis of one or two cells a neighbour can be the cell itself or the
// same cell twice, as for the neighbours of a home cell) and leaving out
// cells beyond a closed one.  After one pass per axis, each cell holds the
// count over the 3^D block around it; the integer sums are exact, so the
// order of the passes does not matter.
__global__ __launch_bounds__(256) void k_box_axis(MeshDev m, int a, const unsigned int* __restrict__ in,
                                                  unsigned int* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.M) return;
    int64_t st = 1;
    for (int b = 0; b < a; ++b) st *= m.n[b];
    const int64_t n = m.n[a];
    const int64_t i = (c / st) % n;
    unsigned int v = in[c];
    if (i > 0)
        v += in[c - st];
    else if (m.periodic[a])
        v += in[c + (n - 1) * st];
    if (i < n - 1)
        v += in[c + st];
    else if (m.periodic[a])
        v += in[c - (n - 1) * st];
    out[c] = v;
}

// ---------------------------------------------------------------- features + network
// LDS row strides (bf16 elements) of the staged weights and of the network's
// activation tiles: rows padded by 4 (W1, Z) and 4 (W2, H1) elements so that
// the 16 rows an MFMA fragment reads start in different bank pairs (a
// 16 x 64 bf16 tile with 128-byte rows puts all 16 rows in the same banks).
constexpr int kW1S = 20;
constexpr int kW2S = 68;
struct MlpW {
    unsigned short W1[kHidden][kW1S];    // bf16, inputs padded to 16 (columns 16.. unused)
    unsigned short W2[kHidden][kW2S];    // columns 64.. unused
    float b1[kHidden], b2[kHidden], w3[kHidden];   // w3 rounded to bf16
    float b3, mu[kFeat], sd[kFeat];
};

__device__ inline void stage_weights(const float* th, MlpW& W)
{
    for (int e = threadIdx.x; e < kHidden * 16; e += blockDim.x) {
        int o = e / 16, k = e % 16;
        W.W1[o][k] = k < kFeat ? bf16_bits(th[kOffW1 + o * kFeat + k]) : (unsigned short)0;
    }
    for (int e = threadIdx.x; e < kHidden * kHidden; e += blockDim.x) W.W2[e / kHidden][e % kHidden] = bf16_bits(th[kOffW2 + e]);
    for (int e = threadIdx.x; e < kHidden; e += blockDim.x) {
        W.b1[e] = th[kOffB1 + e];
        W.b2[e] = th[kOffB2 + e];
        W.w3[e] = round_bf16(th[kOffW3 + e]);
    }
    if (threadIdx.x == 0) {
        W.b3 = th[kOffB3];
        for (int k = 0; k < kFeat; ++k) {
            W.mu[k] = th[kOffMu + k];
            W.sd[k] = th[kOffSd + k];
        }
    }
}

constexpr int kMlpWaves = 4;

// The 5-64-64-1 network on bf16 MFMA, held to 128 registers for four waves
// per SIMD (the binary32 activations bound it; 136 -> 125 us at 2M with a
// few bytes of spill).  One wave takes 64 feature records
// per step (one per lane, into LDS), completing each with its fifth input,
// log(1 + N_nbr) from one read of the box-summed counts at the home cell;
// then four 16-trajectory groups go through the layers.  The output o gives
// the factor exp(s_max tanh o), 1 for an invalid trajectory.
__global__ __launch_bounds__(kWave * kMlpWaves, 4) void k_mlp(const float* __restrict__ theta, int64_t N,
                                                            const uint4* __restrict__ zb,
                                                            const unsigned int* __restrict__ box,
                                                            float* __restrict__ hfac, float* __restrict__ oout,
                                                            float* __restrict__ zout, float* __restrict__ fraw)
{
    __shared__ MlpW W;
    __shared__ __align__(16) unsigned short Z[kMlpWaves][kWave][kW1S];   // [traj][feature]
    __shared__ __align__(16) unsigned short H1[kMlpWaves][16][kW2S];      // [traj][hidden]
    __shared__ int vld[kMlpWaves][kWave];
    stage_weights(theta, W);
    __syncthreads();
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int r16 = lane % 16, g4 = lane / 16;
    // the biases (each layer's accumulator starts from them) and output
    // weights of the lane's hidden rows 16 mt + 4 g4 + j
    float b1r[4][4], b2r[4][4], w3r[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int hrow = 16 * mt + 4 * g4 + j;
            b1r[mt][j] = W.b1[hrow];
            b2r[mt][j] = W.b2[hrow];
            w3r[mt][j] = W.w3[hrow];
        }
    // the record and box count of the wave's next step are loaded one step
    // ahead (the count read depends on the record)
    const int64_t stride = (int64_t)gridDim.x * kMlpWaves * kWave;
    int64_t base = ((int64_t)blockIdx.x * kMlpWaves + wave) * kWave;
    uint4 q4 = base + lane < N ? zb[base + lane] : make_uint4(0u, 0u, kNoHome, 0u);
    unsigned int nbox = (q4.w >> 16) != 0u ? box[q4.z] : 0u;
    for (; base < N; base += stride) {
        const int64_t i = base + lane;
        const bool valid = (q4.w >> 16) != 0u;
        const int64_t inext = i + stride;
        const uint4 q4n = inext < N ? zb[inext] : make_uint4(0u, 0u, kNoHome, 0u);
        // the fifth input from the box-summed count at the home cell, in
        // binary64 as the oracle forms it
        uint32_t z4 = 0u;
        if (valid) {
            const double fd = log1p((double)nbox);
            const float f = (float)((fd - (double)W.mu[4]) / (double)W.sd[4]);
            z4 = bf16_bits(f);
            if (fraw) fraw[4 * N + i] = (float)fd;
            if (zout) zout[4 * N + i] = bf16_val((unsigned short)z4);
        } else if (i < N) {
            if (fraw) fraw[4 * N + i] = __builtin_nanf("");
            if (zout) zout[4 * N + i] = 0.0f;
        }
        // features 0..4 then zeros up to 16 (the MFMA's k padding), 8-byte stores
        uint2* zrow = reinterpret_cast<uint2*>(&Z[wave][lane][0]);
        zrow[0] = make_uint2(q4.x, q4.y);
        zrow[1] = make_uint2(z4, 0u);
        zrow[2] = make_uint2(0u, 0u);
        zrow[3] = make_uint2(0u, 0u);
        vld[wave][lane] = valid;
        wave_sync();
        for (int q = 0; q < 4; ++q) {
            // layer 1: a1^T[64 x 16] = W1[64 x 16] * Z^T[16 x 16]
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 acc = {b1r[mt][0], b1r[mt][1], b1r[mt][2], b1r[mt][3]};
                acc = mfma16(load4(&W.W1[16 * mt + r16][4 * g4]), load4(&Z[wave][16 * q + r16][4 * g4]), acc);
                uint32_t hb[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) hb[j] = bf16_bits(silu_f(acc[j]));
                // hidden rows 16 mt + 4 g4 .. + 3 of trajectory r16: one 8-byte store
                *reinterpret_cast<uint2*>(&H1[wave][r16][16 * mt + 4 * g4]) =
                    make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
            }
            wave_sync();
            if (q == 0) nbox = (q4n.w >> 16) != 0u ? box[q4n.z] : 0u;
            // layer 2 and the output dot product
            float op = 0.0f;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4 acc = {b2r[mt][0], b2r[mt][1], b2r[mt][2], b2r[mt][3]};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    acc = mfma16(load4(&W.W2[16 * mt + r16][16 * kb + 4 * g4]), load4(&H1[wave][r16][16 * kb + 4 * g4]), acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) op += w3r[mt][j] * silu_f(acc[j]);
            }
            op += __shfl_xor(op, 16, kWave);
            op += __shfl_xor(op, 32, kWave);
            const int64_t ti = base + 16 * q + r16;
            if (g4 == 0 && ti < N) {
                float o = op + W.b3;
                bool v = vld[wave][16 * q + r16] != 0;
                hfac[ti] = v ? expf(kSmax * tanhf(o)) : 1.0f;
                if (oout) oout[ti] = v ? o : 0.0f;
            }
            wave_sync();
        }
        q4 = q4n;
    }
}

// ---------------------------------------------------------------- feature standardisation
// Moments of the raw features over the valid trajectories (finite features;
// skipped trajectories carry NaN), in a fixed order: thread j of block b
// takes trajectories b * 256 + j + k * (grid * 256), the block adds its
// threads in a fixed tree, and k_feat_accum adds the blocks in block order.
// pass 0: [count, sum f_k]; pass 1: [count, sum (f_k - mean_k)^2] with the
// mean from the finished pass-0 sums.
constexpr int kMomBlocks = 1024;
constexpr int kMomW = 1 + kFeat;

__global__ __launch_bounds__(256) void k_feat_moments(const float* __restrict__ fraw, int64_t N, int pass,
                                                      const double* __restrict__ acc0, double* __restrict__ part)
{
    __shared__ double red[kMomW][256];
    double mean[kFeat];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) mean[k] = (pass == 1 && acc0[0] > 0.0) ? acc0[1 + k] / acc0[0] : 0.0;
    double v[kMomW] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const float f0 = fraw[i];
        if (!isfinite(f0)) continue;
        v[0] += 1.0;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) {
            const double d = (double)fraw[(int64_t)k * N + i] - mean[k];
            v[1 + k] += pass == 0 ? d : d * d;
        }
    }
#pragma unroll
    for (int k = 0; k < kMomW; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kMomW; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kMomW) part[(int64_t)blockIdx.x * kMomW + threadIdx.x] = red[threadIdx.x][0];
}

// a + p[0] + p[stride] + ... + p[(n - 1) stride], added in that order; each
// round issues its 16 loads before the first add so that they are in flight
// together
__device__ inline double ordered_column_sum(double a, const double* __restrict__ p, int n, int stride)
{
    constexpr int kRound = 16;
    int i = 0;
    for (; i + kRound <= n; i += kRound) {
        double v[kRound];
#pragma unroll
        for (int k = 0; k < kRound; ++k) v[k] = p[(int64_t)(i + k) * stride];
#pragma unroll
        for (int k = 0; k < kRound; ++k) a += v[k];
    }
    for (; i < n; ++i) a += p[(int64_t)i * stride];
    return a;
}

__global__ void k_feat_accum(const double* __restrict__ part, int nblk, double* __restrict__ acc)
{
    if (threadIdx.x >= kMomW) return;
    acc[threadIdx.x] = ordered_column_sum(acc[threadIdx.x], part + threadIdx.x, nblk, kMomW);
}

// mu = mean, sd = sample standard deviation (Bessel-corrected) + 1e-3
__global__ void k_feat_finish(const double* __restrict__ acc0, const double* __restrict__ acc1, float* theta)
{
    const int k = threadIdx.x;
    if (k >= kFeat) return;
    const double n = acc0[0];
    const double mean = n > 0.0 ? acc0[1 + k] / n : 0.0;
    const double var = n > 1.0 ? acc1[1 + k] / (n - 1.0) : 0.0;
    theta[kOffMu + k] = (float)mean;
    theta[kOffSd + k] = (float)(sqrt(var) + 1e-3);
}

hipError_t launch_feat_moments(const float* fraw, int64_t N, int pass, const double* acc0, double* part, double* acc,
                               hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    int nb = (int)((N + 255) / 256);
    if (nb > kMomBlocks) nb = kMomBlocks;
    FLA_LAUNCH(k_feat_moments, dim3(nb), dim3(256), 0, s, fraw, N, pass, acc0, part);
    FLA_LAUNCH(k_feat_accum, dim3(1), dim3(64), 0, s, part, nb, acc);
    return hipGetLastError();
}

hipError_t launch_feat_finish(const double* acc0, const double* acc1, float* theta, hipStream_t s)
{
    FLA_LAUNCH(k_feat_finish, dim3(1), dim3(64), 0, s, acc0, acc1, theta);
    return hipGetLastError();
}

// ---------------------------------------------------------------- estimator backward
// Per cell: a = -scale cs / D (0 where D = 0), b_k = a g_k, e = a sum_k g_k N_k / D.
// b is stored cell-major, four floats per cell (unused channels zero), so
// that the trajectory pass reads it with one 16-byte load per pair.
template <typename R>
__global__ void k_cell_grad(int C, int64_t M, Planes S, const void* den, Planes dLdS, double scale,
                            const void* cell_scale, float4* b, float* e)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    double cs = cell_scale ? (double)((const R*)cell_scale)[c] : 1.0;
    double d = (double)((const R*)den)[c];
    double f = -scale * cs;
    double a = (d > 0.0) ? f / d : 0.0;
    double ee = 0.0;
    float bk[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = 0; k < C; ++k) {
        double g = (double)((const R*)dLdS.p[k])[c];
        double shat = (d > 0.0 && f != 0.0) ? (double)((const R*)S.p[k])[c] / f : 0.0;
        bk[k] = (float)(a * g);
        ee += g * shat;
    }
    b[c] = make_float4(bk[0], bk[1], bk[2], bk[3]);
    e[c] = (float)(a * ee);
}

// dL/dlog h_i = h_i dL/dh_i = sum over the included cells of
//   K_ci (s_ci - 1) (sum_k b_kc q_ik - e_c),   K = (1/h) prod_a exp(-s_a/2),
// one wave per trajectory over its support box (same per-axis factors and
// inclusion test as the gather), reduced with a fixed butterfly.
constexpr int kBTab = 128;
template <typename R, int D>
__global__ __launch_bounds__(64) void k_traj_backward(MeshDev m, double cutoff, const uint32_t* keys, uint32_t sentinel,
                                                      const double4* rpos, const R* rw, const float4* b, const float* e,
                                                      float* out, int64_t N)
{
    constexpr int C = D + 1;
    __shared__ R S[3][kBTab];
    __shared__ R E[3][kBTab];
    __shared__ int64_t IX[3][kBTab];   // wrapped cell index times the axis stride
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    if (keys[i] == sentinel) {
        if (lane == 0) out[i] = 0.0f;
        return;
    }
    const double4 P = rpos[i];
    const double x[3] = {P.x, P.y, P.z};
    const double inv_h = P.w;
    const double rc = cutoff / inv_h * (1.0 + kSupportMargin);
    R c2;
    {
        R c = (R)cutoff;
        c2 = c * c;
    }
    float q[C];
    {
        const R* w = rw + (size_t)i * kRecW;
        for (int k = 0; k < C; ++k) q[k] = (float)((double)w[1 + k] / inv_h);
    }
    int64_t lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    for (int a = 0; a < D; ++a) {
        double flo = (x[a] - rc - m.lo[a]) / m.w[a] - 0.5 - 1e-9;
        double fhi = (x[a] + rc - m.lo[a]) / m.w[a] - 0.5 + 1e-9;
        flo = fmin(fmax(flo, -4.0e15), 4.0e15);
        fhi = fmin(fmax(fhi, -4.0e15), 4.0e15);
        int64_t ilo = (int64_t)ceil(flo), ihi = (int64_t)floor(fhi);
        if (m.periodic[a]) {
            if (ihi - ilo + 1 >= m.n[a]) {
                ilo = 0;
                ihi = m.n[a] - 1;
            }
        } else {
            ilo = ilo < 0 ? 0 : ilo;
            ihi = ihi >= m.n[a] ? m.n[a] - 1 : ihi;
        }
        lo[a] = ilo;
        cnt[a] = ihi - ilo + 1 < 0 ? 0 : ihi - ilo + 1;
    }
    double acc = 0.0;
    for (int64_t bz = 0; bz < cnt[2]; bz += kBTab)
    for (int64_t by = 0; by < cnt[1]; by += kBTab)
    for (int64_t bx = 0; bx < cnt[0]; bx += kBTab) {
        int64_t b0[3] = {bx, by, bz};
        int len[3];
        for (int a = 0; a < 3; ++a) {
            int64_t l = cnt[a] - b0[a];
            len[a] = (int)(l < kBTab ? l : kBTab);
        }
        __syncthreads();
        int64_t stride = 1;
        for (int a = 0; a < D; ++a) {
            for (int j = lane; j < len[a]; j += kWave) {
                int64_t ci = lo[a] + b0[a] + j;
                if (m.periodic[a]) ci = posmod(ci, m.n[a]);
                axis_factor<R>(m, a, ci, x[a], inv_h, S[a][j], E[a][j]);
                IX[a][j] = ci * stride;
            }
            stride *= m.n[a];
        }
        if (D == 2 && lane == 0) {
            S[2][0] = 0;
            E[2][0] = 1;
            IX[2][0] = 0;
        }
        __syncthreads();
        // at most kBTab^3 = 2^21 cells per block: 32-bit index arithmetic, the
        // quotients by the row lengths from a binary32 reciprocal (within
        // one of the true quotient for j < 2^21, then corrected)
        const int tot = len[0] * len[1] * (D == 3 ? len[2] : 1);
        const float r0 = 1.0f / (float)len[0], r1 = 1.0f / (float)len[1];
        auto divmod = [](int j, int l, float r, int& q, int& rem) {
            q = (int)((float)j * r);
            rem = j - q * l;
            if (rem < 0) {
                --q;
                rem += l;
            } else if (rem >= l) {
                ++q;
                rem -= l;
            }
        };
        for (int j = lane; j < tot; j += kWave) {
            int jx, r2, jy, jz;
            divmod(j, len[0], r0, r2, jx);
            divmod(r2, len[1], r1, jz, jy);
            R s = S[0][jx] + S[1][jy];
            if (D == 3) s = s + S[2][jz];
            if (!(s <= c2)) continue;
            const int64_t lin = IX[0][jx] + IX[1][jy] + IX[2][jz];
            const float4 bb = b[lin];
            const float bk[4] = {bb.x, bb.y, bb.z, bb.w};
            float G = -e[lin];
#pragma unroll
            for (int k = 0; k < C; ++k) G += bk[k] * q[k];
            double K = inv_h * (double)(E[0][jx] * E[1][jy] * (D == 3 ? E[2][jz] : (R)1));
            acc += K * ((double)s - 1.0) * (double)G;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) out[i] = (float)acc;
}

// ---------------------------------------------------------------- network backward
// Gradient of the loss with respect to W1 .. b3 given dL/dlog h_i: the chain
// dL/do = dL/dlog h * s_max (1 - tanh^2 o), then back through the layers.
// Deltas enter the MFMA as bf16 hi + lo pairs (two products each), so the
// weight gradients keep about 16 significant bits per term.  Each block
// writes one partial gradient; a second kernel adds the partials in block
// order.
constexpr int kBwdWaves = 4;
// Held to 256 registers (a few bytes of spill) so that, with the shared
// tiles below, two workgroups fit on a CU (one wave per SIMD took 1.7x as
// long at 2M).
template <int D>
__global__ __launch_bounds__(kWave * kBwdWaves, 2) void k_mlp_backward(const float* theta, int64_t N, const float* z,
                                                                    const float* o, const float* dlogh, float* partial)
{
    __shared__ MlpW W;
    __shared__ unsigned short W2T[kHidden][kW2S];         // W2 transposed, bf16 (padded rows)
    // the waves' tiles of the loop and, after it, the block's gradient sum
    // share one buffer (LDS for two workgroups per CU)
    struct Tiles {
        unsigned short Zs[kBwdWaves][16][kW1S];    // [traj][feature]
        unsigned short H1[kBwdWaves][16][kW2S];    // [traj][hidden]
        unsigned short D2h[kBwdWaves][kHidden][kW1S], D2l[kBwdWaves][kHidden][kW1S];   // [hidden][traj]
        unsigned short D1h[kBwdWaves][kHidden][kW1S], D1l[kBwdWaves][kHidden][kW1S];
        float dO[kBwdWaves][16];
    };
    union Shared {
        Tiles t;
        float gsum[kTrain];
    };
    __shared__ Shared U;
    auto& Zs = U.t.Zs;
    auto& H1 = U.t.H1;
    auto& D2h = U.t.D2h;
    auto& D2l = U.t.D2l;
    auto& D1h = U.t.D1h;
    auto& D1l = U.t.D1l;
    auto& dO = U.t.dO;
    float* gsum = U.gsum;
    stage_weights(theta, W);
    for (int e = threadIdx.x; e < kHidden * kHidden; e += blockDim.x)
        W2T[e % kHidden][e / kHidden] = bf16_bits(theta[kOffW2 + e]);
    __syncthreads();
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int r16 = lane % 16, g4 = lane / 16;
    f32x4 gW2[4][4], gW1[4];
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gW2[a][b] = f32x4{0, 0, 0, 0};
            gb1[a][b] = gb2[a][b] = gw3[a][b] = 0.0f;
        }
    }
    for (int64_t base = ((int64_t)blockIdx.x * kBwdWaves + wave) * 16; base < N;
         base += (int64_t)gridDim.x * kBwdWaves * 16) {
        const int64_t ti = base + r16;
        const bool in = ti < N;
        if (g4 == 0) {
            float dl = in ? dlogh[ti] : 0.0f;
            float oo = in ? o[ti] : 0.0f;
            float th = tanhf(oo);
            dO[wave][r16] = dl * kSmax * (1.0f - th * th);
        }
        if (lane < 16)
#pragma unroll
            for (int k = 0; k < 16; ++k)
                Zs[wave][lane][k] = (k < kFeat && in) ? bf16_bits(z[(int64_t)k * N + ti]) : (unsigned short)0;
        wave_sync();
        const float dob = dO[wave][r16];
        // forward recomputation
        float a1[4][4], a2[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0, 0, 0, 0};
            acc = mfma16(load4(&W.W1[16 * mt + r16][4 * g4]), load4(&Zs[wave][r16][4 * g4]), acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int hrow = 16 * mt + 4 * g4 + j;
                a1[mt][j] = acc[j] + W.b1[hrow];
                H1[wave][r16][hrow] = bf16_bits(silu_f(a1[mt][j]));
            }
        }
        wave_sync();
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                acc = mfma16(load4(&W.W2[16 * mt + r16][16 * kb + 4 * g4]), load4(&H1[wave][r16][16 * kb + 4 * g4]), acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int hrow = 16 * mt + 4 * g4 + j;
                a2[mt][j] = acc[j] + W.b2[hrow];
                float h2 = silu_f(a2[mt][j]);
                gw3[mt][j] += h2 * dob;
                float d2 = W.w3[hrow] * dob * dsilu_f(a2[mt][j]);
                gb2[mt][j] += d2;
                unsigned short hb = bf16_bits(d2);
                D2h[wave][hrow][r16] = hb;
                D2l[wave][hrow][r16] = bf16_bits(d2 - bf16_val(hb));
            }
        }
        gb3 += (g4 == 0) ? dob : 0.0f;
        wave_sync();
        // gW2[out][in] += sum_traj d2[out][traj] h1[in][traj]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            bf16x4 ah = load4(&D2h[wave][16 * mt + r16][4 * g4]);
            bf16x4 al = load4(&D2l[wave][16 * mt + r16][4 * g4]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                bf16x4 bb = load4s(&H1[wave][4 * g4][16 * nt + r16], kW2S);
                gW2[mt][nt] = mfma16(ah, bb, gW2[mt][nt]);
                gW2[mt][nt] = mfma16(al, bb, gW2[mt][nt]);
            }
        }
        // dh1[in][traj] = sum_out W2[out][in] d2[out][traj]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                bf16x4 aa = load4(&W2T[16 * mt + r16][16 * kb + 4 * g4]);
                acc = mfma16(aa, load4s(&D2h[wave][16 * kb + 4 * g4][r16], kW1S), acc);
                acc = mfma16(aa, load4s(&D2l[wave][16 * kb + 4 * g4][r16], kW1S), acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int hrow = 16 * mt + 4 * g4 + j;
                float d1 = acc[j] * dsilu_f(a1[mt][j]);
                gb1[mt][j] += d1;
                unsigned short hb = bf16_bits(d1);
                D1h[wave][hrow][r16] = hb;
                D1l[wave][hrow][r16] = bf16_bits(d1 - bf16_val(hb));
            }
        }
        wave_sync();
        // gW1[out][feat] += sum_traj d1[out][traj] z[feat][traj]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            bf16x4 bb = load4s(&Zs[wave][4 * g4][r16], kW1S);
            gW1[mt] = mfma16(load4(&D1h[wave][16 * mt + r16][4 * g4]), bb, gW1[mt]);
            gW1[mt] = mfma16(load4(&D1l[wave][16 * mt + r16][4 * g4]), bb, gW1[mt]);
        }
        wave_sync();
    }
    // per-lane bias partials: sum over the 16 lanes that share g4 (trajectories)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                gb1[mt][j] += __shfl_xor(gb1[mt][j], off, kWave);
                gb2[mt][j] += __shfl_xor(gb2[mt][j], off, kWave);
                gw3[mt][j] += __shfl_xor(gw3[mt][j], off, kWave);
            }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) gb3 += __shfl_xor(gb3, off, kWave);
    // waves add into the block sum one after the other (fixed order), once
    // every wave has left the loop's tiles
    __syncthreads();
    for (int e = threadIdx.x; e < kTrain; e += blockDim.x) gsum[e] = 0.0f;
    __syncthreads();
    for (int w = 0; w < kBwdWaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        gsum[kOffW2 + (16 * mt + 4 * g4 + j) * kHidden + 16 * nt + r16] += gW2[mt][nt][j];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (r16 < kFeat) gsum[kOffW1 + (16 * mt + 4 * g4 + j) * kFeat + r16] += gW1[mt][j];
                    if (r16 == 0) {
                        int hrow = 16 * mt + 4 * g4 + j;
                        gsum[kOffB1 + hrow] += gb1[mt][j];
                        gsum[kOffB2 + hrow] += gb2[mt][j];
                        gsum[kOffW3 + hrow] += gw3[mt][j];
                    }
                }
            }
            if (lane == 0) gsum[kOffB3] += gb3;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kTrain; e += blockDim.x) partial[(int64_t)blockIdx.x * kTrain + e] = gsum[e];
}

__global__ void k_grad_reduce(const float* partial, int nblocks, float* grad)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    double acc = 0.0;
    if (p < kTrain) {
        // the partials are added in block order; each round issues its 16
        // loads before the first add so that they are in flight together
        constexpr int kRound = 16;
        int b = 0;
        for (; b + kRound <= nblocks; b += kRound) {
            float v[kRound];
#pragma unroll
            for (int k = 0; k < kRound; ++k) v[k] = partial[(int64_t)(b + k) * kTrain + p];
#pragma unroll
            for (int k = 0; k < kRound; ++k) acc += (double)v[k];
        }
        for (; b < nblocks; ++b) acc += (double)partial[(int64_t)b * kTrain + p];
    }
    grad[p] = (float)acc;
}

// Moments and update in binary64 from the binary64 hyper-parameters (1 - b
// formed from b exactly as given), stored in binary32.
__global__ void k_adam(float* theta, float* mm, float* vv, const float* grad, double step, double lr, double b1,
                       double b2, double eps)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kTrain) return;
    const double g = (double)grad[p];
    const float m = (float)(b1 * (double)mm[p] + (1.0 - b1) * g);
    const float v = (float)(b2 * (double)vv[p] + (1.0 - b2) * (g * g));
    mm[p] = m;
    vv[p] = v;
    double mh = (double)m / (1.0 - pow(b1, step));
    double vh = (double)v / (1.0 - pow(b2, step));
    theta[p] = (float)((double)theta[p] - lr * mh / (sqrt(vh) + eps));
}

// ---------------------------------------------------------------- relative-L2 loss
constexpr int kLossBlocks = 256;
template <typename R>
__global__ __launch_bounds__(256) void k_loss_partial(int C, int64_t M, Planes S, Planes Rf, double* part)
{
    __shared__ double red[2 * 4][256 / kWave];
    double num[4] = {0, 0, 0, 0}, den[4] = {0, 0, 0, 0};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < M; c += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < C; ++k) {
            double s = (double)((const R*)S.p[k])[c], r = (double)((const R*)Rf.p[k])[c];
            num[k] += (s - r) * (s - r);
            den[k] += r * r;
        }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    for (int k = 0; k < 4; ++k) {
        double a = num[k], b = den[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o, kWave);
            b += __shfl_xor(b, o, kWave);
        }
        if (lane == 0) {
            red[2 * k][wave] = a;
            red[2 * k + 1][wave] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double a = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) a += red[threadIdx.x][w];
        part[(int64_t)blockIdx.x * 8 + threadIdx.x] = a;
    }
}

// out: the loss, then |S - R|^2 and |R|^2 of each channel; thread j adds
// column j of the block partials in block order
__global__ void k_loss_final(int C, const double* part, int nb, double* out)
{
    __shared__ double col[8];
    const int j = threadIdx.x;
    if (j < 2 * C) {
        col[j] = ordered_column_sum(0.0, part + j, nb, 8);
        out[1 + j] = col[j];
    }
    __syncthreads();
    if (j == 0) {
        double loss = 0.0;
        for (int k = 0; k < C; ++k) loss += col[2 * k + 1] > 0.0 ? col[2 * k] / col[2 * k + 1] : 0.0;
        out[0] = loss;
    }
}

template <typename R>
__global__ void k_loss_grad(int C, int64_t M, Planes S, Planes Rf, const double* res, MutPlanes G)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    for (int k = 0; k < C; ++k) {
        double nr = res[2 + 2 * k];
        double s = (double)((const R*)S.p[k])[c], r = (double)((const R*)Rf.p[k])[c];
        ((R*)G.p[k])[c] = (R)(nr > 0.0 ? 2.0 * (s - r) / nr : 0.0);
    }
}

// ---------------------------------------------------------------- launchers
template <typename R, int D>
hipError_t launch_bandwidth_forward(const TrajDev& t, const MeshDev& m, const float* theta, unsigned int* cnt, void* zb,
                                    float* hfac, float* z, float* o, float* fraw, hipStream_t s)
{
    hipError_t e = launch_fill_u32(cnt, m.M, 0u, s);
    if (e != hipSuccess || t.count == 0) return e;
    const unsigned g = (unsigned)((t.count + 255) / 256);
    FLA_LAUNCH((k_home_count<R, D>), dim3(g), dim3(256), 0, s, t, m, theta, cnt, (uint4*)zb, z, fraw);
    // box sums over the 3^D neighbourhoods, one pass per axis between the two
    // halves of cnt (2 M words)
    unsigned int* buf[2] = {cnt, cnt + m.M};
    const unsigned gm = (unsigned)((m.M + 255) / 256);
    for (int a = 0; a < D; ++a)
        FLA_LAUNCH(k_box_axis, dim3(gm), dim3(256), 0, s, m, a, (const unsigned int*)buf[a & 1], buf[(a + 1) & 1]);
    const unsigned int* box = buf[D & 1];
    int64_t groups = (t.count + kWave * kMlpWaves - 1) / (kWave * kMlpWaves);
    unsigned gb = (unsigned)(groups < 2048 ? groups : 2048);
    FLA_LAUNCH(k_mlp, dim3(gb), dim3(kWave * kMlpWaves), 0, s, theta, t.count, (const uint4*)zb, box, hfac, o, z,
               fraw);
    return hipGetLastError();
}

template <typename R, int D>
hipError_t launch_traj_backward(const MeshDev& m, double cutoff, const uint32_t* keys, uint32_t sentinel,
                                const double4* rpos, const R* rw, Planes S, const void* den, Planes dLdS,
                                double scale, const void* cell_scale, float* bcells, float* eplane, float* out,
                                int64_t N, hipStream_t s)
{
    unsigned g = (unsigned)((m.M + 255) / 256);
    float4* b4 = reinterpret_cast<float4*>(bcells);
    FLA_LAUNCH((k_cell_grad<R>), dim3(g), dim3(256), 0, s, D + 1, m.M, S, den, dLdS, scale, cell_scale, b4,
                       eplane);
    if (N > 0)
        FLA_LAUNCH((k_traj_backward<R, D>), dim3((unsigned)N), dim3(64), 0, s, m, cutoff, keys, sentinel, rpos, rw,
                           (const float4*)b4, eplane, out, N);
    return hipGetLastError();
}

int mlp_backward_blocks(int64_t N)
{
    int64_t b = (N + 16 * kBwdWaves * 8 - 1) / (16 * kBwdWaves * 8);
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

template <int D>
hipError_t launch_mlp_backward(const float* theta, int64_t N, const float* z, const float* o, const float* dlogh,
                               float* partial, int nblocks, float* grad, hipStream_t s)
{
    FLA_LAUNCH((k_mlp_backward<D>), dim3(nblocks), dim3(kWave * kBwdWaves), 0, s, theta, N, z, o, dlogh, partial);
    FLA_LAUNCH(k_grad_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, partial, nblocks, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int64_t step, double lr, double b1,
                       double b2, double eps, hipStream_t s)
{
    FLA_LAUNCH(k_adam, dim3((kTrain + 255) / 256), dim3(256), 0, s, theta, m, v, grad, (double)step, lr, b1, b2, eps);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_loss(int C, int64_t M, Planes S, Planes Rf, MutPlanes G, bool want_grad, double* part, double* res,
                       hipStream_t s)
{
    FLA_LAUNCH((k_loss_partial<R>), dim3(kLossBlocks), dim3(256), 0, s, C, M, S, Rf, part);
    FLA_LAUNCH(k_loss_final, dim3(1), dim3(64), 0, s, C, part, kLossBlocks, res);
    if (want_grad) {
        unsigned g = (unsigned)((M + 255) / 256);
        FLA_LAUNCH((k_loss_grad<R>), dim3(g), dim3(256), 0, s, C, M, S, Rf, res, G);
    }
    return hipGetLastError();
}

#define FLP_LINST(R, D)                                                                                               \
    template hipError_t launch_bandwidth_forward<R, D>(const TrajDev&, const MeshDev&, const float*, unsigned int*, \
                                                       void*, float*, float*, float*, float*, hipStream_t);         \
    template hipError_t launch_traj_backward<R, D>(const MeshDev&, double, const uint32_t*, uint32_t,              \
                                                   const double4*, const R*, Planes, const void*, Planes, double,   \
                                                   const void*, float*, float*, float*, int64_t, hipStream_t);
FLP_LINST(float, 2)
FLP_LINST(float, 3)
FLP_LINST(double, 2)
FLP_LINST(double, 3)
template hipError_t launch_mlp_backward<2>(const float*, int64_t, const float*, const float*, const float*, float*, int,
                                           float*, hipStream_t);
template hipError_t launch_mlp_backward<3>(const float*, int64_t, const float*, const float*, const float*, float*, int,
                                           float*, hipStream_t);
template hipError_t launch_loss<float>(int, int64_t, Planes, Planes, MutPlanes, bool, double*, double*, hipStream_t);
template hipError_t launch_loss<double>(int, int64_t, Planes, Planes, MutPlanes, bool, double*, double*, hipStream_t);

}  // namespace flp
