// PSI-CELL box counting (eqs. vol-avg-discrete and coupling-terms-definition)
// and small fill kernels.
//
// The per-cell sums are made order-independent by exact integer arithmetic:
// each phi_k is quantised to a multiple of 2^-e_k, e_k chosen from the
// largest |phi_k| so that count * max|phi_k| * 2^e_k < 2^62 (no partial sum
// can overflow int64), and the integers are added.  The quantisation error of
// one particle is at most 2^-(e_k+1), which grows with the count; binary64
// records therefore carry a second integer word per channel: the remainder
// phi_k 2^e_k - rint(phi_k 2^e_k), in [-1/2, 1/2], quantised to 2^-f with
// f = 62 - ceil(log2(count + 1)) (so the remainder sums cannot overflow
// either).  A particle's error is then at most 2^-(e_k+f+1), below 2^-62
// max|phi_k| for any count under 2^31, and each cell's value is formed from
// the two exact sums.
//
// Particles arrive in arbitrary spatial order, so the sums are not formed by
// global atomics (one contended 64-bit atomic per particle and channel) but
// in streaming passes over coarse tiles of cells, grouped into bins of
// kPsiTilesPerBin consecutive tiles:
//   count   per particle, from its position only: the (tile, cell in tile)
//           code (-1 outside a closed box, counted as outside, or for a
//           non-finite position, counted as skipped);
//           per-block tile and bin histograms in LDS, written tile-major
//           and bin-major for exclusive scans that give every tile's bucket
//           and every (bin, block) output range;
//   scatter per particle with a code: phi, the per-channel max |phi|, and
//           the record (code, phi), sorted by bin in LDS round by round and
//           written out as one contiguous run per bin; a particle whose
//           velocities, radius or phi are not finite gets a record marked
//           skip and is counted as skipped;
//   tiles   per bin: its records sorted by tile in LDS round by round and
//           written to the tile buckets in contiguous runs;
//   reduce  one workgroup per tile: quantise and add in LDS (integer atomics),
//           then scale by -w/V_c and write the tile's cells.
// Storing each record straight into one of thousands of tile buckets would
// leave every 20-byte store on its own and the cache lines partly written;
// the two sorted partitions write whole runs instead.  A mesh that takes at
// most kPsiMaxBins tiles as large as one workgroup's LDS sums allow (4096
// cells for binary32 records, 2048 for binary64) is run direct: the bins are
// those tiles, the scatter's runs are the tile buckets, and the tile pass
// (one more write and read of every record) is not needed.  Every pass gives each
// thread several particles per step (kPsiUnroll, PsiRoundPerThread,
// kPsiUnrollReduce) and issues all their loads before any use, to keep
// enough reads in flight; the scatter forms the binary32 source terms of
// binary32 records in binary32.
#include "internal.hpp"
#include "kernels.hpp"

namespace flp {

constexpr int kPsiUnroll = 4;          // count
constexpr int kPsiUnrollReduce = 8;    // reduce
// particles (records) per thread in a round of the two partitions: a
// round's records take 120 KiB of LDS (one block per compute unit); the
// longer a round, the longer its run per bin, and the fewer partly written
// cache lines (with 512 direct tiles, rounds of 2048, 4096 and 6144
// binary32 records took the 200M-particle call to 6.72, 6.36 and 6.25 ms)
template <typename R> struct PsiRoundPerThread { static constexpr int value = sizeof(R) == 4 ? 24 : 12; };
// threads of a scatter block (a round is kPsiScatterThreads * U records)
constexpr int kPsiScatterThreads = 256;
constexpr uint32_t kPsiSkip = 0xFFFFFFFFu;     // cell of a skipped record in a tile bucket
constexpr uint32_t kPsiSkipBit = 0x80000000u;  // skip mark of a binned record (codes < 2^24)
static_assert(kPsiTilesPerBin == kWave, "the tile pass scans one tile per lane of one wave");

// Cell indices of a particle from its position alone: 1 if it has a cell,
// 0 for a position outside a closed box (x == hi goes to the last cell), -1
// for a non-finite position.
template <int D>
__device__ inline int psi_cell(const MeshDev& m, const double* x, int* idx)
{
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
        if (!isfinite(x[ax])) return -1;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        // floor((x - lo)/w): a multiply by 1/w differs from the rounded
        // quotient by a few ulps, which can change the floor only next to an
        // integer; there the quotient is formed exactly
        const double dx = x[ax] - m.lo[ax];
        double q = dx * (1.0 / m.w[ax]);
        if (fabs(q - rint(q)) < 1e-6 * (1.0 + fabs(q))) q = dx / m.w[ax];
        double g = floor(q);
        if (!(fabs(g) < 9.0e15)) return 0;
        int64_t k = (int64_t)g;
        if (m.periodic[ax]) {
            k = posmod(k, m.n[ax]);
        } else if (k < 0 || k >= m.n[ax]) {
            if (k == m.n[ax] && x[ax] == m.hi[ax])
                k = m.n[ax] - 1;
            else
                return 0;
        }
        idx[ax] = (int)k;
    }
    return 1;
}

// (tile, cell-in-tile) code of a valid particle: tile * cpt + cell in tile
// (tile edges and cpt are powers of two)
template <int D>
__device__ inline int psi_code(const PsiArgs& a, const int* idx)
{
    int tile = 0, loc = 0, ts = 1, lsh = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        tile += (idx[ax] >> a.ptlog[ax]) * ts;
        ts *= a.pnt[ax];
        loc += (idx[ax] & (a.pt[ax] - 1)) << lsh;
        lsh += a.ptlog[ax];
    }
    return (tile << a.cptlog) | loc;
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_psi_count(PsiArgs a)
{
    extern __shared__ unsigned int hist[];
    const int ntl = a.pntiles;
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int64_t N = a.p.count;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < N ? beg + chunk : N;
    const int64_t stepw = (int64_t)blockDim.x * kPsiUnroll;
    unsigned long long outside = 0, bad = 0;
    for (int64_t p0 = beg + threadIdx.x; p0 < end; p0 += stepw) {
        double x[kPsiUnroll][3];
#pragma unroll
        for (int u = 0; u < kPsiUnroll; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) x[u][ax] = p < end ? a.p.x[ax][p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPsiUnroll; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
            if (p >= end) break;
            int idx[3] = {0, 0, 0};
            int code = -1;
            const int where = psi_cell<D>(a.m, x[u], idx);
            if (where > 0) {
                code = psi_code<D>(a, idx);
                atomicAdd(&hist[code >> a.cptlog], 1u);
            } else if (where == 0) {
                ++outside;
            } else {
                ++bad;
            }
            a.codes[p] = code;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) a.blockhist[(int64_t)t * gridDim.x + blockIdx.x] = hist[t];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.blockhist[(int64_t)ntl * gridDim.x] = 0;
    // the same counts summed over the tiles of each bin (the tiles are read
    // in a rotated order so that the lanes hit different LDS banks); direct
    // runs use the tile counts themselves
    for (int c = threadIdx.x; c < (a.direct ? 0 : a.pnbins); c += blockDim.x) {
        const int t0 = c << kPsiTilesPerBinLog;
        unsigned int sum = 0;
        for (int j = 0; j < kPsiTilesPerBin; ++j) {
            const int t = t0 + ((j + c) & (kPsiTilesPerBin - 1));
            if (t < ntl) sum += hist[t];
        }
        a.binhist[(int64_t)c * gridDim.x + blockIdx.x] = sum;
    }
    if (!a.direct && blockIdx.x == 0 && threadIdx.x == 0) a.binhist[(int64_t)a.pnbins * gridDim.x] = 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        outside += __shfl_xor(outside, o, kWave);
        bad += __shfl_xor(bad, o, kWave);
    }
    if ((threadIdx.x % kWave) == 0 && outside) atomicAdd(&a.stats[ST_OUTSIDE], outside);
    if ((threadIdx.x % kWave) == 0 && bad) atomicAdd(&a.stats[ST_SKIPPED], bad);
}

// Exclusive prefix sum of one value per thread of an NT-thread block, and
// the block total.  ws holds NT / 64 words of LDS; the call contains a
// barrier.
template <int NT>
__device__ inline unsigned int block_exclusive_sum(unsigned int v, unsigned int* ws, unsigned int& total)
{
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    unsigned int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) ws[w] = inc;
    __syncthreads();
    unsigned int pre = 0;
    total = 0;
#pragma unroll
    for (int j = 0; j < NT / kWave; ++j) {
        const unsigned int t = ws[j];
        pre += j < w ? t : 0u;
        total += t;
    }
    return pre + inc - v;
}

// Exclusive prefix sum over the 64 lanes of one wave, and the wave total.
__device__ inline unsigned int wave_exclusive_sum(unsigned int v, unsigned int& total)
{
    const int lane = threadIdx.x % kWave;
    unsigned int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const unsigned int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    total = __shfl(inc, kWave - 1, kWave);
    return inc - v;
}

// First partition: each block takes its contiguous range of particles in
// rounds of 256 U, forms their records, orders a round's records by bin in
// LDS (counting sort) and writes them out bin by bin, so a round gives one
// contiguous run of records per bin and the stores are coalesced.  The
// slots come from the scanned per-block bin counts of the count pass (a
// block's share of a bin is one contiguous range, filled round by round).
template <typename R, int D>
__global__ __launch_bounds__(kPsiScatterThreads) void k_psi_scatter(PsiArgs a)
{
    constexpr int C = D + 1;
    constexpr int NT = kPsiScatterThreads;
    constexpr int U = PsiRoundPerThread<R>::value * 256 / NT;
    constexpr int RB = NT * U;
    constexpr int BPT = (kPsiMaxBins + NT - 1) / NT;   // bins per thread in the bin scan
    __shared__ PsiRec<R> stage[RB];
    // per bin: this round's count, its first position in the stage, global
    // slot minus stage position, and the block's next global slot
    __shared__ unsigned int cnt[kPsiMaxBins], off[kPsiMaxBins], delta[kPsiMaxBins], cursor[kPsiMaxBins];
    __shared__ unsigned int ws[NT / kWave];
    const int tid = threadIdx.x;
    const int nbin = a.pnbins;
    const int bsh = a.cptlog + a.binlog;
    for (int b = tid; b < nbin; b += NT) {
        cursor[b] = a.binhist[(int64_t)b * gridDim.x + blockIdx.x];
        cnt[b] = 0;
    }
    __syncthreads();
    const int64_t N = a.p.count;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < N ? beg + chunk : N;
    PsiRec<R>* binned = (PsiRec<R>*)a.binned;
    double mx[C];
#pragma unroll
    for (int k = 0; k < C; ++k) mx[k] = 0.0;
    unsigned long long bad = 0;
    for (int64_t r0 = beg; r0 < end; r0 += RB) {
        int code[U];
        R v[U][3], ug[U][3], r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = r0 + (int64_t)u * NT + tid;
            code[u] = p < end ? a.codes[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = r0 + (int64_t)u * NT + tid;
            const bool live = code[u] >= 0;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                v[u][ax] = live ? ((const R*)a.p.v[ax])[p] : (R)0;
                ug[u][ax] = live ? ((const R*)a.p.ug[ax])[p] : (R)0;
            }
            r[u] = live ? ((const R*)a.p.r)[p] : (R)1;
        }
        PsiRec<R> rec[U];
        unsigned int rank[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rank[u] = 0;
            if (code[u] < 0) continue;
            // the source terms in the precision of the records (binary32
            // records: binary32 arithmetic, within a few ulps of the binary64
            // terms rounded)
            R phi[4];
            bool ok = isfinite(r[u]);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) ok = ok && isfinite(v[u][ax]) && isfinite(ug[u][ax]);
            if (ok) {
                droplet_phi_t<D, R>(r[u], v[u], ug[u], a.ph, phi);
#pragma unroll
                for (int k = 0; k < C; ++k) ok = ok && isfinite(phi[k]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) rec[u].phi[k] = (ok && k < C) ? phi[k] : (R)0;
            rec[u].loc = (uint32_t)code[u] | (ok ? 0u : kPsiSkipBit);
            bad += ok ? 0ull : 1ull;
#pragma unroll
            for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], fabs((double)rec[u].phi[k]));
            rank[u] = atomicAdd(&cnt[code[u] >> bsh], 1u);
        }
        __syncthreads();
        // bins BPT tid .. BPT tid + BPT - 1
        const int b0 = BPT * tid;
        unsigned int c[BPT], sum = 0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            c[k] = b0 + k < nbin ? cnt[b0 + k] : 0u;
            sum += c[k];
        }
        unsigned int total;
        unsigned int ex = block_exclusive_sum<NT>(sum, ws, total);
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (b0 + k < nbin) {
                off[b0 + k] = ex;
                delta[b0 + k] = cursor[b0 + k] - ex;
                cursor[b0 + k] += c[k];
                cnt[b0 + k] = 0;
            }
            ex += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (code[u] < 0) continue;
            stage[off[code[u] >> bsh] + rank[u]] = rec[u];
        }
        __syncthreads();
        for (unsigned int i = tid; i < total; i += NT) {
            const PsiRec<R> r = stage[i];
            binned[delta[(r.loc & ~kPsiSkipBit) >> bsh] + i] = r;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, kWave);
    if ((threadIdx.x % kWave) == 0 && bad) atomicAdd(&a.stats[ST_SKIPPED], bad);
    // per-block maxima (a separate pass reduces them: no contended atomics)
    __shared__ double bm[NT / kWave][4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], __shfl_xor(mx[k], o, kWave));
    if ((threadIdx.x % kWave) == 0)
#pragma unroll
        for (int k = 0; k < C; ++k) bm[threadIdx.x / kWave][k] = mx[k];
    __syncthreads();
    if (threadIdx.x < C) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) v = fmax(v, bm[w][threadIdx.x]);
        a.blockmax[(int64_t)blockIdx.x * 4 + threadIdx.x] = (unsigned long long)__double_as_longlong(v);
    }
}

// Second partition: nsplit workgroups per bin each take a contiguous share
// of the bin's records in rounds, order a round by tile in LDS and reserve
// each tile's run with one atomic add on the tile's cursor, so the stores
// are again contiguous runs.  The order of records inside a tile bucket then
// depends on the schedule; the reduce adds integers, so the sums do not.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_psi_tiles(PsiArgs a)
{
    constexpr int U = PsiRoundPerThread<R>::value;
    constexpr int RB = 256 * U;
    __shared__ PsiRec<R> stage[RB];
    __shared__ uint32_t sslot[RB];
    __shared__ unsigned int cnt[kPsiTilesPerBin], off[kPsiTilesPerBin], gbase[kPsiTilesPerBin];
    __shared__ unsigned int stotal;
    const int tid = threadIdx.x;
    const int bin = blockIdx.x / a.nsplit, part = blockIdx.x % a.nsplit;
    const int64_t nbk = a.nblocks;
    const int64_t c0 = a.binhist[(int64_t)bin * nbk], c1 = a.binhist[(int64_t)(bin + 1) * nbk];
    const int64_t len = c1 - c0;
    const int64_t beg = c0 + len * part / a.nsplit, end = c0 + len * (part + 1) / a.nsplit;
    const uint32_t tile0 = (uint32_t)bin << kPsiTilesPerBinLog;
    const uint32_t cmask = (uint32_t)a.cpt - 1u;
    if (tid < kPsiTilesPerBin) cnt[tid] = 0;
    __syncthreads();
    const PsiRec<R>* src = (const PsiRec<R>*)a.binned;
    PsiRec<R>* dst = (PsiRec<R>*)a.bucket;
    R ph[U][4], phn[U][4];
    uint32_t lc[U], lcn[U];
    auto load = [&](int64_t r0, R (&p)[U][4], uint32_t (&l)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = r0 + (int64_t)u * 256 + tid;
            const bool in = i < end;
            const PsiRec<R>* q = src + (in ? i : 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) p[u][k] = in ? q->phi[k] : (R)0;
            l[u] = in ? q->loc : 0u;
        }
    };
    if (beg < end) load(beg, ph, lc);
    for (int64_t r0 = beg; r0 < end; r0 += RB) {
        int t[U];
        unsigned int rank[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rank[u] = 0;
            t[u] = -1;
            const int64_t i = r0 + (int64_t)u * 256 + tid;
            if (i >= end) continue;
            const uint32_t code = lc[u] & ~kPsiSkipBit;
            t[u] = (int)((code >> a.cptlog) - tile0);
            lc[u] = (lc[u] & kPsiSkipBit) ? kPsiSkip : (code & cmask);
            rank[u] = atomicAdd(&cnt[t[u]], 1u);
        }
        // the next round's records are read while this round is sorted and written
        if (r0 + RB < end) load(r0 + RB, phn, lcn);
        __syncthreads();
        if (tid < kWave) {
            // wave 0: one tile per lane
            const unsigned int c = cnt[tid];
            unsigned int total;
            const unsigned int ex = wave_exclusive_sum(c, total);
            off[tid] = ex;
            gbase[tid] = c ? atomicAdd(&a.tcursor[tile0 + tid], c) : 0u;
            cnt[tid] = 0;
            if (tid == 0) stotal = total;
        }
        __syncthreads();
        const unsigned int total = stotal;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t[u] < 0) continue;
            const unsigned int pos = off[t[u]] + rank[u];
#pragma unroll
            for (int k = 0; k < 4; ++k) stage[pos].phi[k] = ph[u][k];
            stage[pos].loc = lc[u];
            sslot[pos] = gbase[t[u]] + rank[u];
        }
        __syncthreads();
        for (unsigned int i = tid; i < total; i += 256) dst[sslot[i]] = stage[i];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) ph[u][k] = phn[u][k];
            lc[u] = lcn[u];
        }
    }
}

template <int D>
__global__ void k_psi_scale(PsiArgs a)
{
    constexpr int C = D + 1;
    // max over the per-block maxima: one wave per channel
    const int lane = threadIdx.x % kWave;
    for (int k = threadIdx.x / kWave; k < C; k += blockDim.x / kWave) {
        double v = 0.0;
        if (a.p.count > 0)
            for (int b = lane; b < a.nblocks; b += kWave)
                v = fmax(v, __longlong_as_double((long long)a.blockmax[(int64_t)b * 4 + k]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
        if (lane == 0) a.maxbits[k] = (unsigned long long)__double_as_longlong(v);
    }
    // cursors of the tile buckets for the tile pass
    for (int t = threadIdx.x; t < a.pntiles; t += blockDim.x) a.tcursor[t] = a.blockhist[(int64_t)t * a.nblocks];
    __syncthreads();
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double n = (double)(a.p.count > 0 ? a.p.count : 1);
    {
        // fine word of binary64 sums: remainders of at most 2^(f-1) each,
        // at most count of them per cell, count < 2^fx
        int fx;
        frexp(n + 1.0, &fx);
        a.qscale[4] = ldexp(1.0, 62 - fx);
    }
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

// One workgroup per tile: exact integer sums in LDS, then the tile's cells.
// Records come from the tile pass (cell in tile, or kPsiSkip) or straight
// from the scatter (the whole code, with the skip bit); both carry the cell
// in the low bits and the skip bit set when skipped.
template <typename R, int D, int NT>
__global__ __launch_bounds__(NT) void k_psi_reduce(PsiArgs a)
{
    constexpr int C = D + 1;
    constexpr int W = PsiWords<R>::value;           // integer words per channel sum
    extern __shared__ unsigned long long sacc[];    // W * C * cpt sums, then cpt counts (u32)
    const int cpt = a.cpt;
    unsigned int* scnt = reinterpret_cast<unsigned int*>(sacc + (size_t)W * C * cpt);
    for (int i = threadIdx.x; i < W * C * cpt; i += blockDim.x) sacc[i] = 0ull;
    for (int i = threadIdx.x; i < cpt; i += blockDim.x) scnt[i] = 0u;
    double qs[C];
#pragma unroll
    for (int k = 0; k < C; ++k) qs[k] = a.qscale[k];
    const double qf = a.qscale[4];                  // 2^f, the fine word's scale
    __syncthreads();
    const int tile = blockIdx.x;
    const int64_t nbk = a.nblocks;
    const int64_t beg = a.blockhist[(int64_t)tile * nbk];
    const int64_t end = a.blockhist[(int64_t)(tile + 1) * nbk];
    const PsiRec<R>* bucket = (const PsiRec<R>*)a.bucket;
    const int64_t stepw = (int64_t)blockDim.x * kPsiUnrollReduce;
    const bool count = a.den != nullptr;   // the per-cell counts are only an output
    for (int64_t s0 = beg + threadIdx.x; s0 < end; s0 += stepw) {
        PsiRec<R> rec[kPsiUnrollReduce];
#pragma unroll
        for (int u = 0; u < kPsiUnrollReduce; ++u) {
            const int64_t sl = s0 + (int64_t)u * blockDim.x;
            if (sl < end) rec[u] = bucket[sl];
            else rec[u].loc = kPsiSkip;
        }
#pragma unroll
        for (int u = 0; u < kPsiUnrollReduce; ++u) {
            if (rec[u].loc & kPsiSkipBit) continue;
            const int loc = (int)(rec[u].loc & (uint32_t)(cpt - 1));
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const double v = (double)rec[u].phi[k] * qs[k];   // exact: a power-of-two scale
                const double hi = rint(v);
                atomicAdd(&sacc[k * cpt + loc], (unsigned long long)(long long)hi);
                if (W == 2) {
                    // v - hi is exact (|v - hi| <= 1/2 and hi is v's nearest integer)
                    const long long lo = llrint((v - hi) * qf);
                    atomicAdd(&sacc[(C + k) * cpt + loc], (unsigned long long)lo);
                }
            }
            if (count) atomicAdd(&scnt[loc], 1u);
        }
    }
    __syncthreads();
    const MeshDev& m = a.m;
    int tc[3];
    tc[0] = tile % a.pnt[0];
    tc[1] = (tile / a.pnt[0]) % a.pnt[1];
    tc[2] = (D == 3) ? tile / (a.pnt[0] * a.pnt[1]) : 0;
    const double fw = -(a.weight / m.vol);
    for (int loc = threadIdx.x; loc < cpt; loc += blockDim.x) {
        int l0 = loc % a.pt[0];
        int l1 = (loc / a.pt[0]) % a.pt[1];
        int l2 = (D == 3) ? loc / (a.pt[0] * a.pt[1]) : 0;
        int64_t i0 = (int64_t)tc[0] * a.pt[0] + l0;
        int64_t i1 = (int64_t)tc[1] * a.pt[1] + l1;
        int64_t i2 = (int64_t)tc[2] * a.pt[2] + l2;
        if (i0 >= m.n[0] || i1 >= m.n[1] || (D == 3 && i2 >= m.n[2])) continue;
        int64_t c = i0 + (int64_t)m.n[0] * (i1 + (int64_t)m.n[1] * i2);
        double cs = a.cell_scale ? (double)((const R*)a.cell_scale)[c] : 1.0;
        double f = fw * cs;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            double units = (double)(long long)sacc[k * cpt + loc];
            if (W == 2) units += (double)(long long)sacc[(C + k) * cpt + loc] / qf;
            const double sum = units / qs[k];
            ((R*)a.out[k])[c] = (R)(f * sum);
        }
        if (a.den) ((R*)a.den)[c] = (R)scnt[loc];
    }
}

// ---------------------------------------------------------------- cloud in cell
// Each particle's phi is shared among the 2^D cell centres around it with
// per-axis hat weights (1 - f, f), f the fractional offset of the particle
// from the lower centre in cell widths; on a periodic axis the upper centre
// of the last cell is the first cell; on a closed axis a particle less than
// half a cell from a wall puts all of that axis's weight on the boundary
// cell (f = 0).  The sums are exact integer sums as in PSI-CELL, formed per
// tile in LDS over the tile's cells and a one-cell halo on the upper side
// of every axis, then added to a global integer accumulator (one atomic
// per halo'd cell and word, order-independent); a weight channel sums the
// weights themselves.

// Lower-corner cell and fraction along axis ax; false for a position
// outside a closed box (x == hi belongs to the box).  Binary64, in the
// order of the definition (u = (x - lo)/w - 1/2, k = floor(u), f = u - k).
__device__ inline bool cic_axis(const MeshDev& m, int ax, double x, int& k0, double& f)
{
    const double u = (x - m.lo[ax]) / m.w[ax] - 0.5;
    const double fl = floor(u);
    f = u - fl;
    if (!(fabs(fl) < 9.0e15)) return false;
    int64_t k = (int64_t)fl;
    const int64_t n = m.n[ax];
    if (m.periodic[ax]) {
        k0 = (int)posmod(k, n);
        return true;
    }
    // inside the closed box: (x - lo)/w in [0, n], i.e. u in [-1/2, n - 1/2]
    if (!(u >= -0.5 && u <= (double)n - 0.5)) return false;
    if (k < 0) {
        k0 = 0;
        f = 0.0;
    } else if (k >= n - 1) {
        k0 = (int)(n - 1);
        f = 0.0;
    } else {
        k0 = (int)k;
    }
    return true;
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_cic_count(PsiArgs a)
{
    extern __shared__ unsigned int hist[];
    const int ntl = a.pntiles;
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int64_t N = a.p.count;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < N ? beg + chunk : N;
    unsigned long long outside = 0, bad = 0;
    for (int64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
        double x[3];
        bool fin = true;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            x[ax] = a.p.x[ax][p];
            fin = fin && isfinite(x[ax]);
        }
        int code = -1;
        if (!fin) {
            ++bad;
        } else {
            int idx[3] = {0, 0, 0};
            bool in = true;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                double f;
                in = in && cic_axis(a.m, ax, x[ax], idx[ax], f);
            }
            if (in) {
                code = psi_code<D>(a, idx);
                atomicAdd(&hist[code >> a.cptlog], 1u);
            } else {
                ++outside;
            }
        }
        a.codes[p] = code;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) a.blockhist[(int64_t)t * gridDim.x + blockIdx.x] = hist[t];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.blockhist[(int64_t)ntl * gridDim.x] = 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        outside += __shfl_xor(outside, o, kWave);
        bad += __shfl_xor(bad, o, kWave);
    }
    if ((threadIdx.x % kWave) == 0 && outside) atomicAdd(&a.stats[ST_OUTSIDE], outside);
    if ((threadIdx.x % kWave) == 0 && bad) atomicAdd(&a.stats[ST_SKIPPED], bad);
}

// Records into tile buckets: the slots of a block's particles come from its
// scanned per-tile counts, handed out by LDS cursors (the order inside a
// bucket does not matter: the sums are integer sums).
template <typename R, int D>
__global__ __launch_bounds__(256) void k_cic_scatter(PsiArgs a)
{
    constexpr int C = D + 1;
    extern __shared__ unsigned int cursor[];
    const int ntl = a.pntiles;
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) cursor[t] = a.blockhist[(int64_t)t * gridDim.x + blockIdx.x];
    __syncthreads();
    const int64_t N = a.p.count;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < N ? beg + chunk : N;
    CicRec<R>* bucket = (CicRec<R>*)a.bucket;
    double mx[C];
#pragma unroll
    for (int k = 0; k < C; ++k) mx[k] = 0.0;
    unsigned long long bad = 0;
    const uint32_t cmask = (uint32_t)a.cpt - 1u;
    for (int64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
        const int code = a.codes[p];
        if (code < 0) continue;
        R v[3], ug[3];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            v[ax] = ((const R*)a.p.v[ax])[p];
            ug[ax] = ((const R*)a.p.ug[ax])[p];
        }
        const R r = ((const R*)a.p.r)[p];
        bool ok = isfinite(r);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) ok = ok && isfinite(v[ax]) && isfinite(ug[ax]);
        R phi[4] = {0, 0, 0, 0};
        if (ok) {
            droplet_phi_t<D, R>(r, v, ug, a.ph, phi);
#pragma unroll
            for (int k = 0; k < C; ++k) ok = ok && isfinite(phi[k]);
        }
        CicRec<R> rec;
#pragma unroll
        for (int k = 0; k < 4; ++k) rec.phi[k] = (ok && k < C) ? phi[k] : (R)0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) rec.frac[ax] = (R)0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            int k0;
            double f;
            cic_axis(a.m, ax, a.p.x[ax][p], k0, f);
            rec.frac[ax] = (R)f;
        }
        rec.loc = ok ? ((uint32_t)code & cmask) : kPsiSkip;
        bad += ok ? 0ull : 1ull;
#pragma unroll
        for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], fabs((double)rec.phi[k]));
        const unsigned int slot = atomicAdd(&cursor[code >> a.cptlog], 1u);
        bucket[slot] = rec;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, kWave);
    if ((threadIdx.x % kWave) == 0 && bad) atomicAdd(&a.stats[ST_SKIPPED], bad);
    __shared__ double bm[256 / kWave][4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], __shfl_xor(mx[k], o, kWave));
    if ((threadIdx.x % kWave) == 0)
#pragma unroll
        for (int k = 0; k < C; ++k) bm[threadIdx.x / kWave][k] = mx[k];
    __syncthreads();
    if (threadIdx.x < C) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) v = fmax(v, bm[w][threadIdx.x]);
        a.blockmax[(int64_t)blockIdx.x * 4 + threadIdx.x] = (unsigned long long)__double_as_longlong(v);
    }
}

// Records into tile buckets, sorted: each block takes its contiguous range
// of particles in rounds, orders a round's records by tile in LDS (counting
// sort) and writes them out as one contiguous run per tile, at the slots of
// its scanned per-tile counts (as the PSI-CELL scatter does with its bins;
// here the bins are the tiles, at most kCicMaxBins of them).  Records keep
// their whole code (tile and cell) with the skip bit.
template <typename R> struct CicRoundPerThread { static constexpr int value = sizeof(R) == 4 ? 14 : 7; };
template <typename R, int D>
__global__ __launch_bounds__(256) void k_cic_scatter_sorted(PsiArgs a)
{
    constexpr int C = D + 1;
    constexpr int NT = 256;
    constexpr int U = CicRoundPerThread<R>::value;
    constexpr int RB = NT * U;
    constexpr int BPT = kCicMaxBins / NT;
    __shared__ CicRec<R> stage[RB];
    __shared__ unsigned int cnt[kCicMaxBins], off[kCicMaxBins], delta[kCicMaxBins], cursor[kCicMaxBins];
    __shared__ unsigned int ws[NT / kWave];
    const int tid = threadIdx.x;
    const int nbin = a.pntiles;
    const int bsh = a.cptlog;
    for (int b = tid; b < nbin; b += NT) {
        cursor[b] = a.blockhist[(int64_t)b * gridDim.x + blockIdx.x];
        cnt[b] = 0;
    }
    __syncthreads();
    const int64_t N = a.p.count;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < N ? beg + chunk : N;
    CicRec<R>* bucket = (CicRec<R>*)a.bucket;
    double mx[C];
#pragma unroll
    for (int k = 0; k < C; ++k) mx[k] = 0.0;
    unsigned long long bad = 0;
    for (int64_t r0 = beg; r0 < end; r0 += RB) {
        int code[U];
        unsigned int rank[U];
        CicRec<R> rec[U];
        R v[U][3], ug[U][3], rr[U];
        double xp[U][3];
        // the round's loads first: codes, then the inputs of every live particle
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = r0 + (int64_t)u * NT + tid;
            code[u] = p < end ? a.codes[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = r0 + (int64_t)u * NT + tid;
            const bool live = code[u] >= 0;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                v[u][ax] = live ? ((const R*)a.p.v[ax])[p] : (R)0;
                ug[u][ax] = live ? ((const R*)a.p.ug[ax])[p] : (R)0;
                xp[u][ax] = live ? a.p.x[ax][p] : 0.0;
            }
            rr[u] = live ? ((const R*)a.p.r)[p] : (R)1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rank[u] = 0;
            if (code[u] < 0) continue;
            bool ok = isfinite(rr[u]);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) ok = ok && isfinite(v[u][ax]) && isfinite(ug[u][ax]);
            R phi[4] = {0, 0, 0, 0};
            if (ok) {
                droplet_phi_t<D, R>(rr[u], v[u], ug[u], a.ph, phi);
#pragma unroll
                for (int k = 0; k < C; ++k) ok = ok && isfinite(phi[k]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) rec[u].phi[k] = (ok && k < C) ? phi[k] : (R)0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) rec[u].frac[ax] = (R)0;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                int k0;
                double f;
                cic_axis(a.m, ax, xp[u][ax], k0, f);
                rec[u].frac[ax] = (R)f;
            }
            rec[u].loc = (uint32_t)code[u] | (ok ? 0u : kPsiSkipBit);
            bad += ok ? 0ull : 1ull;
#pragma unroll
            for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], fabs((double)rec[u].phi[k]));
            rank[u] = atomicAdd(&cnt[code[u] >> bsh], 1u);
        }
        __syncthreads();
        // tiles BPT tid .. BPT tid + BPT - 1
        const int b0 = BPT * tid;
        unsigned int c[BPT], sum = 0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            c[k] = b0 + k < nbin ? cnt[b0 + k] : 0u;
            sum += c[k];
        }
        unsigned int total;
        unsigned int ex = block_exclusive_sum<NT>(sum, ws, total);
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (b0 + k < nbin) {
                off[b0 + k] = ex;
                delta[b0 + k] = cursor[b0 + k] - ex;
                cursor[b0 + k] += c[k];
                cnt[b0 + k] = 0;
            }
            ex += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (code[u] < 0) continue;
            stage[off[code[u] >> bsh] + rank[u]] = rec[u];
        }
        __syncthreads();
        for (unsigned int i = tid; i < total; i += NT) {
            const CicRec<R> q = stage[i];
            bucket[delta[(q.loc & ~kPsiSkipBit) >> bsh] + i] = q;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, kWave);
    if ((threadIdx.x % kWave) == 0 && bad) atomicAdd(&a.stats[ST_SKIPPED], bad);
    __shared__ double bm[NT / kWave][4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < C; ++k) mx[k] = fmax(mx[k], __shfl_xor(mx[k], o, kWave));
    if ((threadIdx.x % kWave) == 0)
#pragma unroll
        for (int k = 0; k < C; ++k) bm[threadIdx.x / kWave][k] = mx[k];
    __syncthreads();
    if (threadIdx.x < C) {
        double v = 0.0;
        for (int w = 0; w < NT / kWave; ++w) v = fmax(v, bm[w][threadIdx.x]);
        a.blockmax[(int64_t)blockIdx.x * 4 + threadIdx.x] = (unsigned long long)__double_as_longlong(v);
    }
}

// One workgroup per tile: the tile's particles deposit into LDS sums over
// the tile and its upper halo, which are then added to the global sums.
// Channels 0..C-1 carry phi (W words each), channel C the weights (W words,
// at the scale of the fine word: at most one unit of weight per particle and
// corner).
template <typename R, int D, int NT>
__global__ __launch_bounds__(NT) void k_cic_reduce(PsiArgs a)
{
    constexpr int C = D + 1;
    constexpr int W = PsiWords<R>::value;
    constexpr int NCH = W * (C + 1);     // integer words per cell: C channels, then the weights
    extern __shared__ unsigned long long sacc[];
    const int hx = a.pt[0] + 1, hy = a.pt[1] + 1, hz = D == 3 ? a.pt[2] + 1 : 1;
    const int HC = hx * hy * hz;
    for (int i = threadIdx.x; i < NCH * HC; i += blockDim.x) sacc[i] = 0ull;
    double qs[C];
#pragma unroll
    for (int k = 0; k < C; ++k) qs[k] = a.qscale[k];
    // a particle can put up to 2^D remainders (and weights) on one cell
    // (periodic axes of one cell): 2^-D of the PSI-CELL fine scale
    const double qf = a.qscale[4] / (double)(1 << D);
    __syncthreads();
    const int tile = blockIdx.x;
    const int64_t nbk = a.nblocks;
    const int64_t beg = a.blockhist[(int64_t)tile * nbk];
    const int64_t end = a.blockhist[(int64_t)(tile + 1) * nbk];
    const CicRec<R>* bucket = (const CicRec<R>*)a.bucket;
    for (int64_t sl = beg + threadIdx.x; sl < end; sl += blockDim.x) {
        const CicRec<R> rec = bucket[sl];
        // the cell in the tile: the low bits of a full code (sorted scatter)
        // or of the cell itself; skipped records carry the skip bit
        if (rec.loc & kPsiSkipBit) continue;
        const uint32_t cl = rec.loc & (uint32_t)(a.cpt - 1);
        const int l0 = (int)(cl & (uint32_t)(a.pt[0] - 1));
        const int l1 = (int)((cl >> a.ptlog[0]) & (uint32_t)(a.pt[1] - 1));
        const int l2 = D == 3 ? (int)(cl >> (a.ptlog[0] + a.ptlog[1])) : 0;
        double wa[3][2];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double f = ax < D ? (double)rec.frac[ax] : 0.0;
            wa[ax][0] = 1.0 - f;
            wa[ax][1] = f;
        }
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) {
            const int b0 = q & 1, b1 = (q >> 1) & 1, b2 = D == 3 ? (q >> 2) & 1 : 0;
            const double w = wa[0][b0] * wa[1][b1] * (D == 3 ? wa[2][b2] : 1.0);
            if (w == 0.0) continue;
            const int hc = (l0 + b0) + hx * ((l1 + b1) + hy * (l2 + b2));
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const double v = (double)rec.phi[k] * w * qs[k];
                const double hi = rint(v);
                atomicAdd(&sacc[(size_t)(W * k) * HC + hc], (unsigned long long)(long long)hi);
                if (W == 2) {
                    const long long lo = llrint((v - hi) * qf);
                    atomicAdd(&sacc[(size_t)(W * k + 1) * HC + hc], (unsigned long long)lo);
                }
            }
            // the weights, W words as the channels (the fine word keeps the
            // remainder of each quantised weight, so sparse cells keep their
            // relative accuracy)
            const double wq = w * qf;
            const double wh = rint(wq);
            atomicAdd(&sacc[(size_t)(W * C) * HC + hc], (unsigned long long)(long long)wh);
            if (W == 2) atomicAdd(&sacc[(size_t)(W * C + 1) * HC + hc], (unsigned long long)llrint((wq - wh) * qf));
        }
    }
    __syncthreads();
    const MeshDev& m = a.m;
    int tc[3];
    tc[0] = tile % a.pnt[0];
    tc[1] = (tile / a.pnt[0]) % a.pnt[1];
    tc[2] = (D == 3) ? tile / (a.pnt[0] * a.pnt[1]) : 0;
    const int64_t M = m.M;
    for (int hc = threadIdx.x; hc < HC; hc += blockDim.x) {
        const int h0 = hc % hx, h1 = (hc / hx) % hy, h2 = hc / (hx * hy);
        int64_t i[3] = {(int64_t)tc[0] * a.pt[0] + h0, (int64_t)tc[1] * a.pt[1] + h1,
                        D == 3 ? (int64_t)tc[2] * a.pt[2] + h2 : 0};
        bool inside = true;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            if (i[ax] >= m.n[ax]) {
                if (m.periodic[ax])
                    i[ax] -= m.n[ax];
                else
                    inside = false;
            }
        }
        if (!inside) continue;
        const int64_t c = i[0] + (int64_t)m.n[0] * (i[1] + (int64_t)m.n[1] * i[2]);
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const unsigned long long v = sacc[(size_t)j * HC + hc];
            if (v) atomicAdd(&a.acc[(size_t)j * M + c], v);
        }
    }
}

template <typename R, int D>
__global__ void k_cic_finish(PsiArgs a)
{
    constexpr int C = D + 1;
    constexpr int W = PsiWords<R>::value;
    const MeshDev& m = a.m;
    const int64_t M = m.M;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    const double qf = a.qscale[4] / (double)(1 << D);
    const double cs = a.cell_scale ? (double)((const R*)a.cell_scale)[c] : 1.0;
    const double f = -(a.weight / m.vol) * cs;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        double units = (double)(long long)a.acc[(size_t)(W * k) * M + c];
        if (W == 2) units += (double)(long long)a.acc[(size_t)(W * k + 1) * M + c] / qf;
        ((R*)a.out[k])[c] = (R)(f * (units / a.qscale[k]));
    }
    if (a.den) {
        double units = (double)(long long)a.acc[(size_t)(W * C) * M + c];
        if (W == 2) units += (double)(long long)a.acc[(size_t)(W * C + 1) * M + c] / qf;
        ((R*)a.den)[c] = (R)(units / qf);
    }
}

template <typename R, int D>
hipError_t launch_cic(const PsiArgs& a, hipStream_t s)
{
    constexpr int C = D + 1;
    constexpr int W = PsiWords<R>::value;
    hipError_t e = launch_fill_u64(a.maxbits, C, 0ull, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u64(a.acc, (int64_t)(W * (C + 1)) * a.m.M, 0ull, s);
    if (e != hipSuccess) return e;
    const size_t lds_t = sizeof(unsigned int) * (size_t)a.pntiles;
    if (a.p.count == 0) {
        e = launch_fill_u32(a.blockhist, (int64_t)a.pntiles * a.nblocks + 1, 0u, s);
        if (e != hipSuccess) return e;
        e = launch_fill_u64(a.blockmax, (int64_t)a.nblocks * 4, 0ull, s);
        if (e != hipSuccess) return e;
    } else {
        FLA_LAUNCH((k_cic_count<R, D>), dim3(a.nblocks), dim3(256), lds_t, s, a);
        e = launch_exclusive_scan_u32(a.blockhist, (int64_t)a.pntiles * a.nblocks + 1, a.scan_tmp, a.scan_words, s);
        if (e != hipSuccess) return e;
        if (a.direct)
            FLA_LAUNCH((k_cic_scatter_sorted<R, D>), dim3(a.nblocks), dim3(256), 0, s, a);
        else
            FLA_LAUNCH((k_cic_scatter<R, D>), dim3(a.nblocks), dim3(256), lds_t, s, a);
    }
    FLA_LAUNCH((k_psi_scale<D>), dim3(1), dim3(256), 0, s, a);
    const int hcells = (a.pt[0] + 1) * (a.pt[1] + 1) * (D == 3 ? a.pt[2] + 1 : 1);
    const size_t lds_r = sizeof(unsigned long long) * (size_t)(W * (C + 1)) * (size_t)hcells;
    // large (sorted) tiles: one workgroup of 1024 threads per compute unit,
    // so that enough waves issue the LDS atomics
    if (a.direct) {
        e = hipFuncSetAttribute((const void*)k_cic_reduce<R, D, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_r);
        if (e != hipSuccess) return e;
        FLA_LAUNCH((k_cic_reduce<R, D, 1024>), dim3(a.pntiles), dim3(1024), lds_r, s, a);
    } else {
        FLA_LAUNCH((k_cic_reduce<R, D, 256>), dim3(a.pntiles), dim3(256), lds_r, s, a);
    }
    FLA_LAUNCH((k_cic_finish<R, D>), dim3((unsigned)((a.m.M + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_cic<float, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_cic<float, 3>(const PsiArgs&, hipStream_t);
template hipError_t launch_cic<double, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_cic<double, 3>(const PsiArgs&, hipStream_t);

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
    FLA_LAUNCH(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    FLA_LAUNCH(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_fill_real(R* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    FLA_LAUNCH((k_fill_real<R>), dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
template hipError_t launch_fill_real<float>(float*, int64_t, hipStream_t);
template hipError_t launch_fill_real<double>(double*, int64_t, hipStream_t);

template <typename R, int D>
hipError_t launch_psicell(const PsiArgs& a, hipStream_t s)
{
    constexpr int C = D + 1;
    hipError_t e = launch_fill_u64(a.maxbits, C, 0ull, s);
    if (e != hipSuccess) return e;
    if (a.p.count == 0) {
        // no particle: every tile reduces an empty bucket
        e = launch_fill_u32(a.blockhist, (int64_t)a.pntiles * a.nblocks + 1, 0u, s);
        if (e != hipSuccess) return e;
    } else {
        size_t lds_t = sizeof(unsigned int) * (size_t)a.pntiles;
        FLA_LAUNCH((k_psi_count<R, D>), dim3(a.nblocks), dim3(256), lds_t, s, a);
        e = launch_exclusive_scan_u32(a.blockhist, (int64_t)a.pntiles * a.nblocks + 1, a.scan_tmp, a.scan_words, s);
        if (e != hipSuccess) return e;
        if (!a.direct) {
            e = launch_exclusive_scan_u32(a.binhist, (int64_t)a.pnbins * a.nblocks + 1, a.scan_tmp, a.scan_words, s);
            if (e != hipSuccess) return e;
        }
        FLA_LAUNCH((k_psi_scatter<R, D>), dim3(a.nblocks), dim3(kPsiScatterThreads), 0, s, a);
    }
    FLA_LAUNCH((k_psi_scale<D>), dim3(1), dim3(256), 0, s, a);
    if (a.p.count > 0 && !a.direct)
        FLA_LAUNCH((k_psi_tiles<R, D>), dim3(a.pnbins * a.nsplit), dim3(256), 0, s, a);
    size_t lds_r = (sizeof(unsigned long long) * C * PsiWords<R>::value + sizeof(unsigned int)) * (size_t)a.cpt;
    if (a.direct) {
        e = hipFuncSetAttribute((const void*)k_psi_reduce<R, D, kPsiDirectThreads>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r);
        if (e != hipSuccess) return e;
        FLA_LAUNCH((k_psi_reduce<R, D, kPsiDirectThreads>), dim3(a.pntiles), dim3(kPsiDirectThreads), lds_r, s, a);
    }
    else
        FLA_LAUNCH((k_psi_reduce<R, D, 256>), dim3(a.pntiles), dim3(256), lds_r, s, a);
    return hipGetLastError();
}

template hipError_t launch_psicell<float, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<float, 3>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<double, 2>(const PsiArgs&, hipStream_t);
template hipError_t launch_psicell<double, 3>(const PsiArgs&, hipStream_t);

}  // namespace flp
