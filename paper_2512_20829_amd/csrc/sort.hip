// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs, written for 64-wide wavefronts.  Both are deterministic: ranks inside
// a block come from wavefront ballots in item order, never from atomics.
#include "internal.hpp"

namespace flp {

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;   // 1024 elements per block

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one 1024-element block in place; writes the block total.
__global__ __launch_bounds__(kScanThreads) void k_scan_block(uint32_t* data, int64_t n, uint32_t* sums)
{
    __shared__ uint32_t wsum[kScanThreads / kWave];
    int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? data[base + k] : 0u;
        tot += v[k];
    }
    uint32_t inc = wave_incl_scan(tot, lane);
    if (lane == kWave - 1) wsum[wv] = inc;
    __syncthreads();
    uint32_t woff = 0;
    for (int w = 0; w < wv; ++w) woff += wsum[w];
    uint32_t run = woff + inc - tot;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) data[base + k] = run;
        run += v[k];
    }
    if (t == kScanThreads - 1) sums[blockIdx.x] = woff + inc;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t* data, int64_t n, const uint32_t* offs)
{
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t o = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) data[base + k] += o;
}

int64_t scan_tmp_words(int64_t n)
{
    int64_t words = 0;
    while (n > 1) {
        n = (n + kScanBlock - 1) / kScanBlock;
        words += n + 1;
    }
    return words + 1;
}

hipError_t launch_exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* tmp, int64_t tmp_words,
                                     hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb + 1 > tmp_words) return hipErrorInvalidValue;
    FLA_LAUNCH(k_scan_block, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    if (nb > 1) {
        hipError_t e = launch_exclusive_scan_u32(tmp, nb, tmp + nb + 1, tmp_words - nb - 1, s);
        if (e != hipSuccess) return e;
        FLA_LAUNCH(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 items per block
constexpr int kDigits = 256;

int64_t radix_hist_words(int64_t n)
{
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    return nb * kDigits;
}

// Per-block digit histogram, stored digit-major: hist[d * nblocks + b].
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* keys, int64_t n, int shift,
                                                           uint32_t* hist, int nblocks)
{
    __shared__ uint32_t cnt[kDigits];
    int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + (int64_t)k * kSortThreads + t;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = cnt[t];
}

// Stable scatter.  Items are visited in 16 rounds of 256 consecutive items;
// inside a wave the rank among equal digits comes from 8 ballots, across
// the 4 waves of a round from a prefix over per-wave counts.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* keys, const uint32_t* vals,
                                                              int64_t n, int shift, const uint32_t* offs,
                                                              int nblocks, uint32_t* keys_out,
                                                              uint32_t* vals_out)
{
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t run[kDigits];
    __shared__ uint32_t wcnt[NW][kDigits];
    int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    run[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int k = 0; k < kSortItems; ++k) {
        for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;
        __syncthreads();
        int64_t i = base + (int64_t)k * kSortThreads + t;
        bool valid = i < n;
        uint32_t key = valid ? keys[i] : 0u;
        uint32_t val = valid ? vals[i] : 0u;
        uint32_t d = (key >> shift) & 0xFF;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < NW; ++w) add += wcnt[w][t];
        run[t] += add;
        __syncthreads();
    }
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                            int64_t n, int key_bits, uint32_t* hist, int64_t hist_words,
                            uint32_t* scan_tmp, int64_t scan_tmp_words_, hipStream_t s,
                            bool* result_in_alt)
{
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    if ((int64_t)nblocks * kDigits > hist_words) return hipErrorInvalidValue;
    uint32_t *ka = keys, *va = vals, *kb = keys_alt, *vb = vals_alt;
    for (int shift = 0; shift < key_bits; shift += 8) {
        FLA_LAUNCH(k_radix_hist, dim3(nblocks), dim3(kSortThreads), 0, s, ka, n, shift, hist,
                           nblocks);
        hipError_t e = launch_exclusive_scan_u32(hist, (int64_t)nblocks * kDigits, scan_tmp,
                                                 scan_tmp_words_, s);
        if (e != hipSuccess) return e;
        FLA_LAUNCH(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, s, ka, va, n, shift,
                           hist, nblocks, kb, vb);
        uint32_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
        *result_in_alt = !*result_in_alt;
    }
    return hipGetLastError();
}

}  // namespace flp
