// Launcher declarations shared between the kernel translation units and the
// host runtime.
#pragma once

#include "internal.hpp"

namespace flp {

struct GatherArgs {
    MeshDev m;
    const double4* rpos;        // sorted {x, y, z, 1/h}; 1/h < 0 flags a delta record
    const void* rw;             // sorted weight records, kRecW reals each
    const uint32_t* bstart;     // bucket starts, kClasses * ntiles + 1 entries
    double cutoff;              // c
    double filt2;               // (c (1 + margin))^2 for the conservative tile filter
    double scale;
    const void* cell_scale;
    void* out[4];
    void* den;
    unsigned long long* stats;
};

template <typename R, int D>
hipError_t launch_prepass(const TrajDev& t, const MeshDev& m, const PhysDev& ph, const float* hfac,
                          int deposit, uint32_t* keys, uint32_t* vals, double4* rpos, R* rw,
                          double* qd, unsigned long long* stats, hipStream_t s);

hipError_t launch_bucket_bounds(const uint32_t* keys, int64_t n, uint32_t nb, uint32_t* bstart,
                                hipStream_t s);

template <typename R>
hipError_t launch_permute(const uint32_t* order, int64_t n, const double4* rpos_u, const R* rw_u,
                          double4* rpos, R* rw, int copy_w, hipStream_t s);

template <typename R, int D>
hipError_t launch_deposit_norm(const MeshDev& m, const PhysDev& ph, const uint32_t* nvalid,
                               const uint32_t* order, const double* qd, int64_t N, double4* rpos, R* rw,
                               unsigned long long* stats, hipStream_t s);

template <typename R, int D>
hipError_t launch_gather(const GatherArgs& g, int mode, bool count, hipStream_t s);

// PSI-CELL
struct PsiArgs {
    MeshDev m;
    TrajDev p;
    PhysDev ph;
    double weight;
    const void* cell_scale;
    void* out[4];
    void* den;
    unsigned long long* acc;     // C x M fixed-point sums
    unsigned int* counts;        // M
    unsigned long long* maxbits; // C: bit patterns of max |phi_k| (binary64)
    double* qscale;              // C: 2^e_k
    unsigned long long* stats;
};

template <typename R, int D>
hipError_t launch_psicell(const PsiArgs& a, hipStream_t s);

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
template <typename R>
hipError_t launch_fill_real(R* p, int64_t n, hipStream_t s);

}  // namespace flp
