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
    uint32_t* pairs;            // nullable per-cell included-pair counts (zeroed by the caller)
    unsigned long long* stats;
    // optional (both set or both null): workspace for the work order of the
    // single-snapshot gather, ntiles cost words and 2 * ntiles slot entries
    uint32_t* tile_cost;
    int* order;
    // optional: kXcds counters of workspace for a persistent launch of ncu
    // compute units' worth of workgroups (null: one workgroup per work item)
    uint32_t* queue;
    int ncu;
};

// One snapshot of a batched projection (device table entry).
struct BatchItem {
    GatherArgs g;            // mesh, sorted-record views and outputs of the snapshot
    TrajDev t;
    PhysDev ph;
    const float* hfac;
    int64_t base;            // first global trajectory index of the snapshot
    uint32_t key_base;       // first global bucket of the snapshot
    int tile_base;           // first work item (tile) of the snapshot in the gather launch
};

template <typename R, int D>
hipError_t launch_prepass_batch(const BatchItem* items, int nsnap, int64_t total, uint32_t sentinel, uint32_t* keys,
                                uint32_t* vals, double4* rpos, R* rw, unsigned long long* stats, hipStream_t s);
hipError_t launch_max_class_batch(const BatchItem* items, int nsnap, const uint32_t* bstart,
                                  unsigned long long* stats, hipStream_t s);
// Persistent gather over the work items of a batch; queue holds kXcds
// counters of workspace (zeroed by the launcher), ncu the compute units.
template <typename R, int D>
hipError_t launch_gather_batch(const BatchItem* items, int nsnap, int nwork, int chunk, bool count, int plan_code,
                               bool general, uint32_t* queue, int ncu, hipStream_t s);

// Trajectory producer: the gas field and the droplet state it advances.
struct FlowDev {
    int kind;                 // FLA_FLOW_*
    double U, k;
    double abc[3], phase[3], u0[3];
    double G[9];              // du_a/dx_b at G[a*3 + b]
};
struct ProduceArgs {
    int64_t count;
    double* x[3];
    double* v[3];
    double* J;                // dim*dim planes
    double* dJ;               // dim*dim planes
    double* r;
    const double* n0;
    double n0_scalar;
    double seed_volume;
    double* phibar;           // nullable: 1 + dim planes of the step's source rates
    FlowDev flow;
    double dt;
    int substeps;
    int update;               // write the advanced state back
};

// Advances every droplet over the step and emits the prepass records of the
// advanced state with the step's source rates (as launch_prepass does for a
// given state).
template <typename R, int D>
hipError_t launch_produce(const ProduceArgs& p, const MeshDev& m, const PhysDev& ph, const float* hfac, int deposit,
                          uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, double* qd, unsigned long long* stats,
                          hipStream_t s);

template <typename R, int D>
hipError_t launch_prepass(const TrajDev& t, const MeshDev& m, const PhysDev& ph, const float* hfac,
                          int deposit, uint32_t* keys, uint32_t* vals, double4* rpos, R* rw,
                          double* qd, unsigned long long* stats, hipStream_t s);

hipError_t launch_bucket_bounds(const uint32_t* keys, int64_t n, uint32_t nb, uint32_t* bstart,
                                hipStream_t s);
hipError_t launch_max_class(const uint32_t* bstart, int ntiles, unsigned long long* stats, hipStream_t s);

template <typename R>
hipError_t launch_permute(const uint32_t* order, int64_t n, const double4* rpos_u, const R* rw_u,
                          double4* rpos, R* rw, int copy_w, hipStream_t s);

template <typename R, int D>
hipError_t launch_deposit_norm(const MeshDev& m, const PhysDev& ph, const uint32_t* nvalid,
                               const uint32_t* order, const double* qd, int64_t N, double4* rpos, R* rw,
                               unsigned long long* stats, hipStream_t s);

// Gather plan codes: plan + kGatherPlans * shape.  The plan sets how finely
// the gather skips unreachable sub-blocks; the shape the part of a tile one
// workgroup owns (0: half a tile along x in 3-D, the whole tile in 2-D;
// 1: the whole tile, 3-D only).
constexpr int kGatherPlans = 4;
constexpr int kGatherShapes = 2;
template <int D> constexpr int gather_plan_codes() { return D == 3 ? kGatherPlans * kGatherShapes : kGatherPlans; }
template <typename R, int D>
hipError_t launch_gather(const GatherArgs& g, int mode, bool count, int plan_code, hipStream_t s);

// PSI-CELL
struct PsiArgs {
    MeshDev m;
    TrajDev p;
    PhysDev ph;
    double weight;
    const void* cell_scale;
    void* out[4];
    void* den;
    unsigned long long* maxbits; // C: bit patterns of max |phi_k| (binary64)
    double* qscale;              // 5: 2^e_k per channel, then 2^f (fine word of binary64 sums)
    unsigned long long* stats;
    // tile buckets
    int pt[3];                   // tile edge per axis (cells)
    int pnt[3];                  // tiles per axis
    int pntiles;
    int cpt;                     // cells per tile
    int ptlog[3];                // log2 of pt (tile edges are powers of two)
    int cptlog;                  // log2 of cpt
    int nblocks;                 // blocks of the count / scatter passes
    int* codes;                  // per particle: tile * cpt + cell in tile, or -1
    unsigned int* blockhist;     // pntiles * nblocks + 1, scanned in place
    int pnbins;                  // bins of 2^binlog consecutive tiles
    int binlog;                  // log2 tiles per bin: kPsiTilesPerBinLog, or 0 when direct
    int direct;                  // the scatter writes the tile buckets itself (bins are tiles; no tile pass)
    int nsplit;                  // workgroups per bin in the tile pass
    unsigned int* binhist;       // pnbins * nblocks + 1, scanned in place
    unsigned int* tcursor;       // pntiles: next free slot of each tile bucket
    void* binned;                // records grouped by bin (loc = code, top bit = skip)
    void* bucket;                // records grouped by tile (loc = cell in tile or kPsiSkip)
    unsigned long long* blockmax; // nblocks x C bit patterns of per-block max |phi_k|
    unsigned long long* acc;     // CIC: (C + 1) channels x words x M integer sums (zeroed by the launcher)
    uint32_t* scan_tmp;
    int64_t scan_words;
};

// One bucketed PSI-CELL particle, written and read as one contiguous record.
template <typename R> struct PsiRec {
    R phi[4];
    uint32_t loc;
};

// integer words per channel sum: binary64 records add a fine remainder word
template <typename R> struct PsiWords { static constexpr int value = sizeof(R) == 8 ? 2 : 1; };

constexpr int kPsiMaxTiles = 16384;   // LDS histogram of the count pass <= 64 KiB
constexpr int kPsiTilesPerBinLog = 6;
constexpr int kPsiTilesPerBin = 1 << kPsiTilesPerBinLog;    // tiles per bin of the first partition
constexpr int kPsiMaxBins = 512;       // bins of the scatter: two per thread in its bin scans
static_assert(kPsiMaxTiles / kPsiTilesPerBin <= kPsiMaxBins, "the bins of the tile partition must fit the scatter");
constexpr int kPsiMaxCellsPerTile = 1024;  // LDS sums of the reduce pass <= 36 KiB
constexpr int kPsiDirectThreads = 1024;    // threads of a reduce workgroup over one large tile
constexpr int kPsiBlocks = 1024;

template <typename R, int D>
hipError_t launch_psicell(const PsiArgs& a, hipStream_t s);

// One bucketed CIC particle: source terms, the fractional offsets from the
// lower-corner cell centre along each axis, and that cell in its tile.
template <typename R> struct CicRec {
    R phi[4];
    R frac[3];
    uint32_t loc;
};

// Cloud-in-cell accumulation on the PSI-CELL tile buckets (tiles of a.pt
// cells, keyed by each particle's lower-corner cell).  With a.direct the
// scatter sorts its rounds by tile in LDS (at most kCicMaxBins tiles).
constexpr int kCicMaxBins = 1024;
template <typename R, int D>
hipError_t launch_cic(const PsiArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// General meshes: cells given by their centroids.  A rectilinear grid of
// buckets (per-axis edges at quantiles of the centroid coordinates, so that
// the buckets hold similar numbers of cells) replaces the Cartesian tiles:
// cells are sorted by bucket, trajectories keyed by home bucket and
// neighbourhood class exactly as on the Cartesian mesh, with distances in
// buckets.
constexpr int kCellsMaxBuckets = 1024;   // per axis
constexpr int kCellsHistBins = 65536;    // per axis, for the quantile edges
constexpr int kCellsPerLane = 2;         // cells owned by each lane of the gather
constexpr int kCellsPerItem = kWave * kCellsPerLane;

struct CellGridDev {
    int dim;
    int nb[3];                // buckets per axis
    int periodic[3];
    int nbuckets;
    double lo[3], hi[3], L[3];
    const double* edges[3];   // nb[a] + 1 edges per axis: lo, interior edges, hi
};

struct CellsGatherArgs {
    CellGridDev g;
    const double* xc[3];      // centroids in bucket order
    const double* vol;        // volumes in bucket order (nullable)
    const uint32_t* perm;     // bucket order -> caller's cell index
    const int4* work;         // {bucket, first cell (bucket order), cells, 0}
    int nwork;
    const double4* rpos;      // sorted trajectory records, as for the Cartesian gather
    const void* rw;
    const uint32_t* bstart;   // kClasses * nbuckets + 1 bucket starts
    double cutoff;
    double filt2;             // (c (1 + margin))^2 for the conservative record filter
    double scale;             // multiplier of every cell: scale, or scale * (n_hat per unit volume)
    int use_vol;              // multiply by the cell volume as well (n_hat of App. A)
    void* out[4];
    void* den;
    uint32_t* pairs;
    unsigned long long* stats;
};

hipError_t launch_cells_hist(int dim, int64_t M, const double* const* xc, const double* lo, const double* hi,
                             uint32_t* hist, uint32_t* bad, const double* vol, hipStream_t s);
hipError_t launch_cells_key(const CellGridDev& g, int64_t M, const double* const* xc, uint32_t* keys, uint32_t* vals,
                            hipStream_t s);
hipError_t launch_cells_sorted(int dim, int64_t M, const uint32_t* order, const double* const* xc, const double* vol,
                               double* const* xs, double* vs, uint32_t* perm, hipStream_t s);
template <typename R, int D>
hipError_t launch_cells_prepass(const TrajDev& t, const CellGridDev& g, const PhysDev& ph, const float* hfac,
                                uint32_t* keys, uint32_t* vals, double4* rpos, R* rw, unsigned long long* stats,
                                hipStream_t s);
template <typename R, int D>
hipError_t launch_cells_gather(const CellsGatherArgs& a, bool count, hipStream_t s);

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
template <typename R>
hipError_t launch_fill_real(R* p, int64_t n, hipStream_t s);

}  // namespace flp
