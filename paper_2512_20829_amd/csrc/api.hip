// Host runtime and C ABI of the FLA projection library: argument validation,
// the grow-only workspace, and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "flaproj.h"
#include "internal.hpp"
#include "host_logic.hpp"
#include "kernels.hpp"
#include "learned.hpp"

using namespace flp;

struct fla_ctx {
    int device = 0;
    std::string err;
    void* ws = nullptr;
    size_t ws_size = 0;
    // training workspace: the intermediates of fla_mlp_train_step and
    // fla_bandwidth_standardise, which live across calls that use ws
    void* tws = nullptr;
    size_t tws_size = 0;
    unsigned long long* stats = nullptr;   // ST_N counters
    int plan[2][2] = {{-1, -1}, {-1, -1}};  // gather plan per (dim - 2, precision); -1 = default
    bool prof = false;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    // batched projection: plan per (dim - 2, precision), snapshot table, cached graph
    int batch_plan[2][2] = {{-1, -1}, {-1, -1}};
    int batch_chunk[2][2] = {{-1, -1}, {-1, -1}};
    bool batch_graph = true;
    void* items = nullptr;                 // device snapshot table
    size_t items_size = 0;
    hipEvent_t items_done = nullptr;       // recorded after the last batch call's work
    bool items_pending = false;
    hipStream_t capture = nullptr;         // stream the launch sequence is captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;
    int64_t graph_replays = 0;
    // single calls (fla_set_graph): the cached graph of fla_project_sources,
    // its argument key, and the key of the last direct call
    bool single_graph = false;
    hipGraph_t sgraph = nullptr;
    hipGraphExec_t sgraph_exec = nullptr;
    std::vector<unsigned char> sgraph_key, sgraph_seen;
    // testing aid (FLA_FAIL_ALLOC=k at creation): the k-th device allocation
    // made for this context fails as if the device were out of memory
    int64_t fail_alloc = 0;
};

namespace flp {
int g_trace = 0;

void trace_launch(const char* kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    std::fprintf(stderr, "[flaproj] launch %s grid=(%u,%u,%u) block=(%u,%u,%u) lds=%zu stream=%p\n", kernel, grid.x,
                 grid.y, grid.z, block.x, block.y, block.z, lds, (void*)s);
    std::fflush(stderr);
}
}  // namespace flp

static thread_local std::string g_create_error;

// Workspace of fla_project_sources_noalloc: a fixed array in the code object,
// one copy per GPU, held until the process ends.  Host code never uses the
// name `scratch` as an address (on the host it is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once, with that
// GPU current, when the first context on it is created, and kept here.
static __device__ __align__(256) unsigned char scratch[FLA_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

// gather plan used until fla_set_plan or fla_autotune chooses one: skips at
// the granularity of sub-block pairs, the fastest plan on the 128^3 ABC case
static constexpr int kDefaultPlan = 1;
// XCD chunk of the batched gather until fla_set_batch_plan or
// fla_autotune_batch chooses one, and the candidates the autotuner tries
static constexpr int kDefaultChunk = 16;
static constexpr int kChunkChoices[FLA_BATCH_CHUNKS] = {1, 4, 16, 64};

namespace {

struct Fail {
    fla_status st;
};

#define FLA_EXPORT __attribute__((visibility("default")))

#define CHECK_ARG(cond, msg)                    \
    do {                                        \
        if (!(cond)) {                          \
            ctx->err = std::string(msg);        \
            return FLA_ERR_INVALID_ARG;         \
        }                                       \
    } while (0)

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            ctx->err = std::string("HIP error in ") + #expr + ": " + hipGetErrorString(_e); \
            return _e == hipErrorOutOfMemory ? FLA_ERR_OUT_OF_MEMORY : FLA_ERR_DEVICE;      \
        }                                                                                  \
    } while (0)

// Carves aligned sub-buffers out of one device allocation.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T> T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Device allocation made for a context (honours the FLA_FAIL_ALLOC testing aid).
hipError_t dev_malloc(fla_ctx* ctx, void** p, size_t bytes)
{
    if (ctx->fail_alloc > 0 && --ctx->fail_alloc == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

// Entry-point line of the launch log: the call, a short description of its
// arguments, its status and the host time it took.
struct TraceCall {
    const fla_ctx* ctx;
    const char* name;
    std::string what;
    std::chrono::steady_clock::time_point t0;
    TraceCall(const fla_ctx* c, const char* n) : ctx(c), name(n)
    {
        if (g_trace) t0 = std::chrono::steady_clock::now();
    }
    fla_status done(fla_status st)
    {
        if (g_trace) {
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            std::fprintf(stderr, "[flaproj] call %s %s -> %d (%.3f ms host)%s%s\n", name, what.c_str(), (int)st, ms,
                         st != FLA_OK && ctx ? ": " : "", st != FLA_OK && ctx ? ctx->err.c_str() : "");
            std::fflush(stderr);
        }
        return st;
    }
};

std::string traj_desc(const fla_trajectories* t)
{
    if (!t) return "traj=NULL";
    return "N=" + std::to_string(t->count) + (t->prec == FLA_F64 ? " f64" : " f32");
}
std::string mesh_desc(const fla_mesh* m)
{
    if (!m) return "mesh=NULL";
    std::string r = "mesh=" + std::to_string(m->n[0]) + "x" + std::to_string(m->n[1]);
    if (m->dim == 3) r += "x" + std::to_string(m->n[2]);
    return r;
}

fla_status ensure_ws(fla_ctx* ctx, size_t need)
{
    if (need <= ctx->ws_size) return FLA_OK;
    if (ctx->ws) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            ctx->err = std::string("hipDeviceSynchronize: ") + hipGetErrorString(e);
            return FLA_ERR_DEVICE;
        }
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    size_t sz = need + need / 4 + (1 << 20);
    hipError_t e = dev_malloc(ctx, &ctx->ws, sz);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        ctx->err = "workspace allocation of " + std::to_string(sz) + " bytes failed: " + hipGetErrorString(e);
        return FLA_ERR_OUT_OF_MEMORY;
    }
    ctx->ws_size = sz;
    return FLA_OK;
}

fla_status ensure_tws(fla_ctx* ctx, size_t need)
{
    if (need <= ctx->tws_size) return FLA_OK;
    if (ctx->tws) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            ctx->err = std::string("hipDeviceSynchronize: ") + hipGetErrorString(e);
            return FLA_ERR_DEVICE;
        }
        (void)hipFree(ctx->tws);
        ctx->tws = nullptr;
        ctx->tws_size = 0;
    }
    size_t sz = need + need / 4 + (1 << 20);
    hipError_t e = dev_malloc(ctx, &ctx->tws, sz);
    if (e != hipSuccess) {
        ctx->tws = nullptr;
        ctx->err = "training workspace allocation of " + std::to_string(sz) + " bytes failed: " + hipGetErrorString(e);
        return FLA_ERR_OUT_OF_MEMORY;
    }
    ctx->tws_size = sz;
    return FLA_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

// Records a pair of events around one stage when profiling is on.
struct StageTimer {
    fla_ctx* ctx;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(fla_ctx* c, int st, hipStream_t str) : ctx(c), stage(st), s(str)
    {
        if (!ctx->prof) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~StageTimer()
    {
        if (!a) return;
        (void)hipEventRecord(b, s);
        ctx->recs.push_back({stage, a, b});
    }
};

fla_status check_mesh(fla_ctx* ctx, const fla_mesh* mesh, MeshDev* md, int te)
{
    CHECK_ARG(mesh != nullptr, "mesh is NULL");
    CHECK_ARG(mesh->dim == 2 || mesh->dim == 3, "mesh.dim must be 2 or 3");
    MeshDev m{};
    m.dim = mesh->dim;
    m.te = te;
    int64_t M = 1, NT = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < mesh->dim) {
            CHECK_ARG(mesh->n[a] >= 1 && mesh->n[a] <= (1 << 24), "mesh.n out of range");
            CHECK_ARG(is_fin(mesh->lo[a]) && is_fin(mesh->hi[a]) && mesh->hi[a] > mesh->lo[a],
                      "mesh.lo/hi must be finite with hi > lo");
            m.n[a] = mesh->n[a];
            m.periodic[a] = mesh->periodic[a] ? 1 : 0;
            m.lo[a] = mesh->lo[a];
            m.hi[a] = mesh->hi[a];
            m.L[a] = mesh->hi[a] - mesh->lo[a];
            m.w[a] = m.L[a] / (double)mesh->n[a];
            CHECK_ARG(m.w[a] > 0.0 && is_fin(m.w[a]), "mesh cell width is not a positive finite number");
            m.nt[a] = (mesh->n[a] + te - 1) / te;
            m.edges[a] = mesh->edges[a];
        } else {
            m.n[a] = 1;
            m.periodic[a] = 0;
            m.lo[a] = 0.0;
            m.hi[a] = 1.0;
            m.L[a] = 1.0;
            m.w[a] = 1.0;
            m.nt[a] = 1;
        }
        M *= m.n[a];
        NT *= m.nt[a];
    }
    CHECK_ARG(M <= (int64_t(1) << 31), "mesh has more than 2^31 cells");
    CHECK_ARG(NT * kClasses + 1 < (int64_t(1) << 31), "mesh has too many tiles");
    m.M = M;
    m.ntiles = (int)NT;
    m.vol = 1.0;
    for (int a = 0; a < mesh->dim; ++a) m.vol *= m.w[a];
    *md = m;
    return FLA_OK;
}

bool has_edges(const fla_mesh* mesh)
{
    for (int a = 0; a < mesh->dim; ++a)
        if (mesh->edges[a]) return true;
    return false;
}

fla_status check_traj(fla_ctx* ctx, const fla_trajectories* t, int dim, bool need_J, TrajDev* td)
{
    CHECK_ARG(t != nullptr, "trajectories is NULL");
    CHECK_ARG(t->count >= 0 && t->count < (int64_t(1) << 31), "count must be in [0, 2^31)");
    CHECK_ARG(t->prec == FLA_F32 || t->prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    TrajDev d{};
    d.count = t->count;
    if (t->count > 0) {
        for (int a = 0; a < dim; ++a) {
            CHECK_ARG(t->x[a] && t->v[a] && t->ug[a], "x, v and ug must be non-NULL for every axis");
            d.x[a] = t->x[a];
            d.v[a] = t->v[a];
            d.ug[a] = t->ug[a];
        }
        CHECK_ARG(t->r != nullptr, "r is NULL");
        if (need_J) {
            CHECK_ARG(t->J != nullptr, "J is NULL");
            CHECK_ARG(t->n0 != nullptr || is_fin(t->n0_scalar), "n0_scalar must be finite when n0 is NULL");
        }
    }
    d.J = t->J;
    d.r = t->r;
    d.n0 = t->n0;
    d.n0_scalar = t->n0_scalar;
    d.seed_volume = t->seed_volume;
    *td = d;
    return FLA_OK;
}

fla_status check_fields(fla_ctx* ctx, const fla_fields* out, int dim)
{
    CHECK_ARG(out != nullptr, "out is NULL");
    CHECK_ARG(out->S_mass != nullptr, "out.S_mass is NULL");
    for (int a = 0; a < dim; ++a) CHECK_ARG(out->S_mom[a] != nullptr, "out.S_mom[a] is NULL for an axis a < dim");
    return FLA_OK;
}

template <typename R>
fla_status zero_outputs(fla_ctx* ctx, const MeshDev& m, const fla_fields* out, hipStream_t s)
{
    HIP_OK(launch_fill_real<R>((R*)out->S_mass, m.M, s));
    for (int a = 0; a < m.dim; ++a) HIP_OK(launch_fill_real<R>((R*)out->S_mom[a], m.M, s));
    if (out->den) HIP_OK(launch_fill_real<R>((R*)out->den, m.M, s));
    if (out->pairs) HIP_OK(launch_fill_u32(out->pairs, m.M, 0u, s));
    return FLA_OK;
}

int bits_for(uint64_t maxval)
{
    int b = 0;
    while (b < 32 && (uint64_t(1) << b) <= maxval) ++b;
    return b;
}

// fixed: a caller-provided workspace of fixed_size bytes (the allocation-free
// entry point) instead of the context's grow-only one
// prod: the trajectory producer advances the droplets and emits the records
// in place of the prepass (fla_advance_project)
template <typename R, int D>
fla_status project_impl(fla_ctx* ctx, const MeshDev& m, const TrajDev& t, const fla_params* p,
                        const fla_mesh* mesh, const fla_fields* out, hipStream_t s, void* fixed = nullptr,
                        size_t fixed_size = 0, const ProduceArgs* prod = nullptr)
{
    const int64_t N = t.count;
    const int deposit = p->mode == FLA_DEPOSIT;
    const uint32_t nb = (uint32_t)kClasses * (uint32_t)m.ntiles;
    const int key_bits = bits_for(nb);
    const int64_t hist_w = radix_hist_words(N);
    const int64_t scan_w = scan_tmp_words(hist_w > (int64_t)nb + 1 ? hist_w : (int64_t)nb + 1);
    const int C = D + 1;

    auto layout = [&](Carver& c, uint32_t** keys, uint32_t** vals, uint32_t** keys2, uint32_t** vals2,
                      double4** rpos_u, double4** rpos, R** rw_u, R** rw, double** qd, uint32_t** bstart,
                      uint32_t** hist, uint32_t** scan, uint32_t** tcost, int** order, uint32_t** queue) {
        *keys = c.take<uint32_t>(N);
        *vals = c.take<uint32_t>(N);
        *keys2 = c.take<uint32_t>(N);
        *vals2 = c.take<uint32_t>(N);
        *rpos_u = c.take<double4>(N);
        *rpos = c.take<double4>(N);
        *rw_u = c.take<R>((size_t)N * kRecW);
        *rw = c.take<R>((size_t)N * kRecW);
        *qd = c.take<double>(deposit ? (size_t)N * C : 1);
        *bstart = c.take<uint32_t>(nb + 1);
        *hist = c.take<uint32_t>(hist_w > 0 ? hist_w : 1);
        *scan = c.take<uint32_t>(scan_w);
        *tcost = c.take<uint32_t>(m.ntiles > 0 ? m.ntiles : 1);
        *order = c.take<int>(m.ntiles > 0 ? 2 * (size_t)m.ntiles : 1);
        *queue = c.take<uint32_t>(kXcds);
    };
    uint32_t *keys, *vals, *keys2, *vals2, *bstart, *hist, *scan, *tcost, *queue;
    int* order;
    double4 *rpos_u, *rpos;
    R *rw_u, *rw;
    double* qd;
    {
        Carver probe(nullptr);
        layout(probe, &keys, &vals, &keys2, &vals2, &rpos_u, &rpos, &rw_u, &rw, &qd, &bstart, &hist, &scan, &tcost,
               &order, &queue);
        if (fixed) {
            CHECK_ARG(probe.off + 256 <= fixed_size,
                      "these inputs need " + std::to_string(probe.off + 256) +
                          " bytes of workspace, more than the fixed " + std::to_string(fixed_size) +
                          " bytes of fla_project_sources_noalloc");
        } else {
            fla_status st = ensure_ws(ctx, probe.off + 256);
            if (st != FLA_OK) return st;
        }
    }
    Carver c(fixed ? fixed : ctx->ws);
    layout(c, &keys, &vals, &keys2, &vals2, &rpos_u, &rpos, &rw_u, &rw, &qd, &bstart, &hist, &scan, &tcost, &order,
           &queue);

    PhysDev ph{p->rho_d, p->mu, p->delta, p->h0, p->cutoff, p->scale};
    HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
    HIP_OK(launch_fill_u64(ctx->stats + ST_TRAJ, 1, (unsigned long long)N, s));
    {
        StageTimer tm(ctx, 0, s);
        if (prod)
            HIP_OK((launch_produce<R, D>(*prod, m, ph, p->h_factor, deposit, keys, vals, rpos_u, rw_u, qd, ctx->stats,
                                         s)));
        else
            HIP_OK((launch_prepass<R, D>(t, m, ph, p->h_factor, deposit, keys, vals, rpos_u, rw_u, qd, ctx->stats, s)));
    }
    bool in_alt = false;
    uint32_t *skeys, *svals;
    {
        StageTimer tm(ctx, 1, s);
        HIP_OK(radix_sort_pairs(keys, vals, keys2, vals2, N, key_bits, hist, hist_w, scan, scan_w, s, &in_alt));
        skeys = in_alt ? keys2 : keys;
        svals = in_alt ? vals2 : vals;
        HIP_OK(launch_bucket_bounds(skeys, N, nb, bstart, s));
        HIP_OK(launch_max_class(bstart, m.ntiles, ctx->stats, s));
        HIP_OK(launch_permute<R>(svals, N, rpos_u, rw_u, rpos, rw, deposit ? 0 : 1, s));
    }
    if (deposit) {
        StageTimer tm(ctx, 2, s);
        HIP_OK((launch_deposit_norm<R, D>(m, ph, bstart + nb, svals, qd, N, rpos, rw, ctx->stats, s)));
    }

    GatherArgs g{};
    g.m = m;
    g.rpos = rpos;
    g.rw = rw;
    g.bstart = bstart;
    g.cutoff = p->cutoff;
    double cf = p->cutoff * (1.0 + kSupportMargin);
    g.filt2 = cf * cf;
    g.scale = p->scale;
    g.cell_scale = mesh->cell_scale;
    g.out[0] = out->S_mass;
    for (int a = 0; a < D; ++a) g.out[1 + a] = out->S_mom[a];
    g.den = out->den;
    g.pairs = out->pairs;
    g.stats = ctx->stats;
    g.tile_cost = tcost;
    g.order = order;
    g.queue = queue;
    HIP_OK(hipDeviceGetAttribute(&g.ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    {
        StageTimer tm(ctx, 3, s);
        int plan = ctx->plan[D - 2][sizeof(R) == 8 ? 1 : 0];
        if (plan < 0) plan = kDefaultPlan;
        if (out->pairs) HIP_OK(launch_fill_u32(out->pairs, m.M, 0u, s));
        HIP_OK((launch_gather<R, D>(g, p->mode, p->count_pairs != 0 || out->pairs != nullptr, plan, s)));
    }
    return FLA_OK;
}

void drop_single_graph(fla_ctx* ctx)
{
    if (ctx->sgraph_exec) (void)hipGraphExecDestroy(ctx->sgraph_exec);
    if (ctx->sgraph) (void)hipGraphDestroy(ctx->sgraph);
    ctx->sgraph_exec = nullptr;
    ctx->sgraph = nullptr;
    ctx->sgraph_key.clear();
    ctx->sgraph_seen.clear();
}

void drop_graph(fla_ctx* ctx)
{
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
}

// Batched projection (see fla_project_batch).  md, td: validated snapshots.
template <typename R, int D>
fla_status batch_impl(fla_ctx* ctx, int nsnap, const MeshDev* md, const TrajDev* td, const fla_params* ps,
                      const fla_mesh* meshes, const fla_fields* outs, hipStream_t s, int plan, int chunk,
                      bool use_graph)
{
    constexpr int TE = Geo<D>::TE;
    // work-list order: estimated candidates per tile (trajectory density
    // times the volume within reach of a tile at the initial bandwidth),
    // largest first; ties keep the caller's order
    std::vector<double> cost(nsnap);
    for (int i = 0; i < nsnap; ++i) {
        double vol = 1.0, reach = 1.0;
        for (int a = 0; a < D; ++a) {
            vol *= md[i].L[a];
            reach *= TE * md[i].w[a] + 2.0 * ps[i].cutoff * ps[i].h0;
        }
        cost[i] = (double)td[i].count / vol * reach;
    }
    std::vector<int> order(nsnap);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

    std::vector<BatchItem> items(nsnap);
    std::memset((void*)items.data(), 0, sizeof(BatchItem) * nsnap);
    int64_t total = 0, nbk = 0, nwork = 0;
    bool count = false;
    for (int j = 0; j < nsnap; ++j) {
        const int i = order[j];
        BatchItem& it = items[j];
        it.t = td[i];
        it.ph = PhysDev{ps[i].rho_d, ps[i].mu, ps[i].delta, ps[i].h0, ps[i].cutoff, ps[i].scale};
        it.hfac = ps[i].h_factor;
        it.base = total;
        it.key_base = (uint32_t)nbk;
        it.tile_base = (int)nwork;
        total += td[i].count;
        nbk += (int64_t)kClasses * md[i].ntiles;
        nwork += md[i].ntiles;
        count = count || ps[i].count_pairs != 0 || outs[i].pairs != nullptr;
        CHECK_ARG(total < (int64_t(1) << 31), "the batch holds 2^31 or more trajectories");
        CHECK_ARG(nbk < (int64_t(1) << 31) - 1, "the batch meshes hold too many tiles");
    }
    const uint32_t nb = (uint32_t)nbk;
    const int key_bits = bits_for(nb);
    int ncu = 0;
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int64_t hist_w = radix_hist_words(total);
    const int64_t scan_w = scan_tmp_words(hist_w > (int64_t)nb + 1 ? hist_w : (int64_t)nb + 1);
    const int64_t n1 = total > 0 ? total : 1;

    uint32_t *keys, *vals, *keys2, *vals2, *bstart, *hist, *scan, *queue;
    double4 *rpos_u, *rpos;
    R *rw_u, *rw;
    auto layout = [&](Carver& c) {
        queue = c.take<uint32_t>(kXcds);
        keys = c.take<uint32_t>(n1);
        vals = c.take<uint32_t>(n1);
        keys2 = c.take<uint32_t>(n1);
        vals2 = c.take<uint32_t>(n1);
        rpos_u = c.take<double4>(n1);
        rpos = c.take<double4>(n1);
        rw_u = c.take<R>((size_t)n1 * kRecW);
        rw = c.take<R>((size_t)n1 * kRecW);
        bstart = c.take<uint32_t>((size_t)nb + 1);
        hist = c.take<uint32_t>(hist_w > 0 ? hist_w : 1);
        scan = c.take<uint32_t>(scan_w);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    layout(c);
    const double cf0 = 1.0 + kSupportMargin;
    for (int j = 0; j < nsnap; ++j) {
        const int i = order[j];
        GatherArgs& g = items[j].g;
        g.m = md[i];
        g.rpos = rpos;
        g.rw = rw;
        g.bstart = bstart + items[j].key_base;
        g.cutoff = ps[i].cutoff;
        const double cf = ps[i].cutoff * cf0;
        g.filt2 = cf * cf;
        g.scale = ps[i].scale;
        g.cell_scale = meshes[i].cell_scale;
        g.out[0] = outs[i].S_mass;
        for (int a = 0; a < D; ++a) g.out[1 + a] = outs[i].S_mom[a];
        g.den = outs[i].den;
        g.pairs = outs[i].pairs;
        g.stats = ctx->stats;
    }

    // the arguments a captured graph depends on
    std::vector<unsigned char> key;
    auto put = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        key.insert(key.end(), b, b + n);
    };
    const int shape[6] = {nsnap, D, (int)sizeof(R), plan, chunk, count ? 1 : 0};
    put(shape, sizeof(shape));
    put(&s, sizeof(s));
    put(items.data(), sizeof(BatchItem) * nsnap);

    if (use_graph && ctx->graph_exec && key == ctx->graph_key) {
        HIP_OK(hipGraphLaunch(ctx->graph_exec, s));
        HIP_OK(hipEventRecord(ctx->items_done, s));
        ctx->items_pending = true;
        ++ctx->graph_replays;
        return FLA_OK;
    }

    // a new snapshot table: wait until no earlier batch call can read the old one
    if (ctx->items_pending) HIP_OK(hipEventSynchronize(ctx->items_done));
    ctx->items_pending = false;
    drop_graph(ctx);
    const size_t isz = sizeof(BatchItem) * (size_t)nsnap;
    if (isz > ctx->items_size) {
        if (ctx->items) HIP_OK(hipFree(ctx->items));
        ctx->items = nullptr;
        ctx->items_size = 0;
        hipError_t e = dev_malloc(ctx, &ctx->items, isz);
        if (e != hipSuccess) {
            ctx->items = nullptr;
            ctx->err = std::string("snapshot table allocation failed: ") + hipGetErrorString(e);
            return FLA_ERR_OUT_OF_MEMORY;
        }
        ctx->items_size = isz;
    }
    HIP_OK(hipMemcpy(ctx->items, items.data(), isz, hipMemcpyHostToDevice));
    if (!ctx->items_done) HIP_OK(hipEventCreateWithFlags(&ctx->items_done, hipEventDisableTiming));
    const BatchItem* dev_items = (const BatchItem*)ctx->items;
    const uint32_t sentinel = nb;

    auto enqueue = [&](hipStream_t q) -> fla_status {
        HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, q));
        HIP_OK(launch_fill_u64(ctx->stats + ST_TRAJ, 1, (unsigned long long)total, q));
        {
            StageTimer tm(ctx, 0, q);
            HIP_OK((launch_prepass_batch<R, D>(dev_items, nsnap, total, sentinel, keys, vals, rpos_u, rw_u, ctx->stats,
                                               q)));
        }
        {
            StageTimer tm(ctx, 1, q);
            bool in_alt = false;
            HIP_OK(radix_sort_pairs(keys, vals, keys2, vals2, total, key_bits, hist, hist_w, scan, scan_w, q, &in_alt));
            const uint32_t* skeys = in_alt ? keys2 : keys;
            const uint32_t* svals = in_alt ? vals2 : vals;
            HIP_OK(launch_bucket_bounds(skeys, total, nb, bstart, q));
            HIP_OK(launch_max_class_batch(dev_items, nsnap, bstart, ctx->stats, q));
            HIP_OK(launch_permute<R>(svals, total, rpos_u, rw_u, rpos, rw, 1, q));
        }
        for (int i = 0; i < nsnap; ++i)
            if (outs[i].pairs) HIP_OK(launch_fill_u32(outs[i].pairs, md[i].M, 0u, q));
        {
            StageTimer tm(ctx, 3, q);
            bool general = false;     // any rectilinear axis in the batch
            for (int i = 0; i < nsnap; ++i)
                for (int a = 0; a < 3; ++a) general = general || md[i].edges[a] != nullptr;
            HIP_OK((launch_gather_batch<R, D>(dev_items, nsnap, (int)nwork, chunk, count, plan, general, queue,
                                              ncu, q)));
        }
        return FLA_OK;
    };

    if (use_graph) {
        if (!ctx->capture) HIP_OK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        HIP_OK(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        const fla_status st = enqueue(ctx->capture);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
        if (st != FLA_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (st != FLA_OK) return st;
            ctx->err = std::string("graph capture failed: ") + hipGetErrorString(e);
            return FLA_ERR_DEVICE;
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            ctx->err = std::string("graph instantiation failed: ") + hipGetErrorString(ei);
            return FLA_ERR_DEVICE;
        }
        ctx->graph = graph;
        ctx->graph_exec = exec;
        ctx->graph_key.swap(key);
        HIP_OK(hipGraphLaunch(exec, s));
    } else {
        const fla_status st = enqueue(s);
        if (st != FLA_OK) return st;
    }
    HIP_OK(hipEventRecord(ctx->items_done, s));
    ctx->items_pending = true;
    return FLA_OK;
}

template <typename R, int D>
fla_status psicell_impl(fla_ctx* ctx, const MeshDev& m, const TrajDev& t, double weight, const fla_params* p,
                        const fla_mesh* mesh, const fla_fields* out, hipStream_t s)
{
    const int C = D + 1;
    PsiArgs a{};
    constexpr bool f64 = sizeof(R) == 8;
    auto ntiles_of = [&](const int* t) {
        int64_t nt = 1;
        for (int ax = 0; ax < D; ++ax) nt *= (m.n[ax] + t[ax] - 1) / t[ax];
        return nt;
    };
    // direct: tiles as large as one workgroup's LDS sums allow (16^3 cells,
    // 64^2 in 2-D; half that for binary64, whose sums take two words), when
    // the mesh needs at most kPsiMaxBins of them; otherwise coarse tiles of
    // kPsiMaxCellsPerTile cells (16 x 8 x 8, 32^2 in 2-D; 8^3 for binary64
    // in 3-D) grouped into bins of kPsiTilesPerBin
    const int ptd[3] = {D == 3 ? 16 : 64, D == 3 ? 16 : (f64 ? 32 : 64), D == 3 ? (f64 ? 8 : 16) : 1};
    int max_lds = 0;
    HIP_OK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    const int64_t lds_direct = (int64_t)(8 * C * PsiWords<R>::value + 4) * ptd[0] * ptd[1] * ptd[2];
    const bool direct = ntiles_of(ptd) <= kPsiMaxBins && lds_direct <= max_lds;
    int pt[3] = {D == 3 ? (f64 ? 8 : 16) : 32, D == 3 ? 8 : 32, D == 3 ? 8 : 1};
    if (direct)
        for (int ax = 0; ax < 3; ++ax) pt[ax] = ptd[ax];
    auto ntiles = [&]() { return ntiles_of(pt); };
    CHECK_ARG(ntiles() <= kPsiMaxTiles, sizeof(R) == 8 && D == 3
                                            ? "psicell_accumulate supports at most 16384 * 512 cells in binary64 3-D"
                                            : "psicell_accumulate supports at most 16384 * 1024 cells");
    for (int ax = 0; ax < 3; ++ax) {
        a.pt[ax] = ax < D ? pt[ax] : 1;
        a.pnt[ax] = ax < D ? (m.n[ax] + pt[ax] - 1) / pt[ax] : 1;
    }
    a.pntiles = (int)ntiles();
    a.cpt = a.pt[0] * a.pt[1] * a.pt[2];
    for (int ax = 0; ax < 3; ++ax) a.ptlog[ax] = __builtin_ctz((unsigned)a.pt[ax]);
    a.cptlog = a.ptlog[0] + a.ptlog[1] + a.ptlog[2];
    a.nblocks = kPsiBlocks;
    a.direct = direct ? 1 : 0;
    a.binlog = direct ? 0 : kPsiTilesPerBinLog;
    a.pnbins = direct ? a.pntiles : (a.pntiles + kPsiTilesPerBin - 1) / kPsiTilesPerBin;
    // about 2048 workgroups in the tile pass
    a.nsplit = a.pnbins >= 2048 ? 1 : 2048 / a.pnbins;
    const int64_t N = t.count;
    const int64_t hw = (int64_t)a.pntiles * a.nblocks + 1;
    const int64_t hb = direct ? 1 : (int64_t)a.pnbins * a.nblocks + 1;
    const int64_t sw = scan_tmp_words(hw > hb ? hw : hb);
    auto layout = [&](Carver& c) {
        a.maxbits = c.take<unsigned long long>(4);
        a.qscale = c.take<double>(5);
        a.codes = c.take<int>(N > 0 ? N : 1);
        a.blockhist = c.take<unsigned int>(hw);
        a.binhist = c.take<unsigned int>(hb);
        a.tcursor = c.take<unsigned int>(a.pntiles);
        a.binned = c.take<PsiRec<R>>(direct || N <= 0 ? 1 : N);
        a.bucket = c.take<PsiRec<R>>(N > 0 ? N : 1);
        if (direct) {
            // the scatter's bins are the tiles: their counts, and their buckets
            a.binhist = a.blockhist;
            a.binned = a.bucket;
        }
        a.blockmax = c.take<unsigned long long>((size_t)a.nblocks * 4);
        a.scan_tmp = c.take<uint32_t>(sw);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    layout(c);
    a.scan_words = sw;
    HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
    HIP_OK(launch_fill_u64(ctx->stats + ST_TRAJ, 1, (unsigned long long)t.count, s));
    a.m = m;
    a.p = t;
    a.ph = PhysDev{p->rho_d, p->mu, p->delta, p->h0, p->cutoff, p->scale};
    a.weight = weight;
    a.cell_scale = mesh->cell_scale;
    a.out[0] = out->S_mass;
    for (int ax = 0; ax < D; ++ax) a.out[1 + ax] = out->S_mom[ax];
    a.den = out->den;
    a.stats = ctx->stats;
    {
        StageTimer tm(ctx, 4, s);
        HIP_OK((launch_psicell<R, D>(a, s)));
    }
    return FLA_OK;
}

template <typename R, int D>
fla_status cic_impl(fla_ctx* ctx, const MeshDev& m, const TrajDev& t, double weight, const fla_params* p,
                    const fla_mesh* mesh, const fla_fields* out, hipStream_t s)
{
    constexpr int C = D + 1;
    constexpr int W = PsiWords<R>::value;
    PsiArgs a{};
    // tiles of power-of-two edges whose upper halo fits the LDS sums:
    // 16 x 8 x 8 (binary64: 8^3) in 3-D, 32^2 (binary64: 32 x 16) in 2-D;
    // or, sorted, the larger tiles 16 x 16 x 8 (binary64: 16 x 8 x 8) in 3-D,
    // 64^2 (binary64: 64 x 32) in 2-D, when the mesh needs at most
    // kCicMaxBins of them and the device allows their LDS sums
    const bool f64 = sizeof(R) == 8;
    auto tiles_of = [&](const int* t) {
        int64_t n = 1;
        for (int ax = 0; ax < D; ++ax) n *= (m.n[ax] + t[ax] - 1) / t[ax];
        return n;
    };
    const int pts[3] = {D == 3 ? 16 : 64, D == 3 ? (f64 ? 8 : 16) : (f64 ? 32 : 64), D == 3 ? 8 : 1};
    int max_lds = 0;
    HIP_OK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    const int64_t halo_s = (int64_t)(pts[0] + 1) * (pts[1] + 1) * (D == 3 ? pts[2] + 1 : 1);
    const bool sorted = tiles_of(pts) <= kCicMaxBins && halo_s * (W * (C + 1)) * 8 <= max_lds;
    int pt[3] = {D == 3 ? (f64 ? 8 : 16) : 32, D == 3 ? 8 : (f64 ? 16 : 32), D == 3 ? 8 : 1};
    if (sorted)
        for (int ax = 0; ax < 3; ++ax) pt[ax] = pts[ax];
    const int64_t nt = tiles_of(pt);
    CHECK_ARG(nt <= kPsiMaxTiles, f64 ? "cic_accumulate supports at most 16384 * 512 cells in binary64"
                                      : "cic_accumulate supports at most 16384 * 1024 cells");
    for (int ax = 0; ax < 3; ++ax) {
        a.pt[ax] = ax < D ? pt[ax] : 1;
        a.pnt[ax] = ax < D ? (m.n[ax] + pt[ax] - 1) / pt[ax] : 1;
        a.ptlog[ax] = __builtin_ctz((unsigned)a.pt[ax]);
    }
    a.pntiles = (int)nt;
    a.cpt = a.pt[0] * a.pt[1] * a.pt[2];
    a.cptlog = a.ptlog[0] + a.ptlog[1] + a.ptlog[2];
    a.nblocks = kPsiBlocks;
    a.direct = sorted ? 1 : 0;
    const int64_t N = t.count;
    const int64_t hw = (int64_t)a.pntiles * a.nblocks + 1;
    const int64_t sw = scan_tmp_words(hw);
    auto layout = [&](Carver& c) {
        a.maxbits = c.take<unsigned long long>(4);
        a.qscale = c.take<double>(5);
        a.codes = c.take<int>(N > 0 ? N : 1);
        a.blockhist = c.take<unsigned int>(hw);
        a.tcursor = c.take<unsigned int>(a.pntiles);
        a.bucket = c.take<CicRec<R>>(N > 0 ? N : 1);
        a.blockmax = c.take<unsigned long long>((size_t)a.nblocks * 4);
        a.acc = c.take<unsigned long long>((size_t)(W * (C + 1)) * (size_t)m.M);
        a.scan_tmp = c.take<uint32_t>(sw);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    layout(c);
    a.scan_words = sw;
    HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
    HIP_OK(launch_fill_u64(ctx->stats + ST_TRAJ, 1, (unsigned long long)t.count, s));
    a.m = m;
    a.p = t;
    a.ph = PhysDev{p->rho_d, p->mu, p->delta, p->h0, p->cutoff, p->scale};
    a.weight = weight;
    a.cell_scale = mesh->cell_scale;
    a.out[0] = out->S_mass;
    for (int ax = 0; ax < D; ++ax) a.out[1 + ax] = out->S_mom[ax];
    a.den = out->den;
    a.stats = ctx->stats;
    {
        StageTimer tm(ctx, 4, s);
        HIP_OK((launch_cic<R, D>(a, s)));
    }
    return FLA_OK;
}

template <typename R, int D>
fla_status bandwidth_forward_impl(fla_ctx* ctx, const MeshDev& m, const TrajDev& t, const float* theta, float* hfac,
                                  float* z, float* o, float* fraw, hipStream_t s)
{
    unsigned int* cnt;
    uint4* zb;
    {
        Carver probe(nullptr);
        probe.take<unsigned int>(2 * (size_t)m.M);
        probe.take<uint4>(t.count > 0 ? t.count : 1);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    cnt = c.take<unsigned int>(2 * (size_t)m.M);   // counts, then their box sums
    zb = c.take<uint4>(t.count > 0 ? t.count : 1);
    StageTimer tm(ctx, 5, s);
    HIP_OK((launch_bandwidth_forward<R, D>(t, m, theta, cnt, zb, hfac, z, o, fraw, s)));
    return FLA_OK;
}

template <typename R, int D>
fla_status project_backward_impl(fla_ctx* ctx, const MeshDev& m, const TrajDev& t, const fla_params* p,
                                 const fla_mesh* mesh, const fla_fields* S, const fla_fields* G, float* out,
                                 hipStream_t s)
{
    const int64_t N = t.count;
    uint32_t *keys, *vals;
    double4* rpos;
    R* rw;
    float *bpl, *epl;
    auto layout = [&](Carver& c) {
        keys = c.take<uint32_t>(N > 0 ? N : 1);
        vals = c.take<uint32_t>(N > 0 ? N : 1);
        rpos = c.take<double4>(N > 0 ? N : 1);
        rw = c.take<R>((size_t)(N > 0 ? N : 1) * kRecW);
        bpl = c.take<float>((size_t)4 * m.M);   // four floats per cell (float4 aligned)
        epl = c.take<float>(m.M);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    layout(c);
    PhysDev ph{p->rho_d, p->mu, p->delta, p->h0, p->cutoff, p->scale};
    HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
    StageTimer tm(ctx, 6, s);
    if (N > 0)
        HIP_OK((launch_prepass<R, D>(t, m, ph, p->h_factor, 0, keys, vals, rpos, rw, nullptr, ctx->stats, s)));
    Planes Sp{{S->S_mass, S->S_mom[0], S->S_mom[1], S->S_mom[2]}};
    Planes Gp{{G->S_mass, G->S_mom[0], G->S_mom[1], G->S_mom[2]}};
    const uint32_t sentinel = (uint32_t)kClasses * (uint32_t)m.ntiles;
    HIP_OK((launch_traj_backward<R, D>(m, p->cutoff, keys, sentinel, rpos, rw, Sp, S->den, Gp, p->scale,
                                       mesh->cell_scale, bpl, epl, out, N, s)));
    return FLA_OK;
}

fla_status check_params(fla_ctx* ctx, const fla_params* p, bool projection)
{
    CHECK_ARG(p != nullptr, "params is NULL");
    CHECK_ARG(is_fin(p->rho_d) && p->rho_d > 0.0, "rho_d must be positive and finite");
    CHECK_ARG(is_fin(p->mu) && p->mu > 0.0, "mu must be positive and finite");
    CHECK_ARG(is_fin(p->delta), "delta must be finite");
    if (projection) {
        CHECK_ARG(is_fin(p->h0) && p->h0 > 0.0, "h0 must be positive and finite");
        CHECK_ARG(is_fin(p->cutoff) && p->cutoff > 0.0 && p->cutoff < 1.0e3, "cutoff must be in (0, 1000)");
        CHECK_ARG(is_fin(p->scale), "scale must be finite");
        CHECK_ARG(p->mode == FLA_NW || p->mode == FLA_DEPOSIT, "mode must be FLA_NW or FLA_DEPOSIT");
    }
    return FLA_OK;
}

// Validates a batch and runs it with the given plan and chunk (-1: the
// context's choice) and launch form.
fla_status batch_entry(fla_ctx* ctx, int nsnap, const fla_mesh* meshes, const fla_trajectories* trajs,
                       const fla_params* params, const fla_fields* outs, void* stream, int plan, int chunk,
                       bool use_graph)
{
    CHECK_ARG(nsnap >= 1 && nsnap <= FLA_BATCH_MAX, "nsnap must be in [1, FLA_BATCH_MAX]");
    CHECK_ARG(meshes && trajs && params && outs, "meshes, trajs, params and outs are required");
    const int dim = meshes[0].dim;
    const int prec = trajs[0].prec;
    std::vector<MeshDev> md(nsnap);
    std::vector<TrajDev> td(nsnap);
    for (int k = 0; k < nsnap; ++k) {
        fla_status st = check_mesh(ctx, &meshes[k], &md[k], meshes[k].dim == 2 ? Geo<2>::TE : Geo<3>::TE);
        if (st == FLA_OK && meshes[k].dim != dim) {
            ctx->err = "all snapshots must have the same mesh.dim";
            st = FLA_ERR_INVALID_ARG;
        }
        if (st == FLA_OK) st = check_traj(ctx, &trajs[k], dim, true, &td[k]);
        if (st == FLA_OK && trajs[k].prec != prec) {
            ctx->err = "all snapshots must have the same prec";
            st = FLA_ERR_INVALID_ARG;
        }
        if (st == FLA_OK) st = check_params(ctx, &params[k], true);
        if (st == FLA_OK && params[k].mode != FLA_NW) {
            ctx->err = "fla_project_batch supports FLA_NW only";
            st = FLA_ERR_INVALID_ARG;
        }
        if (st == FLA_OK) st = check_fields(ctx, &outs[k], dim);
        if (st != FLA_OK) {
            ctx->err = "snapshot " + std::to_string(k) + ": " + ctx->err;
            return st;
        }
    }
    HIP_OK(hipSetDevice(ctx->device));
    const int d = dim - 2;
    if (plan < 0) plan = ctx->batch_plan[d][prec] < 0 ? kDefaultPlan : ctx->batch_plan[d][prec];
    if (chunk < 0) chunk = ctx->batch_chunk[d][prec] < 0 ? kDefaultChunk : ctx->batch_chunk[d][prec];
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = prec == FLA_F64;
    if (dim == 2)
        return f64 ? batch_impl<double, 2>(ctx, nsnap, md.data(), td.data(), params, meshes, outs, s, plan, chunk,
                                           use_graph)
                   : batch_impl<float, 2>(ctx, nsnap, md.data(), td.data(), params, meshes, outs, s, plan, chunk,
                                          use_graph);
    return f64 ? batch_impl<double, 3>(ctx, nsnap, md.data(), td.data(), params, meshes, outs, s, plan, chunk,
                                       use_graph)
               : batch_impl<float, 3>(ctx, nsnap, md.data(), td.data(), params, meshes, outs, s, plan, chunk,
                                      use_graph);
}

}  // namespace

static void drop_records(fla_ctx* ctx);
static fla_status project_entry(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                const fla_params* params, const fla_fields* out, void* stream, void* fixed,
                                size_t fixed_size);

extern "C" {

FLA_EXPORT fla_status fla_ctx_create(fla_ctx** out, int device)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return FLA_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
        return FLA_ERR_DEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_error = "device index out of range";
        return FLA_ERR_INVALID_ARG;
    }
    fla_ctx* ctx = new (std::nothrow) fla_ctx();
    if (!ctx) {
        g_create_error = "host allocation failed";
        return FLA_ERR_OUT_OF_MEMORY;
    }
    ctx->device = device;
    if (const char* t = std::getenv("FLA_TRACE")) g_trace = std::atoi(t) != 0 || t[0] == 'y';
    if (const char* f = std::getenv("FLA_FAIL_ALLOC")) ctx->fail_alloc = std::atoll(f);
    e = hipSetDevice(device);
    if (e == hipSuccess && device < kMaxScratchDevices) {
        // device address of this GPU's copy of the fixed workspace (once per GPU)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e == hipSuccess && ptr) g_scratch_ptr[device] = ptr;
        }
    }
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->stats, sizeof(unsigned long long) * ST_N);
    if (e == hipSuccess) e = hipMemset(ctx->stats, 0, sizeof(unsigned long long) * ST_N);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        g_create_error = std::string("HIP initialisation failed: ") + hipGetErrorString(e);
        if (ctx->stats) (void)hipFree(ctx->stats);
        delete ctx;
        return FLA_ERR_DEVICE;
    }
    *out = ctx;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_ctx_destroy(fla_ctx* ctx)
{
    if (!ctx) return FLA_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    drop_records(ctx);
    drop_graph(ctx);
    drop_single_graph(ctx);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->items_done) (void)hipEventDestroy(ctx->items_done);
    if (ctx->items) (void)hipFree(ctx->items);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->tws) (void)hipFree(ctx->tws);
    if (ctx->stats) (void)hipFree(ctx->stats);
    delete ctx;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_project_sources(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                               const fla_params* params, const fla_fields* out, void* stream)
{
    TraceCall tc(ctx, "fla_project_sources");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        return project_entry(ctx, mesh, traj, params, out, stream, nullptr, 0);
    }());
}

FLA_EXPORT fla_status fla_project_sources_noalloc(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                                  const fla_params* params, const fla_fields* out, void* stream)
{
    TraceCall tc(ctx, "fla_project_sources_noalloc");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        void* ptr = nullptr;
        if (ctx->device >= 0 && ctx->device < kMaxScratchDevices) {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            ptr = g_scratch_ptr[ctx->device];
        }
        if (!ptr) {
            ctx->err = "fla_project_sources_noalloc: no fixed workspace on this device";
            return FLA_ERR_UNSUPPORTED;
        }
        // no profiling events here: creating them is an allocation
        const bool prof = ctx->prof;
        ctx->prof = false;
        const fla_status st = project_entry(ctx, mesh, traj, params, out, stream, ptr, FLA_NOALLOC_SCRATCH_BYTES);
        ctx->prof = prof;
        return st;
    }());
}

}  // extern "C"

static fla_status project_entry(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                const fla_params* params, const fla_fields* out, void* stream, void* fixed,
                                size_t fixed_size)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    try {
        MeshDev m;
        fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
        if (st != FLA_OK) return st;
        CHECK_ARG(!(params && params->mode == FLA_DEPOSIT && has_edges(mesh)),
                  "FLA_DEPOSIT needs a uniform mesh (divides by one cell volume); edges were given");
        TrajDev t;
        st = check_traj(ctx, traj, m.dim, true, &t);
        if (st != FLA_OK) return st;
        st = check_params(ctx, params, true);
        if (st != FLA_OK) return st;
        st = check_fields(ctx, out, m.dim);
        if (st != FLA_OK) return st;
        if (params->mode == FLA_DEPOSIT)
            CHECK_ARG(is_fin(traj->seed_volume) && traj->seed_volume > 0.0,
                      "seed_volume must be positive and finite in FLA_DEPOSIT mode");
        HIP_OK(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        bool f64 = traj->prec == FLA_F64;
        if (t.count == 0) {
            HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
            return f64 ? zero_outputs<double>(ctx, m, out, s) : zero_outputs<float>(ctx, m, out, s);
        }
        auto run = [&](hipStream_t q) -> fla_status {
            if (m.dim == 2)
                return f64 ? project_impl<double, 2>(ctx, m, t, params, mesh, out, q, fixed, fixed_size)
                           : project_impl<float, 2>(ctx, m, t, params, mesh, out, q, fixed, fixed_size);
            return f64 ? project_impl<double, 3>(ctx, m, t, params, mesh, out, q, fixed, fixed_size)
                       : project_impl<float, 3>(ctx, m, t, params, mesh, out, q, fixed, fixed_size);
        };
        // single-call graphs: not on a fixed workspace, while profiling (stage
        // events) or while tracing (a replay launches nothing the log sees)
        if (!ctx->single_graph || fixed || ctx->prof || g_trace) return run(s);
        auto make_key = [&]() {
            std::vector<unsigned char> k;
            auto put = [&](const void* p, size_t n) {
                const unsigned char* b = (const unsigned char*)p;
                k.insert(k.end(), b, b + n);
            };
            put(mesh, sizeof(*mesh));
            put(traj, sizeof(*traj));
            put(params, sizeof(*params));
            put(out, sizeof(*out));
            put(&s, sizeof(s));
            put(&ctx->ws, sizeof(ctx->ws));
            put(&ctx->plan[m.dim - 2][traj->prec], sizeof(int));
            return k;
        };
        std::vector<unsigned char> key = make_key();
        if (ctx->sgraph_exec && key == ctx->sgraph_key) {
            HIP_OK(hipGraphLaunch(ctx->sgraph_exec, s));
            ++ctx->graph_replays;
            return FLA_OK;
        }
        if (key != ctx->sgraph_seen) {
            // a new set of arguments runs directly once (it may grow the
            // workspace, which a capture must not do); its key is taken after
            // the call, with the workspace it left
            const fla_status dst = run(s);
            if (dst == FLA_OK) ctx->sgraph_seen = make_key();
            return dst;
        }
        // the same arguments again: capture, keep and launch
        drop_single_graph(ctx);
        if (!ctx->capture) HIP_OK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        HIP_OK(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        const fla_status cst = run(ctx->capture);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
        if (cst != FLA_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (cst != FLA_OK) return cst;
            ctx->err = std::string("graph capture failed: ") + hipGetErrorString(e);
            return FLA_ERR_DEVICE;
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            ctx->err = std::string("graph instantiation failed: ") + hipGetErrorString(ei);
            return FLA_ERR_DEVICE;
        }
        ctx->sgraph = graph;
        ctx->sgraph_exec = exec;
        ctx->sgraph_key.swap(key);
        HIP_OK(hipGraphLaunch(exec, s));
        return FLA_OK;
    } catch (...) {
        ctx->err = "internal error";
        return FLA_ERR_DEVICE;
    }
}

extern "C" {

FLA_EXPORT fla_status psicell_accumulate(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* particles,
                              double particle_weight, const fla_params* params, const fla_fields* out,
                              void* stream)
{
    TraceCall tc(ctx, "psicell_accumulate");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(particles);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev m;
            fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!has_edges(mesh), "rectilinear mesh edges are taken by the FLA_NW projection only");
            TrajDev t;
            st = check_traj(ctx, particles, m.dim, false, &t);
            if (st != FLA_OK) return st;
            st = check_params(ctx, params, false);
            if (st != FLA_OK) return st;
            st = check_fields(ctx, out, m.dim);
            if (st != FLA_OK) return st;
            CHECK_ARG(is_fin(particle_weight), "particle_weight must be finite");
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            bool f64 = particles->prec == FLA_F64;
            if (m.dim == 2)
                return f64 ? psicell_impl<double, 2>(ctx, m, t, particle_weight, params, mesh, out, s)
                           : psicell_impl<float, 2>(ctx, m, t, particle_weight, params, mesh, out, s);
            return f64 ? psicell_impl<double, 3>(ctx, m, t, particle_weight, params, mesh, out, s)
                       : psicell_impl<float, 3>(ctx, m, t, particle_weight, params, mesh, out, s);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status cic_accumulate(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* particles,
                                     double particle_weight, const fla_params* params, const fla_fields* out,
                                     void* stream)
{
    TraceCall tc(ctx, "cic_accumulate");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(particles);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev m;
            fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!has_edges(mesh), "rectilinear mesh edges are taken by the FLA_NW projection only");
            TrajDev t;
            st = check_traj(ctx, particles, m.dim, false, &t);
            if (st != FLA_OK) return st;
            st = check_params(ctx, params, false);
            if (st != FLA_OK) return st;
            st = check_fields(ctx, out, m.dim);
            if (st != FLA_OK) return st;
            CHECK_ARG(is_fin(particle_weight), "particle_weight must be finite");
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            bool f64 = particles->prec == FLA_F64;
            if (m.dim == 2)
                return f64 ? cic_impl<double, 2>(ctx, m, t, particle_weight, params, mesh, out, s)
                           : cic_impl<float, 2>(ctx, m, t, particle_weight, params, mesh, out, s);
            return f64 ? cic_impl<double, 3>(ctx, m, t, particle_weight, params, mesh, out, s)
                       : cic_impl<float, 3>(ctx, m, t, particle_weight, params, mesh, out, s);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status fla_get_stats(fla_ctx* ctx, fla_stats* out)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    CHECK_ARG(out != nullptr, "out is NULL");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipDeviceSynchronize());
    unsigned long long h[ST_N];
    HIP_OK(hipMemcpy(h, ctx->stats, sizeof(h), hipMemcpyDeviceToHost));
    out->trajectories = (int64_t)h[ST_TRAJ];
    out->skipped = (int64_t)h[ST_SKIPPED];
    out->no_support = (int64_t)h[ST_NOSUPPORT];
    out->pairs = (int64_t)h[ST_PAIRS];
    out->outside = (int64_t)h[ST_OUTSIDE];
    out->zero_support = (int64_t)h[ST_ZERO];
    out->max_class = (int64_t)h[ST_MAXCLASS];
    out->graph_replays = ctx->graph_replays;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_bandwidth_forward(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                            const float* theta, float* h_factor, float* z, float* o, float* features,
                                            void* stream)
{
    TraceCall tc(ctx, "fla_bandwidth_forward");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev m;
            fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!has_edges(mesh), "rectilinear mesh edges are taken by the FLA_NW projection only");
            TrajDev t;
            st = check_traj(ctx, traj, m.dim, true, &t);
            if (st != FLA_OK) return st;
            CHECK_ARG(theta != nullptr, "theta is NULL");
            CHECK_ARG(h_factor != nullptr || t.count == 0, "h_factor is NULL");
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            bool f64 = traj->prec == FLA_F64;
            if (m.dim == 2)
                return f64 ? bandwidth_forward_impl<double, 2>(ctx, m, t, theta, h_factor, z, o, features, s)
                           : bandwidth_forward_impl<float, 2>(ctx, m, t, theta, h_factor, z, o, features, s);
            return f64 ? bandwidth_forward_impl<double, 3>(ctx, m, t, theta, h_factor, z, o, features, s)
                       : bandwidth_forward_impl<float, 3>(ctx, m, t, theta, h_factor, z, o, features, s);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status fla_project_backward(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                           const fla_params* params, const fla_fields* S, const fla_fields* dL_dS,
                                           float* dL_dlogh, void* stream)
{
    TraceCall tc(ctx, "fla_project_backward");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev m;
            fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!has_edges(mesh), "rectilinear mesh edges are taken by the FLA_NW projection only");
            TrajDev t;
            st = check_traj(ctx, traj, m.dim, true, &t);
            if (st != FLA_OK) return st;
            st = check_params(ctx, params, true);
            if (st != FLA_OK) return st;
            CHECK_ARG(params->mode == FLA_NW, "fla_project_backward differentiates the FLA_NW estimator");
            st = check_fields(ctx, S, m.dim);
            if (st != FLA_OK) return st;
            CHECK_ARG(S->den != nullptr, "S.den is required");
            st = check_fields(ctx, dL_dS, m.dim);
            if (st != FLA_OK) return st;
            CHECK_ARG(dL_dlogh != nullptr || t.count == 0, "dL_dlogh is NULL");
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            bool f64 = traj->prec == FLA_F64;
            if (m.dim == 2)
                return f64 ? project_backward_impl<double, 2>(ctx, m, t, params, mesh, S, dL_dS, dL_dlogh, s)
                           : project_backward_impl<float, 2>(ctx, m, t, params, mesh, S, dL_dS, dL_dlogh, s);
            return f64 ? project_backward_impl<double, 3>(ctx, m, t, params, mesh, S, dL_dS, dL_dlogh, s)
                       : project_backward_impl<float, 3>(ctx, m, t, params, mesh, S, dL_dS, dL_dlogh, s);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status fla_bandwidth_backward(fla_ctx* ctx, int dim, const float* theta, int64_t count, const float* z,
                                             const float* o, const float* dL_dlogh, float* grad, void* stream)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(dim == 2 || dim == 3, "dim must be 2 or 3");
    CHECK_ARG(count >= 0 && count < (int64_t(1) << 31), "count out of range");
    CHECK_ARG(theta && grad, "theta and grad are required");
    CHECK_ARG(count == 0 || (z && o && dL_dlogh), "z, o and dL_dlogh are required");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int nb = mlp_backward_blocks(count);
    float* partial;
    {
        Carver probe(nullptr);
        probe.take<float>((size_t)nb * kTrain);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    partial = c.take<float>((size_t)nb * kTrain);
    StageTimer tm(ctx, 7, s);
    if (dim == 2)
        HIP_OK((launch_mlp_backward<2>(theta, count, z, o, dL_dlogh, partial, nb, grad, s)));
    else
        HIP_OK((launch_mlp_backward<3>(theta, count, z, o, dL_dlogh, partial, nb, grad, s)));
    return FLA_OK;
}

FLA_EXPORT fla_status fla_adam_step(fla_ctx* ctx, float* theta, float* m, float* v, const float* grad, int64_t step,
                                    double lr, double beta1, double beta2, double eps, void* stream)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(theta && m && v && grad, "theta, m, v and grad are required");
    CHECK_ARG(step >= 1, "step counts from 1");
    CHECK_ARG(is_fin(lr) && lr >= 0.0 && beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0,
              "invalid Adam hyper-parameters");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(launch_adam(theta, m, v, grad, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return FLA_OK;
}

FLA_EXPORT fla_status fla_rel_l2_loss(fla_ctx* ctx, int channels, int64_t cells, int prec, const fla_fields* S,
                                      const fla_fields* R, const fla_fields* dL_dS, double* result, void* stream)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(channels >= 1 && channels <= 4, "channels must be 1..4");
    CHECK_ARG(cells >= 1, "cells must be positive");
    CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    CHECK_ARG(S && R && result, "S, R and result are required");
    const void* sp[4] = {S->S_mass, S->S_mom[0], S->S_mom[1], S->S_mom[2]};
    const void* rp[4] = {R->S_mass, R->S_mom[0], R->S_mom[1], R->S_mom[2]};
    for (int k = 0; k < channels; ++k) CHECK_ARG(sp[k] && rp[k], "a field plane of S or R is NULL");
    MutPlanes G{{nullptr, nullptr, nullptr, nullptr}};
    if (dL_dS) {
        void* gp[4] = {dL_dS->S_mass, dL_dS->S_mom[0], dL_dS->S_mom[1], dL_dS->S_mom[2]};
        for (int k = 0; k < channels; ++k) CHECK_ARG(gp[k], "a field plane of dL_dS is NULL");
        for (int k = 0; k < 4; ++k) G.p[k] = gp[k];
    }
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    double* part;
    {
        Carver probe(nullptr);
        probe.take<double>(256 * 8);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    part = c.take<double>(256 * 8);
    Planes Sp{{sp[0], sp[1], sp[2], sp[3]}}, Rp{{rp[0], rp[1], rp[2], rp[3]}};
    if (prec == FLA_F64)
        HIP_OK(launch_loss<double>(channels, cells, Sp, Rp, G, dL_dS != nullptr, part, result, s));
    else
        HIP_OK(launch_loss<float>(channels, cells, Sp, Rp, G, dL_dS != nullptr, part, result, s));
    return FLA_OK;
}

static void drop_records(fla_ctx* ctx)
{
    for (auto& r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->recs.clear();
}

FLA_EXPORT fla_status fla_profile_enable(fla_ctx* ctx, int on)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    HIP_OK(hipSetDevice(ctx->device));
    if (!ctx->recs.empty()) {
        HIP_OK(hipDeviceSynchronize());
        drop_records(ctx);
    }
    ctx->prof = on != 0;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_profile_read(fla_ctx* ctx, fla_profile* out)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    CHECK_ARG(out != nullptr, "out is NULL");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipDeviceSynchronize());
    for (int k = 0; k < FLA_PROFILE_STAGES; ++k) {
        out->ms[k] = 0.0;
        out->launches[k] = 0;
    }
    for (auto& r : ctx->recs) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.stage >= 0 && r.stage < FLA_PROFILE_STAGES) {
            out->ms[r.stage] += (double)ms;
            out->launches[r.stage] += 1;
        }
    }
    return FLA_OK;
}

// gather plan codes of a dimension: plan + kGatherPlans * shape
static_assert(FLA_GATHER_PLANS == kGatherPlans && FLA_GATHER_SHAPES == kGatherShapes, "plan codes of the header");
static int plan_codes(int dim) { return dim == 3 ? gather_plan_codes<3>() : gather_plan_codes<2>(); }

FLA_EXPORT fla_status fla_set_plan(fla_ctx* ctx, int dim, int prec, int gather_plan)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(dim == 2 || dim == 3, "dim must be 2 or 3");
    CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    CHECK_ARG(gather_plan >= -1 && gather_plan < plan_codes(dim), "gather_plan out of range");
    ctx->plan[dim - 2][prec] = gather_plan;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_get_plan(fla_ctx* ctx, int dim, int prec, int* gather_plan)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(dim == 2 || dim == 3, "dim must be 2 or 3");
    CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    CHECK_ARG(gather_plan != nullptr, "gather_plan is NULL");
    int p = ctx->plan[dim - 2][prec];
    *gather_plan = p < 0 ? kDefaultPlan : p;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_autotune(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                   const fla_params* params, const fla_fields* out, void* stream,
                                   double* times_ms)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(mesh && traj && params && out, "NULL argument");
    CHECK_ARG(mesh->dim == 2 || mesh->dim == 3, "mesh.dim must be 2 or 3");
    CHECK_ARG(traj->prec == FLA_F32 || traj->prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int d = mesh->dim - 2, pr = traj->prec;
    const int saved = ctx->plan[d][pr];
    const bool was_prof = ctx->prof;
    fla_status st = fla_profile_enable(ctx, 1);
    if (st != FLA_OK) return st;
    double best = 1e300;
    int best_plan = saved < 0 ? kDefaultPlan : saved;
    if (times_ms)
        for (int k = 0; k < FLA_GATHER_CONFIGS; ++k) times_ms[k] = -1.0;
    for (int plan = 0; plan < plan_codes(mesh->dim); ++plan) {
        ctx->plan[d][pr] = plan;
        // first call warms the workspace, the second is timed
        for (int rep = 0; rep < 2; ++rep) {
            if (rep == 1) {
                st = fla_profile_enable(ctx, 1);
                if (st != FLA_OK) break;
            }
            st = fla_project_sources(ctx, mesh, traj, params, out, stream);
            if (st != FLA_OK) break;
        }
        if (st != FLA_OK) break;
        fla_profile pf;
        st = fla_profile_read(ctx, &pf);
        if (st != FLA_OK) break;
        double ms = pf.launches[3] ? pf.ms[3] / (double)pf.launches[3] : 1e300;
        if (times_ms) times_ms[plan] = ms;
        if (ms < best) {
            best = ms;
            best_plan = plan;
        }
    }
    (void)fla_profile_enable(ctx, was_prof ? 1 : 0);
    if (st != FLA_OK) {
        ctx->plan[d][pr] = saved;
        return st;
    }
    ctx->plan[d][pr] = best_plan;
    (void)s;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_project_batch(fla_ctx* ctx, int nsnap, const fla_mesh* meshes,
                                        const fla_trajectories* trajs, const fla_params* params,
                                        const fla_fields* outs, void* stream)
{
    TraceCall tc(ctx, "fla_project_batch");
    if (g_trace) tc.what = "nsnap=" + std::to_string(nsnap);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            return batch_entry(ctx, nsnap, meshes, trajs, params, outs, stream, -1, -1, ctx->batch_graph && !ctx->prof);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status fla_set_graph(fla_ctx* ctx, int enable)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipDeviceSynchronize());
    drop_single_graph(ctx);
    ctx->single_graph = enable != 0;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_set_batch_graph(fla_ctx* ctx, int enable)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->items_pending) HIP_OK(hipEventSynchronize(ctx->items_done));
    ctx->items_pending = false;
    drop_graph(ctx);
    ctx->batch_graph = enable != 0;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_set_batch_plan(fla_ctx* ctx, int dim, int prec, int gather_plan, int chunk)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(dim == 2 || dim == 3, "dim must be 2 or 3");
    CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    CHECK_ARG(gather_plan >= -1 && gather_plan < plan_codes(dim), "gather_plan out of range");
    CHECK_ARG(gather_plan == -1 || (chunk >= 1 && chunk <= 4096), "chunk must be in [1, 4096]");
    ctx->batch_plan[dim - 2][prec] = gather_plan;
    ctx->batch_chunk[dim - 2][prec] = gather_plan < 0 ? -1 : chunk;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_get_batch_plan(fla_ctx* ctx, int dim, int prec, int* gather_plan, int* chunk)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(dim == 2 || dim == 3, "dim must be 2 or 3");
    CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    CHECK_ARG(gather_plan != nullptr && chunk != nullptr, "gather_plan and chunk are required");
    const int p = ctx->batch_plan[dim - 2][prec], c = ctx->batch_chunk[dim - 2][prec];
    *gather_plan = p < 0 ? kDefaultPlan : p;
    *chunk = c < 0 ? kDefaultChunk : c;
    return FLA_OK;
}

// Architecture name of the context's device (the key of saved plans).
static fla_status device_arch(fla_ctx* ctx, std::string& arch)
{
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, ctx->device));
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);   // target features do not change the plans
    if (arch.empty()) arch = "unknown";
    return FLA_OK;
}

static const char* kPlansHeader = "flaproj-plans 1";

FLA_EXPORT fla_status fla_save_plans(fla_ctx* ctx, const char* path)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(path != nullptr, "path is NULL");
    std::string arch;
    fla_status st = device_arch(ctx, arch);
    if (st != FLA_OK) return st;
    FILE* f = std::fopen(path, "w");
    CHECK_ARG(f != nullptr, std::string("cannot open ") + path + " for writing");
    std::fprintf(f, "%s\n", kPlansHeader);
    for (int d = 0; d < 2; ++d)
        for (int pr = 0; pr < 2; ++pr)
            std::fprintf(f, "%s %d %d %d %d %d\n", arch.c_str(), d + 2, pr, ctx->plan[d][pr], ctx->batch_plan[d][pr],
                         ctx->batch_chunk[d][pr]);
    const bool ok = std::fflush(f) == 0 && !std::ferror(f);
    std::fclose(f);
    CHECK_ARG(ok, std::string("cannot write ") + path);
    return FLA_OK;
}

FLA_EXPORT fla_status fla_load_plans(fla_ctx* ctx, const char* path)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(path != nullptr, "path is NULL");
    std::string arch;
    fla_status st = device_arch(ctx, arch);
    if (st != FLA_OK) return st;
    FILE* f = std::fopen(path, "r");
    CHECK_ARG(f != nullptr, std::string("cannot open ") + path);
    struct Entry {
        int d, pr, plan, bplan, chunk;
    };
    std::vector<Entry> take;
    char line[512];
    bool header = false, bad = false;
    while (std::fgets(line, sizeof(line), f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (l.empty()) continue;
        if (!header) {
            header = l == kPlansHeader;
            if (!header) bad = true;
            if (bad) break;
            continue;
        }
        char a[256];
        int dim, pr, plan, bplan, chunk;
        char extra;
        if (std::sscanf(l.c_str(), "%255s %d %d %d %d %d %c", a, &dim, &pr, &plan, &bplan, &chunk, &extra) != 6 ||
            (dim != 2 && dim != 3) || (pr != FLA_F32 && pr != FLA_F64) || plan < -1 || plan >= plan_codes(dim) ||
            bplan < -1 || bplan >= plan_codes(dim) || (bplan >= 0 && (chunk < 1 || chunk > 4096))) {
            bad = true;
            break;
        }
        if (arch == a) take.push_back({dim - 2, pr, plan, bplan, bplan < 0 ? -1 : chunk});
    }
    std::fclose(f);
    CHECK_ARG(header && !bad, std::string(path) + " is not a plan file of this library (nothing was changed)");
    for (const Entry& e : take) {
        ctx->plan[e.d][e.pr] = e.plan;
        ctx->batch_plan[e.d][e.pr] = e.bplan;
        ctx->batch_chunk[e.d][e.pr] = e.chunk;
    }
    return FLA_OK;
}

FLA_EXPORT fla_status fla_autotune_batch(fla_ctx* ctx, int nsnap, const fla_mesh* meshes,
                                         const fla_trajectories* trajs, const fla_params* params,
                                         const fla_fields* outs, void* stream, double* times_ms)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    CHECK_ARG(nsnap >= 1 && meshes && trajs, "meshes and trajs are required");
    CHECK_ARG(meshes[0].dim == 2 || meshes[0].dim == 3, "mesh.dim must be 2 or 3");
    CHECK_ARG(trajs[0].prec == FLA_F32 || trajs[0].prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
    const int d = meshes[0].dim - 2, pr = trajs[0].prec;
    const bool was_prof = ctx->prof;
    double best = 1e300;
    int best_plan = -1, best_chunk = -1;
    fla_status st = FLA_OK;
    try {
        if (times_ms)
            for (int k = 0; k < FLA_GATHER_CONFIGS * FLA_BATCH_CHUNKS; ++k) times_ms[k] = -1.0;
        for (int plan = 0; plan < plan_codes(meshes[0].dim) && st == FLA_OK; ++plan)
            for (int ci = 0; ci < FLA_BATCH_CHUNKS && st == FLA_OK; ++ci) {
                // first call warms the workspace, the second is timed
                st = fla_profile_enable(ctx, 0);
                if (st == FLA_OK)
                    st = batch_entry(ctx, nsnap, meshes, trajs, params, outs, stream, plan, kChunkChoices[ci], false);
                if (st == FLA_OK) st = fla_profile_enable(ctx, 1);
                if (st == FLA_OK)
                    st = batch_entry(ctx, nsnap, meshes, trajs, params, outs, stream, plan, kChunkChoices[ci], false);
                fla_profile pf;
                if (st == FLA_OK) st = fla_profile_read(ctx, &pf);
                if (st != FLA_OK) break;
                const double ms = pf.launches[3] ? pf.ms[3] / (double)pf.launches[3] : 1e300;
                if (times_ms) times_ms[plan * FLA_BATCH_CHUNKS + ci] = ms;
                if (ms < best) {
                    best = ms;
                    best_plan = plan;
                    best_chunk = kChunkChoices[ci];
                }
            }
    } catch (...) {
        ctx->err = "internal error";
        st = FLA_ERR_DEVICE;
    }
    const std::string err = ctx->err;
    (void)fla_profile_enable(ctx, was_prof ? 1 : 0);
    ctx->err = err;
    if (st != FLA_OK) return st;
    ctx->batch_plan[d][pr] = best_plan;
    ctx->batch_chunk[d][pr] = best_chunk;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_advance_project(fla_ctx* ctx, const fla_mesh* mesh, const fla_droplets* drops,
                                          const fla_flow* flow, const fla_step* step, const fla_params* params,
                                          int prec, const fla_fields* out, void* stream)
{
    TraceCall tc(ctx, "fla_advance_project");
    if (g_trace) tc.what = mesh_desc(mesh) + (drops ? " N=" + std::to_string(drops->count) : std::string(" drops=NULL"));
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev m;
            fla_status st = check_mesh(ctx, mesh, &m, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!(params && params->mode == FLA_DEPOSIT && has_edges(mesh)),
                      "FLA_DEPOSIT needs a uniform mesh (divides by one cell volume); edges were given");
            const int D = m.dim;
            CHECK_ARG(drops != nullptr, "droplets is NULL");
            CHECK_ARG(drops->count >= 0 && drops->count < (int64_t(1) << 31), "count must be in [0, 2^31)");
            if (drops->count > 0) {
                for (int a = 0; a < D; ++a) CHECK_ARG(drops->x[a] && drops->v[a], "x and v must be non-NULL for every axis");
                CHECK_ARG(drops->J && drops->dJ && drops->r, "J, dJ and r are required");
                CHECK_ARG(drops->n0 != nullptr || is_fin(drops->n0_scalar), "n0_scalar must be finite when n0 is NULL");
            }
            CHECK_ARG(flow != nullptr, "flow is NULL");
            CHECK_ARG(flow->kind == FLA_FLOW_NONE || (flow->kind == FLA_FLOW_TAYLOR_GREEN && D == 2) ||
                          (flow->kind == FLA_FLOW_ABC && D == 3),
                      "flow.kind must be FLA_FLOW_NONE, FLA_FLOW_TAYLOR_GREEN (2-D) or FLA_FLOW_ABC (3-D)");
            bool fin = is_fin(flow->U) && is_fin(flow->k);
            for (int a = 0; a < 3; ++a) fin = fin && is_fin(flow->abc[a]) && is_fin(flow->phase[a]) && is_fin(flow->u0[a]);
            for (int e = 0; e < 9; ++e) fin = fin && is_fin(flow->G[e]);
            CHECK_ARG(fin, "flow parameters must be finite");
            CHECK_ARG(step != nullptr, "step is NULL");
            CHECK_ARG(is_fin(step->dt) && step->dt > 0.0, "step.dt must be positive and finite");
            CHECK_ARG(step->substeps >= 1 && step->substeps <= (1 << 20), "step.substeps must be in [1, 2^20]");
            CHECK_ARG(prec == FLA_F32 || prec == FLA_F64, "prec must be FLA_F32 or FLA_F64");
            st = check_params(ctx, params, true);
            if (st != FLA_OK) return st;
            st = check_fields(ctx, out, D);
            if (st != FLA_OK) return st;
            if (params->mode == FLA_DEPOSIT)
                CHECK_ARG(is_fin(drops->seed_volume) && drops->seed_volume > 0.0,
                          "seed_volume must be positive and finite in FLA_DEPOSIT mode");
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            const bool f64 = prec == FLA_F64;
            if (drops->count == 0) {
                HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
                return f64 ? zero_outputs<double>(ctx, m, out, s) : zero_outputs<float>(ctx, m, out, s);
            }
            ProduceArgs pa{};
            pa.count = drops->count;
            for (int a = 0; a < 3; ++a) {
                pa.x[a] = a < D ? drops->x[a] : nullptr;
                pa.v[a] = a < D ? drops->v[a] : nullptr;
            }
            pa.J = drops->J;
            pa.dJ = drops->dJ;
            pa.r = drops->r;
            pa.n0 = drops->n0;
            pa.n0_scalar = drops->n0_scalar;
            pa.seed_volume = drops->seed_volume;
            pa.phibar = drops->phibar;
            pa.flow.kind = flow->kind;
            pa.flow.U = flow->U;
            pa.flow.k = flow->k;
            for (int a = 0; a < 3; ++a) {
                pa.flow.abc[a] = flow->abc[a];
                pa.flow.phase[a] = flow->phase[a];
                pa.flow.u0[a] = flow->u0[a];
            }
            for (int e = 0; e < 9; ++e) pa.flow.G[e] = flow->G[e];
            pa.dt = step->dt;
            pa.substeps = step->substeps;
            pa.update = step->update_state != 0;
            TrajDev t{};
            t.count = drops->count;
            t.n0 = drops->n0;
            t.n0_scalar = drops->n0_scalar;
            t.seed_volume = drops->seed_volume;
            if (D == 2)
                return f64 ? project_impl<double, 2>(ctx, m, t, params, mesh, out, s, nullptr, 0, &pa)
                           : project_impl<float, 2>(ctx, m, t, params, mesh, out, s, nullptr, 0, &pa);
            return f64 ? project_impl<double, 3>(ctx, m, t, params, mesh, out, s, nullptr, 0, &pa)
                       : project_impl<float, 3>(ctx, m, t, params, mesh, out, s, nullptr, 0, &pa);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT fla_status fla_bandwidth_standardise(fla_ctx* ctx, int nsnap, const fla_mesh* meshes,
                                                const fla_trajectories* trajs, float* theta, void* stream)
{
    if (!ctx) return FLA_ERR_INVALID_ARG;
    ctx->err.clear();
    try {
        CHECK_ARG(nsnap >= 1 && meshes && trajs, "nsnap >= 1 snapshots with meshes and trajs are required");
        CHECK_ARG(theta != nullptr, "theta is NULL");
        int64_t nmax = 1;
        for (int k = 0; k < nsnap; ++k) {
            MeshDev m;
            fla_status st = check_mesh(ctx, &meshes[k], &m, meshes[k].dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            TrajDev t;
            if (st == FLA_OK) st = check_traj(ctx, &trajs[k], m.dim, true, &t);
            if (st != FLA_OK) {
            CHECK_ARG(!has_edges(&meshes[k]), "rectilinear mesh edges are taken by the FLA_NW projection only");
                ctx->err = "snapshot " + std::to_string(k) + ": " + ctx->err;
                return st;
            }
            nmax = std::max<int64_t>(nmax, trajs[k].count);
        }
        HIP_OK(hipSetDevice(ctx->device));
        hipStream_t s = (hipStream_t)stream;
        float *hf, *fr;
        double *part, *acc0, *acc1;
        auto layout = [&](Carver& c) {
            hf = c.take<float>(nmax);
            fr = c.take<float>((size_t)kFeat * nmax);
            part = c.take<double>(kMomParts);
            acc0 = c.take<double>(8);
            acc1 = c.take<double>(8);
        };
        {
            Carver probe(nullptr);
            layout(probe);
            fla_status st = ensure_tws(ctx, probe.off + 256);
            if (st != FLA_OK) return st;
        }
        Carver c(ctx->tws);
        layout(c);
        HIP_OK(launch_fill_u64((unsigned long long*)acc0, 8, 0ull, s));
        HIP_OK(launch_fill_u64((unsigned long long*)acc1, 8, 0ull, s));
        // pass 0: counts and sums; pass 1: squared deviations from the mean
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < nsnap; ++k) {
                if (trajs[k].count == 0) continue;
                fla_status st = fla_bandwidth_forward(ctx, &meshes[k], &trajs[k], theta, hf, nullptr, nullptr, fr, stream);
                if (st != FLA_OK) return st;
                HIP_OK(launch_feat_moments(fr, trajs[k].count, pass, acc0, part, pass == 0 ? acc0 : acc1, s));
            }
        HIP_OK(launch_feat_finish(acc0, acc1, theta, s));
        return FLA_OK;
    } catch (...) {
        ctx->err = "internal error";
        return FLA_ERR_DEVICE;
    }
}

FLA_EXPORT fla_status fla_mlp_train_step(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                         const fla_params* params, const fla_fields* ref, float* theta, float* m,
                                         float* v, int64_t step, double lr, double beta1, double beta2, double eps,
                                         double* loss, void* stream)
{
    TraceCall tc(ctx, "fla_mlp_train_step");
    if (g_trace) tc.what = mesh_desc(mesh) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            MeshDev md;
            fla_status st = check_mesh(ctx, mesh, &md, mesh && mesh->dim == 2 ? Geo<2>::TE : Geo<3>::TE);
            if (st != FLA_OK) return st;
            CHECK_ARG(!has_edges(mesh), "rectilinear mesh edges are taken by the FLA_NW projection only");
            TrajDev td;
            st = check_traj(ctx, traj, md.dim, true, &td);
            if (st != FLA_OK) return st;
            st = check_params(ctx, params, true);
            if (st != FLA_OK) return st;
            CHECK_ARG(params->mode == FLA_NW, "fla_mlp_train_step trains on the FLA_NW estimator");
            CHECK_ARG(params->h_factor == nullptr, "params.h_factor must be NULL (the step forms the factors)");
            st = check_fields(ctx, ref, md.dim);
            if (st != FLA_OK) return st;
            CHECK_ARG(theta && m && v, "theta, m and v are required");
            CHECK_ARG(step >= 1, "step counts from 1");
            CHECK_ARG(is_fin(lr) && lr >= 0.0 && beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0,
                      "invalid Adam hyper-parameters");
            HIP_OK(hipSetDevice(ctx->device));
            const int64_t N = traj->count, M = md.M;
            const int C = md.dim + 1;
            const size_t rb = traj->prec == FLA_F64 ? 8 : 4;
            float *hf, *z, *o, *dlogh, *grad;
            unsigned char *Sp[4], *den, *Gp[4];
            double* res;
            auto layout = [&](Carver& c) {
                hf = c.take<float>(N > 0 ? N : 1);
                z = c.take<float>((size_t)kFeat * (N > 0 ? N : 1));
                o = c.take<float>(N > 0 ? N : 1);
                dlogh = c.take<float>(N > 0 ? N : 1);
                for (int k = 0; k < C; ++k) Sp[k] = c.take<unsigned char>((size_t)M * rb);
                den = c.take<unsigned char>((size_t)M * rb);
                for (int k = 0; k < C; ++k) Gp[k] = c.take<unsigned char>((size_t)M * rb);
                grad = c.take<float>(kParams);
                res = c.take<double>(1 + 2 * 4);
            };
            {
                Carver probe(nullptr);
                layout(probe);
                st = ensure_tws(ctx, probe.off + 256);
                if (st != FLA_OK) return st;
            }
            Carver c(ctx->tws);
            layout(c);
            fla_params p = *params;
            p.h_factor = hf;
            fla_fields S{}, G{};
            S.S_mass = Sp[0];
            G.S_mass = Gp[0];
            for (int a = 0; a < md.dim; ++a) {
                S.S_mom[a] = Sp[1 + a];
                G.S_mom[a] = Gp[1 + a];
            }
            S.den = den;
            // 1. features and network; 2. projection with the factors; 3. loss and
            // dL/dS; 4. estimator backward; 5. network backward; 6. Adam
            st = fla_bandwidth_forward(ctx, mesh, traj, theta, hf, z, o, nullptr, stream);
            if (st == FLA_OK) st = fla_project_sources(ctx, mesh, traj, &p, &S, stream);
            if (st == FLA_OK) st = fla_rel_l2_loss(ctx, C, M, traj->prec, &S, ref, &G, loss ? loss : res, stream);
            if (st == FLA_OK) st = fla_project_backward(ctx, mesh, traj, &p, &S, &G, dlogh, stream);
            if (st == FLA_OK) st = fla_bandwidth_backward(ctx, md.dim, theta, N, z, o, dlogh, grad, stream);
            if (st == FLA_OK) st = fla_adam_step(ctx, theta, m, v, grad, step, lr, beta1, beta2, eps, stream);
            return st;
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

FLA_EXPORT const char* fla_last_error(const fla_ctx* ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// General meshes: the cell index and the projection at centroids.
// ---------------------------------------------------------------------------
struct fla_cell_index {
    int device = 0;
    int dim = 0;
    int64_t M = 0;
    CellGridDev g{};            // edges point into `edges`
    double* edges = nullptr;    // dim * (kCellsMaxBuckets + 1) values
    double* xs[3] = {nullptr, nullptr, nullptr};
    double* vs = nullptr;       // volumes in bucket order, or NULL
    uint32_t* perm = nullptr;
    int4* work = nullptr;
    int nwork = 0;
};

namespace {

constexpr int kDefaultCellsPerBucket = 112;

void free_index(fla_cell_index* ix)
{
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    if (ix->edges) (void)hipFree(ix->edges);
    for (int a = 0; a < 3; ++a)
        if (ix->xs[a]) (void)hipFree(ix->xs[a]);
    if (ix->vs) (void)hipFree(ix->vs);
    if (ix->perm) (void)hipFree(ix->perm);
    if (ix->work) (void)hipFree(ix->work);
    delete ix;
}

fla_status cell_index_build(fla_ctx* ctx, const fla_cells* c, int32_t per_bucket, fla_cell_index* ix)
{
    const int D = c->dim;
    const int64_t M = c->count;
    const double* xc[3] = {c->centroid[0], c->centroid[1], D == 3 ? c->centroid[2] : nullptr};
    // 1. histogram of the coordinates and validation
    uint32_t *hist, *bad;
    {
        Carver probe(nullptr);
        hist = probe.take<uint32_t>((size_t)3 * kCellsHistBins);
        bad = probe.take<uint32_t>(1);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
        Carver cv(ctx->ws);
        hist = cv.take<uint32_t>((size_t)3 * kCellsHistBins);
        bad = cv.take<uint32_t>(1);
    }
    hipStream_t s = nullptr;
    HIP_OK(launch_fill_u32(hist, (int64_t)3 * kCellsHistBins, 0u, s));
    HIP_OK(launch_fill_u32(bad, 1, 0u, s));
    HIP_OK(launch_cells_hist(D, M, xc, c->lo, c->hi, hist, bad, c->volume, s));
    std::vector<uint32_t> hh((size_t)3 * kCellsHistBins);
    uint32_t nbad = 0;
    HIP_OK(hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(&nbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    CHECK_ARG(nbad == 0, std::to_string(nbad) +
                             " cells have a centroid outside the box or not finite, or a negative or "
                             "non-finite volume");
    // 2. buckets per axis: about M / per_bucket in all, shared out in
    // proportion to the box edges, then edges at the coordinate quantiles
    double Ls[3];
    for (int a = 0; a < D; ++a) Ls[a] = c->hi[a] - c->lo[a];
    const std::vector<int> nbw = host::bucket_counts(D, Ls, (double)M / (double)per_bucket, kCellsMaxBuckets);
    std::vector<double> edges[3];
    int64_t nbk = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < D)
            edges[a] = host::quantile_edges(hh.data() + (size_t)a * kCellsHistBins, kCellsHistBins, M, nbw[a],
                                            c->lo[a], c->hi[a]);
        else
            edges[a] = {0.0, 1.0};
        nbk *= (int64_t)edges[a].size() - 1;
    }
    CHECK_ARG(nbk * kClasses + 1 < (int64_t(1) << 31), "too many buckets");
    CellGridDev g{};
    g.dim = D;
    g.nbuckets = (int)nbk;
    HIP_OK(dev_malloc(ctx, (void**)&ix->edges, sizeof(double) * 3 * (kCellsMaxBuckets + 1)));
    for (int a = 0; a < 3; ++a) {
        g.nb[a] = (int)edges[a].size() - 1;
        g.periodic[a] = a < D ? (c->periodic[a] != 0) : 0;
        g.lo[a] = a < D ? c->lo[a] : 0.0;
        g.hi[a] = a < D ? c->hi[a] : 1.0;
        g.L[a] = g.hi[a] - g.lo[a];
        g.edges[a] = ix->edges + (size_t)a * (kCellsMaxBuckets + 1);
        HIP_OK(hipMemcpy((void*)g.edges[a], edges[a].data(), sizeof(double) * edges[a].size(),
                         hipMemcpyHostToDevice));
    }
    // 3. cells sorted by bucket
    uint32_t *keys, *vals, *keys2, *vals2, *rh, *scan, *cstart;
    const int64_t hist_w = radix_hist_words(M);
    const int64_t scan_w = scan_tmp_words(std::max(hist_w, nbk + 1));
    auto layout = [&](Carver& cv) {
        keys = cv.take<uint32_t>(M);
        vals = cv.take<uint32_t>(M);
        keys2 = cv.take<uint32_t>(M);
        vals2 = cv.take<uint32_t>(M);
        rh = cv.take<uint32_t>(hist_w > 0 ? hist_w : 1);
        scan = cv.take<uint32_t>(scan_w);
        cstart = cv.take<uint32_t>((size_t)nbk + 1);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver cv(ctx->ws);
    layout(cv);
    HIP_OK(launch_cells_key(g, M, xc, keys, vals, s));
    bool in_alt = false;
    HIP_OK(radix_sort_pairs(keys, vals, keys2, vals2, M, bits_for((uint64_t)nbk), rh, hist_w, scan, scan_w, s,
                            &in_alt));
    const uint32_t* skeys = in_alt ? keys2 : keys;
    const uint32_t* svals = in_alt ? vals2 : vals;
    HIP_OK(launch_bucket_bounds(skeys, M, (uint32_t)nbk, cstart, s));
    for (int a = 0; a < D; ++a) HIP_OK(dev_malloc(ctx, (void**)&ix->xs[a], sizeof(double) * M));
    if (c->volume) HIP_OK(dev_malloc(ctx, (void**)&ix->vs, sizeof(double) * M));
    HIP_OK(dev_malloc(ctx, (void**)&ix->perm, sizeof(uint32_t) * M));
    double* xsd[3] = {ix->xs[0], ix->xs[1], ix->xs[2]};
    HIP_OK(launch_cells_sorted(D, M, svals, xc, c->volume, xsd, ix->vs, ix->perm, s));
    // 4. work items: runs of at most kCellsPerItem cells of one bucket, a
    // bucket's cells shared evenly between its items
    std::vector<uint32_t> cs((size_t)nbk + 1);
    HIP_OK(hipMemcpyAsync(cs.data(), cstart, sizeof(uint32_t) * cs.size(), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int4> work;
    for (const host::WorkItem& w : host::work_items(cs.data(), nbk, kCellsPerItem))
        work.push_back(make_int4(w.bucket, w.first, w.count, 0));
    CHECK_ARG(work.size() < (size_t)(1 << 29), "too many gather work items");
    ix->nwork = (int)work.size();
    HIP_OK(dev_malloc(ctx, (void**)&ix->work, sizeof(int4) * std::max<size_t>(work.size(), 1)));
    HIP_OK(hipMemcpy(ix->work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
    HIP_OK(hipDeviceSynchronize());
    ix->g = g;
    ix->dim = D;
    ix->M = M;
    return FLA_OK;
}

template <typename R, int D>
fla_status project_cells_impl(fla_ctx* ctx, const fla_cell_index* ix, const TrajDev& t, const fla_params* p,
                              double kinj, bool use_vol, const fla_fields* out, hipStream_t s)
{
    const int64_t N = t.count;
    const uint32_t nb = (uint32_t)kClasses * (uint32_t)ix->g.nbuckets;
    const int key_bits = bits_for(nb);
    const int64_t hist_w = radix_hist_words(N);
    const int64_t scan_w = scan_tmp_words(hist_w > (int64_t)nb + 1 ? hist_w : (int64_t)nb + 1);
    uint32_t *keys, *vals, *keys2, *vals2, *bstart, *hist, *scan;
    double4 *rpos_u, *rpos;
    R *rw_u, *rw;
    auto layout = [&](Carver& c) {
        keys = c.take<uint32_t>(N);
        vals = c.take<uint32_t>(N);
        keys2 = c.take<uint32_t>(N);
        vals2 = c.take<uint32_t>(N);
        rpos_u = c.take<double4>(N);
        rpos = c.take<double4>(N);
        rw_u = c.take<R>((size_t)N * kRecW);
        rw = c.take<R>((size_t)N * kRecW);
        bstart = c.take<uint32_t>(nb + 1);
        hist = c.take<uint32_t>(hist_w > 0 ? hist_w : 1);
        scan = c.take<uint32_t>(scan_w);
    };
    {
        Carver probe(nullptr);
        layout(probe);
        fla_status st = ensure_ws(ctx, probe.off + 256);
        if (st != FLA_OK) return st;
    }
    Carver c(ctx->ws);
    layout(c);
    PhysDev ph{p->rho_d, p->mu, p->delta, p->h0, p->cutoff, p->scale};
    HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
    HIP_OK(launch_fill_u64(ctx->stats + ST_TRAJ, 1, (unsigned long long)N, s));
    {
        StageTimer tm(ctx, 0, s);
        HIP_OK((launch_cells_prepass<R, D>(t, ix->g, ph, p->h_factor, keys, vals, rpos_u, rw_u, ctx->stats, s)));
    }
    {
        StageTimer tm(ctx, 1, s);
        bool in_alt = false;
        HIP_OK(radix_sort_pairs(keys, vals, keys2, vals2, N, key_bits, hist, hist_w, scan, scan_w, s, &in_alt));
        const uint32_t* skeys = in_alt ? keys2 : keys;
        const uint32_t* svals = in_alt ? vals2 : vals;
        HIP_OK(launch_bucket_bounds(skeys, N, nb, bstart, s));
        HIP_OK(launch_max_class(bstart, ix->g.nbuckets, ctx->stats, s));
        HIP_OK(launch_permute<R>(svals, N, rpos_u, rw_u, rpos, rw, 1, s));
    }
    CellsGatherArgs a{};
    a.g = ix->g;
    for (int ax = 0; ax < 3; ++ax) a.xc[ax] = ix->xs[ax];
    a.vol = ix->vs;
    a.perm = ix->perm;
    a.work = ix->work;
    a.nwork = ix->nwork;
    a.rpos = rpos;
    a.rw = rw;
    a.bstart = bstart;
    a.cutoff = p->cutoff;
    const double cf = p->cutoff * (1.0 + kSupportMargin);
    a.filt2 = cf * cf;
    a.scale = p->scale * kinj;
    a.use_vol = use_vol ? 1 : 0;
    a.out[0] = out->S_mass;
    for (int ax = 0; ax < D; ++ax) a.out[1 + ax] = out->S_mom[ax];
    a.den = out->den;
    a.pairs = out->pairs;
    a.stats = ctx->stats;
    {
        StageTimer tm(ctx, 3, s);
        HIP_OK((launch_cells_gather<R, D>(a, p->count_pairs != 0 || out->pairs != nullptr, s)));
    }
    return FLA_OK;
}

}  // namespace

extern "C" {

FLA_EXPORT fla_status fla_cell_index_create(fla_ctx* ctx, const fla_cells* cells, int32_t cells_per_bucket,
                                            fla_cell_index** out)
{
    TraceCall tc(ctx, "fla_cell_index_create");
    if (g_trace) tc.what = (cells ? "cells=" + std::to_string(cells->count) : std::string("cells=NULL"));
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        CHECK_ARG(out != nullptr, "out is NULL");
        *out = nullptr;
        CHECK_ARG(cells != nullptr, "cells is NULL");
        CHECK_ARG(cells->dim == 2 || cells->dim == 3, "cells.dim must be 2 or 3");
        CHECK_ARG(cells->count >= 1 && cells->count < (int64_t(1) << 31), "cells.count must be in [1, 2^31)");
        for (int a = 0; a < cells->dim; ++a) {
            CHECK_ARG(is_fin(cells->lo[a]) && is_fin(cells->hi[a]) && cells->hi[a] > cells->lo[a] &&
                          is_fin(cells->hi[a] - cells->lo[a]),
                      "cells box: lo and hi must be finite with hi > lo");
            CHECK_ARG(cells->centroid[a] != nullptr, "cells.centroid[a] is NULL for an axis a < dim");
        }
        const int32_t per = cells_per_bucket <= 0 ? kDefaultCellsPerBucket : std::min(cells_per_bucket, 1 << 20);
        fla_cell_index* ix = new (std::nothrow) fla_cell_index();
        if (!ix) {
            ctx->err = "host allocation failed";
            return FLA_ERR_OUT_OF_MEMORY;
        }
        ix->device = ctx->device;
        fla_status st;
        try {
            hipError_t e = hipSetDevice(ctx->device);
            if (e != hipSuccess) {
                ctx->err = std::string("hipSetDevice: ") + hipGetErrorString(e);
                st = FLA_ERR_DEVICE;
            } else {
                st = cell_index_build(ctx, cells, per, ix);
            }
        } catch (...) {
            ctx->err = "internal error";
            st = FLA_ERR_DEVICE;
        }
        if (st != FLA_OK) {
            free_index(ix);
            return st;
        }
        *out = ix;
        return FLA_OK;
    }());
}

FLA_EXPORT fla_status fla_cell_index_destroy(fla_cell_index* index)
{
    if (!index) return FLA_OK;
    (void)hipSetDevice(index->device);
    (void)hipDeviceSynchronize();
    free_index(index);
    return FLA_OK;
}

FLA_EXPORT fla_status fla_cell_index_shape(const fla_cell_index* index, int32_t nb[3], int64_t* work_items)
{
    if (!index || !nb || !work_items) return FLA_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a) nb[a] = index->g.nb[a];
    *work_items = index->nwork;
    return FLA_OK;
}

FLA_EXPORT fla_status fla_project_cells(fla_ctx* ctx, const fla_cell_index* index, const fla_trajectories* traj,
                                        const fla_params* params, const fla_injection* inj, const fla_fields* out,
                                        void* stream)
{
    TraceCall tc(ctx, "fla_project_cells");
    if (g_trace) tc.what = (index ? "cells=" + std::to_string(index->M) : std::string("index=NULL")) + " " + traj_desc(traj);
    return tc.done([&]() -> fla_status {
        if (!ctx) return FLA_ERR_INVALID_ARG;
        ctx->err.clear();
        try {
            CHECK_ARG(index != nullptr, "index is NULL");
            CHECK_ARG(index->device == ctx->device, "the index was built on another device");
            const int D = index->dim;
            TrajDev t;
            fla_status st = check_traj(ctx, traj, D, true, &t);
            if (st != FLA_OK) return st;
            st = check_params(ctx, params, true);
            if (st != FLA_OK) return st;
            CHECK_ARG(params->mode == FLA_NW, "fla_project_cells supports FLA_NW only");
            st = check_fields(ctx, out, D);
            if (st != FLA_OK) return st;
            double kinj = 1.0;
            if (inj) {
                CHECK_ARG(is_fin(inj->n_ref) && inj->n_ref > 0.0 && is_fin(inj->tau_ref) && inj->tau_ref > 0.0 &&
                              is_fin(inj->area) && inj->area > 0.0 && is_fin(inj->v_inj) && inj->v_inj > 0.0,
                          "injection parameters must be positive and finite");
                CHECK_ARG(index->vs != nullptr, "n_hat needs cell volumes: the index was built without them");
                kinj = inj->n_ref / (inj->area * inj->v_inj * inj->tau_ref);
                CHECK_ARG(is_fin(kinj) && is_fin(kinj * params->scale), "n_hat per unit volume is not finite");
            }
            HIP_OK(hipSetDevice(ctx->device));
            hipStream_t s = (hipStream_t)stream;
            const bool f64 = traj->prec == FLA_F64;
            if (t.count == 0) {
                // no trajectory: every cell has den = 0 and S = 0
                MeshDev m{};
                m.dim = D;
                m.M = index->M;
                HIP_OK(launch_fill_u64(ctx->stats, ST_N, 0ull, s));
                return f64 ? zero_outputs<double>(ctx, m, out, s) : zero_outputs<float>(ctx, m, out, s);
            }
            if (D == 2)
                return f64 ? project_cells_impl<double, 2>(ctx, index, t, params, kinj, inj != nullptr, out, s)
                           : project_cells_impl<float, 2>(ctx, index, t, params, kinj, inj != nullptr, out, s);
            return f64 ? project_cells_impl<double, 3>(ctx, index, t, params, kinj, inj != nullptr, out, s)
                       : project_cells_impl<float, 3>(ctx, index, t, params, kinj, inj != nullptr, out, s);
        } catch (...) {
            ctx->err = "internal error";
            return FLA_ERR_DEVICE;
        }
    }());
}

}  // extern "C"
