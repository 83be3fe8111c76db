/*
 * flaproj.h - C ABI of the MI355X (gfx950) FLA source-projection library.
 *
 * The library projects the mass and momentum exchange terms carried by
 * fully-Lagrangian-approach (FLA) droplet trajectories onto an Eulerian
 * mesh (uniform Cartesian, or general: cells given by centroids and
 * volumes) with the Nadaraya-Watson kernel estimator of Stafford &
 * Rybdylova (arXiv 2512.20829), advances the droplets that carry them, and
 * accumulates the PSI-CELL box-counting and cloud-in-cell source terms of a
 * particle cloud as the comparison paths.
 *
 * Conventions shared by every entry point:
 *  - Pointers inside the argument structs are DEVICE pointers (HIP device
 *    memory of the context's device) unless marked "host".  The structs
 *    themselves are host memory and are read during the call only.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and the call returns without waiting, except where stated.
 *  - The caller owns every input and output buffer; the library never frees
 *    or retains them.  The context owns a grow-only device workspace.
 *  - Invalid arguments are detected on the host before anything is enqueued:
 *    the call returns FLA_ERR_INVALID_ARG, writes nothing and records a
 *    message readable with fla_last_error.  No C++ exception crosses the ABI.
 *  - Data-dependent conditions are not errors: trajectories with det J = 0 or
 *    any non-finite input, and PSI-CELL particles outside a closed box, are
 *    skipped and counted (fla_get_stats).
 *  - Results are deterministic: the same inputs give bitwise-identical
 *    outputs (no floating-point atomics; fixed summation orders).
 *  - Mesh cells are indexed i0 + n0*(i1 + n1*i2); a field is a plane of
 *    M = n0*n1(*n2) values in that order.
 *  - A context is used by one host thread at a time.  Its workspace and
 *    statistics are shared by every call on it, so work enqueued on
 *    different streams must not overlap in time: order such streams (or
 *    use one context per stream).  Growing the workspace synchronises the
 *    device.
 */
#ifndef FLAPROJ_H
#define FLAPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FLA_OK = 0,
    FLA_ERR_INVALID_ARG = 1,
    FLA_ERR_OUT_OF_MEMORY = 2,
    FLA_ERR_DEVICE = 3,
    FLA_ERR_UNSUPPORTED = 4
} fla_status;

/* Arithmetic of a call.  FLA_F32: velocities, radii and outputs are binary32
 * and kernel weights are evaluated in binary32 with compensated binary32
 * sums; det J, number density, smoothing length and cell offsets stay in
 * binary64.  FLA_F64: everything in binary64. */
typedef enum { FLA_F32 = 0, FLA_F64 = 1 } fla_precision;

/* FLA_NW: the Nadaraya-Watson estimator of the paper (eqs. kernel-estimator,
 * kernel, smoothing-length and coupling-terms-kernel).  FLA_DEPOSIT: the
 * normalised-kernel deposition that conserves the carried totals exactly:
 * trajectory i carries Q_i = n0_i V_seed phi_i, spread over the cells it
 * reaches with weights K_ci / Z_i, Z_i = sum_c K_ci, and the cell value is
 * divided by the cell volume; if no cell centre is within reach (Z_i = 0)
 * the whole of Q_i goes to the cell containing x_i. */
typedef enum { FLA_NW = 0, FLA_DEPOSIT = 1 } fla_mode;

typedef struct fla_ctx fla_ctx;

/* Cartesian mesh on [lo, hi) with n[a] cells along axis a; cell centres at
 * lo + (i + 1/2)(hi - lo)/n.  Periodic axes use minimum-image offsets.
 * cell_scale (nullable, device, M values in the call's precision)
 * multiplies every source term of a cell: the per-cell factor n_hat of
 * App. A, eqs. (A.13)-(A.14), on a mesh where it varies.
 * edges[a] (nullable, device, binary64): a rectilinear (stretched) axis,
 * its n[a] + 1 cell edges, strictly increasing, edges[a][0] = lo[a] and
 * edges[a][n[a]] = hi[a]; the cell centres are then the edge midpoints
 * (e[i] + e[i+1])/2.  The library reads but does not check them (memory
 * accesses stay in bounds whatever they hold).  Rectilinear axes are taken
 * by the FLA_NW projection (fla_project_sources, its allocation-free form,
 * fla_project_batch, fla_advance_project); every other entry point returns
 * FLA_ERR_INVALID_ARG for a mesh with edges. */
typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t n[3];           /* cells per axis, >= 1; n[2] ignored if dim == 2 */
    double lo[3];
    double hi[3];           /* hi[a] > lo[a] */
    int32_t periodic[3];    /* nonzero = periodic axis */
    const void* cell_scale; /* nullable */
    const double* edges[3]; /* nullable per axis: uniform */
} fla_mesh;

/* Trajectory (or particle) records, structure of arrays, count values each.
 *   x[a]   binary64 positions (eq. Stokes-drag trajectory x_d)
 *   J      binary64 deformation Jacobian dx_d/dx_0 (eq. for J), dim*dim planes:
 *          entry (a, b) of trajectory i at J[(a*dim + b)*count + i]
 *   v[a]   droplet velocity, ug[a] gas velocity at the droplet, r radius:
 *          binary32 if prec == FLA_F32, binary64 if FLA_F64
 *   n0     nullable per-trajectory initial number density n_d(x_0, t_0)
 *          (eq. FLA-COM); if NULL, n0_scalar is used for all
 *   seed_volume  volume represented by one seed, V_seed (FLA_DEPOSIT only)
 * For psicell_accumulate, J, n0 and seed_volume are ignored. */
typedef struct {
    int64_t count;          /* >= 0, < 2^31 */
    int32_t prec;           /* fla_precision */
    int32_t reserved;
    const double* x[3];
    const double* J;
    const void* v[3];
    const void* ug[3];
    const void* r;
    const double* n0;
    double n0_scalar;
    double seed_volume;
} fla_trajectories;

/* Physical and kernel parameters.
 *   rho_d   droplet density; mu gas dynamic viscosity; delta the rate of
 *           change of droplet surface area (eqs. evap-model and 5, SI units):
 *           m = 4/3 pi rho_d r^3, tau = 2 rho_d r^2/(9 mu),
 *           F = m (ug - v)/tau, mdot = 4 pi rho_d r^2 delta/(2 r)
 *   h0      initial smoothing length (eq. smoothing-length), > 0
 *   cutoff  truncation of the Gaussian kernel in bandwidths, > 0: a pair is
 *           included iff sum_a (d_a/h)^2 <= cutoff^2 (per-axis terms rounded
 *           to binary32 and summed in binary32 for FLA_F32)
 *   scale   global multiplier of every source term (n_hat of App. A when
 *           it is uniform; 1 when n0 is already physical)
 *   mode    fla_mode
 *   count_pairs  nonzero: also count included (trajectory, cell) pairs into
 *           the statistics (costs extra ALU work)
 *   h_factor nullable device binary32 array of count positive factors that
 *           multiply h_i (the learned bandwidth correction); NULL = 1 */
typedef struct {
    double rho_d;
    double mu;
    double delta;
    double h0;
    double cutoff;
    double scale;
    int32_t mode;
    int32_t count_pairs;
    const float* h_factor;
} fla_params;

/* Output fields: device planes of M values in the call's precision.
 * S_mass = S_Mass, S_mom[a] = component a of S_Mom (eq. coupling-terms-
 * kernel, with the minus sign of eq. coupling-terms-averaged); den
 * (nullable) receives the estimator denominator sum_i K(x_c, x_i)
 * (FLA_NW) or, for psicell_accumulate, the particle count as a real.
 * pairs (nullable, uint32 per cell; fla_project_sources, fla_project_batch,
 * fla_advance_project and fla_project_cells only, ignored elsewhere)
 * receives the number of
 * trajectories whose kernel reaches the cell centre (the included pairs
 * of the truncation test; in FLA_DEPOSIT a trajectory whose support holds
 * no centre counts once at its home cell).  Asking for it costs extra
 * ALU work in the gather. */
typedef struct {
    void* S_mass;
    void* S_mom[3];
    void* den;
    uint32_t* pairs;
} fla_fields;

typedef struct {
    int64_t trajectories;     /* records seen by the last call */
    int64_t skipped;          /* det J == 0 or non-finite input */
    int64_t no_support;       /* valid, but no cell of a closed box within reach */
    int64_t pairs;            /* included pairs (only if count_pairs was set or a
                                 pairs plane was given) */
    int64_t outside;          /* PSI-CELL particles outside a closed box */
    int64_t zero_support;     /* FLA_DEPOSIT: trajectories with Z_i = 0 */
    int64_t max_class;        /* largest neighbourhood class used by the gather */
    int64_t graph_replays;    /* fla_project_batch and fla_project_sources calls on this
                                 context that replayed a captured graph (host counter,
                                 never reset) */
} fla_stats;

/* Create a context on HIP device `device` (host pointer out).  Errors:
 * INVALID_ARG for a bad device or NULL out, DEVICE if HIP fails.
 * Two environment variables are read here:
 *   FLA_TRACE=1       turns on the launch log for the process (=0 turns it
 *                     off): every kernel launch (name, grid, block, LDS
 *                     bytes, stream) and every call of the main entry
 *                     points (arguments, status, host time) is written to
 *                     stderr as a line starting "[flaproj]";
 *   FLA_FAIL_ALLOC=k  testing aid for callers' error paths: the k-th device
 *                     allocation made for this context fails as if the
 *                     device were out of memory (the entry point returns
 *                     FLA_ERR_OUT_OF_MEMORY before it launches anything, so
 *                     its outputs are untouched); later allocations proceed. */
fla_status fla_ctx_create(fla_ctx** out, int device);

/* Destroy a context; waits for the device first.  NULL is accepted. */
fla_status fla_ctx_destroy(fla_ctx* ctx);

/* FLA source projection (paper: eqs. FLA-COM, smoothing-length, kernel,
 * kernel-estimator, coupling-terms-kernel; App. B steps 1c-1d and 2a-2c).
 * For every cell centre x_c, over trajectories i that are not skipped:
 *   detJ_i = det J_i (binary64), n_i = n0_i/|detJ_i|, h_i = h0 |detJ_i| f_i,
 *   q_i = n_i [mdot_i, F_i + mdot_i v_i],
 *   K_ci = (1/h_i) exp(-|x_c - x_i|^2 / (2 h_i^2)) if included, else 0,
 *   S_k(c) = -scale * cell_scale(c) * sum_i K_ci q_ik / sum_i K_ci
 *            (0 where the denominator is 0)                  [FLA_NW]
 *   S_k(c) = -scale * cell_scale(c) / V_c * sum_i Q_ik K_ci / Z_i
 *                                                            [FLA_DEPOSIT]
 * Output channels: S_mass and S_mom[0..dim-1] (all required), den optional.
 * count == 0 writes zeros.  Errors: INVALID_ARG (checked on the host),
 * OUT_OF_MEMORY (workspace), DEVICE (launch failure). */
fla_status fla_project_sources(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                               const fla_params* params, const fla_fields* out, void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results (bit for bit, under the same gather plan) and errors as
 * fla_project_sources, but the workspace is a fixed device array of
 * FLA_NOALLOC_SCRATCH_BYTES compiled into the library instead of the
 * context's grow-only workspace, so the call allocates nothing (no device
 * memory, no events; profiling does not record it).  Each GPU holds its own
 * copy of the array from the creation of the first context on it until the
 * process ends.  Inputs whose workspace would not fit (144 B per binary32
 * trajectory and 208 B per binary64 one, 8 B per channel more in
 * FLA_DEPOSIT, plus about 44 B per tile of 8^3 or 16^2 cells) return
 * FLA_ERR_INVALID_ARG with the size they need; nothing is written then.
 * Every call on one GPU, from any context or thread, shares that GPU's
 * array and its contents: calls that overlap in time on one GPU race, so
 * the caller orders them (one stream, or events).  FLA_ERR_UNSUPPORTED if
 * the context's device has no such array (device index >= 64). */
#define FLA_NOALLOC_SCRATCH_BYTES (64u << 20)
fla_status fla_project_sources_noalloc(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                       const fla_params* params, const fla_fields* out, void* stream);

/* PSI-CELL box counting (paper: eqs. vol-avg-discrete and coupling-terms-
 * definition): every particle p with finite inputs is assigned the cell
 * floor((x_p - lo)/dx) per axis (periodic axes wrap; on a closed axis
 * x == hi goes to the last cell and any other outside position is skipped
 * and counted) and
 *   S_k(c) = -(particle_weight / V_c) * cell_scale(c) * sum_{p in c} phi_pk,
 *   phi_p = [mdot_p, F_p + mdot_p v_p]   (n = 1 per droplet),
 * particle_weight being the number of real droplets one computational
 * particle stands for.  phi is evaluated in the call's precision (binary32
 * arithmetic for binary32 inputs: within a few ulps of the binary64 terms
 * rounded to binary32); the sums are exact integer sums of these values
 * quantised to 2^-e (e chosen per channel from the largest |phi| so that no
 * sum can overflow), hence order-independent.  Binary64 calls add a second
 * integer word per channel for the quantisation remainders, so that the
 * error of a particle stays below 2^-62 of the largest |phi| whatever the
 * count.  den, if given, receives the particle count per cell.  A particle
 * with a finite position outside a closed box is counted in stats.outside
 * (whatever its other inputs); any other particle with a non-finite input
 * or source term is skipped and counted in stats.skipped.  Meshes of more than 16384 * 1024 cells (16384 * 512 in
 * binary64 3-D) return INVALID_ARG.  Other errors as fla_project_sources. */
fla_status psicell_accumulate(fla_ctx* ctx, const fla_mesh* mesh,
                              const fla_trajectories* particles, double particle_weight,
                              const fla_params* params, const fla_fields* out, void* stream);

/* Cloud-in-cell accumulation, the linear-interpolation comparator the paper
 * names beside PSI-CELL (introduction): each particle's
 * phi_p = [mdot_p, F_p + mdot_p v_p] is shared among the 2^dim cell centres
 * around it with per-axis hat weights 1 - |d|/dx (d the offset to the
 * centre; the corners of the dual cell that holds the particle):
 *   S_k(c) = -(particle_weight / V_c) * cell_scale(c) * sum_p W_cp phi_pk.
 * Periodic axes wrap; on a closed axis a particle less than half a cell from
 * a wall puts that axis's whole weight on the boundary cell, so every
 * particle deposits all of phi_p.  den, if given, receives sum_p W_cp.
 * Particles outside a closed box (x == hi belongs to it) are counted in
 * stats.outside, other particles with a non-finite input in stats.skipped
 * (the position decides first, as in psicell_accumulate).  The
 * sums are exact integer sums as in psicell_accumulate (two words per
 * channel for binary64), hence deterministic.  Meshes of more than
 * 16384 * 1024 cells (16384 * 512 in binary64) return INVALID_ARG.  Other
 * errors as psicell_accumulate. */
fla_status cic_accumulate(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* particles,
                          double particle_weight, const fla_params* params, const fla_fields* out, void* stream);

/* Statistics of the last call on ctx.  Synchronises the device, then copies
 * into *out (host).  Errors: INVALID_ARG for NULL, DEVICE. */
fla_status fla_get_stats(fla_ctx* ctx, fla_stats* out);

/* Per-stage device timing.  While enabled, every call records a pair of HIP
 * events around each of its stages on the call's stream; fla_profile_read
 * synchronises the device and returns, per stage, the summed elapsed time
 * and the number of timed launches since profiling was enabled.  Stages:
 * 0 prepass, 1 key sort + bucket bounds + record permutation, 2 deposition
 * normaliser, 3 gather with fused epilogue, 4 PSI-CELL accumulation,
 * 5 bandwidth network forward, 6 estimator backward, 7 network backward
 * (fla_project_batch records stages 0, 1 and 3 once for the whole batch and
 * runs without a graph while profiling is on).
 * Errors: INVALID_ARG for NULL, DEVICE. */
#define FLA_PROFILE_STAGES 8
typedef struct {
    double ms[FLA_PROFILE_STAGES];
    int64_t launches[FLA_PROFILE_STAGES];
} fla_profile;

/* on != 0: clear previous records and start recording; on == 0: stop. */
fla_status fla_profile_enable(fla_ctx* ctx, int on);
fla_status fla_profile_read(fla_ctx* ctx, fla_profile* out);

/* Gather plan code: plan + FLA_GATHER_PLANS * shape.
 * The plan is the granularity at which the gather skips the sub-blocks
 * (blocks of 4^3 or 8^2 cells) that a trajectory cannot reach:
 *   0: each sub-block;
 *   1: pairs of sub-blocks along z (3-D, the default; the binary32 loop,
 *      which takes four trajectories per step, adds a test per sub-block);
 *   2, 3: only the workgroup's whole part.
 * In 2-D, plans 1-3 skip only the whole tile.
 * The shape is the part of a tile (8^3 or 16^2 cells) one workgroup owns:
 *   0: in 3-D half a tile along x (4 sub-blocks; the default), in 2-D the
 *      whole tile;
 *   1: the whole tile in 3-D (8 sub-blocks: the candidates are scanned and
 *      staged once per tile instead of once per half, with fewer workgroups
 *      per compute unit); not in 2-D.
 * So codes 0..7 are valid in 3-D and 0..3 in 2-D.  Under one shape every
 * plan produces the same values (up to the sign of zero); they differ only
 * in speed.  Between shapes, binary64 values are the same as well; binary32
 * values can differ by the rounding of the compensated sums, whose partial
 * sums are folded at other points.  Codes are kept per (dim, prec) in the
 * context; -1 restores the library default (code 1).
 * Errors: INVALID_ARG for out-of-range arguments. */
#define FLA_GATHER_PLANS 4
#define FLA_GATHER_SHAPES 2
#define FLA_GATHER_CONFIGS (FLA_GATHER_PLANS * FLA_GATHER_SHAPES)
fla_status fla_set_plan(fla_ctx* ctx, int dim, int prec, int gather_plan);
fla_status fla_get_plan(fla_ctx* ctx, int dim, int prec, int* gather_plan);

/* Autotuner: runs fla_project_sources once per gather plan code of the
 * mesh's dimension on the given inputs (a warm-up call, then a call timed
 * with HIP events), keeps the fastest code for (mesh->dim, traj->prec) in the
 * context and, if times_ms (host, FLA_GATHER_CONFIGS values, index = code) is
 * not NULL, returns the gather time of each code (-1 for codes the
 * dimension does not have).  Synchronises the device.  out receives the
 * projection.  Errors as fla_project_sources. */
fla_status fla_autotune(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                        const fla_params* params, const fla_fields* out, void* stream,
                        double* times_ms);

/* ---------------------------------------------------------------------------
 * Trajectory producer.  The droplets of the FLA are advanced over one carrier
 * time step in an analytic gas field and projected in the same call, the
 * integration fused with the prepass (the advanced position and Jacobian go
 * from registers into the projection's records).
 *
 * Gas field (steady): u(x) = u0 + G x + a periodic part of amplitude U and
 * wavenumber k, w = 2 pi k:
 *   FLA_FLOW_NONE          none (uniform and linear flows)
 *   FLA_FLOW_TAYLOR_GREEN  2-D: U (sin(w x) cos(w y), -cos(w x) sin(w y))
 *   FLA_FLOW_ABC           3-D: U (A sin(w z + pz) + C cos(w y + py),
 *                                  B sin(w x + px) + A cos(w z + pz),
 *                                  C sin(w y + py) + B cos(w x + px))
 * with abc = (A, B, C), phase = (px, py, pz), G[a*3 + b] = du_a/dx_b. */
typedef enum { FLA_FLOW_NONE = 0, FLA_FLOW_TAYLOR_GREEN = 1, FLA_FLOW_ABC = 2 } fla_flow_kind;
typedef struct {
    int32_t kind;           /* fla_flow_kind */
    int32_t reserved;
    double U;               /* amplitude of the periodic part, m/s */
    double k;               /* wavenumber, periods per unit length */
    double abc[3];
    double phase[3];
    double u0[3];           /* uniform part */
    double G[9];            /* linear part */
} fla_flow;

/* Droplet state: binary64 device planes of count values, updated in place
 * when step.update_state is set.  x[a] positions, v[a] velocities, J the
 * Jacobian dx/dx0 and dJ its time derivative (dim*dim planes, entry (a, b)
 * at plane a*dim + b; at seeding J = I and dJ = dv0/dx0, eq.
 * Jacobian-evolution), r radii; n0 (nullable, else n0_scalar) the initial
 * number density; seed_volume as in fla_trajectories.  phibar (nullable,
 * 1 + dim planes) receives the step's source rates of one droplet (see
 * fla_advance_project; 0 for skipped droplets). */
typedef struct {
    int64_t count;          /* >= 0, < 2^31 */
    double* x[3];
    double* v[3];
    double* J;
    double* dJ;
    double* r;
    const double* n0;
    double n0_scalar;
    double seed_volume;
    double* phibar;
} fla_droplets;

/* One carrier time step: length dt (s) in `substeps` equal substeps;
 * update_state nonzero writes the advanced state back. */
typedef struct {
    double dt;
    int32_t substeps;       /* 1 .. 2^20 */
    int32_t update_state;
} fla_step;

/* Advance and project (paper: eqs. Stokes-drag, evap-model and
 * Jacobian-evolution integrated along the trajectories, App. B steps 1a-1d
 * and 2a-2c).  Every droplet is advanced over the step with the classical
 * fourth-order Runge-Kutta method in binary64, in dimensional form
 * (tau = 2 rho_d r^2/(9 mu)):
 *   x' = v, v' = (u(x) - v)/tau, r' = delta/(2 r),
 *   J' = dJ, dJ' = (grad u(x) J - dJ)/tau,
 * and its contributions Q' = [mdot, F + mdot v] (F = m (u - v)/tau,
 * mdot = 4 pi rho_d r^2 r') are integrated over the same substeps and
 * summed over the step; the step's source rates are phibar = Q/dt.  The
 * advanced droplets are then projected as fla_project_sources projects
 * trajectories (params.mode, h = h0 |det J| times params.h_factor,
 * n = n0/|det J|), with phibar in place of the instantaneous source terms;
 * prec (fla_precision) selects the arithmetic of the projection.  A
 * droplet is skipped and counted (stats.skipped) if an input is not finite,
 * r <= 0, it evaporates within the step (r^2 + delta dt <= 0), the
 * advanced state is not finite or det J = 0; its state is left as it was.
 * Errors: INVALID_ARG (checked on the host), OUT_OF_MEMORY, DEVICE. */
fla_status fla_advance_project(fla_ctx* ctx, const fla_mesh* mesh, const fla_droplets* drops, const fla_flow* flow,
                               const fla_step* step, const fla_params* params, int prec, const fla_fields* out,
                               void* stream);

/* ---------------------------------------------------------------------------
 * Learned bandwidth correction.  A 5-64-64-1 network (SiLU hidden layers)
 * predicts a per-trajectory factor g_i = exp(ln4 * tanh o_i) multiplying the
 * smoothing length h_i = h0 |det J_i| of eq. (smoothing-length).  Its inputs
 * are z = (f - mu)/sd for the features
 *   f = [log s1, log s2, log s3, log(n/n0) = -log|det J|, log(1 + N_nbr)]
 * (s_k the singular values of J, largest first, s3 = 1 in 2-D; N_nbr the
 * valid trajectories whose home cell is in the 3^d block of cells around the
 * trajectory's home cell).  Weights are held as an FP32 parameter block of
 * FLA_MLP_PARAMS floats (device):
 *   W1[64][5], b1[64], W2[64][64], b2[64], w3[64], b3   (trainable, 4609)
 *   mu[5], sd[5]                                         (standardisation)
 * The network runs on bf16 MFMA with FP32 accumulation: z, the first hidden
 * layer and W1, W2, w3 are rounded to bf16; biases stay FP32.
 * ------------------------------------------------------------------------- */
#define FLA_MLP_TRAINABLE 4609
#define FLA_MLP_PARAMS 4619

/* Features and network.  theta: device parameter block.  h_factor (device,
 * count floats, required) receives g_i (1 for skipped trajectories); z
 * (5*count, plane k = input k), o (count) and features (5*count, raw f;
 * NaN for skipped trajectories) are optional device outputs (the backward
 * needs z and o).  The result feeds fla_params.h_factor.  Errors as
 * fla_project_sources. */
fla_status fla_bandwidth_forward(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                 const float* theta, float* h_factor, float* z, float* o,
                                 float* features, void* stream);

/* Gradient through the estimator: given the fields S (S_mass, S_mom and
 * den, all required) of an FLA_NW projection with these same inputs and
 * params (h_factor included), and dL/dS (same layout; den ignored), writes
 *   dL_dlogh[i] = h_i dL/dh_i = sum_c K_ci (s_ci - 1) a_c (sum_k g_kc q_ik - sum_k g_kc S~_kc),
 * K the kernel, s = |x_c - x_i|^2/h_i^2, g = dL/dS, a_c = -scale cs_c/den_c
 * and S~ = S/(-scale cs) the unsigned estimate, summed over the included
 * pairs (device, count floats; 0 for skipped trajectories).  The movement of
 * the truncation radius with h is not differentiated (its term is of the
 * order of the kernel tail, exp(-cutoff^2/2)).  Errors as fla_project_sources. */
fla_status fla_project_backward(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                                const fla_params* params, const fla_fields* S, const fla_fields* dL_dS,
                                float* dL_dlogh, void* stream);

/* Network backward: with z and o from fla_bandwidth_forward and dL/dlog h
 * from fla_project_backward, writes dL/dtheta (device, FLA_MLP_PARAMS floats;
 * zeros for mu, sd).  Partial sums per block are added in block order
 * (deterministic).  dim is 2 or 3.  Errors: INVALID_ARG, DEVICE. */
fla_status fla_bandwidth_backward(fla_ctx* ctx, int dim, const float* theta, int64_t count, const float* z,
                                  const float* o, const float* dL_dlogh, float* grad, void* stream);

/* One Adam step on the trainable entries of theta with moments m, v (all
 * device, FLA_MLP_PARAMS floats; the entries past the trainable ones are
 * left untouched): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2 and
 * theta -= lr m^ / (sqrt(v^) + eps) with m^ = m/(1 - b1^step), v^ =
 * v/(1 - b2^step), evaluated in binary64 from the binary64 arguments and
 * stored in binary32; step counts from 1.  Errors: INVALID_ARG, DEVICE. */
fla_status fla_adam_step(fla_ctx* ctx, float* theta, float* m, float* v, const float* grad, int64_t step,
                         double lr, double beta1, double beta2, double eps, void* stream);

/* Relative-L2 loss over the channels (S_mass, S_mom[0..channels-2]):
 *   L = sum_k |S_k - R_k|^2 / |R_k|^2
 * result (device, 1 + 2*channels doubles): L, then |S_k - R_k|^2 and |R_k|^2
 * per channel; dL_dS (nullable) receives 2 (S_k - R_k)/|R_k|^2.  Sums are
 * formed in a fixed order (deterministic).  Errors: INVALID_ARG, DEVICE. */
fla_status fla_rel_l2_loss(fla_ctx* ctx, int channels, int64_t cells, int prec, const fla_fields* S,
                           const fla_fields* R, const fla_fields* dL_dS, double* result, void* stream);

/* Feature standardisation of the network inputs: sets mu[5] and sd[5] of
 * theta (device parameter block; the trainable entries are left as they
 * are) to the mean and the Bessel-corrected standard deviation plus 1e-3 of
 * the raw features f over the valid trajectories of nsnap snapshots (host
 * arrays of meshes and trajectories; a trajectory is valid when it is not
 * skipped, as in fla_project_sources).  The sums are formed in binary64 in
 * a fixed order (deterministic), the deviations in a second pass from the
 * finished mean.  Errors: INVALID_ARG (naming the snapshot), OUT_OF_MEMORY,
 * DEVICE. */
fla_status fla_bandwidth_standardise(fla_ctx* ctx, int nsnap, const fla_mesh* meshes, const fla_trajectories* trajs,
                                     float* theta, void* stream);

/* One training step of the bandwidth network on one snapshot, every stage in
 * the library's kernels on one stream: features and network
 * (fla_bandwidth_forward) -> FLA_NW projection with the factors
 * (fla_project_sources) -> relative-L2 loss against the reference fields ref
 * and dL/dS (fla_rel_l2_loss; ref holds C = dim + 1 planes in the call's
 * precision, typically a dense PSI-CELL field) -> estimator backward
 * (fla_project_backward) -> network backward (fla_bandwidth_backward) ->
 * one Adam step (fla_adam_step) on theta with moments m and v (device,
 * FLA_MLP_PARAMS floats each, updated in place; step counts from 1).  The
 * result is bit for bit that of the six calls made in that order.  params
 * gives the physics and kernel parameters (mode FLA_NW, h_factor NULL: the
 * step forms the factors).  loss (nullable, device, 1 + 2 C doubles)
 * receives the loss and its per-channel terms as fla_rel_l2_loss writes
 * them.  The intermediates live in a context-owned training workspace.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
fla_status fla_mlp_train_step(fla_ctx* ctx, const fla_mesh* mesh, const fla_trajectories* traj,
                              const fla_params* params, const fla_fields* ref, float* theta, float* m, float* v,
                              int64_t step, double lr, double beta1, double beta2, double eps, double* loss,
                              void* stream);

/* ---------------------------------------------------------------------------
 * Batched projection of many independent snapshots of uneven size.  Each
 * snapshot is projected with the estimator of fla_project_sources; batching
 * changes only how the work is launched.
 * meshes, trajs, params and outs are host arrays of nsnap structs; snapshot s
 * writes outs[s] bit for bit as fla_project_sources(meshes[s], trajs[s],
 * params[s], outs[s]) does under the same gather plan.  All snapshots share
 * dim and prec; every mode must be FLA_NW.  Statistics are summed over the
 * batch (max_class is the largest over the snapshots); pairs are counted
 * if any params[s].count_pairs is set.
 * Launch sequence: one prepass over the trajectories of all snapshots, one
 * key sort whose buckets are (snapshot, class, tile), one record permutation
 * and one gather launch with a workgroup per (snapshot, tile).  Snapshots
 * are ordered by estimated work per tile, largest first, so that the
 * longest workgroups start first.
 * Graphs (default on, see fla_set_batch_graph) while profiling is off: the
 * first call with a given set of arguments (every field of every struct,
 * the stream, the batch plan, the context's workspace) waits for the
 * previous batch call's work, uploads a snapshot table, captures the launch
 * sequence into a HIP graph and launches it; a later call with identical
 * arguments only launches that graph.  Buffer contents may change between
 * such calls; pointers, sizes and parameters may not.  The context keeps
 * one graph.  Errors: INVALID_ARG (nsnap outside [1, FLA_BATCH_MAX], mixed
 * dim or prec, a mode other than FLA_NW, more than 2^31 - 1 trajectories or
 * buckets in total, or any check of fla_project_sources on a snapshot),
 * OUT_OF_MEMORY, DEVICE. */
#define FLA_BATCH_MAX 65536
fla_status fla_project_batch(fla_ctx* ctx, int nsnap, const fla_mesh* meshes, const fla_trajectories* trajs,
                             const fla_params* params, const fla_fields* outs, void* stream);

/* enable != 0: batch calls go through the cached graph (default);
 * enable == 0: every batch call uploads its table and enqueues the
 * launches directly.  Drops the cached graph.  Errors: INVALID_ARG. */
fla_status fla_set_batch_graph(fla_ctx* ctx, int enable);

/* Graphs for single calls of fla_project_sources (default off; for callers
 * that repeat a small projection, whose time is mostly launch latency).
 * While enabled, and while profiling and FLA_TRACE are off, the first call
 * with a given set of arguments (every field of the mesh, trajectory,
 * parameter and field structs, the stream, the gather plan code, the
 * context's workspace) runs directly; the next call with the same arguments
 * captures its launch sequence into a HIP graph and launches it, and later
 * identical calls only launch that graph (counted in
 * fla_stats.graph_replays).  Buffer contents may change between such calls;
 * pointers, sizes and parameters may not (a change is a new set of
 * arguments).  One graph is kept per context.  fla_project_sources_noalloc
 * never uses it.  Synchronises the device and drops the cached graph.
 * Errors: INVALID_ARG. */
fla_status fla_set_graph(fla_ctx* ctx, int enable);

/* Batch plan per (dim, prec): the gather plan code (as fla_set_plan) and the
 * XCD chunk, the number of consecutive work items (tiles) that one of the
 * eight XCDs receives from each run of 8 * chunk items, 1..4096.
 * gather_plan == -1 restores the library defaults (chunk is then ignored).
 * Errors: INVALID_ARG for out-of-range arguments. */
fla_status fla_set_batch_plan(fla_ctx* ctx, int dim, int prec, int gather_plan, int chunk);
fla_status fla_get_batch_plan(fla_ctx* ctx, int dim, int prec, int* gather_plan, int* chunk);

/* Batch autotuner: runs fla_project_batch directly (no graph) for every
 * gather plan code of the dimension and every chunk in {1, 4, 16, 64} (a
 * warm-up call, then a call whose gather launch is timed with HIP events),
 * keeps the fastest pair for (dim, prec) and, if times_ms (host,
 * FLA_GATHER_CONFIGS * FLA_BATCH_CHUNKS values, index code *
 * FLA_BATCH_CHUNKS + chunk index, -1 for codes the dimension does not have)
 * is not NULL, returns every gather time.  Synchronises the device; outs
 * receive the projection.  Errors as fla_project_batch. */
#define FLA_BATCH_CHUNKS 4
fla_status fla_autotune_batch(fla_ctx* ctx, int nsnap, const fla_mesh* meshes, const fla_trajectories* trajs,
                              const fla_params* params, const fla_fields* outs, void* stream,
                              double* times_ms);

/* Saving the plans: callers keep the autotuners' choices across processes.
 * fla_save_plans writes, to the text file at path, the context's gather
 * plan code and batch plan (code and chunk) for every (dim, prec), -1 where
 * the library default is in use, keyed by the device's architecture name
 * (for example gfx950): a header line "flaproj-plans 1", then one line
 * "<arch> <dim> <prec> <plan code> <batch plan code> <chunk>" each.
 * fla_load_plans reads such a file and sets the plans of the lines for this
 * device's architecture (lines for other architectures are ignored).  A
 * file that cannot be read, lacks the header or holds a malformed or
 * out-of-range line changes nothing and returns INVALID_ARG (message in
 * fla_last_error).  Host files only; no device work. */
fla_status fla_save_plans(fla_ctx* ctx, const char* path);
fla_status fla_load_plans(fla_ctx* ctx, const char* path);

/* ------------------------------------------------------------------------
 * General meshes (App. A, "Cell volume scaling" and "Combining the mass and
 * volume scaling factors"): the carrier solver's cells are given by their
 * centroids and volumes, in the solver's own cell order, as on an
 * unstructured finite-volume mesh.  The kernel estimator is evaluated at
 * each centroid exactly as fla_project_sources evaluates it at a Cartesian
 * cell centre; the mesh enters only through n_hat of eq. mv-scal, which is
 * proportional to the cell volume.
 * ------------------------------------------------------------------------ */

/* Cells of a general mesh.  centroid[a] (device, binary64, count values per
 * axis a < dim) must lie in the box [lo, hi] on every axis (the box also
 * gives the period hi - lo of a periodic axis, on which offsets take the
 * minimum image); volume (device, binary64, count values, >= 0) may be NULL
 * when no n_hat is asked for.  The arrays are read by fla_cell_index_create
 * only: the index keeps its own copies. */
typedef struct {
    int32_t dim;                /* 2 or 3 */
    int32_t periodic[3];        /* nonzero = periodic axis */
    double lo[3];
    double hi[3];               /* hi[a] > lo[a] */
    int64_t count;              /* cells, in [1, 2^31) */
    const double* centroid[3];
    const double* volume;       /* nullable */
} fla_cells;

typedef struct fla_cell_index fla_cell_index;

/* Spatial index of a general mesh, built once per mesh on ctx's device:
 * a rectilinear grid of buckets whose per-axis edges sit at quantiles of the
 * centroid coordinates (at most 1024 buckets per axis), aiming at about
 * cells_per_bucket cells per bucket (<= 0: the default, 112), and the cells
 * sorted by bucket.  Synchronises the device.  *out (host pointer) is owned
 * by the caller and released with fla_cell_index_destroy, which must come
 * before the context is destroyed.  Errors: INVALID_ARG (bad dim, count or
 * box, a NULL centroid array, a centroid outside the box or not finite, a
 * negative or non-finite volume), OUT_OF_MEMORY, DEVICE. */
fla_status fla_cell_index_create(fla_ctx* ctx, const fla_cells* cells, int32_t cells_per_bucket,
                                 fla_cell_index** out);
fla_status fla_cell_index_destroy(fla_cell_index* index);

/* Shape of an index: buckets per axis (nb[2] = 1 in 2-D) and the number of
 * gather work items (runs of at most 128 cells of one bucket).  Host call.
 * Errors: INVALID_ARG for NULL arguments. */
fla_status fla_cell_index_shape(const fla_cell_index* index, int32_t nb[3], int64_t* work_items);

/* Injection parameters of the reference (PSI-CELL) run for n_hat (eq.
 * mv-scal): N^ref droplets injected every tau_inj^ref through a face of
 * area A_inj at mean speed v_inj.  For a mass-flow specification (eq.
 * mv-scal-massflow) set n_ref / tau_ref = mdot_ref / m. */
typedef struct {
    double n_ref;
    double tau_ref;
    double area;
    double v_inj;
} fla_injection;

/* FLA source projection at the centroids of an indexed general mesh (the
 * estimator of fla_project_sources, FLA_NW mode):
 *   S_k(c) = -scale * n_hat(c) * num_k(c) / den(c),  0 where den(c) = 0,
 *   n_hat(c) = V_c * n_ref / (A_inj v_inj tau_ref)   if inj is not NULL,
 *   n_hat(c) = 1                                      if inj is NULL,
 * with the pair offsets, the inclusion test (sum_a (d_a/h)^2 <= cutoff^2,
 * binary32 terms and sum for FLA_F32) and the precisions of
 * fla_project_sources.  out planes hold index's cell count values in the
 * mesh's own cell order; den and pairs are optional as there.  Statistics:
 * trajectories, skipped, no_support (no centroid of a closed box within
 * reach), pairs (if counted), max_class (neighbourhood class in buckets).
 * Uses the context's workspace; asynchronous on stream.  Errors:
 * INVALID_ARG (as fla_project_sources; a mode other than FLA_NW; an index
 * of another device; inj with a non-positive or non-finite entry, or with
 * an index built without volumes), OUT_OF_MEMORY, DEVICE. */
fla_status fla_project_cells(fla_ctx* ctx, const fla_cell_index* index, const fla_trajectories* traj,
                             const fla_params* params, const fla_injection* inj, const fla_fields* out,
                             void* stream);

/* Message of the last error on ctx (host string owned by ctx, valid until
 * the next call on ctx); "" if the last call succeeded.  NULL ctx returns
 * the message of the last failed fla_ctx_create. */
const char* fla_last_error(const fla_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FLAPROJ_H */
