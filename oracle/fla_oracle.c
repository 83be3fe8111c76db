/*
 * FP64 CPU oracle for the FLA source projection and the PSI-CELL comparator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * Everything is IEEE binary64, evaluated in the order written (build with
 * -ffp-contract=off so that no multiply-add is fused).  Paper references are
 * to Stafford & Rybdylova, "Interphase coupling for gas-droplet flows using
 * the fully Lagrangian approach" (arXiv 2512.20829).
 *
 * Readings of the paper taken here (the paper is silent on them):
 *  - the Gaussian kernel (eq. "kernel") is truncated: a trajectory contributes
 *    to a cell centre only if sum_a (d_a/h)^2 <= c^2 (c = cutoff, 4 by
 *    default), where d_a is the per-axis offset (minimum image on periodic
 *    axes).  The test itself is evaluated either in binary64 or, for the
 *    single-precision product path, by rounding each (d_a/h)^2 to binary32 and
 *    summing in binary32 in axis order, so that both sides take the same
 *    integer decision;
 *  - the kernel keeps the paper's 1/h prefactor in every dimension;
 *  - each source term is returned with the minus sign of the averaged coupling
 *    terms (eq. "coupling-terms-averaged");
 *  - a cell with zero kernel denominator gets S = 0;
 *  - trajectories with det J = 0 or any non-finite input are skipped.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Mesh geometry: uniform Cartesian cells on [lo, hi), cell centres at       */
/* lo + (i + 1/2) * (hi - lo)/n.  Linear cell index: i0 + n0*(i1 + n1*i2).   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim;
    int n[3];
    double lo[3];
    double hi[3];
    int periodic[3];
} orc_mesh;

static double cell_width(const orc_mesh* m, int a) { return (m->hi[a] - m->lo[a]) / (double)m->n[a]; }

static double cell_centre(const orc_mesh* m, int a, int64_t i)
{
    double w = cell_width(m, a);
    double t = ((double)i + 0.5) * w;
    return m->lo[a] + t;
}

static void cell_coords(const orc_mesh* m, int64_t c, int64_t idx[3])
{
    idx[0] = c % m->n[0];
    c /= m->n[0];
    idx[1] = c % m->n[1];
    idx[2] = (m->dim == 3) ? c / m->n[1] : 0;
}

static double cell_volume(const orc_mesh* m)
{
    double v = 1.0;
    for (int a = 0; a < m->dim; ++a) v *= cell_width(m, a);
    return v;
}

/* Offset from a point to a cell centre along one axis; minimum image on a
 * periodic axis. */
static double axis_offset(const orc_mesh* m, int a, double xc, double xp)
{
    double d = xc - xp;
    if (m->periodic[a]) {
        double L = m->hi[a] - m->lo[a];
        double k = rint(d / L);
        double s = L * k;
        d = d - s;
    }
    return d;
}

/* ------------------------------------------------------------------------ */
/* Determinant by cofactor expansion along the first row (row-major J).      */
/* ------------------------------------------------------------------------ */
double orc_det(int dim, const double* J)
{
    if (dim == 2) {
        double p = J[0] * J[3];
        double q = J[1] * J[2];
        return p - q;
    }
    double m0 = J[4] * J[8] - J[5] * J[7];
    double m1 = J[3] * J[8] - J[5] * J[6];
    double m2 = J[3] * J[7] - J[4] * J[6];
    double t0 = J[0] * m0;
    double t1 = J[1] * m1;
    double t2 = J[2] * m2;
    return (t0 - t1) + t2;
}

/* ------------------------------------------------------------------------ */
/* Droplet physics for one droplet (dimensional forms of eqs. 3-5).          */
/*   m     = (4/3) pi rho_d r^3               (sphere volume x density)     */
/*   tau   = 2 rho_d r^2 / (9 mu)             (Stokes relaxation, eq. 5)    */
/*   F     = m (u_g - v) / tau                (F = m x'', x'' from eq. 3)   */
/*   mdot  = 4 pi rho_d r^2 rdot, rdot = delta/(2 r)   (eq. 4)               */
/* Channel vector phi = [mdot, F_a + mdot v_a] (eq. coupling-terms-spec.).   */
/* ------------------------------------------------------------------------ */
void orc_droplet_phi(int dim, double r, const double* v, const double* ug,
                     double rho_d, double mu, double delta, double* phi,
                     double* m_out, double* tau_out, double* mdot_out)
{
    double m = (4.0 / 3.0) * ORC_PI * rho_d * r * r * r;
    double tau = 2.0 * rho_d * r * r / (9.0 * mu);
    double rdot = delta / (2.0 * r);
    double mdot = 4.0 * ORC_PI * rho_d * r * r * rdot;
    phi[0] = mdot;
    for (int a = 0; a < dim; ++a) {
        double F = m * (ug[a] - v[a]) / tau;
        phi[1 + a] = F + mdot * v[a];
    }
    if (m_out) *m_out = m;
    if (tau_out) *tau_out = tau;
    if (mdot_out) *mdot_out = mdot;
}

/* ------------------------------------------------------------------------ */
/* Per-trajectory terms: det J, n = n0/|det J| (eq. FLA-COM), h = h0|det J| */
/* (eq. smoothing-length) times an optional bandwidth factor, and           */
/* q = n * phi (eq. coupling-terms-kernel numerators).                      */
/* Arrays: x, v, ug are dim x N planes; J is dim*dim x N planes.            */
/* ------------------------------------------------------------------------ */
static int all_finite(const double* a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int64_t orc_trajectory_terms(int dim, int64_t N, const double* x, const double* J,
                             const double* v, const double* ug, const double* r,
                             const double* n0, double n0_scalar, double rho_d, double mu,
                             double delta, double h0, const double* hfac,
                             double* det_out, double* h_out, double* n_out, double* q_out,
                             int* valid_out)
{
    int C = 1 + dim;
    int64_t skipped = 0;
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t i = 0; i < N; ++i) {
        double Ji[9], xi[3], vi[3], ui[3];
        for (int e = 0; e < dim * dim; ++e) Ji[e] = J[e * N + i];
        for (int a = 0; a < dim; ++a) {
            xi[a] = x[a * N + i];
            vi[a] = v[a * N + i];
            ui[a] = ug[a * N + i];
        }
        double ri = r[i];
        double n0i = n0 ? n0[i] : n0_scalar;
        double det = orc_det(dim, Ji);
        double adet = fabs(det);
        double fac = hfac ? hfac[i] : 1.0;
        int ok = all_finite(Ji, dim * dim) && all_finite(xi, dim) && all_finite(vi, dim) &&
                 all_finite(ui, dim) && isfinite(ri) && isfinite(n0i) && isfinite(det) &&
                 det != 0.0 && isfinite(fac) && fac > 0.0;
        double h = h0 * adet;
        h = h * fac;
        double n = n0i / adet;
        double phi[4] = {0, 0, 0, 0};
        if (ok) orc_droplet_phi(dim, ri, vi, ui, rho_d, mu, delta, phi, 0, 0, 0);
        if (ok && !(isfinite(h) && h > 0.0 && isfinite(n) && all_finite(phi, C))) ok = 0;
        if (!ok) ++skipped;
        if (det_out) det_out[i] = det;
        h_out[i] = ok ? h : 0.0;
        if (n_out) n_out[i] = ok ? n : 0.0;
        for (int k = 0; k < C; ++k) q_out[k * N + i] = ok ? n * phi[k] : 0.0;
        valid_out[i] = ok;
    }
    return skipped;
}

/* ------------------------------------------------------------------------ */
/* Truncation test (reading of the infinite-support kernel, see header).    */
/* ------------------------------------------------------------------------ */
static int pair_included(int dim, const double s[3], double cutoff, int f32_decision)
{
    if (f32_decision) {
        float c = (float)cutoff;
        float c2 = c * c;
        float acc = (float)s[0];
        acc = acc + (float)s[1];
        if (dim == 3) acc = acc + (float)s[2];
        return acc <= c2;
    }
    double acc = s[0] + s[1];
    if (dim == 3) acc = acc + s[2];
    return acc <= cutoff * cutoff;
}

/* Kernel of eq. "kernel": K_h(x, x_i) = (1/h) exp(-|x - x_i|^2 / (2 h^2)). */
static double gauss_kernel(double r2, double h) { return (1.0 / h) * exp(-r2 / (2.0 * h * h)); }

/* Evaluate the kernel between one cell centre and one trajectory.  Returns 1
 * and the weight if the pair passes the truncation test. */
static int cell_traj_weight(const orc_mesh* m, const int64_t idx[3], const double* x, int64_t N,
                            int64_t i, double h, double cutoff, int f32_decision, double* K)
{
    double s[3] = {0, 0, 0};
    double r2 = 0.0;
    double inv_h = 1.0 / h;
    for (int a = 0; a < m->dim; ++a) {
        double d = axis_offset(m, a, cell_centre(m, a, idx[a]), x[a * N + i]);
        double u = d * inv_h;
        s[a] = u * u;
        r2 += d * d;
    }
    if (!pair_included(m->dim, s, cutoff, f32_decision)) return 0;
    *K = gauss_kernel(r2, h);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Nadaraya-Watson projection, evaluated at listed cell centres by brute    */
/* force over all trajectories (eq. kernel-estimator applied as in           */
/* eq. coupling-terms-kernel; App. B steps 1c, 1d, 2a and 2c).               */
/*   num_k(c) = sum_i K(x_c, x_i) q_ik,  den(c) = sum_i K(x_c, x_i)          */
/*   S_k(c)   = -scale * cell_scale(c) * num_k(c) / den(c), 0 if den = 0     */
/* Outputs are C x ncells (S), ncells (den), ncells (pair counts).           */
/* ------------------------------------------------------------------------ */
void orc_nw_cells(const orc_mesh* m, int64_t N, const double* x, const double* h,
                  const double* q, const int* valid, double cutoff, int f32_decision,
                  double scale, const double* cell_scale, int64_t ncells, const int64_t* cells,
                  double* S, double* den_out, int64_t* pairs_out)
{
    int C = 1 + m->dim;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < ncells; ++j) {
        int64_t idx[3];
        cell_coords(m, cells[j], idx);
        double num[4] = {0, 0, 0, 0};
        double den = 0.0;
        int64_t np = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (!valid[i]) continue;
            double K;
            if (!cell_traj_weight(m, idx, x, N, i, h[i], cutoff, f32_decision, &K)) continue;
            den += K;
            for (int k = 0; k < C; ++k) num[k] += K * q[k * N + i];
            ++np;
        }
        double cs = cell_scale ? cell_scale[cells[j]] : 1.0;
        for (int k = 0; k < C; ++k) S[k * ncells + j] = (den > 0.0) ? -scale * cs * (num[k] / den) : 0.0;
        if (den_out) den_out[j] = den;
        if (pairs_out) pairs_out[j] = np;
    }
}

/* ------------------------------------------------------------------------ */
/* Nadaraya-Watson projection on a general mesh: the cells are given by     */
/* their centroids (dim x M planes, xc[a*M + c]) instead of a lattice, as   */
/* the kernel estimator needs nothing of a cell but the point where it is   */
/* evaluated (the interpolation is meshfree; the mesh enters only through  */
/* the per-cell factor n_hat of App. A, eq. mv-scal, passed in cell_scale). */
/* Offsets on periodic axes take the minimum image with period L[a]; the     */
/* estimator, truncation and epilogue are those of orc_nw_cells, so         */
/* centroids placed at a lattice's cell centres reproduce it bit for bit.   */
/* Outputs for the listed cells as in orc_nw_cells.                          */
/* ------------------------------------------------------------------------ */
static double point_offset(int periodic, double L, double xc, double xp)
{
    double d = xc - xp;
    if (periodic) {
        double k = rint(d / L);
        double s = L * k;
        d = d - s;
    }
    return d;
}

void orc_nw_points(int dim, int64_t M, const double* xc, const int* periodic, const double* L, int64_t N,
                   const double* x, const double* h, const double* q, const int* valid, double cutoff,
                   int f32_decision, double scale, const double* cell_scale, int64_t ncells,
                   const int64_t* cells, double* S, double* den_out, int64_t* pairs_out)
{
    int C = 1 + dim;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < ncells; ++j) {
        int64_t c = cells[j];
        double num[4] = {0, 0, 0, 0};
        double den = 0.0;
        int64_t np = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (!valid[i]) continue;
            double s[3] = {0, 0, 0};
            double r2 = 0.0;
            double inv_h = 1.0 / h[i];
            for (int a = 0; a < dim; ++a) {
                double d = point_offset(periodic[a], L[a], xc[a * M + c], x[a * N + i]);
                double u = d * inv_h;
                s[a] = u * u;
                r2 += d * d;
            }
            if (!pair_included(dim, s, cutoff, f32_decision)) continue;
            double K = gauss_kernel(r2, h[i]);
            den += K;
            for (int k = 0; k < C; ++k) num[k] += K * q[k * N + i];
            ++np;
        }
        double cs = cell_scale ? cell_scale[c] : 1.0;
        for (int k = 0; k < C; ++k) S[k * ncells + j] = (den > 0.0) ? -scale * cs * (num[k] / den) : 0.0;
        if (den_out) den_out[j] = den;
        if (pairs_out) pairs_out[j] = np;
    }
}

/* Home cell of a point: the cell containing it; periodic axes wrap, other  */
/* axes clamp to the nearest cell.                                           */
static int64_t home_cell(const orc_mesh* m, const double* x, int64_t N, int64_t i)
{
    int64_t lin = 0, stride = 1;
    for (int a = 0; a < m->dim; ++a) {
        double g = floor((x[a * N + i] - m->lo[a]) / cell_width(m, a));
        int64_t k = (int64_t)g;
        if (m->periodic[a]) {
            k %= m->n[a];
            if (k < 0) k += m->n[a];
        } else {
            if (k < 0) k = 0;
            if (k >= m->n[a]) k = m->n[a] - 1;
        }
        lin += k * stride;
        stride *= m->n[a];
    }
    return lin;
}

/* ------------------------------------------------------------------------ */
/* Normalised-kernel deposition (conservative companion of the estimator).  */
/* Each trajectory carries the amount Q_i = q_i * V_seed * |det J_i|         */
/* (= n0_i V_seed phi_i), spread over the cells it reaches with weights     */
/* K_ci / Z_i, Z_i = sum_c K_ci; if Z_i = 0 the whole amount goes to its     */
/* home cell.  S(c) = -scale * cell_scale(c) / V_c * sum_i Q_i K_ci / Z_i.   */
/* Z is returned per trajectory (0 for skipped ones).                        */
/* ------------------------------------------------------------------------ */
void orc_deposit(const orc_mesh* m, int64_t N, const double* x, const double* h,
                 const double* q, const double* det, const int* valid, double seed_volume,
                 double cutoff, int f32_decision, double scale, const double* cell_scale,
                 double* S /* C x M */, double* Z_out)
{
    int C = 1 + m->dim;
    int64_t M = 1;
    for (int a = 0; a < m->dim; ++a) M *= m->n[a];
    double Vc = cell_volume(m);
    double* Z = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        if (!valid[i]) continue;
        double z = 0.0;
        for (int64_t c = 0; c < M; ++c) {
            int64_t idx[3];
            double K;
            cell_coords(m, c, idx);
            if (cell_traj_weight(m, idx, x, N, i, h[i], cutoff, f32_decision, &K)) z += K;
        }
        Z[i] = z;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < M; ++c) {
        int64_t idx[3];
        cell_coords(m, c, idx);
        double acc[4] = {0, 0, 0, 0};
        for (int64_t i = 0; i < N; ++i) {
            if (!valid[i]) continue;
            double w;
            if (Z[i] > 0.0) {
                double K;
                if (!cell_traj_weight(m, idx, x, N, i, h[i], cutoff, f32_decision, &K)) continue;
                w = K / Z[i];
            } else {
                if (home_cell(m, x, N, i) != c) continue;
                w = 1.0;
            }
            double amount_scale = seed_volume * fabs(det[i]);
            for (int k = 0; k < C; ++k) acc[k] += w * (q[k * N + i] * amount_scale);
        }
        double cs = cell_scale ? cell_scale[c] : 1.0;
        for (int k = 0; k < C; ++k) S[k * M + c] = -scale * cs * acc[k] / Vc;
    }
    if (Z_out)
        for (int64_t i = 0; i < N; ++i) Z_out[i] = Z[i];
    free(Z);
}

/* ------------------------------------------------------------------------ */
/* Trajectory-centric forms (O(P) instead of O(N*M)).  The same estimator   */
/* and deposition as above, with each trajectory visiting only the cells    */
/* inside the bounding box of its cutoff sphere (App. B steps 1c-1d: loop   */
/* over trajectories, each adding its kernel contributions to the cells).   */
/* Every pair goes through the same cell_traj_weight as the brute-force     */
/* forms and every cell adds its trajectories in ascending index order, so  */
/* the results are those of the brute-force forms bit for bit; only the     */
/* cells that cannot hold an included pair are never looked at.             */
/* ------------------------------------------------------------------------ */

/* Cells of axis a whose centre can lie within reach of a trajectory at      */
/* coordinate xp with bandwidth h, in ascending index order.  A pair is      */
/* included only if (d/h)^2 <= c^2 on every axis (binary64; the binary32     */
/* decision differs by a few ulps), so the list widens the interval          */
/* |d| <= c h by a relative 1e-6 and one cell on each side; the inclusion    */
/* test itself decides.  Periodic axes wrap (minimum image), closed axes     */
/* clip.  Returns the number of cells written to list (at most n).           */
static int64_t axis_reach(const orc_mesh* m, int a, double xp, double h, double cutoff, int64_t* list)
{
    int64_t n = m->n[a];
    double w = cell_width(m, a);
    double u = (xp - m->lo[a]) / w - 0.5;     /* position in cell-centre index units */
    double R = cutoff * h / w * (1.0 + 1e-6) + 1.0;
    double klo = floor(u - R), khi = ceil(u + R);
    if (m->periodic[a]) {
        if (!(khi - klo + 1.0 < (double)n)) {
            for (int64_t k = 0; k < n; ++k) list[k] = k;
            return n;
        }
        /* shift the interval so that it starts in [0, n) */
        double sh = floor(klo / (double)n) * (double)n;
        int64_t k0 = (int64_t)(klo - sh), k1 = (int64_t)(khi - sh);
        int64_t cnt = 0;
        if (k1 >= n) {
            for (int64_t k = 0; k <= k1 - n; ++k) list[cnt++] = k;
            for (int64_t k = k0; k < n; ++k) list[cnt++] = k;
        } else {
            for (int64_t k = k0; k <= k1; ++k) list[cnt++] = k;
        }
        return cnt;
    }
    if (klo < 0.0) klo = 0.0;
    if (khi > (double)(n - 1)) khi = (double)(n - 1);
    if (klo > khi) return 0;
    int64_t cnt = 0;
    for (int64_t k = (int64_t)klo; k <= (int64_t)khi; ++k) list[cnt++] = k;
    return cnt;
}

/* Position of mesh index k of axis a inside a box of cells starting at      */
/* box_lo with box_n cells (wrapping on a periodic axis), or -1.             */
static int64_t box_pos(const orc_mesh* m, int a, int64_t k, int64_t box_lo, int64_t box_n)
{
    int64_t j = k - box_lo;
    if (m->periodic[a]) {
        j %= m->n[a];
        if (j < 0) j += m->n[a];
    }
    return (j >= 0 && j < box_n) ? j : -1;
}

/* Per-axis terms of one trajectory at the listed cells of axis a: the      */
/* offset d to each cell centre (minimum image), d^2 and (d/h)^2, exactly   */
/* as cell_traj_weight forms them.  A pair then sums these over the axes    */
/* in axis order, so its weight and inclusion are those of the brute-force  */
/* forms bit for bit; only the repeated per-axis work is done once.         */
static void axis_terms(const orc_mesh* m, int a, const int64_t* list, int64_t cnt, double xp, double inv_h,
                       double* dd, double* sq)
{
    for (int64_t e = 0; e < cnt; ++e) {
        double d = axis_offset(m, a, cell_centre(m, a, list[e]), xp);
        double u = d * inv_h;
        sq[e] = u * u;
        dd[e] = d * d;
    }
}

/* Weight of one pair from its per-axis terms (see cell_traj_weight).        */
static int pair_weight(int dim, const double* dd, const double* sq, double h, double cutoff, int f32_decision,
                       double* K)
{
    if (!pair_included(dim, sq, cutoff, f32_decision)) return 0;
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) r2 += dd[a];
    *K = gauss_kernel(r2, h);
    return 1;
}

/* Nadaraya-Watson source terms on a box of cells (form ii).  The box starts */
/* at cell box_lo[a] and spans box_n[a] cells on each axis (wrapping across  */
/* a periodic boundary); results are stored in box order                    */
/* j0 + b0*(j1 + b1*j2).  The whole field is box_lo = 0, box_n = n.         */
/* OpenMP threads own contiguous planes of the box along its last axis; each */
/* visits the trajectories in ascending order, so the sums of every cell    */
/* are formed in the order of the brute-force form and are deterministic.   */
/* Returns 0, or -1 for a box that does not fit the mesh.                   */
int orc_nw_box(const orc_mesh* m, int64_t N, const double* x, const double* h, const double* q,
               const int* valid, double cutoff, int f32_decision, double scale, const double* cell_scale,
               const int64_t* box_lo, const int64_t* box_n, double* S, double* den_out, int64_t* pairs_out)
{
    int C = 1 + m->dim, la = m->dim - 1;
    int64_t bn[3] = {1, 1, 1}, bl[3] = {0, 0, 0}, B = 1;
    for (int a = 0; a < m->dim; ++a) {
        bl[a] = box_lo[a];
        bn[a] = box_n[a];
        if (bn[a] < 1 || bn[a] > m->n[a]) return -1;
        if (!m->periodic[a] && (bl[a] < 0 || bl[a] + bn[a] > m->n[a])) return -1;
        B *= bn[a];
    }
    /* per cell: den, num[C], pair count (one record, so a pair touches one line) */
    typedef struct {
        double den, num[4];
        int64_t np;
    } cell_acc;
    cell_acc* acc = (cell_acc*)calloc((size_t)B, sizeof(cell_acc));
    int64_t nmax = 1;
    for (int a = 0; a < m->dim; ++a) nmax = m->n[a] > nmax ? m->n[a] : nmax;
#pragma omp parallel
    {
        int nt = 1, t = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        /* planes [p0, p1) of the box along its last axis belong to thread t */
        int64_t p0 = bn[la] * t / nt, p1 = bn[la] * (t + 1) / nt;
        int64_t* lists = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * nmax));
        int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * nmax));
        double* dd = (double*)malloc(sizeof(double) * (size_t)(3 * nmax));
        double* sq = (double*)malloc(sizeof(double) * (size_t)(3 * nmax));
        for (int64_t i = 0; i < N && p0 < p1; ++i) {
            if (!valid[i]) continue;
            int64_t cnt[3] = {1, 1, 1};
            int skip = 0;
            /* the last axis first: most trajectories miss this thread's planes */
            for (int a = la; a >= 0 && !skip; --a) {
                int64_t* L = lists + a * nmax;
                int64_t* P = pos + a * nmax;
                int64_t c = axis_reach(m, a, x[a * N + i], h[i], cutoff, L);
                int64_t kept = 0;
                for (int64_t e = 0; e < c; ++e) {
                    int64_t j = box_pos(m, a, L[e], bl[a], bn[a]);
                    if (j < 0 || (a == la && (j < p0 || j >= p1))) continue;
                    L[kept] = L[e];
                    P[kept] = j;
                    ++kept;
                }
                cnt[a] = kept;
                if (kept == 0) skip = 1;
            }
            if (skip) continue;
            double inv_h = 1.0 / h[i];
            for (int a = 0; a < m->dim; ++a)
                axis_terms(m, a, lists + a * nmax, cnt[a], x[a * N + i], inv_h, dd + a * nmax, sq + a * nmax);
            double qi[4] = {0, 0, 0, 0};
            for (int k = 0; k < C; ++k) qi[k] = q[k * N + i];
            for (int64_t e2 = 0; e2 < cnt[2]; ++e2)
                for (int64_t e1 = 0; e1 < cnt[1]; ++e1)
                    for (int64_t e0 = 0; e0 < cnt[0]; ++e0) {
                        int64_t j = pos[e0] + bn[0] * (pos[nmax + e1] + bn[1] * (m->dim == 3 ? pos[2 * nmax + e2] : 0));
                        double pd[3] = {dd[e0], dd[nmax + e1], m->dim == 3 ? dd[2 * nmax + e2] : 0.0};
                        double ps[3] = {sq[e0], sq[nmax + e1], m->dim == 3 ? sq[2 * nmax + e2] : 0.0};
                        double K;
                        if (!pair_weight(m->dim, pd, ps, h[i], cutoff, f32_decision, &K)) continue;
                        acc[j].den += K;
                        for (int k = 0; k < C; ++k) acc[j].num[k] += K * qi[k];
                        ++acc[j].np;
                    }
        }
        free(lists);
        free(pos);
        free(dd);
        free(sq);
    }
    for (int64_t j = 0; j < B; ++j) {
        int64_t jj[3] = {j % bn[0], (j / bn[0]) % bn[1], m->dim == 3 ? j / (bn[0] * bn[1]) : 0};
        int64_t lin = 0, stride = 1;
        for (int a = 0; a < m->dim; ++a) {
            int64_t k = bl[a] + jj[a];
            if (m->periodic[a]) {
                k %= m->n[a];
                if (k < 0) k += m->n[a];
            }
            lin += k * stride;
            stride *= m->n[a];
        }
        double cs = cell_scale ? cell_scale[lin] : 1.0;
        double den = acc[j].den;
        for (int k = 0; k < C; ++k) S[k * B + j] = (den > 0.0) ? -scale * cs * (acc[j].num[k] / den) : 0.0;
        if (den_out) den_out[j] = den;
        if (pairs_out) pairs_out[j] = acc[j].np;
    }
    free(acc);
    return 0;
}

/* Linear indices of the cells of a box (in box order), for the caller.      */
void orc_box_cells(const orc_mesh* m, const int64_t* box_lo, const int64_t* box_n, int64_t* cells)
{
    int64_t bn[3] = {1, 1, 1};
    for (int a = 0; a < m->dim; ++a) bn[a] = box_n[a];
    int64_t B = bn[0] * bn[1] * bn[2];
    for (int64_t j = 0; j < B; ++j) {
        int64_t jj[3] = {j % bn[0], (j / bn[0]) % bn[1], j / (bn[0] * bn[1])};
        int64_t lin = 0, stride = 1;
        for (int a = 0; a < m->dim; ++a) {
            int64_t k = box_lo[a] + jj[a];
            if (m->periodic[a]) {
                k %= m->n[a];
                if (k < 0) k += m->n[a];
            }
            lin += k * stride;
            stride *= m->n[a];
        }
        cells[j] = lin;
    }
}

/* Normalised-kernel deposition, trajectory-centric (form ii of            */
/* orc_deposit): Z_i sums the trajectory's kernel over the cells of its     */
/* reach in ascending linear order (the order of the brute-force form),     */
/* then threads owning planes along the last axis add Q_i K_ci / Z_i in     */
/* ascending trajectory order.  Bit for bit the brute-force result.         */
void orc_deposit_scatter(const orc_mesh* m, int64_t N, const double* x, const double* h,
                         const double* q, const double* det, const int* valid, double seed_volume,
                         double cutoff, int f32_decision, double scale, const double* cell_scale,
                         double* S /* C x M */, double* Z_out)
{
    int C = 1 + m->dim, la = m->dim - 1;
    int64_t M = 1, nmax = 1;
    for (int a = 0; a < m->dim; ++a) {
        M *= m->n[a];
        nmax = m->n[a] > nmax ? m->n[a] : nmax;
    }
    double Vc = cell_volume(m);
    double* Z = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double* acc = (double*)calloc((size_t)(C * M), sizeof(double));
#pragma omp parallel
    {
        int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * nmax));
        double* dd = (double*)malloc(sizeof(double) * (size_t)(3 * nmax));
        double* sq = (double*)malloc(sizeof(double) * (size_t)(3 * nmax));
        int64_t cnt[3];
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < N; ++i) {
            if (!valid[i]) continue;
            cnt[1] = cnt[2] = 1;
            L[nmax] = L[2 * nmax] = 0;
            double inv_h = 1.0 / h[i];
            for (int a = 0; a < m->dim; ++a) {
                cnt[a] = axis_reach(m, a, x[a * N + i], h[i], cutoff, L + a * nmax);
                axis_terms(m, a, L + a * nmax, cnt[a], x[a * N + i], inv_h, dd + a * nmax, sq + a * nmax);
            }
            double z = 0.0;
            for (int64_t e2 = 0; e2 < cnt[2]; ++e2)
                for (int64_t e1 = 0; e1 < cnt[1]; ++e1)
                    for (int64_t e0 = 0; e0 < cnt[0]; ++e0) {
                        double pd[3] = {dd[e0], dd[nmax + e1], m->dim == 3 ? dd[2 * nmax + e2] : 0.0};
                        double ps[3] = {sq[e0], sq[nmax + e1], m->dim == 3 ? sq[2 * nmax + e2] : 0.0};
                        double K;
                        if (pair_weight(m->dim, pd, ps, h[i], cutoff, f32_decision, &K)) z += K;
                    }
            Z[i] = z;
        }
        int nt = 1, t = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        int64_t p0 = (int64_t)m->n[la] * t / nt, p1 = (int64_t)m->n[la] * (t + 1) / nt;
        for (int64_t i = 0; i < N && p0 < p1; ++i) {
            if (!valid[i]) continue;
            double amount_scale = seed_volume * fabs(det[i]);
            if (!(Z[i] > 0.0)) {
                int64_t hc = home_cell(m, x, N, i);
                int64_t hz = m->dim == 3 ? hc / ((int64_t)m->n[0] * m->n[1]) : hc / m->n[0];
                if (hz < p0 || hz >= p1) continue;
                for (int k = 0; k < C; ++k) acc[k * M + hc] += 1.0 * (q[k * N + i] * amount_scale);
                continue;
            }
            cnt[0] = cnt[1] = cnt[2] = 1;
            L[nmax] = L[2 * nmax] = 0;
            int skip = 0;
            for (int a = la; a >= 0 && !skip; --a) {
                int64_t c = axis_reach(m, a, x[a * N + i], h[i], cutoff, L + a * nmax);
                if (a == la) {
                    int64_t kept = 0;
                    for (int64_t e = 0; e < c; ++e)
                        if (L[a * nmax + e] >= p0 && L[a * nmax + e] < p1) L[a * nmax + kept++] = L[a * nmax + e];
                    c = kept;
                }
                cnt[a] = c;
                if (c == 0) skip = 1;
            }
            if (skip) continue;
            double inv_h = 1.0 / h[i];
            for (int a = 0; a < m->dim; ++a)
                axis_terms(m, a, L + a * nmax, cnt[a], x[a * N + i], inv_h, dd + a * nmax, sq + a * nmax);
            for (int64_t e2 = 0; e2 < cnt[2]; ++e2)
                for (int64_t e1 = 0; e1 < cnt[1]; ++e1)
                    for (int64_t e0 = 0; e0 < cnt[0]; ++e0) {
                        int64_t idx[3] = {L[e0], L[nmax + e1], L[2 * nmax + e2]};
                        double pd[3] = {dd[e0], dd[nmax + e1], m->dim == 3 ? dd[2 * nmax + e2] : 0.0};
                        double ps[3] = {sq[e0], sq[nmax + e1], m->dim == 3 ? sq[2 * nmax + e2] : 0.0};
                        double K;
                        if (!pair_weight(m->dim, pd, ps, h[i], cutoff, f32_decision, &K)) continue;
                        int64_t c = idx[0] + (int64_t)m->n[0] * (idx[1] + (int64_t)m->n[1] * idx[2]);
                        double w = K / Z[i];
                        for (int k = 0; k < C; ++k) acc[k * M + c] += w * (q[k * N + i] * amount_scale);
                    }
        }
        free(L);
        free(dd);
        free(sq);
    }
    for (int64_t c = 0; c < M; ++c) {
        double cs = cell_scale ? cell_scale[c] : 1.0;
        for (int k = 0; k < C; ++k) S[k * M + c] = -scale * cs * acc[k * M + c] / Vc;
    }
    if (Z_out)
        for (int64_t i = 0; i < N; ++i) Z_out[i] = Z[i];
    free(Z);
    free(acc);
}

/* ------------------------------------------------------------------------ */
/* PSI-CELL box counting (eqs. vol-avg-discrete and coupling-terms-         */
/* definition): S(c) = -(w / V_c) * cell_scale(c) * sum_{p in c} phi_p,     */
/* with w the statistical weight of one computational particle (real        */
/* droplets it stands for).  Cell of a particle: floor((x - lo)/dx) per      */
/* axis; periodic axes wrap; on a closed axis x == hi goes to the last cell */
/* and any other outside position is skipped.  Particles with non-finite    */
/* inputs are skipped.  Returns the number of particles skipped; of these,  */
/* the ones with a non-finite input go to *nonfinite_out.                   */
/* ------------------------------------------------------------------------ */
int64_t orc_psicell_cell_of(const orc_mesh* m, const double* xp)
{
    int64_t lin = 0, stride = 1;
    for (int a = 0; a < m->dim; ++a) {
        if (!isfinite(xp[a])) return -1;
        double g = floor((xp[a] - m->lo[a]) / cell_width(m, a));
        if (!(fabs(g) < 9.0e15)) return -1;
        int64_t k = (int64_t)g;
        if (m->periodic[a]) {
            k %= m->n[a];
            if (k < 0) k += m->n[a];
        } else if (k < 0 || k >= m->n[a]) {
            if (k == m->n[a] && xp[a] == m->hi[a])
                k = m->n[a] - 1;
            else
                return -1;
        }
        lin += k * stride;
        stride *= m->n[a];
    }
    return lin;
}

int64_t orc_psicell(const orc_mesh* m, int64_t Np, const double* x, const double* v,
                    const double* ug, const double* r, double rho_d, double mu, double delta,
                    double weight, const double* cell_scale, double* S /* C x M */,
                    int64_t* counts /* M, nullable */, int64_t* nonfinite_out /* nullable */)
{
    int64_t nonfinite = 0;
    int C = 1 + m->dim;
    int64_t M = 1;
    for (int a = 0; a < m->dim; ++a) M *= m->n[a];
    double* acc = (double*)calloc((size_t)(C * M), sizeof(double));
    if (counts) memset(counts, 0, sizeof(int64_t) * (size_t)M);
    int64_t skipped = 0;
    for (int64_t p = 0; p < Np; ++p) {
        double xp[3], vp[3], up[3], phi[4];
        for (int a = 0; a < m->dim; ++a) {
            xp[a] = x[a * Np + p];
            vp[a] = v[a * Np + p];
            up[a] = ug[a * Np + p];
        }
        int64_t c = orc_psicell_cell_of(m, xp);
        if (!all_finite(xp, m->dim)) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        if (c < 0) {
            ++skipped;
            continue;
        }
        if (!all_finite(vp, m->dim) || !all_finite(up, m->dim) || !isfinite(r[p])) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        orc_droplet_phi(m->dim, r[p], vp, up, rho_d, mu, delta, phi, 0, 0, 0);
        if (!all_finite(phi, C)) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        for (int k = 0; k < C; ++k) acc[k * M + c] += phi[k];
        if (counts) counts[c] += 1;
    }
    double Vc = cell_volume(m);
    for (int64_t c = 0; c < M; ++c) {
        double cs = cell_scale ? cell_scale[c] : 1.0;
        for (int k = 0; k < C; ++k) S[k * M + c] = -(weight / Vc) * cs * acc[k * M + c];
    }
    free(acc);
    if (nonfinite_out) *nonfinite_out = nonfinite;
    return skipped;
}

/* ------------------------------------------------------------------------ */
/* Cloud-in-cell (CIC) accumulation, the linear-interpolation comparator   */
/* named beside PSI-CELL: each particle's phi is shared among the 2^dim     */
/* cell centres around it with the per-axis hat weights 1 - |d|/dx (d the  */
/* offset to the centre), i.e. the corners of the dual cell holding it.    */
/* On a periodic axis the stencil wraps; on a closed axis the weight of a  */
/* centre beyond the wall goes to the boundary cell, so every particle     */
/* deposits its whole phi.  S(c) = -(w/V_c) cs(c) sum_p W_cp phi_p, and    */
/* wsum(c) = sum_p W_cp.  Particles outside a closed box (x == hi belongs  */
/* to the box) and particles with a non-finite input are skipped.          */
/* ------------------------------------------------------------------------ */
int64_t orc_cic(const orc_mesh* m, int64_t Np, const double* x, const double* v, const double* ug,
                const double* r, double rho_d, double mu, double delta, double weight,
                const double* cell_scale, double* S /* C x M */, double* wsum /* M, nullable */,
                int64_t* nonfinite_out /* nullable */)
{
    int C = 1 + m->dim;
    int64_t M = 1;
    for (int a = 0; a < m->dim; ++a) M *= m->n[a];
    double* acc = (double*)calloc((size_t)(C * M), sizeof(double));
    double* ws = (double*)calloc((size_t)M, sizeof(double));
    int64_t skipped = 0, nonfinite = 0;
    for (int64_t p = 0; p < Np; ++p) {
        double xp[3] = {0, 0, 0}, vp[3], up[3], phi[4];
        for (int a = 0; a < m->dim; ++a) {
            xp[a] = x[a * Np + p];
            vp[a] = v[a * Np + p];
            up[a] = ug[a * Np + p];
        }
        /* as in PSI-CELL: the position decides first (outside a closed box */
        /* is counted as outside whatever the other inputs)                */
        if (!all_finite(xp, m->dim)) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        if (orc_psicell_cell_of(m, xp) < 0) {
            ++skipped;
            continue;
        }
        if (!all_finite(vp, m->dim) || !all_finite(up, m->dim) || !isfinite(r[p])) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        orc_droplet_phi(m->dim, r[p], vp, up, rho_d, mu, delta, phi, 0, 0, 0);
        if (!all_finite(phi, C)) {
            ++skipped;
            ++nonfinite;
            continue;
        }
        /* per axis: the two centres around x and their weights */
        int64_t kk[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        double ww[3][2] = {{1, 0}, {1, 0}, {1, 0}};
        for (int a = 0; a < m->dim; ++a) {
            int64_t n = m->n[a];
            double u = (xp[a] - m->lo[a]) / cell_width(m, a) - 0.5;
            double fl = floor(u);
            double f = u - fl;
            int64_t k = (int64_t)fl;
            if (m->periodic[a]) {
                int64_t k0 = k % n;
                if (k0 < 0) k0 += n;
                kk[a][0] = k0;
                kk[a][1] = (k0 + 1) % n;
            } else if (k < 0) {
                kk[a][0] = kk[a][1] = 0;
            } else if (k >= n - 1) {
                kk[a][0] = kk[a][1] = n - 1;
            } else {
                kk[a][0] = k;
                kk[a][1] = k + 1;
            }
            ww[a][0] = 1.0 - f;
            ww[a][1] = f;
        }
        int corners = 1 << m->dim;
        for (int q = 0; q < corners; ++q) {
            double W = 1.0;
            int64_t lin = 0, stride = 1;
            for (int a = 0; a < m->dim; ++a) {
                int b = (q >> a) & 1;
                W *= ww[a][b];
                lin += kk[a][b] * stride;
                stride *= m->n[a];
            }
            for (int k = 0; k < C; ++k) acc[k * M + lin] += W * phi[k];
            ws[lin] += W;
        }
    }
    double Vc = cell_volume(m);
    for (int64_t c = 0; c < M; ++c) {
        double cs = cell_scale ? cell_scale[c] : 1.0;
        for (int k = 0; k < C; ++k) S[k * M + c] = -(weight / Vc) * cs * acc[k * M + c];
        if (wsum) wsum[c] = ws[c];
    }
    free(acc);
    free(ws);
    if (nonfinite_out) *nonfinite_out = nonfinite;
    return skipped;
}

/* ------------------------------------------------------------------------ */
/* Trajectory producer: droplets advanced over one carrier time step in an  */
/* analytic gas field (eqs. Stokes-drag, evap-model and Jacobian-evolution, */
/* dimensional forms), with the droplet's mass and momentum contributions   */
/* summed over the substeps (App. B steps 1a-1b).                           */
/*   x' = v,  v' = (u(x) - v)/tau(r),  r' = delta/(2 r),                    */
/*   J' = K,  K' = (grad u(x) J - K)/tau(r),                                */
/*   Q_mass' = mdot = 4 pi rho r^2 r',  Q_mom' = F + mdot v,                */
/*   tau = 2 rho r^2/(9 mu), F = m (u - v)/tau, m = 4/3 pi rho r^3,         */
/* integrated with the classical fourth-order Runge-Kutta method over       */
/* `substeps` equal substeps; the step's source rates are phibar = Q/dt.    */
/* The gas field is u = u0 + G x + (a periodic part by kind): 0 none, 1 the */
/* Taylor-Green vortex U (sin(w x) cos(w y), -cos(w x) sin(w y)) in 2-D, 2  */
/* the ABC flow U (A sin(w z + pz) + C cos(w y + py), B sin(w x + px) +     */
/* A cos(w z + pz), C sin(w y + py) + B cos(w x + px)) in 3-D; w = 2 pi k.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;
    double U, k;
    double abc[3];
    double phase[3];
    double u0[3];
    double G[9];   /* du_a/dx_b at G[a*3 + b] */
} orc_flow;

void orc_flow_eval(int dim, const orc_flow* f, const double* x, double* u, double* gu /* dim*dim */)
{
    for (int a = 0; a < dim; ++a) {
        u[a] = f->u0[a];
        for (int b = 0; b < dim; ++b) {
            u[a] += f->G[a * 3 + b] * x[b];
            gu[a * dim + b] = f->G[a * 3 + b];
        }
    }
    double w = 2.0 * ORC_PI * f->k, U = f->U;
    if (f->kind == 1 && dim == 2) {
        double sx = sin(w * x[0]), cx = cos(w * x[0]), sy = sin(w * x[1]), cy = cos(w * x[1]);
        u[0] += U * sx * cy;
        u[1] -= U * cx * sy;
        gu[0] += U * w * cx * cy;
        gu[1] -= U * w * sx * sy;
        gu[2] += U * w * sx * sy;
        gu[3] -= U * w * cx * cy;
    } else if (f->kind == 2 && dim == 3) {
        double A = f->abc[0], B = f->abc[1], C = f->abc[2];
        double ax = w * x[0] + f->phase[0], ay = w * x[1] + f->phase[1], az = w * x[2] + f->phase[2];
        double sx = sin(ax), cx = cos(ax), sy = sin(ay), cy = cos(ay), sz = sin(az), cz = cos(az);
        u[0] += U * (A * sz + C * cy);
        u[1] += U * (B * sx + A * cz);
        u[2] += U * (C * sy + B * cx);
        gu[0 * 3 + 1] -= U * C * w * sy;
        gu[0 * 3 + 2] += U * A * w * cz;
        gu[1 * 3 + 0] += U * B * w * cx;
        gu[1 * 3 + 2] -= U * A * w * sz;
        gu[2 * 3 + 0] -= U * B * w * sx;
        gu[2 * 3 + 1] += U * C * w * cy;
    }
}

/* State vector y = [x (d), v (d), r, J (d*d), K (d*d), Q (1 + d)] and its  */
/* time derivative.                                                          */
static void producer_rhs(int dim, const orc_flow* f, double rho, double mu, double delta, const double* y,
                         double* dy)
{
    const double* x = y;
    const double* v = y + dim;
    double r = y[2 * dim];
    const double* J = y + 2 * dim + 1;
    const double* K = J + dim * dim;
    double u[3], gu[9];
    orc_flow_eval(dim, f, x, u, gu);
    double tau = 2.0 * rho * r * r / (9.0 * mu);
    double m = (4.0 / 3.0) * ORC_PI * rho * r * r * r;
    double rdot = delta / (2.0 * r);
    double mdot = 4.0 * ORC_PI * rho * r * r * rdot;
    double* dx = dy;
    double* dv = dy + dim;
    double* dJ = dy + 2 * dim + 1;
    double* dK = dJ + dim * dim;
    double* dQ = dK + dim * dim;
    for (int a = 0; a < dim; ++a) {
        dx[a] = v[a];
        dv[a] = (u[a] - v[a]) / tau;
    }
    dy[2 * dim] = rdot;
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double gJ = 0.0;
            for (int c = 0; c < dim; ++c) gJ += gu[a * dim + c] * J[c * dim + b];
            dJ[a * dim + b] = K[a * dim + b];
            dK[a * dim + b] = (gJ - K[a * dim + b]) / tau;
        }
    dQ[0] = mdot;
    for (int a = 0; a < dim; ++a) {
        double F = m * (u[a] - v[a]) / tau;
        dQ[1 + a] = F + mdot * v[a];
    }
}

/* Advances N droplets (binary64 planes x, v: dim x N; J, K: dim*dim x N;    */
/* r: N, updated in place) by dt in `substeps` RK4 substeps and writes the   */
/* step's source rates phibar (1 + dim planes of N).  A droplet is skipped   */
/* (valid = 0, state left as it was, phibar 0) if any input is not finite,   */
/* r <= 0, it would evaporate within the step (r^2 + delta dt <= 0) or the   */
/* result is not finite.  Returns the number skipped.                        */
int64_t orc_advance(int dim, int64_t N, double* x, double* v, double* J, double* K, double* r,
                    const orc_flow* flow, double rho_d, double mu, double delta, double dt, int substeps,
                    double* phibar, int* valid)
{
    int C = 1 + dim;
    int ny = 2 * dim + 1 + 2 * dim * dim + C;
    int64_t skipped = 0;
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t i = 0; i < N; ++i) {
        double y[40], k1[40], k2[40], k3[40], k4[40], yt[40];
        for (int a = 0; a < dim; ++a) {
            y[a] = x[a * N + i];
            y[dim + a] = v[a * N + i];
        }
        y[2 * dim] = r[i];
        for (int e = 0; e < dim * dim; ++e) {
            y[2 * dim + 1 + e] = J[e * N + i];
            y[2 * dim + 1 + dim * dim + e] = K[e * N + i];
        }
        for (int k = 0; k < C; ++k) y[ny - C + k] = 0.0;
        int ok = all_finite(y, ny) && r[i] > 0.0 && r[i] * r[i] + delta * dt > 0.0;
        double h = dt / (double)substeps;
        for (int s = 0; s < substeps && ok; ++s) {
            producer_rhs(dim, flow, rho_d, mu, delta, y, k1);
            for (int e = 0; e < ny; ++e) yt[e] = y[e] + 0.5 * h * k1[e];
            producer_rhs(dim, flow, rho_d, mu, delta, yt, k2);
            for (int e = 0; e < ny; ++e) yt[e] = y[e] + 0.5 * h * k2[e];
            producer_rhs(dim, flow, rho_d, mu, delta, yt, k3);
            for (int e = 0; e < ny; ++e) yt[e] = y[e] + h * k3[e];
            producer_rhs(dim, flow, rho_d, mu, delta, yt, k4);
            for (int e = 0; e < ny; ++e) y[e] = y[e] + (h / 6.0) * (k1[e] + 2.0 * k2[e] + 2.0 * k3[e] + k4[e]);
        }
        ok = ok && all_finite(y, ny) && y[2 * dim] > 0.0;
        if (!ok) {
            ++skipped;
            valid[i] = 0;
            for (int k = 0; k < C; ++k) phibar[k * N + i] = 0.0;
            continue;
        }
        valid[i] = 1;
        for (int a = 0; a < dim; ++a) {
            x[a * N + i] = y[a];
            v[a * N + i] = y[dim + a];
        }
        r[i] = y[2 * dim];
        for (int e = 0; e < dim * dim; ++e) {
            J[e * N + i] = y[2 * dim + 1 + e];
            K[e * N + i] = y[2 * dim + 1 + dim * dim + e];
        }
        for (int k = 0; k < C; ++k) phibar[k * N + i] = y[ny - C + k] / dt;
    }
    return skipped;
}

/* Estimator terms of advanced droplets: det J, n = n0/|det J| (eq. FLA-COM), */
/* h = h0 |det J| (eq. smoothing-length) and q = n phibar; a droplet is      */
/* skipped if it was not advanced, det J = 0 or a term is not finite.        */
int64_t orc_state_terms(int dim, int64_t N, const double* x, const double* J, const double* phibar,
                        const int* valid_in, const double* n0, double n0_scalar, double h0, double* det_out,
                        double* h_out, double* n_out, double* q_out, int* valid_out)
{
    int C = 1 + dim;
    int64_t skipped = 0;
    for (int64_t i = 0; i < N; ++i) {
        double Ji[9], xi[3], ph[4];
        for (int e = 0; e < dim * dim; ++e) Ji[e] = J[e * N + i];
        for (int a = 0; a < dim; ++a) xi[a] = x[a * N + i];
        for (int k = 0; k < C; ++k) ph[k] = phibar[k * N + i];
        double n0i = n0 ? n0[i] : n0_scalar;
        double det = orc_det(dim, Ji);
        double adet = fabs(det);
        int ok = valid_in[i] && all_finite(Ji, dim * dim) && all_finite(xi, dim) && all_finite(ph, C) &&
                 isfinite(n0i) && isfinite(det) && det != 0.0;
        double h = h0 * adet;
        double n = n0i / adet;
        if (ok && !(isfinite(h) && h > 0.0 && isfinite(n))) ok = 0;
        if (!ok) ++skipped;
        det_out[i] = det;
        h_out[i] = ok ? h : 0.0;
        n_out[i] = ok ? n : 0.0;
        for (int k = 0; k < C; ++k) q_out[k * N + i] = ok ? n * ph[k] : 0.0;
        valid_out[i] = ok;
    }
    return skipped;
}

/* ------------------------------------------------------------------------ */
/* App. A scaling factors.                                                   */
/*   M_scal = N_ref tau_FLA / (N_FLA tau_ref)                   (eq. A.6)    */
/*   V_scal = V_cell N_FLA / (A_inj v_inj tau_FLA)              (eq. A.12)   */
/*   n_hat  = M_scal * V_scal                                   (eq. A.13)   */
/* ------------------------------------------------------------------------ */
void orc_app_a_scaling(double N_ref, double tau_ref, double N_fla, double tau_fla,
                       double V_cell, double A_inj, double v_inj, double out[3])
{
    double M_scal = (N_ref * tau_fla) / (N_fla * tau_ref);
    double V_fla = (A_inj * (v_inj * tau_fla)) / N_fla;
    double V_scal = V_cell / V_fla;
    out[0] = M_scal;
    out[1] = V_scal;
    out[2] = M_scal * V_scal;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
