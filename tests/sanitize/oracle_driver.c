/* Drives every entry of the FP64 oracle on small random cases (ragged and
 * one-cell axes, periodic and closed, positions outside the box, NaN and
 * det J = 0 inputs, bandwidths from tiny to wider than the box) so that a
 * build under the address and undefined-behaviour sanitizers checks its
 * memory accesses and arithmetic.  Also checks that the brute-force and
 * trajectory-centric forms agree bit for bit.  Exits non-zero on a
 * mismatch; the sanitizers abort on an error. */
#include "../../oracle/fla_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int dim, const int n[3], const int per[3], int64_t N, double hmin, double hmax)
{
    orc_mesh m;
    memset(&m, 0, sizeof m);
    m.dim = dim;
    int64_t M = 1;
    for (int a = 0; a < 3; ++a) {
        m.n[a] = a < dim ? n[a] : 1;
        m.lo[a] = a < dim ? -0.25 * a : 0.0;
        m.hi[a] = a < dim ? m.lo[a] + 1.0 + 0.1 * a : 1.0;
        m.periodic[a] = a < dim ? per[a] : 0;
        M *= m.n[a];
    }
    const int C = 1 + dim;
    double* x = malloc(sizeof(double) * dim * N);
    double* J = malloc(sizeof(double) * dim * dim * N);
    double* v = malloc(sizeof(double) * dim * N);
    double* ug = malloc(sizeof(double) * dim * N);
    double* r = malloc(sizeof(double) * N);
    double *det = malloc(sizeof(double) * N), *h = malloc(sizeof(double) * N), *nn = malloc(sizeof(double) * N);
    double* q = malloc(sizeof(double) * C * N);
    int* valid = malloc(sizeof(int) * N);
    for (int64_t i = 0; i < N; ++i) {
        for (int a = 0; a < dim; ++a) {
            x[a * N + i] = m.lo[a] - 0.2 + 1.4 * (m.hi[a] - m.lo[a]) * urand();
            v[a * N + i] = urand() - 0.5;
            ug[a * N + i] = urand() - 0.5;
        }
        for (int e = 0; e < dim * dim; ++e) J[e * N + i] = (e % (dim + 1) == 0 ? 1.0 : 0.0) + 0.3 * (urand() - 0.5);
        r[i] = 5e-6 + 15e-6 * urand();
    }
    if (N > 2) {
        r[0] = NAN;                                          /* a skipped record */
        for (int e = 0; e < dim * dim; ++e) J[e * N + 1] = 0.0;  /* det J = 0 */
    }
    int64_t sk = orc_trajectory_terms(dim, N, x, J, v, ug, r, NULL, 1e10, 1000.0, 1.81e-5, -1e-9, 1.0, NULL, det, h,
                                      nn, q, valid);
    for (int64_t i = 0; i < N; ++i)
        if (valid[i]) h[i] = hmin * pow(hmax / hmin, urand());
    int bad = N > 2 && sk < 2;
    int64_t* cells = malloc(sizeof(int64_t) * M);
    for (int64_t c = 0; c < M; ++c) cells[c] = c;
    double *S1 = malloc(sizeof(double) * C * M), *S2 = malloc(sizeof(double) * C * M);
    double *d1 = malloc(sizeof(double) * M), *d2 = malloc(sizeof(double) * M);
    int64_t *p1 = malloc(sizeof(int64_t) * M), *p2 = malloc(sizeof(int64_t) * M);
    for (int f32 = 0; f32 < 2; ++f32) {
        orc_nw_cells(&m, N, x, h, q, valid, 4.0, f32, 1.0, NULL, M, cells, S1, d1, p1);
        int64_t lo[3] = {0, 0, 0}, bn[3] = {m.n[0], m.n[1], m.n[2]};
        if (orc_nw_box(&m, N, x, h, q, valid, 4.0, f32, 1.0, NULL, lo, bn, S2, d2, p2) != 0) bad = 1;
        int64_t* bc = malloc(sizeof(int64_t) * M);
        orc_box_cells(&m, lo, bn, bc);
        for (int64_t j = 0; j < M; ++j) {
            int64_t c = bc[j];
            if (d1[c] != d2[j] || p1[c] != p2[j]) bad = 1;
            for (int k = 0; k < C; ++k)
                if (S1[k * M + c] != S2[k * M + j]) bad = 1;
        }
        free(bc);
        /* a box that wraps on periodic axes */
        int64_t lo2[3], bn2[3];
        for (int a = 0; a < 3; ++a) {
            lo2[a] = (a < dim && m.periodic[a]) ? m.n[a] - 1 : 0;
            bn2[a] = a < dim ? (m.n[a] > 1 ? m.n[a] - (m.periodic[a] ? 0 : 1) : 1) : 1;
        }
        int64_t B = bn2[0] * bn2[1] * bn2[2];
        double* S3 = malloc(sizeof(double) * C * B);
        if (orc_nw_box(&m, N, x, h, q, valid, 4.0, f32, 1.0, NULL, lo2, bn2, S3, NULL, NULL) != 0) bad = 1;
        free(S3);
        /* general-mesh form at the lattice centres */
        double* xc = malloc(sizeof(double) * dim * M);
        double L[3];
        for (int a = 0; a < 3; ++a) L[a] = m.hi[a] - m.lo[a];
        for (int64_t c = 0; c < M; ++c) {
            int64_t idx[3];
            cell_coords(&m, c, idx);
            for (int a = 0; a < dim; ++a) xc[a * M + c] = cell_centre(&m, a, idx[a]);
        }
        orc_nw_points(dim, M, xc, m.periodic, L, N, x, h, q, valid, 4.0, f32, 1.0, NULL, M, cells, S2, d2, p2);
        for (int64_t c = 0; c < M; ++c) {
            if (d1[c] != d2[c] || p1[c] != p2[c]) bad = 1;
            for (int k = 0; k < C; ++k)
                if (S1[k * M + c] != S2[k * M + c]) bad = 1;
        }
        free(xc);
        double *Z1 = malloc(sizeof(double) * N), *Z2 = malloc(sizeof(double) * N);
        orc_deposit(&m, N, x, h, q, det, valid, 1e-3, 4.0, f32, 1.0, NULL, S1, Z1);
        orc_deposit_scatter(&m, N, x, h, q, det, valid, 1e-3, 4.0, f32, 1.0, NULL, S2, Z2);
        for (int64_t i = 0; i < N; ++i)
            if (Z1[i] != Z2[i]) bad = 1;
        for (int64_t e = 0; e < C * M; ++e)
            if (fabs(S1[e] - S2[e]) > 1e-12 * (fabs(S1[e]) + 1e-300)) bad = 1;
        free(Z1);
        free(Z2);
    }
    int64_t nf = 0, counts_n = 0;
    int64_t* counts = malloc(sizeof(int64_t) * M);
    (void)orc_psicell(&m, N, x, v, ug, r, 1000.0, 1.81e-5, -1e-9, 1.0, NULL, S1, counts, &nf);
    (void)orc_cic(&m, N, x, v, ug, r, 1000.0, 1.81e-5, -1e-9, 1.0, NULL, S2, d2, &nf);
    for (int64_t c = 0; c < M; ++c) counts_n += counts[c];
    free(counts);
    /* producer: advance a few droplets through each flow kind */
    orc_flow fl;
    memset(&fl, 0, sizeof fl);
    fl.kind = dim == 2 ? 1 : 2;
    fl.U = 0.2;
    fl.k = 1.0;
    for (int a = 0; a < 3; ++a) fl.abc[a] = 1.0;
    double* K = calloc((size_t)dim * dim * N, sizeof(double));
    double* phib = malloc(sizeof(double) * C * N);
    int* ok = malloc(sizeof(int) * N);
    (void)orc_advance(dim, N, x, v, J, K, r, &fl, 1000.0, 1.81e-5, -1e-9, 1e-3, 8, phib, ok);
    (void)orc_state_terms(dim, N, x, J, phib, ok, NULL, 1e10, 0.01, det, h, nn, q, valid);
    double sc[3];
    orc_app_a_scaling(1e5, 1e-3, 10.0, 0.02, 1e-9, 1e-4, 3.0, sc);
    free(K); free(phib); free(ok);
    free(x); free(J); free(v); free(ug); free(r); free(det); free(h); free(nn); free(q); free(valid);
    free(cells); free(S1); free(S2); free(d1); free(d2); free(p1); free(p2);
    if (bad) printf("mismatch: dim %d n %d %d %d periodic %d %d %d\n", dim, n[0], n[1], n[2], per[0], per[1], per[2]);
    (void)counts_n;
    return bad;
}

int main(void)
{
    int bad = 0;
    const int n3a[3] = {7, 5, 4}, n3b[3] = {1, 6, 3}, n2a[3] = {9, 7, 1}, n2b[3] = {1, 11, 1};
    const int pt[3] = {1, 1, 1}, pf[3] = {0, 0, 0}, pm[3] = {1, 0, 1};
    bad |= run_case(3, n3a, pt, 300, 0.005, 0.6);
    bad |= run_case(3, n3a, pf, 300, 0.005, 0.6);
    bad |= run_case(3, n3b, pm, 200, 0.01, 2.0);
    bad |= run_case(2, n2a, pt, 400, 0.002, 0.5);
    bad |= run_case(2, n2b, pm, 200, 0.01, 3.0);
    bad |= run_case(2, n2a, pf, 1, 0.1, 0.1);
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
