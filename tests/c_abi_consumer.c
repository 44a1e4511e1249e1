/* A plain C caller of the library's host-only entry points: it includes ras.h,
 * links libras.so and uses no Python.  Every expected value is computed here
 * from its definition, not taken from the library:
 *   - the owner of a grid point under a regular 2-D partition (axis bounds
 *     floor(i N / p), Sec. 3.2.1);
 *   - Omega_p = the points within graph distance `overlap` of subdomain p's
 *     block, ext(Omega_p) = the next layer (Sec. 2.1, Fig. 1); on a rectangular
 *     grid graph the distance to a block is the Manhattan distance;
 *   - the communication volume (Sec. 3.2.1, Fig. 2) by counting;
 *   - the band factor by multiplying it out: L L^T = A[Omega_p, Omega_p]
 *     (Sec. 3.3.1), and the sparse factor likewise in its elimination order;
 *   - the asynchronous stop rule's documented precedence (Sec. 3.3.2).
 * Exit status 0 when every check holds; each failure is printed.  */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ras.h"

static int failures = 0;

#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            ++failures;                           \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);         \
            fputc('\n', stderr);                  \
        }                                         \
    } while (0)

enum { NX = 16, NY = 12, PX = 4, PY = 3, P = PX * PY, N = NX * NY, GAMMA = 2 };

/* five-point Laplacian, natural order g = i + NX j, columns ascending */
static int64_t rp[N + 1];
static int32_t ci[5 * N];
static double va[5 * N];

static void laplacian(void) {
    int64_t k = 0;
    for (int j = 0; j < NY; ++j)
        for (int i = 0; i < NX; ++i) {
            const int g = i + NX * j;
            rp[g] = k;
            if (j > 0) { ci[k] = g - NX; va[k++] = -1.0; }
            if (i > 0) { ci[k] = g - 1; va[k++] = -1.0; }
            ci[k] = g; va[k++] = 4.0;
            if (i < NX - 1) { ci[k] = g + 1; va[k++] = -1.0; }
            if (j < NY - 1) { ci[k] = g + NX; va[k++] = -1.0; }
        }
    rp[N] = k;
}

static double a_entry(int r, int c) {
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
        if (ci[k] == c) return va[k];
    return 0.0;
}

static int lo(int b, int extent, int parts) { return (int)(((long)b * extent) / parts); }

/* subdomain owning point (i, j), and the Manhattan distance from (i, j) to block p */
static int owner_of(int i, int j) {
    int bx = 0, by = 0;
    while (bx + 1 < PX && i >= lo(bx + 1, NX, PX)) ++bx;
    while (by + 1 < PY && j >= lo(by + 1, NY, PY)) ++by;
    return bx + PX * by;
}

static int dist_to_block(int i, int j, int p) {
    const int bx = p % PX, by = p / PX;
    const int x0 = lo(bx, NX, PX), x1 = lo(bx + 1, NX, PX) - 1;
    const int y0 = lo(by, NY, PY), y1 = lo(by + 1, NY, PY) - 1;
    const int dx = i < x0 ? x0 - i : (i > x1 ? i - x1 : 0);
    const int dy = j < y0 ? y0 - j : (j > y1 ? j - y1 : 0);
    return dx + dy;
}

static void check_sets_and_volume(ras_plan* plan) {
    int32_t owner[N];
    int64_t optr[P + 1];
    CHECK(ras_plan_sets(plan, owner, optr, NULL) == RAS_OK, "ras_plan_sets sizes: %s", ras_last_error());
    int32_t* oidx = malloc(sizeof(int32_t) * (size_t)optr[P]);
    CHECK(ras_plan_sets(plan, NULL, optr, oidx) == RAS_OK, "ras_plan_sets: %s", ras_last_error());
    for (int g = 0; g < N; ++g)
        CHECK(owner[g] == owner_of(g % NX, g / NX), "owner of %d: %d, expected %d", g, owner[g],
              owner_of(g % NX, g / NX));
    for (int p = 0; p < P; ++p) {
        /* Omega_p in ascending global id, exactly the points within GAMMA of the block */
        int64_t k = optr[p];
        for (int g = 0; g < N; ++g)
            if (dist_to_block(g % NX, g / NX, p) <= GAMMA) {
                CHECK(k < optr[p + 1] && oidx[k] == g, "Omega_%d: position %ld should hold %d", p, (long)(k - optr[p]), g);
                ++k;
            }
        CHECK(k == optr[p + 1], "Omega_%d has %ld points, expected %ld", p, (long)(optr[p + 1] - optr[p]),
              (long)(k - optr[p]));
    }
    free(oidx);

    int64_t vol[P * P];
    CHECK(ras_plan_comm_volume(plan, vol) == RAS_OK, "ras_plan_comm_volume: %s", ras_last_error());
    for (int p = 0; p < P; ++p)
        for (int q = 0; q < P; ++q) {
            int64_t expect = 0;
            if (q != p)
                for (int g = 0; g < N; ++g)
                    if (owner_of(g % NX, g / NX) == q && dist_to_block(g % NX, g / NX, p) <= GAMMA + 1) ++expect;
            CHECK(vol[p * P + q] == expect, "volume[%d][%d] = %ld, expected %ld", p, q, (long)vol[p * P + q],
                  (long)expect);
        }
    CHECK(ras_plan_comm_volume(plan, NULL) == RAS_E_ARG, "NULL volume must be RAS_E_ARG");
}

static void check_factors(ras_plan* plan) {
    int64_t optr[P + 1];
    CHECK(ras_plan_sets(plan, NULL, optr, NULL) == RAS_OK, "sets");
    int32_t* oidx = malloc(sizeof(int32_t) * (size_t)optr[P]);
    CHECK(ras_plan_sets(plan, NULL, optr, oidx) == RAS_OK, "sets");
    int max_w = 0;
    for (int p = 0; p < P; ++p) {
        const int m = (int)(optr[p + 1] - optr[p]);
        const int32_t* om = oidx + optr[p];
        /* the local matrix's lower half-bandwidth, at least 1 */
        int wexp = 1;
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < r; ++c)
                if (a_entry(om[r], om[c]) != 0.0) {
                    if (r - c > wexp) wexp = r - c;
                    break;
                }
        int32_t w = -1;
        CHECK(ras_plan_factor(plan, p, NULL, &w) == RAS_OK, "factor query %d: %s", p, ras_last_error());
        CHECK(w == wexp, "subdomain %d: half-bandwidth %d, expected %d", p, w, wexp);
        if (w > max_w) max_w = w;
        double* band = calloc((size_t)m * (size_t)(w + 1), sizeof(double));
        CHECK(ras_plan_factor(plan, p, band, &w) == RAS_OK, "factor %d: %s", p, ras_last_error());
        /* (L L^T)_rc over the band against A[Omega_p, Omega_p]; zero beyond it */
        double err = 0.0;
        for (int r = 0; r < m; ++r) {
            CHECK(band[(size_t)r * (w + 1) + w] > 0.0, "subdomain %d: non-positive diagonal at row %d", p, r);
            for (int c = (r - w > 0 ? r - w : 0); c <= r; ++c) {
                double s = 0.0;
                for (int k = (r - w > 0 ? r - w : 0); k <= c; ++k)
                    if (k >= c - w) s += band[(size_t)r * (w + 1) + (k - r + w)] * band[(size_t)c * (w + 1) + (k - c + w)];
                const double d = fabs(s - a_entry(om[r], om[c]));
                if (d > err) err = d;
            }
            for (int c = 0; c < r - w; ++c) CHECK(a_entry(om[r], om[c]) == 0.0, "entry outside the band");
        }
        CHECK(err <= 1e-12 * 8.0, "subdomain %d: max |L L^T - A_p| = %g", p, err);
        free(band);
    }
    ras_plan_stats st;
    CHECK(ras_plan_get_stats(plan, &st) == RAS_OK, "stats");
    CHECK(st.max_band == max_w, "stats.max_band %d, expected %d", st.max_band, max_w);
    free(oidx);
}

/* Sparse factor (nested-dissection order): perm is a permutation of the local
 * rows, L is lower triangular with a positive diagonal and columns ascending,
 * and L L^T = A_p[perm, perm] entry by entry (the dense product, small boxes).  */
static void check_sparse_factors(ras_plan* plan) {
    int64_t optr[P + 1];
    CHECK(ras_plan_sets(plan, NULL, optr, NULL) == RAS_OK, "sets");
    int32_t* oidx = malloc(sizeof(int32_t) * (size_t)optr[P]);
    CHECK(ras_plan_sets(plan, NULL, optr, oidx) == RAS_OK, "sets");
    for (int p = 0; p < P; ++p) {
        const int m = (int)(optr[p + 1] - optr[p]);
        const int32_t* om = oidx + optr[p];
        int64_t nnz = -1;
        CHECK(ras_plan_sparse_factor(plan, p, NULL, NULL, NULL, NULL, NULL, &nnz) == RAS_OK && nnz >= 0,
              "sparse query %d: %s", p, ras_last_error());
        int32_t* perm = malloc(sizeof(int32_t) * (size_t)m);
        int64_t* lp = malloc(sizeof(int64_t) * (size_t)(m + 1));
        int32_t* lc = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        double* lv = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        double* dg = malloc(sizeof(double) * (size_t)m);
        double* L = calloc((size_t)m * (size_t)m, sizeof(double));
        int* seen = calloc((size_t)m, sizeof(int));
        CHECK(ras_plan_sparse_factor(plan, p, perm, lp, lc, lv, dg, &nnz) == RAS_OK, "sparse %d: %s", p,
              ras_last_error());
        for (int k = 0; k < m; ++k) {
            CHECK(perm[k] >= 0 && perm[k] < m && !seen[perm[k]], "subdomain %d: perm is not a permutation", p);
            if (perm[k] >= 0 && perm[k] < m) seen[perm[k]] = 1;
            CHECK(dg[k] > 0.0, "subdomain %d: non-positive pivot at step %d", p, k);
            L[(size_t)k * m + k] = dg[k];
            for (int64_t e = lp[k]; e < lp[k + 1]; ++e) {
                CHECK(lc[e] >= 0 && lc[e] < k, "subdomain %d: entry (%d, %d) not strictly lower", p, k, lc[e]);
                CHECK(e == lp[k] || lc[e] > lc[e - 1], "subdomain %d: row %d columns not ascending", p, k);
                if (lc[e] >= 0 && lc[e] < k) L[(size_t)k * m + lc[e]] = lv[e];
            }
        }
        CHECK(lp[0] == 0 && lp[m] == nnz, "subdomain %d: row pointers", p);
        double err = 0.0;
        for (int r = 0; r < m; ++r)
            for (int c = 0; c <= r; ++c) {
                double sum = 0.0;
                for (int k = 0; k <= c; ++k) sum += L[(size_t)r * m + k] * L[(size_t)c * m + k];
                const double d = fabs(sum - a_entry(om[perm[r]], om[perm[c]]));
                if (d > err) err = d;
            }
        CHECK(err <= 8e-12, "subdomain %d: max |L L^T - P A_p P^T| = %g", p, err);
        free(perm); free(lp); free(lc); free(lv); free(dg); free(L); free(seen);
    }
    free(oidx);
}

static void check_stop_rule(void) {
    /* precedence: diverged, converged, limit, resume */
    CHECK(ras_async_next_step(RAS_KSTOP_DIVERGED, 1e-12, 1e-8, 5, 100, 0.0, 0.0, 0) == RAS_STEP_DIVERGED, "kstop diverged");
    CHECK(ras_async_next_step(RAS_KSTOP_DETECTED, NAN, 1e-8, 5, 100, 0.0, 0.0, 0) == RAS_STEP_DIVERGED, "NaN residual");
    CHECK(ras_async_next_step(RAS_KSTOP_DETECTED, 5e-9, 1e-8, 5, 100, 0.0, 0.0, 0) == RAS_STEP_CONVERGED, "converged");
    CHECK(ras_async_next_step(RAS_KSTOP_EXHAUSTED, 5e-9, 1e-8, 100, 100, 0.0, 0.0, 0) == RAS_STEP_CONVERGED,
          "converged beats the limit");
    CHECK(ras_async_next_step(RAS_KSTOP_DETECTED, 2e-8, 1e-8, 100, 100, 0.0, 0.0, 0) == RAS_STEP_LIMIT, "sweep limit");
    CHECK(ras_async_next_step(RAS_KSTOP_TIME, 2e-8, 1e-8, 5, 100, 3.0, 2.0, 0) == RAS_STEP_LIMIT, "time limit");
    CHECK(ras_async_next_step(RAS_KSTOP_DETECTED, 2e-8, 1e-8, 5, 100, 0.0, 0.0, 1) == RAS_STEP_LIMIT, "ordered");
    CHECK(ras_async_next_step(RAS_KSTOP_DETECTED, 2e-8, 1e-8, 5, 100, 1.0, 0.0, 0) == RAS_STEP_RESUME, "resume");
    CHECK(ras_final_status(RAS_STEP_CONVERGED) == RAS_OK, "final converged");
    CHECK(ras_final_status(RAS_STEP_LIMIT) == RAS_NOT_CONVERGED, "final limit");
    CHECK(ras_final_status(RAS_STEP_DIVERGED) == RAS_E_DIVERGED, "final diverged");
    CHECK(ras_final_status(RAS_STEP_RESUME) == RAS_E_STATE, "resume is not final");
}

int main(void) {
    const char* v = ras_version();
    CHECK(v != NULL && strlen(v) > 0, "ras_version");
    laplacian();
    const ras_csr A = {N, rp, ci, va};
    ras_partition part;
    memset(&part, 0, sizeof part);
    part.kind = RAS_PART_REGULAR_2D;
    part.grid[0] = NX; part.grid[1] = NY; part.grid[2] = 1;
    part.parts[0] = PX; part.parts[1] = PY; part.parts[2] = 1;
    const ras_local chol = {RAS_LOCAL_CHOL_BANDED, 0, RAS_STORAGE_FP64, RAS_TRANSMISSION_DIRICHLET, 1.0};

    ras_plan* plan = NULL;
    CHECK(ras_plan_create(&A, &part, GAMMA, &chol, &plan) == RAS_OK && plan, "ras_plan_create: %s", ras_last_error());
    if (plan) {
        ras_plan_stats st;
        CHECK(ras_plan_get_stats(plan, &st) == RAS_OK, "stats: %s", ras_last_error());
        CHECK(st.n == N && st.nnz == 5 * N - 2 * (NX + NY) && st.parts == P, "stats n %ld nnz %ld parts %d",
              (long)st.n, (long)st.nnz, st.parts);
        int64_t sum = 0;
        for (int p = 0; p < P; ++p)
            for (int g = 0; g < N; ++g) sum += dist_to_block(g % NX, g / NX, p) <= GAMMA;
        CHECK(st.sum_local_rows == sum, "sum |Omega_p| %ld, expected %ld", (long)st.sum_local_rows, (long)sum);
        check_sets_and_volume(plan);
        check_factors(plan);
        ras_plan_destroy(plan);
    }
    ras_plan_destroy(NULL);

    const ras_local sparse = {RAS_LOCAL_CHOL_SPARSE, 0, RAS_STORAGE_FP64, RAS_TRANSMISSION_DIRICHLET, 1.0};
    plan = NULL;
    CHECK(ras_plan_create(&A, &part, GAMMA, &sparse, &plan) == RAS_OK && plan, "sparse plan: %s", ras_last_error());
    if (plan) {
        check_sparse_factors(plan);
        /* a banded factor is not held by a sparse plan */
        double one = 0.0;
        int32_t w = 0;
        CHECK(ras_plan_factor(plan, 0, &one, &w) == RAS_E_STATE, "band factor of a sparse plan");
        ras_plan_destroy(plan);
    }

    /* argument and pattern errors, each with a message */
    plan = NULL;
    CHECK(ras_plan_create(NULL, &part, GAMMA, &chol, &plan) == RAS_E_ARG && plan == NULL, "NULL matrix");
    CHECK(strlen(ras_last_error()) > 0, "message after RAS_E_ARG");
    ras_partition bad = part;
    bad.grid[1] = NY - 1;
    CHECK(ras_plan_create(&A, &bad, GAMMA, &chol, &plan) == RAS_E_ARG, "grid product != n");
    CHECK(ras_plan_create(&A, &part, -1, &chol, &plan) == RAS_E_ARG, "negative overlap");
    /* drop the entry (0, 1): the pattern is no longer symmetric */
    int64_t rp2[N + 1];
    int32_t ci2[5 * N];
    double va2[5 * N];
    int64_t k2 = 0;
    for (int r = 0; r < N; ++r) {
        rp2[r] = k2;
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
            if (!(r == 0 && ci[k] == 1)) { ci2[k2] = ci[k]; va2[k2++] = va[k]; }
    }
    rp2[N] = k2;
    const ras_csr A2 = {N, rp2, ci2, va2};
    CHECK(ras_plan_create(&A2, &part, GAMMA, &chol, &plan) == RAS_E_PATTERN, "unsymmetric pattern");
    CHECK(strlen(ras_last_error()) > 0, "message after RAS_E_PATTERN");

    check_stop_rule();
    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    else printf("c consumer ok (%s)\n", v);
    return failures ? 1 : 0;
}
