/*
 * oracle.c -- plain, slow, single-threaded CPU FP64 reference of
 * block-ILU0-preconditioned BiCGStab on BCSR matrices with 3x3 blocks.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library: its own BCSR walk, its own
 * 3x3 inverse, its own orderings.  Built with gcc -O2 -ffp-contract=off so
 * every multiply and add rounds separately, in program order.
 *
 * What it follows (paper: Qiu et al., "An Evaluation and Comparison of GPU
 * Hardware and Solver Libraries for Accelerating the OPM Flow Reservoir
 * Simulator"):
 *   - BCSR layout: values, row pointers and column indices; blocks stored
 *     row-major, one after another (Section "OPM Flow"; Section "Sparse
 *     Matrix-Vector multiplication", last paragraph).
 *   - ILU0 decomposition: Algorithm 2 ("ILU0 decomposition"), restricted to
 *     the sparsity pattern S, with block entries.  Reading for blocks: the
 *     scalar "e = d * a_ir" with d = 1/a_rr becomes the block product
 *     a_ir * inv(a_rr) (right multiplication), the only order for which
 *     L*U reproduces A on S.
 *   - ILU0 application: equations (3) and (4) of Section "ILU0": forward
 *     substitution with the unit lower factor, then backward substitution
 *     with the upper factor.  The body of Algorithm 1 is not printed; the
 *     substitutions are reconstructed from the equations.
 *   - Level scheduling and graph colouring: Section "ILU0" of the
 *     implementation chapter.  LS levels respect direct and indirect lower
 *     dependencies; GC is DSatur (Brelaz, "New methods to color the
 *     vertices of a graph", CACM 1979) on the symmetrised graph, ties broken
 *     by degree, then by the smaller index (the paper does not name its
 *     colouring algorithm; fewer colours mean fewer launches).
 *     Rows are then sorted stably by (level or colour, original index) and a
 *     reordered copy of the matrix and of b is made.
 *   - BiCGStab: named in Section "Bicgstab solver" (spmv, axpy, norm, dot)
 *     but not written out; the preconditioned form of van der Vorst (1992)
 *     as given in Barrett et al., "Templates" (1994), with x0 = 0.
 *   - Stopping rule: relative reduction 1e-2 of the residual 2-norm, at
 *     most 200 iterations (Section "Bicgstab solver"), tested after both the
 *     half step (on s) and the full step (on r).
 *   - Block-Jacobi-ILU0 (Section "Block-Jacobi-ILU0"): the preconditioner is
 *     built from a "Jacobi matrix" that keeps only the blocks coupling rows
 *     of the same partition; the full matrix stays in the SpMV.  The ordering
 *     is computed on the Jacobi matrix's pattern.  The partition is an input.
 *   - Standard wells kept separate (Section "Well Contributions",
 *     Algorithm 5): the operator is y = A x - sum over wells of
 *     C^T D^-1 B x; B and C hold one 4x3 block per perforated cell, D^-1 is
 *     one 4x4 block per well.  The preconditioner is ILU0 of A alone.
 *   - Restarted GMRES, the simulator's other Krylov solver (Section "OPM
 *     Flow": bicgstab by default, or restarted GMRES): not written out in
 *     the paper; right-preconditioned GMRES(m) as in Saad, "Iterative
 *     Methods for Sparse Linear Systems" (GMRES with right
 *     preconditioning), x0 = 0, Arnoldi with classical Gram-Schmidt applied
 *     twice, Givens rotations for the small least-squares problem, the same
 *     relative-reduction test on the residual estimate after every step.
 *   - Zero-diagonal check (Section "Profiling", runtime breakdown table):
 *     a missing diagonal block is a pattern error; a singular diagonal block
 *     during the decomposition is a zero pivot.
 *
 * The mixed-precision apply (FP32 factors and arithmetic) follows one
 * reading of its rounding: input rounded to FP32, each product and each sum
 * rounded separately in row order; a hand-derived fixture pins it bit for
 * bit.  The GPU path contracts multiply-adds, so it is compared with this
 * apply within an element-wise FP32 error bound, not bit for bit.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_BREAKDOWN 2
#define ORC_INVALID -1
#define ORC_BAD_PATTERN -3
#define ORC_MISSING_DIAG -4
#define ORC_ZERO_PIVOT -5
#define ORC_NON_FINITE -6
#define ORC_NO_MEMORY -7

#define ORC_ORDER_NATURAL 0
#define ORC_ORDER_LEVEL 1
#define ORC_ORDER_COLOUR 2
#define ORC_ORDER_RCM_LEVEL 3

#define ORC_PREC_ILU_F64 0
#define ORC_PREC_ILU_F32 1
#define ORC_PREC_NONE 2

typedef struct {
    int status;
    int half_steps;
    double r0_norm;
    double final_norm;
    double true_rel_residual;
} orc_info;

int orc_bicgstab_split(int n, const int *rowptr, const int *colidx, const double *vals, const int *mrow,
                       const int *mcol, const double *lu, const double *dinv, int precond_kind, const double *b,
                       double reduction, int max_iter, double *x, orc_info *info, double *trace);
int orc_solve_jacobi(int n, const int *rowptr, const int *colidx, const double *vals, const int *part,
                     const double *b, int ordering, int precond_kind, double reduction, int max_iter, double *x,
                     orc_info *info, int *perm_out, int *n_sets, int *bad_row);
int orc_solve_wells(int n, const int *rowptr, const int *colidx, const double *vals, const int *part, int n_wells,
                    const int *well_ptr, const int *perf_row, const double *B, const double *C, const double *Dinv,
                    const double *b, int ordering, int precond_kind, double reduction, int max_iter, double *x,
                    orc_info *info, int *perm_out, int *n_sets, int *bad_row);

/* ---------------------------------------------------------------- pattern */

/* Sorted, unique, in-range columns; a diagonal block in every row.
 * Returns 0, ORC_BAD_PATTERN or ORC_MISSING_DIAG; *bad_row names the row. */
int orc_validate(int n, const int *rowptr, const int *colidx, int *bad_row)
{
    *bad_row = -1;
    if (n < 0 || rowptr[0] != 0) return ORC_BAD_PATTERN;
    for (int i = 0; i < n; ++i) {
        int has_diag = 0;
        if (rowptr[i + 1] < rowptr[i]) { *bad_row = i; return ORC_BAD_PATTERN; }
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j < 0 || j >= n) { *bad_row = i; return ORC_BAD_PATTERN; }
            if (p > rowptr[i] && colidx[p - 1] >= j) { *bad_row = i; return ORC_BAD_PATTERN; }
            if (j == i) has_diag = 1;
        }
        if (!has_diag) { *bad_row = i; return ORC_MISSING_DIAG; }
    }
    return ORC_OK;
}

static int find_col(const int *rowptr, const int *colidx, int i, int j)
{
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
        if (colidx[p] == j) return p;
    return -1;
}

/* Stable sort of rows by key (counting sort): perm[new] = old. */
static void sort_by_key(int n, const int *key, int nkeys, int *perm)
{
    int *count = calloc((size_t)nkeys + 1, sizeof(int));
    for (int i = 0; i < n; ++i) count[key[i] + 1]++;
    for (int c = 0; c < nkeys; ++c) count[c + 1] += count[c];
    for (int i = 0; i < n; ++i) perm[count[key[i]]++] = i;
    free(count);
}

/* Level scheduling on lower dependencies: level(i) = 1 + max level(j) over
 * j < i with (i,j) in S, 0 when row i has no lower entry.  Rows sorted
 * stably by level.  Returns the number of levels. */
int orc_level_sets(int n, const int *rowptr, const int *colidx, int *level, int *perm)
{
    int nlev = 0;
    for (int i = 0; i < n; ++i) {
        int lv = 0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j < i && level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    sort_by_key(n, level, nlev, perm);
    return nlev;
}

/* Reverse Cuthill-McKee renumbering, then level scheduling of the
 * renumbered rows (a level-reducing reordering before level sets).
 * Graph: i ~ j when (i,j) or (j,i) is in S, i != j.  Cuthill-McKee (1969):
 * while rows are left unnumbered, start a new breadth-first search at the
 * unnumbered row with the fewest neighbours (the smallest index on a tie);
 * each row taken from the front of the queue appends its unnumbered
 * neighbours in order of increasing neighbour count (smaller index first
 * on a tie).  Reverse the whole sequence: pos[row] = n - 1 - (its place).
 * Then level(row) = 1 + max level over its neighbours with a smaller pos
 * (0 if none), visiting rows by increasing pos.  perm lists rows by
 * (level, pos).  Returns the number of levels. */
static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

int orc_rcm_levels(int n, const int *rowptr, const int *colidx, int *level, int *perm)
{
    size_t nnz = (size_t)rowptr[n];
    size_t nn = (size_t)(n > 0 ? n : 1);
    /* neighbour lists: row entries and column entries, sorted, duplicates dropped */
    int *cnt = calloc(nn + 1, sizeof(int));
    for (int i = 0; i < n; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j == i) continue;
            cnt[i + 1]++;
            cnt[j + 1]++;
        }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int *adj = malloc(sizeof(int) * (2 * nnz + 1)), *fill = malloc(sizeof(int) * nn);
    for (int i = 0; i < n; ++i) fill[i] = cnt[i];
    for (int i = 0; i < n; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j == i) continue;
            adj[fill[i]++] = j;
            adj[fill[j]++] = i;
        }
    int *deg = malloc(sizeof(int) * nn);
    for (int i = 0; i < n; ++i) {
        /* row i's list starts at cnt[i]: sorted, duplicates dropped, its
         * first deg[i] entries hold the neighbours */
        int *a = adj + cnt[i];
        int m = cnt[i + 1] - cnt[i];
        qsort(a, (size_t)m, sizeof(int), cmp_int);
        int u = 0;
        for (int k = 0; k < m; ++k)
            if (u == 0 || a[k] != a[u - 1]) a[u++] = a[k];
        deg[i] = u;
    }
    int *order = malloc(sizeof(int) * nn), *seen = calloc(nn, sizeof(int));
    int *cand = malloc(sizeof(int) * nn);
    int len = 0;
    while (len < n) {
        int s = -1;
        for (int i = 0; i < n; ++i)
            if (!seen[i] && (s < 0 || deg[i] < deg[s])) s = i;
        seen[s] = 1;
        order[len++] = s;
        for (int h = len - 1; h < len; ++h) {
            int v = order[h], m = 0;
            for (int k = 0; k < deg[v]; ++k) {
                int j = adj[cnt[v] + k];
                if (!seen[j]) cand[m++] = j;
            }
            /* insertion sort by (neighbour count, index) */
            for (int a = 1; a < m; ++a) {
                int x = cand[a], b = a - 1;
                while (b >= 0 && (deg[cand[b]] > deg[x] || (deg[cand[b]] == deg[x] && cand[b] > x))) {
                    cand[b + 1] = cand[b];
                    --b;
                }
                cand[b + 1] = x;
            }
            for (int a = 0; a < m; ++a) {
                seen[cand[a]] = 1;
                order[len++] = cand[a];
            }
        }
    }
    int *pos = malloc(sizeof(int) * nn);
    for (int k = 0; k < n; ++k) pos[order[k]] = n - 1 - k;
    int nlev = 0;
    for (int k = n - 1; k >= 0; --k) {
        int v = order[k], lv = 0;
        for (int a = 0; a < deg[v]; ++a) {
            int j = adj[cnt[v] + a];
            if (pos[j] < pos[v] && level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[v] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    /* rows by (level, pos): counting by level over rows in pos order */
    int *c2 = calloc((size_t)nlev + 1, sizeof(int));
    for (int i = 0; i < n; ++i) c2[level[i] + 1]++;
    for (int l = 0; l < nlev; ++l) c2[l + 1] += c2[l];
    for (int k = n - 1; k >= 0; --k) perm[c2[level[order[k]]]++] = order[k];
    free(c2); free(pos); free(cand); free(seen); free(order); free(deg); free(fill); free(adj);
    free(cnt);
    return nlev;
}

/* DSatur colouring (Brelaz 1979) on the symmetrised graph (i ~ j when (i,j)
 * or (j,i) is in S, i != j).  n times: among the uncoloured rows take the one
 * whose neighbours hold the most distinct colours (its saturation), ties to
 * the one with more neighbours, then to the smaller index, and give it the
 * smallest colour none of its neighbours holds.  Rows are then sorted stably
 * by colour.  Returns the number of colours.
 *
 * The candidates sit in a binary heap ordered by (saturation, neighbours,
 * -index); a row whose saturation grows is pushed again and its older
 * entries are skipped when they surface. */
typedef struct { int sat, deg, row; } orc_dsat;

static int dsat_first(orc_dsat a, orc_dsat b)
{
    if (a.sat != b.sat) return a.sat > b.sat;
    if (a.deg != b.deg) return a.deg > b.deg;
    return a.row < b.row;
}

static void dsat_push(orc_dsat *h, int *len, orc_dsat k)
{
    int i = (*len)++;
    h[i] = k;
    while (i > 0) {
        int up = (i - 1) / 2;
        if (!dsat_first(h[i], h[up])) break;
        orc_dsat t = h[i]; h[i] = h[up]; h[up] = t;
        i = up;
    }
}

static orc_dsat dsat_pop(orc_dsat *h, int *len)
{
    orc_dsat top = h[0];
    h[0] = h[--(*len)];
    int i = 0;
    for (;;) {
        int a = 2 * i + 1, b = a + 1, m = i;
        if (a < *len && dsat_first(h[a], h[m])) m = a;
        if (b < *len && dsat_first(h[b], h[m])) m = b;
        if (m == i) break;
        orc_dsat t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

int orc_dsatur_colour(int n, const int *rowptr, const int *colidx, int *colour, int *perm)
{
    int nnz = rowptr[n];
    size_t nn = (size_t)(n > 0 ? n : 1), ne = (size_t)(nnz > 0 ? 2 * (size_t)nnz : 1);
    /* transpose pattern, to see (j,i) entries from row i */
    int *tptr = calloc(nn + 1, sizeof(int));
    int *tcol = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *fill = malloc(sizeof(int) * nn);
    for (int p = 0; p < nnz; ++p) tptr[colidx[p] + 1]++;
    for (int i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    memcpy(fill, tptr, sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) tcol[fill[colidx[p]]++] = i;
    /* neighbour lists: row i's pattern and its transpose, self and repeats dropped */
    int *aptr = malloc(sizeof(int) * (nn + 1)), *adj = malloc(sizeof(int) * ne);
    int *stamp = malloc(sizeof(int) * (nn + 1));
    for (int i = 0; i <= n; ++i) stamp[i] = -1;
    aptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        int len = aptr[i];
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (colidx[p] != i && stamp[colidx[p]] != i) { stamp[colidx[p]] = i; adj[len++] = colidx[p]; }
        for (int p = tptr[i]; p < tptr[i + 1]; ++p)
            if (tcol[p] != i && stamp[tcol[p]] != i) { stamp[tcol[p]] = i; adj[len++] = tcol[p]; }
        aptr[i + 1] = len;
    }
    int *sat = calloc(nn, sizeof(int));
    orc_dsat *heap = malloc(sizeof(orc_dsat) * (nn + (size_t)aptr[n] + 1));
    int hlen = 0, ncol = 0, tick = 0;
    for (int c = 0; c <= n; ++c) stamp[c] = -1;
    for (int i = 0; i < n; ++i) {
        colour[i] = -1;
        orc_dsat k = {0, aptr[i + 1] - aptr[i], i};
        dsat_push(heap, &hlen, k);
    }
    for (int done = 0; done < n;) {
        orc_dsat k = dsat_pop(heap, &hlen);
        int v = k.row;
        if (colour[v] >= 0 || k.sat != sat[v]) continue;   /* stale entry */
        /* smallest colour absent from v's neighbours */
        ++tick;
        for (int p = aptr[v]; p < aptr[v + 1]; ++p)
            if (colour[adj[p]] >= 0) stamp[colour[adj[p]]] = tick;
        int c = 0;
        while (stamp[c] == tick) ++c;
        colour[v] = c;
        if (c + 1 > ncol) ncol = c + 1;
        ++done;
        /* saturation of each uncoloured neighbour, counted afresh */
        for (int p = aptr[v]; p < aptr[v + 1]; ++p) {
            int j = adj[p];
            if (colour[j] >= 0) continue;
            ++tick;
            int s = 0;
            for (int q = aptr[j]; q < aptr[j + 1]; ++q) {
                int cj = colour[adj[q]];
                if (cj >= 0 && stamp[cj] != tick) { stamp[cj] = tick; ++s; }
            }
            if (s != sat[j]) {
                sat[j] = s;
                orc_dsat e = {s, aptr[j + 1] - aptr[j], j};
                dsat_push(heap, &hlen, e);
            }
        }
    }
    sort_by_key(n, colour, ncol, perm);
    free(tptr); free(tcol); free(fill); free(aptr); free(adj); free(stamp); free(sat); free(heap);
    return ncol;
}

/* A' = P A P^T with perm[new] = old: row i of A' is row perm[i] of A, its
 * columns renamed by the inverse permutation and re-sorted ascending.
 * Output arrays are sized like the input. */
void orc_permute(int n, const int *rowptr, const int *colidx, const double *vals, const int *perm,
                 int *prow, int *pcol, double *pvals)
{
    int *iperm = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
    prow[0] = 0;
    for (int i = 0; i < n; ++i) {
        int old = perm[i];
        int len = rowptr[old + 1] - rowptr[old];
        int base = prow[i];
        prow[i + 1] = base + len;
        /* insertion sort by new column index; rows are short */
        for (int q = 0; q < len; ++q) {
            int p = rowptr[old] + q;
            int jn = iperm[colidx[p]];
            int t = base + q;
            while (t > base && pcol[t - 1] > jn) {
                pcol[t] = pcol[t - 1];
                memcpy(pvals + 9 * (size_t)t, pvals + 9 * (size_t)(t - 1), 9 * sizeof(double));
                --t;
            }
            pcol[t] = jn;
            memcpy(pvals + 9 * (size_t)t, vals + 9 * (size_t)p, 9 * sizeof(double));
        }
    }
    free(iperm);
}

/* ------------------------------------------------------------ 3x3 algebra */

/* Inverse by the adjugate: inv(A) = adj(A) / det(A).  Returns 0 when the
 * determinant is zero or not finite. */
static int inv3(const double *a, double *out)
{
    double c00 = a[4] * a[8] - a[5] * a[7];
    double c01 = a[5] * a[6] - a[3] * a[8];
    double c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (det == 0.0 || !isfinite(det)) return 0;
    out[0] = c00 / det;
    out[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    out[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    out[3] = c01 / det;
    out[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    out[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    out[6] = c02 / det;
    out[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    out[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    return 1;
}

/* c = a * b, 3x3 row-major */
static void mul3(const double *a, const double *b, double *c)
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += a[3 * r + m] * b[3 * m + k];
            c[3 * r + k] = s;
        }
}

int orc_inv3(const double *a, double *out) { return inv3(a, out); }

/* -------------------------------------------------------------- ILU0 (Alg 2) */

/* Block ILU0 in place, row by row (IKJ form of Algorithm 2): for each row i
 * and each k < i in row i, ascending, L_ik = a_ik inv(U_kk), then
 * a_ij -= L_ik U_kj for every j > k with (k,j) and (i,j) in S.  When row i
 * is done its diagonal block is U_ii and dinv_i = inv(U_ii).
 * On return vals holds L (strictly lower blocks; unit diagonal implied) and
 * U (diagonal and upper blocks); dinv holds inv(U_ii).
 * A singular or non-finite U_ii gives ORC_ZERO_PIVOT and *bad_row = i. */
int orc_ilu0(int n, const int *rowptr, const int *colidx, double *vals, double *dinv, int *bad_row)
{
    double tmp[9];
    *bad_row = -1;
    for (int i = 0; i < n; ++i) {
        int pdiag = -1;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int k = colidx[p];
            if (k == i) pdiag = p;
            if (k >= i) continue;
            mul3(vals + 9 * (size_t)p, dinv + 9 * (size_t)k, tmp);
            memcpy(vals + 9 * (size_t)p, tmp, sizeof tmp);
            for (int q = rowptr[k]; q < rowptr[k + 1]; ++q) {
                int j = colidx[q];
                if (j <= k) continue;
                int t = find_col(rowptr, colidx, i, j);
                if (t < 0) continue; /* (i,j) not in S: fill is dropped */
                double prod[9];
                mul3(vals + 9 * (size_t)p, vals + 9 * (size_t)q, prod);
                for (int e = 0; e < 9; ++e) vals[9 * (size_t)t + e] -= prod[e];
            }
        }
        if (pdiag < 0) { *bad_row = i; return ORC_MISSING_DIAG; }
        if (!inv3(vals + 9 * (size_t)pdiag, dinv + 9 * (size_t)i)) { *bad_row = i; return ORC_ZERO_PIVOT; }
    }
    return ORC_OK;
}

/* Algorithm 2 as printed (KIJ): for each pivot row r, d = inv(a_rr); for each
 * later row i with (i,r) in S: e = a_ir d, a_ir = e, and a_ij -= e a_rj for
 * j > r with (i,j), (r,j) in S.  Same result as orc_ilu0; kept to check that
 * the row-by-row form performs the same updates in the same order. */
int orc_ilu0_kij(int n, const int *rowptr, const int *colidx, double *vals, double *dinv, int *bad_row)
{
    double e[9], prod[9];
    *bad_row = -1;
    for (int r = 0; r < n; ++r) {
        int prr = find_col(rowptr, colidx, r, r);
        if (prr < 0) { *bad_row = r; return ORC_MISSING_DIAG; }
        if (!inv3(vals + 9 * (size_t)prr, dinv + 9 * (size_t)r)) { *bad_row = r; return ORC_ZERO_PIVOT; }
        for (int i = r + 1; i < n; ++i) {
            int pir = find_col(rowptr, colidx, i, r);
            if (pir < 0) continue;
            mul3(vals + 9 * (size_t)pir, dinv + 9 * (size_t)r, e);
            memcpy(vals + 9 * (size_t)pir, e, sizeof e);
            for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
                int j = colidx[q];
                if (j <= r) continue;
                int t = find_col(rowptr, colidx, i, j);
                if (t < 0) continue;
                mul3(e, vals + 9 * (size_t)q, prod);
                for (int m = 0; m < 9; ++m) vals[9 * (size_t)t + m] -= prod[m];
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------- apply (eqs 3, 4) */

/* z = U^{-1} L^{-1} v: forward substitution y_i = v_i - sum_{j<i} L_ij y_j
 * (i ascending), then backward z_i = dinv_i (y_i - sum_{j>i} U_ij z_j)
 * (i descending); sums over a row in ascending column order. */
void orc_apply(int n, const int *rowptr, const int *colidx, const double *lu, const double *dinv,
               const double *v, double *z)
{
    double *y = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        double acc[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j >= i) break;
            const double *b = lu + 9 * (size_t)p;
            for (int r = 0; r < 3; ++r)
                acc[r] -= b[3 * r] * y[3 * j] + b[3 * r + 1] * y[3 * j + 1] + b[3 * r + 2] * y[3 * j + 2];
        }
        y[3 * i] = acc[0]; y[3 * i + 1] = acc[1]; y[3 * i + 2] = acc[2];
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc[3] = {y[3 * i], y[3 * i + 1], y[3 * i + 2]};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j <= i) continue;
            const double *b = lu + 9 * (size_t)p;
            for (int r = 0; r < 3; ++r)
                acc[r] -= b[3 * r] * z[3 * j] + b[3 * r + 1] * z[3 * j + 1] + b[3 * r + 2] * z[3 * j + 2];
        }
        const double *d = dinv + 9 * (size_t)i;
        for (int r = 0; r < 3; ++r)
            z[3 * i + r] = d[3 * r] * acc[0] + d[3 * r + 1] * acc[1] + d[3 * r + 2] * acc[2];
    }
    free(y);
}

/* The same substitutions with factors and the input vector rounded to FP32
 * (round to nearest even) and every operation of the sweeps in FP32; the
 * result is widened back to FP64.  lu32/dinv32 hold the rounded factors. */
void orc_apply_f32(int n, const int *rowptr, const int *colidx, const float *lu32, const float *dinv32,
                   const double *v, double *z)
{
    float *y = malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
    float *zz = malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        float acc[3] = {(float)v[3 * i], (float)v[3 * i + 1], (float)v[3 * i + 2]};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j >= i) break;
            const float *b = lu32 + 9 * (size_t)p;
            for (int r = 0; r < 3; ++r)
                acc[r] -= b[3 * r] * y[3 * j] + b[3 * r + 1] * y[3 * j + 1] + b[3 * r + 2] * y[3 * j + 2];
        }
        y[3 * i] = acc[0]; y[3 * i + 1] = acc[1]; y[3 * i + 2] = acc[2];
    }
    for (int i = n - 1; i >= 0; --i) {
        float acc[3] = {y[3 * i], y[3 * i + 1], y[3 * i + 2]};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j <= i) continue;
            const float *b = lu32 + 9 * (size_t)p;
            for (int r = 0; r < 3; ++r)
                acc[r] -= b[3 * r] * zz[3 * j] + b[3 * r + 1] * zz[3 * j + 1] + b[3 * r + 2] * zz[3 * j + 2];
        }
        const float *d = dinv32 + 9 * (size_t)i;
        for (int r = 0; r < 3; ++r)
            zz[3 * i + r] = d[3 * r] * acc[0] + d[3 * r + 1] * acc[1] + d[3 * r + 2] * acc[2];
    }
    for (int i = 0; i < 3 * n; ++i) z[i] = (double)zz[i];
    free(y);
    free(zz);
}

/* --------------------------------------------------------- SpMV, vectors */

/* y = A x, blocks row-major, ascending column order within a row. */
void orc_spmv(int n, const int *rowptr, const int *colidx, const double *vals, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double *b = vals + 9 * (size_t)p;
            const double *xj = x + 3 * (size_t)colidx[p];
            for (int r = 0; r < 3; ++r) acc[r] += b[3 * r] * xj[0] + b[3 * r + 1] * xj[1] + b[3 * r + 2] * xj[2];
        }
        y[3 * i] = acc[0]; y[3 * i + 1] = acc[1]; y[3 * i + 2] = acc[2];
    }
}

/* ----------------------------------------------------------- Block-Jacobi */

/* The Jacobi matrix of Section "Block-Jacobi-ILU0": the blocks (i, j) of A
 * with part[i] == part[j] (diagonal blocks always qualify), in A's order.
 * rrow (n + 1), rcol and rvals (room for rowptr[n] blocks).  Returns the
 * number of blocks kept. */
int orc_jacobi_matrix(int n, const int *rowptr, const int *colidx, const double *vals, const int *part,
                      int *rrow, int *rcol, double *rvals)
{
    int k = 0;
    rrow[0] = 0;
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (part[colidx[p]] != part[i]) continue;
            rcol[k] = colidx[p];
            memcpy(rvals + 9 * (size_t)k, vals + 9 * (size_t)p, 9 * sizeof(double));
            ++k;
        }
        rrow[i + 1] = k;
    }
    return k;
}

static double dot(int m, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------ wells */

typedef struct {
    int n_wells;
    const int *well_ptr;    /* perforations of well w: [well_ptr[w], well_ptr[w+1]) */
    const int *perf_row;    /* block row of each perforation */
    const double *B, *C;    /* 4x3 blocks, row-major, one per perforation */
    const double *Dinv;     /* 4x4 blocks, row-major, one per well */
} wells_t;

/* Algorithm 5 for every well: t1 = B x, t2 = D^-1 t1, y -= C^T t2. */
void orc_wells_apply(int n_wells, const int *well_ptr, const int *perf_row, const double *B, const double *C,
                     const double *Dinv, const double *x, double *y)
{
    for (int w = 0; w < n_wells; ++w) {
        double t1[4] = {0.0, 0.0, 0.0, 0.0}, t2[4];
        for (int p = well_ptr[w]; p < well_ptr[w + 1]; ++p) {
            const double *b = B + 12 * (size_t)p, *xc = x + 3 * (size_t)perf_row[p];
            for (int i = 0; i < 4; ++i) t1[i] += b[3 * i] * xc[0] + b[3 * i + 1] * xc[1] + b[3 * i + 2] * xc[2];
        }
        const double *d = Dinv + 16 * (size_t)w;
        for (int i = 0; i < 4; ++i) t2[i] = d[4 * i] * t1[0] + d[4 * i + 1] * t1[1] + d[4 * i + 2] * t1[2] + d[4 * i + 3] * t1[3];
        for (int p = well_ptr[w]; p < well_ptr[w + 1]; ++p) {
            const double *c = C + 12 * (size_t)p;
            double *yc = y + 3 * (size_t)perf_row[p];
            for (int j = 0; j < 3; ++j) yc[j] -= c[j] * t2[0] + c[3 + j] * t2[1] + c[6 + j] * t2[2] + c[9 + j] * t2[3];
        }
    }
}

static void op_apply(int n, const int *rowptr, const int *colidx, const double *vals, const wells_t *w,
                     const double *x, double *y)
{
    orc_spmv(n, rowptr, colidx, vals, x, y);
    if (w && w->n_wells > 0) orc_wells_apply(w->n_wells, w->well_ptr, w->perf_row, w->B, w->C, w->Dinv, x, y);
}

/* --------------------------------------------------------------- BiCGStab */

typedef struct {
    int kind;                  /* ORC_PREC_* */
    int n;
    const int *rowptr, *colidx;
    const double *lu, *dinv;   /* FP64 factors */
    const float *lu32, *dinv32;
} precond;

static void prec_apply(const precond *m, const double *v, double *z)
{
    if (m->kind == ORC_PREC_ILU_F64) orc_apply(m->n, m->rowptr, m->colidx, m->lu, m->dinv, v, z);
    else if (m->kind == ORC_PREC_ILU_F32) orc_apply_f32(m->n, m->rowptr, m->colidx, m->lu32, m->dinv32, v, z);
    else memcpy(z, v, sizeof(double) * 3 * (size_t)m->n);
}

/* Preconditioned BiCGStab on one system (already in the order the factors
 * were computed in).  x0 = 0, r0 = b, rhat = r0, rho_old = alpha = omega = 1,
 * v = p = 0.  Each iteration i:
 *   rho = (rhat, r); beta = (rho / rho_old)(alpha / omega);
 *   p = r + beta (p - omega v); phat = M^{-1} p; v = A phat;
 *   alpha = rho / (rhat, v); s = r - alpha v;
 *   ||s|| <= tol: x += alpha phat, stop after 2i-1 half steps;
 *   shat = M^{-1} s; t = A shat; omega = (t, s) / (t, t);
 *   x += alpha phat + omega shat; r = s - omega t;
 *   ||r|| <= tol: stop after 2i half steps;  rho_old = rho.
 * tol = reduction * ||r0||.  Breakdown when rho, (rhat, v), (t, t) or omega
 * is zero; non-finite scalars give ORC_NON_FINITE.  On an omega breakdown
 * x keeps the half-step update.  max_iter full iterations without meeting
 * the test give ORC_NOT_CONVERGED with the last iterate in x.
 * trace (optional, 8 doubles per iteration): rho, (rhat,v), alpha, ||s||,
 * (t,s), (t,t), omega, ||r||. */
static int bicgstab(int n, const int *rowptr, const int *colidx, const double *vals, const wells_t *wl,
                    const precond *m, const double *b, double reduction, int max_iter, double *x, orc_info *info,
                    double *trace)
{
    size_t m3 = 3 * (size_t)n;
    size_t bytes = sizeof(double) * (m3 > 0 ? m3 : 1);
    double *r = malloc(bytes), *rhat = malloc(bytes), *p = malloc(bytes), *v = malloc(bytes);
    double *phat = malloc(bytes), *s = malloc(bytes), *shat = malloc(bytes), *t = malloc(bytes);
    int status = ORC_NOT_CONVERGED, half = 0;
    for (size_t i = 0; i < m3; ++i) { x[i] = 0.0; r[i] = b[i]; rhat[i] = b[i]; p[i] = 0.0; v[i] = 0.0; }
    double r0 = sqrt(dot((int)m3, r, r));
    double tol = reduction * r0;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    double rho = dot((int)m3, rhat, r);
    double last = r0;
    info->r0_norm = r0;
    if (!isfinite(r0)) { status = ORC_NON_FINITE; goto done; }
    if (r0 == 0.0) { status = ORC_OK; goto done; }
    for (int it = 1; it <= max_iter; ++it) {
        double *tr = trace ? trace + 8 * (size_t)(it - 1) : NULL;
        if (rho == 0.0) { status = ORC_BREAKDOWN; goto done; }
        double beta = (rho / rho_old) * (alpha / omega);
        for (size_t i = 0; i < m3; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        prec_apply(m, p, phat);
        op_apply(n, rowptr, colidx, vals, wl, phat, v);
        double rv = dot((int)m3, rhat, v);
        if (tr) { tr[0] = rho; tr[1] = rv; }
        if (!isfinite(rv)) { status = ORC_NON_FINITE; goto done; }
        if (rv == 0.0) { status = ORC_BREAKDOWN; goto done; }
        alpha = rho / rv;
        for (size_t i = 0; i < m3; ++i) s[i] = r[i] - alpha * v[i];
        double snorm = sqrt(dot((int)m3, s, s));
        if (tr) { tr[2] = alpha; tr[3] = snorm; }
        if (!isfinite(snorm)) { status = ORC_NON_FINITE; goto done; }
        half = 2 * it - 1;
        last = snorm;
        if (snorm <= tol) {
            for (size_t i = 0; i < m3; ++i) x[i] += alpha * phat[i];
            status = ORC_OK;
            goto done;
        }
        prec_apply(m, s, shat);
        op_apply(n, rowptr, colidx, vals, wl, shat, t);
        double ts = dot((int)m3, t, s), tt = dot((int)m3, t, t);
        if (tr) { tr[4] = ts; tr[5] = tt; }
        if (!isfinite(ts) || !isfinite(tt)) { status = ORC_NON_FINITE; goto done; }
        if (tt == 0.0) { status = ORC_BREAKDOWN; goto done; }
        omega = ts / tt;
        if (tr) tr[6] = omega;
        if (omega == 0.0) {
            for (size_t i = 0; i < m3; ++i) x[i] += alpha * phat[i];
            status = ORC_BREAKDOWN;
            goto done;
        }
        for (size_t i = 0; i < m3; ++i) {
            x[i] += alpha * phat[i] + omega * shat[i];
            r[i] = s[i] - omega * t[i];
        }
        double rnorm = sqrt(dot((int)m3, r, r));
        if (tr) tr[7] = rnorm;
        if (!isfinite(rnorm)) { status = ORC_NON_FINITE; goto done; }
        half = 2 * it;
        last = rnorm;
        if (rnorm <= tol) { status = ORC_OK; goto done; }
        rho_old = rho;
        rho = dot((int)m3, rhat, r);
    }
    status = ORC_NOT_CONVERGED;
done:
    info->status = status;
    info->half_steps = half;
    info->final_norm = last;
    free(r); free(rhat); free(p); free(v); free(phat); free(s); free(shat); free(t);
    return status;
}

/* BiCGStab on an already ordered system with given factors (lu, dinv: FP64
 * factors from orc_ilu0 on the same pattern).  precond_kind picks the FP64
 * factors, their FP32 roundings, or no preconditioner. */
int orc_bicgstab(int n, const int *rowptr, const int *colidx, const double *vals, const double *lu,
                 const double *dinv, int precond_kind, const double *b, double reduction, int max_iter,
                 double *x, orc_info *info, double *trace)
{
    return orc_bicgstab_split(n, rowptr, colidx, vals, rowptr, colidx, lu, dinv, precond_kind, b, reduction,
                              max_iter, x, info, trace);
}

/* As orc_bicgstab, with factors on their own pattern (mrow, mcol): the
 * preconditioner of a Jacobi matrix while the SpMV uses the full matrix. */
static int bicgstab_wells(int n, const int *rowptr, const int *colidx, const double *vals, const wells_t *wells,
                          const int *mrow, const int *mcol, const double *lu, const double *dinv, int precond_kind,
                          const double *b, double reduction, int max_iter, double *x, orc_info *info, double *trace);

int orc_bicgstab_split(int n, const int *rowptr, const int *colidx, const double *vals, const int *mrow,
                       const int *mcol, const double *lu, const double *dinv, int precond_kind, const double *b,
                       double reduction, int max_iter, double *x, orc_info *info, double *trace)
{
    return bicgstab_wells(n, rowptr, colidx, vals, NULL, mrow, mcol, lu, dinv, precond_kind, b, reduction, max_iter,
                          x, info, trace);
}

/* The operator A (+ separate wells when given) with factors on (mrow, mcol). */
static int bicgstab_wells(int n, const int *rowptr, const int *colidx, const double *vals, const wells_t *wells,
                          const int *mrow, const int *mcol, const double *lu, const double *dinv, int precond_kind,
                          const double *b, double reduction, int max_iter, double *x, orc_info *info, double *trace)
{
    precond m = {precond_kind, n, mrow, mcol, lu, dinv, NULL, NULL};
    float *lu32 = NULL, *dinv32 = NULL;
    if (precond_kind == ORC_PREC_ILU_F32) {
        size_t nnz = (size_t)mrow[n];
        lu32 = malloc(sizeof(float) * 9 * (nnz > 0 ? nnz : 1));
        dinv32 = malloc(sizeof(float) * 9 * (size_t)(n > 0 ? n : 1));
        for (size_t e = 0; e < 9 * nnz; ++e) lu32[e] = (float)lu[e];
        for (size_t e = 0; e < 9 * (size_t)n; ++e) dinv32[e] = (float)dinv[e];
        m.lu32 = lu32;
        m.dinv32 = dinv32;
    }
    int st = bicgstab(n, rowptr, colidx, vals, wells, &m, b, reduction, max_iter, x, info, trace);
    free(lu32);
    free(dinv32);
    return st;
}

/* The whole path on one system in its original order:
 * validate -> ordering (natural, LS or GC) -> reordered copy of A and b ->
 * ILU0 -> BiCGStab -> x back to the original order -> true residual
 * ||b - A x|| / ||b|| with the original A.  perm_out (n ints, may be NULL)
 * receives perm[new] = old; *n_sets the number of levels or colours
 * (n for the natural order). */
int orc_solve(int n, const int *rowptr, const int *colidx, const double *vals, const double *b,
              int ordering, int precond_kind, double reduction, int max_iter, double *x,
              orc_info *info, int *perm_out, int *n_sets, int *bad_row)
{
    return orc_solve_jacobi(n, rowptr, colidx, vals, NULL, b, ordering, precond_kind, reduction, max_iter, x,
                            info, perm_out, n_sets, bad_row);
}

/* As orc_solve, with the Block-Jacobi-ILU0 preconditioner when part (n
 * partition ids) is given: ordering and ILU0 on the Jacobi matrix, SpMV and
 * true residual with the full matrix.  part == NULL is plain ILU0. */
int orc_solve_jacobi(int n, const int *rowptr, const int *colidx, const double *vals, const int *part,
                     const double *b, int ordering, int precond_kind, double reduction, int max_iter, double *x,
                     orc_info *info, int *perm_out, int *n_sets, int *bad_row)
{
    return orc_solve_wells(n, rowptr, colidx, vals, part, 0, NULL, NULL, NULL, NULL, NULL, b, ordering, precond_kind,
                           reduction, max_iter, x, info, perm_out, n_sets, bad_row);
}

/* As orc_solve_jacobi with n_wells standard wells kept separate (Algorithm
 * 5) in the operator of the SpMVs and of the true residual; perf_row in
 * A's original numbering.  The preconditioner ignores the wells. */
int orc_solve_wells(int n, const int *rowptr, const int *colidx, const double *vals, const int *part, int n_wells,
                    const int *well_ptr, const int *perf_row, const double *B, const double *C, const double *Dinv,
                    const double *b, int ordering, int precond_kind, double reduction, int max_iter, double *x,
                    orc_info *info, int *perm_out, int *n_sets, int *bad_row)
{
    int st = orc_validate(n, rowptr, colidx, bad_row);
    memset(info, 0, sizeof *info);
    info->status = st;
    if (st != ORC_OK) return st;
    size_t nnz = (size_t)rowptr[n];
    size_t nn = (size_t)(n > 0 ? n : 1);
    int *key = malloc(sizeof(int) * nn), *perm = malloc(sizeof(int) * nn);
    int *prow = malloc(sizeof(int) * (nn + 1)), *pcol = malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    double *pvals = malloc(sizeof(double) * 9 * (nnz > 0 ? nnz : 1));
    double *lu = malloc(sizeof(double) * 9 * (nnz > 0 ? nnz : 1));
    double *dinv = malloc(sizeof(double) * 9 * nn);
    double *pb = malloc(sizeof(double) * 3 * nn), *px = malloc(sizeof(double) * 3 * nn);
    double *ax = malloc(sizeof(double) * 3 * nn);
    /* the preconditioner's matrix: A itself, or its Jacobi matrix */
    int *jrow = malloc(sizeof(int) * (nn + 1)), *jcol = malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    double *jvals = malloc(sizeof(double) * 9 * (nnz > 0 ? nnz : 1));
    int *mrow = malloc(sizeof(int) * (nn + 1)), *mcol = malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    if (part) {
        orc_jacobi_matrix(n, rowptr, colidx, vals, part, jrow, jcol, jvals);
    } else {
        memcpy(jrow, rowptr, sizeof(int) * (nn + 1));
        memcpy(jcol, colidx, sizeof(int) * nnz);
        memcpy(jvals, vals, sizeof(double) * 9 * nnz);
    }
    int sets = n;
    if (ordering == ORC_ORDER_LEVEL) sets = orc_level_sets(n, jrow, jcol, key, perm);
    else if (ordering == ORC_ORDER_COLOUR) sets = orc_dsatur_colour(n, jrow, jcol, key, perm);
    else if (ordering == ORC_ORDER_RCM_LEVEL) sets = orc_rcm_levels(n, jrow, jcol, key, perm);
    else for (int i = 0; i < n; ++i) perm[i] = i;
    if (n_sets) *n_sets = sets;
    if (perm_out) memcpy(perm_out, perm, sizeof(int) * (size_t)n);
    orc_permute(n, rowptr, colidx, vals, perm, prow, pcol, pvals);
    orc_permute(n, jrow, jcol, jvals, perm, mrow, mcol, lu);
    if (precond_kind != ORC_PREC_NONE) {
        int brow;
        st = orc_ilu0(n, mrow, mcol, lu, dinv, &brow);
        if (st != ORC_OK) {
            *bad_row = brow >= 0 ? perm[brow] : -1;
            info->status = st;
            goto out;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) pb[3 * i + c] = b[3 * (size_t)perm[i] + c];
    {
        /* the wells in the new numbering */
        int nperf = n_wells > 0 ? well_ptr[n_wells] : 0;
        int *iperm = malloc(sizeof(int) * nn), *prow_w = malloc(sizeof(int) * (size_t)(nperf > 0 ? nperf : 1));
        for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
        for (int p = 0; p < nperf; ++p) prow_w[p] = iperm[perf_row[p]];
        wells_t wl = {n_wells, well_ptr, prow_w, B, C, Dinv};
        st = bicgstab_wells(n, prow, pcol, pvals, n_wells > 0 ? &wl : NULL, mrow, mcol, lu, dinv, precond_kind, pb,
                            reduction, max_iter, px, info, NULL);
        free(iperm);
        free(prow_w);
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) x[3 * (size_t)perm[i] + c] = px[3 * i + c];
    {
        wells_t wl = {n_wells, well_ptr, perf_row, B, C, Dinv};
        op_apply(n, rowptr, colidx, vals, n_wells > 0 ? &wl : NULL, x, ax);
    }
    {
        double rr = 0.0, bb = 0.0;
        for (size_t i = 0; i < 3 * (size_t)n; ++i) {
            double d = b[i] - ax[i];
            rr += d * d;
            bb += b[i] * b[i];
        }
        info->true_rel_residual = bb > 0.0 ? sqrt(rr) / sqrt(bb) : 0.0;
    }
out:
    free(key); free(perm); free(prow); free(pcol); free(pvals); free(lu); free(dinv);
    free(pb); free(px); free(ax); free(jrow); free(jcol); free(jvals); free(mrow); free(mcol);
    return st;
}

/* ------------------------------------------------------------------ GMRES */

/* Right-preconditioned GMRES(m) on an already ordered system, x0 = 0.  Each
 * cycle: v_1 = r / ||r||; for j = 1..m: z = M^-1 v_j, w = A z; Gram-Schmidt
 * of w against v_1..v_j twice (classical: all coefficients from the same w,
 * then w -= V h; the second pass repeats it and adds its coefficients);
 * h_{j+1,j} = ||w||; earlier Givens rotations applied to column j, a new one
 * zeroes h_{j+1,j}; |g_{j+1}| is the residual norm of the current iterate.
 * A cycle ends when it is <= reduction * ||b||, after max_iter steps in
 * total (none when max_iter <= 0), on h_{j+1,j} = 0, or after m steps; then
 * y = H^-1 g (back substitution) and x += M^-1 (V y).  The first two end
 * the solve; otherwise the next cycle starts from the explicit residual
 * r = b - A x (and the solve ends if its norm meets the test).  info->half_steps counts the Arnoldi steps (one
 * preconditioner application and one product with A each).  trace
 * (optional): |g_{j+1}| after every step. */
static int gmres_core(int n, const int *rowptr, const int *colidx, const double *vals, const wells_t *wl,
                      const double *lu, const double *dinv, int precond_kind, const double *b, int m, double reduction,
                      int max_iter, double *x, orc_info *info, double *trace)
{
    size_t n3 = 3 * (size_t)n, nb = n3 > 0 ? n3 : 1;
    if (m < 1) m = 1;
    precond pc = {precond_kind, n, rowptr, colidx, lu, dinv, NULL, NULL};
    float *lu32 = NULL, *dinv32 = NULL;
    if (precond_kind == ORC_PREC_ILU_F32) {
        size_t nnz = (size_t)rowptr[n];
        lu32 = malloc(sizeof(float) * 9 * (nnz > 0 ? nnz : 1));
        dinv32 = malloc(sizeof(float) * 9 * (size_t)(n > 0 ? n : 1));
        for (size_t e = 0; e < 9 * nnz; ++e) lu32[e] = (float)lu[e];
        for (size_t e = 0; e < 9 * (size_t)n; ++e) dinv32[e] = (float)dinv[e];
        pc.lu32 = lu32;
        pc.dinv32 = dinv32;
    }
    double *V = malloc(sizeof(double) * nb * (size_t)(m + 1)), *z = malloc(sizeof(double) * nb);
    double *w = malloc(sizeof(double) * nb), *r = malloc(sizeof(double) * nb);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double)), *cs = malloc(sizeof(double) * m);
    double *sn = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * (m + 1));
    double *h = malloc(sizeof(double) * (m + 1)), *y = malloc(sizeof(double) * m);
    int status = ORC_NOT_CONVERGED, steps = 0;
    for (size_t e = 0; e < n3; ++e) { x[e] = 0.0; r[e] = b[e]; }
    double beta = sqrt(dot((int)n3, r, r));
    const double tol = reduction * beta;
    double last = beta;
    info->r0_norm = beta;
    if (!isfinite(beta)) { status = ORC_NON_FINITE; goto done; }
    if (beta == 0.0) { status = ORC_OK; goto done; }
    if (max_iter <= 0) goto done;
    for (;;) {
        for (size_t e = 0; e < n3; ++e) V[e] = r[e] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int jend = 0, stop = 0;
        double hn = 0.0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * nb;
            prec_apply(&pc, vj, z);
            op_apply(n, rowptr, colidx, vals, wl, z, w);
            for (int i = 0; i <= j; ++i) H[i + (size_t)j * (m + 1)] = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) h[i] = dot((int)n3, w, V + (size_t)i * nb);
                for (size_t e = 0; e < n3; ++e) {
                    double acc = w[e];
                    for (int i = 0; i <= j; ++i) acc -= h[i] * V[(size_t)i * nb + e];
                    w[e] = acc;
                }
                for (int i = 0; i <= j; ++i) H[i + (size_t)j * (m + 1)] += h[i];
            }
            hn = sqrt(dot((int)n3, w, w));
            double *col = H + (size_t)j * (m + 1);
            col[j + 1] = hn;
            for (int k = 0; k < j; ++k) {
                const double t = cs[k] * col[k] + sn[k] * col[k + 1];
                col[k + 1] = -sn[k] * col[k] + cs[k] * col[k + 1];
                col[k] = t;
            }
            const double d = sqrt(col[j] * col[j] + col[j + 1] * col[j + 1]);
            cs[j] = d > 0.0 ? col[j] / d : 1.0;
            sn[j] = d > 0.0 ? col[j + 1] / d : 0.0;
            col[j] = d;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++steps;
            jend = j + 1;
            last = fabs(g[j + 1]);
            if (trace) trace[steps - 1] = last;
            if (!isfinite(last) || !isfinite(hn)) { status = ORC_NON_FINITE; goto done; }
            if (last <= tol) { status = ORC_OK; stop = 1; break; }
            if (steps >= max_iter) { stop = 1; break; }
            if (hn == 0.0) break;
            for (size_t e = 0; e < n3; ++e) V[(size_t)(j + 1) * nb + e] = w[e] / hn;
        }
        for (int i = jend - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < jend; ++k) acc -= H[i + (size_t)k * (m + 1)] * y[k];
            y[i] = acc / H[i + (size_t)i * (m + 1)];
        }
        for (size_t e = 0; e < n3; ++e) {
            double acc = 0.0;
            for (int i = 0; i < jend; ++i) acc += y[i] * V[(size_t)i * nb + e];
            w[e] = acc;
        }
        prec_apply(&pc, w, z);
        for (size_t e = 0; e < n3; ++e) x[e] += z[e];
        if (stop) break;
        op_apply(n, rowptr, colidx, vals, wl, x, w);
        for (size_t e = 0; e < n3; ++e) r[e] = b[e] - w[e];
        beta = sqrt(dot((int)n3, r, r));
        last = beta;
        if (!isfinite(beta)) { status = ORC_NON_FINITE; break; }
        if (beta <= tol) { status = ORC_OK; break; }
    }
done:
    info->status = status;
    info->half_steps = steps;
    info->final_norm = last;
    free(lu32); free(dinv32); free(V); free(z); free(w); free(r); free(H); free(cs); free(sn); free(g); free(h);
    free(y);
    return status;
}

int orc_gmres(int n, const int *rowptr, const int *colidx, const double *vals, const double *lu, const double *dinv,
              int precond_kind, const double *b, int m, double reduction, int max_iter, double *x, orc_info *info,
              double *trace)
{
    return gmres_core(n, rowptr, colidx, vals, NULL, lu, dinv, precond_kind, b, m, reduction, max_iter, x, info,
                      trace);
}

/* The same with standard wells kept separate (Algorithm 5) in every product
 * with A: the operator is A x - sum_w C_w^T D_w^-1 B_w x; the
 * preconditioner stays ILU0 of A.  Wells in this system's numbering. */
int orc_gmres_wells(int n, const int *rowptr, const int *colidx, const double *vals, int n_wells, const int *well_ptr,
                    const int *perf_row, const double *B, const double *C, const double *Dinv, const double *lu,
                    const double *dinv, int precond_kind, const double *b, int m, double reduction, int max_iter,
                    double *x, orc_info *info, double *trace)
{
    wells_t wl = {n_wells, well_ptr, perf_row, B, C, Dinv};
    return gmres_core(n, rowptr, colidx, vals, n_wells > 0 ? &wl : NULL, lu, dinv, precond_kind, b, m, reduction,
                      max_iter, x, info, trace);
}

/* BiCGStab on an already ordered system with n_wells standard wells kept
 * separate in the operator (Algorithm 5), factors on the matrix's own
 * pattern; trace as orc_bicgstab. */
int orc_bicgstab_wells(int n, const int *rowptr, const int *colidx, const double *vals, int n_wells,
                       const int *well_ptr, const int *perf_row, const double *B, const double *C, const double *Dinv,
                       const double *lu, const double *dinv, int precond_kind, const double *b, double reduction,
                       int max_iter, double *x, orc_info *info, double *trace)
{
    wells_t wl = {n_wells, well_ptr, perf_row, B, C, Dinv};
    return bicgstab_wells(n, rowptr, colidx, vals, n_wells > 0 ? &wl : NULL, rowptr, colidx, lu, dinv, precond_kind,
                          b, reduction, max_iter, x, info, trace);
}
