// Host-side pattern analysis: validation, orderings, sweep schedules and the
// factor update lists.  Integer work only, done once per pattern.
#pragma once

#include <cstdint>
#include <vector>

namespace rs {

// Pattern check: row pointers start at 0 and never decrease, columns in
// range, strictly ascending per row, diagonal present.  Returns 0,
// RS_BAD_PATTERN or RS_MISSING_DIAGONAL; *bad_row names the row.
int validate_pattern(int n, int nnzb, const int32_t *rowptr, const int32_t *colidx, int *bad_row);

// perm[new] = old for the four orderings, and set_ptr = the first new
// position of each level/colour.  Returns the number of levels (level sets,
// reverse Cuthill-McKee then level sets), colours (graph colouring) or n
// (natural order: one row per set).
int make_ordering(int n, const int32_t *rowptr, const int32_t *colidx, int ordering, std::vector<int32_t> &perm,
                  std::vector<int32_t> &set_ptr);
int make_ordering(int n, const int32_t *rowptr, const int32_t *colidx, int ordering, std::vector<int32_t> &perm);

// Everything the device needs to factor, sweep and multiply in the new order.
//
// A' = P A P^T is kept in CSR (prow, pcol) with psrc[p] = the caller's block
// position of A'[p].  The lower sweep visits rows in "L-schedule" order
// (levels ascending, new index ascending inside a level); the upper sweep in
// "U-schedule" order (upper levels ascending).  L blocks are stored in
// L-schedule order, U blocks and inv(U_ii) in U-schedule order, so each level
// is one contiguous range of rows and blocks.
//
// With a partition (Block-Jacobi-ILU0) the orderings, sweep schedules and
// update lists are those of the Jacobi matrix (blocks whose two rows share a
// partition); A' stays the full matrix, and lsrc / usrc / dsrc still point
// into it.
struct Schedule {
    int n = 0, nnzb = 0, ordering = 0;
    bool jacobi = false;
    int nnz_m = 0;                  // blocks of the preconditioner's matrix
    int n_sets = 0;                 // levels / colours reported to the caller
    std::vector<int32_t> set_ptr;   // n_sets + 1
    std::vector<int32_t> perm, iperm;
    // reordered matrix
    std::vector<int32_t> prow, pcol, psrc;
    // caller-order block positions of the factor's inputs (psrc composed
    // with lsrc / usrc / dsrc), and the A' blocks the factor does not read
    // (Block-Jacobi: blocks outside the Jacobi matrix) with their sources
    std::vector<int32_t> lsrc_a, usrc_a, dsrc_a, rest_dst, rest_src;
    // lower sweep
    int nl_levels = 0, nL = 0;
    std::vector<int32_t> lrows, lset, lptr, lcol, lsrc, ldq, l2u;
    std::vector<char> lconsec;   // per lower level: its rows are consecutive in the new order
    std::vector<char> lnarrow;   // per lower level: no row holds more than 6 lower or 6 upper blocks
    // upper sweep
    int nu_levels = 0, nU = 0;
    std::vector<int32_t> urows, uset, uptr, ucol, usrc, dsrc;
    // factor: for each L block e, updates upd[upd_ptr[e] .. upd_ptr[e+1])
    // as pairs (target code, source of U_kj); target code = 4 * position +
    // kind, kind 0 = L block, 1 = diagonal of the row, 2 = U block; source =
    // U block position, or ~(A' position) when row k has no lower blocks
    // (then U_kj equals A'_kj, which the reordered copy holds).
    std::vector<int32_t> upd_ptr, upd;
    int max_lrow = 0, max_urow = 0;
    // Rows without lower blocks, when they are exactly the first fuse_n0
    // rows of the new order (at least a quarter of all rows), all hold
    // upper blocks and all sit at the start of one upper level (U-schedule positions fuse_q0 + i for row i): their
    // U rows are their rows of A' (nothing updates them), so the upper launch
    // of that level can also form their rows of the next product with A'.
    // fuse_n0 = 0 when the pattern has no such structure (or with a
    // partition).  fuse_nnz = A' blocks of those rows.
    int fuse_n0 = 0, fuse_q0 = 0, fuse_level = -1;
    long long fuse_nnz = 0;
    // y_in = 1: besides the fuse_n0 rows there are exactly two lower levels
    // (every other row's lower neighbours are among those rows) and none of
    // the other rows holds an upper block.  The y of a row without lower
    // blocks is the sweep's input itself, and every other row finishes in
    // the lower launch (z_i = inv(U_ii) y_i), so an application needs no
    // stored y: the launches read the input instead (bipartite patterns
    // under graph colouring, e.g. the 7-point grids).  Then row i >=
    // fuse_n0 sits at L-schedule position i and U-schedule position
    // i - fuse_n0.
    int y_in = 0;
    // row tiles of the single-launch sweeps: tile t covers schedule
    // positions [start[t], start[t+1]) inside one level, and must wait for
    // the tiles dep[dep_ptr[t] .. dep_ptr[t+1]) (earlier tiles holding rows
    // that its rows read)
    struct Tiles {
        int n = 0;
        std::vector<int32_t> start, dep_ptr, dep;
    } ltiles, utiles;
};

// tile_rows: rows per sweep tile (a multiple of the rows one workgroup covers).
// part: optional partition id per row (Block-Jacobi-ILU0), else plain ILU0.
int build_schedule(int n, int nnzb, const int32_t *rowptr, const int32_t *colidx, int ordering, Schedule &s,
                   int tile_rows, const int32_t *part = nullptr);

// Grow n_parts partitions of near-equal size (sizes differ by at most one):
// each starts from the first unassigned row in natural order and repeatedly
// takes the unassigned row most strongly coupled to it (sum of `weights` of
// the stored blocks joining them; all weights 1 when NULL), jumping to the
// next unassigned row when it has no unassigned neighbour left.
void partition_rows(int n, const int32_t *rowptr, const int32_t *colidx, const double *weights, int n_parts,
                    int32_t *part);

}  // namespace rs
