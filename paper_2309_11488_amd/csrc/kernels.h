// Device data structures and kernel launchers of the BCSR BiCGStab-ILU0 path.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace rs {

// Per-system BiCGStab scalars, kept on the device for the whole solve.
// phase: RUN while iterating, HALF after a half-step stop (x still needs
// x += alpha phat), DONE when finished.
enum Phase : int32_t { PH_RUN = 0, PH_HALF = 1, PH_DONE = 2 };

struct SysState {
    double rho, rho_old, alpha, omega, beta;
    double r0norm, tol, last_norm;
    double true_res;
    int32_t phase, status, half_steps, iter;
    int32_t max_iter, pad0;
};

// Device copies of the schedule (see analysis.h for the meaning).
struct DevSchedule {
    int n, nnzb, nL, nU;
    const int32_t *perm, *prow, *pcol, *psrc;
    const int32_t *lrows, *lptr, *lcol, *lsrc, *ldq, *l2u, *upd_ptr, *upd;
    const int32_t *urows, *uptr, *ucol, *usrc, *dsrc;
    const int32_t *lsrc_a, *usrc_a, *dsrc_a;   // caller-order sources of the factor's blocks
    int nrest;                                 // A' blocks the factor does not read (Block-Jacobi)
    const int32_t *rest_dst, *rest_src;
    // rows 0 .. fuse_n0 hold no lower blocks and sit at U-schedule
    // positions fuse_q0 + i of one upper level (0: no such rows)
    int fuse_n0, fuse_q0;
    // sweep tiles (see Schedule::Tiles)
    int nlt, nut;
    const int32_t *lt_start, *lt_dptr, *lt_dep, *ut_start, *ut_dptr, *ut_dep;
};

// Standard wells kept separate (y -= C^T D^-1 B x for every well), as the
// SpMV kernels see them.  nw == 0: no wells.
struct WellsDev {
    int nw = 0, np = 0;
    const int32_t *well_ptr = nullptr;   // nw + 1: perforations of well w
    const int32_t *perf_x = nullptr;     // np: row of the SpMV's x (and y) each perforation couples
    const int32_t *row_ptr = nullptr;    // n + 1: perforations of output row i are row_perf[row_ptr[i] ..)
    const int32_t *row_perf = nullptr;   // np, ascending within a row
    const int32_t *perf_well = nullptr;  // np
    const double *B = nullptr, *C = nullptr, *Dinv = nullptr;   // per system: np*12, np*12, nw*16
    double *t2 = nullptr;                // per system: nw*4, D^-1 B x of the current x
    // rows [0, fuse_n0) that a perforation couples (their rows of v and t,
    // formed by the fused upper launch, take their well terms afterwards)
    int nfix = 0;
    const int32_t *fix_row = nullptr;
};

// Restarted GMRES: per-system state of the current cycle (Hessenberg matrix
// after the Givens rotations, the rotations, the rotated right-hand side g,
// the Gram-Schmidt coefficients of the current pass).
constexpr int kGmMax = 32;   // largest restart length
struct GmState {
    double H[kGmMax + 1][kGmMax];
    double cs[kGmMax], sn[kGmMax], g[kGmMax + 1], h[kGmMax + 1];
    double beta, hn;
    int32_t jend;   // Arnoldi columns of the current cycle
    int32_t pad;
};

// Work counter of one single-launch sweep kernel: tickets hand out (tile,
// system) items in dependency order; the last workgroup to leave resets the
// tickets and publishes the epoch that marks a tile as done in this sweep.
// error != 0 records a dependency wait that exceeded its spin limit.
struct SweepCtr {
    uint32_t ticket, exit, epoch, error;
};

// Workspace vectors of one solve in the new order: system k's vector starts
// at k * vstride; vstride is 3n rounded up to whole vector tiles and the
// padding holds zeros, so the vector kernels run without bounds checks.
struct Krylov {
    double *r, *rhat, *p, *v, *phat, *s, *shat, *t, *x;
    size_t vstride;
    void *y;            // lower-sweep intermediate, FP64 or FP32 (factor type)
    double *part;       // reduction partials, nsys * part_stride
    size_t part_stride;
    uint32_t *tickets;  // reduction ticket counters, nsys * ticket_stride
    size_t ticket_stride;
    double *spart;      // per-workgroup partials of the two SpMVs, nsys * spart_stride
    size_t spart_stride;
    double *fpart;      // partials of the products formed by the fused upper launch, nsys * fpart_stride
    size_t fpart_stride;
    double *lp;         // lower parts of the second application (k_spmv_lp): 6 values per row, 2 vstride per system, or NULL
    SysState *st;       // nsys states
    int32_t *lflags, *uflags;  // per (system, tile): epoch of the sweep that finished it
    SweepCtr *lctr, *uctr;
};

// Launch geometry shared by host and device code.
constexpr int kWave = 64;
constexpr int kRowsPerWave = 21;                            // 3 lanes per block row, 63 of 64 lanes busy
constexpr int kWavesPerBlock = 4;
constexpr int kRowsPerBlock = kRowsPerWave * kWavesPerBlock;  // 84 block rows per workgroup
constexpr int kRowThreads = kWave * kWavesPerBlock;           // 256
constexpr int kVecThreads = 256;
constexpr int kVecItems = 4;                                // entries per thread per tile
constexpr int kVecTile = kVecThreads * kVecItems;           // 1024 entries
constexpr int kVecMaxBlocks = 2048;

inline int row_blocks(int rows, int waves = kWavesPerBlock) {
    return (rows + waves * kRowsPerWave - 1) / (waves * kRowsPerWave);
}

// Launch shapes of the row kernels (SpMV, per-level sweeps): 4, 2 or 1
// waves per workgroup, blocks staged through LDS or read directly, or staged
// with non-temporal loads.  The arithmetic and its order are the same in
// every shape.
enum RowVariant { RV_W4_LDS = 0, RV_W2_LDS = 1, RV_W1_LDS = 2, RV_W4_DIRECT = 3, RV_W2_DIRECT = 4, RV_W1_DIRECT = 5,
                  RV_W4_LDS_NT = 6, RV_W2_LDS_NT = 7, RV_W1_LDS_NT = 8, RV_COUNT = 9 };
inline int variant_waves(int v) { return v % 3 == 0 ? 4 : (v % 3 == 1 ? 2 : 1); }
// SpMV workgroups: one row tile each.
inline int spmv_grid(int n, int waves) { return std::max(1, row_blocks(n, waves)); }

// Reduction of the dot products fused into an SpMV (RS_OPT_REDUCE_SPLIT):
// 0 = ticket tree in the SpMV, 1 = waves store partials and a one-workgroup
// kernel adds them, 2 = waves store partials and every consumer workgroup
// adds them itself.
constexpr int kTotalThreads = 1024;   // threads of the one-workgroup summing kernel
// Where the consumers of an SpMV's dot products find the sums they add (in
// doubles from the start of the system's partials) and how many pairs:
// the group sums of the ticket tree, or the one total of k_spmv_total
// stored after the wave partials.
struct SpmvSums {
    int offset, count;
};
inline SpmvSums spmv_sums(int n, int waves, int split) {
    const int g = spmv_grid(n, waves);
    if (split == 1) return SpmvSums{2 * g * waves, 1};       // k_spmv_total's sum after the wave partials
    if (split == 2) return SpmvSums{0, g * waves};           // the wave partials themselves
    return SpmvSums{2 * g, (g + 31) / 32};                   // the ticket tree's group sums
}
// Reduction scratch of a system whose largest launch has `blocks` workgroups.
inline size_t part_stride_for(int blocks) { return 2 * (size_t)blocks + 2 * ((size_t)blocks / 32 + 1) + 16; }
// Reduction counters sit on their own 128-byte lines (kTicketPad uint32
// apart): counter 0 is the top of the tree, counter 1 + g that of group g.
constexpr int kTicketPad = 32;
inline size_t ticket_stride_for(int blocks) { return (size_t)kTicketPad * (2 + (size_t)blocks / 32 + 1); }
inline size_t vec_stride(int n) { return (3 * (size_t)n + kVecTile - 1) / kVecTile * kVecTile; }
int vec_blocks(int n);  // workgroups of the vector kernels for one padded vector

// Ap[dst[i]] = A[src[i]] for every system (blocks of 9 doubles).
void launch_gather_pairs(const double *A, size_t a_stride, double *Ap, size_t ap_stride, const int32_t *dst,
                         const int32_t *src, int cnt, int nsys, hipStream_t s);

// One level of the block ILU0 factorisation: L-schedule rows [q0, q1).
// Reads the caller's blocks A, writes the reordered copy Ap of every block
// it reads (the SpMV operand), the FP64 factors and, when Lf is not null,
// their FP32 roundings.  staged: the rows are consecutive in the new order
// and the factor writes every block of their reordered rows (no blocks
// outside the preconditioner's matrix), so workgroups may collect their
// part of Ap in LDS and store it contiguously.
// skip_u0: rows without lower blocks store no U in the factor type (FP64 U,
// or the FP32 U of FP32 factors; their U rows are their rows of A': see
// launch_fill_u).  last: the last level, whose FP64 pivot inverses no
// later level reads (with FP32 factors only the FP32 copy is stored).
// narrow: no row of the level holds more than 6 lower or 6 upper blocks
// (Schedule::lnarrow), which a kernel with fewer registers per lane serves.
void launch_factor_level(const DevSchedule &d, const double *A, size_t a_stride, double *Ap, double *L, double *U,
                         double *Dinv, float *Lf, float *Uf, float *Df, int32_t *bad, int q0, int q1, bool staged,
                         bool skip_u0, bool last, bool narrow, int nsys, hipStream_t s);
// The first level of the factorisation when it is the rows [0, d.fuse_n0)
// of the new order (rows without lower blocks, U-schedule positions fuse_q0
// + i): their blocks of the reordered copy Ap (copied from the caller's A),
// inv(U_ii) = inv(A_ii) into Dinv (and its FP32 rounding into Df when not
// null), a singular or non-finite pivot reported in bad; no U stored.
void launch_factor_first(const DevSchedule &d, const double *A, size_t a_stride, double *Ap, double *Dinv,
                         float *Df, int32_t *bad, int nsys, hipStream_t s);
// U[f] = A'[usrc[f]], rounded to T, for U positions [f0, f1) of every
// system (per-system strides a_stride and u_stride, in elements).
template <typename T>
void launch_fill_u(const DevSchedule &d, const double *Ap, size_t a_stride, T *U, size_t u_stride, int f0, int f1,
                   int nsys, hipStream_t s);

// Lower sweep y = L^{-1} in for L-schedule rows [q0, q1).  When fuse_p is
// set, the input is p = r + beta (p - omega v) computed on the fly (and
// stored); otherwise `in`.  st may be NULL (no phase check).
// When u0_end > 0, rows whose U-schedule position is below u0_end (the
// upper sweep's first level: no upper blocks) also finish the upper sweep:
// z_i = inv(U_ii) y_i (Dinv at d_stride per system), exactly as k_usweep.
// yd (may be NULL): the rows' lower neighbours hold no lower blocks, so
// their y is the application's input itself, read from yd (FP64, at
// vstride per system) instead of y; the launch stores no y, so every row it
// covers must finish here (U-schedule position below u0_end).
template <typename T>
void launch_lsweep(const DevSchedule &d, const T *L, size_t l_stride, const double *in, T *y, size_t vstride,
                   bool fuse_p, const double *r, const double *v, double *p, SysState *st, int q0, int q1, int nsys,
                   int variant, const T *Dinv, size_t d_stride, double *z, int u0_end, const double *yd,
                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// p = r + beta (p - omega v) for the rows [0, d.fuse_n0) of every system
// still iterating (the lower sweep of rows without lower blocks, when the
// sweeps read their y from p: see launch_lsweep's yd).
void launch_p_update(const DevSchedule &d, Krylov &k, int nsys, hipStream_t s);

// Upper sweep z = inv(U_ii) (y - U z) for U-schedule rows [q0, q1).
template <typename T>
// defer: test the system's phase after the walk's loads are issued (the
// first application of an iteration, which runs whenever it is queued).
void launch_usweep(const DevSchedule &d, const T *U, size_t u_stride, const T *Dinv, size_t d_stride, const T *y,
                   double *z, size_t vstride, SysState *st, int q0, int q1, int nsys, int variant, bool defer,
                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ev0 / ev1 (optional, every launcher below that takes them): events the
// dispatch records at the kernel's start and end.

// Single-launch sweeps over all tiles of all nsys systems (L: lower
// schedule, U: upper schedule).  grid = number of workgroups; spin = polls
// before a dependency wait gives up (sets ctr->error and goes on).
constexpr int kSpinLimitDefault = 1 << 22;
template <typename T>
void launch_lsweep_tiles(const DevSchedule &d, const T *L, size_t l_stride, const double *in, T *y, size_t vstride,
                         bool fuse_p, const double *r, const double *v, double *p, SysState *st, int32_t *flags,
                         SweepCtr *ctr, int nsys, int grid, int spin, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
template <typename T>
void launch_usweep_tiles(const DevSchedule &d, const T *U, size_t u_stride, const T *Dinv, size_t d_stride,
                         const T *y, double *z, size_t vstride, SysState *st, int32_t *flags, SweepCtr *ctr, int nsys,
                         int grid, int spin, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Plain y = A x (rows in storage order), FP64.
// y = A x (minus the separate wells, when w has any: t2 is computed first).
void launch_spmv(int n, const int32_t *ptr, const int32_t *col, const double *A, size_t a_stride, const double *x,
                 double *y, size_t vstride, int nsys, int variant, const WellsDev &w, hipStream_t s);

// Solver kernels (new order, all nsys systems of the Krylov workspace).
// The two SpMVs store per-workgroup partial sums; the s- and x/r-updates
// that follow add them (their launch shape fixes the partials' count).
// bad[sys] < n marks a system whose factorisation hit a singular pivot.
void launch_setup(const DevSchedule &d, const double *b_orig, const int32_t *bad, double reduction, int max_iter,
                  Krylov &k, int nsys, hipStream_t s);
// t2 = D^-1 (B x) for every well and system (x at stride xstride): the
// first half of the separate well application, run before an SpMV of x.
void launch_wells_t2(const WellsDev &w, const double *x, size_t xstride, int nsys, hipStream_t s);
// The well terms of the rows w.fix_row, which the fused upper launch formed
// without them (t2 of the whole x already computed): y_i -= (C^T t2)_i, and
// the changes of (w1, y) and (y, y) over those rows stored as one more group
// sum of the fused launch's partials (position `at` of part, per system
// part_stride) that the next vector kernel adds.  Systems not iterating are
// skipped.
void launch_wells_fix(const WellsDev &w, double *y, const double *w1, size_t vstride, double *part,
                      size_t part_stride, int at, SysState *st, int nsys, hipStream_t s);

// ev0 / ev1 (optional): events recorded by the dispatch at the kernel's start and end.
// r0: rows [r0, n) only (the fused upper launch formed rows [0, r0)).
void launch_spmv_v(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant, int split,
                   const WellsDev &w, int r0, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// fused: the product's rows [0, d.fuse_n0) came from the fused upper
// launch, whose group sums are added after those of the SpMV; fix: plus the
// one launch_wells_fix stored after them (at wells_fix_at).
void launch_s_update(const DevSchedule &d, Krylov &k, int nsys, int spmv_variant, int split, bool fused,
                     hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool fix = false);
// Position in k.fpart (per system) of the group sum launch_wells_fix adds.
int wells_fix_at(const DevSchedule &d, int spmv_variant);
void launch_spmv_t(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant, int split,
                   const WellsDev &w, int r0, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_xr_update(const DevSchedule &d, Krylov &k, int nsys, int spmv_variant, int split, bool fused,
                      hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool fix = false);

// Which product the fused upper launch forms.
enum FuseMode { FUSE_NONE = 0, FUSE_V = 1, FUSE_T = 2 };

// Upper launch of the rows [0, d.fuse_n0) (U-schedule positions fuse_q0 +
// i) from their rows of A', fused with the product that follows the
// application: z_i as launch_usweep, and out_i = (A' z)_i with the
// dot-product partials of the mode (FUSE_V: (w1, out), (out, out) for v =
// A phat with w1 = rhat; FUSE_T: the same for t = A shat with w1 = s)
// stored as group sums in k.fpart; FUSE_NONE: z alone (out, w1 unused).
// defer as launch_usweep.  The launch takes the waves per workgroup and the
// load kind of the SpMV shape spmv_variant; fuse_blocks(d.fuse_n0, waves)
// workgroups.
// st may be NULL (no phase test: every system is computed); k supplies the
// vector stride and the partials of the product.  yd (may be NULL): y of
// these rows is the application's input, read from yd (FP64) instead of y.
// lp (FP64 factors, mode FUSE_V): also k.lp = (inv(U_kk) r_k, inv(U_kk)
// v_k) for these rows (see launch_spmv_lp).
template <typename T>
void launch_usweep_spmv(const DevSchedule &d, const double *Ap, size_t a_stride, const T *Dinv, size_t d_stride,
                        const T *y, const double *yd, double *z, double *out, const double *w1, SysState *st,
                        Krylov &k, int nsys, int mode, int spmv_variant, bool defer, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool lp = false);
// Lower parts of BiCGStab's second application on a two-level pattern
// (Schedule::y_in) with FP64 factors.  launch_spmv_lp: v = A phat on the
// rows [fuse_n0, n) exactly as launch_spmv_v with r0 = fuse_n0 (same bits,
// same partials), and in the same walk a_i = sum_k A'_ik inv(U_kk) r_k and
// b_i = sum_k A'_ik inv(U_kk) v_k over the row's lower blocks (k <
// fuse_n0), stored in k.lp at row i.  launch_lower_parts (after the half
// step): shat_i = inv(U_ii) (s_i - (a_i - alpha b_i)) for the rows
// [fuse_n0, n) (the second level, all finished there), which equals the
// lower launch's inv(U_ii) (s_i - sum_k L_ik s_k) up to rounding, since
// L_ik = A'_ik inv(U_kk) there.
void launch_spmv_lp(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant,
                    hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_lower_parts(const DevSchedule &d, const double *Dinv, size_t d_stride, Krylov &k, int nsys,
                        hipStream_t s);
inline int fuse_blocks(int n0, int waves) { return std::max(1, row_blocks(n0, waves)); }
// x_orig[perm[i]] = x'[i]; then r = b - A x_orig with the caller's A, and the
// true relative residual into the states.
void launch_finish(const DevSchedule &d, const int32_t *rowptr, const int32_t *colidx, const double *A,
                   size_t a_stride, const double *b_orig, double *x_orig, Krylov &k, int nsys, int variant, int split,
                   const WellsDev &w, hipStream_t s);

// y = A x on the reordered matrix for the systems still iterating (new
// order, x and y at stride vstride), minus the separate wells.
void launch_spmv_running(const DevSchedule &d, const double *Ap, size_t a_stride, const double *x, double *y,
                         size_t vstride, SysState *st, int nsys, int variant, const WellsDev &w, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int r0 = 0);

// GMRES workspace as the kernels see it.  Vectors of all systems at stride
// vstride; Krylov basis column c of system s at V + c * colstride + s * vstride.
struct GmWork {
    double *V;
    size_t colstride, vstride;
    double *part;        // reduction partials, pstride doubles per system
    size_t pstride;
    uint32_t *tickets;   // reduction counters, tkstride per system
    size_t tkstride;
    GmState *gm;
    SysState *st;
};
inline size_t gm_part_stride() { return (size_t)(kGmMax + 1) * (kVecMaxBlocks + kVecMaxBlocks / 32 + 1) + 16; }

// GMRES building blocks; each acts on the systems still iterating (phase
// PH_RUN) unless stated otherwise.
// A cycle's start after the setup: beta = ||r||, g = beta e_1.
void launch_gm_init(const GmWork &g, int nsys, hipStream_t s);
// V column `col` = src / beta (from_w = 0) or src / h_{j+1,j} (from_w = 1).
void launch_gm_normalise(const GmWork &g, const double *src, int col, int from_w, int n, int nsys, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// First classical Gram-Schmidt pass: h_i = (w, v_i), i < jv; column jv - 1
// of H = h.
void launch_gm_dots(const GmWork &g, int jv, const double *w, int n, int nsys, hipStream_t s,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// w -= V h with the current coefficients; then either the second pass's
// coefficients (added to H's column jv - 1) or, when `last`, ||w|| =
// h_{jv,jv-1}, the Givens update of the column and the step's tests.
void launch_gm_orth(const GmWork &g, int jv, double *w, bool last, int n, int nsys, hipStream_t s,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// End of a cycle, for every system not done: y = H^-1 g, u = V y.
void launch_gm_combine(const GmWork &g, double *u, int n, int nsys, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// x += z for every system not done.
void launch_gm_xupdate(const GmWork &g, double *x, const double *z, int n, int nsys, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// After the update: PH_HALF -> PH_DONE.
void launch_gm_phase(const GmWork &g, int nsys, hipStream_t s);
// Restart: r = rhs - w, beta = ||r||, the reduction test, a fresh cycle.
void launch_gm_restart(const GmWork &g, const double *rhs, const double *w, double *r, int n, int nsys,
                       hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// p[0 .. count) = value, by a kernel (no memset node when the stream is
// being captured).
void launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t s);

// out[i] = in[perm[i]] (gather to the new order) and its inverse scatter;
// the new-order side has stride vstride, the caller side 3n.
void launch_permute_vec(const int32_t *perm, const double *in, double *out, int n, size_t vstride, int nsys,
                        bool scatter, hipStream_t s);

}  // namespace rs
