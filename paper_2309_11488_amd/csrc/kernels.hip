// HIP kernels (gfx950) of the BCSR 3x3 BiCGStab-ILU0 path.
//
// Row kernels (SpMV, ILU0 sweeps, ILU0 factor) give each block row three
// lanes, one per row of the 3x3 blocks: 21 rows per 64-wide wavefront (lane
// 63 idle), 84 rows per 256-thread workgroup.  The values of a workgroup's
// rows are one contiguous range (rows are stored level by level), so they are
// first copied into LDS with fully coalesced loads, then each lane walks its
// row's blocks from LDS.  This is the blocked SpMV idea of Eberhardt and
// Hoemmen cited in Section "Sparse Matrix-Vector multiplication" (lanes with a
// fixed position inside a block), re-shaped for wave64 and LDS.
//
// Reductions are deterministic: every workgroup writes its partial sum, and
// the last workgroup to arrive (ticket counter) adds the partials in a fixed
// order and updates the BiCGStab scalars on the device.  The number of
// workgroups depends only on the system size, so a system gives the same bits
// alone and inside a batch.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <climits>

#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "../../include/rsolve.h"

namespace rs {

namespace {

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap the linear
// workgroup id so each XCD gets one contiguous run of (system, tile) pairs:
// neighbouring tiles then share x/y lines in that XCD's L2.
__device__ inline void xcd_map(int &sys, int &bx) {
    const unsigned gx = gridDim.x, total = gx * gridDim.y;
    const unsigned lin = blockIdx.x + blockIdx.y * gx;
    const unsigned q = total / 8u, rem = total % 8u, xcd = lin % 8u, k = lin / 8u;
    const unsigned logical = (xcd < rem ? xcd * (q + 1u) : rem * (q + 1u) + (xcd - rem) * q) + k;
    sys = (int)(logical / gx);
    bx = (int)(logical % gx);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the workgroup; thread 0 gets the result.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < NV; ++k) lds[w * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int i = 0; i < nw; ++i) s += lds[i * NV + k];
            v[k] = s;
        }
    __syncthreads();
}

// Deterministic grid reduction.  Returns true in the last workgroup to
// finish, where thread 0's v[] holds the grid total.
//
// Two-level ticket tree, so no counter takes more than a few hundred
// atomics: workgroups form groups of kGroup consecutive (logical) ids.  Each
// workgroup stores its partials with agent-scope atomic stores (written
// through to the coherence point, so no writeback of the whole XCD L2 is
// needed), waits until they have completed, then takes a ticket on its
// group's counter.  The last workgroup of a group adds the group's partials
// in id order, stores the group partial the same way and takes a ticket on
// the top counter; the last group's workgroup adds the group partials in
// group order.  Counters are reset by their last taker.  The tree depends
// only on the number of workgroups, so results are reproducible bit for bit.
// Layout: part[0 .. nblk*NV) block partials, then group partials;
// tickets[0] = top counter, tickets[kTicketPad * (1 + g)] = counter of
// group g (one 128-byte line per counter, so groups do not contend).
constexpr int kGroup = 32;

template <int NV>
__device__ bool grid_reduce(double (&v)[NV], double *part, uint32_t *tickets, int nblk, int bx) {
    __shared__ double lds[16 * NV];
    __shared__ int glast, last;
    block_sum<NV>(v, lds);
    const int ng = (nblk + kGroup - 1) / kGroup, g = bx / kGroup;
    const int gsize = min(kGroup, nblk - g * kGroup);
    double *gpart = part + (size_t)nblk * NV;
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(part + (size_t)bx * NV + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t t = __hip_atomic_fetch_add(tickets + (size_t)kTicketPad * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        glast = t == (uint32_t)(gsize - 1);
        last = 0;
    }
    __syncthreads();
    if (glast) {
        // group reduction by wave 0: one partial per lane, butterfly sum
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            double gs[NV];
            for (int k = 0; k < NV; ++k) {
                const double p = lane < gsize ? __hip_atomic_load(part + (size_t)(g * kGroup + lane) * NV + k,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                              : 0.0;
                gs[k] = wave_sum(p);
            }
            if (lane == 0) {
                __hip_atomic_store(tickets + (size_t)kTicketPad * (1 + g), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int k = 0; k < NV; ++k)
                    __hip_atomic_store(gpart + (size_t)g * NV + k, gs[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_s_waitcnt(0);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                const uint32_t t2 = __hip_atomic_fetch_add(tickets, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t2 == (uint32_t)(ng - 1)) {
                    __hip_atomic_store(tickets, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    last = 1;
                }
            }
        }
        __syncthreads();
    }
    if (!last) return false;
    double acc[NV];
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    constexpr int U = NV <= 2 ? 4 : 1;   // same order either way; wide NV keeps registers
    for (int b0 = 0; b0 < ng; b0 += U * (int)blockDim.x) {
        double t[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * blockDim.x + threadIdx.x;
            for (int k = 0; k < NV; ++k)
                t[u][k] = b < ng ? __hip_atomic_load(gpart + (size_t)b * NV + k, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            for (int k = 0; k < NV; ++k) acc[k] += t[u][k];
    }
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) v[k] = acc[k];
    return true;
}

// First level of grid_reduce only: the last workgroup of each group of
// kGroup stores the group's sum at part[nblk*NV + g*NV].  A later kernel adds
// the ceil(nblk / kGroup) group sums (no top-level counter, no serial tail).
template <int NV>
__device__ void group_reduce(double (&v)[NV], double *part, uint32_t *tickets, int nblk, int bx) {
    __shared__ double lds[16 * NV];
    __shared__ int glast;
    block_sum<NV>(v, lds);
    const int g = bx / kGroup, gsize = min(kGroup, nblk - g * kGroup);
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(part + (size_t)bx * NV + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t t = __hip_atomic_fetch_add(tickets + (size_t)kTicketPad * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        glast = t == (uint32_t)(gsize - 1);
    }
    __syncthreads();
    if (glast && threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double gs[NV];
        for (int k = 0; k < NV; ++k) {
            const double p = lane < gsize ? __hip_atomic_load(part + (size_t)(g * kGroup + lane) * NV + k,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                          : 0.0;
            gs[k] = wave_sum(p);
        }
        if (lane == 0) {
            __hip_atomic_store(tickets + (size_t)kTicketPad * (1 + g), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 0; k < NV; ++k) part[(size_t)nblk * NV + (size_t)g * NV + k] = gs[k];
        }
    }
}

__device__ inline bool finite(double x) { return __builtin_isfinite(x); }

// One block-row times a 3-vector, b0 x0 + b1 x1 + b2 x2, with the fused
// multiply-adds written out so every code path rounds the same way.
__device__ inline double dot3(double b0, double b1, double b2, double x0, double x1, double x2) {
    return __builtin_fma(b2, x2, __builtin_fma(b1, x1, b0 * x0));
}
__device__ inline float dot3(float b0, float b1, float b2, float x0, float x1, float x2) {
    return __builtin_fmaf(b2, x2, __builtin_fmaf(b1, x1, b0 * x0));
}

// Lane geometry of the row kernels.
struct RowLane {
    int q;      // row position in the launch's range
    int r;      // row inside the 3x3 block
    int base;   // first lane of this block row in the wave
    bool act;
};

template <int W>
__device__ inline RowLane row_lane(int bx, int q0, int q1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    RowLane L;
    L.q = q0 + bx * (W * kRowsPerWave) + w * kRowsPerWave + lane / 3;
    L.r = lane % 3;
    L.base = lane - L.r;
    L.act = lane < 63 && L.q < q1;
    return L;
}

// LDS image of up to CAP consecutive 3x3 blocks and their column indices.
// Values are copied in aligned 16-byte units; `shift` is the offset (in
// elements) of the first block inside the first unit.
template <typename T, int CAP, int NT = kRowThreads>
struct Stage {
    static constexpr int kThreads = NT;
    static constexpr int kUnits = (CAP * 9 * (int)sizeof(T) + 15) / 16 + 1;
    static constexpr int kPerThread = (kUnits + NT - 1) / NT;
    static constexpr int kColsPerThread = (CAP + NT - 1) / NT;
    uint4 v[kUnits];
    int32_t c[CAP];
};

// Copy blocks [base, base + cnt) of val and col into LDS.  Every thread
// issues all of its loads before any LDS store.  Load and store indices are
// clamped into range instead of branched on (threads past the end rewrite
// the last unit with the same data), so the compiler cannot sink a load
// into a branch and serialise the copy.  Reads stay inside the 16-byte
// units that overlap the range (allocations are padded for that).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// NTL: blocks and column indices, read once per launch, are loaded
// non-temporally, so the caches keep the gathered x entries instead (pays
// when x outgrows an XCD's L2; the autotuner decides).
template <typename T, int CAP, int NT, bool NTL = false>
__device__ inline int stage_copy(const T *__restrict__ val, const int32_t *__restrict__ col, int base, int cnt,
                                 Stage<T, CAP, NT> &st) {
    using S = Stage<T, CAP, NT>;
    const char *first = (const char *)(val + (size_t)base * 9);
    const int mis = (int)((uintptr_t)first & 15);
    const u32x4 *src = (const u32x4 *)(first - mis);
    const int units = (mis + cnt * 9 * (int)sizeof(T) + 15) / 16;
    uint4 t[S::kPerThread];
#pragma unroll
    for (int u = 0; u < S::kPerThread; ++u) {
        const u32x4 *a = src + min(u * NT + (int)threadIdx.x, units - 1);
        const u32x4 w = NTL ? __builtin_nontemporal_load(a) : *a;
        t[u] = make_uint4(w.x, w.y, w.z, w.w);
    }
    int32_t c[S::kColsPerThread];
#pragma unroll
    for (int u = 0; u < S::kColsPerThread; ++u) {
        const int32_t *a = col + base + min(u * NT + (int)threadIdx.x, cnt - 1);
        c[u] = NTL ? __builtin_nontemporal_load(a) : *a;
    }
#pragma unroll
    for (int u = 0; u < S::kPerThread; ++u) st.v[min(u * NT + (int)threadIdx.x, units - 1)] = t[u];
#pragma unroll
    for (int u = 0; u < S::kColsPerThread; ++u) st.c[min(u * NT + (int)threadIdx.x, cnt - 1)] = c[u];
    return mis / (int)sizeof(T);
}

// acc (+|-)= sum_c val[e][r][c] * x[3 col[e] + c] over this lane's blocks
// e in [lo, hi), all staged in LDS from `base`; blocks ascending.  The x
// entries of up to 8 blocks are gathered before use; COH gathers them with
// agent-coherent loads (x written by other workgroups of the same launch).
template <bool SUB, bool COH, typename T, typename TX>
__device__ inline T walk_pass(const T *sv, const int32_t *sc, int shift, int base, int lo, int hi, int r,
                              const TX *__restrict__ x, T acc) {
    for (int e = lo; e < hi; e += 8) {
        TX xv[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = sc[min(e + u, hi - 1) - base];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                xv[u][c] = COH ? __hip_atomic_load(x + 3 * j + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : x[3 * j + c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e + u < hi) {
                const T *b = sv + shift + (e + u - base) * 9 + 3 * r;
                const T s = dot3(b[0], b[1], b[2], (T)xv[u][0], (T)xv[u][1], (T)xv[u][2]);
                if (SUB) acc -= s; else acc += s;
            }
    }
    return acc;
}

// The same sum with blocks and column indices read straight from global
// memory (no LDS): each lane loads its 24-byte row slice of 8 blocks, their
// columns, then the x entries, before any arithmetic.
template <bool SUB, typename T, typename TX>
__device__ inline T direct_walk(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                const T *__restrict__ val, const RowLane &L, const TX *__restrict__ x, T acc) {
    if (!L.act) return acc;
    const int my0 = ptr[L.q], my1 = ptr[L.q + 1];
    for (int e = my0; e < my1; e += 8) {
        int j[8];
        T b[8][3];
        TX xv[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ee = min(e + u, my1 - 1);
            j[u] = col[ee];
            const T *bp = val + (size_t)ee * 9 + 3 * L.r;
            b[u][0] = bp[0]; b[u][1] = bp[1]; b[u][2] = bp[2];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            for (int c = 0; c < 3; ++c) xv[u][c] = x[3 * j[u] + c];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e + u < my1) {
                const T s = dot3(b[u][0], b[u][1], b[u][2], (T)xv[u][0], (T)xv[u][1], (T)xv[u][2]);
                if (SUB) acc -= s; else acc += s;
            }
    }
    return acc;
}

// Walk the blocks of this lane's row, staged through LDS pass by pass.
template <int CAP, bool SUB, bool NTL, typename T, typename TX, int NT>
__device__ inline T stage_walk(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                               const T *__restrict__ val, int qb0, int qb1, const RowLane &L, const TX *__restrict__ x,
                               T acc, Stage<T, CAP, NT> &st) {
    const int e0 = ptr[qb0], e1 = ptr[qb1];
    const int my0 = L.act ? ptr[L.q] : 0, my1 = L.act ? ptr[L.q + 1] : 0;
    for (int base = e0; base < e1; base += CAP) {
        const int cnt = min(CAP, e1 - base);
        __syncthreads();
        const int shift = stage_copy<T, CAP, NT, NTL>(val, col, base, cnt, st);
        __syncthreads();
        acc = walk_pass<SUB, false>((const T *)st.v, st.c, shift, base, max(my0, base), min(my1, base + cnt), L.r,
                                    x, acc);
    }
    return acc;
}

// Row kernels are compiled to keep at least this many waves per SIMD (the
// register budget that leaves; no spills at 5) so their dependent gathers
// have enough waves in flight.
constexpr int kRowWavesPerEU = 5;

// LDS capacity (blocks) per pass: 160 (SpMV) or 128 (per-level sweeps) per
// wave, so a workgroup of 7-block rows copies its blocks in one pass; the
// single-launch sweeps' tiles keep 80 per wave (more workgroups resident to
// wait on their dependencies).
constexpr int kSpmvCapPerWave = 160;
constexpr int kSweepCapPerWave = 128;
constexpr int kSweepCap = 4 * 80;   // single-launch sweeps: 4-wave workgroups

// Row walk of a workgroup of W waves: staged through LDS or direct.
template <int W, int STAGE, int CAPW, bool SUB, typename T, typename TX>
__device__ inline T row_walk(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const T *__restrict__ val, int qb0, int qb1, const RowLane &L, const TX *__restrict__ x,
                             T acc) {
    if constexpr (STAGE != 0) {
        __shared__ Stage<T, CAPW * W, 64 * W> sv;
        return stage_walk<CAPW * W, SUB, STAGE == 2>(ptr, col, val, qb0, qb1, L, x, acc, sv);
    } else {
        return direct_walk<SUB>(ptr, col, val, L, x, acc);
    }
}

// ------------------------------------------------------------------ gather

__global__ void k_gather_pairs(const double *__restrict__ A, size_t a_stride, double *__restrict__ Ap,
                               size_t ap_stride, const int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                               int cnt) {
    const int sys = blockIdx.y;
    const size_t total = (size_t)cnt * 9;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t p = t / 9, e = t % 9;
        Ap[sys * ap_stride + (size_t)dst[p] * 9 + e] = A[sys * a_stride + (size_t)src[p] * 9 + e];
    }
}

// ------------------------------------------------------------------ factor

// Rows with at most FM lower and FM upper blocks keep their slices in
// registers; longer rows work through global memory.  FM is the level's
// register width: kFactorNarrow when every row of the level fits it (the
// 7-point grids under colouring), else kFactorWide.  The narrow kernel's
// 148 VGPRs allow three waves per SIMD, the wide kernel's 176 two.
constexpr int kFactorNarrow = 6, kFactorWide = 8;

__device__ inline void row3_load(const double *p, double (&v)[3]) { v[0] = p[0]; v[1] = p[1]; v[2] = p[2]; }
__device__ inline void row3_store(double *p, const double (&v)[3]) { p[0] = v[0]; p[1] = v[1]; p[2] = v[2]; }
__device__ inline void row3_store(float *p, const double (&v)[3]) {
    p[0] = (float)v[0]; p[1] = (float)v[1]; p[2] = (float)v[2];
}
// out = row (a0 a1 a2) times the 3x3 block m
// out = a m for a 3x3 block m of another block row, which all three lanes of
// this block row need whole: lane r loads row r of m (mr = m + 3r) and the
// rows are exchanged with shuffles, so each lane issues three loads instead
// of nine.  All three lanes of the row must take this call together.
__device__ inline void row3_mul(const double (&a)[3], const double *__restrict__ mr, int base, double (&out)[3]) {
    const double r0 = mr[0], r1 = mr[1], r2 = mr[2];
    double m[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m[k][0] = __shfl(r0, base + k, 64);
        m[k][1] = __shfl(r1, base + k, 64);
        m[k][2] = __shfl(r2, base + k, 64);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = __builtin_fma(a[2], m[2][c], __builtin_fma(a[1], m[1][c], a[0] * m[0][c]));
}

// Row r of inv(a) for a 3x3 block a (row-major) from the adjugate: the
// cofactors of row r's column, divided by the determinant (expanded along
// the first row), which is returned.
__device__ inline double inv3_row(const double (&a)[9], int r, double (&inv)[3]) {
    const double c00 = a[4] * a[8] - a[5] * a[7];
    const double c01 = a[5] * a[6] - a[3] * a[8];
    const double c02 = a[3] * a[7] - a[4] * a[6];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (r == 0) { inv[0] = c00 / det; inv[1] = (a[2] * a[7] - a[1] * a[8]) / det; inv[2] = (a[1] * a[5] - a[2] * a[4]) / det; }
    else if (r == 1) { inv[0] = c01 / det; inv[1] = (a[0] * a[8] - a[2] * a[6]) / det; inv[2] = (a[2] * a[3] - a[0] * a[5]) / det; }
    else { inv[0] = c02 / det; inv[1] = (a[1] * a[6] - a[0] * a[7]) / det; inv[2] = (a[0] * a[4] - a[1] * a[3]) / det; }
    return det;
}

// Block ILU0, one level of the lower schedule.  Lane r of row i owns row r of
// every block of block row i.  In Algorithm 2's order: for each lower block
// (i,k), k ascending, L_ik = a_ik inv(U_kk); then a_ij -= L_ik U_kj over the
// precomputed update list (j ascending).  Finally inv(U_ii) from the
// adjugate; a singular or non-finite pivot is reported by its new index.
// The row's blocks come straight from the caller's matrix and are also
// written to the reordered copy used by the SpMV, so no separate gather
// pass reads A.  With STAGED (the launch's rows are consecutive in the new
// order, and every block of their reordered rows is written here), a
// workgroup whose rows hold at most kApCap blocks collects that copy in LDS
// and writes its contiguous range out with consecutive stores, instead of
// every lane storing 8-byte pieces spread over 21 rows.  FM: the register
// width (kFactorNarrow only for levels whose rows all fit it).
constexpr int kApCap = 640;

template <bool F32, bool STAGED, int FM>
__global__ void __launch_bounds__(kRowThreads) k_factor_level(DevSchedule d, const double *__restrict__ A,
                                                              size_t a_stride, double *__restrict__ Ap,
                                                              double *__restrict__ L, double *__restrict__ U,
                                                              double *__restrict__ Dinv, float *__restrict__ Lf,
                                                              float *__restrict__ Uf, float *__restrict__ Df,
                                                              int32_t *__restrict__ bad, int q0, int q1, int skip_u0,
                                                              int last) {
    __shared__ double sap[STAGED ? kApCap * 9 : 1];
    int sys, bx;
    xcd_map(sys, bx);
    const RowLane rl = row_lane<kWavesPerBlock>(bx, q0, q1);
    const double *As = A + (size_t)sys * a_stride;
    double *Aps = Ap + (size_t)sys * d.nnzb * 9;
    double *Ls = L + (size_t)sys * d.nL * 9;
    double *Us = U + (size_t)sys * d.nU * 9;
    double *Ds = Dinv + (size_t)sys * d.n * 9;
    const int r = rl.r;
    // the workgroup's range of the reordered copy (rows consecutive)
    int ap0 = 0, apn = kApCap + 1;
    // and of L (the L blocks of consecutive L-schedule rows are consecutive)
    int l0 = 0, ln = 0;
    if (STAGED) {
        const int qb0 = q0 + bx * kRowsPerBlock, qb1 = min(qb0 + kRowsPerBlock, q1);
        const int i0 = d.lrows[qb0];
        ap0 = d.prow[i0];
        apn = d.prow[i0 + (qb1 - qb0)] - ap0;
        l0 = d.lptr[qb0];
        ln = d.lptr[qb1] - l0;
    }
    const bool stage = STAGED && apn <= kApCap;
    // On a narrow level (launch_factor_level is given narrow only when no
    // row of the level holds more than kFactorNarrow lower or upper blocks)
    // every row takes the register path below, so the workgroup's L blocks
    // all sit in registers once the rows are done: they
    // go through the same LDS after the copy has left it, and out as one
    // range, instead of as 24-byte slices spread over 21 rows per store.
    constexpr bool SL = STAGED && FM == kFactorNarrow;
    const bool stage_l = SL && stage && ln <= (F32 ? 2 : 1) * kApCap;
    double lkeep[SL ? FM : 1][3];
    int le0 = 0, le1 = 0;
    auto ap_store = [&](int pos, const double (&v)[3]) {
        if (stage) {
            double *t = sap + (size_t)(pos - ap0) * 9 + 3 * r;
            t[0] = v[0]; t[1] = v[1]; t[2] = v[2];
        } else {
            row3_store(Aps + (size_t)pos * 9 + 3 * r, v);
        }
    };
    double dr[3] = {0.0, 0.0, 0.0};
    int uq = 0;
    if (rl.act) {
        const int q = rl.q;
        uq = d.l2u[q];
        const int e0 = d.lptr[q], e1 = d.lptr[q + 1], f0 = d.uptr[uq], f1 = d.uptr[uq + 1];
        row3_load(As + (size_t)d.dsrc_a[uq] * 9 + 3 * r, dr);
        ap_store(d.dsrc[uq], dr);
        if (e1 - e0 <= FM && f1 - f0 <= FM) {
            double lv[FM][3], uv[FM][3];
            int dq[FM];
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (e0 + t < e1) {
                    row3_load(As + (size_t)d.lsrc_a[e0 + t] * 9 + 3 * r, lv[t]);
                    dq[t] = d.ldq[e0 + t];
                }
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (f0 + t < f1) row3_load(As + (size_t)d.usrc_a[f0 + t] * 9 + 3 * r, uv[t]);
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (e0 + t < e1) ap_store(d.lsrc[e0 + t], lv[t]);
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (f0 + t < f1) ap_store(d.usrc[f0 + t], uv[t]);
#pragma unroll
            for (int t = 0; t < FM; ++t) {
                if (e0 + t >= e1) continue;
                double l[3];
                row3_mul(lv[t], Ds + (size_t)dq[t] * 9 + 3 * r, rl.base, l);
                lv[t][0] = l[0]; lv[t][1] = l[1]; lv[t][2] = l[2];
                const int u1 = d.upd_ptr[e0 + t + 1];
                for (int u = d.upd_ptr[e0 + t]; u < u1; ++u) {
                    const int code = d.upd[2 * u], fs = d.upd[2 * u + 1];
                    double pr[3];
                    row3_mul(l, (fs >= 0 ? Us + (size_t)fs * 9 : Aps + (size_t)~fs * 9) + 3 * r, rl.base, pr);
                    const int kind = code & 3, pos = code >> 2;
                    if (kind == 1) {
                        dr[0] -= pr[0]; dr[1] -= pr[1]; dr[2] -= pr[2];
                    } else if (kind == 0) {
#pragma unroll
                        for (int j = 0; j < FM; ++j)
                            if (j == pos - e0) { lv[j][0] -= pr[0]; lv[j][1] -= pr[1]; lv[j][2] -= pr[2]; }
                    } else {
#pragma unroll
                        for (int j = 0; j < FM; ++j)
                            if (j == pos - f0) { uv[j][0] -= pr[0]; uv[j][1] -= pr[1]; uv[j][2] -= pr[2]; }
                    }
                }
            }
            le0 = e0;
            le1 = e1;
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (e0 + t < e1) {
                    if constexpr (SL) {
                        if (stage_l) {
                            lkeep[t][0] = lv[t][0]; lkeep[t][1] = lv[t][1]; lkeep[t][2] = lv[t][2];
                            continue;
                        }
                    }
                    // later levels never read L: with FP32 factors only the FP32 copy is kept
                    if (F32) row3_store(Lf + ((size_t)sys * d.nL + e0 + t) * 9 + 3 * r, lv[t]);
                    else row3_store(Ls + (size_t)(e0 + t) * 9 + 3 * r, lv[t]);
                }
            // with FP32 factors the FP64 U is only read by later levels'
            // updates, which take a row without lower blocks from the
            // reordered copy instead
            const bool keep_u = e1 > e0 || (!F32 && !skip_u0);
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (f0 + t < f1) {
                    if (keep_u) row3_store(Us + (size_t)(f0 + t) * 9 + 3 * r, uv[t]);
                    if (F32 && (e1 > e0 || !skip_u0)) row3_store(Uf + ((size_t)sys * d.nU + f0 + t) * 9 + 3 * r, uv[t]);
                }
        } else {
            // long rows: the same steps on the row's blocks in global memory
            for (int f = f0; f < f1; ++f) {
                double a[3];
                row3_load(As + (size_t)d.usrc_a[f] * 9 + 3 * r, a);
                ap_store(d.usrc[f], a);
                row3_store(Us + (size_t)f * 9 + 3 * r, a);
            }
            for (int e = e0; e < e1; ++e) {
                double a[3];
                row3_load(As + (size_t)d.lsrc_a[e] * 9 + 3 * r, a);
                ap_store(d.lsrc[e], a);
                row3_store(Ls + (size_t)e * 9 + 3 * r, a);
            }
            for (int e = e0; e < e1; ++e) {
                double *le = Ls + (size_t)e * 9 + 3 * r;
                double a[3], l[3];
                row3_load(le, a);
                row3_mul(a, Ds + (size_t)d.ldq[e] * 9 + 3 * r, rl.base, l);
                row3_store(le, l);
                for (int u = d.upd_ptr[e]; u < d.upd_ptr[e + 1]; ++u) {
                    const int code = d.upd[2 * u], fs = d.upd[2 * u + 1];
                    double pr[3];
                    row3_mul(l, (fs >= 0 ? Us + (size_t)fs * 9 : Aps + (size_t)~fs * 9) + 3 * r, rl.base, pr);
                    const int kind = code & 3, pos = code >> 2;
                    if (kind == 1) {
                        dr[0] -= pr[0]; dr[1] -= pr[1]; dr[2] -= pr[2];
                    } else {
                        double *t = (kind == 0 ? Ls : Us) + (size_t)pos * 9 + 3 * r;
                        t[0] -= pr[0]; t[1] -= pr[1]; t[2] -= pr[2];
                    }
                }
            }
            if (F32) {
                for (int e = e0; e < e1; ++e) {
                    double a[3];
                    row3_load(Ls + (size_t)e * 9 + 3 * r, a);
                    row3_store(Lf + ((size_t)sys * d.nL + e) * 9 + 3 * r, a);
                }
                for (int f = f0; f < f1; ++f) {
                    double a[3];
                    row3_load(Us + (size_t)f * 9 + 3 * r, a);
                    row3_store(Uf + ((size_t)sys * d.nU + f) * 9 + 3 * r, a);
                }
            }
        }
    }
    if (stage) {
        // the workgroup's part of the reordered copy, consecutive stores
        __syncthreads();
        double *dst = Aps + (size_t)ap0 * 9;
        for (int k = threadIdx.x; k < apn * 9; k += kRowThreads) dst[k] = sap[k];
    }
    if constexpr (SL) {
      if (stage_l) {
        __syncthreads();   // the copy has been read out of the LDS
        if (rl.act) {
#pragma unroll
            for (int t = 0; t < FM; ++t)
                if (le0 + t < le1) {
                    const size_t o = (size_t)(le0 + t - l0) * 9 + 3 * r;
                    if (F32) {
                        float *sl = (float *)sap + o;
                        sl[0] = (float)lkeep[t][0]; sl[1] = (float)lkeep[t][1]; sl[2] = (float)lkeep[t][2];
                    } else {
                        sap[o] = lkeep[t][0]; sap[o + 1] = lkeep[t][1]; sap[o + 2] = lkeep[t][2];
                    }
                }
        }
        __syncthreads();
        if (F32) {
            const float *sl = (const float *)sap;
            float *dst = Lf + ((size_t)sys * d.nL + l0) * 9;
            for (int k = threadIdx.x; k < ln * 9; k += kRowThreads) dst[k] = sl[k];
        } else {
            double *dst = Ls + (size_t)l0 * 9;
            for (int k = threadIdx.x; k < ln * 9; k += kRowThreads) dst[k] = sap[k];
        }
      }
    }
    // gather the three rows of U_ii from the row's lanes
    double a[9];
    for (int rr = 0; rr < 3; ++rr) {
        a[3 * rr + 0] = __shfl(dr[0], rl.base + rr, 64);
        a[3 * rr + 1] = __shfl(dr[1], rl.base + rr, 64);
        a[3 * rr + 2] = __shfl(dr[2], rl.base + rr, 64);
    }
    if (!rl.act) return;
    double inv[3];
    const double det = inv3_row(a, r, inv);
    // with FP32 factors the FP64 pivot inverses serve only later levels
    if (!F32 || !last) row3_store(Ds + (size_t)uq * 9 + 3 * r, inv);
    if (F32) row3_store(Df + ((size_t)sys * d.n + uq) * 9 + 3 * r, inv);
    if (r == 0 && (det == 0.0 || !finite(det))) atomicMin(bad + sys, d.lrows[rl.q]);
}

// The first level of the factorisation when it is the rows [0, fuse_n0) of
// the new order (no lower blocks: Schedule::fuse_n0).  Nothing updates these
// rows, so their part of the reordered copy is the caller's blocks moved to
// new positions and inv(U_ii) = inv(A_ii); their U is not stored (the
// upper launches read it from the copy).  A workgroup copies the blocks of
// kFirstRows consecutive rows, one 8-byte element per thread and step, so
// consecutive threads load and store consecutive elements, then inverts
// their diagonal blocks (the first block of each row), one row per thread.
constexpr int kFirstRows = 64;
constexpr int kFirstUnroll = 4;

template <bool F32>
__global__ void __launch_bounds__(kRowThreads) k_factor_first(DevSchedule d, const double *__restrict__ A,
                                                              size_t a_stride, double *__restrict__ Ap,
                                                              double *__restrict__ Dinv, float *__restrict__ Df,
                                                              int32_t *__restrict__ bad) {
    const int sys = blockIdx.y;
    const int n0 = d.fuse_n0;
    const int i0 = blockIdx.x * kFirstRows, i1 = min(i0 + kFirstRows, n0);
    const double *As = A + (size_t)sys * a_stride;
    double *Aps = Ap + (size_t)sys * d.nnzb * 9;
    const long long t0 = 9LL * d.prow[i0], t1 = 9LL * d.prow[i1];
    for (long long tb = t0; tb < t1; tb += kFirstUnroll * kRowThreads) {
        double v[kFirstUnroll];
#pragma unroll
        for (int u = 0; u < kFirstUnroll; ++u) {
            const long long t = min(tb + u * kRowThreads + (int)threadIdx.x, t1 - 1);
            const int p = (int)(t / 9);
            v[u] = As[(size_t)d.psrc[p] * 9 + (int)(t - 9LL * p)];
        }
#pragma unroll
        for (int u = 0; u < kFirstUnroll; ++u) {
            const long long t = tb + u * kRowThreads + (int)threadIdx.x;
            if (t < t1) Aps[t] = v[u];
        }
    }
    const int i = i0 + (int)threadIdx.x;
    if (i >= i1) return;
    const int uq = d.fuse_q0 + i;
    const double *src = As + (size_t)d.dsrc_a[uq] * 9;
    double a[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) a[e] = src[e];
    double *Ds = Dinv + ((size_t)sys * d.n + uq) * 9;
    double det = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double inv[3];
        det = inv3_row(a, r, inv);
        row3_store(Ds + 3 * r, inv);
        if (F32) row3_store(Df + ((size_t)sys * d.n + uq) * 9 + 3 * r, inv);
    }
    if (det == 0.0 || !finite(det)) atomicMin(bad + sys, i);
}

// ------------------------------------------------------------------ sweeps

// YIN: the rows' lower neighbours hold no lower blocks, so their y is the
// application's input itself: the walk reads it from yd (FP64, rounded to
// T as the stored y would be), and no y is stored (every row of such a
// launch finishes here).
template <typename T, bool FUSE_P, int W, int STAGE, bool YIN>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kRowWavesPerEU, 8))) k_lsweep(DevSchedule d, const T *__restrict__ L, size_t l_stride,
                                                        const double *__restrict__ in, T *__restrict__ y,
                                                        size_t vstride, const double *__restrict__ rv,
                                                        const double *__restrict__ vv, double *__restrict__ pv,
                                                        SysState *__restrict__ st, int q0, int q1,
                                                        const T *__restrict__ Dinv, size_t d_stride,
                                                        double *__restrict__ z, int u0_end, const double *yd) {
    int sys, bx;
    xcd_map(sys, bx);
    // The fused sweep opens an iteration, which is queued only while the
    // system runs (or past its end, rarely): its phase test waits until the
    // walk's loads are in flight.  The other sweep may follow a half-step
    // stop and tests first.
    if (!FUSE_P && st && st[sys].phase != PH_RUN) return;
    const bool run = !FUSE_P || !st || st[sys].phase == PH_RUN;
    const RowLane rl = row_lane<W>(bx, q0, q1);
    const int qb0 = q0 + bx * W * kRowsPerWave, qb1 = min(qb0 + W * kRowsPerWave, q1);
    const size_t vo = (size_t)sys * vstride;
    const int i = rl.act ? d.lrows[rl.q] : 0;
    const int uq = (u0_end > 0 && rl.act) ? d.l2u[rl.q] : INT_MAX;
    const size_t k = vo + 3 * (size_t)i + rl.r;
    T acc = 0;
    double p = 0.0;
    if (rl.act) {
        if (FUSE_P) {
            const double beta = st[sys].beta, omega = st[sys].omega;
            p = rv[k] + beta * (pv[k] - omega * vv[k]);
            acc = (T)p;
        } else {
            acc = (T)in[k];
        }
    }
    // inv(U_ii) of a row the launch finishes is requested before the walk
    T dq[3] = {0, 0, 0};
    if (uq < u0_end) {
        const T *dp = Dinv + (size_t)sys * d_stride + (size_t)uq * 9 + 3 * rl.r;
        dq[0] = dp[0]; dq[1] = dp[1]; dq[2] = dp[2];
    }
    if constexpr (YIN)
        acc = row_walk<W, STAGE, kSweepCapPerWave, true>(d.lptr, d.lcol, L + (size_t)sys * l_stride, qb0, qb1, rl,
                                                         yd + vo, acc);
    else
        acc = row_walk<W, STAGE, kSweepCapPerWave, true>(d.lptr, d.lcol, L + (size_t)sys * l_stride, qb0, qb1, rl,
                                                         y + vo, acc);
    if (FUSE_P) {
        asm volatile("" ::"v"(acc));
        if (!run) return;
        if (rl.act) pv[k] = p;
    }
    // y of a row the launch finishes is read by no later launch
    if (!YIN && rl.act && uq >= u0_end) y[k] = acc;
    if (u0_end > 0) {
        // rows without upper blocks (the first level of the upper sweep)
        // finish here: z_i = inv(U_ii) y_i, the arithmetic of k_usweep
        const T t0 = __shfl(acc, rl.base, 64), t1 = __shfl(acc, rl.base + 1, 64), t2 = __shfl(acc, rl.base + 2, 64);
        if (uq < u0_end) z[vo + 3 * (size_t)i + rl.r] = (double)dot3(dq[0], dq[1], dq[2], t0, t1, t2);
    }
}

template <typename T, int W, int STAGE>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kRowWavesPerEU, 8))) k_usweep(DevSchedule d, const T *__restrict__ U, size_t u_stride,
                                                        const T *__restrict__ Dinv, size_t d_stride,
                                                        const T *__restrict__ y, double *__restrict__ z,
                                                        size_t vstride, SysState *__restrict__ st, int q0, int q1,
                                                        int defer) {
    int sys, bx;
    xcd_map(sys, bx);
    // defer: the phase test waits until the walk's loads are in flight
    // (the sweep of an iteration's first application, as in k_lsweep)
    if (!defer && st && st[sys].phase != PH_RUN) return;
    const bool run = !st || st[sys].phase == PH_RUN;
    const RowLane rl = row_lane<W>(bx, q0, q1);
    const int qb0 = q0 + bx * W * kRowsPerWave, qb1 = min(qb0 + W * kRowsPerWave, q1);
    const size_t vo = (size_t)sys * vstride;
    const int i = rl.act ? d.urows[rl.q] : 0;
    T acc = rl.act ? y[vo + 3 * (size_t)i + rl.r] : (T)0;
    // inv(U_ii) is requested before the walk
    T dq[3] = {0, 0, 0};
    if (rl.act) {
        const T *dp = Dinv + (size_t)sys * d_stride + (size_t)rl.q * 9 + 3 * rl.r;
        dq[0] = dp[0]; dq[1] = dp[1]; dq[2] = dp[2];
    }
    acc = row_walk<W, STAGE, kSweepCapPerWave, true>(d.uptr, d.ucol, U + (size_t)sys * u_stride, qb0, qb1, rl, z + vo,
                                                     acc);
    asm volatile("" ::"v"(acc));
    if (!run) return;
    const T t0 = __shfl(acc, rl.base, 64), t1 = __shfl(acc, rl.base + 1, 64), t2 = __shfl(acc, rl.base + 2, 64);
    if (!rl.act) return;
    const T zr = dot3(dq[0], dq[1], dq[2], t0, t1, t2);
    z[vo + 3 * (size_t)i + rl.r] = (double)zr;
}

// ------------------------------------------------ single-launch sweeps

// Tiles are handed out by an atomic ticket in schedule order (tile-major,
// system-minor), so a workgroup only ever waits for items with smaller
// tickets, which are held by running workgroups: the launch cannot
// deadlock, whatever the number of resident workgroups.  A tile first copies
// its factor blocks into LDS (independent of the solution), then waits until
// every tile it depends on carries this sweep's epoch, computes, writes its
// rows with agent-coherent stores, waits for those stores to complete and
// publishes its own flag.  Waits are bounded: past `spin` polls (the
// handle's RS_OPT_SPIN_LIMIT) the counter's error word is set and the tile
// proceeds (no hang).

struct TileWalk {
    int item, tile, sys;
};

// Draw the next item for the workgroup; false when none is left.
__device__ inline bool next_item(SweepCtr *ctr, int total, int nsys, TileWalk &w) {
    __shared__ int s_item;
    if (threadIdx.x == 0)
        s_item = (int)__hip_atomic_fetch_add(&ctr->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    w.item = s_item;
    __syncthreads();
    if (w.item >= total) return false;
    w.tile = w.item / nsys;
    w.sys = w.item % nsys;
    return true;
}

__device__ inline void leave_sweep(SweepCtr *ctr, uint32_t epoch) {
    if (threadIdx.x == 0) {
        const uint32_t e = __hip_atomic_fetch_add(&ctr->exit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e == gridDim.x - 1) {
            __hip_atomic_store(&ctr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr->exit, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr->epoch, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__device__ inline void wait_tiles(const int32_t *__restrict__ dptr, const int32_t *__restrict__ dep,
                                  const int32_t *flags, int tile, uint32_t epoch, SweepCtr *ctr, int spin) {
    for (int i = dptr[tile] + threadIdx.x; i < dptr[tile + 1]; i += blockDim.x) {
        const int32_t *f = flags + dep[i];
        int spins = 0;
        while ((uint32_t)__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin) {
                __hip_atomic_fetch_or(&ctr->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
}

// Every wave waits for its own stores, then one thread marks the tile done.
__device__ inline void publish_tile(int32_t *flags, int tile, uint32_t epoch) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + tile, (int32_t)epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, bool FUSE_P>
__global__ void __launch_bounds__(kRowThreads) k_lsweep_tiles(DevSchedule d, const T *__restrict__ L,
                                                              size_t l_stride, const double *__restrict__ in,
                                                              T *__restrict__ y, size_t vstride,
                                                              const double *__restrict__ rv,
                                                              const double *__restrict__ vv, double *__restrict__ pv,
                                                              SysState *__restrict__ st, int32_t *__restrict__ flags,
                                                              SweepCtr *__restrict__ ctr, int nsys, int spin) {
    __shared__ Stage<T, kSweepCap> sv;
    const uint32_t epoch = __hip_atomic_load(&ctr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    const int total = d.nlt * nsys;
    TileWalk w;
    while (next_item(ctr, total, nsys, w)) {
        if (st && st[w.sys].phase != PH_RUN) continue;
        const int q0 = d.lt_start[w.tile], q1 = d.lt_start[w.tile + 1];
        const RowLane rl = row_lane<kWavesPerBlock>(0, q0, q1);
        const size_t vo = (size_t)w.sys * vstride;
        const T *Ls = L + (size_t)w.sys * l_stride;
        const int e0 = d.lptr[q0], e1 = d.lptr[q1];
        const int my0 = rl.act ? d.lptr[rl.q] : 0, my1 = rl.act ? d.lptr[rl.q + 1] : 0;
        int cnt = min(kSweepCap, e1 - e0), shift = 0;
        if (cnt > 0) shift = stage_copy<T, kSweepCap, kRowThreads>(Ls, d.lcol, e0, cnt, sv);
        const int i = rl.act ? d.lrows[rl.q] : 0;
        T acc = 0;
        if (rl.act) {
            const size_t k = vo + 3 * (size_t)i + rl.r;
            if (FUSE_P) {
                const double beta = st[w.sys].beta, omega = st[w.sys].omega;
                const double p = rv[k] + beta * (pv[k] - omega * vv[k]);
                pv[k] = p;
                acc = (T)p;
            } else {
                acc = (T)in[k];
            }
        }
        wait_tiles(d.lt_dptr, d.lt_dep, flags + (size_t)w.sys * d.nlt, w.tile, epoch, ctr, spin);
        __syncthreads();
        for (int base = e0; base < e1; base += kSweepCap) {
            if (base != e0) {
                cnt = min(kSweepCap, e1 - base);
                __syncthreads();
                shift = stage_copy<T, kSweepCap, kRowThreads>(Ls, d.lcol, base, cnt, sv);
                __syncthreads();
            }
            acc = walk_pass<true, true>((const T *)sv.v, sv.c, shift, base, max(my0, base), min(my1, base + cnt),
                                        rl.r, y + vo, acc);
        }
        if (rl.act) __hip_atomic_store(y + vo + 3 * (size_t)i + rl.r, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        publish_tile(flags + (size_t)w.sys * d.nlt, w.tile, epoch);
    }
    leave_sweep(ctr, epoch);
}

template <typename T>
__global__ void __launch_bounds__(kRowThreads) k_usweep_tiles(DevSchedule d, const T *__restrict__ U,
                                                              size_t u_stride, const T *__restrict__ Dinv,
                                                              size_t d_stride, const T *__restrict__ y,
                                                              double *__restrict__ z, size_t vstride,
                                                              SysState *__restrict__ st, int32_t *__restrict__ flags,
                                                              SweepCtr *__restrict__ ctr, int nsys, int spin) {
    __shared__ Stage<T, kSweepCap> sv;
    const uint32_t epoch = __hip_atomic_load(&ctr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    const int total = d.nut * nsys;
    TileWalk w;
    while (next_item(ctr, total, nsys, w)) {
        if (st && st[w.sys].phase != PH_RUN) continue;
        const int q0 = d.ut_start[w.tile], q1 = d.ut_start[w.tile + 1];
        const RowLane rl = row_lane<kWavesPerBlock>(0, q0, q1);
        const size_t vo = (size_t)w.sys * vstride;
        const T *Us = U + (size_t)w.sys * u_stride;
        const int e0 = d.uptr[q0], e1 = d.uptr[q1];
        const int my0 = rl.act ? d.uptr[rl.q] : 0, my1 = rl.act ? d.uptr[rl.q + 1] : 0;
        int cnt = min(kSweepCap, e1 - e0), shift = 0;
        if (cnt > 0) shift = stage_copy<T, kSweepCap, kRowThreads>(Us, d.ucol, e0, cnt, sv);
        const int i = rl.act ? d.urows[rl.q] : 0;
        T acc = rl.act ? y[vo + 3 * (size_t)i + rl.r] : (T)0;
        T dq[3] = {0, 0, 0};
        if (rl.act) {
            const T *dp = Dinv + (size_t)w.sys * d_stride + (size_t)rl.q * 9 + 3 * rl.r;
            dq[0] = dp[0]; dq[1] = dp[1]; dq[2] = dp[2];
        }
        wait_tiles(d.ut_dptr, d.ut_dep, flags + (size_t)w.sys * d.nut, w.tile, epoch, ctr, spin);
        __syncthreads();
        for (int base = e0; base < e1; base += kSweepCap) {
            if (base != e0) {
                cnt = min(kSweepCap, e1 - base);
                __syncthreads();
                shift = stage_copy<T, kSweepCap, kRowThreads>(Us, d.ucol, base, cnt, sv);
                __syncthreads();
            }
            acc = walk_pass<true, true>((const T *)sv.v, sv.c, shift, base, max(my0, base), min(my1, base + cnt),
                                        rl.r, z + vo, acc);
        }
        const T t0 = __shfl(acc, rl.base, 64), t1 = __shfl(acc, rl.base + 1, 64), t2 = __shfl(acc, rl.base + 2, 64);
        if (rl.act) {
            const T zr = dot3(dq[0], dq[1], dq[2], t0, t1, t2);
            __hip_atomic_store(z + vo + 3 * (size_t)i + rl.r, (double)zr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        publish_tile(flags + (size_t)w.sys * d.nut, w.tile, epoch);
    }
    leave_sweep(ctr, epoch);
}

// -------------------------------------------------------------------- SpMV

enum SpmvMode { SPMV_PLAIN = 0, SPMV_V = 1, SPMV_T = 2, SPMV_TRUE = 3, SPMV_RUN = 4 };

// y = A x over rows in storage order, with the epilogue of the mode:
//   SPMV_V:    v = A phat, reduce (rhat, v), alpha = rho / (rhat, v)
//   SPMV_T:    t = A shat, reduce (t, s) and (t, t), omega = (t, s) / (t, t)
//   SPMV_TRUE: reduce ||b - A x||^2 and ||b||^2, true relative residual
//   SPMV_RUN:  y only, for the systems still iterating (GMRES)
// ------------------------------------------------------------------ wells

// (C_p^T t2_w)_r summed over the perforations of output row i, in
// perforation order (Algorithm 5's second half for one row component).
__device__ inline double well_terms(const WellsDev &wl, int sys, int i, int r) {
    double s = 0.0;
    const double *Cs = wl.C + (size_t)sys * wl.np * 12;
    const double *Ts = wl.t2 + (size_t)sys * wl.nw * 4;
    for (int e = wl.row_ptr[i]; e < wl.row_ptr[i + 1]; ++e) {
        const int p = wl.row_perf[e];
        const double *c = Cs + (size_t)p * 12;
        const double *t = Ts + (size_t)wl.perf_well[p] * 4;
        s += c[r] * t[0] + c[3 + r] * t[1] + c[6 + r] * t[2] + c[9 + r] * t[3];
    }
    return s;
}

// t2_w = D_w^-1 (B_w x) for every well: one wave per well, lanes stride over
// its perforations, then a fixed-order wave sum (Algorithm 5's first half).
__global__ void __launch_bounds__(256) k_wells_t2(WellsDev wl, const double *__restrict__ x, size_t xstride) {
    const int sys = blockIdx.y;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= wl.nw) return;
    const double *xs = x + (size_t)sys * xstride;
    const double *Bs = wl.B + (size_t)sys * wl.np * 12;
    double t1[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = wl.well_ptr[w] + lane; p < wl.well_ptr[w + 1]; p += 64) {
        const double *b = Bs + (size_t)p * 12, *xc = xs + 3 * (size_t)wl.perf_x[p];
        const double x0 = xc[0], x1 = xc[1], x2 = xc[2];
        for (int i = 0; i < 4; ++i) t1[i] += b[3 * i] * x0 + b[3 * i + 1] * x1 + b[3 * i + 2] * x2;
    }
    for (int i = 0; i < 4; ++i) t1[i] = wave_sum(t1[i]);
    if (lane != 0) return;
    const double *d = wl.Dinv + ((size_t)sys * wl.nw + w) * 16;
    double *t2 = wl.t2 + ((size_t)sys * wl.nw + w) * 4;
    for (int i = 0; i < 4; ++i) t2[i] = d[4 * i] * t1[0] + d[4 * i + 1] * t1[1] + d[4 * i + 2] * t1[2] + d[4 * i + 3] * t1[3];
}

// The well terms of the rows the fused upper launch formed (rows below
// fuse_n0 that a perforation couples): y_i -= (C^T t2)_i once t2 of the
// whole x exists, and the changes of the launch's two dot-product sums over
// those rows, (w1, y_new - y_old) and (y_new, y_new) - (y_old, y_old), as one
// more group sum.  One workgroup per system.
__global__ void __launch_bounds__(256) k_wells_fix(WellsDev wl, double *__restrict__ y, const double *__restrict__ w1,
                                                   size_t vstride, double *__restrict__ part, size_t part_stride,
                                                   int at, const SysState *__restrict__ st) {
    __shared__ double lds[4 * 2];
    const int sys = blockIdx.y;
    if (st[sys].phase != PH_RUN) return;
    const size_t vo = (size_t)sys * vstride;
    double d[2] = {0.0, 0.0};
    for (int idx = threadIdx.x; idx < 3 * wl.nfix; idx += blockDim.x) {
        const int i = wl.fix_row[idx / 3], r = idx % 3;
        const size_t k = vo + 3 * (size_t)i + r;
        const double yo = y[k], yn = yo - well_terms(wl, sys, i, r);
        y[k] = yn;
        d[0] += w1[k] * (yn - yo);
        d[1] += yn * yn - yo * yo;
    }
    block_sum<2>(d, lds);
    if (threadIdx.x == 0) {
        double *pp = part + sys * part_stride + at;
        pp[0] = d[0];
        pp[1] = d[1];
    }
}

// ------------------------------------------------------------------- SpMV

template <int MODE, int W, int STAGE>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kRowWavesPerEU, 8))) k_spmv(int n, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col, const double *__restrict__ A,
                                                      size_t a_stride, const double *__restrict__ x,
                                                      double *__restrict__ y, size_t vstride,
                                                      const double *__restrict__ w1, const double *__restrict__ w2,
                                                      double *__restrict__ part, size_t part_stride,
                                                      uint32_t *__restrict__ tk, size_t tk_stride,
                                                      SysState *__restrict__ st, int split, WellsDev wl, int r0) {
    int sys, bx;
    xcd_map(sys, bx);
    // whether the system still iterates.  t = A shat often runs after a
    // half-step stop, so it tests first; v = A phat (which runs whenever its
    // iteration starts) tests once the row walk's loads are in flight, which
    // hides the latency of the test; a finished system's launch stores nothing
    if ((MODE == SPMV_T || MODE == SPMV_RUN) && st[sys].phase != PH_RUN) return;
    const bool run = MODE != SPMV_V || st[sys].phase == PH_RUN;
    // workgroup bx walks row tiles [bx * per, (bx + 1) * per); per = 1 with
    // one workgroup per tile
    // rows [r0, n): the fused upper launch formed rows [0, r0)
    constexpr int R = W * kRowsPerWave;
    const int ntiles = (n - r0 + R - 1) / R;
    const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t0 = bx * per, t1 = min(t0 + per, ntiles);
    const size_t vo = (size_t)sys * vstride;
    const double *As = A + (size_t)sys * a_stride;
    double v[2] = {0.0, 0.0};
    for (int t = t0; t < t1; ++t) {
        const RowLane rl = row_lane<W>(t, r0, n);
        const int qb0 = r0 + t * R, qb1 = min(qb0 + R, n);
        const size_t k = vo + 3 * (size_t)rl.q + rl.r;
        // the dot-product operand is loaded before the row walk, so its
        // latency overlaps the walk's
        const double w = (MODE != SPMV_PLAIN && MODE != SPMV_RUN && rl.act) ? w1[k] : 0.0;
        const double acc = row_walk<W, STAGE, kSpmvCapPerWave, false>(ptr, col, As, qb0, qb1, rl, x + vo, 0.0);
        asm volatile("" ::"v"(acc));   // the walk completes before the phase test below
        if (!run) return;
        if (!rl.act) continue;
        const double acc_w = wl.nw > 0 ? acc - well_terms(wl, sys, rl.q, rl.r) : acc;
        if (MODE == SPMV_PLAIN || MODE == SPMV_RUN) {
            y[k] = acc_w;
        } else if (MODE == SPMV_V || MODE == SPMV_T) {
            y[k] = acc_w;
            v[0] += w * acc_w;
            v[1] += acc_w * acc_w;
        } else {  // SPMV_TRUE: w1 = b
            const double res = w - acc_w;
            v[0] += res * res;
            v[1] += w * w;
        }
    }
    if (MODE == SPMV_PLAIN || MODE == SPMV_RUN) return;
    if (split) {
        // one partial per wave (no workgroup barrier); k_spmv_total adds
        // them after the kernel boundary
        const double a = wave_sum(v[0]), b = wave_sum(v[1]);
        if ((threadIdx.x & 63) == 0) {
            double *pp = part + sys * part_stride + ((size_t)bx * W + (threadIdx.x >> 6)) * 2;
            pp[0] = a;
            pp[1] = b;
        }
        return;
    }
    if (MODE == SPMV_V || MODE == SPMV_T) {
        // group sums of (rhat, v) or of (t, s) and (t, t); the next kernel
        // adds the group sums (kernel boundary: no serial tail here)
        group_reduce<2>(v, part + sys * part_stride, tk + sys * tk_stride, gridDim.x, bx);
    } else if (grid_reduce<2>(v, part + sys * part_stride, tk + sys * tk_stride, gridDim.x, bx) &&
               threadIdx.x == 0) {
        st[sys].true_res = v[1] > 0.0 ? sqrt(v[0]) / sqrt(v[1]) : 0.0;
    }
}

// ------------------------------------- upper sweep fused with the product

// LDS capacity (blocks of A') per wave of the fused upper launch.
constexpr int kFuseCapPerWave = 160;

// The rows 0 .. n0 of the new order hold no lower blocks (Schedule::fuse_n0):
// nothing updates them, so their U row is their row of A' past the
// diagonal, and all of them sit in one upper level.  One launch over those
// rows walks each A' row once and gives both
//   the upper sweep  z_i = inv(U_ii) (y_i - sum_j U_ij z_j), in the factor
//                    type T with the operations and order of k_usweep
//                    ((T) of an FP64 block of A' is the stored factor), and
//   the next product out_i = sum_j A'_ij z_j + A'_ii z_i in FP64: the
//                    off-diagonal terms summed in the walk, ascending, the
//                    diagonal's term added once z_i is known (k_spmv adds
//                    the diagonal first: the same terms, another rounding),
// plus that product's dot-product partials (MODE SPMV_V: (rhat, v) with w1 =
// rhat; SPMV_T: (s, t) and (t, t) with w1 = s), reduced to group sums as
// k_spmv does.  MODE SPMV_PLAIN gives the sweep alone (a preconditioner
// application outside BiCGStab's fused iteration; with FP64 factors the
// factorisation then stores no U for these rows).  Every upper column of such a row is a row with lower blocks,
// whose z the earlier upper levels or the lower launches have finished.
// defer: the phase test waits until the walk's loads are in flight (the
// iteration's first application).
// TY: the type y is read in (T, or FP64 when y is the application's input
// itself, rounded to T as the stored y would be).
template <typename T, int MODE, int W, bool NTL, typename TY>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kRowWavesPerEU, 8)))
k_usweep_spmv(DevSchedule d, const double *__restrict__ Ap, size_t a_stride, const T *__restrict__ Dinv,
              size_t d_stride, const TY *__restrict__ y, double *__restrict__ z, double *__restrict__ out,
              const double *__restrict__ w1, size_t vstride, SysState *__restrict__ st, double *__restrict__ part,
              size_t part_stride, uint32_t *__restrict__ tk, size_t tk_stride, int defer,
              const double *__restrict__ rr, double *__restrict__ P) {
    constexpr int CAP = kFuseCapPerWave * W, NT = 64 * W;
    // lower parts (FP64 factors, v = A phat): inv(U_kk) r_k and inv(U_kk)
    // v_k of these rows, six values per row in P (see k_spmv_lp)
    constexpr bool LPC = sizeof(T) == sizeof(double) && MODE == SPMV_V;
    const bool lp = LPC && P != nullptr;
    __shared__ Stage<double, CAP, NT> sv;
    int sys, bx;
    xcd_map(sys, bx);
    // st may be NULL (an application outside a solve: no phase test)
    if (!defer && st && st[sys].phase != PH_RUN) return;
    const int n0 = d.fuse_n0;
    const RowLane rl = row_lane<W>(bx, 0, n0);
    const int qb0 = bx * W * kRowsPerWave, qb1 = min(qb0 + W * kRowsPerWave, n0);
    const size_t vo = (size_t)sys * vstride;
    const size_t k = vo + 3 * (size_t)rl.q + rl.r;
    const double *As = Ap + (size_t)sys * a_stride;
    constexpr bool PRODUCT = MODE != SPMV_PLAIN;
    T acc = 0;
    T dq[3] = {0, 0, 0};
    double w = 0.0, rk = 0.0;
    if (rl.act) {
        acc = (T)y[k];
        const T *dp = Dinv + (size_t)sys * d_stride + (size_t)(d.fuse_q0 + rl.q) * 9 + 3 * rl.r;
        dq[0] = dp[0]; dq[1] = dp[1]; dq[2] = dp[2];
        if (PRODUCT) w = w1[k];
        if (lp) rk = rr[k];
    }
    const int e0 = d.prow[qb0], e1 = d.prow[qb1];
    // the lane's row: diagonal at my0, upper blocks [my0 + 1, my1)
    const int my0 = rl.act ? d.prow[rl.q] : 0, my1 = rl.act ? d.prow[rl.q + 1] : 0;
    const double *x = z + vo;
    double dg[3] = {0.0, 0.0, 0.0};
    double av = 0.0;
    for (int base = e0; base < e1; base += CAP) {
        const int cnt = min(CAP, e1 - base);
        __syncthreads();
        const int shift = stage_copy<double, CAP, NT, NTL>(As, d.pcol, base, cnt, sv);
        __syncthreads();
        const double *vals = (const double *)sv.v + shift;
        if (PRODUCT && rl.act && my0 >= base && my0 < base + cnt) {
            const double *b = vals + (my0 - base) * 9 + 3 * rl.r;
            dg[0] = b[0]; dg[1] = b[1]; dg[2] = b[2];
        }
        const int lo = max(my0 + 1, base), hi = min(my1, base + cnt);
        for (int e = lo; e < hi; e += 8) {
            double xv[8][3];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = sv.c[min(e + u, hi - 1) - base];
#pragma unroll
                for (int c = 0; c < 3; ++c) xv[u][c] = x[3 * j + c];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < hi) {
                    const double *b = vals + (e + u - base) * 9 + 3 * rl.r;
                    acc -= dot3((T)b[0], (T)b[1], (T)b[2], (T)xv[u][0], (T)xv[u][1], (T)xv[u][2]);
                    if (PRODUCT) av += dot3(b[0], b[1], b[2], xv[u][0], xv[u][1], xv[u][2]);
                }
        }
    }
    asm volatile("" ::"v"(acc), "v"(av));
    if (st && st[sys].phase != PH_RUN) return;
    const T t0 = __shfl(acc, rl.base, 64), t1 = __shfl(acc, rl.base + 1, 64), t2 = __shfl(acc, rl.base + 2, 64);
    const double zr = (double)dot3(dq[0], dq[1], dq[2], t0, t1, t2);
    if (!PRODUCT) {
        if (rl.act) z[k] = zr;
        return;
    }
    const double z0 = __shfl(zr, rl.base, 64), z1 = __shfl(zr, rl.base + 1, 64), z2 = __shfl(zr, rl.base + 2, 64);
    av += dot3(dg[0], dg[1], dg[2], z0, z1, z2);
    if constexpr (LPC) {
        if (lp) {
            const double r0v = __shfl(rk, rl.base, 64), r1v = __shfl(rk, rl.base + 1, 64),
                         r2v = __shfl(rk, rl.base + 2, 64);
            const double v0 = __shfl(av, rl.base, 64), v1 = __shfl(av, rl.base + 1, 64),
                         v2 = __shfl(av, rl.base + 2, 64);
            if (rl.act) {
                double *pp = P + 2 * vo + 6 * (size_t)rl.q + rl.r;
                pp[0] = dot3((double)dq[0], (double)dq[1], (double)dq[2], r0v, r1v, r2v);
                pp[3] = dot3((double)dq[0], (double)dq[1], (double)dq[2], v0, v1, v2);
            }
        }
    }
    double v[2] = {0.0, 0.0};
    if (rl.act) {
        z[k] = zr;
        out[k] = av;
        v[0] = w * av;
        v[1] = av * av;
    }
    group_reduce<2>(v, part + sys * part_stride, tk + sys * tk_stride, gridDim.x, bx);
}

// v = A phat on the rows [r0, n) (the rows with lower blocks of a two-level
// pattern, r0 = fuse_n0: every other row's y is its input, see
// Schedule::y_in), with k_spmv's arithmetic, order, partition and group
// sums, and in the same walk the lower parts of the iteration's second
// preconditioner application.  Row i's lower blocks are A'_ik, k < r0, and
// L_ik = A'_ik inv(U_kk) (row k has no lower blocks, so ILU0 leaves A'_ik
// alone and U_kk = A'_kk): with P_k = (inv(U_kk) r_k, inv(U_kk) v_k) (six
// values per row, from the fused upper launch), the sums a_i = sum_k A'_ik
// inv(U_kk) r_k and b_i = sum_k A'_ik inv(U_kk) v_k give sum_k L_ik s_k =
// a_i - alpha b_i for s = r - alpha v once alpha is known (k_lower_parts).
// (a_i, b_i) go to P at row i.  The FP64 block is read once for all three
// sums.  P holds 6 values per row (2 vstride per system).
template <int W, bool NTL>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kRowWavesPerEU, 8)))
k_spmv_lp(int n, int r0, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
          const double *__restrict__ A, size_t a_stride, const double *__restrict__ x, double *__restrict__ y,
          size_t vstride, const double *__restrict__ w1, double *P, double *__restrict__ part,
          size_t part_stride, uint32_t *__restrict__ tk, size_t tk_stride, SysState *__restrict__ st) {
    constexpr int CAP = kSpmvCapPerWave * W, NT = 64 * W;
    __shared__ Stage<double, CAP, NT> sv;
    int sys, bx;
    xcd_map(sys, bx);
    const bool run = st[sys].phase == PH_RUN;   // tested once the walk's loads are in flight
    constexpr int R = W * kRowsPerWave;
    const RowLane rl = row_lane<W>(bx, r0, n);
    const int qb0 = r0 + bx * R, qb1 = min(qb0 + R, n);
    const size_t vo = (size_t)sys * vstride;
    const size_t k = vo + 3 * (size_t)rl.q + rl.r;
    const double *As = A + (size_t)sys * a_stride;
    const double w = rl.act ? w1[k] : 0.0;
    const int e0 = ptr[qb0], e1 = ptr[qb1];
    const int my0 = rl.act ? ptr[rl.q] : 0, my1 = rl.act ? ptr[rl.q + 1] : 0;
    double acc = 0.0, pa = 0.0, pb = 0.0;
    for (int base = e0; base < e1; base += CAP) {
        const int cnt = min(CAP, e1 - base);
        __syncthreads();
        const int shift = stage_copy<double, CAP, NT, NTL>(As, col, base, cnt, sv);
        __syncthreads();
        const double *vals = (const double *)sv.v + shift;
        const int lo = max(my0, base), hi = min(my1, base + cnt);
        for (int e = lo; e < hi; e += 4) {
            double xv[4][3], av[4][3], bv[4][3];
            bool low[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = sv.c[min(e + u, hi - 1) - base];
                low[u] = j < r0;
                const int jl = low[u] ? j : 0;
                const double *pj = P + 2 * vo + 6 * (size_t)jl;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xv[u][c] = x[vo + 3 * (size_t)j + c];
                    av[u][c] = pj[c];
                    bv[u][c] = pj[3 + c];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e + u < hi) {
                    const double *b = vals + (e + u - base) * 9 + 3 * rl.r;
                    acc += dot3(b[0], b[1], b[2], xv[u][0], xv[u][1], xv[u][2]);
                    if (low[u]) {
                        pa += dot3(b[0], b[1], b[2], av[u][0], av[u][1], av[u][2]);
                        pb += dot3(b[0], b[1], b[2], bv[u][0], bv[u][1], bv[u][2]);
                    }
                }
        }
    }
    asm volatile("" ::"v"(acc), "v"(pa), "v"(pb));
    if (!run) return;
    double v[2] = {0.0, 0.0};
    if (rl.act) {
        y[k] = acc;
        double *pp = P + 2 * vo + 6 * (size_t)rl.q + rl.r;
        pp[0] = pa;
        pp[3] = pb;
        v[0] = w * acc;
        v[1] = acc * acc;
    }
    group_reduce<2>(v, part + sys * part_stride, tk + sys * tk_stride, gridDim.x, bx);
}

// The second preconditioner application's lower launch for the rows
// [n0, n) of a two-level pattern (Schedule::y_in: row i at U-schedule
// position i - n0; all rows finish here): z_i = inv(U_ii) (s_i - (a_i -
// alpha b_i)) with (a_i, b_i) from k_spmv_lp in P and alpha of the half step.
__global__ void __launch_bounds__(kRowThreads) k_lower_parts(int n0, int n, const double *__restrict__ Dinv,
                                                             size_t d_stride, const double *__restrict__ s,
                                                             const double *__restrict__ P, double *__restrict__ z,
                                                             size_t vstride, SysState *__restrict__ st) {
    int sys, bx;
    xcd_map(sys, bx);
    const RowLane rl = row_lane<kWavesPerBlock>(bx, n0, n);
    const size_t vo = (size_t)sys * vstride;
    const size_t k = vo + 3 * (size_t)rl.q + rl.r;
    double sv = 0.0, pa = 0.0, pb = 0.0, dq[3] = {0.0, 0.0, 0.0};
    if (rl.act) {
        sv = s[k];
        const double *pp = P + 2 * vo + 6 * (size_t)rl.q + rl.r;
        pa = pp[0];
        pb = pp[3];
        const double *dp = Dinv + (size_t)sys * d_stride + (size_t)(rl.q - n0) * 9 + 3 * rl.r;
        dq[0] = dp[0]; dq[1] = dp[1]; dq[2] = dp[2];
    }
    if (st[sys].phase != PH_RUN) return;
    const double alpha = st[sys].alpha;
    const double t = sv - (pa - alpha * pb);
    const double t0 = __shfl(t, rl.base, 64), t1 = __shfl(t, rl.base + 1, 64), t2 = __shfl(t, rl.base + 2, 64);
    if (rl.act) z[k] = dot3(dq[0], dq[1], dq[2], t0, t1, t2);
}

// ---------------------------------------------------------------- vectors

// Sum the NV-wide partials of nblk workgroups of the previous kernel, the
// same way in every workgroup (thread-strided sums, then the block tree), and
// hand the totals to every thread.
template <int NV>
__device__ inline void sum_partials(const double *__restrict__ p, int nblk, double (&out)[NV]) {
    __shared__ double lds[16 * NV];
    __shared__ double tot[NV];
    double acc[NV];
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    constexpr int U = 4;
    for (int b0 = 0; b0 < nblk; b0 += U * (int)blockDim.x) {
        double t[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = min(b0 + u * (int)blockDim.x + (int)threadIdx.x, nblk - 1);
            for (int k = 0; k < NV; ++k) t[u][k] = p[(size_t)b * NV + k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b0 + u * (int)blockDim.x + (int)threadIdx.x < nblk)
                for (int k = 0; k < NV; ++k) acc[k] += t[u][k];
    }
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) tot[k] = acc[k];
    __syncthreads();
    for (int k = 0; k < NV; ++k) out[k] = tot[k];
}

// The SpMV's dot products in split mode: one workgroup per system adds the
// nblk wave partials (fixed order) and stores the totals right after them,
// where the consumers read them, or the true residual.
template <int MODE>
__global__ void __launch_bounds__(kTotalThreads) k_spmv_total(double *__restrict__ part, size_t part_stride, int nblk,
                                                              SysState *__restrict__ st) {
    const int sys = blockIdx.y;
    if (MODE != SPMV_TRUE && st[sys].phase != PH_RUN) return;
    double *p = part + sys * part_stride;
    double tot[2];
    sum_partials<2>(p, nblk, tot);
    if (threadIdx.x != 0) return;
    if (MODE == SPMV_TRUE) {
        st[sys].true_res = tot[1] > 0.0 ? sqrt(tot[0]) / sqrt(tot[1]) : 0.0;
    } else {
        p[2 * (size_t)nblk] = tot[0];
        p[2 * (size_t)nblk + 1] = tot[1];
    }
}

// Vector kernels: each thread handles kVecItems entries of a 1024-entry
// tile, all loads of a tile issued before the arithmetic; tiles are
// grid-strided.  Vectors are padded to whole tiles with zeros, so there are
// no bounds checks (the padding contributes zeros to every reduction).

// r = rhat = P b, x = p = v = 0 (padding included), ||b||; initial scalars.
__global__ void __launch_bounds__(kVecThreads) k_setup(int n, const int32_t *__restrict__ perm,
                                                       const double *__restrict__ b, Krylov k,
                                                       const int32_t *__restrict__ bad, double reduction,
                                                       int max_iter) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    const size_t vo = (size_t)sys * k.vstride, bo = (size_t)sys * 3 * n, m = 3 * (size_t)n;
    const size_t tiles = k.vstride / kVecTile;
    double v[1] = {0.0};
    for (size_t t = bx; t < tiles; t += gridDim.x) {
        double val[kVecItems];
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const size_t e = t * kVecTile + u * kVecThreads + threadIdx.x;
            val[u] = e < m ? b[bo + 3 * (size_t)perm[e / 3] + e % 3] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const size_t e = vo + t * kVecTile + u * kVecThreads + threadIdx.x;
            k.r[e] = val[u]; k.rhat[e] = val[u];
            k.x[e] = 0.0; k.p[e] = 0.0; k.v[e] = 0.0;
            v[0] += val[u] * val[u];
        }
    }
    if (grid_reduce<1>(v, k.part + sys * k.part_stride, k.tickets + sys * k.ticket_stride, gridDim.x, bx) && threadIdx.x == 0) {
        SysState &S = k.st[sys];
        const double r0 = sqrt(v[0]);
        S.r0norm = r0; S.tol = reduction * r0; S.last_norm = r0;
        S.rho = v[0]; S.rho_old = 1.0; S.alpha = 1.0; S.omega = 1.0;
        S.beta = (S.rho / S.rho_old) * (S.alpha / S.omega);
        S.half_steps = 0; S.iter = 1; S.max_iter = max_iter; S.true_res = 0.0;
        if (bad && bad[sys] < n) { S.status = RS_ZERO_PIVOT; S.phase = PH_DONE; }
        else if (!finite(r0)) { S.status = RS_NON_FINITE; S.phase = PH_DONE; }
        else if (r0 == 0.0) { S.status = RS_OK; S.phase = PH_DONE; }
        else if (max_iter <= 0) { S.status = RS_NOT_CONVERGED; S.phase = PH_DONE; }
        else { S.status = RS_NOT_CONVERGED; S.phase = PH_RUN; }
    }
}

// p = r + beta (p - omega v) on the first m entries of every system's
// vectors: the rows that hold no lower blocks (the first m / 3 rows of the
// new order), whose y is p itself, so the sweeps that follow read it from
// p.  The same arithmetic as the p update of a fused lower sweep.  It opens
// an iteration (queued whenever the iteration is): the phase test waits
// until the tile's loads are in flight.  Loads past m are clamped to the
// last entry; stores stop at m (the other rows' p is the next launch's).
__global__ void __launch_bounds__(kVecThreads) k_p_update(Krylov k, int m) {
    const int sys = blockIdx.y;
    const size_t vo = (size_t)sys * k.vstride;
    const int tiles = (m + kVecTile - 1) / kVecTile;
    const SysState &S = k.st[sys];
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        double r[kVecItems], p[kVecItems], v[kVecItems];
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const size_t e = vo + min(t * kVecTile + u * kVecThreads + (int)threadIdx.x, m - 1);
            r[u] = k.r[e]; p[u] = k.p[e]; v[u] = k.v[e];
        }
        if (S.phase != PH_RUN) return;
        const double beta = S.beta, omega = S.omega;
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const int e = t * kVecTile + u * kVecThreads + (int)threadIdx.x;
            if (e < m) k.p[vo + e] = r[u] + beta * (p[u] - omega * v[u]);
        }
    }
}

// alpha = rho / (rhat, v) from the partials of v = A phat; s = r - alpha v,
// ||s||; half-step test.
__global__ void __launch_bounds__(kVecThreads) k_s_update(Krylov k, int sums_at, int sums, int fsums_at, int fsums) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    const size_t vo = (size_t)sys * k.vstride, tiles = k.vstride / kVecTile;
    // the first tile's vectors are requested before the state and the
    // partial sums, so those round trips overlap
    double r0[kVecItems], w0[kVecItems];
    if ((size_t)bx < tiles) {
        const size_t e0 = vo + (size_t)bx * kVecTile + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) { r0[u] = k.r[e0 + u * kVecThreads]; w0[u] = k.v[e0 + u * kVecThreads]; }
    }
    SysState &S = k.st[sys];
    if (S.phase != PH_RUN) return;
    double rvv[2];
    sum_partials<2>(k.spart + sys * k.spart_stride + sums_at, sums, rvv);
    if (fsums > 0) {
        // rows [0, fuse_n0) of v came from the fused upper launch
        double f[2];
        sum_partials<2>(k.fpart + sys * k.fpart_stride + fsums_at, fsums, f);
        rvv[0] += f[0];
    }
    const double rv = rvv[0];
    if (!finite(rv) || rv == 0.0) {
        if (bx == 0 && threadIdx.x == 0) {
            S.status = finite(rv) ? RS_BREAKDOWN : RS_NON_FINITE;
            S.phase = PH_DONE;
        }
        return;
    }
    const double alpha = S.rho / rv;
    if (bx == 0 && threadIdx.x == 0) S.alpha = alpha;
    double v[1] = {0.0};
    for (size_t t = bx; t < tiles; t += gridDim.x) {
        const size_t e0 = vo + t * kVecTile + threadIdx.x;
        double r[kVecItems], w[kVecItems];
        if (t == (size_t)bx) {
#pragma unroll
            for (int u = 0; u < kVecItems; ++u) { r[u] = r0[u]; w[u] = w0[u]; }
        } else {
#pragma unroll
            for (int u = 0; u < kVecItems; ++u) { r[u] = k.r[e0 + u * kVecThreads]; w[u] = k.v[e0 + u * kVecThreads]; }
        }
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const double sv = r[u] - alpha * w[u];
            k.s[e0 + u * kVecThreads] = sv;
            v[0] += sv * sv;
        }
    }
    if (grid_reduce<1>(v, k.part + sys * k.part_stride, k.tickets + sys * k.ticket_stride, gridDim.x, bx) && threadIdx.x == 0) {
        const double sn = sqrt(v[0]);
        S.half_steps = 2 * S.iter - 1;
        S.last_norm = sn;
        if (!finite(sn)) { S.status = RS_NON_FINITE; S.phase = PH_DONE; }
        else if (sn <= S.tol) { S.status = RS_OK; S.phase = PH_HALF; }
    }
}

// Full step: x += alpha phat + omega shat, r = s - omega t, ||r||, (rhat, r),
// full-step test, next rho and beta.  After a half-step stop (or an omega
// breakdown) only x += alpha phat.
__global__ void __launch_bounds__(kVecThreads) k_xr_update(Krylov k, int sums_at, int sums, int fsums_at, int fsums) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    const size_t vo = (size_t)sys * k.vstride, tiles = k.vstride / kVecTile;
    // the first tile's vectors are requested before the state and the
    // partial sums, so those round trips overlap
    double x0[kVecItems], ph0[kVecItems], sh0[kVecItems], s0[kVecItems], t0[kVecItems], rh0[kVecItems];
    if ((size_t)bx < tiles) {
        const size_t e0 = vo + (size_t)bx * kVecTile + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kVecItems; ++u) {
            const size_t e = e0 + u * kVecThreads;
            x0[u] = k.x[e]; ph0[u] = k.phat[e]; sh0[u] = k.shat[e];
            s0[u] = k.s[e]; t0[u] = k.t[e]; rh0[u] = k.rhat[e];
        }
    }
    SysState &S = k.st[sys];
    int phase = S.phase;
    if (phase == PH_DONE) return;
    const double alpha = S.alpha;
    double omega = S.omega;
    bool omega_zero = false;
    if (phase == PH_RUN) {
        // omega = (t, s) / (t, t) from the partials of t = A shat
        double tv[2];
        sum_partials<2>(k.spart + sys * k.spart_stride + sums_at, sums, tv);
        if (fsums > 0) {
            // rows [0, fuse_n0) of t came from the fused upper launch
            double f[2];
            sum_partials<2>(k.fpart + sys * k.fpart_stride + fsums_at, fsums, f);
            tv[0] += f[0];
            tv[1] += f[1];
        }
        const double ts = tv[0], tt = tv[1];
        if (!finite(ts) || !finite(tt) || tt == 0.0) {
            if (bx == 0 && threadIdx.x == 0) {
                S.status = (finite(ts) && finite(tt)) ? RS_BREAKDOWN : RS_NON_FINITE;
                S.phase = PH_DONE;
            }
            return;
        }
        omega = ts / tt;
        if (omega == 0.0) {
            // breakdown after the half step: keep x + alpha phat
            phase = PH_HALF;
            omega_zero = true;
        }
        if (bx == 0 && threadIdx.x == 0) S.omega = omega;
    }
    double v[2] = {0.0, 0.0};
    for (size_t t = bx; t < tiles; t += gridDim.x) {
        const size_t e0 = vo + t * kVecTile + threadIdx.x;
        const bool first = t == (size_t)bx;
        if (phase == PH_HALF) {
            double xv[kVecItems], ph[kVecItems];
#pragma unroll
            for (int u = 0; u < kVecItems; ++u) {
                xv[u] = first ? x0[u] : k.x[e0 + u * kVecThreads];
                ph[u] = first ? ph0[u] : k.phat[e0 + u * kVecThreads];
            }
#pragma unroll
            for (int u = 0; u < kVecItems; ++u) k.x[e0 + u * kVecThreads] = xv[u] + alpha * ph[u];
        } else {
            double xv[kVecItems], ph[kVecItems], sh[kVecItems], sv[kVecItems], tv[kVecItems], rh[kVecItems];
            if (first) {
#pragma unroll
                for (int u = 0; u < kVecItems; ++u) {
                    xv[u] = x0[u]; ph[u] = ph0[u]; sh[u] = sh0[u]; sv[u] = s0[u]; tv[u] = t0[u]; rh[u] = rh0[u];
                }
            } else {
#pragma unroll
                for (int u = 0; u < kVecItems; ++u) {
                    const size_t e = e0 + u * kVecThreads;
                    xv[u] = k.x[e]; ph[u] = k.phat[e]; sh[u] = k.shat[e];
                    sv[u] = k.s[e]; tv[u] = k.t[e]; rh[u] = k.rhat[e];
                }
            }
#pragma unroll
            for (int u = 0; u < kVecItems; ++u) {
                const size_t e = e0 + u * kVecThreads;
                k.x[e] = xv[u] + (alpha * ph[u] + omega * sh[u]);
                const double r = sv[u] - omega * tv[u];
                k.r[e] = r;
                v[0] += r * r;
                v[1] += rh[u] * r;
            }
        }
    }
    if (grid_reduce<2>(v, k.part + sys * k.part_stride, k.tickets + sys * k.ticket_stride, gridDim.x, bx) && threadIdx.x == 0) {
        // every workgroup computed the same omega: use this one's copy
        if (phase == PH_HALF) {
            if (omega_zero) S.status = RS_BREAKDOWN;
            S.phase = PH_DONE;
            return;
        }
        const double rn = sqrt(v[0]);
        S.half_steps = 2 * S.iter;
        S.last_norm = rn;
        if (!finite(rn)) { S.status = RS_NON_FINITE; S.phase = PH_DONE; }
        else if (rn <= S.tol) { S.status = RS_OK; S.phase = PH_DONE; }
        else if (S.iter >= S.max_iter) { S.status = RS_NOT_CONVERGED; S.phase = PH_DONE; }
        else {
            S.rho_old = S.rho;
            S.rho = v[1];
            if (S.rho == 0.0) { S.status = RS_BREAKDOWN; S.phase = PH_DONE; }
            else {
                S.beta = (S.rho / S.rho_old) * (alpha / omega);
                S.iter += 1;
            }
        }
    }
}

// ------------------------------------------------------------------ GMRES
//
// Right-preconditioned restarted GMRES (the simulator's alternative Krylov
// solver, Section "OPM Flow"), x0 = 0.  All vectors in the new order, padded
// to whole tiles with zeros.  The Arnoldi vector w is orthogonalised against
// the cycle's basis by classical Gram-Schmidt applied twice: each pass takes
// all its coefficients from one w (one reduction of jv dot products), so a
// step needs three grid reductions however long the basis is.  The kernels
// below stream w and the basis columns once per pass; every thread owns one
// entry per 256-entry tile and tiles are grid-strided, so each thread's
// partial sums follow a fixed order that depends only on the system size.
// The scalar work of a step (Givens rotations, tests) runs in the workgroup
// that completes the last reduction, after every other workgroup of its
// launch has passed its phase test.

constexpr int kGmThreads = 256;

__device__ inline void gm_cycle_start(GmState &G, double beta) {
    G.beta = beta;
    G.g[0] = beta;
    for (int i = 1; i <= kGmMax; ++i) G.g[i] = 0.0;
    G.jend = 0;
}

__global__ void k_gm_init(GmWork g, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys || g.st[sys].phase != PH_RUN) return;
    gm_cycle_start(g.gm[sys], g.st[sys].r0norm);
}

__global__ void __launch_bounds__(kGmThreads) k_gm_normalise(GmWork g, const double *__restrict__ src, int col,
                                                             int from_w) {
    const int sys = blockIdx.y;
    if (g.st[sys].phase != PH_RUN) return;
    const double sc = from_w ? g.gm[sys].hn : g.gm[sys].beta;
    const size_t vo = (size_t)sys * g.vstride;
    double *dst = g.V + (size_t)col * g.colstride + vo;
    for (size_t e = (size_t)blockIdx.x * kGmThreads + threadIdx.x; e < g.vstride; e += (size_t)gridDim.x * kGmThreads)
        dst[e] = src[vo + e] / sc;
}

// h_i = (w, v_i) for i < jv (NV >= jv).  Each thread loads IT entries of w
// and of every column before it multiplies, so IT * (NV + 1) loads are in
// flight per thread.
template <int NV, int IT>
__global__ void __launch_bounds__(kGmThreads) k_gm_dots(GmWork g, int jv, const double *__restrict__ w) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    if (g.st[sys].phase != PH_RUN) return;
    const size_t vo = (size_t)sys * g.vstride, chunk = (size_t)kGmThreads * IT;
    const double *V = g.V + vo;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (size_t e0 = (size_t)bx * chunk + threadIdx.x; e0 < g.vstride; e0 += (size_t)gridDim.x * chunk) {
        double v[IT][NV], we[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const size_t e = e0 + (size_t)u * kGmThreads;
            we[u] = w[vo + e];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[u][i] = i < jv ? V[(size_t)i * g.colstride + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < IT; ++u)
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] = __builtin_fma(we[u], v[u][i], acc[i]);
    }
    if (grid_reduce<NV>(acc, g.part + sys * g.pstride, g.tickets + sys * g.tkstride, gridDim.x, bx) &&
        threadIdx.x == 0) {
        GmState &G = g.gm[sys];
        for (int i = 0; i < jv; ++i) {
            G.h[i] = acc[i];
            G.H[i][jv - 1] = acc[i];
        }
    }
}

// The Givens step of Arnoldi column j once h_{j+1,j} = sqrt(nrm2) is known:
// earlier rotations applied to the column, a new rotation that zeroes
// h_{j+1,j}, the rotated right-hand side, and the tests on its last entry
// (the residual norm of the cycle's current iterate).
__device__ inline void gm_givens(GmState &G, SysState &S, int j, double nrm2) {
    const double hn = sqrt(nrm2);
    G.H[j + 1][j] = hn;
    for (int k = 0; k < j; ++k) {
        const double a = G.H[k][j], b = G.H[k + 1][j];
        G.H[k][j] = G.cs[k] * a + G.sn[k] * b;
        G.H[k + 1][j] = -G.sn[k] * a + G.cs[k] * b;
    }
    const double a = G.H[j][j], b = G.H[j + 1][j];
    const double d = sqrt(a * a + b * b);
    const double c = d > 0.0 ? a / d : 1.0, sn = d > 0.0 ? b / d : 0.0;
    G.cs[j] = c;
    G.sn[j] = sn;
    G.H[j][j] = d;
    G.H[j + 1][j] = 0.0;
    const double gj = G.g[j];
    G.g[j + 1] = -sn * gj;
    G.g[j] = c * gj;
    G.hn = hn;
    G.jend = j + 1;
    S.half_steps += 1;
    const double last = fabs(G.g[j + 1]);
    S.last_norm = last;
    if (!finite(last) || !finite(hn)) { S.status = RS_NON_FINITE; S.phase = PH_DONE; }
    else if (last <= S.tol) { S.status = RS_OK; S.phase = PH_HALF; }
    else if (S.half_steps >= S.max_iter) { S.status = RS_NOT_CONVERGED; S.phase = PH_HALF; }
    // h_{j+1,j} = 0 (the Krylov space is invariant) gives sn = 0 and a zero
    // estimate, so the first test has already ended the solve
}

// w -= sum_i h_i v_i (i ascending), then the next pass's coefficients
// (w, v_i) or, when LAST, ||w||^2 and the Givens step.  Loads as k_gm_dots.
template <int NV, bool LAST, int IT>
__global__ void __launch_bounds__(kGmThreads) k_gm_orth(GmWork g, int jv, double *__restrict__ w) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    if (g.st[sys].phase != PH_RUN) return;
    const size_t vo = (size_t)sys * g.vstride, chunk = (size_t)kGmThreads * IT;
    const double *V = g.V + vo;
    double h[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = i < jv ? g.gm[sys].h[i] : 0.0;
    constexpr int NA = LAST ? 1 : NV;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0;
    for (size_t e0 = (size_t)bx * chunk + threadIdx.x; e0 < g.vstride; e0 += (size_t)gridDim.x * chunk) {
        double v[IT][NV], a[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const size_t e = e0 + (size_t)u * kGmThreads;
            a[u] = w[vo + e];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[u][i] = i < jv ? V[(size_t)i * g.colstride + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
#pragma unroll
            for (int i = 0; i < NV; ++i) a[u] = __builtin_fma(-h[i], v[u][i], a[u]);
            w[vo + e0 + (size_t)u * kGmThreads] = a[u];
            if (LAST) {
                acc[0] = __builtin_fma(a[u], a[u], acc[0]);
            } else {
#pragma unroll
                for (int i = 0; i < NA; ++i) acc[i] = __builtin_fma(a[u], v[u][i], acc[i]);
            }
        }
    }
    if (grid_reduce<NA>(acc, g.part + sys * g.pstride, g.tickets + sys * g.tkstride, gridDim.x, bx) &&
        threadIdx.x == 0) {
        GmState &G = g.gm[sys];
        if (LAST) {
            gm_givens(G, g.st[sys], jv - 1, acc[0]);
        } else {
            for (int i = 0; i < jv; ++i) {
                G.h[i] = acc[i];
                G.H[i][jv - 1] += acc[i];
            }
        }
    }
}

// y = H^-1 g by back substitution (every workgroup the same way), u = V y.
__global__ void __launch_bounds__(kGmThreads) k_gm_combine(GmWork g, double *__restrict__ u) {
    const int sys = blockIdx.y;
    if (g.st[sys].phase == PH_DONE) return;
    __shared__ double y[kGmMax];
    __shared__ int s_jend;
    const GmState &G = g.gm[sys];
    if (threadIdx.x == 0) {
        const int jend = min(max(G.jend, 0), kGmMax);
        for (int i = jend - 1; i >= 0; --i) {
            double a = G.g[i];
            for (int k = i + 1; k < jend; ++k) a -= G.H[i][k] * y[k];
            y[i] = a / G.H[i][i];
        }
        s_jend = jend;
    }
    __syncthreads();
    const int jend = s_jend;
    const size_t vo = (size_t)sys * g.vstride;
    const double *V = g.V + vo;
    for (size_t e = (size_t)blockIdx.x * kGmThreads + threadIdx.x; e < g.vstride;
         e += (size_t)gridDim.x * kGmThreads) {
        double a = 0.0;
#pragma unroll 8
        for (int i = 0; i < jend; ++i) a = __builtin_fma(y[i], V[(size_t)i * g.colstride + e], a);
        u[vo + e] = a;
    }
}

__global__ void __launch_bounds__(kGmThreads) k_gm_xupdate(GmWork g, double *__restrict__ x,
                                                           const double *__restrict__ z) {
    const int sys = blockIdx.y;
    if (g.st[sys].phase == PH_DONE) return;
    const size_t vo = (size_t)sys * g.vstride;
    for (size_t e = (size_t)blockIdx.x * kGmThreads + threadIdx.x; e < g.vstride; e += (size_t)gridDim.x * kGmThreads)
        x[vo + e] += z[vo + e];
}

__global__ void k_gm_phase(GmWork g, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys) return;
    if (g.st[sys].phase == PH_HALF) g.st[sys].phase = PH_DONE;
}

__global__ void __launch_bounds__(kGmThreads) k_gm_restart(GmWork g, const double *__restrict__ rhs,
                                                           const double *__restrict__ w, double *__restrict__ r) {
    const int sys = blockIdx.y, bx = blockIdx.x;
    if (g.st[sys].phase != PH_RUN) return;
    const size_t vo = (size_t)sys * g.vstride;
    double acc[1] = {0.0};
    for (size_t e = (size_t)bx * kGmThreads + threadIdx.x; e < g.vstride; e += (size_t)gridDim.x * kGmThreads) {
        const double re = rhs[vo + e] - w[vo + e];
        r[vo + e] = re;
        acc[0] = __builtin_fma(re, re, acc[0]);
    }
    if (grid_reduce<1>(acc, g.part + sys * g.pstride, g.tickets + sys * g.tkstride, gridDim.x, bx) &&
        threadIdx.x == 0) {
        SysState &S = g.st[sys];
        const double beta = sqrt(acc[0]);
        S.last_norm = beta;
        if (!finite(beta)) { S.status = RS_NON_FINITE; S.phase = PH_DONE; }
        else if (beta <= S.tol) { S.status = RS_OK; S.phase = PH_DONE; }
        else gm_cycle_start(g.gm[sys], beta);
    }
}

// U[f] = A'[usrc[f]] (in the factor type T) for U positions [f0, f1) of
// every system: the U blocks of rows without lower blocks, equal to their
// blocks of A', for the consumers that read U (per-level sweeps of FP32
// factors outside the fused iteration, single-launch sweeps, the host copy
// of the factors) when the factorisation did not store them.
template <typename T>
__global__ void k_fill_u(const int32_t *__restrict__ usrc, const double *__restrict__ Ap, size_t a_stride,
                         T *__restrict__ U, size_t u_stride, int f0, int f1) {
    const int sys = blockIdx.y;
    const size_t total = (size_t)(f1 - f0) * 9;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t f = f0 + t / 9, e = t % 9;
        U[sys * u_stride + f * 9 + e] = (T)Ap[sys * a_stride + (size_t)usrc[f] * 9 + e];
    }
}

// p[0 .. count) = value.
__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t count, uint32_t value) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        p[e] = value;
}

// New-order side at stride vstride, caller side at stride 3n.
__global__ void k_permute_vec(const int32_t *__restrict__ perm, const double *__restrict__ in,
                              double *__restrict__ out, int n, size_t vstride, int scatter) {
    const int sys = blockIdx.y;
    const size_t vo = (size_t)sys * vstride, m = 3 * (size_t)n, co = (size_t)sys * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        const size_t o = co + 3 * (size_t)perm[e / 3] + e % 3;
        if (scatter) out[o] = in[vo + e];
        else out[vo + e] = in[o];
    }
}

}  // namespace

// Call f(waves, staging) with compile-time constants for a RowVariant
// (staging 0: direct loads, 1: LDS, 2: LDS with non-temporal loads).
template <typename F>
static void with_variant(int v, F &&f) {
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using Direct = std::integral_constant<int, 0>;
    using Lds = std::integral_constant<int, 1>;
    using LdsNt = std::integral_constant<int, 2>;
    switch (v) {
    case RV_W2_LDS: f(I2{}, Lds{}); break;
    case RV_W1_LDS: f(I1{}, Lds{}); break;
    case RV_W4_DIRECT: f(I4{}, Direct{}); break;
    case RV_W2_DIRECT: f(I2{}, Direct{}); break;
    case RV_W1_DIRECT: f(I1{}, Direct{}); break;
    case RV_W4_LDS_NT: f(I4{}, LdsNt{}); break;
    case RV_W2_LDS_NT: f(I2{}, LdsNt{}); break;
    case RV_W1_LDS_NT: f(I1{}, LdsNt{}); break;
    default: f(I4{}, Lds{}); break;
    }
}

int vec_blocks(int n) {
    long g = (long)(vec_stride(n) / kVecTile);
    if (g < 1) g = 1;
    if (g > kVecMaxBlocks) g = kVecMaxBlocks;
    return (int)g;
}

static int copy_blocks(size_t m) {
    size_t g = (m + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

// Launch with optional dispatch-recorded events (start and end of the
// kernel itself); arguments are converted to the kernel's parameter types.
template <typename... P, typename... A>
static void launch_ev(void (*kernel)(P...), dim3 g, dim3 b, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                      A... args) {
    if (ev0)
        hipExtLaunchKernelGGL(kernel, g, b, 0, s, ev0, ev1, 0, static_cast<P>(args)...);
    else
        hipLaunchKernelGGL(kernel, g, b, 0, s, static_cast<P>(args)...);
}

void launch_gather_pairs(const double *A, size_t a_stride, double *Ap, size_t ap_stride, const int32_t *dst,
                         const int32_t *src, int cnt, int nsys, hipStream_t s) {
    if (cnt <= 0 || nsys <= 0) return;
    k_gather_pairs<<<dim3(copy_blocks((size_t)cnt * 9), nsys), 256, 0, s>>>(A, a_stride, Ap, ap_stride, dst, src,
                                                                             cnt);
}

void launch_factor_level(const DevSchedule &d, const double *A, size_t a_stride, double *Ap, double *L, double *U,
                         double *Dinv, float *Lf, float *Uf, float *Df, int32_t *bad, int q0, int q1, bool staged,
                         bool skip_u0, bool last, bool narrow, int nsys, hipStream_t s) {
    if (q1 <= q0 || nsys <= 0) return;
    const dim3 g(row_blocks(q1 - q0), nsys);
    auto go = [&](auto F32, auto STG, auto FM) {
        k_factor_level<decltype(F32)::value, decltype(STG)::value, decltype(FM)::value><<<g, kRowThreads, 0, s>>>(
            d, A, a_stride, Ap, L, U, Dinv, Lf, Uf, Df, bad, q0, q1, skip_u0 ? 1 : 0, last ? 1 : 0);
    };
    auto width = [&](auto F32, auto STG) {
        if (narrow) go(F32, STG, std::integral_constant<int, kFactorNarrow>{});
        else go(F32, STG, std::integral_constant<int, kFactorWide>{});
    };
    using T = std::true_type;
    using F = std::false_type;
    if (Lf) {
        if (staged) width(T{}, T{}); else width(T{}, F{});
    } else {
        if (staged) width(F{}, T{}); else width(F{}, F{});
    }
}

void launch_factor_first(const DevSchedule &d, const double *A, size_t a_stride, double *Ap, double *Dinv,
                         float *Df, int32_t *bad, int nsys, hipStream_t s) {
    if (d.fuse_n0 <= 0 || nsys <= 0) return;
    const dim3 g((d.fuse_n0 + kFirstRows - 1) / kFirstRows, nsys);
    if (Df) k_factor_first<true><<<g, kRowThreads, 0, s>>>(d, A, a_stride, Ap, Dinv, Df, bad);
    else k_factor_first<false><<<g, kRowThreads, 0, s>>>(d, A, a_stride, Ap, Dinv, Df, bad);
}

template <typename T>
void launch_lsweep(const DevSchedule &d, const T *L, size_t l_stride, const double *in, T *y, size_t vstride,
                   bool fuse_p, const double *r, const double *v, double *p, SysState *st, int q0, int q1, int nsys,
                   int variant, const T *Dinv, size_t d_stride, double *z, int u0_end, const double *yd,
                   hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (q1 <= q0 || nsys <= 0) return;
    with_variant(variant, [&](auto W, auto ST) {
        constexpr int w = decltype(W)::value;
        constexpr int staged = decltype(ST)::value;
        const dim3 g(row_blocks(q1 - q0, w), nsys);
        auto go = [&](auto kern) {
            launch_ev(kern, g, dim3(64 * w), s, ev0, ev1, d, L, l_stride, in, y, vstride, r, v, p, st, q0, q1, Dinv,
                      d_stride, z, u0_end, yd);
        };
        if (yd) {
            if (fuse_p) go(k_lsweep<T, true, w, staged, true>);
            else go(k_lsweep<T, false, w, staged, true>);
        } else {
            if (fuse_p) go(k_lsweep<T, true, w, staged, false>);
            else go(k_lsweep<T, false, w, staged, false>);
        }
    });
}

template <typename T>
void launch_usweep(const DevSchedule &d, const T *U, size_t u_stride, const T *Dinv, size_t d_stride, const T *y,
                   double *z, size_t vstride, SysState *st, int q0, int q1, int nsys, int variant, bool defer,
                   hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (q1 <= q0 || nsys <= 0) return;
    with_variant(variant, [&](auto W, auto ST) {
        constexpr int w = decltype(W)::value;
        constexpr int staged = decltype(ST)::value;
        launch_ev(k_usweep<T, w, staged>, dim3(row_blocks(q1 - q0, w), nsys), dim3(64 * w), s, ev0, ev1, d, U,
                  u_stride, Dinv, d_stride, y, z, vstride, st, q0, q1, defer ? 1 : 0);
    });
}

template void launch_lsweep<double>(const DevSchedule &, const double *, size_t, const double *, double *, size_t,
                                    bool, const double *, const double *, double *, SysState *, int, int, int, int,
                                    const double *, size_t, double *, int, const double *, hipStream_t, hipEvent_t,
                                    hipEvent_t);
template void launch_lsweep<float>(const DevSchedule &, const float *, size_t, const double *, float *, size_t, bool,
                                   const double *, const double *, double *, SysState *, int, int, int, int,
                                   const float *, size_t, double *, int, const double *, hipStream_t, hipEvent_t,
                                   hipEvent_t);
template void launch_usweep<double>(const DevSchedule &, const double *, size_t, const double *, size_t,
                                    const double *, double *, size_t, SysState *, int, int, int, int, bool,
                                    hipStream_t, hipEvent_t, hipEvent_t);
template void launch_usweep<float>(const DevSchedule &, const float *, size_t, const float *, size_t, const float *,
                                   double *, size_t, SysState *, int, int, int, int, bool, hipStream_t, hipEvent_t,
                                   hipEvent_t);

template <typename T>
void launch_lsweep_tiles(const DevSchedule &d, const T *L, size_t l_stride, const double *in, T *y, size_t vstride,
                         bool fuse_p, const double *r, const double *v, double *p, SysState *st, int32_t *flags,
                         SweepCtr *ctr, int nsys, int grid, int spin, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (d.nlt <= 0 || nsys <= 0) return;
    grid = std::max(1, std::min(grid, d.nlt * nsys));
    if (fuse_p)
        launch_ev(k_lsweep_tiles<T, true>, dim3(grid), dim3(kRowThreads), s, ev0, ev1, d, L, l_stride, in, y,
                  vstride, r, v, p, st, flags, ctr, nsys, spin);
    else
        launch_ev(k_lsweep_tiles<T, false>, dim3(grid), dim3(kRowThreads), s, ev0, ev1, d, L, l_stride, in, y,
                  vstride, r, v, p, st, flags, ctr, nsys, spin);
}

template <typename T>
void launch_usweep_tiles(const DevSchedule &d, const T *U, size_t u_stride, const T *Dinv, size_t d_stride,
                         const T *y, double *z, size_t vstride, SysState *st, int32_t *flags, SweepCtr *ctr, int nsys,
                         int grid, int spin, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (d.nut <= 0 || nsys <= 0) return;
    grid = std::max(1, std::min(grid, d.nut * nsys));
    launch_ev(k_usweep_tiles<T>, dim3(grid), dim3(kRowThreads), s, ev0, ev1, d, U, u_stride, Dinv, d_stride, y, z,
              vstride, st, flags, ctr, nsys, spin);
}

template void launch_lsweep_tiles<double>(const DevSchedule &, const double *, size_t, const double *, double *,
                                          size_t, bool, const double *, const double *, double *, SysState *,
                                          int32_t *, SweepCtr *, int, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_lsweep_tiles<float>(const DevSchedule &, const float *, size_t, const double *, float *,
                                         size_t, bool, const double *, const double *, double *, SysState *,
                                         int32_t *, SweepCtr *, int, int, int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_usweep_tiles<double>(const DevSchedule &, const double *, size_t, const double *, size_t,
                                          const double *, double *, size_t, SysState *, int32_t *, SweepCtr *, int,
                                          int, int, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_usweep_tiles<float>(const DevSchedule &, const float *, size_t, const float *, size_t,
                                         const float *, double *, size_t, SysState *, int32_t *, SweepCtr *, int,
                                         int, int, hipStream_t, hipEvent_t, hipEvent_t);

// ev0 / ev1 (optional): events the dispatch itself records at the SpMV
// kernel's start and end (kernel time only, no launch overhead).
template <int MODE>
static void spmv_any(int variant, int n, const int32_t *ptr, const int32_t *col, const double *A, size_t a_stride,
                     const double *x, double *y, size_t vstride, const double *w1, double *part, size_t part_stride,
                     uint32_t *tk, size_t tk_stride, SysState *st, int nsys, int split, const WellsDev &wl,
                     hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int r0 = 0) {
    if (wl.nw > 0) launch_wells_t2(wl, x, vstride, nsys, s);
    int waves = 1;
    with_variant(variant, [&](auto W, auto ST) {
        constexpr int w = decltype(W)::value;
        constexpr int staged = decltype(ST)::value;
        waves = spmv_grid(n - r0, w) * w;
        const dim3 g(spmv_grid(n - r0, w), nsys), b(64 * w);
        if (ev0)
            hipExtLaunchKernelGGL(k_spmv<MODE, w, staged>, g, b, 0, s, ev0, ev1, 0, n, ptr, col, A, a_stride, x, y,
                                  vstride, w1, (const double *)nullptr, part, part_stride, tk, tk_stride, st,
                                  split, wl, r0);
        else
            k_spmv<MODE, w, staged><<<g, b, 0, s>>>(n, ptr, col, A, a_stride, x, y, vstride, w1, nullptr, part,
                                                    part_stride, tk, tk_stride, st, split, wl, r0);
    });
    if (MODE != SPMV_PLAIN && MODE != SPMV_RUN && (split == 1 || (split == 2 && MODE == SPMV_TRUE)))
        k_spmv_total<MODE><<<dim3(1, nsys), kTotalThreads, 0, s>>>(part, part_stride, waves, st);
}

void launch_wells_fix(const WellsDev &w, double *y, const double *w1, size_t vstride, double *part,
                      size_t part_stride, int at, SysState *st, int nsys, hipStream_t s) {
    if (w.nw <= 0 || w.nfix <= 0 || nsys <= 0) return;
    k_wells_fix<<<dim3(1, nsys), 256, 0, s>>>(w, y, w1, vstride, part, part_stride, at, st);
}

void launch_wells_t2(const WellsDev &w, const double *x, size_t xstride, int nsys, hipStream_t s) {
    if (w.nw <= 0 || nsys <= 0) return;
    k_wells_t2<<<dim3((w.nw + 3) / 4, nsys), 256, 0, s>>>(w, x, xstride);
}

void launch_spmv(int n, const int32_t *ptr, const int32_t *col, const double *A, size_t a_stride, const double *x,
                 double *y, size_t vstride, int nsys, int variant, const WellsDev &w, hipStream_t s) {
    if (n <= 0 || nsys <= 0) return;
    spmv_any<SPMV_PLAIN>(variant, n, ptr, col, A, a_stride, x, y, vstride, nullptr, nullptr, 0, nullptr, 0, nullptr,
                         nsys, false, w, s);
}

void launch_setup(const DevSchedule &d, const double *b_orig, const int32_t *bad, double reduction, int max_iter,
                  Krylov &k, int nsys, hipStream_t s) {
    k_setup<<<dim3(vec_blocks(d.n), nsys), kVecThreads, 0, s>>>(d.n, d.perm, b_orig, k, bad, reduction, max_iter);
}

void launch_spmv_v(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant,
                   int split, const WellsDev &w, int r0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    spmv_any<SPMV_V>(variant, d.n, d.prow, d.pcol, Ap, a_stride, k.phat, k.v, k.vstride, k.rhat, k.spart,
                     k.spart_stride, k.tickets, k.ticket_stride, k.st, nsys, split, w, s, ev0, ev1, r0);
}

// Where the consumer of a fused product finds the fused launch's group sums
// (the fused launch takes the waves per workgroup of the SpMV's shape).
static SpmvSums fused_sums(const DevSchedule &d, bool fused, int spmv_variant) {
    if (!fused) return SpmvSums{0, 0};
    const int g = fuse_blocks(d.fuse_n0, variant_waves(spmv_variant));
    return SpmvSums{2 * g, (g + 31) / 32};
}

int wells_fix_at(const DevSchedule &d, int spmv_variant) {
    const SpmvSums f = fused_sums(d, true, spmv_variant);
    return f.offset + 2 * f.count;
}

void launch_s_update(const DevSchedule &d, Krylov &k, int nsys, int spmv_variant, int split, bool fused,
                     hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool fix) {
    const SpmvSums at = spmv_sums(d.n - (fused ? d.fuse_n0 : 0), variant_waves(spmv_variant), split);
    SpmvSums f = fused_sums(d, fused, spmv_variant);
    if (fused && fix) ++f.count;
    launch_ev(k_s_update, dim3(vec_blocks(d.n), nsys), dim3(kVecThreads), s, ev0, ev1, k, at.offset, at.count,
              f.offset, f.count);
}

void launch_p_update(const DevSchedule &d, Krylov &k, int nsys, hipStream_t s) {
    const int m = 3 * d.fuse_n0;
    if (m <= 0 || nsys <= 0) return;
    const int g = std::min((m + kVecTile - 1) / kVecTile, kVecMaxBlocks);
    k_p_update<<<dim3(g, nsys), kVecThreads, 0, s>>>(k, m);
}

void launch_spmv_t(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant,
                   int split, const WellsDev &w, int r0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    spmv_any<SPMV_T>(variant, d.n, d.prow, d.pcol, Ap, a_stride, k.shat, k.t, k.vstride, k.s, k.spart,
                     k.spart_stride, k.tickets, k.ticket_stride, k.st, nsys, split, w, s, ev0, ev1, r0);
}

void launch_xr_update(const DevSchedule &d, Krylov &k, int nsys, int spmv_variant, int split, bool fused,
                      hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool fix) {
    const SpmvSums at = spmv_sums(d.n - (fused ? d.fuse_n0 : 0), variant_waves(spmv_variant), split);
    SpmvSums f = fused_sums(d, fused, spmv_variant);
    if (fused && fix) ++f.count;
    launch_ev(k_xr_update, dim3(vec_blocks(d.n), nsys), dim3(kVecThreads), s, ev0, ev1, k, at.offset, at.count,
              f.offset, f.count);
}

template <typename T>
void launch_usweep_spmv(const DevSchedule &d, const double *Ap, size_t a_stride, const T *Dinv, size_t d_stride,
                        const T *y, const double *yd, double *z, double *out, const double *w1, SysState *st,
                        Krylov &k, int nsys, int mode, int spmv_variant, bool defer, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1, bool lp) {
    if (d.fuse_n0 <= 0 || nsys <= 0) return;
    // the SpMV's launch shape: its waves per workgroup, and non-temporal
    // matrix loads for the shapes that use them (direct shapes stage too:
    // the product walk rereads the staged blocks)
    with_variant(spmv_variant, [&](auto Wc, auto ST) {
        constexpr int w = decltype(Wc)::value;
        constexpr bool nt = decltype(ST)::value == 2;
        const dim3 g(fuse_blocks(d.fuse_n0, w), nsys), b(64 * w);
        auto go = [&](auto kern, auto yp) {
            launch_ev(kern, g, b, s, ev0, ev1, d, Ap, a_stride, Dinv, d_stride, yp, z, out, w1, k.vstride, st,
                      k.fpart, k.fpart_stride, k.tickets, k.ticket_stride, defer ? 1 : 0, (const double *)k.r,
                      lp ? k.lp : (double *)nullptr);
        };
        auto by_mode = [&](auto yp) {
            using TY = std::remove_const_t<std::remove_pointer_t<decltype(yp)>>;
            if (mode == FUSE_V) go(k_usweep_spmv<T, SPMV_V, w, nt, TY>, yp);
            else if (mode == FUSE_T) go(k_usweep_spmv<T, SPMV_T, w, nt, TY>, yp);
            else go(k_usweep_spmv<T, SPMV_PLAIN, w, nt, TY>, yp);
        };
        if constexpr (std::is_same_v<T, double>) by_mode(yd ? yd : y);
        else if (yd) by_mode(yd);
        else by_mode(y);
    });
}
template void launch_usweep_spmv<double>(const DevSchedule &, const double *, size_t, const double *, size_t,
                                         const double *, const double *, double *, double *, const double *,
                                         SysState *, Krylov &, int, int, int, bool, hipStream_t, hipEvent_t,
                                         hipEvent_t, bool);
template void launch_usweep_spmv<float>(const DevSchedule &, const double *, size_t, const float *, size_t,
                                        const float *, const double *, double *, double *, const double *,
                                        SysState *, Krylov &, int, int, int, bool, hipStream_t, hipEvent_t,
                                        hipEvent_t, bool);

void launch_spmv_lp(const DevSchedule &d, const double *Ap, size_t a_stride, Krylov &k, int nsys, int variant,
                    hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int r0 = d.fuse_n0;
    if (d.n - r0 <= 0 || nsys <= 0) return;
    // the SpMV's launch shape (waves per workgroup, load kind); direct
    // shapes stage too
    with_variant(variant, [&](auto Wc, auto ST) {
        constexpr int w = decltype(Wc)::value;
        constexpr bool nt = decltype(ST)::value == 2;
        launch_ev(k_spmv_lp<w, nt>, dim3(spmv_grid(d.n - r0, w), nsys), dim3(64 * w), s, ev0, ev1, d.n, r0, d.prow,
                  d.pcol, Ap, a_stride, (const double *)k.phat, k.v, k.vstride, (const double *)k.rhat, k.lp,
                  k.spart, k.spart_stride, k.tickets, k.ticket_stride, k.st);
    });
}

void launch_lower_parts(const DevSchedule &d, const double *Dinv, size_t d_stride, Krylov &k, int nsys,
                        hipStream_t s) {
    const int n0 = d.fuse_n0;
    if (d.n <= n0 || nsys <= 0) return;
    k_lower_parts<<<dim3(row_blocks(d.n - n0), nsys), kRowThreads, 0, s>>>(n0, d.n, Dinv, d_stride, k.s, k.lp,
                                                                           k.shat, k.vstride, k.st);
}

void launch_permute_vec(const int32_t *perm, const double *in, double *out, int n, size_t vstride, int nsys,
                        bool scatter, hipStream_t s) {
    if (n <= 0 || nsys <= 0) return;
    k_permute_vec<<<dim3(copy_blocks(3 * (size_t)n), nsys), 256, 0, s>>>(perm, in, out, n, vstride,
                                                                         scatter ? 1 : 0);
}

template <typename T>
void launch_fill_u(const DevSchedule &d, const double *Ap, size_t a_stride, T *U, size_t u_stride, int f0, int f1,
                   int nsys, hipStream_t s) {
    if (f1 <= f0 || nsys <= 0) return;
    k_fill_u<T><<<dim3(copy_blocks((size_t)(f1 - f0) * 9), nsys), 256, 0, s>>>(d.usrc, Ap, a_stride, U, u_stride, f0,
                                                                             f1);
}
template void launch_fill_u<double>(const DevSchedule &, const double *, size_t, double *, size_t, int, int, int,
                                    hipStream_t);
template void launch_fill_u<float>(const DevSchedule &, const double *, size_t, float *, size_t, int, int, int,
                                   hipStream_t);

void launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t s) {
    if (count == 0) return;
    k_fill_u32<<<copy_blocks(count), 256, 0, s>>>(p, count, value);
}

void launch_finish(const DevSchedule &d, const int32_t *rowptr, const int32_t *colidx, const double *A,
                   size_t a_stride, const double *b_orig, double *x_orig, Krylov &k, int nsys, int variant,
                   int split, const WellsDev &w, hipStream_t s) {
    if (d.n <= 0 || nsys <= 0) return;
    launch_permute_vec(d.perm, k.x, x_orig, d.n, k.vstride, nsys, true, s);
    spmv_any<SPMV_TRUE>(variant, d.n, rowptr, colidx, A, a_stride, x_orig, nullptr, 3 * (size_t)d.n, b_orig, k.part,
                        k.part_stride, k.tickets, k.ticket_stride, k.st, nsys, split, w, s);
}

// ------------------------------------------------------------------ GMRES

void launch_spmv_running(const DevSchedule &d, const double *Ap, size_t a_stride, const double *x, double *y,
                         size_t vstride, SysState *st, int nsys, int variant, const WellsDev &w, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1, int r0) {
    if (d.n <= r0 || nsys <= 0) return;
    spmv_any<SPMV_RUN>(variant, d.n, d.prow, d.pcol, Ap, a_stride, x, y, vstride, nullptr, nullptr, 0, nullptr, 0,
                       st, nsys, 0, w, s, ev0, ev1, r0);
}

// Workgroups of the GMRES vector kernels: one per 256 * items entries of a
// padded vector (a multiple of 1024), at most kVecMaxBlocks (the partial
// buffers are sized for that).
static int gm_blocks(int n, int items = 1) {
    const size_t g = vec_stride(n) / ((size_t)kGmThreads * items);
    return (int)std::max<size_t>(1, std::min<size_t>(g, kVecMaxBlocks));
}

// Call f(NV, IT) with the smallest compiled coefficient count NV >= jv and
// the entries per thread that keep about 16 loads in flight per thread.
template <typename F>
static void with_nv(int jv, F &&f) {
    using std::integral_constant;
    if (jv <= 2) f(integral_constant<int, 2>{}, integral_constant<int, 4>{});
    else if (jv <= 4) f(integral_constant<int, 4>{}, integral_constant<int, 4>{});
    else if (jv <= 8) f(integral_constant<int, 8>{}, integral_constant<int, 2>{});
    else if (jv <= 16) f(integral_constant<int, 16>{}, integral_constant<int, 1>{});
    else f(integral_constant<int, kGmMax + 1>{}, integral_constant<int, 1>{});
}

void launch_gm_init(const GmWork &g, int nsys, hipStream_t s) {
    if (nsys <= 0) return;
    k_gm_init<<<(nsys + 63) / 64, 64, 0, s>>>(g, nsys);
}

void launch_gm_normalise(const GmWork &g, const double *src, int col, int from_w, int n, int nsys, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0) return;
    launch_ev(k_gm_normalise, dim3(gm_blocks(n), nsys), dim3(kGmThreads), s, ev0, ev1, g, src, col, from_w);
}

void launch_gm_dots(const GmWork &g, int jv, const double *w, int n, int nsys, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0 || jv < 1 || jv > kGmMax) return;
    with_nv(jv, [&](auto NV, auto IT) {
        constexpr int it = decltype(IT)::value;
        launch_ev(k_gm_dots<decltype(NV)::value, it>, dim3(gm_blocks(n, it), nsys), dim3(kGmThreads), s, ev0, ev1, g,
                  jv, w);
    });
}

void launch_gm_orth(const GmWork &g, int jv, double *w, bool last, int n, int nsys, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0 || jv < 1 || jv > kGmMax) return;
    with_nv(jv, [&](auto NV, auto IT) {
        constexpr int nv = decltype(NV)::value, it = decltype(IT)::value;
        const dim3 grid(gm_blocks(n, it), nsys);
        if (last)
            launch_ev(k_gm_orth<nv, true, it>, grid, dim3(kGmThreads), s, ev0, ev1, g, jv, w);
        else
            launch_ev(k_gm_orth<nv, false, it>, grid, dim3(kGmThreads), s, ev0, ev1, g, jv, w);
    });
}

void launch_gm_combine(const GmWork &g, double *u, int n, int nsys, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0) return;
    launch_ev(k_gm_combine, dim3(gm_blocks(n), nsys), dim3(kGmThreads), s, ev0, ev1, g, u);
}

void launch_gm_xupdate(const GmWork &g, double *x, const double *z, int n, int nsys, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0) return;
    launch_ev(k_gm_xupdate, dim3(gm_blocks(n), nsys), dim3(kGmThreads), s, ev0, ev1, g, x, z);
}

void launch_gm_phase(const GmWork &g, int nsys, hipStream_t s) {
    if (nsys <= 0) return;
    k_gm_phase<<<(nsys + 63) / 64, 64, 0, s>>>(g, nsys);
}

void launch_gm_restart(const GmWork &g, const double *rhs, const double *w, double *r, int n, int nsys,
                       hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (n <= 0 || nsys <= 0) return;
    launch_ev(k_gm_restart, dim3(gm_blocks(n), nsys), dim3(kGmThreads), s, ev0, ev1, g, rhs, w, r);
}

}  // namespace rs
