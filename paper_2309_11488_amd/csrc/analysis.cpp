// Host analysis of a BCSR pattern: validation, orderings (natural, level
// scheduling, DSatur graph colouring), the reordered pattern, lower/upper
// sweep schedules and the ILU0 update lists.
//
// Orderings follow Section "ILU0" of the paper's implementation chapter:
// level scheduling respects direct and indirect dependencies; graph colouring
// only separates rows that are directly coupled, so more rows run together;
// the natural order is the sequential reference.  A reordered copy of the
// matrix is made with each level/colour contiguous.
#include "analysis.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <tuple>
#include <utility>

#include "../../include/rsolve.h"

namespace rs {

int validate_pattern(int n, int nnzb, const int32_t *rowptr, const int32_t *colidx, int *bad_row) {
    *bad_row = -1;
    if (rowptr[0] != 0 || rowptr[n] != nnzb) return RS_BAD_PATTERN;
    for (int i = 0; i < n; ++i) {
        const int a = rowptr[i], b = rowptr[i + 1];
        if (b < a || b > nnzb) { *bad_row = i; return RS_BAD_PATTERN; }
        bool diag = false;
        for (int p = a; p < b; ++p) {
            const int j = colidx[p];
            if (j < 0 || j >= n || (p > a && colidx[p - 1] >= j)) { *bad_row = i; return RS_BAD_PATTERN; }
            diag |= (j == i);
        }
        if (!diag) { *bad_row = i; return RS_MISSING_DIAGONAL; }
    }
    return RS_OK;
}

// Stable grouping of rows by an integer key in [0, nkeys): order[pos] = row,
// start[k] = first position of key k.
static void group_by_key(const std::vector<int32_t> &key, int nkeys, std::vector<int32_t> &order,
                         std::vector<int32_t> &start) {
    const int n = (int)key.size();
    start.assign(nkeys + 1, 0);
    for (int i = 0; i < n; ++i) start[key[i] + 1]++;
    for (int k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    std::vector<int32_t> next(start.begin(), start.end() - 1);
    order.resize(n);
    for (int i = 0; i < n; ++i) order[next[key[i]]++] = i;
}

// Longest-path depth through lower (j < i) or upper (j > i) neighbours.
static int depth_lower(int n, const int32_t *rowptr, const int32_t *colidx, std::vector<int32_t> &d) {
    d.assign(n, 0);
    int depth = n > 0 ? 1 : 0;
    for (int i = 0; i < n; ++i) {
        int v = 0;
        for (int p = rowptr[i]; p < rowptr[i + 1] && colidx[p] < i; ++p) v = std::max(v, d[colidx[p]] + 1);
        d[i] = v;
        depth = std::max(depth, v + 1);
    }
    return depth;
}

static int depth_upper(int n, const int32_t *rowptr, const int32_t *colidx, std::vector<int32_t> &d) {
    d.assign(n, 0);
    int depth = n > 0 ? 1 : 0;
    for (int i = n - 1; i >= 0; --i) {
        int v = 0;
        for (int p = rowptr[i + 1] - 1; p >= rowptr[i] && colidx[p] > i; --p) v = std::max(v, d[colidx[p]] + 1);
        d[i] = v;
        depth = std::max(depth, v + 1);
    }
    return depth;
}

// DSatur's result on a bipartite graph, without its queue.  Whenever DSatur
// starts a connected component every uncoloured row has saturation 0, so it
// takes the component's row with the most neighbours (lowest index first)
// and gives it colour 0; from then on each row it picks in that component
// sees one colour only, and takes the other: the colour of a row is the
// parity of its distance from that first row.  One breadth-first pass per
// component gives parities relative to its lowest row, checks that no edge
// joins equal parities and finds the first row; the component is flipped
// when that row's parity is 1.  Returns false (colour undefined) when the
// graph is not bipartite.
static bool bipartite_colour(int n, const std::vector<int32_t> &nptr, const std::vector<int32_t> &nb,
                             std::vector<int32_t> &colour) {
    colour.assign(n, -1);
    std::vector<int32_t> members;
    members.reserve(1024);
    for (int s = 0; s < n; ++s) {
        if (colour[s] >= 0) continue;
        members.clear();
        members.push_back(s);
        colour[s] = 0;
        int first = s;
        for (size_t h = 0; h < members.size(); ++h) {
            const int v = members[h];
            const int dv = nptr[v + 1] - nptr[v], df = nptr[first + 1] - nptr[first];
            if (dv > df || (dv == df && v < first)) first = v;
            for (int p = nptr[v]; p < nptr[v + 1]; ++p) {
                const int j = nb[p];
                if (colour[j] < 0) { colour[j] = 1 - colour[v]; members.push_back(j); }
                else if (colour[j] == colour[v]) return false;
            }
        }
        if (colour[first] == 1)
            for (int32_t v : members) colour[v] = 1 - colour[v];
    }
    return true;
}

// Symmetrised neighbour lists without the row itself, ascending, unique:
// the merge of row i (sorted) with column i (the transpose built row by
// row, so sorted too).  Neighbours of i: nb[nptr[i] .. nptr[i+1]).
static void symmetric_neighbours(int n, const int32_t *rowptr, const int32_t *colidx, std::vector<int32_t> &nptr,
                                 std::vector<int32_t> &nb) {
    const int nnz = rowptr[n];
    std::vector<int32_t> tptr(n + 1, 0), tcol(std::max(nnz, 1));
    for (int p = 0; p < nnz; ++p) tptr[colidx[p] + 1]++;
    for (int i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    {
        std::vector<int32_t> at(tptr.begin(), tptr.end() - 1);
        for (int i = 0; i < n; ++i)
            for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) tcol[at[colidx[p]]++] = i;
    }
    nptr.assign(n + 1, 0);
    nb.clear();
    nb.reserve(std::max(2 * nnz, 1));
    for (int i = 0; i < n; ++i) {
        int a = rowptr[i], b = tptr[i];
        const int ae = rowptr[i + 1], be = tptr[i + 1];
        while (a < ae || b < be) {
            int v;
            if (b >= be || (a < ae && colidx[a] < tcol[b])) v = colidx[a++];
            else if (a >= ae || tcol[b] < colidx[a]) v = tcol[b++];
            else { v = colidx[a++]; ++b; }
            if (v != i) nb.push_back(v);
        }
        nptr[i + 1] = (int32_t)nb.size();
    }
}

// Reverse Cuthill-McKee renumbering followed by level scheduling (the
// level-reducing reordering for patterns whose non-neighbour connections
// chain distant rows; Section "ILU0" of the implementation chapter and the
// comparison of level sets with graph colouring in the results).  On the
// symmetrised graph, Cuthill and McKee (1969): every breadth-first search
// starts at the unnumbered row with the fewest neighbours (lowest index on
// a tie); a row leaving the queue appends its unnumbered neighbours by
// increasing neighbour count (lower index on a tie).  Reversing the
// sequence gives each row its position.  A row's level is one more than the
// deepest level among its neighbours at lower positions (0 if none).
// perm lists rows by (level, position); set_ptr holds the level starts.
static int rcm_levels(int n, const int32_t *rowptr, const int32_t *colidx, std::vector<int32_t> &perm,
                      std::vector<int32_t> &set_ptr) {
    std::vector<int32_t> nptr, nb;
    symmetric_neighbours(n, rowptr, colidx, nptr, nb);
    auto deg = [&](int v) { return nptr[v + 1] - nptr[v]; };
    auto before = [&](int a, int b) { return deg(a) < deg(b) || (deg(a) == deg(b) && a < b); };
    // start rows: all rows by (neighbours, index); a cursor skips numbered ones
    std::vector<int32_t> starts(n);
    for (int i = 0; i < n; ++i) starts[i] = i;
    std::stable_sort(starts.begin(), starts.end(), [&](int a, int b) { return deg(a) < deg(b); });
    std::vector<int32_t> seq;
    seq.reserve(n);
    std::vector<char> taken(n, 0);
    std::vector<int32_t> cand;
    size_t cursor = 0;
    while ((int)seq.size() < n) {
        while (taken[starts[cursor]]) ++cursor;
        const int s0 = starts[cursor];
        taken[s0] = 1;
        seq.push_back(s0);
        for (size_t h = seq.size() - 1; h < seq.size(); ++h) {
            const int v = seq[h];
            cand.clear();
            for (int p = nptr[v]; p < nptr[v + 1]; ++p)
                if (!taken[nb[p]]) cand.push_back(nb[p]);
            std::sort(cand.begin(), cand.end(), before);
            for (int32_t c : cand) {
                taken[c] = 1;
                seq.push_back(c);
            }
        }
    }
    // position of row v: n - 1 - (its place in seq); visit rows by position
    std::vector<int32_t> pos(n), level(n, 0);
    for (int k = 0; k < n; ++k) pos[seq[k]] = n - 1 - k;
    int nlev = n > 0 ? 1 : 0;
    for (int k = n - 1; k >= 0; --k) {
        const int v = seq[k];
        int lv = 0;
        for (int p = nptr[v]; p < nptr[v + 1]; ++p)
            if (pos[nb[p]] < pos[v]) lv = std::max(lv, level[nb[p]] + 1);
        level[v] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    // rows by (level, position): count per level, then place rows in position order
    set_ptr.assign(nlev + 1, 0);
    for (int i = 0; i < n; ++i) set_ptr[level[i] + 1]++;
    for (int l = 0; l < nlev; ++l) set_ptr[l + 1] += set_ptr[l];
    std::vector<int32_t> next(set_ptr.begin(), set_ptr.end() - 1);
    perm.resize(n);
    for (int k = n - 1; k >= 0; --k) perm[next[level[seq[k]]]++] = seq[k];
    return nlev;
}

// DSatur colouring (Brelaz 1979); two rows conflict when either holds the
// other in its pattern.  The next row coloured is the uncoloured one with the
// most distinct colours among its neighbours, then the most neighbours, then
// the lowest index; it takes the lowest colour its neighbours leave free.
// Saturation only grows: when row v takes colour c, a neighbour's saturation
// grows by one unless another of its coloured neighbours already holds c, and
// its queue entry is renewed (entries whose saturation is stale are skipped).
static int dsatur_colour(int n, const int32_t *rowptr, const int32_t *colidx, std::vector<int32_t> &colour) {
    std::vector<int32_t> nptr, nb;
    symmetric_neighbours(n, rowptr, colidx, nptr, nb);
    if (bipartite_colour(n, nptr, nb, colour)) return n == 0 ? 0 : *std::max_element(colour.begin(), colour.end()) + 1;
    std::vector<int32_t> sat(n, 0), seen(n + 1, -1);
    colour.assign(n, -1);
    // Rows of saturation 0 keep their key until they leave it: they wait in
    // one list by (neighbours descending, index ascending), read by a cursor
    // that only moves forward.  Rows of saturation 1 and up, which always
    // come first, sit in the queue below.
    int maxd = 0;
    for (int i = 0; i < n; ++i) maxd = std::max(maxd, nptr[i + 1] - nptr[i]);
    std::vector<int32_t> zero(n);
    {
        std::vector<int32_t> at(maxd + 2, 0);   // counting sort, degree descending
        for (int i = 0; i < n; ++i) ++at[maxd - (nptr[i + 1] - nptr[i]) + 1];
        for (int d = 0; d <= maxd; ++d) at[d + 1] += at[d];
        for (int i = 0; i < n; ++i) zero[at[maxd - (nptr[i + 1] - nptr[i])]++] = i;
    }
    // The queue: with at most kBucketDegree neighbours per row, one bucket per
    // (saturation, neighbours) pair, each a min-heap of row indices, scanned
    // from the highest pair down; else one heap of (saturation, neighbours,
    // -row).  Entries whose saturation is stale are dropped when they surface.
    constexpr int kBucketDegree = 255;
    const bool buckets = maxd <= kBucketDegree;
    const int w = maxd + 1;
    std::vector<std::vector<int32_t>> bk(buckets ? (size_t)w * w : 0);
    int top = -1;
    using Entry = std::tuple<int32_t, int32_t, int32_t>;
    std::priority_queue<Entry> q;
    auto push = [&](int j) {
        const int d = nptr[j + 1] - nptr[j];
        if (buckets) {
            const int b = sat[j] * w + d;
            bk[b].push_back(j);
            std::push_heap(bk[b].begin(), bk[b].end(), std::greater<int32_t>());
            top = std::max(top, b);
        } else {
            q.emplace(sat[j], d, -j);
        }
    };
    // the uncoloured row of highest positive saturation, or -1
    auto pop_best = [&]() -> int {
        if (buckets) {
            while (top >= 0) {
                std::vector<int32_t> &h = bk[top];
                if (h.empty()) { --top; continue; }
                std::pop_heap(h.begin(), h.end(), std::greater<int32_t>());
                const int r = h.back();
                h.pop_back();
                if (colour[r] < 0 && sat[r] * w + (nptr[r + 1] - nptr[r]) == top) return r;
            }
            return -1;
        }
        while (!q.empty()) {
            const auto [s, d, mr] = q.top();
            q.pop();
            if (colour[-mr] < 0 && s == sat[-mr]) return -mr;
        }
        return -1;
    };
    size_t zc = 0;
    int ncol = 0;
    for (int done = 0; done < n; ++done) {
        int v = pop_best();
        if (v < 0) {
            // no row of positive saturation is left uncoloured
            while (colour[zero[zc]] >= 0 || sat[zero[zc]] != 0) ++zc;
            v = zero[zc];
        }
        for (int p = nptr[v]; p < nptr[v + 1]; ++p)
            if (colour[nb[p]] >= 0) seen[colour[nb[p]]] = v;
        int c = 0;
        while (seen[c] == v) ++c;
        colour[v] = c;
        ncol = std::max(ncol, c + 1);
        for (int p = nptr[v]; p < nptr[v + 1]; ++p) {
            const int j = nb[p];
            if (colour[j] >= 0) continue;
            bool held = false;
            for (int r = nptr[j]; r < nptr[j + 1] && !held; ++r) held = nb[r] != v && colour[nb[r]] == c;
            if (!held) {
                ++sat[j];
                push(j);
            }
        }
    }
    return ncol;
}

int make_ordering(int n, const int32_t *rowptr, const int32_t *colidx, int ordering, std::vector<int32_t> &perm,
                  std::vector<int32_t> &set_ptr) {
    std::vector<int32_t> key;
    int nsets;
    if (ordering == RS_ORDER_LEVEL_SET) {
        nsets = depth_lower(n, rowptr, colidx, key);
    } else if (ordering == RS_ORDER_GRAPH_COLOUR) {
        nsets = dsatur_colour(n, rowptr, colidx, key);
    } else if (ordering == RS_ORDER_RCM_LEVEL_SET) {
        return rcm_levels(n, rowptr, colidx, perm, set_ptr);
    } else {
        perm.resize(n);
        set_ptr.resize(n + 1);
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = 0; i <= n; ++i) set_ptr[i] = i;
        return n;
    }
    group_by_key(key, nsets, perm, set_ptr);
    return nsets;
}

int make_ordering(int n, const int32_t *rowptr, const int32_t *colidx, int ordering, std::vector<int32_t> &perm) {
    std::vector<int32_t> sp;
    return make_ordering(n, rowptr, colidx, ordering, perm, sp);
}

// Split every level into tiles of at most R rows and collect each tile's
// dependencies (the tiles owning the rows its blocks reference).
static void make_tiles(int n, int nlev, const std::vector<int32_t> &lev_ptr, int R, const std::vector<int32_t> &ptr,
                       const std::vector<int32_t> &col, const std::vector<int32_t> &pos_of_row, Schedule::Tiles &t) {
    t.start.clear();
    for (int l = 0; l < nlev; ++l)
        for (int q = lev_ptr[l]; q < lev_ptr[l + 1]; q += R) t.start.push_back(q);
    t.n = (int)t.start.size();
    t.start.push_back(n);
    std::vector<int32_t> tile_of(n);
    for (int k = 0; k < t.n; ++k)
        for (int q = t.start[k]; q < t.start[k + 1]; ++q) tile_of[q] = k;
    t.dep_ptr.assign(t.n + 1, 0);
    t.dep.clear();
    std::vector<int32_t> d;
    for (int k = 0; k < t.n; ++k) {
        d.clear();
        for (int e = ptr[t.start[k]]; e < ptr[t.start[k + 1]]; ++e) d.push_back(tile_of[pos_of_row[col[e]]]);
        std::sort(d.begin(), d.end());
        d.erase(std::unique(d.begin(), d.end()), d.end());
        t.dep.insert(t.dep.end(), d.begin(), d.end());
        t.dep_ptr[k + 1] = (int32_t)t.dep.size();
    }
}

int build_schedule(int n, int nnzb, const int32_t *rowptr, const int32_t *colidx, int ordering, Schedule &s,
                   int tile_rows, const int32_t *part) {
    s = Schedule();
    s.n = n;
    s.nnzb = nnzb;
    s.ordering = ordering;
    s.jacobi = part != nullptr;
    // the preconditioner's matrix: A, or its Jacobi matrix
    std::vector<int32_t> jrow, jcol;
    if (part) {
        jrow.assign(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (part[colidx[p]] == part[i]) jcol.push_back(colidx[p]);
            jrow[i + 1] = (int32_t)jcol.size();
        }
        s.n_sets = make_ordering(n, jrow.data(), jcol.data(), ordering, s.perm, s.set_ptr);
    } else {
        s.n_sets = make_ordering(n, rowptr, colidx, ordering, s.perm, s.set_ptr);
    }
    s.iperm.assign(n, 0);
    for (int i = 0; i < n; ++i) s.iperm[s.perm[i]] = i;

    // reordered pattern A' = P A P^T, columns ascending in the new numbering
    s.prow.assign(n + 1, 0);
    s.pcol.resize(nnzb);
    s.psrc.resize(nnzb);
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int i = 0; i < n; ++i) {
        const int old = s.perm[i];
        row.clear();
        for (int p = rowptr[old]; p < rowptr[old + 1]; ++p) row.emplace_back(s.iperm[colidx[p]], p);
        std::sort(row.begin(), row.end());
        const int base = s.prow[i];
        for (size_t q = 0; q < row.size(); ++q) {
            s.pcol[base + q] = row[q].first;
            s.psrc[base + q] = row[q].second;
        }
        s.prow[i + 1] = base + (int)row.size();
    }

    // the preconditioner's reordered pattern (mrow, mcol) with mmap[q] = its
    // position in A'
    std::vector<int32_t> mrow_v, mcol_v, mmap_v;
    const int32_t *mrow = s.prow.data(), *mcol = s.pcol.data();
    if (part) {
        mrow_v.assign(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            for (int p = s.prow[i]; p < s.prow[i + 1]; ++p)
                if (part[s.perm[s.pcol[p]]] == part[s.perm[i]]) {
                    mcol_v.push_back(s.pcol[p]);
                    mmap_v.push_back(p);
                }
            mrow_v[i + 1] = (int32_t)mcol_v.size();
        }
        mrow = mrow_v.data();
        mcol = mcol_v.data();
    }
    const int nnz_m = mrow[n];
    s.nnz_m = nnz_m;
    auto apos = [&](int q) { return part ? mmap_v[q] : q; };

    // sweep schedules on the preconditioner's pattern
    std::vector<int32_t> ldep, udep;
    s.nl_levels = depth_lower(n, mrow, mcol, ldep);
    s.nu_levels = depth_upper(n, mrow, mcol, udep);
    group_by_key(ldep, s.nl_levels, s.lrows, s.lset);
    group_by_key(udep, s.nu_levels, s.urows, s.uset);
    std::vector<int32_t> upos(n);
    for (int q = 0; q < n; ++q) upos[s.urows[q]] = q;

    std::vector<int32_t> a2l(std::max(nnz_m, 1), -1), a2u(std::max(nnz_m, 1), -1), pdiag(n, -1);
    s.lptr.assign(n + 1, 0);
    s.l2u.resize(n);
    for (int q = 0; q < n; ++q) {
        const int i = s.lrows[q];
        int cnt = 0;
        for (int p = mrow[i]; p < mrow[i + 1]; ++p) {
            if (mcol[p] == i) pdiag[i] = apos(p);
            if (mcol[p] >= i) continue;
            a2l[p] = (int)s.lcol.size();
            s.lcol.push_back(mcol[p]);
            s.lsrc.push_back(apos(p));
            s.ldq.push_back(upos[mcol[p]]);
            ++cnt;
        }
        s.lptr[q + 1] = s.lptr[q] + cnt;
        s.l2u[q] = upos[i];
        s.max_lrow = std::max(s.max_lrow, cnt);
    }
    s.uptr.assign(n + 1, 0);
    s.dsrc.resize(n);
    for (int q = 0; q < n; ++q) {
        const int i = s.urows[q];
        int cnt = 0;
        for (int p = mrow[i]; p < mrow[i + 1]; ++p) {
            if (mcol[p] <= i) continue;
            a2u[p] = (int)s.ucol.size();
            s.ucol.push_back(mcol[p]);
            s.usrc.push_back(apos(p));
            ++cnt;
        }
        s.uptr[q + 1] = s.uptr[q] + cnt;
        s.dsrc[q] = pdiag[i];
        s.max_urow = std::max(s.max_urow, cnt);
    }
    s.nL = (int)s.lcol.size();
    s.nU = (int)s.ucol.size();
    s.lsrc_a.resize(s.nL);
    s.usrc_a.resize(s.nU);
    s.dsrc_a.resize(n);
    for (int e = 0; e < s.nL; ++e) s.lsrc_a[e] = s.psrc[s.lsrc[e]];
    for (int f = 0; f < s.nU; ++f) s.usrc_a[f] = s.psrc[s.usrc[f]];
    for (int q = 0; q < n; ++q) s.dsrc_a[q] = s.psrc[s.dsrc[q]];
    if (part) {
        std::vector<char> used(nnzb, 0);
        for (int32_t p : s.lsrc) used[p] = 1;
        for (int32_t p : s.usrc) used[p] = 1;
        for (int32_t p : s.dsrc) used[p] = 1;
        for (int p = 0; p < nnzb; ++p)
            if (!used[p]) {
                s.rest_dst.push_back(p);
                s.rest_src.push_back(s.psrc[p]);
            }
    }

    // update lists: for L block (i,k), every j > k in row k that row i also
    // holds, ascending j, in the order Algorithm 2 applies them.  U_kj is
    // named by its U position, or, when row k has no lower blocks (so
    // nothing updates it and U_kj is A'_kj), by ~(its A' position).
    s.upd_ptr.assign(s.nL + 1, 0);
    for (int q = 0; q < n; ++q) {
        const int i = s.lrows[q];
        for (int e = s.lptr[q]; e < s.lptr[q + 1]; ++e) {
            const int k = s.lcol[e];
            const bool k_no_lower = mcol[mrow[k]] == k;
            const int32_t *ib = mcol + mrow[i], *ie = mcol + mrow[i + 1];
            for (int p = mrow[k]; p < mrow[k + 1]; ++p) {
                const int j = mcol[p];
                if (j <= k) continue;
                const int32_t *hit = std::lower_bound(ib, ie, j);
                if (hit == ie || *hit != j) continue;  // fill outside the pattern is dropped
                const int t = mrow[i] + (int)(hit - ib);
                int code;
                if (j < i) code = 4 * a2l[t] + 0;
                else if (j == i) code = 1;
                else code = 4 * a2u[t] + 2;
                s.upd.push_back(code);
                s.upd.push_back(k_no_lower ? ~s.usrc[a2u[p]] : a2u[p]);
            }
            s.upd_ptr[e + 1] = (int32_t)(s.upd.size() / 2);
        }
    }

    // rows whose upper launch can also form their part of y = A' x (see
    // Schedule::fuse_n0)
    if (!part && n > 0) {
        int n0 = 0;
        while (n0 < n && s.pcol[s.prow[n0]] == n0) ++n0;   // leading rows whose first block is the diagonal
        bool ok = n0 > 0 && 4 * (long long)n0 >= n;   // a quarter of the rows at least
        for (int i = 0; ok && i < n0; ++i)   // no lower block, at least one upper block
            ok = s.pcol[s.prow[i]] == i && s.prow[i + 1] - s.prow[i] >= 2;
        for (int i = n0; ok && i < n; ++i)    // every later row holds a lower block
            ok = s.pcol[s.prow[i]] < i;
        if (ok) {
            const int lf = udep[0];
            ok = lf >= 1 && s.uset[lf + 1] - s.uset[lf] >= n0;
            for (int i = 0; ok && i < n0; ++i) ok = s.urows[s.uset[lf] + i] == i;
            if (ok) {
                s.fuse_n0 = n0;
                s.fuse_q0 = s.uset[lf];
                s.fuse_level = lf;
                s.fuse_nnz = s.prow[n0];
            }
        }
    }
    // (see Schedule::y_in) the upper levels: the rows without upper blocks
    // (all rows from fuse_n0 on), then the fuse_n0 rows
    if (s.fuse_n0 > 0 && s.nl_levels == 2 && s.lset[1] == s.fuse_n0 && s.nu_levels == 2 && s.fuse_level == 1 &&
        s.uset[1] == n - s.fuse_n0) {
        // both schedules keep rows ascending inside a level: the second
        // lower level is rows [fuse_n0, n), the first upper level the same
        // rows at positions 0 .. n - fuse_n0
        bool ok = true;
        for (int q = s.fuse_n0; ok && q < n; ++q) ok = s.lrows[q] == q && s.urows[q - s.fuse_n0] == q;
        s.y_in = ok ? 1 : 0;
    }

    s.lnarrow.assign(s.nl_levels, 1);
    for (int l = 0; l < s.nl_levels; ++l)
        for (int q = s.lset[l]; q < s.lset[l + 1]; ++q) {
            const int uq = s.l2u[q];
            if (s.lptr[q + 1] - s.lptr[q] > 6 || s.uptr[uq + 1] - s.uptr[uq] > 6) {
                s.lnarrow[l] = 0;
                break;
            }
        }
    s.lconsec.assign(s.nl_levels, 1);
    for (int l = 0; l < s.nl_levels; ++l)
        for (int q = s.lset[l]; q < s.lset[l + 1]; ++q)
            if (s.lrows[q] != s.lrows[s.lset[l]] + (q - s.lset[l])) {
                s.lconsec[l] = 0;
                break;
            }
    std::vector<int32_t> lpos(n);
    for (int q = 0; q < n; ++q) lpos[s.lrows[q]] = q;
    make_tiles(n, s.nl_levels, s.lset, tile_rows, s.lptr, s.lcol, lpos, s.ltiles);
    make_tiles(n, s.nu_levels, s.uset, tile_rows, s.uptr, s.ucol, upos, s.utiles);
    return RS_OK;
}

void partition_rows(int n, const int32_t *rowptr, const int32_t *colidx, const double *weights, int n_parts,
                    int32_t *part) {
    if (n <= 0) return;
    n_parts = std::max(1, std::min(n_parts, n));
    std::fill(part, part + n, -1);
    std::vector<double> gain(n, 0.0);       // coupling of an unassigned row to the growing partition
    std::vector<int32_t> touched;
    std::priority_queue<std::pair<double, int32_t>> heap;   // (coupling, -row): strongest, then lowest row
    int cursor = 0;
    for (int q = 0; q < n_parts; ++q) {
        const int target = (int)((int64_t)n * (q + 1) / n_parts - (int64_t)n * q / n_parts);
        heap = {};
        for (int j : touched) gain[j] = 0.0;
        touched.clear();
        int size = 0;
        auto take = [&](int r) {
            part[r] = q;
            ++size;
            for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
                const int j = colidx[p];
                if (part[j] >= 0) continue;
                if (gain[j] == 0.0) touched.push_back(j);
                gain[j] += weights ? std::fabs(weights[p]) + 1e-300 : 1.0;
                heap.emplace(gain[j], -j);
            }
        };
        while (size < target) {
            if (heap.empty()) {              // no unassigned neighbour: jump to the next free row
                while (cursor < n && part[cursor] >= 0) ++cursor;
                if (cursor >= n) break;
                take(cursor);
                continue;
            }
            const auto top = heap.top();
            heap.pop();
            const int r = -top.second;
            if (part[r] >= 0 || top.first != gain[r]) continue;   // taken, or a stale entry
            take(r);
        }
    }
    for (int j = 0; j < n; ++j)
        if (part[j] < 0) part[j] = n_parts - 1;
}

}  // namespace rs
