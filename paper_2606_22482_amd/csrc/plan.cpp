// plan.cpp -- integer preprocessing of A (host, no device calls).
//
// NeutronSparse Sec. 5.2.2: a single scan computes Len(v) (Eq. 4); rows with
// Len <= Thres (Eq. 5) stay on the vector path, the rest are candidates for the
// matrix engine.  Sec. 6.1: the candidates are cut into row windows whose
// height is the tile height; inside a window, columns that are empty (or, by
// the column stage of Sec. 5.2.2 applied per window, too short) are compacted
// away.  The surviving columns are chunked into K-tiles; a tile whose density
// is below alpha goes back to the vector path (Sec. 5.2.1).  Kept tiles are
// stored as a bitmap plus packed values (end of Sec. 5.2.2); everything else
// is the remainder, an index/value list per row.  Sec. 7 (row-window list
// migration): the work is then laid out as lists of items whose costs are
// balanced and whose order puts heavy items first.
#include "plan.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>

namespace spmm {

int dtype_size(int32_t t) { return t == SPMM_F32 ? 4 : 2; }

}  // namespace spmm

extern "C" void spmm_opts_default(spmm_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = SPMM_MODE_AUTO;
    o->window_h = 0;
    o->t_row = SPMM_AUTO_INT;
    o->kt = 0;
    o->n_panel = 0;
    o->row_order = SPMM_ORDER_AUTO;
    o->seg_len = 0;
    o->item_cost = 0;
    o->xcd_remap = -1;
    o->hot_cols = -1;
    o->cold_policy = -1;
    o->pipeline = -1;
    o->win_sched = -1;
    o->local_reorder = -1;
    o->exec = 0;
    o->alpha_c = -1.0f;
    o->alpha = -1.0f;
}

namespace spmm {

uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
        return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

void resolve_options(const spmm_opts *in, const spmm_csr *A, int32_t n, int32_t b_type,
                     spmm_opts *o) {
    spmm_opts d;
    if (in) d = *in; else spmm_opts_default(&d);
    if (d.mode == SPMM_MODE_AUTO) d.mode = SPMM_MODE_MIXED;
    if (d.window_h <= 0) d.window_h = 16;
    if (d.t_row == SPMM_AUTO_INT) d.t_row = 1;
    if (d.kt <= 0) d.kt = 32;
    if (d.n_panel < 0) d.n_panel = 0;
    if (d.row_order == SPMM_ORDER_AUTO) d.row_order = SPMM_ORDER_ORIGINAL_RANGES;
    // Measured on gfx950 with segments launched by column: for f32 B,
    // segments of 128 entries beat 256 on the 2^20-vertex power-law graph
    // (N = 128: 1.033 vs 1.056 ms plain, 1.222 vs 1.317 ms mixed; N = 64:
    // even plain, 0.744 vs 0.804 ms mixed); 16-bit B keeps 256.
    if (d.seg_len <= 0) d.seg_len = b_type == SPMM_F32 ? 128 : 256;
    if (d.item_cost <= 0) {
        double total = (double)(A ? A->nnz : 0) + (double)kRowCost * (double)(A ? A->m : 0);
        // about 2048 items per matrix, so that a matrix run alone (or in a
        // small batch) still fills the device, with items of 32 to 256
        // entries for f32 B and 32 to 512 for 16-bit B (measured on gfx950:
        // 256-entry items beat 512 on the 2^20-vertex power-law graph, 0.962
        // vs 0.970 ms at N = 128 and 0.488 vs 0.492 ms at N = 64, 1024 lost;
        // on the uneven f16 batch 256 lost to 512)
        const double cap = b_type == SPMM_F32 ? 256.0 : 512.0;
        d.item_cost = (int32_t)std::min(cap, std::max(32.0, total / 2048.0));
    }
    if (d.xcd_remap < 0) d.xcd_remap = 1;
    // Measured on gfx950: streaming (non-temporal) gathers of cold rows raise the
    // L2 hit rate but lose Infinity Cache hits and run slower, so by default
    // every B row is gathered with the default policy and no hot set is kept.
    if (d.cold_policy < 0) d.cold_policy = 0;
    if (d.hot_cols < 0) {
        // Sec. 6.2.1: the hottest B rows, capped at 80% of one XCD's L2
        const int np = d.n_panel > 0 ? std::min(d.n_panel, std::max(n, 1)) : std::max(n, 1);
        d.hot_cols = d.cold_policy == 0
                         ? 0
                         : (int32_t)(kHotFraction * kL2BytesPerXcd / ((double)np * dtype_size(b_type)));
    }
    if (d.pipeline < 0) {
        // Measured on gfx950: packing rows by size class pays for 16-bit B rows
        // spanning at most 16 chunk lanes (4 or more lane groups per wavefront:
        // f16 N <= 128 power-law matrices 23% faster).  With 1-2 groups it
        // gains little, and on f32 B (N = 32, 64) it ran 6-15% slower: those
        // gathers are bandwidth-bound and its extra registers cost occupancy.
        const int np = d.n_panel > 0 ? std::min(d.n_panel, std::max(n, 1)) : std::max(n, 1);
        const int chunks = std::min((np + 7) / 8, 128);
        d.pipeline = (b_type != SPMM_F32 && chunks <= 16) ? 3 : 2;
        if (d.cold_policy > 0) d.pipeline = 0;  // only the row-by-row variant selects policies
    }
    if (d.win_sched < 0) d.win_sched = 0;  // window id order: B rows reused in L2
    if (d.local_reorder < 0) d.local_reorder = 0;
    // co-scheduled as two concurrent grids (the vector path keeps its own
    // occupancy beside the LDS-heavy windows); serial kernels for a cold
    // policy, which only the serial kernels select per entry
    if (d.exec <= 0) d.exec = d.cold_policy != 0 ? 1 : 2;
    if (!(d.alpha_c >= 0.0f)) d.alpha_c = 1.0f / (float)d.window_h;
    if (!(d.alpha >= 0.0f)) d.alpha = 1.0f / (float)d.window_h;
    if (d.mode == SPMM_MODE_MFMA_ONLY) {
        d.t_row = -1;
        d.alpha_c = 0.0f;
        d.alpha = 0.0f;
    }
    *o = d;
}

static bool dtype_pair_ok(int32_t v, int32_t b) {
    return (v == SPMM_F32 && b == SPMM_F32) || (v == SPMM_F32 && b == SPMM_BF16) ||
           (v == SPMM_BF16 && b == SPMM_BF16) || (v == SPMM_F16 && b == SPMM_F16);
}

spmm_status validate_shape(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                           std::string &err) {
    if (!A) { err = "A is null"; return SPMM_ERR_INVALID; }
    if (A->m < 0 || A->k < 0 || A->nnz < 0) { err = "negative size"; return SPMM_ERR_INVALID; }
    if (n < 1) { err = "n must be >= 1"; return SPMM_ERR_INVALID; }
    if (A->m >= (1ll << 31) - 1 || A->k >= (1ll << 31) - 1 || A->nnz >= (1ll << 31) - 1) {
        err = "m, k and nnz must be < 2^31 - 1";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (c_type != SPMM_F32) { err = "C must be f32"; return SPMM_ERR_UNSUPPORTED; }
    if (A->val_type < 0 || A->val_type > 2 || b_type < 0 || b_type > 2) {
        err = "unknown dtype";
        return SPMM_ERR_INVALID;
    }
    if (!dtype_pair_ok(A->val_type, b_type)) {
        err = "unsupported (vals, B) dtype pair";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (!A->rowptr) { err = "rowptr is null"; return SPMM_ERR_INVALID; }
    if (A->nnz > 0 && (!A->colidx || !A->vals)) { err = "colidx/vals null"; return SPMM_ERR_INVALID; }
    return SPMM_OK;
}

spmm_status validate_problem(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                             std::string &err) {
    spmm_status st = validate_shape(A, n, b_type, c_type, err);
    if (st != SPMM_OK) return st;
    if (A->rowptr[0] != 0) { err = "rowptr[0] != 0"; return SPMM_ERR_INVALID; }
    for (int64_t r = 0; r < A->m; ++r)
        if (A->rowptr[r + 1] < A->rowptr[r]) { err = "rowptr not monotone"; return SPMM_ERR_INVALID; }
    if (A->rowptr[A->m] != A->nnz) { err = "rowptr[m] != nnz"; return SPMM_ERR_INVALID; }
    for (int64_t p = 0; p < A->nnz; ++p)
        if (A->colidx[p] < 0 || A->colidx[p] >= A->k) {
            err = "column index out of range";
            return SPMM_ERR_INVALID;
        }
    return SPMM_OK;
}

// Sec. 6.1 global stage: the rank of every row in the Rabbit Order of the
// bipartite graph of A (vertices 0..m-1 rows, m..m+k-1 columns, one unit edge
// per stored entry).  Vertices are visited once in increasing degree (ties:
// lower id); a visited vertex u is the root of its community and joins the
// neighbouring community v with the largest modularity gain, compared exactly
// as w_uv * 2M - d_u * d_v > 0 (ties: lower root id), else stays a root.  The
// order lists the roots in visit order, each followed depth first by what
// merged into it, children in merge order.
static std::vector<int64_t> rabbit_rank(int64_t m, int64_t k, const int64_t *rowptr,
                                        const int32_t *colidx) {
    const int64_t n = m + k, nnz = rowptr[m];
    // adjacency: rows -> columns (as m + c), columns -> rows
    std::vector<int64_t> aptr(n + 1, 0);
    for (int64_t r = 0; r < m; ++r) aptr[r + 1] = rowptr[r + 1] - rowptr[r];
    for (int64_t p = 0; p < nnz; ++p) ++aptr[m + colidx[p] + 1];
    for (int64_t v = 0; v < n; ++v) aptr[v + 1] += aptr[v];
    std::vector<int64_t> adj(aptr[n]);
    {
        std::vector<int64_t> fill(aptr.begin(), aptr.end() - 1);
        for (int64_t r = 0; r < m; ++r)
            for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
                const int64_t c = m + colidx[p];
                adj[fill[r]++] = c;
                adj[fill[c]++] = r;
            }
    }
    const __int128 two_m = 2 * (__int128)nnz;
    std::vector<int64_t> deg(n), parent(n);
    std::vector<int64_t> acc(n, 0), touched;
    std::vector<std::vector<int64_t>> children(n);
    // agg[r]: the edges of the vertices merged into root r so far, aggregated
    // as (neighbour, edge count) when each of them was visited; a root's own
    // edges are read from the adjacency when it is visited.  This gives the
    // same counts as scanning every member's adjacency at each visit.
    std::vector<std::vector<std::pair<int64_t, int64_t>>> agg(n);
    for (int64_t v = 0; v < n; ++v) {
        deg[v] = aptr[v + 1] - aptr[v];
        parent[v] = v;
    }
    auto find = [&](int64_t v) {
        int64_t r = v;
        while (parent[r] != r) r = parent[r];
        while (parent[v] != r) {  // path compression; roots are unchanged
            const int64_t up = parent[v];
            parent[v] = r;
            v = up;
        }
        return r;
    };
    std::vector<int64_t> visit(n);
    for (int64_t v = 0; v < n; ++v) visit[v] = v;
    std::stable_sort(visit.begin(), visit.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
    std::vector<int64_t> roots;
    for (int64_t u : visit) {
        touched.clear();
        for (int64_t q = aptr[u]; q < aptr[u + 1]; ++q) {
            const int64_t ry = find(adj[q]);
            if (ry == u) continue;
            if (acc[ry]++ == 0) touched.push_back(ry);
        }
        for (const auto &e : agg[u]) {
            const int64_t ry = find(e.first);
            if (ry == u) continue;
            if (acc[ry] == 0) touched.push_back(ry);
            acc[ry] += e.second;
        }
        std::vector<std::pair<int64_t, int64_t>>().swap(agg[u]);
        int64_t best = -1;
        __int128 best_gain = 0;
        for (int64_t v : touched) {
            const __int128 gain = (__int128)acc[v] * two_m - (__int128)deg[u] * deg[v];
            if (gain > best_gain || (gain == best_gain && best >= 0 && v < best)) {
                best = v;
                best_gain = gain;
            }
        }
        if (best >= 0) {
            std::vector<std::pair<int64_t, int64_t>> &to = agg[best];
            for (int64_t v : touched) to.push_back({v, acc[v]});
        }
        for (int64_t v : touched) acc[v] = 0;
        if (best < 0) {
            roots.push_back(u);
            continue;
        }
        parent[u] = best;
        children[best].push_back(u);
        deg[best] += deg[u];
    }
    std::vector<int64_t> rank(m, 0), stack;
    int64_t pos = 0;
    for (int64_t root : roots) {
        if (parent[root] != root) continue;
        stack.push_back(root);
        while (!stack.empty()) {
            const int64_t v = stack.back();
            stack.pop_back();
            if (v < m) rank[v] = pos++;
            for (auto it = children[v].rbegin(); it != children[v].rend(); ++it) stack.push_back(*it);
        }
    }
    return rank;
}

// Sec. 6.1 local reordering.  D is cut into clusters of crows consecutive
// rows; inside a cluster the current windows (groups of H in D's order) are
// visited in order, and the longest unassigned row of each (ties: earlier)
// becomes an anchor that takes the H-1 unassigned rows of the cluster with
// the highest Jaccard similarity of distinct column sets (compared exactly as
// fractions; ties: earlier in D; an empty union counts as 0).  The rows left
// when every window has been visited form windows in D's order.
static void local_reorder(const std::vector<int32_t> &D, int H, int64_t crows,
                          const int64_t *rowptr, const int32_t *colidx,
                          const std::vector<int64_t> &len, int64_t k,
                          std::vector<std::vector<int32_t>> &out) {
    struct Cand {
        int64_t inter, uni;
        int32_t pos;
    };
    auto better = [](const Cand &a, const Cand &b) {
        const int64_t l = a.inter * b.uni, r = b.inter * a.uni;
        return l != r ? l > r : a.pos < b.pos;
    };
    const int64_t nD = (int64_t)D.size();
    const int64_t nchunks = (nD + crows - 1) / crows;
    // clusters are independent: ranges of them run on threads (each with its
    // own column stamps) and their windows are appended in cluster order
    auto run = [&](int64_t k0, int64_t k1, std::vector<std::vector<int32_t>> &wins) {
        std::vector<int64_t> stamp(std::max<int64_t>(k, 1), 0);
        int64_t now = 0;
        std::vector<Cand> cs;
        for (int64_t ck = k0; ck < k1; ++ck) {
            const int64_t c0 = ck * crows;
            const int32_t n = (int32_t)std::min(crows, nD - c0);
            // distinct columns of each row of the cluster
            std::vector<int64_t> cptr(n + 1, 0);
            std::vector<int32_t> cols;
            for (int32_t i = 0; i < n; ++i) {
                const int32_t r = D[c0 + i];
                const size_t b = cols.size();
                cols.insert(cols.end(), colidx + rowptr[r], colidx + rowptr[r + 1]);
                std::sort(cols.begin() + b, cols.end());
                cols.erase(std::unique(cols.begin() + b, cols.end()), cols.end());
                cptr[i + 1] = (int64_t)cols.size();
            }
            std::vector<uint8_t> used(n, 0);
            for (int32_t w0 = 0; w0 < n; w0 += H) {
                int32_t a = -1;
                for (int32_t i = w0; i < std::min(w0 + H, n); ++i)
                    if (!used[i] && (a < 0 || len[D[c0 + i]] > len[D[c0 + a]])) a = i;
                if (a < 0) continue;
                used[a] = 1;
                ++now;
                for (int64_t q = cptr[a]; q < cptr[a + 1]; ++q) stamp[cols[q]] = now;
                const int64_t na = cptr[a + 1] - cptr[a];
                cs.clear();
                for (int32_t i = 0; i < n; ++i) {
                    if (used[i]) continue;
                    int64_t inter = 0;
                    for (int64_t q = cptr[i]; q < cptr[i + 1]; ++q) inter += stamp[cols[q]] == now;
                    int64_t uni = na + (cptr[i + 1] - cptr[i]) - inter;
                    if (uni == 0) { inter = 0; uni = 1; }
                    cs.push_back({inter, uni, i});
                }
                const size_t take = std::min<size_t>((size_t)(H - 1), cs.size());
                std::partial_sort(cs.begin(), cs.begin() + take, cs.end(), better);
                std::vector<int32_t> slots(H, -1);
                slots[0] = D[c0 + a];
                for (size_t j = 0; j < take; ++j) {
                    slots[j + 1] = D[c0 + cs[j].pos];
                    used[cs[j].pos] = 1;
                }
                wins.push_back(std::move(slots));
            }
            std::vector<int32_t> slots;
            for (int32_t i = 0; i < n; ++i) {
                if (used[i]) continue;
                slots.push_back(D[c0 + i]);
                if ((int)slots.size() == H) {
                    wins.push_back(slots);
                    slots.clear();
                }
            }
            if (!slots.empty()) {
                slots.resize(H, -1);
                wins.push_back(slots);
            }
        }
    };
    size_t nth = std::max<size_t>(1, std::min<size_t>(std::thread::hardware_concurrency(), 16));
    if (const char *env = std::getenv("SPMM_PLAN_THREADS")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v >= 1) nth = (size_t)std::min<long>(v, 64);
    }
    nth = std::min<size_t>(nth, (size_t)std::max<int64_t>(nchunks, 1));
    nth = std::min(nth, std::max<size_t>(1, (size_t(1) << 30) / (8 * (size_t)std::max<int64_t>(k, 1))));
    std::vector<std::vector<std::vector<int32_t>>> parts(nth);
    if (nth == 1) {
        run(0, nchunks, parts[0]);
    } else {
        std::vector<std::thread> th;
        for (size_t i = 0; i < nth; ++i)
            th.emplace_back(run, nchunks * (int64_t)i / (int64_t)nth, nchunks * (int64_t)(i + 1) / (int64_t)nth,
                            std::ref(parts[i]));
        for (auto &t : th) t.join();
    }
    for (auto &pw : parts)
        for (auto &w : pw) out.push_back(std::move(w));
}

spmm_status validate_opts(const spmm_opts &o, std::string &err) {
    if (o.mode < SPMM_MODE_PLAIN_F32 || o.mode > SPMM_MODE_MFMA_ONLY) { err = "mode"; return SPMM_ERR_UNSUPPORTED; }
    if (o.window_h != 16 && o.window_h != 32 && o.window_h != 64) { err = "window_h must be 16, 32 or 64"; return SPMM_ERR_UNSUPPORTED; }
    if (o.kt != 32) { err = "kt must be 32"; return SPMM_ERR_UNSUPPORTED; }
    if (o.row_order < SPMM_ORDER_ORIGINAL_RANGES || o.row_order > SPMM_ORDER_CLUSTERED) { err = "row_order"; return SPMM_ERR_UNSUPPORTED; }
    if (o.seg_len < 1 || o.seg_len > (1 << 30)) { err = "seg_len"; return SPMM_ERR_UNSUPPORTED; }
    if (o.item_cost < 1) { err = "item_cost"; return SPMM_ERR_UNSUPPORTED; }
    if (o.n_panel < 0) { err = "n_panel"; return SPMM_ERR_UNSUPPORTED; }
    if (o.xcd_remap < 0 || o.xcd_remap > 1) { err = "xcd_remap must be 0 or 1"; return SPMM_ERR_UNSUPPORTED; }
    if (o.hot_cols < 0) { err = "hot_cols"; return SPMM_ERR_UNSUPPORTED; }
    if (o.pipeline < 0 || o.pipeline > 3) { err = "pipeline must be 0, 1, 2 or 3"; return SPMM_ERR_UNSUPPORTED; }
    if (o.win_sched < 0 || o.win_sched > 1) { err = "win_sched must be 0 or 1"; return SPMM_ERR_UNSUPPORTED; }
    if (o.local_reorder < 0) { err = "local_reorder"; return SPMM_ERR_UNSUPPORTED; }
    if (o.local_reorder > 0 && o.row_order == SPMM_ORDER_ORIGINAL_RANGES) {
        err = "local_reorder needs the compacted or length-sorted row order";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (o.cold_policy != 0 && o.cold_policy != 2 && o.cold_policy != 16 && o.cold_policy != 18) {
        err = "cold_policy must be 0, 2, 16 or 18";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (o.exec < 1 || o.exec > 3) { err = "exec must be 1, 2 or 3"; return SPMM_ERR_UNSUPPORTED; }
    if (o.cold_policy != 0 && o.exec != 1) {
        err = "a cold policy needs the serial kernels (exec 1)";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (o.cold_policy != 0 && o.pipeline != 0) {
        err = "a cold policy needs the row-by-row vector variant (pipeline 0)";
        return SPMM_ERR_UNSUPPORTED;
    }
    if (!std::isfinite(o.alpha) || o.alpha < 0 || !std::isfinite(o.alpha_c) || o.alpha_c < 0) {
        err = "alpha / alpha_c must be finite and >= 0";
        return SPMM_ERR_UNSUPPORTED;
    }
    return SPMM_OK;
}

// The schedule of a partitioned plan (windows, their tiles and every row's
// remainder known): vector rows, segments of long remainders, cost-balanced
// vector items, window segment ids, window partial items and the window
// launch order (Sec. 7).  Shared by the host builder and the device builder,
// which computes the partition on the device and the schedule here.
int32_t window_item_tiles(int64_t tiles, int32_t n) {
    const int64_t panels = ((int64_t)n + 127) / 128;
    const int64_t want = (tiles * panels + kWindowItems - 1) / kWindowItems;
    int32_t k = kWinTiles;
    while (k < kWinTilesMax && k < want) k *= 2;
    return k;
}

void build_schedule(HostPlan &P) {
    const spmm_opts &o = P.opts;
    const int64_t m = P.m;
    const int H = o.window_h, kt = o.kt, S = o.seg_len;
    const int64_t W = (int64_t)P.windows.size() / H;
    // ---- vector rows, segments ----
    std::vector<uint8_t> covered(m, 0);
    for (int32_t r : P.windows)
        if (r >= 0) covered[r] = 1;
    for (int64_t r = 0; r < m; ++r)
        if (!covered[r]) P.vector_rows.push_back((int32_t)r);
    P.identity_rows = (int64_t)P.vector_rows.size() == m;
    P.nseg.assign(m, 0);
    for (int64_t r = 0; r < m; ++r) {
        int64_t L = P.rem_ptr[r + 1] - P.rem_ptr[r];
        if (L > S) P.nseg[r] = (int32_t)((L + S - 1) / S);
    }
    auto add_segments = [&](int32_t r) {
        for (int32_t j = 0; j < P.nseg[r]; ++j) {
            int64_t b = P.rem_ptr[r] + (int64_t)j * S;
            int64_t e = std::min<int64_t>(b + S, P.rem_ptr[r + 1]);
            P.seg_row.push_back(r);
            P.seg_begin.push_back((int32_t)b);
            P.seg_end.push_back((int32_t)e);
        }
    };

    // vector items: consecutive vector rows with balanced cost (Sec. 7).  Row i
    // (in vector-row order) belongs to item floor(c_i / item_cost), c_i the
    // summed cost of the rows before it (empty items dropped): a rule of prefix
    // sums, so a device-side builder reproduces it exactly.
    P.vitem_ptr.push_back(0);
    {
        int64_t before = 0, bucket = -1;
        const int64_t nv = (int64_t)P.vector_rows.size();
        for (int64_t i = 0; i < nv; ++i) {
            int32_t r = P.vector_rows[i];
            int64_t L = P.rem_ptr[r + 1] - P.rem_ptr[r];
            const int64_t b = before / o.item_cost;
            if (i > 0 && b != bucket) P.vitem_ptr.push_back((int32_t)i);
            bucket = b;
            before += kRowCost + (P.nseg[r] ? P.nseg[r] : L);
        }
        if (nv > 0) P.vitem_ptr.push_back((int32_t)nv);
        // the size-class variant takes each item's rows longest first, so that
        // rows of one size class are packed side by side; split rows go last
        if (o.pipeline == 3 && nv > 0) {
            P.vexec = P.vector_rows;
            auto key = [&](int32_t r) -> int64_t {
                return P.nseg[r] ? -1 : P.rem_ptr[r + 1] - P.rem_ptr[r];
            };
            for (size_t it = 0; it + 1 < P.vitem_ptr.size(); ++it)
                std::stable_sort(P.vexec.begin() + P.vitem_ptr[it], P.vexec.begin() + P.vitem_ptr[it + 1],
                                 [&](int32_t a, int32_t b) { return key(a) > key(b); });
        }
        const std::vector<int32_t> &order = P.vexec.empty() ? P.vector_rows : P.vexec;
        for (size_t it = 0; it + 1 < P.vitem_ptr.size(); ++it) {
            P.vitem_seg.push_back((int32_t)P.seg_row.size());
            for (int32_t i = P.vitem_ptr[it]; i < P.vitem_ptr[it + 1]; ++i) add_segments(order[i]);
        }
    }
    // windows: segment ids in slot order; launch order by window id or heaviest first
    std::vector<int64_t> wcost(W, 0);
    P.win_tiles = window_item_tiles(P.win_tile_ptr.empty() ? 0 : P.win_tile_ptr.back(), P.n);
    P.win_part.push_back(0);
    for (int64_t w = 0; w < W; ++w) {
        P.win_seg.push_back((int32_t)P.seg_row.size());
        const int32_t ta = P.win_tile_ptr[w], tb = P.win_tile_ptr[w + 1];
        // tiles beyond the first win_tiles become partial items of win_tiles each
        for (int32_t t = ta + P.win_tiles; t < tb; t += P.win_tiles) {
            P.wpart_win.push_back((int32_t)w);
            P.wpart_t0.push_back(t);
            P.wpart_t1.push_back(std::min(t + P.win_tiles, tb));
        }
        P.win_part.push_back((int32_t)P.wpart_win.size());
        wcost[w] = (int64_t)std::min(tb - ta, P.win_tiles) * kt +
                   (int64_t)(P.win_part[w + 1] - P.win_part[w]) * H;
        for (int s = 0; s < H; ++s) {
            int32_t r = P.windows[w * H + s];
            if (r < 0) continue;
            int64_t L = P.rem_ptr[r + 1] - P.rem_ptr[r];
            wcost[w] += kRowCost + (P.nseg[r] ? P.nseg[r] : L);
            add_segments(r);
        }
    }
    P.win_order.resize(W);
    for (int64_t w = 0; w < W; ++w) P.win_order[w] = (int32_t)w;
    if (o.win_sched == 1)
        std::stable_sort(P.win_order.begin(), P.win_order.end(),
                         [&](int32_t a, int32_t b) { return wcost[a] > wcost[b]; });

}

spmm_status build_host_plan(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                            const spmm_opts &o, HostPlan &P, std::string &err) {
    auto t_start = std::chrono::steady_clock::now();
    spmm_status st = validate_problem(A, n, b_type, c_type, err);
    if (st != SPMM_OK) return st;
    st = validate_opts(o, err);
    if (st != SPMM_OK) return st;

    const int64_t m = A->m, k = A->k, nnz = A->nnz;
    const int64_t *rowptr = A->rowptr;
    const int32_t *colidx = A->colidx;
    const int H = o.window_h, kt = o.kt;
    const int sval = dtype_size(A->val_type);
    const uint8_t *vbytes = static_cast<const uint8_t *>(A->vals);

    P = HostPlan();
    P.m = m; P.k = k; P.nnz = nnz; P.n = n;
    P.val_type = A->val_type; P.b_type = b_type; P.c_type = c_type;
    P.tile_type = (b_type == SPMM_F16) ? SPMM_F16 : SPMM_BF16;
    P.opts = o;

    std::vector<int64_t> len(m);
    for (int64_t r = 0; r < m; ++r) len[r] = rowptr[r + 1] - rowptr[r];  // Eq. 4

    // ---- row stage (Eq. 5) and windows (Sec. 6.1) ----
    std::vector<std::vector<int32_t>> cand;  // candidate windows, H slots each
    if (o.mode != SPMM_MODE_PLAIN_F32) {
        auto passes = [&](int64_t r) { return len[r] > (int64_t)o.t_row; };
        if (o.row_order == SPMM_ORDER_ORIGINAL_RANGES) {
            for (int64_t w0 = 0; w0 < m; w0 += H) {
                std::vector<int32_t> slots(H, -1);
                bool any = false;
                for (int s = 0; s < H; ++s) {
                    int64_t r = w0 + s;
                    if (r < m && passes(r)) { slots[s] = (int32_t)r; any = true; }
                }
                if (any) cand.push_back(std::move(slots));
                else cand.emplace_back();  // an empty window keeps no tile
            }
        } else {
            std::vector<int32_t> D;
            for (int64_t r = 0; r < m; ++r)
                if (passes(r)) D.push_back((int32_t)r);
            if (o.row_order == SPMM_ORDER_LENGTH_SORTED)
                std::stable_sort(D.begin(), D.end(),
                                 [&](int32_t a, int32_t b) { return len[a] > len[b]; });
            if (o.row_order == SPMM_ORDER_CLUSTERED) {
                const std::vector<int64_t> rank = rabbit_rank(m, k, rowptr, colidx);
                std::sort(D.begin(), D.end(), [&](int32_t a, int32_t b) { return rank[a] < rank[b]; });
            }
            if (o.local_reorder > 0) {
                const int64_t crows = ((int64_t)o.local_reorder + H - 1) / H * H;
                local_reorder(D, H, crows, rowptr, colidx, len, k, cand);
            } else {
                for (size_t w0 = 0; w0 < D.size(); w0 += H) {
                    std::vector<int32_t> slots(H, -1);
                    for (int s = 0; s < H && w0 + s < D.size(); ++s) slots[s] = D[w0 + s];
                    cand.push_back(std::move(slots));
                }
            }
        }
    }

    // ---- column stage, K-tiles, density test, packing ----
    // Candidate windows are independent (each row is in one window, so the
    // in_tile flags they set are disjoint): ranges of them run on separate
    // threads into their own buffers, which are then appended in window order,
    // so the plan is the same for any number of threads.
    const int64_t col_thr = (int64_t)std::floor((double)o.alpha_c * (double)H);
    const double keep_thr = (double)o.alpha * (double)(H * kt);
    std::vector<uint8_t> in_tile(nnz, 0);
    struct StageOut {
        std::vector<int32_t> windows, win_ntiles, tile_cols;
        std::vector<uint32_t> tile_bitmap;
        std::vector<int64_t> tile_nval, tile_src;
        std::vector<uint16_t> tile_vals;
    };
    auto stage = [&](size_t c0, size_t c1, StageOut &out) {
        std::vector<int32_t> cnt(k, 0), pos(k, -1), touched, mcols;
        std::vector<int64_t> src;  // [kept tiles of window][H][kt]
        std::vector<std::pair<int64_t, int64_t>> kept_chunks;  // (start in mcols, ncols)
        for (size_t ci = c0; ci < c1; ++ci) {
            const std::vector<int32_t> &slots = cand[ci];
            if (slots.empty()) continue;
            touched.clear();
            for (int32_t r : slots) {
                if (r < 0) continue;
                for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
                    int32_t c = colidx[p];
                    if (cnt[c]++ == 0) touched.push_back(c);
                }
            }
            mcols.clear();
            for (int32_t c : touched)
                if ((int64_t)cnt[c] > col_thr) mcols.push_back(c);
            std::sort(mcols.begin(), mcols.end());
            kept_chunks.clear();
            for (size_t j0 = 0; j0 < mcols.size(); j0 += kt) {
                size_t nc = std::min<size_t>(kt, mcols.size() - j0);
                int64_t tnnz = 0;
                for (size_t j = 0; j < nc; ++j) tnnz += cnt[mcols[j0 + j]];
                if ((double)tnnz >= keep_thr) kept_chunks.push_back({(int64_t)j0, (int64_t)nc});
            }
            for (int32_t c : touched) cnt[c] = 0;
            if (kept_chunks.empty()) continue;  // dissolved: rows stay vector rows

            out.windows.insert(out.windows.end(), slots.begin(), slots.end());
            const size_t nkt = kept_chunks.size();
            out.win_ntiles.push_back((int32_t)nkt);
            for (size_t t = 0; t < nkt; ++t)
                for (int64_t j = 0; j < kept_chunks[t].second; ++j)
                    pos[mcols[kept_chunks[t].first + j]] = (int32_t)(t * kt + j);
            src.assign(nkt * H * kt, -1);
            for (int s = 0; s < H; ++s) {
                int32_t r = slots[s];
                if (r < 0) continue;
                for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
                    int32_t q = pos[colidx[p]];
                    if (q < 0) continue;
                    int64_t t = q / kt, j = q % kt;
                    int64_t &slot = src[(t * H + s) * kt + j];
                    if (slot < 0) { slot = p; in_tile[p] = 1; }  // first occurrence only
                }
            }
            for (size_t t = 0; t < nkt; ++t) {
                for (int j = 0; j < kt; ++j)
                    out.tile_cols.push_back(j < kept_chunks[t].second ? mcols[kept_chunks[t].first + j] : -1);
                const size_t v0 = out.tile_src.size();
                for (int s = 0; s < H; ++s) {
                    uint32_t word = 0;
                    for (int j = 0; j < kt; ++j) {
                        int64_t p = src[(t * H + s) * kt + j];
                        if (p < 0) continue;
                        word |= 1u << j;
                        out.tile_src.push_back(p);
                        uint16_t bits;
                        if (A->val_type == SPMM_F32) {
                            float f;
                            std::memcpy(&f, vbytes + p * 4, 4);
                            bits = f32_to_bf16_rne(f);
                        } else {
                            std::memcpy(&bits, vbytes + p * 2, 2);
                        }
                        out.tile_vals.push_back(bits);
                    }
                    out.tile_bitmap.push_back(word);
                }
                out.tile_nval.push_back((int64_t)(out.tile_src.size() - v0));
            }
            for (size_t t = 0; t < nkt; ++t)
                for (int64_t j = 0; j < kept_chunks[t].second; ++j)
                    pos[mcols[kept_chunks[t].first + j]] = -1;
        }
    };
    {
        // threads: only for many windows, and bounded by the 8 bytes per
        // column that each one's counters take; SPMM_PLAN_THREADS sets the
        // count (tests use it to compare plans built with different counts)
        const size_t nc = cand.size();
        size_t nth = std::max<size_t>(1, std::min<size_t>(std::thread::hardware_concurrency(), 16));
        nth = std::min(nth, std::max<size_t>(1, nc / 512));
        if (const char *env = std::getenv("SPMM_PLAN_THREADS")) {
            const long v = std::strtol(env, nullptr, 10);
            if (v >= 1) nth = (size_t)std::min<long>(v, 64);
        }
        nth = std::min(nth, std::max<size_t>(1, nc));
        nth = std::min(nth, std::max<size_t>(1, (size_t(1) << 30) / (8 * (size_t)std::max<int64_t>(k, 1))));
        std::vector<StageOut> outs(nth);
        if (nth == 1) {
            stage(0, nc, outs[0]);
        } else {
            std::vector<std::thread> th;
            for (size_t i = 0; i < nth; ++i)
                th.emplace_back(stage, nc * i / nth, nc * (i + 1) / nth, std::ref(outs[i]));
            for (auto &t : th) t.join();
        }
        P.tile_val_ptr.push_back(0);
        P.win_tile_ptr.push_back(0);
        for (StageOut &out : outs) {
            size_t t = 0;
            for (int32_t ntiles : out.win_ntiles) {
                const int32_t widx = (int32_t)(P.win_tile_ptr.size() - 1);
                for (int32_t i = 0; i < ntiles; ++i, ++t) {
                    P.tile_window.push_back(widx);
                    P.tile_val_ptr.push_back(P.tile_val_ptr.back() + out.tile_nval[t]);
                }
                P.win_tile_ptr.push_back((int32_t)P.tile_window.size());
            }
            P.windows.insert(P.windows.end(), out.windows.begin(), out.windows.end());
            P.tile_cols.insert(P.tile_cols.end(), out.tile_cols.begin(), out.tile_cols.end());
            P.tile_bitmap.insert(P.tile_bitmap.end(), out.tile_bitmap.begin(), out.tile_bitmap.end());
            P.tile_vals.insert(P.tile_vals.end(), out.tile_vals.begin(), out.tile_vals.end());
            P.tile_src.insert(P.tile_src.end(), out.tile_src.begin(), out.tile_src.end());
            out = StageOut();
        }
    }

    // ---- remainder (CSR order per row) ----
    // Row ranges run on threads: each counts its rows' remainder entries, a
    // prefix over the ranges places them, and each copies its runs of
    // consecutive non-tile entries in bulk.
    size_t nth_rows = nnz < (int64_t)(1 << 20)
                          ? 1
                          : std::max<size_t>(1, std::min<size_t>(std::thread::hardware_concurrency(), 16));
    if (const char *env = std::getenv("SPMM_PLAN_THREADS")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v >= 1) nth_rows = (size_t)std::min<long>(v, 64);
    }
    // body(r0, r1, range index) over `nth` contiguous row ranges
    auto parallel_rows = [&](size_t nth, auto &&body) {
        if (nth == 1 || m < 2) {
            body((int64_t)0, m, (size_t)0);
            return;
        }
        std::vector<std::thread> th;
        for (size_t i = 0; i < nth; ++i)
            th.emplace_back([&, i] { body(m * (int64_t)i / (int64_t)nth, m * (int64_t)(i + 1) / (int64_t)nth, i); });
        for (auto &t : th) t.join();
    };
    P.rem_ptr.assign(m + 1, 0);
    P.rem_ptr32.assign(m + 1, 0);
    std::vector<int64_t> range_base(nth_rows + 1, 0);
    parallel_rows(nth_rows, [&](int64_t r0, int64_t r1, size_t i) {
        int64_t c = 0;
        for (int64_t r = r0; r < r1; ++r) {
            for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) c += !in_tile[p];
            P.rem_ptr[r + 1] = c;  // local prefix, made global below
        }
        range_base[i + 1] = c;
    });
    for (size_t i = 0; i < nth_rows; ++i) range_base[i + 1] += range_base[i];
    const int64_t nrem = range_base[nth_rows];
    P.rem_src.resize(nrem);
    P.rem_col.resize(nrem);
    P.rem_val.resize((size_t)nrem * sval);
    parallel_rows(nth_rows, [&](int64_t r0, int64_t r1, size_t i) {
        const int64_t base = range_base[i];
        int64_t at = base;
        for (int64_t r = r0; r < r1; ++r) {
            int64_t p = rowptr[r];
            const int64_t pe = rowptr[r + 1];
            while (p < pe) {
                if (in_tile[p]) { ++p; continue; }
                int64_t q = p + 1;
                while (q < pe && !in_tile[q]) ++q;
                for (int64_t x = p; x < q; ++x) P.rem_src[at + (x - p)] = x;
                std::memcpy(P.rem_col.data() + at, colidx + p, (size_t)(q - p) * 4);
                std::memcpy(P.rem_val.data() + (size_t)at * sval, vbytes + p * sval, (size_t)(q - p) * sval);
                at += q - p;
                p = q;
            }
            P.rem_ptr[r + 1] += base;
            P.rem_ptr32[r + 1] = (int32_t)P.rem_ptr[r + 1];
        }
    });

    // ---- hot columns: the most-gathered B rows of the vector path (ties: lower id) ----
    if (o.hot_cols > 0 && !P.rem_col.empty()) {
        std::vector<int32_t> gcount(k, 0);
        std::vector<int32_t> used;
        for (int32_t c : P.rem_col)
            if (gcount[c]++ == 0) used.push_back(c);
        auto hotter = [&](int32_t a, int32_t b) {
            return gcount[a] != gcount[b] ? gcount[a] > gcount[b] : a < b;
        };
        size_t nh = std::min<size_t>((size_t)o.hot_cols, used.size());
        if (nh < used.size())
            std::nth_element(used.begin(), used.begin() + nh, used.end(), hotter);
        std::vector<uint8_t> hot(k, 0);
        for (size_t i = 0; i < nh; ++i) hot[used[i]] = 1;
        for (auto &c : P.rem_col)
            if (hot[c]) c = (int32_t)((uint32_t)c | 0x80000000u);
        P.hot_cols = (int64_t)nh;
    }

    // ---- distinct referenced columns (per-range bitmaps, then their union) ----
    {
        const size_t words = (size_t)(k + 63) / 64;
        // one bitmap of k bits per thread, at most 1 GiB of them in all
        const size_t nth_k = std::min(nth_rows, std::max<size_t>(1, (size_t(1) << 30) / (8 * words + 8)));
        std::vector<std::vector<uint64_t>> seen(nth_k, std::vector<uint64_t>(words, 0));
        parallel_rows(nth_k, [&](int64_t r0, int64_t r1, size_t i) {
            std::vector<uint64_t> &b = seen[i];
            for (int64_t p = rowptr[r0]; p < rowptr[r1]; ++p) {
                const uint32_t c = (uint32_t)colidx[p];
                b[c >> 6] |= uint64_t(1) << (c & 63);
            }
        });
        int64_t kr = 0;
        for (size_t w = 0; w < words; ++w) {
            uint64_t x = 0;
            for (size_t i = 0; i < nth_k; ++i) x |= seen[i][w];
            kr += __builtin_popcountll(x);
        }
        P.k_ref = kr;
    }

    build_schedule(P);

    derive_exec_tables(P);

    auto t_end = std::chrono::steady_clock::now();
    P.plan_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    return SPMM_OK;
}

void derive_exec_tables(HostPlan &P) {
    const int64_t W = (int64_t)P.win_seg.size(), H = P.opts.window_h;
    P.seg_win.clear();
    P.win_dep.assign(W, -1);
    P.win_nsseg.assign(W, 0);
    P.win_row_sid.assign(W * H, -1);
    P.n_dep = 0;
    if (W == 0) return;
    P.seg_win.assign(P.seg_row.size(), -1);
    for (int64_t w = 0; w < W; ++w) {
        int32_t ns = 0;
        for (int64_t s = 0; s < H; ++s) {
            const int32_t r = P.windows[w * H + s];
            if (r < 0 || P.nseg[r] == 0) continue;
            P.win_row_sid[w * H + s] = P.win_seg[w] + ns;
            ns += P.nseg[r];
        }
        // a window's segments are consecutive ids from win_seg[w], in slot order
        for (int32_t j = 0; j < ns; ++j) P.seg_win[(size_t)P.win_seg[w] + j] = (int32_t)w;
        P.win_nsseg[w] = ns;
        if (ns > 0 || P.win_part[w + 1] > P.win_part[w]) P.win_dep[w] = P.n_dep++;
    }
}

void plan_path_work(const HostPlan &P, double *w_vec, double *w_tile, double *w_winrem) {
    double v = 0, wr = 0;
    for (size_t i = 0; i < P.seg_row.size(); ++i) v += (double)(P.seg_end[i] - P.seg_begin[i]);
    for (int32_t r : P.vector_rows)
        if (!P.nseg[r]) v += (double)(P.rem_ptr[r + 1] - P.rem_ptr[r]);
    for (int32_t r : P.windows)
        if (r >= 0 && !P.nseg[r]) wr += (double)(P.rem_ptr[r + 1] - P.rem_ptr[r]);
    *w_vec = v;
    *w_tile = (double)P.tile_window.size() * P.opts.window_h * P.opts.kt;
    *w_winrem = wr;
}

}  // namespace spmm
