// serialize.cpp -- plan images: write every HostPlan array, read one back and
// check the invariants the kernels index by (host only, no device calls).
//
// Layout: "SPMMPLAN", u32 version, u32 sizeof(spmm_opts), the problem scalars
// and the resolved options, then each array as (u64 element count, raw
// elements) in a fixed order, then a 64-bit FNV-1a checksum of everything
// before it.  Little-endian, as the host that writes and the host that reads.
#include <cstring>

#include "plan.hpp"

namespace spmm {
namespace {

constexpr char kMagic[8] = {'S', 'P', 'M', 'M', 'P', 'L', 'A', 'N'};
constexpr uint32_t kVersion = 1;

uint64_t fnv1a(const uint8_t *p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Writer {
    std::vector<uint8_t> &out;
    template <class T>
    void pod(const T &v) {
        const uint8_t *b = reinterpret_cast<const uint8_t *>(&v);
        out.insert(out.end(), b, b + sizeof(T));
    }
    template <class T>
    void vec(const std::vector<T> &v) {
        pod<uint64_t>(v.size());
        const uint8_t *b = reinterpret_cast<const uint8_t *>(v.data());
        out.insert(out.end(), b, b + v.size() * sizeof(T));
    }
};

struct Reader {
    const uint8_t *p;
    size_t n, at = 0;
    bool ok = true;
    template <class T>
    void pod(T &v) {
        if (!ok || n - at < sizeof(T)) { ok = false; return; }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
    }
    template <class T>
    void vec(std::vector<T> &v) {
        uint64_t c = 0;
        pod(c);
        if (!ok || c > (n - at) / sizeof(T)) { ok = false; return; }
        v.resize((size_t)c);
        std::memcpy(v.data(), p + at, (size_t)c * sizeof(T));
        at += (size_t)c * sizeof(T);
    }
};

template <class F>
void each_array(HostPlan &P, F &&f) {
    f(P.windows); f(P.tile_window); f(P.tile_cols); f(P.tile_bitmap); f(P.tile_val_ptr);
    f(P.tile_vals); f(P.tile_src); f(P.rem_ptr); f(P.rem_src); f(P.vector_rows); f(P.nseg);
    f(P.vexec); f(P.vitem_ptr); f(P.vitem_seg); f(P.seg_row); f(P.seg_begin); f(P.seg_end);
    f(P.win_tile_ptr); f(P.win_seg); f(P.win_order); f(P.win_part); f(P.wpart_win);
    f(P.wpart_t0); f(P.wpart_t1); f(P.rem_ptr32); f(P.rem_col); f(P.rem_val);
}

#define SPMM_CHECK(cond, msg)        \
    do {                             \
        if (!(cond)) {               \
            err = msg;               \
            return SPMM_ERR_INVALID; \
        }                            \
    } while (0)

template <class T>
bool monotone_from_zero(const std::vector<T> &v, int64_t last) {
    if (v.empty() || v[0] != 0 || (int64_t)v.back() != last) return false;
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i] < v[i - 1]) return false;
    return true;
}

spmm_status check_plan(const HostPlan &P, std::string &err, int32_t *win_tiles) {
    SPMM_CHECK(P.m >= 0 && P.k >= 0 && P.nnz >= 0 && P.m < INT32_MAX && P.k < INT32_MAX &&
                   P.nnz < INT32_MAX && P.n >= 1,
               "plan image: sizes");
    SPMM_CHECK(P.c_type == SPMM_F32 && P.val_type >= 0 && P.val_type <= 2 && P.b_type >= 0 &&
                   P.b_type <= 2 && (P.tile_type == SPMM_BF16 || P.tile_type == SPMM_F16),
               "plan image: types");
    spmm_status st = validate_opts(P.opts, err);
    if (st != SPMM_OK) return SPMM_ERR_INVALID;
    const int64_t m = P.m, k = P.k, H = P.opts.window_h, kt = P.opts.kt, S = P.opts.seg_len;
    const int sval = dtype_size(P.val_type);
    // remainder (CSR of the entries the vector path gathers)
    SPMM_CHECK((int64_t)P.rem_ptr.size() == m + 1 && monotone_from_zero(P.rem_ptr, (int64_t)P.rem_col.size()),
               "plan image: remainder row pointers");
    SPMM_CHECK(P.rem_ptr32.size() == P.rem_ptr.size(), "plan image: remainder row pointers");
    for (size_t i = 0; i < P.rem_ptr.size(); ++i)
        SPMM_CHECK(P.rem_ptr32[i] == P.rem_ptr[i], "plan image: remainder row pointers");
    for (int32_t c : P.rem_col) SPMM_CHECK((c & 0x7FFFFFFF) < k, "plan image: remainder column");
    SPMM_CHECK(P.rem_val.size() == P.rem_col.size() * (size_t)sval, "plan image: remainder values");
    SPMM_CHECK(P.rem_src.size() == P.rem_col.size(), "plan image: remainder sources");
    for (int64_t e : P.rem_src) SPMM_CHECK(e >= 0 && e < P.nnz, "plan image: remainder source");
    SPMM_CHECK((int64_t)P.nseg.size() == m, "plan image: segment counts");
    for (int64_t r = 0; r < m; ++r) {
        const int64_t L = P.rem_ptr[r + 1] - P.rem_ptr[r];
        SPMM_CHECK(P.nseg[r] == (L > S ? (L + S - 1) / S : 0), "plan image: segment counts");
    }
    // windows and tiles
    SPMM_CHECK((int64_t)P.windows.size() % H == 0, "plan image: windows");
    const int64_t W = (int64_t)P.windows.size() / H;
    std::vector<uint8_t> in_window(m, 0);
    for (int32_t r : P.windows) {
        SPMM_CHECK(r >= -1 && r < m, "plan image: window row");
        if (r >= 0) {
            SPMM_CHECK(!in_window[r], "plan image: row in two windows");
            in_window[r] = 1;
        }
    }
    const int64_t T = (int64_t)P.tile_window.size();
    SPMM_CHECK((int64_t)P.win_tile_ptr.size() == W + 1 && monotone_from_zero(P.win_tile_ptr, T),
               "plan image: window tiles");
    for (int64_t w = 0; w < W; ++w) {
        // the window kernel takes its rows' metadata in its first tile round
        SPMM_CHECK(P.win_tile_ptr[w + 1] > P.win_tile_ptr[w], "plan image: window without tiles");
        for (int32_t t = P.win_tile_ptr[w]; t < P.win_tile_ptr[w + 1]; ++t)
            SPMM_CHECK(P.tile_window[t] == w, "plan image: tile window");
    }
    SPMM_CHECK((int64_t)P.tile_cols.size() == T * kt && (int64_t)P.tile_bitmap.size() == T * H,
               "plan image: tile arrays");
    for (int32_t c : P.tile_cols) SPMM_CHECK(c >= -1 && c < k, "plan image: tile column");
    SPMM_CHECK((int64_t)P.tile_val_ptr.size() == T + 1 &&
                   monotone_from_zero(P.tile_val_ptr, (int64_t)P.tile_vals.size()),
               "plan image: tile values");
    SPMM_CHECK(P.tile_src.size() == P.tile_vals.size(), "plan image: tile sources");
    for (int64_t e : P.tile_src) SPMM_CHECK(e >= 0 && e < P.nnz, "plan image: tile source");
    for (int64_t t = 0; t < T; ++t) {
        int64_t bits = 0;
        const int64_t w = P.tile_window[t];
        for (int64_t s = 0; s < H; ++s) {
            const uint32_t b = P.tile_bitmap[t * H + s];
            SPMM_CHECK(kt >= 32 || (b >> kt) == 0, "plan image: bitmap");
            if (P.windows[w * H + s] < 0) SPMM_CHECK(b == 0, "plan image: bitmap of an empty slot");
            for (int64_t j = 0; j < kt; ++j)
                if ((b >> j) & 1u) SPMM_CHECK(P.tile_cols[t * kt + j] >= 0, "plan image: bitmap column");
            bits += __builtin_popcount(b);
        }
        SPMM_CHECK(bits == P.tile_val_ptr[t + 1] - P.tile_val_ptr[t], "plan image: tile value count");
        // the window kernel reads a round's values at clamped indices
        SPMM_CHECK(bits > 0, "plan image: tile without values");
    }
    // vector rows and items
    for (size_t i = 0; i < P.vector_rows.size(); ++i) {
        const int32_t r = P.vector_rows[i];
        SPMM_CHECK(r >= 0 && r < m && (i == 0 || r > P.vector_rows[i - 1]) && !in_window[r],
                   "plan image: vector rows");
    }
    SPMM_CHECK((int64_t)P.vector_rows.size() + [&] {
        int64_t c = 0;
        for (uint8_t x : in_window) c += x;
        return c;
    }() == m, "plan image: rows not covered");
    const int64_t nv = (int64_t)P.vector_rows.size();
    SPMM_CHECK(P.vexec.empty() || (int64_t)P.vexec.size() == nv, "plan image: launch order");
    const std::vector<int32_t> &order = P.vexec.empty() ? P.vector_rows : P.vexec;
    const int64_t V = (int64_t)P.vitem_ptr.size() - 1;
    SPMM_CHECK(V >= 0 && monotone_from_zero(P.vitem_ptr, nv), "plan image: vector items");
    for (int64_t i = 0; i < V; ++i)
        SPMM_CHECK(P.vitem_ptr[i + 1] > P.vitem_ptr[i], "plan image: empty vector item");
    SPMM_CHECK((int64_t)P.vitem_seg.size() == V, "plan image: item segment ids");
    // segments: items in launch order, then windows in slot order
    const int64_t NS = (int64_t)P.seg_row.size();
    SPMM_CHECK((int64_t)P.seg_begin.size() == NS && (int64_t)P.seg_end.size() == NS,
               "plan image: segments");
    int64_t sid = 0;
    auto walk_row = [&](int32_t r) -> bool {
        for (int32_t j = 0; j < P.nseg[r]; ++j, ++sid) {
            if (sid >= NS || P.seg_row[sid] != r) return false;
            const int64_t b = P.rem_ptr[r] + (int64_t)j * S, e = std::min(b + S, P.rem_ptr[r + 1]);
            if (P.seg_begin[sid] != b || P.seg_end[sid] != e) return false;
        }
        return true;
    };
    {
        std::vector<uint8_t> seen(m, 0);
        for (int64_t i = 0; i < V; ++i) {
            SPMM_CHECK(P.vitem_seg[i] == sid, "plan image: item segment ids");
            for (int32_t q = P.vitem_ptr[i]; q < P.vitem_ptr[i + 1]; ++q) {
                const int32_t r = order[q];
                SPMM_CHECK(r >= 0 && r < m && !in_window[r] && !seen[r], "plan image: launch order");
                seen[r] = 1;
                SPMM_CHECK(walk_row(r), "plan image: segments");
            }
        }
    }
    SPMM_CHECK((int64_t)P.win_seg.size() == W, "plan image: window segment ids");
    for (int64_t w = 0; w < W; ++w) {
        SPMM_CHECK(P.win_seg[w] == sid, "plan image: window segment ids");
        for (int64_t s = 0; s < H; ++s) {
            const int32_t r = P.windows[w * H + s];
            if (r >= 0) SPMM_CHECK(walk_row(r), "plan image: segments");
        }
    }
    SPMM_CHECK(sid == NS, "plan image: segments");
    // window launch order and partial items
    SPMM_CHECK((int64_t)P.win_order.size() == W, "plan image: window order");
    {
        std::vector<uint8_t> seen(W, 0);
        for (int32_t w : P.win_order) {
            SPMM_CHECK(w >= 0 && w < W && !seen[w], "plan image: window order");
            seen[w] = 1;
        }
    }
    const int64_t NP = (int64_t)P.wpart_win.size();
    SPMM_CHECK((int64_t)P.wpart_t0.size() == NP && (int64_t)P.wpart_t1.size() == NP,
               "plan image: window partial items");
    SPMM_CHECK((int64_t)P.win_part.size() == W + 1 && monotone_from_zero(P.win_part, NP),
               "plan image: window partial items");
    // tiles per window item: the first partial item's offset in its window,
    // else (no partial item) enough for the largest window
    int64_t K = kWinTiles;
    if (NP > 0) {
        const int32_t w0 = P.wpart_win[0];
        SPMM_CHECK(w0 >= 0 && w0 < W, "plan image: window partial items");
        K = (int64_t)P.wpart_t0[0] - P.win_tile_ptr[w0];
        SPMM_CHECK(K >= kWinTiles && K <= kWinTilesMax && (K & (K - 1)) == 0, "plan image: window partial items");
    } else {
        for (int64_t w = 0; w < W; ++w) K = std::max<int64_t>(K, (int64_t)P.win_tile_ptr[w + 1] - P.win_tile_ptr[w]);
    }
    *win_tiles = (int32_t)std::min<int64_t>(K, INT32_MAX);
    for (int64_t w = 0; w < W; ++w)
        for (int32_t q = P.win_part[w]; q < P.win_part[w + 1]; ++q)
            SPMM_CHECK(P.wpart_win[q] == w && P.wpart_t0[q] >= P.win_tile_ptr[w] + K &&
                           P.wpart_t0[q] < P.wpart_t1[q] && P.wpart_t1[q] <= P.win_tile_ptr[w + 1] &&
                           P.wpart_t1[q] - P.wpart_t0[q] <= K,
                       "plan image: window partial items");
    for (int64_t w = 0; w < W; ++w) {
        // tiles beyond an owner's first K are exactly covered by its partial items
        int64_t t = P.win_tile_ptr[w] + K;
        for (int32_t q = P.win_part[w]; q < P.win_part[w + 1]; ++q) {
            SPMM_CHECK(P.wpart_t0[q] == t, "plan image: window partial items");
            t = P.wpart_t1[q];
        }
        SPMM_CHECK(t >= P.win_tile_ptr[w + 1], "plan image: window partial items");
    }
    SPMM_CHECK(P.k_ref >= 0 && P.k_ref <= k && P.hot_cols >= 0, "plan image: statistics");
    return SPMM_OK;
}

}  // namespace

void serialize_host_plan(const HostPlan &P, std::vector<uint8_t> &out) {
    out.clear();
    Writer w{out};
    out.insert(out.end(), kMagic, kMagic + 8);
    w.pod(kVersion);
    w.pod<uint32_t>((uint32_t)sizeof(spmm_opts));
    w.pod(P.m); w.pod(P.k); w.pod(P.nnz); w.pod(P.n);
    w.pod(P.val_type); w.pod(P.b_type); w.pod(P.c_type); w.pod(P.tile_type);
    w.pod(P.opts);
    w.pod<uint32_t>(P.identity_rows ? 1u : 0u);
    w.pod(P.k_ref); w.pod(P.hot_cols); w.pod(P.plan_ms);
    each_array(const_cast<HostPlan &>(P), [&](auto &v) { w.vec(v); });
    w.pod(fnv1a(out.data(), out.size()));
}

spmm_status deserialize_host_plan(const uint8_t *buf, size_t size, HostPlan &P, std::string &err) {
    if (!buf || size < 8 + 8 + 8 || std::memcmp(buf, kMagic, 8) != 0) {
        err = "not a plan image";
        return SPMM_ERR_INVALID;
    }
    uint64_t sum = 0;
    std::memcpy(&sum, buf + size - 8, 8);
    if (fnv1a(buf, size - 8) != sum) {
        err = "plan image: checksum";
        return SPMM_ERR_INVALID;
    }
    Reader r{buf, size - 8};
    r.at = 8;
    uint32_t version = 0, opts_size = 0, ident = 0;
    r.pod(version);
    r.pod(opts_size);
    if (!r.ok || version != kVersion || opts_size != sizeof(spmm_opts)) {
        err = "plan image: version";
        return SPMM_ERR_UNSUPPORTED;
    }
    HostPlan Q;
    r.pod(Q.m); r.pod(Q.k); r.pod(Q.nnz); r.pod(Q.n);
    r.pod(Q.val_type); r.pod(Q.b_type); r.pod(Q.c_type); r.pod(Q.tile_type);
    r.pod(Q.opts);
    r.pod(ident);
    r.pod(Q.k_ref); r.pod(Q.hot_cols); r.pod(Q.plan_ms);
    each_array(Q, [&](auto &v) { r.vec(v); });
    if (!r.ok || r.at != size - 8) {
        err = "plan image: truncated or trailing bytes";
        return SPMM_ERR_INVALID;
    }
    Q.identity_rows = ident != 0;
    int32_t win_tiles = kWinTiles;
    spmm_status st = check_plan(Q, err, &win_tiles);
    if (st != SPMM_OK) return st;
    Q.win_tiles = win_tiles;
    if (Q.identity_rows != ((int64_t)Q.vector_rows.size() == Q.m)) {
        err = "plan image: identity flag";
        return SPMM_ERR_INVALID;
    }
    derive_exec_tables(Q);
    P = std::move(Q);
    return SPMM_OK;
}

}  // namespace spmm
