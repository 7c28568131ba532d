// Host-only driver for the planner, built with AddressSanitizer and UBSan by
// tests/test_plan_sanitizers.py.  Builds plans of seeded random CSR matrices
// under every mode / window height / row order and checks the partition's
// invariants: every entry placed exactly once, every row owned exactly once,
// segment ids consecutive in item order.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace spmm;

static int fail(const char *what, int seed) {
    std::fprintf(stderr, "invariant failed: %s (seed %d)\n", what, seed);
    return 1;
}

int main(int argc, char **argv) {
    const int cases = argc > 1 ? std::atoi(argv[1]) : 200;
    for (int seed = 0; seed < cases; ++seed) {
        std::mt19937_64 rng(seed);
        const int64_t m = rng() % 300, k = 1 + rng() % 400;
        const double dens = (rng() % 1000) / 4000.0;
        std::vector<int64_t> rowptr(m + 1, 0);
        std::vector<int32_t> col;
        for (int64_t r = 0; r < m; ++r) {
            int64_t len = (rng() % 7 == 0) ? (int64_t)(rng() % (k * 2)) : (int64_t)(dens * k * (rng() % 100) / 50.0);
            for (int64_t i = 0; i < len; ++i) col.push_back((int32_t)(rng() % k));  // duplicates allowed
            rowptr[r + 1] = (int64_t)col.size();
        }
        const int vt = (int)(rng() % 3);
        std::vector<uint16_t> v16(col.size());
        std::vector<float> v32(col.size());
        for (size_t i = 0; i < col.size(); ++i) {
            v32[i] = (float)((int)(rng() % 9) - 4);
            v16[i] = (uint16_t)(rng() & 0x7BFF);
        }
        spmm_csr A{m, k, (int64_t)col.size(), rowptr.data(), col.data(),
                   vt == SPMM_F32 ? (const void *)v32.data() : (const void *)v16.data(), vt, 0};
        const int bt = vt == SPMM_F16 ? SPMM_F16 : (vt == SPMM_BF16 ? SPMM_BF16 : (int)(rng() % 2));
        spmm_opts o;
        spmm_opts_default(&o);
        o.mode = 1 + (int)(rng() % 3);
        const int hs[3] = {16, 32, 64};
        o.window_h = hs[rng() % 3];
        o.row_order = 1 + (int)(rng() % 3);
        o.t_row = (int)(rng() % 6) - 1;
        o.alpha_c = (float)((rng() % 4) / (double)o.window_h);
        o.alpha = (float)((rng() % 5) / 20.0);
        o.seg_len = 1 + (int)(rng() % 40);
        o.item_cost = 1 + (int)(rng() % 60);
        o.hot_cols = (int)(rng() % 50);
        const int n = 1 + (int)(rng() % 300);
        spmm_opts r;
        resolve_options(&o, &A, n, bt, &r);
        HostPlan P;
        std::string err;
        spmm_status st = build_host_plan(&A, n, bt, SPMM_F32, r, P, err);
        if (st != SPMM_OK) return fail(err.c_str(), seed);
        // every entry exactly once
        std::vector<int> cnt(A.nnz, 0);
        for (int64_t p : P.tile_src) cnt[p]++;
        for (int64_t p : P.rem_src) cnt[p]++;
        for (int c : cnt)
            if (c != 1) return fail("entry coverage", seed);
        // every row owned exactly once
        std::vector<int> own(m, 0);
        for (int32_t x : P.vector_rows) own[x]++;
        for (int32_t x : P.windows)
            if (x >= 0) own[x]++;
        for (int c : own)
            if (c != 1) return fail("row ownership", seed);
        // segments consecutive in item order, then window order
        size_t sid = 0;
        for (size_t it = 0; it + 1 < P.vitem_ptr.size(); ++it) {
            if (P.vitem_seg[it] != (int32_t)sid) return fail("vitem_seg", seed);
            for (int32_t i = P.vitem_ptr[it]; i < P.vitem_ptr[it + 1]; ++i) sid += P.nseg[P.vector_rows[i]];
        }
        const int64_t W = (int64_t)P.windows.size() / r.window_h;
        for (int64_t w = 0; w < W; ++w) {
            if (P.win_seg[w] != (int32_t)sid) return fail("win_seg", seed);
            for (int s = 0; s < r.window_h; ++s) {
                int32_t x = P.windows[w * r.window_h + s];
                if (x >= 0) sid += P.nseg[x];
            }
            if (P.win_tile_ptr[w + 1] <= P.win_tile_ptr[w]) return fail("window without tile", seed);
        }
        if (sid != P.seg_row.size()) return fail("segment count", seed);
        if ((int64_t)P.win_part.size() != W + 1 || (size_t)P.win_part[W] != P.wpart_win.size())
            return fail("window partials", seed);
    }
    std::printf("ok %d cases\n", cases);
    return 0;
}
