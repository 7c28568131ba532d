// autotune.hip -- sparsity-profile keys, the tuned-options cache and the
// measurement-driven search over plan options.
//
// The cost model of NeutronSparse Sec. 5.2.1 (Eq. 1-3) gives the density
// threshold alpha = r * P_vec / P_mfma from a dry run; on CDNA4 r = 1 (one
// engine pool, a cost crossover rather than balanced co-running).  The paper
// then tunes the tile shape (Sec. 6.2.2) and shows the threshold's
// sensitivity (Sec. 8.2); here the remaining knobs are chosen by timing
// candidate plans on the device, staged so that each stage varies one group
// of options around the best plan so far.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "devplan.hpp"
#include "plan.hpp"
#include "runtime.hpp"

using namespace spmm;

namespace {

std::mutex g_cache_mu;
std::map<std::string, spmm_opts> g_cache;
std::map<std::pair<int32_t, int32_t>, std::pair<double, double>> g_dryrun;  // (n, b_type)

std::string opts_to_text(const spmm_opts &o) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %d %d %d %.9g %.9g %d %d %d", o.mode,
                  o.window_h, o.t_row, o.kt, o.n_panel, o.row_order, o.seg_len, o.item_cost,
                  o.xcd_remap, o.hot_cols, (double)o.alpha_c, (double)o.alpha, o.cold_policy,
                  o.pipeline, o.win_sched);
    return buf;
}

bool opts_from_text(const std::string &t, spmm_opts *o) {
    spmm_opts_default(o);
    double ac = 0, al = 0;
    int n = std::sscanf(t.c_str(), "%d %d %d %d %d %d %d %d %d %d %lg %lg %d %d %d", &o->mode,
                        &o->window_h, &o->t_row, &o->kt, &o->n_panel, &o->row_order, &o->seg_len,
                        &o->item_cost, &o->xcd_remap, &o->hot_cols, &ac, &al, &o->cold_policy,
                        &o->pipeline, &o->win_sched);
    o->alpha_c = (float)ac;
    o->alpha = (float)al;
    return n == 15;
}

int ilog2_floor(int64_t x) {
    int l = 0;
    while (x > 1) { x >>= 1; ++l; }
    return l;
}

}  // namespace

namespace spmm {

std::string profile_key(const spmm_csr *A, int32_t n, int32_t b_type) {
    const int64_t m = A->m, k = A->k, nnz = A->nnz;
    // log2 row-length histogram of the entries, tenths
    double hist[32] = {0};
    for (int64_t r = 0; r < m; ++r) {
        const int64_t len = A->rowptr[r + 1] - A->rowptr[r];
        if (len > 0) hist[std::min(31, ilog2_floor(len))] += (double)len;
    }
    // share of entries whose column repeats inside their 16-row window, on a
    // sample of up to 256 evenly spaced windows
    const int64_t nwin = (m + 15) / 16;
    const int64_t step = std::max<int64_t>(1, nwin / 256);
    int64_t seen = 0, shared = 0;
    std::map<int32_t, int> cnt;
    for (int64_t w = 0; w < nwin; w += step) {
        cnt.clear();
        const int64_t r0 = w * 16, r1 = std::min(m, r0 + 16);
        for (int64_t p = A->rowptr[r0]; p < A->rowptr[r1]; ++p) cnt[A->colidx[p]]++;
        for (auto &kv : cnt) {
            seen += kv.second;
            if (kv.second >= 2) shared += kv.second;
        }
    }
    std::ostringstream os;
    os << "m" << ilog2_floor(std::max<int64_t>(m, 1)) << " k" << ilog2_floor(std::max<int64_t>(k, 1))
       << " z" << ilog2_floor(std::max<int64_t>(nnz, 1)) << " n" << n << " v" << A->val_type << " b"
       << b_type << " h";
    for (int i = 0; i < 20; ++i)
        os << (nnz ? (int)std::lround(10.0 * hist[i] / (double)nnz) : 0)
           << (i + 1 < 20 ? "," : "");
    os << " w" << (seen ? (int)std::lround(10.0 * (double)shared / (double)seen) : 0);
    return os.str();
}

bool cache_lookup(const std::string &key, spmm_opts *o) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *o = it->second;
    return true;
}

}  // namespace spmm

extern "C" spmm_status spmm_profile_key(const spmm_csr *A, int32_t n, int32_t b_type, char *buf,
                                        int32_t cap) {
    std::string err;
    spmm_status st = validate_problem(A, n, b_type, SPMM_F32, err);
    if (st != SPMM_OK) return set_error(st, err);
    if (!buf) return set_error(SPMM_ERR_INVALID, "buf is null");
    const std::string key = profile_key(A, n, b_type);
    if ((int64_t)key.size() + 1 > cap) return set_error(SPMM_ERR_INVALID, "buffer too small");
    std::memcpy(buf, key.c_str(), key.size() + 1);
    return SPMM_OK;
}

extern "C" spmm_status spmm_tune_cache_put(const char *key, const spmm_opts *o) {
    if (!key || !o) return set_error(SPMM_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = *o;
    return SPMM_OK;
}

extern "C" spmm_status spmm_tune_cache_get(const char *key, spmm_opts *o, int32_t *found) {
    if (!key || !o || !found) return set_error(SPMM_ERR_INVALID, "null argument");
    *found = cache_lookup(key, o) ? 1 : 0;
    return SPMM_OK;
}

extern "C" spmm_status spmm_tune_cache_save(const char *path) {
    if (!path) return set_error(SPMM_ERR_INVALID, "path is null");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ofstream f(path);
    if (!f) return set_error(SPMM_ERR_INVALID, std::string("cannot write ") + path);
    for (auto &kv : g_cache) f << kv.first << '\t' << opts_to_text(kv.second) << '\n';
    return f ? SPMM_OK : set_error(SPMM_ERR_INVALID, "write failed");
}

extern "C" spmm_status spmm_tune_cache_load(const char *path) {
    if (!path) return set_error(SPMM_ERR_INVALID, "path is null");
    std::ifstream f(path);
    if (!f) return set_error(SPMM_ERR_INVALID, std::string("cannot read ") + path);
    std::string line;
    std::map<std::string, spmm_opts> add;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos) continue;
        spmm_opts o;
        if (!opts_from_text(line.substr(tab + 1), &o))
            return set_error(SPMM_ERR_INVALID, "malformed cache line");
        add[line.substr(0, tab)] = o;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto &kv : add) g_cache[kv.first] = kv.second;
    return SPMM_OK;
}

extern "C" void spmm_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.clear();
}

// ------------------------------------------------------------------------------------------

namespace {

struct Timing {
    spmm_status st;
    double ms;
};

Timing time_opts(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type, const spmm_opts &o,
                 const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s) {
    spmm_plan_t *p = nullptr;
    spmm_status st = spmm_plan(A, n, b_type, c_type, &o, &p);
    if (st != SPMM_OK) return {st, 0.0};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double ms = 0.0;
    do {
        for (int w = 0; w < 2 && st == SPMM_OK; ++w) st = spmm_run(p, B, ldb, C, ldc, s);
        if (st != SPMM_OK) break;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            st = set_error(SPMM_ERR_DEVICE, "hipEventCreate");
            break;
        }
        const int reps = 3;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == SPMM_OK; ++r) st = spmm_run(p, B, ldb, C, ldc, s);
        (void)hipEventRecord(e1, s);
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            st = hip_error(e, "hipEventSynchronize");
            break;
        }
        float x = 0;
        (void)hipEventElapsedTime(&x, e0, e1);
        ms = x / reps;
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)spmm_plan_destroy(p);
    return {st, ms};
}

}  // namespace

extern "C" spmm_status spmm_autotune(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                                     const void *B, int64_t ldb, void *C, int64_t ldc,
                                     void *stream, double budget_ms, spmm_opts *out,
                                     spmm_tune_report *report) {
    if (!out) return set_error(SPMM_ERR_INVALID, "out is null");
    std::string err;
    spmm_status st = validate_problem(A, n, b_type, c_type, err);
    if (st != SPMM_OK) return set_error(st, err);
    if (A->m > 0 && (!C || (A->nnz > 0 && !B))) return set_error(SPMM_ERR_INVALID, "B/C null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    spmm_tune_report rep{};

    // Eq. 1-3: dry-run throughputs and the cost crossover (r = 1)
    double pv = 0, pm = 0;
    {
        std::pair<double, double> cached{0, 0};
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_dryrun.find({n, b_type});
            if (it != g_dryrun.end()) { cached = it->second; have = true; }
        }
        if (!have) {
            st = spmm_dryrun(n, b_type, stream, &cached.first, &cached.second);
            if (st != SPMM_OK) return st;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_dryrun[{n, b_type}] = cached;
        }
        pv = cached.first;
        pm = cached.second;
    }
    const double alpha_cost = pm > 0 ? std::min(1.0, pv / pm) : 1.0;
    rep.p_vec = pv;
    rep.p_mfma = pm;
    rep.alpha_cost = alpha_cost;

    spmm_opts base;
    spmm_opts_default(&base);
    base.mode = SPMM_MODE_PLAIN_F32;
    Timing t = time_opts(A, n, b_type, c_type, base, B, ldb, C, ldc, s);
    if (t.st != SPMM_OK) return t.st;
    rep.candidates = 1;
    rep.default_ms = t.ms;
    spmm_opts best = base;
    double best_ms = t.ms;

    auto try_opts = [&](const spmm_opts &o) -> spmm_status {
        if (elapsed() > budget_ms) return SPMM_OK;
        Timing r = time_opts(A, n, b_type, c_type, o, B, ldb, C, ldc, s);
        if (r.st == SPMM_ERR_UNSUPPORTED) return SPMM_OK;  // option outside its range here
        if (r.st != SPMM_OK) return r.st;
        rep.candidates++;
        if (r.ms < best_ms) {
            best_ms = r.ms;
            best = o;
        }
        return SPMM_OK;
    };
#define SPMM_TRY(x)                       \
    do {                                  \
        spmm_status s_ = (x);             \
        if (s_ != SPMM_OK) return s_;     \
    } while (0)

    // stage 1: vector-only vs mixed with each window order (Sec. 6.1)
    for (int order : {SPMM_ORDER_ORIGINAL_RANGES, SPMM_ORDER_LENGTH_SORTED, SPMM_ORDER_COMPACTED}) {
        spmm_opts o;
        spmm_opts_default(&o);
        o.mode = SPMM_MODE_MIXED;
        o.row_order = order;
        o.window_h = 16;
        o.t_row = order == SPMM_ORDER_ORIGINAL_RANGES ? 1 : 8;
        o.alpha = (float)std::max(alpha_cost, 1.0 / 16.0);
        SPMM_TRY(try_opts(o));
    }
    // stage 2: window height, column and tile thresholds around the best mixed plan
    if (best.mode == SPMM_MODE_MIXED) {
        const spmm_opts b0 = best;
        for (int H : {16, 32, 64})
            for (int cmul : {1, 2})
                for (double amul : {1.0, 2.0}) {
                    spmm_opts o = b0;
                    o.window_h = H;
                    o.alpha_c = (float)cmul / (float)H;
                    o.alpha = (float)std::max(amul * alpha_cost, 1.0 / H);
                    if (o.window_h == b0.window_h && o.alpha_c == b0.alpha_c && o.alpha == b0.alpha)
                        continue;
                    SPMM_TRY(try_opts(o));
                }
        const spmm_opts b1 = best;
        if (b1.row_order != SPMM_ORDER_ORIGINAL_RANGES)
            for (int tr : {1, 32, 128}) {
                spmm_opts o = b1;
                o.t_row = tr;
                SPMM_TRY(try_opts(o));
            }
    }
    // stage 3: segment length and N-panel width (Sec. 6.2.1, the staged B working set)
    {
        const spmm_opts b2 = best;
        for (int sl : {128, 512}) {
            spmm_opts o = b2;
            o.seg_len = sl;
            SPMM_TRY(try_opts(o));
        }
        if (n >= 128) {
            spmm_opts o = best;
            o.n_panel = n / 2;
            SPMM_TRY(try_opts(o));
        }
    }
    // stage 4: vector kernel variant (packed short rows or size classes) and,
    // for a mixed plan, the window launch order
    {
        const spmm_opts b3 = best;
        spmm_opts r;
        resolve_options(&b3, A, n, b_type, &r);
        spmm_opts o = b3;
        o.pipeline = r.pipeline == 3 ? 2 : 3;
        SPMM_TRY(try_opts(o));
        if (best.mode == SPMM_MODE_MIXED) {
            spmm_opts w = best;
            resolve_options(&w, A, n, b_type, &r);
            w.win_sched = r.win_sched == 0 ? 1 : 0;
            SPMM_TRY(try_opts(w));
        }
    }
#undef SPMM_TRY
    rep.best_ms = best_ms;
    rep.search_ms = elapsed();
    *out = best;
    if (report) *report = rep;
    const std::string key = profile_key(A, n, b_type);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = best;
    return SPMM_OK;
}
