// autotune.hip -- sparsity-profile keys, the tuned-options cache and the
// measurement-driven search over plan options.
//
// The cost model of NeutronSparse Sec. 5.2.1 (Eq. 1-3) gives the density
// threshold alpha = r * P_vec / P_mfma from a dry run; on CDNA4 r = 1 (one
// engine pool, a cost crossover rather than balanced co-running).  The paper
// then tunes the tile shape (Sec. 6.2.2) and shows the threshold's
// sensitivity (Sec. 8.3); here the remaining knobs are chosen by timing
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
    std::snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %d %d %d %.9g %.9g %d %d %d %d %d", o.mode,
                  o.window_h, o.t_row, o.kt, o.n_panel, o.row_order, o.seg_len, o.item_cost,
                  o.xcd_remap, o.hot_cols, (double)o.alpha_c, (double)o.alpha, o.cold_policy,
                  o.pipeline, o.win_sched, o.local_reorder, o.exec);
    return buf;
}

bool opts_from_text(const std::string &t, spmm_opts *o) {
    spmm_opts_default(o);
    double ac = 0, al = 0;
    int n = std::sscanf(t.c_str(), "%d %d %d %d %d %d %d %d %d %d %lg %lg %d %d %d %d %d", &o->mode,
                        &o->window_h, &o->t_row, &o->kt, &o->n_panel, &o->row_order, &o->seg_len,
                        &o->item_cost, &o->xcd_remap, &o->hot_cols, &ac, &al, &o->cold_policy,
                        &o->pipeline, &o->win_sched, &o->local_reorder, &o->exec);
    o->alpha_c = (float)ac;
    o->alpha = (float)al;
    return n == 16 || n == 17;  // files written before the exec field: exec stays auto
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

// Copies of one matrix in a tuning batch: enough entries to keep every CU
// busy, so that a candidate is judged by its throughput among other
// matrices' work (as in a large batch), not by the latency of one small
// matrix alone.  The copies write the same values to the same C.
int batch_copies(const spmm_csr *A) {
    constexpr int64_t kFillEntries = int64_t(1) << 22;
    const int64_t nnz = std::max<int64_t>(1, A->nnz);
    return (int)std::min<int64_t>(64, std::max<int64_t>(1, (kFillEntries + nnz - 1) / nnz));
}

// One execution of plan p: a run, or a batch of `copies` items of it whose
// ticket is retired once the timing has been read (tickets[] collects them).
spmm_status exec_once(spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s,
                      int copies, std::vector<spmm_ticket> &tickets) {
    if (copies == 0) return spmm_run(p, B, ldb, C, ldc, s);
    std::vector<spmm_work> w(copies, spmm_work{p, B, ldb, C, ldc});
    spmm_ticket t = 0;
    spmm_status st = spmm_submit(w.data(), copies, s, &t);
    if (st == SPMM_OK) tickets.push_back(t);
    return st;
}

Timing time_opts(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type, const spmm_opts &o,
                 const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s, bool submit,
                 int reps = 3) {
    const int copies = submit ? batch_copies(A) : 0;
    spmm_plan_t *p = nullptr;
    spmm_status st = spmm_plan(A, n, b_type, c_type, &o, &p);
    if (st != SPMM_OK) return {st, 0.0};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double ms = 0.0;
    std::vector<spmm_ticket> tickets;
    do {
        for (int w = 0; w < 2 && st == SPMM_OK; ++w) st = exec_once(p, B, ldb, C, ldc, s, copies, tickets);
        if (st != SPMM_OK) break;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            st = set_error(SPMM_ERR_DEVICE, "hipEventCreate");
            break;
        }
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == SPMM_OK; ++r) st = exec_once(p, B, ldb, C, ldc, s, copies, tickets);
        (void)hipEventRecord(e1, s);
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            st = hip_error(e, "hipEventSynchronize");
            break;
        }
        float x = 0;
        (void)hipEventElapsedTime(&x, e0, e1);
        ms = x / reps / std::max(1, copies);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (spmm_ticket t : tickets) {
        const spmm_status w = spmm_wait(t);
        if (st == SPMM_OK) st = w;
    }
    (void)spmm_plan_destroy(p);
    return {st, ms};
}

}  // namespace

extern "C" spmm_status spmm_autotune(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                                     const void *B, int64_t ldb, void *C, int64_t ldc,
                                     void *stream, double budget_ms, int32_t context,
                                     spmm_opts *out, spmm_tune_report *report) {
    if (!out) return set_error(SPMM_ERR_INVALID, "out is null");
    if (context != SPMM_TUNE_RUN && context != SPMM_TUNE_SUBMIT)
        return set_error(SPMM_ERR_INVALID, "context must be SPMM_TUNE_RUN or SPMM_TUNE_SUBMIT");
    const bool submit = context == SPMM_TUNE_SUBMIT;
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
    Timing t = time_opts(A, n, b_type, c_type, base, B, ldb, C, ldc, s, submit);
    if (t.st != SPMM_OK) return t.st;
    rep.candidates = 1;
    rep.default_ms = t.ms;
    spmm_opts best = base;
    double best_ms = t.ms;

    auto try_opts = [&](const spmm_opts &o) -> spmm_status {
        if (elapsed() > budget_ms) return SPMM_OK;
        Timing r = time_opts(A, n, b_type, c_type, o, B, ldb, C, ldc, s, submit);
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

    // stage 1: vector-only vs mixed with each window order (Sec. 6.1), and the
    // mixed plan that AUTO builds without a profile (the plain one is the
    // base), so that a tuned plan is never slower than the untuned default.
    // With f32 B the problem is on the FP32 path: mixed plans would round
    // tile operands to bf16, so only vector-path options are searched.
    const bool fp32_class = b_type == SPMM_F32;
    if (!fp32_class) {
        spmm_opts d, o;
        spmm_opts_default(&d);
        d.mode = SPMM_MODE_MIXED;
        resolve_options(&d, A, n, b_type, &o);
        SPMM_TRY(try_opts(o));
    }
    for (int order : {SPMM_ORDER_ORIGINAL_RANGES, SPMM_ORDER_LENGTH_SORTED, SPMM_ORDER_COMPACTED}) {
        if (fp32_class) break;
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
    // A search over three-run timings can pick a candidate that only won by
    // noise (small matrices run in tens of microseconds).  The winner is
    // timed again against the untuned plain plan, both over more runs, and
    // kept only if it is at least kKeepMargin faster.
    if (std::memcmp(&best, &base, sizeof(best)) != 0) {
        constexpr int kVerifyReps = 10;
        constexpr double kKeepMargin = 0.03;
        Timing tb = time_opts(A, n, b_type, c_type, base, B, ldb, C, ldc, s, submit, kVerifyReps);
        if (tb.st != SPMM_OK) return tb.st;
        Timing tw = time_opts(A, n, b_type, c_type, best, B, ldb, C, ldc, s, submit, kVerifyReps);
        if (tw.st != SPMM_OK) return tw.st;
        rep.default_ms = tb.ms;
        best_ms = tw.ms;
        if (tw.ms > tb.ms * (1.0 - kKeepMargin)) {
            best = base;
            best_ms = tb.ms;
        }
    }
    rep.best_ms = best_ms;
    rep.search_ms = elapsed();
    *out = best;
    if (report) *report = rep;
    const std::string key = profile_key(A, n, b_type);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = best;
    return SPMM_OK;
}

// ------------------------------------------------------------------------------------------
// Epoch-level adaptive re-partition (Sec. 5.3, Eq. 6-7; one pool of CUs, r = 1)

extern "C" spmm_status spmm_adapt_next(spmm_adapt_state *st, double t_vec_ms, double t_mfma_ms,
                                       double w_vec, double w_tile, double w_winrem,
                                       double p_vec_dry, double p_mfma_dry, float eps) {
    if (!st) return set_error(SPMM_ERR_INVALID, "state is null");
    if (!(t_vec_ms >= 0) || !(t_mfma_ms >= 0) || !(w_vec >= 0) || !(w_tile >= 0) ||
        !(w_winrem >= 0) || !(eps >= 0))
        return set_error(SPMM_ERR_INVALID, "times, work and eps must be >= 0");
    if (!(st->alpha > 0)) return set_error(SPMM_ERR_INVALID, "state alpha must be > 0");
    // Eq. 1 inverted on the epoch; the window kernels' remainder entries are
    // charged at the vector rate, the rest of their time is the tiles'.  A
    // path without work keeps the throughput measured last, else the dry run's.
    const double pv_fb = st->p_vec > 0 ? st->p_vec : p_vec_dry;
    const double pm_fb = st->p_mfma > 0 ? st->p_mfma : p_mfma_dry;
    double pv = (w_vec > 0 && t_vec_ms > 0) ? w_vec / (t_vec_ms * 1e-3) : pv_fb;
    double pm = pm_fb;
    if (w_tile > 0 && t_mfma_ms > 0) {
        if (!(pv > 0)) return set_error(SPMM_ERR_INVALID, "no vector throughput");
        double t_tiles = t_mfma_ms * 1e-3 - w_winrem / pv;
        t_tiles = std::max(t_tiles, 0.1 * t_mfma_ms * 1e-3);
        pm = w_tile / t_tiles;
    }
    if (!(pv > 0) || !(pm > 0)) return set_error(SPMM_ERR_INVALID, "no throughput for a path");
    const double a = st->alpha;
    const double as = std::min(1.0, pv / pm);  // Eq. 3 / Eq. 7, r = 1
    const double sk = std::max(a, as) / std::min(a, as);  // Eq. 6 on a threshold-density tile
    st->alpha_star = as;
    st->skew = sk;
    st->p_vec = pv;
    st->p_mfma = pm;
    st->t_vec_ms = t_vec_ms;
    st->t_mfma_ms = t_mfma_ms;
    st->replanned = 0;
    st->converged = sk <= 1.0 + eps ? 1 : 0;
    if (st->converged || st->rounds >= 7) return SPMM_OK;
    const bool raise = as > a;
    if (raise) st->lo = a;
    else st->hi = a;
    // secant step on log(alpha*/alpha) over this epoch and the previous one,
    // taken when it falls strictly inside the bracket
    double next = -1.0;
    if (st->prev_alpha > 0 && st->prev_alpha_star > 0 && st->prev_alpha != a) {
        const double f = std::log(as / a), fp = std::log(st->prev_alpha_star / st->prev_alpha);
        if (f != fp) {
            const double x = std::log(a) - f * (std::log(a) - std::log(st->prev_alpha)) / (f - fp);
            const double cand = std::exp(x), d = x - std::log(a);
            const bool inside = (st->lo <= 0 || cand > st->lo) && (st->hi <= 0 || cand < st->hi);
            // on alpha*'s side, at most twice its distance: no wild extrapolation
            if (inside && d * f > 0 && std::fabs(d) <= 2.0 * std::fabs(f)) {
                next = cand;
                st->capped = 0;
            }
        }
    }
    if (next < 0) {
        next = as;
        int capped = 0;
        if (raise) {  // tiles at the threshold cost more on the matrix path: sparser tiles to vector
            if (st->hi > 0 && as >= std::sqrt(a * st->hi)) {
                if (st->capped == 1) st->hi = 0;  // a second cut step: drop that bracket end
                else { next = std::sqrt(a * st->hi); capped = 1; }
            }
        } else {  // rows just below the threshold cost more on the vector path: pack them into tiles
            if (st->lo > 0 && as <= std::sqrt(a * st->lo)) {
                if (st->capped == -1) st->lo = 0;
                else { next = std::sqrt(a * st->lo); capped = -1; }
            }
        }
        st->capped = capped;
    }
    st->prev_alpha = a;
    st->prev_alpha_star = as;
    st->alpha = next;
    st->rounds += 1;
    st->replanned = 1;
    return SPMM_OK;
}

extern "C" spmm_status spmm_adapt_epoch(const spmm_csr *A, spmm_plan_t **plan, const void *B,
                                        int64_t ldb, void *C, int64_t ldc, void *stream,
                                        float eps, spmm_adapt_state *st) {
    if (!A || !plan || !*plan || !st) return set_error(SPMM_ERR_INVALID, "null argument");
    spmm_plan_t *p = *plan;
    const HostPlan &h = p->hp;
    if (A->m != h.m || A->k != h.k || A->nnz != h.nnz)
        return set_error(SPMM_ERR_INVALID, "A is not the matrix of the plan");
    if (h.opts.exec == 3)
        return set_error(SPMM_ERR_UNSUPPORTED, "an epoch times the two paths apart: exec 1 or 2");
    spmm_timer_t *t = nullptr;
    spmm_status st0 = spmm_timer_create(16, &t);
    if (st0 != SPMM_OK) return st0;
    st0 = spmm_run_timed(p, B, ldb, C, ldc, stream, t);
    int32_t ids[16], cnt = 0;
    float ms[16];
    if (st0 == SPMM_OK) st0 = spmm_timer_read(t, ids, ms, 16, &cnt);
    (void)spmm_timer_destroy(t);
    if (st0 != SPMM_OK) return st0;
    double tv = 0, tm = 0;
    for (int32_t i = 0; i < cnt; ++i) {
        // the vector path (serial: segment and vector kernels; co-scheduled:
        // its grid) and the MFMA path (window kernels, or its grid, which ran
        // beside the vector path on the same CUs)
        if (ids[i] == SPMM_KERNEL_SEGMENT || ids[i] == SPMM_KERNEL_VECTOR || ids[i] == SPMM_KERNEL_VECTOR_PATH)
            tv += ms[i];
        else
            tm += ms[i];
    }
    double wv = 0, wt = 0, wr = 0;
    plan_path_work(h, &wv, &wt, &wr);
    const double n = (double)h.n;
    if (!(st->alpha > 0)) st->alpha = h.opts.alpha;
    // a path without work takes the dry-run throughput (cached per N and B type)
    double pvd = 0, pmd = 0;
    if (wv == 0 || wt == 0) {
        std::pair<double, double> cached{0, 0};
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_dryrun.find({h.n, h.b_type});
            if (it != g_dryrun.end()) { cached = it->second; have = true; }
        }
        if (!have) {
            st0 = spmm_dryrun(h.n, h.b_type, stream, &cached.first, &cached.second);
            if (st0 != SPMM_OK) return st0;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_dryrun[{h.n, h.b_type}] = cached;
        }
        pvd = cached.first;
        pmd = cached.second;
    }
    const spmm_adapt_state before = *st;
    st0 = spmm_adapt_next(st, tv, tm, wv * n, wt * n, wr * n, pvd, pmd, eps);
    if (st0 != SPMM_OK || !st->replanned) return st0;
    spmm_opts o = h.opts;
    o.mode = SPMM_MODE_MIXED;
    o.alpha = (float)st->alpha;
    spmm_plan_t *np = nullptr;
    st0 = spmm_plan(A, h.n, h.b_type, h.c_type, &o, &np);
    if (st0 != SPMM_OK) {
        *st = before;  // the epoch's result stands; the plan and state are unchanged
        return st0;
    }
    st0 = spmm_plan_destroy(p);
    if (st0 != SPMM_OK) {
        (void)spmm_plan_destroy(np);
        *st = before;
        return st0;
    }
    *plan = np;
    return SPMM_OK;
}
