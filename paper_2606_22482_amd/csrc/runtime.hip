// runtime.hip -- the C ABI (include/spmm.h): plans, uploads, runs, timers, tickets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "devplan.hpp"
#include "plan.hpp"
#include "runtime.hpp"

using namespace spmm;

// ------------------------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

namespace spmm {
spmm_status set_error(spmm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}
spmm_status hip_error(hipError_t e, const char *what) {
    return set_error(SPMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace spmm

#define SPMM_TRY_HIP(call, what)                    \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_error(e_, what); \
    } while (0)

extern "C" int32_t spmm_abi_version(void) { return SPMM_ABI_VERSION; }

extern "C" int64_t spmm_sizeof(int32_t which) {
    switch (which) {
    case 0: return (int64_t)sizeof(spmm_csr);
    case 1: return (int64_t)sizeof(spmm_opts);
    case 2: return (int64_t)sizeof(spmm_plan_stats_t);
    case 3: return (int64_t)sizeof(spmm_plan_dump_t);
    case 4: return (int64_t)sizeof(spmm_work);
    case 5: return (int64_t)sizeof(spmm_adapt_state);
    default: return -1;
    }
}

extern "C" const char *spmm_status_string(spmm_status s) {
    switch (s) {
    case SPMM_OK: return "ok";
    case SPMM_ERR_INVALID: return "invalid argument";
    case SPMM_ERR_OOM: return "out of memory";
    case SPMM_ERR_DEVICE: return "device error";
    case SPMM_ERR_UNSUPPORTED: return "unsupported";
    case SPMM_ERR_BUDGET: return "over budget";
    case SPMM_ERR_BUSY: return "busy";
    default: return "unknown status";
    }
}

extern "C" const char *spmm_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------------
// plans

namespace {

// Every sub-array is followed by at least 16 zero bytes, so a kernel that
// clamps an index into [0, size] (an empty range included) stays inside the
// allocation; the window kernel issues its predicated loads that way.
struct Arena {
    std::vector<std::pair<const void *, size_t>> parts;
    std::vector<size_t> offs;
    std::vector<uint8_t> on_device;  // the part's source is device memory
    size_t total = 0;
    size_t add(const void *p, size_t bytes, bool dev = false) {
        total = (total + 255) & ~size_t(255);
        offs.push_back(total);
        parts.push_back({p, bytes});
        on_device.push_back(dev ? 1 : 0);
        total += bytes + 16;
        return parts.size() - 1;
    }
};

template <class T>
size_t add_vec(Arena &a, const std::vector<T> &v) {
    return a.add(v.data(), v.size() * sizeof(T));
}

}  // namespace

extern "C" spmm_status spmm_plan_build(const spmm_csr *A, int32_t n, int32_t b_type,
                                       int32_t c_type, const spmm_opts *opts, spmm_plan_t **out) {
    if (!out) return set_error(SPMM_ERR_INVALID, "out is null");
    *out = nullptr;
    try {
        std::string err;
        spmm_status st = validate_problem(A, n, b_type, c_type, err);
        if (st != SPMM_OK) return set_error(st, err);
        const bool auto_mode = !opts || opts->mode == SPMM_MODE_AUTO;
        spmm_opts tuned;
        const bool have_tuned = auto_mode && cache_lookup(profile_key(A, n, b_type), &tuned);
        // AUTO keeps the caller's precision class: with f32 B the problem is
        // on the FP32 path (1e-5), and a mixed plan would round B and the
        // values to bf16 in its tiles, so AUTO plans it on the vector path
        // (a tuned profile keeps its other options).  16-bit B is the 16-bit
        // input class (2e-2), where tiles may round f32 values.
        const bool rounds = b_type == SPMM_F32;
        spmm_opts o;
        if (auto_mode && rounds) {
            spmm_opts d;
            if (have_tuned) d = tuned;
            else if (opts) d = *opts;
            else spmm_opts_default(&d);
            d.mode = SPMM_MODE_PLAIN_F32;
            resolve_options(&d, A, n, b_type, &o);
        } else {
            resolve_options(have_tuned ? &tuned : opts, A, n, b_type, &o);
        }
        std::unique_ptr<spmm_plan_s> p(new spmm_plan_s());
        st = build_host_plan(A, n, b_type, c_type, o, p->hp, err);
        if (st != SPMM_OK) return set_error(st, err);
        // AUTO without a tuned profile: keep the mixed partition only when the
        // tiles hold most of the entries, else plan the plain path.  Measured on
        // gfx950: power-law graphs with 1-30% of the entries in tiles run faster
        // plain; block-community matrices with 95% in tiles run 2x faster mixed.
        if (auto_mode && !rounds && !have_tuned && A->nnz > 0 &&
            (double)p->hp.tile_src.size() < 0.5 * (double)A->nnz) {
            o.mode = SPMM_MODE_PLAIN_F32;
            st = build_host_plan(A, n, b_type, c_type, o, p->hp, err);
            if (st != SPMM_OK) return set_error(st, err);
        }
        *out = p.release();
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while planning");
    } catch (const std::exception &e) {
        return set_error(SPMM_ERR_INVALID, e.what());
    }
}

namespace spmm {
// The plan's one device allocation, from its host arrays or, for the arrays
// `da` names, from device memory (a plan partitioned on the device).
spmm_status upload_plan(spmm_plan_t *p, const DeviceArrays *da) {
    if (!p) return set_error(SPMM_ERR_INVALID, "plan is null");
    if (p->dev) return SPMM_OK;
    try {
        HostPlan &h = p->hp;
        Arena a;
        std::vector<int32_t> win_tile_ptr32(h.win_tile_ptr.begin(), h.win_tile_ptr.end());
        std::vector<int32_t> tile_val_ptr32(h.tile_val_ptr.begin(), h.tile_val_ptr.end());
        const size_t i_rem_ptr = add_vec(a, h.rem_ptr32);
        const size_t i_rem_col = da ? a.add(da->rem_col, 4 * da->nrem, true) : add_vec(a, h.rem_col);
        const size_t i_rem_val = da ? a.add(da->rem_val, da->nrem * (size_t)dtype_size(h.val_type), true)
                                    : add_vec(a, h.rem_val);
        const size_t i_vec_rows = add_vec(a, h.vexec.empty() ? h.vector_rows : h.vexec);
        const size_t i_vitem_ptr = add_vec(a, h.vitem_ptr);
        const size_t i_vitem_seg = add_vec(a, h.vitem_seg);
        const size_t i_seg_begin = add_vec(a, h.seg_begin);
        const size_t i_seg_end = add_vec(a, h.seg_end);
        const size_t i_windows = add_vec(a, h.windows);
        const size_t i_win_tile_ptr = add_vec(a, win_tile_ptr32);
        const size_t i_win_seg = add_vec(a, h.win_seg);
        const size_t i_win_order = add_vec(a, h.win_order);
        // Launch order of the segments: by the column of each segment's middle
        // entry (stable).  A row's entries keep their CSR order, which is column
        // order when the CSR's columns are sorted; then segments that run
        // together gather B rows from one stretch of B and share them in L2 and
        // the Infinity Cache.  Any order is correct: each partial lands in its
        // own slot and a row's partials are summed in segment order, so C does
        // not depend on it.
        std::vector<int32_t> seg_order(h.seg_begin.size());
        if (da) {
            seg_order = da->seg_order;  // computed from the device copy of the columns
        } else {
            std::vector<int32_t> key(h.seg_begin.size());
            for (size_t i = 0; i < key.size(); ++i) {
                seg_order[i] = (int32_t)i;
                key[i] = h.rem_col[(size_t)(h.seg_begin[i] + h.seg_end[i] - 1) / 2] & 0x7fffffff;  // bit 31: hot
            }
            std::stable_sort(seg_order.begin(), seg_order.end(),
                             [&](int32_t x, int32_t y) { return key[x] < key[y]; });
            bool id = true;
            for (size_t i = 0; i < seg_order.size() && id; ++i) id = seg_order[i] == (int32_t)i;
            if (id) seg_order.clear();
        }
        const size_t i_seg_order = add_vec(a, seg_order);
        const size_t nt = h.tile_window.size();
        const size_t i_tile_cols = da ? a.add(da->tile_cols, 4 * nt * h.opts.kt, true) : add_vec(a, h.tile_cols);
        const size_t i_tile_bitmap =
            da ? a.add(da->tile_bitmap, 4 * nt * h.opts.window_h, true) : add_vec(a, h.tile_bitmap);
        const size_t i_tile_val_ptr = add_vec(a, tile_val_ptr32);
        const size_t i_tile_vals = da ? a.add(da->tile_vals, 2 * da->nvals, true) : add_vec(a, h.tile_vals);
        const size_t i_win_part = add_vec(a, h.win_part);
        const size_t i_wpart_win = add_vec(a, h.wpart_win);
        const size_t i_wpart_t0 = add_vec(a, h.wpart_t0);
        const size_t i_wpart_t1 = add_vec(a, h.wpart_t1);
        const size_t i_seg_row = add_vec(a, h.seg_row);
        const size_t i_seg_win = add_vec(a, h.seg_win);
        const size_t i_win_dep = add_vec(a, h.win_dep);
        const size_t i_win_nsseg = add_vec(a, h.win_nsseg);
        const size_t i_win_row_sid = add_vec(a, h.win_row_sid);
        static const uint8_t kZeros[256] = {};
        const size_t i_zeros = a.add(kZeros, sizeof(kZeros));
        const size_t total = std::max<size_t>(a.total, 256);

        std::vector<uint8_t> image(total, 0);
        for (size_t i = 0; i < a.parts.size(); ++i)
            if (a.parts[i].second && !a.on_device[i])
                std::memcpy(image.data() + a.offs[i], a.parts[i].first, a.parts[i].second);

        int dev = 0;
        SPMM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, total);
        if (e != hipSuccess) return set_error(SPMM_ERR_OOM, std::string("hipMalloc(plan): ") + hipGetErrorString(e));
        e = hipMemcpy(d, image.data(), total, hipMemcpyHostToDevice);
        for (size_t i = 0; i < a.parts.size() && e == hipSuccess; ++i)
            if (a.parts[i].second && a.on_device[i])
                e = hipMemcpy(static_cast<uint8_t *>(d) + a.offs[i], a.parts[i].first, a.parts[i].second,
                              hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_error(e, "hipMemcpy(plan)");
        }
        auto at = [&](size_t i) -> uint8_t * { return static_cast<uint8_t *>(d) + a.offs[i]; };
        DevPlan &dp = p->dp;
        dp.m = (int32_t)h.m;
        dp.n = h.n;
        dp.seg_len = h.opts.seg_len;
        dp.H = h.opts.window_h;
        dp.kt = h.opts.kt;
        dp.n_vitems = (int32_t)(h.vitem_ptr.size() - 1);
        dp.n_seg = (int32_t)h.seg_row.size();
        dp.n_win = (int32_t)h.win_order.size();
        dp.rem_ptr = reinterpret_cast<const int32_t *>(at(i_rem_ptr));
        dp.rem_col = reinterpret_cast<const int32_t *>(at(i_rem_col));
        dp.rem_val = at(i_rem_val);
        dp.vec_rows = h.identity_rows && h.vexec.empty() ? nullptr
                                                         : reinterpret_cast<const int32_t *>(at(i_vec_rows));
        dp.vitem_ptr = reinterpret_cast<const int32_t *>(at(i_vitem_ptr));
        dp.vitem_seg = reinterpret_cast<const int32_t *>(at(i_vitem_seg));
        dp.seg_begin = reinterpret_cast<const int32_t *>(at(i_seg_begin));
        dp.seg_end = reinterpret_cast<const int32_t *>(at(i_seg_end));
        dp.seg_order = seg_order.empty() ? nullptr : reinterpret_cast<const int32_t *>(at(i_seg_order));
        dp.windows = reinterpret_cast<const int32_t *>(at(i_windows));
        dp.win_tile_ptr = reinterpret_cast<const int32_t *>(at(i_win_tile_ptr));
        dp.win_seg = reinterpret_cast<const int32_t *>(at(i_win_seg));
        bool order_id = true;
        for (size_t w = 0; w < h.win_order.size() && order_id; ++w) order_id = h.win_order[w] == (int32_t)w;
        dp.win_order = order_id ? nullptr : reinterpret_cast<const int32_t *>(at(i_win_order));
        dp.tile_cols = reinterpret_cast<const int32_t *>(at(i_tile_cols));
        dp.tile_bitmap = reinterpret_cast<const uint32_t *>(at(i_tile_bitmap));
        dp.tile_val_ptr = reinterpret_cast<const int32_t *>(at(i_tile_val_ptr));
        dp.tile_vals = reinterpret_cast<const uint16_t *>(at(i_tile_vals));
        dp.n_wpart = (int32_t)h.wpart_win.size();
        dp.win_tmax = h.win_tiles;
        dp.win_part = reinterpret_cast<const int32_t *>(at(i_win_part));
        dp.wpart_win = reinterpret_cast<const int32_t *>(at(i_wpart_win));
        dp.wpart_t0 = reinterpret_cast<const int32_t *>(at(i_wpart_t0));
        dp.wpart_t1 = reinterpret_cast<const int32_t *>(at(i_wpart_t1));
        dp.zeros = reinterpret_cast<const uint16_t *>(at(i_zeros));
        dp.seg_row = reinterpret_cast<const int32_t *>(at(i_seg_row));
        const bool has_win = !h.win_seg.empty();
        dp.seg_win = has_win ? reinterpret_cast<const int32_t *>(at(i_seg_win)) : nullptr;
        dp.win_dep = has_win ? reinterpret_cast<const int32_t *>(at(i_win_dep)) : nullptr;
        dp.win_nsseg = has_win ? reinterpret_cast<const int32_t *>(at(i_win_nsseg)) : nullptr;
        dp.win_row_sid = has_win ? reinterpret_cast<const int32_t *>(at(i_win_row_sid)) : nullptr;
        dp.n_dep = h.n_dep;
        p->dev = d;
        p->dev_bytes = total;
        p->device = dev;
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while uploading");
    }
}
}  // namespace spmm

extern "C" spmm_status spmm_plan_upload(spmm_plan_t *p) { return upload_plan(p, nullptr); }

extern "C" spmm_status spmm_plan(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                                 const spmm_opts *opts, spmm_plan_t **out) {
    spmm_status st = spmm_plan_build(A, n, b_type, c_type, opts, out);
    if (st != SPMM_OK) return st;
    st = spmm_plan_upload(*out);
    if (st != SPMM_OK) {
        delete *out;
        *out = nullptr;
    }
    return st;
}

extern "C" spmm_status spmm_plan_serialize(const spmm_plan_t *p, void *buf, int64_t cap,
                                           int64_t *size) {
    if (!p || !size) return set_error(SPMM_ERR_INVALID, "null argument");
    spmm_status st0 = ensure_host_remainder(const_cast<spmm_plan_t *>(p));
    if (st0 != SPMM_OK) return st0;
    try {
        std::vector<uint8_t> img;
        serialize_host_plan(p->hp, img);
        *size = (int64_t)img.size();
        if (!buf) return SPMM_OK;
        if (cap < (int64_t)img.size()) return set_error(SPMM_ERR_INVALID, "buffer too small");
        std::memcpy(buf, img.data(), img.size());
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while serialising");
    }
}

extern "C" spmm_status spmm_plan_deserialize(const void *buf, int64_t size, int32_t upload,
                                             spmm_plan_t **out) {
    if (!out) return set_error(SPMM_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!buf || size <= 0) return set_error(SPMM_ERR_INVALID, "empty plan image");
    try {
        std::unique_ptr<spmm_plan_s> p(new spmm_plan_s());
        std::string err;
        spmm_status st = deserialize_host_plan(static_cast<const uint8_t *>(buf), (size_t)size,
                                               p->hp, err);
        if (st != SPMM_OK) return set_error(st, err);
        if (upload) {
            st = spmm_plan_upload(p.get());
            if (st != SPMM_OK) return st;
        }
        *out = p.release();
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while loading a plan image");
    }
}

extern "C" spmm_status spmm_plan_destroy(spmm_plan_t *p) {
    if (!p) return SPMM_OK;
    if (p->busy.load() > 0) return set_error(SPMM_ERR_BUSY, "plan has unfinished submissions");
    if (p->dev) (void)hipFree(p->dev);
    if (p->aux) (void)hipFree(p->aux);
    delete p;
    return SPMM_OK;
}

namespace spmm {
size_t workspace_floats(const HostPlan &h, bool serial) {
    const size_t ld = (size_t)(h.n + 3) / 4 * 4;
    // segment partials, window partials, then (co-scheduled) the window slots
    const size_t slots = serial || h.opts.exec == 1 ? 0 : (size_t)h.n_dep * 2 * h.opts.window_h;
    return ((size_t)h.seg_row.size() + (size_t)h.wpart_win.size() * h.opts.window_h + slots) * ld;
}

double algorithmic_bytes(const HostPlan &h) {
    const double sa = dtype_size(h.val_type), sb = dtype_size(h.b_type), sc = 4.0;
    return 4.0 * (double)(h.m + 1) + (double)h.nnz * (4.0 + sa) + (double)h.k_ref * h.n * sb +
           (double)h.m * h.n * sc;
}
}  // namespace spmm

namespace spmm {
spmm_status ensure_host_remainder(spmm_plan_t *p) {
    std::lock_guard<std::mutex> lk(p->host_mu);
    HostPlan &h = p->hp;
    if (p->aux && !p->host_views) {
        // partitioned on the device: the remainder, the tiles and the CSR
        // entry of each of their values
        const size_t nrem = (size_t)p->dev_nrem, nv = (size_t)p->dev_nvals, nt = h.tile_window.size();
        const size_t sval = (size_t)dtype_size(h.val_type);
        h.rem_col.resize(nrem);
        h.rem_val.resize(nrem * sval);
        h.tile_cols.resize(nt * h.opts.kt);
        h.tile_bitmap.resize(nt * h.opts.window_h);
        h.tile_vals.resize(nv);
        std::vector<int32_t> rs(nrem), ts(nv);
        auto d2h = [](void *dst, const void *src, size_t bytes) {
            return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) : hipSuccess;
        };
        SPMM_TRY_HIP(d2h(h.rem_col.data(), p->dp.rem_col, 4 * nrem), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(h.rem_val.data(), p->dp.rem_val, sval * nrem), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(h.tile_cols.data(), p->dp.tile_cols, 4 * h.tile_cols.size()), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(h.tile_bitmap.data(), p->dp.tile_bitmap, 4 * h.tile_bitmap.size()), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(h.tile_vals.data(), p->dp.tile_vals, 2 * nv), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(rs.data(), p->aux, 4 * nrem), "hipMemcpy(plan)");
        SPMM_TRY_HIP(d2h(ts.data(), static_cast<const int32_t *>(p->aux) + nrem, 4 * nv), "hipMemcpy(plan)");
        h.rem_src.assign(rs.begin(), rs.end());
        h.tile_src.assign(ts.begin(), ts.end());
        p->host_views = true;
        return SPMM_OK;
    }
    if (!p->rem_device_only || (int64_t)h.rem_col.size() == h.nnz) return SPMM_OK;
    const size_t n = (size_t)h.nnz, sval = (size_t)dtype_size(h.val_type);
    h.rem_col.resize(n);
    h.rem_val.resize(n * sval);
    SPMM_TRY_HIP(hipMemcpy(h.rem_col.data(), p->dp.rem_col, 4 * n, hipMemcpyDeviceToHost), "hipMemcpy(plan)");
    SPMM_TRY_HIP(hipMemcpy(h.rem_val.data(), p->dp.rem_val, sval * n, hipMemcpyDeviceToHost), "hipMemcpy(plan)");
    h.rem_src.resize(n);
    for (size_t i = 0; i < n; ++i) h.rem_src[i] = (int64_t)i;  // plain: entry p is remainder entry p
    return SPMM_OK;
}
}  // namespace spmm

extern "C" spmm_status spmm_plan_stats(const spmm_plan_t *p, spmm_plan_stats_t *out) {
    if (!p || !out) return set_error(SPMM_ERR_INVALID, "null argument");
    const HostPlan &h = p->hp;
    std::memset(out, 0, sizeof(*out));
    out->m = h.m; out->k = h.k; out->nnz = h.nnz; out->n = h.n;
    out->val_type = h.val_type; out->b_type = h.b_type; out->c_type = h.c_type;
    out->tile_type = h.tile_type;
    out->opts = h.opts;
    out->windows = (int64_t)h.win_order.size();
    out->tiles = (int64_t)h.tile_window.size();
    const bool dev_parts = p->aux != nullptr;  // tiles and remainder partitioned on the device
    out->nnz_tiles = dev_parts ? p->dev_nvals : (int64_t)h.tile_src.size();
    out->nnz_remainder = dev_parts ? p->dev_nrem : p->rem_device_only ? h.nnz : (int64_t)h.rem_src.size();
    out->vector_rows = (int64_t)h.vector_rows.size();
    out->segments = (int64_t)h.seg_row.size();
    out->vector_items = (int64_t)h.vitem_ptr.size() - 1;
    out->k_ref = h.k_ref;
    out->hot_cols = h.hot_cols;
    const double slots = (double)out->tiles * h.opts.window_h * h.opts.kt;
    out->mean_tile_density = slots > 0 ? (double)out->nnz_tiles / slots : 0.0;
    out->zero_fraction_tiles = slots > 0 ? 1.0 - out->mean_tile_density : 0.0;
    out->device_bytes = (int64_t)p->dev_bytes;
    out->workspace_bytes = (int64_t)workspace_floats(h, false) * 4;
    out->algorithmic_bytes = algorithmic_bytes(h);
    out->flops = 2.0 * (double)h.nnz * (double)h.n;
    out->plan_ms = h.plan_ms;
    out->uploaded = p->dev != nullptr;
    out->tol_class = (out->nnz_tiles > 0 && (h.val_type == SPMM_F32 || h.b_type == SPMM_F32))
                         ? SPMM_TOL_ROUNDED16
                         : SPMM_TOL_FP32;
    plan_path_work(h, &out->work_vec, &out->work_tile, &out->work_winrem);
    return SPMM_OK;
}

extern "C" spmm_status spmm_plan_export(const spmm_plan_t *p, spmm_plan_dump_t *out) {
    if (!p || !out) return set_error(SPMM_ERR_INVALID, "null argument");
    {
        spmm_status st = ensure_host_remainder(const_cast<spmm_plan_t *>(p));
        if (st != SPMM_OK) return st;
    }
    const HostPlan &h = p->hp;
    std::memset(out, 0, sizeof(*out));
    out->m = h.m;
    out->nnz = h.nnz;
    out->window_h = h.opts.window_h;
    out->kt = h.opts.kt;
    out->n_windows = (int64_t)h.windows.size() / h.opts.window_h;
    out->windows = h.windows.data();
    out->n_tiles = (int64_t)h.tile_window.size();
    out->tile_window = h.tile_window.data();
    out->tile_cols = h.tile_cols.data();
    out->tile_bitmap = h.tile_bitmap.data();
    out->tile_val_ptr = h.tile_val_ptr.data();
    out->tile_vals = h.tile_vals.data();
    out->tile_src = h.tile_src.data();
    out->rem_ptr = h.rem_ptr.data();
    out->rem_src = h.rem_src.data();
    out->n_vector_rows = (int64_t)h.vector_rows.size();
    out->vector_rows = h.vector_rows.data();
    out->nseg = h.nseg.data();
    out->n_vitems = (int64_t)h.vitem_ptr.size() - 1;
    out->vitem_ptr = h.vitem_ptr.data();
    out->vitem_seg = h.vitem_seg.data();
    out->n_segments = (int64_t)h.seg_row.size();
    out->seg_row = h.seg_row.data();
    out->seg_begin = h.seg_begin.data();
    out->seg_end = h.seg_end.data();
    out->win_seg = h.win_seg.data();
    out->win_order = h.win_order.data();
    out->rem_col_dev = h.rem_col.data();
    out->n_wparts = (int64_t)h.wpart_win.size();
    out->win_part = h.win_part.data();
    out->wpart_win = h.wpart_win.data();
    out->wpart_t0 = h.wpart_t0.data();
    out->wpart_t1 = h.wpart_t1.data();
    out->vexec_rows = h.vexec.empty() ? h.vector_rows.data() : h.vexec.data();
    out->n_dep = h.n_dep;
    out->seg_win = h.seg_win.empty() ? nullptr : h.seg_win.data();
    out->win_dep = h.win_dep.data();
    out->win_nsseg = h.win_nsseg.data();
    return SPMM_OK;
}

// ------------------------------------------------------------------------------------------
// per-stream run context: workspace for partial sums and window slots, the
// arrival counters of co-scheduled runs, and the second stream they fork to

namespace {
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    int32_t *cnt = nullptr;  // arrival counters: zeroed when allocated, cleared by each run's last arrivals
    size_t cnt_ints = 0;
    hipStream_t side = nullptr;  // second stream of co-scheduled runs (default priority)
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
}  // namespace

namespace spmm {
spmm_status run_context(hipStream_t s, size_t bytes, size_t cnt_ints, bool side, RunContext *ctx,
                        std::unique_lock<std::mutex> &lk) {
    *ctx = RunContext{};
    if (bytes == 0 && cnt_ints == 0 && !side) return SPMM_OK;
    int dev = 0;
    SPMM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    // held by the caller until its kernels are enqueued, so that another
    // thread growing this stream's buffers cannot free them in between
    lk = std::unique_lock<std::mutex>(g_ws_mu);
    Workspace &w = g_ws[{dev, s}];
    if (cnt_ints > w.cnt_ints) {
        const size_t old = w.cnt_ints;
        if (w.cnt) {
            SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(counters)");
            (void)hipFree(w.cnt);
            w.cnt = nullptr;
            w.cnt_ints = 0;
        }
        const size_t want = std::max(cnt_ints, old * 2);
        hipError_t e = hipMalloc(&w.cnt, want * sizeof(int32_t));
        if (e != hipSuccess) {
            w.cnt = nullptr;
            return set_error(SPMM_ERR_OOM, std::string("hipMalloc(counters): ") + hipGetErrorString(e));
        }
        // a fill kernel rather than a memset node, so the run stays capturable
        e = launch_zero(w.cnt, (int64_t)want, s);
        if (e != hipSuccess) return hip_error(e, "zero counters");
        w.cnt_ints = want;
    }
    if (side && !w.side) {
        SPMM_TRY_HIP(hipStreamCreateWithFlags(&w.side, hipStreamNonBlocking), "hipStreamCreate(side)");
        SPMM_TRY_HIP(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming), "hipEventCreate");
        SPMM_TRY_HIP(hipEventCreateWithFlags(&w.join, hipEventDisableTiming), "hipEventCreate");
    }
    ctx->cnt = w.cnt;
    ctx->side = side ? w.side : nullptr;
    ctx->fork = w.fork;
    ctx->join = w.join;
    if (bytes == 0) return SPMM_OK;
    if (w.bytes < bytes) {
        const size_t old = w.bytes;
        if (w.ptr) {
            // earlier work on this stream may still read the old buffer
            SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize(workspace)");
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t want = std::max(bytes, old * 2);
        hipError_t e = hipMalloc(&w.ptr, want);
        if (e != hipSuccess) {
            w.ptr = nullptr;
            return set_error(SPMM_ERR_OOM, std::string("hipMalloc(workspace): ") + hipGetErrorString(e));
        }
        w.bytes = want;
    }
    ctx->work = static_cast<float *>(w.ptr);
    return SPMM_OK;
}

static int ilog2_ceil(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

spmm_status make_run_args(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                          RunArgs &a) {
    const HostPlan &h = p->hp;
    const int N = h.n;
    const int E = chunk_elems(h.b_type);
    const int sb = dtype_size(h.b_type);
    a = RunArgs{};
    a.B = B;
    a.ldb = ldb;
    a.C = static_cast<float *>(C);
    a.ldc = ldc;
    a.work = nullptr;
    a.work_ld = (N + 3) / 4 * 4;
    a.vec_ok = (N % E == 0) && (ldb % E == 0) && (ldc % 4 == 0) &&
               ((uintptr_t)B % 16 == 0) && ((uintptr_t)C % 16 == 0) && (sb * E == 16);
    int np = h.opts.n_panel > 0 ? std::min(h.opts.n_panel, N) : N;
    const int maxnp = a.vec_ok ? 128 * E : 128;
    np = std::min(np, maxnp);
    if (a.vec_ok) np = std::max(E, np / E * E);
    a.np = np;
    a.n_panels = (N + np - 1) / np;
    const int chunks = a.vec_ok ? np / E : np;
    a.lpr_log2 = ilog2_ceil(std::min(chunks, 64));
    a.xcd = h.opts.xcd_remap ? 1 : 0;
    // cold B rows go through a raw buffer load (32-bit byte offsets from B)
    const double b_span = ((double)std::max<int64_t>(h.k, 1) - 1.0) * (double)ldb * sb + (double)N * sb;
    a.cold_aux = (b_span < 4294967295.0 && h.opts.cold_policy != 0) ? h.opts.cold_policy : -1;
    a.b_rec = b_span < 4294967040.0 ? (uint32_t)b_span : 0u;
    a.pipeline = h.opts.pipeline;
    // narrow 16-bit B: windows stage panels of 64 or 32 columns, so that no
    // staged column and no MFMA block is padding
    int wnp = 128;
    if (a.vec_ok && sb == 2) wnp = N <= 32 ? 32 : N <= 64 ? 64 : 128;
    set_window_panels(a, N, E, wnp);
    return SPMM_OK;
}

void set_window_panels(RunArgs &a, int N, int E, int np) {
    a.win_np = np;
    a.win_panels = (N + np - 1) / np;
    const int wchunks = a.vec_ok ? np / E : np;
    a.win_lpr_log2 = ilog2_ceil(std::min(wchunks, 64));
}
}  // namespace spmm

// ------------------------------------------------------------------------------------------
// timers

struct spmm_timer_s {
    int32_t cap = 0;
    int32_t used = 0;
    std::vector<int32_t> ids;
    std::vector<hipEvent_t> ev;  // 2 per launch
};

extern "C" spmm_status spmm_timer_create(int32_t capacity, spmm_timer_t **out) {
    if (!out || capacity < 1) return set_error(SPMM_ERR_INVALID, "bad timer arguments");
    std::unique_ptr<spmm_timer_s> t(new spmm_timer_s());
    t->cap = capacity;
    t->ids.resize(capacity);
    t->ev.resize(2 * (size_t)capacity, nullptr);
    for (auto &e : t->ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            for (auto &x : t->ev)
                if (x) (void)hipEventDestroy(x);
            return hip_error(r, "hipEventCreate");
        }
    }
    *out = t.release();
    return SPMM_OK;
}

extern "C" spmm_status spmm_timer_reset(spmm_timer_t *t) {
    if (!t) return set_error(SPMM_ERR_INVALID, "timer is null");
    t->used = 0;
    return SPMM_OK;
}

extern "C" spmm_status spmm_timer_read(spmm_timer_t *t, int32_t *ids, float *ms, int32_t cap,
                                       int32_t *count) {
    if (!t || !count) return set_error(SPMM_ERR_INVALID, "null argument");
    const int32_t n = std::min(t->used, cap);
    for (int32_t i = 0; i < n; ++i) {
        SPMM_TRY_HIP(hipEventSynchronize(t->ev[2 * i + 1]), "hipEventSynchronize");
        float x = 0;
        SPMM_TRY_HIP(hipEventElapsedTime(&x, t->ev[2 * i], t->ev[2 * i + 1]), "hipEventElapsedTime");
        if (ids) ids[i] = t->ids[i];
        if (ms) ms[i] = x;
    }
    *count = n;
    return SPMM_OK;
}

extern "C" spmm_status spmm_timer_destroy(spmm_timer_t *t) {
    if (!t) return SPMM_OK;
    for (auto &e : t->ev)
        if (e) (void)hipEventDestroy(e);
    delete t;
    return SPMM_OK;
}

// ------------------------------------------------------------------------------------------
// runs

namespace spmm {
spmm_status check_run(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc) {
    if (!p) return set_error(SPMM_ERR_INVALID, "plan is null");
    if (!p->dev) return set_error(SPMM_ERR_UNSUPPORTED, "plan is not uploaded");
    const HostPlan &h = p->hp;
    if (h.m > 0 && !C) return set_error(SPMM_ERR_INVALID, "C is null");
    if (h.k > 0 && h.nnz > 0 && !B) return set_error(SPMM_ERR_INVALID, "B is null");
    if (ldb < h.n || ldc < h.n) return set_error(SPMM_ERR_INVALID, "leading dimension < n");
    return SPMM_OK;
}

LaunchEvents &launch_events() {
    thread_local LaunchEvents ev;
    return ev;
}

bool serial_exec(const spmm_plan_t *p, const RunArgs &a) {
    // co-scheduled runs address their workspace through a 32-bit buffer range
    return p->hp.opts.exec == 1 || a.cold_aux >= 0 ||
           (double)workspace_floats(p->hp, false) * 4.0 >= 4294967040.0;
}

// Workgroup ranges of a co-scheduled run: segment and window-partial ranges
// padded to a multiple of 8 so that the range after them starts on XCD 0.
void coschedule_layout(const spmm_plan_t *p, RunArgs &a) {
    const DevPlan &P = p->dp;
    auto up8 = [](int64_t x) { return (int32_t)((x + 7) & ~int64_t(7)); };
    a.seg_blocks = up8(((int64_t)P.n_seg * a.n_panels + 3) / 4);
    a.vec_blocks = (int32_t)(((int64_t)P.n_vitems * a.n_panels + 3) / 4);
    a.wpart_blocks = up8((int64_t)P.n_wpart * a.win_panels);
    a.win_blocks = (int32_t)((int64_t)P.n_win * a.win_panels);
}

// The two grids of a co-scheduled run go to two streams only when each has
// at least a workgroup per CU (256); otherwise one of them is too small to
// pay for the fork and join (measured about 25-30 us on gfx950) and both run
// on the run's stream, the MFMA path first.
bool fork_paths(const RunArgs &a) {
    return a.seg_blocks + a.vec_blocks >= 256 && a.wpart_blocks + a.win_blocks >= 256;
}

size_t counter_ints(const spmm_plan_t *p, const RunArgs &a) {
    if (serial_exec(p, a)) return 0;
    return (size_t)a.n_panels * p->dp.n_seg + (size_t)a.win_panels * p->dp.n_dep;
}

spmm_status launch_plan(const spmm_plan_t *p, const RunArgs &a0, hipStream_t s, spmm_timer_t *t,
                        const RunContext &ctx) {
    const HostPlan &h = p->hp;
    const DevPlan &P = p->dp;
    RunArgs a = a0;
    a.work = ctx.work;
    // a timed kernel records its pair of events inside its own dispatch
    auto timed = [&](int kid, hipStream_t ks, auto &&launch) -> spmm_status {
        const bool rec = t != nullptr;
        if (rec && t->used >= t->cap) return set_error(SPMM_ERR_INVALID, "timer is full");
        if (rec) launch_events() = LaunchEvents{t->ev[2 * t->used], t->ev[2 * t->used + 1]};
        hipError_t e = launch();
        const bool launched = launch_events().start == nullptr;
        launch_events() = LaunchEvents{};
        if (e != hipSuccess) return hip_error(e, "kernel launch");
        if (rec) {
            if (!launched) {  // nothing to launch: an empty interval
                SPMM_TRY_HIP(hipEventRecord(t->ev[2 * t->used], ks), "hipEventRecord");
                SPMM_TRY_HIP(hipEventRecord(t->ev[2 * t->used + 1], ks), "hipEventRecord");
            }
            t->ids[t->used] = kid;
            t->used++;
        }
        return SPMM_OK;
    };
    spmm_status st;
    if (serial_exec(p, a)) {
        if (P.n_seg > 0) {
            // Column-ordered segments go out in dispatch order, not in one
            // contiguous share per XCD: then all XCDs work on one stretch of B at
            // a time and share it in the Infinity Cache (measured faster on the
            // 2^20-vertex power-law graph: 0.306 vs 0.332 ms).
            RunArgs as = a;
            if (P.seg_order) as.xcd = 0;
            st = timed(SPMM_KERNEL_SEGMENT, s, [&] { return launch_segment(P, h.val_type, h.b_type, as, s); });
            if (st != SPMM_OK) return st;
        }
        if (P.n_wpart > 0) {
            st = timed(SPMM_KERNEL_WINDOW_PARTIAL, s,
                       [&] { return launch_window_partial(P, h.val_type, h.b_type, h.tile_type, a, s); });
            if (st != SPMM_OK) return st;
        }
        if (P.n_vitems > 0) {
            st = timed(SPMM_KERNEL_VECTOR, s, [&] { return launch_vector(P, h.val_type, h.b_type, a, s); });
            if (st != SPMM_OK) return st;
        }
        if (P.n_win > 0) {
            st = timed(SPMM_KERNEL_WINDOW, s,
                       [&] { return launch_window(P, h.val_type, h.b_type, h.tile_type, a, s); });
            if (st != SPMM_OK) return st;
        }
        return SPMM_OK;
    }
    // co-scheduled
    a.cnt = ctx.cnt;
    a.dep = ctx.work ? ctx.work + ((int64_t)P.n_seg + (int64_t)P.H * P.n_wpart) * a.work_ld : nullptr;
    a.ws_rec = (uint32_t)(workspace_floats(h, false) * sizeof(float));
    coschedule_layout(p, a);
    const bool mfma = a.wpart_blocks + a.win_blocks > 0, vec = a.seg_blocks + a.vec_blocks > 0;
    if (mfma && !vec && P.n_wpart == 0) {
        // only window owners, nothing to combine: the serial window kernel
        // (bitwise the same C; without the co-scheduled combine's code it
        // holds fewer scalar registers and ran 0.168 against 0.178 ms on the
        // block-community matrix)
        return timed(SPMM_KERNEL_WINDOW, s,
                     [&] { return launch_window(P, h.val_type, h.b_type, h.tile_type, a, s); });
    }
    if (h.opts.exec == 3 && mfma && vec && one_grid_supported(h.b_type, a))
        return timed(SPMM_KERNEL_ONE_GRID, s,
                     [&] { return launch_one_grid(P, h.val_type, h.b_type, h.tile_type, a, s); });
    const bool fork = ctx.allow_fork && fork_paths(a);
    const hipStream_t ms = fork ? ctx.side : s;
    if (mfma) {
        // the MFMA path on the second stream, forked from and joined to the
        // run's stream, so that it runs beside the vector path
        if (fork) {
            SPMM_TRY_HIP(hipEventRecord(ctx.fork, s), "hipEventRecord(fork)");
            SPMM_TRY_HIP(hipStreamWaitEvent(ctx.side, ctx.fork, 0), "hipStreamWaitEvent(fork)");
        }
        st = timed(SPMM_KERNEL_MFMA_PATH, ms,
                   [&] { return launch_mfma_path(P, h.val_type, h.b_type, h.tile_type, a, ms); });
        if (st != SPMM_OK) return st;
        if (fork) SPMM_TRY_HIP(hipEventRecord(ctx.join, ctx.side), "hipEventRecord(join)");
    }
    if (vec) {
        st = timed(SPMM_KERNEL_VECTOR_PATH, s, [&] { return launch_vector_path(P, h.val_type, h.b_type, a, s); });
        if (st != SPMM_OK) return st;
    }
    if (mfma && fork) SPMM_TRY_HIP(hipStreamWaitEvent(s, ctx.join, 0), "hipStreamWaitEvent(join)");
    return SPMM_OK;
}
}  // namespace spmm

static spmm_status run_impl(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                            void *stream, spmm_timer_t *t) {
    spmm_status st = check_run(p, B, ldb, C, ldc);
    if (st != SPMM_OK) return st;
    if (p->hp.m == 0) return SPMM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    RunArgs a;
    make_run_args(p, B, ldb, C, ldc, a);
    const bool serial = serial_exec(p, a);
    RunArgs lay = a;
    coschedule_layout(p, lay);
    const bool side = !serial && fork_paths(lay);
    std::unique_lock<std::mutex> ws_lock;
    RunContext ctx;
    st = run_context(s, workspace_floats(p->hp, serial) * sizeof(float), counter_ints(p, a), side, &ctx,
                     ws_lock);
    if (st != SPMM_OK) return st;
    return launch_plan(p, a, s, t, ctx);
}

extern "C" spmm_status spmm_run(const spmm_plan_t *p, const void *B, int64_t ldb, void *C,
                                int64_t ldc, void *stream) {
    return run_impl(p, B, ldb, C, ldc, stream, nullptr);
}

extern "C" spmm_status spmm_run_bytes(const spmm_plan_t *p, int64_t ldb, int64_t ldc, int32_t batched,
                                      int64_t budget, int64_t *bytes) {
    if (!p || !bytes) return set_error(SPMM_ERR_INVALID, "null argument");
    const HostPlan &h = p->hp;
    if (ldb < h.n || ldc < h.n) return set_error(SPMM_ERR_INVALID, "leading dimension < n");
    const double sb = dtype_size(h.b_type);
    double total = (double)h.k * (double)ldb * sb + (double)h.m * (double)ldc * 4.0;
    if (batched) {
        total += (double)workspace_floats(h, true) * 4.0;
    } else {
        // the run's arguments with B and C aligned (the alignment decides the
        // panel width and so the counters)
        RunArgs a;
        make_run_args(p, reinterpret_cast<const void *>(256), ldb, reinterpret_cast<void *>(256), ldc, a);
        const bool serial = serial_exec(p, a);
        total += (double)workspace_floats(h, serial) * 4.0 + (double)counter_ints(p, a) * 4.0;
    }
    *bytes = (int64_t)total;
    if (budget >= 0 && total > (double)budget) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "execution needs %.0f bytes, beyond the budget of %lld", total,
                      (long long)budget);
        return set_error(SPMM_ERR_BUDGET, msg);
    }
    return SPMM_OK;
}

// ------------------------------------------------------------------------------------------
// A run that allocates nothing: its workspace and arrival counters live in a
// fixed device array of this library, held by every device the library runs
// on until the process ends.  Layout: kScratchCounterBytes of int32 arrival
// counters (zero between runs: cleared once at set-up, then by each run's
// last arrivals), then the float workspace.

namespace {
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr size_t kScratchCounterBytes = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_ptr;  // device -> address of `scratch` there
}  // namespace

// The device address of this device's `scratch` (taken once per device, with
// the device current; the array's name in host code is not a device address),
// with its counters cleared on `s` the first time.
static spmm_status scratch_on_device(hipStream_t s, unsigned char **out) {
    int dev = 0;
    SPMM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return SPMM_OK;
    }
    void *ptr = nullptr;
    SPMM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    hipError_t e = launch_zero(static_cast<int32_t *>(ptr), (int64_t)(kScratchCounterBytes / 4), s);
    if (e != hipSuccess) return hip_error(e, "zero scratch counters");
    g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    *out = static_cast<unsigned char *>(ptr);
    return SPMM_OK;
}

extern "C" spmm_status spmm_run_noalloc(const spmm_plan_t *p, const void *B, int64_t ldb, void *C,
                                        int64_t ldc, void *stream) {
    spmm_status st = check_run(p, B, ldb, C, ldc);
    if (st != SPMM_OK) return st;
    if (p->hp.m == 0) return SPMM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    RunArgs a;
    make_run_args(p, B, ldb, C, ldc, a);
    const bool serial = serial_exec(p, a);
    const size_t bytes = workspace_floats(p->hp, serial) * sizeof(float);
    const size_t cnt_bytes = counter_ints(p, a) * sizeof(int32_t);
    if (bytes > kScratchBytes - kScratchCounterBytes || cnt_bytes > kScratchCounterBytes) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "spmm_run_noalloc: the run needs %zu bytes of workspace and %zu of counters, "
                      "beyond the fixed %zu and %zu", bytes, cnt_bytes,
                      kScratchBytes - kScratchCounterBytes, kScratchCounterBytes);
        return set_error(SPMM_ERR_BUDGET, msg);
    }
    unsigned char *base = nullptr;
    st = scratch_on_device(s, &base);
    if (st != SPMM_OK) return st;
    RunContext ctx;
    ctx.cnt = reinterpret_cast<int32_t *>(base);
    ctx.work = bytes ? reinterpret_cast<float *>(base + kScratchCounterBytes) : nullptr;
    ctx.allow_fork = false;  // a second stream would have to be created
    return launch_plan(p, a, s, nullptr, ctx);
}

extern "C" spmm_status spmm_run_timed(const spmm_plan_t *p, const void *B, int64_t ldb, void *C,
                                      int64_t ldc, void *stream, spmm_timer_t *t) {
    if (!t) return set_error(SPMM_ERR_INVALID, "timer is null");
    return run_impl(p, B, ldb, C, ldc, stream, t);
}

// ------------------------------------------------------------------------------------------
// copy bandwidth probe

extern "C" spmm_status spmm_copy_bandwidth(int64_t bytes, void *stream, double *bps) {
    if (!bps || bytes < 4096) return set_error(SPMM_ERR_INVALID, "bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n4 = bytes / 16;
    void *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, n4 * 16) != hipSuccess) return set_error(SPMM_ERR_OOM, "hipMalloc(src)");
    if (hipMalloc(&dst, n4 * 16) != hipSuccess) {
        (void)hipFree(src);
        return set_error(SPMM_ERR_OOM, "hipMalloc(dst)");
    }
    spmm_status st = SPMM_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        hipError_t e = hipMemsetAsync(src, 0, n4 * 16, s);
        if (e != hipSuccess) { st = hip_error(e, "hipMemsetAsync"); break; }
        for (int w = 0; w < 3 && st == SPMM_OK; ++w) {
            e = launch_copy(static_cast<const float4 *>(src), static_cast<float4 *>(dst), n4, s);
            if (e != hipSuccess) st = hip_error(e, "copy kernel");
        }
        if (st != SPMM_OK) break;
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
            st = hip_error(e, "hipEventCreate");
            break;
        }
        const int reps = 10;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)launch_copy(static_cast<const float4 *>(src), static_cast<float4 *>(dst), n4, s);
        (void)hipEventRecord(e1, s);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = hip_error(e, "hipEventSynchronize"); break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *bps = 2.0 * (double)n4 * 16.0 * reps / (ms * 1e-3);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    return st;
}
