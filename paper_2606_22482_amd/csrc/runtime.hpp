// runtime.hpp -- internals shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "devplan.hpp"
#include "plan.hpp"

struct spmm_plan_s {
    spmm::HostPlan hp;
    spmm::DevPlan dp{};
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int device = -1;
    std::atomic<int> busy{0};  // unfinished batched submissions using this plan
    // built on the device: the remainder columns and values live only in the
    // device allocation until a host view is asked for (export, serialize)
    bool rem_device_only = false;
    // partitioned on the device (mixed plans): the CSR entry of every
    // remainder entry and then of every packed tile value (int32), kept for
    // host views; the remainder and tile arrays live only in `dev`
    void *aux = nullptr;
    int64_t dev_nrem = 0, dev_nvals = 0;
    bool host_views = false;  // the device-only arrays have been copied to hp
    std::mutex host_mu;
};

namespace spmm {
// Arrays of a plan partitioned on the device, uploaded device to device.
struct DeviceArrays {
    const void *rem_col = nullptr, *rem_val = nullptr;     // [nrem]
    const void *tile_cols = nullptr, *tile_bitmap = nullptr;  // [T * kt], [T * H]
    const void *tile_vals = nullptr;                        // [nvals]
    size_t nrem = 0, nvals = 0;
    std::vector<int32_t> seg_order;  // launch order of the segments (empty: id order)
};
spmm_status upload_plan(spmm_plan_t *p, const DeviceArrays *da);
// Device builders (devbuild.hip): exclusive (inclusive != 0: inclusive) scan of
// n int64 values; `sums` holds ceil(n / 2048) + 1 values, its last the total.
hipError_t scan64(const int64_t *in, int64_t *out, int64_t n, int inclusive, int64_t *sums,
                  hipStream_t s);
int64_t scan_sums_len(int64_t n);
// The mixed plan (original-ranges windows) built on the device (devmixed.hip).
spmm_status plan_device_mixed(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                              const spmm_opts &o, hipStream_t s, spmm_plan_t **out);
spmm_status set_error(spmm_status s, const std::string &msg);
spmm_status hip_error(hipError_t e, const char *what);
// What one run on a stream uses besides the plan: the stream's workspace (at
// least `bytes`), its arrival counters (at least cnt_ints, zero between runs),
// and for a co-scheduled run with windows the second stream and the fork and
// join events.  `lk` holds the table until the caller has enqueued the
// kernels that use them.
struct RunContext {
    float *work = nullptr;
    int32_t *cnt = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool allow_fork = true;  // false: both co-scheduled grids on the run's stream
};
spmm_status run_context(hipStream_t s, size_t bytes, size_t cnt_ints, bool side, RunContext *ctx,
                        std::unique_lock<std::mutex> &lk);
// Whether a run of the plan uses the serial kernels (exec 1, or a cold policy).
bool serial_exec(const spmm_plan_t *p, const RunArgs &a);
// Workgroup ranges of a co-scheduled run (RunArgs' *_blocks).
void coschedule_layout(const spmm_plan_t *p, RunArgs &a);
// Whether a co-scheduled run forks its MFMA path to the second stream.
bool fork_paths(const RunArgs &a);
// Arrival counters a run of the plan uses (0 when serial).
size_t counter_ints(const spmm_plan_t *p, const RunArgs &a);
spmm_status make_run_args(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                          RunArgs &a);
// Window panels of np columns (128, 64 or 32) for a run with N columns.
void set_window_panels(RunArgs &a, int N, int E, int np);
spmm_status check_run(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc);
spmm_status launch_plan(const spmm_plan_t *p, const RunArgs &a, hipStream_t s, spmm_timer_t *t,
                        const RunContext &ctx);
double algorithmic_bytes(const HostPlan &h);
// Host copies of a device-built plan's remainder (no-op for host-built plans).
spmm_status ensure_host_remainder(spmm_plan_t *p);
// Floats of workspace a run needs: segment partials, window partials and,
// unless `serial` or the plan's exec is 1, the window slots of co-scheduled runs.
size_t workspace_floats(const HostPlan &h, bool serial);
std::string profile_key(const spmm_csr *A, int32_t n, int32_t b_type);
bool cache_lookup(const std::string &key, spmm_opts *o);
}  // namespace spmm
