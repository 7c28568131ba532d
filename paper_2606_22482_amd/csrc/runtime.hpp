// runtime.hpp -- internals shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>

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
    std::mutex host_mu;
};

namespace spmm {
spmm_status set_error(spmm_status s, const std::string &msg);
spmm_status hip_error(hipError_t e, const char *what);
// The stream's workspace of at least `bytes`; `lk` holds the workspace table
// until the caller has enqueued the kernels that use it.
spmm_status workspace_for(hipStream_t s, size_t bytes, float **out, std::unique_lock<std::mutex> &lk);
spmm_status make_run_args(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                          RunArgs &a);
spmm_status check_run(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc);
spmm_status launch_plan(const spmm_plan_t *p, const RunArgs &a, hipStream_t s, spmm_timer_t *t);
double algorithmic_bytes(const HostPlan &h);
// Host copies of a device-built plan's remainder (no-op for host-built plans).
spmm_status ensure_host_remainder(spmm_plan_t *p);
size_t workspace_floats(const HostPlan &h);
std::string profile_key(const spmm_csr *A, int32_t n, int32_t b_type);
bool cache_lookup(const std::string &key, spmm_opts *o);
}  // namespace spmm
