// probe.hip -- the gather ceiling of a column sequence (gfx950).
//
// The vector path's time on a power-law graph is set by its B-row gathers
// (one B row per entry, Eq. 1).  This probe measures how fast the device can
// gather the same sequence of B rows when nothing else is done: no entry
// values, no multiply, no C rows, as many independent loads in flight as the
// CUs hold.  Groups of L lanes (a row's 16-byte chunks, rounded up to a
// power of two; rows of up to 128 f32) take sequence positions g, g + G, ...
// (G groups in the grid), U positions per step; each lane reads one chunk of
// its position's row and adds it to a register sum, which is stored only if
// it is NaN (never, for finite B): the loads cannot be dropped and nothing
// is written.
#include <hip/hip_runtime.h>

#include "runtime.hpp"
#include "spmm.h"

namespace spmm {
namespace {

constexpr int kGatherU = 8;           // positions per group per step
constexpr int kGatherBlocks = 32768;  // 256-thread workgroups

// LPR lanes per row (16 bytes each): a row of up to LPR * 4 f32
template <int LPR>
__global__ __launch_bounds__(256) void gather_probe_kernel(const float4 *__restrict__ B, int64_t ld4,
                                                           int chunks, int32_t k,
                                                           const int32_t *__restrict__ rows,
                                                           int64_t n, float4 *__restrict__ sink) {
    constexpr int GPB = 256 / LPR;  // groups per workgroup
    const int64_t G = (int64_t)gridDim.x * GPB;
    const int64_t g = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    const bool on = lane < chunks;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t p = g; p < n; p += G * kGatherU) {
        int r[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const int64_t q = p + u * G;
            // a row id outside [0, k) is clamped: every read stays inside B
            r[u] = q < n ? min(max(__builtin_nontemporal_load(rows + q), 0), k - 1) : 0;
        }
        float4 b[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u)
            b[u] = on ? B[(int64_t)r[u] * ld4 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            if (p + u * G < n) {
                acc.x += b[u].x; acc.y += b[u].y; acc.z += b[u].z; acc.w += b[u].w;
            }
        }
    }
    if (acc.x != acc.x) sink[0] = acc;
}

}  // namespace
}  // namespace spmm

extern "C" spmm_status spmm_gather_bandwidth(const int32_t *rows, int64_t n, const void *B, int64_t k,
                                             int64_t ldb, int32_t n_cols, int32_t reps, void *stream,
                                             double *bytes_per_s) {
    using namespace spmm;
    if (!bytes_per_s || !rows || !B || n <= 0 || k <= 0 || k > INT32_MAX || reps <= 0)
        return set_error(SPMM_ERR_INVALID, "gather probe: null pointer, or a size out of range");
    if (n_cols <= 0 || n_cols > 128 || n_cols % 4 != 0 || ldb < n_cols || ldb % 4 != 0)
        return set_error(SPMM_ERR_INVALID, "gather probe: n_cols must be a multiple of 4 in [4, 128], "
                                           "ldb a multiple of 4 and >= n_cols");
    if ((reinterpret_cast<uintptr_t>(B) & 15) != 0)
        return set_error(SPMM_ERR_INVALID, "gather probe: B must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *sink = nullptr;
    hipError_t e = hipMalloc(&sink, 256);
    if (e != hipSuccess) return set_error(SPMM_ERR_OOM, "hipMalloc(sink)");
    spmm_status st = SPMM_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // lanes per row: the row's 16-byte chunks rounded up to a power of two
    const int chunks = n_cols / 4;
    const int lpr = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : chunks <= 8 ? 8 : chunks <= 16 ? 16 : 32;
    auto launch = [&]() {
#define SPMM_GATHER_PROBE(L)                                                                            \
    hipLaunchKernelGGL(gather_probe_kernel<L>, dim3(kGatherBlocks), dim3(256), 0, s,                   \
                       static_cast<const float4 *>(B), ldb / 4, chunks, (int32_t)k, rows, n,           \
                       static_cast<float4 *>(sink))
        switch (lpr) {
            case 1: SPMM_GATHER_PROBE(1); break;
            case 2: SPMM_GATHER_PROBE(2); break;
            case 4: SPMM_GATHER_PROBE(4); break;
            case 8: SPMM_GATHER_PROBE(8); break;
            case 16: SPMM_GATHER_PROBE(16); break;
            default: SPMM_GATHER_PROBE(32); break;
        }
#undef SPMM_GATHER_PROBE
        return hipGetLastError();
    };
    do {
        for (int w = 0; w < 3 && st == SPMM_OK; ++w)
            if ((e = launch()) != hipSuccess) st = hip_error(e, "gather probe kernel");
        if (st != SPMM_OK) break;
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
            st = hip_error(e, "hipEventCreate");
            break;
        }
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)launch();
        (void)hipEventRecord(e1, s);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = hip_error(e, "hipEventSynchronize"); break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *bytes_per_s = (double)n * n_cols * 4.0 * reps / (ms * 1e-3);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(sink);
    return st;
}
