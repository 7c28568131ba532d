// devbuild.hip -- the plain plan built on the device, from a CSR that is
// already in device memory (Sec. 5.2.2 preprocessing without moving A through
// the host).
//
// Every row is a vector row (PLAIN).  The device computes, in order:
//   1. row lengths Len(r) (Eq. 4), segment counts and item costs, and checks
//      the CSR (monotone row pointers, columns in range); the host reads the
//      error flag back before anything is indexed by a row length;
//   2. the item cut: row r belongs to item floor(c_r / item_cost), c_r the
//      exclusive prefix of the costs (the host builder uses the same rule);
//   3. for the size-class variant, each item's rows longest first (a stable
//      rank sort per item, split rows last), as std::stable_sort on the host;
//   4. segment ids in launch order, the segments' entry ranges, and copies of
//      the columns and values.
// Only O(m) schedule arrays come back to the host (for statistics and the
// workspace size); the O(nnz) arrays never leave the device.  The integer
// scans are our own three-phase scans (tiles of 2048, deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <numeric>

#include "devplan.hpp"
#include "plan.hpp"
#include "runtime.hpp"

using namespace spmm;

#define SPMM_TRY_HIP(call, what)                          \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_error(e_, what); \
    } while (0)

namespace {

constexpr int kThreads = 256;
constexpr int kPer = 8;
constexpr int kTile = kThreads * kPer;

__device__ __forceinline__ int64_t wave_scan_incl64(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive prefix of v over the 256 threads of the block; *total = block sum.
__device__ int64_t block_scan_excl64(int64_t v, int64_t *sm, int64_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t incl = wave_scan_incl64(v);
    if (lane == 63) sm[wave] = incl;
    __syncthreads();
    int64_t off = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) off += sm[w];
        all += sm[w];
    }
    __syncthreads();
    *total = all;
    return off + incl - v;
}

__global__ __launch_bounds__(kThreads) void k_tile_sums(int64_t n, const int64_t *__restrict__ in,
                                                        int64_t *__restrict__ sums) {
    __shared__ int64_t sm[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = t0 + (int64_t)threadIdx.x * kPer + j;
        if (i < n) s += in[i];
    }
    int64_t total = 0;
    (void)block_scan_excl64(s, sm, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// one block: exclusive scan of the nb tile sums in place; sums[nb] = total
__global__ __launch_bounds__(kThreads) void k_scan_sums(int64_t nb, int64_t *__restrict__ sums) {
    __shared__ int64_t sm[kThreads / 64];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        int64_t total = 0;
        const int64_t ex = block_scan_excl64(v, sm, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(int64_t n, const int64_t *__restrict__ in,
                                                         const int64_t *__restrict__ sums,
                                                         int64_t *__restrict__ out, int inclusive) {
    __shared__ int64_t sm[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const int64_t base = t0 + (int64_t)threadIdx.x * kPer;
    int64_t v[kPer], s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    int64_t total = 0;
    int64_t run = sums[blockIdx.x] + block_scan_excl64(s, sm, &total);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (inclusive) run += v[j];
        if (base + j < n) out[base + j] = run;
        if (!inclusive) run += v[j];
    }
}

// rows: lengths, segment counts, costs, int32 row pointers, CSR checks
__global__ __launch_bounds__(kThreads) void k_rows(int64_t m, int64_t nnz, const int64_t *__restrict__ rowptr,
                                                   int32_t seg_len, int64_t *__restrict__ cost,
                                                   int64_t *__restrict__ nseg64, int32_t *__restrict__ nseg,
                                                   int32_t *__restrict__ rp32, int32_t *__restrict__ bad) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r > m) return;
    if (r == m) {
        const int64_t e = rowptr[m];
        if (e != nnz) atomicOr(bad, 1);
        rp32[m] = (int32_t)nnz;
        return;
    }
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    const bool ok = b >= 0 && e >= b && e <= nnz && (r != 0 || b == 0);
    if (!ok) atomicOr(bad, 1);
    const int64_t L = ok ? e - b : 0;
    const int32_t ns = L > seg_len ? (int32_t)((L + seg_len - 1) / seg_len) : 0;
    nseg[r] = ns;
    nseg64[r] = ns;
    cost[r] = kRowCost + (ns ? ns : L);
    rp32[r] = ok ? (int32_t)b : 0;
}

__global__ __launch_bounds__(kThreads) void k_cols(int64_t nnz, int64_t k, const int32_t *__restrict__ colidx,
                                                   uint8_t *__restrict__ seen, int32_t *__restrict__ bad) {
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * kThreads) {
        const int32_t c = colidx[p];
        if (c < 0 || c >= k) atomicOr(bad, 2);
        else seen[c] = 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_count_seen(int64_t k, const uint8_t *__restrict__ seen,
                                                         unsigned long long *__restrict__ count) {
    __shared__ int64_t sm[kThreads / 64];
    int64_t s = 0;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < k; c += (int64_t)gridDim.x * kThreads)
        s += seen[c];
    int64_t total = 0;
    (void)block_scan_excl64(s, sm, &total);
    if (threadIdx.x == 0 && total) atomicAdd(count, (unsigned long long)total);
}

// new item at r when floor(c_r / C) differs from the previous row's
__global__ __launch_bounds__(kThreads) void k_item_flags(int64_t m, const int64_t *__restrict__ start,
                                                         int64_t C, int64_t *__restrict__ flag) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= m) return;
    flag[r] = (r == 0 || start[r] / C != start[r - 1] / C) ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_item_ptr(int64_t m, const int64_t *__restrict__ flag,
                                                       const int64_t *__restrict__ idx,
                                                       int32_t *__restrict__ vitem_ptr) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= m) return;
    if (flag[r]) vitem_ptr[idx[r] - 1] = (int32_t)r;
    if (r == m - 1) vitem_ptr[idx[r]] = (int32_t)m;
}

// size-class variant: each item's rows by remainder length, longest first,
// split rows last, ties in row order (one wavefront per item, rank sort)
__global__ __launch_bounds__(kThreads) void k_item_sort(int64_t V, const int32_t *__restrict__ vitem_ptr,
                                                        const int32_t *__restrict__ rp32,
                                                        const int32_t *__restrict__ nseg,
                                                        int32_t *__restrict__ order) {
    const int64_t it = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (it >= V) return;
    const int lane = threadIdx.x & 63;
    const int32_t b = vitem_ptr[it], e = vitem_ptr[it + 1];
    for (int32_t i = b + lane; i < e; i += 64) {
        const int64_t ki = nseg[i] ? -1 : (int64_t)(rp32[i + 1] - rp32[i]);
        int32_t rank = 0;
        for (int32_t j = b; j < e; ++j) {
            const int64_t kj = nseg[j] ? -1 : (int64_t)(rp32[j + 1] - rp32[j]);
            rank += (kj > ki) || (kj == ki && j < i);
        }
        order[b + rank] = i;
    }
}

__global__ __launch_bounds__(kThreads) void k_exec_nseg(int64_t m, const int32_t *__restrict__ order,
                                                        const int32_t *__restrict__ nseg,
                                                        int64_t *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= m) return;
    out[q] = nseg[order ? order[q] : (int32_t)q];
}

__global__ __launch_bounds__(kThreads) void k_item_seg(int64_t V, const int32_t *__restrict__ vitem_ptr,
                                                       const int64_t *__restrict__ segbase,
                                                       int32_t *__restrict__ vitem_seg) {
    const int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (it >= V) return;
    vitem_seg[it] = (int32_t)segbase[vitem_ptr[it]];
}

__global__ __launch_bounds__(kThreads) void k_segments(int64_t m, int64_t S, int32_t seg_len,
                                                       const int32_t *__restrict__ order,
                                                       const int32_t *__restrict__ nseg,
                                                       const int32_t *__restrict__ rp32,
                                                       const int64_t *__restrict__ segbase,
                                                       int32_t *__restrict__ seg_begin,
                                                       int32_t *__restrict__ seg_end,
                                                       int32_t *__restrict__ seg_row) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= m) return;
    const int32_t r = order ? order[q] : (int32_t)q;
    const int64_t base = segbase[q];
    for (int32_t j = 0; j < nseg[r] && base + j < S; ++j) {
        const int64_t b = (int64_t)rp32[r] + (int64_t)j * seg_len;
        seg_begin[base + j] = (int32_t)b;
        seg_end[base + j] = (int32_t)std::min<int64_t>(b + seg_len, rp32[r + 1]);
        seg_row[base + j] = r;
    }
}

// Sort key of each segment's launch: the column of its middle entry (the
// hot-column flag is never set in a plan built here).
__global__ __launch_bounds__(kThreads) void k_seg_keys(int64_t S, const int32_t *__restrict__ seg_begin,
                                                       const int32_t *__restrict__ seg_end,
                                                       const int32_t *__restrict__ col,
                                                       int32_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= S) return;
    key[i] = col[((int64_t)seg_begin[i] + seg_end[i] - 1) / 2] & 0x7fffffff;
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }

// 0 .. n-1 stably sorted by non-negative keys: two counting passes over
// 16-bit digits, lowest first (the order a stable comparison sort gives).
std::vector<int32_t> order_by_key(const std::vector<int32_t> &key) {
    const size_t n = key.size();
    std::vector<int32_t> a(n), b(n);
    std::iota(a.begin(), a.end(), 0);
    std::vector<size_t> cnt((size_t)1 << 16);
    for (int shift = 0; shift < 32; shift += 16) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; ++i) ++cnt[((uint32_t)key[a[i]] >> shift) & 0xFFFFu];
        size_t sum = 0;
        for (size_t &c : cnt) {
            const size_t t = c;
            c = sum;
            sum += t;
        }
        for (size_t i = 0; i < n; ++i) b[cnt[((uint32_t)key[a[i]] >> shift) & 0xFFFFu]++] = a[i];
        a.swap(b);
    }
    return a;
}


struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

namespace spmm {
// exclusive (or inclusive) scan of n int64 values; sums[nb] (device) = total
hipError_t scan64(const int64_t *in, int64_t *out, int64_t n, int inclusive, int64_t *sums,
                  hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(kThreads), 0, s, n, in, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, s, nb, sums);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, n, in, sums, out, inclusive);
    return hipGetLastError();
}
int64_t scan_sums_len(int64_t n) { return std::max<int64_t>(1, (n + kTile - 1) / kTile) + 1; }
}  // namespace spmm

extern "C" spmm_status spmm_plan_device(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                                        const spmm_opts *opts, void *stream, spmm_plan_t **out) {
    if (!out) return set_error(SPMM_ERR_INVALID, "out is null");
    *out = nullptr;
    std::string err;
    spmm_status st = validate_shape(A, n, b_type, c_type, err);
    if (st != SPMM_OK) return set_error(st, err);
    spmm_opts o;
    {
        spmm_opts in;
        if (opts) in = *opts;
        else spmm_opts_default(&in);
        if (in.mode == SPMM_MODE_AUTO) in.mode = SPMM_MODE_PLAIN_F32;
        resolve_options(&in, A, n, b_type, &o);
    }
    if (o.mode != SPMM_MODE_PLAIN_F32)  // windows and tiles partitioned on the device
        return plan_device_mixed(A, n, b_type, c_type, o, static_cast<hipStream_t>(stream), out);
    if (o.cold_policy != 0) return set_error(SPMM_ERR_UNSUPPORTED, "device-built plans gather with the default policy");
    if (o.item_cost > 4096) return set_error(SPMM_ERR_UNSUPPORTED, "device-built plans need item_cost <= 4096");
    st = validate_opts(o, err);
    if (st != SPMM_OK) return set_error(st, err);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t m = A->m, k = A->k, nnz = A->nnz;
    const int sval = dtype_size(A->val_type);
    try {
        std::unique_ptr<spmm_plan_s> p(new spmm_plan_s());
        HostPlan &h = p->hp;
        h.m = m; h.k = k; h.nnz = nnz; h.n = n;
        h.val_type = A->val_type; h.b_type = b_type; h.c_type = c_type;
        h.tile_type = (b_type == SPMM_F16) ? SPMM_F16 : SPMM_BF16;
        h.opts = o;
        h.win_tile_ptr.push_back(0);
        h.win_part.push_back(0);
        h.tile_val_ptr.push_back(0);
        h.vitem_ptr.push_back(0);
        // scratch
        const int64_t nb = std::max<int64_t>(1, (std::max<int64_t>(m, 1) + kTile - 1) / kTile);
        size_t off = 0;
        auto carve = [&](size_t bytes) { off = (off + 255) & ~size_t(255); size_t at = off; off += bytes; return at; };
        const size_t o_cost = carve(8 * (size_t)std::max<int64_t>(m, 1)),
                     o_start = carve(8 * (size_t)std::max<int64_t>(m, 1)),
                     o_ns64 = carve(8 * (size_t)std::max<int64_t>(m, 1)),
                     o_flag = carve(8 * (size_t)std::max<int64_t>(m, 1)),
                     o_idx = carve(8 * (size_t)std::max<int64_t>(m, 1)),
                     o_nseg = carve(4 * (size_t)std::max<int64_t>(m, 1)),
                     o_rp32 = carve(4 * (size_t)(m + 1)),
                     o_sums = carve(8 * (size_t)(nb + 1)),
                     o_sums2 = carve(8 * (size_t)(nb + 1)),
                     o_seen = carve((size_t)std::max<int64_t>(k, 1)),
                     o_cnt = carve(64);
        DevBuf scratch;
        SPMM_TRY_HIP(hipMalloc(&scratch.p, off), "hipMalloc(device plan scratch)");
        auto at = [&](size_t o2) { return static_cast<uint8_t *>(scratch.p) + o2; };
        auto *cost = reinterpret_cast<int64_t *>(at(o_cost));
        auto *start = reinterpret_cast<int64_t *>(at(o_start));
        auto *ns64 = reinterpret_cast<int64_t *>(at(o_ns64));
        auto *flag = reinterpret_cast<int64_t *>(at(o_flag));
        auto *idx = reinterpret_cast<int64_t *>(at(o_idx));
        auto *nseg = reinterpret_cast<int32_t *>(at(o_nseg));
        auto *rp32 = reinterpret_cast<int32_t *>(at(o_rp32));
        auto *sums = reinterpret_cast<int64_t *>(at(o_sums));
        auto *sums2 = reinterpret_cast<int64_t *>(at(o_sums2));
        auto *seen = at(o_seen);
        auto *bad = reinterpret_cast<int32_t *>(at(o_cnt));
        auto *kcount = reinterpret_cast<unsigned long long *>(at(o_cnt) + 8);
        SPMM_TRY_HIP(hipMemsetAsync(seen, 0, (size_t)std::max<int64_t>(k, 1), s), "hipMemsetAsync");
        SPMM_TRY_HIP(hipMemsetAsync(at(o_cnt), 0, 64, s), "hipMemsetAsync");
        // 1. rows and columns, checked before anything is indexed by them
        hipLaunchKernelGGL(k_rows, dim3(blocks_for(m + 1)), dim3(kThreads), 0, s, m, nnz, A->rowptr,
                           o.seg_len, cost, ns64, nseg, rp32, bad);
        if (nnz > 0)
            hipLaunchKernelGGL(k_cols, dim3((unsigned)std::min<int64_t>(blocks_for(nnz), 65536)), dim3(kThreads),
                               0, s, nnz, k, A->colidx, seen, bad);
        SPMM_TRY_HIP(hipGetLastError(), "device plan kernels");
        int32_t bad_h = 0;
        SPMM_TRY_HIP(hipMemcpyAsync(&bad_h, bad, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (bad_h & 1) return set_error(SPMM_ERR_INVALID, "rowptr not monotone from 0 to nnz");
        if (bad_h & 2) return set_error(SPMM_ERR_INVALID, "column index out of range");
        // 2. item cut and segment total
        int64_t V = 0, S = 0;
        if (m > 0) {
            SPMM_TRY_HIP(scan64(cost, start, m, 0, sums, s), "scan");
            hipLaunchKernelGGL(k_item_flags, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, start,
                               (int64_t)o.item_cost, flag);
            SPMM_TRY_HIP(scan64(flag, idx, m, 1, sums, s), "scan");
            SPMM_TRY_HIP(scan64(ns64, start, m, 0, sums2, s), "scan");  // only its total is used
            SPMM_TRY_HIP(hipMemcpyAsync(&V, sums + ((m + kTile - 1) / kTile), 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(hipMemcpyAsync(&S, sums2 + ((m + kTile - 1) / kTile), 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        if (V > INT32_MAX || S > INT32_MAX) return set_error(SPMM_ERR_UNSUPPORTED, "too many items");
        // 3. the plan allocation (layout as an uploaded plan: every array is
        // followed by at least 16 zero bytes, which the kernels' clamped loads
        // of an empty range may read)
        const bool sorted = o.pipeline == 3 && m > 0;
        size_t poff = 0;
        std::vector<size_t> tails;  // offsets of the 16-byte zero tails
        auto pcarve = [&](size_t bytes) {
            poff = (poff + 255) & ~size_t(255);
            size_t a = poff;
            tails.push_back(a + bytes);
            poff += bytes + 16;
            return a;
        };
        const size_t p_rem_ptr = pcarve(4 * (size_t)(m + 1)), p_rem_col = pcarve(4 * (size_t)nnz),
                     p_rem_val = pcarve((size_t)sval * (size_t)nnz),
                     p_vec = pcarve(sorted ? 4 * (size_t)m : 0), p_vptr = pcarve(4 * (size_t)(V + 1)),
                     p_vseg = pcarve(4 * (size_t)V), p_sb = pcarve(4 * (size_t)S),
                     p_se = pcarve(4 * (size_t)S), p_sr = pcarve(4 * (size_t)S),
                     p_so = pcarve(4 * (size_t)S);
        const size_t ptotal = std::max<size_t>(poff, 256);
        int dev = 0;
        SPMM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
        void *d = nullptr;
        hipError_t he = hipMalloc(&d, ptotal);
        if (he != hipSuccess) return set_error(SPMM_ERR_OOM, std::string("hipMalloc(plan): ") + hipGetErrorString(he));
        DevBuf plan_mem;
        plan_mem.p = d;
        auto pat = [&](size_t a) { return static_cast<uint8_t *>(d) + a; };
        auto *vitem_ptr = reinterpret_cast<int32_t *>(pat(p_vptr));
        auto *vitem_seg = reinterpret_cast<int32_t *>(pat(p_vseg));
        auto *order = sorted ? reinterpret_cast<int32_t *>(pat(p_vec)) : nullptr;
        auto *seg_begin = reinterpret_cast<int32_t *>(pat(p_sb));
        auto *seg_end = reinterpret_cast<int32_t *>(pat(p_se));
        auto *seg_row = reinterpret_cast<int32_t *>(pat(p_sr));  // row of each segment
        auto *seg_order = reinterpret_cast<int32_t *>(pat(p_so));  // sort keys, then the launch order
        for (size_t t : tails)
            SPMM_TRY_HIP(hipMemsetAsync(pat(t), 0, 16, s), "hipMemsetAsync");
        SPMM_TRY_HIP(hipMemcpyAsync(pat(p_rem_ptr), rp32, 4 * (size_t)(m + 1), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        if (nnz > 0) {
            SPMM_TRY_HIP(hipMemcpyAsync(pat(p_rem_col), A->colidx, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(hipMemcpyAsync(pat(p_rem_val), A->vals, (size_t)sval * (size_t)nnz, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        }
        if (m > 0) {
            hipLaunchKernelGGL(k_item_ptr, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, flag, idx, vitem_ptr);
            // 4. launch order, segment ids and ranges
            if (sorted)
                hipLaunchKernelGGL(k_item_sort, dim3((unsigned)std::max<int64_t>(1, (V + 3) / 4)), dim3(kThreads), 0,
                                   s, V, vitem_ptr, rp32, nseg, order);
            hipLaunchKernelGGL(k_exec_nseg, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, order, nseg, ns64);
            SPMM_TRY_HIP(scan64(ns64, start, m, 0, sums, s), "scan");
            hipLaunchKernelGGL(k_item_seg, dim3(blocks_for(V)), dim3(kThreads), 0, s, V, vitem_ptr, start, vitem_seg);
            hipLaunchKernelGGL(k_segments, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, S, o.seg_len, order, nseg,
                               rp32, start, seg_begin, seg_end, seg_row);
            if (S > 0)
                hipLaunchKernelGGL(k_seg_keys, dim3(blocks_for(S)), dim3(kThreads), 0, s, S, seg_begin, seg_end,
                                   reinterpret_cast<const int32_t *>(pat(p_rem_col)), seg_order);
        }
        if (k > 0)
            hipLaunchKernelGGL(k_count_seen, dim3((unsigned)std::min<int64_t>(blocks_for(k), 4096)), dim3(kThreads),
                               0, s, k, seen, kcount);
        SPMM_TRY_HIP(hipGetLastError(), "device plan kernels");
        // O(m) schedule arrays to the host (statistics, workspace size, checks)
        h.rem_ptr32.resize(m + 1);
        h.nseg.resize(m);
        h.vitem_ptr.resize(V + 1);
        h.vitem_seg.resize(V);
        h.seg_begin.resize(S);
        h.seg_end.resize(S);
        h.seg_row.resize(S);
        if (sorted) h.vexec.resize(m);
        unsigned long long kref = 0;
        auto d2h = [&](void *dst, const void *src, size_t bytes) {
            return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
        };
        SPMM_TRY_HIP(d2h(h.rem_ptr32.data(), rp32, 4 * (size_t)(m + 1)), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.nseg.data(), nseg, 4 * (size_t)m), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.vitem_ptr.data(), vitem_ptr, m > 0 ? 4 * (size_t)(V + 1) : 0), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.vitem_seg.data(), vitem_seg, 4 * (size_t)V), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.seg_begin.data(), seg_begin, 4 * (size_t)S), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.seg_end.data(), seg_end, 4 * (size_t)S), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(h.seg_row.data(), seg_row, 4 * (size_t)S), "hipMemcpyAsync");
        std::vector<int32_t> seg_key((size_t)S);
        SPMM_TRY_HIP(d2h(seg_key.data(), seg_order, 4 * (size_t)S), "hipMemcpyAsync");
        if (sorted) SPMM_TRY_HIP(d2h(h.vexec.data(), order, 4 * (size_t)m), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(&kref, kcount, 8), "hipMemcpyAsync");
        SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        // Launch order of the segments by the column of their middle entry
        // (stable), as for an uploaded host plan: segments that run together
        // gather from one stretch of B.  C does not depend on the order.
        const std::vector<int32_t> so = order_by_key(seg_key);
        bool so_id = true;
        for (int64_t i = 0; i < S && so_id; ++i) so_id = so[i] == (int32_t)i;
        if (!so_id) {
            SPMM_TRY_HIP(hipMemcpyAsync(seg_order, so.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        h.rem_ptr.assign(h.rem_ptr32.begin(), h.rem_ptr32.end());
        h.vector_rows.resize(m);
        std::iota(h.vector_rows.begin(), h.vector_rows.end(), 0);
        h.identity_rows = true;
        h.k_ref = (int64_t)kref;
        derive_exec_tables(h);
        // the device plan
        DevPlan &dp = p->dp;
        dp.m = (int32_t)m;
        dp.n = n;
        dp.seg_len = o.seg_len;
        dp.H = o.window_h;
        dp.kt = o.kt;
        dp.n_vitems = (int32_t)V;
        dp.n_seg = (int32_t)S;
        dp.n_win = 0;
        dp.rem_ptr = reinterpret_cast<const int32_t *>(pat(p_rem_ptr));
        dp.rem_col = reinterpret_cast<const int32_t *>(pat(p_rem_col));
        dp.rem_val = pat(p_rem_val);
        dp.vec_rows = order;
        dp.vitem_ptr = vitem_ptr;
        dp.vitem_seg = vitem_seg;
        dp.seg_begin = seg_begin;
        dp.seg_end = seg_end;
        dp.seg_order = so_id ? nullptr : seg_order;
        dp.seg_row = seg_row;
        dp.seg_win = nullptr;  // no windows
        dp.win_dep = nullptr;
        dp.win_nsseg = nullptr;
        dp.win_row_sid = nullptr;
        dp.n_dep = 0;
        dp.n_wpart = 0;
        dp.win_tmax = kWinTiles;
        p->dev = d;
        p->dev_bytes = ptotal;
        p->device = dev;
        p->rem_device_only = true;
        plan_mem.p = nullptr;  // owned by the plan now
        *out = p.release();
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while building a device plan");
    }
}
