// devplan.hpp -- the uploaded plan as seen by the kernels, and kernel launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace spmm {

// Pointers into one device allocation (see runtime.hip for the layout).
struct DevPlan {
    int32_t m, n;              // rows of A / C, columns of B / C
    int32_t seg_len;           // remainder entries per segment (longer rows are split)
    int32_t H, kt;             // window height, K-tile width (32)
    int32_t n_vitems, n_seg, n_win;
    const int32_t *rem_ptr;    // [m+1]
    const int32_t *rem_col;    // [nnz_rem]
    const void *rem_val;       // [nnz_rem] of the value type
    const int32_t *vec_rows;   // [n_vector_rows] or null when every row is a vector row
    const int32_t *vitem_ptr;  // [n_vitems+1]
    const int32_t *vitem_seg;  // [n_vitems]
    const int32_t *seg_begin;  // [n_seg]
    const int32_t *seg_end;    // [n_seg]
    const int32_t *seg_order;  // [n_seg] launch order of segments, or null for id order
    const int32_t *windows;    // [n_win*H]
    const int32_t *win_tile_ptr;  // [n_win+1]
    const int32_t *win_seg;    // [n_win]
    const int32_t *win_order;  // [n_win], or null when windows run in id order
    const int32_t *tile_cols;  // [T*kt]
    const uint32_t *tile_bitmap;  // [T*H]
    const int32_t *tile_val_ptr;  // [T+1]
    const uint16_t *tile_vals;
    int32_t n_wpart, win_tmax;  // window partial items; tiles an owner item computes itself
    const int32_t *win_part;    // [n_win+1]
    const int32_t *wpart_win;   // [n_wpart]
    const int32_t *wpart_t0;    // [n_wpart]
    const int32_t *wpart_t1;    // [n_wpart]
    const uint16_t *zeros;      // 256 zero bytes (source of staged padding columns)
    // co-scheduled execution (last-finisher combine)
    const int32_t *seg_row;     // [n_seg] row of each segment
    const int32_t *seg_win;     // [n_seg] window holding the segment's row, -1 for a vector row;
                                // null when the plan has no windows
    const int32_t *win_dep;     // [n_win] slot of a window whose result needs other items (partial
                                // tiles or split rows), else -1; null when the plan has no windows
    const int32_t *win_nsseg;   // [n_win] segments of the window's split rows
    const int32_t *win_row_sid; // [n_win*H] first segment of a window row split into segments, else -1
    int32_t n_dep;              // windows with a slot
};

// Launch geometry and operand description of one execution.
struct RunArgs {
    const void *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    float *work;        // segment partial sums [n_seg * work_ld], then window partials
                        // [n_wpart * H * work_ld]
    int32_t work_ld;    // row stride of `work` (N rounded up to 4)
    int32_t vec_ok;     // 16-byte chunks usable for B and C
    int32_t np;         // columns per panel of the vector / segment kernels
    int32_t n_panels;
    int32_t lpr_log2;   // log2(lanes per entry group) for the vector / segment kernels
    int32_t xcd;        // remap consecutive items onto one XCD
    int32_t win_panels; // panels of the window items (win_np columns each)
    int32_t win_np;     // columns per window panel: 128, or 64 / 32 for 16-bit B with N <= 64
    int32_t win_lpr_log2;
    int32_t cold_aux;   // buffer-load policy bits for non-hot B rows; -1: plain loads for all
    uint32_t b_rec;     // bytes of B reachable through a buffer resource (its span);
                        // 0 when B spans 4 GiB or more (predicated plain loads)
    int32_t pipeline;   // vector kernel variant: 0 row by row, 1 row-pipelined, 2 short rows packed,
                        // 3 rows packed by size class
    // co-scheduled execution
    int32_t *cnt;       // arrival counters: [n_panels * n_seg] per split vector row (at its first
                        // segment id), then [win_panels * n_dep] per window slot; zero between runs
    float *dep;         // window slots: [n_dep][2][H][work_ld] (MFMA result, rows' remainders)
    uint32_t ws_rec;    // bytes of the workspace (below 4 GiB for a co-scheduled run)
    int32_t seg_blocks; // workgroups of segment waves in a fused launch (a multiple of 8)
    int32_t vec_blocks; // workgroups of vector-item waves
    int32_t wpart_blocks; // workgroups of window partial items in a fused launch (a multiple of 8)
    int32_t win_blocks;   // workgroups of window owner items
};

// One matrix of a batched execution.  `*_end` are exclusive prefix sums of
// the global item counts (segment waves, vector waves, window workgroups), so
// a persistent kernel can walk the table forward as its item ids increase.
struct BatchEntry {
    DevPlan P;
    RunArgs a;
    int32_t seg_end, vec_end, win_end, wpart_end;      // exclusive prefix over the table
    int32_t seg_base, vec_base, win_base, wpart_base;  // matrix item index of the first item
};

// An entry is a contiguous range of one matrix's items of each kind, either
// the whole matrix or one of 8 chunks of it.  Entries are grouped by the XCD
// they are assigned to; x_* hold, per XCD x, the first entry and the first
// item of each kind (exclusive prefix sums, 9 values each).  Workgroup b of a
// persistent kernel runs on XCD b % 8 and walks only its XCD's items.
struct BatchHeader {
    int32_t count, total_seg, total_vec, total_win, total_wpart, pad[3];
    int32_t x_entry[9], x_seg[9], x_vec[9], x_win[9], x_wpart[9];
};

// Workgroup counts of the batched kernels: segment kernel, vector kernel and
// the two window kernels (partial items, then owners).
struct BatchGrids {
    unsigned seg = 0, vec = 0, win = 0;
};
// Persistent batched launches over a device table (header + entries).
hipError_t launch_batch(const BatchHeader *hdr, const BatchEntry *tab, int32_t val_t, int32_t b_t,
                        int32_t tile_t, int vec_ok, int cpl, int var, const BatchGrids &grids,
                        hipStream_t s);
// Resident workgroups per CU of each batched kernel of this variant.
hipError_t batch_occupancy(int32_t val_t, int32_t b_t, int32_t tile_t, int vec_ok, int cpl,
                           int var, BatchGrids *per_cu);

// dtype codes as in spmm.h
hipError_t launch_segment(const DevPlan &P, int32_t val_t, int32_t b_t, const RunArgs &a,
                          hipStream_t s);
hipError_t launch_vector(const DevPlan &P, int32_t val_t, int32_t b_t, const RunArgs &a,
                         hipStream_t s);
hipError_t launch_window(const DevPlan &P, int32_t val_t, int32_t b_t, int32_t tile_t,
                         const RunArgs &a, hipStream_t s);
hipError_t launch_window_partial(const DevPlan &P, int32_t val_t, int32_t b_t, int32_t tile_t,
                                 const RunArgs &a, hipStream_t s);
hipError_t launch_copy(const float4 *src, float4 *dst, int64_t n4, hipStream_t s);

// co-scheduled execution (fused.hip): the vector path (segments + vector
// items), the MFMA path (window partials + owners), or both in one grid;
// RunArgs' cnt, dep and *_blocks must be set.
// Events that the next kernel launched through launch_kernel on this thread
// records around itself, inside its own dispatch (a timed run sets them; no
// separate marker commands sit between the run's kernels).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &launch_events();

template <typename F, typename... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args) {
    LaunchEvents &ev = launch_events();
    if (ev.start) {
        const LaunchEvents e = ev;
        ev = LaunchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e.start, e.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

hipError_t launch_vector_path(const DevPlan &P, int32_t val_t, int32_t b_t, const RunArgs &a,
                              hipStream_t s);
hipError_t launch_mfma_path(const DevPlan &P, int32_t val_t, int32_t b_t, int32_t tile_t,
                            const RunArgs &a, hipStream_t s);
bool one_grid_supported(int32_t b_t, const RunArgs &a);
hipError_t launch_one_grid(const DevPlan &P, int32_t val_t, int32_t b_t, int32_t tile_t,
                           const RunArgs &a, hipStream_t s);
// p[0 .. n) = 0 by a kernel (capturable, unlike a memset node)
hipError_t launch_zero(int32_t *p, int64_t n, hipStream_t s);

// chunk width (elements per 16-byte load) of a B type
inline int chunk_elems(int32_t b_t) { return b_t == 0 ? 4 : 8; }

}  // namespace spmm
