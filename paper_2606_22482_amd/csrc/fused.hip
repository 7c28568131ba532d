// fused.hip -- co-scheduled execution of a plan (gfx950).
//
// The paper runs its two engines side by side and balances them (Sec. 5.3,
// Fig. 10 pipelining): on CDNA4 the matrix cores and the vector ALUs sit in
// the same CU, so "side by side" means MFMA window work and FP32 gather work
// resident on the CUs at the same time rather than one kernel after another.
// Two launch forms:
//
//   vector path + MFMA path -- two grids, launched on two streams of the
//       caller's stream (fork and join by events), that run concurrently:
//       the vector path (segment waves, then vector-item waves) and the MFMA
//       path (window partial items, then window owners).  Each grid keeps its
//       own register and LDS allocation, so the vector path keeps its
//       occupancy next to the LDS-heavy windows.
//   one grid -- all four item kinds in one launch (workgroup ranges of window
//       partials, window owners, segments, vector items); every workgroup is
//       given the window item's LDS and registers.
//
// Results that need several items are finished by their last contributor
// (items.hpp, co-scheduled execution), so neither form has a barrier or a
// wait between items, and both give C bitwise equal to the serial kernels.
#include <algorithm>

#include "items.hpp"

namespace spmm {

// Workgroup b of the vector path: segment waves first, in their launch order
// and in dispatch order across the XCDs (column-ordered segments then share
// one stretch of B in the Infinity Cache), then the vector items, each XCD
// taking consecutive items.
template <int VT, int BT, int E, int CPL, int VAR>
__device__ __forceinline__ void vector_path(const DevPlan &P, const RunArgs &a, int b) {
    if (b < a.seg_blocks) {
        const int wid = b * 4 + wave_id();
        if (wid < P.n_seg * a.n_panels) segment_item<VT, BT, E, CPL, false, true>(P, a, wid);
    } else {
        const int j = b - a.seg_blocks;
        if (j >= a.vec_blocks) return;
        const int vb = a.xcd ? remap_block(j, a.vec_blocks) : j;
        const int wid = vb * 4 + wave_id();
        if (wid < P.n_vitems * a.n_panels) vector_item_var<VT, BT, E, CPL, VAR, true>(P, a, wid);
    }
}

// Workgroup b of the MFMA path: window partial items first, then the owners
// (in window launch order, each XCD taking consecutive windows).
template <int VT, int BT, int TT, int MB, int E, int CPL, int NPW = 128>
__device__ __forceinline__ void mfma_path(const DevPlan &P, const RunArgs &a, int b, WinSmem<MB, NPW> &sm) {
    if (b < a.wpart_blocks) {
        if (b < P.n_wpart * a.win_panels)
            window_item<VT, BT, TT, MB, E, CPL, MB, true, NPW>(P, a, b, sm, true);
    } else {
        // padding workgroups of the one-grid form (j beyond the range) stay
        // idle: the remap is a permutation of [0, win_blocks) only
        const int j = b - a.wpart_blocks;
        if (j >= a.win_blocks) return;
        const int item = a.xcd ? remap_block(j, a.win_blocks) : j;
        window_item<VT, BT, TT, MB, E, CPL, MB, true, NPW>(P, a, item, sm, false);
    }
}

template <int VT, int BT, int E, int CPL, int VAR>
__global__ __launch_bounds__(256) void vector_path_kernel(DevPlan P, RunArgs a) {
    vector_path<VT, BT, E, CPL, VAR>(P, a, blockIdx.x);
}

template <int VT, int BT, int TT, int MB, int E, int CPL, int NPW>
__global__ __launch_bounds__(256) void mfma_path_kernel(DevPlan P, RunArgs a) {
    __shared__ WinSmem<MB, NPW> sm;
    mfma_path<VT, BT, TT, MB, E, CPL, NPW>(P, a, blockIdx.x, sm);
}

// The MFMA path's workgroups (padded to a multiple of 8), then the vector path's.
template <int VT, int BT, int TT, int MB, int E, int CPL, int VAR>
__global__ __launch_bounds__(256) void one_grid_kernel(DevPlan P, RunArgs a) {
    __shared__ WinSmem<MB> sm;
    const int wb = a.wpart_blocks + ((a.win_blocks + 7) & ~7);
    const int b = blockIdx.x;
    if (b < wb) mfma_path<VT, BT, TT, MB, E, CPL>(P, a, b, sm);
    else vector_path<VT, BT, E, CPL, VAR>(P, a, b - wb);
}

// ------------------------------------------------------------------------------------------
// launchers

template <int VT, int BT, int E, int CPL>
static hipError_t vp_var(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)(a.seg_blocks + a.vec_blocks)), block(256);
    switch (a.pipeline) {
    case 3: launch_kernel((vector_path_kernel<VT, BT, E, CPL, 3>), grid, block, 0, s, P, a); break;
    case 2: launch_kernel((vector_path_kernel<VT, BT, E, CPL, 2>), grid, block, 0, s, P, a); break;
    case 1: launch_kernel((vector_path_kernel<VT, BT, E, CPL, 1>), grid, block, 0, s, P, a); break;
    default: launch_kernel((vector_path_kernel<VT, BT, E, CPL, 0>), grid, block, 0, s, P, a); break;
    }
    return hipGetLastError();
}

template <int VT, int BT>
static hipError_t vp_types(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    if (!a.vec_ok) return vp_var<VT, BT, 1, 2>(P, a, s);
    if ((a.np + EV - 1) / EV <= 64) return vp_var<VT, BT, EV, 1>(P, a, s);
    return vp_var<VT, BT, EV, 2>(P, a, s);
}

hipError_t launch_vector_path(const DevPlan &P, int32_t vt, int32_t bt, const RunArgs &a, hipStream_t s) {
    if (a.seg_blocks + a.vec_blocks == 0) return hipSuccess;
    if (vt == DT_F32 && bt == DT_F32) return vp_types<DT_F32, DT_F32>(P, a, s);
    if (vt == DT_F32 && bt == DT_BF16) return vp_types<DT_F32, DT_BF16>(P, a, s);
    if (vt == DT_BF16 && bt == DT_BF16) return vp_types<DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_F16 && bt == DT_F16) return vp_types<DT_F16, DT_F16>(P, a, s);
    return hipErrorInvalidValue;
}

template <int VT, int BT, int TT, int MB>
static hipError_t mp_mb(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    const dim3 grid((unsigned)(a.wpart_blocks + a.win_blocks)), block(256);
    if (!a.vec_ok) {
        launch_kernel((mfma_path_kernel<VT, BT, TT, MB, 1, 2, 128>), grid, block, 0, s, P, a);
    } else if constexpr (BT == DT_F32) {
        launch_kernel((mfma_path_kernel<VT, BT, TT, MB, EV, 1, 128>), grid, block, 0, s, P, a);
    } else {
        // narrow 16-bit B stages 64- or 32-column panels
        if (a.win_np == 128)
            launch_kernel((mfma_path_kernel<VT, BT, TT, MB, EV, 1, 128>), grid, block, 0, s, P, a);
        else if (a.win_np == 64)
            launch_kernel((mfma_path_kernel<VT, BT, TT, MB, EV, 1, 64>), grid, block, 0, s, P, a);
        else
            launch_kernel((mfma_path_kernel<VT, BT, TT, MB, EV, 1, 32>), grid, block, 0, s, P, a);
    }
    return hipGetLastError();
}

template <int VT, int BT, int TT>
static hipError_t mp_types(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    switch (P.H) {
    case 16: return mp_mb<VT, BT, TT, 1>(P, a, s);
    case 32: return mp_mb<VT, BT, TT, 2>(P, a, s);
    case 64: return mp_mb<VT, BT, TT, 4>(P, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mfma_path(const DevPlan &P, int32_t vt, int32_t bt, int32_t tt, const RunArgs &a,
                            hipStream_t s) {
    if (a.wpart_blocks + a.win_blocks == 0) return hipSuccess;
    if (vt == DT_F32 && bt == DT_F32 && tt == DT_BF16) return mp_types<DT_F32, DT_F32, DT_BF16>(P, a, s);
    if (vt == DT_F32 && bt == DT_BF16 && tt == DT_BF16) return mp_types<DT_F32, DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_BF16 && bt == DT_BF16 && tt == DT_BF16) return mp_types<DT_BF16, DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_F16 && bt == DT_F16 && tt == DT_F16) return mp_types<DT_F16, DT_F16, DT_F16>(P, a, s);
    return hipErrorInvalidValue;
}

// One grid: built for 16-byte chunks with one chunk per lane, the packed
// vector variants (2, 3), which cover the defaults, and 128-column window
// panels; other plans report hipErrorNotSupported and run as two grids.
template <int VT, int BT, int TT, int MB>
static hipError_t og_mb(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    const unsigned wb = (unsigned)(a.wpart_blocks + ((a.win_blocks + 7) & ~7));
    const dim3 grid(wb + (unsigned)(a.seg_blocks + a.vec_blocks)), block(256);
    if (a.pipeline == 3)
        launch_kernel((one_grid_kernel<VT, BT, TT, MB, EV, 1, 3>), grid, block, 0, s, P, a);
    else
        launch_kernel((one_grid_kernel<VT, BT, TT, MB, EV, 1, 2>), grid, block, 0, s, P, a);
    return hipGetLastError();
}

template <int VT, int BT, int TT>
static hipError_t og_types(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    switch (P.H) {
    case 16: return og_mb<VT, BT, TT, 1>(P, a, s);
    case 32: return og_mb<VT, BT, TT, 2>(P, a, s);
    case 64: return og_mb<VT, BT, TT, 4>(P, a, s);
    default: return hipErrorInvalidValue;
    }
}

bool one_grid_supported(int32_t b_t, const RunArgs &a) {
    const int ev = b_t == DT_F32 ? 4 : 8;
    return a.vec_ok && (a.np + ev - 1) / ev <= 64 && (a.pipeline == 2 || a.pipeline == 3) &&
           a.win_np == 128;
}

hipError_t launch_one_grid(const DevPlan &P, int32_t vt, int32_t bt, int32_t tt, const RunArgs &a,
                           hipStream_t s) {
    if (!one_grid_supported(bt, a)) return hipErrorNotSupported;
    if (vt == DT_F32 && bt == DT_F32 && tt == DT_BF16) return og_types<DT_F32, DT_F32, DT_BF16>(P, a, s);
    if (vt == DT_F32 && bt == DT_BF16 && tt == DT_BF16) return og_types<DT_F32, DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_BF16 && bt == DT_BF16 && tt == DT_BF16) return og_types<DT_BF16, DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_F16 && bt == DT_F16 && tt == DT_F16) return og_types<DT_F16, DT_F16, DT_F16>(P, a, s);
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void zero_kernel(int32_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

hipError_t launch_zero(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace spmm
