// kernels.hip -- gfx950 kernels of the hybrid SpMM: one kernel per item kind
// (segments, vector items, windows, window partials) launched in dependency
// order, the batched persistent kernels, and the copy kernel.  The items
// themselves are in items.hpp.
#include "items.hpp"
namespace spmm {

template <int VT, int BT, int E, int CPL, bool POL>
__global__ __launch_bounds__(256) void segment_kernel(DevPlan P, RunArgs a) {
    const int wid = logical_block(a.xcd) * 4 + wave_id();
    if (wid < P.n_seg * a.n_panels) segment_item<VT, BT, E, CPL, POL>(P, a, wid);
}


template <int VT, int BT, int E, int CPL, int VAR>
__global__ __launch_bounds__(256) void vector_kernel(DevPlan P, RunArgs a) {
    const int wid = logical_block(a.xcd) * 4 + wave_id();
    if (wid < P.n_vitems * a.n_panels) vector_item_var<VT, BT, E, CPL, VAR>(P, a, wid);
}


template <int VT, int BT, int TT, int MB, int E, int CPL, int NPW>
__global__ __launch_bounds__(256) void window_kernel(DevPlan P, RunArgs a) {
    __shared__ WinSmem<MB, NPW> sm;
    const int item = logical_block(a.xcd);
    if (item < P.n_win * a.win_panels)
        window_item<VT, BT, TT, MB, E, CPL, MB, false, NPW>(P, a, item, sm, false);
}

template <int VT, int BT, int TT, int MB, int E, int CPL, int NPW>
__global__ __launch_bounds__(256) void window_partial_kernel(DevPlan P, RunArgs a) {
    __shared__ WinSmem<MB, NPW> sm;
    const int item = logical_block(a.xcd);
    if (item < P.n_wpart * a.win_panels)
        window_item<VT, BT, TT, MB, E, CPL, MB, false, NPW>(P, a, item, sm, true);
}


// ------------------------------------------------------------------------------------------
// Batched persistent kernels: a fixed grid walks the global item space of a
// descriptor table with a static stride, so the item -> matrix lookup only
// moves forward.  Each matrix's items run exactly the code of a single run, so
// a matrix's result is bitwise the same alone and in a batch.

// Persistent walk over one XCD's items of one kind: item ids g of XCD x are
// [xb[x], xb[x+1]); entries of XCD x start at x_entry[x]; `end` gives an
// entry's exclusive item prefix (global over the table), `base` the matrix
// item index of its first item.
#define SPMM_XCD_WALK(XB, END, BASE, PER_WG, BODY)                                     \
    do {                                                                               \
        const int x = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;   \
        const int lo = hdr->XB[x], hi = hdr->XB[x + 1];                                \
        int d = hdr->x_entry[x];                                                       \
        for (int g = lo + local * PER_WG + sub; g < hi; g += nloc * PER_WG) {          \
            while (g >= tab[d].END) ++d;                                               \
            const int item = g - (d ? tab[d - 1].END : 0) + tab[d].BASE;               \
            BODY;                                                                      \
        }                                                                              \
    } while (0)

template <int VT, int BT, int E, int CPL, bool POL>
__global__ __launch_bounds__(256) void batch_segment_kernel(const BatchHeader *__restrict__ hdr,
                                                            const BatchEntry *__restrict__ tab) {
    const int sub = wave_id();
    SPMM_XCD_WALK(x_seg, seg_end, seg_base, 4, (segment_item<VT, BT, E, CPL, POL>(tab[d].P, tab[d].a, item)));
}

// Entries per group and step of the batched vector kernel: 4 for 16-bit B in
// one chunk per lane (the persistent walk over many matrices holds more
// registers, and half the step brings the kernel from 4 to 5 waves per SIMD:
// measured 10.78 -> 10.01 ms on 512 uneven f16 matrices, where single runs
// are faster with 8); a row's sum does not depend on it, so a batched result
// stays bitwise equal to the same plan run alone.
template <int E, int CPL>
constexpr int batch_unroll() { return (E == 8 && CPL == 1) ? 4 : unroll_of<E, CPL>(); }

template <int VT, int BT, int E, int CPL, int VAR>
__global__ __launch_bounds__(256) void batch_vector_kernel(const BatchHeader *__restrict__ hdr,
                                                           const BatchEntry *__restrict__ tab) {
    const int sub = wave_id();
    SPMM_XCD_WALK(x_vec, vec_end, vec_base, 4,
                  (vector_item_var<VT, BT, E, CPL, VAR, false, batch_unroll<E, CPL>()>(tab[d].P, tab[d].a, item)));
}

template <int VT, int BT, int TT, int E, int CPL, int MB>
__device__ __forceinline__ void window_item_h(const BatchEntry &e, int item, WinSmem<4> &sm,
                                              bool partial) {
    window_item<VT, BT, TT, MB, E, CPL, 4>(e.P, e.a, item, sm, partial);
    __syncthreads();  // the next item reuses the LDS
}

template <int VT, int BT, int TT, int E, int CPL, bool PARTIAL>
__global__ __launch_bounds__(256) void batch_window_kernel(const BatchHeader *__restrict__ hdr,
                                                           const BatchEntry *__restrict__ tab) {
    __shared__ WinSmem<4> sm;
    const int sub = 0;
    if (PARTIAL) {
        SPMM_XCD_WALK(x_wpart, wpart_end, wpart_base, 1,
                      (tab[d].P.H == 16 ? window_item_h<VT, BT, TT, E, CPL, 1>(tab[d], item, sm, true)
                       : tab[d].P.H == 32 ? window_item_h<VT, BT, TT, E, CPL, 2>(tab[d], item, sm, true)
                                          : window_item_h<VT, BT, TT, E, CPL, 4>(tab[d], item, sm, true)));
    } else {
        SPMM_XCD_WALK(x_win, win_end, win_base, 1,
                      (tab[d].P.H == 16 ? window_item_h<VT, BT, TT, E, CPL, 1>(tab[d], item, sm, false)
                       : tab[d].P.H == 32 ? window_item_h<VT, BT, TT, E, CPL, 2>(tab[d], item, sm, false)
                                          : window_item_h<VT, BT, TT, E, CPL, 4>(tab[d], item, sm, false)));
    }
}

// Streaming copy used as the achievable-bandwidth reference: one 16-byte
// load and store per lane per round over a large grid (measured on gfx950:
// 5.4 TB/s read + write over 1 GiB; four loads in flight per lane over an
// eight-workgroups-per-CU grid reached only 4.5 TB/s).
__global__ __launch_bounds__(256) void copy_kernel(const f32x4 *__restrict__ src,
                                                   f32x4 *__restrict__ dst, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ------------------------------------------------------------------------------------------
// launchers

static inline unsigned grid_for_waves(int64_t waves) { return (unsigned)((waves + 3) / 4); }

template <int VT, int BT, bool POL>
static hipError_t seg_dispatch_pol(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    const int64_t waves = (int64_t)P.n_seg * a.n_panels;
    if (waves == 0) return hipSuccess;
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    const int chunks = a.vec_ok ? (a.np + EV - 1) / EV : a.np;
    dim3 grid(grid_for_waves(waves)), block(256);
    if (a.vec_ok) {
        if (chunks <= 64) launch_kernel((segment_kernel<VT, BT, EV, 1, POL>), grid, block, 0, s, P, a);
        else launch_kernel((segment_kernel<VT, BT, EV, 2, POL>), grid, block, 0, s, P, a);
    } else {
        launch_kernel((segment_kernel<VT, BT, 1, 2, POL>), grid, block, 0, s, P, a);
    }
    return hipGetLastError();
}

template <int VT, int BT>
static hipError_t seg_dispatch(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    // the per-entry cache-policy choice only for plans with a cold policy
    return a.cold_aux >= 0 ? seg_dispatch_pol<VT, BT, true>(P, a, s)
                           : seg_dispatch_pol<VT, BT, false>(P, a, s);
}

template <int VT, int BT, int VAR>
static hipError_t vec_dispatch_var(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    const int64_t waves = (int64_t)P.n_vitems * a.n_panels;
    if (waves == 0) return hipSuccess;
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    const int chunks = a.vec_ok ? (a.np + EV - 1) / EV : a.np;
    dim3 grid(grid_for_waves(waves)), block(256);
    if (a.vec_ok) {
        if (chunks <= 64) launch_kernel((vector_kernel<VT, BT, EV, 1, VAR>), grid, block, 0, s, P, a);
        else launch_kernel((vector_kernel<VT, BT, EV, 2, VAR>), grid, block, 0, s, P, a);
    } else {
        launch_kernel((vector_kernel<VT, BT, 1, 2, VAR>), grid, block, 0, s, P, a);
    }
    return hipGetLastError();
}

template <int VT, int BT>
static hipError_t vec_dispatch(const DevPlan &P, const RunArgs &a, hipStream_t s) {
    if (a.pipeline == 3) return vec_dispatch_var<VT, BT, 3>(P, a, s);
    if (a.pipeline == 2) return vec_dispatch_var<VT, BT, 2>(P, a, s);
    if (a.pipeline == 1) return vec_dispatch_var<VT, BT, 1>(P, a, s);
    return vec_dispatch_var<VT, BT, 0>(P, a, s);
}

template <int VT, int BT, int TT>
static hipError_t win_dispatch(const DevPlan &P, const RunArgs &a, hipStream_t s, bool partial) {
    const int64_t wgs = (int64_t)(partial ? P.n_wpart : P.n_win) * a.win_panels;
    if (wgs == 0) return hipSuccess;
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    dim3 grid((unsigned)wgs), block(256);
#define SPMM_WIN_NP(MB, NP)                                                                          \
    do {                                                                                             \
        if (partial)                                                                                 \
            launch_kernel((window_partial_kernel<VT, BT, TT, MB, EV, 1, NP>), grid, block, 0, s, P, a); \
        else                                                                                         \
            launch_kernel((window_kernel<VT, BT, TT, MB, EV, 1, NP>), grid, block, 0, s, P, a);  \
    } while (0)
#define SPMM_WIN(MB)                                                                                 \
    do {                                                                                             \
        if (!a.vec_ok) {                                                                             \
            if (partial)                                                                             \
                launch_kernel((window_partial_kernel<VT, BT, TT, MB, 1, 2, 128>), grid, block, 0, s, P, a); \
            else                                                                                     \
                launch_kernel((window_kernel<VT, BT, TT, MB, 1, 2, 128>), grid, block, 0, s, P, a); \
        } else if constexpr (BT == DT_F32) {                                                         \
            SPMM_WIN_NP(MB, 128);                                                                    \
        } else {                                                                                     \
            if (a.win_np == 128) SPMM_WIN_NP(MB, 128);                                               \
            else if (a.win_np == 64) SPMM_WIN_NP(MB, 64);                                            \
            else SPMM_WIN_NP(MB, 32);                                                                \
        }                                                                                            \
    } while (0)
    switch (P.H) {
    case 16: SPMM_WIN(1); break;
    case 32: SPMM_WIN(2); break;
    case 64: SPMM_WIN(4); break;
    default: return hipErrorInvalidValue;
    }
#undef SPMM_WIN
#undef SPMM_WIN_NP
    return hipGetLastError();
}

hipError_t launch_segment(const DevPlan &P, int32_t vt, int32_t bt, const RunArgs &a, hipStream_t s) {
    if (vt == DT_F32 && bt == DT_F32) return seg_dispatch<DT_F32, DT_F32>(P, a, s);
    if (vt == DT_F32 && bt == DT_BF16) return seg_dispatch<DT_F32, DT_BF16>(P, a, s);
    if (vt == DT_BF16 && bt == DT_BF16) return seg_dispatch<DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_F16 && bt == DT_F16) return seg_dispatch<DT_F16, DT_F16>(P, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_vector(const DevPlan &P, int32_t vt, int32_t bt, const RunArgs &a, hipStream_t s) {
    if (vt == DT_F32 && bt == DT_F32) return vec_dispatch<DT_F32, DT_F32>(P, a, s);
    if (vt == DT_F32 && bt == DT_BF16) return vec_dispatch<DT_F32, DT_BF16>(P, a, s);
    if (vt == DT_BF16 && bt == DT_BF16) return vec_dispatch<DT_BF16, DT_BF16>(P, a, s);
    if (vt == DT_F16 && bt == DT_F16) return vec_dispatch<DT_F16, DT_F16>(P, a, s);
    return hipErrorInvalidValue;
}

static hipError_t window_any(const DevPlan &P, int32_t vt, int32_t bt, int32_t tt, const RunArgs &a,
                             hipStream_t s, bool partial) {
    if (vt == DT_F32 && bt == DT_F32 && tt == DT_BF16) return win_dispatch<DT_F32, DT_F32, DT_BF16>(P, a, s, partial);
    if (vt == DT_F32 && bt == DT_BF16 && tt == DT_BF16) return win_dispatch<DT_F32, DT_BF16, DT_BF16>(P, a, s, partial);
    if (vt == DT_BF16 && bt == DT_BF16 && tt == DT_BF16) return win_dispatch<DT_BF16, DT_BF16, DT_BF16>(P, a, s, partial);
    if (vt == DT_F16 && bt == DT_F16 && tt == DT_F16) return win_dispatch<DT_F16, DT_F16, DT_F16>(P, a, s, partial);
    return hipErrorInvalidValue;
}

hipError_t launch_window(const DevPlan &P, int32_t vt, int32_t bt, int32_t tt, const RunArgs &a,
                         hipStream_t s) {
    return window_any(P, vt, bt, tt, a, s, false);
}

hipError_t launch_window_partial(const DevPlan &P, int32_t vt, int32_t bt, int32_t tt,
                                 const RunArgs &a, hipStream_t s) {
    return window_any(P, vt, bt, tt, a, s, true);
}

template <int VT, int BT, int TT, int E, int CPL, int VAR>
static hipError_t batch_variant(const BatchHeader *hdr, const BatchEntry *tab, const BatchGrids &g,
                                hipStream_t s, BatchGrids *occ) {
    if (occ) {
        int o = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &o, batch_segment_kernel<VT, BT, E, CPL, VAR == 0>, 256, 0);
        if (e != hipSuccess) return e;
        occ->seg = (unsigned)o;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, batch_vector_kernel<VT, BT, E, CPL, VAR>, 256, 0);
        if (e != hipSuccess) return e;
        occ->vec = (unsigned)o;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &o, batch_window_kernel<VT, BT, TT, E, CPL, false>, 256, 0);
        occ->win = (unsigned)o;
        return e;
    }
    // phase 1: partial sums (segments, window tile chunks); phase 2: owners
    hipLaunchKernelGGL((batch_segment_kernel<VT, BT, E, CPL, VAR == 0>), dim3(g.seg), dim3(256), 0, s, hdr, tab);
    hipLaunchKernelGGL((batch_window_kernel<VT, BT, TT, E, CPL, true>), dim3(g.win), dim3(256), 0, s,
                       hdr, tab);
    hipLaunchKernelGGL((batch_vector_kernel<VT, BT, E, CPL, VAR>), dim3(g.vec), dim3(256), 0, s, hdr, tab);
    hipLaunchKernelGGL((batch_window_kernel<VT, BT, TT, E, CPL, false>), dim3(g.win), dim3(256), 0,
                       s, hdr, tab);
    return hipGetLastError();
}

template <int VT, int BT, int TT, int VAR>
static hipError_t batch_types_var(const BatchHeader *hdr, const BatchEntry *tab, int vec_ok,
                                  int cpl, const BatchGrids &g, hipStream_t s, BatchGrids *occ) {
    constexpr int EV = BT == DT_F32 ? 4 : 8;
    if (!vec_ok) return batch_variant<VT, BT, TT, 1, 2, VAR>(hdr, tab, g, s, occ);
    if (cpl == 1) return batch_variant<VT, BT, TT, EV, 1, VAR>(hdr, tab, g, s, occ);
    return batch_variant<VT, BT, TT, EV, 2, VAR>(hdr, tab, g, s, occ);
}

template <int VT, int BT, int TT>
static hipError_t batch_types(const BatchHeader *hdr, const BatchEntry *tab, int vec_ok, int cpl,
                              int var, const BatchGrids &g, hipStream_t s, BatchGrids *occ) {
    if (var == 3) return batch_types_var<VT, BT, TT, 3>(hdr, tab, vec_ok, cpl, g, s, occ);
    if (var == 2) return batch_types_var<VT, BT, TT, 2>(hdr, tab, vec_ok, cpl, g, s, occ);
    if (var == 1) return batch_types_var<VT, BT, TT, 1>(hdr, tab, vec_ok, cpl, g, s, occ);
    return batch_types_var<VT, BT, TT, 0>(hdr, tab, vec_ok, cpl, g, s, occ);
}

static hipError_t batch_any(const BatchHeader *hdr, const BatchEntry *tab, int32_t vt, int32_t bt,
                            int32_t tt, int vec_ok, int cpl, int var, const BatchGrids &g,
                            hipStream_t s, BatchGrids *occ) {
    if (vt == DT_F32 && bt == DT_F32 && tt == DT_BF16)
        return batch_types<DT_F32, DT_F32, DT_BF16>(hdr, tab, vec_ok, cpl, var, g, s, occ);
    if (vt == DT_F32 && bt == DT_BF16 && tt == DT_BF16)
        return batch_types<DT_F32, DT_BF16, DT_BF16>(hdr, tab, vec_ok, cpl, var, g, s, occ);
    if (vt == DT_BF16 && bt == DT_BF16 && tt == DT_BF16)
        return batch_types<DT_BF16, DT_BF16, DT_BF16>(hdr, tab, vec_ok, cpl, var, g, s, occ);
    if (vt == DT_F16 && bt == DT_F16 && tt == DT_F16)
        return batch_types<DT_F16, DT_F16, DT_F16>(hdr, tab, vec_ok, cpl, var, g, s, occ);
    return hipErrorInvalidValue;
}

hipError_t launch_batch(const BatchHeader *hdr, const BatchEntry *tab, int32_t vt, int32_t bt,
                        int32_t tt, int vec_ok, int cpl, int var, const BatchGrids &grids,
                        hipStream_t s) {
    return batch_any(hdr, tab, vt, bt, tt, vec_ok, cpl, var, grids, s, nullptr);
}

hipError_t batch_occupancy(int32_t vt, int32_t bt, int32_t tt, int vec_ok, int cpl, int var,
                           BatchGrids *per_cu) {
    return batch_any(nullptr, nullptr, vt, bt, tt, vec_ok, cpl, var, BatchGrids{}, nullptr, per_cu);
}

hipError_t launch_copy(const float4 *src, float4 *dst, int64_t n4, hipStream_t s) {
    if (n4 <= 0) return hipSuccess;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const f32x4 *>(src), reinterpret_cast<f32x4 *>(dst), n4);
    return hipGetLastError();
}

}  // namespace spmm

