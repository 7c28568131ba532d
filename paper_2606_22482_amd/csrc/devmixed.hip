// devmixed.hip -- a mixed plan partitioned on the device, from a CSR already
// in device memory (Sec. 5.2.2 and Sec. 6.1 preprocessing without moving A
// through the host; Sec. 8.6 overheads).
//
// The partition is the host builder's, step for step, so the plan equals the
// host plan of the same matrix and options array for array:
//   1. rows: Len(r) (Eq. 4) and the row stage Len(r) > t_row (Eq. 5); CSR
//      checks (the host reads the error flag before anything is indexed);
//      the window slots: original ranges (slot i is row i when it passes),
//      or the passing rows compacted in row order (a stream compaction),
//      optionally stably sorted by decreasing length (a radix sort of the
//      lengths, which keeps equal lengths in row order) -- window w takes
//      slots [wH, wH + H);
//   2. the column stage of every window w (its slots' rows): the keys
//      (w, column) of its passing rows' entries are sorted and counted, and a
//      column whose count exceeds floor(alpha_c H) is a tile column; tile
//      columns in ascending order are cut into K-tiles of kt, a K-tile is
//      kept when its entry count reaches alpha H kt (Sec. 5.2.1), and a
//      window without a kept tile is dissolved;
//   3. every entry of a kept window's passing rows in a kept K-tile takes its
//      (row, column) slot, the first entry in CSR order of a repeated pair
//      winning (an atomic minimum of entry indices); the others stay in the
//      row's remainder, in CSR order;
//   4. bitmaps (one kt-bit word per window row, LSB first) and the packed
//      values in row-major order over the set bits, f32 values rounded to
//      bf16 to nearest even.
// Only O(m + windows + tiles) arrays come back to the host, which builds the
// schedule (vector items, segments, window items: build_schedule, as for a
// host plan); the remainder and the tiles go device to device into the plan.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
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
constexpr int kKt = 32;

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }
// one wavefront per row, four per workgroup
unsigned row_blocks(int64_t m) { return (unsigned)std::max<int64_t>(1, (m + 3) / 4); }

__device__ __forceinline__ float bf16_bits_of(float f, uint16_t *bits) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) *bits = (uint16_t)((u >> 16) | 0x40u);
    else *bits = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    return f;
}

// rows: checks, passing-entry counts (Len(r) > t_row), int32 row pointers
__global__ __launch_bounds__(kThreads) void k_mrows(int64_t m, int64_t nnz, const int64_t *__restrict__ rowptr,
                                                    int32_t t_row, int64_t *__restrict__ plen,
                                                    int32_t *__restrict__ rp32, int32_t *__restrict__ bad) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r > m) return;
    if (r == m) {
        if (rowptr[m] != nnz) atomicOr(bad, 1);
        rp32[m] = (int32_t)nnz;
        return;
    }
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    const bool ok = b >= 0 && e >= b && e <= nnz && (r != 0 || b == 0);
    if (!ok) atomicOr(bad, 1);
    const int64_t L = ok ? e - b : 0;
    plen[r] = L > (int64_t)t_row ? L : 0;
    rp32[r] = ok ? (int32_t)b : 0;
}

__global__ __launch_bounds__(kThreads) void k_mcols(int64_t nnz, int64_t k, const int32_t *__restrict__ colidx,
                                                    uint8_t *__restrict__ seen, int32_t *__restrict__ bad) {
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kThreads) {
        const int32_t c = colidx[p];
        if (c < 0 || c >= k) atomicOr(bad, 2);
        else seen[c] = 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_mcount_seen(int64_t k, const uint8_t *__restrict__ seen,
                                                          unsigned long long *__restrict__ count) {
    unsigned long long s = 0;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < k; c += (int64_t)gridDim.x * kThreads)
        s += seen[c];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(count, s);
}

// row stage flags (Len(r) > t_row, Eq. 5) for the compacted slot list
__global__ __launch_bounds__(kThreads) void k_passflag(int64_t m, int32_t t_row, const int32_t *__restrict__ rp32,
                                                       int64_t *__restrict__ flag) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < m) flag[r] = (int64_t)(rp32[r + 1] - rp32[r]) > (int64_t)t_row ? 1 : 0;
}

// the passing rows in row order (flag scanned into pos)
__global__ __launch_bounds__(kThreads) void k_compact(int64_t m, const int64_t *__restrict__ flag,
                                                      const int64_t *__restrict__ pos, int32_t *__restrict__ D) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < m && flag[r]) D[pos[r]] = (int32_t)r;
}

__global__ __launch_bounds__(kThreads) void k_lenkeys(int64_t nD, const int32_t *__restrict__ D,
                                                      const int32_t *__restrict__ rp32, int32_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < nD) key[i] = rp32[D[i] + 1] - rp32[D[i]];
}

// slot i of the windows holds row D[i] (-1 past the list); wpos is its inverse
__global__ __launch_bounds__(kThreads) void k_slots(int64_t WH, int64_t nD, const int32_t *__restrict__ D,
                                                    int32_t *__restrict__ slot_row, int32_t *__restrict__ wpos) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= WH) return;
    const int32_t r = i < nD ? D[i] : -1;
    slot_row[i] = r;
    if (r >= 0) wpos[r] = (int32_t)i;
}

// window slot of a passing row: the row itself (original ranges) or its
// position in the compacted / sorted slot list
__device__ __forceinline__ int64_t slot_of(const int32_t *__restrict__ wpos, int64_t r) {
    return wpos ? (int64_t)wpos[r] : r;
}

// keys (window << 32 | column) of the passing rows' entries, row by row
__global__ __launch_bounds__(kThreads) void k_keys(int64_t m, int32_t H, const int32_t *__restrict__ rp32,
                                                   const int32_t *__restrict__ colidx,
                                                   const int64_t *__restrict__ plen,
                                                   const int32_t *__restrict__ wpos,
                                                   const int64_t *__restrict__ kpos, uint64_t *__restrict__ keys) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m || plen[r] == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = rp32[r], e = rp32[r + 1], o = kpos[r];
    const uint64_t w = (uint64_t)(slot_of(wpos, r) / H) << 32;
    for (int64_t p = b + lane; p < e; p += 64) keys[o + (p - b)] = w | (uint32_t)colidx[p];
}

// tile columns: run counts above floor(alpha_c H)
__global__ __launch_bounds__(kThreads) void k_mflag(int64_t n, const int32_t *__restrict__ cnt, int32_t thr,
                                                    int64_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) flag[i] = cnt[i] > thr ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_mscatter(int64_t n, const int64_t *__restrict__ flag,
                                                       const int64_t *__restrict__ pos,
                                                       const uint64_t *__restrict__ key, const int32_t *__restrict__ cnt,
                                                       uint64_t *__restrict__ mkey, int32_t *__restrict__ mcnt) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || !flag[i]) return;
    mkey[pos[i]] = key[i];
    mcnt[pos[i]] = cnt[i];
}

// first tile column of each window (lower bound of w << 32), and the window's K-tile count
__global__ __launch_bounds__(kThreads) void k_wstart(int64_t W, int64_t nmc, const uint64_t *__restrict__ mkey,
                                                     int64_t *__restrict__ start, int64_t *__restrict__ nchunk) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w > W) return;
    const uint64_t want = (uint64_t)w << 32;
    int64_t lo = 0, hi = nmc;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (mkey[mid] < want) lo = mid + 1;
        else hi = mid;
    }
    start[w] = lo;
    (void)nchunk;
}

__global__ __launch_bounds__(kThreads) void k_nchunk(int64_t W, const int64_t *__restrict__ start,
                                                     int64_t *__restrict__ nchunk) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= W) return;
    nchunk[w] = (start[w + 1] - start[w] + kKt - 1) / kKt;
}

// density test of every K-tile (as the host: (double) count >= alpha H kt)
__global__ __launch_bounds__(kThreads) void k_chunks(int64_t W, const int64_t *__restrict__ start,
                                                     const int64_t *__restrict__ cbase,
                                                     const int32_t *__restrict__ mcnt, double keep_thr,
                                                     int64_t *__restrict__ kept) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= W) return;
    const int64_t s0 = start[w], s1 = start[w + 1];
    int64_t c = cbase[w];
    for (int64_t j0 = s0; j0 < s1; j0 += kKt, ++c) {
        int64_t t = 0;
        for (int64_t j = j0; j < min(j0 + kKt, s1); ++j) t += mcnt[j];
        kept[c] = (double)t >= keep_thr ? 1 : 0;
    }
}

// per window: kept K-tiles (for the window compaction) and its first tile id
__global__ __launch_bounds__(kThreads) void k_wkept(int64_t W, const int64_t *__restrict__ cbase,
                                                    const int64_t *__restrict__ kept,
                                                    const int64_t *__restrict__ tile_id,
                                                    int64_t *__restrict__ wkeep, int64_t *__restrict__ wtile0) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= W) return;
    int64_t n = 0;
    for (int64_t c = cbase[w]; c < cbase[w + 1]; ++c) n += kept[c];
    wkeep[w] = n > 0 ? 1 : 0;
    wtile0[w] = cbase[w] < cbase[w + 1] ? tile_id[cbase[w]] : 0;
}

// kept windows: their row slots, first tile, and the tiles' columns
__global__ __launch_bounds__(kThreads) void k_wfill(int64_t W, int64_t m, int32_t H, int32_t t_row,
                                                    const int32_t *__restrict__ rp32,
                                                    const int32_t *__restrict__ slot_row,
                                                    const int64_t *__restrict__ wkeep, const int64_t *__restrict__ widx,
                                                    const int64_t *__restrict__ wtile0,
                                                    int32_t *__restrict__ windows, int32_t *__restrict__ win_tile_ptr) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= W || !wkeep[w]) return;
    const int64_t x = widx[w];
    for (int s = 0; s < H; ++s) {
        const int64_t r = w * H + s;
        if (slot_row) {
            windows[x * H + s] = slot_row[r];
        } else {
            const bool pass = r < m && (int64_t)(rp32[r + 1] - rp32[r]) > (int64_t)t_row;
            windows[x * H + s] = pass ? (int32_t)r : -1;
        }
    }
    win_tile_ptr[x] = (int32_t)wtile0[w];
}

__global__ __launch_bounds__(kThreads) void k_tcols(int64_t W, const int64_t *__restrict__ start,
                                                    const int64_t *__restrict__ cbase, const int64_t *__restrict__ kept,
                                                    const int64_t *__restrict__ tile_id, const uint64_t *__restrict__ mkey,
                                                    int32_t *__restrict__ tile_cols) {
    const int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= W) return;
    const int64_t s0 = start[w], s1 = start[w + 1];
    int64_t c = cbase[w];
    for (int64_t j0 = s0; j0 < s1; j0 += kKt, ++c) {
        if (!kept[c]) continue;
        const int64_t t = tile_id[c];
        for (int j = 0; j < kKt; ++j)
            tile_cols[t * kKt + j] = j0 + j < s1 ? (int32_t)(mkey[j0 + j] & 0xFFFFFFFFu) : -1;
    }
}

// slot of entry p (the row in window slot wH + s, column c) in a kept K-tile, or -1
__device__ __forceinline__ int64_t entry_slot(int64_t w, int s, int32_t c, int32_t H,
                                              const int64_t *__restrict__ start, const int64_t *__restrict__ cbase,
                                              const int64_t *__restrict__ kept, const int64_t *__restrict__ tile_id,
                                              const uint64_t *__restrict__ mkey) {
    const uint64_t want = ((uint64_t)w << 32) | (uint32_t)c;
    int64_t lo = start[w], hi = start[w + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (mkey[mid] < want) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= start[w + 1] || mkey[lo] != want) return -1;
    const int64_t i = lo - start[w], chunk = cbase[w] + i / kKt;
    if (!kept[chunk]) return -1;
    return (tile_id[chunk] * H + s) * kKt + i % kKt;
}

// step 3: the winning (first) entry of every slot
__global__ __launch_bounds__(kThreads) void k_assign(int64_t m, int32_t H, const int32_t *__restrict__ rp32,
                                                     const int32_t *__restrict__ colidx, const int64_t *__restrict__ plen,
                                                     const int32_t *__restrict__ wpos,
                                                     const int64_t *__restrict__ wkeep, const int64_t *__restrict__ start,
                                                     const int64_t *__restrict__ cbase, const int64_t *__restrict__ kept,
                                                     const int64_t *__restrict__ tile_id,
                                                     const uint64_t *__restrict__ mkey, int32_t *__restrict__ src) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m || plen[r] == 0) return;
    const int64_t pos = slot_of(wpos, r), w = pos / H;
    if (!wkeep[w]) return;
    const int s = (int)(pos - w * H), lane = threadIdx.x & 63;
    for (int64_t p = rp32[r] + lane; p < rp32[r + 1]; p += 64) {
        const int64_t slot = entry_slot(w, s, colidx[p], H, start, cbase, kept, tile_id, mkey);
        if (slot >= 0) atomicMin(src + slot, (int32_t)p);
    }
}

// in-tile flags of every entry, and the row's remainder length
__global__ __launch_bounds__(kThreads) void k_intile(int64_t m, int32_t H, const int32_t *__restrict__ rp32,
                                                     const int32_t *__restrict__ colidx, const int64_t *__restrict__ plen,
                                                     const int32_t *__restrict__ wpos,
                                                     const int64_t *__restrict__ wkeep, const int64_t *__restrict__ start,
                                                     const int64_t *__restrict__ cbase, const int64_t *__restrict__ kept,
                                                     const int64_t *__restrict__ tile_id,
                                                     const uint64_t *__restrict__ mkey, const int32_t *__restrict__ src,
                                                     uint8_t *__restrict__ in_tile, int64_t *__restrict__ rem_len) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m) return;
    const int lane = threadIdx.x & 63;
    // a row with entries past the row stage has a window slot; no other row
    // looks one up
    const int64_t pos = plen[r] > 0 ? slot_of(wpos, r) : 0;
    const int64_t w = pos / H, b = rp32[r], e = rp32[r + 1];
    const bool maybe = plen[r] > 0 && wkeep[w];
    const int s = (int)(pos - w * H);
    int64_t tin = 0;
    for (int64_t p = b + lane; p < e; p += 64) {
        bool t = false;
        if (maybe) {
            const int64_t slot = entry_slot(w, s, colidx[p], H, start, cbase, kept, tile_id, mkey);
            t = slot >= 0 && src[slot] == (int32_t)p;
        }
        in_tile[p] = t ? 1 : 0;
        tin += t ? 1 : 0;
    }
    for (int off = 32; off >= 1; off >>= 1) tin += __shfl_xor(tin, off, 64);
    if (lane == 0) rem_len[r] = (e - b) - tin;
}

// the remainder of each row in CSR order (ballot compaction, 64 entries a step)
__global__ __launch_bounds__(kThreads) void k_remainder(int64_t m, int sval, const int32_t *__restrict__ rp32,
                                                        const int32_t *__restrict__ colidx,
                                                        const uint8_t *__restrict__ vals,
                                                        const uint8_t *__restrict__ in_tile,
                                                        const int64_t *__restrict__ rem_ptr,
                                                        int32_t *__restrict__ rem_col, uint8_t *__restrict__ rem_val,
                                                        int32_t *__restrict__ rem_src) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = rp32[r], e = rp32[r + 1];
    int64_t at = rem_ptr[r];
    for (int64_t p0 = b; p0 < e; p0 += 64) {
        const int64_t p = p0 + lane;
        const bool keep = p < e && !in_tile[p];
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const int64_t q = at + __popcll(mask & ((1ull << lane) - 1ull));
            rem_col[q] = colidx[p];
            rem_src[q] = (int32_t)p;
            if (sval == 4) reinterpret_cast<uint32_t *>(rem_val)[q] = reinterpret_cast<const uint32_t *>(vals)[p];
            else reinterpret_cast<uint16_t *>(rem_val)[q] = reinterpret_cast<const uint16_t *>(vals)[p];
        }
        at += __popcll(mask);
    }
}

// bitmap word and value count of every (tile, window row)
__global__ __launch_bounds__(kThreads) void k_bitmap(int64_t TH, const int32_t *__restrict__ src,
                                                     uint32_t *__restrict__ bitmap, int64_t *__restrict__ nval) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= TH) return;
    uint32_t w = 0;
    for (int j = 0; j < kKt; ++j)
        if (src[i * kKt + j] != INT_MAX) w |= 1u << j;
    bitmap[i] = w;
    nval[i] = __popc(w);
}

__global__ __launch_bounds__(kThreads) void k_tvptr(int64_t T, int32_t H, const int64_t *__restrict__ vpos,
                                                    int64_t nv, int32_t *__restrict__ tile_val_ptr) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t > T) return;
    tile_val_ptr[t] = (int32_t)(t < T ? vpos[t * H] : nv);
}

// packed values (row-major over set bits) and their CSR entries
__global__ __launch_bounds__(kThreads) void k_values(int64_t TH, int32_t val_type, const int32_t *__restrict__ src,
                                                     const uint32_t *__restrict__ bitmap,
                                                     const int64_t *__restrict__ vpos, const uint8_t *__restrict__ vals,
                                                     uint16_t *__restrict__ tile_vals, int32_t *__restrict__ tile_src) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= TH) return;
    int64_t q = vpos[i];
    const uint32_t w = bitmap[i];
    for (int j = 0; j < kKt; ++j) {
        if (!((w >> j) & 1u)) continue;
        const int32_t p = src[i * kKt + j];
        uint16_t bits;
        if (val_type == SPMM_F32) bf16_bits_of(reinterpret_cast<const float *>(vals)[p], &bits);
        else bits = reinterpret_cast<const uint16_t *>(vals)[p];
        tile_vals[q] = bits;
        tile_src[q] = p;
        ++q;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill32(int64_t n, int32_t v, int32_t *__restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_mseg_keys(int64_t S, const int32_t *__restrict__ seg_begin,
                                                        const int32_t *__restrict__ seg_end,
                                                        const int32_t *__restrict__ col, int32_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= S) return;
    key[i] = col[((int64_t)seg_begin[i] + seg_end[i] - 1) / 2] & 0x7fffffff;
}

// device memory released when the builder returns
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(T **out, size_t count) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T) + 16);
        if (e == hipSuccess) ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return e;
    }
};

#define SPMM_ALLOC(ptr, count)                                                                    \
    do {                                                                                          \
        if (scratch.get(&(ptr), (size_t)(count)) != hipSuccess)                                   \
            return set_error(SPMM_ERR_OOM, "hipMalloc(device plan scratch)");                     \
    } while (0)

// 0 .. n-1 stably ordered by non-negative keys (two 16-bit counting passes)
std::vector<int32_t> order_by_key32(const std::vector<int32_t> &key) {
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

}  // namespace

namespace spmm {

spmm_status plan_device_mixed(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                              const spmm_opts &o, hipStream_t s, spmm_plan_t **out) {
    std::string err;
    spmm_status st = validate_opts(o, err);
    if (st != SPMM_OK) return set_error(st, err);
    if (o.cold_policy != 0) return set_error(SPMM_ERR_UNSUPPORTED, "device-built plans gather with the default policy");
    if (o.kt != kKt) return set_error(SPMM_ERR_UNSUPPORTED, "kt must be 32");
    const int64_t m = A->m, k = A->k, nnz = A->nnz;
    if (o.row_order != SPMM_ORDER_ORIGINAL_RANGES && o.row_order != SPMM_ORDER_COMPACTED &&
        o.row_order != SPMM_ORDER_LENGTH_SORTED)
        return set_error(SPMM_ERR_UNSUPPORTED, "device-built mixed plans use original-ranges, compacted or "
                                               "length-sorted windows");
    if (o.local_reorder > 0)
        return set_error(SPMM_ERR_UNSUPPORTED, "device-built mixed plans take no local reordering");
    const int H = o.window_h, sval = dtype_size(A->val_type);
    int64_t W = (m + H - 1) / H;  // candidate windows (at most one per H rows)
    const int32_t col_thr = (int32_t)std::floor((double)o.alpha_c * (double)H);
    const double keep_thr = (double)o.alpha * (double)(H * kKt);
    auto sync = [&]() { return hipStreamSynchronize(s); };
    try {
        std::unique_ptr<spmm_plan_s> p(new spmm_plan_s());
        HostPlan &h = p->hp;
        h.m = m; h.k = k; h.nnz = nnz; h.n = n;
        h.val_type = A->val_type; h.b_type = b_type; h.c_type = c_type;
        h.tile_type = (b_type == SPMM_F16) ? SPMM_F16 : SPMM_BF16;
        h.opts = o;
        Scratch scratch;
        int64_t *plen, *kpos, *sums;
        int32_t *rp32, *bad;
        uint8_t *seen;
        unsigned long long *kcount;
        SPMM_ALLOC(plen, m);
        SPMM_ALLOC(kpos, m);
        SPMM_ALLOC(rp32, m + 1);
        SPMM_ALLOC(bad, 4);
        SPMM_ALLOC(kcount, 1);
        SPMM_ALLOC(seen, k);
        const int64_t big = std::max<int64_t>({m, nnz, W + 1});
        SPMM_ALLOC(sums, scan_sums_len(big));
        SPMM_TRY_HIP(hipMemsetAsync(bad, 0, 16, s), "hipMemsetAsync");
        SPMM_TRY_HIP(hipMemsetAsync(kcount, 0, 8, s), "hipMemsetAsync");
        SPMM_TRY_HIP(hipMemsetAsync(seen, 0, (size_t)std::max<int64_t>(k, 1), s), "hipMemsetAsync");
        // 1. rows, columns, checks
        hipLaunchKernelGGL(k_mrows, dim3(blocks_for(m + 1)), dim3(kThreads), 0, s, m, nnz, A->rowptr, o.t_row,
                           plen, rp32, bad);
        if (nnz > 0)
            hipLaunchKernelGGL(k_mcols, dim3((unsigned)std::min<int64_t>(blocks_for(nnz), 65536)), dim3(kThreads),
                               0, s, nnz, k, A->colidx, seen, bad);
        SPMM_TRY_HIP(hipGetLastError(), "device plan kernels");
        int32_t bad_h = 0;
        SPMM_TRY_HIP(hipMemcpyAsync(&bad_h, bad, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        if (bad_h & 1) return set_error(SPMM_ERR_INVALID, "rowptr not monotone from 0 to nnz");
        if (bad_h & 2) return set_error(SPMM_ERR_INVALID, "column index out of range");
        // window slots: original ranges need no list; otherwise the passing
        // rows compacted in row order, for length-sorted windows stably
        // sorted by decreasing length (the radix sort keeps equal keys in
        // their input order, i.e. row order, as the host's stable sort)
        int32_t *wpos = nullptr, *slot_row = nullptr;
        if (o.row_order != SPMM_ORDER_ORIGINAL_RANGES && m > 0) {
            int64_t *pflag, *ppos;
            SPMM_ALLOC(pflag, m);
            SPMM_ALLOC(ppos, m);
            hipLaunchKernelGGL(k_passflag, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, o.t_row, rp32, pflag);
            SPMM_TRY_HIP(scan64(pflag, ppos, m, 0, sums, s), "scan");
            int64_t nD = 0;
            SPMM_TRY_HIP(hipMemcpyAsync(&nD, sums + (scan_sums_len(m) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
            int32_t *D;
            SPMM_ALLOC(D, nD);
            SPMM_ALLOC(wpos, m);
            hipLaunchKernelGGL(k_fill32, dim3((unsigned)std::min<int64_t>(blocks_for(m), 65536)), dim3(kThreads), 0, s,
                               m, (int32_t)-1, wpos);
            if (nD > 0)
                hipLaunchKernelGGL(k_compact, dim3(blocks_for(m)), dim3(kThreads), 0, s, m, pflag, ppos, D);
            const int32_t *Dord = D;
            if (o.row_order == SPMM_ORDER_LENGTH_SORTED && nD > 1) {
                int32_t *Ds, *lk, *lks;
                SPMM_ALLOC(Ds, nD);
                SPMM_ALLOC(lk, nD);
                SPMM_ALLOC(lks, nD);
                hipLaunchKernelGGL(k_lenkeys, dim3(blocks_for(nD)), dim3(kThreads), 0, s, nD, D, rp32, lk);
                size_t tb = 0;
                SPMM_TRY_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tb, lk, lks, D, Ds, (int)nD, 0, 32, s),
                             "radix sort");
                uint8_t *tmp;
                SPMM_ALLOC(tmp, tb);
                SPMM_TRY_HIP(hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, lk, lks, D, Ds, (int)nD, 0, 32, s),
                             "radix sort");
                Dord = Ds;
            }
            W = (nD + H - 1) / H;
            SPMM_ALLOC(slot_row, W * H);
            if (W > 0)
                hipLaunchKernelGGL(k_slots, dim3(blocks_for(W * H)), dim3(kThreads), 0, s, W * H, nD, Dord, slot_row,
                                   wpos);
            SPMM_TRY_HIP(hipGetLastError(), "device plan kernels");
        }
        // 2. column stage: sorted (window, column) keys and their counts
        int64_t npass = 0;
        if (m > 0) {
            SPMM_TRY_HIP(scan64(plen, kpos, m, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&npass, sums + (scan_sums_len(m) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        }
        uint64_t *keys, *skeys, *ukeys, *mkey;
        int32_t *ucnt, *nruns, *mcnt;
        int64_t *uflag, *upos;
        SPMM_ALLOC(keys, npass);
        SPMM_ALLOC(skeys, npass);
        SPMM_ALLOC(ukeys, npass);
        SPMM_ALLOC(ucnt, npass);
        SPMM_ALLOC(nruns, 1);
        int64_t nrun = 0;
        if (npass > 0) {
            hipLaunchKernelGGL(k_keys, dim3(row_blocks(m)), dim3(kThreads), 0, s, m, H, rp32, A->colidx, plen, wpos,
                               kpos, keys);
            int end_bit = 33;
            while (end_bit < 64 && (W >> (end_bit - 32)) > 0) ++end_bit;
            size_t tb = 0, tb2 = 0;
            SPMM_TRY_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, keys, skeys, (int)npass, 0, end_bit, s),
                         "radix sort");
            SPMM_TRY_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb2, skeys, ukeys, ucnt, nruns, (int)npass, s),
                         "run-length encode");
            uint8_t *tmp;
            SPMM_ALLOC(tmp, std::max(tb, tb2));
            SPMM_TRY_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb, keys, skeys, (int)npass, 0, end_bit, s),
                         "radix sort");
            SPMM_TRY_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb2, skeys, ukeys, ucnt, nruns, (int)npass, s),
                         "run-length encode");
            int32_t nr = 0;
            SPMM_TRY_HIP(hipMemcpyAsync(&nr, nruns, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
            nrun = nr;
        }
        SPMM_ALLOC(uflag, nrun);
        SPMM_ALLOC(upos, nrun);
        int64_t nmc = 0;
        if (nrun > 0) {
            hipLaunchKernelGGL(k_mflag, dim3(blocks_for(nrun)), dim3(kThreads), 0, s, nrun, ucnt, col_thr, uflag);
            SPMM_TRY_HIP(scan64(uflag, upos, nrun, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&nmc, sums + (scan_sums_len(nrun) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        }
        SPMM_ALLOC(mkey, nmc);
        SPMM_ALLOC(mcnt, nmc);
        if (nmc > 0)
            hipLaunchKernelGGL(k_mscatter, dim3(blocks_for(nrun)), dim3(kThreads), 0, s, nrun, uflag, upos, ukeys, ucnt,
                               mkey, mcnt);
        // windows: first tile column, K-tiles, density test, kept tiles and windows
        int64_t *start, *nchunk, *cbase, *kept, *tile_id, *wkeep, *widx, *wtile0;
        SPMM_ALLOC(start, W + 1);
        SPMM_ALLOC(nchunk, W + 1);
        SPMM_ALLOC(cbase, W + 1);
        SPMM_ALLOC(wkeep, W + 1);
        SPMM_ALLOC(widx, W + 1);
        SPMM_ALLOC(wtile0, W + 1);
        int64_t nch = 0, T = 0, Wk = 0;
        if (W > 0) {
            hipLaunchKernelGGL(k_wstart, dim3(blocks_for(W + 1)), dim3(kThreads), 0, s, W, nmc, mkey, start, nchunk);
            hipLaunchKernelGGL(k_nchunk, dim3(blocks_for(W)), dim3(kThreads), 0, s, W, start, nchunk);
            SPMM_TRY_HIP(scan64(nchunk, cbase, W, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&nch, sums + (scan_sums_len(W) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(hipMemcpyAsync(cbase + W, sums + (scan_sums_len(W) - 1), 8, hipMemcpyDeviceToDevice, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        }
        SPMM_ALLOC(kept, nch);
        SPMM_ALLOC(tile_id, nch);
        if (nch > 0) {
            hipLaunchKernelGGL(k_chunks, dim3(blocks_for(W)), dim3(kThreads), 0, s, W, start, cbase, mcnt, keep_thr,
                               kept);
            SPMM_TRY_HIP(scan64(kept, tile_id, nch, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&T, sums + (scan_sums_len(nch) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            hipLaunchKernelGGL(k_wkept, dim3(blocks_for(W)), dim3(kThreads), 0, s, W, cbase, kept, tile_id, wkeep, wtile0);
            SPMM_TRY_HIP(scan64(wkeep, widx, W, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&Wk, sums + (scan_sums_len(W) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        } else if (W > 0) {
            SPMM_TRY_HIP(hipMemsetAsync(wkeep, 0, 8 * (size_t)(W + 1), s), "hipMemsetAsync");
        }
        if (T > INT32_MAX / (H * kKt)) return set_error(SPMM_ERR_UNSUPPORTED, "too many tiles");
        int32_t *windows, *win_tile_ptr, *tile_cols, *src;
        SPMM_ALLOC(windows, Wk * H);
        SPMM_ALLOC(win_tile_ptr, Wk + 1);
        SPMM_ALLOC(tile_cols, T * kKt);
        SPMM_ALLOC(src, T * H * kKt);
        if (Wk > 0) {
            hipLaunchKernelGGL(k_wfill, dim3(blocks_for(W)), dim3(kThreads), 0, s, W, m, H, o.t_row, rp32, slot_row,
                               wkeep, widx, wtile0, windows, win_tile_ptr);
            const int32_t Ti = (int32_t)T;
            SPMM_TRY_HIP(hipMemcpyAsync(win_tile_ptr + Wk, &Ti, 4, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
            hipLaunchKernelGGL(k_tcols, dim3(blocks_for(W)), dim3(kThreads), 0, s, W, start, cbase, kept, tile_id, mkey,
                               tile_cols);
            hipLaunchKernelGGL(k_fill32, dim3((unsigned)std::min<int64_t>(blocks_for(T * H * kKt), 65536)),
                               dim3(kThreads), 0, s, T * H * kKt, (int32_t)INT_MAX, src);
            hipLaunchKernelGGL(k_assign, dim3(row_blocks(m)), dim3(kThreads), 0, s, m, H, rp32, A->colidx, plen, wpos,
                               wkeep, start, cbase, kept, tile_id, mkey, src);
        }
        // 3. in-tile flags, remainder lengths and the remainder
        uint8_t *in_tile;
        int64_t *rem_len, *rem_ptr;
        SPMM_ALLOC(in_tile, nnz);
        SPMM_ALLOC(rem_len, m);
        SPMM_ALLOC(rem_ptr, m + 1);
        int64_t nrem = 0;
        if (m > 0) {
            hipLaunchKernelGGL(k_intile, dim3(row_blocks(m)), dim3(kThreads), 0, s, m, H, rp32, A->colidx, plen, wpos,
                               wkeep, start, cbase, kept, tile_id, mkey, src, in_tile, rem_len);
            SPMM_TRY_HIP(scan64(rem_len, rem_ptr, m, 0, sums, s), "scan");
            SPMM_TRY_HIP(hipMemcpyAsync(&nrem, sums + (scan_sums_len(m) - 1), 8, hipMemcpyDeviceToHost, s),
                         "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        }
        const int64_t nv = nnz - nrem;  // every entry is in a tile or the remainder
        int32_t *rem_col, *rem_aux;
        uint8_t *rem_val;
        uint32_t *tile_bitmap;
        uint16_t *tile_vals;
        int64_t *vcnt, *vpos;
        int32_t *tile_val_ptr;
        SPMM_ALLOC(rem_col, nrem);
        SPMM_ALLOC(rem_val, nrem * sval);
        SPMM_ALLOC(tile_bitmap, T * H);
        SPMM_ALLOC(tile_vals, nv);
        SPMM_ALLOC(vcnt, T * H);
        SPMM_ALLOC(vpos, T * H);
        SPMM_ALLOC(tile_val_ptr, T + 1);
        // the CSR entries of the remainder then of the tile values (kept by the plan)
        void *aux = nullptr;
        if (hipMalloc(&aux, 4 * (size_t)(nrem + nv) + 16) != hipSuccess)
            return set_error(SPMM_ERR_OOM, "hipMalloc(device plan entries)");
        std::unique_ptr<void, hipError_t (*)(void *)> aux_guard(aux, hipFree);
        rem_aux = static_cast<int32_t *>(aux);
        if (m > 0)
            hipLaunchKernelGGL(k_remainder, dim3(row_blocks(m)), dim3(kThreads), 0, s, m, sval, rp32, A->colidx,
                               static_cast<const uint8_t *>(A->vals), in_tile, rem_ptr, rem_col, rem_val, rem_aux);
        // 4. bitmaps, value offsets, packed values
        if (T > 0) {
            hipLaunchKernelGGL(k_bitmap, dim3(blocks_for(T * H)), dim3(kThreads), 0, s, T * H, src, tile_bitmap, vcnt);
            SPMM_TRY_HIP(scan64(vcnt, vpos, T * H, 0, sums, s), "scan");
            hipLaunchKernelGGL(k_tvptr, dim3(blocks_for(T + 1)), dim3(kThreads), 0, s, T, H, vpos, nv, tile_val_ptr);
            hipLaunchKernelGGL(k_values, dim3(blocks_for(T * H)), dim3(kThreads), 0, s, T * H, A->val_type, src,
                               tile_bitmap, vpos, static_cast<const uint8_t *>(A->vals), tile_vals, rem_aux + nrem);
        }
        if (k > 0)
            hipLaunchKernelGGL(k_mcount_seen, dim3((unsigned)std::min<int64_t>(blocks_for(k), 4096)), dim3(kThreads),
                               0, s, k, seen, kcount);
        SPMM_TRY_HIP(hipGetLastError(), "device plan kernels");
        // O(m + windows + tiles) arrays to the host, then the schedule there
        h.windows.resize(Wk * H);
        std::vector<int32_t> wtp(Wk + 1, 0), tvp(T + 1, 0);
        h.rem_ptr32.resize(m + 1);
        unsigned long long kref = 0;
        auto d2h = [&](void *dst, const void *srcp, size_t bytes) {
            return bytes ? hipMemcpyAsync(dst, srcp, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
        };
        std::vector<int64_t> rp64(m + 1, 0);
        SPMM_TRY_HIP(d2h(h.windows.data(), windows, 4 * (size_t)(Wk * H)), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(wtp.data(), win_tile_ptr, Wk > 0 ? 4 * (size_t)(Wk + 1) : 0), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(tvp.data(), tile_val_ptr, T > 0 ? 4 * (size_t)(T + 1) : 0), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(rp64.data(), rem_ptr, 8 * (size_t)m), "hipMemcpyAsync");
        SPMM_TRY_HIP(d2h(&kref, kcount, 8), "hipMemcpyAsync");
        SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        rp64[m] = nrem;
        h.rem_ptr = rp64;
        for (int64_t r = 0; r <= m; ++r) h.rem_ptr32[r] = (int32_t)rp64[r];
        h.win_tile_ptr = wtp;
        h.tile_val_ptr.assign(tvp.begin(), tvp.end());
        h.tile_window.resize(T);
        for (int64_t w = 0; w < Wk; ++w)
            for (int32_t t = wtp[w]; t < wtp[w + 1]; ++t) h.tile_window[t] = (int32_t)w;
        h.k_ref = (int64_t)kref;
        build_schedule(h);
        derive_exec_tables(h);
        // the segments' launch order, by the column of their middle entry
        DeviceArrays da;
        da.rem_col = rem_col;
        da.rem_val = rem_val;
        da.tile_cols = tile_cols;
        da.tile_bitmap = tile_bitmap;
        da.tile_vals = tile_vals;
        da.nrem = (size_t)nrem;
        da.nvals = (size_t)nv;
        const int64_t S = (int64_t)h.seg_row.size();
        if (S > 0) {
            int32_t *sb, *se, *sk;
            SPMM_ALLOC(sb, S);
            SPMM_ALLOC(se, S);
            SPMM_ALLOC(sk, S);
            SPMM_TRY_HIP(hipMemcpyAsync(sb, h.seg_begin.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(hipMemcpyAsync(se, h.seg_end.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
            hipLaunchKernelGGL(k_mseg_keys, dim3(blocks_for(S)), dim3(kThreads), 0, s, S, sb, se, rem_col, sk);
            std::vector<int32_t> key(S);
            SPMM_TRY_HIP(hipMemcpyAsync(key.data(), sk, 4 * (size_t)S, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
            SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
            da.seg_order = order_by_key32(key);
            bool id = true;
            for (int64_t i = 0; i < S && id; ++i) id = da.seg_order[i] == (int32_t)i;
            if (id) da.seg_order.clear();
        }
        SPMM_TRY_HIP(sync(), "hipStreamSynchronize");
        st = upload_plan(p.get(), &da);
        if (st != SPMM_OK) return st;
        p->aux = aux_guard.release();
        p->dev_nrem = nrem;
        p->dev_nvals = nv;
        *out = p.release();
        return SPMM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SPMM_ERR_OOM, "host allocation failed while building a device plan");
    }
}

}  // namespace spmm
