// items.hpp -- device functions of one work item of each kind (gfx950).
//
// The kernels that execute a plan (NeutronSparse Sec. 5.1 execution models,
// adapted to CDNA4 where the matrix cores and the vector ALUs share a CU) are
// built from three items:
//
//   segment  -- one wavefront per segment of a long remainder row: FP32
//               gather-FMA partial sum into a per-run workspace.
//   vector   -- one wavefront per vector work item (consecutive rows): FP32
//               gather-FMA over each row's remainder (Sec. 5.1, gather then
//               accumulate), or the fixed-order sum of its segment partials,
//               then one write of the C row.
//   window   -- one workgroup per (row window, column panel of 128, or of 64
//               or 32 for narrow 16-bit B): the B rows
//               of the window's compacted tile columns are staged in LDS once
//               and reused by every row of the window (Sec. 6.2, intra-core
//               reuse; Sec. 5.1, matrix-engine execution), each tile's bitmap
//               and packed values are expanded into dense rows in LDS and read
//               as MFMA operands (bf16 / f16 in, f32 accumulate), then each
//               row adds its remainder and is written once.
//
// Summation order of a remainder segment (identical in every kernel that
// computes one, so a row's bits depend only on the plan and N, never on the
// schedule): the wavefront is split into G groups of LPR lanes; entry i of the
// segment is accumulated by group i mod G with fmaf, in increasing i; the
// groups are then combined by an xor butterfly.  Segments of a split row are
// added in segment order.  No floating-point atomics are used anywhere.
#pragma once

#include <type_traits>

#include "devplan.hpp"
namespace spmm {

enum { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
}

// float -> bf16 bits, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (u >> 16) | 0x40u;
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

template <int DT>
__device__ __forceinline__ float load_val(const void *base, int idx) {
    if constexpr (DT == DT_F32) {
        return __builtin_nontemporal_load(static_cast<const float *>(base) + idx);
    } else {
        uint32_t b = __builtin_nontemporal_load(static_cast<const unsigned short *>(base) + idx);
        return DT == DT_BF16 ? bf16_to_f32(b) : f16_to_f32(b);
    }
}

// E consecutive elements of B (as float) starting at element offset `off`.
// NT selects the non-temporal cache policy (the line is streamed through L2
// and is the first to be evicted), used for B rows outside the hot set.
template <bool NT, class T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int BT, int E, bool NT = false>
__device__ __forceinline__ void load_chunk(const void *B, int64_t off, float (&v)[E]) {
    if constexpr (E == 1) {
        if constexpr (BT == DT_F32)
            v[0] = ld<NT>(static_cast<const float *>(B) + off);
        else if constexpr (BT == DT_BF16)
            v[0] = bf16_to_f32(ld<NT>(static_cast<const unsigned short *>(B) + off));
        else
            v[0] = f16_to_f32(ld<NT>(static_cast<const unsigned short *>(B) + off));
    } else if constexpr (BT == DT_F32) {
        static_assert(E == 4, "f32 chunks are 4 wide");
        f32x4 x = ld<NT>(reinterpret_cast<const f32x4 *>(static_cast<const float *>(B) + off));
        v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
    } else {
        static_assert(E == 8, "16-bit chunks are 8 wide");
        u32x4 x = ld<NT>(reinterpret_cast<const u32x4 *>(static_cast<const unsigned short *>(B) + off));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (BT == DT_BF16) {
                v[2 * i] = __uint_as_float(x[i] << 16);
                v[2 * i + 1] = __uint_as_float(x[i] & 0xFFFF0000u);
            } else {
                v[2 * i] = f16_to_f32(x[i] & 0xFFFFu);
                v[2 * i + 1] = f16_to_f32(x[i] >> 16);
            }
        }
    }
}

// A gathered chunk kept in its stored form until it is consumed, so that 16-bit
// B rows hold 4 registers per 8 elements while loads are in flight.
template <int BT, int E>
struct Raw {
    using T = typename std::conditional<E == 1, uint32_t,
                                        typename std::conditional<BT == DT_F32, f32x4, u32x4>::type>::type;
    T x;
};

template <int BT, int E, bool NT>
__device__ __forceinline__ void load_raw(const void *B, int64_t off, Raw<BT, E> &r) {
    if constexpr (E == 1) {
        if constexpr (BT == DT_F32)
            r.x = __float_as_uint(ld<NT>(static_cast<const float *>(B) + off));
        else
            r.x = ld<NT>(static_cast<const unsigned short *>(B) + off);
    } else if constexpr (BT == DT_F32) {
        r.x = ld<NT>(reinterpret_cast<const f32x4 *>(static_cast<const float *>(B) + off));
    } else {
        r.x = ld<NT>(reinterpret_cast<const u32x4 *>(static_cast<const unsigned short *>(B) + off));
    }
}

template <int BT, int E>
__device__ __forceinline__ void zero_raw(Raw<BT, E> &r) {
    if constexpr (E == 1) r.x = 0u;
    else if constexpr (BT == DT_F32) r.x = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    else r.x = u32x4{0u, 0u, 0u, 0u};
}

// acc[e] = fma(v, chunk[e], acc[e]) for the E elements of a raw chunk.
template <int BT, int E>
__device__ __forceinline__ void fma_raw(float v, const Raw<BT, E> &r, float (&acc)[E]) {
    if constexpr (E == 1) {
        const float b = BT == DT_F32 ? __uint_as_float(r.x)
                                     : (BT == DT_BF16 ? bf16_to_f32(r.x) : f16_to_f32(r.x));
        acc[0] = __builtin_fmaf(v, b, acc[0]);
    } else if constexpr (BT == DT_F32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaf(v, r.x[e], acc[e]);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float lo, hi;
            if constexpr (BT == DT_BF16) {
                lo = __uint_as_float(r.x[i] << 16);
                hi = __uint_as_float(r.x[i] & 0xFFFF0000u);
            } else {
                lo = f16_to_f32(r.x[i] & 0xFFFFu);
                hi = f16_to_f32(r.x[i] >> 16);
            }
            acc[2 * i] = __builtin_fmaf(v, lo, acc[2 * i]);
            acc[2 * i + 1] = __builtin_fmaf(v, hi, acc[2 * i + 1]);
        }
    }
}

// The same chunk through a raw buffer load whose cache-policy bits are `aux`
// (gfx950: bit 0 sc0, bit 1 nt, bit 4 sc1).  A distinct intrinsic, so the
// compiler never merges it with the default-policy load of a hot row.
template <int AUX>
__device__ __forceinline__ u32x4 buf16(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, AUX);
}
template <int AUX>
__device__ __forceinline__ uint32_t buf4(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, AUX);
}
template <int AUX>
__device__ __forceinline__ uint32_t buf2(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, AUX);
}

template <int BT, int E>
__device__ __forceinline__ void load_chunk_policy(__amdgpu_buffer_rsrc_t rs, int64_t off, int aux,
                                                  float (&v)[E]) {
    constexpr int SB = BT == DT_F32 ? 4 : 2;
    const uint32_t boff = (uint32_t)(off * SB);
    if constexpr (E == 1) {
        uint32_t x;
        if constexpr (SB == 4) {
            switch (aux) {
            case 2: x = buf4<2>(rs, boff); break;
            case 16: x = buf4<16>(rs, boff); break;
            case 18: x = buf4<18>(rs, boff); break;
            default: x = buf4<0>(rs, boff); break;
            }
            v[0] = __uint_as_float(x);
        } else {
            switch (aux) {
            case 2: x = buf2<2>(rs, boff); break;
            case 16: x = buf2<16>(rs, boff); break;
            case 18: x = buf2<18>(rs, boff); break;
            default: x = buf2<0>(rs, boff); break;
            }
            v[0] = BT == DT_BF16 ? bf16_to_f32(x) : f16_to_f32(x);
        }
    } else {
        u32x4 x;
        switch (aux) {
        case 2: x = buf16<2>(rs, boff); break;
        case 16: x = buf16<16>(rs, boff); break;
        case 18: x = buf16<18>(rs, boff); break;
        default: x = buf16<0>(rs, boff); break;
        }
        if constexpr (BT == DT_F32) {
            v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
            v[2] = __uint_as_float(x[2]); v[3] = __uint_as_float(x[3]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (BT == DT_BF16) {
                    v[2 * i] = __uint_as_float(x[i] << 16);
                    v[2 * i + 1] = __uint_as_float(x[i] & 0xFFFF0000u);
                } else {
                    v[2 * i] = f16_to_f32(x[i] & 0xFFFFu);
                    v[2 * i + 1] = f16_to_f32(x[i] >> 16);
                }
            }
        }
    }
}

template <int BT, int E>
__device__ __forceinline__ void load_raw_policy(__amdgpu_buffer_rsrc_t rs, int64_t off, int aux,
                                                Raw<BT, E> &r) {
    constexpr int SB = BT == DT_F32 ? 4 : 2;
    const uint32_t boff = (uint32_t)(off * SB);
    if constexpr (E == 1) {
        if constexpr (SB == 4) {
            switch (aux) {
            case 2: r.x = buf4<2>(rs, boff); break;
            case 16: r.x = buf4<16>(rs, boff); break;
            case 18: r.x = buf4<18>(rs, boff); break;
            default: r.x = buf4<0>(rs, boff); break;
            }
        } else {
            switch (aux) {
            case 2: r.x = buf2<2>(rs, boff); break;
            case 16: r.x = buf2<16>(rs, boff); break;
            case 18: r.x = buf2<18>(rs, boff); break;
            default: r.x = buf2<0>(rs, boff); break;
            }
        }
    } else {
        u32x4 x;
        switch (aux) {
        case 2: x = buf16<2>(rs, boff); break;
        case 16: x = buf16<16>(rs, boff); break;
        case 18: x = buf16<18>(rs, boff); break;
        default: x = buf16<0>(rs, boff); break;
        }
        if constexpr (BT == DT_F32) r.x = __builtin_bit_cast(f32x4, x);
        else r.x = x;
    }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t b_resource(const void *B, uint32_t rec) {
    // raw buffer over B: stride 0, `rec` bytes addressable (all 2^32-1 when 0),
    // gfx9 word-3 flags; a load at or beyond `rec` returns zeros and moves no data
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(B), (short)0,
                                             rec ? (int)rec : (int)0xFFFFFFFF, 0x00020000);
}

// A raw chunk through the default-policy buffer load at byte offset `off`.
template <int BT, int E>
__device__ __forceinline__ void load_raw_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, Raw<BT, E> &r) {
    if constexpr (E == 1) {
        if constexpr (BT == DT_F32) r.x = buf4<0>(rs, off);
        else r.x = buf2<0>(rs, off);
    } else {
        const u32x4 x = buf16<0>(rs, off);
        if constexpr (BT == DT_F32) r.x = __builtin_bit_cast(f32x4, x);
        else r.x = x;
    }
}

template <int E>
__device__ __forceinline__ void store_chunk(float *C, int64_t off, const float (&v)[E]) {
    if constexpr (E == 1) {
        __builtin_nontemporal_store(v[0], C + off);
    } else {
#pragma unroll
        for (int i = 0; i < E; i += 4) {
            f32x4 x = {v[i], v[i + 1], v[i + 2], v[i + 3]};
            __builtin_nontemporal_store(x, reinterpret_cast<f32x4 *>(C + off + i));
        }
    }
}

template <int E>
__device__ __forceinline__ void load_f32_chunk(const float *W, int64_t off, float (&v)[E]) {
    if constexpr (E == 1) {
        v[0] = W[off];
    } else {
#pragma unroll
        for (int i = 0; i < E; i += 4) {
            f32x4 x = *reinterpret_cast<const f32x4 *>(W + off + i);
            v[i] = x[0]; v[i + 1] = x[1]; v[i + 2] = x[2]; v[i + 3] = x[3];
        }
    }
}

// Workgroup id after the optional XCD remap: workgroups are dispatched
// round-robin over the 8 XCDs, so id b runs on XCD b % 8.  The remap gives
// each XCD one contiguous range of logical ids, so neighbouring items (which
// tend to share rows of B) share that XCD's L2.
// Logical id of workgroup b of a range of nwg workgroups whose first one runs
// on XCD 0 (ranges of a fused launch start at multiples of 8).
__device__ __forceinline__ int remap_block(int b, int nwg) {
    const int full = nwg >> 3, rem = nwg & 7, x = b & 7, local = b >> 3;
    return (x < rem ? x * (full + 1) : rem * (full + 1) + (x - rem) * full) + local;
}

__device__ __forceinline__ int logical_block(int xcd) {
    const int b = blockIdx.x;
    if (!xcd) return b;
    return remap_block(b, gridDim.x);
}

// This wave's index in its workgroup, as a wave-uniform (scalar) value, so
// that the item and descriptor loads that depend on it are scalar loads.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Lane layout of the gather-FMA: lane = group * LPR + li; lane li of a group
// owns chunks q = c * LPR + li (c < CPL), i.e. columns q*E .. q*E+E-1 of the
// panel.
struct Lanes {
    int lpr_log2, lpr, groups, group, li;
    __device__ __forceinline__ Lanes() = default;
    __device__ __forceinline__ explicit Lanes(int lg) {
        const int lane = threadIdx.x & 63;
        lpr_log2 = lg;
        lpr = 1 << lg;
        groups = 64 >> lg;
        group = lane >> lg;
        li = lane & (lpr - 1);
    }
    // the same lane position with entry stride 1: the group walks a row alone
    __device__ __forceinline__ Lanes single() const {
        Lanes o = *this;
        o.groups = 1;
        return o;
    }
};

// Entries p, p + G, ..., p + (U-1)G of a group (masked at p1): columns and values.
// CLAMP: every load is issued, at an index clamped into [0, p1 - 1], with no
// branch around it (a branch can make the compiler wait for each load before
// issuing the next); a masked entry gets value 0 and the column of the
// clamped entry, which is a real column when p < p1 (the plan arrays carry a
// zero tail for the empty case).  Otherwise masked entries are not loaded, so
// a step whose entries are all masked issues nothing.  Measured: clamping
// pays where gathers are small and latency-bound (16-bit B), predication
// where they are large and bandwidth-bound (f32 B).
template <int VT, int U, bool CLAMP>
__device__ __forceinline__ void load_entries(const int32_t *__restrict__ rcol,
                                             const void *__restrict__ rval, int p, int p1,
                                             const Lanes &L, int (&col)[U], float (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int pp = p + u * L.groups;
        if constexpr (CLAMP) {
            const int q = max(min(pp, p1 - 1), 0);
            col[u] = __builtin_nontemporal_load(rcol + q);
            const float x = load_val<VT>(rval, q);
            v[u] = pp < p1 ? x : 0.0f;
        } else {
            const bool ok = pp < p1;
            col[u] = ok ? __builtin_nontemporal_load(rcol + pp) : 0;
            v[u] = ok ? load_val<VT>(rval, pp) : 0.0f;
        }
    }
}

// Gathers the B rows of U loaded entries (hot rows cacheable, the others with
// the cold policy) and accumulates them in entry order.
// POL: the per-entry cache-policy choice is compiled in (row-by-row variant
// and segments of plans with a cold policy); without it every gather uses the
// default policy and the loop carries no per-entry branches.
template <int BT, int E, int CPL, int U, bool POL = false>
__device__ __forceinline__ void gather_fma(const int (&col)[U], const float (&v)[U], int p, int p1,
                                           const void *__restrict__ B,
                                           __amdgpu_buffer_rsrc_t rs, int64_t ldb, uint32_t brec,
                                           const bool (&cok)[CPL], const int64_t (&coff)[CPL],
                                           const Lanes &L, int cold_aux, float (&acc)[CPL][E]) {
    constexpr int SB = BT == DT_F32 ? 4 : 2;
    Raw<BT, E> b[U][CPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = p + u * L.groups < p1;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            // bit 31 of a column marks a hot B row (cacheable gather)
            const int64_t boff = (int64_t)(col[u] & 0x7FFFFFFF) * ldb + coff[c];
            if constexpr (POL) {
                (void)brec;
                if (ok && cok[c] && (col[u] < 0 || cold_aux < 0)) {
                    load_raw<BT, E, false>(B, boff, b[u][c]);
                } else if (ok && cok[c]) {
                    load_raw_policy<BT, E>(rs, boff, cold_aux, b[u][c]);
                } else {
                    zero_raw<BT, E>(b[u][c]);
                }
            } else {
                // No branch around a load when B is addressable by a buffer
                // resource (a branch makes the compiler wait for each load
                // before issuing the next): a masked entry or a chunk outside
                // the panel loads at offset brec, out of the buffer's range,
                // which returns zeros without a memory access.  B spanning
                // 4 GiB or more takes predicated plain loads.
                (void)cold_aux;
                if (brec != 0) {
                    load_raw_buf<BT, E>(rs, ok && cok[c] ? (uint32_t)(boff * SB) : brec, b[u][c]);
                } else if (ok && cok[c]) {
                    load_raw<BT, E, false>(B, boff, b[u][c]);
                } else {
                    zero_raw<BT, E>(b[u][c]);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (p + u * L.groups < p1) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) fma_raw<BT, E>(v[u], b[u][c], acc[c]);
        }
    }
}

// acc += v_u * b_u over the entries below p1, in entry order (the FMA half of
// gather_fma, for B chunks gathered earlier by the caller).
template <int BT, int E, int CPL, int U>
__device__ __forceinline__ void fma_rows(const float (&v)[U], const Raw<BT, E> (&b)[U][CPL], int p,
                                         int p1, const Lanes &L, float (&acc)[CPL][E]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (p + u * L.groups < p1) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) fma_raw<BT, E>(v[u], b[u][c], acc[c]);
        }
    }
}

template <int E, int CPL>
__device__ __forceinline__ void chunk_layout(int ncol0, int ncols, const Lanes &L, bool (&cok)[CPL],
                                             int64_t (&coff)[CPL]) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = c * L.lpr + L.li;
        cok[c] = q * E < ncols;
        coff[c] = ncol0 + (cok[c] ? (int64_t)q * E : 0);  // a valid chunk when outside the panel
    }
}

// acc += sum over entries [p0, p1) of v_p * B[col_p][panel columns], entry
// p0 + i taken by group i % G in increasing i (see the file comment).
template <int VT, int BT, int E, int CPL, int U, bool POL = false>
__device__ __forceinline__ void seg_accumulate(const int32_t *__restrict__ rcol,
                                               const void *__restrict__ rval, int p0, int p1,
                                               const void *__restrict__ B, int64_t ldb, uint32_t brec,
                                               int ncol0, int ncols, const Lanes &L, int cold_aux,
                                               float (&acc)[CPL][E]) {
    const __amdgpu_buffer_rsrc_t rs = b_resource(B, brec);
    bool cok[CPL];
    int64_t coff[CPL];
    chunk_layout<E, CPL>(ncol0, ncols, L, cok, coff);
    const int step = L.groups * U;
    for (int p = p0 + L.group; p < p1; p += step) {
        int col[U];
        float v[U];
        load_entries<VT, U, BT != DT_F32>(rcol, rval, p, p1, L, col, v);
        gather_fma<BT, E, CPL, U, POL>(col, v, p, p1, B, rs, ldb, brec, cok, coff, L, cold_aux, acc);
    }
}

// acc += sum over entries [p0, p1) of one row, all taken by this lane's group
// in increasing order (each group works on its own row).
template <int VT, int BT, int E, int CPL, int U, bool POL = false>
__device__ __forceinline__ void row_accumulate_group(const int32_t *__restrict__ rcol,
                                                     const void *__restrict__ rval, int p0, int p1,
                                                     const void *__restrict__ B, int64_t ldb,
                                                     uint32_t brec, int ncol0, int ncols,
                                                     const Lanes &L, int cold_aux,
                                                     float (&acc)[CPL][E]) {
    const __amdgpu_buffer_rsrc_t rs = b_resource(B, brec);
    bool cok[CPL];
    int64_t coff[CPL];
    chunk_layout<E, CPL>(ncol0, ncols, L, cok, coff);
    const Lanes one = L.single();
    for (int p = p0; p < p1; p += U) {
        int col[U];
        float v[U];
        load_entries<VT, U, BT != DT_F32>(rcol, rval, p, p1, one, col, v);
        gather_fma<BT, E, CPL, U, POL>(col, v, p, p1, B, rs, ldb, brec, cok, coff, one, cold_aux, acc);
    }
}

template <int E, int CPL>
__device__ __forceinline__ void group_reduce(float (&acc)[CPL][E], const Lanes &L) {
    for (int off = 32; off >= L.lpr; off >>= 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[c][e] += __shfl_xor(acc[c][e], off, 64);
    }
}

// Stores and loads of parts exchanged between the workgroups of one launch
// (co-scheduled execution) go through the workspace as a raw buffer with the
// device-scope cache policy (sc1): stores write through an XCD's L2 (each XCD
// has its own) and loads read past it, so a part stored on one XCD is read
// intact on another once its store has completed.  Offsets are in floats from
// the workspace base (a co-scheduled run keeps its workspace below 4 GiB).
constexpr int kDevScope = 16;  // gfx950 buffer cache-policy bits: sc1

__device__ __forceinline__ __amdgpu_buffer_rsrc_t ws_resource(const RunArgs &a) {
    return b_resource(a.work, a.ws_rec);
}
__device__ __forceinline__ void st_dev1(__amdgpu_buffer_rsrc_t rs, int64_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, (uint32_t)(off * 4), 0, kDevScope);
}
__device__ __forceinline__ f32x4 ld_dev4(__amdgpu_buffer_rsrc_t rs, int64_t off) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)(off * 4), 0, kDevScope));
}
template <int E>
__device__ __forceinline__ void st_dev_chunk(__amdgpu_buffer_rsrc_t rs, int64_t off, const float (&v)[E]) {
    if constexpr (E == 1) {
        st_dev1(rs, off, v[0]);
    } else {
#pragma unroll
        for (int i = 0; i < E; i += 4)
            __builtin_amdgcn_raw_buffer_store_b128(
                __builtin_bit_cast(u32x4, f32x4{v[i], v[i + 1], v[i + 2], v[i + 3]}), rs,
                (uint32_t)((off + i) * 4), 0, kDevScope);
    }
}
template <int E>
__device__ __forceinline__ void ld_dev_chunk(__amdgpu_buffer_rsrc_t rs, int64_t off, float (&v)[E]) {
    if constexpr (E == 1) {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)(off * 4), 0, kDevScope));
    } else {
#pragma unroll
        for (int i = 0; i < E; i += 4) {
            const f32x4 x = ld_dev4(rs, off + i);
            v[i] = x[0]; v[i + 1] = x[1]; v[i + 2] = x[2]; v[i + 3] = x[3];
        }
    }
}

// acc = P[sid] + P[sid+1] + ... + P[sid+ns-1] (panel columns), in that order.
// DEV: the partials were stored by other workgroups of this launch (rs: the
// workspace); loads go out four segments at a time.
template <int E, int CPL, bool DEV = false>
__device__ __forceinline__ void sum_partials(const float *__restrict__ work, int64_t ld, int sid,
                                             int ns, int ncol0, int ncols, const Lanes &L,
                                             float (&acc)[CPL][E],
                                             __amdgpu_buffer_rsrc_t rs = b_resource(nullptr, 0u)) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = c * L.lpr + L.li;
        if (q * E >= ncols) continue;
        const int64_t off = ncol0 + (int64_t)q * E;
        if constexpr (DEV) {
            (void)work;
            ld_dev_chunk<E>(rs, (int64_t)sid * ld + off, acc[c]);
            for (int j0 = 1; j0 < ns; j0 += 4) {
                float t[4][E];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    ld_dev_chunk<E>(rs, (int64_t)(sid + min(j0 + u, ns - 1)) * ld + off, t[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j0 + u < ns) {
#pragma unroll
                        for (int e = 0; e < E; ++e) acc[c][e] += t[u][e];
                    }
            }
        } else {
            load_f32_chunk<E>(work, (int64_t)sid * ld + off, acc[c]);
            for (int j = 1; j < ns; ++j) {
                float t[E];
                load_f32_chunk<E>(work, (int64_t)(sid + j) * ld + off, t);
#pragma unroll
                for (int e = 0; e < E; ++e) acc[c][e] += t[e];
            }
        }
    }
}

template <int E, int CPL>
__device__ __forceinline__ void store_row(float *C, int64_t row_off, int ncol0, int ncols,
                                          const Lanes &L, const float (&acc)[CPL][E]) {
    if (L.group != 0) return;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int q = c * L.lpr + L.li;
        if (q * E < ncols) store_chunk<E>(C, row_off + ncol0 + (int64_t)q * E, acc[c]);
    }
}

template <int E, int CPL>
constexpr int unroll_of() { return E == 1 ? 4 : (CPL == 1 ? 8 : 4); }

// ------------------------------------------------------------------------------------------
// Co-scheduled execution.  Segments, vector items, window owners and window
// partial items run side by side, so no item waits for a kernel boundary.  A
// result made of several items' parts (a split row's segment partials; a
// window's MFMA result, its partial tiles and its split rows) is finished by
// whichever contributor comes last: each contributor stores its part with
// device-coherent stores (st_dev), waits until they have completed, then adds
// 1 to the result's integer counter in global memory with a device-scope
// atomic; the one whose increment reaches the target reads every part with
// device-coherent loads (ld_dev), sums them in the same fixed order as the
// serial kernels, writes C, and clears the counter for the next run.  No
// contributor ever waits for another, so any schedule completes, and C is
// bitwise the same as with one kernel per item kind.  (A full device-scope
// fence instead writes back the whole XCD L2 at every arrival: measured 4x
// slower on the 2^20-vertex graph's 62,629 segments.)

// Waits until this wave's stores have completed.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// One wavefront arrives at a counter; true on every lane of the last arrival.
__device__ __forceinline__ bool wave_arrive(int32_t *cnt, int target) {
    stores_done();
    int old = 0;
    if ((threadIdx.x & 63) == 0) {
        old = atomicAdd(cnt, 1);
        if (old == target - 1) atomicExch(cnt, 0);
    }
    old = __shfl(old, 0, 64);
    return old == target - 1;
}

// A whole workgroup arrives (after all its threads' stores); `flag` is LDS.
__device__ __forceinline__ bool group_arrive(int32_t *cnt, int target, int32_t *flag) {
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int old = atomicAdd(cnt, 1);
        const bool last = old == target - 1;
        if (last) atomicExch(cnt, 0);
        *flag = last ? 1 : 0;
    }
    __syncthreads();
    return *flag != 0;
}

// Counter of window slot `dep` in window panel q (win_np columns).
__device__ __forceinline__ int32_t *win_counter(const DevPlan &P, const RunArgs &a, int q, int dep) {
    return a.cnt + (int64_t)a.n_panels * P.n_seg + (int64_t)q * P.n_dep + dep;
}

// Arrivals a window panel waits for: its owner, its partial items, and every
// segment panel (width np) overlapping the window panel for each segment of
// the window's split rows.
__device__ __forceinline__ int win_target(const DevPlan &P, const RunArgs &a, int w, int q) {
    const int c0 = q * a.win_np, c1 = min(P.n, c0 + a.win_np) - 1;
    return 1 + (P.win_part[w + 1] - P.win_part[w]) + P.win_nsseg[w] * (c1 / a.np - c0 / a.np + 1);
}

// The last arrival of window w, panel q: for each window row, its MFMA result
// plus the partial tiles' results in tile order, plus its remainder (the
// owner's sum, or the row's segment partials in segment order), written to C.
// Thread t of T participating threads takes 4-column chunks t, t + T, ... of
// the window's rows x panel columns (the workspace rows are padded to a
// multiple of 4 columns, so a chunk load stays in its row).
__device__ __forceinline__ void window_combine(const DevPlan &P, const RunArgs &a, int w, int q, int dep,
                                               int t, int T) {
    const int H = P.H;
    const int ncol0 = q * a.win_np, ncols = min(a.win_np, P.n - ncol0), nch = (ncols + 3) >> 2;
    const int pa = P.win_part[w], pb = P.win_part[w + 1];
    const int64_t ld = a.work_ld;
    const __amdgpu_buffer_rsrc_t rs = ws_resource(a);
    const int64_t wp0 = (int64_t)P.n_seg * ld;                                // window partials
    const int64_t cs0 = wp0 + ((int64_t)H * P.n_wpart + (int64_t)dep * 2 * H) * ld;  // slot: MFMA result
    const int64_t rm0 = cs0 + (int64_t)H * ld;                                // slot: remainders
    for (int u = t; u < H * nch; u += T) {
        const int s = u / nch, c = u - s * nch;
        const int r = P.windows[(int64_t)w * H + s];
        if (r < 0) continue;
        const int64_t col = ncol0 + 4 * c;
        f32x4 v = ld_dev4(rs, cs0 + (int64_t)s * ld + col);
        for (int k0 = pa; k0 < pb; k0 += 4) {
            f32x4 x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = ld_dev4(rs, wp0 + ((int64_t)min(k0 + i, pb - 1) * H + s) * ld + col);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (k0 + i < pb) v += x[i];
        }
        f32x4 y;
        const int sid0 = P.win_row_sid[(int64_t)w * H + s];
        if (sid0 >= 0) {
            const int len = P.rem_ptr[r + 1] - P.rem_ptr[r];
            const int ns = (len + P.seg_len - 1) / P.seg_len;
            y = ld_dev4(rs, (int64_t)sid0 * ld + col);
            for (int j0 = 1; j0 < ns; j0 += 4) {
                f32x4 x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = ld_dev4(rs, (int64_t)(sid0 + min(j0 + i, ns - 1)) * ld + col);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (j0 + i < ns) y += x[i];
            }
        } else {
            y = ld_dev4(rs, rm0 + (int64_t)s * ld + col);
        }
        const f32x4 z = v + y;
        float *dst = a.C + (int64_t)r * a.ldc + col;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * c + e < ncols) dst[e] = z[e];
    }
}

// ------------------------------------------------------------------------------------------
// One segment (of one panel) per wavefront: wid in [0, n_seg * n_panels).
// FUSED: the segment then arrives at its row's counter (a vector row) or its
// window's counters (a window row), and the last arrival finishes the result.
template <int VT, int BT, int E, int CPL, bool POL, bool FUSED = false>
__device__ __forceinline__ void segment_item(const DevPlan &P, const RunArgs &a, int wid) {
    const int panel = wid / P.n_seg, li = wid - panel * P.n_seg;
    const int sid = P.seg_order ? P.seg_order[li] : li;  // the partial's slot
    const int ncol0 = panel * a.np, ncols = min(a.np, P.n - ncol0);
    const Lanes L(a.lpr_log2);
    float acc[CPL][E];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[c][e] = 0.0f;
    seg_accumulate<VT, BT, E, CPL, unroll_of<E, CPL>(), POL>(P.rem_col, P.rem_val, P.seg_begin[sid],
                                                        P.seg_end[sid], a.B, a.ldb, a.b_rec, ncol0, ncols,
                                                        L, a.cold_aux, acc);
    group_reduce<E, CPL>(acc, L);
    if (L.group == 0) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int q = c * L.lpr + L.li;
            if (q * E < ncols) {
                float *dst = a.work + (int64_t)sid * a.work_ld + ncol0 + (int64_t)q * E;
                if constexpr (FUSED) {
                    st_dev_chunk<E>(ws_resource(a), (int64_t)sid * a.work_ld + ncol0 + (int64_t)q * E, acc[c]);
                } else if constexpr (E == 1) {
                    dst[0] = acc[c][0];
                } else {
#pragma unroll
                    for (int i = 0; i < E; i += 4)
                        *reinterpret_cast<f32x4 *>(dst + i) =
                            f32x4{acc[c][i], acc[c][i + 1], acc[c][i + 2], acc[c][i + 3]};
                }
            }
        }
    }
    if constexpr (FUSED) {
        // segments of a row have consecutive ids, segment j starting j * seg_len
        // entries into the row's remainder
        const int r = P.seg_row[sid];
        const int rb = P.rem_ptr[r], re = P.rem_ptr[r + 1];
        const int ns = (re - rb + P.seg_len - 1) / P.seg_len;
        const int sid0 = sid - (P.seg_begin[sid] - rb) / P.seg_len;
        const int w = P.seg_win ? P.seg_win[sid] : -1;
        if (w < 0) {
            if (wave_arrive(a.cnt + (int64_t)panel * P.n_seg + sid0, ns)) {
                // the vector items' sum of a split row, in segment order
                sum_partials<E, CPL, true>(a.work, a.work_ld, sid0, ns, ncol0, ncols, L, acc, ws_resource(a));
                store_row<E, CPL>(a.C, (int64_t)r * a.ldc, ncol0, ncols, L, acc);
            }
        } else {
            const int dep = P.win_dep[w];
            for (int q = ncol0 / a.win_np; q <= (ncol0 + ncols - 1) / a.win_np; ++q)
                if (wave_arrive(win_counter(P, a, q, dep), win_target(P, a, w, q)))
                    window_combine(P, a, w, q, dep, threadIdx.x & 63, 64);
        }
    }
}

// One vector work item (of one panel) per wavefront: wid in [0, n_vitems * n_panels).
// FUSED (every variant): a split row is finished by its last segment, so the
// item skips it.
template <int VT, int BT, int E, int CPL, bool FUSED = false>
__device__ __forceinline__ void vector_item(const DevPlan &P, const RunArgs &a, int wid) {
    const int panel = wid / P.n_vitems, item = wid - panel * P.n_vitems;
    const int ncol0 = panel * a.np, ncols = min(a.np, P.n - ncol0);
    const Lanes L(a.lpr_log2);
    int sid = P.vitem_seg[item];
    const int i0 = P.vitem_ptr[item], i1 = P.vitem_ptr[item + 1];
    for (int i = i0; i < i1; ++i) {
        const int r = P.vec_rows ? P.vec_rows[i] : i;
        const int b = P.rem_ptr[r], e = P.rem_ptr[r + 1];
        float acc[CPL][E];
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int x = 0; x < E; ++x) acc[c][x] = 0.0f;
        if (e - b <= P.seg_len) {
            seg_accumulate<VT, BT, E, CPL, unroll_of<E, CPL>(), true>(P.rem_col, P.rem_val, b, e, a.B,
                                                                a.ldb, a.b_rec, ncol0, ncols, L, a.cold_aux,
                                                                acc);
            group_reduce<E, CPL>(acc, L);
        } else {
            if constexpr (FUSED) continue;
            const int ns = (e - b + P.seg_len - 1) / P.seg_len;
            sum_partials<E, CPL>(a.work, a.work_ld, sid, ns, ncol0, ncols, L, acc);
            sid += ns;
        }
        store_row<E, CPL>(a.C, (int64_t)r * a.ldc, ncol0, ncols, L, acc);
    }
}

// Vector work item with a software pipeline across its rows: while a row's
// B rows are being gathered, the next row's pointers and first batch of
// (column, value) are already in flight.  Each row's entries are consumed in
// exactly the order of vector_item, so the results are bitwise identical.
template <int VT, int BT, int E, int CPL, bool FUSED = false>
__device__ __forceinline__ void vector_item_pipelined(const DevPlan &P, const RunArgs &a, int wid) {
    constexpr int U = unroll_of<E, CPL>();
    const int panel = wid / P.n_vitems, item = wid - panel * P.n_vitems;
    const int ncol0 = panel * a.np, ncols = min(a.np, P.n - ncol0);
    const Lanes L(a.lpr_log2);
    const int step = L.groups * U;
    const __amdgpu_buffer_rsrc_t rs = b_resource(a.B, a.b_rec);
    bool cok[CPL];
    int64_t coff[CPL];
    chunk_layout<E, CPL>(ncol0, ncols, L, cok, coff);
    int sid = P.vitem_seg[item];
    const int i0 = P.vitem_ptr[item], i1 = P.vitem_ptr[item + 1];

    int r = P.vec_rows ? P.vec_rows[i0] : i0;
    int b = P.rem_ptr[r], e = P.rem_ptr[r + 1];
    int col[U];
    float v[U];
    load_entries<VT, U, BT != DT_F32>(P.rem_col, P.rem_val, b + L.group, e - b <= P.seg_len ? e : b, L, col, v);
    for (int i = i0; i < i1; ++i) {
        int nr = r, nb = 0, ne = 0;
        if (i + 1 < i1) {
            nr = P.vec_rows ? P.vec_rows[i + 1] : i + 1;
            nb = P.rem_ptr[nr];
            ne = P.rem_ptr[nr + 1];
        }
        float acc[CPL][E];
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int x = 0; x < E; ++x) acc[c][x] = 0.0f;
        int ncl[U];
        float nv[U];
        if (e - b <= P.seg_len) {
            Raw<BT, E> bv[U][CPL];
            // gathers of this row's first batch
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = b + L.group + u * L.groups < e;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int64_t boff = (int64_t)(col[u] & 0x7FFFFFFF) * a.ldb + coff[c];
                    if (ok && cok[c]) load_raw<BT, E, false>(a.B, boff, bv[u][c]);
                    else zero_raw<BT, E>(bv[u][c]);
                }
            }
            // the next row's first batch, in flight behind the gathers
            load_entries<VT, U, BT != DT_F32>(P.rem_col, P.rem_val, nb + L.group, ne - nb <= P.seg_len ? ne : nb,
                                L, ncl, nv);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b + L.group + u * L.groups < e) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) fma_raw<BT, E>(v[u], bv[u][c], acc[c]);
                }
            }
            // the rest of a row longer than one batch, continuing the same order
            for (int p = b + step + L.group; p < e; p += step) {
                int c2[U];
                float v2[U];
                load_entries<VT, U, BT != DT_F32>(P.rem_col, P.rem_val, p, e, L, c2, v2);
                gather_fma<BT, E, CPL, U>(c2, v2, p, e, a.B, rs, a.ldb, a.b_rec, cok, coff, L, a.cold_aux,
                                          acc);
            }
            group_reduce<E, CPL>(acc, L);
        } else {
            load_entries<VT, U, BT != DT_F32>(P.rem_col, P.rem_val, nb + L.group, ne - nb <= P.seg_len ? ne : nb,
                                L, ncl, nv);
            if constexpr (!FUSED) {
                const int ns = (e - b + P.seg_len - 1) / P.seg_len;
                sum_partials<E, CPL>(a.work, a.work_ld, sid, ns, ncol0, ncols, L, acc);
                sid += ns;
            }
        }
        if (!FUSED || e - b <= P.seg_len) store_row<E, CPL>(a.C, (int64_t)r * a.ldc, ncol0, ncols, L, acc);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            col[u] = ncl[u];
            v[u] = nv[u];
        }
        r = nr;
        b = nb;
        e = ne;
    }
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ int wave_inclusive_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    return x;
}

// Vector work item with short rows packed one per lane group: a row whose
// remainder has at most 2U entries is summed in entry order by one group, and
// up to G such consecutive rows are gathered at once; longer rows take the
// whole wavefront as in vector_item.  The rule depends only on a row's length.
// The row ids and remainder ranges of the next 64 rows are loaded once, one
// row per lane, and handed to the groups by lane shuffles as the rows are
// taken, so a batch of short rows starts with its entry loads.
// UL: entries per group and step; the short-row bound stays 2 unroll_of, so
// the summation order (which depends only on a row's length) is the same for
// any UL.
template <int VT, int BT, int E, int CPL, bool FUSED = false, int UL = unroll_of<E, CPL>()>
__device__ __forceinline__ void vector_item_packed(const DevPlan &P, const RunArgs &a, int wid) {
    constexpr int U = UL;
    constexpr int SHORT = 2 * unroll_of<E, CPL>();
    const int panel = wid / P.n_vitems, item = wid - panel * P.n_vitems;
    const int ncol0 = panel * a.np, ncols = min(a.np, P.n - ncol0);
    const Lanes L(a.lpr_log2);
    const int lane = threadIdx.x & 63;
    int sid = P.vitem_seg[item];
    const int i0 = P.vitem_ptr[item], i1 = P.vitem_ptr[item + 1];
    for (int i = i0; i < i1; i += 64) {
        // the next (up to 64) rows, one per lane: id and remainder range
        const int li_row = i + lane;
        int rr = 0, rb = 0, re = 0, len = 0x7FFFFFFF;
        if (li_row < i1) {
            rr = P.vec_rows ? P.vec_rows[li_row] : li_row;
            rb = P.rem_ptr[rr];
            re = P.rem_ptr[rr + 1];
            len = re - rb;
        }
        const uint64_t longmask = __ballot(len > SHORT || len > P.seg_len || li_row >= i1);
        const int avail = min(64, i1 - i);
        int j = 0;
        while (j < avail) {
            // k = consecutive short rows from j, at most G
            const uint64_t lm = longmask >> j;
            int k = lm ? __builtin_ctzll(lm) : 64 - j;
            k = min(k, L.groups);
            if (k > 0) {
                const int src = min(j + L.group, 63);
                const int r = __shfl(rr, src, 64), b = __shfl(rb, src, 64), e = __shfl(re, src, 64);
                float acc[CPL][E];
#pragma unroll
                for (int c = 0; c < CPL; ++c)
#pragma unroll
                    for (int x = 0; x < E; ++x) acc[c][x] = 0.0f;
                if (L.group < k) {
                    row_accumulate_group<VT, BT, E, CPL, U>(P.rem_col, P.rem_val, b, e, a.B, a.ldb, a.b_rec,
                                                            ncol0, ncols, L, a.cold_aux, acc);
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const int q = c * L.lpr + L.li;
                        if (q * E < ncols) store_chunk<E>(a.C, (int64_t)r * a.ldc + ncol0 + (int64_t)q * E, acc[c]);
                    }
                }
                j += k;
                continue;
            }
            // a long row: the whole wavefront, as in vector_item
            const int r = __shfl(rr, j, 64), b = __shfl(rb, j, 64), e = __shfl(re, j, 64);
            ++j;
            float acc[CPL][E];
#pragma unroll
            for (int c = 0; c < CPL; ++c)
#pragma unroll
                for (int x = 0; x < E; ++x) acc[c][x] = 0.0f;
            if (e - b <= P.seg_len) {
                seg_accumulate<VT, BT, E, CPL, U>(P.rem_col, P.rem_val, b, e, a.B, a.ldb, a.b_rec, ncol0, ncols,
                                                  L, a.cold_aux, acc);
                group_reduce<E, CPL>(acc, L);
            } else {
                if constexpr (FUSED) continue;
                const int ns = (e - b + P.seg_len - 1) / P.seg_len;
                sum_partials<E, CPL>(a.work, a.work_ld, sid, ns, ncol0, ncols, L, acc);
                sid += ns;
            }
            store_row<E, CPL>(a.C, (int64_t)r * a.ldc, ncol0, ncols, L, acc);
        }
    }
}

// Size class of a row: the least power of two S of lane groups with
// len <= u2 * S, at most every group of the wavefront.
__device__ __forceinline__ int size_class(int len, int u2, int groups) {
    int s = 1;
    while (s < groups && len > u2 * s) s <<= 1;
    return s;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        lo |= __shfl_xor(lo, off, 64);
        hi |= __shfl_xor(hi, off, 64);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Vector work item with rows packed by size class: a row of class S is summed
// by an aligned block of S lane groups (entry p of the row by group p mod S,
// each group in entry order, then the groups' sums by an xor butterfly inside
// the block), so the order depends only on the row's length.  One pass takes
// consecutive rows while their classes do not grow and the blocks fit in the
// wavefront; with rows ordered longest first every block is aligned.  Split
// rows (class 1) sum their segment partials in segment order.
// UL: entries per group and step; size classes are counted in units of
// 2 unroll_of entries for any UL, and a class-S row's entry p goes to group
// p mod S in entry order whatever the step, so the result does not depend on UL.
template <int VT, int BT, int E, int CPL, bool FUSED = false, int UL = unroll_of<E, CPL>()>
__device__ __forceinline__ void vector_item_classed(const DevPlan &P, const RunArgs &a, int wid) {
    constexpr int U = UL;
    const int panel = wid / P.n_vitems, item = wid - panel * P.n_vitems;
    const int ncol0 = panel * a.np, ncols = min(a.np, P.n - ncol0);
    const Lanes L(a.lpr_log2);
    const int lane = threadIdx.x & 63;
    const __amdgpu_buffer_rsrc_t rs = b_resource(a.B, a.b_rec);
    bool cok[CPL];
    int64_t coff[CPL];
    chunk_layout<E, CPL>(ncol0, ncols, L, cok, coff);
    int sid = P.vitem_seg[item];
    const int i0 = P.vitem_ptr[item], i1 = P.vitem_ptr[item + 1];
    // id, remainder range, class and segments of rows base .. base + 63, one
    // per lane, loaded again only when fewer rows than a full pass takes
    // (L.groups) remain loaded
    int base = i0 - 64;
    int wr = -1, wb = 0, we = 0, wcls = 1, wns = 0;
    for (int i = i0; i < i1;) {
        if (i - base + L.groups > 64) {
            base = i;
            const int l_row = i + lane;
            wr = -1; wb = 0; we = 0; wcls = 1; wns = 0;
            if (l_row < i1) {
                wr = P.vec_rows ? P.vec_rows[l_row] : l_row;
                wb = P.rem_ptr[wr];
                we = P.rem_ptr[wr + 1];
                if (we - wb > P.seg_len) {
                    wns = (we - wb + P.seg_len - 1) / P.seg_len;
                    we = wb;  // the entries were summed by the segment kernel
                } else {
                    wcls = size_class(we - wb, 2 * unroll_of<E, CPL>(), L.groups);
                }
            }
        }
        // row i + lane, from the loaded rows (a lane past them ends the pass)
        const int j_row = i + lane, off = i - base;
        const bool have = lane + off < 64;
        const int srcl = min(lane + off, 63);
        int r = __shfl(wr, srcl, 64), b = __shfl(wb, srcl, 64), e = __shfl(we, srcl, 64);
        int cls = __shfl(wcls, srcl, 64), ns = __shfl(wns, srcl, 64);
        if (!have) {
            r = -1; b = 0; e = 0; cls = 1; ns = 0;
        }
        // the pass: rows before the first class increase whose blocks fit
        const int prev = __shfl_up(cls, 1, 64);
        const uint64_t cut = __ballot(j_row >= i1 || !have || (lane > 0 && cls > prev));
        const int kmax = cut ? __builtin_ctzll(cut) : 64;
        const int cin = lane < kmax ? cls : 0;
        const int incl = wave_inclusive_scan(cin);
        const uint64_t fits = __ballot(lane < kmax && incl <= L.groups);
        const int k = __popcll(fits);  // >= 1: row i always fits
        const int excl = incl - cin;
        // this lane group's row: the last block start at or below the group
        const uint64_t starts = wave_or64(lane < k ? (1ull << excl) : 0ull);
        const int g = L.group;
        const uint64_t upto = g >= 63 ? ~0ull : ((2ull << g) - 1ull);
        const int jr = (g < __shfl(incl, k - 1, 64)) ? __popcll(starts & upto) - 1 : -1;
        const int src = jr < 0 ? 0 : jr;
        int my_r = __shfl(r, src, 64), my_b = __shfl(b, src, 64), my_e = __shfl(e, src, 64);
        const int my_s = __shfl(cls, src, 64), my_ns = __shfl(ns, src, 64);
        const int local = g - __shfl(excl, src, 64);
        int my_sid = sid;
        if (__ballot(lane < k && ns > 0)) {
            const int nin = lane < k ? ns : 0;
            const int nincl = wave_inclusive_scan(nin);
            my_sid = sid + __shfl(nincl - nin, src, 64);
            sid += __shfl(nincl, k - 1, 64);
        }
        if (jr < 0) my_b = my_e = 0;
        const int smax = __builtin_amdgcn_readfirstlane(cls);  // the pass's largest class (lane 0)
        // the first group of a row's block stores it (fused: not a split row,
        // which its last segment stores)
        const bool writes = jr >= 0 && local == 0 && !(FUSED && my_ns > 0);

        float acc[CPL][E];
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int x = 0; x < E; ++x) acc[c][x] = 0.0f;
        // split rows (no entries left to gather) start from their segment sums
        if (!FUSED && jr >= 0 && my_ns > 0)
            sum_partials<E, CPL>(a.work, a.work_ld, my_sid, my_ns, ncol0, ncols, L, acc);
        Lanes Ls = L;
        Ls.groups = my_s;
        for (int p = my_b + local; p < my_e; p += my_s * U) {
            int col[U];
            float v[U];
            load_entries<VT, U, BT != DT_F32>(P.rem_col, P.rem_val, p, my_e, Ls, col, v);
            gather_fma<BT, E, CPL, U>(col, v, p, my_e, a.B, rs, a.ldb, a.b_rec, cok, coff, Ls, a.cold_aux,
                                      acc);
        }
        // butterfly inside each block, from the pass's largest class down
        for (int off = (smax * L.lpr) >> 1; off >= L.lpr; off >>= 1) {
            const bool take = off < my_s * L.lpr;
#pragma unroll
            for (int c = 0; c < CPL; ++c)
#pragma unroll
                for (int x = 0; x < E; ++x) {
                    const float t = __shfl_xor(acc[c][x], off, 64);
                    if (take) acc[c][x] += t;
                }
        }
        if (writes) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int q = c * L.lpr + L.li;
                if (q * E < ncols) store_chunk<E>(a.C, (int64_t)my_r * a.ldc + ncol0 + (int64_t)q * E, acc[c]);
            }
        }
        i += k;
    }
}
template <int VT, int BT, int E, int CPL, int VAR, bool FUSED = false, int UL = unroll_of<E, CPL>()>
__device__ __forceinline__ void vector_item_var(const DevPlan &P, const RunArgs &a, int wid) {
    if constexpr (VAR == 3) vector_item_classed<VT, BT, E, CPL, FUSED, UL>(P, a, wid);
    else if constexpr (VAR == 2) vector_item_packed<VT, BT, E, CPL, FUSED, UL>(P, a, wid);
    else if constexpr (VAR == 1) vector_item_pipelined<VT, BT, E, CPL, FUSED>(P, a, wid);
    else vector_item<VT, BT, E, CPL, FUSED>(P, a, wid);
}

// LDS of a window item: the staged B rows (reused for the f32 C tile), the
// round's tiles expanded from bitmap + packed values to dense 16-bit rows, and
// the window's rows, remainder ranges and segment ids.  MB = H / 16; NPWv =
// the panel width of an item (128 columns, or 64 / 32 for narrow 16-bit B).
// Staged B row k occupies NPWv * 2 bytes (NCH chunks of 8 elements) with
// chunk c stored in slot c ^ bswz<NCH>(k): the 8-row groups that one MFMA
// operand read touches then fall in different banks without padding, so a
// wave's 64 x 16-byte chunks are one contiguous kilobyte and can be written
// by one direct global-to-LDS load.
template <int MB, int NPWv = 128>
struct WinSmem {
    static constexpr int NPW = NPWv;         // panel columns of a window item
    static constexpr int NCH = NPW / 8;      // 16-byte chunks of a staged B row
    static constexpr int TC = 4;             // tiles staged per round
    static constexpr int KROWS = TC * 32;    // B rows staged per round
    static constexpr int BSTR = NPW;         // LDS row stride (16-bit elements)
    static constexpr int H = MB * 16;
    static_assert(NPW == 32 || NPW == 64 || NPW == 128, "panel width");
    __attribute__((aligned(16))) unsigned short Bs[KROWS * BSTR];
    __attribute__((aligned(16))) unsigned short As[TC * H * 32];  // expanded tiles, row-major
    int32_t rows[H], rb[H], re[H], sid[H];
    int32_t flag;  // last-arrival flag of a fused window item
};

template <int TT>
__device__ __forceinline__ f32x4 mfma_16x16x32(const u16x8 &a, const u16x8 &b, const f32x4 &c) {
    if constexpr (TT == DT_BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// 8 consecutive B elements (columns n .. n+7 of B row `col`) as TT bit patterns.
template <int BT, int TT>
__device__ __forceinline__ void stage_b8(const void *B, int64_t off, int valid, int vec,
                                         uint32_t (&w)[4]) {
    uint32_t h[8];
    if constexpr (BT == DT_F32) {
        float f[8];
        if (vec && valid == 8) {
            f32x4 x0 = *reinterpret_cast<const f32x4 *>(static_cast<const float *>(B) + off);
            f32x4 x1 = *reinterpret_cast<const f32x4 *>(static_cast<const float *>(B) + off + 4);
            f[0] = x0[0]; f[1] = x0[1]; f[2] = x0[2]; f[3] = x0[3];
            f[4] = x1[0]; f[5] = x1[1]; f[6] = x1[2]; f[7] = x1[3];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = i < valid ? static_cast<const float *>(B)[off + i] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) h[i] = f32_to_bf16_bits(f[i]);
    } else {
        const unsigned short *p = static_cast<const unsigned short *>(B) + off;
        if (vec && valid == 8) {
            u32x4 x = *reinterpret_cast<const u32x4 *>(p);
            w[0] = x[0]; w[1] = x[1]; w[2] = x[2]; w[3] = x[3];
            return;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) h[i] = i < valid ? p[i] : 0u;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = h[2 * i] | (h[2 * i + 1] << 16);
}

typedef short v4i16 __attribute__((ext_vector_type(4)));

// Slot of a chunk in a staged B row (see WinSmem).
template <int NCH>
__device__ __forceinline__ int bswz(int k) { return ((k >> 3) & (NCH / 4 - 1)) << 1; }

// One (window, NPWv-column panel) per workgroup: item in [0, n_win * win_panels),
// panel innermost, so a window's panels run side by side on one XCD and share
// its tile data in that XCD's L2.
// Every thread of the workgroup calls it with the same item.  Per round of up
// to TC tiles, with one barrier: each thread loads the columns of its own B
// staging chunks and then those B rows (16-bit B straight into LDS, f32 B
// through registers, converted to bf16), wave w expands tile w of the round
// from bitmap + packed values into dense 16-bit rows in LDS, and (first
// round) the window's row metadata goes to LDS; then MFMA from LDS only (an
// A operand is one 16-byte read, a B operand two transposing reads).  Then
// each row adds its remainder and is written once.
// A workgroup spends most of its life waiting on chains of dependent loads,
// so the loads of a round are issued level by level (item -> tile range and
// window rows -> tile columns, bitmaps, value base and row ranges -> B rows,
// values and remainder entries -> their B rows) with no branch around a load
// that would make the next one wait; the window order is skipped when it is
// the identity; the first remainder pass (window rows 0 .. 4G-1, one per lane
// group) gathers its rows' first U1 entries alongside the first round's tile
// loads and consumes them after the MFMA rounds.
// FUSED: partial items and owners of windows with a slot (win_dep) store
// their parts in the workspace and arrive at the window panel's counter; the
// last arrival combines (window_combine).  Owners skip split rows, which the
// combine takes from the segments' partials.
template <int VT, int BT, int TT, int MB, int E, int CPL, int SMB, bool FUSED = false, int NPWv = 128>
__device__ __forceinline__ void window_item(const DevPlan &P, const RunArgs &a, int item,
                                            WinSmem<SMB, NPWv> &sm, bool partial) {
    constexpr int H = MB * 16;
    using S = WinSmem<SMB, NPWv>;
    constexpr int NPW = S::NPW, NCH = S::NCH, TC = S::TC, BSTR = S::BSTR, KROWS = S::KROWS;
    constexpr int PER = KROWS * NCH / 256;        // 16-byte staging chunks per thread
    constexpr int RPP = 256 / NCH;                // B rows staged per pass
    constexpr int NB = NPW / 16;                  // 16-column MFMA blocks of the panel
    constexpr int NBW = (NB + 3) / 4;             // ... per wave (block wave + 4 nbi)
    constexpr int U1 = MB == 1 ? 4 : 2;           // remainder entries per row gathered early
    static_assert(MB <= SMB, "LDS sized for a smaller window");
    static_assert(H * NPW * 4 <= KROWS * BSTR * 2, "C tile must fit in the B stage");
    static_assert(TC <= 4, "wave w expands tile w of a round");
    unsigned short *Bs = sm.Bs;

    // owner items: (window in launch order, panel), tiles [t0, t0 + win_tmax);
    // partial items: (partial slot, panel), tiles [wpart_t0, wpart_t1)
    const int j_item = item / a.win_panels, panel = item - j_item * a.win_panels;
    const int wi = partial ? P.wpart_win[j_item] : (P.win_order ? P.win_order[j_item] : j_item);
    const int ncol0 = panel * NPW, ncols = min(NPW, P.n - ncol0);
    const bool full = a.vec_ok && ncols == NPW;  // every staging chunk is whole
    const int tid = threadIdx.x, wave = wave_id(), lane = tid & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int t0 = partial ? P.wpart_t0[j_item] : P.win_tile_ptr[wi];
    const int t1 = partial ? P.wpart_t1[j_item] : min(P.win_tile_ptr[wi + 1], t0 + P.win_tmax);
    const int pa = partial ? 0 : P.win_part[wi], pb = partial ? 0 : P.win_part[wi + 1];
    const int seg0 = partial ? 0 : P.win_seg[wi];  // first segment id of the window's rows
    float *wpart = a.work + (int64_t)P.n_seg * a.work_ld;  // window partials follow the segments

    // window rows: lane `lane` of every wave holds row lane % H (wave 0 puts
    // them in LDS), lane group `group` of wave `wave` owns row s1 of the first
    // remainder pass
    const Lanes L(a.win_lpr_log2);
    const Lanes one = L.single();
    const int s1 = wave * L.groups + L.group;
    const int64_t wrow0 = (int64_t)(partial ? 0 : wi) * H;
    const int rm = P.windows[wrow0 + (lane & (H - 1))];
    const int r1 = P.windows[wrow0 + min(s1, H - 1)];

    bool cok[CPL];
    int64_t coff[CPL];
    chunk_layout<E, CPL>(ncol0, ncols, L, cok, coff);
    int col1[U1];
    float val1[U1];
    Raw<BT, E> g1[U1][CPL];
    int b1 = 0, e1 = 0;

    f32x4 acc[MB][NBW];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int j = 0; j < NBW; ++j) acc[mb][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // level 2 of a round: the tile columns of this thread's staging chunks,
    // and the bitmap words and value offsets of the tile this wave expands
    // (wave w expands tile w of the round).  The next round's are loaded
    // alongside this round's staging loads, so a round after the first
    // starts with its tile values and B rows.
    struct RoundMeta {
        int colr[PER];
        uint32_t wrd[MB];
        int tv, vend;
    };
    auto fetch_meta = [&](int tc0, RoundMeta &m) {
        const int nt = min(TC, t1 - tc0);
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int kr = (tid + it * 256) / NCH;
            const int c = P.tile_cols[(int64_t)tc0 * 32 + min(kr, nt * 32 - 1)];
            m.colr[it] = kr < nt * 32 ? c : -1;
        }
        const int wv = min(wave, nt - 1);
        m.vend = P.tile_val_ptr[tc0 + nt];
        m.tv = P.tile_val_ptr[tc0 + wv];
#pragma unroll
        for (int rp = 0; rp < MB; ++rp) m.wrd[rp] = P.tile_bitmap[(int64_t)(tc0 + wv) * H + rp * 16 + (lane >> 2)];
    };

    auto round = [&](auto first_tag, int tc0, const RoundMeta &m, RoundMeta &next) {
        constexpr bool FIRST = decltype(first_tag)::value;
        const int nt = min(TC, t1 - tc0);
        const int(&colr)[PER] = m.colr;
        const uint32_t(&wrd)[MB] = m.wrd;
        const int tv = m.tv, vend = m.vend;
        // lane (r, q) = (lane / 4, lane % 4) of wave w takes columns
        // 8q .. 8q+7 of rows r, r + 16, .. of tile w
        const int q4 = lane & 3;
        int bm_ = 0, em_ = 0;
        if constexpr (FIRST) {
            bm_ = P.rem_ptr[max(rm, 0)];
            em_ = P.rem_ptr[max(rm, 0) + 1];
            b1 = P.rem_ptr[max(r1, 0)];
            e1 = P.rem_ptr[max(r1, 0) + 1];
        }
        // level 3: tile values, remainder entries, B rows of the staging chunks.
        // A row's values follow those of the tile's earlier rows (prefix over
        // the 16-row passes by a wave scan) and, inside the row, the bitmap
        // order; every load is issued at a clamped index and masked after.
        uint32_t av[MB][4];
        {
            int carry = 0;
#pragma unroll
            for (int rp = 0; rp < MB; ++rp) {
                const uint32_t word = wrd[rp], mine = (word >> (8 * q4)) & 0xFFu;
                const int pc = __popc(word);
                const int incl = wave_inclusive_scan(q4 == 0 ? pc : 0);
                const int base = tv + carry + incl - pc + __popc(word & ((1u << (8 * q4)) - 1u));
                carry += __shfl(incl, 63, 64);
                // this lane's values are consecutive in the packed order:
                // one (2-byte aligned) 16-byte load at `base` holds them (the
                // plan's arrays end in at least 16 zero bytes), then set bit
                // i takes the next value in turn
                u32x4 raw;
                __builtin_memcpy(&raw, P.tile_vals + max(min(base, vend), 0), 16);
                uint64_t lo = (uint64_t)raw[0] | ((uint64_t)raw[1] << 32);
                uint64_t hi = (uint64_t)raw[2] | ((uint64_t)raw[3] << 32);
                unsigned short x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bool set = (mine >> i) & 1u;
                    x[i] = set ? (unsigned short)(lo & 0xFFFFu) : (unsigned short)0;
                    const uint64_t nlo = (lo >> 16) | (hi << 48), nhi = hi >> 16;
                    lo = set ? nlo : lo;
                    hi = set ? nhi : hi;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) av[rp][i] = (uint32_t)x[2 * i] | ((uint32_t)x[2 * i + 1] << 16);
            }
        }
        bool live1 = false, split1 = false;
        int q1 = 0;
        if constexpr (FIRST) {
            live1 = !partial && s1 < H && r1 >= 0;
            split1 = e1 - b1 > P.seg_len;
            q1 = live1 && !split1 ? e1 : b1;  // end of the entries gathered here
            // indices clamped into [0, q1 - 1] (the plan arrays carry a zero
            // tail for an empty range); entries at and beyond q1 are not used
#pragma unroll
            for (int u = 0; u < U1; ++u) {
                const int pp = max(min(b1 + u, q1 - 1), 0);
                col1[u] = __builtin_nontemporal_load(P.rem_col + pp);
                val1[u] = load_val<VT>(P.rem_val, pp);
            }
        }
        // B rows of the staging chunks: thread tid stages, in pass it, row
        // kr = RPP it + tid / NCH into LDS bytes [4096 it + 16 tid, +16), i.e.
        // slot tid % NCH of that row, which holds chunk (tid % NCH) ^ bswz(kr)
        if constexpr (BT != DT_F32) {
            if (full) {
                // one direct global-to-LDS load per pass and wave; chunks
                // without a column (tile padding, rows beyond the round) read
                // the plan's zero block
#pragma unroll
                for (int it = 0; it < PER; ++it) {
                    const int kr = RPP * it + tid / NCH, cg = (tid & (NCH - 1)) ^ bswz<NCH>(kr);
                    const unsigned short *src =
                        colr[it] >= 0 ? static_cast<const unsigned short *>(a.B) +
                                            (int64_t)colr[it] * a.ldb + ncol0 + cg * 8
                                      : P.zeros;
                    __builtin_amdgcn_global_load_lds(
                        src, (__attribute__((address_space(3))) void *)(Bs + it * 2048 + wave * 512), 16, 0,
                        0);
                }
            } else {
#pragma unroll
                for (int it = 0; it < PER; ++it) {
                    const int kr = RPP * it + tid / NCH, cg = (tid & (NCH - 1)) ^ bswz<NCH>(kr);
                    uint32_t w[4] = {0u, 0u, 0u, 0u};
                    const int valid = min(8, ncols - cg * 8);
                    if (colr[it] >= 0 && valid > 0)
                        stage_b8<BT, TT>(a.B, (int64_t)colr[it] * a.ldb + ncol0 + cg * 8, valid, a.vec_ok, w);
                    *reinterpret_cast<u32x4 *>(&Bs[it * 2048 + tid * 8]) = u32x4{w[0], w[1], w[2], w[3]};
                }
            }
        } else {
            // f32 B, converted to bf16: two passes' loads in flight at a time
#pragma unroll
            for (int h = 0; h < PER; h += 2) {
                uint32_t w[2][4];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int it = h + q, kr = RPP * it + tid / NCH, cg = (tid & (NCH - 1)) ^ bswz<NCH>(kr);
                    w[q][0] = w[q][1] = w[q][2] = w[q][3] = 0u;
                    const int valid = min(8, ncols - cg * 8);
                    if (full) {
                        const float *b = static_cast<const float *>(a.B) +
                                         (int64_t)max(colr[it], 0) * a.ldb + ncol0 + cg * 8;
                        const f32x4 x0 = *reinterpret_cast<const f32x4 *>(b);
                        const f32x4 x1 = *reinterpret_cast<const f32x4 *>(b + 4);
                        const bool ok = colr[it] >= 0;
                        w[q][0] = ok ? (f32_to_bf16_bits(x0[0]) | (f32_to_bf16_bits(x0[1]) << 16)) : 0u;
                        w[q][1] = ok ? (f32_to_bf16_bits(x0[2]) | (f32_to_bf16_bits(x0[3]) << 16)) : 0u;
                        w[q][2] = ok ? (f32_to_bf16_bits(x1[0]) | (f32_to_bf16_bits(x1[1]) << 16)) : 0u;
                        w[q][3] = ok ? (f32_to_bf16_bits(x1[2]) | (f32_to_bf16_bits(x1[3]) << 16)) : 0u;
                    } else if (colr[it] >= 0 && valid > 0) {
                        stage_b8<BT, TT>(a.B, (int64_t)colr[it] * a.ldb + ncol0 + cg * 8, valid, a.vec_ok,
                                         w[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    *reinterpret_cast<u32x4 *>(&Bs[(h + q) * 2048 + tid * 8]) =
                        u32x4{w[q][0], w[q][1], w[q][2], w[q][3]};
            }
        }
        // the next round's level 2, in flight with this round's staging
        if (tc0 + TC < t1) fetch_meta(tc0 + TC, next);
        // LDS: expanded tiles (tile w, row r, columns 8q ..: 16 bytes at
        // ((w H + r) 32 + 8q) elements), row metadata
        if (wave < nt) {
#pragma unroll
            for (int rp = 0; rp < MB; ++rp)
                *reinterpret_cast<u32x4 *>(&sm.As[((wave * H + rp * 16 + (lane >> 2)) * 32) + 8 * q4]) =
                    u32x4{av[rp][0], av[rp][1], av[rp][2], av[rp][3]};
        }
        if constexpr (FIRST) {
            if (wave == 0 && !partial) {
                // the window's rows, their remainder ranges and segment ids
                const bool own = lane < H && rm >= 0;
                const int len = own ? em_ - bm_ : 0;
                const int ns = len > P.seg_len ? (len + P.seg_len - 1) / P.seg_len : 0;
                const int x = wave_inclusive_scan(ns);
                if (lane < H) {
                    sm.rows[lane] = rm;
                    sm.rb[lane] = bm_;
                    sm.re[lane] = em_;
                    sm.sid[lane] = seg0 + x - ns;
                }
            }
        }
        __syncthreads();
        if constexpr (FIRST) {
            // level 4: the early remainder entries' B rows (a valid row for
            // unused entries and chunks outside the panel), issued after the
            // barrier (which waits for the staging loads) and consumed after
            // the MFMA rounds
#pragma unroll
            for (int u = 0; u < U1; ++u)
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    load_raw<BT, E, false>(a.B, (int64_t)(col1[u] & 0x7FFFFFFF) * a.ldb + coff[c], g1[u][c]);
        }
        for (int j = 0; j < nt; ++j) {
            // A operand: lane (g, m) takes row m, columns 8g .. 8g+7 of tile j
            u16x8 af[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                af[mb] = *reinterpret_cast<const u16x8 *>(&sm.As[((j * H + mb * 16 + l16) * 32) + 8 * g]);
#pragma unroll
            for (int nbi = 0; nbi < NBW; ++nbi) {
                const int nb = wave + 4 * nbi;
                if (NB < 4 && nb >= NB) continue;  // narrow panels: waves without a block
                // B operand: lane (g, n) needs rows 8g .. 8g+7 of column n.
                // ds_read_b64_tr_b16 transposes within each 16-lane block:
                // lane a of the block reads 4 consecutive columns of one row,
                // and lane n receives element i from lane 4i + n/4, column
                // n % 4; so lane a reads row 4h + a/4, columns 4(a % 4) ..
                u16x8 bf;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = j * 32 + 8 * g + 4 * h + (l16 >> 2), n0 = nb * 16 + 4 * (l16 & 3);
                    const v4i16 t = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                        (__attribute__((address_space(3))) v4i16 *)(Bs + k * BSTR +
                                                                    (((n0 >> 3) ^ bswz<NCH>(k)) << 3) + (n0 & 7)));
#pragma unroll
                    for (int i = 0; i < 4; ++i) bf[4 * h + i] = (unsigned short)t[i];
                }
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[mb][nbi] = mfma_16x16x32<TT>(af[mb], bf, acc[mb][nbi]);
            }
        }
        return q1;
    };
    // a valid plan gives every window and partial item at least one tile
    RoundMeta cur, nxt;
    fetch_meta(t0, cur);
    const int q1 = round(std::true_type{}, t0, cur, nxt);
    for (int tc0 = t0 + TC; tc0 < t1; tc0 += TC) {
        __syncthreads();  // the previous round's LDS reads are done
        cur = nxt;
        (void)round(std::false_type{}, tc0, cur, nxt);
    }
    // fused: the window's slot when its result needs other items' parts
    const int dep = FUSED ? P.win_dep[wi] : -1;
    if (partial || dep >= 0) {
        // the MFMA result of these tiles: for the owner item (or the last
        // arrival) to add, or the owner's own, kept in the window's slot
        float *dst = (partial ? wpart + (int64_t)j_item * H * a.work_ld
                              : a.dep + (int64_t)dep * 2 * H * a.work_ld) + ncol0;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nbi = 0; nbi < NBW; ++nbi) {
                const int col = (wave + 4 * nbi) * 16 + l16;
                if (wave + 4 * nbi < NB && col < ncols) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float *d = dst + (int64_t)(mb * 16 + 4 * g + i) * a.work_ld + col;
                        if constexpr (FUSED) st_dev1(ws_resource(a), d - a.work, acc[mb][nbi][i]);
                        else *d = acc[mb][nbi][i];
                    }
                }
            }
        if (partial) {
            if constexpr (FUSED) {
                if (group_arrive(win_counter(P, a, panel, dep), win_target(P, a, wi, panel), &sm.flag))
                    window_combine(P, a, wi, panel, dep, tid, 256);
            }
            return;
        }
    }
    // the first pass's rows: their early entries, then the rest in order
    float v1[CPL][E];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int x = 0; x < E; ++x) v1[c][x] = 0.0f;
    fma_rows<BT, E, CPL, U1>(val1, g1, b1, q1, one, v1);
    if (q1 > b1 + U1)
        row_accumulate_group<VT, BT, E, CPL, unroll_of<E, CPL>()>(
            P.rem_col, P.rem_val, b1 + U1, q1, a.B, a.ldb, a.b_rec, ncol0, ncols, L, a.cold_aux, v1);
    __syncthreads();
    float *Cs = reinterpret_cast<float *>(Bs);
    if (dep < 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nbi = 0; nbi < NBW; ++nbi)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (wave + 4 * nbi < NB)
                        Cs[(mb * 16 + 4 * g + i) * NPW + (wave + 4 * nbi) * 16 + l16] = acc[mb][nbi][i];
    }
    // add the partial results of the window's other tiles, in tile order
    // (fused: a window with partial items has a slot, combined at the end)
    if (!FUSED && pb > pa) {
        __syncthreads();
        for (int x = tid; x < H * NPW; x += 256) {
            const int srow = x / NPW, col = x - srow * NPW;
            if (col < ncols) {
                float v = Cs[x];
                for (int k = pa; k < pb; ++k)
                    v += wpart[((int64_t)k * H + srow) * a.work_ld + ncol0 + col];
                Cs[x] = v;
            }
        }
    }
    __syncthreads();

    // Remainders: every lane group takes its own row of the window, so up to
    // 4 * G rows progress at once; a row's entries are summed in order by its
    // group.  Rows then add the tile result and are written once.
    for (int s0 = 0; s0 < H; s0 += 4 * L.groups) {
        const int s = s0 + s1;
        const int r = s < H ? sm.rows[s] : -1;
        float v[CPL][E];
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
            for (int x = 0; x < E; ++x) v[c][x] = s0 == 0 ? v1[c][x] : 0.0f;
        if (r >= 0) {
            const int b = sm.rb[s], e = sm.re[s];
            const bool split = e - b > P.seg_len;
            if (split) {
                // fused: only windows with a slot have split rows; the
                // combine sums their segment partials
                if constexpr (!FUSED) {
                    const int ns = (e - b + P.seg_len - 1) / P.seg_len;
                    sum_partials<E, CPL>(a.work, a.work_ld, sm.sid[s], ns, ncol0, ncols, L, v);
                }
            } else if (s0 != 0) {
                row_accumulate_group<VT, BT, E, CPL, unroll_of<E, CPL>()>(
                    P.rem_col, P.rem_val, b, e, a.B, a.ldb, a.b_rec, ncol0, ncols, L, a.cold_aux, v);
            }
            if (dep >= 0) {
                // the row's remainder, for the combine
                if (!split) {
                    const int64_t rm = (a.dep - a.work) + ((int64_t)dep * 2 + 1) * H * a.work_ld +
                                       (int64_t)s * a.work_ld + ncol0;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const int q = c * L.lpr + L.li;
                        if (q * E < ncols) st_dev_chunk<E>(ws_resource(a), rm + (int64_t)q * E, v[c]);
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int q = c * L.lpr + L.li;
                    if (q * E < ncols) {
#pragma unroll
                        for (int x = 0; x < E; ++x) v[c][x] = Cs[s * NPW + q * E + x] + v[c][x];
                        store_chunk<E>(a.C, (int64_t)r * a.ldc + ncol0 + (int64_t)q * E, v[c]);
                    }
                }
            }
        }
    }
    if constexpr (FUSED) {
        if (dep >= 0 && group_arrive(win_counter(P, a, panel, dep), win_target(P, a, wi, panel), &sm.flag))
            window_combine(P, a, wi, panel, dep, tid, 256);
    }
}
}  // namespace spmm
