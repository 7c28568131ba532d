// plan.hpp -- host-side plan: the integer partition of A and its work lists.
//
// Built by build_host_plan() from a CSR matrix and resolved options; no HIP
// call is made here, so the builder also runs (and is tested) without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "spmm.h"

namespace spmm {

constexpr int kWave = 64;
constexpr int kRowCost = 4;  // per-row overhead of a vector item, in entry units
// Tiles a window item computes itself (the rest of a window's tiles go to
// partial items of as many tiles each): the least power of two in
// [kWinTiles, kWinTilesMax] that brings the plan's tiles over all 128-column
// panels down to about kWindowItems items, i.e. about as many as the CUs
// hold at once (window_item_tiles).  More, smaller items only add partial
// results that go through memory and back (an item's partial C tile is as
// large as its whole result).
constexpr int kWinTiles = 16;
constexpr int kWinTilesMax = 128;
constexpr int64_t kWindowItems = 1024;
int32_t window_item_tiles(int64_t tiles, int32_t n);

struct HostPlan {
    // ---- problem and resolved options ----
    int64_t m = 0, k = 0, nnz = 0;
    int32_t n = 0;
    int32_t val_type = SPMM_F32, b_type = SPMM_F32, c_type = SPMM_F32, tile_type = SPMM_BF16;
    spmm_opts opts{};  // every field resolved (no "auto" left)

    // ---- partition (compared bit-for-bit with the reference) ----
    std::vector<int32_t> windows;       // [W*H], -1 = empty slot
    std::vector<int32_t> tile_window;   // [T]
    std::vector<int32_t> tile_cols;     // [T*kt], -1 = padding
    std::vector<uint32_t> tile_bitmap;  // [T*H]
    std::vector<int64_t> tile_val_ptr;  // [T+1]
    std::vector<uint16_t> tile_vals;    // bf16 / f16 bit patterns
    std::vector<int64_t> tile_src;      // CSR entry of each packed value
    std::vector<int64_t> rem_ptr;       // [m+1]
    std::vector<int64_t> rem_src;       // CSR entry of each remainder entry
    std::vector<int32_t> vector_rows;   // ascending
    std::vector<int32_t> nseg;          // [m]

    // ---- schedule ----
    std::vector<int32_t> vexec;         // launch order of vector rows (item by item); empty: vector_rows
    std::vector<int32_t> vitem_ptr;     // [V+1] into the launch order
    std::vector<int32_t> vitem_seg;     // [V]
    std::vector<int32_t> seg_row, seg_begin, seg_end;  // [S]
    std::vector<int32_t> win_tile_ptr;  // [W+1]
    std::vector<int32_t> win_seg;       // [W]
    std::vector<int32_t> win_order;     // [W]
    std::vector<int32_t> win_part;      // [W+1]: partial items of window w are [win_part[w], win_part[w+1])
    std::vector<int32_t> wpart_win, wpart_t0, wpart_t1;  // [n_wparts]
    int32_t win_tiles = kWinTiles;      // tiles an owner item computes; partial items take as many
    bool identity_rows = false;         // vector_rows == 0..m-1

    // ---- co-scheduled execution (derive_exec_tables, from the schedule) ----
    std::vector<int32_t> seg_win;       // [S] window of the segment's row, -1 for a vector row (empty: W = 0)
    std::vector<int32_t> win_dep;       // [W] slot of a window needing other items' parts, else -1
    std::vector<int32_t> win_nsseg;     // [W] segments of the window's split rows
    std::vector<int32_t> win_row_sid;   // [W*H] first segment of a window row that is split, else -1
    int32_t n_dep = 0;                  // windows with a slot

    // ---- device-facing copies of the remainder ----
    std::vector<int32_t> rem_ptr32;     // [m+1]
    std::vector<int32_t> rem_col;       // [nnz_rem], bit 31 set for hot columns
    std::vector<uint8_t> rem_val;       // [nnz_rem * s_val] raw bytes of val_type

    // ---- statistics ----
    int64_t k_ref = 0;
    int64_t hot_cols = 0;               // columns flagged for cacheable gathers
    double plan_ms = 0.0;
};

int dtype_size(int32_t t);

constexpr double kL2BytesPerXcd = 4.0 * 1024 * 1024;  // gfx950: 4 MiB L2 per XCD
constexpr double kHotFraction = 0.8;                   // cap of the cached B working set

// Fill *o with library defaults for every "auto" field of `in` (in may be null).
// Needs only the problem shape; never reads the matrix values.
void resolve_options(const spmm_opts *in, const spmm_csr *A, int32_t n, int32_t b_type,
                     spmm_opts *o);

// Sizes, dtypes and null pointers only (the arrays are not read).
spmm_status validate_shape(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                           std::string &err);

// Validate the CSR and sizes.  Returns SPMM_OK or an error with a message.
spmm_status validate_problem(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                             std::string &err);

// Range checks of resolved options (no "auto" left).
spmm_status validate_opts(const spmm_opts &o, std::string &err);

// Plan serialisation: a versioned, checksummed image of every HostPlan array.
void serialize_host_plan(const HostPlan &P, std::vector<uint8_t> &out);
// Parses an image and checks every index invariant the kernels rely on, so
// that a plan that loads cannot make a kernel read or write out of bounds.
spmm_status deserialize_host_plan(const uint8_t *buf, size_t size, HostPlan &P, std::string &err);

// Work of the two paths of a plan: entries gathered by the segment and vector
// kernels, tile slots (tiles * H * kt), and remainder entries of window rows
// gathered inside the window kernels.
void plan_path_work(const HostPlan &P, double *w_vec, double *w_tile, double *w_winrem);

// Build the full host plan for already-resolved options.
spmm_status build_host_plan(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                            const spmm_opts &o, HostPlan &P, std::string &err);

// The schedule of a partitioned plan (P.opts, m, windows, win_tile_ptr and
// rem_ptr set): vector rows, segments, vector items, window segment ids,
// window partial items and the window launch order (Sec. 7).
void build_schedule(HostPlan &P);

// The tables of co-scheduled execution: which window each segment's row
// belongs to, and a slot for every window whose result needs other items
// (partial tiles beyond its first win_tiles, or rows split into segments).
void derive_exec_tables(HostPlan &P);

// float -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN).
uint16_t f32_to_bf16_rne(float f);

}  // namespace spmm
