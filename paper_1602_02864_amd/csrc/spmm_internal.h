// Internal types shared by the host builder, the ABI layer and the kernels.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/spmm.h"

namespace spmm {

constexpr uint32_t kMaxTileRows = 4096;
constexpr uint32_t kDefaultTileRows = 256;
constexpr uint32_t kDefaultTileCols = 65536;
constexpr uint32_t kDefaultItemNnz = 16384;
// Rows longer than this are cut into several row segments in the ROW
// variant, so that one lane never walks an unbounded row.
constexpr uint32_t kRowLaneMax = 1024;
// Rows at least this long go to a whole wavefront in the HYBRID variant.
constexpr uint32_t kWaveRowMin = 64;
// Largest column chunk one kernel launch accumulates (LDS budget).
constexpr int kMaxKc = 32;

// One work item = one wavefront.  It owns a part of one tile row (slab):
// its LDS accumulator covers the slab's h rows.  All offsets are in bytes,
// relative to the item's payload start in the blob.
//
// Payload layout (16-byte aligned start):
//   coo_ent   u32[n_coo]        (row << 16) | col, grouped by tile
//   coo_val   f32[n_coo]        only for weighted A
//   coo_tile  u32x2[n_coo_tiles] {strip J, first entry}, 8-byte aligned
//   lr_desc   u32[n_lr]         row | (strip ordinal << 16)
//   lr_start  u32[n_lr + 1]     segment extents into cols
//   lr_J      u32[n_lr_tiles]   strip of each ordinal
//   wr_seg    u32x4[n_wr]       {J, row, first col, length}, 16-byte aligned
//   cols      u16[...]          columns of lr and wr segments
//   col_val   f32[...]          only for weighted A, 4-byte aligned
struct ItemDesc {
    uint64_t blob_off;
    uint32_t slab;
    int32_t part;  // -1: the item owns its slab; else its partial-result slot
    uint32_t n_coo, n_coo_tiles, n_lr, n_wr;
    uint32_t cid;  // split slabs: index of the slab's CombineDesc (coo_val sits at 4 * n_coo)
    uint32_t o_coo_tile, o_lr_desc, o_lr_start, o_lr_J, o_wr, o_cols, o_col_val;
};
static_assert(sizeof(ItemDesc) == 64, "ItemDesc must stay 64 bytes");

// A split slab: Y rows = sum of the partial slots [part_begin, part_end),
// formed by whichever of its items finishes last.
struct CombineDesc {
    uint32_t slab, part_begin, part_end, pad;
};

// Canonical tile (host): entries ent[ent_begin, ent_begin + nnz) sorted by
// local row, then local column.
struct Tile {
    uint64_t ent_begin;
    uint32_t slab, J;
    uint32_t nnz, nnr, nnc, max_row, n_single;
};

struct Encoded {
    std::vector<ItemDesc> items;
    std::vector<uint32_t> item_nnz;
    std::vector<CombineDesc> combine;
    std::vector<uint8_t> blob;
    uint64_t n_parts = 0;
    uint64_t variant_tiles[SPMM_NUM_VARIANTS] = {};
    uint64_t variant_nnz[SPMM_NUM_VARIANTS] = {};
};

struct Handle {
    int64_t n_rows = 0, n_cols = 0, nnz = 0;
    uint32_t h = 0, w = 0, wshift = 0;
    uint32_t item_nnz = 0;
    uint32_t threads = 0;
    uint32_t place = SPMM_PLACE_DEVICE;
    bool has_val = false;
    uint64_t n_slabs = 0, n_strips = 0;
    // canonical tile store (host)
    std::vector<uint32_t> ent;   // (row << 16) | col, tile-major
    std::vector<float> val;      // per entry, weighted A only
    std::vector<Tile> tiles;
    std::vector<uint64_t> slab_tiles;  // tiles of slab s: [slab_tiles[s], slab_tiles[s+1])
    std::vector<uint8_t> variant;      // per tile
    uint64_t sum_nnr = 0, sum_nnc = 0;
    uint64_t blob_bytes = 0;
    // encoded work
    Encoded enc;
    // device / pinned copies
    void* d_blob = nullptr;       // device blob (PLACE_DEVICE)
    void* h_blob = nullptr;       // pinned host blob (PLACE_PINNED_HOST)
    ItemDesc* d_items = nullptr;
    CombineDesc* d_combine = nullptr;
    float* d_part = nullptr;      // partial results, n_parts * h * kMaxKc floats
    uint32_t* d_count = nullptr;  // per split slab: items finished in this launch
    uint64_t part_cap = 0;
    int max_kc = 16;              // widest column chunk per launch (16 or 32)
    int device = 0;
    bool uploaded = false;
};

// Widest column chunk whose per-wavefront accumulator (h x kc FP32) fits
// in 64 KB of LDS, bounded by the handle's max_kc.
inline int kc_cap(const Handle& H) {
    int cap = H.max_kc;
    while (cap > 1 && (uint64_t)H.h * cap * 4u > 65536u) cap >>= 1;
    return cap;
}

// builder.cpp
spmm_status_t build_canonical(Handle& H, const int64_t* row_ptr, const int32_t* col,
                              const float* val, bool validate, std::string& err);
spmm_status_t encode(Handle& H, std::string& err);
spmm_status_t decode(const Handle& H, int64_t* row_ptr, int32_t* col, float* val, std::string& err);
void tile_features(const Handle& H, int k, int xbytes, float* out);
spmm_status_t model_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                          const int32_t* col, int64_t t, uint32_t threads, uint64_t* n_tiles,
                          uint64_t* sum_nnr, uint64_t* sum_nnc);
void parallel_for(uint64_t n, uint32_t threads, uint64_t grain,
                  const std::function<void(uint64_t, uint64_t)>& fn);

// kernels.hip launchers
struct RunArgs {
    const void* X;
    int k;
    int64_t ldx;
    int dtype;
    const float* col_scale;
    float* Y;
    int64_t ldy;
    hipStream_t stream;
    const uint8_t* blob;     // device base of the payload bytes being read
    uint64_t blob_bias;      // subtracted from ItemDesc::blob_off
    const ItemDesc* items;   // device
    uint32_t n_items;
    const CombineDesc* combine;  // device
    uint32_t n_combine;
    uint32_t* count;             // device, n_combine counters, zero between launches
};
hipError_t launch_spmm(const Handle& H, const RunArgs& a);

// quant_kernels.hip
hipError_t launch_quantize(const float* X, int64_t n, int k, int64_t ldx, int dtype, void* Xq,
                           int64_t ldq, float* col_scale, bool scales_given, hipStream_t s);

}  // namespace spmm
