// Internal types shared by the host builder, the ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/spmm.h"

namespace spmm {

constexpr uint32_t kMaxTileRows = 4096;
constexpr uint32_t kDefaultTileRows = 32;
constexpr uint32_t kDefaultTileCols = 65536;
constexpr uint32_t kDefaultItemNnz = 16384;
constexpr uint32_t kMaxItemNnz = 131072;
// Rows longer than this are cut into several row segments in the ROW
// variant, so that one lane never walks an unbounded row.
constexpr uint32_t kRowLaneMax = 1024;
// Rows at least this long go to a whole wavefront in the HYBRID variant.
constexpr uint32_t kWaveRowMin = 64;
// Largest column chunk one kernel launch accumulates (LDS budget).
constexpr int kMaxKc = 32;

// One work item = one wavefront.  It owns the local rows [lo, hi) of one
// tile row (slab) -- its LDS accumulator rows -- and all of their entries in
// every tile of the slab, unless it is one piece of a row too long for one
// item (then hi = lo + 1 and `part` names the partial slot it writes).
//
// Payload layout (byte offsets from blob_off, see item_layout):
//   coo_ent  u32[n_coo]      bit 31: first entry of a new strip run;
//                            bits 16..27: local row; bits 0..15: local col;
//                            column-major order inside each strip run
//   coo_val  f32[n_coo]      weighted A only
//   coo_J    u32[n_coo_J]    strip (tile column) of each COO tile run
//   lr_seg   u32x2[n_lr]     x = row | strip ordinal << 12,
//                            y = first col slot | length << 21   (8-aligned)
//   lr_J     u32[n_lr_J]     strip of each ordinal
//   wr_seg   u32x4[n_wr]     {strip, row, first col, length}     (16-aligned)
//   cols     u16[n_cols]     row-lane segments interleaved in blocks of 64
//                            (element t of segment i of a block at
//                            block_base + i + 64 t), then wavefront segments
//   col_val  f32[n_cols]     weighted A only                     (4-aligned)
struct ItemDesc {
    uint64_t blob_off;
    uint32_t slab;
    int32_t part;  // -1: the item owns rows [lo, hi); else its partial slot
    uint32_t rows; // lo | hi << 16
    uint32_t cid;  // split rows: index of the row's CombineDesc
    uint32_t n_coo, n_coo_J, n_lr, n_lr_J, n_wr, n_cols;
};
static_assert(sizeof(ItemDesc) == 48, "ItemDesc must stay 48 bytes");

struct ItemLayout {
    uint32_t o_coo_J, o_lr, o_lr_J, o_wr, o_cols, o_cval, bytes;
};

__host__ __device__ inline uint32_t align_to(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline ItemLayout item_layout(const ItemDesc& d, bool has_val) {
    ItemLayout L;
    L.o_coo_J = 4u * d.n_coo * (has_val ? 2u : 1u);
    L.o_lr = align_to(L.o_coo_J + 4u * d.n_coo_J, 8);
    L.o_lr_J = L.o_lr + 8u * d.n_lr;
    L.o_wr = align_to(L.o_lr_J + 4u * d.n_lr_J, 16);
    L.o_cols = L.o_wr + 16u * d.n_wr;
    L.o_cval = align_to(L.o_cols + 2u * d.n_cols, 4);
    L.bytes = align_to(L.o_cval + (has_val ? 4u * d.n_cols : 0u), 16);
    return L;
}

constexpr uint32_t kCooNewTile = 0x80000000u;
constexpr uint32_t kLrStartBits = 21;  // lr_seg.y: start < 2^21, length < 2^11

// A row split across several items: Y[row] = sum of the partial slots
// [part_begin, part_end), formed by whichever piece finishes last.
struct CombineDesc {
    uint32_t slab, row, part_begin, part_end;
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

// Untiled CSR store (format SPMM_FORMAT_CSR, the V-csr baseline): rows in
// order of descending length (row_old maps them back), columns in the
// handle's column order, sorted within each row.
constexpr int64_t kCsrWaveMin = 128;  // rows longer than this: one wavefront each
constexpr int64_t kCsrPiece = 8192;   // rows longer than this: pieces of this many entries
struct CsrStore {
    std::vector<int64_t> rp;          // n_rows + 1, in row order
    std::vector<int32_t> col;
    std::vector<int64_t> seg;         // per wavefront segment: row, first entry, end entry, partial slot or -1
    std::vector<int64_t> srow, pb;    // split rows; their first partial slot (n_split + 1 entries)
    int64_t n_seg = 0, n_split = 0, n_wave_rows = 0, n_pieces = 0;
    int64_t* d_rp = nullptr;
    int32_t* d_col = nullptr;
    int64_t* d_seg = nullptr;
    int64_t* d_srow = nullptr;
    int64_t* d_pb = nullptr;
    float* d_part = nullptr;          // n_pieces x 32 partial sums
};

struct Handle {
    int64_t n_rows = 0, n_cols = 0, nnz = 0;
    uint32_t format = SPMM_FORMAT_TILES;
    CsrStore csr;
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
    double max_row_l1 = 0.0;           // max over rows of sum |a_ij|
    uint32_t* d_colmax = nullptr;      // per X column: max |x| (FP32 bits)
    int32_t* d_fexp = nullptr;         // per X column: fixed-point exponent
    // Column relabelling: tile columns are ranks by descending in-degree, so
    // the X rows of hub columns are contiguous (cache-resident).
    bool relabel = false;
    std::vector<int32_t> col_new;      // new index of original column c
    std::vector<int32_t> col_old;      // original column of new index
    int32_t* d_col_old = nullptr;      // device copy of col_old
    std::vector<uint32_t> col_count;   // entries per original column
    uint32_t* d_col_count = nullptr;   // device copy (PageRank out-degrees)
    void* d_xperm = nullptr;           // X in relabelled row order
    uint64_t xperm_bytes = 0;
    // Row relabelling: tile rows hold the rows in order of descending
    // out-degree; rows [n_tiled_rows, n_rows) of that order have no entries
    // and are zero-filled.  Without relabelling row_old is empty and
    // n_tiled_rows = n_rows.
    bool row_relabel = false;
    std::vector<int32_t> row_old;      // original row of tiled row r
    int64_t n_tiled_rows = 0;
    int32_t* d_row_old = nullptr;      // device copy of row_old
    void* d_nmf_ws = nullptr;          // NMF workspace (kept between calls)
    size_t nmf_ws_bytes = 0;
    // The canonical tile store (tiles, ent, val, variant, slab_tiles) holds
    // tile rows slab_base .. n_slabs-1.  A one-shot build keeps all of them
    // (canonical = true: the selector can re-encode); a slab-wise build
    // encodes each block of tile rows as it is cut and drops it
    // (canonical = false: only the encoded payload remains).
    bool canonical = true;
    uint64_t slab_base = 0;
    uint64_t n_tiles_total = 0;        // tiles cut so far, dropped or not
    // slab-wise build state: rows appended so far, rows not yet tiled (a
    // partial tile row), rows without entries (zero-filled)
    bool building = false;
    bool validate_rows = false;
    bool has_val_known = true;         // a slab-wise build learns it from its first block
    int32_t fixed_variant = -1;
    int64_t next_row = 0;
    std::vector<int64_t> pend_row;
    std::vector<uint64_t> pend_off;
    std::vector<int32_t> pend_col;
    std::vector<float> pend_val;
    std::vector<int32_t> zero_rows;
    // encoded work
    Encoded enc;
    // device / pinned copies
    void* d_blob = nullptr;       // device blob (PLACE_DEVICE)
    void* h_blob = nullptr;       // pinned host blob (PLACE_PINNED_HOST)
    ItemDesc* d_items = nullptr;
    CombineDesc* d_combine = nullptr;
    int64_t* d_part = nullptr;    // partial results of split rows, n_parts * kc fixed-point
    uint32_t* d_count = nullptr;  // per split slab: items finished in this launch
    uint64_t part_cap = 0;
    int max_kc = 16;              // widest column chunk per launch (16 or 32)
    uint64_t stage_bytes = 0;     // LDS per workgroup for staged X rows (0 = none)
    // streamed mode: item groups copied host -> device ring per SpMM
    struct Group {
        uint64_t i0, i1;          // items
        uint64_t b0, b1;          // payload bytes
        uint64_t r0, r1;          // tiled rows the items write
    };
    std::vector<Group> groups;
    uint64_t stream_bytes = 0;
    uint32_t ring_depth = 0;
    std::vector<void*> ring;      // device slots, each max group bytes
    std::vector<hipEvent_t> ev_ready, ev_free;
    std::vector<uint8_t> ring_used;  // slot has been read by a kernel (ev_free recorded)
    // Y streamed out to host memory: one device Y slot per ring slot
    void* d_yring = nullptr;
    uint64_t yslot_bytes = 0;
    std::vector<hipEvent_t> ev_y_ready, ev_y_free;
    std::vector<uint8_t> y_used;     // slot's copy-out has been enqueued (ev_y_free recorded)
    // side stream that zero-fills the rows without entries while the SpMM
    // runs (fork and join events on the caller's stream)
    hipStream_t zstream = nullptr;
    hipEvent_t ev_zfork = nullptr, ev_zjoin = nullptr;
    int device = 0;
    bool uploaded = false;
    // optional timing of the SpMM launches of each run (event pairs)
    bool timing = false;
    size_t timing_used = 0;
    std::vector<hipEvent_t> timing_ev;  // start, stop, start, stop, ...
};

// Strip-table entries of an item's COO stream staged in LDS per wavefront.
constexpr uint32_t kJTab = 256;

// Widest column chunk per launch: a wavefront's 64-bit accumulators for h
// rows plus its strip table fit in 64 KiB of LDS, within the handle's max_kc.
inline int kc_cap(const Handle& H) {
    int cap = H.max_kc;
    while (cap > 1 && (uint64_t)H.h * cap * 8u + kJTab * 4u > 65536u) cap >>= 1;
    return cap;
}

// builder.cpp
// Fields of H a build starts from (shape, tile geometry and options set).
void build_init(Handle& H, bool has_val);
// One-shot build of the tile store from a whole CSR (rp[0] = 0).
spmm_status_t build_canonical(Handle& H, const int64_t* row_ptr, const int32_t* col,
                              const float* val, bool validate, std::string& err);
// Slab-wise build: rows [row0, row0 + nr) with local row pointers (rp[0] =
// 0), appended in order; columns keep the given order.
spmm_status_t build_append(Handle& H, int64_t row0, int64_t nr, const int64_t* rp, const int32_t* col,
                           const float* val, bool validate, std::string& err);
// Tile the rows still pending and complete the row map.
spmm_status_t build_finish_rows(Handle& H, std::string& err);
spmm_status_t flush_slabs(Handle& H, std::string& err);
// The untiled CSR store of a binary matrix (format SPMM_FORMAT_CSR).
spmm_status_t build_csr(Handle& H, const int64_t* row_ptr, const int32_t* col, bool validate, std::string& err);
spmm_status_t encode(Handle& H, std::string& err);
// Encode tile rows [s0, s1) of the canonical store and append them to H.enc.
spmm_status_t encode_range(Handle& H, uint64_t s0, uint64_t s1, std::string& err);
// CSR of the transpose of an n_rows x n_cols CSR (rows ascending within each
// row of the result; duplicates kept), with range checks on the input.
spmm_status_t transpose_csr(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr, const int32_t* col,
                            const float* val, uint32_t threads, std::vector<int64_t>& tp, std::vector<int32_t>& tc,
                            std::vector<float>& tv, std::string& err);
// Transfer groups of streamed mode: consecutive items of about stream_bytes
// of payload, never splitting the pieces of one split row.
std::vector<Handle::Group> make_groups(const Encoded& E, uint64_t stream_bytes, uint32_t h);
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
    int64_t* part;               // device, split-row partial sums (n_parts * column chunk)
    uint32_t* count;             // device, n_combine counters, zero between launches
    const int32_t* fexp;         // device, per column of X: fixed-point exponent
    const int32_t* rmap;         // device, original row of each tiled row (NULL: identity)
};
hipError_t launch_spmm(const Handle& H, const RunArgs& a);
// csr_kernels.hip: Y = A X over the CSR store, FP32 X in the handle's
// column order (k columns, row stride ldx), Y rows through H.d_row_old.
hipError_t launch_csr(const Handle& H, const float* X, int64_t ldx, int k, float* Y, int64_t ldy, hipStream_t s);
// Zero the k columns of the Y rows that have no entries (the original rows
// rmap[n_tiled .. n_rows) of a row-relabelled handle).
hipError_t launch_zero_rows(float* Y, int64_t ldy, int k, const int32_t* rows, int64_t count, hipStream_t s);
// X prepared for a launch: optionally gathered into the handle's column
// order (Xp row i = X row old_of_new[i], row stride ldp; Xp NULL = read in
// place), and the per-column fixed-point exponents of the accumulators:
// with M_j = max |x_j| and R = max row L1 norm of A, f_j = 61 - e_j where
// R M_j < 2^e_j, so every partial sum of a row, scaled by 2^f_j, stays below
// 2^61 in magnitude.
hipError_t launch_prepare_x(const void* X, int dtype, int64_t ldx, int k, const int32_t* old_of_new, int64_t n,
                            void* Xp, int64_t ldp, double row_l1, uint32_t* colmax, int32_t* fexp,
                            hipStream_t s);

// apps_kernels.hip
hipError_t launch_pr_init(float* pr, int64_t n, float v, hipStream_t s);
hipError_t launch_pr_prepare(const float* pr, const uint32_t* outdeg, const int32_t* old_of_new, int64_t n,
                             float* xp, double* dpart, double* D, hipStream_t s);
hipError_t launch_pr_update(float* pr, const float* y, int64_t n, double damping, const double* D,
                            int redistribute, double* rpart, double* resid_slot, hipStream_t s);
int gram_blocks();
hipError_t launch_gram(const float* M, int64_t n, int r, double* part, float* G, hipStream_t s);
hipError_t launch_mu_update(float* M, const float* S, const float* G, int64_t n, int r, float eps, hipStream_t s);

// mlp_kernels.hip: device workspace of a gradient evaluation over n rows
struct MlpScratch {
    float *x, *a1, *a2, *d1, *d2, *d3;  // n x 8, n x 64 (four), n x V
    double* loss_rows;                   // n
    uint32_t* count;                     // 1: measured targets
};
hipError_t launch_mlp_predict(const float* params, const float* feat, int64_t n, float* out, uint8_t* choice,
                              hipStream_t s);
hipError_t launch_mlp_grad(const float* params, const float* feat, const float* target, const uint8_t* mask,
                           const int32_t* idx, int64_t n, const MlpScratch& w, float* grad, double* loss,
                           hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int np, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);

// probe_kernels.hip: one streaming read of bytes (a multiple of 16) at buf
hipError_t launch_read_probe(const void* buf, uint64_t bytes, float* sink, hipStream_t s);

// Layout of a tall FP32 block of columns: element (i, c) is at
// base + (c / bw) * bstride + (c % bw) + i * ld.  Row-major with row stride
// ld: bw at least the column count and bstride 0.  Column-blocked (arrays of
// bw columns, each n x bw contiguous, bstride elements apart): ld = bw.
struct ColLayout {
    int64_t ld;
    int32_t bw;
    int64_t bstride;
};
inline ColLayout row_major(int64_t ld) { return ColLayout{ld, 0x7fffffff, 0}; }
__host__ __device__ inline int64_t col_off(const ColLayout& L, int c) {
    return (int64_t)(c / L.bw) * L.bstride + (c % L.bw);
}

// Tall-skinny dense kernels of the eigensolver (FP32 data, FP64 arithmetic).
int ts_max_outputs();          // largest p * q launch_ts_tn accepts
int ts_max_width();            // largest p + q launch_ts_tn accepts
size_t ts_partial_doubles();   // size of the part buffer launch_ts_tn needs
// C (p x q FP64, row-major) = A^T B; A n x p (layout LA), B n x q (stride ldb).
hipError_t launch_ts_tn(const float* A, ColLayout LA, int p, const float* B, int64_t ldb, int q, int64_t n,
                        double* part, double* C, hipStream_t s);
// W = alpha W + beta A C; A n x p (layout LA), C p x q FP64, W n x q (layout
// LW; must not alias A).
hipError_t launch_ts_nn(const float* A, ColLayout LA, int p, const double* C, int q, double alpha, double beta,
                        float* W, ColLayout LW, int64_t n, hipStream_t s);
// X[i][c] (c < q <= 64) uniform in [-1/2, 1/2), a function of (seed, i, c).
hipError_t launch_fill_uniform(float* X, int64_t ldx, int q, int64_t n, uint64_t seed, hipStream_t s);

// quant_kernels.hip
hipError_t launch_quantize(const float* X, int64_t n, int k, int64_t ldx, int dtype, void* Xq,
                           int64_t ldq, float* col_scale, bool scales_given, hipStream_t s);

}  // namespace spmm
