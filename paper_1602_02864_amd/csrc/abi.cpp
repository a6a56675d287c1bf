// C ABI: argument checks, handle lifecycle, device upload, dispatch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "spmm_internal.h"

struct spmm_handle_s {
    spmm::Handle H;
};

namespace {

thread_local std::string g_err;

spmm_status_t fail(spmm_status_t st, const std::string& msg) {
    g_err = msg;
    return st;
}

spmm_status_t hip_fail(hipError_t e, const char* what) {
    return fail(SPMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

void free_device(spmm::Handle& H) {
    if (H.d_blob) hipFree(H.d_blob);
    if (H.d_items) hipFree(H.d_items);
    if (H.d_combine) hipFree(H.d_combine);
    if (H.d_part) hipFree(H.d_part);
    if (H.d_count) hipFree(H.d_count);
    if (H.d_col_old) hipFree(H.d_col_old);
    if (H.d_xperm) hipFree(H.d_xperm);
    H.d_col_old = nullptr;
    H.d_xperm = nullptr;
    H.xperm_bytes = 0;
    if (H.h_blob) hipHostFree(H.h_blob);
    H.d_blob = H.h_blob = nullptr;
    H.d_items = nullptr;
    H.d_combine = nullptr;
    H.d_part = nullptr;
    H.d_count = nullptr;
    H.part_cap = 0;
    H.uploaded = false;
}

// Copy the encoded work to the device (descriptors always; the payload to
// HBM or to pinned host memory depending on the placement).
spmm_status_t upload(spmm::Handle& H) {
    spmm::Encoded& E = H.enc;
    hipError_t e;
    if ((e = hipGetDevice(&H.device)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    const size_t nb = E.blob.size() ? E.blob.size() : 16;
    if (H.place == SPMM_PLACE_DEVICE) {
        if ((e = hipMalloc(&H.d_blob, nb)) != hipSuccess) return fail(SPMM_ENOMEM, "hipMalloc(tile payload) failed");
        if (E.blob.size() && (e = hipMemcpy(H.d_blob, E.blob.data(), E.blob.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(tile payload)");
    } else {
        if ((e = hipHostMalloc(&H.h_blob, nb, hipHostMallocDefault)) != hipSuccess)
            return fail(SPMM_ENOMEM, "hipHostMalloc(tile payload) failed");
        if (E.blob.size()) std::memcpy(H.h_blob, E.blob.data(), E.blob.size());
    }
    const size_t ni = E.items.size() ? E.items.size() : 1;
    if ((e = hipMalloc(&H.d_items, ni * sizeof(spmm::ItemDesc))) != hipSuccess)
        return fail(SPMM_ENOMEM, "hipMalloc(item descriptors) failed");
    if (E.items.size() &&
        (e = hipMemcpy(H.d_items, E.items.data(), E.items.size() * sizeof(spmm::ItemDesc), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(item descriptors)");
    const size_t nc = E.combine.size() ? E.combine.size() : 1;
    if ((e = hipMalloc(&H.d_combine, nc * sizeof(spmm::CombineDesc))) != hipSuccess)
        return fail(SPMM_ENOMEM, "hipMalloc(combine list) failed");
    if (E.combine.size() &&
        (e = hipMemcpy(H.d_combine, E.combine.data(), E.combine.size() * sizeof(spmm::CombineDesc), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(combine list)");
    if ((e = hipMalloc(&H.d_count, nc * sizeof(uint32_t))) != hipSuccess)
        return fail(SPMM_ENOMEM, "hipMalloc(combine counters) failed");
    if ((e = hipMemset(H.d_count, 0, nc * sizeof(uint32_t))) != hipSuccess)
        return hip_fail(e, "hipMemset(combine counters)");
    if (H.relabel && H.n_cols > 0) {
        if ((e = hipMalloc(&H.d_col_old, sizeof(int32_t) * (size_t)H.n_cols)) != hipSuccess)
            return fail(SPMM_ENOMEM, "hipMalloc(column order) failed");
        if ((e = hipMemcpy(H.d_col_old, H.col_old.data(), sizeof(int32_t) * (size_t)H.n_cols,
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(column order)");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if (H.place == SPMM_PLACE_PINNED_HOST) std::vector<uint8_t>().swap(E.blob);  // pinned copy replaces it
    H.uploaded = true;
    return SPMM_OK;
}

spmm_status_t ensure_uploaded(spmm::Handle& H) {
    if (H.uploaded) return SPMM_OK;
    spmm_status_t st = upload(H);
    if (st != SPMM_OK) free_device(H);
    return st;
}

spmm_status_t ensure_partials(spmm::Handle& H) {
    const uint64_t need = H.enc.n_parts * (uint64_t)spmm::kc_cap(H);
    if (need == 0 || need <= H.part_cap) return SPMM_OK;
    if (H.d_part) hipFree(H.d_part);
    H.d_part = nullptr;
    H.part_cap = 0;
    if (hipMalloc(&H.d_part, need * sizeof(float)) != hipSuccess)
        return fail(SPMM_ENOMEM, "hipMalloc(partial results) failed");
    H.part_cap = need;
    return SPMM_OK;
}

spmm_status_t check_run_args(const spmm::Handle& H, const void* X, int k, int64_t ldx,
                             spmm_xdtype_t dt, const float* col_scale, const float* Y, int64_t ldy) {
    if (k < 1 || k > 64) return fail(SPMM_EINVAL, "k must be in 1..64");
    if (ldx < k || ldy < k) return fail(SPMM_EINVAL, "ldx and ldy must be >= k");
    if (dt != SPMM_X_F32 && dt != SPMM_X_BF16 && dt != SPMM_X_FP8_E4M3)
        return fail(SPMM_EINVAL, "unknown X dtype");
    if ((dt == SPMM_X_FP8_E4M3) != (col_scale != nullptr))
        return fail(SPMM_EINVAL, "col_scale must be given exactly when X is FP8");
    if ((H.n_cols > 0 && !X) || (H.n_rows > 0 && !Y)) return fail(SPMM_EINVAL, "X or Y is NULL");
    return SPMM_OK;
}

}  // namespace

extern "C" {

const char* spmm_last_error(void) { return g_err.c_str(); }

spmm_status_t spmm_build_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, const float* values,
                               const spmm_build_opts* opts, spmm_handle_t* out) {
    try {
        if (!out) return fail(SPMM_EINVAL, "out is NULL");
        if (n_rows < 0 || n_cols < 0 || n_rows > INT32_MAX || n_cols > INT32_MAX)
            return fail(SPMM_EINVAL, "n_rows and n_cols must be in 0..2^31-1");
        if (!row_ptr) return fail(SPMM_EINVAL, "row_ptr is NULL");
        if (row_ptr[n_rows] > 0 && !col_idx) return fail(SPMM_EINVAL, "col_idx is NULL");
        spmm_build_opts o{};
        if (opts) o = *opts;
        if (o.max_kc == 0) o.max_kc = 32;
        if (o.max_kc != 16 && o.max_kc != 32) return fail(SPMM_EINVAL, "max_kc must be 16 or 32");
        if (o.tile_rows == 0) o.tile_rows = spmm::kDefaultTileRows;
        if (o.tile_cols == 0) o.tile_cols = spmm::kDefaultTileCols;
        if (o.item_nnz == 0) o.item_nnz = spmm::kDefaultItemNnz;
        if (o.tile_rows > spmm::kMaxTileRows) return fail(SPMM_EINVAL, "tile_rows must be <= 4096");
        if (o.item_nnz > spmm::kMaxItemNnz) return fail(SPMM_EINVAL, "item_nnz must be <= 131072");
        if (!is_pow2(o.tile_cols) || o.tile_cols > 65536)
            return fail(SPMM_EINVAL, "tile_cols must be a power of two <= 65536");
        if (o.fixed_variant >= SPMM_NUM_VARIANTS) return fail(SPMM_EINVAL, "unknown variant");
        if (o.place != SPMM_PLACE_DEVICE && o.place != SPMM_PLACE_PINNED_HOST)
            return fail(SPMM_EINVAL, "unknown placement");
        std::unique_ptr<spmm_handle_s> hs(new spmm_handle_s);
        spmm::Handle& H = hs->H;
        H.n_rows = n_rows;
        H.n_cols = n_cols;
        H.h = o.tile_rows;
        H.w = o.tile_cols;
        H.item_nnz = o.item_nnz;
        H.threads = o.threads;
        H.place = o.place;
        H.max_kc = (int)o.max_kc;
        H.relabel = o.keep_order == 0;
        std::string err;
        spmm_status_t st = spmm::build_canonical(H, row_ptr, col_idx, values, o.validate != 0, err);
        if (st != SPMM_OK) return fail(st, err);
        if (o.fixed_variant >= 0) std::fill(H.variant.begin(), H.variant.end(), (uint8_t)o.fixed_variant);
        st = spmm::encode(H, err);
        if (st != SPMM_OK) return fail(st, err);
        *out = hs.release();
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    } catch (const std::exception& e) {
        return fail(SPMM_EINVAL, e.what());
    }
}

void spmm_destroy(spmm_handle_t h) {
    if (!h) return;
    free_device(h->H);
    delete h;
}

spmm_status_t spmm_run(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                       const float* col_scale, float* Y, int64_t ldy, hipStream_t s) {
    try {
        if (!h) return fail(SPMM_EINVAL, "handle is NULL");
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_DEVICE) return fail(SPMM_ESTATE, "tiles are placed in host memory; use spmm_stream_run");
        spmm_status_t st = check_run_args(H, X, k, ldx, dt, col_scale, Y, ldy);
        if (st != SPMM_OK) return st;
        if (H.n_rows == 0) return SPMM_OK;
        if ((st = ensure_uploaded(H)) != SPMM_OK) return st;
        if ((st = ensure_partials(H)) != SPMM_OK) return st;
        spmm::RunArgs a{};
        a.X = X;
        a.k = k;
        a.ldx = ldx;
        if (H.relabel && H.n_cols > 0) {
            // gather X into the relabelled row order, rows padded to 4 elements
            const int esize = dt == SPMM_X_F32 ? 4 : dt == SPMM_X_BF16 ? 2 : 1;
            const int64_t ldp = (k + 3) / 4 * 4;
            const uint64_t need = (uint64_t)H.n_cols * ldp * esize;
            if (need > H.xperm_bytes) {
                if (H.d_xperm) hipFree(H.d_xperm);
                H.d_xperm = nullptr;
                H.xperm_bytes = 0;
                if (hipMalloc(&H.d_xperm, need) != hipSuccess)
                    return fail(SPMM_ENOMEM, "hipMalloc(relabelled X) failed");
                H.xperm_bytes = need;
            }
            hipError_t pe = spmm::launch_permute_rows(X, ldx, k, esize, H.d_col_old, H.n_cols, H.d_xperm, ldp, s);
            if (pe != hipSuccess) return hip_fail(pe, "X permutation launch");
            a.X = H.d_xperm;
            a.ldx = ldp;
        }
        a.dtype = dt;
        a.col_scale = col_scale;
        a.Y = Y;
        a.ldy = ldy;
        a.stream = s;
        a.blob = static_cast<const uint8_t*>(H.d_blob);
        a.blob_bias = 0;
        a.items = H.d_items;
        a.n_items = (uint32_t)H.enc.items.size();
        a.combine = H.d_combine;
        a.n_combine = (uint32_t)H.enc.combine.size();
        a.count = H.d_count;
        hipError_t e = spmm::launch_spmm(H, a);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return SPMM_OK;
    } catch (const std::exception& e) {
        return fail(SPMM_EINVAL, e.what());
    }
}

spmm_status_t spmm_quantize_x(const float* X, int64_t n, int k, int64_t ldx, spmm_xdtype_t dt,
                              void* Xq, int64_t ldq, float* col_scale, uint32_t flags,
                              hipStream_t s) {
    if (n < 0 || k < 1 || k > 64) return fail(SPMM_EINVAL, "need n >= 0 and 1 <= k <= 64");
    if (ldx < k || ldq < k) return fail(SPMM_EINVAL, "ldx and ldq must be >= k");
    if (dt != SPMM_X_BF16 && dt != SPMM_X_FP8_E4M3)
        return fail(SPMM_EINVAL, "dt must be SPMM_X_BF16 or SPMM_X_FP8_E4M3");
    if ((dt == SPMM_X_FP8_E4M3) != (col_scale != nullptr))
        return fail(SPMM_EINVAL, "col_scale must be given exactly when dt is FP8");
    if (flags & ~SPMM_QUANT_SCALES_GIVEN) return fail(SPMM_EINVAL, "unknown flags");
    if (n > 0 && (!X || !Xq)) return fail(SPMM_EINVAL, "X or Xq is NULL");
    hipError_t e = spmm::launch_quantize(X, n, k, ldx, dt, Xq, ldq, col_scale,
                                         (flags & SPMM_QUANT_SCALES_GIVEN) != 0, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "quantize launch");
}

spmm_status_t spmm_get_stats(spmm_handle_t h, spmm_stats_t* out) {
    if (!h || !out) return fail(SPMM_EINVAL, "NULL argument");
    const spmm::Handle& H = h->H;
    spmm_stats_t s{};
    s.n_rows = (uint64_t)H.n_rows;
    s.n_cols = (uint64_t)H.n_cols;
    s.nnz = (uint64_t)H.nnz;
    s.tile_rows = H.h;
    s.tile_cols = H.w;
    s.n_slabs = H.n_slabs;
    s.n_tiles = H.tiles.size();
    s.sum_nnr = H.sum_nnr;
    s.sum_nnc = H.sum_nnc;
    s.n_items = H.enc.items.size();
    s.n_parts = H.enc.n_parts;
    s.blob_bytes = H.blob_bytes;
    s.desc_bytes = H.enc.items.size() * sizeof(spmm::ItemDesc) + H.enc.combine.size() * sizeof(spmm::CombineDesc);
    for (int v = 0; v < SPMM_NUM_VARIANTS; ++v) {
        s.variant_tiles[v] = H.enc.variant_tiles[v];
        s.variant_nnz[v] = H.enc.variant_nnz[v];
    }
    *out = s;
    return SPMM_OK;
}

spmm_status_t spmm_decode_tiles(spmm_handle_t h, int64_t* row_ptr, int32_t* col_idx, float* values) {
    try {
        if (!h || !row_ptr || (h->H.nnz > 0 && !col_idx)) return fail(SPMM_EINVAL, "NULL argument");
        if (values && !h->H.has_val) return fail(SPMM_EINVAL, "the matrix is binary; pass values = NULL");
        std::string err;
        spmm_status_t st = spmm::decode(h->H, row_ptr, col_idx, values, err);
        return st == SPMM_OK ? st : fail(st, err);
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_model_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, int64_t t, uint64_t* n_tiles,
                               uint64_t* sum_nnr, uint64_t* sum_nnc) {
    try {
        if (n_rows < 0 || n_cols < 0 || t < 1 || !row_ptr || !n_tiles || !sum_nnr || !sum_nnc)
            return fail(SPMM_EINVAL, "bad argument");
        if (row_ptr[n_rows] > 0 && !col_idx) return fail(SPMM_EINVAL, "col_idx is NULL");
        return spmm::model_tiles(n_rows, n_cols, row_ptr, col_idx, t, 0, n_tiles, sum_nnr, sum_nnc);
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

}  // extern "C"
