// C ABI: argument checks, handle lifecycle, device upload, dispatch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "abi_internal.h"
#include "stream_plan.h"

namespace spmm_abi {

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
    if (H.d_blob) (void)hipFree(H.d_blob);
    if (H.d_items) (void)hipFree(H.d_items);
    if (H.d_combine) (void)hipFree(H.d_combine);
    if (H.d_part) (void)hipFree(H.d_part);
    if (H.d_count) (void)hipFree(H.d_count);
    if (H.d_colmax) (void)hipFree(H.d_colmax);
    if (H.d_fexp) (void)hipFree(H.d_fexp);
    H.d_colmax = nullptr;
    H.d_fexp = nullptr;
    if (H.d_col_old) (void)hipFree(H.d_col_old);
    if (H.d_row_old) (void)hipFree(H.d_row_old);
    H.d_row_old = nullptr;
    {
        spmm::CsrStore& C = H.csr;
        for (void* q : {(void*)C.d_rp, (void*)C.d_col, (void*)C.d_seg, (void*)C.d_srow, (void*)C.d_pb, (void*)C.d_part})
            if (q) (void)hipFree(q);
        C.d_rp = nullptr;
        C.d_col = nullptr;
        C.d_seg = C.d_srow = C.d_pb = nullptr;
        C.d_part = nullptr;
    }
    if (H.d_nmf_ws) (void)hipFree(H.d_nmf_ws);
    H.d_nmf_ws = nullptr;
    H.nmf_ws_bytes = 0;
    if (H.d_col_count) (void)hipFree(H.d_col_count);
    H.d_col_count = nullptr;
    if (H.d_xperm) (void)hipFree(H.d_xperm);
    H.d_col_old = nullptr;
    H.d_xperm = nullptr;
    H.xperm_bytes = 0;
    if (H.h_blob) (void)hipHostFree(H.h_blob);
    for (void* q : H.ring) (void)hipFree(q);
    for (hipEvent_t e : H.ev_ready) (void)hipEventDestroy(e);
    for (hipEvent_t e : H.ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : H.ev_y_ready) (void)hipEventDestroy(e);
    for (hipEvent_t e : H.ev_y_free) (void)hipEventDestroy(e);
    H.ev_y_ready.clear();
    H.ev_y_free.clear();
    H.y_used.clear();
    if (H.d_yring) (void)hipFree(H.d_yring);
    H.d_yring = nullptr;
    H.yslot_bytes = 0;
    if (H.ev_zfork) (void)hipEventDestroy(H.ev_zfork);
    if (H.ev_zjoin) (void)hipEventDestroy(H.ev_zjoin);
    if (H.zstream) (void)hipStreamDestroy(H.zstream);
    H.ev_zfork = H.ev_zjoin = nullptr;
    H.zstream = nullptr;
    for (hipEvent_t e : H.timing_ev) (void)hipEventDestroy(e);
    H.timing_ev.clear();
    H.timing_used = 0;
    H.timing = false;
    H.ring.clear();
    H.ring_used.clear();
    H.ev_ready.clear();
    H.ev_free.clear();
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
        H.groups = spmm::make_groups(E, H.stream_bytes, H.h);
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
    if (hipMalloc(&H.d_colmax, 64 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&H.d_fexp, 64 * sizeof(int32_t)) != hipSuccess)
        return fail(SPMM_ENOMEM, "hipMalloc(fixed-point scales) failed");
    if ((e = hipMemset(H.d_count, 0, nc * sizeof(uint32_t))) != hipSuccess)
        return hip_fail(e, "hipMemset(combine counters)");
    if (H.relabel && H.n_cols > 0) {
        if ((e = hipMalloc(&H.d_col_old, sizeof(int32_t) * (size_t)H.n_cols)) != hipSuccess)
            return fail(SPMM_ENOMEM, "hipMalloc(column order) failed");
        if ((e = hipMemcpy(H.d_col_old, H.col_old.data(), sizeof(int32_t) * (size_t)H.n_cols,
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(column order)");
    }
    if (H.format == SPMM_FORMAT_CSR) {
        spmm::CsrStore& C = H.csr;
        auto put = [&](auto** dst, const auto& v, const char* what) -> spmm_status_t {
            const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(v[0]);
            if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess)
                return fail(SPMM_ENOMEM, std::string("hipMalloc(") + what + ") failed");
            if (!v.empty()) {
                hipError_t ce = hipMemcpy(*dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
                if (ce != hipSuccess) return hip_fail(ce, what);
            }
            return SPMM_OK;
        };
        spmm_status_t ps;
        if ((ps = put(&C.d_rp, C.rp, "CSR row pointers")) != SPMM_OK || (ps = put(&C.d_col, C.col, "CSR columns")) != SPMM_OK ||
            (ps = put(&C.d_seg, C.seg, "CSR segments")) != SPMM_OK || (ps = put(&C.d_srow, C.srow, "CSR split rows")) != SPMM_OK ||
            (ps = put(&C.d_pb, C.pb, "CSR pieces")) != SPMM_OK)
            return ps;
        if (hipMalloc(&C.d_part, std::max<int64_t>(C.n_pieces, 1) * 32 * sizeof(float)) != hipSuccess)
            return fail(SPMM_ENOMEM, "hipMalloc(CSR partial sums) failed");
    }
    if (!H.row_old.empty()) {
        if ((e = hipMalloc(&H.d_row_old, sizeof(int32_t) * H.row_old.size())) != hipSuccess)
            return fail(SPMM_ENOMEM, "hipMalloc(row order) failed");
        if ((e = hipMemcpy(H.d_row_old, H.row_old.data(), sizeof(int32_t) * H.row_old.size(),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(row order)");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if (H.place == SPMM_PLACE_PINNED_HOST) std::vector<uint8_t>().swap(E.blob);  // pinned copy replaces it
    H.uploaded = true;
    return SPMM_OK;
}

spmm_status_t check_ready(spmm_handle_t h) {
    if (!h) return fail(SPMM_EINVAL, "handle is NULL");
    if (h->H.building) return fail(SPMM_ESTATE, "the handle is still being built (call spmm_build_end)");
    return SPMM_OK;
}

spmm_status_t ensure_uploaded(spmm::Handle& H) {
    if (H.building) return fail(SPMM_ESTATE, "the handle is still being built (call spmm_build_end)");
    if (H.uploaded) return SPMM_OK;
    spmm_status_t st = upload(H);
    if (st != SPMM_OK) free_device(H);
    return st;
}

spmm_status_t ensure_partials(spmm::Handle& H) {
    const uint64_t need = H.enc.n_parts * (uint64_t)spmm::kc_cap(H);  // int64 slots
    if (need == 0 || need <= H.part_cap) return SPMM_OK;
    if (H.d_part) (void)hipFree(H.d_part);
    H.d_part = nullptr;
    H.part_cap = 0;
    if (hipMalloc(&H.d_part, need * sizeof(int64_t)) != hipSuccess)
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

spmm_status_t prepare_device(spmm::Handle& H) {
    spmm_status_t st = ensure_uploaded(H);
    if (st != SPMM_OK) return st;
    return ensure_partials(H);
}

spmm_status_t ensure_xperm(spmm::Handle& H, uint64_t need) {
    if (need <= H.xperm_bytes) return SPMM_OK;
    if (H.d_xperm) (void)hipFree(H.d_xperm);
    H.d_xperm = nullptr;
    H.xperm_bytes = 0;
    if (hipMalloc(&H.d_xperm, need) != hipSuccess) return fail(SPMM_ENOMEM, "hipMalloc(relabelled X) failed");
    H.xperm_bytes = need;
    return SPMM_OK;
}

// Enqueue Y = A X on s over the device-resident payload.  With
// x_in_handle_order the rows of X are already in the handle's column order;
// otherwise (and if the handle relabels columns) X is first gathered into a
// handle-owned buffer in that order.  Buffers must already exist when this
// runs under stream capture (it allocates only when X needs gathering).
// X for the SpMM launches of one run: gathered into the handle's column
// order when the handle relabels columns and X is not already in that order
// (rows of 1 or 2 elements stay dense; wider rows are padded to a multiple
// of 4 elements so that they can be read as 16-byte vectors), and the
// fixed-point exponents taken from the values read.
spmm_status_t prepare_x(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt, hipStream_t s,
                        bool x_in_handle_order, spmm::RunArgs& a) {
    a.X = X;
    a.k = k;
    a.ldx = ldx;
    const int32_t* perm = nullptr;
    void* Xp = nullptr;
    int64_t ldp = ldx;
    if (H.relabel && H.n_cols > 0 && !x_in_handle_order) {
        const int esize = dt == SPMM_X_F32 ? 4 : dt == SPMM_X_BF16 ? 2 : 1;
        ldp = k <= 2 ? k : (k + 3) / 4 * 4;
        spmm_status_t st = ensure_xperm(H, (uint64_t)H.n_cols * ldp * esize);
        if (st != SPMM_OK) return st;
        perm = H.d_col_old;
        Xp = H.d_xperm;
    }
    hipError_t e = spmm::launch_prepare_x(X, dt, ldx, k, perm, H.n_cols, Xp, ldp, H.max_row_l1, H.d_colmax,
                                          H.d_fexp, s);
    if (e != hipSuccess) return hip_fail(e, "X preparation launch");
    if (Xp) {
        a.X = Xp;
        a.ldx = ldp;
    }
    a.fexp = H.d_fexp;
    return SPMM_OK;
}

// Rows without entries of a row-relabelled handle are not tiled: zero them.
spmm_status_t zero_empty_rows(const spmm::Handle& H, float* Y, int64_t ldy, int k, hipStream_t s) {
    if (!H.d_row_old || H.n_tiled_rows >= H.n_rows) return SPMM_OK;
    hipError_t e = spmm::launch_zero_rows(Y, ldy, k, H.d_row_old + H.n_tiled_rows, H.n_rows - H.n_tiled_rows, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "zero-row launch");
}

// Zero-fill the rows without entries on a side stream, concurrently with the
// X preparation and the SpMM (the two write disjoint rows of Y), when there
// are enough of them to matter and s is not being captured into a graph.
// Returns true when the fill was enqueued there; the caller then joins with
// join_zero_rows after the SpMM launches.
// Below 2^26 values (256 MB) the fill is shorter than what the fork, the
// join and the fill's share of the CUs cost the SpMM (measured at scale 25:
// slower by 0.1-0.2 ms for k <= 4, faster by 0.4-0.7 ms for k >= 16).
// Zero-fill wavefronts inside the SpMM launch were measured too: after the
// last item they gained less, spread among the items they slowed it.
constexpr int64_t kZeroSideMin = int64_t(1) << 26;   // zero-filled values

bool fork_zero_rows(spmm::Handle& H, float* Y, int64_t ldy, int k, hipStream_t s) {
    if (!H.d_row_old || H.n_tiled_rows >= H.n_rows) return false;
    const int64_t nz = H.n_rows - H.n_tiled_rows;
    if (nz * k < kZeroSideMin) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    if (!H.zstream) {
        hipStream_t z = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
        if (hipStreamCreateWithFlags(&z, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            if (z) (void)hipStreamDestroy(z);
            return false;
        }
        H.zstream = z;
        H.ev_zfork = a;
        H.ev_zjoin = b;
    }
    if (hipEventRecord(H.ev_zfork, s) != hipSuccess || hipStreamWaitEvent(H.zstream, H.ev_zfork, 0) != hipSuccess)
        return false;
    if (spmm::launch_zero_rows(Y, ldy, k, H.d_row_old + H.n_tiled_rows, nz, H.zstream) != hipSuccess) return false;
    return hipEventRecord(H.ev_zjoin, H.zstream) == hipSuccess;
}

spmm_status_t join_zero_rows(spmm::Handle& H, hipStream_t s) {
    hipError_t e = hipStreamWaitEvent(s, H.ev_zjoin, 0);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "hipStreamWaitEvent (zero rows)");
}

spmm_status_t run_device(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt, const float* col_scale,
                         float* Y, int64_t ldy, hipStream_t s, bool x_in_handle_order) {
    if (H.format == SPMM_FORMAT_CSR && dt != SPMM_X_F32)
        return fail(SPMM_EUNSUPPORTED, "the CSR format takes FP32 X");
    spmm::RunArgs a{};
    const bool zside = fork_zero_rows(H, Y, ldy, k, s);
    spmm_status_t st = prepare_x(H, X, k, ldx, dt, s, x_in_handle_order, a);
    if (st != SPMM_OK) {
        if (zside) (void)join_zero_rows(H, s);
        return st;
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
    a.part = H.d_part;
    a.rmap = H.d_row_old;
    hipEvent_t* ev = nullptr;
    if (H.timing) {
        if (H.timing_used + 2 > H.timing_ev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t q = nullptr;
                if (hipEventCreate(&q) != hipSuccess) return fail(SPMM_EHIP, "hipEventCreate");
                H.timing_ev.push_back(q);
            }
        }
        ev = &H.timing_ev[H.timing_used];
        H.timing_used += 2;
        hipError_t re = hipEventRecord(ev[0], s);
        if (re != hipSuccess) return hip_fail(re, "hipEventRecord");
    }
    hipError_t e = H.format == SPMM_FORMAT_CSR
        ? spmm::launch_csr(H, static_cast<const float*>(a.X), a.ldx, k, Y, ldy, s)
        : spmm::launch_spmm(H, a);
    if (e != hipSuccess) {
        if (zside) (void)join_zero_rows(H, s);
        return hip_fail(e, "kernel launch");
    }
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return zside ? join_zero_rows(H, s) : zero_empty_rows(H, Y, ldy, k, s);
}

// spmm_run's work on a device-placed handle whose columns keep the given
// order (X is read in place), with its scratch given by the caller: part
// (split-row partial sums), count (their counters, zero on entry), colmax
// and fexp (64 entries each).  Allocates nothing.
spmm_status_t run_device_scratch(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt,
                                 const float* col_scale, float* Y, int64_t ldy, hipStream_t s, int64_t* part,
                                 uint32_t* count, uint32_t* colmax, int32_t* fexp) {
    hipError_t e = spmm::launch_prepare_x(X, dt, ldx, k, nullptr, H.n_cols, nullptr, ldx, H.max_row_l1, colmax,
                                          fexp, s);
    if (e != hipSuccess) return hip_fail(e, "X preparation launch");
    spmm::RunArgs a{};
    a.X = X;
    a.k = k;
    a.ldx = ldx;
    a.fexp = fexp;
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
    a.count = count;
    a.part = part;
    a.rmap = H.d_row_old;
    if ((e = spmm::launch_spmm(H, a)) != hipSuccess) return hip_fail(e, "kernel launch");
    return zero_empty_rows(H, Y, ldy, k, s);
}

// The SpMM launches alone, with fixed-point exponents already in fexp and X
// in the handle's column order (used to time buckets of tiles).
spmm_status_t launch_items_only(spmm::Handle& H, const void* X, int k, int64_t ldx, int dt,
                                const float* col_scale, float* Y, int64_t ldy, hipStream_t s,
                                const int32_t* fexp) {
    spmm::RunArgs a{};
    a.X = X;
    a.k = k;
    a.ldx = ldx;
    a.dtype = dt;
    a.col_scale = col_scale;
    a.Y = Y;
    a.ldy = ldy;
    a.stream = s;
    a.fexp = fexp;
    a.blob = static_cast<const uint8_t*>(H.d_blob);
    a.blob_bias = 0;
    a.items = H.d_items;
    a.n_items = (uint32_t)H.enc.items.size();
    a.combine = H.d_combine;
    a.n_combine = (uint32_t)H.enc.combine.size();
    a.count = H.d_count;
    a.part = H.d_part;
    a.rmap = H.d_row_old;
    hipError_t e = spmm::launch_spmm(H, a);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "kernel launch");
}

// Defaults and range checks of the build options.
spmm_status_t parse_opts(const spmm_build_opts* opts, spmm_build_opts& o) {
    o = spmm_build_opts{};
    if (opts) o = *opts;
    if (o.max_kc == 0) o.max_kc = 32;
    if (o.max_kc != 16 && o.max_kc != 32) return fail(SPMM_EINVAL, "max_kc must be 16 or 32");
    if (o.tile_rows == 0) o.tile_rows = spmm::kDefaultTileRows;
    if (o.tile_cols == 0) o.tile_cols = spmm::kDefaultTileCols;
    if (o.item_nnz == 0) o.item_nnz = spmm::kDefaultItemNnz;
    if (o.tile_rows > spmm::kMaxTileRows) return fail(SPMM_EINVAL, "tile_rows must be <= 4096");
    if (o.item_nnz > spmm::kMaxItemNnz) return fail(SPMM_EINVAL, "item_nnz must be <= 131072");
    if (!is_pow2(o.tile_cols) || o.tile_cols > 65536) return fail(SPMM_EINVAL, "tile_cols must be a power of two <= 65536");
    if (o.fixed_variant >= SPMM_NUM_VARIANTS) return fail(SPMM_EINVAL, "unknown variant");
    if (o.place != SPMM_PLACE_DEVICE && o.place != SPMM_PLACE_PINNED_HOST) return fail(SPMM_EINVAL, "unknown placement");
    if (o.transpose > 1) return fail(SPMM_EINVAL, "transpose must be 0 or 1");
    if (o.format != SPMM_FORMAT_TILES && o.format != SPMM_FORMAT_CSR) return fail(SPMM_EINVAL, "unknown format");
    if (o.format == SPMM_FORMAT_CSR && o.place != SPMM_PLACE_DEVICE)
        return fail(SPMM_EUNSUPPORTED, "the CSR format runs in HBM only");
    const uint32_t ring = o.ring_depth ? o.ring_depth : 3u;
    if (ring < 2 || ring > 16) return fail(SPMM_EINVAL, "ring_depth must be in 2..16");
    return SPMM_OK;
}

void init_handle(spmm::Handle& H, int64_t n_rows, int64_t n_cols, const spmm_build_opts& o) {
    H.n_rows = n_rows;
    H.n_cols = n_cols;
    H.format = o.format;
    H.h = o.tile_rows;
    H.w = o.tile_cols;
    H.item_nnz = o.item_nnz;
    H.threads = o.threads;
    H.place = o.place;
    H.max_kc = (int)o.max_kc;
    H.relabel = o.keep_order == 0;
    H.row_relabel = o.keep_order == 0 && o.keep_row_order == 0;
    H.stream_bytes = (uint64_t)(o.stream_kib ? o.stream_kib : 262144u) << 10;
    H.ring_depth = o.ring_depth ? o.ring_depth : 3u;
    H.stage_bytes = o.x_stage_kib > 0 ? (uint64_t)o.x_stage_kib << 10 : 0u;
}

// Device ring of streamed mode: ring_depth slots of the largest transfer
// group, with their ready/free events (created once per handle).
spmm_status_t ensure_ring(spmm::Handle& H) {
    if (!H.ring.empty()) return SPMM_OK;
    uint64_t slot = 16;
    for (const auto& g : H.groups) slot = std::max(slot, g.b1 - g.b0);
    for (uint32_t r = 0; r < H.ring_depth; ++r) {
        void* q = nullptr;
        if (hipMalloc(&q, slot) != hipSuccess) return fail(SPMM_ENOMEM, "hipMalloc(stream ring) failed");
        H.ring.push_back(q);
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            return fail(SPMM_EHIP, "hipEventCreate(stream ring) failed");
        }
        H.ev_ready.push_back(a);
        H.ev_free.push_back(b);
        H.ring_used.push_back(0);
    }
    return SPMM_OK;
}

// The HIP side of the streamed plans (stream_plan.h).  With ybase set, the
// kernels of a group write its rows into Y slot s (rows r0..r1 of the group
// at ybase + s * yslot floats, k per row) and copy_out moves them to the
// host matrix yhost (row stride ldh).
struct StreamOps {
    spmm::Handle& H;
    spmm::RunArgs& a;
    hipStream_t kstream, cstream;   // compute, copy
    hipStream_t ostream;            // output (Y to host)
    float* yhost;
    int64_t ldh;
    int k;
    spmm_status_t st;
    bool check(hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        st = hip_fail(e, what);
        return false;
    }
    bool wait_free(uint32_t s) { return check(hipStreamWaitEvent(cstream, H.ev_free[s], 0), "wait (slot free)"); }
    bool copy(uint64_t g, uint32_t s) {
        const auto& G = H.groups[g];
        return check(hipMemcpyAsync(H.ring[s], static_cast<uint8_t*>(H.h_blob) + G.b0, G.b1 - G.b0,
                                    hipMemcpyHostToDevice, cstream),
                     "hipMemcpyAsync(tile group)");
    }
    bool record_ready(uint32_t s) { return check(hipEventRecord(H.ev_ready[s], cstream), "record (slot ready)"); }
    bool wait_ready(uint32_t s) { return check(hipStreamWaitEvent(kstream, H.ev_ready[s], 0), "wait (slot ready)"); }
    float* yslot(uint32_t s) const {
        return reinterpret_cast<float*>(static_cast<uint8_t*>(H.d_yring) + (size_t)s * H.yslot_bytes);
    }
    bool launch(uint64_t g, uint32_t s) {
        const auto& G = H.groups[g];
        a.blob = static_cast<const uint8_t*>(H.ring[s]);
        a.blob_bias = G.b0;
        a.items = H.d_items + G.i0;
        a.n_items = (uint32_t)(G.i1 - G.i0);
        if (yhost) {
            // row r of the group lands at yslot(s) + (r - r0) * k: the
            // kernels index Y by tiled row, so hand them the slot's address
            // moved back by r0 rows
            a.Y = reinterpret_cast<float*>(reinterpret_cast<uintptr_t>(yslot(s)) - (uintptr_t)G.r0 * k * sizeof(float));
            a.ldy = k;
        }
        return check(spmm::launch_spmm(H, a), "kernel launch");
    }
    bool record_free(uint32_t s) { return check(hipEventRecord(H.ev_free[s], kstream), "record (slot free)"); }
    bool wait_y_free(uint32_t s) { return check(hipStreamWaitEvent(kstream, H.ev_y_free[s], 0), "wait (Y slot free)"); }
    bool record_y_ready(uint32_t s) { return check(hipEventRecord(H.ev_y_ready[s], kstream), "record (Y slot ready)"); }
    bool wait_y_ready(uint32_t s) { return check(hipStreamWaitEvent(ostream, H.ev_y_ready[s], 0), "wait (Y slot ready)"); }
    bool copy_out(uint64_t g, uint32_t s) {
        const auto& G = H.groups[g];
        const size_t rows = (size_t)(G.r1 - G.r0);
        if (!rows) return true;
        float* dst = yhost + (size_t)G.r0 * ldh;
        const hipError_t e = (ldh == k)
            ? hipMemcpyAsync(dst, yslot(s), rows * k * sizeof(float), hipMemcpyDeviceToHost, ostream)
            : hipMemcpy2DAsync(dst, (size_t)ldh * sizeof(float), yslot(s), (size_t)k * sizeof(float),
                               (size_t)k * sizeof(float), rows, hipMemcpyDeviceToHost, ostream);
        return check(e, "copy of finished Y rows");
    }
    bool record_y_free(uint32_t s) { return check(hipEventRecord(H.ev_y_free[s], ostream), "record (Y slot free)"); }
};

}  // namespace spmm_abi

using namespace spmm_abi;

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
        spmm_status_t st = parse_opts(opts, o);
        if (st != SPMM_OK) return st;
        // with transpose, tile the CSR of A^T instead (rows and columns swap)
        std::vector<int64_t> t_ptr;
        std::vector<int32_t> t_col;
        std::vector<float> t_val;
        if (o.transpose) {
            std::string terr;
            spmm_status_t ts = spmm::transpose_csr(n_rows, n_cols, row_ptr, col_idx, values, o.threads, t_ptr,
                                                   t_col, t_val, terr);
            if (ts != SPMM_OK) return fail(ts, terr);
            std::swap(n_rows, n_cols);
            row_ptr = t_ptr.data();
            col_idx = t_col.empty() ? nullptr : t_col.data();
            values = values ? t_val.data() : nullptr;
        }
        std::unique_ptr<spmm_handle_s> hs(new spmm_handle_s);
        spmm::Handle& H = hs->H;
        init_handle(H, n_rows, n_cols, o);
        std::string err;
        if (o.format == SPMM_FORMAT_CSR) {
            if (values) return fail(SPMM_EUNSUPPORTED, "the CSR format takes a binary matrix (values = NULL)");
            st = spmm::build_csr(H, row_ptr, col_idx, o.validate != 0, err);
            if (st != SPMM_OK) return fail(st, err);
            *out = hs.release();
            return SPMM_OK;
        }
        st = spmm::build_canonical(H, row_ptr, col_idx, values, o.validate != 0, err);
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

spmm_status_t spmm_build_begin(int64_t n_rows, int64_t n_cols, const spmm_build_opts* opts, spmm_handle_t* out) {
    try {
        if (!out) return fail(SPMM_EINVAL, "out is NULL");
        if (n_rows < 0 || n_cols < 0 || n_rows > INT32_MAX || n_cols > INT32_MAX)
            return fail(SPMM_EINVAL, "n_rows and n_cols must be in 0..2^31-1");
        spmm_build_opts o{};
        spmm_status_t st = parse_opts(opts, o);
        if (st != SPMM_OK) return st;
        if (o.transpose) return fail(SPMM_EUNSUPPORTED, "a slab-wise build cannot transpose; build A^T's rows instead");
        if (o.format != SPMM_FORMAT_TILES) return fail(SPMM_EUNSUPPORTED, "a slab-wise build makes the tile store");
        std::unique_ptr<spmm_handle_s> hs(new spmm_handle_s);
        spmm::Handle& H = hs->H;
        init_handle(H, n_rows, n_cols, o);
        // the column order would need every column's in-degree before the
        // first tile: a slab-wise build keeps the given column order
        H.relabel = false;
        H.building = true;
        H.validate_rows = o.validate != 0;
        H.fixed_variant = o.fixed_variant;
        spmm::build_init(H, false);
        H.has_val_known = false;
        *out = hs.release();
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_build_append_rows(spmm_handle_t h, int64_t row0, int64_t nrows, const int64_t* row_ptr_local,
                                     const int32_t* col_idx, const float* values) {
    try {
        if (!h || !row_ptr_local) return fail(SPMM_EINVAL, "NULL argument");
        spmm::Handle& H = h->H;
        if (!H.building) return fail(SPMM_ESTATE, "the handle is not being built (spmm_build_begin)");
        if (nrows < 0) return fail(SPMM_EINVAL, "nrows must be >= 0");
        if (row_ptr_local[nrows] > 0 && !col_idx) return fail(SPMM_EINVAL, "col_idx is NULL");
        if (!H.has_val_known) {
            H.has_val = values != nullptr;
            H.has_val_known = true;
        }
        std::string err;
        spmm_status_t st = spmm::build_append(H, row0, nrows, row_ptr_local, col_idx, values, H.validate_rows, err);
        return st == SPMM_OK ? st : fail(st, err);
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_build_end(spmm_handle_t h) {
    try {
        if (!h) return fail(SPMM_EINVAL, "handle is NULL");
        spmm::Handle& H = h->H;
        if (!H.building) return fail(SPMM_ESTATE, "the handle is not being built (spmm_build_begin)");
        if (H.next_row != H.n_rows)
            return fail(SPMM_ESTATE, "rows " + std::to_string(H.next_row) + ".." + std::to_string(H.n_rows) +
                                         " have not been appended");
        std::string err;
        spmm_status_t st = spmm::build_finish_rows(H, err);
        if (st != SPMM_OK) return fail(st, err);
        if ((st = spmm::flush_slabs(H, err)) != SPMM_OK) return fail(st, err);
        H.building = false;
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
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
        if ((st = prepare_device(H)) != SPMM_OK) return st;
        return run_device(H, X, k, ldx, dt, col_scale, Y, ldy, s, false);
    } catch (const std::exception& e) {
        return fail(SPMM_EINVAL, e.what());
    }
}

spmm_status_t spmm_stream_run(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                              const float* col_scale, float* Y, int64_t ldy, hipStream_t compute,
                              hipStream_t copy) {
    try {
        if (!h) return fail(SPMM_EINVAL, "handle is NULL");
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_PINNED_HOST)
            return fail(SPMM_ESTATE, "tiles are placed in HBM; build with place = SPMM_PLACE_PINNED_HOST");
        spmm_status_t st = check_run_args(H, X, k, ldx, dt, col_scale, Y, ldy);
        if (st != SPMM_OK) return st;
        if (H.n_rows == 0) return SPMM_OK;
        if ((st = prepare_device(H)) != SPMM_OK) return st;
        if ((st = ensure_ring(H)) != SPMM_OK) return st;
        spmm::RunArgs a{};
        if ((st = prepare_x(H, X, k, ldx, dt, compute, false, a)) != SPMM_OK) return st;
        a.dtype = dt;
        a.col_scale = col_scale;
        a.Y = Y;
        a.ldy = ldy;
        a.stream = compute;
        a.combine = H.d_combine;
        a.n_combine = (uint32_t)H.enc.combine.size();
        a.count = H.d_count;
        a.part = H.d_part;
        a.rmap = H.d_row_old;
        // The slot/event ordering of the ring (stream_plan.h): every copy
        // into a slot waits for the kernels that last read it, also across
        // calls, so consecutive calls need no host synchronisation.
        StreamOps ops{H, a, compute, copy, nullptr, nullptr, 0, 0, SPMM_OK};
        if (!spmm::run_stream_plan(H.groups.size(), (uint32_t)H.ring.size(), H.ring_used.data(), ops)) return ops.st;
        return zero_empty_rows(H, Y, ldy, k, compute);
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
    }
}

spmm_status_t spmm_stream_run_yhost(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                                    const float* col_scale, float* Y, int64_t ldy, hipStream_t compute,
                                    hipStream_t copy, hipStream_t out) {
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_PINNED_HOST)
            return fail(SPMM_ESTATE, "tiles are placed in HBM; build with place = SPMM_PLACE_PINNED_HOST");
        if (!H.row_old.empty() || H.n_tiled_rows != H.n_rows)
            return fail(SPMM_EUNSUPPORTED, "Y rows are streamed out by tile row: build with keep_row_order = 1");
        spmm_status_t st = check_run_args(H, X, k, ldx, dt, col_scale, Y, ldy);
        if (st != SPMM_OK) return st;
        if (H.n_rows == 0) return SPMM_OK;
        if ((st = prepare_device(H)) != SPMM_OK) return st;
        if ((st = ensure_ring(H)) != SPMM_OK) return st;
        // Y slots: the largest group's rows at this k (regrown if k grows,
        // after the copy-outs still reading the old slots)
        uint64_t rows_max = 1;
        for (const auto& g : H.groups) rows_max = std::max<uint64_t>(rows_max, g.r1 - g.r0);
        const uint64_t need = (rows_max * (uint64_t)k * sizeof(float) + 255) / 256 * 256;
        if (need > H.yslot_bytes || H.ev_y_ready.empty()) {
            for (size_t r = 0; r < H.y_used.size(); ++r) {
                if (!H.y_used[r]) continue;
                hipError_t e = hipEventSynchronize(H.ev_y_free[r]);
                if (e != hipSuccess) return hip_fail(e, "earlier Y copy-out");
            }
            if (H.d_yring) (void)hipFree(H.d_yring);
            H.d_yring = nullptr;
            H.yslot_bytes = 0;
            if (hipMalloc(&H.d_yring, need * H.ring.size()) != hipSuccess)
                return fail(SPMM_ENOMEM, "hipMalloc(Y slots) failed");
            H.yslot_bytes = need;
            H.y_used.assign(H.ring.size(), 0);
            while (H.ev_y_ready.size() < H.ring.size()) {
                hipEvent_t a = nullptr, b = nullptr;
                if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
                    hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
                    if (a) (void)hipEventDestroy(a);
                    return fail(SPMM_EHIP, "hipEventCreate(Y slots) failed");
                }
                H.ev_y_ready.push_back(a);
                H.ev_y_free.push_back(b);
            }
        }
        spmm::RunArgs a{};
        if ((st = prepare_x(H, X, k, ldx, dt, compute, false, a)) != SPMM_OK) return st;
        a.dtype = dt;
        a.col_scale = col_scale;
        a.stream = compute;
        a.combine = H.d_combine;
        a.n_combine = (uint32_t)H.enc.combine.size();
        a.count = H.d_count;
        a.part = H.d_part;
        a.rmap = nullptr;
        // the slot/event ordering of stream_plan.h, with the Y slots: a
        // group's kernels wait for the previous copy-out of their Y slot
        StreamOps ops{H, a, compute, copy, out, Y, ldy, k, SPMM_OK};
        if (!spmm::run_stream_plan_yout(H.groups.size(), (uint32_t)H.ring.size(), H.ring_used.data(),
                                        H.y_used.data(), ops))
            return ops.st;
        return SPMM_OK;
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
    }
}

spmm_status_t spmm_stream_run_host(spmm_handle_t h, const float* X, int k, int64_t ldx, float* Y, int64_t ldy,
                                   int cols_per_block, uint32_t flags) {
    try {
        if (!h) return fail(SPMM_EINVAL, "handle is NULL");
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_PINNED_HOST)
            return fail(SPMM_ESTATE, "tiles are placed in HBM; build with place = SPMM_PLACE_PINNED_HOST");
        if (k < 1 || k > 64) return fail(SPMM_EINVAL, "k must be in 1..64");
        if (cols_per_block < 1 || cols_per_block > k) return fail(SPMM_EINVAL, "cols_per_block must be in 1..k");
        if (flags & ~SPMM_HOSTXY_BLOCKED) return fail(SPMM_EINVAL, "unknown flags");
        const bool blocked = (flags & SPMM_HOSTXY_BLOCKED) != 0;
        if (!blocked && (ldx < k || ldy < k)) return fail(SPMM_EINVAL, "ldx and ldy must be >= k");
        if ((H.n_cols > 0 && !X) || (H.n_rows > 0 && !Y)) return fail(SPMM_EINVAL, "X or Y is NULL");
        if (H.n_rows == 0) return SPMM_OK;
        const int cb = cols_per_block;
        const size_t xrows = (size_t)std::max<int64_t>(H.n_cols, 1), yrows = (size_t)H.n_rows;
        DevBufs B;
        float* xb[2] = {B.get<float>(xrows * cb), B.get<float>(xrows * cb)};
        float* yb[2] = {B.get<float>(yrows * cb), B.get<float>(yrows * cb)};
        if (!xb[0] || !xb[1] || !yb[0] || !yb[1]) return fail(SPMM_ENOMEM, "hipMalloc(column blocks) failed");
        hipStream_t st[3] = {nullptr, nullptr, nullptr};  // compute, host -> device, device -> host
        hipEvent_t ev[7] = {};  // x ready, x free (2), y ready, y free (2), spare
        struct Guard {
            hipStream_t* st;
            hipEvent_t* ev;
            ~Guard() {
                for (int i = 0; i < 3; ++i)
                    if (st[i]) (void)hipStreamSynchronize(st[i]);
                for (int i = 0; i < 7; ++i)
                    if (ev[i]) (void)hipEventDestroy(ev[i]);
                for (int i = 0; i < 3; ++i)
                    if (st[i]) (void)hipStreamDestroy(st[i]);
            }
        } guard{st, ev};
        hipError_t e;
        for (int i = 0; i < 3; ++i)
            if ((e = hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
        for (int i = 0; i < 7; ++i)
            if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreate");
        hipEvent_t x_ready = ev[0], x_free[2] = {ev[1], ev[2]}, y_ready = ev[3], y_free[2] = {ev[4], ev[5]};
        const int nblk = (k + cb - 1) / cb;
        for (int b = 0; b < nblk; ++b) {
            const int c0 = b * cb, w = std::min(cb, k - c0), slot = b & 1;
            // X block b -> device, once the kernels of block b - 2 have read the slot
            if (b >= 2 && (e = hipStreamWaitEvent(st[1], x_free[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
            if (H.n_cols > 0) {
                // block b's X in host memory: contiguous (blocked layout, or a
                // full-width row-major X) or w columns of ldx-strided rows
                const float* xs = blocked ? X + (size_t)c0 * H.n_cols : X + c0;
                const bool contiguous = blocked || (size_t)w == (size_t)ldx;
                e = contiguous ? hipMemcpyAsync(xb[slot], xs, (size_t)w * 4 * H.n_cols, hipMemcpyHostToDevice, st[1])
                               : hipMemcpy2DAsync(xb[slot], (size_t)w * 4, xs, (size_t)ldx * 4, (size_t)w * 4,
                                                  (size_t)H.n_cols, hipMemcpyHostToDevice, st[1]);
                if (e != hipSuccess) return hip_fail(e, "copy of an X block");
            }
            if ((e = hipEventRecord(x_ready, st[1])) != hipSuccess || (e = hipStreamWaitEvent(st[0], x_ready, 0)) != hipSuccess)
                return hip_fail(e, "X block ordering");
            // the Y slot is free once block b - 2 has been copied back
            if (b >= 2 && (e = hipStreamWaitEvent(st[0], y_free[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
            spmm_status_t rs = spmm_stream_run(h, xb[slot], w, w, SPMM_X_F32, nullptr, yb[slot], w, st[0], st[1]);
            if (rs != SPMM_OK) return rs;
            if ((e = hipEventRecord(x_free[slot], st[0])) != hipSuccess || (e = hipEventRecord(y_ready, st[0])) != hipSuccess ||
                (e = hipStreamWaitEvent(st[2], y_ready, 0)) != hipSuccess)
                return hip_fail(e, "Y block ordering");
            {
                float* ys = blocked ? Y + (size_t)c0 * yrows : Y + c0;
                const bool contiguous = blocked || (size_t)w == (size_t)ldy;
                e = contiguous ? hipMemcpyAsync(ys, yb[slot], (size_t)w * 4 * yrows, hipMemcpyDeviceToHost, st[2])
                               : hipMemcpy2DAsync(ys, (size_t)ldy * 4, yb[slot], (size_t)w * 4, (size_t)w * 4, yrows,
                                                  hipMemcpyDeviceToHost, st[2]);
                if (e != hipSuccess) return hip_fail(e, "copy of a Y block");
            }
            if ((e = hipEventRecord(y_free[slot], st[2])) != hipSuccess) return hip_fail(e, "record");
        }
        for (int i = 0; i < 3; ++i)
            if ((e = hipStreamSynchronize(st[i])) != hipSuccess) return hip_fail(e, "column-block SpMM");
        return SPMM_OK;
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
    }
}

spmm_status_t spmm_pagerank(spmm_handle_t h, float damping, int iters, uint32_t flags, float* pr,
                            double* resid, hipStream_t s) {
    try {
        if (!h || !pr) return fail(SPMM_EINVAL, "NULL argument");
        spmm::Handle& H = h->H;
        if (H.n_rows != H.n_cols) return fail(SPMM_EINVAL, "PageRank needs a square matrix");
        if (iters < 0 || !(damping >= 0.0f && damping <= 1.0f)) return fail(SPMM_EINVAL, "bad damping or iters");
        if (flags & ~(SPMM_PR_INIT_GIVEN | SPMM_PR_NO_REDISTRIBUTE | SPMM_PR_NO_GRAPH))
            return fail(SPMM_EINVAL, "unknown flags");
        if (H.place != SPMM_PLACE_DEVICE) return fail(SPMM_ESTATE, "tiles are placed in host memory");
        const int64_t n = H.n_rows;
        if (n == 0) return SPMM_OK;
        spmm_status_t st = prepare_device(H);
        if (st != SPMM_OK) return st;
        hipError_t e;
        if (!H.d_col_count) {
            if (hipMalloc(&H.d_col_count, sizeof(uint32_t) * (size_t)n) != hipSuccess)
                return fail(SPMM_ENOMEM, "hipMalloc(out-degrees) failed");
            if ((e = hipMemcpy(H.d_col_count, H.col_count.data(), sizeof(uint32_t) * (size_t)n,
                               hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy(out-degrees)");
        }
        DevBufs B;
        float* xp = B.get<float>((size_t)n);
        float* y = B.get<float>((size_t)n);
        double* dpart = B.get<double>(1024);
        double* rpart = B.get<double>(1024);
        double* D = B.get<double>(1);
        double* dres = B.get<double>((size_t)std::max(iters, 1));
        if (!xp || !y || !dpart || !rpart || !D || !dres) return fail(SPMM_ENOMEM, "hipMalloc(PageRank workspace) failed");
        hipStream_t cs = nullptr;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
        hipEvent_t ev = nullptr;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return hip_fail(e, "hipEventCreate");
        }
        struct Cleanup {
            hipStream_t cs;
            hipEvent_t ev;
            ~Cleanup() {
                (void)hipStreamSynchronize(cs);
                (void)hipEventDestroy(ev);
                (void)hipStreamDestroy(cs);
            }
        } cleanup{cs, ev};
        // the internal stream starts after the caller's stream's prior work
        if ((e = hipEventRecord(ev, s)) != hipSuccess || (e = hipStreamWaitEvent(cs, ev, 0)) != hipSuccess)
            return hip_fail(e, "stream ordering");
        if (!(flags & SPMM_PR_INIT_GIVEN) &&
            (e = spmm::launch_pr_init(pr, n, (float)(1.0 / (double)n), cs)) != hipSuccess)
            return hip_fail(e, "PageRank init launch");
        const int redistribute = (flags & SPMM_PR_NO_REDISTRIBUTE) ? 0 : 1;
        // no timing events inside the captured iterations
        struct TimingOff {
            spmm::Handle& H;
            bool was;
            ~TimingOff() { H.timing = was; }
        } timing_off{H, H.timing};
        H.timing = false;
        const int32_t* perm = H.relabel ? H.d_col_old : nullptr;
        auto enqueue = [&]() -> spmm_status_t {
            for (int it = 0; it < iters; ++it) {
                hipError_t pe = spmm::launch_pr_prepare(pr, H.d_col_count, perm, n, xp, dpart, D, cs);
                if (pe != hipSuccess) return hip_fail(pe, "PageRank prepare launch");
                spmm_status_t rs = run_device(H, xp, 1, 1, SPMM_X_F32, nullptr, y, 1, cs, true);
                if (rs != SPMM_OK) return rs;
                pe = spmm::launch_pr_update(pr, y, n, (double)damping, D, redistribute, rpart, dres + it, cs);
                if (pe != hipSuccess) return hip_fail(pe, "PageRank update launch");
            }
            return SPMM_OK;
        };
        spmm_status_t rs = SPMM_OK;
        if (flags & SPMM_PR_NO_GRAPH) {
            rs = enqueue();
        } else {
            // all iterations as one HIP graph
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
                rs = hip_fail(e, "hipStreamBeginCapture");
            } else {
                rs = enqueue();
                hipError_t ce = hipStreamEndCapture(cs, &graph);
                if (rs == SPMM_OK && ce != hipSuccess) rs = hip_fail(ce, "hipStreamEndCapture");
                if (rs == SPMM_OK && (e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
                    rs = hip_fail(e, "hipGraphInstantiate");
                if (rs == SPMM_OK && (e = hipGraphLaunch(exec, cs)) != hipSuccess) rs = hip_fail(e, "hipGraphLaunch");
            }
            if (rs == SPMM_OK) (void)hipStreamSynchronize(cs);  // checked below
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
        }
        if (rs == SPMM_OK && resid && iters > 0)
            if ((e = hipMemcpyAsync(resid, dres, sizeof(double) * (size_t)iters, hipMemcpyDeviceToHost, cs)) != hipSuccess)
                rs = hip_fail(e, "hipMemcpy(residuals)");
        hipError_t se = hipStreamSynchronize(cs);
        if (rs == SPMM_OK && se != hipSuccess) rs = hip_fail(se, "PageRank execution");
        return rs;
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
    }
}

spmm_status_t spmm_nmf(spmm_handle_t hA, spmm_handle_t hAT, int rank, int iters, float eps, float* W, float* Hm,
                       hipStream_t s) {
    try {
        if (!hA || !hAT || !W || !Hm) return fail(SPMM_EINVAL, "NULL argument");
        spmm::Handle& A = hA->H;
        spmm::Handle& AT = hAT->H;
        if (rank < 1 || rank > 32) return fail(SPMM_EINVAL, "rank must be in 1..32");
        if (iters < 0 || !(eps >= 0.0f)) return fail(SPMM_EINVAL, "bad iters or eps");
        if (AT.n_rows != A.n_cols || AT.n_cols != A.n_rows)
            return fail(SPMM_EINVAL, "hAT must hold the transpose of hA (the same handle if A is symmetric)");
        if (A.place != SPMM_PLACE_DEVICE || AT.place != SPMM_PLACE_DEVICE)
            return fail(SPMM_ESTATE, "tiles are placed in host memory");
        const int64_t n = A.n_rows, m = A.n_cols;
        spmm_status_t st = prepare_device(A);
        if (st == SPMM_OK && hAT != hA) st = prepare_device(AT);
        if (st != SPMM_OK) return st;
        // workspace owned by hA and kept between calls, so that the call is
        // asynchronous: S (max(n, m) x rank), the Gram partials and G
        const size_t s_bytes = (((size_t)std::max(n, m) * rank * sizeof(float)) + 255) / 256 * 256;
        const size_t p_bytes = ((size_t)spmm::gram_blocks() * rank * rank * sizeof(double) + 255) / 256 * 256;
        const size_t need = s_bytes + p_bytes + (size_t)rank * rank * sizeof(float);
        if (need > A.nmf_ws_bytes) {
            if (A.d_nmf_ws) {
                // the previous workspace may still be in use by queued work
                hipError_t se = hipStreamSynchronize(s);
                if (se != hipSuccess) return hip_fail(se, "NMF workspace resize");
                (void)hipFree(A.d_nmf_ws);
                A.d_nmf_ws = nullptr;
                A.nmf_ws_bytes = 0;
            }
            if (hipMalloc(&A.d_nmf_ws, need) != hipSuccess) return fail(SPMM_ENOMEM, "hipMalloc(NMF workspace) failed");
            A.nmf_ws_bytes = need;
        }
        uint8_t* ws = static_cast<uint8_t*>(A.d_nmf_ws);
        float* S = reinterpret_cast<float*>(ws);
        double* part = reinterpret_cast<double*>(ws + s_bytes);
        float* G = reinterpret_cast<float*>(ws + s_bytes + p_bytes);
        hipError_t e;
        for (int it = 0; it < iters; ++it) {
            // H <- H * (A^T W) / (H (W^T W) + eps)
            if ((e = spmm::launch_gram(W, n, rank, part, G, s)) != hipSuccess) return hip_fail(e, "Gram launch");
            if ((st = run_device(AT, W, rank, rank, SPMM_X_F32, nullptr, S, rank, s, false)) != SPMM_OK) return st;
            if ((e = spmm::launch_mu_update(Hm, S, G, m, rank, eps, s)) != hipSuccess) return hip_fail(e, "update launch");
            // W <- W * (A H) / (W (H^T H) + eps)
            if ((e = spmm::launch_gram(Hm, m, rank, part, G, s)) != hipSuccess) return hip_fail(e, "Gram launch");
            if ((st = run_device(A, Hm, rank, rank, SPMM_X_F32, nullptr, S, rank, s, false)) != SPMM_OK) return st;
            if ((e = spmm::launch_mu_update(W, S, G, n, rank, eps, s)) != hipSuccess) return hip_fail(e, "update launch");
        }
        return SPMM_OK;
    } catch (const std::exception& ex) {
        return fail(SPMM_EINVAL, ex.what());
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

spmm_status_t spmm_read_probe(const void* buf, uint64_t bytes, float* sink, hipStream_t s) {
    if (!buf || !sink) return fail(SPMM_EINVAL, "NULL argument");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(buf) % 16)
        return fail(SPMM_EINVAL, "buf and bytes must be multiples of 16");
    hipError_t e = spmm::launch_read_probe(buf, bytes, sink, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "read probe launch");
}

spmm_status_t spmm_timing_begin(spmm_handle_t h) {
    if (spmm_status_t rs = check_ready(h)) return rs;
    if (!h) return fail(SPMM_EINVAL, "handle is NULL");
    h->H.timing = true;
    h->H.timing_used = 0;
    return SPMM_OK;
}

spmm_status_t spmm_timing_end(spmm_handle_t h, double* total_ms, uint64_t* n_runs) {
    if (!h || !total_ms) return fail(SPMM_EINVAL, "NULL argument");
    spmm::Handle& H = h->H;
    double sum = 0.0;
    for (size_t i = 0; i + 1 < H.timing_used; i += 2) {
        hipError_t e = hipEventSynchronize(H.timing_ev[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "timing");
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, H.timing_ev[i], H.timing_ev[i + 1])) != hipSuccess)
            return hip_fail(e, "hipEventElapsedTime");
        sum += ms;
    }
    *total_ms = sum;
    if (n_runs) *n_runs = H.timing_used / 2;
    H.timing = false;
    H.timing_used = 0;
    return SPMM_OK;
}

spmm_status_t spmm_get_stats(spmm_handle_t h, spmm_stats_t* out) {
    if (spmm_status_t rs = check_ready(h)) return rs;
    if (!h || !out) return fail(SPMM_EINVAL, "NULL argument");
    const spmm::Handle& H = h->H;
    spmm_stats_t s{};
    s.n_rows = (uint64_t)H.n_rows;
    s.n_cols = (uint64_t)H.n_cols;
    s.nnz = (uint64_t)H.nnz;
    s.tile_rows = H.h;
    s.tile_cols = H.w;
    s.n_slabs = H.n_slabs;
    s.n_tiles = H.n_tiles_total;
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
        if (spmm_status_t rs = check_ready(h)) return rs;
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
