// Per-tile variant selection: tile features, variant get/set, bucketed
// timing of every variant, the exhaustive autotuner, and the learned cost
// model (initialisation, gradient, Adam, training loop, selection).
//
// The paper fixes one tile layout (SCSR plus COO, Section 3.2); choosing a
// layout per tile by measurement or by a learned model is this library's
// extension, and every choice computes the same Y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "abi_internal.h"

using namespace spmm_abi;

namespace {

// SplitMix64 (Steele, Lea and Flood, 2014): a Weyl sequence with step
// 0x9E3779B97F4A7C15 finalised by the MurmurHash3-style mixer.
struct SplitMix64 {
    uint64_t state;
    uint64_t next() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // uniform in [0, 1) with 53 random bits
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
    // uniform in [0, n) by rejection (no modulo bias)
    uint64_t below(uint64_t n) {
        const uint64_t lim = UINT64_MAX - UINT64_MAX % n;
        uint64_t x;
        do x = next();
        while (x >= lim);
        return x % n;
    }
};

int xbytes_of(int dt) { return dt == SPMM_X_F32 ? 4 : dt == SPMM_X_BF16 ? 2 : 1; }

bool valid_dt(int dt) { return dt == SPMM_X_F32 || dt == SPMM_X_BF16 || dt == SPMM_X_FP8_E4M3; }

spmm_status_t reencode(spmm::Handle& H) {
    free_device(H);
    H.enc = spmm::Encoded();
    std::string err;
    spmm_status_t st = spmm::encode(H, err);
    return st == SPMM_OK ? st : fail(st, err);
}

// Variant selection works on the canonical tile store: a tile-format
// handle built in one pass.  A slab-wise build encodes each block as it is
// cut and keeps only the encoding.
spmm_status_t need_tiles(spmm_handle_t h) {
    if (h->H.format != SPMM_FORMAT_TILES) return fail(SPMM_EUNSUPPORTED, "variants are chosen per tile");
    if (!h->H.canonical)
        return fail(SPMM_EUNSUPPORTED,
                    "a slab-wise build keeps no per-tile store; choose the variant with fixed_variant");
    return SPMM_OK;
}

// Bucket of a feature cell: size class floor(f0) (0..15), skew class of f5
// (< 1, < 2, < 3, >= 3) and whether most non-empty rows hold one entry.
uint32_t feature_cell(const float* f) {
    const uint32_t b0 = (uint32_t)std::min(15.0f, std::max(0.0f, std::floor(f[0])));
    const uint32_t b1 = f[5] < 1.0f ? 0u : f[5] < 2.0f ? 1u : f[5] < 3.0f ? 2u : 3u;
    const uint32_t b2 = f[4] >= 0.5f ? 1u : 0u;
    return (b0 * 4u + b1) * 2u + b2;  // < 128 = SPMM_MAX_BUCKETS
}

// Consecutive non-empty cells merge until a bucket holds min_tiles tiles; a
// short last bucket joins the one before it.
uint32_t make_buckets(const std::vector<float>& feat, uint64_t T, uint32_t min_tiles,
                      std::vector<uint32_t>& bucket) {
    std::vector<uint32_t> cell(T);
    std::vector<uint64_t> count(SPMM_MAX_BUCKETS, 0);
    for (uint64_t t = 0; t < T; ++t) {
        cell[t] = feature_cell(&feat[t * SPMM_NUM_FEATURES]);
        count[cell[t]]++;
    }
    std::vector<uint32_t> map(SPMM_MAX_BUCKETS, 0);
    std::vector<uint64_t> size;
    uint64_t cur = 0;
    bool open = false;
    for (uint32_t c = 0; c < SPMM_MAX_BUCKETS; ++c) {
        if (!count[c]) continue;
        if (!open) {
            size.push_back(0);
            open = true;
        }
        map[c] = (uint32_t)size.size() - 1;
        size.back() += count[c];
        cur = size.back();
        if (cur >= min_tiles) open = false;
    }
    if (size.size() > 1 && size.back() < min_tiles) {
        const uint32_t last = (uint32_t)size.size() - 1;
        for (uint32_t c = 0; c < SPMM_MAX_BUCKETS; ++c)
            if (count[c] && map[c] == last) map[c] = last - 1;
        size.pop_back();
    }
    bucket.resize(T);
    for (uint64_t t = 0; t < T; ++t) bucket[t] = map[cell[t]];
    return (uint32_t)size.size();
}

// A handle holding only the listed tiles of H (in H's order), their tile
// rows renumbered consecutively so that the sub-matrix has no empty slabs;
// the whole list is repeated `copies` times as further tile rows.
void make_subset(const spmm::Handle& H, const std::vector<uint64_t>& sel, spmm::Handle& S, uint32_t copies) {
    S.n_cols = H.n_cols;
    S.h = H.h;
    S.w = H.w;
    S.wshift = H.wshift;
    S.item_nnz = H.item_nnz;
    S.threads = H.threads;
    S.place = SPMM_PLACE_DEVICE;
    S.has_val = H.has_val;
    S.n_strips = H.n_strips;
    S.max_row_l1 = H.max_row_l1;
    S.max_kc = H.max_kc;
    S.stage_bytes = H.stage_bytes;
    S.relabel = false;
    uint64_t nnz1 = 0;
    for (uint64_t t : sel) nnz1 += H.tiles[t].nnz;
    const uint64_t nnz = nnz1 * copies;
    S.ent.resize(nnz);
    if (H.has_val) S.val.resize(nnz);
    S.tiles.resize(sel.size() * copies);
    S.slab_tiles.clear();
    S.slab_tiles.push_back(0);
    uint64_t pos = 0, i = 0;
    for (uint32_t c = 0; c < copies; ++c) {
        uint32_t prev_slab = UINT32_MAX;
        for (size_t j = 0; j < sel.size(); ++j, ++i) {
            const spmm::Tile& src = H.tiles[sel[j]];
            if (src.slab != prev_slab) {
                if (i) S.slab_tiles.push_back(i);
                prev_slab = src.slab;
            }
            spmm::Tile d = src;
            d.slab = (uint32_t)(S.slab_tiles.size() - 1);
            d.ent_begin = pos;
            std::memcpy(&S.ent[pos], &H.ent[src.ent_begin], sizeof(uint32_t) * src.nnz);
            if (H.has_val) std::memcpy(&S.val[pos], &H.val[src.ent_begin], sizeof(float) * src.nnz);
            pos += src.nnz;
            S.tiles[i] = d;
        }
    }
    S.slab_tiles.push_back(S.tiles.size());
    S.n_slabs = S.slab_tiles.size() - 1;
    S.n_rows = (int64_t)S.n_slabs * H.h;
    S.n_tiled_rows = S.n_rows;
    S.nnz = (int64_t)nnz;
}

// A bucket is timed with at least this many work items (wavefronts) in
// flight, repeating its tiles if needed: a handful of items would leave the
// GPU nearly idle and time each variant's latency rather than its cost
// inside a full SpMM.  The repetition stops at kFillMaxNnz entries.
constexpr uint64_t kFillItems = 2048;
constexpr uint64_t kFillMaxNnz = uint64_t(1) << 22;

// Median of the per-launch times of reps launches of the sub-handle.
spmm_status_t time_launches(spmm::Handle& S, const void* X, int k, int dt, const float* cs, float* Y,
                            const int32_t* fexp, uint32_t reps, hipStream_t s, float& ms) {
    spmm_status_t st = prepare_device(S);
    if (st != SPMM_OK) return st;
    std::vector<hipEvent_t> ev(reps + 1, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(SPMM_EHIP, "hipEventCreate");
    struct Guard {
        std::vector<hipEvent_t>& v;
        ~Guard() {
            for (auto e : v)
                if (e) (void)hipEventDestroy(e);
        }
    } guard{ev};
    if ((st = launch_items_only(S, X, k, k, dt, cs, Y, k, s, fexp)) != SPMM_OK) return st;  // warm-up
    hipError_t e = hipEventRecord(ev[0], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (uint32_t r = 0; r < reps; ++r) {
        if ((st = launch_items_only(S, X, k, k, dt, cs, Y, k, s, fexp)) != SPMM_OK) return st;
        if ((e = hipEventRecord(ev[r + 1], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if ((e = hipEventSynchronize(ev[reps])) != hipSuccess) return hip_fail(e, "bucket timing");
    std::vector<float> t(reps);
    for (uint32_t r = 0; r < reps; ++r)
        if ((e = hipEventElapsedTime(&t[r], ev[r], ev[r + 1])) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    ms = t[reps / 2];
    return SPMM_OK;
}

spmm_status_t collect(spmm::Handle& H, int k, int dt, const spmm_tune_opts* opts, std::vector<uint32_t>& bucket,
                      uint32_t& nb, std::vector<float>& ns, hipStream_t s) {
    const uint32_t min_tiles = opts && opts->min_tiles ? opts->min_tiles : 64u;
    const uint32_t reps = opts && opts->reps ? opts->reps : 5u;
    const uint64_t T = H.tiles.size();
    std::vector<float> feat(T * SPMM_NUM_FEATURES);
    spmm::tile_features(H, k, xbytes_of(dt), feat.data());
    nb = T ? make_buckets(feat, T, min_tiles, bucket) : 0;
    ns.assign((size_t)SPMM_MAX_BUCKETS * SPMM_NUM_VARIANTS, 0.0f);
    if (!nb) return SPMM_OK;
    std::vector<std::vector<uint64_t>> members(nb);
    for (uint64_t t = 0; t < T; ++t) members[bucket[t]].push_back(t);
    DevBufs B;
    B.sync_on(s);
    const size_t esz = (size_t)xbytes_of(dt);
    void* X = B.get<uint8_t>((size_t)std::max<int64_t>(H.n_cols, 1) * k * esz);
    int32_t* fexp = B.get<int32_t>(64);
    float* cs = B.get<float>(64);
    if (!X || !fexp || !cs) return fail(SPMM_ENOMEM, "hipMalloc(timing buffers) failed");
    hipError_t e;
    // X = 0 (every encoding's zero) with exponent 0: the kernels take the
    // same path as for any finite X, and FP8 scales of 1 keep Y finite.
    const std::vector<float> ones(64, 1.0f);
    if ((e = hipMemsetAsync(X, 0, (size_t)std::max<int64_t>(H.n_cols, 1) * k * esz, s)) != hipSuccess ||
        (e = hipMemsetAsync(fexp, 0, 64 * sizeof(int32_t), s)) != hipSuccess ||
        (e = hipMemcpyAsync(cs, ones.data(), 64 * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "timing buffer set-up");
    for (uint32_t b = 0; b < nb; ++b) {
        // copies of the bucket's tiles so that a launch has kFillItems items
        uint32_t copies = 1;
        {
            spmm::Handle S1;
            make_subset(H, members[b], S1, 1);
            S1.variant.assign(S1.tiles.size(), (uint8_t)SPMM_VAR_HYBRID);
            spmm_status_t st = reencode(S1);
            if (st != SPMM_OK) return st;
            const uint64_t items = std::max<uint64_t>(S1.enc.items.size(), 1);
            const uint64_t by_items = (kFillItems + items - 1) / items;
            const uint64_t by_nnz = std::max<uint64_t>(1, kFillMaxNnz / std::max<uint64_t>(S1.nnz, 1));
            copies = (uint32_t)std::max<uint64_t>(1, std::min(by_items, by_nnz));
        }
        spmm::Handle S;
        make_subset(H, members[b], S, copies);
        DevBufs BY;
        BY.sync_on(s);
        float* Y = BY.get<float>((size_t)S.n_rows * k);
        if (!Y) return fail(SPMM_ENOMEM, "hipMalloc(timing buffers) failed");
        for (int v = 0; v < SPMM_NUM_VARIANTS; ++v) {
            S.variant.assign(S.tiles.size(), (uint8_t)v);
            spmm_status_t st = reencode(S);
            float ms = 0.0f;
            if (st == SPMM_OK)
                st = time_launches(S, X, k, dt, dt == SPMM_X_FP8_E4M3 ? cs : nullptr, Y, fexp, reps, s, ms);
            free_device(S);
            if (st != SPMM_OK) return st;
            ns[(size_t)b * SPMM_NUM_VARIANTS + v] = ms * 1.0e6f / ((float)members[b].size() * (float)copies);
        }
    }
    return SPMM_OK;
}

}  // namespace

extern "C" {

spmm_status_t spmm_tile_features(spmm_handle_t h, int k, spmm_xdtype_t dt, float* feat) {
    if (spmm_status_t rs = check_ready(h)) return rs;
    if (spmm_status_t rs = need_tiles(h)) return rs;
    if (!h || (!feat && !h->H.tiles.empty())) return fail(SPMM_EINVAL, "NULL argument");
    if (k < 1 || k > 64 || !valid_dt(dt)) return fail(SPMM_EINVAL, "need 1 <= k <= 64 and a known dt");
    spmm::tile_features(h->H, k, xbytes_of(dt), feat);
    return SPMM_OK;
}

spmm_status_t spmm_get_variants(spmm_handle_t h, uint8_t* variant) {
    if (spmm_status_t rs = check_ready(h)) return rs;
    if (spmm_status_t rs = need_tiles(h)) return rs;
    if (!h || (!variant && !h->H.tiles.empty())) return fail(SPMM_EINVAL, "NULL argument");
    if (!h->H.variant.empty()) std::memcpy(variant, h->H.variant.data(), h->H.variant.size());
    return SPMM_OK;
}

spmm_status_t spmm_set_variants(spmm_handle_t h, const uint8_t* variant) {
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        if (spmm_status_t rs = need_tiles(h)) return rs;
        if (!variant && !h->H.tiles.empty()) return fail(SPMM_EINVAL, "NULL argument");
        spmm::Handle& H = h->H;
        for (size_t t = 0; t < H.tiles.size(); ++t)
            if (variant[t] >= SPMM_NUM_VARIANTS) return fail(SPMM_EINVAL, "variant out of range");
        if (!H.variant.empty()) std::memcpy(H.variant.data(), variant, H.variant.size());
        return reencode(H);
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_selector_collect(spmm_handle_t h, int k, spmm_xdtype_t dt, const spmm_tune_opts* opts,
                                    uint32_t* bucket, uint32_t* n_buckets, float* ns, hipStream_t s) {
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        if (spmm_status_t rs = need_tiles(h)) return rs;
        if (!n_buckets || !ns || (!bucket && !h->H.tiles.empty())) return fail(SPMM_EINVAL, "NULL argument");
        if (k < 1 || k > 64 || !valid_dt(dt)) return fail(SPMM_EINVAL, "need 1 <= k <= 64 and a known dt");
        if (h->H.place != SPMM_PLACE_DEVICE) return fail(SPMM_ESTATE, "bucket timing needs device placement");
        std::vector<uint32_t> b;
        std::vector<float> t;
        uint32_t nb = 0;
        spmm_status_t st = collect(h->H, k, dt, opts, b, nb, t, s);
        if (st != SPMM_OK) return st;
        if (!b.empty()) std::memcpy(bucket, b.data(), b.size() * sizeof(uint32_t));
        std::memcpy(ns, t.data(), t.size() * sizeof(float));
        *n_buckets = nb;
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_autotune(spmm_handle_t h, int k, spmm_xdtype_t dt, const spmm_tune_opts* opts,
                            uint32_t* n_buckets, float* ns, hipStream_t s) {
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        if (spmm_status_t rs = need_tiles(h)) return rs;
        if (k < 1 || k > 64 || !valid_dt(dt)) return fail(SPMM_EINVAL, "need 1 <= k <= 64 and a known dt");
        spmm::Handle& H = h->H;
        if (H.place != SPMM_PLACE_DEVICE) return fail(SPMM_ESTATE, "bucket timing needs device placement");
        std::vector<uint32_t> b;
        std::vector<float> t;
        uint32_t nb = 0;
        spmm_status_t st = collect(H, k, dt, opts, b, nb, t, s);
        if (st != SPMM_OK) return st;
        std::vector<uint8_t> best(std::max<uint32_t>(nb, 1), (uint8_t)SPMM_VAR_HYBRID);
        for (uint32_t q = 0; q < nb; ++q) {
            int v0 = 0;
            for (int v = 1; v < SPMM_NUM_VARIANTS; ++v)
                if (t[(size_t)q * SPMM_NUM_VARIANTS + v] < t[(size_t)q * SPMM_NUM_VARIANTS + v0]) v0 = v;
            best[q] = (uint8_t)v0;
        }
        for (size_t i = 0; i < H.variant.size(); ++i) H.variant[i] = best[b[i]];
        if ((st = reencode(H)) != SPMM_OK) return st;
        if (n_buckets) *n_buckets = nb;
        if (ns) std::memcpy(ns, t.data(), t.size() * sizeof(float));
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_mlp_init(uint64_t seed, float* params) {
    if (!params) return fail(SPMM_EINVAL, "NULL argument");
    SplitMix64 g{seed};
    std::fill(params, params + SPMM_MLP_PARAMS, 0.0f);
    const struct {
        int off, fan_in, fan_out;
    } layers[3] = {{SPMM_MLP_OFF_W1, SPMM_NUM_FEATURES, SPMM_MLP_HIDDEN},
                   {SPMM_MLP_OFF_W2, SPMM_MLP_HIDDEN, SPMM_MLP_HIDDEN},
                   {SPMM_MLP_OFF_W3, SPMM_MLP_HIDDEN, SPMM_NUM_VARIANTS}};
    for (const auto& L : layers) {
        const double lim = std::sqrt(6.0 / (double)L.fan_in);
        for (int i = 0; i < L.fan_in * L.fan_out; ++i) params[L.off + i] = (float)((2.0 * g.uniform() - 1.0) * lim);
    }
    return SPMM_OK;
}

spmm_status_t spmm_mlp_predict(const float* params, const float* feat, int64_t n, float* out, uint8_t* choice,
                               hipStream_t s) {
    if (n < 0) return fail(SPMM_EINVAL, "n must be >= 0");
    if (n > 0 && (!params || !feat)) return fail(SPMM_EINVAL, "NULL argument");
    hipError_t e = spmm::launch_mlp_predict(params, feat, n, out, choice, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "MLP inference launch");
}

spmm_status_t spmm_mlp_grad(const float* params, const float* feat, const float* target, const uint8_t* mask,
                            int64_t n, float* grad, double* loss, hipStream_t s) {
    if (n < 0) return fail(SPMM_EINVAL, "n must be >= 0");
    if (!params || !grad || (n > 0 && (!feat || !target))) return fail(SPMM_EINVAL, "NULL argument");
    DevBufs B;
    B.sync_on(s);
    const size_t r = (size_t)std::max<int64_t>(n, 1);
    spmm::MlpScratch w{};
    w.x = B.get<float>(r * SPMM_NUM_FEATURES);
    w.a1 = B.get<float>(r * SPMM_MLP_HIDDEN);
    w.a2 = B.get<float>(r * SPMM_MLP_HIDDEN);
    w.d1 = B.get<float>(r * SPMM_MLP_HIDDEN);
    w.d2 = B.get<float>(r * SPMM_MLP_HIDDEN);
    w.d3 = B.get<float>(r * SPMM_NUM_VARIANTS);
    w.loss_rows = B.get<double>(r);
    w.count = B.get<uint32_t>(1);
    if (!w.x || !w.a1 || !w.a2 || !w.d1 || !w.d2 || !w.d3 || !w.loss_rows || !w.count)
        return fail(SPMM_ENOMEM, "hipMalloc(MLP workspace) failed");
    hipError_t e = spmm::launch_mlp_grad(params, feat, target, mask, nullptr, n, w, grad, loss, s);
    if (e != hipSuccess) return hip_fail(e, "MLP gradient launch");
    // the workspace is freed on return
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "MLP gradient");
    return SPMM_OK;
}

spmm_status_t spmm_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t t, float lr,
                            float beta1, float beta2, float eps, hipStream_t s) {
    if (!params || !m || !v || !grad) return fail(SPMM_EINVAL, "NULL argument");
    if (t < 1) return fail(SPMM_EINVAL, "t must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f)) return fail(SPMM_EINVAL, "bad betas");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t)));
    hipError_t e = spmm::launch_adam(params, m, v, grad, SPMM_MLP_PARAMS, lr, beta1, beta2, eps, c1, c2, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "Adam launch");
}

spmm_status_t spmm_selector_train(const float* feat, const float* target, const uint8_t* mask, int64_t n,
                                  const spmm_train_opts* opts, float* params, double* loss_trace) {
    try {
        if (n < 1) return fail(SPMM_EINVAL, "need at least one row");
        if (!feat || !target || !params) return fail(SPMM_EINVAL, "NULL argument");
        if (n > INT32_MAX) return fail(SPMM_EINVAL, "at most 2^31-1 rows");
        const uint32_t epochs = opts && opts->epochs ? opts->epochs : 30u;
        const uint32_t batch = opts && opts->batch ? opts->batch : 1024u;
        const float lr = opts && opts->lr > 0.0f ? opts->lr : 1.0e-3f;
        const uint64_t seed = opts ? opts->seed : 0;
        const int64_t nbat = (n + batch - 1) / batch;
        const size_t V = SPMM_NUM_VARIANTS, F = SPMM_NUM_FEATURES, Hd = SPMM_MLP_HIDDEN;
        DevBufs B;
        float* dfeat = B.get<float>((size_t)n * F);
        float* dtgt = B.get<float>((size_t)n * V);
        uint8_t* dmask = mask ? B.get<uint8_t>((size_t)n * V) : nullptr;
        float* dp = B.get<float>(SPMM_MLP_PARAMS);
        float* dm = B.get<float>(SPMM_MLP_PARAMS);
        float* dv = B.get<float>(SPMM_MLP_PARAMS);
        float* dg = B.get<float>(SPMM_MLP_PARAMS);
        int32_t* didx = B.get<int32_t>((size_t)n);
        double* dloss = B.get<double>((size_t)nbat);
        spmm::MlpScratch w{};
        w.x = B.get<float>((size_t)batch * F);
        w.a1 = B.get<float>((size_t)batch * Hd);
        w.a2 = B.get<float>((size_t)batch * Hd);
        w.d1 = B.get<float>((size_t)batch * Hd);
        w.d2 = B.get<float>((size_t)batch * Hd);
        w.d3 = B.get<float>((size_t)batch * V);
        w.loss_rows = B.get<double>(batch);
        w.count = B.get<uint32_t>(1);
        if (!dfeat || !dtgt || (mask && !dmask) || !dp || !dm || !dv || !dg || !didx || !dloss || !w.x || !w.a1 ||
            !w.a2 || !w.d1 || !w.d2 || !w.d3 || !w.loss_rows || !w.count)
            return fail(SPMM_ENOMEM, "hipMalloc(training workspace) failed");
        hipStream_t s = nullptr;
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
        struct StreamGuard {
            hipStream_t s;
            ~StreamGuard() {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
        } sg{s};
        if ((e = hipMemcpyAsync(dfeat, feat, (size_t)n * F * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(dtgt, target, (size_t)n * V * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (mask && (e = hipMemcpyAsync(dmask, mask, (size_t)n * V, hipMemcpyHostToDevice, s)) != hipSuccess) ||
            (e = hipMemcpyAsync(dp, params, SPMM_MLP_PARAMS * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemsetAsync(dm, 0, SPMM_MLP_PARAMS * 4, s)) != hipSuccess ||
            (e = hipMemsetAsync(dv, 0, SPMM_MLP_PARAMS * 4, s)) != hipSuccess)
            return hip_fail(e, "training upload");
        SplitMix64 g{seed};
        std::vector<int32_t> perm((size_t)n);
        std::vector<double> lb((size_t)nbat);
        int64_t step = 0;
        for (uint32_t ep = 0; ep < epochs; ++ep) {
            std::iota(perm.begin(), perm.end(), 0);
            for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[g.below((uint64_t)i + 1)]);
            // the previous epoch's kernels still read didx: wait before reuse
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "training");
            if ((e = hipMemcpyAsync(didx, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpy(permutation)");
            for (int64_t q = 0; q < nbat; ++q) {
                const int64_t r0 = q * batch, nb = std::min<int64_t>(batch, n - r0);
                if ((e = spmm::launch_mlp_grad(dp, dfeat, dtgt, dmask, didx + r0, nb, w, dg, dloss + q, s)) !=
                    hipSuccess)
                    return hip_fail(e, "MLP gradient launch");
                spmm_status_t st = spmm_mlp_adam(dp, dm, dv, dg, ++step, lr, 0.9f, 0.999f, 1.0e-8f, s);
                if (st != SPMM_OK) return st;
            }
            if (loss_trace) {
                if ((e = hipMemcpyAsync(lb.data(), dloss, (size_t)nbat * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                    (e = hipStreamSynchronize(s)) != hipSuccess)
                    return hip_fail(e, "hipMemcpy(loss)");
                double sum = 0.0;
                for (double x : lb) sum += x;
                loss_trace[ep] = sum / (double)nbat;
            }
        }
        if ((e = hipMemcpyAsync(params, dp, SPMM_MLP_PARAMS * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(trained weights)");
        return SPMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

spmm_status_t spmm_select_learned(spmm_handle_t h, const float* params, int k, spmm_xdtype_t dt) {
    try {
        if (spmm_status_t rs = check_ready(h)) return rs;
        if (spmm_status_t rs = need_tiles(h)) return rs;
        if (!params) return fail(SPMM_EINVAL, "NULL argument");
        if (k < 1 || k > 64 || !valid_dt(dt)) return fail(SPMM_EINVAL, "need 1 <= k <= 64 and a known dt");
        spmm::Handle& H = h->H;
        const uint64_t T = H.tiles.size();
        if (T == 0) return SPMM_OK;
        std::vector<float> feat(T * SPMM_NUM_FEATURES);
        spmm::tile_features(H, k, xbytes_of(dt), feat.data());
        DevBufs B;
        float* dp = B.get<float>(SPMM_MLP_PARAMS);
        float* df = B.get<float>(feat.size());
        uint8_t* dc = B.get<uint8_t>(T);
        if (!dp || !df || !dc) return fail(SPMM_ENOMEM, "hipMalloc(selection workspace) failed");
        hipError_t e;
        if ((e = hipMemcpy(dp, params, SPMM_MLP_PARAMS * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(df, feat.data(), feat.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "selection upload");
        if ((e = spmm::launch_mlp_predict(dp, df, (int64_t)T, nullptr, dc, nullptr)) != hipSuccess)
            return hip_fail(e, "MLP inference launch");
        std::vector<uint8_t> choice(T);
        if ((e = hipMemcpy(choice.data(), dc, T, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, "hipMemcpy(choices)");
        std::memcpy(H.variant.data(), choice.data(), T);
        return reencode(H);
    } catch (const std::bad_alloc&) {
        return fail(SPMM_ENOMEM, "out of host memory");
    }
}

}  // extern "C"
