// Host-side tile builder: CSR -> canonical tile store -> encoded work items.
//
// The canonical store follows the paper's sparse format (Section 3.2): the
// matrix is cut into h x w tiles, tiles of one tile row ("slab") are kept in
// column order, and every entry is a 16-bit local row and a 16-bit local
// column inside its tile.  Conversion is one linear pass over the CSR
// (Section 5, Table 3).  The encoder then turns each slab into work items
// for the GPU, routing every row of every tile to the lane mapping its tile
// variant asks for (COO pairs, one lane per row, or one wavefront per row).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "spmm_internal.h"

namespace spmm {

void parallel_for(uint64_t n, uint32_t threads, uint64_t grain,
                  const std::function<void(uint64_t, uint64_t)>& fn) {
    if (n == 0) return;
    uint32_t T = threads ? threads : std::max(1u, std::thread::hardware_concurrency());
    grain = std::max<uint64_t>(grain, 1);
    if (T <= 1 || n <= grain) {
        fn(0, n);
        return;
    }
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> pool;
    auto work = [&]() {
        for (;;) {
            uint64_t b = next.fetch_add(grain);
            if (b >= n) break;
            fn(b, std::min(n, b + grain));
        }
    };
    for (uint32_t t = 1; t < T; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
}

static uint32_t log2_exact(uint32_t x) {
    uint32_t s = 0;
    while ((1u << s) < x) ++s;
    return s;
}

spmm_status_t transpose_csr(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr, const int32_t* col,
                            const float* val, uint32_t threads, std::vector<int64_t>& tp, std::vector<int32_t>& tc,
                            std::vector<float>& tv, std::string& err) {
    if (row_ptr[0] != 0) {
        err = "row_ptr[0] must be 0";
        return SPMM_EINVAL;
    }
    const int64_t nnz = row_ptr[n_rows];
    // the same range checks as the tile build, before any index is used
    std::atomic<int> bad{0};
    parallel_for((uint64_t)n_rows, threads, 1 << 16, [&](uint64_t a, uint64_t b) {
        for (uint64_t i = a; i < b && !bad; ++i) {
            if (row_ptr[i + 1] < row_ptr[i]) { bad = 1; return; }
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                if (col[p] < 0 || col[p] >= n_cols) { bad = 2; return; }
        }
    });
    if (bad) {
        err = bad == 1 ? "row_ptr is not non-decreasing" : "column index out of range";
        return SPMM_EINVAL;
    }
    tp.assign((size_t)n_cols + 1, 0);
    tc.resize((size_t)nnz);
    if (val) tv.resize((size_t)nnz);
    // counts per column, then positions by prefix sum
    parallel_for((uint64_t)n_rows, threads, 1 << 14, [&](uint64_t a, uint64_t b) {
        for (int64_t p = row_ptr[a]; p < row_ptr[b]; ++p) __atomic_fetch_add(&tp[(size_t)col[p] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int64_t c = 0; c < n_cols; ++c) tp[(size_t)c + 1] += tp[(size_t)c];
    std::vector<int64_t> cursor(tp.begin(), tp.end() - 1);
    parallel_for((uint64_t)n_rows, threads, 1 << 14, [&](uint64_t a, uint64_t b) {
        for (uint64_t i = a; i < b; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                const int64_t q = __atomic_fetch_add(&cursor[(size_t)col[p]], 1, __ATOMIC_RELAXED);
                tc[(size_t)q] = (int32_t)i;
                if (val) tv[(size_t)q] = val[p];
            }
    });
    // the scatter order depends on thread timing: sort every row of the
    // transpose (by source row, which is unique within it)
    parallel_for((uint64_t)n_cols, threads, 1 << 12, [&](uint64_t a, uint64_t b) {
        std::vector<std::pair<int32_t, float>> tmp;
        for (uint64_t c = a; c < b; ++c) {
            const int64_t lo = tp[c], hi = tp[c + 1];
            if (!val) {
                std::sort(tc.begin() + lo, tc.begin() + hi);
                continue;
            }
            tmp.resize((size_t)(hi - lo));
            for (int64_t q = lo; q < hi; ++q) tmp[(size_t)(q - lo)] = {tc[(size_t)q], tv[(size_t)q]};
            std::sort(tmp.begin(), tmp.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
            for (int64_t q = lo; q < hi; ++q) {
                tc[(size_t)q] = tmp[(size_t)(q - lo)].first;
                tv[(size_t)q] = tmp[(size_t)(q - lo)].second;
            }
        }
    });
    return SPMM_OK;
}

namespace {

// One row to tile: its original id and its entries.
struct RowRef {
    int64_t row;
    const int32_t* col;
    const float* val;
    uint64_t len;
};

// Append `rows` (in tile order) to H as new tile rows of h rows each; every
// tile row must be full except the last of the whole matrix.  Columns pass
// through H's column map.  The tile store grows by the rows' entries, tile
// major, sorted by (local row, local column) within each tile.
spmm_status_t tile_rows(Handle& H, const RowRef* rows, int64_t count, std::string& err) {
    if (count <= 0) return SPMM_OK;
    if (H.n_tiled_rows % H.h) {
        err = "internal: a partial tile row is not last";
        return SPMM_ESTATE;
    }
    const int32_t* cmap = H.relabel ? H.col_new.data() : nullptr;
    auto colmap = [cmap](int32_t c) -> uint32_t { return cmap ? (uint32_t)cmap[c] : (uint32_t)c; };
    const bool hv = H.has_val;
    const uint64_t s_first = H.n_slabs;
    const uint64_t ns = (uint64_t)((count + H.h - 1) / H.h);
    // entry offset of each new slab within the block
    std::vector<uint64_t> sbase(ns + 1, 0);
    for (uint64_t s = 0; s < ns; ++s) {
        uint64_t e = 0;
        const int64_t r0 = (int64_t)s * H.h, r1 = std::min<int64_t>(count, r0 + H.h);
        for (int64_t r = r0; r < r1; ++r) e += rows[r].len;
        sbase[s + 1] = sbase[s] + e;
    }
    const uint64_t ent0 = H.ent.size(), bnnz = sbase[ns];

    // Pass 1: non-empty tiles per new slab.
    std::vector<uint64_t> ntile(ns + 1, 0);
    const uint32_t nstrip = (uint32_t)H.n_strips;
    parallel_for(ns, H.threads, 64, [&](uint64_t a, uint64_t b) {
        std::vector<uint32_t> cnt(nstrip, 0);
        std::vector<uint32_t> used;
        for (uint64_t s = a; s < b; ++s) {
            const int64_t r0 = (int64_t)s * H.h, r1 = std::min<int64_t>(count, r0 + H.h);
            used.clear();
            for (int64_t r = r0; r < r1; ++r)
                for (uint64_t p = 0; p < rows[r].len; ++p) {
                    const uint32_t J = colmap(rows[r].col[p]) >> H.wshift;
                    if (cnt[J]++ == 0) used.push_back(J);
                }
            ntile[s + 1] = used.size();
            for (uint32_t J : used) cnt[J] = 0;
        }
    });
    const uint64_t t_first = H.tiles.size();
    if (H.slab_tiles.empty()) H.slab_tiles.push_back(0);
    for (uint64_t s = 0; s < ns; ++s) H.slab_tiles.push_back(H.slab_tiles.back() + ntile[s + 1]);
    const uint64_t T = H.slab_tiles.back();
    const uint64_t lbase = s_first - H.slab_base;   // local index of the first new slab
    try {
        // grow by at least a quarter, so that a build in many blocks does
        // not reallocate per block (and never doubles its peak footprint)
        auto grow = [](auto& v, size_t need) {
            if (need > v.capacity()) v.reserve(std::max(need, v.capacity() + v.capacity() / 4));
            v.resize(need);
        };
        H.tiles.resize(T);
        grow(H.ent, ent0 + bnnz);
        if (hv) grow(H.val, ent0 + bnnz);
        H.variant.resize(T, (uint8_t)(H.fixed_variant >= 0 ? H.fixed_variant : SPMM_VAR_HYBRID));
        if (H.row_relabel) {
            grow(H.row_old, (size_t)(H.n_tiled_rows + count));
            for (int64_t r = 0; r < count; ++r) H.row_old[(size_t)(H.n_tiled_rows + r)] = (int32_t)rows[r].row;
        }
    } catch (const std::bad_alloc&) {
        err = "out of host memory for the tile store";
        return SPMM_ENOMEM;
    }

    // Pass 2: scatter entries tile-major, then per-tile statistics.
    std::atomic<uint64_t> tot_nnr{0}, tot_nnc{0};
    parallel_for(ns, H.threads, 64, [&](uint64_t a, uint64_t b) {
        std::vector<uint32_t> cnt(nstrip, 0);
        std::vector<uint64_t> pos(nstrip, 0);
        std::vector<uint32_t> used;
        std::vector<uint64_t> seen((H.w + 63) / 64, 0);
        uint64_t my_nnr = 0, my_nnc = 0;
        for (uint64_t s = a; s < b; ++s) {
            const int64_t r0 = (int64_t)s * H.h, r1 = std::min<int64_t>(count, r0 + H.h);
            const uint64_t gs = s_first + s;
            used.clear();
            for (int64_t r = r0; r < r1; ++r)
                for (uint64_t p = 0; p < rows[r].len; ++p) {
                    const uint32_t J = colmap(rows[r].col[p]) >> H.wshift;
                    if (cnt[J]++ == 0) used.push_back(J);
                }
            std::sort(used.begin(), used.end());
            uint64_t e = ent0 + sbase[s];
            uint64_t t = H.slab_tiles[lbase + s];
            for (uint32_t J : used) {
                Tile& tl = H.tiles[t++];
                tl.ent_begin = e;
                tl.slab = (uint32_t)gs;
                tl.J = J;
                tl.nnz = cnt[J];
                pos[J] = e;
                e += cnt[J];
                cnt[J] = 0;
            }
            for (int64_t r = r0; r < r1; ++r) {
                const uint32_t rl = (uint32_t)(r - r0);
                for (uint64_t p = 0; p < rows[r].len; ++p) {
                    const uint32_t c = colmap(rows[r].col[p]);
                    const uint64_t q = pos[c >> H.wshift]++;
                    H.ent[q] = (rl << 16) | (c & (H.w - 1));
                    if (hv) H.val[q] = rows[r].val[p];
                }
            }
            if (cmap) {
                // relabelled columns arrive unordered within a row: sort each
                // tile's entries by (row, column), carrying the values along
                for (uint64_t ti = H.slab_tiles[lbase + s]; ti < H.slab_tiles[lbase + s + 1]; ++ti) {
                    const Tile& tl = H.tiles[ti];
                    uint32_t* E = H.ent.data() + tl.ent_begin;
                    if (!hv) {
                        std::sort(E, E + tl.nnz);
                    } else {
                        std::vector<std::pair<uint32_t, float>> tmp(tl.nnz);
                        for (uint32_t i = 0; i < tl.nnz; ++i) tmp[i] = {E[i], H.val[tl.ent_begin + i]};
                        std::sort(tmp.begin(), tmp.end(),
                                  [](const auto& x, const auto& y) { return x.first < y.first; });
                        for (uint32_t i = 0; i < tl.nnz; ++i) {
                            E[i] = tmp[i].first;
                            H.val[tl.ent_begin + i] = tmp[i].second;
                        }
                    }
                }
            }
            for (uint64_t ti = H.slab_tiles[lbase + s]; ti < H.slab_tiles[lbase + s + 1]; ++ti) {
                Tile& tl = H.tiles[ti];
                const uint32_t* E = H.ent.data() + tl.ent_begin;
                uint32_t nnr = 0, maxr = 0, single = 0, run = 0, nnc = 0;
                for (uint32_t i = 0; i < tl.nnz; ++i) {
                    if (i == 0 || (E[i] >> 16) != (E[i - 1] >> 16)) {
                        if (i) { maxr = std::max(maxr, run); single += run == 1; }
                        ++nnr;
                        run = 0;
                    }
                    ++run;
                    const uint32_t c = E[i] & 0xFFFFu;
                    const uint64_t bit = 1ull << (c & 63);
                    if (!(seen[c >> 6] & bit)) { seen[c >> 6] |= bit; ++nnc; }
                }
                maxr = std::max(maxr, run);
                single += run == 1;
                for (uint32_t i = 0; i < tl.nnz; ++i) seen[(E[i] & 0xFFFFu) >> 6] = 0;
                tl.nnr = nnr;
                tl.nnc = nnc;
                tl.max_row = maxr;
                tl.n_single = single;
                my_nnr += nnr;
                my_nnc += nnc;
            }
        }
        tot_nnr += my_nnr;
        tot_nnc += my_nnc;
    });
    H.n_tiles_total += T - t_first;
    H.sum_nnr += tot_nnr;
    H.sum_nnc += tot_nnc;
    H.n_slabs += ns;
    H.n_tiled_rows += count;
    return SPMM_OK;
}

// Checks and statistics of nr CSR rows (row_ptr relative to col/val):
// monotone row pointers, columns in range (sorted and unique when validate),
// finite values; the largest row L1 norm and the per-column entry counts of
// H are updated.
spmm_status_t scan_rows(Handle& H, int64_t nr, const int64_t* rp, const int32_t* col, const float* val,
                        bool validate, std::string& err) {
    std::atomic<int> bad{0};
    std::atomic<uint64_t> best{0};
    {
        double cur = H.max_row_l1;
        uint64_t bits;
        std::memcpy(&bits, &cur, 8);
        best = bits;
    }
    parallel_for((uint64_t)nr, H.threads, 1 << 14, [&](uint64_t a, uint64_t b) {
        double m = 0.0;
        for (uint64_t i = a; i < b; ++i) {
            if (rp[i + 1] < rp[i]) { bad = 1; return; }
            double r = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                if (col[p] < 0 || col[p] >= H.n_cols) { bad = 2; return; }
                if (validate && p > rp[i] && col[p] <= col[p - 1]) { bad = 3; return; }
                if (val) r += std::fabs((double)val[p]);
            }
            if (!val) r = (double)(rp[i + 1] - rp[i]);
            m = std::max(m, r);
        }
        if (!std::isfinite(m)) { bad = 4; return; }
        uint64_t bits;
        std::memcpy(&bits, &m, 8);
        uint64_t cur = best.load();
        while (bits > cur && !best.compare_exchange_weak(cur, bits)) {}
    });
    if (bad) {
        err = bad == 1 ? "row_ptr is not non-decreasing"
            : bad == 2 ? "column index out of range"
            : bad == 3 ? "columns not sorted and unique within a row"
                       : "values must be finite";
        return SPMM_EINVAL;
    }
    const uint64_t bits = best.load();
    std::memcpy(&H.max_row_l1, &bits, 8);
    std::vector<uint32_t>& cc = H.col_count;
    parallel_for((uint64_t)nr, H.threads, 1 << 14, [&](uint64_t a, uint64_t b) {
        for (int64_t p = rp[a]; p < rp[b]; ++p) __atomic_fetch_add(&cc[col[p]], 1u, __ATOMIC_RELAXED);
    });
    return SPMM_OK;
}

// Tile the pending rows of H plus the rows [row0, row0 + nr) given by
// (rp, col, val).  With row relabelling, rows without entries join the
// zero-filled list and the others are taken by descending out-degree (ties
// by row id); without it, rows keep their order.  Only whole tile rows are
// tiled unless `last`; the remainder stays pending (copied into H).
spmm_status_t tile_block(Handle& H, int64_t row0, int64_t nr, const int64_t* rp, const int32_t* col,
                         const float* val, bool last, std::string& err) {
    std::vector<RowRef> rows;
    rows.reserve(H.pend_row.size() + (size_t)nr);
    for (size_t i = 0; i < H.pend_row.size(); ++i)
        rows.push_back({H.pend_row[i], H.pend_col.data() + H.pend_off[i],
                        H.has_val ? H.pend_val.data() + H.pend_off[i] : nullptr, H.pend_off[i + 1] - H.pend_off[i]});
    for (int64_t i = 0; i < nr; ++i) {
        const uint64_t len = (uint64_t)(rp[i + 1] - rp[i]);
        if (H.row_relabel && len == 0) {
            H.zero_rows.push_back((int32_t)(row0 + i));
            continue;
        }
        rows.push_back({row0 + i, col + rp[i], val ? val + rp[i] : nullptr, len});
    }
    if (H.row_relabel && rows.size() > 1) {
        // counting sort by descending length, stable (pending rows precede
        // the block's and hold smaller ids, so ties stay in row-id order);
        // lengths >= cap share the first bucket, then are ordered exactly
        uint64_t maxl = 0;
        for (const RowRef& r : rows) maxl = std::max(maxl, r.len);
        const uint64_t cap = std::min<uint64_t>(maxl, 1u << 20);
        auto key = [cap](uint64_t len) { return cap - std::min(cap, len); };
        std::vector<uint64_t> start(cap + 2, 0);
        for (const RowRef& r : rows) start[key(r.len) + 1]++;
        for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
        const uint64_t nbig = start[1];
        std::vector<RowRef> sorted(rows.size());
        for (const RowRef& r : rows) sorted[start[key(r.len)]++] = r;
        std::stable_sort(sorted.begin(), sorted.begin() + (int64_t)nbig,
                         [](const RowRef& a, const RowRef& b) { return a.len > b.len; });
        rows.swap(sorted);
    }
    const int64_t now = last ? (int64_t)rows.size() : (int64_t)(rows.size() / H.h * H.h);
    spmm_status_t st = tile_rows(H, rows.data(), now, err);
    if (st != SPMM_OK) return st;
    // the remainder becomes the new pending set (copied before the old one
    // it may point into is released)
    std::vector<int64_t> prow;
    std::vector<uint64_t> poff(1, 0);
    std::vector<int32_t> pcol;
    std::vector<float> pval;
    for (size_t i = (size_t)now; i < rows.size(); ++i) {
        prow.push_back(rows[i].row);
        pcol.insert(pcol.end(), rows[i].col, rows[i].col + rows[i].len);
        if (H.has_val) pval.insert(pval.end(), rows[i].val, rows[i].val + rows[i].len);
        poff.push_back(pcol.size());
    }
    H.pend_row.swap(prow);
    H.pend_off.swap(poff);
    H.pend_col.swap(pcol);
    H.pend_val.swap(pval);
    return SPMM_OK;
}

}  // namespace

// Column relabelling by descending in-degree (ties by column id) from the
// column counts: a counting sort over degrees, stable in the original order.
static void relabel_columns(Handle& H) {
    const std::vector<uint32_t>& indeg = H.col_count;
    const int64_t m = H.n_cols;
    uint32_t maxd = 0;
    for (int64_t c = 0; c < m; ++c) maxd = std::max(maxd, indeg[c]);
    std::vector<uint64_t> start((size_t)maxd + 2, 0);
    for (int64_t c = 0; c < m; ++c) start[maxd - indeg[c] + 1]++;
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    H.col_new.resize((size_t)m);
    H.col_old.resize((size_t)m);
    for (int64_t c = 0; c < m; ++c) {
        const uint64_t r = start[maxd - indeg[c]]++;
        H.col_new[c] = (int32_t)r;
        H.col_old[r] = (int32_t)c;
    }
}

void build_init(Handle& H, bool has_val) {
    H.has_val = has_val;
    H.wshift = log2_exact(H.w);
    H.n_strips = (uint64_t)((H.n_cols + H.w - 1) / H.w);
    if (H.n_strips == 0) H.n_strips = 1;
    H.col_count.assign((size_t)H.n_cols, 0);
    H.max_row_l1 = 0.0;
    H.nnz = 0;
    H.n_slabs = 0;
    H.n_tiled_rows = 0;
    H.sum_nnr = H.sum_nnc = 0;
    H.next_row = 0;
    H.pend_off.assign(1, 0);
}

spmm_status_t build_canonical(Handle& H, const int64_t* row_ptr, const int32_t* col,
                              const float* val, bool validate, std::string& err) {
    const int64_t n = H.n_rows;
    if (row_ptr[0] != 0) {
        err = "row_ptr[0] must be 0";
        return SPMM_EINVAL;
    }
    if (row_ptr[n] < 0) {
        err = "row_ptr[n_rows] is negative";
        return SPMM_EINVAL;
    }
    build_init(H, val != nullptr);
    spmm_status_t st = scan_rows(H, n, row_ptr, col, val, validate, err);
    if (st != SPMM_OK) return st;
    H.nnz = row_ptr[n];
    // Column relabelling by descending in-degree (ties by column id).
    if (H.relabel) relabel_columns(H);
    try {
        H.ent.reserve((size_t)H.nnz);
        if (val) H.val.reserve((size_t)H.nnz);
    } catch (const std::bad_alloc&) {
        err = "out of host memory for the tile store";
        return SPMM_ENOMEM;
    }
    // Row order (one block: the whole matrix).  With row relabelling, tile
    // rows take the rows by descending out-degree (ties by row id), so that
    // rows sharing the hub columns sit in the same tile rows and gather those
    // X rows once per tile row; rows without entries are left out of the
    // tiles and zero-filled at run time.
    if ((st = tile_block(H, 0, n, row_ptr, col, val, true, err)) != SPMM_OK) return st;
    return build_finish_rows(H, err);
}

spmm_status_t build_csr(Handle& H, const int64_t* row_ptr, const int32_t* col, bool validate, std::string& err) {
    const int64_t n = H.n_rows;
    if (row_ptr[0] != 0 || row_ptr[n] < 0) {
        err = "row_ptr[0] must be 0 and row_ptr[n_rows] >= 0";
        return SPMM_EINVAL;
    }
    build_init(H, false);
    spmm_status_t st = scan_rows(H, n, row_ptr, col, nullptr, validate, err);
    if (st != SPMM_OK) return st;
    H.nnz = row_ptr[n];
    if (H.relabel) relabel_columns(H);
    CsrStore& C = H.csr;
    // rows by descending length, ties by row id (stable counting sort on
    // cap - min(length, cap), then the longest rows ordered exactly)
    uint64_t maxl = 0;
    for (int64_t r = 0; r < n; ++r) maxl = std::max<uint64_t>(maxl, (uint64_t)(row_ptr[r + 1] - row_ptr[r]));
    const uint64_t cap = std::min<uint64_t>(maxl, 1u << 20);
    auto key = [&](int64_t r) { return cap - std::min<uint64_t>(cap, (uint64_t)(row_ptr[r + 1] - row_ptr[r])); };
    std::vector<uint64_t> start(cap + 2, 0);
    for (int64_t r = 0; r < n; ++r) start[key(r) + 1]++;
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    const uint64_t nbig = start[1];
    H.row_old.resize((size_t)n);
    for (int64_t r = 0; r < n; ++r) H.row_old[start[key(r)]++] = (int32_t)r;
    std::stable_sort(H.row_old.begin(), H.row_old.begin() + (int64_t)nbig, [&](int32_t a, int32_t b) {
        return row_ptr[a + 1] - row_ptr[a] > row_ptr[b + 1] - row_ptr[b];
    });
    C.rp.resize((size_t)n + 1);
    C.rp[0] = 0;
    for (int64_t r = 0; r < n; ++r) C.rp[r + 1] = C.rp[r] + (row_ptr[H.row_old[r] + 1] - row_ptr[H.row_old[r]]);
    C.col.resize((size_t)H.nnz);
    const int32_t* cmap = H.relabel ? H.col_new.data() : nullptr;
    parallel_for((uint64_t)n, H.threads, 1 << 12, [&](uint64_t a, uint64_t b) {
        for (uint64_t r = a; r < b; ++r) {
            const int64_t o = H.row_old[r];
            int32_t* dst = C.col.data() + C.rp[r];
            const int64_t len = row_ptr[o + 1] - row_ptr[o];
            for (int64_t p = 0; p < len; ++p) {
                const int32_t c = col[row_ptr[o] + p];
                dst[p] = cmap ? cmap[c] : c;
            }
            if (cmap) std::sort(dst, dst + len);
        }
    });
    // row classes: split rows first, then wavefront rows, then group rows
    C.seg.clear();
    C.srow.clear();
    C.pb.assign(1, 0);
    C.n_split = C.n_wave_rows = C.n_pieces = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t len = C.rp[r + 1] - C.rp[r];
        if (len <= kCsrWaveMin) break;
        C.n_wave_rows = r + 1;
        if (len > kCsrPiece) {
            C.srow.push_back(r);
            for (int64_t q = C.rp[r]; q < C.rp[r + 1]; q += kCsrPiece)
                C.seg.insert(C.seg.end(), {r, q, std::min(C.rp[r + 1], q + kCsrPiece), C.n_pieces++});
            C.pb.push_back(C.n_pieces);
            C.n_split++;
        } else {
            C.seg.insert(C.seg.end(), {r, C.rp[r], C.rp[r + 1], -1});
        }
    }
    C.n_seg = (int64_t)C.seg.size() / 4;
    H.n_tiled_rows = n;   // every row is written by the kernels (empty ones with zeros)
    return SPMM_OK;
}

// Encode the tile rows cut since the last flush, append them to the
// encoding, and release their canonical tiles: a slab-wise build holds one
// block's tiles at a time.
spmm_status_t flush_slabs(Handle& H, std::string& err) {
    if (H.n_slabs == H.slab_base) return SPMM_OK;
    spmm_status_t st = encode_range(H, H.slab_base, H.n_slabs, err);
    if (st != SPMM_OK) return st;
    H.slab_base = H.n_slabs;
    std::vector<Tile>().swap(H.tiles);
    std::vector<uint32_t>().swap(H.ent);
    std::vector<float>().swap(H.val);
    std::vector<uint8_t>().swap(H.variant);
    std::vector<uint64_t>().swap(H.slab_tiles);
    H.canonical = false;
    return SPMM_OK;
}

spmm_status_t build_append(Handle& H, int64_t row0, int64_t nr, const int64_t* rp, const int32_t* col,
                           const float* val, bool validate, std::string& err) {
    if (row0 != H.next_row || nr < 0 || row0 + nr > H.n_rows) {
        err = "rows must be appended in order: expected row " + std::to_string(H.next_row);
        return SPMM_EINVAL;
    }
    if (rp[0] != 0) {
        err = "row_ptr_local[0] must be 0";
        return SPMM_EINVAL;
    }
    if ((val != nullptr) != H.has_val) {
        err = "values must be given for every block or for none";
        return SPMM_EINVAL;
    }
    spmm_status_t st = scan_rows(H, nr, rp, col, val, validate, err);
    if (st != SPMM_OK) return st;
    if ((st = tile_block(H, row0, nr, rp, col, val, false, err)) != SPMM_OK) return st;
    H.nnz += rp[nr];
    H.next_row = row0 + nr;
    return flush_slabs(H, err);
}

spmm_status_t build_finish_rows(Handle& H, std::string& err) {
    if (!H.pend_row.empty()) {
        spmm_status_t st = tile_block(H, H.next_row, 0, nullptr, nullptr, nullptr, true, err);
        if (st != SPMM_OK) return st;
    }
    if (H.row_relabel) {
        H.row_old.insert(H.row_old.end(), H.zero_rows.begin(), H.zero_rows.end());
        std::vector<int32_t>().swap(H.zero_rows);
        if ((int64_t)H.row_old.size() != H.n_rows) {
            err = "internal: row order does not cover every row";
            return SPMM_ESTATE;
        }
        // a relabelled handle whose rows all stayed in place needs no map
        bool identity = H.n_tiled_rows == H.n_rows;
        for (int64_t r = 0; r < H.n_rows && identity; ++r) identity = H.row_old[(size_t)r] == (int32_t)r;
        if (identity) std::vector<int32_t>().swap(H.row_old);
    }
    std::vector<int64_t>().swap(H.pend_row);
    std::vector<uint64_t>().swap(H.pend_off);
    std::vector<int32_t>().swap(H.pend_col);
    std::vector<float>().swap(H.pend_val);
    return SPMM_OK;
}

namespace {

// A run of one row inside one tile: entries ent[ent, ent + len).
struct Seg {
    uint32_t J, row, len;
    uint64_t ent;
};

struct ChunkOut {
    std::vector<ItemDesc> items;  // blob_off relative to the chunk blob
    std::vector<uint32_t> nnz;
    std::vector<uint8_t> blob;
    std::vector<CombineDesc> combine;  // part_* relative to the chunk's first part
    uint32_t n_parts = 0;
    uint64_t vt[SPMM_NUM_VARIANTS] = {}, vn[SPMM_NUM_VARIANTS] = {};
};

struct CooEnt {
    uint32_t J, e;   // strip, (row << 16) | col
    uint64_t src;    // canonical entry (for the value)
};

struct Scratch {
    std::vector<CooEnt> coo;
    std::vector<uint32_t> rdeg;
    std::vector<uint64_t> cursor;
    std::vector<Seg> segs, lr, wr, piece;
    std::vector<uint32_t> coo_ent, coo_J, Js;
    std::vector<float> coo_val;
};

// Encode the row segments `segs` (tile order) as one work item owning local
// rows [lo, hi) (or, with part >= 0, one piece of the split row lo).
void emit_item(const Handle& H, uint32_t slab, uint32_t lo, uint32_t hi, int32_t part,
               uint32_t cid, const std::vector<Seg>& segs, ChunkOut& out, Scratch& S) {
    const bool hv = H.has_val;
    S.coo_ent.clear();
    S.coo_val.clear();
    S.coo_J.clear();
    S.lr.clear();
    S.wr.clear();
    S.coo.clear();
    uint32_t nnz = 0;
    for (const Seg& g : segs) {
        nnz += g.len;
        const int v = g.row >> 16;  // the tile's variant rides in the high bits
        const uint32_t row = g.row & 0xFFFFu;
        const bool coo = v == SPMM_VAR_COO || g.len == 1 || (v == SPMM_VAR_HYBRID && g.len < kWaveRowMin);
        if (coo) {
            for (uint32_t q = 0; q < g.len; ++q) S.coo.push_back({g.J, H.ent[g.ent + q], g.ent + q});
        } else if (v == SPMM_VAR_ROW) {
            for (uint32_t q = 0; q < g.len; q += kRowLaneMax)
                S.lr.push_back({g.J, row, std::min(kRowLaneMax, g.len - q), g.ent + q});
        } else {
            S.wr.push_back({g.J, row, g.len, g.ent});
        }
    }
    // COO entries in column-major order inside each tile, so that lanes of
    // one step gathering the same (or a neighbouring) X row share its cache
    // line.  (Accumulation is exact integer arithmetic, so any order gives
    // the same result.)
    std::sort(S.coo.begin(), S.coo.end(), [](const CooEnt& a, const CooEnt& b) {
        if (a.J != b.J) return a.J < b.J;
        const uint32_t ca = a.e & 0xFFFFu, cb = b.e & 0xFFFFu;
        return ca != cb ? ca < cb : a.e < b.e;
    });
    for (size_t q = 0; q < S.coo.size(); ++q) {
        const bool first = q == 0 || S.coo[q].J != S.coo[q - 1].J;
        if (first) S.coo_J.push_back(S.coo[q].J);
        S.coo_ent.push_back((first ? kCooNewTile : 0u) | S.coo[q].e);
        if (hv) S.coo_val.push_back(H.val[S.coo[q].src]);
    }
    // row-lane segments: longest first, interleaved in blocks of 64
    std::stable_sort(S.lr.begin(), S.lr.end(), [](const Seg& a, const Seg& b) { return a.len > b.len; });
    S.Js.clear();
    for (const Seg& g : S.lr) S.Js.push_back(g.J);
    std::sort(S.Js.begin(), S.Js.end());
    S.Js.erase(std::unique(S.Js.begin(), S.Js.end()), S.Js.end());
    uint32_t lr_cols = 0;
    for (size_t b = 0; b < S.lr.size(); b += 64) lr_cols += 64u * S.lr[b].len;
    uint32_t wr_cols = 0;
    for (const Seg& g : S.wr) wr_cols += g.len;

    ItemDesc d{};
    d.slab = slab;
    d.part = part;
    d.rows = lo | (hi << 16);
    d.cid = cid;
    d.n_coo = (uint32_t)S.coo_ent.size();
    d.n_coo_J = (uint32_t)S.coo_J.size();
    d.n_lr = (uint32_t)S.lr.size();
    d.n_lr_J = (uint32_t)S.Js.size();
    d.n_wr = (uint32_t)S.wr.size();
    d.n_cols = lr_cols + wr_cols;
    const ItemLayout L = item_layout(d, hv);
    const uint64_t base = out.blob.size();
    d.blob_off = base;
    out.blob.resize(base + L.bytes, 0);
    uint8_t* P = out.blob.data() + base;
    auto* pe = reinterpret_cast<uint32_t*>(P);
    auto* pv = reinterpret_cast<float*>(P + 4 * (size_t)d.n_coo);
    auto* pj = reinterpret_cast<uint32_t*>(P + L.o_coo_J);
    auto* pl = reinterpret_cast<uint32_t*>(P + L.o_lr);
    auto* plj = reinterpret_cast<uint32_t*>(P + L.o_lr_J);
    auto* pw = reinterpret_cast<uint32_t*>(P + L.o_wr);
    auto* pc = reinterpret_cast<uint16_t*>(P + L.o_cols);
    auto* pcv = reinterpret_cast<float*>(P + L.o_cval);
    for (uint32_t e = 0; e < d.n_coo; ++e) {
        pe[e] = S.coo_ent[e];
        if (hv) pv[e] = S.coo_val[e];
    }
    for (uint32_t q = 0; q < d.n_coo_J; ++q) pj[q] = S.coo_J[q];
    for (uint32_t q = 0; q < d.n_lr_J; ++q) plj[q] = S.Js[q];
    uint32_t block_base = 0;
    for (uint32_t q = 0; q < d.n_lr; ++q) {
        const Seg& g = S.lr[q];
        if (q % 64 == 0 && q) block_base += 64u * S.lr[q - 64].len;
        const uint32_t start = block_base + (q % 64);
        const uint32_t ord = (uint32_t)(std::lower_bound(S.Js.begin(), S.Js.end(), g.J) - S.Js.begin());
        pl[2 * q] = g.row | (ord << 12);
        pl[2 * q + 1] = start | (g.len << kLrStartBits);
        for (uint32_t t = 0; t < g.len; ++t) {
            pc[start + 64u * t] = (uint16_t)(H.ent[g.ent + t] & 0xFFFFu);
            if (hv) pcv[start + 64u * t] = H.val[g.ent + t];
        }
    }
    uint32_t cpos = lr_cols;
    for (uint32_t q = 0; q < d.n_wr; ++q) {
        const Seg& g = S.wr[q];
        pw[4 * q] = g.J;
        pw[4 * q + 1] = g.row;
        pw[4 * q + 2] = cpos;
        pw[4 * q + 3] = g.len;
        for (uint32_t t = 0; t < g.len; ++t) {
            pc[cpos + t] = (uint16_t)(H.ent[g.ent + t] & 0xFFFFu);
            if (hv) pcv[cpos + t] = H.val[g.ent + t];
        }
        cpos += g.len;
    }
    out.items.push_back(d);
    out.nnz.push_back(nnz);
}

// Cut one slab into row-range items of about C non-zeros; a row longer than
// C becomes its own items ("pieces") combined through partial slots.
void encode_slab(const Handle& H, uint64_t s, ChunkOut& out, Scratch& S) {
    const uint32_t C = H.item_nnz;
    const int64_t r0 = (int64_t)s * H.h;
    const uint32_t nr = (uint32_t)std::min<int64_t>(H.h, H.n_tiled_rows - r0);
    const uint64_t t0 = H.slab_tiles[s - H.slab_base], t1 = H.slab_tiles[s - H.slab_base + 1];
    S.rdeg.assign(nr, 0);
    S.cursor.resize(t1 - t0);
    for (uint64_t t = t0; t < t1; ++t) {
        const Tile& tl = H.tiles[t];
        out.vt[H.variant[t]] += 1;
        out.vn[H.variant[t]] += tl.nnz;
        for (uint32_t i = 0; i < tl.nnz; ++i) S.rdeg[H.ent[tl.ent_begin + i] >> 16]++;
        S.cursor[t - t0] = tl.ent_begin;
    }
    // gather the segments of rows [lo, hi) from every tile (cursors advance
    // monotonically because ranges are visited in row order)
    auto collect = [&](uint32_t lo, uint32_t hi) {
        S.segs.clear();
        for (uint64_t t = t0; t < t1; ++t) {
            const Tile& tl = H.tiles[t];
            const uint64_t end = tl.ent_begin + tl.nnz;
            uint64_t& c = S.cursor[t - t0];
            while (c < end && (H.ent[c] >> 16) < hi) {
                const uint32_t r = H.ent[c] >> 16;
                uint64_t e = c;
                while (e < end && (H.ent[e] >> 16) == r) ++e;
                if (r >= lo)
                    S.segs.push_back({tl.J, r | ((uint32_t)H.variant[t] << 16), (uint32_t)(e - c), c});
                c = e;
            }
        }
    };
    uint32_t lo = 0, running = 0;
    bool any = false;
    for (uint32_t r = 0; r < nr; ++r) {
        const uint32_t dgr = S.rdeg[r];
        if (dgr > C) {
            if (r > lo) {
                collect(lo, r);
                emit_item(H, (uint32_t)s, lo, r, -1, 0, S.segs, out, S);
            }
            collect(r, r + 1);
            // pieces of at most C entries; segments longer than C are cut
            const uint32_t cid = (uint32_t)out.combine.size();
            const uint32_t pb = out.n_parts;
            uint32_t acc = 0;
            S.piece.clear();
            for (const Seg& g0 : S.segs) {
                Seg g = g0;
                while (g.len) {
                    uint32_t take = std::min(g.len, C - acc);
                    S.piece.push_back({g.J, g.row, take, g.ent});
                    acc += take;
                    g.len -= take;
                    g.ent += take;
                    if (acc == C) {
                        emit_item(H, (uint32_t)s, r, r + 1, (int32_t)out.n_parts++, cid, S.piece, out, S);
                        S.piece.clear();
                        acc = 0;
                    }
                }
            }
            if (!S.piece.empty())
                emit_item(H, (uint32_t)s, r, r + 1, (int32_t)out.n_parts++, cid, S.piece, out, S);
            out.combine.push_back({(uint32_t)s, r, pb, out.n_parts});
            lo = r + 1;
            running = 0;
            any = true;
            continue;
        }
        if (running + dgr > C && r > lo) {
            collect(lo, r);
            emit_item(H, (uint32_t)s, lo, r, -1, 0, S.segs, out, S);
            lo = r;
            running = 0;
            any = true;
        }
        running += dgr;
    }
    if (lo < nr || !any) {
        collect(lo, nr);
        emit_item(H, (uint32_t)s, lo, nr, -1, 0, S.segs, out, S);
    }
}

}  // namespace

std::vector<Handle::Group> make_groups(const Encoded& E, uint64_t stream_bytes, uint32_t h) {
    // consecutive items whose payload adds up to about stream_bytes form one
    // transfer group (items are laid out back to back in the blob)
    std::vector<Handle::Group> groups;
    const uint64_t ni = E.items.size();
    uint64_t i0 = 0;
    while (i0 < ni) {
        const uint64_t b0 = E.items[i0].blob_off;
        uint64_t i1 = i0 + 1;
        while (i1 < ni && E.items[i1].blob_off - b0 < stream_bytes) ++i1;
        // never split the pieces of one split row across groups: each launch
        // must see all pieces of a row, so that its per-row counter and
        // partial slots are used by one column chunk at a time
        while (i1 < ni && E.items[i1].part >= 0 && E.items[i1 - 1].part >= 0 && E.items[i1].cid == E.items[i1 - 1].cid)
            ++i1;
        const uint64_t b1 = i1 < ni ? E.items[i1].blob_off : (uint64_t)E.blob.size();
        // items come in tiled-row order, so the group writes one row range
        const ItemDesc& f = E.items[i0];
        const ItemDesc& l = E.items[i1 - 1];
        const uint64_t r0 = (uint64_t)f.slab * h + (f.rows & 0xFFFFu);
        const uint64_t r1 = (uint64_t)l.slab * h + (l.rows >> 16);
        groups.push_back({i0, i1, b0, b1, r0, r1});
        i0 = i1;
    }
    return groups;
}

spmm_status_t encode(Handle& H, std::string& err) {
    H.enc = Encoded{};
    return encode_range(H, H.slab_base, H.n_slabs, err);
}

spmm_status_t encode_range(Handle& H, uint64_t s0, uint64_t s1, std::string& err) {
    const uint64_t S = s1 - s0;
    const uint64_t chunk = 256;
    const uint64_t nchunks = (S + chunk - 1) / chunk;
    std::vector<ChunkOut> outs(nchunks);
    try {
        parallel_for(nchunks, H.threads, 1, [&](uint64_t a, uint64_t b) {
            Scratch sc;
            for (uint64_t c = a; c < b; ++c) {
                const uint64_t e1 = s0 + std::min(S, (c + 1) * chunk);
                for (uint64_t s = s0 + c * chunk; s < e1; ++s) encode_slab(H, s, outs[c], sc);
            }
        });
    } catch (const std::bad_alloc&) {
        err = "out of host memory while encoding tiles";
        return SPMM_ENOMEM;
    }
    Encoded& E = H.enc;
    // offsets of this range's output in the accumulated encoding
    const uint64_t item0 = E.items.size(), byte0 = E.blob.size(), comb0 = E.combine.size();
    const uint64_t part0 = E.n_parts;
    std::vector<uint64_t> item_off(nchunks + 1, item0), byte_off(nchunks + 1, byte0), comb_off(nchunks + 1, comb0);
    std::vector<uint64_t> part_off(nchunks + 1, part0);
    for (uint64_t c = 0; c < nchunks; ++c) {
        item_off[c + 1] = item_off[c] + outs[c].items.size();
        byte_off[c + 1] = byte_off[c] + outs[c].blob.size();
        comb_off[c + 1] = comb_off[c] + outs[c].combine.size();
        part_off[c + 1] = part_off[c] + outs[c].n_parts;
        for (int v = 0; v < SPMM_NUM_VARIANTS; ++v) {
            E.variant_tiles[v] += outs[c].vt[v];
            E.variant_nnz[v] += outs[c].vn[v];
        }
    }
    if (part_off[nchunks] > INT32_MAX) {
        err = "too many split-row pieces for 32-bit slot indices";
        return SPMM_EUNSUPPORTED;
    }
    try {
        E.items.resize(item_off[nchunks]);
        E.item_nnz.resize(item_off[nchunks]);
        E.blob.resize(byte_off[nchunks]);
        E.combine.resize(comb_off[nchunks]);
    } catch (const std::bad_alloc&) {
        err = "out of host memory for the encoded tiles";
        return SPMM_ENOMEM;
    }
    parallel_for(nchunks, H.threads, 1, [&](uint64_t a, uint64_t b) {
        for (uint64_t c = a; c < b; ++c) {
            ChunkOut& o = outs[c];
            if (!o.blob.empty()) std::memcpy(E.blob.data() + byte_off[c], o.blob.data(), o.blob.size());
            for (size_t i = 0; i < o.items.size(); ++i) {
                ItemDesc d = o.items[i];
                d.blob_off += byte_off[c];
                if (d.part >= 0) {
                    d.part += (int32_t)part_off[c];
                    d.cid += (uint32_t)comb_off[c];
                }
                E.items[item_off[c] + i] = d;
                E.item_nnz[item_off[c] + i] = o.nnz[i];
            }
            for (size_t i = 0; i < o.combine.size(); ++i) {
                CombineDesc cd = o.combine[i];
                cd.part_begin += (uint32_t)part_off[c];
                cd.part_end += (uint32_t)part_off[c];
                E.combine[comb_off[c] + i] = cd;
            }
            std::vector<uint8_t>().swap(o.blob);
        }
    });
    E.n_parts = part_off[nchunks];
    H.blob_bytes = E.blob.size();
    return SPMM_OK;
}

}  // namespace spmm

namespace spmm {

void tile_features(const Handle& H, int k, int xbytes, float* out) {
    parallel_for(H.tiles.size(), H.threads, 1 << 14, [&](uint64_t a, uint64_t b) {
        for (uint64_t t = a; t < b; ++t) {
            const Tile& tl = H.tiles[t];
            float* f = out + t * SPMM_NUM_FEATURES;
            float mean = (float)tl.nnz / (float)std::max(1u, tl.nnr);
            f[0] = std::log2(1.0f + (float)tl.nnz);
            f[1] = std::log2(1.0f + (float)tl.nnr);
            f[2] = std::log2(1.0f + (float)tl.nnc);
            f[3] = std::log2(1.0f + (float)tl.max_row);
            f[4] = (float)tl.n_single / (float)std::max(1u, tl.nnr);
            f[5] = std::log2((float)tl.max_row / std::max(mean, 1.0f));
            f[6] = std::log2((float)k);
            f[7] = std::log2((float)xbytes);
        }
    });
}

spmm_status_t model_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                          const int32_t* col, int64_t t, uint32_t threads, uint64_t* n_tiles,
                          uint64_t* sum_nnr, uint64_t* sum_nnc) {
    const uint64_t S = (uint64_t)((n_rows + t - 1) / t);
    const uint64_t nstrip = (uint64_t)((n_cols + t - 1) / t);
    std::atomic<uint64_t> T{0}, R{0}, Cc{0};
    parallel_for(S, threads, 1, [&](uint64_t a, uint64_t b) {
        std::vector<uint64_t> colbits((size_t)((n_cols + 63) / 64), 0);
        std::vector<uint64_t> stripbits((size_t)((nstrip + 63) / 64), 0);
        uint64_t myT = 0, myR = 0, myC = 0;
        for (uint64_t s = a; s < b; ++s) {
            int64_t r0 = (int64_t)s * t, r1 = std::min<int64_t>(n_rows, r0 + t);
            for (int64_t r = r0; r < r1; ++r) {
                int64_t prevJ = -1;
                for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
                    int64_t c = col[p], J = c / t;
                    if (J != prevJ) { ++myR; prevJ = J; }  // columns sorted within a row
                    uint64_t bit = 1ull << (c & 63);
                    if (!(colbits[c >> 6] & bit)) { colbits[c >> 6] |= bit; ++myC; }
                    uint64_t jb = 1ull << (J & 63);
                    if (!(stripbits[J >> 6] & jb)) { stripbits[J >> 6] |= jb; ++myT; }
                }
            }
            for (int64_t p = row_ptr[r0]; p < row_ptr[r1]; ++p) {
                colbits[col[p] >> 6] = 0;
                stripbits[(col[p] / t) >> 6] = 0;
            }
        }
        T += myT;
        R += myR;
        Cc += myC;
    });
    *n_tiles = T;
    *sum_nnr = R;
    *sum_nnc = Cc;
    return SPMM_OK;
}

}  // namespace spmm

namespace spmm {

// Walk every item exactly as the kernel does and emit its (row, col, val)
// entries; sort them back into CSR order.
spmm_status_t decode(const Handle& H, int64_t* row_ptr, int32_t* col, float* val,
                     std::string& err) {
    if (H.format == SPMM_FORMAT_CSR) {
        // the CSR store in the original row and column order
        const CsrStore& C = H.csr;
        std::vector<int64_t> len((size_t)H.n_rows, 0), at((size_t)H.n_rows, 0);
        for (int64_t r = 0; r < H.n_rows; ++r) len[(size_t)H.row_old[r]] = C.rp[r + 1] - C.rp[r];
        row_ptr[0] = 0;
        for (int64_t r = 0; r < H.n_rows; ++r) row_ptr[r + 1] = row_ptr[r] + len[(size_t)r];
        for (int64_t r = 0; r < H.n_rows; ++r) {
            const int64_t o = H.row_old[r];
            int32_t* dst = col + row_ptr[o];
            for (int64_t p = C.rp[r]; p < C.rp[r + 1]; ++p)
                *dst++ = H.relabel ? H.col_old[(size_t)C.col[(size_t)p]] : C.col[(size_t)p];
            std::sort(col + row_ptr[o], dst);
            if (val) std::fill(val + row_ptr[o], val + row_ptr[o + 1], 1.0f);
        }
        (void)at;
        (void)err;
        return SPMM_OK;
    }
    static const uint8_t empty_payload[16] = {};
    const uint8_t* blob = H.enc.blob.empty() ? static_cast<const uint8_t*>(H.h_blob) : H.enc.blob.data();
    if (!blob && H.blob_bytes == 0) blob = empty_payload;
    if (!blob) {
        err = "no host copy of the tile payload";
        return SPMM_ESTATE;
    }
    struct Trip { int64_t r; int64_t c; float v; };
    std::vector<Trip> out;
    out.reserve((size_t)H.nnz);
    const bool hv = H.has_val;
    for (const ItemDesc& d : H.enc.items) {
        const ItemLayout L = item_layout(d, hv);
        const uint8_t* base = blob + d.blob_off;
        const int64_t row0 = (int64_t)d.slab * H.h;
        const uint32_t lo = d.rows & 0xFFFFu, hi = d.rows >> 16;
        auto check_row = [&](uint32_t r) { return r >= lo && r < hi; };
        const uint32_t* ent = reinterpret_cast<const uint32_t*>(base);
        const float* cval = reinterpret_cast<const float*>(base + 4 * (size_t)d.n_coo);
        const uint32_t* cJ = reinterpret_cast<const uint32_t*>(base + L.o_coo_J);
        int64_t ord = -1;
        for (uint32_t e = 0; e < d.n_coo; ++e) {
            if (ent[e] & kCooNewTile) ++ord;
            const uint32_t r = (ent[e] >> 16) & 0xFFFu;
            if (ord < 0 || ord >= (int64_t)d.n_coo_J || !check_row(r)) {
                err = "COO entry outside its item";
                return SPMM_ESTATE;
            }
            int64_t c = ((int64_t)cJ[ord] << H.wshift) + (ent[e] & 0xFFFFu);
            out.push_back({row0 + r, c, hv ? cval[e] : 1.0f});
        }
        const uint32_t* ls = reinterpret_cast<const uint32_t*>(base + L.o_lr);
        const uint32_t* lj = reinterpret_cast<const uint32_t*>(base + L.o_lr_J);
        const uint16_t* cols = reinterpret_cast<const uint16_t*>(base + L.o_cols);
        const float* cv = reinterpret_cast<const float*>(base + L.o_cval);
        for (uint32_t q = 0; q < d.n_lr; ++q) {
            const uint32_t r = ls[2 * q] & 0xFFFu, tord = ls[2 * q] >> 12;
            const uint32_t start = ls[2 * q + 1] & ((1u << kLrStartBits) - 1), len = ls[2 * q + 1] >> kLrStartBits;
            if (tord >= d.n_lr_J || !check_row(r) || start + 64u * (len ? len - 1 : 0) >= d.n_cols + (len ? 0 : 1)) {
                err = "row segment outside its item";
                return SPMM_ESTATE;
            }
            int64_t cb = (int64_t)lj[tord] << H.wshift;
            for (uint32_t t = 0; t < len; ++t)
                out.push_back({row0 + r, cb + cols[start + 64u * t], hv ? cv[start + 64u * t] : 1.0f});
        }
        const uint32_t* wr = reinterpret_cast<const uint32_t*>(base + L.o_wr);
        for (uint32_t q = 0; q < d.n_wr; ++q) {
            const uint32_t* g = wr + 4 * q;
            if (!check_row(g[1]) || g[2] + g[3] > d.n_cols) {
                err = "wavefront segment outside its item";
                return SPMM_ESTATE;
            }
            int64_t cb = (int64_t)g[0] << H.wshift;
            for (uint32_t t = 0; t < g[3]; ++t)
                out.push_back({row0 + g[1], cb + cols[g[2] + t], hv ? cv[g[2] + t] : 1.0f});
        }
    }
    if ((int64_t)out.size() != H.nnz) {
        err = "decoded entry count differs from nnz";
        return SPMM_ESTATE;
    }
    // every tiled row must be written by exactly one owner: an item's row
    // range, or the combine of a split row (rows past n_tiled_rows of a
    // row-relabelled handle have no entries and are zero-filled)
    std::vector<uint8_t> own((size_t)H.n_tiled_rows, 0);
    for (const ItemDesc& d : H.enc.items) {
        if (d.part >= 0) continue;
        const int64_t row0 = (int64_t)d.slab * H.h;
        for (uint32_t r = d.rows & 0xFFFFu; r < (d.rows >> 16); ++r) own[row0 + r]++;
    }
    for (const CombineDesc& c : H.enc.combine) own[(int64_t)c.slab * H.h + c.row]++;
    for (int64_t r = 0; r < H.n_tiled_rows; ++r)
        if (own[r] != 1) {
            err = "row " + std::to_string(r) + " has " + std::to_string(own[r]) + " owners";
            return SPMM_ESTATE;
        }
    if (!H.row_old.empty())
        for (Trip& t : out) {
            if (t.r < 0 || t.r >= H.n_tiled_rows) {
                err = "decoded row out of range";
                return SPMM_ESTATE;
            }
            t.r = H.row_old[(size_t)t.r];
        }
    if (H.relabel)
        for (Trip& t : out) t.c = H.col_old[(size_t)t.c];
    std::sort(out.begin(), out.end(), [](const Trip& a, const Trip& b) {
        return a.r != b.r ? a.r < b.r : a.c < b.c;
    });
    std::fill(row_ptr, row_ptr + H.n_rows + 1, 0);
    for (size_t i = 0; i < out.size(); ++i) {
        if (out[i].r < 0 || out[i].r >= H.n_rows) {
            err = "decoded row out of range";
            return SPMM_ESTATE;
        }
        row_ptr[out[i].r + 1]++;
        col[i] = (int32_t)out[i].c;
        if (val) val[i] = out[i].v;
    }
    for (int64_t r = 0; r < H.n_rows; ++r) row_ptr[r + 1] += row_ptr[r];
    return SPMM_OK;
}

}  // namespace spmm
