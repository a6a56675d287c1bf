// Host-side tile builder: CSR -> canonical tile store -> encoded work items.
//
// The canonical store follows the paper's sparse format (Section 3.2): the
// matrix is cut into h x w tiles, tiles of one tile row ("slab") are kept in
// column order, and every entry is a 16-bit local row and a 16-bit local
// column inside its tile.  Conversion is one linear pass over the CSR
// (Section 6, Table 3).  The encoder then turns each slab into work items
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

spmm_status_t build_canonical(Handle& H, const int64_t* row_ptr, const int32_t* col,
                              const float* val, bool validate, std::string& err) {
    const int64_t n = H.n_rows;
    if (row_ptr[0] != 0) {
        err = "row_ptr[0] must be 0";
        return SPMM_EINVAL;
    }
    const int64_t nnz = row_ptr[n];
    if (nnz < 0) {
        err = "row_ptr[n_rows] is negative";
        return SPMM_EINVAL;
    }
    H.nnz = nnz;
    H.has_val = val != nullptr;
    H.wshift = log2_exact(H.w);
    H.n_slabs = (uint64_t)((n + H.h - 1) / H.h);
    H.n_strips = (uint64_t)((H.n_cols + H.w - 1) / H.w);
    if (H.n_strips == 0) H.n_strips = 1;

    // Row pointers must be monotone; columns in range (and sorted, unique when
    // validation is on: the tile encoding relies on sorted rows only for
    // determinism of the layout, not for correctness).
    std::atomic<int> bad{0};
    parallel_for((uint64_t)n, H.threads, 1 << 16, [&](uint64_t a, uint64_t b) {
        for (uint64_t i = a; i < b; ++i) {
            if (row_ptr[i + 1] < row_ptr[i]) { bad = 1; return; }
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                if (col[p] < 0 || col[p] >= H.n_cols) { bad = 2; return; }
                if (validate && p > row_ptr[i] && col[p] <= col[p - 1]) { bad = 3; return; }
            }
        }
    });
    if (bad) {
        err = bad == 1 ? "row_ptr is not non-decreasing"
            : bad == 2 ? "column index out of range"
                       : "columns not sorted and unique within a row";
        return SPMM_EINVAL;
    }

    // Pass 1: non-empty tiles per slab.
    std::vector<uint64_t> ntile(H.n_slabs + 1, 0);
    const uint32_t nstrip = (uint32_t)H.n_strips;
    parallel_for(H.n_slabs, H.threads, 64, [&](uint64_t a, uint64_t b) {
        std::vector<uint32_t> cnt(nstrip, 0);
        std::vector<uint32_t> used;
        for (uint64_t s = a; s < b; ++s) {
            int64_t r0 = (int64_t)s * H.h, r1 = std::min<int64_t>(n, r0 + H.h);
            used.clear();
            for (int64_t p = row_ptr[r0]; p < row_ptr[r1]; ++p) {
                uint32_t J = (uint32_t)col[p] >> H.wshift;
                if (cnt[J]++ == 0) used.push_back(J);
            }
            ntile[s + 1] = used.size();
            for (uint32_t J : used) cnt[J] = 0;
        }
    });
    H.slab_tiles.assign(H.n_slabs + 1, 0);
    for (uint64_t s = 0; s < H.n_slabs; ++s) H.slab_tiles[s + 1] = H.slab_tiles[s] + ntile[s + 1];
    const uint64_t T = H.slab_tiles[H.n_slabs];
    try {
        H.tiles.resize(T);
        H.ent.resize((size_t)nnz);
        if (val) H.val.resize((size_t)nnz);
        H.variant.assign(T, (uint8_t)SPMM_VAR_HYBRID);
    } catch (const std::bad_alloc&) {
        err = "out of host memory for the tile store";
        return SPMM_ENOMEM;
    }

    // Pass 2: scatter entries tile-major, then per-tile statistics.
    std::atomic<uint64_t> tot_nnr{0}, tot_nnc{0};
    parallel_for(H.n_slabs, H.threads, 64, [&](uint64_t a, uint64_t b) {
        std::vector<uint32_t> cnt(nstrip, 0);
        std::vector<uint64_t> pos(nstrip, 0);
        std::vector<uint32_t> used;
        std::vector<uint64_t> seen((H.w + 63) / 64, 0);
        uint64_t my_nnr = 0, my_nnc = 0;
        for (uint64_t s = a; s < b; ++s) {
            int64_t r0 = (int64_t)s * H.h, r1 = std::min<int64_t>(n, r0 + H.h);
            used.clear();
            for (int64_t p = row_ptr[r0]; p < row_ptr[r1]; ++p) {
                uint32_t J = (uint32_t)col[p] >> H.wshift;
                if (cnt[J]++ == 0) used.push_back(J);
            }
            std::sort(used.begin(), used.end());
            uint64_t e = (uint64_t)row_ptr[r0];
            uint64_t t = H.slab_tiles[s];
            for (uint32_t J : used) {
                Tile& tl = H.tiles[t++];
                tl.ent_begin = e;
                tl.slab = (uint32_t)s;
                tl.J = J;
                tl.nnz = cnt[J];
                pos[J] = e;
                e += cnt[J];
                cnt[J] = 0;
            }
            for (int64_t r = r0; r < r1; ++r) {
                uint32_t rl = (uint32_t)(r - r0);
                for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
                    uint32_t c = (uint32_t)col[p];
                    uint64_t q = pos[c >> H.wshift]++;
                    H.ent[q] = (rl << 16) | (c & (H.w - 1));
                    if (val) H.val[q] = val[p];
                }
            }
            for (uint64_t ti = H.slab_tiles[s]; ti < H.slab_tiles[s + 1]; ++ti) {
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
                    uint32_t c = E[i] & 0xFFFFu;
                    uint64_t bit = 1ull << (c & 63);
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
    H.sum_nnr = tot_nnr;
    H.sum_nnc = tot_nnc;
    return SPMM_OK;
}

namespace {

struct Seg {
    uint32_t J, row, len;
    uint64_t ent;  // first canonical entry
};

inline uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

struct ChunkOut {
    std::vector<ItemDesc> items;  // blob_off relative to the chunk blob
    std::vector<uint32_t> nnz;
    std::vector<uint8_t> blob;
    uint64_t vt[SPMM_NUM_VARIANTS] = {}, vn[SPMM_NUM_VARIANTS] = {};
};

// Encode one slab into items appended to `out`.
void encode_slab(const Handle& H, uint64_t s, ChunkOut& out, std::vector<uint32_t>& coo_ent,
                 std::vector<float>& coo_val, std::vector<uint32_t>& coo_J,
                 std::vector<Seg>& lr, std::vector<Seg>& wr) {
    coo_ent.clear();
    coo_val.clear();
    coo_J.clear();
    lr.clear();
    wr.clear();
    const bool hv = H.has_val;
    const uint32_t C = H.item_nnz;
    for (uint64_t t = H.slab_tiles[s]; t < H.slab_tiles[s + 1]; ++t) {
        const Tile& tl = H.tiles[t];
        const int v = H.variant[t];
        out.vt[v] += 1;
        out.vn[v] += tl.nnz;
        const uint32_t* E = H.ent.data() + tl.ent_begin;
        uint32_t i = 0;
        while (i < tl.nnz) {
            uint32_t r = E[i] >> 16, j = i;
            while (j < tl.nnz && (E[j] >> 16) == r) ++j;
            uint32_t len = j - i;
            if (v == SPMM_VAR_COO || len == 1) {
                for (uint32_t q = i; q < j; ++q) {
                    coo_ent.push_back(E[q]);
                    if (hv) coo_val.push_back(H.val[tl.ent_begin + q]);
                    coo_J.push_back(tl.J);
                }
            } else if (v == SPMM_VAR_ROW || (v == SPMM_VAR_HYBRID && len < kWaveRowMin)) {
                for (uint32_t q = i; q < j; q += kRowLaneMax)
                    lr.push_back({tl.J, r, std::min(kRowLaneMax, j - q), tl.ent_begin + q});
            } else {
                for (uint32_t q = i; q < j; q += C)
                    wr.push_back({tl.J, r, std::min(C, j - q), tl.ent_begin + q});
            }
            i = j;
        }
    }
    std::stable_sort(lr.begin(), lr.end(), [](const Seg& a, const Seg& b) { return a.len > b.len; });

    // Cut the unit sequence (COO entries, then row segments, then wavefront
    // segments) into items of about C non-zeros.
    struct Range { uint32_t ca, cb, la, lb, wa, wb, nnz; };
    std::vector<Range> ranges;
    Range cur{0, 0, 0, 0, 0, 0, 0};
    auto close = [&]() {
        ranges.push_back(cur);
        cur = {cur.cb, cur.cb, cur.lb, cur.lb, cur.wb, cur.wb, 0};
    };
    const uint32_t nc = (uint32_t)coo_ent.size(), nl = (uint32_t)lr.size(), nw = (uint32_t)wr.size();
    while (cur.cb < nc) {
        uint32_t take = std::min(nc - cur.cb, C - cur.nnz);
        cur.cb += take;
        cur.nnz += take;
        if (cur.nnz >= C) close();
    }
    while (cur.lb < nl) {
        cur.nnz += lr[cur.lb++].len;
        if (cur.nnz >= C) close();
    }
    while (cur.wb < nw) {
        cur.nnz += wr[cur.wb++].len;
        if (cur.nnz >= C) close();
    }
    if (cur.nnz > 0 || ranges.empty()) ranges.push_back(cur);

    std::vector<uint32_t> Js;
    for (const Range& R : ranges) {
        ItemDesc d{};
        d.slab = (uint32_t)s;
        d.part = ranges.size() > 1 ? 0 : -1;  // fixed up globally
        d.n_coo = R.cb - R.ca;
        // strip runs of the COO entries
        uint32_t n_ct = 0;
        for (uint32_t e = R.ca; e < R.cb; ++e)
            if (e == R.ca || coo_J[e] != coo_J[e - 1]) ++n_ct;
        d.n_coo_tiles = n_ct;
        d.n_lr = R.lb - R.la;
        d.n_wr = R.wb - R.wa;
        Js.clear();
        for (uint32_t q = R.la; q < R.lb; ++q) Js.push_back(lr[q].J);
        std::sort(Js.begin(), Js.end());
        Js.erase(std::unique(Js.begin(), Js.end()), Js.end());
        uint32_t n_cols = 0;
        for (uint32_t q = R.la; q < R.lb; ++q) n_cols += lr[q].len;
        for (uint32_t q = R.wa; q < R.wb; ++q) n_cols += wr[q].len;

        uint32_t o = 4 * d.n_coo;
        if (hv) o += 4 * d.n_coo;  // coo_val at 4 * n_coo
        o = align_up(o, 8);
        d.o_coo_tile = o;
        o += 8 * n_ct;
        d.o_lr_desc = o;
        o += 4 * d.n_lr;
        d.o_lr_start = o;
        o += 4 * (d.n_lr + 1);
        d.o_lr_J = o;
        o += 4 * (uint32_t)Js.size();
        o = align_up(o, 16);
        d.o_wr = o;
        o += 16 * d.n_wr;
        d.o_cols = o;
        o += 2 * n_cols;
        o = align_up(o, 4);
        d.o_col_val = o;
        if (hv) o += 4 * n_cols;
        o = align_up(o, 16);

        const uint64_t base = out.blob.size();
        d.blob_off = base;
        out.blob.resize(base + o, 0);
        uint8_t* P = out.blob.data() + base;
        uint32_t* pe = reinterpret_cast<uint32_t*>(P);
        float* pv = reinterpret_cast<float*>(P + 4 * d.n_coo);
        uint32_t* pt = reinterpret_cast<uint32_t*>(P + d.o_coo_tile);
        uint32_t ti = 0;
        for (uint32_t e = R.ca; e < R.cb; ++e) {
            pe[e - R.ca] = coo_ent[e];
            if (hv) pv[e - R.ca] = coo_val[e];
            if (e == R.ca || coo_J[e] != coo_J[e - 1]) {
                pt[2 * ti] = coo_J[e];
                pt[2 * ti + 1] = e - R.ca;
                ++ti;
            }
        }
        uint32_t* pd = reinterpret_cast<uint32_t*>(P + d.o_lr_desc);
        uint32_t* ps = reinterpret_cast<uint32_t*>(P + d.o_lr_start);
        uint32_t* pj = reinterpret_cast<uint32_t*>(P + d.o_lr_J);
        uint32_t* pw = reinterpret_cast<uint32_t*>(P + d.o_wr);
        uint16_t* pc = reinterpret_cast<uint16_t*>(P + d.o_cols);
        float* pcv = reinterpret_cast<float*>(P + d.o_col_val);
        for (size_t q = 0; q < Js.size(); ++q) pj[q] = Js[q];
        uint32_t cpos = 0;
        auto put_cols = [&](const Seg& g) {
            const uint32_t* E = H.ent.data() + g.ent;
            for (uint32_t q = 0; q < g.len; ++q) {
                pc[cpos + q] = (uint16_t)(E[q] & 0xFFFFu);
                if (hv) pcv[cpos + q] = H.val[g.ent + q];
            }
            cpos += g.len;
        };
        for (uint32_t q = R.la; q < R.lb; ++q) {
            const Seg& g = lr[q];
            uint32_t ord = (uint32_t)(std::lower_bound(Js.begin(), Js.end(), g.J) - Js.begin());
            pd[q - R.la] = g.row | (ord << 16);
            ps[q - R.la] = cpos;
            put_cols(g);
        }
        ps[d.n_lr] = cpos;
        for (uint32_t q = R.wa; q < R.wb; ++q) {
            const Seg& g = wr[q];
            uint32_t* w4 = pw + 4 * (q - R.wa);
            w4[0] = g.J;
            w4[1] = g.row;
            w4[2] = cpos;
            w4[3] = g.len;
            put_cols(g);
        }
        out.items.push_back(d);
        out.nnz.push_back(R.nnz);
    }
}

}  // namespace

spmm_status_t encode(Handle& H, std::string& err) {
    const uint64_t S = H.n_slabs;
    const uint64_t chunk = 256;
    const uint64_t nchunks = (S + chunk - 1) / chunk;
    std::vector<ChunkOut> outs(nchunks);
    try {
        parallel_for(nchunks, H.threads, 1, [&](uint64_t a, uint64_t b) {
            std::vector<uint32_t> coo_ent, coo_J;
            std::vector<float> coo_val;
            std::vector<Seg> lr, wr;
            for (uint64_t c = a; c < b; ++c) {
                uint64_t s1 = std::min(S, (c + 1) * chunk);
                for (uint64_t s = c * chunk; s < s1; ++s)
                    encode_slab(H, s, outs[c], coo_ent, coo_val, coo_J, lr, wr);
            }
        });
    } catch (const std::bad_alloc&) {
        err = "out of host memory while encoding tiles";
        return SPMM_ENOMEM;
    }
    Encoded E;
    uint64_t n_items = 0, n_bytes = 0;
    std::vector<uint64_t> item_off(nchunks + 1, 0), byte_off(nchunks + 1, 0);
    for (uint64_t c = 0; c < nchunks; ++c) {
        item_off[c + 1] = item_off[c] + outs[c].items.size();
        byte_off[c + 1] = byte_off[c] + outs[c].blob.size();
        for (int v = 0; v < SPMM_NUM_VARIANTS; ++v) {
            E.variant_tiles[v] += outs[c].vt[v];
            E.variant_nnz[v] += outs[c].vn[v];
        }
    }
    n_items = item_off[nchunks];
    n_bytes = byte_off[nchunks];
    try {
        E.items.resize(n_items);
        E.item_nnz.resize(n_items);
        E.blob.resize(n_bytes);
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
                E.items[item_off[c] + i] = d;
                E.item_nnz[item_off[c] + i] = o.nnz[i];
            }
            std::vector<uint8_t>().swap(o.blob);
        }
    });
    // partial slots for split slabs, in item order
    uint32_t part = 0;
    for (uint64_t i = 0; i < n_items;) {
        uint64_t j = i;
        while (j < n_items && E.items[j].slab == E.items[i].slab) ++j;
        if (j - i > 1) {
            CombineDesc cd{E.items[i].slab, part, part + (uint32_t)(j - i), 0};
            for (uint64_t q = i; q < j; ++q) {
                E.items[q].part = (int32_t)part++;
                E.items[q].cid = (uint32_t)E.combine.size();
            }
            E.combine.push_back(cd);
        } else {
            E.items[i].part = -1;
        }
        i = j;
    }
    E.n_parts = part;
    H.blob_bytes = E.blob.size();
    H.enc = std::move(E);
    return SPMM_OK;
}

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
    const uint8_t* blob = H.enc.blob.empty() ? static_cast<const uint8_t*>(H.h_blob) : H.enc.blob.data();
    if (!blob && !H.enc.items.empty()) {
        err = "no host copy of the tile payload";
        return SPMM_ESTATE;
    }
    struct Trip { int64_t r; int64_t c; float v; };
    std::vector<Trip> out;
    out.reserve((size_t)H.nnz);
    for (const ItemDesc& d : H.enc.items) {
        const uint8_t* base = blob + d.blob_off;
        const int64_t row0 = (int64_t)d.slab * H.h;
        const uint32_t* ent = reinterpret_cast<const uint32_t*>(base);
        const float* cval = reinterpret_cast<const float*>(base + 4 * (size_t)d.n_coo);
        const uint32_t* ct = reinterpret_cast<const uint32_t*>(base + d.o_coo_tile);
        uint32_t ord = 0;
        for (uint32_t e = 0; e < d.n_coo; ++e) {
            while (ord + 1 < d.n_coo_tiles && ct[2 * (ord + 1) + 1] <= e) ++ord;
            int64_t c = ((int64_t)ct[2 * ord] << H.wshift) + (ent[e] & 0xFFFFu);
            out.push_back({row0 + (ent[e] >> 16), c, H.has_val ? cval[e] : 1.0f});
        }
        const uint32_t* ld = reinterpret_cast<const uint32_t*>(base + d.o_lr_desc);
        const uint32_t* ls = reinterpret_cast<const uint32_t*>(base + d.o_lr_start);
        const uint32_t* lj = reinterpret_cast<const uint32_t*>(base + d.o_lr_J);
        const uint16_t* cols = reinterpret_cast<const uint16_t*>(base + d.o_cols);
        const float* cv = reinterpret_cast<const float*>(base + d.o_col_val);
        for (uint32_t s = 0; s < d.n_lr; ++s) {
            int64_t cb = (int64_t)lj[ld[s] >> 16] << H.wshift;
            for (uint32_t t = ls[s]; t < ls[s + 1]; ++t)
                out.push_back({row0 + (ld[s] & 0xFFFFu), cb + cols[t], H.has_val ? cv[t] : 1.0f});
        }
        const uint32_t* wr = reinterpret_cast<const uint32_t*>(base + d.o_wr);
        for (uint32_t q = 0; q < d.n_wr; ++q) {
            const uint32_t* g = wr + 4 * q;
            int64_t cb = (int64_t)g[0] << H.wshift;
            for (uint32_t t = 0; t < g[3]; ++t)
                out.push_back({row0 + g[1], cb + cols[g[2] + t], H.has_val ? cv[g[2] + t] : 1.0f});
        }
    }
    if ((int64_t)out.size() != H.nnz) {
        err = "decoded entry count differs from nnz";
        return SPMM_ESTATE;
    }
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
