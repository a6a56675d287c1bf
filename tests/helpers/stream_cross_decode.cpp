// What a kernel of streamed mode gathers when its ring slot holds the wrong
// transfer group (test infrastructure; no device code).
//
// The library's builder (csrc/builder.cpp) is compiled with g++ against the
// host stand-in of the HIP headers: it tiles a CSR, encodes the work items
// and cuts them into transfer groups exactly as for spmm_stream_run.  The
// helper then walks one group's items the way the SpMM kernel reads them --
// COO entries with their strip table, row-lane segments, wavefront segments
// -- from a slot image: the group's own payload, or another group's payload
// as left in the slot by a copy that overtook the kernel.  It counts the X
// rows each read would gather that lie outside X, and reads that fall outside
// the slot's bytes.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "spmm_internal.h"

namespace {

// Segment lengths read from a wrong payload can be anything: walk at most
// this many elements of one segment (the kernel would walk all of them).
constexpr uint32_t kWalkCap = 1u << 16;

struct Counts {
    uint64_t gathers = 0, x_out = 0, payload_out = 0;
};

// Items [i0, i1) decoded against slot bytes S (the kernel addresses item d's
// payload at S + d.blob_off - b0, where b0 is the first byte of the group
// the launch was issued for).
Counts walk(const spmm::Handle& H, uint64_t i0, uint64_t i1, uint64_t b0, const std::vector<uint8_t>& S) {
    Counts c;
    auto rd32 = [&](uint64_t off, uint32_t& v) {
        if (off + 4 > S.size()) { ++c.payload_out; v = 0; return; }
        std::memcpy(&v, S.data() + off, 4);
    };
    auto rd16 = [&](uint64_t off, uint32_t& v) {
        if (off + 2 > S.size()) { ++c.payload_out; v = 0; return; }
        uint16_t t;
        std::memcpy(&t, S.data() + off, 2);
        v = t;
    };
    auto gather = [&](uint64_t J, uint32_t col) {
        ++c.gathers;
        const uint64_t xr = (J << H.wshift) + col;
        if (xr >= (uint64_t)H.n_cols) ++c.x_out;
    };
    for (uint64_t it = i0; it < i1; ++it) {
        const spmm::ItemDesc& d = H.enc.items[it];
        const spmm::ItemLayout L = spmm::item_layout(d, H.has_val);
        const uint64_t base = d.blob_off - b0;
        // COO: an entry's strip is the table entry of its run (run starts
        // flagged in bit 31, counted from the item's first entry)
        int64_t seen = 0;
        for (uint32_t e = 0; e < d.n_coo; ++e) {
            uint32_t en;
            rd32(base + 4ull * e, en);
            if (en & spmm::kCooNewTile) ++seen;
            const int64_t ord = std::max<int64_t>(seen - 1, 0);
            uint32_t J;
            rd32(base + L.o_coo_J + 4ull * (uint64_t)ord, J);
            gather(J, en & 0xFFFFu);
        }
        // row-lane segments
        for (uint32_t q = 0; q < d.n_lr; ++q) {
            uint32_t sx, sy, J;
            rd32(base + L.o_lr + 8ull * q, sx);
            rd32(base + L.o_lr + 8ull * q + 4, sy);
            rd32(base + L.o_lr_J + 4ull * (sx >> 12), J);
            const uint32_t len = sy >> spmm::kLrStartBits, start = sy & ((1u << spmm::kLrStartBits) - 1);
            for (uint32_t t = 0; t < std::min(len, kWalkCap); ++t) {
                uint32_t col;
                rd16(base + L.o_cols + 2ull * (start + 64ull * t), col);
                gather(J, col);
            }
        }
        // wavefront segments {strip, row, first column slot, length}
        for (uint32_t q = 0; q < d.n_wr; ++q) {
            uint32_t J, first, len;
            rd32(base + L.o_wr + 16ull * q, J);
            rd32(base + L.o_wr + 16ull * q + 8, first);
            rd32(base + L.o_wr + 16ull * q + 12, len);
            for (uint32_t t = 0; t < std::min(len, kWalkCap); ++t) {
                uint32_t col;
                rd16(base + L.o_cols + 2ull * ((uint64_t)first + t), col);
                gather(J, col);
            }
        }
    }
    return c;
}

}  // namespace

// out[0..2]: gathers, X rows out of range, payload reads out of the slot for
// group `ga` decoded against its own payload; out[3..5]: the same against
// group `gb`'s payload.  Returns the number of groups, or -1 on error.
extern "C" int64_t cross_decode(int64_t n, const int64_t* row_ptr, const int32_t* col, uint32_t tile_rows,
                                uint32_t item_nnz, uint64_t stream_bytes, int64_t ga, int64_t gb, uint64_t* out) {
    spmm::Handle H;
    H.n_rows = H.n_cols = n;
    H.h = tile_rows;
    H.w = 65536;
    H.item_nnz = item_nnz;
    H.threads = 1;
    H.relabel = true;
    H.max_kc = 32;
    std::string err;
    if (spmm::build_canonical(H, row_ptr, col, nullptr, true, err) != SPMM_OK) return -1;
    if (spmm::encode(H, err) != SPMM_OK) return -1;
    const auto groups = spmm::make_groups(H.enc, stream_bytes, H.h);
    const int64_t ng = (int64_t)groups.size();
    if (ga < 0 || gb < 0 || ga >= ng || gb >= ng) return ng;
    uint64_t slot = 16;
    for (const auto& g : groups) slot = std::max<uint64_t>(slot, g.b1 - g.b0);
    auto image = [&](int64_t g) {
        std::vector<uint8_t> S(slot, 0);
        std::memcpy(S.data(), H.enc.blob.data() + groups[g].b0, groups[g].b1 - groups[g].b0);
        return S;
    };
    const auto& A = groups[ga];
    const Counts own = walk(H, A.i0, A.i1, A.b0, image(ga));
    const Counts other = walk(H, A.i0, A.i1, A.b0, image(gb));
    out[0] = own.gathers;
    out[1] = own.x_out;
    out[2] = own.payload_out;
    out[3] = other.gathers;
    out[4] = other.x_out;
    out[5] = other.payload_out;
    return ng;
}
