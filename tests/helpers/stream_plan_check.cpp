// Host check of the streamed-SpMM ring ordering (csrc/stream_plan.h).
//
// The plan is run against a recorder instead of HIP.  Every enqueued
// operation gets a vector clock over the streams (copy, compute, and the
// output stream of the Y-out plan): an
// operation on a stream follows everything earlier on that stream, an event
// record snapshots the stream's clock, and a wait merges the snapshot of the
// event's latest record into the waiting stream (a wait on an event never
// recorded orders nothing).  Then:
//   * every copy into a slot must come after every kernel launch that read
//     the slot earlier in host order (else the copy engine may overwrite a
//     group that a kernel is still decoding);
//   * every launch must come after the copy of its own group;
//   * with Y streamed out, every launch must also come after the earlier
//     copy-outs of its Y slot, and every copy-out after its group's launch.
// stream_plan_violations() runs `calls` back-to-back calls of the library's
// plan; legacy_plan_violations() runs a plan that waits for a slot only when
// g >= R within a call, the ordering the ring had before it kept the "slot
// used" state across calls, to show that the check catches that mistake.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "stream_plan.h"

namespace {

struct Op {
    int stream;          // 0 copy, 1 compute, 2 output
    int kind;            // 0 copy in, 1 launch, 2 copy out
    uint32_t slot;
    uint64_t group;
    uint64_t vc[3];
};

using Clock = std::vector<uint64_t>;

struct Clocked {
    Clock vc[3] = {Clock(3, 0), Clock(3, 0), Clock(3, 0)};  // vc[stream] = that stream's vector clock
    std::vector<Clock> ev_ready, ev_free, ev_y_ready, ev_y_free;  // empty = never recorded
    std::vector<Op> ops;
    explicit Clocked(uint32_t R) : ev_ready(R), ev_free(R), ev_y_ready(R), ev_y_free(R) {}
    void op(int s, int kind, uint32_t slot, uint64_t g) {
        ++vc[s][s];
        ops.push_back(Op{s, kind, slot, g, {vc[s][0], vc[s][1], vc[s][2]}});
    }
    void record(int s, Clock& ev) { ev = vc[s]; }
    void wait(int s, const Clock& ev) {
        if (ev.empty()) return;
        for (int i = 0; i < 3; ++i) vc[s][i] = std::max(vc[s][i], ev[i]);
    }
    // the Ops interface of run_stream_plan / run_stream_plan_yout
    bool wait_free(uint32_t s) { wait(0, ev_free[s]); return true; }
    bool copy(uint64_t g, uint32_t s) { op(0, 0, s, g); return true; }
    bool record_ready(uint32_t s) { record(0, ev_ready[s]); return true; }
    bool wait_ready(uint32_t s) { wait(1, ev_ready[s]); return true; }
    bool launch(uint64_t g, uint32_t s) { op(1, 1, s, g); return true; }
    bool record_free(uint32_t s) { record(1, ev_free[s]); return true; }
    bool wait_y_free(uint32_t s) { wait(1, ev_y_free[s]); return true; }
    bool record_y_ready(uint32_t s) { record(1, ev_y_ready[s]); return true; }
    bool wait_y_ready(uint32_t s) { wait(2, ev_y_ready[s]); return true; }
    bool copy_out(uint64_t g, uint32_t s) { op(2, 2, s, g); return true; }
    bool record_y_free(uint32_t s) { record(2, ev_y_free[s]); return true; }
};

bool hb(const Op& a, const Op& b) { return a.vc[a.stream] <= b.vc[a.stream]; }

// Violations of the ordering rules over the recorded operations:
//   a copy into an A slot follows every launch that read the slot before;
//   a launch follows the copy of its own group into its A slot, and every
//     copy-out of its Y slot issued before it;
//   a copy-out follows the launch of its own group (the latest launch that
//     wrote its Y slot).
int count_violations(const std::vector<Op>& ops) {
    int bad = 0;
    for (size_t j = 0; j < ops.size(); ++j) {
        const Op& b = ops[j];
        if (b.kind == 0) {
            for (size_t i = 0; i < j; ++i)
                if (ops[i].kind == 1 && ops[i].slot == b.slot && !hb(ops[i], b)) ++bad;
        } else if (b.kind == 1) {
            bool found = false;
            for (size_t i = j; i-- > 0;)
                if (ops[i].kind == 0 && ops[i].slot == b.slot) {
                    found = true;
                    if (ops[i].group != b.group || !hb(ops[i], b)) ++bad;
                    break;
                }
            if (!found) ++bad;
            for (size_t i = 0; i < j; ++i)
                if (ops[i].kind == 2 && ops[i].slot == b.slot && !hb(ops[i], b)) ++bad;
        } else {
            bool found = false;
            for (size_t i = j; i-- > 0;)
                if (ops[i].kind == 1 && ops[i].slot == b.slot) {
                    found = true;
                    if (ops[i].group != b.group || !hb(ops[i], b)) ++bad;
                    break;
                }
            if (!found) ++bad;
        }
    }
    return bad;
}

}  // namespace

extern "C" int stream_plan_violations(uint64_t n_groups, uint32_t R, int calls) {
    Clocked rec(R);
    std::vector<uint8_t> used(R, 0);
    for (int c = 0; c < calls; ++c)
        if (!spmm::run_stream_plan(n_groups, R, used.data(), rec)) return -1;
    return count_violations(rec.ops);
}

extern "C" int yout_plan_violations(uint64_t n_groups, uint32_t R, int calls) {
    Clocked rec(R);
    std::vector<uint8_t> used(R, 0), y_used(R, 0);
    for (int c = 0; c < calls; ++c)
        if (!spmm::run_stream_plan_yout(n_groups, R, used.data(), y_used.data(), rec)) return -1;
    return count_violations(rec.ops);
}

// The Y-out plan without the wait for a Y slot's previous copy-out: the
// kernels may overwrite rows the output stream has not copied yet.
extern "C" int yout_nowait_plan_violations(uint64_t n_groups, uint32_t R, int calls) {
    Clocked rec(R);
    std::vector<uint8_t> used(R, 0);
    for (int c = 0; c < calls; ++c)
        for (uint64_t g = 0; g < n_groups; ++g) {
            const uint32_t s = (uint32_t)(g % R);
            if (used[s]) rec.wait_free(s);
            rec.copy(g, s);
            rec.record_ready(s);
            rec.wait_ready(s);
            rec.launch(g, s);
            rec.record_free(s);
            rec.record_y_ready(s);
            rec.wait_y_ready(s);
            rec.copy_out(g, s);
            rec.record_y_free(s);
            used[s] = 1;
        }
    return count_violations(rec.ops);
}

extern "C" int legacy_plan_violations(uint64_t n_groups, uint32_t R, int calls) {
    Clocked rec(R);
    for (int c = 0; c < calls; ++c)
        for (uint64_t g = 0; g < n_groups; ++g) {
            const uint32_t s = (uint32_t)(g % R);
            if (g >= R) rec.wait_free(s);
            rec.copy(g, s);
            rec.record_ready(s);
            rec.wait_ready(s);
            rec.launch(g, s);
            rec.record_free(s);
        }
    return count_violations(rec.ops);
}
