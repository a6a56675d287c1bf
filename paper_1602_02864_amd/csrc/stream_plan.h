// Ordering plan of one streamed SpMM call (the device analogue of
// Algorithm 1's asynchronous read of the next tile rows before they are
// multiplied, Section 3.1 and 3.5).
//
// The tile payload sits in pinned host memory, cut into transfer groups
// 0..G-1.  Group g is copied into ring slot g mod R on the copy stream and
// read there by the SpMM kernels on the compute stream.  Two events per
// slot carry the ordering between the streams:
//   ready[s]  recorded on the copy stream after a copy into s; the compute
//             stream waits for it before the kernels that read s;
//   free[s]   recorded on the compute stream after those kernels; the copy
//             stream waits for it before the next copy into s.
// used[s] says that free[s] holds a record, i.e. some kernel has read s, in
// this call or an earlier one.  It must persist across calls: the first R
// copies of a call overwrite slots that the previous call's last kernels may
// still be reading, so they wait on free[s] too.  (Waiting only for g >= R,
// as if every call started with an idle ring, lets the copy engine
// overwrite a slot under a running kernel, which then decodes another
// group's strip and column ids and gathers X out of range.)
//
// The plan is a template over the operations so that the host library runs
// it with HIP calls and a CPU test runs it with a recorder that checks the
// happens-before relation of every copy and every kernel.
#pragma once

#include <cstdint>

namespace spmm {

// Ops must provide (each returning true on success):
//   wait_free(slot)        copy stream waits for free[slot]
//   copy(group, slot)      enqueue the host->device copy of group into slot
//   record_ready(slot)     record ready[slot] on the copy stream
//   wait_ready(slot)       compute stream waits for ready[slot]
//   launch(group, slot)    enqueue the SpMM kernels of group, reading slot
//   record_free(slot)      record free[slot] on the compute stream
// used has R entries and is updated in place.
template <class Ops>
bool run_stream_plan(uint64_t n_groups, uint32_t R, uint8_t* used, Ops& ops) {
    for (uint64_t g = 0; g < n_groups; ++g) {
        const uint32_t slot = (uint32_t)(g % R);
        if (used[slot] && !ops.wait_free(slot)) return false;
        if (!ops.copy(g, slot) || !ops.record_ready(slot) || !ops.wait_ready(slot)) return false;
        if (!ops.launch(g, slot) || !ops.record_free(slot)) return false;
        used[slot] = 1;
    }
    return true;
}

// The same plan with Y streamed out as well (Algorithm 1's asynchronous
// write of finished output rows): the kernels of group g write its rows of
// Y into Y slot g mod R, and a third stream copies that slot to host memory.
// Two more events per slot:
//   y_ready[s]  recorded on the compute stream after the kernels that wrote
//               Y slot s; the output stream waits for it before copying out;
//   y_free[s]   recorded on the output stream after that copy; the compute
//               stream waits for it before kernels write the slot again.
// Ops also provides wait_y_free(slot) [compute], record_y_ready(slot)
// [compute], wait_y_ready(slot) [output], copy_out(group, slot) [output] and
// record_y_free(slot) [output]; y_used persists across calls like used.
template <class Ops>
bool run_stream_plan_yout(uint64_t n_groups, uint32_t R, uint8_t* used, uint8_t* y_used, Ops& ops) {
    for (uint64_t g = 0; g < n_groups; ++g) {
        const uint32_t slot = (uint32_t)(g % R);
        if (used[slot] && !ops.wait_free(slot)) return false;
        if (!ops.copy(g, slot) || !ops.record_ready(slot) || !ops.wait_ready(slot)) return false;
        if (y_used[slot] && !ops.wait_y_free(slot)) return false;
        if (!ops.launch(g, slot) || !ops.record_free(slot) || !ops.record_y_ready(slot)) return false;
        if (!ops.wait_y_ready(slot) || !ops.copy_out(g, slot) || !ops.record_y_free(slot)) return false;
        used[slot] = 1;
        y_used[slot] = 1;
    }
    return true;
}

}  // namespace spmm
