// Queue launch of a batch pass: every layer of every matrix of the batch (Alg. 2 applied to each
// matrix) in one kernel launch, instead of one grouped launch per layer.
//
// Work items are (matrix, upper tile, layer). Each matrix belongs to one XCD; XCD x's items form
// its own queue, ordered layer-major (all items of layer 0 of its matrices, then layer 1, ...).
// The launch has one workgroup per item and queue slot; a workgroup reads its XCD from the
// hardware and takes the next ticket of that queue. Item (m, t, l) starts once matrix m has
// completed l x (tiles of m) items, i.e. its whole layer l - 1. Every wait is on items of smaller
// tickets of the same queue, each held by a running workgroup (a ticket is taken only by a
// running workgroup, which holds it until that item is done), so the smallest unfinished ticket
// can always proceed: no deadlock, whatever the number of resident workgroups. A matrix's
// producers and consumers share one L2 (its XCD's), so a hand-off needs the producer's stores to
// have completed (they are then in that L2) and the consumer CU's L1 to be invalidated (one
// invalidate per workgroup); no L2 write-back is involved.
#pragma once

#include "fe_internal.h"

namespace fe {

struct BatchQueue {
    const int4* items;      // per queue, in ticket order: {matrix, tile, layer, need}; need =
                            // layer x (upper tiles of the matrix)
    const int32_t* qoff;    // [nq + 1]: queue x holds items[qoff[x] .. qoff[x + 1])
    int nq;                 // queues, one per XCD
    int32_t* ticket;        // [nq] next ticket of each queue
    int32_t* done;          // [count] completed items per matrix
    int32_t* err;           // [count + 1]: a wait of that matrix gave up; [count]: abort flag
    int spin_limit;         // polls before a wait gives up
    int need_offset;        // added to every item's need: 0, or (to test the give-up path) a
                            // count no matrix reaches
};
// Integers of one pass's counters (ticket, done, err and the abort flag) for `count` matrices;
// ticket, done and err are consecutive in that order.
inline int64_t batch_queue_counters(int nq, int count) { return nq + 2 * (int64_t)count + 1; }

// Zeroes Q's counters (a kernel, so that the plan's captured graph holds no memset node).
hipError_t launch_batch_queue_reset(const BatchQueue& Q, int count, hipStream_t s);
// One pass over every layer of every matrix (q.layer, q.parity and q.map unused) on `grid`
// workgroups: the number of queues times the longest queue (the hardware deals consecutive
// workgroups to consecutive XCDs, so each XCD gets the same number).
hipError_t launch_batch_queue(const BatchLayerArgs& q, const BatchQueue& Q, int64_t grid, int bf16,
                              int tile, hipStream_t s);
// Whether the queue launch's assumptions hold on the current device with nq XCDs: consecutive
// workgroups run on consecutive XCDs (round-robin, from whichever XCD the dispatch starts at), and
// each reads its XCD's id from the hardware (a probe launch; synchronizes).
hipError_t batch_queue_probe(int nq, bool* ok);
// After the pass: a matrix whose items did not all complete, or one of whose waits gave up,
// gets status FE_ERR_HIP (its traces then become NaN in the reduction).
hipError_t launch_batch_queue_check(const BatchMat* mats, int count, const BatchQueue& Q,
                                    BatchCoef cf, Params* P, int tile, hipStream_t s);

}  // namespace fe
