// gfq_drain.h -- the loop of a persistent workgroup draining a queue of work items.
//
// One code path for the device and for a host model: the device kernel instantiates it with
// the workgroup's barrier, an LDS word and a device-memory head counter; the host check
// (tests/drain_host_check.cpp) instantiates it with threads, a barrier of its own and an
// atomic, and runs it under ThreadSanitizer.  The properties the loop keeps, whoever runs it:
//   - the leader (one thread on the host; on the device the whole first wave, chosen by a
//     branch that is uniform in every wave) takes the next item index (an atomic
//     fetch-and-add of 1 on the queue head) and publishes it in workgroup-shared memory;
//     every thread reads it only after a barrier, and the slot is written again only after
//     a second barrier that follows every read;
//   - no branch inside the loop is taken by some threads of a wave and not by others around
//     a barrier: a branch at the loop's head that only one lane takes lets the compiler give
//     the other lanes a shorter path back to the first barrier, so that they loop on a stale
//     slot while the lane that must fetch the next index waits for them (what a first draft
//     of this loop compiled to, and the likely cause of an earlier version's hang);
//   - the index every thread acts on is one value for the whole workgroup (the device takes
//     it through readfirstlane, so the compiler knows it is uniform), so the exit test and
//     every barrier inside the item are reached by all threads of the workgroup or by none;
//   - every pass of the loop advances the head by one, so after (items + workgroups) fetches
//     every workgroup has exited: no pass waits on another workgroup.
// Ctx provides: leader() (uniform per wave), barrier(), fetch_head() (called by every
// leader thread: one atomic add of 1, the old value returned to all of them), slot_store(u32)
// (every leader thread stores the same value), slot_load(), uniform(u32), and run(item) (the
// item's work: it may call barrier() any number of times, the same number in every thread).
#pragma once
#include <stdint.h>

#ifndef GFQ_DRAIN_FN
#define GFQ_DRAIN_FN inline
#endif

namespace gfq {

template <class Ctx>
GFQ_DRAIN_FN void drain_queue(Ctx &c, uint32_t items) {
    for (;;) {
        if (c.leader()) c.slot_store(c.fetch_head());
        c.barrier();                             // the slot holds this pass's index
        const uint32_t it = c.uniform(c.slot_load());
        c.barrier();                             // every thread has read it
        if (it >= items) break;
        c.run(it);
    }
}

}  // namespace gfq
