// Arrival-counter barrier of the persistent step kernel, written once for the
// device and for a host-thread check of the same logic.
//
// Every participant (one per workgroup on the device) adds 1 to *count on
// arrival at barrier number `epoch` (1, 2, ...) and may go on once *count has
// reached epoch * n.  The counter only grows, so no reset races with late
// readers.  Polling is bounded: after max_polls polls a participant sets *err
// and leaves, and one that finds *err set leaves at once, so every
// participant ends whatever happens to the others; the caller then reports
// the failure.  Ops supplies the atomics (release add, relaxed load and
// store, acquire fence) and a pause between polls.  Polls are relaxed loads
// and one acquire fence follows the last: on the GPU an acquire invalidates
// the cache that other workgroups are still working from.
#pragma once

#ifndef WLSENO_HD
#define WLSENO_HD
#endif

namespace wlseno {

template <class Ops>
WLSENO_HD inline bool arrive_and_wait(unsigned *count, unsigned *err, unsigned n, unsigned epoch, unsigned max_polls)
{
    Ops::add_release(count, 1u);
    const unsigned target = epoch * n;
    for (unsigned polls = 0;; ++polls) {
        // wrap-safe "count >= target"
        if ((int)(Ops::load_relaxed(count) - target) >= 0) {
            Ops::acquire();
            return true;
        }
        if (Ops::load_relaxed(err) != 0u) return false;
        if (polls >= max_polls) {
            Ops::store_relaxed(err, 1u);
            return false;
        }
        Ops::pause();
    }
}

}  // namespace wlseno
