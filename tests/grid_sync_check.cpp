// Host-thread check of the device-wide barrier of the persistent step kernel
// (paper_1602_02694_amd/csrc/grid_sync.hpp): the same template, with host
// atomics standing in for the device's.  Exit status 0 when every check holds.
//
//   1. ordering: in every epoch each thread writes its slot, meets the others
//      at a barrier, checks that every slot holds this epoch's value, and
//      meets them again before the next write;
//   2. failure: one thread never arrives; every other thread must leave the
//      barrier with "false" within its poll bound, and the flag must be set.
#include <cstdio>
#include <thread>
#include <vector>

#include "grid_sync.hpp"

struct HostOps {
    static void add_release(unsigned *p, unsigned v) { __atomic_fetch_add(p, v, __ATOMIC_RELEASE); }
    static unsigned load_relaxed(unsigned *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    static void store_relaxed(unsigned *p, unsigned v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    static void acquire() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
    static void pause() { std::this_thread::yield(); }
};

int main()
{
    const unsigned T = 8, E = 3000;
    int bad = 0;
    {
        unsigned count = 0, err = 0;
        std::vector<unsigned> slot(T, 0u);
        std::vector<int> fails(T, 0);
        std::vector<std::thread> th;
        for (unsigned t = 0; t < T; ++t)
            th.emplace_back([&, t] {
                unsigned epoch = 0;
                for (unsigned e = 1; e <= E; ++e) {
                    __atomic_store_n(&slot[t], e, __ATOMIC_RELAXED);
                    if (!wlseno::arrive_and_wait<HostOps>(&count, &err, T, ++epoch, 1u << 30)) ++fails[t];
                    for (unsigned j = 0; j < T; ++j)
                        if (__atomic_load_n(&slot[j], __ATOMIC_RELAXED) != e) ++fails[t];
                    if (!wlseno::arrive_and_wait<HostOps>(&count, &err, T, ++epoch, 1u << 30)) ++fails[t];
                }
            });
        for (auto &x : th) x.join();
        for (unsigned t = 0; t < T; ++t) bad += fails[t];
        if (count != 2 * E * T || err != 0) ++bad;
        std::printf("ordering: %u threads x %u epochs, %d failures, count %u\n", T, E, bad, count);
    }
    {
        unsigned count = 0, err = 0;
        std::vector<int> result(T, -1);
        std::vector<std::thread> th;
        for (unsigned t = 1; t < T; ++t)   // thread 0 never arrives
            th.emplace_back([&, t] { result[t] = wlseno::arrive_and_wait<HostOps>(&count, &err, T, 1, 100000) ? 1 : 0; });
        for (auto &x : th) x.join();
        int left = 0;
        for (unsigned t = 1; t < T; ++t) left += result[t] == 0;
        std::printf("failure: %d of %u waiting threads left with false, flag %u\n", left, T - 1, err);
        if (left != (int)T - 1 || err != 1) ++bad;
    }
    return bad == 0 ? 0 : 1;
}
