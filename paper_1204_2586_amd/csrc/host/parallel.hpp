// Host worker threads of the setup passes.  Every parallel pass produces
// exactly the result of the sequential one (disjoint outputs, sums kept in
// their sequential order).
#pragma once

#include <algorithm>
#include <cstdlib>
#include <exception>
#include <thread>
#include <vector>

namespace auxp {

// Host threads for a setup pass over `work` items: up to 16 (or the
// AUXPREC_SETUP_THREADS environment variable, if set), one per 64K items.
inline int setup_threads(size_t work)
{
    const unsigned hw = std::thread::hardware_concurrency();
    size_t n = std::min<size_t>(hw ? hw : 1, 16);
    if (const char *env = std::getenv("AUXPREC_SETUP_THREADS")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v >= 1) n = (size_t)std::min<long>(v, 64);
    }
    return (int)std::max<size_t>(1, std::min(n, work / 65536));
}

// f(task) for task in [0, ntask), one thread each.  An exception thrown by a
// task (e.g. std::bad_alloc) is kept, every started thread is joined, and the
// first task's exception in task order is rethrown on the calling thread; if a
// thread cannot be started, the remaining tasks run on the calling thread.
template <typename F>
void run_tasks(int ntask, F f)
{
    if (ntask == 1) {
        f(0);
        return;
    }
    std::vector<std::exception_ptr> err((size_t)ntask);
    auto body = [&](int i) {
        try {
            f(i);
        } catch (...) {
            err[i] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve(ntask);
    int started = 0;
    try {
        for (; started < ntask; started++) th.emplace_back(body, started);
    } catch (...) {
        // no further threads (std::system_error): run the rest here
    }
    for (int i = started; i < ntask; i++) body(i);
    for (std::thread &t : th) t.join();
    for (const std::exception_ptr &e : err)
        if (e) std::rethrow_exception(e);
}

}  // namespace auxp
