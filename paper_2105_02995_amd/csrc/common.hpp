// Shared host utilities: complex type, error reporting, a small thread pool loop.
#pragma once

#include <cstring>
#include <atomic>
#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <sched.h>
#include <cstdlib>
#include <thread>
#include <vector>

#include "fio.h"

namespace fio {

using cd = std::complex<double>;

// Error carried from deep inside the build to the C ABI boundary.
struct Error : std::runtime_error {
    fio_status status;
    Error(fio_status s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(fio_status s, const std::string &msg) { throw Error(s, msg); }

// Host threads of the build: the request, else OMP_NUM_THREADS, else the CPUs this
// process may run on (its affinity mask, which follows container CPU sets), else the
// hardware count.  Computed once.
inline int hw_threads(int requested) {
    if (requested > 0) return requested;
    static const int dflt = [] {
        if (const char *e = std::getenv("OMP_NUM_THREADS")) {
            const int v = std::atoi(e);
            if (v > 0) return v;
        }
        cpu_set_t set;
        if (sched_getaffinity(0, sizeof(set), &set) == 0) {
            const int c = CPU_COUNT(&set);
            if (c > 0) return c;
        }
        const unsigned h = std::thread::hardware_concurrency();
        return h ? (int)h : 4;
    }();
    return dflt;
}

// Threads currently running parallel_for work (callers included), so that a loop
// nested in another uses only the cores the outer one leaves idle.
inline std::atomic<int> &pool_active() {
    static std::atomic<int> n(0);
    return n;
}
inline bool &pool_member() {
    thread_local bool in = false;
    return in;
}

// Run fn(i) for i in [0, n) on nthreads threads (dynamic scheduling).
template <class Fn>
void parallel_for(int64_t n, int nthreads, Fn &&fn) {
    if (n <= 0) return;
    const int hw = hw_threads(nthreads);
    const int avail = hw - pool_active().load() + (pool_member() ? 1 : 0);
    int nt = (int)std::min<int64_t>(std::min(hw, std::max(1, avail)), n);
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next(0);
    std::exception_ptr err = nullptr;
    std::atomic<bool> failed(false);
    auto work = [&](bool spawned) {
        const bool was = pool_member();
        if (spawned || !was) pool_active().fetch_add(1);
        pool_member() = true;
        try {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n || failed.load()) break;
                fn(i);
            }
        } catch (...) {
            if (!failed.exchange(true)) err = std::current_exception();
        }
        pool_member() = was;
        if (spawned || !was) pool_active().fetch_sub(1);
    };
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int t = 0; t < nt - 1; ++t) th.emplace_back(work, true);
    work(false);
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
}

// parallel_for for the dense kernels of a single large matrix: runs serially when
// the work (in complex multiply-adds) is too small to pay for the threads.
template <class Fn>
void par_cols(int64_t n, double work, Fn &&fn) {
    if (work < 4.0e5 || n < 2) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    parallel_for(n, 0, fn);
}

// 64-bit fingerprint of a run of bytes (multiply-xor over 8-byte words): verbose
// builds print them for the peeled matrix and each inverse-factor step, so two
// builds can be compared.
inline uint64_t fingerprint(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *b = (const unsigned char *)p;
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        std::memcpy(&w, b + i, 8);
        h = (h ^ w) * 0x100000001B3ULL;
        h ^= h >> 29;
    }
    for (; i < bytes; ++i) h = (h ^ b[i]) * 0x100000001B3ULL;
    return h;
}

// Progress line on stderr (build phases); flushed so a watcher sees it at once.
void progress(bool on, const char *fmt, ...);

// splitmix64: the builder's own counter-based generator for random probes.
inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

// Standard normal from two counter values (Box-Muller), deterministic in (seed, k).
inline double gauss(uint64_t seed, uint64_t k) {
    uint64_t a = splitmix64(seed ^ splitmix64(2 * k + 1));
    uint64_t b = splitmix64(seed ^ splitmix64(2 * k + 2));
    double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    double u2 = (b >> 11) * (1.0 / 9007199254740992.0);           // [0, 1)
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace fio
