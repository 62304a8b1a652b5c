// Optional host-side ranges for profiling (FEWHA_TRACE=1 in the environment): the library's
// enqueueing calls and, inside a solve, the right-hand side, every PCG pass and the last pass's
// coarse levels are bracketed by roctx ranges, which `rocprofv3 --marker-trace` records beside the
// kernels.  The roctx library is opened on the first range (no link-time dependency); without it,
// or without the variable, a range costs one branch.  Ranges mark when work is enqueued; during
// HIP graph capture they mark the capture, not the replays.
#pragma once

#include <dlfcn.h>

#include <cstdlib>

namespace fewha {
namespace trace {

struct Fns {
    int (*push)(const char *);
    int (*pop)();
};

inline const Fns &fns() {
    static const Fns f = [] {
        Fns r{nullptr, nullptr};
        const char *e = std::getenv("FEWHA_TRACE");
        if (!e || !*e || (e[0] == '0' && !e[1])) return r;
        void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
        if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
        if (!h) return r;
        r.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
        r.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        if (!r.push || !r.pop) r = Fns{nullptr, nullptr};
        return r;
    }();
    return f;
}

// One range for the lifetime of the object (names must outlive it: string literals).
class Range {
  public:
    explicit Range(const char *name) : on_(fns().push != nullptr) {
        if (on_) fns().push(name);
    }
    ~Range() {
        if (on_) fns().pop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

  private:
    bool on_;
};

// Whether ranges are recorded (FEWHA_TRACE set and roctx found).
inline bool enabled() { return fns().push != nullptr; }

}  // namespace trace
}  // namespace fewha
