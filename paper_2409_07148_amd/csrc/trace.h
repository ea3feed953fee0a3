// Host-side trace ranges (roctx) around the library's entry points, for
// rocprofv3 --marker-trace: set RESTORE_TRACE=1 in the environment before
// the first call.  The roctx library of the ROCm profiler SDK is opened at
// run time on first use, so the library has no link-time dependency on it;
// without the variable, or without that library, a range costs one
// predictable branch.  A range covers the host call (enqueueing its
// launches), not the kernels themselves, which the kernel trace times.
#pragma once

#include <dlfcn.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

namespace restore {

struct RoctxApi {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};

inline const RoctxApi &roctx_api() {
    static RoctxApi api;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *on = getenv("RESTORE_TRACE");
        if (!on || !*on || strcmp(on, "0") == 0) return;
        void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
        if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_GLOBAL);
        if (!h) return;
        auto push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
        auto pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        if (push && pop) {
            api.push = push;
            api.pop = pop;
        }
    });
    return api;
}

// RAII range: pushed on construction, popped on destruction (every return
// path of the entry point closes it).
class TraceRange {
  public:
    explicit TraceRange(const char *name) : api_(roctx_api()) {
        if (api_.push) api_.push(name);
    }
    ~TraceRange() {
        if (api_.pop) api_.pop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;

  private:
    const RoctxApi &api_;
};

}  // namespace restore
