// roctx ranges around the entry points of the C ABI (host code).
#pragma once

namespace mgs {

// With MGS_ROCTX=1 in the environment, every entry point of the C ABI opens a
// roctx range named after itself for the time of the call, so that
// `rocprofv3 --marker-trace` shows the host side of each call beside its
// kernels.  The roctx library is looked up once per process (dlopen); when it
// is absent, or the variable is unset, a range costs one check.
bool roctx_push(const char *name);
void roctx_pop();
struct ApiRange {
    bool on;
    explicit ApiRange(const char *name) : on(roctx_push(name)) {}
    ~ApiRange() {
        if (on) roctx_pop();
    }
    ApiRange(const ApiRange &) = delete;
    ApiRange &operator=(const ApiRange &) = delete;
};

}  // namespace mgs
