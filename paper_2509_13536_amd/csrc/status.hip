// Status strings and last-error tracking of the C ABI; the read-back mailbox.
#include <dlfcn.h>

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "api_range.hpp"
#include "common.hpp"

namespace mgs {
namespace {
thread_local char g_last_error[256] = {0};

// roctx entry points, resolved once (both or neither)
int (*g_roctx_push)(const char *) = nullptr;
int (*g_roctx_pop)() = nullptr;
std::once_flag g_roctx_once;
void roctx_init() {
    const char *e = getenv("MGS_ROCTX");
    if (!e || e[0] != '1') return;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_GLOBAL);
    if (!h) return;
    auto push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
    auto pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (push && pop) {
        g_roctx_push = push;
        g_roctx_pop = pop;
    }
}
}  // namespace

bool roctx_push(const char *name) {
    std::call_once(g_roctx_once, roctx_init);
    if (!g_roctx_push) return false;
    g_roctx_push(name);
    return true;
}
void roctx_pop() {
    if (g_roctx_pop) g_roctx_pop();
}
// Owner of a thread's mailbox: allocated on the thread's first call that reads
// a count back, freed when the thread ends.  Every call waits for its own
// ticket before returning, so no kernel writes the words after that.
struct MailboxOwner {
    Mailbox box;
    bool tried = false;
    ~MailboxOwner() {
        if (box.host) {
            (void)hipHostFree(box.host);
            (void)hipGetLastError();
        }
    }
};

Mailbox host_mailbox() {
    thread_local MailboxOwner own;
    if (!own.tried) {
        own.tried = true;
        void *p = nullptr, *d = nullptr;
        if (hipHostMalloc(&p, kMailWords * sizeof(uint32_t),
                          hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent) == hipSuccess &&
            hipHostGetDevicePointer(&d, p, 0) == hipSuccess && d) {
            // the flag starts at 0, a value no ticket takes
            memset(p, 0, kMailWords * sizeof(uint32_t));
            own.box.host = static_cast<uint32_t *>(p);
            own.box.dev = static_cast<uint32_t *>(d);
        } else {
            if (p) (void)hipHostFree(p);
            (void)hipGetLastError();  // leave no error behind for the next call
        }
    }
    return own.box;
}

uint32_t mailbox_ticket() {
    thread_local uint32_t t = 0;
    if (++t == 0) t = 1;  // never 0, the flag's initial value
    return t;
}

hipError_t mailbox_wait(const Mailbox &m, uint32_t ticket, hipStream_t s) {
    const volatile uint32_t *flag = m.host + kMailFlag;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t it = 1;; ++it) {
        if (*flag == ticket) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return hipSuccess;
        }
        if ((it & 4095u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) break;
        __builtin_ia32_pause();
    }
    return hipStreamSynchronize(s);
}

void set_hip_error(hipError_t e) {
    const char *msg = hipGetErrorString(e);
    int i = 0;
    for (; msg && msg[i] && i < 255; ++i) g_last_error[i] = msg[i];
    g_last_error[i] = 0;
}
}  // namespace mgs

extern "C" const char *mgs_status_string(mgs_status status) {
    switch (status) {
        case MGS_OK: return "ok";
        case MGS_ERR_INVALID_ARG: return "invalid argument";
        case MGS_ERR_WORKSPACE: return "workspace too small";
        case MGS_ERR_HIP: return "HIP runtime error";
        case MGS_ERR_TOO_LARGE: return "problem too large";
        case MGS_ERR_SCRATCH: return "input exceeds the fixed scratch of the allocation-free entry point";
        default: return "unknown status";
    }
}

extern "C" const char *mgs_last_hip_error(void) { return mgs::g_last_error; }

extern "C" int32_t mgs_abi_version(void) { return (2 << 16) | 0; }
