// api.hpp -- exception barrier of the C ABI (internal to libltsim).  No C++ exception may leave an extern "C"
// entry point: each one's body runs inside LTS_API_BEGIN / LTS_API_END, which turns a host allocation failure into
// LTS_ERR_OOM and any other exception into LTS_ERR_DEVICE with a message.  Neither is made sticky: the device state
// of the object is untouched by a host-side failure, so the caller may retry.
#pragma once

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>

#include "../../include/ltsim.h"

namespace ltsim {

template <class Obj>
lts_status api_fail(Obj *o, lts_status s, const char *msg) noexcept {
    if (o) {
        try {
            o->err = msg;
        } catch (...) {
        }
    }
    return s;
}
inline lts_status api_fail(std::nullptr_t, lts_status s, const char *) noexcept { return s; }

// Test hook behind lts_debug_fail_host_alloc: countdown to an injected host allocation failure (-1 = off).
extern std::atomic<int64_t> g_host_alloc_fail;

// A point where the library allocates host memory; throws std::bad_alloc when the test hook's countdown hits it.
inline void host_alloc_point() {
    if (g_host_alloc_fail.load(std::memory_order_relaxed) < 0) return;
    if (g_host_alloc_fail.fetch_sub(1) == 0) throw std::bad_alloc();
}

}  // namespace ltsim

#define LTS_API_BEGIN try {
#define LTS_API_END(obj)                                                                                    \
    }                                                                                                       \
    catch (const std::bad_alloc &) {                                                                        \
        return ::ltsim::api_fail((obj), LTS_ERR_OOM, "host memory allocation failed");                      \
    }                                                                                                       \
    catch (const std::exception &e_) {                                                                      \
        return ::ltsim::api_fail((obj), LTS_ERR_DEVICE, e_.what());                                         \
    }                                                                                                       \
    catch (...) {                                                                                           \
        return ::ltsim::api_fail((obj), LTS_ERR_DEVICE, "unknown C++ exception");                           \
    }
