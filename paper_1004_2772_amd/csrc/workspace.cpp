// Per-device workspace of the synchronous library calls: one device region
// and one pinned host region, grown on demand (to the next power of two) and
// kept for later calls, so that a call costs no allocation once warm.  A
// call holds the device's lock for as long as it uses the regions.  The
// regions live until the process ends.
#include <map>
#include <memory>
#include <mutex>

#include "internal.h"

namespace lhs {

namespace {
std::mutex g_map_mu;
std::map<int, std::unique_ptr<Workspace>> g_ws;

size_t grow_to(size_t want) {
    size_t c = 1 << 20;
    while (c < want)
        c <<= 1;
    return c;
}
}  // namespace

Workspace &workspace(int device) {
    std::lock_guard<std::mutex> lk(g_map_mu);
    auto &p = g_ws[device];
    if (!p)
        p.reset(new Workspace());
    return *p;
}

lhs_status ws_reserve(Workspace &w, size_t dev_bytes, size_t host_bytes) {
    if (dev_bytes > w.dev_bytes) {
        if (w.dev) {
            if (hipDeviceSynchronize() != hipSuccess)
                return LHS_EDEVICE;
            (void)hipFree(w.dev);
            w.dev = nullptr;
            w.dev_bytes = 0;
        }
        const size_t c = grow_to(dev_bytes);
        if (hipMalloc(&w.dev, c) != hipSuccess) {
            (void)hipGetLastError();
            w.dev = nullptr;
            return LHS_ENOMEM;
        }
        w.dev_bytes = c;
    }
    if (host_bytes > w.host_bytes) {
        if (w.host) {
            (void)hipHostFree(w.host);
            w.host = nullptr;
            w.host_bytes = 0;
        }
        const size_t c = grow_to(host_bytes);
        if (hipHostMalloc(&w.host, c, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            w.host = nullptr;
            return LHS_ENOMEM;
        }
        w.host_bytes = c;
    }
    if (!w.ev[0] && (hipEventCreate(&w.ev[0]) != hipSuccess || hipEventCreate(&w.ev[1]) != hipSuccess))
        return LHS_EDEVICE;
    return LHS_OK;
}

}  // namespace lhs
