// Device allocations of the library: hipMalloc/hipFree, or the caller's
// allocator (pxSetAllocator), e.g. a framework's caching allocator, so that
// the solver's memory shows up in the caller's accounting and is reused by it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "px_internal.h"

namespace px {
namespace {

struct Hook {
    pxDeviceAllocFn alloc = nullptr;
    pxDeviceFreeFn free = nullptr;
    void* user = nullptr;
};

struct Owner {
    Hook hook;   // alloc == nullptr: hipMalloc
    int dev;
};

std::mutex g_mu;
Hook g_hook;
std::unordered_map<void*, Owner>* g_live = new std::unordered_map<void*, Owner>();   // never destroyed

}  // namespace

bool caller_allocator()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_hook.alloc != nullptr;
}

void set_allocator(pxDeviceAllocFn alloc, pxDeviceFreeFn free, void* user)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_hook = Hook{alloc, free, user};
}

hipError_t dev_malloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Hook h;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        h = g_hook;
    }
    if (!h.alloc) {
        e = hipMalloc(p, bytes);
        if (e != hipSuccess) return e;
    } else {
        void* q = h.alloc(bytes, dev, h.user);
        if (!q) return hipErrorOutOfMemory;
        // the block may have been in use by the caller's own work on another
        // stream until just now: the library's streams start after it
        e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            h.free(q, dev, h.user);
            return e;
        }
        *p = q;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    (*g_live)[*p] = Owner{h, dev};
    return hipSuccess;
}

void dev_free(void* p)
{
    if (!p) return;
    Owner o{};
    bool known = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_live->find(p);
        if (it != g_live->end()) {
            o = it->second;
            known = true;
            g_live->erase(it);
        }
    }
    if (!known || !o.hook.alloc) {
        (void)hipFree(p);
        return;
    }
    // as hipFree: no stream of the library may still use the block
    (void)hipDeviceSynchronize();
    o.hook.free(p, o.dev, o.hook.user);
}

}  // namespace px
