// Device memory of the library: hipMalloc / hipFree, or a caller's allocator
// installed with pfe_set_allocator (for example a caching allocator that owns
// the process's device memory).  Every device allocation of the library goes
// through dev_alloc / dev_free (or their stream-ordered forms for temporaries
// inside one call); a count of live allocations keeps the allocator from being
// switched while memory from the other one is still out.
#include <atomic>
#include <mutex>

#include "common.hpp"

namespace pfe {

namespace {
std::mutex g_mu;
pfe_alloc_fn g_alloc = nullptr;
pfe_free_fn g_free = nullptr;
void* g_user = nullptr;
std::atomic<long long> g_live{0};

void current(pfe_alloc_fn& a, pfe_free_fn& f, void*& u) {
    std::lock_guard<std::mutex> lock(g_mu);
    a = g_alloc;
    f = g_free;
    u = g_user;
}
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
    pfe_alloc_fn a;
    pfe_free_fn f;
    void* u;
    current(a, f, u);
    if (!a) {
        const hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) ++g_live;
        return e;
    }
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    *p = a(bytes ? bytes : 1, dev, u);
    if (!*p) return hipErrorOutOfMemory;
    ++g_live;
    return hipSuccess;
}

hipError_t dev_free(void* p) {
    if (!p) return hipSuccess;
    pfe_alloc_fn a;
    pfe_free_fn f;
    void* u;
    current(a, f, u);
    --g_live;
    if (!f) return hipFree(p);
    // like hipFree, return the memory only after the device is done with it
    const hipError_t e = hipDeviceSynchronize();
    int dev = 0;
    (void)hipGetDevice(&dev);
    f(p, dev, u);
    return e;
}

hipError_t dev_alloc_async(void** p, size_t bytes, hipStream_t st) {
    pfe_alloc_fn a;
    pfe_free_fn f;
    void* u;
    current(a, f, u);
    if (!a) return hipMallocAsync(p, bytes, st);
    return dev_alloc(p, bytes);
}

hipError_t dev_free_async(void* p, hipStream_t st) {
    if (!p) return hipSuccess;
    pfe_alloc_fn a;
    pfe_free_fn f;
    void* u;
    current(a, f, u);
    if (!f) return hipFreeAsync(p, st);
    const hipError_t e = hipStreamSynchronize(st);
    const hipError_t e2 = dev_free(p);
    return e != hipSuccess ? e : e2;
}

}  // namespace pfe

extern "C" pfe_status pfe_set_allocator(pfe_alloc_fn alloc, pfe_free_fn release, void* user) {
    using namespace pfe;
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("pfe_set_allocator: give both functions or neither");
        return PFE_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_live.load() != 0) {
        set_error("pfe_set_allocator: %lld device allocations of the library are still live", g_live.load());
        return PFE_E_STATE;
    }
    g_alloc = alloc;
    g_free = release;
    g_user = alloc ? user : nullptr;
    return PFE_OK;
}

extern "C" int64_t pfe_live_allocations(void) { return (int64_t)pfe::g_live.load(); }
