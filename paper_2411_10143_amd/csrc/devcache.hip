// Per-device cache of device memory blocks for matrix handles (devcache.hpp).
#include "devcache.hpp"

#include <map>
#include <mutex>
#include <unordered_map>

namespace ck {
namespace {

struct Block {
    size_t bytes;
    int device;
};

std::mutex g_mu;
std::unordered_map<void *, Block> g_live;          // every block handed out
std::map<int, std::multimap<size_t, void *>> g_free;   // per device: class -> blocks
std::map<int, size_t> g_cached;                        // per device: bytes held free

// Smallest size class >= bytes: 4 KiB, then 2^k * {1.25, 1.5, 1.75, 2}.
size_t size_class(size_t bytes) {
    if (bytes <= 4096)
        return 4096;
    size_t p = 4096;
    while (p < bytes)
        p <<= 1;
    const size_t h = p >> 1;
    for (size_t q = 5; q <= 8; ++q) {
        const size_t c = h / 4 * q;
        if (c >= bytes)
            return c;
    }
    return p;
}

void release_cached(int device) {   // with g_mu held
    auto &fl = g_free[device];
    for (auto &kv : fl)
        (void)hipFree(kv.second);
    fl.clear();
    g_cached[device] = 0;
}

}  // namespace

ck_status dev_cache_alloc(void **p, size_t bytes) {
    *p = nullptr;
    int device = 0;
    CK_HIP(hipGetDevice(&device));
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    auto &fl = g_free[device];
    auto it = fl.find(cls);
    if (it != fl.end()) {
        *p = it->second;
        fl.erase(it);
        g_cached[device] -= cls;
        g_live[*p] = Block{cls, device};
        return CK_OK;
    }
    hipError_t e = hipMalloc(p, cls);
    if (e != hipSuccess && g_cached[device] > 0) {   // give the cache back, then retry
        (void)hipGetLastError();
        release_cached(device);
        e = hipMalloc(p, cls);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(CK_E_NOMEM, "device allocation of %zu bytes failed: %s", cls,
                    hipGetErrorString(e));
    }
    g_live[*p] = Block{cls, device};
    return CK_OK;
}

void dev_cache_free(void *p) {
    if (!p)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end())
        return;
    const Block b = it->second;
    g_live.erase(it);
    if (g_cached[b.device] + b.bytes > kDevCacheBytes) {
        (void)hipFree(p);
        return;
    }
    g_free[b.device].emplace(b.bytes, p);
    g_cached[b.device] += b.bytes;
}

ck_status mem_alloc(MemSource &m, void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (!m.user)
        return dev_cache_alloc(p, bytes);
    void *q = m.a.alloc(bytes > 0 ? bytes : 1, s, m.a.ctx);
    if (!q)
        return fail(CK_E_NOMEM, "the caller's allocator returned NULL for %zu bytes", bytes);
    std::lock_guard<std::mutex> lk(m.mu);
    m.streams[q] = s;
    *p = q;
    return CK_OK;
}

void mem_free(MemSource &m, void *p) {
    if (!p)
        return;
    if (!m.user) {
        dev_cache_free(p);
        return;
    }
    hipStream_t s = nullptr;
    {
        std::lock_guard<std::mutex> lk(m.mu);
        auto it = m.streams.find(p);
        if (it == m.streams.end())
            return;
        s = it->second;
        m.streams.erase(it);
    }
    m.a.free(p, s, m.a.ctx);
}

}  // namespace ck
