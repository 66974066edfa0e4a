// Device memory of matrix handles: a per-device cache of freed blocks.
#pragma once

#include <unordered_map>

#include "common.hpp"

namespace ck {

// Blocks freed by a destroyed handle (or a failed conversion) are kept, up
// to kDevCacheBytes per device, and handed to later allocations of the same
// size class (sizes are rounded up to 4 KiB or to 2^k times 1.25, 1.5, 1.75
// or 2, at most 25 % over).  Creating and destroying matrices then maps no pages and
// does not synchronise the device, as hipMalloc / hipFree do.  A block goes
// back to the cache only when no work that uses it can still be pending (the
// callers guarantee it), so it may be reused on any stream at once.
constexpr size_t kDevCacheBytes = size_t(16) << 30;

ck_status dev_cache_alloc(void **p, size_t bytes);
void dev_cache_free(void *p);   // NULL is ignored

template <typename T>
ck_status dev_alloc(T **p, int64_t count) {
    void *q = nullptr;
    const ck_status st = dev_cache_alloc(&q, (size_t)(count > 0 ? count : 1) * sizeof(T));
    *p = (T *)q;
    return st;
}

// Where one handle's device memory comes from: the caller's allocator
// (spmv_create's `alloc`), or the per-device cache above when there is none.
// Every block of the handle -- its format copies, feature and conversion
// temporaries, product carries and solver workspaces -- comes from here.
// A block is given back only once no work that uses it can be pending.
struct MemSource {
    ck_allocator a{};
    bool user = false;
    std::mutex mu;
    std::unordered_map<void *, hipStream_t> streams;   // user blocks -> allocation stream
};

ck_status mem_alloc(MemSource &m, void **p, size_t bytes, hipStream_t s);
void mem_free(MemSource &m, void *p);   // NULL is ignored

}  // namespace ck
