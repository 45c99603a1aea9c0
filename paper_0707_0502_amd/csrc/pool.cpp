// Device-memory cache of the contexts (declared in engine.h): per-context
// idle lists, a process-wide registry of the live caches per device, and the
// device-wide cap on idle bytes.
#include <atomic>

#include "engine.h"

namespace gdr {
namespace {

constexpr int MAXDEV = 64;

struct DevShare {
    std::atomic<size_t> idle{0};   // idle bytes of every cache on the device
    size_t cap = 0;                // set at the first attach: half of the device
};
DevShare g_share[MAXDEV];

std::mutex g_reg_mu;
std::vector<DevPool*> g_reg;   // live caches (all devices)

DevShare& share(int dev) { return g_share[dev >= 0 && dev < MAXDEV ? dev : 0]; }

}  // namespace

size_t pool_idle_bytes(int dev) { return share(dev).idle.load(); }
size_t pool_idle_cap(int dev) { return share(dev).cap; }

void DevPool::attach(int dev) {
    device = dev;
    std::lock_guard<std::mutex> g(g_reg_mu);
    DevShare& s = share(dev);
    if (s.cap == 0) {
        // a block released to the driver is expensive to get back (after
        // large frees, hipMalloc of a multi-GB block has taken 0.3-0.9 s), so
        // up to 60 % of the device may stay idle: enough for every phase of a
        // 32^3x64 solve (about 130 GB) to find its buffers again while other
        // contexts on the device keep theirs (at half the device, ten small
        // lattices' caches pushed the 32^3x64 lattice's projection buffers
        // out between solves, and each solve allocated them again)
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) s.cap = tot / 10 * 6;
        else (void)hipGetLastError();
    }
    g_reg.push_back(this);
}

void DevPool::detach() {
    {
        std::lock_guard<std::mutex> g(g_reg_mu);
        for (size_t i = 0; i < g_reg.size(); ++i)
            if (g_reg[i] == this) {
                g_reg.erase(g_reg.begin() + (long)i);
                break;
            }
    }
    release();
}

void DevPool::drop_oldest() {
    auto oldest = lru.begin();
    auto range = bysize.equal_range(oldest->sz);
    for (auto it = range.first; it != range.second; ++it)
        if (it->second == oldest) {
            bysize.erase(it);
            break;
        }
    idle_bytes -= oldest->sz;
    share(device).idle -= oldest->sz;
    (void)hipFree(oldest->p);
    lru.erase(oldest);
}

void* DevPool::get(size_t bytes) {
    bytes = round(bytes);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = bysize.lower_bound(bytes);
        if (it != bysize.end() && it->first <= bytes + bytes / 4) {
            auto li = it->second;
            void* p = li->p;
            const size_t sz = li->sz;
            used[p] = sz;
            idle_bytes -= sz;
            share(device).idle -= sz;
            lru.erase(li);
            bysize.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    bool ok = hipMalloc(&p, bytes) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        release();
        ok = hipMalloc(&p, bytes) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        // the idle blocks of the other contexts on this device (one cache
        // locked at a time; the registry lock keeps them alive meanwhile)
        {
            std::lock_guard<std::mutex> g(g_reg_mu);
            for (DevPool* q : g_reg)
                if (q != this && q->device == device) q->release();
        }
        ok = hipMalloc(&p, bytes) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    std::lock_guard<std::mutex> g(mu);
    used[p] = bytes;
    return p;
}

void DevPool::put(void* p) {
    std::lock_guard<std::mutex> g(mu);
    auto u = used.find(p);
    if (u == used.end()) return;
    const size_t sz = u->second;
    used.erase(u);
    DevShare& s = share(device);
    if (sz > s.cap) {
        (void)hipFree(p);
        return;
    }
    lru.push_back({sz, p});
    bysize.emplace(sz, std::prev(lru.end()));
    idle_bytes += sz;
    s.idle += sz;
    while (s.idle.load() > s.cap && !lru.empty()) drop_oldest();
}

size_t DevPool::release() {
    std::lock_guard<std::mutex> g(mu);
    const size_t b = idle_bytes;
    for (auto& blk : lru) (void)hipFree(blk.p);
    share(device).idle -= idle_bytes;
    lru.clear();
    bysize.clear();
    idle_bytes = 0;
    return b;
}

}  // namespace gdr
