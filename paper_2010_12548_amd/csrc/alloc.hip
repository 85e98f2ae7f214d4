// alloc.hip -- device memory of builds and handles without driver calls in
// steady state.
//
// Blocks come from a per-device cache in size classes of four steps per
// octave (at most 25% over the request).  A build's temporaries are taken by
// a Workspace bound to the build's stream: a block it releases goes to its
// own spare list and serves later requests of the same build (same stream,
// so stream order separates the old and new contents); when the build has
// synchronised its stream, every block returns to the cache for any later
// build.  Handle arrays come from the same cache and return to it when the
// handle is freed (the caller guarantees that no queued work still reads
// them).  Small values read back to the host go through one pinned staging
// buffer per workspace, so a group of reads costs one synchronisation.
// A build given a device allocator of the caller's takes every block of its
// temporaries and of its handle from it instead, and gives each back to it.
#include <map>
#include <mutex>
#include <vector>

#include "sba_internal.h"

namespace {

constexpr int MAX_DEV = 64;

struct DevCache {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free_blocks;
    std::vector<void *> pinned;  // idle staging buffers (PINNED_BYTES each)
};

DevCache g_cache[MAX_DEV];

constexpr size_t PINNED_BYTES = 4096;

size_t class_size(size_t bytes)
{
    if (bytes <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)(bytes - 1));  // 2^e < bytes <= 2^(e+1)
    size_t base = (size_t)1 << e, step = base / 4;
    return base + ((bytes - base + step - 1) / step) * step;
}

int current_device(int *dev)
{
    if (hipGetDevice(dev) != hipSuccess || *dev < 0 || *dev >= MAX_DEV) {
        (void)hipGetLastError();
        return SBA_EDEVICE;
    }
    return 0;
}

// give every idle cached block of the device back to the driver
void trim(int dev)
{
    std::vector<void *> all;
    {
        std::lock_guard<std::mutex> lk(g_cache[dev].mu);
        for (auto &kv : g_cache[dev].free_blocks)
            for (void *p : kv.second) all.push_back(p);
        g_cache[dev].free_blocks.clear();
    }
    for (void *p : all) (void)hipFree(p);
    (void)hipGetLastError();
}

}  // namespace

int cache_get(size_t bytes, DevBlock *out)
{
    int dev = 0;
    RC(current_device(&dev));
    const size_t c = class_size(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(g_cache[dev].mu);
        auto it = g_cache[dev].free_blocks.find(c);
        if (it != g_cache[dev].free_blocks.end() && !it->second.empty()) {
            *out = DevBlock{it->second.back(), c, dev, UserAlloc{}};
            it->second.pop_back();
            return 0;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        trim(dev);
        if (hipMalloc(&p, c) != hipSuccess) {
            (void)hipGetLastError();
            return SBA_ENOMEM;
        }
    }
    *out = DevBlock{p, c, dev, UserAlloc{}};
    return 0;
}

int block_get(size_t bytes, const UserAlloc &ua, DevBlock *out)
{
    if (!ua.alloc) return cache_get(bytes, out);
    int dev = 0;
    RC(current_device(&dev));
    const size_t c = class_size(bytes ? bytes : 1);
    void *p = ua.alloc(c, ua.ctx);
    if (!p) return SBA_ENOMEM;
    if (((uintptr_t)p & 255) != 0) {  // the kernels' vector loads need the alignment
        ua.release(p, ua.ctx);
        return SBA_EINVAL;
    }
    *out = DevBlock{p, c, dev, ua};
    return 0;
}

void cache_put(const DevBlock &b)
{
    if (!b.p) return;
    if (b.ua.alloc) {
        b.ua.release(b.p, b.ua.ctx);
        return;
    }
    if (b.dev < 0 || b.dev >= MAX_DEV) return;
    std::lock_guard<std::mutex> lk(g_cache[b.dev].mu);
    g_cache[b.dev].free_blocks[b.cls].push_back(b.p);
}

// ---------------------------------------------------------------- Workspace

Workspace::Workspace(hipStream_t st) : st_(st)
{
    if (current_device(&dev_)) dev_ = -1;
}

Workspace::~Workspace()
{
    (void)hipStreamSynchronize(st_);
    (void)hipGetLastError();
    for (const DevBlock &b : live_) cache_put(b);
    for (const DevBlock &b : spare_) cache_put(b);
    if (pinned_ && dev_ >= 0) {
        std::lock_guard<std::mutex> lk(g_cache[dev_].mu);
        g_cache[dev_].pinned.push_back(pinned_);
    }
}

int Workspace::get(void **p, size_t bytes)
{
    *p = nullptr;
    if (dev_ < 0) return SBA_EDEVICE;
    const size_t c = class_size(bytes ? bytes : 1);
    for (size_t k = 0; k < spare_.size(); k++) {
        if (spare_[k].cls == c) {
            DevBlock b = spare_[k];
            spare_[k] = spare_.back();
            spare_.pop_back();
            live_.push_back(b);
            *p = b.p;
            return 0;
        }
    }
    DevBlock b{};
    RC(block_get(bytes, ua_, &b));
    live_.push_back(b);
    *p = b.p;
    return 0;
}

void Workspace::put(void *p)
{
    if (!p) return;
    for (size_t k = 0; k < live_.size(); k++) {
        if (live_[k].p == p) {
            spare_.push_back(live_[k]);
            live_[k] = live_.back();
            live_.pop_back();
            return;
        }
    }
}

int Workspace::read(void *host, const void *dev, size_t bytes)
{
    if (dev_ < 0) return SBA_EDEVICE;
    if (!pinned_) {
        {
            std::lock_guard<std::mutex> lk(g_cache[dev_].mu);
            if (!g_cache[dev_].pinned.empty()) {
                pinned_ = (char *)g_cache[dev_].pinned.back();
                g_cache[dev_].pinned.pop_back();
            }
        }
        if (!pinned_ && hipHostMalloc((void **)&pinned_, PINNED_BYTES, hipHostMallocDefault) !=
                            hipSuccess) {
            (void)hipGetLastError();
            pinned_ = nullptr;
            return SBA_ENOMEM;
        }
    }
    size_t off = (staged_ + 15) & ~(size_t)15;
    if (off + bytes > PINNED_BYTES) return SBA_ELIMIT;
    HIP_OK(hipMemcpyAsync(pinned_ + off, dev, bytes, hipMemcpyDeviceToHost, st_));
    reads_.push_back(Read{host, off, bytes});
    staged_ = off + bytes;
    return 0;
}

int Workspace::sync()
{
    HIP_OK(hipStreamSynchronize(st_));
    for (const Read &r : reads_) memcpy(r.host, pinned_ + r.off, r.bytes);
    reads_.clear();
    staged_ = 0;
    return 0;
}

// ---------------------------------------------------------------- handles

int handle_get(sba_handle *h, void **p, size_t bytes)
{
    DevBlock b{};
    RC(block_get(bytes, h->ua, &b));
    h->blocks_owned.push_back(b);
    h->bytes += (int64_t)bytes;
    *p = b.p;
    return 0;
}

void handle_put_all(sba_handle *h)
{
    for (const DevBlock &b : h->blocks_owned) cache_put(b);
    h->blocks_owned.clear();
}
