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
// buffer per workspace, so a group of reads costs one synchronisation: one
// small kernel copies them into the (coherent) staging buffer and then raises
// a flag there, which the host polls for a short while before it falls back
// to a blocking stream synchronisation.  A build makes several such reads, and
// the poll returns in a few microseconds where waking from a blocking wait
// and a copy-engine transfer take tens.
// A build given a device allocator of the caller's takes every block of its
// temporaries and of its handle from it instead, and gives each back to it.
#include <atomic>
#include <chrono>
#include <cstring>
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
// the staged values sit below FLAG_OFF; the flag word (a number unique to
// each sync) above it
constexpr size_t FLAG_OFF = PINNED_BYTES - 64;
// how long the host polls the flag before it blocks on the stream
constexpr double POLL_US = 300.0;
std::atomic<uint32_t> g_read_seq{0};

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

// Copies the queued reads into the staging buffer (one workgroup; sizes and
// offsets in bytes, 8-byte words where both ends allow), then makes them
// visible to the host before it writes `seq` to the flag word.
struct ReadSet {
    const unsigned char *src[WS_MAX_READS];
    uint32_t off[WS_MAX_READS], bytes[WS_MAX_READS];
    int n;
    unsigned char *dst;  // device address of the staging buffer
    uint32_t seq;
};

__global__ __launch_bounds__(64) void k_readback(ReadSet R)
{
    for (int r = 0; r < R.n; r++) {
        const unsigned char *src = R.src[r];
        unsigned char *dst = R.dst + R.off[r];
        const uint32_t nb = R.bytes[r];
        if ((((uintptr_t)src | (uintptr_t)dst | nb) & 7) == 0) {
            for (uint32_t k = threadIdx.x; k < nb / 8; k += 64)
                ((uint64_t *)dst)[k] = ((const uint64_t *)src)[k];
        } else {
            for (uint32_t k = threadIdx.x; k < nb; k += 64) dst[k] = src[k];
        }
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        *(volatile uint32_t *)(R.dst + FLAG_OFF) = R.seq;
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
        if (!pinned_) {
            if (hipHostMalloc((void **)&pinned_, PINNED_BYTES, hipHostMallocCoherent) !=
                hipSuccess) {
                (void)hipGetLastError();
                pinned_ = nullptr;
                return SBA_ENOMEM;
            }
            *(volatile uint32_t *)(pinned_ + FLAG_OFF) = 0;
        }
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, pinned_, 0) != hipSuccess || !dp) {
            (void)hipGetLastError();
            return SBA_EDEVICE;
        }
        pinned_dev_ = (char *)dp;
    }
    size_t off = (staged_ + 15) & ~(size_t)15;
    if (off + bytes > FLAG_OFF || reads_.size() >= WS_MAX_READS) return SBA_ELIMIT;
    reads_.push_back(Read{host, dev, off, bytes});
    staged_ = off + bytes;
    return 0;
}

int Workspace::sync()
{
    if (reads_.empty()) {
        HIP_OK(hipStreamSynchronize(st_));
        return 0;
    }
    ReadSet R{};
    for (size_t k = 0; k < reads_.size(); k++) {
        R.src[k] = (const unsigned char *)reads_[k].dev;
        R.off[k] = (uint32_t)reads_[k].off;
        R.bytes[k] = (uint32_t)reads_[k].bytes;
    }
    R.n = (int)reads_.size();
    R.dst = (unsigned char *)pinned_dev_;
    uint32_t seq = g_read_seq.fetch_add(1) + 1;
    if (seq == 0) seq = g_read_seq.fetch_add(1) + 1;  // 0 marks a fresh buffer
    R.seq = seq;
    hipLaunchKernelGGL(k_readback, dim3(1), dim3(64), 0, st_, R);
    HIP_OK(hipGetLastError());
    volatile uint32_t *flag = (volatile uint32_t *)(pinned_ + FLAG_OFF);
    const auto t0 = std::chrono::steady_clock::now();
    while (*flag != seq) {
        if (std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
                .count() > POLL_US) {
            // a long stretch of work ahead of the reads: block instead (the
            // kernel has ended, and its writes are visible, once this returns)
            HIP_OK(hipStreamSynchronize(st_));
            if (*flag != seq) return SBA_EDEVICE;
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
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
