// C entry points over the library's field cache and pool allocator with a
// fake mover (host byte arrays stand in for device memory and the pinned
// spill area), so the LRU / spill / fill / limit logic is tested on the CPU.
#include <cstdint>
#include <cstring>
#include <vector>

#include "cache.hpp"

namespace {
struct FakeMover : qdpmi::Mover {
    std::vector<unsigned char> dev, host;
    uint64_t copies = 0;
    bool host_area_ready() override { return !host.empty(); }
    bool d2h(size_t d, size_t h, size_t n) override { std::memcpy(&host[h], &dev[d], n); ++copies; return true; }
    bool h2d(size_t h, size_t d, size_t n) override { std::memcpy(&dev[d], &host[h], n); ++copies; return true; }
    bool d2d(size_t s, size_t d, size_t n) override { std::memmove(&dev[d], &dev[s], n); ++copies; return true; }
};
struct Harness {
    FakeMover m;
    qdpmi::FieldCache c;
};
}  // namespace

extern "C" {
void* hl_create(size_t dev_bytes, size_t host_bytes) {
    auto* h = new Harness();
    h->m.dev.assign(dev_bytes, 0);
    h->m.host.assign(host_bytes, 0);
    h->c.reset(dev_bytes, host_bytes, &h->m);
    return h;
}
void hl_destroy(void* p) { delete static_cast<Harness*>(p); }
int hl_create_field(void* p, uint64_t id, size_t bytes) { return static_cast<Harness*>(p)->c.create(id, bytes); }
int hl_destroy_field(void* p, uint64_t id) { return static_cast<Harness*>(p)->c.destroy(id); }
int hl_acquire(void* p, uint64_t id, int need) { return static_cast<Harness*>(p)->c.acquire(id, need != 0); }
void hl_release(void* p, uint64_t id) { static_cast<Harness*>(p)->c.release(id); }
int hl_evict(void* p, uint64_t id) { return static_cast<Harness*>(p)->c.evict(id); }
int hl_evict_all(void* p) { return static_cast<Harness*>(p)->c.evict_all(); }
int hl_set_limit(void* p, size_t b) { return static_cast<Harness*>(p)->c.set_limit(b); }
void hl_fault_after(void* p, int64_t n) { static_cast<Harness*>(p)->c.fault_after(n); }
int hl_swap(void* p, uint64_t a, uint64_t b) { return static_cast<Harness*>(p)->c.swap_storage(a, b); }
// Fill / verify the bytes of a resident entry with a pattern.
int hl_write(void* p, uint64_t id, uint8_t seed) {
    auto* h = static_cast<Harness*>(p);
    const qdpmi::CacheEntry* e = h->c.find(id);
    if (!e || !e->on_device) return -1;
    for (size_t i = 0; i < e->bytes; ++i) h->m.dev[e->dev_off + i] = (unsigned char)(seed + i * 7);
    return 0;
}
int hl_verify(void* p, uint64_t id, uint8_t seed) {
    auto* h = static_cast<Harness*>(p);
    const qdpmi::CacheEntry* e = h->c.find(id);
    if (!e || !e->on_device) return -1;
    for (size_t i = 0; i < e->bytes; ++i)
        if (h->m.dev[e->dev_off + i] != (unsigned char)(seed + i * 7)) return 1;
    return 0;
}
int hl_info(void* p, uint64_t id, int64_t* out) {
    const qdpmi::CacheEntry* e = static_cast<Harness*>(p)->c.find(id);
    if (!e) return -1;
    out[0] = e->on_device; out[1] = (int64_t)e->dev_off; out[2] = e->on_host;
    out[3] = (int64_t)e->host_off; out[4] = e->pins; out[5] = (int64_t)e->bytes;
    return 0;
}
void hl_counters(void* p, uint64_t* out) {
    auto* h = static_cast<Harness*>(p);
    const auto& k = h->c.counters();
    out[0] = k.hits; out[1] = k.misses; out[2] = k.spills; out[3] = k.fills;
    out[4] = k.bytes_spilled; out[5] = k.bytes_filled;
    out[6] = h->c.device_pool().used_bytes(); out[7] = h->c.device_pool().high_water();
    out[8] = h->c.host_pool().used_bytes(); out[9] = h->c.device_pool().limit();
    out[10] = h->m.copies;
}
int hl_check(void* p) {
    auto* h = static_cast<Harness*>(p);
    return h->c.device_pool().check() && h->c.host_pool().check() ? 0 : 1;
}
// Direct pool allocator access.
void* pl_create(size_t cap) { auto* o = new qdpmi::OffsetPool(); o->reset(cap); return o; }
void pl_destroy(void* p) { delete static_cast<qdpmi::OffsetPool*>(p); }
int64_t pl_alloc(void* p, size_t n) { size_t off; return static_cast<qdpmi::OffsetPool*>(p)->alloc(n, &off) ? (int64_t)off : -1; }
int pl_release(void* p, size_t off) { return static_cast<qdpmi::OffsetPool*>(p)->release(off) ? 0 : -1; }
int pl_check(void* p) { return static_cast<qdpmi::OffsetPool*>(p)->check() ? 0 : 1; }
size_t pl_used(void* p) { return static_cast<qdpmi::OffsetPool*>(p)->used_bytes(); }
size_t pl_largest(void* p) { return static_cast<qdpmi::OffsetPool*>(p)->largest_free(); }
void pl_set_limit(void* p, size_t l) { static_cast<qdpmi::OffsetPool*>(p)->set_limit(l); }
}
