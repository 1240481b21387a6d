// Software cache controlling where lattice objects live (device pool or
// pinned host memory), after section 4.1 and Figure 2 of the paper: the pool
// manager owns a large region of device memory; on allocation the cache
// spills least-recently-used objects to make room; referencing an object that
// is already on the device transfers nothing.
//
// Policy only: the byte movement is delegated to a Mover (HIP copies on the
// context stream in the library, plain memcpy in the CPU unit tests).  All
// copies are enqueued in program order on one stream, so a spill is ordered
// after every kernel that was enqueued before it, and a block freed here can
// be reused immediately by later work on that stream.
#pragma once

#include <cstdint>
#include <unordered_map>

#include "../../include/qdpmi.h"
#include "pool.hpp"

namespace qdpmi {

struct Mover {
    virtual ~Mover() = default;
    virtual bool host_area_ready() = 0;  // lazily create the spill area
    virtual bool d2h(size_t dev_off, size_t host_off, size_t bytes) = 0;
    virtual bool h2d(size_t host_off, size_t dev_off, size_t bytes) = 0;
    virtual bool d2d(size_t src_off, size_t dst_off, size_t bytes) = 0;
};

struct CacheEntry {
    size_t bytes = 0;
    bool on_device = false;
    size_t dev_off = 0;
    bool on_host = false;  // a host copy exists (only while not on device)
    size_t host_off = 0;
    int pins = 0;
    uint64_t last_use = 0;
};

struct CacheCounters {
    uint64_t hits = 0, misses = 0, spills = 0, fills = 0;
    uint64_t bytes_spilled = 0, bytes_filled = 0;
};

class FieldCache {
public:
    void reset(size_t dev_capacity, size_t host_capacity, Mover* mover) {
        dev_.reset(dev_capacity);
        host_.reset(host_capacity);
        entries_.clear();
        mover_ = mover;
        tick_ = 0;
        counters_ = CacheCounters{};
        fault_countdown_ = 0;
    }

    // Arm allocation-failure injection: the n-th device allocation from now
    // fails once (n >= 1); 0 disarms.
    void fault_after(int64_t n) { fault_countdown_ = n > 0 ? n : 0; }

    // New entry with device storage (contents undefined).
    qdp_status create(uint64_t id, size_t bytes) {
        if (entries_.count(id)) return QDP_ERR_STATE;
        size_t off;
        qdp_status s = device_alloc(bytes, &off);
        if (s != QDP_OK) return s;
        CacheEntry e;
        e.bytes = bytes;
        e.on_device = true;
        e.dev_off = off;
        e.last_use = ++tick_;
        entries_[id] = e;
        return QDP_OK;
    }

    qdp_status destroy(uint64_t id) {
        auto it = entries_.find(id);
        if (it == entries_.end()) return QDP_ERR_STATE;
        CacheEntry& e = it->second;
        if (e.pins) return QDP_ERR_STATE;
        if (e.on_device) dev_.release(e.dev_off);
        if (e.on_host) host_.release(e.host_off);
        entries_.erase(it);
        return QDP_OK;
    }

    // Pin an entry on the device for the duration of an operation.  With
    // need_contents the host copy of a spilled entry is brought back;
    // without it (the operation overwrites every byte) the copy is dropped.
    qdp_status acquire(uint64_t id, bool need_contents) {
        auto it = entries_.find(id);
        if (it == entries_.end()) return QDP_ERR_STATE;
        CacheEntry& e = it->second;
        e.pins++;  // pinned first: the allocation below must not evict it
        if (e.on_device) {
            counters_.hits++;
        } else {
            counters_.misses++;
            size_t off;
            qdp_status s = device_alloc(e.bytes, &off);
            if (s != QDP_OK) {
                e.pins--;
                return s;
            }
            if (need_contents && e.on_host) {
                if (!mover_->h2d(e.host_off, off, e.bytes)) {
                    dev_.release(off);
                    e.pins--;
                    return QDP_ERR_HIP;
                }
                counters_.fills++;
                counters_.bytes_filled += e.bytes;
            }
            if (e.on_host) host_.release(e.host_off);
            e.on_host = false;
            e.on_device = true;
            e.dev_off = off;
        }
        e.last_use = ++tick_;
        return QDP_OK;
    }

    void release(uint64_t id) {
        auto it = entries_.find(id);
        if (it != entries_.end() && it->second.pins > 0) it->second.pins--;
    }

    // Move one unpinned entry to the host now.
    qdp_status evict(uint64_t id) {
        auto it = entries_.find(id);
        if (it == entries_.end()) return QDP_ERR_STATE;
        if (!it->second.on_device) return QDP_OK;
        if (it->second.pins) return QDP_ERR_STATE;
        return spill(it->second);
    }

    qdp_status evict_all() {
        for (auto& kv : entries_) {
            if (kv.second.on_device && !kv.second.pins) {
                qdp_status s = spill(kv.second);
                if (s != QDP_OK) return s;
            }
        }
        return QDP_OK;
    }

    // Shrink (or grow) the usable part of the device pool.  Entries that end
    // above the new limit move below it (device copy) or, failing that, are
    // spilled.
    qdp_status set_limit(size_t bytes) {
        if (bytes > dev_.capacity()) return QDP_ERR_ARG;
        // a pinned entry (in use, or an external block) above the limit
        // cannot move: refuse before changing anything
        for (const auto& kv : entries_) {
            const CacheEntry& e = kv.second;
            if (e.on_device && e.pins && e.dev_off + OffsetPool::round_up(e.bytes) > bytes) return QDP_ERR_STATE;
        }
        dev_.set_limit(bytes);
        for (auto& kv : entries_) {
            CacheEntry& e = kv.second;
            if (!e.on_device || e.dev_off + OffsetPool::round_up(e.bytes) <= dev_.limit()) continue;
            if (e.pins) return QDP_ERR_STATE;
            size_t off;
            if (dev_.alloc(e.bytes, &off)) {
                if (!mover_->d2d(e.dev_off, off, e.bytes)) return QDP_ERR_HIP;
                dev_.release(e.dev_off);
                e.dev_off = off;
            } else {
                qdp_status s = spill(e);
                if (s != QDP_OK) return s;
            }
        }
        return QDP_OK;
    }

    // Exchange the device storage of two resident entries of equal size
    // (used to hand a finished ping-pong buffer to its destination without
    // a copy).
    qdp_status swap_storage(uint64_t a, uint64_t b) {
        auto ia = entries_.find(a), ib = entries_.find(b);
        if (ia == entries_.end() || ib == entries_.end()) return QDP_ERR_STATE;
        CacheEntry &ea = ia->second, &eb = ib->second;
        if (!ea.on_device || !eb.on_device || ea.bytes != eb.bytes) return QDP_ERR_STATE;
        const size_t t = ea.dev_off;
        ea.dev_off = eb.dev_off;
        eb.dev_off = t;
        return QDP_OK;
    }

    const CacheEntry* find(uint64_t id) const {
        auto it = entries_.find(id);
        return it == entries_.end() ? nullptr : &it->second;
    }

    const CacheCounters& counters() const { return counters_; }
    const OffsetPool& device_pool() const { return dev_; }
    const OffsetPool& host_pool() const { return host_; }
    size_t n_entries() const { return entries_.size(); }

private:
    qdp_status device_alloc(size_t bytes, size_t* off) {
        if (fault_countdown_ > 0 && --fault_countdown_ == 0) return QDP_ERR_NOMEM;
        while (!dev_.alloc(bytes, off)) {
            CacheEntry* victim = nullptr;
            for (auto& kv : entries_) {
                CacheEntry& e = kv.second;
                if (e.on_device && !e.pins && (!victim || e.last_use < victim->last_use)) victim = &e;
            }
            if (!victim) return QDP_ERR_NOMEM;
            qdp_status s = spill(*victim);
            if (s != QDP_OK) return s;
        }
        return QDP_OK;
    }

    qdp_status spill(CacheEntry& e) {
        if (!mover_->host_area_ready()) return QDP_ERR_NOMEM;
        size_t hoff;
        if (!host_.alloc(e.bytes, &hoff)) return QDP_ERR_NOMEM;
        if (!mover_->d2h(e.dev_off, hoff, e.bytes)) {
            host_.release(hoff);
            return QDP_ERR_HIP;
        }
        dev_.release(e.dev_off);
        e.on_device = false;
        e.on_host = true;
        e.host_off = hoff;
        counters_.spills++;
        counters_.bytes_spilled += e.bytes;
        return QDP_OK;
    }

    OffsetPool dev_, host_;
    std::unordered_map<uint64_t, CacheEntry> entries_;
    Mover* mover_ = nullptr;
    uint64_t tick_ = 0;
    CacheCounters counters_;
    int64_t fault_countdown_ = 0;
};

}  // namespace qdpmi
