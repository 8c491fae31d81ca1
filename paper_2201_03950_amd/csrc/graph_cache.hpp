// graph_cache.hpp -- bounded caches of captured launches (hipGraphExec) and of
// other per-key device state, with least-recently-used eviction.
//
// Keys hold raw device pointers, so a caller whose buffers move (autograd
// loops, a caching allocator) produces a new key on most calls; the caches
// therefore keep at most `cap` entries and release the least recently used
// one when a new entry would exceed it.  An evicted graph may still be
// executing: its stream is synchronised before the exec is destroyed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <utility>

namespace trid {

template <class K, class V>
struct LruMap {
    size_t cap;
    uint64_t tick = 0;
    std::map<K, std::pair<V, uint64_t>> m;

    explicit LruMap(size_t c) : cap(c) {}

    // Entry for k (marked as used), or nullptr.
    V *find(const K &k) {
        auto it = m.find(k);
        if (it == m.end()) return nullptr;
        it->second.second = ++tick;
        return &it->second.first;
    }
    // Insert (k, v).  If that makes the map exceed its capacity, the least
    // recently used other entry is removed and passed to drop(key, value).
    template <class Drop>
    V *insert(const K &k, V v, Drop &&drop) {
        auto res = m.emplace(k, std::make_pair(v, ++tick));
        if (!res.second) res.first->second = std::make_pair(v, tick);
        while (m.size() > cap) {
            auto victim = m.end();
            for (auto it = m.begin(); it != m.end(); ++it)
                if (it != res.first && (victim == m.end() || it->second.second < victim->second.second))
                    victim = it;
            if (victim == m.end()) break;
            drop(victim->first, victim->second.first);
            m.erase(victim);
        }
        return &res.first->second.first;
    }
    template <class Drop>
    void clear(Drop &&drop) {
        for (auto &kv : m) drop(kv.first, kv.second.first);
        m.clear();
    }
    size_t size() const { return m.size(); }
    template <class F>
    void for_each(F &&f) const {
        for (auto &kv : m) f(kv.first, kv.second.first);
    }
};

// Destroy an exec that may still run on `s`.
inline void destroy_graph_exec(hipGraphExec_t g, hipStream_t s) {
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(g);
}

}  // namespace trid
