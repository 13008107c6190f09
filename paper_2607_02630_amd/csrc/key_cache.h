// key_cache.h -- which expanded keys a serving engine keeps resident in its
// device key table.
//
// Pure C++ (no HIP), driven by the engine's one driver thread, so it needs no
// lock and can be exercised on the CPU by itself.
//
// The engine owns a device table of `slots` key records (the round-key words
// of one expanded key each).  When it forms a launch it asks the cache, per
// cipher request, where the launch should read that request's round keys:
//   - hit: the key sits in a valid slot; the launch reads the slot and the
//     request's descriptor carries only the slot index;
//   - miss: the key travels inline in the launch's own table.  If a slot can
//     be taken (a free one, else the least recently used slot that no launch
//     in flight reads), the launch also writes the key into that slot
//     ("install"); the slot turns valid when that launch completes, so no
//     launch can read a slot before the launch that fills it has finished.
// A slot is never overwritten while a launch in flight reads it or installs
// into it: each such launch holds a reference until it completes.
#pragma once

#include <stdint.h>
#include <string.h>
#include <unordered_map>
#include <vector>

namespace aesctr {

class KeyCache {
public:
    // Round-key words of one expanded key as the kernels read them (up to 60
    // column words) and its round count; two keys are equal when nr and the
    // first 4*(nr+1) words are.
    static constexpr int kWords = 60;

    struct Ref {
        int32_t slot = -1;      // slot read (resident) or written (install); -1 = none
        bool resident = false;  // the launch reads the key from `slot`
        bool install = false;   // the launch carries the key inline and writes it to `slot`
        int32_t pending = -1;   // on a miss: the slot whose install of this key is
                                // still in flight (no reference is held on it)
    };

    explicit KeyCache(int slots) : slots_(slots > 0 ? static_cast<size_t>(slots) : 0)
    {
        for (size_t i = 0; i < slots_.size(); ++i)
            lru_push_back(static_cast<int32_t>(i));
        index_.reserve(slots_.size() * 2);
    }

    int slots() const { return static_cast<int>(slots_.size()); }
    uint64_t hits() const { return hits_; }
    uint64_t misses() const { return misses_; }
    uint64_t installs() const { return installs_; }
    uint64_t evictions() const { return evictions_; }

    Ref acquire(const uint32_t *rk, uint32_t nr)
    {
        Ref r;
        if (slots_.empty())
            return r;
        const uint64_t h = hash(rk, nr);
        auto it = index_.find(h);
        if (it != index_.end()) {
            Slot &s = slots_[it->second];
            if (same(s, rk, nr)) {
                if (s.state == kValid) {
                    if (s.refs++ == 0)
                        lru_unlink(it->second);
                    ++hits_;
                    r.slot = it->second;
                    r.resident = true;
                    return r;
                }
                ++misses_;          // its install is still in flight: carry it inline
                r.pending = it->second;
                return r;
            }
            ++misses_;              // a different key with the same hash: inline, no install
            return r;
        }
        ++misses_;
        const int32_t v = lru_head_;
        if (v < 0)
            return r;               // every slot is read or filled by a launch in flight
        Slot &s = slots_[v];
        lru_unlink(v);
        if (s.state == kValid) {
            index_.erase(s.hash);
            ++evictions_;
        }
        s.state = kPending;
        s.refs = 1;
        s.nr = nr;
        s.hash = h;
        memset(s.rk, 0, sizeof(s.rk));
        memcpy(s.rk, rk, sizeof(uint32_t) * words(nr));
        index_.emplace(h, v);
        ++installs_;
        r.slot = v;
        r.install = true;
        return r;
    }

    // The launch holding r has completed (ok = its work ran; otherwise an
    // install it carried never reached the slot).
    void release(const Ref &r, bool ok)
    {
        if (r.slot < 0)
            return;
        Slot &s = slots_[r.slot];
        if (r.install) {
            if (ok) {
                s.state = kValid;
            } else {
                index_.erase(s.hash);
                s.state = kFree;
            }
        }
        if (--s.refs == 0)
            lru_push_back(r.slot);
    }

    // Bookkeeping invariants, for tests: every slot is either referenced or
    // on the LRU list (never both), and the index maps exactly the pending
    // and valid slots.
    bool consistent() const
    {
        size_t on_list = 0;
        for (int32_t i = lru_head_; i >= 0; i = slots_[i].next) {
            if (slots_[i].refs != 0 || slots_[i].state == kPending)
                return false;
            ++on_list;
        }
        size_t mapped = 0;
        for (size_t i = 0; i < slots_.size(); ++i) {
            const Slot &s = slots_[i];
            if (s.refs == 0 && s.state != kPending && !s.listed)
                return false;
            if (s.state != kFree) {
                auto it = index_.find(s.hash);
                if (it == index_.end() || it->second != static_cast<int32_t>(i))
                    return false;
                ++mapped;
            }
        }
        return mapped == index_.size() && on_list <= slots_.size();
    }

private:
    enum State : uint8_t { kFree = 0, kPending = 1, kValid = 2 };

    struct Slot {
        uint32_t rk[kWords] = {};
        uint32_t nr = 0;
        uint64_t hash = 0;
        uint32_t refs = 0;
        State state = kFree;
        bool listed = false;
        int32_t prev = -1, next = -1;   // LRU list links
    };

    static size_t words(uint32_t nr) { return nr <= 14 ? 4 * (nr + 1) : kWords; }

    // Hashes the cipher key alone (the first Nk = nr - 6 words of a schedule
    // are the key, FIPS-197 Sec. 5.2): a few steps per request on the driver
    // thread instead of one per round-key word.  Equality still compares the
    // whole schedule (`same`), so a schedule that shares its first words with
    // another and differs later is a different key.
    static uint64_t hash(const uint32_t *rk, uint32_t nr)
    {
        uint64_t h = 0x9e3779b97f4a7c15ull ^ nr;
        const size_t nk = nr >= 10 && nr <= 14 ? nr - 6 : words(nr);
        const size_t n = nk < words(nr) ? nk : words(nr);
        for (size_t i = 0; i < n; ++i) {
            h ^= rk[i];
            h *= 0xff51afd7ed558ccdull;
            h ^= h >> 29;
        }
        return h;
    }

    static bool same(const Slot &s, const uint32_t *rk, uint32_t nr)
    {
        return s.nr == nr && memcmp(s.rk, rk, sizeof(uint32_t) * words(nr)) == 0;
    }

    void lru_push_back(int32_t i)
    {
        Slot &s = slots_[i];
        s.prev = lru_tail_;
        s.next = -1;
        s.listed = true;
        if (lru_tail_ >= 0)
            slots_[lru_tail_].next = i;
        else
            lru_head_ = i;
        lru_tail_ = i;
    }

    void lru_unlink(int32_t i)
    {
        Slot &s = slots_[i];
        if (!s.listed)
            return;
        if (s.prev >= 0)
            slots_[s.prev].next = s.next;
        else
            lru_head_ = s.next;
        if (s.next >= 0)
            slots_[s.next].prev = s.prev;
        else
            lru_tail_ = s.prev;
        s.prev = s.next = -1;
        s.listed = false;
    }

    std::vector<Slot> slots_;
    std::unordered_map<uint64_t, int32_t> index_;
    int32_t lru_head_ = -1, lru_tail_ = -1;
    uint64_t hits_ = 0, misses_ = 0, installs_ = 0, evictions_ = 0;
};

}  // namespace aesctr
