// First-fit allocator over a byte range [0, size): the bookkeeping of the
// serving engine's device pool (host-only, no device calls).  Offsets and
// sizes are multiples of 256 bytes; freed neighbours are coalesced.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace btas {

class RangeAllocator {
   public:
    static size_t round(size_t x) { return (x + 255) / 256 * 256; }

    void reset(size_t size) {
        size_ = round(size);
        used_ = peak_ = 0;
        free_.clear();
        if (size_) free_[0] = size_;
    }
    // Offset of a block of at least `bytes`, or SIZE_MAX if none is free.
    size_t alloc(size_t bytes) {
        bytes = round(bytes);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }

   private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace btas
