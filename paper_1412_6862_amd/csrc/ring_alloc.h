// Circular allocator over [0, size) for the server's output pool: allocations
// are handed out and reclaimed in the same (FIFO) order.  Host code only.
#pragma once

#include <stdint.h>

namespace hm {

class RingAllocator {
public:
    explicit RingAllocator(uint64_t size = 0) : size_(size) {}

    // Reserve `bytes` (> 0); false when no contiguous range is free.  The
    // free space is [head, size) and [0, tail) while nothing has wrapped, and
    // [head, tail) once allocations have wrapped to the start; head == tail
    // with live allocations means full.
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        if (live_ == 0) head_ = tail_ = 0;
        if (bytes == 0 || bytes > size_) return false;
        if (live_ == 0 || head_ > tail_) {
            if (size_ - head_ >= bytes) {
                *off = head_;
                head_ += bytes;
            } else if (tail_ >= bytes) {    // wrap; [head, size) is skipped
                *off = 0;
                head_ = bytes;
            } else {
                return false;
            }
        } else {
            if (tail_ - head_ < bytes) return false;
            *off = head_;
            head_ += bytes;
        }
        ++live_;
        used_ += bytes;
        return true;
    }

    // Reclaim the oldest live allocation (off, bytes as handed out).
    void release_oldest(uint64_t off, uint64_t bytes)
    {
        tail_ = off + bytes;
        --live_;
        used_ -= bytes;
        if (live_ == 0) head_ = tail_ = 0;
    }

    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t live() const { return live_; }

private:
    uint64_t size_;
    uint64_t head_ = 0, tail_ = 0, used_ = 0, live_ = 0;
};

}  // namespace hm
