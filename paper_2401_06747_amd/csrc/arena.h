// Host-side memory and block bookkeeping, free of HIP: the overlapping block
// geometry of the Schwarz smoothers, the bump allocator that lays buffers out
// in a caller's workspace, and the first-fit allocator the server runs over
// its arena. Pure C++17, so that the sanitizer tests can build it alone.
#pragma once
#include <stddef.h>
#include <iterator>
#include <map>

namespace hdi {

inline size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// Geometry of the overlapping tile x tile blocks along one dimension (Sec. 3.1,
// 3.3): count = ceil((n - tile) / (tile - overlap)) + 1, the last block shifted
// to end at the border.
struct Blocks1D {
    int n;       // pixels along the dimension
    int count;   // number of blocks
    int stride;  // start of block i is min(i*stride, n-tile)
};

inline Blocks1D make_blocks(int n, int overlap, int tile) {
    Blocks1D b;
    b.n = n;
    if (n <= tile) {
        b.count = 1;
        b.stride = tile;
    } else {
        b.stride = tile - overlap;
        b.count = (n - tile + b.stride - 1) / b.stride + 1;
    }
    return b;
}

// Bump allocator over the caller's workspace: 256-byte aligned offsets; with
// base == nullptr it only counts the bytes a layout needs.
struct Arena {
    char *base;
    size_t size, used;
    void *take(size_t bytes) {
        size_t off = up256(used);
        if (!base) { used = off + bytes; return nullptr; }
        if (off + bytes > size) return nullptr;
        used = off + bytes;
        return base + off;
    }
};

// First-fit allocator over a byte range; blocks are multiples of 256 bytes and
// neighbouring free blocks merge on release.
class ArenaAlloc {
public:
    void init(char *base, size_t size) {
        base_ = base;
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
    }
    size_t capacity() const { return size_; }
    char *alloc(size_t n) {
        n = up256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            return base_ + off;
        }
        return nullptr;
    }
    void release(char *p, size_t n) {
        n = up256(n);
        size_t off = (size_t)(p - base_);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    // free blocks, in address order (for tests)
    const std::map<size_t, size_t> &free_blocks() const { return free_; }

private:
    char *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
};

}  // namespace hdi
