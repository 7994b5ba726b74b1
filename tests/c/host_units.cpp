// Host-only units of libhdi under AddressSanitizer and UndefinedBehaviorSanitizer:
// the overlapping block geometry (Sec. 3.1, 3.3), the workspace bump allocator
// and the server's first-fit arena allocator. Prints "host units: ok" and exits
// 0 when every check holds; a failed check prints it and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2401_06747_amd/csrc/arena.h"

using namespace hdi;

static int g_fail = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::printf("check failed: %s (line %d)\n", #cond, __LINE__);    \
            ++g_fail;                                                        \
        }                                                                    \
    } while (0)

static void blocks() {
    // Sec. 3.3: 32x32 blocks with overlap 6 on a 4K colour image give 36852
    // local problems (148 x 83 blocks per channel)
    CHECK(make_blocks(3840, 6, 32).count == 148);
    CHECK(make_blocks(2160, 6, 32).count == 83);
    CHECK(3 * make_blocks(3840, 6, 32).count * make_blocks(2160, 6, 32).count == 36852);
    for (int tile : {16, 32, 64}) {
        for (int ov = 2; ov <= tile / 2; ov += 2) {
            for (int n = 1; n <= 700; ++n) {
                const Blocks1D b = make_blocks(n, ov, tile);
                CHECK(b.count >= 1);
                if (n <= tile) {
                    CHECK(b.count == 1);
                    continue;
                }
                // every pixel is covered, consecutive blocks overlap by at least
                // `ov`, and the last block ends at the border
                std::vector<int> cover(n, 0);
                int prev_start = -1;
                for (int i = 0; i < b.count; ++i) {
                    const int s = std::min(i * b.stride, n - tile);
                    CHECK(s >= 0 && s + tile <= n);
                    if (prev_start >= 0) CHECK(s > prev_start && prev_start + tile - s >= ov);
                    for (int x = s; x < s + tile; ++x) cover[x] += 1;
                    prev_start = s;
                }
                CHECK(prev_start + tile == n);
                for (int x = 0; x < n; ++x) CHECK(cover[x] >= 1);
                // one block fewer would not reach the border
                CHECK((b.count - 1 - 1) * b.stride + tile < n);
            }
        }
    }
}

static void bump() {
    Arena q{nullptr, 0, 0};
    CHECK(q.take(10) == nullptr && q.used == 10);
    CHECK(q.take(1) == nullptr && q.used == 257);
    std::vector<char> buf(4096 + 256);
    char *base = (char *)(((uintptr_t)buf.data() + 255) & ~(uintptr_t)255);
    Arena a{base, 4096, 0};
    char *p = (char *)a.take(100);
    char *r = (char *)a.take(300);
    CHECK(p == base && r == base + 256);
    std::memset(p, 1, 100);
    std::memset(r, 2, 300);
    CHECK(a.take(4096) == nullptr);                 // does not fit: nothing taken
    CHECK(a.used == 556);
    char *s = (char *)a.take(4096 - 768);
    CHECK(s == base + 768);
    std::memset(s, 3, 4096 - 768);
    CHECK(a.take(1) == nullptr);
}

static void first_fit() {
    const size_t cap = 1 << 20;
    std::vector<char> buf(cap);
    ArenaAlloc al;
    al.init(buf.data(), cap);
    CHECK(al.capacity() == cap);
    std::vector<unsigned char> owner(cap / 256, 0);   // 0 = free, else live block id
    struct Live { char *p; size_t n; unsigned char id; };
    std::vector<Live> live;
    std::mt19937_64 rng(2401);
    unsigned char next_id = 1;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t n = 1 + rng() % (cap / 16);
            char *p = al.alloc(n);
            if (!p) continue;
            const size_t off = (size_t)(p - buf.data());
            CHECK(off % 256 == 0 && off + up256(n) <= cap);
            for (size_t k = off / 256; k < (off + up256(n)) / 256; ++k) {
                CHECK(owner[k] == 0);   // no overlap with a live block
                owner[k] = next_id;
            }
            std::memset(p, next_id, n);
            live.push_back({p, n, next_id});
            next_id = next_id == 255 ? 1 : next_id + 1;
        } else {
            const size_t i = rng() % live.size();
            const Live l = live[i];
            // the block still holds what its owner wrote
            for (size_t k = 0; k < l.n; k += 97) CHECK((unsigned char)l.p[k] == l.id);
            const size_t off = (size_t)(l.p - buf.data());
            for (size_t k = off / 256; k < (off + up256(l.n)) / 256; ++k) owner[k] = 0;
            al.release(l.p, l.n);
            live.erase(live.begin() + i);
        }
        // free blocks are disjoint, sorted, never adjacent (merged), and cover
        // exactly the bytes no live block holds
        size_t free_bytes = 0, end = 0;
        bool first = true;
        for (const auto &kv : al.free_blocks()) {
            CHECK(first || kv.first > end);
            end = kv.first + kv.second;
            first = false;
            free_bytes += kv.second;
            for (size_t k = kv.first / 256; k < end / 256; ++k) CHECK(owner[k] == 0);
        }
        size_t live_bytes = 0;
        for (const Live &l : live) live_bytes += up256(l.n);
        CHECK(free_bytes + live_bytes == cap);
        if (g_fail) return;
    }
    for (const Live &l : live) al.release(l.p, l.n);
    CHECK(al.free_blocks().size() == 1 && al.free_blocks().begin()->second == cap);
    CHECK(al.alloc(cap) == buf.data());
    CHECK(al.alloc(1) == nullptr);
}

int main() {
    blocks();
    bump();
    first_fit();
    if (g_fail) {
        std::printf("host units: %d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host units: ok\n");
    return 0;
}
