// One Delaunay (or Voronoi) densification step (paper Sec. 4.1, Alg. 1) on the
// GPU, and its C-ABI entry point.
//
// Exact discrete reading of the step, all in integer arithmetic so that the
// result is reproducible bit for bit:
//   1 labels     nearest mask pixel of every pixel, by (squared distance,
//                linear index); the paper builds this Voronoi diagram to get
//                the Delaunay triangulation (Sec. 4.2)
//   2 triangles  every 2x2 pixel quad whose corners carry three or four
//                different labels gives one or two triangles of mask pixels;
//                the sorted index triple is the key, duplicates are merged and
//                collinear triples dropped
//   3 ownership  a pixel belongs to the covering closed triangle with the
//                smallest key, or, if none covers it, to its Voronoi cell
//   4 errors     cell sums of round(e * 2^20) (64-bit integers)
//   5 ranking    cells by (sum descending, key ascending)
//   6 selection  in ranked order, each cell with a free pixel adds its free
//                pixel of largest error (ties to the smaller index), until
//                n_add pixels are added (Alg. 1: at most one per triangle)
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <climits>

#include "hdi_internal.h"

namespace hdi {

void launch_compact(int N, const uint8_t *mask, int *chunk_cnt, int *chunk_off, int *total, int *idx, int *pos,
                    hipStream_t s);

constexpr int SEG = 64;   // rows per column segment of the column pass

// ------------------------------------------------------------------ 1 labels

// Nearest mask pixel in the same column, inside one segment of SEG rows;
// seg_first/seg_last record the first and last mask rows of the segment.
__global__ void k_col_seg(int W, int H, int nseg, const uint8_t *__restrict__ mask, int *__restrict__ colnear,
                          int *__restrict__ seg_first, int *__restrict__ seg_last) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * nseg) return;
    const int x = t % W, sg = t / W;
    const int y0 = sg * SEG, y1 = min(y0 + SEG, H);
    int last = -1, first = -1;
    for (int y = y0; y < y1; ++y) {           // downward: nearest at or above
        if (mask[(size_t)y * W + x]) { last = y; if (first < 0) first = y; }
        colnear[(size_t)y * W + x] = last;
    }
    seg_first[sg * W + x] = first;
    seg_last[sg * W + x] = last;
    int below = -1;
    for (int y = y1 - 1; y >= y0; --y) {       // upward: nearest at or below
        if (mask[(size_t)y * W + x]) below = y;
        const int above = colnear[(size_t)y * W + x];
        int best = above;
        // (|dy|, row) order: the upper one wins a tie (smaller index)
        if (below >= 0 && (best < 0 || below - y < y - best)) best = below;
        colnear[(size_t)y * W + x] = best;
    }
}

// Combine with the nearest mask rows outside the segment.
__global__ void k_col_fix(int W, int H, int nseg, const int *__restrict__ seg_first, const int *__restrict__ seg_last,
                          int *__restrict__ colnear) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * nseg) return;
    const int x = t % W, sg = t / W;
    int above = -1, below = -1;
    for (int k = sg - 1; k >= 0 && above < 0; --k) above = seg_last[k * W + x];
    for (int k = sg + 1; k < nseg && below < 0; ++k) below = seg_first[k * W + x];
    if (above < 0 && below < 0) return;
    const int y0 = sg * SEG, y1 = min(y0 + SEG, H);
    for (int y = y0; y < y1; ++y) {
        int best = colnear[(size_t)y * W + x];
        const int db = best < 0 ? INT_MAX : abs(best - y);
        int cand = best, dc = db;
        if (above >= 0 && (y - above < dc || (y - above == dc && above < cand))) { cand = above; dc = y - above; }
        if (below >= 0 && (below - y < dc || (below - y == dc && below < cand))) { cand = below; dc = below - y; }
        colnear[(size_t)y * W + x] = cand;
    }
}

// label(p) = argmin over columns x' of (dx^2 + dy^2, index) using each column's
// nearest mask row; scanning outwards from x until dx^2 exceeds the best.
__global__ void k_labels(int W, int H, const int *__restrict__ colnear, int *__restrict__ labels) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    const int x = i % W, y = i / W;
    long long bd = LLONG_MAX;
    int bi = INT_MAX;
    const int *row = colnear + (size_t)y * W;
    for (int dx = 0; dx < W; ++dx) {
        const long long dx2 = (long long)dx * dx;
        if (dx2 > bd) break;
        const int xs[2] = {x - dx, x + dx};
        for (int k = 0; k < (dx ? 2 : 1); ++k) {
            const int xx = xs[k];
            if (xx < 0 || xx >= W) continue;
            const int ys = row[xx];
            if (ys < 0) continue;
            const long long d = dx2 + (long long)(ys - y) * (ys - y);
            const int idx = ys * W + xx;
            if (d < bd || (d == bd && idx < bi)) { bd = d; bi = idx; }
        }
    }
    labels[i] = bi;
}

// Jump flooding (Sec. 4.2, after Rong and Tan): labels start as the pixel's own
// index on mask pixels and -1 elsewhere; a pass with step k gives every pixel
// the best label held before the pass at the nine pixels p + k (i, j),
// i, j in {-1, 0, 1}, by (squared distance, index). Integer-exact, so the
// result depends only on the mask and the steps.
__global__ void k_jfa_init(int N, const uint8_t *__restrict__ mask, int *__restrict__ lab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) lab[i] = mask[i] ? i : -1;
}

__global__ void k_jfa_pass(int W, int H, int k, const int *__restrict__ in, int *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    const int x = i % W, y = i / W;
    long long bd = LLONG_MAX;
    int bl = -1;
    for (int dy = -k; dy <= k; dy += k) {
        const int ny = y + dy;
        if (ny < 0 || ny >= H) continue;
        for (int dx = -k; dx <= k; dx += k) {
            const int nx = x + dx;
            if (nx < 0 || nx >= W) continue;
            const int c = in[ny * W + nx];
            if (c < 0) continue;
            const long long ex = c % W - x, ey = c / W - y;
            const long long d = ex * ex + ey * ey;
            if (d < bd || (d == bd && c < bl)) { bd = d; bl = c; }
        }
    }
    out[i] = bl;
}

// out[0]: the largest squared distance from a pixel to its label; out[1] is
// set if a pixel has no label (jump flooding from too small a start step).
// Grid-stride over RED_BLOCKS workgroups of 256 threads, one atomic each.
constexpr int RED_BLOCKS = 1024;
__global__ void __launch_bounds__(256)
k_label_max_d2(int W, int H, const int *__restrict__ lab, unsigned long long *__restrict__ out) {
    unsigned long long m = 0, none = 0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < (long)W * H; i += (long)RED_BLOCKS * 256) {
        const int l = lab[i];
        if (l < 0) {
            none = 1;
            continue;
        }
        const long long ex = l % W - i % W, ey = l / W - i / W;
        m = max(m, (unsigned long long)(ex * ex + ey * ey));
    }
    __shared__ unsigned long long sm[256], sn[256];
    sm[threadIdx.x] = m;
    sn[threadIdx.x] = none;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + h]);
            sn[threadIdx.x] |= sn[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(out, sm[0]);
        if (sn[0]) atomicOr(out + 1, 1ull);
    }
}

// ------------------------------------------------------------------ 2 triangles

__device__ __forceinline__ long long orient(int W, int a, int b, int c) {
    const long long ax = a % W, ay = a / W, bx = b % W, by = b / W, cx = c % W, cy = c / W;
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// A candidate triangle: its labels in increasing order; false if collinear.
__device__ __forceinline__ bool make_tri(int W, int a, int b, int c, int3 &t) {
    if (a > b) { const int u = a; a = b; b = u; }
    if (b > c) { const int u = b; b = c; c = u; }
    if (a > b) { const int u = a; a = b; b = u; }
    t = make_int3(a, b, c);
    return orient(W, a, b, c) != 0;
}

// Each quad of 2x2 pixels with three distinct labels gives one triangle, with
// four (l0 l1 l2 l3 around the quad) the two triangles l0 l1 l2 and l0 l2 l3.
__device__ __forceinline__ void quad_tris(int W, int H, const int *__restrict__ labels, int i, int3 &t0, int3 &t1,
                                          bool &e0, bool &e1) {
    e0 = e1 = false;
    if (i >= (W - 1) * (H - 1)) return;
    const int x = i % (W - 1), y = i / (W - 1);
    const int l0 = labels[y * W + x], l1 = labels[y * W + x + 1];
    const int l2 = labels[(y + 1) * W + x + 1], l3 = labels[(y + 1) * W + x];
    const int nd = 1 + (l1 != l0) + (l2 != l0 && l2 != l1) + (l3 != l0 && l3 != l1 && l3 != l2);
    if (nd == 4) {
        e0 = make_tri(W, l0, l1, l2, t0);
        e1 = make_tri(W, l0, l2, l3, t1);
    } else if (nd == 3) {
        // the three distinct labels
        int a = l0, b, c;
        b = (l1 != a) ? l1 : l2;
        const int cands[3] = {l1, l2, l3};
        c = a;
        for (int k = 0; k < 3; ++k)
            if (cands[k] != a && cands[k] != b) c = cands[k];
        e0 = make_tri(W, a, b, c, t0);
    }
}

// The triangles are listed without a shared counter (same-address atomics
// serialise): k_quads_count counts each workgroup's triangles, an exclusive
// scan gives every workgroup its offset, and k_quads_write evaluates the quads
// again and writes the triangles there, wavefront by wavefront (the order in
// the list is arbitrary: the triangles are sorted and merged afterwards).
// Every lane takes part in the ballots, also those past the last quad.
__global__ void __launch_bounds__(256)
k_quads_count(int W, int H, const int *__restrict__ labels, int *__restrict__ block_count) {
    int3 t0, t1;
    bool e0, e1;
    quad_tris(W, H, labels, blockIdx.x * blockDim.x + threadIdx.x, t0, t1, e0, e1);
    const int n = __popcll(__ballot(e0)) + __popcll(__ballot(e1));
    __shared__ int s_n[4];
    if ((threadIdx.x & 63) == 0) s_n[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) block_count[blockIdx.x] = s_n[0] + s_n[1] + s_n[2] + s_n[3];
}

__global__ void __launch_bounds__(256)
k_quads_write(int W, int H, const int *__restrict__ labels, const int *__restrict__ block_count,
              const int *__restrict__ block_off, int *__restrict__ ta, int *__restrict__ tb, int *__restrict__ tc,
              unsigned int *__restrict__ total) {
    int3 t0 = make_int3(0, 0, 0), t1 = make_int3(0, 0, 0);
    bool e0, e1;
    quad_tris(W, H, labels, blockIdx.x * blockDim.x + threadIdx.x, t0, t1, e0, e1);
    const unsigned long long m0 = __ballot(e0), m1 = __ballot(e1);
    const int n0 = __popcll(m0), n = n0 + __popcll(m1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ int s_n[4];
    if (lane == 0) s_n[w] = n;
    __syncthreads();
    int base = block_off[blockIdx.x];
    for (int k = 0; k < w; ++k) base += s_n[k];
    const unsigned long long below = (1ull << lane) - 1ull;
    if (e0) {
        const int k = base + __popcll(m0 & below);
        ta[k] = t0.x;
        tb[k] = t0.y;
        tc[k] = t0.z;
    }
    if (e1) {
        const int k = base + n0 + __popcll(m1 & below);
        ta[k] = t1.x;
        tb[k] = t1.y;
        tc[k] = t1.z;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *total = (unsigned int)(block_off[blockIdx.x] + block_count[blockIdx.x]);
}

// out = a[0] + b[0] (the last exclusive offset plus the last flag: a count)
__global__ void k_last_sum(const int *__restrict__ a, const int *__restrict__ b, int *__restrict__ out) {
    if (threadIdx.x == 0) *out = *a + *b;
}

__global__ void k_iota(int n, int *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ void k_key_c(int n, const int *__restrict__ tc, unsigned int *__restrict__ key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = (unsigned int)tc[i];
}

__global__ void k_key_ab(int n, const int *__restrict__ order, const int *__restrict__ ta, const int *__restrict__ tb,
                         unsigned long long *__restrict__ key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int j = order[i];
        key[i] = ((unsigned long long)(unsigned int)ta[j] << 32) | (unsigned int)tb[j];
    }
}

// flag[i] = 1 if the i-th triangle in sorted order differs from the previous
__global__ void k_uniq_flags(int n, const int *__restrict__ order, const int *__restrict__ ta,
                             const int *__restrict__ tb, const int *__restrict__ tc, int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = order[i];
    int f = 1;
    if (i > 0) {
        const int k = order[i - 1];
        f = (ta[j] != ta[k]) || (tb[j] != tb[k]) || (tc[j] != tc[k]);
    }
    flag[i] = f;
}

__global__ void k_uniq_scatter(int n, const int *__restrict__ order, const int *__restrict__ flag,
                               const int *__restrict__ off, const int *__restrict__ ta, const int *__restrict__ tb,
                               const int *__restrict__ tc, int *__restrict__ ua, int *__restrict__ ub,
                               int *__restrict__ uc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int j = order[i], r = off[i];
    ua[r] = ta[j];
    ub[r] = tb[j];
    uc[r] = tc[j];
}

// ------------------------------------------------------------------ 3 ownership

__global__ void k_fill_i32(int n, int v, int *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(int n, unsigned long long *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Whether any mask pixel is set (count > 0 afterwards): one atomic per wave
// that sees one, and waves stop looking once the count is positive.
__global__ void k_count_set(int N, const uint8_t *__restrict__ m, unsigned long long *__restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool set = i < N && m[i] != 0;
    const unsigned long long b = __ballot(set);
    if ((threadIdx.x & 63) == 0 && b && __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicAdd(count, (unsigned long long)__popcll(b));
}

// Closed-triangle coverage with the smallest rank winning (ranks follow the
// key order). One thread per triangle walks its bounding box.
// Ownership: every pixel inside or on a triangle takes the smallest index of
// those triangles. RASTER_LANES lanes share a triangle and stride over the
// pixels of its bounding box, so large triangles (sparse regions) do not hold
// a whole wavefront up. I: the integer type of the edge functions; int suffices
// while 2 W H < 2^31 (each product of coordinate differences is at most W H).
constexpr int RASTER_LANES = 16;
template <typename I>
__global__ void k_raster(int W, int T, const int *__restrict__ ua, const int *__restrict__ ub,
                         const int *__restrict__ uc, int *__restrict__ owner) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(g / RASTER_LANES), sub = (int)(g % RASTER_LANES);
    if (r >= T) return;
    I ax = ua[r] % W, ay = ua[r] / W, bx = ub[r] % W, by = ub[r] / W, cx = uc[r] % W, cy = uc[r] / W;
    if ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax) < 0) {
        I t = bx; bx = cx; cx = t;
        t = by; by = cy; cy = t;
    }
    const I x0 = min(ax, min(bx, cx)), x1 = max(ax, max(bx, cx));
    const I y0 = min(ay, min(by, cy)), y1 = max(ay, max(by, cy));
    const I bw = x1 - x0 + 1, area = bw * (y1 - y0 + 1);
    for (I k = sub; k < area; k += RASTER_LANES) {
        const I y = y0 + k / bw, x = x0 + k % bw;
        const I e0 = (bx - ax) * (y - ay) - (by - ay) * (x - ax);
        const I e1 = (cx - bx) * (y - by) - (cy - by) * (x - bx);
        const I e2 = (ax - cx) * (y - cy) - (ay - cy) * (x - cx);
        if (e0 >= 0 && e1 >= 0 && e2 >= 0) atomicMin(&owner[y * W + x], r);
    }
}

// ------------------------------------------------------------------ 4 cell errors and argmax

__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, int d) {
    const int lo = __shfl_up((int)(unsigned)v, d, 64), hi = __shfl_up((int)(unsigned)(v >> 32), d, 64);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Each pixel adds its error (fixed point, 2^-20) to its cell and offers its
// argmax key. Runs of lanes with the same cell (cells are spatially coherent,
// so neighbouring pixels mostly share one) are combined first by a segmented
// scan in lane order, and only the last lane of a run issues the atomics:
// integer sums and maxima, so the result does not depend on how the pixels
// are grouped.
__global__ void k_cells(int N, int T, const int *__restrict__ owner, const int *__restrict__ labels,
                        const int *__restrict__ seed_pos, const uint8_t *__restrict__ mask, const float *__restrict__ err,
                        unsigned long long *__restrict__ E, unsigned long long *__restrict__ best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int cell = -1 - lane;   // lanes past the end: a run of their own each
    unsigned long long q = 0, key = 0;
    if (i < N) {
        const int o = owner ? owner[i] : INT_MAX;
        cell = o < T ? o : T + seed_pos[labels[i]];
        const float e = err[i];
        q = (unsigned long long)rint(ldexp((double)e, 20));
        if (!mask[i]) {
            // larger error first, then smaller index; e >= 0 so its bits order like its value,
            // once -0 (accepted as e >= 0, but with the sign bit set) is made +0
            const unsigned eb = e == 0.f ? 0u : __float_as_uint(e);
            key = ((unsigned long long)eb << 32) | (0xFFFFFFFFu - (unsigned)i);
        }
    }
    // (every lane executes every shuffle: a lane that skipped one would leave
    // its value undefined for the lanes reading it)
    const int cprev = __shfl_up(cell, 1, 64), cnext = __shfl_down(cell, 1, 64);
    int head = lane == 0 || cprev != cell;
    for (int d = 1; d < 64; d <<= 1) {
        const int ho = __shfl_up(head, d, 64);
        const unsigned long long qo = shfl_up_u64(q, d), ko = shfl_up_u64(key, d);
        if (lane >= d && !head) {
            q += qo;
            key = ko > key ? ko : key;
            head = ho;
        }
    }
    const bool last = lane == 63 || cnext != cell;
    if (last && cell >= 0) {
        if (q) atomicAdd(&E[cell], q);
        if (key) atomicMax(&best[cell], key);
    }
}

__global__ void k_rank_keys(int n, const unsigned long long *__restrict__ E, unsigned long long *__restrict__ key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = ~E[i];
}

// ------------------------------------------------------------------ 6 selection

__global__ void k_nonempty(int n, const int *__restrict__ order, const unsigned long long *__restrict__ best,
                           int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = best[order[i]] != 0ull;
}

__global__ void k_select(int n, long long n_add, const int *__restrict__ order, const unsigned long long *__restrict__ best,
                         const int *__restrict__ flag, const int *__restrict__ off, uint8_t *__restrict__ newpix) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i] || off[i] >= n_add) return;
    const unsigned int p = 0xFFFFFFFFu - (unsigned int)(best[order[i]] & 0xFFFFFFFFull);
    newpix[p] = 1;
}

__global__ void k_apply(int N, const uint8_t *__restrict__ newpix, uint8_t *__restrict__ mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && newpix[i]) mask[i] = 1;
}

__global__ void k_copy_i32(int n, const int *__restrict__ a, int *__restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------------ host

// flag[0] = 1 if an error value is negative, not finite or above emax (the
// bound that keeps the 2^-20 fixed-point cell sums exact in 64 bits)
__global__ void k_check_err(int N, const float *__restrict__ err, float emax, int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float e = err[i];
    if (!(e >= 0.f && e <= emax)) flag[0] = 1;
}

static inline dim3 gd(long n) { return dim3((unsigned)std::max<long>(1, (n + 255) / 256)); }

size_t voronoi_scratch_ints(int W, int H) {
    return (size_t)W * H + 2 * (size_t)((H + SEG - 1) / SEG) * W;
}

int jfa_default_step(int W, int H) {
    const int n = std::max(W, H);
    int k = 1;
    while (2 * k < n) k *= 2;
    return n > 1 ? k : 0;
}

void launch_jfa_labels(int W, int H, const uint8_t *mask, int k0, int *scratch, int *labels, hipStream_t s) {
    const int N = W * H;
    int passes = 0;
    for (int k = k0; k >= 1; k /= 2) ++passes;
    // ping-pong so that the last pass writes into labels
    int *a = (passes % 2 == 0) ? labels : scratch, *b = (passes % 2 == 0) ? scratch : labels;
    hipLaunchKernelGGL(k_jfa_init, gd(N), dim3(256), 0, s, N, mask, a);
    for (int k = k0; k >= 1; k /= 2) {
        hipLaunchKernelGGL(k_jfa_pass, gd(N), dim3(256), 0, s, W, H, k, a, b);
        std::swap(a, b);
    }
}

void launch_label_max_d2(int W, int H, const int *labels, unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, 2, out);
    hipLaunchKernelGGL(k_label_max_d2, dim3(RED_BLOCKS), dim3(256), 0, s, W, H, labels, out);
}

void launch_voronoi_labels(int W, int H, const uint8_t *mask, int *scratch, int *labels, hipStream_t s) {
    const int N = W * H, nseg = (H + SEG - 1) / SEG;
    int *colnear = scratch, *seg_first = scratch + N, *seg_last = seg_first + (size_t)nseg * W;
    hipLaunchKernelGGL(k_col_seg, gd((long)W * nseg), dim3(256), 0, s, W, H, nseg, mask, colnear, seg_first,
                       seg_last);
    hipLaunchKernelGGL(k_col_fix, gd((long)W * nseg), dim3(256), 0, s, W, H, nseg, seg_first, seg_last, colnear);
    hipLaunchKernelGGL(k_labels, gd(N), dim3(256), 0, s, W, H, colnear, labels);
}

struct DensWs {
    int *colnear, *labels, *owner;   // colnear: voronoi_scratch_ints(W, H) ints
    int *seed_idx, *seed_pos, *chunk_cnt, *chunk_off, *total;
    int *ta, *tb, *tc, *ua, *ub, *uc;
    int *ord0, *ord1, *flag, *off;
    unsigned int *keyc0, *keyc1, *count;
    unsigned long long *keyab0, *keyab1, *E, *best, *rk0, *rk1, *maxd2;
    uint8_t *newpix;
    void *tmp;
    size_t tmp_bytes;
};

// Temporary storage of the rocPRIM radix sorts (32- and 64-bit keys with int
// values) and the exclusive int scan for up to maxn items.
static size_t sort_tmp_bytes(int maxn) {
    size_t a = 0, b = 0, c = 0;
    (void)rocprim::radix_sort_pairs(nullptr, a, (unsigned int *)nullptr, (unsigned int *)nullptr, (int *)nullptr,
                                    (int *)nullptr, maxn);
    (void)rocprim::radix_sort_pairs(nullptr, b, (unsigned long long *)nullptr, (unsigned long long *)nullptr,
                                    (int *)nullptr, (int *)nullptr, maxn);
    (void)rocprim::exclusive_scan(nullptr, c, (int *)nullptr, (int *)nullptr, 0, (size_t)maxn, rocprim::plus<int>());
    return std::max(std::max(a, b), c);
}

// Exclusive prefix sum of n ints on the stream.
static hipError_t scan_exclusive(void *tmp, size_t tmp_bytes, const int *in, int *out, int n, hipStream_t s) {
    return rocprim::exclusive_scan(tmp, tmp_bytes, in, out, 0, (size_t)n, rocprim::plus<int>(), s);
}

static bool plan_densify(DensWs &d, Arena &a, int W, int H) {
    const size_t N = (size_t)W * H;
    const size_t maxT = 2 * (size_t)std::max(W - 1, 1) * std::max(H - 1, 1);
    const size_t maxC = maxT + N;   // triangles + Voronoi cells
    d.colnear = (int *)a.take(voronoi_scratch_ints(W, H) * 4);
    d.labels = (int *)a.take(N * 4);
    d.owner = (int *)a.take(N * 4);
    d.seed_idx = (int *)a.take(N * 4);
    d.seed_pos = (int *)a.take(N * 4);
    d.chunk_cnt = (int *)a.take(((N + 1023) / 1024) * 4);
    d.chunk_off = (int *)a.take(((N + 1023) / 1024) * 4);
    d.total = (int *)a.take(16);
    int **t3[] = {&d.ta, &d.tb, &d.tc, &d.ua, &d.ub, &d.uc};
    for (int **p : t3) *p = (int *)a.take(maxT * 4);
    d.ord0 = (int *)a.take(maxC * 4);
    d.ord1 = (int *)a.take(maxC * 4);
    d.flag = (int *)a.take(maxC * 4);
    d.off = (int *)a.take(maxC * 4);
    d.keyc0 = (unsigned int *)a.take(maxT * 4);
    d.keyc1 = (unsigned int *)a.take(maxT * 4);
    d.count = (unsigned int *)a.take(16);
    d.maxd2 = (unsigned long long *)a.take(16);
    d.keyab0 = (unsigned long long *)a.take(maxT * 8);
    d.keyab1 = (unsigned long long *)a.take(maxT * 8);
    d.E = (unsigned long long *)a.take(maxC * 8);
    d.best = (unsigned long long *)a.take(maxC * 8);
    d.rk0 = (unsigned long long *)a.take(maxC * 8);
    d.rk1 = (unsigned long long *)a.take(maxC * 8);
    d.newpix = (uint8_t *)a.take((N + 3) & ~(size_t)3);   // zeroed in 4-byte words
    d.tmp_bytes = sort_tmp_bytes((int)maxC);
    d.tmp = a.take(d.tmp_bytes);
    return a.base == nullptr || a.used <= a.size;
}

static size_t densify_ws_bytes(int W, int H) {
    DensWs d;
    Arena a{nullptr, 0, 0};
    plan_densify(d, a, W, H);
    return a.used + 256;
}

#define D_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

static int32_t run_densify(DensWs &d, int W, int H, uint8_t *mask, const float *err, long long n_add, int partition,
                           int jfa_k0, int32_t *added, int64_t *n_added, uint64_t *max_d2, hipStream_t s) {
    const bool jfa = (partition & HDI_PART_JFA) != 0;
    partition &= ~HDI_PART_JFA;
    const int N = W * H;
    // seeds in ascending order (the Voronoi cell order) and their ranks
    launch_compact(N, mask, d.chunk_cnt, d.chunk_off, d.total, d.seed_idx, d.seed_pos, s);
    const float emax = (float)std::min(std::ldexp(1.0, 43) / N, 3.0e38);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, 1, 0, d.total + 1);
    hipLaunchKernelGGL(k_check_err, gd(N), dim3(256), 0, s, N, err, emax, d.total + 1);
    int mb[2] = {0, 0};
    D_TRY(read_to_host(mb, d.total, 2 * sizeof(int), s));
    const int m = mb[0];
    if (m == 0) {
        set_error("empty mask: densification needs at least one mask pixel");
        return HDI_ERR_EMPTY_MASK;
    }
    if (mb[1]) {
        set_error("error map holds a value that is negative, not finite or above %g", (double)emax);
        return HDI_ERR_ARG;
    }
    // 1 labels (exact, or by jump flooding)
    if (jfa) {
        launch_jfa_labels(W, H, mask, jfa_k0 > 0 ? jfa_k0 : jfa_default_step(W, H), d.colnear, d.labels, s);
        // every later stage indexes by label: refuse unlabelled pixels
        launch_label_max_d2(W, H, d.labels, d.maxd2, s);
        unsigned long long r[2] = {0, 0};
        D_TRY(read_to_host(r, d.maxd2, sizeof r, s));
        if (r[1]) {
            set_error("jump flooding from step %d left pixels without a label", jfa_k0);
            return HDI_ERR_ARG;
        }
    } else {
        launch_voronoi_labels(W, H, mask, d.colnear, d.labels, s);
        if (max_d2) launch_label_max_d2(W, H, d.labels, d.maxd2, s);
    }
    int T = 0;
    if (partition == HDI_PART_DELAUNAY && W > 1 && H > 1) {
        // 2 triangles: emit, sort by (a, b, c) with two stable radix passes, merge duplicates
        // (the block counts and offsets use the triangle flag and offset arrays,
        // free until the merge below)
        const long nq = (long)(W - 1) * (H - 1);
        const int nqb = (int)((nq + 255) / 256);
        hipLaunchKernelGGL(k_quads_count, dim3(nqb), dim3(256), 0, s, W, H, d.labels, d.flag);
        size_t tq = d.tmp_bytes;
        D_TRY(scan_exclusive(d.tmp, tq, d.flag, d.off, nqb, s));
        hipLaunchKernelGGL(k_quads_write, dim3(nqb), dim3(256), 0, s, W, H, d.labels, d.flag, d.off, d.ta, d.tb, d.tc,
                           d.count);
        unsigned int nt = 0;
        D_TRY(read_to_host(&nt, d.count, sizeof(unsigned int), s));
        if (nt > 0) {
            const int n = (int)nt;
            hipLaunchKernelGGL(k_iota, gd(n), dim3(256), 0, s, n, d.ord0);
            hipLaunchKernelGGL(k_key_c, gd(n), dim3(256), 0, s, n, d.tc, d.keyc0);
            size_t tb = d.tmp_bytes;
            D_TRY(rocprim::radix_sort_pairs(d.tmp, tb, d.keyc0, d.keyc1, d.ord0, d.ord1, n, 0u, 32u, s));
            hipLaunchKernelGGL(k_key_ab, gd(n), dim3(256), 0, s, n, d.ord1, d.ta, d.tb, d.keyab0);
            tb = d.tmp_bytes;
            D_TRY(rocprim::radix_sort_pairs(d.tmp, tb, d.keyab0, d.keyab1, d.ord1, d.ord0, n, 0u, 64u, s));
            hipLaunchKernelGGL(k_uniq_flags, gd(n), dim3(256), 0, s, n, d.ord0, d.ta, d.tb, d.tc, d.flag);
            tb = d.tmp_bytes;
            D_TRY(scan_exclusive(d.tmp, tb, d.flag, d.off, n, s));
            hipLaunchKernelGGL(k_uniq_scatter, gd(n), dim3(256), 0, s, n, d.ord0, d.flag, d.off, d.ta, d.tb, d.tc,
                               d.ua, d.ub, d.uc);
            // the number of distinct triangles, read back in one copy
            hipLaunchKernelGGL(k_last_sum, dim3(1), dim3(64), 0, s, d.off + n - 1, d.flag + n - 1, (int *)d.count);
            D_TRY(read_to_host(&T, d.count, sizeof(int), s));
        }
        // 3 ownership
        hipLaunchKernelGGL(k_fill_i32, gd(N), dim3(256), 0, s, N, INT_MAX, d.owner);
        if (T > 0 && 2LL * W * H < (1LL << 31))
            hipLaunchKernelGGL(k_raster<int>, gd((long)T * RASTER_LANES), dim3(256), 0, s, W, T, d.ua, d.ub, d.uc,
                               d.owner);
        else if (T > 0)
            hipLaunchKernelGGL(k_raster<long long>, gd((long)T * RASTER_LANES), dim3(256), 0, s, W, T, d.ua, d.ub,
                               d.uc, d.owner);
    }
    // 4 cell sums and argmax
    const int ncell = T + m;
    hipLaunchKernelGGL(k_fill_u64, gd(ncell), dim3(256), 0, s, ncell, d.E);
    hipLaunchKernelGGL(k_fill_u64, gd(ncell), dim3(256), 0, s, ncell, d.best);
    hipLaunchKernelGGL(k_cells, gd(N), dim3(256), 0, s, N, T, T > 0 ? d.owner : (const int *)nullptr, d.labels,
                       d.seed_pos, mask, err, d.E, d.best);
    // 5 ranking: E descending, cell order ascending (stable radix sort of ~E)
    hipLaunchKernelGGL(k_rank_keys, gd(ncell), dim3(256), 0, s, ncell, d.E, d.rk0);
    hipLaunchKernelGGL(k_iota, gd(ncell), dim3(256), 0, s, ncell, d.ord0);
    size_t tb = d.tmp_bytes;
    D_TRY(rocprim::radix_sort_pairs(d.tmp, tb, d.rk0, d.rk1, d.ord0, d.ord1, ncell, 0u, 64u, s));
    // 6 selection
    hipLaunchKernelGGL(k_nonempty, gd(ncell), dim3(256), 0, s, ncell, d.ord1, d.best, d.flag);
    tb = d.tmp_bytes;
    D_TRY(scan_exclusive(d.tmp, tb, d.flag, d.off, ncell, s));
    hipLaunchKernelGGL(k_fill_i32, gd((N + 3) / 4), dim3(256), 0, s, (N + 3) / 4, 0, (int *)d.newpix);
    hipLaunchKernelGGL(k_select, gd(ncell), dim3(256), 0, s, ncell, n_add, d.ord1, d.best, d.flag, d.off, d.newpix);
    hipLaunchKernelGGL(k_apply, gd(N), dim3(256), 0, s, N, d.newpix, mask);
    // added pixels in ascending order: compaction of the new-pixel flags
    launch_compact(N, d.newpix, d.chunk_cnt, d.chunk_off, d.total, d.seed_idx, d.seed_pos, s);
    int na = 0;
    D_TRY(read_to_host(&na, d.total, sizeof(int), s));
    if (added && na > 0) hipLaunchKernelGGL(k_copy_i32, gd(na), dim3(256), 0, s, na, d.seed_idx, added);
    if (max_d2) D_TRY(hipMemcpyAsync(max_d2, d.maxd2, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    D_TRY(hipGetLastError());
    D_TRY(wait_for(s));
    *n_added = na;
    return HDI_OK;
}

int32_t densify_step_ex(int W, int H, uint8_t *mask, const float *err, long long n_add, int partition, int jfa_k0,
                        int32_t *added, int64_t *n_added, uint64_t *max_d2, void *ws, size_t ws_bytes, hipStream_t s) {
    hdi_image img{W, H, 1};
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !err || !n_added) {
        set_error("mask, err and n_added must be non-null");
        return HDI_ERR_ARG;
    }
    const int base = partition & ~HDI_PART_JFA;
    if (n_add < 0 || (base != HDI_PART_DELAUNAY && base != HDI_PART_VORONOI) || jfa_k0 < 0 ||
        (jfa_k0 & (jfa_k0 - 1))) {
        set_error("n_add must be >= 0, partition HDI_PART_DELAUNAY or HDI_PART_VORONOI (optionally | HDI_PART_JFA) "
                  "and a jump-flooding start a power of two");
        return HDI_ERR_ARG;
    }
    const size_t need = densify_ws_bytes(W, H);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    Arena a{(char *)ws, ws_bytes, 0};
    DensWs d;
    plan_densify(d, a, W, H);
    return run_densify(d, W, H, mask, err, n_add, partition, jfa_k0, added, n_added, max_d2, s);
}

// Error map of the densification loop: e = fp32(sum_c (u_c - f_c)^2), summed in
// FP64 in channel order and rounded once to nearest. Explicit _rn operations
// keep the compiler from contracting the square and the sum into an FMA.
__global__ void k_error_map(int N, int C, const double *__restrict__ u, const float *__restrict__ f,
                            float *__restrict__ e) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int c = 0; c < C; ++c) {
        const double d = __dsub_rn(u[(size_t)c * N + i], (double)f[(size_t)c * N + i]);
        acc = __dadd_rn(acc, __dmul_rn(d, d));
    }
    e[i] = __double2float_rn(acc);
}

}  // namespace hdi

using namespace hdi;

extern "C" {

int32_t hdi_error_map(hdi_image img, const double *u, const float *f, float *err, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!u || !f || !err) {
        set_error("u, f and err must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    const int N = img.width * img.height;
    hipLaunchKernelGGL(k_error_map, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, N, img.channels, u, f,
                       err);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("error map launch failed: %s", hipGetErrorString(e));
        return HDI_ERR_HIP;
    }
    return HDI_OK;
}

size_t hdi_densify_workspace_bytes(int32_t width, int32_t height) {
    if (width < 1 || height < 1 || (int64_t)width * height > (int64_t)1 << 30) return 0;
    return densify_ws_bytes(width, height);
}

int32_t densify_step(int32_t width, int32_t height, uint8_t *mask, const float *err, int64_t n_add,
                     int32_t partition, int32_t *added, int64_t *n_added, void *ws, size_t ws_bytes, void *stream) {
    return densify_step_ex(width, height, mask, err, n_add, partition, 0, added, n_added, nullptr, ws, ws_bytes,
                           (hipStream_t)stream);
}

size_t hdi_labels_workspace_bytes(int32_t width, int32_t height) {
    if (width < 1 || height < 1 || (int64_t)width * height > (int64_t)1 << 30) return 0;
    return voronoi_scratch_ints(width, height) * sizeof(int) + 2 * 256;
}

int32_t hdi_voronoi_labels(int32_t width, int32_t height, const uint8_t *mask, int32_t *labels, int32_t jfa_step,
                           uint64_t *max_d2, void *ws, size_t ws_bytes, void *stream) {
    hdi_image img{width, height, 1};
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !labels) {
        set_error("mask and labels must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    if (jfa_step < -1 || (jfa_step > 0 && (jfa_step & (jfa_step - 1)))) {
        set_error("jfa_step must be 0 (exact), -1 (jump flooding from the default step) or a power of two");
        return HDI_ERR_ARG;
    }
    const size_t need = hdi_labels_workspace_bytes(width, height);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    const int N = width * height;
    Arena a{(char *)ws, ws_bytes, 0};
    int *scratch = (int *)a.take(voronoi_scratch_ints(width, height) * sizeof(int));
    unsigned long long *slot = (unsigned long long *)a.take(32);
    // an empty mask has no labels
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, 4, slot);
    hipLaunchKernelGGL(k_count_set, gd(N), dim3(256), 0, s, N, mask, slot + 2);
    unsigned long long cnt = 0;
    D_TRY(read_to_host(&cnt, slot + 2, sizeof cnt, s));
    if (cnt == 0) {
        set_error("empty mask: no labels");
        return HDI_ERR_EMPTY_MASK;
    }
    if (jfa_step == 0)
        launch_voronoi_labels(width, height, mask, scratch, labels, s);
    else
        launch_jfa_labels(width, height, mask, jfa_step > 0 ? jfa_step : jfa_default_step(width, height), scratch,
                          labels, s);
    if (max_d2) {
        launch_label_max_d2(width, height, labels, slot, s);
        D_TRY(hipMemcpyAsync(max_d2, slot, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    }
    D_TRY(hipGetLastError());
    D_TRY(wait_for(s));
    return HDI_OK;
}

}  // extern "C"
