// Linear BVH over triangles for gfx950.
//
// The paper accelerates ray casting with a kD-tree searched recursively on the
// CPU (Sec. 5.1).  Here the structure is a binary LBVH built entirely on the
// GPU, one thread per triangle or node:
//   0. a check of the copied mesh (indices in range, finite coordinates);
//   1. vertex bounds and centroid bounds (ordered-integer atomics);
//   2. 63-bit Morton codes of the centroids (21 bits per axis, one cell size);
//   3. a stable LSD radix sort (8 bits per pass, 4096-key tiles, wave64
//      ballot matching for stable in-tile ranks);
//   4. the binary radix tree of Karras (2012), "Maximizing parallelism in the
//      construction of BVHs, octrees, and k-d trees" (equal keys ordered by
//      their sorted position);
//   5. leaf records gathered in sorted order (48 B: three vertices + original id);
//   6. internal nodes grouped by depth (a per-block LDS histogram, then one
//      global slot grab per block and depth); the deepest internal node's
//      depth + 1 is the deepest leaf, which bounds the traversal stack;
//   7. child boxes, one launch per depth, deepest first: a child's box is its
//      triangle's or the union of the boxes the child holds, written one launch
//      earlier.  A bottom-up pass with per-node arrival counters needs an
//      agent-scope release and acquire per node, and on a chip whose L2s are
//      per XCD those cost far more than the few dozen launches;
//   8. the four-wide view for the cone pass.
// Node boxes are exact FP32 bounds; the traversal pads them per ray.  A refit
// (new vertex positions, same tree) repeats 7 and 8.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <stdint.h>

#include "vls_internal.h"

namespace vls {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys
constexpr int kScanThreads = 1024;

__device__ __forceinline__ unsigned f2ord(float f)
{
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord2f(unsigned u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_fill_i32(int32_t* p, long long n, int32_t v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(unsigned* p, long long n, unsigned v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ubounds[0..5] = vertex lo.xyz, hi.xyz; [6..11] = centroid lo.xyz, hi.xyz; [12] = max |coord|
__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ verts, const int32_t* __restrict__ tri,
                                                long long n_tri, unsigned* __restrict__ ub)
{
    __shared__ unsigned s[13];
    if (threadIdx.x < 13) s[threadIdx.x] = (threadIdx.x < 3 || (threadIdx.x >= 6 && threadIdx.x < 9)) ? 0xffffffffu : 0u;
    __syncthreads();
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // per lane: vertex lo/hi, centroid lo/hi, largest |coordinate| (identities
    // on lanes past the end), reduced over the wavefront before the atomics
    float r[13];
    for (int a = 0; a < 3; ++a) {
        r[a] = INFINITY;
        r[3 + a] = -INFINITY;
        r[6 + a] = INFINITY;
        r[9 + a] = -INFINITY;
    }
    r[12] = 0.0f;
    if (i < n_tri) {
        float c[3] = {0.f, 0.f, 0.f};
        for (int q = 0; q < 3; ++q) {
            long long v = tri[3 * i + q];
            for (int a = 0; a < 3; ++a) {
                float x = verts[3 * v + a];
                r[a] = fminf(r[a], x);
                r[3 + a] = fmaxf(r[3 + a], x);
                c[a] += x;
                r[12] = fmaxf(r[12], fabsf(x));
            }
        }
        for (int a = 0; a < 3; ++a) {
            c[a] *= (1.0f / 3.0f);
            r[6 + a] = c[a];
            r[9 + a] = c[a];
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            r[a] = fminf(r[a], __shfl_xor(r[a], off));
            r[3 + a] = fmaxf(r[3 + a], __shfl_xor(r[3 + a], off));
            r[6 + a] = fminf(r[6 + a], __shfl_xor(r[6 + a], off));
            r[9 + a] = fmaxf(r[9 + a], __shfl_xor(r[9 + a], off));
        }
        r[12] = fmaxf(r[12], __shfl_xor(r[12], off));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&s[a], f2ord(r[a]));
            atomicMax(&s[3 + a], f2ord(r[3 + a]));
            atomicMin(&s[6 + a], f2ord(r[6 + a]));
            atomicMax(&s[9 + a], f2ord(r[9 + a]));
        }
        atomicMax(&s[12], f2ord(r[12]));
    }
    __syncthreads();
    if (threadIdx.x < 13) {
        bool is_min = threadIdx.x < 3 || (threadIdx.x >= 6 && threadIdx.x < 9);
        if (is_min) atomicMin(&ub[threadIdx.x], s[threadIdx.x]);
        else atomicMax(&ub[threadIdx.x], s[threadIdx.x]);
    }
}

__global__ void k_bounds_finish(const unsigned* __restrict__ ub, float* __restrict__ out)
{
    if (threadIdx.x < 13) out[threadIdx.x] = ord2f(ub[threadIdx.x]);
}

__device__ __forceinline__ unsigned long long spread3(unsigned long long x)
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ verts, const int32_t* __restrict__ tri,
                                                long long n_tri, const float* __restrict__ bounds,
                                                unsigned long long* __restrict__ keys, int32_t* __restrict__ vals)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tri) return;
    unsigned long long q[3];
    // one cell size for all axes (the longest centroid extent), so a flat
    // scene's short axis does not get the same number of splits as the long ones
    float ext = fmaxf(fmaxf(bounds[9] - bounds[6], bounds[10] - bounds[7]), bounds[11] - bounds[8]);
    for (int a = 0; a < 3; ++a) {
        float c = (verts[3 * (long long)tri[3 * i] + a] + verts[3 * (long long)tri[3 * i + 1] + a] +
                   verts[3 * (long long)tri[3 * i + 2] + a]) * (1.0f / 3.0f);
        float lo = bounds[6 + a];
        float f = ext > 0.f ? (c - lo) / ext : 0.f;
        f = fminf(fmaxf(f * 2097152.0f, 0.0f), 2097151.0f);
        q[a] = (unsigned long long)f;
    }
    keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------- radix sort

__global__ __launch_bounds__(kSortThreads) void k_hist(const unsigned long long* __restrict__ keys, long long n,
                                                       int shift, unsigned* __restrict__ hist, int n_tiles)
{
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    long long base = (long long)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        long long idx = base + r * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the counts [base, base + 4 * kScanThreads) of a (those below
// total), plus carry, by one block: four consecutive counts per thread, read and
// written coalesced; wavefront scans by lane shifts, then one scan of the
// wavefront sums.  Returns the tile's sum (to every thread).
__device__ __forceinline__ unsigned scan_tile(unsigned* __restrict__ a, long long base, long long total, unsigned carry,
                                              unsigned* wsum)
{
    constexpr int W = kScanThreads / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const long long i0 = base + 4 * (long long)threadIdx.x;
    unsigned v[4];
    for (int q = 0; q < 4; ++q) v[q] = i0 + q < total ? a[i0 + q] : 0u;
    const unsigned t = v[0] + v[1] + v[2] + v[3];
    unsigned x = t;  // inclusive scan over the wavefront
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        unsigned ws = lane < W ? wsum[lane] : 0u;
        for (int off = 1; off < W; off <<= 1) {
            const unsigned y = __shfl_up(ws, off);
            if (lane >= off) ws += y;
        }
        if (lane < W) wsum[lane] = ws;
    }
    __syncthreads();
    unsigned run = carry + (w > 0 ? wsum[w - 1] : 0u) + x - t;
    for (int q = 0; q < 4; ++q) {
        if (i0 + q < total) a[i0 + q] = run;
        run += v[q];
    }
    const unsigned sum = wsum[W - 1];
    __syncthreads();
    return sum;
}

// Exclusive scan of `total` counts in one block: tile after tile with a carry.
__global__ __launch_bounds__(kScanThreads) void k_scan(unsigned* __restrict__ a, long long total)
{
    __shared__ unsigned wsum[kScanThreads / kWave];
    unsigned carry = 0;
    for (long long base = 0; base < total; base += 4 * kScanThreads) carry += scan_tile(a, base, total, carry, wsum);
}

// Larger scans: each block scans its own tile and writes the tile's sum; the
// sums are scanned by k_scan; k_scan_add then adds each tile's offset.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(unsigned* __restrict__ a, long long total,
                                                             unsigned* __restrict__ sums)
{
    __shared__ unsigned wsum[kScanThreads / kWave];
    const unsigned s = scan_tile(a, (long long)blockIdx.x * 4 * kScanThreads, total, 0u, wsum);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(unsigned* __restrict__ a, long long total,
                                                           const unsigned* __restrict__ sums)
{
    const unsigned add = sums[blockIdx.x];
    const long long i0 = (long long)blockIdx.x * 4 * kScanThreads + 4 * (long long)threadIdx.x;
    for (int q = 0; q < 4; ++q)
        if (i0 + q < total) a[i0 + q] += add;
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__global__ __launch_bounds__(kSortThreads) void k_scatter(const unsigned long long* __restrict__ keys_in,
                                                          const int32_t* __restrict__ vals_in,
                                                          unsigned long long* __restrict__ keys_out,
                                                          int32_t* __restrict__ vals_out, long long n, int shift,
                                                          const unsigned* __restrict__ hist, int n_tiles)
{
    constexpr int W = kSortThreads / kWave;
    __shared__ unsigned run[256];
    __shared__ unsigned base[256];
    __shared__ unsigned wc[W][256];
    const int tid = threadIdx.x, w = tid / kWave;
    run[tid] = 0;
    base[tid] = hist[(long long)tid * n_tiles + blockIdx.x];
    long long tile0 = (long long)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        long long idx = tile0 + r * kSortThreads + tid;
        bool valid = idx < n;
        unsigned long long key = valid ? keys_in[idx] : 0ull;
        int32_t val = valid ? vals_in[idx] : 0;
        unsigned d = (unsigned)(key >> shift) & 255u;
        for (int q = 0; q < W; ++q) wc[q][tid] = 0;
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            unsigned long long bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        unsigned rank = lanes_below(m);
        __syncthreads();
        if (valid && rank == 0) wc[w][d] = (unsigned)__popcll(m);
        __syncthreads();
        if (valid) {
            unsigned pre = run[d];
            for (int q = 0; q < w; ++q) pre += wc[q][d];
            long long pos = (long long)base[d] + pre + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        unsigned add = 0;
        for (int q = 0; q < W; ++q) add += wc[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hierarchy

__device__ __forceinline__ int delta(const unsigned long long* __restrict__ k, long long n, long long i, long long j)
{
    if (j < 0 || j >= n) return -1;
    unsigned long long a = k[i], b = k[j];
    if (a == b) return 64 + __clzll((unsigned long long)(i ^ j));
    return __clzll(a ^ b);
}

__device__ __forceinline__ float* node_words(float4* nodes, long long i) { return reinterpret_cast<float*>(nodes + 4 * i); }

__global__ __launch_bounds__(256) void k_karras(const unsigned long long* __restrict__ k, long long n,
                                                float4* __restrict__ nodes, int32_t* __restrict__ leaf_parent,
                                                int32_t* __restrict__ node_parent)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int dir = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(k, n, i, i - dir);
    long long lmax = 2;
    while (delta(k, n, i, i + lmax * dir) > dmin) lmax <<= 1;
    long long l = 0;
    for (long long t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(k, n, i, i + (l + t) * dir) > dmin) l += t;
    long long j = i + l * dir;
    int dnode = delta(k, n, i, j);
    long long s = 0;
    long long div = 2;
    long long t;
    do {
        t = (l + div - 1) / div;
        if (delta(k, n, i, i + (s + t) * dir) > dnode) s += t;
        div <<= 1;
    } while (t > 1);
    long long gamma = i + s * dir + (dir < 0 ? -1 : 0);
    long long lo = i < j ? i : j, hi = i < j ? j : i;
    int left, right;
    if (lo == gamma) { left = ~(int)gamma; leaf_parent[gamma] = (int32_t)i; }
    else { left = (int)gamma; node_parent[gamma] = (int32_t)i; }
    if (hi == gamma + 1) { right = ~(int)(gamma + 1); leaf_parent[gamma + 1] = (int32_t)i; }
    else { right = (int)(gamma + 1); node_parent[gamma + 1] = (int32_t)i; }
    float* w = node_words(nodes, i);
    w[12] = __int_as_float(left);
    w[13] = __int_as_float(right);
    w[15] = 0.0f;
    if (i == 0) node_parent[0] = -1;
}

__global__ __launch_bounds__(256) void k_parent_words(float4* __restrict__ nodes, const int32_t* __restrict__ node_parent,
                                                      long long n_int)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_int) node_words(nodes, i)[14] = __int_as_float(node_parent[i]);
}

__global__ __launch_bounds__(256) void k_leaves(const float* __restrict__ verts, const int32_t* __restrict__ tri,
                                                const int32_t* order, long long n,
                                                float4* __restrict__ recs, int32_t* leaf_tri)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = order[i];
    float v[3][3];
    for (int q = 0; q < 3; ++q) {
        long long vi = tri[3 * (long long)o + q];
        v[q][0] = verts[3 * vi];
        v[q][1] = verts[3 * vi + 1];
        v[q][2] = verts[3 * vi + 2];
    }
    recs[3 * i + 0] = make_float4(v[0][0], v[0][1], v[0][2], __int_as_float(o));
    recs[3 * i + 1] = make_float4(v[1][0], v[1][1], v[1][2], 0.0f);
    recs[3 * i + 2] = make_float4(v[2][0], v[2][1], v[2][2], 0.0f);
    if (leaf_tri) leaf_tri[i] = o;
}

// Depth of every internal node (steps up to the root), and a histogram of the
// depths (capped at kMaxLevel, which only a corrupted structure reaches).
__global__ __launch_bounds__(256) void k_node_depth(const int32_t* __restrict__ node_parent, long long n_int,
                                                    int32_t* __restrict__ depth, unsigned* __restrict__ hist)
{
    __shared__ unsigned h[kMaxLevel + 1];
    for (int q = threadIdx.x; q <= kMaxLevel; q += blockDim.x) h[q] = 0;
    __syncthreads();
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_int) {
        int d = 0;
        for (int p = node_parent[i]; p >= 0 && d < kMaxLevel; p = node_parent[p]) ++d;
        depth[i] = d;
        atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= kMaxLevel; q += blockDim.x)
        if (h[q]) atomicAdd(&hist[q], h[q]);
}

// Internal nodes grouped by depth: cursor[d] starts at the first slot of depth
// d in `order` (the order within a depth does not matter).  Each block counts
// its nodes per depth in LDS and takes its slots with one global atomic per
// depth it holds; depths are < n_levels.
__global__ __launch_bounds__(256) void k_level_scatter(const int32_t* __restrict__ depth, long long n_int,
                                                       int n_levels, unsigned* __restrict__ cursor,
                                                       int32_t* __restrict__ order)
{
    __shared__ unsigned cnt[kMaxLevel + 1];
    __shared__ unsigned base[kMaxLevel + 1];
    for (int q = threadIdx.x; q < n_levels; q += blockDim.x) cnt[q] = 0;
    __syncthreads();
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int d = -1;
    unsigned local = 0;
    if (i < n_int) {
        d = depth[i];
        if (d >= 0 && d < n_levels) local = atomicAdd(&cnt[d], 1u);
        else d = -1;  // only a corrupted structure gets here
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n_levels; q += blockDim.x)
        if (cnt[q]) base[q] = atomicAdd(&cursor[q], cnt[q]);
    __syncthreads();
    if (d >= 0) order[base[d] + local] = (int32_t)i;
}

// Boxes of one depth of internal nodes: a child's box is its triangle's (leaf)
// or the union of the two boxes the child node holds, written one launch
// earlier (children are one level deeper).
__global__ __launch_bounds__(256) void k_refit_level(const float4* __restrict__ recs, float4* nodes,
                                                     const int32_t* __restrict__ order, long long count,
                                                     long long n_int, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int p = order[i];
    float* w = node_words(nodes, p);
    for (int side = 0; side < 2; ++side) {
        const int c = __float_as_int(w[12 + side]);
        float box[6];
        if (c < 0) {
            const long long li = ~(long long)c;
            if (li >= n) continue;  // only a corrupted structure gets here
            const float4 a = recs[3 * li], b = recs[3 * li + 1], d = recs[3 * li + 2];
            box[0] = fminf(fminf(a.x, b.x), d.x);
            box[1] = fminf(fminf(a.y, b.y), d.y);
            box[2] = fminf(fminf(a.z, b.z), d.z);
            box[3] = fmaxf(fmaxf(a.x, b.x), d.x);
            box[4] = fmaxf(fmaxf(a.y, b.y), d.y);
            box[5] = fmaxf(fmaxf(a.z, b.z), d.z);
        } else {
            if (c >= n_int) continue;  // only a corrupted structure gets here
            const float* wc = node_words(nodes, c);
            for (int q = 0; q < 3; ++q) box[q] = fminf(wc[q], wc[6 + q]);
            for (int q = 3; q < 6; ++q) box[q] = fmaxf(wc[q], wc[6 + q]);
        }
        for (int q = 0; q < 6; ++q) w[6 * side + q] = box[q];
    }
}

// Four-wide view of the binary tree for the cone pass.  Record b (8 x float4)
// holds, for binary node b, the boxes and refs of its grandchildren -- or of a
// child itself when that child is a leaf -- so one fetch covers two levels:
// words [4q .. 4q+3] of float4 q = 0..5 are lo.x, lo.y, lo.z, hi.x, hi.y, hi.z of
// slots 0..3; float4 6 holds the four refs as int bits (>= 0: record of an
// internal node, < 0: leaf ~ref, kEmpty4: unused slot).  A child's box contains
// its children's boxes, so testing the grandchildren alone loses nothing.
__global__ __launch_bounds__(256) void k_collapse4(const float4* __restrict__ nodes, long long n_int,
                                                   float4* __restrict__ nodes4)
{
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_int) return;
    const float* w = reinterpret_cast<const float*>(nodes + 4 * b);
    float box[6][4];
    int ref[4];
    for (int side = 0; side < 2; ++side) {
        const int c = __float_as_int(w[12 + side]);
        const float* cb = w + 6 * side;
        if (c >= 0 && c < n_int) {
            const float* wc = reinterpret_cast<const float*>(nodes + 4 * (long long)c);
            for (int h = 0; h < 2; ++h) {
                for (int q = 0; q < 6; ++q) box[q][2 * side + h] = wc[6 * h + q];
                ref[2 * side + h] = __float_as_int(wc[12 + h]);
            }
        } else {
            for (int q = 0; q < 6; ++q) box[q][2 * side] = cb[q];
            ref[2 * side] = c;
            for (int q = 0; q < 3; ++q) box[q][2 * side + 1] = INFINITY;
            for (int q = 3; q < 6; ++q) box[q][2 * side + 1] = -INFINITY;
            ref[2 * side + 1] = kEmpty4;
        }
    }
    float4* o = nodes4 + 8 * b;
    for (int q = 0; q < 6; ++q) o[q] = make_float4(box[q][0], box[q][1], box[q][2], box[q][3]);
    o[6] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]), __int_as_float(ref[3]));
    o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Checked before anything reads vertices through the indices: bit 0 marks an
// index outside [0, nv), bit 1 a non-finite vertex coordinate.
__global__ __launch_bounds__(256) void k_check_mesh(const float* __restrict__ verts, long long nv,
                                                    const int32_t* __restrict__ tri, long long nt,
                                                    unsigned* __restrict__ bad)
{
    const long long n3 = 3 * (nv > nt ? nv : nt);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (long long)gridDim.x * blockDim.x) {
        unsigned f = 0;
        if (i < 3 * nt) {
            const int32_t v = tri[i];
            if (v < 0 || v >= nv) f |= 1u;
        }
        if (i < 3 * nv && !isfinite(verts[i])) f |= 2u;
        if (f) atomicOr(bad, f);
    }
}

inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_fill_u64(unsigned long long* p, long long n, unsigned long long v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

#define VLS_TRY(x)                         \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

static hipError_t bounds_pass(BvhBuffers& b, unsigned* ub, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(16), 0, stream, ub, 13ll, 0u);
    // minima start at the largest ordered value
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(3), 0, stream, ub, 3ll, 0xffffffffu);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(3), 0, stream, ub + 6, 3ll, 0xffffffffu);
    hipLaunchKernelGGL(k_bounds, dim3(grid_for(b.n_tri, 256)), dim3(256), 0, stream, b.verts, b.tri_idx, b.n_tri, ub);
    hipLaunchKernelGGL(k_bounds_finish, dim3(1), dim3(64), 0, stream, ub, b.bounds);
    return hipGetLastError();
}

hipError_t mesh_check(const BvhBuffers& b, hipStream_t stream, unsigned& bad)
{
    bad = 0;
    if (b.n_tri == 0 && b.n_vert == 0) return hipSuccess;
    unsigned* flag = reinterpret_cast<unsigned*>(b.bounds + 30);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, flag, 1ll, 0u);
    const long long n3 = 3 * std::max(b.n_tri, b.n_vert);
    hipLaunchKernelGGL(k_check_mesh, dim3(std::min(grid_for(n3, 256), 4096u)), dim3(256), 0, stream, b.verts,
                       (long long)b.n_vert, b.tri_idx, (long long)b.n_tri, flag);
    VLS_TRY(hipGetLastError());
    VLS_TRY(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, stream));
    return hipStreamSynchronize(stream);
}

// Histogram words of a sort of n keys, plus room for the tile sums of their scan.
long long radix_sort_hist_words(long long n)
{
    const long long words = 256ll * ((n + kSortTile - 1) / kSortTile);
    return words + (words + 4 * kScanThreads - 1) / (4 * kScanThreads);
}

hipError_t radix_sort_pairs(unsigned long long* keys, int32_t* vals, unsigned long long* keys2, int32_t* vals2,
                            unsigned* hist, long long n, int passes, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int n_tiles = (int)((n + kSortTile - 1) / kSortTile);
    unsigned long long *kin = keys, *kout = keys2;
    int32_t *vin = vals, *vout = vals2;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_hist, dim3(n_tiles), dim3(kSortThreads), 0, stream, kin, n, shift, hist, n_tiles);
        const long long words = 256ll * n_tiles;
        const long long scan_tiles = (words + 4 * kScanThreads - 1) / (4 * kScanThreads);
        if (scan_tiles <= 8) {
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, stream, hist, words);
        } else {
            unsigned* sums = hist + words;
            hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)scan_tiles), dim3(kScanThreads), 0, stream, hist, words, sums);
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, stream, sums, scan_tiles);
            hipLaunchKernelGGL(k_scan_add, dim3((unsigned)scan_tiles), dim3(kScanThreads), 0, stream, hist, words, sums);
        }
        hipLaunchKernelGGL(k_scatter, dim3(n_tiles), dim3(kSortThreads), 0, stream, kin, vin, kout, vout, n, shift,
                           hist, n_tiles);
        unsigned long long* tk = kin; kin = kout; kout = tk;
        int32_t* tv = vin; vin = vout; vout = tv;
    }
    return hipGetLastError();
}

hipError_t bvh_build(BvhBuffers& b, hipStream_t stream, std::string& err)
{
    const long long n = b.n_tri;
    if (n == 0) return hipSuccess;
    const int n_tiles = (int)((n + kSortTile - 1) / kSortTile);
    unsigned long long* keys2 = nullptr;
    int32_t *vals = nullptr, *vals2 = nullptr;
    unsigned *hist = nullptr, *ub = nullptr, *lv = nullptr;
    std::vector<unsigned> cur;  // level cursors: the copy to the device reads them until the final synchronisation
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t x, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(x);
        return x;
    };
    do {
        if ((e = hipMalloc(&keys2, sizeof(unsigned long long) * n)) != hipSuccess) { (void)fail(e, "alloc keys"); break; }
        if ((e = hipMalloc(&vals, sizeof(int32_t) * n)) != hipSuccess) { (void)fail(e, "alloc vals"); break; }
        if ((e = hipMalloc(&vals2, sizeof(int32_t) * n)) != hipSuccess) { (void)fail(e, "alloc vals"); break; }
        if ((e = hipMalloc(&hist, sizeof(unsigned) * (size_t)radix_sort_hist_words(n))) != hipSuccess) { (void)fail(e, "alloc hist"); break; }
        if ((e = hipMalloc(&ub, sizeof(unsigned) * 16)) != hipSuccess) { (void)fail(e, "alloc bounds"); break; }
        if ((e = bounds_pass(b, ub, stream)) != hipSuccess) { (void)fail(e, "bounds"); break; }
        hipLaunchKernelGGL(k_morton, dim3(grid_for(n, 256)), dim3(256), 0, stream, b.verts, b.tri_idx, n, b.bounds,
                           b.morton, vals);
        // 8 passes: the sorted data is back in b.morton / vals
        if ((e = radix_sort_pairs(b.morton, vals, keys2, vals2, hist, n, 8, stream)) != hipSuccess) { (void)fail(e, "sort"); break; }
        if (n > 1) {
            hipLaunchKernelGGL(k_karras, dim3(grid_for(n - 1, 256)), dim3(256), 0, stream, b.morton, n, b.nodes,
                               b.leaf_parent, b.node_parent);
            hipLaunchKernelGGL(k_parent_words, dim3(grid_for(n - 1, 256)), dim3(256), 0, stream, b.nodes,
                               b.node_parent, n - 1);
        } else {
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, b.leaf_parent, 1ll, -1);
        }
        hipLaunchKernelGGL(k_leaves, dim3(grid_for(n, 256)), dim3(256), 0, stream, b.verts, b.tri_idx, vals, n, b.tris,
                           b.leaf_tri);
        if ((e = hipGetLastError()) != hipSuccess) { (void)fail(e, "hierarchy"); break; }
        b.level_off.assign(1, 0);
        if (n > 1) {
            // internal nodes grouped by depth, for the refit's one launch per depth
            const long long ni = n - 1;
            if ((e = hipMalloc(&lv, sizeof(unsigned) * 2 * (kMaxLevel + 1))) != hipSuccess) { (void)fail(e, "alloc levels"); break; }
            hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(kMaxLevel + 1, 256)), dim3(256), 0, stream, lv,
                               (long long)kMaxLevel + 1, 0u);
            hipLaunchKernelGGL(k_node_depth, dim3(grid_for(ni, 256)), dim3(256), 0, stream, b.node_parent, ni,
                               b.node_depth, lv);
            std::vector<unsigned> h(kMaxLevel + 1);
            if ((e = hipMemcpyAsync(h.data(), lv, sizeof(unsigned) * h.size(), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess) { (void)fail(e, "levels"); break; }
            int top = kMaxLevel;
            while (top > 0 && h[top] == 0) --top;
            cur.assign(top + 1, 0u);
            b.level_off.assign(top + 2, 0);
            for (int d = 0; d <= top; ++d) {
                cur[d] = (unsigned)b.level_off[d];
                b.level_off[d + 1] = b.level_off[d] + h[d];
            }
            if ((e = hipMemcpyAsync(lv + kMaxLevel + 1, cur.data(), sizeof(unsigned) * cur.size(),
                                    hipMemcpyHostToDevice, stream)) != hipSuccess) { (void)fail(e, "levels"); break; }
            hipLaunchKernelGGL(k_level_scatter, dim3(grid_for(ni, 256)), dim3(256), 0, stream, b.node_depth, ni,
                               top + 1, lv + kMaxLevel + 1, b.level_order);
            if ((e = hipGetLastError()) != hipSuccess) { (void)fail(e, "levels"); break; }
        }
        // the deepest leaves hang below the deepest internal nodes
        const unsigned leaf_depth = n > 1 ? (unsigned)b.level_off.size() - 1 : 0u;
        if ((e = bvh_refit(b, stream)) != hipSuccess) { (void)fail(e, "refit"); break; }
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, stream, reinterpret_cast<unsigned*>(b.bounds + 13), 1ll,
                           leaf_depth);
        if ((e = hipGetLastError()) != hipSuccess) { (void)fail(e, "depth"); break; }
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) { (void)fail(e, "build"); break; }
    } while (0);
    (void)hipFree(keys2);
    (void)hipFree(vals);
    (void)hipFree(vals2);
    (void)hipFree(hist);
    (void)hipFree(ub);
    (void)hipFree(lv);
    return e;
}

hipError_t bvh_refit(BvhBuffers& b, hipStream_t stream)
{
    const long long n = b.n_tri;
    if (n == 0) return hipSuccess;
    unsigned* ub = reinterpret_cast<unsigned*>(b.bounds + 16);  // scratch words after the results
    VLS_TRY(bounds_pass(b, ub, stream));
    if (n > 1) {
        // one launch per depth, deepest first (the levels come from the build)
        for (size_t d = b.level_off.size() - 1; d-- > 0;) {
            const long long lo = b.level_off[d], cnt = b.level_off[d + 1] - lo;
            if (cnt > 0)
                hipLaunchKernelGGL(k_refit_level, dim3(grid_for(cnt, 256)), dim3(256), 0, stream, b.tris, b.nodes,
                                   b.level_order + lo, cnt, n - 1, n);
        }
        if (b.nodes4)
            hipLaunchKernelGGL(k_collapse4, dim3(grid_for(n - 1, 256)), dim3(256), 0, stream, b.nodes, n - 1,
                               b.nodes4);
    }
    return hipGetLastError();
}

// Leaf records from new vertices (same sorted order), then boxes.
hipError_t bvh_update_vertices(BvhBuffers& b, hipStream_t stream)
{
    const long long n = b.n_tri;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaves, dim3(grid_for(n, 256)), dim3(256), 0, stream, b.verts, b.tri_idx, b.leaf_tri, n,
                       b.tris, (int32_t*)nullptr);
    VLS_TRY(hipGetLastError());
    return bvh_refit(b, stream);
}

}  // namespace vls
